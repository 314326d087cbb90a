// Integration driver: work plans, the cached and graph-captured pass, the
// points-per-thread autotuner, variance-driven budget allocation, and the
// integrate / per-sector results / sampling-hook entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace sdi {


// Everything one pass needs: per-sector lattice sizes, tiles and their order,
// the device copy of the sector records for this pass, and workspace slots.
struct Plan {
  int R = 0, rows = 0;
  int tile_log2 = 14;            // points per final-pass tile (log2; shorter lattices make one tile)
  uint32_t range_lo = 0, range_hi = 0;  // lattice indices of this pass per shift (hi 0: the whole lattice)
  double small_x = 0.0;          // endpoint-precision threshold of the final pass (0: off)
  bool warm = false;
  bool flow = false;             // final points come from the learned sampler
  bool mc = false;               // final points are Monte Carlo points (integrator 2)
  std::vector<PointRun> fruns;   // per final tile: its points in the flow buffers
  std::vector<int64_t> fchunk, fx_off, fpt_off;
  int64_t fx_total = 0, fpt_total = 0;
  std::vector<int> msec;
  std::vector<SecDev> secs;
  std::vector<TileDesc> ftiles;
  std::vector<int32_t> forder, pair_start, pair_sector;
  std::vector<int32_t> xorder;   // flow tiles (LPT order); forder then holds the lattice tiles
  std::vector<TileDesc> wtiles;
  std::vector<int32_t> worder, wsec_start;
  std::vector<int64_t> whist_off, hsec_off, hsec_prefix;
  int64_t whist_total = 0, hsec_total = 0;
  size_t shmem_final = 0, shmem_warm = 0;
  std::vector<uint64_t> zp_final, zp_warm;
  SecDev* d_secs = nullptr;
  TileDesc* d_ftiles = nullptr;
  int32_t* d_forder = nullptr;
  int32_t* d_xorder = nullptr;
  int32_t* d_pair_start = nullptr;
  int32_t* d_pair_sector = nullptr;
  double* d_partial = nullptr;
  int32_t* d_nonfinite = nullptr;
  double* d_per_shift = nullptr;
  double* d_sec_stats = nullptr;
  double* d_res = nullptr;
  double* d_carry_in = nullptr;     // resumable pass: sums and counts of the earlier slices
  int64_t* d_carry_in_counts = nullptr;
  double* d_carry_out = nullptr;    // ... and after this slice
  int64_t* d_carry_out_counts = nullptr;
  int64_t* d_counts = nullptr;
  int64_t* d_pair_nonfinite = nullptr;
  int64_t* d_sec_nonfinite = nullptr;
  int32_t* d_counter = nullptr;
  uint64_t* d_shifts = nullptr;
  uint64_t* d_zp_final = nullptr;
  PointRun* d_fruns = nullptr;
  int64_t* d_fchunk = nullptr;
  int64_t* d_fx_off = nullptr;
  int64_t* d_fpt_off = nullptr;
  double* d_px = nullptr;
  double* d_pw = nullptr;
  uint64_t* d_zp_warm = nullptr;
  TileDesc* d_wtiles = nullptr;
  int32_t* d_worder = nullptr;
  int64_t* d_whist_off = nullptr;
  int32_t* d_wsec_start = nullptr;
  int32_t* d_wnonfinite = nullptr;
  double* d_wpartial = nullptr;
  double* d_whist = nullptr;
  double* d_hsec = nullptr;
  int64_t* d_hsec_off = nullptr;
  int64_t* d_hsec_prefix = nullptr;
  Carve carve;
};

struct PassState {
  std::string key;
  Plan P;
  int ppt = 1, wpe = 4, km = 4, gf = 1, gw = 1, gx = 1;
  bool lists = false;   // final pass on the generic (per-corner list) instances
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};   // warm-up, final tiles, reductions
  void* own_ws = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // recorded between segment launches
  ~PassState() {
    for (hipGraphExec_t x : exec)
      if (x) (void)hipGraphExecDestroy(x);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (own_ws) (void)hipFree(own_ws);
    (void)hipGetLastError();
  }
};

// The expression tape of a problem given as text.
ExprArgs expr_args(const sdi_problem* pb) {
  return ExprArgs{pb->d_expr, (int32_t)pb->expr_nins, pb->expr_slots, pb->expr_out, pb->expr_cplx ? 1 : 0};
}

void free_passes(std::vector<PassState*>& v) {
  for (PassState* p : v) delete p;
  v.clear();
}

namespace {

void lpt_order(const std::vector<TileDesc>& tiles, const std::vector<double>& cost, std::vector<int32_t>& order) {
  order.resize(tiles.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ca = cost[tiles[a].sector] * tiles[a].count;
    const double cb = cost[tiles[b].sector] * tiles[b].count;
    return ca > cb;
  });
}

// Grid offsets and parameter-dependent fields of the sector records.
void sector_fields(const Params& prm, const sdi_problem* pb, const std::vector<int>& msec, int rows,
                   std::vector<SecDev>& secs, size_t& goff) {
  secs = pb->secs;
  goff = 0;
  for (int s = 0; s < pb->nsec; ++s) {
    SecDev& S = secs[s];
    S.m = msec[s];
    S.mw = prm.mw;
    S.nbins = prm.nbins;
    S.shift_row = s * rows;
    S.grid_off = (int32_t)goff;
    goff += (size_t)S.n * (prm.nbins + 1);
    S.flags &= ~(F_USE_GRID | F_BAKER);
    if (prm.baker) S.flags |= F_BAKER;
    if (prm.warmup > 0) S.flags |= F_USE_GRID;
  }
}

int make_plan(sdi_ctx* ctx, sdi_problem* pb, Plan& P, const std::vector<int>& msec, bool warm, int tile_log2,
              uint32_t range_lo = 0, uint32_t range_hi = 0) {
  const Params& prm = ctx->params;
  P.R = prm.R;
  P.tile_log2 = tile_log2;
  P.range_lo = range_lo;
  P.range_hi = range_hi;
  P.rows = prm.R + prm.warmup;
  P.warm = warm && prm.warmup > 0;
  P.flow = prm.sampler == 1;
  P.mc = prm.integrator == 2;
  P.small_x = (prm.small_x > 0.0 && !pb->is_expr()) ? prm.small_x : 0.0;
  if (P.mc && P.flow) return fail(ctx, SDI_ENOTSUP, "Monte Carlo points and the flow sampler exclude each other");
  if (P.mc && pb->is_expr()) return fail(ctx, SDI_ENOTSUP, "Monte Carlo points: not available for integrands given as text");
  if (P.flow && !pb->flow) return fail(ctx, SDI_ESTATE, "sampler flow needs sdi_flow_init on this problem");
  if (P.flow && prm.warmup > 0) return fail(ctx, SDI_ENOTSUP, "the flow sampler replaces the Vegas warm-up (set warmup 0)");
  P.msec = msec;
  const int nsec = pb->nsec;
  size_t goff = 0;
  sector_fields(prm, pb, msec, P.rows, P.secs, goff);
  for (int s = 0; s < nsec; ++s)
    if (msec[s] < 4 || msec[s] > 30) return fail(ctx, SDI_EINVAL, "lattice log2 outside 4..30");
  P.pair_start.clear();
  P.pair_sector.clear();
  P.ftiles.clear();
  for (int s = 0; s < nsec; ++s) {
    const uint32_t N = 1u << msec[s];
    // a slice of a resumable pass covers indices [range_lo, range_hi) of every shift
    const uint32_t lo = range_hi ? range_lo : 0u, hi = range_hi ? std::min(range_hi, N) : N;
    const uint32_t tsz = std::min<uint32_t>(hi - lo, 1u << tile_log2);
    for (int r = 0; r < prm.R; ++r) {
      P.pair_start.push_back((int32_t)P.ftiles.size());
      P.pair_sector.push_back(s);
      for (uint32_t i0 = lo; i0 < hi; i0 += tsz) P.ftiles.push_back(TileDesc{s, r, i0, std::min(tsz, hi - i0)});
    }
  }
  P.pair_start.push_back((int32_t)P.ftiles.size());
  lpt_order(P.ftiles, pb->cost, P.forder);
  P.xorder.clear();
  P.fruns.clear();
  P.fchunk.clear();
  P.fx_off.clear();
  P.fpt_off.clear();
  P.fx_total = P.fpt_total = 0;
  if (P.flow || P.mc) {
    // explicit-point tiles: sectors with an active flow (or every sector, for
    // Monte Carlo points); the others stay on the lattice
    const std::vector<uint8_t>* act = P.flow ? &pb->flow->active : nullptr;
    int64_t chunks = 0;
    for (const TileDesc& t : P.ftiles) {
      if (act && !(*act)[t.sector]) {
        P.fx_off.push_back(-1);
        P.fpt_off.push_back(-1);
        continue;
      }
      const SecDev& S = P.secs[t.sector];
      P.fruns.push_back(PointRun{t.sector, S.shift_row + t.shift, t.i0, t.count, P.fpt_total, P.fx_total});
      P.fchunk.push_back(chunks);
      P.fx_off.push_back(P.fx_total);
      P.fpt_off.push_back(P.fpt_total);
      chunks += ((int64_t)t.count + 63) / 64;
      P.fx_total += (int64_t)t.count * S.n;
      P.fpt_total += t.count;
    }
    P.fchunk.push_back(chunks);
    std::vector<int32_t> lat;
    for (int32_t t : P.forder) ((!act || (*act)[P.ftiles[t].sector]) ? P.xorder : lat).push_back(t);
    P.forder.swap(lat);
    if ((P.fx_total + P.fpt_total) * 8 > ((int64_t)64 << 30))
      return fail(ctx, SDI_ENOTSUP, "explicit-point pass needs more than 64 GiB of point buffers; lower the lattice size");
  }
  P.wtiles.clear();
  P.whist_off.clear();
  P.wsec_start.clear();
  P.hsec_off.clear();
  P.hsec_prefix.clear();
  P.whist_total = P.hsec_total = 0;
  if (P.warm) {
    const uint32_t Nw = 1u << prm.mw;
    const uint32_t wsz = std::min<uint32_t>(Nw, 1u << std::min(tile_log2, 12));
    for (int s = 0; s < nsec; ++s) {
      const SecDev& S = P.secs[s];
      P.wsec_start.push_back((int32_t)P.wtiles.size());
      const int64_t hs = (int64_t)S.n * prm.nbins * std::max(S.kf, 1);
      P.hsec_off.push_back(P.hsec_total);
      P.hsec_prefix.push_back(P.hsec_total);
      P.hsec_total += hs;
      for (uint32_t i0 = 0; i0 < Nw; i0 += wsz) {
        P.wtiles.push_back(TileDesc{s, prm.R, i0, wsz});
        P.whist_off.push_back(P.whist_total);
        P.whist_total += hs;
      }
    }
    P.wsec_start.push_back((int32_t)P.wtiles.size());
    lpt_order(P.wtiles, pb->cost, P.worder);
  }
  size_t gmax = 0, hmax = 0;
  for (int s = 0; s < nsec; ++s) {
    const SecDev& S = P.secs[s];
    gmax = std::max(gmax, (size_t)S.n * (prm.nbins + 1));
    hmax = std::max(hmax, (size_t)S.n * prm.nbins * std::max(S.kf, 1));
  }
  P.shmem_final = prm.warmup > 0 ? gmax * 8 : 0;
  P.shmem_warm = (gmax + hmax) * 8;
  if (P.warm && P.shmem_warm > 64 * 1024)
    return fail(ctx, SDI_ENOTSUP, "Vegas grid plus histogram exceed 64 KiB of LDS; lower nbins");
  if (pb->is_expr()) {
    const size_t slots = expr_slot_bytes(expr_args(pb));
    if (std::max(P.shmem_final, P.warm ? P.shmem_warm : 0) + slots > 64 * 1024)
      return fail(ctx, SDI_ENOTSUP, "expression slots plus Vegas grid exceed 64 KiB of LDS; lower nbins");
  }
  P.zp_final.assign((size_t)nsec * MAXV, 0);
  for (int s = 0; s < nsec; ++s) {
    const std::vector<uint32_t>& zf = lattice_vector16(msec[s]);
    for (int j = 0; j < MAXV; ++j) P.zp_final[(size_t)s * MAXV + j] = (uint64_t)zf[j] << (53 - msec[s]);
  }
  if (P.warm) {
    const std::vector<uint32_t>& zw = lattice_vector16(prm.mw);
    P.zp_warm.assign((size_t)nsec * MAXV, 0);
    for (int s = 0; s < nsec; ++s)
      for (int j = 0; j < MAXV; ++j) P.zp_warm[(size_t)s * MAXV + j] = (uint64_t)zw[j] << (53 - prm.mw);
  }
  Carve& C = P.carve;
  C.items.clear();
  const size_t nft = P.ftiles.size(), npairs = P.pair_sector.size();
  C.add((void**)&P.d_secs, (size_t)nsec * sizeof(SecDev));
  C.add((void**)&P.d_ftiles, nft * sizeof(TileDesc));
  C.add((void**)&P.d_forder, nft * 4);
  C.add((void**)&P.d_xorder, nft * 4);
  C.add((void**)&P.d_pair_start, (npairs + 1) * 4);
  C.add((void**)&P.d_pair_sector, npairs * 4);
  C.add((void**)&P.d_partial, nft * KMAX * PART_STRIDE * 8);
  C.add((void**)&P.d_nonfinite, nft * 8);
  C.add((void**)&P.d_per_shift, npairs * KMAX * 2 * 8);
  C.add((void**)&P.d_sec_stats, (size_t)nsec * KMAX * 4 * 8);
  C.add((void**)&P.d_res, KMAX * 4 * 8);
  C.add((void**)&P.d_carry_in, npairs * KMAX * 4 * 8);
  C.add((void**)&P.d_carry_in_counts, npairs * 16);
  C.add((void**)&P.d_carry_out, npairs * KMAX * 4 * 8);
  C.add((void**)&P.d_carry_out_counts, npairs * 16);
  C.add((void**)&P.d_counts, 2 * 8);
  C.add((void**)&P.d_pair_nonfinite, npairs * 16);
  C.add((void**)&P.d_sec_nonfinite, (size_t)nsec * 16);
  C.add((void**)&P.d_counter, 8 * 4);
  C.add((void**)&P.d_shifts, (size_t)nsec * P.rows * MAXV * 8);
  C.add((void**)&P.d_zp_final, (size_t)nsec * MAXV * 8);
  if (P.flow || P.mc) {
    C.add((void**)&P.d_fruns, P.fruns.size() * sizeof(PointRun));
    C.add((void**)&P.d_fchunk, P.fchunk.size() * 8);
    C.add((void**)&P.d_fx_off, P.fx_off.size() * 8);
    C.add((void**)&P.d_fpt_off, P.fpt_off.size() * 8);
    C.add((void**)&P.d_px, (size_t)P.fx_total * 8);
    C.add((void**)&P.d_pw, (size_t)P.fpt_total * 8);
  }
  if (P.warm) {
    const size_t nwt = P.wtiles.size();
    C.add((void**)&P.d_zp_warm, (size_t)nsec * MAXV * 8);
    C.add((void**)&P.d_wtiles, nwt * sizeof(TileDesc) * prm.warmup);
    C.add((void**)&P.d_worder, nwt * 4);
    C.add((void**)&P.d_whist_off, nwt * 8);
    C.add((void**)&P.d_wsec_start, (nsec + 1) * 4);
    C.add((void**)&P.d_wnonfinite, nwt * 8);
    C.add((void**)&P.d_wpartial, nwt * KMAX * PART_STRIDE * 8);
    C.add((void**)&P.d_whist, (size_t)P.whist_total * 8);
    C.add((void**)&P.d_hsec, (size_t)P.hsec_total * 8);
    C.add((void**)&P.d_hsec_off, nsec * 8);
    C.add((void**)&P.d_hsec_prefix, nsec * 8);
  }
  // persistent Vegas grids live with the problem
  if (prm.warmup > 0 && (pb->grid_doubles < goff || pb->grid_nbins != prm.nbins)) {
    if (pb->d_grids) (void)hipFree(pb->d_grids);
    pb->d_grids = nullptr;
    pb->grid_doubles = 0;
    pb->grid_valid = false;
    HIPCHK(ctx, hipMalloc((void**)&pb->d_grids, goff * 8));
    pb->grid_doubles = goff;
    pb->grid_nbins = prm.nbins;
  }
  return SDI_OK;
}

bool uses_dd(const sdi_problem* pb, const Params& p) {
  return p.small_x > 0.0 && !pb->is_expr();
}

// Family of real-mode final-pass instances of a problem under the current
// parameters (see real_family).
int final_family(const sdi_problem* pb, const Params& p) {
  return real_family(pb->nsmax, pb->nfmax, 0, uses_dd(pb, p));
}

// Final-pass launch variants the autotuner times, encoded as 10 * points per
// thread + minimum waves per SIMD (1: no constraint), plus CORNER_LISTS for the
// generic instances that evaluate each corner's own term lists: where the
// grouped instances (each term once) exist, the tuner times both kinds, since
// the grouped ones hold every corner's factor values in registers and win only
// where the polynomials outweigh that (measured: the 2000-sector synthetic
// set gains, the double box with its 16 corners loses).
constexpr int CORNER_LISTS = 100;
// Problems with factor exponents above 3 run one generic instance (1 point per
// thread, 4 waves per SIMD) in every mode.
constexpr int E7_VARIANT = 14;

std::vector<int> generic_variants(const sdi_problem* pb) {
  if (pb->nvmax >= 10) return {14, 23, 24};
  return {14, 23, 24, 42};
}

std::vector<int> tile_variants(const sdi_problem* pb, const Params& p) {
  if (pb->is_expr()) return {11};
  if (pb->exp7) return {E7_VARIANT};
  if (pb->complex_mode) {
    if (uses_dd(pb, p)) return {11};   // the endpoint-precision instance (one point per thread)
    return pb->nvmax <= 4 ? std::vector<int>{11, 12, 21} : std::vector<int>{11, 12};
  }
  std::vector<int> v;
  switch (final_family(pb, p)) {
    case RF_G3: v = {12, 14, 22, 23}; break;
    case RF_G4: v = {12, 13, 21, 22}; break;
    case RF_S2: v = generic_variants(pb); break;
    case RF_DD: return {12};
    default: return generic_variants(pb);
  }
  if (!uses_dd(pb, p))
    for (int g : generic_variants(pb)) v.push_back(CORNER_LISTS + g);
  return v;
}

// The endpoint-precision instance outside the two-singular-variable family
// (real mode, small_x > 0): one point per thread, at least 2 waves per SIMD,
// the only final-pass variant there.  Problems in that family keep the tuned
// variants, in their double-double-capable copies.
constexpr int DD_VARIANT = 12;

// The variant used for a fixed points-per-thread request.
int default_variant(const sdi_problem* pb, const Params& p, int ppt) {
  if (pb->is_expr()) return 11;   // one point per lane and step
  if (pb->exp7) return E7_VARIANT;
  if (pb->complex_mode) return uses_dd(pb, p) ? 11 : 10 * ppt + 1;
  switch (final_family(pb, p)) {
    case RF_G3: return ppt == 1 ? 14 : 22;
    case RF_G4: return ppt == 1 ? 12 : 22;
    case RF_DD: return DD_VARIANT;
    default: break;
  }
  return ppt == 4 ? (pb->nvmax >= 10 ? 24 : 42) : 10 * ppt + 4;
}

// Whether an encoded variant is one the tuner or a points-per-thread request
// can select for the problem's class.
bool variant_known(const sdi_problem* pb, const Params& p, int v) {
  for (int u : tile_variants(pb, p))
    if (u == v) return true;
  for (int q : {1, 2, 4})
    if (default_variant(pb, p, q) == v) return true;
  return false;
}

// corner_lists: the generic instances (each corner's term lists) even where
// grouped ones exist.
int launch_tiles(const sdi_problem* pb, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a,
                 hipStream_t st, bool corner_lists = false) {
  if (pb->is_expr()) return launch_tiles_expr(grid, shmem, a, expr_args(pb), st);
  if (pb->complex_mode) return launch_tiles_cplx(pb->nvmax, ppt, wpe, km, grid, shmem, a, pb->d_cx, pb->d_dir, st);
  if (pb->exp7) return launch_tiles_real_e7(pb->nvmax, km, grid, shmem, a, st);
  return launch_tiles_real(pb->nvmax, pb->nsmax, corner_lists ? MAXF + 1 : pb->nfmax, ppt, wpe, km, grid, shmem, a,
                           st);
}

int persistent_grid(sdi_ctx* ctx, const sdi_problem* pb, int mode, int ppt, int wpe, int km, size_t shmem,
                    size_t ntiles, bool corner_lists = false) {
  const int nvmax = pb->nvmax;
  const int nf = corner_lists ? MAXF + 1 : pb->nfmax;
  int occ = pb->is_expr()                             ? tiles_expr_occupancy(mode, shmem, expr_args(pb))
            : pb->complex_mode ? tiles_cplx_occupancy(nvmax, mode, ppt, wpe, km, uses_dd(pb, ctx->params), shmem)
            : pb->exp7 ? occupancy_tiles_real_e7(nvmax, mode, km, uses_dd(pb, ctx->params), shmem)
                                                      : tiles_real_occupancy(nvmax, pb->nsmax, nf, mode, ppt, wpe, km,
                                                                             uses_dd(pb, ctx->params), shmem);
  if (occ < 1) occ = 1;
  const size_t g = (size_t)occ * std::max(ctx->ncu, 1);
  return (int)std::max<size_t>(1, std::min(g, ntiles));
}

std::string pass_key(const Params& p, const std::vector<int>& msec, bool warm, const void* ws, size_t wsb,
                     uint32_t lo = 0, uint32_t hi = 0) {
  char buf[360];
  unsigned long long h = 1469598103934665603ull;
  for (int m : msec) h = (h ^ (unsigned)m) * 1099511628211ull;
  snprintf(buf, sizeof buf, "R%d s%llu b%d w%d/%d mw%d nb%d t%d p%d g%d f%d i%d x%.17g m%llx ws%p:%zu r%u:%u", p.R,
           (unsigned long long)p.seed, p.baker, p.warmup, (int)warm, p.mw, p.nbins, p.tile_log2, p.ppt, p.graph,
           p.sampler, p.integrator, p.small_x, h, ws, wsb, lo, hi);
  return buf;
}

TileArgs base_args(const sdi_problem* pb, const Plan& P) {
  TileArgs A{};
  A.secs = P.d_secs;
  A.terms = pb->d_terms;
  A.shifts = P.d_shifts;
  A.grids = pb->d_grids;
  return A;
}

// The final pass's lattice tiles (flow = false) or flow-sampled tiles (flow = true).
TileArgs final_args(const sdi_problem* pb, const Plan& P, bool flow = false) {
  TileArgs F = base_args(pb, P);
  F.zp = P.d_zp_final;
  F.tiles = P.d_ftiles;
  F.order = flow ? P.d_xorder : P.d_forder;
  F.partial = P.d_partial;
  F.nonfinite = P.d_nonfinite;
  F.counter = P.d_counter + (flow ? 2 : 1);
  F.ntiles = (int)(flow ? P.xorder.size() : P.forder.size());
  F.mode = flow ? 2 : 0;
  F.px = P.d_px;
  F.pw = P.d_pw;
  F.x_off = P.d_fx_off;
  F.pt_off = P.d_fpt_off;
  F.small_x = P.small_x;
  return F;
}

// Enqueue one segment of a pass on st: 0 = shifts and warm-up iterations,
// 1 = the final-pass tile kernel, 2 = reductions and combination.
int record_segment(sdi_ctx* ctx, sdi_problem* pb, PassState& S, int seg, hipStream_t st) {
  const Params& prm = ctx->params;
  Plan& P = S.P;
  const int nsec = pb->nsec;
  const int npairs = (int)P.pair_sector.size();
  if (seg == 0) {
    KCHK(ctx, launch_shifts(P.d_secs, nsec, P.rows, prm.R, prm.seed, 0u, P.d_shifts, st));
    if (P.flow) {
      const FlowState& Fl = *pb->flow;
      FlowTileArgs A{};
      A.fs = Fl.d_desc;
      A.params = Fl.d_params;
      A.bw = Fl.d_bw;
      A.zp = P.d_zp_final;
      A.shifts = P.d_shifts;
      A.tiles = P.d_fruns;
      A.chunk_prefix = P.d_fchunk;
      A.ntiles = (int)P.fruns.size();
      A.baker = prm.baker;
      A.nchunks = P.fchunk.back();
      A.x = P.d_px;
      A.w = P.d_pw;
      A.lq = nullptr;
      KCHK(ctx, launch_flow_sample_tiles(A, pb->nvmax, st));
    }
    if (P.warm) {
      KCHK(ctx, launch_grid_identity(P.d_secs, nsec, pb->d_grids, st));
      const int nwt = (int)P.wtiles.size();
      for (int it = 0; it < prm.warmup; ++it) {
        KCHK(ctx, launch_fill_i32(P.d_counter, 0, 1, st));
        TileArgs W = base_args(pb, P);
        W.zp = P.d_zp_warm;
        W.tiles = P.d_wtiles + (size_t)it * nwt;
        W.order = P.d_worder;
        W.partial = P.d_wpartial;
        W.nonfinite = P.d_wnonfinite;
        W.hist = P.d_whist;
        W.hist_off = P.d_whist_off;
        W.counter = P.d_counter;
        W.ntiles = nwt;
        W.mode = 1;
        KCHK(ctx, launch_tiles(pb, S.ppt, S.wpe, S.km, S.gw, P.shmem_warm, W, st));
        KCHK(ctx, launch_hist_reduce(P.d_whist, P.d_whist_off, P.d_wsec_start, P.d_secs, P.d_hsec_off, nsec,
                                     P.hsec_total, P.d_hsec_prefix, P.d_hsec, st));
        KCHK(ctx, launch_refit(P.d_secs, nsec, P.d_hsec, P.d_hsec_off, pb->d_grids, 1.5, st));
      }
    }
    if (P.mc) {
      // Monte Carlo points through the grids the warm-up has just left
      McArgs M{};
      M.secs = P.d_secs;
      M.runs = P.d_fruns;
      M.chunk_prefix = P.d_fchunk;
      M.nruns = (int32_t)P.fruns.size();
      M.nchunks = P.fchunk.back();
      M.grids = pb->d_grids;
      M.seed = prm.seed;
      M.x = P.d_px;
      M.w = P.d_pw;
      KCHK(ctx, launch_mc_points(M, st));
    }
  } else if (seg == 1) {
    KCHK(ctx, launch_fill_i32(P.d_counter + 1, 0, 2, st));
    if (!P.forder.empty())
      KCHK(ctx, launch_tiles(pb, S.ppt, S.wpe, S.km, S.gf, P.shmem_final, final_args(pb, P), st, S.lists));
    if (!P.xorder.empty())
      KCHK(ctx, launch_tiles(pb, 1, 4, S.km, S.gx, P.shmem_final, final_args(pb, P, true), st));
  } else {
    const bool sliced = P.range_hi != 0;
    KCHK(ctx, launch_reduce_pairs(P.d_partial, P.d_pair_start, P.d_pair_sector, P.d_secs, npairs, P.d_per_shift,
                                  P.d_nonfinite, P.d_pair_nonfinite, sliced && P.range_lo ? P.d_carry_in : nullptr,
                                  sliced && P.range_lo ? P.d_carry_in_counts : nullptr, sliced ? P.d_carry_out : nullptr,
                                  sliced ? P.d_carry_out_counts : nullptr, sliced ? (int64_t)P.range_hi : 0, st));
    KCHK(ctx, launch_sector_stats(P.d_per_shift, nsec, prm.R, P.d_sec_stats, P.d_pair_nonfinite, P.d_sec_nonfinite,
                                  st));
    KCHK(ctx, launch_combine(P.d_sec_stats, nsec, P.d_sec_nonfinite, P.d_res, P.d_counts, st));
  }
  return SDI_OK;
}

// Final-pass tile sizes (log2) to consider: the requested one, or under
// tile_log2 = 0 every size from 2^10 to 2^14 points (2^6 to 2^10 for text
// integrands, whose blocks are one wave) that is not longer than the longest
// lattice (a tile never exceeds its sector's lattice, so larger sizes would
// repeat a plan) and gives at most about 2^20 tiles, largest first.  Without tuning the automatic size is 2^14
// (2^6 for text integrands: one tile per wave-step keeps every wave busy).
std::vector<int> tile_candidates(const sdi_problem* pb, const Params& prm, const std::vector<int>& msec) {
  if (prm.tile_log2 > 0) return {prm.tile_log2};
  const int top = pb->is_expr() ? 10 : 14;
  if (prm.tune == 0) return {pb->is_expr() ? 6 : 14};
  int mmax = 4;
  double total = 0.0;   // points of one pass
  for (int m : msec) {
    mmax = std::max(mmax, m);
    total += std::ldexp((double)prm.R, m);
  }
  const int hi = std::min(top, mmax);
  int lo = std::min(top - 4, hi);
  // smaller tiles than needed for 2^20 tiles only add plan and partial-sum size
  while (lo < hi && total / std::ldexp(1.0, lo) > (double)(1 << 20)) ++lo;
  std::vector<int> v;
  for (int t = hi; t >= lo; --t) v.push_back(t);
  return v;
}

// Builds the plan for one tile size on dev_ws (or on the pass's own
// allocation), uploads it and waits for the copies.
int setup_pass(sdi_ctx* ctx, sdi_problem* pb, PassState& S, const std::vector<int>& msec, bool warm, int tile_log2,
               void* dev_ws, size_t ws_bytes, uint32_t lo = 0, uint32_t hi = 0) {
  const Params& prm = ctx->params;
  int rc = make_plan(ctx, pb, S.P, msec, warm, tile_log2, lo, hi);
  if (rc != SDI_OK) return rc;
  Plan& P = S.P;
  const size_t need = P.carve.total();
  void* base = dev_ws;
  if (base) {
    if (ws_bytes < need) return fail(ctx, SDI_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  } else {
    if (hipMalloc(&S.own_ws, need) != hipSuccess) {
      S.own_ws = nullptr;
      (void)hipGetLastError();
      return fail(ctx, SDI_ENOMEM, "workspace allocation failed");
    }
    base = S.own_ws;
  }
  P.carve.assign(base);
  for (auto& e : S.ev) HIPCHK(ctx, hipEventCreate(&e));
  hipStream_t st = ctx->stream;
  const int nsec = pb->nsec;
  const int npairs = (int)P.pair_sector.size();
  const int nft = (int)P.ftiles.size();
  HIPCHK(ctx, hipMemcpyAsync(P.d_secs, P.secs.data(), (size_t)nsec * sizeof(SecDev), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_ftiles, P.ftiles.data(), nft * sizeof(TileDesc), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_forder, P.forder.data(), P.forder.size() * 4, hipMemcpyHostToDevice, st));
  if (!P.xorder.empty())
    HIPCHK(ctx, hipMemcpyAsync(P.d_xorder, P.xorder.data(), P.xorder.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_pair_start, P.pair_start.data(), (npairs + 1) * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_pair_sector, P.pair_sector.data(), npairs * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_zp_final, P.zp_final.data(), P.zp_final.size() * 8, hipMemcpyHostToDevice, st));
  if (P.flow || P.mc) {
    HIPCHK(ctx, hipMemcpyAsync(P.d_fruns, P.fruns.data(), P.fruns.size() * sizeof(PointRun), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_fchunk, P.fchunk.data(), P.fchunk.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_fx_off, P.fx_off.data(), P.fx_off.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_fpt_off, P.fpt_off.data(), P.fpt_off.size() * 8, hipMemcpyHostToDevice, st));
  }
  std::vector<TileDesc> wall;
  if (P.warm) {
    const size_t nwt = P.wtiles.size();
    wall.reserve(nwt * prm.warmup);
    for (int it = 0; it < prm.warmup; ++it)
      for (const TileDesc& t : P.wtiles) wall.push_back(TileDesc{t.sector, prm.R + it, t.i0, t.count});
    HIPCHK(ctx, hipMemcpyAsync(P.d_zp_warm, P.zp_warm.data(), P.zp_warm.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_wtiles, wall.data(), wall.size() * sizeof(TileDesc), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_worder, P.worder.data(), nwt * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_whist_off, P.whist_off.data(), nwt * 8, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_wsec_start, P.wsec_start.data(), (nsec + 1) * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_hsec_off, P.hsec_off.data(), nsec * 8, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_hsec_prefix, P.hsec_prefix.data(), nsec * 8, hipMemcpyHostToDevice, st));
  }
  HIPCHK(ctx, hipStreamSynchronize(st));
  S.km = pb->kfmax <= 4 ? 4 : 8;
  return SDI_OK;
}

// Device time of one final-pass tile launch of an encoded variant on S's
// lattice tiles: the fastest of the launches after the first (which warms
// caches and code); three of them when a launch is short.
int time_final(sdi_ctx* ctx, sdi_problem* pb, PassState& S, int variant, float* ms_out) {
  const Params& prm = ctx->params;
  hipStream_t st = ctx->stream;
  Plan& P = S.P;
  KCHK(ctx, launch_shifts(P.d_secs, pb->nsec, P.rows, prm.R, prm.seed, 0u, P.d_shifts, st));
  if (prm.warmup > 0 && !pb->grid_valid) KCHK(ctx, launch_grid_identity(P.d_secs, pb->nsec, pb->d_grids, st));
  const TileArgs F = final_args(pb, P);
  const bool lists = variant >= CORNER_LISTS;
  const int ppt = (variant % CORNER_LISTS) / 10, wpe = variant % 10;
  const int g = persistent_grid(ctx, pb, 0, ppt, wpe, S.km, P.shmem_final, P.forder.size(), lists);
  float best = 0.f;
  int reps = 2;
  for (int rep = 0; rep < reps; ++rep) {
    float ms = 0.f;
    KCHK(ctx, launch_fill_i32(F.counter, 0, 1, st));
    HIPCHK(ctx, hipEventRecord(S.ev[1], st));
    KCHK(ctx, launch_tiles(pb, ppt, wpe, S.km, g, P.shmem_final, F, st, lists));
    HIPCHK(ctx, hipEventRecord(S.ev[2], st));
    HIPCHK(ctx, hipEventSynchronize(S.ev[2]));
    HIPCHK(ctx, hipEventElapsedTime(&ms, S.ev[1], S.ev[2]));
    if (rep == 0) {
      if (ms < 20.f) reps = 4;
      continue;
    }
    if (rep == 1 || ms < best) best = ms;
  }
  *ms_out = best;
  return SDI_OK;
}

// Everything the tuned launch depends on: device, kernel build, problem class
// and shape, per-sector lattice sizes, the tile and points-per-thread requests.
std::string tune_key(const sdi_ctx* ctx, const sdi_problem* pb, const std::vector<int>& msec, bool warm) {
  const Params& p = ctx->params;
  unsigned long long h = 1469598103934665603ull;
  for (int m : msec) h = (h ^ (unsigned)m) * 1099511628211ull;
  if (p.sampler == 1 && pb->flow)
    for (uint8_t a : pb->flow->active) h = (h ^ a) * 1099511628211ull;
  char buf[320];
  snprintf(buf, sizeof buf, "%s|c%d|x%d|nv%d|ns%d|nf%d|kf%d|sec%d|terms%zu|m%llx|R%d|w%d|t%d|p%d|s%d|d%d",
           ctx->prop.gcnArchName, pb->complex_mode, (int)pb->is_expr(), pb->nvmax, pb->nsmax, pb->nfmax, pb->kfmax,
           pb->nsec,
           pb->is_expr() ? pb->expr_nins : pb->terms.size(), h, p.R, (int)(warm && p.warmup > 0), p.tile_log2, p.ppt,
           p.sampler, (int)uses_dd(pb, p));
  return buf;
}

// The autotuner: times the final-pass tile kernel on the problem's own tiles
// for every launch variant (points per thread x minimum waves per SIMD) at the
// largest candidate tile size, then for each smaller tile size with the best
// variant so far, then every variant at the best tile size, and keeps the
// fastest pair.  Results are cached per
// tune_key (and can be saved and loaded with the kernel build's hash).
// fixed_variant >= 0 skips the variant search.  With a caller workspace every
// candidate plan is built on it in turn; a size that does not fit is skipped.
int autotune(sdi_ctx* ctx, sdi_problem* pb, const std::vector<int>& msec, bool warm, const std::vector<int>& tiles,
             int fixed_variant, void* dev_ws, size_t ws_bytes, TuneChoice& out, uint32_t lo = 0, uint32_t hi = 0) {
  const Params& prm = ctx->params;
  const std::string key = tune_key(ctx, pb, msec, warm);
  if (prm.tune == 1)
    for (const TuneEntry& e : ctx->tune_cache)
      if (e.key == key && variant_known(pb, prm, e.variant) &&
          std::find(tiles.begin(), tiles.end(), e.tile_log2) != tiles.end() &&
          (fixed_variant < 0 || e.variant == fixed_variant)) {
        out = TuneChoice{e.tile_log2, e.variant};
        return SDI_OK;
      }
  TuneChoice best{tiles.front(), fixed_variant >= 0 ? fixed_variant : default_variant(pb, prm, 1)};
  float best_ms = 1e30f;
  ctx->tune_report.clear();
  // Coordinate search: every variant at the largest tile size, every tile size
  // with the best variant, then every variant again at the best tile size.
  std::vector<std::pair<int, std::vector<int>>> rounds;
  const std::vector<int> all = fixed_variant >= 0 ? std::vector<int>{fixed_variant} : tile_variants(pb, prm);
  rounds.push_back({tiles.front(), all});
  for (size_t i = 1; i < tiles.size(); ++i) rounds.push_back({tiles[i], {}});
  if (tiles.size() > 1 && all.size() > 1) rounds.push_back({-1, all});
  for (size_t r = 0; r < rounds.size(); ++r) {
    const int tl = rounds[r].first < 0 ? best.tile_log2 : rounds[r].first;
    if (rounds[r].first < 0 && tl == tiles.front()) break;   // the first round already timed these
    PassState C;
    int rc = setup_pass(ctx, pb, C, msec, warm, tl, dev_ws, ws_bytes, lo, hi);
    if (rc == SDI_ENOMEM && r > 0) {
      ctx->err.clear();
      continue;
    }
    if (rc != SDI_OK) return rc;
    if (C.P.forder.empty()) break;   // no lattice tiles to time
    const std::vector<int> vs = rounds[r].second.empty() ? std::vector<int>{best.variant} : rounds[r].second;
    for (int v : vs) {
      if (rounds[r].first < 0 && v == best.variant) continue;   // timed in the tile round
      float ms = 0.f;
      rc = time_final(ctx, pb, C, v, &ms);
      if (rc != SDI_OK) return rc;
      {
        char line[96];
        snprintf(line, sizeof line, "tile_log2=%d ppt=%d waves=%d lists=%d ms=%.4f\n", tl, (v % CORNER_LISTS) / 10,
                 v % 10, (int)(v >= CORNER_LISTS), ms);
        ctx->tune_report += line;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = TuneChoice{tl, v};
      }
    }
  }
  bool found = false;
  for (TuneEntry& e : ctx->tune_cache)
    if (e.key == key) {
      e.tile_log2 = best.tile_log2;
      e.variant = best.variant;
      found = true;
    }
  if (!found) ctx->tune_cache.push_back(TuneEntry{key, best.tile_log2, best.variant});
  out = best;
  return SDI_OK;
}

// The cached pass for (parameters, per-sector lattice sizes, warm-up flag,
// workspace), tuned, built, uploaded and captured on first use.
int get_pass(sdi_ctx* ctx, sdi_problem* pb, const std::vector<int>& msec, bool warm, void* dev_ws, size_t ws_bytes,
             PassState** out, uint32_t lo = 0, uint32_t hi = 0) {
  const Params& prm = ctx->params;
  const std::string key = pass_key(prm, msec, warm, dev_ws, ws_bytes, lo, hi);
  for (size_t i = 0; i < pb->passes.size(); ++i)
    if (pb->passes[i]->key == key) {
      *out = pb->passes[i];
      return SDI_OK;
    }
  // plans on a caller workspace share it: drop them before anything writes there
  if (dev_ws) {
    for (size_t i = 0; i < pb->passes.size();)
      if (!pb->passes[i]->own_ws) {
        delete pb->passes[i];
        pb->passes.erase(pb->passes.begin() + i);
      } else {
        ++i;
      }
  }
  const std::vector<int> tiles = tile_candidates(pb, prm, msec);
  TuneChoice ch{tiles.front(), -1};
  if (!pb->complex_mode && !pb->is_expr() && final_family(pb, prm) == RF_DD)
    ch.variant = DD_VARIANT;
  else if (prm.ppt > 0)
    ch.variant = default_variant(pb, prm, prm.ppt);
  else if (prm.tune == 0)
    ch.variant = (pb->complex_mode || pb->is_expr()) ? 11 : default_variant(pb, prm, 2);
  if (ch.variant < 0 || tiles.size() > 1) {
    const int rc = autotune(ctx, pb, msec, warm, tiles, ch.variant, dev_ws, ws_bytes, ch, lo, hi);
    if (rc != SDI_OK) return rc;
  }
  PassState* S = new PassState();
  int rc = setup_pass(ctx, pb, *S, msec, warm, ch.tile_log2, dev_ws, ws_bytes, lo, hi);
  if (rc != SDI_OK) {
    delete S;
    return rc;
  }
  // keep at most four plans
  if (pb->passes.size() >= 4) {
    delete pb->passes.front();
    pb->passes.erase(pb->passes.begin());
  }
  pb->passes.push_back(S);
  hipStream_t st = ctx->stream;
  Plan& P = S->P;
  S->lists = ch.variant >= CORNER_LISTS;
  S->ppt = (ch.variant % CORNER_LISTS) / 10;
  S->wpe = ch.variant % 10;
  S->gf = persistent_grid(ctx, pb, 0, S->ppt, S->wpe, S->km, P.shmem_final, std::max<size_t>(1, P.forder.size()),
                          S->lists);
  // explicit (flow) points are read by the one-point-per-thread instances
  S->gx = persistent_grid(ctx, pb, 2, 1, 4, S->km, P.shmem_final, std::max<size_t>(1, P.xorder.size()));
  S->gw = P.warm ? persistent_grid(ctx, pb, 1, S->ppt, S->wpe, S->km, P.shmem_warm, P.wtiles.size()) : 1;
  if (prm.graph) {
    // Capture each segment once; replays skip the launch overheads.  Timing
    // events stay outside the graphs, between segment launches.  Any failure
    // falls back to eager launches for that segment.
    for (int seg = 0; seg < 3; ++seg) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      const int rr = record_segment(ctx, pb, *S, seg, st);
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (!(rr == SDI_OK && ec == hipSuccess && g &&
            hipGraphInstantiate(&S->exec[seg], g, nullptr, nullptr, 0) == hipSuccess))
        S->exec[seg] = nullptr;
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
    }
    ctx->err.clear();
  }
  S->key = key;
  *out = S;
  return SDI_OK;
}

struct PassOut {
  std::vector<double> res, sec_stats, per_shift, carry;
  std::vector<int64_t> carry_counts;
  int64_t counts[2] = {0, 0};
  float ms_warm = 0.f, ms_final = 0.f, ms_kernel = 0.f;
};

int run_pass(sdi_ctx* ctx, sdi_problem* pb, PassState& S, PassOut& o) {
  hipStream_t st = ctx->stream;
  Plan& P = S.P;
  const size_t npairs = P.pair_sector.size();
  if (P.range_hi && P.range_lo) {
    if (pb->resume_sums.size() != npairs * KMAX * 4 || pb->resume_counts.size() != npairs * 2)
      return fail(ctx, SDI_ESTATE, "resumable pass: no sums of the earlier slices");
    HIPCHK(ctx, hipMemcpyAsync(P.d_carry_in, pb->resume_sums.data(), npairs * KMAX * 4 * 8, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(P.d_carry_in_counts, pb->resume_counts.data(), npairs * 16, hipMemcpyHostToDevice, st));
  }
  for (int seg = 0; seg < 3; ++seg) {
    HIPCHK(ctx, hipEventRecord(S.ev[seg], st));
    if (S.exec[seg]) {
      HIPCHK(ctx, hipGraphLaunch(S.exec[seg], st));
    } else {
      const int rc = record_segment(ctx, pb, S, seg, st);
      if (rc != SDI_OK) return rc;
    }
  }
  HIPCHK(ctx, hipEventRecord(S.ev[3], st));
  o.res.assign(KMAX * 4, 0.0);
  o.sec_stats.assign((size_t)pb->nsec * KMAX * 4, 0.0);
  o.per_shift.assign(P.pair_sector.size() * KMAX * 2, 0.0);
  HIPCHK(ctx, hipMemcpyAsync(o.res.data(), P.d_res, o.res.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(o.counts, P.d_counts, 16, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(o.sec_stats.data(), P.d_sec_stats, o.sec_stats.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(o.per_shift.data(), P.d_per_shift, o.per_shift.size() * 8, hipMemcpyDeviceToHost, st));
  if (P.range_hi) {
    o.carry.assign(npairs * KMAX * 4, 0.0);
    o.carry_counts.assign(npairs * 2, 0);
    HIPCHK(ctx, hipMemcpyAsync(o.carry.data(), P.d_carry_out, npairs * KMAX * 4 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(o.carry_counts.data(), P.d_carry_out_counts, npairs * 16, hipMemcpyDeviceToHost, st));
  }
  HIPCHK(ctx, hipStreamSynchronize(st));
  HIPCHK(ctx, hipEventElapsedTime(&o.ms_warm, S.ev[0], S.ev[1]));
  HIPCHK(ctx, hipEventElapsedTime(&o.ms_kernel, S.ev[1], S.ev[2]));
  HIPCHK(ctx, hipEventElapsedTime(&o.ms_final, S.ev[1], S.ev[3]));
  return SDI_OK;
}

}  // namespace

// Settings a resumable pass's sums belong to: a slice continues the sums of
// the earlier ones only under the same lattice, shifts, seed, tent map, slice
// and launch requests (the tile size and points per thread decide which
// points a block sums, so they fix the rounding of the partial sums).
std::string resume_key(const Params& p, int nsec) {
  char buf[256];
  snprintf(buf, sizeof buf, "n%d m%d R%d s%llu b%d sl%d t%d p%d x%.17g", nsec, p.m, p.R, (unsigned long long)p.seed,
           p.baker, p.slice_log2, p.tile_log2, p.ppt, p.small_x);
  return buf;
}

// Neyman-style allocation of the final-pass budget: for every order k with a
// nonzero total, sector s gets the weight sigma_{s,k} / sqrt(sum_s sigma_{s,k}^2)
// (sigma^2 = err_re^2 + err_im^2 of the pilot); weights add over orders and
// the sector's share is n_s = budget * weight_s / sum weight (equal shares when
// every pilot error is zero).  Lattices are powers of two: every sector starts
// at the largest m in [alloc_min, alloc_max] with R 2^m <= n_s (alloc_min if
// none); then, while a doubling fits in the budget, the sector furthest below
// its share (largest n_s / 2^m, ties to the lower index) among those that can
// still double is doubled.  The budget is spent to within one doubling.
std::vector<int> neyman_allocation(const sdi_problem* pb, const std::vector<double>& sec_stats, const Params& prm) {
  const int nsec = pb->nsec;
  std::vector<double> wsec(nsec, 0.0);
  for (int k = 0; k < pb->K; ++k) {
    double tot = 0.0;
    for (int s = 0; s < nsec; ++s) {
      const double* q = sec_stats.data() + ((size_t)s * KMAX + k) * 4;
      tot += q[2] * q[2] + q[3] * q[3];
    }
    if (!(tot > 0.0) || !std::isfinite(tot)) continue;
    const double rt = std::sqrt(tot);
    for (int s = 0; s < nsec; ++s) {
      const double* q = sec_stats.data() + ((size_t)s * KMAX + k) * 4;
      wsec[s] += std::sqrt(q[2] * q[2] + q[3] * q[3]) / rt;
    }
  }
  double W = 0.0;
  for (double w : wsec) W += w;
  std::vector<double> share(nsec);
  std::vector<int> m(nsec);
  int64_t used = 0;
  for (int s = 0; s < nsec; ++s) {
    share[s] = W > 0.0 ? (double)prm.budget * wsec[s] / W : (double)prm.budget / nsec;
    int v = prm.alloc_min;
    while (v < prm.alloc_max && (double)prm.R * std::ldexp(1.0, v + 1) <= share[s]) ++v;
    m[s] = v;
    used += (int64_t)prm.R << v;
  }
  // greedy doublings: largest share / 2^m first; a sector that does not fit
  // now never fits later (the remaining budget only shrinks)
  auto worse = [&](int a, int b) {
    const double ra = std::ldexp(share[a], -m[a]), rb = std::ldexp(share[b], -m[b]);
    return ra < rb || (ra == rb && a > b);
  };
  std::vector<int> heap;
  for (int s = 0; s < nsec; ++s)
    if (m[s] < prm.alloc_max) heap.push_back(s);
  std::make_heap(heap.begin(), heap.end(), worse);
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end(), worse);
    const int s = heap.back();
    heap.pop_back();
    const int64_t cost = (int64_t)prm.R << m[s];
    if (used + cost > prm.budget) continue;
    used += cost;
    ++m[s];
    if (m[s] < prm.alloc_max) {
      heap.push_back(s);
      std::push_heap(heap.begin(), heap.end(), worse);
    }
  }
  return m;
}

}  // namespace sdi

namespace {

// Minimal reader for the file sdi_tune_save writes: string values hold no
// quotes or escapes, numbers are small integers.
struct TuneReader {
  const std::string& t;
  size_t p = 0;
  explicit TuneReader(const std::string& s) : t(s) {}
  void ws() {
    while (p < t.size() && (t[p] == ' ' || t[p] == '\n' || t[p] == '\r' || t[p] == '\t')) ++p;
  }
  bool lit(char c) {
    ws();
    if (p < t.size() && t[p] == c) {
      ++p;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    if (!lit('"')) return false;
    const size_t q = t.find('"', p);
    if (q == std::string::npos) return false;
    out = t.substr(p, q - p);
    if (out.find('\\') != std::string::npos) return false;
    p = q + 1;
    return true;
  }
  bool num(int& out) {
    ws();
    size_t q = p;
    if (q < t.size() && t[q] == '-') ++q;
    const size_t d0 = q;
    while (q < t.size() && t[q] >= '0' && t[q] <= '9' && q - d0 < 9) ++q;
    if (q == d0 || (q < t.size() && t[q] >= '0' && t[q] <= '9')) return false;
    out = std::stoi(t.substr(p, q - p));
    p = q;
    return true;
  }
};

}  // namespace

using namespace sdi;

extern "C" {

size_t sdi_workspace_bytes(sdi_ctx* ctx, const sdi_problem* prob) {
  if (!ctx || !prob) return 0;
  const Params& prm = ctx->params;
  Plan P;
  sdi_problem tmp = *prob;        // make_plan may resize the problem's grids; plan on a copy
  tmp.passes.clear();
  tmp.d_grids = nullptr;
  tmp.grid_doubles = (size_t)-1;
  tmp.grid_nbins = prm.nbins;
  // with allocation the largest final pass is every sector at alloc_max
  const int m = prm.budget > 0 ? prm.alloc_max : prm.m;
  const std::vector<int> msec(prob->nsec, m);
  // every tile size the autotuner may try is built on the same workspace
  size_t need = 0;
  for (int t : tile_candidates(prob, prm, msec)) {
    if (make_plan(ctx, &tmp, P, msec, prm.budget == 0, t) != SDI_OK) return 0;
    need = std::max(need, P.carve.total());
  }
  return need;
}

int sdi_integrate(sdi_ctx* ctx, sdi_problem* pb, void* dev_ws, size_t ws_bytes, sdi_result* out) {
  if (!ctx || !pb || !out) return fail(ctx, SDI_EINVAL, "integrate: null argument");
  if (pb->ctx != ctx) return fail(ctx, SDI_EINVAL, "problem belongs to another context");
  if (!out->val_re || !out->val_im || !out->err_re || !out->err_im)
    return fail(ctx, SDI_EINVAL, "integrate: result arrays must be allocated");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  const Params& prm = ctx->params;
  if (prm.integrator == 1 || prm.integrator >= 3) return run_cubature(ctx, pb, out);
  if (prm.budget > 0 && dev_ws) return fail(ctx, SDI_ENOTSUP, "budget allocation needs the library workspace");
  if (prm.alloc_min > prm.alloc_max) return fail(ctx, SDI_EINVAL, "alloc_min_log2 > alloc_max_log2");
  const int nsec = pb->nsec;
  // resumable pass: this call's slice [lo, hi) of every shift
  uint32_t lo = 0, hi = 0;
  std::string rkey;
  if (prm.slice_log2 > 0) {
    if (prm.budget > 0 || prm.warmup > 0 || prm.sampler != 0 || prm.integrator != 0)
      return fail(ctx, SDI_ENOTSUP,
                  "slice_log2 needs a uniform lattice pass (budget 0, warmup 0, sampler 0, integrator 0)");
    rkey = resume_key(prm, nsec);
    const uint32_t N = 1u << prm.m;
    if (pb->resume_key != rkey || pb->resume_done <= 0 || pb->resume_done >= (int64_t)N) pb->resume_done = 0;
    lo = (uint32_t)pb->resume_done;
    hi = (uint32_t)std::min<uint64_t>(N, (uint64_t)lo + (1ull << std::min(prm.slice_log2, 31)));
    if (lo == 0) {
      pb->resume_sums.clear();
      pb->resume_counts.clear();
    }
  }
  PassOut o;
  float ms_pilot = 0.f, ms_pilot_kernel = 0.f;
  std::vector<int> pilot_kernel;   // launch variant of the pilot's tile kernel
  int64_t pilot_evals = 0;
  std::vector<int> msec(nsec, prm.m);
  bool warm = prm.warmup > 0;
  PassState* S = nullptr;
  int rc;
  if (prm.budget > 0) {
    rc = get_pass(ctx, pb, std::vector<int>(nsec, prm.pilot_log2), warm, nullptr, 0, &S);
    if (rc != SDI_OK) return rc;
    rc = run_pass(ctx, pb, *S, o);
    if (rc != SDI_OK) return rc;
    ms_pilot = o.ms_warm + o.ms_final;
    ms_pilot_kernel = o.ms_kernel;
    pilot_kernel = {S->ppt, S->wpe, S->lists ? 1 : 0, S->km};
    if (prm.warmup > 0) pb->grid_valid = true;   // the final pass reuses the adapted grids
    pilot_evals = ((int64_t)prm.R << prm.pilot_log2) * nsec;
    msec = neyman_allocation(pb, o.sec_stats, prm);
    warm = false;
  }
  rc = get_pass(ctx, pb, msec, warm, dev_ws, ws_bytes, &S, lo, hi);
  if (rc != SDI_OK) return rc;
  const bool had_warm = S->P.warm;
  rc = run_pass(ctx, pb, *S, o);
  if (rc != SDI_OK) return rc;
  if (prm.warmup > 0 && (had_warm || prm.budget > 0)) pb->grid_valid = true;
  if (prm.warmup == 0) pb->grid_valid = false;
  pb->last_R = prm.R;
  pb->have_results = true;
  pb->last_sampler = prm.sampler;
  pb->last_m = prm.budget > 0 ? -1 : prm.m;
  pb->last_warmup = prm.warmup;
  pb->last_seed = prm.seed;
  pb->sec_stats = o.sec_stats;
  pb->per_shift = o.per_shift;
  pb->sec_evals.assign(nsec, 0);
  int64_t final_evals = 0;
  for (int s = 0; s < nsec; ++s) {
    pb->sec_evals[s] = hi ? (int64_t)prm.R * hi : (int64_t)prm.R << msec[s];
    final_evals += hi ? (int64_t)prm.R * (hi - lo) : pb->sec_evals[s];
  }
  if (hi) {
    pb->resume_sums = o.carry;
    pb->resume_counts = o.carry_counts;
    pb->resume_done = hi;
    pb->resume_key = rkey;
  }
  out->lattice_done = hi ? (int64_t)hi : ((int64_t)1 << prm.m);
  if (pb->flow) {
    out->ms_flow_train = pb->flow->train_ms_pending;
    pb->flow->train_ms_pending = 0.0;
  } else {
    out->ms_flow_train = 0.0;
  }
  out->order_min = pb->order_min;
  out->norders = pb->K;
  for (int k = 0; k < pb->K; ++k) {
    out->val_re[k] = o.res[k * 4 + 0];
    out->val_im[k] = o.res[k * 4 + 1];
    out->err_re[k] = o.res[k * 4 + 2];
    out->err_im[k] = o.res[k * 4 + 3];
  }
  out->n_evals = final_evals + pilot_evals + (prm.warmup > 0 ? (int64_t)prm.warmup * nsec * ((int64_t)1 << prm.mw) : 0);
  out->n_nonfinite = o.counts[0];
  out->n_imf_positive = o.counts[1];
  out->ms_sample_eval_reduce = o.ms_final;
  out->ms_refit = o.ms_warm + ms_pilot;
  out->ms_total = o.ms_warm + o.ms_final + ms_pilot;
  out->ms_eval_kernel = o.ms_kernel;
  out->ms_pilot_kernel = ms_pilot_kernel;
  out->pilot_same_kernel = pilot_kernel == std::vector<int>{S->ppt, S->wpe, S->lists ? 1 : 0, S->km} ? 1 : 0;
  out->points_per_thread = S->ppt;
  out->blocks = S->gf;
  out->tile_log2 = S->P.tile_log2;
  out->waves_per_simd = S->wpe;
  out->grouped = (!pb->complex_mode && !pb->is_expr() && !S->lists &&
                  (final_family(pb, prm) == RF_S2 || final_family(pb, prm) == RF_G3 ||
                   final_family(pb, prm) == RF_G4))
                     ? 1
                     : 0;
  return o.counts[0] ? fail(ctx, SDI_ENONFINITE, "non-finite integrand values") : SDI_OK;
}

int sdi_sector_results(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, double* mean, double* err, double* per_shift,
                       int64_t* nevals) {
  if (!ctx || !pb || !mean || !err) return fail(ctx, SDI_EINVAL, "sector_results: null argument");
  if (!pb->have_results) return fail(ctx, SDI_ESTATE, "no integration has run on this problem");
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  for (int k = 0; k < pb->K; ++k) {
    const double* q = pb->sec_stats.data() + ((size_t)s * KMAX + k) * 4;
    mean[2 * k] = q[0];
    mean[2 * k + 1] = q[1];
    err[2 * k] = q[2];
    err[2 * k + 1] = q[3];
  }
  if (per_shift)
    for (int r = 0; r < pb->last_R; ++r)
      for (int k = 0; k < pb->K; ++k) {
        const double* q = pb->per_shift.data() + (((size_t)s * pb->last_R + r) * KMAX + k) * 2;
        per_shift[((size_t)r * pb->K + k) * 2] = q[0];
        per_shift[((size_t)r * pb->K + k) * 2 + 1] = q[1];
      }
  if (nevals) *nevals = pb->sec_evals[s];
  return SDI_OK;
}

}  // extern "C"

namespace {

// Arguments of sdi_sample_points and sdi_sample_points_noalloc; on success the
// sector's record under the current parameters (own device copy) and the
// generating vector are filled in, and *grid is the sector's grid or NULL.
int sample_setup(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, int32_t shift, int64_t i0, int64_t npts,
                 const void* x_dev, SecDev& one, std::vector<uint64_t>& zp, const double** grid) {
  if (!ctx || !pb || (!x_dev && npts > 0)) return fail(ctx, SDI_EINVAL, "sample_points: null argument");
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  const Params& prm = ctx->params;
  if (shift < 0 || shift >= prm.R) return fail(ctx, SDI_EINVAL, "shift index out of range");
  if (npts < 0 || i0 < 0 || i0 + npts > ((int64_t)1 << prm.m)) return fail(ctx, SDI_EINVAL, "point range outside the lattice");
  const int rows = prm.R + prm.warmup;
  std::vector<SecDev> secs;
  size_t goff = 0;
  sector_fields(prm, pb, std::vector<int>(pb->nsec, prm.m), rows, secs, goff);
  const bool use_grid = pb->grid_valid && prm.warmup > 0 && pb->d_grids && pb->grid_nbins == prm.nbins &&
                        pb->grid_doubles >= goff;
  one = secs[s];
  if (!use_grid) one.flags &= ~F_USE_GRID;
  one.shift_row = 0;
  zp.assign(MAXV, 0);
  const std::vector<uint32_t>& z = lattice_vector16(prm.m);
  for (int j = 0; j < MAXV; ++j) zp[j] = (uint64_t)z[j] << (53 - prm.m);
  *grid = use_grid ? pb->d_grids + secs[s].grid_off : nullptr;
  return SDI_OK;
}

// Enqueues the shift row and the sampling kernel on device copies already
// holding the record (d_one) and generating vector (d_zp); d_row receives row
// `shift` (computed alone: the Philox counter carries the row index).
int sample_launch(sdi_ctx* ctx, SecDev* d_one, uint64_t* d_zp, uint64_t* d_row, const double* grid, int32_t shift,
                  int64_t i0, int64_t npts, void* x_dev, void* w_dev) {
  hipStream_t st = ctx->stream;
  int e = launch_shifts(d_one, 1, 1, 1, ctx->params.seed, (uint32_t)shift, d_row, st);
  if (e == 0) {
    SampleArgs A{};
    A.sec = d_one;
    A.zp = d_zp;
    A.shift = d_row;
    A.grid = grid;
    A.x = (double*)x_dev;
    A.w = (double*)w_dev;
    A.i0 = (uint64_t)i0;
    A.npts = npts;
    e = launch_sample_points(A, st);
  }
  return e;
}

}  // namespace

extern "C" {

int sdi_sample_points(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, int32_t shift, int64_t i0, int64_t npts,
                      void* x_dev, void* w_dev) {
  SecDev one{};
  std::vector<uint64_t> zp;
  const double* grid = nullptr;
  int rc = sample_setup(ctx, pb, s, shift, i0, npts, x_dev, one, zp, &grid);
  if (rc != SDI_OK) return rc;
  if (npts == 0) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  hipStream_t st = ctx->stream;
  SecDev* d_one = nullptr;
  uint64_t* d_sh = nullptr;
  uint64_t* d_zp = nullptr;
  hipError_t he = hipMalloc((void**)&d_one, sizeof(SecDev));
  if (he == hipSuccess) he = hipMalloc((void**)&d_sh, MAXV * 8);
  if (he == hipSuccess) he = hipMalloc((void**)&d_zp, MAXV * 8);
  int e = 0;
  if (he == hipSuccess) he = hipMemcpyAsync(d_one, &one, sizeof(SecDev), hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = hipMemcpyAsync(d_zp, zp.data(), MAXV * 8, hipMemcpyHostToDevice, st);
  if (he == hipSuccess) e = sample_launch(ctx, d_one, d_zp, d_sh, grid, shift, i0, npts, x_dev, w_dev);
  const hipError_t hs = hipStreamSynchronize(st);
  if (d_one) (void)hipFree(d_one);
  if (d_sh) (void)hipFree(d_sh);
  if (d_zp) (void)hipFree(d_zp);
  if (he != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("sample setup: ") + hipGetErrorString(he));
  if (e != 0) return fail(ctx, SDI_EDEVICE, std::string("sample kernel: ") + hipGetErrorString((hipError_t)e));
  if (hs != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("sample sync: ") + hipGetErrorString(hs));
  return SDI_OK;
}

int sdi_sample_points_noalloc(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, int32_t shift, int64_t i0,
                              int64_t npts, void* x_dev, void* w_dev) {
  SecDev one{};
  std::vector<uint64_t> zp;
  const double* grid = nullptr;
  int rc = sample_setup(ctx, pb, s, shift, i0, npts, x_dev, one, zp, &grid);
  if (rc != SDI_OK) return rc;
  // layout in this device's fixed scratch: record, generating vector, shift row
  constexpr size_t off_zp = (sizeof(SecDev) + 255) / 256 * 256;
  constexpr size_t off_row = off_zp + 256;
  constexpr size_t need = off_row + MAXV * 8;
  static_assert(need <= NOALLOC_SCRATCH_BYTES, "scratch too small for one sector record");
  if (!ctx->scratch) return fail(ctx, SDI_ESTATE, "sample_points_noalloc: no scratch address on this context");
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(ctx, SDI_ENOMEM, "sample_points_noalloc: needs " + std::to_string(need) + " bytes of the " +
                                     std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch");
  if (npts == 0) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  hipStream_t st = ctx->stream;
  unsigned char* base = (unsigned char*)ctx->scratch;
  SecDev* d_one = (SecDev*)base;
  uint64_t* d_zp = (uint64_t*)(base + off_zp);
  uint64_t* d_row = (uint64_t*)(base + off_row);
  HIPCHK(ctx, hipMemcpyAsync(d_one, &one, sizeof(SecDev), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_zp, zp.data(), MAXV * 8, hipMemcpyHostToDevice, st));
  KCHK(ctx, sample_launch(ctx, d_one, d_zp, d_row, grid, shift, i0, npts, x_dev, w_dev));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return SDI_OK;
}

namespace {
struct CheckpointHeader {
  char magic[8];
  int32_t nsec, R, m, baker, slice_log2, tile_log2, ppt, pad;
  uint64_t seed;
  double small_x;
  int64_t done, npairs;
};
constexpr char CKPT_MAGIC[8] = {'S', 'D', 'I', 'R', 'S', 'M', '0', '1'};
}  // namespace

int sdi_checkpoint_export(sdi_ctx* ctx, const sdi_problem* pb, void* buf, size_t len, size_t* needed) {
  if (!ctx || !pb || !needed) return fail(ctx, SDI_EINVAL, "checkpoint_export: null argument");
  if (pb->resume_key.empty() || pb->resume_done <= 0)
    return fail(ctx, SDI_ESTATE, "checkpoint_export: no resumable pass in progress on this problem");
  const size_t npairs = pb->resume_counts.size() / 2;
  const size_t bytes = sizeof(CheckpointHeader) + npairs * KMAX * 4 * 8 + npairs * 16;
  *needed = bytes;
  if (!buf) return SDI_OK;
  if (len < bytes) return fail(ctx, SDI_ENOMEM, "checkpoint_export: buffer needs " + std::to_string(bytes) + " bytes");
  // the settings are those of the key the sums were made under
  CheckpointHeader h{};
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  unsigned long long seed = 0;
  double sx = 0.0;
  if (sscanf(pb->resume_key.c_str(), "n%d m%d R%d s%llu b%d sl%d t%d p%d x%lg", &h.nsec, &h.m, &h.R, &seed, &h.baker,
             &h.slice_log2, &h.tile_log2, &h.ppt, &sx) != 9)
    return fail(ctx, SDI_ESTATE, "checkpoint_export: unreadable pass settings");
  h.seed = seed;
  h.small_x = sx;
  h.done = pb->resume_done;
  h.npairs = (int64_t)npairs;
  unsigned char* p = (unsigned char*)buf;
  std::memcpy(p, &h, sizeof h);
  std::memcpy(p + sizeof h, pb->resume_sums.data(), npairs * KMAX * 4 * 8);
  std::memcpy(p + sizeof h + npairs * KMAX * 4 * 8, pb->resume_counts.data(), npairs * 16);
  return SDI_OK;
}

int sdi_checkpoint_import(sdi_ctx* ctx, sdi_problem* pb, const void* buf, size_t len) {
  if (!ctx || !pb || !buf) return fail(ctx, SDI_EINVAL, "checkpoint_import: null argument");
  if (pb->ctx != ctx) return fail(ctx, SDI_EINVAL, "problem belongs to another context");
  CheckpointHeader h{};
  if (len < sizeof h) return fail(ctx, SDI_EINVAL, "checkpoint_import: too short");
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0) return fail(ctx, SDI_EINVAL, "checkpoint_import: not a checkpoint");
  if (h.npairs != (int64_t)pb->nsec * h.R || h.nsec != pb->nsec)
    return fail(ctx, SDI_EINVAL, "checkpoint_import: made for another problem (sector or shift count differs)");
  const size_t bytes = sizeof h + (size_t)h.npairs * KMAX * 4 * 8 + (size_t)h.npairs * 16;
  if (len != bytes) return fail(ctx, SDI_EINVAL, "checkpoint_import: size does not match its header");
  if (h.done <= 0 || h.m < 4 || h.m > 30 || h.done > ((int64_t)1 << h.m))
    return fail(ctx, SDI_EINVAL, "checkpoint_import: progress outside the lattice");
  Params q = ctx->params;
  q.m = h.m;
  q.R = h.R;
  q.seed = h.seed;
  q.baker = h.baker;
  q.slice_log2 = h.slice_log2;
  q.tile_log2 = h.tile_log2;
  q.ppt = h.ppt;
  q.small_x = h.small_x;
  const std::string key = resume_key(q, pb->nsec);
  if (key != resume_key(ctx->params, pb->nsec))
    return fail(ctx, SDI_EINVAL, "checkpoint_import: the context's parameters differ from the checkpoint's (" + key + ")");
  const unsigned char* p = (const unsigned char*)buf + sizeof h;
  pb->resume_sums.assign((size_t)h.npairs * KMAX * 4, 0.0);
  pb->resume_counts.assign((size_t)h.npairs * 2, 0);
  std::memcpy(pb->resume_sums.data(), p, pb->resume_sums.size() * 8);
  std::memcpy(pb->resume_counts.data(), p + pb->resume_sums.size() * 8, pb->resume_counts.size() * 8);
  pb->resume_done = h.done;
  pb->resume_key = key;
  return SDI_OK;
}

int sdi_tune_report(sdi_ctx* ctx, char* buf, size_t len, size_t* needed) {
  if (!ctx || !needed) return fail(ctx, SDI_EINVAL, "tune_report: null argument");
  *needed = ctx->tune_report.size() + 1;
  if (!buf) return SDI_OK;
  if (len < *needed) return fail(ctx, SDI_ENOMEM, "tune_report: buffer too small");
  std::memcpy(buf, ctx->tune_report.c_str(), *needed);
  return SDI_OK;
}

int sdi_vegas_refit(sdi_ctx* ctx, int32_t n, int32_t nbins, int32_t k, const void* hist_dev, void* grid_dev,
                    double alpha) {
  if (!ctx || !hist_dev || !grid_dev) return fail(ctx, SDI_EINVAL, "vegas_refit: null argument");
  if (n < 1 || n > MAXV) return fail(ctx, SDI_EINVAL, "vegas_refit: n must be 1..16");
  if (nbins < 2 || nbins > NBMAX || (nbins & (nbins - 1))) return fail(ctx, SDI_EINVAL, "vegas_refit: nbins must be a power of 2 in 2..256");
  if (k < 1 || k > KMAX) return fail(ctx, SDI_EINVAL, "vegas_refit: k must be 1..8");
  if (!(std::isfinite(alpha) && alpha >= 0.0)) return fail(ctx, SDI_EINVAL, "vegas_refit: alpha must be finite and >= 0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  // one sector record that carries the shapes; grid and histogram at offset 0
  SecDev one{};
  one.n = n;
  one.nbins = nbins;
  one.kf = k;
  one.grid_off = 0;
  const int64_t off0 = 0;
  hipStream_t st = ctx->stream;
  SecDev* d_one = nullptr;
  int64_t* d_off = nullptr;
  hipError_t he = hipMalloc((void**)&d_one, sizeof(SecDev));
  if (he == hipSuccess) he = hipMalloc((void**)&d_off, sizeof(int64_t));
  if (he == hipSuccess) he = hipMemcpyAsync(d_one, &one, sizeof(SecDev), hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = hipMemcpyAsync(d_off, &off0, sizeof(int64_t), hipMemcpyHostToDevice, st);
  int e = 0;
  if (he == hipSuccess) e = launch_refit(d_one, 1, (const double*)hist_dev, d_off, (double*)grid_dev, alpha, st);
  const hipError_t hs = hipStreamSynchronize(st);
  if (d_one) (void)hipFree(d_one);
  if (d_off) (void)hipFree(d_off);
  if (he != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("vegas_refit setup: ") + hipGetErrorString(he));
  if (e != 0) return fail(ctx, SDI_EDEVICE, std::string("vegas_refit kernel: ") + hipGetErrorString((hipError_t)e));
  if (hs != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("vegas_refit sync: ") + hipGetErrorString(hs));
  return SDI_OK;
}

// Autotuner cache as JSON: {"format": ..., "kernel_hash": ..., "entries":
// [{"key": ..., "tile_log2": t, "points_per_thread": p, "waves_per_simd": w}, ...]}.
int sdi_tune_save(sdi_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(ctx, SDI_EINVAL, "tune_save: null argument");
  FILE* f = fopen(path, "w");
  if (!f) return fail(ctx, SDI_EINVAL, std::string("tune_save: cannot open ") + path);
  fprintf(f, "{\n  \"format\": \"sdint-autotune-1\",\n  \"kernel_hash\": \"%s\",\n  \"entries\": [", SDI_KERNEL_HASH);
  for (size_t i = 0; i < ctx->tune_cache.size(); ++i) {
    const TuneEntry& e = ctx->tune_cache[i];
    fprintf(f,
            "%s\n    {\"key\": \"%s\", \"tile_log2\": %d, \"points_per_thread\": %d, \"waves_per_simd\": %d, "
            "\"corner_lists\": %d}",
            i ? "," : "", e.key.c_str(), e.tile_log2, (e.variant % CORNER_LISTS) / 10, e.variant % 10,
            e.variant >= CORNER_LISTS ? 1 : 0);
  }
  fprintf(f, "\n  ]\n}\n");
  const bool ok = !ferror(f);
  if (fclose(f) != 0 || !ok) return fail(ctx, SDI_EINVAL, std::string("tune_save: write failed on ") + path);
  return SDI_OK;
}

int sdi_tune_load(sdi_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(ctx, SDI_EINVAL, "tune_load: null argument");
  FILE* f = fopen(path, "r");
  if (!f) return fail(ctx, SDI_EINVAL, std::string("tune_load: cannot open ") + path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < ((size_t)16 << 20)) text.append(buf, got);
  fclose(f);
  const std::string bad = std::string("tune_load: malformed file ") + path;
  TuneReader r(text);
  std::string k, v, format, hash;
  std::vector<TuneEntry> entries;
  if (!r.lit('{')) return fail(ctx, SDI_EINVAL, bad);
  bool first = true;
  while (!r.lit('}')) {
    if (!first && !r.lit(',')) return fail(ctx, SDI_EINVAL, bad);
    first = false;
    if (!r.str(k) || !r.lit(':')) return fail(ctx, SDI_EINVAL, bad);
    if (k == "format" || k == "kernel_hash") {
      if (!r.str(v)) return fail(ctx, SDI_EINVAL, bad);
      (k == "format" ? format : hash) = v;
    } else if (k == "entries") {
      if (!r.lit('[')) return fail(ctx, SDI_EINVAL, bad);
      bool efirst = true;
      while (!r.lit(']')) {
        if (!efirst && !r.lit(',')) return fail(ctx, SDI_EINVAL, bad);
        efirst = false;
        if (!r.lit('{')) return fail(ctx, SDI_EINVAL, bad);
        TuneEntry e{"", -1, -1};
        int ppt = -1, wpe = -1, lists = 0;
        bool ffirst = true;
        while (!r.lit('}')) {
          if (!ffirst && !r.lit(',')) return fail(ctx, SDI_EINVAL, bad);
          ffirst = false;
          std::string fk;
          if (!r.str(fk) || !r.lit(':')) return fail(ctx, SDI_EINVAL, bad);
          bool ok;
          if (fk == "key") ok = r.str(e.key);
          else if (fk == "tile_log2") ok = r.num(e.tile_log2);
          else if (fk == "points_per_thread") ok = r.num(ppt);
          else if (fk == "waves_per_simd") ok = r.num(wpe);
          else if (fk == "corner_lists") ok = r.num(lists) && (lists == 0 || lists == 1);
          else ok = false;
          if (!ok) return fail(ctx, SDI_EINVAL, bad);
        }
        if (e.key.empty() || e.tile_log2 < 6 || e.tile_log2 > 24 || !(ppt == 1 || ppt == 2 || ppt == 4) ||
            wpe < 1 || wpe > 9)
          return fail(ctx, SDI_EINVAL, bad);
        e.variant = 10 * ppt + wpe + (lists ? CORNER_LISTS : 0);
        entries.push_back(e);
      }
    } else {
      return fail(ctx, SDI_EINVAL, bad);
    }
  }
  r.ws();
  if (r.p != text.size() || format != "sdint-autotune-1") return fail(ctx, SDI_EINVAL, bad);
  // entries of another kernel build are stale: load none of them
  if (hash != SDI_KERNEL_HASH) return 0;
  int n = 0;
  for (const TuneEntry& e : entries) {
    bool found = false;
    for (TuneEntry& c : ctx->tune_cache)
      if (c.key == e.key) {
        c = e;
        found = true;
      }
    if (!found) ctx->tune_cache.push_back(e);
    ++n;
  }
  return n;
}

}  // extern "C"
