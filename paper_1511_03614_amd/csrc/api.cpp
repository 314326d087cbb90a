// libsdint C ABI: context, parameters, problem compilation and the integration driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "host.h"
#include "kernels.h"

using namespace sdi;

namespace {

int fail(sdi_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, SDI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define KCHK(ctx, call)                                                                          \
  do {                                                                                           \
    int e_ = (call);                                                                             \
    if (e_ != 0)                                                                                 \
      return fail(ctx, SDI_EDEVICE,                                                              \
                  std::string(#call) + ": " + hipGetErrorString((hipError_t)e_));               \
  } while (0)

bool is_int(double v, double lim) { return std::isfinite(v) && v == std::floor(v) && std::fabs(v) <= lim; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace carving: a list of (pointer slot, bytes).
struct Carve {
  std::vector<std::pair<void**, size_t>> items;
  void add(void** p, size_t bytes) { items.push_back({p, align256(std::max<size_t>(bytes, 8))}); }
  size_t total() const {
    size_t t = 0;
    for (auto& i : items) t += i.second;
    return t;
  }
  void assign(void* base) {
    char* b = (char*)base;
    for (auto& i : items) {
      *i.first = b;
      b += i.second;
    }
  }
};

// Everything one integrate call needs that depends on the parameters.
struct Plan {
  int R = 0, rows = 0;
  std::vector<TileDesc> ftiles;       // final pass, canonical order
  std::vector<int32_t> forder;        // processing order
  std::vector<int32_t> pair_start, pair_sector;
  std::vector<TileDesc> wtiles;       // warm-up tiles of one iteration (shift row filled per iteration)
  std::vector<int32_t> worder;
  std::vector<int64_t> whist_off;
  std::vector<int32_t> wsec_start;
  std::vector<int64_t> hsec_off, hsec_prefix;
  int64_t whist_total = 0, hsec_total = 0;
  size_t shmem_final = 0, shmem_warm = 0;
  std::vector<uint64_t> zp_final, zp_warm;
  // device slots
  TileDesc* d_ftiles = nullptr;
  int32_t* d_forder = nullptr;
  int32_t* d_pair_start = nullptr;
  int32_t* d_pair_sector = nullptr;
  double* d_partial = nullptr;
  int32_t* d_nonfinite = nullptr;
  double* d_per_shift = nullptr;
  double* d_sec_stats = nullptr;
  double* d_res = nullptr;
  int64_t* d_counts = nullptr;
  int32_t* d_counter = nullptr;
  uint64_t* d_shifts = nullptr;
  uint64_t* d_zp_final = nullptr;
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
  int64_t* d_pair_nonfinite = nullptr;
  int64_t* d_sec_nonfinite = nullptr;
  Carve carve;
};

void lpt_order(const std::vector<TileDesc>& tiles, const std::vector<double>& cost, std::vector<int32_t>& order) {
  order.resize(tiles.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ca = cost[tiles[a].sector] * tiles[a].count;
    const double cb = cost[tiles[b].sector] * tiles[b].count;
    return ca > cb;
  });
}

int make_plan(sdi_ctx* ctx, sdi_problem* pb, Plan& P) {
  const Params& prm = ctx->params;
  P.R = prm.R;
  P.rows = prm.R + prm.warmup;
  const int nsec = pb->nsec;
  // per-sector parameter-dependent fields
  size_t goff = 0;
  for (int s = 0; s < nsec; ++s) {
    SecDev& S = pb->secs[s];
    S.m = prm.m;
    S.mw = prm.mw;
    S.nbins = prm.nbins;
    S.shift_row = s * P.rows;
    S.grid_off = (int32_t)goff;
    goff += (size_t)S.n * (prm.nbins + 1);
    S.flags &= ~(F_USE_GRID | F_BAKER);
    if (prm.baker) S.flags |= F_BAKER;
    if (prm.warmup > 0) S.flags |= F_USE_GRID;
  }
  // final tiles
  const uint32_t N = 1u << prm.m;
  const uint32_t tsz = std::min<uint32_t>(N, 1u << prm.tile_log2);
  P.pair_start.clear();
  P.pair_sector.clear();
  P.ftiles.clear();
  for (int s = 0; s < nsec; ++s)
    for (int r = 0; r < prm.R; ++r) {
      P.pair_start.push_back((int32_t)P.ftiles.size());
      P.pair_sector.push_back(s);
      for (uint32_t i0 = 0; i0 < N; i0 += tsz) P.ftiles.push_back(TileDesc{s, r, i0, tsz});
    }
  P.pair_start.push_back((int32_t)P.ftiles.size());
  lpt_order(P.ftiles, pb->cost, P.forder);
  // warm-up tiles (one iteration)
  P.wtiles.clear();
  P.whist_off.clear();
  P.wsec_start.clear();
  P.hsec_off.clear();
  P.hsec_prefix.clear();
  P.whist_total = P.hsec_total = 0;
  if (prm.warmup > 0) {
    const uint32_t Nw = 1u << prm.mw;
    const uint32_t wsz = std::min<uint32_t>(Nw, 1u << std::min(prm.tile_log2, 12));
    for (int s = 0; s < nsec; ++s) {
      const SecDev& S = pb->secs[s];
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
  // shared memory: grid plus (warm-up) histogram of the largest sector
  size_t gmax = 0, hmax = 0;
  for (int s = 0; s < nsec; ++s) {
    const SecDev& S = pb->secs[s];
    gmax = std::max(gmax, (size_t)S.n * (prm.nbins + 1));
    hmax = std::max(hmax, (size_t)S.n * prm.nbins * std::max(S.kf, 1));
  }
  P.shmem_final = prm.warmup > 0 ? gmax * 8 : 0;
  P.shmem_warm = (gmax + hmax) * 8;
  if (P.shmem_warm > 64 * 1024)
    return fail(ctx, SDI_ENOTSUP, "Vegas grid plus histogram exceed 64 KiB of LDS; lower nbins");
  // generating vectors
  const std::vector<uint32_t>& zf = lattice_vector16(prm.m);
  P.zp_final.assign((size_t)nsec * MAXV, 0);
  for (int s = 0; s < nsec; ++s)
    for (int j = 0; j < MAXV; ++j) P.zp_final[(size_t)s * MAXV + j] = (uint64_t)zf[j] << (53 - prm.m);
  if (prm.warmup > 0) {
    const std::vector<uint32_t>& zw = lattice_vector16(prm.mw);
    P.zp_warm.assign((size_t)nsec * MAXV, 0);
    for (int s = 0; s < nsec; ++s)
      for (int j = 0; j < MAXV; ++j) P.zp_warm[(size_t)s * MAXV + j] = (uint64_t)zw[j] << (53 - prm.mw);
  }
  // carve
  Carve& C = P.carve;
  C.items.clear();
  const size_t nft = P.ftiles.size(), npairs = P.pair_sector.size();
  C.add((void**)&P.d_ftiles, nft * sizeof(TileDesc));
  C.add((void**)&P.d_forder, nft * 4);
  C.add((void**)&P.d_pair_start, (npairs + 1) * 4);
  C.add((void**)&P.d_pair_sector, npairs * 4);
  C.add((void**)&P.d_partial, nft * KMAX * PART_STRIDE * 8);
  C.add((void**)&P.d_nonfinite, nft * 8);
  C.add((void**)&P.d_per_shift, npairs * KMAX * 2 * 8);
  C.add((void**)&P.d_sec_stats, (size_t)nsec * KMAX * 4 * 8);
  C.add((void**)&P.d_res, KMAX * 4 * 8);
  C.add((void**)&P.d_counts, 2 * 8);
  C.add((void**)&P.d_pair_nonfinite, npairs * 16);
  C.add((void**)&P.d_sec_nonfinite, (size_t)nsec * 16);
  C.add((void**)&P.d_counter, 8 * 4);
  C.add((void**)&P.d_shifts, (size_t)nsec * P.rows * MAXV * 8);
  C.add((void**)&P.d_zp_final, (size_t)nsec * MAXV * 8);
  if (prm.warmup > 0) {
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
  // persistent grids live with the problem
  if (pb->grid_doubles < goff || pb->grid_nbins != prm.nbins) {
    if (pb->d_grids) (void)hipFree(pb->d_grids);
    pb->d_grids = nullptr;
    pb->grid_doubles = 0;
    pb->grid_valid = false;
    if (goff) {
      HIPCHK(ctx, hipMalloc((void**)&pb->d_grids, goff * 8));
      pb->grid_doubles = goff;
    }
    pb->grid_nbins = prm.nbins;
  }
  return SDI_OK;
}

// Candidate points-per-thread values of the tile kernel for a variable class.
std::vector<int> ppt_candidates(const sdi_problem* pb) {
  if (pb->complex_mode) return pb->nvmax <= 4 ? std::vector<int>{1, 2} : std::vector<int>{1};
  if (pb->nvmax >= 16) return {1, 2};
  return {1, 2, 4};
}

// The tile-kernel family of a problem: real, or complex (contour deformation).
int launch_tiles(const sdi_problem* pb, int ppt, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
  if (pb->complex_mode) return launch_tiles_cplx(pb->nvmax, ppt, km, grid, shmem, a, pb->d_cx, pb->d_dir, st);
  return launch_tiles_real(pb->nvmax, ppt, km, grid, shmem, a, st);
}

int persistent_grid(sdi_ctx* ctx, const sdi_problem* pb, int ppt, int km, size_t shmem, size_t ntiles) {
  const int nvmax = pb->nvmax;
  int occ = pb->complex_mode ? tiles_cplx_occupancy(nvmax, ppt, km, shmem) : tiles_real_occupancy(nvmax, ppt, km, shmem);
  if (occ < 1) occ = 1;
  const size_t g = (size_t)occ * std::max(ctx->ncu, 1);
  return (int)std::max<size_t>(1, std::min(g, ntiles));
}

}  // namespace

// ============================================================================ C ABI

extern "C" {

int sdi_ctx_create(int device_ordinal, void* hip_stream, sdi_ctx** out) {
  if (!out) return SDI_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return SDI_EDEVICE;
  if (device_ordinal < 0 || device_ordinal >= ndev) return SDI_EINVAL;
  sdi_ctx* c = new sdi_ctx();
  c->device = device_ordinal;
  if (hipSetDevice(device_ordinal) != hipSuccess || hipGetDeviceProperties(&c->prop, device_ordinal) != hipSuccess) {
    delete c;
    return SDI_EDEVICE;
  }
  c->ncu = c->prop.multiProcessorCount;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    // A blocking stream: ordered with the legacy default stream that torch uses by default.
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return SDI_EDEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return SDI_OK;
}

void sdi_ctx_destroy(sdi_ctx* ctx) {
  if (!ctx) return;
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* sdi_last_error(const sdi_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sdi_device_info(sdi_ctx* ctx, char* buf, size_t len) {
  if (!ctx || !buf || len == 0) return fail(ctx, SDI_EINVAL, "device_info: null argument");
  const hipDeviceProp_t& p = ctx->prop;
  snprintf(buf, len, "device=%d name=%s arch=%s cus=%d lds_per_block=%zu clock_khz=%d mem_bytes=%zu wavefront=%d",
           ctx->device, p.name, p.gcnArchName, p.multiProcessorCount, (size_t)p.sharedMemPerBlock, p.clockRate,
           (size_t)p.totalGlobalMem, p.warpSize);
  return SDI_OK;
}

int sdi_set_param(sdi_ctx* ctx, const char* key, const char* value) {
  if (!ctx || !key || !value) return fail(ctx, SDI_EINVAL, "set_param: null argument");
  const std::string k(key), v(value);
  Params& p = ctx->params;
  if (k == "tune") {
    if (v == "off") p.tune = 0;
    else if (v == "cached") p.tune = 1;
    else if (v == "search") p.tune = 2;
    else return fail(ctx, SDI_EINVAL, "tune must be off, cached or search");
    return SDI_OK;
  }
  char* end = nullptr;
  errno = 0;
  const long long iv = strtoll(value, &end, 10);
  if (errno || !end || *end != '\0' || end == value) return fail(ctx, SDI_EINVAL, "value of " + k + " must be an integer");
  auto range = [&](long long lo, long long hi) { return iv >= lo && iv <= hi; };
  if (k == "lattice_log2") {
    if (!range(4, 30)) return fail(ctx, SDI_EINVAL, "lattice_log2 must be in 4..30");
    p.m = (int)iv;
  } else if (k == "shifts") {
    if (!range(2, 256)) return fail(ctx, SDI_EINVAL, "shifts must be in 2..256");
    p.R = (int)iv;
  } else if (k == "seed") {
    p.seed = (uint64_t)iv;
  } else if (k == "baker") {
    if (!range(0, 1)) return fail(ctx, SDI_EINVAL, "baker must be 0 or 1");
    p.baker = (int)iv;
  } else if (k == "warmup") {
    if (!range(0, 64)) return fail(ctx, SDI_EINVAL, "warmup must be in 0..64");
    p.warmup = (int)iv;
  } else if (k == "warmup_log2") {
    if (!range(4, 24)) return fail(ctx, SDI_EINVAL, "warmup_log2 must be in 4..24");
    p.mw = (int)iv;
  } else if (k == "nbins") {
    if (!range(2, NBMAX) || (iv & (iv - 1))) return fail(ctx, SDI_EINVAL, "nbins must be a power of 2 in 2..256");
    p.nbins = (int)iv;
  } else if (k == "tile_log2") {
    if (!range(6, 24)) return fail(ctx, SDI_EINVAL, "tile_log2 must be in 6..24");
    p.tile_log2 = (int)iv;
  } else if (k == "ppt") {
    if (!(iv == 0 || iv == 1 || iv == 2 || iv == 4)) return fail(ctx, SDI_EINVAL, "ppt must be 0, 1, 2 or 4");
    p.ppt = (int)iv;
  } else if (k == "graph") {
    if (!range(0, 1)) return fail(ctx, SDI_EINVAL, "graph must be 0 or 1");
    p.graph = (int)iv;
  } else {
    return fail(ctx, SDI_EINVAL, "unknown parameter " + k);
  }
  return SDI_OK;
}

int sdi_get_param(sdi_ctx* ctx, const char* key, char* buf, size_t len) {
  if (!ctx || !key || !buf || len == 0) return fail(ctx, SDI_EINVAL, "get_param: null argument");
  const std::string k(key);
  const Params& p = ctx->params;
  long long v;
  if (k == "tune") {
    snprintf(buf, len, "%s", p.tune == 0 ? "off" : (p.tune == 1 ? "cached" : "search"));
    return SDI_OK;
  } else if (k == "lattice_log2") v = p.m;
  else if (k == "shifts") v = p.R;
  else if (k == "seed") v = (long long)p.seed;
  else if (k == "baker") v = p.baker;
  else if (k == "warmup") v = p.warmup;
  else if (k == "warmup_log2") v = p.mw;
  else if (k == "nbins") v = p.nbins;
  else if (k == "tile_log2") v = p.tile_log2;
  else if (k == "ppt") v = p.ppt;
  else if (k == "graph") v = p.graph;
  else return fail(ctx, SDI_EINVAL, "unknown parameter " + k);
  snprintf(buf, len, "%lld", v);
  return SDI_OK;
}

int sdi_prefactor_feynman(int32_t loops, const int32_t* indices, int32_t nprops, int32_t d0, int32_t len,
                          int32_t* lead, double* out) {
  std::string err;
  int ld = 0;
  std::vector<double> tmp(len > 0 ? len : 1);
  const int rc = prefactor_series(loops, indices, nprops, d0, len, &ld, tmp.data(), err);
  if (rc != SDI_OK) return rc;
  *lead = ld;
  std::copy(tmp.begin(), tmp.begin() + len, out);
  return SDI_OK;
}

int sdi_lattice_vector(int32_t m, int32_t dims, uint32_t* out) {
  if (m < 4 || m > 30 || dims < 1 || dims > MAXV || !out) return SDI_EINVAL;
  const std::vector<uint32_t>& z = lattice_vector16(m);
  std::copy(z.begin(), z.begin() + dims, out);
  return SDI_OK;
}

int sdi_problem_create(sdi_ctx* ctx, const sdi_problem_desc* d, sdi_problem** out) {
  if (!ctx || !d || !out) return fail(ctx, SDI_EINVAL, "problem_create: null argument");
  *out = nullptr;
  if (d->nsectors < 1 || !d->sectors) return fail(ctx, SDI_EINVAL, "need at least one sector");
  const int K = d->order_max - d->order_min + 1;
  if (K < 1 || K > KMAX) return fail(ctx, SDI_EINVAL, "need 1..8 requested orders");
  if (d->pref_len < 1 || d->pref_len > 64 || !d->pref_re) return fail(ctx, SDI_EINVAL, "prefactor series missing");
  if (d->complex_mode && !(std::isfinite(d->lambda) && d->lambda >= 0.0))
    return fail(ctx, SDI_EINVAL, "lambda must be finite and non-negative");
  sdi_problem* pb = new sdi_problem();
  pb->ctx = ctx;
  pb->nsec = d->nsectors;
  pb->K = K;
  pb->order_min = d->order_min;
  pb->complex_mode = d->complex_mode;
  pb->lambda = d->lambda;
  auto bad = [&](int code, const std::string& m) {
    delete pb;
    return fail(ctx, code, m);
  };
  const int kf_max = d->order_max - d->pref_lead;
  for (int s = 0; s < d->nsectors; ++s) {
    const sdi_sector_desc& sd = d->sectors[s];
    const std::string where = "sector " + std::to_string(s) + ": ";
    const int n = sd.nvars;
    if (n < 1 || n > MAXV) return bad(SDI_EINVAL, where + "nvars must be 1..16");
    if (sd.nfactors < 0 || sd.nfactors > MAXF) return bad(SDI_EINVAL, where + "nfactors must be 0..4");
    if (sd.reserved != 0) return bad(SDI_EINVAL, where + "reserved must be 0");
    if (sd.deform_factor < -1 || sd.deform_factor >= sd.nfactors) return bad(SDI_EINVAL, where + "bad deform_factor");
    if (!sd.mono_a || !sd.mono_b || (sd.nfactors && (!sd.fac_nterms || !sd.fac_gamma || !sd.fac_delta)))
      return bad(SDI_EINVAL, where + "null array");
    if (!std::isfinite(sd.coeff_re) || !std::isfinite(sd.coeff_im)) return bad(SDI_EINVAL, where + "coefficient not finite");
    std::vector<int> S, rest;
    for (int j = 0; j < n; ++j) {
      const double a = sd.mono_a[j], b = sd.mono_b[j];
      if (!std::isfinite(a) || !std::isfinite(b)) return bad(SDI_EINVAL, where + "exponent not finite");
      if (a == -1.0) {
        if (b == 0.0) return bad(SDI_EINVAL, where + "a_j = -1 needs b_j != 0");
        S.push_back(j);
      } else if (a > -1.0) {
        rest.push_back(j);
      } else {
        return bad(SDI_EINVAL, where + "a_j < -1 needs higher-order subtraction");
      }
    }
    if ((int)S.size() > MAXS) return bad(SDI_ENOTSUP, where + "more than 4 singular variables");
    if (d->complex_mode && n > 8) return bad(SDI_ENOTSUP, where + "complex mode supports up to 8 variables");
    SecDev R{};
    R.n = n;
    R.ns = (int)S.size();
    R.nfac = sd.nfactors;
    R.kf = std::max(0, kf_max + R.ns + 1);
    if (R.kf > KMAX) return bad(SDI_ENOTSUP, where + "more than 8 internal eps orders");
    R.K = K;
    R.nvc = n <= 4 ? 0 : (n <= 8 ? 1 : 2);
    R.cls = R.nvc;   // complex mode: 0 (n <= 4) or 1 (n <= 8)
    R.sector = s;
    std::vector<int> perm(S);
    perm.insert(perm.end(), rest.begin(), rest.end());
    for (int j = 0; j < n; ++j) R.perm[j] = perm[j];
    bool int_mono = true;
    for (int j = 0; j < n; ++j) {
      const double a = sd.mono_a[perm[j]], b = sd.mono_b[perm[j]];
      R.a[j] = a;
      R.b[j] = b;
      if (j >= R.ns) {
        if (is_int(a, 64) && a >= 0 && is_int(b, 8)) {
          R.a_int[j] = (int)a;
          R.b_int[j] = (int)b;
        } else {
          int_mono = false;
        }
      }
    }
    for (int i = 0; i < R.ns; ++i) R.bS[i] = sd.mono_b[S[i]];
    for (int T = 0; T < (1 << R.ns); ++T) {
      double v = 1.0;
      for (int i = 0; i < R.ns; ++i)
        if (T >> i & 1) v = v / R.bS[i];
      R.invb[T] = v;
    }
    bool int_pow = true;
    for (int m = 0; m < sd.nfactors; ++m) {
      const double g = sd.fac_gamma[m], dl = sd.fac_delta[m];
      if (!std::isfinite(g) || !std::isfinite(dl)) return bad(SDI_EINVAL, where + "gamma/delta not finite");
      R.gam[m] = g;
      R.del[m] = dl;
      if (is_int(g, 64) && is_int(dl, 64)) {
        R.gam_int[m] = (int)g;
        R.del_int[m] = (int)dl;
      } else {
        int_pow = false;
      }
    }
    R.flags = (int_pow ? F_INT_POW : 0) | (int_mono ? F_INT_MONO : 0);
    // terms per (factor, corner)
    size_t t0 = 0;
    for (int m = 0; m < sd.nfactors; ++m) {
      const int nt = sd.fac_nterms[m];
      if (nt < 0) return bad(SDI_EINVAL, where + "negative term count");
      if (nt > 0 && (!sd.term_coef || !sd.term_exps)) return bad(SDI_EINVAL, where + "null term arrays");
      for (int t = 0; t < nt; ++t) {
        if (!std::isfinite(sd.term_coef[t0 + t])) return bad(SDI_EINVAL, where + "term coefficient not finite");
        for (int j = 0; j < n; ++j)
          if (sd.term_exps[(t0 + t) * n + j] > 3)
            return bad(SDI_ENOTSUP, where + "polynomial exponents above 3 are not supported");
      }
      for (int W = 0; W < (1 << R.ns); ++W) {
        R.tab_off[m][W] = (uint32_t)pb->terms.size();
        uint32_t cnt = 0;
        for (int t = 0; t < nt; ++t) {
          const uint8_t* e = sd.term_exps + (t0 + t) * n;
          bool alive = true;
          for (int i = 0; i < R.ns; ++i)
            if ((W >> i & 1) && e[S[i]] != 0) alive = false;
          if (!alive) continue;
          uint64_t word = 0;
          for (int j = 0; j < n; ++j) word |= (uint64_t)e[perm[j]] << (4 * j);
          pb->terms.push_back(Term{sd.term_coef[t0 + t], word});
          ++cnt;
        }
        R.tab_cnt[m][W] = cnt;
      }
      t0 += nt;
    }
    if (d->complex_mode) {
      // derivative lists of the full F = x^mono * P_F (internal variable order), per corner
      CplxDev X{};
      X.lam = d->lambda;
      X.fac_f = sd.deform_factor;
      for (int j = 0; j < n; ++j) X.mono_f[j] = sd.deform_mono ? sd.deform_mono[perm[j]] : 0;
      for (int j = 0; j < n; ++j)
        if (X.mono_f[j] < 0 || X.mono_f[j] > 7) return bad(SDI_ENOTSUP, where + "deform_mono outside 0..7");
      X.nd = n + n * (n + 1) / 2;
      X.dir_off = (int32_t)pb->dir.size();
      pb->dir.resize(pb->dir.size() + (size_t)X.nd * MAXC * 2, 0);
      if (sd.deform_factor >= 0) {
        // full-F terms: coefficient and integer exponents
        size_t tf = 0;
        for (int m = 0; m < sd.deform_factor; ++m) tf += sd.fac_nterms[m];
        const int ntf = sd.fac_nterms[sd.deform_factor];
        std::vector<std::pair<double, std::vector<int>>> F;
        for (int t = 0; t < ntf; ++t) {
          std::vector<int> e(n);
          for (int j = 0; j < n; ++j) e[j] = sd.term_exps[(tf + t) * n + perm[j]] + X.mono_f[j];
          F.push_back({sd.term_coef[tf + t], e});
        }
        auto deriv = [&](const std::vector<std::pair<double, std::vector<int>>>& P, int j) {
          std::vector<std::pair<double, std::vector<int>>> D;
          for (auto& t : P)
            if (t.second[j] > 0) {
              auto e = t.second;
              const double c = t.first * e[j];
              e[j] -= 1;
              D.push_back({c, e});
            }
          return D;
        };
        auto emit = [&](int dd, const std::vector<std::pair<double, std::vector<int>>>& P) -> bool {
          for (int W = 0; W < (1 << R.ns); ++W) {
            const uint32_t off = (uint32_t)pb->terms.size();
            uint32_t cnt = 0;
            for (auto& t : P) {
              bool alive = true;
              for (int i = 0; i < R.ns; ++i)
                if ((W >> i & 1) && t.second[i] != 0) alive = false;
              if (!alive) continue;
              uint64_t word = 0;
              for (int j = 0; j < n; ++j) {
                if (t.second[j] > 7) return false;
                word |= (uint64_t)t.second[j] << (4 * j);
              }
              pb->terms.push_back(Term{t.first, word});
              ++cnt;
            }
            pb->dir[(size_t)X.dir_off + ((size_t)dd * MAXC + W) * 2] = off;
            pb->dir[(size_t)X.dir_off + ((size_t)dd * MAXC + W) * 2 + 1] = cnt;
          }
          return true;
        };
        for (int j = 0; j < n; ++j)
          if (!emit(j, deriv(F, j))) return bad(SDI_ENOTSUP, where + "full-F exponents above 7");
        for (int j = 0; j < n; ++j) {
          const auto Dj = deriv(F, j);
          for (int k = 0; k <= j; ++k)
            if (!emit(n + j * (j + 1) / 2 + k, deriv(Dj, k)))
              return bad(SDI_ENOTSUP, where + "full-F exponents above 7");
        }
      }
      pb->cx.push_back(X);
    }
    // fold: F_k = sum_kk c_s Pi_i f_kk, i = k - lead - (kk - ns)
    bool has_im = false;
    for (int k = 0; k < K; ++k)
      for (int kk = 0; kk < KMAX; ++kk) {
        const int i = (d->order_min + k) - d->pref_lead - (kk - R.ns);
        double fr = 0.0, fi = 0.0;
        if (kk < R.kf && i >= 0 && i < d->pref_len) {
          const double pr = d->pref_re[i], pi = d->pref_im ? d->pref_im[i] : 0.0;
          fr = sd.coeff_re * pr - sd.coeff_im * pi;
          fi = sd.coeff_re * pi + sd.coeff_im * pr;
        }
        R.fold_re[k][kk] = fr;
        R.fold_im[k][kk] = fi;
        if (fi != 0.0) has_im = true;
      }
    if (has_im) R.flags |= F_HAS_IM;
    // cost estimate per point: polynomial work over corners plus series and logs
    double c = 40.0 * (n + 1);
    for (int W = 0; W < (1 << R.ns); ++W) {
      for (int m = 0; m < sd.nfactors; ++m) c += 6.0 * R.tab_cnt[m][W];
      c += 80.0 + 3.0 * R.kf * (1 << R.ns);
    }
    pb->cost.push_back(c);
    pb->secs.push_back(R);
    pb->nvmax = std::max(pb->nvmax, n <= 4 ? 4 : (n <= 8 ? 8 : 16));
    if (d->complex_mode) c *= 8.0 + 2.0 * n * n;
    pb->kfmax = std::max(pb->kfmax, R.kf);
  }
  if (pb->terms.empty()) pb->terms.push_back(Term{0.0, 0});
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_secs, pb->secs.size() * sizeof(SecDev));
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_terms, pb->terms.size() * sizeof(Term));
  if (e == hipSuccess)
    e = hipMemcpy(pb->d_terms, pb->terms.data(), pb->terms.size() * sizeof(Term), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pb->d_secs, pb->secs.data(), pb->secs.size() * sizeof(SecDev), hipMemcpyHostToDevice);
  if (e == hipSuccess && pb->complex_mode) {
    if (pb->dir.empty()) pb->dir.push_back(0);
    e = hipMalloc((void**)&pb->d_cx, pb->cx.size() * sizeof(CplxDev));
    if (e == hipSuccess) e = hipMalloc((void**)&pb->d_dir, pb->dir.size() * sizeof(uint32_t));
    if (e == hipSuccess)
      e = hipMemcpy(pb->d_cx, pb->cx.data(), pb->cx.size() * sizeof(CplxDev), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(pb->d_dir, pb->dir.data(), pb->dir.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    sdi_problem_destroy(pb);
    return fail(ctx, SDI_EDEVICE, std::string("problem upload: ") + hipGetErrorString(e));
  }
  *out = pb;
  return SDI_OK;
}

void sdi_problem_destroy(sdi_problem* pb) {
  if (!pb) return;
  delete pb->pass;
  if (pb->d_secs) (void)hipFree(pb->d_secs);
  if (pb->d_terms) (void)hipFree(pb->d_terms);
  if (pb->d_grids) (void)hipFree(pb->d_grids);
  if (pb->d_ws) (void)hipFree(pb->d_ws);
  if (pb->d_cx) (void)hipFree(pb->d_cx);
  if (pb->d_dir) (void)hipFree(pb->d_dir);
  delete pb;
}

int sdi_problem_norders(const sdi_problem* pb) { return pb ? pb->K : SDI_EINVAL; }

size_t sdi_workspace_bytes(sdi_ctx* ctx, const sdi_problem* prob) {
  if (!ctx || !prob) return 0;
  Plan P;
  sdi_problem tmp = *prob;        // make_plan edits per-sector fields; work on a copy
  tmp.d_grids = nullptr;
  tmp.grid_doubles = (size_t)-1;  // do not (re)allocate grids here
  tmp.grid_nbins = ctx->params.nbins;
  tmp.pass = nullptr;
  const int rc = make_plan(ctx, &tmp, P);
  return rc == SDI_OK ? P.carve.total() : 0;
}

}  // extern "C"

namespace sdi {

struct PassState {
  std::string key;
  Plan P;
  int ppt = 1, km = 4, gf = 1, gw = 1;
  hipGraphExec_t exec = nullptr;
  bool graph_failed = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  ~PassState() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

}  // namespace sdi

namespace {

std::string pass_key(const Params& p, const void* ws, size_t wsb) {
  char buf[256];
  snprintf(buf, sizeof buf, "m%d R%d s%llu b%d w%d mw%d nb%d t%d p%d g%d ws%p:%zu", p.m, p.R,
           (unsigned long long)p.seed, p.baker, p.warmup, p.mw, p.nbins, p.tile_log2, p.ppt, p.graph, ws, wsb);
  return buf;
}

// Enqueue one full pass (shifts, warm-up iterations, final pass, reductions) on st.
int record_pass(sdi_ctx* ctx, sdi_problem* pb, PassState& S, hipStream_t st) {
  const Params& prm = ctx->params;
  Plan& P = S.P;
  const int nsec = pb->nsec;
  const int npairs = (int)P.pair_sector.size();
  const int nft = (int)P.ftiles.size();
  HIPCHK(ctx, hipEventRecord(S.ev[0], st));
  KCHK(ctx, launch_shifts(pb->d_secs, nsec, P.rows, prm.R, prm.seed, P.d_shifts, st));
  TileArgs A{};
  A.secs = pb->d_secs;
  A.terms = pb->d_terms;
  A.shifts = P.d_shifts;
  A.grids = pb->d_grids;
  if (prm.warmup > 0) {
    KCHK(ctx, launch_grid_identity(pb->d_secs, nsec, pb->d_grids, st));
    const int nwt = (int)P.wtiles.size();
    for (int it = 0; it < prm.warmup; ++it) {
      KCHK(ctx, launch_fill_i32(P.d_counter, 0, 1, st));
      TileArgs W = A;
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
      KCHK(ctx, launch_tiles(pb, S.ppt, S.km, S.gw, P.shmem_warm, W, st));
      KCHK(ctx, launch_hist_reduce(P.d_whist, P.d_whist_off, P.d_wsec_start, pb->d_secs, P.d_hsec_off, nsec,
                                   P.hsec_total, P.d_hsec_prefix, P.d_hsec, st));
      KCHK(ctx, launch_refit(pb->d_secs, nsec, P.d_hsec, P.d_hsec_off, pb->d_grids, 1.5, st));
    }
  }
  HIPCHK(ctx, hipEventRecord(S.ev[1], st));
  KCHK(ctx, launch_fill_i32(P.d_counter + 1, 0, 1, st));
  TileArgs F = A;
  F.zp = P.d_zp_final;
  F.tiles = P.d_ftiles;
  F.order = P.d_forder;
  F.partial = P.d_partial;
  F.nonfinite = P.d_nonfinite;
  F.counter = P.d_counter + 1;
  F.ntiles = nft;
  F.mode = 0;
  HIPCHK(ctx, hipEventRecord(S.ev[2], st));
  KCHK(ctx, launch_tiles(pb, S.ppt, S.km, S.gf, P.shmem_final, F, st));
  HIPCHK(ctx, hipEventRecord(S.ev[3], st));
  KCHK(ctx, launch_reduce_pairs(P.d_partial, P.d_pair_start, P.d_pair_sector, pb->d_secs, npairs, P.d_per_shift,
                                P.d_nonfinite, P.d_pair_nonfinite, st));
  KCHK(ctx, launch_sector_stats(P.d_per_shift, nsec, prm.R, P.d_sec_stats, P.d_pair_nonfinite, P.d_sec_nonfinite, st));
  KCHK(ctx, launch_combine(P.d_sec_stats, nsec, P.d_sec_nonfinite, P.d_res, P.d_counts, st));
  HIPCHK(ctx, hipEventRecord(S.ev[4], st));
  return SDI_OK;
}

// Times the final-pass tile kernel for each points-per-thread candidate on the
// problem's own tiles and keeps the fastest (cached per device, class and problem shape).
int autotune_ppt(sdi_ctx* ctx, sdi_problem* pb, PassState& S, hipStream_t st) {
  const Params& prm = ctx->params;
  char keyb[256];
  snprintf(keyb, sizeof keyb, "%s|c%d|nv%d|km%d|sec%d|terms%zu|m%d|t%d|grid%d", ctx->prop.gcnArchName,
           pb->complex_mode, pb->nvmax, S.km, pb->nsec, pb->terms.size(), prm.m, prm.tile_log2, prm.warmup > 0);
  const std::string key(keyb);
  if (prm.tune == 1)
    for (auto& kv : ctx->tune_cache)
      if (kv.first == key) return kv.second;
  Plan& P = S.P;
  KCHK(ctx, launch_shifts(pb->d_secs, pb->nsec, P.rows, prm.R, prm.seed, P.d_shifts, st));
  if (prm.warmup > 0) KCHK(ctx, launch_grid_identity(pb->d_secs, pb->nsec, pb->d_grids, st));
  TileArgs F{};
  F.secs = pb->d_secs;
  F.terms = pb->d_terms;
  F.shifts = P.d_shifts;
  F.grids = pb->d_grids;
  F.zp = P.d_zp_final;
  F.tiles = P.d_ftiles;
  F.order = P.d_forder;
  F.partial = P.d_partial;
  F.nonfinite = P.d_nonfinite;
  F.counter = P.d_counter + 1;
  F.ntiles = (int)P.ftiles.size();
  F.mode = 0;
  int best = 1;
  float best_ms = 1e30f;
  for (int ppt : ppt_candidates(pb)) {
    const int g = persistent_grid(ctx, pb, ppt, S.km, P.shmem_final, P.ftiles.size());
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      KCHK(ctx, launch_fill_i32(F.counter, 0, 1, st));
      HIPCHK(ctx, hipEventRecord(S.ev[2], st));
      KCHK(ctx, launch_tiles(pb, ppt, S.km, g, P.shmem_final, F, st));
      HIPCHK(ctx, hipEventRecord(S.ev[3], st));
      HIPCHK(ctx, hipEventSynchronize(S.ev[3]));
      HIPCHK(ctx, hipEventElapsedTime(&ms, S.ev[2], S.ev[3]));
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = ppt;
    }
  }
  ctx->tune_cache.push_back({key, best});
  return best;
}

// (Re)build the cached pass state when parameters or workspace change.
int prepare_pass(sdi_ctx* ctx, sdi_problem* pb, void* dev_ws, size_t ws_bytes) {
  const Params& prm = ctx->params;
  const std::string key = pass_key(prm, dev_ws, ws_bytes);
  if (pb->pass && pb->pass->key == key) return SDI_OK;
  delete pb->pass;
  pb->pass = nullptr;
  PassState* S = new PassState();
  int rc = make_plan(ctx, pb, S->P);
  if (rc != SDI_OK) {
    delete S;
    return rc;
  }
  Plan& P = S->P;
  const size_t need = P.carve.total();
  void* base = dev_ws;
  if (base) {
    if (ws_bytes < need) {
      delete S;
      return fail(ctx, SDI_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    }
  } else {
    if (pb->ws_size < need) {
      if (pb->d_ws) (void)hipFree(pb->d_ws);
      pb->d_ws = nullptr;
      pb->ws_size = 0;
      if (hipMalloc(&pb->d_ws, need) != hipSuccess) {
        delete S;
        return fail(ctx, SDI_ENOMEM, "workspace allocation failed");
      }
      pb->ws_size = need;
    }
    base = pb->d_ws;
  }
  P.carve.assign(base);
  pb->pass = S;
  for (auto& e : S->ev) HIPCHK(ctx, hipEventCreate(&e));
  hipStream_t st = ctx->stream;
  const int nsec = pb->nsec;
  const int npairs = (int)P.pair_sector.size();
  const int nft = (int)P.ftiles.size();
  HIPCHK(ctx, hipMemcpyAsync(pb->d_secs, pb->secs.data(), pb->secs.size() * sizeof(SecDev), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_ftiles, P.ftiles.data(), nft * sizeof(TileDesc), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_forder, P.forder.data(), nft * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_pair_start, P.pair_start.data(), (npairs + 1) * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_pair_sector, P.pair_sector.data(), npairs * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(P.d_zp_final, P.zp_final.data(), P.zp_final.size() * 8, hipMemcpyHostToDevice, st));
  std::vector<TileDesc> wall;
  if (prm.warmup > 0) {
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
  S->km = pb->kfmax <= 4 ? 4 : 8;
  if (prm.ppt > 0) S->ppt = prm.ppt;
  else if (prm.tune == 0) S->ppt = (pb->nvmax >= 16 || pb->complex_mode) ? 1 : 2;
  else {
    rc = autotune_ppt(ctx, pb, *S, st);
    if (rc < 0) return rc;
    S->ppt = rc;
  }
  S->gf = persistent_grid(ctx, pb, S->ppt, S->km, P.shmem_final, P.ftiles.size());
  S->gw = prm.warmup > 0 ? persistent_grid(ctx, pb, S->ppt, S->km, P.shmem_warm, P.wtiles.size()) : 1;
  if (prm.graph) {
    // Capture the whole pass once; replays skip the launch overheads.  Any
    // failure falls back to eager launches on this key.
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const int rr = record_pass(ctx, pb, *S, st);
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (rr == SDI_OK && ec == hipSuccess && g && hipGraphInstantiate(&S->exec, g, nullptr, nullptr, 0) == hipSuccess) {
        // instantiated
      } else {
        S->exec = nullptr;
        S->graph_failed = true;
      }
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
    } else {
      S->graph_failed = true;
    }
  }
  S->key = key;
  return SDI_OK;
}

}  // namespace

extern "C" {

int sdi_integrate(sdi_ctx* ctx, sdi_problem* pb, void* dev_ws, size_t ws_bytes, sdi_result* out) {
  if (!ctx || !pb || !out) return fail(ctx, SDI_EINVAL, "integrate: null argument");
  if (pb->ctx != ctx) return fail(ctx, SDI_EINVAL, "problem belongs to another context");
  if (!out->val_re || !out->val_im || !out->err_re || !out->err_im)
    return fail(ctx, SDI_EINVAL, "integrate: result arrays must be allocated");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const Params& prm = ctx->params;
  int rc = prepare_pass(ctx, pb, dev_ws, ws_bytes);
  if (rc != SDI_OK) return rc;
  PassState& S = *pb->pass;
  Plan& P = S.P;
  hipStream_t st = ctx->stream;
  const int nsec = pb->nsec;
  const int npairs = (int)P.pair_sector.size();
  if (S.exec) {
    HIPCHK(ctx, hipGraphLaunch(S.exec, st));
  } else {
    rc = record_pass(ctx, pb, S, st);
    if (rc != SDI_OK) return rc;
  }
  std::vector<double> res(KMAX * 4);
  int64_t counts[2] = {0, 0};
  pb->sec_stats.assign((size_t)nsec * KMAX * 4, 0.0);
  pb->per_shift.assign((size_t)npairs * KMAX * 2, 0.0);
  HIPCHK(ctx, hipMemcpyAsync(res.data(), P.d_res, res.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(counts, P.d_counts, 16, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(pb->sec_stats.data(), P.d_sec_stats, pb->sec_stats.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(pb->per_shift.data(), P.d_per_shift, pb->per_shift.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  float ms_w = 0.f, ms_f = 0.f, ms_k = 0.f;
  (void)hipEventElapsedTime(&ms_w, S.ev[0], S.ev[1]);
  (void)hipEventElapsedTime(&ms_f, S.ev[1], S.ev[4]);
  (void)hipEventElapsedTime(&ms_k, S.ev[2], S.ev[3]);
  pb->grid_valid = prm.warmup > 0;
  pb->last_R = prm.R;
  pb->have_results = true;
  const int64_t per_sec = (int64_t)prm.R << prm.m;
  pb->sec_evals.assign(nsec, per_sec);
  out->order_min = pb->order_min;
  out->norders = pb->K;
  for (int k = 0; k < pb->K; ++k) {
    out->val_re[k] = res[k * 4 + 0];
    out->val_im[k] = res[k * 4 + 1];
    out->err_re[k] = res[k * 4 + 2];
    out->err_im[k] = res[k * 4 + 3];
  }
  out->n_evals = per_sec * nsec + (int64_t)prm.warmup * nsec * ((int64_t)1 << prm.mw);
  out->n_nonfinite = counts[0];
  out->n_imf_positive = counts[1];
  out->ms_sample_eval_reduce = ms_f;
  out->ms_refit = ms_w;
  out->ms_total = ms_w + ms_f;
  out->ms_eval_kernel = ms_k;
  out->points_per_thread = S.ppt;
  out->blocks = S.gf;
  return counts[0] ? fail(ctx, SDI_ENONFINITE, "non-finite integrand values") : SDI_OK;
}

int sdi_sector_results(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, double* mean, double* err,
                       double* per_shift, int64_t* nevals) {
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

int sdi_evaluate(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, const void* x_dev, int64_t npts, void* out_dev) {
  if (!ctx || !pb || (!x_dev && npts > 0) || (!out_dev && npts > 0)) return fail(ctx, SDI_EINVAL, "evaluate: null argument");
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  if (npts < 0) return fail(ctx, SDI_EINVAL, "negative point count");
  if (npts == 0) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  EvalArgs A{};
  A.sec = pb->d_secs + s;
  A.terms = pb->d_terms;
  A.x = (const double*)x_dev;
  A.out = (double*)out_dev;
  A.npts = npts;
  if (pb->complex_mode)
    KCHK(ctx, launch_eval_points_cplx(pb->kfmax <= 4 ? 4 : 8, A, pb->d_cx + s, pb->d_dir, ctx->stream));
  else
    KCHK(ctx, launch_eval_points_real(pb->kfmax <= 4 ? 4 : 8, A, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return SDI_OK;
}

int sdi_sample_points(sdi_ctx* ctx, const sdi_problem* pbc, int32_t s, int32_t shift, int64_t i0, int64_t npts,
                      void* x_dev, void* w_dev) {
  sdi_problem* pb = const_cast<sdi_problem*>(pbc);
  if (!ctx || !pb || (!x_dev && npts > 0)) return fail(ctx, SDI_EINVAL, "sample_points: null argument");
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  const Params& prm = ctx->params;
  if (shift < 0 || shift >= prm.R) return fail(ctx, SDI_EINVAL, "shift index out of range");
  if (npts < 0 || i0 < 0 || i0 + npts > ((int64_t)1 << prm.m)) return fail(ctx, SDI_EINVAL, "point range outside the lattice");
  if (npts == 0) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const bool keep_grid = pb->grid_valid && prm.warmup > 0;
  Plan P;
  int rc = make_plan(ctx, pb, P);
  if (rc != SDI_OK) return rc;
  if (!keep_grid)
    for (auto& S : pb->secs) S.flags &= ~F_USE_GRID;
  hipStream_t st = ctx->stream;
  uint64_t* d_sh = nullptr;
  uint64_t* d_zp = nullptr;
  HIPCHK(ctx, hipMalloc((void**)&d_sh, (size_t)pb->nsec * P.rows * MAXV * 8));
  HIPCHK(ctx, hipMalloc((void**)&d_zp, MAXV * 8));
  HIPCHK(ctx, hipMemcpyAsync(pb->d_secs, pb->secs.data(), pb->secs.size() * sizeof(SecDev), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_zp, P.zp_final.data() + (size_t)s * MAXV, MAXV * 8, hipMemcpyHostToDevice, st));
  int e = launch_shifts(pb->d_secs, pb->nsec, P.rows, prm.R, prm.seed, d_sh, st);
  SampleArgs A{};
  A.sec = pb->d_secs + s;
  A.zp = d_zp;
  A.shift = d_sh + ((size_t)pb->secs[s].shift_row + shift) * MAXV;
  A.grid = pb->d_grids ? pb->d_grids + pb->secs[s].grid_off : nullptr;
  A.x = (double*)x_dev;
  A.w = (double*)w_dev;
  A.i0 = (uint64_t)i0;
  A.npts = npts;
  if (e == 0) e = launch_sample_points(A, st);
  hipError_t he = hipStreamSynchronize(st);
  (void)hipFree(d_sh);
  (void)hipFree(d_zp);
  if (e != 0) return fail(ctx, SDI_EDEVICE, std::string("sample kernel: ") + hipGetErrorString((hipError_t)e));
  if (he != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("sample sync: ") + hipGetErrorString(he));
  return SDI_OK;
}

}  // extern "C"
