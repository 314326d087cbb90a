// Adaptive deterministic cubature over the sectors: the integrator option
// cuhreCuba of CurrentIntegrator (section 4.4), globally adaptive subdivision
// driven by the Genz-Malik degree-7 rule and its embedded degree-5 rule.
//
// Host bookkeeping, GPU rules: every round the host picks the regions to
// halve and the GPU applies the rule pair to all their children in one launch
// (k_cubature, one wave per region).  Definitions:
//  * region error of order k: vol |S7_k - S5_k| (re and im apart); totals
//    T_k = sum of vol S7_k, errors E_k = sum of the region errors;
//  * tolerance tau_k = max(epsabs, epsrel |T_k|), order weights omega_k =
//    1 / tau_k (1 where tau_k = 0);
//  * rounding scale of a region's order k: sigma_k = vol u sum_p (|w7_p| +
//    |w5_p|) |F_k(x_p)|_1 (u = 2^-52); the order counts as converged in the
//    region when e_k = e_re + e_im <= 2^20 sigma_k (below that the rule
//    difference is rounding noise);
//  * priority of a region: max_k omega_k e_k over its orders not converged (0
//    if none: never halved), compared at 8 significant bits (sectors equal up
//    to the order of their terms give twin regions whose errors differ by
//    rounding noise only, sigma/e <= 2^-20; at 8 bits they still tie);
//    equal priorities: the older region;
//  * a round halves the B regions of highest priority, B = max(ceil(frac *
//    alive), min(alive, batch_min)), cut to the longest prefix whose children
//    fit in maxeval, each along the axis the rule chose for it when it was
//    evaluated (the weights of that round); it stops when every order meets
//    its tolerance, when nothing fits or when no region can be halved (zero
//    priority, or 30 halvings of its axis already).
#include <chrono>
#include <cmath>
#include <cstring>

#include "host.h"
#include "kernels.h"

namespace sdi {

namespace {

constexpr int MAX_LEVEL = 30;
constexpr double NOISE = 0x1p20;   // rule differences within NOISE units of roundoff are noise

int64_t rule_points(int n) { return 1 + 4 * (int64_t)n + 2 * (int64_t)n * (n - 1) + ((int64_t)1 << n); }

// v >= 0 rounded to 8 significant bits (half up); NaN and infinity give infinity.
double coarse(double v) {
  if (!(v <= 1.7976931348623157e308)) return INFINITY;
  if (v <= 0.0) return v;
  uint64_t b;
  std::memcpy(&b, &v, 8);
  b = (b + (1ull << 44)) & ~((1ull << 45) - 1);
  std::memcpy(&v, &b, 8);
  return v;
}

// Per-class weights (means over the cube) of the degree-7 rule, then of the
// embedded degree-5 rule, for n = 0..MAXV.
std::vector<double> weight_table() {
  std::vector<double> w((MAXV + 1) * 10, 0.0);
  for (int n = 0; n <= MAXV; ++n) {
    const double d = n;
    double* t = w.data() + n * 10;
    t[0] = (12824.0 - 9120.0 * d + 400.0 * d * d) / 19683.0;
    t[1] = 980.0 / 6561.0;
    t[2] = (1820.0 - 400.0 * d) / 19683.0;
    t[3] = 200.0 / 19683.0;
    t[4] = 6859.0 / 19683.0 / std::ldexp(1.0, n);
    t[5] = (729.0 - 950.0 * d + 50.0 * d * d) / 729.0;
    t[6] = 245.0 / 486.0;
    t[7] = (265.0 - 100.0 * d) / 1458.0;
    t[8] = 25.0 / 729.0;
    t[9] = 0.0;
  }
  return w;
}

// Device buffers of one round (grown on demand, kept with the problem).
int ensure_device(sdi_ctx* ctx, CubState& C, int64_t nreg, int K) {
  const size_t need = align256((size_t)nreg * 4) + align256((size_t)nreg * MAXV) + align256((size_t)nreg * MAXV * 4) +
                      2 * align256((size_t)nreg * K * 16) + align256((size_t)nreg * K * 8) + align256((size_t)nreg * 4) +
                      align256((size_t)nreg * 8) +
                      align256((MAXV + 1) * 10 * 8) + align256((size_t)nreg * 8) + align256(MAXV * 4);
  if (need > C.d_bytes) {
    const size_t bytes = std::max(need, C.d_bytes * 2);
    if (C.d_buf) (void)hipFree(C.d_buf);
    C.d_buf = nullptr;
    C.d_bytes = 0;
    HIPCHK(ctx, hipMalloc(&C.d_buf, bytes));
    C.d_bytes = bytes;
  }
  return SDI_OK;
}

}  // namespace

CubState::~CubState() {
  if (d_buf) (void)hipFree(d_buf);
}

// Counter tag of the partition phase of integrator 4 ("DIV1").
constexpr uint32_t DIV_PART_TAG = 0x44495631u;

// Apply the rule pair (mode 0), the Monte Carlo sample (1: integrator 3; 2:
// the partition phase of integrator 4, with the spreads) to regions [first,
// first + count) of C on the GPU and store their values, errors, axes and counts.
static int evaluate_regions(sdi_ctx* ctx, sdi_problem* pb, CubState& C, int64_t first, int64_t count,
                            const std::vector<double>& omega, float& ms_kernel, int mode) {
  const bool mc = mode != 0;
  if (count <= 0) return SDI_OK;
  const int K = pb->K;
  int rc = ensure_device(ctx, C, count, K);
  if (rc != SDI_OK) return rc;
  char* b = (char*)C.d_buf;
  auto carve = [&](size_t bytes) {
    char* p = b;
    b += align256(bytes);
    return (void*)p;
  };
  int32_t* d_sec = (int32_t*)carve((size_t)count * 4);
  uint8_t* d_lev = (uint8_t*)carve((size_t)count * MAXV);
  uint32_t* d_idx = (uint32_t*)carve((size_t)count * MAXV * 4);
  double* d_val = (double*)carve((size_t)count * K * 16);
  double* d_err = (double*)carve((size_t)count * K * 16);
  double* d_sig = (double*)carve((size_t)count * K * 8);
  int32_t* d_axis = (int32_t*)carve((size_t)count * 4);
  int32_t* d_cnt = (int32_t*)carve((size_t)count * 8);
  double* d_w = (double*)carve((MAXV + 1) * 10 * 8);
  double* d_spread = (double*)carve((size_t)count * 8);
  hipStream_t st = ctx->stream;
  const std::vector<double> wt = weight_table();
  HIPCHK(ctx, hipMemcpyAsync(d_sec, C.sector.data() + first, (size_t)count * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_lev, C.level.data() + first * MAXV, (size_t)count * MAXV, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_idx, C.index.data() + first * MAXV, (size_t)count * MAXV * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_w, wt.data(), wt.size() * 8, hipMemcpyHostToDevice, st));
  CubArgs A{};
  A.secs = pb->d_secs;
  A.terms = pb->d_terms;
  A.cx = pb->complex_mode ? pb->d_cx : nullptr;
  A.dir = pb->complex_mode ? pb->d_dir : nullptr;
  A.reg_sector = d_sec;
  A.reg_level = d_lev;
  A.reg_index = d_idx;
  A.wtab = d_w;
  A.lam[0] = std::sqrt(9.0 / 70.0);
  A.lam[1] = std::sqrt(9.0 / 10.0);
  A.lam[2] = std::sqrt(9.0 / 10.0);
  A.lam[3] = std::sqrt(9.0 / 19.0);
  for (int k = 0; k < KMAX; ++k) A.omega[k] = k < K ? omega[k] : 0.0;
  A.nreg = count;
  A.K = K;
  A.out_val = d_val;
  A.out_err = d_err;
  A.out_sig = d_sig;
  A.out_axis = d_axis;
  A.out_count = d_cnt;
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  HIPCHK(ctx, hipEventRecord(e0, st));
  const int km = pb->kfmax <= 4 ? 4 : 8;
  int krc = 0;
  if (mc) {
    SuaveArgs M{};
    M.secs = pb->d_secs;
    M.terms = pb->d_terms;
    M.cx = A.cx;
    M.dir = A.dir;
    M.reg_sector = d_sec;
    M.reg_level = d_lev;
    M.reg_index = d_idx;
    for (int k = 0; k < KMAX; ++k) M.omega[k] = A.omega[k];
    M.nreg = count;
    M.uid0 = first;
    M.seed = ctx->params.seed;
    M.K = K;
    M.npts = ctx->params.suave_nnew;
    M.out_val = d_val;
    M.out_err = d_err;
    M.out_axis = d_axis;
    M.out_count = d_cnt;
    M.tag = DIV_PART_TAG;
    M.out_spread = d_spread;
    if (mode == 2)
      krc = pb->complex_mode ? launch_divonne_part_cplx(pb->nvmax, km, M, st)
                             : launch_divonne_part_real(pb->nvmax, km, M, st);
    else
      krc = pb->complex_mode ? launch_suave_cplx(pb->nvmax, km, M, st) : launch_suave_real(pb->nvmax, km, M, st);
    if (krc == 0) HIPCHK(ctx, hipMemsetAsync(d_sig, 0, (size_t)count * K * 8, st));
  } else {
    krc = pb->complex_mode ? launch_cubature_cplx(pb->nvmax, km, A, st) : launch_cubature_real(pb->nvmax, km, A, st);
  }
  HIPCHK(ctx, hipEventRecord(e1, st));
  if (krc != 0) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    KCHK(ctx, krc);
  }
  HIPCHK(ctx, hipMemcpyAsync(C.val.data() + first * K * 2, d_val, (size_t)count * K * 16, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(C.err.data() + first * K * 2, d_err, (size_t)count * K * 16, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(C.sig.data() + first * K, d_sig, (size_t)count * K * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(C.axis.data() + first, d_axis, (size_t)count * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(C.count.data() + first * 2, d_cnt, (size_t)count * 8, hipMemcpyDeviceToHost, st));
  if (mode == 2)
    HIPCHK(ctx, hipMemcpyAsync(C.spread.data() + first, d_spread, (size_t)count * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  float ms = 0.f;
  HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
  ms_kernel += ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return SDI_OK;
}

// Grow the host arrays of C to hold n regions.
static void reserve_regions(CubState& C, int64_t n, int K) {
  C.sector.resize(n);
  C.level.resize((size_t)n * MAXV);
  C.index.resize((size_t)n * MAXV);
  C.val.resize((size_t)n * K * 2);
  C.err.resize((size_t)n * K * 2);
  C.sig.resize((size_t)n * K);
  C.axis.resize(n);
  C.count.resize((size_t)n * 2);
  C.alive.resize(n);
  C.spread.resize(n);
}

// The final phase of integrator 4: the lattice rule (divonne.hpp) on the
// regions idx of C, numbered uid0, uid0 + 1, ... in that order; values,
// errors and counts are stored at those regions.
static int lattice_regions(sdi_ctx* ctx, sdi_problem* pb, CubState& C, const std::vector<int64_t>& idx,
                           int64_t uid0, float& ms_kernel) {
  const int64_t count = (int64_t)idx.size();
  if (count == 0) return SDI_OK;
  const int K = pb->K;
  int rc = ensure_device(ctx, C, count, K);
  if (rc != SDI_OK) return rc;
  std::vector<int32_t> sec(count);
  std::vector<uint8_t> lev((size_t)count * MAXV);
  std::vector<uint32_t> ind((size_t)count * MAXV);
  for (int64_t i = 0; i < count; ++i) {
    const int64_t r = idx[i];
    sec[i] = C.sector[r];
    std::memcpy(&lev[(size_t)i * MAXV], &C.level[(size_t)r * MAXV], MAXV);
    std::memcpy(&ind[(size_t)i * MAXV], &C.index[(size_t)r * MAXV], MAXV * 4);
  }
  const Params& prm = ctx->params;
  const std::vector<uint32_t>& z = lattice_vector16(prm.m);
  char* b = (char*)C.d_buf;
  auto carve = [&](size_t bytes) {
    char* p = b;
    b += align256(bytes);
    return (void*)p;
  };
  int32_t* d_sec = (int32_t*)carve((size_t)count * 4);
  uint8_t* d_lev = (uint8_t*)carve((size_t)count * MAXV);
  uint32_t* d_idx = (uint32_t*)carve((size_t)count * MAXV * 4);
  double* d_val = (double*)carve((size_t)count * K * 16);
  double* d_err = (double*)carve((size_t)count * K * 16);
  int32_t* d_cnt = (int32_t*)carve((size_t)count * 8);
  uint32_t* d_z = (uint32_t*)carve(MAXV * 4);
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(d_sec, sec.data(), (size_t)count * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_lev, lev.data(), lev.size(), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_idx, ind.data(), ind.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_z, z.data(), MAXV * 4, hipMemcpyHostToDevice, st));
  DivLatArgs A{};
  A.secs = pb->d_secs;
  A.terms = pb->d_terms;
  A.cx = pb->complex_mode ? pb->d_cx : nullptr;
  A.dir = pb->complex_mode ? pb->d_dir : nullptr;
  A.reg_sector = d_sec;
  A.reg_level = d_lev;
  A.reg_index = d_idx;
  A.zvec = d_z;
  A.nreg = count;
  A.uid0 = uid0;
  A.seed = prm.seed;
  A.K = K;
  A.m = prm.m;
  A.R = prm.R;
  A.baker = prm.baker;
  A.out_val = d_val;
  A.out_err = d_err;
  A.out_count = d_cnt;
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  HIPCHK(ctx, hipEventRecord(e0, st));
  const int km = pb->kfmax <= 4 ? 4 : 8;
  const int krc = pb->complex_mode ? launch_divonne_lattice_cplx(pb->nvmax, km, A, st)
                                   : launch_divonne_lattice_real(pb->nvmax, km, A, st);
  HIPCHK(ctx, hipEventRecord(e1, st));
  if (krc != 0) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    KCHK(ctx, krc);
  }
  std::vector<double> val((size_t)count * K * 2), err((size_t)count * K * 2);
  std::vector<int32_t> cnt((size_t)count * 2);
  HIPCHK(ctx, hipMemcpyAsync(val.data(), d_val, val.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(err.data(), d_err, err.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(cnt.data(), d_cnt, cnt.size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  float ms = 0.f;
  HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
  ms_kernel += ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int64_t i = 0; i < count; ++i) {
    const int64_t r = idx[i];
    std::memcpy(&C.val[(size_t)r * K * 2], &val[(size_t)i * K * 2], (size_t)K * 16);
    std::memcpy(&C.err[(size_t)r * K * 2], &err[(size_t)i * K * 2], (size_t)K * 16);
    C.count[2 * r] += cnt[2 * i];
    C.count[2 * r + 1] += cnt[2 * i + 1];
  }
  return SDI_OK;
}

int run_cubature(sdi_ctx* ctx, sdi_problem* pb, sdi_result* out) {
  const Params& prm = ctx->params;
  const auto t0 = std::chrono::steady_clock::now();
  // integrator 3: the same loop over regions with a Monte Carlo sample per
  // region (suave.hpp): errors are standard errors, combined as a root sum of
  // squares; a region costs suave_nnew evaluations
  // integrator 4: the same loop as the partition phase (Monte Carlo samples,
  // regions halved by spread, divonne.hpp), then a lattice rule on every
  // region of the partition and one refinement of the regions whose two
  // estimates disagree
  const bool div = prm.integrator == 4;
  const bool mc = prm.integrator == 3 || div;
  const int emode = div ? 2 : (mc ? 1 : 0);
  if (div && prm.R < 2) return fail(ctx, SDI_EINVAL, "integrator 4 needs at least 2 shifts");
  if (pb->is_expr()) return fail(ctx, SDI_ENOTSUP, "the adaptive integrators take sector problems, not text integrands");
  if (prm.budget > 0 || prm.warmup > 0 || prm.sampler != 0 || prm.slice_log2 > 0)
    return fail(ctx, SDI_ENOTSUP, "the adaptive integrators run without budget, warmup, sampler or slice_log2");
  auto region_cost = [&](int n) -> int64_t { return mc ? (int64_t)prm.suave_nnew : rule_points(n); };
  const int K = pb->K, nsec = pb->nsec;
  if (!pb->cub) pb->cub = new CubState();
  CubState& C = *pb->cub;
  C.sector.clear();
  C.level.clear();
  C.index.clear();
  C.val.clear();
  C.err.clear();
  C.sig.clear();
  C.axis.clear();
  C.count.clear();
  C.alive.clear();
  int64_t evals = 0;
  for (int s = 0; s < nsec; ++s) evals += region_cost(pb->secs[s].n);
  if (evals > prm.cub_maxeval)
    return fail(ctx, SDI_EINVAL, std::string(mc ? "cub_maxeval is below suave_nnew points per sector ("
                                                 : "cub_maxeval is below one rule application per sector (") +
                                     std::to_string(evals) + ")");
  reserve_regions(C, nsec, K);
  for (int s = 0; s < nsec; ++s) {
    C.sector[s] = s;
    C.alive[s] = 1;
  }
  std::fill(C.level.begin(), C.level.end(), (uint8_t)0);
  std::fill(C.index.begin(), C.index.end(), 0u);
  std::vector<double> omega(K, 1.0), tau(K, 0.0);
  float ms_kernel = 0.f;
  int rc = evaluate_regions(ctx, pb, C, 0, nsec, omega, ms_kernel, emode);
  if (rc != SDI_OK) return rc;
  int rounds = 1;
  bool converged = false;
  int64_t nalive = nsec;
  std::vector<std::pair<double, int64_t>> cand;
  std::vector<double> tot_re(K), tot_im(K), esum(K);
  for (;;) {
    const int64_t nreg = (int64_t)C.sector.size();
    std::fill(tot_re.begin(), tot_re.end(), 0.0);
    std::fill(tot_im.begin(), tot_im.end(), 0.0);
    std::fill(esum.begin(), esum.end(), 0.0);
    std::vector<double> e2re(K, 0.0), e2im(K, 0.0);
    for (int64_t r = 0; r < nreg; ++r) {
      if (!C.alive[r]) continue;
      for (int k = 0; k < K; ++k) {
        tot_re[k] += C.val[(r * K + k) * 2];
        tot_im[k] += C.val[(r * K + k) * 2 + 1];
        const double er = C.err[(r * K + k) * 2], ei = C.err[(r * K + k) * 2 + 1];
        esum[k] += er + ei;
        e2re[k] += er * er;
        e2im[k] += ei * ei;
      }
    }
    if (mc)
      for (int k = 0; k < K; ++k) esum[k] = std::sqrt(e2re[k]) + std::sqrt(e2im[k]);
    bool all = true;
    for (int k = 0; k < K; ++k) {
      tau[k] = std::max(prm.cub_epsabs, prm.cub_epsrel * std::hypot(tot_re[k], tot_im[k]));
      omega[k] = tau[k] > 0.0 ? 1.0 / tau[k] : 1.0;
      all = all && esum[k] <= tau[k];
    }
    if (div) all = false;   // the partition spends its budget (spreads carry the weights of their round)
    if (all) {
      converged = true;
      break;
    }
    cand.clear();
    for (int64_t r = 0; r < nreg; ++r) {
      if (!C.alive[r] || C.level[(size_t)r * MAXV + C.axis[r]] >= MAX_LEVEL) continue;
      double p = 0.0;
      bool bad = false;
      if (div) {
        p = std::isnan(C.spread[r]) ? INFINITY : coarse(C.spread[r]);
        if (p > 0.0) cand.push_back({-p, r});
        continue;
      }
      for (int k = 0; k < K; ++k) {
        const double e = C.err[(r * K + k) * 2] + C.err[(r * K + k) * 2 + 1];
        if (e <= NOISE * C.sig[r * K + k]) continue;   // converged to rounding noise
        const double v = omega[k] * e;
        bad = bad || std::isnan(v);
        p = v > p ? v : p;
      }
      p = bad ? INFINITY : coarse(p);
      if (p > 0.0) cand.push_back({-p, r});
    }
    const int64_t B = std::max<int64_t>((int64_t)std::ceil(prm.cub_split_frac * (double)nalive),
                                        std::min<int64_t>(nalive, prm.cub_batch_min));
    const int64_t take = std::min<int64_t>(B, (int64_t)cand.size());
    std::partial_sort(cand.begin(), cand.begin() + take, cand.end());
    int64_t chosen = 0;
    for (; chosen < take; ++chosen) {
      const int64_t cost = 2 * region_cost(pb->secs[C.sector[cand[chosen].second]].n);
      if (evals + cost > prm.cub_maxeval) break;
      evals += cost;
    }
    if (chosen == 0) break;
    reserve_regions(C, nreg + 2 * chosen, K);
    for (int64_t i = 0; i < chosen; ++i) {
      const int64_t r = cand[i].second;
      C.alive[r] = 0;
      const int ax = C.axis[r];
      for (int h = 0; h < 2; ++h) {
        const int64_t c = nreg + 2 * i + h;
        C.sector[c] = C.sector[r];
        std::memcpy(&C.level[(size_t)c * MAXV], &C.level[(size_t)r * MAXV], MAXV);
        std::memcpy(&C.index[(size_t)c * MAXV], &C.index[(size_t)r * MAXV], MAXV * 4);
        C.level[(size_t)c * MAXV + ax] += 1;
        C.index[(size_t)c * MAXV + ax] = 2 * C.index[(size_t)r * MAXV + ax] + h;
        C.alive[c] = 1;
      }
    }
    nalive += chosen;
    rc = evaluate_regions(ctx, pb, C, nreg, 2 * chosen, omega, ms_kernel, emode);
    if (rc != SDI_OK) return rc;
    ++rounds;
  }
  // integrator 4: the final phase and the refinement
  const int64_t nreg_part = (int64_t)C.sector.size();
  std::vector<int64_t> lat_evals;
  if (div) {
    const int64_t per = (int64_t)prm.R << prm.m;
    const std::vector<double> v1(C.val), e1(C.err);
    std::vector<int64_t> idx;
    for (int64_t r = 0; r < nreg_part; ++r)
      if (C.alive[r]) idx.push_back(r);
    rc = lattice_regions(ctx, pb, C, idx, 0, ms_kernel);
    if (rc != SDI_OK) return rc;
    std::vector<int64_t> redo;
    for (int64_t r : idx) {
      if (C.level[(size_t)r * MAXV + C.axis[r]] >= MAX_LEVEL) continue;
      bool bad = false;
      for (int q = 0; q < K * 2; ++q) {
        const size_t o = (size_t)r * K * 2 + q;
        bad = bad || !(std::fabs(C.val[o] - v1[o]) <= 4.0 * std::hypot(C.err[o], e1[o]));
      }
      if (bad) redo.push_back(r);
    }
    const int64_t nh = 2 * (int64_t)redo.size();
    reserve_regions(C, nreg_part + nh, K);
    std::vector<int64_t> halves;
    for (size_t i = 0; i < redo.size(); ++i) {
      const int64_t r = redo[i];
      C.alive[r] = 0;
      const int ax = C.axis[r];
      for (int h = 0; h < 2; ++h) {
        const int64_t c = nreg_part + 2 * (int64_t)i + h;
        C.sector[c] = C.sector[r];
        std::memcpy(&C.level[(size_t)c * MAXV], &C.level[(size_t)r * MAXV], MAXV);
        std::memcpy(&C.index[(size_t)c * MAXV], &C.index[(size_t)r * MAXV], MAXV * 4);
        C.level[(size_t)c * MAXV + ax] += 1;
        C.index[(size_t)c * MAXV + ax] = 2 * C.index[(size_t)r * MAXV + ax] + h;
        C.axis[c] = ax;
        C.alive[c] = 1;
        halves.push_back(c);
      }
    }
    rc = lattice_regions(ctx, pb, C, halves, (int64_t)idx.size(), ms_kernel);
    if (rc != SDI_OK) return rc;
    lat_evals.assign(nreg_part + nh, 0);
    for (int64_t r : idx) lat_evals[r] = per;
    for (int64_t c : halves) lat_evals[c] = per;
    evals += (int64_t)(idx.size() + halves.size()) * per;
    nalive += (int64_t)redo.size();
    // converged: the final errors within the tolerance per order
    converged = true;
    for (int k = 0; k < K; ++k) {
      double vr = 0.0, vi = 0.0, e2r = 0.0, e2i = 0.0;
      for (int64_t r = 0; r < (int64_t)C.sector.size(); ++r) {
        if (!C.alive[r]) continue;
        vr += C.val[(r * K + k) * 2];
        vi += C.val[(r * K + k) * 2 + 1];
        e2r += C.err[(r * K + k) * 2] * C.err[(r * K + k) * 2];
        e2i += C.err[(r * K + k) * 2 + 1] * C.err[(r * K + k) * 2 + 1];
      }
      const double t = std::max(prm.cub_epsabs, prm.cub_epsrel * std::hypot(vr, vi));
      converged = converged && std::sqrt(e2r) + std::sqrt(e2i) <= t;
    }
  }
  // results: sums over the regions alive, per sector and in total
  const int64_t nreg = (int64_t)C.sector.size();
  pb->sec_stats.assign((size_t)nsec * KMAX * 4, 0.0);
  pb->sec_evals.assign(nsec, 0);
  int64_t nonfin = 0, npos = 0;
  for (int64_t r = 0; r < nreg; ++r) {
    const int s = C.sector[r];
    pb->sec_evals[s] += (r < nreg_part ? region_cost(pb->secs[s].n) : 0) + (div ? lat_evals[r] : 0);
    nonfin += C.count[2 * r];
    npos += C.count[2 * r + 1];
    if (!C.alive[r]) continue;
    for (int k = 0; k < K; ++k) {
      double* q = pb->sec_stats.data() + ((size_t)s * KMAX + k) * 4;
      const double er = C.err[(r * K + k) * 2], ei = C.err[(r * K + k) * 2 + 1];
      q[0] += C.val[(r * K + k) * 2];
      q[1] += C.val[(r * K + k) * 2 + 1];
      q[2] += mc ? er * er : er;   // Monte Carlo: squares first, roots below
      q[3] += mc ? ei * ei : ei;
    }
  }
  for (int k = 0; k < K; ++k) {
    double vr = 0.0, vi = 0.0, er = 0.0, ei = 0.0;
    for (int s = 0; s < nsec; ++s) {
      double* q = pb->sec_stats.data() + ((size_t)s * KMAX + k) * 4;
      vr += q[0];
      vi += q[1];
      er += q[2];
      ei += q[3];
      if (mc) {
        q[2] = std::sqrt(q[2]);
        q[3] = std::sqrt(q[3]);
      }
    }
    out->val_re[k] = vr;
    out->val_im[k] = vi;
    out->err_re[k] = mc ? std::sqrt(er) : er;
    out->err_im[k] = mc ? std::sqrt(ei) : ei;
  }
  pb->per_shift.clear();
  pb->last_R = 0;
  pb->have_results = true;
  pb->last_sampler = -1;
  pb->last_m = -1;
  out->order_min = pb->order_min;
  out->norders = K;
  out->n_evals = evals;
  out->n_nonfinite = nonfin;
  out->n_imf_positive = npos;
  out->ms_sample_eval_reduce = ms_kernel;
  out->ms_refit = 0.0;
  out->ms_eval_kernel = ms_kernel;
  out->points_per_thread = 1;
  out->blocks = 0;
  out->tile_log2 = 0;
  out->waves_per_simd = 0;
  out->grouped = 0;
  out->ms_pilot_kernel = 0.0;
  out->pilot_same_kernel = 0;
  out->lattice_done = 0;
  out->cub_regions = nalive;
  out->cub_rounds = rounds;
  out->cub_converged = converged ? 1 : 0;
  out->ms_flow_train = 0.0;
  out->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return nonfin > 0 ? SDI_ENONFINITE : SDI_OK;
}

}  // namespace sdi

extern "C" {

int sdi_cubature_regions(sdi_ctx* ctx, const sdi_problem* pb, int64_t cap, int64_t* nregions, int32_t* sector,
                         uint8_t* level, uint32_t* index, double* value, double* error, int32_t* axis) {
  if (!ctx || !pb || !nregions) return sdi::fail(ctx, SDI_EINVAL, "cubature_regions: null argument");
  if (!pb->cub || pb->cub->alive.empty()) return sdi::fail(ctx, SDI_ESTATE, "no cubature run on this problem");
  const sdi::CubState& C = *pb->cub;
  const int K = pb->K;
  int64_t n = 0;
  for (size_t r = 0; r < C.alive.size(); ++r) {
    if (!C.alive[r]) continue;
    if (n < cap) {
      if (sector) sector[n] = C.sector[r];
      if (level) std::memcpy(level + n * sdi::MAXV, &C.level[r * sdi::MAXV], sdi::MAXV);
      if (index) std::memcpy(index + n * sdi::MAXV, &C.index[r * sdi::MAXV], sdi::MAXV * 4);
      if (value) std::memcpy(value + n * K * 2, &C.val[r * K * 2], (size_t)K * 16);
      if (error) std::memcpy(error + n * K * 2, &C.err[r * K * 2], (size_t)K * 16);
      if (axis) axis[n] = C.axis[r];
    }
    ++n;
  }
  *nregions = n;
  return SDI_OK;
}

}  // extern "C"
