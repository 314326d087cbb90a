// libsdint C ABI: context, parameters, problem compilation and the integration driver.
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "host.h"
#include "poles.h"
#include "kernels.h"
#include "poles.h"

using namespace sdi;

namespace sdi {

int fail(sdi_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

}  // namespace sdi

namespace {



bool is_int(double v, double lim) { return std::isfinite(v) && v == std::floor(v) && std::fabs(v) <= lim; }


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
  // the fixed scratch of the allocation-free entry point: its address on this
  // device, taken once per device with the device current
  {
    static std::mutex mu;
    static std::vector<void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)addr.size() < ndev) addr.resize(ndev, nullptr);
    if (!addr[device_ordinal] && noalloc_scratch_address(&addr[device_ordinal]) != 0) {
      addr[device_ordinal] = nullptr;
      (void)hipGetLastError();
      delete c;
      return SDI_EDEVICE;
    }
    c->scratch = addr[device_ordinal];
  }
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
  if (k == "sampler" && (v == "lattice" || v == "vegas" || v == "flow")) {
    p.sampler = v == "flow" ? 1 : 0;
    if (v == "vegas" && p.warmup == 0) p.warmup = 5;
    return SDI_OK;
  }
  if (k == "tune") {
    if (v == "off") p.tune = 0;
    else if (v == "cached") p.tune = 1;
    else if (v == "search") p.tune = 2;
    else return fail(ctx, SDI_EINVAL, "tune must be off, cached or search");
    return SDI_OK;
  }
  if (k == "small_x" || k == "cub_epsrel" || k == "cub_epsabs" || k == "cub_split_frac") {
    char* e = nullptr;
    errno = 0;
    const double d = strtod(value, &e);
    if (errno || !e || *e != '\0' || e == value) return fail(ctx, SDI_EINVAL, k + " must be a number");
    if (k == "small_x") {
      if (!(d >= 0.0 && d <= 1.0)) return fail(ctx, SDI_EINVAL, "small_x must be a number in [0, 1]");
      p.small_x = d;
    } else if (k == "cub_split_frac") {
      if (!(d > 0.0 && d <= 1.0)) return fail(ctx, SDI_EINVAL, "cub_split_frac must be in (0, 1]");
      p.cub_split_frac = d;
    } else {
      if (!(d >= 0.0 && d <= 1.0)) return fail(ctx, SDI_EINVAL, k + " must be in [0, 1]");
      (k == "cub_epsrel" ? p.cub_epsrel : p.cub_epsabs) = d;
    }
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
    if (!(iv == 0 || range(6, 24))) return fail(ctx, SDI_EINVAL, "tile_log2 must be 0 (autotuned) or in 6..24");
    p.tile_log2 = (int)iv;
  } else if (k == "ppt") {
    if (!(iv == 0 || iv == 1 || iv == 2 || iv == 4)) return fail(ctx, SDI_EINVAL, "ppt must be 0, 1, 2 or 4");
    p.ppt = (int)iv;
  } else if (k == "graph") {
    if (!range(0, 1)) return fail(ctx, SDI_EINVAL, "graph must be 0 or 1");
    p.graph = (int)iv;
  } else if (k == "slice_log2") {
    if (!range(0, 30)) return fail(ctx, SDI_EINVAL, "slice_log2 must be in 0..30");
    p.slice_log2 = (int)iv;
  } else if (k == "points" || k == "budget_min" || k == "budget_max") {
    // evaluations per sector = shifts x 2^m
    const long long r = p.R;
    if (iv < 16 * r || iv % r != 0 || ((iv / r) & (iv / r - 1)) != 0)
      return fail(ctx, SDI_EINVAL, k + " must be shifts x 2^m with m >= 4 (shifts = " + std::to_string(r) + ")");
    int m = 0;
    while ((1ll << m) < iv / r) ++m;
    if (k == "points") {
      if (m > 30) return fail(ctx, SDI_EINVAL, "points: lattice_log2 above 30");
      p.m = m;
    } else if (k == "budget_min") {
      if (m > 24) return fail(ctx, SDI_EINVAL, "budget_min: alloc_min_log2 above 24");
      p.alloc_min = m;
    } else {
      if (m > 26) return fail(ctx, SDI_EINVAL, "budget_max: alloc_max_log2 above 26");
      p.alloc_max = m;
    }
  } else if (k == "budget_total") {
    if (!range(0, (long long)1 << 40)) return fail(ctx, SDI_EINVAL, "budget_total must be in 0..2^40");
    p.budget = iv;
  } else if (k == "iterations") {
    if (!range(0, 64)) return fail(ctx, SDI_EINVAL, "iterations must be in 0..64");
    p.warmup = (int)iv;
  } else if (k == "integrator") {
    if (!range(0, 4))
      return fail(ctx, SDI_EINVAL,
                  "integrator must be 0 (lattice), 1 (cubature), 2 (Monte Carlo points), 3 (subregion-adaptive "
                  "Monte Carlo) or 4 (partition by spreads, then lattice rules)");
    p.integrator = (int)iv;
  } else if (k == "cub_maxeval") {
    if (!range(1, (long long)1 << 40)) return fail(ctx, SDI_EINVAL, "cub_maxeval must be in 1..2^40");
    p.cub_maxeval = iv;
  } else if (k == "cub_batch_min") {
    if (!range(1, 1 << 24)) return fail(ctx, SDI_EINVAL, "cub_batch_min must be in 1..2^24");
    p.cub_batch_min = (int)iv;
  } else if (k == "suave_nnew") {
    if (!range(16, 1 << 20)) return fail(ctx, SDI_EINVAL, "suave_nnew must be in 16..2^20");
    p.suave_nnew = (int)iv;
  } else if (k == "separate_terms") {
    if (!range(0, 1)) return fail(ctx, SDI_EINVAL, "separate_terms must be 0 or 1");
    p.separate_terms = (int)iv;
  } else if (k == "budget") {
    if (!range(0, (long long)1 << 40)) return fail(ctx, SDI_EINVAL, "budget must be in 0..2^40");
    p.budget = iv;
  } else if (k == "alloc_min_log2") {
    if (!range(4, 24)) return fail(ctx, SDI_EINVAL, "alloc_min_log2 must be in 4..24");
    p.alloc_min = (int)iv;
  } else if (k == "alloc_max_log2") {
    if (!range(4, 26)) return fail(ctx, SDI_EINVAL, "alloc_max_log2 must be in 4..26");
    p.alloc_max = (int)iv;
  } else if (k == "sampler") {
    if (!range(0, 1)) return fail(ctx, SDI_EINVAL, "sampler must be 0 (lattice) or 1 (flow)");
    p.sampler = (int)iv;
  } else if (k == "pilot_log2") {
    if (!range(4, 20)) return fail(ctx, SDI_EINVAL, "pilot_log2 must be in 4..20");
    p.pilot_log2 = (int)iv;
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
  } else if (k == "small_x" || k == "cub_epsrel" || k == "cub_epsabs" || k == "cub_split_frac") {
    snprintf(buf, len, "%.17g",
             k == "small_x" ? p.small_x : (k == "cub_epsrel" ? p.cub_epsrel : (k == "cub_epsabs" ? p.cub_epsabs : p.cub_split_frac)));
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
  else if (k == "budget") v = p.budget;
  else if (k == "slice_log2") v = p.slice_log2;
  else if (k == "integrator") v = p.integrator;
  else if (k == "points") v = (long long)p.R << p.m;
  else if (k == "budget_total") v = p.budget;
  else if (k == "budget_min") v = (long long)p.R << p.alloc_min;
  else if (k == "budget_max") v = (long long)p.R << p.alloc_max;
  else if (k == "iterations") v = p.warmup;
  else if (k == "cub_maxeval") v = p.cub_maxeval;
  else if (k == "cub_batch_min") v = p.cub_batch_min;
  else if (k == "suave_nnew") v = p.suave_nnew;
  else if (k == "separate_terms") v = p.separate_terms;
  else if (k == "alloc_min_log2") v = p.alloc_min;
  else if (k == "alloc_max_log2") v = p.alloc_max;
  else if (k == "pilot_log2") v = p.pilot_log2;
  else if (k == "sampler") v = p.sampler;
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
  // sectors with a_j < -1 are replaced by their integration-by-parts parts
  PoleExpansion X;
  {
    std::string err;
    int rc = expand_poles(d, X, err);
    if (rc != SDI_OK) return fail(ctx, rc, err);
    if (ctx->params.separate_terms) {
      // the subtraction terms of a deformed sector share the deformation's
      // corner factors w_j^(b_j eps), so they are separated in real mode only
      if (d->complex_mode) return fail(ctx, SDI_ENOTSUP, "separate_terms works in real mode only");
      rc = separate_terms(X, err);
      if (rc != SDI_OK) return fail(ctx, rc, err);
    }
  }
  sdi_problem* pb = new sdi_problem();
  pb->ctx = ctx;
  pb->nsec = (int)X.descs.size();
  pb->origin = X.origin;
  pb->K = K;
  pb->order_min = d->order_min;
  pb->complex_mode = d->complex_mode;
  pb->lambda = d->lambda;
  auto bad = [&](int code, const std::string& m) {
    delete pb;
    return fail(ctx, code, m);
  };
  const int kf_max = d->order_max - d->pref_lead;
  for (int s = 0; s < pb->nsec; ++s) {
    const sdi_sector_desc& sd = X.descs[s];
    const std::string where = "sector " + std::to_string(X.origin[s]) +
                              (pb->nsec != d->nsectors ? " (part " + std::to_string(s) + ")" : "") + ": ";
    const int n = sd.nvars;
    if (n < 1 || n > MAXV) return bad(SDI_EINVAL, where + "nvars must be 1..16");
    if (sd.nfactors < 0 || sd.nfactors > MAXF) return bad(SDI_EINVAL, where + "nfactors must be 0..4");
    if (sd.reserved != 0) return bad(SDI_EINVAL, where + "reserved must be 0");
    if (sd.deform_factor < -1 || sd.deform_factor >= sd.nfactors) return bad(SDI_EINVAL, where + "bad deform_factor");
    if (!sd.mono_a || !sd.mono_b || (sd.nfactors && (!sd.fac_nterms || !sd.fac_gamma || !sd.fac_delta)))
      return bad(SDI_EINVAL, where + "null array");
    if (!std::isfinite(sd.coeff_re) || !std::isfinite(sd.coeff_im)) return bad(SDI_EINVAL, where + "coefficient not finite");
    if (sd.term_coef_im && !d->complex_mode)
      return bad(SDI_EINVAL, where + "complex term coefficients need complex mode");
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
    // a separated term carries eps^-shift; sub_only drops its boundary terms
    const int shift = X.shift.empty() ? 0 : X.shift[s];
    const bool sub_only = !X.sub_only.empty() && X.sub_only[s];
    R.kf = std::max(0, kf_max + R.ns + shift + 1);
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
      R.invb[T] = (sub_only && T != 0) ? 0.0 : v;
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
    // terms per (factor, corner); the imaginary parts of complex coefficients
    // go to terms_im at the same index (0 for real ones and for the
    // deformation lists, which follow the real part of F)
    size_t t0 = 0;
    bool exp7 = false;
    bool cplx_coef = false;
    auto push_term = [&](double re, double im, uint64_t word) {
      pb->terms.push_back(Term{re, word});
      pb->terms_im.push_back(im);
    };
    for (int m = 0; m < sd.nfactors; ++m) {
      const int nt = sd.fac_nterms[m];
      if (nt < 0) return bad(SDI_EINVAL, where + "negative term count");
      if (nt > 0 && (!sd.term_coef || !sd.term_exps)) return bad(SDI_EINVAL, where + "null term arrays");
      for (int t = 0; t < nt; ++t) {
        if (!std::isfinite(sd.term_coef[t0 + t]) || (sd.term_coef_im && !std::isfinite(sd.term_coef_im[t0 + t])))
          return bad(SDI_EINVAL, where + "term coefficient not finite");
        if (sd.term_coef_im && sd.term_coef_im[t0 + t] != 0.0) cplx_coef = true;
        for (int j = 0; j < n; ++j) {
          const int e = sd.term_exps[(t0 + t) * n + j];
          if (e > (d->complex_mode ? 3 : 7))
            return bad(SDI_ENOTSUP, where + (d->complex_mode ? "polynomial exponents above 3 are not supported in complex mode"
                                                             : "polynomial exponents above 7 are not supported"));
          if (e > 3) exp7 = true;
        }
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
          push_term(sd.term_coef[t0 + t], sd.term_coef_im ? sd.term_coef_im[t0 + t] : 0.0, word);
          ++cnt;
        }
        R.tab_cnt[m][W] = cnt;
      }
      // the same terms by singular support (each term once)
      R.grp_mask[m] = 0;
      for (int sg = 0; sg < (1 << R.ns); ++sg) {
        R.grp_off[m][sg] = (uint32_t)pb->terms.size();
        uint32_t cnt = 0;
        for (int t = 0; t < nt; ++t) {
          const uint8_t* e = sd.term_exps + (t0 + t) * n;
          int sup = 0;
          for (int i = 0; i < R.ns; ++i)
            if (e[S[i]] != 0) sup |= 1 << i;
          if (sup != sg) continue;
          uint64_t word = 0;
          for (int j = 0; j < n; ++j) word |= (uint64_t)e[perm[j]] << (4 * j);
          push_term(sd.term_coef[t0 + t], sd.term_coef_im ? sd.term_coef_im[t0 + t] : 0.0, word);
          ++cnt;
        }
        R.grp_cnt[m][sg] = cnt;
        if (cnt) R.grp_mask[m] |= 1u << sg;
      }
      t0 += nt;
    }
    if (exp7) {
      R.flags |= F_EXP7;
      pb->exp7 = true;
    }
    if (d->complex_mode) {
      // derivative lists of the full F = x^mono * P_F (internal variable order), per corner
      CplxDev X{};
      X.lam = d->lambda;
      X.fac_f = sd.deform_factor;
      X.coef_im = nullptr;   // set to the device table after the upload when cplx_coef
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
              push_term(t.first, 0.0, word);
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
      pb->cx_cplx_coef.push_back(cplx_coef ? 1 : 0);
    }
    // fold: F_k = sum_kk c_s (Pi * C)_i f_kk, i = k - lead - (kk - ns - shift),
    // C the coefficient series of a part of a sector with a_j < -1 or of a
    // separated term (1 otherwise)
    bool has_im = false;
    const std::vector<std::complex<double>>& cser = X.series[s];
    for (int k = 0; k < K; ++k)
      for (int kk = 0; kk < KMAX; ++kk) {
        const int i = (d->order_min + k) - d->pref_lead - (kk - R.ns - shift);
        double fr = 0.0, fi = 0.0;
        if (kk < R.kf && i >= 0) {
          std::complex<double> pc = 0.0;
          for (int q = 0; q <= i && q < (int)cser.size(); ++q)
            if (i - q < d->pref_len)
              pc += std::complex<double>(d->pref_re[i - q], d->pref_im ? d->pref_im[i - q] : 0.0) * cser[q];
          const double pr = pc.real(), pi = pc.imag();
          fr = sd.coeff_re * pr - sd.coeff_im * pi;
          fi = sd.coeff_re * pi + sd.coeff_im * pr;
        }
        R.fold_re[k][kk] = fr;
        R.fold_im[k][kk] = fi;
        if (fi != 0.0) has_im = true;
      }
    if (has_im) R.flags |= F_HAS_IM;
    // cost estimate per point: polynomial work (every term once, by singular
    // support, plus the corner sums), corners with their logs, and the series
    double c = 40.0 * (n + 1);
    for (int m = 0; m < sd.nfactors; ++m)
      for (int sg = 0; sg < (1 << R.ns); ++sg) c += (2.0 + n) * R.grp_cnt[m][sg] + 2.0 * (1 << R.ns);
    for (int W = 0; W < (1 << R.ns); ++W) c += 80.0 + 3.0 * R.kf * (1 << R.ns);
    pb->cost.push_back(c);
    pb->secs.push_back(R);
    // variable class of the persistent kernel instance; the <= 6 and <= 10
    // classes need fewer registers (higher occupancy, fewer spills) than the
    // next larger one for the common 5-6 and 9-10 variable sectors
    const int nvc = n <= 4 ? 4 : (n <= 6 ? 6 : (n <= 8 ? 8 : (n <= 10 ? 10 : 16)));
    pb->nvmax = std::max(pb->nvmax, nvc);
    if (d->complex_mode) c *= 8.0 + 2.0 * n * n;
    pb->kfmax = std::max(pb->kfmax, R.kf);
    pb->nsmax = std::max(pb->nsmax, R.ns);
    pb->nfmax = std::max(pb->nfmax, R.nfac);
  }
  if (pb->terms.empty()) {
    pb->terms.push_back(Term{0.0, 0});
    pb->terms_im.push_back(0.0);
  }
  bool any_cplx_coef = false;
  for (char c : pb->cx_cplx_coef) any_cplx_coef = any_cplx_coef || c;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_secs, pb->secs.size() * sizeof(SecDev));
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_terms, pb->terms.size() * sizeof(Term));
  if (e == hipSuccess)
    e = hipMemcpy(pb->d_terms, pb->terms.data(), pb->terms.size() * sizeof(Term), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pb->d_secs, pb->secs.data(), pb->secs.size() * sizeof(SecDev), hipMemcpyHostToDevice);
  if (e == hipSuccess && any_cplx_coef) {
    e = hipMalloc((void**)&pb->d_terms_im, pb->terms_im.size() * sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpy(pb->d_terms_im, pb->terms_im.data(), pb->terms_im.size() * sizeof(double),
                    hipMemcpyHostToDevice);
    for (size_t s = 0; s < pb->cx.size(); ++s)
      if (pb->cx_cplx_coef[s]) pb->cx[s].coef_im = pb->d_terms_im;
  }
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
  free_passes(pb->passes);
  if (pb->d_secs) (void)hipFree(pb->d_secs);
  if (pb->d_terms) (void)hipFree(pb->d_terms);
  if (pb->d_terms_im) (void)hipFree(pb->d_terms_im);
  if (pb->d_grids) (void)hipFree(pb->d_grids);
  if (pb->d_ws) (void)hipFree(pb->d_ws);
  if (pb->d_cx) (void)hipFree(pb->d_cx);
  if (pb->d_dir) (void)hipFree(pb->d_dir);
  if (pb->d_expr) (void)hipFree(pb->d_expr);
  delete pb->flow;
  delete pb->cub;
  delete pb;
}

int sdi_problem_norders(const sdi_problem* pb) { return pb ? pb->K : SDI_EINVAL; }

int sdi_problem_nsectors(const sdi_problem* pb) { return pb ? pb->nsec : SDI_EINVAL; }

int sdi_problem_sector_origin(const sdi_problem* pb, int32_t s) {
  if (!pb || s < 0 || s >= pb->nsec) return SDI_EINVAL;
  return pb->origin.empty() ? s : pb->origin[s];
}

int sdi_problem_nvars(const sdi_problem* pb, int32_t s) {
  if (!pb || s < 0 || s >= pb->nsec) return SDI_EINVAL;
  return pb->secs[s].n;
}

int sdi_evaluate(sdi_ctx* ctx, const sdi_problem* pb, int32_t s, const void* x_dev, int64_t npts, void* out_dev,
                 void* cond_dev) {
  if (!ctx || !pb || (!x_dev && npts > 0) || (!out_dev && npts > 0)) return fail(ctx, SDI_EINVAL, "evaluate: null argument");
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  if (npts < 0) return fail(ctx, SDI_EINVAL, "negative point count");
  if (npts == 0) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  EvalArgs A{};
  A.sec = pb->d_secs + s;
  A.terms = pb->d_terms;
  A.x = (const double*)x_dev;
  A.out = (double*)out_dev;
  A.npts = npts;
  A.cond = (double*)cond_dev;
  A.small_x = pb->is_expr() ? 0.0 : ctx->params.small_x;
  if (pb->is_expr())
    KCHK(ctx, launch_eval_points_expr(A, ExprArgs{pb->d_expr, (int32_t)pb->expr_nins, pb->expr_slots, pb->expr_out, pb->expr_cplx ? 1 : 0},
                                      ctx->stream));
  else if (pb->complex_mode)
    KCHK(ctx, launch_eval_points_cplx(pb->kfmax <= 4 ? 4 : 8, A, pb->d_cx + s, pb->d_dir, ctx->stream));
  else
    KCHK(ctx, launch_eval_points_real(pb->kfmax <= 4 ? 4 : 8, A, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return SDI_OK;
}

}  // extern "C"
