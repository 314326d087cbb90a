// Automatic choice of the contour-deformation size per sector (the ComplexMode
// tuning of section 4.4): candidates lam_k = top * k / split, k = split .. 1,
// are tested on the first 2^m points of the sector's tent-transformed lattice
// (Philox shift row 65535); the largest lam_k under which no test point has
// Im F(z) > 0 at any corner is kept; if none passes, top /= split and the next
// round starts (at most four rounds, then lam = 0).  Conservative mode halves
// the result.  All candidates of a round are tested in one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "host.h"
#include "kernels.h"

using namespace sdi;

extern "C" int sdi_tune_deformation(sdi_ctx* ctx, sdi_problem* pb, double lam_max, int32_t split,
                                    int32_t points_log2, int32_t conservative, double* lam_out) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "tune_deformation: null argument");
  if (!pb->complex_mode) return fail(ctx, SDI_ESTATE, "tune_deformation: the problem is not in complex mode");
  if (!(lam_max > 0.0) || !std::isfinite(lam_max)) return fail(ctx, SDI_EINVAL, "lambda_max must be positive");
  if (split < 1 || split > 16) return fail(ctx, SDI_EINVAL, "split must be in 1..16");
  if (points_log2 < 4 || points_log2 > 20) return fail(ctx, SDI_EINVAL, "points_log2 must be in 4..20");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  const int nsec = pb->nsec;
  const int m = points_log2;
  std::vector<SecDev> secs = pb->secs;
  for (int s = 0; s < nsec; ++s) {
    secs[s].m = m;
    secs[s].mw = m;
    secs[s].shift_row = s;
    secs[s].flags = (secs[s].flags & ~F_USE_GRID) | F_BAKER;
  }
  std::vector<uint64_t> zp((size_t)nsec * MAXV);
  const std::vector<uint32_t>& z = lattice_vector16(m);
  for (int s = 0; s < nsec; ++s)
    for (int j = 0; j < MAXV; ++j) zp[(size_t)s * MAXV + j] = (uint64_t)z[j] << (53 - m);
  Carve C;
  SecDev* d_secs = nullptr;
  uint64_t *d_zp = nullptr, *d_sh = nullptr;
  double* d_cand = nullptr;
  int32_t* d_fail = nullptr;
  C.add((void**)&d_secs, sizeof(SecDev) * nsec);
  C.add((void**)&d_zp, zp.size() * 8);
  C.add((void**)&d_sh, (size_t)nsec * MAXV * 8);
  C.add((void**)&d_cand, (size_t)nsec * split * 8);
  C.add((void**)&d_fail, (size_t)nsec * 4);
  void* base = nullptr;
  if (hipMalloc(&base, C.total()) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, SDI_ENOMEM, "tune_deformation: allocation failed");
  }
  struct Free {
    void* p;
    ~Free() { (void)hipFree(p); }
  } guard{base};
  C.assign(base);
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(d_secs, secs.data(), sizeof(SecDev) * nsec, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_zp, zp.data(), zp.size() * 8, hipMemcpyHostToDevice, st));
  KCHK(ctx, launch_shifts(d_secs, nsec, 1, 1, ctx->params.seed, 65535u, d_sh, st));
  std::vector<double> top(nsec, lam_max), chosen(nsec, -1.0), cand((size_t)nsec * split);
  std::vector<int32_t> fails(nsec);
  for (int round = 0; round < 4; ++round) {
    bool open = false;
    for (int s = 0; s < nsec; ++s)
      for (int k = 0; k < split; ++k) cand[(size_t)s * split + k] = top[s] * (double)(k + 1) / (double)split;
    for (int s = 0; s < nsec; ++s) open = open || chosen[s] < 0.0;
    if (!open) break;
    HIPCHK(ctx, hipMemcpyAsync(d_cand, cand.data(), cand.size() * 8, hipMemcpyHostToDevice, st));
    KCHK(ctx, launch_fill_i32(d_fail, 0, nsec, st));
    KCHK(ctx, launch_lambda_test(pb->nvmax, d_secs, nsec, pb->d_cx, pb->d_dir, pb->d_terms, d_zp, d_sh,
                                 (int64_t)1 << m, d_cand, split, d_fail, st));
    HIPCHK(ctx, hipMemcpyAsync(fails.data(), d_fail, (size_t)nsec * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    for (int s = 0; s < nsec; ++s) {
      if (chosen[s] >= 0.0) continue;
      for (int k = split - 1; k >= 0; --k)
        if (!((fails[s] >> k) & 1)) {
          chosen[s] = cand[(size_t)s * split + k];
          break;
        }
      if (chosen[s] < 0.0) top[s] /= (double)split;
    }
  }
  for (int s = 0; s < nsec; ++s) {
    double l = chosen[s] < 0.0 ? 0.0 : chosen[s];
    if (conservative) l *= 0.5;
    pb->cx[s].lam = l;
    if (lam_out) lam_out[s] = l;
  }
  HIPCHK(ctx, hipMemcpyAsync(pb->d_cx, pb->cx.data(), sizeof(CplxDev) * nsec, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return SDI_OK;
}
