// Dispatch of the complex-mode (contour-deformed) tile kernel over its variable
// classes, and the complex point evaluators.
#include "kernels.h"
#include "tiles_cplx.hpp"

namespace sdi {

int launch_tiles_cplx(int nvmax, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a,
                      const void* cx, const uint32_t* dir, hipStream_t st) {
  const CplxArgs X{(const CplxDev*)cx, dir};
  if (a.mode != 1 && a.small_x > 0.0) return nvmax <= 8 ? launch_tiles_cplx_dd(km, grid, shmem, a, X, st)
                                                        : (int)hipErrorInvalidValue;
  if (nvmax <= 4) return launch_tiles_cplx_nv4(ppt, wpe, km, grid, shmem, a, X, st);
  if (nvmax <= 6) return launch_tiles_cplx_nv6(ppt, wpe, km, grid, shmem, a, X, st);
  if (nvmax <= 8) return launch_tiles_cplx_nv8(ppt, wpe, km, grid, shmem, a, X, st);
  return (int)hipErrorInvalidValue;
}

int tiles_cplx_occupancy(int nvmax, int mode, int ppt, int wpe, int km, bool dd, size_t shmem) {
  if (mode != 1 && dd) return nvmax <= 8 ? occupancy_tiles_cplx_dd(mode, km, shmem) : 0;
  if (nvmax <= 4) return occupancy_tiles_cplx_nv4(mode, ppt, wpe, km, shmem);
  if (nvmax <= 6) return occupancy_tiles_cplx_nv6(mode, ppt, wpe, km, shmem);
  if (nvmax <= 8) return occupancy_tiles_cplx_nv8(mode, ppt, wpe, km, shmem);
  return 0;
}

int launch_eval_points_cplx(int km, const EvalArgs& a, const void* cx, const uint32_t* dir, hipStream_t st) {
  if (a.npts <= 0) return 0;
  const CplxArgs X{(const CplxDev*)cx, dir};
  const unsigned g = (unsigned)((a.npts + BLOCK - 1) / BLOCK);
  if (km == 4)
    k_eval_points_cplx<4><<<dim3(g), dim3(BLOCK), 0, st>>>(a, X);
  else
    k_eval_points_cplx<8><<<dim3(g), dim3(BLOCK), 0, st>>>(a, X);
  return (int)hipGetLastError();
}

int launch_eval_tiles_cplx(int km, const EvalTilesArgs& a, const void* cx, const uint32_t* dir, hipStream_t st) {
  if (a.nchunks <= 0) return 0;
  const CplxArgs X{(const CplxDev*)cx, dir};
  const unsigned g = (unsigned)(a.nchunks < (1 << 20) ? a.nchunks : (1 << 20));
  if (km == 4)
    k_eval_tiles_cplx<4><<<dim3(g), dim3(BLOCK), 0, st>>>(a, X);
  else
    k_eval_tiles_cplx<8><<<dim3(g), dim3(BLOCK), 0, st>>>(a, X);
  return (int)hipGetLastError();
}

int launch_lambda_test(int nvmax, const SecDev* secs, int nsec, const void* cx, const uint32_t* dir,
                       const Term* terms, const uint64_t* zp, const uint64_t* shifts, int64_t npts,
                       const double* cand, int ncand, int32_t* fail, hipStream_t st) {
  if (nsec <= 0 || npts <= 0) return 0;
  const dim3 grid((unsigned)((npts + BLOCK - 1) / BLOCK), (unsigned)nsec);
  const CplxDev* c = (const CplxDev*)cx;
  if (nvmax <= 4)
    k_lambda_test<4><<<grid, dim3(BLOCK), 0, st>>>(secs, c, dir, terms, zp, shifts, npts, cand, ncand, fail);
  else if (nvmax <= 6)
    k_lambda_test<6><<<grid, dim3(BLOCK), 0, st>>>(secs, c, dir, terms, zp, shifts, npts, cand, ncand, fail);
  else
    k_lambda_test<8><<<grid, dim3(BLOCK), 0, st>>>(secs, c, dir, terms, zp, shifts, npts, cand, ncand, fail);
  return (int)hipGetLastError();
}

}  // namespace sdi
