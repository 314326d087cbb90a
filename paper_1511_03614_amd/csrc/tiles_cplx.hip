// Instances of the complex-mode (contour-deformed) tile kernel and point evaluator.
#include "kernels.h"
#include "tiles_cplx.hpp"

namespace sdi {

int launch_tiles_cplx(int nvmax, int ppt, int km, int grid, size_t shmem, const TileArgs& a, const void* cx,
                      const uint32_t* dir, hipStream_t st) {
  const CplxArgs X{(const CplxDev*)cx, dir};
  const int mode = a.mode;
  if (mode == 2) ppt = 1;
#define SDI_L(M, NV, P, K)                                                             \
  if (mode == M && nvmax == NV && ppt == P && km == K) {                                \
    k_tiles_cplx<NV, P, K, M><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a, X);            \
    return (int)hipGetLastError();                                                     \
  }
  SDI_L(0, 4, 1, 4) SDI_L(0, 4, 2, 4) SDI_L(0, 4, 1, 8) SDI_L(0, 4, 2, 8) SDI_L(0, 6, 1, 4) SDI_L(0, 6, 1, 8) SDI_L(0, 8, 1, 4) SDI_L(0, 8, 1, 8) SDI_L(1, 4, 1, 4) SDI_L(1, 4, 2, 4) SDI_L(1, 4, 1, 8) SDI_L(1, 4, 2, 8) SDI_L(1, 6, 1, 4) SDI_L(1, 6, 1, 8) SDI_L(1, 8, 1, 4) SDI_L(1, 8, 1, 8) SDI_L(2, 4, 1, 4) SDI_L(2, 4, 1, 8) SDI_L(2, 6, 1, 4) SDI_L(2, 6, 1, 8) SDI_L(2, 8, 1, 4) SDI_L(2, 8, 1, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int tiles_cplx_occupancy(int nvmax, int mode, int ppt, int km, size_t shmem) {
  int nb = 0;
  if (mode == 2) ppt = 1;
#define SDI_O(M, NV, P, K)                                                                                      \
  if (mode == M && nvmax == NV && ppt == P && km == K) {                                                        \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_cplx<NV, P, K, M>, BLOCK, shmem) != hipSuccess) \
      return 0;                                                                                                \
    return nb;                                                                                                 \
  }
  SDI_O(0, 4, 1, 4) SDI_O(0, 4, 2, 4) SDI_O(0, 4, 1, 8) SDI_O(0, 4, 2, 8) SDI_O(0, 6, 1, 4) SDI_O(0, 6, 1, 8) SDI_O(0, 8, 1, 4) SDI_O(0, 8, 1, 8) SDI_O(1, 4, 1, 4) SDI_O(1, 4, 2, 4) SDI_O(1, 4, 1, 8) SDI_O(1, 4, 2, 8) SDI_O(1, 6, 1, 4) SDI_O(1, 6, 1, 8) SDI_O(1, 8, 1, 4) SDI_O(1, 8, 1, 8) SDI_O(2, 4, 1, 4) SDI_O(2, 4, 1, 8) SDI_O(2, 6, 1, 4) SDI_O(2, 6, 1, 8) SDI_O(2, 8, 1, 4) SDI_O(2, 8, 1, 8)
#undef SDI_O
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
