// Instances of the complex-mode (contour-deformed) tile kernel for sectors of
// up to 8 variables: final pass (mode 0) and Vegas warm-up (mode 1) for the
// autotuner's candidates (points per thread x minimum waves per SIMD), and
// explicit points (mode 2) at one point per thread.
#include "kernels.h"
#include "tiles_cplx.hpp"

namespace sdi {

namespace {
// Explicit points take one point per thread; minimum waves per SIMD is 1 or 2.
void cplx_variant(int mode, int& ppt, int& wpe) {
  if (mode == 2) ppt = 1;
  wpe = wpe >= 2 ? 2 : 1;
}
}  // namespace

int launch_tiles_cplx_nv8(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, const CplxArgs& X,
                           hipStream_t st) {
  const int mode = a.mode;
  cplx_variant(mode, ppt, wpe);
#define SDI_L(M, P, W, K)                                                                    \
  if (mode == M && ppt == P && wpe == W && km == K) {                                         \
    k_tiles_cplx<8, P, K, M, W><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a, X);              \
    return (int)hipGetLastError();                                                            \
  }
  SDI_L(0, 1, 1, 4) SDI_L(0, 1, 2, 4) SDI_L(1, 1, 1, 4) SDI_L(1, 1, 2, 4) SDI_L(2, 1, 1, 4) SDI_L(2, 1, 2, 4) SDI_L(0, 1, 1, 8) SDI_L(0, 1, 2, 8) SDI_L(1, 1, 1, 8) SDI_L(1, 1, 2, 8) SDI_L(2, 1, 1, 8) SDI_L(2, 1, 2, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_cplx_nv8(int mode, int ppt, int wpe, int km, size_t shmem) {
  int nb = 0;
  cplx_variant(mode, ppt, wpe);
#define SDI_O(M, P, W, K)                                                                              \
  if (mode == M && ppt == P && wpe == W && km == K) {                                                   \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_cplx<8, P, K, M, W>, BLOCK, shmem) \
        != hipSuccess) return 0;                                                                        \
    return nb;                                                                                          \
  }
  SDI_O(0, 1, 1, 4) SDI_O(0, 1, 2, 4) SDI_O(1, 1, 1, 4) SDI_O(1, 1, 2, 4) SDI_O(2, 1, 1, 4) SDI_O(2, 1, 2, 4) SDI_O(0, 1, 1, 8) SDI_O(0, 1, 2, 8) SDI_O(1, 1, 1, 8) SDI_O(1, 1, 2, 8) SDI_O(2, 1, 1, 8) SDI_O(2, 1, 2, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
