// Instances of the real-mode tile kernel for problems with factor exponents
// above 3 (up to 7: the x^4 bit of the term words): per variable class one
// generic instance (each corner's term lists, one point per thread, at least
// 4 waves per SIMD) for the final pass, the Vegas warm-up and explicit points,
// and the endpoint-precision final pass (lattice or explicit points; every
// class, one point per thread, 2 waves per SIMD, points below small_x again in
// double-double).
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_e7(int nvmax, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
  const int mode = a.mode;
  if (mode != 1 && a.small_x > 0.0) {
#define SDI_D(M, K)                                                                              \
  if (mode == M && km == K) {                                                                    \
    k_tiles_real<MAXV, 1, K, M, 2, MAXS, true, 0, 1><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a); \
    return (int)hipGetLastError();                                                               \
  }
    SDI_D(0, 4) SDI_D(0, 8) SDI_D(2, 4) SDI_D(2, 8)
#undef SDI_D
    return (int)hipErrorInvalidValue;
  }
#define SDI_L(NV, M, K)                                                                      \
  if (mode == M && km == K) {                                                                \
    k_tiles_real<NV, 1, K, M, 4, MAXS, false, 0, 1><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a); \
    return (int)hipGetLastError();                                                           \
  }
#define SDI_NV(NV) SDI_L(NV, 0, 4) SDI_L(NV, 1, 4) SDI_L(NV, 2, 4) SDI_L(NV, 0, 8) SDI_L(NV, 1, 8) SDI_L(NV, 2, 8)
  if (nvmax <= 4) {
    SDI_NV(4)
  } else if (nvmax <= 6) {
    SDI_NV(6)
  } else if (nvmax <= 8) {
    SDI_NV(8)
  } else if (nvmax <= 10) {
    SDI_NV(10)
  } else {
    SDI_NV(16)
  }
#undef SDI_NV
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_e7(int nvmax, int mode, int km, bool dd, size_t shmem) {
  int nb = 0;
  if (mode != 1 && dd) {
#define SDI_D(M, K)                                                                                         \
  if (mode == M && km == K)                                                                                 \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<MAXV, 1, K, M, 2, MAXS, true, 0, 1>, \
                                                        BLOCK, shmem) == hipSuccess                         \
               ? nb                                                                                         \
               : 0;
    SDI_D(0, 4) SDI_D(0, 8) SDI_D(2, 4) SDI_D(2, 8)
#undef SDI_D
    return 0;
  }
#define SDI_O(NV, M, K)                                                                                    \
  if (mode == M && km == K) {                                                                              \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<NV, 1, K, M, 4, MAXS, false, 0, 1>, \
                                                     BLOCK, shmem) != hipSuccess)                          \
      return 0;                                                                                            \
    return nb;                                                                                             \
  }
#define SDI_NV(NV) SDI_O(NV, 0, 4) SDI_O(NV, 1, 4) SDI_O(NV, 2, 4) SDI_O(NV, 0, 8) SDI_O(NV, 1, 8) SDI_O(NV, 2, 8)
  if (nvmax <= 4) {
    SDI_NV(4)
  } else if (nvmax <= 6) {
    SDI_NV(6)
  } else if (nvmax <= 8) {
    SDI_NV(8)
  } else if (nvmax <= 10) {
    SDI_NV(10)
  } else {
    SDI_NV(16)
  }
#undef SDI_NV
#undef SDI_O
  return 0;
}

}  // namespace sdi
