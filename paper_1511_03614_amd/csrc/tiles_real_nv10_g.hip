// Final-pass instances of the real-mode tile kernel for sectors of up to 10
// variables in problems whose sectors have 3 or 4 singular variables at most
// (NSM = 3, 4) and at most two regular factors: every polynomial term is
// evaluated once per point by singular support and the corner values are sums
// of the group sums, so the per-corner values of both factors stay in registers
// (16 or 32 per point); points per thread x minimum waves per SIMD as the
// autotuner's candidates.
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_nv10_g(int nsm, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a,
                               hipStream_t st) {
  if (a.mode != 0) return (int)hipErrorInvalidValue;
#define SDI_L(N, P, W, K)                                                                   \
  if (nsm == N && ppt == P && wpe == W && km == K) {                                        \
    k_tiles_real<10, P, K, 0, W, N, false, 2><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);   \
    return (int)hipGetLastError();                                                          \
  }
  SDI_L(3, 1, 2, 4) SDI_L(3, 1, 4, 4) SDI_L(3, 2, 2, 4) SDI_L(3, 2, 3, 4)
  SDI_L(3, 1, 2, 8) SDI_L(3, 1, 4, 8) SDI_L(3, 2, 2, 8) SDI_L(3, 2, 3, 8)
  SDI_L(4, 1, 2, 4) SDI_L(4, 1, 3, 4) SDI_L(4, 2, 1, 4) SDI_L(4, 2, 2, 4)
  SDI_L(4, 1, 2, 8) SDI_L(4, 1, 3, 8) SDI_L(4, 2, 1, 8) SDI_L(4, 2, 2, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_nv10_g(int nsm, int ppt, int wpe, int km, size_t shmem) {
  int nb = 0;
#define SDI_O(N, P, W, K)                                                                            \
  if (nsm == N && ppt == P && wpe == W && km == K) {                                                 \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<10, P, K, 0, W, N, false, 2>, \
                                                     BLOCK, shmem) != hipSuccess)                    \
      return 0;                                                                                      \
    return nb;                                                                                       \
  }
  SDI_O(3, 1, 2, 4) SDI_O(3, 1, 4, 4) SDI_O(3, 2, 2, 4) SDI_O(3, 2, 3, 4)
  SDI_O(3, 1, 2, 8) SDI_O(3, 1, 4, 8) SDI_O(3, 2, 2, 8) SDI_O(3, 2, 3, 8)
  SDI_O(4, 1, 2, 4) SDI_O(4, 1, 3, 4) SDI_O(4, 2, 1, 4) SDI_O(4, 2, 2, 4)
  SDI_O(4, 1, 2, 8) SDI_O(4, 1, 3, 8) SDI_O(4, 2, 1, 8) SDI_O(4, 2, 2, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
