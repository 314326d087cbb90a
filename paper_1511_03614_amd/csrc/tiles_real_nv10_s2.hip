// Final-pass instances of the real-mode tile kernel for sectors of up to 10
// variables in problems whose sectors have at most 2 singular variables (the
// smaller per-point arrays leave registers for the 3- and 4-wave variants);
// dd: the endpoint-precision copies (points below small_x again in double-double).
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_nv10_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
  if (a.mode != 0) return (int)hipErrorInvalidValue;
#define SDI_L(P, W, K)                                                                       \
  if (ppt == P && wpe == W && km == K) {                                                     \
    if (dd)                                                                                  \
      k_tiles_real<10, P, K, 0, W, 2, true, 2><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);     \
    else                                                                                     \
      k_tiles_real<10, P, K, 0, W, 2, false, 2><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);           \
    return (int)hipGetLastError();                                                            \
  }
  SDI_L(1, 4, 4) SDI_L(2, 3, 4) SDI_L(2, 4, 4) SDI_L(1, 4, 8) SDI_L(2, 3, 8) SDI_L(2, 4, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_nv10_s2(int ppt, int wpe, int km, bool dd, size_t shmem) {
  int nb = 0;
#define SDI_O(P, W, K)                                                                                     \
  if (ppt == P && wpe == W && km == K) {                                                                   \
    const hipError_t e = dd ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                \
                                  &nb, k_tiles_real<10, P, K, 0, W, 2, true, 2>, BLOCK, shmem)               \
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                \
                                  &nb, k_tiles_real<10, P, K, 0, W, 2, false, 2>, BLOCK, shmem);                    \
    return e == hipSuccess ? nb : 0;                                                                       \
  }
  SDI_O(1, 4, 4) SDI_O(2, 3, 4) SDI_O(2, 4, 4) SDI_O(1, 4, 8) SDI_O(2, 3, 8) SDI_O(2, 4, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
