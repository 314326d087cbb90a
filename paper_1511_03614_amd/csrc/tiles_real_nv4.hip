// Instances of the real-mode tile kernel for sectors of up to 4 variables.
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_nv4(int ppt, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
#define SDI_L(P, K)                                                                          \
  if (ppt == P && km == K) {                                                                  \
    k_tiles_real<4, P, K><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);                     \
    return (int)hipGetLastError();                                                            \
  }
  SDI_L(1, 4) SDI_L(2, 4) SDI_L(4, 4) SDI_L(1, 8) SDI_L(2, 8) SDI_L(4, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_nv4(int ppt, int km, size_t shmem) {
  int nb = 0;
#define SDI_O(P, K)                                                                               \
  if (ppt == P && km == K) {                                                                       \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<4, P, K>, BLOCK, shmem) \
        != hipSuccess) return 0;                                                                   \
    return nb;                                                                                     \
  }
  SDI_O(1, 4) SDI_O(2, 4) SDI_O(4, 4) SDI_O(1, 8) SDI_O(2, 8) SDI_O(4, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
