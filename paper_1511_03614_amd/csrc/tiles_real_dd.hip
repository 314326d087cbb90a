// Final-pass instances of the real-mode tile kernel for the endpoint-precision
// mode: every variable class, one point per thread, and points closer to a
// singular face than the small_x parameter evaluated again in double-double
// (mode 0: lattice points; mode 2: a learned sampler's explicit points).
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_dd(int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
#define SDI_L(M, K)                                                                        \
  if (a.mode == M && km == K) {                                                            \
    k_tiles_real<MAXV, 1, K, M, 2, MAXS, true><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a); \
    return (int)hipGetLastError();                                                         \
  }
  SDI_L(0, 4) SDI_L(0, 8) SDI_L(2, 4) SDI_L(2, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_dd(int mode, int km, size_t shmem) {
  int nb = 0;
#define SDI_O(M, K)                                                                                            \
  if (mode == M && km == K)                                                                                    \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<MAXV, 1, K, M, 2, MAXS, true>, BLOCK, \
                                                        shmem) == hipSuccess                                   \
               ? nb                                                                                            \
               : 0;
  SDI_O(0, 4) SDI_O(0, 8) SDI_O(2, 4) SDI_O(2, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
