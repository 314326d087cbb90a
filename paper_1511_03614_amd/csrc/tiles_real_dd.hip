// Final-pass instances of the real-mode tile kernel for the endpoint-precision
// mode: every variable class, one point per thread, and points closer to a
// singular face than the small_x parameter evaluated again in double-double.
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_dd(int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
  if (a.mode != 0) return (int)hipErrorInvalidValue;
  if (km == 4)
    k_tiles_real<MAXV, 1, 4, 0, 2, MAXS, true><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);
  else if (km == 8)
    k_tiles_real<MAXV, 1, 8, 0, 2, MAXS, true><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int occupancy_tiles_real_dd(int km, size_t shmem) {
  int nb = 0;
  const hipError_t e = km == 4
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<MAXV, 1, 4, 0, 2, MAXS, true>, BLOCK, shmem)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<MAXV, 1, 8, 0, 2, MAXS, true>, BLOCK, shmem);
  return e == hipSuccess ? nb : 0;
}

}  // namespace sdi
