// Endpoint-precision instances of the complex-mode tile kernel: final pass on
// lattice points (mode 0) or a learned sampler's explicit points (mode 2),
// sectors of up to 8 variables, one point per thread; points closer to a
// singular face than the small_x parameter are evaluated again in
// double-double.
#include "kernels.h"
#include "tiles_cplx.hpp"

namespace sdi {

int launch_tiles_cplx_dd(int km, int grid, size_t shmem, const TileArgs& a, const CplxArgs& X, hipStream_t st) {
#define SDI_L(M, K)                                                                          \
  if (a.mode == M && km == K) {                                                              \
    k_tiles_cplx<8, 1, K, M, 1, true><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a, X);         \
    return (int)hipGetLastError();                                                           \
  }
  SDI_L(0, 4) SDI_L(0, 8) SDI_L(2, 4) SDI_L(2, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_cplx_dd(int mode, int km, size_t shmem) {
  int nb = 0;
#define SDI_O(M, K)                                                                                        \
  if (mode == M && km == K)                                                                                \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_cplx<8, 1, K, M, 1, true>, BLOCK,      \
                                                        shmem) == hipSuccess                               \
               ? nb                                                                                        \
               : 0;
  SDI_O(0, 4) SDI_O(0, 8) SDI_O(2, 4) SDI_O(2, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
