// Instances of the real-mode tile kernel for sectors of up to 16 variables:
// final pass (mode 0), Vegas warm-up with histograms (mode 1, at most 2 points
// per thread) and explicit points (mode 2, one point per thread).
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

namespace {
// Warm-up instances exist for 1 and 2 points per thread, explicit ones for 1.
int mode_ppt(int mode, int ppt) { return mode == 2 ? 1 : (mode == 1 && ppt > 2 ? 2 : ppt); }
}  // namespace

int launch_tiles_real_nv16(int ppt, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
  const int mode = a.mode;
  ppt = mode_ppt(mode, ppt);
#define SDI_L(M, P, K)                                                                       \
  if (mode == M && ppt == P && km == K) {                                                    \
    k_tiles_real<16, P, K, M><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);                     \
    return (int)hipGetLastError();                                                            \
  }
  SDI_L(0, 1, 4) SDI_L(0, 2, 4) SDI_L(0, 1, 8) SDI_L(0, 2, 8) SDI_L(1, 1, 4) SDI_L(1, 2, 4) SDI_L(1, 1, 8) SDI_L(1, 2, 8) SDI_L(2, 1, 4) SDI_L(2, 1, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_nv16(int mode, int ppt, int km, size_t shmem) {
  int nb = 0;
  ppt = mode_ppt(mode, ppt);
#define SDI_O(M, P, K)                                                                                \
  if (mode == M && ppt == P && km == K) {                                                             \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<16, P, K, M>, BLOCK, shmem) \
        != hipSuccess) return 0;                                                                       \
    return nb;                                                                                         \
  }
  SDI_O(0, 1, 4) SDI_O(0, 2, 4) SDI_O(0, 1, 8) SDI_O(0, 2, 8) SDI_O(1, 1, 4) SDI_O(1, 2, 4) SDI_O(1, 1, 8) SDI_O(1, 2, 8) SDI_O(2, 1, 4) SDI_O(2, 1, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
