// Instances of the real-mode tile kernel for sectors of up to 10 variables:
// final pass (mode 0; points per thread x minimum waves per SIMD as the
// autotuner's candidates), Vegas warm-up with histograms (mode 1) and explicit
// points (mode 2), the last two at 4 waves per SIMD.
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

namespace {
// Warm-up instances exist for 1 and 2 points per thread, explicit ones for 1.
void mode_variant(int mode, int& ppt, int& wpe) {
  if (mode == 2) {
    ppt = 1;
    wpe = 4;
  } else if (mode == 1) {
    ppt = ppt > 2 ? 2 : ppt;
    wpe = 4;
  }
}
}  // namespace

int launch_tiles_real_nv10(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st) {
  const int mode = a.mode;
  mode_variant(mode, ppt, wpe);
#define SDI_L(M, P, W, K)                                                                    \
  if (mode == M && ppt == P && wpe == W && km == K) {                                         \
    k_tiles_real<10, P, K, M, W><<<dim3(grid), dim3(BLOCK), shmem, st>>>(a);                  \
    return (int)hipGetLastError();                                                            \
  }
  SDI_L(0, 1, 4, 4) SDI_L(0, 2, 3, 4) SDI_L(0, 2, 4, 4) SDI_L(1, 1, 4, 4) SDI_L(1, 2, 4, 4) SDI_L(2, 1, 4, 4) SDI_L(0, 1, 4, 8) SDI_L(0, 2, 3, 8) SDI_L(0, 2, 4, 8) SDI_L(1, 1, 4, 8) SDI_L(1, 2, 4, 8) SDI_L(2, 1, 4, 8)
#undef SDI_L
  return (int)hipErrorInvalidValue;
}

int occupancy_tiles_real_nv10(int mode, int ppt, int wpe, int km, size_t shmem) {
  int nb = 0;
  mode_variant(mode, ppt, wpe);
#define SDI_O(M, P, W, K)                                                                              \
  if (mode == M && ppt == P && wpe == W && km == K) {                                                   \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_real<10, P, K, M, W>, BLOCK, shmem) \
        != hipSuccess) return 0;                                                                        \
    return nb;                                                                                          \
  }
  SDI_O(0, 1, 4, 4) SDI_O(0, 2, 3, 4) SDI_O(0, 2, 4, 4) SDI_O(1, 1, 4, 4) SDI_O(1, 2, 4, 4) SDI_O(2, 1, 4, 4) SDI_O(0, 1, 4, 8) SDI_O(0, 2, 3, 8) SDI_O(0, 2, 4, 8) SDI_O(1, 1, 4, 8) SDI_O(1, 2, 4, 8) SDI_O(2, 1, 4, 8)
#undef SDI_O
  return 0;
}

}  // namespace sdi
