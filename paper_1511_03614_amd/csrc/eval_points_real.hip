// Explicit-point evaluation (justEvaluate) and dispatch of the tile kernel families.
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_nv4(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv6(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv8(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv16(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int occupancy_tiles_real_nv4(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv6(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv8(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv16(int mode, int ppt, int wpe, int km, size_t shmem);

int launch_tiles_real_nv4_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv6_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv8_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv16_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int occupancy_tiles_real_nv4_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv6_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv8_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv16_s2(int ppt, int wpe, int km, bool dd, size_t shmem);

int launch_tiles_real(int nvmax, int nsmax, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a,
                      hipStream_t st) {
  const bool dd = a.mode == 0 && a.small_x > 0.0;
  if (a.mode == 0 && nsmax <= 2) {
    if (nvmax <= 4) return launch_tiles_real_nv4_s2(ppt, wpe, km, dd, grid, shmem, a, st);
    if (nvmax <= 6) return launch_tiles_real_nv6_s2(ppt, wpe, km, dd, grid, shmem, a, st);
    if (nvmax <= 8) return launch_tiles_real_nv8_s2(ppt, wpe, km, dd, grid, shmem, a, st);
    return launch_tiles_real_nv16_s2(ppt, wpe, km, dd, grid, shmem, a, st);
  }
  if (dd) return launch_tiles_real_dd(km, grid, shmem, a, st);
  if (nvmax <= 4) return launch_tiles_real_nv4(ppt, wpe, km, grid, shmem, a, st);
  if (nvmax <= 6) return launch_tiles_real_nv6(ppt, wpe, km, grid, shmem, a, st);
  if (nvmax <= 8) return launch_tiles_real_nv8(ppt, wpe, km, grid, shmem, a, st);
  return launch_tiles_real_nv16(ppt, wpe, km, grid, shmem, a, st);
}

int tiles_real_occupancy(int nvmax, int nsmax, int mode, int ppt, int wpe, int km, bool dd, size_t shmem) {
  dd = dd && mode == 0;
  if (mode == 0 && nsmax <= 2) {
    if (nvmax <= 4) return occupancy_tiles_real_nv4_s2(ppt, wpe, km, dd, shmem);
    if (nvmax <= 6) return occupancy_tiles_real_nv6_s2(ppt, wpe, km, dd, shmem);
    if (nvmax <= 8) return occupancy_tiles_real_nv8_s2(ppt, wpe, km, dd, shmem);
    return occupancy_tiles_real_nv16_s2(ppt, wpe, km, dd, shmem);
  }
  if (dd) return occupancy_tiles_real_dd(km, shmem);
  if (nvmax <= 4) return occupancy_tiles_real_nv4(mode, ppt, wpe, km, shmem);
  if (nvmax <= 6) return occupancy_tiles_real_nv6(mode, ppt, wpe, km, shmem);
  if (nvmax <= 8) return occupancy_tiles_real_nv8(mode, ppt, wpe, km, shmem);
  return occupancy_tiles_real_nv16(mode, ppt, wpe, km, shmem);
}

int launch_eval_points_real(int km, const EvalArgs& a, hipStream_t st) {
  if (a.npts <= 0) return 0;
  const unsigned g = (unsigned)((a.npts + BLOCK - 1) / BLOCK);
  if (km == 4)
    k_eval_points_real<4><<<dim3(g), dim3(BLOCK), 0, st>>>(a);
  else
    k_eval_points_real<8><<<dim3(g), dim3(BLOCK), 0, st>>>(a);
  return (int)hipGetLastError();
}

int launch_eval_tiles_real(int km, int nvmax, const EvalTilesArgs& a, hipStream_t st) {
  if (a.nchunks <= 0) return 0;
  const dim3 g((unsigned)(a.nchunks < (1 << 20) ? a.nchunks : (1 << 20))), b(BLOCK);
#define SDI_E(K, NV) k_eval_tiles_real<K, NV><<<g, b, 0, st>>>(a)
  if (km == 4) {
    if (nvmax <= 4) SDI_E(4, 4); else if (nvmax <= 6) SDI_E(4, 6); else if (nvmax <= 8) SDI_E(4, 8); else SDI_E(4, 16);
  } else {
    if (nvmax <= 4) SDI_E(8, 4); else if (nvmax <= 6) SDI_E(8, 6); else if (nvmax <= 8) SDI_E(8, 8); else SDI_E(8, 16);
  }
#undef SDI_E
  return (int)hipGetLastError();
}

}  // namespace sdi
