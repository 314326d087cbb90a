// Explicit-point evaluation (justEvaluate) and dispatch of the tile kernel families.
#include "kernels.h"
#include "tiles_real.hpp"

namespace sdi {

int launch_tiles_real_nv4(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv6(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv8(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv10(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv16(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int occupancy_tiles_real_nv4(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv6(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv8(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv10(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv16(int mode, int ppt, int wpe, int km, size_t shmem);

int launch_tiles_real_nv4_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv6_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv8_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv10_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv16_s2(int ppt, int wpe, int km, bool dd, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int occupancy_tiles_real_nv4_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv6_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv8_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv10_s2(int ppt, int wpe, int km, bool dd, size_t shmem);
int occupancy_tiles_real_nv16_s2(int ppt, int wpe, int km, bool dd, size_t shmem);

int launch_tiles_real_nv4_g(int nsm, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv6_g(int nsm, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv8_g(int nsm, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv10_g(int nsm, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int launch_tiles_real_nv16_g(int nsm, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int occupancy_tiles_real_nv4_g(int nsm, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv6_g(int nsm, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv8_g(int nsm, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv10_g(int nsm, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_real_nv16_g(int nsm, int ppt, int wpe, int km, size_t shmem);

int real_family(int nsmax, int nfmax, int mode, bool dd) {
  if (mode != 0 || nfmax > 2) return dd && mode != 1 ? RF_DD : RF_GENERIC;
  if (nsmax <= 2) return RF_S2;
  if (dd) return RF_DD;
  return nsmax == 3 ? RF_G3 : RF_G4;
}

int launch_tiles_real(int nvmax, int nsmax, int nfmax, int ppt, int wpe, int km, int grid, size_t shmem,
                      const TileArgs& a, hipStream_t st) {
  const bool dd = a.mode != 1 && a.small_x > 0.0;
  switch (real_family(nsmax, nfmax, a.mode, dd)) {
    case RF_S2:
      if (nvmax <= 4) return launch_tiles_real_nv4_s2(ppt, wpe, km, dd, grid, shmem, a, st);
      if (nvmax <= 6) return launch_tiles_real_nv6_s2(ppt, wpe, km, dd, grid, shmem, a, st);
      if (nvmax <= 8) return launch_tiles_real_nv8_s2(ppt, wpe, km, dd, grid, shmem, a, st);
      if (nvmax <= 10) return launch_tiles_real_nv10_s2(ppt, wpe, km, dd, grid, shmem, a, st);
      return launch_tiles_real_nv16_s2(ppt, wpe, km, dd, grid, shmem, a, st);
    case RF_G3:
    case RF_G4: {
      const int nsm = nsmax == 3 ? 3 : 4;
      if (nvmax <= 4) return launch_tiles_real_nv4_g(nsm, ppt, wpe, km, grid, shmem, a, st);
      if (nvmax <= 6) return launch_tiles_real_nv6_g(nsm, ppt, wpe, km, grid, shmem, a, st);
      if (nvmax <= 8) return launch_tiles_real_nv8_g(nsm, ppt, wpe, km, grid, shmem, a, st);
      if (nvmax <= 10) return launch_tiles_real_nv10_g(nsm, ppt, wpe, km, grid, shmem, a, st);
      return launch_tiles_real_nv16_g(nsm, ppt, wpe, km, grid, shmem, a, st);
    }
    case RF_DD:
      return launch_tiles_real_dd(km, grid, shmem, a, st);
    default:
      if (nvmax <= 4) return launch_tiles_real_nv4(ppt, wpe, km, grid, shmem, a, st);
      if (nvmax <= 6) return launch_tiles_real_nv6(ppt, wpe, km, grid, shmem, a, st);
      if (nvmax <= 8) return launch_tiles_real_nv8(ppt, wpe, km, grid, shmem, a, st);
      if (nvmax <= 10) return launch_tiles_real_nv10(ppt, wpe, km, grid, shmem, a, st);
      return launch_tiles_real_nv16(ppt, wpe, km, grid, shmem, a, st);
  }
}

int tiles_real_occupancy(int nvmax, int nsmax, int nfmax, int mode, int ppt, int wpe, int km, bool dd,
                         size_t shmem) {
  dd = dd && mode != 1;
  switch (real_family(nsmax, nfmax, mode, dd)) {
    case RF_S2:
      if (nvmax <= 4) return occupancy_tiles_real_nv4_s2(ppt, wpe, km, dd, shmem);
      if (nvmax <= 6) return occupancy_tiles_real_nv6_s2(ppt, wpe, km, dd, shmem);
      if (nvmax <= 8) return occupancy_tiles_real_nv8_s2(ppt, wpe, km, dd, shmem);
      if (nvmax <= 10) return occupancy_tiles_real_nv10_s2(ppt, wpe, km, dd, shmem);
      return occupancy_tiles_real_nv16_s2(ppt, wpe, km, dd, shmem);
    case RF_G3:
    case RF_G4: {
      const int nsm = nsmax == 3 ? 3 : 4;
      if (nvmax <= 4) return occupancy_tiles_real_nv4_g(nsm, ppt, wpe, km, shmem);
      if (nvmax <= 6) return occupancy_tiles_real_nv6_g(nsm, ppt, wpe, km, shmem);
      if (nvmax <= 8) return occupancy_tiles_real_nv8_g(nsm, ppt, wpe, km, shmem);
      if (nvmax <= 10) return occupancy_tiles_real_nv10_g(nsm, ppt, wpe, km, shmem);
      return occupancy_tiles_real_nv16_g(nsm, ppt, wpe, km, shmem);
    }
    case RF_DD:
      return occupancy_tiles_real_dd(mode, km, shmem);
    default:
      if (nvmax <= 4) return occupancy_tiles_real_nv4(mode, ppt, wpe, km, shmem);
      if (nvmax <= 6) return occupancy_tiles_real_nv6(mode, ppt, wpe, km, shmem);
      if (nvmax <= 8) return occupancy_tiles_real_nv8(mode, ppt, wpe, km, shmem);
      if (nvmax <= 10) return occupancy_tiles_real_nv10(mode, ppt, wpe, km, shmem);
      return occupancy_tiles_real_nv16(mode, ppt, wpe, km, shmem);
  }
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
