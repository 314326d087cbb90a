// Monte Carlo points for the final pass (integrator 2): the pseudo-random
// counterpart of the lattice, the sampling of the paper's default final
// integrator (vegasCuba, section 4.4: Vegas over pseudo-random points).
//
// Point i of shift r of sector s, caller variable c: Philox4x32-10 (key = the
// seed's two 32-bit halves, counter = (i, c + 16 r, s, 0x4D433031)) gives two
// 32-bit words; their top 52 bits b make u = (b + 1/2) 2^-52, exactly
// representable and inside (0, 1).  Without a Vegas grid x = u and weight 1;
// with one (after warm-up) x and the weight come from the sector's grid as in
// the lattice sampler.  The R shifts are R independent samples, so the error
// estimate of the pass is the usual one over shifts.  Points are written as
// explicit points (caller variable order) for the mode-2 final pass; one wave
// per 64-point chunk, a chunk never spans two tiles.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "eval_real.hpp"
#include "kernels.h"
#include "philox.hpp"

namespace sdi {

__global__ void __launch_bounds__(256) k_mc_points(McArgs A) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
  for (int64_t c = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); c < A.nchunks; c += (int64_t)gridDim.x * wpb) {
    const int t = find_run(A.chunk_prefix, A.nruns, c);
    const PointRun T = A.runs[t];
    const int64_t local = (c - A.chunk_prefix[t]) * 64 + lane;
    if (local >= (int64_t)T.count) continue;
    CSec* S = tape(A.secs) + T.sector;
    const int n = S->n;
    const int nb = S->nbins;
    const bool grid = (S->flags & F_USE_GRID) != 0;
    const double* g = A.grids + S->grid_off;
    const uint32_t shift = (uint32_t)(T.row - S->shift_row);
    const uint32_t i = T.i0 + (uint32_t)local;
    double w = 1.0;
    double* xo = A.x + T.x_off + local * n;
    for (int cj = 0; cj < n; ++cj) {
      uint32_t ctr[4] = {i, (uint32_t)cj + 16u * shift, (uint32_t)T.sector, 0x4D433031u};
      philox4x32_10(ctr, k0, k1);
      const uint64_t b = ((uint64_t)ctr[0] << 20) | (ctr[1] >> 12);
      double u = ((double)b + 0.5) * 0x1p-52;
      if (grid) u = vegas_coord(g + cj * (nb + 1), nb, u, w);
      xo[cj] = u;
    }
    A.w[T.pt_off + local] = w;
  }
}

int launch_mc_points(const McArgs& a, hipStream_t st) {
  if (a.nchunks <= 0) return 0;
  const int64_t waves = a.nchunks;
  const unsigned g = (unsigned)std::min<int64_t>((waves + 3) / 4, 1 << 20);
  k_mc_points<<<dim3(g), dim3(256), 0, st>>>(a);
  return (int)hipGetLastError();
}

}  // namespace sdi
