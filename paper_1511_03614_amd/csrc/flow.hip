// Launchers of the learned-sampler kernels (coupling flow on matrix cores).
#include <algorithm>

#include "flow.hpp"
#include "kernels.h"

namespace sdi {

namespace {
unsigned clamp_grid(int64_t want, int64_t cap) {
  if (want < 1) want = 1;
  return (unsigned)(want < cap ? want : cap);
}
}  // namespace

int launch_flow_init(const FlowSecDesc* fs, int nsec, float* params, uint64_t seed, hipStream_t st) {
  if (nsec <= 0) return 0;
  k_flow_init<<<dim3(32, nsec), dim3(256), 0, st>>>(fs, nsec, params, seed);
  return (int)hipGetLastError();
}

int launch_flow_copies(const FlowSecDesc* fs, const FlowTile* runs, int nruns, int nsec, const float* params,
                       uint16_t* bw, hipStream_t st) {
  const int ny = runs ? nruns : nsec;
  if (ny <= 0) return 0;
  k_flow_copies<<<dim3(32, ny), dim3(256), 0, st>>>(fs, runs, nsec, params, bw);
  return (int)hipGetLastError();
}

int launch_flow_adam(float* params, const float* grad, float* m, float* v, const FlowSecDesc* fs,
                     const FlowTile* runs, int nruns, int64_t max_nparam, double lr, const double* bc,
                     hipStream_t st) {
  if (nruns <= 0) return 0;
  const unsigned gx = (unsigned)std::min<int64_t>(64, (max_nparam + 255) / 256);
  k_flow_adam<<<dim3(gx, nruns), dim3(256), 0, st>>>(params, grad, m, v, fs, runs, lr, bc);
  return (int)hipGetLastError();
}

int launch_flow_sample(const FlowSampleArgs& a, int nvmax, hipStream_t st) {
  if (a.npts <= 0) return 0;
  const dim3 grid(clamp_grid((a.npts + 63) / 64, 1 << 16)), block(64);
  if (nvmax <= 4)
    k_flow_sample<4><<<grid, block, 0, st>>>(a);
  else if (nvmax <= 8)
    k_flow_sample<8><<<grid, block, 0, st>>>(a);
  else
    k_flow_sample<16><<<grid, block, 0, st>>>(a);
  return (int)hipGetLastError();
}

int launch_flow_sample_tiles(const FlowTileArgs& a, int nvmax, hipStream_t st) {
  if (a.nchunks <= 0) return 0;
  const dim3 grid(clamp_grid(a.nchunks, 1 << 22)), block(64);
  if (nvmax <= 4)
    k_flow_sample_tiles<4><<<grid, block, 0, st>>>(a);
  else if (nvmax <= 8)
    k_flow_sample_tiles<8><<<grid, block, 0, st>>>(a);
  else
    k_flow_sample_tiles<16><<<grid, block, 0, st>>>(a);
  return (int)hipGetLastError();
}

int launch_flow_grad(const FlowGradArgs& a, int nvmax, int ncu, hipStream_t st) {
  if (a.nchunks <= 0) return 0;
  const dim3 grid(clamp_grid(a.nchunks, 1 << 22)), block(64);
  // fewer chunks than 2 waves per SIMD: latency decides, take the spill-free instance
  const bool wide = a.nchunks > 8 * (int64_t)(ncu > 0 ? ncu : 256);
#define SDI_G(NV)                                                  \
  if (wide)                                                        \
    k_flow_grad<NV, 2><<<grid, block, 0, st>>>(a);                 \
  else                                                             \
    k_flow_grad<NV, 1><<<grid, block, 0, st>>>(a);
  if (nvmax <= 4) {
    SDI_G(4)
  } else if (nvmax <= 8) {
    SDI_G(8)
  } else {
    SDI_G(16)
  }
#undef SDI_G
  return (int)hipGetLastError();
}

int launch_flow_chunk_reduce(const FlowSecDesc* fs, const FlowTile* runs, const int64_t* chunk_prefix, int nruns,
                             const float* part, int64_t stride, int64_t max_nparam, float* grad, hipStream_t st) {
  if (nruns <= 0) return 0;
  k_flow_chunk_reduce<<<dim3((unsigned)((max_nparam + 255) / 256), nruns), dim3(256), 0, st>>>(
      fs, runs, chunk_prefix, part, stride, grad);
  return (int)hipGetLastError();
}

int launch_flow_weights(const FlowTile* tiles, int ntiles, int K, const double* f, const double* lq, const double* ow,
                        double* c, hipStream_t st) {
  if (ntiles <= 0) return 0;
  k_flow_weights<<<dim3(ntiles), dim3(256), 0, st>>>(tiles, K, f, lq, ow, c);
  return (int)hipGetLastError();
}

int launch_flow_shifts(const FlowSecDesc* fs, const FlowTile* runs, int nruns, int iters, int m, uint64_t seed,
                       uint32_t row0, uint64_t* out, hipStream_t st) {
  const int64_t tot = (int64_t)iters * nruns * MAXV;
  if (tot <= 0) return 0;
  k_flow_shifts<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st>>>(fs, runs, nruns, iters, m, seed, row0,
                                                                           out);
  return (int)hipGetLastError();
}

}  // namespace sdi
