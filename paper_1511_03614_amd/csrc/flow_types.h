// Layout of the learned sampler's parameters and descriptors, shared by the
// host code and the HIP kernels (plain C++).
//
// Per sector one flow of FL_L coupling layers; layer l stores, contiguously
// from offset w1 of the sector's fp32 block: W1 [64][max(nA,1)], b1 [64],
// W2 [64][64], b2 [64], W3 [nB*32][64], b3 [nB*32] (row-major, the
// storage order of the oracle).  bf16 copies of the weights, plain and
// transposed, live in a separate array at the c* and t* offsets.
#pragma once
#include <stdint.h>

#include "sdint_internal.h"

namespace sdi {

constexpr int FL_L = 4;        // coupling layers
constexpr int FL_H = 64;       // hidden units
constexpr int FL_NB = 32;      // bins per transformed variable
constexpr int FL_K1 = 16;      // first-layer input width (padded)
constexpr int FL_MAXB = 8;     // transformed / conditioning variables per layer (n <= 16)
constexpr int FL_CHUNK = 64;   // samples per wave of the sampling and gradient kernels
constexpr int FL_MAXO = FL_MAXB * FL_NB;  // logits per layer at most
constexpr float FL_ZRANGE = 60.f;         // logits are raised to at most this far below the largest

struct FlowLayerDesc {
  int32_t nA, nB;
  int32_t A[FL_MAXB], B[FL_MAXB];  // variable indices (caller order)
  int64_t w1, b1, w2, b2, w3, b3;  // fp32 offsets from the flow's base; W1 is [64][max(nA,1)]
  int64_t c1, c2, c3;              // bf16 copies: W1 padded [64][16], W2 [64][64], W3 [nB*32][64]
  int64_t t1, t2, t3;              // bf16 transposes: W1^T [16][64], W2^T [64][64], W3^T [64][nB*32]
};

struct FlowSecDesc {
  int32_t n, nparam;               // variables, fp32 parameters of this flow
  int64_t base;                    // offset of this flow's fp32 parameters
  FlowLayerDesc layer[FL_L];
};

using FlowTile = PointRun;

struct FlowSampleArgs {
  const FlowSecDesc* fs;     // flow descriptors [nsec]
  const float* params;       // fp32 master parameters (biases are read from here)
  const uint16_t* bw;        // bf16 weight copies
  const double* u;           // [npts][n] latent points
  double* x;                 // [npts][n]
  double* lq;                // [npts]
  int32_t sector;
  int64_t npts;
};

struct FlowTileArgs {
  const FlowSecDesc* fs;
  const float* params;
  const uint16_t* bw;
  const uint64_t* zp;            // [nsec][MAXV] generating vector << (53 - m), caller order
  const uint64_t* shifts;        // [rows][MAXV]
  const FlowTile* tiles;
  const int64_t* chunk_prefix;   // [ntiles + 1], chunks of 64 points
  int32_t ntiles;
  int32_t baker;
  int64_t nchunks;
  double* x;                     // caller-order points at x_off
  double* w;                     // 1 / q at pt_off
  double* lq;                    // log q at pt_off (may be null)
  double* hsave;                 // each layer's input, [(x_off + i * n) * FL_L + l * n + j] (may be null)
};

struct FlowGradArgs {
  const FlowSecDesc* fs;
  const float* params;
  const uint16_t* bw;
  const FlowTile* runs;          // one run per sector: count, x_off, pt_off (row and i0 unused)
  const int64_t* chunk_prefix;   // [nruns + 1], chunks of 64 samples
  int32_t nruns;
  int64_t nchunks;
  const double* x;               // caller-order points at x_off
  const double* c;               // loss weights at pt_off
  double* hsave;                 // layer inputs: [(x_off + i * n) * FL_L + l * n + j]
  int32_t inputs_saved;          // hsave already holds them (written by the sampler)
  float* part;                   // [nchunks][part_stride] per-chunk gradients
  int64_t part_stride;
};

}  // namespace sdi
