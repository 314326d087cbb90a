// Learned importance-sampling map on gfx950: piecewise-linear coupling flow
// (Mueller et al., "Neural Importance Sampling", 2019) as a replacement for the
// Vegas grid of the paper's integrator (section 4.4).
//
// The conditioner of every coupling layer is an MLP  in -> 64 -> 64 -> nB*32
// evaluated with bf16 matrix cores and fp32 accumulation.  Every kernel here
// runs one 64-sample chunk per wave with lane = sample: the sample's state
// (fp64) stays in the lane's LDS row, and the matrix products take the 64
// samples as four 16-column tiles, so each weight operand is loaded once per
// 64 samples and the accumulator layout of one layer (lane holds rows
// 4g..4g+3 of sample column l%16, g = l/16) is exactly the activation operand
// of the next.  The 32 logits of a transformed variable go through LDS so that
// each lane finishes its own sample's softmax (fp32 exponentials of logits
// held within FL_ZRANGE of the largest, fp64 normalisation), bin search and
// Jacobian (fp64) without cross-lane traffic;
// the importance weight 1/q is the exact Jacobian of the map actually applied,
// so the estimator stays unbiased whatever the network's precision.
//
// Training (gradient of -sum_i c_i log q(x_i)): one wave takes a chunk through
// the forward direction (storing every layer's input), then back through the
// layers.  Weight gradients are products over the chunk's samples; their
// operands need the samples along the K dimension, which a matrix-core
// product with the identity provides: a 16x16 block held in accumulator
// layout, passed as the A operand against B = I, comes back transposed.  Each
// chunk writes its partial gradient; a fixed-order sum over a sector's chunks
// gives a deterministic gradient.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eval_real.hpp"
#include "flow_types.h"
#include "philox.hpp"

namespace sdi {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bfv4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bfv8_t __attribute__((ext_vector_type(8)));
typedef short bf16x4_t __attribute__((ext_vector_type(4)));

constexpr int FL_LGS = 36;   // floats per sample row of the wave's logit buffer (32 used)
constexpr int FL_A0S = 12;   // bf16 per sample row of the staged conditioner inputs (8 used)
constexpr int FL_G3S = 40;   // bf16 per sample row of the staged logit gradients (32 used)

// Round-to-nearest-even fp32 -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Orders LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ f32x4_t mfma32(bfv8_t a, bfv8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4_t mfma16b(bfv4_t a, bfv4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4_t, a), __builtin_bit_cast(bf16x4_t, b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ bfv4_t ld_bfv4(const uint16_t* p) { return *reinterpret_cast<const bfv4_t*>(p); }
__device__ __forceinline__ bfv8_t cat8(bfv4_t a, bfv4_t b) {
  return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}
__device__ __forceinline__ float4 ld_f4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ f32x4_t zero4() { return f32x4_t{0.f, 0.f, 0.f, 0.f}; }
__device__ __forceinline__ bfv4_t relu_bf4(f32x4_t v, float4 b) {
  bfv4_t o;
  o[0] = (__bf16)fmaxf(v[0] + b.x, 0.f);
  o[1] = (__bf16)fmaxf(v[1] + b.y, 0.f);
  o[2] = (__bf16)fmaxf(v[2] + b.z, 0.f);
  o[3] = (__bf16)fmaxf(v[3] + b.w, 0.f);
  return o;
}
// v where the activation is positive (relu'), rounded to bf16.
__device__ __forceinline__ bfv4_t mask_bf4(f32x4_t v, bfv4_t act) {
  bfv4_t o;
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = (__bf16)((float)act[i] > 0.f ? v[i] : 0.f);
  return o;
}

// e^x for x <= 0: 2^t with t = x log2(e), the product split Cody-Waite style
// into its fp32 rounding t and the remainder (x log2(e) - t), which enters as
// the first-order factor 1 + remainder * ln 2.  About one ulp, like expf, in a
// third of the instructions; results below 2^-126 may flush to zero, which
// only drops bins of negligible probability.
__device__ __forceinline__ float exp_nonpos(float x) {
  const float l2e_hi = 1.44269502e+00f;   // log2(e) rounded to fp32
  const float l2e_lo = 1.92596299e-08f;   // log2(e) - l2e_hi
  const float t = x * l2e_hi;
  const float rem = fmaf(x, l2e_hi, -t) + x * l2e_lo;
  return __builtin_amdgcn_exp2f(t) * fmaf(rem, 0.693147182f, 1.0f);
}

// Operand of a K = 32 product for rows ob*16.. and inputs 32c..32c+31 of a
// row-major bf16 matrix with row length ld.  Within a K = 32 step the lane of
// group g supplies inputs 32c + 4g + (0..3) and 32c + 16 + 4g + (0..3): the
// order in which two 16-row accumulator blocks (rows 4g..4g+3 each) feed the
// other operand, so no data moves between layers.
__device__ __forceinline__ bfv8_t w_k32(const uint16_t* W, int ld, int ob, int c) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const uint16_t* row = W + (ob * 16 + r) * ld + 32 * c + 4 * g;
  return cat8(ld_bfv4(row), ld_bfv4(row + 16));
}

// B = I of a 16x16x16 product: the A operand comes back transposed.
__device__ __forceinline__ bfv4_t ident4() {
  const int lane = threadIdx.x & 63;
  const int s = lane & 15, g = lane >> 4;
  bfv4_t o;
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = (__bf16)(4 * g + i == s ? 1.f : 0.f);
  return o;
}
// A 16x16 bf16 block in accumulator layout (lane: rows 4g..4g+3 of column s)
// -> the same block with rows and columns swapped, in the same layout; exact.
__device__ __forceinline__ bfv4_t transpose16(bfv4_t x, bfv4_t id) {
  const f32x4_t d = mfma16b(x, id, zero4());
  bfv4_t o;
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = (__bf16)d[i];
  return o;
}

// ---------------------------------------------------------------- conditioner

// LDS of one wave: the logit buffer (also the staging area of the
// conditioner inputs and of the logit gradients) and a row of fp64 state per
// sample (the gradient kernel adds a row of state gradients), padded so that
// lanes indexing the same variable hit distinct banks.
template <int NV>
struct FlowWaveLds {
  float lg[64 * FL_LGS];
  double h[64 * (NV + 1)];
};
template <int NV>
struct FlowGradLds {
  float lg[64 * FL_LGS];
  double h[64 * (NV + 1)];
  double d[64 * (NV + 1)];
};

// Stages the conditioner inputs bf16(2 h_A - 1) of layer l and returns the
// B-operand slices (rows 4g..4g+3) of the four sample tiles.  The coupling
// masks are the parity masks, so input k is variable 2k + 1 - (l mod 2).
template <int NV>
__device__ __forceinline__ void stage_inputs(const double* h, int nA, int l, float* lds, bfv4_t (&b0)[4]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  __bf16* a0s = reinterpret_cast<__bf16*>(lds);
  const bool odd = (l & 1) != 0;
  bfv4_t v0, v1;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float a = 0.f;
    if (2 * k + 1 < NV && k < nA) a = (float)(2.0 * h[2 * k + (odd ? 0 : 1)] - 1.0);
    if (k < 4) v0[k] = (__bf16)a; else v1[k - 4] = (__bf16)a;
  }
  *reinterpret_cast<bfv4_t*>(a0s + lane * FL_A0S) = v0;
  *reinterpret_cast<bfv4_t*>(a0s + lane * FL_A0S + 4) = v1;
  wave_sync();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    if (g < 2) {
      b0[nt] = *reinterpret_cast<const bfv4_t*>(a0s + (16 * nt + r) * FL_A0S + 4 * g);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) b0[nt][k] = (__bf16)0.f;
    }
  }
  wave_sync();
}

// a1 = bf16(relu(W1 a0 + b1)), [sample tile][row block].
__device__ __forceinline__ void hidden1(const uint16_t* __restrict__ bw, const float* __restrict__ P,
                                        const SDI_TAPE FlowLayerDesc* D, const bfv4_t (&b0)[4],
                                        bfv4_t (&a1)[4][4]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const bfv4_t w = ld_bfv4(bw + D->c1 + (ob * 16 + r) * FL_K1 + 4 * g);
    const float4 b = ld_f4(P + D->b1 + ob * 16 + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) a1[nt][ob] = relu_bf4(mfma16b(w, b0[nt], zero4()), b);
  }
}

// a2 = bf16(relu(W2 a1 + b2)).
__device__ __forceinline__ void hidden2(const uint16_t* __restrict__ bw, const float* __restrict__ P,
                                        const SDI_TAPE FlowLayerDesc* D, const bfv4_t (&a1)[4][4],
                                        bfv4_t (&a2)[4][4]) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4_t acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = zero4();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bfv8_t w = w_k32(bw + D->c2, FL_H, ob, c);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma32(w, cat8(a1[nt][2 * c], a1[nt][2 * c + 1]), acc[nt]);
    }
    const float4 b = ld_f4(P + D->b2 + ob * 16 + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) a2[nt][ob] = relu_bf4(acc[nt], b);
  }
}

// Logits of transformed variable jj (W3 a2 + b3) into the LDS buffer [sample][bin].
__device__ __forceinline__ void logits_to_lds(const uint16_t* __restrict__ bw, const float* __restrict__ P,
                                              const SDI_TAPE FlowLayerDesc* D, const bfv4_t (&a2)[4][4], int jj,
                                              float* lds) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int ob = 2 * jj + half;
    f32x4_t acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = zero4();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bfv8_t w = w_k32(bw + D->c3, FL_H, ob, c);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma32(w, cat8(a2[nt][2 * c], a2[nt][2 * c + 1]), acc[nt]);
    }
    const float4 b = ld_f4(P + D->b3 + ob * 16 + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      *reinterpret_cast<float4*>(lds + (16 * nt + r) * FL_LGS + half * 16 + 4 * g) =
          make_float4(acc[nt][0] + b.x, acc[nt][1] + b.y, acc[nt][2] + b.z, acc[nt][3] + b.w);
  }
}

// exp(z - max) of one logit, with z raised to at most FL_ZRANGE below the
// maximum so that every bin keeps a positive probability (the map's density
// stays positive on the whole cube).
__device__ __forceinline__ float bin_exp(float z, float mx) { return exp_nonpos(fmaxf(z - mx, -FL_ZRANGE)); }

// Softmax of this lane's row of 32 logits: e_k = bin_exp(z_k, max) in fp32,
// gs = fp64 sums of the groups of 4 bins; returns the fp64 total.  The row
// stays in LDS (a bin's e_k can be recomputed from it bit-identically).
__device__ __forceinline__ double lane_softmax(const float* row, float& mx, float (&e)[FL_NB], double (&gs)[FL_NB / 4]) {
#pragma unroll
  for (int k = 0; k < FL_NB; k += 4) {
    const float4 v = *reinterpret_cast<const float4*>(row + k);
    e[k] = v.x;
    e[k + 1] = v.y;
    e[k + 2] = v.z;
    e[k + 3] = v.w;
  }
  mx = e[0];
#pragma unroll
  for (int k = 1; k < FL_NB; ++k) mx = fmaxf(mx, e[k]);
#pragma unroll
  for (int m = 0; m < FL_NB / 4; ++m) {
#pragma unroll
    for (int i = 0; i < 4; ++i) e[4 * m + i] = bin_exp(e[4 * m + i], mx);
    gs[m] = (((double)e[4 * m] + (double)e[4 * m + 1]) + (double)e[4 * m + 2]) + (double)e[4 * m + 3];
  }
  return ((gs[0] + gs[1]) + (gs[2] + gs[3])) + ((gs[4] + gs[5]) + (gs[6] + gs[7]));
}

// Forward coupling of one coordinate h in [0, 1]: bin b = min(floor(h NB),
// NB - 1), offset alpha = h NB - b; returns the unnormalised running sum
// below b (cbu) and e_b, from the group sums and the 4 bins of b's group
// (recomputed from the LDS row).
__device__ __forceinline__ void forward_bin(const float* row, float mx, const double (&gs)[FL_NB / 4], double h,
                                            int& b, double& alpha, double& cbu, double& eb) {
  int bb = (int)(h * FL_NB);
  bb = bb > FL_NB - 1 ? FL_NB - 1 : (bb < 0 ? 0 : bb);
  alpha = h * FL_NB - bb;
  b = bb;
  const int gb = bb >> 2;
  double c = 0.0;
#pragma unroll
  for (int m = 0; m < FL_NB / 4; ++m)
    if (m < gb) c += gs[m];
  const float4 v = *reinterpret_cast<const float4*>(row + 4 * gb);
  const float eg[4] = {bin_exp(v.x, mx), bin_exp(v.y, mx), bin_exp(v.z, mx), bin_exp(v.w, mx)};
  double e = (double)eg[0];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < (bb & 3)) c += (double)eg[i];
    if (i == (bb & 3)) e = (double)eg[i];
  }
  cbu = c;
  eb = e;
}

// ---------------------------------------------------------------- sampling

// Inverse of all coupling layers for the wave's 64 samples (all lanes call it
// together).  h: this lane's state row, latent on entry, data point on
// return; lq: log q of the sample.  hsave (may be null): receives the state
// after each layer l, which is that layer's input in the forward direction,
// at hsave[l * n + j].
template <int NV>
__device__ __forceinline__ void flow_inverse_wave(const SDI_TAPE FlowSecDesc* F, const float* __restrict__ P,
                                                  const uint16_t* __restrict__ bw, double* h, float* lds,
                                                  double& lq, double* hsave) {
  const int lane = threadIdx.x & 63;
  const int n = F->n;
  lq = 0.0;
  for (int l = FL_L - 1; l >= 0; --l) {
    const SDI_TAPE FlowLayerDesc* D = &F->layer[l];
    bfv4_t b0[4], a1[4][4], a2[4][4];
    stage_inputs<NV>(h, D->nA, l, lds, b0);
    hidden1(bw, P, D, b0, a1);
    hidden2(bw, P, D, a1, a2);
    for (int jj = 0; jj < D->nB; ++jj) {
      logits_to_lds(bw, P, D, a2, jj, lds);
      wave_sync();
      float mx, e[FL_NB];
      double gs[FL_NB / 4];
      const double inv = 1.0 / lane_softmax(lds + lane * FL_LGS, mx, e, gs);
      wave_sync();
      // the last bin whose running sum is <= y, first over groups of 4 bins
      const int j = n == 1 ? 0 : 2 * jj + (l & 1);
      const double y = h[j];
      double c = 0.0, cg = 0.0;
      int gsel = 0;
#pragma unroll
      for (int m = 0; m < FL_NB / 4; ++m) {
        if (c * inv <= y) {
          gsel = m;
          cg = c;
        }
        c += gs[m];
      }
      float eg[4] = {e[0], e[1], e[2], e[3]};
#pragma unroll
      for (int m = 1; m < FL_NB / 4; ++m)
        if (gsel == m) {
#pragma unroll
          for (int i = 0; i < 4; ++i) eg[i] = e[4 * m + i];
        }
      int b = 4 * gsel;
      double cb = cg, eb = (double)eg[0];
      c = cg;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (c * inv <= y) {
          b = 4 * gsel + i;
          cb = c;
          eb = (double)eg[i];
        }
        c += (double)eg[i];
      }
      const double qb = eb * inv;
      double frac = (y - cb * inv) / qb;
      frac = frac < 0.0 ? 0.0 : (frac > 1.0 ? 1.0 : frac);
      h[j] = ((double)b + frac) / (double)FL_NB;
      lq += log((double)FL_NB * qb);
    }
    if (hsave)
      for (int j = 0; j < n; ++j) hsave[l * n + j] = h[j];
  }
}

// Latent u -> x, log q for one sector (explicit latent points); one wave per
// block and per 64-sample chunk.
template <int NV>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_flow_sample(FlowSampleArgs A) {
  __shared__ __attribute__((aligned(16))) FlowWaveLds<NV> L;
  const int lane = threadIdx.x;
  double* h = L.h + lane * (NV + 1);
  const SDI_TAPE FlowSecDesc* F = tape(A.fs) + A.sector;
  const int n = F->n;
  const float* P = A.params + F->base;
  const int64_t chunks = (A.npts + 63) / 64;
  for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
    const int64_t i = ch * 64 + lane;
    const bool valid = i < A.npts;
    for (int j = 0; j < n; ++j) h[j] = valid ? A.u[i * n + j] : 0.5;
    double lq;
    flow_inverse_wave<NV>(F, P, A.bw, h, L.lg, lq, nullptr);
    if (valid) {
      for (int j = 0; j < n; ++j) A.x[i * n + j] = h[j];
      A.lq[i] = lq;
    }
    wave_sync();
  }
}

// Shifted-lattice latent points (tent-transformed when baker is set) pushed
// through the flow: the sampler of a pass or of a training batch.  One wave
// per block and per 64-point chunk; a chunk never spans two tiles.
template <int NV>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_flow_sample_tiles(FlowTileArgs A) {
  __shared__ __attribute__((aligned(16))) FlowWaveLds<NV> L;
  const int lane = threadIdx.x;
  double* h = L.h + lane * (NV + 1);
  for (int64_t c = blockIdx.x; c < A.nchunks; c += gridDim.x) {
    const int t = find_run(A.chunk_prefix, A.ntiles, c);
    const FlowTile T = A.tiles[t];
    const SDI_TAPE FlowSecDesc* F = tape(A.fs) + T.sector;
    const int n = F->n;
    const int64_t local = (c - A.chunk_prefix[t]) * FL_CHUNK + lane;
    const bool valid = local < (int64_t)T.count;
    CU64* zp = tape(A.zp) + (size_t)T.sector * MAXV;
    CU64* sh = tape(A.shifts) + (size_t)T.row * MAXV;
    for (int j = 0; j < n; ++j) {
      double u = 0.5;
      if (valid) {
        u = lattice_coord((uint64_t)T.i0 + (uint64_t)local, zp[j], sh[j]);
        if (A.baker) u = tent(u);
      }
      h[j] = u;
    }
    double lq;
    double* hs = (A.hsave && valid) ? A.hsave + (T.x_off + local * n) * FL_L : nullptr;
    flow_inverse_wave<NV>(F, A.params + F->base, A.bw, h, L.lg, lq, hs);
    if (valid) {
      double* xo = A.x + T.x_off + local * n;
      for (int j = 0; j < n; ++j) xo[j] = h[j];
      A.w[T.pt_off + local] = exp(-lq);
      if (A.lq) A.lq[T.pt_off + local] = lq;
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- parameters

// Initial fp32 parameters: W1, W2 uniform in (-1/sqrt(fan_in), 1/sqrt(fan_in))
// from Philox4x32-10 (key = seed, counter = (index within the layer, layer,
// sector, 0x464c4f57)) with 24-bit uniforms; biases and the output layer zero,
// so the initial map is the identity; W1 zero when the layer has no
// conditioning variables.
__global__ void k_flow_init(const FlowSecDesc* fs, int nsec, float* P, uint64_t seed) {
  const int s = blockIdx.y;
  if (s >= nsec) return;
  const FlowSecDesc& F = fs[s];
  for (int l = 0; l < FL_L; ++l) {
    const FlowLayerDesc& D = F.layer[l];
    const int64_t lsize = D.b3 + (int64_t)D.nB * FL_NB - D.w1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lsize;
         i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t off = D.w1 + i;
      int fan = 0;
      if (off >= D.w1 && off < D.b1) fan = D.nA;
      if (off >= D.w2 && off < D.b2) fan = FL_H;
      float v = 0.f;
      if (fan > 0) {
        uint32_t c[4] = {(uint32_t)i, (uint32_t)l, (uint32_t)s, 0x464C4F57u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u = (double)(c[0] >> 8) * 0x1p-24;
        const double sc = 1.0 / sqrt((double)fan);
        v = (float)(sc * (2.0 * u - 1.0));
      }
      P[F.base + off] = v;
    }
  }
}

// bf16 copies (padded row-major and transposed) of every weight matrix of the
// sectors of `runs` (blockIdx.y = run), or of sector blockIdx.y when runs is null.
__global__ void k_flow_copies(const FlowSecDesc* fs, const FlowTile* runs, int nsec, const float* P, uint16_t* bw) {
  const int s = runs ? runs[blockIdx.y].sector : (int)blockIdx.y;
  if (s >= nsec) return;
  const FlowSecDesc& F = fs[s];
  const float* Ps = P + F.base;
  for (int l = 0; l < FL_L; ++l) {
    const FlowLayerDesc& D = F.layer[l];
    const int nA1 = D.nA > 0 ? D.nA : 1;
    const int nO = D.nB * FL_NB;
    const int tot = FL_H * FL_K1 + FL_H * FL_H + nO * FL_H;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
      if (i < FL_H * FL_K1) {
        const int r = i / FL_K1, c = i % FL_K1;
        const uint16_t v = c < nA1 ? f2bf(Ps[D.w1 + r * nA1 + c]) : (uint16_t)0;
        bw[D.c1 + r * FL_K1 + c] = v;
        bw[D.t1 + c * FL_H + r] = v;
      } else if (i < FL_H * FL_K1 + FL_H * FL_H) {
        const int k = i - FL_H * FL_K1;
        const int r = k / FL_H, c = k % FL_H;
        const uint16_t v = f2bf(Ps[D.w2 + k]);
        bw[D.c2 + k] = v;
        bw[D.t2 + c * FL_H + r] = v;
      } else {
        const int k = i - FL_H * FL_K1 - FL_H * FL_H;
        const int r = k / FL_H, c = k % FL_H;
        const uint16_t v = f2bf(Ps[D.w3 + k]);
        bw[D.c3 + k] = v;
        bw[D.t3 + c * nO + r] = v;
      }
    }
  }
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the fp32 master parameters of
// the sectors of `runs` (blockIdx.y = run): moments and update in fp64, each
// stored value rounded to fp32; bc[2 r], bc[2 r + 1] = 1 - beta^t of that
// sector's step count.
__global__ void k_flow_adam(float* P, const float* G, float* M, float* V, const FlowSecDesc* fs,
                            const FlowTile* runs, double lr, const double* bc) {
#pragma clang fp contract(off)
  const FlowSecDesc& F = fs[runs[blockIdx.y].sector];
  const double bc1 = bc[2 * blockIdx.y], bc2 = bc[2 * blockIdx.y + 1];
  const double b1 = 0.9, b2 = 0.999;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < F.nparam;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = F.base + k;
    const double g = (double)G[i];
    const float m = (float)(b1 * (double)M[i] + (1.0 - b1) * g);
    const float v = (float)(b2 * (double)V[i] + (1.0 - b2) * g * g);
    M[i] = m;
    V[i] = v;
    const double mh = (double)m / bc1;
    const double vh = (double)v / bc2;
    P[i] = (float)((double)P[i] - lr * mh / (sqrt(vh) + 1e-8));
  }
}

// ---------------------------------------------------------------- gradient

// A 16x16 fp32 tile in accumulator layout (lane: rows 4g..4g+3 of column s)
// to out[(row0 + 4g + i) * ld + col0 + s], columns below ncol.
__device__ __forceinline__ void put_tile(float* out, int ld, int row0, int col0, int ncol, f32x4_t v) {
  const int lane = threadIdx.x & 63;
  const int s = lane & 15, g = lane >> 4;
  if (col0 + s < ncol) {
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(int64_t)(row0 + 4 * g + i) * ld + col0 + s] = v[i];
  }
}
// Column 0 of such a tile to out[row0 + 4g + i].
__device__ __forceinline__ void put_col0(float* out, int row0, f32x4_t v) {
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) out[row0 + 4 * (lane >> 4) + i] = v[i];
  }
}

// Sum over the chunk's 64 samples of G[row][smp] Act[col][smp] for one 16x16
// block, both factors given transposed (lane: samples 4g..4g+3 of a sample
// tile, of feature s) for the four sample tiles.  With act = the ones column
// (1 in column 0) it gives the row sums of G.
__device__ __forceinline__ f32x4_t smp_product(const bfv4_t (&gT)[4], const bfv4_t (&aT)[4]) {
  const f32x4_t acc = mfma32(cat8(gT[0], gT[1]), cat8(aT[0], aT[1]), zero4());
  return mfma32(cat8(gT[2], gT[3]), cat8(aT[2], aT[3]), acc);
}
__device__ __forceinline__ f32x4_t smp_rowsum(const bfv4_t (&gT)[4], bfv8_t ones) {
  const f32x4_t acc = mfma32(cat8(gT[0], gT[1]), ones, zero4());
  return mfma32(cat8(gT[2], gT[3]), ones, acc);
}

// Per 64-sample chunk of a batch: forward direction x -> latent (storing every
// layer's input), then back through the layers; writes the chunk's gradient of
// -sum_i c_i log q(x_i) (every parameter of the sector's flow) to its row of
// `part`.  Padding samples of a partial chunk carry c = 0 and contribute zero.
// WPE = 1: all 512 registers per lane, no scratch (for batches with fewer
// chunks than SIMDs, where a wave's latency is the step's); WPE = 2: two waves
// per SIMD with some spills (large batches).
template <int NV, int WPE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) k_flow_grad(FlowGradArgs A) {
  __shared__ __attribute__((aligned(16))) FlowGradLds<NV> L;
  const int lane = threadIdx.x;
  const int r = lane & 15, g = lane >> 4;
  double* h = L.h + lane * (NV + 1);
  double* dl = L.d + lane * (NV + 1);
  const bfv4_t id = ident4();
  bfv8_t ones;
#pragma unroll
  for (int i = 0; i < 8; ++i) ones[i] = (__bf16)(r == 0 ? 1.f : 0.f);
  for (int64_t ch = blockIdx.x; ch < A.nchunks; ch += gridDim.x) {
    const int t = find_run(A.chunk_prefix, A.nruns, ch);
    const FlowTile T = A.runs[t];
    const SDI_TAPE FlowSecDesc* F = tape(A.fs) + T.sector;
    const int n = F->n;
    const float* P = A.params + F->base;
    float* part = A.part + ch * A.part_stride;
    const int64_t local = (ch - A.chunk_prefix[t]) * FL_CHUNK + lane;
    const bool valid = local < (int64_t)T.count;
    const double cw = valid ? A.c[T.pt_off + local] : 0.0;
    double* hs = A.hsave + (T.x_off + (valid ? local : 0) * n) * FL_L;
    for (int j = 0; j < n; ++j) {
      h[j] = valid ? A.x[T.x_off + local * n + j] : 0.5;
      dl[j] = 0.0;
    }
    // forward: data -> latent (skipped when the sampler stored the layer inputs)
    for (int l = 0; l < (A.inputs_saved ? 0 : FL_L); ++l) {
      const SDI_TAPE FlowLayerDesc* D = &F->layer[l];
      if (valid)
        for (int j = 0; j < n; ++j) hs[l * n + j] = h[j];
      bfv4_t b0[4], a1[4][4], a2[4][4];
      stage_inputs<NV>(h, D->nA, l, L.lg, b0);
      hidden1(A.bw, P, D, b0, a1);
      hidden2(A.bw, P, D, a1, a2);
      for (int jj = 0; jj < D->nB; ++jj) {
        logits_to_lds(A.bw, P, D, a2, jj, L.lg);
        wave_sync();
        const float* row = L.lg + lane * FL_LGS;
        float mx, e[FL_NB];
        double gs[FL_NB / 4];
        const double inv = 1.0 / lane_softmax(row, mx, e, gs);
        const int j = n == 1 ? 0 : 2 * jj + (l & 1);
        int b;
        double alpha, cbu, eb;
        forward_bin(row, mx, gs, h[j], b, alpha, cbu, eb);
        wave_sync();
        h[j] = cbu * inv + alpha * (eb * inv);
      }
    }
    // backward, layer by layer; dl holds dL/d(state) at the current layer boundary
    for (int l = FL_L - 1; l >= 0; --l) {
      const SDI_TAPE FlowLayerDesc* D = &F->layer[l];
      const int nA = D->nA, nB = D->nB, nO = nB * FL_NB;
      const int nA1 = nA > 0 ? nA : 1;
      for (int j = 0; j < n; ++j) h[j] = valid ? hs[l * n + j] : 0.5;
      bfv4_t b0[4], a2[4][4];
      {
        bfv4_t a1[4][4];
        stage_inputs<NV>(h, nA, l, L.lg, b0);
        hidden1(A.bw, P, D, b0, a1);
        hidden2(A.bw, P, D, a1, a2);
      }
      f32x4_t da2[4][4];   // [row block][sample tile]: W3^T dlogits
#pragma unroll
      for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) da2[ob][nt] = zero4();
      for (int jj = 0; jj < nB; ++jj) {
        logits_to_lds(A.bw, P, D, a2, jj, L.lg);
        wave_sync();
        const float* row = L.lg + lane * FL_LGS;
        float mx, e[FL_NB];
        double gs[FL_NB / 4];
        const double inv = 1.0 / lane_softmax(row, mx, e, gs);
        const int j = n == 1 ? 0 : 2 * jj + (l & 1);
        int b;
        double alpha, cbu, eb;
        forward_bin(row, mx, gs, h[j], b, alpha, cbu, eb);
        const double qb = eb * inv;
        const double y = cbu * inv + alpha * qb;
        const double dy = dl[j];
        // d/dlogit_k of (dy y - c log q_b) = q_k (dy (ind_k - y) + c) - c delta_kb, with
        // ind_k = 1 below b, alpha at b, 0 above; in fp32 (the result is rounded to bf16)
        const float invf = (float)inv;
        const float a_lo = (float)(dy * (1.0 - y) + cw), a_hi = (float)(cw - dy * y);
        const float g_b = (float)(qb * (dy * (alpha - y) + cw) - cw);
        // a logit held at the range bound has no gradient
        const float e_floor = bin_exp(-FL_ZRANGE, 0.f);
        bfv4_t gv[FL_NB / 4];
#pragma unroll
        for (int k = 0; k < FL_NB; ++k) {
          float gk = e[k] * invf * (k < b ? a_lo : a_hi);
          if (k == b) gk = g_b;
          if (e[k] <= e_floor) gk = 0.f;
          gv[k >> 2][k & 3] = (__bf16)gk;
        }
        dl[j] = dy * FL_NB * qb;
        wave_sync();
        __bf16* g3 = reinterpret_cast<__bf16*>(L.lg);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<bfv8_t*>(g3 + lane * FL_G3S + 8 * q) = cat8(gv[2 * q], gv[2 * q + 1]);
        wave_sync();
        bfv4_t glo[4], ghi[4];   // bins 4g..4g+3 and 16+4g..16+4g+3 of sample 16nt + r
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          glo[nt] = *reinterpret_cast<const bfv4_t*>(g3 + (16 * nt + r) * FL_G3S + 4 * g);
          ghi[nt] = *reinterpret_cast<const bfv4_t*>(g3 + (16 * nt + r) * FL_G3S + 16 + 4 * g);
        }
        wave_sync();
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const bfv8_t w = w_k32(A.bw + D->t3, nO, mb, jj);
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) da2[mb][nt] = mfma32(w, cat8(glo[nt], ghi[nt]), da2[mb][nt]);
        }
        bfv4_t gTlo[4], gThi[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          gTlo[nt] = transpose16(glo[nt], id);
          gThi[nt] = transpose16(ghi[nt], id);
        }
        put_col0(part + D->b3, 32 * jj, smp_rowsum(gTlo, ones));
        put_col0(part + D->b3, 32 * jj + 16, smp_rowsum(gThi, ones));
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          bfv4_t aT[4];   // a2 rows 16nb.. transposed
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) aT[nt] = transpose16(a2[nt][nb], id);
          put_tile(part + D->w3, FL_H, 32 * jj, 16 * nb, FL_H, smp_product(gTlo, aT));
          put_tile(part + D->w3, FL_H, 32 * jj + 16, 16 * nb, FL_H, smp_product(gThi, aT));
        }
      }
      // dz2 = (W3^T dlogits) relu'(z2) -> dW2, db2; dz1 = (W2^T dz2) relu'(z1)
      bfv4_t dz2[4][4], dz1[4][4];   // [sample tile][row block]
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) dz2[nt][ob] = mask_bf4(da2[ob][nt], a2[nt][ob]);
      {
        bfv4_t a1[4][4], a1T[4][4];
        hidden1(A.bw, P, D, b0, a1);
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) a1T[ib][nt] = transpose16(a1[nt][ib], id);
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
          bfv4_t gT[4];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) gT[nt] = transpose16(dz2[nt][ob], id);
#pragma unroll
          for (int ib = 0; ib < 4; ++ib) put_tile(part + D->w2, FL_H, 16 * ob, 16 * ib, FL_H, smp_product(gT, a1T[ib]));
          put_col0(part + D->b2, 16 * ob, smp_rowsum(gT, ones));
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          f32x4_t acc[4];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) acc[nt] = zero4();
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const bfv8_t w = w_k32(A.bw + D->t2, FL_H, mb, c);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma32(w, cat8(dz2[nt][2 * c], dz2[nt][2 * c + 1]), acc[nt]);
          }
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) dz1[nt][mb] = mask_bf4(acc[nt], a1[nt][mb]);
        }
      }
      // dW1, db1, and the input gradient 2 W1^T dz1 (a0 = 2 h_A - 1)
      {
        bfv4_t a0T[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) a0T[nt] = transpose16(b0[nt], id);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          bfv4_t gT[4];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) gT[nt] = transpose16(dz1[nt][mb], id);
          put_tile(part + D->w1, nA1, 16 * mb, 0, nA1, smp_product(gT, a0T));
          put_col0(part + D->b1, 16 * mb, smp_rowsum(gT, ones));
        }
        const int par = (l & 1) ? 0 : 1;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          f32x4_t acc = zero4();
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc = mfma32(w_k32(A.bw + D->t1, FL_H, 0, c), cat8(dz1[nt][2 * c], dz1[nt][2 * c + 1]), acc);
          // lane (r, g): conditioning input k = 4g + i of sample 16nt + r
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            if (k < nA) L.d[(16 * nt + r) * (NV + 1) + 2 * k + par] += 2.0 * (double)acc[i];
          }
        }
      }
      wave_sync();
    }
  }
}

// grad of every run's sector = the sum of its chunks' rows of `part`, in chunk order.
__global__ void k_flow_chunk_reduce(const FlowSecDesc* fs, const FlowTile* runs, const int64_t* chunk_prefix,
                                    const float* part, int64_t stride, float* grad) {
  const FlowTile T = runs[blockIdx.y];
  const FlowSecDesc& F = fs[T.sector];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= F.nparam) return;
  float acc = 0.f;
  for (int64_t ch = chunk_prefix[blockIdx.y]; ch < chunk_prefix[blockIdx.y + 1]; ++ch) acc += part[ch * stride + p];
  grad[F.base + p] = acc;
}


// Loss weights of one batch per block: c_i = sum_k w_k (|f_k(x_i)|^2 / q_i^2) / S_k,
// S_k the batch total of that order, orders with a zero or non-finite total
// skipped.  f: [pt][K][2] (result orders), lq: log q, ow: the order weights w_k.
__global__ void __launch_bounds__(256) k_flow_weights(const FlowTile* tiles, int K, const double* f,
                                                      const double* lq, const double* ow, double* c) {
  __shared__ double red[256];
  __shared__ double inv[KMAX];
  const FlowTile T = tiles[blockIdx.x];
  const int64_t cnt = T.count;
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
      const double* fi = f + ((T.pt_off + i) * K + k) * 2;
      const double w2 = exp(-2.0 * lq[T.pt_off + i]);
      acc += (fi[0] * fi[0] + fi[1] * fi[1]) * w2;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double tot = red[0];
      inv[k] = (tot > 0.0 && isfinite(tot)) ? ow[k] / tot : 0.0;
    }
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const double w2 = exp(-2.0 * lq[T.pt_off + i]);
    double ci = 0.0;
    for (int k = 0; k < K; ++k) {
      if (inv[k] == 0.0) continue;
      const double* fi = f + ((T.pt_off + i) * K + k) * 2;
      ci += (fi[0] * fi[0] + fi[1] * fi[1]) * w2 * inv[k];
    }
    c[T.pt_off + i] = ci;
  }
}

// Training shifts: D(seed, sector, row0 + it, j) for a lattice of 2^m points,
// out[(it * nruns + r) * MAXV + j] for the sector of run r (zero beyond its
// variables); the draw is redrawn while it is a multiple of 2^(53-m), as for
// the pass shifts.
__global__ void k_flow_shifts(const FlowSecDesc* fs, const FlowTile* runs, int nruns, int iters, int m,
                              uint64_t seed, uint32_t row0, uint64_t* out) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)iters * nruns * MAXV) return;
  const int j = (int)(gid % MAXV);
  const int r = (int)((gid / MAXV) % nruns);
  const int it = (int)(gid / ((int64_t)MAXV * nruns));
  const int s = runs[r].sector;
  uint64_t d = 0;
  if (j < fs[s].n) {
    const uint64_t mod = 1ull << (53 - m);
    d = 1;
    for (uint32_t t = 0; t < 64u; ++t) {
      uint32_t c[4] = {(uint32_t)j, row0 + (uint32_t)it, (uint32_t)s, t};
      philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
      const uint64_t v = (((uint64_t)c[0] << 21) | ((uint64_t)c[1] >> 11)) & MASK53;
      if (v % mod != 0) {
        d = v;
        break;
      }
    }
  }
  out[gid] = d;
}

}  // namespace sdi
