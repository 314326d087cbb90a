// Learned importance-sampling map on gfx950: piecewise-linear coupling flow
// (Mueller et al., "Neural Importance Sampling", 2019) as a replacement for the
// Vegas grid of the paper's integrator (section 4.4).
//
// The conditioner of every coupling layer is an MLP  in -> 64 -> 64 -> nB*32
// evaluated with bf16 matrix cores (v_mfma_f32_16x16x16_bf16, fp32
// accumulation): one wave evaluates 16 samples, samples are the N dimension of
// every product, so the accumulator layout of one layer (lane l holds rows
// 4(l/16)..+3 of column l%16) is exactly the B-operand layout of the next.
// Softmax runs in fp32, the bin probabilities are renormalised in fp64, and the
// map and its Jacobian are applied in fp64, so the importance weight 1/q is the
// exact Jacobian of the map actually applied and the estimator stays unbiased.
//
// Training (gradient of -sum_i c_i log q(x_i)) runs layer by layer: a forward
// kernel stores every layer's input, then one backward kernel per layer
// recomputes that layer's conditioner, back-propagates through it with matrix
// cores (transposed bf16 weights) and accumulates the weight gradients as
// [rows x samples] x [samples x cols] products over 64-sample chunks staged in
// LDS, in registers that persist over the block's chunks.  Each block writes
// its partial gradient; a fixed-order reduction sums them, so the gradient is
// deterministic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eval_real.hpp"
#include "flow_types.h"
#include "philox.hpp"

namespace sdi {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Round-to-nearest-even fp32 -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x4_t load_bf4(const uint16_t* p) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  bf16x4_t r;
  r[0] = (short)(v.x & 0xFFFF);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFF);
  r[3] = (short)(v.y >> 16);
  return r;
}

__device__ __forceinline__ bf16x4_t pack_bf4(float a, float b, float c, float d) {
  bf16x4_t r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}

__device__ __forceinline__ f32x4_t mfma16(bf16x4_t a, bf16x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Orders LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hidden activations of one layer's conditioner for the wave's 16 samples.
// a0: this lane's 4 inputs (rows 4g..4g+3 of the input column of sample l%16);
// returns a1, a2 (bf16, 4 blocks of 16 rows) and the pre-activations z1, z2.
struct MlpHidden {
  bf16x4_t a1[4], a2[4];
  f32x4_t z1[4], z2[4];
};

__device__ __forceinline__ void mlp_hidden(const uint16_t* __restrict__ bw, const float* __restrict__ P,
                                           const FlowLayerDesc& D, bf16x4_t a0, MlpHidden& o) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma16(load_bf4(bw + D.c1 + (ob * 16 + r) * FL_K1 + 4 * g), a0, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += P[D.b1 + ob * 16 + 4 * g + i];
    o.z1[ob] = acc;
    o.a1[ob] = pack_bf4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = mfma16(load_bf4(bw + D.c2 + (ob * 16 + r) * FL_H + kb * 16 + 4 * g), o.a1[kb], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += P[D.b2 + ob * 16 + 4 * g + i];
    o.z2[ob] = acc;
    o.a2[ob] = pack_bf4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
  }
}

// Logits of transformed variable jj: this lane holds bins 4g..4g+3 (lo) and 16+4g..16+4g+3 (hi).
__device__ __forceinline__ void mlp_logits(const uint16_t* __restrict__ bw, const float* __restrict__ P,
                                           const FlowLayerDesc& D, const MlpHidden& h, int jj, f32x4_t& lo,
                                           f32x4_t& hi) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int ob = 2 * jj + half;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = mfma16(load_bf4(bw + D.c3 + (ob * 16 + r) * FL_H + kb * 16 + 4 * g), h.a2[kb], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += P[D.b3 + ob * 16 + 4 * g + i];
    if (half == 0) lo = acc; else hi = acc;
  }
}

// fp32 softmax over the 32 bins of one sample (4 lanes hold 8 bins each), then
// fp64 renormalisation; returns this lane's 8 probabilities (bin order lo then hi).
__device__ __forceinline__ void softmax_bins(const f32x4_t lo, const f32x4_t hi, double (&q)[8]) {
  float mx = lo[0];
#pragma unroll
  for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fmaxf(lo[i], hi[i]));
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  float e[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    e[i] = expf(lo[i] - mx);
    e[4 + i] = expf(hi[i] - mx);
  }
  double sd = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) sd += (double)e[i];
  sd += __shfl_xor(sd, 16, 64);
  sd += __shfl_xor(sd, 32, 64);
  const double inv = 1.0 / sd;
#pragma unroll
  for (int i = 0; i < 8; ++i) q[i] = (double)e[i] * inv;
}

// Stores this lane's 8 probabilities into the sample's row of 32 (LDS).
__device__ __forceinline__ void store_bins(double* qrow, const double (&q)[8]) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    qrow[4 * g + i] = q[i];
    qrow[16 + 4 * g + i] = q[4 + i];
  }
}

// Forward coupling of one variable: data h -> latent y; bin b, offset alpha, q_b.
__device__ __forceinline__ double forward_bins(const double* qrow, double h, int& b, double& alpha,
                                               double& qb) {
  int bb = (int)(h * FL_NB);
  bb = bb > FL_NB - 1 ? FL_NB - 1 : (bb < 0 ? 0 : bb);
  alpha = h * FL_NB - bb;
  double cb = 0.0;
  for (int k = 0; k < bb; ++k) cb += qrow[k];
  qb = qrow[bb];
  b = bb;
  return cb + alpha * qb;
}

// This lane's 4 conditioner inputs a0 = bf16(2 h_A - 1) (rows 4g..4g+3).
__device__ __forceinline__ bf16x4_t layer_input(const FlowLayerDesc& D, const double* h) {
  const int g = (threadIdx.x & 63) >> 4;
  float in[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = 4 * g + i;
    in[i] = k < D.nA ? (float)(2.0 * h[D.A[k < FL_MAXB ? k : 0]] - 1.0) : 0.f;
  }
  return pack_bf4(in[0], in[1], in[2], in[3]);
}

// ---------------------------------------------------------------- sampling
//
// The sampler runs one 64-sample chunk per wave with lane = sample: the
// sample's state h (fp64) stays in registers, the conditioner's products take
// the 64 samples as four 16-column tiles (so each weight operand is loaded
// once per 64 samples), the hidden products use the K = 32 matrix-core
// instruction, and the 32 logits of a transformed variable are moved through
// LDS so that each lane finishes its own sample's softmax, bin search and
// Jacobian without cross-lane traffic.

typedef __bf16 bfv4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bfv8_t __attribute__((ext_vector_type(8)));

constexpr int FL_LGS = 36;   // floats per sample row of the wave's logit buffer (32 used)
constexpr int FL_A0S = 12;   // bf16 per sample row of the staged conditioner inputs (8 used)

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
__device__ __forceinline__ bfv4_t relu_bf4(f32x4_t v, float4 b) {
  bfv4_t o;
  o[0] = (__bf16)fmaxf(v[0] + b.x, 0.f);
  o[1] = (__bf16)fmaxf(v[1] + b.y, 0.f);
  o[2] = (__bf16)fmaxf(v[2] + b.z, 0.f);
  o[3] = (__bf16)fmaxf(v[3] + b.w, 0.f);
  return o;
}
__device__ __forceinline__ float4 ld_f4(const float* p) { return *reinterpret_cast<const float4*>(p); }

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

// Weight operand of the K = 32 products for output rows ob*16.. and inputs
// 32c..32c+31 of a [rows][64] bf16 matrix.  Within a K = 32 step the lane of
// group g supplies inputs 32c + 4g + (0..3) and 32c + 16 + 4g + (0..3): the
// same order in which the previous layer's accumulators (rows 4g..4g+3 of two
// 16-row blocks) feed the activation operand, so no data moves between layers.
__device__ __forceinline__ bfv8_t w_k32(const uint16_t* W, int ob, int c) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const uint16_t* row = W + (ob * 16 + r) * FL_H + 32 * c + 4 * g;
  return cat8(ld_bfv4(row), ld_bfv4(row + 16));
}

// LDS of one sampling wave: the logit buffer (also the staging area of the
// conditioner inputs) and the 64 sample states, one padded row per lane so
// that lanes indexing the same variable hit distinct banks.
template <int NV>
struct FlowWaveLds {
  float lg[64 * FL_LGS];
  double h[64 * (NV + 1)];
};

// Inverse of all coupling layers for the wave's 64 samples (all lanes call it
// together).  h: this lane's sample row in LDS, latent on entry, data point on
// return; lq: log q of the sample.  lds: the wave's logit buffer.
template <int NV>
__device__ __forceinline__ void flow_inverse_wave(const SDI_TAPE FlowSecDesc* F, const float* __restrict__ P,
                                                  const uint16_t* __restrict__ bw, double* h, float* lds,
                                                  double& lq) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  __bf16* a0s = reinterpret_cast<__bf16*>(lds);
  const int n = F->n;
  lq = 0.0;
  for (int l = FL_L - 1; l >= 0; --l) {
    const SDI_TAPE FlowLayerDesc* D = &F->layer[l];
    const int nA = D->nA, nB = D->nB;
    // conditioner inputs bf16(2 h_A - 1), staged so that every lane can read
    // the 4-row slices of the four sample tiles.  The coupling masks are the
    // parity masks, so input k is variable 2k + 1 - (l mod 2).
    {
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
    }
    wave_sync();
    bfv4_t b0[4];
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
    // hidden layers
    bfv4_t a1[4][4], a2[4][4];   // [sample tile][row block]
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      const bfv4_t w = ld_bfv4(bw + D->c1 + (ob * 16 + r) * FL_K1 + 4 * g);
      const float4 b = ld_f4(P + D->b1 + ob * 16 + 4 * g);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) a1[nt][ob] = relu_bf4(mfma16b(w, b0[nt], f32x4_t{0.f, 0.f, 0.f, 0.f}), b);
    }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      f32x4_t acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const bfv8_t w = w_k32(bw + D->c2, ob, c);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma32(w, cat8(a1[nt][2 * c], a1[nt][2 * c + 1]), acc[nt]);
      }
      const float4 b = ld_f4(P + D->b2 + ob * 16 + 4 * g);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) a2[nt][ob] = relu_bf4(acc[nt], b);
    }
    for (int jj = 0; jj < nB; ++jj) {
      // logits of variable jj -> LDS [sample][bin]
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int ob = 2 * jj + half;
        f32x4_t acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const bfv8_t w = w_k32(bw + D->c3, ob, c);
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma32(w, cat8(a2[nt][2 * c], a2[nt][2 * c + 1]), acc[nt]);
        }
        const float4 b = ld_f4(P + D->b3 + ob * 16 + 4 * g);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
          *reinterpret_cast<float4*>(lds + (16 * nt + r) * FL_LGS + half * 16 + 4 * g) =
              make_float4(acc[nt][0] + b.x, acc[nt][1] + b.y, acc[nt][2] + b.z, acc[nt][3] + b.w);
      }
      wave_sync();
      float e[FL_NB];
#pragma unroll
      for (int k = 0; k < FL_NB; k += 4) {
        const float4 v = *reinterpret_cast<const float4*>(lds + lane * FL_LGS + k);
        e[k] = v.x;
        e[k + 1] = v.y;
        e[k + 2] = v.z;
        e[k + 3] = v.w;
      }
      wave_sync();
      // softmax: fp32 exponentials, fp64 sums
      float mx = e[0];
#pragma unroll
      for (int k = 1; k < FL_NB; ++k) mx = fmaxf(mx, e[k]);
      double gs[FL_NB / 4];
#pragma unroll
      for (int m = 0; m < FL_NB / 4; ++m) {
#pragma unroll
        for (int i = 0; i < 4; ++i) e[4 * m + i] = exp_nonpos(e[4 * m + i] - mx);
        gs[m] = (((double)e[4 * m] + (double)e[4 * m + 1]) + (double)e[4 * m + 2]) + (double)e[4 * m + 3];
      }
      const double sd = ((gs[0] + gs[1]) + (gs[2] + gs[3])) + ((gs[4] + gs[5]) + (gs[6] + gs[7]));
      const double inv = 1.0 / sd;
      // bin search: the last bin whose running sum is <= y, first over groups of 4 bins
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
    flow_inverse_wave<NV>(F, P, A.bw, h, L.lg, lq);
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
    flow_inverse_wave<NV>(F, A.params + F->base, A.bw, h, L.lg, lq);
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


// Forward direction x -> latent: stores every layer's input, zeroes dl.
__global__ void __launch_bounds__(256) k_flow_fwd_store(FlowBatchArgs A) {
  __shared__ double hs_all[4][16 * 16];
  __shared__ double qs_all[4][16 * FL_NB];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int s = lane & 15, g = lane >> 4;
  double* hs = hs_all[wave];
  double* qs = qs_all[wave];
  const FlowTile T = A.tiles[blockIdx.y];
  const FlowSecDesc* F = A.fs + T.sector;
  const int n = F->n;
  const float* P = A.params + F->base;
  const int64_t groups = ((int64_t)T.count + 15) / 16;
  for (int64_t grp = (int64_t)blockIdx.x * 4 + wave; grp < groups; grp += (int64_t)gridDim.x * 4) {
    const int64_t i = grp * 16 + s;
    const bool valid = i < (int64_t)T.count;
    if (g == 0)
      for (int j = 0; j < 16; ++j) {
        hs[s * 16 + j] = (valid && j < n) ? A.x[T.x_off + i * n + j] : 0.5;
        if (valid && j < n) A.dl[T.x_off + i * n + j] = 0.0;
      }
    wave_sync();
    for (int l = 0; l < FL_L; ++l) {
      const FlowLayerDesc& D = F->layer[l];
      if (valid && g == 0)
        for (int j = 0; j < n; ++j) A.hsave[T.x_off * FL_L + (i * FL_L + l) * n + j] = hs[s * 16 + j];
      MlpHidden hid;
      mlp_hidden(A.bw, P, D, layer_input(D, hs + s * 16), hid);
      for (int jj = 0; jj < D.nB; ++jj) {
        f32x4_t lo, hi;
        mlp_logits(A.bw, P, D, hid, jj, lo, hi);
        double q[8];
        softmax_bins(lo, hi, q);
        store_bins(qs + s * FL_NB, q);
        wave_sync();
        const int j = D.B[jj];
        int b;
        double alpha, qb;
        const double y = forward_bins(qs + s * FL_NB, hs[s * 16 + j], b, alpha, qb);
        wave_sync();
        if (g == 0) hs[s * 16 + j] = y;
        wave_sync();
      }
    }
  }
}

// LDS operand tile of the weight-gradient products: [row][64 samples + pad] bf16.
__device__ __forceinline__ void put_block(uint16_t* base, int row0, int col, const float (&v)[4]) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) base[(row0 + 4 * g + i) * FL_LS + col] = f2bf(v[i]);
}

// Accumulates tiles  acc[q] += G[rb*16.., :] x Act[cb*16.., :]^T  over the 64
// samples of the chunk; this wave owns tiles t = wave + 4q.
template <int MAXT>
__device__ __forceinline__ void grad_tiles(const uint16_t* G, const uint16_t* Act, int ncb, int ntiles,
                                           f32x4_t (&acc)[MAXT]) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = wave + 4 * q;
    if (t < ntiles) {
      const int rb = t / ncb, cb = t % ncb;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        acc[q] = mfma16(load_bf4(G + (rb * 16 + r) * FL_LS + ks * 16 + 4 * g),
                        load_bf4(Act + (cb * 16 + r) * FL_LS + ks * 16 + 4 * g), acc[q]);
    }
  }
}

// Writes a wave's accumulated tiles to the block's partial gradient: column
// c < ncols goes to W[row][c] (offset w, row stride ncols), column bias_col to b[row].
template <int MAXT>
__device__ __forceinline__ void flush_tiles(float* part, const f32x4_t (&acc)[MAXT], int ncb, int ntiles,
                                            int64_t w, int ncols, int64_t b, int bias_col) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = wave + 4 * q;
    if (t < ntiles) {
      const int rb = t / ncb, cb = t % ncb;
      const int col = cb * 16 + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb * 16 + 4 * g + i;
        if (col < ncols) part[w + (int64_t)row * ncols + col] = acc[q][i];
        else if (col == bias_col) part[b + row] = acc[q][i];
      }
    }
  }
}

// Backward through one coupling layer for one tile (sector batch) per blockIdx.y;
// block x of gridDim.x takes a contiguous range of 64-sample chunks.
__global__ void __launch_bounds__(256) k_flow_bwd_layer(FlowBatchArgs A) {
  constexpr int MAXT3 = (FL_MAXO / 16) * 5 / 4;   // W3 tiles per wave: (nO/16) x 5 column blocks
  constexpr int MAXT2 = 5;                        // W2: 4 x 5 tiles over 4 waves
  __shared__ double qs_all[4][16 * FL_NB];
  __shared__ __attribute__((aligned(16))) uint16_t R[(FL_MAXO + 80) * FL_LS];  // operand tiles per stage
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int s = lane & 15, g = lane >> 4;
  double* qs = qs_all[wave];
  const FlowTile T = A.tiles[blockIdx.y];
  const FlowSecDesc* F = A.fs + T.sector;
  const int n = F->n;
  const int l = A.layer;
  const FlowLayerDesc& D = F->layer[l];
  const float* P = A.params + F->base;
  const int nA = D.nA, nB = D.nB;
  const int nA1 = nA > 0 ? nA : 1;
  const int nO = nB * FL_NB;
  const int nt3 = (nO / 16) * 5, nt2 = 20, nt1 = 4;
  f32x4_t acc3[MAXT3], acc2[MAXT2], acc1[1];
#pragma unroll
  for (int q = 0; q < MAXT3; ++q) acc3[q] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < MAXT2; ++q) acc2[q] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  acc1[0] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int64_t nchunks = ((int64_t)T.count + FL_CHUNK - 1) / FL_CHUNK;
  const int64_t per = (nchunks + gridDim.x - 1) / gridDim.x;
  const int64_t c0 = (int64_t)blockIdx.x * per;
  const int64_t c1 = c0 + per < nchunks ? c0 + per : nchunks;
  const int col = wave * 16 + s;          // this sample's column in the operand tiles
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int64_t i = ch * FL_CHUNK + col;
    const bool valid = i < (int64_t)T.count;
    const int64_t ii = valid ? i : 0;       // padding samples read sample 0 and contribute zero
    const double cw = valid ? A.c[T.pt_off + i] : 0.0;
    const double* hin = A.hsave + T.x_off * FL_L + (ii * FL_L + l) * n;
    double* dli = A.dl + T.x_off + ii * n;
    const bf16x4_t a0 = layer_input(D, hin);
    MlpHidden hid;
    mlp_hidden(A.bw, P, D, a0, hid);
    // stage 3: logit gradients -> G3 (rows 0..nO-1), activations a2 + ones row -> A2 (80 rows)
    uint16_t* G3 = R;
    uint16_t* A2 = R + nO * FL_LS;
    for (int jj = 0; jj < nB; ++jj) {
      f32x4_t lo, hi;
      mlp_logits(A.bw, P, D, hid, jj, lo, hi);
      double q[8];
      softmax_bins(lo, hi, q);
      store_bins(qs + s * FL_NB, q);
      wave_sync();
      const int j = D.B[jj];
      int b;
      double alpha, qb;
      const double y = forward_bins(qs + s * FL_NB, hin[j], b, alpha, qb);
      const double dy = valid ? dli[j] : 0.0;
      float v0[4], v1[4];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int m = k < 4 ? 4 * g + k : 16 + 4 * g + (k - 4);
        const double ind = (m < b ? 1.0 : 0.0) + (m == b ? alpha : 0.0);
        const double v = q[k] * dy * (ind - y) - cw * ((m == b ? 1.0 : 0.0) - q[k]);
        if (k < 4) v0[k] = (float)v; else v1[k - 4] = (float)v;
      }
      put_block(G3, jj * 32, col, v0);
      put_block(G3, jj * 32 + 16, col, v1);
      wave_sync();
      if (g == 0 && valid) dli[j] = dy * FL_NB * qb;
      wave_sync();
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const float v[4] = {bf2f((uint16_t)hid.a2[kb][0]), bf2f((uint16_t)hid.a2[kb][1]),
                          bf2f((uint16_t)hid.a2[kb][2]), bf2f((uint16_t)hid.a2[kb][3])};
      put_block(A2, kb * 16, col, v);
    }
    {
      const float v[4] = {g == 0 ? 1.f : 0.f, 0.f, 0.f, 0.f};
      put_block(A2, 64, col, v);
    }
    __syncthreads();
    grad_tiles<MAXT3>(G3, A2, 5, nt3, acc3);
    // dz2 = (W3^T dlog) * relu'(z2), the logit gradients read back from G3
    f32x4_t dz2[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
      for (int kb = 0; kb < nO / 16; ++kb) {
        bf16x4_t bt;
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) bt[i4] = (short)G3[(kb * 16 + 4 * g + i4) * FL_LS + col];
        acc = mfma16(load_bf4(A.bw + D.t3 + (mb * 16 + s) * nO + kb * 16 + 4 * g), bt, acc);
      }
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4) acc[i4] = hid.z2[mb][i4] > 0.f ? acc[i4] : 0.f;
      dz2[mb] = acc;
    }
    __syncthreads();
    // stage 2: G2 = dz2 (rows 0..63), A1 = a1 + ones row (80 rows)
    uint16_t* G2 = R;
    uint16_t* A1 = R + 64 * FL_LS;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const float v[4] = {dz2[mb][0], dz2[mb][1], dz2[mb][2], dz2[mb][3]};
      put_block(G2, mb * 16, col, v);
      const float a[4] = {bf2f((uint16_t)hid.a1[mb][0]), bf2f((uint16_t)hid.a1[mb][1]),
                          bf2f((uint16_t)hid.a1[mb][2]), bf2f((uint16_t)hid.a1[mb][3])};
      put_block(A1, mb * 16, col, a);
    }
    {
      const float v[4] = {g == 0 ? 1.f : 0.f, 0.f, 0.f, 0.f};
      put_block(A1, 64, col, v);
    }
    __syncthreads();
    grad_tiles<MAXT2>(G2, A1, 5, nt2, acc2);
    // dz1 = (W2^T dz2) * relu'(z1)
    f32x4_t dz1[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        acc = mfma16(load_bf4(A.bw + D.t2 + (mb * 16 + s) * FL_H + kb * 16 + 4 * g),
                     pack_bf4(dz2[kb][0], dz2[kb][1], dz2[kb][2], dz2[kb][3]), acc);
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4) acc[i4] = hid.z1[mb][i4] > 0.f ? acc[i4] : 0.f;
      dz1[mb] = acc;
    }
    __syncthreads();
    // stage 1: G1 = dz1 (rows 0..63), A0 = inputs (rows 0..nA-1) and ones (row 15)
    uint16_t* G1 = R;
    uint16_t* A0 = R + 64 * FL_LS;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const float v[4] = {dz1[mb][0], dz1[mb][1], dz1[mb][2], dz1[mb][3]};
      put_block(G1, mb * 16, col, v);
    }
    {
      float a[4];
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4) a[i4] = (4 * g + i4 == 15) ? 1.f : bf2f((uint16_t)a0[i4]);
      put_block(A0, 0, col, a);
    }
    __syncthreads();
    grad_tiles<1>(G1, A0, 1, nt1, acc1);
    // input gradient: dh_A += 2 W1^T dz1 (the lane holds input rows 4g..4g+3 of its sample)
    {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        acc = mfma16(load_bf4(A.bw + D.t1 + s * FL_H + kb * 16 + 4 * g),
                     pack_bf4(dz1[kb][0], dz1[kb][1], dz1[kb][2], dz1[kb][3]), acc);
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4) {
        const int k = 4 * g + i4;
        if (valid && k < nA) dli[D.A[k < FL_MAXB ? k : 0]] += 2.0 * (double)acc[i4];
      }
    }
    __syncthreads();
  }
  float* part = A.part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * A.part_stride;
  const int64_t o = D.w1;
  flush_tiles<MAXT3>(part, acc3, 5, nt3, D.w3 - o, FL_H, D.b3 - o, FL_H);
  flush_tiles<MAXT2>(part, acc2, 5, nt2, D.w2 - o, FL_H, D.b2 - o, FL_H);
  flush_tiles<1>(part, acc1, 1, nt1, D.w1 - o, nA1, D.b1 - o, 15);
}

// grad[layer] of every tile's flow = sum over the tile's block partials, in block order.
__global__ void k_flow_grad_reduce(const FlowSecDesc* fs, const FlowTile* tiles, int layer, const float* part,
                                   int64_t part_stride, int nblk, float* grad) {
  const FlowTile T = tiles[blockIdx.y];
  const FlowSecDesc& F = fs[T.sector];
  const FlowLayerDesc& D = F.layer[layer];
  const int64_t lsize = D.b3 + (int64_t)D.nB * FL_NB - D.w1;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= lsize) return;
  const float* src = part + (size_t)blockIdx.y * nblk * part_stride + p;
  float acc = 0.f;
  for (int b = 0; b < nblk; ++b) acc += src[(size_t)b * part_stride];
  grad[F.base + D.w1 + p] = acc;
}

// Loss weights of one batch per block: c_i = sum_k (|f_k(x_i)|^2 / q_i^2) / S_k,
// S_k the batch total of that order, orders with a zero or non-finite total
// skipped.  f: [pt][K][2] (result orders), lq: log q.
__global__ void __launch_bounds__(256) k_flow_weights(const FlowTile* tiles, int K, const double* f,
                                                      const double* lq, double* c) {
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
      inv[k] = (tot > 0.0 && isfinite(tot)) ? 1.0 / tot : 0.0;
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
