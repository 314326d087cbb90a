// Kernels for integrands given as text: the persistent tile kernel (final pass
// and Vegas warm-up) and the point evaluator, both running the expression tape.
//
// The tape is read with wave-uniform scalar loads, so each instruction's
// operation is one scalar branch and its slot numbers sit in SGPRs.  A lane's
// slots live in LDS, 64 doubles apart (the 64 lanes of a wave read and write
// consecutive doubles: no bank conflicts); blocks are one wave, so the slots of
// a wave take nslots x 512 bytes.  The tile kernel takes (shift, index range)
// tiles from the same work counter, writes the same per-tile partial sums and
// histograms, and runs under the same reductions as the sector kernels.
#include "kernels.h"
#include "eval_cplx.hpp"

namespace sdi {

typedef const SDI_TAPE ExprIns CIns;

namespace {

// x^k by binary powering of |k|, then one division for k < 0 (as the host folds constants).
__device__ __forceinline__ double powi_dev(double x, int k) {
  unsigned e = k < 0 ? 0u - (unsigned)k : (unsigned)k;
  double r = 1.0, b = x;
  while (e) {
    if (e & 1u) r *= b;
    e >>= 1;
    if (e) b *= b;
  }
  return k < 0 ? 1.0 / r : r;
}

__device__ __forceinline__ double apply_op(int op, double a, double b, int k, double imm) {
  switch (op) {
    case X_CONST: return imm;
    case X_ADD: return a + b;
    case X_SUB: return a - b;
    case X_MUL: return a * b;
    case X_DIV: return a / b;
    case X_NEG: return -a;
    case X_LOG: return log(a);
    case X_POWI: return powi_dev(a, k);
    case X_POW: return pow(a, b);
    default: return 0.0;
  }
}


// Runs the tape for one point per lane; R points at the lane's slot 0.
// Instructions come EXPR_FETCH at a time in one round of scalar loads, and the
// empty asm statements make every word arrive before the first LDS access:
// scalar loads and LDS accesses share one wait counter, so a field the
// compiler loads late (an immediate, say) would otherwise hold up LDS reads.
__device__ __forceinline__ double run_expr(CIns* ins, int nins, int out, double* R) {
  for (int i = 0; i < nins; i += EXPR_FETCH) {
    const SDI_TAPE uint32_t* wp = (const SDI_TAPE uint32_t*)(ins + i);
    uint32_t w[4 * EXPR_FETCH];
#pragma unroll
    for (int q = 0; q < 4 * EXPR_FETCH; ++q) w[q] = wp[q];
#pragma unroll
    for (int q = 0; q < 4 * EXPR_FETCH; ++q) asm volatile("" ::"s"(w[q]));
#pragma unroll
    for (int u = 0; u < EXPR_FETCH; ++u) {
      const uint32_t h = w[4 * u];                     // op, dst, a, b (little endian bytes)
      const int op = h & X_OPMASK;
      if (op == X_NOP) continue;
      const double imm = __builtin_bit_cast(double, (uint64_t)w[4 * u + 2] | ((uint64_t)w[4 * u + 3] << 32));
      const double a = (h & X_IMMA) ? imm : R[((h >> 16) & 0xff) * 64];
      const double b = (h & X_IMMB) ? imm : R[(h >> 24) * 64];
      R[((h >> 8) & 0xff) * 64] = apply_op(op, a, b, (int32_t)w[4 * u + 1], imm);
    }
  }
  return R[out * 64];
}

// a / b by Smith's algorithm (scaled by the larger part of b).
__device__ __forceinline__ cd cdiv_smith(cd a, cd b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return cd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return cd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// Complex tapes: x^k by binary powering, then one reciprocal for k < 0.
__device__ __forceinline__ cd cpowi_dev(cd x, int k) {
  unsigned e = k < 0 ? 0u - (unsigned)k : (unsigned)k;
  cd r = cd{1.0, 0.0}, b = x;
  while (e) {
    if (e & 1u) r = cmul(r, b);
    e >>= 1;
    if (e) b = cmul(b, b);
  }
  return k < 0 ? cdiv_smith(cd{1.0, 0.0}, r) : r;
}

__device__ __forceinline__ cd apply_op_c(int op, cd a, cd b, int k, double imm) {
  switch (op) {
    case X_CONST: return cd{imm, 0.0};
    case X_ADD: return cadd(a, b);
    case X_SUB: return csub(a, b);
    case X_MUL: return cmul(a, b);
    case X_DIV: return cdiv_smith(a, b);
    case X_NEG: return cd{-a.re, -a.im};
    case X_LOG: return clog_mi0(a);
    case X_POWI: return cpowi_dev(a, k);
    case X_POW: return cexp_(cmul(b, clog_mi0(a)));
    case X_IUNIT: return cd{0.0, 1.0};
    default: return cd{0.0, 0.0};
  }
}

// The complex tape for one point per lane: slot s is rows 2s (real part) and
// 2s + 1 (imaginary part) of the lane's LDS column; immediates are real.
__device__ __forceinline__ cd run_expr_c(CIns* ins, int nins, int out, double* R) {
  for (int i = 0; i < nins; i += EXPR_FETCH) {
    const SDI_TAPE uint32_t* wp = (const SDI_TAPE uint32_t*)(ins + i);
    uint32_t w[4 * EXPR_FETCH];
#pragma unroll
    for (int q = 0; q < 4 * EXPR_FETCH; ++q) w[q] = wp[q];
#pragma unroll
    for (int q = 0; q < 4 * EXPR_FETCH; ++q) asm volatile("" ::"s"(w[q]));
#pragma unroll
    for (int u = 0; u < EXPR_FETCH; ++u) {
      const uint32_t h = w[4 * u];
      const int op = h & X_OPMASK;
      if (op == X_NOP) continue;
      const double imm = __builtin_bit_cast(double, (uint64_t)w[4 * u + 2] | ((uint64_t)w[4 * u + 3] << 32));
      const int sa = (h >> 16) & 0xff, sb = h >> 24, sd = (h >> 8) & 0xff;
      const cd a = (h & X_IMMA) ? cd{imm, 0.0} : cd{R[(2 * sa) * 64], R[(2 * sa + 1) * 64]};
      const cd b = (h & X_IMMB) ? cd{imm, 0.0} : cd{R[(2 * sb) * 64], R[(2 * sb + 1) * 64]};
      const cd v = apply_op_c(op, a, b, (int32_t)w[4 * u + 1], imm);
      R[(2 * sd) * 64] = v.re;
      R[(2 * sd + 1) * 64] = v.im;
    }
  }
  return cd{R[(2 * out) * 64], R[(2 * out + 1) * 64]};
}

// Writes the point's coordinates into slots 0 .. n-1 (imaginary parts 0 for a complex tape).
template <bool CPLX>
__device__ __forceinline__ void put_point(double* R, int n, const double (&x)[MAXV]) {
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    if (j >= n) break;
    if constexpr (CPLX) {
      R[(2 * j) * 64] = x[j];
      R[(2 * j + 1) * 64] = 0.0;
    } else {
      R[j * 64] = x[j];
    }
  }
}

template <bool CPLX>
__device__ __forceinline__ cd run_tape(const ExprArgs& X, double* R) {
  if constexpr (CPLX) return run_expr_c(tape(X.ins), X.nins, X.out, R);
  else return cd{run_expr(tape(X.ins), X.nins, X.out, R), 0.0};
}

// MODE 0: final pass; MODE 1: warm-up iteration with Vegas histograms.
// Dynamic LDS: [grid n*(nb+1)] [histogram n*nb] [slots nslots*64].
// CPLX: complex tape (real and imaginary sums, |f|^2 in the histograms).
template <int MODE, bool CPLX>
__global__ void __launch_bounds__(EXPR_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) k_tiles_expr(TileArgs A,
                                                                                               ExprArgs X) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x;
  for (;;) {
    __syncthreads();
    int t = 0;
    if (lane == 0) t = atomicAdd(A.counter, 1);
    const int ti = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
    if (ti >= A.ntiles) return;
    const int tc = A.order[ti];
    const TileDesc td = A.tiles[tc];
    CSec* S = tape(A.secs) + td.sector;
    const int n = S->n;
    const int nb = S->nbins;
    double* lgrid = nullptr;
    double* lhist = nullptr;
    size_t soff = 0;
    if (S->flags & F_USE_GRID) {
      lgrid = smem;
      const double* g = A.grids + S->grid_off;
      for (int i = lane; i < n * (nb + 1); i += EXPR_BLOCK) lgrid[i] = g[i];
      soff = (size_t)n * (nb + 1);
    }
    if constexpr (MODE == 1) {
      lhist = smem + soff;
      for (int i = lane; i < n * nb; i += EXPR_BLOCK) lhist[i] = 0.0;
      soff += (size_t)n * nb;
    }
    double* R = smem + soff + lane;
    __syncthreads();
    CU64* zp = tape(A.zp) + (size_t)td.sector * MAXV;
    CU64* sh = tape(A.shifts) + ((size_t)S->shift_row + td.shift) * MAXV;
    double s = 0.0, c = 0.0, si = 0.0, ci = 0.0;
    int nonfin = 0;
    for (uint32_t base = 0; base < td.count; base += EXPR_BLOCK) {
      const uint32_t off = base + (uint32_t)lane;
      const bool act = off < td.count;
      double x[1][MAXV], w[1];
      int bins[1][MAXV];
      make_points<MAXV, 1>(S, zp, sh, lgrid, (uint64_t)td.i0 + (act ? off : 0u), x, w, bins);
      put_point<CPLX>(R, n, x[0]);
      const cd f = run_tape<CPLX>(X, R);
      const double v = act ? w[0] * f.re : 0.0;
      const double vi = act ? w[0] * f.im : 0.0;
      two_sum_acc(s, c, v);
      if constexpr (CPLX) two_sum_acc(si, ci, vi);
      nonfin += isfinite(v) && isfinite(vi) ? 0 : 1;
      if constexpr (MODE == 1) {
        if (act)
#pragma unroll
          for (int j = 0; j < MAXV; ++j)
            if (j < n) atomicAdd(&lhist[(size_t)S->perm[j] * nb + bins[0][j]], v * v + vi * vi);
      }
    }
    double hi = s + c;
    double lo = c - (hi - s);
    double hi2 = si + ci;
    double lo2 = ci - (hi2 - si);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double h2 = __shfl_xor(hi, o, 64);
      const double l2 = __shfl_xor(lo, o, 64);
      dd_add(hi, lo, h2, l2);
      if constexpr (CPLX) {
        const double h3 = __shfl_xor(hi2, o, 64);
        const double l3 = __shfl_xor(lo2, o, 64);
        dd_add(hi2, lo2, h3, l3);
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nonfin += __shfl_xor(nonfin, o, 64);
    if (lane == 0) {
      double* out = A.partial + (size_t)tc * KMAX * PART_STRIDE;
      out[0] = hi;
      out[1] = lo;
      out[2] = CPLX ? hi2 : 0.0;
      out[3] = CPLX ? lo2 : 0.0;
      A.nonfinite[2 * tc] = nonfin;
      A.nonfinite[2 * tc + 1] = 0;
    }
    if constexpr (MODE == 1) {
      __syncthreads();
      double* gh = A.hist + A.hist_off[tc];
      for (int i = lane; i < n * nb; i += EXPR_BLOCK) gh[i] = lhist[i];
    }
  }
}

template <bool CPLX>
__global__ void __launch_bounds__(EXPR_BLOCK) k_eval_points_expr(EvalArgs A, ExprArgs X) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * EXPR_BLOCK + lane;
  CSec* S = tape(A.sec);
  const int n = S->n;
  double* R = smem + lane;
  double x[MAXV];
  for (int j = 0; j < n; ++j) x[j] = i < A.npts ? A.x[i * n + j] : 0.5;
  put_point<CPLX>(R, n, x);
  const cd v = run_tape<CPLX>(X, R);
  if (i < A.npts) {
    A.out[2 * i] = v.re;
    A.out[2 * i + 1] = v.im;
    if (A.cond) A.cond[i] = 0.0;   // no subtraction sums in a text integrand
  }
}

}  // namespace

size_t expr_slot_bytes(const ExprArgs& x) { return (size_t)x.nslots * (x.cplx ? 2 : 1) * 64 * sizeof(double); }

int launch_tiles_expr(int grid, size_t shmem, const TileArgs& a, const ExprArgs& x, hipStream_t st) {
  const size_t sh = shmem + expr_slot_bytes(x);
  const dim3 g(grid), b(EXPR_BLOCK);
  if (a.mode == 0 && !x.cplx)
    k_tiles_expr<0, false><<<g, b, sh, st>>>(a, x);
  else if (a.mode == 1 && !x.cplx)
    k_tiles_expr<1, false><<<g, b, sh, st>>>(a, x);
  else if (a.mode == 0)
    k_tiles_expr<0, true><<<g, b, sh, st>>>(a, x);
  else if (a.mode == 1)
    k_tiles_expr<1, true><<<g, b, sh, st>>>(a, x);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int tiles_expr_occupancy(int mode, size_t shmem, const ExprArgs& x) {
  int nb = 0;
  const size_t sh = shmem + expr_slot_bytes(x);
  hipError_t e;
  if (x.cplx)
    e = mode == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_expr<1, true>, EXPR_BLOCK, sh)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_expr<0, true>, EXPR_BLOCK, sh);
  else
    e = mode == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_expr<1, false>, EXPR_BLOCK, sh)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_expr<0, false>, EXPR_BLOCK, sh);
  return e == hipSuccess ? nb : 0;
}

int launch_eval_points_expr(const EvalArgs& a, const ExprArgs& x, hipStream_t st) {
  const int64_t blocks = (a.npts + EXPR_BLOCK - 1) / EXPR_BLOCK;
  if (blocks > ((int64_t)1 << 30)) return (int)hipErrorInvalidValue;
  if (x.cplx)
    k_eval_points_expr<true><<<dim3((unsigned)blocks), dim3(EXPR_BLOCK), expr_slot_bytes(x), st>>>(a, x);
  else
    k_eval_points_expr<false><<<dim3((unsigned)blocks), dim3(EXPR_BLOCK), expr_slot_bytes(x), st>>>(a, x);
  return (int)hipGetLastError();
}

}  // namespace sdi
