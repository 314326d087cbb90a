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
#include "eval_real.hpp"

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

// One tape instruction for this lane; R points at the lane's slot 0.
__device__ __forceinline__ void exec_ins(const ExprIns& I, double* R) {
  const int a = I.a, b = I.b;
  double v;
  switch (I.op) {
    case X_CONST: v = I.imm; break;
    case X_ADD: v = R[a * 64] + R[b * 64]; break;
    case X_SUB: v = R[a * 64] - R[b * 64]; break;
    case X_MUL: v = R[a * 64] * R[b * 64]; break;
    case X_DIV: v = R[a * 64] / R[b * 64]; break;
    case X_NEG: v = -R[a * 64]; break;
    case X_LOG: v = log(R[a * 64]); break;
    case X_POWI: v = powi_dev(R[a * 64], I.k); break;
    case X_POW: v = pow(R[a * 64], R[b * 64]); break;
    default: v = __builtin_nan(""); break;
  }
  R[I.dst * 64] = v;
}

__device__ __forceinline__ ExprIns load_ins(CIns* p) {
  ExprIns r;
  r.op = p->op;
  r.dst = p->dst;
  r.a = p->a;
  r.b = p->b;
  r.k = p->k;
  r.imm = p->imm;
  return r;
}

// Runs the tape for one point per lane.  Instructions are fetched eight at a
// time, so their scalar loads are in flight together (a long tape does not fit
// the scalar cache, and one fetch per instruction would wait on L2 each time).
__device__ __forceinline__ double run_expr(CIns* ins, int nins, int out, double* R) {
  int i = 0;
  for (; i + 8 <= nins; i += 8) {
    ExprIns I[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) I[u] = load_ins(ins + i + u);
#pragma unroll
    for (int u = 0; u < 8; ++u) exec_ins(I[u], R);
  }
  for (; i < nins; ++i) {
    const ExprIns I = load_ins(ins + i);
    exec_ins(I, R);
  }
  return R[out * 64];
}

// MODE 0: final pass; MODE 1: warm-up iteration with Vegas histograms.
// Dynamic LDS: [grid n*(nb+1)] [histogram n*nb] [slots nslots*64].
template <int MODE>
__global__ void __launch_bounds__(EXPR_BLOCK) k_tiles_expr(TileArgs A, ExprArgs X) {
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
    double s = 0.0, c = 0.0;
    int nonfin = 0;
    for (uint32_t base = 0; base < td.count; base += EXPR_BLOCK) {
      const uint32_t off = base + (uint32_t)lane;
      const bool act = off < td.count;
      double x[1][MAXV], w[1];
      int bins[1][MAXV];
      make_points<MAXV, 1>(S, zp, sh, lgrid, (uint64_t)td.i0 + (act ? off : 0u), x, w, bins);
#pragma unroll
      for (int j = 0; j < MAXV; ++j)
        if (j < n) R[j * 64] = x[0][j];
      const double v = act ? w[0] * run_expr(tape(X.ins), X.nins, X.out, R) : 0.0;
      two_sum_acc(s, c, v);
      nonfin += isfinite(v) ? 0 : 1;
      if constexpr (MODE == 1) {
        if (act)
#pragma unroll
          for (int j = 0; j < MAXV; ++j)
            if (j < n) atomicAdd(&lhist[(size_t)S->perm[j] * nb + bins[0][j]], v * v);
      }
    }
    double hi = s + c;
    double lo = c - (hi - s);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double h2 = __shfl_xor(hi, o, 64);
      const double l2 = __shfl_xor(lo, o, 64);
      dd_add(hi, lo, h2, l2);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nonfin += __shfl_xor(nonfin, o, 64);
    if (lane == 0) {
      double* out = A.partial + (size_t)tc * KMAX * PART_STRIDE;
      out[0] = hi;
      out[1] = lo;
      out[2] = 0.0;
      out[3] = 0.0;
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

__global__ void __launch_bounds__(EXPR_BLOCK) k_eval_points_expr(EvalArgs A, ExprArgs X) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * EXPR_BLOCK + lane;
  CSec* S = tape(A.sec);
  const int n = S->n;
  double* R = smem + lane;
  for (int j = 0; j < n; ++j) R[j * 64] = i < A.npts ? A.x[i * n + j] : 0.5;
  const double v = run_expr(tape(X.ins), X.nins, X.out, R);
  if (i < A.npts) {
    A.out[2 * i] = v;
    A.out[2 * i + 1] = 0.0;
    if (A.cond) A.cond[i] = 0.0;   // no subtraction sums in a text integrand
  }
}

}  // namespace

size_t expr_slot_bytes(const ExprArgs& x) { return (size_t)x.nslots * 64 * sizeof(double); }

int launch_tiles_expr(int grid, size_t shmem, const TileArgs& a, const ExprArgs& x, hipStream_t st) {
  const size_t sh = shmem + expr_slot_bytes(x);
  if (a.mode == 0)
    k_tiles_expr<0><<<dim3(grid), dim3(EXPR_BLOCK), sh, st>>>(a, x);
  else if (a.mode == 1)
    k_tiles_expr<1><<<dim3(grid), dim3(EXPR_BLOCK), sh, st>>>(a, x);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int tiles_expr_occupancy(int mode, size_t shmem, const ExprArgs& x) {
  int nb = 0;
  const size_t sh = shmem + expr_slot_bytes(x);
  const hipError_t e = mode == 1
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_expr<1>, EXPR_BLOCK, sh)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_expr<0>, EXPR_BLOCK, sh);
  return e == hipSuccess ? nb : 0;
}

int launch_eval_points_expr(const EvalArgs& a, const ExprArgs& x, hipStream_t st) {
  const int64_t blocks = (a.npts + EXPR_BLOCK - 1) / EXPR_BLOCK;
  if (blocks > ((int64_t)1 << 30)) return (int)hipErrorInvalidValue;
  k_eval_points_expr<<<dim3((unsigned)blocks), dim3(EXPR_BLOCK), expr_slot_bytes(x), st>>>(a, x);
  return (int)hipGetLastError();
}

}  // namespace sdi
