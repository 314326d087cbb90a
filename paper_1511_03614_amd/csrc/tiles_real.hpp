// Persistent multi-sector tile kernel (real mode).
//
// One launch covers every (sector, shift, index range) tile of a pass.  Blocks
// take tiles from an atomic counter in longest-first order; the tile's sector
// record selects, with a wave-uniform switch, the evaluator instance compiled
// for its variable class and number of singular variables.  Each tile writes
// its own partial sums (and, in warm-up, its own Vegas histogram), so the
// result does not depend on which block ran which tile.
#pragma once
#include "eval_dd.hpp"

namespace sdi {

template <int NV, int PPT, int KM, int MODE, int NSM, int MF, int E7M>
__device__ __forceinline__ void run_tile_real(const TileArgs& A, CSec* S,
                                              const TileDesc& td, int tc, const double* __restrict__ lgrid,
                                              double* __restrict__ lhist, double (&s)[KM],
                                              double (&c)[KM], int& nonfin) {
  const uint32_t step = (uint32_t)blockDim.x * PPT;
  for (uint32_t off = threadIdx.x * PPT; off < td.count; off += step) {
    // Re-read the sector record every iteration instead of pinning all of it in
    // SGPRs for the whole tile (scalar loads are cheap and cached).
    asm volatile("" ::: "memory");
    CU64* zp = tape(A.zp) + (size_t)td.sector * MAXV;
    CU64* sh = tape(A.shifts) + ((size_t)S->shift_row + td.shift) * MAXV;
    double x[PPT][NV], w[PPT];
    int bins[PPT][NV];
    if constexpr (MODE == 2) {
      static_assert(PPT == 1, "explicit points are read one per thread");
      {
        // explicit points (a learned sampler): caller order, weight 1/q
        const int n = S->n;
        const double* xp = A.px + A.x_off[tc] + (size_t)off * n;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          x[0][j] = j < n ? xp[S->perm[j]] : 0.5;
          bins[0][j] = 0;
        }
        w[0] = A.pw[A.pt_off[tc] + off];
      }
    } else {
      make_points<NV, PPT>(S, zp, sh, lgrid, (uint64_t)td.i0 + off, x, w, bins);
    }
    double f[PPT][KM];
    eval_f_real<NV, PPT, KM, NSM, MF, E7M>(S, tape(A.terms), x, f);
    const int kf = S->kf;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      bool bad = false;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const double v = w[p] * f[p][k];
        two_sum_acc(s[k], c[k], v);
        bad |= !isfinite(v);
      }
      nonfin += bad ? 1 : 0;
      if constexpr (MODE == 1) {
        const int n = S->n;
        const int nb = S->nbins;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (k < kf) {
            const double v = w[p] * f[p][k];
#pragma unroll
            for (int j = 0; j < NV; ++j)
              if (j < n) atomicAdd(&lhist[((size_t)S->perm[j] * nb + bins[p][j]) * kf + k], v * v);
          }
        }
      }
    }
  }
}

// Final-pass tile of the endpoint-precision instances.  Points whose smallest
// singular coordinate is below A.small_x are not accumulated where they are
// sampled: each wave queues their offsets in LDS (ballot and prefix count, all
// control flow wave-uniform), and once 64 are queued the 64 lanes evaluate one
// each in double-double and add it to their own sums (compensated, so the
// order does not matter).  A flagged point thus costs one lane of a full
// double-double call instead of holding its whole wave in one.  q: this
// wave's DDQ_CAP entries.  MODE 2 (explicit points of a learned sampler)
// queues the point's offset in the tile's point list the same way.

// One point per lane for the endpoint-precision instances: lattice point
// td.i0 + off (MODE 0) or the tile's explicit point off (MODE 2).
template <int NV, int MODE>
__device__ __forceinline__ void load_point_real(const TileArgs& A, CSec* S, const TileDesc& td, int tc,
                                                const double* __restrict__ lgrid, uint32_t off, double (&x)[1][NV],
                                                double (&w)[1]) {
  if constexpr (MODE == 2) {
    const int n = S->n;
    const double* xp = A.px + A.x_off[tc] + (size_t)off * n;
#pragma unroll
    for (int j = 0; j < NV; ++j) x[0][j] = j < n ? xp[S->perm[j]] : 0.5;
    w[0] = A.pw[A.pt_off[tc] + off];
  } else {
    CU64* zp = tape(A.zp) + (size_t)td.sector * MAXV;
    CU64* sh = tape(A.shifts) + ((size_t)S->shift_row + td.shift) * MAXV;
    int bins[1][NV];
    make_points<NV, 1>(S, zp, sh, lgrid, (uint64_t)td.i0 + off, x, w, bins);
  }
}

template <int NV, int KM, int MODE>
__device__ __forceinline__ void dd_flush(const TileArgs& A, CSec* S, const TileDesc& td, int tc,
                                         const double* __restrict__ lgrid, const uint32_t* q, int cnt,
                                         double (&s)[KM], double (&c)[KM], int& nonfin) {
  const int lane = threadIdx.x & 63;
  if (lane < cnt) {
    double x[1][NV], w[1];
    load_point_real<NV, MODE>(A, S, td, tc, lgrid, q[lane], x, w);
    double f[KM], cd[KM];
    eval_f_real_dd<KM>(S, tape(A.terms), x[0], f, cd);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const double v = w[0] * f[k];
      two_sum_acc(s[k], c[k], v);
      bad |= !isfinite(v);
    }
    nonfin += bad ? 1 : 0;
  }
}

// Explicit points (MODE 2) are read one per thread; lanes past the tile's end
// take a placeholder point that is neither accumulated nor queued.
template <int NV, int PPT, int KM, int MODE, int NSM, int MF, int E7M>
__device__ __forceinline__ void run_tile_real_ddq(const TileArgs& A, CSec* S, const TileDesc& td, int tc,
                                                  const double* __restrict__ lgrid, uint32_t* q,
                                                  double (&s)[KM], double (&c)[KM], int& nonfin) {
  static_assert(MODE != 2 || PPT == 1, "explicit points are read one per thread");
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;   // lanes under this one
  const uint32_t step = (uint32_t)blockDim.x * PPT;
  const int ns = S->ns;
  int qn = 0;   // queued entries of this wave (wave-uniform)
  // every lane runs every iteration (td.count need not be a multiple of step)
  for (uint32_t base = 0; base < td.count; base += step) {
    asm volatile("" ::: "memory");
    const uint32_t off = base + threadIdx.x * PPT;
    double x[PPT][NV], w[PPT];
    if constexpr (MODE == 2) {
      if (off < td.count) {
        load_point_real<NV, 2>(A, S, td, tc, lgrid, off, x, w);
      } else {
#pragma unroll
        for (int j = 0; j < NV; ++j) x[0][j] = 0.5;
        w[0] = 0.0;
      }
    } else {
      CU64* zp = tape(A.zp) + (size_t)td.sector * MAXV;
      CU64* sh = tape(A.shifts) + ((size_t)S->shift_row + td.shift) * MAXV;
      int bins[PPT][NV];
      make_points<NV, PPT>(S, zp, sh, lgrid, (uint64_t)td.i0 + off, x, w, bins);
    }
    double f[PPT][KM];
    eval_f_real<NV, PPT, KM, NSM, MF, E7M>(S, tape(A.terms), x, f);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const bool act = off + (uint32_t)p < td.count;
      const bool flag = act && near_face<NV>(x[p], ns, A.small_x);
      if (act && !flag) {
        bool bad = false;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const double v = w[p] * f[p][k];
          two_sum_acc(s[k], c[k], v);
          bad |= !isfinite(v);
        }
        nonfin += bad ? 1 : 0;
      }
      // queue the flagged points of this round: qn < 64 here, so qn + 64 <= DDQ_CAP
      const uint64_t bal = __ballot(flag);
      if (flag) q[qn + __popcll(bal & below)] = off + (uint32_t)p;
      qn += __popcll(bal);
      if (qn >= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        dd_flush<NV, KM, MODE>(A, S, td, tc, lgrid, q, 64, s, c, nonfin);
        // move the rest (fewer than 64) to the front: lane l reads 64 + l, writes l
        const uint32_t rest = lane < qn - 64 ? q[64 + lane] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < qn - 64) q[lane] = rest;
        qn -= 64;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  if (qn > 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    dd_flush<NV, KM, MODE>(A, S, td, tc, lgrid, q, qn, s, c, nonfin);
  }
}

template <int NV, int PPT, int KM, int MODE, int NSM, bool DD, int MF, int E7M>
__device__ __forceinline__ void run_tile_any(const TileArgs& A, CSec* S, const TileDesc& td, int tc,
                                             const double* __restrict__ lgrid, double* __restrict__ lhist,
                                             uint32_t* q, double (&s)[KM], double (&c)[KM], int& nonfin) {
  if constexpr (DD)
    run_tile_real_ddq<NV, PPT, KM, MODE, NSM, MF, E7M>(A, S, td, tc, lgrid, q, s, c, nonfin);
  else
    run_tile_real<NV, PPT, KM, MODE, NSM, MF, E7M>(A, S, td, tc, lgrid, lhist, s, c, nonfin);
}

// WPE: minimum waves per SIMD the register allocation must allow (the
// autotuner picks it with PPT; occupancy pays more than a few spills here).
// NSM: bound on the singular variables of every sector of the launch (the
// final pass has NSM = 2 instances for problems without deeper poles).
// DD: points closer to a singular face than A.small_x are evaluated again in
// double-double (the final-pass instances of the endpoint-precision mode, on
// lattice points or on a learned sampler's explicit points).
// MF: 0 evaluates each corner's term lists; 2 (problems whose sectors have at
// most two regular factors) evaluates each term once by singular support.
// E7M: 0 for problems whose factor exponents are at most 3, 1 for problems
// with exponents up to 7 (the x^4 bit of the term words; their own instances,
// so that the others carry no code for it).
template <int NVMAX, int PPT, int KM, int MODE, int WPE, int NSM = MAXS, bool DD = false, int MF = 0, int E7M = 0>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) k_tiles_real(TileArgs A) {
  extern __shared__ double smem[];
  __shared__ int s_tile;
  __shared__ int s_nonfin;
  __shared__ double s_red[BLOCK / 64][KM][2];
  __shared__ uint32_t s_q[DD ? (BLOCK / 64) * DDQ_CAP : 1];
  static_assert(!DD || MODE != 1, "endpoint precision is a final-pass mode");
  constexpr int NVC = NVMAX <= 4 ? 0 : (NVMAX <= 8 ? 1 : 2);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      s_tile = atomicAdd(A.counter, 1);
      s_nonfin = 0;
    }
    __syncthreads();
    const int ti = __builtin_amdgcn_readfirstlane(s_tile);
    if (ti >= A.ntiles) return;
    const int tc = A.order[ti];
    const TileDesc td = A.tiles[tc];
    CSec* S = tape(A.secs) + td.sector;
    const int n = S->n;
    const int nb = S->nbins;
    const int kf = S->kf;
    double* lgrid = nullptr;
    double* lhist = nullptr;
    size_t soff = 0;
    if (S->flags & F_USE_GRID) {
      lgrid = smem;
      const double* g = A.grids + S->grid_off;
      for (int i = threadIdx.x; i < n * (nb + 1); i += blockDim.x) lgrid[i] = g[i];
      soff = (size_t)n * (nb + 1);
    }
    if constexpr (MODE == 1) {
      lhist = smem + soff;
      for (int i = threadIdx.x; i < n * nb * kf; i += blockDim.x) lhist[i] = 0.0;
    }
    __syncthreads();

    double s[KM], c[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) { s[k] = 0.0; c[k] = 0.0; }
    int nonfin = 0;
    const int cls = S->cls;
    uint32_t* q = DD ? s_q + (threadIdx.x >> 6) * DDQ_CAP : nullptr;
    switch (cls) {
      case 0:
        run_tile_any<4, PPT, KM, MODE, NSM, DD, MF, E7M>(A, S, td, tc, lgrid, lhist, q, s, c, nonfin);
        break;
      case 1:
        if constexpr (NVMAX == 6)
          run_tile_any<6, PPT, KM, MODE, NSM, DD, MF, E7M>(A, S, td, tc, lgrid, lhist, q, s, c, nonfin);
        else if constexpr (NVC >= 1)
          run_tile_any<8, PPT, KM, MODE, NSM, DD, MF, E7M>(A, S, td, tc, lgrid, lhist, q, s, c, nonfin);
        break;
      case 2:
        if constexpr (NVC >= 2)
          run_tile_any<(NVMAX == 10 ? 10 : 16), PPT, KM, MODE, NSM, DD, MF, E7M>(A, S, td, tc, lgrid, lhist, q, s, c, nonfin);
        break;
      default:
        break;
    }

    // block reduction: double-double sums over lanes, then over waves in order
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      double hi = s[k] + c[k];
      double lo = c[k] - (hi - s[k]);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double h2 = __shfl_xor(hi, o, 64);
        const double l2 = __shfl_xor(lo, o, 64);
        dd_add(hi, lo, h2, l2);
      }
      if (lane == 0) {
        s_red[wave][k][0] = hi;
        s_red[wave][k][1] = lo;
      }
    }
    if (nonfin) atomicAdd(&s_nonfin, nonfin);
    __syncthreads();
    if (threadIdx.x < KM) {
      const int k = threadIdx.x;
      double hi = s_red[0][k][0], lo = s_red[0][k][1];
      for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) dd_add(hi, lo, s_red[wv][k][0], s_red[wv][k][1]);
      double* out = A.partial + ((size_t)tc * KMAX + k) * PART_STRIDE;
      out[0] = hi;
      out[1] = lo;
      out[2] = 0.0;
      out[3] = 0.0;
    }
    if (threadIdx.x == 0) {
      A.nonfinite[2 * tc] = s_nonfin;
      A.nonfinite[2 * tc + 1] = 0;
    }
    if constexpr (MODE == 1) {
      double* gh = A.hist + A.hist_off[tc];
      for (int i = threadIdx.x; i < n * nb * kf; i += blockDim.x) gh[i] = lhist[i];
    }
  }
}

// Values of every result order at caller points (justEvaluate, parity checks).
template <int NV, int KM>
__device__ __forceinline__ void eval_point_real(const EvalArgs& A, int64_t i) {
  CSec* S = tape(A.sec);
  const int n = S->n;
  const int K = S->K;
  double x[1][NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) x[0][j] = j < n ? A.x[i * n + S->perm[j]] : 0.5;
  double f[1][KM], cnd[1][KM];
  if (A.cond)
    eval_f_real_c<NV, 1, KM, true>(S, tape(A.terms), x, f, cnd);
  else
    eval_f_real<NV, 1, KM>(S, tape(A.terms), x, f);
  if (A.small_x > 0.0 && near_face<NV>(x[0], S->ns, A.small_x)) {
    double xd[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) xd[j] = x[0][j];
    eval_f_real_dd<KM>(S, tape(A.terms), xd, f[0], cnd[0]);
  }
  for (int k = 0; k < K; ++k) {
    double fr = 0.0, fi = 0.0, cs = 0.0;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
      fr += S->fold_re[k][kk] * f[0][kk];
      fi += S->fold_im[k][kk] * f[0][kk];
      if (A.cond) cs += hypot(S->fold_re[k][kk], S->fold_im[k][kk]) * cnd[0][kk];
    }
    A.out[(i * K + k) * 2] = fr;
    A.out[(i * K + k) * 2 + 1] = fi;
    if (A.cond) A.cond[i * K + k] = cs;
  }
}

template <int KM>
__global__ void __launch_bounds__(BLOCK) k_eval_points_real(EvalArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.npts) return;
  switch (tape(A.sec)->cls) {
    case 0: eval_point_real<4, KM>(A, i); break;
    case 1: eval_point_real<8, KM>(A, i); break;
    case 2: eval_point_real<16, KM>(A, i); break;
    default: break;
  }
}

// Values of every result order at the explicit points of several sectors;
// NVMAX: the problem's variable class (the 6-variable class needs fewer
// registers than the 8-variable one).
template <int KM, int NVMAX>
__global__ void __launch_bounds__(BLOCK) k_eval_tiles_real(EvalTilesArgs T) {
  for (int64_t c = blockIdx.x; c < T.nchunks; c += gridDim.x) {
    const int r = find_run(T.chunk_prefix, T.nruns, c);
    const PointRun run = T.runs[r];
    const int64_t i = (c - T.chunk_prefix[r]) * BLOCK + threadIdx.x;
    if (i >= (int64_t)run.count) continue;
    EvalArgs A{};
    A.sec = T.secs + run.sector;
    A.terms = T.terms;
    A.x = T.x + run.x_off;
    A.out = T.out + run.pt_off * T.K * 2;
    A.npts = run.count;
    switch (tape(A.sec)->cls) {
      case 0: eval_point_real<4, KM>(A, i); break;
      case 1:
        if constexpr (NVMAX == 6)
          eval_point_real<6, KM>(A, i);
        else if constexpr (NVMAX >= 8)
          eval_point_real<8, KM>(A, i);
        break;
      case 2:
        if constexpr (NVMAX >= 16) eval_point_real<16, KM>(A, i);
        break;
      default: break;
    }
  }
}

}  // namespace sdi
