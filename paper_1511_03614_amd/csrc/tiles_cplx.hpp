// Persistent multi-sector tile kernel, complex mode (contour deformation).
// Same scheduling, partial sums and reductions as the real kernel; each tile
// also counts the points where Im F(z) > 0 (the TestF check of section 4.6).
#pragma once
#include "cplx_args.h"
#include "eval_cplx_dd.hpp"

namespace sdi {

template <int NV, int PPT, int KM, int MODE>
__device__ __forceinline__ void run_tile_cplx(const TileArgs& A, const CplxArgs& X, CSec* S,
                                              const TileDesc& td, int tc, const double* __restrict__ lgrid,
                                              double* __restrict__ lhist, double (&sr)[KM], double (&cr)[KM],
                                              double (&si)[KM], double (&ci)[KM], int& nonfin, int& npos) {
  const uint32_t step = (uint32_t)blockDim.x * PPT;
  const SDI_TAPE CplxDev* cx = tape(X.cx) + td.sector;
  for (uint32_t off = threadIdx.x * PPT; off < td.count; off += step) {
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
    cd f[PPT][KM];
    int imf[PPT];
    eval_f_cplx<NV, PPT, KM>(S, cx, tape(X.dir), tape(A.terms), x, f, imf);
    const int kf = S->kf;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      bool bad = false;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const double vr = w[p] * f[p][k].re;
        const double vi = w[p] * f[p][k].im;
        two_sum_acc(sr[k], cr[k], vr);
        two_sum_acc(si[k], ci[k], vi);
        bad |= !isfinite(vr) || !isfinite(vi);
      }
      nonfin += bad ? 1 : 0;
      npos += imf[p];
      if constexpr (MODE == 1) {
        const int n = S->n;
        const int nb = S->nbins;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (k < kf) {
            const double v2 = w[p] * w[p] * (f[p][k].re * f[p][k].re + f[p][k].im * f[p][k].im);
#pragma unroll
            for (int j = 0; j < NV; ++j)
              if (j < n) atomicAdd(&lhist[((size_t)S->perm[j] * nb + bins[p][j]) * kf + k], v2);
          }
        }
      }
    }
  }
}

// One point per lane for the endpoint-precision instances: lattice point
// td.i0 + off (MODE 0) or the tile's explicit point off (MODE 2).
template <int NV, int MODE>
__device__ __forceinline__ void load_point_cplx(const TileArgs& A, CSec* S, const TileDesc& td, int tc,
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
__device__ __forceinline__ void dd_flush_cplx(const TileArgs& A, const CplxArgs& X, CSec* S, const TileDesc& td,
                                              int tc, const double* __restrict__ lgrid, const uint32_t* q, int cnt,
                                              double (&sr)[KM], double (&cr)[KM], double (&si)[KM],
                                              double (&ci)[KM], int& nonfin) {
  const int lane = threadIdx.x & 63;
  if (lane < cnt) {
    double x[1][NV], w[1];
    load_point_cplx<NV, MODE>(A, S, td, tc, lgrid, q[lane], x, w);
    double fr[KM], fi[KM], cd_[KM];
    eval_f_cplx_dd<KM>(S, tape(X.cx) + td.sector, tape(X.dir), tape(A.terms), x[0], fr, fi, cd_);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const double vr = w[0] * fr[k];
      const double vi = w[0] * fi[k];
      two_sum_acc(sr[k], cr[k], vr);
      two_sum_acc(si[k], ci[k], vi);
      bad |= !isfinite(vr) || !isfinite(vi);
    }
    nonfin += bad ? 1 : 0;
  }
}

// Final-pass tile of the endpoint-precision instances, one point per thread:
// points whose smallest singular coordinate is below A.small_x are queued per
// wave in LDS (ballot and prefix count) and evaluated 64 at a time in
// double-double, as in the real kernel; their Im F(z) > 0 flags come from the
// fp64 evaluation.  Lanes past the tile's end take a placeholder point that is
// neither accumulated, counted nor queued.
template <int NV, int KM, int MODE>
__device__ __forceinline__ void run_tile_cplx_ddq(const TileArgs& A, const CplxArgs& X, CSec* S,
                                                  const TileDesc& td, int tc, const double* __restrict__ lgrid,
                                                  uint32_t* q, double (&sr)[KM], double (&cr)[KM], double (&si)[KM],
                                                  double (&ci)[KM], int& nonfin, int& npos) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;   // lanes under this one
  const SDI_TAPE CplxDev* cx = tape(X.cx) + td.sector;
  const int ns = S->ns;
  int qn = 0;   // queued entries of this wave (wave-uniform)
  for (uint32_t base = 0; base < td.count; base += blockDim.x) {
    asm volatile("" ::: "memory");
    const uint32_t off = base + threadIdx.x;
    const bool act = off < td.count;
    double x[1][NV], w[1];
    if (act) {
      load_point_cplx<NV, MODE>(A, S, td, tc, lgrid, off, x, w);
    } else {
#pragma unroll
      for (int j = 0; j < NV; ++j) x[0][j] = 0.5;
      w[0] = 0.0;
    }
    cd f[1][KM];
    int imf[1];
    eval_f_cplx<NV, 1, KM>(S, cx, tape(X.dir), tape(A.terms), x, f, imf);
    const bool flag = act && near_face<NV>(x[0], ns, A.small_x);
    if (act) npos += imf[0];
    if (act && !flag) {
      bool bad = false;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const double vr = w[0] * f[0][k].re;
        const double vi = w[0] * f[0][k].im;
        two_sum_acc(sr[k], cr[k], vr);
        two_sum_acc(si[k], ci[k], vi);
        bad |= !isfinite(vr) || !isfinite(vi);
      }
      nonfin += bad ? 1 : 0;
    }
    // queue the flagged points of this round: qn < 64 here, so qn + 64 <= DDQ_CAP
    const uint64_t bal = __ballot(flag);
    if (flag) q[qn + __popcll(bal & below)] = off;
    qn += __popcll(bal);
    if (qn >= 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      dd_flush_cplx<NV, KM, MODE>(A, X, S, td, tc, lgrid, q, 64, sr, cr, si, ci, nonfin);
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
  if (qn > 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    dd_flush_cplx<NV, KM, MODE>(A, X, S, td, tc, lgrid, q, qn, sr, cr, si, ci, nonfin);
  }
}

// Double-double sum over the 64 lanes of a wave (every lane ends with the total).
__device__ __forceinline__ void wave_dd_reduce(double hi, double lo, double& ohi, double& olo) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double h2 = __shfl_xor(hi, o, 64);
    const double l2 = __shfl_xor(lo, o, 64);
    dd_add(hi, lo, h2, l2);
  }
  ohi = hi;
  olo = lo;
}

// WPE: minimum waves per SIMD the register allocation must allow (1 = no
// constraint; 2 trades some scratch spills for twice the waves).
// DD: the endpoint-precision instances (final pass on lattice or explicit
// points, one point per thread; points below A.small_x again in double-double).
template <int NVMAX, int PPT, int KM, int MODE, int WPE, bool DD = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) k_tiles_cplx(TileArgs A,
                                                                                                 CplxArgs X) {
  extern __shared__ double smem[];
  __shared__ int s_tile, s_nonfin, s_pos;
  __shared__ double s_red[BLOCK / 64][KM][4];
  __shared__ uint32_t s_q[DD ? (BLOCK / 64) * DDQ_CAP : 1];
  static_assert(!DD || (PPT == 1 && MODE != 1), "endpoint precision is a final-pass mode, one point per thread");
  constexpr int NVC = NVMAX <= 4 ? 0 : 1;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      s_tile = atomicAdd(A.counter, 1);
      s_nonfin = 0;
      s_pos = 0;
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
    double sr[KM], cr[KM], si[KM], ci[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) { sr[k] = 0.0; cr[k] = 0.0; si[k] = 0.0; ci[k] = 0.0; }
    int nonfin = 0, npos = 0;
    if constexpr (DD) {
      uint32_t* q = s_q + (threadIdx.x >> 6) * DDQ_CAP;
      switch (S->cls) {
        case 0:
          run_tile_cplx_ddq<4, KM, MODE>(A, X, S, td, tc, lgrid, q, sr, cr, si, ci, nonfin, npos);
          break;
        case 1:
          if constexpr (NVC >= 1)
            run_tile_cplx_ddq<8, KM, MODE>(A, X, S, td, tc, lgrid, q, sr, cr, si, ci, nonfin, npos);
          break;
        default:
          break;
      }
    } else {
      switch (S->cls) {
        case 0:
          run_tile_cplx<4, PPT, KM, MODE>(A, X, S, td, tc, lgrid, lhist, sr, cr, si, ci, nonfin, npos);
          break;
        case 1:
          if constexpr (NVMAX == 6)
            run_tile_cplx<6, PPT, KM, MODE>(A, X, S, td, tc, lgrid, lhist, sr, cr, si, ci, nonfin, npos);
          else if constexpr (NVC >= 1)
            run_tile_cplx<8, PPT, KM, MODE>(A, X, S, td, tc, lgrid, lhist, sr, cr, si, ci, nonfin, npos);
          break;
        default:
          break;
      }
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      double h, l;
      double hi = sr[k] + cr[k];
      double lo = cr[k] - (hi - sr[k]);
      wave_dd_reduce(hi, lo, h, l);
      double h2, l2;
      hi = si[k] + ci[k];
      lo = ci[k] - (hi - si[k]);
      wave_dd_reduce(hi, lo, h2, l2);
      if (lane == 0) {
        s_red[wave][k][0] = h;
        s_red[wave][k][1] = l;
        s_red[wave][k][2] = h2;
        s_red[wave][k][3] = l2;
      }
    }
    if (nonfin) atomicAdd(&s_nonfin, nonfin);
    if (npos) atomicAdd(&s_pos, npos);
    __syncthreads();
    if (threadIdx.x < KM) {
      const int k = threadIdx.x;
      double hr = s_red[0][k][0], lr = s_red[0][k][1], hi = s_red[0][k][2], li = s_red[0][k][3];
      for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) {
        dd_add(hr, lr, s_red[wv][k][0], s_red[wv][k][1]);
        dd_add(hi, li, s_red[wv][k][2], s_red[wv][k][3]);
      }
      double* out = A.partial + ((size_t)tc * KMAX + k) * PART_STRIDE;
      out[0] = hr;
      out[1] = lr;
      out[2] = hi;
      out[3] = li;
    }
    if (threadIdx.x == 0) {
      A.nonfinite[2 * tc] = s_nonfin;
      A.nonfinite[2 * tc + 1] = s_pos;
    }
    if constexpr (MODE == 1) {
      double* gh = A.hist + A.hist_off[tc];
      for (int i = threadIdx.x; i < n * nb * kf; i += blockDim.x) gh[i] = lhist[i];
    }
  }
}

template <int NV, int KM>
__device__ __forceinline__ void eval_point_cplx(const EvalArgs& A, const CplxArgs& X, int64_t i) {
  CSec* S = tape(A.sec);
  const int n = S->n;
  const int K = S->K;
  double x[1][NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) x[0][j] = j < n ? A.x[i * n + S->perm[j]] : 0.5;
  cd f[1][KM];
  double cnd[1][KM];
  int imf[1];
  if (A.cond)
    eval_f_cplx_c<NV, 1, KM, true>(S, tape(X.cx), tape(X.dir), tape(A.terms), x, f, imf, cnd);
  else
    eval_f_cplx<NV, 1, KM>(S, tape(X.cx), tape(X.dir), tape(A.terms), x, f, imf);
  (void)imf;
  if (A.small_x > 0.0 && near_face<NV>(x[0], S->ns, A.small_x)) {
    double fr[KM], fi[KM];
    eval_f_cplx_dd<KM>(S, tape(X.cx), tape(X.dir), tape(A.terms), x[0], fr, fi, cnd[0]);
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) f[0][kk] = cd{fr[kk], fi[kk]};
  }
  for (int k = 0; k < K; ++k) {
    double fr = 0.0, fi = 0.0, cs = 0.0;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
      fr += S->fold_re[k][kk] * f[0][kk].re - S->fold_im[k][kk] * f[0][kk].im;
      fi += S->fold_re[k][kk] * f[0][kk].im + S->fold_im[k][kk] * f[0][kk].re;
      if (A.cond) cs += hypot(S->fold_re[k][kk], S->fold_im[k][kk]) * cnd[0][kk];
    }
    A.out[(i * K + k) * 2] = fr;
    A.out[(i * K + k) * 2 + 1] = fi;
    if (A.cond) A.cond[i * K + k] = cs;
  }
}

template <int KM>
__global__ void __launch_bounds__(BLOCK) k_eval_points_cplx(EvalArgs A, CplxArgs X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.npts) return;
  switch (tape(A.sec)->cls) {
    case 0: eval_point_cplx<4, KM>(A, X, i); break;
    case 1: eval_point_cplx<8, KM>(A, X, i); break;
    default: break;
  }
}

// Values of every result order at the explicit points of several sectors.
template <int KM>
__global__ void __launch_bounds__(BLOCK) k_eval_tiles_cplx(EvalTilesArgs T, CplxArgs X) {
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
    const CplxArgs Xs{X.cx + run.sector, X.dir};
    switch (tape(A.sec)->cls) {
      case 0: eval_point_cplx<4, KM>(A, Xs, i); break;
      case 1: eval_point_cplx<8, KM>(A, Xs, i); break;
      default: break;
    }
  }
}

// True when Im F(z) > 0 at some corner x_W = 0 of the pole subtraction for
// the deformation size lam (the F - i0 side is left): the per-point test of
// the automatic deformation-size search.
template <int NV>
__device__ __forceinline__ bool imf_any_corner(CSec* S, const SDI_TAPE CplxDev* X, CU32* dir, CTerm* terms,
                                               const double (&x)[1][NV], double lam) {
  const int n = S->n;
  const int ns = S->ns;
  const int facf = X->fac_f;
  if (facf < 0) return false;
  bool pos = false;
  const int C = 1 << ns;
  for (int W = 0; W < C; ++W) {
    cd z[1][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double y = (j < MAXS && ((W >> j) & 1)) ? 0.0 : x[0][j];
      double g = 0.0;
      if (j < n) {
        double v[1];
        CU32* d = dir + (size_t)X->dir_off + ((size_t)j * MAXC + W) * 2;
        poly_real3<NV, 1>(terms + d[0], d[1], x, v);
        g = v[0];
      }
      const double t = lam * (1.0 - y) * g;
      z[0][j] = cd{y, -y * t};
    }
    cd P[1];
    poly_cplx<NV, 1>(terms + S->tab_off[facf][W], coef_im_at(X, S->tab_off[facf][W]), S->tab_cnt[facf][W], z, P);
    cd fz = P[0];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int e = X->mono_f[j];
      for (int k = 0; k < e; ++k) fz = cmul(fz, z[0][j]);
    }
    pos = pos || (fz.im > 0.0);
  }
  return pos;
}

template <int NVMAX>
__global__ void __launch_bounds__(BLOCK) k_lambda_test(const SecDev* secs, const CplxDev* cx, const uint32_t* dir,
                                                       const Term* terms, const uint64_t* zp, const uint64_t* shifts,
                                                       int64_t npts, const double* cand, int ncand, int32_t* fail) {
  __shared__ int32_t s_fail;
  const int s = blockIdx.y;
  CSec* S = tape(secs) + s;
  if (threadIdx.x == 0) s_fail = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t mask = 0;
  if (i < npts) {
    double x[1][NVMAX], w[1];
    int bins[1][NVMAX];
    make_points<NVMAX, 1>(S, tape(zp) + (size_t)s * MAXV, tape(shifts) + (size_t)S->shift_row * MAXV, nullptr,
                          (uint64_t)i, x, w, bins);
    for (int k = 0; k < ncand; ++k)
      if (imf_any_corner<NVMAX>(S, tape(cx) + s, tape(dir), tape(terms), x, cand[s * ncand + k])) mask |= 1 << k;
  }
  if (mask) atomicOr(&s_fail, mask);
  __syncthreads();
  if (threadIdx.x == 0 && s_fail) atomicOr(fail + s, s_fail);
}

}  // namespace sdi
