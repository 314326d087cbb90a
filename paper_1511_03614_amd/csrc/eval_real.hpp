// Real-mode sector-integrand evaluation on gfx950: device building blocks.
//
// One wave evaluates 64 x PPT points of one sector at a time.  Everything that
// depends on the sector (term lists, exponents, gamma/delta, fold matrix) is
// read from the SecDev record and the Term tables with wave-uniform scalar
// loads, so it lands in SGPRs; per-point data (x, powers, logs, series) stays
// in VGPRs.  The method (pole subtraction at x_j = 0 and eps expansion of
// x^(b eps) and P^(delta eps) into log powers; paper section 1 and eq. (2))
// is evaluated per corner W of the singular set S:
//   G0_W = prod_m P_m(x^(W))^gamma_m,  Lambda_W = sum_m delta_m ln P_m(x^(W)),
//   f_k += (-1)^|W\T| prod_{T} 1/b prod_{S\T} 1/x_j G0_W (L_T + Lambda_W)^q / q!,
// q = k + |T|, with L_T = sum_{j in S\T} b_j ln x_j + sum_{j not in S} b_j ln x_j,
// then F_k = mono * sum fold[k][kk] f_kk carries c_s and the prefactor series.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdint_internal.h"

namespace sdi {

// The sector tape (SecDev records, Term lists, complex tables, derivative
// directory, lattice vectors and shifts) is read-only while a kernel runs, and
// is read at wave-uniform addresses.  Reading it through the constant address
// space lets those loads compile to scalar loads into SGPRs, although the
// kernels also store to global memory (which otherwise forces vector loads and
// readfirstlane).
#define SDI_TAPE __attribute__((address_space(4)))
typedef const SDI_TAPE SecDev CSec;
typedef const SDI_TAPE Term CTerm;
typedef const SDI_TAPE uint64_t CU64;
typedef const SDI_TAPE uint32_t CU32;
template <class T>
__device__ __forceinline__ const SDI_TAPE T* tape(const T* p) {
  return (const SDI_TAPE T*)p;
}

// --------------------------------------------------------------- compensated sums

// Knuth's branch-free two-sum: s + v = t + err exactly.
__device__ __forceinline__ void two_sum_acc(double& s, double& c, double v) {
  const double t = s + v;
  const double bp = t - s;
  const double err = (s - (t - bp)) + (v - bp);
  s = t;
  c += err;
}

// (hi, lo) += (h2, l2) as double-double.
__device__ __forceinline__ void dd_add(double& hi, double& lo, double h2, double l2) {
  const double s = hi + h2;
  const double bp = s - hi;
  const double e = (hi - (s - bp)) + (h2 - bp);
  const double l = lo + l2 + e;
  hi = s + l;
  lo = l - (hi - s);
}

// --------------------------------------------------------------- sampling

// Shifted rank-1 lattice coordinate, exact: U = (i * (z << (53-m)) + D) mod 2^53.
__device__ __forceinline__ double lattice_coord(uint64_t i, uint64_t zp, uint64_t d) {
  const uint64_t u = (i * zp + d) & MASK53;
  return (double)u * 0x1p-53;
}

// Index of the run holding chunk c: the last r with prefix[r] <= c.
__device__ __forceinline__ int find_run(const int64_t* prefix, int nruns, int64_t c) {
  int lo = 0, hi = nruns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tent map u -> 2u (u < 1/2), 2(1-u) otherwise: exact in fp64.  Written as
// 2 min(u, 1-u): for u < 1/2 the rounded 1-u is still >= 1/2 > u, for u >= 1/2
// 1-u is exact (Sterbenz) and <= u, so both forms give the same bits.
__device__ __forceinline__ double tent(double u) {
  return 2.0 * fmin(u, 1.0 - u);
}

// Vegas map of one coordinate, no contraction so that the host reference
// arithmetic (one rounding per operation) is reproduced bit for bit.
__device__ __forceinline__ double vegas_coord(const double* __restrict__ g, int nb, double u,
                                              double& w) {
#pragma clang fp contract(off)
  const double un = u * (double)nb;
  int b = (int)un;
  b = b > nb - 1 ? nb - 1 : b;
  const double d = un - (double)b;
  const double lo = g[b];
  const double width = g[b + 1] - lo;
  const double prod = d * width;
  w = w * ((double)nb * width);
  return lo + prod;
}

// Points i = i_first .. i_first+PPT-1 (consecutive lattice indices) of one sector and shift.
// Writes x in internal variable order and the Vegas weight; also the bins (warm-up).
template <int NV, int PPT>
__device__ __forceinline__ void make_points(CSec* S, CU64* zp, CU64* sh, const double* __restrict__ lgrid,
                                            uint64_t i_first, double (&x)[PPT][NV], double (&w)[PPT],
                                            int (&bins)[PPT][NV]) {
  const int n = S->n;
  const int flags = S->flags;
  const int nb = S->nbins;
#pragma unroll
  for (int p = 0; p < PPT; ++p) w[p] = 1.0;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j < n) {
      const int oj = S->perm[j];
      const uint64_t z = zp[oj];
      const uint64_t d = sh[oj];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        double u = lattice_coord(i_first + (uint64_t)p, z, d);
        if (flags & F_BAKER) u = tent(u);
        if (flags & F_USE_GRID) {
          const double un = u * (double)nb;
          int b = (int)un;
          bins[p][j] = b > nb - 1 ? nb - 1 : b;
          u = vegas_coord(lgrid + oj * (nb + 1), nb, u, w[p]);
        } else {
          bins[p][j] = 0;
        }
        x[p][j] = u;
      }
    } else {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        x[p][j] = 0.5;
        bins[p][j] = 0;
      }
    }
  }
}

// --------------------------------------------------------------- polynomials

// out += coef prod_j x_j^e_j for one term, PPT points.  The exponent word is
// wave-uniform (an SGPR), so every exponent bit is a scalar branch; the empty
// asm keeps the compiler from turning the skipped multiplies into per-lane
// selects.  Bit 1 (x^2) multiplies by x twice: per-point squares held for the
// whole evaluation cost more in register spills than the extra multiply.
template <int NV, int PPT, bool E7 = false>
__device__ __forceinline__ void add_term(double c, uint64_t e, const double (&x)[PPT][NV],
                                         double (&out)[PPT]) {
  double m[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) m[p] = c;
  // 32-bit halves of the word: one scalar test per bit instead of a 64-bit compare
  const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const uint32_t w = j < 8 ? elo : ehi;
    const int sh = 4 * (j & 7);
    if (w & (1u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] *= x[p][j];
    }
    if (w & (2u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] = (m[p] * x[p][j]) * x[p][j];
    }
    if constexpr (E7) {
      if (w & (4u << sh)) {
        asm volatile("" ::);
#pragma unroll
        for (int p = 0; p < PPT; ++p) m[p] = (((m[p] * x[p][j]) * x[p][j]) * x[p][j]) * x[p][j];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] += m[p];
}

// sum_t coef_t prod_j x_j^e_tj over one term list, for PPT points, terms in
// list order.  Terms are read four at a time so that their scalar loads are in
// flight together (one wait per four terms instead of one per term).
// E7: exponents up to 7 (the x^4 bit is tested too; sectors with F_EXP7).
template <int NV, int PPT, bool E7 = false>
__device__ __forceinline__ void poly_real(CTerm* t, uint32_t cnt,
                                          const double (&x)[PPT][NV],
                                          double (&out)[PPT]) {
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] = 0.0;
  uint32_t i = 0;
  for (; i + 4 <= cnt; i += 4) {
    const double c0 = t[i].coef, c1 = t[i + 1].coef, c2 = t[i + 2].coef, c3 = t[i + 3].coef;
    const uint64_t e0 = t[i].exps, e1 = t[i + 1].exps, e2 = t[i + 2].exps, e3 = t[i + 3].exps;
    add_term<NV, PPT, E7>(c0, e0, x, out);
    add_term<NV, PPT, E7>(c1, e1, x, out);
    add_term<NV, PPT, E7>(c2, e2, x, out);
    add_term<NV, PPT, E7>(c3, e3, x, out);
  }
  for (; i < cnt; ++i) add_term<NV, PPT, E7>(t[i].coef, t[i].exps, x, out);
}

// out += coef prod_{j<NK} x_j^e_j: add_term for terms whose exponents vanish
// beyond the first NK variables (the sector's own variable count), so that a
// sector of n variables in a wider register class tests only its n variables.
template <int NK, int NV, int PPT, bool E7>
__device__ __forceinline__ void add_term_k(double c, uint64_t e, const double (&x)[PPT][NV],
                                           double (&out)[PPT]) {
  static_assert(NK >= 1 && NK <= NV, "variable bound");
  double m[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) m[p] = c;
  const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const uint32_t w = j < 8 ? elo : ehi;
    const int sh = 4 * (j & 7);
    if (w & (1u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] *= x[p][j];
    }
    if (w & (2u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] = (m[p] * x[p][j]) * x[p][j];
    }
    if constexpr (E7) {
      if (w & (4u << sh)) {
        asm volatile("" ::);
#pragma unroll
        for (int p = 0; p < PPT; ++p) m[p] = (((m[p] * x[p][j]) * x[p][j]) * x[p][j]) * x[p][j];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] += m[p];
}

// out += sum over one term list.  Terms are read four at a time, and the next
// four are requested before the current four are evaluated, so their scalar
// loads are in flight while the multiplies of these run.
template <int NK, int NV, int PPT, bool E7>
__device__ __forceinline__ void poly_acc_k(CTerm* t, uint32_t cnt, const double (&x)[PPT][NV],
                                           double (&out)[PPT]) {
  uint32_t i = 0;
  if (cnt >= 4) {
    double c0 = t[0].coef, c1 = t[1].coef, c2 = t[2].coef, c3 = t[3].coef;
    uint64_t e0 = t[0].exps, e1 = t[1].exps, e2 = t[2].exps, e3 = t[3].exps;
    for (; i + 8 <= cnt; i += 4) {
      const double n0 = t[i + 4].coef, n1 = t[i + 5].coef, n2 = t[i + 6].coef, n3 = t[i + 7].coef;
      const uint64_t f0 = t[i + 4].exps, f1 = t[i + 5].exps, f2 = t[i + 6].exps, f3 = t[i + 7].exps;
      add_term_k<NK, NV, PPT, E7>(c0, e0, x, out);
      add_term_k<NK, NV, PPT, E7>(c1, e1, x, out);
      add_term_k<NK, NV, PPT, E7>(c2, e2, x, out);
      add_term_k<NK, NV, PPT, E7>(c3, e3, x, out);
      c0 = n0; c1 = n1; c2 = n2; c3 = n3;
      e0 = f0; e1 = f1; e2 = f2; e3 = f3;
    }
    add_term_k<NK, NV, PPT, E7>(c0, e0, x, out);
    add_term_k<NK, NV, PPT, E7>(c1, e1, x, out);
    add_term_k<NK, NV, PPT, E7>(c2, e2, x, out);
    add_term_k<NK, NV, PPT, E7>(c3, e3, x, out);
    i += 4;
  }
  for (; i < cnt; ++i) add_term_k<NK, NV, PPT, E7>(t[i].coef, t[i].exps, x, out);
}

// poly_acc_k with NK = the sector's variable count n (wave-uniform), for n in
// K .. NV; smaller n takes NK = K.
template <int K, int NV, int PPT, bool E7>
__device__ __forceinline__ void poly_acc_n(CTerm* t, uint32_t cnt, int n, const double (&x)[PPT][NV],
                                           double (&out)[PPT]) {
  if constexpr (K >= NV) {
    poly_acc_k<NV, NV, PPT, E7>(t, cnt, x, out);
  } else {
    if (n <= K)
      poly_acc_k<K, NV, PPT, E7>(t, cnt, x, out);
    else
      poly_acc_n<K + 1, NV, PPT, E7>(t, cnt, n, x, out);
  }
}

// Smallest variable count a sector of register class NV can have (the classes
// are n <= 4, 5..6, 5..8 and 9..16), the first bound poly_acc_n distinguishes.
template <int NV>
constexpr int class_low() {
  return NV <= 4 ? NV : (NV <= 8 ? 5 : 9);
}

// The regular factors at every corner, each term evaluated once: for every
// non-empty group (m, sigma) of terms with singular support sigma, the group
// sum q at x is added to Pc[m][W] for every corner W with W & sigma == 0 (the
// corners where those terms survive).  Pc[m][W] = P_m(x^(W)) for W < 2^ns.
// E7M: 0 - exponents up to 3 only (the x^4 bit is never tested), 1 - up to 7,
// 2 - by the sector's F_EXP7 flag (both codes in the caller).
template <int NV, int PPT, int NSM, int MF, int E7M>
__device__ __forceinline__ void corner_polys(CSec* S, CTerm* terms, const double (&x)[PPT][NV],
                                             double (&Pc)[MF][1 << NSM][PPT]) {
  constexpr int NC = 1 << NSM;
  const int n = S->n;
  const int nfac = S->nfac;
  const int C = 1 << S->ns;
#pragma unroll
  for (int fm = 0; fm < MF; ++fm)
#pragma unroll
    for (int W = 0; W < NC; ++W)
#pragma unroll
      for (int p = 0; p < PPT; ++p) Pc[fm][W][p] = 0.0;
#pragma unroll
  for (int fm = 0; fm < MF; ++fm) {
    if (fm < nfac) {
      uint32_t gm = S->grp_mask[fm];
      while (gm) {
        const int sg = __builtin_ctz(gm);
        gm &= gm - 1;
        double q[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) q[p] = 0.0;
        if (E7M == 1 || (E7M == 2 && (S->flags & F_EXP7)))
          poly_acc_n<class_low<NV>(), NV, PPT, E7M != 0>(terms + S->grp_off[fm][sg], S->grp_cnt[fm][sg], n, x, q);
        else
          poly_acc_n<class_low<NV>(), NV, PPT, false>(terms + S->grp_off[fm][sg], S->grp_cnt[fm][sg], n, x, q);
#pragma unroll
        for (int W = 0; W < NC; ++W) {
          if (W < C && (W & sg) == 0) {
            asm volatile("" ::);
#pragma unroll
            for (int p = 0; p < PPT; ++p) Pc[fm][W][p] += q[p];
          }
        }
      }
    }
  }
}

// P[m] = Pc[m][W] for a wave-uniform corner W (one scalar branch per case).
template <int NSM, int MF, int PPT>
__device__ __forceinline__ void select_corner(const double (&Pc)[MF][1 << NSM][PPT], int W,
                                              double (&P)[MF][PPT]) {
#pragma unroll
  for (int k = 0; k < (1 << NSM); ++k) {
    if (W == k) {
      asm volatile("" ::);
#pragma unroll
      for (int fm = 0; fm < MF; ++fm)
#pragma unroll
        for (int p = 0; p < PPT; ++p) P[fm][p] = Pc[fm][k][p];
    }
  }
}

// 1/v for positive normal v: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - v r), each of which squares the relative
// error; within an ulp or two of the correctly rounded quotient, in half the
// instructions of an IEEE division.
__device__ __forceinline__ double fast_rcp(double v) {
  double r = __builtin_amdgcn_rcp(v);
  double e = fma(-v, r, 1.0);
  r = fma(r, e, r);
  e = fma(-v, r, 1.0);
  return fma(r, e, r);
}

// Mantissa in [0.5, 1) and binary exponent; non-positive values give NaN so that
// logarithms of non-positive factors stay NaN in real mode.
__device__ __forceinline__ double mant_exp(double v, int& e) {
  const double m = frexp(v, &e);
  return v > 0.0 ? m : __builtin_nan("");
}

// G0 and Lambda at corner W for PPT points.
template <int NV, int PPT, int E7M>
__device__ __forceinline__ void corner_regular(CSec* S, CTerm* terms,
                                               int W, const double (&x)[PPT][NV],
                                               double (&g0)[PPT],
                                               double (&lam)[PPT]) {
  const int nfac = S->nfac;
  const int flags = S->flags;
  if (flags & F_INT_POW) {
    double num[PPT], den[PPT], mnum[PPT], mden[PPT];
    int esum[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      num[p] = 1.0; den[p] = 1.0; mnum[p] = 1.0; mden[p] = 1.0; esum[p] = 0;
    }
#pragma unroll
    for (int fm = 0; fm < MAXF; ++fm) {
      if (fm < nfac) {
        double P[PPT];
        if (E7M == 1 || (E7M == 2 && (flags & F_EXP7)))
          poly_real<NV, PPT, E7M != 0>(terms + S->tab_off[fm][W], S->tab_cnt[fm][W], x, P);
        else
          poly_real<NV, PPT, false>(terms + S->tab_off[fm][W], S->tab_cnt[fm][W], x, P);
        const int g = S->gam_int[fm];
        const int d = S->del_int[fm];
        const int ga = g < 0 ? -g : g;
        const int da = d < 0 ? -d : d;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          int e;
          const double mt = mant_exp(P[p], e);
          double pg = 1.0, md = 1.0;
          for (int k = 0; k < ga; ++k) pg *= P[p];
          for (int k = 0; k < da; ++k) md *= mt;
          if (g >= 0) num[p] *= pg; else den[p] *= pg;
          if (d >= 0) mnum[p] *= md; else mden[p] *= md;
          esum[p] += d * e;
        }
      }
    }
    // one reciprocal serves both quotients: num/den and mnum/mden
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const double inv = fast_rcp(den[p] * mden[p]);
      g0[p] = num[p] * mden[p] * inv;
      lam[p] = log(mnum[p] * den[p] * inv) + (double)esum[p] * 0.69314718055994530942;
    }
  } else {
    double lg[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) { lg[p] = 0.0; lam[p] = 0.0; }
#pragma unroll
    for (int fm = 0; fm < MAXF; ++fm) {
      if (fm < nfac) {
        double P[PPT];
        if (E7M == 1 || (E7M == 2 && (flags & F_EXP7)))
          poly_real<NV, PPT, E7M != 0>(terms + S->tab_off[fm][W], S->tab_cnt[fm][W], x, P);
        else
          poly_real<NV, PPT, false>(terms + S->tab_off[fm][W], S->tab_cnt[fm][W], x, P);
        const double gm = S->gam[fm];
        const double dm = S->del[fm];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const double l = log(P[p]);
          lg[p] += gm * l;
          lam[p] += dm * l;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) g0[p] = exp(lg[p]);
  }
}

// G0 and Lambda at one corner from the factor values P[m] there (as
// corner_regular, without evaluating the polynomials).
template <int PPT, int MF>
__device__ __forceinline__ void corner_from_polys(CSec* S, const double (&P)[MF][PPT], double (&g0)[PPT],
                                                  double (&lam)[PPT]) {
  const int nfac = S->nfac;
  const int flags = S->flags;
  if (flags & F_INT_POW) {
    double num[PPT], den[PPT], mnum[PPT], mden[PPT];
    int esum[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      num[p] = 1.0; den[p] = 1.0; mnum[p] = 1.0; mden[p] = 1.0; esum[p] = 0;
    }
#pragma unroll
    for (int fm = 0; fm < MF; ++fm) {
      if (fm < nfac) {
        const int g = S->gam_int[fm];
        const int d = S->del_int[fm];
        const int ga = g < 0 ? -g : g;
        const int da = d < 0 ? -d : d;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          int e;
          const double mt = mant_exp(P[fm][p], e);
          double pg = 1.0, md = 1.0;
          for (int k = 0; k < ga; ++k) pg *= P[fm][p];
          for (int k = 0; k < da; ++k) md *= mt;
          if (g >= 0) num[p] *= pg; else den[p] *= pg;
          if (d >= 0) mnum[p] *= md; else mden[p] *= md;
          esum[p] += d * e;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const double inv = fast_rcp(den[p] * mden[p]);
      g0[p] = num[p] * mden[p] * inv;
      lam[p] = log(mnum[p] * den[p] * inv) + (double)esum[p] * 0.69314718055994530942;
    }
  } else {
    double lg[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) { lg[p] = 0.0; lam[p] = 0.0; }
#pragma unroll
    for (int fm = 0; fm < MF; ++fm) {
      if (fm < nfac) {
        const double gm = S->gam[fm];
        const double dm = S->del[fm];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const double l = log(P[fm][p]);
          lg[p] += gm * l;
          lam[p] += dm * l;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) g0[p] = exp(lg[p]);
  }
}

// Adds t_q = base z^q / q! to f[OFF + q] for the orders the sector keeps
// (and |t_q| to c when COND: the conditioning sums of the evaluate hook).
template <int OFF, int KM, bool COND>
__device__ __forceinline__ void add_series(double (&f)[KM], double (&c)[KM], double t, double z, int kf) {
#pragma unroll
  for (int kk = OFF; kk < KM; ++kk) {
    if (kk < kf) {
      f[kk] += t;
      if constexpr (COND) c[kk] += fabs(t);
      t = t * z * (1.0 / (double)(kk - OFF + 1));
    }
  }
}

// f_kk (kk = k + ns, k = -ns .. kf-1-ns) of one sector at PPT points, times the
// non-singular monomial.  Internal variables 0..ns-1 are the singular ones.
// Corners W and subsets T of S are wave-uniform runtime loops; the offset of
// q = 0 in f (ns - |T|) selects one of MAXS+1 static accumulation bodies.
// COND: also the sums of |term| per order (cnd), for the evaluate hook.
// NSM: bound on the sector's singular variables (the per-point log x_j and
// 1/x_j arrays are sized by it, which matters for the register budget).
// MF: 0 evaluates each corner's own term lists (any number of factors);
// MF > 0 (sectors of at most MF factors) evaluates every term once by singular
// support (corner_polys) and picks the corner's values from those sums.
template <int NV, int PPT, int KM, bool COND, int NSM = MAXS, int MF = 0, int E7M = 2>
__device__ __forceinline__ void eval_f_real_c(CSec* S, CTerm* terms, const double (&x)[PPT][NV],
                                              double (&f)[PPT][KM], double (&cnd)[PPT][KM]) {
  static_assert(NSM >= 1 && NSM <= MAXS, "singular-variable bound");
  const int n = S->n;
  const int ns = S->ns;
  const int kf = S->kf;
  const int flags = S->flags;
  double lx[PPT][NSM], ix[PPT][NSM];
#pragma unroll
  for (int i = 0; i < NSM; ++i) {
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      lx[p][i] = 0.0;
      ix[p][i] = 1.0;
    }
    if (i < ns && i < NV) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        lx[p][i] = log(x[p][i < NV ? i : 0]);
        ix[p][i] = fast_rcp(x[p][i < NV ? i : 0]);
      }
    }
  }

  // L_rest = sum_{j >= ns} b_j ln x_j and the monomial prod_{j >= ns} x_j^a_j
  double lrest[PPT], mono[PPT];
  if (flags & F_INT_MONO) {
    double pn[PPT], pd[PPT];
    int es[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) { pn[p] = 1.0; pd[p] = 1.0; es[p] = 0; mono[p] = 1.0; }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      if (j >= ns && j < n) {
        const int bj = S->b_int[j];
        const int aj = S->a_int[j];
        const int ba = bj < 0 ? -bj : bj;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          int e;
          const double mt = frexp(x[p][j], &e);
          double q = 1.0;
          for (int k = 0; k < ba; ++k) q *= mt;
          if (bj >= 0) pn[p] *= q; else pd[p] *= q;
          es[p] += bj * e;
          for (int k = 0; k < aj; ++k) mono[p] *= x[p][j];
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p)
      lrest[p] = log(pn[p] * fast_rcp(pd[p])) + (double)es[p] * 0.69314718055994530942;
  } else {
    double la[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) { lrest[p] = 0.0; la[p] = 0.0; }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      if (j >= ns && j < n) {
        const double bj = S->b[j];
        const double aj = S->a[j];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const double l = log(x[p][j]);
          lrest[p] += bj * l;
          la[p] += aj * l;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) mono[p] = exp(la[p]);
  }

#pragma unroll
  for (int p = 0; p < PPT; ++p)
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      f[p][k] = 0.0;
      if constexpr (COND) cnd[p][k] = 0.0;
    }

  constexpr int MFC = MF > 0 ? MF : 1;
  double Pc[MFC][1 << NSM][PPT];
  if constexpr (MF > 0) corner_polys<NV, PPT, NSM, MF, E7M>(S, terms, x, Pc);
  const int C = 1 << ns;
  for (int W = 0; W < C; ++W) {
    double g0[PPT], lam[PPT];
    if constexpr (MF > 0) {
      double P[MF][PPT];
      select_corner<NSM, MF, PPT>(Pc, W, P);
      corner_from_polys<PPT, MF>(S, P, g0, lam);
    } else {
      corner_regular<NV, PPT, E7M>(S, terms, W, x, g0, lam);
    }
    for (int T = W;; T = (T - 1) & W) {
      const int nt = __builtin_popcount(T);
      const int off = ns - nt;
      const double ib = S->invb[T];
      const double sgn = (__builtin_popcount(W & ~T) & 1) ? -ib : ib;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        double coef = sgn * g0[p];
        double z = lrest[p] + lam[p];
#pragma unroll
        for (int i = 0; i < NSM; ++i) {
          if (i < ns && !((T >> i) & 1)) {
            coef *= ix[p][i];
            z += S->bS[i] * lx[p][i];
          }
        }
        switch (off) {
          case 0: add_series<0, KM, COND>(f[p], cnd[p], coef, z, kf); break;
          case 1: add_series<1, KM, COND>(f[p], cnd[p], coef, z, kf); break;
          case 2: add_series<2, KM, COND>(f[p], cnd[p], coef, z, kf); break;
          case 3: add_series<3, KM, COND>(f[p], cnd[p], coef, z, kf); break;
          default: add_series<4, KM, COND>(f[p], cnd[p], coef, z, kf); break;
        }
      }
      if (T == 0) break;
    }
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p)
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      f[p][k] *= mono[p];
      if constexpr (COND) cnd[p][k] *= fabs(mono[p]);
    }
}

template <int NV, int PPT, int KM, int NSM = MAXS, int MF = 0, int E7M = 2>
__device__ __forceinline__ void eval_f_real(CSec* S, CTerm* terms, const double (&x)[PPT][NV],
                                            double (&f)[PPT][KM]) {
  double unused[PPT][KM];
  eval_f_real_c<NV, PPT, KM, false, NSM, MF, E7M>(S, terms, x, f, unused);
}

}  // namespace sdi
