// Double-double evaluation of the real sector integrand at single points, for
// points near the faces x_j = 0 of singular variables.
//
// There the corner terms of the pole subtraction (prod 1/x_j times G0 at the
// corners W of S) are large and cancel, by about log10(1/x_j) digits per
// singular variable, so fp64 leaves few correct digits in f_k.  The paper's
// answer is to evaluate such points in higher precision (the SmallX /
// MPThreshold options of the mixed arithmetic mode, section 4.6, which switch
// to MPFR below a threshold).  Here the same formula as eval_f_real is
// evaluated in double-double arithmetic (about 106 significant bits): the
// cancellation then costs digits of a 32-digit value, and the result is
// rounded to fp64 once at the end.
//
// Arithmetic: error-free transformations (Knuth's two-sum, the fma product),
// renormalisation after each operation (Dekker; Hida, Li and Bailey's QD
// library describe the same operations).  Every function here compiles with
// floating-point contraction off: the compiler would otherwise fuse a product
// into a later sum or difference that reads it (h - s with s = a*b becomes
// fma(-a, b, h)), which subtracts the exact product where the rounded one is
// meant and leaves only fp64 accuracy in the low word.  exp reduces by k ln 2 and 2^-10,
// sums the Taylor series of expm1 and squares back; log is one Newton step
// y + a e^-y - 1 from the fp64 logarithm.  These functions are called for
// the few points below the threshold, so they favour simplicity: runtime
// loops over the sector's variables, one non-inlined function per order count.
#pragma once
#include "eval_real.hpp"

namespace sdi {
namespace xdd {

struct D {
  double h, l;
};

__device__ __forceinline__ D mk(double a) { return D{a, 0.0}; }

// |s| >= |e| (or s = 0): h + l = s + e exactly, h = fl(s + e)
__device__ __forceinline__ D quick(double s, double e) {
#pragma clang fp contract(off)
  const double h = s + e;
  return D{h, e - (h - s)};
}

__device__ __forceinline__ D two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return D{s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ D two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return D{p, fma(a, b, -p)};
}

__device__ __forceinline__ D add(D a, D b) {
#pragma clang fp contract(off)
  const D s = two_sum(a.h, b.h);
  const D t = two_sum(a.l, b.l);
  const D u = quick(s.h, s.l + t.h);
  return quick(u.h, u.l + t.l);
}

__device__ __forceinline__ D neg(D a) { return D{-a.h, -a.l}; }
__device__ __forceinline__ D sub(D a, D b) { return add(a, neg(b)); }

__device__ __forceinline__ D mul(D a, D b) {
#pragma clang fp contract(off)
  const D p = two_prod(a.h, b.h);
  return quick(p.h, p.l + (a.h * b.l + a.l * b.h));
}

__device__ __forceinline__ D mul(D a, double b) {
#pragma clang fp contract(off)
  const D p = two_prod(a.h, b);
  return quick(p.h, p.l + a.l * b);
}

// Long division: three fp64 quotient digits.
__device__ __forceinline__ D div(D a, D b) {
#pragma clang fp contract(off)
  const double q1 = a.h / b.h;
  D r = sub(a, mul(b, q1));
  const double q2 = r.h / b.h;
  r = sub(r, mul(b, q2));
  const double q3 = r.h / b.h;
  return add(quick(q1, q2), mk(q3));
}

__device__ __forceinline__ D scale2(D a, int k) { return D{ldexp(a.h, k), ldexp(a.l, k)}; }

// ln 2 to about 107 bits: the fp64 value nearest ln 2, and the fp64 value
// nearest the remainder.
constexpr double LN2_HI = 0x1.62e42fefa39efp-1;
constexpr double LN2_LO = 0x1.abc9e3b39803fp-56;

__device__ inline D exp(D a) {
#pragma clang fp contract(off)
  if (a.h != a.h) return a;
  if (a.h > 709.782712893384) return mk(__builtin_inf());   // above ln(DBL_MAX)
  if (a.h < -745.0) return mk(0.0);
  // a = k ln 2 + r, |r| <~ ln2/2 (k from an fp64 estimate; r is formed in double-double)
  const double k = rint(a.h * 1.4426950408889634);
  D r = sub(a, mul(D{LN2_HI, LN2_LO}, k));
  r = scale2(r, -10);
  // expm1(r) = r (1 + r/2 (1 + r/3 (1 + ... (1 + r/11)))), |r| < 3.4e-4: the
  // first omitted term is below 1e-45 of the sum
  D s = mk(1.0);
  for (int j = 11; j >= 2; --j) s = add(mk(1.0), div(mul(s, r), mk((double)j)));
  s = mul(s, r);
  // expm1(2r) = 2 expm1(r) + expm1(r)^2, ten times
  for (int i = 0; i < 10; ++i) s = add(scale2(s, 1), mul(s, s));
  return scale2(add(mk(1.0), s), (int)k);
}

// Natural log; NaN for a < 0 (as the fp64 path: real mode has no branch cut), -inf for 0.
// a = m 2^e with m in [0.5, 1) (exact scaling, so subnormal a is no special case):
// ln a = y + (m e^-y - 1) + e ln 2, y the fp64 ln m (one Newton step).
__device__ inline D log(D a) {
#pragma clang fp contract(off)
  if (!(a.h > 0.0)) return mk(a.h == 0.0 ? -__builtin_inf() : __builtin_nan(""));
  if (a.h == __builtin_inf()) return a;
  int e = 0;
  (void)frexp(a.h, &e);
  const D m = scale2(a, -e);
  const double y = ::log(m.h);
  const D r = mul(m, exp(mk(-y)));
  return add(add(mk(y), sub(r, mk(1.0))), mul(D{LN2_HI, LN2_LO}, (double)e));
}

__device__ inline D powi(D a, int k) {
#pragma clang fp contract(off)
  const int e = k < 0 ? -k : k;
  D r = mk(1.0);
  for (int i = 0; i < e; ++i) r = mul(r, a);
  return k < 0 ? div(mk(1.0), r) : r;
}

}  // namespace xdd

// Entries of a wave's queue of points awaiting double-double evaluation (the
// endpoint-precision tile instances): a round adds at most 64 to fewer than 64.
constexpr int DDQ_CAP = 128;

// Whether a point is evaluated in double-double: its smallest singular
// coordinate (internal variables 0 .. ns-1) lies below small_x.
template <int NV>
__device__ __forceinline__ bool near_face(const double (&x)[NV], int ns, double small_x) {
  bool near = false;
#pragma unroll
  for (int i = 0; i < MAXS && i < NV; ++i)
    if (i < ns && x[i] < small_x) near = true;
  return near;
}

// f_kk (kk = k + ns) of one sector at one point (internal variable order), the
// formula of eval_f_real_c in double-double; f and cnd (the sums of |term| per
// order, as the fp64 path returns them) are rounded to fp64 at the end.
template <int KM>
__device__ __attribute__((noinline)) void eval_f_real_dd(CSec* S, CTerm* terms, const double* x, double* f_out,
                                                         double* cnd_out) {
#pragma clang fp contract(off)
  using namespace xdd;
  const int n = S->n;
  const int ns = S->ns;
  const int kf = S->kf;
  const int nfac = S->nfac;
  const int flags = S->flags;

  D lx[MAXS], ix[MAXS];
  for (int i = 0; i < ns; ++i) {
    lx[i] = log(mk(x[i]));
    ix[i] = div(mk(1.0), mk(x[i]));
  }
  // L_rest = sum_{j >= ns} b_j ln x_j and the monomial prod_{j >= ns} x_j^a_j
  D lrest = mk(0.0), mono = mk(1.0);
  for (int j = ns; j < n; ++j) {
    const D l = log(mk(x[j]));
    lrest = add(lrest, mul(l, S->b[j]));
    if (flags & F_INT_MONO) {
      for (int k = 0; k < S->a_int[j]; ++k) mono = mul(mono, x[j]);
    } else {
      mono = mul(mono, exp(mul(l, S->a[j])));
    }
  }

  D f[KM];
  double c[KM];
  for (int k = 0; k < KM; ++k) {
    f[k] = mk(0.0);
    c[k] = 0.0;
  }
  const int C = 1 << ns;
  for (int W = 0; W < C; ++W) {
    // G0 and Lambda at the corner W: the corner's term lists already omit x_j, j in W
    D g0 = mk(1.0), lam = mk(0.0);
    for (int fm = 0; fm < nfac; ++fm) {
      CTerm* t = terms + S->tab_off[fm][W];
      const uint32_t cnt = S->tab_cnt[fm][W];
      D P = mk(0.0);
      for (uint32_t u = 0; u < cnt; ++u) {
        const uint64_t e = t[u].exps;
        D m = mk(t[u].coef);
        for (int j = 0; j < n; ++j) {
          const int nib = (int)((e >> (4 * j)) & 0xfu);
          const int pw = (nib & 1) + 2 * ((nib >> 1) & 1) + 4 * ((nib >> 2) & 1);
          for (int q = 0; q < pw; ++q) m = mul(m, x[j]);
        }
        P = add(P, m);
      }
      // a factor with delta = 0 has no eps dependence and may vanish (the
      // derivative factors of the reduction of a_j < -1): no logarithm then
      if (flags & F_INT_POW) {
        g0 = mul(g0, powi(P, S->gam_int[fm]));
        if (S->del[fm] != 0.0) lam = add(lam, mul(log(P), S->del[fm]));
      } else {
        const D lp = log(P);
        g0 = mul(g0, exp(mul(lp, S->gam[fm])));
        lam = add(lam, mul(lp, S->del[fm]));
      }
    }
    for (int T = W;; T = (T - 1) & W) {
      if (T != 0 && S->invb[T] == 0.0) continue;   // a separated term: no boundary terms
      const int off = ns - __builtin_popcount(T);
      D coef = g0;
      D z = add(lrest, lam);
      for (int i = 0; i < ns; ++i) {
        if ((T >> i) & 1) {
          coef = div(coef, mk(S->bS[i]));
        } else {
          coef = mul(coef, ix[i]);
          z = add(z, mul(lx[i], S->bS[i]));
        }
      }
      if (__builtin_popcount(W & ~T) & 1) coef = neg(coef);
      // t_q = coef z^q / q! into f[off + q]
      D tq = coef;
      for (int kk = off; kk < KM && kk < kf; ++kk) {
        f[kk] = add(f[kk], tq);
        c[kk] += fabs(tq.h);
        tq = div(mul(tq, z), mk((double)(kk - off + 1)));
      }
      if (T == 0) break;
    }
  }
  for (int k = 0; k < KM; ++k) {
    const D v = mul(f[k], mono);
    f_out[k] = v.h + v.l;
    cnd_out[k] = c[k] * fabs(mono.h);
  }
}

}  // namespace sdi
