// Double-double evaluation of the complex-mode (contour-deformed) sector
// integrand at single points near the faces x_j = 0 of singular variables.
//
// The corner terms of the pole subtraction cancel near a face in complex mode
// as they do in real mode (by about log10(1/x_j) digits per singular
// variable), so the SmallX / MPThreshold switch of the mixed arithmetic mode
// (sections 4.4 and 4.6) applies to deformed integrands too.  The formula is
// that of eval_f_cplx_c (deformation, Jacobian determinant by LDL^T, principal
// logarithms with arg = -pi on the negative real axis, subtraction and eps
// series) in double-double complex arithmetic; the values are rounded to fp64
// once at the end.
//
// Functions beyond eval_dd.hpp's, with contraction off as there:
//   sqrt: one Newton step s + (a - s^2) / (2 s) from the fp64 root;
//   sin and cos: reduction by k pi/2 (pi/2 in three fp64 parts), Taylor series
//     to the 29th power on |r| <= pi/4 (first omitted term below 1e-34);
//   atan2: the fp64 angle t0 corrected by tan(t - t0) = (y cos t0 - x sin t0) /
//     (x cos t0 + y sin t0) (|t - t0| ~ 1e-16, so tan equals its argument to
//     well below 2^-106).
// These run for the few points below the threshold only: runtime loops, one
// non-inlined function per order count.
#pragma once
#include "eval_cplx.hpp"
#include "eval_dd.hpp"

namespace sdi {
namespace xdd {

// pi/2 in three fp64 parts (about 160 bits) and pi in two (about 107 bits)
constexpr double PIO2_1 = 0x1.921fb54442d18p+0;
constexpr double PIO2_2 = 0x1.1a62633145c07p-54;
constexpr double PIO2_3 = -0x1.f1976b7ed8fbcp-110;
constexpr double PI_HI = 0x1.921fb54442d18p+1;
constexpr double PI_LO = 0x1.1a62633145c07p-53;

__device__ inline D sqrt(D a) {
#pragma clang fp contract(off)
  if (!(a.h > 0.0)) return mk(a.h == 0.0 ? 0.0 : __builtin_nan(""));
  const double s = ::sqrt(a.h);
  const D r = sub(a, two_prod(s, s));
  return add(mk(s), mk(r.h / (2.0 * s)));
}

__device__ inline void sincos(D a, D& sn, D& cs) {
#pragma clang fp contract(off)
  const double k = rint(a.h * 0x1.45f306dc9c883p-1);   // a / (pi/2), rounded
  D r = sub(a, two_prod(k, PIO2_1));
  r = sub(r, two_prod(k, PIO2_2));
  r = sub(r, mk(k * PIO2_3));
  const D r2 = mul(r, r);
  // sin r = r (1 - r^2/(2*3) (1 - r^2/(4*5) (...))), cos r = 1 - r^2/(1*2) (1 - r^2/(3*4) (...))
  D s = mk(1.0), c = mk(1.0);
  for (int i = 14; i >= 1; --i) {
    s = sub(mk(1.0), div(mul(s, r2), mk((double)((2 * i) * (2 * i + 1)))));
    c = sub(mk(1.0), div(mul(c, r2), mk((double)((2 * i - 1) * (2 * i)))));
  }
  s = mul(s, r);
  const int q = (((int)k % 4) + 4) % 4;
  if (q == 0) {
    sn = s;
    cs = c;
  } else if (q == 1) {
    sn = c;
    cs = neg(s);
  } else if (q == 2) {
    sn = neg(s);
    cs = neg(c);
  } else {
    sn = neg(c);
    cs = s;
  }
}

__device__ inline D atan2(D y, D x) {
#pragma clang fp contract(off)
  const double t0 = ::atan2(y.h, x.h);
  if ((x.h == 0.0 && y.h == 0.0) || !isfinite(t0)) return mk(t0);
  D s, c;
  sincos(mk(t0), s, c);
  const D num = sub(mul(y, c), mul(x, s));
  const D den = add(mul(x, c), mul(y, s));
  return add(mk(t0), div(num, den));
}

struct Z {
  D re, im;
};

__device__ __forceinline__ Z zre(D a) { return Z{a, mk(0.0)}; }
__device__ __forceinline__ Z zadd(Z a, Z b) { return Z{add(a.re, b.re), add(a.im, b.im)}; }
__device__ __forceinline__ Z zsub(Z a, Z b) { return Z{sub(a.re, b.re), sub(a.im, b.im)}; }
__device__ __forceinline__ Z zmul(Z a, Z b) {
  return Z{sub(mul(a.re, b.re), mul(a.im, b.im)), add(mul(a.re, b.im), mul(a.im, b.re))};
}
__device__ __forceinline__ Z zmul(Z a, D b) { return Z{mul(a.re, b), mul(a.im, b)}; }
__device__ __forceinline__ Z zmul(Z a, double b) { return Z{mul(a.re, b), mul(a.im, b)}; }
__device__ __forceinline__ Z zinv(Z a) {
  const D d = add(mul(a.re, a.re), mul(a.im, a.im));
  return Z{div(a.re, d), neg(div(a.im, d))};
}

// Principal log; a real negative argument takes arg = -pi (the side F - i0 approaches).
__device__ inline Z zlog_mi0(Z p) {
#pragma clang fp contract(off)
  const D m2 = add(mul(p.re, p.re), mul(p.im, p.im));
  const D lr = scale2(log(m2), -1);
  if (p.im.h == 0.0 && p.im.l == 0.0 && p.re.h < 0.0) return Z{lr, D{-PI_HI, -PI_LO}};
  return Z{lr, atan2(p.im, p.re)};
}

__device__ inline Z zexp(Z a) {
  D s, c;
  sincos(a.im, s, c);
  const D e = exp(a.re);
  return Z{mul(e, c), mul(e, s)};
}

// sum_t coef_t prod_j v_j^e_tj over a term list (exponent bits x, x^2, x^4 per
// variable), at real points
__device__ inline D poly_dd(CTerm* t, uint32_t cnt, int n, const D* v) {
  D P = mk(0.0);
  for (uint32_t u = 0; u < cnt; ++u) {
    const uint64_t e = t[u].exps;
    D m = mk(t[u].coef);
    for (int j = 0; j < n; ++j) {
      const int nib = (int)((e >> (4 * j)) & 0xfu);
      const int pw = (nib & 1) + 2 * ((nib >> 1) & 1) + 4 * ((nib >> 2) & 1);
      for (int q = 0; q < pw; ++q) m = mul(m, v[j]);
    }
    P = add(P, m);
  }
  return P;
}

// the same at complex points; tim: imaginary parts of the coefficients, or null
__device__ inline Z poly_zdd(CTerm* t, const SDI_TAPE double* tim, uint32_t cnt, int n, const Z* v) {
  Z P = zre(mk(0.0));
  for (uint32_t u = 0; u < cnt; ++u) {
    const uint64_t e = t[u].exps;
    Z m = Z{mk(t[u].coef), mk(tim ? tim[u] : 0.0)};
    for (int j = 0; j < n; ++j) {
      const int nib = (int)((e >> (4 * j)) & 0xfu);
      const int pw = (nib & 1) + 2 * ((nib >> 1) & 1) + 4 * ((nib >> 2) & 1);
      for (int q = 0; q < pw; ++q) m = zmul(m, v[j]);
    }
    P = zadd(P, m);
  }
  return P;
}

}  // namespace xdd

// Largest variable count of a deformed sector.
constexpr int MAXV_CPLX = 8;

// f_kk (kk = k + ns) of one complex-mode sector at one point (internal
// variable order), the formula of eval_f_cplx_c in double-double; f (real and
// imaginary parts) and cnd (the sums of |term| per order) are rounded to fp64
// at the end.  The Im F(z) > 0 flags are left to the fp64 evaluation of the
// same point.
template <int KM>
__device__ __attribute__((noinline)) void eval_f_cplx_dd(CSec* S, const SDI_TAPE CplxDev* X, CU32* dir,
                                                         CTerm* terms, const double* x, double* f_re,
                                                         double* f_im, double* cnd_out) {
#pragma clang fp contract(off)
  using namespace xdd;
  constexpr int NT = MAXV_CPLX * (MAXV_CPLX + 1) / 2;
  const int n = S->n;
  const int ns = S->ns;
  const int kf = S->kf;
  const int nfac = S->nfac;
  const double lam = X->lam;
  const int facf = X->fac_f;

  D xd[MAXV_CPLX], lx[MAXS], ix[MAXS];
  for (int j = 0; j < n; ++j) xd[j] = mk(x[j]);
  for (int i = 0; i < ns; ++i) {
    lx[i] = log(xd[i]);
    ix[i] = div(mk(1.0), xd[i]);
  }
  // L_rest = sum_{j >= ns} b_j ln x_j and the monomial exp(sum_{j >= ns} a_j ln x_j)
  D lrest = mk(0.0), la = mk(0.0);
  for (int j = ns; j < n; ++j) {
    const D l = log(xd[j]);
    lrest = add(lrest, mul(l, S->b[j]));
    la = add(la, mul(l, S->a[j]));
  }
  const D mono = exp(la);

  Z f[KM];
  double c[KM];
  for (int k = 0; k < KM; ++k) {
    f[k] = zre(mk(0.0));
    c[k] = 0.0;
  }
  const int C = 1 << ns;
  for (int W = 0; W < C; ++W) {
    D y[MAXV_CPLX], g[MAXV_CPLX];
    for (int j = 0; j < n; ++j) {
      y[j] = (j < ns && ((W >> j) & 1)) ? mk(0.0) : xd[j];
      g[j] = mk(0.0);
      if (facf >= 0) {
        CU32* d = dir + (size_t)X->dir_off + ((size_t)j * MAXC + W) * 2;
        g[j] = poly_dd(terms + d[0], d[1], n, xd);
      }
    }
    // det(I - i lam S), S = D_a + D_y^(1/2) H D_y^(1/2), by LDL^T of the lower triangle
    Z det = zre(mk(1.0));
    {
      Z A[NT];
      D r[MAXV_CPLX], yy[MAXV_CPLX];
      for (int j = 0; j < n; ++j) {
        yy[j] = mul(y[j], sub(mk(1.0), y[j]));
        r[j] = sqrt(yy[j]);
      }
      for (int j = 0; j < n; ++j) {
        for (int k = 0; k <= j; ++k) {
          const int q = j * (j + 1) / 2 + k;
          A[q] = zre(mk(j == k ? 1.0 : 0.0));
          if (facf >= 0) {
            const int dd = n + j * (j + 1) / 2 + k;
            CU32* d = dir + (size_t)X->dir_off + ((size_t)dd * MAXC + W) * 2;
            const D h = poly_dd(terms + d[0], d[1], n, xd);
            D sjk = mul(mul(r[j], r[k]), h);
            if (j == k) sjk = add(mul(sub(mk(1.0), scale2(y[j], 1)), g[j]), mul(yy[j], h));
            A[q].im = neg(mul(sjk, lam));
          }
        }
      }
      for (int k = 0; k < n; ++k) {
        const Z dk = A[k * (k + 1) / 2 + k];
        det = zmul(det, dk);
        const Z inv = zinv(dk);
        for (int i = k + 1; i < n; ++i) {
          const Z lik = zmul(A[i * (i + 1) / 2 + k], inv);
          for (int j = k + 1; j <= i; ++j)
            A[i * (i + 1) / 2 + j] = zsub(A[i * (i + 1) / 2 + j], zmul(lik, A[j * (j + 1) / 2 + k]));
        }
      }
    }
    // deformed point and the logarithms of w_j = 1 - i t_j, t_j = lam (1 - y_j) g_j
    Z z[MAXV_CPLX];
    Z lg = zre(mk(0.0)), lw = zre(mk(0.0));
    for (int j = 0; j < n; ++j) {
      const D t = mul(mul(sub(mk(1.0), y[j]), g[j]), lam);
      z[j] = Z{y[j], neg(mul(y[j], t))};
      const Z l = zlog_mi0(Z{mk(1.0), neg(t)});
      lg = zadd(lg, zmul(l, S->a[j]));
      lw = zadd(lw, zmul(l, S->b[j]));
    }
    for (int fm = 0; fm < nfac; ++fm) {
      const Z P = poly_zdd(terms + S->tab_off[fm][W], coef_im_at(X, S->tab_off[fm][W]), S->tab_cnt[fm][W], n, z);
      const Z l = zlog_mi0(P);
      lg = zadd(lg, zmul(l, S->gam[fm]));
      lw = zadd(lw, zmul(l, S->del[fm]));
    }
    const Z g0 = zmul(det, zexp(lg));
    for (int T = W;; T = (T - 1) & W) {
      const int off = ns - __builtin_popcount(T);
      D coef = mk(1.0);
      D zr = lrest;
      for (int i = 0; i < ns; ++i) {
        if ((T >> i) & 1) {
          coef = div(coef, mk(S->bS[i]));
        } else {
          coef = mul(coef, ix[i]);
          zr = add(zr, mul(lx[i], S->bS[i]));
        }
      }
      if (__builtin_popcount(W & ~T) & 1) coef = neg(coef);
      const Z zz = Z{add(zr, lw.re), lw.im};
      Z t = zmul(g0, coef);
      for (int kk = off; kk < KM && kk < kf; ++kk) {
        f[kk] = zadd(f[kk], t);
        c[kk] += hypot(t.re.h, t.im.h);
        t = zmul(zmul(t, zz), div(mk(1.0), mk((double)(kk - off + 1))));
      }
      if (T == 0) break;
    }
  }
  for (int k = 0; k < KM; ++k) {
    const Z v = zmul(f[k], mono);
    f_re[k] = v.re.h + v.re.l;
    f_im[k] = v.im.h + v.im.l;
    cnd_out[k] = c[k] * fabs(mono.h);
  }
}

}  // namespace sdi
