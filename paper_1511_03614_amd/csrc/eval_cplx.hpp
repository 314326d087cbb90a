// Complex-mode (contour-deformed) sector-integrand evaluation on gfx950.
//
// ComplexMode of the paper (section 4.4) moves the sector variables off the
// real cube, z_j = y_j - i lam y_j (1 - y_j) dF/dy_j with F the sector's
// deformation polynomial y^m P_F (P_F the reduced F factor, which has a
// constant term; m the optional monomial of the sector, zero by default), so
// that Im F(z) <= 0 (the F - i0 of eq. (1) and eq. (2)).  At each
// corner y = x^(W) of the pole subtraction:
//   w_j = 1 - i lam (1 - y_j) g_j,  z_j = y_j w_j,  g = grad F(y),
//   det(dz/dy) = det(I - i lam S),  S = D_a + D_y^(1/2) H D_y^(1/2),
//   D_a = diag((1 - 2 y_j) g_j), D_y = diag(y_j (1 - y_j)), H = hess F(y),
// (S is real symmetric, so the determinant is taken by an LDL^T factorisation of
// the complex symmetric matrix without pivoting: its real part is the identity,
// which keeps elimination stable), and
//   G0 = det * exp(sum_j a_j Log w_j + sum_m gamma_m Log P_m(z)),
//   Lambda = sum_j b_j Log w_j + sum_m delta_m Log P_m(z),
// with principal logarithms and arg = -pi on the negative real axis.  The
// subtraction and eps series then follow the real path with complex G0, Lambda.
// Term coefficients may be complex (complex masses); the deformation lists
// then hold the derivatives of the real part of F.
#pragma once
#include "eval_real.hpp"

namespace sdi {

struct cd {
  double re, im;
};

__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cinv(cd a) {
  const double d = a.re * a.re + a.im * a.im;
  return cd{a.re / d, -a.im / d};
}

// Principal log; a real negative argument takes arg = -pi (the side F - i0 approaches).
__device__ __forceinline__ cd clog_mi0(cd p) {
  double ang = atan2(p.im, p.re);
  if (p.im == 0.0 && p.re < 0.0) ang = -3.14159265358979323846;
  return cd{log(hypot(p.re, p.im)), ang};
}

__device__ __forceinline__ cd cexp_(cd z) {
  const double e = exp(z.re);
  double s, c;
  sincos(z.im, &s, &c);
  return cd{e * c, e * s};
}

// out += coef prod_j x_j^e_j for one term with exponent bits x, x^2, x^4; the
// bits are tested on 32-bit halves of the wave-uniform word (scalar branches).
// The powers are repeated multiplications by x: per-point squares and fourth
// powers held for the whole evaluation cost more in spills than the multiplies.
template <int NV, int PPT>
__device__ __forceinline__ void add_term3(double c, uint64_t e, const double (&x)[PPT][NV],
                                          double (&out)[PPT]) {
  double m[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) m[p] = c;
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
    if (w & (4u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] = (((m[p] * x[p][j]) * x[p][j]) * x[p][j]) * x[p][j];
    }
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] += m[p];
}

// Real polynomial with exponent bits x, x^2, x^4 (exponents up to 7), terms in
// list order.
template <int NV, int PPT>
__device__ __forceinline__ void poly_real3(CTerm* t, uint32_t cnt, const double (&x)[PPT][NV],
                                           double (&out)[PPT]) {
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] = 0.0;
  for (uint32_t i = 0; i < cnt; ++i) add_term3<NV, PPT>(t[i].coef, t[i].exps, x, out);
}

// out += (c + i ci) prod_j z_j^e_j for one term at complex points (exponents up to 3).
template <int NV, int PPT>
__device__ __forceinline__ void add_term_c(double c, double ci, uint64_t e, const cd (&z)[PPT][NV],
                                           cd (&out)[PPT]) {
  cd m[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) m[p] = cd{c, ci};
  const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const uint32_t w = j < 8 ? elo : ehi;
    const int sh = 4 * (j & 7);
    if (w & (1u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] = cmul(m[p], z[p][j]);
    }
    if (w & (2u << sh)) {
      asm volatile("" ::);
#pragma unroll
      for (int p = 0; p < PPT; ++p) m[p] = cmul(cmul(m[p], z[p][j]), z[p][j]);
    }
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] = cadd(out[p], m[p]);
}

// Polynomial at complex points (exponents up to 3), terms in list order; tim:
// the imaginary parts of the list's coefficients, or null (real coefficients).
template <int NV, int PPT>
__device__ __forceinline__ void poly_cplx(CTerm* t, const SDI_TAPE double* tim, uint32_t cnt,
                                          const cd (&z)[PPT][NV], cd (&out)[PPT]) {
#pragma unroll
  for (int p = 0; p < PPT; ++p) out[p] = cd{0.0, 0.0};
  for (uint32_t i = 0; i < cnt; ++i) add_term_c<NV, PPT>(t[i].coef, tim ? tim[i] : 0.0, t[i].exps, z, out);
}

// The imaginary parts of the coefficients of the term list at offset off, or
// null where the sector's coefficients are real.
__device__ __forceinline__ const SDI_TAPE double* coef_im_at(const SDI_TAPE CplxDev* X, uint32_t off) {
  const double* p = X->coef_im;
  return p ? tape(p) + off : nullptr;
}

// f_kk of one sector at PPT points, complex mode.  imf counts points whose F(z)
// has a positive imaginary part at some corner.
// COND: also the sums of |term| per order (cnd), for the evaluate hook.
template <int NV, int PPT, int KM, bool COND>
__device__ __forceinline__ void eval_f_cplx_c(CSec* S, const SDI_TAPE CplxDev* X, CU32* dir, CTerm* terms,
                                              const double (&x)[PPT][NV], cd (&f)[PPT][KM], int (&imf)[PPT],
                                              double (&cnd)[PPT][KM]) {
  constexpr int NT = NV * (NV + 1) / 2;
  const int n = S->n;
  const int ns = S->ns;
  const int kf = S->kf;
  const int flags = S->flags;
  const int nfac = S->nfac;
  const double lam = X->lam;
  const int facf = X->fac_f;
  double lx[PPT][MAXS], ix[PPT][MAXS];
#pragma unroll
  for (int i = 0; i < MAXS; ++i) {
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      lx[p][i] = 0.0;
      ix[p][i] = 1.0;
    }
    if (i < ns && i < NV) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        lx[p][i] = log(x[p][i < NV ? i : 0]);
        ix[p][i] = 1.0 / x[p][i < NV ? i : 0];
      }
    }
  }
  double lrest[PPT], mono[PPT];
  {
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
  for (int p = 0; p < PPT; ++p) {
    imf[p] = 0;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      f[p][k] = cd{0.0, 0.0};
      if constexpr (COND) cnd[p][k] = 0.0;
    }
  }
  const int C = 1 << ns;
  for (int W = 0; W < C; ++W) {
    // corner point y: singular variables in W are zero
    double y[PPT][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int p = 0; p < PPT; ++p) y[p][j] = (j < MAXS && ((W >> j) & 1)) ? 0.0 : x[p][j];
    // gradient of the deformation polynomial at y
    double g[PPT][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) g[p][j] = 0.0;
      if (j < n && facf >= 0) {
        double v[PPT];
        CU32* d = dir + (size_t)X->dir_off + ((size_t)j * MAXC + W) * 2;
        poly_real3<NV, PPT>(terms + d[0], d[1], x, v);
#pragma unroll
        for (int p = 0; p < PPT; ++p) g[p][j] = v[p];
      }
    }
    // det(I - i lam S) by LDL^T of the lower triangle
    cd det[PPT];
    {
      cd A[PPT][NT];
      double r[PPT][NV];
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int p = 0; p < PPT; ++p) r[p][j] = sqrt(y[p][j] * (1.0 - y[p][j]));
      int q = 0;
#pragma unroll
      for (int j = 0; j < NV; ++j) {
#pragma unroll
        for (int k = 0; k <= j; ++k, ++q) {
#pragma unroll
          for (int p = 0; p < PPT; ++p) A[p][q] = cd{j == k ? 1.0 : 0.0, 0.0};
          if (j < n && facf >= 0) {
            // second derivative (k, j), k <= j, is polynomial n + j(j+1)/2 + k
            double v[PPT];
            const int dd = n + j * (j + 1) / 2 + k;
            CU32* d = dir + (size_t)X->dir_off + ((size_t)dd * MAXC + W) * 2;
            poly_real3<NV, PPT>(terms + d[0], d[1], x, v);
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
              double sjk = r[p][j] * r[p][k] * v[p];
              if (j == k) sjk = (1.0 - 2.0 * y[p][j]) * g[p][j] + y[p][j] * (1.0 - y[p][j]) * v[p];
              A[p][q].im = -lam * sjk;
            }
          }
        }
      }
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        cd dt = cd{1.0, 0.0};
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          if (k < n) {
            const cd dk = A[p][k * (k + 1) / 2 + k];
            dt = cmul(dt, dk);
            const cd inv = cinv(dk);
#pragma unroll
            for (int i = k + 1; i < NV; ++i) {
              if (i < n) {
                const cd lik = cmul(A[p][i * (i + 1) / 2 + k], inv);
#pragma unroll
                for (int j = k + 1; j <= i; ++j)
                  A[p][i * (i + 1) / 2 + j] = csub(A[p][i * (i + 1) / 2 + j], cmul(lik, A[p][j * (j + 1) / 2 + k]));
              }
            }
          }
        }
        det[p] = dt;
      }
    }
    // deformed point, logs of w_j
    cd z[PPT][NV];
    cd lg[PPT], lam_w[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      lg[p] = cd{0.0, 0.0};
      lam_w[p] = cd{0.0, 0.0};
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        const double t = lam * (1.0 - y[p][j]) * g[p][j];
        const cd w = cd{1.0, -t};
        z[p][j] = cd{y[p][j], -y[p][j] * t};
        if (j < n) {
          const cd lw = clog_mi0(w);
          lg[p] = cadd(lg[p], cscale(lw, S->a[j]));
          lam_w[p] = cadd(lam_w[p], cscale(lw, S->b[j]));
        }
      }
    }
    // factors at z
#pragma unroll
    for (int fm = 0; fm < MAXF; ++fm) {
      if (fm < nfac) {
        cd P[PPT];
        poly_cplx<NV, PPT>(terms + S->tab_off[fm][W], coef_im_at(X, S->tab_off[fm][W]), S->tab_cnt[fm][W], z, P);
        const double gm = S->gam[fm];
        const double dm = S->del[fm];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const cd l = clog_mi0(P[p]);
          lg[p] = cadd(lg[p], cscale(l, gm));
          lam_w[p] = cadd(lam_w[p], cscale(l, dm));
          if (fm == facf) {
            cd fz = P[p];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
              const int e = X->mono_f[j];
              for (int k = 0; k < e; ++k) fz = cmul(fz, z[p][j]);
            }
            if (fz.im > 0.0) imf[p] = 1;
          }
        }
      }
    }
    // subtraction and series
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const cd g0 = cmul(det[p], cexp_(lg[p]));
      for (int T = W;; T = (T - 1) & W) {
        const int nt = __builtin_popcount(T);
        const int off = ns - nt;
        const double ib = S->invb[T];
        double coef = (__builtin_popcount(W & ~T) & 1) ? -ib : ib;
        double zr = lrest[p];
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
          if (i < ns && !((T >> i) & 1)) {
            coef *= ix[p][i];
            zr += S->bS[i] * lx[p][i];
          }
        }
        const cd zz = cd{zr + lam_w[p].re, lam_w[p].im};
        cd t = cscale(g0, coef);
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) {
          if (kk >= off && kk < kf) {
            f[p][kk] = cadd(f[p][kk], t);
            if constexpr (COND) cnd[p][kk] += hypot(t.re, t.im);
            t = cscale(cmul(t, zz), 1.0 / (double)(kk - off + 1));
          }
        }
        if (T == 0) break;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p)
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      f[p][k] = cscale(f[p][k], mono[p]);
      if constexpr (COND) cnd[p][k] *= fabs(mono[p]);
    }
  (void)flags;
}

template <int NV, int PPT, int KM>
__device__ __forceinline__ void eval_f_cplx(CSec* S, const SDI_TAPE CplxDev* X, CU32* dir, CTerm* terms,
                                            const double (&x)[PPT][NV], cd (&f)[PPT][KM], int (&imf)[PPT]) {
  double unused[PPT][KM];
  eval_f_cplx_c<NV, PPT, KM, false>(S, X, dir, terms, x, f, imf, unused);
}

}  // namespace sdi
