// Subregion-adaptive Monte Carlo (integrator 3, the role of suaveCuba among
// the CurrentIntegrator options of section 4.4) on the dyadic regions of the
// adaptive cubature: per region N pseudo-random points, the region's value and
// standard errors per result order, and the axis along which the samples'
// spread suggests halving it.
//
// Point p of region number r, caller variable c: Philox4x32-10 with key = the
// seed's 32-bit halves and counter (p, c, r mod 2^32, (r / 2^32) xor
// 0x53554156); u = (b + 1/2) 2^-52 from the top 52 bits b of the first two
// words; x_c = lo_c + u_c w_c (w_c a power of two, so one rounding).  Values:
// vol * S1 / N; errors vol * sqrt(var / N), var = max(0, (S2 - S1^2 / N) /
// (N - 1)) per real and imaginary part, S1 and S2 double-double sums.  Axis:
// with g = sum_k omega_k |F_k|_1 and the samples split by u_c < 1/2, the
// variable with the smallest sum of the halves' spreads sqrt(mean g^2 -
// (mean g)^2), compared at 8 significant bits (ties: the lowest variable; a
// half with fewer than 2 samples: infinite; all infinite: variable 0).
//
// One wave per region; the lanes take points p = lane, lane + 64, ... .
//
// DIV (the partition phase of integrator 4, divonne.hpp): the counter's last
// word is (r / 2^32) xor A.tag, and instead of the spreads the statistic is
// the range of g: the region's spread vol (max g - min g) / 2 goes to
// out_spread, and the axis is the variable whose halves' ranges
// max_h (max_h g - min_h g) are the smallest (8 significant bits, ties the
// lowest variable, a half with fewer than 2 samples infinite, all infinite:
// variable 0).
#pragma once
#include "eval_cplx.hpp"
#include "kernels.h"
#include "philox.hpp"

namespace sdi {

// v > 0 rounded to 8 significant bits (the 45 lowest mantissa bits rounded
// away, half up); NaN and infinity give infinity.
__device__ __forceinline__ double coarse8(double v) {
  if (!(v <= 1.7976931348623157e308)) return __builtin_inf();
  if (v <= 0.0) return v;
  uint64_t b = __builtin_bit_cast(uint64_t, v);
  b = (b + (1ull << 44)) & ~((1ull << 45) - 1);
  return __builtin_bit_cast(double, b);
}

// Double-double sum over the 64 lanes (every lane ends with the total).
__device__ __forceinline__ void wave_dd(double& hi, double& lo) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double h2 = __shfl_xor(hi, o, 64);
    const double l2 = __shfl_xor(lo, o, 64);
    dd_add(hi, lo, h2, l2);
  }
}

template <int NV, int KM, bool CPLX, bool DIV = false>
__global__ void __launch_bounds__(BLOCK) k_suave(SuaveArgs A) {
  const uint32_t tag = DIV ? A.tag : 0x53554156u;
  constexpr int WPB = BLOCK / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
  for (int64_t r0 = (int64_t)blockIdx.x * WPB; r0 < A.nreg; r0 += (int64_t)gridDim.x * WPB) {
    const int64_t r = r0 + wave;
    if (r >= A.nreg) continue;   // wave-uniform: no block-level synchronisation below
    const int s = __builtin_amdgcn_readfirstlane(A.reg_sector[r]);
    CSec* S = tape(A.secs + s);
    const int n = S->n;
    const int K = S->K;
    const int64_t uid = A.uid0 + r;
    double lo_c[NV], w_c[NV];
    int levsum = 0;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      lo_c[c] = 0.0;
      w_c[c] = 1.0;
      if (c < n) {
        const int lev = A.reg_level[r * MAXV + c];
        w_c[c] = ldexp(1.0, -lev);
        lo_c[c] = (double)A.reg_index[r * MAXV + c] * w_c[c];
        levsum += lev;
      }
    }
    const double vol = ldexp(1.0, -levsum);
    double s1r[KMAX], c1r[KMAX], s1i[KMAX], c1i[KMAX], s2r[KMAX], c2r[KMAX], s2i[KMAX], c2i[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) s1r[k] = c1r[k] = s1i[k] = c1i[k] = s2r[k] = c2r[k] = s2i[k] = c2i[k] = 0.0;
    double gl[NV], g2l[NV], gt = 0.0, g2t = 0.0;
    int nl[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      gl[c] = g2l[c] = 0.0;
      nl[c] = 0;
    }
    // DIV: gl / g2l hold min and max of g over the lower half, gt / g2t over
    // the whole region, and the upper half's in hl / h2l
    double hl[DIV ? NV : 1], h2l[DIV ? NV : 1];
    if constexpr (DIV) {
      gt = __builtin_inf();
      g2t = -__builtin_inf();
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        gl[c] = hl[c] = __builtin_inf();
        g2l[c] = h2l[c] = -__builtin_inf();
      }
    }
    int nonfin = 0, npos = 0;
    for (int p = lane; p < A.npts; p += 64) {
      double u[NV], xc[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        u[c] = 0.5;
        xc[c] = 0.5;
        if (c < n) {
          uint32_t ctr[4] = {(uint32_t)p, (uint32_t)c, (uint32_t)uid, (uint32_t)(uid >> 32) ^ tag};
          philox4x32_10(ctr, k0, k1);
          const uint64_t b = ((uint64_t)ctr[0] << 20) | (ctr[1] >> 12);
          u[c] = ((double)b + 0.5) * 0x1p-52;
          xc[c] = lo_c[c] + u[c] * w_c[c];   // w_c a power of two: the product is exact
        }
      }
      double x[1][NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        double v = 0.5;
#pragma unroll
        for (int c = 0; c < NV; ++c)
          if (j < n && c == S->perm[j]) v = xc[c];
        x[0][j] = v;
      }
      double fv[KM * (CPLX ? 2 : 1)];
      if constexpr (CPLX) {
        cd f[1][KM];
        int imf[1];
        eval_f_cplx<NV, 1, KM>(S, tape(A.cx) + s, tape(A.dir), tape(A.terms), x, f, imf);
        npos += imf[0] ? 1 : 0;
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) {
          fv[2 * kk] = f[0][kk].re;
          fv[2 * kk + 1] = f[0][kk].im;
        }
      } else {
        double f[1][KM];
        eval_f_real<NV, 1, KM>(S, tape(A.terms), x, f);
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) fv[kk] = f[0][kk];
      }
      bool fin = true;
      double g = 0.0;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
          double re = 0.0, im = 0.0;
#pragma unroll
          for (int kk = 0; kk < KM; ++kk) {
            if constexpr (CPLX) {
              re += S->fold_re[k][kk] * fv[2 * kk] - S->fold_im[k][kk] * fv[2 * kk + 1];
              im += S->fold_re[k][kk] * fv[2 * kk + 1] + S->fold_im[k][kk] * fv[2 * kk];
            } else {
              re += S->fold_re[k][kk] * fv[kk];
              im += S->fold_im[k][kk] * fv[kk];
            }
          }
          fin = fin && isfinite(re) && isfinite(im);
          two_sum_acc(s1r[k], c1r[k], re);
          two_sum_acc(s1i[k], c1i[k], im);
          two_sum_acc(s2r[k], c2r[k], re * re);
          two_sum_acc(s2i[k], c2i[k], im * im);
          g += A.omega[k] * (fabs(re) + fabs(im));
        }
      }
      nonfin += fin ? 0 : 1;
      if constexpr (DIV) {
        gt = fmin(gt, g);
        g2t = fmax(g2t, g);
#pragma unroll
        for (int c = 0; c < NV; ++c)
          if (c < n) {
            if (u[c] < 0.5) {
              gl[c] = fmin(gl[c], g);
              g2l[c] = fmax(g2l[c], g);
              nl[c] += 1;
            } else {
              hl[c] = fmin(hl[c], g);
              h2l[c] = fmax(h2l[c], g);
            }
          }
      } else {
        gt += g;
        g2t += g * g;
#pragma unroll
        for (int c = 0; c < NV; ++c)
          if (c < n && u[c] < 0.5) {
            gl[c] += g;
            g2l[c] += g * g;
            nl[c] += 1;
          }
      }
    }
    // reductions: the double-double sums per order, the axis statistics
    double v1r[KMAX], v1i[KMAX], v2r[KMAX], v2i[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      double h = s1r[k] + c1r[k], l = c1r[k] - (h - s1r[k]);
      wave_dd(h, l);
      v1r[k] = h + l;
      h = s1i[k] + c1i[k];
      l = c1i[k] - (h - s1i[k]);
      wave_dd(h, l);
      v1i[k] = h + l;
      h = s2r[k] + c2r[k];
      l = c2r[k] - (h - s2r[k]);
      wave_dd(h, l);
      v2r[k] = h + l;
      h = s2i[k] + c2i[k];
      l = c2i[k] - (h - s2i[k]);
      wave_dd(h, l);
      v2i[k] = h + l;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      if constexpr (DIV) {
        gt = fmin(gt, __shfl_xor(gt, o, 64));
        g2t = fmax(g2t, __shfl_xor(g2t, o, 64));
      } else {
        gt += __shfl_xor(gt, o, 64);
        g2t += __shfl_xor(g2t, o, 64);
      }
      nonfin += __shfl_xor(nonfin, o, 64);
      npos += __shfl_xor(npos, o, 64);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        if constexpr (DIV) {
          gl[c] = fmin(gl[c], __shfl_xor(gl[c], o, 64));
          g2l[c] = fmax(g2l[c], __shfl_xor(g2l[c], o, 64));
          hl[c] = fmin(hl[c], __shfl_xor(hl[c], o, 64));
          h2l[c] = fmax(h2l[c], __shfl_xor(h2l[c], o, 64));
        } else {
          gl[c] += __shfl_xor(gl[c], o, 64);
          g2l[c] += __shfl_xor(g2l[c], o, 64);
        }
        nl[c] += __shfl_xor(nl[c], o, 64);
      }
    if (lane == 0) {
      const double N = (double)A.npts;
      for (int k = 0; k < K; ++k) {
        double vr = 0.0, vi = 0.0, m1r = 0.0, m1i = 0.0;
#pragma unroll
        for (int kk = 0; kk < KMAX; ++kk)
          if (kk == k) {
            m1r = v1r[kk];
            m1i = v1i[kk];
            vr = (v2r[kk] - v1r[kk] * v1r[kk] / N) / (N - 1.0);
            vi = (v2i[kk] - v1i[kk] * v1i[kk] / N) / (N - 1.0);
          }
        double* ov = A.out_val + (r * A.K + k) * 2;
        double* oe = A.out_err + (r * A.K + k) * 2;
        ov[0] = vol * (m1r / N);
        ov[1] = vol * (m1i / N);
        oe[0] = vol * sqrt((vr > 0.0 ? vr : 0.0) / N);
        oe[1] = vol * sqrt((vi > 0.0 ? vi : 0.0) / N);
      }
      double best = __builtin_inf();
      int axis = 0;
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        if (c < n) {
          const int a = nl[c], bcount = A.npts - nl[c];
          if (a >= 2 && bcount >= 2) {
            double phi;
            if constexpr (DIV) {
              phi = coarse8(fmax(g2l[c] - gl[c], h2l[c] - hl[c]));
            } else {
              const double ml = gl[c] / a, mr = (gt - gl[c]) / bcount;
              const double ql = g2l[c] / a - ml * ml, qr = (g2t - g2l[c]) / bcount - mr * mr;
              phi = coarse8(sqrt(ql > 0.0 ? ql : 0.0) + sqrt(qr > 0.0 ? qr : 0.0));
            }
            if (phi < best) {
              best = phi;
              axis = c;
            }
          }
        }
      }
      A.out_axis[r] = axis;
      if constexpr (DIV) A.out_spread[r] = vol * (g2t - gt) * 0.5;
      A.out_count[2 * r] = nonfin;
      A.out_count[2 * r + 1] = npos;
    }
  }
}

}  // namespace sdi
