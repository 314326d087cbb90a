// Integrator 4, the role of divonneCuba among the CurrentIntegrator options of
// section 4.4: stratified sampling on a partition of every sector cube into
// dyadic regions of small spread.  The partition phase is k_suave with DIV
// (suave.hpp); this is the final phase: every region of the partition is
// integrated by a shifted rank-1 lattice rule of 2^m points.
//
// Region number r, shift t, caller variable c: D = (top 53 bits of
// Philox4x32-10 with key = the seed's halves and counter (c, t, r mod 2^32,
// (r / 2^32) xor 0x44495632)) | 1 (odd, so no point lands on u = 0);
// u_i = ((i z_c 2^(53-m) + D) mod 2^53) 2^-53, the tent map when baker is on,
// x_c = lo_c + u w_c.  Per shift the mean of F_k over the 2^m points
// (double-double sums); the region's value is vol times the mean of the shift
// means, its error vol times their standard error (per real and imaginary
// part), both by Welford's running update (the shift means agree to many
// digits, where the sum of squares would cancel).  One wave per region; lanes take the points i = lane, lane + 64, ...
#pragma once
#include "suave.hpp"

namespace sdi {

template <int NV, int KM, bool CPLX>
__global__ void __launch_bounds__(BLOCK) k_divonne_lattice(DivLatArgs A) {
  constexpr int WPB = BLOCK / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
  const int64_t N = (int64_t)1 << A.m;
  for (int64_t r0 = (int64_t)blockIdx.x * WPB; r0 < A.nreg; r0 += (int64_t)gridDim.x * WPB) {
    const int64_t r = r0 + wave;
    if (r >= A.nreg) continue;   // wave-uniform: no block-level synchronisation below
    const int s = __builtin_amdgcn_readfirstlane(A.reg_sector[r]);
    CSec* S = tape(A.secs + s);
    const int n = S->n;
    const int K = S->K;
    const int64_t uid = A.uid0 + r;
    double lo_c[NV], w_c[NV];
    uint64_t zp[NV];
    int levsum = 0;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      lo_c[c] = 0.0;
      w_c[c] = 1.0;
      zp[c] = 0;
      if (c < n) {
        const int lev = A.reg_level[r * MAXV + c];
        w_c[c] = ldexp(1.0, -lev);
        lo_c[c] = (double)A.reg_index[r * MAXV + c] * w_c[c];
        zp[c] = (uint64_t)A.zvec[c] << (53 - A.m);
        levsum += lev;
      }
    }
    const double vol = ldexp(1.0, -levsum);
    double m1r[KMAX], m1i[KMAX], m2r[KMAX], m2i[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) m1r[k] = m1i[k] = m2r[k] = m2i[k] = 0.0;
    int nonfin = 0, npos = 0;
    for (int t = 0; t < A.R; ++t) {
      uint64_t D[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        D[c] = 0;
        if (c < n) {
          uint32_t ctr[4] = {(uint32_t)c, (uint32_t)t, (uint32_t)uid, (uint32_t)(uid >> 32) ^ 0x44495632u};
          philox4x32_10(ctr, k0, k1);
          D[c] = ((((uint64_t)ctr[0] << 21) | (ctr[1] >> 11)) & MASK53) | 1ull;
        }
      }
      double s1r[KMAX], c1r[KMAX], s1i[KMAX], c1i[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) s1r[k] = c1r[k] = s1i[k] = c1i[k] = 0.0;
      for (int64_t i = lane; i < N; i += 64) {
        double xc[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          xc[c] = 0.5;
          if (c < n) {
            double u = lattice_coord((uint64_t)i, zp[c], D[c]);
            if (A.baker) u = tent(u);
            xc[c] = lo_c[c] + u * w_c[c];   // w_c a power of two: the product is exact
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
          }
        }
        nonfin += fin ? 0 : 1;
      }
      // the shift's means (every lane ends with them), then Welford's update
      // of their mean (m1) and sum of squared deviations (m2)
      const double tinv = 1.0 / (double)(t + 1);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        double h = s1r[k] + c1r[k], l = c1r[k] - (h - s1r[k]);
        wave_dd(h, l);
        const double qr = (h + l) / (double)N;
        h = s1i[k] + c1i[k];
        l = c1i[k] - (h - s1i[k]);
        wave_dd(h, l);
        const double qi = (h + l) / (double)N;
        const double dr = qr - m1r[k], di = qi - m1i[k];
        m1r[k] += dr * tinv;
        m1i[k] += di * tinv;
        m2r[k] += dr * (qr - m1r[k]);
        m2i[k] += di * (qi - m1i[k]);
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      nonfin += __shfl_xor(nonfin, o, 64);
      npos += __shfl_xor(npos, o, 64);
    }
    if (lane == 0) {
      const double R = (double)A.R;
      for (int k = 0; k < K; ++k) {
        double ar = 0.0, ai = 0.0, vr = 0.0, vi = 0.0;
#pragma unroll
        for (int kk = 0; kk < KMAX; ++kk)
          if (kk == k) {
            ar = m1r[kk];
            ai = m1i[kk];
            vr = m2r[kk] / (R - 1.0);
            vi = m2i[kk] / (R - 1.0);
          }
        double* ov = A.out_val + (r * A.K + k) * 2;
        double* oe = A.out_err + (r * A.K + k) * 2;
        ov[0] = vol * ar;
        ov[1] = vol * ai;
        oe[0] = vol * sqrt((vr > 0.0 ? vr : 0.0) / R);
        oe[1] = vol * sqrt((vi > 0.0 ? vi : 0.0) / R);
      }
      A.out_count[2 * r] = nonfin;
      A.out_count[2 * r + 1] = npos;
    }
  }
}

}  // namespace sdi
