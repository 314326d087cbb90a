// The rule pair of the adaptive deterministic cubature (the cuhreCuba option
// of CurrentIntegrator, section 4.4) on dyadic regions of the sector cubes.
//
// Rule (Genz and Malik, J. Comput. Appl. Math. 6 (1980) 295): on [-1, 1]^n
// the degree-7 rule takes the centre, +-l2 e_i, +-l3 e_i, +-l4 e_i +- l4 e_j
// (i < j) and the 2^n corners (+-l5, ..., +-l5); the embedded degree-5 rule
// the first four classes.  A region with centre c and half-widths h maps node
// xi to c + xi h.  Per region the kernel returns, for every result order k,
// vol * S7_k, vol * |Re(S7_k - S5_k)|, vol * |Im(S7_k - S5_k)| (S7, S5 the
// weighted node sums), the rounding scale sigma_k = vol u sum_p (|w7_p| +
// |w5_p|) |F_k(x_p)|_1 (u = 2^-52, |z|_1 = |Re z| + |Im z|), and the split
// axis: the lowest caller variable j whose D_j = max_k omega_k |Delta_jk|_1
// is within 2^20 nu of the largest, Delta_j the fourth divided difference
//   (F(c + l2 h_j e_j) + F(c - l2 h_j e_j) - 2F(c))
//     - (l2^2 / l3^2) (F(c + l3 h_j e_j) + F(c - l3 h_j e_j) - 2F(c))
// and nu = u max_k omega_k max_p |F_k(x_p)|_1 over the centre and the axis
// nodes (smaller differences are rounding noise; a NaN counts as infinite).
//
// One wave per region: the lanes take the nodes in turn (node p = lane,
// lane + 64, ...), so a region of n variables costs ceil(P(n) / 64) rounds,
// P(n) = 1 + 4n + 2n(n-1) + 2^n.  Node sums are reduced across the wave in a
// fixed order; the centre and the 4n axis nodes are kept in LDS for the
// fourth differences, folded into result orders.  The rule sums run over the
// internal f orders and are folded once per region (the fold is linear); the
// rounding scale needs |F_k| per node, so each node is folded too.
#pragma once
#include "eval_cplx.hpp"
#include "kernels.h"

namespace sdi {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Node p of the rule in n variables: its weight class (0 centre, 1 l2 axis,
// 2 l3 axis, 3 l4 pairs, 4 l5 corners) and its coordinate along caller
// variable c.  Order: centre; class 1 by axis, + before -; class 2 likewise;
// pairs (i < j, i outer) with signs ++, +-, -+, --; corners with the sign of
// variable c in bit n-1-c of the corner index (set: negative).
struct Node {
  int cls, a, b;      // class; axes (class 1, 2: a; class 3: a < b)
  int sa, sb;         // signs of a and b (+1 / -1); class 4: corner index in sa
};

__device__ __forceinline__ Node decode_node(int p, int n) {
  Node d{0, -1, -1, 1, 1};
  if (p == 0) return d;
  int q = p - 1;
  if (q < 2 * n) {
    d.cls = 1;
    d.a = q >> 1;
    d.sa = (q & 1) ? -1 : 1;
    return d;
  }
  q -= 2 * n;
  if (q < 2 * n) {
    d.cls = 2;
    d.a = q >> 1;
    d.sa = (q & 1) ? -1 : 1;
    return d;
  }
  q -= 2 * n;
  const int npair4 = 2 * n * (n - 1);
  if (q < npair4) {
    d.cls = 3;
    int pair = q >> 2;
    d.sa = (q & 2) ? -1 : 1;
    d.sb = (q & 1) ? -1 : 1;
    int i = 0;
    while (pair >= n - 1 - i) {
      pair -= n - 1 - i;
      ++i;
    }
    d.a = i;
    d.b = i + 1 + pair;
    return d;
  }
  d.cls = 4;
  d.sa = q - npair4;
  return d;
}

__device__ __forceinline__ double node_coord(const Node& d, int c, int n, const double (&lam)[4]) {
  switch (d.cls) {
    case 1: return c == d.a ? d.sa * lam[0] : 0.0;
    case 2: return c == d.a ? d.sa * lam[1] : 0.0;
    case 3: return c == d.a ? d.sa * lam[2] : (c == d.b ? d.sb * lam[2] : 0.0);
    case 4: return ((d.sa >> (n - 1 - c)) & 1) ? -lam[3] : lam[3];
    default: return 0.0;
  }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

template <int NV, int KM, bool CPLX>
__global__ void __launch_bounds__(BLOCK) k_cubature(CubArgs A) {
  constexpr int WPB = BLOCK / 64;
  constexpr int NF = CPLX ? 2 : 1;           // doubles per internal-order value
  constexpr int NSLOT = 1 + 4 * NV;
  constexpr double U = 0x1p-52, NOISE = 0x1p20;
  __shared__ double lf[WPB][NSLOT][2 * KMAX]; // folded centre and axis-node values per wave
  __shared__ double ld[WPB][NV];              // D_j per caller variable
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t r0 = (int64_t)blockIdx.x * WPB; r0 < A.nreg; r0 += (int64_t)gridDim.x * WPB) {
    const int64_t r = r0 + wave;
    const bool act = r < A.nreg;
    double a7[KM * NF], a5[KM * NF], sg[KMAX];
#pragma unroll
    for (int i = 0; i < KM * NF; ++i) a7[i] = a5[i] = 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) sg[k] = 0.0;
    int nonfin = 0, npos = 0, n = 0, s = 0;
    double vol = 1.0;
    CSec* S = nullptr;
    if (act) {
      s = __builtin_amdgcn_readfirstlane(A.reg_sector[r]);
      S = tape(A.secs + s);
      n = S->n;
      // centre and half-width per internal variable (caller variable perm[j])
      double cen[NV], half[NV];
      int levsum = 0;
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        cen[j] = 0.5;
        half[j] = 0.0;
        if (j < n) {
          const int c = S->perm[j];
          const int lev = A.reg_level[r * MAXV + c];
          const uint32_t idx = A.reg_index[r * MAXV + c];
          half[j] = ldexp(0.5, -lev);
          cen[j] = (2.0 * (double)idx + 1.0) * half[j];
          levsum += lev;
        }
      }
      vol = ldexp(1.0, -levsum);
      const double lam[4] = {A.lam[0], A.lam[1], A.lam[2], A.lam[3]};
      const int npts = 1 + 4 * n + 2 * n * (n - 1) + (1 << n);
      const double* wt = A.wtab + n * 10;
      for (int p = lane; p < npts; p += 64) {
        const Node d = decode_node(p, n);
        double x[1][NV];
#pragma unroll
        for (int j = 0; j < NV; ++j)
          x[0][j] = j < n ? cen[j] + node_coord(d, S->perm[j], n, lam) * half[j] : 0.5;
        const double w7 = wt[d.cls], w5 = wt[5 + d.cls];
        double fv[KM * NF];
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
        for (int i = 0; i < KM * NF; ++i) {
          fin = fin && isfinite(fv[i]);
          a7[i] += w7 * fv[i];
          a5[i] += w5 * fv[i];
        }
        nonfin += fin ? 0 : 1;
        // the node's result orders: rounding scale, and the axis nodes' values
        const double wa = fabs(w7) + fabs(w5);
        const bool axis_node = p < 1 + 4 * n;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          if (k < S->K) {
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
            sg[k] += wa * (fabs(re) + fabs(im));
            if (axis_node) {
              lf[wave][p][2 * k] = re;
              lf[wave][p][2 * k + 1] = im;
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < KM * NF; ++i) {
        a7[i] = wave_sum(a7[i]);
        a5[i] = wave_sum(a5[i]);
      }
#pragma unroll
      for (int k = 0; k < KMAX; ++k) sg[k] = wave_sum(sg[k]);
      nonfin = wave_sum_i(nonfin);
      npos = wave_sum_i(npos);
    }
    __syncthreads();
    if (act) {
      const int K = S->K;
      // fourth differences: lane c handles caller variable c
      if (lane < n) {
        const int c = lane;
        const double r17 = 1.0 / 7.0;        // l2^2 / l3^2
        double m = 0.0;
        bool bad = false;
        for (int k = 0; k < K; ++k) {
          double d1 = 0.0;
          for (int q = 0; q < 2; ++q) {
            const int i = 2 * k + q;
            const double f0 = lf[wave][0][i];
            const double d2 = lf[wave][1 + 2 * c][i] + lf[wave][2 + 2 * c][i] - 2.0 * f0;
            const double d3 = lf[wave][1 + 2 * n + 2 * c][i] + lf[wave][2 + 2 * n + 2 * c][i] - 2.0 * f0;
            d1 += fabs(d2 - r17 * d3);
          }
          const double v = A.omega[k] * d1;
          bad = bad || isnan(v);
          m = v > m ? v : m;
        }
        ld[wave][c] = bad ? __builtin_inf() : m;
      }
      // nu: largest weighted |F_k|_1 over the centre and the axis nodes
      double nu = 0.0;
      bool nbad = false;
      for (int p = lane; p < 1 + 4 * n; p += 64)
        for (int k = 0; k < K; ++k) {
          const double v = A.omega[k] * (fabs(lf[wave][p][2 * k]) + fabs(lf[wave][p][2 * k + 1]));
          nbad = nbad || isnan(v);
          nu = v > nu ? v : nu;
        }
      nu = wave_max(nbad ? __builtin_inf() : nu);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // lane k < K writes order k
      if (lane < K) {
        const int k = lane;
        double r7 = 0.0, i7 = 0.0, r5 = 0.0, i5 = 0.0;
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) {
          if constexpr (CPLX) {
            r7 += S->fold_re[k][kk] * a7[2 * kk] - S->fold_im[k][kk] * a7[2 * kk + 1];
            i7 += S->fold_re[k][kk] * a7[2 * kk + 1] + S->fold_im[k][kk] * a7[2 * kk];
            r5 += S->fold_re[k][kk] * a5[2 * kk] - S->fold_im[k][kk] * a5[2 * kk + 1];
            i5 += S->fold_re[k][kk] * a5[2 * kk + 1] + S->fold_im[k][kk] * a5[2 * kk];
          } else {
            r7 += S->fold_re[k][kk] * a7[kk];
            i7 += S->fold_im[k][kk] * a7[kk];
            r5 += S->fold_re[k][kk] * a5[kk];
            i5 += S->fold_im[k][kk] * a5[kk];
          }
        }
        double* ov = A.out_val + (r * A.K + k) * 2;
        double* oe = A.out_err + (r * A.K + k) * 2;
        ov[0] = vol * r7;
        ov[1] = vol * i7;
        oe[0] = vol * fabs(r7 - r5);
        oe[1] = vol * fabs(i7 - i5);
        double sk = 0.0;
#pragma unroll
        for (int kk = 0; kk < KMAX; ++kk) sk = kk == k ? sg[kk] : sk;
        A.out_sig[r * A.K + k] = vol * U * sk;
      }
      if (lane == 0) {
        double top = 0.0;
        for (int c = 0; c < n; ++c) top = ld[wave][c] > top ? ld[wave][c] : top;
        const double tol = nu <= 1.7976931348623157e308 ? NOISE * U * nu : 0.0;
        int axis = 0;
        for (int c = n - 1; c >= 0; --c)
          if (ld[wave][c] >= top - tol) axis = c;
        A.out_axis[r] = axis;
        A.out_count[2 * r] = nonfin;
        A.out_count[2 * r + 1] = npos;
      }
    }
    __syncthreads();
  }
}

}  // namespace sdi
