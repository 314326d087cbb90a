// Small kernels around the tile pass: Philox shifts, fixed-order reductions of
// tile partials, per-sector estimates and their combination, Vegas histogram
// reduction and grid refit, and the point-sampling hook.
#include <hip/hip_runtime.h>

#include "eval_real.hpp"
#include "kernels.h"
#include "philox.hpp"

namespace sdi {

// ------------------------------------------------------------ fill (graph-safe zeroing)

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------ Philox4x32-10 shifts

// D_{s,r,j}: 53 bits (word0 << 21 | word1 >> 11) of Philox(key = seed, counter =
// (j, row0 + r, s, t)), redrawn (t = 1, 2, ...) while D is a multiple of 2^(53-m).
__global__ void k_shifts(const SecDev* secs, int nsec, int rows, int nfinal, uint64_t seed, uint32_t row0,
                         uint64_t* shifts) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nsec * rows * MAXV) return;
  const int j = (int)(gid % MAXV);
  const int r = (int)((gid / MAXV) % rows);
  const int s = (int)(gid / ((int64_t)MAXV * rows));
  const SecDev& S = secs[s];
  uint64_t* out = shifts + ((size_t)S.shift_row + r) * MAXV + j;
  if (j >= S.n) {
    *out = 0;
    return;
  }
  const int m = r < nfinal ? S.m : S.mw;
  const uint64_t mod = 1ull << (53 - m);
  uint64_t d = 1;
  for (uint32_t t = 0; t < 64u; ++t) {
    uint32_t c[4] = {(uint32_t)j, row0 + (uint32_t)r, (uint32_t)S.sector, t};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t v = (((uint64_t)c[0] << 21) | ((uint64_t)c[1] >> 11)) & MASK53;
    if (v % mod != 0) {
      d = v;
      break;
    }
  }
  *out = d;
}

// ------------------------------------------------------------ reductions

// Per (sector, final shift): fixed-order double-double sums over the pair's
// tiles of every internal order, Q_kk = sum / N, then the prefactor fold
// Q_k = sum_kk fold[k][kk] Q_kk (linear, so it commutes with the sum).
// out: [npairs][KMAX][2] = Q_re, Q_im.  A slice of a resumable pass starts
// from the sums carried from the earlier slices (the same double-double
// additions in the same tile order as one pass over the whole lattice) and
// divides by the points done so far (npts > 0; 0: the whole lattice).
__global__ void k_reduce_pairs(const double* partial, const int32_t* pair_start, const int32_t* pair_sector,
                               const SecDev* secs, int npairs, double* out, const int32_t* nonfinite,
                               int64_t* pair_nonfinite, const double* carry_in, const int64_t* carry_in_counts,
                               double* carry_out, int64_t* carry_out_counts, int64_t npts) {
  const int pr = blockIdx.x * blockDim.x + threadIdx.x;
  if (pr >= npairs) return;
  const SecDev& S = secs[pair_sector[pr]];
  int64_t nf = carry_in_counts ? carry_in_counts[2 * pr] : 0, np = carry_in_counts ? carry_in_counts[2 * pr + 1] : 0;
  for (int t = pair_start[pr]; t < pair_start[pr + 1]; ++t) {
    nf += nonfinite[2 * t];
    np += nonfinite[2 * t + 1];
  }
  pair_nonfinite[2 * pr] = nf;
  pair_nonfinite[2 * pr + 1] = np;
  if (carry_out_counts) {
    carry_out_counts[2 * pr] = nf;
    carry_out_counts[2 * pr + 1] = np;
  }
  const double N = npts > 0 ? (double)npts : (double)(1ull << S.m);
  // only the sector's kf internal orders are written by the tile kernels
  const int kf = S.kf;
  double qr[KMAX], qi[KMAX];
  for (int kk = 0; kk < KMAX; ++kk) {
    qr[kk] = 0.0;
    qi[kk] = 0.0;
    if (kk >= kf) continue;
    double hr = 0.0, lr = 0.0, hi = 0.0, li = 0.0;
    if (carry_in) {
      const double* c = carry_in + ((size_t)pr * KMAX + kk) * 4;
      hr = c[0];
      lr = c[1];
      hi = c[2];
      li = c[3];
    }
    for (int t = pair_start[pr]; t < pair_start[pr + 1]; ++t) {
      const double* p = partial + ((size_t)t * KMAX + kk) * PART_STRIDE;
      dd_add(hr, lr, p[0], p[1]);
      dd_add(hi, li, p[2], p[3]);
    }
    if (carry_out) {
      double* c = carry_out + ((size_t)pr * KMAX + kk) * 4;
      c[0] = hr;
      c[1] = lr;
      c[2] = hi;
      c[3] = li;
    }
    qr[kk] = (hr + lr) / N;
    qi[kk] = (hi + li) / N;
  }
  for (int k = 0; k < KMAX; ++k) {
    double re = 0.0, im = 0.0;
    if (k < S.K) {
      for (int kk = 0; kk < kf; ++kk) {
        re += S.fold_re[k][kk] * qr[kk] - S.fold_im[k][kk] * qi[kk];
        im += S.fold_re[k][kk] * qi[kk] + S.fold_im[k][kk] * qr[kk];
      }
    }
    out[((size_t)pr * KMAX + k) * 2] = re;
    out[((size_t)pr * KMAX + k) * 2 + 1] = im;
  }
}

// Per sector and order: mean over the R shifts and the shift-to-shift error
// sigma^2 = sum_r (Q_r - mean)^2 / (R (R - 1)), real and imaginary apart.
// out: [nsec][KMAX][4] = mean_re, mean_im, err_re, err_im.
__global__ void k_sector_stats(const double* per_shift, int nsec, int R, double* out,
                               const int64_t* pair_nonfinite, int64_t* sec_nonfinite) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nsec * KMAX) return;
  const int s = gid / KMAX;
  const int k = gid % KMAX;
  if (k < 2) {
    int64_t nf = 0;
    for (int r = 0; r < R; ++r) nf += pair_nonfinite[2 * ((size_t)s * R + r) + k];
    sec_nonfinite[2 * s + k] = nf;
  }
  double hr = 0.0, lr = 0.0, hi = 0.0, li = 0.0;
  for (int r = 0; r < R; ++r) {
    const double* q = per_shift + (((size_t)s * R + r) * KMAX + k) * 2;
    dd_add(hr, lr, q[0], 0.0);
    dd_add(hi, li, q[1], 0.0);
  }
  const double mr = (hr + lr) / R;
  const double mi = (hi + li) / R;
  double vr = 0.0, vi = 0.0;
  for (int r = 0; r < R; ++r) {
    const double* q = per_shift + (((size_t)s * R + r) * KMAX + k) * 2;
    vr += (q[0] - mr) * (q[0] - mr);
    vi += (q[1] - mi) * (q[1] - mi);
  }
  const double den = R > 1 ? (double)R * (R - 1) : 1.0;
  double* o = out + ((size_t)s * KMAX + k) * 4;
  o[0] = mr;
  o[1] = mi;
  o[2] = R > 1 ? sqrt(vr / den) : 0.0;
  o[3] = R > 1 ? sqrt(vi / den) : 0.0;
}

// Result_k = sum_s mean_{s,k}, err_k = sqrt(sum_s err_{s,k}^2): one block per
// order; thread t sums a contiguous run of sectors in order, then a fixed
// tree over threads (deterministic).  Block KMAX sums the non-finite counts.
// res: [KMAX][4]; counts: [2].
constexpr int COMBINE_THREADS = 256;
__global__ void __launch_bounds__(COMBINE_THREADS) k_combine(const double* sec_stats, int nsec,
                                                            const int64_t* sec_nonfinite, double* res,
                                                            int64_t* counts) {
  __shared__ double sh[COMBINE_THREADS][6];
  __shared__ int64_t si[COMBINE_THREADS];
  const int k = blockIdx.x;
  const int t = threadIdx.x;
  const int chunk = (nsec + COMBINE_THREADS - 1) / COMBINE_THREADS;
  const int s0 = t * chunk;
  const int s1 = min(nsec, s0 + chunk);
  if (k < KMAX) {
    double hr = 0.0, lr = 0.0, hi = 0.0, li = 0.0, er = 0.0, ei = 0.0;
    for (int s = s0; s < s1; ++s) {
      const double* q = sec_stats + ((size_t)s * KMAX + k) * 4;
      dd_add(hr, lr, q[0], 0.0);
      dd_add(hi, li, q[1], 0.0);
      er += q[2] * q[2];
      ei += q[3] * q[3];
    }
    sh[t][0] = hr; sh[t][1] = lr; sh[t][2] = hi; sh[t][3] = li; sh[t][4] = er; sh[t][5] = ei;
    __syncthreads();
    for (int w = COMBINE_THREADS / 2; w >= 1; w >>= 1) {
      if (t < w) {
        dd_add(sh[t][0], sh[t][1], sh[t + w][0], sh[t + w][1]);
        dd_add(sh[t][2], sh[t][3], sh[t + w][2], sh[t + w][3]);
        sh[t][4] += sh[t + w][4];
        sh[t][5] += sh[t + w][5];
      }
      __syncthreads();
    }
    if (t == 0) {
      res[k * 4 + 0] = sh[0][0] + sh[0][1];
      res[k * 4 + 1] = sh[0][2] + sh[0][3];
      res[k * 4 + 2] = sqrt(sh[0][4]);
      res[k * 4 + 3] = sqrt(sh[0][5]);
    }
  } else {
    for (int c = 0; c < 2; ++c) {
      int64_t nf = 0;
      for (int s = s0; s < s1; ++s) nf += sec_nonfinite[2 * s + c];
      si[t] = nf;
      __syncthreads();
      for (int w = COMBINE_THREADS / 2; w >= 1; w >>= 1) {
        if (t < w) si[t] += si[t + w];
        __syncthreads();
      }
      if (t == 0) counts[c] = si[0];
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ Vegas

__global__ void k_grid_identity(const SecDev* secs, int nsec, double* grids) {
  const int s = blockIdx.x;
  if (s >= nsec) return;
  const SecDev& S = secs[s];
  const int nb = S.nbins;
  for (int i = threadIdx.x; i < S.n * (nb + 1); i += blockDim.x) {
    const int b = i % (nb + 1);
    grids[S.grid_off + i] = (double)b / (double)nb;
  }
}

// Sector histogram = sum of its warm-up tiles' histograms, in tile order.
__global__ void k_hist_reduce(const double* hist, const int64_t* hist_off, const int32_t* sec_tile_start,
                              const SecDev* secs, const int64_t* hsec_off, int nsec, int64_t total,
                              const int64_t* hsec_prefix, double* hsec) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  // locate sector by binary search over hsec_prefix
  int lo = 0, hi = nsec - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hsec_prefix[mid] <= gid) lo = mid; else hi = mid - 1;
  }
  const int s = lo;
  const int64_t e = gid - hsec_prefix[s];
  double acc = 0.0;
  for (int t = sec_tile_start[s]; t < sec_tile_start[s + 1]; ++t) acc += hist[hist_off[t] + e];
  hsec[hsec_off[s] + e] = acc;
  (void)secs;
}

// Lepage refit of one (sector, dimension) per block, one thread per bin:
// importance d_b = sum_k h_bk / H_k over the internal orders k, 3-point
// smoothing, compression m_b = ((r_b - 1)/ln r_b)^alpha, equal shares of
// sum m per new bin, linear inside the old bins.  The running sums are taken
// by one thread in bin order; per-bin work and the search for each new edge
// run in parallel.
__global__ void __launch_bounds__(NBMAX) k_refit(const SecDev* secs, int nsec, const double* hsec,
                                                 const int64_t* hsec_off, double* grids, double alpha) {
  __shared__ double d[NBMAX], sm[NBMAX], mm[NBMAX], cum[NBMAX + 1], g[NBMAX + 1];
  __shared__ double H[KMAX], tot_s, share_s;
  __shared__ int any_s;
  const int s = blockIdx.x / MAXV;
  const int j = blockIdx.x % MAXV;
  if (s >= nsec) return;
  const SecDev& S = secs[s];
  const int K = S.kf;        // histogram rows are the internal eps orders f_kk
  if (j >= S.n || K <= 0) return;
  const int nb = S.nbins;
  const int b = threadIdx.x;
  const double* h = hsec + hsec_off[s] + (size_t)j * nb * K;
  double* gr = grids + S.grid_off + (size_t)j * (nb + 1);
  if (b <= nb) g[b] = gr[b];
  if (b == 0) {
    any_s = 0;
    for (int k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int i = 0; i < nb; ++i) acc += h[(size_t)i * K + k];
      H[k] = acc;
      if (acc > 0.0) any_s = 1;
    }
  }
  __syncthreads();
  if (!any_s) return;
  if (b < nb) {
    double v = 0.0;
    for (int k = 0; k < K; ++k)
      if (H[k] > 0.0) v += h[(size_t)b * K + k] / H[k];
    d[b] = v;
  }
  __syncthreads();
  if (b < nb) {
    if (b == 0) sm[b] = (d[0] + d[1]) / 2.0;
    else if (b == nb - 1) sm[b] = (d[nb - 2] + d[nb - 1]) / 2.0;
    else sm[b] = (d[b - 1] + d[b] + d[b + 1]) / 3.0;
  }
  __syncthreads();
  if (b == 0) {
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) acc += sm[i];
    tot_s = acc;
  }
  __syncthreads();
  if (b < nb) {
    const double r = sm[b] / tot_s;
    double m;
    if (r == 0.0) m = 0.0;
    else if (fabs(r - 1.0) < 1e-12) m = 1.0;
    else m = pow((r - 1.0) / log(r), alpha);
    mm[b] = m;
  }
  __syncthreads();
  if (b == 0) {
    double acc = 0.0;
    cum[0] = 0.0;
    for (int i = 0; i < nb; ++i) {
      acc += mm[i];
      cum[i + 1] = acc;
    }
    share_s = acc / nb;
  }
  __syncthreads();
  if (b >= 1 && b < nb) {
    const double t = b * share_s;
    // first bin c (capped at nb-1) whose running sum passes t: cum[c] <= t < cum[c] + m_c
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cum[mid] + mm[mid] <= t) lo = mid + 1; else hi = mid;
    }
    const int c = lo;
    double frac = mm[c] > 0.0 ? (t - cum[c]) / mm[c] : 1.0;
    frac = frac < 1.0 ? frac : 1.0;
    gr[b] = g[c] + frac * (g[c + 1] - g[c]);
  }
  if (b == 0) {
    gr[0] = 0.0;
    gr[nb] = 1.0;
  }
}

// ------------------------------------------------------------ sampling hook

__global__ void k_sample_points(SampleArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.npts) return;
  const SecDev* S = A.sec;
  const int n = S->n;
  const int nb = S->nbins;
  double w = 1.0;
  for (int oj = 0; oj < n; ++oj) {
    double u = lattice_coord(A.i0 + (uint64_t)i, A.zp[oj], A.shift[oj]);
    if (S->flags & F_BAKER) u = tent(u);
    if (S->flags & F_USE_GRID) u = vegas_coord(A.grid + (size_t)oj * (nb + 1), nb, u, w);
    A.x[i * n + oj] = u;
  }
  if (A.w) A.w[i] = w;
}

// ------------------------------------------------------------ fixed scratch

// Device memory of the allocation-free entry point (sdi_sample_points_noalloc):
// the sector record, generating vector and shift row it hands to the sampling
// kernels.  Each device holds its own copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// ------------------------------------------------------------ launchers

#define SDI_CHECK(call)                    \
  do {                                     \
    hipError_t e_ = (call);                \
    if (e_ != hipSuccess) return (int)e_;  \
  } while (0)

int launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return 0;
  k_fill_i32<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(p, v, n);
  return (int)hipGetLastError();
}

int launch_shifts(const SecDev* secs, int nsec, int rows, int nfinal, uint64_t seed, uint32_t row0, uint64_t* shifts,
                  hipStream_t st) {
  const int64_t tot = (int64_t)nsec * rows * MAXV;
  k_shifts<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st>>>(secs, nsec, rows, nfinal, seed, row0, shifts);
  return (int)hipGetLastError();
}

int launch_reduce_pairs(const double* partial, const int32_t* pair_start, const int32_t* pair_sector,
                        const SecDev* secs, int npairs, double* out, const int32_t* nonfinite,
                        int64_t* pair_nonfinite, const double* carry_in, const int64_t* carry_in_counts,
                        double* carry_out, int64_t* carry_out_counts, int64_t npts, hipStream_t st) {
  if (npairs <= 0) return 0;
  k_reduce_pairs<<<dim3((unsigned)((npairs + 127) / 128)), dim3(128), 0, st>>>(
      partial, pair_start, pair_sector, secs, npairs, out, nonfinite, pair_nonfinite, carry_in, carry_in_counts,
      carry_out, carry_out_counts, npts);
  return (int)hipGetLastError();
}

int launch_sector_stats(const double* per_shift, int nsec, int R, double* out, const int64_t* pair_nonfinite,
                        int64_t* sec_nonfinite, hipStream_t st) {
  const int tot = nsec * KMAX;
  k_sector_stats<<<dim3((tot + 127) / 128), dim3(128), 0, st>>>(per_shift, nsec, R, out, pair_nonfinite,
                                                                sec_nonfinite);
  return (int)hipGetLastError();
}

int launch_combine(const double* sec_stats, int nsec, const int64_t* sec_nonfinite, double* res, int64_t* counts,
                   hipStream_t st) {
  k_combine<<<dim3(KMAX + 1), dim3(COMBINE_THREADS), 0, st>>>(sec_stats, nsec, sec_nonfinite, res, counts);
  return (int)hipGetLastError();
}

int launch_grid_identity(const SecDev* secs, int nsec, double* grids, hipStream_t st) {
  k_grid_identity<<<dim3(nsec), dim3(256), 0, st>>>(secs, nsec, grids);
  return (int)hipGetLastError();
}

int launch_hist_reduce(const double* hist, const int64_t* hist_off, const int32_t* sec_tile_start,
                       const SecDev* secs, const int64_t* hsec_off, int nsec, int64_t total,
                       const int64_t* hsec_prefix, double* hsec, hipStream_t st) {
  if (total <= 0) return 0;
  k_hist_reduce<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(
      hist, hist_off, sec_tile_start, secs, hsec_off, nsec, total, hsec_prefix, hsec);
  return (int)hipGetLastError();
}

int launch_refit(const SecDev* secs, int nsec, const double* hsec, const int64_t* hsec_off, double* grids,
                 double alpha, hipStream_t st) {
  k_refit<<<dim3(nsec * MAXV), dim3(NBMAX), 0, st>>>(secs, nsec, hsec, hsec_off, grids, alpha);
  return (int)hipGetLastError();
}

int launch_sample_points(const SampleArgs& a, hipStream_t st) {
  if (a.npts <= 0) return 0;
  k_sample_points<<<dim3((unsigned)((a.npts + 255) / 256)), dim3(256), 0, st>>>(a);
  return (int)hipGetLastError();
}

int noalloc_scratch_address(void** out) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  *out = p;
  return 0;
}

}  // namespace sdi
