// Internal layout shared by the host compiler (api.cpp) and the HIP kernels.
//
// A compiled problem lives in device memory as:
//   SecDev[nsec]      one record per sector, read by the kernels with
//                     wave-uniform scalar loads (the "sector tape");
//   Term[]            polynomial terms, one contiguous list per
//                     (sector, factor, corner W), so the corner x_W = 0 of the
//                     pole subtraction is a choice of list, not a branch;
//   uint64 zp[][16]   lattice generating vector, pre-shifted by 53 - m;
//   uint64 shift[][]  53-bit Philox shifts per (sector, shift, variable);
//   double grid[]     Vegas grids, (n x (NB+1)) per sector.
// Inside a sector record the variables are reordered so that the singular
// variables (a_j = -1) come first; perm[] maps back to the caller's order so
// that point coordinates, shifts and grids stay attached to the caller's
// variable j.
#pragma once
#include <stdint.h>

namespace sdi {

constexpr int MAXV = 16;     // variables per sector
constexpr int MAXF = 4;      // regular factors per sector
constexpr int MAXS = 4;      // singular variables per sector
constexpr int MAXC = 16;     // corners 2^MAXS
constexpr int KMAX = 8;      // result orders and internal f orders
constexpr int NBMAX = 256;   // Vegas bins per dimension
constexpr int BLOCK = 256;   // threads per block of the tile kernels
constexpr uint64_t MASK53 = (1ull << 53) - 1;

// Polynomial term: coefficient and packed exponents, one nibble per variable:
// bit 0 multiplies by x, bit 1 by x^2, bit 2 by x^4.
struct alignas(16) Term {
  double coef;
  uint64_t exps;
};

enum SecFlags : int32_t {
  F_HAS_IM = 1,        // fold coefficients have imaginary parts
  F_INT_POW = 2,       // all gamma_m, delta_m integers: powers by products, one log per corner
  F_INT_MONO = 4,      // non-singular a_j small non-negative integers, b_j integers |b| <= 8
  F_USE_GRID = 8,      // Vegas map active
  F_BAKER = 16,        // tent transform of the lattice
  F_EXP7 = 32,         // some factor exponent above 3 (the x^4 bit of the term words is used)
};

struct alignas(16) SecDev {
  int32_t n, ns, nfac, kf;          // variables, singular variables, factors, f orders
  int32_t K, flags, nvc, cls;       // result orders, SecFlags, variable class, kernel class
  int32_t grid_off, shift_row, m, mw;  // grid offset (doubles), row of shift table, log2 N, warm-up log2 N
  int32_t nbins, sector, pad0, pad1;
  int32_t perm[MAXV];               // internal variable j = caller variable perm[j]
  int32_t a_int[MAXV];              // integer a_j (F_INT_MONO)
  int32_t b_int[MAXV];              // integer b_j (F_INT_MONO)
  uint32_t tab_off[MAXF][MAXC];     // term list offset per (factor, corner)
  uint32_t tab_cnt[MAXF][MAXC];
  // The same terms grouped by their singular support: group (m, sigma) holds
  // the terms of factor m whose exponents are nonzero exactly on the singular
  // variables of mask sigma.  A term of group sigma is alive at corner W iff
  // W & sigma == 0, so P_m(x^(W)) = sum over sigma with W & sigma == 0 of the
  // group sums at x: each term is evaluated once for all corners.
  uint32_t grp_off[MAXF][MAXC];
  uint32_t grp_cnt[MAXF][MAXC];
  uint32_t grp_mask[MAXF];          // bit sigma set iff group (m, sigma) is not empty
  int32_t gam_int[MAXF], del_int[MAXF];
  double gam[MAXF], del[MAXF];
  double a[MAXV], b[MAXV];
  double invb[MAXC];                // prod_{i in T} 1/b_{S_i} per subset mask T
  double bS[MAXS];
  double fold_re[KMAX][KMAX];       // F_k = mono * sum_kk fold[k][kk] f_kk
  double fold_im[KMAX][KMAX];
};

// Complex-mode tables of one sector, next to its SecDev record.
struct alignas(16) CplxDev {
  int32_t nd;                  // derivative polynomials: n first, then n(n+1)/2 second (k <= j)
  int32_t dir_off;             // offset of this sector's (offset, count) directory [nd][MAXC][2]
  int32_t mono_f[MAXV];        // exponents of the monomial factored out of F (internal order)
  int32_t fac_f;               // factor index of F, -1 if none
  int32_t pad;
  double lam;
  const double* coef_im;       // imaginary parts of the coefficients of the problem's term
                               // lists (same indexing as the Term table), null if this
                               // sector's coefficients are real
};

struct alignas(16) TileDesc {
  int32_t sector;
  int32_t shift;      // row in the shift table (final shifts 0..R-1, warm-up R+it)
  uint32_t i0;        // first lattice index
  uint32_t count;     // points in the tile
};

// Per-tile partial sums per internal order f_kk (the prefactor fold is linear and
// is applied after the reduction): hi/lo of sum w f (re), hi/lo (im).
constexpr int PART_STRIDE = 4;      // doubles per order

struct TileArgs {
  const SecDev* secs;
  const Term* terms;
  const uint64_t* zp;        // [nsec][MAXV] generating vector << (53 - m) of this pass
  const uint64_t* shifts;    // [rows][MAXV]
  const double* grids;
  const TileDesc* tiles;     // canonical order
  const int32_t* order;      // processing order (LPT), indices into tiles
  double* partial;           // [ntiles][KMAX][PART_STRIDE]
  int32_t* nonfinite;        // [ntiles][2]: non-finite points, points with Im F(z) > 0
  double* hist;              // warm-up histograms [ntiles][n*NB*K] or null
  const int64_t* hist_off;   // per tile offset into hist (doubles)
  int32_t* counter;          // work counter (zeroed by the launcher's fill kernel)
  int32_t ntiles;
  int32_t mode;              // 0 final pass, 1 warm-up (histograms), 2 explicit points
  const double* px;          // mode 2: caller-order points of tile t at px + x_off[t]
  const double* pw;          //         and their weights at pw + pt_off[t]
  const int64_t* x_off;
  const int64_t* pt_off;
  double small_x;            // modes 0 and 2: points whose smallest singular coordinate is below it
                             // are evaluated in double-double (0: never)
};

// A run of points of one sector (explicit-point passes and flow batches):
// lattice indices i0 .. i0+count-1 with shift row `row`; per-point outputs at
// point offset pt_off, caller-order coordinates at double offset x_off.
struct PointRun {
  int32_t sector;
  int32_t row;
  uint32_t i0;
  uint32_t count;
  int64_t pt_off;
  int64_t x_off;
};

struct EvalTilesArgs {       // explicit points of several sectors (training batches)
  const SecDev* secs;
  const Term* terms;
  const PointRun* runs;
  const int64_t* chunk_prefix;  // [nruns + 1], chunks of BLOCK points
  int32_t nruns;
  int32_t K;                 // result orders (output stride)
  int64_t nchunks;
  const double* x;
  double* out;               // [pt][K][2]
};

struct EvalArgs {            // explicit points (justEvaluate / parity)
  const SecDev* sec;
  const Term* terms;
  const double* x;           // [npts][n] caller variable order
  double* out;               // [npts][K][2]
  int64_t npts;
  double* cond;              // [npts][K] sums of |term| per result order, or null
  double small_x;            // double-double below this smallest singular coordinate (0: never)
};

struct SampleArgs {
  const SecDev* sec;
  const uint64_t* zp;        // [MAXV] of this sector
  const uint64_t* shift;     // [MAXV] row
  const double* grid;
  double* x;                 // [npts][n] caller order
  double* w;                 // [npts] or null
  uint64_t i0;
  int64_t npts;
};

}  // namespace sdi
