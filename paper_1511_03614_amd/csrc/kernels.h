// Host-callable launchers of the HIP kernels.  Each returns a hipError_t value
// (0 on success) and only enqueues work on the given stream.
#pragma once
#include <hip/hip_runtime.h>

#include "cplx_args.h"
#include "expr_types.h"
#include "flow_types.h"
#include "sdint_internal.h"

namespace sdi {

int launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
int launch_shifts(const SecDev* secs, int nsec, int rows, int nfinal, uint64_t seed, uint32_t row0,
                  uint64_t* shifts, hipStream_t st);
// carry_in (may be null): running sums [npairs][KMAX][4] and counts [npairs][2]
// of earlier slices of the same pass, continued by this pass's tiles in
// order; carry_out (may be null) receives the continued sums and counts;
// npts: points per shift done with this pass (the divisor of the means).
int launch_reduce_pairs(const double* partial, const int32_t* pair_start, const int32_t* pair_sector,
                        const SecDev* secs, int npairs, double* out, const int32_t* nonfinite,
                        int64_t* pair_nonfinite, const double* carry_in, const int64_t* carry_in_counts,
                        double* carry_out, int64_t* carry_out_counts, int64_t npts, hipStream_t st);
int launch_sector_stats(const double* per_shift, int nsec, int R, double* out, const int64_t* pair_nonfinite,
                        int64_t* sec_nonfinite, hipStream_t st);
int launch_combine(const double* sec_stats, int nsec, const int64_t* sec_nonfinite, double* res, int64_t* counts,
                   hipStream_t st);
int launch_grid_identity(const SecDev* secs, int nsec, double* grids, hipStream_t st);
int launch_hist_reduce(const double* hist, const int64_t* hist_off, const int32_t* sec_tile_start,
                       const SecDev* secs, const int64_t* hsec_off, int nsec, int64_t total,
                       const int64_t* hsec_prefix, double* hsec, hipStream_t st);
int launch_refit(const SecDev* secs, int nsec, const double* hsec, const int64_t* hsec_off, double* grids,
                 double alpha, hipStream_t st);
int launch_sample_points(const SampleArgs& a, hipStream_t st);

// Bytes of the per-device fixed scratch array of the allocation-free entry
// point, and its device address on the current device (hipGetSymbolAddress;
// call with the device current, once per device).
constexpr size_t NOALLOC_SCRATCH_BYTES = 8192;
int noalloc_scratch_address(void** out);

// Integrands given as text: the persistent tile kernel (a.mode 0 final pass, 1
// warm-up with histograms; blocks of one wave; shmem = grid and histogram
// bytes, the expression slots are added) and the point evaluator.
size_t expr_slot_bytes(const ExprArgs& x);
int launch_tiles_expr(int grid, size_t shmem, const TileArgs& a, const ExprArgs& x, hipStream_t st);
int tiles_expr_occupancy(int mode, size_t shmem, const ExprArgs& x);
int launch_eval_points_expr(const EvalArgs& a, const ExprArgs& x, hipStream_t st);

// Tile kernel of variable class nvmax (4, 6, 8, 10 or 16), points per thread ppt and
// minimum waves per SIMD wpe, order capacity km (4 or 8), in the pass mode
// a.mode (0 final, 1 warm-up with at most 2 points per thread, 2 explicit
// points with 1; modes 1 and 2 run at 4 waves).  nsmax bounds the singular
// variables and nfmax the regular factors of every sector.  Families of
// instances (real_family): final passes of problems with at most two factors
// evaluate each term once by singular support, in instances sized by nsmax
// (RF_S2: nsmax <= 2, variants (1,4), (2,3), (2,4), (4,2), the last not for
// class 16, with endpoint-precision copies; RF_G3 / RF_G4: nsmax 3 / 4,
// variants (1,2), (1,4), (2,2), (2,3) / (1,2), (1,3), (2,1), (2,2)); other
// problems, warm-up and explicit points run the generic instances that
// evaluate each corner's term lists (RF_GENERIC, final-pass variants as RF_S2);
// endpoint precision outside RF_S2 runs the one instance of
// launch_tiles_real_dd (RF_DD; ppt and wpe ignored).  A final pass (mode 0,
// or mode 2 on explicit points) with a.small_x > 0 evaluates points below
// a.small_x again in double-double.
// grid = number of persistent blocks.
enum { RF_GENERIC = 0, RF_S2 = 1, RF_G3 = 2, RF_G4 = 3, RF_DD = 4 };
int real_family(int nsmax, int nfmax, int mode, bool dd);
int launch_tiles_real(int nvmax, int nsmax, int nfmax, int ppt, int wpe, int km, int grid, size_t shmem,
                      const TileArgs& a, hipStream_t st);
int launch_eval_points_real(int km, const EvalArgs& a, hipStream_t st);
// Occupancy (resident blocks per CU) of a tile kernel instance (dd: the
// endpoint-precision one of a final pass); 0 if not built.
int tiles_real_occupancy(int nvmax, int nsmax, int nfmax, int mode, int ppt, int wpe, int km, bool dd,
                         size_t shmem);
// Final pass (a.mode 0 on the lattice, 2 on explicit points) of the
// endpoint-precision mode: every variable class, one point per thread, points
// with a singular coordinate below a.small_x evaluated in double-double.  km 4 or 8.
int launch_tiles_real_dd(int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
// Problems with factor exponents above 3: one generic instance per variable
// class (1 point per thread, 4 waves per SIMD) for every mode, and the
// endpoint-precision final pass (modes 0 and 2 with a.small_x > 0; dd for the
// occupancy); km 4 or 8.
int launch_tiles_real_e7(int nvmax, int km, int grid, size_t shmem, const TileArgs& a, hipStream_t st);
int occupancy_tiles_real_e7(int nvmax, int mode, int km, bool dd, size_t shmem);
int occupancy_tiles_real_dd(int mode, int km, size_t shmem);

// Complex mode: nvmax 4 or 8; cx is the CplxDev array (tile kernel) or one sector's
// record (point evaluation); dir the derivative-list directory.  A final pass
// (mode 0 or 2) with a.small_x > 0 runs the endpoint-precision instance
// (launch_tiles_cplx_dd: one point per thread, ppt and wpe ignored, points
// below a.small_x again in double-double; dd for the occupancy).
int launch_tiles_cplx(int nvmax, int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a,
                      const void* cx, const uint32_t* dir, hipStream_t st);
int tiles_cplx_occupancy(int nvmax, int mode, int ppt, int wpe, int km, bool dd, size_t shmem);
int launch_tiles_cplx_dd(int km, int grid, size_t shmem, const TileArgs& a, const CplxArgs& X, hipStream_t st);
int occupancy_tiles_cplx_dd(int mode, int km, size_t shmem);
int launch_tiles_cplx_nv4(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, const CplxArgs& X,
                          hipStream_t st);
int launch_tiles_cplx_nv6(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, const CplxArgs& X,
                          hipStream_t st);
int launch_tiles_cplx_nv8(int ppt, int wpe, int km, int grid, size_t shmem, const TileArgs& a, const CplxArgs& X,
                          hipStream_t st);
int occupancy_tiles_cplx_nv4(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_cplx_nv6(int mode, int ppt, int wpe, int km, size_t shmem);
int occupancy_tiles_cplx_nv8(int mode, int ppt, int wpe, int km, size_t shmem);
int launch_eval_points_cplx(int km, const EvalArgs& a, const void* cx, const uint32_t* dir, hipStream_t st);
// Deformation-size test: fail[s] |= 1 << k when some test point of sector s has
// Im F(z) > 0 at some corner with lam = cand[s * ncand + k] (ncand <= 16).
int launch_lambda_test(int nvmax, const SecDev* secs, int nsec, const void* cx, const uint32_t* dir,
                       const Term* terms, const uint64_t* zp, const uint64_t* shifts, int64_t npts,
                       const double* cand, int ncand, int32_t* fail, hipStream_t st);

// Explicit points of several sectors (training batches).
int launch_eval_tiles_real(int km, int nvmax, const EvalTilesArgs& a, hipStream_t st);
int launch_eval_tiles_cplx(int km, const EvalTilesArgs& a, const void* cx, const uint32_t* dir, hipStream_t st);

// Learned sampler (coupling flow).
int launch_flow_init(const FlowSecDesc* fs, int nsec, float* params, uint64_t seed, hipStream_t st);
// bf16 copies of the flows of the sectors of runs (all nsec sectors when runs is null).
int launch_flow_copies(const FlowSecDesc* fs, const FlowTile* runs, int nruns, int nsec, const float* params,
                       uint16_t* bw, hipStream_t st);
// Adam over the parameters of the sectors of runs; bc: device [nruns][2] = 1 - beta1^t, 1 - beta2^t.
int launch_flow_adam(float* params, const float* grad, float* m, float* v, const FlowSecDesc* fs,
                     const FlowTile* runs, int nruns, int64_t max_nparam, double lr, const double* bc,
                     hipStream_t st);
int launch_flow_sample(const FlowSampleArgs& a, int nvmax, hipStream_t st);
int launch_flow_sample_tiles(const FlowTileArgs& a, int nvmax, hipStream_t st);

// Monte Carlo points of the final pass (integrator 2, mc_points.hip): for every
// run (a final tile: sector, shift row, lattice index range, offsets into x and
// w) its points from Philox4x32-10, through the sector's Vegas grid when it has
// one, as explicit points x (caller variable order) and weights w.
struct McArgs {
  const SecDev* secs;
  const PointRun* runs;
  const int64_t* chunk_prefix;  // [nruns + 1], chunks of 64 points
  int32_t nruns;
  int64_t nchunks;
  const double* grids;
  uint64_t seed;
  double* x;
  double* w;
};
int launch_mc_points(const McArgs& a, hipStream_t st);
int launch_flow_grad(const FlowGradArgs& a, int nvmax, int ncu, hipStream_t st);
int launch_flow_chunk_reduce(const FlowSecDesc* fs, const FlowTile* runs, const int64_t* chunk_prefix, int nruns,
                             const float* part, int64_t stride, int64_t max_nparam, float* grad, hipStream_t st);
int launch_flow_weights(const FlowTile* tiles, int ntiles, int K, const double* f, const double* lq, const double* ow,
                        double* c, hipStream_t st);
int launch_flow_shifts(const FlowSecDesc* fs, const FlowTile* runs, int nruns, int iters, int m, uint64_t seed,
                       uint32_t row0, uint64_t* out, hipStream_t st);

// Adaptive cubature: the degree-7/degree-5 rule pair on dyadic regions (one
// wave per region).  Region r covers [index 2^-level, (index + 1) 2^-level]
// along every caller variable of sector reg_sector[r].
struct CubArgs {
  const SecDev* secs;
  const Term* terms;
  const CplxDev* cx;          // complex mode: per-sector deformation records, else null
  const uint32_t* dir;
  const int32_t* reg_sector;  // [nreg]
  const uint8_t* reg_level;   // [nreg][MAXV], caller variable order
  const uint32_t* reg_index;  // [nreg][MAXV]
  const double* wtab;         // [MAXV + 1][10]: per n the degree-7 then degree-5 class weights
  double lam[4];              // node radii l2, l3, l4, l5
  double omega[KMAX];         // order weights of the split-axis measure
  int64_t nreg;
  int32_t K;
  int32_t pad;
  double* out_val;            // [nreg][K][2]  vol * S7
  double* out_err;            // [nreg][K][2]  vol |Re(S7 - S5)|, vol |Im(S7 - S5)|
  double* out_sig;            // [nreg][K]     rounding scale vol u sum_p (|w7| + |w5|) |F_k|_1
  int32_t* out_axis;          // [nreg] caller variable to halve
  int32_t* out_count;         // [nreg][2] nodes with a non-finite value, nodes with Im F(z) > 0
};
int launch_cubature_real(int nvmax, int km, const CubArgs& a, hipStream_t st);
int launch_cubature_cplx(int nvmax, int km, const CubArgs& a, hipStream_t st);

// Subregion-adaptive Monte Carlo (integrator 3, suave.hpp): npts pseudo-random
// points per region (regions uid0 .. uid0 + nreg - 1 in creation order), the
// region's value and standard errors per result order and its split axis.
struct SuaveArgs {
  const SecDev* secs;
  const Term* terms;
  const CplxDev* cx;
  const uint32_t* dir;
  const int32_t* reg_sector;  // [nreg]
  const uint8_t* reg_level;   // [nreg][MAXV], caller variable order
  const uint32_t* reg_index;  // [nreg][MAXV]
  double omega[KMAX];         // order weights of the split statistic
  int64_t nreg;
  int64_t uid0;
  uint64_t seed;
  int32_t K;
  int32_t npts;
  double* out_val;            // [nreg][K][2]  vol * mean
  double* out_err;            // [nreg][K][2]  vol * standard error of Re, Im
  int32_t* out_axis;          // [nreg]
  int32_t* out_count;         // [nreg][2] points with a non-finite value, points with Im F(z) > 0
  uint32_t tag;               // partition phase of integrator 4: the counter's tag
  double* out_spread;         // partition phase of integrator 4: [nreg] vol (max g - min g) / 2
};
int launch_suave_real(int nvmax, int km, const SuaveArgs& a, hipStream_t st);
int launch_suave_cplx(int nvmax, int km, const SuaveArgs& a, hipStream_t st);

// Integrator 4 (divonne.hpp): the partition phase (k_suave with DIV) and the
// final phase, a shifted rank-1 lattice rule on every region.
struct DivLatArgs {
  const SecDev* secs;
  const Term* terms;
  const CplxDev* cx;
  const uint32_t* dir;
  const int32_t* reg_sector;  // [nreg]
  const uint8_t* reg_level;   // [nreg][MAXV], caller variable order
  const uint32_t* reg_index;  // [nreg][MAXV]
  const uint32_t* zvec;       // [MAXV] generating vector of 2^m points
  int64_t nreg;
  int64_t uid0;
  uint64_t seed;
  int32_t K;
  int32_t m;                  // 2^m points per shift
  int32_t R;                  // shifts, >= 2
  int32_t baker;              // tent transform of the lattice coordinates
  double* out_val;            // [nreg][K][2]  vol * mean over shifts
  double* out_err;            // [nreg][K][2]  vol * standard error of the shift means
  int32_t* out_count;         // [nreg][2]
};
int launch_divonne_part_real(int nvmax, int km, const SuaveArgs& a, hipStream_t st);
int launch_divonne_part_cplx(int nvmax, int km, const SuaveArgs& a, hipStream_t st);
int launch_divonne_lattice_real(int nvmax, int km, const DivLatArgs& a, hipStream_t st);
int launch_divonne_lattice_cplx(int nvmax, int km, const DivLatArgs& a, hipStream_t st);

}  // namespace sdi
