// Host-side declarations of libsdint: context, compiled problem, helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sdint.h"
#include "expr_types.h"
#include "flow_types.h"
#include "sdint_internal.h"

struct sdi_ctx;

// Return from the calling API function with SDI_EDEVICE if a HIP call (HIPCHK)
// or a kernel launcher (KCHK, returns a hipError_t value) fails.
#define HIPCHK(ctx, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return sdi::fail(ctx, SDI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define KCHK(ctx, call)                                                                          \
  do {                                                                                           \
    int e_ = (call);                                                                             \
    if (e_ != 0)                                                                                 \
      return sdi::fail(ctx, SDI_EDEVICE,                                                         \
                       std::string(#call) + ": " + hipGetErrorString((hipError_t)e_));          \
  } while (0)

// Hash of the kernel sources this library was built from (set by the build);
// saved autotuner entries of another build are not loaded.
#ifndef SDI_KERNEL_HASH
#define SDI_KERNEL_HASH "unversioned"
#endif

namespace sdi {

struct Params {
  int m = 16;            // lattice_log2
  int R = 16;            // shifts
  uint64_t seed = 1;
  int baker = 1;
  int warmup = 0;
  int mw = 14;           // warmup_log2
  int nbins = 128;
  int tile_log2 = 0;     // 0: autotuned (2^14 with tuning off)
  int ppt = 0;           // 0: autotune
  int tune = 1;          // 0 off, 1 cached, 2 search
  int graph = 1;         // capture the pass into a hipGraph and replay it
  int64_t budget = 0;    // total final-pass evaluations to distribute by variance (0: uniform m)
  int alloc_min = 12;    // bounds of the per-sector lattice log2 under allocation
  int alloc_max = 20;
  int pilot_log2 = 12;   // lattice log2 of the pilot pass that measures the variances
  int sampler = 0;       // 0: lattice (+ Vegas grid), 1: the learned flow
  double small_x = 0.0;  // double-double below this smallest singular coordinate (0: off)
  int slice_log2 = 0;    // > 0: a call processes the next 2^slice_log2 lattice points per shift (resumable)
  int integrator = 0;    // 0: lattice QMC, 1: adaptive deterministic cubature
  int64_t cub_maxeval = 1 << 24;  // cubature: evaluation budget over all sectors
  double cub_epsrel = 1e-6;       // cubature: relative tolerance per order
  double cub_epsabs = 0.0;        // cubature: absolute tolerance per order
  double cub_split_frac = 0.25;   // cubature: share of the live regions halved per round
  int cub_batch_min = 1024;       // cubature: regions halved per round at least (while there are as many)
  int suave_nnew = 1024;          // subregion-adaptive Monte Carlo: points per new region
  int separate_terms = 0;         // 1: problems are compiled term by term (SeparateTerms)
};

// One autotuner decision: final-pass tile size and launch variant
// (10 * points per thread + minimum waves per SIMD).
struct TuneChoice {
  int tile_log2, variant;
};
struct TuneEntry {
  std::string key;
  int tile_log2, variant;
};

const std::vector<uint32_t>& lattice_vector16(int m);
struct PassState;
void free_passes(std::vector<PassState*>& v);

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace carving: a list of (pointer slot, bytes).
struct Carve {
  std::vector<std::pair<void**, size_t>> items;
  void add(void** p, size_t bytes) { items.push_back({p, align256(std::max<size_t>(bytes, 8))}); }
  size_t total() const {
    size_t t = 0;
    for (auto& i : items) t += i.second;
    return t;
  }
  void assign(void* base) {
    char* b = (char*)base;
    for (auto& i : items) {
      *i.first = b;
      b += i.second;
    }
  }
};

// Learned sampler of a problem: one coupling flow per sector.
struct FlowState {
  uint64_t seed = 0;
  int64_t nparam = 0;        // fp32 parameters of all flows
  int64_t nbw = 0;           // bf16 weight-copy elements
  int64_t max_lsize = 0;     // largest layer (parameters)
  int32_t max_nparam = 0;   // largest flow (parameters)
  std::vector<int64_t> t;    // Adam steps taken, per sector
  std::vector<uint8_t> active;  // sectors whose flow samples the integration passes
  std::vector<FlowSecDesc> desc;
  FlowSecDesc* d_desc = nullptr;
  float* d_params = nullptr;
  uint16_t* d_bw = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_grad = nullptr;
  void* d_scratch = nullptr; // training and gradient buffers, grown on demand
  size_t scratch_bytes = 0;
  double train_ms_pending = 0.0;   // device time of sdi_flow_train since the last sdi_integrate
  ~FlowState();
};
int fail(sdi_ctx* ctx, int code, const std::string& msg);

// Regions of the adaptive cubature (dyadic boxes per sector, in creation
// order) and their rule results; device buffers of a round.
struct CubState {
  std::vector<int32_t> sector;
  std::vector<uint8_t> level;     // [r][MAXV] halvings per caller variable
  std::vector<uint32_t> index;    // [r][MAXV]
  std::vector<double> val, err;   // [r][K][2]
  std::vector<double> sig;        // [r][K] rounding scale
  std::vector<int32_t> axis;      // caller variable to halve
  std::vector<int32_t> count;     // [r][2] non-finite nodes, Im F > 0 nodes
  std::vector<uint8_t> alive;     // not yet halved
  std::vector<double> spread;     // integrator 4: vol (max g - min g) / 2 of the partition sample
  void* d_buf = nullptr;
  size_t d_bytes = 0;
  ~CubState();
};
int run_cubature(sdi_ctx* ctx, sdi_problem* pb, sdi_result* out);
int prefactor_series(int loops, const int32_t* idx, int nprops, int d0, int len, int* lead, double* out,
                     std::string& err);

}  // namespace sdi

struct sdi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  sdi::Params params;
  hipDeviceProp_t prop{};
  int ncu = 0;
  std::vector<sdi::TuneEntry> tune_cache;
  void* scratch = nullptr;   // this device's fixed scratch array (allocation-free entry point)
  std::string tune_report;   // launch variants and times of the last autotuner search
};

struct sdi_problem {
  sdi_ctx* ctx = nullptr;
  int nsec = 0, K = 0, order_min = 0, kfmax = 0, nvmax = 4, complex_mode = 0;
  int nsmax = 0;                      // most singular variables of any sector
  int nfmax = 0;                      // most regular factors of any sector
  std::vector<int> origin;            // input sector of each compiled sector (parts of a_j < -1 sectors)
  bool exp7 = false;                  // some factor exponent above 3 (real mode)
  // resumable lattice pass (slice_log2 > 0): per (sector, shift) the running
  // double-double sums [npairs][KMAX][4] (re hi, re lo, im hi, im lo) of the
  // points done, the non-finite and Im F > 0 counts [npairs][2], the points
  // done per shift and the settings the sums belong to
  std::vector<double> resume_sums;
  std::vector<int64_t> resume_counts;
  int64_t resume_done = 0;
  std::string resume_key;
  double lambda = 0.0;
  std::vector<sdi::SecDev> secs;      // host copy (updated per integrate)
  std::vector<sdi::Term> terms;
  std::vector<double> terms_im;     // imaginary parts of the term coefficients (same indexing)
  double* d_terms_im = nullptr;     // on the device when some sector has complex coefficients
  std::vector<char> cx_cplx_coef;   // per sector (complex mode): its coefficients are complex
  std::vector<double> cost;           // relative cost per point of each sector
  sdi::SecDev* d_secs = nullptr;
  sdi::Term* d_terms = nullptr;
  double* d_grids = nullptr;          // persistent Vegas grids
  size_t grid_doubles = 0;
  int grid_nbins = 0;
  bool grid_valid = false;
  void* d_ws = nullptr;               // library-owned workspace
  size_t ws_size = 0;
  // results of the last integrate
  int last_R = 0;
  bool have_results = false;
  int last_sampler = -1;              // parameters of the pass that produced the last results
  int last_m = -1;                    // uniform lattice log2, -1 under budget allocation
  int last_warmup = 0;
  uint64_t last_seed = 0;
  std::vector<double> sec_stats;      // [nsec][KMAX][4]
  std::vector<double> per_shift;      // [nsec*R][KMAX][2]
  std::vector<int64_t> sec_evals;
  std::vector<sdi::PassState*> passes;   // cached plans (most recent last)
  // complex mode
  std::vector<sdi::CplxDev> cx;
  std::vector<uint32_t> dir;
  sdi::CplxDev* d_cx = nullptr;
  uint32_t* d_dir = nullptr;
  // learned sampler (created by sdi_flow_init)
  sdi::FlowState* flow = nullptr;
  // adaptive cubature (integrator 1): regions of the last run
  sdi::CubState* cub = nullptr;
  // integrand given as text (sdi_problem_from_text): one sector, one order
  std::vector<sdi::ExprIns> expr;
  sdi::ExprIns* d_expr = nullptr;
  size_t expr_nins = 0;
  int expr_slots = 0, expr_out = 0;
  bool expr_cplx = false;          // complex tape (the text uses I)
  bool is_expr() const { return d_expr != nullptr; }
};
