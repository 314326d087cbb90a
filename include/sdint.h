/*
 * sdint.h - C ABI of the MI355X sector-integrand library (libsdint.so).
 *
 * The library evaluates eps-expanded, sector-decomposed Feynman-parameter
 * integrands at very many sampling points on one AMD Instinct MI355X (gfx950)
 * and reduces them to eps-expansion coefficients with error estimates, the
 * numerical-integration stage of the sector-decomposition method described in
 * FIESTA 4 (A.V. Smirnov, arXiv:1511.03614): section 1 and eq. (2) define the
 * integrals, section 4.3 (SDEvaluate) the output (coefficients of eps^k with
 * "pm" errors combined in the mean-square norm), section 4.4 the Vegas
 * integrator and the contour deformation (ComplexMode), section 4.6 the
 * worker's single-point evaluation and TestF check.
 *
 * Conventions shared by every entry point:
 *  - Return value: SDI_OK (0) or a negative SDI_E* code.  The message of the
 *    last failure on a context is available from sdi_last_error(ctx) until the
 *    next call on that context.  On error no output argument is written,
 *    except where an entry point says otherwise.
 *  - Host pointers are plain CPU memory; arguments documented as "device" are
 *    HIP device pointers (e.g. torch tensors on cuda:N) on the context's device.
 *  - A context is not thread-safe: use one context per host thread.
 *  - Device work is issued on the context's stream; entry points that return
 *    host results synchronise that stream before returning.
 */
#ifndef SDINT_H
#define SDINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDI_OK = 0,
  SDI_EINVAL = -1,      /* invalid argument or input outside the supported domain   */
  SDI_ENOMEM = -2,      /* host or device allocation failed, or workspace too small */
  SDI_EDEVICE = -3,     /* a HIP call failed                                        */
  SDI_ENOTSUP = -4,     /* valid input that the library does not support           */
  SDI_ENONFINITE = -5,  /* results written, but some integrand values were NaN/Inf  */
  SDI_ESTATE = -6       /* call order violated (e.g. flow sampler before training)  */
};

#define SDI_MAX_VARS 16     /* variables per sector                          */
#define SDI_MAX_FACTORS 4   /* regular factors P_m per sector                */
#define SDI_MAX_SINGULAR 4  /* variables with a_j = -1 per sector            */
#define SDI_MAX_ORDERS 8    /* requested orders, and internal log-power depth */

typedef struct sdi_ctx sdi_ctx;
typedef struct sdi_problem sdi_problem;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device_ordinal`.  `hip_stream` is a
 * hipStream_t to issue work on (the caller keeps ownership), or NULL for a
 * library-owned stream.  *out receives the context. */
int sdi_ctx_create(int device_ordinal, void* hip_stream, sdi_ctx** out);
void sdi_ctx_destroy(sdi_ctx* ctx);
/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char* sdi_last_error(const sdi_ctx* ctx);
/* Device description (name, CUs, LDS, clock) as text: the GPUData command of
 * section 4.6.  Writes at most len bytes including the terminating NUL. */
int sdi_device_info(sdi_ctx* ctx, char* buf, size_t len);

/* Integrator parameters, the SetCurrentIntegratorParameter command of
 * section 4.6.  Keys (values are decimal text unless noted):
 *   lattice_log2   m, lattice points per shift N = 2^m          (default 16, 4..30)
 *   shifts         R, random shifts per sector                  (default 16, 2..256)
 *   seed           64-bit seed of the Philox4x32-10 shifts     (default 1)
 *   baker          1: tent-transform the lattice, 0: off        (default 1)
 *   warmup         Vegas grid-adaptation iterations             (default 0)
 *   warmup_log2    lattice points per warm-up iteration         (default 14)
 *   nbins          Vegas bins per dimension, power of 2 <= 256  (default 128)
 *   tile_log2      points per final-pass work tile: 0 = autotuned among
 *                  2^10..2^14 (2^14 when tune is off), or 6..24 (default 0)
 *   ppt            points per thread: 0 = autotuned, 1, 2 or 4  (default 0)
 *   tune           off | cached | search: the autotuner times the final-pass
 *                  kernel on the problem's own tiles for each launch variant
 *                  and tile size; "cached" reuses a decision for the same
 *                  device, problem shape and requests (sdi_tune_save/load
 *                  keep decisions across processes), "search" always times
 *                                                               (default cached)
 *   graph          1: capture each pass into HIP graphs and replay them (default 1)
 *   budget         total final-pass evaluations distributed over the sectors by
 *                  their pilot-pass errors (Neyman allocation); 0 = every
 *                  sector gets 2^lattice_log2 per shift            (default 0)
 *   alloc_min_log2, alloc_max_log2   bounds of the per-sector lattice log2
 *                  under allocation                             (default 12, 20)
 *   pilot_log2     lattice log2 of the pilot pass               (default 12)
 *   sampler        0: shifted lattice (+ Vegas grid), 1: the learned flow of
 *                  sdi_flow_init (warmup must be 0)             (default 0)
 *   slice_log2     resumable lattice pass (the -continue option of section
 *                  4.5): > 0 makes each sdi_integrate call process the next
 *                  2^slice_log2 lattice points of every shift of every
 *                  sector, continuing the per-(sector, shift) sums of the
 *                  earlier calls (sdi_checkpoint_export/import move them
 *                  between processes); results report the points done so far,
 *                  and once the lattice is complete they equal one call over
 *                  the whole lattice bit for bit when tile_log2 <= slice_log2
 *                  and tile_log2 and ppt are fixed (nonzero).  A call with
 *                  other settings, or after the last slice, starts a new pass.
 *                  Needs budget 0, warmup 0, sampler 0 (else SDI_ENOTSUP).
 *                  0 = off                                      (default 0)
 *   small_x        endpoint precision, a number in [0, 1] (decimal or
 *                  exponent notation): points whose smallest singular
 *                  coordinate lies below it are evaluated in double-double
 *                  arithmetic (about 106 bits) and rounded to fp64 once, by
 *                  sdi_evaluate and by the final pass on lattice points and
 *                  on flow-sampled points, in real and in complex mode (real
 *                  problems with at most 2 singular variables per sector keep
 *                  the tuned launch variants; deeper ones run one instance, 1
 *                  point per thread, 2 waves per SIMD; complex problems run
 *                  one instance, 1 point per thread); the role of the SmallX
 *                  / MPThreshold switch to MPFR of sections 4.4 and 4.6.  The
 *                  warm-up, the adaptive cubature and text integrands stay in
 *                  fp64.  0 = off                             (default 0)
 *   integrator     the final-stage integrator (CurrentIntegrator of section
 *                  4.4): 0 = shifted lattice QMC with optional Vegas grids;
 *                  1 = globally adaptive deterministic cubature, the role of
 *                  cuhreCuba: the Genz-Malik degree-7 rule with its embedded
 *                  degree-5 rule on dyadic regions of every sector cube,
 *                  rounds that halve the regions of largest weighted error
 *                  (one launch applies the rule pair to all new regions),
 *                  each along its largest fourth difference; errors are the
 *                  summed rule differences (not standard deviations).  It
 *                  takes sector problems (real or complex mode), not text
 *                  integrands, and no budget, warmup, sampler or slice_log2
 *                  (SDI_ENOTSUP); the workspace argument is not used;
 *                  2 = Monte Carlo points, the sampling of vegasCuba (the
 *                  paper's default): the final pass takes pseudo-random points
 *                  (Philox4x32-10, key = seed, counter = (index, variable +
 *                  16 shift, sector, 0x4D433031), u = (top 52 bits + 1/2)
 *                  2^-52) through the Vegas grids of the warm-up when it ran,
 *                  the R shifts being R independent samples; everything else
 *                  as for 0 (budget, warm-up, small_x); not with the flow
 *                  sampler, text integrands or slice_log2 (SDI_ENOTSUP);
 *                  3 = subregion-adaptive Monte Carlo, the role of suaveCuba:
 *                  the regions, rounds, budget (cub_maxeval), tolerances and
 *                  batches of 1, each new region sampled with suave_nnew
 *                  Philox points (counter (point, variable, region number,
 *                  0x53554156)), its value and standard errors from the sample,
 *                  halved along the variable whose halves' spreads of the
 *                  weighted |F| sum to the least; errors are root sums of
 *                  squares; the same restrictions as 1;
 *                  4 = partition by spreads, then lattice rules, the role of
 *                  divonneCuba: the loop of 3 (budget cub_maxeval, batches,
 *                  suave_nnew Philox points per new region, counter tag
 *                  0x44495631) halving the regions of largest spread
 *                  vol (max g - min g) / 2 along the variable whose halves'
 *                  larger range of g is the least, until the budget is spent;
 *                  then every region takes the shifted lattice rule of
 *                  2^lattice_log2 points x shifts (at least 2; shift counter
 *                  (variable, shift, region, 0x44495632), the tent map under
 *                  baker), value and standard error from the shift means;
 *                  a region whose two estimates differ by more than 4
 *                  combined errors is halved once more and its halves take
 *                  the lattice rule.  n_evals counts both phases; the same
 *                  restrictions as 1.                           (default 0)
 *   suave_nnew     integrator 3: points per new region, 16..2^20 (default 1024)
 *   separate_terms SeparateTerms of section 4.4, read when a problem is
 *                  created (sdi_problem_create, sdi_problem_from_feynman):
 *                  1 compiles every sector with singular variables S as its
 *                  2^|S| integrable terms, each a sector of its own for every
 *                  integrator, sampler and the allocation.  Term T (a bit mask
 *                  over S, variables in increasing index): prod_{j in T}
 *                  1/(b_j eps) times the integral over the variables outside T
 *                  of the integrand at x_T = 0 (factor terms free of x_T),
 *                  subtracted in S \ T with no boundary terms; a term left
 *                  with no variable gets one constant variable.  The terms of
 *                  a sector follow each other in the order of T, and
 *                  sdi_problem_sector_origin names their input sector.  Real
 *                  mode only (SDI_ENOTSUP in complex mode: the deformation's
 *                  corner factors tie the terms together); a factor with no
 *                  term on a face x_T = 0 gives SDI_ENOTSUP.     (default 0)
 *   cub_maxeval    cubature: integrand evaluations over all sectors; below one
 *                  rule application per sector SDI_EINVAL    (default 2^24)
 *   cub_epsrel, cub_epsabs   cubature: tolerance per order
 *                  max(epsabs, epsrel |value|), numbers in [0, 1]
 *                                                     (default 1e-6, 0)
 *   cub_split_frac cubature: share of the live regions halved per round, in
 *                  (0, 1]                                    (default 0.25)
 *   cub_batch_min  cubature: regions halved per round at least, while there
 *                  are as many (1..2^24)                     (default 1024)
 * Aliases: points (evaluations per sector = shifts x
 * 2^lattice_log2, a power-of-two multiple of the current shifts), budget_total
 * (= budget), budget_min / budget_max (per-sector evaluations under
 * allocation = shifts x 2^alloc_min_log2 / 2^alloc_max_log2), iterations
 * (= warmup), and sampler = lattice | vegas | flow (vegas: the lattice with
 * grid adaptation, 5 warm-up iterations unless warmup is set).  lambda and
 * complex mode belong to the problem (sdi_problem_desc), the flow's shape and
 * training settings to sdi_flow_init / sdi_flow_train.
 * Unknown keys or malformed values return SDI_EINVAL. */
int sdi_set_param(sdi_ctx* ctx, const char* key, const char* value);
int sdi_get_param(sdi_ctx* ctx, const char* key, char* buf, size_t len);

/* Autotuner decisions.  Section 2.2 sizes each GPU batch from the device's
 * multiprocessor count and memory; here the launch variant (points per
 * thread, waves per SIMD) and the final-pass tile size are instead chosen by
 * timing the kernel, once per device, problem shape and request, and kept in
 * ctx.  sdi_tune_save writes every decision of ctx to the file `path` as JSON,
 * together with the hash of the sources the library was built from
 * (the device name is part of every entry's key); returns SDI_OK or
 * SDI_EINVAL if the file cannot be written.  sdi_tune_load reads such a file
 * into ctx (an entry with the key of an existing one replaces it) and returns
 * the number of entries loaded: 0 if the file comes from another kernel build,
 * SDI_EINVAL if it cannot be read or is not in the format sdi_tune_save
 * writes (ctx is then unchanged).  A loaded decision is used under tune =
 * cached. */
/* The candidates the last autotuner search timed on ctx, one line each
 * ("tile_log2=.. ppt=.. waves=.. lists=.. ms=.."; lists = 1: per-corner term
 * lists instead of terms grouped by singular support), empty when the last
 * decision came from the cache.  buf NULL: *needed receives the size. */
int sdi_tune_report(sdi_ctx* ctx, char* buf, size_t len, size_t* needed);
int sdi_tune_save(sdi_ctx* ctx, const char* path);
int sdi_tune_load(sdi_ctx* ctx, const char* path);

/* ------------------------------------------------------------------ problem */

/* One sector (section 1, eq. (2) after sector decomposition):
 *
 *   I_s = c_s int_[0,1]^n prod_j x_j^(a_j + b_j eps) prod_m P_m(x)^(gamma_m + delta_m eps) dx,
 *   P_m(x) = sum_t coef_t prod_j x_j^exps_tj.
 *
 * a_j must be exactly -1 (then b_j != 0) or greater than -1.  Term
 * coefficients may be complex in complex mode (complex masses, say): their
 * imaginary parts in term_coef_im; the contour deformation then follows the
 * gradient of the real part of x^m P_F.  All arrays are host memory owned by
 * the caller and copied by sdi_problem_create. */
typedef struct {
  int32_t nvars;              /* n, 1..SDI_MAX_VARS                                 */
  int32_t nfactors;           /* M, 0..SDI_MAX_FACTORS                              */
  int32_t deform_factor;      /* index of the F polynomial among the factors, or -1 */
  int32_t reserved;           /* must be 0                                          */
  double coeff_re, coeff_im;  /* c_s                                                */
  const double* mono_a;       /* [n] a_j (below -1: reduced, sdi_problem_create)   */
  const double* mono_b;       /* [n] b_j                                            */
  const int32_t* deform_mono; /* [n] exponents of a monomial m: the deformation follows
                                 the gradient of x^m P_F; NULL = 0 (P_F itself)     */
  const int32_t* fac_nterms;  /* [M] terms per factor                               */
  const double* fac_gamma;    /* [M] gamma_m                                        */
  const double* fac_delta;    /* [M] delta_m                                        */
  const double* term_coef;    /* [sum nterms] coefficients, factor-major            */
  const uint8_t* term_exps;   /* [sum nterms][n] exponents, row-major               */
  const double* term_coef_im; /* [sum nterms] imaginary parts of term_coef, or NULL
                                 (real); non-NULL only in complex mode (SDI_EINVAL) */
} sdi_sector_desc;

/* The problem: sectors, requested orders, prefactor series, complex mode.
 * Result_k = sum_i Pi_i sum_s I_s[eps^(k - pref_lead - i)] for
 * k = order_min .. order_max (at most SDI_MAX_ORDERS orders). */
typedef struct {
  int32_t nsectors;
  const sdi_sector_desc* sectors;
  int32_t order_min, order_max;
  int32_t pref_lead, pref_len;  /* Pi(eps) = sum_{i<pref_len} Pi_i eps^(pref_lead + i) */
  const double* pref_re;        /* [pref_len]                                          */
  const double* pref_im;        /* [pref_len] or NULL                                  */
  int32_t complex_mode;         /* 1: deform x -> x - i lambda x (1-x) dF/dx (section 4.4) */
  double lambda;
} sdi_problem_desc;

/* Validate and compile a problem into device tables (one host-to-device upload).
 * Sectors with monomial exponents a_j < -1 (b_j != 0; real mode, integer
 * factor exponents) are reduced first, on the host, by integration by parts
 * in x_j (the analytic continuation in eps: with alpha = a_j + 1 + b_j eps,
 * the boundary part G(x_j = 1)/alpha and the derivative parts
 * -(g_m + d_m eps)/alpha x_j^alpha dP_m/dx_j P_m^(g_m - 1 + d_m eps) ...),
 * until every a_j >= -1; each part keeps a coefficient series in eps that
 * multiplies the prefactor.  The compiled sectors are then those parts, in the
 * order of the input sectors (sdi_problem_nsectors counts them,
 * sdi_problem_sector_origin names the input sector of each).  Returns
 * SDI_EINVAL for inputs outside the domain above and SDI_ENOTSUP for valid
 * inputs beyond the library (more than SDI_MAX_SINGULAR singular variables;
 * factor exponents above 7 in real mode or above 3 in complex mode; exponents
 * of the deformation polynomial's monomial times P_F above 7; more than 8
 * variables in complex mode; a_j < -1 in complex mode, with non-integer factor
 * exponents, or needing more than SDI_MAX_FACTORS factors). */
int sdi_problem_create(sdi_ctx* ctx, const sdi_problem_desc* desc, sdi_problem** out);

/* A Feynman integral by its Symanzik polynomials: SDEvaluate[{U, F, l},
 * indices, order] of section 4.3.  Eq. (2): prod_j x_j^(a_j - 1)
 * U^(A - (l+1) d/2) / F^(A - l d/2) over the simplex, A = sum_j a_j,
 * d = d0 - 2 eps, times exp(l gamma_E eps) Gamma(A - l d/2) / prod_j
 * Gamma(a_j).  The library forms the primary sectors (x_k = 1) and decomposes
 * each until U and F have constant terms after their monomials are taken out
 * (iterated decomposition with the smallest vanishing set of variables, the
 * classic strategy S of STRATEGY, section 4.4); result orders run from the
 * leading pole (the prefactor's lead minus the most singular variables of any
 * sector) to `order`.  The polynomials are host arrays owned by the caller
 * (terms in any order; equal exponent rows are merged). */
typedef struct {
  int32_t nvars;              /* n Feynman parameters, 2..17 (sectors get n - 1)   */
  int32_t loops;              /* l, 1..8                                            */
  int32_t d0;                 /* d = d0 - 2 eps, 1..12                              */
  int32_t order;              /* highest result order (at most 8 orders in all)     */
  const int32_t* indices;     /* [n] propagator powers a_j, 1..8                    */
  int32_t u_nterms, f_nterms;
  const double* u_coef;       /* [u_nterms]                                         */
  const uint8_t* u_exps;      /* [u_nterms][n]                                      */
  const double* f_coef;       /* [f_nterms]                                         */
  const uint8_t* f_exps;      /* [f_nterms][n]                                      */
  int32_t complex_mode;       /* 1: contour deformation along the sector's F        */
  int32_t reserved;           /* must be 0                                          */
  double lambda;              /* deformation size (complex mode)                    */
  const double* f_coef_im;    /* [f_nterms] imaginary parts of F's coefficients
                                 (complex masses), or NULL; complex mode only        */
} sdi_feynman_desc;

/* Compile the sectors of a Feynman integral (see sdi_feynman_desc).  Returns
 * SDI_EINVAL for malformed input or an order outside the 8 orders from the
 * leading pole, SDI_ENOTSUP where a decomposed sector leaves the library's
 * limits or needs what sdi_problem_create does not do (the reduction of a
 * sector exponent a_j < -1 in complex mode). */
int sdi_problem_from_feynman(sdi_ctx* ctx, const sdi_feynman_desc* desc, sdi_problem** out);
/* The same decomposition on the host only (no context, no device): the
 * number of sectors, the lowest result order and the variables per sector. */
int sdi_feynman_sectors(const sdi_feynman_desc* desc, int32_t* nsectors, int32_t* order_min, int32_t* max_vars);

/* An integrand given as text in the integration workers' input format
 * (section 4.6, CIntegrate options; the text that follows the Integrate
 * command, which may be included): a line with the number of variables n
 * (1..SDI_MAX_VARS), a line with the number of intermediate functions m, m
 * lines defining f[1] .. f[m], a line with the integrand, every line ended by
 * ';', then a line '|'.  Expressions use + - * /, round brackets, decimal
 * numbers, x[1] .. x[n], earlier f[i], p[base,exponent] (real power), l[arg]
 * (natural logarithm), P (pi), G (Euler's gamma) and the built-in values
 * PolyGamma[1,1], PolyGamma[2,1..4], PolyGamma[3,1..2].  A text that names
 * the imaginary unit I is a complex integrand (the complex workers of section
 * 4.2): every value is complex, l[a] is the principal logarithm with arg = -pi
 * on the negative real axis, p[a,b] is a^b by products for a whole-number
 * constant |b| <= 64 and exp(b l[a]) otherwise.  The result is a
 * problem of one sector and one order (order 0): sdi_integrate returns the
 * integral over [0,1]^n with the lattice sampler and optional Vegas warm-up
 * (not the flow sampler); sdi_evaluate gives the integrand at points (out
 * [npts][1][2], imaginary part 0 for a real integrand); sdi_sample_points
 * works as for sectors.
 * `text` is a NUL-terminated host string owned by the caller.  Returns
 * SDI_EINVAL for malformed text (the message names the offset),
 * SDI_ENOTSUP for PolyGamma arguments that are not built in, integrands of
 * more than 2^24 operations or ones that need more than 96 live temporaries
 * (48 complex ones), SDI_EDEVICE if the upload fails. */
int sdi_problem_from_text(sdi_ctx* ctx, const char* text, sdi_problem** out);

/* Compiles text as sdi_problem_from_text does, on the host only (no context,
 * no device): *nvars, *ninstructions (tape length, a multiple of 8) and
 * *nslots (per-point slots, complex ones for a complex integrand) receive the
 * result when not NULL; on failure the
 * same status as sdi_problem_from_text and, if err is not NULL, the message
 * (at most errlen bytes with the NUL). */
int sdi_text_info(const char* text, int32_t* nvars, int64_t* ninstructions, int32_t* nslots, char* err,
                  size_t errlen);
void sdi_problem_destroy(sdi_problem* prob);
/* Number of result orders K / of sectors of a problem (SDI_EINVAL for NULL). */
int sdi_problem_norders(const sdi_problem* prob);
int sdi_problem_nsectors(const sdi_problem* prob);
/* The input sector a compiled sector s comes from (s itself unless sectors with
 * a_j < -1 were expanded or terms separated, separate_terms); SDI_EINVAL for
 * an index out of range. */
int sdi_problem_sector_origin(const sdi_problem* prob, int32_t s);
/* Number of variables n of sector s (the column count of its points in
 * sdi_evaluate, sdi_sample_points and the flow calls); SDI_EINVAL for a NULL
 * problem or s out of range. */
int sdi_problem_nvars(const sdi_problem* prob, int32_t s);

/* Laurent series of the Feynman prefactor of eq. (2) with (i pi^(d/2))^l and
 * exp(-l gamma_E eps) pulled out (section 4.3):
 *   Pi(eps) = exp(l gamma_E eps) Gamma(A - l d/2) / prod_i Gamma(a_i),  d = d0 - 2 eps,
 * A = sum of the `nprops` indices (each >= 1).  Writes *lead and out[0..len-1]. */
int sdi_prefactor_feynman(int32_t loops, const int32_t* indices, int32_t nprops, int32_t d0,
                          int32_t len, int32_t* lead, double* out);

/* Rank-1 lattice generating vector for N = 2^m points and `dims` dimensions
 * (component-by-component search), as used by the integrator.  out[dims]. */
int sdi_lattice_vector(int32_t m, int32_t dims, uint32_t* out);

/* ------------------------------------------------------------------ integrate */

typedef struct {
  int32_t order_min, norders;   /* filled by the library                              */
  double* val_re;               /* [norders] caller-allocated                         */
  double* val_im;
  double* err_re;               /* one standard deviation, re and im apart            */
  double* err_im;
  int64_t n_evals;              /* sector-point evaluations, all orders at once       */
  int64_t n_nonfinite;          /* non-finite weighted values (they enter the sums)   */
  int64_t n_imf_positive;       /* points with Im F(z) > 0 (TestF of section 4.6)     */
  double ms_sample_eval_reduce; /* device time of the final pass                      */
  double ms_refit;              /* device time of the warm-up iterations and refits   */
  double ms_total;
  double ms_eval_kernel;        /* device time of the final-pass tile kernel alone    */
  int32_t points_per_thread;    /* launch configuration of that kernel                */
  int32_t blocks;
  int32_t tile_log2;            /* final-pass tile size used (log2 of points)         */
  int32_t waves_per_simd;       /* minimum waves per SIMD the kernel was built for    */
  int32_t grouped;              /* 1: that kernel evaluated every polynomial term once
                                   per point (terms grouped by singular support),
                                   0: once per subtraction corner                      */
  double ms_pilot_kernel;       /* device time of the pilot pass's tile kernel (budget
                                   allocation; 0 without)                              */
  int32_t pilot_same_kernel;    /* 1: the pilot pass ran the same kernel instance as the
                                   final pass (budget allocation; 0 without)           */
  int64_t lattice_done;         /* lattice points per shift the estimates rest on: 2^m,
                                   or under slice_log2 the points done so far          */
  int64_t cub_regions;          /* cubature: regions the estimates sum over            */
  int32_t cub_rounds;           /* cubature: rule launches (rounds of halving + 1)     */
  int32_t cub_converged;        /* cubature: 1 if every order met its tolerance        */
  double ms_flow_train;         /* device time of sdi_flow_train on this problem since
                                   its previous sdi_integrate (the learned form's
                                   training share of this result; 0 without)          */
} sdi_result;

/* Bytes of device workspace sdi_integrate needs under the current parameters. */
size_t sdi_workspace_bytes(sdi_ctx* ctx, const sdi_problem* prob);

/* Integrate every sector: optional Vegas warm-up iterations (grid refit),
 * then the frozen-grid pass over R shifted lattices; per-sector means and
 * shift-to-shift errors; root-sum-square combination (section 4.3).
 * `dev_workspace` is device memory of at least sdi_workspace_bytes, or NULL
 * to let the library allocate (kept with the problem for reuse).  Synchronises
 * the stream and fills *out; returns SDI_ENONFINITE (with *out filled) if any
 * value was not finite. */
int sdi_integrate(sdi_ctx* ctx, sdi_problem* prob, void* dev_workspace, size_t ws_bytes,
                  sdi_result* out);

/* Regions of the last cubature run on prob (integrator 1), in creation order:
 * per region its sector, per caller variable the halvings level[r][16] and
 * index[r][16] (the region is [index 2^-level, (index + 1) 2^-level] along
 * that variable), value[r][norders][2] (its degree-7 integral),
 * error[r][norders][2] (|degree 7 - degree 5|, re and im apart) and the axis
 * it would be halved along.  Host arrays of cap regions (each may be NULL);
 * *nregions receives the total.  SDI_ESTATE without such a run. */
int sdi_cubature_regions(sdi_ctx* ctx, const sdi_problem* prob, int64_t cap, int64_t* nregions, int32_t* sector,
                         uint8_t* level, uint32_t* index, double* value, double* error, int32_t* axis);

/* Checkpoints of a resumable pass (slice_log2 > 0; the -continue option and the
 * saved partial results of sections 2.5 and 4.5): the per-(sector, shift)
 * double-double sums of the lattice points done so far, their non-finite and
 * Im F > 0 counts, the progress and the settings they were made under.
 * sdi_checkpoint_export writes them to host memory buf (len bytes); *needed
 * receives the size (buf NULL: only the size).  SDI_ESTATE without a pass in
 * progress, SDI_ENOMEM if len is too small.  sdi_checkpoint_import loads such
 * a buffer into prob (same sectors and shifts) of a context whose parameters
 * equal the checkpoint's settings (lattice_log2, shifts, seed, baker,
 * slice_log2, tile_log2, ppt, small_x; SDI_EINVAL otherwise, naming them); the
 * next sdi_integrate continues the pass.  The buffer is a plain host-endian
 * binary record, valid on machines of the same byte order. */
int sdi_checkpoint_export(sdi_ctx* ctx, const sdi_problem* prob, void* buf, size_t len, size_t* needed);
int sdi_checkpoint_import(sdi_ctx* ctx, sdi_problem* prob, const void* buf, size_t len);

/* Per-sector results of the last sdi_integrate: mean[K][2] (re, im),
 * err[K][2], per_shift[R][K][2] (may be NULL), *nevals. */
int sdi_sector_results(sdi_ctx* ctx, const sdi_problem* prob, int32_t s, double* mean,
                       double* err, double* per_shift, int64_t* nevals);

/* Values of every requested order of sector s (prefactor and c_s folded in,
 * no sampling weight) at caller points: the justEvaluate integrator of
 * section 4.4.  x: device [npts][n] doubles in the sector's variable order;
 * out: device [npts][K][2] doubles (re, im).  cond: device [npts][K] doubles
 * or NULL; receives per order the sum of the absolute values of every
 * subtraction and series term (times |c_s Pi_i| of the fold), the scale of
 * the rounding error of the value near the faces (0 for text integrands).
 * Stream-ordered; synchronises. */
int sdi_evaluate(sdi_ctx* ctx, const sdi_problem* prob, int32_t s, const void* x_dev,
                 int64_t npts, void* out_dev, void* cond_dev);

/* The exact points and weights the integrator uses for sector s, shift r,
 * lattice indices i0 .. i0+npts-1, under the current grid of that sector:
 * x: device [npts][n], w: device [npts] (NULL allowed).  Synchronises. */
int sdi_sample_points(sdi_ctx* ctx, const sdi_problem* prob, int32_t s, int32_t shift,
                      int64_t i0, int64_t npts, void* x_dev, void* w_dev);

/* sdi_sample_points for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same points and weights, bit for bit, with no hipMalloc, hipFree or other
 * allocating call.  The sector record, generating vector and shift row the
 * kernels read are staged in a fixed array of 8 KiB of device memory that the
 * library holds on every device it runs on until the process ends (its
 * address is taken once per device when the first context is created there);
 * a call needs about 3.2 KB of it whatever npts is, and returns SDI_ENOMEM if
 * the record ever outgrew the array.  The caller still provides x and w.  Every
 * call on one device shares that array and overwrites it (nothing in it has
 * to start at zero): calls that overlap on one device, from several threads or
 * contexts, race; calls on one context are ordered, since each synchronises
 * its stream before returning.  Arguments and errors as sdi_sample_points. */
int sdi_sample_points_noalloc(sdi_ctx* ctx, const sdi_problem* prob, int32_t s, int32_t shift,
                              int64_t i0, int64_t npts, void* x_dev, void* w_dev);

/* One refit of a Vegas grid on caller data, the step sdi_integrate's warm-up
 * takes after every iteration (Lepage's VEGAS refinement behind the Vegas
 * integrator of section 4.4; parity hook): for each dimension j < n,
 * hist_dev [n][nbins][k] holds per bin the sums of |w f_kk|^2 of the points in
 * it for the k internal orders; the importance d_b = sum over orders with a
 * nonzero total H of h_bk / H, smoothed over 3 bins (2 at the ends), is
 * compressed to ((r - 1) / ln r)^alpha with r = d_b / sum d, and the edges
 * grid_dev [n][nbins + 1] (device, in place) are moved so that each new bin
 * holds an equal share of the compressed importance, linearly inside the old
 * bins.  A dimension whose histogram is all zero keeps its edges.  n 1..16,
 * nbins a power of 2 in 2..256, k 1..8, alpha >= 0 (the integrator uses 1.5).
 * Stream-ordered; synchronises.  SDI_EINVAL for arguments out of range. */
int sdi_vegas_refit(sdi_ctx* ctx, int32_t n, int32_t nbins, int32_t k, const void* hist_dev, void* grid_dev,
                    double alpha);

/* Automatic deformation size (the ComplexMode tuning of section 4.4) for a
 * complex-mode problem: per sector, candidates lam_k = top * k / split
 * (k = split .. 1, top = lambda_max at first) are tested on the first
 * 2^points_log2 points of the sector's tent-transformed rank-1 lattice (Philox
 * shift row 65535 of the context's seed); the largest lam_k under which no
 * test point has Im F(z) > 0 at any corner x_W = 0 of the pole subtraction is
 * kept.  If none passes, top /= split and the search repeats (four rounds at
 * most, then lam = 0).  conservative != 0 halves the result
 * (ConservativeComplexShift).  The chosen values replace the problem's lambda
 * for every later call; lam_out (host, [nsectors], may be NULL) receives them.
 * split in 1..16, points_log2 in 4..20; SDI_ESTATE for a real-mode problem. */
int sdi_tune_deformation(sdi_ctx* ctx, sdi_problem* prob, double lambda_max, int32_t split,
                         int32_t points_log2, int32_t conservative, double* lam_out);

/* ---------------------------------------------------------- learned sampler
 * The importance-sampling map that replaces the Vegas grid of section 4.4 for
 * sampler = 1: per sector a flow of 4 piecewise-linear coupling layers (32
 * bins; conditioner MLP with 64 hidden units, bf16 weights and activations on
 * the matrix cores, fp32 accumulation; the map and its Jacobian in fp64, so
 * the weight 1/q is exact for the map applied).  Parameters are fp32, per
 * sector in the order layer 0..3 x (W1 [64][max(nA,1)], b1 [64], W2 [64][64],
 * b2 [64], W3 [nB*32][64], b3 [nB*32]); layer l transforms the variables
 * j = l mod 2 (variable 0 when n = 1) given the others.  All calls are
 * stream-ordered on ctx's stream and synchronise it; device buffers are the
 * caller's.  Errors: SDI_EINVAL (arguments), SDI_ESTATE (no flow yet),
 * SDI_ENOMEM, SDI_EDEVICE. */

/* (Re)create every sector's flow: W1, W2 uniform in +-1/sqrt(fan_in) from
 * Philox4x32-10 (key seed, counter (index in layer, layer, sector,
 * 0x464c4f57)), biases and W3 zero (the identity map); Adam state cleared. */
int sdi_flow_init(sdi_ctx* ctx, sdi_problem* prob, uint64_t seed);
/* fp32 parameters of sector s's flow (negative error code without a flow). */
int64_t sdi_flow_nparams(const sdi_problem* prob, int32_t s);
/* Copy sector s's parameters to / from host memory (n = sdi_flow_nparams). */
int sdi_flow_params(sdi_ctx* ctx, sdi_problem* prob, int32_t s, float* out, int64_t n);
int sdi_flow_set_params(sdi_ctx* ctx, sdi_problem* prob, int32_t s, const float* in, int64_t n);
/* Latent points u (device [npts][n]) to x (device [npts][n]) and log q(x)
 * (device [npts]) by the inverse layers 3..0. */
int sdi_flow_sample(sdi_ctx* ctx, sdi_problem* prob, int32_t s, const void* u_dev, int64_t npts,
                    void* x_dev, void* lq_dev);
/* Gradient of L = -sum_i c_i log q(x_i) with respect to sector s's
 * parameters (straight-through for every bf16 rounding) into the library's
 * gradient buffer and, if grad_out is not NULL, to host grad_out[nparams].
 * x: device [npts][n], c: device [npts]. */
int sdi_flow_grad(sdi_ctx* ctx, sdi_problem* prob, int32_t s, const void* x_dev, const void* c_dev,
                  int64_t npts, float* grad_out);
/* Overwrite sector s's slot of the gradient buffer from host memory. */
int sdi_flow_set_grad(sdi_ctx* ctx, sdi_problem* prob, int32_t s, const float* in, int64_t n);
/* One Adam step (beta 0.9, 0.999, eps 1e-8; moments and update in fp64,
 * stored in fp32) of every sector's parameters from the gradient buffer
 * (bias correction by each sector's own step count). */
int sdi_flow_adam(sdi_ctx* ctx, sdi_problem* prob, double lr);
/* Train the flows of the listed sectors (all sectors when `sectors` is NULL)
 * on the GPU for `iters` steps of 2^batch_log2 latent lattice points per
 * sector (shift rows 65536 + step of the Philox shifts), loss weights
 * c_i = sum_k w_k (|F_k(x_i)|^2 / q_i^2) / S_k with S_k the batch total of
 * order k and w_k = order_weights[k] (host [norders], finite, >= 0, not all
 * zero; NULL = all 1: which coefficients the maps should serve); one Adam
 * step per iteration (per-sector step counts).  The trained sectors become
 * active.  *ms_out: device time (may be NULL). */
int sdi_flow_train(sdi_ctx* ctx, sdi_problem* prob, const int32_t* sectors, int32_t nsel, int32_t iters,
                   int32_t batch_log2, double lr, const double* order_weights, float* ms_out);
/* The loss weights of sdi_flow_train on caller data (parity hook): with
 * S_k = sum_i |F_k(x_i)|^2 exp(-2 lq_i), c_i = sum over orders with S_k > 0
 * and finite of w_k |F_k(x_i)|^2 exp(-2 lq_i) / S_k, w_k = order_weights[k]
 * (host [K], finite, >= 0, not all zero; NULL = all 1).  f_dev device
 * [npts][K][2] (re, im), lq_dev device [npts] (log q), c_dev device [npts]
 * (out); npts 0..2^32-1, K 1..8.  Stream-ordered; synchronises. */
int sdi_flow_weights(sdi_ctx* ctx, int64_t npts, int32_t K, const void* f_dev, const void* lq_dev,
                     const double* order_weights, void* c_dev);
/* Sectors whose flow is active take their points from it in passes with
 * sampler = 1; the others stay on the lattice (with sdi_flow_set_params or
 * training a sector becomes active; sdi_flow_init clears every flag). */
int sdi_flow_set_active(sdi_ctx* ctx, sdi_problem* prob, int32_t s, int32_t active);
/* Validation with the lattice as the reference: one lattice pass and one flow pass
 * at 2^lattice_log2 points per shift (other parameters from ctx); with I_k and
 * V_k the lattice pass's estimate and total variance of order k and
 * S_k = max(|I_k|^2, V_k), an active sector keeps its flow only if
 * sum_k w_k var_flow(s,k)/S_k < sum_k w_k var_lattice(s,k)/S_k (its share of
 * the squared relative errors of the coefficients, w_k = order_weights[k],
 * host [norders] >= 0, NULL = all 1) and, in every order, the flow pass's
 * estimate of the sector lies within 5 combined standard errors of the
 * lattice pass's.  kept (host [nsectors], may be NULL) receives the active flags,
 * *ms_out (may be NULL) the device time of the passes run.  If the problem's
 * last results come from a lattice pass with the same lattice_log2, shifts and
 * seed (no warm-up, no allocation), they serve as the lattice pass and only
 * the flow pass runs.  The per-sector results left on the problem are those of
 * the flow pass. */
int sdi_flow_validate(sdi_ctx* ctx, sdi_problem* prob, int32_t lattice_log2, const double* order_weights,
                      int32_t* kept, float* ms_out);

#ifdef __cplusplus
}
#endif
#endif /* SDINT_H */
