// Host side of the learned sampler: parameter layout and initialisation,
// the parity hooks (sample, gradient, Adam), and the on-GPU training loop
// (sample a batch through the flow, evaluate the integrand there, form the
// loss weights, back-propagate, Adam, refresh the bf16 copies).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace sdi {

FlowState::~FlowState() {
  for (void* p : {(void*)d_desc, (void*)d_params, (void*)d_bw, (void*)d_m, (void*)d_v, (void*)d_grad, d_scratch})
    if (p) (void)hipFree(p);
}

namespace {

// Coupling masks: layer l transforms B_l = {j : j = l mod 2} given A_l = the
// others; a one-variable flow transforms variable 0 in every layer.
void flow_masks(int n, int l, std::vector<int>& A, std::vector<int>& B) {
  A.clear();
  B.clear();
  if (n == 1) {
    B.push_back(0);
    return;
  }
  for (int j = 0; j < n; ++j) (j % 2 == l % 2 ? B : A).push_back(j);
}

void flow_layout(const sdi_problem* pb, FlowState& F) {
  F.desc.assign(pb->nsec, FlowSecDesc{});
  int64_t base = 0, bw = 0;
  F.max_lsize = 0;
  for (int s = 0; s < pb->nsec; ++s) {
    FlowSecDesc& D = F.desc[s];
    D.n = pb->secs[s].n;
    D.base = base;
    int64_t off = 0;
    for (int l = 0; l < FL_L; ++l) {
      std::vector<int> A, B;
      flow_masks(D.n, l, A, B);
      FlowLayerDesc& L = D.layer[l];
      L.nA = (int)A.size();
      L.nB = (int)B.size();
      for (int k = 0; k < FL_MAXB; ++k) {
        L.A[k] = k < L.nA ? A[k] : 0;
        L.B[k] = k < L.nB ? B[k] : 0;
      }
      const int nA1 = std::max(L.nA, 1);
      const int nO = L.nB * FL_NB;
      L.w1 = off; off += (int64_t)FL_H * nA1;
      L.b1 = off; off += FL_H;
      L.w2 = off; off += (int64_t)FL_H * FL_H;
      L.b2 = off; off += FL_H;
      L.w3 = off; off += (int64_t)nO * FL_H;
      L.b3 = off; off += nO;
      F.max_lsize = std::max(F.max_lsize, off - L.w1);
      L.c1 = bw; bw += FL_H * FL_K1;
      L.c2 = bw; bw += FL_H * FL_H;
      L.c3 = bw; bw += (int64_t)nO * FL_H;
      L.t1 = bw; bw += FL_K1 * FL_H;
      L.t2 = bw; bw += FL_H * FL_H;
      L.t3 = bw; bw += (int64_t)FL_H * nO;
    }
    D.nparam = (int32_t)off;
    F.max_nparam = std::max(F.max_nparam, D.nparam);
    base += off;
  }
  F.nparam = base;
  F.nbw = bw;
}

int flow_ready(sdi_ctx* ctx, const sdi_problem* pb) {
  if (!pb->flow) return fail(ctx, SDI_ESTATE, "no learned sampler on this problem (call sdi_flow_init first)");
  return SDI_OK;
}

// Grows the flow's scratch to at least `bytes`.
int flow_scratch(sdi_ctx* ctx, FlowState& F, size_t bytes) {
  if (F.scratch_bytes >= bytes) return SDI_OK;
  if (F.d_scratch) (void)hipFree(F.d_scratch);
  F.d_scratch = nullptr;
  F.scratch_bytes = 0;
  if (hipMalloc(&F.d_scratch, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, SDI_ENOMEM, "flow scratch allocation failed (" + std::to_string(bytes) + " bytes)");
  }
  F.scratch_bytes = bytes;
  return SDI_OK;
}

}  // namespace

// Gradient of -sum_i c_i log q(x_i) for every run (one run per sector) into
// F.d_grad: per-chunk gradients, then their fixed-order sum per run.
int flow_gradient(sdi_ctx* ctx, sdi_problem* pb, const PointRun* d_runs, const int64_t* d_chunk_prefix, int nruns,
                  int64_t nchunks, const double* x, const double* c, double* hsave, bool inputs_saved, float* part,
                  hipStream_t st) {
  FlowState& F = *pb->flow;
  FlowGradArgs A{};
  A.fs = F.d_desc;
  A.params = F.d_params;
  A.bw = F.d_bw;
  A.runs = d_runs;
  A.chunk_prefix = d_chunk_prefix;
  A.nruns = nruns;
  A.nchunks = nchunks;
  A.x = x;
  A.c = c;
  A.hsave = hsave;
  A.inputs_saved = inputs_saved ? 1 : 0;
  A.part = part;
  A.part_stride = F.max_nparam;
  KCHK(ctx, launch_flow_grad(A, pb->nvmax, ctx->ncu, st));
  KCHK(ctx, launch_flow_chunk_reduce(F.d_desc, d_runs, d_chunk_prefix, nruns, part, F.max_nparam, F.max_nparam,
                                     F.d_grad, st));
  return SDI_OK;
}

size_t flow_grad_part_bytes(const FlowState& F, int64_t nchunks) {
  return (size_t)nchunks * F.max_nparam * sizeof(float);
}

}  // namespace sdi

using namespace sdi;

extern "C" {

int sdi_flow_init(sdi_ctx* ctx, sdi_problem* pb, uint64_t seed) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_init: null argument");
  if (pb->is_expr()) return fail(ctx, SDI_ENOTSUP, "flow: not available for integrands given as text");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  for (int s = 0; s < pb->nsec; ++s)
    if (pb->secs[s].n > 2 * FL_MAXB) return fail(ctx, SDI_ENOTSUP, "flow: more than 16 variables");
  free_passes(pb->passes);   // cached passes hold the old parameter pointers
  delete pb->flow;
  pb->flow = new FlowState();
  FlowState& F = *pb->flow;
  F.seed = seed;
  flow_layout(pb, F);
  F.t.assign(pb->nsec, 0);
  F.active.assign(pb->nsec, 0);
  const size_t np = (size_t)std::max<int64_t>(F.nparam, 1);
  HIPCHK(ctx, hipMalloc((void**)&F.d_desc, sizeof(FlowSecDesc) * std::max(pb->nsec, 1)));
  HIPCHK(ctx, hipMalloc((void**)&F.d_params, np * 4));
  HIPCHK(ctx, hipMalloc((void**)&F.d_m, np * 4));
  HIPCHK(ctx, hipMalloc((void**)&F.d_v, np * 4));
  HIPCHK(ctx, hipMalloc((void**)&F.d_grad, np * 4));
  HIPCHK(ctx, hipMalloc((void**)&F.d_bw, (size_t)std::max<int64_t>(F.nbw, 1) * 2));
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(F.d_desc, F.desc.data(), sizeof(FlowSecDesc) * pb->nsec, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemsetAsync(F.d_m, 0, np * 4, st));
  HIPCHK(ctx, hipMemsetAsync(F.d_v, 0, np * 4, st));
  HIPCHK(ctx, hipMemsetAsync(F.d_grad, 0, np * 4, st));
  KCHK(ctx, launch_flow_init(F.d_desc, pb->nsec, F.d_params, seed, st));
  KCHK(ctx, launch_flow_copies(F.d_desc, nullptr, 0, pb->nsec, F.d_params, F.d_bw, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return SDI_OK;
}

int64_t sdi_flow_nparams(const sdi_problem* pb, int32_t s) {
  if (!pb || !pb->flow || s < 0 || s >= pb->nsec) return SDI_EINVAL;
  return pb->flow->desc[s].nparam;
}

int sdi_flow_params(sdi_ctx* ctx, sdi_problem* pb, int32_t s, float* out, int64_t n) {
  if (!ctx || !pb || !out) return fail(ctx, SDI_EINVAL, "flow_params: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  const FlowSecDesc& D = pb->flow->desc[s];
  if (n != D.nparam) return fail(ctx, SDI_EINVAL, "flow_params: wrong parameter count");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipMemcpyAsync(out, pb->flow->d_params + D.base, n * 4, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return SDI_OK;
}

int sdi_flow_set_params(sdi_ctx* ctx, sdi_problem* pb, int32_t s, const float* in, int64_t n) {
  if (!ctx || !pb || !in) return fail(ctx, SDI_EINVAL, "flow_set_params: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  FlowState& F = *pb->flow;
  const FlowSecDesc& D = F.desc[s];
  if (n != D.nparam) return fail(ctx, SDI_EINVAL, "flow_set_params: wrong parameter count");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipMemcpyAsync(F.d_params + D.base, in, n * 4, hipMemcpyHostToDevice, ctx->stream));
  KCHK(ctx, launch_flow_copies(F.d_desc, nullptr, 0, pb->nsec, F.d_params, F.d_bw, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (!F.active[s]) free_passes(pb->passes);   // the split of the pass between lattice and flow changes
  F.active[s] = 1;
  return SDI_OK;
}

int sdi_flow_weights(sdi_ctx* ctx, int64_t npts, int32_t K, const void* f_dev, const void* lq_dev,
                     const double* order_weights, void* c_dev) {
  if (!ctx || (npts > 0 && (!f_dev || !lq_dev || !c_dev))) return fail(ctx, SDI_EINVAL, "flow_weights: null argument");
  if (npts < 0 || npts > (int64_t)0xFFFFFFFFu) return fail(ctx, SDI_EINVAL, "flow_weights: npts must be 0..2^32-1");
  if (K < 1 || K > KMAX) return fail(ctx, SDI_EINVAL, "flow_weights: K must be 1..8");
  std::vector<double> ow(K, 1.0);
  if (order_weights) {
    bool any = false;
    for (int k = 0; k < K; ++k) {
      if (!(std::isfinite(order_weights[k]) && order_weights[k] >= 0.0))
        return fail(ctx, SDI_EINVAL, "flow_weights: order weights must be finite and >= 0");
      ow[k] = order_weights[k];
      any = any || ow[k] > 0.0;
    }
    if (!any) return fail(ctx, SDI_EINVAL, "flow_weights: order weights are all zero");
  }
  if (npts == 0) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  FlowTile t{0, 0, 0, (uint32_t)npts, 0, 0};
  hipStream_t st = ctx->stream;
  FlowTile* d_t = nullptr;
  double* d_ow = nullptr;
  hipError_t he = hipMalloc((void**)&d_t, sizeof(FlowTile));
  if (he == hipSuccess) he = hipMalloc((void**)&d_ow, K * sizeof(double));
  if (he == hipSuccess) he = hipMemcpyAsync(d_t, &t, sizeof(FlowTile), hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = hipMemcpyAsync(d_ow, ow.data(), K * sizeof(double), hipMemcpyHostToDevice, st);
  int e = 0;
  if (he == hipSuccess)
    e = launch_flow_weights(d_t, 1, K, (const double*)f_dev, (const double*)lq_dev, d_ow, (double*)c_dev, st);
  const hipError_t hs = hipStreamSynchronize(st);
  if (d_t) (void)hipFree(d_t);
  if (d_ow) (void)hipFree(d_ow);
  if (he != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("flow_weights setup: ") + hipGetErrorString(he));
  if (e != 0) return fail(ctx, SDI_EDEVICE, std::string("flow_weights kernel: ") + hipGetErrorString((hipError_t)e));
  if (hs != hipSuccess) return fail(ctx, SDI_EDEVICE, std::string("flow_weights sync: ") + hipGetErrorString(hs));
  return SDI_OK;
}

int sdi_flow_set_active(sdi_ctx* ctx, sdi_problem* pb, int32_t s, int32_t active) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_set_active: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  pb->flow->active[s] = active ? 1 : 0;
  free_passes(pb->passes);   // the split of the pass between lattice and flow changed
  return SDI_OK;
}

int sdi_flow_sample(sdi_ctx* ctx, sdi_problem* pb, int32_t s, const void* u_dev, int64_t npts, void* x_dev,
                    void* lq_dev) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_sample: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  if (npts < 0) return fail(ctx, SDI_EINVAL, "negative point count");
  if (npts == 0) return SDI_OK;
  if (!u_dev || !x_dev || !lq_dev) return fail(ctx, SDI_EINVAL, "flow_sample: null buffer");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  FlowState& F = *pb->flow;
  FlowSampleArgs A{F.d_desc, F.d_params, F.d_bw, (const double*)u_dev, (double*)x_dev, (double*)lq_dev, s, npts};
  KCHK(ctx, launch_flow_sample(A, pb->nvmax, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return SDI_OK;
}

int sdi_flow_grad(sdi_ctx* ctx, sdi_problem* pb, int32_t s, const void* x_dev, const void* c_dev, int64_t npts,
                  float* grad_out) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_grad: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  if (npts <= 0 || npts > (int64_t)UINT32_MAX) return fail(ctx, SDI_EINVAL, "flow_grad: point count out of range");
  if (!x_dev || !c_dev) return fail(ctx, SDI_EINVAL, "flow_grad: null buffer");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  FlowState& F = *pb->flow;
  const int n = F.desc[s].n;
  const int64_t nchunks = (npts + FL_CHUNK - 1) / FL_CHUNK;
  Carve C;
  PointRun* d_run = nullptr;
  int64_t* d_prefix = nullptr;
  double* hsave = nullptr;
  float* part = nullptr;
  C.add((void**)&d_run, sizeof(PointRun));
  C.add((void**)&d_prefix, 2 * sizeof(int64_t));
  C.add((void**)&hsave, (size_t)npts * FL_L * n * 8);
  C.add((void**)&part, flow_grad_part_bytes(F, nchunks));
  rc = flow_scratch(ctx, F, C.total());
  if (rc) return rc;
  C.assign(F.d_scratch);
  hipStream_t st = ctx->stream;
  const PointRun run{s, 0, 0u, (uint32_t)npts, 0, 0};
  const int64_t prefix[2] = {0, nchunks};
  HIPCHK(ctx, hipMemcpyAsync(d_run, &run, sizeof run, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_prefix, prefix, sizeof prefix, hipMemcpyHostToDevice, st));
  rc = flow_gradient(ctx, pb, d_run, d_prefix, 1, nchunks, (const double*)x_dev, (const double*)c_dev, hsave, false,
                     part, st);
  if (rc) return rc;
  if (grad_out)
    HIPCHK(ctx, hipMemcpyAsync(grad_out, F.d_grad + F.desc[s].base, (size_t)F.desc[s].nparam * 4,
                               hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return SDI_OK;
}

int sdi_flow_set_grad(sdi_ctx* ctx, sdi_problem* pb, int32_t s, const float* in, int64_t n) {
  if (!ctx || !pb || !in) return fail(ctx, SDI_EINVAL, "flow_set_grad: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (s < 0 || s >= pb->nsec) return fail(ctx, SDI_EINVAL, "sector index out of range");
  FlowState& F = *pb->flow;
  if (n != F.desc[s].nparam) return fail(ctx, SDI_EINVAL, "flow_set_grad: wrong parameter count");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipMemcpyAsync(F.d_grad + F.desc[s].base, in, n * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return SDI_OK;
}

int sdi_flow_adam(sdi_ctx* ctx, sdi_problem* pb, double lr) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_adam: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(ctx, SDI_EINVAL, "flow_adam: learning rate must be positive");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  FlowState& F = *pb->flow;
  const int nsec = pb->nsec;
  std::vector<PointRun> runs(nsec);
  std::vector<double> bc(2 * (size_t)nsec);
  for (int s = 0; s < nsec; ++s) {
    runs[s] = PointRun{s, 0, 0u, 0u, 0, 0};
    F.t[s] += 1;
    bc[2 * s] = 1.0 - std::pow(0.9, (double)F.t[s]);
    bc[2 * s + 1] = 1.0 - std::pow(0.999, (double)F.t[s]);
  }
  Carve C;
  PointRun* d_runs = nullptr;
  double* d_bc = nullptr;
  C.add((void**)&d_runs, sizeof(PointRun) * nsec);
  C.add((void**)&d_bc, bc.size() * 8);
  rc = flow_scratch(ctx, F, C.total());
  if (rc) return rc;
  C.assign(F.d_scratch);
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(d_runs, runs.data(), sizeof(PointRun) * nsec, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_bc, bc.data(), bc.size() * 8, hipMemcpyHostToDevice, st));
  KCHK(ctx, launch_flow_adam(F.d_params, F.d_grad, F.d_m, F.d_v, F.d_desc, d_runs, nsec, F.max_nparam, lr, d_bc, st));
  KCHK(ctx, launch_flow_copies(F.d_desc, nullptr, 0, nsec, F.d_params, F.d_bw, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return SDI_OK;
}

// Training: `iters` steps for the selected sectors (all when sectors is NULL);
// each step draws 2^batch_log2 latent lattice points per sector (training
// shift rows 65536 + step), maps them through the flow, evaluates the
// integrand there, and takes one Adam step on the loss weights
// c_i = sum_k w_k (|f_k|^2 / q^2) / S_k (w_k: order_weights, 1 when NULL).
// The trained sectors become active.
int sdi_flow_train(sdi_ctx* ctx, sdi_problem* pb, const int32_t* sectors, int32_t nsel, int32_t iters,
                   int32_t batch_log2, double lr, const double* order_weights, float* ms_out) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_train: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (iters < 0 || iters > 100000) return fail(ctx, SDI_EINVAL, "flow_train: iterations out of range");
  if (batch_log2 < 6 || batch_log2 > 20) return fail(ctx, SDI_EINVAL, "flow_train: batch_log2 must be in 6..20");
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(ctx, SDI_EINVAL, "flow_train: learning rate must be positive");
  std::vector<double> ow(pb->K, 1.0);
  if (order_weights) {
    double tot = 0.0;
    for (int k = 0; k < pb->K; ++k) {
      if (!(order_weights[k] >= 0.0) || !std::isfinite(order_weights[k]))
        return fail(ctx, SDI_EINVAL, "flow_train: order weights must be finite and >= 0");
      ow[k] = order_weights[k];
      tot += ow[k];
    }
    if (!(tot > 0.0)) return fail(ctx, SDI_EINVAL, "flow_train: order weights are all zero");
  }
  std::vector<int32_t> sel;
  if (sectors) {
    if (nsel < 0 || nsel > pb->nsec) return fail(ctx, SDI_EINVAL, "flow_train: bad sector count");
    std::vector<uint8_t> seen(pb->nsec, 0);
    for (int i = 0; i < nsel; ++i) {
      if (sectors[i] < 0 || sectors[i] >= pb->nsec || seen[sectors[i]])
        return fail(ctx, SDI_EINVAL, "flow_train: sector list has an invalid or repeated index");
      seen[sectors[i]] = 1;
      sel.push_back(sectors[i]);
    }
  } else {
    for (int s = 0; s < pb->nsec; ++s) sel.push_back(s);
  }
  if (ms_out) *ms_out = 0.f;
  if (iters == 0 || sel.empty()) return SDI_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  (void)hipGetLastError();
  FlowState& F = *pb->flow;
  const int nr = (int)sel.size(), K = pb->K;
  const int64_t Bt = (int64_t)1 << batch_log2;
  std::vector<PointRun> runs(nr);
  std::vector<int64_t> pre64(nr + 1), pre256(nr + 1);
  int64_t xtot = 0;
  for (int r = 0; r < nr; ++r) {
    runs[r] = PointRun{sel[r], r, 0u, (uint32_t)Bt, (int64_t)r * Bt, xtot};
    xtot += Bt * F.desc[sel[r]].n;
    pre64[r] = (int64_t)r * (Bt / FL_CHUNK);
    pre256[r] = (int64_t)r * ((Bt + BLOCK - 1) / BLOCK);
  }
  pre64[nr] = (int64_t)nr * (Bt / FL_CHUNK);
  pre256[nr] = (int64_t)nr * ((Bt + BLOCK - 1) / BLOCK);
  const int64_t npts = Bt * nr;
  std::vector<uint64_t> zp((size_t)pb->nsec * MAXV, 0);
  const std::vector<uint32_t>& z = lattice_vector16(batch_log2);
  for (int s = 0; s < pb->nsec; ++s)
    for (int j = 0; j < MAXV; ++j) zp[(size_t)s * MAXV + j] = (uint64_t)z[j] << (53 - batch_log2);
  std::vector<double> bc((size_t)iters * nr * 2);
  for (int it = 0; it < iters; ++it)
    for (int r = 0; r < nr; ++r) {
      const double t = (double)(F.t[sel[r]] + it + 1);
      bc[((size_t)it * nr + r) * 2] = 1.0 - std::pow(0.9, t);
      bc[((size_t)it * nr + r) * 2 + 1] = 1.0 - std::pow(0.999, t);
    }
  Carve C;
  PointRun* d_runs = nullptr;
  int64_t *d_pre64 = nullptr, *d_pre256 = nullptr;
  uint64_t *d_zp = nullptr, *d_shifts = nullptr;
  double *x = nullptr, *w = nullptr, *lq = nullptr, *f = nullptr, *c = nullptr, *hsave = nullptr;
  double *d_bc = nullptr, *d_ow = nullptr;
  float* part = nullptr;
  C.add((void**)&d_runs, sizeof(PointRun) * nr);
  C.add((void**)&d_ow, (size_t)K * 8);
  C.add((void**)&d_pre64, 8 * (nr + 1));
  C.add((void**)&d_pre256, 8 * (nr + 1));
  C.add((void**)&d_zp, zp.size() * 8);
  C.add((void**)&d_shifts, (size_t)iters * nr * MAXV * 8);
  C.add((void**)&d_bc, bc.size() * 8);
  C.add((void**)&x, (size_t)xtot * 8);
  C.add((void**)&w, (size_t)npts * 8);
  C.add((void**)&lq, (size_t)npts * 8);
  C.add((void**)&f, (size_t)npts * K * 2 * 8);
  C.add((void**)&c, (size_t)npts * 8);
  C.add((void**)&hsave, (size_t)xtot * FL_L * 8);
  C.add((void**)&part, flow_grad_part_bytes(F, pre64[nr]));
  rc = flow_scratch(ctx, F, C.total());
  if (rc) return rc;
  C.assign(F.d_scratch);
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(d_runs, runs.data(), sizeof(PointRun) * nr, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_pre64, pre64.data(), 8 * (nr + 1), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_pre256, pre256.data(), 8 * (nr + 1), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_zp, zp.data(), zp.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_bc, bc.data(), bc.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(d_ow, ow.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  const int km = pb->kfmax <= 4 ? 4 : 8;
  // every step of every iteration, enqueued on st
  auto enqueue = [&]() -> int {
    KCHK(ctx, launch_flow_shifts(F.d_desc, d_runs, nr, iters, batch_log2, ctx->params.seed, 65536u, d_shifts, st));
    for (int it = 0; it < iters; ++it) {
      FlowTileArgs S{};
      S.fs = F.d_desc;
      S.params = F.d_params;
      S.bw = F.d_bw;
      S.zp = d_zp;
      S.shifts = d_shifts + (size_t)it * nr * MAXV;
      S.tiles = d_runs;
      S.chunk_prefix = d_pre64;
      S.ntiles = nr;
      S.baker = ctx->params.baker;
      S.nchunks = pre64[nr];
      S.x = x;
      S.w = w;
      S.lq = lq;
      S.hsave = hsave;
      KCHK(ctx, launch_flow_sample_tiles(S, pb->nvmax, st));
      EvalTilesArgs E{};
      E.secs = pb->d_secs;
      E.terms = pb->d_terms;
      E.runs = d_runs;
      E.chunk_prefix = d_pre256;
      E.nruns = nr;
      E.K = K;
      E.nchunks = pre256[nr];
      E.x = x;
      E.out = f;
      if (pb->complex_mode)
        KCHK(ctx, launch_eval_tiles_cplx(km, E, pb->d_cx, pb->d_dir, st));
      else
        KCHK(ctx, launch_eval_tiles_real(km, pb->nvmax, E, st));
      KCHK(ctx, launch_flow_weights(d_runs, nr, K, f, lq, d_ow, c, st));
      const int r2 = flow_gradient(ctx, pb, d_runs, d_pre64, nr, pre64[nr], x, c, hsave, true, part, st);
      if (r2) return r2;
      KCHK(ctx, launch_flow_adam(F.d_params, F.d_grad, F.d_m, F.d_v, F.d_desc, d_runs, nr, F.max_nparam, lr,
                                 d_bc + (size_t)it * nr * 2, st));
      KCHK(ctx, launch_flow_copies(F.d_desc, d_runs, nr, pb->nsec, F.d_params, F.d_bw, st));
    }
    return SDI_OK;
  };
  // one graph for the whole loop (launch overheads dominate small batches);
  // eager launches if capture is off or fails
  struct GraphGuard {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    ~GraphGuard() {
      if (ge) (void)hipGraphExecDestroy(ge);
      if (g) (void)hipGraphDestroy(g);
    }
  } gg;
  if (ctx->params.graph) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const int rr = enqueue();
      const hipError_t ec = hipStreamEndCapture(st, &gg.g);
      if (!(rr == SDI_OK && ec == hipSuccess && gg.g &&
            hipGraphInstantiate(&gg.ge, gg.g, nullptr, nullptr, 0) == hipSuccess))
        gg.ge = nullptr;
    }
    (void)hipGetLastError();
    ctx->err.clear();
  }
  if (gg.ge) {
    HIPCHK(ctx, hipEventRecord(e0, st));
    HIPCHK(ctx, hipGraphLaunch(gg.ge, st));
    HIPCHK(ctx, hipEventRecord(e1, st));
    HIPCHK(ctx, hipEventSynchronize(e1));
  } else {
    HIPCHK(ctx, hipEventRecord(e0, st));
    rc = enqueue();
    if (rc) return rc;
    HIPCHK(ctx, hipEventRecord(e1, st));
    HIPCHK(ctx, hipEventSynchronize(e1));
  }
  float ms = 0.f;
  HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
  if (ms_out) *ms_out = ms;
  F.train_ms_pending += ms;
  for (int s : sel) {
    F.t[s] += iters;
    F.active[s] = 1;
  }
  free_passes(pb->passes);   // the split of the pass between lattice and flow may have changed
  return SDI_OK;
}

// Keeps a sector's flow only where it lowers that sector's share of the
// error: one lattice pass and one flow pass at 2^lattice_log2 points per shift
// (the context's other parameters).  With I_k and V_k the lattice pass's
// estimate and total variance of order k and S_k = max(|I_k|^2, V_k), the flow
// of sector s stays active when sum_k var_flow(s,k) / S_k < sum_k
// var_lattice(s,k) / S_k: the sector's contribution to the squared relative
// errors of the coefficients, summed over the orders, so that the orders with
// the largest relative error decide (each term times the caller's weight of
// that order, 1 by default); and when, in every order, the two estimates of
// the sector agree within 5 combined standard errors.  kept (host,
// [nsectors], may be NULL) receives the flags.
int sdi_flow_validate(sdi_ctx* ctx, sdi_problem* pb, int32_t lattice_log2, const double* order_weights,
                      int32_t* kept, float* ms_out) {
  if (!ctx || !pb) return fail(ctx, SDI_EINVAL, "flow_validate: null argument");
  int rc = flow_ready(ctx, pb);
  if (rc) return rc;
  if (lattice_log2 < 4 || lattice_log2 > 24) return fail(ctx, SDI_EINVAL, "flow_validate: lattice_log2 in 4..24");
  std::vector<double> ow(pb->K, 1.0);
  if (order_weights)
    for (int k = 0; k < pb->K; ++k) {
      if (!(order_weights[k] >= 0.0) || !std::isfinite(order_weights[k]))
        return fail(ctx, SDI_EINVAL, "flow_validate: order weights must be finite and >= 0");
      ow[k] = order_weights[k];
    }
  FlowState& F = *pb->flow;
  const Params saved = ctx->params;
  // per sector and order: variance of each pass; mean (re, im) of the lattice and of the flow pass
  std::vector<double> v[2], mean[2], fmean[2];
  const int K = pb->K;
  std::vector<double> re(K), im(K), er(K), ei(K);
  double ms = 0.0;
  // a lattice pass with these parameters that already ran is not repeated
  const bool reuse = pb->have_results && pb->last_sampler == 0 && pb->last_m == lattice_log2 &&
                     pb->last_R == saved.R && pb->last_seed == saved.seed && pb->last_warmup == 0;
  for (int pass = reuse ? 1 : 0; pass < 2; ++pass) {
    if (pass == 1 && reuse) {
      v[0].assign((size_t)pb->nsec * K, 0.0);
      mean[0].assign((size_t)pb->nsec * K, 0.0);
      mean[1].assign((size_t)pb->nsec * K, 0.0);
      for (int s = 0; s < pb->nsec; ++s)
        for (int k = 0; k < K; ++k) {
          const double* q = pb->sec_stats.data() + ((size_t)s * KMAX + k) * 4;
          v[0][(size_t)s * K + k] = q[2] * q[2] + q[3] * q[3];
          mean[0][(size_t)s * K + k] = q[0];
          mean[1][(size_t)s * K + k] = q[1];
        }
    }
    ctx->params.m = lattice_log2;
    ctx->params.sampler = pass;
    ctx->params.warmup = 0;
    ctx->params.budget = 0;
    sdi_result res{};
    res.val_re = re.data();
    res.val_im = im.data();
    res.err_re = er.data();
    res.err_im = ei.data();
    rc = sdi_integrate(ctx, pb, nullptr, 0, &res);
    if (rc != SDI_OK && rc != SDI_ENONFINITE) {
      ctx->params = saved;
      return rc;
    }
    ms += res.ms_total;
    v[pass].assign((size_t)pb->nsec * K, 0.0);
    std::vector<double>* mm = pass == 0 ? mean : fmean;
    mm[0].assign((size_t)pb->nsec * K, 0.0);
    mm[1].assign((size_t)pb->nsec * K, 0.0);
    for (int s = 0; s < pb->nsec; ++s)
      for (int k = 0; k < K; ++k) {
        const double* q = pb->sec_stats.data() + ((size_t)s * KMAX + k) * 4;
        v[pass][(size_t)s * K + k] = q[2] * q[2] + q[3] * q[3];
        mm[0][(size_t)s * K + k] = q[0];
        mm[1][(size_t)s * K + k] = q[1];
      }
  }
  ctx->params = saved;
  // scale of order k: the squared magnitude of its lattice estimate, or the
  // lattice pass's total variance of that order where that is larger
  std::vector<double> V(K, 0.0);
  for (int k = 0; k < K; ++k) {
    double tr = 0.0, ti = 0.0, tv = 0.0;
    for (int s = 0; s < pb->nsec; ++s) {
      tr += mean[0][(size_t)s * K + k];
      ti += mean[1][(size_t)s * K + k];
      tv += v[0][(size_t)s * K + k];
    }
    V[k] = std::max(tr * tr + ti * ti, tv);
  }
  bool changed = false;
  for (int s = 0; s < pb->nsec; ++s) {
    if (F.active[s]) {
      double sf = 0.0, sl = 0.0;
      for (int k = 0; k < K; ++k)
        if (V[k] > 0.0) {
          sf += ow[k] * v[1][(size_t)s * K + k] / V[k];
          sl += ow[k] * v[0][(size_t)s * K + k] / V[k];
        }
      // the two passes estimate the same integral: a flow whose estimate sits
      // more than 5 combined standard errors from the lattice's in some order
      // is rejected whatever its variance (a map that rarely visits part of
      // the cube can look precise and still be off)
      bool consistent = true;
      for (int k = 0; k < K; ++k) {
        const size_t i = (size_t)s * K + k;
        const double dr = fmean[0][i] - mean[0][i], di = fmean[1][i] - mean[1][i];
        if (!(dr * dr + di * di <= 25.0 * (v[0][i] + v[1][i]))) consistent = false;
      }
      if (!(sf < sl) || !consistent) {
        F.active[s] = 0;
        changed = true;
      }
    }
    if (kept) kept[s] = F.active[s];
  }
  if (changed) free_passes(pb->passes);
  if (ms_out) *ms_out = (float)ms;
  return SDI_OK;
}

}  // extern "C"
