// te_runtime.cpp -- host side of the C ABI declared in include/te.h.
//
// Builds the device layout of an instance (path -> link CSR, link -> path CSC, demand -> path
// ranges, normalised capacities and demands), owns the device state, drives the iterations of
// the graph engine as captured HIP graphs of fixed-length iteration chunks, and runs the
// workgroup engine for small instances and batches.
#include <hip/hip_runtime.h>
#include <map>
#include <utility>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "te.h"
#include "te_internal.h"

namespace te {
hipError_t launch_init(const Prob &, const State &, const Params *, const float *, double, hipStream_t);
hipError_t launch_warm(const Prob &, const State &, const Params *, double, hipStream_t);
hipError_t launch_iteration(const Prob &, const State &, const Params *, int, hipStream_t);
hipError_t launch_demand_timed(const Prob &, const State &, const Params *, int, hipStream_t, hipEvent_t, hipEvent_t);
hipError_t launch_link_timed(const Prob &, const State &, const Params *, int, hipStream_t, hipEvent_t, hipEvent_t);
hipError_t launch_finish(const State &, const Params *, int, hipStream_t);
hipError_t launch_project(const Prob &, const State &, const ProjBuf &, float *, float *, double, int, hipStream_t);
hipError_t launch_project_rates(const Prob &, const ProjBuf &, const float *, double, float *, float *, double,
                                hipStream_t);
hipError_t launch_block_solve(const BatchDesc *, int, const Pools &, const Params *, int, float *, float *,
                              BatchOut *, size_t, int, int, hipStream_t);
size_t block_lds_bytes(int E, int P, int D, int nnz);
hipError_t launch_adj_seed(const Prob &, const AdjState &, const float *, hipStream_t);
hipError_t launch_adj_iteration(const Prob &, int, const FwdState &, const FwdState &, const AdjState &, double,
                                double, double, hipStream_t);
hipError_t launch_adj_x0(const Prob &, const AdjState &, hipStream_t);
hipError_t prepare_scatter_kernels();
hipError_t launch_get_state(const Prob &, const State &, double, double *, double *, hipStream_t);
hipError_t static_scratch(void **, size_t *);
}  // namespace te

using namespace te;

namespace {

thread_local std::string g_err;

te_status fail(te_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(TE_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Makes a handle's device current for the duration of an entry point and gives the caller's
// current device back when the entry point returns.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  DeviceScope(const DeviceScope &) = delete;
  DeviceScope &operator=(const DeviceScope &) = delete;
};

constexpr int kChunk = 16;                 // iterations per captured graph (even)
constexpr size_t kMaxBlockLds = 160 * 1024 - 4096;

template <class T>
hipError_t dalloc(T **p, size_t n) {
  return hipMalloc((void **)p, sizeof(T) * (n ? n : 1));
}

}  // namespace

struct te_ctx {
  int device = 0;
  int32_t E = 0, P = 0, D = 0, nnz = 0, maxp = 0, G = 1, logG = 0, H = 0, H2 = 0, ppl = 1, logGp = 0;
  int32_t lsum = kLinkSumsCsc;  // link sums of the graph engine in use (Prob::lsum)
  int32_t nB_csc = 0;           // workgroups of the CSC link kernel (also the adjoint's link kernel)
  int32_t ncu = 256;            // compute units of the device
  double scale = 1.0;
  // host layout (kept for batches and updates)
  std::vector<int32_t> pptr, plinks, dptr, lptr, lpaths;
  std::vector<int32_t> lpf, nzlink, nzptr, blk;  // link-kernel work split
  std::vector<double> cap, dem;  // caller units
  std::vector<double> Dn;
  std::vector<double> Cn;
  // device
  Prob prob{};
  State st{};
  FwdState work{};  // the iteration state block; st.x, st.uneg, st.udem, st.S and st.gq point into it
  ProjBuf pb{};
  Params *d_params = nullptr;
  Params *h_params = nullptr;  // pinned staging
  hipEvent_t params_ev = nullptr;
  double *d_sched = nullptr;
  int32_t sched_cap = 0;
  int32_t *d_i32 = nullptr;
  int4 *d_wtab = nullptr;
  uint16_t *d_lent = nullptr;  // link lists of the privatised sums (Prob::lent, lgrp, lchk)
  int64_t n_lent = 0;          // their entries
  int2 *d_lgrp = nullptr;
  int4 *d_lchk = nullptr;
  uint16_t *d_hops = nullptr;
  uint16_t *d_hops2 = nullptr;
  int32_t *d_dovf = nullptr;
  double *d_Dn = nullptr;
  double *d_Cn = nullptr;
  // workgroup engine (single instance)
  BatchDesc *d_desc = nullptr;
  BatchOut *d_bout = nullptr;
  // graph of kChunk iterations, and the same with the (beta, alpha) log of a recorded solve
  hipGraphExec_t chunk = nullptr;
  hipGraphExec_t rec_chunk = nullptr;
  double *rec_chunk_log = nullptr;
  // the same with the per-iteration trace (te_options.trace) into d_trace
  hipGraphExec_t trace_chunk = nullptr;
  double *trace_chunk_log = nullptr;
  int32_t *h_flag = nullptr;  // pinned: stop flags of chunks in flight
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // timing
  hipEvent_t pe[2] = {nullptr, nullptr};    // polling of the stop flag
  // workgroup engine: (block_threads, paths_per_lane) picked on the first solve that leaves one or
  // both at 0, per requested pair
  std::map<std::pair<int, int>, std::pair<int, int>> tuned;
  size_t lds_bytes = 0;
  // recorded solve for te_grad
  int32_t rec_K = 0, rec_ck = 16, rec_warm = 0;
  int64_t rec_gen = 0;  // bumped by every completed recording and every te_update
  double state_scale = 0.0;  // unit scale of the state the last graph-engine solve left (0: none)
  double *d_log = nullptr;      // [4 * log_cap]: beta, alpha, r, s of the recorded iterations
  int32_t log_cap = 0;
  double *d_trace = nullptr;    // [4 * trace_cap]: the same for a solve run with trace = 1
  int32_t trace_cap = 0;
  int32_t trace_engine = 0;     // engine of the last traced solve (0: none since the last untraced one)
  double *trace_src = nullptr;  // d_log or d_trace: where the last traced solve wrote
  int32_t trace_src_cap = 0;
  std::vector<FwdState> ckpt;   // checkpoints every rec_ck iterations
  std::vector<Ctrl *> ckpt_ctrl;
  std::vector<FwdState> seg;    // one segment of recomputed states
  AdjState adj{};
  int adj_ready = 0;
};

struct te_batch {
  int device = 0;
  int32_t n = 0;
  std::vector<int32_t> P, D, Eoff;
  std::vector<BatchDesc> desc;
  BatchDesc *d_desc = nullptr;
  BatchOut *d_out = nullptr;
  int32_t *d_i32 = nullptr;
  double *d_Dn = nullptr;
  double *d_Cn = nullptr;
  Params *d_params = nullptr;
  Params *h_params = nullptr;
  hipEvent_t params_ev = nullptr;
  double *d_sched = nullptr;
  int32_t sched_cap = 0;
  size_t lds_bytes = 0;
  int64_t totP = 0, totD = 0;
  std::vector<double> scales;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // (block_threads, paths_per_lane) picked on the first solve that leaves one or both at 0, per
  // requested pair
  std::map<std::pair<int, int>, std::pair<int, int>> tuned;
  // every instance fits one workgroup's LDS (else only the graph engine runs the batch)
  bool all_fit = true;
  std::vector<te_ctx *> members;
  // the graph engine's batch: one handle on the disjoint union of the instances, each in its own
  // normalised units, built on the first solve that uses it; per-demand output scales
  te_ctx *uni = nullptr;
  double *d_dscale = nullptr;
};

extern "C" {

const char *te_last_error(void) { return g_err.c_str(); }

void te_default_options(te_options *o) {
  std::memset(o, 0, sizeof(*o));
  o->alpha_target = INFINITY;
  o->gamma = 1e-3;
  o->beta0 = 1.0;
  o->A = 10.0;
  o->C = 2.0;
  o->beta_min = 1e-3;
  o->beta_max = 1e3;
  o->max_iters = 20000;
  o->alpha_max = 64;
  o->fixed_iters = 0;
  o->adapt_beta = 1;
  o->beta_every = 1;
  o->project = 1;
  o->engine = TE_ENGINE_AUTO;
  o->record = 0;
  o->ckpt_every = 16;
  o->sched_beta = nullptr;
  o->sched_alpha = nullptr;
  o->sched_len = 0;
  o->trace = 0;
  o->link_sums = TE_LINK_SUMS_AUTO;
  o->per_link = 0;
  o->w_min = 0.25;
  o->w_max = 4.0;
}

te_status te_validate(int32_t n_links, const double *capacity, int32_t n_paths, const int64_t *path_ptr,
                      const int32_t *path_links, int32_t n_demands, const int32_t *demand_path_ptr,
                      const double *demand) {
  if (n_links <= 0 || n_paths <= 0 || n_demands <= 0)
    return fail(TE_ERR_INVALID, "empty instance (links %d, paths %d, demands %d)", n_links, n_paths, n_demands);
  if (!capacity || !path_ptr || !path_links || !demand_path_ptr || !demand)
    return fail(TE_ERR_INVALID, "null input array");
  if (path_ptr[0] != 0) return fail(TE_ERR_INVALID, "path_ptr[0] must be 0");
  for (int32_t r = 0; r < n_paths; ++r)
    if (path_ptr[r + 1] <= path_ptr[r]) return fail(TE_ERR_INVALID, "path %d is empty or path_ptr decreases", r);
  const int64_t nnz = path_ptr[n_paths];
  if (nnz >= (int64_t)INT32_MAX) return fail(TE_ERR_INVALID, "too many path-link incidences (%lld)", (long long)nnz);
  std::vector<int32_t> stamp(n_links, -1);
  std::vector<char> used(n_links, 0);
  for (int32_t r = 0; r < n_paths; ++r)
    for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) {
      const int32_t e = path_links[i];
      if (e < 0 || e >= n_links) return fail(TE_ERR_INVALID, "path %d uses link id %d out of range", r, e);
      if (stamp[e] == r) return fail(TE_ERR_INVALID, "path %d uses link %d twice", r, e);
      stamp[e] = r;
      used[e] = 1;
    }
  if (demand_path_ptr[0] != 0) return fail(TE_ERR_INVALID, "demand_path_ptr[0] must be 0");
  if (demand_path_ptr[n_demands] != n_paths)
    return fail(TE_ERR_INVALID, "demand_path_ptr[n_demands] = %d, expected n_paths = %d", demand_path_ptr[n_demands],
                n_paths);
  for (int32_t c = 0; c < n_demands; ++c) {
    const int32_t m = demand_path_ptr[c + 1] - demand_path_ptr[c];
    if (m <= 0) return fail(TE_ERR_INVALID, "demand %d has no path", c);
    if (m > 64) return fail(TE_ERR_INVALID, "demand %d has %d paths (at most 64 supported)", c, m);
    if (!std::isfinite(demand[c]) || !(demand[c] > 0.0))
      return fail(TE_ERR_INVALID, "demand %d is %g (must be finite and > 0)", c, demand[c]);
  }
  for (int32_t e = 0; e < n_links; ++e) {
    if (!std::isfinite(capacity[e])) return fail(TE_ERR_INVALID, "capacity of link %d is not finite", e);
    if (used[e] && !(capacity[e] > 0.0))
      return fail(TE_ERR_INVALID, "link %d is used by a path but has capacity %g", e, capacity[e]);
  }
  return TE_OK;
}

}  // extern "C"

namespace {

void normalise(te_ctx *c) {
  double s = 0.0;
  for (int32_t i = 0; i < c->nnz; ++i) s = std::max(s, c->cap[c->plinks[i]]);
  c->scale = s;
  c->Cn.resize(c->E);
  c->Dn.resize(c->D);
  for (int32_t e = 0; e < c->E; ++e) c->Cn[e] = c->cap[e] / s;
  for (int32_t k = 0; k < c->D; ++k) c->Dn[k] = c->dem[k] / s;
}

te_status upload_values(te_ctx *c) {
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  HIPCHK(hipMemcpy(c->d_Cn, c->Cn.data(), sizeof(double) * c->E, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_Dn, c->Dn.data(), sizeof(double) * c->D, hipMemcpyHostToDevice));
  BatchDesc d{};
  d.E = c->E;
  d.P = c->P;
  d.D = c->D;
  d.nnz = c->nnz;
  d.G = c->G;
  d.logG = c->logG;
  d.off_pptr = 0;
  d.off_plinks = (int64_t)c->P + 1;
  d.off_dptr = d.off_plinks + c->nnz;
  d.off_lptr = d.off_dptr + c->D + 1;
  d.off_lpf = d.off_lptr + c->E + 1 + c->nnz;  // the pool holds lpaths, then lpf
  d.off_nzl = d.off_lpf + c->nnz;
  d.nzl = (int32_t)c->nzlink.size();
  d.off_E = d.off_P = d.off_D = 0;
  d.scale = c->scale;
  HIPCHK(hipMemcpy(c->d_desc, &d, sizeof(d), hipMemcpyHostToDevice));
  return TE_OK;
}

te_status stage_params(Params **d_params, Params *h_params, hipEvent_t ev, double **d_sched, int32_t *sched_cap,
                       const te_options *o, hipStream_t stream) {
  HIPCHK(hipEventSynchronize(ev));  // previous staging copy done
  Params p{};
  p.alpha_target = o->alpha_target;
  p.gamma = o->gamma;
  p.A = o->A;
  p.C = o->C;
  p.beta_min = o->beta_min;
  p.beta_max = o->beta_max;
  p.beta0 = o->beta0;
  p.fixed = o->fixed_iters > 0;
  p.kmax = o->fixed_iters > 0 ? o->fixed_iters : o->max_iters;
  p.adapt_beta = o->adapt_beta;
  p.beta_every = o->beta_every > 0 ? o->beta_every : 1;
  p.alpha_max = o->alpha_max;
  p.per_link = o->per_link;
  p.w_min = o->w_min;
  p.w_max = o->w_max;
  p.sched_len = 0;
  p.sched_beta = p.sched_alpha = nullptr;
  if (o->sched_beta && o->sched_alpha && o->sched_len > 0) {
    if (*sched_cap < o->sched_len) {
      if (*d_sched) HIPCHK(hipFree(*d_sched));
      *d_sched = nullptr;
      HIPCHK(dalloc(d_sched, 2 * (size_t)o->sched_len));
      *sched_cap = o->sched_len;
    }
    HIPCHK(hipMemcpyAsync(*d_sched, o->sched_beta, sizeof(double) * o->sched_len, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(*d_sched + o->sched_len, o->sched_alpha, sizeof(double) * o->sched_len,
                          hipMemcpyHostToDevice, stream));
    p.sched_len = o->sched_len;
    p.sched_beta = *d_sched;
    p.sched_alpha = *d_sched + o->sched_len;
  }
  *h_params = p;
  HIPCHK(hipMemcpyAsync(*d_params, h_params, sizeof(Params), hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(ev, stream));
  return TE_OK;
}

// The workgroup engine's (threads, paths per lane) for a solve that left one or both at 0: every
// candidate pair (the unspecified members vary over {1024, 512, 256} x {1, 2, 4, 8}) runs
// launch(threads, ppl, iterations) for min(max(fixed_iters, 256), 512) iterations after a short
// warm-up launch, timed with events on the stream; the fastest pair is returned.  The launches
// write the caller's outputs, which the solve that follows overwrites.
template <class Launch>
te_status tune_block_shape(int threads, int ppl, int fixed_iters, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1,
                           Launch &&launch, std::pair<int, int> *pick) {
  const int K_t = std::min(std::max(fixed_iters, 256), 512);
  const int cand_t[3] = {1024, 512, 256}, cand_p[4] = {1, 2, 4, 8};
  float best = 0.f;
  *pick = std::make_pair(0, 0);
  for (int i = 0; i < 3; ++i) {
    if (threads != 0 && cand_t[i] != threads) continue;
    for (int k = 0; k < 4; ++k) {
      if (ppl != 0 && cand_p[k] != ppl) continue;
      for (int q = 0; q < 2; ++q) {  // q = 0: warm-up launch that also sets up the kernel
        HIPCHK(hipEventRecord(ev0, stream));
        te_status s = launch(cand_t[i], cand_p[k], q == 0 ? 8 : K_t);
        if (s != TE_OK) return s;
        HIPCHK(hipEventRecord(ev1, stream));
      }
      HIPCHK(hipEventSynchronize(ev1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      if (pick->first == 0 || ms < best) {
        best = ms;
        *pick = std::make_pair(cand_t[i], cand_p[k]);
      }
    }
  }
  return TE_OK;
}

te_status check_options(const te_options *o) {
  if (!(o->gamma >= 0.0) || !(o->beta0 > 0.0) || !(o->A > 0.0) || !(o->C > 1.0) || !(o->beta_min > 0.0) ||
      !(o->beta_max >= o->beta_min) || !(o->alpha_target >= 0.0))
    return fail(TE_ERR_INVALID, "invalid options (gamma, beta0, A, C, beta bounds or alpha_target)");
  if (o->fixed_iters <= 0 && o->max_iters <= 0) return fail(TE_ERR_INVALID, "max_iters must be > 0");
  if (o->sched_len < 0) return fail(TE_ERR_INVALID, "sched_len < 0");
  if (o->block_threads != 0 && o->block_threads != 256 && o->block_threads != 512 && o->block_threads != 1024)
    return fail(TE_ERR_INVALID, "block_threads must be 0, 256, 512 or 1024");
  if (o->paths_per_lane != 0 && o->paths_per_lane != 1 && o->paths_per_lane != 2 && o->paths_per_lane != 4 &&
      o->paths_per_lane != 8)
    return fail(TE_ERR_INVALID, "paths_per_lane must be 0, 1, 2, 4 or 8");
  if (o->link_sums < 0 || o->link_sums > 3) return fail(TE_ERR_INVALID, "link_sums must be 0, 1, 2 or 3");
  if (o->per_link) {
    if (!(o->w_min > 0.0) || !(o->w_max >= o->w_min) || !(1.0 >= o->w_min) || !(1.0 <= o->w_max))
      return fail(TE_ERR_INVALID, "per_link needs 0 < w_min <= 1 <= w_max");
    if (o->link_sums == TE_LINK_SUMS_PRIVATE || o->link_sums == TE_LINK_SUMS_PRIVATE_ATOMIC)
      return fail(TE_ERR_INVALID, "per_link runs with the CSC link sums (link_sums 0 or 2)");
    if (o->record) return fail(TE_ERR_INVALID, "per_link cannot be recorded for te_grad");
    if (o->engine == TE_ENGINE_BLOCK) return fail(TE_ERR_INVALID, "per_link runs on the graph engine");
  }
  return TE_OK;
}

// Captures kChunk iterations on state st into *out (once; kept until the handle is destroyed).
te_status capture_chunk(te_ctx *c, const State &st, hipGraphExec_t *out) {
  if (*out) return TE_OK;
  hipStream_t cap;
  HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < kChunk; ++i) {
    hipError_t e = launch_iteration(c->prob, st, c->d_params, i & 1, cap);
    if (e != hipSuccess) {
      hipGraph_t g;
      (void)hipStreamEndCapture(cap, &g);
      (void)hipStreamDestroy(cap);
      return fail(TE_ERR_DEVICE, "iteration launch during capture: %s", hipGetErrorString(e));
    }
  }
  hipGraph_t g;
  HIPCHK(hipStreamEndCapture(cap, &g));
  HIPCHK(hipGraphInstantiate(out, g, nullptr, nullptr, 0));
  HIPCHK(hipGraphDestroy(g));
  HIPCHK(hipStreamDestroy(cap));
  return TE_OK;
}

te_status build_chunk_graph(te_ctx *c, hipStream_t) { return capture_chunk(c, c->st, &c->chunk); }

// The iteration chunk that also writes the per-iteration trace into st.log (recaptured when the
// trace buffer has moved).
te_status trace_graph(te_ctx *c, const State &st, hipGraphExec_t *out) {
  if (c->trace_chunk && c->trace_chunk_log != st.log) {
    HIPCHK(hipGraphExecDestroy(c->trace_chunk));
    c->trace_chunk = nullptr;
  }
  te_status s = capture_chunk(c, st, &c->trace_chunk);
  if (s != TE_OK) return s;
  c->trace_chunk_log = st.log;
  *out = c->trace_chunk;
  return TE_OK;
}

// Paths per lane of the graph engine's demand kernel: one lane per path, or -- for instances with
// at least kMultiLanes lane slots (demands x G), where that kernel is bound by issue and bandwidth
// rather than latency -- min(G, kMultiPaths).
int default_graph_ppl(const te_ctx *c) {
  return (int64_t)c->D * c->G >= kMultiLanes ? std::min(c->G, kMultiPaths) : 1;
}

// Rows of per-wavefront partial sums the demand kernels can leave: one lane per path with the CSC
// link kernel (the largest grid), or 16 per scatter workgroup.
int64_t partA_rows(const te_ctx *c) {
  const int64_t csc = (int64_t)((c->D + (kThreads >> c->logG) - 1) / (kThreads >> c->logG)) * (kThreads / 64);
  const int64_t scat = (int64_t)c->ncu * (kScatThreads / 64);
  return std::max(csc, scat);
}

// Link lists of the privatised sums for the launch shape in c->prob (Prob::cpp .. Prob::lchk): the
// longest chunks of passes whose paths' rates fit the LDS beside the E loads, as even as that
// count of chunks allows.  A chunk's link runs (the rate slots of its paths on one link) are cut
// into pieces of at most kPieceLen, sorted by length (longest first, then by link) and dealt 64 to
// a group, so that the lanes of a group sum pieces of about one length (the chunks of the
// 1,000-node instance hold runs of 1 to ~2,300 entries, 4 at the median).  cpp = 0 (an LDS atomic
// addition per incidence) when one pass does not fit or the lists cannot be allocated.
void build_lists(te_ctx *c) {
  Prob &p = c->prob;
  if (c->d_lent) (void)hipFree(c->d_lent);
  if (c->d_lgrp) (void)hipFree(c->d_lgrp);
  if (c->d_lchk) (void)hipFree(c->d_lchk);
  c->d_lent = nullptr;
  c->d_lgrp = nullptr;
  c->d_lchk = nullptr;
  c->n_lent = 0;
  p.cpp = p.cpw = p.zslot = 0;
  p.lent = nullptr;
  p.lgrp = nullptr;
  p.lchk = nullptr;
  if (c->E > 0x7fff) return;  // link ids of the group headers hold 15 bits
  const int per = kScatThreads >> c->logGp;
  const int64_t slots = ((int64_t)kScatLds - 8 * (int64_t)c->E) / 8 - 1;  // one more: the zero slot
  auto first_path = [&](int64_t ps) { return c->dptr[std::min<int64_t>(ps * per, c->D)]; };
  // most paths of a chunk when the passes of each workgroup go in chunks of cpp
  auto most_paths = [&](int cpp) {
    int64_t m = 0;
    for (int64_t b = 0; b < p.nF; ++b) {
      const int64_t pe = std::min<int64_t>((b + 1) * p.spw, p.npass);
      for (int64_t ps = b * p.spw; ps < pe; ps += cpp)
        m = std::max<int64_t>(m, first_path(std::min<int64_t>(ps + cpp, pe)) - first_path(ps));
    }
    return m;
  };
  int cmax = 0;
  for (int cpp = p.spw; cpp >= 1 && cmax == 0; --cpp)
    if (most_paths(cpp) <= slots) cmax = cpp;
  if (cmax == 0) return;
  const int nch = (p.spw + cmax - 1) / cmax;
  int cpp = (p.spw + nch - 1) / nch;
  if (most_paths(cpp) > slots) cpp = cmax;
  const int cpw = (p.spw + cpp - 1) / cpp;
  const int32_t zslot = (int32_t)most_paths(cpp);
  std::vector<int4> chk((size_t)p.nF * cpw, make_int4(0, 0, 0, 0));
  std::vector<int2> grp;
  std::vector<uint16_t> ent;
  ent.reserve((size_t)c->nnz * 9 / 8 + 64);
  std::vector<int32_t> cnt(c->E, 0), st(c->E, 0), pos(c->E, 0);
  std::vector<int32_t> run;  // the chunk's rate slots, link after link
  struct Piece {
    int32_t len, e, start;
    bool split;
  };
  std::vector<Piece> pc;
  for (int64_t b = 0; b < p.nF; ++b) {
    const int64_t pe = std::min<int64_t>((b + 1) * p.spw, p.npass);
    for (int k = 0; k < cpw; ++k) {
      const int64_t ps = b * p.spw + (int64_t)k * cpp;
      const int64_t ps1 = std::min<int64_t>(ps + cpp, pe);
      int4 &ch = chk[(size_t)b * cpw + k];
      ch = make_int4((int)grp.size(), (int)grp.size(), 0, 0);
      if (ps >= ps1) continue;
      const int32_t r0 = first_path(ps), r1 = first_path(ps1);
      ch.z = r0;
      int32_t emin = c->E, emax = -1;
      for (int32_t i = c->pptr[r0]; i < c->pptr[r1]; ++i) {
        const int32_t e = c->plinks[i];
        ++cnt[e];
        emin = std::min(emin, e);
        emax = std::max(emax, e);
      }
      if (emax < 0) continue;
      int32_t n = 0;
      for (int32_t e = emin; e <= emax; ++e) {
        st[e] = pos[e] = n;
        n += cnt[e];
      }
      run.assign(n, 0);
      for (int32_t r = r0; r < r1; ++r)  // paths ascending: every run in path order
        for (int32_t i = c->pptr[r]; i < c->pptr[r + 1]; ++i) run[pos[c->plinks[i]]++] = r - r0;
      pc.clear();
      for (int32_t e = emin; e <= emax; ++e)
        for (int32_t q = 0; q < cnt[e]; q += kPieceLen)
          pc.push_back({std::min(kPieceLen, cnt[e] - q), e, st[e] + q, cnt[e] > kPieceLen});
      std::stable_sort(pc.begin(), pc.end(), [](const Piece &x, const Piece &y) { return x.len > y.len; });
      for (size_t g0 = 0; g0 < pc.size(); g0 += 64) {
        const int32_t nb = (pc[g0].len + 7) / 8;  // blocks of 8 rows
        const size_t off = ent.size();
        if (off + (size_t)(1 + 8 * nb) * 64 > (size_t)INT32_MAX) return;
        grp.push_back(make_int2((int)off, nb));
        ent.resize(off + (size_t)(1 + 8 * nb) * 64, (uint16_t)zslot);
        uint16_t *ge = ent.data() + off;
        for (int i = 0; i < 64; ++i) {
          if (g0 + i >= pc.size()) {
            ge[i] = 0xffff;  // no piece
            continue;
          }
          const Piece &q = pc[g0 + i];
          ge[i] = (uint16_t)(q.e | (q.split ? 0x8000 : 0));
          for (int32_t j = 0; j < q.len; ++j) ge[64 + 512 * (j / 8) + 8 * i + (j % 8)] = (uint16_t)run[q.start + j];
        }
      }
      ch.y = (int)grp.size();
      for (int32_t e = emin; e <= emax; ++e) cnt[e] = 0;
    }
  }
  if (grp.empty() || dalloc(&c->d_lent, ent.size()) != hipSuccess || dalloc(&c->d_lgrp, grp.size()) != hipSuccess ||
      dalloc(&c->d_lchk, chk.size()) != hipSuccess ||
      hipMemcpy(c->d_lent, ent.data(), sizeof(uint16_t) * ent.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_lgrp, grp.data(), sizeof(int2) * grp.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_lchk, chk.data(), sizeof(int4) * chk.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    void *bufs[] = {c->d_lent, c->d_lgrp, c->d_lchk};
    for (void *q : bufs)
      if (q) (void)hipFree(q);
    c->d_lent = nullptr;
    c->d_lgrp = nullptr;
    c->d_lchk = nullptr;
    return;
  }
  c->n_lent = (int64_t)ent.size();
  p.cpp = cpp;
  p.cpw = cpw;
  p.zslot = zslot;
  p.lent = c->d_lent;
  p.lgrp = c->d_lgrp;
  p.lchk = c->d_lchk;
}

// Launch shape of the graph engine for ppl paths per lane and link sums lsum (kLinkSums*).
// Privatised sums: passes of kScatThreads / 2^logGp demands, dealt in runs of spw consecutive
// passes to at most one scatter workgroup per compute unit (each holds the E loads in LDS).
void set_graph_shape(te_ctx *c, int ppl, int lsum) {
  int logp = 0;
  while ((1 << logp) < ppl) ++logp;
  c->ppl = ppl;
  c->logGp = c->logG > logp ? c->logG - logp : 0;
  c->lsum = lsum;
  Prob &p = c->prob;
  p.ppl = c->ppl;
  p.logGp = c->logGp;
  const bool priv = lsum == kLinkSumsPrivate || lsum == kLinkSumsPrivateAtomic;
  p.lsum = priv ? kLinkSumsPrivate : lsum;
  if (priv) {
    const int per = kScatThreads >> c->logGp;
    p.npass = (c->D + per - 1) / per;
    p.spw = (p.npass + c->ncu - 1) / c->ncu;
    p.nF = (p.npass + p.spw - 1) / p.spw;
    c->st.nA = p.nF;
    c->st.nArows = p.nF * (kScatThreads / 64);
    c->st.nB = (c->E + 63) / 64;
    if (lsum == kLinkSumsPrivate) {
      build_lists(c);
    } else {
      p.cpp = 0;
    }
  } else {
    p.npass = p.spw = p.nF = 0;
    p.cpp = 0;
    c->st.nA = (c->D + (kThreads >> c->logGp) - 1) / (kThreads >> c->logGp);
    c->st.nArows = c->st.nA * (kThreads / 64);
    c->st.nB = c->nB_csc;
  }
}

// Link sums of the graph engine by default: privatised for instances with at least kMultiLanes lane
// slots (demands x G) whose links fit one workgroup's LDS -- there the kernels are bound by bandwidth
// and issue, and the privatised sums save the second pass over the incidence (measured on the
// 1,000-node instance) -- else CSC: smaller instances are latency-bound, and the scatter kernel's one
// pass of 1,024-thread workgroups plus the row reduction cost more than the CSC link kernel
// (measured on the 150-node instance).
int default_link_sums(const te_ctx *c) {
  return ((int64_t)c->D * c->G >= kMultiLanes && c->E <= kMaxScatterLinks) ? kLinkSumsPrivate : kLinkSumsCsc;
}

// The options' paths per lane (0: the default) and link sums (0: default_link_sums) for the graph
// engine; a change recaptures the iteration graphs, which hold the kernels' launch shapes.
te_status select_graph_shape(te_ctx *c, const te_options &o) {
  const int want = o.paths_per_lane ? o.paths_per_lane : default_graph_ppl(c);
  int lsum = o.link_sums ? o.link_sums : default_link_sums(c);
  if (o.per_link) lsum = kLinkSumsCsc;  // the per-link rule needs per-link sums of (x' - x)^2
  if ((lsum == kLinkSumsPrivate || lsum == kLinkSumsPrivateAtomic) && c->E > kMaxScatterLinks)
    return fail(TE_ERR_INVALID, "privatised link sums hold at most %d links (instance: %d)", kMaxScatterLinks, c->E);
  if (want == c->ppl && lsum == c->lsum) return TE_OK;
  HIPCHK(hipDeviceSynchronize());  // no launch of the old graphs may still be in flight
  if (c->chunk) HIPCHK(hipGraphExecDestroy(c->chunk));
  if (c->rec_chunk) HIPCHK(hipGraphExecDestroy(c->rec_chunk));
  if (c->trace_chunk) HIPCHK(hipGraphExecDestroy(c->trace_chunk));
  c->chunk = nullptr;
  c->rec_chunk = nullptr;
  c->trace_chunk = nullptr;
  set_graph_shape(c, want, lsum);
  return TE_OK;
}

// An iteration state (x, u_neg, u_dem, S, (g, q)) lives in one block, x | u_neg | u_dem | S | gq,
// so that a checkpoint or a segment step is one copy.
size_t fwd_doubles(const te_ctx *c) { return 2 * (size_t)c->P + 2 * (size_t)c->D + 2 * (size_t)c->E; }

FwdState fwd_in(double *base, const te_ctx *c) {
  FwdState f;
  f.x = base;
  f.uneg = f.x + c->P;
  f.udem = f.uneg + c->P;
  f.S = f.udem + c->D;
  f.gq = reinterpret_cast<double2 *>(f.S + c->D);  // offset 2(P + D) doubles: 16-byte aligned
  return f;
}

hipError_t alloc_fwd(FwdState &f, const te_ctx *c) {
  double *base = nullptr;
  hipError_t e = dalloc(&base, fwd_doubles(c));
  if (e == hipSuccess) f = fwd_in(base, c);
  return e;
}

void free_fwd(FwdState &f) {
  if (f.x) (void)hipFree(f.x);
  f = FwdState{};
}

te_status ensure_ckpts(te_ctx *c, int n) {
  while ((int)c->ckpt.size() < n) {
    FwdState f{};
    Ctrl *cc = nullptr;
    if (alloc_fwd(f, c) != hipSuccess || dalloc(&cc, 1) != hipSuccess) {
      free_fwd(f);
      if (cc) (void)hipFree(cc);
      return fail(TE_ERR_OOM, "checkpoint allocation failed");
    }
    c->ckpt.push_back(f);
    c->ckpt_ctrl.push_back(cc);
  }
  return TE_OK;
}

hipError_t copy_fwd(const FwdState &dst, const FwdState &src, const te_ctx *c, hipStream_t st) {
  return hipMemcpyAsync(dst.x, src.x, sizeof(double) * fwd_doubles(c), hipMemcpyDeviceToDevice, st);
}

void fill_stats(te_stats *s, const Ctrl &c, int engine, double ms, int block_threads, int ppl) {
  s->iters = c.k;
  s->flags = c.flags;
  s->stop_iter = c.stop_iter;
  s->engine = engine;
  s->block_threads = engine == TE_ENGINE_BLOCK ? block_threads : 0;
  s->paths_per_lane = ppl;
  s->final_alpha = c.alpha;
  s->beta = c.beta;
  s->r = c.r;
  s->s = c.s;
  s->max_cap_viol_rel = c.cap_viol;
  s->max_dem_viol_rel = c.dem_viol;
  s->ms = ms;
}

}  // namespace

extern "C" {

te_status te_create(int32_t n_links, const double *capacity, int32_t n_paths, const int64_t *path_ptr,
                    const int32_t *path_links, int32_t n_demands, const int32_t *demand_path_ptr,
                    const double *demand, int32_t hip_device, te_ctx **out) {
  if (!out) return fail(TE_ERR_INVALID, "out is null");
  *out = nullptr;
  te_status v = te_validate(n_links, capacity, n_paths, path_ptr, path_links, n_demands, demand_path_ptr, demand);
  if (v != TE_OK) return v;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(TE_ERR_DEVICE, "no HIP device available");
  if (hip_device < 0 || hip_device >= ndev) return fail(TE_ERR_INVALID, "hip_device %d out of range", hip_device);
  te_ctx *c = new (std::nothrow) te_ctx();
  if (!c) return fail(TE_ERR_OOM, "host allocation");
  c->device = hip_device;
  c->E = n_links;
  c->P = n_paths;
  c->D = n_demands;
  c->nnz = (int32_t)path_ptr[n_paths];
  c->cap.assign(capacity, capacity + n_links);
  c->dem.assign(demand, demand + n_demands);
  c->pptr.resize(n_paths + 1);
  for (int32_t r = 0; r <= n_paths; ++r) c->pptr[r] = (int32_t)path_ptr[r];
  c->plinks.assign(path_links, path_links + c->nnz);
  c->dptr.assign(demand_path_ptr, demand_path_ptr + n_demands + 1);
  // link -> path CSC, paths ascending within a link
  c->lptr.assign(n_links + 1, 0);
  for (int32_t i = 0; i < c->nnz; ++i) c->lptr[c->plinks[i] + 1]++;
  for (int32_t e = 0; e < n_links; ++e) c->lptr[e + 1] += c->lptr[e];
  c->lpaths.resize(c->nnz);
  {
    std::vector<int32_t> fill(c->lptr.begin(), c->lptr.end() - 1);
    for (int32_t r = 0; r < n_paths; ++r)
      for (int32_t i = c->pptr[r]; i < c->pptr[r + 1]; ++i) c->lpaths[fill[c->plinks[i]]++] = r;
  }
  // link-kernel work split: workgroups own contiguous runs of non-empty links of ~nnz/nB entries
  c->lpf = c->lpaths;
  for (int32_t e = 0; e < n_links; ++e) {
    if (c->lptr[e + 1] > c->lptr[e]) {
      c->lpf[c->lptr[e]] |= (int32_t)0x80000000u;
      c->nzlink.push_back(e);
      c->nzptr.push_back(c->lptr[e]);
    }
  }
  c->nzptr.push_back(c->nnz);
  {
    // runs of whole links of about `target` entries (at most kMaxLinksPerBlock links); links larger
    // than the target make runs of their own, so the target grows until at most kMaxLinkBlocks
    // workgroups result (the control prefetch reads that many partial-sum rows)
    const int64_t want = std::min<int64_t>(kMaxLinkBlocks, std::max<int64_t>(1, (c->nnz + 4095) / 4096));
    int64_t target = std::max<int64_t>(1, (c->nnz + want - 1) / want);
    for (;;) {
      c->blk.assign(1, 0);
      int64_t cur = 0;
      int cnt = 0;
      for (size_t k = 0; k < c->nzlink.size(); ++k) {
        const int64_t d = c->nzptr[k + 1] - c->nzptr[k];
        if (cnt > 0 && (cur + d > target || cnt == kMaxLinksPerBlock)) {
          c->blk.push_back((int32_t)k);
          cur = 0;
          cnt = 0;
        }
        cur += d;
        ++cnt;
      }
      c->blk.push_back((int32_t)c->nzlink.size());
      if ((int64_t)c->blk.size() - 1 <= kMaxLinkBlocks) break;
      if (target >= (int64_t)c->nnz) {  // only reachable with more than kMaxLinkBlocks * kMaxLinksPerBlock links
        te_destroy(c);
        return fail(TE_ERR_INVALID, "more than %d used links", kMaxLinkBlocks * kMaxLinksPerBlock);
      }
      target += target / 8 + 1;
    }
  }
  const int nB = (int)c->blk.size() - 1;
  // per-wavefront parts of each workgroup's CSC entries (the split the link kernels use)
  std::vector<int4> wtab((size_t)nB * kLinkWaves);
  for (int b = 0; b < nB; ++b) {
    const int32_t k0 = c->blk[b], k1 = c->blk[b + 1];
    const int32_t j0 = c->nzptr[k0], len = c->nzptr[k1] - j0;
    const int32_t per = (len + kLinkWaves - 1) / kLinkWaves;
    int32_t k = k0;
    for (int w = 0; w < kLinkWaves; ++w) {
      const int32_t ja = j0 + std::min(len, w * per), jb = j0 + std::min(len, (w + 1) * per);
      while (k + 1 < k1 && c->nzptr[k + 1] <= ja) ++k;
      wtab[(size_t)b * kLinkWaves + w] = make_int4(ja, jb, k, 0);
    }
  }
  c->maxp = 0;
  for (int32_t k = 0; k < n_demands; ++k) c->maxp = std::max(c->maxp, c->dptr[k + 1] - c->dptr[k]);
  c->G = 1;
  c->logG = 0;
  while (c->G < c->maxp) {
    c->G <<= 1;
    c->logG++;
  }
  normalise(c);
  c->lds_bytes = block_lds_bytes(c->E, c->P, c->D, c->nnz);

  auto cleanup_fail = [&](te_status s) {
    te_destroy(c);
    return s;
  };
  DeviceScope dscope(hip_device);
  if (dscope.err != hipSuccess) return cleanup_fail(fail(TE_ERR_DEVICE, "hipSetDevice failed"));
  // index pool: pptr | plinks | dptr | lptr | lpaths
  const size_t ni = (size_t)(c->P + 1) + c->nnz + (c->D + 1) + (c->E + 1) + c->nnz + c->nnz + c->nzlink.size() +
                    c->nzptr.size() + c->blk.size();
  // launch shapes: CSC link kernel of nB workgroups, or the privatised sums when the links fit
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
      c->ncu = prop.multiProcessorCount;
  }
  c->nB_csc = nB;
  const bool priv_ok = c->E <= kMaxScatterLinks;
  set_graph_shape(c, default_graph_ppl(c), default_link_sums(c));
  const int64_t nBmax = std::max<int64_t>(nB, (c->E + 63) / 64);
  bool ok = dalloc(&c->d_i32, ni) == hipSuccess && dalloc(&c->d_Dn, c->D) == hipSuccess &&
            dalloc(&c->d_Cn, c->E) == hipSuccess && alloc_fwd(c->work, c) == hipSuccess &&
            dalloc(&c->st.ctrl, 3) == hipSuccess && dalloc(&c->st.partA, (size_t)2 * partA_rows(c) * 4) == hipSuccess &&
            dalloc(&c->st.partB, (size_t)2 * nBmax * 4) == hipSuccess &&
            (!priv_ok || dalloc(&c->st.partL, (size_t)c->ncu * c->E) == hipSuccess) &&
            dalloc(&c->st.w, c->E) == hipSuccess && dalloc(&c->st.dx2, c->P) == hipSuccess &&
            dalloc(&c->pb.xd, c->P) == hipSuccess && dalloc(&c->pb.S, c->D) == hipSuccess &&
            dalloc(&c->pb.L, c->E) == hipSuccess && dalloc(&c->pb.Cp, c->P) == hipSuccess &&
            dalloc(&c->pb.lsc, c->P) == hipSuccess && dalloc(&c->pb.trim, c->P) == hipSuccess &&
            dalloc(&c->d_params, 1) == hipSuccess && dalloc(&c->d_desc, 1) == hipSuccess &&
            dalloc(&c->d_bout, 1) == hipSuccess && dalloc(&c->d_wtab, wtab.size()) == hipSuccess;
  if (!ok) return cleanup_fail(fail(TE_ERR_OOM, "device allocation failed"));
  c->st.x = c->st.xo = c->work.x;
  c->st.uneg = c->st.unego = c->work.uneg;
  c->st.udem = c->st.udemo = c->work.udem;
  c->st.S = c->st.So = c->work.S;
  c->st.gq = c->st.gqo = c->work.gq;
  if (hipMemcpy(c->d_wtab, wtab.data(), sizeof(int4) * wtab.size(), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup_fail(fail(TE_ERR_DEVICE, "copy of the link work table failed"));
  if (hipHostMalloc((void **)&c->h_params, sizeof(Params)) != hipSuccess ||
      hipHostMalloc((void **)&c->h_flag, sizeof(int32_t) * 4) != hipSuccess)
    return cleanup_fail(fail(TE_ERR_OOM, "pinned host allocation failed"));
  if (hipEventCreate(&c->params_ev) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
      hipEventCreate(&c->ev1) != hipSuccess || hipEventCreate(&c->pe[0]) != hipSuccess ||
      hipEventCreate(&c->pe[1]) != hipSuccess)
    return cleanup_fail(fail(TE_ERR_DEVICE, "event creation failed"));
  {
    void *sb = nullptr;  // the static scratch of te_project_rates_static: address looked up once per device
    size_t sbytes = 0;
    if (static_scratch(&sb, &sbytes) != hipSuccess)
      return cleanup_fail(fail(TE_ERR_DEVICE, "address of the static scratch could not be looked up"));
  }
  if (priv_ok) {
    static bool prepared[64] = {false};
    if (hip_device < 64 && !prepared[hip_device]) {
      if (prepare_scatter_kernels() != hipSuccess)
        return cleanup_fail(fail(TE_ERR_DEVICE, "LDS limit of the privatised-sum kernels could not be raised"));
      prepared[hip_device] = true;
    }
  }
  {
    std::vector<int32_t> pool;
    pool.reserve(ni);
    pool.insert(pool.end(), c->pptr.begin(), c->pptr.end());
    pool.insert(pool.end(), c->plinks.begin(), c->plinks.end());
    pool.insert(pool.end(), c->dptr.begin(), c->dptr.end());
    pool.insert(pool.end(), c->lptr.begin(), c->lptr.end());
    pool.insert(pool.end(), c->lpaths.begin(), c->lpaths.end());
    pool.insert(pool.end(), c->lpf.begin(), c->lpf.end());
    pool.insert(pool.end(), c->nzlink.begin(), c->nzlink.end());
    pool.insert(pool.end(), c->nzptr.begin(), c->nzptr.end());
    pool.insert(pool.end(), c->blk.begin(), c->blk.end());
    if (hipMemcpy(c->d_i32, pool.data(), sizeof(int32_t) * ni, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup_fail(fail(TE_ERR_DEVICE, "copy of the index pool failed"));
  }
  // fixed-width hop records of the demand kernels (when every path fits kMaxHopSlots and every
  // link id fits 16 bits): the row-pointer load before the link ids is then not needed.  A path's
  // first kPrimarySlots ids sit in its primary record; the paths of a demand with a longer path
  // continue in overflow records of H2 more slots, one per path of that demand, so that paths of
  // up to 16 hops do not pad every record to 16 slots (1,000-node instance: 5.9 hops on average,
  // 15 at most, 15 % of the demands with a path of more than 8)
  {
    int maxh = 0;
    for (int32_t r = 0; r < c->P; ++r) maxh = std::max(maxh, c->pptr[r + 1] - c->pptr[r]);
    const int Htot = (maxh + 3) & ~3;
    if (Htot <= kMaxHopSlots && c->E < 0xffff) {
      c->H = std::min(Htot, kPrimarySlots);
      c->H2 = Htot - c->H;
      std::vector<uint16_t> hops((size_t)c->P * c->H, (uint16_t)0xffff);
      for (int32_t r = 0; r < c->P; ++r)
        for (int32_t i = c->pptr[r]; i < std::min(c->pptr[r + 1], c->pptr[r] + c->H); ++i)
          hops[(size_t)r * c->H + (i - c->pptr[r])] = (uint16_t)c->plinks[i];
      if (dalloc(&c->d_hops, hops.size()) != hipSuccess)
        return cleanup_fail(fail(TE_ERR_OOM, "device allocation failed"));
      if (hipMemcpy(c->d_hops, hops.data(), sizeof(uint16_t) * hops.size(), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup_fail(fail(TE_ERR_DEVICE, "copy of the hop records failed"));
      if (c->H2 > 0) {
        std::vector<int32_t> dovf(c->D, -1);
        int64_t n2 = 0;
        for (int32_t d = 0; d < c->D; ++d) {
          bool longp = false;
          for (int32_t r = c->dptr[d]; r < c->dptr[d + 1]; ++r) longp = longp || c->pptr[r + 1] - c->pptr[r] > c->H;
          if (longp) {
            dovf[d] = (int32_t)n2;
            n2 += c->dptr[d + 1] - c->dptr[d];
          }
        }
        std::vector<uint16_t> hops2((size_t)n2 * c->H2, (uint16_t)0xffff);
        for (int32_t d = 0; d < c->D; ++d) {
          if (dovf[d] < 0) continue;
          for (int32_t r = c->dptr[d]; r < c->dptr[d + 1]; ++r) {
            const size_t rec = (size_t)(dovf[d] + (r - c->dptr[d])) * c->H2;
            for (int32_t i = c->pptr[r] + c->H; i < c->pptr[r + 1]; ++i)
              hops2[rec + (i - c->pptr[r] - c->H)] = (uint16_t)c->plinks[i];
          }
        }
        if (dalloc(&c->d_hops2, hops2.size()) != hipSuccess || dalloc(&c->d_dovf, dovf.size()) != hipSuccess)
          return cleanup_fail(fail(TE_ERR_OOM, "device allocation failed"));
        if (hipMemcpy(c->d_hops2, hops2.data(), sizeof(uint16_t) * hops2.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->d_dovf, dovf.data(), sizeof(int32_t) * dovf.size(), hipMemcpyHostToDevice) != hipSuccess)
          return cleanup_fail(fail(TE_ERR_DEVICE, "copy of the overflow hop records failed"));
      }
    }
  }
  te_status s = upload_values(c);
  if (s != TE_OK) return cleanup_fail(s);
  Prob &p = c->prob;
  p.E = c->E;
  p.P = c->P;
  p.D = c->D;
  p.nnz = c->nnz;
  p.G = c->G;
  p.logG = c->logG;
  p.pptr = c->d_i32;
  p.plinks = p.pptr + c->P + 1;
  p.dptr = p.plinks + c->nnz;
  p.lptr = p.dptr + c->D + 1;
  p.lpaths = p.lptr + c->E + 1;
  p.lpf = p.lpaths + c->nnz;
  p.nzlink = p.lpf + c->nnz;
  p.nzptr = p.nzlink + c->nzlink.size();
  p.blk = p.nzptr + c->nzptr.size();
  p.wtab = c->d_wtab;
  p.hops = c->d_hops;
  p.H = c->d_hops ? c->H : 0;
  p.hops2 = c->d_hops2;
  p.H2 = c->d_hops2 ? c->H2 : 0;
  p.dovf = c->d_dovf;
  p.Dn = c->d_Dn;
  p.Cn = c->d_Cn;
  *out = c;
  return TE_OK;
}

te_status te_update(te_ctx *c, const double *capacity, const double *demand) {
  if (!c) return fail(TE_ERR_INVALID, "null handle");
  std::vector<double> cap = capacity ? std::vector<double>(capacity, capacity + c->E) : c->cap;
  std::vector<double> dem = demand ? std::vector<double>(demand, demand + c->D) : c->dem;
  std::vector<int64_t> pp(c->pptr.begin(), c->pptr.end());
  te_status v = te_validate(c->E, cap.data(), c->P, pp.data(), c->plinks.data(), c->D, c->dptr.data(), dem.data());
  if (v != TE_OK) return v;
  c->cap = cap;
  c->dem = dem;
  normalise(c);
  // a recording describes the trajectory under the old capacities and demands: te_grad refuses it
  c->rec_K = 0;
  c->rec_gen++;
  return upload_values(c);
}

te_status te_info(const te_ctx *c, int64_t *sz) {
  if (!c || !sz) return fail(TE_ERR_INVALID, "null argument");
  sz[0] = c->E;
  sz[1] = c->P;
  sz[2] = c->D;
  sz[3] = c->nnz;
  sz[4] = c->maxp;
  sz[5] = c->lds_bytes <= kMaxBlockLds ? TE_ENGINE_BLOCK : TE_ENGINE_GRAPH;
  sz[6] = c->st.nA;
  sz[7] = c->st.nB;
  sz[8] = c->d_hops ? c->H + (c->d_hops2 ? c->H2 : 0) : 0;
  sz[9] = c->rec_K > 0 ? c->rec_gen : 0;
  sz[10] = c->lsum;
  sz[11] = c->prob.nF;
  const bool lists = c->prob.lsum == kLinkSumsPrivate && c->prob.cpp > 0;
  sz[12] = lists ? c->prob.cpp : 0;
  sz[13] = lists ? c->n_lent : 0;
  return TE_OK;
}

te_status te_solve(te_ctx *c, const te_options *opt, void *hip_stream, const float *x0_dev, float *x_out_dev,
                   float *S_out_dev, te_stats *stats) {
  if (!c || !x_out_dev) return fail(TE_ERR_INVALID, "null handle or output");
  te_options o;
  if (opt) o = *opt; else te_default_options(&o);
  te_status s = check_options(&o);
  if (s != TE_OK) return s;
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  int engine = o.engine;
  if (o.record) {
    if (o.fixed_iters <= 0) return fail(TE_ERR_INVALID, "record = 1 needs fixed_iters > 0");
    engine = TE_ENGINE_GRAPH;
  }
  if (o.warm) {
    if (c->state_scale <= 0.0) return fail(TE_ERR_STATE, "warm = 1 needs an earlier graph-engine solve on this handle");
    if (o.record) return fail(TE_ERR_INVALID, "warm = 1 cannot be recorded for te_grad (the gradient starts cold)");
    if (engine == TE_ENGINE_BLOCK) return fail(TE_ERR_INVALID, "warm = 1 runs on the graph engine");
    engine = TE_ENGINE_GRAPH;
  }
  if (o.per_link) engine = TE_ENGINE_GRAPH;
  if (engine == TE_ENGINE_AUTO) engine = c->lds_bytes <= kMaxBlockLds ? TE_ENGINE_BLOCK : TE_ENGINE_GRAPH;
  if (engine == TE_ENGINE_BLOCK && c->lds_bytes > kMaxBlockLds)
    return fail(TE_ERR_INVALID, "instance needs %zu bytes of LDS, more than one workgroup has", c->lds_bytes);
  int bthreads = o.block_threads, bppl = o.paths_per_lane;
  if (engine == TE_ENGINE_BLOCK && (bthreads == 0 || bppl == 0)) {
    const std::pair<int, int> key(bthreads, bppl);
    auto it = c->tuned.find(key);
    if (it == c->tuned.end()) {
      std::pair<int, int> pick;
      Pools tp{c->d_i32, c->d_Dn, c->d_Cn, nullptr, nullptr, 0};
      s = tune_block_shape(bthreads, bppl, o.fixed_iters, stream, c->ev0, c->ev1,
                           [&](int th, int pl, int iters) -> te_status {
                             te_options t;
                             te_default_options(&t);
                             t.fixed_iters = iters;
                             t.project = 0;
                             te_status st = stage_params(&c->d_params, c->h_params, c->params_ev, &c->d_sched,
                                                         &c->sched_cap, &t, stream);
                             if (st != TE_OK) return st;
                             HIPCHK(launch_block_solve(c->d_desc, 1, tp, c->d_params, 0, x_out_dev, S_out_dev,
                                                       c->d_bout, c->lds_bytes, th, pl, stream));
                             return TE_OK;
                           },
                           &pick);
      if (s != TE_OK) return s;
      it = c->tuned.emplace(key, pick).first;
    }
    bthreads = it->second.first;
    bppl = it->second.second;
  }
  s = stage_params(&c->d_params, c->h_params, c->params_ev, &c->d_sched, &c->sched_cap, &o, stream);
  if (s != TE_OK) return s;
  // per-iteration trace (beta_k, alpha_k, r_k, s_k) of a solve that asks for it; a recorded solve
  // writes the same rows into its recording log
  const int kcap = o.fixed_iters > 0 ? o.fixed_iters : o.max_iters;
  c->trace_engine = 0;
  if (o.trace && !o.record) {
    if (c->trace_cap < kcap) {
      if (c->d_trace) HIPCHK(hipFree(c->d_trace));
      c->d_trace = nullptr;
      c->trace_cap = 0;
      HIPCHK(dalloc(&c->d_trace, 4 * (size_t)kcap));
      c->trace_cap = kcap;
    }
    c->trace_engine = engine;
    c->trace_src = c->d_trace;
    c->trace_src_cap = c->trace_cap;
  }
  HIPCHK(hipEventRecord(c->ev0, stream));
  if (engine == TE_ENGINE_BLOCK) {
    Pools pools{c->d_i32, c->d_Dn, c->d_Cn, x0_dev, o.trace ? c->d_trace : nullptr, o.trace ? c->trace_cap : 0};
    HIPCHK(launch_block_solve(c->d_desc, 1, pools, c->d_params, o.project, x_out_dev, S_out_dev, c->d_bout,
                              c->lds_bytes, bthreads, bppl, stream));
  } else {
    s = select_graph_shape(c, o);
    if (s != TE_OK) return s;
    s = build_chunk_graph(c, stream);
    if (s != TE_OK) return s;
    if (o.warm)
      HIPCHK(launch_warm(c->prob, c->st, c->d_params, c->state_scale / c->scale, stream));
    else
      HIPCHK(launch_init(c->prob, c->st, c->d_params, x0_dev, 1.0 / c->scale, stream));
    c->state_scale = c->scale;
    int launched = 0;
    if (o.record) {
      // plain launches with the (beta, alpha) log; the gradient pass replays it
      if (c->log_cap < o.fixed_iters) {
        if (c->d_log) HIPCHK(hipFree(c->d_log));
        c->d_log = nullptr;
        c->log_cap = 0;
        HIPCHK(dalloc(&c->d_log, 4 * (size_t)o.fixed_iters));
        c->log_cap = o.fixed_iters;
      }
      State sr = c->st;
      sr.log = c->d_log;
      sr.log_cap = c->log_cap;
      c->trace_engine = engine;  // the recording log doubles as the trace
      c->trace_src = c->d_log;
      c->trace_src_cap = c->log_cap;
      // checkpoints for te_grad every ck iterations: the state and the control record the next
      // iteration reads
      const int ck = o.ckpt_every > 0 ? o.ckpt_every : 16;
      s = ensure_ckpts(c, (o.fixed_iters + ck - 1) / ck);
      if (s != TE_OK) return s;
      c->rec_K = 0;  // valid again once the recording is complete
      if (ck % kChunk == 0) {  // the logging iterations as captured chunks (recaptured if the log moved)
        if (c->rec_chunk && c->rec_chunk_log != c->d_log) {
          HIPCHK(hipGraphExecDestroy(c->rec_chunk));
          c->rec_chunk = nullptr;
        }
        s = capture_chunk(c, sr, &c->rec_chunk);
        if (s != TE_OK) return s;
        c->rec_chunk_log = c->d_log;
      }
      for (launched = 0; launched < o.fixed_iters;) {
        if (launched % ck == 0) {
          HIPCHK(copy_fwd(c->ckpt[launched / ck], c->work, c, stream));
          HIPCHK(hipMemcpyAsync(c->ckpt_ctrl[launched / ck], c->st.ctrl + ((launched + 1) & 1), sizeof(Ctrl),
                                hipMemcpyDeviceToDevice, stream));
        }
        if (ck % kChunk == 0 && launched + kChunk <= o.fixed_iters) {
          HIPCHK(hipGraphLaunch(c->rec_chunk, stream));
          launched += kChunk;
        } else {
          HIPCHK(launch_iteration(c->prob, sr, c->d_params, launched & 1, stream));
          ++launched;
        }
      }
      c->rec_K = o.fixed_iters;
      c->rec_gen++;
      c->rec_ck = ck;
      c->rec_warm = x0_dev != nullptr;  // a given x^0 does not depend on the demands
    } else if (o.fixed_iters > 0) {
      const int K = o.fixed_iters;
      State si = c->st;
      hipGraphExec_t g = c->chunk;
      if (o.trace) {
        si.log = c->d_trace;
        si.log_cap = c->trace_cap;
        s = trace_graph(c, si, &g);
        if (s != TE_OK) return s;
      }
      while (launched + kChunk <= K) {
        HIPCHK(hipGraphLaunch(g, stream));
        launched += kChunk;
      }
      while (launched < K) {
        HIPCHK(launch_iteration(c->prob, si, c->d_params, launched & 1, stream));
        ++launched;
      }
    } else {
      // adaptive: chunks until the device-side stop flag is seen (one chunk in flight ahead)
      const int K = o.max_iters;
      hipGraphExec_t g = c->chunk;
      if (o.trace) {
        State si = c->st;
        si.log = c->d_trace;
        si.log_cap = c->trace_cap;
        s = trace_graph(c, si, &g);
        if (s != TE_OK) return s;
      }
      bool stopped = false;
      while (launched < K && !stopped) {
        HIPCHK(hipGraphLaunch(g, stream));
        launched += kChunk;
        const int slot = (launched / kChunk) & 1;
        HIPCHK(hipMemcpyAsync(&c->h_flag[slot], &c->st.ctrl[(launched - 1) & 1].stop, sizeof(int32_t),
                              hipMemcpyDeviceToHost, stream));
        HIPCHK(hipEventRecord(c->pe[slot], stream));
        if (launched / kChunk >= 2) {
          const int prev = slot ^ 1;
          HIPCHK(hipEventSynchronize(c->pe[prev]));
          if (c->h_flag[prev]) stopped = true;
        }
      }
    }
    const int last_par = launched > 0 ? (launched - 1) & 1 : 1;
    State sf = c->st;
    if (c->trace_engine) {
      sf.log = c->trace_src;
      sf.log_cap = c->trace_src_cap;
    }
    HIPCHK(launch_finish(sf, c->d_params, last_par, stream));
    HIPCHK(launch_project(c->prob, c->st, c->pb, x_out_dev, S_out_dev, c->scale, o.project, stream));
  }
  HIPCHK(hipEventRecord(c->ev1, stream));
  if (stats) {
    HIPCHK(hipStreamSynchronize(stream));
    Ctrl fin{};
    if (engine == TE_ENGINE_BLOCK) {
      BatchOut bo;
      HIPCHK(hipMemcpy(&bo, c->d_bout, sizeof(bo), hipMemcpyDeviceToHost));
      fin.k = bo.iters;
      fin.flags = bo.flags;
      fin.stop_iter = bo.stop_iter;
      fin.alpha = bo.alpha;
      fin.beta = bo.beta;
      fin.r = bo.r;
      fin.s = bo.s;
      fin.cap_viol = bo.cap_viol;
      fin.dem_viol = bo.dem_viol;
    } else {
      HIPCHK(hipMemcpy(&fin, c->st.ctrl + 2, sizeof(Ctrl), hipMemcpyDeviceToHost));
    }
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    fill_stats(stats, fin, engine, ms, engine == TE_ENGINE_BLOCK ? bthreads : 0,
               engine == TE_ENGINE_BLOCK ? bppl : c->ppl);
    if (!std::isfinite(fin.r) || !std::isfinite(fin.s))
      return fail(TE_ERR_NUMERIC, "non-finite residuals (r=%g, s=%g)", fin.r, fin.s);
  }
  return TE_OK;
}

te_status te_kernel_times(te_ctx *c, const te_options *opt, void *hip_stream, int32_t iters, double *ms_out) {
  if (!c || !ms_out) return fail(TE_ERR_INVALID, "null handle or output");
  if (iters < 1 || iters > 4096) return fail(TE_ERR_INVALID, "iters must be in 1..4096");
  te_options o;
  if (opt) o = *opt; else te_default_options(&o);
  o.fixed_iters = iters;
  te_status s = check_options(&o);
  if (s != TE_OK) return s;
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  s = select_graph_shape(c, o);
  if (s != TE_OK) return s;
  s = stage_params(&c->d_params, c->h_params, c->params_ev, &c->d_sched, &c->sched_cap, &o, stream);
  if (s != TE_OK) return s;
  std::vector<hipEvent_t> ev(4 * (size_t)iters, nullptr);
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto &f : ev)
        if (f) (void)hipEventDestroy(f);
      return fail(TE_ERR_DEVICE, "event creation failed");
    }
  c->state_scale = 0.0;  // this run overwrites the state a warm restart would continue from
  c->trace_engine = 0;   // and the control record a trace is read with
  hipError_t err = launch_init(c->prob, c->st, c->d_params, nullptr, 1.0 / c->scale, stream);
  for (int k = 0; k < iters && err == hipSuccess; ++k) {
    err = launch_demand_timed(c->prob, c->st, c->d_params, k & 1, stream, ev[4 * k], ev[4 * k + 1]);
    if (err == hipSuccess)
      err = launch_link_timed(c->prob, c->st, c->d_params, k & 1, stream, ev[4 * k + 2], ev[4 * k + 3]);
  }
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  double sd = 0.0, sl = 0.0;
  for (int k = 0; k < iters && err == hipSuccess; ++k) {
    float a = 0.f, b = 0.f;
    err = hipEventElapsedTime(&a, ev[4 * k], ev[4 * k + 1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&b, ev[4 * k + 2], ev[4 * k + 3]);
    sd += a;
    sl += b;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(TE_ERR_DEVICE, "kernel timing: %s", hipGetErrorString(err));
  ms_out[0] = sd / iters;
  ms_out[1] = sl / iters;
  return TE_OK;
}

te_status te_project(te_ctx *c, void *hip_stream, float *x_out_dev, float *S_out_dev) {
  if (!c || !x_out_dev) return fail(TE_ERR_INVALID, "null handle or output");
  if (c->state_scale <= 0.0) return fail(TE_ERR_STATE, "no graph-engine state on this handle");
  if (c->state_scale != c->scale)
    return fail(TE_ERR_STATE, "te_update changed the unit scale since the last solve (continue with warm = 1 first)");
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  HIPCHK(launch_project(c->prob, c->st, c->pb, x_out_dev, S_out_dev, c->scale, 1, stream));
  return TE_OK;
}

// The projection's working arrays (ProjBuf) carved from a scratch region at `base`, each part
// 256-byte aligned; returns the bytes used.
size_t carve_projbuf(void *base, int32_t P, int32_t D, int32_t E, ProjBuf *b) {
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t at = off;
    off += (n + 255) & ~size_t(255);
    return base ? static_cast<unsigned char *>(base) + at : nullptr;
  };
  ProjBuf r{};
  r.xd = reinterpret_cast<double *>(take(sizeof(double) * (size_t)P));
  r.S = reinterpret_cast<double *>(take(sizeof(double) * (size_t)D));
  r.L = reinterpret_cast<double *>(take(sizeof(double) * (size_t)E));
  r.Cp = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)P));
  r.lsc = reinterpret_cast<float *>(take(sizeof(float) * (size_t)P));
  r.trim = reinterpret_cast<uint64_t *>(take(sizeof(uint64_t) * (size_t)P));
  if (b) *b = r;
  return off;
}

te_status te_get_state(te_ctx *c, void *hip_stream, double *x_out_dev, double *S_out_dev, double *w_out_dev) {
  if (!c || !x_out_dev) return fail(TE_ERR_INVALID, "null handle or output");
  if (c->state_scale <= 0.0) return fail(TE_ERR_STATE, "no graph-engine state on this handle");
  if (c->state_scale != c->scale)
    return fail(TE_ERR_STATE, "te_update changed the unit scale since the last solve (continue with warm = 1 first)");
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  HIPCHK(launch_get_state(c->prob, c->st, c->scale, x_out_dev, S_out_dev, stream));
  if (w_out_dev)
    HIPCHK(hipMemcpyAsync(w_out_dev, c->st.w, sizeof(double) * c->E, hipMemcpyDeviceToDevice, stream));
  return TE_OK;
}

te_status te_project_rates(te_ctx *c, void *hip_stream, const float *x_in_dev, double alpha, float *x_out_dev,
                           float *S_out_dev) {
  if (!c || !x_in_dev || !x_out_dev) return fail(TE_ERR_INVALID, "null handle or buffer");
  if (!std::isfinite(alpha) || alpha < 0.0) return fail(TE_ERR_INVALID, "alpha must be finite and >= 0");
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  HIPCHK(launch_project_rates(c->prob, c->pb, x_in_dev, alpha, x_out_dev, S_out_dev, c->scale, stream));
  return TE_OK;
}

te_status te_trace(te_ctx *c, void *hip_stream, int32_t cap, double *out, int32_t *n_out) {
  if (!c || !out || !n_out || cap < 0) return fail(TE_ERR_INVALID, "null handle or buffer, or cap < 0");
  *n_out = 0;
  if (!c->trace_engine) return fail(TE_ERR_STATE, "the handle's last solve ran without trace = 1 or record = 1");
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  HIPCHK(hipStreamSynchronize(stream));
  int32_t k = 0;
  if (c->trace_engine == TE_ENGINE_BLOCK) {
    BatchOut bo;
    HIPCHK(hipMemcpy(&bo, c->d_bout, sizeof(bo), hipMemcpyDeviceToHost));
    k = bo.iters;
  } else {
    Ctrl fin;
    HIPCHK(hipMemcpy(&fin, c->st.ctrl + 2, sizeof(Ctrl), hipMemcpyDeviceToHost));
    k = fin.k;
  }
  const int32_t n = std::min(std::min(k, c->trace_src_cap), cap);
  for (int row = 0; row < 4 && n > 0; ++row)
    HIPCHK(hipMemcpy(out + (size_t)row * cap, c->trace_src + (size_t)row * c->trace_src_cap, sizeof(double) * n,
                     hipMemcpyDeviceToHost));
  *n_out = n;
  return TE_OK;
}

te_status te_project_rates_static(te_ctx *c, void *hip_stream, const float *x_in_dev, double alpha,
                                  float *x_out_dev, float *S_out_dev) {
  if (!c || !x_in_dev || !x_out_dev) return fail(TE_ERR_INVALID, "null handle or buffer");
  if (!std::isfinite(alpha) || alpha < 0.0) return fail(TE_ERR_INVALID, "alpha must be finite and >= 0");
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  void *base = nullptr;
  size_t cap = 0;
  HIPCHK(static_scratch(&base, &cap));
  const size_t need = carve_projbuf(nullptr, c->P, c->D, c->E, nullptr);
  if (need > cap)
    return fail(TE_ERR_INVALID, "te_project_rates_static: the instance needs %zu bytes of scratch, the static "
                                "scratch holds %zu (24 P + 8 D + 8 E bytes, rounded per array)", need, cap);
  ProjBuf b;
  carve_projbuf(base, c->P, c->D, c->E, &b);
  HIPCHK(launch_project_rates(c->prob, b, x_in_dev, alpha, x_out_dev, S_out_dev, c->scale, stream));
  return TE_OK;
}

te_status te_grad(te_ctx *c, void *hip_stream, const float *dS_dev, double *dC_dev, double *dD_dev) {
  if (!c || !dS_dev || !dC_dev || !dD_dev) return fail(TE_ERR_INVALID, "null handle or buffer");
  if (c->rec_K <= 0) return fail(TE_ERR_STATE, "no recorded solve on this handle (te_solve with record = 1)");
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(c->device);
  HIPCHK(dscope.err);
  const int K = c->rec_K, ck = c->rec_ck;
  const int nck = (K + ck - 1) / ck;
  // the recorded schedule on the host (beta_k, alpha_k, rescale rho_k)
  std::vector<double> lb(K), la(K);
  HIPCHK(hipMemcpyAsync(lb.data(), c->d_log, sizeof(double) * K, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(la.data(), c->d_log + c->log_cap, sizeof(double) * K, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  // buffers (kept on the handle); the checkpoints were taken by the recorded solve
  if ((int)c->ckpt.size() < nck) return fail(TE_ERR_STATE, "checkpoints of the recorded solve are missing");
  while ((int)c->seg.size() < ck + 1) {
    FwdState f{};
    if (alloc_fwd(f, c) != hipSuccess) {
      free_fwd(f);
      return fail(TE_ERR_OOM, "segment allocation failed");
    }
    c->seg.push_back(f);
  }
  if (!c->adj_ready) {
    AdjState &a = c->adj;
    bool ok = dalloc(&a.xb, c->P) == hipSuccess && dalloc(&a.unb, c->P) == hipSuccess &&
              dalloc(&a.udb, c->D) == hipSuccess && dalloc(&a.gb, c->E) == hipSuccess &&
              dalloc(&a.qb, c->E) == hipSuccess && dalloc(&a.ab, c->P) == hipSuccess;
    if (!ok) return fail(TE_ERR_OOM, "adjoint allocation failed");
    c->adj_ready = 1;
  }
  AdjState a = c->adj;
  a.Cb = dC_dev;
  a.Db = dD_dev;
  // replay parameters: the recorded schedule, fixed iteration count
  te_options o;
  te_default_options(&o);
  o.fixed_iters = K;
  o.sched_beta = lb.data();
  o.sched_alpha = la.data();
  o.sched_len = K;
  te_status s = stage_params(&c->d_params, c->h_params, c->params_ev, &c->d_sched, &c->sched_cap, &o, stream);
  if (s != TE_OK) return s;
  HIPCHK(hipStreamSynchronize(stream));  // the host schedule arrays are local to this call
  c->state_scale = 0.0;  // the segment recomputation overwrites the state a warm restart would continue from
  c->trace_engine = 0;   // and the control record a trace is read with
  // reverse, segment by segment: restore the segment's checkpoint, recompute its iterations with
  // the recorded schedule keeping every state, then run the adjoint iterations backwards
  HIPCHK(launch_adj_seed(c->prob, a, dS_dev, stream));
  for (int sgi = nck - 1; sgi >= 0; --sgi) {
    const int k0 = sgi * ck, k1 = std::min(K, k0 + ck);
    HIPCHK(copy_fwd(c->seg[0], c->ckpt[sgi], c, stream));
    HIPCHK(hipMemcpyAsync(c->st.ctrl + ((k0 + 1) & 1), c->ckpt_ctrl[sgi], sizeof(Ctrl), hipMemcpyDeviceToDevice,
                          stream));
    for (int k = k0; k < k1; ++k) {  // iteration k reads state k - k0 and writes state k - k0 + 1
      State sk = c->st;
      const FwdState &fi = c->seg[k - k0], &fo = c->seg[k - k0 + 1];
      sk.x = fi.x;
      sk.uneg = fi.uneg;
      sk.udem = fi.udem;
      sk.S = fi.S;
      sk.gq = fi.gq;
      sk.xo = fo.x;
      sk.unego = fo.uneg;
      sk.udemo = fo.udem;
      sk.So = fo.S;
      sk.gqo = fo.gq;
      HIPCHK(launch_iteration(c->prob, sk, c->d_params, k & 1, stream));
    }
    for (int k = k1 - 1; k >= k0; --k) {
      const double rho = k > 0 ? lb[k - 1] / lb[k] : 1.0;
      HIPCHK(launch_adj_iteration(c->prob, c->nB_csc, c->seg[k - k0], c->seg[k - k0 + 1], a, lb[k],
                                  la[k], rho, stream));
    }
  }
  if (!c->rec_warm) HIPCHK(launch_adj_x0(c->prob, a, stream));
  return TE_OK;
}

void te_destroy(te_ctx *c) {
  if (!c) return;
  DeviceScope dscope(c->device);
  if (c->chunk) (void)hipGraphExecDestroy(c->chunk);
  if (c->rec_chunk) (void)hipGraphExecDestroy(c->rec_chunk);
  if (c->trace_chunk) (void)hipGraphExecDestroy(c->trace_chunk);
  for (auto &f : c->ckpt) free_fwd(f);
  for (auto &f : c->seg) free_fwd(f);
  for (Ctrl *p : c->ckpt_ctrl)
    if (p) (void)hipFree(p);
  {
    void *ab[] = {c->adj.xb, c->adj.unb, c->adj.udb, c->adj.gb, c->adj.qb, c->adj.ab, c->d_log};
    for (void *p : ab)
      if (p) (void)hipFree(p);
  }
  free_fwd(c->work);
  void *bufs[] = {c->d_i32, c->d_Dn, c->d_Cn, c->d_trace, c->st.partL, c->st.w, c->st.dx2, c->st.ctrl,
                  c->st.partA, c->st.partB, c->pb.xd, c->pb.S, c->pb.L, c->pb.Cp, c->pb.lsc, c->pb.trim,
                  c->d_params, c->d_desc, c->d_bout, c->d_sched, c->d_wtab, c->d_hops, c->d_hops2, c->d_dovf, c->d_lent, c->d_lgrp, c->d_lchk};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (c->h_params) (void)hipHostFree(c->h_params);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->params_ev) (void)hipEventDestroy(c->params_ev);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->pe)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

// ----------------------------------------------------------------------------------------------
// batches
// ----------------------------------------------------------------------------------------------
te_status te_create_batch(int32_t n, te_ctx *const *inst, te_batch **out) {
  if (!out || !inst || n <= 0) return fail(TE_ERR_INVALID, "invalid batch arguments");
  *out = nullptr;
  const int dev = inst[0]->device;
  te_batch *b = new (std::nothrow) te_batch();
  if (!b) return fail(TE_ERR_OOM, "host allocation");
  b->device = dev;
  b->n = n;
  std::vector<int32_t> pool;
  std::vector<double> Dn;
  std::vector<double> Cn;
  int64_t offE = 0, offP = 0, offD = 0;
  for (int32_t k = 0; k < n; ++k) {
    const te_ctx *c = inst[k];
    if (!c || c->device != dev) {
      delete b;
      return fail(TE_ERR_INVALID, "batch instance %d is null or on another device", k);
    }
    b->members.push_back(inst[k]);
    if (c->lds_bytes > kMaxBlockLds) b->all_fit = false;
    BatchDesc d{};
    d.E = c->E;
    d.P = c->P;
    d.D = c->D;
    d.nnz = c->nnz;
    d.G = c->G;
    d.logG = c->logG;
    d.off_pptr = (int64_t)pool.size();
    pool.insert(pool.end(), c->pptr.begin(), c->pptr.end());
    d.off_plinks = (int64_t)pool.size();
    pool.insert(pool.end(), c->plinks.begin(), c->plinks.end());
    d.off_dptr = (int64_t)pool.size();
    pool.insert(pool.end(), c->dptr.begin(), c->dptr.end());
    d.off_lptr = (int64_t)pool.size();
    pool.insert(pool.end(), c->lptr.begin(), c->lptr.end());
    d.off_lpf = (int64_t)pool.size();
    pool.insert(pool.end(), c->lpf.begin(), c->lpf.end());
    d.off_nzl = (int64_t)pool.size();
    pool.insert(pool.end(), c->nzlink.begin(), c->nzlink.end());
    d.nzl = (int32_t)c->nzlink.size();
    d.off_E = offE;
    d.off_P = offP;
    d.off_D = offD;
    d.scale = c->scale;
    Dn.insert(Dn.end(), c->Dn.begin(), c->Dn.end());
    Cn.insert(Cn.end(), c->Cn.begin(), c->Cn.end());
    offE += c->E;
    offP += c->P;
    offD += c->D;
    if (c->lds_bytes <= kMaxBlockLds) b->lds_bytes = std::max(b->lds_bytes, c->lds_bytes);
    b->desc.push_back(d);
  }
  b->totP = offP;
  b->totD = offD;
  auto bail = [&](te_status s) {
    te_destroy_batch(b);
    return s;
  };
  DeviceScope dscope(dev);
  if (dscope.err != hipSuccess) return bail(fail(TE_ERR_DEVICE, "hipSetDevice failed"));
  bool ok = dalloc(&b->d_desc, n) == hipSuccess && dalloc(&b->d_out, n) == hipSuccess &&
            dalloc(&b->d_i32, pool.size()) == hipSuccess && dalloc(&b->d_Dn, Dn.size()) == hipSuccess &&
            dalloc(&b->d_Cn, Cn.size()) == hipSuccess && dalloc(&b->d_params, 1) == hipSuccess;
  if (!ok) return bail(fail(TE_ERR_OOM, "device allocation failed"));
  if (hipHostMalloc((void **)&b->h_params, sizeof(Params)) != hipSuccess)
    return bail(fail(TE_ERR_OOM, "pinned host allocation failed"));
  if (hipEventCreate(&b->params_ev) != hipSuccess || hipEventCreate(&b->ev0) != hipSuccess ||
      hipEventCreate(&b->ev1) != hipSuccess)
    return bail(fail(TE_ERR_DEVICE, "event creation failed"));
  if (hipMemcpy(b->d_desc, b->desc.data(), sizeof(BatchDesc) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_i32, pool.data(), sizeof(int32_t) * pool.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_Dn, Dn.data(), sizeof(double) * Dn.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_Cn, Cn.data(), sizeof(double) * Cn.size(), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(TE_ERR_DEVICE, "batch upload failed"));
  *out = b;
  return TE_OK;
}

// The disjoint union of a batch's instances as one handle: link, path and demand ids offset, every
// instance's capacities and demands in its own normalised units (so the union's unit scale is 1 and
// each instance iterates exactly as alone under the union's (beta, alpha) schedule), outputs scaled
// back per demand.
te_status build_union(te_batch *b) {
  std::vector<double> cap, dem, dsc;
  std::vector<int64_t> pptr(1, 0);
  std::vector<int32_t> plinks, dptr(1, 0);
  int32_t offE = 0, offP = 0;
  for (const te_ctx *c : b->members) {
    cap.insert(cap.end(), c->Cn.begin(), c->Cn.end());
    dem.insert(dem.end(), c->Dn.begin(), c->Dn.end());
    dsc.insert(dsc.end(), (size_t)c->D, c->scale);
    for (int32_t r = 0; r < c->P; ++r) pptr.push_back(pptr.back() + (c->pptr[r + 1] - c->pptr[r]));
    for (int32_t i = 0; i < c->nnz; ++i) plinks.push_back(c->plinks[i] + offE);
    for (int32_t k = 1; k <= c->D; ++k) dptr.push_back(c->dptr[k] + offP);
    offE += c->E;
    offP += c->P;
  }
  te_ctx *u = nullptr;
  te_status s = te_create(offE, cap.data(), offP, pptr.data(), plinks.data(), (int32_t)dem.size(), dptr.data(),
                          dem.data(), b->device, &u);
  if (s != TE_OK) return s;
  if (dalloc(&b->d_dscale, dsc.size()) != hipSuccess ||
      hipMemcpy(b->d_dscale, dsc.data(), sizeof(double) * dsc.size(), hipMemcpyHostToDevice) != hipSuccess) {
    te_destroy(u);
    return fail(TE_ERR_OOM, "union scale upload failed");
  }
  u->prob.dscale = b->d_dscale;  // before any capture: the captured launches hold the Prob
  b->uni = u;
  return TE_OK;
}

te_status te_solve_batch(te_batch *b, const te_options *opt, void *hip_stream, float *x_out_dev, float *S_out_dev,
                         te_stats *stats) {
  if (!b || !x_out_dev) return fail(TE_ERR_INVALID, "null batch or output");
  te_options o;
  if (opt) o = *opt; else te_default_options(&o);
  te_status s = check_options(&o);
  if (s != TE_OK) return s;
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceScope dscope(b->device);
  HIPCHK(dscope.err);
  if (o.warm || o.record || o.trace) return fail(TE_ERR_INVALID, "batches take no warm, record or trace");
  const bool graph = o.engine == TE_ENGINE_GRAPH || o.per_link || (o.engine == TE_ENGINE_AUTO && !b->all_fit);
  if (!graph && !b->all_fit)
    return fail(TE_ERR_INVALID, "an instance of the batch does not fit one workgroup's LDS (use the graph engine)");
  if (graph) {
    if (!b->uni) {
      s = build_union(b);
      if (s != TE_OK) return s;
    }
    te_options g = o;
    g.engine = TE_ENGINE_GRAPH;
    te_stats st{};
    s = te_solve(b->uni, &g, hip_stream, nullptr, x_out_dev, S_out_dev, stats ? &st : nullptr);
    if (s != TE_OK) return s;
    if (stats)
      for (int32_t k = 0; k < b->n; ++k) stats[k] = st;
    return TE_OK;
  }
  Pools pools{b->d_i32, b->d_Dn, b->d_Cn, nullptr, nullptr, 0};
  int threads = o.block_threads, ppl = o.paths_per_lane;
  if (threads == 0 || ppl == 0) {
    const std::pair<int, int> key(threads, ppl);
    auto it = b->tuned.find(key);
    if (it == b->tuned.end()) {
      std::pair<int, int> pick;
      s = tune_block_shape(threads, ppl, o.fixed_iters, stream, b->ev0, b->ev1,
                           [&](int th, int pl, int iters) -> te_status {
                             te_options t;
                             te_default_options(&t);
                             t.fixed_iters = iters;
                             t.project = 0;
                             te_status st = stage_params(&b->d_params, b->h_params, b->params_ev, &b->d_sched,
                                                         &b->sched_cap, &t, stream);
                             if (st != TE_OK) return st;
                             HIPCHK(launch_block_solve(b->d_desc, b->n, pools, b->d_params, 0, x_out_dev, S_out_dev,
                                                       b->d_out, b->lds_bytes, th, pl, stream));
                             return TE_OK;
                           },
                           &pick);
      if (s != TE_OK) return s;
      it = b->tuned.emplace(key, pick).first;
    }
    threads = it->second.first;
    ppl = it->second.second;
  }
  s = stage_params(&b->d_params, b->h_params, b->params_ev, &b->d_sched, &b->sched_cap, &o, stream);
  if (s != TE_OK) return s;
  HIPCHK(hipEventRecord(b->ev0, stream));
  HIPCHK(launch_block_solve(b->d_desc, b->n, pools, b->d_params, o.project, x_out_dev, S_out_dev, b->d_out,
                            b->lds_bytes, threads, ppl, stream));
  HIPCHK(hipEventRecord(b->ev1, stream));
  if (stats) {
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<BatchOut> outs(b->n);
    HIPCHK(hipMemcpy(outs.data(), b->d_out, sizeof(BatchOut) * b->n, hipMemcpyDeviceToHost));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    for (int32_t k = 0; k < b->n; ++k) {
      Ctrl fin{};
      fin.k = outs[k].iters;
      fin.flags = outs[k].flags;
      fin.stop_iter = outs[k].stop_iter;
      fin.alpha = outs[k].alpha;
      fin.beta = outs[k].beta;
      fin.r = outs[k].r;
      fin.s = outs[k].s;
      fin.cap_viol = outs[k].cap_viol;
      fin.dem_viol = outs[k].dem_viol;
      fill_stats(&stats[k], fin, TE_ENGINE_BLOCK, ms, threads, ppl);
    }
  }
  return TE_OK;
}

void te_destroy_batch(te_batch *b) {
  if (!b) return;
  if (b->uni) te_destroy(b->uni);
  DeviceScope dscope(b->device);
  void *bufs[] = {b->d_desc, b->d_out, b->d_i32, b->d_Dn, b->d_Cn, b->d_params, b->d_sched, b->d_dscale};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  if (b->h_params) (void)hipHostFree(b->h_params);
  if (b->params_ev) (void)hipEventDestroy(b->params_ev);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
}

}  // extern "C"
