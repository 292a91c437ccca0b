/*
 * te.h -- C ABI of the GATE traffic-engineering solver for AMD Instinct MI355X (gfx950).
 *
 * The library solves the path-based multicommodity-flow TE problem of the
 * paper "GATE: GPU-Accelerated Traffic Engineering for the WAN" (section 3.1,
 * "TE Formulation"):
 *
 *     maximise   sum_c U_alpha(S_c),      S_c = sum_{r in P_c} x_r,
 *     subject to S_c <= D_c               (demand constraint)
 *                sum_{r : e in r} x_r <= C_e   (capacity constraint)
 *                x_r >= 0                 (non-negativity)
 *
 * with the alpha-fair utility U_alpha(b) = (b^(1-alpha) - 1)/(1 - alpha)
 * (alpha = 0: max-flow, 1: proportional fairness, infinity: max-min
 * fairness), by the paper's iterative decomposition (section 3.3, Algorithm 1):
 * per iteration a gather of per-link prices along every path, a per-demand
 * update of its split (sum equation of appendix B.2 solved by Newton-bisection,
 * rate update of section 3.3), a segmented sum of path rates into link loads
 * and a per-link capacity/dual update, with the residual-balancing penalty of
 * section 3.4, alpha-increments (section 3.4) and the feasibility projection
 * of Algorithm 2 (section 3.5) at the end.
 *
 * Conventions
 *  - Every function returns te_status; nothing is thrown and nothing aborts.
 *    On a non-OK status te_last_error() gives a message (thread-local).
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *  - "_dev" pointers are device pointers on the handle's device (for example
 *    torch tensors); the library never frees them.  Work on them is ordered on
 *    the hip_stream argument (a hipStream_t, NULL = legacy default stream).
 *  - A handle may be used by one host thread at a time; separate handles are
 *    independent.  A handle owns its device buffers until te_destroy.
 *  - Units: the library divides capacities and demands by s = the largest
 *    capacity of a link used by some path, iterates in those units, and
 *    returns rates and sums in the caller's units.
 *  - Admissible instance (appendix C, Part I(b): every commodity has a path and
 *    a positive demand, every used link a positive capacity): at least one
 *    demand (an instance without commodities has nothing to solve), at most
 *    524,288 links used by paths (the link kernel's work split), path_ptr
 *    non-decreasing from 0, no empty path, link ids in range, no link twice in
 *    one path, every demand with 1..64 paths, demand > 0 and finite, capacity
 *    finite everywhere and > 0 on every used link.  Anything else returns
 *    TE_ERR_INVALID.
 */
#ifndef TE_GATE_H
#define TE_GATE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct te_ctx te_ctx;
typedef struct te_batch te_batch;

typedef enum {
  TE_OK = 0,
  TE_ERR_INVALID = 1, /* argument or instance not admissible */
  TE_ERR_OOM = 2,     /* device or host allocation failed */
  TE_ERR_DEVICE = 3,  /* HIP runtime error (no device, launch failure, ...) */
  TE_ERR_NUMERIC = 4, /* non-finite value reached the state */
  TE_ERR_STATE = 5    /* call not valid in the handle's state (e.g. te_grad without a recorded solve) */
} te_status;

/* te_stats.flags */
enum {
  TE_CONVERGED = 1,      /* residuals below gamma at the target alpha, or stagnation across an alpha step */
  TE_HIT_MAX_ITERS = 2,  /* adaptive mode stopped at max_iters */
  TE_HIT_ALPHA_MAX = 4,  /* an alpha step would have exceeded alpha_max */
  TE_HIT_BETA_BOUND = 8  /* the residual-balancing rule hit beta_min or beta_max */
};

/* te_options.engine */
enum {
  TE_ENGINE_AUTO = 0,  /* workgroup engine when the instance fits one workgroup's LDS, else graph engine */
  TE_ENGINE_GRAPH = 1, /* device-wide kernels per iteration, replayed as a captured HIP graph */
  TE_ENGINE_BLOCK = 2  /* whole solve inside one workgroup, state resident in LDS */
};

/* te_options.link_sums */
enum {
  TE_LINK_SUMS_AUTO = 0,
  TE_LINK_SUMS_PRIVATE = 1, /* every demand workgroup adds its paths' rates into its own copy of the link
                               loads (LDS), rows reduced per link in a second kernel; the workgroup
                               keeps a chunk of its paths' new rates in LDS and adds them by
                               segmented sums over the chunk's own link -> path list (built at
                               te_create or on the switch), or, where one pass of rates does not
                               fit beside the loads, as TE_LINK_SUMS_PRIVATE_ATOMIC */
  TE_LINK_SUMS_CSC = 2,     /* segmented sums over the link -> path incidence list */
  TE_LINK_SUMS_PRIVATE_ATOMIC = 3 /* privatised as TE_LINK_SUMS_PRIVATE, one LDS atomic addition per
                                     path-link incidence */
};

typedef struct {
  double alpha_target; /* fairness target: INFINITY = max-min (default), 0 = max-flow, 1 = proportional */
  double gamma;        /* residual threshold of the stop test (section 3.4); default 1e-3 */
  double beta0;        /* initial penalty (Algorithm 1 optional input); default 1 */
  double A, C;         /* residual-balancing constants (section 3.6: A = 10, C = 2) */
  double beta_min;     /* bounds on beta (absolute); default 1e-3 * beta0 and 1e3 * beta0 */
  double beta_max;
  int32_t max_iters;   /* adaptive mode: stop after this many iterations (flag TE_HIT_MAX_ITERS) */
  int32_t alpha_max;   /* largest alpha an increment may reach (flag TE_HIT_ALPHA_MAX); default 64 */
  int32_t fixed_iters; /* > 0: run exactly this many iterations, no stop test; alpha and beta still adapt */
  int32_t adapt_beta;  /* 0: keep beta = beta0 */
  int32_t beta_every;  /* the residual-balancing rule may act only after every beta_every-th iteration;
                          default 1 (every iteration, section 3.4).  After the n-th reversal of beta's
                          direction the rule rests for the next 2^n - 1 iterations (2^20 at most), so
                          it cannot cycle; the per-link rule acts on the same iterations */
  int32_t project;     /* 1: run the feasibility projection of Algorithm 2 before returning (default) */
  int32_t engine;      /* TE_ENGINE_* */
  int32_t record;      /* 1: keep the (beta, alpha) schedule and checkpoints for te_grad */
  int32_t ckpt_every;  /* te_grad checkpoint spacing in iterations; default 16 */
  int32_t block_threads; /* workgroup engine: threads per workgroup, 256, 512 or 1024; 0 (default):
                            tuned on the handle's first such solve (see paths_per_lane) */
  int32_t paths_per_lane; /* paths of a demand held by one lane in the demand step, 1, 2, 4 or 8 (a
                            demand with G path slots gets max(1, G / paths_per_lane) lanes); 0
                            (default): graph engine 1, or 2 for instances with at least 2^20 lane
                            slots (demands x G: there the kernel is bound by issue and bandwidth,
                            not latency); workgroup engine: the members of (block_threads,
                            paths_per_lane) left at 0 are tuned on the handle's (or batch's) first
                            such solve (every candidate timed over min(max(fixed_iters, 256), 512)
                            iterations; up to 12 short launches) and kept by the handle.
                            A new value for the graph engine recaptures its iteration graphs
                            (after a device-wide synchronisation). */
  int32_t warm;        /* 1: continue from the state the handle's last graph-engine solve left (rates,
                          every dual, beta and alpha; alpha capped at alpha_target) instead of
                          initialising, e.g. after te_update; the iteration count restarts at 0.
                          Uses the graph engine; TE_ERR_STATE if there is no such state (none yet,
                          or te_grad / te_kernel_times ran since).  If te_update changed the unit
                          scale, the state is converted to the new units. */
  /* Optional replay of a (beta_k, alpha_k) schedule, host arrays of sched_len entries: iteration k
   * uses beta = sched_beta[k], alpha = sched_alpha[k] (the last entry repeats), no adaptation. */
  const double *sched_beta;
  const double *sched_alpha;
  int32_t sched_len;
  int32_t trace;       /* 1: log, for every iteration k, the beta_k and alpha_k it used and its residuals
                          r_k, s_k (section 3.4), read back with te_trace (a recorded solve logs them
                          anyway); te_solve only, either engine */
  int32_t link_sums;   /* graph engine, how the link loads sum_{r on e} x_r are formed: TE_LINK_SUMS_*;
                          0 (default): privatised (TE_LINK_SUMS_PRIVATE) for instances with at least 2^20
                          lane slots (demands x G) and at most 19,456 links, else CSC.
                          A change recaptures the iteration graphs (after a device-wide synchronisation). */
  int32_t per_link;    /* 1: per-link penalties (the conclusion's learning rates adaptive across parts of
                          the topology, read as: link e's consensus and capacity constraints carry the
                          penalty beta * w_e, and the residual-balancing rule of section 3.4, on link e's
                          own residuals and the same cadence, moves w_e by C within [w_min, w_max],
                          dividing link e's scaled duals by the same factor).  Graph engine with CSC link
                          sums; not with record.  Default 0 */
  double w_min, w_max; /* bounds on w_e; default 0.25 and 4 */
} te_options;

typedef struct {
  int32_t iters;       /* iterations run */
  int32_t flags;       /* TE_CONVERGED | ... */
  int32_t stop_iter;   /* first iteration at which the stop test passed, -1 if never */
  int32_t engine;      /* engine that ran */
  int32_t block_threads; /* workgroup engine: threads per workgroup that ran (0 for the graph engine) */
  int32_t paths_per_lane; /* paths per lane of the demand step that ran (either engine) */
  double final_alpha;
  double beta;         /* final penalty */
  double r, s;         /* last primal and dual residuals (section 3.4) */
  double max_cap_viol_rel; /* max over links of (load - C)/C before projection */
  double max_dem_viol_rel; /* max over demands of (S - D)/D before projection */
  double ms;           /* device time of the solve (init to output), milliseconds */
} te_stats;

/* Fill *opt with the defaults listed above. */
void te_default_options(te_options *opt);

/*
 * Validate an instance on the host without touching any GPU; same rules as
 * te_create.  Returns TE_OK or TE_ERR_INVALID (message in te_last_error()).
 *   capacity        [n_links]        link capacities
 *   path_ptr        [n_paths + 1]    CSR row pointer of the path -> link incidence (int64)
 *   path_links      [path_ptr[n_paths]] link ids of each path, in path order
 *   demand_path_ptr [n_demands + 1]  the paths of demand c are demand_path_ptr[c] .. [c+1]-1
 *   demand          [n_demands]      requested demand D_c
 */
te_status te_validate(int32_t n_links, const double *capacity, int32_t n_paths, const int64_t *path_ptr,
                      const int32_t *path_links, int32_t n_demands, const int32_t *demand_path_ptr,
                      const double *demand);

/*
 * Build a solver handle on HIP device hip_device: validates (as te_validate),
 * normalises units, builds the path -> link CSR and link -> path CSC layouts
 * and copies them to the device (synchronously).  Host arrays as in
 * te_validate.  *out receives the handle (NULL on error).
 */
te_status te_create(int32_t n_links, const double *capacity, int32_t n_paths, const int64_t *path_ptr,
                    const int32_t *path_links, int32_t n_demands, const int32_t *demand_path_ptr,
                    const double *demand, int32_t hip_device, te_ctx **out);

/* Replace capacities and/or demands (host arrays, nullable) of an existing handle; same validity rules.
 * A warm start from the previous allocation is then te_solve with x0_dev. */
te_status te_update(te_ctx *ctx, const double *capacity, const double *demand);

/*
 * Run Algorithm 1 (and Algorithm 2 if opt->project) on the handle's instance.
 *   opt        options (NULL = defaults)
 *   hip_stream hipStream_t to order the work on
 *   x0_dev     nullable [n_paths] float warm start in caller units (default D_c / |P_c|)
 *   x_out_dev  [n_paths] float: path rates, caller units
 *   S_out_dev  nullable [n_demands] float: per-demand sums of x_out
 *   stats      nullable; when given the call synchronises the stream and fills it
 */
te_status te_solve(te_ctx *ctx, const te_options *opt, void *hip_stream, const float *x0_dev, float *x_out_dev,
                   float *S_out_dev, te_stats *stats);

/*
 * Feasible allocation from the state the handle's last graph-engine solve left: Algorithm 2
 * (section 3.5) applied to its current rates at its final alpha, without iterating.  With
 * te_solve(project = 0) and warm = 1 this gives an allocation at any point of a long solve.
 *   x_out_dev [n_paths] float, S_out_dev nullable [n_demands] float: caller units.
 * TE_ERR_STATE if there is no such state (none yet, te_grad / te_kernel_times ran since, or
 * te_update changed the unit scale since: continue with warm = 1 first).
 */
te_status te_project(te_ctx *ctx, void *hip_stream, float *x_out_dev, float *S_out_dev);

/*
 * The FP64 iterate the handle's last graph-engine solve left, before any projection: its path rates
 * x_r and per-demand sums S_c = sum of the rates of c, in caller units.  This is what that solve's
 * projection started from, and the exact state a later warm = 1 solve continues from.
 *   x_out_dev [n_paths] double, S_out_dev nullable [n_demands] double,
 *   w_out_dev nullable [n_links] double: per-link penalty factors w_e (all 1 unless per_link)
 * TE_ERR_STATE as te_project.
 */
te_status te_get_state(te_ctx *ctx, void *hip_stream, double *x_out_dev, double *S_out_dev, double *w_out_dev);

/*
 * Algorithm 2 (section 3.5) applied to caller-supplied path rates under the handle's CURRENT
 * capacities and demands (those of te_create or the last te_update), with the trim order of the
 * given alpha.  This is how an allocation computed for an earlier network state is scored under a
 * later one: the drift-adjusted optimality of section 4.1 applies the rates found at T_0 to the
 * state at T_K (te_update to T_K, then this call), and the paths keep at most their T_0 rates.
 *   x_in_dev  [n_paths] float, caller units; read once at the start, so it may alias x_out_dev
 *   alpha     finite, >= 0: the alpha of the trim scores (the final alpha of the solve that
 *             produced x_in; any value for rates from elsewhere)
 *   x_out_dev [n_paths] float, S_out_dev nullable [n_demands] float: caller units, rounded
 *             toward zero so that the result stays feasible
 * Stream-ordered; uses the handle's projection buffers (not its solver state, so a warm restart
 * is unaffected).  TE_ERR_INVALID on a null buffer or a bad alpha.
 */
te_status te_project_rates(te_ctx *ctx, void *hip_stream, const float *x_in_dev, double alpha, float *x_out_dev,
                           float *S_out_dev);

/*
 * te_project_rates without allocating: for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * semantics and results as te_project_rates, but the projection's working arrays (24 P + 8 D + 8 E
 * bytes, each array rounded up to 256 bytes) come from a static device array of 32 MiB that every
 * GPU the library runs on holds until the process ends, not from the handle.  All calls on one GPU
 * share that array: calls that overlap on one GPU (on different streams or threads) race and must
 * be ordered by the caller.  Every array is rewritten before it is read, so nothing of an earlier
 * call's contents carries over.  Calls no hipMalloc/hipFree.
 * TE_ERR_INVALID if the instance needs more scratch than the array holds, or as te_project_rates.
 */
te_status te_project_rates_static(te_ctx *ctx, void *hip_stream, const float *x_in_dev, double alpha,
                                  float *x_out_dev, float *S_out_dev);

/*
 * Vector-Jacobian product through the last solve run with opt->record = 1 and
 * opt->fixed_iters = K: the unprojected sums S^(K) as a function of capacities
 * and demands, with the recorded (beta, alpha) schedule and the unit scale
 * held fixed.
 *   dS_dev  [n_demands] float cotangent on S^(K), caller units (ones: total throughput;
 *           1/S: sum of log-allocations)
 *   dC_dev  [n_links]   double gradient with respect to capacities (caller units)
 *   dD_dev  [n_demands] double gradient with respect to demands
 * Recomputes the forward iterations segment by segment from checkpoints taken every
 * opt->ckpt_every iterations.  TE_ERR_STATE if no recorded solve exists.
 */
te_status te_grad(te_ctx *ctx, void *hip_stream, const float *dS_dev, double *dC_dev, double *dD_dev);

/*
 * Batched solves: n instances (handles on the same device, used read-only) in one launch.
 *  - Workgroup engine (opt->engine BLOCK, or AUTO when every instance fits one workgroup's LDS):
 *    one workgroup per instance, each with its own beta / alpha / stop state.
 *  - Graph engine (opt->engine GRAPH, AUTO when some instance does not fit, or per_link): the
 *    instances' disjoint union as one instance (built on the first such solve), each instance in
 *    its own normalised units.  The union shares one beta / alpha schedule and one stop, driven by
 *    the union's residuals; as the instances share no link or demand, each one's iterates are
 *    exactly those of its own solve under that schedule, and its optimum (max-min or alpha-fair) is
 *    its own.  Every te_stats entry then holds the union's control.
 * BLOCK with an instance that does not fit returns TE_ERR_INVALID.  No warm, record or trace.
 */
te_status te_create_batch(int32_t n, te_ctx *const *instances, te_batch **out);

/*   x_out_dev  [sum of n_paths] float, instances concatenated in order
 *   S_out_dev  nullable [sum of n_demands] float
 *   stats      nullable [n] te_stats, synchronises the stream when given */
te_status te_solve_batch(te_batch *batch, const te_options *opt, void *hip_stream, float *x_out_dev,
                         float *S_out_dev, te_stats *stats);

/*
 * Device time of the graph engine's two per-iteration kernels (profiling aid): runs the solve of
 * opt with opt->fixed_iters = iters as individually launched kernels on hip_stream, each launch
 * carrying HIP events attached to its dispatch (start and end of its execution), synchronises, and
 * writes the mean duration in milliseconds of the demand kernel to ms_out[0] and of the link
 * kernel to ms_out[1].  The work is that of te_solve without the projection.  iters in 1..4096.
 */
te_status te_kernel_times(te_ctx *ctx, const te_options *opt, void *hip_stream, int32_t iters, double *ms_out);

void te_destroy(te_ctx *ctx);
void te_destroy_batch(te_batch *batch);

/* Sizes of a handle: n_links, n_paths, n_demands, nnz, max paths per demand, engine AUTO would pick,
 * workgroups of the graph engine's demand kernel and of its link kernel, the 16-bit slots per
 * path of the demand kernel's hop records (0: it reads the CSR path layout instead), the
 * generation of the recording te_grad would use (0: none; every recorded solve and every
 * te_update changes it, and te_update discards the recording), the graph engine's link sums in use
 * (TE_LINK_SUMS_*) and its privatised-sum workgroups (0 with CSC sums), and with TE_LINK_SUMS_PRIVATE
 * the passes per chunk of its link lists and their 16-bit entries (both 0 where the privatised sums
 * add one incidence at a time). The demand and link workgroups are those of the link sums in use. */
te_status te_info(const te_ctx *ctx, int64_t *sizes_out /* [14] */);

/*
 * Per-iteration trace of the handle's last te_solve, when it ran with opt->trace = 1 or
 * opt->record = 1: the control sequence of Algorithm 1 with the residual balancing of section 3.4.
 *   hip_stream the stream that solve ran on (synchronised here)
 *   cap        rows of out; out is a host array [4][cap]: out[k] = beta_k, out[cap + k] = alpha_k
 *              (penalty and fairness used in iteration k), out[2 cap + k] = r_k, out[3 cap + k] = s_k
 *              (dual and primal residual of iteration k, normalised units)
 *   n_out      iterations written: min(iterations run, cap)
 * TE_ERR_STATE if that solve ran without a trace, or te_grad / te_kernel_times ran since.
 */
te_status te_trace(te_ctx *ctx, void *hip_stream, int32_t cap, double *out, int32_t *n_out);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *te_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TE_GATE_H */
