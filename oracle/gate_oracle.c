/*
 * gate_oracle.c -- FP64 CPU oracle of GATE's iterative decomposition.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path; both sides only read the same
 * synthetic inputs.
 *
 * What it computes (paper: "GATE: GPU-Accelerated Traffic Engineering for
 * the WAN", section 3 "Design" and appendix B):
 *
 *   Problem (section 3.1, "TE Formulation"): path rates x_r >= 0 over
 *   precomputed paths, sum_{r in P_c} x_r <= D_c per commodity (demand
 *   constraint), sum_{r: e in r} x_r <= C_e per link (capacity constraint),
 *   maximise sum_c U_alpha(S_c) with S_c = sum_{r in P_c} x_r and the
 *   alpha-fair utility U_alpha(b) = (b^(1-alpha) - 1) / (1 - alpha).
 *
 *   Reformulation (section 3.2): one copy y_{e,r} of x_r per incidence,
 *   capacity written on y, consensus x_r = y_{e,r}; augmented Lagrangian
 *   in scaled-dual form with penalty beta and duals dual_dem (per commodity),
 *   dual_cap (per link), dual_neg (per path), dual_con (per incidence); the
 *   inequalities carry slack variables (appendix B.1).
 *
 *   One iteration (section 3.3, Algorithm 1) is read as the two-block ADMM
 *   sweep that the convergence proof (appendix C, Part I) invokes, each
 *   block minimised exactly:
 *     1. x-block, per commodity: the sum S_c is the unique root of a
 *        monotone scalar equation (appendix B.2, Newton-bisection); the
 *        rates follow in closed form (boxed rate-update equation of
 *        section 3.3, here with the slack hinges kept).
 *     2. y-block, per link: the rate suggestions jointly with slack_cap.
 *     3. dual updates exactly as printed in section 3.3 ("Dual and Slack
 *        Updates"), evaluated on the new x and y.
 *     4. residuals s = ||x^{k+1} - x^k||, r = ||dual^{k+1} - dual^k||
 *        (section 3.4, dual and primal residual).
 *     5. adaptive beta by residual balancing (section 3.4, A = 10, C = 2
 *        from section 3.6); scaled duals are divided by the same factor.
 *        READING: applied after every sweep, as the paper states, except
 *        that after the n-th reversal of beta's direction the rule rests for
 *        the next 2^n - 1 sweeps (on instances where it cycles).
 *     6. alpha-increments and the stagnation stop (section 3.4,
 *        Algorithm 1).
 *   After the loop, the feasibility projection of Algorithm 2 (section 3.5).
 *
 * Readings of points where the paper is silent or inconsistent are listed in
 * the design notes; each is marked READING below.
 *
 * Units: capacities and demands are divided by s = max capacity over links
 * used by some path; outputs are multiplied back by s.
 *
 * Parity pins for every function are in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops for later calls (n > 0), or just the current setting (n <= 0);
   returns the number the next parallel loop may use (1 when built without OpenMP).  Timing aid of
   the CPU baseline only: the arithmetic does not depend on it. */
int gate_oracle_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

#define GO_CONVERGED 1
#define GO_HIT_MAX_ITERS 2
#define GO_HIT_ALPHA_MAX 4
#define GO_HIT_BETA_BOUND 8
#define GO_NUMERIC 16

/* Optional warm state: the whole iterate an earlier solve left (Algorithm 1 takes x^0 and beta as
 * optional inputs; here every dual, the last sums and alpha come along, as when a solve is continued
 * after the network state changed).  Caller units: every array is divided by this solve's scale s,
 * i.e. the scaled duals, which have the units of rates, are converted like the rates.  All pointers
 * are required. */
typedef struct {
  const double *x;     /* [P] rates */
  const double *S;     /* [D] last sums (start of the root solve) */
  const double *y;     /* [nnz] rate suggestions, CSR incidence order */
  const double *ucon;  /* [nnz] consensus duals, CSR incidence order */
  const double *ucap;  /* [E] */
  const double *udem;  /* [D] */
  const double *uneg;  /* [P] */
  double beta;         /* penalty the duals are scaled for */
  double alpha;        /* fairness reached (capped at alpha_target) */
  const double *w;     /* nullable [E]: per-link penalty factors (per_link); the link duals are scaled
                          for beta * w_e */
  int32_t last_dir, n_rev, rule_rest; /* back-off of the balancing rule (go_stats) */
} go_warm;

typedef struct {
  double alpha_target; /* INFINITY = max-min fairness */
  double gamma;        /* residual threshold */
  double beta0;        /* initial penalty */
  double A, C;         /* residual-balancing constants */
  double beta_min, beta_max;
  int32_t max_iters;   /* safeguard in adaptive mode */
  int32_t alpha_max;   /* safeguard on alpha-increments */
  int32_t fixed_iters; /* > 0: run exactly this many sweeps, no stop */
  int32_t adapt_beta;  /* 0: keep beta fixed */
  int32_t project;     /* run Algorithm 2 at the end */
  int32_t collapsed;   /* 1: per-link (g, q) bookkeeping instead of per-incidence (y, dual_con) */
  const double *sched_beta;  /* nullable: replay beta_k per sweep */
  const double *sched_alpha; /* nullable: replay alpha_k per sweep */
  int32_t sched_len;
  int32_t root_max_steps;    /* Newton-bisection step cap (default 200) */
  int32_t dual_res_scaled;   /* 1: s = beta * ||x^{k+1} - x^k||, 0: as printed, without beta */
  int32_t beta_every;        /* rule cadence: only after every T-th sweep (1 = every sweep, READING) */
  const go_warm *warm;       /* nullable: continue from this state instead of initialising */
  int32_t per_link;          /* 1: per-link penalties beta * w_e, w_e adapted per link (READING) */
  double w_min, w_max;       /* bounds on w_e */
} go_options;

typedef struct {
  int32_t iters, flags, stop_iter;
  double final_alpha, beta, r, s;
  double max_cap_viol_rel, max_dem_viol_rel; /* before projection */
  double collapse_dev;                       /* max |dual_con_{e,r} - dual_cap_e| over all sweeps */
  double root_steps_mean;
  int32_t root_steps_max;
  /* back-off of the balancing rule at the end: direction of its last change of beta, reversals so
     far, sweeps it still rests */
  int32_t last_dir, n_rev, rule_rest;
} go_stats;

/* Optional state read-back (all nullable, normalised units). */
typedef struct {
  double *dual_dem; /* [D] */
  double *dual_cap; /* [E] */
  double *dual_neg; /* [P] */
  double *dual_con; /* [nnz], CSR incidence order */
  double *y;        /* [nnz], CSR incidence order */
  double *x_raw;    /* [P] unprojected x */
  double *S_raw;    /* [D] unprojected sums */
  double *trace;    /* [5 * n] rows (alpha, beta, r, s, flags-so-far) per sweep */
  int32_t trace_cap;
  double scale;     /* out: normalisation scale s */
  double *w;        /* [E] per-link penalty factors at the end (all 1 without per_link) */
} go_state;

/* ------------------------------------------------------------------------ */
/* x-block helpers (appendix B.2)                                            */
/* ------------------------------------------------------------------------ */

/* The commodity sub-problem, with the slacks minimised out, is
 *   min_x  -U_alpha(S)/beta + 1/2 [S - D + dual_dem]_+^2
 *          + sum_r 1/2 [dual_neg_r - x_r]_+^2
 *          + sum_r sum_{e in r} 1/2 (dual_con_{e,r} + x_r - y_{e,r})^2.
 * Setting the derivative in x_r to zero gives
 *   n_r x_r - [dual_neg_r - x_r]_+ = a_r - h(S),
 *   a_r = sum_{e in r} (y_{e,r} - dual_con_{e,r}),
 *   h(S) = [S - D + dual_dem]_+ - S^{-alpha} / beta,
 * whose left side is strictly increasing in x_r; xi_r below is its inverse.
 * Summing over the paths gives F(S) = sum_r xi_r(a_r - h(S)) - S = 0, with F
 * continuous and strictly decreasing: the root is unique. */
typedef struct {
  int np;
  const double *a;
  const double *n;     /* links per path: n_r, or with per-link penalties W_r = sum_{e in r} w_e */
  const double *uneg;  /* dual_neg per path */
  double D, udem, alpha, beta;
} commodity_t;

static double pow_neg_alpha(double S, double alpha) {
  if (alpha == 0.0) return 1.0;
  if (!(S > 0.0)) return INFINITY;
  return exp(-alpha * log(S));
}

static double h_of(const commodity_t *c, double S) {
  double t = S - c->D + c->udem;
  return (t > 0.0 ? t : 0.0) - pow_neg_alpha(S, c->alpha) / c->beta;
}

static double dh_of(const commodity_t *c, double S) {
  double t = S - c->D + c->udem;
  double d = t > 0.0 ? 1.0 : 0.0;
  if (c->alpha != 0.0) d += c->alpha * pow_neg_alpha(S, c->alpha + 1.0) / c->beta;
  return d;
}

static double xi(double b, double n, double uneg) {
  return (b >= n * uneg) ? b / n : (b + uneg) / (n + 1);
}

static double dxi(double b, double n, double uneg) {
  return (b >= n * uneg) ? 1.0 / n : 1.0 / (n + 1);
}

static double F_of(const commodity_t *c, double S) {
  if (c->alpha > 0.0 && !(S > 0.0)) return INFINITY;
  double h = h_of(c, S);
  if (isinf(h)) return h < 0 ? INFINITY : -INFINITY;
  double sum = 0.0;
  for (int r = 0; r < c->np; ++r) sum += xi(c->a[r] - h, c->n[r], c->uneg[r]);
  return sum - S;
}

static double dF_of(const commodity_t *c, double S) {
  double h = h_of(c, S), k = 0.0;
  for (int r = 0; r < c->np; ++r) k += dxi(c->a[r] - h, c->n[r], c->uneg[r]);
  return -dh_of(c, S) * k - 1.0;
}

/* Safeguarded Newton on the bracketed root of F (appendix B.2): Newton
 * steps while they stay strictly inside the bracket [lo, hi] with
 * F(lo) > 0 > F(hi), bisection otherwise.  Returns the root; *steps gets
 * the number of F evaluations after bracketing. */
static double sum_root(const commodity_t *c, double S0, int max_steps, int *steps) {
  const double tol = 1e-13;
  if (c->alpha > 0.0 && !(S0 > 0.0)) S0 = (c->D > 0.0 ? c->D : 1.0);
  double F0 = F_of(c, S0);
  *steps = 0;
  if (F0 == 0.0) return S0;
  const double d0 = dF_of(c, S0);
  /* first trial end of the bracket: 1.5 Newton steps from the warm start, then doubling */
  double guess = (isfinite(F0) && isfinite(d0) && d0 < 0.0) ? -1.5 * F0 / d0 : 0.0;
  double lo, hi;
  if (F0 > 0.0) {
    lo = S0;
    double step = guess > 0.0 ? guess : (fabs(S0) > 1e-6 ? fabs(S0) : 1e-6);
    for (;;) {
      hi = S0 + step;
      double Fh = F_of(c, hi);
      if (Fh == 0.0) return hi;
      if (Fh < 0.0) break;
      lo = hi;
      step *= 2.0;
    }
  } else {
    hi = S0;
    if (c->alpha > 0.0) {
      lo = (guess < 0.0 && S0 + guess > 0.0) ? S0 + guess : 0.5 * S0;
      for (;;) {
        double Fl = F_of(c, lo);
        if (Fl == 0.0) return lo;
        if (Fl > 0.0) break;
        hi = lo;
        lo *= 0.5;
        if (lo < 1e-300) return lo;
      }
    } else {
      double step = guess < 0.0 ? -guess : (fabs(S0) > 1e-6 ? fabs(S0) : 1e-6);
      for (;;) {
        lo = S0 - step;
        double Fl = F_of(c, lo);
        if (Fl == 0.0) return lo;
        if (Fl > 0.0) break;
        hi = lo;
        step *= 2.0;
      }
    }
  }
  double S = (F0 > 0.0) ? lo : hi;
  for (int it = 0; it < max_steps; ++it) {
    double Fs = F_of(c, S), dFs = dF_of(c, S);
    double scale = fabs(S) > 1.0 ? fabs(S) : 1.0;
    double Sn = 0.0;
    int newton = isfinite(Fs) && isfinite(dFs) && dFs < 0.0;
    if (newton) {
      double step = Fs / dFs;
      if (fabs(step) <= tol * scale) return S - step; /* Newton correction below tolerance */
      Sn = S - step;
      newton = (Sn > lo && Sn < hi);
    }
    if (!newton) Sn = 0.5 * (lo + hi);
    double Fn = F_of(c, Sn);
    ++*steps;
    if (Fn == 0.0) return Sn;
    if (Fn > 0.0) lo = Sn; else hi = Sn;
    scale = fabs(Sn) > 1.0 ? fabs(Sn) : 1.0;
    if (hi - lo <= tol * scale) return Sn;
    S = Sn;
  }
  return S;
}

/* Exported for pins: solve one commodity's sum equation and the rates. */
int gate_oracle_sum_root(int np, const double *a, const double *n_links, const double *uneg,
                         double D, double udem, double alpha, double beta, double S0,
                         double *S_out, double *x_out) {
  /* n_links: n_r, or the weights W_r of per-link penalties */
  double *n = (double *)malloc(sizeof(double) * (size_t)np);
  for (int r = 0; r < np; ++r) n[r] = n_links[r];
  commodity_t c = {np, a, n, uneg, D, udem, alpha, beta};
  int steps;
  double S = sum_root(&c, S0, 200, &steps);
  double h = h_of(&c, S);
  for (int r = 0; r < np; ++r) x_out[r] = xi(a[r] - h, n[r], uneg[r]);
  *S_out = S;
  free(n);
  return steps;
}

/* ------------------------------------------------------------------------ */
/* Projection (Algorithm 2, section 3.5)                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double key; int32_t p; double x; } trim_item;

/* Descending score; ties: higher path index first (READING). */
static int trim_cmp(const void *A, const void *B) {
  const trim_item *a = (const trim_item *)A, *b = (const trim_item *)B;
  if (a->key > b->key) return -1;
  if (a->key < b->key) return 1;
  return (a->p > b->p) ? -1 : (a->p < b->p ? 1 : 0);
}

/* log of score_p = S_c^alpha * C_p (Algorithm 2); -inf when C_p = 0 or S_c = 0.  The paper fixes
   no precision for the score, so it is taken in FP64 like everything else here. */
static double log_score(double S, int Cp, double alpha) {
  if (Cp <= 0 || !(S > 0.0)) return -INFINITY;
  return alpha * log(S) + log((double)Cp);
}

static void aux_vars(int E, const double *C, int P, const int64_t *pptr, const int32_t *plinks, int D,
                     const int32_t *dptr, const double *Dem, const double *x, double *S, double *L,
                     double *Vv, int *Cp) {
  for (int c = 0; c < D; ++c) {
    double s = 0.0;
    for (int r = dptr[c]; r < dptr[c + 1]; ++r) s += x[r];
    S[c] = s;
  }
  for (int e = 0; e < E; ++e) L[e] = 0.0;
  for (int r = 0; r < P; ++r)
    for (int64_t i = pptr[r]; i < pptr[r + 1]; ++i) L[plinks[i]] += x[r];
  for (int e = 0; e < E; ++e) Vv[e] = L[e] > C[e] ? L[e] - C[e] : 0.0;
  for (int r = 0; r < P; ++r) {
    int k = 0;
    for (int64_t i = pptr[r]; i < pptr[r + 1]; ++i) k += Vv[plinks[i]] > 0.0;
    Cp[r] = k;
  }
  (void)Dem;
}

/* x_mid (nullable): the rates after the demand trims (step 3); score (nullable): the log-scores of
   the link phase (after the recompute of step 4). */
static void project(int E, const double *C, int P, const int64_t *pptr, const int32_t *plinks, int D,
                    const int32_t *dptr, const double *Dem, const int32_t *lptr, const int32_t *lpaths,
                    double alpha, double *x, double *x_mid, double *score) {
  double *S = (double *)malloc(sizeof(double) * (size_t)(D ? D : 1));
  double *L = (double *)malloc(sizeof(double) * (size_t)E);
  double *Vv = (double *)malloc(sizeof(double) * (size_t)E);
  int *Cp = (int *)malloc(sizeof(int) * (size_t)(P ? P : 1));
  /* 1. non-negativity */
  for (int r = 0; r < P; ++r) x[r] = x[r] > 0.0 ? x[r] : 0.0;
  /* 2. auxiliary variables */
  aux_vars(E, C, P, pptr, plinks, D, dptr, Dem, x, S, L, Vv, Cp);
  /* 3. demand violations, per commodity, paths in descending score */
  int maxdeg = 1;
  for (int c = 0; c < D; ++c) if (dptr[c + 1] - dptr[c] > maxdeg) maxdeg = dptr[c + 1] - dptr[c];
  for (int e = 0; e < E; ++e) if (lptr[e + 1] - lptr[e] > maxdeg) maxdeg = lptr[e + 1] - lptr[e];
  trim_item *it = (trim_item *)malloc(sizeof(trim_item) * (size_t)maxdeg);
  for (int c = 0; c < D; ++c) {
    double Ec = S[c] > Dem[c] ? S[c] - Dem[c] : 0.0;
    if (!(Ec > 0.0)) continue;
    int m = 0;
    for (int r = dptr[c]; r < dptr[c + 1]; ++r) {
      it[m].key = log_score(S[c], Cp[r], alpha); it[m].p = r; it[m].x = x[r]; ++m;
    }
    qsort(it, (size_t)m, sizeof(trim_item), trim_cmp);
    for (int j = 0; j < m && Ec > 0.0; ++j) {
      int r = it[j].p;
      double d = Ec < x[r] ? Ec : x[r];
      x[r] -= d;
      Ec -= d;
    }
  }
  /* 4. recompute auxiliary variables */
  aux_vars(E, C, P, pptr, plinks, D, dptr, Dem, x, S, L, Vv, Cp);
  int *dem_of = (int *)malloc(sizeof(int) * (size_t)(P ? P : 1));
  for (int c = 0; c < D; ++c) for (int r = dptr[c]; r < dptr[c + 1]; ++r) dem_of[r] = c;
  if (x_mid) memcpy(x_mid, x, sizeof(double) * (size_t)P);
  if (score) for (int r = 0; r < P; ++r) score[r] = log_score(S[dem_of[r]], Cp[r], alpha);
  /* 5. capacity violations.  READING: every link trims from the same
   * snapshot of x ("in parallel" in Algorithm 2); a path trimmed by several
   * links gives up the largest of those trims. */
  double *trim = (double *)calloc((size_t)(P ? P : 1), sizeof(double));
  for (int e = 0; e < E; ++e) {
    double Ve = Vv[e];
    if (!(Ve > 0.0)) continue;
    int m = 0;
    for (int j = lptr[e]; j < lptr[e + 1]; ++j) {
      int r = lpaths[j];
      it[m].key = log_score(S[dem_of[r]], Cp[r], alpha); it[m].p = r; it[m].x = x[r]; ++m;
    }
    qsort(it, (size_t)m, sizeof(trim_item), trim_cmp);
    for (int j = 0; j < m && Ve > 0.0; ++j) {
      double d = Ve < it[j].x ? Ve : it[j].x;
      if (d > trim[it[j].p]) trim[it[j].p] = d;
      Ve -= d;
    }
  }
  for (int r = 0; r < P; ++r) x[r] -= trim[r];
  free(trim); free(dem_of); free(it); free(S); free(L); free(Vv); free(Cp);
}

/* Exported for pins: Algorithm 2 on given rates (original units); x_mid / score as in project(). */
int gate_oracle_project(int n_links, const double *capacity, int n_paths, const int64_t *path_ptr,
                        const int32_t *path_links, int n_demands, const int32_t *demand_path_ptr,
                        const double *demand, double alpha, double *x, double *x_mid, double *score) {
  int E = n_links, P = n_paths;
  int32_t *lptr = (int32_t *)calloc((size_t)E + 1, sizeof(int32_t));
  for (int64_t i = 0; i < path_ptr[P]; ++i) lptr[path_links[i] + 1]++;
  for (int e = 0; e < E; ++e) lptr[e + 1] += lptr[e];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
  memcpy(fill, lptr, sizeof(int32_t) * (size_t)E);
  int32_t *lpaths = (int32_t *)malloc(sizeof(int32_t) * (size_t)(path_ptr[P] ? path_ptr[P] : 1));
  for (int r = 0; r < P; ++r)
    for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) lpaths[fill[path_links[i]]++] = r;
  project(E, capacity, P, path_ptr, path_links, n_demands, demand_path_ptr, demand, lptr, lpaths, alpha, x,
          x_mid, score);
  free(lptr); free(fill); free(lpaths);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The solve                                                                 */
/* ------------------------------------------------------------------------ */
static double sq(double v) { return v * v; }

int gate_oracle_solve(int n_links, const double *capacity, int n_paths, const int64_t *path_ptr,
                      const int32_t *path_links, int n_demands, const int32_t *demand_path_ptr,
                      const double *demand, const go_options *opt, const double *x0,
                      double *x_out, double *S_out, go_state *st, go_stats *stats) {
  const int E = n_links, P = n_paths, D = n_demands;
  const int64_t nnz = path_ptr[P];
  memset(stats, 0, sizeof(*stats));
  stats->stop_iter = -1;

  /* units (READING): divide by the largest capacity of a used link */
  double scale = 0.0;
  for (int64_t i = 0; i < nnz; ++i) if (capacity[path_links[i]] > scale) scale = capacity[path_links[i]];
  if (!(scale > 0.0)) return 1;
  double *C = (double *)malloc(sizeof(double) * (size_t)E);
  double *Dm = (double *)malloc(sizeof(double) * (size_t)D);
  for (int e = 0; e < E; ++e) C[e] = capacity[e] / scale;
  for (int c = 0; c < D; ++c) Dm[c] = demand[c] / scale;

  /* incidence bookkeeping: n_r, link -> incidences (CSR positions), n_e */
  int *n_r = (int *)malloc(sizeof(int) * (size_t)P);
  for (int r = 0; r < P; ++r) n_r[r] = (int)(path_ptr[r + 1] - path_ptr[r]);
  /* per-link penalty factors w_e (READING, per-link penalties): link e's consensus and capacity
     constraints carry the penalty beta * w_e, the demand and non-negativity constraints beta; the
     x-block weighs link e's terms by w_e, so n_r becomes W_r = sum_{e in r} w_e */
  double *w = (double *)malloc(sizeof(double) * (size_t)(E ? E : 1));
  double *W_r = (double *)malloc(sizeof(double) * (size_t)(P ? P : 1));
  for (int e = 0; e < E; ++e) w[e] = (opt->warm && opt->warm->w) ? opt->warm->w[e] : 1.0;
  int32_t *lptr = (int32_t *)calloc((size_t)E + 1, sizeof(int32_t));
  for (int64_t i = 0; i < nnz; ++i) lptr[path_links[i] + 1]++;
  for (int e = 0; e < E; ++e) lptr[e + 1] += lptr[e];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
  memcpy(fill, lptr, sizeof(int32_t) * (size_t)E);
  int64_t *linc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1)); /* CSR positions */
  int32_t *lpaths = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  int32_t *inc_path = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  for (int r = 0; r < P; ++r)
    for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) {
      int32_t j = fill[path_links[i]]++;
      linc[j] = i;
      lpaths[j] = r;
      inc_path[i] = r;
    }

  /* variables (Algorithm 1 initialisation) */
  double *x = (double *)malloc(sizeof(double) * (size_t)P);
  double *x_prev = (double *)malloc(sizeof(double) * (size_t)P);
  double *y = (double *)malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
  double *ucon = (double *)calloc((size_t)(nnz ? nnz : 1), sizeof(double));
  double *ucap = (double *)calloc((size_t)E, sizeof(double));
  double *udem = (double *)calloc((size_t)(D ? D : 1), sizeof(double));
  double *uneg = (double *)calloc((size_t)(P ? P : 1), sizeof(double));
  double *S = (double *)malloc(sizeof(double) * (size_t)(D ? D : 1));
  double *a = (double *)malloc(sizeof(double) * (size_t)(P ? P : 1));
  double *gq_g = (double *)calloc((size_t)E, sizeof(double)); /* collapsed form: g_e */
  double *gq_q = (double *)calloc((size_t)E, sizeof(double)); /* collapsed form: q_e */
  double *dr = (double *)malloc(sizeof(double) * (size_t)(P ? P : 1));  /* per-element residual terms */
  double *ds = (double *)malloc(sizeof(double) * (size_t)(P ? P : 1));
  double *dd = (double *)malloc(sizeof(double) * (size_t)(D ? D : 1));
  double *de = (double *)malloc(sizeof(double) * (size_t)E);
  int *steps_c = (int *)calloc((size_t)(D ? D : 1), sizeof(int));

  const go_warm *wm = opt->warm;
  if (wm) {
    /* continuation: the earlier iterate, converted to this solve's units */
    for (int r = 0; r < P; ++r) { x[r] = wm->x[r] / scale; uneg[r] = wm->uneg[r] / scale; }
    for (int c = 0; c < D; ++c) { S[c] = wm->S[c] / scale; udem[c] = wm->udem[c] / scale; }
    for (int64_t i = 0; i < nnz; ++i) { y[i] = wm->y[i] / scale; ucon[i] = wm->ucon[i] / scale; }
    for (int e = 0; e < E; ++e) ucap[e] = wm->ucap[e] / scale;
    /* collapsed bookkeeping: g_e = dual_cap_e and q_e = y_{e,r} - x_r (the same for every r on e
       once a sweep has run) */
    for (int e = 0; e < E; ++e) {
      gq_g[e] = ucap[e];
      gq_q[e] = lptr[e + 1] > lptr[e] ? y[linc[lptr[e]]] - x[inc_path[linc[lptr[e]]]] : 0.0;
    }
  } else {
    for (int c = 0; c < D; ++c) {
      int m = demand_path_ptr[c + 1] - demand_path_ptr[c];
      for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r)
        x[r] = x0 ? x0[r] / scale : Dm[c] / m; /* x^0 = D/|P_st| unless given */
    }
    for (int c = 0; c < D; ++c) {
      double s = 0.0;
      for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r) s += x[r];
      S[c] = s;
    }
    for (int r = 0; r < P; ++r)
      for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) y[i] = x[r]; /* y^0 = x^0 */
  }

  const int replay = opt->sched_beta != NULL && opt->sched_alpha != NULL;
  const int fixed = opt->fixed_iters > 0;
  const int K = fixed ? opt->fixed_iters : opt->max_iters;
  const int max_steps = opt->root_max_steps > 0 ? opt->root_max_steps : 200;
  double alpha = replay ? opt->sched_alpha[0] : (wm ? wm->alpha : 0.0);
  if (!replay && opt->alpha_target < alpha) alpha = opt->alpha_target;
  double beta = replay ? opt->sched_beta[0] : (wm ? wm->beta : opt->beta0);
  if (wm && beta != wm->beta) {
    /* a replayed schedule starting at another penalty: the scaled duals are divided by the
       factor, as on every change of beta */
    const double f0 = beta / wm->beta;
    for (int c = 0; c < D; ++c) udem[c] /= f0;
    for (int e = 0; e < E; ++e) { ucap[e] /= f0; gq_g[e] /= f0; }
    for (int r = 0; r < P; ++r) uneg[r] /= f0;
    for (int64_t i = 0; i < nnz; ++i) ucon[i] /= f0;
  }
  int j = 0, k = 0, stop = 0;
  double r_res = 0.0, s_res = 0.0;
  /* back-off of the residual-balancing rule: direction of its last change of beta (+1, -1, 0 for
     none yet), number of reversals of that direction, and the first sweep count at which it may act
     again */
  int last_dir = wm ? wm->last_dir : 0, n_rev = wm ? wm->n_rev : 0, rule_from = wm ? wm->rule_rest : 0;
  long long steps_total = 0;
  int steps_max = 0;

  for (k = 0; k < K && !stop; ++k) {
    if (replay) {
      int kk = k < opt->sched_len ? k : opt->sched_len - 1;
      alpha = opt->sched_alpha[kk];
      beta = opt->sched_beta[kk];
    }
    memcpy(x_prev, x, sizeof(double) * (size_t)P);
    for (int r = 0; r < P; ++r) {
      double t = 0.0;
      for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) t += w[path_links[i]];
      W_r[r] = opt->per_link ? t : (double)n_r[r];
    }

    /* 1. x-block: per commodity, exact minimisation via the sum equation */
#pragma omp parallel for schedule(dynamic, 64) if (D > 1024)
    for (int c = 0; c < D; ++c) {
      int r0 = demand_path_ptr[c], m = demand_path_ptr[c + 1] - r0;
      for (int r = r0; r < r0 + m; ++r) {
        double s = 0.0;
        if (opt->collapsed) {
          /* a_r = W_r x_r - sum_{e in r} w_e (g_e - q_e) (equal to the line below after sweep 1) */
          for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) {
            const int e = path_links[i];
            s += opt->per_link ? w[e] * (gq_q[e] - gq_g[e]) : gq_q[e] - gq_g[e];
          }
          s += W_r[r] * x[r];
        } else {
          for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i)
            s += opt->per_link ? w[path_links[i]] * (y[i] - ucon[i]) : y[i] - ucon[i];
        }
        a[r] = s;
      }
      commodity_t cm = {m, a + r0, W_r + r0, uneg + r0, Dm[c], udem[c], alpha, beta};
      int steps;
      double Sst = sum_root(&cm, S[c], max_steps, &steps);
      steps_c[c] = steps;
      double h = h_of(&cm, Sst);
      double sum = 0.0;
      for (int r = r0; r < r0 + m; ++r) {
        x[r] = xi(a[r] - h, W_r[r], uneg[r]);
        sum += x[r];
      }
      S[c] = sum;
    }
    for (int c = 0; c < D; ++c) { steps_total += steps_c[c]; if (steps_c[c] > steps_max) steps_max = steps_c[c]; }

    /* 2. y-block: per link, exact minimisation jointly with slack_cap */
    /* 3. dual updates (section 3.3), on the new x and y */
#pragma omp parallel for schedule(dynamic, 16) if (E > 256)
    for (int e = 0; e < E; ++e) {
      int n_e = lptr[e + 1] - lptr[e];
      if (opt->collapsed) {
        double load = 0.0;
        for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) load += x[lpaths[jj]];
        double g_old = gq_g[e];
        double g = g_old + (load - C[e]) / (1 + n_e);
        g = g > 0.0 ? g : 0.0;
        gq_q[e] = g_old - g;
        gq_g[e] = g;
        de[e] = (1 + n_e) * sq(g - g_old);
        continue;
      }
      double V = 0.0;
      for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) { int64_t i = linc[jj]; V += x[inc_path[i]] + ucon[i]; }
      double W = ucap[e] + V - C[e];
      double g = (W > 0.0 ? W : 0.0) / (1 + n_e);
      double ysum = 0.0;
      for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) {
        int64_t i = linc[jj];
        y[i] = x[inc_path[i]] + ucon[i] - g;
        ysum += y[i];
      }
      /* dual_cap_e <- [dual_cap_e + sum_r y_{e,r} - C_e]_+ */
      double ucap_new = ucap[e] + ysum - C[e];
      ucap_new = ucap_new > 0.0 ? ucap_new : 0.0;
      double acc = sq(ucap_new - ucap[e]);
      /* dual_con_{e,r} <- [dual_con_{e,r} + x_r - y_{e,r}]_+ */
      for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) {
        int64_t i = linc[jj];
        double u = ucon[i] + x[inc_path[i]] - y[i];
        u = u > 0.0 ? u : 0.0;
        acc += sq(u - ucon[i]);
        ucon[i] = u;
      }
      ucap[e] = ucap_new;
      de[e] = acc;
    }
    if (!opt->collapsed) {
      double dev = stats->collapse_dev;
      for (int e = 0; e < E; ++e)
        for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) {
          double dlt = fabs(ucon[linc[jj]] - ucap[e]);
          if (dlt > dev) dev = dlt;
        }
      stats->collapse_dev = dev;
    }
    /* dual_dem_c <- [dual_dem_c + S_c - D_c]_+ ; dual_neg_r <- [dual_neg_r - x_r]_+ */
    for (int c = 0; c < D; ++c) {
      double u = udem[c] + S[c] - Dm[c];
      u = u > 0.0 ? u : 0.0;
      dd[c] = sq(u - udem[c]);
      udem[c] = u;
    }
    for (int r = 0; r < P; ++r) {
      double u = uneg[r] - x[r];
      u = u > 0.0 ? u : 0.0;
      dr[r] = sq(u - uneg[r]);
      uneg[r] = u;
      ds[r] = sq(x[r] - x_prev[r]);
    }

    /* 4. residuals (plain L2 over all entries, READING) */
    double rr = 0.0, ss = 0.0;
    for (int c = 0; c < D; ++c) rr += dd[c];
    for (int e = 0; e < E; ++e) rr += de[e];
    for (int r = 0; r < P; ++r) { rr += dr[r]; ss += ds[r]; }
    r_res = sqrt(rr);
    s_res = sqrt(ss);
    if (opt->dual_res_scaled) s_res *= beta;

    if (st && st->trace && k < st->trace_cap) {
      st->trace[5 * k + 0] = alpha;
      st->trace[5 * k + 1] = beta;
      st->trace[5 * k + 2] = r_res;
      st->trace[5 * k + 3] = s_res;
      st->trace[5 * k + 4] = stats->flags;
    }

    /* 5. adaptive beta (residual balancing) and rescale of the scaled duals.  READING: the rule
       may act after sweep k + 1 when the cadence admits it and its back-off has run out; a change
       of beta opposite to the previous one is the n-th reversal and makes the rule rest for the
       next 2^n - 1 sweeps (2^20 at most) */
    double f = 1.0;
    const int rule_now = ((k + 1) % (opt->beta_every > 0 ? opt->beta_every : 1)) == 0 && k + 1 >= rule_from;
    if (replay) {
      if (k + 1 < opt->sched_len) f = opt->sched_beta[k + 1] / opt->sched_beta[k];
    } else if (opt->adapt_beta && rule_now) {
      if (r_res > opt->A * s_res) {
        if (beta * opt->C <= opt->beta_max) f = opt->C; else stats->flags |= GO_HIT_BETA_BOUND;
      } else if (s_res > opt->A * r_res) {
        if (beta / opt->C >= opt->beta_min) f = 1.0 / opt->C; else stats->flags |= GO_HIT_BETA_BOUND;
      }
      if (f != 1.0) {
        const int dir = f > 1.0 ? 1 : -1;
        if (last_dir != 0 && dir != last_dir) {
          ++n_rev;
          rule_from = k + 1 + (1 << (n_rev < 20 ? n_rev : 20));
        }
        last_dir = dir;
      }
    }
    if (f != 1.0) {
      beta *= f;
      for (int c = 0; c < D; ++c) udem[c] /= f;
      for (int e = 0; e < E; ++e) { ucap[e] /= f; gq_g[e] /= f; }
      for (int r = 0; r < P; ++r) uneg[r] /= f;
      for (int64_t i = 0; i < nnz; ++i) ucon[i] /= f;
    }
    /* 5b. per-link penalties (READING): the same residual-balancing rule, on the same cadence, per
       link e on its own residuals -- r_e = the change of link e's scaled duals (its capacity dual
       and the consensus duals of its paths; each equals that constraint's residual), s_e = the
       change of the rates of the paths through e -- moves w_e by C within [w_min, w_max] and divides
       link e's scaled duals by the same factor; it acts on the sweeps where the global rule may
       act (the same cadence and back-off) */
    if (opt->per_link && rule_now) {
      for (int e = 0; e < E; ++e) {
        if (lptr[e + 1] == lptr[e]) continue;
        double s2 = 0.0;
        for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) s2 += ds[lpaths[jj]];
        const double re = sqrt(de[e]), se = sqrt(s2);
        double fe = 1.0;
        if (re > opt->A * se) {
          if (w[e] * opt->C <= opt->w_max) fe = opt->C;
        } else if (se > opt->A * re) {
          if (w[e] / opt->C >= opt->w_min) fe = 1.0 / opt->C;
        }
        if (fe == 1.0) continue;
        w[e] *= fe;
        ucap[e] /= fe;
        gq_g[e] /= fe;
        for (int jj = lptr[e]; jj < lptr[e + 1]; ++jj) ucon[linc[jj]] /= fe;
      }
    }

    /* 6. alpha-increments and stop (Algorithm 1).  READING: a stop needs
     * alpha >= 1 and convergence on the first sweep after an increment;
     * with a fixed sweep count there is no stop and alpha keeps rising. */
    ++j;
    if (!replay && r_res <= opt->gamma && s_res <= opt->gamma) {
      int would_stop = 0;
      if (alpha >= opt->alpha_target) would_stop = 1;
      else if (alpha >= 1.0 && j <= 1) would_stop = 1;
      if (would_stop) {
        stats->flags |= GO_CONVERGED;
        if (stats->stop_iter < 0) stats->stop_iter = k + 1;
        if (!fixed) stop = 1;
      }
      if (!stop && alpha < opt->alpha_target) {
        double na = alpha + 1.0;
        if (na > opt->alpha_target) na = opt->alpha_target;
        if (na > opt->alpha_max) {
          stats->flags |= GO_HIT_ALPHA_MAX;
          if (!fixed) stop = 1;
        } else {
          alpha = na;
          j = 0;
        }
      }
    }
  }
  stats->iters = k;
  if (!fixed && !stop && !replay) stats->flags |= GO_HIT_MAX_ITERS;
  stats->final_alpha = alpha;
  stats->beta = beta;
  stats->r = r_res;
  stats->s = s_res;
  stats->root_steps_mean = (k > 0 && D > 0) ? (double)steps_total / ((double)k * D) : 0.0;
  stats->root_steps_max = steps_max;
  stats->last_dir = last_dir;
  stats->n_rev = n_rev;
  stats->rule_rest = rule_from > k ? rule_from - k : 0;

  /* violations before projection */
  {
    double mc = 0.0, md = 0.0;
    double *L = (double *)calloc((size_t)E, sizeof(double));
    for (int r = 0; r < P; ++r)
      for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) L[path_links[i]] += x[r];
    for (int e = 0; e < E; ++e) { double v = (L[e] - C[e]) / C[e]; if (v > mc) mc = v; }
    for (int c = 0; c < D; ++c) { double v = (S[c] - Dm[c]) / Dm[c]; if (v > md) md = v; }
    stats->max_cap_viol_rel = mc;
    stats->max_dem_viol_rel = md;
    free(L);
  }

  if (st) {
    st->scale = scale;
    if (st->w) memcpy(st->w, w, sizeof(double) * (size_t)E);
    if (st->x_raw) for (int r = 0; r < P; ++r) st->x_raw[r] = x[r];
    if (st->S_raw) for (int c = 0; c < D; ++c) st->S_raw[c] = S[c];
    if (st->dual_dem) memcpy(st->dual_dem, udem, sizeof(double) * (size_t)D);
    if (st->dual_cap) {
      if (opt->collapsed) memcpy(st->dual_cap, gq_g, sizeof(double) * (size_t)E);
      else memcpy(st->dual_cap, ucap, sizeof(double) * (size_t)E);
    }
    if (st->dual_neg) memcpy(st->dual_neg, uneg, sizeof(double) * (size_t)P);
    if (st->dual_con) {
      if (opt->collapsed) for (int64_t i = 0; i < nnz; ++i) st->dual_con[i] = gq_g[path_links[i]];
      else memcpy(st->dual_con, ucon, sizeof(double) * (size_t)nnz);
    }
    if (st->y) {
      if (opt->collapsed) for (int64_t i = 0; i < nnz; ++i) st->y[i] = x[inc_path[i]] + gq_q[path_links[i]];
      else memcpy(st->y, y, sizeof(double) * (size_t)nnz);
    }
  }

  if (opt->project)
    project(E, C, P, path_ptr, path_links, D, demand_path_ptr, Dm, lptr, lpaths, alpha, x, NULL, NULL);
  for (int r = 0; r < P; ++r) x_out[r] = x[r] * scale;
  if (S_out)
    for (int c = 0; c < D; ++c) {
      double s = 0.0;
      for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r) s += x[r];
      S_out[c] = s * scale;
    }

  free(C); free(Dm); free(n_r); free(w); free(W_r); free(lptr); free(fill); free(linc); free(lpaths); free(inc_path);
  free(x); free(x_prev); free(y); free(ucon); free(ucap); free(udem); free(uneg); free(S); free(a);
  free(gq_g); free(gq_q); free(dr); free(ds); free(dd); free(de); free(steps_c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse pass (vector-Jacobian product) through K sweeps                    */
/* ------------------------------------------------------------------------ */
/*
 * Differentiates the unprojected sums S^(K)_c = sum_{r in P_c} x^(K)_r with respect to the
 * capacities C_e and demands D_c, for K sweeps of the full per-incidence iteration above with
 * the (beta_k, alpha_k) schedule given and the unit scale s given (both held fixed).  Every
 * [.]_+ takes its derivative on the branch taken (1 if the argument is > 0, else 0); the root
 * S*_c of the sum equation is differentiated through the implicit function theorem,
 * dS* = -(dF/dtheta) / (dF/dS).  The forward states of all K sweeps are kept in memory.
 *
 * Inputs in caller units; dS [D] cotangent on S^(K) (caller units); outputs dC [E], dD [D] are
 * gradients in caller units (with s fixed they equal the normalised-unit gradients).
 */
typedef struct {
  double *y, *ucon, *ucap, *udem, *uneg; /* state at the start of the sweep */
  double *x;                              /* x^{k+1} after the x-block */
  double *Sst;                            /* roots S*_c */
  double *S;                              /* sums of x^{k+1} */
  double *g;                              /* per-link g of the y-block */
  double *W;                              /* per-link W of the y-block */
  double *yn;                             /* y^{k+1} */
} sweep_t;

int gate_oracle_grad(int n_links, const double *capacity, int n_paths, const int64_t *path_ptr,
                     const int32_t *path_links, int n_demands, const int32_t *demand_path_ptr,
                     const double *demand, double scale, int K, const double *sched_beta,
                     const double *sched_alpha, const double *dS, double *S_out, double *dC, double *dD) {
  const int E = n_links, P = n_paths, D = n_demands;
  const int64_t nnz = path_ptr[P];
  if (!(scale > 0.0) || K <= 0) return 1;
  double *C = (double *)malloc(sizeof(double) * (size_t)E);
  double *Dm = (double *)malloc(sizeof(double) * (size_t)D);
  for (int e = 0; e < E; ++e) C[e] = capacity[e] / scale;
  for (int c = 0; c < D; ++c) Dm[c] = demand[c] / scale;
  int *n_r = (int *)malloc(sizeof(int) * (size_t)P);
  int *dem_of = (int *)malloc(sizeof(int) * (size_t)P);
  for (int r = 0; r < P; ++r) n_r[r] = (int)(path_ptr[r + 1] - path_ptr[r]);
  double *n_rd = (double *)malloc(sizeof(double) * (size_t)(P ? P : 1)); /* n_r as the x-block takes it */
  for (int r = 0; r < P; ++r) n_rd[r] = n_r[r];
  for (int c = 0; c < D; ++c) for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r) dem_of[r] = c;
  int32_t *lptr = (int32_t *)calloc((size_t)E + 1, sizeof(int32_t));
  for (int64_t i = 0; i < nnz; ++i) lptr[path_links[i] + 1]++;
  for (int e = 0; e < E; ++e) lptr[e + 1] += lptr[e];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)E);
  memcpy(fill, lptr, sizeof(int32_t) * (size_t)E);
  int64_t *linc = (int64_t *)malloc(sizeof(int64_t) * (size_t)nnz);
  int32_t *inc_path = (int32_t *)malloc(sizeof(int32_t) * (size_t)nnz);
  for (int r = 0; r < P; ++r)
    for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) {
      linc[fill[path_links[i]]++] = i;
      inc_path[i] = r;
    }

  sweep_t *sw = (sweep_t *)calloc((size_t)K, sizeof(sweep_t));
  double *y = (double *)malloc(sizeof(double) * (size_t)nnz);
  double *ucon = (double *)calloc((size_t)nnz, sizeof(double));
  double *ucap = (double *)calloc((size_t)E, sizeof(double));
  double *udem = (double *)calloc((size_t)D, sizeof(double));
  double *uneg = (double *)calloc((size_t)P, sizeof(double));
  double *Sws = (double *)malloc(sizeof(double) * (size_t)D);
  double *a = (double *)malloc(sizeof(double) * (size_t)P);
  for (int c = 0; c < D; ++c) {
    int m = demand_path_ptr[c + 1] - demand_path_ptr[c];
    for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r)
      for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) y[i] = Dm[c] / m;
    Sws[c] = Dm[c];
  }
#define ALLOC(n) (double *)malloc(sizeof(double) * (size_t)((n) ? (n) : 1))
  /* forward */
  for (int k = 0; k < K; ++k) {
    sweep_t *s = &sw[k];
    const double alpha = sched_alpha[k], beta = sched_beta[k];
    s->y = ALLOC(nnz); memcpy(s->y, y, sizeof(double) * (size_t)nnz);
    s->ucon = ALLOC(nnz); memcpy(s->ucon, ucon, sizeof(double) * (size_t)nnz);
    s->ucap = ALLOC(E); memcpy(s->ucap, ucap, sizeof(double) * (size_t)E);
    s->udem = ALLOC(D); memcpy(s->udem, udem, sizeof(double) * (size_t)D);
    s->uneg = ALLOC(P); memcpy(s->uneg, uneg, sizeof(double) * (size_t)P);
    s->x = ALLOC(P); s->Sst = ALLOC(D); s->S = ALLOC(D); s->g = ALLOC(E); s->W = ALLOC(E); s->yn = ALLOC(nnz);
    for (int c = 0; c < D; ++c) {
      int r0 = demand_path_ptr[c], m = demand_path_ptr[c + 1] - r0;
      for (int r = r0; r < r0 + m; ++r) {
        double acc = 0.0;
        for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) acc += y[i] - ucon[i];
        a[r] = acc;
      }
      commodity_t cm = {m, a + r0, n_rd + r0, uneg + r0, Dm[c], udem[c], alpha, beta};
      int steps;
      double Sst = sum_root(&cm, Sws[c], 200, &steps);
      double h = h_of(&cm, Sst), sum = 0.0;
      for (int r = r0; r < r0 + m; ++r) { s->x[r] = xi(a[r] - h, n_r[r], uneg[r]); sum += s->x[r]; }
      s->Sst[c] = Sst;
      s->S[c] = sum;
      Sws[c] = Sst;
    }
    for (int e = 0; e < E; ++e) {
      int ne = lptr[e + 1] - lptr[e];
      double V = 0.0;
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) V += s->x[inc_path[linc[j]]] + ucon[linc[j]];
      double W = ucap[e] + V - C[e];
      double g = (W > 0.0 ? W : 0.0) / (1 + ne);
      s->W[e] = W;
      s->g[e] = g;
      double ysum = 0.0;
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) {
        int64_t i = linc[j];
        s->yn[i] = s->x[inc_path[i]] + ucon[i] - g;
        ysum += s->yn[i];
      }
      double uc = ucap[e] + ysum - C[e];
      ucap[e] = uc > 0.0 ? uc : 0.0;
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) {
        int64_t i = linc[j];
        double u = ucon[i] + s->x[inc_path[i]] - s->yn[i];
        ucon[i] = u > 0.0 ? u : 0.0;
      }
    }
    memcpy(y, s->yn, sizeof(double) * (size_t)nnz);
    for (int c = 0; c < D; ++c) { double u = udem[c] + s->S[c] - Dm[c]; udem[c] = u > 0.0 ? u : 0.0; }
    for (int r = 0; r < P; ++r) { double u = uneg[r] - s->x[r]; uneg[r] = u > 0.0 ? u : 0.0; }
    double f = (k + 1 < K) ? sched_beta[k + 1] / sched_beta[k] : 1.0;
    if (f != 1.0) {
      for (int c = 0; c < D; ++c) udem[c] /= f;
      for (int e = 0; e < E; ++e) ucap[e] /= f;
      for (int r = 0; r < P; ++r) uneg[r] /= f;
      for (int64_t i = 0; i < nnz; ++i) ucon[i] /= f;
    }
  }
  if (S_out) for (int c = 0; c < D; ++c) S_out[c] = sw[K - 1].S[c] * scale;

  /* reverse: adjoints of the state after sweep k (before the rescale of that sweep) */
  double *bx = (double *)calloc((size_t)P, sizeof(double));      /* x^{k+1} */
  double *by = (double *)calloc((size_t)nnz, sizeof(double));    /* y^{k+1} */
  double *bucon = (double *)calloc((size_t)nnz, sizeof(double));
  double *bucap = (double *)calloc((size_t)E, sizeof(double));
  double *budem = (double *)calloc((size_t)D, sizeof(double));
  double *buneg = (double *)calloc((size_t)P, sizeof(double));
  double *bC = (double *)calloc((size_t)E, sizeof(double));
  double *bD = (double *)calloc((size_t)D, sizeof(double));
  double *nby = (double *)calloc((size_t)nnz, sizeof(double));  /* adjoint of y^k (input) */
  double *nucon = (double *)calloc((size_t)nnz, sizeof(double));
  double *nucap = (double *)calloc((size_t)E, sizeof(double));
  double *nudem = (double *)calloc((size_t)D, sizeof(double));
  double *nuneg = (double *)calloc((size_t)P, sizeof(double));
  double *bS = (double *)calloc((size_t)D, sizeof(double));
  double *ba = (double *)calloc((size_t)P, sizeof(double));
  /* S^(K) = sum x^(K): seed */
  for (int c = 0; c < D; ++c)
    for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r) bx[r] = dS[c];
  for (int k = K - 1; k >= 0; --k) {
    sweep_t *s = &sw[k];
    const double alpha = sched_alpha[k], beta = sched_beta[k];
    const double f = (k + 1 < K) ? sched_beta[k + 1] / sched_beta[k] : 1.0;
    /* rescale of sweep k: u_out = u_pre / f */
    for (int c = 0; c < D; ++c) budem[c] /= f;
    for (int e = 0; e < E; ++e) bucap[e] /= f;
    for (int r = 0; r < P; ++r) buneg[r] /= f;
    for (int64_t i = 0; i < nnz; ++i) bucon[i] /= f;
    memset(nby, 0, sizeof(double) * (size_t)nnz);
    memset(nucon, 0, sizeof(double) * (size_t)nnz);
    memset(nucap, 0, sizeof(double) * (size_t)E);
    memset(nudem, 0, sizeof(double) * (size_t)D);
    memset(nuneg, 0, sizeof(double) * (size_t)P);
    memset(bS, 0, sizeof(double) * (size_t)D);
    /* dual updates */
    for (int r = 0; r < P; ++r) {
      double m = (s->uneg[r] - s->x[r] > 0.0) ? 1.0 : 0.0;
      nuneg[r] += m * buneg[r];
      bx[r] -= m * buneg[r];
    }
    for (int c = 0; c < D; ++c) {
      double m = (s->udem[c] + s->S[c] - Dm[c] > 0.0) ? 1.0 : 0.0;
      nudem[c] += m * budem[c];
      bS[c] += m * budem[c];
      bD[c] -= m * budem[c];
    }
    for (int e = 0; e < E; ++e) {
      double ysum = 0.0;
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) ysum += s->yn[linc[j]];
      double m = (s->ucap[e] + ysum - C[e] > 0.0) ? 1.0 : 0.0;
      nucap[e] += m * bucap[e];
      bC[e] -= m * bucap[e];
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) {
        int64_t i = linc[j];
        by[i] += m * bucap[e];
        double mi = (s->ucon[i] + s->x[inc_path[i]] - s->yn[i] > 0.0) ? 1.0 : 0.0;
        nucon[i] += mi * bucon[i];
        bx[inc_path[i]] += mi * bucon[i];
        by[i] -= mi * bucon[i];
      }
    }
    /* y-block: y'_i = x'_r + ucon_i - g_e, g_e = [W_e]_+ / (1 + n_e), W_e = ucap_e + sum(x' + ucon) - C_e */
    for (int e = 0; e < E; ++e) {
      int ne = lptr[e + 1] - lptr[e];
      double bg = 0.0;
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) {
        int64_t i = linc[j];
        bx[inc_path[i]] += by[i];
        nucon[i] += by[i];
        bg -= by[i];
      }
      double bW = (s->W[e] > 0.0 ? 1.0 : 0.0) * bg / (1 + ne);
      nucap[e] += bW;
      bC[e] -= bW;
      for (int j = lptr[e]; j < lptr[e + 1]; ++j) {
        int64_t i = linc[j];
        bx[inc_path[i]] += bW;
        nucon[i] += bW;
      }
    }
    /* x-block: S_c = sum x'_r; x'_r = xi(a_r - h(S*)); S* root of F */
    for (int c = 0; c < D; ++c) {
      int r0 = demand_path_ptr[c], m = demand_path_ptr[c + 1] - r0;
      for (int r = r0; r < r0 + m; ++r) bx[r] += bS[c];
      double Sst = s->Sst[c];
      double t = Sst - Dm[c] + s->udem[c];
      double mh = t > 0.0 ? 1.0 : 0.0;
      double pw = (alpha == 0.0) ? 1.0 : exp(-alpha * log(Sst));
      double h = (t > 0.0 ? t : 0.0) - pw / beta;
      double dh = mh + (alpha == 0.0 ? 0.0 : alpha * pw / (beta * Sst));
      double sk = 0.0, bh = 0.0;
      for (int r = r0; r < r0 + m; ++r) {
        double ar = 0.0;
        for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) ar += s->y[i] - s->ucon[i];
        double b = ar - h;
        int hi = b >= n_r[r] * s->uneg[r];
        double kap = hi ? 1.0 / n_r[r] : 1.0 / (n_r[r] + 1);
        double xu = hi ? 0.0 : 1.0 / (n_r[r] + 1);
        sk += kap;
        double bb = bx[r] * kap;
        nuneg[r] += bx[r] * xu;
        ba[r] = bb;
        bh -= bb;
      }
      /* h(S*, D, udem) */
      double bSst = bh * dh;
      bD[c] -= bh * mh;
      nudem[c] += bh * mh;
      /* implicit root: mu = -bS* / F_S, F_S = -dh * sum kappa - 1 */
      double FS = -dh * sk - 1.0;
      double mu = -bSst / FS;
      bD[c] += mu * sk * mh;
      nudem[c] -= mu * sk * mh;
      for (int r = r0; r < r0 + m; ++r) {
        double ar = 0.0;
        for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) ar += s->y[i] - s->ucon[i];
        double b = ar - h;
        int hi = b >= n_r[r] * s->uneg[r];
        double kap = hi ? 1.0 / n_r[r] : 1.0 / (n_r[r] + 1);
        double xu = hi ? 0.0 : 1.0 / (n_r[r] + 1);
        ba[r] += mu * kap;
        nuneg[r] += mu * xu;
        /* a_r = sum (y_i - ucon_i) */
        for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) {
          nby[i] += ba[r];
          nucon[i] -= ba[r];
        }
      }
    }
    /* the inputs of sweep k become the outputs of sweep k-1 */
    memset(bx, 0, sizeof(double) * (size_t)P); /* x^k is not an input of the full-form sweep */
    memcpy(by, nby, sizeof(double) * (size_t)nnz);
    memcpy(bucon, nucon, sizeof(double) * (size_t)nnz);
    memcpy(bucap, nucap, sizeof(double) * (size_t)E);
    memcpy(budem, nudem, sizeof(double) * (size_t)D);
    memcpy(buneg, nuneg, sizeof(double) * (size_t)P);
  }
  /* initial point: y^0_i = D_c / |P_c| for the incidences of the paths of c */
  for (int c = 0; c < D; ++c) {
    int m = demand_path_ptr[c + 1] - demand_path_ptr[c];
    for (int r = demand_path_ptr[c]; r < demand_path_ptr[c + 1]; ++r)
      for (int64_t i = path_ptr[r]; i < path_ptr[r + 1]; ++i) bD[c] += by[i] / m;
  }
  for (int e = 0; e < E; ++e) dC[e] = bC[e];
  for (int c = 0; c < D; ++c) dD[c] = bD[c];
  for (int k = 0; k < K; ++k) {
    free(sw[k].y); free(sw[k].ucon); free(sw[k].ucap); free(sw[k].udem); free(sw[k].uneg);
    free(sw[k].x); free(sw[k].Sst); free(sw[k].S); free(sw[k].g); free(sw[k].W); free(sw[k].yn);
  }
#undef ALLOC
  free(sw); free(y); free(ucon); free(ucap); free(udem); free(uneg); free(Sws); free(a);
  free(bx); free(by); free(bucon); free(bucap); free(budem); free(buneg); free(bC); free(bD);
  free(nby); free(nucon); free(nucap); free(nudem); free(nuneg); free(bS); free(ba);
  free(C); free(Dm); free(n_r); free(n_rd); free(dem_of); free(lptr); free(fill); free(linc); free(inc_path);
  return 0;
}
