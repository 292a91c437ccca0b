// te_kernels.hip -- gfx950 kernels of the GATE iteration (section 3.3, Algorithm 1) and of the
// feasibility projection (section 3.5, Algorithm 2).
//
// Graph engine (large instances): one iteration = two device-wide kernels,
//   k_demand: per demand (G lanes, one per path): gather of (g_e, q_e) along each path,
//             sum equation by Newton-bisection, rate update, u_dem / u_neg updates;
//   k_link:   per run of links (one workgroup; its wavefronts walk contiguous parts of the CSC
//             list): segmented FP64 sums of the new rates, capacity/consensus dual update.
// Both kernels first apply the control decision of the previous iteration (residual balancing,
// alpha step, stop) redundantly in every workgroup from the previous iteration's partial sums,
// so no extra launch or grid-wide barrier is needed; iterations are replayed from a HIP graph.
//
// Workgroup engine (small instances, batches): one workgroup runs the whole solve with the
// instance resident in LDS and __syncthreads() between the steps; PPL paths per lane in the
// demand step, a group of lanes per link in the link step.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "te_device.h"
#include "te_internal.h"

namespace te {

// ------------------------------------------------------------------------------------------
// control record of this iteration, identical in every workgroup.  Wave 0 prefetches the
// previous record and its partial sums (prefetch_ctrl) before the workgroup's gathers and
// applies the decision afterwards (finish_ctrl), so the loads overlap with the gathers.
// ------------------------------------------------------------------------------------------
struct CtrlPrefetch {
  Ctrl prev;
  double v[4];
};

__device__ __forceinline__ void prefetch_ctrl(const State &s, int par, CtrlPrefetch &cp) {
  // par = k & 1 of this iteration; record k-1 and its partial sums live in slot par^1
  cp.prev = s.ctrl[par ^ 1];
  cp.v[0] = 0.0;
  cp.v[1] = 0.0;
  cp.v[2] = -INFINITY;
  cp.v[3] = -INFINITY;
  // all rows' loads are issued before the first add (nB <= 8 * 64), so they take one round trip:
  // they are unconditional (a slot past the rows reads the last row again: harmless for the maxima,
  // and masked out of the sums by a product -- a select, or a load inside a branch, would be waited
  // for before the next load is issued)
  const double2 *pb = reinterpret_cast<const double2 *>(s.partB + (size_t)(par ^ 1) * s.nB * 4);
  constexpr int R = kMaxLinkBlocks / 64;
  double2 lo[R], hi[R];
  double m[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = (threadIdx.x & 63) + 64 * u;
    const int ic = i < s.nB ? i : s.nB - 1;
    m[u] = i < s.nB ? 1.0 : 0.0;
    lo[u] = pb[2 * ic];
    hi[u] = pb[2 * ic + 1];
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    cp.v[0] = fma(lo[u].x, m[u], cp.v[0]);
    cp.v[1] = fma(lo[u].y, m[u], cp.v[1]);
    cp.v[2] = fmax(cp.v[2], hi[u].x);
    cp.v[3] = fmax(cp.v[3], hi[u].y);
  }
}

__device__ __forceinline__ void finish_ctrl(CtrlPrefetch &cp, const Params &prm, Ctrl *out) {
  cp.v[0] = wave_sum_d(cp.v[0]);
  cp.v[1] = wave_sum_d(cp.v[1]);
  cp.v[2] = wave_max_d(cp.v[2]);
  cp.v[3] = wave_max_d(cp.v[3]);
  if ((threadIdx.x & 63) == 0) *out = decide(cp.prev, cp.v, prm);
}

// per-wavefront partial sums (sum, sum, -, max) into dst[4 w .. 4 w + 3] by the wavefront's lane 0
__device__ __forceinline__ void wave_partials(double a, double b, double d, double *dst) {
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  d = wave_max_d(d);
  if ((threadIdx.x & 63) == 0) {
    double *o = dst + (threadIdx.x >> 6) * 4;
    o[0] = a;
    o[1] = b;
    o[2] = -INFINITY;
    o[3] = d;
  }
}

// The link kernel's workgroup 0 publishes this iteration's control record (pending: its decision
// is taken by the next iteration's kernels) and logs it when a log is attached: iteration k's beta
// and alpha, and the residuals of iteration k - 1 that the decision was taken from.
__device__ __forceinline__ void publish_ctrl(const State &s, const Ctrl &cs, int par) {
  Ctrl wr = cs;
  wr.pending = cs.stop ? 0 : 1;
  s.ctrl[par] = wr;
  if (s.log) {
    if (!cs.stop && cs.k < s.log_cap) {
      s.log[cs.k] = cs.beta;
      s.log[s.log_cap + cs.k] = cs.alpha;
    }
    if (cs.k >= 1 && cs.k <= s.log_cap) {
      s.log[2 * s.log_cap + cs.k - 1] = cs.r;
      s.log[3 * s.log_cap + cs.k - 1] = cs.s;
    }
  }
}

// XCD-aware work order.  The dispatcher deals the workgroups of a launch round-robin over the 8
// XCDs (workgroup b runs on XCD b % 8, each XCD with its own L2).  Processing logical block
// xcd_chunk(b) instead of b gives every XCD one contiguous range of the logical work: the demand
// kernel's blocks of consecutive demands and the link kernel's blocks of consecutive links then
// touch compact parts of the path arrays per XCD (one less trip to the memory side for what the
// same XCD wrote or read before).  A bijection of [0, n).
__device__ __forceinline__ int xcd_chunk(int b, int n) {
  const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + i;
}

// block-wide reduction of 4 partials (sum, sum, max, max) into dst[0..3] by thread 0
__device__ void block_partials(double p0, double p1, double p2, double p3, double *dst) {
  __shared__ double red[4][16];
  p0 = wave_sum_d(p0);
  p1 = wave_sum_d(p1);
  p2 = wave_max_d(p2);
  p3 = wave_max_d(p3);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = p0;
    red[1][w] = p1;
    red[2][w] = p2;
    red[3][w] = p3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = -INFINITY, d = -INFINITY;
    for (int i = 0; i < nw; ++i) {
      a += red[0][i];
      b += red[1][i];
      c = fmax(c, red[2][i]);
      d = fmax(d, red[3][i]);
    }
    dst[0] = a;
    dst[1] = b;
    dst[2] = c;
    dst[3] = d;
  }
}

// ------------------------------------------------------------------------------------------
// Initialisation (Algorithm 1): x^0 = D_c / |P_c| or the warm start, duals zero, y^0 = x^0.
// ------------------------------------------------------------------------------------------
__global__ void k_init(Prob p, State s, const Params *prmp, const float *x0, double inv_scale) {
  const Params &prm = *prmp;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    const int r0 = p.dptr[c], r1 = p.dptr[c + 1];
    double sum = 0.0;
    for (int r = r0; r < r1; ++r) {
      const double v = x0 ? (double)x0[r] * inv_scale : p.Dn[c] / (double)(r1 - r0);
      s.x[r] = v;
      s.uneg[r] = 0.0;
      sum += v;
    }
    s.udem[c] = 0.0;
    s.S[c] = sum;
  }
  for (int e = tid; e < p.E; e += nth) {
    s.gq[e] = make_double2(0.0, 0.0);
    s.w[e] = 1.0;
  }
  if (tid == 0) {
    Ctrl c = initial_ctrl(prm);
    s.ctrl[1] = c;   // read as "iteration -1" by iteration 0, not pending
    s.ctrl[0] = c;
    s.ctrl[2] = c;
  }
}

// Continuation from the state of the previous solve (warm restart): rate-like state converted to
// the current units (rescale = old scale / new scale), the control record restarted at iteration 0
// with the previous beta and alpha (alpha capped at the target; a replayed schedule overrides both)
// and the balancing rule's back-off where it stood (the rest still due counts from iteration 0).
// The scaled duals in memory are still at the penalty of the last iteration run (the rescale that
// the final decision took is applied lazily by the next iteration), so the first iteration divides
// them by beta_new / beta_last, like any other change of beta.
__global__ void k_warm(Prob p, State s, const Params *prmp, double rescale) {
  const Params &prm = *prmp;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  if (rescale != 1.0) {
    for (int r = tid; r < p.P; r += nth) {
      s.x[r] *= rescale;
      s.uneg[r] *= rescale;
    }
    for (int c = tid; c < p.D; c += nth) {
      s.udem[c] *= rescale;
      s.S[c] *= rescale;
    }
    for (int e = tid; e < p.E; e += nth) {
      const double2 v = s.gq[e];
      s.gq[e] = make_double2(v.x * rescale, v.y * rescale);
    }
  }
  if (tid == 0) {
    const Ctrl fin = s.ctrl[2];
    Ctrl c = initial_ctrl(prm);
    if (prm.sched_beta == nullptr) {
      c.beta = fin.beta;
      c.alpha = fmin(fin.alpha, prm.alpha_target);
      c.last_dir = fin.last_dir;
      c.n_rev = fin.n_rev;
      c.rule_from = fin.rule_from > fin.k ? fin.rule_from - fin.k : 0;
    }
    c.inv_f = fin.beta * fin.inv_f / c.beta;  // penalty of the stored duals over the new one
    s.ctrl[0] = c;
    s.ctrl[1] = c;
    s.ctrl[2] = c;
  }
}

// ------------------------------------------------------------------------------------------
// Step a1 + a2: gather along paths, per-demand Newton-bisection, rate and dual updates.
// ------------------------------------------------------------------------------------------
// Gathers of the (g, q) pairs along paths.  The kernels' time goes into dependent memory latency, so
// every load of a round is issued unconditionally and in one straight-line block: a padding slot, a
// slot past the path's end or a lane without a path reads a valid entry (g, q of link 0, a repeated
// record word) and is masked out of the sums.  A load inside a divergent branch is waited for before
// the branch rejoins, which would serialise the hops of a path into one round trip each.  The sums
// are taken in hop order, a masked slot adding 0 (so they equal a plain loop's up to the sign of a
// zero sum).

// id of slot k of a fixed-width hop record (16-bit link ids in path order, 0xffff past the end)
__device__ __forceinline__ unsigned hop_id(const uint2 (&w)[kMaxHopSlots / 4], int k) {
  const uint2 q = w[k >> 2];
  const unsigned h = (k & 2) ? q.y : q.x;
  return (k & 1) ? (h >> 16) : (h & 0xffffu);
}

// overflow record of path r of a demand whose first path is r0 and whose dovf entry is dv (-1: the
// demand has none)
__device__ __forceinline__ int overflow_record(int dv, int r, int r0) { return dv >= 0 ? dv + (r - r0) : -1; }

// the record of path r (its primary record, then its overflow record ovf if ovf >= 0); words past
// them read as padding.  The loads are unconditional (a word past a record reads its word 0), so
// that they issue together; the overflow records' loads are skipped only where the instance has
// none (a uniform condition).
__device__ __forceinline__ void load_record(const Prob &p, int r, int ovf, uint2 (&w)[kMaxHopSlots / 4]) {
  const uint2 *rec = reinterpret_cast<const uint2 *>(p.hops + (size_t)r * p.H);
#pragma unroll
  for (int q = 0; q < kMaxHopSlots / 4; ++q) {
    const bool in = 4 * q < p.H;
    const uint2 v = rec[in ? q : 0];
    w[q] = in ? v : make_uint2(~0u, ~0u);
  }
  if (p.H2 > 0) {
    const uint2 *rec2 = reinterpret_cast<const uint2 *>(p.hops2 + (size_t)(ovf >= 0 ? ovf : 0) * p.H2);
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) {
      const int q2 = q - p.H / 4;
      const bool in = q2 >= 0 && 4 * q2 < p.H2;
      const uint2 v = rec2[in ? q2 : 0];
      if (in) w[q] = ovf >= 0 ? v : make_uint2(~0u, ~0u);
    }
  }
}

// word q of the record of path r (primary, then overflow record ovf), padding past them
__device__ __forceinline__ uint2 record_word(const Prob &p, int r, int ovf, int q) {
  if (4 * q < p.H) return reinterpret_cast<const uint2 *>(p.hops + (size_t)r * p.H)[q];
  const int q2 = q - p.H / 4;
  if (ovf >= 0 && 4 * q2 < p.H2) return reinterpret_cast<const uint2 *>(p.hops2 + (size_t)ovf * p.H2)[q2];
  return make_uint2(~0u, ~0u);
}

// hop count of a record (its ids; padding only at the end).  Computed from every word, so that the
// record's loads are all waited for at once rather than split around the first use.
__device__ __forceinline__ int record_hops(const uint2 (&w)[kMaxHopSlots / 4]) {
  int n = 0;
#pragma unroll
  for (int k = 0; k < kMaxHopSlots; ++k) n += hop_id(w, k) != 0xffffu ? 1 : 0;
  return n;
}

// Sums of g and q, and hop counts, over the NP paths of a lane whose records are w[j] (path j taken
// where bit j of on is set), in rounds of R slots: a round issues the R * NP loads together and runs
// only while some lane of the wavefront has a hop in it.
template <int NP, int R>
__device__ __forceinline__ void gather_records(const State &s, const uint2 (&w)[NP][kMaxHopSlots / 4], unsigned on,
                                               double (&sg)[NP], double (&sq)[NP], int (&n)[NP]) {
  int nmax = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    sg[j] = 0.0;
    sq[j] = 0.0;
    n[j] = ((on >> j) & 1u) ? record_hops(w[j]) : 0;
    nmax = max(nmax, n[j]);
  }
#pragma unroll
  for (int k0 = 0; k0 < kMaxHopSlots; k0 += R) {
    if (!__any(nmax > k0)) break;
    unsigned id[NP][R];
    double2 v[NP][R];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int u = 0; u < R; ++u) id[j][u] = k0 + u < n[j] ? hop_id(w[j], k0 + u) : 0u;
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int u = 0; u < R; ++u) v[j][u] = s.gq[id[j][u]];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const double m = k0 + u < n[j] ? 1.0 : 0.0;  // a product, not a select: a select of a
        sg[j] = fma(v[j][u].x, m, sg[j]);             // loaded value is turned into a branch
        sq[j] = fma(v[j][u].y, m, sq[j]);             // around the load
      }
  }
}

// The same from the CSR layout (no hop records: a path with more than kMaxHopSlots hops, or a link id
// that does not fit 16 bits), eight hops of each path a round.  With per-link penalties (WEIGHTED)
// the sums are of w_e g_e and w_e q_e, and Wr[j] = sum of w_e (the path's weight in the rate update);
// otherwise Wr[j] is the hop count.  Every path has at least one link, so its first entry is a valid
// stand-in for a slot past its end.
template <int NP, bool WEIGHTED>
__device__ __forceinline__ void gather_csr(const Prob &p, const State &s, const int (&r)[NP], unsigned on,
                                           double (&sg)[NP], double (&sq)[NP], double (&Wr)[NP]) {
  int i0[NP], len[NP];
  int lmax = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    i0[j] = p.pptr[r[j]];
    len[j] = ((on >> j) & 1u) ? p.pptr[r[j] + 1] - i0[j] : 0;
    lmax = max(lmax, len[j]);
    sg[j] = 0.0;
    sq[j] = 0.0;
    Wr[j] = 0.0;
  }
  for (int k0 = 0; __any(k0 < lmax); k0 += 8) {
    int e[NP][8];
    double2 v[NP][8];
    double we[NP][8];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int u = 0; u < 8; ++u) e[j][u] = p.plinks[k0 + u < len[j] ? i0[j] + k0 + u : i0[j]];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[j][u] = s.gq[e[j][u]];
        we[j][u] = WEIGHTED ? s.w[e[j][u]] : 1.0;
      }
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double m = k0 + u < len[j] ? 1.0 : 0.0;  // a product, not a select (see above)
        const double wm = we[j][u] * m;
        sg[j] = fma(WEIGHTED ? we[j][u] * v[j][u].x : v[j][u].x, m, sg[j]);
        sq[j] = fma(WEIGHTED ? we[j][u] * v[j][u].y : v[j][u].y, m, sq[j]);
        Wr[j] += wm;
      }
  }
}

// Sums along the NP paths r[j] of a lane (bit j of on): from the hop records where the instance has
// them, else from the CSR layout; with per-link penalties always from the CSR layout, weighted.
template <int NP>
__device__ __forceinline__ void gather_paths(const Prob &p, const State &s, bool per_link, const int (&r)[NP],
                                             const int (&ovf)[NP], unsigned on, double (&sg)[NP], double (&sq)[NP],
                                             double (&Wr)[NP]) {
  if (per_link) {
    gather_csr<NP, true>(p, s, r, on, sg, sq, Wr);
  } else if (p.H > 0) {
    // one path after the other: a path's record and its round of eight loads are then all that is
    // live, which keeps the kernels with several paths per lane within their register budget
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      uint2 w[1][kMaxHopSlots / 4];
      load_record(p, r[j], ovf[j], w[0]);
      double g1[1], q1[1];
      int n1[1];
      gather_records<1, 8>(s, w, (on >> j) & 1u, g1, q1, n1);
      sg[j] = g1[0];
      sq[j] = q1[0];
      Wr[j] = (double)n1[0];
    }
  } else {
    gather_csr<NP, false>(p, s, r, on, sg, sq, Wr);
  }
}

// the per-link rule acts after this iteration (the iterations where the residual-balancing rule
// may act: the same cadence and back-off)
__device__ __forceinline__ bool per_link_rule_now(const Params &prm, const Ctrl &cs) {
  return prm.per_link && rule_may_act(prm, cs);
}

__global__ __launch_bounds__(kThreads + 64) void k_demand(Prob p, State s, const Params *prmp, int par) {
  const Params &prm = *prmp;
  __shared__ Ctrl cs;
  CtrlPrefetch cp;
  // the extra fifth wavefront takes the control decision (its loads and reductions are then off
  // the path lanes' critical path: -0.8 us per iteration on the 150-node instance)
  const bool ctl = threadIdx.x >= kThreads;
  if (ctl) prefetch_ctrl(s, par, cp);
  const int G = p.G;
  const int t = threadIdx.x;
  const int lane = t & (G - 1);
  const int bl = xcd_chunk(blockIdx.x, gridDim.x);
  const int c = bl * (kThreads >> p.logG) + (t >> p.logG);
  // gathers (independent of the control record): sums of g and q along the path
  int r0 = 0, np = 0, r = 0, dv = -1;
  double xr = 0.0, ung = 0.0, Dc = 0.0, Wn = 1.0;
  double sg = 0.0, sq = 0.0, udc = 0.0, S0 = 0.0;
  bool on = false;
  if (!ctl) {
    if (c < p.D) {
      Dc = p.Dn[c];  // per-demand loads first: they depend on c only
      udc = s.udem[c];
      S0 = s.S[c];
      r0 = p.dptr[c];
      np = p.dptr[c + 1] - r0;
      if (p.H2 > 0) dv = p.dovf[c];
    }
    on = lane < np;
    r = r0 + (on ? lane : 0);  // a lane without a path reads the demand's first (or path 0)
    const double xv = s.x[r], uv = s.uneg[r];
    xr = on ? xv : 0.0;
    ung = on ? uv : 0.0;
    const int rr[1] = {r}, ro[1] = {overflow_record(dv, r, r0)};
    double g1[1], q1[1], w1[1];
    gather_paths<1>(p, s, prm.per_link, rr, ro, on ? 1u : 0u, g1, q1, w1);
    sg = g1[0];
    sq = q1[0];
    Wn = on ? w1[0] : 1.0;
  }
  if (ctl) finish_ctrl(cp, prm, &cs);
  __syncthreads();
  if (cs.stop || ctl) return;
  const double inv_f = cs.inv_f;
  double ds2 = 0.0, dr2 = 0.0, dem_v = -INFINITY;
  if (c < p.D) {
    Lane L;
    L.on = on;
    L.a = on ? Wn * xr - (sg * inv_f - sq) : 0.0;
    L.un = ung * inv_f;
    L.n = Wn;
    L.rn = 1.0 / Wn;
    L.rn1 = 1.0 / (Wn + 1.0);
    Dem dm;
    dm.D = Dc;
    dm.u = udc * inv_f;
    dm.alpha = cs.alpha;
    dm.binv = 1.0 / cs.beta;
    int steps;
    const double Sst = sum_root(S0, L, dm, G, &steps);
    const double h = h_of(Sst, dm);
    const double xn = L.on ? xi_of(L.a - h, L) : 0.0;
    const double Ssum = group_sum_d(xn, G);
    if (L.on) {
      const double un = fmax(L.un - xn, 0.0);
      s.xo[r] = xn;
      s.unego[r] = un;
      ds2 = (xn - xr) * (xn - xr);
      dr2 = (un - L.un) * (un - L.un);
      if (per_link_rule_now(prm, cs)) s.dx2[r] = ds2;
    }
    if (lane == 0) {
      const double ud = fmax(dm.u + Ssum - dm.D, 0.0);
      s.udemo[c] = ud;
      s.So[c] = Sst;
      dr2 += (ud - dm.u) * (ud - dm.u);
      dem_v = (Ssum - dm.D) / dm.D;
    }
  }
  wave_partials(ds2, dr2, dem_v, s.partA + ((size_t)par * s.nA + bl) * (kThreads / 64) * 4);
}

// The same step with PPL (2, 4 or 8) paths per lane, for instances large enough to be bound by
// issue and bandwidth rather than latency: a demand with G path slots gets Gp = max(1, G / PPL)
// lanes (p.logGp), lane l holding the demand's paths l, l + Gp, ...; the per-demand part of the root
// solve is then replicated over fewer lanes, and its Newton steps get Halley's correction.
template <int PPL>
__global__ __launch_bounds__(kThreads) void k_demand_multi(Prob p, State s, const Params *prmp, int par) {
  const Params &prm = *prmp;
  __shared__ Ctrl cs;
  CtrlPrefetch cp;
  if (threadIdx.x < 64) prefetch_ctrl(s, par, cp);
  const int logGp = p.logGp, Gp = 1 << logGp;
  const int t = threadIdx.x;
  const int lane = t & (Gp - 1);
  const int bl = xcd_chunk(blockIdx.x, gridDim.x);
  const int c = bl * (kThreads >> logGp) + (t >> logGp);
  int r0 = 0, np = 0;
  double Dc = 0.0, udc = 0.0, S0 = 0.0;
  double xr[PPL], ung[PPL], sg[PPL], sq[PPL], Wn[PPL];
  unsigned on = 0u;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    xr[j] = ung[j] = sg[j] = sq[j] = 0.0;
    Wn[j] = 1.0;
  }
  int dv = -1;
  if (c < p.D) {
    Dc = p.Dn[c];
    udc = s.udem[c];
    S0 = s.S[c];
    r0 = p.dptr[c];
    np = p.dptr[c + 1] - r0;
    if (p.H2 > 0) dv = p.dovf[c];
  }
  {
    int rr[PPL], ro[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int idx = lane + j * Gp;
      const bool oj = idx < np;
      on |= oj ? 1u << j : 0u;
      rr[j] = r0 + (oj ? idx : 0);  // a slot without a path reads the demand's first (or path 0)
      ro[j] = overflow_record(dv, rr[j], r0);
      const double xv = s.x[rr[j]], uv = s.uneg[rr[j]];
      xr[j] = oj ? xv : 0.0;
      ung[j] = oj ? uv : 0.0;
    }
    double W[PPL];
    gather_paths<PPL>(p, s, prm.per_link, rr, ro, on, sg, sq, W);
#pragma unroll
    for (int j = 0; j < PPL; ++j) Wn[j] = ((on >> j) & 1u) ? W[j] : 1.0;
  }
  if (threadIdx.x < 64) finish_ctrl(cp, prm, &cs);
  __syncthreads();
  if (cs.stop) return;
  const double inv_f = cs.inv_f;
  double ds2 = 0.0, dr2 = 0.0, dem_v = -INFINITY;
  if (c < p.D) {
    LaneN<PPL> L;
    L.on = on;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const bool oj = (on >> j) & 1u;
      L.a[j] = oj ? Wn[j] * xr[j] - (sg[j] * inv_f - sq[j]) : 0.0;
      L.un[j] = ung[j] * inv_f;
      L.n[j] = Wn[j];
      L.rn[j] = 1.0 / Wn[j];
      L.rn1[j] = 1.0 / (Wn[j] + 1.0);
    }
    Dem dm;
    dm.D = Dc;
    dm.u = udc * inv_f;
    dm.alpha = cs.alpha;
    dm.binv = 1.0 / cs.beta;
    int steps;
    const double Sst = sum_root(S0, L, dm, Gp, &steps);
    const double h = h_of(Sst, dm);
    const bool rule = per_link_rule_now(prm, cs);
    double xsum = 0.0;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      if (!((on >> j) & 1u)) continue;
      const int r = r0 + lane + j * Gp;
      const double b = L.a[j] - h;
      const double xn = (b >= L.n[j] * L.un[j]) ? b * L.rn[j] : (b + L.un[j]) * L.rn1[j];
      const double un = fmax(L.un[j] - xn, 0.0);
      s.xo[r] = xn;
      s.unego[r] = un;
      if (rule) s.dx2[r] = (xn - xr[j]) * (xn - xr[j]);
      xsum += xn;
      ds2 += (xn - xr[j]) * (xn - xr[j]);
      dr2 += (un - L.un[j]) * (un - L.un[j]);
    }
    const double Ssum = group_sum_d(xsum, Gp);
    if (lane == 0) {
      const double ud = fmax(dm.u + Ssum - dm.D, 0.0);
      s.udemo[c] = ud;
      s.So[c] = Sst;
      dr2 += (ud - dm.u) * (ud - dm.u);
      dem_v = (Ssum - dm.D) / dm.D;
    }
  }
  wave_partials(ds2, dr2, dem_v, s.partA + ((size_t)par * s.nA + bl) * (kThreads / 64) * 4);
}

// CSC entry encodings: int32 (graph engine) with bit 31 on a link's first entry, uint16 (workgroup
// engine, LDS) with bit 15 on it.
__device__ __forceinline__ bool csc_head(int32_t v) { return v < 0; }
__device__ __forceinline__ int csc_path(int32_t v) { return v & 0x7fffffff; }
__device__ __forceinline__ bool csc_head(uint16_t v) { return (v & 0x8000u) != 0; }
__device__ __forceinline__ int csc_path(uint16_t v) { return v & 0x7fff; }

// Segmented sums over the CSC entries of the non-empty links owned by this workgroup (ranks k0..):
// acc[k - k0] += sum of vals[path] over the entries of link nzlink[k].  Each wavefront walks its
// contiguous part wt = {first entry, end, rank of the link holding the first entry} of the
// workgroup's entries in coalesced rows of 64.  A full row in which no link starts belongs wholly
// to the current link: each lane just adds its entry to a carried share (one add instead of a
// scan; most rows, since links hold hundreds to thousands of entries).  A row in which a link
// starts, or the part's last row, first hands the carried share in (wavefront sum, one LDS atomic),
// then reduces its runs of equal link by a segmented scan whose tail lanes add one partial each.
template <class I, class T>
__device__ __forceinline__ void seg_rows_sum(const I *lpf, const T *vals, int k0, int4 wt, double *acc) {
  const int lane = threadIdx.x & 63;
  const int ja = wt.x, jb = wt.y;
  if (ja >= jb) return;
  int kbase = wt.z;
  double carry = 0.0;    // this lane's share of link kbase over full rows in which no link starts
  bool carried = false;  // wavefront-uniform
  constexpr int U = 4;  // rows whose loads are issued together
  for (int j = ja; j < jb; j += 64 * U) {
    I v[U];
    double val[U];
    // unconditional loads (an entry past the part reads its first one, masked below), so that the
    // U rows' index loads, then their value loads, are in flight together
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int jj = j + 64 * u + lane;
      v[u] = lpf[jj < jb ? jj : ja];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int jj = j + 64 * u + lane;
      val[u] = (double)vals[csc_path(v[u])] * (jj < jb ? 1.0 : 0.0);  // a product, not a select
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int jj = j + 64 * u + lane;
      const bool valid = jj < jb;
      const bool head = valid && csc_head(v[u]) && jj != ja;
      const uint64_t hm = __ballot(head);
      if (hm == 0ull && j + 64 * u + 63 < jb) {  // the whole row belongs to link kbase
        carry += val[u];
        carried = true;
        continue;
      }
      if (carried) {  // the carried share goes in before the row's runs
        const double cs = wave_sum_d(carry);
        if (lane == 0) atomicAdd(&acc[kbase - k0], cs);
        carry = 0.0;
        carried = false;
      }
      const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
      // segment key: rank of the entry's link; lanes past the end get -3 (after every valid lane)
      const int key = valid ? kbase + __popcll(hm & le) : -3;
      const double x = seg_scan_d(val[u], key);
      const bool tail = valid && next_lane_key(key) != key;
      if (tail) atomicAdd(&acc[key - k0], x);
      kbase += __popcll(hm);
    }
  }
  if (carried) {
    const double cs = wave_sum_d(carry);
    if (lane == 0) atomicAdd(&acc[kbase - k0], cs);
  }
}

// rates of eight slots (one 16-byte block row of a link-list piece) into two partial sums
__device__ __forceinline__ void add_slots(const double *xs, uint4 q, double &v0, double &v1) {
  v0 += xs[q.x & 0xffffu];
  v1 += xs[q.x >> 16];
  v0 += xs[q.y & 0xffffu];
  v1 += xs[q.y >> 16];
  v0 += xs[q.z & 0xffffu];
  v1 += xs[q.z >> 16];
  v0 += xs[q.w & 0xffffu];
  v1 += xs[q.w >> 16];
}

// the sum v of a lane's piece of a group goes to acc at the piece's link: an atomic addition where the
// link has other pieces, else a plain one (no other lane of the workgroup adds to it in the chunk)
__device__ __forceinline__ void add_piece(unsigned lk, double v, double *acc) {
  if (lk == 0xffffu) return;
  const int e = (int)(lk & 0x7fffu);
  if (lk & 0x8000u)
    atomicAdd(&acc[e], v);
  else
    acc[e] += v;
}

// A chunk's link-list sums (Prob::lent): wavefront w of the scatter workgroup takes groups g0 + w,
// g0 + w + 16, ... of the chunk's groups [g0, g1), every block load of a group issued before the
// first is used; lane i sums the rates of piece i of a group.  (Two groups in flight at a time
// spilled registers in the two-paths-per-lane kernel and ran slower.)
__device__ __forceinline__ void list_sums(const Prob &p, int g0, int g1, const double *xs, double *acc) {
  constexpr int NB = kPieceLen / 8;
  const int lane = threadIdx.x & 63;
  for (int g = g0 + (threadIdx.x >> 6); g < g1; g += kScatWaves) {  // uniform in the wavefront
    const int2 gd = p.lgrp[g];
    const uint16_t *gh = p.lent + gd.x;
    const unsigned lk = gh[lane];
    const uint4 *gb = reinterpret_cast<const uint4 *>(gh + 64) + lane;
    uint4 q[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) q[b] = gb[64 * (b < gd.y ? b : 0)];
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b < gd.y) add_slots(xs, q[b], v0, v1);
    add_piece(lk, v0 + v1, acc);
  }
}

// ------------------------------------------------------------------------------------------
// Step a3 + a4: link loads by segmented FP64 sums over the CSC lists, capacity/consensus duals.
// Workgroup b owns a contiguous range of non-empty links holding ~nnz/nB CSC entries; each
// wavefront walks a contiguous part of it in coalesced rows of 64 entries, reduces runs of equal
// link inside the row with a segmented scan and adds one partial per run into an LDS FP64
// accumulator.  Also folds a slice of the demand kernel's partial sums into its row.
// ------------------------------------------------------------------------------------------
// Per-link penalties: the residual-balancing rule on link e's own residuals r_e (the change of its
// scaled duals, sqrt((1 + n_e)) |g' - g|) and s_e (the change of the rates of its paths,
// sqrt(sum_{r on e} (x'_r - x_r)^2)) moves w_e by C within [w_min, w_max]; the new g is divided by
// the same factor (q is a rate offset and keeps its value).  Returns the g to store.
__device__ __forceinline__ double per_link_rule(const Params &prm, double *w, int e, int ne, double gold,
                                                double gn, double sx2) {
  const double re = sqrt((double)(1 + ne) * ((gn - gold) * (gn - gold)));
  const double se = sqrt(sx2);
  const double we = w[e];
  double fe = 1.0;
  if (re > prm.A * se) {
    if (we * prm.C <= prm.w_max) fe = prm.C;
  } else if (se > prm.A * re) {
    if (we / prm.C >= prm.w_min) fe = 1.0 / prm.C;
  }
  if (fe == 1.0) return gn;
  w[e] = we * fe;
  return gn / fe;
}

__global__ __launch_bounds__(kLinkThreads) void k_link(Prob p, State s, const Params *prmp, int par) {
  const Params &prm = *prmp;
  __shared__ Ctrl cs;
  __shared__ double acc[kMaxLinksPerBlock];
  __shared__ double acc2[kMaxLinksPerBlock];  // per-link rule: sum of (x' - x)^2 over the link's paths
  __shared__ double fold[3];
  CtrlPrefetch cp;
  if (threadIdx.x < 64) prefetch_ctrl(s, par, cp);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bl = xcd_chunk(blockIdx.x, gridDim.x);
  const int4 wt = p.wtab[bl * kLinkWaves + w];
  const int k0 = p.blk[bl], k1 = p.blk[bl + 1];
  for (int k = threadIdx.x; k < k1 - k0; k += blockDim.x) acc[k] = 0.0;
  // the per-link values of this thread's first link and its slice of the demand kernel's
  // partial sums are loaded before the segmented sums, so their latency overlaps with them
  const int kf = k0 + threadIdx.x;
  int e_f = 0, ne_f = 0;
  double2 gq_f = make_double2(0.0, 0.0);
  double C_f = 1.0;
  if (kf < k1) {
    e_f = p.nzlink[kf];
    ne_f = p.nzptr[kf + 1] - p.nzptr[kf];
    gq_f = s.gq[e_f];
    C_f = p.Cn[e_f];
  }
  double a0 = 0.0, a1 = 0.0, a3 = -INFINITY;
  if (w == 1) {  // fold the demand kernel's per-wavefront rows b, b + nB, ... (fixed order)
    const double *pa = s.partA + (size_t)par * s.nArows * 4;
    for (int i = bl + lane * gridDim.x; i < s.nArows; i += 64 * gridDim.x) {
      a0 += pa[4 * i + 0];
      a1 += pa[4 * i + 1];
      a3 = fmax(a3, pa[4 * i + 3]);
    }
    a0 = wave_sum_d(a0);
    a1 = wave_sum_d(a1);
    a3 = wave_max_d(a3);
    if (lane == 0) {
      fold[0] = a0;
      fold[1] = a1;
      fold[2] = a3;
    }
  }
  __syncthreads();
  seg_rows_sum(p.lpf, (const double *)s.xo, k0, wt, acc);
  if (threadIdx.x < 64) finish_ctrl(cp, prm, &cs);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) publish_ctrl(s, cs, par);
  if (cs.stop) return;
  const bool rule = per_link_rule_now(prm, cs);  // uniform in the workgroup
  if (rule) {
    for (int k = threadIdx.x; k < k1 - k0; k += blockDim.x) acc2[k] = 0.0;
    __syncthreads();
    seg_rows_sum(p.lpf, (const double *)s.dx2, k0, wt, acc2);
    __syncthreads();
  }
  const double inv_f = cs.inv_f;
  double dr2 = 0.0, cap_v = -INFINITY;
  if (k1 - k0 <= 64) {
    // at most 64 links: the first wavefront updates them all and writes the workgroup's row
    // itself, without a second barrier
    if (threadIdx.x >= 64) return;
    if (kf < k1) {
      const double load = acc[kf - k0];
      const double gold = gq_f.x * inv_f;
      const double gn = fmax(gold + (load - C_f) / (double)(1 + ne_f), 0.0);
      const double gs = rule ? per_link_rule(prm, s.w, e_f, ne_f, gold, gn, acc2[kf - k0]) : gn;
      s.gqo[e_f] = make_double2(gs, gold - gn);
      dr2 = (double)(1 + ne_f) * (gn - gold) * (gn - gold);
      cap_v = (load - C_f) / C_f;
    }
    dr2 = wave_sum_d(dr2);
    cap_v = wave_max_d(cap_v);
    if (lane == 0) {
      double *o = s.partB + ((size_t)par * s.nB + bl) * 4;
      o[0] = fold[0];
      o[1] = dr2 + fold[1];
      o[2] = cap_v;
      o[3] = fold[2];
    }
    return;
  }
  for (int k = kf; k < k1; k += blockDim.x) {
    int e = e_f, ne = ne_f;
    double2 v = gq_f;
    double Ce = C_f;
    if (k != kf) {  // more links than threads
      e = p.nzlink[k];
      ne = p.nzptr[k + 1] - p.nzptr[k];
      v = s.gq[e];
      Ce = p.Cn[e];
    }
    const double load = acc[k - k0];
    const double gold = v.x * inv_f;
    const double gn = fmax(gold + (load - Ce) / (double)(1 + ne), 0.0);
    const double gs = rule ? per_link_rule(prm, s.w, e, ne, gold, gn, acc2[k - k0]) : gn;
    s.gqo[e] = make_double2(gs, gold - gn);
    dr2 += (double)(1 + ne) * (gn - gold) * (gn - gold);
    cap_v = fmax(cap_v, (load - Ce) / Ce);
  }
  const bool t0 = threadIdx.x == 0;
  block_partials(t0 ? fold[0] : 0.0, dr2 + (t0 ? fold[1] : 0.0), cap_v, t0 ? fold[2] : -INFINITY,
                 s.partB + ((size_t)par * s.nB + bl) * 4);
}

// ------------------------------------------------------------------------------------------
// Privatised link sums (instances with at most kMaxScatterLinks links).  One iteration =
//   k_demand_scatter: steps a1 + a2 as in the demand kernels above, and step a3 inside the
//                     workgroup: every path's new rate is added into the workgroup's own LDS copy of
//                     the E link loads (FP64 atomics in LDS, on the link ids already in registers
//                     from the gather), written out once as the workgroup's row of partial loads;
//   k_link_reduce:    per link, the sum of those rows in workgroup order, then step a4.
// Neither reads the link -> path list nor gathers a rate a second time.  A scatter workgroup runs
// spw passes over consecutive demands (kScatThreads / 2^logGp demands a pass), so there are few
// rows: one per workgroup.
// ------------------------------------------------------------------------------------------

// Link ids of one path as the gather read them, kept in registers for the scatter: the words of its
// hop record (H > 0), or its CSR range.
struct PathIds {
  uint2 w[kMaxHopSlots / 4];
  int i0, i1;
};

// Gathers of the scatter kernel: the loads of a path's hops inside the branches of a plain loop,
// which the compiler waits for one at a time.  The straight-line gathers above (several loads in
// flight) made this kernel spill: at 1,024 threads it has 128 registers a lane, and its time went up
// (1,000-node instance, 143 -> 159 us with two paths per lane).
__device__ __forceinline__ void gather_path_serial(const Prob &p, const State &s, int r, int ovf, double &sg,
                                                   double &sq, int &n) {
  sg = 0.0;
  sq = 0.0;
  if (p.H > 0) {
    uint2 w[kMaxHopSlots / 4];
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) w[q] = record_word(p, r, ovf, q);
    n = 0;
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) {
      const unsigned id[4] = {w[q].x & 0xffffu, w[q].x >> 16, w[q].y & 0xffffu, w[q].y >> 16};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (id[u] != 0xffffu) {
          const double2 v = s.gq[id[u]];
          sg += v.x;
          sq += v.y;
          ++n;
        }
    }
  } else {
    const int i0 = p.pptr[r], i1 = p.pptr[r + 1];
    n = i1 - i0;
    for (int ib = i0; ib < i1; ib += 8) {
      int e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = ib + u < i1 ? p.plinks[ib + u] : -1;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e[u] >= 0) {
          const double2 v = s.gq[e[u]];
          sg += v.x;
          sq += v.y;
        }
    }
  }
}

__device__ __forceinline__ void gather_ids(const Prob &p, const State &s, int r, int ovf, PathIds &id, double &sg,
                                           double &sq, int &n) {
  sg = 0.0;
  sq = 0.0;
  if (p.H > 0) {
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) id.w[q] = record_word(p, r, ovf, q);
    n = 0;
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) {
      const unsigned e4[4] = {id.w[q].x & 0xffffu, id.w[q].x >> 16, id.w[q].y & 0xffffu, id.w[q].y >> 16};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e4[u] != 0xffffu) {
          const double2 v = s.gq[e4[u]];
          sg += v.x;
          sq += v.y;
          ++n;
        }
    }
  } else {
    id.i0 = p.pptr[r];
    id.i1 = p.pptr[r + 1];
    n = id.i1 - id.i0;
    for (int ib = id.i0; ib < id.i1; ib += 8) {
      int e8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e8[u] = ib + u < id.i1 ? p.plinks[ib + u] : -1;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e8[u] >= 0) {
          const double2 v = s.gq[e8[u]];
          sg += v.x;
          sq += v.y;
        }
    }
  }
}

// acc[e] += v for every link e of path r, its link ids read again (from the caches: the gather
// read them in the same pass)
__device__ __forceinline__ void scatter_path(const Prob &p, int r, int ovf, double v, double *acc) {
  if (p.H > 0) {
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) {
      if (4 * q >= p.H + (ovf >= 0 ? p.H2 : 0)) break;
      const uint2 wq = record_word(p, r, ovf, q);
      const unsigned e4[4] = {wq.x & 0xffffu, wq.x >> 16, wq.y & 0xffffu, wq.y >> 16};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e4[u] != 0xffffu) atomicAdd(&acc[e4[u]], v);
    }
  } else {
    for (int i = p.pptr[r]; i < p.pptr[r + 1]; ++i) atomicAdd(&acc[p.plinks[i]], v);
  }
}

// acc[e] += v for every link e of the path
__device__ __forceinline__ void scatter_ids(const Prob &p, const PathIds &id, double v, double *acc) {
  if (p.H > 0) {
#pragma unroll
    for (int q = 0; q < kMaxHopSlots / 4; ++q) {
      const unsigned e4[4] = {id.w[q].x & 0xffffu, id.w[q].x >> 16, id.w[q].y & 0xffffu, id.w[q].y >> 16};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e4[u] != 0xffffu) atomicAdd(&acc[e4[u]], v);
    }
  } else {
    for (int i = id.i0; i < id.i1; ++i) atomicAdd(&acc[p.plinks[i]], v);
  }
}

// LISTS (link lists, p.cpp > 0): the new rates of a chunk of passes go to LDS, and after the chunk
// the workgroup sums them per link over the chunk's list (one LDS addition per piece of a link's
// run, not one per incidence).  Without: every incidence is an LDS atomic addition; KEEP: the
// gather's link ids stay in registers for it (one path per lane), or are read again (several paths
// per lane, where keeping them would spill).
template <int PPL, bool LISTS>
__global__ __launch_bounds__(kScatThreads) void k_demand_scatter(Prob p, State s, const Params *prmp, int par) {
  constexpr bool KEEP = PPL == 1 && !LISTS;
  const Params &prm = *prmp;
  // [E]: this workgroup's share of every link load; with link lists then [zslot + 1]: the new rates
  // of the current chunk's paths
  extern __shared__ double acc[];
  double *xs = acc + p.E;
  __shared__ Ctrl cs;
  CtrlPrefetch cp;
  const int t = threadIdx.x;
  if (t < 64) prefetch_ctrl(s, par, cp);
  for (int e = t; e < p.E; e += kScatThreads) acc[e] = 0.0;
  if (LISTS && t == 0) xs[p.zslot] = 0.0;
  const int logGp = p.logGp, Gp = 1 << logGp;
  const int lane = t & (Gp - 1);
  const int per = kScatThreads >> logGp;
  const int bl = xcd_chunk(blockIdx.x, gridDim.x);
  const int ps0 = bl * p.spw, ps1 = min(ps0 + p.spw, p.npass);
  double ds2 = 0.0, dr2 = 0.0, dem_v = -INFINITY;
  for (int ps = ps0; ps < ps1; ++ps) {  // bounds uniform in the workgroup
    const int c = ps * per + (t >> logGp);
    const int kc = LISTS ? (ps - ps0) / p.cpp : 0;                // the pass's chunk
    const int rlo = LISTS ? p.lchk[(size_t)bl * p.cpw + kc].z : 0;  // its first path
    int r0 = 0, np = 0;
    double Dc = 0.0, udc = 0.0, S0 = 0.0;
    double xr[PPL], ung[PPL], sg[PPL], sq[PPL];
    int n[PPL];
    PathIds ids[KEEP ? PPL : 1];
    unsigned on = 0u;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      xr[j] = ung[j] = sg[j] = sq[j] = 0.0;
      n[j] = 1;
    }
    int dv = -1;
    if (c < p.D) {
      Dc = p.Dn[c];
      udc = s.udem[c];
      S0 = s.S[c];
      r0 = p.dptr[c];
      np = p.dptr[c + 1] - r0;
      if (p.H2 > 0) dv = p.dovf[c];
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const int idx = lane + j * Gp;
        if (idx < np) {
          const int r = r0 + idx;
          on |= 1u << j;
          xr[j] = s.x[r];
          ung[j] = s.uneg[r];
          if (KEEP)
            gather_ids(p, s, r, overflow_record(dv, r, r0), ids[0], sg[j], sq[j], n[j]);
          else
            gather_path_serial(p, s, r, overflow_record(dv, r, r0), sg[j], sq[j], n[j]);
        }
      }
    }
    if (ps == ps0) {
      if (t < 64) finish_ctrl(cp, prm, &cs);
      __syncthreads();  // the decision, and the zeroed accumulators
      if (cs.stop) return;
    }
    if (c < p.D) {
      const double inv_f = cs.inv_f;
      LaneN<PPL> L;
      L.on = on;
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const bool oj = (on >> j) & 1u;
        L.a[j] = oj ? (double)n[j] * xr[j] - (sg[j] * inv_f - sq[j]) : 0.0;
        L.un[j] = ung[j] * inv_f;
        L.n[j] = (double)n[j];
        L.rn[j] = 1.0 / (double)n[j];
        L.rn1[j] = 1.0 / (double)(n[j] + 1);
      }
      Dem dm;
      dm.D = Dc;
      dm.u = udc * inv_f;
      dm.alpha = cs.alpha;
      dm.binv = 1.0 / cs.beta;
      int steps;
      const double Sst = sum_root(S0, L, dm, Gp, &steps);
      const double h = h_of(Sst, dm);
      double xsum = 0.0;
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        if (!((on >> j) & 1u)) continue;
        const int r = r0 + lane + j * Gp;
        const double b = L.a[j] - h;
        const double xn = (b >= L.n[j] * L.un[j]) ? b * L.rn[j] : (b + L.un[j]) * L.rn1[j];
        const double un = fmax(L.un[j] - xn, 0.0);
        s.xo[r] = xn;
        s.unego[r] = un;
        if (LISTS)
          xs[r - rlo] = xn;
        else if (KEEP)
          scatter_ids(p, ids[0], xn, acc);
        else
          scatter_path(p, r, overflow_record(dv, r, r0), xn, acc);
        xsum += xn;
        ds2 += (xn - xr[j]) * (xn - xr[j]);
        dr2 += (un - L.un[j]) * (un - L.un[j]);
      }
      const double Ssum = group_sum_d(xsum, Gp);
      if (lane == 0) {
        const double ud = fmax(dm.u + Ssum - dm.D, 0.0);
        s.udemo[c] = ud;
        s.So[c] = Sst;
        dr2 += (ud - dm.u) * (ud - dm.u);
        dem_v = fmax(dem_v, (Ssum - dm.D) / dm.D);
      }
    }
    if (LISTS && ((ps - ps0) % p.cpp == p.cpp - 1 || ps == ps1 - 1)) {  // the chunk's last pass
      __syncthreads();  // the chunk's rates are in LDS
      const int4 ch = p.lchk[(size_t)bl * p.cpw + kc];
      list_sums(p, ch.x, ch.y, xs, acc);
      __syncthreads();  // and read, before the next chunk's overwrite them
    }
  }
  wave_partials(ds2, dr2, dem_v, s.partA + ((size_t)par * s.nA + bl) * (kScatThreads / 64) * 4);
  __syncthreads();  // every LDS addition done
  double *row = s.partL + (size_t)bl * p.E;
  for (int e = t; e < p.E; e += kScatThreads) row[e] = acc[e];
}

// Step a3 across workgroups + step a4: workgroup b owns links 64 b .. 64 b + 63; wavefront w sums
// rows w, w + 16, ... of the partial loads (eight loads in flight), the per-wavefront sums are added
// in wavefront order, and the first wavefront updates the links' duals and writes the workgroup's
// row of partial sums.  Also folds a slice of the scatter kernel's per-wavefront rows into that row.
__global__ __launch_bounds__(kLinkThreads) void k_link_reduce(Prob p, State s, const Params *prmp, int par) {
  const Params &prm = *prmp;
  __shared__ Ctrl cs;
  __shared__ double red[kLinkWaves][64];
  __shared__ double fold[3];
  CtrlPrefetch cp;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  if (t < 64) prefetch_ctrl(s, par, cp);
  const int bl = xcd_chunk(blockIdx.x, gridDim.x);
  const int e = bl * 64 + lane;
  const bool in = e < p.E;
  int ne = 0;
  double2 gq_f = make_double2(0.0, 0.0);
  double C_f = 1.0;
  if (w == 0 && in) {
    ne = p.lptr[e + 1] - p.lptr[e];
    gq_f = s.gq[e];
    C_f = p.Cn[e];
  }
  if (w == 1) {  // fold the scatter kernel's per-wavefront rows b, b + nB, ... (fixed order)
    double a0 = 0.0, a1 = 0.0, a3 = -INFINITY;
    const double *pa = s.partA + (size_t)par * s.nArows * 4;
    for (int i = bl + lane * gridDim.x; i < s.nArows; i += 64 * gridDim.x) {
      a0 += pa[4 * i + 0];
      a1 += pa[4 * i + 1];
      a3 = fmax(a3, pa[4 * i + 3]);
    }
    a0 = wave_sum_d(a0);
    a1 = wave_sum_d(a1);
    a3 = wave_max_d(a3);
    if (lane == 0) {
      fold[0] = a0;
      fold[1] = a1;
      fold[2] = a3;
    }
  }
  double a = 0.0;
  if (in) {
    const double *col = s.partL + e;
    int r = w;
    for (; r + 7 * kLinkWaves < p.nF; r += 8 * kLinkWaves) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[(size_t)(r + u * kLinkWaves) * p.E];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; r < p.nF; r += kLinkWaves) a += col[(size_t)r * p.E];
  }
  red[w][lane] = a;
  if (t < 64) finish_ctrl(cp, prm, &cs);
  __syncthreads();
  if (blockIdx.x == 0 && t == 0) publish_ctrl(s, cs, par);
  if (cs.stop || w != 0) return;
  double load = 0.0;
#pragma unroll
  for (int i = 0; i < kLinkWaves; ++i) load += red[i][lane];
  double dr2 = 0.0, cap_v = -INFINITY;
  if (in && ne > 0) {
    const double gold = gq_f.x * cs.inv_f;
    const double gn = fmax(gold + (load - C_f) / (double)(1 + ne), 0.0);
    s.gqo[e] = make_double2(gn, gold - gn);
    dr2 = (double)(1 + ne) * (gn - gold) * (gn - gold);
    cap_v = (load - C_f) / C_f;
  }
  dr2 = wave_sum_d(dr2);
  cap_v = wave_max_d(cap_v);
  if (lane == 0) {
    double *o = s.partB + ((size_t)par * s.nB + bl) * 4;
    o[0] = fold[0];
    o[1] = dr2 + fold[1];
    o[2] = cap_v;
    o[3] = fold[2];
  }
}

// Final control record: applies the decision pending after the last iteration.
__global__ void k_finish(State s, const Params *prmp, int last_par) {
  const Params &prm = *prmp;
  if (threadIdx.x < 64) {
    const Ctrl prev = s.ctrl[last_par];
    double v[4] = {0.0, 0.0, -INFINITY, -INFINITY};
    if (prev.pending) {
      const double *pb = s.partB + (size_t)last_par * s.nB * 4;
      for (int i = threadIdx.x; i < s.nB; i += 64) {
        v[0] += pb[4 * i + 0];
        v[1] += pb[4 * i + 1];
        v[2] = fmax(v[2], pb[4 * i + 2]);
        v[3] = fmax(v[3], pb[4 * i + 3]);
      }
      v[0] = wave_sum_d(v[0]);
      v[1] = wave_sum_d(v[1]);
      v[2] = wave_max_d(v[2]);
      v[3] = wave_max_d(v[3]);
    }
    if (threadIdx.x == 0) {
      const Ctrl fin = decide(prev, v, prm);
      s.ctrl[2] = fin;
      if (s.log && fin.k >= 1 && fin.k <= s.log_cap) {  // residuals of the last iteration
        s.log[2 * s.log_cap + fin.k - 1] = fin.r;
        s.log[3 * s.log_cap + fin.k - 1] = fin.s;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Algorithm 2 on the graph engine.  FP64 loads and trims; final rates rounded toward zero.
// ------------------------------------------------------------------------------------------
// clamp at zero (step 1) and demand sums
__global__ void kp_clamp_sums(Prob p, State s, ProjBuf b) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    double sum = 0.0;
    for (int r = p.dptr[c]; r < p.dptr[c + 1]; ++r) {
      const double v = fmax((double)s.x[r], 0.0);
      b.xd[r] = v;
      sum += v;
      b.trim[r] = 0ull;
    }
    b.S[c] = sum;
  }
}

// step 1 on caller rates (caller units): clamp into the working copy in normalised units
__global__ void kp_clamp_sums_in(Prob p, const float *x_in, double scale, ProjBuf b) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    if (p.dscale) scale = p.dscale[c];
    double sum = 0.0;
    for (int r = p.dptr[c]; r < p.dptr[c + 1]; ++r) {
      const double v = fmax((double)x_in[r] / scale, 0.0);
      b.xd[r] = v;
      sum += v;
      b.trim[r] = 0ull;
    }
    b.S[c] = sum;
  }
}

// one wavefront per link; lane l sums entries l, l + 64, ... in that order, four entries' loads
// issued together
__global__ void kp_loads(Prob p, ProjBuf b) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int e = w; e < p.E; e += nw) {
    double acc = 0.0;
    const int j1 = p.lptr[e + 1];
    for (int j = p.lptr[e] + lane; j < j1; j += 256) {
      int r[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) r[u] = j + 64 * u < j1 ? p.lpaths[j + 64 * u] : -1;
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = r[u] >= 0 ? b.xd[r[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (r[u] >= 0) acc += v[u];
    }
    acc = wave_sum_d(acc);
    if (lane == 0) b.L[e] = acc;
  }
}

// C_p = number of violated links on p, and the log score
// alpha of the scores: the solve's final alpha (fin) or, with fin null, the given one
// one lane per path (G lanes per demand, as in the demand kernel): the number of violated links on
// the path and its log score
__global__ void kp_counts(Prob p, ProjBuf b, const Ctrl *fin, double alpha_in) {
  const float alpha = (float)(fin ? fin->alpha : alpha_in);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = t >> p.logG, lane = t & (p.G - 1);
  if (c >= p.D) return;
  const int r0 = p.dptr[c];
  if (lane >= p.dptr[c + 1] - r0) return;
  const int r = r0 + lane;
  int k = 0;
  for (int i = p.pptr[r]; i < p.pptr[r + 1]; ++i) {
    const int e = p.plinks[i];
    k += b.L[e] > p.Cn[e];
  }
  b.Cp[r] = k;
  b.lsc[r] = log_score(b.S[c], k, alpha);
}

// step 3: per demand, trim the excess over D_c from paths in descending score
// (S_c is common to the demand's paths: the order is by C_p, ties to the higher index)
__global__ void kp_demand_trim(Prob p, ProjBuf b) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    double excess = b.S[c] - (double)p.Dn[c];
    if (!(excess > 0.0)) continue;
    const int r0 = p.dptr[c], r1 = p.dptr[c + 1];
    // selection by repeated arg-max over at most 64 paths
    uint64_t done = 0ull;
    for (int it = 0; it < r1 - r0 && excess > 0.0; ++it) {
      int best = -1;
      for (int r = r0; r < r1; ++r) {
        if (done >> (r - r0) & 1ull) continue;
        if (best < 0 || trim_key(b.lsc[r], r) > trim_key(b.lsc[best], best)) best = r;
      }
      done |= 1ull << (best - r0);
      const double d = fmin(excess, b.xd[best]);
      b.xd[best] -= d;
      excess -= d;
    }
    double sum = 0.0;
    for (int r = r0; r < r1; ++r) sum += b.xd[r];
    b.S[c] = sum;
  }
}

// step 5: one workgroup per link; every link trims from the same snapshot: the paths above
// the threshold key K* (the key at which the descending cumulative rate reaches V_e) give up
// all their rate, the path at K* the remainder; a path trimmed by several links keeps the max.
__global__ __launch_bounds__(256) void kp_link_trim(Prob p, ProjBuf b) {
  __shared__ double red[4];
  __shared__ uint64_t kred[4];
  __shared__ double xred[4];
  __shared__ uint64_t keyT;
  __shared__ unsigned long long aboveT;
  __shared__ unsigned long long hist[256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = blockIdx.x; e < p.E; e += gridDim.x) {
    const double V = b.L[e] - p.Cn[e];
    if (!(V > 0.0)) continue;  // uniform in the workgroup
    const int j0 = p.lptr[e], j1 = p.lptr[e + 1];
    // fast path: the path with the largest key usually absorbs the whole violation
    uint64_t km = 0ull;
    double xm = 0.0;
    for (int j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      const int r = p.lpaths[j];
      const uint64_t k = trim_key(b.lsc[r], r);
      if (k > km) {
        km = k;
        xm = b.xd[r];
      }
    }
    for (int m = 1; m < 64; m <<= 1) {
      const uint64_t ko = __shfl_xor(km, m, 64);
      const double xo = __shfl_xor(xm, m, 64);
      if (ko > km) {
        km = ko;
        xm = xo;
      }
    }
    if (lane == 0) {
      kred[w] = km;
      xred[w] = xm;
    }
    __syncthreads();
    km = kred[0];
    xm = xred[0];
    for (int i = 1; i < 4; ++i)
      if (kred[i] > km) {
        km = kred[i];
        xm = xred[i];
      }
    __syncthreads();
    if (xm >= V) {
      if (threadIdx.x == 0) {
        const int r = (int)(uint32_t)(km & 0xffffffffull);
        atomicMax((unsigned long long *)&b.trim[r], (unsigned long long)__double_as_longlong(V));
      }
      continue;
    }
    // general case: threshold key K* where the descending cumulative rate reaches V,
    // f(T) = sum of x over incidences with key >= T; the largest T with f(T) >= V.  Radix
    // selection from the top byte down: per pass a 256-bucket histogram of the rates of the keys
    // that share the bytes chosen so far, summed in 64-bit fixed point (exact and independent
    // of the order of the atomic adds, so the choice is deterministic); scale 2^sh with
    // L_e * 2^sh < 2^62, so no partial sum overflows.
    int ex2;
    (void)frexp(b.L[e], &ex2);
    const int sh = 62 - ex2;
    const unsigned long long Vq = (unsigned long long)ceil(ldexp(V, sh));
    uint64_t prefix = 0ull;
    unsigned long long above_q = 0ull;
    for (int pass = 0; pass < 8; ++pass) {
      const int shift = 56 - 8 * pass;
      const uint64_t hmask = pass == 0 ? 0ull : (~0ull << (shift + 8));  // bytes chosen so far
      hist[threadIdx.x] = 0ull;  // blockDim.x == 256
      __syncthreads();
      for (int j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
        const int r = p.lpaths[j];
        const uint64_t k = trim_key(b.lsc[r], r);
        if (((k ^ prefix) & hmask) == 0ull)
          atomicAdd(&hist[(k >> shift) & 255ull], (unsigned long long)ldexp(b.xd[r], sh));
      }
      __syncthreads();
      if (w == 0) {
        // lane l holds digits 255-4l .. 252-4l, i.e. the buckets in descending digit order
        unsigned long long hv[4], tot = 0ull;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hv[i] = hist[255 - 4 * lane - i];
          tot += hv[i];
        }
        unsigned long long inc = tot;  // inclusive prefix over lanes (higher digits first)
        for (int d = 1; d < 64; d <<= 1) {
          const unsigned long long y = __shfl_up(inc, d, 64);
          if (lane >= d) inc += y;
        }
        unsigned long long cum = above_q + (inc - tot);  // rate of the keys above this lane's digits
        int dig = -1;
        unsigned long long cum_at = 0ull;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (dig < 0 && cum + hv[i] >= Vq) {
            dig = 255 - 4 * lane - i;
            cum_at = cum;
          }
          cum += hv[i];
        }
        const uint64_t hit = __ballot(dig >= 0);
        const int src = hit ? __ffsll((unsigned long long)hit) - 1 : 63;
        if (!hit && lane == 63) {  // rounding left f(0) below V: digit 0, all higher digits above
          dig = 0;
          cum_at = above_q + (inc - hv[3]);
        }
        if (lane == src) {
          keyT = prefix | ((uint64_t)dig << shift);
          aboveT = cum_at;
        }
      }
      __syncthreads();
      prefix = keyT;
      above_q = aboveT;
      __syncthreads();
    }
    const uint64_t T = prefix;
    double acc = 0.0;
    for (int j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      const int r = p.lpaths[j];
      if (trim_key(b.lsc[r], r) > T) acc += b.xd[r];
    }
    acc = wave_sum_d(acc);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    const double above = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    for (int j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      const int r = p.lpaths[j];
      const uint64_t k = trim_key(b.lsc[r], r);
      double d = 0.0;
      if (k > T) d = b.xd[r];
      else if (k == T) d = fmin(b.xd[r], fmax(V - above, 0.0));
      if (d > 0.0) atomicMax((unsigned long long *)&b.trim[r], (unsigned long long)__double_as_longlong(d));
    }
    __syncthreads();
  }
}

// step 6 and outputs in caller units.  Projected rates are rounded toward zero (the FP32 rates stay
// feasible) and S is the sum of the returned rates; unprojected rates are rounded to nearest and S
// is their FP64 sum rounded once (the rates of a demand may have either sign before the projection,
// so a sum of rounded rates could lose the small sums to cancellation).
__global__ void kp_output(Prob p, ProjBuf b, float *x_out, float *S_out, double scale, int project, const double *xs) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    if (p.dscale) scale = p.dscale[c];
    double sum = 0.0;
    for (int r = p.dptr[c]; r < p.dptr[c + 1]; ++r) {
      if (project) {
        double v = b.xd[r] - __longlong_as_double((long long)b.trim[r]);
        v = fmax(v, 0.0) * scale;
        x_out[r] = __double2float_rz(v);
        sum += (double)x_out[r];
      } else {
        x_out[r] = (float)(xs[r] * scale);
        sum += xs[r];
      }
    }
    if (S_out) S_out[c] = project ? (float)sum : (float)(sum * scale);
  }
}

// the FP64 rates (and sums) of the state, caller units
__global__ void k_get_state(Prob p, State s, double scale, double *x_out, double *S_out) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    if (p.dscale) scale = p.dscale[c];
    double sum = 0.0;
    for (int r = p.dptr[c]; r < p.dptr[c + 1]; ++r) {
      x_out[r] = s.x[r] * scale;
      sum += s.x[r];
    }
    if (S_out) S_out[c] = sum * scale;
  }
}

hipError_t launch_get_state(const Prob &p, const State &s, double scale, double *x_out, double *S_out,
                            hipStream_t st) {
  int blocks = (p.D + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_get_state, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, p, s, scale, x_out, S_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Workgroup engine: the whole solve of one instance inside one workgroup, state in LDS.
// ------------------------------------------------------------------------------------------
// PPL: paths per lane in the demand step.  A demand with G path slots gets G / PPL lanes (at least
// one), each holding up to PPL of its paths; fewer lanes per demand share the per-demand work of the
// root solve (bracket, Newton step, S^-alpha) between fewer lanes and need fewer group sums.
template <int NT, int PPL>
__global__ __launch_bounds__(NT) void k_block_solve(const BatchDesc *descs, Pools pools,
                                                               const Params *prmp, int project, float *x_out,
                                                               float *S_out, BatchOut *outs) {
  const Params &prm = *prmp;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Ctrl cs;
  __shared__ double red[4][16];
  const BatchDesc d = descs[blockIdx.x];
  const int E = d.E, P = d.P, D = d.D, nnz = d.nnz, logG = d.logG;
  // LDS layout
  double2 *gq = (double2 *)smem;                     // E
  double *Cn = (double *)(gq + E);                   // E
  double *Lx = Cn + E;                               // E  (loads, FP64)
  double *udem = Lx + E;                             // D
  double *S = udem + D;                              // D
  double *x = S + D;                                 // P
  double *uneg = x + P;                              // P
  double *Dn = uneg + P;                             // D
  // 16-bit indices (the host admits only instances with P < 2^15 and nnz, E, D < 2^16 here)
  double *Sp = Dn + D;                               // D: the root before the last one
  uint16_t *pptr = (uint16_t *)(Sp + D);             // P + 1
  uint16_t *plinks = pptr + P + 1;                   // nnz
  uint16_t *dptr = plinks + nnz;                     // D + 1
  uint16_t *lptr = dptr + D + 1;                     // E + 1
  uint16_t *lpf = lptr + E + 1;                      // nnz: CSC path ids, bit 15 on a link's first entry
  uint16_t *nzl = lpf + nnz;                         // non-empty links in order
  const int tid = threadIdx.x, nth = NT;
  const int32_t *gi = pools.i32;
  for (int i = tid; i <= P; i += nth) pptr[i] = (uint16_t)gi[d.off_pptr + i];
  for (int i = tid; i < nnz; i += nth) plinks[i] = (uint16_t)gi[d.off_plinks + i];
  for (int i = tid; i <= D; i += nth) dptr[i] = (uint16_t)gi[d.off_dptr + i];
  for (int i = tid; i <= E; i += nth) lptr[i] = (uint16_t)gi[d.off_lptr + i];
  for (int i = tid; i < nnz; i += nth) {
    const int32_t v = gi[d.off_lpf + i];
    lpf[i] = (uint16_t)((v & 0x7fff) | (v < 0 ? 0x8000 : 0));
  }
  for (int i = tid; i < d.nzl; i += nth) nzl[i] = (uint16_t)gi[d.off_nzl + i];
  for (int i = tid; i < E; i += nth) {
    Cn[i] = pools.Cn[d.off_E + i];
    gq[i] = make_double2(0.0, 0.0);
  }
  for (int i = tid; i < D; i += nth) Dn[i] = pools.Dn[d.off_D + i];
  __syncthreads();
  const double inv_scale = 1.0 / d.scale;
  for (int c = tid; c < D; c += nth) {
    const int r0 = dptr[c], r1 = dptr[c + 1];
    double sum = 0.0;
    for (int r = r0; r < r1; ++r) {
      const double v = pools.x0 ? (double)pools.x0[d.off_P + r] * inv_scale : Dn[c] / (double)(r1 - r0);
      x[r] = v;
      uneg[r] = 0.0;
      sum += v;
    }
    udem[c] = 0.0;
    S[c] = sum;
    Sp[c] = sum;
  }
  if (tid == 0) cs = initial_ctrl(prm);
  __syncthreads();

  constexpr int kLogPPL = PPL >= 8 ? 3 : PPL >= 4 ? 2 : PPL >= 2 ? 1 : 0;
  const int logGp = logG > kLogPPL ? logG - kLogPPL : 0;  // lanes per demand: Gp = G / PPL, at least 1
  const int Gp = 1 << logGp;
  const int lane = tid & (Gp - 1);
  const int groups = nth >> logGp;
  const int w = tid >> 6, l64 = tid & 63, nw = nth >> 6;
  // link step: Lg lanes per non-empty link (a power of two, about NT / #links, at most 64)
  int logLg = 0;
  while (logLg < 6 && (d.nzl << (logLg + 1)) <= nth) ++logLg;
  const int Lg = 1 << logLg, lg = tid & (Lg - 1), links_per_pass = nth >> logLg;
  while (!cs.stop) {
    const double inv_f = cs.inv_f;
    Dem dm;
    dm.alpha = cs.alpha;
    dm.binv = 1.0 / cs.beta;
    double ds2 = 0.0, dr2 = 0.0, dem_v = -INFINITY, cap_v = -INFINITY;
    // demand step
    for (int c0 = 0; c0 < D; c0 += groups) {
      const int c = c0 + (tid >> logGp);
      if (c < D) {
        const int r0 = dptr[c], np = dptr[c + 1] - r0;
        LaneN<PPL> L;
        L.on = 0u;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const int idx = lane + j * Gp;
          int n = 1;
          L.a[j] = 0.0;
          L.un[j] = 0.0;
          if (idx < np) {
            const int r = r0 + idx;
            const int i0 = pptr[r], i1 = pptr[r + 1];
            n = i1 - i0;
            double sg = 0.0, sq = 0.0;
            for (int i = i0; i < i1; ++i) {
              const double2 v = gq[plinks[i]];
              sg += v.x;
              sq += v.y;
            }
            L.a[j] = (double)n * x[r] - (sg * inv_f - sq);
            L.un[j] = uneg[r] * inv_f;
            L.on |= 1u << j;
          }
          L.n[j] = (double)n;
          L.rn[j] = 1.0 / (double)n;
          L.rn1[j] = 1.0 / (double)(n + 1);
        }
        dm.D = Dn[c];
        dm.u = udem[c] * inv_f;
        int steps;
        const double Sk = S[c];
        // the root solve starts from the linear extrapolation of the last two roots (fewer
        // evaluations than from the last root: with up to 64 demands per wavefront the slowest
        // demand decides a wavefront's time)
        double Sstart = Sk + (Sk - Sp[c]);
        if (dm.alpha > 0.0 && !(Sstart > 0.0)) Sstart = Sk;
        const double Sst = sum_root(Sstart, L, dm, Gp, &steps);
        const double h = h_of(Sst, dm);
        double xsum = 0.0;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          if (!((L.on >> j) & 1u)) continue;
          const int r = r0 + lane + j * Gp;
          const double b = L.a[j] - h;
          const double xn = (b >= L.n[j] * L.un[j]) ? b * L.rn[j] : (b + L.un[j]) * L.rn1[j];
          const double xr = x[r];
          const double un = fmax(L.un[j] - xn, 0.0);
          x[r] = xn;
          uneg[r] = un;
          xsum += xn;
          ds2 += (xn - xr) * (xn - xr);
          dr2 += (un - L.un[j]) * (un - L.un[j]);
        }
        const double Ssum = group_sum_d(xsum, Gp);
        if (lane == 0) {
          const double ud = fmax(dm.u + Ssum - dm.D, 0.0);
          udem[c] = ud;
          Sp[c] = Sk;
          S[c] = Sst;
          dr2 += (ud - dm.u) * (ud - dm.u);
          dem_v = fmax(dem_v, (Ssum - dm.D) / dm.D);
        }
      }
    }
    __syncthreads();
    // link step: each group of Lg lanes sums the new rates over one link's CSC entries (lane i
    // takes entries i, i + Lg, ...; the group's sum by DPP butterflies, so the order is fixed), then
    // the group's first lane updates the link's duals
    for (int k0 = 0; k0 < d.nzl; k0 += links_per_pass) {
      const int k = k0 + (tid >> logLg);
      double load = 0.0;
      int e = 0, ne = 0;
      if (k < d.nzl) {
        e = nzl[k];
        const int j0 = lptr[e], j1 = lptr[e + 1];
        ne = j1 - j0;
#pragma unroll 4
        for (int j = j0 + lg; j < j1; j += Lg) load += x[csc_path(lpf[j])];
      }
      load = group_sum_d(load, Lg);
      if (k < d.nzl && lg == 0) {
        const double2 v = gq[e];
        const double gold = v.x * inv_f;
        const double gn = fmax(gold + (load - Cn[e]) / (double)(1 + ne), 0.0);
        gq[e] = make_double2(gn, gold - gn);
        dr2 += (double)(1 + ne) * (gn - gold) * (gn - gold);
        cap_v = fmax(cap_v, (load - Cn[e]) / Cn[e]);
      }
    }
    // partial sums and decision
    ds2 = wave_sum_d(ds2);
    dr2 = wave_sum_d(dr2);
    cap_v = wave_max_d(cap_v);
    dem_v = wave_max_d(dem_v);
    if (l64 == 0) {
      red[0][w] = ds2;
      red[1][w] = dr2;
      red[2][w] = cap_v;
      red[3][w] = dem_v;
    }
    __syncthreads();
    if (tid == 0) {
      double v[4] = {0.0, 0.0, -INFINITY, -INFINITY};
      for (int i = 0; i < nw; ++i) {
        v[0] += red[0][i];
        v[1] += red[1][i];
        v[2] = fmax(v[2], red[2][i]);
        v[3] = fmax(v[3], red[3][i]);
      }
      Ctrl c = cs;
      c.pending = 1;
      const Ctrl nc = decide(c, v, prm);
      if (pools.log && blockIdx.x == 0 && c.k < pools.log_cap) {  // this iteration's beta, alpha, r, s
        const int L = pools.log_cap;
        pools.log[c.k] = c.beta;
        pools.log[L + c.k] = c.alpha;
        pools.log[2 * L + c.k] = nc.r;
        pools.log[3 * L + c.k] = nc.s;
      }
      cs = nc;
    }
    __syncthreads();
  }

  // ---------------- Algorithm 2 (if requested) ----------------
  // x (LDS) holds the working rates; per-path log scores (FP32 values) go to uneg; per-path trims of the
  // link phase are combined by max in x_out (float bits of non-negative values).
  const float alpha = (float)cs.alpha;
  float *xo = x_out + d.off_P;
  for (int r = tid; r < P; r += nth) xo[r] = 0.f;
  if (project) {
    for (int r = tid; r < P; r += nth) x[r] = fmax(x[r], 0.0);
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int e = w; e < E; e += nw) {
        double acc = 0.0;
        for (int j = lptr[e] + l64; j < lptr[e + 1]; j += 64) acc += x[csc_path(lpf[j])];
        acc = wave_sum_d(acc);
        if (l64 == 0) Lx[e] = acc;
      }
      __syncthreads();
      for (int c = tid; c < D; c += nth) {
        double sum = 0.0;
        for (int r = dptr[c]; r < dptr[c + 1]; ++r) sum += x[r];
        for (int r = dptr[c]; r < dptr[c + 1]; ++r) {
          int k = 0;
          for (int i = pptr[r]; i < pptr[r + 1]; ++i) k += Lx[plinks[i]] > Cn[plinks[i]];
          uneg[r] = log_score(sum, k, alpha);
        }
        if (pass == 0) {
          // demand phase: trim the excess over D_c in descending score
          const int r0 = dptr[c], r1 = dptr[c + 1];
          double excess = sum - Dn[c];
          uint64_t done = 0ull;
          for (int it = 0; it < r1 - r0 && excess > 0.0; ++it) {
            int best = -1;
            for (int r = r0; r < r1; ++r) {
              if (done >> (r - r0) & 1ull) continue;
              if (best < 0 || trim_key((float)uneg[r], r) > trim_key((float)uneg[best], best)) best = r;
            }
            done |= 1ull << (best - r0);
            const double dd = fmin(excess, x[best]);
            x[best] = x[best] - dd;
            excess -= dd;
          }
        }
      }
      __syncthreads();
    }
    // link phase: every violated link trims from the same snapshot, one wavefront per link,
    // X_before(p) = rate of the link's paths with a larger key; a path keeps the largest trim
    for (int e = w; e < E; e += nw) {
      const double V = Lx[e] - Cn[e];
      if (!(V > 0.0)) continue;
      const int j0 = lptr[e], j1 = lptr[e + 1];
      for (int j = j0 + l64; j < j1; j += 64) {
        const int r = csc_path(lpf[j]);
        const uint64_t kr = trim_key((float)uneg[r], r);
        double before = 0.0;
        for (int i = j0; i < j1; ++i) {
          const int q = csc_path(lpf[i]);
          if (trim_key((float)uneg[q], q) > kr) before += x[q];
        }
        const double dd = fmin(x[r], fmax(V - before, 0.0));
        // rounded up, so that the FP32 trim removes at least the link's share of the excess
        if (dd > 0.0) atomicMax((unsigned int *)&xo[r], __float_as_uint(__double2float_ru(dd)));
      }
    }
  }
  __syncthreads();
  // outputs: x_out holds the per-path trims (float bits, non-negative) when projecting
  const double scale = d.scale;
  for (int c = tid; c < D; c += nth) {
    double sum = 0.0;
    for (int r = dptr[c]; r < dptr[c + 1]; ++r) {
      double v = x[r];
      if (project) v = fmax(v - (double)xo[r], 0.0);
      const float o = project ? __double2float_rz(v * scale) : (float)(v * scale);
      xo[r] = o;
      sum += project ? (double)o : v;  // unprojected: the FP64 sum, rounded once (as kp_output)
    }
    if (S_out) S_out[d.off_D + c] = project ? (float)sum : (float)(sum * scale);
  }
  if (tid == 0) {
    BatchOut o;
    o.beta = cs.beta;
    o.alpha = cs.alpha;
    o.r = cs.r;
    o.s = cs.s;
    o.cap_viol = cs.cap_viol;
    o.dem_viol = cs.dem_viol;
    o.iters = cs.k;
    o.flags = cs.flags;
    o.stop_iter = cs.stop_iter;
    o.pad = 0;
    outs[blockIdx.x] = o;
  }
}

// ------------------------------------------------------------------------------------------
// Reverse pass of one iteration (vector-Jacobian product, FP64), schedule and unit scale fixed.
// fin: state at the start of iteration k, fout: state after it; rho: rescale of the scaled duals
// at the start of iteration k.  Every [.]_+ differentiates on the branch taken; the root S* of the
// sum equation through the implicit function theorem (dS* = -F_theta / F_S).
// Inputs: a = adjoints of iteration k's outputs; outputs: adjoints of its inputs (in place).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_adj_demand(Prob p, FwdState fin, FwdState fout, AdjState a,
                                                         double beta, double alpha, double rho) {
  const int G = p.G;
  const int t = threadIdx.x;
  const int lane = t & (G - 1);
  const int c = xcd_chunk(blockIdx.x, gridDim.x) * (kThreads >> p.logG) + (t >> p.logG);
  if (c >= p.D) return;  // uniform in the lane group
  const int r0 = p.dptr[c], np = p.dptr[c + 1] - r0;
  const bool on = lane < np;
  const int r = r0 + (on ? lane : 0);
  int n = 1;
  double sg = 0.0, sq = 0.0, lb = 0.0;
  if (on) {
    const int i0 = p.pptr[r], i1 = p.pptr[r + 1];
    n = i1 - i0;
    for (int i = i0; i < i1; ++i) {
      const int e = p.plinks[i];
      const double2 v = fin.gq[e];
      sg += v.x;
      sq += v.y;
      // link step adjoint: t_e = g~_e + (load_e - C_e)/(1+n_e), g' = [t]_+, q' = g~ - g'
      const double tb = fout.gq[e].x > 0.0 ? (a.gb[e] - a.qb[e]) : 0.0;
      lb += tb / (double)(1 + (p.lptr[e + 1] - p.lptr[e]));
    }
  }
  const double Dc = (double)p.Dn[c];
  const double udt = fin.udem[c] * rho;
  const double unt = on ? (double)fin.uneg[r] * rho : 0.0;
  const double a_r = on ? (double)n * (double)fin.x[r] - (sg * rho - sq) : 0.0;
  double xb = on ? a.xb[r] + lb : 0.0;
  // dual updates: u_dem' = [u~ + S - D]_+, u_neg' = [u~ - x']_+
  const double v = fout.udem[c] > 0.0 ? a.udb[c] : 0.0;
  double untb = (on && fout.uneg[r] > 0.0) ? a.unb[r] : 0.0;
  xb -= untb;
  xb += v;  // S_c = sum x'_r
  double Dl = -v, udtb = v;
  // rate update x' = xi(a - h(S*)) and the implicit root
  const double Sst = fout.S[c];
  Dem dm;
  dm.D = Dc;
  dm.u = udt;
  dm.alpha = alpha;
  dm.binv = 1.0 / beta;
  const double tt = Sst - Dc + udt;
  const double mh = tt > 0.0 ? 1.0 : 0.0;
  const double invS = 1.0 / Sst;
  const double pw = pow_neg_alpha(Sst, invS, alpha);
  const double h = fmax(tt, 0.0) - pw * dm.binv;
  const double dh = mh + (alpha > 0.0 ? alpha * pw * dm.binv * invS : 0.0);
  const double b = a_r - h;
  const bool hib = b >= (double)n * unt;
  const double kap = on ? (hib ? 1.0 / n : 1.0 / (n + 1)) : 0.0;
  const double xu = on ? (hib ? 0.0 : 1.0 / (n + 1)) : 0.0;
  const double bb = xb * kap;
  untb += xb * xu;
  const double hb = -group_sum_d(bb, G);
  const double skap = group_sum_d(kap, G);
  double ab = bb;
  const double Sstb = hb * dh;
  Dl -= hb * mh;
  udtb += hb * mh;
  const double FS = -dh * skap - 1.0;
  const double mu = -Sstb / FS;
  ab += mu * kap;
  untb += mu * xu;
  Dl += mu * skap * mh;
  udtb -= mu * skap * mh;
  if (on) {
    a.ab[r] = ab;
    a.xb[r] = (double)n * ab;  // a_r = n_r x_r - ...
    a.unb[r] = rho * untb;
  }
  if (lane == 0) {
    a.udb[c] = rho * udtb;
    a.Db[c] += Dl;
  }
}

__global__ __launch_bounds__(kLinkThreads) void k_adj_link(Prob p, FwdState fout, AdjState a, double rho) {
  __shared__ double acc[kMaxLinksPerBlock];
  const int bl = xcd_chunk(blockIdx.x, gridDim.x);
  const int4 wt = p.wtab[bl * kLinkWaves + (threadIdx.x >> 6)];
  const int k0 = p.blk[bl], k1 = p.blk[bl + 1];
  for (int k = threadIdx.x; k < k1 - k0; k += blockDim.x) acc[k] = 0.0;
  __syncthreads();
  seg_rows_sum(p.lpf, a.ab, k0, wt, acc);
  __syncthreads();
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const int e = p.nzlink[k];
    const int ne = p.nzptr[k + 1] - p.nzptr[k];
    const double sa = acc[k - k0];
    const double tb = fout.gq[e].x > 0.0 ? (a.gb[e] - a.qb[e]) : 0.0;
    a.Cb[e] -= tb / (double)(1 + ne);
    const double gtb = tb + a.qb[e] - sa;  // g~ enters t, q' and (with minus) a_r
    a.gb[e] = rho * gtb;
    a.qb[e] = sa;
  }
}

// seed: adjoint of x^(K) from the cotangent on S^(K) = sum_r x_r; zero everything else
__global__ void k_adj_seed(Prob p, AdjState a, const float *dS) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    for (int r = p.dptr[c]; r < p.dptr[c + 1]; ++r) {
      a.xb[r] = (double)dS[c];
      a.unb[r] = 0.0;
      a.ab[r] = 0.0;
    }
    a.udb[c] = 0.0;
    a.Db[c] = 0.0;
  }
  for (int e = tid; e < p.E; e += nth) {
    a.gb[e] = 0.0;
    a.qb[e] = 0.0;
    a.Cb[e] = 0.0;
  }
}

// x^0_r = D_c / |P_c| (cold start): dD_c += sum_r xb_r / |P_c|
__global__ void k_adj_x0(Prob p, AdjState a) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  for (int c = tid; c < p.D; c += nth) {
    const int r0 = p.dptr[c], r1 = p.dptr[c + 1];
    double acc = 0.0;
    for (int r = r0; r < r1; ++r) acc += a.xb[r];
    a.Db[c] += acc / (double)(r1 - r0);
  }
}

hipError_t launch_adj_seed(const Prob &p, const AdjState &a, const float *dS, hipStream_t st) {
  int n = p.D > p.E ? p.D : p.E;
  int blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_adj_seed, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, p, a, dS);
  return hipGetLastError();
}

hipError_t launch_adj_iteration(const Prob &p, int nB, const FwdState &fin, const FwdState &fout,
                                const AdjState &a, double beta, double alpha, double rho, hipStream_t st) {
  const int nAdj = (p.D + (kThreads >> p.logG) - 1) / (kThreads >> p.logG);  // G lanes per demand
  hipLaunchKernelGGL(k_adj_demand, dim3(nAdj), dim3(kThreads), 0, st, p, fin, fout, a, beta, alpha, rho);
  hipLaunchKernelGGL(k_adj_link, dim3(nB), dim3(kLinkThreads), 0, st, p, fout, a, rho);
  return hipGetLastError();
}

hipError_t launch_adj_x0(const Prob &p, const AdjState &a, hipStream_t st) {
  int blocks = (p.D + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_adj_x0, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, p, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------------------------------
hipError_t launch_init(const Prob &p, const State &s, const Params *prm, const float *x0, double inv_scale,
                       hipStream_t st) {
  int n = p.D > p.E ? p.D : p.E;
  int blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, st, p, s, prm, x0, inv_scale);
  return hipGetLastError();
}

hipError_t launch_warm(const Prob &p, const State &s, const Params *prm, double rescale, hipStream_t st) {
  int n = p.P > p.E ? p.P : p.E;
  int blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_warm, dim3(blocks), dim3(256), 0, st, p, s, prm, rescale);
  return hipGetLastError();
}

// the demand kernel for the handle's paths per lane (p.ppl); with ev0/ev1 the events are attached
// to the dispatch itself (start and end of the kernel's execution), so their difference excludes
// the queueing of separate event packets
template <class K>
static void launch_demand_k(K kern, int threads, const Prob &p, const State &s, const Params *prm, int par,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL(kern, dim3(s.nA), dim3(threads), 0, st, ev0, ev1, 0, p, s, prm, par);
  else
    hipLaunchKernelGGL(kern, dim3(s.nA), dim3(threads), 0, st, p, s, prm, par);
}

template <class K>
static void launch_scatter_k(K kern, const Prob &p, const State &s, const Params *prm, int par, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev1) {
  const size_t lds = sizeof(double) * ((size_t)p.E + (p.cpp > 0 ? (size_t)p.zslot + 1 : 0));
  if (ev0)
    hipExtLaunchKernelGGL(kern, dim3(p.nF), dim3(kScatThreads), lds, st, ev0, ev1, 0, p, s, prm, par);
  else
    hipLaunchKernelGGL(kern, dim3(p.nF), dim3(kScatThreads), lds, st, p, s, prm, par);
}

static void launch_demand_kernel(const Prob &p, const State &s, const Params *prm, int par, hipStream_t st,
                                 hipEvent_t ev0, hipEvent_t ev1) {
  if (p.lsum == kLinkSumsPrivate) {
    if (p.cpp > 0) {
      switch (p.ppl) {
        case 2: launch_scatter_k(k_demand_scatter<2, true>, p, s, prm, par, st, ev0, ev1); break;
        case 4: launch_scatter_k(k_demand_scatter<4, true>, p, s, prm, par, st, ev0, ev1); break;
        case 8: launch_scatter_k(k_demand_scatter<8, true>, p, s, prm, par, st, ev0, ev1); break;
        default: launch_scatter_k(k_demand_scatter<1, true>, p, s, prm, par, st, ev0, ev1);
      }
    } else {
      switch (p.ppl) {
        case 2: launch_scatter_k(k_demand_scatter<2, false>, p, s, prm, par, st, ev0, ev1); break;
        case 4: launch_scatter_k(k_demand_scatter<4, false>, p, s, prm, par, st, ev0, ev1); break;
        case 8: launch_scatter_k(k_demand_scatter<8, false>, p, s, prm, par, st, ev0, ev1); break;
        default: launch_scatter_k(k_demand_scatter<1, false>, p, s, prm, par, st, ev0, ev1);
      }
    }
    return;
  }
  switch (p.ppl) {
    case 2: launch_demand_k(k_demand_multi<2>, kThreads, p, s, prm, par, st, ev0, ev1); break;
    case 4: launch_demand_k(k_demand_multi<4>, kThreads, p, s, prm, par, st, ev0, ev1); break;
    case 8: launch_demand_k(k_demand_multi<8>, kThreads, p, s, prm, par, st, ev0, ev1); break;
    default: launch_demand_k(k_demand, kThreads + 64, p, s, prm, par, st, ev0, ev1);
  }
}

static void launch_link_kernel(const Prob &p, const State &s, const Params *prm, int par, hipStream_t st,
                               hipEvent_t ev0, hipEvent_t ev1) {
  if (p.lsum == kLinkSumsPrivate) {
    if (ev0)
      hipExtLaunchKernelGGL(k_link_reduce, dim3(s.nB), dim3(kLinkThreads), 0, st, ev0, ev1, 0, p, s, prm, par);
    else
      hipLaunchKernelGGL(k_link_reduce, dim3(s.nB), dim3(kLinkThreads), 0, st, p, s, prm, par);
  } else if (ev0) {
    hipExtLaunchKernelGGL(k_link, dim3(s.nB), dim3(kLinkThreads), 0, st, ev0, ev1, 0, p, s, prm, par);
  } else {
    hipLaunchKernelGGL(k_link, dim3(s.nB), dim3(kLinkThreads), 0, st, p, s, prm, par);
  }
}

// dynamic LDS of the privatised-sum demand kernels up to kScatLds bytes (above the default limit of
// a launch); once per process and device before their first launch
hipError_t prepare_scatter_kernels() {
  const int lds = kScatLds;
  const void *ks[] = {(const void *)k_demand_scatter<1, false>, (const void *)k_demand_scatter<2, false>,
                      (const void *)k_demand_scatter<4, false>, (const void *)k_demand_scatter<8, false>,
                      (const void *)k_demand_scatter<1, true>,  (const void *)k_demand_scatter<2, true>,
                      (const void *)k_demand_scatter<4, true>,  (const void *)k_demand_scatter<8, true>};
  for (const void *k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_iteration(const Prob &p, const State &s, const Params *prm, int par, hipStream_t st) {
  launch_demand_kernel(p, s, prm, par, st, nullptr, nullptr);
  launch_link_kernel(p, s, prm, par, st, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_demand_timed(const Prob &p, const State &s, const Params *prm, int par, hipStream_t st,
                               hipEvent_t ev0, hipEvent_t ev1) {
  launch_demand_kernel(p, s, prm, par, st, ev0, ev1);
  return hipGetLastError();
}

hipError_t launch_link_timed(const Prob &p, const State &s, const Params *prm, int par, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev1) {
  launch_link_kernel(p, s, prm, par, st, ev0, ev1);
  return hipGetLastError();
}

hipError_t launch_finish(const State &s, const Params *prm, int last_par, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, s, prm, last_par);
  return hipGetLastError();
}

// steps 2-5 of Algorithm 2 on the clamped working copy b.xd / b.S
static void launch_trims(const Prob &p, const ProjBuf &b, const Ctrl *fin, double alpha, hipStream_t st) {
  const int nD = (p.D + 255) / 256, nE = (p.E * 64 + 255) / 256;
  const int nC = (int)(((int64_t)p.D * p.G + 255) / 256);  // one lane per path slot
  hipLaunchKernelGGL(kp_loads, dim3(nE), dim3(256), 0, st, p, b);
  hipLaunchKernelGGL(kp_counts, dim3(nC), dim3(256), 0, st, p, b, fin, alpha);
  hipLaunchKernelGGL(kp_demand_trim, dim3(nD), dim3(256), 0, st, p, b);
  hipLaunchKernelGGL(kp_loads, dim3(nE), dim3(256), 0, st, p, b);
  hipLaunchKernelGGL(kp_counts, dim3(nC), dim3(256), 0, st, p, b, fin, alpha);
  int nl = p.E < 4096 ? p.E : 4096;
  hipLaunchKernelGGL(kp_link_trim, dim3(nl > 0 ? nl : 1), dim3(256), 0, st, p, b);
}

hipError_t launch_project(const Prob &p, const State &s, const ProjBuf &b, float *x_out, float *S_out,
                          double scale, int project, hipStream_t st) {
  const int nD = (p.D + 255) / 256;
  if (project) {
    hipLaunchKernelGGL(kp_clamp_sums, dim3(nD), dim3(256), 0, st, p, s, b);
    launch_trims(p, b, s.ctrl + 2, 0.0, st);
  }
  hipLaunchKernelGGL(kp_output, dim3(nD), dim3(256), 0, st, p, b, x_out, S_out, scale, project, s.x);
  return hipGetLastError();
}

// Scratch of te_project_rates_static, the entry point that allocates nothing: the projection's
// working arrays carved from one file-scope device array of kStaticScratchBytes.  Every GPU the
// library runs on holds its own copy until the process ends; all calls on one GPU share it (calls
// that overlap on one GPU race).  In host code `scratch` only names the array: its device address
// comes from hipGetSymbolAddress, once per device, kept in g_scratch.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {nullptr};
}  // namespace

// Device address and size of the current device's copy of the static scratch (looked up on the
// first call per device, with that device current).
hipError_t static_scratch(void **out, size_t *bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

// Algorithm 2 on caller rates x_in (caller units) at the given alpha; x_out may alias x_in
hipError_t launch_project_rates(const Prob &p, const ProjBuf &b, const float *x_in, double alpha, float *x_out,
                                float *S_out, double scale, hipStream_t st) {
  const int nD = (p.D + 255) / 256;
  hipLaunchKernelGGL(kp_clamp_sums_in, dim3(nD), dim3(256), 0, st, p, x_in, scale, b);
  launch_trims(p, b, nullptr, alpha, st);
  hipLaunchKernelGGL(kp_output, dim3(nD), dim3(256), 0, st, p, b, x_out, S_out, scale, 1, (const double *)nullptr);
  return hipGetLastError();
}

template <int NT, int PPL>
hipError_t launch_block_nt(const BatchDesc *descs, int n, const Pools &pools, const Params *prm, int project,
                           float *x_out, float *S_out, BatchOut *outs, size_t lds_bytes, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void *)k_block_solve<NT, PPL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_block_solve<NT, PPL>), dim3(n), dim3(NT), lds_bytes, st, descs, pools, prm, project, x_out,
                     S_out, outs);
  return hipGetLastError();
}

template <int NT>
hipError_t launch_block_ppl(const BatchDesc *descs, int n, const Pools &pools, const Params *prm, int project,
                            float *x_out, float *S_out, BatchOut *outs, size_t lds_bytes, int ppl, hipStream_t st) {
  switch (ppl) {
    case 1: return launch_block_nt<NT, 1>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, st);
    case 2: return launch_block_nt<NT, 2>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, st);
    case 4: return launch_block_nt<NT, 4>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, st);
    case 8: return launch_block_nt<NT, 8>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, st);
    default: return hipErrorInvalidValue;
  }
}

// threads: 256, 512 or 1024 per workgroup (one instance per workgroup); ppl: paths per lane, 1, 2, 4 or 8
hipError_t launch_block_solve(const BatchDesc *descs, int n, const Pools &pools, const Params *prm, int project,
                              float *x_out, float *S_out, BatchOut *outs, size_t lds_bytes, int threads, int ppl,
                              hipStream_t st) {
  switch (threads) {
    case 256: return launch_block_ppl<256>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, ppl, st);
    case 512: return launch_block_ppl<512>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, ppl, st);
    case 1024: return launch_block_ppl<1024>(descs, n, pools, prm, project, x_out, S_out, outs, lds_bytes, ppl, st);
    default: return hipErrorInvalidValue;
  }
}

// Dynamic LDS of the workgroup engine for one instance; SIZE_MAX when its indices do not fit the
// 16-bit LDS encoding (P < 2^15 for the head bit, nnz, E, D < 2^16).
size_t block_lds_bytes(int E, int P, int D, int nnz) {
  if (P >= 32768 || nnz >= 65536 || E >= 65536 || D >= 65536) return SIZE_MAX;
  return (size_t)E * (16 + 8 + 8) + (size_t)D * (8 + 8 + 8 + 8) + (size_t)P * 8 * 2 +
         (size_t)2 * ((P + 1) + nnz + (D + 1) + (E + 1) + nnz + E) + 16;
}

}  // namespace te
