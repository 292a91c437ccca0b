// te_device.h -- device-side arithmetic of one GATE iteration, shared by both engines.
//
// Notation (paper, section 3): x_r path rate, S_c demand sum, D_c demand, C_e capacity,
// n_r links on path r, n_e paths on link e, beta penalty, alpha fairness, scaled duals
// u_dem (per demand), u_neg (per path).  The capacity and consensus duals of a link
// coincide after every sweep (dual_con_{e,r} = dual_cap_e = g_e), and every rate
// suggestion of a link is y_{e,r} = x_r + q_e with one offset q_e per link, so the
// per-incidence variables of section 3.2 collapse to the per-link pair (g_e, q_e):
//   rate-update consensus term   a_r = n_r x_r - sum_{e in r} (g_e - q_e)
//   rate suggestion + cap dual   g_e' = [g_e + (load_e - C_e) / (1 + n_e)]_+,  q_e' = g_e - g_e'
// (derived from the exact per-link minimisation with slack_cap, appendix B.1).
#pragma once

#include <math.h>
#include "te_internal.h"

namespace te {

enum { F_CONVERGED = 1, F_MAX_ITERS = 2, F_ALPHA_MAX = 4, F_BETA_BOUND = 8 };

// ------------------------------------------------------------------------------------------
// lane-group reductions (G lanes, power of two, aligned inside one 64-wide wavefront).
// Butterflies whose pairings are symmetric, so every lane of the group ends with the bit-identical
// result: DPP lane moves inside a row of 16 (quad permutes for distance 1 and 2, the half-row
// mirror j <-> 7-j and the row mirror j <-> 15-j, which pair lanes holding equal partial results
// after the previous stages), cross-lane permutes for distances 16 and 32.  All lanes of a group
// must be active (the callers keep control flow uniform per group).
// ------------------------------------------------------------------------------------------
enum : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// DPP move with an explicit value for lanes whose source is outside the pattern (or whose row is
// not in the row mask RM)
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_old_d(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, RM, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int RM>
__device__ __forceinline__ void seg_scan_step(double &x, int key) {
  const double y = dpp_old_d<CTRL, RM>(x, 0.0);
  const int ky = __builtin_amdgcn_update_dpp(-1, key, CTRL, RM, 0xF, false);
  if (ky == key) x += y;
}

// Inclusive segmented sum over the 64 lanes: runs of equal key (keys >= 0, non-decreasing with
// the lane index) are the segments.  Hillis-Steele steps inside each row of 16 lanes (row shifts
// by 1, 2, 4, 8), then the row carries (lane 15 into row 1 and lane 47 into row 3, then lane 31
// into rows 2 and 3), each added only where the source lane has the same key.  Every lane must be
// active.
__device__ __forceinline__ double seg_scan_d(double x, int key) {
  seg_scan_step<0x111, 0xF>(x, key);  // row_shr:1
  seg_scan_step<0x112, 0xF>(x, key);  // row_shr:2
  seg_scan_step<0x114, 0xF>(x, key);  // row_shr:4
  seg_scan_step<0x118, 0xF>(x, key);  // row_shr:8
  seg_scan_step<0x142, 0xA>(x, key);  // row_bcast:15 into rows 1, 3
  seg_scan_step<0x143, 0xC>(x, key);  // row_bcast:31 into rows 2, 3
  return x;
}

// key of the next lane (lane 63: -2)
__device__ __forceinline__ int next_lane_key(int key) {
  return __builtin_amdgcn_update_dpp(-2, key, 0x130, 0xF, 0xF, false);  // wave_shl:1
}

__device__ __forceinline__ double group_sum_d(double v, int G) {
  if (G >= 2) v += dpp_d<kDppXor1>(v);
  if (G >= 4) v += dpp_d<kDppXor2>(v);
  if (G >= 8) v += dpp_d<kDppHalfMirror>(v);
  if (G >= 16) v += dpp_d<kDppMirror>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) { return group_sum_d(v, 64); }
__device__ __forceinline__ double wave_max_d(double v) {
  v = fmax(v, dpp_d<kDppXor1>(v));
  v = fmax(v, dpp_d<kDppXor2>(v));
  v = fmax(v, dpp_d<kDppHalfMirror>(v));
  v = fmax(v, dpp_d<kDppMirror>(v));
  v = fmax(v, __shfl_xor(v, 16, 64));
  return fmax(v, __shfl_xor(v, 32, 64));
}

// ------------------------------------------------------------------------------------------
// per-demand update: the sum equation of appendix B.2 and the rate update of section 3.3.
// The commodity sub-problem's stationarity in x_r reads n_r x_r - [u_neg_r - x_r]_+ = a_r - h(S),
// h(S) = [S - D + u_dem]_+ - S^-alpha / beta; xi_r inverts the left side; the root of
// F(S) = sum_r xi_r(a_r - h(S)) - S (continuous, strictly decreasing) gives S, then x.
// ------------------------------------------------------------------------------------------
struct Lane {
  double a;     // a_r
  double un;    // u_neg_r (current beta scale)
  double n;     // n_r
  double rn;    // 1 / n_r
  double rn1;   // 1 / (n_r + 1)
  bool on;      // lane holds a path of the demand
};

// A lane holding up to PPL paths of one demand (slot j: path lane + j * (lanes per demand) of the
// demand's list; bit j of `on` set if that path exists).  The per-demand work of the root solve is
// then shared by fewer lanes per demand, and PPL = 1 is the one-path lane above.
template <int PPL>
struct LaneN {
  double a[PPL], un[PPL], n[PPL], rn[PPL], rn1[PPL];
  unsigned on;
};

// 1/d from the hardware reciprocal estimate and two Newton-Raphson steps r <- r + r (1 - d r)
// (each roughly squares the relative error), for the divisions of the root solve: within ~1 ulp,
// at a third of the instructions of a correctly rounded FP64 division.  d normal and nonzero.
__device__ __forceinline__ double rcp_refined(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  return fma(fma(-d, r, 1.0), r, r);
}

struct Dem {
  double D, u, binv;  // demand, u_dem (current scale), 1/beta
  double alpha;
};

// S^-alpha in FP64 from invS = 1/S.  Integer alpha up to 64 (every alpha the continuation produces
// from 0) by binary powering of 1/S (relative error below ~2 alpha ulps), other alpha by exp/log.
// FP32 is not enough here: the iteration at alpha >= 1 amplifies a 1e-7 relative error of this
// term over a few hundred iterations to ~4e-4 in the sums.
__device__ __forceinline__ double pow_neg_alpha(double S, double invS, double alpha) {
  if (alpha == 0.0) return 1.0;
  const int ia = (int)alpha;
  if ((double)ia == alpha && ia > 0 && ia <= 64) {
    double r = 1.0, b = invS;
    for (int m = ia;;) {
      if (m & 1) r *= b;
      m >>= 1;
      if (!m) break;
      b *= b;
    }
    return r;
  }
  return exp(-alpha * log(S));
}

__device__ __forceinline__ double xi_of(double b, const Lane &L) {
  return (b >= L.n * L.un) ? b * L.rn : (b + L.un) * L.rn1;
}

__device__ __forceinline__ double h_of(double S, const Dem &c) {
  const double invS = c.alpha > 0.0 ? rcp_refined(S) : 0.0;  // alpha = 0: S^-alpha = 1, no division
  return fmax(S - c.D + c.u, 0.0) - pow_neg_alpha(S, invS, c.alpha) * c.binv;
}

// F(S), F'(S) and the smooth part of F''(S), summed over the group (uniform inside the group).
__device__ __forceinline__ void F_eval(double S, const Lane &L, const Dem &c, int G, double &F, double &dF,
                                       double &d2F) {
  if (c.alpha > 0.0 && !(S > 0.0)) {
    F = INFINITY;
    dF = -INFINITY;
    d2F = 0.0;
    return;
  }
  const double t = S - c.D + c.u;
  const double invS = c.alpha > 0.0 ? rcp_refined(S) : 0.0;  // alpha = 0: S^-alpha = 1, no division
  const double pw = pow_neg_alpha(S, invS, c.alpha);
  const double h = fmax(t, 0.0) - pw * c.binv;
  const double dh = (t > 0.0 ? 1.0 : 0.0) + (c.alpha > 0.0 ? c.alpha * pw * c.binv * invS : 0.0);
  const double b = L.a - h;
  const bool hi_branch = b >= L.n * L.un;
  double v = L.on ? (hi_branch ? b * L.rn : (b + L.un) * L.rn1) : 0.0;
  double dv = L.on ? (hi_branch ? L.rn : L.rn1) : 0.0;
  v = group_sum_d(v, G);
  dv = group_sum_d(dv, G);
  F = v - S;
  dF = -dh * dv - 1.0;
  // plain Newton steps here: in the device-wide kernel a wavefront holds eight demands, whose
  // slowest root decides its time, and the curvature correction measured no faster there
  d2F = 0.0;
}

template <int PPL>
__device__ __forceinline__ void F_eval(double S, const LaneN<PPL> &L, const Dem &c, int G, double &F, double &dF,
                                       double &d2F) {
  if (c.alpha > 0.0 && !(S > 0.0)) {
    F = INFINITY;
    dF = -INFINITY;
    d2F = 0.0;
    return;
  }
  const double t = S - c.D + c.u;
  const double invS = c.alpha > 0.0 ? rcp_refined(S) : 0.0;
  const double pw = pow_neg_alpha(S, invS, c.alpha);
  const double h = fmax(t, 0.0) - pw * c.binv;
  const double dh = (t > 0.0 ? 1.0 : 0.0) + (c.alpha > 0.0 ? c.alpha * pw * c.binv * invS : 0.0);
  double v = 0.0, dv = 0.0;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    if (!((L.on >> j) & 1u)) continue;
    const double b = L.a[j] - h;
    const bool hi_branch = b >= L.n[j] * L.un[j];
    v += hi_branch ? b * L.rn[j] : (b + L.un[j]) * L.rn1[j];
    dv += hi_branch ? L.rn[j] : L.rn1[j];
  }
  v = group_sum_d(v, G);
  dv = group_sum_d(dv, G);
  F = v - S;
  dF = -dh * dv - 1.0;
  // away from the kinks F'' = -h''(S) dv with h'' = -alpha (alpha + 1) S^(-alpha-2) / beta
  d2F = c.alpha > 0.0 ? c.alpha * (c.alpha + 1.0) * pw * c.binv * invS * invS * dv : 0.0;
}

// Safeguarded Newton (appendix B.2) from the warm start S0: every evaluation narrows the bracket
// [lo, hi] with F(lo) > 0 > F(hi) (ends infinite until a sign of each kind has been seen); the next
// point is the Newton point -- with Halley's correction for the curvature of the S^-alpha term,
// step / (1 - step F'' / (2 F')), when F'' is given and that factor lies in (1/2, 2): cubic instead
// of quadratic convergence on the smooth part, for the price of one product per evaluation; the
// workgroup engine, whose wavefronts hold up to 64 demands, gives F'' -- when it lies
// strictly inside the bracket (and stays positive for alpha > 0), else the midpoint once both ends
// are known, else an expansion (doubling steps, or halving towards 0 for alpha > 0).  Stops when
// the correction or the bracket falls below 1e-13 max(1, |S|) (normalised units, where F's
// rounding noise is ~1e-16 of its O(1) terms).  The root is the same as the oracle's to that
// tolerance; only the path to it is shorter.
// alpha = 0: F is piecewise linear, with kinks where the demand hinge t = S - D + u_dem or a
// path's branch b_r = a_r - h(S) >= n_r u_neg_r changes (the same expressions as F_eval's).  True
// when one of them changes between S and Sn for this lane.
__device__ __forceinline__ bool kink_between(double S, double Sn, const Lane &L, const Dem &c) {
  const double t0 = S - c.D + c.u, t1 = Sn - c.D + c.u;
  if ((t0 > 0.0) != (t1 > 0.0)) return true;
  if (!L.on) return false;
  const double h0 = fmax(t0, 0.0) - c.binv, h1 = fmax(t1, 0.0) - c.binv;
  const double th = L.n * L.un;
  return (L.a - h0 >= th) != (L.a - h1 >= th);
}

template <int PPL>
__device__ __forceinline__ bool kink_between(double S, double Sn, const LaneN<PPL> &L, const Dem &c) {
  const double t0 = S - c.D + c.u, t1 = Sn - c.D + c.u;
  if ((t0 > 0.0) != (t1 > 0.0)) return true;
  const double h0 = fmax(t0, 0.0) - c.binv, h1 = fmax(t1, 0.0) - c.binv;
  bool k = false;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const double th = L.n[j] * L.un[j];
    k = k || (((L.on >> j) & 1u) && ((L.a[j] - h0 >= th) != (L.a[j] - h1 >= th)));
  }
  return k;
}

// true on every lane of a group of G lanes (aligned, a power of two) when it is true on one of them
// (the group sum of the F evaluation, applied to a flag)
__device__ __forceinline__ bool group_any(bool pred, int G) { return group_sum_d(pred ? 1.0 : 0.0, G) > 0.0; }

template <class LaneT>
__device__ double sum_root(double S, const LaneT &L, const Dem &c, int G, int *evals) {
  const double tol = 1e-13;
  if (c.alpha > 0.0 && !(S > 0.0)) S = fmax(c.D, 1e-6);
  double lo = -INFINITY, hi = INFINITY, expand = 0.0;
  *evals = 0;
  for (int it = 0; it < 1200; ++it) {
    double F, dF, d2F;
    F_eval(S, L, c, G, F, dF, d2F);
    ++*evals;
    if (F == 0.0) return S;
    if (F > 0.0) lo = S; else hi = S;
    const double scale = fmax(fabs(S), 1.0);
    if (hi - lo <= tol * scale) return S;
    double Sn = 0.0;
    bool ok = isfinite(F) && isfinite(dF) && dF < 0.0;
    if (ok) {
      const double rdF = rcp_refined(dF);
      double step = F * rdF;
      if (d2F != 0.0) {
        const double den = 1.0 - 0.5 * step * d2F * rdF;
        if (den > 0.5 && den < 2.0) step *= rcp_refined(den);
      }
      if (fabs(step) <= tol * scale) return S - step;  // correction below tolerance
      Sn = S - step;
      ok = Sn > lo && Sn < hi && !(c.alpha > 0.0 && !(Sn > 0.0));
      // alpha = 0: on a linear piece of F the Newton point is its root; when no kink lies between
      // S and Sn it is returned without the evaluation that would only confirm it (F(Sn) is zero
      // to rounding there)
      if (ok && c.alpha == 0.0 && !group_any(kink_between(S, Sn, L, c), G)) return Sn;
    }
    if (!ok) {
      if (lo > -INFINITY && hi < INFINITY) {
        Sn = 0.5 * (lo + hi);
      } else if (F > 0.0 || c.alpha == 0.0) {
        expand = expand > 0.0 ? 2.0 * expand : fmax(fabs(S), 1e-6);
        Sn = F > 0.0 ? S + expand : S - expand;
      } else {
        Sn = 0.5 * S;
      }
    }
    S = Sn;
  }
  return S;
}

// ------------------------------------------------------------------------------------------
// Control decision after iteration k (sections 3.4): residual balancing of beta with
// rescale of the scaled duals, alpha-increments, stop test.  Sums: [s2, r2, cap, dem].
// The balancing rule may act after iteration k when the cadence admits k + 1 and the back-off
// has run out: a change of beta opposite to the previous one is the n-th reversal and rests the
// rule for the next 2^n - 1 iterations (2^20 at most).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ bool rule_may_act(const Params &prm, const Ctrl &c) {
  return ((c.k + 1) % prm.beta_every) == 0 && c.k + 1 >= c.rule_from;
}

__device__ inline Ctrl decide(const Ctrl &prev, const double *sums, const Params &prm) {
#pragma clang fp contract(off)
  if (!prev.pending) return prev;
  Ctrl c = prev;
  c.pending = 0;
  double r = sqrt(sums[1]), s = sqrt(sums[0]);
  c.r = r;
  c.s = s;
  c.cap_viol = sums[2];
  c.dem_viol = sums[3];
  int kdone = prev.k + 1;
  const bool replay = prm.sched_beta != nullptr;
  double f = 1.0;
  if (replay) {
    int kk = kdone < prm.sched_len ? kdone : prm.sched_len - 1;
    double nb = prm.sched_beta[kk];
    f = nb / prev.beta;
    c.beta = nb;
    c.alpha = prm.sched_alpha[kk];
  } else {
    if (prm.adapt_beta && rule_may_act(prm, prev)) {
      if (r > prm.A * s) {
        if (prev.beta * prm.C <= prm.beta_max) f = prm.C; else c.flags |= F_BETA_BOUND;
      } else if (s > prm.A * r) {
        if (prev.beta / prm.C >= prm.beta_min) f = 1.0 / prm.C; else c.flags |= F_BETA_BOUND;
      }
      if (f != 1.0) {
        const int dir = f > 1.0 ? 1 : -1;
        if (prev.last_dir != 0 && dir != prev.last_dir) {
          c.n_rev = prev.n_rev + 1;
          c.rule_from = kdone + (1 << (c.n_rev < 20 ? c.n_rev : 20));
        }
        c.last_dir = dir;
      }
    }
    c.beta = prev.beta * f;
    int j = prev.j + 1;
    bool stop = false;
    if (r <= prm.gamma && s <= prm.gamma) {
      bool would_stop = (prev.alpha >= prm.alpha_target) || (prev.alpha >= 1.0 && j <= 1);
      if (would_stop) {
        c.flags |= F_CONVERGED;
        if (c.stop_iter < 0) c.stop_iter = kdone;
        if (!prm.fixed) stop = true;
      }
      if (!stop && prev.alpha < prm.alpha_target) {
        double na = prev.alpha + 1.0;
        if (na > prm.alpha_target) na = prm.alpha_target;
        if (na > (double)prm.alpha_max) {
          c.flags |= F_ALPHA_MAX;
          if (!prm.fixed) stop = true;
        } else {
          c.alpha = na;
          j = 0;
        }
      }
    }
    c.j = j;
    if (stop) c.stop = 1;
  }
  c.inv_f = 1.0 / f;
  c.k = kdone;
  if (kdone >= prm.kmax) {
    if (!c.stop && !prm.fixed && !replay) c.flags |= F_MAX_ITERS;
    c.stop = 1;
  }
  return c;
}

__device__ inline Ctrl initial_ctrl(const Params &prm) {
  Ctrl c;
  const bool replay = prm.sched_beta != nullptr;
  c.beta = replay ? prm.sched_beta[0] : prm.beta0;
  c.alpha = replay ? prm.sched_alpha[0] : (prm.alpha_target < 0.0 ? prm.alpha_target : 0.0);
  c.inv_f = 1.0;
  c.r = c.s = 0.0;
  c.cap_viol = c.dem_viol = 0.0;
  c.k = 0;
  c.j = 0;
  c.stop = prm.kmax <= 0;
  c.flags = 0;
  c.stop_iter = -1;
  c.pending = 0;
  c.last_dir = 0;
  c.n_rev = 0;
  c.rule_from = 0;
  return c;
}

// 64-bit ordering key of a path in the projection: descending score S_c^alpha * C_p compared
// through alpha ln S_c + ln C_p, ties broken towards the higher path index.
__device__ __forceinline__ uint64_t trim_key(float logscore, int32_t p) {
  uint32_t b = __float_as_uint(logscore);
  b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // order-preserving map of the float
  return ((uint64_t)b << 32) | (uint32_t)p;
}

__device__ __forceinline__ float log_score(double S, int Cp, float alpha) {
  if (Cp <= 0 || !(S > 0.0)) return -INFINITY;
  return __fadd_rn(__fmul_rn(alpha, logf((float)S)), logf((float)Cp));  // rounded product, no fused multiply-add
}

}  // namespace te
