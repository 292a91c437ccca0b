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
// xor butterflies: every lane of the group ends with the bit-identical sum.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float group_sum(float v, int G) {
  for (int m = 1; m < G; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double group_sum_d(double v, int G) {
  for (int m = 1; m < G; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int m = 1; m < 64; m <<= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
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

struct Dem {
  double D, u, binv;  // demand, u_dem (current scale), 1/beta
  float alpha;
};

// S^-alpha in FP32: at the root the term's own slope alpha S^-alpha / (beta S) damps its rounding,
// a relative error eps in it moves the root by at most eps / alpha relative.
__device__ __forceinline__ double pow_neg_alpha(double S, float alpha) {
  return alpha == 0.f ? 1.0 : (double)exp2f(-alpha * log2f((float)S));
}

__device__ __forceinline__ double xi_of(double b, const Lane &L) {
  return (b >= L.n * L.un) ? b * L.rn : (b + L.un) * L.rn1;
}

__device__ __forceinline__ double h_of(double S, const Dem &c) {
  return fmax(S - c.D + c.u, 0.0) - pow_neg_alpha(S, c.alpha) * c.binv;
}

// F(S) and F'(S) summed over the group (uniform inside the group).
__device__ __forceinline__ void F_eval(double S, const Lane &L, const Dem &c, int G, double &F, double &dF) {
  if (c.alpha > 0.f && !(S > 0.0)) {
    F = INFINITY;
    dF = -INFINITY;
    return;
  }
  const double t = S - c.D + c.u;
  const double pw = pow_neg_alpha(S, c.alpha);
  const double h = fmax(t, 0.0) - pw * c.binv;
  const double dh = (t > 0.0 ? 1.0 : 0.0) + (c.alpha > 0.f ? (double)c.alpha * pw * c.binv / S : 0.0);
  const double b = L.a - h;
  const bool hi_branch = b >= L.n * L.un;
  double v = L.on ? (hi_branch ? b * L.rn : (b + L.un) * L.rn1) : 0.0;
  double dv = L.on ? (hi_branch ? L.rn : L.rn1) : 0.0;
  v = group_sum_d(v, G);
  dv = group_sum_d(dv, G);
  F = v - S;
  dF = -dh * dv - 1.0;
}

// Safeguarded Newton (appendix B.2): bracket [lo, hi] with F(lo) > 0 > F(hi), its first trial end
// 1.5 Newton steps from the warm start (then doubling), Newton steps while they stay inside the
// bracket, bisection otherwise; stops when the Newton correction or the bracket falls below
// 1e-13 max(1, |S|) (normalised units, where F's rounding noise is ~1e-16 of its O(1) terms).
__device__ double sum_root(double S0, const Lane &L, const Dem &c, int G, int *steps) {
  const double tol = 1e-13;
  if (c.alpha > 0.f && !(S0 > 0.0)) S0 = fmax(c.D, 1e-6);
  double F0, d0;
  F_eval(S0, L, c, G, F0, d0);
  *steps = 0;
  if (F0 == 0.0) return S0;
  const double guess = (isfinite(F0) && isfinite(d0) && d0 < 0.0) ? -1.5 * F0 / d0 : 0.0;
  double lo, hi, Fs, dFs, S;
  if (F0 > 0.0) {
    lo = S0;
    double Flo = F0, dlo = d0;
    double step = guess > 0.0 ? guess : fmax(fabs(S0), 1e-6);
    hi = S0 + step;
    for (int i = 0; i < 1100; ++i) {
      double Fh, dh;
      hi = S0 + step;
      F_eval(hi, L, c, G, Fh, dh);
      if (Fh == 0.0) return hi;
      if (Fh < 0.0) break;
      lo = hi;
      Flo = Fh;
      dlo = dh;
      step *= 2.0;
    }
    S = lo;
    Fs = Flo;
    dFs = dlo;
  } else {
    hi = S0;
    double Fhi = F0, dhi = d0;
    if (c.alpha > 0.f) {
      lo = (guess < 0.0 && S0 + guess > 0.0) ? S0 + guess : 0.5 * S0;
      for (int i = 0; i < 1100; ++i) {
        double Fl, dl;
        F_eval(lo, L, c, G, Fl, dl);
        if (Fl == 0.0) return lo;
        if (Fl > 0.0) break;
        hi = lo;
        Fhi = Fl;
        dhi = dl;
        lo *= 0.5;
      }
    } else {
      double step = guess < 0.0 ? -guess : fmax(fabs(S0), 1e-6);
      lo = S0 - step;
      for (int i = 0; i < 1100; ++i) {
        double Fl, dl;
        lo = S0 - step;
        F_eval(lo, L, c, G, Fl, dl);
        if (Fl == 0.0) return lo;
        if (Fl > 0.0) break;
        hi = lo;
        Fhi = Fl;
        dhi = dl;
        step *= 2.0;
      }
    }
    S = hi;
    Fs = Fhi;
    dFs = dhi;
  }
  for (int it = 0; it < 100; ++it) {
    double Sn = 0.0;
    bool newton = isfinite(Fs) && isfinite(dFs) && dFs < 0.0;
    if (newton) {
      const double step = Fs / dFs;
      if (fabs(step) <= tol * fmax(fabs(S), 1.0)) return S - step;  // correction below tolerance
      Sn = S - step;
      newton = (Sn > lo && Sn < hi);
    }
    if (!newton) Sn = 0.5 * (lo + hi);
    double Fn, dn;
    F_eval(Sn, L, c, G, Fn, dn);
    ++*steps;
    if (Fn == 0.0) return Sn;
    if (Fn > 0.0) lo = Sn; else hi = Sn;
    if (hi - lo <= tol * fmax(fabs(Sn), 1.0)) return Sn;
    S = Sn;
    Fs = Fn;
    dFs = dn;
  }
  return S;
}

// ------------------------------------------------------------------------------------------
// Control decision after iteration k (sections 3.4): residual balancing of beta with
// rescale of the scaled duals, alpha-increments, stop test.  Sums: [s2, r2, cap, dem].
// ------------------------------------------------------------------------------------------
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
    if (prm.adapt_beta && (kdone % prm.beta_every) == 0) {
      if (r > prm.A * s) {
        if (prev.beta * prm.C <= prm.beta_max) f = prm.C; else c.flags |= F_BETA_BOUND;
      } else if (s > prm.A * r) {
        if (prev.beta / prm.C >= prm.beta_min) f = 1.0 / prm.C; else c.flags |= F_BETA_BOUND;
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
  return alpha * logf((float)S) + logf((float)Cp);
}

}  // namespace te
