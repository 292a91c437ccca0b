// te_internal.h -- structures shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace te {

// Control record of one iteration: the penalty, alpha and stop state that
// Algorithm 1 (section 3.3) carries from one iteration to the next.
// Slot (k & 1) holds the record of iteration k; `pending` = 1 means the
// residual-balancing / alpha / stop decision taken after iteration k has not
// been applied yet (it is applied redundantly, and identically, by every
// workgroup that reads the record).
struct Ctrl {
  double beta;   // penalty used in iteration k
  double alpha;  // alpha used in iteration k
  double inv_f;  // 1/f: rescale of the scaled duals decided after iteration k-1
  double r, s;   // residuals of iteration k-1
  double cap_viol, dem_viol;  // max relative violations seen in iteration k-1
  int32_t k;          // iteration index
  int32_t j;          // iterations since the last alpha increment
  int32_t stop;       // 1: no further iterations
  int32_t flags;      // TE_* flags
  int32_t stop_iter;  // first iteration whose stop test passed (-1 none)
  int32_t pending;
  int32_t last_dir;   // direction of the rule's last change of beta: +1, -1, 0 (none yet)
  int32_t n_rev;      // reversals of that direction so far
  int32_t rule_from;  // the rule rests until iteration count rule_from (back-off after a reversal)
};

// Constant parameters of one solve.
struct Params {
  double alpha_target, gamma, A, C, beta_min, beta_max, beta0;
  int32_t kmax;        // iteration cap
  int32_t fixed;       // 1: fixed iteration count, no stop
  int32_t adapt_beta, beta_every, alpha_max;
  int32_t per_link;    // 1: link e's constraints carry beta * w_e, w_e moved by the per-link rule
  double w_min, w_max; // bounds on w_e
  int32_t sched_len;
  const double *sched_beta;   // device, nullable
  const double *sched_alpha;  // device, nullable
};

// Problem arrays on the device (normalised units).
struct Prob {
  int32_t E, P, D, nnz;
  int32_t G, logG;         // lanes per demand (power of two >= max paths per demand)
  const int32_t *pptr;     // [P+1] path -> incidence range
  const int32_t *plinks;   // [nnz] link of each incidence (path-major)
  const int32_t *dptr;     // [D+1] demand -> path range
  const int32_t *lptr;     // [E+1] link -> CSC range
  const int32_t *lpaths;   // [nnz] path of each CSC entry (link-major, path-ascending)
  const double *Dn;        // [D] demand
  const double *Cn;        // [E] capacity
  // link kernel work split: non-empty links in order (nzlink), their CSC starts (nzptr, one more
  // entry at the end), per-workgroup ranges of non-empty-link ranks (blk[nB+1]); lpf = lpaths
  // with bit 31 set on the first entry of every link
  const int32_t *lpf;
  const int32_t *nzlink;
  const int32_t *nzptr;
  const int32_t *blk;
  // per wavefront of the link kernels ([nB * kLinkWaves]): its CSC entry range [x, y) and the rank
  // (index into nzlink) of the link holding entry x, precomputed so that no wavefront searches
  const int4 *wtab;
  // per path, its first H link ids as 16-bit slots in path order, unused slots 0xffff (H = 4 or 8);
  // H = 0 when some path has more than kMaxHopSlots hops or a link id does not fit 16 bits.  The
  // paths of a demand that has a path longer than H continue in overflow records of H2 slots (H2 =
  // 4 or 8): the demand's paths hold records dovf[d], dovf[d] + 1, ... of hops2, in path order;
  // dovf[d] = -1 for a demand whose paths all fit H (H2 = 0, hops2 and dovf null when every path does)
  const uint16_t *hops;
  int32_t H;
  const uint16_t *hops2;
  int32_t H2;
  const int32_t *dovf;
  // demand kernel of the graph engine: paths per lane (1 = one lane per path) and log2 of its
  // lanes per demand, max(1, G / ppl)
  int32_t ppl, logGp;
  // how the link loads are summed: kLinkSumsPrivate (each demand workgroup sums its paths' rates
  // into an LDS copy of the E loads, one row per workgroup, rows reduced per link) or kLinkSumsCsc
  // (segmented sums over the link -> path CSC list)
  int32_t lsum;
  // privatised sums: passes of kScatThreads / 2^logGp demands, spw consecutive passes per scatter
  // workgroup, nF workgroups (rows of partial loads)
  int32_t npass, spw, nF;
  // privatised sums by link lists (cpp > 0): a scatter workgroup takes its passes in chunks of cpp
  // (cpw chunks); a chunk's new rates stay in LDS (path r at r minus the chunk's first path, slot
  // zslot holding 0) and are summed per link over the chunk's list.  The list holds the rate slots of
  // each link's paths in pieces of at most kPieceLen, 64 pieces to a group; group g is lgrp[g] =
  // {offset into lent (a multiple of 8), blocks}: 64 header entries (the piece's link, bit 15 when
  // the link has other pieces, 0xffff for no piece), then blocks of 512 entries, block b holding
  // slots 8 b .. 8 b + 7 of piece i at 8 i .. 8 i + 7 (zslot past a piece's end).
  // lchk[b * cpw + k] = {first group, end, first path, 0} of chunk k of workgroup b.  cpp = 0: one
  // LDS atomic addition per incidence instead.
  int32_t cpp, cpw, zslot;
  const uint16_t *lent;
  const int2 *lgrp;
  const int4 *lchk;
  // nullable [D]: per-demand unit scale of the outputs (a batch solved as the union of its
  // instances, each in its own units), in place of the handle's one scale
  const double *dscale;
};

enum { kLinkSumsPrivate = 1, kLinkSumsCsc = 2, kLinkSumsPrivateAtomic = 3 };

constexpr int kMaxHopSlots = 16;
constexpr int kPrimarySlots = 8;  // slots of a path's primary hop record
// graph engine: instances with at least kMultiLanes lane slots (demands x G) run the demand step
// with min(G, kMultiPaths) paths per lane
constexpr int64_t kMultiLanes = 1 << 20;
constexpr int kMultiPaths = 2;

// Iteration state on the device.
struct State {
  double *x, *uneg;  // [P] path rates and non-negativity duals
  double *udem, *S;  // [D] demand duals and last root of the sum equation
  double2 *gq;       // [E] (g, q): g = capacity / consensus dual, q = consensus offset
  double *w;         // [E] per-link penalty factors (1 without per-link penalties)
  double *dx2;       // [P] (x' - x)^2 of the iteration, written where the per-link rule needs it
  // where an iteration writes its new x, u_neg, u_dem, S and (g, q): the arrays above (in place),
  // or another state block (the gradient's recomputation writes iteration k + 1 next to k)
  double *xo, *unego, *udemo, *So;
  double2 *gqo;
  Ctrl *ctrl;        // [3]
  double *partA;     // [2][nArows][4]: the demand kernels' per-wavefront rows (nA workgroups)
  double *partB;     // [2][nB][4]: the link kernel's per-workgroup rows
  int32_t nA, nB, nArows;
  double *partL;     // [nF][E] privatised sums: each scatter workgroup's share of the link loads
  // nullable [4][log_cap]: per iteration k the beta_k and alpha_k it used and its residuals r_k, s_k
  // (rows beta | alpha | r | s), written when recording for the gradient or tracing
  double *log;
  int32_t log_cap;
};

// Adjoint state of the reverse pass (FP64), adjoints of one iteration's outputs.
struct AdjState {
  double *xb, *unb;  // [P]
  double *udb;       // [D]
  double *gb, *qb;   // [E]
  double *ab;        // [P] scratch: adjoint of the consensus term a_r
  double *Cb;        // [E] accumulated gradient w.r.t. capacities (normalised units)
  double *Db;        // [D] accumulated gradient w.r.t. demands
};

// One stored forward state (the iteration state of State, without control data).
struct FwdState {
  double *x, *uneg;
  double *udem, *S;
  double2 *gq;
};

constexpr int kMaxLinkBlocks = 512;  // workgroups of the link kernel (partB rows), at most
constexpr int kMaxLinksPerBlock = 1024;
constexpr int kThreads = 256;        // threads per workgroup of the graph-engine demand kernels
constexpr int kLinkThreads = 1024;   // threads per workgroup of the link kernels (16 wavefronts)
constexpr int kLinkWaves = kLinkThreads / 64;
constexpr int kScatThreads = 1024;   // threads per workgroup of the privatised-sum demand kernel
constexpr int kScatWaves = kScatThreads / 64;
constexpr int kPieceLen = 32;  // link-list entries of a piece, at most (four blocks of 8)
// privatised sums: the scatter workgroup's LDS copy of the loads (8 bytes a link) and the link
// reduction's workgroups (64 links each, at most kMaxLinkBlocks) bound the links
constexpr int kMaxScatterLinks = 19456;
constexpr int kScatLds = 8 * kMaxScatterLinks;  // dynamic LDS of a scatter workgroup, at most (bytes)

// Workgroup-engine instance descriptor: offsets into concatenated arrays.
struct BatchDesc {
  int32_t E, P, D, nnz, G, logG;
  int32_t nzl;  // non-empty links
  // into int32 pools: CSR, demand ranges, CSC pointers, CSC path ids with bit 31 on each link's
  // first entry, the non-empty links in order
  int64_t off_pptr, off_plinks, off_dptr, off_lptr, off_lpf, off_nzl;
  int64_t off_E, off_P, off_D;  // element offsets of per-link / per-path / per-demand arrays
  double scale;
};

// Scratch of the graph-engine projection (Algorithm 2).
struct ProjBuf {
  double *xd;      // [P] working rates
  double *S;       // [D]
  double *L;       // [E]
  int32_t *Cp;     // [P] violated links per path
  float *lsc;      // [P] log score
  uint64_t *trim;  // [P] largest trim (double bits)
};

// Concatenated inputs of the workgroup engine.
struct Pools {
  const int32_t *i32;  // index pool
  const double *Dn;    // [sum D]
  const double *Cn;    // [sum E]
  const float *x0;     // nullable [sum P] warm start, caller units
  double *log;         // nullable [4][log_cap] per-iteration log of workgroup 0's instance (as State::log)
  int32_t log_cap;
};

struct BatchOut {
  double beta, alpha, r, s, cap_viol, dem_viol;
  int32_t iters, flags, stop_iter, pad;
};

}  // namespace te
