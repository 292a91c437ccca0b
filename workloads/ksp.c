/*
 * k shortest loopless paths (Yen's algorithm) for the synthetic WAN inputs.
 *
 * Paths are the first k simple s->t paths in the total order
 * (cost, node sequence), cost being the sum of arc weights taken in path
 * order and the node sequence compared lexicographically.  The TE problem
 * takes its path sets as given input (paper, section "TE Formulation"); this
 * file only builds such inputs.  It holds none of the solver's arithmetic.
 *
 * Each spur search is a Dijkstra run backwards from the target on the graph
 * with the root's nodes and the forbidden arcs removed, followed by a greedy
 * walk from the spur node that always takes the smallest next node on some
 * shortest path.  That walk yields the lexicographically smallest shortest
 * spur path, so Yen's candidate selection by (cost, sequence) reproduces the
 * total order above exactly (tests compare against brute-force enumeration).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC ksp.c -o libksp.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
  int n, m;
  const int32_t *out_ptr, *out_arc; /* forward CSR: arcs leaving u, sorted by head */
  const int32_t *in_ptr, *in_arc;   /* reverse CSR: arcs entering v */
  const int32_t *src, *dst;
  const double *w;
} graph_t;

typedef struct { double d; int32_t v; } heap_item;

typedef struct {
  double *dist;
  uint8_t *done, *node_off, *arc_off;
  heap_item *heap; int hcap;
  int32_t *path_tmp;
} work_t;

static void heap_push(work_t *W, int *hn, double d, int32_t v) {
  int i = (*hn)++;
  heap_item *h = W->heap;
  while (i > 0) {
    int p = (i - 1) / 2;
    if (h[p].d <= d) break;
    h[i] = h[p]; i = p;
  }
  h[i].d = d; h[i].v = v;
}

static heap_item heap_pop(work_t *W, int *hn) {
  heap_item *h = W->heap;
  heap_item top = h[0];
  heap_item last = h[--(*hn)];
  int i = 0, n = *hn;
  for (;;) {
    int c = 2 * i + 1;
    if (c >= n) break;
    if (c + 1 < n && h[c + 1].d < h[c].d) c++;
    if (h[c].d >= last.d) break;
    h[i] = h[c]; i = c;
  }
  if (n > 0) h[i] = last;
  return top;
}

/* Lexicographically smallest shortest path s->t avoiding node_off/arc_off.
 * Writes node sequence into nodes (length returned, 0 if unreachable). */
static int spur_path(const graph_t *G, work_t *W, int s, int t, int32_t *nodes, double *cost) {
  int n = G->n;
  for (int i = 0; i < n; ++i) { W->dist[i] = INFINITY; W->done[i] = 0; }
  if (W->node_off[s] || W->node_off[t]) return 0;
  int hn = 0;
  W->dist[t] = 0.0;
  heap_push(W, &hn, 0.0, t);
  while (hn > 0) {
    heap_item it = heap_pop(W, &hn);
    int v = it.v;
    if (W->done[v] || it.d > W->dist[v]) continue;
    W->done[v] = 1;
    if (v == s) break;
    for (int k = G->in_ptr[v]; k < G->in_ptr[v + 1]; ++k) {
      int a = G->in_arc[k];
      if (W->arc_off[a]) continue;
      int u = G->src[a];
      if (W->node_off[u] || W->done[u]) continue;
      double nd = G->w[a] + W->dist[v];
      if (nd < W->dist[u]) { W->dist[u] = nd; heap_push(W, &hn, nd, u); }
    }
  }
  if (!W->done[s]) return 0;
  int len = 0, u = s;
  nodes[len++] = u;
  while (u != t) {
    int best = -1;
    for (int k = G->out_ptr[u]; k < G->out_ptr[u + 1]; ++k) {
      int a = G->out_arc[k];
      if (W->arc_off[a]) continue;
      int v = G->dst[a];
      if (W->node_off[v] || !W->done[v]) continue;
      if (G->w[a] + W->dist[v] == W->dist[u]) { if (best < 0 || v < best) best = v; }
    }
    if (best < 0) return 0; /* cannot happen with positive weights */
    u = best;
    nodes[len++] = u;
  }
  *cost = W->dist[s];
  return len;
}

static int find_arc(const graph_t *G, int u, int v) {
  for (int k = G->out_ptr[u]; k < G->out_ptr[u + 1]; ++k)
    if (G->dst[G->out_arc[k]] == v) return G->out_arc[k];
  return -1;
}

static double path_cost(const graph_t *G, const int32_t *nodes, int len) {
  double c = 0.0;
  for (int i = 0; i + 1 < len; ++i) c += G->w[find_arc(G, nodes[i], nodes[i + 1])];
  return c;
}

typedef struct { double cost; int len; int32_t *nodes; } cand_t;

static int cmp_path(double ca, const int32_t *a, int la, double cb, const int32_t *b, int lb) {
  if (ca < cb) return -1;
  if (ca > cb) return 1;
  int l = la < lb ? la : lb;
  for (int i = 0; i < l; ++i) { if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1; }
  return la < lb ? -1 : (la > lb ? 1 : 0);
}

static int same_seq(const int32_t *a, int la, const int32_t *b, int lb) {
  if (la != lb) return 0;
  return memcmp(a, b, sizeof(int32_t) * (size_t)la) == 0;
}

/* Yen for one pair.  out_nodes holds k*n ints (path j at offset j*n); out_len[k].
 * Returns the number of paths found (<= k). */
static int yen_pair(const graph_t *G, work_t *W, int s, int t, int k, int32_t *out_nodes, int32_t *out_len) {
  int n = G->n;
  memset(W->node_off, 0, (size_t)n);
  memset(W->arc_off, 0, (size_t)G->m);
  double c0;
  int l0 = spur_path(G, W, s, t, out_nodes, &c0);
  if (l0 == 0) return 0;
  out_len[0] = l0;
  int found = 1;
  int ncand = 0, capc = 16;
  cand_t *B = (cand_t *)malloc(sizeof(cand_t) * (size_t)capc);
  int32_t *sp = W->path_tmp;
  while (found < k) {
    const int32_t *prev = out_nodes + (size_t)(found - 1) * n;
    int lp = out_len[found - 1];
    for (int i = 0; i + 1 < lp; ++i) {
      int spur = prev[i];
      for (int j = 0; j < found; ++j) {
        const int32_t *pj = out_nodes + (size_t)j * n;
        if (out_len[j] > i + 1 && memcmp(pj, prev, sizeof(int32_t) * (size_t)(i + 1)) == 0) {
          int a = find_arc(G, pj[i], pj[i + 1]);
          if (a >= 0) W->arc_off[a] = 1;
        }
      }
      for (int j = 0; j < i; ++j) W->node_off[prev[j]] = 1;
      double cs;
      int ls = spur_path(G, W, spur, t, sp, &cs);
      for (int j = 0; j < i; ++j) W->node_off[prev[j]] = 0;
      memset(W->arc_off, 0, (size_t)G->m);
      if (ls == 0) continue;
      int lt = i + ls;
      int32_t *tot = (int32_t *)malloc(sizeof(int32_t) * (size_t)lt);
      memcpy(tot, prev, sizeof(int32_t) * (size_t)i);
      memcpy(tot + i, sp, sizeof(int32_t) * (size_t)ls);
      double ct = path_cost(G, tot, lt);
      int dup = 0;
      for (int j = 0; j < ncand && !dup; ++j) dup = same_seq(B[j].nodes, B[j].len, tot, lt);
      for (int j = 0; j < found && !dup; ++j) dup = same_seq(out_nodes + (size_t)j * n, out_len[j], tot, lt);
      if (dup) { free(tot); continue; }
      if (ncand == capc) { capc *= 2; B = (cand_t *)realloc(B, sizeof(cand_t) * (size_t)capc); }
      B[ncand].cost = ct; B[ncand].len = lt; B[ncand].nodes = tot; ncand++;
    }
    if (ncand == 0) break;
    int best = 0;
    for (int j = 1; j < ncand; ++j)
      if (cmp_path(B[j].cost, B[j].nodes, B[j].len, B[best].cost, B[best].nodes, B[best].len) < 0) best = j;
    memcpy(out_nodes + (size_t)found * n, B[best].nodes, sizeof(int32_t) * (size_t)B[best].len);
    out_len[found] = B[best].len;
    found++;
    free(B[best].nodes);
    B[best] = B[--ncand];
  }
  for (int j = 0; j < ncand; ++j) free(B[j].nodes);
  free(B);
  return found;
}

/*
 * Batch entry.  Arcs (src[a] -> dst[a], weight w[a] > 0); the caller gives the
 * forward CSR (out_ptr/out_arc) and reverse CSR (in_ptr/in_arc).
 * For pair q: k_per[q] paths from ps[q] to pt[q].  Output: npaths[q], and the
 * arc sequence of path j of pair q at out_arcs[(q*kmax + j)*(n-1) ...],
 * with its hop count in out_hops[q*kmax + j].
 */
int ksp_batch(int n, int m, const int32_t *src, const int32_t *dst, const double *w,
              const int32_t *out_ptr, const int32_t *out_arc, const int32_t *in_ptr, const int32_t *in_arc,
              int npairs, const int32_t *ps, const int32_t *pt, const int32_t *k_per, int kmax,
              int32_t *npaths, int32_t *out_hops, int32_t *out_arcs) {
  graph_t G = {n, m, out_ptr, out_arc, in_ptr, in_arc, src, dst, w};
  int err = 0;
#pragma omp parallel
  {
    work_t W;
    W.dist = (double *)malloc(sizeof(double) * (size_t)n);
    W.done = (uint8_t *)malloc((size_t)n);
    W.node_off = (uint8_t *)malloc((size_t)n);
    W.arc_off = (uint8_t *)malloc((size_t)m);
    W.hcap = m + n + 1;
    W.heap = (heap_item *)malloc(sizeof(heap_item) * (size_t)W.hcap);
    W.path_tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nodes = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax * n);
    int32_t *lens = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
#pragma omp for schedule(dynamic, 16)
    for (int q = 0; q < npairs; ++q) {
      int k = k_per[q] < kmax ? k_per[q] : kmax;
      int f = (ps[q] == pt[q] || k <= 0) ? 0 : yen_pair(&G, &W, ps[q], pt[q], k, nodes, lens);
      npaths[q] = f;
      for (int j = 0; j < f; ++j) {
        int hops = lens[j] - 1;
        out_hops[(size_t)q * kmax + j] = hops;
        int32_t *dstp = out_arcs + ((size_t)q * kmax + j) * (size_t)(n - 1);
        for (int h = 0; h < hops; ++h) {
          int a = find_arc(&G, nodes[(size_t)j * n + h], nodes[(size_t)j * n + h + 1]);
          if (a < 0) {
#pragma omp atomic write
            err = 1;
          }
          dstp[h] = a;
        }
      }
    }
    free(W.dist); free(W.done); free(W.node_off); free(W.arc_off); free(W.heap); free(W.path_tmp);
    free(nodes); free(lens);
  }
  return err;
}
