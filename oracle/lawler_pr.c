/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  It shares nothing with the HIP library: it builds the
 * Lawler expansion explicitly, as an ordinary directed graph with paired
 * residual arcs, and runs a textbook sequential FIFO push-relabel on it.
 *
 * What it computes (paper, section "Preliminaries", paragraphs "Flows",
 * "Push-Relabel Algorithm" and "Flows on Hypergraphs"):
 *
 *   Nodes    v in [0,V)            hypernodes
 *            ein  = V + e          net in-node
 *            eout = V + E + e      net out-node
 *            sig  = V + 2E         super source (contracts S)
 *            tau  = V + 2E + 1     super sink   (contracts T)
 *   Arcs     (v, ein)  INF  and (eout, v) INF for every pin v of e
 *            (ein, eout) w(e)      bridging arc
 *            (sig, v) INF for v in S,  (v, tau) INF for v in T
 *   INF      1 + sum of all net weights, which exceeds the weight of every
 *            finite cut, so no minimum cut ever uses an INF arc.
 *
 * Algorithm: push / relabel with the discharge routine and FIFO selection of
 * active nodes; global relabeling (exact labels by reverse residual BFS from
 * the sink) at the start and after every n relabels.  It stops once no node
 * with positive excess has a label below n ("cuts only" termination: the
 * maximum preflow already determines the minimum cut).  The flow value is
 * the excess collected at tau.
 *
 * Source side (section "Intricacies with Preflows and FlowCutter",
 * paragraph "Source-Side Cut"): forward residual BFS seeded with sig and all
 * non-terminal nodes that still hold excess.  The reached set is the unique
 * inclusion-minimal source side of a minimum cut.
 *
 * Sink side (same section, algorithm "FlowCutter Core": the sink-side cut is
 * the reverse residual BFS from T): every node that can still reach tau in
 * the residual network.  Its vertices form the unique inclusion-maximal sink
 * side of a minimum cut (the complement of the union of all minimum-cut
 * source sides).
 *
 * Optional self-check (flag bit 0): convert the preflow into a flow by
 * continuing push / relabel above label n until every excess has returned to
 * sig, then BFS from sig alone and require the identical reached set.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  OR_OK = 0,
  OR_ERR_ALLOC = -1,
  OR_ERR_SINK_REACHED = -2,
  OR_ERR_SELFCHECK = -3,
  OR_ERR_INPUT = -4,
  OR_ERR_CONSERVATION = -5
};

typedef struct {
  int32_t n;        /* number of nodes */
  int64_t m;        /* number of arcs (each original arc gives two) */
  int64_t *first;   /* n + 1 offsets into the arc arrays */
  int32_t *head;    /* arc -> head node */
  int64_t *rev;     /* arc -> paired reverse arc */
  int64_t *cap;     /* arc -> residual capacity */
} graph_t;

static void graph_free(graph_t *g) {
  free(g->first);
  free(g->head);
  free(g->rev);
  free(g->cap);
}

/* Build the explicit Lawler network.  Returns 0 or an error code. */
static int build_lawler(graph_t *g, int32_t V, int32_t E, const int32_t *off,
                        const int32_t *pins, const int32_t *w, const int32_t *S,
                        int32_t nS, const int32_t *T, int32_t nT, int64_t *inf_out) {
  int64_t P = off[E];
  int32_t n = V + 2 * E + 2;
  int32_t sig = V + 2 * E, tau = sig + 1;
  int64_t inf = 1;
  for (int32_t e = 0; e < E; ++e) inf += w[e];
  *inf_out = inf;

  int64_t narcs = 2 * P + E + nS + nT; /* original arcs */
  g->n = n;
  g->m = 2 * narcs;
  g->first = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->head = (int32_t *)malloc((size_t)g->m * sizeof(int32_t));
  g->rev = (int64_t *)malloc((size_t)g->m * sizeof(int64_t));
  g->cap = (int64_t *)malloc((size_t)g->m * sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!g->first || !g->head || !g->rev || !g->cap || !fill) {
    free(fill);
    return OR_ERR_ALLOC;
  }
  /* pass 1: out-degree in the residual graph (each arc counts at both ends) */
#define COUNT_ARC(a, b) do { g->first[(a) + 1]++; g->first[(b) + 1]++; } while (0)
  for (int32_t e = 0; e < E; ++e) {
    int32_t ein = V + e, eout = V + E + e;
    for (int64_t p = off[e]; p < off[e + 1]; ++p) {
      COUNT_ARC(pins[p], ein);
      COUNT_ARC(eout, pins[p]);
    }
    COUNT_ARC(ein, eout);
  }
  for (int32_t i = 0; i < nS; ++i) COUNT_ARC(sig, S[i]);
  for (int32_t i = 0; i < nT; ++i) COUNT_ARC(T[i], tau);
#undef COUNT_ARC
  for (int32_t v = 0; v < n; ++v) g->first[v + 1] += g->first[v];
  memcpy(fill, g->first, ((size_t)n + 1) * sizeof(int64_t));
  /* pass 2: place each arc and its reverse */
#define ADD_ARC(a, b, c) do {                                   \
    int64_t fa = fill[(a)]++, fb = fill[(b)]++;                  \
    g->head[fa] = (b); g->cap[fa] = (c); g->rev[fa] = fb;         \
    g->head[fb] = (a); g->cap[fb] = 0;   g->rev[fb] = fa;         \
  } while (0)
  for (int32_t e = 0; e < E; ++e) {
    int32_t ein = V + e, eout = V + E + e;
    for (int64_t p = off[e]; p < off[e + 1]; ++p) {
      ADD_ARC(pins[p], ein, inf);
      ADD_ARC(eout, pins[p], inf);
    }
    ADD_ARC(ein, eout, (int64_t)w[e]);
  }
  for (int32_t i = 0; i < nS; ++i) ADD_ARC(sig, S[i], inf);
  for (int32_t i = 0; i < nT; ++i) ADD_ARC(T[i], tau, inf);
#undef ADD_ARC
  free(fill);
  (void)tau;
  return OR_OK;
}

typedef struct {
  graph_t *g;
  int32_t sig, tau, n;
  int64_t *exc;
  int32_t *d;
  int64_t *cur;
  int32_t *queue; /* FIFO ring of active nodes */
  int64_t qhead, qtail, qcap;
  uint8_t *inq;
  int32_t *bfs;
  int64_t relabels, pushes, global_relabels, since_global;
} pr_t;

static void q_push(pr_t *s, int32_t v) {
  s->queue[s->qtail % s->qcap] = v;
  s->qtail++;
  s->inq[v] = 1;
}

static int32_t q_pop(pr_t *s) {
  int32_t v = s->queue[s->qhead % s->qcap];
  s->qhead++;
  s->inq[v] = 0;
  return v;
}

static int is_active(const pr_t *s, int32_t v) {
  return v != s->sig && v != s->tau && s->exc[v] > 0 && s->d[v] < s->n;
}

/* Exact labels: d(v) = residual distance from v to tau (reverse BFS), n when
 * tau is unreachable; d(sig) stays n.  Rebuilds the active queue. */
static void global_relabel(pr_t *s) {
  graph_t *g = s->g;
  int32_t n = s->n;
  for (int32_t v = 0; v < n; ++v) s->d[v] = n;
  s->d[s->tau] = 0;
  int64_t h = 0, t = 0;
  s->bfs[t++] = s->tau;
  while (h < t) {
    int32_t x = s->bfs[h++];
    for (int64_t a = g->first[x]; a < g->first[x + 1]; ++a) {
      int32_t y = g->head[a];
      /* arc (y, x) is rev[a]; y reaches x if it has residual capacity */
      if (y != s->sig && s->d[y] == n && g->cap[g->rev[a]] > 0) {
        s->d[y] = s->d[x] + 1;
        s->bfs[t++] = y;
      }
    }
  }
  s->d[s->sig] = n;
  for (int32_t v = 0; v < n; ++v) s->cur[v] = g->first[v];
  s->qhead = s->qtail = 0;
  for (int32_t v = 0; v < n; ++v) s->inq[v] = 0;
  for (int32_t v = 0; v < n; ++v)
    if (is_active(s, v)) q_push(s, v);
  s->global_relabels++;
  s->since_global = 0;
}

/* Discharge u: push along admissible arcs; when the scan is exhausted,
 * relabel to 1 + min label over residual arcs (capped at `limit`). */
static void discharge(pr_t *s, int32_t u, int32_t limit, int requeue_above_n) {
  graph_t *g = s->g;
  while (s->exc[u] > 0) {
    if (s->cur[u] == g->first[u + 1]) {
      int64_t m = INT64_MAX;
      for (int64_t a = g->first[u]; a < g->first[u + 1]; ++a)
        if (g->cap[a] > 0 && (int64_t)s->d[g->head[a]] + 1 < m) m = s->d[g->head[a]] + 1;
      s->d[u] = (m > limit) ? limit : (int32_t)m;
      s->cur[u] = g->first[u];
      s->relabels++;
      s->since_global++;
      if (s->d[u] >= limit) break;
      continue;
    }
    int64_t a = s->cur[u];
    int32_t v = g->head[a];
    if (g->cap[a] > 0 && s->d[u] == s->d[v] + 1) {
      int64_t delta = s->exc[u] < g->cap[a] ? s->exc[u] : g->cap[a];
      g->cap[a] -= delta;
      g->cap[g->rev[a]] += delta;
      s->exc[u] -= delta;
      s->exc[v] += delta;
      s->pushes++;
      if (v != s->sig && v != s->tau && !s->inq[v] &&
          (requeue_above_n || s->d[v] < s->n))
        q_push(s, v);
    } else {
      s->cur[u]++;
    }
  }
}

/* Forward residual BFS from the given seeds; marks reached nodes. */
static void forward_bfs(pr_t *s, uint8_t *reached, int seed_excess) {
  graph_t *g = s->g;
  int64_t h = 0, t = 0;
  memset(reached, 0, (size_t)s->n);
  reached[s->sig] = 1;
  s->bfs[t++] = s->sig;
  if (seed_excess)
    for (int32_t v = 0; v < s->n; ++v)
      if (v != s->sig && v != s->tau && s->exc[v] > 0 && !reached[v]) {
        reached[v] = 1;
        s->bfs[t++] = v;
      }
  while (h < t) {
    int32_t x = s->bfs[h++];
    for (int64_t a = g->first[x]; a < g->first[x + 1]; ++a) {
      int32_t y = g->head[a];
      if (!reached[y] && g->cap[a] > 0) {
        reached[y] = 1;
        s->bfs[t++] = y;
      }
    }
  }
}

/* Reverse residual BFS from tau: marks every node with a residual path to
 * tau.  A node a joins when some arc (a, b) with b marked has residual
 * capacity; that arc is the pair of an arc stored at b. */
static void reverse_bfs(pr_t *s, uint8_t *reaches) {
  graph_t *g = s->g;
  int64_t h = 0, t = 0;
  memset(reaches, 0, (size_t)s->n);
  reaches[s->tau] = 1;
  s->bfs[t++] = s->tau;
  while (h < t) {
    int32_t b = s->bfs[h++];
    for (int64_t x = g->first[b]; x < g->first[b + 1]; ++x) {
      int32_t a = g->head[x];
      if (!reaches[a] && g->cap[g->rev[x]] > 0) {
        reaches[a] = 1;
        s->bfs[t++] = a;
      }
    }
  }
}

static int solve(int32_t V, int32_t E, const int32_t *off, const int32_t *pins, const int32_t *w,
                 const int32_t *S, int32_t nS, const int32_t *T, int32_t nT, int32_t flags,
                 int64_t *F, uint8_t *vside, uint8_t *nside, uint8_t *tside, int64_t *stats);

/*
 * oracle_maxflow: minimum S-T cut of a hypergraph via its Lawler expansion.
 *
 *   flags bit 0 : self-check by converting the preflow into a flow.
 *   F           : out, maximum flow value = minimum cut weight.
 *   vside[V]    : out, 1 if the vertex is on the minimal source side.
 *   nside[E]    : out, bit 0 = ein reached, bit 1 = eout reached.
 *   stats[8]    : out (may be NULL): relabels, pushes, global relabels,
 *                 nodes, arcs, INF value, -, -.
 * Returns 0, or a negative OR_ERR_* code.
 */
int oracle_maxflow(int32_t V, int32_t E, const int32_t *off, const int32_t *pins,
                   const int32_t *w, const int32_t *S, int32_t nS, const int32_t *T,
                   int32_t nT, int32_t flags, int64_t *F, uint8_t *vside,
                   uint8_t *nside, int64_t *stats) {
  return solve(V, E, off, pins, w, S, nS, T, nT, flags, F, vside, nside, NULL, stats);
}

/* As oracle_maxflow, and tside[V] (may be NULL): 1 if the vertex is on the
 * maximal sink side (reaches tau in the residual network). */
int oracle_maxflow_sides(int32_t V, int32_t E, const int32_t *off, const int32_t *pins,
                         const int32_t *w, const int32_t *S, int32_t nS, const int32_t *T,
                         int32_t nT, int32_t flags, int64_t *F, uint8_t *vside,
                         uint8_t *nside, uint8_t *tside, int64_t *stats) {
  return solve(V, E, off, pins, w, S, nS, T, nT, flags, F, vside, nside, tside, stats);
}

static int solve(int32_t V, int32_t E, const int32_t *off, const int32_t *pins, const int32_t *w,
                 const int32_t *S, int32_t nS, const int32_t *T, int32_t nT, int32_t flags,
                 int64_t *F, uint8_t *vside, uint8_t *nside, uint8_t *tside, int64_t *stats) {
  if (V < 0 || E < 0 || nS < 1 || nT < 1 || off[0] != 0) return OR_ERR_INPUT;
  for (int32_t e = 0; e < E; ++e)
    if (off[e + 1] < off[e] || w[e] < 1) return OR_ERR_INPUT;
  for (int64_t p = 0; p < off[E]; ++p)
    if (pins[p] < 0 || pins[p] >= V) return OR_ERR_INPUT;

  graph_t g;
  memset(&g, 0, sizeof(g));
  int64_t inf = 0;
  int rc = build_lawler(&g, V, E, off, pins, w, S, nS, T, nT, &inf);
  if (rc) {
    graph_free(&g);
    return rc;
  }
  pr_t s;
  memset(&s, 0, sizeof(s));
  s.g = &g;
  s.n = g.n;
  s.sig = V + 2 * E;
  s.tau = s.sig + 1;
  s.exc = (int64_t *)calloc((size_t)s.n, sizeof(int64_t));
  s.d = (int32_t *)calloc((size_t)s.n, sizeof(int32_t));
  s.cur = (int64_t *)malloc((size_t)s.n * sizeof(int64_t));
  s.qcap = s.n;
  s.queue = (int32_t *)malloc((size_t)s.qcap * sizeof(int32_t));
  s.inq = (uint8_t *)calloc((size_t)s.n, 1);
  s.bfs = (int32_t *)malloc((size_t)s.n * sizeof(int32_t));
  uint8_t *reached = (uint8_t *)malloc((size_t)s.n);
  uint8_t *reached2 = NULL;
  if (!s.exc || !s.d || !s.cur || !s.queue || !s.inq || !s.bfs || !reached) {
    rc = OR_ERR_ALLOC;
    goto done;
  }

  /* initial preflow: saturate every arc leaving the source */
  s.d[s.sig] = s.n;
  for (int64_t a = g.first[s.sig]; a < g.first[s.sig + 1]; ++a) {
    int64_t c = g.cap[a];
    g.cap[a] = 0;
    g.cap[g.rev[a]] += c;
    s.exc[g.head[a]] += c;
  }
  global_relabel(&s);
  for (;;) {
    while (s.qhead != s.qtail) {
      int32_t u = q_pop(&s);
      if (!is_active(&s, u)) continue;
      discharge(&s, u, s.n, 0);
      if (s.since_global >= s.n) global_relabel(&s);
    }
    /* empty queue: confirm with exact labels, continue if anything is left */
    global_relabel(&s);
    if (s.qhead == s.qtail) break;
  }
  *F = s.exc[s.tau];

  forward_bfs(&s, reached, 1);
  if (reached[s.tau]) {
    rc = OR_ERR_SINK_REACHED;
    goto done;
  }
  for (int32_t v = 0; v < V; ++v) vside[v] = reached[v];
  for (int32_t e = 0; e < E; ++e)
    nside[e] = (uint8_t)(reached[V + e] | (reached[V + E + e] << 1));
  if (tside) {
    uint8_t *reaches = (uint8_t *)malloc((size_t)s.n);
    if (!reaches) {
      rc = OR_ERR_ALLOC;
      goto done;
    }
    reverse_bfs(&s, reaches);
    int clash = reaches[s.sig];
    for (int32_t v = 0; v < V; ++v) {
      tside[v] = reaches[v];
      clash |= reaches[v] & reached[v];
    }
    free(reaches);
    if (clash) {
      rc = OR_ERR_SINK_REACHED; /* a source-side node reaches the sink */
      goto done;
    }
  }

  if (flags & 1) {
    /* Return every remaining excess to the source: labels may now exceed n;
     * relabel bound 2n keeps the textbook termination argument. */
    int32_t limit = 2 * s.n;
    s.qhead = s.qtail = 0;
    for (int32_t v = 0; v < s.n; ++v) {
      s.inq[v] = 0;
      s.cur[v] = g.first[v];
    }
    for (int32_t v = 0; v < s.n; ++v)
      if (v != s.sig && v != s.tau && s.exc[v] > 0) q_push(&s, v);
    while (s.qhead != s.qtail) {
      int32_t u = q_pop(&s);
      if (u == s.sig || u == s.tau || s.exc[u] <= 0) continue;
      discharge(&s, u, limit, 1);
      if (s.exc[u] > 0 && !s.inq[u]) {
        rc = OR_ERR_SELFCHECK; /* excess stuck although a path to sig exists */
        goto done;
      }
    }
    for (int32_t v = 0; v < s.n; ++v)
      if (v != s.sig && v != s.tau && s.exc[v] != 0) {
        rc = OR_ERR_CONSERVATION;
        goto done;
      }
    if (s.exc[s.tau] != *F) {
      rc = OR_ERR_SELFCHECK;
      goto done;
    }
    reached2 = (uint8_t *)malloc((size_t)s.n);
    if (!reached2) {
      rc = OR_ERR_ALLOC;
      goto done;
    }
    forward_bfs(&s, reached2, 0);
    if (memcmp(reached, reached2, (size_t)s.n) != 0) {
      rc = OR_ERR_SELFCHECK;
      goto done;
    }
  }
  if (stats) {
    stats[0] = s.relabels;
    stats[1] = s.pushes;
    stats[2] = s.global_relabels;
    stats[3] = s.n;
    stats[4] = g.m;
    stats[5] = inf;
    stats[6] = 0;
    stats[7] = 0;
  }
  rc = OR_OK;
done:
  free(reached);
  free(reached2);
  free(s.exc);
  free(s.d);
  free(s.cur);
  free(s.queue);
  free(s.inq);
  free(s.bfs);
  graph_free(&g);
  return rc;
}
