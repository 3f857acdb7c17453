/*
 * Block-pair flow problems around the cuts of a k-way partition (host code,
 * input generation only: no max-flow arithmetic lives here).
 *
 * Given a hypergraph and an initial k-way partition this builds what the
 * paper's refinement feeds to the flow solver (section "Network
 * Construction"): for a pair of adjacent blocks (Vi, Vj) a region Bi u Bj
 * grown by breadth-first search from the pins of the nets cut between the two
 * blocks, with the rest of Vi contracted into a source s and the rest of Vj
 * into a sink t.  Before that, a few rounds of label propagation refine the
 * random partition (section "Preliminaries" defines the connectivity
 * objective, sum over nets of w(e) (lambda(e) - 1)).
 *
 * Readings fixed here (the paper leaves them open):
 *  - label propagation visits vertices in id order; a vertex moves to the
 *    adjacent block with the largest positive connectivity gain among the
 *    blocks that stay within Lmax after the move (ties: smaller block id);
 *  - the cut size of a pair is the weight of the nets with pins in both
 *    blocks; pairs are ranked by cut weight (descending), then (i, j);
 *  - each side of a region grows level by level (each level in increasing
 *    vertex id order) while its weight stays within
 *    min(side_factor * cut, scale * ceil((c(Vi) + c(Vj)) / 2) - c(other))
 *    and it keeps at least one vertex of its block outside the region;
 *    growth stops at the first vertex that does not fit;
 *  - in the flow problem pins of other blocks are dropped, nets left with a
 *    single pin or with both s and t are dropped (the latter are cut by
 *    every bipartition of the region and do not change the improvement).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define EXPORT __attribute__((visibility("default")))

typedef struct {
  int32_t* mark;    /* V: region membership tag of a vertex */
  int32_t* local;   /* V: local id in the current region */
  int32_t* nmark;   /* E: net collected for the current region */
  int32_t* xmark;   /* E: net expanded by the BFS of a side */
  int32_t* lvl;     /* V: BFS level buffers */
  int32_t* nxt;
  int32_t* members; /* V */
  int32_t* nets;    /* E */
  int32_t stamp;
} Scratch;

typedef struct {
  int32_t nv, ne, n;
  int64_t np;
  int64_t info[14];
  int32_t* off;
  int32_t* pins;
  int32_t* w;
  int32_t* vw;
  int32_t* gid;
} Region;

typedef struct {
  int32_t V, E, k;
  int64_t P;
  const int32_t* off;
  const int32_t* pins;
  const int32_t* w;
  const int32_t* cv;
  int32_t* block;
  int64_t* bw;
  int64_t* bn;      /* k: vertices per block */
  int32_t* voff;
  int32_t* vnet;
  uint16_t* phi;    /* E * k pin counts per block */
  uint64_t* mask;   /* E: blocks holding a pin */
  int32_t* boff;    /* k+1: nets holding a pin of each block (built lazily) */
  int32_t* bnet;
  int32_t nreg;
  Region* reg;
} Ctx;

static void free_region(Region* r) {
  free(r->off); free(r->pins); free(r->w); free(r->vw); free(r->gid);
  memset(r, 0, sizeof(Region));
}

static void free_regions(Ctx* c) {
  for (int32_t r = 0; r < c->nreg; ++r) free_region(&c->reg[r]);
  free(c->reg);
  c->reg = NULL;
  c->nreg = 0;
}

EXPORT void hfr_free(Ctx* c) {
  if (!c) return;
  free_regions(c);
  free(c->block); free(c->bw); free(c->bn); free(c->voff); free(c->vnet); free(c->phi);
  free(c->mask); free(c->boff); free(c->bnet);
  free(c);
}

/* Returns NULL on invalid input or allocation failure.  Net sizes must stay
 * below 65536 and k in [2, 64]. */
EXPORT Ctx* hfr_new(int32_t V, int32_t E, const int32_t* off, const int32_t* pins,
                    const int32_t* w, const int32_t* cv, int32_t k, const int32_t* block0) {
  if (V < 2 || E < 0 || k < 2 || k > 64) return NULL;
  for (int32_t e = 0; e < E; ++e)
    if (off[e + 1] < off[e] || off[e + 1] - off[e] >= 65536) return NULL;
  Ctx* c = (Ctx*)calloc(1, sizeof(Ctx));
  if (!c) return NULL;
  c->V = V; c->E = E; c->k = k; c->P = off[E];
  c->off = off; c->pins = pins; c->w = w; c->cv = cv;
  c->block = (int32_t*)malloc(sizeof(int32_t) * V);
  c->bw = (int64_t*)calloc(k, sizeof(int64_t));
  c->bn = (int64_t*)calloc(k, sizeof(int64_t));
  c->voff = (int32_t*)calloc((size_t)V + 1, sizeof(int32_t));
  c->vnet = (int32_t*)malloc(sizeof(int32_t) * (c->P ? c->P : 1));
  c->phi = (uint16_t*)calloc((size_t)E * k + 1, sizeof(uint16_t));
  c->mask = (uint64_t*)calloc((size_t)E + 1, sizeof(uint64_t));
  if (!c->block || !c->bw || !c->bn || !c->voff || !c->vnet || !c->phi || !c->mask) {
    hfr_free(c);
    return NULL;
  }
  for (int32_t v = 0; v < V; ++v) {
    if (block0[v] < 0 || block0[v] >= k) { hfr_free(c); return NULL; }
    c->block[v] = block0[v];
    c->bw[block0[v]] += cv[v];
    c->bn[block0[v]] += 1;
  }
  for (int64_t p = 0; p < c->P; ++p) {
    if (pins[p] < 0 || pins[p] >= V) { hfr_free(c); return NULL; }
    c->voff[pins[p] + 1]++;
  }
  for (int32_t v = 0; v < V; ++v) c->voff[v + 1] += c->voff[v];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * V);
  if (!fill) { hfr_free(c); return NULL; }
  memcpy(fill, c->voff, sizeof(int32_t) * V);
  for (int32_t e = 0; e < E; ++e)
    for (int32_t p = off[e]; p < off[e + 1]; ++p) {
      const int32_t u = pins[p];
      c->vnet[fill[u]++] = e;  /* nets of a vertex in increasing id order */
      const int32_t b = c->block[u];
      if (c->phi[(size_t)e * k + b]++ == 0) c->mask[e] |= 1ull << b;
    }
  free(fill);
  return c;
}

/* Connectivity objective sum_e w(e) (lambda(e) - 1) over nets with pins. */
EXPORT int64_t hfr_objective(const Ctx* c) {
  int64_t s = 0;
  for (int32_t e = 0; e < c->E; ++e)
    if (c->mask[e]) s += (int64_t)c->w[e] * (__builtin_popcountll(c->mask[e]) - 1);
  return s;
}

/* `rounds` sweeps of label propagation; returns the number of moves. */
EXPORT int64_t hfr_lp(Ctx* c, int32_t rounds, int64_t lmax) {
  const int32_t k = c->k;
  int64_t conn[64];
  int64_t moves = 0;
  free(c->boff);
  free(c->bnet);
  c->boff = c->bnet = NULL;
  free_regions(c);
  for (int32_t r = 0; r < rounds; ++r) {
    for (int32_t v = 0; v < c->V; ++v) {
      const int32_t a = c->block[v];
      int64_t benefit = 0, W = 0;
      uint64_t adj = 0;
      for (int32_t b = 0; b < k; ++b) conn[b] = 0;
      for (int32_t i = c->voff[v]; i < c->voff[v + 1]; ++i) {
        const int32_t e = c->vnet[i];
        const int64_t we = c->w[e];
        W += we;
        if (c->phi[(size_t)e * k + a] == 1) benefit += we;
        uint64_t m = c->mask[e] & ~(1ull << a);
        adj |= m;
        while (m) {
          const int b = __builtin_ctzll(m);
          m &= m - 1;
          conn[b] += we;
        }
      }
      int32_t best = -1;
      int64_t best_gain = 0;
      uint64_t m = adj;
      while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1;
        const int64_t gain = benefit - W + conn[b];
        if (gain > best_gain && c->bw[b] + c->cv[v] <= lmax) {
          best_gain = gain;
          best = b;
        }
      }
      if (best < 0) continue;
      for (int32_t i = c->voff[v]; i < c->voff[v + 1]; ++i) {
        const int32_t e = c->vnet[i];
        uint16_t* ph = c->phi + (size_t)e * k;
        if (--ph[a] == 0) c->mask[e] &= ~(1ull << a);
        if (ph[best]++ == 0) c->mask[e] |= 1ull << best;
      }
      c->bw[a] -= c->cv[v];
      c->bw[best] += c->cv[v];
      c->bn[a] -= 1;
      c->bn[best] += 1;
      c->block[v] = best;
      ++moves;
    }
  }
  return moves;
}

EXPORT void hfr_blocks(const Ctx* c, int32_t* block, int64_t* bw) {
  memcpy(block, c->block, sizeof(int32_t) * c->V);
  memcpy(bw, c->bw, sizeof(int64_t) * c->k);
}

typedef struct {
  int64_t cut;
  int32_t i, j;
} Pair;

static int pair_cmp(const void* x, const void* y) {
  const Pair* a = (const Pair*)x;
  const Pair* b = (const Pair*)y;
  if (a->cut != b->cut) return a->cut > b->cut ? -1 : 1;
  if (a->i != b->i) return a->i < b->i ? -1 : 1;
  return a->j < b->j ? -1 : (a->j > b->j);
}

/* Adjacent block pairs with cut weight >= min_cut, heaviest first; at most
 * max_pairs are written.  Returns the number written. */
EXPORT int32_t hfr_pairs(const Ctx* c, int64_t min_cut, int32_t max_pairs, int32_t* pi,
                         int32_t* pj, int64_t* cut) {
  const int32_t k = c->k;
  int64_t* q = (int64_t*)calloc((size_t)k * k, sizeof(int64_t));
  Pair* all = (Pair*)malloc(sizeof(Pair) * (size_t)k * k);
  if (!q || !all) { free(q); free(all); return -1; }
  for (int32_t e = 0; e < c->E; ++e) {
    uint64_t m = c->mask[e];
    if (__builtin_popcountll(m) < 2) continue;
    while (m) {
      const int i = __builtin_ctzll(m);
      m &= m - 1;
      uint64_t r = m;
      while (r) {
        const int j = __builtin_ctzll(r);
        r &= r - 1;
        q[i * k + j] += c->w[e];
      }
    }
  }
  int32_t n = 0;
  for (int32_t i = 0; i < k; ++i)
    for (int32_t j = i + 1; j < k; ++j)
      if (q[i * k + j] >= min_cut && q[i * k + j] > 0) {
        all[n].cut = q[i * k + j];
        all[n].i = i;
        all[n].j = j;
        ++n;
      }
  qsort(all, n, sizeof(Pair), pair_cmp);
  if (n > max_pairs) n = max_pairs;
  for (int32_t t = 0; t < n; ++t) {
    pi[t] = all[t].i;
    pj[t] = all[t].j;
    cut[t] = all[t].cut;
  }
  free(q);
  free(all);
  return n;
}

static int int_cmp(const void* x, const void* y) {
  const int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}

/* Nets holding a pin of each block (CSR over blocks, increasing net id). */
static int build_block_nets(Ctx* c) {
  if (c->boff) return 0;
  const int32_t k = c->k;
  int64_t total = 0;
  for (int32_t e = 0; e < c->E; ++e) total += __builtin_popcountll(c->mask[e]);
  if (total >= (1ll << 31)) return -1;
  c->boff = (int32_t*)calloc((size_t)k + 1, sizeof(int32_t));
  c->bnet = (int32_t*)malloc(sizeof(int32_t) * ((size_t)total + 1));
  if (!c->boff || !c->bnet) return -1;
  for (int32_t e = 0; e < c->E; ++e) {
    uint64_t m = c->mask[e];
    while (m) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      c->boff[b + 1]++;
    }
  }
  for (int32_t b = 0; b < k; ++b) c->boff[b + 1] += c->boff[b];
  int32_t fill[64];
  for (int32_t b = 0; b < k; ++b) fill[b] = c->boff[b];
  for (int32_t e = 0; e < c->E; ++e) {
    uint64_t m = c->mask[e];
    while (m) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      c->bnet[fill[b]++] = e;
    }
  }
  return 0;
}

static void free_scratch(Scratch* s) {
  free(s->mark); free(s->local); free(s->nmark); free(s->xmark);
  free(s->lvl); free(s->nxt); free(s->members); free(s->nets);
}

static int alloc_scratch(const Ctx* c, Scratch* s) {
  memset(s, 0, sizeof(Scratch));
  s->mark = (int32_t*)calloc(c->V, sizeof(int32_t));
  s->local = (int32_t*)malloc(sizeof(int32_t) * c->V);
  s->nmark = (int32_t*)calloc((size_t)c->E + 1, sizeof(int32_t));
  s->xmark = (int32_t*)calloc((size_t)c->E + 1, sizeof(int32_t));
  s->lvl = (int32_t*)malloc(sizeof(int32_t) * c->V);
  s->nxt = (int32_t*)malloc(sizeof(int32_t) * c->V);
  s->members = (int32_t*)malloc(sizeof(int32_t) * c->V);
  s->nets = (int32_t*)malloc(sizeof(int32_t) * ((size_t)c->E + 1));
  if (!s->mark || !s->local || !s->nmark || !s->xmark || !s->lvl || !s->nxt || !s->members ||
      !s->nets) {
    free_scratch(s);
    return -1;
  }
  return 0;
}

/* Grow one side: BFS inside block `blk` from its pins on the nets cut
 * between blocks i and j, adding vertices (mark = tag) to s->members while
 * the side stays within cap_w weight and cap_n vertices.  Returns the
 * side's weight; *boundary counts the level-0 vertices. */
static int64_t grow_side(const Ctx* c, Scratch* s, int32_t blk, int32_t i, int32_t j,
                         int64_t cap_w, int64_t cap_n, int32_t tag, int32_t* nm,
                         int64_t* boundary) {
  int32_t nl = 0;
  /* level 0: pins of blk on cut nets, increasing id */
  for (int32_t q = c->boff[blk]; q < c->boff[blk + 1]; ++q) {
    const int32_t e = c->bnet[q];
    const uint64_t m = c->mask[e];
    if (!((m >> i) & 1) || !((m >> j) & 1)) continue;
    for (int32_t p = c->off[e]; p < c->off[e + 1]; ++p) {
      const int32_t u = c->pins[p];
      if (c->block[u] == blk && s->mark[u] != -tag) {
        s->mark[u] = -tag;  /* queued */
        s->lvl[nl++] = u;
      }
    }
  }
  *boundary += nl;
  qsort(s->lvl, nl, sizeof(int32_t), int_cmp);
  int64_t wsum = 0, cnt = 0;
  int stop = 0;
  while (nl > 0) {
    int32_t added = 0;
    for (int32_t t = 0; t < nl; ++t) {
      const int32_t u = s->lvl[t];
      if (wsum + c->cv[u] > cap_w || cnt + 1 > cap_n) { stop = 1; break; }
      s->mark[u] = tag;
      wsum += c->cv[u];
      ++cnt;
      s->members[(*nm)++] = u;
      s->lvl[added++] = u;
    }
    if (stop) break;
    /* next level: unqueued block neighbours of the added vertices */
    int32_t nn = 0;
    for (int32_t t = 0; t < added; ++t) {
      const int32_t u = s->lvl[t];
      for (int32_t a = c->voff[u]; a < c->voff[u + 1]; ++a) {
        const int32_t e = c->vnet[a];
        if (s->xmark[e] == tag) continue;  /* its block pins are queued already */
        s->xmark[e] = tag;
        for (int32_t p = c->off[e]; p < c->off[e + 1]; ++p) {
          const int32_t x = c->pins[p];
          if (c->block[x] == blk && s->mark[x] != tag && s->mark[x] != -tag) {
            s->mark[x] = -tag;
            s->nxt[nn++] = x;
          }
        }
      }
    }
    qsort(s->nxt, nn, sizeof(int32_t), int_cmp);
    memcpy(s->lvl, s->nxt, sizeof(int32_t) * nn);
    nl = nn;
  }
  return wsum;
}

/* Build the flow problem of pair (i, j) into r.  r->info receives
 * [nv, ne, np, cut_before, boundary, side_i_weight, side_j_weight,
 *  bins 0..6].  Returns 0, or -1 on allocation failure. */
static int build_region(const Ctx* c, Scratch* s, Region* r, int32_t i, int32_t j, int64_t cut,
                        int64_t side_factor, int64_t scale_num, int64_t scale_den) {
  /* fresh tags: 2*stamp+1 (side i), 2*stamp+2 (side j); queued = negative */
  s->stamp += 1;
  if (s->stamp > (1 << 29)) {
    memset(s->mark, 0, sizeof(int32_t) * c->V);
    memset(s->nmark, 0, sizeof(int32_t) * ((size_t)c->E + 1));
    memset(s->xmark, 0, sizeof(int32_t) * ((size_t)c->E + 1));
    s->stamp = 1;
  }
  const int32_t ti = 2 * s->stamp + 1, tj = 2 * s->stamp + 2;
  const int64_t cvi = c->bw[i], cvj = c->bw[j];
  const int64_t half = (cvi + cvj + 1) / 2;
  const int64_t lim = scale_num * half / scale_den;
  int64_t capi = side_factor * cut, capj = side_factor * cut;
  if (lim - cvj < capi) capi = lim - cvj;
  if (lim - cvi < capj) capj = lim - cvi;
  if (capi < 0) capi = 0;
  if (capj < 0) capj = 0;
  int32_t nm = 0;
  int64_t boundary = 0;
  const int64_t wi = grow_side(c, s, i, i, j, capi, c->bn[i] - 1, ti, &nm, &boundary);
  const int64_t wj = grow_side(c, s, j, i, j, capj, c->bn[j] - 1, tj, &nm, &boundary);
  /* region vertices in increasing global id; local ids 0..n-1, s = n, t = n+1 */
  qsort(s->members, nm, sizeof(int32_t), int_cmp);
  const int32_t n = nm;
  for (int32_t t = 0; t < n; ++t) s->local[s->members[t]] = t;
  /* nets touching the region, increasing id */
  int32_t ne_touch = 0;
  const int32_t nt = s->stamp;
  for (int32_t t = 0; t < n; ++t) {
    const int32_t u = s->members[t];
    for (int32_t a = c->voff[u]; a < c->voff[u + 1]; ++a) {
      const int32_t e = c->vnet[a];
      if (s->nmark[e] != nt) {
        s->nmark[e] = nt;
        s->nets[ne_touch++] = e;
      }
    }
  }
  qsort(s->nets, ne_touch, sizeof(int32_t), int_cmp);
  int64_t pin_cap = 0;
  for (int32_t t = 0; t < ne_touch; ++t) pin_cap += c->off[s->nets[t] + 1] - c->off[s->nets[t]] + 2;
  r->off = (int32_t*)malloc(sizeof(int32_t) * ((size_t)ne_touch + 1));
  r->w = (int32_t*)malloc(sizeof(int32_t) * ((size_t)ne_touch + 1));
  r->vw = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 2));
  r->gid = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  r->pins = (int32_t*)malloc(sizeof(int32_t) * ((size_t)pin_cap + 1));
  if (!r->off || !r->w || !r->vw || !r->gid || !r->pins) return -1;
  int64_t np = 0, cut_before = 0, bins[7] = {0, 0, 0, 0, 0, 0, 0};
  int32_t ne = 0;
  r->off[0] = 0;
  for (int32_t t = 0; t < ne_touch; ++t) {
    const int32_t e = s->nets[t];
    const int64_t start = np;
    int has_s = 0, has_t = 0, in_i = 0, in_j = 0;
    for (int32_t p = c->off[e]; p < c->off[e + 1]; ++p) {
      const int32_t u = c->pins[p];
      const int32_t b = c->block[u];
      if (s->mark[u] == ti) { r->pins[np++] = s->local[u]; in_i = 1; }
      else if (s->mark[u] == tj) { r->pins[np++] = s->local[u]; in_j = 1; }
      else if (b == i) has_s = 1;
      else if (b == j) has_t = 1;
    }
    if (has_s) r->pins[np++] = n;
    if (has_t) r->pins[np++] = n + 1;
    const int64_t sz = np - start;
    if (sz < 2 || (has_s && has_t)) {
      np = start;
      continue;
    }
    if ((in_i || has_s) && (in_j || has_t)) cut_before += c->w[e];
    const int bin = sz <= 2 ? 0 : sz <= 4 ? 1 : sz <= 8 ? 2 : sz <= 16 ? 3 : sz <= 64 ? 4 : sz <= 256 ? 5 : 6;
    bins[bin]++;
    r->w[ne] = c->w[e];
    r->off[++ne] = (int32_t)np;
  }
  for (int32_t t = 0; t < n; ++t) {
    r->vw[t] = c->cv[s->members[t]];
    r->gid[t] = s->members[t];
  }
  r->vw[n] = (int32_t)(cvi - wi);
  r->vw[n + 1] = (int32_t)(cvj - wj);
  r->n = n;
  r->nv = n + 2;
  r->ne = ne;
  r->np = np;
  r->info[0] = r->nv;
  r->info[1] = r->ne;
  r->info[2] = r->np;
  r->info[3] = cut_before;
  r->info[4] = boundary;
  r->info[5] = wi;
  r->info[6] = wj;
  for (int b = 0; b < 7; ++b) r->info[7 + b] = bins[b];
  return 0;
}

/* Build the flow problems of pairs (pi[t], pj[t]) with cut weights cut[t]
 * on `threads` threads (<= 0: OpenMP default).  Regions are independent;
 * each thread keeps its own scratch.  Returns 0, or -1 on allocation
 * failure. */
EXPORT int32_t hfr_regions(Ctx* c, int32_t n, const int32_t* pi, const int32_t* pj,
                           const int64_t* cut, int64_t side_factor, int64_t scale_num,
                           int64_t scale_den, int32_t threads) {
  free_regions(c);
  if (build_block_nets(c)) return -1;
  c->reg = (Region*)calloc(n > 0 ? n : 1, sizeof(Region));
  if (!c->reg) return -1;
  c->nreg = n;
  int failed = 0;
  const int nth = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nth) reduction(| : failed)
  {
    Scratch s;
    if (alloc_scratch(c, &s)) {
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int32_t t = 0; t < n; ++t)
        if (build_region(c, &s, &c->reg[t], pi[t], pj[t], cut[t], side_factor, scale_num,
                         scale_den))
          failed = 1;
      free_scratch(&s);
    }
  }
  return failed ? -1 : 0;
}

EXPORT void hfr_region_info(const Ctx* c, int32_t r, int64_t* info) {
  memcpy(info, c->reg[r].info, sizeof(int64_t) * 14);
}

/* Copy region r out: off[ne+1], pins[np], w[ne], vw[nv], gid[nv-2] (global
 * id of each region vertex), then release its buffers. */
EXPORT void hfr_region_take(Ctx* c, int32_t r, int32_t* off, int32_t* pins, int32_t* w,
                            int32_t* vw, int32_t* gid) {
  Region* g = &c->reg[r];
  memcpy(off, g->off, sizeof(int32_t) * ((size_t)g->ne + 1));
  memcpy(pins, g->pins, sizeof(int32_t) * (size_t)g->np);
  memcpy(w, g->w, sizeof(int32_t) * (size_t)g->ne);
  memcpy(vw, g->vw, sizeof(int32_t) * (size_t)g->nv);
  memcpy(gid, g->gid, sizeof(int32_t) * (size_t)g->n);
  free_region(g);
}
