/* Host C under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
 * oracle (oracle/lawler_pr.c) and the block-pair workload builder
 * (paper_2201_01556_amd/regions.c) run on seeded random inputs; any memory
 * error or undefined behaviour aborts the program.  Built and run by
 * tests/test_sanitizers.py. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_maxflow_sides(int32_t V, int32_t E, const int32_t *off, const int32_t *pins,
                         const int32_t *w, const int32_t *S, int32_t nS, const int32_t *T,
                         int32_t nT, int32_t flags, int64_t *F, uint8_t *vside,
                         uint8_t *nside, uint8_t *tside, int64_t *stats);

typedef struct Ctx Ctx;
Ctx *hfr_new(int32_t V, int32_t E, const int32_t *off, const int32_t *pins, const int32_t *w,
             const int32_t *cv, int32_t k, const int32_t *block0);
void hfr_free(Ctx *c);
int64_t hfr_objective(const Ctx *c);
int64_t hfr_lp(Ctx *c, int32_t rounds, int64_t lmax);
void hfr_blocks(const Ctx *c, int32_t *block, int64_t *bw);
int32_t hfr_pairs(const Ctx *c, int64_t min_cut, int32_t max_pairs, int32_t *pi, int32_t *pj,
                  int64_t *cut);
int32_t hfr_regions(Ctx *c, int32_t n, const int32_t *pi, const int32_t *pj, const int64_t *cut,
                    int64_t side_factor, int64_t scale_num, int64_t scale_den, int32_t threads);
void hfr_region_info(const Ctx *c, int32_t r, int64_t *info);
void hfr_region_take(Ctx *c, int32_t r, int32_t *off, int32_t *pins, int32_t *w, int32_t *vw,
                     int32_t *gid);

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(uint32_t n) {  /* xorshift64 */
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return (uint32_t)(rs % n);
}

/* random hypergraph with distinct pins per net */
static void random_hypergraph(int32_t V, int32_t E, int32_t smax, int32_t **off_o,
                              int32_t **pins_o) {
  int32_t *off = malloc(sizeof(int32_t) * (E + 1));
  int32_t *pins = malloc(sizeof(int32_t) * (size_t)E * smax);
  uint8_t *used = calloc(V, 1);
  off[0] = 0;
  for (int32_t e = 0; e < E; ++e) {
    int32_t s = 1 + rnd(smax < V ? smax : V);
    int32_t n = 0;
    while (n < s) {
      int32_t v = rnd(V);
      if (used[v]) continue;
      used[v] = 1;
      pins[off[e] + n++] = v;
    }
    for (int32_t i = 0; i < n; ++i) used[pins[off[e] + i]] = 0;
    off[e + 1] = off[e] + n;
  }
  free(used);
  *off_o = off;
  *pins_o = pins;
}

static int oracle_cases(void) {
  for (int it = 0; it < 300; ++it) {
    int32_t V = 2 + rnd(60), E = rnd(90), smax = 2 + rnd(7);
    int32_t *off, *pins;
    random_hypergraph(V, E, smax, &off, &pins);
    int32_t *w = malloc(sizeof(int32_t) * (E + 1));
    for (int32_t e = 0; e < E; ++e) w[e] = 1 + rnd(5);
    int32_t nS = 1 + rnd(V / 2 > 1 ? V / 2 : 1), nT = 1 + rnd((V - nS) > 1 ? V - nS : 1);
    if (nS + nT > V) nT = V - nS;
    if (nT < 1) { nS = 1; nT = 1; }
    int32_t *perm = malloc(sizeof(int32_t) * V);
    for (int32_t v = 0; v < V; ++v) perm[v] = v;
    for (int32_t v = V - 1; v > 0; --v) {
      int32_t j = rnd(v + 1), t = perm[v];
      perm[v] = perm[j];
      perm[j] = t;
    }
    int64_t F = 0, stats[8];
    uint8_t *vs = malloc(V), *ns = malloc(E + 1), *ts = malloc(V);
    int rc = oracle_maxflow_sides(V, E, off, pins, w, perm, nS, perm + nS, nT, it & 1, &F, vs,
                                  ns, ts, stats);
    if (rc != 0) {
      fprintf(stderr, "oracle case %d: rc %d\n", it, rc);
      return 1;
    }
    free(off); free(pins); free(w); free(perm); free(vs); free(ns); free(ts);
  }
  return 0;
}

static int region_cases(void) {
  const int32_t V = 6000, E = 9000, k = 8;
  int32_t *off, *pins;
  random_hypergraph(V, E, 12, &off, &pins);
  int32_t *w = malloc(sizeof(int32_t) * E), *cv = malloc(sizeof(int32_t) * V);
  int32_t *b0 = malloc(sizeof(int32_t) * V);
  for (int32_t e = 0; e < E; ++e) w[e] = 1;
  for (int32_t v = 0; v < V; ++v) { cv[v] = 1; b0[v] = v % k; }
  Ctx *c = hfr_new(V, E, off, pins, w, cv, k, b0);
  if (!c) return 1;
  const int64_t lmax = (103 * ((V + k - 1) / k)) / 100;
  (void)hfr_objective(c);
  (void)hfr_lp(c, 3, lmax);
  int32_t *block = malloc(sizeof(int32_t) * V);
  int64_t bw[64];
  hfr_blocks(c, block, bw);
  int32_t pi[64], pj[64];
  int64_t cut[64];
  int32_t n = hfr_pairs(c, 10, 28, pi, pj, cut);
  if (n < 1) return 1;
  if (hfr_regions(c, n, pi, pj, cut, 8, 148, 100, 2) != 0) return 1;
  for (int32_t r = 0; r < n; ++r) {
    int64_t info[14];
    hfr_region_info(c, r, info);
    int32_t nv = (int32_t)info[0], ne = (int32_t)info[1], np = (int32_t)info[2];
    int32_t *roff = malloc(sizeof(int32_t) * (ne + 1)), *rp = malloc(sizeof(int32_t) * (np + 1));
    int32_t *rw = malloc(sizeof(int32_t) * (ne + 1)), *rvw = malloc(sizeof(int32_t) * nv);
    int32_t *gid = malloc(sizeof(int32_t) * (nv > 2 ? nv - 2 : 1));
    hfr_region_take(c, r, roff, rp, rw, rvw, gid);
    free(roff); free(rp); free(rw); free(rvw); free(gid);
  }
  hfr_free(c);
  free(off); free(pins); free(w); free(cv); free(b0); free(block);
  return 0;
}

int main(void) {
  if (oracle_cases()) return 2;
  if (region_cases()) return 3;
  printf("sanitized runs clean\n");
  return 0;
}
