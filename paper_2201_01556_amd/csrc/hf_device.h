// Device-side phases of the hypergraph push-relabel solver (gfx950).
//
// Network (Lawler expansion, paper section "Preliminaries", paragraph "Flows
// on Hypergraphs"), simulated on the hypergraph itself as the paper's
// paragraph "Hypergraph Implementation" describes -- the expanded graph is
// never built.  Node ids:
//   v            in [0, V)      hypernode
//   NB + 2e                     e_in  of net e     (NB = V rounded up to even,
//   NB + 2e + 1                 e_out of net e      so (e_in, e_out) labels form
//                                                   an aligned int2)
// Source and sink sets are contracted: a net with a source pin receives w(e)
// units into e_in at initialisation (its contracted source arc, capped at
// w(e)); sinks keep label 0 and absorb whatever is pushed into them.
// Source vertices keep label N+1 so that nothing is ever pushed into them.
//
// Per pin slot p (net-CSR order) the state is {r_in, f_out}:
//   r_in  = w(e) - flow(u, e_in)      residual of the capped arc u -> e_in
//   f_out = flow(e_out, u)            residual of the reverse arc u -> e_out
// per net: fb = flow(e_in, e_out).  Residual capacities:
//   u     -> e_in   r_in              u     -> e_out  f_out
//   e_in  -> e_out  w - fb            e_in  -> u      w - r_in
//   e_out -> u      infinite          e_out -> e_in   fb
//
// One discharge round (paper section "Synchronous Parallel Push-Relabel") is
// two phases with an ordering point between them:
//   push   every frontier node u first folds the excess it received in the
//          previous round (dx[prev]) into x[u].  If its label k = d(u) < N it
//          pushes along arcs admissible under the round-start labels
//          (residual > 0 and d(v) = k - 1), distributing its excess over them
//          in arc order; received amounts go to dx[cur][v] (the "excess
//          differences aggregated in a second array" of the paper), so no
//          node ever reads an excess that is still changing and rounds are
//          deterministic.  A node left with excess records
//          cand = 1 + min label over the arcs that stay residual after its own
//          pushes.  Admissibility is antisymmetric in the labels, so each arc
//          pair has a single writer per round and no winning criterion is
//          needed.
//   apply  a node left with excess is relabelled to
//          min(cand, d(u) + 2 if something was pushed into u this round, N).
//          Pushes into u come from nodes labelled d(u) + 1 and are the only
//          residual arcs u could not see; the bound keeps every label valid
//          (d(a) <= d(b) + 1 on every residual arc), which rules out the
//          push-relabel conflict described in section "A Bug in the
//          Synchronous Algorithm".
// Frontier of the next round = nodes pushed into (deduplicated by a
// per-round stamp) plus nodes relabelled below N (paragraph "Active Nodes").
// Appends are staged per wave in LDS and flushed with one global atomic per
// batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

constexpr int kWave = 64;
constexpr int kInf = 0x7fffffff;
// Nodes with more arcs than this are scanned by a whole workgroup in the
// reverse BFS (a wave alone would take thousands of steps).
constexpr int kHugeDeg = 2048;

// error bits reported through Ctl::err
enum : int32_t {
  ERR_LABEL = 1,         // a relabel did not raise the label
  ERR_SINK_REACHED = 2,  // forward cut BFS reached a sink
  ERR_INVARIANT = 4,     // debug invariant check failed
  ERR_SOURCE_REACHED = 8,  // sink-side BFS reached a source
  ERR_PIERCE_TERMINAL = 1024,  // a piercing vertex is a terminal of the other side
  ERR_GUARD = 2048,  // a solve inside one workgroup passed its round or level bound
  ERR_BUILD_PIN = 16,
  ERR_BUILD_OFFSETS = 32,
  ERR_BUILD_WEIGHT = 64,
  ERR_BUILD_DUP = 128,
  ERR_BUILD_TERMINAL = 256,
  ERR_BUILD_ST = 512,
};

// kernel classes for the device byte / item counters
enum : int {
  KC_PUSH = 0,
  KC_APPLY = 1,
  KC_BFS_REV = 2,
  KC_BFS_FWD = 3,
  KC_LOOP_ROUNDS = 4,
  KC_LOOP_BFS = 5,
  KC_BATCH = 6,
  KC_N = 8
};

// A frontier is four lists: small vertices, small e_in, small e_out (nodes
// with at most big_deg arcs, processed by groups of G lanes) and big nodes of
// any kind (processed by whole waves).  Splitting by kind keeps every wave
// item on one code path.
constexpr int kNL = 4;
constexpr int kLvlHist = 64;  // reverse-BFS levels whose sizes are kept
constexpr int kBigList = 3;

struct Ctl {
  int32_t fcnt[3][kNL];  // round frontier counts, ring by epoch % 3
  int32_t bcnt[3][kNL];  // BFS level counts, ring by level % 3
  int32_t err;
  int32_t loop_rounds;  // rounds run by the last single-workgroup round loop
  int32_t loop_levels;  // levels run by the last single-workgroup BFS loop
  int32_t loop_exit;
  unsigned long long flow;      // flow value (into sinks)
  unsigned long long relabels;  // relabel operations
  unsigned long long bytes[KC_N];
  unsigned long long items[KC_N];
  unsigned long long side_weight[2];  // FlowCutter: c(S_r), c(T_r)
  int32_t pierce[5];  // FlowCutter: per side s, [3s] smallest free boundary pin and
                      // [3s + 1] smallest augmenting pin; [2] smallest free vertex
  int32_t big_last;   // last reverse-BFS level of the current global relabel
                      // whose frontier exceeded the single-workgroup tail
  int32_t lvl_nf[kLvlHist];  // size of each of the first reverse-BFS levels of
                             // the current global relabel
};

struct Dev {
  int32_t V, E, P, NB, N, nT, big_deg, bfs_arc;  // bfs_arc: arc-parallel BFS levels
  int32_t bfs_flat;        // reverse-BFS levels spread each wave's 64 nodes' arcs over its lanes
  int32_t relabel_block;   // a node pushed to in a round does not relabel in it
  const int32_t* net_off;  // E+1
  const int32_t* pin_v;    // P
  const int32_t* pin_net;  // P   net of each pin slot
  const int32_t* w;        // E
  const int32_t* vtx_off;  // V+1
  const int2* vinc;        // P   {net, pin slot}, per vertex sorted by slot
  int32_t* role;           // V   0 free, 1 source, 2 sink
  int32_t* nflag;          // E   bit0 has a source pin, bit1 has a sink pin
  int32_t* fpin;           // 2P  {r_in, f_out}
  int32_t* fb;             // E
  int32_t* d;              // N   labels
  int32_t* x;              // N   excess (written by the node itself)
  int32_t* dx[2];          // N   excess received in a round, by round parity
  int32_t* cand;           // N   relabel candidate of a node left with excess, -1 = none
  int32_t* stamp;          // N
  const uint32_t* bigbits; // ceil(N/32) words: bit v set when node v has more than big_deg arcs
  const uint32_t* hugebits;  // ceil(N/32) words: bit v set when node v has more than kHugeDeg arcs
  uint32_t* seen;          // ceil(N/32) words: reverse BFS hint "node has a label" (see label_rev)
  uint8_t* lev;            // N bytes or null: reverse BFS marks, 0 unlabelled, 1 reached by
                           // the level being expanded, 2 labelled (see label_rev)
  int32_t* xbuf;           // null, or the per-workgroup, per-slice arc heads of an expanded
                           // reverse-BFS level (kMaxSliceGroups x 8 x xseg; see xpush)
  int32_t* xcnt;           // kMaxSliceGroups x 8 counts of xbuf
  int32_t xseg;            // entries per workgroup and slice
  uint32_t* pinres;        // ceil(P/32) words: bit of pin slot p = flow(u, e_in) > 0
  uint32_t* netres;        // ceil(E/8) words, 4 bits per net: bit0 = e_in -> e_out
                           // residual (fb < w), bit1 = pins carry flow out of
                           // e_out, bit2 = e_out -> e_in residual (fb > 0)
  int32_t* list[2][kNL];   // [parity][list]: capacities V, E, E, N
  Ctl* ctl;
};

// ---------------------------------------------------------------------------
// wave / group utilities
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ unsigned long long lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

// Workgroup sums of up to three per-thread counters, added to the global
// counters by thread 0: one atomic per workgroup and counter.  Same-address
// atomics issued by every wave of a full grid serialise in the memory system
// and cost more than the work they count.  Block-uniform (every thread of the
// workgroup calls it); blockDim a multiple of 64, at most 1024.
__device__ void block_add_u64(unsigned long long* d0, unsigned long long v0,
                              unsigned long long* d1 = nullptr, unsigned long long v1 = 0ull,
                              unsigned long long* d2 = nullptr, unsigned long long v2 = 0ull) {
  __shared__ unsigned long long part[3][16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v0 += __shfl_xor(v0, o);
    v1 += __shfl_xor(v1, o);
    v2 += __shfl_xor(v2, o);
  }
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 0) {
    part[0][wid] = v0;
    part[1][wid] = v1;
    part[2][wid] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int c = threadIdx.x;
    unsigned long long s = 0ull;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[c][w];
    unsigned long long* d = c == 0 ? d0 : (c == 1 ? d1 : d2);
    if (d != nullptr && s != 0ull) atomicAdd(d, s);
  }
  __syncthreads();  // part may be written again by a later call
}

// Workgroup minima of two per-thread values, folded into the global values
// by thread 0 (atomic min).  Block-uniform, as block_add_u64.
__device__ void block_min_i32(int32_t* d0, int v0, int32_t* d1, int v1) {
  __shared__ int part[2][16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v0 = min(v0, __shfl_xor(v0, o));
    v1 = min(v1, __shfl_xor(v1, o));
  }
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 0) {
    part[0][wid] = v0;
    part[1][wid] = v1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int c = threadIdx.x;
    int m = part[c][0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = min(m, part[c][w]);
    if (m != kInf) atomicMin(c == 0 ? d0 : d1, m);
  }
  __syncthreads();
}

template <int G>
__device__ __forceinline__ uint32_t g_scan_sat(uint32_t v, uint32_t cap, int gl) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, G);
    if (gl >= o) v = min(v + t, cap);
  }
  return v;
}

template <int G>
__device__ __forceinline__ int g_min(int v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, G));
  return v;
}

// Loads that bypass the compiler's value caching (counters written by other
// waves between workgroup barriers).
__device__ __forceinline__ int ld_vol(const int32_t* p) {
  return *reinterpret_cast<const volatile int32_t*>(p);
}
__device__ __forceinline__ unsigned long long ld_vol64(const unsigned long long* p) {
  return *reinterpret_cast<const volatile unsigned long long*>(p);
}

__device__ __forceinline__ int count_all(const int32_t* c) {
  int n = 0;
#pragma unroll
  for (int k = 0; k < kNL; ++k) n += c[k];
  return n;
}
__device__ __forceinline__ int count_all_vol(const int32_t* c) {
  int n = 0;
#pragma unroll
  for (int k = 0; k < kNL; ++k) n += ld_vol(c + k);
  return n;
}

__device__ __forceinline__ int deg_of(const Dev& g, int v) {
  if (v < g.V) return g.vtx_off[v + 1] - g.vtx_off[v];
  const int e = (v - g.NB) >> 1;
  return g.net_off[e + 1] - g.net_off[e] + 1;
}

// ---------------------------------------------------------------------------
// block-level LDS staging of list appends
//
// Appends to a global list reserve space with an atomic on one counter, and
// same-address atomics serialise across the whole chip.  A workgroup
// therefore stages its appends in LDS (wave-aggregated LDS atomics) and
// reserves global space once per flush.  Flushes happen at block-uniform
// points: when the staging area may not hold the next tile's appends, and at
// the end of a phase.  A wave whose appends do not fit any more writes the
// excess straight to the global list (one global atomic for that wave).
// ---------------------------------------------------------------------------

// Staged entries per list: 4 per thread of the workgroup.  LDS words of a
// workgroup's staging area plus the arc tile of the arc-parallel BFS levels:
constexpr int kQPerThread = 4;
constexpr int lds_words(int block) {
  return kNL * kQPerThread * block + 2 * kNL + 3 * block + 1 + 32;
}
__device__ __forceinline__ int bq_words() { return kNL * kQPerThread * (int)blockDim.x + 2 * kNL; }

typedef __attribute__((address_space(3))) int32_t lds_int;

struct BlockQ {
  lds_int* buf;         // [kNL][cap]
  lds_int* n;           // [kNL] staged counts (may exceed cap after overflow)
  lds_int* base;        // [kNL] global base of the current flush
  int32_t* gcnt;        // global counts [kNL]
  int32_t* dst[kNL];    // global lists
  int cap;              // staged entries per list
};

__device__ __forceinline__ int lds_add(lds_int* p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Block-uniform: every thread of the workgroup calls it.
__device__ __forceinline__ BlockQ bq_bind(lds_int* lds, int32_t* gcnt, int32_t* const lists[kNL]) {
  BlockQ q;
  q.cap = kQPerThread * (int)blockDim.x;
  q.buf = lds;
  q.n = lds + kNL * q.cap;
  q.base = lds + kNL * q.cap + kNL;
  q.gcnt = gcnt;
#pragma unroll
  for (int k = 0; k < kNL; ++k) q.dst[k] = lists[k];
  __syncthreads();  // earlier users of the area are done with it
  if (threadIdx.x < kNL) q.n[threadIdx.x] = 0;
  __syncthreads();
  return q;
}

// Called by all active lanes of a wave.
__device__ __forceinline__ void bq_push1(const BlockQ& q, int k, int v, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const int cnt = __popcll(m);
  const int leader = __builtin_ctzll(m);
  int pos = 0;
  if (lane_id() == leader) pos = lds_add(q.n + k, cnt);
  pos = __shfl(pos, leader);
  const int rank = __popcll(m & lanemask_lt());
  const int room = max(0, q.cap - pos);
  if (cnt <= room) {
    if (pred) q.buf[k * q.cap + pos + rank] = v;
    return;
  }
  int gb = 0;
  if (lane_id() == leader) gb = atomicAdd(&q.gcnt[k], cnt - room);
  gb = __shfl(gb, leader);
  if (pred) {
    if (rank < room) q.buf[k * q.cap + pos + rank] = v;
    else q.dst[k][gb + rank - room] = v;
  }
}

__device__ __forceinline__ bool is_big(const Dev& g, int v) {
  return (g.bigbits[v >> 5] >> (v & 31)) & 1u;
}
__device__ __forceinline__ bool is_huge(const Dev& g, int v) {
  return (g.hugebits[v >> 5] >> (v & 31)) & 1u;
}

// list of a node: big nodes together, small ones by kind
__device__ __forceinline__ int list_of(const Dev& g, int v) {
  if (is_big(g, v)) return kBigList;
  return v < g.V ? 0 : 1 + ((v - g.NB) & 1);
}

// Stage v (if pred) into its list.  Called by all active lanes.
__device__ __forceinline__ void qpush(const Dev& g, const BlockQ& q, int v, bool pred) {
  const int k = pred ? list_of(g, v) : -1;
#pragma unroll
  for (int j = 0; j < kNL; ++j) bq_push1(q, j, v, k == j);
}

// Block-uniform: move the staged entries to the global lists.
__device__ __forceinline__ void bq_flush(const BlockQ& q) {
  __syncthreads();
  if (threadIdx.x < kNL) {
    const int k = threadIdx.x;
    const int c = min((int)q.n[k], q.cap);
    q.base[k] = c ? atomicAdd(&q.gcnt[k], c) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kNL; ++k) {
    const int c = min((int)q.n[k], q.cap);
    const int b = q.base[k];
    for (int i = threadIdx.x; i < c; i += blockDim.x) q.dst[k][b + i] = q.buf[k * q.cap + i];
  }
  __syncthreads();
  if (threadIdx.x < kNL) q.n[threadIdx.x] = 0;
  __syncthreads();
}

// Block-uniform: flush unless `reserve` more entries per list still fit.
__device__ __forceinline__ void bq_tile_end(const BlockQ& q, int reserve) {
  __syncthreads();
  int mx = 0;
#pragma unroll
  for (int k = 0; k < kNL; ++k) mx = max(mx, (int)q.n[k]);
  __syncthreads();  // every thread has read the counts before anyone appends
  if (mx > q.cap - reserve) bq_flush(q);
}

// Four values selected by a runtime index without a local array (which would
// live in scratch memory).
struct Quad {
  int v0, v1, v2, v3;
  __device__ __forceinline__ int operator[](int k) const {
    return k == 0 ? v0 : (k == 1 ? v1 : (k == 2 ? v2 : v3));
  }
};

__device__ __forceinline__ Quad load_counts(const int32_t* c) {
  return Quad{c[0], c[1], c[2], c[3]};
}

// Exclusive prefix of four counts: start of each list in the concatenation
// and the total.
struct Prefix4 {
  Quad start;
  int total;
  __device__ __forceinline__ explicit Prefix4(const Quad& n) {
    start = Quad{0, n.v0, n.v0 + n.v1, n.v0 + n.v1 + n.v2};
    total = start.v3 + n.v3;
  }
  // list holding concatenated index i
  __device__ __forceinline__ int list_of(int i) const {
    return (i >= start.v1) + (i >= start.v2) + (i >= start.v3);
  }
};

// Lanes per small node: G for a vertex, half of it (at least 4) for a net
// node, which has half as many arcs on average (nets of 3.7 pins against
// vertices in 7.4 nets on the Zipf workloads); 16 and 8 measured best.
template <int G>
__host__ __device__ constexpr int lanes_of(int k) {
  return k == 0 ? G : (G >= 8 ? G / 2 : G);
}

// Item layout of a frontier or BFS level: for each small list k, groups of
// lanes_of<G>(k) lanes take one node each; then one big node per wave item.
template <int G>
struct Items {
  Quad n;
  Quad start;  // first item of each list
  int end;
  __device__ __forceinline__ explicit Items(const int32_t* cnt) {
    constexpr int NV = kWave / lanes_of<G>(0), NN = kWave / lanes_of<G>(1);
    n = load_counts(cnt);
    const int i0 = (n.v0 + NV - 1) / NV, i1 = (n.v1 + NN - 1) / NN,
              i2 = (n.v2 + NN - 1) / NN;
    start = Quad{0, i0, i0 + i1, i0 + i1 + i2};
    end = start.v3 + n.v3;
  }
  __device__ __forceinline__ int total() const { return end; }
  __device__ __forceinline__ int list_of_item(int it) const {
    return (it >= start.v1) + (it >= start.v2) + (it >= start.v3);
  }
};

// Node i of a frontier given as kNL lists with prefix p.
__device__ __forceinline__ int frontier_node(const Dev& g, int par, const Prefix4& p, int i) {
  const int k = p.list_of(i);
  return g.list[par][k][i - p.start[k]];
}

// Round-scoped stamp: true for exactly one caller per (v, epoch).
__device__ __forceinline__ bool stamp_first(const Dev& g, int v, int epoch) {
  if (g.stamp[v] == epoch) return false;
  return atomicExch(&g.stamp[v], epoch) != epoch;
}

struct RoundArgs {
  int epoch;  // unique id of this round
  int cur3;   // epoch % 3
  int nxt3;   // (epoch + 1) % 3
  int cur;    // epoch % 2: list parity of this round, dx buffer written
  int nxt;    // (epoch + 1) % 2
};

__device__ __forceinline__ RoundArgs round_args(int epoch) {
  RoundArgs a;
  a.epoch = epoch;
  a.cur3 = epoch % 3;
  a.nxt3 = (epoch + 1) % 3;
  a.cur = epoch & 1;
  a.nxt = a.cur ^ 1;
  return a;
}

__device__ __forceinline__ BlockQ round_queue(const Dev& g, const RoundArgs& ra, lds_int* lds) {
  return bq_bind(lds, g.ctl->fcnt[ra.nxt3], g.list[ra.nxt]);
}

// push received by v: amount into dx[cur][v] and v into the next frontier
__device__ __forceinline__ void deliver(const Dev& g, const RoundArgs& ra, const BlockQ& q, int v,
                                        uint32_t amount) {
  bool fresh = false;
  if (amount) {
    atomicAdd(&g.dx[ra.cur][v], (int)amount);
    fresh = stamp_first(g, v, ra.epoch);
  }
  qpush(g, q, v, fresh);
}

// Excess at the start of the round: x plus what arrived last round.
__device__ __forceinline__ int take_excess(const Dev& g, const RoundArgs& ra, int u, int gl) {
  const int xv = g.x[u];
  const int dv = g.dx[ra.nxt][u];  // previous round's buffer (parity of epoch - 1)
  const int X = xv + dv;
  if (dv != 0 && gl == 0) {
    g.x[u] = X;
    g.dx[ra.nxt][u] = 0;
  }
  return X;
}

// End of a node's push scan.
template <int G>
__device__ __forceinline__ void finish_push(const Dev& g, int u, uint32_t X, uint32_t pushed,
                                            int cand, int gl, bool active) {
  if (active && gl == 0 && pushed > 0u) g.x[u] = (int)(X - pushed);
  const bool left = active && pushed < X;
  if (left) {
    cand = g_min<G>(cand);
    if (gl == 0) g.cand[u] = cand;
  }
}

// ---------------------------------------------------------------------------
// push phase, per node kind (G lanes per node, group-uniform control flow)
// nbytes accumulates algorithmic bytes: a node's own fields once per node
// (lane 0 of its group), each arc's fields by the lane that scans the arc.
// ---------------------------------------------------------------------------

template <int G>
__device__ void push_vertex(const Dev& g, const RoundArgs& ra, const BlockQ& q, int u, bool has,
                            int gl, uint32_t& nbytes) {
  int k = 0, X = 0, beg = 0, end = 0;
  if (has) {
    k = g.d[u];
    X = take_excess(g, ra, u, gl);
    beg = g.vtx_off[u];
    end = g.vtx_off[u + 1];
    if (gl == 0) nbytes += 20;
  }
  const bool active = has && k < g.N && X > 0;
  const uint32_t UX = active ? (uint32_t)X : 0u;
  uint32_t carry = 0;
  int cand = kInf;
  if (active) {
    for (int base = beg; base < end; base += G) {
      const int i = base + gl;
      const bool valid = i < end;
      int e = 0, p = 0;
      int2 dl = make_int2(0, 0), fp = make_int2(0, 0);
      if (valid) {
        const int2 ep = g.vinc[i];
        e = ep.x;
        p = ep.y;
        dl = *reinterpret_cast<const int2*>(g.d + g.NB + 2 * e);
        fp = *reinterpret_cast<const int2*>(g.fpin + 2 * p);
        nbytes += 24;
      }
      const uint32_t r1 = (uint32_t)fp.x, r2 = (uint32_t)fp.y;
      const bool a1 = valid && r1 > 0u && dl.x == k - 1;
      const bool a2 = valid && r2 > 0u && dl.y == k - 1;
      const uint32_t want = min((a1 ? r1 : 0u) + (a2 ? r2 : 0u), UX);
      const uint32_t incl = g_scan_sat<G>(want, UX, gl);
      uint32_t excl = __shfl_up(incl, 1, G);
      if (gl == 0) excl = 0u;
      const uint32_t used = min(carry + excl, UX);
      const uint32_t give = min(want, UX - used);
      const uint32_t g1 = a1 ? min(give, r1) : 0u;
      const uint32_t g2 = give - g1;
      if (g1) g.fpin[2 * p] = (int)(r1 - g1);
      if (g2) g.fpin[2 * p + 1] = (int)(r2 - g2);
      deliver(g, ra, q, g.NB + 2 * e, g1);
      deliver(g, ra, q, g.NB + 2 * e + 1, g2);
      if (valid) {
        if (r1 > g1) cand = min(cand, dl.x + 1);
        if (r2 > g2) cand = min(cand, dl.y + 1);
      }
      carry = min(carry + __shfl(incl, G - 1, G), UX);
      if (carry >= UX) break;
    }
  }
  finish_push<G>(g, u, UX, carry, cand, gl, active);
}

template <int G>
__device__ void push_ein(const Dev& g, const RoundArgs& ra, const BlockQ& q, int node, bool has,
                         int gl, uint32_t& nbytes, unsigned long long& to_sink) {
  const int e = (node - g.NB) >> 1;
  int k = 0, X = 0;
  if (has) {
    k = g.d[node];
    X = take_excess(g, ra, node, gl);
    if (gl == 0) nbytes += 12;
  }
  const bool active = has && k < g.N && X > 0;
  const uint32_t UX = active ? (uint32_t)X : 0u;
  uint32_t carry = 0;
  int cand = kInf;
  if (active) {
    const int we = g.w[e];
    const int fbv = g.fb[e];
    const int dout = g.d[node + 1];
    if (gl == 0) nbytes += 20;
    const uint32_t rb = (uint32_t)(we - fbv);
    const bool ab = rb > 0u && dout == k - 1;
    const uint32_t gb = ab ? min(rb, UX) : 0u;
    if (gb && gl == 0) g.fb[e] = fbv + (int)gb;
    deliver(g, ra, q, node + 1, gl == 0 ? gb : 0u);
    carry = gb;
    if (rb > gb) cand = dout + 1;
    if (carry < UX) {
      const int beg = g.net_off[e], end = g.net_off[e + 1];
      for (int base = beg; base < end; base += G) {
        const int i = base + gl;
        const bool valid = i < end;
        int u = 0, rin = 0, du = 0;
        if (valid) {
          u = g.pin_v[i];
          rin = g.fpin[2 * i];
          du = g.d[u];
          nbytes += 12;
        }
        const uint32_t r = valid ? (uint32_t)(we - rin) : 0u;  // flow(u, e_in)
        const bool a = r > 0u && du == k - 1;
        const uint32_t want = a ? min(r, UX) : 0u;
        const uint32_t incl = g_scan_sat<G>(want, UX, gl);
        uint32_t excl = __shfl_up(incl, 1, G);
        if (gl == 0) excl = 0u;
        const uint32_t used = min(carry + excl, UX);
        const uint32_t give = min(want, UX - used);
        if (give) g.fpin[2 * i] = rin + (int)give;
        // a pin labelled 0 is a sink: a vertex pierced into the sink side
        // can still carry flow into e_in, and returning it reaches the sink
        if (du == 0) to_sink += give;
        deliver(g, ra, q, u, du != 0 ? give : 0u);
        if (valid && r > give) cand = min(cand, du + 1);
        carry = min(carry + __shfl(incl, G - 1, G), UX);
        if (carry >= UX) break;
      }
    }
  }
  finish_push<G>(g, node, UX, carry, cand, gl, active);
}

template <int G>
__device__ void push_eout(const Dev& g, const RoundArgs& ra, const BlockQ& q, int node, bool has,
                          int gl, uint32_t& nbytes, unsigned long long& to_sink) {
  const int e = (node - g.NB) >> 1;
  int k = 0, X = 0;
  if (has) {
    k = g.d[node];
    X = take_excess(g, ra, node, gl);
    if (gl == 0) nbytes += 12;
  }
  const bool active = has && k < g.N && X > 0;
  const uint32_t UX = active ? (uint32_t)X : 0u;
  uint32_t carry = 0;
  int cand = kInf;
  if (active) {
    const int beg = g.net_off[e], end = g.net_off[e + 1];
    if (gl == 0) nbytes += 8;
    // pins first: the arcs e_out -> u are infinite, so the first admissible
    // pin takes all remaining excess
    for (int base = beg; base < end; base += G) {
      const int i = base + gl;
      const bool valid = i < end;
      int u = 0, du = 0;
      if (valid) {
        u = g.pin_v[i];
        du = g.d[u];
        nbytes += 8;
      }
      const bool a = valid && du == k - 1;
      const uint32_t want = a ? UX : 0u;
      const uint32_t incl = g_scan_sat<G>(want, UX, gl);
      uint32_t excl = __shfl_up(incl, 1, G);
      if (gl == 0) excl = 0u;
      const uint32_t used = min(carry + excl, UX);
      const uint32_t give = min(want, UX - used);
      if (give) {
        g.fpin[2 * i + 1] += (int)give;
        nbytes += 8;
        if (du == 0) to_sink += give;  // only sinks carry label 0
      }
      deliver(g, ra, q, u, du != 0 ? give : 0u);
      if (valid) cand = min(cand, du + 1);
      carry = min(carry + __shfl(incl, G - 1, G), UX);
      if (carry >= UX) break;
    }
    if (carry < UX) {  // reverse bridge e_out -> e_in
      const int rb = g.fb[e];
      const int din = g.d[node - 1];
      if (gl == 0) nbytes += 8;
      const bool ab = rb > 0 && din == k - 1;
      const uint32_t gb = ab ? min((uint32_t)rb, UX - carry) : 0u;
      if (gb && gl == 0) g.fb[e] = rb - (int)gb;
      deliver(g, ra, q, node - 1, gl == 0 ? gb : 0u);
      carry += gb;
      if ((uint32_t)rb > gb) cand = min(cand, din + 1);
    }
  }
  finish_push<G>(g, node, UX, carry, cand, gl, active);
}

template <int G>
__device__ __forceinline__ void push_node(const Dev& g, const RoundArgs& ra, const BlockQ& q, int v,
                                          bool has, int gl, uint32_t& nbytes,
                                          unsigned long long& to_sink) {
  // kind is wave-divergent only across groups; each branch is group-uniform
  if (!has || v < g.V) push_vertex<G>(g, ra, q, v, has, gl, nbytes);
  else if (((v - g.NB) & 1) == 0) push_ein<G>(g, ra, q, v, has, gl, nbytes, to_sink);
  else push_eout<G>(g, ra, q, v, has, gl, nbytes, to_sink);
}

// Work items of a frontier: small nodes in groups of G lanes (64/G nodes per
// wave item), then big nodes one per wave item.  A workgroup takes tiles of
// one item per wave (block-uniform loop, so the staging area can be flushed
// between tiles).
template <int G>
__device__ void phase_push(const Dev& g, int epoch, int tile0, int tstride, int kc, lds_int* lds) {
  const RoundArgs ra = round_args(epoch);
  if (tile0 == 0 && threadIdx.x < kNL) {
    // ring slot that nobody reads this round: the next round's append target
    g.ctl->fcnt[(epoch + 2) % 3][threadIdx.x] = 0;
  }
  const BlockQ q = round_queue(g, ra, lds);
  const Items<G> its(g.ctl->fcnt[ra.cur3]);
  constexpr int GN = lanes_of<G>(1);
  const int total = its.total();
  const int wpb = blockDim.x >> 6, wid = threadIdx.x >> 6;
  const int ntiles = (total + wpb - 1) / wpb;
  const int lane = lane_id();
  uint32_t nbytes = 0;
  uint32_t nitems = 0;
  unsigned long long to_sink = 0;
  for (int tile = tile0; tile < ntiles; tile += tstride) {
    const int it = tile * wpb + wid;
    if (it < total) {
      const int k = its.list_of_item(it);
      if (k < kBigList) {
        const int gk = k == 0 ? G : GN;
        const int idx = (it - its.start[k]) * (kWave / gk) + lane / gk;
        const bool has = idx < its.n[k];
        const int v = has ? g.list[ra.cur][k][idx] : 0;
        nitems += has && (lane % gk) == 0;
        if (k == 0) push_vertex<G>(g, ra, q, v, has, lane % G, nbytes);
        else if (k == 1) push_ein<GN>(g, ra, q, v, has, lane % GN, nbytes, to_sink);
        else push_eout<GN>(g, ra, q, v, has, lane % GN, nbytes, to_sink);
      } else {
        const int v = g.list[ra.cur][kBigList][it - its.start[kBigList]];
        nitems += lane == 0;
        push_node<kWave>(g, ra, q, v, true, lane, nbytes, to_sink);
      }
    }
    bq_tile_end(q, q.cap / 2);
  }
  bq_flush(q);
  block_add_u64(&g.ctl->flow, to_sink, &g.ctl->bytes[kc],
                (unsigned long long)nbytes + 4ull * nitems, &g.ctl->items[kc], nitems);
}

// Apply phase over the same frontier: relabel nodes left with excess; thread
// per node, small list then big list, tiles of one node per thread.
__device__ void phase_apply(const Dev& g, int epoch, int tile0, int tstride, int kc, lds_int* lds) {
  const RoundArgs ra = round_args(epoch);
  const BlockQ q = round_queue(g, ra, lds);
  const Prefix4 pre(load_counts(g.ctl->fcnt[ra.cur3]));
  const int n = pre.total;
  const int ntiles = (n + blockDim.x - 1) / blockDim.x;
  unsigned long long nrel = 0;
  uint32_t nbytes = 0;
  for (int tile = tile0; tile < ntiles; tile += tstride) {
    const int i = tile * blockDim.x + threadIdx.x;
    bool app = false;
    int v = 0;
    if (i < n) {
      v = frontier_node(g, ra.cur, pre, i);
      const int c = g.cand[v];
      nbytes += 8;
      const bool rec = c >= 0 && g.stamp[v] == ra.epoch;
      if (c >= 0 && rec && g.relabel_block) {
        // blocking variant (section "A Bug in the Synchronous Algorithm",
        // the first fix): a node pushed to in this round keeps its label;
        // the push listed it for the next round, where it tries again
        g.cand[v] = -1;
      } else if (c >= 0) {
        g.cand[v] = -1;
        const int k = g.d[v];
        int nd = c;
        if (rec) nd = min(nd, k + 2);
        nd = min(nd, g.N);
        if (nd <= k) atomicOr(&g.ctl->err, ERR_LABEL);
        g.d[v] = nd;
        nrel += 1;
        nbytes += 12;
        app = !rec && nd < g.N;
      }
    }
    qpush(g, q, v, app);
    bq_tile_end(q, (int)blockDim.x);
  }
  bq_flush(q);
  block_add_u64(&g.ctl->relabels, nrel, &g.ctl->bytes[kc], nbytes, &g.ctl->items[kc], nrel);
}

// ---------------------------------------------------------------------------
// reverse residual BFS from the sinks (global relabel) over the capped network
// ---------------------------------------------------------------------------

// Global relabel, step 2: residual bits that the reverse BFS tests, so that
// its checks of an arc hit two small bitmaps instead of scattered flows.
// The flow state does not change during a global relabel.
//   pinres: one bit per pin slot p of net e: flow(u, e_in) = w(e) - r_in > 0
//           (the reverse arc e_in -> u is residual)
//   netres: four bits per net: bit0 fb < w (e_in -> e_out residual), bit1
//           some pin carries flow out of e_out (fb exceeds e_out's excess),
//           bit2 fb > 0 (e_out -> e_in residual)
// Thread per slot, then per net; t0 wave-aligned, tstride a multiple of 64.
__device__ void phase_gr_bits(const Dev& g, int t0, int tstride) {
  const int lane = lane_id();
  // pin slots: a lane per slot, a wave per 64 slots (two words of the bitmap)
  const int np = (g.P + 63) & ~63;
  const int pwords = (g.P + 31) >> 5;
  for (int p = t0; p < np; p += tstride) {
    const bool f = p < g.P && g.fpin[2 * p] < g.w[g.pin_net[p]];
    const unsigned long long m = __ballot(f);
    const int word = ((p - lane) >> 5) + lane;
    if (lane < 2 && word < pwords) g.pinres[word] = (uint32_t)(m >> (32 * lane));
  }
  // nets: a lane per net, eight nibbles per word
  const int ne = (g.E + 63) & ~63;
  for (int e = t0; e < ne; e += tstride) {
    uint32_t b = 0;
    if (e < g.E) {
      const int fbv = g.fb[e], eo = g.NB + 2 * e + 1;
      const int out = fbv - (g.x[eo] + g.dx[0][eo] + g.dx[1][eo]);
      b = (fbv < g.w[e] ? 1u : 0u) | (out > 0 ? 2u : 0u) | (fbv > 0 ? 4u : 0u);
    }
    uint32_t v = b << (4 * (lane & 7));
    v |= __shfl_xor(v, 1);
    v |= __shfl_xor(v, 2);
    v |= __shfl_xor(v, 4);
    if ((lane & 7) == 0 && e < g.E) g.netres[e >> 3] = v;
  }
}

__device__ __forceinline__ bool pin_flow_in(const Dev& g, int p) {
  return (g.pinres[p >> 5] >> (p & 31)) & 1u;
}
__device__ __forceinline__ uint32_t net_bits(const Dev& g, int e) {
  return (g.netres[e >> 3] >> (4 * (e & 7))) & 15u;
}

// The "labelled" hint of the reverse BFS is a bitmap small enough to stay in
// the L2, so checking an arc whose tail is already labelled costs no access
// to the large label array.  Bits are set with a plain read-modify-write; a
// bit lost to a concurrent update only sends a later check to the label
// itself, which stays the source of truth.
__device__ __forceinline__ bool seen_bit(const Dev& g, int v) {
  return (g.seen[v >> 5] >> (v & 31)) & 1u;
}
__device__ __forceinline__ void set_seen(const Dev& g, int v) {
  g.seen[v >> 5] |= 1u << (v & 31);
}

// Label v with lvl if it is unlabelled.  With kClaim the first writer wins
// by compare-and-swap on the label and reports it; otherwise a plain store
// (all writers of a level store the same value).  With the byte marks `lev`
// an expanded level only marks v (byte 1, a 5 MB array for 5 M nodes
// instead of the 20 MB label array) and the collect sweep writes the label
// and lists v; a claimed node gets byte 2 at once.
// kChecked: the caller has just read v's hint bit and found it clear.
template <bool kClaim, bool kChecked = false>
__device__ __forceinline__ bool label_rev(const Dev& g, int v, int lvl) {
  if (!kChecked && seen_bit(g, v)) return false;
  if (!kClaim) {
    if (g.lev) {
      if (g.lev[v] != 0) return false;
      g.lev[v] = 1;
    } else {
      if (g.d[v] != g.N) return false;
      g.d[v] = lvl;
    }
    set_seen(g, v);
    return false;
  }
  if (atomicCAS(&g.d[v], g.N, lvl) != g.N) return false;
  if (g.lev) g.lev[v] = 2;
  set_seen(g, v);
  return true;
}

// Slices of the node range for the XCD-local expansion of reverse-BFS
// levels: 1024-node chunks dealt round-robin to the eight XCDs (workgroup b
// of a grid runs on XCD b mod 8), so each XCD's share of the label array
// (a quarter of its 4 MB L2 for 5 M nodes) and of the labelled bitmap stays
// in its own L2.
constexpr int kSlices = 8;
constexpr int kMaxSliceGroups = 512;
__device__ __forceinline__ int xslice(int v) { return (v >> 10) & (kSlices - 1); }

// An arc head of an expanded level: labelled at once (visit_rev = label_rev)
// or, with kSlice, only pre-checked against the labelled bitmap and handed
// to its slice (xpush); the slice kernel then labels it on the XCD that
// owns it.
template <bool kClaim, bool kChecked = false, bool kSlice = false>
__device__ __forceinline__ bool visit_rev(const Dev& g, int v, int lvl) {
  if (kSlice) return kChecked ? true : !seen_bit(g, v);
  return label_rev<kClaim, kChecked>(g, v, lvl);
}

// Append arc head t (where pred) to this workgroup's segment of its slice:
// wave-aggregated LDS counters xc[8]; an entry past the segment's end is
// labelled here instead.  Called by the active lanes of a wave.
__device__ __forceinline__ void xpush(const Dev& g, lds_int* xc, int t, bool pred, int lvl) {
  if (__ballot(pred) == 0ull) return;
  const int me = xslice(t);
  int32_t* seg = g.xbuf + (long long)blockIdx.x * kSlices * g.xseg;
#pragma unroll 1
  for (int sl = 0; sl < kSlices; ++sl) {
    const bool mine = pred && me == sl;
    const unsigned long long m = __ballot(mine);
    if (m == 0ull) continue;
    const int leader = __builtin_ctzll(m);
    int pos = 0;
    if (lane_id() == leader) pos = lds_add(xc + sl, __popcll(m));
    pos = __shfl(pos, leader);
    if (mine) {
      const int idx = pos + __popcll(m & lanemask_lt());
      if (idx < g.xseg) seg[sl * g.xseg + idx] = t;
      else label_rev<false, true>(g, t, lvl);
    }
  }
}

// Node-grouped reverse BFS: a group of `stride` lanes scans node x (G lanes
// per small node, a wave per big node, the workgroup per huge node); gl is
// the lane's index in the group.
template <bool kClaim, bool kSlice = false>
__device__ __forceinline__ void bfs_rev_node(const Dev& g, const BlockQ& q, int x, bool has,
                                             int gl, int stride, int lvl, uint32_t& nbytes,
                                             lds_int* xc = nullptr) {
  const bool isv = has && x < g.V;
  const bool isnet = has && x >= g.NB;
  if (!has || isv) {
    int beg = 0, end = 0;
    if (isv) {
      beg = g.vtx_off[x];
      end = g.vtx_off[x + 1];
    }
    for (int base = beg; base < end; base += stride) {
      const int i = base + gl;
      const bool valid = i < end;
      bool vin = false, vout = false;
      int t1 = 0;
      if (valid) {
        const int2 ep = g.vinc[i];
        t1 = g.NB + 2 * ep.x;
        // bits of e_in and e_out share a word (NB and 2e are even)
        const uint32_t sw = g.seen[t1 >> 5] >> (t1 & 31);
        nbytes += 12;
        if (!(sw & 2u)) vout = visit_rev<kClaim, true, kSlice>(g, t1 + 1, lvl);  // e_out -> x infinite
        if (!(sw & 1u) && pin_flow_in(g, ep.y))                    // e_in -> x reverse
          vin = visit_rev<kClaim, true, kSlice>(g, t1, lvl);
      }
      if (kClaim) {
        qpush(g, q, t1, vin);
        qpush(g, q, t1 + 1, vout);
      }
      if (kSlice) {
        xpush(g, xc, t1, vin, lvl);
        xpush(g, xc, t1 + 1, vout, lvl);
      }
    }
  } else if (isnet) {
    const int e = (x - g.NB) >> 1;
    const bool in = ((x - g.NB) & 1) == 0;
    const uint32_t nb = net_bits(g, e);
    int beg = g.net_off[e], end = g.net_off[e + 1];
    // in-arcs of e_out from pins carry flow(e_out, u) > 0; their sum is the
    // outflow fb - excess(e_out), so a net without outflow skips its pins
    if (!in && !(nb & 2u)) end = beg;
    if (gl == 0) nbytes += 16;
    bool vb = false;
    if (gl == 0) {
      if (in) vb = (nb & 4u) && visit_rev<kClaim, false, kSlice>(g, x + 1, lvl);  // e_out -> e_in residual fb
      else vb = (nb & 1u) && visit_rev<kClaim, false, kSlice>(g, x - 1, lvl);     // e_in -> e_out residual w - fb
    }
    if (kClaim) qpush(g, q, in ? x + 1 : x - 1, vb);
    if (kSlice) xpush(g, xc, in ? x + 1 : x - 1, vb, lvl);
    for (int base = beg; base < end; base += stride) {
      const int i = base + gl;
      const bool valid = i < end;
      bool vu = false;
      int u = 0;
      if (valid) {
        u = g.pin_v[i];
        const int f = g.fpin[2 * i + (in ? 0 : 1)];  // r_in (u->e_in) or f_out (u->e_out)
        nbytes += 12;
        if (f > 0) vu = visit_rev<kClaim, false, kSlice>(g, u, lvl);
      }
      if (kClaim) qpush(g, q, u, vu);
      if (kSlice) xpush(g, xc, u, vu, lvl);
    }
  }
}

// Visit v in the forward BFS stamped ep.  With kClaim the first visitor wins
// (exchange on the stamp) and lists v; otherwise an unvisited v gets the
// level's provisional stamp ep_tmp by a plain store (every writer stores the
// same value) and the collect sweep lists it and stamps it ep.
template <bool kClaim>
__device__ __forceinline__ bool fwd_visit(const Dev& g, int v, int ep, int ep_tmp) {
  if (kClaim) return stamp_first(g, v, ep);
  const int sv = g.stamp[v];
  if (sv != ep && sv != ep_tmp) g.stamp[v] = ep_tmp;
  return false;
}

// Node-grouped forward BFS of the uncapped residual network (source side): a
// group of `stride` lanes scans node x's residual out-arcs.
//   vertex u:  u -> e_in always (uncapped), u -> e_out when flow(e_out, u) > 0
//   e_in:      e_in -> e_out when fb < w, e_in -> u when flow(u, e_in) > 0
//   e_out:     e_out -> e_in when fb > 0, e_out -> u always (a sink reached
//              is an internal error: the flow would not be maximum)
template <bool kClaim>
__device__ __forceinline__ void bfs_fwd_node(const Dev& g, const BlockQ& q, int x, bool has,
                                             int gl, int stride, int ep, int ep_tmp,
                                             uint32_t& nbytes) {
  const bool isv = has && x < g.V;
  const bool isnet = has && x >= g.NB;
  if (!has || isv) {
    int beg = 0, end = 0;
    if (isv) {
      beg = g.vtx_off[x];
      end = g.vtx_off[x + 1];
    }
    for (int base = beg; base < end; base += stride) {
      const int i = base + gl;
      bool vin = false, vout = false;
      int t1 = 0;
      if (i < end) {
        const int2 ep2 = g.vinc[i];
        t1 = g.NB + 2 * ep2.x;
        nbytes += 12;
        vin = fwd_visit<kClaim>(g, t1, ep, ep_tmp);
        if (g.fpin[2 * ep2.y + 1] > 0) vout = fwd_visit<kClaim>(g, t1 + 1, ep, ep_tmp);
      }
      if (kClaim) {
        qpush(g, q, t1, vin);
        qpush(g, q, t1 + 1, vout);
      }
    }
  } else if (isnet) {
    const int e = (x - g.NB) >> 1;
    const bool in = ((x - g.NB) & 1) == 0;
    const int beg = g.net_off[e], end = g.net_off[e + 1];
    const int we = g.w[e];
    bool vb = false;
    if (gl == 0) {
      const int fbv = g.fb[e];
      nbytes += 16;
      if (in ? fbv < we : fbv > 0) vb = fwd_visit<kClaim>(g, in ? x + 1 : x - 1, ep, ep_tmp);
    }
    if (kClaim) qpush(g, q, in ? x + 1 : x - 1, vb);
    for (int base = beg; base < end; base += stride) {
      const int i = base + gl;
      bool vu = false;
      int u = 0;
      if (i < end) {
        u = g.pin_v[i];
        nbytes += 8;
        if (in) {
          if (we - g.fpin[2 * i] > 0) vu = fwd_visit<kClaim>(g, u, ep, ep_tmp);
        } else {
          const int r = g.role[u];
          if (r == 2) atomicOr(&g.ctl->err, ERR_SINK_REACHED);
          else if (r == 0) vu = fwd_visit<kClaim>(g, u, ep, ep_tmp);
        }
      }
      if (kClaim) qpush(g, q, u, vu);
    }
  }
}

// Node-grouped reverse BFS of the uncapped residual network (maximal sink
// side), claiming by exchange on the stamp ep: node x's residual in-arcs.
//   vertex x:  from e_out always, from e_in when flow(x, e_in) > 0
//   e_in:      from e_out when fb > 0, from every pin (uncapped)
//   e_out:     from e_in when fb < w, from pins u with flow(e_out, u) > 0
// A source reached is an internal error (the flow would not be maximum).
__device__ __forceinline__ void bfs_sink_node(const Dev& g, const BlockQ& q, int x, bool has,
                                              int gl, int stride, int ep, uint32_t& nbytes) {
  const bool isv = has && x < g.V;
  const bool isnet = has && x >= g.NB;
  if (!has || isv) {
    int beg = 0, end = 0;
    if (isv) {
      beg = g.vtx_off[x];
      end = g.vtx_off[x + 1];
    }
    for (int base = beg; base < end; base += stride) {
      const int i = base + gl;
      bool vin = false, vout = false;
      int t1 = 0;
      if (i < end) {
        const int2 ep2 = g.vinc[i];
        t1 = g.NB + 2 * ep2.x;
        nbytes += 12;
        vout = stamp_first(g, t1 + 1, ep);                                       // e_out -> x
        if (g.w[ep2.x] - g.fpin[2 * ep2.y] > 0) vin = stamp_first(g, t1, ep);  // e_in -> x
      }
      qpush(g, q, t1, vin);
      qpush(g, q, t1 + 1, vout);
    }
  } else if (isnet) {
    const int e = (x - g.NB) >> 1;
    const bool in = ((x - g.NB) & 1) == 0;
    const int beg = g.net_off[e], end = g.net_off[e + 1];
    bool vb = false;
    if (gl == 0) {
      const int fbv = g.fb[e];
      nbytes += 16;
      if (in ? fbv > 0 : fbv < g.w[e]) vb = stamp_first(g, in ? x + 1 : x - 1, ep);
    }
    qpush(g, q, in ? x + 1 : x - 1, vb);
    for (int base = beg; base < end; base += stride) {
      const int i = base + gl;
      bool vu = false;
      int u = 0;
      if (i < end) {
        u = g.pin_v[i];
        nbytes += 8;
        if (in || g.fpin[2 * i + 1] > 0) {  // u -> e_in always, u -> e_out by flow
          if (g.role[u] == 1) atomicOr(&g.ctl->err, ERR_SOURCE_REACHED);
          else vu = stamp_first(g, u, ep);
        }
      }
      qpush(g, q, u, vu);
    }
  }
}

constexpr int kDirRelabel = 0;  // reverse BFS of a global relabel (capped network)
constexpr int kDirSource = 1;   // forward BFS of the source side (uncapped)
constexpr int kDirSink = 2;     // reverse BFS of the sink side (uncapped)

// One BFS level, node-grouped: the reverse BFS of a global relabel (labels
// level+1), the forward BFS of the source side (stamp ep, provisional stamp
// ep_tmp when expanding) or the reverse BFS of the sink side (stamp ep,
// claiming only).
template <int G, bool kClaim, int kDir>
__device__ void phase_bfs_node(const Dev& g, int level, int ep, int ep_tmp, int tile0,
                               int tstride, int kc, lds_int* lds) {
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (tile0 == 0 && threadIdx.x < kNL) g.ctl->bcnt[z3][threadIdx.x] = 0;
  const int cp = level & 1, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  const Items<G> its(g.ctl->bcnt[c3]);
  constexpr int GN = lanes_of<G>(1);
  const int total = its.total();
  const int wpb = blockDim.x >> 6, wid = threadIdx.x >> 6;
  const int ntiles = (total + wpb - 1) / wpb;
  const int lane = lane_id();
  uint32_t nbytes = 0, nitems = 0;
  // tiles of wave items, then one tile per big-list node in which only a huge
  // node (more arcs than a wave should scan alone, such as a contracted
  // terminal) is scanned, by the whole workgroup; a wave item skips it
  const int nbig = its.n[kBigList];
  for (int tile = tile0; tile < ntiles + nbig; tile += tstride) {
    int v = 0, gl = 0, stride = G;
    bool has = false;
    if (tile < ntiles) {
      const int it = tile * wpb + wid;
      if (it < total) {
        const int k = its.list_of_item(it);
        if (k < kBigList) {
          stride = k == 0 ? G : GN;
          const int idx = (it - its.start[k]) * (kWave / stride) + lane / stride;
          has = idx < its.n[k];
          v = has ? g.list[cp][k][idx] : 0;
          gl = lane % stride;
        } else {
          v = g.list[cp][kBigList][it - its.start[kBigList]];
          has = !is_huge(g, v);
          gl = lane;
          stride = kWave;
        }
      }
    } else {
      v = g.list[cp][kBigList][tile - ntiles];
      has = is_huge(g, v);  // block-uniform
      gl = threadIdx.x;
      stride = blockDim.x;
    }
    nitems += has && gl == 0;
    if constexpr (kDir == kDirSource)
      bfs_fwd_node<kClaim>(g, q, v, has, gl, stride, ep, ep_tmp, nbytes);
    else if constexpr (kDir == kDirSink)
      bfs_sink_node(g, q, v, has, gl, stride, ep, nbytes);
    else bfs_rev_node<kClaim>(g, q, v, has, gl, stride, level + 1, nbytes);
    if (kClaim) bq_tile_end(q, q.cap / 2);
  }
  if (kClaim) bq_flush(q);
  block_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 4ull * nitems, &g.ctl->items[kc],
                nitems);
}

// frontier of level `level` -> label level+1
template <int G, bool kClaim>
__device__ void phase_bfs_rev_node(const Dev& g, int level, int tile0, int tstride, int kc,
                                   lds_int* lds) {
  phase_bfs_node<G, kClaim, kDirRelabel>(g, level, 0, 0, tile0, tstride, kc, lds);
}

// ---------------------------------------------------------------------------
// flattened reverse-BFS levels
//
// A wave takes 64 consecutive entries of one small-node list, one node per
// lane, and spreads the nodes' arcs over its 64 lanes: a wave prefix sum of
// the arc counts, then in every step each lane finds the node owning its arc
// by a binary search over the lanes' offsets (shuffles, no LDS, no barrier).
// All loads of a step are independent and every lane has an arc until the
// last step, so a level's latency chains overlap far more than with a fixed
// group of lanes per node (a net node holds 3.7 arcs on average, a vertex
// 7.4, and most e_out nodes only their bridge).  Big nodes keep a wave each,
// huge nodes the workgroup, as in the node-grouped levels.
// ---------------------------------------------------------------------------

template <bool kClaim, bool kSlice = false>
__device__ __forceinline__ void phase_bfs_rev_flat(const Dev& g, int level, int tile0, int tstride, int kc,
                                   lds_int* lds) {
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (tile0 == 0 && threadIdx.x < kNL) g.ctl->bcnt[z3][threadIdx.x] = 0;
  const int cp = level & 1, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  lds_int* const xc = lds + bq_words();  // slice counts (in the arc-tile area, unused here)
  if (kSlice) {
    if (threadIdx.x < kSlices) xc[threadIdx.x] = 0;
    __syncthreads();
  }
  const Quad n = load_counts(g.ctl->bcnt[c3]);
  // wave items: 64 entries of list 0, of list 1, of list 2, then one big node each
  const int s1 = (n.v0 + kWave - 1) / kWave;
  const int s2 = s1 + (n.v1 + kWave - 1) / kWave;
  const int s3 = s2 + (n.v2 + kWave - 1) / kWave;
  const int total = s3 + n.v3;
  const int wpb = blockDim.x >> 6, wid = threadIdx.x >> 6, lane = lane_id();
  const int ntiles = (total + wpb - 1) / wpb;
  const int lvl = level + 1;
  uint32_t nbytes = 0, nitems = 0;
  for (int tile = tile0; tile < ntiles + n.v3; tile += tstride) {
    if (tile < ntiles) {
      const int it = tile * wpb + wid;
      if (it < s3) {
        const int k = (it >= s1) + (it >= s2);  // wave-uniform list
        const int idx = (it - (k == 0 ? 0 : (k == 1 ? s1 : s2))) * kWave + lane;
        int x = 0, beg = 0, deg = 0;
        uint32_t nb = 0;
        if (idx < n[k]) {
          x = g.list[cp][k][idx];
          if (k == 0) {
            beg = g.vtx_off[x];
            deg = g.vtx_off[x + 1] - beg;
          } else {
            const int e = (x - g.NB) >> 1;
            nb = net_bits(g, e);
            beg = g.net_off[e];
            int sz = g.net_off[e + 1] - beg;
            // in-arcs of e_out from pins carry flow(e_out, u) > 0; a net
            // without outflow has none
            if (k == 2 && !(nb & 2u)) sz = 0;
            deg = 1 + sz;  // arc 0 is the bridge
            nbytes += 16;
          }
          nitems += 1;
        }
        int incl = deg;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const int t = __shfl_up(incl, o);
          if (lane >= o) incl += t;
        }
        const int excl = incl - deg;
        const int A = __shfl(incl, kWave - 1);
        for (int a0 = 0; a0 < A; a0 += kWave) {
          const int a = a0 + lane;
          // owner: the last lane whose offset is <= a (lanes without arcs
          // share the next lane's offset, so the last one owns the arc)
          int lo = 0;
#pragma unroll
          for (int st = kWave / 2; st > 0; st >>= 1) {
            const int c = lo + st;
            if (__shfl(excl, c) <= a) lo = c;
          }
          const int xo = __shfl(x, lo), bo = __shfl(beg, lo);
          const int j = a - __shfl(excl, lo);
          const uint32_t nbo = __shfl((int)nb, lo);
          int t1 = 0, t2 = 0;
          bool v1 = false, v2 = false;
          if (a < A) {
            if (k == 0) {
              const int2 ep = g.vinc[bo + j];
              t1 = g.NB + 2 * ep.x;
              t2 = t1 + 1;
              // bits of e_in and e_out share a word (NB and 2e are even)
              const uint32_t sw = g.seen[t1 >> 5] >> (t1 & 31);
              nbytes += 12;
              if (!(sw & 2u)) v2 = visit_rev<kClaim, true, kSlice>(g, t2, lvl);  // e_out -> x infinite
              if (!(sw & 1u) && pin_flow_in(g, ep.y))                    // e_in -> x reverse
                v1 = visit_rev<kClaim, true, kSlice>(g, t1, lvl);
            } else if (j == 0) {
              if (k == 1) {
                t1 = xo + 1;  // e_out -> e_in residual fb
                v1 = (nbo & 4u) && visit_rev<kClaim, false, kSlice>(g, t1, lvl);
              } else {
                t1 = xo - 1;  // e_in -> e_out residual w - fb
                v1 = (nbo & 1u) && visit_rev<kClaim, false, kSlice>(g, t1, lvl);
              }
            } else {
              const int i = bo + j - 1;
              t1 = g.pin_v[i];
              // r_in (u -> e_in) or f_out (u -> e_out)
              const int f = g.fpin[2 * i + (k == 1 ? 0 : 1)];
              nbytes += 12;
              if (f > 0) v1 = visit_rev<kClaim, false, kSlice>(g, t1, lvl);
            }
          }
          if (kClaim) {
            qpush(g, q, t1, v1);
            qpush(g, q, t2, v2);
          }
          if (kSlice) {
            xpush(g, xc, t1, v1, lvl);
            xpush(g, xc, t2, v2, lvl);
          }
        }
      } else if (it < total) {
        const int v = g.list[cp][kBigList][it - s3];
        const bool has = !is_huge(g, v);
        nitems += has && lane == 0;
        bfs_rev_node<kClaim, kSlice>(g, q, v, has, lane, kWave, lvl, nbytes, xc);
      }
    } else {
      const int v = g.list[cp][kBigList][tile - ntiles];
      const bool has = is_huge(g, v);  // block-uniform
      nitems += has && threadIdx.x == 0;
      bfs_rev_node<kClaim, kSlice>(g, q, v, has, threadIdx.x, blockDim.x, lvl, nbytes, xc);
    }
    if (kClaim) bq_tile_end(q, q.cap / 2);
  }
  if (kClaim) bq_flush(q);
  if (kSlice) {
    __syncthreads();
    if (threadIdx.x < kSlices)
      g.xcnt[blockIdx.x * kSlices + threadIdx.x] = min((int)xc[threadIdx.x], g.xseg);
  }
  block_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 4ull * nitems, &g.ctl->items[kc],
                nitems);
}

// The labelling half of an XCD-local expanded level: workgroup b serves
// slice b mod 8 (so it runs on the XCD that owns the slice) and labels the
// heads that every workgroup of the scan handed to that slice.
__device__ void phase_bfs_slices(const Dev& g, int level, int nseg) {
  const int sl = blockIdx.x & (kSlices - 1);
  const int w = blockIdx.x / kSlices, nw = gridDim.x / kSlices;
  const int lvl = level + 1;
  for (int b = w; b < nseg; b += nw) {
    const int c = g.xcnt[b * kSlices + sl];
    const int32_t* src = g.xbuf + ((long long)b * kSlices + sl) * g.xseg;
    for (int i = threadIdx.x; i < c; i += blockDim.x) label_rev<false>(g, src[i], lvl);
  }
}

// ---------------------------------------------------------------------------
// arc-parallel BFS levels
//
// A workgroup takes a tile of up to blockDim frontier nodes, computes their
// arc counts and an exclusive prefix sum in LDS, and then every thread takes
// one arc per step (locating its node by binary search in the prefix), so
// all loads of a step are independent and nodes of any degree are spread
// over the whole workgroup.  Arc 0 of a net node is its bridge.
// ---------------------------------------------------------------------------

// tile area after the staging area: node[bd], beg[bd], off[bd + 1], wave
// sums[32] (bd = blockDim, at most 1024)

struct ArcTile {
  lds_int* node;
  lds_int* beg;
  lds_int* off;
  lds_int* wsum;
};

__device__ __forceinline__ ArcTile arc_tile(lds_int* lds) {
  ArcTile t;
  t.node = lds;
  const int bd = blockDim.x;
  t.beg = lds + bd;
  t.off = lds + 2 * bd;
  t.wsum = lds + 3 * bd + 1;
  return t;
}

// Block-uniform exclusive prefix sum of one int per thread; returns the
// thread's offset, *total gets the sum (same in every thread).
__device__ __forceinline__ int block_excl_scan(int v, lds_int* wsum, int* total) {
  const int lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  __syncthreads();  // wsum is free (previous readers are done)
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < nw; ++i) {
      const int t = wsum[i];
      wsum[i] = run;
      run += t;
    }
    wsum[nw] = run;
  }
  __syncthreads();
  *total = wsum[nw];
  return wsum[wid] + incl - v;
}

// Block-uniform: load tile `tile` of the frontier into LDS; returns the arc
// count of the tile and the node count in *nt_out.
__device__ __forceinline__ int load_arc_tile(const Dev& g, const ArcTile& t, int par,
                                             const Prefix4& pre, int tile, int* nt_out) {
  const int nf = pre.total;
  const int first = tile * blockDim.x;
  const int nt = min((int)blockDim.x, nf - first);
  int deg = 0, beg = 0, v = 0;
  if ((int)threadIdx.x < nt) {
    v = frontier_node(g, par, pre, first + threadIdx.x);
    if (v < g.V) {
      beg = g.vtx_off[v];
      deg = g.vtx_off[v + 1] - beg;
    } else {
      const int e = (v - g.NB) >> 1;
      beg = g.net_off[e];
      deg = g.net_off[e + 1] - beg + 1;
    }
  }
  int total = 0;
  const int o = block_excl_scan(deg, t.wsum, &total);
  if ((int)threadIdx.x < nt) {
    t.node[threadIdx.x] = v;
    t.beg[threadIdx.x] = beg;
    t.off[threadIdx.x] = o;
  }
  if (threadIdx.x == 0) t.off[nt] = total;
  __syncthreads();
  *nt_out = nt;
  return total;
}

// index k of the tile node owning arc a: largest k with off[k] <= a
__device__ __forceinline__ int arc_owner(const ArcTile& t, int nt, int a) {
  int lo = 0, hi = nt;  // off[lo] <= a < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (t.off[mid] <= a) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One level of the reverse BFS (labels level+1), arc-parallel.
template <bool kClaim>
__device__ void phase_bfs_rev_lb(const Dev& g, int level, int tile0, int tstride, int kc,
                                 lds_int* lds) {
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (tile0 == 0 && threadIdx.x < kNL) g.ctl->bcnt[z3][threadIdx.x] = 0;
  const int cp = level & 1, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  const ArcTile t = arc_tile(lds + bq_words());
  const Prefix4 pre(load_counts(g.ctl->bcnt[c3]));
  const int ntiles = (pre.total + blockDim.x - 1) / blockDim.x;
  const int lvl = level + 1;
  uint32_t nbytes = 0, narcs = 0;
  for (int tile = tile0; tile < ntiles; tile += tstride) {
    int nt = 0;
    const int A = load_arc_tile(g, t, cp, pre, tile, &nt);
    for (int a0 = 0; a0 < A; a0 += blockDim.x) {
      const int a = a0 + threadIdx.x;
      int t1 = 0, t2 = 0;
      bool v1 = false, v2 = false;
      if (a < A) {
        const int k = arc_owner(t, nt, a);
        const int x = t.node[k];
        const int j = a - t.off[k];
        const int b = t.beg[k];
        ++narcs;
        if (x < g.V) {
          const int2 ep = g.vinc[b + j];
          const int e = ep.x;
          t1 = g.NB + 2 * e;
          t2 = t1 + 1;
          const uint32_t sw = g.seen[t1 >> 5] >> (t1 & 31);
          nbytes += 12;
          if (!(sw & 2u)) v2 = label_rev<kClaim, true>(g, t2, lvl);  // e_out -> x infinite
          if (!(sw & 1u) && g.w[e] - g.fpin[2 * ep.y] > 0)     // e_in -> x reverse
            v1 = label_rev<kClaim, true>(g, t1, lvl);
        } else {
          const int e = (x - g.NB) >> 1;
          const bool in = ((x - g.NB) & 1) == 0;
          if (j == 0) {  // bridge
            const int fbv = g.fb[e];
            nbytes += 8;
            t1 = in ? x + 1 : x - 1;
            if (in ? fbv > 0 : g.w[e] - fbv > 0) v1 = label_rev<kClaim>(g, t1, lvl);
          } else {
            const int i = b + j - 1;
            t1 = g.pin_v[i];
            const int f = g.fpin[2 * i + (in ? 0 : 1)];  // r_in (u->e_in) or f_out (u->e_out)
            nbytes += 9;
            if (f > 0) v1 = label_rev<kClaim>(g, t1, lvl);
          }
        }
      }
      if (kClaim) {
        qpush(g, q, t1, v1);
        qpush(g, q, t2, v2);
        bq_tile_end(q, 2 * blockDim.x);
      }
    }
    __syncthreads();  // the tile area is rewritten by the next tile
  }
  if (kClaim) bq_flush(q);
  block_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 12ull * narcs, &g.ctl->items[kc],
                narcs);
}

// One level of the forward BFS of the uncapped network, arc-parallel.
template <bool kClaim>
__device__ void phase_bfs_fwd_lb(const Dev& g, int level, int ep, int ep_tmp, int tile0,
                                 int tstride, int kc, lds_int* lds) {
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (tile0 == 0 && threadIdx.x < kNL) g.ctl->bcnt[z3][threadIdx.x] = 0;
  const int cp = level & 1, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  const ArcTile t = arc_tile(lds + bq_words());
  const Prefix4 pre(load_counts(g.ctl->bcnt[c3]));
  const int ntiles = (pre.total + blockDim.x - 1) / blockDim.x;
  uint32_t nbytes = 0, narcs = 0;
  for (int tile = tile0; tile < ntiles; tile += tstride) {
    int nt = 0;
    const int A = load_arc_tile(g, t, cp, pre, tile, &nt);
    for (int a0 = 0; a0 < A; a0 += blockDim.x) {
      const int a = a0 + threadIdx.x;
      int t1 = 0, t2 = 0;
      bool v1 = false, v2 = false;
      if (a < A) {
        const int k = arc_owner(t, nt, a);
        const int x = t.node[k];
        const int j = a - t.off[k];
        const int b = t.beg[k];
        ++narcs;
        if (x < g.V) {
          const int2 ep2 = g.vinc[b + j];
          t1 = g.NB + 2 * ep2.x;
          t2 = t1 + 1;
          nbytes += 12;
          v1 = fwd_visit<kClaim>(g, t1, ep, ep_tmp);                    // x -> e_in (uncapped)
          if (g.fpin[2 * ep2.y + 1] > 0) v2 = fwd_visit<kClaim>(g, t2, ep, ep_tmp);  // x -> e_out reverse
        } else {
          const int e = (x - g.NB) >> 1;
          const bool in = ((x - g.NB) & 1) == 0;
          if (j == 0) {  // bridge
            const int fbv = g.fb[e];
            nbytes += 8;
            t1 = in ? x + 1 : x - 1;
            if (in ? fbv < g.w[e] : fbv > 0) v1 = fwd_visit<kClaim>(g, t1, ep, ep_tmp);
          } else {
            const int i = b + j - 1;
            t1 = g.pin_v[i];
            nbytes += 8;
            if (in) {
              if (g.w[e] - g.fpin[2 * i] > 0) v1 = fwd_visit<kClaim>(g, t1, ep, ep_tmp);  // e_in -> u reverse
            } else {
              const int r = g.role[t1];
              if (r == 2) atomicOr(&g.ctl->err, ERR_SINK_REACHED);
              else if (r == 0) v1 = fwd_visit<kClaim>(g, t1, ep, ep_tmp);  // e_out -> u infinite
            }
          }
        }
      }
      if (kClaim) {
        qpush(g, q, t1, v1);
        qpush(g, q, t2, v2);
        bq_tile_end(q, 2 * blockDim.x);
      }
    }
    __syncthreads();  // the tile area is rewritten by the next tile
  }
  if (kClaim) bq_flush(q);
  block_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 12ull * narcs, &g.ctl->items[kc],
                narcs);
}

// Bottom-up (pull) level, thread per node in id order: every unlabelled
// node scans its residual out-arcs of the capped network and takes label
// level+1 at the first arc into the level (only its own thread writes it):
//   vertex u:  u -> e_in if r_in > 0, u -> e_out if flow(e_out, u) > 0
//   e_in:      e_in -> e_out if fb < w, e_in -> u if flow(u, e_in) > 0
//   e_out:     e_out -> e_in if fb > 0, e_out -> u always
// The labels of the next level are then collected by the sweep.
__device__ void phase_bfs_rev_pull(const Dev& g, int level, int t0, int tstride, int kc) {
  // ring slot that nobody reads this level: the count of level+2
  if (t0 < kNL) g.ctl->bcnt[(level + 2) % 3][t0] = 0;
  const int lvl = level + 1;
  uint32_t nbytes = 0, narcs = 0;
  for (int v = t0; v < g.N; v += tstride) {
    if (seen_bit(g, v) || (v >= g.V && v < g.NB)) continue;
    if (g.d[v] != g.N) continue;
    bool hit = false;
    if (v < g.V) {
      const int beg = g.vtx_off[v], end = g.vtx_off[v + 1];
      nbytes += 12;
      for (int i = beg; i < end && !hit; ++i) {
        const int2 ep = g.vinc[i];
        const int2 dl = *reinterpret_cast<const int2*>(g.d + g.NB + 2 * ep.x);
        const int2 fp = *reinterpret_cast<const int2*>(g.fpin + 2 * ep.y);
        hit = (fp.x > 0 && dl.x == level) || (fp.y > 0 && dl.y == level);
        nbytes += 24;
        ++narcs;
      }
    } else {
      const int e = (v - g.NB) >> 1;
      const bool in = ((v - g.NB) & 1) == 0;
      const uint32_t nb = net_bits(g, e);
      nbytes += 16;
      ++narcs;
      hit = in ? ((nb & 1u) && g.d[v + 1] == level) : ((nb & 4u) && g.d[v - 1] == level);
      const int beg = g.net_off[e], end = g.net_off[e + 1];
      for (int p = beg; p < end && !hit; ++p) {
        if (in && !pin_flow_in(g, p)) continue;
        hit = g.d[g.pin_v[p]] == level;
        nbytes += 8;
        ++narcs;
      }
    }
    if (hit) {
      g.d[v] = lvl;
      if (g.lev) g.lev[v] = 1;  // listed (and marked 2) by the collect sweep
      set_seen(g, v);
    }
  }
  block_add_u64(&g.ctl->bytes[kc], nbytes, &g.ctl->items[kc], narcs);
}

template <int G>
__device__ void phase_bfs_rev(const Dev& g, int level, int tile0, int tstride, int kc,
                              lds_int* lds) {
  if (g.bfs_arc) phase_bfs_rev_lb<true>(g, level, tile0, tstride, kc, lds);
  else phase_bfs_rev_node<G, true>(g, level, tile0, tstride, kc, lds);
}

// Large levels run in two steps without claiming atomics: expand the level
// from its list, labelling unlabelled in-neighbours with plain stores (every
// writer stores the same value), then collect the next level by one sweep
// over the labels.
template <int G>
__device__ void phase_bfs_rev_expand(const Dev& g, int level, int tile0, int tstride, int kc,
                                     lds_int* lds) {
  if (g.bfs_arc) phase_bfs_rev_lb<false>(g, level, tile0, tstride, kc, lds);
  else phase_bfs_rev_node<G, false>(g, level, tile0, tstride, kc, lds);
}

// Sweep tiles: 2 nodes per thread, so a tile appends at most 2 * blockDim
// entries per list.
__device__ __forceinline__ int sweep_tiles(const Dev& g) {
  const int ts = 2 * blockDim.x;
  return (g.N + ts - 1) / ts;
}

__device__ void phase_bfs_collect(const Dev& g, int level, int tile0, int tstride, lds_int* lds) {
  // nodes labelled level+1 become the list of level+1
  const int n3 = (level + 1) % 3, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  const int lab = level + 1;
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      bool fresh = false;
      if (g.lev) {  // byte marks: the level's nodes carry mark 1 and get their label here
        fresh = v < g.N && g.lev[v] == 1;
        if (fresh) {
          g.lev[v] = 2;
          g.d[v] = lab;
        }
      } else {
        fresh = v < g.N && g.d[v] == lab;
      }
      qpush(g, q, v, fresh);
    }
    bq_tile_end(q, 2 * blockDim.x);
  }
  bq_flush(q);
}

// ---------------------------------------------------------------------------
// forward residual BFS of the uncapped network (source-side cut)
// ---------------------------------------------------------------------------

template <int G>
__device__ void phase_bfs_fwd(const Dev& g, int level, int ep, int tile0, int tstride, int kc,
                              lds_int* lds) {
  if (g.bfs_arc) phase_bfs_fwd_lb<true>(g, level, ep, 0, tile0, tstride, kc, lds);
  else phase_bfs_node<G, true, kDirSource>(g, level, ep, 0, tile0, tstride, kc, lds);
}

// Large forward levels: expand with provisional stamps, then list the next
// level by one sweep that turns them into the BFS stamp.
template <int G>
__device__ void phase_bfs_fwd_expand(const Dev& g, int level, int ep, int ep_tmp, int tile0,
                                     int tstride, int kc, lds_int* lds) {
  if (g.bfs_arc) phase_bfs_fwd_lb<false>(g, level, ep, ep_tmp, tile0, tstride, kc, lds);
  else phase_bfs_node<G, false, kDirSource>(g, level, ep, ep_tmp, tile0, tstride, kc, lds);
}

__device__ void phase_bfs_fwd_collect(const Dev& g, int level, int ep, int ep_tmp, int tile0,
                                      int tstride, lds_int* lds) {
  const int n3 = (level + 1) % 3, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      const bool fresh = v < g.N && g.stamp[v] == ep_tmp;
      if (fresh) g.stamp[v] = ep;
      qpush(g, q, v, fresh);
    }
    bq_tile_end(q, 2 * blockDim.x);
  }
  bq_flush(q);
}

// ---------------------------------------------------------------------------
// sweeps (thread per node); t0 wave-aligned, tstride a multiple of 64
// ---------------------------------------------------------------------------

// Zero flow, excess only at e_in of nets with a source pin (their contracted
// source arc saturated at w(e)), all counters cleared.
__device__ void phase_init(const Dev& g, int t0, int tstride) {
  if (t0 == 0) {
    Ctl* c = g.ctl;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) c->fcnt[i][k] = c->bcnt[i][k] = 0;
    c->err = 0;
    c->flow = 0ull;
    c->relabels = 0ull;
    for (int i = 0; i < KC_N; ++i) c->bytes[i] = c->items[i] = 0ull;
  }
  const int n = max(g.P, g.N);
  for (int i = t0; i < n; i += tstride) {
    if (i < g.P) {  // slot i: r_in = w(e), no flow (slots of a net are contiguous)
      *reinterpret_cast<int2*>(g.fpin + 2 * i) = make_int2(g.w[g.pin_net[i]], 0);
    }
    if (i < g.N) {
      g.stamp[i] = -1;
      g.cand[i] = -1;
      g.dx[0][i] = 0;
      g.dx[1][i] = 0;
      int xv = 0;
      if (i >= g.NB) {
        const int e = (i - g.NB) >> 1;
        if (((i - g.NB) & 1) == 0) {
          if (g.nflag[e] & 1) xv = g.w[e];
          g.fb[e] = 0;
        }
      }
      g.x[i] = xv;
    }
  }
}

// Global relabel, step 1: labels N for free nodes, 0 for sinks, N+1 for
// sources and padding; sinks form BFS level 0.  Round counters are cleared
// (the frontier is rebuilt by phase_gather).
__device__ void phase_gr_reset(const Dev& g, int tile0, int tstride, lds_int* lds) {
  if (tile0 == 0 && threadIdx.x == 0) {
    Ctl* c = g.ctl;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) c->fcnt[i][k] = 0;
    c->big_last = -1;
  }
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[0], g.list[0]);
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      bool seed = false;
      if (v < g.N) {
        int lab = g.N;
        if (v < g.V) {
          const int r = g.role[v];
          lab = r == 1 ? g.N + 1 : (r == 2 ? 0 : g.N);
          seed = r == 2;
        } else if (v < g.NB) {
          lab = g.N + 1;
        }
        g.d[v] = lab;
        if (g.lev) g.lev[v] = lab == g.N ? 0 : 2;
      }
      qpush(g, q, v, seed);
    }
    bq_tile_end(q, 2 * blockDim.x);
  }
  bq_flush(q);
  // labelled hint: sinks, sources and padding start labelled
  const int words = (g.N + 31) >> 5;
  for (int w = tile0 * blockDim.x + threadIdx.x; w < words; w += tstride * blockDim.x) {
    uint32_t m = 0;
    const int v0 = w << 5;
    if (v0 < g.NB) {
      for (int b = 0; b < 32; ++b) {
        const int v = v0 + b;
        if (v >= g.V ? v < g.NB : g.role[v] != 0) m |= 1u << b;
      }
    }
    g.seen[w] = m;
  }
}

// Global relabel, step 3: fold outstanding excess deltas; frontier =
// non-terminal nodes with excess and a label below N; stale relabel
// candidates dropped.  BFS counters are cleared for the next BFS.
__device__ void phase_gather(const Dev& g, int epoch, int tile0, int tstride, lds_int* lds) {
  const int c3 = epoch % 3, cp = epoch & 1;
  if (tile0 == 0 && threadIdx.x == 0) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) g.ctl->bcnt[i][k] = 0;
  }
  const BlockQ q = bq_bind(lds, g.ctl->fcnt[c3], g.list[cp]);
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      bool act = false;
      if (v < g.N) {
        const int a = g.dx[0][v], b = g.dx[1][v];
        int xv = g.x[v];
        if (a | b) {
          xv += a + b;
          g.x[v] = xv;
          g.dx[0][v] = 0;
          g.dx[1][v] = 0;
        }
        if (g.cand[v] >= 0) g.cand[v] = -1;
        if (v >= g.NB || (v < g.V && g.role[v] == 0)) act = xv > 0 && g.d[v] < g.N;
      }
      qpush(g, q, v, act);
    }
    bq_tile_end(q, 2 * blockDim.x);
  }
  bq_flush(q);
}

// Cut BFS seeds: sources (marked, nothing to expand: their only arcs are the
// contracted source arcs into e_in), e_in of nets with a source pin, and
// every non-terminal node holding excess.  With only_new, nodes that already
// carry ep are left out (growing an existing source side).
__device__ void phase_cut_seed(const Dev& g, int ep, bool only_new, int tile0, int tstride,
                               lds_int* lds) {
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[0], g.list[0]);
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      bool seed = false;
      if (v < g.N) {
        if (v < g.V) {
          const int r = g.role[v];
          if (r == 1) g.stamp[v] = ep;
          else if (r == 0 && g.x[v] > 0) seed = true;
        } else if (v >= g.NB) {
          const int e = (v - g.NB) >> 1;
          const bool in = ((v - g.NB) & 1) == 0;
          seed = g.x[v] > 0 || (in && (g.nflag[e] & 1));
        }
        if (seed && only_new && g.stamp[v] == ep) seed = false;
        if (seed) g.stamp[v] = ep;
      }
      qpush(g, q, v, seed);
    }
    bq_tile_end(q, 2 * blockDim.x);
  }
  bq_flush(q);
}

// Write the side bitmaps and clear BFS counters.
__device__ void phase_cut_out(const Dev& g, int ep, uint8_t* vside, uint8_t* nside, int t0,
                              int tstride) {
  if (t0 == 0) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) g.ctl->bcnt[i][k] = 0;
  }
  const int n = max(g.V, g.E);
  for (int i = t0; i < n; i += tstride) {
    if (i < g.V) {
      const int r = g.role[i];
      vside[i] = (uint8_t)(r == 1 ? 1 : (r == 2 ? 0 : (g.stamp[i] == ep)));
    }
    if (i < g.E && nside) {
      const int a = g.stamp[g.NB + 2 * i] == ep;
      const int b = g.stamp[g.NB + 2 * i + 1] == ep;
      nside[i] = (uint8_t)(a | (b << 1));
    }
  }
}

// ---------------------------------------------------------------------------
// maximal sink side: reverse residual BFS from the sinks over the uncapped
// network (paper, algorithm "FlowCutter Core": T_r by backward residual
// BFS).  Node a joins when it has a residual arc into the current level:
//   into a vertex u   from e_out (infinite) and from e_in if flow(u, e_in) > 0
//   into e_in         from every pin (u -> e_in uncapped) and from e_out if fb > 0
//   into e_out        from e_in if fb < w and from pins u with flow(e_out, u) > 0
// Sources never join (a maximum preflow leaves no residual path from the
// source to a sink); reaching one is reported as ERR_SOURCE_REACHED.
// ---------------------------------------------------------------------------

// Seeds: the sinks.  The BFS counters must be clear (phase_reset_bfs).
__device__ void phase_sink_seed(const Dev& g, int ep, int tile0, int tstride, lds_int* lds) {
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[0], g.list[0]);
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      const bool seed = v < g.V && g.role[v] == 2;
      if (seed) g.stamp[v] = ep;
      qpush(g, q, v, seed);
    }
    bq_tile_end(q, 2 * blockDim.x);
  }
  bq_flush(q);
}

// The same sink side from exact labels of the capped network (the labels
// of a global relabel that found no active node): a node reaches a sink in
// the capped residual network exactly when its label is below N, and that
// set D lies in T_r, the uncapped network having every residual arc of the
// capped one.  The two networks differ only in the pin arcs u -> e_in,
// residual in the uncapped network even when saturated, so a residual path
// from outside D enters D by such an arc: its tail u (label N or more, arc
// saturated into an e_in of D) is a seed, and the reverse BFS of the
// uncapped network continues from the seeds through the nodes outside D.
// Stamps D with ep and lists the seeds as level 0 (counters clear).  A
// source's pin arcs carry no flow, so none qualifies; one that did would
// reach a sink (ERR_SOURCE_REACHED).
__device__ void phase_sink_seed_labels(const Dev& g, int ep, int tile0, int tstride,
                                       lds_int* lds) {
  const int ntiles = sweep_tiles(g);
  for (int tile = tile0; tile < ntiles; tile += tstride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int v = (2 * tile + j) * blockDim.x + threadIdx.x;
      if (v < g.N && g.d[v] < g.N) g.stamp[v] = ep;
    }
  }
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[0], g.list[0]);
  const int ptiles = (g.P + (int)blockDim.x - 1) / (int)blockDim.x;
  for (int tile = tile0; tile < ptiles; tile += tstride) {
    const int p = tile * (int)blockDim.x + (int)threadIdx.x;
    int u = 0;
    bool seed = false;
    if (p < g.P && g.fpin[2 * p] == 0) {  // u -> e_in saturated (flow w(e))
      u = g.pin_v[p];
      if (g.d[g.NB + 2 * g.pin_net[p]] < g.N && g.d[u] >= g.N) {
        if (g.role[u] == 1) atomicOr(&g.ctl->err, ERR_SOURCE_REACHED);
        else seed = stamp_first(g, u, ep);
      }
    }
    qpush(g, q, u, seed);
    bq_tile_end(q, (int)blockDim.x);
  }
  bq_flush(q);
}

__device__ void phase_bfs_sink_lb(const Dev& g, int level, int ep, int tile0, int tstride, int kc,
                                  lds_int* lds) {
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (tile0 == 0 && threadIdx.x < kNL) g.ctl->bcnt[z3][threadIdx.x] = 0;
  const int cp = level & 1, np = (level + 1) & 1;
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[n3], g.list[np]);
  const ArcTile t = arc_tile(lds + bq_words());
  const Prefix4 pre(load_counts(g.ctl->bcnt[c3]));
  const int ntiles = (pre.total + blockDim.x - 1) / blockDim.x;
  uint32_t nbytes = 0, narcs = 0;
  bool hit_source = false;
  for (int tile = tile0; tile < ntiles; tile += tstride) {
    int nt = 0;
    const int A = load_arc_tile(g, t, cp, pre, tile, &nt);
    for (int a0 = 0; a0 < A; a0 += blockDim.x) {
      const int a = a0 + threadIdx.x;
      int t1 = 0, t2 = 0;
      bool v1 = false, v2 = false;
      if (a < A) {
        const int k = arc_owner(t, nt, a);
        const int x = t.node[k];
        const int j = a - t.off[k];
        const int b = t.beg[k];
        ++narcs;
        if (x < g.V) {
          const int2 ep2 = g.vinc[b + j];
          t1 = g.NB + 2 * ep2.x;
          t2 = t1 + 1;
          nbytes += 12;
          v2 = stamp_first(g, t2, ep);                                         // e_out -> x
          if (g.w[ep2.x] - g.fpin[2 * ep2.y] > 0) v1 = stamp_first(g, t1, ep);  // e_in -> x
        } else {
          const int e = (x - g.NB) >> 1;
          const bool in = ((x - g.NB) & 1) == 0;
          if (j == 0) {  // bridge
            const int fbv = g.fb[e];
            nbytes += 8;
            t1 = in ? x + 1 : x - 1;
            if (in ? fbv > 0 : fbv < g.w[e]) v1 = stamp_first(g, t1, ep);
          } else {
            const int i = b + j - 1;
            t1 = g.pin_v[i];
            const int r = g.role[t1];
            nbytes += 8;
            const bool arc = in || g.fpin[2 * i + 1] > 0;  // u -> e_in always, u -> e_out by flow
            if (arc) {
              if (r == 1) hit_source = true;
              else v1 = stamp_first(g, t1, ep);
            }
          }
        }
      }
      qpush(g, q, t1, v1);
      qpush(g, q, t2, v2);
      bq_tile_end(q, 2 * blockDim.x);
    }
    __syncthreads();  // the tile area is rewritten by the next tile
  }
  bq_flush(q);
  if (hit_source) atomicOr(&g.ctl->err, ERR_SOURCE_REACHED);
  block_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 12ull * narcs, &g.ctl->items[kc],
                narcs);
}

template <int G>
__device__ void phase_bfs_sink(const Dev& g, int level, int ep, int tile0, int tstride, int kc,
                               lds_int* lds) {
  if (g.bfs_arc) phase_bfs_sink_lb(g, level, ep, tile0, tstride, kc, lds);
  else phase_bfs_node<G, true, kDirSink>(g, level, ep, 0, tile0, tstride, kc, lds);
}

// Clear the BFS counters and the FlowCutter side weights (own launch: the
// next phase appends to the counters).
__device__ void phase_reset_bfs(const Dev& g) {
  if (threadIdx.x == 0) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) g.ctl->bcnt[i][k] = 0;
    g.ctl->side_weight[0] = 0ull;
    g.ctl->side_weight[1] = 0ull;
    for (int i = 0; i < 5; ++i) g.ctl->pierce[i] = kInf;
  }
}

// Clear the frontier counters of all three round slots (a solve that starts
// from the labels it has, without a global relabel, gathers into one).
__device__ void phase_clear_frontiers(const Dev& g) {
  if (threadIdx.x == 0)
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) g.ctl->fcnt[i][k] = 0;
}

// One seed vertex p (already stamped by the caller) as BFS level 0.  The
// BFS counters must be clear (phase_reset_bfs).
__device__ void phase_seed_vertex(const Dev& g, int p) {
  if (threadIdx.x == 0) {
    const int k = list_of(g, p);
    g.list[0][k][0] = p;
    g.ctl->bcnt[0][k] = 1;
  }
}

// Bulk piercing (paragraph "Bulk Piercing"): flag[u] = 1 for every augmenting
// candidate of side `side` -- a pin of a net cut by that side's bipartition
// that lies on the opposite side's reachable set and is not a terminal yet.
// Thread per net; flags are cleared by the caller.
// Whether net e is cut by (S_r, V - S_r) (.x) and by (V - T_r, T_r) (.y),
// read from the stamps of its two nodes (e_in, e_out adjacent: one 8-byte
// load).  In the uncapped network every pin reaches e_in and e_out reaches
// every pin, so a non-empty net has a pin in S_r iff e_in is in S_r and all
// its pins in S_r when e_out is; it has a pin in T_r iff e_out is in T_r and
// all its pins in T_r when e_in is.  A net flagged here may still have all
// its pins on one side (its bridge blocks); the pin scans that follow then
// find no pin outside, so the flag changes nothing.
struct bool2_t {
  bool a, b;
};

__device__ __forceinline__ bool2_t net_cut_flags(const Dev& g, int e, int ep_s, int ep_t) {
  const int2 st = reinterpret_cast<const int2*>(g.stamp + g.NB)[e];
  return bool2_t{st.x == ep_s && st.y != ep_s, st.y == ep_t && st.x != ep_t};
}

// Flags the pins of nets cut by side `side`'s bipartition that lie on the
// other side and are not its terminals yet (the augmenting candidates of a
// bulk pierce).  Lanes take one net each; the nets that are cut are then
// scanned by the whole wave, one after another, 64 pins at a time.
__device__ void phase_fc_mark_augmenting(const Dev& g, int side, int ep_s, int ep_t,
                                         uint8_t* flag, int t0, int tstride) {
  const int lane = lane_id();
  const int other = side == 0 ? ep_t : ep_s;
  const int other_role = side == 0 ? 2 : 1;
  for (int base = t0 - lane; base < g.E; base += tstride) {
    const int e = base + lane;
    bool cut = false;
    if (e < g.E) {
      const bool2_t c = net_cut_flags(g, e, ep_s, ep_t);
      cut = side == 0 ? c.a : c.b;
    }
    unsigned long long m = __ballot(cut);
    while (m) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      const int en = base + b;
      const int beg = g.net_off[en], end = g.net_off[en + 1];
      for (int p = beg + lane; p < end; p += 64) {
        const int u = g.pin_v[p];
        if (g.stamp[u] == other && g.role[u] != other_role) flag[u] = 1;
      }
    }
  }
}

// Exclusive prefix of per-thread 0/1 values over a workgroup (blockDim a
// multiple of 64, at most 1024); *total gets the workgroup's sum.
__device__ int block_rank(int f, int* total) {
  __shared__ int wsum[17];
  const int lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long m = __ballot(f != 0);
  const int below = __popcll(m & lanemask_lt());
  if (lane == 0) wsum[wid] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < nw; ++i) {
      const int t = wsum[i];
      wsum[i] = run;
      run += t;
    }
    wsum[nw] = run;
  }
  __syncthreads();
  const int r = wsum[wid] + below;
  *total = wsum[nw];
  __syncthreads();
  return r;
}

// Flag counts per workgroup tile of blockDim vertices.
__device__ void phase_count_flags(const uint8_t* flag, int V, int32_t* counts) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  int total = 0;
  block_rank(v < V && flag[v] != 0, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Stamp with ep the k flagged vertices of smallest id; offsets[b] = flags
// before tile b.
__device__ void phase_select_flags(Dev g, const uint8_t* flag, int V, const int32_t* offsets,
                                   int k, int ep) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool f = v < V && flag[v] != 0;
  int total = 0;
  const int r = offsets[blockIdx.x] + block_rank(f, &total);
  if (f && r < k) g.stamp[v] = ep;
}

// Vertex bitmap of a BFS: 1 where the vertex carries stamp ep (when
// invert, 1 where it does not).
__device__ void phase_side_out(const Dev& g, int ep, bool invert, uint8_t* vside, int t0,
                               int tstride) {
  if (t0 == 0) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < kNL; ++k) g.ctl->bcnt[i][k] = 0;
  }
  for (int v = t0; v < g.V; v += tstride) vside[v] = (uint8_t)((g.stamp[v] == ep) != invert);
}

// ---------------------------------------------------------------------------
// FlowCutter steps (paper, section "Flow-Based Refinement": algorithm
// "FlowCutter Core", paragraphs "Piercing", "Sink-Side Piercing" and
// "Maintain Distance Labels").  S_r carries stamp ep_s (sources included),
// T_r stamp ep_t (sinks included).
// ---------------------------------------------------------------------------

// Weights c(S_r) and c(T_r), and pierce[2] = the smallest vertex outside
// both (the counters are cleared by phase_reset_bfs).
__device__ void phase_fc_weights(const Dev& g, const int32_t* cw, int ep_s, int ep_t, int t0,
                                 int tstride) {
  unsigned long long ws = 0, wt = 0;
  int first_free = kInf;
  for (int v = t0; v < g.V; v += tstride) {
    const int st = g.stamp[v];
    if (st == ep_s) ws += (unsigned long long)cw[v];
    else if (st == ep_t) wt += (unsigned long long)cw[v];
    else first_free = min(first_free, v);
  }
  block_add_u64(&g.ctl->side_weight[0], ws, &g.ctl->side_weight[1], wt);
  block_min_i32(&g.ctl->pierce[2], first_free, &g.ctl->pierce[2], kInf);
}

// Piercing candidates of the side that is pierced next, the lighter one
// (s = 0 when c(S_r) <= c(T_r), from the weights phase_fc_weights summed
// before): pierce[3s] = the smallest vertex outside S_r and T_r on a net cut
// by side s's bipartition; pierce[3s + 1] = the smallest vertex of the
// opposite reachable set on such a net that is not a terminal yet.  The
// second is only used when no vertex is outside both sets (pierce[2] =
// kInf), so only then is it searched, and then the first has no candidate.
// Vertex order, with the uncapped network's reachability: a vertex outside
// S_r lies on a net cut by (S_r, V - S_r) exactly when one of its nets has
// e_in in S_r (were e_out in S_r, its pins would be too); one outside T_r
// lies on a net cut by (V - T_r, T_r) exactly when one of its nets has e_out
// in T_r.  Workgroups take chunks of blockDim vertices in increasing order
// (chunk b, b + gridDim, ...) and stop at the first chunk that starts above
// the best candidate found so far: a vertex of that chunk or a later one
// cannot be the smallest, and most free vertices next to a side are found
// in the first chunks.
__device__ void phase_fc_pick(const Dev& g, int ep_s, int ep_t) {
  __shared__ int best_sh;
  const unsigned long long cs = ld_vol64(&g.ctl->side_weight[0]);
  const unsigned long long ct = ld_vol64(&g.ctl->side_weight[1]);
  const int side = cs <= ct ? 0 : 1;
  const bool aug = ld_vol(&g.ctl->pierce[2]) == kInf;
  const int want = side == 0 ? ep_s : ep_t;  // stamp of the net node that makes a net cut
  const int opp = side == 0 ? ep_t : ep_s;
  const int opp_role = side == 0 ? 2 : 1;
  int32_t* const out = &g.ctl->pierce[3 * side + (aug ? 1 : 0)];
  const int nchunks = (g.V + (int)blockDim.x - 1) / (int)blockDim.x;
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int u = c * (int)blockDim.x + (int)threadIdx.x;
    int found = kInf;
    if (u < g.V) {
      const int st = g.stamp[u];
      const bool look = aug ? (st == opp && g.role[u] != opp_role) : (st != ep_s && st != ep_t);
      if (look) {
        const int end = g.vtx_off[u + 1];
        for (int i = g.vtx_off[u]; i < end; ++i) {
          if (g.stamp[g.NB + 2 * g.vinc[i].x + side] == want) {
            found = u;
            break;
          }
        }
      }
    }
    block_min_i32(out, found, out, kInf);
    if (threadIdx.x == 0) best_sh = ld_vol(out);
    __syncthreads();
    const int best = best_sh;
    __syncthreads();
    if ((long long)(c + gridDim.x) * blockDim.x > (long long)best) break;
  }
}

// Every free vertex with stamp ep_s becomes a source.  The flows of its
// pin arcs are cancelled (flow(u, e_in) back out of e_in's excess, flow
// (e_out, u) back into e_out's excess), and a net that gains its first
// source pin receives w(e) through its contracted source arc, so the state
// stays a preflow of the new network with the same flow value.  The vertex
// takes the sources' label N + 1.  No residual arc between non-terminal
// nodes appears (the arcs that change all start or end at the new source),
// so the other labels stay valid and the next solve may start from them
// (paragraph "Maintain Distance Labels").
// Incidence i (net e) of a vertex u that becomes a source: the flows of u's
// pin arcs are cancelled -- e_in loses the flow u sent it and, when e gets its
// first source pin, gains w(e) from the contracted source arc; e_out keeps as
// excess the flow it sent to u.  Returns e and the flow returned to e_out.
__device__ __forceinline__ int2 cancel_source_pin(const Dev& g, int i) {
  const int2 ep = g.vinc[i];
  const int e = ep.x;
  const int we = g.w[e];
  const int fin = we - g.fpin[2 * ep.y];
  const int fout = g.fpin[2 * ep.y + 1];
  int add_in = -fin;
  const int old = atomicOr(&g.nflag[e], 1);
  if (!(old & 1)) add_in += we;
  if (add_in) atomicAdd(&g.x[g.NB + 2 * e], add_in);
  if (fout) atomicAdd(&g.x[g.NB + 2 * e + 1], fout);
  g.fpin[2 * ep.y] = we;
  g.fpin[2 * ep.y + 1] = 0;
  return make_int2(e, fout);
}

__device__ void phase_pierce_sources(const Dev& g, int ep_s, int t0, int tstride) {
  for (int v = t0; v < g.V; v += tstride) {
    if (g.role[v] != 0 || g.stamp[v] != ep_s) continue;
    g.role[v] = 1;
    g.d[v] = g.N + 1;  // a source's label: nothing is pushed into it
    for (int i = g.vtx_off[v]; i < g.vtx_off[v + 1]; ++i) cancel_source_pin(g, i);
  }
}

// The source pierce above that also lists the seeds of the source side's
// growth (a pierce that avoids augmenting paths keeps S_r, which the growth
// extends): converting a vertex gives e_in of each of its nets a source arc
// and, where flow came back, e_out excess; no other node gains excess or a
// source arc, and every node that held them before is already in S_r.  Each
// such net node not yet stamped ep_s is stamped and listed once (exchange on
// the stamp), so level 0 is exactly what the seed sweep over all nodes would
// find.  Thread per vertex in tiles of blockDim; level 0's count and lists
// must be empty.
__device__ void phase_pierce_sources_seed(const Dev& g, int ep_s, int tile0, int tstride,
                                          lds_int* lds) {
  const BlockQ q = bq_bind(lds, g.ctl->bcnt[0], g.list[0]);
  const int ntiles = (g.V + (int)blockDim.x - 1) / (int)blockDim.x;
  for (int tile = tile0; tile < ntiles; tile += tstride) {
    const int v = tile * (int)blockDim.x + (int)threadIdx.x;
    int beg = 0, end = 0;
    if (v < g.V && g.role[v] == 0 && g.stamp[v] == ep_s) {
      g.role[v] = 1;
      g.d[v] = g.N + 1;
      beg = g.vtx_off[v];
      end = g.vtx_off[v + 1];
    }
    for (int i = beg; i < end; ++i) {
      const int2 ef = cancel_source_pin(g, i);
      const int ein = g.NB + 2 * ef.x;
      qpush(g, q, ein, stamp_first(g, ein, ep_s));
      qpush(g, q, ein + 1, ef.y > 0 && stamp_first(g, ein + 1, ep_s));
    }
    bq_tile_end(q, q.cap / 2);
  }
  bq_flush(q);
}

// Every free vertex with stamp ep_t becomes a sink; excess it holds joins
// the flow value (paragraph "Sink-Side Piercing").
__device__ void phase_pierce_sinks(const Dev& g, int ep_t, int t0, int tstride) {
  unsigned long long gained = 0;
  for (int v = t0; v < g.V; v += tstride) {
    if (g.role[v] != 0 || g.stamp[v] != ep_t) continue;
    g.role[v] = 2;
    const int xv = g.x[v];
    if (xv > 0) {
      gained += (unsigned long long)xv;
      g.x[v] = 0;
    }
    for (int i = g.vtx_off[v]; i < g.vtx_off[v + 1]; ++i) atomicOr(&g.nflag[g.vinc[i].x], 2);
  }
  block_add_u64(&g.ctl->flow, gained);
}

// Stamp the given vertices with ep; a vertex that is a terminal of kind
// `forbidden` is reported as ERR_PIERCE_TERMINAL.
__device__ void phase_mark(const Dev& g, const int32_t* vs, int n, int ep, int forbidden, int t0,
                           int tstride) {
  for (int i = t0; i < n; i += tstride) {
    const int v = vs[i];
    if (g.role[v] == forbidden) atomicOr(&g.ctl->err, ERR_PIERCE_TERMINAL);
    else if (g.role[v] == 0) g.stamp[v] = ep;
  }
}

// Debug: preflow feasibility (excess = inflow - outflow >= 0, capacities) and
// label validity on every residual arc of the capped network, after a
// completed round.  Thread per vertex / net / pin.
__device__ __forceinline__ long long excess_of(const Dev& g, int v) {
  return (long long)g.x[v] + g.dx[0][v] + g.dx[1][v];
}

__device__ void phase_check(const Dev& g, int t0, int tstride) {
  const int n = max(g.P, max(g.E, g.V));
  bool bad = false;
  for (int i = t0; i < n; i += tstride) {
    if (i < g.V) {
      const int r = g.role[i];
      if (r == 0) {
        long long s = 0;
        for (int j = g.vtx_off[i]; j < g.vtx_off[i + 1]; ++j) {
          const int2 ep = g.vinc[j];
          s += (long long)g.fpin[2 * ep.y + 1] - (long long)(g.w[ep.x] - g.fpin[2 * ep.y]);
        }
        if (s != excess_of(g, i) || s < 0) bad = true;
      }
    }
    if (i < g.E) {
      const int we = g.w[i], fbv = g.fb[i];
      if (fbv < 0 || fbv > we) bad = true;
      long long sin = (g.nflag[i] & 1) ? we : 0, sout = 0;
      for (int p = g.net_off[i]; p < g.net_off[i + 1]; ++p) {
        sin += we - g.fpin[2 * p];
        sout += g.fpin[2 * p + 1];
      }
      const long long xin = excess_of(g, g.NB + 2 * i), xout = excess_of(g, g.NB + 2 * i + 1);
      if (sin - fbv != xin || fbv - sout != xout || xin < 0 || xout < 0) bad = true;
      const int din = g.d[g.NB + 2 * i], dout = g.d[g.NB + 2 * i + 1];
      if (din < g.N && fbv < we && din > dout + 1) bad = true;
      if (dout < g.N && fbv > 0 && dout > din + 1) bad = true;
    }
    if (i < g.P) {
      const int2 ep = g.vinc[i];
      const int e = ep.x, p = ep.y;
      const int u = g.pin_v[p];
      const int rin = g.fpin[2 * p], fout = g.fpin[2 * p + 1];
      const int we = g.w[e];
      if (rin < 0 || rin > we || fout < 0) bad = true;
      const int r = g.role[u];
      if (r == 1 && rin != we) bad = true;  // no flow leaves a source
      if (r == 1 && fout != 0) bad = true;  // nothing enters a source
      const int du = g.d[u], din = g.d[g.NB + 2 * e], dout = g.d[g.NB + 2 * e + 1];
      if (r == 0) {
        if (du < g.N && rin > 0 && du > din + 1) bad = true;        // u -> e_in
        if (du < g.N && fout > 0 && du > dout + 1) bad = true;      // u -> e_out
        if (din < g.N && we - rin > 0 && din > du + 1) bad = true;  // e_in -> u
      }
      if (dout < g.N && r != 1 && dout > du + 1) bad = true;  // e_out -> u
    }
  }
  if (bad) atomicOr(&g.ctl->err, ERR_INVARIANT);
}

}  // namespace hf
