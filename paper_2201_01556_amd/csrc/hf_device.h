// Device-side phases of the hypergraph push-relabel solver (gfx950).
//
// Network (Lawler expansion, paper section "Preliminaries", paragraph "Flows
// on Hypergraphs"), simulated on the hypergraph itself as the paper's
// paragraph "Hypergraph Implementation" describes -- the expanded graph is
// never built.  Node ids:
//   v            in [0, V)      hypernode
//   NB + 2e                     e_in  of net e     (NB = V rounded up to even,
//   NB + 2e + 1                 e_out of net e      so (e_in, e_out) labels and
//                                                   excesses form an int2)
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
// split into two phases with a device-wide ordering point between them:
//   push   every frontier node u with label k = d(u) < N and excess X pushes
//          along arcs admissible under the round-start labels
//          (residual > 0 and d(v) = k - 1) and distributes X over them in arc
//          order; it records cand = 1 + min label over the arcs that stay
//          residual after its own pushes.  Admissibility is antisymmetric in
//          the labels, so each arc pair has a single writer per round and no
//          winning criterion is needed.
//   apply  a node left with excess is relabelled to
//          min(cand, d(u) + 2 if something was pushed into u this round, N).
//          Pushes into u come from nodes labelled d(u) + 1 and are the only
//          residual arcs u could not see; the bound keeps every label valid
//          (d(a) <= d(b) + 1 on every residual arc), which rules out the
//          push-relabel conflict described in section "A Bug in the
//          Synchronous Algorithm".
// Frontier = nodes pushed into (deduplicated by a per-round stamp) plus nodes
// relabelled below N, compacted with wave ballots (paragraph "Active Nodes").
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

constexpr int kWave = 64;
constexpr int kInf = 0x7fffffff;

// error bits reported through Ctl::err
enum : int32_t {
  ERR_LABEL = 1,        // a relabel did not raise the label
  ERR_SINK_REACHED = 2, // forward cut BFS reached a sink
  ERR_INVARIANT = 4,    // debug invariant check failed
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
  KC_N = 8
};

struct Ctl {
  int32_t fcnt[3][2];  // round frontier counts, ring by epoch % 3, [small, big]
  int32_t lcnt[3];     // leftover (relabel) list counts, ring by epoch % 3
  int32_t bcnt[3][2];  // BFS level counts, ring by level % 3
  int32_t err;
  int32_t loop_rounds;  // rounds run by the last single-workgroup round loop
  int32_t loop_levels;  // levels run by the last single-workgroup BFS loop
  int32_t loop_exit;
  int32_t pad0;
  unsigned long long flow;      // flow value (into sinks)
  unsigned long long relabels;  // relabel operations
  unsigned long long bytes[KC_N];
  unsigned long long items[KC_N];
};

struct Dev {
  int32_t V, E, P, NB, N, nT, big_deg, pad;
  const int32_t* net_off;  // E+1
  const int32_t* pin_v;    // P
  const int32_t* w;        // E
  const int32_t* vtx_off;  // V+1
  const int2* vinc;        // P   {net, pin slot}, per vertex sorted by slot
  int32_t* role;           // V   0 free, 1 source, 2 sink
  int32_t* nflag;          // E   bit0 has a source pin, bit1 has a sink pin
  int32_t* tlist;          // sinks (capacity V)
  int32_t* fpin;           // 2P  {r_in, f_out}
  int32_t* fb;             // E
  int32_t* d;              // N   labels
  int32_t* x;              // N   excess
  int32_t* stamp;          // N
  int32_t* list[2][2];     // [parity][small, big], capacity N each
  int2* left;              // N   {node, cand}
  Ctl* ctl;
};

// ---------------------------------------------------------------------------
// wave / group utilities
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Aggregated append: every active lane calls it; lanes with pred get
// consecutive slots from one atomic per wave.
__device__ __forceinline__ int wave_append(int32_t* cnt, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return 0;
  const int leader = __builtin_ctzll(m);
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, leader);
  return base + __popcll(m & ((1ull << lane_id()) - 1ull));
}

// Sum over the wave, one atomic.  The whole wave must be active.
__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane_id() == 0 && v != 0ull) atomicAdd(dst, v);
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

template <int G>
__device__ __forceinline__ uint32_t g_sum(uint32_t v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

__device__ __forceinline__ int deg_of(const Dev& g, int v) {
  if (v < g.V) return g.vtx_off[v + 1] - g.vtx_off[v];
  const int e = (v - g.NB) >> 1;
  return g.net_off[e + 1] - g.net_off[e] + 1;
}

// Append v (if pred) to the small or big list of a frontier.
__device__ __forceinline__ void push_frontier(const Dev& g, int32_t* cnt2, int32_t* ls,
                                              int32_t* lb, int v, bool pred) {
  bool big = false;
  if (pred) big = deg_of(g, v) > g.big_deg;
  const int is = wave_append(&cnt2[0], pred && !big);
  const int ib = wave_append(&cnt2[1], pred && big);
  if (pred) {
    if (big) lb[ib] = v;
    else ls[is] = v;
  }
}

// Round-scoped stamp: true for exactly one caller per (v, epoch).
__device__ __forceinline__ bool stamp_first(const Dev& g, int v, int epoch) {
  if (g.stamp[v] == epoch) return false;
  return atomicExch(&g.stamp[v], epoch) != epoch;
}

struct RoundArgs {
  int epoch;   // unique id of this round
  int cur3;    // epoch % 3
  int nxt3;    // (epoch + 1) % 3
  int nxtp;    // (epoch + 1) % 2
};

__device__ __forceinline__ RoundArgs round_args(int epoch) {
  RoundArgs a;
  a.epoch = epoch;
  a.cur3 = epoch % 3;
  a.nxt3 = (epoch + 1) % 3;
  a.nxtp = (epoch + 1) & 1;
  return a;
}

__device__ __forceinline__ void mark_pushed(const Dev& g, const RoundArgs& ra, int v, bool pred) {
  bool fresh = false;
  if (pred) fresh = stamp_first(g, v, ra.epoch);
  push_frontier(g, g.ctl->fcnt[ra.nxt3], g.list[ra.nxtp][0], g.list[ra.nxtp][1], v, fresh);
}

// End of a node's push scan: give up the pushed excess; a node left with
// excess goes to the relabel list with its candidate label.
template <int G>
__device__ __forceinline__ void finish_push(const Dev& g, const RoundArgs& ra, int u,
                                            uint32_t X, uint32_t pushed, int cand, int gl,
                                            bool active) {
  if (active && gl == 0 && pushed > 0u) atomicSub(&g.x[u], (int)pushed);
  const bool left = active && pushed < X;
  if (left) cand = g_min<G>(cand);
  const int slot = wave_append(&g.ctl->lcnt[ra.cur3], left && gl == 0);
  if (left && gl == 0) g.left[slot] = make_int2(u, cand);
}

// ---------------------------------------------------------------------------
// push phase, per node kind (G lanes per node, group-uniform control flow)
// ---------------------------------------------------------------------------

template <int G>
__device__ void push_vertex(const Dev& g, const RoundArgs& ra, int u, bool has, int gl,
                            uint32_t& nbytes) {
  int k = 0, X = 0, beg = 0, end = 0;
  if (has) {
    k = g.d[u];
    X = g.x[u];
    beg = g.vtx_off[u];
    end = g.vtx_off[u + 1];
  }
  const bool active = has && k < g.N && X > 0;
  const uint32_t UX = active ? (uint32_t)X : 0u;
  uint32_t carry = 0;
  int cand = kInf;
  if (active) {
    nbytes += 16;
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
      if (g1) {
        g.fpin[2 * p] = (int)(r1 - g1);
        atomicAdd(&g.x[g.NB + 2 * e], (int)g1);
      }
      if (g2) {
        g.fpin[2 * p + 1] = (int)(r2 - g2);
        atomicAdd(&g.x[g.NB + 2 * e + 1], (int)g2);
      }
      mark_pushed(g, ra, g.NB + 2 * e, g1 > 0u);
      mark_pushed(g, ra, g.NB + 2 * e + 1, g2 > 0u);
      if (valid) {
        if (r1 > g1) cand = min(cand, dl.x + 1);
        if (r2 > g2) cand = min(cand, dl.y + 1);
      }
      carry = min(carry + __shfl(incl, G - 1, G), UX);
      if (carry >= UX) break;
    }
  }
  finish_push<G>(g, ra, u, UX, carry, cand, gl, active);
}

template <int G>
__device__ void push_ein(const Dev& g, const RoundArgs& ra, int node, bool has, int gl,
                         uint32_t& nbytes) {
  const int e = (node - g.NB) >> 1;
  int k = 0, X = 0;
  if (has) {
    k = g.d[node];
    X = g.x[node];
  }
  const bool active = has && k < g.N && X > 0;
  const uint32_t UX = active ? (uint32_t)X : 0u;
  uint32_t carry = 0;
  int cand = kInf;
  if (active) {
    const int we = g.w[e];
    const int fbv = g.fb[e];
    const int dout = g.d[node + 1];
    nbytes += 32;
    const uint32_t rb = (uint32_t)(we - fbv);
    const bool ab = rb > 0u && dout == k - 1;
    const uint32_t gb = ab ? min(rb, UX) : 0u;
    if (gb && gl == 0) {
      g.fb[e] = fbv + (int)gb;
      atomicAdd(&g.x[node + 1], (int)gb);
    }
    mark_pushed(g, ra, node + 1, gb > 0u && gl == 0);
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
        if (give) {
          g.fpin[2 * i] = rin + (int)give;
          atomicAdd(&g.x[u], (int)give);
        }
        mark_pushed(g, ra, u, give > 0u);
        if (valid && r > give) cand = min(cand, du + 1);
        carry = min(carry + __shfl(incl, G - 1, G), UX);
        if (carry >= UX) break;
      }
    }
  }
  finish_push<G>(g, ra, node, UX, carry, cand, gl, active);
}

template <int G>
__device__ void push_eout(const Dev& g, const RoundArgs& ra, int node, bool has, int gl,
                          uint32_t& nbytes, unsigned long long& to_sink) {
  const int e = (node - g.NB) >> 1;
  int k = 0, X = 0;
  if (has) {
    k = g.d[node];
    X = g.x[node];
  }
  const bool active = has && k < g.N && X > 0;
  const uint32_t UX = active ? (uint32_t)X : 0u;
  uint32_t carry = 0;
  int cand = kInf;
  if (active) {
    nbytes += 16;
    const int beg = g.net_off[e], end = g.net_off[e + 1];
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
        else atomicAdd(&g.x[u], (int)give);
      }
      mark_pushed(g, ra, u, give > 0u && du != 0);
      if (valid) cand = min(cand, du + 1);
      carry = min(carry + __shfl(incl, G - 1, G), UX);
      if (carry >= UX) break;
    }
    if (carry < UX) {  // reverse bridge e_out -> e_in
      const int rb = g.fb[e];
      const int din = g.d[node - 1];
      nbytes += 8;
      const bool ab = rb > 0 && din == k - 1;
      const uint32_t gb = ab ? min((uint32_t)rb, UX - carry) : 0u;
      if (gb && gl == 0) {
        g.fb[e] = rb - (int)gb;
        atomicAdd(&g.x[node - 1], (int)gb);
      }
      mark_pushed(g, ra, node - 1, gb > 0u && gl == 0);
      carry += gb;
      if ((uint32_t)rb > gb) cand = min(cand, din + 1);
    }
  }
  finish_push<G>(g, ra, node, UX, carry, cand, gl, active);
}

template <int G>
__device__ __forceinline__ void push_node(const Dev& g, const RoundArgs& ra, int v, bool has,
                                          int gl, uint32_t& nbytes,
                                          unsigned long long& to_sink) {
  // kind is wave-divergent only across groups; each branch is group-uniform
  if (!has || v < g.V) push_vertex<G>(g, ra, v, has, gl, nbytes);
  else if (((v - g.NB) & 1) == 0) push_ein<G>(g, ra, v, has, gl, nbytes);
  else push_eout<G>(g, ra, v, has, gl, nbytes, to_sink);
}

// Work items of a frontier: small nodes in groups of G lanes (64/G nodes per
// wave item), then big nodes one per wave item.
template <int G>
__device__ void phase_push(const Dev& g, int epoch, int w0, int wstride, int kc) {
  const RoundArgs ra = round_args(epoch);
  if (w0 == 0 && lane_id() == 0) {
    // ring slots no one reads in this round: next round's append targets
    g.ctl->fcnt[(epoch + 2) % 3][0] = 0;
    g.ctl->fcnt[(epoch + 2) % 3][1] = 0;
    g.ctl->lcnt[ra.nxt3] = 0;
  }
  const int ns = g.ctl->fcnt[ra.cur3][0];
  const int nb = g.ctl->fcnt[ra.cur3][1];
  const int cur = epoch & 1;
  const int32_t* ls = g.list[cur][0];
  const int32_t* lb = g.list[cur][1];
  constexpr int NPW = kWave / G;
  const int nsi = (ns + NPW - 1) / NPW;
  const int total = nsi + nb;
  const int lane = lane_id();
  uint32_t nbytes = 0;
  uint32_t nitems = 0;
  unsigned long long to_sink = 0;
  for (int it = w0; it < total; it += wstride) {
    if (it < nsi) {
      const int idx = it * NPW + lane / G;
      const bool has = idx < ns;
      const int v = has ? ls[idx] : 0;
      nitems += has && (lane % G) == 0;
      push_node<G>(g, ra, v, has, lane % G, nbytes, to_sink);
    } else {
      const int v = lb[it - nsi];
      nitems += lane == 0;
      push_node<kWave>(g, ra, v, true, lane, nbytes, to_sink);
    }
  }
  wave_add_u64(&g.ctl->flow, to_sink);
  wave_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 4ull * nitems);
  wave_add_u64(&g.ctl->items[kc], nitems);
}

// Apply phase: relabel nodes left with excess; thread per entry.
__device__ void phase_apply(const Dev& g, int epoch, int t0, int tstride, int kc) {
  const RoundArgs ra = round_args(epoch);
  const int n = g.ctl->lcnt[ra.cur3];
  unsigned long long nrel = 0;
  uint32_t nbytes = 0;
  // t0 is wave-aligned and tstride a multiple of 64, so lanes of a wave run
  // the same iterations (needed by the ballots in push_frontier)
  for (int base = t0 - lane_id(); base < n; base += tstride) {
    const int i = base + lane_id();
    const bool has = i < n;
    int v = 0;
    bool app = false;
    if (has) {
      const int2 en = g.left[i];
      v = en.x;
      const int k = g.d[v];
      const bool rec = g.stamp[v] == ra.epoch;
      int nd = en.y;
      if (rec) nd = min(nd, k + 2);
      nd = min(nd, g.N);
      if (nd <= k) atomicOr(&g.ctl->err, ERR_LABEL);
      g.d[v] = nd;
      nrel += 1;
      nbytes += 20;
      app = !rec && nd < g.N;
    }
    push_frontier(g, g.ctl->fcnt[ra.nxt3], g.list[ra.nxtp][0], g.list[ra.nxtp][1], v, app);
  }
  wave_add_u64(&g.ctl->relabels, nrel);
  wave_add_u64(&g.ctl->bytes[kc], nbytes);
  wave_add_u64(&g.ctl->items[kc], nrel);
}

// ---------------------------------------------------------------------------
// reverse residual BFS from the sinks (global relabel) over the capped network
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool visit_rev(const Dev& g, int v, int lvl) {
  if (g.d[v] != g.N) return false;
  return atomicCAS(&g.d[v], g.N, lvl) == g.N;
}

template <int G>
__device__ void bfs_rev_node(const Dev& g, int x, bool has, int gl, int lvl, int32_t* cnt2,
                             int32_t* ls, int32_t* lb, uint32_t& nbytes) {
  // lvl = label to give to newly reached nodes
  const bool isv = has && x < g.V;
  const bool isnet = has && x >= g.NB;
  if (!has || isv) {
    int beg = 0, end = 0;
    if (isv) {
      beg = g.vtx_off[x];
      end = g.vtx_off[x + 1];
    }
    for (int base = beg; base < end; base += G) {
      const int i = base + gl;
      const bool valid = i < end;
      bool vin = false, vout = false;
      int e = 0;
      if (valid) {
        const int2 ep = g.vinc[i];
        e = ep.x;
        const int2 dl = *reinterpret_cast<const int2*>(g.d + g.NB + 2 * e);
        nbytes += 16;
        if (dl.y == g.N) vout = atomicCAS(&g.d[g.NB + 2 * e + 1], g.N, lvl) == g.N;
        if (dl.x == g.N) {
          const int rin = g.fpin[2 * ep.y];
          const int we = g.w[e];
          nbytes += 8;
          if (we - rin > 0) vin = atomicCAS(&g.d[g.NB + 2 * e], g.N, lvl) == g.N;
        }
      }
      push_frontier(g, cnt2, ls, lb, g.NB + 2 * e, vin);
      push_frontier(g, cnt2, ls, lb, g.NB + 2 * e + 1, vout);
    }
  } else if (isnet) {
    const int e = (x - g.NB) >> 1;
    const bool in = ((x - g.NB) & 1) == 0;
    const int beg = g.net_off[e], end = g.net_off[e + 1];
    const int we = g.w[e];
    const int fbv = g.fb[e];
    nbytes += 16;
    bool vb = false;
    if (gl == 0) {
      if (in) vb = fbv > 0 && visit_rev(g, x + 1, lvl);       // e_out -> e_in residual fb
      else vb = we - fbv > 0 && visit_rev(g, x - 1, lvl);     // e_in -> e_out residual w - fb
    }
    push_frontier(g, cnt2, ls, lb, in ? x + 1 : x - 1, vb);
    for (int base = beg; base < end; base += G) {
      const int i = base + gl;
      const bool valid = i < end;
      bool vu = false;
      int u = 0;
      if (valid) {
        u = g.pin_v[i];
        const int f = g.fpin[2 * i + (in ? 0 : 1)];  // r_in (u->e_in) or f_out (u->e_out)
        nbytes += 12;
        if (f > 0) vu = visit_rev(g, u, lvl);
      }
      push_frontier(g, cnt2, ls, lb, u, vu);
    }
  }
}

template <int G>
__device__ void phase_bfs_rev(const Dev& g, int level, int w0, int wstride, int kc) {
  // frontier of level `level` -> label level+1
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (w0 == 0 && lane_id() == 0) {
    g.ctl->bcnt[z3][0] = 0;
    g.ctl->bcnt[z3][1] = 0;
  }
  const int ns = g.ctl->bcnt[c3][0];
  const int nb = g.ctl->bcnt[c3][1];
  const int cp = level & 1, np = (level + 1) & 1;
  constexpr int NPW = kWave / G;
  const int nsi = (ns + NPW - 1) / NPW;
  const int total = nsi + nb;
  const int lane = lane_id();
  uint32_t nbytes = 0, nitems = 0;
  for (int it = w0; it < total; it += wstride) {
    if (it < nsi) {
      const int idx = it * NPW + lane / G;
      const bool has = idx < ns;
      const int v = has ? g.list[cp][0][idx] : 0;
      nitems += has && (lane % G) == 0;
      bfs_rev_node<G>(g, v, has, lane % G, level + 1, g.ctl->bcnt[n3], g.list[np][0],
                      g.list[np][1], nbytes);
    } else {
      const int v = g.list[cp][1][it - nsi];
      nitems += lane == 0;
      bfs_rev_node<kWave>(g, v, true, lane, level + 1, g.ctl->bcnt[n3], g.list[np][0],
                          g.list[np][1], nbytes);
    }
  }
  wave_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 4ull * nitems);
  wave_add_u64(&g.ctl->items[kc], nitems);
}

// ---------------------------------------------------------------------------
// forward residual BFS of the uncapped network (source-side cut)
// ---------------------------------------------------------------------------

template <int G>
__device__ void bfs_fwd_node(const Dev& g, int x, bool has, int gl, int ep, int32_t* cnt2,
                             int32_t* ls, int32_t* lb, uint32_t& nbytes) {
  const bool isv = has && x < g.V;
  const bool isnet = has && x >= g.NB;
  if (!has || isv) {
    int beg = 0, end = 0;
    if (isv) {
      beg = g.vtx_off[x];
      end = g.vtx_off[x + 1];
    }
    for (int base = beg; base < end; base += G) {
      const int i = base + gl;
      const bool valid = i < end;
      bool vin = false, vout = false;
      int e = 0;
      if (valid) {
        const int2 ep2 = g.vinc[i];
        e = ep2.x;
        nbytes += 12;
        vin = stamp_first(g, g.NB + 2 * e, ep);                    // u -> e_in (uncapped)
        if (g.fpin[2 * ep2.y + 1] > 0) vout = stamp_first(g, g.NB + 2 * e + 1, ep);
      }
      push_frontier(g, cnt2, ls, lb, g.NB + 2 * e, vin);
      push_frontier(g, cnt2, ls, lb, g.NB + 2 * e + 1, vout);
    }
  } else if (isnet) {
    const int e = (x - g.NB) >> 1;
    const bool in = ((x - g.NB) & 1) == 0;
    const int beg = g.net_off[e], end = g.net_off[e + 1];
    const int we = g.w[e];
    const int fbv = g.fb[e];
    nbytes += 16;
    bool vb = false;
    if (gl == 0) {
      if (in) vb = fbv < we && stamp_first(g, x + 1, ep);   // bridge residual
      else vb = fbv > 0 && stamp_first(g, x - 1, ep);       // reverse bridge
    }
    push_frontier(g, cnt2, ls, lb, in ? x + 1 : x - 1, vb);
    for (int base = beg; base < end; base += G) {
      const int i = base + gl;
      const bool valid = i < end;
      bool vu = false;
      int u = 0;
      if (valid) {
        u = g.pin_v[i];
        nbytes += 8;
        if (in) {
          const int rin = g.fpin[2 * i];
          if (we - rin > 0) vu = stamp_first(g, u, ep);       // e_in -> u reverse
        } else {
          const int r = g.role[u];
          if (r == 2) atomicOr(&g.ctl->err, ERR_SINK_REACHED);
          else if (r == 0) vu = stamp_first(g, u, ep);        // e_out -> u infinite
        }
      }
      push_frontier(g, cnt2, ls, lb, u, vu);
    }
  }
}

template <int G>
__device__ void phase_bfs_fwd(const Dev& g, int level, int ep, int w0, int wstride, int kc) {
  const int c3 = level % 3, n3 = (level + 1) % 3, z3 = (level + 2) % 3;
  if (w0 == 0 && lane_id() == 0) {
    g.ctl->bcnt[z3][0] = 0;
    g.ctl->bcnt[z3][1] = 0;
  }
  const int ns = g.ctl->bcnt[c3][0];
  const int nb = g.ctl->bcnt[c3][1];
  const int cp = level & 1, np = (level + 1) & 1;
  constexpr int NPW = kWave / G;
  const int nsi = (ns + NPW - 1) / NPW;
  const int total = nsi + nb;
  const int lane = lane_id();
  uint32_t nbytes = 0, nitems = 0;
  for (int it = w0; it < total; it += wstride) {
    if (it < nsi) {
      const int idx = it * NPW + lane / G;
      const bool has = idx < ns;
      const int v = has ? g.list[cp][0][idx] : 0;
      nitems += has && (lane % G) == 0;
      bfs_fwd_node<G>(g, v, has, lane % G, ep, g.ctl->bcnt[n3], g.list[np][0], g.list[np][1],
                      nbytes);
    } else {
      const int v = g.list[cp][1][it - nsi];
      nitems += lane == 0;
      bfs_fwd_node<kWave>(g, v, true, lane, ep, g.ctl->bcnt[n3], g.list[np][0],
                          g.list[np][1], nbytes);
    }
  }
  wave_add_u64(&g.ctl->bytes[kc], (unsigned long long)nbytes + 4ull * nitems);
  wave_add_u64(&g.ctl->items[kc], nitems);
}

// ---------------------------------------------------------------------------
// sweeps (thread per node); t0 wave-aligned, tstride a multiple of 64
// ---------------------------------------------------------------------------

// Zero flow, excess only at e_in of nets with a source pin (their contracted
// source arc saturated at w(e)), all counters cleared.
__device__ void phase_init(const Dev& g, int t0, int tstride) {
  if (t0 == 0) {
    Ctl* c = g.ctl;
    for (int i = 0; i < 3; ++i) {
      c->fcnt[i][0] = c->fcnt[i][1] = 0;
      c->bcnt[i][0] = c->bcnt[i][1] = 0;
      c->lcnt[i] = 0;
    }
    c->err = 0;
    c->flow = 0ull;
    c->relabels = 0ull;
    for (int i = 0; i < KC_N; ++i) c->bytes[i] = c->items[i] = 0ull;
  }
  const int n = max(g.P, g.N);
  for (int i = t0; i < n; i += tstride) {
    if (i < g.P) {
      const int2 ep = g.vinc[i];
      g.fpin[2 * ep.y] = g.w[ep.x];
      g.fpin[2 * ep.y + 1] = 0;
    }
    if (i < g.N) {
      g.stamp[i] = -1;
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
__device__ void phase_gr_reset(const Dev& g, int t0, int tstride) {
  if (t0 == 0) {
    Ctl* c = g.ctl;
    for (int i = 0; i < 3; ++i) {
      c->fcnt[i][0] = c->fcnt[i][1] = 0;
      c->lcnt[i] = 0;
    }
  }
  for (int base = t0 - lane_id(); base < g.N; base += tstride) {
    const int v = base + lane_id();
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
    }
    push_frontier(g, g.ctl->bcnt[0], g.list[0][0], g.list[0][1], v, seed);
  }
}

// Global relabel, step 3: frontier = non-terminal nodes with excess and a
// label below N.  BFS counters are cleared for the next BFS.
__device__ void phase_gather(const Dev& g, int epoch, int t0, int tstride) {
  const int c3 = epoch % 3, cp = epoch & 1;
  if (t0 == 0) {
    for (int i = 0; i < 3; ++i) g.ctl->bcnt[i][0] = g.ctl->bcnt[i][1] = 0;
  }
  for (int base = t0 - lane_id(); base < g.N; base += tstride) {
    const int v = base + lane_id();
    bool act = false;
    if (v < g.N && (v >= g.NB || (v < g.V && g.role[v] == 0)))
      act = g.x[v] > 0 && g.d[v] < g.N;
    push_frontier(g, g.ctl->fcnt[c3], g.list[cp][0], g.list[cp][1], v, act);
  }
}

// Cut BFS seeds: sources (marked, nothing to expand: their only arcs are the
// contracted source arcs into e_in), e_in of nets with a source pin, and
// every non-terminal node holding excess.
__device__ void phase_cut_seed(const Dev& g, int ep, int t0, int tstride) {
  for (int base = t0 - lane_id(); base < g.N; base += tstride) {
    const int v = base + lane_id();
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
      if (seed) g.stamp[v] = ep;
    }
    push_frontier(g, g.ctl->bcnt[0], g.list[0][0], g.list[0][1], v, seed);
  }
}

// Write the side bitmaps and clear BFS counters.
__device__ void phase_cut_out(const Dev& g, int ep, uint8_t* vside, uint8_t* nside, int t0,
                              int tstride) {
  if (t0 == 0) {
    for (int i = 0; i < 3; ++i) g.ctl->bcnt[i][0] = g.ctl->bcnt[i][1] = 0;
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

// Debug: preflow feasibility and label validity on every residual arc of the
// capped network.  Thread per pin / net / vertex.
__device__ void phase_check(const Dev& g, int t0, int tstride) {
  const int n = max(g.P, max(g.E, g.V));
  bool bad = false;
  for (int i = t0; i < n; i += tstride) {
    if (i < g.V) {
      const int r = g.role[i];
      const int xv = g.x[i];
      if (r == 0 && xv < 0) bad = true;
      if (r == 0) {
        // excess equals inflow - outflow
        long long s = 0;
        for (int j = g.vtx_off[i]; j < g.vtx_off[i + 1]; ++j) {
          const int2 ep = g.vinc[j];
          s += (long long)g.fpin[2 * ep.y + 1] - (long long)(g.w[ep.x] - g.fpin[2 * ep.y]);
        }
        if (s != xv) bad = true;
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
      if (sin - fbv != g.x[g.NB + 2 * i]) bad = true;
      if (fbv - sout != g.x[g.NB + 2 * i + 1]) bad = true;
      if (g.x[g.NB + 2 * i] < 0 || g.x[g.NB + 2 * i + 1] < 0) bad = true;
      const int din = g.d[g.NB + 2 * i], dout = g.d[g.NB + 2 * i + 1];
      if (din < g.N && fbv < we && din > dout + 1) bad = true;
      if (dout < g.N && fbv > 0 && dout > din + 1) bad = true;
    }
    if (i < g.P) {
      // pin arcs: find the net by the vertex side entry (pins are scanned
      // through vinc for the net id)
      const int2 ep = g.vinc[i];
      const int e = ep.x, p = ep.y;
      const int u = g.pin_v[p];
      const int rin = g.fpin[2 * p], fout = g.fpin[2 * p + 1];
      const int we = g.w[e];
      if (rin < 0 || rin > we || fout < 0) bad = true;
      const int r = g.role[u];
      if (r != 0 && rin != we) bad = true;  // no flow leaves a terminal
      if (r == 1 && fout != 0) bad = true;  // nothing enters a source
      const int du = g.d[u], din = g.d[g.NB + 2 * e], dout = g.d[g.NB + 2 * e + 1];
      if (r == 0) {
        if (du < g.N && rin > 0 && du > din + 1) bad = true;        // u -> e_in
        if (du < g.N && fout > 0 && du > dout + 1) bad = true;      // u -> e_out
        if (din < g.N && we - rin > 0 && din > du + 1) bad = true;  // e_in -> u
      }
      if (dout < g.N && r != 1 && dout > du + 1) bad = true;        // e_out -> u
    }
  }
  if (bad) atomicOr(&g.ctl->err, ERR_INVARIANT);
}

}  // namespace hf
