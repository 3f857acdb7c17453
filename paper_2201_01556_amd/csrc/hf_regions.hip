// Flow problems of block pairs built on the device (paper, section "Network
// Construction": paragraphs "Region Growing", "Construction Algorithms" and
// "Identical Net Removal").
//
// For each pair (i, j) of blocks of a k-way partition two breadth-first
// searches grow B_i inside block i and B_j inside block j from the blocks'
// pins on the nets cut between them; the flow problem keeps the nets with a
// region pin, contracts the rest of block i into a source s and the rest of
// block j into a sink t, drops the pins of other blocks, discards nets left
// with fewer than two pins or with both s and t, and optionally merges nets
// with equal pin sets.  Readings, in the terms of the pair's caps (inputs):
// a search visits each level in increasing vertex id and adds vertices while
// the side's weight stays within its cap and one vertex of the block stays
// outside; it stops for good at the first vertex that does not fit; region
// vertices get local ids in increasing global id (s = n, t = n + 1); nets
// keep increasing global id and list their pins in increasing local id; a
// merged group is represented by its smallest net id.
//
// Device layout of the work (all pairs at once):
//   hypergraph: net CSR, pin -> net, vertex -> nets (radix sort of the pins by
//     vertex), vertices by block (radix sort by block id; a vertex's
//     position in its block is its block-local id), per net the mask of the
//     blocks holding a pin (k <= 64);
//   per pair side (one workgroup each): bitmaps over the block's local ids
//     (visited, next level, added), the level list, a bitmap over the nets
//     (expanded by this side; afterwards the nets touched by the pair);
//   outputs: per pair CSR with relative offsets, weights, vertex weights,
//     global ids of vertices and nets, facts.
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <memory>
#include <new>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "hf_host.h"

namespace {

constexpr int kRegBlock = 1024;
constexpr int kInfoLen = 16;

enum : int {
  RERR_OFFSETS = 1,
  RERR_PINS = 2,
  RERR_WEIGHTS = 4,
  RERR_VWEIGHTS = 8,
  RERR_BLOCKS = 16,
};

}  // namespace

namespace hf {

// ---------------------------------------------------------------------------
// workgroup helpers (blockDim = kRegBlock)
// ---------------------------------------------------------------------------

// Inclusive prefix sum of one value per thread over the workgroup; *total
// receives the workgroup's sum.  Block-uniform.
__device__ long long rg_scan_i64(long long v, long long* total) {
  __shared__ long long wsum[kRegBlock / 64 + 1];
  const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == 63) wsum[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int i = 0; i < nw; ++i) {
      const long long t = wsum[i];
      wsum[i] = run;
      run += t;
    }
    wsum[nw] = run;
  }
  __syncthreads();
  const long long r = v + wsum[wid];
  *total = wsum[nw];
  __syncthreads();
  return r;
}

// Lists the set bits of bits[0..words) in increasing order into out and
// clears them (when clear); returns the count.  Block-uniform.
__device__ int rg_compact_bits(uint32_t* bits, int words, int32_t* out, bool clear) {
  int base = 0;
  for (int w0 = 0; w0 < words; w0 += blockDim.x) {
    const int wi = w0 + (int)threadIdx.x;
    uint32_t m = wi < words ? bits[wi] : 0u;
    if (clear && wi < words && m) bits[wi] = 0u;
    long long tot = 0;
    const int pos = (int)rg_scan_i64(__popc(m), &tot) - __popc(m);
    int k = base + pos;
    while (m) {
      const int b = __builtin_ctz(m);
      m &= m - 1u;
      out[k++] = (wi << 5) + b;
    }
    base += (int)tot;
  }
  __syncthreads();
  return base;
}

// ---------------------------------------------------------------------------
// hypergraph preparation
// ---------------------------------------------------------------------------

__global__ void k_rg_check_nets(int E, const int32_t* off, const int32_t* w, int* err) {
  int e_ = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
    if (off[e + 1] < off[e]) e_ |= RERR_OFFSETS;
    if (w[e] < 1) e_ |= RERR_WEIGHTS;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && off[0] != 0) e_ |= RERR_OFFSETS;
  if (e_) atomicOr(err, e_);
}

__global__ void k_rg_check_rest(int V, int P, int k, const int32_t* pins, const int32_t* cv,
                                const int32_t* block, int* err) {
  int e_ = 0;
  const int stride = gridDim.x * blockDim.x;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int p = t0; p < P; p += stride)
    if (pins[p] < 0 || pins[p] >= V) e_ |= RERR_PINS;
  for (int v = t0; v < V; v += stride) {
    if (cv[v] < 1) e_ |= RERR_VWEIGHTS;
    if (block[v] < 0 || block[v] >= k) e_ |= RERR_BLOCKS;
  }
  if (e_) atomicOr(err, e_);
}

__global__ void k_rg_pin_net(int E, const int32_t* off, int32_t* pin_net) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x)
    for (int p = off[e]; p < off[e + 1]; ++p) pin_net[p] = e;
}

// off[x] = first sorted position holding a key >= x, for x in [0, n]
__global__ void k_rg_offsets(const int32_t* keys, int count, int n, int32_t* offs) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= count; i += gridDim.x * blockDim.x) {
    const int prev = i == 0 ? -1 : keys[i - 1];
    const int cur = i == count ? n : keys[i];
    for (int x = prev + 1; x <= cur; ++x) offs[x] = i;
  }
}

__global__ void k_rg_local(int V, const int32_t* bverts, const int32_t* bkeys,
                           const int32_t* boff, int32_t* blocal) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < V; i += gridDim.x * blockDim.x)
    blocal[bverts[i]] = i - boff[bkeys[i]];
}

__global__ void k_rg_masks(int E, const int32_t* off, const int32_t* pins, const int32_t* block,
                           unsigned long long* mask) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
    unsigned long long m = 0ull;
    for (int p = off[e]; p < off[e + 1]; ++p) m |= 1ull << block[pins[p]];
    mask[e] = m;
  }
}

__global__ void k_rg_zero(uint32_t* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// region growing: one workgroup per pair side
// ---------------------------------------------------------------------------

struct RgGraph {
  int V, E;
  const int32_t* off;     // net CSR
  const int32_t* pins;
  const int32_t* w;
  const int32_t* cv;      // vertex weights
  const int32_t* block;
  const int32_t* voff;    // vertex -> nets
  const int32_t* vnet;
  const int32_t* bverts;  // vertices by block, increasing id
  const int32_t* boff;
  const int32_t* blocal;
  const unsigned long long* mask;
};

struct RgSide {
  // per pair side s = 2 q + (0: block i, 1: block j)
  const int32_t* pairs;       // 2 per pair
  const long long* caps;      // 2 per pair
  const long long* bits_at;   // word offset of side s's three block bitmaps
  const long long* lev_at;    // int offset of side s's level list / local-id map
  uint32_t* bits;
  int32_t* lev;
  uint32_t* xmark;            // per side (E + 31) / 32 words
  long long xwords;
  long long* out;             // per side: weight, count, boundary, c(block)
};

__global__ void __launch_bounds__(kRegBlock) k_rg_grow(RgGraph g, RgSide r) {
  const int s = blockIdx.x, q = s >> 1, side = s & 1;
  const int blk = r.pairs[2 * q + side], oth = r.pairs[2 * q + 1 - side];
  const long long cap_w = r.caps[2 * q + side];
  const int nb = g.boff[blk + 1] - g.boff[blk];
  const long long cap_n = (long long)nb - 1;
  const int32_t* bv = g.bverts + g.boff[blk];
  const int words = (nb + 31) >> 5;
  uint32_t* vis = r.bits + r.bits_at[s];
  uint32_t* nq = vis + words;
  uint32_t* added = nq + words;
  int32_t* lev = r.lev + r.lev_at[s];
  uint32_t* xm = r.xmark + (long long)s * r.xwords;
  const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;

  // block weight; level 0: the block's vertices on a net with a pin in the
  // other block of the pair (every net of a block vertex has a pin in the
  // block), i.e. its pins on the nets cut between the two blocks
  long long bw = 0;
  for (int l = threadIdx.x; l < nb; l += blockDim.x) {
    const int u = bv[l];
    bw += g.cv[u];
    for (int a = g.voff[u]; a < g.voff[u + 1]; ++a)
      if ((g.mask[g.vnet[a]] >> oth) & 1ull) {
        atomicOr(&vis[l >> 5], 1u << (l & 31));
        atomicOr(&nq[l >> 5], 1u << (l & 31));
        break;
      }
  }
  long long bw_tot = 0;
  rg_scan_i64(bw, &bw_tot);
  long long wsum = 0, cnt = 0, boundary = -1;
  while (true) {
    const int L = rg_compact_bits(nq, words, lev, true);
    if (boundary < 0) boundary = L;
    if (L == 0) break;
    // add the level's vertices in increasing id while they fit; weights are
    // positive, so those that fit in a chunk form its prefix
    bool stop = false;
    for (int b0 = 0; b0 < L; b0 += blockDim.x) {
      const int i = b0 + (int)threadIdx.x;
      const int chunk = min((int)blockDim.x, L - b0);
      const long long c = i < L ? (long long)g.cv[bv[lev[i]]] : 0ll;
      long long tot = 0;
      const long long pre = rg_scan_i64(c, &tot);
      const bool fits = i < L && wsum + pre <= cap_w && cnt + (i - b0) + 1 <= cap_n;
      long long wfit = 0, nfit = 0;
      rg_scan_i64(fits ? c : 0ll, &wfit);
      rg_scan_i64(fits ? 1ll : 0ll, &nfit);
      if (fits) atomicOr(&added[lev[i] >> 5], 1u << (lev[i] & 31));
      wsum += wfit;
      cnt += nfit;
      if (nfit < chunk) {
        stop = true;
        break;
      }
    }
    if (stop) break;  // the growth ends at the first vertex that does not fit
    __syncthreads();
    // next level: a wave per added vertex, its lanes over the pins of each of
    // its nets that this side has not expanded yet
    for (int a = wid; a < L; a += nw) {
      const int u = bv[lev[a]];
      for (int x = g.voff[u]; x < g.voff[u + 1]; ++x) {
        const int e = g.vnet[x];
        uint32_t old = 0;
        if (lane == 0) old = atomicOr(&xm[e >> 5], 1u << (e & 31));
        old = __shfl(old, 0);
        if (old & (1u << (e & 31))) continue;
        for (int p = g.off[e] + lane; p < g.off[e + 1]; p += 64) {
          const int y = g.pins[p];
          if (g.block[y] != blk) continue;
          const int l = g.blocal[y];
          const uint32_t bit = 1u << (l & 31);
          if (!(__atomic_load_n(&vis[l >> 5], __ATOMIC_RELAXED) & bit)) {
            const uint32_t o = atomicOr(&vis[l >> 5], bit);
            if (!(o & bit)) atomicOr(&nq[l >> 5], bit);
          }
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    r.out[4 * s + 0] = wsum;
    r.out[4 * s + 1] = cnt;
    r.out[4 * s + 2] = boundary;
    r.out[4 * s + 3] = bw_tot;
  }
}

// ---------------------------------------------------------------------------
// members, local ids and the nets a pair touches: one workgroup per pair
// ---------------------------------------------------------------------------

struct RgOut {
  const long long* vbase;     // per pair: first member slot (vgid), vw starts at vbase + 2 q
  int32_t* vgid;
  int8_t* vside;              // per member: 0 = from block i, 1 = from block j
  int32_t* vw;
  int32_t* terms;
  int32_t* lmap;              // per side, indexed like lev: local id of an added vertex
  long long* ntouch;          // per pair
};

__device__ __forceinline__ int rg_lower_bound(const int32_t* lst, const int32_t* bv, int n,
                                              int gid) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bv[lst[mid]] < gid) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kRegBlock) k_rg_members(RgGraph g, RgSide r, RgOut o) {
  const int q = blockIdx.x;
  int n[2];
  const int32_t* bvs[2];
  int32_t* lst[2];
  int32_t* lm[2];
  for (int side = 0; side < 2; ++side) {
    const int s = 2 * q + side;
    const int blk = r.pairs[s];
    const int nb = g.boff[blk + 1] - g.boff[blk];
    const int words = (nb + 31) >> 5;
    uint32_t* added = r.bits + r.bits_at[s] + 2ll * words;
    lst[side] = r.lev + r.lev_at[s];
    lm[side] = o.lmap + r.lev_at[s];
    bvs[side] = g.bverts + g.boff[blk];
    n[side] = rg_compact_bits(added, words, lst[side], false);
  }
  const long long vb = o.vbase[q];
  const int nn = n[0] + n[1];
  for (int side = 0; side < 2; ++side) {
    for (int a = threadIdx.x; a < n[side]; a += blockDim.x) {
      const int l = lst[side][a];
      const int gid = bvs[side][l];
      const int rank = a + rg_lower_bound(lst[1 - side], bvs[1 - side], n[1 - side], gid);
      lm[side][l] = rank;
      o.vgid[vb + rank] = gid;
      o.vside[vb + rank] = (int8_t)side;
      o.vw[vb + 2ll * q + rank] = g.cv[gid];
    }
  }
  if (threadIdx.x < 2) {
    const int s = 2 * q + (int)threadIdx.x;
    o.vw[vb + 2ll * q + nn + threadIdx.x] = (int32_t)(r.out[4 * s + 3] - r.out[4 * s + 0]);
    o.terms[2 * q + threadIdx.x] = nn + (int)threadIdx.x;
  }
  // the nets the pair touches: side 0's net bitmap is cleared and refilled
  uint32_t* eb = r.xmark + (long long)(2 * q) * r.xwords;
  for (long long w = threadIdx.x; w < r.xwords; w += blockDim.x) eb[w] = 0u;
  __syncthreads();
  for (int side = 0; side < 2; ++side)
    for (int a = threadIdx.x; a < n[side]; a += blockDim.x) {
      const int u = bvs[side][lst[side][a]];
      for (int x = g.voff[u]; x < g.voff[u + 1]; ++x) {
        const int e = g.vnet[x];
        atomicOr(&eb[e >> 5], 1u << (e & 31));
      }
    }
  __syncthreads();
  long long c = 0;
  for (long long w = threadIdx.x; w < r.xwords; w += blockDim.x) c += __popc(eb[w]);
  long long tot = 0;
  rg_scan_i64(c, &tot);
  if (threadIdx.x == 0) o.ntouch[q] = tot;
}

__global__ void __launch_bounds__(kRegBlock) k_rg_touch_list(RgSide r, const long long* tbase,
                                                             int32_t* tnet, int32_t* tpair) {
  const int q = blockIdx.x;
  uint32_t* eb = r.xmark + (long long)(2 * q) * r.xwords;
  const long long b = tbase[q];
  const int cnt = rg_compact_bits(eb, (int)r.xwords, tnet + b, false);
  for (int a = threadIdx.x; a < cnt; a += blockDim.x) tpair[b + a] = q;
}

// ---------------------------------------------------------------------------
// construction: thread per touched net
// ---------------------------------------------------------------------------

struct RgNets {
  int32_t nt;                 // touched nets (all pairs)
  const int32_t* tnet;
  const int32_t* tpair;
  int32_t* keep;              // 0/1
  long long* osz;             // output size (0 when dropped)
  unsigned long long* cutb;   // per pair
};

// Pin y of a net touched by pair q: 0 = another block (dropped), 1 = region
// vertex (*lid set), 2 = block i outside the region (s), 3 = block j outside
// (t).
__device__ __forceinline__ int rg_classify(const RgGraph& g, const RgSide& r, const int32_t* lmap,
                                           int q, int y, int* lid, bool* in_i) {
  const int b = g.block[y];
  const int i = r.pairs[2 * q], j = r.pairs[2 * q + 1];
  if (b != i && b != j) return 0;
  const int side = b == i ? 0 : 1;
  const int s = 2 * q + side;
  const int nb = g.boff[b + 1] - g.boff[b];
  const int words = (nb + 31) >> 5;
  const uint32_t* added = r.bits + r.bits_at[s] + 2ll * words;
  const int l = g.blocal[y];
  *in_i = side == 0;
  if ((added[l >> 5] >> (l & 31)) & 1u) {
    *lid = lmap[r.lev_at[s] + l];
    return 1;
  }
  return side == 0 ? 2 : 3;
}

struct RgKept {
  const int32_t* kidx;        // exclusive scan of keep
  const long long* opos;      // exclusive scan of osz
  const long long* nloc;      // per pair n (members)
  long long* koff;            // nk + 1 pin offsets
  int32_t* kpins;             // local ids
  int32_t* kpair;
  int32_t* kgid;
  long long* kw;              // weights (summed over merged groups)
  int* unsorted;
};

// Flat versions of the two passes: a wave takes 64 touched nets and spreads
// their pins evenly over its lanes (prefix sum of the sizes, each lane finds
// its pin's net by binary search), so a 2,000-pin net does not hold 63 idle
// lanes; per-net tallies live in LDS slots of the wave (64 per wave).
constexpr int kFlatBlock = 256;

struct RgWaveItem {
  int k, e, q, deg, excl, A;
};

__device__ __forceinline__ RgWaveItem rg_wave_item(const RgGraph& g, const RgNets& t, int base) {
  RgWaveItem it;
  const int lane = __lane_id();
  it.k = base + lane;
  it.e = it.k < t.nt ? t.tnet[it.k] : 0;
  it.q = it.k < t.nt ? t.tpair[it.k] : 0;
  it.deg = it.k < t.nt ? g.off[it.e + 1] - g.off[it.e] : 0;
  int incl = it.deg;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  it.excl = incl - it.deg;
  it.A = __shfl(incl, 63);
  return it;
}

__device__ __forceinline__ int rg_owner(int excl, int a) {
  int lo = 0;
#pragma unroll
  for (int st = 32; st > 0; st >>= 1) {
    const int c = lo + st;
    if (__shfl(excl, c) <= a) lo = c;
  }
  return lo;
}

__global__ void __launch_bounds__(kFlatBlock) k_rg_count_flat(RgGraph g, RgSide r,
                                                              const int32_t* lmap, RgNets t) {
  __shared__ int cnt_s[kFlatBlock], flg_s[kFlatBlock];
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  int* cnt = cnt_s + wid * 64;
  int* flg = flg_s + wid * 64;
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  for (int base = (blockIdx.x * (blockDim.x >> 6) + wid) * 64; base < t.nt; base += nwaves * 64) {
    const RgWaveItem it = rg_wave_item(g, t, base);
    cnt[lane] = 0;
    flg[lane] = 0;
    for (int a0 = 0; a0 < it.A; a0 += 64) {
      const int a = a0 + lane;
      const int lo = rg_owner(it.excl, a);
      const int eo = __shfl(it.e, lo), qo = __shfl(it.q, lo), xo = __shfl(it.excl, lo);
      if (a < it.A) {
        int lid = 0;
        bool si = false;
        const int c = rg_classify(g, r, lmap, qo, g.pins[g.off[eo] + (a - xo)], &lid, &si);
        if (c == 1) {
          atomicAdd(&cnt[lo], 1);
          atomicOr(&flg[lo], si ? 4 : 8);
        } else if (c == 2) {
          atomicOr(&flg[lo], 1);
        } else if (c == 3) {
          atomicOr(&flg[lo], 2);
        }
      }
    }
    bool keep = false, cut = false;
    if (it.k < t.nt) {
      const int f = flg[lane];
      const bool has_s = f & 1, has_t = f & 2;
      const int size = cnt[lane] + (int)has_s + (int)has_t;
      keep = size >= 2 && !(has_s && has_t);
      t.keep[it.k] = keep ? 1 : 0;
      t.osz[it.k] = keep ? size : 0;
      cut = keep && ((f & 4) || has_s) && ((f & 8) || has_t);
    }
    // cut weights per pair: one atomic per run of lanes of the same pair
    unsigned long long w = cut ? (unsigned long long)g.w[it.e] : 0ull;
    unsigned long long left = __ballot(cut);
    while (left) {
      const int lead = __builtin_ctzll(left);
      const int q0 = __shfl(it.q, lead);
      const bool mine = cut && it.q == q0;
      unsigned long long v = mine ? w : 0ull;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == lead) atomicAdd(&t.cutb[q0], v);
      left &= ~__ballot(mine);
    }
  }
}

__global__ void __launch_bounds__(kFlatBlock) k_rg_write_flat(RgGraph g, RgSide r,
                                                              const int32_t* lmap, RgNets t,
                                                              RgKept o) {
  __shared__ int cnt_s[kFlatBlock], flg_s[kFlatBlock];
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  int* cnt = cnt_s + wid * 64;
  int* flg = flg_s + wid * 64;
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int base = (blockIdx.x * (blockDim.x >> 6) + wid) * 64; base < t.nt; base += nwaves * 64) {
    const RgWaveItem it = rg_wave_item(g, t, base);
    const int keep = it.k < t.nt ? t.keep[it.k] : 0;
    const long long pos0 = keep ? o.opos[it.k] : 0;
    cnt[lane] = 0;
    flg[lane] = 0;
    for (int a0 = 0; a0 < it.A; a0 += 64) {
      const int a = a0 + lane;
      const int lo = rg_owner(it.excl, a);
      const int eo = __shfl(it.e, lo), qo = __shfl(it.q, lo), xo = __shfl(it.excl, lo);
      const int ko = __shfl(keep, lo);
      const long long po = __shfl(pos0, lo);
      int lid = 0, c = 0;
      bool si = false;
      if (a < it.A && ko) c = rg_classify(g, r, lmap, qo, g.pins[g.off[eo] + (a - xo)], &lid, &si);
      // rank of a region pin among its net's region pins: those in earlier
      // steps (cnt) plus the lanes before it in this step (lanes of one net
      // are contiguous, starting at max(0, xo - a0))
      const unsigned long long reg = __ballot(c == 1);
      const int first = max(0, xo - a0);
      const unsigned long long from = first >= 64 ? 0ull : ~((1ull << first) - 1ull);
      const int before = cnt[lo];
      if (c == 1) o.kpins[po + before + __popcll(reg & lt & from)] = lid;
      if (c == 1) atomicAdd(&cnt[lo], 1);
      if (c == 2) atomicOr(&flg[lo], 1);
      if (c == 3) atomicOr(&flg[lo], 2);
    }
    if (keep) {
      const int K = o.kidx[it.k];
      long long p = pos0 + cnt[lane];
      const int n = (int)o.nloc[it.q];
      if (flg[lane] & 1) o.kpins[p++] = n;
      if (flg[lane] & 2) o.kpins[p++] = n + 1;
      o.koff[K] = pos0;
      o.kpair[K] = it.q;
      o.kgid[K] = it.e;
      o.kw[K] = g.w[it.e];
    }
  }
}

// kept nets per pair, from the scan of the keep flags at the pairs' bounds
__global__ void k_rg_kept_per_pair(int npairs, const long long* tbase, int nt,
                                   const int32_t* kidx, unsigned long long* kcount) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npairs; q += gridDim.x * blockDim.x) {
    const long long end = q + 1 < npairs ? tbase[q + 1] : nt;
    kcount[q] = (unsigned long long)(kidx[end] - kidx[tbase[q]]);
  }
}

// kept nets whose region pins are out of increasing local id
__global__ void k_rg_check_sorted(long long nk, const long long* koff, const int32_t* kpins,
                                  int* unsorted) {
  int bad = 0;
  for (long long K = blockIdx.x * (long long)blockDim.x + threadIdx.x; K < nk;
       K += (long long)gridDim.x * blockDim.x)
    for (long long p = koff[K] + 1; p < koff[K + 1]; ++p)
      if (kpins[p] < kpins[p - 1]) bad = 1;
  if (bad) atomicOr(unsorted, 1);
}

// sort keys (net << 32 | local id) of the kept nets' pins, and back
__global__ void k_rg_sort_keys(long long nk, const long long* koff, const int32_t* kpins,
                               unsigned long long* keys) {
  for (long long K = blockIdx.x * (long long)blockDim.x + threadIdx.x; K < nk;
       K += (long long)gridDim.x * blockDim.x)
    for (long long p = koff[K]; p < koff[K + 1]; ++p)
      keys[p] = ((unsigned long long)K << 32) | (uint32_t)kpins[p];
}

__global__ void k_rg_sort_back(long long np, const unsigned long long* keys, int32_t* kpins) {
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np;
       p += (long long)gridDim.x * blockDim.x)
    kpins[p] = (int32_t)(keys[p] & 0xffffffffull);
}

// ---------------------------------------------------------------------------
// identical nets (paragraph "Identical Net Removal"): fingerprints
// sum (v + 1)^2 with the size and the pair hashed into one key, a stable
// sort of the nets by key, then an exact comparison inside each run of
// equal keys: a net equal to an earlier one of its run is merged into the
// first such net (the smallest id of the group, since the sort is stable)
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long rg_mix(unsigned long long x) {
  // the finalizer of splitmix64 (a published bijective mixing function)
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__global__ void k_rg_fingerprint(long long nk, const long long* koff, const int32_t* kpins,
                                 const int32_t* kpair, unsigned long long* key, int32_t* val) {
  for (long long K = blockIdx.x * (long long)blockDim.x + threadIdx.x; K < nk;
       K += (long long)gridDim.x * blockDim.x) {
    unsigned long long f = 0ull;
    for (long long p = koff[K]; p < koff[K + 1]; ++p) {
      const unsigned long long v = (unsigned long long)kpins[p] + 1ull;
      f += v * v;
    }
    const unsigned long long size = (unsigned long long)(koff[K + 1] - koff[K]);
    key[K] = rg_mix(rg_mix(f) ^ rg_mix((size << 32) | (uint32_t)kpair[K]));
    val[K] = (int32_t)K;
  }
}

__global__ void k_rg_run_heads(long long nk, const unsigned long long* key, int32_t* head) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nk;
       i += (long long)gridDim.x * blockDim.x)
    head[i] = (i == 0 || key[i] != key[i - 1]) ? (int32_t)i : 0;
}

__device__ __forceinline__ bool rg_same(const long long* koff, const int32_t* kpins,
                                        const int32_t* kpair, int a, int b) {
  if (kpair[a] != kpair[b]) return false;
  const long long la = koff[a + 1] - koff[a];
  if (la != koff[b + 1] - koff[b]) return false;
  for (long long t = 0; t < la; ++t)
    if (kpins[koff[a] + t] != kpins[koff[b] + t]) return false;
  return true;
}

__global__ void k_rg_dups(long long nk, const int32_t* val, const int32_t* run,
                          const long long* koff, const int32_t* kpins, const int32_t* kpair,
                          const long long* w0, long long* kw, int32_t* dead) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nk;
       i += (long long)gridDim.x * blockDim.x) {
    const int K = val[i];
    for (long long r = run[i]; r < i; ++r) {
      const int R = val[r];
      if (rg_same(koff, kpins, kpair, R, K)) {
        dead[K] = 1;
        atomicAdd(reinterpret_cast<unsigned long long*>(&kw[R]), (unsigned long long)w0[K]);
        break;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// final output: thread per kept net
// ---------------------------------------------------------------------------

struct RgFinal {
  const int32_t* dead;        // or NULL
  const long long* fidx;      // exclusive scan of alive
  const long long* fpos;      // exclusive scan of alive sizes
  const long long* nbase;     // per pair: first final net
  const long long* pbase;     // per pair: first final pin
  int32_t* off;
  int32_t* pins;
  int32_t* w;
  int32_t* ngid;
  unsigned long long* bins;   // 7 per pair
  int* err;
};

__global__ void k_rg_alive_sizes(long long nk, const long long* koff, const int32_t* dead,
                                 long long* alive, long long* asz, const int32_t* kpair,
                                 unsigned long long* ne, unsigned long long* np) {
  for (long long K = blockIdx.x * (long long)blockDim.x + threadIdx.x; K < nk;
       K += (long long)gridDim.x * blockDim.x) {
    const bool a = dead == nullptr || !dead[K];
    const long long sz = koff[K + 1] - koff[K];
    alive[K] = a ? 1 : 0;
    asz[K] = a ? sz : 0;
    if (a) {
      atomicAdd(&ne[kpair[K]], 1ull);
      atomicAdd(&np[kpair[K]], (unsigned long long)sz);
    }
  }
}

__global__ void k_rg_final(long long nk, const long long* koff, const int32_t* kpins,
                           const int32_t* kpair, const int32_t* kgid, const long long* kw,
                           RgFinal f) {
  int bad = 0;
  for (long long K = blockIdx.x * (long long)blockDim.x + threadIdx.x; K < nk;
       K += (long long)gridDim.x * blockDim.x) {
    if (f.dead && f.dead[K]) continue;
    const int q = kpair[K];
    const long long F = f.fidx[K];
    const long long pos = f.fpos[K];
    const long long sz = koff[K + 1] - koff[K];
    f.off[F + q] = (int32_t)(pos - f.pbase[q]);
    for (long long t = 0; t < sz; ++t) f.pins[pos + t] = kpins[koff[K] + t];
    if (kw[K] > 0x7fffffffll) bad = 1;
    f.w[F] = (int32_t)kw[K];
    f.ngid[F] = kgid[K];
    const int bin = sz <= 2 ? 0 : sz <= 4 ? 1 : sz <= 8 ? 2 : sz <= 16 ? 3 : sz <= 64 ? 4
                  : sz <= 256 ? 5 : 6;
    atomicAdd(&f.bins[7 * q + bin], 1ull);
  }
  if (bad) atomicOr(f.err, 1);
}

__global__ void k_rg_last_offsets(int npairs, const long long* nbase, const long long* pbase,
                                  const unsigned long long* ne, const unsigned long long* np,
                                  int32_t* off) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npairs; q += gridDim.x * blockDim.x) {
    off[nbase[q] + q + (long long)ne[q]] = (int32_t)np[q];
  }
}

}  // namespace hf

// ---------------------------------------------------------------------------
// the kept pairs' problems as one disjoint-union network, straight from the
// regions' arrays: kept pair i (pair ids[i]) owns union vertices
// [voff[i], voff[i+1]) (its n region vertices, then s and t), nets
// [eoff[i], eoff[i+1]) and pins [poff[i], poff[i+1])
// ---------------------------------------------------------------------------

namespace hf {

struct RgUnion {
  int32_t n;
  const int32_t* ids;
  const int32_t* voff;
  const int32_t* eoff;
  const int32_t* poff;
  const long long* nbase;  // per pair (all pairs): first net / pin / vertex in the regions
  const long long* pbase;
  const long long* vbase;
};

__device__ __forceinline__ int rg_part(const int32_t* off, int n, int x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_ru_nets(RgUnion m, const int32_t* off, const int32_t* w, int32_t E,
                          int32_t* off_u, int32_t* w_u) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t <= E; t += gridDim.x * blockDim.x) {
    if (t == E) {
      off_u[E] = m.poff[m.n];
      continue;
    }
    const int i = rg_part(m.eoff, m.n, t);
    const int q = m.ids[i];
    const int r = t - m.eoff[i];
    off_u[t] = m.poff[i] + off[m.nbase[q] + q + r];
    w_u[t] = w[m.nbase[q] + r];
  }
}

__global__ void k_ru_pins(RgUnion m, const int32_t* pins, int32_t P, int32_t* pins_u) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
    const int i = rg_part(m.poff, m.n, p);
    const int q = m.ids[i];
    pins_u[p] = pins[m.pbase[q] + (p - m.poff[i])] + m.voff[i];
  }
}

// flows of the kept pairs (weight of their nets cut by the union's minimal
// source side) and their vertex sides scattered into the regions' buffer
__global__ void __launch_bounds__(256) k_ru_flows(RgUnion m, const int32_t* w_u,
                                                  const uint8_t* ns_u, unsigned long long* flows) {
  const int i = blockIdx.x;
  unsigned long long sum = 0ull;
  for (int e = m.eoff[i] + threadIdx.x; e < m.eoff[i + 1]; e += blockDim.x)
    if ((ns_u[e] & 3u) == 1u) sum += (unsigned long long)w_u[e];
  block_add_u64(&flows[i], sum);
}

__global__ void k_ru_sides(RgUnion m, int32_t V, const uint8_t* vs_u, uint8_t* sides) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    const int i = rg_part(m.voff, m.n, v);
    const int q = m.ids[i];
    sides[m.vbase[q] + 2ll * q + (v - m.voff[i])] = vs_u[v];
  }
}

}  // namespace hf

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace hf {
namespace {

size_t rg_align(size_t x) { return (x + 255) & ~size_t(255); }

int rg_grid(long long n, int threads = 256) {
  long long b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

// Device allocations released together when the build returns.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t get(size_t count, T** out) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, rg_align(count * sizeof(T) + 1));
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return hipSuccess;
  }
};

fp_status rg_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    set_error("%s: out of device memory", what);
    return FP_ERR_OOM;
  }
  return hip_fail(e, what);
}

#define RG_TRY(expr, what)                   \
  do {                                       \
    const hipError_t e_ = (expr);            \
    if (e_ != hipSuccess) return rg_fail(e_, what); \
  } while (0)

template <class T>
hipError_t rg_exclusive_scan(Scratch& sc, const T* in, T* out, size_t n, hipStream_t s) {
  size_t tb = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, tb, in, out, T(0), n, rocprim::plus<T>(), s);
  if (e != hipSuccess) return e;
  void* tmp = nullptr;
  e = sc.get<char>(tb, reinterpret_cast<char**>(&tmp));
  if (e != hipSuccess) return e;
  return rocprim::exclusive_scan(tmp, tb, in, out, T(0), n, rocprim::plus<T>(), s);
}

unsigned rg_bits(long long n) {
  unsigned b = 1;
  while (b < 62 && (1ll << b) < n) ++b;
  return b;
}

}  // namespace

fp_status regions_build(int32_t V, int32_t E, const int32_t* off_in, const int32_t* pins_in,
                        const int32_t* w_in, const int32_t* cv_in, const int32_t* block_in,
                        int32_t k, int32_t npairs, const int32_t* pairs, const int64_t* caps,
                        int32_t flags, int32_t mem_kind, hipStream_t s, fp_regions** out) {
  Scratch sc;
  int dev = 0;
  RG_TRY(hipGetDevice(&dev), "hipGetDevice");
  // inputs on the device
  int32_t P = 0;
  const int32_t *off = off_in, *pins = pins_in, *w = w_in, *cv = cv_in, *block = block_in;
  if (mem_kind == 0) {
    P = off_in[E];
    if (P < 0) {
      set_error("net_offsets[num_nets] = %d is negative", P);
      return FP_ERR_INVALID;
    }
    int32_t *d_off, *d_pins, *d_w, *d_cv, *d_block;
    RG_TRY(sc.get(E + 1ull, &d_off), "allocating the hypergraph");
    RG_TRY(sc.get((size_t)P, &d_pins), "allocating the hypergraph");
    RG_TRY(sc.get((size_t)E, &d_w), "allocating the hypergraph");
    RG_TRY(sc.get((size_t)V, &d_cv), "allocating the hypergraph");
    RG_TRY(sc.get((size_t)V, &d_block), "allocating the hypergraph");
    RG_TRY(hipMemcpyAsync(d_off, off_in, (E + 1ull) * 4, hipMemcpyHostToDevice, s), "copy");
    if (P) RG_TRY(hipMemcpyAsync(d_pins, pins_in, P * 4ull, hipMemcpyHostToDevice, s), "copy");
    if (E) RG_TRY(hipMemcpyAsync(d_w, w_in, E * 4ull, hipMemcpyHostToDevice, s), "copy");
    if (V) {
      RG_TRY(hipMemcpyAsync(d_cv, cv_in, V * 4ull, hipMemcpyHostToDevice, s), "copy");
      RG_TRY(hipMemcpyAsync(d_block, block_in, V * 4ull, hipMemcpyHostToDevice, s), "copy");
    }
    off = d_off;
    pins = d_pins;
    w = d_w;
    cv = d_cv;
    block = d_block;
  }
  int* err = nullptr;
  RG_TRY(sc.get(1, &err), "allocating");
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(err), 1);
  k_rg_check_nets<<<rg_grid(E), 256, 0, s>>>(E, off, w, err);
  int herr = 0;
  RG_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "reading the checks");
  if (mem_kind != 0) RG_TRY(hipMemcpyAsync(&P, off + E, 4, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "checking the nets");
  if (herr & RERR_OFFSETS) {
    set_error("net_offsets must start at 0 and be nondecreasing");
    return FP_ERR_INVALID;
  }
  if (herr & RERR_WEIGHTS) {
    set_error("net weights must be >= 1");
    return FP_ERR_INVALID;
  }
  k_rg_check_rest<<<rg_grid(std::max<long long>(P, V)), 256, 0, s>>>(V, P, k, pins, cv, block,
                                                                         err);
  RG_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "reading the checks");
  RG_TRY(hipStreamSynchronize(s), "checking the pins");
  if (herr & RERR_PINS) {
    set_error("pin ids must lie in [0, num_vertices)");
    return FP_ERR_INVALID;
  }
  if (herr & RERR_VWEIGHTS) {
    set_error("vertex weights must be >= 1");
    return FP_ERR_INVALID;
  }
  if (herr & RERR_BLOCKS) {
    set_error("block ids must lie in [0, k)");
    return FP_ERR_INVALID;
  }

  // vertex -> nets (stable radix sort of the pins by vertex, values = nets)
  int32_t *pin_net, *vkeys, *vnet, *voff, *bkeys, *bverts, *boff, *blocal, *iota;
  unsigned long long* mask;
  RG_TRY(sc.get((size_t)P, &pin_net), "allocating");
  RG_TRY(sc.get((size_t)P, &vkeys), "allocating");
  RG_TRY(sc.get((size_t)P, &vnet), "allocating");
  RG_TRY(sc.get(V + 1ull, &voff), "allocating");
  RG_TRY(sc.get((size_t)V, &bkeys), "allocating");
  RG_TRY(sc.get((size_t)V, &bverts), "allocating");
  RG_TRY(sc.get(k + 1ull, &boff), "allocating");
  RG_TRY(sc.get((size_t)V, &blocal), "allocating");
  RG_TRY(sc.get((size_t)V, &iota), "allocating");
  RG_TRY(sc.get((size_t)E, &mask), "allocating");
  k_rg_pin_net<<<rg_grid(E), 256, 0, s>>>(E, off, pin_net);
  {
    const unsigned vb = rg_bits(V);
    size_t tb = 0;
    RG_TRY(rocprim::radix_sort_pairs(nullptr, tb, pins, vkeys, pin_net, vnet, (size_t)P, 0u, vb,
                                     s), "sizing the pin sort");
    char* tmp = nullptr;
    RG_TRY(sc.get(tb, &tmp), "allocating");
    RG_TRY(rocprim::radix_sort_pairs(tmp, tb, pins, vkeys, pin_net, vnet, (size_t)P, 0u, vb, s),
           "sorting the pins by vertex");
    k_rg_offsets<<<rg_grid(P + 1ll), 256, 0, s>>>(vkeys, P, V, voff);
  }
  {
    const auto cnt = rocprim::counting_iterator<int32_t>(0);
    const unsigned kb = rg_bits(k);
    size_t tb = 0;
    RG_TRY(rocprim::radix_sort_pairs(nullptr, tb, block, bkeys, cnt, bverts, (size_t)V, 0u, kb,
                                     s), "sizing the vertex sort");
    char* tmp = nullptr;
    RG_TRY(sc.get(tb, &tmp), "allocating");
    RG_TRY(rocprim::radix_sort_pairs(tmp, tb, block, bkeys, cnt, bverts, (size_t)V, 0u, kb, s),
           "sorting the vertices by block");
    k_rg_offsets<<<rg_grid(V + 1ll), 256, 0, s>>>(bkeys, V, k, boff);
    k_rg_local<<<rg_grid(V), 256, 0, s>>>(V, bverts, bkeys, boff, blocal);
  }
  k_rg_masks<<<rg_grid(E), 256, 0, s>>>(E, off, pins, block, mask);
  std::vector<int32_t> boff_h(k + 1);
  RG_TRY(hipMemcpyAsync(boff_h.data(), boff, (k + 1) * 4ull, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "preparing the hypergraph");

  fp_regions* r = new fp_regions();
  std::unique_ptr<fp_regions, void (*)(fp_regions*)> guard(r, [](fp_regions* x) {
    if (x->mem) (void)hipFree(x->mem);
    delete x;
  });
  r->device = dev;
  r->npairs = npairs;
  r->k = k;
  r->V = V;
  r->pairs.assign(pairs, pairs + 2ll * npairs);
  r->info.assign((size_t)npairs * kInfoLen, 0);
  if (npairs == 0) {
    *out = guard.release();
    return FP_OK;
  }

  // per side scratch: three bitmaps over the block, the level list / local
  // ids, a bitmap over the nets
  const int S = 2 * npairs;
  std::vector<long long> bits_at(S), lev_at(S);
  long long bw = 0, lw = 0;
  for (int t = 0; t < S; ++t) {
    const int b = pairs[t];
    const long long nb = boff_h[b + 1] - boff_h[b];
    bits_at[t] = bw;
    lev_at[t] = lw;
    bw += 3 * ((nb + 31) / 32);
    lw += nb;
  }
  const long long xwords = (E + 31ll) / 32;
  int32_t *pairs_d, *lev, *lmap;
  long long *caps_d, *bits_at_d, *lev_at_d, *side_out;
  uint32_t *bits, *xmark;
  RG_TRY(sc.get((size_t)S, &pairs_d), "allocating");
  RG_TRY(sc.get((size_t)S, &caps_d), "allocating");
  RG_TRY(sc.get((size_t)S, &bits_at_d), "allocating");
  RG_TRY(sc.get((size_t)S, &lev_at_d), "allocating");
  RG_TRY(sc.get(4ull * S, &side_out), "allocating");
  RG_TRY(sc.get((size_t)std::max(bw, 1ll), &bits), "allocating the region bitmaps");
  RG_TRY(sc.get((size_t)std::max(lw, 1ll), &lev), "allocating the level lists");
  RG_TRY(sc.get((size_t)std::max(lw, 1ll), &lmap), "allocating the local ids");
  RG_TRY(sc.get((size_t)S * xwords, &xmark), "allocating the net bitmaps");
  RG_TRY(hipMemcpyAsync(pairs_d, pairs, S * 4ull, hipMemcpyHostToDevice, s), "copy");
  RG_TRY(hipMemcpyAsync(caps_d, caps, S * 8ull, hipMemcpyHostToDevice, s), "copy");
  RG_TRY(hipMemcpyAsync(bits_at_d, bits_at.data(), S * 8ull, hipMemcpyHostToDevice, s), "copy");
  RG_TRY(hipMemcpyAsync(lev_at_d, lev_at.data(), S * 8ull, hipMemcpyHostToDevice, s), "copy");
  k_rg_zero<<<rg_grid(bw, 256), 256, 0, s>>>(bits, bw);
  k_rg_zero<<<4096, 256, 0, s>>>(xmark, (long long)S * xwords);

  RgGraph g{V, E, off, pins, w, cv, block, voff, vnet, bverts, boff, blocal, mask};
  RgSide rs{pairs_d, caps_d, bits_at_d, lev_at_d, bits, lev, xmark, xwords, side_out};
  k_rg_grow<<<S, kRegBlock, 0, s>>>(g, rs);
  std::vector<long long> side_h(4ull * S);
  RG_TRY(hipMemcpyAsync(side_h.data(), side_out, 32ull * S, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "growing the regions");

  // vertex outputs
  std::vector<long long> nloc(npairs), vbase(npairs);
  long long nv_tot = 0;
  for (int q = 0; q < npairs; ++q) {
    nloc[q] = side_h[4 * (2 * q) + 1] + side_h[4 * (2 * q + 1) + 1];
    vbase[q] = nv_tot;
    nv_tot += nloc[q];
  }
  r->vtx_base = vbase;
  r->nloc = nloc;
  long long *vbase_d, *nloc_d, *ntouch_d;
  RG_TRY(sc.get((size_t)npairs, &vbase_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &nloc_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &ntouch_d), "allocating");
  RG_TRY(hipMemcpyAsync(vbase_d, vbase.data(), npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  RG_TRY(hipMemcpyAsync(nloc_d, nloc.data(), npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  int32_t *vgid_d, *vw_d, *terms_d;
  int8_t* vside_d;
  RG_TRY(sc.get((size_t)std::max(nv_tot, 1ll), &vgid_d), "allocating");
  RG_TRY(sc.get((size_t)std::max(nv_tot, 1ll), &vside_d), "allocating");
  RG_TRY(sc.get((size_t)(nv_tot + 2ll * npairs), &vw_d), "allocating");
  RG_TRY(sc.get((size_t)(2ll * npairs), &terms_d), "allocating");
  RgOut ro{vbase_d, vgid_d, vside_d, vw_d, terms_d, lmap, ntouch_d};
  k_rg_members<<<npairs, kRegBlock, 0, s>>>(g, rs, ro);
  std::vector<long long> ntouch(npairs), tbase(npairs);
  RG_TRY(hipMemcpyAsync(ntouch.data(), ntouch_d, npairs * 8ull, hipMemcpyDeviceToHost, s), "read");
  RG_TRY(hipStreamSynchronize(s), "listing the region vertices");
  long long nt = 0;
  for (int q = 0; q < npairs; ++q) {
    tbase[q] = nt;
    nt += ntouch[q];
  }
  if (nt >= (1ll << 31)) {
    set_error("the regions touch %lld nets in all, more than 31-bit ids allow", nt);
    return FP_ERR_OVERFLOW;
  }
  long long* tbase_d;
  int32_t *tnet, *tpair, *keep, *kidx;
  long long *osz, *opos;
  unsigned long long* cutb;
  RG_TRY(sc.get((size_t)npairs, &tbase_d), "allocating");
  RG_TRY(sc.get((size_t)std::max(nt, 1ll), &tnet), "allocating");
  RG_TRY(sc.get((size_t)std::max(nt, 1ll), &tpair), "allocating");
  RG_TRY(sc.get((size_t)nt + 1, &keep), "allocating");
  RG_TRY(sc.get((size_t)nt + 1, &kidx), "allocating");
  RG_TRY(sc.get((size_t)nt + 1, &osz), "allocating");
  RG_TRY(sc.get((size_t)nt + 1, &opos), "allocating");
  RG_TRY(sc.get((size_t)npairs, &cutb), "allocating");
  RG_TRY(hipMemcpyAsync(tbase_d, tbase.data(), npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  k_rg_zero<<<rg_grid(2ll * npairs), 256, 0, s>>>(reinterpret_cast<uint32_t*>(cutb),
                                                   2ll * npairs);
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(keep + nt), 1);
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(osz + nt), 2);
  k_rg_touch_list<<<npairs, kRegBlock, 0, s>>>(rs, tbase_d, tnet, tpair);
  RgNets tn{(int32_t)nt, tnet, tpair, keep, osz, cutb};
  k_rg_count_flat<<<rg_grid(nt, kFlatBlock * 4), kFlatBlock, 0, s>>>(g, rs, lmap, tn);
  RG_TRY(rg_exclusive_scan<int32_t>(sc, keep, kidx, (size_t)nt + 1, s), "scanning the nets");
  RG_TRY(rg_exclusive_scan<long long>(sc, osz, opos, (size_t)nt + 1, s), "scanning the pins");
  int32_t nk32 = 0;
  long long npk = 0;
  RG_TRY(hipMemcpyAsync(&nk32, kidx + nt, 4, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipMemcpyAsync(&npk, opos + nt, 8, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "counting the nets");
  const long long nk = nk32;
  if (npk >= (1ll << 31)) {
    set_error("the regions hold %lld pins in all, more than 31-bit offsets allow", npk);
    return FP_ERR_OVERFLOW;
  }
  long long *koff, *kw, *kw0;
  int32_t *kpins, *kpair, *kgid, *unsorted;
  RG_TRY(sc.get((size_t)nk + 1, &koff), "allocating");
  RG_TRY(sc.get((size_t)std::max(npk, 1ll), &kpins), "allocating");
  RG_TRY(sc.get((size_t)std::max(nk, 1ll), &kpair), "allocating");
  RG_TRY(sc.get((size_t)std::max(nk, 1ll), &kgid), "allocating");
  RG_TRY(sc.get((size_t)std::max(nk, 1ll), &kw), "allocating");
  RG_TRY(sc.get((size_t)std::max(nk, 1ll), &kw0), "allocating");
  unsigned long long* kcount;
  RG_TRY(sc.get(1, &unsorted), "allocating");
  RG_TRY(sc.get((size_t)npairs, &kcount), "allocating");
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(unsorted), 1);
  k_rg_kept_per_pair<<<rg_grid(npairs), 256, 0, s>>>(npairs, tbase_d, (int)nt, kidx, kcount);
  RG_TRY(hipMemcpyAsync(koff + nk, &npk, 8, hipMemcpyHostToDevice, s), "copy");
  RgKept kp{kidx, opos, nloc_d, koff, kpins, kpair, kgid, kw, unsorted};
  k_rg_write_flat<<<rg_grid(nt, kFlatBlock * 4), kFlatBlock, 0, s>>>(g, rs, lmap, tn, kp);
  k_rg_check_sorted<<<rg_grid(nk), 256, 0, s>>>(nk, koff, kpins, unsorted);
  int hunsorted = 0;
  RG_TRY(hipMemcpyAsync(&hunsorted, unsorted, 4, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "writing the nets");
  if (hunsorted && npk > 0) {
    // some net lists its region pins out of order: sort every net's pins by
    // (net, local id) keys
    unsigned long long *keys, *keys2;
    RG_TRY(sc.get((size_t)npk, &keys), "allocating");
    RG_TRY(sc.get((size_t)npk, &keys2), "allocating");
    k_rg_sort_keys<<<rg_grid(nk), 256, 0, s>>>(nk, koff, kpins, keys);
    const unsigned eb = 32 + rg_bits(nk + 1);
    size_t tb = 0;
    RG_TRY(rocprim::radix_sort_keys(nullptr, tb, keys, keys2, (size_t)npk, 0u, eb, s), "sizing");
    char* tmp = nullptr;
    RG_TRY(sc.get(tb, &tmp), "allocating");
    RG_TRY(rocprim::radix_sort_keys(tmp, tb, keys, keys2, (size_t)npk, 0u, eb, s),
           "sorting the pins of the nets");
    k_rg_sort_back<<<rg_grid(npk), 256, 0, s>>>(npk, keys2, kpins);
  }
  int32_t* dead = nullptr;
  if ((flags & 1) && nk > 1) {
    unsigned long long *fkey, *fkey2;
    int32_t *fval, *fval2, *head, *run;
    RG_TRY(sc.get((size_t)nk, &fkey), "allocating");
    RG_TRY(sc.get((size_t)nk, &fkey2), "allocating");
    RG_TRY(sc.get((size_t)nk, &fval), "allocating");
    RG_TRY(sc.get((size_t)nk, &fval2), "allocating");
    RG_TRY(sc.get((size_t)nk, &head), "allocating");
    RG_TRY(sc.get((size_t)nk, &run), "allocating");
    RG_TRY(sc.get((size_t)nk, &dead), "allocating");
    k_rg_zero<<<rg_grid(nk), 256, 0, s>>>(reinterpret_cast<uint32_t*>(dead), nk);
    k_rg_fingerprint<<<rg_grid(nk), 256, 0, s>>>(nk, koff, kpins, kpair, fkey, fval);
    size_t tb = 0;
    RG_TRY(rocprim::radix_sort_pairs(nullptr, tb, fkey, fkey2, fval, fval2, (size_t)nk, 0u, 64u,
                                     s), "sizing");
    char* tmp = nullptr;
    RG_TRY(sc.get(tb, &tmp), "allocating");
    RG_TRY(rocprim::radix_sort_pairs(tmp, tb, fkey, fkey2, fval, fval2, (size_t)nk, 0u, 64u, s),
           "sorting the fingerprints");
    k_rg_run_heads<<<rg_grid(nk), 256, 0, s>>>(nk, fkey2, head);
    size_t tb2 = 0;
    RG_TRY(rocprim::inclusive_scan(nullptr, tb2, head, run, (size_t)nk, rocprim::maximum<int32_t>(),
                                   s), "sizing");
    char* tmp2 = nullptr;
    RG_TRY(sc.get(tb2, &tmp2), "allocating");
    RG_TRY(rocprim::inclusive_scan(tmp2, tb2, head, run, (size_t)nk, rocprim::maximum<int32_t>(),
                                   s), "finding runs");
    RG_TRY(hipMemcpyAsync(kw0, kw, nk * 8ull, hipMemcpyDeviceToDevice, s), "copy");
    k_rg_dups<<<rg_grid(nk), 256, 0, s>>>(nk, fval2, run, koff, kpins, kpair, kw0, kw, dead);
  }
  // final layout
  long long *alive, *asz, *fidx, *fpos, *nbase_d, *pbase_d;
  unsigned long long *ne_d, *np_d, *bins_d;
  RG_TRY(sc.get((size_t)nk + 1, &alive), "allocating");
  RG_TRY(sc.get((size_t)nk + 1, &asz), "allocating");
  RG_TRY(sc.get((size_t)nk + 1, &fidx), "allocating");
  RG_TRY(sc.get((size_t)nk + 1, &fpos), "allocating");
  RG_TRY(sc.get((size_t)npairs, &nbase_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &pbase_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &ne_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &np_d), "allocating");
  RG_TRY(sc.get(7ull * npairs, &bins_d), "allocating");
  k_rg_zero<<<rg_grid(4ll * npairs), 256, 0, s>>>(reinterpret_cast<uint32_t*>(ne_d),
                                                   2ll * npairs);
  k_rg_zero<<<rg_grid(4ll * npairs), 256, 0, s>>>(reinterpret_cast<uint32_t*>(np_d),
                                                   2ll * npairs);
  k_rg_zero<<<rg_grid(14ll * npairs), 256, 0, s>>>(reinterpret_cast<uint32_t*>(bins_d),
                                                    14ll * npairs);
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(alive + nk), 2);
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(asz + nk), 2);
  k_rg_alive_sizes<<<rg_grid(nk), 256, 0, s>>>(nk, koff, dead, alive, asz, kpair, ne_d, np_d);
  RG_TRY(rg_exclusive_scan<long long>(sc, alive, fidx, (size_t)nk + 1, s), "scanning");
  RG_TRY(rg_exclusive_scan<long long>(sc, asz, fpos, (size_t)nk + 1, s), "scanning");
  std::vector<unsigned long long> ne_h(npairs), np_h(npairs), cut_h(npairs);
  RG_TRY(hipMemcpyAsync(ne_h.data(), ne_d, npairs * 8ull, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipMemcpyAsync(np_h.data(), np_d, npairs * 8ull, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipMemcpyAsync(cut_h.data(), cutb, npairs * 8ull, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "merging identical nets");
  std::vector<long long> nbase(npairs), pbase(npairs);
  long long ne_tot = 0, np_tot = 0;
  for (int q = 0; q < npairs; ++q) {
    nbase[q] = ne_tot;
    pbase[q] = np_tot;
    ne_tot += (long long)ne_h[q];
    np_tot += (long long)np_h[q];
  }
  r->net_base = nbase;
  r->pin_base = pbase;
  // one allocation for the outputs
  size_t bytes = 0;
  auto add = [&](size_t n) {
    const size_t at = bytes;
    bytes += rg_align(n * 4 + 1);
    return at;
  };
  const size_t o_off = add(ne_tot + npairs), o_pins = add(np_tot), o_w = add(ne_tot),
               o_ngid = add(ne_tot), o_vw = add(nv_tot + 2ll * npairs), o_vgid = add(nv_tot),
               o_terms = add(2ll * npairs), o_vside = add((nv_tot + 3) / 4);
  RG_TRY(hipMalloc(&r->mem, bytes), "allocating the regions");
  char* base = static_cast<char*>(r->mem);
  r->off = reinterpret_cast<int32_t*>(base + o_off);
  r->pins = reinterpret_cast<int32_t*>(base + o_pins);
  r->w = reinterpret_cast<int32_t*>(base + o_w);
  r->ngid = reinterpret_cast<int32_t*>(base + o_ngid);
  r->vw = reinterpret_cast<int32_t*>(base + o_vw);
  r->vgid = reinterpret_cast<int32_t*>(base + o_vgid);
  r->terms = reinterpret_cast<int32_t*>(base + o_terms);
  r->vside = reinterpret_cast<int8_t*>(base + o_vside);
  RG_TRY(hipMemcpyAsync(nbase_d, nbase.data(), npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  RG_TRY(hipMemcpyAsync(pbase_d, pbase.data(), npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  RgFinal fo{dead, fidx, fpos, nbase_d, pbase_d, r->off, r->pins, r->w, r->ngid, bins_d, err};
  k_rg_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(err), 1);
  k_rg_final<<<rg_grid(nk), 256, 0, s>>>(nk, koff, kpins, kpair, kgid, kw, fo);
  k_rg_last_offsets<<<rg_grid(npairs), 256, 0, s>>>(npairs, nbase_d, pbase_d, ne_d, np_d, r->off);
  if (nv_tot)
    RG_TRY(hipMemcpyAsync(r->vgid, vgid_d, nv_tot * 4ull, hipMemcpyDeviceToDevice, s), "copy");
  RG_TRY(hipMemcpyAsync(r->vw, vw_d, (nv_tot + 2ll * npairs) * 4ull, hipMemcpyDeviceToDevice, s),
         "copy");
  RG_TRY(hipMemcpyAsync(r->terms, terms_d, 2ll * npairs * 4, hipMemcpyDeviceToDevice, s), "copy");
  if (nv_tot)
    RG_TRY(hipMemcpyAsync(r->vside, vside_d, nv_tot, hipMemcpyDeviceToDevice, s), "copy");
  std::vector<unsigned long long> bins_h(7ull * npairs);
  RG_TRY(hipMemcpyAsync(bins_h.data(), bins_d, 56ull * npairs, hipMemcpyDeviceToHost, s), "read");
  RG_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "reading");
  RG_TRY(hipStreamSynchronize(s), "writing the regions");
  if (herr) {
    set_error("merged net weights exceed INT32_MAX");
    return FP_ERR_OVERFLOW;
  }
  for (int q = 0; q < npairs; ++q) {
    int64_t* in = &r->info[(size_t)q * kInfoLen];
    const long long* s0 = &side_h[4 * (2 * q)];
    const long long* s1 = &side_h[4 * (2 * q + 1)];
    in[0] = nloc[q];
    in[1] = nloc[q] + 2;
    in[2] = (int64_t)ne_h[q];
    in[3] = (int64_t)np_h[q];
    in[4] = (int64_t)cut_h[q];
    in[5] = s0[2] + s1[2];
    in[6] = s0[0];
    in[7] = s1[0];
    for (int b = 0; b < 7; ++b) in[8 + b] = (int64_t)bins_h[7 * q + b];
  }
  // nets merged per pair: kept nets minus final nets
  {
    std::vector<unsigned long long> kc(npairs);
    RG_TRY(hipMemcpyAsync(kc.data(), kcount, npairs * 8ull, hipMemcpyDeviceToHost, s), "read");
    RG_TRY(hipStreamSynchronize(s), "reading");
    for (int q = 0; q < npairs; ++q)
      r->info[(size_t)q * kInfoLen + 15] = (int64_t)kc[q] - (int64_t)ne_h[q];
  }
  *out = guard.release();
  return FP_OK;
}

// Solve the kept pairs as disjoint-union networks (split where 31-bit ids
// or the INT32_MAX bound of a network's weight sum would be exceeded); flows
// of skipped pairs are -1.  The minimal source sides are kept in r->sides.
fp_status regions_solve(fp_regions* r, const uint8_t* skip, hipStream_t s, int64_t* flows) {
  const int npairs = r->npairs;
  if (npairs == 0) return FP_OK;
  if (!r->sides) {
    long long nb = 0;
    for (int q = 0; q < npairs; ++q) nb += r->nloc[q] + 2;
    RG_TRY(hipMalloc(&r->sides, (size_t)nb + 1), "allocating the source sides");
  }
  if (r->wsum.empty()) {
    // net weight sum of every pair
    r->wsum.assign(npairs, 0);
    std::vector<int32_t> w((size_t)std::max<long long>(r->net_base.back() + r->info[(size_t)(npairs - 1) * kInfoLen + 2], 1));
    const long long ne_tot = r->net_base.back() + r->info[(size_t)(npairs - 1) * kInfoLen + 2];
    if (ne_tot)
      RG_TRY(hipMemcpyAsync(w.data(), r->w, ne_tot * 4ull, hipMemcpyDeviceToHost, s), "reading");
    RG_TRY(hipStreamSynchronize(s), "reading the net weights");
    for (int q = 0; q < npairs; ++q) {
      long long acc = 0;
      const long long b = r->net_base[q], ne = r->info[(size_t)q * kInfoLen + 2];
      for (long long e = 0; e < ne; ++e) acc += w[b + e];
      r->wsum[q] = acc;
    }
  }
  Scratch sc;
  long long *nbase_d, *pbase_d, *vbase_d;
  RG_TRY(sc.get((size_t)npairs, &nbase_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &pbase_d), "allocating");
  RG_TRY(sc.get((size_t)npairs, &vbase_d), "allocating");
  RG_TRY(hipMemcpyAsync(nbase_d, r->net_base.data(), npairs * 8ull, hipMemcpyHostToDevice, s),
         "copy");
  RG_TRY(hipMemcpyAsync(pbase_d, r->pin_base.data(), npairs * 8ull, hipMemcpyHostToDevice, s),
         "copy");
  RG_TRY(hipMemcpyAsync(vbase_d, r->vtx_base.data(), npairs * 8ull, hipMemcpyHostToDevice, s),
         "copy");
  for (int q = 0; q < npairs; ++q) flows[q] = -1;
  const long long kLimit = (1ll << 30);
  int q = 0;
  while (q < npairs) {
    // next chunk of kept pairs
    std::vector<int32_t> ids, voff(1, 0), eoff(1, 0), poff(1, 0), src, snk;
    long long V = 0, E = 0, P = 0, W = 0;
    for (; q < npairs; ++q) {
      if (skip && skip[q]) continue;
      const int64_t* in = &r->info[(size_t)q * kInfoLen];
      const long long nv = in[1], ne = in[2], np = in[3];
      if (!ids.empty() && (V + nv + 2 * (E + ne) >= kLimit || P + np >= kLimit ||
                           W + r->wsum[q] > 0x7fffffffll))
        break;
      ids.push_back(q);
      src.push_back((int32_t)(V + in[0]));
      snk.push_back((int32_t)(V + in[0] + 1));
      V += nv;
      E += ne;
      P += np;
      W += r->wsum[q];
      voff.push_back((int32_t)V);
      eoff.push_back((int32_t)E);
      poff.push_back((int32_t)P);
    }
    if (ids.empty()) break;
    const int n = (int)ids.size();
    int32_t *ids_d, *voff_d, *eoff_d, *poff_d, *off_u, *w_u, *pins_u, *src_d, *snk_d;
    uint8_t *vs_u, *ns_u;
    unsigned long long* fl_d;
    RG_TRY(sc.get((size_t)n, &ids_d), "allocating");
    RG_TRY(sc.get(n + 1ull, &voff_d), "allocating");
    RG_TRY(sc.get(n + 1ull, &eoff_d), "allocating");
    RG_TRY(sc.get(n + 1ull, &poff_d), "allocating");
    RG_TRY(sc.get(E + 1ull, &off_u), "allocating the union");
    RG_TRY(sc.get(E + 1ull, &w_u), "allocating the union");
    RG_TRY(sc.get(P + 1ull, &pins_u), "allocating the union");
    RG_TRY(sc.get((size_t)n, &src_d), "allocating");
    RG_TRY(sc.get((size_t)n, &snk_d), "allocating");
    RG_TRY(sc.get(V + 1ull, &vs_u), "allocating");
    RG_TRY(sc.get(E + 1ull, &ns_u), "allocating");
    RG_TRY(sc.get((size_t)n, &fl_d), "allocating");
    RG_TRY(hipMemcpyAsync(ids_d, ids.data(), n * 4ull, hipMemcpyHostToDevice, s), "copy");
    RG_TRY(hipMemcpyAsync(voff_d, voff.data(), (n + 1) * 4ull, hipMemcpyHostToDevice, s), "copy");
    RG_TRY(hipMemcpyAsync(eoff_d, eoff.data(), (n + 1) * 4ull, hipMemcpyHostToDevice, s), "copy");
    RG_TRY(hipMemcpyAsync(poff_d, poff.data(), (n + 1) * 4ull, hipMemcpyHostToDevice, s), "copy");
    RG_TRY(hipMemcpyAsync(src_d, src.data(), n * 4ull, hipMemcpyHostToDevice, s), "copy");
    RG_TRY(hipMemcpyAsync(snk_d, snk.data(), n * 4ull, hipMemcpyHostToDevice, s), "copy");
    k_rg_zero<<<rg_grid(2ll * n), 256, 0, s>>>(reinterpret_cast<uint32_t*>(fl_d), 2ll * n);
    RgUnion m{n, ids_d, voff_d, eoff_d, poff_d, nbase_d, pbase_d, vbase_d};
    k_ru_nets<<<rg_grid(E + 1), 256, 0, s>>>(m, r->off, r->w, (int32_t)E, off_u, w_u);
    if (P) k_ru_pins<<<rg_grid(P), 256, 0, s>>>(m, r->pins, (int32_t)P, pins_u);
    fp_problem* u = new (std::nothrow) fp_problem();
    if (!u) {
      set_error("host allocation failed");
      return FP_ERR_OOM;
    }
    u->device = r->device;
    u->V = (int32_t)V;
    u->E = (int32_t)E;
    fp_options o{};
    o.group_lanes = 8;
    o.gr_interval = 8;
    u->opt = resolve_options(&o);
    fp_status st = build_problem(u, off_u, pins_u, w_u, src_d, n, snk_d, n, 1, s);
    int64_t F = 0;
    if (st == FP_OK) st = solve_problem(u, s, &F);
    if (st == FP_OK) st = cut_problem(u, s, 1, vs_u, ns_u);
    std::vector<unsigned long long> fh(n, 0ull);
    if (st == FP_OK) {
      k_ru_flows<<<n, 256, 0, s>>>(m, u->dev.w, ns_u, fl_d);
      k_ru_sides<<<rg_grid(V), 256, 0, s>>>(m, (int32_t)V, vs_u, r->sides);
      hipError_t he = hipMemcpyAsync(fh.data(), fl_d, n * 8ull, hipMemcpyDeviceToHost, s);
      if (he == hipSuccess) he = hipStreamSynchronize(s);
      if (he != hipSuccess) st = hip_fail(he, "splitting the union's flow");
    }
    if (st != FP_OK) (void)hipStreamSynchronize(s);
    release_problem(u);
    delete u;
    if (st != FP_OK) return st;
    unsigned long long tot = 0ull;
    for (int i = 0; i < n; ++i) {
      flows[ids[i]] = (int64_t)fh[i];
      tot += fh[i];
    }
    if ((int64_t)tot != F) {
      set_error("internal check: the pairs' cut weights sum to %llu, the union's flow is %lld",
                tot, (long long)F);
      return FP_ERR_DEVICE;
    }
    r->solved = true;
  }
  return FP_OK;
}

void release_regions(fp_regions* r) {
  if (!r) return;
  if (r->mem) (void)hipFree(r->mem);
  if (r->sides) (void)hipFree(r->sides);
  delete r;
}

}  // namespace hf

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

using namespace hf;

#pragma GCC visibility push(default)
extern "C" {

fp_status flow_regions_build(int32_t num_vertices, int32_t num_nets, const int32_t* net_offsets,
                             const int32_t* pins, const int32_t* net_weights,
                             const int32_t* vertex_weights, const int32_t* blocks, int32_t k,
                             int32_t num_pairs, const int32_t* pairs, const int64_t* caps,
                             int32_t flags, int32_t mem_kind, void* hip_stream,
                             fp_regions** out) {
  set_error("");
  if (!out) {
    set_error("out is NULL");
    return FP_ERR_INVALID;
  }
  *out = nullptr;
  if (num_vertices < 1 || num_nets < 0 || num_pairs < 0) {
    set_error("need num_vertices >= 1, num_nets >= 0, num_pairs >= 0 (got %d, %d, %d)",
              num_vertices, num_nets, num_pairs);
    return FP_ERR_INVALID;
  }
  if (k < 2 || k > 64) {
    set_error("k must lie in [2, 64], got %d", k);
    return FP_ERR_INVALID;
  }
  if (mem_kind != 0 && mem_kind != 1) {
    set_error("mem_kind must be 0 (host) or 1 (device), got %d", mem_kind);
    return FP_ERR_INVALID;
  }
  if ((flags & ~1) != 0) {
    set_error("unknown flags 0x%x", flags);
    return FP_ERR_INVALID;
  }
  if (!net_offsets || !vertex_weights || !blocks || (num_nets > 0 && !net_weights) ||
      (num_pairs > 0 && (!pairs || !caps))) {
    set_error("NULL input pointer");
    return FP_ERR_INVALID;
  }
  for (int32_t q = 0; q < num_pairs; ++q) {
    const int32_t i = pairs[2 * q], j = pairs[2 * q + 1];
    if (i < 0 || i >= k || j < 0 || j >= k || i == j) {
      set_error("pair %d = (%d, %d): blocks must be distinct ids in [0, k)", q, i, j);
      return FP_ERR_INVALID;
    }
    if (caps[2 * q] < 0 || caps[2 * q + 1] < 0) {
      set_error("pair %d: caps must be >= 0", q);
      return FP_ERR_INVALID;
    }
  }
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const fp_status st = regions_build(num_vertices, num_nets, net_offsets, pins, net_weights,
                                     vertex_weights, blocks, k, num_pairs, pairs, caps, flags,
                                     mem_kind, s, out);
  if (st != FP_OK) (void)hipStreamSynchronize(s);
  return st;
}

fp_status flow_regions_info(const fp_regions* regions, int32_t pair, int64_t* info) {
  set_error("");
  if (!regions || !info) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  if (pair < 0 || pair >= regions->npairs) {
    set_error("pair %d out of range [0, %d)", pair, regions->npairs);
    return FP_ERR_INVALID;
  }
  std::memcpy(info, &regions->info[(size_t)pair * kInfoLen], sizeof(int64_t) * kInfoLen);
  return FP_OK;
}

fp_status flow_regions_export(const fp_regions* regions, int32_t pair, int32_t mem_kind,
                              void* hip_stream, int32_t* net_offsets, int32_t* pins,
                              int32_t* net_weights, int32_t* vertex_weights, int32_t* vertex_ids,
                              int32_t* net_ids) {
  set_error("");
  if (!regions) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  if (pair < 0 || pair >= regions->npairs) {
    set_error("pair %d out of range [0, %d)", pair, regions->npairs);
    return FP_ERR_INVALID;
  }
  if (mem_kind != 0 && mem_kind != 1) {
    set_error("mem_kind must be 0 (host) or 1 (device), got %d", mem_kind);
    return FP_ERR_INVALID;
  }
  const int64_t* in = &regions->info[(size_t)pair * kInfoLen];
  const long long n = in[0], ne = in[2], np = in[3];
  const long long nb = regions->net_base[pair], pb = regions->pin_base[pair],
                  vb = regions->vtx_base[pair];
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const hipMemcpyKind kind = mem_kind == 0 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  struct Part {
    int32_t* dst;
    const int32_t* src;
    long long count;
  } parts[] = {{net_offsets, regions->off + nb + pair, ne + 1},
               {pins, regions->pins + pb, np},
               {net_weights, regions->w + nb, ne},
               {vertex_weights, regions->vw + vb + 2ll * pair, n + 2},
               {vertex_ids, regions->vgid + vb, n},
               {net_ids, regions->ngid + nb, ne}};
  for (const Part& p : parts) {
    if (!p.dst || p.count == 0) continue;
    const hipError_t e = hipMemcpyAsync(p.dst, p.src, p.count * 4ull, kind, s);
    if (e != hipSuccess) return hip_fail(e, "copying a region out");
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "copying a region out");
  return FP_OK;
}

fp_status flow_regions_problem(const fp_regions* regions, int32_t pair, const fp_options* opts,
                               void* hip_stream, fp_problem** out) {
  set_error("");
  if (!regions || !out) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  if (pair < 0 || pair >= regions->npairs) {
    set_error("pair %d out of range [0, %d)", pair, regions->npairs);
    return FP_ERR_INVALID;
  }
  const int64_t* in = &regions->info[(size_t)pair * kInfoLen];
  const long long nb = regions->net_base[pair], pb = regions->pin_base[pair];
  return flow_problem_create((int32_t)in[1], (int32_t)in[2], regions->off + nb + pair,
                             regions->pins + pb, regions->w + nb, regions->terms + 2 * pair, 1,
                             regions->terms + 2 * pair + 1, 1, 1, opts, hip_stream, out);
}

fp_status flow_regions_solve(fp_regions* regions, const uint8_t* skip, void* hip_stream,
                             int64_t* flow_values) {
  set_error("");
  if (!regions || (regions->npairs > 0 && !flow_values)) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const fp_status st = regions_solve(regions, skip, s, flow_values);
  if (st != FP_OK) (void)hipStreamSynchronize(s);
  return st;
}

fp_status flow_regions_source_side(const fp_regions* regions, int32_t pair, int32_t mem_kind,
                                   void* hip_stream, uint8_t* vertex_side) {
  set_error("");
  if (!regions || !vertex_side) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  if (pair < 0 || pair >= regions->npairs) {
    set_error("pair %d out of range [0, %d)", pair, regions->npairs);
    return FP_ERR_INVALID;
  }
  if (!regions->solved) {
    set_error("the regions have not been solved");
    return FP_ERR_STATE;
  }
  const long long n = regions->nloc[pair];
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  if (n) e = hipMemcpyAsync(vertex_side, regions->sides + regions->vtx_base[pair] + 2ll * pair,
                            (size_t)n, mem_kind ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "copying a source side");
  return FP_OK;
}

void flow_regions_destroy(fp_regions* regions) { release_regions(regions); }

}  // extern "C"
#pragma GCC visibility pop
