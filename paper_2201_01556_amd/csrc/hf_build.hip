// Problem creation: copy the inputs to the device, validate them and build
// the device layout (net CSR as given, vertex incidence CSR by a stable radix
// sort of the pins by vertex, so each vertex lists its pins in slot order;
// terminal roles, per-net terminal flags).  Every step runs on the device.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include <mutex>
#include <vector>

#include "hf_host.h"

namespace hf {

// ---------------------------------------------------------------------------
// Reuse of released device pools and pinned control blocks.  A handle's pool
// is one hipMalloc (hundreds of MB for large problems) and its control block
// one pinned host allocation; creating and destroying handles in a loop
// would otherwise pay both every time.  Released blocks are kept per device
// (at most kCachedPoolBytes of pools and kCachedCtl control blocks) and
// reused for a request they cover without wasting more than half of them.
// Handles are destroyed only after their device work has finished, so a
// cached block is idle.
// ---------------------------------------------------------------------------

constexpr size_t kCachedPoolBytes = 4ull << 30;
constexpr size_t kCachedCtl = 256;

struct CachedPool {
  int device;
  void* ptr;
  size_t bytes;
};

static std::mutex g_cache_mu;
static std::vector<CachedPool> g_pools;
static std::vector<void*> g_ctls;

static hipError_t pool_acquire(int device, size_t bytes, void** out, size_t* got) {
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_pools.size(); ++i) {
      const CachedPool& c = g_pools[i];
      if (c.device != device || c.bytes < bytes || c.bytes > 2 * bytes) continue;
      if (best < 0 || c.bytes < g_pools[best].bytes) best = i;
    }
    if (best >= 0) {
      *out = g_pools[best].ptr;
      *got = g_pools[best].bytes;
      g_pools.erase(g_pools.begin() + best);
      return hipSuccess;
    }
  }
  *got = bytes;
  return hipMalloc(out, bytes);
}

static void pool_release(int device, void* ptr, size_t bytes) {
  if (!ptr) return;
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_pools.push_back(CachedPool{device, ptr, bytes});
    size_t total = 0;
    for (const CachedPool& c : g_pools) total += c.bytes;
    while (total > kCachedPoolBytes && !g_pools.empty()) {  // oldest first
      total -= g_pools.front().bytes;
      drop.push_back(g_pools.front().ptr);
      g_pools.erase(g_pools.begin());
    }
  }
  for (void* p : drop) (void)hipFree(p);
}

static hipError_t ctl_acquire(Ctl** out) {
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (!g_ctls.empty()) {
      *out = static_cast<Ctl*>(g_ctls.back());
      g_ctls.pop_back();
      return hipSuccess;
    }
  }
  return hipHostMalloc((void**)out, sizeof(Ctl), hipHostMallocDefault);
}

static void ctl_release(Ctl* c) {
  if (!c) return;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_ctls.size() < kCachedCtl) {
      g_ctls.push_back(c);
      return;
    }
  }
  (void)hipHostFree(c);
}

void release_cached_memory() {
  std::vector<CachedPool> pools;
  std::vector<void*> ctls;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    pools.swap(g_pools);
    ctls.swap(g_ctls);
  }
  for (const CachedPool& c : pools) {
    (void)hipSetDevice(c.device);
    (void)hipFree(c.ptr);
  }
  for (void* c : ctls) (void)hipHostFree(c);
}

// ---------------------------------------------------------------------------
// validation / layout kernels (thread per element, grid-stride)
// ---------------------------------------------------------------------------

__global__ void k_check_nets(Dev g, unsigned long long* wsum) {
  unsigned long long s = 0;
  int err = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.E; e += gridDim.x * blockDim.x) {
    const int lo = g.net_off[e], hi = g.net_off[e + 1];
    if (hi < lo || lo < 0 || hi > g.P) err |= ERR_BUILD_OFFSETS;
    if (e == 0 && lo != 0) err |= ERR_BUILD_OFFSETS;
    const int we = g.w[e];
    if (we < 1) err |= ERR_BUILD_WEIGHT;
    else s += (unsigned long long)we;
  }
  if (err) atomicOr(&g.ctl->err, err);
  block_add_u64(wsum, s);
}

__global__ void k_check_pins(Dev g) {
  int err = 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < g.P; p += gridDim.x * blockDim.x) {
    const int u = g.pin_v[p];
    if (u < 0 || u >= g.V) err |= ERR_BUILD_PIN;
  }
  if (err) atomicOr(&g.ctl->err, err);
}

__global__ void k_roles(Dev g, const int32_t* S, int nS, const int32_t* T, int nT) {
  int err = 0;
  const int n = nS + nT;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const bool src = i < nS;
    const int v = src ? S[i] : T[i - nS];
    if (v < 0 || v >= g.V) err |= ERR_BUILD_TERMINAL;
    else atomicOr(&g.role[v], src ? 1 : 2);
  }
  if (err) atomicOr(&g.ctl->err, err);
}

__global__ void k_role_check(Dev g) {
  int err = 0;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.V; v += gridDim.x * blockDim.x)
    if (g.role[v] == 3) err |= ERR_BUILD_ST;
  if (err) atomicOr(&g.ctl->err, err);
}

// Net of every pin slot: thread per net over its slot range (offsets were
// validated first).
__global__ void k_pin_nets(Dev g) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.E; e += gridDim.x * blockDim.x) {
    const int end = g.net_off[e + 1];
    for (int p = g.net_off[e]; p < end; ++p) const_cast<int32_t*>(g.pin_net)[p] = e;
  }
}

// Vertex offsets from the pins sorted by vertex: vtx_off[u] = first sorted
// position holding a vertex >= u (position P past the last); each position
// fills the offsets of the vertices between its predecessor's vertex and its
// own, so vertices without pins get empty ranges.
__global__ void k_vtx_offsets(const int32_t* keys, int P, int V, int32_t* vtx_off) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= P; i += gridDim.x * blockDim.x) {
    const int prev = i == 0 ? -1 : keys[i - 1];
    const int cur = i == P ? V : keys[i];
    for (int u = prev + 1; u <= cur; ++u) vtx_off[u] = i;
  }
}

// Sort value of pin slot p: the incidence {net, slot} as one 64-bit word
// (little-endian int2), read in slot order.
struct IncidenceOfSlot {
  const int32_t* pin_net;
  __host__ __device__ unsigned long long operator()(int32_t p) const {
    return ((unsigned long long)(uint32_t)p << 32) | (uint32_t)pin_net[p];
  }
};

// Checks over the incidences in sorted order (vinc[i] = {net, slot} of the
// i-th pin sorted by vertex): a vertex's pins are in slot order, hence
// grouped by net, so a vertex twice in one net shows as two neighbours with
// the same net.  Nets learn whether they hold a source or a sink pin.
__global__ void k_incidences(Dev g, const int32_t* keys) {
  int err = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.P; i += gridDim.x * blockDim.x) {
    const int e = g.vinc[i].x;
    const int u = keys[i];
    if (i > 0 && keys[i - 1] == u && g.vinc[i - 1].x == e) err |= ERR_BUILD_DUP;
    const int r = g.role[u];
    if (r) atomicOr(&g.nflag[e], r);
  }
  if (err) atomicOr(&g.ctl->err, err);
}

// bit v of the bitmaps: node v has more than big_deg (kHugeDeg) arcs
// (vertex: incident nets; net node: pins plus the bridge); padding nodes are
// never big
__global__ void k_bigbits(Dev g, uint32_t* bits, uint32_t* huge) {
  const int words = (g.N + 31) >> 5;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
    uint32_t m = 0, h = 0;
    for (int b = 0; b < 32; ++b) {
      const int v = (w << 5) + b;
      if (v >= g.N || (v >= g.V && v < g.NB)) continue;
      const int d = deg_of(g, v);
      if (d > g.big_deg) m |= 1u << b;
      if (d > kHugeDeg) h |= 1u << b;
    }
    bits[w] = m;
    huge[w] = h;
  }
}

// Clears n 32-bit words (a kernel rather than hipMemsetAsync, so that
// nothing in the build records a memset node when a caller captures it).
__global__ void k_zero_u32(uint32_t* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += align_up(count * sizeof(T) + 1);
    return p;
  }
};

static int grid_for(long long n, int threads = 256, int cap = 4096) {
  long long b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

fp_options resolve_options(const fp_options* o) {
  fp_options r{};
  if (o) r = *o;
  if (r.relabel_factor_x16 <= 0) r.relabel_factor_x16 = 16;
  if (r.tail_threshold <= 0) r.tail_threshold = 256;
  if (r.group_lanes != 4 && r.group_lanes != 8 && r.group_lanes != 16) r.group_lanes = 16;
  if (r.big_degree <= 0) r.big_degree = 32;
  if (r.gr_interval == 0) r.gr_interval = 16;
  if (r.gr_interval < 0) r.gr_interval = 0;
  if (r.stale_rounds == 0) r.stale_rounds = 500;
  if (r.stale_rounds < 0) r.stale_rounds = 0;
  if (r.bfs_flat == 0) r.bfs_flat = 1;
  if (r.bfs_marks == 0) r.bfs_marks = -1;
  if (r.bfs_xcd == 0) r.bfs_xcd = -1;
  return r;
}

// Temporary bytes of the radix sort of P pins by vertex (keys of `bits` bits).
static hipError_t sort_temp_bytes(const Dev& g, int32_t* keys, int2* vinc, int32_t P,
                                  unsigned bits, hipStream_t s, size_t* out) {
  const auto inc = rocprim::make_transform_iterator(rocprim::counting_iterator<int32_t>(0),
                                                    IncidenceOfSlot{g.pin_net});
  unsigned long long* vinc_out = reinterpret_cast<unsigned long long*>(vinc);
  return rocprim::radix_sort_pairs(nullptr, *out, g.pin_v, keys, inc, vinc_out, (size_t)P, 0u,
                                   bits, s);
}

fp_status build_problem(fp_problem* pb, const int32_t* net_offsets, const int32_t* pins,
                        const int32_t* net_weights, const int32_t* sources, int32_t nS,
                        const int32_t* sinks, int32_t nT, int32_t mem_kind, hipStream_t s,
                        void* ext, size_t ext_bytes) {
  hipError_t he;
  const int32_t V = pb->V, E = pb->E;
  // number of pins
  int32_t P = 0;
  if (mem_kind == 0) {
    P = net_offsets[E];
  } else {
    he = hipMemcpyAsync(&P, net_offsets + E, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) return hip_fail(he, "reading net_offsets[num_nets]");
    he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "reading net_offsets[num_nets]");
  }
  if (P < 0) {
    set_error("net_offsets[num_nets] = %d is negative", P);
    return FP_ERR_INVALID;
  }
  if (P > 0 && pins == nullptr) {
    set_error("pins is NULL but the nets hold %d pins", P);
    return FP_ERR_INVALID;
  }
  const long long NB = ((long long)V + 1) & ~1ll;
  const long long N = NB + 2ll * E;
  if (N + 4 >= (1ll << 31) || 2ll * P >= (1ll << 31)) {
    set_error("network too large for 31-bit ids (V=%d E=%d P=%d)", V, E, P);
    return FP_ERR_OVERFLOW;
  }
  if (pb->opt.bottom_up_min == 0) pb->opt.bottom_up_min = (int32_t)std::max<long long>(N / 50, 1024);
  if (pb->opt.bottom_up_min < 0) pb->opt.bottom_up_min = 0;
  pb->P = P;
  pb->NB = (int32_t)NB;
  pb->N = (int32_t)N;
  pb->nS = nS;
  pb->nT = nT;

  // one device pool for the whole handle
  size_t bytes = 0;
  auto add = [&](size_t n) { bytes += align_up(n + 1); };
  add((E + 1) * 4ull);        // net_off
  add(P * 4ull);              // pin_v
  add(P * 4ull);              // pin_net
  add(E * 4ull);              // w
  add((V + 1) * 4ull);        // vtx_off
  add(P * 8ull);              // vinc
  add(V * 4ull);              // role
  add(E * 4ull);              // nflag
  add((nS + nT) * 4ull);      // terminal lists (build input copy)
  add(2ull * P * 4ull);       // fpin
  add(E * 4ull);              // fb
  add(N * 4ull);              // d
  add(N * 4ull);              // x
  add(N * 4ull);              // stamp
  add(2ull * (V + 2ull * E + N) * 4ull);  // frontier lists, two parities
  add(N * 4ull);              // cand
  add(N * 4ull);              // dx[0]
  add(N * 4ull);              // dx[1]
  add(((N + 31) / 32) * 4ull); // big-node bitmap
  add(((N + 31) / 32) * 4ull); // huge-node bitmap
  add(((N + 31) / 32) * 4ull); // labelled hint bitmap
  add(((P + 31) / 32) * 4ull); // residual bits of the pin arcs (global relabel)
  add(((E + 7) / 8) * 4ull);   // residual bits of the nets (global relabel)
  add(N);                      // reverse-BFS byte marks
  // slices of the XCD-local expanded levels (large networks only)
  const bool xcd = !ext && (pb->opt.bfs_xcd > 1 || (pb->opt.bfs_xcd == 1 && N >= (1ll << 20)));
  const long long xseg = xcd ? std::max<long long>(256, (2ll * P + 2ll * E) / 4096 + 1) : 0;
  if (xcd) {
    add((size_t)kMaxSliceGroups * kSlices * xseg * 4ull);
    add((size_t)kMaxSliceGroups * kSlices * 4ull);
  }
  add(sizeof(Ctl));           // ctl
  add(64);                    // scratch for the weight sum
  unsigned bits = 1;          // key bits of the sort of the pins by vertex
  while (bits < 31 && (1ll << bits) < (long long)V) ++bits;
  char* base = nullptr;
  size_t sort_bytes = 0;      // radix sort temporary: from the caller's memory, or allocated
  if (ext) {
    if (P) {
      Dev q{};  // only the iterator types matter for the size query
      he = sort_temp_bytes(q, nullptr, nullptr, P, bits, s, &sort_bytes);
      if (he != hipSuccess) return hip_fail(he, "sizing the pin sort");
    }
    const size_t need = bytes + align_up(sort_bytes + 1);
    if (need > ext_bytes) {
      set_error("the problem needs %zu bytes of device scratch (|V|=%d |E|=%d pins=%d); the "
                "limit is %zu bytes", need, V, E, P, ext_bytes);
      return FP_ERR_OVERFLOW;
    }
    base = static_cast<char*>(ext);
    pb->pool = nullptr;
    pb->pool_bytes = 0;
  } else {
    he = pool_acquire(pb->device, bytes, &pb->pool, &pb->pool_bytes);
    if (he != hipSuccess) {
      pb->pool = nullptr;
      set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(he));
      return FP_ERR_OOM;
    }
    base = static_cast<char*>(pb->pool);
  }
  Carve c{base};
  Dev& g = pb->dev;
  g.V = V;
  g.E = E;
  g.P = P;
  g.NB = (int32_t)NB;
  g.N = (int32_t)N;
  g.nT = nT;
  g.big_deg = pb->opt.big_degree;
  int32_t* net_off = c.take<int32_t>(E + 1);
  int32_t* pin_v = c.take<int32_t>(P);
  int32_t* w = c.take<int32_t>(E);
  int32_t* vtx_off = c.take<int32_t>(V + 1);
  int2* vinc = c.take<int2>(P);
  g.role = c.take<int32_t>(V);
  g.nflag = c.take<int32_t>(E);
  int32_t* terms = c.take<int32_t>(nS + nT);
  g.fpin = c.take<int32_t>(2ull * P);
  g.fb = c.take<int32_t>(E);
  g.d = c.take<int32_t>(N);
  g.x = c.take<int32_t>(N);
  g.stamp = c.take<int32_t>(N);
  int32_t* lists = c.take<int32_t>(2ull * (V + 2ull * E + N));
  for (int par = 0; par < 2; ++par) {
    // capacities: small vertices V, small e_in E, small e_out E, big N
    g.list[par][0] = lists;
    g.list[par][1] = lists + V;
    g.list[par][2] = lists + V + E;
    g.list[par][3] = lists + V + 2ll * E;
    lists += V + 2ll * E + N;
  }
  g.cand = c.take<int32_t>(N);
  g.dx[0] = c.take<int32_t>(N);
  g.dx[1] = c.take<int32_t>(N);
  uint32_t* bigbits = c.take<uint32_t>((N + 31) / 32);
  g.bigbits = bigbits;
  uint32_t* hugebits = c.take<uint32_t>((N + 31) / 32);
  g.hugebits = hugebits;
  g.seen = c.take<uint32_t>((N + 31) / 32);
  g.pinres = c.take<uint32_t>((P + 31) / 32);
  g.netres = c.take<uint32_t>((E + 7) / 8);
  uint8_t* lev = c.take<uint8_t>(N);
  g.lev = pb->opt.bfs_marks > 0 ? lev : nullptr;
  g.xbuf = nullptr;
  g.xcnt = nullptr;
  g.xseg = 0;
  if (xcd) {
    g.xbuf = c.take<int32_t>((size_t)kMaxSliceGroups * kSlices * xseg);
    g.xcnt = c.take<int32_t>((size_t)kMaxSliceGroups * kSlices);
    g.xseg = (int32_t)xseg;
  }
  g.bfs_flat = pb->opt.bfs_flat > 0 ? 1 : 0;
  g.relabel_block = pb->opt.relabel_blocking > 0 ? 1 : 0;
  g.bfs_arc = pb->opt.bfs_arc_parallel;
  g.ctl = c.take<Ctl>(1);
  unsigned long long* wsum = c.take<unsigned long long>(1);
  g.net_off = net_off;
  g.pin_v = pin_v;
  g.pin_net = c.take<int32_t>(P);
  g.w = w;
  g.vtx_off = vtx_off;
  g.vinc = vinc;

  const hipMemcpyKind kind = mem_kind == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  he = hipMemcpyAsync(net_off, net_offsets, (E + 1) * 4ull, kind, s);
  if (he == hipSuccess && P) he = hipMemcpyAsync(pin_v, pins, P * 4ull, kind, s);
  if (he == hipSuccess && E) he = hipMemcpyAsync(w, net_weights, E * 4ull, kind, s);
  if (he == hipSuccess) he = hipMemcpyAsync(terms, sources, nS * 4ull, kind, s);
  if (he == hipSuccess) he = hipMemcpyAsync(terms + nS, sinks, nT * 4ull, kind, s);
  if (he != hipSuccess) return hip_fail(he, "copying inputs");
  k_zero_u32<<<1, 256, 0, s>>>(reinterpret_cast<uint32_t*>(g.ctl), (long long)(sizeof(Ctl) / 4));
  k_zero_u32<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(wsum), 2);
  k_zero_u32<<<grid_for(V), 256, 0, s>>>(reinterpret_cast<uint32_t*>(g.role), V);
  if (E) k_zero_u32<<<grid_for(E), 256, 0, s>>>(reinterpret_cast<uint32_t*>(g.nflag), E);

  // validation
  if (E) k_check_nets<<<grid_for(E), 256, 0, s>>>(g, wsum);
  if (P) k_check_pins<<<grid_for(P), 256, 0, s>>>(g);
  k_roles<<<grid_for(nS + nT), 256, 0, s>>>(g, terms, nS, terms + nS, nT);
  k_role_check<<<grid_for(V), 256, 0, s>>>(g);
  int32_t err = 0;
  unsigned long long wtot = 0;
  he = hipMemcpyAsync(&err, &g.ctl->err, 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipMemcpyAsync(&wtot, wsum, 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "validating inputs");
  if (err & ERR_BUILD_OFFSETS) {
    set_error("net_offsets must start at 0 and be nondecreasing up to the pin count");
    return FP_ERR_INVALID;
  }
  if (err & ERR_BUILD_WEIGHT) {
    set_error("net weights must be >= 1");
    return FP_ERR_INVALID;
  }
  if (err & ERR_BUILD_PIN) {
    set_error("pin ids must lie in [0, num_vertices)");
    return FP_ERR_INVALID;
  }
  if (err & ERR_BUILD_TERMINAL) {
    set_error("source and sink ids must lie in [0, num_vertices)");
    return FP_ERR_INVALID;
  }
  if (err & ERR_BUILD_ST) {
    set_error("a vertex is both a source and a sink");
    return FP_ERR_INVALID;
  }
  if (wtot > 0x7fffffffull) {
    set_error("sum of net weights %llu exceeds INT32_MAX", wtot);
    return FP_ERR_OVERFLOW;
  }
  pb->wsum = (int64_t)wtot;

  // vertex incidence CSR: stable radix sort of the pins by vertex carrying
  // their {net, slot} incidence straight into vinc; the pin-flow array is
  // scratch for the sorted vertices until the first solve initialises it
  int32_t* keys = g.fpin;
  if (P) {
    k_pin_nets<<<grid_for(E), 256, 0, s>>>(g);
    const auto inc = rocprim::make_transform_iterator(rocprim::counting_iterator<int32_t>(0),
                                                      IncidenceOfSlot{g.pin_net});
    unsigned long long* vinc_out = reinterpret_cast<unsigned long long*>(vinc);
    size_t tb = 0;
    he = rocprim::radix_sort_pairs(nullptr, tb, pin_v, keys, inc, vinc_out, (size_t)P, 0u, bits,
                                   s);
    void* tmp = nullptr;
    bool owned = false;
    if (he == hipSuccess) {
      if (ext) {
        if (tb > sort_bytes) {
          set_error("internal check: the pin sort asks for %zu temporary bytes, %zu sized",
                    tb, sort_bytes);
          return FP_ERR_DEVICE;
        }
        tmp = base + bytes;
      } else {
        he = hipMallocAsync(&tmp, std::max<size_t>(tb, 1), s);
        owned = he == hipSuccess;
      }
    }
    if (he == hipSuccess)
      he = rocprim::radix_sort_pairs(tmp, tb, pin_v, keys, inc, vinc_out, (size_t)P, 0u, bits, s);
    if (owned) (void)hipFreeAsync(tmp, s);
    if (he != hipSuccess) return hip_fail(he, "sorting the pins by vertex");
  }
  k_vtx_offsets<<<grid_for((long long)P + 1), 256, 0, s>>>(keys, P, V, vtx_off);
  if (P) k_incidences<<<grid_for(P), 256, 0, s>>>(g, keys);
  k_bigbits<<<grid_for((N + 31) / 32), 256, 0, s>>>(g, bigbits, hugebits);
  he = hipMemcpyAsync(&err, &g.ctl->err, 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he == hipSuccess) he = hipGetLastError();
  if (he != hipSuccess) return hip_fail(he, "building incidences");
  if (err & ERR_BUILD_DUP) {
    set_error("a vertex appears twice in one net");
    return FP_ERR_INVALID;
  }
  if (ext) {  // the caller provides the host mirror of the control block
    memset(pb->ctl_h, 0, sizeof(Ctl));
    return FP_OK;
  }
  he = ctl_acquire(&pb->ctl_h);
  if (he != hipSuccess) {
    pb->ctl_h = nullptr;
    return hip_fail(he, "allocating the pinned control block");
  }
  memset(pb->ctl_h, 0, sizeof(Ctl));
  return FP_OK;
}

// pin state {r_in, f_out} -> separate flow arrays; labels / excess without
// the padding node between vertices and nets
__global__ void k_export(Dev g, int32_t* f_in, int32_t* f_out, int32_t* lab, int32_t* exc) {
  const int n = max(g.P, g.V + 2 * g.E);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < g.P) {
      const int2 ep = g.vinc[i];
      f_in[ep.y] = g.w[ep.x] - g.fpin[2 * ep.y];
      f_out[ep.y] = g.fpin[2 * ep.y + 1];
    }
    if (i < g.V + 2 * g.E) {
      const int src = i < g.V ? i : i - g.V + g.NB;
      lab[i] = g.d[src];
      exc[i] = g.x[src] + g.dx[0][src] + g.dx[1][src];
    }
  }
}

fp_status export_state(fp_problem* pb, hipStream_t s, int32_t* f_in, int32_t* f_out,
                       int32_t* f_b, int32_t* labels, int32_t* excess) {
  if (!pb->inited) {
    set_error("no flow state before the first solve");
    return FP_ERR_STATE;
  }
  Dev& g = pb->dev;
  const size_t P = g.P, M = (size_t)g.V + 2ull * g.E;
  int32_t* tmp = nullptr;
  hipError_t he = hipMalloc(&tmp, (2 * P + 2 * M + 2) * sizeof(int32_t));
  if (he != hipSuccess) return hip_fail(he, "export buffer");
  int32_t *dfi = tmp, *dfo = tmp + P, *dl = tmp + 2 * P, *dx = tmp + 2 * P + M;
  k_export<<<grid_for((long long)std::max(P, M)), 256, 0, s>>>(g, dfi, dfo, dl, dx);
  he = hipGetLastError();
  if (he == hipSuccess && f_in && P) he = hipMemcpyAsync(f_in, dfi, P * 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && f_out && P) he = hipMemcpyAsync(f_out, dfo, P * 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && f_b && g.E) he = hipMemcpyAsync(f_b, g.fb, g.E * 4ull, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && labels) he = hipMemcpyAsync(labels, dl, M * 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && excess) he = hipMemcpyAsync(excess, dx, M * 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  hipFree(tmp);
  if (he != hipSuccess) return hip_fail(he, "exporting state");
  return FP_OK;
}

void release_problem(fp_problem* pb) {
  if (!pb) return;
  for (auto& t : pb->pending) {  // recorded work has finished or is dropped with the handle
    event_pool_put(pb->device, t.a);
    event_pool_put(pb->device, t.b);
  }
  pb->pending.clear();
  pool_release(pb->device, pb->pool, pb->pool_bytes);
  if (pb->cw) hipFree(pb->cw);
  if (pb->fc_mem) hipFree(pb->fc_mem);
  pb->fc_mem = nullptr;
  ctl_release(pb->ctl_h);
  pb->pool = nullptr;
  pb->cw = nullptr;
  pb->ctl_h = nullptr;
}

}  // namespace hf
