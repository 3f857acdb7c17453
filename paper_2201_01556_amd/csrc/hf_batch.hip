// Batched solve of many independent flow problems (the paper's refinement
// runs many block-pair flow problems at once, section "Parallel Active Block
// Scheduling").  Two schedules, both with the single-problem device phases:
//   union    the kept problems are copied into one network, their disjoint
//            union, solved once with the device-wide kernels: one global
//            relabel is one BFS over every problem, one round discharges all
//            of their frontiers (the default, and the tuner's choice on
//            large batches);
//   workers  host workers take problems from a shared queue, largest first,
//            and drive the single-problem path on HIP streams of their own,
//            so the kernels and host round trips of different problems
//            overlap.
// Results are identical.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hf_host.h"

struct fp_batch {
  int device = 0;
  int32_t count = 0;
  std::vector<fp_problem*> pbs;
  std::vector<int32_t> order;
  fp_batch_config cfg{};
  bool has_vs = false;
  bool has_ns = false;
  void* dmem = nullptr;  // device: the problems' layouts and side pointers
  hf::Dev* devs_d = nullptr;
  uint8_t** vs_d = nullptr;
  uint8_t** ns_d = nullptr;
  void* hmem = nullptr;  // pinned: devs_h
  hf::Dev* devs_h = nullptr;
  std::vector<hipStream_t> workers;  // streams of the workers schedule
  void* umem = nullptr;              // scratch of the union schedule
  size_t umem_bytes = 0;
  // workgroups schedule: [queue counter][order][skip flags][results] on the
  // device, the results' pinned host copy, the captured launch and the
  // stream it is captured on, with the arguments it was captured with
  void* wmem = nullptr;
  void* wres_h = nullptr;
  hipStream_t wg_stream = nullptr;
  hipGraph_t wg_graph = nullptr;
  hipGraphExec_t wg_exec = nullptr;
  int32_t wg_key[8] = {};
};

namespace hf {

constexpr int32_t kScheduleUnion = 1;
constexpr int32_t kScheduleWorkers = 2;
constexpr int32_t kScheduleWorkgroups = 3;

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static fp_batch_config resolve_batch_config(const fp_batch_config* c) {
  fp_batch_config r{};
  if (c) r = *c;
  if (r.schedule == 0) r.schedule = kScheduleUnion;
  if (r.group_lanes == 0) r.group_lanes = 8;
  if (r.gr_interval == 0 && r.schedule == kScheduleUnion) r.gr_interval = 8;
  // one workgroup per problem: relabel every 16 rounds (512 problems of 2,000
  // vertices: 11.9 ms against 14.9 at 64; the 500 block pairs: 74 against 103)
  if (r.gr_interval == 0 && r.schedule == kScheduleWorkgroups) r.gr_interval = 16;
  if (r.streams == 0) r.streams = 4;
  if (r.wg_threads == 0) r.wg_threads = 1024;
  return r;
}

static bool batch_config_valid(const fp_batch_config& c) {
  return (c.group_lanes == 4 || c.group_lanes == 8 || c.group_lanes == 16) &&
         c.gr_interval >= -1 && c.streams >= 1 && c.streams <= 64 &&
         (c.schedule == kScheduleUnion || c.schedule == kScheduleWorkers ||
          c.schedule == kScheduleWorkgroups) &&
         c.union_pins >= 0 && (c.wg_threads == 256 || c.wg_threads == 1024) &&
         c.reserved0 == 0 && c.reserved1 == 0;
}

bool batch_config_ok(const fp_batch_config* c) {
  return batch_config_valid(resolve_batch_config(c));
}

void release_batch(fp_batch* b) {
  for (hipStream_t w : b->workers) (void)hipStreamDestroy(w);
  b->workers.clear();
  if (b->wg_exec) (void)hipGraphExecDestroy(b->wg_exec);
  if (b->wg_graph) (void)hipGraphDestroy(b->wg_graph);
  if (b->wg_stream) (void)hipStreamDestroy(b->wg_stream);
  if (b->wmem) (void)hipFree(b->wmem);
  if (b->wres_h) (void)hipHostFree(b->wres_h);
  b->wg_exec = nullptr;
  b->wg_graph = nullptr;
  b->wg_stream = nullptr;
  b->wmem = b->wres_h = nullptr;
  if (b->dmem) (void)hipFree(b->dmem);
  if (b->hmem) (void)hipHostFree(b->hmem);
  if (b->umem) (void)hipFree(b->umem);
  b->dmem = b->hmem = b->umem = nullptr;
  b->umem_bytes = 0;
}

fp_status create_batch(fp_problem* const* pbs, int32_t count, uint8_t* const* vsides,
                       uint8_t* const* nsides, const fp_batch_config* config, hipStream_t s,
                       fp_batch** out) {
  fp_batch* b = new (std::nothrow) fp_batch();
  if (!b) {
    set_error("host allocation failed");
    return FP_ERR_OOM;
  }
  hipGetDevice(&b->device);
  b->count = count;
  b->pbs.assign(pbs, pbs + count);
  b->cfg = resolve_batch_config(config);
  b->has_vs = vsides != nullptr;
  b->has_ns = nsides != nullptr;
  // largest problems first (pins + network nodes), ties by index
  b->order.resize(count);
  for (int32_t i = 0; i < count; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t a, int32_t c) {
    const long long wa = (long long)pbs[a]->P + pbs[a]->N;
    const long long wc = (long long)pbs[c]->P + pbs[c]->N;
    return wa > wc;
  });
  const size_t n = count > 0 ? (size_t)count : 1;
  size_t off = 0;
  const size_t o_devs = off;
  off = align_up(off + n * sizeof(Dev));
  const size_t o_vs = off;
  off = align_up(off + n * sizeof(uint8_t*));
  const size_t o_ns = off;
  off = align_up(off + n * sizeof(uint8_t*));
  hipError_t he = hipMalloc(&b->dmem, off);
  if (he != hipSuccess) {
    fp_status st = hip_fail(he, "allocating the batch plan");
    delete b;
    return st;
  }
  char* d = static_cast<char*>(b->dmem);
  b->devs_d = reinterpret_cast<Dev*>(d + o_devs);
  b->vs_d = reinterpret_cast<uint8_t**>(d + o_vs);
  b->ns_d = reinterpret_cast<uint8_t**>(d + o_ns);
  he = hipHostMalloc(&b->hmem, n * sizeof(Dev), hipHostMallocDefault);
  if (he == hipSuccess) {
    b->devs_h = static_cast<Dev*>(b->hmem);
    std::memset(b->hmem, 0, n * sizeof(Dev));
  }
  if (he == hipSuccess && vsides)
    he = hipMemcpyAsync(b->vs_d, vsides, (size_t)count * sizeof(uint8_t*), hipMemcpyHostToDevice,
                        s);
  if (he == hipSuccess && nsides)
    he = hipMemcpyAsync(b->ns_d, nsides, (size_t)count * sizeof(uint8_t*), hipMemcpyHostToDevice,
                        s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    fp_status st = hip_fail(he, "setting up the batch plan");
    release_batch(b);
    delete b;
    return st;
  }
  *out = b;
  return FP_OK;
}

// Workers schedule: `force_init` starts every problem from the zero flow
// (tuning).  Problems spread over `streams` workers, each a host thread driving the
// single-problem path on its own stream; problems are taken from a shared
// counter in the plan's order (largest first).  The batch configuration's
// lanes per node and relabel interval apply to every problem for the run.
static fp_status batch_concurrent(fp_batch* b, const uint8_t* skip, int32_t with_cut,
                                  bool force_init, hipStream_t s, int64_t* flows, float* ms) {
  const int nw = std::max(1, std::min<int>(b->cfg.streams, b->count));
  while ((int)b->workers.size() < nw) {
    hipStream_t w = nullptr;
    hipError_t he = hipStreamCreateWithFlags(&w, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_fail(he, "creating a batch stream");
    b->workers.push_back(w);
  }
  std::vector<uint8_t*> vs, ns;
  if (with_cut) {
    vs.resize(b->count);
    ns.resize(b->count);
    hipError_t he = hipMemcpy(vs.data(), b->vs_d, (size_t)b->count * sizeof(uint8_t*),
                              hipMemcpyDeviceToHost);
    if (he == hipSuccess && b->has_ns)
      he = hipMemcpy(ns.data(), b->ns_d, (size_t)b->count * sizeof(uint8_t*),
                     hipMemcpyDeviceToHost);
    if (he != hipSuccess) return hip_fail(he, "reading the batch side pointers");
  }
  // work queued on the caller's stream comes first
  hipEvent_t ready = nullptr;
  hipError_t he = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
  if (he == hipSuccess) he = hipEventRecord(ready, s);
  for (int w = 0; w < nw && he == hipSuccess; ++w) he = hipStreamWaitEvent(b->workers[w], ready, 0);
  if (he != hipSuccess) {
    if (ready) (void)hipEventDestroy(ready);
    return hip_fail(he, "ordering the batch after the caller's stream");
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::atomic<int32_t> next{0};
  std::atomic<bool> stop{false};
  std::mutex mu;
  fp_status first = FP_OK;
  std::string first_msg;
  const fp_batch_config cfg = b->cfg;
  auto worker = [&](int w) {
    (void)hipSetDevice(b->device);
    hipStream_t ws = b->workers[w];
    for (;;) {
      if (stop.load()) return;
      const int32_t k = next.fetch_add(1);
      if (k >= b->count) return;
      const int32_t i = b->order[k];
      if (skip && skip[i]) {
        if (flows) flows[i] = -1;
        continue;
      }
      fp_problem* pb = b->pbs[i];
      if (force_init) {
        pb->inited = false;
        pb->solved = false;
        pb->labels_exact = false;
      }
      const fp_options saved = pb->opt;
      pb->opt.group_lanes = cfg.group_lanes;
      if (cfg.gr_interval != 0) pb->opt.gr_interval = cfg.gr_interval;
      int64_t f = -1;
      fp_status st = solve_problem(pb, ws, &f);
      if (st == FP_OK && with_cut) st = cut_problem(pb, ws, 1, vs[i], b->has_ns ? ns[i] : nullptr);
      pb->opt = saved;
      if (flows) flows[i] = st == FP_OK ? f : -1;
      if (st != FP_OK) {
        std::lock_guard<std::mutex> lock(mu);
        if (first == FP_OK || (st == FP_ERR_DEVICE && first != FP_ERR_DEVICE)) {
          first = st;
          first_msg = std::string("problem ") + std::to_string(i) + ": " + fp_last_error();
        }
        if (st == FP_ERR_DEVICE) stop.store(true);  // the device state is not usable
      }
    }
  };
  if (nw == 1) {
    worker(0);
  } else {
    std::vector<std::thread> pool;
    pool.reserve(nw);
    for (int w = 0; w < nw; ++w) pool.emplace_back(worker, w);
    for (auto& t : pool) t.join();
  }
  (void)hipEventDestroy(ready);
  if (ms)
    *ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (first != FP_OK) set_error("%s", first_msg.c_str());
  return first;
}


// ---------------------------------------------------------------------------
// union schedule: the kept problems as one network
//
// The problems are independent, so their disjoint union is one flow network
// (the sources and sinks of all problems together).  A maximum preflow of the
// union restricted to a problem is a maximum preflow of that problem, and the
// minimal minimum cut of the union is the union of the problems' minimal
// minimum cuts, since the cut weight is a sum over the components.  One solve
// of the union therefore runs every problem in the same device-wide kernels:
// a global relabel is one reverse BFS over all problems and a round
// discharges all their frontiers.  A problem's flow value is the weight of
// its nets cut by the minimal source side (maximum flow equals minimum cut);
// their sum must equal the union's flow value.
// ---------------------------------------------------------------------------

struct UnionMap {
  const int32_t* ids;   // [n] problem index of each kept problem
  const int32_t* voff;  // [n+1] first union vertex of each kept problem
  const int32_t* eoff;  // [n+1] first union net
  const int32_t* poff;  // [n+1] first union pin slot
  int32_t n;
};

// kept problem owning union element x: the largest i < n with off[i] <= x
// (off[n] is the total, above x)
__device__ __forceinline__ int union_part(const int32_t* off, int n, int x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_union_nets(const Dev* devs, UnionMap m, int32_t E,
                                                    int32_t* net_off, int32_t* w) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, ts = gridDim.x * blockDim.x;
  for (int e = t0; e < E; e += ts) {
    const int i = union_part(m.eoff, m.n, e);
    const Dev& d = devs[m.ids[i]];
    const int le = e - m.eoff[i];
    net_off[e] = m.poff[i] + d.net_off[le];
    w[e] = d.w[le];
  }
  if (t0 == 0) net_off[E] = m.poff[m.n];
}

__global__ void __launch_bounds__(256) k_union_pins(const Dev* devs, UnionMap m, int32_t P,
                                                    int32_t* pins) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, ts = gridDim.x * blockDim.x;
  for (int p = t0; p < P; p += ts) {
    const int i = union_part(m.poff, m.n, p);
    pins[p] = m.voff[i] + devs[m.ids[i]].pin_v[p - m.poff[i]];
  }
}

// Terminal lists of the union from the problems' current roles (piercing
// included); list order does not matter.
__global__ void __launch_bounds__(256) k_union_terminals(const Dev* devs, UnionMap m, int32_t V,
                                                         int32_t* src, int32_t* snk,
                                                         int32_t* counts) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, ts = gridDim.x * blockDim.x;
  for (int v = t0; v < V; v += ts) {
    const int i = union_part(m.voff, m.n, v);
    const int r = devs[m.ids[i]].role[v - m.voff[i]];
    if (r == 1) src[atomicAdd(&counts[0], 1)] = v;
    else if (r == 2) snk[atomicAdd(&counts[1], 1)] = v;
  }
}

// Flow value of kept problem blockIdx.x: weight of its nets with e_in on the
// source side and e_out not (bit0 set, bit1 clear).
__global__ void __launch_bounds__(256) k_union_flows(UnionMap m, const int32_t* w,
                                                     const uint8_t* nside,
                                                     unsigned long long* flows) {
  const int i = blockIdx.x;
  unsigned long long sum = 0ull;
  for (int e = m.eoff[i] + threadIdx.x; e < m.eoff[i + 1]; e += blockDim.x)
    if ((nside[e] & 3u) == 1u) sum += (unsigned long long)w[e];
  block_add_u64(&flows[i], sum);
}

// Scatter the union's sides into the problems' side buffers.
__global__ void __launch_bounds__(256) k_union_sides(UnionMap m, int32_t V, int32_t E,
                                                     const uint8_t* vside, const uint8_t* nside,
                                                     uint8_t* const* vs, uint8_t* const* ns) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, ts = gridDim.x * blockDim.x;
  for (int v = t0; v < V; v += ts) {
    const int i = union_part(m.voff, m.n, v);
    vs[m.ids[i]][v - m.voff[i]] = vside[v];
  }
  if (ns == nullptr) return;
  for (int e = t0; e < E; e += ts) {
    const int i = union_part(m.eoff, m.n, e);
    uint8_t* dst = ns[m.ids[i]];
    if (dst) dst[e - m.eoff[i]] = nside[e];
  }
}

static int union_grid(long long n) {
  const long long b = (n + 255) / 256;
  return (int)std::max<long long>(1, std::min<long long>(b, 8192));
}

// Solve the kept problems as one network.  The problems' own handles are not
// touched: every run starts from the zero flow of each problem's current
// terminals, which gives the same flow values and minimal source sides as a
// warm start would.
// One union of the problems `ids` (index order).
static fp_status union_chunk(fp_batch* b, const std::vector<int32_t>& ids, int32_t with_cut,
                             hipStream_t s, int64_t* flows) {
  std::vector<int32_t> voff(1, 0), eoff(1, 0), poff(1, 0);
  long long V = 0, E = 0, P = 0;
  for (int32_t i : ids) {
    const fp_problem* pb = b->pbs[i];
    V += pb->V;
    E += pb->E;
    P += pb->P;
    voff.push_back((int32_t)V);
    eoff.push_back((int32_t)E);
    poff.push_back((int32_t)P);
  }
  const int32_t n = (int32_t)ids.size();
  // scratch: map, union inputs, terminal lists, sides, flows
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t o_ids = carve((size_t)n * 4);
  const size_t o_voff = carve((size_t)(n + 1) * 4);
  const size_t o_eoff = carve((size_t)(n + 1) * 4);
  const size_t o_poff = carve((size_t)(n + 1) * 4);
  const size_t o_noff = carve((size_t)(E + 1) * 4);
  const size_t o_w = carve((size_t)E * 4 + 4);
  const size_t o_pins = carve((size_t)P * 4 + 4);
  const size_t o_src = carve((size_t)V * 4);
  const size_t o_snk = carve((size_t)V * 4);
  const size_t o_cnt = carve(8);
  const size_t o_flows = carve((size_t)n * 8);
  const size_t o_vs = carve((size_t)V);
  const size_t o_ns = carve((size_t)E + 1);
  hipError_t he = hipSuccess;
  if (off > b->umem_bytes) {
    if (b->umem) (void)hipFree(b->umem);
    b->umem = nullptr;
    b->umem_bytes = 0;
    he = hipMalloc(&b->umem, off);
    if (he != hipSuccess) {
      b->umem = nullptr;
      return hip_fail(he, "allocating the union scratch");
    }
    b->umem_bytes = off;
  }
  char* d = static_cast<char*>(b->umem);
  UnionMap m;
  m.ids = reinterpret_cast<const int32_t*>(d + o_ids);
  m.voff = reinterpret_cast<const int32_t*>(d + o_voff);
  m.eoff = reinterpret_cast<const int32_t*>(d + o_eoff);
  m.poff = reinterpret_cast<const int32_t*>(d + o_poff);
  m.n = n;
  int32_t* noff_u = reinterpret_cast<int32_t*>(d + o_noff);
  int32_t* w_u = reinterpret_cast<int32_t*>(d + o_w);
  int32_t* pins_u = reinterpret_cast<int32_t*>(d + o_pins);
  int32_t* src = reinterpret_cast<int32_t*>(d + o_src);
  int32_t* snk = reinterpret_cast<int32_t*>(d + o_snk);
  int32_t* cnt = reinterpret_cast<int32_t*>(d + o_cnt);
  unsigned long long* flows_d = reinterpret_cast<unsigned long long*>(d + o_flows);
  uint8_t* vs_u = reinterpret_cast<uint8_t*>(d + o_vs);
  uint8_t* ns_u = reinterpret_cast<uint8_t*>(d + o_ns);
  for (int32_t i = 0; i < b->count; ++i) b->devs_h[i] = b->pbs[i]->dev;
  he = hipMemcpyAsync(b->devs_d, b->devs_h, (size_t)b->count * sizeof(Dev), hipMemcpyHostToDevice,
                      s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(d + o_ids, ids.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(d + o_voff, voff.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(d + o_eoff, eoff.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(d + o_poff, poff.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemsetAsync(cnt, 0, 8, s);
  if (he == hipSuccess) he = hipMemsetAsync(flows_d, 0, (size_t)n * 8, s);
  if (he != hipSuccess) return hip_fail(he, "staging the union map");
  k_union_nets<<<union_grid(E + 1), 256, 0, s>>>(b->devs_d, m, (int32_t)E, noff_u, w_u);
  if (P) k_union_pins<<<union_grid(P), 256, 0, s>>>(b->devs_d, m, (int32_t)P, pins_u);
  k_union_terminals<<<union_grid(V), 256, 0, s>>>(b->devs_d, m, (int32_t)V, src, snk, cnt);
  int32_t counts[2] = {0, 0};
  he = hipGetLastError();
  if (he == hipSuccess) he = hipMemcpyAsync(counts, cnt, 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);  // the host vectors are read until here
  if (he != hipSuccess) return hip_fail(he, "building the union network");
  fp_problem* u = new (std::nothrow) fp_problem();
  if (!u) {
    set_error("host allocation failed");
    return FP_ERR_OOM;
  }
  u->device = b->device;
  u->V = (int32_t)V;
  u->E = (int32_t)E;
  fp_options o{};
  o.group_lanes = b->cfg.group_lanes;
  o.gr_interval = b->cfg.gr_interval;
  u->opt = resolve_options(&o);
  fp_status st = FP_OK;
  if (counts[0] < 1 || counts[1] < 1) {
    set_error("the kept problems hold %d sources and %d sinks", counts[0], counts[1]);
    st = FP_ERR_INVALID;
  }
  if (st == FP_OK) st = build_problem(u, noff_u, pins_u, w_u, src, counts[0], snk, counts[1], 1, s);
  int64_t F = 0;
  if (st == FP_OK) st = solve_problem(u, s, &F);
  if (st == FP_OK) st = cut_problem(u, s, 1, vs_u, ns_u);
  std::vector<unsigned long long> fh(n, 0ull);
  if (st == FP_OK) {
    k_union_flows<<<n, 256, 0, s>>>(m, u->dev.w, ns_u, flows_d);
    if (with_cut)
      k_union_sides<<<union_grid(std::max(V, E)), 256, 0, s>>>(
          m, (int32_t)V, (int32_t)E, vs_u, ns_u, b->vs_d, b->has_ns ? b->ns_d : nullptr);
    he = hipGetLastError();
    if (he == hipSuccess)
      he = hipMemcpyAsync(fh.data(), flows_d, (size_t)n * 8, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) st = hip_fail(he, "splitting the union's flow");
  }
  if (st != FP_OK) {
    (void)hipStreamSynchronize(s);
    release_problem(u);
    delete u;
    return st;
  }
  release_problem(u);
  delete u;
  unsigned long long total = 0ull;
  for (int32_t k = 0; k < n; ++k) total += fh[k];
  if ((int64_t)total != F) {
    set_error("internal check: the problems' cut weights sum to %llu, the union's flow is %lld",
              total, (long long)F);
    return FP_ERR_DEVICE;
  }
  if (flows)
    for (int32_t k = 0; k < n; ++k) flows[ids[k]] = (int64_t)fh[k];
  return FP_OK;
}

// ---------------------------------------------------------------------------
// workgroups schedule: one persistent launch, a workgroup per problem
//
// Each workgroup takes the next problem of the plan's order (largest first)
// from a device counter and solves it alone with the single-problem phases
// in their one-workgroup form: init (zero flow of the current terminals), a
// global relabel (reverse BFS whose levels claim, then the gather of the
// active nodes), discharge rounds with the host loop's relabel triggers
// (relabel work, interval, stale flow), the terminating relabel that
// confirms an empty frontier (paper, section "A Bug in the Synchronous
// Algorithm"), and on request the source side.  The waves of a workgroup
// share one CU, so workgroup barriers order their memory traffic and no
// device-wide synchronisation is needed; a problem costs no launches and no
// host round trips of its own (the paper's many small flow problems at once,
// section "Parallel Active Block Scheduling", paragraph "Parallelization").
// The launch is replayed from a captured HIP graph.
// ---------------------------------------------------------------------------

constexpr long long kWgRoundGuard = 1000000ll;  // rounds per solve before giving up
constexpr int kWgStaleFrontier = 1500;  // "only few active nodes" (paragraph "Avoid Pushing Flow Back")

struct WgParams {
  int32_t count;        // problems in the plan
  int32_t epoch0;       // first stamp value of every solve (init clears the stamps)
  int32_t gr_interval;  // rounds between global relabels; <= 0 off
  int32_t stale_limit;  // rounds without a flow change (few active nodes); <= 0 off
  int32_t relabel_x16;  // relabel work between global relabels: N * x / 16 relabels
  int32_t with_cut;     // also write the minimal source side
};

struct WgResult {
  unsigned long long flow;
  long long rounds;
  int32_t epoch;  // first stamp value not used by the solve
  int32_t err;    // the problem's error flags
  int32_t global_relabels;
  int32_t restarts;
};

// Global relabel inside one workgroup: exact labels by the reverse BFS of
// the capped network (levels claim their nodes), then the active nodes
// gathered as round `epoch`'s frontier.  False (flagged ERR_GUARD) when a
// level breaks the bounds of a BFS.  Block-uniform.
__device__ bool wg_global_relabel(const Dev& g, int epoch, lds_int* lds) {
  phase_gr_reset(g, 0, 1, lds);
  __syncthreads();
  bool ok = true;
  for (int level = 0;; ++level) {
    const int nf = count_all_vol(g.ctl->bcnt[level % 3]);
    if (nf == 0) break;
    if (nf > g.N || level > g.N) {  // a level holds distinct nodes; at most N levels
      ok = false;
      break;
    }
    __syncthreads();  // every wave has read the count before the level changes it
    phase_bfs_rev_lb<true>(g, level, 0, 1, KC_LOOP_BFS, lds);
    __syncthreads();
  }
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(&g.ctl->err, ERR_GUARD);
    __syncthreads();
    return false;
  }
  phase_gather(g, epoch, 0, 1, lds);
  __syncthreads();
  return true;
}

// Source side inside one workgroup: seeds, forward BFS levels of the
// uncapped network, the bitmaps.  Block-uniform.
__device__ void wg_cut(const Dev& g, int ep, uint8_t* vs, uint8_t* ns, lds_int* lds) {
  phase_cut_seed(g, ep, false, 0, 1, lds);
  __syncthreads();
  for (int level = 0;; ++level) {
    const int nf = count_all_vol(g.ctl->bcnt[level % 3]);
    if (nf == 0) break;
    if (nf > g.N || level > g.N) {
      if (threadIdx.x == 0) atomicOr(&g.ctl->err, ERR_GUARD);
      break;
    }
    __syncthreads();
    phase_bfs_fwd_lb<true>(g, level, ep, 0, 0, 1, KC_LOOP_BFS, lds);
    __syncthreads();
  }
  __syncthreads();
  phase_cut_out(g, ep, vs, ns, threadIdx.x, blockDim.x);
  __syncthreads();
}

// One problem, start to end, in one workgroup (the host loop of
// solve_impl moved on the device).  Every decision reads counters after a
// barrier that no wave passes before the next phase, so it is block-uniform.
template <int G>
__device__ void wg_solve(const Dev& g, const WgParams& p, uint8_t* vs, uint8_t* ns,
                         lds_int* lds, WgResult* out) {
  phase_init(g, threadIdx.x, blockDim.x);
  __syncthreads();
  int epoch = p.epoch0;
  int ngr = 1, restarts = 0;
  long long rounds = 0;
  bool ok = wg_global_relabel(g, epoch, lds);
  const unsigned long long budget =
      (unsigned long long)g.N * (unsigned long long)p.relabel_x16 / 16ull + 1ull;
  unsigned long long rel_at = ld_vol64(&g.ctl->relabels);
  unsigned long long last_flow = ld_vol64(&g.ctl->flow);
  int since = 0, stale = 0;
  bool fresh = true;  // the frontier was just gathered by a global relabel
  while (ok) {
    const int nf = count_all_vol(g.ctl->fcnt[epoch % 3]);
    if (ld_vol(&g.ctl->err) & ERR_LABEL) break;
    bool gr = false;
    if (nf == 0) {
      if (fresh) break;
      gr = true;  // apparent termination: confirm with exact labels
    } else {
      if (rounds >= kWgRoundGuard) {
        __syncthreads();
        if (threadIdx.x == 0) atomicOr(&g.ctl->err, ERR_GUARD);
        ok = false;
        break;
      }
      fresh = false;
      __syncthreads();  // every wave has read the counters before they change
      phase_push<G>(g, epoch, 0, 1, KC_LOOP_ROUNDS, lds);
      __syncthreads();
      phase_apply(g, epoch, 0, 1, KC_LOOP_ROUNDS, lds);
      __syncthreads();
      ++epoch;
      ++rounds;
      ++since;
      const unsigned long long fl = ld_vol64(&g.ctl->flow);
      if (fl != last_flow) {
        last_flow = fl;
        stale = 0;
      } else if (nf < kWgStaleFrontier) {
        ++stale;
      } else {
        stale = 0;
      }
      if (ld_vol64(&g.ctl->relabels) - rel_at >= budget) gr = true;
      if (p.gr_interval > 0 && since >= p.gr_interval) gr = true;
      if (p.stale_limit > 0 && stale >= p.stale_limit) gr = true;
    }
    if (gr) {
      __syncthreads();  // every wave has read the counters before the relabel changes them
      ok = wg_global_relabel(g, epoch, lds);
      ++ngr;
      if (ok && nf == 0 && count_all_vol(g.ctl->fcnt[epoch % 3]) > 0) ++restarts;
      rel_at = ld_vol64(&g.ctl->relabels);
      last_flow = ld_vol64(&g.ctl->flow);
      since = 0;
      stale = 0;
      fresh = true;
    }
  }
  __syncthreads();
  if (ok && p.with_cut && vs != nullptr && !(ld_vol(&g.ctl->err) & ERR_LABEL)) {
    const int ep = epoch++;
    wg_cut(g, ep, vs, ns, lds);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out->flow = ld_vol64(&g.ctl->flow);
    out->rounds = rounds;
    out->epoch = epoch;
    out->err = ld_vol(&g.ctl->err);
    out->global_relabels = ngr;
    out->restarts = restarts;
  }
  __syncthreads();
}

// The persistent launch: workgroups take problems from the counter `next`
// until every problem of the order is taken.  Skipped problems are passed
// over and keep their result slot.
template <int G, int B>
__global__ void __launch_bounds__(B) k_batch_wg(const Dev* devs, const int32_t* order,
                                                         const uint8_t* skip,
                                                         uint8_t* const* vs_ptrs,
                                                         uint8_t* const* ns_ptrs, int32_t* next,
                                                         WgParams p, WgResult* res) {
  __shared__ int32_t bq[lds_words(B)];
  lds_int* const lds = (lds_int*)bq;
  __shared__ int32_t slot;
  for (;;) {
    if (threadIdx.x == 0) slot = atomicAdd(next, 1);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(slot);
    __syncthreads();  // every wave has read the slot before it is written again
    if (k >= p.count) break;
    const int i = __builtin_amdgcn_readfirstlane(order[k]);
    if (skip[i]) continue;
    uint8_t* vs = p.with_cut ? vs_ptrs[i] : nullptr;
    uint8_t* ns = p.with_cut && ns_ptrs ? ns_ptrs[i] : nullptr;
    // the layout is read where it lies (uniform address): a private copy
    // would be indexed dynamically (list slots) and live in scratch
    const Dev& g = devs[i];
    wg_solve<G>(g, p, vs, ns, lds, res + i);
  }
}

__global__ void k_wg_reset(int32_t* next) {
  if (threadIdx.x == 0) *next = 0;
}

// Rounds between global relabels inside one workgroup (the resolved
// configuration's; -1 turns them off).
static int32_t wg_interval(const fp_batch* b) {
  return b->cfg.gr_interval < 0 ? 0 : b->cfg.gr_interval;
}

template <int G, int B>
static int wg_grid_for(const fp_batch* b) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_batch_wg<G, B>), B, 0) != hipSuccess)
    per_cu = 1;
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, b->device);
  const long long grid = (long long)std::max(1, per_cu) * std::max(1, prop.multiProcessorCount);
  return (int)std::max(1ll, std::min<long long>(grid, b->count));
}

template <int G, int B>
static hipError_t wg_capture(fp_batch* b, int grid, const WgParams& p, int32_t* next,
                             const int32_t* order, const uint8_t* skip_d, WgResult* res_d) {
  hipStream_t ws = b->wg_stream;
  hipError_t he = hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) return he;
  k_wg_reset<<<1, 64, 0, ws>>>(next);
  k_batch_wg<G, B><<<grid, B, 0, ws>>>(b->devs_d, order, skip_d, b->vs_d,
                                       b->has_ns ? b->ns_d : nullptr, next, p, res_d);
  hipGraph_t graph = nullptr;
  const hipError_t launch = hipGetLastError();
  he = hipStreamEndCapture(ws, &graph);
  if (launch != hipSuccess) he = launch;
  if (he == hipSuccess) he = hipGraphInstantiate(&b->wg_exec, graph, nullptr, nullptr, 0);
  if (he == hipSuccess) b->wg_graph = graph;
  else if (graph) (void)hipGraphDestroy(graph);
  return he;
}

// Workgroups schedule: every kept problem solved from the zero flow of its
// current terminals inside one workgroup of one persistent launch; every
// solved handle then behaves as after maxflow_solve.
static fp_status batch_workgroups(fp_batch* b, const uint8_t* skip, int32_t with_cut,
                                  hipStream_t s, int64_t* flows, float* ms) {
  const auto t0 = std::chrono::steady_clock::now();
  const int32_t n = b->count;
  const size_t o_next = 0;
  const size_t o_order = align_up(o_next + 4);
  const size_t o_skip = align_up(o_order + (size_t)n * 4);
  const size_t o_res = align_up(o_skip + (size_t)n);
  const size_t bytes = align_up(o_res + (size_t)n * sizeof(WgResult));
  hipError_t he = hipSuccess;
  if (!b->wmem) {
    he = hipMalloc(&b->wmem, bytes);
    if (he == hipSuccess) he = hipHostMalloc(&b->wres_h, (size_t)n * sizeof(WgResult),
                                             hipHostMallocDefault);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&b->wg_stream, hipStreamNonBlocking);
    if (he == hipSuccess)
      he = hipMemcpyAsync(static_cast<char*>(b->wmem) + o_order, b->order.data(),
                          (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (he != hipSuccess) return hip_fail(he, "allocating the workgroups schedule");
  }
  char* d = static_cast<char*>(b->wmem);
  int32_t* next = reinterpret_cast<int32_t*>(d + o_next);
  const int32_t* order = reinterpret_cast<const int32_t*>(d + o_order);
  uint8_t* skip_d = reinterpret_cast<uint8_t*>(d + o_skip);
  WgResult* res_d = reinterpret_cast<WgResult*>(d + o_res);
  WgResult* res_h = static_cast<WgResult*>(b->wres_h);
  for (int32_t i = 0; i < n; ++i) b->devs_h[i] = b->pbs[i]->dev;
  he = hipMemcpyAsync(b->devs_d, b->devs_h, (size_t)n * sizeof(Dev), hipMemcpyHostToDevice, s);
  if (he == hipSuccess) {
    if (skip) he = hipMemcpyAsync(skip_d, skip, (size_t)n, hipMemcpyHostToDevice, s);
    else he = hipMemsetAsync(skip_d, 0, (size_t)n, s);
  }
  if (he != hipSuccess) return hip_fail(he, "staging the workgroups schedule");
  const fp_options& o = b->pbs[0]->opt;
  WgParams p{};
  p.count = n;
  p.epoch0 = 1;
  p.gr_interval = wg_interval(b);
  p.stale_limit = o.stale_rounds;
  p.relabel_x16 = o.relabel_factor_x16;
  p.with_cut = with_cut ? 1 : 0;
  const int G = b->cfg.group_lanes;
  const bool big = b->cfg.wg_threads == 1024;
  int grid = 0;
  if (big) grid = G == 4 ? wg_grid_for<4, 1024>(b) : G == 16 ? wg_grid_for<16, 1024>(b)
                                                          : wg_grid_for<8, 1024>(b);
  else grid = G == 4 ? wg_grid_for<4, 256>(b) : G == 16 ? wg_grid_for<16, 256>(b)
                                                       : wg_grid_for<8, 256>(b);
  const int32_t key[8] = {G * (big ? -1 : 1), grid, p.gr_interval, p.stale_limit,
                          p.relabel_x16, p.with_cut, b->has_ns ? 1 : 0, n};
  if (!b->wg_exec || std::memcmp(key, b->wg_key, sizeof(key)) != 0) {
    if (b->wg_exec) (void)hipGraphExecDestroy(b->wg_exec);
    if (b->wg_graph) (void)hipGraphDestroy(b->wg_graph);
    b->wg_exec = nullptr;
    b->wg_graph = nullptr;
    if (big)
      he = G == 4    ? wg_capture<4, 1024>(b, grid, p, next, order, skip_d, res_d)
           : G == 16 ? wg_capture<16, 1024>(b, grid, p, next, order, skip_d, res_d)
                     : wg_capture<8, 1024>(b, grid, p, next, order, skip_d, res_d);
    else
      he = G == 4    ? wg_capture<4, 256>(b, grid, p, next, order, skip_d, res_d)
           : G == 16 ? wg_capture<16, 256>(b, grid, p, next, order, skip_d, res_d)
                     : wg_capture<8, 256>(b, grid, p, next, order, skip_d, res_d);
    if (he != hipSuccess) {
      b->wg_exec = nullptr;
      return hip_fail(he, "capturing the workgroups launch");
    }
    std::memcpy(b->wg_key, key, sizeof(key));
  }
  he = hipGraphLaunch(b->wg_exec, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(res_h, res_d, (size_t)n * sizeof(WgResult), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "running the workgroups schedule");
  fp_status st = FP_OK;
  for (int32_t i = 0; i < n; ++i) {
    if (skip && skip[i]) {
      if (flows) flows[i] = -1;
      continue;
    }
    const WgResult& r = res_h[i];
    fp_problem* pb = b->pbs[i];
    pb->st.rounds += r.rounds;
    pb->st.tail_rounds += r.rounds;
    pb->st.global_relabels += r.global_relabels;
    pb->st.restarts += r.restarts;
    pb->epoch = std::max(pb->epoch, r.epoch + 1);
    const bool bad = r.err & (ERR_LABEL | ERR_GUARD | ERR_SINK_REACHED);
    if (bad && st == FP_OK) {
      set_error("problem %d: %s", i,
                (r.err & ERR_LABEL)   ? "internal check: a relabel did not raise a label"
                : (r.err & ERR_GUARD) ? "no convergence within the round or level bound"
                                      : "internal check: a sink is reachable from the source side");
      st = FP_ERR_DEVICE;
    }
    pb->inited = true;
    pb->solved = !bad;
    pb->labels_exact = false;
    pb->st.flow_value = (int64_t)r.flow;
    if (flows) flows[i] = bad ? -1 : (int64_t)r.flow;
  }
  if (ms)
    *ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

// The kept problems in unions that fit 31-bit ids (a handle holds fewer than
// 2^30 pins and 2^31 network nodes), union_pins and a net-weight sum of at
// most INT32_MAX, in index order.
static fp_status batch_union(fp_batch* b, const uint8_t* skip, int32_t with_cut, hipStream_t s,
                             int64_t* flows, float* ms) {
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int32_t> chunk;
  long long V = 0, E = 0, P = 0, W = 0;
  const long long max_pins = b->cfg.union_pins > 0 ? b->cfg.union_pins : (1ll << 30) - 1;
  for (int32_t i = 0; i <= b->count; ++i) {
    const bool last = i == b->count;
    if (!last && skip && skip[i]) {
      if (flows) flows[i] = -1;
      continue;
    }
    const fp_problem* pb = last ? nullptr : b->pbs[i];
    // a union must fit 31-bit ids, the pin bound and (like every problem)
    // a sum of net weights of at most INT32_MAX
    const bool full = !last && !chunk.empty() &&
                      (P + pb->P > max_pins ||
                       V + pb->V + 2 + 2 * (E + pb->E) >= (1ll << 31) - 16 ||
                       W + pb->wsum > 0x7fffffffll);
    if ((last || full) && !chunk.empty()) {
      fp_status st = union_chunk(b, chunk, with_cut, s, flows);
      if (st) return st;
      chunk.clear();
      V = E = P = W = 0;
    }
    if (last) break;
    chunk.push_back(i);
    V += pb->V;
    E += pb->E;
    P += pb->P;
    W += pb->wsum;
  }
  if (ms)
    *ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return FP_OK;
}

static fp_status batch_replay(fp_batch* b, const uint8_t* skip, int32_t with_cut, bool force_init,
                              hipStream_t s, int64_t* flows, float* ms) {
  if (b->cfg.schedule == kScheduleUnion) return batch_union(b, skip, with_cut, s, flows, ms);
  if (b->cfg.schedule == kScheduleWorkgroups)
    return batch_workgroups(b, skip, with_cut, s, flows, ms);
  return batch_concurrent(b, skip, with_cut, force_init, s, flows, ms);
}

fp_status run_batch(fp_batch* b, const uint8_t* skip, int32_t with_cut, hipStream_t s,
                    int64_t* flows) {
  if (with_cut && !b->has_vs) {
    set_error("this batch plan was created without vertex_sides");
    return FP_ERR_INVALID;
  }
  if (b->count == 0) return FP_OK;
  return batch_replay(b, skip, with_cut, false, s, flows, nullptr);
}

static std::string batch_signature(const fp_batch* b) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, b->device);
  long long pins = 0, nodes = 0;
  for (const fp_problem* pb : b->pbs) {
    pins += pb->P;
    nodes += pb->N;
  }
  char buf[256];
  snprintf(buf, sizeof(buf), "%s/%d/%d/%lld/%lld", prop.gcnArchName, prop.multiProcessorCount,
           b->count, pins, nodes);
  std::string sig = buf;
  for (char& ch : sig)
    if (ch == ' ') ch = '_';
  return sig;
}

static bool cache_lookup(const char* path, const std::string& sig, fp_batch_config* c) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512], key[256];
  int g = 0, gr = 0, ns = 0, sc = 0, wt = 0;
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    // lines of another layout are skipped
    if (sscanf(line, "%255s v3 %d %d %d %d %d", key, &g, &gr, &ns, &sc, &wt) != 6) continue;
    if (sig == key) {  // the last entry for a signature wins
      *c = fp_batch_config{};
      c->group_lanes = g;
      c->gr_interval = gr;
      c->streams = ns;
      c->schedule = sc;
      c->wg_threads = wt;
      found = batch_config_valid(*c);
    }
  }
  fclose(f);
  return found;
}

static void cache_store(const char* path, const std::string& sig, const fp_batch_config& c) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s v3 %d %d %d %d %d\n", sig.c_str(), c.group_lanes, c.gr_interval, c.streams,
          c.schedule, c.wg_threads);
  fclose(f);
}

fp_status tune_batch(fp_batch* b, hipStream_t s, const char* cache_path, fp_batch_config* chosen) {
  if (b->count == 0) {
    if (chosen) *chosen = b->cfg;
    return FP_OK;
  }
  const std::string sig = batch_signature(b);
  fp_batch_config cached{};
  if (cache_lookup(cache_path, sig, &cached)) {
    cached.union_pins = b->cfg.union_pins;  // the caller's memory bound is not tuned
    b->cfg = cached;
    fp_status st = batch_replay(b, nullptr, 0, true, s, nullptr, nullptr);
    if (st) return st;
    if (chosen) *chosen = b->cfg;
    return FP_OK;
  }
  const fp_batch_config base = b->cfg;
  fp_batch_config best = base;
  float best_ms = 1e30f;
  auto trial = [&](const fp_batch_config& c) -> fp_status {
    b->cfg = c;
    // the better of two runs (the first of a schedule also sets it up), with
    // the source sides when the plan has buffers for them (the union always
    // extracts them to split its flow; the other schedules only on request)
    float ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      float t = 0.f;
      fp_status st = batch_replay(b, nullptr, b->has_vs ? 1 : 0, true, s, nullptr, &t);
      if (st) return st;
      ms = std::min(ms, t);
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return FP_OK;
  };
  // one knob at a time, each from the best so far: schedule and concurrency
  // (worker streams or the union), lanes per node, relabel interval
  {
    const int streams[5] = {1, 2, 4, 8, 16};
    for (int ns : streams) {
      fp_batch_config c = base;
      c.schedule = kScheduleWorkers;
      c.streams = ns;
      fp_status st = trial(c);
      if (st) return st;
    }
    fp_batch_config c = base;
    c.schedule = kScheduleUnion;
    fp_status st = trial(c);
    if (st) return st;
    c.schedule = kScheduleWorkgroups;
    for (int t : {256, 1024}) {
      c.wg_threads = t;
      st = trial(c);
      if (st) return st;
    }
  }
  const int lanes[3] = {4, 8, 16};
  const fp_batch_config conc = best;
  for (int g : lanes) {
    fp_batch_config c = conc;
    c.group_lanes = g;
    if (c.group_lanes == conc.group_lanes) continue;
    fp_status st = trial(c);
    if (st) return st;
  }
  const int intervals[4] = {8, 16, 32, 64};
  const fp_batch_config shape = best;
  for (int gr : intervals) {
    fp_batch_config c = shape;
    c.gr_interval = gr;
    if (c.gr_interval == shape.gr_interval) continue;
    fp_status st = trial(c);
    if (st) return st;
  }
  b->cfg = best;
  // leave every problem solved with the chosen configuration
  fp_status st = batch_replay(b, nullptr, 0, true, s, nullptr, nullptr);
  if (st) return st;
  cache_store(cache_path, sig, best);
  if (chosen) *chosen = best;
  return FP_OK;
}

fp_status batch_config(const fp_batch* b, fp_batch_config* out) {
  *out = b->cfg;
  return FP_OK;
}

fp_status batch_solve(fp_problem* const* pbs, int32_t count, const uint8_t* skip, hipStream_t s,
                      int64_t* flows) {
  if (count == 0) return FP_OK;
  fp_batch* b = nullptr;
  fp_status st = create_batch(pbs, count, nullptr, nullptr, nullptr, s, &b);
  if (st) return st;
  st = run_batch(b, skip, 0, s, flows);
  release_batch(b);
  delete b;
  return st;
}

}  // namespace hf
