// Batched solve of many independent flow problems.
//
// The paper's refinement runs many block-pair flow problems at once (section
// "Parallel Active Block Scheduling").  The persistent kernel below takes
// problems from a shared queue, largest first, and each workgroup runs a
// whole problem -- initialisation, global relabels, discharge rounds,
// termination check and, optionally, the source-side cut -- with workgroup
// barriers as the only ordering points, replayed from a captured HIP graph.
//
// That persistent path is switched off (kPersistentBatch): its first GPU run
// ended in a memory access fault whose cause has not been found.  Until it
// is, a plan runs its problems concurrently with the single-problem path
// (same device phases, device-wide kernels and single-workgroup tail loops):
// `streams` host workers take problems from a shared queue, largest first,
// and drive each on a HIP stream of their own, so the kernels and host
// round trips of different problems overlap.  Results are identical.
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

namespace hf {

struct BatchParam {
  int32_t epoch0;        // stamp value of the first round
  int32_t init;          // start from the zero flow
  int32_t skip;          // leave the problem alone
  int32_t gr_interval;   // rounds between global relabels (<= 0: off)
  int32_t stale_rounds;  // stale-flow global relabel trigger (<= 0: off)
  int32_t want_cut;      // also write the minimal source side
  int32_t pad0, pad1;
  unsigned long long relabel_budget;  // relabels between global relabels
  long long round_budget;             // rounds of this solve (<= 0: no limit)
  long long round_guard;              // give up (no convergence) after this many rounds
};

enum BatchStatus : int32_t {
  BST_OK = 0,
  BST_BUDGET = 1,   // round budget exhausted
  BST_GUARD = 2,    // no convergence
  BST_LABEL = 3,    // a relabel did not raise a label
  BST_SINK = 4,     // the cut BFS reached a sink
  BST_SKIPPED = 5,
};

struct BatchResult {
  long long flow;
  long long rounds;
  unsigned long long relabels;
  int32_t epoch_end;  // stamp value of the next round
  int32_t global_relabels;
  int32_t bfs_levels;
  int32_t restarts;
  int32_t status;
  int32_t pad;
};

// Rounds per problem before a batched solve gives up; far above what any
// converging solve needs, and small enough that a workgroup never spins for
// long.
constexpr long long kBatchGuardBase = 1000000ll;
constexpr bool kPersistentBatch = false;  // see the note at the top of the file
constexpr long long kBatchGuardPerNode = 20ll;
constexpr int kStaleFrontier = 1500;  // "only few active nodes" (paper)

// Global relabel inside one workgroup: reset labels, reverse BFS level by
// level, gather the active nodes.  Returns the size of the new frontier
// (the same value in every thread).
template <int G>
__device__ int wg_global_relabel(const Dev& g, int epoch, lds_int* lds, int* levels) {
  phase_gr_reset(g, 0, 1, lds);
  phase_gr_bits(g, threadIdx.x, blockDim.x);
  __syncthreads();
  int level = 0;
  for (;;) {
    const int nf = count_all_vol(g.ctl->bcnt[level % 3]);
    if (nf == 0) break;
    __syncthreads();  // every thread has read the count before it changes
    phase_bfs_rev<G>(g, level, 0, 1, KC_BATCH, lds);
    __syncthreads();
    ++level;
  }
  *levels += level;
  phase_gather(g, epoch, 0, 1, lds);
  __syncthreads();
  const int nf = count_all_vol(g.ctl->fcnt[epoch % 3]);
  __syncthreads();
  return nf;
}

// Push-relabel to a maximum preflow inside one workgroup, with the global
// relabel triggers of the single-problem path: relabel work, rounds since
// the last global relabel, stale flow value, and the terminating relabel
// when the frontier empties (paper, section "A Bug in the Synchronous
// Algorithm").  Every decision reads counters after a barrier, so all
// threads take the same branch.
template <int G>
__device__ void wg_solve(const Dev& g, const BatchParam& p, BatchResult& r, int* epoch_io,
                         lds_int* lds) {
  int epoch = *epoch_io;
  if (p.init) {
    phase_init(g, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  int levels = 0, grs = 1, restarts = 0, status = BST_OK;
  long long rounds = 0;
  int nf = wg_global_relabel<G>(g, epoch, lds, &levels);
  unsigned long long rel_at_gr = ld_vol64(&g.ctl->relabels);
  unsigned long long last_flow = ld_vol64(&g.ctl->flow);
  int stale = 0, since = 0;
  bool fresh = true;
  for (;;) {
    if (ld_vol(&g.ctl->err) & ERR_LABEL) {
      status = BST_LABEL;
      break;
    }
    if (nf == 0) {
      if (fresh) break;
      nf = wg_global_relabel<G>(g, epoch, lds, &levels);
      ++grs;
      if (nf > 0) ++restarts;
      rel_at_gr = ld_vol64(&g.ctl->relabels);
      last_flow = ld_vol64(&g.ctl->flow);
      since = stale = 0;
      fresh = true;
      __syncthreads();
      continue;
    }
    if (p.round_budget > 0 && rounds >= p.round_budget) {
      status = BST_BUDGET;
      break;
    }
    if (rounds >= p.round_guard) {
      status = BST_GUARD;
      break;
    }
    fresh = false;
    phase_push<G>(g, epoch, 0, 1, KC_BATCH, lds);
    __syncthreads();
    phase_apply(g, epoch, 0, 1, KC_BATCH, lds);
    __syncthreads();
    ++epoch;
    ++rounds;
    ++since;
    const unsigned long long fl = ld_vol64(&g.ctl->flow);
    if (fl != last_flow) {
      last_flow = fl;
      stale = 0;
    } else if (nf < kStaleFrontier) {
      ++stale;
    }
    const bool gr = (p.stale_rounds > 0 && stale >= p.stale_rounds) ||
                    ld_vol64(&g.ctl->relabels) - rel_at_gr >= p.relabel_budget ||
                    (p.gr_interval > 0 && since >= p.gr_interval);
    if (gr) {
      nf = wg_global_relabel<G>(g, epoch, lds, &levels);
      ++grs;
      rel_at_gr = ld_vol64(&g.ctl->relabels);
      last_flow = ld_vol64(&g.ctl->flow);
      since = stale = 0;
      fresh = true;
    } else {
      nf = count_all_vol(g.ctl->fcnt[epoch % 3]);
    }
    __syncthreads();  // counters read before the next phase changes them
  }
  r.flow = (long long)ld_vol64(&g.ctl->flow);
  r.rounds = rounds;
  r.relabels = ld_vol64(&g.ctl->relabels);
  r.global_relabels = grs;
  r.bfs_levels = levels;
  r.restarts = restarts;
  r.status = status;
  *epoch_io = epoch;
  __syncthreads();
}

// Source side inside one workgroup: seeds, forward BFS of the uncapped
// residual network, side bitmaps (paper, paragraph "Source-Side Cut").
// Returns true if the BFS reached a sink.
template <int G>
__device__ bool wg_cut(const Dev& g, int ep, uint8_t* vs, uint8_t* ns, lds_int* lds,
                       int* levels) {
  phase_cut_seed(g, ep, false, 0, 1, lds);
  __syncthreads();
  int level = 0;
  for (;;) {
    const int nf = count_all_vol(g.ctl->bcnt[level % 3]);
    if (nf == 0) break;
    __syncthreads();
    phase_bfs_fwd<G>(g, level, ep, 0, 1, KC_BATCH, lds);
    __syncthreads();
    ++level;
  }
  *levels += level;
  const int err = ld_vol(&g.ctl->err);
  __syncthreads();
  phase_cut_out(g, ep, vs, ns, threadIdx.x, blockDim.x);
  __syncthreads();
  return (err & ERR_SINK_REACHED) != 0;
}

// Persistent batch kernel: workgroups take problem indices from *head in
// the order `order` (largest first) until the queue is exhausted.  Every
// workgroup leaves once the queue is empty, so the grid always drains.
template <int G, int BS>
__global__ void __launch_bounds__(BS)
    k_batch(const Dev* __restrict__ devs, const BatchParam* __restrict__ params,
            const int32_t* __restrict__ order, int32_t count, int32_t* head,
            BatchResult* __restrict__ res, uint8_t* const* __restrict__ vsides,
            uint8_t* const* __restrict__ nsides) {
  __shared__ int32_t hf_bq[lds_words(BS)];
  __shared__ int32_t s_next;
  lds_int* const lds = (lds_int*)hf_bq;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(head, 1);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();  // s_next is rewritten only after every thread read it
    if (k >= count) break;
    const int pid = __builtin_amdgcn_readfirstlane(order[k]);
    const BatchParam& p = params[pid];
    BatchResult r{};
    if (p.skip) {
      if (threadIdx.x == 0) {
        r.status = BST_SKIPPED;
        r.epoch_end = p.epoch0;
        r.flow = -1;
        res[pid] = r;
      }
      continue;
    }
    const Dev& g = devs[pid];
    int epoch = p.epoch0;
    wg_solve<G>(g, p, r, &epoch, lds);
    if (r.status == BST_OK && p.want_cut) {
      int levels = 0;
      const bool sink = wg_cut<G>(g, epoch, vsides[pid], nsides ? nsides[pid] : nullptr, lds,
                                  &levels);
      ++epoch;
      r.bfs_levels += levels;
      if (sink) r.status = BST_SINK;
    }
    r.epoch_end = epoch;
    if (threadIdx.x == 0) res[pid] = r;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t n, int32_t v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = v;
}

typedef void (*BatchKernel)(const Dev*, const BatchParam*, const int32_t*, int32_t, int32_t*,
                            BatchResult*, uint8_t* const*, uint8_t* const*);

static BatchKernel batch_kernel(int G, int BS) {
  if (BS == 256) {
    if (G == 4) return k_batch<4, 256>;
    if (G == 8) return k_batch<8, 256>;
    if (G == 16) return k_batch<16, 256>;
  } else if (BS == 1024) {
    if (G == 4) return k_batch<4, 1024>;
    if (G == 8) return k_batch<8, 1024>;
    if (G == 16) return k_batch<16, 1024>;
  }
  return nullptr;
}

}  // namespace hf

struct fp_batch {
  int device = 0;
  int32_t count = 0;
  std::vector<fp_problem*> pbs;
  std::vector<int32_t> order;
  fp_batch_config cfg{};
  bool has_vs = false;
  bool has_ns = false;
  void* dmem = nullptr;
  hf::Dev* devs_d = nullptr;
  hf::BatchParam* params_d = nullptr;
  int32_t* order_d = nullptr;
  int32_t* head_d = nullptr;
  hf::BatchResult* res_d = nullptr;
  uint8_t** vs_d = nullptr;
  uint8_t** ns_d = nullptr;
  void* hmem = nullptr;  // pinned: devs_h, params_h, res_h
  hf::Dev* devs_h = nullptr;
  hf::BatchParam* params_h = nullptr;
  hf::BatchResult* res_h = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  fp_batch_config exec_cfg[2]{};
  int cus = 0;
  std::vector<hipStream_t> workers;  // streams of the concurrent schedule
  void* umem = nullptr;              // scratch of the union schedule
  size_t umem_bytes = 0;
};

namespace hf {

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static fp_batch_config resolve_batch_config(const fp_batch_config* c) {
  fp_batch_config r{};
  if (c) r = *c;
  if (r.group_lanes == 0) r.group_lanes = 4;
  if (r.block_threads == 0) r.block_threads = 1024;
  if (r.streams == 0) r.streams = 4;
  return r;
}

static bool batch_config_valid(const fp_batch_config& c) {
  return (c.group_lanes == 4 || c.group_lanes == 8 || c.group_lanes == 16) &&
         (c.block_threads == 256 || c.block_threads == 1024) && c.gr_interval >= -1 &&
         c.workgroups >= 0 && c.streams >= 1 && c.streams <= 64 &&
         (c.schedule == 0 || c.schedule == 1) && c.union_pins >= 0;
}

bool batch_config_ok(const fp_batch_config* c) {
  return batch_config_valid(resolve_batch_config(c));
}

static void drop_graphs(fp_batch* b) {
  for (int i = 0; i < 2; ++i)
    if (b->exec[i]) {
      (void)hipGraphExecDestroy(b->exec[i]);
      b->exec[i] = nullptr;
    }
}

void release_batch(fp_batch* b) {
  drop_graphs(b);
  for (hipStream_t w : b->workers) (void)hipStreamDestroy(w);
  b->workers.clear();
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->dmem) (void)hipFree(b->dmem);
  if (b->hmem) (void)hipHostFree(b->hmem);
  if (b->umem) (void)hipFree(b->umem);
  b->cap = nullptr;
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
  const size_t o_params = off;
  off = align_up(off + n * sizeof(BatchParam));
  const size_t o_order = off;
  off = align_up(off + n * sizeof(int32_t));
  const size_t o_head = off;
  off = align_up(off + sizeof(int32_t));
  const size_t o_res = off;
  off = align_up(off + n * sizeof(BatchResult));
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
  b->params_d = reinterpret_cast<BatchParam*>(d + o_params);
  b->order_d = reinterpret_cast<int32_t*>(d + o_order);
  b->head_d = reinterpret_cast<int32_t*>(d + o_head);
  b->res_d = reinterpret_cast<BatchResult*>(d + o_res);
  b->vs_d = reinterpret_cast<uint8_t**>(d + o_vs);
  b->ns_d = reinterpret_cast<uint8_t**>(d + o_ns);
  size_t hoff = 0;
  const size_t h_devs = hoff;
  hoff = align_up(hoff + n * sizeof(Dev));
  const size_t h_params = hoff;
  hoff = align_up(hoff + n * sizeof(BatchParam));
  const size_t h_res = hoff;
  hoff = align_up(hoff + n * sizeof(BatchResult));
  he = hipHostMalloc(&b->hmem, hoff, hipHostMallocDefault);
  if (he == hipSuccess) {
    char* h = static_cast<char*>(b->hmem);
    b->devs_h = reinterpret_cast<Dev*>(h + h_devs);
    b->params_h = reinterpret_cast<BatchParam*>(h + h_params);
    b->res_h = reinterpret_cast<BatchResult*>(h + h_res);
    std::memset(b->hmem, 0, hoff);
    he = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  }
  if (he == hipSuccess)
    he = hipMemcpyAsync(b->order_d, b->order.data(), (size_t)count * sizeof(int32_t),
                        hipMemcpyHostToDevice, s);
  if (he == hipSuccess && vsides)
    he = hipMemcpyAsync(b->vs_d, vsides, (size_t)count * sizeof(uint8_t*), hipMemcpyHostToDevice,
                        s);
  if (he == hipSuccess && nsides)
    he = hipMemcpyAsync(b->ns_d, nsides, (size_t)count * sizeof(uint8_t*), hipMemcpyHostToDevice,
                        s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  int cus = 0;
  if (he == hipSuccess) he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                                   b->device);
  if (he != hipSuccess) {
    fp_status st = hip_fail(he, "setting up the batch plan");
    release_batch(b);
    delete b;
    return st;
  }
  b->cus = cus;
  *out = b;
  return FP_OK;
}

// Capture (or reuse) the graph of one run variant.
static fp_status batch_graph(fp_batch* b, int with_cut, hipGraphExec_t* exec) {
  const fp_batch_config& c = b->cfg;
  if (b->exec[with_cut] && std::memcmp(&b->exec_cfg[with_cut], &c, sizeof(c)) == 0) {
    *exec = b->exec[with_cut];
    return FP_OK;
  }
  if (b->exec[with_cut]) {
    (void)hipGraphExecDestroy(b->exec[with_cut]);
    b->exec[with_cut] = nullptr;
  }
  BatchKernel kern = batch_kernel(c.group_lanes, c.block_threads);
  if (!kern) {
    set_error("no batch kernel for group_lanes %d, block_threads %d", c.group_lanes,
              c.block_threads);
    return FP_ERR_INVALID;
  }
  int per_cu = 0;
  hipError_t he =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, c.block_threads, 0);
  if (he != hipSuccess) return hip_fail(he, "batch kernel occupancy");
  long long grid = (long long)std::max(per_cu, 1) * std::max(b->cus, 1);
  if (c.workgroups > 0) grid = std::min<long long>(grid, c.workgroups);
  grid = std::max<long long>(1, std::min<long long>(grid, b->count));
  const size_t n = (size_t)b->count;
  hipGraph_t graph = nullptr;
  he = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) return hip_fail(he, "beginning the batch graph capture");
  hipError_t e1 = hipMemcpyAsync(b->devs_d, b->devs_h, n * sizeof(Dev), hipMemcpyHostToDevice,
                                 b->cap);
  if (e1 == hipSuccess)
    e1 = hipMemcpyAsync(b->params_d, b->params_h, n * sizeof(BatchParam), hipMemcpyHostToDevice,
                        b->cap);
  if (e1 == hipSuccess) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, b->cap, b->head_d, 1, 0);
    e1 = hipGetLastError();
  }
  if (e1 == hipSuccess) {
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(c.block_threads), 0, b->cap,
                       (const Dev*)b->devs_d, (const BatchParam*)b->params_d,
                       (const int32_t*)b->order_d, b->count, b->head_d, b->res_d,
                       (uint8_t* const*)b->vs_d, (uint8_t* const*)(b->has_ns ? b->ns_d : nullptr));
    e1 = hipGetLastError();
  }
  if (e1 == hipSuccess)
    e1 = hipMemcpyAsync(b->res_h, b->res_d, n * sizeof(BatchResult), hipMemcpyDeviceToHost,
                        b->cap);
  he = hipStreamEndCapture(b->cap, &graph);
  if (e1 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(e1, "capturing the batch graph");
  }
  if (he != hipSuccess) return hip_fail(he, "ending the batch graph capture");
  he = hipGraphInstantiate(&b->exec[with_cut], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (he != hipSuccess) {
    b->exec[with_cut] = nullptr;
    return hip_fail(he, "instantiating the batch graph");
  }
  b->exec_cfg[with_cut] = c;
  *exec = b->exec[with_cut];
  return FP_OK;
}

// One replay: fill the parameters from the handles, launch, read results.
// `force_init` starts every problem from the zero flow (tuning).
// Problems spread over `streams` workers, each a host thread driving the
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

// The kept problems in unions that fit 31-bit ids (a handle holds fewer than
// 2^30 pins and 2^31 network nodes) and union_pins, in index order.
static fp_status batch_union(fp_batch* b, const uint8_t* skip, int32_t with_cut, hipStream_t s,
                             int64_t* flows, float* ms) {
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int32_t> chunk;
  long long V = 0, E = 0, P = 0;
  const long long max_pins = b->cfg.union_pins > 0 ? b->cfg.union_pins : (1ll << 30) - 1;
  for (int32_t i = 0; i <= b->count; ++i) {
    const bool last = i == b->count;
    if (!last && skip && skip[i]) {
      if (flows) flows[i] = -1;
      continue;
    }
    const fp_problem* pb = last ? nullptr : b->pbs[i];
    const bool full = !last && !chunk.empty() &&
                      (P + pb->P > max_pins ||
                       V + pb->V + 2 + 2 * (E + pb->E) >= (1ll << 31) - 16);
    if ((last || full) && !chunk.empty()) {
      fp_status st = union_chunk(b, chunk, with_cut, s, flows);
      if (st) return st;
      chunk.clear();
      V = E = P = 0;
    }
    if (last) break;
    chunk.push_back(i);
    V += pb->V;
    E += pb->E;
    P += pb->P;
  }
  if (ms)
    *ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return FP_OK;
}

static fp_status batch_replay(fp_batch* b, const uint8_t* skip, int32_t with_cut, bool force_init,
                              hipStream_t s, int64_t* flows, float* ms) {
  if (b->cfg.schedule == 1) return batch_union(b, skip, with_cut, s, flows, ms);
  if (!kPersistentBatch) return batch_concurrent(b, skip, with_cut, force_init, s, flows, ms);
  hipGraphExec_t exec = nullptr;
  fp_status st = batch_graph(b, with_cut ? 1 : 0, &exec);
  if (st) return st;
  for (int32_t i = 0; i < b->count; ++i) {
    fp_problem* pb = b->pbs[i];
    Dev d = pb->dev;
    d.bfs_arc = 0;  // node-grouped reverse BFS levels inside a workgroup
    b->devs_h[i] = d;
    BatchParam& p = b->params_h[i];
    p = BatchParam{};
    p.epoch0 = pb->epoch;
    p.init = (force_init || !pb->inited) ? 1 : 0;
    p.skip = skip && skip[i] ? 1 : 0;
    p.gr_interval = b->cfg.gr_interval != 0 ? b->cfg.gr_interval : pb->opt.gr_interval;
    p.stale_rounds = pb->opt.stale_rounds;
    p.want_cut = with_cut ? 1 : 0;
    p.relabel_budget =
        (unsigned long long)((double)pb->N * pb->opt.relabel_factor_x16 / 16.0) + 1ull;
    p.round_budget = pb->opt.round_budget;
    p.round_guard = kBatchGuardBase + kBatchGuardPerNode * (long long)pb->N;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, s);
  }
  hipError_t he = hipGraphLaunch(exec, s);
  if (ms && he == hipSuccess) he = hipEventRecord(e1, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (ms) {
    if (he == hipSuccess) he = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (he != hipSuccess) return hip_fail(he, "batched solve");
  fp_status first = FP_OK;
  for (int32_t i = 0; i < b->count; ++i) {
    fp_problem* pb = b->pbs[i];
    const BatchResult& r = b->res_h[i];
    if (r.status == BST_SKIPPED) {
      if (flows) flows[i] = -1;
      continue;
    }
    pb->epoch = r.epoch_end;
    pb->inited = true;
    pb->st.rounds += r.rounds;
    pb->st.tail_rounds += r.rounds;
    pb->st.relabels = (int64_t)r.relabels;
    pb->st.global_relabels += r.global_relabels;
    pb->st.bfs_levels += r.bfs_levels;
    pb->st.restarts += r.restarts;
    pb->st.host_syncs += 1;
    pb->st.flow_value = r.flow;
    pb->solved = r.status == BST_OK;
    if (flows) flows[i] = r.status == BST_OK ? r.flow : -1;
    if (r.status != BST_OK && first == FP_OK) {
      switch (r.status) {
        case BST_BUDGET:
          set_error("problem %d: round budget of %d rounds exhausted", i, pb->opt.round_budget);
          first = FP_ERR_ABORTED;
          break;
        case BST_GUARD:
          set_error("problem %d: no convergence after %lld rounds", i, (long long)r.rounds);
          first = FP_ERR_DEVICE;
          break;
        case BST_LABEL:
          set_error("problem %d: internal check: a relabel did not raise a label", i);
          first = FP_ERR_DEVICE;
          break;
        case BST_SINK:
          set_error("problem %d: internal check: a sink is reachable from the source side", i);
          first = FP_ERR_DEVICE;
          break;
        default:
          set_error("problem %d: unknown batch status %d", i, r.status);
          first = FP_ERR_DEVICE;
      }
    }
  }
  return first;
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
  int g = 0, bs = 0, gr = 0, wg = 0, ns = 0, sc = 0;
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    // lines of another layout are skipped
    if (sscanf(line, "%255s %d %d %d %d %d %d", key, &g, &bs, &gr, &wg, &ns, &sc) != 7) continue;
    if (sig == key) {  // the last entry for a signature wins
      *c = fp_batch_config{};
      c->group_lanes = g;
      c->block_threads = bs;
      c->gr_interval = gr;
      c->workgroups = wg;
      c->streams = ns;
      c->schedule = sc;
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
  fprintf(f, "%s %d %d %d %d %d %d\n", sig.c_str(), c.group_lanes, c.block_threads,
          c.gr_interval, c.workgroups, c.streams, c.schedule);
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
    float ms = 0.f;
    fp_status st = batch_replay(b, nullptr, 0, true, s, nullptr, &ms);
    if (st) return st;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return FP_OK;
  };
  // one knob at a time, each from the best so far: schedule and concurrency
  // (worker streams or the union; block size for the persistent kernel),
  // lanes per node, relabel interval
  if (kPersistentBatch) {
    const int blocks[2] = {1024, 256};
    for (int bs : blocks) {
      fp_batch_config c = base;
      c.block_threads = bs;
      fp_status st = trial(c);
      if (st) return st;
    }
  } else {
    const int streams[5] = {1, 2, 4, 8, 16};
    for (int ns : streams) {
      fp_batch_config c = base;
      c.schedule = 0;
      c.streams = ns;
      fp_status st = trial(c);
      if (st) return st;
    }
    fp_batch_config c = base;
    c.schedule = 1;
    fp_status st = trial(c);
    if (st) return st;
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
