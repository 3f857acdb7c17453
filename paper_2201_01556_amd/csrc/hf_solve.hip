// Solver kernels and their host orchestration.
//
// Large frontiers run as device-wide kernels (one launch per phase, the
// kernel boundary is the ordering point).  Frontiers at or below the tail
// threshold run inside one workgroup that loops over rounds (or BFS levels)
// with workgroup barriers, so the long power-law tail of small rounds the
// paper observes (paragraph "Avoid Pushing Flow Back") costs no launches and
// no host round trips.  Both paths call the same phase functions.
#include <cstdio>
#include <cstring>

#include "hf_host.h"

namespace hf {

constexpr int kThreads = 256;    // device-wide kernels
constexpr int kLoopThreads = 1024;  // single-workgroup loops
constexpr int kMaxBlocks = 2048;
constexpr long long kRoundGuard = 200000000ll;  // rounds per solve before giving up

__device__ __forceinline__ int ld_vol(const int32_t* p) {
  return __atomic_load_n(p, __ATOMIC_RELAXED);
}
__device__ __forceinline__ unsigned long long ld_vol64(const unsigned long long* p) {
  return __atomic_load_n(p, __ATOMIC_RELAXED);
}

// ordering point inside one workgroup: all global writes of the workgroup
// become visible to all its waves (L1 is invalidated by the agent fence)
__device__ __forceinline__ void wg_sync() {
  __threadfence();
  __syncthreads();
}

__device__ __forceinline__ int gwave() { return (blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ __forceinline__ int gwaves() { return (gridDim.x * blockDim.x) >> 6; }
__device__ __forceinline__ int gthread() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int gthreads() { return gridDim.x * blockDim.x; }

__global__ void __launch_bounds__(kThreads) k_init(Dev g) { phase_init(g, gthread(), gthreads()); }

__global__ void __launch_bounds__(kThreads) k_gr_reset(Dev g) {
  phase_gr_reset(g, gthread(), gthreads());
}

template <int G>
__global__ void __launch_bounds__(kThreads) k_bfs_rev(Dev g, int level) {
  phase_bfs_rev<G>(g, level, gwave(), gwaves(), KC_BFS_REV);
}

__global__ void __launch_bounds__(kThreads) k_gather(Dev g, int epoch) {
  phase_gather(g, epoch, gthread(), gthreads());
}

template <int G>
__global__ void __launch_bounds__(kThreads) k_push(Dev g, int epoch) {
  phase_push<G>(g, epoch, gwave(), gwaves(), KC_PUSH);
}

__global__ void __launch_bounds__(kThreads) k_apply(Dev g, int epoch) {
  phase_apply(g, epoch, gthread(), gthreads(), KC_APPLY);
}

__global__ void __launch_bounds__(kThreads) k_cut_seed(Dev g, int ep) {
  phase_cut_seed(g, ep, gthread(), gthreads());
}

template <int G>
__global__ void __launch_bounds__(kThreads) k_bfs_fwd(Dev g, int level, int ep) {
  phase_bfs_fwd<G>(g, level, ep, gwave(), gwaves(), KC_BFS_FWD);
}

__global__ void __launch_bounds__(kThreads) k_cut_out(Dev g, int ep, uint8_t* vs, uint8_t* ns) {
  phase_cut_out(g, ep, vs, ns, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_check(Dev g) {
  phase_check(g, gthread(), gthreads());
}

// Rounds inside one workgroup.  Stops when the frontier is empty, exceeds
// `cap`, `max_rounds` rounds ran, or the relabel count reached
// `relabel_limit` (a global relabel is due).
template <int G>
__global__ void __launch_bounds__(kLoopThreads) k_round_loop(Dev g, int epoch0, int max_rounds,
                                                             int cap,
                                                             unsigned long long relabel_limit) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int epoch = epoch0;
  int r = 0;
  int why = 0;
  for (;;) {
    const int c3 = epoch % 3;
    const int nf = ld_vol(&g.ctl->fcnt[c3][0]) + ld_vol(&g.ctl->fcnt[c3][1]);
    if (nf == 0) { why = 1; break; }
    if (nf > cap) { why = 2; break; }
    if (r >= max_rounds) { why = 3; break; }
    if (ld_vol64(&g.ctl->relabels) >= relabel_limit) { why = 4; break; }
    phase_push<G>(g, epoch, wv, nw, KC_LOOP_ROUNDS);
    wg_sync();
    phase_apply(g, epoch, threadIdx.x, blockDim.x, KC_LOOP_ROUNDS);
    wg_sync();
    ++epoch;
    ++r;
  }
  if (threadIdx.x == 0) {
    g.ctl->loop_rounds = r;
    g.ctl->loop_exit = why;
  }
}

// BFS levels inside one workgroup (reverse when ep < 0, forward otherwise).
template <int G>
__global__ void __launch_bounds__(kLoopThreads) k_bfs_loop(Dev g, int level0, int cap, int ep) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int level = level0;
  for (;;) {
    const int c3 = level % 3;
    const int nf = ld_vol(&g.ctl->bcnt[c3][0]) + ld_vol(&g.ctl->bcnt[c3][1]);
    if (nf == 0 || nf > cap) break;
    if (ep < 0) phase_bfs_rev<G>(g, level, wv, nw, KC_LOOP_BFS);
    else phase_bfs_fwd<G>(g, level, ep, wv, nw, KC_LOOP_BFS);
    wg_sync();
    ++level;
  }
  if (threadIdx.x == 0) g.ctl->loop_levels = level - level0;
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

static int sweep_grid(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

// grid for a frontier phase with `items` wave items (unknown: use the cap)
static int frontier_grid(long long items) {
  long long b = (items + (kThreads / 64) - 1) / (kThreads / 64);
  if (b < 64) b = 64;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return (int)b;
}

struct Launch {
  fp_problem* pb;
  hipStream_t s;
  Timer t;
  bool on;
  Launch(fp_problem* p, hipStream_t st, int kind) : pb(p), s(st), on(p->opt.profile != 0) {
    if (on) prof_begin(pb, kind, s, &t);
  }
  ~Launch() {
    if (on) prof_end(pb, &t, s);
  }
};

static fp_status sync_ctl(fp_problem* pb, hipStream_t s) {
  hipError_t he = hipGetLastError();
  if (he == hipSuccess)
    he = hipMemcpyAsync(pb->ctl_h, pb->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "solver step");
  pb->st.host_syncs++;
  if (pb->opt.profile) prof_collect(pb);
  return FP_OK;
}

template <int G>
static fp_status run_bfs(fp_problem* pb, hipStream_t s, int ep, int* levels_out) {
  // level 0 is already in bcnt[0]; ep < 0 = reverse (global relabel)
  Dev& g = pb->dev;
  const int cap = pb->opt.tail_threshold;
  int level = 0;
  fp_status st = sync_ctl(pb, s);
  if (st) return st;
  for (;;) {
    const int c3 = level % 3;
    const long long nf = (long long)pb->ctl_h->bcnt[c3][0] + pb->ctl_h->bcnt[c3][1];
    if (nf == 0) break;
    if (nf <= cap && !pb->opt.debug_checks) {
      {
        Launch L(pb, s, ep < 0 ? KK_BFS_REV_LOOP : KK_BFS_FWD_LOOP);
        k_bfs_loop<G><<<1, kLoopThreads, 0, s>>>(g, level, cap, ep);
      }
      st = sync_ctl(pb, s);
      if (st) return st;
      level += pb->ctl_h->loop_levels;
    } else {
      const int steps = 4;
      const int grid = frontier_grid(nf);
      for (int i = 0; i < steps; ++i) {
        if (ep < 0) {
          Launch L(pb, s, KK_BFS_REV);
          k_bfs_rev<G><<<grid, kThreads, 0, s>>>(g, level + i);
        } else {
          Launch L(pb, s, KK_BFS_FWD);
          k_bfs_fwd<G><<<grid, kThreads, 0, s>>>(g, level + i, ep);
        }
      }
      level += steps;
      st = sync_ctl(pb, s);
      if (st) return st;
    }
  }
  *levels_out = level;
  return FP_OK;
}

template <int G>
static fp_status global_relabel(fp_problem* pb, hipStream_t s) {
  Dev& g = pb->dev;
  {
    Launch L(pb, s, KK_GR_RESET);
    k_gr_reset<<<sweep_grid(g.N), kThreads, 0, s>>>(g);
  }
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, -1, &levels);
  if (st) return st;
  {
    Launch L(pb, s, KK_GATHER);
    k_gather<<<sweep_grid(g.N), kThreads, 0, s>>>(g, pb->epoch);
  }
  pb->st.global_relabels++;
  pb->st.bfs_levels += levels;
  return sync_ctl(pb, s);
}

static fp_status debug_check(fp_problem* pb, hipStream_t s) {
  Dev& g = pb->dev;
  {
    Launch L(pb, s, KK_CHECK);
    k_check<<<sweep_grid(std::max(g.P, std::max(g.E, g.V))), kThreads, 0, s>>>(g);
  }
  fp_status st = sync_ctl(pb, s);
  if (st) return st;
  if (pb->ctl_h->err & ERR_INVARIANT) {
    set_error("debug check: preflow or labelling invariant violated after round %lld",
              (long long)pb->st.rounds);
    return FP_ERR_DEVICE;
  }
  return FP_OK;
}

template <int G>
static fp_status solve_impl(fp_problem* pb, hipStream_t s, int64_t* flow) {
  Dev& g = pb->dev;
  fp_status st;
  if (!pb->inited) {
    {
      Launch L(pb, s, KK_INIT);
      k_init<<<sweep_grid(std::max(g.P, g.N)), kThreads, 0, s>>>(g);
    }
    pb->inited = true;
  }
  st = global_relabel<G>(pb, s);
  if (st) return st;
  const unsigned long long budget =
      (unsigned long long)((double)g.N * pb->opt.relabel_factor_x16 / 16.0) + 1ull;
  unsigned long long rel_at_gr = pb->ctl_h->relabels;
  bool fresh_gr = true;  // frontier was just gathered by a global relabel
  const int cap = pb->opt.tail_threshold;
  const int rounds_per_sync = pb->opt.debug_checks ? 1 : 8;
  int64_t rounds_this_solve = 0;
  for (;;) {
    if (pb->ctl_h->err & ERR_LABEL) {
      set_error("internal check: a relabel did not raise a label");
      return FP_ERR_DEVICE;
    }
    const int c3 = pb->epoch % 3;
    const long long nf = (long long)pb->ctl_h->fcnt[c3][0] + pb->ctl_h->fcnt[c3][1];
    if (nf == 0) {
      if (fresh_gr) break;
      // apparent termination: confirm with exact labels, restart if active
      // nodes remain (paper, section "A Bug in the Synchronous Algorithm")
      st = global_relabel<G>(pb, s);
      if (st) return st;
      rel_at_gr = pb->ctl_h->relabels;
      fresh_gr = true;
      const int c3b = pb->epoch % 3;
      if (pb->ctl_h->fcnt[c3b][0] + pb->ctl_h->fcnt[c3b][1] > 0) pb->st.restarts++;
      continue;
    }
    if (rounds_this_solve > kRoundGuard) {
      set_error("no convergence after %lld rounds", (long long)rounds_this_solve);
      return FP_ERR_DEVICE;
    }
    if (pb->opt.round_budget > 0 && rounds_this_solve >= pb->opt.round_budget) {
      set_error("round budget of %d rounds exhausted", pb->opt.round_budget);
      return FP_ERR_ABORTED;
    }
    fresh_gr = false;
    if (nf <= cap && !pb->opt.debug_checks) {
      int max_rounds = 1 << 16;  // per launch; the host loop continues
      if (pb->opt.round_budget > 0)
        max_rounds = (int)std::min<int64_t>(max_rounds, pb->opt.round_budget - rounds_this_solve);
      {
        Launch L(pb, s, KK_ROUND_LOOP);
        k_round_loop<G><<<1, kLoopThreads, 0, s>>>(g, pb->epoch, max_rounds, cap,
                                                  rel_at_gr + budget);
      }
      st = sync_ctl(pb, s);
      if (st) return st;
      const int r = pb->ctl_h->loop_rounds;
      pb->epoch += r;
      pb->st.rounds += r;
      pb->st.tail_rounds += r;
      rounds_this_solve += r;
    } else {
      const int grid = frontier_grid(nf);
      for (int i = 0; i < rounds_per_sync; ++i) {
        {
          Launch L(pb, s, KK_PUSH);
          k_push<G><<<grid, kThreads, 0, s>>>(g, pb->epoch);
        }
        {
          Launch L(pb, s, KK_APPLY);
          k_apply<<<grid, kThreads, 0, s>>>(g, pb->epoch);
        }
        pb->epoch++;
      }
      pb->st.rounds += rounds_per_sync;
      rounds_this_solve += rounds_per_sync;
      if (pb->opt.debug_checks) {
        st = debug_check(pb, s);
        if (st) return st;
      } else {
        st = sync_ctl(pb, s);
        if (st) return st;
      }
    }
    if (pb->ctl_h->relabels - rel_at_gr >= budget) {
      st = global_relabel<G>(pb, s);
      if (st) return st;
      rel_at_gr = pb->ctl_h->relabels;
      fresh_gr = true;
    }
  }
  if (pb->ctl_h->err & ERR_LABEL) {
    set_error("internal check: a relabel did not raise a label");
    return FP_ERR_DEVICE;
  }
  pb->st.relabels = (int64_t)pb->ctl_h->relabels;
  pb->st.flow_value = (int64_t)pb->ctl_h->flow;
  pb->solved = true;
  *flow = (int64_t)pb->ctl_h->flow;
  return FP_OK;
}

fp_status solve_problem(fp_problem* pb, hipStream_t s, int64_t* flow) {
  switch (pb->opt.group_lanes) {
    case 4: return solve_impl<4>(pb, s, flow);
    case 16: return solve_impl<16>(pb, s, flow);
    default: return solve_impl<8>(pb, s, flow);
  }
}

template <int G>
static fp_status cut_impl(fp_problem* pb, hipStream_t s, uint8_t* vs, uint8_t* ns) {
  Dev& g = pb->dev;
  const int ep = pb->epoch++;
  {
    Launch L(pb, s, KK_CUT_SEED);
    k_cut_seed<<<sweep_grid(g.N), kThreads, 0, s>>>(g, ep);
  }
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, ep, &levels);
  if (st) return st;
  pb->st.bfs_levels += levels;
  {
    Launch L(pb, s, KK_CUT_OUT);
    k_cut_out<<<sweep_grid(std::max(g.V, g.E)), kThreads, 0, s>>>(g, ep, vs, ns);
  }
  st = sync_ctl(pb, s);
  if (st) return st;
  if (pb->ctl_h->err & ERR_SINK_REACHED) {
    set_error("internal check: a sink is reachable from the source side");
    return FP_ERR_DEVICE;
  }
  return FP_OK;
}

fp_status cut_problem(fp_problem* pb, hipStream_t s, int32_t mem_kind, uint8_t* vside,
                      uint8_t* nside) {
  if (!pb->solved) {
    set_error("mincut_source_side called before a successful maxflow_solve");
    return FP_ERR_STATE;
  }
  uint8_t* vs = vside;
  uint8_t* ns = nside;
  if (mem_kind == 0) {  // stage in the relabel list memory (8N bytes >= V + E)
    vs = reinterpret_cast<uint8_t*>(pb->dev.left);
    ns = nside ? vs + pb->V : nullptr;
  }
  fp_status st;
  switch (pb->opt.group_lanes) {
    case 4: st = cut_impl<4>(pb, s, vs, ns); break;
    case 16: st = cut_impl<16>(pb, s, vs, ns); break;
    default: st = cut_impl<8>(pb, s, vs, ns); break;
  }
  if (st) return st;
  if (mem_kind == 0) {
    hipError_t he = hipMemcpyAsync(vside, vs, pb->V, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess && nside && pb->E)
      he = hipMemcpyAsync(nside, ns, pb->E, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "copying the cut to the host");
  }
  return FP_OK;
}

fp_status batch_solve(fp_problem* const* pbs, int32_t count, const uint8_t* skip,
                      hipStream_t s, int64_t* flows) {
  // plain schedule: one problem after the other with the same kernels
  for (int32_t i = 0; i < count; ++i) {
    if (skip && skip[i]) {
      flows[i] = -1;
      continue;
    }
    fp_status st = solve_problem(pbs[i], s, &flows[i]);
    if (st) return st;
  }
  return FP_OK;
}

fp_status pierce_problem(fp_problem*, int32_t, const int32_t*, int32_t, hipStream_t) {
  set_error("flow_problem_pierce is not available in this build");
  return FP_ERR_STATE;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------

const char* kernel_kind_name(int k) {
  static const char* names[KK_COUNT] = {
      "init",      "gr_reset", "bfs_rev",       "bfs_rev_loop", "gather",
      "push",      "apply",    "round_loop",    "cut_seed",     "bfs_fwd",
      "bfs_fwd_loop", "cut_out", "check",       "batch"};
  return (k >= 0 && k < KK_COUNT) ? names[k] : "?";
}

int kernel_kind_class(int k) {
  switch (k) {
    case KK_PUSH: return KC_PUSH;
    case KK_APPLY: return KC_APPLY;
    case KK_BFS_REV: return KC_BFS_REV;
    case KK_BFS_FWD: return KC_BFS_FWD;
    case KK_ROUND_LOOP: return KC_LOOP_ROUNDS;
    case KK_BFS_REV_LOOP:
    case KK_BFS_FWD_LOOP: return KC_LOOP_BFS;
    default: return -1;
  }
}

static hipEvent_t get_event(fp_problem* pb) {
  if (!pb->free_events.empty()) {
    hipEvent_t e = pb->free_events.back();
    pb->free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(fp_problem* pb, int kind, hipStream_t s, Timer* t) {
  t->kind = kind;
  t->a = get_event(pb);
  t->b = get_event(pb);
  (void)hipEventRecord(t->a, s);
}

void prof_end(fp_problem* pb, Timer* t, hipStream_t s) {
  (void)hipEventRecord(t->b, s);
  pb->pending.push_back(*t);
}

void prof_collect(fp_problem* pb) {
  for (auto& t : pb->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      pb->k_ms[t.kind] += ms;
      pb->k_launches[t.kind]++;
    }
    pb->free_events.push_back(t.a);
    pb->free_events.push_back(t.b);
  }
  pb->pending.clear();
}

}  // namespace hf
