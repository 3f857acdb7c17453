// Solver kernels and their host orchestration.
//
// Large frontiers run as device-wide kernels (one launch per phase, the
// kernel boundary is the ordering point).  Frontiers at or below the tail
// threshold run inside one workgroup that loops over rounds (or BFS levels)
// with workgroup barriers, so the long power-law tail of small rounds the
// paper observes (paragraph "Avoid Pushing Flow Back") costs no launches and
// no host round trips.  Both paths call the same phase functions.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <hip/hip_ext.h>

#include <map>
#include <mutex>

#include "hf_host.h"

namespace hf {

constexpr int kThreads = 256;  // plain element-wise kernels
constexpr int kBlock = 1024;   // frontier, sweep and single-workgroup kernels
constexpr int kFcGrid = 128;   // FlowCutter weight and candidate sweeps
constexpr int kLoopBlock = 512;  // the single-workgroup round loop (1024 threads spill 48 bytes a lane)
constexpr int kMaxFrontierBlocks = 512;
static_assert(kMaxFrontierBlocks <= kMaxSliceGroups, "one slice segment per scan workgroup");
constexpr int kMaxSweepBlocks = 512;
constexpr long long kRoundGuard = 200000000ll;  // rounds per solve before giving up

__device__ __forceinline__ int gwave() { return (blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ __forceinline__ int gwaves() { return (gridDim.x * blockDim.x) >> 6; }
__device__ __forceinline__ int gthread() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int gthreads() { return gridDim.x * blockDim.x; }

// BFS level kernels are latency bound: ask the compiler to fit eight waves per
// SIMD (two 1024-thread workgroups per CU, which the LDS allows), spilling a
// few scalar registers into vector lanes instead of leaving one workgroup per
// CU.
#define HF_TWO_WORKGROUPS_PER_CU __attribute__((amdgpu_waves_per_eu(8)))

// LDS staging area of the workgroup's list appends
#define HF_QUEUE_LDS __shared__ int32_t hf_bq[lds_words(kBlock)]; lds_int* const lds = (lds_int*)hf_bq

__global__ void __launch_bounds__(kThreads) k_init(Dev g) { phase_init(g, gthread(), gthreads()); }

__global__ void __launch_bounds__(kThreads) k_gr_bits(Dev g) {
  phase_gr_bits(g, gthread(), gthreads());
}

__global__ void __launch_bounds__(kBlock) k_gr_reset(Dev g) {
  HF_QUEUE_LDS;
  phase_gr_reset(g, blockIdx.x, gridDim.x, lds);
}

// One level of the reverse BFS.  A level holding at least `big_min` nodes
// is only expanded here (plain stores) and k_bfs_collect lists the next
// level; smaller levels claim and list new nodes directly.  Both kernels read
// the same count, so they agree on the mode.  A level larger than `tail`
// (the single-workgroup loop's bound) is recorded in big_last, from which the
// host sizes the first batch of level launches of the next global relabel.
template <int G>
__global__ void __launch_bounds__(kBlock) HF_TWO_WORKGROUPS_PER_CU
k_bfs_rev(Dev g, int level, int big_min, int pull_min, int tail) {
  HF_QUEUE_LDS;
  const int c3 = level % 3;
  const int nf = count_all(g.ctl->bcnt[c3]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (nf > tail) atomicMax(&g.ctl->big_last, level);
    if (level < kLvlHist) g.ctl->lvl_nf[level] = nf;
  }
  if (nf >= pull_min)
    phase_bfs_rev_pull(g, level, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                       KC_BFS_REV);
  else if (nf >= big_min)
    phase_bfs_rev_expand<G>(g, level, blockIdx.x, gridDim.x, KC_BFS_REV, lds);
  else phase_bfs_rev<G>(g, level, blockIdx.x, gridDim.x, KC_BFS_REV, lds);
}

// The same level with the expanded (large) levels' arcs flattened per wave
// (phase_bfs_rev_flat), a kernel of its own so that neither variant's
// register and inlining budget weighs on the other.  Claiming levels stay
// node-grouped: they are the smaller ones, and 64 nodes per wave leave most
// of the grid idle there.
template <int G>
__global__ void __launch_bounds__(kBlock) HF_TWO_WORKGROUPS_PER_CU
k_bfs_rev_flat(Dev g, int level, int big_min, int pull_min, int tail) {
  HF_QUEUE_LDS;
  const int c3 = level % 3;
  const int nf = count_all(g.ctl->bcnt[c3]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (nf > tail) atomicMax(&g.ctl->big_last, level);
    if (level < kLvlHist) g.ctl->lvl_nf[level] = nf;
  }
  if (nf >= pull_min)
    phase_bfs_rev_pull(g, level, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                       KC_BFS_REV);
  else if (nf >= big_min)
    phase_bfs_rev_flat<false>(g, level, blockIdx.x, gridDim.x, KC_BFS_REV, lds);
  else phase_bfs_rev_node<G, true>(g, level, blockIdx.x, gridDim.x, KC_BFS_REV, lds);
}

// As k_bfs_rev_flat, with expanded levels split in two (XCD-local labels):
// this kernel scans the level's arcs and hands each head that is not
// labelled yet to its slice; k_bfs_slices then labels the heads of each
// slice on the XCD that owns it.
template <int G>
__global__ void __launch_bounds__(kBlock) HF_TWO_WORKGROUPS_PER_CU
k_bfs_rev_xflat(Dev g, int level, int big_min, int pull_min, int tail) {
  HF_QUEUE_LDS;
  const int c3 = level % 3;
  const int nf = count_all(g.ctl->bcnt[c3]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (nf > tail) atomicMax(&g.ctl->big_last, level);
    if (level < kLvlHist) g.ctl->lvl_nf[level] = nf;
  }
  if (nf >= pull_min)
    phase_bfs_rev_pull(g, level, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                       KC_BFS_REV);
  else if (nf >= big_min)
    phase_bfs_rev_flat<false, true>(g, level, blockIdx.x, gridDim.x, KC_BFS_REV, lds);
  else phase_bfs_rev_node<G, true>(g, level, blockIdx.x, gridDim.x, KC_BFS_REV, lds);
}

// nseg: the grid of the k_bfs_rev_xflat launch of this level.
__global__ void __launch_bounds__(kBlock) k_bfs_slices(Dev g, int level, int big_min,
                                                       int pull_min, int nseg) {
  const int nf = count_all(g.ctl->bcnt[level % 3]);
  if (nf >= big_min && nf < pull_min) phase_bfs_slices(g, level, nseg);
}

// Expanded and pulled levels list their new nodes by a sweep over the labels.
__global__ void __launch_bounds__(kBlock) k_bfs_collect(Dev g, int level, int big_min,
                                                        int pull_min) {
  HF_QUEUE_LDS;
  const int c3 = level % 3;
  const int nf = count_all(g.ctl->bcnt[c3]);
  if (nf >= min(big_min, pull_min)) phase_bfs_collect(g, level, blockIdx.x, gridDim.x, lds);
}

__global__ void k_clear_frontiers(Dev g) { phase_clear_frontiers(g); }

__global__ void __launch_bounds__(kBlock) k_gather(Dev g, int epoch) {
  HF_QUEUE_LDS;
  phase_gather(g, epoch, blockIdx.x, gridDim.x, lds);
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_push(Dev g, int epoch) {
  HF_QUEUE_LDS;
  phase_push<G>(g, epoch, blockIdx.x, gridDim.x, KC_PUSH, lds);
}

__global__ void __launch_bounds__(kBlock) k_apply(Dev g, int epoch) {
  HF_QUEUE_LDS;
  phase_apply(g, epoch, blockIdx.x, gridDim.x, KC_APPLY, lds);
}

__global__ void __launch_bounds__(kBlock) k_cut_seed(Dev g, int ep, int only_new) {
  HF_QUEUE_LDS;
  phase_cut_seed(g, ep, only_new != 0, blockIdx.x, gridDim.x, lds);
}

// One level of the forward BFS (source side).  A level holding at least
// `big_min` nodes gives its new nodes a provisional stamp (plain stores) and
// k_bfs_fwd_collect lists them; smaller levels claim and list directly.
template <int G>
__global__ void __launch_bounds__(kBlock) HF_TWO_WORKGROUPS_PER_CU
k_bfs_fwd(Dev g, int level, int ep, int big_min, int ep_tmp) {
  HF_QUEUE_LDS;
  const int nf = count_all(g.ctl->bcnt[level % 3]);
  if (nf >= big_min)
    phase_bfs_fwd_expand<G>(g, level, ep, ep_tmp, blockIdx.x, gridDim.x, KC_BFS_FWD, lds);
  else phase_bfs_fwd<G>(g, level, ep, blockIdx.x, gridDim.x, KC_BFS_FWD, lds);
}

__global__ void __launch_bounds__(kBlock) k_bfs_fwd_collect(Dev g, int level, int ep, int ep_tmp,
                                                            int big_min) {
  HF_QUEUE_LDS;
  const int nf = count_all(g.ctl->bcnt[level % 3]);
  if (nf >= big_min) phase_bfs_fwd_collect(g, level, ep, ep_tmp, blockIdx.x, gridDim.x, lds);
}

template <int G>
__global__ void __launch_bounds__(kBlock) HF_TWO_WORKGROUPS_PER_CU
k_bfs_sink(Dev g, int level, int ep) {
  HF_QUEUE_LDS;
  phase_bfs_sink<G>(g, level, ep, blockIdx.x, gridDim.x, KC_BFS_FWD, lds);
}

__global__ void __launch_bounds__(kBlock) k_sink_seed(Dev g, int ep) {
  HF_QUEUE_LDS;
  phase_sink_seed(g, ep, blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(kBlock) k_sink_seed_labels(Dev g, int ep) {
  HF_QUEUE_LDS;
  phase_sink_seed_labels(g, ep, blockIdx.x, gridDim.x, lds);
}

__global__ void k_reset_bfs(Dev g) { phase_reset_bfs(g); }

__global__ void k_seed_vertex(Dev g, int p) { phase_seed_vertex(g, p); }

__global__ void __launch_bounds__(kThreads) k_side_out(Dev g, int ep, int invert, uint8_t* vs) {
  phase_side_out(g, ep, invert != 0, vs, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_fc_weights(Dev g, const int32_t* cw, int ep_s,
                                                         int ep_t) {
  phase_fc_weights(g, cw, ep_s, ep_t, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_fc_pick(Dev g, int ep_s, int ep_t) {
  phase_fc_pick(g, ep_s, ep_t);
}

__global__ void __launch_bounds__(kThreads) k_fc_mark_augmenting(Dev g, int side, int ep_s,
                                                                 int ep_t, uint8_t* flag) {
  phase_fc_mark_augmenting(g, side, ep_s, ep_t, flag, gthread(), gthreads());
}

__global__ void __launch_bounds__(kBlock) k_count_flags(const uint8_t* flag, int V,
                                                        int32_t* counts) {
  phase_count_flags(flag, V, counts);
}

// exclusive scan of n tile counts in place, total to counts[n]; one workgroup
__global__ void __launch_bounds__(kBlock) k_scan_counts(int32_t* counts, int n) {
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const int c = i < n ? counts[i] : 0;
    // inclusive scan over the workgroup in LDS (Hillis-Steele)
    __shared__ int buf[kBlock];
    buf[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      const int t = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) counts[i] = carry + buf[threadIdx.x] - c;
    __syncthreads();
    if (threadIdx.x == 0) carry += buf[blockDim.x - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[n] = carry;
}

__global__ void __launch_bounds__(kBlock) k_select_flags(Dev g, const uint8_t* flag, int V,
                                                         const int32_t* offsets, int k, int ep) {
  phase_select_flags(g, flag, V, offsets, k, ep);
}

__global__ void k_stamp_vertex(Dev g, int p, int ep) {
  if (threadIdx.x == 0) g.stamp[p] = ep;
}

__global__ void __launch_bounds__(kBlock) k_pierce_sources_seed(Dev g, int ep_s) {
  HF_QUEUE_LDS;
  phase_pierce_sources_seed(g, ep_s, blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(kThreads) k_pierce_sources(Dev g, int ep_s) {
  phase_pierce_sources(g, ep_s, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_pierce_sinks(Dev g, int ep_t) {
  phase_pierce_sinks(g, ep_t, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_mark(Dev g, const int32_t* vs, int n, int ep,
                                                   int forbidden) {
  phase_mark(g, vs, n, ep, forbidden, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_cut_out(Dev g, int ep, uint8_t* vs, uint8_t* ns) {
  phase_cut_out(g, ep, vs, ns, gthread(), gthreads());
}

__global__ void __launch_bounds__(kThreads) k_check(Dev g) {
  phase_check(g, gthread(), gthreads());
}

// Rounds inside one workgroup.  All waves of the workgroup share one CU, so
// a workgroup barrier orders their global memory traffic; no device-scope
// fence (which would write back and invalidate the L2) is needed.  Stops when
// the frontier is empty (1), exceeds `cap` (2), `max_rounds` rounds ran (3),
// the relabel count reached `relabel_limit` (4), or the flow value did not
// change for `stale_limit` rounds (5).  The exit tests read values that no
// wave writes between the barrier and the test, so every wave takes the same
// decision.
template <int G>
__global__ void __launch_bounds__(kLoopBlock) k_round_loop(Dev g, int epoch0, int max_rounds,
                                                           int cap,
                                                           unsigned long long relabel_limit,
                                                           int stale_limit) {
  __shared__ int32_t hf_bq[lds_words(kLoopBlock)];
  lds_int* const lds = (lds_int*)hf_bq;
  int epoch = epoch0;
  int r = 0;
  int why = 0;
  int stale = 0;
  unsigned long long last_flow = ld_vol64(&g.ctl->flow);
  for (;;) {
    const int c3 = epoch % 3;
    const int nf = count_all_vol(g.ctl->fcnt[c3]);
    const unsigned long long fl = ld_vol64(&g.ctl->flow);
    if (fl != last_flow) {
      last_flow = fl;
      stale = 0;
    }
    if (nf == 0) { why = 1; break; }
    if (nf > cap) { why = 2; break; }
    if (r >= max_rounds) { why = 3; break; }
    if (ld_vol64(&g.ctl->relabels) >= relabel_limit) { why = 4; break; }
    if (stale_limit > 0 && stale >= stale_limit) { why = 5; break; }
    __syncthreads();  // every wave has read the counters before they change
    phase_push<G>(g, epoch, 0, 1, KC_LOOP_ROUNDS, lds);
    __syncthreads();
    phase_apply(g, epoch, 0, 1, KC_LOOP_ROUNDS, lds);
    __syncthreads();
    ++epoch;
    ++r;
    ++stale;
  }
  if (threadIdx.x == 0) {
    g.ctl->loop_rounds = r;
    g.ctl->loop_exit = why;
  }
}

// BFS levels inside one workgroup: mode 0 the global relabel (reverse,
// capped), 1 the source side (forward, uncapped), 2 the sink side (reverse,
// uncapped).  Levels this small are latency bound: arc-parallel levels spread
// even one node's arcs over the whole workgroup, which node-grouped levels do
// not (the FlowCutter's incremental sides run here: 1.92 -> 1.85 s on the
// 200k-vertex region).
template <int G>
__global__ void __launch_bounds__(kBlock) k_bfs_loop(Dev g, int level0, int cap, int ep,
                                                     int mode) {
  HF_QUEUE_LDS;
  int level = level0;
  for (;;) {
    const int c3 = level % 3;
    const int nf = count_all_vol(g.ctl->bcnt[c3]);
    if (nf == 0 || nf > cap) break;
    if (mode == 0 && threadIdx.x == 0 && level < kLvlHist) g.ctl->lvl_nf[level] = nf;
    __syncthreads();
    if (mode == 0) phase_bfs_rev_lb<true>(g, level, 0, 1, KC_LOOP_BFS, lds);
    else if (mode == 1) phase_bfs_fwd_lb<true>(g, level, ep, 0, 0, 1, KC_LOOP_BFS, lds);
    else phase_bfs_sink_lb(g, level, ep, 0, 1, KC_LOOP_BFS, lds);
    __syncthreads();
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

// grid for a sweep over n nodes (tiles of 2 * kBlock nodes)
static int sweep_blocks(long long n) {
  long long b = (n + 2 * kBlock - 1) / (2 * kBlock);
  if (b < 1) b = 1;
  if (b > kMaxSweepBlocks) b = kMaxSweepBlocks;
  return (int)b;
}

static hipEvent_t get_event(fp_problem* pb);

// Launch of the reverse-BFS level kernel.  With its timing on, the start and
// stop events are recorded by the dispatch itself (hipExtLaunchKernel): the
// time is the kernel's own, and no marker packets sit between the launches
// of a batch of levels.
template <typename... KArgs, typename... Args>
static void launch_timed(fp_problem* pb, hipStream_t s, void (*kernel)(KArgs...), dim3 grid,
                         dim3 block, Args... args) {
  const bool on = pb->opt.profile == 1 || pb->opt.profile == 2;
  hipEvent_t a = on ? get_event(pb) : nullptr;
  hipEvent_t b = on ? get_event(pb) : nullptr;
  if (!a || !b) {
    event_pool_put(pb->device, a);  // a null event is ignored
    event_pool_put(pb->device, b);
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
  pb->pending.push_back(Timer{KK_BFS_REV, a, b});
}

struct Launch {
  fp_problem* pb;
  hipStream_t s;
  Timer t;
  bool on;
  // profile 1: every kernel; profile 2: only the reverse-BFS level kernel
  Launch(fp_problem* p, hipStream_t st, int kind)
      : pb(p), s(st), on(p->opt.profile == 1 || (p->opt.profile == 2 && kind == KK_BFS_REV)) {
    if (on) prof_begin(pb, kind, s, &t);
  }
  ~Launch() {
    if (on) prof_end(pb, &t, s);
  }
};

static long long host_count(const int32_t* c) {
  long long n = 0;
  for (int k = 0; k < kNL; ++k) n += c[k];
  return n;
}

static bool trace_on() {
  static const bool on = [] {
    const char* e = getenv("HYPERFLOW_TRACE");
    return e && e[0] && e[0] != '0';
  }();
  return on;
}

static fp_status sync_ctl(fp_problem* pb, hipStream_t s, const char* what = "") {
  hipError_t he = hipGetLastError();
  if (he == hipSuccess)
    he = hipMemcpyAsync(pb->ctl_h, pb->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "solver step");
  pb->st.host_syncs++;
  if (trace_on()) {
    const Ctl* c = pb->ctl_h;
    const int c3 = pb->epoch % 3;
    fprintf(stderr,
            "[hyperflow] %-10s epoch=%d rounds=%lld flow=%llu frontier=%d/%d/%d/%d bfs=%d|%d|%d "
            "relabels=%llu loop=%d/%d/%d\n",
            what, pb->epoch, (long long)pb->st.rounds, c->flow, c->fcnt[c3][0], c->fcnt[c3][1],
            c->fcnt[c3][2], c->fcnt[c3][3], host_count(c->bcnt[0]), host_count(c->bcnt[1]),
            host_count(c->bcnt[2]), c->relabels, c->loop_rounds, c->loop_levels, c->loop_exit);
  }
  if (pb->opt.profile) prof_collect(pb);
  return FP_OK;
}

// Device-wide BFS levels level .. level+steps-1 of the given mode.  With
// `predict`, a reverse-BFS level that the previous global relabel also
// reached is sized from that relabel's level and its two neighbours: a level
// expected to be small runs on a smaller grid (128 workgroups at least) and
// may not expand (it claims, so no collect sweep is launched for it).  Both
// choices change only the schedule: any grid covers any level, and claiming
// is correct at every size.
template <int G>
static void launch_levels(fp_problem* pb, hipStream_t s, int ep, int ep_tmp, int mode, int level,
                          int steps, bool predict) {
  Dev& g = pb->dev;
  const int cap = pb->opt.tail_threshold;
  const int big_min = pb->opt.bottom_up_min > 0 ? pb->opt.bottom_up_min : (1 << 30);
  const int pull_min = pb->opt.pull_min > 0 ? pb->opt.pull_min : (1 << 30);
  const int off = 1 << 30;
  for (int i = 0; i < steps; ++i) {
    const int lv = level + i;
    if (mode == 0) {
      int grid = kMaxFrontierBlocks, bmin = big_min, pmin = pull_min;
      if (predict && lv < pb->gr_hist_levels) {
        long long p = 0;
        for (int j = lv - 1; j <= lv + 1; ++j)
          if (j >= 0 && j < pb->gr_hist_levels) p = std::max<long long>(p, pb->gr_hist[j]);
        grid = (int)std::min<long long>(kMaxFrontierBlocks, std::max<long long>(128, (2 * p + 63) / 64));
        if (2 * p < big_min) bmin = off;
        if (2 * p < pull_min) pmin = off;
      }
      const bool xcd = g.xbuf && g.bfs_flat && !g.bfs_arc;
      if (xcd) launch_timed(pb, s, k_bfs_rev_xflat<G>, dim3(grid), dim3(kBlock), g, lv, bmin, pmin, cap);
      else if (g.bfs_flat && !g.bfs_arc)
        launch_timed(pb, s, k_bfs_rev_flat<G>, dim3(grid), dim3(kBlock), g, lv, bmin, pmin, cap);
      else launch_timed(pb, s, k_bfs_rev<G>, dim3(grid), dim3(kBlock), g, lv, bmin, pmin, cap);
      if (xcd && bmin != off) {
        Launch L(pb, s, KK_BFS_REV);
        k_bfs_slices<<<kSlices * 64, kBlock, 0, s>>>(g, lv, bmin, pmin, grid);
      }
      if (bmin != off || pmin != off) {
        Launch L(pb, s, KK_BFS_COLLECT);
        k_bfs_collect<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, lv, bmin, pmin);
      }
    } else if (mode == 1) {
      {
        Launch L(pb, s, KK_BFS_FWD);
        k_bfs_fwd<G><<<kMaxFrontierBlocks, kBlock, 0, s>>>(g, lv, ep, big_min, ep_tmp);
      }
      if (big_min != off) {
        Launch L(pb, s, KK_BFS_COLLECT);
        k_bfs_fwd_collect<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, lv, ep, ep_tmp, big_min);
      }
    } else {
      Launch L(pb, s, KK_BFS_FWD);
      k_bfs_sink<G><<<kMaxFrontierBlocks, kBlock, 0, s>>>(g, lv, ep);
    }
  }
}

template <int G>
static fp_status run_bfs(fp_problem* pb, hipStream_t s, int ep, int mode, int* levels_out,
                         long long level0_count = -1, int level_start = 0) {
  // Level `level_start` (0 unless the caller continues a search) is already
  // in its ring slot (level0_count nodes when the caller knows).  mode 0
  // global relabel (ep unused), 1 source side, 2 sink side (stamps ep).
  //
  // Levels are launched in batches without reading their sizes: a batch of
  // device-wide levels is followed by the single-workgroup loop, which runs
  // the levels that follow while they hold at most `cap` nodes and exits at
  // once otherwise; one host round trip per batch then reads where the BFS
  // stands.  A global relabel's first batch is as long as the previous
  // relabel's device-wide part (big_last + 1), so a relabel usually costs one
  // round trip.  Levels with no nodes do nothing, so launching past the end
  // of a BFS is safe.  With the invariant checker on, every level is
  // device-wide and every batch is read back.
  Dev& g = pb->dev;
  const int cap = pb->opt.tail_threshold;
  const bool use_loop = !pb->opt.debug_checks;
  // provisional stamp of the forward BFS's expanded levels (never a stamp
  // value of anything else)
  const int ep_tmp = mode == 1 ? pb->epoch++ : 0;
  int level = level_start;
  long long nf = level0_count;  // size of `level`, < 0 while unknown on the host
  fp_status st = FP_OK;
  // only a global relabel starts without reading the size of level 0 (its
  // sinks are many in the common case); the other searches often start small
  if (nf < 0 && (!use_loop || mode != 0)) {
    st = sync_ctl(pb, s);
    if (st) return st;
    nf = host_count(pb->ctl_h->bcnt[level % 3]);
  }
  bool first = true;
  for (;;) {
    if (nf == 0) break;
    // a level holds distinct nodes and a BFS has at most N levels
    if (nf > g.N || level > g.N + 16) {
      set_error("internal check: BFS level %d holds %lld nodes (N = %d)", level, nf, g.N);
      return FP_ERR_DEVICE;
    }
    int steps = 0;
    const bool predict = mode == 0 && use_loop && pb->gr_hist_levels > 0;
    if (!use_loop || nf > cap || (nf < 0 && g.N > cap)) {
      steps = 8;
      if (mode == 0 && first && use_loop) steps = pb->gr_batch;
    }
    first = false;
    launch_levels<G>(pb, s, ep, ep_tmp, mode, level, steps, predict);
    if (use_loop) {
      Launch L(pb, s, mode == 0 ? KK_BFS_REV_LOOP : KK_BFS_FWD_LOOP);
      k_bfs_loop<G><<<1, kBlock, 0, s>>>(g, level + steps, cap, ep, mode);
    }
    st = sync_ctl(pb, s, "bfs");
    if (st) return st;
    level += steps + (use_loop ? pb->ctl_h->loop_levels : 0);
    nf = host_count(pb->ctl_h->bcnt[level % 3]);
  }
  if (mode == 0) {
    pb->gr_batch = std::min(kLvlHist, std::max(1, pb->ctl_h->big_last + 1));
    pb->gr_hist_levels = std::min(level, kLvlHist);
    for (int j = 0; j < pb->gr_hist_levels; ++j) pb->gr_hist[j] = pb->ctl_h->lvl_nf[j];
    if (trace_on()) {
      fprintf(stderr, "[hyperflow] relabel levels:");
      for (int j = 0; j < pb->gr_hist_levels; ++j) fprintf(stderr, " %d", pb->gr_hist[j]);
      fprintf(stderr, "\n");
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
    k_gr_reset<<<sweep_blocks(g.N), kBlock, 0, s>>>(g);
    k_gr_bits<<<sweep_grid(std::max(g.P, g.E)), kThreads, 0, s>>>(g);
  }
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, -1, 0, &levels);
  if (st) return st;
  {
    Launch L(pb, s, KK_GATHER);
    k_gather<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, pb->epoch);
  }
  pb->st.global_relabels++;
  pb->st.bfs_levels += levels;
  return sync_ctl(pb, s, "gather");
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
  // After a source pierce the labels are still valid (paragraph "Maintain
  // Distance Labels"): the solve only gathers the active nodes, and its end
  // is confirmed by a global relabel as usual.  Otherwise it starts with one.
  const bool warm = pb->warm_labels && pb->inited;
  pb->warm_labels = false;
  pb->labels_exact = false;
  if (warm) {
    {
      Launch L(pb, s, KK_GATHER);
      k_clear_frontiers<<<1, 64, 0, s>>>(g);
      k_gather<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, pb->epoch);
    }
    st = sync_ctl(pb, s, "gather");
  } else {
    st = global_relabel<G>(pb, s);
  }
  if (st) return st;
  // global relabel triggers (paper: "after linear push and relabel work",
  // and the stale-flow rule of paragraph "Avoid Pushing Flow Back")
  const unsigned long long budget =
      (unsigned long long)((double)g.N * pb->opt.relabel_factor_x16 / 16.0) + 1ull;
  const int gr_interval = pb->opt.gr_interval;
  // Once the frontier fits one workgroup, rounds cost a few microseconds and
  // a global relabel (a BFS over every node) as much as two hundred of them,
  // so the tail relabels less often (7.4M-pin flows, three seeds: every 64
  // tail rounds is at most as slow as every 16 on each seed).
  const int tail_interval = pb->opt.tail_gr_interval > 0 ? pb->opt.tail_gr_interval
                            : pb->opt.tail_gr_interval < 0 ? gr_interval
                                                           : 4 * gr_interval;
  const int stale_limit = pb->opt.stale_rounds;
  constexpr long long kStaleFrontier = 1500;  // "only few active nodes" (paper)
  unsigned long long rel_at_gr = pb->ctl_h->relabels;
  unsigned long long last_flow = pb->ctl_h->flow;
  long long stale = 0;
  long long rounds_since_gr = 0;
  bool fresh_gr = !warm;  // frontier was just gathered by a global relabel
  const int cap = pb->opt.tail_threshold;
  const int rounds_per_sync = pb->opt.debug_checks ? 1 : 8;
  int64_t rounds_this_solve = 0;
  for (;;) {
    if (pb->ctl_h->err & ERR_LABEL) {
      set_error("internal check: a relabel did not raise a label");
      return FP_ERR_DEVICE;
    }
    const int c3 = pb->epoch % 3;
    const long long nf = host_count(pb->ctl_h->fcnt[c3]);
    bool do_gr = false;
    bool in_tail = false;  // these rounds ran in the single-workgroup loop
    if (nf == 0) {
      if (fresh_gr) break;
      // apparent termination: confirm with exact labels and restart if
      // active nodes remain (paper, section "A Bug in the Synchronous
      // Algorithm")
      st = global_relabel<G>(pb, s);
      if (st) return st;
      const int c3b = pb->epoch % 3;
      if (host_count(pb->ctl_h->fcnt[c3b]) > 0) pb->st.restarts++;
      rel_at_gr = pb->ctl_h->relabels;
      rounds_since_gr = 0;
      stale = 0;
      fresh_gr = true;
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
    int ran = 0;
    if (nf <= cap && !pb->opt.debug_checks) {
      long long max_rounds = 1 << 16;  // per launch; the host loop continues
      if (tail_interval > 0)
        max_rounds = std::min<long long>(max_rounds, tail_interval - rounds_since_gr);
      if (pb->opt.round_budget > 0)
        max_rounds = std::min<long long>(max_rounds, pb->opt.round_budget - rounds_this_solve);
      max_rounds = std::max<long long>(max_rounds, 1);
      const int stale_left = stale_limit > 0 ? (int)std::max<long long>(1, stale_limit - stale) : 0;
      {
        Launch L(pb, s, KK_ROUND_LOOP);
        k_round_loop<G><<<1, kLoopBlock, 0, s>>>(g, pb->epoch, (int)max_rounds, cap,
                                                  rel_at_gr + budget, stale_left);
      }
      st = sync_ctl(pb, s, "loop");
      if (st) return st;
      ran = pb->ctl_h->loop_rounds;
      in_tail = true;
      pb->st.tail_rounds += ran;
      if (pb->ctl_h->loop_exit == 5) do_gr = true;
    } else {
      // later rounds of the batch may hold larger frontiers than the
      // count known now, so the batch uses the full grid; it runs up to the
      // next interval relabel (at most 16 rounds) between two round trips
      const int grid = kMaxFrontierBlocks;
      int batch = rounds_per_sync;
      if (!pb->opt.debug_checks && gr_interval > 0)
        batch = (int)std::max<long long>(1, std::min<long long>(16, gr_interval - rounds_since_gr));
      if (pb->opt.round_budget > 0)
        batch = (int)std::max<long long>(
            1, std::min<long long>(batch, pb->opt.round_budget - rounds_this_solve));
      for (int i = 0; i < batch; ++i) {
        {
          Launch L(pb, s, KK_PUSH);
          k_push<G><<<grid, kBlock, 0, s>>>(g, pb->epoch + i);
        }
        {
          Launch L(pb, s, KK_APPLY);
          k_apply<<<grid, kBlock, 0, s>>>(g, pb->epoch + i);
        }
      }
      ran = batch;
      if (pb->opt.debug_checks) {
        st = debug_check(pb, s);
        if (st) return st;
      } else {
        st = sync_ctl(pb, s, "rounds");
        if (st) return st;
      }
    }
    pb->epoch += ran;
    pb->st.rounds += ran;
    rounds_this_solve += ran;
    rounds_since_gr += ran;
    // stale-flow bookkeeping (paragraph "Avoid Pushing Flow Back": the flow
    // value unchanged over consecutive rounds that each had few active
    // nodes); the loop kernel keeps its own count of such rounds and
    // reports exit 5.  A batch of device-wide rounds is judged by the
    // frontier it started from; a large one ends the run of small rounds.
    if (pb->ctl_h->flow != last_flow) {
      last_flow = pb->ctl_h->flow;
      stale = 0;
    } else if (nf < kStaleFrontier) {
      stale += ran;
    } else {
      stale = 0;
    }
    if (stale_limit > 0 && stale >= stale_limit) do_gr = true;
    if (pb->ctl_h->relabels - rel_at_gr >= budget) do_gr = true;
    const int interval = in_tail ? tail_interval : gr_interval;
    if (interval > 0 && rounds_since_gr >= interval) do_gr = true;
    if (do_gr) {
      st = global_relabel<G>(pb, s);
      if (st) return st;
      rel_at_gr = pb->ctl_h->relabels;
      rounds_since_gr = 0;
      stale = 0;
      last_flow = pb->ctl_h->flow;
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
  pb->labels_exact = true;  // the loop ends right after a global relabel
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
    k_cut_seed<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, ep, 0);
  }
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, ep, 1, &levels);
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
    vs = reinterpret_cast<uint8_t*>(pb->dev.list[1][kBigList]);  // 4N bytes >= V + E, free after the BFS
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

// ---------------------------------------------------------------------------
// source / sink sides, piercing and the FlowCutter loop (paper, section
// "Flow-Based Refinement", algorithm "FlowCutter Core")
// ---------------------------------------------------------------------------

// Stamp S_r (sources, then the forward residual BFS of the uncapped network
// seeded with the excess nodes); returns the stamp value.
template <int G>
static fp_status source_side_stamps(fp_problem* pb, hipStream_t s, int* ep_out) {
  Dev& g = pb->dev;
  const int ep = pb->epoch++;
  {
    Launch L(pb, s, KK_CUT_SEED);
    k_cut_seed<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, ep, 0);
  }
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, ep, 1, &levels);
  if (st) return st;
  pb->st.bfs_levels += levels;
  k_reset_bfs<<<1, 64, 0, s>>>(g);
  st = sync_ctl(pb, s);
  if (st) return st;
  if (pb->ctl_h->err & ERR_SINK_REACHED) {
    set_error("internal check: a sink is reachable from the source side");
    return FP_ERR_DEVICE;
  }
  *ep_out = ep;
  return FP_OK;
}

// Stamp T_r (sinks, then the reverse residual BFS of the uncapped network).
template <int G>
static fp_status sink_side_stamps(fp_problem* pb, hipStream_t s, int* ep_out) {
  Dev& g = pb->dev;
  const int ep = pb->epoch++;
  k_reset_bfs<<<1, 64, 0, s>>>(g);
  {
    // after a solve the labels give most of T_r at once (phase_sink_seed_labels)
    Launch L(pb, s, KK_CUT_SEED);
    if (pb->labels_exact)
      k_sink_seed_labels<<<sweep_blocks(std::max(g.N, g.P)), kBlock, 0, s>>>(g, ep);
    else k_sink_seed<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, ep);
  }
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, ep, 2, &levels);
  if (st) return st;
  pb->st.bfs_levels += levels;
  k_reset_bfs<<<1, 64, 0, s>>>(g);
  st = sync_ctl(pb, s);
  if (st) return st;
  if (pb->ctl_h->err & ERR_SOURCE_REACHED) {
    set_error("internal check: a source reaches a sink in the residual network");
    return FP_ERR_DEVICE;
  }
  *ep_out = ep;
  return FP_OK;
}

template <int G>
static fp_status sides_impl(fp_problem* pb, hipStream_t s, int want, int* ep_s, int* ep_t) {
  fp_status st = FP_OK;
  if (want & 1) st = source_side_stamps<G>(pb, s, ep_s);
  if (st == FP_OK && (want & 2)) st = sink_side_stamps<G>(pb, s, ep_t);
  return st;
}

// Grow the reachable set stamped ep -- S_r (side 0, forward BFS) or T_r
// (side 1, reverse BFS) -- after vertex p, which already carries ep, was
// pierced into that side without an augmenting path.  The flow is then
// unchanged, and so is the other side's reachable set.  Piercing adds no residual arc: a sink pierce changes
// no arc, so T_r grows by what reaches p; a source pierce removes the arcs
// that carried flow between new sources and their nets and leaves the
// returned flow as excess at the arc heads, so the old S_r stays reachable
// and S_r grows by what the new seeds reach (every seed of the full source
// side that does not carry ep yet: e_in of p's nets, heads that received
// returned flow).
template <int G>
static fp_status grow_side_impl(fp_problem* pb, hipStream_t s, int side, int ep, int p) {
  Dev& g = pb->dev;
  k_reset_bfs<<<1, 64, 0, s>>>(g);
  if (side == 0) k_cut_seed<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, ep, 1);
  else k_seed_vertex<<<1, 64, 0, s>>>(g, p);
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, ep, side == 0 ? 1 : 2, &levels, side == 0 ? -1 : 1);
  if (st) return st;
  pb->st.bfs_levels += levels;
  k_reset_bfs<<<1, 64, 0, s>>>(g);  // the caller's next sync checks the error flags
  return FP_OK;
}

static fp_status grow_side(fp_problem* pb, hipStream_t s, int side, int ep, int p) {
  switch (pb->opt.group_lanes) {
    case 4: return grow_side_impl<4>(pb, s, side, ep, p);
    case 16: return grow_side_impl<16>(pb, s, side, ep, p);
    default: return grow_side_impl<8>(pb, s, side, ep, p);
  }
}

// The same growth without host round trips, for the common case of a small
// one: seeds, then the single-workgroup loop from level 0, nothing read back.
// The caller launches its side-weight and candidate kernels behind it, reads
// everything in one round trip, and calls grow_side_finish when the loop
// stopped at a level too large for it (its count is then nonzero).
template <int G>
static fp_status grow_side_start_impl(fp_problem* pb, hipStream_t s, int side, int ep, int p,
                                      bool seeded) {
  Dev& g = pb->dev;
  if (!seeded) {  // else the source pierce listed level 0 (apply_pierce)
    k_reset_bfs<<<1, 64, 0, s>>>(g);
    if (side == 0) k_cut_seed<<<sweep_blocks(g.N), kBlock, 0, s>>>(g, ep, 1);
    else k_seed_vertex<<<1, 64, 0, s>>>(g, p);
  }
  {
    Launch L(pb, s, KK_BFS_FWD_LOOP);
    k_bfs_loop<G><<<1, kBlock, 0, s>>>(g, 0, pb->opt.tail_threshold, ep, side == 0 ? 1 : 2);
  }
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return hip_fail(he, "growing a reachable set");
  return FP_OK;
}

// Finish a growth that grow_side_start left at `level` (nf nodes) with
// device-wide levels, and clear the BFS counters and FlowCutter outputs.
template <int G>
static fp_status grow_side_finish_impl(fp_problem* pb, hipStream_t s, int side, int ep, int level,
                                       long long nf) {
  int levels = 0;
  fp_status st = run_bfs<G>(pb, s, ep, side == 0 ? 1 : 2, &levels, nf, level);
  if (st) return st;
  pb->st.bfs_levels += levels - level;
  k_reset_bfs<<<1, 64, 0, s>>>(pb->dev);
  return FP_OK;
}

static fp_status grow_side_start(fp_problem* pb, hipStream_t s, int side, int ep, int p,
                                 bool seeded) {
  switch (pb->opt.group_lanes) {
    case 4: return grow_side_start_impl<4>(pb, s, side, ep, p, seeded);
    case 16: return grow_side_start_impl<16>(pb, s, side, ep, p, seeded);
    default: return grow_side_start_impl<8>(pb, s, side, ep, p, seeded);
  }
}

static fp_status grow_side_finish(fp_problem* pb, hipStream_t s, int side, int ep, int level,
                                  long long nf) {
  switch (pb->opt.group_lanes) {
    case 4: return grow_side_finish_impl<4>(pb, s, side, ep, level, nf);
    case 16: return grow_side_finish_impl<16>(pb, s, side, ep, level, nf);
    default: return grow_side_finish_impl<8>(pb, s, side, ep, level, nf);
  }
}

static fp_status sides(fp_problem* pb, hipStream_t s, int want, int* ep_s, int* ep_t) {
  switch (pb->opt.group_lanes) {
    case 4: return sides_impl<4>(pb, s, want, ep_s, ep_t);
    case 16: return sides_impl<16>(pb, s, want, ep_s, ep_t);
    default: return sides_impl<8>(pb, s, want, ep_s, ep_t);
  }
}

fp_status sink_side_problem(fp_problem* pb, hipStream_t s, int32_t mem_kind, uint8_t* vside) {
  if (!pb->solved) {
    set_error("flow_problem_sink_side called before a successful maxflow_solve");
    return FP_ERR_STATE;
  }
  int ep_t = 0;
  fp_status st = sides(pb, s, 2, nullptr, &ep_t);
  if (st) return st;
  uint8_t* vs = mem_kind == 0 ? reinterpret_cast<uint8_t*>(pb->dev.list[1][kBigList]) : vside;
  k_side_out<<<sweep_grid(pb->V), kThreads, 0, s>>>(pb->dev, ep_t, 0, vs);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess && mem_kind == 0)
    he = hipMemcpyAsync(vside, vs, pb->V, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "writing the sink side");
  return FP_OK;
}

// Turn S_r (side 0) or T_r (side 1), stamped ep, plus the stamped piercing
// vertices into terminals.  With seed_growth (a source pierce that avoids
// augmenting paths, whose S_r the next iteration grows) the pierce also lists
// the growth's level 0, after clearing the BFS counters and FlowCutter outputs.
static fp_status apply_pierce(fp_problem* pb, hipStream_t s, int side, int ep,
                              bool seed_growth = false) {
  Dev& g = pb->dev;
  pb->labels_exact = false;  // flows and terminals change
  if (side == 0 && seed_growth) {
    k_reset_bfs<<<1, 64, 0, s>>>(g);
    const long long tiles = ((long long)g.V + kBlock - 1) / kBlock;
    k_pierce_sources_seed<<<(int)std::max<long long>(1, std::min<long long>(tiles, kMaxSweepBlocks)),
                            kBlock, 0, s>>>(g, ep);
  } else if (side == 0) {
    k_pierce_sources<<<sweep_grid(g.V), kThreads, 0, s>>>(g, ep);
  } else {
    k_pierce_sinks<<<sweep_grid(g.V), kThreads, 0, s>>>(g, ep);
  }
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return hip_fail(he, "piercing");
  pb->solved = false;
  return FP_OK;
}

fp_status pierce_problem(fp_problem* pb, int32_t side, const int32_t* vertices, int32_t n,
                         hipStream_t s) {
  if (!pb->solved) {
    set_error("flow_problem_pierce called before a successful maxflow_solve");
    return FP_ERR_STATE;
  }
  for (int32_t i = 0; i < n; ++i)
    if (vertices[i] < 0 || vertices[i] >= pb->V) {
      set_error("piercing vertex %d out of range", vertices[i]);
      return FP_ERR_INVALID;
    }
  int ep_s = 0, ep_t = 0;
  fp_status st = sides(pb, s, side == 0 ? 1 : 2, &ep_s, &ep_t);
  if (st) return st;
  const int ep = side == 0 ? ep_s : ep_t;
  if (n > 0) {
    int32_t* dv = nullptr;
    hipError_t he = hipMallocAsync(reinterpret_cast<void**>(&dv), (size_t)n * sizeof(int32_t), s);
    if (he == hipSuccess)
      he = hipMemcpyAsync(dv, vertices, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) {
      k_mark<<<sweep_grid(n), kThreads, 0, s>>>(pb->dev, dv, n, ep, side == 0 ? 2 : 1);
      he = hipGetLastError();
    }
    if (dv) (void)hipFreeAsync(dv, s);
    if (he != hipSuccess) return hip_fail(he, "marking piercing vertices");
    st = sync_ctl(pb, s);
    if (st) return st;
    if (pb->ctl_h->err & ERR_PIERCE_TERMINAL) {
      // clear the flag; nothing has been pierced
      pb->ctl_h->err &= ~ERR_PIERCE_TERMINAL;
      he = hipMemcpyAsync(&pb->dev.ctl->err, &pb->ctl_h->err, sizeof(int32_t),
                          hipMemcpyHostToDevice, s);
      if (he == hipSuccess) he = hipStreamSynchronize(s);
      if (he != hipSuccess) return hip_fail(he, "clearing the pierce check");
      set_error("a piercing vertex is a terminal of the other side");
      return FP_ERR_INVALID;
    }
  }
  return apply_pierce(pb, s, side, ep);
}

// Pierces of a side made one vertex at a time before bulk piercing measures
// (paragraph "Bulk Piercing": one node for the first few rounds).
constexpr int kBulkWarmup = 3;

// Roles as bytes (0 free, 1 source, 2 sink).
__global__ void __launch_bounds__(kThreads) k_roles_out(Dev g, uint8_t* roles) {
  for (int v = gthread(); v < g.V; v += gthreads()) roles[v] = (uint8_t)g.role[v];
}

fp_status terminals_problem(fp_problem* pb, hipStream_t s, int32_t mem_kind, uint8_t* roles) {
  Dev& g = pb->dev;
  // host outputs are staged in the big-node list of parity 1 (4N bytes >= V)
  uint8_t* out = mem_kind == 0 ? reinterpret_cast<uint8_t*>(g.list[1][kBigList]) : roles;
  k_roles_out<<<sweep_grid(pb->V), kThreads, 0, s>>>(g, out);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess && mem_kind == 0)
    he = hipMemcpyAsync(roles, out, pb->V, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "exporting the terminals");
  return FP_OK;
}

// The weights of S_r and T_r, the smallest vertex outside both and the
// piercing candidates of the lighter side, into the control block (read
// after the next round trip).  Both kernels fold workgroup results into the
// same few counters, and same-address atomics from many workgroups
// serialise, so their grids are kept small.
static void fc_side_stats(fp_problem* pb, hipStream_t s, int ep_s, int ep_t) {
  const int grid = std::min(sweep_grid(pb->V), kFcGrid);
  k_fc_weights<<<grid, kThreads, 0, s>>>(pb->dev, pb->cw, ep_s, ep_t);
  k_fc_pick<<<grid, kThreads, 0, s>>>(pb->dev, ep_s, ep_t);
}

// Up to `slice` more iterations of the FlowCutter run held in pb->fc (see
// flowcutter_problem); trace[0 .. slice) receives this call's iterations.
static fp_status flowcutter_run(fp_problem* pb, int32_t slice, hipStream_t s, int32_t mem_kind,
                                uint8_t* vside, fp_cutter_result* res, fp_cutter_step* trace) {
  Dev& g = pb->dev;
  FcRun& f = pb->fc;
  // labels kept for a solve of this run only: whatever runs next on the
  // handle (a continued run included) starts with a global relabel
  struct WarmReset {
    fp_problem* pb;
    ~WarmReset() { pb->warm_labels = false; }
  } warm_reset{pb};
  f.active = false;  // set again below if the slice ends at its limit
  const long long total = f.total;
  const int64_t max_src = f.max_src, max_snk = f.max_snk;
  const int32_t bulk_percent = f.bulk_percent, most_balanced = f.most_balanced;
  hipError_t he = hipSuccess;
  const int ntiles = (pb->V + kBlock - 1) / kBlock;
  const size_t flag_bytes = ((size_t)pb->V + 3) & ~(size_t)3;
  const size_t count_bytes = 4 * ((size_t)ntiles + 1);
  // [flags: V bytes][tile counts][most balanced side so far: V bytes]
  uint8_t* flags = static_cast<uint8_t*>(pb->fc_mem);
  int32_t* tile_counts = flags ? reinterpret_cast<int32_t*>(flags + flag_bytes) : nullptr;
  uint8_t* best_side = flags ? flags + flag_bytes + count_bytes : nullptr;
  uint8_t* vs = mem_kind == 0 ? reinterpret_cast<uint8_t*>(pb->dev.list[1][kBigList]) : vside;
  fp_cutter_result& r = f.r;
  r.status = 2;  // iteration limit unless a branch below decides
  int32_t done_here = 0;
  bool side_written = false;  // the limit's result side, written before the last pierce
  for (int32_t n = 0; n < slice; ++n) {
    const int32_t it = ++f.it;
    ++done_here;
    int64_t F = 0;
    fp_status st = FP_OK;
    if (f.grow >= 0 && !pb->opt.debug_checks) {
      // the last pierce took a vertex outside S_r and T_r: no residual path
      // joins it to the other side (paragraph "Piercing"), so the preflow
      // stays maximum and the flow value unchanged; no solve is needed
      F = f.last_F;
      pb->solved = true;
    } else {
      const int64_t rounds0 = pb->st.rounds;
      st = solve_problem(pb, s, &F);
      if (st) return st;
      if (f.grow >= 0 && (pb->st.rounds != rounds0 || F != f.last_F)) {
        set_error("internal check: a pierce without augmenting path changed the flow");
        return FP_ERR_DEVICE;
      }
    }
    f.last_F = F;
    int ep_s = 0, ep_t = 0;
    const int grown = f.grow;
    const bool spec = f.grow >= 0 && !pb->opt.debug_checks;  // growth without round trips
    f.seeded = f.seeded && spec;
    if (f.grow >= 0) {
      ep_s = f.prev_ep_s;
      ep_t = f.prev_ep_t;
      const int ep = f.grow == 0 ? ep_s : ep_t;
      st = spec ? grow_side_start(pb, s, f.grow, ep, f.grow_vertex, f.seeded)
                : grow_side(pb, s, f.grow, ep, f.grow_vertex);
    } else {
      st = sides(pb, s, 3, &ep_s, &ep_t);
    }
    if (st) return st;
    f.grow = -1;
    f.prev_ep_s = ep_s;
    f.prev_ep_t = ep_t;
    fc_side_stats(pb, s, ep_s, ep_t);
    st = sync_ctl(pb, s);
    if (st) return st;
    if (spec) {
      const int lv = pb->ctl_h->loop_levels;
      const long long nf = host_count(pb->ctl_h->bcnt[lv % 3]);
      pb->st.bfs_levels += lv;
      if (nf > 0) {  // the growth outgrew the single-workgroup loop
        st = grow_side_finish(pb, s, grown, grown == 0 ? ep_s : ep_t, lv, nf);
        if (st) return st;
        fc_side_stats(pb, s, ep_s, ep_t);
        st = sync_ctl(pb, s);
        if (st) return st;
      }
    }
    if (pb->ctl_h->err & (ERR_SINK_REACHED | ERR_SOURCE_REACHED)) {
      set_error("internal check: a pierce without augmenting path connected a source and a sink");
      return FP_ERR_DEVICE;
    }
    const long long cs = (long long)pb->ctl_h->side_weight[0];
    const long long ct = (long long)pb->ctl_h->side_weight[1];
    if (f.pend_side >= 0) {  // gain of the side pierced last iteration
      const int ps = f.pend_side;
      const long long gain = std::max(0ll, (ps == 0 ? cs : ct) - f.pend_before);
      f.gained[ps] += gain;
      f.pierced[ps] += f.pend_count;
      if (f.pend_goal >= 0) f.missed[ps] = std::max(0ll, f.pend_goal - gain);
      f.pend_side = -1;
    }
    r.iterations = it;
    r.flow = F;
    f.out_ep = ep_s;  // the iteration limit reports this iteration's S_r
    f.last_cs = cs;
    fp_cutter_step step{};
    step.flow = F;
    step.source_weight = cs;
    step.sink_weight = ct;
    step.side = -1;
    step.node = -1;
    step.count = 0;
    bool done = false;
    const bool bal0 = cs <= max_src && total - cs <= max_snk;  // (S_r, V \ S_r)
    const bool bal1 = total - ct <= max_src && ct <= max_snk;  // (V \ T_r, T_r)
    if (!most_balanced && bal0) {
      r.status = 0;
      r.side = 0;
      r.source_weight = cs;
      r.sink_weight = total - cs;
      f.out_ep = ep_s;
      f.out_invert = 0;
      f.first_balanced = it;
      done = true;
    } else if (!most_balanced && bal1) {
      r.status = 0;
      r.side = 1;
      r.source_weight = total - ct;
      r.sink_weight = ct;
      f.out_ep = ep_t;
      f.out_invert = 1;
      f.first_balanced = it;
      done = true;
    } else if (most_balanced && (bal0 || bal1 || f.best_heavier >= 0)) {
      // most balanced cut: keep the best balanced cut offered so far (its
      // side is copied now: later pierces grow the stamped sets) and pierce
      // on while a vertex outside S_r and T_r is left
      if (f.first_balanced == 0) f.first_balanced = it;
      for (int kind = 0; kind < 2; ++kind) {
        if (!(kind == 0 ? bal0 : bal1)) continue;
        const long long src = kind == 0 ? cs : total - ct;
        const long long heavier = std::max(src, total - src);
        if (f.best_heavier >= 0 && heavier >= f.best_heavier) continue;
        f.best_heavier = heavier;
        f.best_kind = kind;
        f.best_src = src;
        f.best_snk = total - src;
        f.best_F = F;
        k_side_out<<<sweep_grid(pb->V), kThreads, 0, s>>>(g, kind == 0 ? ep_s : ep_t, kind,
                                                          best_side);
        he = hipGetLastError();
        if (he != hipSuccess) return hip_fail(he, "keeping the most balanced cut");
      }
      const int side = cs <= ct ? 0 : 1;
      int p = pb->ctl_h->pierce[3 * side];  // a free boundary pin, else any free vertex
      if (p == kInf) p = pb->ctl_h->pierce[2];
      if (p == kInf) {
        r.status = 0;  // finished: the best cut kept is the result, nothing to resume
        done = true;
      } else {
        step.side = side;
        step.node = p;
        step.count = 1;
        f.grow = side;
        f.grow_vertex = p;
        k_stamp_vertex<<<1, 64, 0, s>>>(g, p, side == 0 ? ep_s : ep_t);
        he = hipGetLastError();
        if (he != hipSuccess) return hip_fail(he, "marking the piercing vertex");
        f.seeded = side == 0 && !pb->opt.debug_checks;
        st = apply_pierce(pb, s, side, side == 0 ? ep_s : ep_t, f.seeded);
        if (st) return st;
      }
    } else {
      const int side = cs <= ct ? 0 : 1;
      // a free boundary pin, else any free vertex, else an augmenting pin
      int p = pb->ctl_h->pierce[3 * side];
      bool aug = false;
      if (p == kInf) p = pb->ctl_h->pierce[2];
      if (p == kInf) {
        p = pb->ctl_h->pierce[3 * side + 1];
        aug = true;
      }
      step.side = side;
      step.node = p == kInf ? -1 : p;
      if (p == kInf) {
        r.status = 1;
        r.side = side;
        if (side == 0) {
          r.source_weight = cs;
          r.sink_weight = total - cs;
          f.out_ep = ep_s;
          f.out_invert = 0;
        } else {
          r.source_weight = total - ct;
          r.sink_weight = ct;
          f.out_ep = ep_t;
          f.out_invert = 1;
        }
        done = true;
      } else {
        if (n + 1 == slice) {
          // the call stops at its limit after this iteration and returns
          // this iteration's S_r: written now, before the pierce stamps the
          // new sources with S_r's stamp
          k_side_out<<<sweep_grid(pb->V), kThreads, 0, s>>>(g, ep_s, 0, vs);
          he = hipGetLastError();
          if (he == hipSuccess && mem_kind == 0)
            he = hipMemcpyAsync(vside, vs, pb->V, hipMemcpyDeviceToHost, s);
          if (he != hipSuccess) return hip_fail(he, "writing the FlowCutter side");
          side_written = true;
        }
        if (aug) r.augmenting++;
        else {
          f.grow = side;
          f.grow_vertex = p;
        }
        const int ep = side == 0 ? ep_s : ep_t;
        const long long weight = side == 0 ? cs : ct;
        long long k = 1, goal = -1;
        if (aug && bulk_percent > 0 && f.pierces[side] >= kBulkWarmup && f.gained[side] > 0) {
          if (f.term[side] < 0) f.term[side] = std::max(0ll, total / 2 - weight);
          f.term[side] = f.term[side] * bulk_percent / 100;
          goal = f.term[side] + f.missed[side];
          k = std::max(1ll, goal * f.pierced[side] / f.gained[side]);
        }
        long long count = 1;
        if (k > 1) {
          // the k smallest-id augmenting candidates of this side
          he = hipMemsetAsync(flags, 0, flag_bytes, s);
          if (he != hipSuccess) return hip_fail(he, "clearing the candidate flags");
          k_fc_mark_augmenting<<<sweep_grid(pb->E), kThreads, 0, s>>>(g, side, ep_s, ep_t, flags);
          k_count_flags<<<ntiles, kBlock, 0, s>>>(flags, pb->V, tile_counts);
          k_scan_counts<<<1, kBlock, 0, s>>>(tile_counts, ntiles);
          const int kk = (int)std::min<long long>(k, pb->V);
          k_select_flags<<<ntiles, kBlock, 0, s>>>(g, flags, pb->V, tile_counts, kk, ep);
          int32_t found = 0;
          he = hipGetLastError();
          if (he == hipSuccess)
            he = hipMemcpyAsync(&found, tile_counts + ntiles, 4, hipMemcpyDeviceToHost, s);
          if (he == hipSuccess) he = hipStreamSynchronize(s);
          if (he != hipSuccess) return hip_fail(he, "selecting the piercing vertices");
          count = std::min<long long>(k, found);
        } else {
          k_stamp_vertex<<<1, 64, 0, s>>>(g, p, ep);
          he = hipGetLastError();
          if (he != hipSuccess) return hip_fail(he, "marking the piercing vertex");
        }
        step.count = (int32_t)count;
        f.pierces[side] += 1;
        f.pend_side = side;
        f.pend_before = weight;
        f.pend_count = count;
        f.pend_goal = goal;
        f.seeded = !aug && side == 0 && !pb->opt.debug_checks;
        st = apply_pierce(pb, s, side, ep, f.seeded);
        if (st) return st;
        // an augmenting source pierce is followed by a solve that keeps the labels
        pb->warm_labels = aug && side == 0;
      }
    }
    if (trace) trace[n] = step;
    if (done) break;
  }
  if (f.grow >= 0) {
    // the call ends with a growth pending for the next iteration: the seeds
    // a source pierce listed for it would otherwise stay in the BFS
    // counters for whatever runs next on the handle, so they are dropped
    // and a continued run re-derives its sides (a warm solve, same result)
    k_reset_bfs<<<1, 64, 0, s>>>(g);
    f.grow = -1;
    f.seeded = false;
  }
  fp_cutter_result out = r;
  out.first_balanced = f.first_balanced;
  out.slice_iterations = done_here;
  out.resumable = r.status == 2 ? 1 : 0;
  if (f.best_heavier >= 0) {  // most balanced cut (also when the limit ended the call)
    out.status = 0;
    out.side = f.best_kind;
    out.flow = f.best_F;
    out.source_weight = f.best_src;
    out.sink_weight = f.best_snk;
    he = hipMemcpyAsync(vside, best_side, pb->V,
                        mem_kind == 0 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s);
  } else {
    int invert = f.out_invert;
    if (r.status == 2) {  // iteration limit: the last iteration's S_r
      out.side = 0;
      out.source_weight = f.last_cs;
      out.sink_weight = total - f.last_cs;
      invert = 0;
    }
    if (!side_written) {
      k_side_out<<<sweep_grid(pb->V), kThreads, 0, s>>>(g, f.out_ep, invert, vs);
      he = hipGetLastError();
      if (he == hipSuccess && mem_kind == 0)
        he = hipMemcpyAsync(vside, vs, pb->V, hipMemcpyDeviceToHost, s);
    }
  }
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "writing the FlowCutter side");
  f.active = r.status == 2;
  *res = out;
  return FP_OK;
}

fp_status flowcutter_problem(fp_problem* pb, const int32_t* vw, int64_t max_src, int64_t max_snk,
                             int32_t max_iters, int32_t bulk_percent, int32_t most_balanced,
                             hipStream_t s, int32_t mem_kind, uint8_t* vside,
                             fp_cutter_result* res, fp_cutter_step* trace) {
  long long total = 0;
  for (int32_t v = 0; v < pb->V; ++v) {
    if (vw[v] < 0) {
      set_error("vertex weight of %d is negative", v);
      return FP_ERR_INVALID;
    }
    total += vw[v];
  }
  if (max_iters < 1) {
    set_error("max_iterations must be at least 1");
    return FP_ERR_INVALID;
  }
  // The warm solves of a run move little flow each: relabel every 8 rounds
  // (16 in the single-workgroup loop) and claim every BFS level, unless the
  // caller chose these options (on the 200k-vertex region: 575 -> 756
  // iterations/s with one vertex per pierce, bulk piercing unchanged)
  if (pb->opt_user.gr_interval == 0) pb->opt.gr_interval = 8;
  if (pb->opt_user.tail_gr_interval == 0) pb->opt.tail_gr_interval = 16;
  if (pb->opt_user.bottom_up_min == 0) pb->opt.bottom_up_min = 0;
  hipError_t he = hipSuccess;
  if (!pb->cw) {
    he = hipMalloc(reinterpret_cast<void**>(&pb->cw), (size_t)pb->V * sizeof(int32_t));
    if (he != hipSuccess) {
      pb->cw = nullptr;
      return hip_fail(he, "allocating vertex weights");
    }
  }
  he = hipMemcpyAsync(pb->cw, vw, (size_t)pb->V * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (he != hipSuccess) return hip_fail(he, "copying vertex weights");
  if ((bulk_percent > 0 || most_balanced) && !pb->fc_mem) {
    const int ntiles = (pb->V + kBlock - 1) / kBlock;
    const size_t flag_bytes = ((size_t)pb->V + 3) & ~(size_t)3;
    const size_t count_bytes = 4 * ((size_t)ntiles + 1);
    he = hipMalloc(&pb->fc_mem, 2 * flag_bytes + count_bytes);
    if (he != hipSuccess) {
      pb->fc_mem = nullptr;
      return hip_fail(he, "allocating the FlowCutter scratch");
    }
  }
  pb->fc = FcRun{};
  FcRun& f = pb->fc;
  f.max_src = max_src;
  f.max_snk = max_snk;
  f.bulk_percent = bulk_percent;
  f.most_balanced = most_balanced;
  f.total = total;
  return flowcutter_run(pb, max_iters, s, mem_kind, vside, res, trace);
}

fp_status flowcutter_continue(fp_problem* pb, int32_t max_iters, hipStream_t s, int32_t mem_kind,
                              uint8_t* vside, fp_cutter_result* res, fp_cutter_step* trace) {
  if (!pb->fc.active) {
    set_error("no FlowCutter run to continue (none started, or the last one finished)");
    return FP_ERR_STATE;
  }
  if (max_iters < 1) {
    set_error("max_iterations must be at least 1");
    return FP_ERR_INVALID;
  }
  // the sides of the next iteration are derived afresh (the previous call
  // dropped any growth it left pending)
  return flowcutter_run(pb, max_iters, s, mem_kind, vside, res, trace);
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------

const char* kernel_kind_name(int k) {
  static const char* names[KK_COUNT] = {
      "init",      "gr_reset", "bfs_rev",       "bfs_rev_loop", "gather",
      "push",      "apply",    "round_loop",    "cut_seed",     "bfs_fwd",
      "bfs_fwd_loop", "cut_out", "check",       "batch",        "bfs_collect"};
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

// Timing events are kept per device for the whole process and shared by
// every handle: a handle's run records a few hundred of them, and creating
// and destroying that many per handle costs more than the kernels they time.
static std::mutex g_event_mu;
static std::map<int, std::vector<hipEvent_t>> g_events;

void event_pool_put(int device, hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lock(g_event_mu);
  g_events[device].push_back(e);
}

static hipEvent_t get_event(fp_problem* pb) {
  {
    std::lock_guard<std::mutex> lock(g_event_mu);
    std::vector<hipEvent_t>& pool = g_events[pb->device];
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
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
    event_pool_put(pb->device, t.a);
    event_pool_put(pb->device, t.b);
  }
  pb->pending.clear();
}

}  // namespace hf
