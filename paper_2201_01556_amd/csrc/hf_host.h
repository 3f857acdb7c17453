// Host-side state of a flow problem handle and internal entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hf_device.h"
#include "hyperflow.h"

namespace hf {

// kernel kinds for per-launch timing
enum KernelKind : int {
  KK_INIT = 0,
  KK_GR_RESET,
  KK_BFS_REV,
  KK_BFS_REV_LOOP,
  KK_GATHER,
  KK_PUSH,
  KK_APPLY,
  KK_ROUND_LOOP,
  KK_CUT_SEED,
  KK_BFS_FWD,
  KK_BFS_FWD_LOOP,
  KK_CUT_OUT,
  KK_CHECK,
  KK_BATCH,
  KK_BFS_COLLECT,
  KK_COUNT
};

const char* kernel_kind_name(int k);
// device byte-counter class of a kernel kind (-1: none)
int kernel_kind_class(int k);

struct Timer {
  int kind;
  hipEvent_t a, b;
};

// State of a FlowCutter run between calls: flow_problem_flowcutter starts a
// run, flow_problem_flowcutter_continue resumes one that stopped at its
// iteration limit (the loop variables below are exactly those of one
// uninterrupted run).
struct FcRun {
  bool active = false;  // stopped at the iteration limit; may be continued
  int64_t max_src = 0, max_snk = 0;
  int32_t bulk_percent = 0, most_balanced = 0;
  long long total = 0;  // c(V)
  int32_t it = 0;       // iterations done
  fp_cutter_result r{};
  // most balanced cut so far
  long long best_heavier = -1, best_src = 0, best_snk = 0;
  int best_kind = 0;
  int64_t best_F = 0;
  int32_t first_balanced = 0;
  // bulk piercing bookkeeping per side
  long long pierces[2] = {0, 0}, gained[2] = {0, 0}, pierced[2] = {0, 0};
  long long term[2] = {-1, -1}, missed[2] = {0, 0};
  int pend_side = -1;
  long long pend_before = 0, pend_count = 0, pend_goal = -1;
  // reachable sets kept across a pierce without augmenting path
  int prev_ep_s = -1, prev_ep_t = -1, grow = -1, grow_vertex = -1;
  bool seeded = false;
  int64_t last_F = 0;
  long long last_cs = 0;
  int out_ep = -1, out_invert = 0;
};

}  // namespace hf

struct fp_problem {
  int device = 0;
  int32_t V = 0, E = 0, P = 0, NB = 0, N = 0;
  int32_t nS = 0, nT = 0;
  int64_t wsum = 0;          // sum of the net weights (at most INT32_MAX)
  fp_options opt{};
  fp_options opt_user{};     // the options as the caller gave them (zeros = defaults)
  hf::Dev dev{};
  void* pool = nullptr;
  size_t pool_bytes = 0;     // capacity of the pool (a reused block may be larger)
  hf::Ctl* ctl_h = nullptr;  // pinned host mirror of the control block
  int32_t epoch = 1;         // stamp value of the next round / BFS
  int32_t gr_batch = 8;      // device-wide levels launched first by a global relabel
  int32_t gr_hist[hf::kLvlHist] = {};  // level sizes of the previous global relabel's BFS
  int32_t gr_hist_levels = 0;
  bool inited = false;
  bool solved = false;
  bool warm_labels = false;  // the labels are valid for the next solve (after a source pierce)
  bool labels_exact = false;  // the labels are exact distances of the current flow (a solve ended)
  int32_t* cw = nullptr;     // vertex weights of the last FlowCutter run (device)
  void* fc_mem = nullptr;    // FlowCutter scratch: candidate flags, tile counts, best side
  hf::FcRun fc;
  fp_stats st{};
  // profiling
  std::vector<hf::Timer> pending;
  int64_t k_launches[hf::KK_COUNT] = {};
  double k_ms[hf::KK_COUNT] = {};
  unsigned long long bytes_at_sync[hf::KC_N] = {};
  double k_bytes[hf::KK_COUNT] = {};
};

// Flow problems of block pairs built on the device (hf_regions.hip).
struct fp_regions {
  int device = 0;
  int32_t npairs = 0, k = 0, V = 0;
  void* mem = nullptr;                   // device outputs (one allocation)
  int32_t* off = nullptr;                // per pair ne+1 relative offsets
  int32_t* pins = nullptr;               // local ids
  int32_t* w = nullptr;                  // net weights
  int32_t* ngid = nullptr;               // global net id (smallest of a group)
  int32_t* vw = nullptr;                 // per pair n+2 vertex weights
  int32_t* vgid = nullptr;               // per pair n global vertex ids
  int8_t* vside = nullptr;               // per pair n: 0 = region of block i, 1 = of block j
  int32_t* terms = nullptr;              // per pair {n, n+1}
  std::vector<int32_t> pairs;            // 2 per pair
  std::vector<int64_t> info;             // npairs * 16
  std::vector<long long> net_base, pin_base, vtx_base, nloc;  // where pair q starts; n
  std::vector<long long> wsum;           // net weight sum per pair (filled by the first solve)
  uint8_t* sides = nullptr;              // per pair n+2 bytes: minimal source side of the last solve
  bool solved = false;
};

namespace hf {

void set_error(const char* fmt, ...);
fp_status hip_fail(hipError_t e, const char* what);

// defaults filled in
fp_options resolve_options(const fp_options* o);

// Validate the inputs and build the device layout.  With `ext` the layout
// (and the temporary memory of the build) is carved from the caller's
// ext_bytes of device memory and pb->ctl_h must point to the caller's host
// mirror of the control block; otherwise the handle's pool and control
// block are allocated (or taken from the cache).
fp_status build_problem(fp_problem* pb, const int32_t* net_offsets, const int32_t* pins,
                        const int32_t* net_weights, const int32_t* sources, int32_t nS,
                        const int32_t* sinks, int32_t nT, int32_t mem_kind,
                        hipStream_t s, void* ext = nullptr, size_t ext_bytes = 0);
fp_status solve_problem(fp_problem* pb, hipStream_t s, int64_t* flow);
fp_status cut_problem(fp_problem* pb, hipStream_t s, int32_t mem_kind, uint8_t* vside,
                      uint8_t* nside);
fp_status batch_solve(fp_problem* const* pbs, int32_t count, const uint8_t* skip,
                      hipStream_t s, int64_t* flows);
// a configuration (zero fields = defaults) that create_batch accepts
bool batch_config_ok(const fp_batch_config* c);
fp_status create_batch(fp_problem* const* pbs, int32_t count, uint8_t* const* vsides,
                       uint8_t* const* nsides, const fp_batch_config* config, hipStream_t s,
                       fp_batch** out);
fp_status run_batch(fp_batch* b, const uint8_t* skip, int32_t with_cut, hipStream_t s,
                    int64_t* flows);
fp_status tune_batch(fp_batch* b, hipStream_t s, const char* cache_path, fp_batch_config* chosen);
fp_status batch_config(const fp_batch* b, fp_batch_config* out);
void release_batch(fp_batch* b);
fp_status scorer_create_impl(const float* init, hipStream_t s, fp_scorer** out);
void scorer_destroy_impl(fp_scorer* sc);
fp_status scorer_fit_impl(fp_scorer* sc, const int64_t* f, int n, int mem_kind, hipStream_t s);
fp_status scorer_gradient_impl(fp_scorer* sc, const int64_t* f, const float* y, int n,
                               int mem_kind, hipStream_t s, float* grad, float* loss);
fp_status scorer_train_impl(fp_scorer* sc, const int64_t* f, const float* y, int n, int mem_kind,
                            int steps, float lr, hipStream_t s, float* losses);
fp_status scorer_predict_impl(fp_scorer* sc, const int64_t* f, int n, int mem_kind,
                              hipStream_t s, float* prob);
fp_status scorer_get_impl(const fp_scorer* sc, float* params, double* mean_std);
fp_status scorer_set_impl(fp_scorer* sc, const float* params, const double* mean_std);
fp_status pierce_problem(fp_problem* pb, int32_t side, const int32_t* vertices, int32_t n,
                         hipStream_t s);
fp_status sink_side_problem(fp_problem* pb, hipStream_t s, int32_t mem_kind, uint8_t* vside);
fp_status flowcutter_problem(fp_problem* pb, const int32_t* vw, int64_t max_src, int64_t max_snk,
                             int32_t max_iters, int32_t bulk_percent, int32_t most_balanced,
                             hipStream_t s, int32_t mem_kind, uint8_t* vside,
                             fp_cutter_result* res, fp_cutter_step* trace);
fp_status flowcutter_continue(fp_problem* pb, int32_t max_iters, hipStream_t s, int32_t mem_kind,
                              uint8_t* vside, fp_cutter_result* res, fp_cutter_step* trace);
fp_status terminals_problem(fp_problem* pb, hipStream_t s, int32_t mem_kind, uint8_t* roles);
fp_status export_state(fp_problem* pb, hipStream_t s, int32_t* f_in, int32_t* f_out,
                       int32_t* f_b, int32_t* labels, int32_t* excess);
void release_problem(fp_problem* pb);
// free the device pools and pinned control blocks kept for reuse
void release_cached_memory();

// profiling helpers
void prof_begin(fp_problem* pb, int kind, hipStream_t s, Timer* t);
void prof_end(fp_problem* pb, Timer* t, hipStream_t s);
void prof_collect(fp_problem* pb);
// timing events go back to the process-wide pool of their device
void event_pool_put(int device, hipEvent_t e);

}  // namespace hf
