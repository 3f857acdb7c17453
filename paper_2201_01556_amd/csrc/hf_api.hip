// C ABI entry points (include/hyperflow.h): argument checks, error strings
// and handle lifetime; the work is done in hf_build.hip / hf_solve.hip.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "hf_host.h"

namespace hf {

// Message of the last failed call on this thread: a fixed buffer, so that
// reporting an error allocates nothing.
struct LastError {
  char buf[512];
  void clear() { buf[0] = 0; }
  const char* c_str() const { return buf; }
};
static thread_local LastError g_last_error;

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error.buf, sizeof(g_last_error.buf), fmt, ap);
  va_end(ap);
}

fp_status hip_fail(hipError_t e, const char* what) {
  set_error("%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FP_ERR_OOM : FP_ERR_DEVICE;
}

}  // namespace hf

using namespace hf;

#pragma GCC visibility push(default)
extern "C" {

const char* fp_last_error(void) { return g_last_error.c_str(); }

fp_status flow_problem_create(int32_t num_vertices, int32_t num_nets, const int32_t* net_offsets,
                              const int32_t* pins, const int32_t* net_weights,
                              const int32_t* sources, int32_t num_sources, const int32_t* sinks,
                              int32_t num_sinks, int32_t mem_kind, const fp_options* opts,
                              void* hip_stream, fp_problem** out) {
  g_last_error.clear();
  if (!out) {
    set_error("out is NULL");
    return FP_ERR_INVALID;
  }
  *out = nullptr;
  if (num_vertices < 1 || num_nets < 0) {
    set_error("need num_vertices >= 1 and num_nets >= 0 (got %d, %d)", num_vertices, num_nets);
    return FP_ERR_INVALID;
  }
  if (num_sources < 1 || num_sinks < 1) {
    set_error("source and sink sets must be nonempty (got %d, %d)", num_sources, num_sinks);
    return FP_ERR_INVALID;
  }
  if (!net_offsets || !sources || !sinks || (num_nets > 0 && !net_weights)) {
    set_error("NULL input pointer");
    return FP_ERR_INVALID;
  }
  if (mem_kind != 0 && mem_kind != 1) {
    set_error("mem_kind must be 0 (host) or 1 (device), got %d", mem_kind);
    return FP_ERR_INVALID;
  }
  if ((long long)num_sources + num_sinks >= (1ll << 31)) {
    set_error("too many terminals");
    return FP_ERR_OVERFLOW;
  }
  fp_problem* pb = new (std::nothrow) fp_problem();
  if (!pb) {
    set_error("host allocation failed");
    return FP_ERR_OOM;
  }
  hipGetDevice(&pb->device);
  pb->V = num_vertices;
  pb->E = num_nets;
  pb->opt = resolve_options(opts);
  if (opts) pb->opt_user = *opts;
  fp_status st = build_problem(pb, net_offsets, pins, net_weights, sources, num_sources, sinks,
                               num_sinks, mem_kind, static_cast<hipStream_t>(hip_stream));
  if (st != FP_OK) {
    hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
    release_problem(pb);
    delete pb;
    return st;
  }
  *out = pb;
  return FP_OK;
}

fp_status maxflow_solve(fp_problem* problem, void* hip_stream, int64_t* flow_value) {
  g_last_error.clear();
  if (!problem || !flow_value) {
    set_error("NULL argument");
    return problem ? FP_ERR_INVALID : FP_ERR_STATE;
  }
  int64_t f = 0;
  fp_status st = solve_problem(problem, static_cast<hipStream_t>(hip_stream), &f);
  if (st == FP_OK) *flow_value = f;
  return st;
}

fp_status mincut_source_side(fp_problem* problem, void* hip_stream, int32_t mem_kind,
                             uint8_t* vertex_side, uint8_t* net_side) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  if (!vertex_side || (mem_kind != 0 && mem_kind != 1)) {
    set_error("vertex_side must be non-NULL and mem_kind 0 or 1");
    return FP_ERR_INVALID;
  }
  return cut_problem(problem, static_cast<hipStream_t>(hip_stream), mem_kind, vertex_side,
                     net_side);
}

// distinct, non-NULL handles on the current device
static fp_status check_batch_problems(fp_problem* const* problems, int32_t count) {
  if (count < 0 || (count > 0 && !problems)) {
    set_error("invalid batch arguments");
    return FP_ERR_INVALID;
  }
  int dev = 0;
  hipGetDevice(&dev);
  std::vector<fp_problem*> seen(problems, problems + count);
  std::sort(seen.begin(), seen.end());
  for (int32_t i = 0; i < count; ++i) {
    if (!problems[i]) {
      set_error("problem %d is NULL", i);
      return FP_ERR_INVALID;
    }
    if (problems[i]->device != dev) {
      set_error("problem %d lives on device %d, the current device is %d", i,
                problems[i]->device, dev);
      return FP_ERR_INVALID;
    }
    if (i > 0 && seen[i] == seen[i - 1]) {
      set_error("a problem appears twice in the batch");
      return FP_ERR_INVALID;
    }
  }
  return FP_OK;
}

fp_status flow_batch_solve(fp_problem* const* problems, int32_t count, const uint8_t* skip,
                           void* hip_stream, int64_t* flow_values) {
  g_last_error.clear();
  fp_status st = check_batch_problems(problems, count);
  if (st) return st;
  if (count > 0 && !flow_values) {
    set_error("flow_values is NULL");
    return FP_ERR_INVALID;
  }
  return batch_solve(problems, count, skip, static_cast<hipStream_t>(hip_stream), flow_values);
}

fp_status flow_batch_create(fp_problem* const* problems, int32_t count,
                            uint8_t* const* vertex_sides, uint8_t* const* net_sides,
                            const fp_batch_config* config, void* hip_stream, fp_batch** out) {
  g_last_error.clear();
  if (!out) {
    set_error("out is NULL");
    return FP_ERR_INVALID;
  }
  *out = nullptr;
  fp_status st = check_batch_problems(problems, count);
  if (st) return st;
  if (net_sides && !vertex_sides) {
    set_error("net_sides given without vertex_sides");
    return FP_ERR_INVALID;
  }
  if (vertex_sides)
    for (int32_t i = 0; i < count; ++i)
      if (!vertex_sides[i]) {
        set_error("vertex_sides[%d] is NULL", i);
        return FP_ERR_INVALID;
      }
  if (config && !batch_config_ok(config)) {
    set_error("invalid batch configuration");
    return FP_ERR_INVALID;
  }
  return create_batch(problems, count, vertex_sides, net_sides, config,
                      static_cast<hipStream_t>(hip_stream), out);
}

fp_status flow_batch_run(fp_batch* batch, const uint8_t* skip, int32_t with_cut, void* hip_stream,
                         int64_t* flow_values) {
  g_last_error.clear();
  if (!batch) {
    set_error("NULL batch");
    return FP_ERR_STATE;
  }
  if (with_cut != 0 && with_cut != 1) {
    set_error("with_cut must be 0 or 1");
    return FP_ERR_INVALID;
  }
  return run_batch(batch, skip, with_cut, static_cast<hipStream_t>(hip_stream), flow_values);
}

fp_status flow_batch_tune(fp_batch* batch, void* hip_stream, const char* cache_path,
                          fp_batch_config* chosen) {
  g_last_error.clear();
  if (!batch) {
    set_error("NULL batch");
    return FP_ERR_STATE;
  }
  return tune_batch(batch, static_cast<hipStream_t>(hip_stream), cache_path, chosen);
}

fp_status flow_batch_get_config(const fp_batch* batch, fp_batch_config* out) {
  if (!batch || !out) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  return batch_config(batch, out);
}

void flow_batch_destroy(fp_batch* batch) {
  if (!batch) return;
  release_batch(batch);
  delete batch;
}

fp_status flow_problem_reset(fp_problem* problem) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  problem->inited = false;
  problem->solved = false;
  problem->labels_exact = false;
  return FP_OK;
}

fp_status flow_problem_pierce(fp_problem* problem, int32_t side, const int32_t* vertices,
                              int32_t n, void* hip_stream) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  if ((side != 0 && side != 1) || n < 0 || (n > 0 && !vertices)) {
    set_error("invalid pierce arguments");
    return FP_ERR_INVALID;
  }
  return pierce_problem(problem, side, vertices, n, static_cast<hipStream_t>(hip_stream));
}

fp_status flow_problem_sink_side(fp_problem* problem, void* hip_stream, int32_t mem_kind,
                                 uint8_t* vertex_side) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  if (!vertex_side || (mem_kind != 0 && mem_kind != 1)) {
    set_error("vertex_side must be non-NULL and mem_kind 0 or 1");
    return FP_ERR_INVALID;
  }
  return sink_side_problem(problem, static_cast<hipStream_t>(hip_stream), mem_kind, vertex_side);
}

fp_status flow_problem_flowcutter(fp_problem* problem, const int32_t* vertex_weights,
                                  int64_t max_source_weight, int64_t max_sink_weight,
                                  int32_t max_iterations, int32_t bulk_percent,
                                  int32_t most_balanced, void* hip_stream, int32_t mem_kind,
                                  uint8_t* vertex_side, fp_cutter_result* result,
                                  fp_cutter_step* trace) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  if (!vertex_weights || !vertex_side || !result || max_iterations < 1 ||
      (mem_kind != 0 && mem_kind != 1) || bulk_percent < 0 || bulk_percent > 99 ||
      (most_balanced != 0 && most_balanced != 1)) {
    set_error("invalid FlowCutter arguments");
    return FP_ERR_INVALID;
  }
  return flowcutter_problem(problem, vertex_weights, max_source_weight, max_sink_weight,
                            max_iterations, bulk_percent, most_balanced,
                            static_cast<hipStream_t>(hip_stream), mem_kind, vertex_side, result,
                            trace);
}

fp_status flow_problem_flowcutter_continue(fp_problem* problem, int32_t max_iterations,
                                           void* hip_stream, int32_t mem_kind,
                                           uint8_t* vertex_side, fp_cutter_result* result,
                                           fp_cutter_step* trace) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  if (!vertex_side || !result || max_iterations < 1 || (mem_kind != 0 && mem_kind != 1)) {
    set_error("invalid FlowCutter arguments");
    return FP_ERR_INVALID;
  }
  return flowcutter_continue(problem, max_iterations, static_cast<hipStream_t>(hip_stream),
                             mem_kind, vertex_side, result, trace);
}

fp_status flow_problem_terminals(fp_problem* problem, void* hip_stream, int32_t mem_kind,
                                 uint8_t* roles) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  if (!roles || (mem_kind != 0 && mem_kind != 1)) {
    set_error("roles must be non-NULL and mem_kind 0 or 1");
    return FP_ERR_INVALID;
  }
  return terminals_problem(problem, static_cast<hipStream_t>(hip_stream), mem_kind, roles);
}

static fp_status check_samples(const void* f, int32_t n, int32_t mem_kind) {
  if (!f || n < 1 || (mem_kind != 0 && mem_kind != 1)) {
    set_error("need features, n >= 1 and mem_kind 0 or 1");
    return FP_ERR_INVALID;
  }
  return FP_OK;
}

fp_status scorer_create(const float* init_params, void* hip_stream, fp_scorer** out) {
  g_last_error.clear();
  if (!out || !init_params) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  *out = nullptr;
  return scorer_create_impl(init_params, static_cast<hipStream_t>(hip_stream), out);
}

fp_status scorer_fit_normalization(fp_scorer* scorer, const int64_t* features, int32_t n,
                                   int32_t mem_kind, void* hip_stream) {
  g_last_error.clear();
  if (!scorer) {
    set_error("NULL scorer");
    return FP_ERR_STATE;
  }
  fp_status st = check_samples(features, n, mem_kind);
  if (st) return st;
  return scorer_fit_impl(scorer, features, n, mem_kind, static_cast<hipStream_t>(hip_stream));
}

fp_status scorer_gradient(fp_scorer* scorer, const int64_t* features, const float* labels,
                          int32_t n, int32_t mem_kind, void* hip_stream, float* gradient,
                          float* loss) {
  g_last_error.clear();
  if (!scorer) {
    set_error("NULL scorer");
    return FP_ERR_STATE;
  }
  fp_status st = check_samples(features, n, mem_kind);
  if (st) return st;
  if (!labels || !gradient || !loss) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  return scorer_gradient_impl(scorer, features, labels, n, mem_kind,
                              static_cast<hipStream_t>(hip_stream), gradient, loss);
}

fp_status scorer_train(fp_scorer* scorer, const int64_t* features, const float* labels,
                       int32_t n, int32_t mem_kind, int32_t steps, float lr, void* hip_stream,
                       float* losses) {
  g_last_error.clear();
  if (!scorer) {
    set_error("NULL scorer");
    return FP_ERR_STATE;
  }
  fp_status st = check_samples(features, n, mem_kind);
  if (st) return st;
  if (!labels || steps < 0 || !(lr > 0.f)) {
    set_error("need labels, steps >= 0 and lr > 0");
    return FP_ERR_INVALID;
  }
  return scorer_train_impl(scorer, features, labels, n, mem_kind, steps, lr,
                           static_cast<hipStream_t>(hip_stream), losses);
}

fp_status scorer_predict(fp_scorer* scorer, const int64_t* features, int32_t n, int32_t mem_kind,
                         void* hip_stream, float* probabilities) {
  g_last_error.clear();
  if (!scorer) {
    set_error("NULL scorer");
    return FP_ERR_STATE;
  }
  fp_status st = check_samples(features, n, mem_kind);
  if (st) return st;
  if (!probabilities) {
    set_error("NULL probabilities");
    return FP_ERR_INVALID;
  }
  return scorer_predict_impl(scorer, features, n, mem_kind, static_cast<hipStream_t>(hip_stream),
                             probabilities);
}

fp_status scorer_get_params(const fp_scorer* scorer, float* params, double* mean_std) {
  g_last_error.clear();
  if (!scorer || !params) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  return scorer_get_impl(scorer, params, mean_std);
}

fp_status scorer_set_params(fp_scorer* scorer, const float* params, const double* mean_std) {
  g_last_error.clear();
  if (!scorer || !params) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  return scorer_set_impl(scorer, params, mean_std);
}

void scorer_destroy(fp_scorer* scorer) {
  if (scorer) scorer_destroy_impl(scorer);
}

fp_status flow_problem_stats(const fp_problem* problem, fp_stats* out) {
  if (!problem || !out) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  *out = problem->st;
  out->alg_bytes = 0;
  if (problem->ctl_h)
    for (int c = 0; c < KC_N; ++c) out->alg_bytes += (int64_t)problem->ctl_h->bytes[c];
  return FP_OK;
}

int32_t flow_problem_kernel_times(const fp_problem* problem, int32_t max_kinds, const char** names,
                                  int64_t* launches, double* milliseconds, double* bytes) {
  if (!problem) return FP_ERR_STATE;
  int32_t n = 0;
  for (int k = 0; k < KK_COUNT && n < max_kinds; ++k, ++n) {
    if (names) names[n] = kernel_kind_name(k);
    if (launches) launches[n] = problem->k_launches[k];
    if (milliseconds) milliseconds[n] = problem->k_ms[k];
    if (bytes) {
      const int c = kernel_kind_class(k);
      bytes[n] = c >= 0 ? (double)problem->ctl_h->bytes[c] : 0.0;
    }
  }
  return n;
}

fp_status flow_problem_export_state(fp_problem* problem, void* hip_stream, int32_t* f_in,
                                    int32_t* f_out, int32_t* f_b, int32_t* labels,
                                    int32_t* excess) {
  g_last_error.clear();
  if (!problem) {
    set_error("NULL handle");
    return FP_ERR_STATE;
  }
  return export_state(problem, static_cast<hipStream_t>(hip_stream), f_in, f_out, f_b, labels,
                      excess);
}

void flow_problem_destroy(fp_problem* problem) {
  if (!problem) return;
  hipSetDevice(problem->device);
  hipDeviceSynchronize();
  release_problem(problem);
  delete problem;
}

void flow_release_cached_memory(void) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceSynchronize();
  release_cached_memory();
  (void)hipSetDevice(dev);
}

}  // extern "C"
#pragma GCC visibility pop
