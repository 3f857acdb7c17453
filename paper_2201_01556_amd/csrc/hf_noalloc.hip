// maxflow_mincut_noalloc: the create -> solve -> source side sequence of
// one problem in a single call that allocates nothing.  Every device buffer
// the problem needs -- the layout that flow_problem_create would place in a
// pool of its own, the temporary memory of its pin sort, the control block
// -- is carved from one file-scope device array per GPU, and the host mirror
// of the control block is a file-scope host array per GPU.  The kernels are
// those of the other entry points; they receive pointers into the array as
// arguments.
#include <cstring>
#include <mutex>

#include "hf_host.h"

namespace hf {

// Largest scratch a problem may use: 64 MiB (problems up to roughly
// 700,000 pins; larger ones are rejected with FP_ERR_OVERFLOW).  Each GPU
// the library runs on holds the array until the process ends.
constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device (from hipGetSymbolAddress with that
// device current; the name itself is a host-side stand-in, not a device
// address) and the host mirror of the control block per device.
static void* g_scratch_ptr[kMaxDevices];
static Ctl g_ctl_mirror[kMaxDevices];
static std::mutex g_scratch_mu;

static fp_status scratch_of_current_device(int* dev_out, void** out) {
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d is beyond the %d devices the scratch table holds", dev, kMaxDevices);
    return FP_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (he != hipSuccess) return hip_fail(he, "hipGetSymbolAddress of the scratch array");
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the scratch array");
      return FP_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *dev_out = dev;
  *out = g_scratch_ptr[dev];
  return FP_OK;
}

}  // namespace hf

using namespace hf;

#pragma GCC visibility push(default)
extern "C" {

fp_status maxflow_mincut_noalloc(int32_t num_vertices, int32_t num_nets,
                                 const int32_t* net_offsets, const int32_t* pins,
                                 const int32_t* net_weights, const int32_t* sources,
                                 int32_t num_sources, const int32_t* sinks, int32_t num_sinks,
                                 int32_t mem_kind, void* hip_stream, int64_t* flow_value,
                                 uint8_t* vertex_side, uint8_t* net_side) {
  set_error("%s", "");
  if (num_vertices < 1 || num_nets < 0) {
    set_error("need num_vertices >= 1 and num_nets >= 0 (got %d, %d)", num_vertices, num_nets);
    return FP_ERR_INVALID;
  }
  if (num_sources < 1 || num_sinks < 1) {
    set_error("source and sink sets must be nonempty (got %d, %d)", num_sources, num_sinks);
    return FP_ERR_INVALID;
  }
  if (!net_offsets || !sources || !sinks || (num_nets > 0 && !net_weights) || !flow_value ||
      !vertex_side) {
    set_error("NULL argument");
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
  int dev = 0;
  void* ptr = nullptr;
  fp_status st = scratch_of_current_device(&dev, &ptr);
  if (st) return st;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  fp_problem pb;  // on the stack; its buffers live in the scratch array
  pb.device = dev;
  pb.V = num_vertices;
  pb.E = num_nets;
  pb.opt = resolve_options(nullptr);
  pb.ctl_h = &g_ctl_mirror[dev];
  st = build_problem(&pb, net_offsets, pins, net_weights, sources, num_sources, sinks, num_sinks,
                     mem_kind, s, ptr, kScratchBytes);
  if (st == FP_OK) {
    int64_t F = 0;
    st = solve_problem(&pb, s, &F);
    if (st == FP_OK) st = cut_problem(&pb, s, mem_kind, vertex_side, net_side);
    if (st == FP_OK) *flow_value = F;
  }
  if (st != FP_OK) (void)hipStreamSynchronize(s);  // leave no work on the scratch behind
  return st;
}

}  // extern "C"
#pragma GCC visibility pop
