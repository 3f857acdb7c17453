// Applying the move sequences of block-pair refinements to a k-way partition
// on the device (paper, section "Parallel Active Block Scheduling",
// paragraph "Apply Moves").
//
// The partition lives on the device with the pin count phi(e, b) of every
// net and block and the block weights.  A pair's result is the source side
// X of its region (built by flow_regions_build): a region vertex of block i
// outside X moves to block j, one of block j inside X to block i.  The
// sequences are applied one after another in the given order by one
// workgroup: moves whose vertex left its expected block are dropped; if
// blocks i or j would exceed Lmax nothing is applied; otherwise every move
// is applied and the exact change of sum w(e) (lambda(e) - 1) is summed from
// the pin-count transitions (a count of the source block dropping to zero
// gains w(e), a count of the target block rising to one loses w(e); with
// atomics on the counts every transition is seen exactly once, so the sum
// equals the sequential one); a negative total undoes the sequence.
// Readings: a sequence is tried only when its expected gain is positive;
// blocks other than i and j do not change, so only those two are checked.
#include <cstring>
#include <algorithm>
#include <memory>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "hf_host.h"

struct fp_partition {
  int device = 0;
  int32_t V = 0, E = 0, k = 0;
  int64_t P = 0;
  void* mem = nullptr;
  int32_t *off = nullptr, *pins = nullptr, *w = nullptr, *cv = nullptr, *block = nullptr;
  int32_t *voff = nullptr, *vnet = nullptr;
  int32_t* phi = nullptr;                 // E * k pin counts
  unsigned long long* bw = nullptr;       // k block weights
  unsigned long long* red = nullptr;      // reduction scratch
};

namespace hf {
namespace {

constexpr int kMvBlock = 1024;

size_t mv_align(size_t x) { return (x + 255) & ~size_t(255); }

int mv_grid(long long n) {
  long long b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

unsigned mv_bits(long long n) {
  unsigned b = 1;
  while (b < 31 && (1ll << b) < n) ++b;
  return b;
}

}  // namespace

__global__ void k_mv_zero(uint32_t* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_mv_check(int V, int E, int k, const int32_t* off, const int32_t* pins,
                           const int32_t* w, const int32_t* cv, const int32_t* block, int* err) {
  int e_ = 0;
  const int stride = gridDim.x * blockDim.x, t0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int e = t0; e < E; e += stride) {
    if (off[e + 1] < off[e]) e_ |= 1;
    if (w[e] < 1) e_ |= 2;
  }
  for (int v = t0; v < V; v += stride) {
    if (cv[v] < 1) e_ |= 4;
    if (block[v] < 0 || block[v] >= k) e_ |= 8;
  }
  if (t0 == 0 && off[0] != 0) e_ |= 1;
  if (e_) atomicOr(err, e_);
}

__global__ void k_mv_check_pins(int V, long long P, const int32_t* pins, int* err) {
  int e_ = 0;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P;
       p += (long long)gridDim.x * blockDim.x)
    if (pins[p] < 0 || pins[p] >= V) e_ |= 16;
  if (e_) atomicOr(err, e_);
}

__global__ void k_mv_pin_net(int E, const int32_t* off, int32_t* pin_net) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x)
    for (int p = off[e]; p < off[e + 1]; ++p) pin_net[p] = e;
}

__global__ void k_mv_offsets(const int32_t* keys, long long count, int n, int32_t* offs) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i <= count;
       i += (long long)gridDim.x * blockDim.x) {
    const int prev = i == 0 ? -1 : keys[i - 1];
    const int cur = i == count ? n : keys[i];
    for (int x = prev + 1; x <= cur; ++x) offs[x] = (int32_t)i;
  }
}

// phi(e, b) and block weights from the partition
__global__ void k_mv_counts(fp_partition pt) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < pt.E; e += gridDim.x * blockDim.x)
    for (int p = pt.off[e]; p < pt.off[e + 1]; ++p)
      atomicAdd(&pt.phi[(long long)e * pt.k + pt.block[pt.pins[p]]], 1);
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < pt.V; v += gridDim.x * blockDim.x)
    atomicAdd(&pt.bw[pt.block[v]], (unsigned long long)pt.cv[v]);
}

// objective sum w(e) (lambda(e) - 1), added into *out
__global__ void k_mv_objective(fp_partition pt, unsigned long long* out) {
  unsigned long long acc = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < pt.E; e += gridDim.x * blockDim.x) {
    int lam = 0;
    for (int b = 0; b < pt.k; ++b) lam += pt.phi[(long long)e * pt.k + b] > 0;
    if (lam > 1) acc += (unsigned long long)pt.w[e] * (unsigned long long)(lam - 1);
  }
  if (acc) atomicAdd(out, acc);
}

// Workgroup sum of one value per thread (block-uniform).
__device__ long long mv_sum(long long v) {
  __shared__ long long part[kMvBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wid = threadIdx.x >> 6;
  if (__lane_id() == 0) part[wid] = v;
  __syncthreads();
  long long s = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += part[i];
  __syncthreads();
  return s;
}

struct MvSeq {
  int32_t npairs;
  const int32_t* pairs;        // 2 per pair
  const long long* vbase;      // per pair: first region vertex
  const long long* nloc;       // per pair: region vertices
  const int32_t* vgid;
  const int8_t* vside;         // 0 = region of block i, 1 = of block j
  const uint8_t* const* sides; // per pair: device pointer to its source side map
  const long long* gain_exp;   // per pair
  long long lmax;
  uint8_t* flag;               // scratch: max n bytes
  long long* out;              // per pair: status, gain, moves
};

// One workgroup; the sequences in order.
__global__ void __launch_bounds__(kMvBlock) k_mv_apply(fp_partition pt, MvSeq s) {
  for (int q = 0; q < s.npairs; ++q) {
    if (s.gain_exp[q] <= 0) {
      if (threadIdx.x == 0) {
        s.out[3 * q] = 0;
        s.out[3 * q + 1] = 0;
        s.out[3 * q + 2] = 0;
      }
      continue;
    }
    const int i = s.pairs[2 * q], j = s.pairs[2 * q + 1];
    const long long vb = s.vbase[q];
    const int n = (int)s.nloc[q];
    const uint8_t* side = s.sides[q];
    long long dwi = 0, cnt = 0;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
      const int u = s.vgid[vb + l];
      const int exp = s.vside[vb + l] ? j : i;
      const int to = side[l] ? i : j;
      const bool mv = to != exp && pt.block[u] == exp;
      s.flag[l] = mv ? 1 : 0;
      if (mv) {
        dwi += to == i ? (long long)pt.cv[u] : -(long long)pt.cv[u];
        ++cnt;
      }
    }
    dwi = mv_sum(dwi);
    cnt = mv_sum(cnt);
    const long long wi = (long long)pt.bw[i] + dwi, wj = (long long)pt.bw[j] - dwi;
    if (wi > s.lmax || wj > s.lmax) {
      if (threadIdx.x == 0) {
        s.out[3 * q] = 2;
        s.out[3 * q + 1] = 0;
        s.out[3 * q + 2] = 0;
      }
      continue;
    }
    long long gain = 0;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
      if (!s.flag[l]) continue;
      const int u = s.vgid[vb + l];
      const int frm = s.vside[vb + l] ? j : i, to = frm == i ? j : i;
      pt.block[u] = to;
      for (int x = pt.voff[u]; x < pt.voff[u + 1]; ++x) {
        const int e = pt.vnet[x];
        const long long base = (long long)e * pt.k;
        if (atomicSub(&pt.phi[base + frm], 1) == 1) gain += pt.w[e];
        if (atomicAdd(&pt.phi[base + to], 1) == 0) gain -= pt.w[e];
      }
    }
    gain = mv_sum(gain);
    if (gain < 0) {
      for (int l = threadIdx.x; l < n; l += blockDim.x) {
        if (!s.flag[l]) continue;
        const int u = s.vgid[vb + l];
        const int frm = s.vside[vb + l] ? j : i, to = frm == i ? j : i;
        pt.block[u] = frm;
        for (int x = pt.voff[u]; x < pt.voff[u + 1]; ++x) {
          const long long base = (long long)pt.vnet[x] * pt.k;
          atomicSub(&pt.phi[base + to], 1);
          atomicAdd(&pt.phi[base + frm], 1);
        }
      }
    } else if (threadIdx.x == 0) {
      pt.bw[i] = (unsigned long long)wi;
      pt.bw[j] = (unsigned long long)wj;
    }
    if (threadIdx.x == 0) {
      s.out[3 * q] = gain < 0 ? 3 : 1;
      s.out[3 * q + 1] = gain;
      s.out[3 * q + 2] = cnt;
    }
    __syncthreads();
  }
}

// cut[a * k + b] (a < b) = weight of the nets with pins in blocks a and b
// (the quotient graph; k <= 64)
__global__ void k_mv_pair_cuts(fp_partition pt, unsigned long long* cut) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < pt.E; e += gridDim.x * blockDim.x) {
    unsigned long long m = 0ull;
    for (int b = 0; b < pt.k; ++b)
      if (pt.phi[(long long)e * pt.k + b] > 0) m |= 1ull << b;
    if (__popcll(m) < 2) continue;
    const unsigned long long w = (unsigned long long)pt.w[e];
    for (unsigned long long ma = m; ma; ma &= ma - 1) {
      const int a = __builtin_ctzll(ma);
      for (unsigned long long mb = ma & (ma - 1); mb; mb &= mb - 1)
        atomicAdd(&cut[a * pt.k + __builtin_ctzll(mb)], w);
    }
  }
}

namespace {

fp_status mv_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    set_error("%s: out of device memory", what);
    return FP_ERR_OOM;
  }
  return hip_fail(e, what);
}

#define MV_TRY(expr, what)                          \
  do {                                              \
    const hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return mv_fail(e_, what); \
  } while (0)

}  // namespace

static fp_status partition_create(int32_t V, int32_t E, const int32_t* off_in,
                                  const int32_t* pins_in, const int32_t* w_in,
                                  const int32_t* cv_in, const int32_t* block_in, int32_t k,
                                  int32_t mem_kind, hipStream_t s, fp_partition** out) {
  int64_t P = 0;
  if (mem_kind == 0) {
    P = off_in[E];
  } else {
    int32_t p32 = 0;
    MV_TRY(hipMemcpyAsync(&p32, off_in + E, 4, hipMemcpyDeviceToHost, s), "reading");
    MV_TRY(hipStreamSynchronize(s), "reading");
    P = p32;
  }
  if (P < 0) {
    set_error("net_offsets[num_nets] = %lld is negative", (long long)P);
    return FP_ERR_INVALID;
  }
  std::unique_ptr<fp_partition, void (*)(fp_partition*)> pt(new fp_partition(),
                                                              [](fp_partition* x) {
                                                                if (x->mem) (void)hipFree(x->mem);
                                                                delete x;
                                                              });
  MV_TRY(hipGetDevice(&pt->device), "hipGetDevice");
  pt->V = V;
  pt->E = E;
  pt->k = k;
  pt->P = P;
  // sort temporary of the pins by vertex
  size_t tb = 0;
  MV_TRY(rocprim::radix_sort_pairs(nullptr, tb, (const int32_t*)nullptr, (int32_t*)nullptr,
                                   (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)P, 0u,
                                   mv_bits(V), s), "sizing the pin sort");
  size_t bytes = 0;
  std::vector<size_t> at;
  auto add = [&](size_t n) {
    at.push_back(bytes);
    bytes += mv_align(n + 1);
  };
  add((E + 1ull) * 4);             // 0 off
  add(P * 4ull);                   // 1 pins
  add(E * 4ull);                   // 2 w
  add(V * 4ull);                   // 3 cv
  add(V * 4ull);                   // 4 block
  add((V + 1ull) * 4);             // 5 voff
  add(P * 4ull);                   // 6 vnet
  add((size_t)E * k * 4ull);       // 7 phi
  add(k * 8ull);                   // 8 bw
  add(64);                         // 9 red
  add(P * 4ull);                   // 10 pin_net (build scratch)
  add(P * 4ull);                   // 11 sorted keys (build scratch)
  add(tb);                         // 12 sort temporary
  add(64);                         // 13 err
  MV_TRY(hipMalloc(&pt->mem, bytes), "allocating the partition");
  char* b = static_cast<char*>(pt->mem);
  pt->off = reinterpret_cast<int32_t*>(b + at[0]);
  pt->pins = reinterpret_cast<int32_t*>(b + at[1]);
  pt->w = reinterpret_cast<int32_t*>(b + at[2]);
  pt->cv = reinterpret_cast<int32_t*>(b + at[3]);
  pt->block = reinterpret_cast<int32_t*>(b + at[4]);
  pt->voff = reinterpret_cast<int32_t*>(b + at[5]);
  pt->vnet = reinterpret_cast<int32_t*>(b + at[6]);
  pt->phi = reinterpret_cast<int32_t*>(b + at[7]);
  pt->bw = reinterpret_cast<unsigned long long*>(b + at[8]);
  pt->red = reinterpret_cast<unsigned long long*>(b + at[9]);
  int32_t* pin_net = reinterpret_cast<int32_t*>(b + at[10]);
  int32_t* keys = reinterpret_cast<int32_t*>(b + at[11]);
  void* tmp = b + at[12];
  int* err = reinterpret_cast<int*>(b + at[13]);
  const hipMemcpyKind kind = mem_kind == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  MV_TRY(hipMemcpyAsync(pt->off, off_in, (E + 1ull) * 4, kind, s), "copying the hypergraph");
  if (P) MV_TRY(hipMemcpyAsync(pt->pins, pins_in, P * 4ull, kind, s), "copying the hypergraph");
  if (E) MV_TRY(hipMemcpyAsync(pt->w, w_in, E * 4ull, kind, s), "copying the hypergraph");
  MV_TRY(hipMemcpyAsync(pt->cv, cv_in, V * 4ull, kind, s), "copying the vertex weights");
  MV_TRY(hipMemcpyAsync(pt->block, block_in, V * 4ull, kind, s), "copying the blocks");
  k_mv_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(err), 1);
  k_mv_check<<<mv_grid(std::max(E, V)), 256, 0, s>>>(V, E, k, pt->off, pt->pins, pt->w, pt->cv,
                                                      pt->block, err);
  int herr = 0;
  MV_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "checking");
  MV_TRY(hipStreamSynchronize(s), "checking");
  if (!(herr & 1)) {
    k_mv_check_pins<<<mv_grid(P), 256, 0, s>>>(V, P, pt->pins, err);
    MV_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "checking");
    MV_TRY(hipStreamSynchronize(s), "checking");
  }
  if (herr) {
    set_error("invalid partition input (%s)",
              herr & 1 ? "net_offsets must start at 0 and be nondecreasing"
              : herr & 2 ? "net weights must be >= 1"
              : herr & 4 ? "vertex weights must be >= 1"
              : herr & 8 ? "block ids must lie in [0, k)"
                         : "pin ids must lie in [0, num_vertices)");
    return FP_ERR_INVALID;
  }
  k_mv_pin_net<<<mv_grid(E), 256, 0, s>>>(E, pt->off, pin_net);
  MV_TRY(rocprim::radix_sort_pairs(tmp, tb, pt->pins, keys, pin_net, pt->vnet, (size_t)P, 0u,
                                   mv_bits(V), s), "sorting the pins by vertex");
  k_mv_offsets<<<mv_grid(P + 1), 256, 0, s>>>(keys, P, V, pt->voff);
  k_mv_zero<<<mv_grid((long long)E * k), 256, 0, s>>>(reinterpret_cast<uint32_t*>(pt->phi),
                                                      (long long)E * k);
  k_mv_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(pt->bw), 2ll * k);
  k_mv_counts<<<mv_grid(std::max(E, V)), 256, 0, s>>>(*pt);
  MV_TRY(hipStreamSynchronize(s), "counting the pins per block");
  *out = pt.release();
  return FP_OK;
}

static fp_status partition_apply(fp_partition* pt, const fp_regions* rg,
                                 const uint8_t* const* sides, const int64_t* gains, int64_t lmax,
                                 hipStream_t s, int32_t* status, int64_t* gain_out,
                                 int32_t* moved) {
  const int npairs = rg->npairs;
  if (npairs == 0) return FP_OK;
  long long nmax = 1;
  for (int q = 0; q < npairs; ++q) nmax = std::max(nmax, rg->nloc[q]);
  void* mem = nullptr;
  size_t bytes = 0;
  std::vector<size_t> at;
  auto add = [&](size_t n) {
    at.push_back(bytes);
    bytes += mv_align(n + 1);
  };
  add(npairs * 8ull);   // 0 pairs (int32 x2)
  add(npairs * 8ull);   // 1 vbase
  add(npairs * 8ull);   // 2 nloc
  add(npairs * 8ull);   // 3 side pointers
  add(npairs * 8ull);   // 4 expected gains
  add((size_t)nmax);    // 5 flags
  add(npairs * 24ull);  // 6 out
  MV_TRY(hipMalloc(&mem, bytes), "allocating");
  std::unique_ptr<void, void (*)(void*)> guard(mem, [](void* p) { (void)hipFree(p); });
  char* b = static_cast<char*>(mem);
  MvSeq q{};
  q.npairs = npairs;
  q.pairs = reinterpret_cast<int32_t*>(b + at[0]);
  q.vbase = reinterpret_cast<long long*>(b + at[1]);
  q.nloc = reinterpret_cast<long long*>(b + at[2]);
  q.sides = reinterpret_cast<const uint8_t* const*>(b + at[3]);
  q.gain_exp = reinterpret_cast<long long*>(b + at[4]);
  q.flag = reinterpret_cast<uint8_t*>(b + at[5]);
  q.out = reinterpret_cast<long long*>(b + at[6]);
  q.vgid = rg->vgid;
  q.vside = rg->vside;
  q.lmax = lmax;
  MV_TRY(hipMemcpyAsync(b + at[0], rg->pairs.data(), npairs * 8ull, hipMemcpyHostToDevice, s),
         "copy");
  MV_TRY(hipMemcpyAsync(b + at[1], rg->vtx_base.data(), npairs * 8ull, hipMemcpyHostToDevice, s),
         "copy");
  MV_TRY(hipMemcpyAsync(b + at[2], rg->nloc.data(), npairs * 8ull, hipMemcpyHostToDevice, s),
         "copy");
  MV_TRY(hipMemcpyAsync(b + at[3], sides, npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  MV_TRY(hipMemcpyAsync(b + at[4], gains, npairs * 8ull, hipMemcpyHostToDevice, s), "copy");
  k_mv_apply<<<1, kMvBlock, 0, s>>>(*pt, q);
  std::vector<long long> res(3ull * npairs);
  MV_TRY(hipMemcpyAsync(res.data(), q.out, 24ull * npairs, hipMemcpyDeviceToHost, s), "reading");
  MV_TRY(hipStreamSynchronize(s), "applying the moves");
  for (int t = 0; t < npairs; ++t) {
    if (status) status[t] = (int32_t)res[3 * t];
    if (gain_out) gain_out[t] = res[3 * t + 1];
    if (moved) moved[t] = (int32_t)res[3 * t + 2];
  }
  return FP_OK;
}

// Refinement rounds around the batched solver (the paper's algorithm
// "Parallel Flow-Based Refinement" with its section "Parallel Active Block
// Scheduling"), synchronous rounds: the block pairs with a cut of at least
// min_cut and an active block, heaviest cut first (then block ids), get
// their regions built on the device, are solved at once as one disjoint-
// union network built from the regions (minimum cuts; the expected gain is
// cut_before - F) and their results applied in that order; the blocks of every pair applied with a
// positive gain are active in the next round.  The rounds stop when none is
// left, after max_rounds, or when a round improves the objective by less
// than min_improvement_ppm parts per million.
static fp_status partition_refine(fp_partition* pt, const fp_refine_config& c, hipStream_t s,
                                  fp_refine_result* res, int64_t* traj) {
  const int k = pt->k;
  if (k > 64) {
    set_error("refinement rounds need k <= 64, got %d", k);
    return FP_ERR_INVALID;
  }
  fp_refine_result r{};
  std::vector<unsigned long long> bw(k);
  int64_t obj = 0;
  fp_status st = flow_partition_get(pt, 0, s, nullptr, reinterpret_cast<int64_t*>(bw.data()),
                                    &obj);
  if (st != FP_OK) return st;
  long long cv = 0;
  for (int b = 0; b < k; ++b) cv += (long long)bw[b];
  const long long lmax = (100ll + c.eps_percent) * ((cv + k - 1) / k) / 100;
  r.objective_before = obj;
  if (traj) traj[0] = obj;
  std::vector<char> active(k, 1);
  unsigned long long* cut_d = nullptr;
  MV_TRY(hipMalloc(&cut_d, (size_t)k * k * 8), "allocating");
  std::unique_ptr<void, void (*)(void*)> cut_guard(cut_d, [](void* p) { (void)hipFree(p); });
  std::vector<unsigned long long> cut((size_t)k * k);
  for (int round = 0; round < c.max_rounds; ++round) {
    k_mv_zero<<<mv_grid(2ll * k * k), 256, 0, s>>>(reinterpret_cast<uint32_t*>(cut_d),
                                                    2ll * k * k);
    k_mv_pair_cuts<<<mv_grid(pt->E), 256, 0, s>>>(*pt, cut_d);
    MV_TRY(hipMemcpyAsync(cut.data(), cut_d, (size_t)k * k * 8, hipMemcpyDeviceToHost, s),
           "reading the quotient graph");
    MV_TRY(hipStreamSynchronize(s), "building the quotient graph");
    struct Cand {
      unsigned long long cut;
      int a, b;
    };
    std::vector<Cand> cand;
    for (int a = 0; a < k; ++a)
      for (int b = a + 1; b < k; ++b) {
        const unsigned long long w = cut[(size_t)a * k + b];
        if (w >= (unsigned long long)c.min_cut && w > 0 && (active[a] || active[b]))
          cand.push_back({w, a, b});
      }
    std::sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
      if (x.cut != y.cut) return x.cut > y.cut;
      if (x.a != y.a) return x.a < y.a;
      return x.b < y.b;
    });
    if (c.max_pairs > 0 && (int)cand.size() > c.max_pairs) cand.resize(c.max_pairs);
    if (cand.empty()) break;
    const int np = (int)cand.size();
    std::vector<int32_t> pairs(2ull * np);
    std::vector<int64_t> caps(2ull * np);
    for (int q = 0; q < np; ++q) {
      const long long cvi = (long long)bw[cand[q].a], cvj = (long long)bw[cand[q].b];
      const long long lim = (100ll + (long long)c.alpha * c.eps_percent) * ((cvi + cvj + 1) / 2) /
                            100;
      const long long side = (long long)(c.alpha / 2) * (long long)cand[q].cut;
      pairs[2 * q] = cand[q].a;
      pairs[2 * q + 1] = cand[q].b;
      caps[2 * q] = std::max(0ll, std::min(side, lim - cvj));
      caps[2 * q + 1] = std::max(0ll, std::min(side, lim - cvi));
    }
    fp_regions* rg = nullptr;
    st = flow_regions_build(pt->V, pt->E, pt->off, pt->pins, pt->w, pt->cv, pt->block, k, np,
                            pairs.data(), caps.data(), c.merge_identical ? 1 : 0, 1, s, &rg);
    if (st != FP_OK) return st;
    std::unique_ptr<fp_regions, void (*)(fp_regions*)> rg_guard(rg, flow_regions_destroy);
    std::vector<int64_t> flows(np);
    st = flow_regions_solve(rg, nullptr, s, flows.data());
    if (st != FP_OK) return st;
    std::vector<int64_t> gains(np), exact(np);
    std::vector<int32_t> status(np), moved(np);
    for (int q = 0; q < np; ++q) gains[q] = rg->info[(size_t)q * 16 + 4] - flows[q];
    st = flow_partition_apply(pt, rg, nullptr, gains.data(), lmax, s, status.data(),
                              exact.data(), moved.data());
    if (st != FP_OK) return st;
    std::vector<char> next(k, 0);
    for (int q = 0; q < np; ++q) {
      ++r.pairs_tried;
      if (status[q] == 1) {
        ++r.pairs_applied;
        r.moves += moved[q];
        if (exact[q] > 0) next[cand[q].a] = next[cand[q].b] = 1;
      } else if (status[q] == 2) {
        ++r.pairs_unbalanced;
      } else if (status[q] == 3) {
        ++r.pairs_reverted;
      }
    }
    active.swap(next);
    const int64_t prev = obj;
    st = flow_partition_get(pt, 0, s, nullptr, reinterpret_cast<int64_t*>(bw.data()), &obj);
    if (st != FP_OK) return st;
    r.rounds = round + 1;
    if (traj) traj[round + 1] = obj;
    if ((prev - obj) * 1000000ll < (int64_t)c.min_improvement_ppm * prev) break;
  }
  r.objective_after = obj;
  *res = r;
  return FP_OK;
}

}  // namespace hf

using namespace hf;

#pragma GCC visibility push(default)
extern "C" {

fp_status flow_partition_create(int32_t num_vertices, int32_t num_nets,
                                const int32_t* net_offsets, const int32_t* pins,
                                const int32_t* net_weights, const int32_t* vertex_weights,
                                const int32_t* blocks, int32_t k, int32_t mem_kind,
                                void* hip_stream, fp_partition** out) {
  set_error("");
  if (!out) {
    set_error("out is NULL");
    return FP_ERR_INVALID;
  }
  *out = nullptr;
  if (num_vertices < 1 || num_nets < 0) {
    set_error("need num_vertices >= 1 and num_nets >= 0 (got %d, %d)", num_vertices, num_nets);
    return FP_ERR_INVALID;
  }
  if (k < 2 || k > 4096) {
    set_error("k must lie in [2, 4096], got %d", k);
    return FP_ERR_INVALID;
  }
  if (mem_kind != 0 && mem_kind != 1) {
    set_error("mem_kind must be 0 (host) or 1 (device), got %d", mem_kind);
    return FP_ERR_INVALID;
  }
  if (!net_offsets || !vertex_weights || !blocks || (num_nets > 0 && !net_weights)) {
    set_error("NULL input pointer");
    return FP_ERR_INVALID;
  }
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const fp_status st = partition_create(num_vertices, num_nets, net_offsets, pins, net_weights,
                                        vertex_weights, blocks, k, mem_kind, s, out);
  if (st != FP_OK) (void)hipStreamSynchronize(s);
  return st;
}

fp_status flow_partition_apply(fp_partition* partition, const fp_regions* regions,
                               const uint8_t* const* vertex_sides, const int64_t* expected_gains,
                               int64_t lmax, void* hip_stream, int32_t* status, int64_t* gains,
                               int32_t* moved) {
  set_error("");
  if (!partition || !regions || (regions->npairs > 0 && !expected_gains)) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  std::vector<const uint8_t*> own;
  if (!vertex_sides) {
    if (!regions->solved) {
      set_error("vertex_sides is NULL and the regions have not been solved");
      return FP_ERR_STATE;
    }
    own.resize(regions->npairs);
    for (int q = 0; q < regions->npairs; ++q)
      own[q] = regions->sides + regions->vtx_base[q] + 2ll * q;
    vertex_sides = own.data();
  }
  if (regions->V != partition->V || regions->k != partition->k) {
    set_error("the regions were built for another hypergraph or k (V %d / %d, k %d / %d)",
              regions->V, partition->V, regions->k, partition->k);
    return FP_ERR_INVALID;
  }
  for (int q = 0; q < regions->npairs; ++q)
    if (!vertex_sides[q] && regions->nloc[q] > 0) {
      set_error("vertex_sides[%d] is NULL", q);
      return FP_ERR_INVALID;
    }
  return partition_apply(partition, regions, vertex_sides, expected_gains, lmax,
                         static_cast<hipStream_t>(hip_stream), status, gains, moved);
}

fp_status flow_partition_get(fp_partition* partition, int32_t mem_kind, void* hip_stream,
                             int32_t* blocks, int64_t* block_weights, int64_t* objective) {
  set_error("");
  if (!partition) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  if (mem_kind != 0 && mem_kind != 1) {
    set_error("mem_kind must be 0 (host) or 1 (device), got %d", mem_kind);
    return FP_ERR_INVALID;
  }
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  fp_partition* pt = partition;
  if (blocks) {
    const hipError_t e = hipMemcpyAsync(blocks, pt->block, pt->V * 4ull,
                                        mem_kind ? hipMemcpyDeviceToDevice
                                                 : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copying the blocks");
  }
  if (block_weights) {
    const hipError_t e = hipMemcpyAsync(block_weights, pt->bw, pt->k * 8ull,
                                        hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copying the block weights");
  }
  unsigned long long obj = 0;
  if (objective) {
    k_mv_zero<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(pt->red), 2);
    k_mv_objective<<<mv_grid(pt->E), 256, 0, s>>>(*pt, pt->red);
    const hipError_t e = hipMemcpyAsync(&obj, pt->red, 8, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "reading the objective");
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading the partition");
  if (objective) *objective = (int64_t)obj;
  return FP_OK;
}

fp_status flow_partition_refine(fp_partition* partition, const fp_refine_config* config,
                                void* hip_stream, fp_refine_result* result,
                                int64_t* objective_per_round) {
  set_error("");
  if (!partition || !result) {
    set_error("NULL argument");
    return FP_ERR_INVALID;
  }
  fp_refine_config c{};
  if (config) c = *config;
  if (c.max_rounds < 0 || c.min_cut < 0 || c.alpha < 0 || c.eps_percent < 0 ||
      c.min_improvement_ppm < 0 || c.max_pairs < 0 || c.reserved != 0) {
    set_error("invalid refinement configuration");
    return FP_ERR_INVALID;
  }
  if (c.max_rounds == 0) c.max_rounds = 16;
  if (c.min_cut == 0) c.min_cut = 10;
  if (c.alpha == 0) c.alpha = 16;
  if (c.eps_percent == 0) c.eps_percent = 3;
  if (c.min_improvement_ppm == 0) c.min_improvement_ppm = 1000;
  return partition_refine(partition, c, static_cast<hipStream_t>(hip_stream), result,
                          objective_per_round);
}

void flow_partition_destroy(fp_partition* partition) {
  if (!partition) return;
  if (partition->mem) (void)hipFree(partition->mem);
  delete partition;
}

}  // extern "C"
#pragma GCC visibility pop
