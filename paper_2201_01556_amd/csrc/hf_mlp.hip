// Learned pruning scorer: a 12 -> 64 -> 64 -> 1 perceptron (ReLU hidden
// units, sigmoid output) that scores block-pair flow problems by the
// probability that refining them improves the cut, so that low-scoring
// problems can be skipped.  It replaces the fixed pruning rule of the paper
// (section "Parallel Active Block Scheduling", paragraph "Implementation
// Details": skip pairs with a small cut) and is trained on outcomes of the
// plain run-everything schedule.
//
// Hand-written FP32 kernels (plain VALU: the layers are 64 wide and the
// whole network has 5,057 parameters):
//   k_norm_stats   column mean and population deviation of log1p(features)
//                  in float64 (one wave per column)
//   k_norm_apply   z-scored float features
//   k_fwd_bwd      one workgroup per tile of 64 samples: forward pass with
//                  parameters and activations in LDS, mean binary
//                  cross-entropy on logits, backward pass, per-tile partial
//                  gradients (fixed summation order)
//   k_reduce_adam  sum of the tile partials in tile order (deterministic),
//                  optional Adam step (Kingma and Ba)
//   k_predict      forward pass only, sigmoid probabilities
//
// Parameter layout (row-major): W1 [64 x 12], b1 [64], W2 [64 x 64], b2 [64],
// W3 [64], b3.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hf_host.h"

namespace hf {

constexpr int kIn = 12;
constexpr int kHid = 64;
constexpr int kTile = 64;  // samples per workgroup
constexpr int kMlpThreads = 256;
constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kHid * kIn;    // 768
constexpr int oW2 = ob1 + kHid;          // 832
constexpr int ob2 = oW2 + kHid * kHid;   // 4928
constexpr int oW3 = ob2 + kHid;          // 4992
constexpr int ob3 = oW3 + kHid;          // 5056
constexpr int kParams = ob3 + 1;         // 5057
static_assert(kParams == FP_SCORER_PARAMS, "parameter count");
constexpr int kPart = kParams + 1;       // partial gradients + partial loss

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per feature column: mean, then the population deviation (two
// passes, float64); a deviation below 1e-9 counts as a constant column.
__global__ void __launch_bounds__(kIn * 64) k_norm_stats(const int64_t* __restrict__ f, int n,
                                                         double* __restrict__ ms) {
  const int col = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) s += log1p((double)f[(size_t)i * kIn + col]);
  const double mean = wave_sum_f64(s) / (double)n;
  double q = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double d = log1p((double)f[(size_t)i * kIn + col]) - mean;
    q += d * d;
  }
  const double sd = sqrt(wave_sum_f64(q) / (double)n);
  if (lane == 0) {
    ms[col] = mean;
    ms[kIn + col] = sd > 1e-9 ? sd : 1.0;
  }
}

__global__ void k_norm_apply(const int64_t* __restrict__ f, int n, const double* __restrict__ ms,
                             float* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kIn) return;
  const int col = i % kIn;
  x[i] = (float)((log1p((double)f[i]) - ms[col]) / ms[kIn + col]);
}

// Forward (and with kGrad the backward) pass over one tile of samples.
template <bool kGrad>
__global__ void __launch_bounds__(kMlpThreads)
    k_fwd_bwd(const float* __restrict__ prm, const float* __restrict__ x,
              const float* __restrict__ y, int n, float inv_n, float* __restrict__ part,
              float* __restrict__ prob) {
  __shared__ float P[kParams];
  __shared__ float X[kTile * kIn];
  __shared__ float H1[kTile * kHid];
  __shared__ float H2[kTile * kHid];
  __shared__ float D2[kTile * kHid];  // dL/dz2, then dL/dz1
  __shared__ float DZ[kTile];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kTile;
  const int ns = min(kTile, n - s0);
  for (int i = tid; i < kParams; i += kMlpThreads) P[i] = prm[i];
  for (int i = tid; i < kTile * kIn; i += kMlpThreads)
    X[i] = i < ns * kIn ? x[(size_t)s0 * kIn + i] : 0.f;
  __syncthreads();
  const int h = tid & (kHid - 1);  // unit of this thread
  const int sq = tid >> 6;         // first sample (stride 4)
  // layer 1
  for (int s = sq; s < kTile; s += 4) {
    float z = P[ob1 + h];
#pragma unroll
    for (int j = 0; j < kIn; ++j) z += P[oW1 + h * kIn + j] * X[s * kIn + j];
    H1[s * kHid + h] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  // layer 2
  for (int s = sq; s < kTile; s += 4) {
    float z = P[ob2 + h];
    for (int k = 0; k < kHid; ++k) z += P[oW2 + h * kHid + k] * H1[s * kHid + k];
    H2[s * kHid + h] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  // output, dL/dz
  if (tid < kTile) {
    const int s = tid;
    float z = P[ob3];
    for (int k = 0; k < kHid; ++k) z += P[oW3 + k] * H2[s * kHid + k];
    float dz = 0.f;
    if (s < ns) {
      const float p = 1.f / (1.f + expf(-z));
      if (prob) prob[s0 + s] = p;
      if (kGrad) dz = (p - y[s0 + s]) * inv_n;
    }
    DZ[s] = dz;
  }
  if (!kGrad) return;
  __syncthreads();
  float* out = part + (size_t)blockIdx.x * kPart;
  // output layer gradients; dL/dz2
  if (tid < kHid) {
    float g = 0.f;
    for (int s = 0; s < kTile; ++s) g += DZ[s] * H2[s * kHid + tid];
    out[oW3 + tid] = g;
  }
  if (tid == kHid) {
    float g = 0.f;
    for (int s = 0; s < kTile; ++s) g += DZ[s];
    out[ob3] = g;
  }
  if (tid == kHid + 1) {
    // the tile's loss: softplus(z) - y z per sample (without overflow),
    // summed in sample order
    float l = 0.f;
    for (int s = 0; s < ns; ++s) {
      const float yy = y[s0 + s];
      float z = P[ob3];
      for (int k = 0; k < kHid; ++k) z += P[oW3 + k] * H2[s * kHid + k];
      const float sp = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
      l += (sp - yy * z) * inv_n;
    }
    out[kParams] = l;
  }
  for (int s = sq; s < kTile; s += 4)
    D2[s * kHid + h] = H2[s * kHid + h] > 0.f ? DZ[s] * P[oW3 + h] : 0.f;
  __syncthreads();
  // W2, b2: thread (h, quarter) sums over all samples for 16 inputs k
  {
    const int kq = tid >> 6;  // inputs kq*16 .. kq*16+15
    for (int kk = 0; kk < 16; ++kk) {
      const int k = kq * 16 + kk;
      float g = 0.f;
      for (int s = 0; s < kTile; ++s) g += D2[s * kHid + h] * H1[s * kHid + k];
      out[oW2 + h * kHid + k] = g;
    }
    if (kq == 0) {
      float g = 0.f;
      for (int s = 0; s < kTile; ++s) g += D2[s * kHid + h];
      out[ob2 + h] = g;
    }
  }
  __syncthreads();
  // dL/dz1 = (W2^T dz2) masked by layer 1, into H2 (no longer needed)
  for (int s = sq; s < kTile; s += 4) {
    float d = 0.f;
    for (int u = 0; u < kHid; ++u) d += D2[s * kHid + u] * P[oW2 + u * kHid + h];
    H2[s * kHid + h] = H1[s * kHid + h] > 0.f ? d : 0.f;
  }
  __syncthreads();
  // W1, b1
  for (int i = tid; i < kHid * kIn; i += kMlpThreads) {
    const int u = i / kIn, j = i % kIn;
    float g = 0.f;
    for (int s = 0; s < kTile; ++s) g += H2[s * kHid + u] * X[s * kIn + j];
    out[oW1 + i] = g;
  }
  if (tid < kHid) {
    float g = 0.f;
    for (int s = 0; s < kTile; ++s) g += H2[s * kHid + tid];
    out[ob1 + tid] = g;
  }
}

// Thread per parameter: gradient = sum of the tile partials in tile order;
// with update, one Adam step (c1, c2 = bias corrections 1/(1 - beta^t)).
__global__ void k_reduce_adam(const float* __restrict__ part, int tiles, float* __restrict__ prm,
                              float* __restrict__ m, float* __restrict__ v,
                              float* __restrict__ grad, float* __restrict__ loss, int update,
                              float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kParams) return;
  float g = 0.f;
  for (int t = 0; t < tiles; ++t) g += part[(size_t)t * kPart + i];
  if (i == kParams) {
    if (loss) *loss = g;
    return;
  }
  if (grad) grad[i] = g;
  if (update) {
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

}  // namespace hf

struct fp_scorer {
  int device = 0;
  void* mem = nullptr;  // params, m, v, grad, mean/std, loss
  float* prm = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  double* ms = nullptr;
  float* loss = nullptr;
  bool normalized = false;
  int step = 0;
};

namespace hf {

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

fp_status scorer_create_impl(const float* init, hipStream_t s, fp_scorer** out) {
  fp_scorer* sc = new (std::nothrow) fp_scorer();
  if (!sc) {
    set_error("host allocation failed");
    return FP_ERR_OOM;
  }
  for (int i = 0; i < kParams; ++i)
    if (!std::isfinite(init[i])) {
      delete sc;
      set_error("initial parameter %d is not finite", i);
      return FP_ERR_INVALID;
    }
  hipGetDevice(&sc->device);
  const size_t fp = al(kParams * sizeof(float));
  const size_t total = 4 * fp + al(2 * kIn * sizeof(double)) + al(sizeof(float));
  hipError_t he = hipMalloc(&sc->mem, total);
  if (he != hipSuccess) {
    delete sc;
    return hip_fail(he, "allocating the scorer");
  }
  char* p = static_cast<char*>(sc->mem);
  sc->prm = reinterpret_cast<float*>(p);
  sc->m = reinterpret_cast<float*>(p + fp);
  sc->v = reinterpret_cast<float*>(p + 2 * fp);
  sc->grad = reinterpret_cast<float*>(p + 3 * fp);
  sc->ms = reinterpret_cast<double*>(p + 4 * fp);
  sc->loss = reinterpret_cast<float*>(p + 4 * fp + al(2 * kIn * sizeof(double)));
  he = hipMemsetAsync(sc->mem, 0, total, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(sc->prm, init, kParams * sizeof(float), hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    (void)hipFree(sc->mem);
    delete sc;
    return hip_fail(he, "initialising the scorer");
  }
  *out = sc;
  return FP_OK;
}

void scorer_destroy_impl(fp_scorer* sc) {
  if (sc->mem) (void)hipFree(sc->mem);
  delete sc;
}

// Device copies of features (and labels) with lifetime of the call.
struct Staged {
  void* mem = nullptr;
  const int64_t* f = nullptr;
  const float* y = nullptr;
  float* x = nullptr;
  float* part = nullptr;
  float* prob = nullptr;
  float* losses = nullptr;
  ~Staged() {
    if (mem) (void)hipFree(mem);
  }
};

static fp_status stage(const int64_t* f, const float* y, int n, int mem_kind, int tiles,
                       bool want_part, bool want_prob, int loss_slots, hipStream_t s, Staged* st) {
  const size_t fb = (size_t)n * kIn * sizeof(int64_t);
  const size_t yb = y ? (size_t)n * sizeof(float) : 0;
  size_t total = al((size_t)n * kIn * sizeof(float));
  if (mem_kind == 0) total += al(fb) + al(yb);
  if (want_part) total += al((size_t)tiles * kPart * sizeof(float));
  if (want_prob) total += al((size_t)n * sizeof(float));
  total += al((size_t)loss_slots * sizeof(float));
  hipError_t he = hipMalloc(&st->mem, total);
  if (he != hipSuccess) {
    st->mem = nullptr;
    return hip_fail(he, "allocating scorer buffers");
  }
  char* p = static_cast<char*>(st->mem);
  st->x = reinterpret_cast<float*>(p);
  p += al((size_t)n * kIn * sizeof(float));
  if (mem_kind == 0) {
    int64_t* fd = reinterpret_cast<int64_t*>(p);
    p += al(fb);
    he = hipMemcpyAsync(fd, f, fb, hipMemcpyHostToDevice, s);
    st->f = fd;
    if (y) {
      float* yd = reinterpret_cast<float*>(p);
      p += al(yb);
      if (he == hipSuccess) he = hipMemcpyAsync(yd, y, yb, hipMemcpyHostToDevice, s);
      st->y = yd;
    }
    if (he != hipSuccess) return hip_fail(he, "copying scorer inputs");
  } else {
    st->f = f;
    st->y = y;
  }
  if (want_part) {
    st->part = reinterpret_cast<float*>(p);
    p += al((size_t)tiles * kPart * sizeof(float));
  }
  if (want_prob) {
    st->prob = reinterpret_cast<float*>(p);
    p += al((size_t)n * sizeof(float));
  }
  st->losses = reinterpret_cast<float*>(p);
  return FP_OK;
}

fp_status scorer_fit_impl(fp_scorer* sc, const int64_t* f, int n, int mem_kind, hipStream_t s) {
  Staged st;
  fp_status r = stage(f, nullptr, n, mem_kind, 0, false, false, 0, s, &st);
  if (r) return r;
  k_norm_stats<<<1, kIn * 64, 0, s>>>(st.f, n, sc->ms);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "feature statistics");
  sc->normalized = true;
  return FP_OK;
}

// Shared by gradient and training: normalized features, then `steps`
// forward / backward / reduce (+ Adam when update) rounds.
static fp_status run_steps(fp_scorer* sc, const int64_t* f, const float* y, int n, int mem_kind,
                           int steps, bool update, float lr, hipStream_t s, float* grad_host,
                           float* loss_host, float* losses_host) {
  if (!sc->normalized) {
    set_error("fit the feature normalization first");
    return FP_ERR_STATE;
  }
  const int tiles = (n + kTile - 1) / kTile;
  Staged st;
  fp_status r = stage(f, y, n, mem_kind, tiles, true, false, steps, s, &st);
  if (r) return r;
  k_norm_apply<<<(n * kIn + 255) / 256, 256, 0, s>>>(st.f, n, sc->ms, st.x);
  const float inv_n = 1.f / (float)n;
  const double b1 = 0.9, b2 = 0.999;
  for (int t = 0; t < steps; ++t) {
    k_fwd_bwd<true><<<tiles, kMlpThreads, 0, s>>>(sc->prm, st.x, st.y, n, inv_n, st.part,
                                                  nullptr);
    const int step = sc->step + 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, step)));
    k_reduce_adam<<<(kParams + 1 + 255) / 256, 256, 0, s>>>(
        st.part, tiles, sc->prm, sc->m, sc->v, sc->grad, st.losses + t, update ? 1 : 0, lr,
        (float)b1, (float)b2, 1e-8f, c1, c2);
    if (update) sc->step = step;
  }
  hipError_t he = hipGetLastError();
  if (he == hipSuccess && grad_host)
    he = hipMemcpyAsync(grad_host, sc->grad, kParams * sizeof(float), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && loss_host && steps > 0)
    he = hipMemcpyAsync(loss_host, st.losses + steps - 1, sizeof(float), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && losses_host && steps > 0)
    he = hipMemcpyAsync(losses_host, st.losses, (size_t)steps * sizeof(float),
                        hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "scorer steps");
  return FP_OK;
}

fp_status scorer_gradient_impl(fp_scorer* sc, const int64_t* f, const float* y, int n,
                               int mem_kind, hipStream_t s, float* grad, float* loss) {
  return run_steps(sc, f, y, n, mem_kind, 1, false, 0.f, s, grad, loss, nullptr);
}

fp_status scorer_train_impl(fp_scorer* sc, const int64_t* f, const float* y, int n, int mem_kind,
                            int steps, float lr, hipStream_t s, float* losses) {
  return run_steps(sc, f, y, n, mem_kind, steps, true, lr, s, nullptr, nullptr, losses);
}

fp_status scorer_predict_impl(fp_scorer* sc, const int64_t* f, int n, int mem_kind,
                              hipStream_t s, float* prob) {
  if (!sc->normalized) {
    set_error("fit the feature normalization first");
    return FP_ERR_STATE;
  }
  const int tiles = (n + kTile - 1) / kTile;
  Staged st;
  fp_status r = stage(f, nullptr, n, mem_kind, tiles, false, mem_kind == 0, 0, s, &st);
  if (r) return r;
  float* out = mem_kind == 0 ? st.prob : prob;
  k_norm_apply<<<(n * kIn + 255) / 256, 256, 0, s>>>(st.f, n, sc->ms, st.x);
  k_fwd_bwd<false><<<tiles, kMlpThreads, 0, s>>>(sc->prm, st.x, nullptr, n, 0.f, nullptr, out);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess && mem_kind == 0)
    he = hipMemcpyAsync(prob, out, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "scorer prediction");
  return FP_OK;
}

fp_status scorer_get_impl(const fp_scorer* sc, float* params, double* mean_std) {
  hipError_t he = hipMemcpy(params, sc->prm, kParams * sizeof(float), hipMemcpyDeviceToHost);
  if (he == hipSuccess && mean_std)
    he = hipMemcpy(mean_std, sc->ms, 2 * kIn * sizeof(double), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return hip_fail(he, "reading the scorer");
  return FP_OK;
}

fp_status scorer_set_impl(fp_scorer* sc, const float* params, const double* mean_std) {
  for (int i = 0; i < kParams; ++i)
    if (!std::isfinite(params[i])) {
      set_error("parameter %d is not finite", i);
      return FP_ERR_INVALID;
    }
  for (int i = 0; mean_std && i < 2 * kIn; ++i)
    if (!std::isfinite(mean_std[i]) || (i >= kIn && mean_std[i] <= 0.0)) {
      set_error("normalization entry %d is not usable", i);
      return FP_ERR_INVALID;
    }
  hipError_t he = hipMemcpy(sc->prm, params, kParams * sizeof(float), hipMemcpyHostToDevice);
  if (he == hipSuccess && mean_std) {
    he = hipMemcpy(sc->ms, mean_std, 2 * kIn * sizeof(double), hipMemcpyHostToDevice);
    sc->normalized = true;
  }
  if (he != hipSuccess) return hip_fail(he, "loading the scorer");
  return FP_OK;
}

}  // namespace hf
