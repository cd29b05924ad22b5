// Learned split network of libconvreal: 3 -> 64 -> 64 -> 2 perceptron, tanh hidden layers.
//
// One training step is two launches plus a loss reduction:
//   mlp_sample_kernel  one thread per sample: forward pass with the parameters staged in LDS (the
//                      whole network is 18 KB), then the back-propagated deltas of that sample
//                      dy = (y - t) / n, dh2 = (W3^T dy) (1 - h2^2), dh1 = (W2^T dh2) (1 - h1^2),
//                      written with the activations to per-sample rows
//   mlp_param_kernel   one thread per parameter: its gradient as a sum over samples in fixed order
//                      (FP64 accumulator, so results do not depend on the launch) and, when
//                      training, the Adam update of that parameter
//   mlp_loss_kernel    one workgroup: the loss, a fixed-order tree sum of per-sample terms
// The gradient needs no atomics and every step is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/convlearn.h"
#include "internal.h"

using convreal::set_error;

namespace {

constexpr int H = CONV_MLP_HIDDEN;
constexpr int NIN = CONV_MLP_IN;
constexpr int NOUT = CONV_MLP_OUT;
constexpr int NP = CONV_MLP_NPARAMS;
constexpr int OW1 = 0;
constexpr int OB1 = OW1 + H * NIN;
constexpr int OW2 = OB1 + H;
constexpr int OB2 = OW2 + H * H;
constexpr int OW3 = OB2 + H;
constexpr int OB3 = OW3 + NOUT * H;
static_assert(OB3 + NOUT == NP, "parameter layout");

constexpr int kThreads = 256;

struct Buffers {
  float* h1;    // [n][H]
  float* h2;    // [n][H]
  float* dh1;   // [n][H]
  float* dh2;   // [n][H]
  float* dy;    // [n][NOUT]
  float* lossv; // [n]
};

struct AdamArgs {
  float lr, b1, b2, eps;
  float bc1, bc2;  // 1 - b1^t, 1 - b2^t
};

__device__ __forceinline__ void stage_params(const float* __restrict__ params, float* __restrict__ P) {
  for (int k = threadIdx.x; k < NP; k += blockDim.x) P[k] = params[k];
  __syncthreads();
}

__device__ __forceinline__ void forward_one(const float* __restrict__ P, const float (&x)[NIN], float (&h1)[H],
                                            float (&h2)[H], float (&y)[NOUT]) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    float s = P[OB1 + i];
#pragma unroll
    for (int k = 0; k < NIN; ++k) s = fmaf(P[OW1 + NIN * i + k], x[k], s);
    h1[i] = tanhf(s);
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    float s = P[OB2 + i];
#pragma unroll
    for (int k = 0; k < H; ++k) s = fmaf(P[OW2 + H * i + k], h1[k], s);
    h2[i] = tanhf(s);
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float s = P[OB3 + o];
#pragma unroll
    for (int k = 0; k < H; ++k) s = fmaf(P[OW3 + H * o + k], h2[k], s);
    y[o] = s;
  }
}

__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(const float* __restrict__ params,
                                                               const float* __restrict__ x, int n,
                                                               float* __restrict__ y) {
  __shared__ float P[NP];
  stage_params(params, P);
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= n) return;
  float xi[NIN], h1[H], h2[H], yo[NOUT];
#pragma unroll
  for (int k = 0; k < NIN; ++k) xi[k] = x[static_cast<size_t>(s) * NIN + k];
  forward_one(P, xi, h1, h2, yo);
#pragma unroll
  for (int o = 0; o < NOUT; ++o) y[static_cast<size_t>(s) * NOUT + o] = yo[o];
}

__global__ __launch_bounds__(kThreads) void mlp_sample_kernel(const float* __restrict__ params,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ t, int n, Buffers b) {
  __shared__ float P[NP];
  stage_params(params, P);
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= n) return;
  float xi[NIN], h1[H], h2[H], y[NOUT];
#pragma unroll
  for (int k = 0; k < NIN; ++k) xi[k] = x[static_cast<size_t>(s) * NIN + k];
  forward_one(P, xi, h1, h2, y);
  const float inv_n = 1.0f / static_cast<float>(n);
  float dy[NOUT];
  float l = 0.0f;
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const float r = y[o] - t[static_cast<size_t>(s) * NOUT + o];
    dy[o] = r * inv_n;
    l = fmaf(r, r, l);
  }
  b.lossv[s] = 0.5f * l * inv_n;
  float dh2[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    float g = 0.0f;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) g = fmaf(P[OW3 + H * o + k], dy[o], g);
    dh2[k] = g * (1.0f - h2[k] * h2[k]);
  }
  float* h1r = b.h1 + static_cast<size_t>(s) * H;
  float* h2r = b.h2 + static_cast<size_t>(s) * H;
  float* d1r = b.dh1 + static_cast<size_t>(s) * H;
  float* d2r = b.dh2 + static_cast<size_t>(s) * H;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    float g = 0.0f;
#pragma unroll
    for (int i = 0; i < H; ++i) g = fmaf(P[OW2 + H * i + k], dh2[i], g);
    d1r[k] = g * (1.0f - h1[k] * h1[k]);
    h1r[k] = h1[k];
    h2r[k] = h2[k];
    d2r[k] = dh2[k];
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) b.dy[static_cast<size_t>(s) * NOUT + o] = dy[o];
}

// gradient of parameter p: sum over samples of (delta of its output unit) x (its input activation)
__global__ __launch_bounds__(kThreads) void mlp_param_kernel(const float* __restrict__ x, int n, Buffers b,
                                                             float* __restrict__ grad, float* __restrict__ params,
                                                             float* __restrict__ m1, float* __restrict__ m2,
                                                             AdamArgs a, int update) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= NP) return;
  const float* delta;
  int dstride, di;
  const float* act = nullptr;  // nullptr: bias (input activation 1)
  int astride = 0, ai = 0;
  if (p < OB1) {
    delta = b.dh1; dstride = H; di = p / NIN;
    act = x; astride = NIN; ai = p % NIN;
  } else if (p < OW2) {
    delta = b.dh1; dstride = H; di = p - OB1;
  } else if (p < OB2) {
    delta = b.dh2; dstride = H; di = (p - OW2) / H;
    act = b.h1; astride = H; ai = (p - OW2) % H;
  } else if (p < OW3) {
    delta = b.dh2; dstride = H; di = p - OB2;
  } else if (p < OB3) {
    delta = b.dy; dstride = NOUT; di = (p - OW3) / H;
    act = b.h2; astride = H; ai = (p - OW3) % H;
  } else {
    delta = b.dy; dstride = NOUT; di = p - OB3;
  }
  double acc = 0.0;
  if (act) {
    for (int s = 0; s < n; ++s)
      acc = fma(static_cast<double>(delta[static_cast<size_t>(s) * dstride + di]),
                static_cast<double>(act[static_cast<size_t>(s) * astride + ai]), acc);
  } else {
    for (int s = 0; s < n; ++s) acc += static_cast<double>(delta[static_cast<size_t>(s) * dstride + di]);
  }
  const float g = static_cast<float>(acc);
  if (grad) grad[p] = g;
  if (update) {
    const float mm = a.b1 * m1[p] + (1.0f - a.b1) * g;
    const float vv = a.b2 * m2[p] + (1.0f - a.b2) * g * g;
    m1[p] = mm;
    m2[p] = vv;
    params[p] -= a.lr * (mm / a.bc1) / (sqrtf(vv / a.bc2) + a.eps);
  }
}

__global__ __launch_bounds__(kThreads) void mlp_loss_kernel(const float* __restrict__ lossv, int n,
                                                            float* __restrict__ out) {
  __shared__ double part[kThreads];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += kThreads) s += static_cast<double>(lossv[k]);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = static_cast<float>(part[0]);
}

}  // namespace

struct conv_mlp {
  int device = 0;
  int max_batch = 0;
  long long step = 0;
  float* params = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  Buffers b{};
  float* scratch_loss = nullptr;
};

namespace {

int hip_err(hipError_t e, const char* what) {
  (void)hipGetLastError();
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CONV_REAL_ENOMEM : CONV_REAL_EHIP;
}

void free_all(conv_mlp* m) {
  for (void* p : {static_cast<void*>(m->params), static_cast<void*>(m->m1), static_cast<void*>(m->m2),
                  static_cast<void*>(m->b.h1), static_cast<void*>(m->b.h2), static_cast<void*>(m->b.dh1),
                  static_cast<void*>(m->b.dh2), static_cast<void*>(m->b.dy), static_cast<void*>(m->b.lossv),
                  static_cast<void*>(m->scratch_loss)})
    if (p) (void)hipFree(p);
}

int check_batch(const conv_mlp* m, int n, const char* who) {
  if (!m) {
    set_error(std::string(who) + ": NULL network");
    return CONV_REAL_EINVAL;
  }
  if (n < 1 || n > m->max_batch) {
    set_error(std::string(who) + ": n must be in [1, max_batch]");
    return CONV_REAL_EINVAL;
  }
  return CONV_REAL_OK;
}

// activations and deltas for the batch, then per-parameter gradients (and the Adam update)
hipError_t launch_step(conv_mlp* m, const float* x, const float* t, int n, float* grad, float* loss,
                       const AdamArgs* adam, hipStream_t st) {
  const unsigned gs = static_cast<unsigned>((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(mlp_sample_kernel, dim3(gs), dim3(kThreads), 0, st, m->params, x, t, n, m->b);
  if (loss) hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(kThreads), 0, st, m->b.lossv, n, loss);
  AdamArgs a{};
  if (adam) a = *adam;
  const unsigned gp = static_cast<unsigned>((NP + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(mlp_param_kernel, dim3(gp), dim3(kThreads), 0, st, x, n, m->b, grad, m->params, m->m1, m->m2,
                     a, adam ? 1 : 0);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int conv_mlp_create(conv_mlp** out, int max_batch) {
  if (!out || max_batch < 1 || max_batch > CONV_MLP_MAX_BATCH) {
    set_error("conv_mlp_create: NULL output or max_batch out of range");
    return CONV_REAL_EINVAL;
  }
  conv_mlp* m = new (std::nothrow) conv_mlp;
  if (!m) {
    set_error("conv_mlp_create: out of memory");
    return CONV_REAL_ENOMEM;
  }
  hipError_t e = hipGetDevice(&m->device);
  if (e != hipSuccess) {
    delete m;
    return hip_err(e, "conv_mlp_create");
  }
  m->max_batch = max_batch;
  const size_t nb = static_cast<size_t>(max_batch);
  struct {
    float** p;
    size_t count;
  } allocs[] = {{&m->params, NP},      {&m->m1, NP},         {&m->m2, NP},        {&m->b.h1, nb * H},
                {&m->b.h2, nb * H},    {&m->b.dh1, nb * H},  {&m->b.dh2, nb * H}, {&m->b.dy, nb * NOUT},
                {&m->b.lossv, nb},     {&m->scratch_loss, 1}};
  for (auto& a : allocs) {
    e = hipMalloc(reinterpret_cast<void**>(a.p), a.count * sizeof(float));
    if (e != hipSuccess) {
      free_all(m);
      delete m;
      return hip_err(e, "conv_mlp_create");
    }
  }
  for (float* p : {m->params, m->m1, m->m2}) {
    e = hipMemset(p, 0, NP * sizeof(float));
    if (e != hipSuccess) {
      free_all(m);
      delete m;
      return hip_err(e, "conv_mlp_create");
    }
  }
  *out = m;
  return CONV_REAL_OK;
}

int conv_mlp_destroy(conv_mlp* m) {
  if (!m) return CONV_REAL_OK;
  (void)hipDeviceSynchronize();
  free_all(m);
  delete m;
  return CONV_REAL_OK;
}

int conv_mlp_set_params(conv_mlp* m, const float* host_params) {
  if (!m || !host_params) {
    set_error("conv_mlp_set_params: NULL argument");
    return CONV_REAL_EINVAL;
  }
  for (int k = 0; k < NP; ++k) {
    if (!std::isfinite(host_params[k])) {
      set_error("conv_mlp_set_params: non-finite parameter");
      return CONV_REAL_EINVAL;
    }
  }
  hipError_t e = hipMemcpy(m->params, host_params, NP * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->m1, 0, NP * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->m2, 0, NP * sizeof(float));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_err(e, "conv_mlp_set_params");
  m->step = 0;
  return CONV_REAL_OK;
}

int conv_mlp_get_params(conv_mlp* m, float* host_params) {
  if (!m || !host_params) {
    set_error("conv_mlp_get_params: NULL argument");
    return CONV_REAL_EINVAL;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host_params, m->params, NP * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_err(e, "conv_mlp_get_params");
  return CONV_REAL_OK;
}

int conv_mlp_forward(conv_mlp* m, const float* x, int n, float* y, void* stream) {
  if (int r = check_batch(m, n, "conv_mlp_forward")) return r;
  if (!x || !y) {
    set_error("conv_mlp_forward: NULL x or y");
    return CONV_REAL_EINVAL;
  }
  const unsigned gs = static_cast<unsigned>((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(gs), dim3(kThreads), 0, static_cast<hipStream_t>(stream), m->params, x,
                     n, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "conv_mlp_forward");
  return CONV_REAL_OK;
}

int conv_mlp_gradient(conv_mlp* m, const float* x, const float* t, int n, float* grad, float* loss, void* stream) {
  if (int r = check_batch(m, n, "conv_mlp_gradient")) return r;
  if (!x || !t || !grad || !loss) {
    set_error("conv_mlp_gradient: NULL argument");
    return CONV_REAL_EINVAL;
  }
  hipError_t e = launch_step(m, x, t, n, grad, loss, nullptr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_err(e, "conv_mlp_gradient");
  return CONV_REAL_OK;
}

int conv_mlp_train(conv_mlp* m, const float* x, const float* t, int n, int steps, const conv_adam* opt,
                   float* loss_hist, void* stream) {
  if (int r = check_batch(m, n, "conv_mlp_train")) return r;
  if (!x || !t || !opt || steps < 0) {
    set_error("conv_mlp_train: NULL argument or steps < 0");
    return CONV_REAL_EINVAL;
  }
  if (!(opt->lr > 0.0f) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) || !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) ||
      !(opt->eps > 0.0f)) {
    set_error("conv_mlp_train: need lr > 0, beta1 and beta2 in [0, 1), eps > 0");
    return CONV_REAL_EINVAL;
  }
  const hipStream_t st = static_cast<hipStream_t>(stream);
  for (int k = 0; k < steps; ++k) {
    const long long t_adam = m->step + 1;
    AdamArgs a;
    a.lr = opt->lr;
    a.b1 = opt->beta1;
    a.b2 = opt->beta2;
    a.eps = opt->eps;
    a.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(opt->beta1), static_cast<double>(t_adam)));
    a.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(opt->beta2), static_cast<double>(t_adam)));
    hipError_t e = launch_step(m, x, t, n, nullptr, loss_hist ? loss_hist + k : nullptr, &a, st);
    if (e != hipSuccess) return hip_err(e, "conv_mlp_train");
    m->step = t_adam;
  }
  return CONV_REAL_OK;
}

}  // extern "C"
