// Kernel tabulation: K(d_k) = sum_l (2l+1)/(4 pi) k_l P_l(cos theta_k) on chord nodes d_k = k h.
//
// One thread per node. With u = 1 - cos(theta) = d^2 / 2, the three-term recurrence
// (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1} becomes, for D_l = P_l - P_{l-1},
//   D_{l+1} = (l D_l - (2l+1) u P_l) / (l+1),   P_{l+1} = P_l + D_{l+1},
// which never forms 1 - x and so keeps full relative precision near theta = 0.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace {

constexpr int kChunk = 1024;

__global__ __launch_bounds__(256) void tabulate_kernel(const double* __restrict__ k_ell, int lmax,
                                                       double h, int n_tab,
                                                       double* __restrict__ out) {
  __shared__ double s_k[kChunk];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double d = static_cast<double>(k) * h;
  const double u = fmin(0.5 * d * d, 2.0);
  const double inv4pi = 1.0 / (4.0 * M_PI);
  double p = 1.0;
  double dd = 0.0;
  double acc = 0.0;
  for (int base = 0; base <= lmax; base += kChunk) {
    __syncthreads();
    for (int t = threadIdx.x; t < kChunk && base + t <= lmax; t += blockDim.x) s_k[t] = k_ell[base + t];
    __syncthreads();
    const int end = min(lmax, base + kChunk - 1);
    for (int l = base; l <= end; ++l) {
      if (l > 0) {
        const int lm = l - 1;  // step P_{l-1} -> P_l
        dd = (static_cast<double>(lm) * dd - static_cast<double>(2 * lm + 1) * u * p) /
             static_cast<double>(lm + 1);
        p = p + dd;
      }
      acc += (static_cast<double>(2 * l + 1) * inv4pi) * s_k[l - base] * p;
    }
  }
  if (k < n_tab) out[k] = acc;
}

}  // namespace

namespace convreal {

hipError_t tabulate_device(const double* k_ell, int lmax, double h, int n_tab, double* table_host) {
  double* dk = nullptr;
  double* dt = nullptr;
  hipError_t e = hipMalloc(&dk, sizeof(double) * (lmax + 1));
  if (e != hipSuccess) return e;
  e = hipMalloc(&dt, sizeof(double) * n_tab);
  if (e == hipSuccess) e = hipMemcpy(dk, k_ell, sizeof(double) * (lmax + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const unsigned grid = static_cast<unsigned>((n_tab + 255) / 256);
    hipLaunchKernelGGL(tabulate_kernel, dim3(grid), dim3(256), 0, nullptr, dk, lmax, h, n_tab, dt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(table_host, dt, sizeof(double) * n_tab, hipMemcpyDeviceToHost);
  (void)hipFree(dk);
  if (dt) (void)hipFree(dt);
  return e;
}

}  // namespace convreal
