// ring_window: for every (output ring i, neighbour ring j) pair, the constants of the
// pixel-pair chord and the azimuthal half-width of ring j inside the cut.
//
// For pixels on rings i and j separated by dphi in azimuth,
//   d^2 = (z_i - z_j)^2 + (s_i - s_j)^2 + 4 s_i s_j sin^2(dphi / 2) = A_ij + B_ij sin^2(dphi/2),
// (s = sin theta), so d <= d_cut  <=>  sin^2(dphi/2) <= (d_cut^2 - A_ij) / B_ij. The window half-width
// in pixels of ring j is dphi_max * n_j / (2 pi); a value >= n_j / 2 means the whole ring.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace {

__global__ __launch_bounds__(256) void ring_window_kernel(long long npairs, const int* __restrict__ pi,
                                                          const int* __restrict__ pj,
                                                          const long long* __restrict__ Z,
                                                          const double* __restrict__ s,
                                                          const int* __restrict__ rn, double q,
                                                          double dcut2, double* __restrict__ pA,
                                                          double* __restrict__ pB,
                                                          double* __restrict__ phw) {
  const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= npairs) return;
  const int i = pi[k];
  const int j = pj[k];
  double A, B;
  convreal::chord_constants(Z[i], Z[j], s[i], s[j], q, &A, &B);
  const int nj = rn[j];
  const double s2 = (dcut2 - A) / B;
  double hw;
  if (!(B > 0.0) || s2 >= 1.0) {
    hw = static_cast<double>(nj);
  } else if (s2 <= 0.0) {
    hw = 0.0;
  } else {
    hw = 2.0 * asin(sqrt(s2)) * static_cast<double>(nj) * (0.5 / M_PI);
  }
  pA[k] = A;
  pB[k] = B;
  phw[k] = hw;
}

}  // namespace

namespace convreal {

hipError_t launch_ring_window(const conv_real_plan* p, hipStream_t st) {
  const long long n = p->npairs_ring;
  const unsigned grid = static_cast<unsigned>((n + 255) / 256);
  const double q = 3.0 * static_cast<double>(p->nside) * static_cast<double>(p->nside);
  hipLaunchKernelGGL(ring_window_kernel, dim3(grid), dim3(256), 0, st, n, p->d_pi, p->d_pj, p->d_Z,
                     p->d_s, p->d_rn, q, p->dcut2, p->d_pA, p->d_pB, p->d_phw);
  return hipGetLastError();
}

}  // namespace convreal
