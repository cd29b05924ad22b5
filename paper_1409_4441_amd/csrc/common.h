// Device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace convreal {

// Blocks are dealt round-robin to the 8 XCDs of the MI355X; give each XCD a contiguous run of
// work items so that items sharing neighbour rings share an L2. Bijective on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int xcd = b & 7;
  const int idx = b >> 3;
  const int base = n >> 3;
  const int rem = n & 7;
  return xcd * base + min(xcd, rem) + idx;
}

// Chord constants of a ring pair: d^2 = A + B sin^2(dphi / 2), with
//   A = (z_i - z_j)^2 + (s_i - s_j)^2,  B = 4 s_i s_j  (s = sin theta),
// z and s differences formed from the exact integer numerators z = Z / q, q = 3 N^2:
//   s_i - s_j = (s_i^2 - s_j^2) / (s_i + s_j) = -(Z_i - Z_j)(Z_i + Z_j) / (q^2 (s_i + s_j)).
__device__ __forceinline__ void chord_constants(long long Zi, long long Zj, double si, double sj,
                                                double q, double* A, double* B) {
  const long long dZ = Zi - Zj;
  const long long sZ = Zi + Zj;
  const double dz = static_cast<double>(dZ) / q;
  const double ds = -static_cast<double>(dZ * sZ) / (q * q * (si + sj));
  *A = dz * dz + ds * ds;
  *B = 4.0 * si * sj;
}

// 4-point Lagrange interpolation on the uniform chord grid (FP64): segment k = floor(d/h)
// clamped to n_tab - 3, nodes k-1..k+2, ghost node T[-1] = T[1] (K is even in d).
__device__ __forceinline__ double interp_f64(const double* __restrict__ tab, int n_tab, double d,
                                             double inv_h) {
  const double t = d * inv_h;
  int k = static_cast<int>(t);
  if (k > n_tab - 3) k = n_tab - 3;
  const double f = t - static_cast<double>(k);
  const double tm1 = tab[k == 0 ? 1 : k - 1];
  const double t0 = tab[k];
  const double t1 = tab[k + 1];
  const double t2 = tab[k + 2];
  const double fm1 = f - 1.0;
  const double fm2 = f - 2.0;
  const double fp1 = f + 1.0;
  const double ff1 = f * fm1;
  const double g = fp1 * fm2;
  const double wm1 = -(ff1 * fm2) * (1.0 / 6.0);
  const double w2 = (fp1 * ff1) * (1.0 / 6.0);
  const double w0 = (g * fm1) * 0.5;
  const double w1 = -(g * f) * 0.5;
  return wm1 * tm1 + w0 * t0 + w1 * t1 + w2 * t2;
}

}  // namespace convreal
