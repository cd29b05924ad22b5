// Device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace convreal {

// Buffer resources: word 3 for untyped 32-bit accesses, the range given to every resource, and the
// offset that a lane with nothing to load gives (past the range: the hardware returns zeros without
// a memory access). Such loads are issued by every lane on every path, so that the compiler can
// count the loads in flight, while only the data in use moves through the caches. Offsets are 32-bit
// byte offsets from the resource's base.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kBufferRange = 0x7fffffff;
constexpr unsigned kNoLoad = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_resource(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, kBufferRange, kBufferWord3);
}

// Load of a value that is the same in every lane and read-only for the kernel's lifetime (plan
// tables written at set-up): through the constant address space, so that it becomes a scalar load
// into SGPRs and the compiler treats the result as wave-uniform.
template <typename T>
__device__ __forceinline__ T ldu(const T& ref) {
  return *(const __attribute__((address_space(4))) T*)(&ref);
}

// ldu for a record, word by word (the words merge into one wide scalar load)
template <typename T>
__device__ __forceinline__ T ldu_record(const T& ref) {
  static_assert(sizeof(T) % 4 == 0, "records are whole 32-bit words");
  T out;
  const __attribute__((address_space(4))) unsigned* src = (const __attribute__((address_space(4))) unsigned*)(&ref);
  unsigned* dst = reinterpret_cast<unsigned*>(&out);
#pragma unroll
  for (int k = 0; k < static_cast<int>(sizeof(T) / 4); ++k) dst[k] = src[k];
  return out;
}

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
