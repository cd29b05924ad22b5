// Radix-2 FFT in LDS (FP64), shared by the ring-FFT real-space method and the spherical-harmonic
// transforms: n a power of two, the sequence placed in bit-reversed order, then log2 n butterfly
// stages, two per pass over LDS where they pair up; twiddles exp(-2 pi i m / n), m < n / 2, from a
// table written by the host or from two small tables in LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace convreal {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}

__device__ __forceinline__ int bitrev(int v, int logn) {
  return static_cast<int>(__builtin_bitreverse32(static_cast<unsigned>(v)) >> (32 - logn));
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return double2{a.x - b.x, a.y - b.y}; }

// Twiddles exp(-2 pi i m / n), m < n / 2, as the product of two small tables in LDS (m = 64 h + l):
// no global load inside the butterfly passes, one complex multiply each.
struct LdsTwiddles {
  const double2* hi;   // exp(-2 pi i 64 h / n), h < max(1, n / 128)
  const double2* lo;   // exp(-2 pi i l / n), l < 64
  __device__ __forceinline__ double2 operator()(int m) const { return cmul(hi[m >> 6], lo[m & 63]); }
};

// fill the two tables for size n (n a power of two, at most 8192); the caller synchronises
__device__ inline void lds_twiddles_fill(double2* hi, double2* lo, int n) {
  const int nhi = n >= 128 ? n / 128 : 1;
  for (int t = threadIdx.x; t < 64 + nhi; t += blockDim.x) {
    const int m = t < 64 ? t : 64 * (t - 64);
    double sv, cv;
    sincospi(-2.0 * static_cast<double>(m) / static_cast<double>(n), &sv, &cv);
    if (t < 64)
      lo[t] = double2{cv, sv};
    else
      hi[t - 64] = double2{cv, sv};
  }
}

// in-place forward FFT of s[0, n) held in bit-reversed order (natural order out): radix-2 stages of
// span len = 2, 4, ..., n, taken two at a time (spans len and 2 len in one pass over LDS, each thread
// on the 4 points that the two stages connect; the same butterflies and twiddles as one stage at a
// time), and a last single stage when log2 n is odd; tw(m) = exp(-2 pi i m / n). total (a multiple of
// n): s holds total / n sequences back to back, transformed together (every pass and barrier shared).
template <typename TW>
__device__ inline void fft_stages_tw(double2* s, int n, TW tw, int total) {
  int len = 2;
  for (; 2 * len <= n; len <<= 2) {
    const int h = len >> 1;
    const int step1 = n / len, step2 = step1 >> 1;
    for (int t = threadIdx.x; t < total / 4; t += blockDim.x) {
      const int k = t & (h - 1);
      const int base = (t - k) * 4 + k;
      const double2 w1 = tw(k * step1);
      const double2 a = s[base], c = s[base + len];
      const double2 b = cmul(s[base + h], w1), d = cmul(s[base + len + h], w1);
      const double2 a1 = cadd(a, b), b1 = csub(a, b);
      const double2 c1 = cmul(cadd(c, d), tw(k * step2)), d1 = cmul(csub(c, d), tw((k + h) * step2));
      s[base] = cadd(a1, c1);
      s[base + len] = csub(a1, c1);
      s[base + h] = cadd(b1, d1);
      s[base + len + h] = csub(b1, d1);
    }
    __syncthreads();
  }
  if (len <= n) {
    const int h = len >> 1;
    for (int t = threadIdx.x; t < total / 2; t += blockDim.x) {
      const int k = t & (h - 1);
      const int i0 = (t - k) * 2 + k;
      const double2 b = cmul(s[i0 + h], tw(k));
      const double2 a = s[i0];
      s[i0] = cadd(a, b);
      s[i0 + h] = csub(a, b);
    }
    __syncthreads();
  }
}

template <typename TW>
__device__ inline void fft_stages_tw(double2* s, int n, TW tw) {
  fft_stages_tw(s, n, tw, n);
}

// the same with the twiddles from a table in memory (n / 2 entries)
__device__ inline void fft_stages(double2* s, int n, const double2* __restrict__ tw) {
  fft_stages_tw(s, n, [tw](int m) { return tw[m]; }, n);
}

}  // namespace convreal
