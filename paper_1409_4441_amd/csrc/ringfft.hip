// Ring-FFT form of the real-space sum for ring pairs inside the equatorial belt (FP64).
//
//   y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) x_q
//
// Every belt ring has n = 4 Nside pixels at azimuths phi(a) = (pi / 2 Nside)(a + c / 2). For a belt
// output ring i and belt input ring j the pair's chord depends on a - b only:
//   d^2 = A_ij + B_ij sin^2(alpha),  alpha = (pi / n)(a - b + (c_i - c_j) / 2),
// so ring j's contribution to ring i is the circular convolution y_i[a] = sum_b k_ij[(a - b) mod n]
// x_j[b] with k_ij[m] = Ktilde(d) where d <= d_cut and 0 elsewhere: exactly the pairs and values of
// the per-pair sum. In Fourier space it is a product per frequency, so a belt output ring costs one
// multiply-add per frequency and neighbour ring plus one inverse FFT, whatever the number of pixels
// inside the cut: the cost grows linearly with theta_cut instead of quadratically (the scaling of the
// paper's real-space convolver, Eq. 7). The spectra of all k_ij are computed once per plan. Since
// Ktilde depends on sin^2(alpha) only, k_ij is the sampling at a - b + (c_i - c_j) / 2 of an even
// n-periodic function, so its spectrum is exp(i pi f (c_i - c_j) / n) times a real amplitude: the plan
// keeps the amplitude (8 bytes a frequency), and an output ring applies the phase once per frequency to
// the sum over its input rings of the other azimuth offset (c_i - c_j is 0 or 2 c_i - 1). Pairs
// that touch a polar cap (rings of different lengths) are summed per pair, each weight once for its
// 16 symmetric images on the FP64 matrix cores (cap_mfma64_kernel).
//
// FFTs: radix-2 decimation in time in LDS, FP64, n a power of two up to 8192 (128 KB of LDS); the
// input is placed in bit-reversed order and log2 n butterfly stages follow. Real sequences keep the
// n / 2 + 1 frequencies of their Hermitian spectra; every transform carries two real rings, one as the
// real and one as the imaginary part.
// Twiddles exp(-2 pi i m / n), m < n / 2, come from a table written by the host.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace {

constexpr int kFftMaxThreads = 1024;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}

__device__ __forceinline__ int bitrev(int v, int logn) {
  return static_cast<int>(__builtin_bitreverse32(static_cast<unsigned>(v)) >> (32 - logn));
}

// in-place forward FFT of s[0, n) held in bit-reversed order (natural order out)
__device__ void fft_stages(double2* s, int n, const double2* __restrict__ tw) {
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1;
    const int step = n / len;
    for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
      const int k = t & (half - 1);
      const int i0 = (t - k) * 2 + k;
      const int i1 = i0 + half;
      const double2 w = tw[k * step];
      const double2 b = cmul(s[i1], w);
      const double2 a = s[i0];
      s[i0] = double2{a.x + b.x, a.y + b.y};
      s[i1] = double2{a.x - b.x, a.y - b.y};
    }
    __syncthreads();
  }
}

struct FftArgs {
  const double* table;     // kernel table nodes (n_tab)
  const double2* tw;       // n / 2 twiddles
  const int* pj;           // per belt pair: input ring
  const int* pi;           // per belt pair: output ring
  const double* pA;        // per belt pair: chord constants
  const double* pB;
  const int* rc;           // per ring: azimuth offset numerator
  const long long* rstart; // per ring: first pixel
  const long long* boff;   // per north belt output ring (from belt_lo): first belt pair and first pair of an
                           // input ring with the other azimuth offset (2 entries a ring), + 1 entry
  double* K;               // per belt pair: nbins real amplitudes of the spectrum of k_ij
  double2* X;              // per belt ring (from belt_lo): nbins spectrum of x
  int n, logn, nbins;
  int belt_lo;
  int nbelt;              // belt rings (from belt_lo)
  int nnorth;             // belt output rings from belt_lo through the equator
  int nrings;
  int n_tab;
  double inv_h;
  double dcut2;
  double omega;
};

// Ktilde at chord^2 d2 <= d_cut^2: 4-point Lagrange on the uniform chord grid (segment floor(d/h)
// clamped to n_tab - 3, nodes k-1..k+2, ghost node T[-1] = T[1])
__device__ double ktilde(const double* __restrict__ tab, int n_tab, double d2, double inv_h) {
  return convreal::interp_f64(tab, n_tab, sqrt(d2), inv_h);
}

// Plan time, one workgroup per belt pair q: spectrum of k_q, times exp(-i pi f (c_i - c_j) / n) (real up
// to rounding; its real part is kept).
__global__ __launch_bounds__(kFftMaxThreads) void ring_fft_spectra_kernel(FftArgs a) {
  extern __shared__ double2 s_fft[];
  const long long q = blockIdx.x;
  const int i = a.pi[q], j = a.pj[q];
  const double A = a.pA[q], B = a.pB[q];
  const int dc = a.rc[i] - a.rc[j];
  for (int m = threadIdx.x; m < a.n; m += blockDim.x) {
    // sin(alpha) with alpha = pi (2m + c_i - c_j) / (2n): exact rational argument
    const double sa = sinpi(static_cast<double>(2 * m + dc) / static_cast<double>(2 * a.n));
    const double d2 = fma(B, sa * sa, A);
    const double k = d2 <= a.dcut2 ? ktilde(a.table, a.n_tab, d2, a.inv_h) : 0.0;
    s_fft[bitrev(m, a.logn)] = double2{k, 0.0};
  }
  __syncthreads();
  fft_stages(s_fft, a.n, a.tw);
  double* out = a.K + q * a.nbins;
  for (int f = threadIdx.x; f < a.nbins; f += blockDim.x) {
    double sp, cp;
    sincospi(static_cast<double>(f * dc) / static_cast<double>(a.n), &sp, &cp);
    out[f] = fma(s_fft[f].x, cp, s_fft[f].y * sp);
  }
}

// Apply, one workgroup per two belt rings (belt rings 2 b and 2 b + 1 from belt_lo; the last alone when
// their count is odd): one complex FFT of z = x_a + i x_b, split by the Hermitian symmetry of real
// sequences, X_a(f) = (Z(f) + conj Z(n - f)) / 2 and X_b(f) = (Z(f) - conj Z(n - f)) / (2 i).
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void ring_fft_forward_kernel(FftArgs a, const T* __restrict__ x) {
  extern __shared__ double2 s_fft[];
  const int ra = 2 * static_cast<int>(blockIdx.x);
  const bool two = ra + 1 < a.nbelt;
  const T* xa = x + a.rstart[a.belt_lo + ra];
  const T* xb = x + a.rstart[a.belt_lo + (two ? ra + 1 : ra)];
  for (int m = threadIdx.x; m < a.n; m += blockDim.x)
    s_fft[bitrev(m, a.logn)] = double2{static_cast<double>(xa[m]), two ? static_cast<double>(xb[m]) : 0.0};
  __syncthreads();
  fft_stages(s_fft, a.n, a.tw);
  double2* oa = a.X + static_cast<long long>(ra) * a.nbins;
  double2* ob = oa + a.nbins;
  for (int f = threadIdx.x; f < a.nbins; f += blockDim.x) {
    const double2 z = s_fft[f], w = s_fft[(a.n - f) & (a.n - 1)];
    oa[f] = double2{0.5 * (z.x + w.x), 0.5 * (z.y - w.y)};
    if (two) ob[f] = double2{0.5 * (z.y + w.y), 0.5 * (w.x - z.x)};
  }
}

constexpr int kMaxBins = 4;   // frequencies below n / 2 per thread (n / 2 <= 4 x 1024)

// Apply, one workgroup per two north belt output rings i and i + 2 (the same azimuth offset, so the
// same split of their input rings into offset groups; the blocks of i + 1 and i + 3 read nearly the
// same input spectra, and the launch keeps such blocks on one XCD) and their mirror rings m:
//   Y_i = sum_j K_ij X_j,  Y_m = sum_j K_ij X_mirror(j)
// per frequency (the mirror pair (m, mirror(j)) has the same chord constants and azimuth offsets, so
// the same kernel spectrum, read once for both). Each input spectrum is loaded once for both output
// rings. The group of input rings with the other azimuth offset is summed first and turned by the
// half-pixel phase. At f = n / 2 only the same-offset group contributes (the other group's amplitude
// vanishes there: its kernel is odd under the half-pixel reflection), summed by wave 0. The two real
// outputs of a ring and its mirror come from one complex inverse FFT of Z = Y_i + i Y_m:
// conj(Z) is transformed forward, y_i = Re / n and y_m = -Im / n. Belt rings are written (=);
// cap-touching pairs are added later.
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void ring_fft_inverse_kernel(FftArgs a, T* __restrict__ y) {
  extern __shared__ double2 s_fft[];
  const int nblk = 2 * ((a.nnorth + 3) / 4);
  const int b = convreal::xcd_remap(static_cast<int>(blockIdx.x), nblk);
  const int ib = 4 * (b >> 1) + (b & 1);
  if (ib >= a.nnorth) return;
  const int nr = ib + 2 < a.nnorth ? 2 : 1;
  const int half = a.n / 2;
  const int i0 = a.belt_lo + ib;
  // per output ring r and offset group g (0: same offset, 1: the other): pairs [qb, qe), input rings
  // jf, jf + 2, ..., jl
  long long qb[2][2];
  int jf[2][2], jl[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int row = 2 * (ib + 2 * r) + g;
      const long long q0 = r < nr ? a.boff[row] : 0, q1 = r < nr ? a.boff[row + 1] : 0;
      qb[r][g] = q0;
      jf[r][g] = q1 > q0 ? a.pj[q0] : 0x3fffffff;
      jl[r][g] = q1 > q0 ? a.pj[q0] + 2 * static_cast<int>(q1 - q0 - 1) : -0x3fffffff;
    }
  double2 acc[2][kMaxBins], accm[2][kMaxBins];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int u = 0; u < kMaxBins; ++u) {
      acc[r][u] = double2{0.0, 0.0};
      accm[r][u] = double2{0.0, 0.0};
    }
#pragma unroll
  for (int gg = 0; gg < 2; ++gg) {
    const int g = 1 - gg;
    const int ju = min(jf[0][g], jf[1][g]), jv = max(jl[0][g], jl[1][g]);
    for (int j = ju; j <= jv; j += 2) {
      const double2* xr = a.X + static_cast<long long>(j - a.belt_lo) * a.nbins;
      const double2* xm = a.X + static_cast<long long>(a.nrings - 1 - j - a.belt_lo) * a.nbins;
      double2 xv[kMaxBins], xw[kMaxBins];
#pragma unroll
      for (int u = 0; u < kMaxBins; ++u) {
        const int f = threadIdx.x + u * blockDim.x;
        if (f < half) {
          xv[u] = xr[f];
          xw[u] = xm[f];
        }
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (j < jf[r][g] || j > jl[r][g]) continue;
        const double* kr = a.K + (qb[r][g] + ((j - jf[r][g]) >> 1)) * a.nbins;
#pragma unroll
        for (int u = 0; u < kMaxBins; ++u) {
          const int f = threadIdx.x + u * blockDim.x;
          if (f >= half) continue;
          const double k = kr[f];
          acc[r][u].x = fma(k, xv[u].x, acc[r][u].x);
          acc[r][u].y = fma(k, xv[u].y, acc[r][u].y);
          accm[r][u].x = fma(k, xw[u].x, accm[r][u].x);
          accm[r][u].y = fma(k, xw[u].y, accm[r][u].y);
        }
      }
    }
    if (g == 1) {
      // the other group's phase exp(i pi f (c_i - c_j) / n), c_i - c_j = 2 c_i - 1 (belt offsets alternate)
      const int dc = 2 * a.rc[i0] - 1;
#pragma unroll
      for (int u = 0; u < kMaxBins; ++u) {
        const int f = threadIdx.x + u * blockDim.x;
        double sp, cp;
        sincospi(static_cast<double>(f * dc) / static_cast<double>(a.n), &sp, &cp);
        const double2 ph = double2{cp, sp};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          acc[r][u] = cmul(ph, acc[r][u]);
          accm[r][u] = cmul(ph, accm[r][u]);
        }
      }
    }
  }
  // f = n / 2 (real): wave 0, lanes striding over the same-offset pairs
  double yn[2] = {0.0, 0.0}, ynm[2] = {0.0, 0.0};
  if (threadIdx.x < 64) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const long long q1 = r < nr ? a.boff[2 * (ib + 2 * r) + 1] : 0;
      for (long long q = qb[r][0] + threadIdx.x; q < q1; q += 64) {
        const int j = a.pj[q];
        const double k = a.K[q * a.nbins + half];
        yn[r] = fma(k, a.X[static_cast<long long>(j - a.belt_lo) * a.nbins + half].x, yn[r]);
        ynm[r] = fma(k, a.X[static_cast<long long>(a.nrings - 1 - j - a.belt_lo) * a.nbins + half].x, ynm[r]);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        yn[r] += __shfl_xor(yn[r], o);
        ynm[r] += __shfl_xor(ynm[r], o);
      }
    }
  }
  const double scale = a.omega / static_cast<double>(a.n);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (r >= nr) break;
    const int i = i0 + 2 * r, mi = a.nrings - 1 - i;
    // conj(Z): Z(f) = Y(f) + i M(f) and Z(n - f) = conj Y(f) + i conj M(f); Y(0), M(0) real
#pragma unroll
    for (int u = 0; u < kMaxBins; ++u) {
      const int f = threadIdx.x + u * blockDim.x;
      if (f >= half) continue;
      const double2 Y = acc[r][u], M = accm[r][u];
      if (f == 0) {
        s_fft[0] = double2{Y.x, -M.x};
      } else {
        s_fft[bitrev(f, a.logn)] = double2{Y.x - M.y, -(Y.y + M.x)};
        s_fft[bitrev(a.n - f, a.logn)] = double2{Y.x + M.y, Y.y - M.x};
      }
    }
    if (threadIdx.x == 0) s_fft[bitrev(half, a.logn)] = double2{yn[r], -ynm[r]};
    __syncthreads();
    fft_stages(s_fft, a.n, a.tw);
    T* yr = y + a.rstart[i];
    T* ym = y + a.rstart[mi];
    for (int m = threadIdx.x; m < a.n; m += blockDim.x) {
      const double2 v = s_fft[m];
      yr[m] = static_cast<T>(scale * v.x);
      if (mi != i) ym[m] = static_cast<T>(-scale * v.y);
    }
    __syncthreads();
  }
}

FftArgs make_fft_args(const conv_real_plan* p) {
  FftArgs a;
  a.table = p->d_table;
  a.tw = p->d_fft_tw;
  a.pj = p->d_fft_pj;
  a.pi = p->d_fft_pi;
  a.pA = p->d_fft_pA;
  a.pB = p->d_fft_pB;
  a.rc = p->d_rc;
  a.rstart = p->d_rstart;
  a.boff = p->d_fft_boff;
  a.K = p->d_fft_K;
  a.X = p->d_fft_X;
  a.n = p->fft_n;
  a.logn = p->fft_logn;
  a.nbins = p->fft_n / 2 + 1;
  a.belt_lo = p->belt_lo;
  a.nbelt = p->belt_hi - p->belt_lo + 1;
  a.nnorth = (p->nrings - 1) / 2 - p->belt_lo + 1;
  a.nrings = p->nrings;
  a.n_tab = p->n_tab;
  a.inv_h = p->inv_h;
  a.dcut2 = p->dcut2;
  a.omega = p->omega;
  return a;
}

int fft_threads(int n) { return n / 2 < kFftMaxThreads ? (n / 2 < 64 ? 64 : n / 2) : kFftMaxThreads; }

}  // namespace

namespace convreal {

hipError_t ring_fft_spectra(const conv_real_plan* p) {
  if (p->fft_npairs == 0) return hipSuccess;
  const FftArgs a = make_fft_args(p);
  const size_t lds = sizeof(double2) * static_cast<size_t>(p->fft_n);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_fft_spectra_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ring_fft_spectra_kernel, dim3(static_cast<unsigned>(p->fft_npairs)), dim3(fft_threads(p->fft_n)),
                     lds, nullptr, a);
  return hipGetLastError();
}

template <typename T>
hipError_t ring_fft_apply_one(const conv_real_plan* p, const T* x, T* y, hipStream_t st) {
  const FftArgs a = make_fft_args(p);
  const size_t lds = sizeof(double2) * static_cast<size_t>(p->fft_n);
  const unsigned nbelt = static_cast<unsigned>(p->belt_hi - p->belt_lo + 1);
  const unsigned nnorth = static_cast<unsigned>((p->nrings - 1) / 2 - p->belt_lo + 1);   // through the equator
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_fft_forward_kernel<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ring_fft_inverse_kernel<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ring_fft_forward_kernel<T>, dim3((nbelt + 1) / 2), dim3(fft_threads(p->fft_n)), lds, st, a, x);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark(p, st, "ring_fft_forward_kernel", 0);
  hipLaunchKernelGGL(ring_fft_inverse_kernel<T>, dim3(2 * ((nnorth + 3) / 4)), dim3(fft_threads(p->fft_n)), lds, st,
                     a, y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark(p, st, "ring_fft_inverse_kernel", p->pairs - p->pairs_rest);
  return hipSuccess;
}

// Belt ring pairs of every map through the ring FFTs (one map at a time: the spectra of x are a
// per-plan workspace), then the cap-touching pairs over the symmetry group's fundamental domain,
// added to the belt rings.
hipError_t launch_ring_fft(const conv_real_plan* p, const void* x, void* y, int nmaps, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (p->belt_hi >= p->belt_lo) {
    for (int m = 0; m < nmaps && e == hipSuccess; ++m) {
      const size_t off = static_cast<size_t>(m) * static_cast<size_t>(p->npix);
      e = ring_fft_apply_one(p, static_cast<const double*>(x) + off, static_cast<double*>(y) + off, st);
    }
    if (e != hipSuccess) return e;
  }
  return launch_cap_mfma64(p, static_cast<const double*>(x), static_cast<double*>(y), nmaps, st);
}

}  // namespace convreal
