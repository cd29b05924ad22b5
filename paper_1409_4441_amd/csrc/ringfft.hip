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
// n / 2 + 1 frequencies of their Hermitian spectra; the inverse rebuilds the full spectrum.
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

// Apply, one workgroup per belt ring j: spectrum of x_j.
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void ring_fft_forward_kernel(FftArgs a, const T* __restrict__ x) {
  extern __shared__ double2 s_fft[];
  const int r = a.belt_lo + static_cast<int>(blockIdx.x);
  const T* xr = x + a.rstart[r];
  for (int m = threadIdx.x; m < a.n; m += blockDim.x)
    s_fft[bitrev(m, a.logn)] = double2{static_cast<double>(xr[m]), 0.0};
  __syncthreads();
  fft_stages(s_fft, a.n, a.tw);
  double2* out = a.X + static_cast<long long>(blockIdx.x) * a.nbins;
  for (int f = threadIdx.x; f < a.nbins; f += blockDim.x) out[f] = s_fft[f];
}

// conj(Y) at f into the transform's input, and at n - f the conjugate of that (Hermitian spectrum of a
// real sequence)
__device__ __forceinline__ void put_conj(double2* s, double2 v, int f, int n, int logn) {
  s[bitrev(f, logn)] = double2{v.x, -v.y};
  if (f > 0 && f < n - f) s[bitrev(n - f, logn)] = v;
}

// y = Omega x the inverse FFT of the spectrum in s (ifft(Y) = conj(fft(conj(Y))) / n, whose real part
// is Re(fft(conj(Y))) / n)
template <typename T>
__device__ __forceinline__ void inverse_out(double2* s, const FftArgs& a, T* __restrict__ yr) {
  __syncthreads();
  fft_stages(s, a.n, a.tw);
  const double scale = a.omega / static_cast<double>(a.n);
  for (int m = threadIdx.x; m < a.n; m += blockDim.x) yr[m] = static_cast<T>(scale * s[m].x);
  __syncthreads();
}

constexpr int kMaxBinsPerThread = 5;   // (8192 / 2 + 1) frequencies over 1024 threads

// Apply, one workgroup per north belt output ring i and its mirror ring m: Y_i = sum_j K_ij X_j and
// Y_m = sum_j K_ij X_mirror(j) per frequency (the mirror pair (m, mirror(j)) has the same chord
// constants and azimuth offsets, so the same kernel spectrum, read once for both), the half-pixel phase
// applied once to the sum over input rings of the other azimuth offset, then the inverse FFTs. Belt
// rings are written (=); cap-touching pairs are added later.
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void ring_fft_inverse_kernel(FftArgs a, T* __restrict__ y) {
  extern __shared__ double2 s_fft[];
  const int ib = static_cast<int>(blockIdx.x);
  const int i = a.belt_lo + ib;
  const int mi = a.nrings - 1 - i;
  const bool pair = mi != i;
  const long long q0 = a.boff[2 * ib], qm = a.boff[2 * ib + 1], q1 = a.boff[2 * ib + 2];
  const int dc = qm < q1 ? a.rc[i] - a.rc[a.pj[qm]] : 0;
  double2 ym[kMaxBinsPerThread];
#pragma unroll
  for (int u = 0; u < kMaxBinsPerThread; ++u) {
    const int f = threadIdx.x + u * blockDim.x;
    if (f >= a.nbins) break;
    double2 acc[2], accm[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      acc[g] = double2{0.0, 0.0};
      accm[g] = double2{0.0, 0.0};
      const long long qb = g == 0 ? q0 : qm, qe = g == 0 ? qm : q1;
      for (long long q = qb; q < qe; ++q) {
        const double k = a.K[q * a.nbins + f];
        const int j = a.pj[q];
        const double2 xv = a.X[static_cast<long long>(j - a.belt_lo) * a.nbins + f];
        acc[g].x = fma(k, xv.x, acc[g].x);
        acc[g].y = fma(k, xv.y, acc[g].y);
        if (pair) {
          const double2 xw = a.X[static_cast<long long>(a.nrings - 1 - j - a.belt_lo) * a.nbins + f];
          accm[g].x = fma(k, xw.x, accm[g].x);
          accm[g].y = fma(k, xw.y, accm[g].y);
        }
      }
    }
    double sp, cp;
    sincospi(static_cast<double>(f * dc) / static_cast<double>(a.n), &sp, &cp);
    const double2 ph = double2{cp, sp};
    const double2 t = cmul(ph, acc[1]), tm = cmul(ph, accm[1]);
    put_conj(s_fft, double2{acc[0].x + t.x, acc[0].y + t.y}, f, a.n, a.logn);
    ym[u] = double2{accm[0].x + tm.x, accm[0].y + tm.y};
  }
  inverse_out(s_fft, a, y + a.rstart[i]);
  if (!pair) return;
#pragma unroll
  for (int u = 0; u < kMaxBinsPerThread; ++u) {
    const int f = threadIdx.x + u * blockDim.x;
    if (f >= a.nbins) break;
    put_conj(s_fft, ym[u], f, a.n, a.logn);
  }
  inverse_out(s_fft, a, y + a.rstart[mi]);
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
  hipLaunchKernelGGL(ring_fft_forward_kernel<T>, dim3(nbelt), dim3(fft_threads(p->fft_n)), lds, st, a, x);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark(p, st, "ring_fft_forward_kernel", 0);
  hipLaunchKernelGGL(ring_fft_inverse_kernel<T>, dim3(nnorth), dim3(fft_threads(p->fft_n)), lds, st, a, y);
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
