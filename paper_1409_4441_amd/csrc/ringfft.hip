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
// input is placed in bit-reversed order and log2 n butterfly stages follow, two per pass over LDS
// where they pair up. Real sequences keep the
// n / 2 + 1 frequencies of their Hermitian spectra; every transform carries two real rings, one as the
// real and one as the imaginary part.
// Twiddles exp(-2 pi i m / n), m < n / 2, come from a table written by the host.
#include <hip/hip_runtime.h>

#include "common.h"
#include "fft.h"
#include "internal.h"

namespace {

constexpr int kFftMaxThreads = 1024;

using convreal::bitrev;
using convreal::cadd;
using convreal::cmul;
using convreal::csub;
using convreal::fft_stages;

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
  double2* Y;              // per belt ring (from belt_lo): nbins spectrum of its belt-pair output
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
  __shared__ double2 s_twh[64], s_twl[64];
  convreal::lds_twiddles_fill(s_twh, s_twl, a.n);
  const int ra = 2 * static_cast<int>(blockIdx.x);
  const bool two = ra + 1 < a.nbelt;
  const T* xa = x + a.rstart[a.belt_lo + ra];
  const T* xb = x + a.rstart[a.belt_lo + (two ? ra + 1 : ra)];
  for (int m = threadIdx.x; m < a.n; m += blockDim.x)
    s_fft[bitrev(m, a.logn)] = double2{static_cast<double>(xa[m]), two ? static_cast<double>(xb[m]) : 0.0};
  __syncthreads();
  convreal::fft_stages_tw(s_fft, a.n, convreal::LdsTwiddles{s_twh, s_twl});
  double2* oa = a.X + static_cast<long long>(ra) * a.nbins;
  double2* ob = oa + a.nbins;
  for (int f = threadIdx.x; f < a.nbins; f += blockDim.x) {
    const double2 z = s_fft[f], w = s_fft[(a.n - f) & (a.n - 1)];
    oa[f] = double2{0.5 * (z.x + w.x), 0.5 * (z.y - w.y)};
    if (two) ob[f] = double2{0.5 * (z.y + w.y), 0.5 * (w.x - z.x)};
  }
}

constexpr int kAccThreads = 256;   // frequencies per workgroup (at most)
constexpr long long kAccFill = 1 << 18;   // threads that keep every CU busy (256 CUs x 16 waves x 64)

// Apply, per frequency: Y_i = sum_j K_ij X_j and Y_m = sum_j K_ij X_mirror(j) for the north belt output
// rings i and their mirror rings m (the mirror pair (m, mirror(j)) has the same chord constants and
// azimuth offsets, so the same kernel spectrum, read once for both). One workgroup per run of
// frequencies (one a thread) and group of kAccRings north rings i0, i0 + 2, ... (the same azimuth
// offset, so the same split of the input rings into offset groups): each input spectrum value is
// loaded once for all of them. The input rings with the other azimuth offset are summed first and
// turned by the half-pixel phase. Work items are numbered ring group fastest, so that consecutive ones
// share input spectra, and each XCD takes a contiguous run. kAccRings is the largest of 8, 4, 2, 1 that
// still gives the launch kAccFill threads.
template <int kAccRings>
__global__ __launch_bounds__(kAccThreads) void ring_fft_accumulate_kernel(FftArgs a, int nchunks, int chunk_len,
                                                                          int ngroups) {
  const int item = convreal::xcd_remap(static_cast<int>(blockIdx.x), nchunks * ngroups);
  const int grp = item % ngroups, chunk = item / ngroups;
  const int ib0 = 2 * kAccRings * (grp >> 1) + (grp & 1);
  if (ib0 >= a.nnorth) return;
  const int nr = min(kAccRings, (a.nnorth - ib0 + 1) / 2);   // rings ib0 + 2 r below nnorth
  const int f = chunk * chunk_len + static_cast<int>(threadIdx.x);
  const bool live = static_cast<int>(threadIdx.x) < chunk_len && f < a.nbins;
  const int fl = live ? f : 0;   // idle lanes read frequency 0 and store nothing
  double2 acc[kAccRings], accm[kAccRings];
#pragma unroll
  for (int r = 0; r < kAccRings; ++r) {
    acc[r] = double2{0.0, 0.0};
    accm[r] = double2{0.0, 0.0};
  }
#pragma unroll
  for (int gg = 0; gg < 2; ++gg) {
    const int g = 1 - gg;   // 1: the other azimuth offset, 0: the same
    // per ring: pairs [qb, qb + cnt) with input rings jf, jf + 2, ...; their union
    long long qb[kAccRings];
    int jf[kAccRings], jl[kAccRings];
    int ju = 0x3fffffff, jv = -0x3fffffff;
#pragma unroll
    for (int r = 0; r < kAccRings; ++r) {
      const int row = 2 * (ib0 + 2 * r) + g;
      const long long q0 = r < nr ? a.boff[row] : 0, q1 = r < nr ? a.boff[row + 1] : 0;
      qb[r] = q0;
      jf[r] = q1 > q0 ? a.pj[q0] : 0x3fffffff;
      jl[r] = q1 > q0 ? a.pj[q0] + 2 * static_cast<int>(q1 - q0 - 1) : -0x3fffffff;
      ju = min(ju, jf[r]);
      jv = max(jv, jl[r]);
    }
    for (int j = ju; j <= jv; j += 2) {
      const double2 xv = a.X[static_cast<long long>(j - a.belt_lo) * a.nbins + fl];
      const double2 xw = a.X[static_cast<long long>(a.nrings - 1 - j - a.belt_lo) * a.nbins + fl];
      // every ring's amplitude is loaded before any is used (a ring outside its range reads pair 0,
      // which always exists, and takes 0), so that the loads overlap
      double kv[kAccRings];
#pragma unroll
      for (int r = 0; r < kAccRings; ++r) {
        const bool in = j >= jf[r] && j <= jl[r];
        kv[r] = a.K[(in ? qb[r] + ((j - jf[r]) >> 1) : 0) * a.nbins + fl];
        kv[r] = in ? kv[r] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < kAccRings; ++r) {
        const double k = kv[r];
        acc[r].x = fma(k, xv.x, acc[r].x);
        acc[r].y = fma(k, xv.y, acc[r].y);
        accm[r].x = fma(k, xw.x, accm[r].x);
        accm[r].y = fma(k, xw.y, accm[r].y);
      }
    }
    if (g == 1) {
      // the other group's phase exp(i pi f (c_i - c_j) / n), c_i - c_j = 2 c_i - 1 (belt offsets alternate)
      const int dc = 2 * a.rc[a.belt_lo + ib0] - 1;
      double sp, cp;
      sincospi(static_cast<double>(fl * dc) / static_cast<double>(a.n), &sp, &cp);
      const double2 ph = double2{cp, sp};
#pragma unroll
      for (int r = 0; r < kAccRings; ++r) {
        acc[r] = cmul(ph, acc[r]);
        accm[r] = cmul(ph, accm[r]);
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int r = 0; r < kAccRings; ++r) {
    if (r >= nr) break;
    const int i = a.belt_lo + ib0 + 2 * r, mi = a.nrings - 1 - i;
    a.Y[static_cast<long long>(i - a.belt_lo) * a.nbins + f] = acc[r];
    if (mi != i) a.Y[static_cast<long long>(mi - a.belt_lo) * a.nbins + f] = accm[r];
  }
}

// Apply, one workgroup per north belt output ring i and its mirror ring m (the equator ring alone): both
// real outputs from one complex inverse FFT of Z = Y_i + i Y_m. conj(Z) is transformed forward, and
// y_i = Re / n, y_m = -Im / n, with Z(f) = Y(f) + i M(f) and Z(n - f) = conj Y(f) + i conj M(f); at
// f = 0 and n / 2 the spectra of real rings are real (the other offset group's amplitude vanishes at
// n / 2: its kernel is odd under the half-pixel reflection there), so only their real parts enter. Belt
// rings are written (=); cap-touching pairs are added later.
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void ring_fft_inverse_kernel(FftArgs a, T* __restrict__ y) {
  extern __shared__ double2 s_fft[];
  __shared__ double2 s_twh[64], s_twl[64];
  convreal::lds_twiddles_fill(s_twh, s_twl, a.n);
  const int ib = static_cast<int>(blockIdx.x);
  const int i = a.belt_lo + ib, mi = a.nrings - 1 - i;
  const int half = a.n / 2;
  const double2* Yi = a.Y + static_cast<long long>(ib) * a.nbins;
  const double2* Ym = a.Y + static_cast<long long>(mi - a.belt_lo) * a.nbins;
  for (int f = threadIdx.x; f <= half; f += blockDim.x) {
    const double2 Y = Yi[f], M = mi != i ? Ym[f] : double2{0.0, 0.0};
    if (f == 0 || f == half) {
      s_fft[bitrev(f, a.logn)] = double2{Y.x, -M.x};
    } else {
      s_fft[bitrev(f, a.logn)] = double2{Y.x - M.y, -(Y.y + M.x)};
      s_fft[bitrev(a.n - f, a.logn)] = double2{Y.x + M.y, Y.y - M.x};
    }
  }
  __syncthreads();
  convreal::fft_stages_tw(s_fft, a.n, convreal::LdsTwiddles{s_twh, s_twl});
  const double scale = a.omega / static_cast<double>(a.n);
  T* yr = y + a.rstart[i];
  T* ym = y + a.rstart[mi];
  for (int m = threadIdx.x; m < a.n; m += blockDim.x) {
    const double2 v = s_fft[m];
    yr[m] = static_cast<T>(scale * v.x);
    if (mi != i) ym[m] = static_cast<T>(-scale * v.y);
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
  a.Y = p->d_fft_Y;
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
  const size_t lds = sizeof(double2) * static_cast<size_t>(p->fft_n);
  // the LDS limits of every transform kernel, set here (plan set-up) so that applies make no
  // attribute calls (they may run under stream capture); the limit is per kernel, not per plan, so
  // it is the largest any plan needs (8192-point rings at Nside 2048)
  const int lds_max = static_cast<int>(sizeof(double2) * 8192);
  const void* fns[] = {reinterpret_cast<const void*>(&ring_fft_spectra_kernel),
                       reinterpret_cast<const void*>(&ring_fft_forward_kernel<double>),
                       reinterpret_cast<const void*>(&ring_fft_forward_kernel<float>),
                       reinterpret_cast<const void*>(&ring_fft_inverse_kernel<double>),
                       reinterpret_cast<const void*>(&ring_fft_inverse_kernel<float>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (e != hipSuccess) return e;
  }
  if (p->fft_npairs == 0) return hipSuccess;
  const FftArgs a = make_fft_args(p);
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
  hipError_t e;
  hipLaunchKernelGGL(ring_fft_forward_kernel<T>, dim3((nbelt + 1) / 2), dim3(fft_threads(p->fft_n)), lds, st, a, x);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark(p, st, "ring_fft_forward_kernel", 0);
  const int nchunks = (a.nbins + kAccThreads - 1) / kAccThreads;
  const int chunk_len = (a.nbins + nchunks - 1) / nchunks;
  auto groups = [&](int rings) { return 2 * ((a.nnorth + 2 * rings - 1) / (2 * rings)); };
  int rings = 8;
  while (rings > 1 && static_cast<long long>(a.nbins) * groups(rings) < kAccFill) rings /= 2;
  const int ngroups = groups(rings);
  const dim3 grid(static_cast<unsigned>(nchunks * ngroups));
  switch (rings) {
    case 8:
      hipLaunchKernelGGL(ring_fft_accumulate_kernel<8>, grid, dim3(kAccThreads), 0, st, a, nchunks, chunk_len, ngroups);
      break;
    case 4:
      hipLaunchKernelGGL(ring_fft_accumulate_kernel<4>, grid, dim3(kAccThreads), 0, st, a, nchunks, chunk_len, ngroups);
      break;
    case 2:
      hipLaunchKernelGGL(ring_fft_accumulate_kernel<2>, grid, dim3(kAccThreads), 0, st, a, nchunks, chunk_len, ngroups);
      break;
    default:
      hipLaunchKernelGGL(ring_fft_accumulate_kernel<1>, grid, dim3(kAccThreads), 0, st, a, nchunks, chunk_len, ngroups);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark(p, st, "ring_fft_accumulate_kernel", p->pairs - p->pairs_rest);
  hipLaunchKernelGGL(ring_fft_inverse_kernel<T>, dim3(nnorth), dim3(fft_threads(p->fft_n)), lds, st, a, y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark(p, st, "ring_fft_inverse_kernel", 0);
  return hipSuccess;
}

hipError_t ring_fft_belt_f32(const conv_real_plan* p, const float* x, float* y, hipStream_t st) {
  return ring_fft_apply_one(p, x, y, st);
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
