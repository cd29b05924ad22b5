// Spherical-harmonic transforms on the ring grid (FP64) and the hybrid apply: the harmonic half of
// the kernel split (Eq. 1: K~_l = K^_l + P_l,theta K^_theta; Fig. 1: both halves run at once and their
// maps are summed).
//
//   analysis   a_lm = Omega sum_rings lambda_lm(z_r) G_m(r),   G_m(r) = sum_{a in ring r} x_a e^{-i m phi_a}
//   synthesis  y_a  = Re sum_m w_m F_m(r) e^{i m phi_a},       F_m(r) = sum_l b_lm lambda_lm(z_r)
//              (w_0 = 1, w_m = 2 for m > 0: the m < 0 half of a real map)
//
// Ring sums. Ring r has n = 4k pixels at phi_a = pi (2a + c) / n, so G_m(r) = e^{-i m pi c / n} X[m mod n]
// with X the n-point DFT of the ring. With a = q k + a' (q = 0..3 quarter rings), e^{-2 pi i j a / n} =
// (-i)^{jq} e^{-2 pi i j a' / n}, so X[j] = sum_{a'} c_{j mod 4}[a'] z_j^{a'} (z_j = e^{-2 pi i j / n})
// with four folded sequences (x0+x1+x2+x3, x0-x1+x2-x3, (x0-x2) -+ i (x1-x3)): k terms per frequency,
// summed by Horner's rule with one complex multiply-add a term; a wave holds one residue j mod 4, so
// every lane reads the same folded value (an LDS broadcast). Synthesis runs the same fold backwards:
// B[j] = sum_{m = j mod n} w_m F_m e^{i m pi c / n}, and for each a' the four residue classes of j are
// Horner sums in e^{2 pi i a' / k}, combined with i^{(j mod 4) q} into the four pixels q k + a'.
// Only the frequencies below min(n, L + 1) are formed. On a grid whose Nside is a power of two the
// belt rings (n = 4 Nside, a power of two) take a radix-2 FFT in LDS instead (n log n work against
// n min(n, L + 1) / 4). The other rings with k >= kChirpMin (the polar-cap rings, and the belt rings of
// other grids) take each folded class's k-point DFT as a chirp-z convolution through the same radix-2
// FFTs (below); the smallest rings keep the folded Horner sums. Neighbouring rings run on one XCD
// (their G / F entries of one order share cache lines).
//
// Legendre sums. lambda_lm by the recurrence in l at fixed m,
//   lambda_mm = (-1)^m sqrt((2m+1)/(4 pi) prod_{k<=m} (2k-1)/(2k)) sin^m theta,
//   lambda_lm = a_lm (z lambda_{l-1,m} - b_lm lambda_{l-2,m}),
//   a_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)), b_lm = sqrt(((l-1)^2 - m^2) / (4 (l-1)^2 - 1)),
// carried within each group of kFlush values of l as mu_l = lambda_l / C_l (C_l the product of the
// a's since the group started), which turns a step into mu_l = z mu_{l-1} - e_l mu_{l-2}: one multiply
// and one multiply-add, with (e_l, C_l) from a table written at set-up and staged in LDS; C_l is folded
// into the output coefficients (analysis) or the staged a_lm (synthesis), and the last two values of a
// group go back to lambda before the next. lambda_mm below about e^-600 starts scaled by 2^(600 e)
// with the exponent e kept beside it (C_l <= 2^85 then keeps mu above the FP64 normal range); after
// every group a scaled value above 2^400 is brought down by 2^-600, and a ring contributes once its
// exponent is 0 (scaled values are true values times 2^(600 e) <= 2^-144: dropped). The mirror
// ring (z -> -z) has lambda_lm(-z) = (-1)^(l+m) lambda_lm(z), so one recurrence serves a ring pair:
// analysis sums G(north) +- G(south), synthesis splits into the even and odd l + m parts.
// A workgroup of 512 threads (synthesis; 256 in the analysis) takes one order m and up to 512 R
// (256 R) north rings (R per thread); analysis
// reduces over rings after every group through LDS (each thread first adds its R rings), synthesis
// needs no reduction. Per order, the leading chunks of 256 polar rings whose scaled values never reach
// the sums before L (they would add exact zeros) are left out; a set-up kernel counts them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/convsht.h"
#include "common.h"
#include "fft.h"
#include "internal.h"

namespace {

constexpr int kLegThreads = 512;   // Legendre synthesis: 8 waves
constexpr int kLegThreadsA = 256;  // Legendre analysis: 4 waves (two workgroups per CU overlap their reductions' barriers)
constexpr int kFlush = 16;         // l values per group: recurrence scaling, rescale checks, analysis reductions
constexpr int kFlushS = 8;         // l values per unrolled step group of the synthesis (two per kFlush group)
static_assert(kFlush % kFlushS == 0 && kFlush / kFlushS == 2, "the synthesis converts back every second unit");
constexpr int kLegChunk = kLegThreads;   // values of l whose coefficients (and alm) are staged in LDS at a time
static_assert(kLegChunk % kFlush == 0, "groups of l values never straddle a chunk");
static_assert(kFlush * (kLegThreadsA / kFlush) == kLegThreadsA && kLegThreadsA / kFlush <= 64,
              "the analysis reduces each group's values of l with kLegThreadsA / kFlush lanes of one wave each");
constexpr int kDftThreads = 256;   // ring sum kernels: 4 waves, one per residue class mod 4
constexpr int kDftChains = 4;      // frequencies per lane at a time in the analysis ring sums
constexpr int kFftThreads = 512;   // belt ring FFT kernels and chirp-z ring sums
constexpr int kChirpMin = 16;      // rings with k = n / 4 at least this take the chirp-z ring sums
constexpr double kInvScale = 0x1p-600;
constexpr double kRescaleAbove = 0x1p400;
constexpr double kLogScale = 600.0 * 0.69314718055994530942;
constexpr double kLogFloor = -600.0;
// North rings are grouped in chunks of kDeadChunk (ring 0 the northernmost) for skipping, per order m,
// the polar rings whose scaled Legendre values never come back into the sums before l = L
constexpr int kDeadChunk = 256;
static_assert(kLegThreadsA == kDeadChunk && kLegThreads == 2 * kDeadChunk,
              "a thread's ring ranges are one chunk wide (analysis) or two (synthesis)");
static_assert(kDftThreads == 256, "four waves: one per residue class mod 4");

// Blocks are dealt round-robin to the 8 XCDs. Within each window of 8 g consecutive blocks (first
// block w), the g blocks that XCD x receives take items w + g x .. w + g x + g - 1, so that
// neighbouring rings, whose G / F entries of one order share cache lines, run on one XCD and meet in
// its L2. A trailing partial window keeps the identity; the map is a bijection on [0, n).
__device__ __forceinline__ int xcd_group(int b, int n, int g) {
  const int w = b - b % (8 * g);
  if (w + 8 * g > n) return b;
  return w + (b & 7) * g + (b >> 3) % g;
}

struct ShtRing {
  double z;          // cos theta
  double s;          // sin theta
  long long start;   // first pixel
  int n;             // pixels (a multiple of 4)
  int c;             // azimuth offset numerator: phi_a = pi (2a + c) / n
};

struct LegArgs {
  const ShtRing* rings;
  const double2* coef;     // per (l, m), m-major: (a_lm, b_lm); unused at l = m
  const double* logpre;    // per m: log of the l = m normalisation
  double2* G;              // [m][ring]: ring sums (analysis input) or F_m (synthesis output)
  double2* alm;            // m-major alm (analysis output, synthesis input)
  const int* dead;         // per m: leading chunks of kDeadChunk north rings that add nothing
  int L;
  int nrings;
  int nnorth;              // rings 0 .. nnorth - 1 are the north half, the last one the equator
  double omega;
};

__device__ __forceinline__ long long alm_base(int L, int m) {
  return static_cast<long long>(m) * (2 * L + 3 - m) / 2;
}

// ---------------------------------------------------------------------------- ring sums (analysis)
// rings [skip0, skip0 + nskip) are left to the FFT kernels
template <typename T>
__global__ __launch_bounds__(kDftThreads) void sht_ring_dft_kernel(const T* __restrict__ x,
                                                                   const ShtRing* __restrict__ rings,
                                                                   const int* __restrict__ list, int nrings, int L,
                                                                   double2* __restrict__ G) {
  extern __shared__ double s_fold[];   // s0[k], s2[k], then (d, e) pairs [k]
  const int r = list[blockIdx.x];
  const ShtRing R = convreal::ldu_record(rings[r]);
  const int n = R.n, k = n >> 2;
  double* s0 = s_fold;
  double* s2 = s_fold + k;
  double2* de = reinterpret_cast<double2*>(s_fold + 2 * k);
  const T* xr = x + R.start;
  for (int a = threadIdx.x; a < k; a += blockDim.x) {
    const double x0 = static_cast<double>(xr[a]), x1 = static_cast<double>(xr[a + k]);
    const double x2 = static_cast<double>(xr[a + 2 * k]), x3 = static_cast<double>(xr[a + 3 * k]);
    s0[a] = (x0 + x2) + (x1 + x3);
    s2[a] = (x0 + x2) - (x1 + x3);
    de[a] = double2{x0 - x2, x1 - x3};
  }
  __syncthreads();
  const int nk = n < L + 1 ? n : L + 1;   // < 4 kChirpMin: the list holds rings with k < kChirpMin only
  __shared__ double2 s_x[4 * kChirpMin];
  const int kappa = threadIdx.x >> 6;          // the wave's residue class j mod 4
  const int lane = threadIdx.x & 63;
  // kDftChains frequencies per lane at a time (j = 4 jq + kappa, jq = jq0 + 64 t): independent Horner
  // chains that share each folded value, so that their latencies overlap
  for (int jq0 = lane; 4 * jq0 + kappa < nk; jq0 += 64 * kDftChains) {
    double zs[kDftChains], zc[kDftChains], ar[kDftChains], ai[kDftChains];
#pragma unroll
    for (int t = 0; t < kDftChains; ++t) {
      const int j = 4 * (jq0 + 64 * t) + kappa;
      sincospi(-2.0 * static_cast<double>(j < nk ? j : 4 * jq0 + kappa) / static_cast<double>(n), &zs[t], &zc[t]);
      ar[t] = 0.0;
      ai[t] = 0.0;
    }
    if (kappa == 0 || kappa == 2) {
      const double* cs = kappa == 0 ? s0 : s2;
      for (int a = k - 1; a >= 0; --a) {
        const double c = cs[a];
#pragma unroll
        for (int t = 0; t < kDftChains; ++t) {
          const double nr = fma(ar[t], zc[t], fma(-ai[t], zs[t], c));
          ai[t] = fma(ar[t], zs[t], ai[t] * zc[t]);
          ar[t] = nr;
        }
      }
    } else {
      // kappa 1: (x0 - x2) - i (x1 - x3); kappa 3: (x0 - x2) + i (x1 - x3)
      const double sg = kappa == 1 ? -1.0 : 1.0;
      for (int a = k - 1; a >= 0; --a) {
        const double2 c = de[a];
#pragma unroll
        for (int t = 0; t < kDftChains; ++t) {
          const double nr = fma(ar[t], zc[t], fma(-ai[t], zs[t], c.x));
          ai[t] = fma(ar[t], zs[t], fma(ai[t], zc[t], sg * c.y));
          ar[t] = nr;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kDftChains; ++t) {
      const int j = 4 * (jq0 + 64 * t) + kappa;
      if (j < nk) s_x[j] = double2{ar[t], ai[t]};
    }
  }
  __syncthreads();
  // G_m = e^{-i m pi c / n} X[m mod n] for every m up to L (a small ring folds many m onto each j:
  // the whole workgroup shares them out)
  for (int m = threadIdx.x; m <= L; m += blockDim.x) {
    const double2 X = s_x[m % n];
    const long long num = (static_cast<long long>(m) * R.c) % (2LL * n);
    double ps, pc;
    sincospi(-static_cast<double>(num) / static_cast<double>(n), &ps, &pc);
    G[static_cast<size_t>(m) * nrings + r] = double2{X.x * pc - X.y * ps, X.x * ps + X.y * pc};
  }
}

// threads per frequency when the folded sums of B (each over every m = j mod n up to L) are shared out:
// the largest power of two up to 64 with 2 nsub nj <= blockDim
__device__ __forceinline__ int fold_split(int nj) {
  int nsub = 1;
  while (nsub < 64 && 2 * nsub * nj <= static_cast<int>(blockDim.x)) nsub *= 2;
  return nsub;
}

// B[j] = sum_{m = j mod n, m <= L} w_m F_m e^{i m pi c / n} for one j, its terms split over the nsub
// lanes of the calling group (aligned, consecutive lanes; sub = lane within the group); every lane of
// the group gets the sum (fixed-order butterfly)
__device__ __forceinline__ double2 fold_sum(const double2* __restrict__ F, int nrings, int r, int L, int n, int c,
                                            int j, int sub, int nsub) {
  double br = 0.0, bi = 0.0;
  for (int m = j + sub * n; m <= L; m += nsub * n) {
    const double2 f = F[static_cast<size_t>(m) * nrings + r];
    const long long num = (static_cast<long long>(m) * c) % (2LL * n);
    double ps, pc;
    sincospi(static_cast<double>(num) / static_cast<double>(n), &ps, &pc);
    const double w = m == 0 ? 1.0 : 2.0;
    br += w * (f.x * pc - f.y * ps);
    bi += w * (f.x * ps + f.y * pc);
  }
  for (int o = 1; o < nsub; o <<= 1) {
    br += __shfl_xor(br, o);
    bi += __shfl_xor(bi, o);
  }
  return double2{br, bi};
}

// ---------------------------------------------------------------------------- ring sums (synthesis)
template <typename T, bool ACC>
__global__ __launch_bounds__(kDftThreads) void sht_ring_idft_kernel(const double2* __restrict__ F,
                                                                    const ShtRing* __restrict__ rings,
                                                                    const int* __restrict__ list, int nrings, int L,
                                                                    T* __restrict__ y) {
  extern __shared__ double2 s_b[];     // residue class c at s_b[c * nq + j / 4]
  const int r = list[blockIdx.x];
  const ShtRing R = convreal::ldu_record(rings[r]);
  const int n = R.n, k = n >> 2;
  const int nk = n < L + 1 ? n : L + 1;
  const int nq = (nk + 3) >> 2;
  for (int t = threadIdx.x; t < 4 * nq; t += blockDim.x) s_b[t] = double2{0.0, 0.0};
  __syncthreads();
  {
    const int nsub = fold_split(nk), sub = static_cast<int>(threadIdx.x) & (nsub - 1);
    for (int j = static_cast<int>(threadIdx.x) / nsub; j < nk; j += static_cast<int>(blockDim.x) / nsub) {
      const double2 b = fold_sum(F, nrings, r, L, n, R.c, j, sub, nsub);
      if (sub == 0) s_b[(j & 3) * nq + (j >> 2)] = b;
    }
  }
  __syncthreads();
  T* yr = y + R.start;
  for (int ap = threadIdx.x; ap < k; ap += blockDim.x) {
    double zs, zc;
    sincospi(2.0 * static_cast<double>(ap) / static_cast<double>(k), &zs, &zc);
    // the four residue classes' Horner sums in one loop (independent chains); a class with fewer
    // than nq terms reads zeros first (s_b is cleared up to nq per class), which leaves its chain at
    // exactly zero until its own terms start
    double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
    for (int jq = nq - 1; jq >= 0; --jq) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double2 v = s_b[c * nq + jq];
        const double nr = fma(ar[c], zc, fma(-ai[c], zs, v.x));
        ai[c] = fma(ar[c], zs, fma(ai[c], zc, v.y));
        ar[c] = nr;
      }
    }
    double ur[4], ui[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // times e^{2 pi i c a' / n}
      double ps, pc;
      sincospi(2.0 * static_cast<double>(c * ap) / static_cast<double>(n), &ps, &pc);
      ur[c] = ar[c] * pc - ai[c] * ps;
      ui[c] = ar[c] * ps + ai[c] * pc;
    }
    // pixel q k + a': Re sum_c i^{c q} U_c
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int p = (c * q) & 3;
        v += p == 0 ? ur[c] : (p == 1 ? -ui[c] : (p == 2 ? -ur[c] : ui[c]));
      }
      T* dst = yr + q * k + ap;
      if (ACC)
        *dst = static_cast<T>(static_cast<double>(*dst) + v);
      else
        *dst = static_cast<T>(v);
    }
  }
}

// ---------------------------------------------------------------------------- ring FFTs (belt rings)
// Rings ring0 .. ring0 + nr - 1, each of n = 2^logn pixels, two rings a workgroup (n x 16 bytes of
// LDS): one complex FFT carries both, the first ring in the real part and the second in the imaginary
// part. Analysis: Z = FFT(x1 + i x2), X1[j] = (Z[j] + conj Z[-j]) / 2, X2[j] = (Z[j] - conj Z[-j]) / 2i,
// G_m = e^{-i m pi c / n} X[m mod n].
template <typename T>
__global__ __launch_bounds__(kFftThreads) void sht_belt_fft_kernel(const T* __restrict__ x,
                                                                   const ShtRing* __restrict__ rings, int nrings,
                                                                   int ring0, int nr, int L, int logn,
                                                                   double2* __restrict__ G) {
  extern __shared__ double2 s_fft[];
  __shared__ double2 s_twh[64], s_twl[64];
  const int r1 = ring0 + 2 * xcd_group(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), 4);
  const bool two = r1 + 1 < ring0 + nr;
  const int r2 = two ? r1 + 1 : r1;
  const ShtRing R1 = convreal::ldu_record(rings[r1]);
  const ShtRing R2 = convreal::ldu_record(rings[r2]);
  const int n = R1.n;
  const T* x1 = x + R1.start;
  const T* x2 = x + R2.start;
  convreal::lds_twiddles_fill(s_twh, s_twl, n);
  for (int a = threadIdx.x; a < n; a += blockDim.x)
    s_fft[convreal::bitrev(a, logn)] = double2{static_cast<double>(x1[a]), two ? static_cast<double>(x2[a]) : 0.0};
  __syncthreads();
  convreal::fft_stages_tw(s_fft, n, convreal::LdsTwiddles{s_twh, s_twl});
  for (int m = threadIdx.x; m <= L; m += blockDim.x) {
    const int j = m & (n - 1);
    const double2 zj = s_fft[j], zc = s_fft[(n - j) & (n - 1)];   // Z[j], Z[-j]
    const double2 X1{0.5 * (zj.x + zc.x), 0.5 * (zj.y - zc.y)};
    const double2 X2{0.5 * (zj.y + zc.y), 0.5 * (zc.x - zj.x)};
    double ps, pc;
    sincospi(-static_cast<double>((static_cast<long long>(m) * R1.c) % (2LL * n)) / static_cast<double>(n), &ps, &pc);
    G[static_cast<size_t>(m) * nrings + r1] = double2{X1.x * pc - X1.y * ps, X1.x * ps + X1.y * pc};
    if (two) {
      sincospi(-static_cast<double>((static_cast<long long>(m) * R2.c) % (2LL * n)) / static_cast<double>(n), &ps, &pc);
      G[static_cast<size_t>(m) * nrings + r2] = double2{X2.x * pc - X2.y * ps, X2.x * ps + X2.y * pc};
    }
  }
}

// B[j] = sum_{m = j mod n, m <= L} w_m F_m e^{i m pi c / n} of ring r
__device__ __forceinline__ double2 belt_fold(const double2* __restrict__ F, int nrings, int r, int L, int n, int c,
                                             int j) {
  double br = 0.0, bi = 0.0;
  for (int m = j; m <= L; m += n) {
    const double2 f = F[static_cast<size_t>(m) * nrings + r];
    const long long num = (static_cast<long long>(m) * c) % (2LL * n);
    double ps, pc;
    sincospi(static_cast<double>(num) / static_cast<double>(n), &ps, &pc);
    const double w = m == 0 ? 1.0 : 2.0;
    br += w * (f.x * pc - f.y * ps);
    bi += w * (f.x * ps + f.y * pc);
  }
  return double2{br, bi};
}

// Synthesis: y_a = Re sum_j B[j] e^{2 pi i j a / n} = Re FFT(u)[a] with u = conj B, which is FFT(C)[a]
// for the Hermitian C[j] = (u[j] + conj u[-j]) / 2; two rings a workgroup: FFT(C1 + i C2) = y1 + i y2.
template <typename T, bool ACC>
__global__ __launch_bounds__(kFftThreads) void sht_belt_ifft_kernel(const double2* __restrict__ F,
                                                                    const ShtRing* __restrict__ rings, int nrings,
                                                                    int ring0, int nr, int L, int logn,
                                                                    T* __restrict__ y) {
  extern __shared__ double2 s_fft[];
  __shared__ double2 s_twh[64], s_twl[64];
  const int r1 = ring0 + 2 * xcd_group(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), 4);
  const bool two = r1 + 1 < ring0 + nr;
  const int r2 = two ? r1 + 1 : r1;
  const ShtRing R1 = convreal::ldu_record(rings[r1]);
  const ShtRing R2 = convreal::ldu_record(rings[r2]);
  const int n = R1.n;
  convreal::lds_twiddles_fill(s_twh, s_twl, n);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int jm = (n - j) & (n - 1);
    // C[j] = (conj B[j] + B[-j]) / 2
    const double2 a1 = belt_fold(F, nrings, r1, L, n, R1.c, j), b1 = belt_fold(F, nrings, r1, L, n, R1.c, jm);
    const double2 c1{0.5 * (a1.x + b1.x), 0.5 * (b1.y - a1.y)};
    double2 c2{0.0, 0.0};
    if (two) {
      const double2 a2 = belt_fold(F, nrings, r2, L, n, R2.c, j), b2 = belt_fold(F, nrings, r2, L, n, R2.c, jm);
      c2 = double2{0.5 * (a2.x + b2.x), 0.5 * (b2.y - a2.y)};
    }
    // C1 + i C2
    s_fft[convreal::bitrev(j, logn)] = double2{c1.x - c2.y, c1.y + c2.x};
  }
  __syncthreads();
  convreal::fft_stages_tw(s_fft, n, convreal::LdsTwiddles{s_twh, s_twl});
  T* y1 = y + R1.start;
  T* y2 = y + R2.start;
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    const double2 v = s_fft[a];
    if (ACC) {
      y1[a] = static_cast<T>(static_cast<double>(y1[a]) + v.x);
      if (two) y2[a] = static_cast<T>(static_cast<double>(y2[a]) + v.y);
    } else {
      y1[a] = static_cast<T>(v.x);
      if (two) y2[a] = static_cast<T>(v.y);
    }
  }
}

// ---------------------------------------------------------------------------- ring sums by chirp-z
// Rings with k = n / 4 >= kChirpMin that are not belt rings of a power-of-two grid. Each residue
// class of the folded sums is a k-point DFT, X[4 jq + kappa] = sum_a' d[a'] e^{-2 pi i jq a' / k} with
// d[a'] = c_kappa[a'] e^{-i pi kappa a' / (2 k)}, needed at jq < Q (Q = ceil((min(n, L + 1) - kappa) / 4)).
// Bluestein's chirp-z identity jq a' = (jq^2 + a'^2 - (jq - a')^2) / 2 turns it into a convolution: with
// w(t) = e^{-i pi t^2 / k},
//   X[4 jq + kappa] = w(jq) sum_a' (d[a'] w(a')) conj(w(jq - a')),
// a circular convolution of length M (a power of two, M >= k + Q - 1) taken as FFT(d w) . H, then an
// inverse FFT, where H = FFT(b), b[t] = conj(w(t)) for t in [0, Q), b[M - t] = conj(w(t)) for t in [1, k)
// and zeros between (written at set-up, one table per k, with w(t) for t < k; t^2 mod 2k in integers).
// The synthesis ring sums sum_jq B[jq] e^{2 pi i jq a' / k} = conj(w(a')) sum_jq (B[jq] conj(w(jq))) w(a' - jq)
// for a' < k take the same route with kernel transform conj(H) (that kernel is b mirrored and
// conjugated). O(M log M) per class instead of k Q multiply-adds. The inverse transform is the forward
// one between two conjugations.
struct ChirpTabs {
  const double2* w;          // per k: w(t), t < k
  const double2* h;          // per k: H[f], f < M(k)
  const long long* w_off;    // per k (index k): offset of its w table
  const long long* h_off;    // per k: offset of its H table
};

__device__ __forceinline__ double2 cconj(double2 a) { return double2{a.x, -a.y}; }

// log2 of the convolution length of a ring with k = n / 4 pixels per quarter
__device__ __forceinline__ int chirp_logm(int k, int nk) {
  const int q0 = (nk + 3) >> 2;
  const int len = k + q0 - 1;
  int lg = 1;
  while ((1 << lg) < len) ++lg;
  return lg;
}

// s holds FFT(v) of total / M sequences in natural order; leave conj(FFT(v) . H~) of each in bit-reversed
// order (H~ = H, or conj(H) for the synthesis), ready for the forward FFT that completes the inverse
// transform
__device__ __forceinline__ void chirp_product(double2* s, int M, int logm, const double2* __restrict__ H, bool conj_h,
                                              int total) {
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = t & (M - 1), base = t - i;
    const int j = convreal::bitrev(i, logm);
    if (i > j) continue;
    double2 hi = H[i], hj = H[j];
    if (conj_h) {
      hi = cconj(hi);
      hj = cconj(hj);
    }
    const double2 vi = convreal::cmul(s[base + i], hi), vj = convreal::cmul(s[base + j], hj);
    s[base + j] = cconj(vi);
    s[base + i] = cconj(vj);
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void sht_ring_dft_chirp_kernel(const T* __restrict__ x,
                                                                         const ShtRing* __restrict__ rings,
                                                                         const int* __restrict__ list, int nrings,
                                                                         int L, ChirpTabs c, int lds_elems,
                                                                         double2* __restrict__ G) {
  extern __shared__ double2 s_fft[];
  const int r = list[xcd_group(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), 8)];
  const ShtRing R = convreal::ldu_record(rings[r]);
  const int n = R.n, k = n >> 2;
  const int nk = n < L + 1 ? n : L + 1;
  const int logm = chirp_logm(k, nk), M = 1 << logm;
  const double2* w = c.w + convreal::ldu(c.w_off[k]);
  const double2* H = c.h + convreal::ldu(c.h_off[k]);
  __shared__ double2 s_twh[64], s_twl[64];
  convreal::lds_twiddles_fill(s_twh, s_twl, M);
  const convreal::LdsTwiddles tw{s_twh, s_twl};
  const T* xr = x + R.start;
  const double inv_m = 1.0 / static_cast<double>(M);
  // classes transformed at once: as many M-point sequences as the LDS buffer holds (every FFT pass and
  // barrier shared), up to all four
  const int nc = min(4, lds_elems >> logm);
  for (int k0 = 0; k0 < 4 && k0 < nk; k0 += nc) {
    const int ncb = min(nc, 4 - k0);
    for (int ci = 0; ci < ncb; ++ci) {
      const int kappa = k0 + ci;
      double2* sb = s_fft + ci * M;
      for (int t = threadIdx.x; t < M; t += blockDim.x) {
        double2 v{0.0, 0.0};
        if (t < k && kappa < nk) {
          const double x0 = static_cast<double>(xr[t]), x1 = static_cast<double>(xr[t + k]);
          const double x2 = static_cast<double>(xr[t + 2 * k]), x3 = static_cast<double>(xr[t + 3 * k]);
          // folded value c_kappa[t] (kappa 1: (x0 - x2) - i (x1 - x3), kappa 3: (x0 - x2) + i (x1 - x3))
          const double2 cv = kappa == 0 ? double2{(x0 + x2) + (x1 + x3), 0.0}
                           : kappa == 2 ? double2{(x0 + x2) - (x1 + x3), 0.0}
                           : double2{x0 - x2, kappa == 1 ? x3 - x1 : x1 - x3};
          double2 ph = w[t];
          if (kappa != 0) {
            double ps, pc;
            sincospi(-static_cast<double>(kappa * t) / static_cast<double>(2 * k), &ps, &pc);
            ph = convreal::cmul(double2{pc, ps}, ph);
          }
          v = convreal::cmul(cv, ph);
        }
        sb[convreal::bitrev(t, logm)] = v;
      }
    }
    __syncthreads();
    convreal::fft_stages_tw(s_fft, M, tw, ncb * M);
    chirp_product(s_fft, M, logm, H, false, ncb * M);
    convreal::fft_stages_tw(s_fft, M, tw, ncb * M);
    for (int ci = 0; ci < ncb; ++ci) {
      const int kappa = k0 + ci;
      if (kappa >= nk) break;
      const double2* sb = s_fft + ci * M;
      // G_m = e^{-i m pi c / n} X[m mod n] for every m = kappa (mod 4) up to L (m mod n = 4 jq + kappa
      // with jq < qk, n being a multiple of 4)
      for (int u = threadIdx.x; 4 * u + kappa <= L; u += blockDim.x) {
        const int m = 4 * u + kappa;
        const int jq = (m % n) >> 2;
        const double2 sv = sb[jq];
        const double2 X = convreal::cmul(w[jq], double2{sv.x * inv_m, -sv.y * inv_m});
        const long long num = (static_cast<long long>(m) * R.c) % (2LL * n);
        double ps, pc;
        sincospi(-static_cast<double>(num) / static_cast<double>(n), &ps, &pc);
        G[static_cast<size_t>(m) * nrings + r] = double2{X.x * pc - X.y * ps, X.x * ps + X.y * pc};
      }
    }
    __syncthreads();
  }
}

constexpr int kChirpPer = 4;   // a' values per thread in the synthesis (k <= kChirpPer * kFftThreads)
static_assert(kChirpPer * kFftThreads >= CONV_SHT_MAX_NSIDE, "a ring's quarter fits the synthesis threads");

template <typename T, bool ACC>
__global__ __launch_bounds__(kFftThreads) void sht_ring_idft_chirp_kernel(const double2* __restrict__ F,
                                                                          const ShtRing* __restrict__ rings,
                                                                          const int* __restrict__ list, int nrings,
                                                                          int L, ChirpTabs c, int lds_elems,
                                                                          T* __restrict__ y) {
  extern __shared__ double2 s_fft[];
  const int r = list[xcd_group(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), 8)];
  const ShtRing R = convreal::ldu_record(rings[r]);
  const int n = R.n, k = n >> 2;
  const int nk = n < L + 1 ? n : L + 1;
  const int logm = chirp_logm(k, nk), M = 1 << logm;
  const double2* w = c.w + convreal::ldu(c.w_off[k]);
  const double2* H = c.h + convreal::ldu(c.h_off[k]);
  __shared__ double2 s_twh[64], s_twl[64];
  convreal::lds_twiddles_fill(s_twh, s_twl, M);
  const convreal::LdsTwiddles tw{s_twh, s_twl};
  const double inv_m = 1.0 / static_cast<double>(M);
  double acc[kChirpPer][4];
#pragma unroll
  for (int u = 0; u < kChirpPer; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[u][q] = 0.0;
  // classes transformed at once, as in the analysis
  const int nc = min(4, lds_elems >> logm);
  for (int k0 = 0; k0 < 4 && k0 < nk; k0 += nc) {
    const int ncb = min(nc, 4 - k0);
    for (int t = threadIdx.x; t < ncb * M; t += blockDim.x) s_fft[t] = double2{0.0, 0.0};
    __syncthreads();
    for (int ci = 0; ci < ncb; ++ci) {
      const int kappa = k0 + ci;
      if (kappa >= nk) break;
      const int qk = (nk - kappa + 3) >> 2;
      double2* sb = s_fft + ci * M;
      // B[j], j = 4 t + kappa, times conj(w(t)), in bit-reversed order
      const int nsub = fold_split(qk), sub = static_cast<int>(threadIdx.x) & (nsub - 1);
      for (int t = static_cast<int>(threadIdx.x) / nsub; t < qk; t += static_cast<int>(blockDim.x) / nsub) {
        const double2 b = fold_sum(F, nrings, r, L, n, R.c, 4 * t + kappa, sub, nsub);
        if (sub == 0) sb[convreal::bitrev(t, logm)] = convreal::cmul(b, cconj(w[t]));
      }
    }
    __syncthreads();
    convreal::fft_stages_tw(s_fft, M, tw, ncb * M);
    chirp_product(s_fft, M, logm, H, true, ncb * M);
    convreal::fft_stages_tw(s_fft, M, tw, ncb * M);
    for (int ci = 0; ci < ncb; ++ci) {
      const int kappa = k0 + ci;
      if (kappa >= nk) break;
      const double2* sb = s_fft + ci * M;
  #pragma unroll
      for (int u = 0; u < kChirpPer; ++u) {
        const int ap = static_cast<int>(threadIdx.x) + u * static_cast<int>(blockDim.x);
        if (ap >= k) continue;
        const double2 sv = sb[ap];
        // U = e^{i pi kappa a' / (2k)} conj(w(a')) conv[a'], conv = conj(FFT(...)) / M
        double2 U = convreal::cmul(cconj(w[ap]), double2{sv.x * inv_m, -sv.y * inv_m});
        if (kappa != 0) {
          double ps, pc;
          sincospi(static_cast<double>(kappa * ap) / static_cast<double>(2 * k), &ps, &pc);
          U = convreal::cmul(double2{pc, ps}, U);
        }
        // pixel q k + a': Re(i^{kappa q} U)
  #pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int p = (kappa * q) & 3;
          acc[u][q] += p == 0 ? U.x : (p == 1 ? -U.y : (p == 2 ? -U.x : U.y));
        }
      }
    }
    __syncthreads();
  }
  T* yr = y + R.start;
#pragma unroll
  for (int u = 0; u < kChirpPer; ++u) {
    const int ap = static_cast<int>(threadIdx.x) + u * static_cast<int>(blockDim.x);
    if (ap >= k) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T* dst = yr + q * k + ap;
      if (ACC)
        *dst = static_cast<T>(static_cast<double>(*dst) + acc[u][q]);
      else
        *dst = static_cast<T>(acc[u][q]);
    }
  }
}

// set-up, one workgroup per chirp length k (klist): w(t) for t < k, and H = FFT(b) in natural order
__global__ __launch_bounds__(kFftThreads) void sht_chirp_setup_kernel(const int* __restrict__ klist, int L,
                                                                      const long long* __restrict__ w_off,
                                                                      const long long* __restrict__ h_off,
                                                                      double2* __restrict__ w_tab,
                                                                      double2* __restrict__ h_tab) {
  extern __shared__ double2 s_fft[];
  __shared__ double2 s_twh[64], s_twl[64];
  const int k = klist[blockIdx.x];
  const int n = 4 * k;
  const int nk = n < L + 1 ? n : L + 1;
  const int q0 = (nk + 3) >> 2;
  const int logm = chirp_logm(k, nk), M = 1 << logm;
  double2* w = w_tab + w_off[k];
  convreal::lds_twiddles_fill(s_twh, s_twl, M);
  for (int t = threadIdx.x; t < M; t += blockDim.x) {
    // b[t] = conj(w(t)) on [0, q0) and b[M - t'] = conj(w(t')) on t' in [1, k)
    int tt = -1;
    if (t < q0) tt = t;
    else if (M - t < k) tt = M - t;
    double2 v{0.0, 0.0};
    if (tt >= 0) {
      const long long num = (static_cast<long long>(tt) * tt) % (2LL * k);
      double ps, pc;
      sincospi(static_cast<double>(num) / static_cast<double>(k), &ps, &pc);
      v = double2{pc, ps};   // conj(w(tt)) = e^{+i pi tt^2 / k}
    }
    s_fft[convreal::bitrev(t, logm)] = v;
    if (t < k) {
      const long long num = (static_cast<long long>(t) * t) % (2LL * k);
      double ps, pc;
      sincospi(-static_cast<double>(num) / static_cast<double>(k), &ps, &pc);
      w[t] = double2{pc, ps};
    }
  }
  __syncthreads();
  convreal::fft_stages_tw(s_fft, M, convreal::LdsTwiddles{s_twh, s_twl}, M);
  double2* H = h_tab + h_off[k];
  for (int f = threadIdx.x; f < M; f += blockDim.x) H[f] = s_fft[f];
}

// ---------------------------------------------------------------------------- Legendre sums
// lambda_mm (scaled by 2^(600 e)) for one ring
__device__ __forceinline__ void start_value(double logpre_m, int m, double s, double* p, int* e) {
  const double lg = m == 0 ? logpre_m : fma(static_cast<double>(m), log(s), logpre_m);
  int ee = 0;
  if (lg < kLogFloor) ee = static_cast<int>(ceil((kLogFloor - lg) / kLogScale));
  const double v = exp(fma(static_cast<double>(ee), kLogScale, lg));
  *p = (m & 1) ? -v : v;
  *e = ee;
}

// Per order m, dead[m]: the number of leading chunks of kDeadChunk north rings whose rings never take
// part in either transform's sums. A ring adds to the sums once its carried exponent is zero: from the
// start if log lambda_mm >= kLogFloor, else once the rescaled value has passed kRescaleAbove at a
// check, i.e. once the true |lambda_lm| exceeds 2^-200 at some l <= L. This pass follows the plain
// recurrence lambda_l = a_l (z lambda_{l-1} - lambda_{l-2} / a_{l-1}), a_l = sqrt((4l^2-1)/(l^2-m^2)),
// and calls a ring live once log lambda_mm > kLogFloor - 64 or the true |lambda_lm| passes 2^-300 at
// any l: margins of 2^64 and 2^100 over the transforms' own tests, far beyond any rounding difference.
// Below its turning point |lambda_lm| grows with the colatitude, so a chunk whose last (most
// equatorial) ring is dead is dead throughout; the chunks from the first live one on are all kept.
__global__ void sht_dead_chunks_kernel(const ShtRing* __restrict__ rings, const double* __restrict__ logpre, int L,
                                       int nnorth, int* __restrict__ dead) {
  __shared__ int s_first;
  const int m = blockIdx.x;
  const int nchunks = (nnorth + kDeadChunk - 1) / kDeadChunk;
  if (threadIdx.x == 0) s_first = nchunks;
  __syncthreads();
  for (int c = threadIdx.x; c < nchunks; c += blockDim.x) {
    const ShtRing Rg = rings[min((c + 1) * kDeadChunk, nnorth) - 1];
    const double lg = m == 0 ? logpre[m] : fma(static_cast<double>(m), log(Rg.s), logpre[m]);
    bool live = lg > kLogFloor - 64.0;
    if (!live) {
      int e = static_cast<int>(ceil((kLogFloor - lg) / kLogScale));   // lambda_mm = p1 2^(-600 e)
      double p0 = 0.0, p1 = exp(fma(static_cast<double>(e), kLogScale, lg)), a_prev = 1.0;
      const double mm = static_cast<double>(m) * m;
      for (int l = m + 1; l <= L && !live; ++l) {
        const double dl = l;
        const double al = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - mm));
        const double p2 = al * (Rg.z * p1 - p0 / a_prev);
        p0 = p1;
        p1 = p2;
        a_prev = al;
        if (fabs(p1) > kRescaleAbove) {
          p0 *= kInvScale;
          p1 *= kInvScale;
          --e;
        }
        live = e <= 0 || (e == 1 && fabs(p1) > 0x1p300);
      }
    }
    if (live) atomicMin(&s_first, c);
  }
  __syncthreads();
  if (threadIdx.x == 0) dead[m] = s_first;
}

// The analysis sums of order m over R rings per thread, rings ring0 + j kLegThreadsA + tid; out and
// scale: where the sums go (alm, or the block's partial sums) and their factor.
template <int R>
__device__ __forceinline__ void analysis_body(const LegArgs& a, int m, int ring0, double2* __restrict__ out,
                                              double scale, double2 (&s_red)[kFlush][kLegThreadsA],
                                              double2 (&s_ab)[kLegChunk]) {
  const int tid = threadIdx.x;
  const double2* Gm = a.G + static_cast<size_t>(m) * a.nrings;
  double z[R], ser[R], sei[R], sor[R], soi[R], p0[R], p1[R];
  int e[R], ring[R];
  const double logpre = convreal::ldu(a.logpre[m]);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int rn = ring0 + j * kLegThreadsA + tid;
    ring[j] = rn;
    z[j] = 0.0; ser[j] = sei[j] = sor[j] = soi[j] = 0.0; p0[j] = p1[j] = 0.0; e[j] = 0;
    if (rn < a.nnorth) {
      const ShtRing Rg = a.rings[rn];
      z[j] = Rg.z;
      start_value(logpre, m, Rg.s, &p1[j], &e[j]);
      if (e[j] == 0) {
        const int rs = a.nrings - 1 - rn;
        const double2 gn = Gm[rn];
        const double2 gs = rs != rn ? Gm[rs] : double2{0.0, 0.0};
        ser[j] = gn.x + gs.x; sei[j] = gn.y + gs.y;
        sor[j] = gn.x - gs.x; soi[j] = gn.y - gs.y;
      }
    }
  }
  const double2* coef = a.coef + alm_base(a.L, m);
  // One group: l = l0 .. l0 + kFlush - 1 (l0 - m a multiple of kFlush), the recurrence coefficients
  // from the chunk staged in LDS at c0 (CHECK: tests for l = m, with no recurrence step, and l > L).
  auto group = [&](int l0, int c0, auto check_tag) {
    constexpr bool CHECK = decltype(check_tag)::value;
#pragma unroll
    for (int u = 0; u < kFlush; ++u) {
      const int l = l0 + u;
      if (CHECK && l > a.L) break;
      if (!CHECK || l > m) {
        const double el = s_ab[l - c0].x;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const double p2 = fma(z[j], p1[j], -el * p0[j]);
          p0[j] = p1[j];
          p1[j] = p2;
        }
      }
      // two accumulators per part (rings of even and odd j), so that the sums' chains are half as long
      double tr[2] = {0.0, 0.0}, ti[2] = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < R; ++j) {
        // l - m has the parity of u (l0 - m is a multiple of kFlush)
        tr[j & 1] = fma(p1[j], (u & 1) ? sor[j] : ser[j], tr[j & 1]);
        ti[j & 1] = fma(p1[j], (u & 1) ? soi[j] : sei[j], ti[j & 1]);
      }
      s_red[u][tid] = double2{tr[0] + tr[1], ti[0] + ti[1]};
    }
    __syncthreads();
    // S = kLegThreadsA / kFlush threads per l: thread (u, seg) adds the partial sums seg, seg + S, ...
    // of l = l0 + u, then a butterfly over the S (rows past L hold stale values and are not written)
    {
      constexpr int S = kLegThreadsA / kFlush;
      const int u = tid / S, seg = tid % S;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < kLegThreadsA / S; ++q) {
        const double2 v = s_red[u][seg + S * q];
        sr += v.x;
        si += v.y;
      }
#pragma unroll
      for (int off = S / 2; off >= 1; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
      }
      const int l = l0 + u;
      if (seg == 0 && l <= a.L) {
        const double sc = scale * s_ab[l - c0].y;   // the sums are of mu_l = lambda_l / C_l
        out[l - m] = double2{sc * sr, sc * si};
      }
    }
    // back to lambda for the next group (the last group may end past L: nothing follows it)
    if (l0 + kFlush - 1 <= a.L) {
      const double c1 = s_ab[l0 + kFlush - 1 - c0].y, c0v = s_ab[l0 + kFlush - 2 - c0].y;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        p1[j] *= c1;
        p0[j] *= c0v;
      }
    }
    __syncthreads();
    // bring scaled values back towards the FP64 range; a ring joins the sums once it is unscaled
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (e[j] > 0 && fabs(p1[j]) > kRescaleAbove) {
        p0[j] *= kInvScale;
        p1[j] *= kInvScale;
        e[j] -= 1;
        if (e[j] == 0) {
          const int rn = ring[j], rs = a.nrings - 1 - rn;
          const double2 gn = Gm[rn];
          const double2 gs = rs != rn ? Gm[rs] : double2{0.0, 0.0};
          ser[j] = gn.x + gs.x; sei[j] = gn.y + gs.y;
          sor[j] = gn.x - gs.x; soi[j] = gn.y - gs.y;
        }
      }
    }
  };
  // the coefficients in chunks of kLegChunk values of l (a multiple of kFlush, so groups never
  // straddle a chunk), loaded by all threads at once
  for (int c0 = m; c0 <= a.L; c0 += kLegChunk) {
    const int cn = min(kLegChunk, a.L + 1 - c0);
    for (int i = tid; i < cn; i += kLegThreadsA) s_ab[i] = coef[c0 - m + i];
    __syncthreads();
    // every group checks its bounds: with 8 rings per thread an unchecked copy of the group exceeds
    // the register file
    for (int l0 = c0; l0 < c0 + cn; l0 += kFlush) group(l0, c0, std::true_type{});
    // the groups end with a barrier: the next chunk may overwrite s_ab
  }
}

template <int R>
__global__ __launch_bounds__(kLegThreadsA) void sht_analysis_legendre_kernel(LegArgs a, int nblk, double2* partial) {
  __shared__ double2 s_red[kFlush][kLegThreadsA];
  __shared__ double2 s_ab[kLegChunk];
  const int item = blockIdx.x;
  const int m = item / nblk;
  const int blk = item - m * nblk;
  const long long base = alm_base(a.L, m);
  double2* out = nblk == 1 ? a.alm + base : partial + static_cast<size_t>(blk) * ((a.L + 1LL) * (a.L + 2) / 2) + base;
  const double scale = nblk == 1 ? a.omega : 1.0;
  // thread ring j covers chunk blk R + j: the leading dead ones are left out in pairs (so that the
  // remaining rings keep the parity of j that picks their accumulator); a block of dead rings only
  // writes zero sums
  const int jd = min(max(convreal::ldu(a.dead[m]) - blk * R, 0), R);
  if (jd == R) {
    for (int l = m + static_cast<int>(threadIdx.x); l <= a.L; l += kLegThreadsA) out[l - m] = double2{0.0, 0.0};
    return;
  }
  const int j0 = jd & ~1;
  const int ring0 = (blk * R + j0) * kLegThreadsA;
  if (j0 == 0) {
    analysis_body<R>(a, m, ring0, out, scale, s_red, s_ab);
  } else if constexpr (R == 8) {
    if (j0 == 2)
      analysis_body<6>(a, m, ring0, out, scale, s_red, s_ab);
    else if (j0 == 4)
      analysis_body<4>(a, m, ring0, out, scale, s_red, s_ab);
    else
      analysis_body<2>(a, m, ring0, out, scale, s_red, s_ab);
  } else if constexpr (R == 4) {
    analysis_body<2>(a, m, ring0, out, scale, s_red, s_ab);
  }
}

// a_lm = Omega sum over ring blocks of the partial sums (several blocks per order)
__global__ void sht_reduce_kernel(const double2* __restrict__ partial, int nblk, long long nalm, double omega,
                                  double2* __restrict__ alm) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  double sr = 0.0, si = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double2 v = partial[static_cast<size_t>(b) * nalm + i];
    sr += v.x;
    si += v.y;
  }
  alm[i] = double2{omega * sr, omega * si};
}

// F_m of R rings per thread, rings ring0 + j kLegThreads + tid
template <int R>
__device__ __forceinline__ void synthesis_body(const LegArgs& a, int m, int ring0, double2 (&s_ab)[kLegChunk],
                                               double2 (&s_al)[kLegChunk]) {
  const int tid = threadIdx.x;
  double z[R], fer[R], fei[R], forr[R], foi[R], p0[R], p1[R];
  int e[R];
  const double logpre = convreal::ldu(a.logpre[m]);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int rn = ring0 + j * kLegThreads + tid;
    z[j] = 0.0; p0[j] = p1[j] = 0.0; e[j] = 0;
    fer[j] = fei[j] = forr[j] = foi[j] = 0.0;
    if (rn < a.nnorth) {
      const ShtRing Rg = a.rings[rn];
      z[j] = Rg.z;
      start_value(logpre, m, Rg.s, &p1[j], &e[j]);
    }
  }
  const long long base = alm_base(a.L, m);
  const double2* coef = a.coef + base;
  const double2* alm = a.alm + base;
  // one unit l0 .. l0 + kFlushS - 1 (CHECK for the units that hold l = m or run past L), coefficients
  // and alm from the chunk staged in LDS at c0; the scaled recurrence goes back to lambda after the
  // second unit of each kFlush group (the rescale test between may see mu <= lambda: it then acts one
  // unit later, far inside the FP64 range)
  auto group = [&](int l0, int c0, auto check_tag) {
    constexpr bool CHECK = decltype(check_tag)::value;
#pragma unroll
    for (int u = 0; u < kFlushS; ++u) {
      const int l = l0 + u;
      if (CHECK && l > a.L) break;
      if (!CHECK || l > m) {
        const double el = s_ab[l - c0].x;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const double p2 = fma(z[j], p1[j], -el * p0[j]);
          p0[j] = p1[j];
          p1[j] = p2;
        }
      }
      const double2 b = s_al[l - c0];   // b_lm C_l: the recurrence carries mu_l = lambda_l / C_l
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (u & 1) {
          forr[j] = fma(p1[j], b.x, forr[j]);
          foi[j] = fma(p1[j], b.y, foi[j]);
        } else {
          fer[j] = fma(p1[j], b.x, fer[j]);
          fei[j] = fma(p1[j], b.y, fei[j]);
        }
      }
    }
    // back to lambda at the end of a kFlush group (the last group may end past L: nothing follows it)
    if (((l0 - m) % kFlush) == kFlush - kFlushS && l0 + kFlushS - 1 <= a.L) {
      const double c1 = s_ab[l0 + kFlushS - 1 - c0].y, c0v = s_ab[l0 + kFlushS - 2 - c0].y;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        p1[j] *= c1;
        p0[j] *= c0v;
      }
    }
    // rings still scaled drop what they added (true values below 2^-144 of the scaled ones)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (e[j] > 0) {
        fer[j] = fei[j] = forr[j] = foi[j] = 0.0;
        if (fabs(p1[j]) > kRescaleAbove) {
          p0[j] *= kInvScale;
          p1[j] *= kInvScale;
          e[j] -= 1;
        }
      }
    }
  };
  for (int c0 = m; c0 <= a.L; c0 += kLegChunk) {
    const int cn = min(kLegChunk, a.L + 1 - c0);
    __syncthreads();   // the previous chunk's values are read by every thread
    if (tid < cn) {
      const double2 cf = coef[c0 - m + tid], b = alm[c0 - m + tid];
      s_ab[tid] = cf;
      s_al[tid] = double2{b.x * cf.y, b.y * cf.y};
    }
    __syncthreads();
    for (int l0 = c0; l0 < c0 + cn; l0 += kFlushS) {
      if (l0 > m && l0 + kFlushS - 1 <= a.L)
        group(l0, c0, std::false_type{});
      else
        group(l0, c0, std::true_type{});
    }
  }
  double2* Fm = a.G + static_cast<size_t>(m) * a.nrings;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int rn = ring0 + j * kLegThreads + tid;
    if (rn < a.nnorth) {
      const int rs = a.nrings - 1 - rn;
      Fm[rn] = double2{fer[j] + forr[j], fei[j] + foi[j]};
      if (rs != rn) Fm[rs] = double2{fer[j] - forr[j], fei[j] - foi[j]};
    }
  }
}

template <int R>
__global__ __launch_bounds__(kLegThreads) void sht_synthesis_legendre_kernel(LegArgs a, int nblk) {
  __shared__ double2 s_ab[kLegChunk];
  __shared__ double2 s_al[kLegChunk];
  const int item = blockIdx.x;
  const int m = item / nblk;
  const int blk = item - m * nblk;
  // thread ring j covers chunks 2 (blk R + j) and 2 (blk R + j) + 1: the leading dead ones are left
  // out, their F_m (both hemispheres) set to zero
  const int jd = min(max(convreal::ldu(a.dead[m]) / 2 - blk * R, 0), R);
  double2* Fm = a.G + static_cast<size_t>(m) * a.nrings;
  for (int j = 0; j < jd; ++j) {
    const int rn = (blk * R + j) * kLegThreads + static_cast<int>(threadIdx.x);
    if (rn < a.nnorth) {
      const int rs = a.nrings - 1 - rn;
      Fm[rn] = double2{0.0, 0.0};
      if (rs != rn) Fm[rs] = double2{0.0, 0.0};
    }
  }
  if (jd == R) return;
  const int ring0 = (blk * R + jd) * kLegThreads;
  if (jd == 0)
    synthesis_body<R>(a, m, ring0, s_ab, s_al);
  else if constexpr (R == 2)
    synthesis_body<1>(a, m, ring0, s_ab, s_al);
}

// ---------------------------------------------------------------------------- alm helpers
__global__ void sht_almxfl_kernel(const double2* __restrict__ in, const double* __restrict__ fl, int L,
                                  double2* __restrict__ out) {
  const int m = blockIdx.x;
  const long long base = alm_base(L, m);
  for (int l = m + threadIdx.x; l <= L; l += blockDim.x) {
    const double f = fl[l];
    const double2 v = in[base + l - m];
    out[base + l - m] = double2{f * v.x, f * v.y};
  }
}

__global__ void sht_power_kernel(const double2* __restrict__ alm, int L, double* __restrict__ cl) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l > L) return;
  double s = 0.0;
  for (int m = 0; m <= l; ++m) {
    const double2 v = alm[alm_base(L, m) + l - m];
    const double p = v.x * v.x + v.y * v.y;
    s += m == 0 ? p : 2.0 * p;
  }
  cl[l] = s / (2.0 * l + 1.0);
}

}  // namespace

// ---------------------------------------------------------------------------- plan
struct conv_sht_plan {
  unsigned magic = 0;
  int device = 0;
  int nside = 0;
  int L = 0;
  int nrings = 0;
  int nnorth = 0;
  long long npix = 0;
  long long nalm = 0;
  int R = 1;                 // north rings per thread in the synthesis Legendre kernel
  int nblk = 1;              // its ring blocks per order
  int Ra = 1;                // the same for the analysis kernel, whose blocks each reduce over rings
  int nblk_a = 1;
  double omega = 0.0;
  ShtRing* d_rings = nullptr;
  double2* d_coef = nullptr;
  double* d_logpre = nullptr;
  double2* d_G = nullptr;
  double2* d_alm = nullptr;       // workspace of conv_sht_convolve and the hybrid apply
  double2* d_partial = nullptr;   // nblk > 1: per-block partial sums of the analysis
  int* d_dead = nullptr;          // per m: leading chunks of polar rings left out of the Legendre sums
  int fft_ring0 = 0;              // belt rings ring0 .. ring0 + fft_nrings - 1 by FFT (power-of-two Nside)
  int fft_nrings = 0;
  int fft_logn = 0;
  int* d_direct = nullptr;        // rings of the folded Horner sums (k < kChirpMin)
  int n_direct = 0;
  int* d_chirp = nullptr;         // rings of the chirp-z ring sums
  int n_chirp = 0;
  int chirp_logm_max = 0;         // largest convolution length (log2) among them
  struct ChirpRange { int logm, off, count; };
  std::vector<ChirpRange> chirp_ranges;   // launches over d_chirp (one, largest convolutions first; logm
                                          // sizes its LDS buffer, which shorter rings fill with several classes)
  double2* d_chirp_w = nullptr;   // chirp tables (ChirpTabs)
  double2* d_chirp_h = nullptr;
  long long* d_chirp_woff = nullptr;
  long long* d_chirp_hoff = nullptr;
  hipEvent_t ev_in = nullptr, ev_real = nullptr, ev_done = nullptr;
  std::vector<void*> owned;
};

namespace {

constexpr unsigned kShtMagic = 0x53485450u;  // "SHTP"

using convreal::DeviceGuard;
using convreal::hip_fail;
using convreal::set_error;

bool plan_ok(const conv_sht_plan* p) { return p && p->magic == kShtMagic; }

template <typename T>
hipError_t sht_alloc(conv_sht_plan* p, T** out, size_t count) {
  *out = nullptr;
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, (count ? count : 1) * sizeof(T));
  if (e != hipSuccess) return e;
  p->owned.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return hipSuccess;
}

void free_sht(conv_sht_plan* p) {
  for (void* ptr : p->owned) (void)hipFree(ptr);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_real) (void)hipEventDestroy(p->ev_real);
  if (p->ev_done) (void)hipEventDestroy(p->ev_done);
  p->magic = 0;
  delete p;
}

size_t dft_lds(int nside) { return 32 * static_cast<size_t>(nside); }
size_t idft_lds(int nside, int L) {
  const int nk = std::min(4 * nside, L + 1);
  return 16 * static_cast<size_t>(4 * ((nk + 3) / 4));
}

hipError_t set_lds_attributes(int nside, int L) {
  const int a = static_cast<int>(std::max<size_t>(dft_lds(nside), 16));
  const int s = static_cast<int>(std::max<size_t>(idft_lds(nside, L), 16));
  const void* fa[] = {reinterpret_cast<const void*>(&sht_ring_dft_kernel<double>),
                      reinterpret_cast<const void*>(&sht_ring_dft_kernel<float>)};
  const void* fs[] = {reinterpret_cast<const void*>(&sht_ring_idft_kernel<double, false>),
                      reinterpret_cast<const void*>(&sht_ring_idft_kernel<double, true>),
                      reinterpret_cast<const void*>(&sht_ring_idft_kernel<float, false>),
                      reinterpret_cast<const void*>(&sht_ring_idft_kernel<float, true>)};
  for (const void* f : fa) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, std::max(a, 65536));
    if (e != hipSuccess) return e;
  }
  for (const void* f : fs) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, std::max(s, 65536));
    if (e != hipSuccess) return e;
  }
  const int nf = std::max(static_cast<int>(16 * 4 * static_cast<size_t>(nside)), 65536);
  const void* ff[] = {reinterpret_cast<const void*>(&sht_belt_fft_kernel<double>),
                      reinterpret_cast<const void*>(&sht_belt_fft_kernel<float>),
                      reinterpret_cast<const void*>(&sht_belt_ifft_kernel<double, false>),
                      reinterpret_cast<const void*>(&sht_belt_ifft_kernel<double, true>),
                      reinterpret_cast<const void*>(&sht_belt_ifft_kernel<float, false>),
                      reinterpret_cast<const void*>(&sht_belt_ifft_kernel<float, true>)};
  for (const void* f : ff) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, nf);
    if (e != hipSuccess) return e;
  }
  // chirp-z convolutions of at most 4096 points (k + Q - 1 <= 2 k - 1 < 4096 for Nside <= 2048)
  const void* fc[] = {reinterpret_cast<const void*>(&sht_ring_dft_chirp_kernel<double>),
                      reinterpret_cast<const void*>(&sht_ring_dft_chirp_kernel<float>),
                      reinterpret_cast<const void*>(&sht_ring_idft_chirp_kernel<double, false>),
                      reinterpret_cast<const void*>(&sht_ring_idft_chirp_kernel<double, true>),
                      reinterpret_cast<const void*>(&sht_ring_idft_chirp_kernel<float, false>),
                      reinterpret_cast<const void*>(&sht_ring_idft_chirp_kernel<float, true>),
                      reinterpret_cast<const void*>(&sht_chirp_setup_kernel)};
  for (const void* f : fc) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 16 * 4096);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

ChirpTabs chirp_tabs(const conv_sht_plan* p) {
  return ChirpTabs{p->d_chirp_w, p->d_chirp_h, p->d_chirp_woff, p->d_chirp_hoff};
}

hipError_t launch_analysis_legendre(const conv_sht_plan* p, double2* alm, hipStream_t st) {
  LegArgs a{p->d_rings, p->d_coef, p->d_logpre, p->d_G, alm, p->d_dead, p->L, p->nrings, p->nnorth, p->omega};
  const dim3 g(static_cast<unsigned>((p->L + 1) * p->nblk_a)), b(kLegThreadsA);
  switch (p->Ra) {
    case 1: hipLaunchKernelGGL(sht_analysis_legendre_kernel<1>, g, b, 0, st, a, p->nblk_a, p->d_partial); break;
    case 2: hipLaunchKernelGGL(sht_analysis_legendre_kernel<2>, g, b, 0, st, a, p->nblk_a, p->d_partial); break;
    case 4: hipLaunchKernelGGL(sht_analysis_legendre_kernel<4>, g, b, 0, st, a, p->nblk_a, p->d_partial); break;
    default: hipLaunchKernelGGL(sht_analysis_legendre_kernel<8>, g, b, 0, st, a, p->nblk_a, p->d_partial); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p->nblk_a == 1) return e;
  const unsigned gr = static_cast<unsigned>((p->nalm + 255) / 256);
  hipLaunchKernelGGL(sht_reduce_kernel, dim3(gr), dim3(256), 0, st, p->d_partial, p->nblk_a, p->nalm, p->omega, alm);
  return hipGetLastError();
}

hipError_t launch_synthesis_legendre(const conv_sht_plan* p, const double2* alm, hipStream_t st) {
  LegArgs a{p->d_rings, p->d_coef, p->d_logpre, p->d_G, const_cast<double2*>(alm), p->d_dead, p->L, p->nrings,
            p->nnorth, p->omega};
  const dim3 g(static_cast<unsigned>((p->L + 1) * p->nblk)), b(kLegThreads);
  switch (p->R) {
    case 1: hipLaunchKernelGGL(sht_synthesis_legendre_kernel<1>, g, b, 0, st, a, p->nblk); break;
    default: hipLaunchKernelGGL(sht_synthesis_legendre_kernel<2>, g, b, 0, st, a, p->nblk); break;
  }
  return hipGetLastError();
}

hipError_t launch_analysis(const conv_sht_plan* p, const void* map, int dtype, double2* alm, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (p->n_direct > 0) {
    const size_t lds = dft_lds(p->nside);
    const dim3 g(static_cast<unsigned>(p->n_direct)), b(kDftThreads);
    if (dtype == CONV_SHT_F64)
      hipLaunchKernelGGL(sht_ring_dft_kernel<double>, g, b, lds, st, static_cast<const double*>(map), p->d_rings,
                         p->d_direct, p->nrings, p->L, p->d_G);
    else
      hipLaunchKernelGGL(sht_ring_dft_kernel<float>, g, b, lds, st, static_cast<const float*>(map), p->d_rings,
                         p->d_direct, p->nrings, p->L, p->d_G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (const auto& cr : p->chirp_ranges) {
    const size_t lds = sizeof(double2) << cr.logm;
    const dim3 g(static_cast<unsigned>(cr.count)), b(kFftThreads);
    const int* lst = p->d_chirp + cr.off;
    if (dtype == CONV_SHT_F64)
      hipLaunchKernelGGL(sht_ring_dft_chirp_kernel<double>, g, b, lds, st, static_cast<const double*>(map),
                         p->d_rings, lst, p->nrings, p->L, chirp_tabs(p), 1 << cr.logm, p->d_G);
    else
      hipLaunchKernelGGL(sht_ring_dft_chirp_kernel<float>, g, b, lds, st, static_cast<const float*>(map),
                         p->d_rings, lst, p->nrings, p->L, chirp_tabs(p), 1 << cr.logm, p->d_G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (p->fft_nrings > 0) {
    const size_t lf = sizeof(double2) * (static_cast<size_t>(1) << p->fft_logn);
    const dim3 g(static_cast<unsigned>((p->fft_nrings + 1) / 2)), b(kFftThreads);
    if (dtype == CONV_SHT_F64)
      hipLaunchKernelGGL(sht_belt_fft_kernel<double>, g, b, lf, st, static_cast<const double*>(map), p->d_rings,
                         p->nrings, p->fft_ring0, p->fft_nrings, p->L, p->fft_logn, p->d_G);
    else
      hipLaunchKernelGGL(sht_belt_fft_kernel<float>, g, b, lf, st, static_cast<const float*>(map), p->d_rings,
                         p->nrings, p->fft_ring0, p->fft_nrings, p->L, p->fft_logn, p->d_G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return launch_analysis_legendre(p, alm, st);
}

hipError_t launch_ring_synthesis(const conv_sht_plan* p, void* map, int dtype, int accumulate, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (p->n_direct > 0) {
    const size_t lds = idft_lds(p->nside, p->L);
    const dim3 g(static_cast<unsigned>(p->n_direct)), b(kDftThreads);
    const int* lst = p->d_direct;
    if (dtype == CONV_SHT_F64) {
      double* y = static_cast<double*>(map);
      if (accumulate)
        hipLaunchKernelGGL((sht_ring_idft_kernel<double, true>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, y);
      else
        hipLaunchKernelGGL((sht_ring_idft_kernel<double, false>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, y);
    } else {
      float* y = static_cast<float*>(map);
      if (accumulate)
        hipLaunchKernelGGL((sht_ring_idft_kernel<float, true>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, y);
      else
        hipLaunchKernelGGL((sht_ring_idft_kernel<float, false>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, y);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (const auto& cr : p->chirp_ranges) {
    const size_t lds = sizeof(double2) << cr.logm;
    const dim3 g(static_cast<unsigned>(cr.count)), b(kFftThreads);
    const int* lst = p->d_chirp + cr.off;
    const ChirpTabs c = chirp_tabs(p);
    if (dtype == CONV_SHT_F64) {
      double* y = static_cast<double*>(map);
      if (accumulate)
        hipLaunchKernelGGL((sht_ring_idft_chirp_kernel<double, true>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, c, 1 << cr.logm, y);
      else
        hipLaunchKernelGGL((sht_ring_idft_chirp_kernel<double, false>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, c, 1 << cr.logm, y);
    } else {
      float* y = static_cast<float*>(map);
      if (accumulate)
        hipLaunchKernelGGL((sht_ring_idft_chirp_kernel<float, true>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, c, 1 << cr.logm, y);
      else
        hipLaunchKernelGGL((sht_ring_idft_chirp_kernel<float, false>), g, b, lds, st, p->d_G, p->d_rings, lst, p->nrings, p->L, c, 1 << cr.logm, y);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int s0 = p->fft_ring0, ns = p->fft_nrings;
  if (ns == 0) return hipSuccess;
  const size_t lf = sizeof(double2) * (static_cast<size_t>(1) << p->fft_logn);
  const dim3 gf(static_cast<unsigned>((ns + 1) / 2)), bf(kFftThreads);
  if (dtype == CONV_SHT_F64) {
    double* y = static_cast<double*>(map);
    if (accumulate)
      hipLaunchKernelGGL((sht_belt_ifft_kernel<double, true>), gf, bf, lf, st, p->d_G, p->d_rings, p->nrings, s0, ns, p->L, p->fft_logn, y);
    else
      hipLaunchKernelGGL((sht_belt_ifft_kernel<double, false>), gf, bf, lf, st, p->d_G, p->d_rings, p->nrings, s0, ns, p->L, p->fft_logn, y);
  } else {
    float* y = static_cast<float*>(map);
    if (accumulate)
      hipLaunchKernelGGL((sht_belt_ifft_kernel<float, true>), gf, bf, lf, st, p->d_G, p->d_rings, p->nrings, s0, ns, p->L, p->fft_logn, y);
    else
      hipLaunchKernelGGL((sht_belt_ifft_kernel<float, false>), gf, bf, lf, st, p->d_G, p->d_rings, p->nrings, s0, ns, p->L, p->fft_logn, y);
  }
  return hipGetLastError();
}

hipError_t launch_almxfl(const conv_sht_plan* p, const double2* in, const double* fl, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(sht_almxfl_kernel, dim3(p->L + 1), dim3(256), 0, st, in, fl, p->L, out);
  return hipGetLastError();
}

int check_dtype(int dtype, const char* where) {
  if (dtype != CONV_SHT_F64 && dtype != CONV_SHT_F32) {
    set_error(std::string(where) + ": dtype must be CONV_SHT_F64 or CONV_SHT_F32");
    return CONV_REAL_EINVAL;
  }
  return CONV_REAL_OK;
}

}  // namespace

extern "C" {

int conv_sht_alm_size(int lmax, long long* n) {
  if (!n || lmax < 0 || lmax > CONV_SHT_MAX_LMAX) {
    set_error("conv_sht_alm_size: invalid argument");
    return CONV_REAL_EINVAL;
  }
  *n = (static_cast<long long>(lmax) + 1) * (lmax + 2) / 2;
  return CONV_REAL_OK;
}

int conv_sht_init(conv_sht_plan** plan, int nside, int lmax) {
  if (!plan) { set_error("conv_sht_init: NULL plan pointer"); return CONV_REAL_EINVAL; }
  *plan = nullptr;
  if (nside < 1 || nside > CONV_SHT_MAX_NSIDE) { set_error("conv_sht_init: nside out of range"); return CONV_REAL_EINVAL; }
  if (lmax < 0 || lmax > CONV_SHT_MAX_LMAX) { set_error("conv_sht_init: lmax out of range"); return CONV_REAL_EINVAL; }
  int dev = 0;
  int rc = convreal::check_device(&dev);
  if (rc != CONV_REAL_OK) return rc;
  auto* p = new (std::nothrow) conv_sht_plan();
  if (!p) { set_error("conv_sht_init: host allocation failed"); return CONV_REAL_ENOMEM; }
  p->magic = kShtMagic;
  p->device = dev;
  p->nside = nside;
  p->L = lmax;
  p->nrings = 4 * nside - 1;
  p->nnorth = 2 * nside;
  p->npix = 12LL * nside * nside;
  p->nalm = (static_cast<long long>(lmax) + 1) * (lmax + 2) / 2;
  p->omega = 4.0 * M_PI / static_cast<double>(p->npix);
  // synthesis: up to 2 rings per thread, more rings in several ring blocks per order (more waves per
  // SIMD; at Nside 2048 1-5% faster than 4, while 8 exceed the register file once the unrolled steps
  // keep their values in registers); analysis: up to 8, since every block reduces over its rings for
  // every l (fewer blocks, fewer reductions)
  p->R = 1;
  while (p->R < 2 && static_cast<long long>(p->R) * kLegThreads < p->nnorth) p->R *= 2;
  p->nblk = static_cast<int>((p->nnorth + static_cast<long long>(p->R) * kLegThreads - 1) /
                             (static_cast<long long>(p->R) * kLegThreads));
  p->Ra = 1;
  while (p->Ra < 8 && static_cast<long long>(p->Ra) * kLegThreadsA < p->nnorth) p->Ra *= 2;
  p->nblk_a = static_cast<int>((p->nnorth + static_cast<long long>(p->Ra) * kLegThreadsA - 1) /
                               (static_cast<long long>(p->Ra) * kLegThreadsA));

  // rings from the grid's exact integer numerators
  const convreal::RingGrid g = convreal::make_ring_grid(nside);
  std::vector<ShtRing> rings(g.nrings);
  for (int r = 0; r < g.nrings; ++r) rings[r] = ShtRing{g.z[r], g.s[r], g.start[r], g.n[r], g.c[r]};
  // recurrence coefficients in the scaled form of the kernels, and l = m normalisations. Within a group
  // of kFlush values of l (l0 - m a multiple of kFlush) the kernels carry mu_l = lambda_l / C_l with
  // C_l = a_l C_{l-1} (C = 1 for the two values entering the group, and at l = m), so that
  // lambda_l = a_l (z lambda_{l-1} - b_l lambda_{l-2}) becomes mu_l = z mu_{l-1} - e_l mu_{l-2},
  // e_l = b_l C_{l-2} / C_{l-1}: one multiply and one multiply-add a step; the table holds (e_l, C_l).
  std::vector<double2> coef(static_cast<size_t>(p->nalm));
  std::vector<double> logpre(lmax + 1);
  double acc = 0.0;
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) acc += std::log((2.0 * m - 1.0) / (2.0 * m));
    logpre[m] = 0.5 * (std::log((2.0 * m + 1.0) / (4.0 * M_PI)) + acc);
    const long long base = static_cast<long long>(m) * (2 * lmax + 3 - m) / 2;
    coef[base] = double2{0.0, 1.0};
    const double mm = static_cast<double>(m) * m;
    double c1 = 1.0, c2 = 1.0;   // C_{l-1}, C_{l-2} within the group
    for (int l = m + 1; l <= lmax; ++l) {
      const int u = (l - m) % kFlush;
      if (u == 0) c1 = c2 = 1.0;
      if (u == 1) c2 = 1.0;
      const double dl = l, dl1 = l - 1.0;
      const double al = std::sqrt((4.0 * dl * dl - 1.0) / (dl * dl - mm));
      const double bl = std::sqrt((dl1 * dl1 - mm) / (4.0 * dl1 * dl1 - 1.0));
      const double cl = al * c1;
      coef[base + l - m] = double2{bl * c2 / c1, cl};
      c2 = c1;
      c1 = cl;
    }
  }
  // belt rings (i = N..3N, n = 4N) by FFT when 4N is a power of two (and at least 16)
  if ((nside & (nside - 1)) == 0 && nside >= 4) {
    const int n = 4 * nside;
    p->fft_ring0 = nside - 1;
    p->fft_nrings = 2 * nside + 1;
    while ((1 << p->fft_logn) < n) ++p->fft_logn;
  }
  // the other rings: chirp-z ring sums from k = kChirpMin on, folded sums below; one chirp table per k
  std::vector<int> direct, chirp, klist;
  std::vector<long long> woff, hoff;
  long long wtot = 0, htot = 0;
  {
    std::vector<char> need(nside + 1, 0);
    for (int r = 0; r < g.nrings; ++r) {
      if (r >= p->fft_ring0 && r < p->fft_ring0 + p->fft_nrings) continue;
      const int k = g.n[r] / 4;
      if (k >= kChirpMin) {
        chirp.push_back(r);
        need[k] = 1;
      } else {
        direct.push_back(r);
      }
    }
    woff.assign(nside + 1, 0);
    hoff.assign(nside + 1, 0);
    auto logm_of = [lmax](int k) {
      const int nk = std::min(4 * k, lmax + 1);
      const int len = k + (nk + 3) / 4 - 1;
      int lg = 1;
      while ((1 << lg) < len) ++lg;
      return lg;
    };
    // one launch, largest convolutions first (the shortest rings fill the tail); launches per length
    // with only the LDS each needs measured slower (each launch's tail idles the device)
    std::stable_sort(chirp.begin(), chirp.end(),
                     [&](int a, int b) { return logm_of(g.n[a] / 4) > logm_of(g.n[b] / 4); });
    if (!chirp.empty())
      p->chirp_ranges.push_back(conv_sht_plan::ChirpRange{logm_of(g.n[chirp[0]] / 4), 0, static_cast<int>(chirp.size())});
    for (int k = 1; k <= nside; ++k) {
      if (!need[k]) continue;
      const int lg = logm_of(k);
      woff[k] = wtot;
      hoff[k] = htot;
      wtot += k;
      htot += 1LL << lg;
      p->chirp_logm_max = std::max(p->chirp_logm_max, lg);
      klist.push_back(k);
    }
  }
  p->n_direct = static_cast<int>(direct.size());
  p->n_chirp = static_cast<int>(chirp.size());
  DeviceGuard guard;
  hipError_t e = guard.enter(dev);
  if (e == hipSuccess) e = set_lds_attributes(nside, lmax);
  if (e == hipSuccess && !direct.empty()) e = sht_alloc(p, &p->d_direct, direct.size());
  if (e == hipSuccess && !direct.empty())
    e = hipMemcpy(p->d_direct, direct.data(), direct.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && !chirp.empty()) {
    int* d_klist = nullptr;
    if (e == hipSuccess) e = sht_alloc(p, &p->d_chirp, chirp.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_chirp, chirp.data(), chirp.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sht_alloc(p, &d_klist, klist.size());
    if (e == hipSuccess) e = hipMemcpy(d_klist, klist.data(), klist.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sht_alloc(p, &p->d_chirp_woff, woff.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_chirp_woff, woff.data(), woff.size() * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sht_alloc(p, &p->d_chirp_hoff, hoff.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_chirp_hoff, hoff.data(), hoff.size() * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sht_alloc(p, &p->d_chirp_w, static_cast<size_t>(wtot));
    if (e == hipSuccess) e = sht_alloc(p, &p->d_chirp_h, static_cast<size_t>(htot));
    if (e == hipSuccess) {
      hipLaunchKernelGGL(sht_chirp_setup_kernel, dim3(static_cast<unsigned>(klist.size())), dim3(kFftThreads),
                         sizeof(double2) << p->chirp_logm_max, nullptr, d_klist, lmax, p->d_chirp_woff,
                         p->d_chirp_hoff, p->d_chirp_w, p->d_chirp_h);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  }
  if (e == hipSuccess) e = sht_alloc(p, &p->d_rings, rings.size());
  if (e == hipSuccess) e = hipMemcpy(p->d_rings, rings.data(), rings.size() * sizeof(ShtRing), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sht_alloc(p, &p->d_coef, coef.size());
  if (e == hipSuccess) e = hipMemcpy(p->d_coef, coef.data(), coef.size() * sizeof(double2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sht_alloc(p, &p->d_logpre, logpre.size());
  if (e == hipSuccess) e = hipMemcpy(p->d_logpre, logpre.data(), logpre.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sht_alloc(p, &p->d_G, static_cast<size_t>(lmax + 1) * p->nrings);
  if (e == hipSuccess) e = sht_alloc(p, &p->d_alm, static_cast<size_t>(p->nalm));
  if (e == hipSuccess && p->nblk_a > 1) e = sht_alloc(p, &p->d_partial, static_cast<size_t>(p->nalm) * p->nblk_a);
  if (e == hipSuccess) e = sht_alloc(p, &p->d_dead, static_cast<size_t>(lmax) + 1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(sht_dead_chunks_kernel, dim3(static_cast<unsigned>(lmax + 1)), dim3(64), 0, nullptr,
                       p->d_rings, p->d_logpre, lmax, p->nnorth, p->d_dead);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_real, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    rc = hip_fail(e, "conv_sht_init");
    free_sht(p);
    return rc;
  }
  *plan = p;
  return CONV_REAL_OK;
}

int conv_sht_analysis(conv_sht_plan* plan, const void* map, int dtype, void* alm, void* stream) {
  if (!plan_ok(plan) || !map || !alm) { set_error("conv_sht_analysis: invalid argument"); return CONV_REAL_EINVAL; }
  int rc = check_dtype(dtype, "conv_sht_analysis");
  if (rc != CONV_REAL_OK) return rc;
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e == hipSuccess) e = launch_analysis(plan, map, dtype, static_cast<double2*>(alm), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? CONV_REAL_OK : hip_fail(e, "conv_sht_analysis");
}

int conv_sht_synthesis(conv_sht_plan* plan, const void* alm, void* map, int dtype, int accumulate, void* stream) {
  if (!plan_ok(plan) || !map || !alm) { set_error("conv_sht_synthesis: invalid argument"); return CONV_REAL_EINVAL; }
  int rc = check_dtype(dtype, "conv_sht_synthesis");
  if (rc != CONV_REAL_OK) return rc;
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (e == hipSuccess) e = launch_synthesis_legendre(plan, static_cast<const double2*>(alm), st);
  if (e == hipSuccess) e = launch_ring_synthesis(plan, map, dtype, accumulate, st);
  return e == hipSuccess ? CONV_REAL_OK : hip_fail(e, "conv_sht_synthesis");
}

int conv_sht_almxfl(conv_sht_plan* plan, const void* alm_in, const double* fl, void* alm_out, void* stream) {
  if (!plan_ok(plan) || !alm_in || !fl || !alm_out) { set_error("conv_sht_almxfl: invalid argument"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e == hipSuccess)
    e = launch_almxfl(plan, static_cast<const double2*>(alm_in), fl, static_cast<double2*>(alm_out),
                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? CONV_REAL_OK : hip_fail(e, "conv_sht_almxfl");
}

int conv_sht_convolve(conv_sht_plan* plan, const void* map_in, const double* k_ell, void* map_out, int dtype,
                      int accumulate, void* stream) {
  if (!plan_ok(plan) || !map_in || !k_ell || !map_out) { set_error("conv_sht_convolve: invalid argument"); return CONV_REAL_EINVAL; }
  int rc = check_dtype(dtype, "conv_sht_convolve");
  if (rc != CONV_REAL_OK) return rc;
  const size_t bytes = static_cast<size_t>(plan->npix) * (dtype == CONV_SHT_F64 ? 8 : 4);
  const char* i0 = static_cast<const char*>(map_in);
  const char* o0 = static_cast<const char*>(map_out);
  if (i0 < o0 + bytes && o0 < i0 + bytes) { set_error("conv_sht_convolve: maps overlap"); return CONV_REAL_EALIAS; }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (e == hipSuccess) e = launch_analysis(plan, map_in, dtype, plan->d_alm, st);
  if (e == hipSuccess) e = launch_almxfl(plan, plan->d_alm, k_ell, plan->d_alm, st);
  if (e == hipSuccess) e = launch_synthesis_legendre(plan, plan->d_alm, st);
  if (e == hipSuccess) e = launch_ring_synthesis(plan, map_out, dtype, accumulate, st);
  return e == hipSuccess ? CONV_REAL_OK : hip_fail(e, "conv_sht_convolve");
}

int conv_sht_power_spectrum(conv_sht_plan* plan, const void* alm, double* cl, void* stream) {
  if (!plan_ok(plan) || !alm || !cl) { set_error("conv_sht_power_spectrum: invalid argument"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(sht_power_kernel, dim3((plan->L + 256) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double2*>(alm), plan->L, cl);
    e = hipGetLastError();
  }
  return e == hipSuccess ? CONV_REAL_OK : hip_fail(e, "conv_sht_power_spectrum");
}

int conv_hybrid_apply(conv_real_plan* real, conv_sht_plan* sht, const double* k_hat, const void* maps_in,
                      void* maps_out, int nmaps, void* stream, void* stream_sht) {
  if (!plan_ok(sht) || !real || !k_hat || !maps_in || !maps_out || nmaps < 1) {
    set_error("conv_hybrid_apply: invalid argument");
    return CONV_REAL_EINVAL;
  }
  int nside = 0, precision = 0, device = 0;
  int rc = convreal::plan_info(real, &nside, &precision, &device);
  if (rc != CONV_REAL_OK) return rc;
  if (nside != sht->nside || device != sht->device) {
    set_error("conv_hybrid_apply: the two plans differ in grid or device");
    return CONV_REAL_EINVAL;
  }
  const int dtype = precision == CONV_REAL_F64 ? CONV_SHT_F64 : CONV_SHT_F32;
  const size_t elem = dtype == CONV_SHT_F64 ? 8 : 4;
  const size_t bytes = static_cast<size_t>(nmaps) * sht->npix * elem;
  const char* i0 = static_cast<const char*>(maps_in);
  const char* o0 = static_cast<const char*>(maps_out);
  if (i0 < o0 + bytes && o0 < i0 + bytes) { set_error("conv_hybrid_apply: maps_in and maps_out overlap"); return CONV_REAL_EALIAS; }
  DeviceGuard guard;
  hipError_t e = guard.enter(sht->device);
  if (e != hipSuccess) return hip_fail(e, "conv_hybrid_apply: hipSetDevice");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const hipStream_t s2 = stream_sht ? static_cast<hipStream_t>(stream_sht) : st;
  const bool two = s2 != st;
  for (int k = 0; k < nmaps && e == hipSuccess; ++k) {
    const void* x = static_cast<const char*>(maps_in) + k * sht->npix * elem;
    void* y = static_cast<char*>(maps_out) + k * sht->npix * elem;
    if (two) {
      // the harmonic stream starts once the inputs are ready in the caller's stream
      if ((e = hipEventRecord(sht->ev_in, st)) != hipSuccess || (e = hipStreamWaitEvent(s2, sht->ev_in, 0)) != hipSuccess)
        break;
    }
    rc = conv_real_apply(real, x, y, 1, stream);
    if (rc != CONV_REAL_OK) return rc;
    if ((e = launch_analysis(sht, x, dtype, sht->d_alm, s2)) != hipSuccess) break;
    if ((e = launch_almxfl(sht, sht->d_alm, k_hat, sht->d_alm, s2)) != hipSuccess) break;
    if ((e = launch_synthesis_legendre(sht, sht->d_alm, s2)) != hipSuccess) break;
    if (two) {
      if ((e = hipEventRecord(sht->ev_real, st)) != hipSuccess || (e = hipStreamWaitEvent(s2, sht->ev_real, 0)) != hipSuccess)
        break;
    }
    if ((e = launch_ring_synthesis(sht, y, dtype, 1, s2)) != hipSuccess) break;
    if (two) {
      if ((e = hipEventRecord(sht->ev_done, s2)) != hipSuccess || (e = hipStreamWaitEvent(st, sht->ev_done, 0)) != hipSuccess)
        break;
    }
  }
  return e == hipSuccess ? CONV_REAL_OK : hip_fail(e, "conv_hybrid_apply");
}

int conv_sht_destroy(conv_sht_plan* plan) {
  if (!plan) return CONV_REAL_OK;
  if (!plan_ok(plan)) { set_error("conv_sht_destroy: invalid plan"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  (void)guard.enter(plan->device);
  free_sht(plan);
  return CONV_REAL_OK;
}

}  // extern "C"
