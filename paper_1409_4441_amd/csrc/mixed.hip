// Mixed-precision path: belt ring pairs as dense contractions on the gfx950 matrix cores.
//
// In the equatorial belt every ring has 4N pixels on the same azimuth grid (up to a half-pixel
// offset), so the weight between output pixel a of ring i and input pixel b of ring j depends only
// on (i, j, m = b - a):
//   w_ij[m] = Omega * Ktilde(d),  d^2 = A_ij + B_ij sin^2(pi (2m - delta_ij) / (8N)),
//   delta_ij = c_i - c_j (azimuth offsets phi = pi (2a + c) / 4N).
// For a band of 16 output rings and a run of output pixels, the contribution of input ring j is a
// matrix product
//   Y[i][a] += sum_m W_j[i][m] X_j[m][a],   X_j[m][a] = x_j[a + m]   (Hankel windows of ring j),
// with M = 16 output rings, N = output pixels, K = window offsets m (a tight range per (band, j),
// in chunks of 32). One v_mfma_f32_16x16x32_f16 computes a 16 x 16 x 32 block. Precision: weights
// and map values are split into FP16 pairs, w s_w = w_hi + w_lo, x s_x = x_hi + x_lo (s_w, s_x
// powers of two), and each block is the sum of the three products w_hi x_hi + w_lo x_hi + w_hi x_lo
// accumulated in FP32; the dropped w_lo x_lo and the split residues are ~2^-22 relative. Every few
// input rings the FP32 accumulators are folded into FP64 so that rounding does not build up over the
// ~50 ring pairs of an output.
//
// Data layout:
//   weight fragments: per (band, input ring j, K-chunk q) 2 x 64 lanes x 8 FP16 (hi then lo), in
//   the lane order of the MFMA A operand (lane l: row l % 16, offsets 8 (l / 16) .. + 7);
//   map windows: staged per input ring into LDS as 8 copies shifted by one pixel each, so that
//   every lane's 8 consecutive FP16 values start on a 16-byte boundary in one of the copies; the
//   copy stride is padded so that the 8 copies fall on different LDS bank groups.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "internal.h"

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kSeg = 256;                  // output pixels per workgroup
constexpr int kWaves = 4;
constexpr int kNB = kSeg / (16 * kWaves);  // 16-pixel blocks per wave
constexpr int kFold = 4;                   // input rings per FP32 -> FP64 fold

// ---------------------------------------------------------------- per-map |x| maximum
__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0u;
}

__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ x, long long npix,
                                                     unsigned* __restrict__ amax) {
  const int m = blockIdx.y;
  const float* xm = x + static_cast<long long>(m) * npix;
  float v = 0.0f;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < npix;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    v = fmaxf(v, fabsf(xm[i]));
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  // non-negative floats order like their bit patterns
  if ((threadIdx.x & 63) == 0) atomicMax(amax + m, __float_as_uint(v));
}

// power of two s with max|x| * s in [2^12, 2^13)
__device__ __forceinline__ float map_scale(unsigned bits) {
  const float mx = __uint_as_float(bits);
  if (!(mx > 0.0f) || !isfinite(mx)) return 1.0f;
  int e;
  (void)frexpf(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  return ldexpf(1.0f, 13 - e);
}

// ---------------------------------------------------------------- weight fragments (init)
struct WeightArgs {
  const double* table;
  const long long* Z;
  const double* s;
  const int* rc;
  const int* chunk_band;  // per K-chunk: band
  const int* chunk_j;     // per K-chunk: input ring
  const int* chunk_m0;    // per K-chunk: first window offset
  _Float16* wt;
  long long nthreads;
  int belt_lo;
  int belt_hi;
  int nside;
  int n_tab;
  double q3;              // 3 N^2
  double inv_h;
  double dcut2;
  double omega;
  double sw;
};

__global__ __launch_bounds__(256) void belt_weights_kernel(WeightArgs a) {
  const long long tid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= a.nthreads) return;
  const int e = static_cast<int>(tid & 7);
  const int l = static_cast<int>((tid >> 3) & 63);
  const long long ch = tid >> 9;
  const int band = a.chunk_band[ch];
  const int j = a.chunk_j[ch];
  const int row = l & 15;
  const int m = a.chunk_m0[ch] + 8 * (l >> 4) + e;
  const int i = a.belt_lo + 16 * band + row;
  double w = 0.0;
  if (i <= a.belt_hi) {
    double A, B;
    convreal::chord_constants(a.Z[i], a.Z[j], a.s[i], a.s[j], a.q3, &A, &B);
    const int delta = a.rc[i] - a.rc[j];
    const double sn = sin(M_PI * static_cast<double>(2 * m - delta) / (8.0 * a.nside));
    const double d2 = fma(B, sn * sn, A);
    if (d2 <= a.dcut2) w = a.omega * convreal::interp_f64(a.table, a.n_tab, sqrt(d2), a.inv_h);
  }
  const double ws = w * a.sw;
  const _Float16 hi = static_cast<_Float16>(ws);
  const _Float16 lo = static_cast<_Float16>(ws - static_cast<double>(hi));
  const long long base = ch * 1024;  // 2 planes x 64 lanes x 8
  a.wt[base + l * 8 + e] = hi;
  a.wt[base + 512 + l * 8 + e] = lo;
}

// ---------------------------------------------------------------- belt contraction
struct BeltArgs {
  const half8* wt;
  const int* band_jf;
  const int* band_nj;
  const int* band_woff;
  const int* blk_koff;   // per (band, input ring): first K-chunk
  const int* blk_nk;     // per (band, input ring): K-chunks
  const int* blk_mlo;    // per (band, input ring): first window offset
  const long long* rstart;
  const unsigned* amax;
  int nbands;
  int nsegs;
  int belt_lo;
  int belt_hi;
  int ring_n;            // 4N
  float inv_sw;
  long long npix;
};

template <int NK>
struct StageLayout {
  static constexpr int L = kSeg + 32 * NK;          // staged window length (pixels)
  // copy stride in halves: 2L plus padding so that the stride is 144 bytes mod 256, which puts the
  // 8 copies on 8 different 16-byte bank groups
  static constexpr int CS = 2 * L + ((NK & 1) ? 8 : 72);
  static constexpr int BUF = 8 * CS;
};

template <int NK>
__device__ __forceinline__ void stage_ring(_Float16* __restrict__ S, const float* __restrict__ xj,
                                           int start_px, int len, int ring_n, float sx) {
  using SL = StageLayout<NK>;
  for (int u = threadIdx.x; u < len; u += blockDim.x) {
    int p = start_px + u;
    while (p < 0) p += ring_n;
    while (p >= ring_n) p -= ring_n;
    const float xs = xj[p] * sx;
    const _Float16 hh = static_cast<_Float16>(xs);
    const _Float16 ll = static_cast<_Float16>(xs - static_cast<float>(hh));
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (u >= c) {
        S[c * SL::CS + u - c] = hh;
        S[c * SL::CS + SL::L + u - c] = ll;
      }
    }
  }
}

template <int NK>
__global__ __launch_bounds__(kSeg) void belt_mfma_kernel(BeltArgs a, const float* __restrict__ x,
                                                         float* __restrict__ y) {
  using SL = StageLayout<NK>;
  __shared__ __attribute__((aligned(16))) _Float16 S[2 * SL::BUF];
  const int item = convreal::xcd_remap(blockIdx.x, a.nbands * a.nsegs);
  const int band = item / a.nsegs;
  const int seg = item % a.nsegs;
  const int map = blockIdx.y;
  const float* xm = x + static_cast<long long>(map) * a.npix;
  float* ym = y + static_cast<long long>(map) * a.npix;
  const float sx = map_scale(a.amax[map]);
  const int a0 = seg * kSeg;
  const int jf = a.band_jf[band];
  const int nj = a.band_nj[band];
  const int woff = a.band_woff[band];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15;
  const int g = lane >> 4;
  const int cpy = n & 7;
  // offset (halves) of this lane's first B value within its shifted copy, for block 0, chunk 0
  const int lane_off = cpy * SL::CS + 16 * (kNB * wave) + (n - cpy) + 8 * g;

  floatx4 acc[kNB];
  double accd[kNB][4];
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[b][r] = 0.0;
  }

  {
    const int nk0 = a.blk_nk[woff];
    stage_ring<NK>(S, xm + a.rstart[jf], a0 + a.blk_mlo[woff], kSeg + 32 * nk0, a.ring_n, sx);
  }
  __syncthreads();
  for (int jj = 0; jj < nj; ++jj) {
    const int buf = jj & 1;
    if (jj + 1 < nj) {
      const int nb1 = a.blk_nk[woff + jj + 1];
      stage_ring<NK>(S + (buf ^ 1) * SL::BUF, xm + a.rstart[jf + jj + 1], a0 + a.blk_mlo[woff + jj + 1],
                     kSeg + 32 * nb1, a.ring_n, sx);
    }
    const int nk = a.blk_nk[woff + jj];
    const half8* wblk = a.wt + static_cast<long long>(a.blk_koff[woff + jj]) * 128;
    const _Float16* Sb = S + buf * SL::BUF + lane_off;
    for (int q = 0; q < nk; ++q) {
      const half8 whi = wblk[q * 128 + lane];
      const half8 wlo = wblk[q * 128 + 64 + lane];
      half8 xhi[kNB], xlo[kNB];
#pragma unroll
      for (int b = 0; b < kNB; ++b) {
        xhi[b] = *reinterpret_cast<const half8*>(Sb + 16 * b + 32 * q);
        xlo[b] = *reinterpret_cast<const half8*>(Sb + SL::L + 16 * b + 32 * q);
      }
#pragma unroll
      for (int b = 0; b < kNB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xhi[b], acc[b], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < kNB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, xhi[b], acc[b], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < kNB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xlo[b], acc[b], 0, 0, 0);
    }
    if ((jj % kFold) == kFold - 1 || jj + 1 == nj) {
#pragma unroll
      for (int b = 0; b < kNB; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[b][r] += static_cast<double>(acc[b][r]);
        acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
  }

  const double inv = static_cast<double>(a.inv_sw) / static_cast<double>(sx);
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const int px = a0 + 16 * (kNB * wave + b) + n;
    if (px >= a.ring_n) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ring = a.belt_lo + 16 * band + 4 * g + r;
      if (ring <= a.belt_hi) ym[a.rstart[ring] + px] = static_cast<float>(accd[b][r] * inv);
    }
  }
}

}  // namespace

namespace convreal {

hipError_t build_belt_weights(conv_real_plan* p) {
  WeightArgs a;
  a.table = p->d_table;
  a.Z = p->d_Z;
  a.s = p->d_s;
  a.rc = p->d_rc;
  a.chunk_band = p->d_chunk_band;
  a.chunk_j = p->d_chunk_j;
  a.chunk_m0 = p->d_chunk_m0;
  a.wt = p->d_wt;
  a.nthreads = static_cast<long long>(p->n_chunks) * 512;
  a.belt_lo = p->belt_lo;
  a.belt_hi = p->belt_hi;
  a.nside = p->nside;
  a.n_tab = p->n_tab;
  a.q3 = 3.0 * static_cast<double>(p->nside) * static_cast<double>(p->nside);
  a.inv_h = p->inv_h;
  a.dcut2 = p->dcut2;
  a.omega = p->omega;
  a.sw = p->belt_sw;
  const unsigned grid = static_cast<unsigned>((a.nthreads + 255) / 256);
  hipLaunchKernelGGL(belt_weights_kernel, dim3(grid), dim3(256), 0, nullptr, a);
  return hipGetLastError();
}

hipError_t launch_mixed(const conv_real_plan* p, const float* x, float* y, int nmaps, hipStream_t st) {
  for (int m0 = 0; m0 < nmaps; m0 += kMaxMixedMaps) {
    const int nm = nmaps - m0 < kMaxMixedMaps ? nmaps - m0 : kMaxMixedMaps;
    const float* xi = x + static_cast<size_t>(m0) * p->npix;
    float* yo = y + static_cast<size_t>(m0) * p->npix;
    if (p->belt_enabled) {
      hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, p->d_amax, nm);
      mark(p, st, "zero_u32_kernel", 0);
      const long long want = (p->npix + 255) / 256;
      const unsigned gx = static_cast<unsigned>(want < 1024 ? want : 1024);
      hipLaunchKernelGGL(absmax_kernel, dim3(gx, nm), dim3(256), 0, st, xi, p->npix, p->d_amax);
      mark(p, st, "absmax_kernel", 0);
      BeltArgs a;
      a.wt = reinterpret_cast<const half8*>(p->d_wt);
      a.band_jf = p->d_band_jf;
      a.band_nj = p->d_band_nj;
      a.band_woff = p->d_band_woff;
      a.blk_koff = p->d_blk_koff;
      a.blk_nk = p->d_blk_nk;
      a.blk_mlo = p->d_blk_mlo;
      a.rstart = p->d_rstart;
      a.amax = p->d_amax;
      a.nbands = p->belt_nbands;
      a.nsegs = p->belt_nsegs;
      a.belt_lo = p->belt_lo;
      a.belt_hi = p->belt_hi;
      a.ring_n = 4 * p->nside;
      a.inv_sw = static_cast<float>(1.0 / p->belt_sw);
      a.npix = p->npix;
      const dim3 grid(static_cast<unsigned>(p->belt_nbands * p->belt_nsegs), static_cast<unsigned>(nm));
      switch (p->belt_nk) {
        case 1: hipLaunchKernelGGL(belt_mfma_kernel<1>, grid, dim3(kSeg), 0, st, a, xi, yo); break;
        case 2: hipLaunchKernelGGL(belt_mfma_kernel<2>, grid, dim3(kSeg), 0, st, a, xi, yo); break;
        case 3: hipLaunchKernelGGL(belt_mfma_kernel<3>, grid, dim3(kSeg), 0, st, a, xi, yo); break;
        default: hipLaunchKernelGGL(belt_mfma_kernel<4>, grid, dim3(kSeg), 0, st, a, xi, yo); break;
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      mark(p, st, "belt_mfma_kernel", (p->pairs - p->pairs_rest) * nm);
    }
    hipError_t e = launch_remainder(p, xi, yo, nm, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace convreal
