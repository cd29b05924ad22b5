// Mixed-precision path: all ring pairs on the gfx950 matrix cores, in one persistent launch.
//
// Belt ring pairs (both rings in the equatorial belt, 4N pixels on one azimuth grid up to a
// half-pixel offset): the weight between output pixel a of ring i and input pixel b of ring j
// depends only on (i, j, m = b - a),
//   w_ij[m] = Omega * Ktilde(d),  d^2 = A_ij + B_ij sin^2(pi (2m - delta_ij) / (8N)),
//   delta_ij = c_i - c_j (azimuth offsets phi = pi (2a + c) / 4N),
// so for a band of 16 output rings and a run of output pixels the contribution of input ring j is
//   Y[i][a] += sum_m W_j[i][m] X_j[m][a],   X_j[m][a] = x_j[a + m]   (Hankel windows of ring j),
// with M = 16 output rings, N = output pixels, K = window offsets m (a tight range per (band, j)).
// Weight fragments are built once per plan in FP64 and stored split into FP16 pairs in the lane
// order of the MFMA A operand (lane l: row l % 16, offsets 8 (l / 16) .. + 7). Map windows are
// staged in LDS as 8 copies shifted by one pixel, so that every lane's 8 consecutive FP16 values
// start on a 16-byte boundary in one of them; the copy stride puts the copies on different banks.
//
// Ring pairs that touch a polar cap: the pixelization's 16-element symmetry group (quarter turn
// a -> a + n/4, reflection phi -> -phi i.e. a -> n - a - c, north/south mirror i -> 4N - i) leaves
// every weight invariant when both pixels move together, so one weight row of output pixel a
// serves its 16 images: y[img_g(a)] = sum_b w(a, b) x[img_g(b)]. A wave takes 16 output pixels of
// the group's fundamental domain and, per neighbour ring, computes D[16 pixels][16 images] +=
// W[16][K] X[K][16]. W is evaluated on the fly: integer azimuth numerator -> alpha = dphi/2,
// sin^2 alpha by a polynomial, d^2 = A + B sin^2 alpha, all in FP64 (the oscillating kernel is
// sensitive to d at the 1e-8 level near the cut), then the 4-point interpolant in cubic form from
// an LDS table of per-segment FP32 coefficients. Images that coincide are stored once.
//
// Precision of both: weights and map values are split into FP16 pairs, w s_w = w_hi + w_lo,
// x s_x = x_hi + x_lo (powers of two), and each block is w_hi x_hi + w_lo x_hi + w_hi x_lo
// accumulated in FP32 by v_mfma_f32_16x16x32_f16; the dropped w_lo x_lo and the split residues are
// ~2^-22 relative. FP32 accumulators are folded into FP64 every few ring pairs.
//
// Scheduling: one workgroup of 4 waves repeatedly takes the next item of a cost-sorted queue: a
// belt item (one band x one segment of output pixels, MFMA-bound) or a cap item (4 tiles, one per
// wave, VALU-bound by weight evaluation), so that both kinds share every CU. Rows that receive a
// belt and a cap-pair contribution (belt rings near the belt edge) are zeroed beforehand and get
// exactly two atomic adds, which is order-independent: fl(0 + a + b) = fl(0 + b + a).
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "internal.h"

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kFold = 4;   // ring pairs per FP32 -> FP64 fold
constexpr int kNKMax = 4;  // largest K-chunk count of a belt weight block

// ---------------------------------------------------------------- shared helpers
// power of two s with max|x| * s in [2^12, 2^13)
__device__ __forceinline__ float map_scale(unsigned bits) {
  const float mx = __uint_as_float(bits);
  if (!(mx > 0.0f) || !isfinite(mx)) return 1.0f;
  int e;
  (void)frexpf(mx, &e);
  return ldexpf(1.0f, 13 - e);
}

__device__ __forceinline__ void put(float* p, double v, bool add) {
  if (add)
    atomicAdd(p, static_cast<float>(v));
  else
    *p = static_cast<float>(v);
}

template <int SEG>
struct BeltLayout {
  static constexpr int L = SEG + 32 * kNKMax;    // staged window length (pixels)
  // copy stride (halves): 2L plus padding so that it is 144 bytes mod 256
  static constexpr int CS = 2 * L + ((((2 * L * 2) % 256) == 0) ? 72 : 8);
  static constexpr int BUF = 8 * CS;
  static constexpr int BYTES = 2 * BUF * 2;      // two buffers of FP16
  static_assert(((CS * 2) % 256) == 144, "copy stride must spread the 8 copies over LDS banks");
};

// ---------------------------------------------------------------- prep kernels
__global__ void zero_state_kernel(unsigned* amax, int n, unsigned* counter) {
  const int t = threadIdx.x;
  if (t < n) amax[t] = 0u;
  if (t == 0) *counter = 0u;
}

// per slot: |x| maximum (atomicMax on the bit pattern: non-negative floats order like their bits),
// and zero of the rows that will receive two atomic adds
__global__ __launch_bounds__(256) void prep_kernel(convreal::Slots S, unsigned* __restrict__ amax) {
  const int slot = blockIdx.y;
  const convreal::MixedDesc* d = S.desc[slot];
  const long long npix = d->npix;
  const float* x = S.x[slot];
  float* y = S.y[slot];
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  float v = 0.0f;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < npix; i += stride)
    v = fmaxf(v, fabsf(x[i]));
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) atomicMax(amax + slot, __float_as_uint(v));
  for (int z = 0; z < 2; ++z) {
    const long long z0 = d->zero_lo[z], z1 = d->zero_hi[z];
    for (long long i = z0 + static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < z1; i += stride)
      y[i] = 0.0f;
  }
}

// ---------------------------------------------------------------- belt weight fragments (init)
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

// ---------------------------------------------------------------- belt item
template <int SEG>
__device__ __forceinline__ void stage_ring(_Float16* __restrict__ S, const float* __restrict__ xj,
                                           int start_px, int len, int ring_n, float sx) {
  using BL = BeltLayout<SEG>;
  for (int u = threadIdx.x; u < len; u += kBlock) {
    int p = start_px + u;
    while (p < 0) p += ring_n;
    while (p >= ring_n) p -= ring_n;
    const float xs = xj[p] * sx;
    const _Float16 hh = static_cast<_Float16>(xs);
    const _Float16 ll = static_cast<_Float16>(xs - static_cast<float>(hh));
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (u >= c) {
        S[c * BL::CS + u - c] = hh;
        S[c * BL::CS + BL::L + u - c] = ll;
      }
    }
  }
}

template <int SEG>
__device__ void belt_item(const convreal::MixedDesc* __restrict__ d, int idx, const float* __restrict__ xm,
                          float* __restrict__ ym, float sx, _Float16* __restrict__ S) {
  using BL = BeltLayout<SEG>;
  constexpr int NB = SEG / (16 * kWaves);  // 16-pixel blocks per wave
  const int nsegs = (d->ring_n + SEG - 1) / SEG;
  const int band = idx / nsegs;
  const int seg = idx % nsegs;
  const int a0 = seg * SEG;
  const int jf = d->band_jf[band];
  const int nj = d->band_nj[band];
  const int woff = d->band_woff[band];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15;
  const int g = lane >> 4;
  const int cpy = n & 7;
  const int lane_off = cpy * BL::CS + 16 * (NB * wave) + (n - cpy) + 8 * g;
  const half8* wt = reinterpret_cast<const half8*>(d->wt);

  floatx4 acc[NB];
  double accd[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[b][r] = 0.0;
  }

  stage_ring<SEG>(S, xm + d->rstart[jf], a0 + d->blk_mlo[woff], SEG + 32 * d->blk_nk[woff], d->ring_n, sx);
  __syncthreads();
  for (int jj = 0; jj < nj; ++jj) {
    const int buf = jj & 1;
    if (jj + 1 < nj)
      stage_ring<SEG>(S + (buf ^ 1) * BL::BUF, xm + d->rstart[jf + jj + 1], a0 + d->blk_mlo[woff + jj + 1],
                      SEG + 32 * d->blk_nk[woff + jj + 1], d->ring_n, sx);
    const int nk = d->blk_nk[woff + jj];
    const half8* wblk = wt + static_cast<long long>(d->blk_koff[woff + jj]) * 128;
    const _Float16* Sb = S + buf * BL::BUF + lane_off;
    for (int q = 0; q < nk; ++q) {
      const half8 whi = wblk[q * 128 + lane];
      const half8 wlo = wblk[q * 128 + 64 + lane];
      half8 xhi[NB], xlo[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        xhi[b] = *reinterpret_cast<const half8*>(Sb + 16 * b + 32 * q);
        xlo[b] = *reinterpret_cast<const half8*>(Sb + BL::L + 16 * b + 32 * q);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xhi[b], acc[b], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, xhi[b], acc[b], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xlo[b], acc[b], 0, 0, 0);
    }
    if ((jj % kFold) == kFold - 1 || jj + 1 == nj) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[b][r] += static_cast<double>(acc[b][r]);
        acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
  }

  const double inv = static_cast<double>(d->inv_sw) / static_cast<double>(sx);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int px = a0 + 16 * (NB * wave + b) + n;
    if (px >= d->ring_n) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ring = d->belt_lo + 16 * band + 4 * g + r;
      if (ring <= d->belt_hi) put(ym + d->rstart[ring] + px, accd[b][r] * inv, d->ring_add[ring] != 0);
    }
  }
}

// ---------------------------------------------------------------- cap item
__device__ __forceinline__ double sin2_of(double alpha) {
  // sin^2(alpha) = t P(t), t = alpha^2; P fitted on t in [0, 2.6] (|alpha| <= 1.61), relative
  // error below 1e-11 there.
  const double t = alpha * alpha;
  double p = -1.366547170656072e-09;
  p = fma(p, t, 9.31392155360743e-08);
  p = fma(p, t, -4.273732374386684e-06);
  p = fma(p, t, 0.00014109120522641625);
  p = fma(p, t, -0.0031746016082493094);
  p = fma(p, t, 0.04444444389087041);
  p = fma(p, t, -0.3333333332512937);
  p = fma(p, t, 0.9999999999970449);
  return t * p;
}

// sqrt for d^2 > 0 from the hardware reciprocal square root and one Newton step; 0 for d^2 = 0
__device__ __forceinline__ double chord_of(double d2) {
  double y = __builtin_amdgcn_rsq(d2);
  y = y * fma(-0.5 * d2, y * y, 1.5);
  return d2 > 0.0 ? d2 * y : 0.0;
}

// first and last input pixel of ring j in the window of output pixel a of ring i
__device__ __forceinline__ void row_window(int a, int ni, int ci, int nj, int cj, double hw, bool whole,
                                           long long* lo, long long* hi) {
  const double bc =
      static_cast<double>(static_cast<long long>(2 * a + ci) * nj - static_cast<long long>(cj) * ni) / (2.0 * ni);
  if (whole) {
    *lo = static_cast<long long>(floor(bc)) - nj / 2;
    *hi = *lo + nj - 1;
  } else {
    *lo = static_cast<long long>(ceil(bc - hw - 1e-7));
    *hi = static_cast<long long>(floor(bc + hw + 1e-7));
  }
}

__device__ __forceinline__ long long wrap_num(long long v, long long M) {
  const long long m2 = 2 * M;
  while (v > M) v -= m2;
  while (v <= -M) v += m2;
  return v;
}

__device__ __forceinline__ int mod_pos(long long v, int n) {
  long long r = v % n;
  if (r < 0) r += n;
  return static_cast<int>(r);
}

// one wave: tile t (16 output pixels of the fundamental domain of one north-half ring)
__device__ void cap_tile(const convreal::MixedDesc* __restrict__ d, int t, const float* __restrict__ xm,
                         float* __restrict__ ym, float sx, const float4* __restrict__ s_coef) {
  const int r = d->citem_ring[t];
  const int a0 = d->citem_a0[t];
  const int ni = d->rn[r];
  const int ci = d->rc[r];
  const int mr = d->nrings - 1 - r;
  const int lane = threadIdx.x & 63;
  const int row = lane & 15;       // A operand: output pixel a0 + row
  const int kgrp = lane >> 4;      // A and B operands: k-group of 8
  const int col = lane & 15;       // B operand / D: image index
  const int ch = col >> 3;         // hemisphere
  const int cf = (col >> 2) & 1;   // reflection
  const int cq = col & 3;          // quarter turn
  const int arow = a0 + row;

  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  double accd[4] = {0.0, 0.0, 0.0, 0.0};
  const long long k0 = d->rest_off[r];
  const long long k1 = d->rest_off[r + 1];
  int nfold = 0;
  for (long long kk = k0; kk < k1; ++kk) {
    const long long k = d->rest_idx[kk];
    const int j = d->pj[k];
    const int nj = d->rn[j];
    const int cj = d->rc[j];
    const double hw = d->phw[k];
    const double A = d->pA[k];
    const double B = d->pB[k];
    const bool whole = 2.0 * hw >= static_cast<double>(nj);
    long long b0, bend, lo_r, hi_r, tmp;
    row_window(a0, ni, ci, nj, cj, hw, whole, &b0, &tmp);
    row_window(a0 + 15, ni, ci, nj, cj, hw, whole, &tmp, &bend);
    row_window(arow, ni, ci, nj, cj, hw, whole, &lo_r, &hi_r);
    const int K = static_cast<int>(bend - b0 + 1);
    if (K <= 0) continue;
    const int nk = (K + 31) >> 5;
    const long long M = static_cast<long long>(ni) * nj;
    const double alpha_scale = M_PI / (2.0 * static_cast<double>(M));
    const int jh = ch ? (d->nrings - 1 - j) : j;
    const float* xj = xm + d->rstart[jh];
    const int qoff = cq * (nj >> 2);
    for (int q = 0; q < nk; ++q) {
      // A operand: weights of row arow for inputs b = b0 + 32q + 8 kgrp + e; the FP64 test
      // d^2 <= d_cut^2 decides the pairs in the window's slack exactly as the per-pair path does
      const long long bA = b0 + 32 * q + 8 * kgrp;
      long long num = wrap_num(static_cast<long long>(2 * arow + ci) * nj - (2 * bA + cj) * static_cast<long long>(ni), M);
      half8 whi, wlo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const long long b = bA + e;
        float w = 0.0f;
        const double d2 = fma(B, sin2_of(static_cast<double>(num) * alpha_scale), A);
        if (b >= lo_r && b <= hi_r && d2 <= d->dcut2) {
          const double tt = chord_of(d2) * d->inv_h;
          int sg = static_cast<int>(tt);
          sg = min(sg, d->nseg - 1);
          const float f = static_cast<float>(tt - static_cast<double>(sg));
          const float4 c = s_coef[sg];
          w = fmaf(fmaf(fmaf(c.w, f, c.z), f, c.y), f, c.x);
        }
        const _Float16 h = static_cast<_Float16>(w);
        whi[e] = h;
        wlo[e] = static_cast<_Float16>(w - static_cast<float>(h));
        num = wrap_num(num - 2 * static_cast<long long>(ni), M);
      }
      // B operand: image col of the same inputs
      int p = cf ? mod_pos(static_cast<long long>(nj) - bA - cj + qoff, nj) : mod_pos(bA + qoff, nj);
      half8 xhi, xlo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float xs = xj[p] * sx;
        const _Float16 h = static_cast<_Float16>(xs);
        xhi[e] = h;
        xlo[e] = static_cast<_Float16>(xs - static_cast<float>(h));
        if (cf)
          p = (p == 0) ? nj - 1 : p - 1;
        else
          p = (p + 1 == nj) ? 0 : p + 1;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xhi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, xhi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xlo, acc, 0, 0, 0);
    }
    if (++nfold == kFold) {
      nfold = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) accd[u] += static_cast<double>(acc[u]);
      acc = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) accd[u] += static_cast<double>(acc[u]);

  // store: D rows 4 kgrp + u (output pixel a0 + 4 kgrp + u), column col (image); each output
  // pixel once: rows beyond the fundamental domain [0, F), reflections of pixels on a reflection
  // axis and the mirror of the equator ring are skipped
  const int F = ((ni >> 2) - ci) / 2 + 1;
  if (ch && mr == r) return;
  const int rr = ch ? mr : r;
  const double inv = static_cast<double>(d->inv_sw) / static_cast<double>(sx);
  float* yr = ym + d->rstart[rr];
  const bool add = d->ring_add[rr] != 0;
  const int quarter = ni >> 2;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ao = a0 + 4 * kgrp + u;
    if (ao >= F) continue;
    if (cf && ((2 * ao + ci) % quarter) == 0) continue;
    int P = cf ? (ni - ao - ci + cq * quarter) : (ao + cq * quarter);
    P %= ni;
    if (P < 0) P += ni;
    put(yr + P, accd[u] * inv, add);
  }
}

// ---------------------------------------------------------------- persistent queue kernel
template <int SEG>
// at least two waves per SIMD, so that belt (matrix-core) and cap (VALU) items share a SIMD
__global__ __launch_bounds__(kBlock, 2) void mixed_persistent_kernel(convreal::Slots S,
                                                                  const int2* __restrict__ items,
                                                                  int n_items, int nrep,
                                                                  const unsigned* __restrict__ amax,
                                                                  unsigned* __restrict__ counter,
                                                                  int coef_offset_bytes) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ int s_item;
  __shared__ const convreal::MixedDesc* s_coef_owner;
  _Float16* stage = reinterpret_cast<_Float16*>(lds);
  float4* s_coef = reinterpret_cast<float4*>(lds + coef_offset_bytes);
  if (threadIdx.x == 0) s_coef_owner = nullptr;
  const long long total = static_cast<long long>(n_items) * nrep;
  for (;;) {
    if (threadIdx.x == 0) s_item = static_cast<int>(atomicAdd(counter, 1u));
    __syncthreads();
    const long long gi = s_item;
    const convreal::MixedDesc* owner = s_coef_owner;
    __syncthreads();
    if (gi >= total) break;
    const int2 it = items[gi % n_items];
    const int slot = it.x + static_cast<int>(gi / n_items);
    const int kind = it.y >> 30;
    const int idx = it.y & 0x3fffffff;
    const convreal::MixedDesc* d = S.desc[slot];
    const float sx = map_scale(amax[slot]);
    if (kind == 0) {
      belt_item<SEG>(d, idx, S.x[slot], S.y[slot], sx, stage);
    } else {
      if (owner != d) {
        const float4* coef = reinterpret_cast<const float4*>(d->coef);
        for (int k = threadIdx.x; k < d->nseg; k += kBlock) s_coef[k] = coef[k];
        __syncthreads();
        if (threadIdx.x == 0) s_coef_owner = d;
      }
      const int t = idx * kWaves + (threadIdx.x >> 6);
      if (t < d->n_citems) cap_tile(d, t, S.x[slot], S.y[slot], sx, s_coef);
    }
    __syncthreads();
  }
}

}  // namespace

namespace convreal {

size_t belt_stage_bytes(int seg) {
  return seg == 512 ? static_cast<size_t>(BeltLayout<512>::BYTES) : static_cast<size_t>(BeltLayout<256>::BYTES);
}

// Dynamic LDS of the persistent kernel: the belt stage, then the coefficient table.
size_t persistent_lds_bytes(int seg, int nseg) {
  const size_t coef_off = (belt_stage_bytes(seg) + 15) / 16 * 16;
  return coef_off + sizeof(float4) * static_cast<size_t>(nseg > 0 ? nseg : 1);
}

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

// Launch the prep kernels and the persistent kernel over `nslots` maps whose descriptors are in S.
hipError_t launch_mixed_queue(const conv_real_plan* mark_plan, const Slots& S, int nslots, const int2* items,
                              int n_items, int nrep, unsigned* amax, unsigned* counter, const Tuning& tune,
                              int max_nseg, long long npix_max, long long pairs, hipStream_t st) {
  hipLaunchKernelGGL(zero_state_kernel, dim3(1), dim3(kMaxSlots), 0, st, amax, nslots, counter);
  mark(mark_plan, st, "zero_state_kernel", 0);
  const long long want = (npix_max + 255) / 256;
  const unsigned gx = static_cast<unsigned>(want < 1024 ? want : 1024);
  hipLaunchKernelGGL(prep_kernel, dim3(gx, nslots), dim3(256), 0, st, S, amax);
  mark(mark_plan, st, "prep_kernel", 0);
  if (n_items > 0 && nrep > 0) {
    const size_t coef_off = (belt_stage_bytes(tune.seg) + 15) / 16 * 16;
    const size_t lds = persistent_lds_bytes(tune.seg, max_nseg);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    long long total = static_cast<long long>(n_items) * nrep;
    long long grid = static_cast<long long>(ncu) * (tune.wg_per_cu > 0 ? tune.wg_per_cu : 2);
    if (grid > total) grid = total;
    if (tune.seg == 512)
      hipLaunchKernelGGL(mixed_persistent_kernel<512>, dim3(static_cast<unsigned>(grid)), dim3(kBlock), lds, st, S,
                         items, n_items, nrep, amax, counter, static_cast<int>(coef_off));
    else
      hipLaunchKernelGGL(mixed_persistent_kernel<256>, dim3(static_cast<unsigned>(grid)), dim3(kBlock), lds, st, S,
                         items, n_items, nrep, amax, counter, static_cast<int>(coef_off));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mark(mark_plan, st, "mixed_persistent_kernel", pairs);
  }
  return hipGetLastError();
}

hipError_t set_lds_limits(int nseg) {
  // enough for the larger belt stage and this plan's coefficient table, within the device limit
  int dev = 0, optin = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
  if (e != hipSuccess || optin <= 0) optin = 65536;
  const size_t need = persistent_lds_bytes(512, nseg);
  if (need > static_cast<size_t>(optin)) return hipErrorInvalidValue;
  const int bytes = static_cast<int>(need);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mixed_persistent_kernel<256>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&mixed_persistent_kernel<512>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_mixed(const conv_real_plan* p, const float* x, float* y, int nmaps, hipStream_t st) {
  for (int m0 = 0; m0 < nmaps; m0 += kMaxSlots) {
    const int nm = nmaps - m0 < kMaxSlots ? nmaps - m0 : kMaxSlots;
    Slots S;
    for (int k = 0; k < nm; ++k) {
      S.desc[k] = p->d_desc;
      S.x[k] = x + static_cast<size_t>(m0 + k) * p->npix;
      S.y[k] = y + static_cast<size_t>(m0 + k) * p->npix;
    }
    hipError_t e = launch_mixed_queue(p, S, nm, p->d_items, p->n_items, nm, p->d_amax, p->d_counter, p->tune,
                                      p->cap_nseg, p->npix, p->pairs * nm, st);
    if (e != hipSuccess) return e;
    if (!p->cap_mode) {
      // table too large for the LDS coefficient form: cap-touching pairs per pair in FP64, added to
      // the belt result
      e = launch_remainder(p, x + static_cast<size_t>(m0) * p->npix, y + static_cast<size_t>(m0) * p->npix, nm, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace convreal
