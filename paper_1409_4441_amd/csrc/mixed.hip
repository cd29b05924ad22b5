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
// the group's fundamental domain (32 from a weight store: two blocks that share each step's inputs)
// and, per neighbour ring, computes D[16 pixels][16 images] += W[16][K] X[K][16] per block. W is either evaluated on the fly: integer azimuth numerator -> alpha = dphi/2,
// sin^2 alpha by a polynomial, d^2 = A + B sin^2 alpha, all in FP64 (the oscillating kernel is
// sensitive to d at the 1e-8 level near the cut), then the 4-point interpolant in cubic form from
// an LDS table of per-segment FP32 coefficients; or it is streamed from a weight store built once
// per plan (the same weights, already split, in groups of 4 inputs that meet a row's window), with
// the loads of several steps in flight. Images that coincide are stored once.
//
// Precision of both: weights and map values are split into FP16 pairs, w s_w = w_hi + w_lo,
// x s_x = x_hi + x_lo (powers of two), and each block is w_hi x_hi + w_lo x_hi + w_hi x_lo
// accumulated in FP32 by v_mfma_f32_16x16x32_f16; the dropped w_lo x_lo and the split residues are
// ~2^-22 relative. FP32 accumulators are folded into FP64 every few ring pairs.
//
// Scheduling: one workgroup of 4 waves repeatedly takes the next item of a cost-sorted queue: a
// belt item (one band x one segment of output pixels, MFMA-bound) or a cap item (4 tiles, one per
// wave, VALU-bound by weight evaluation or bound by the store's stream), so that both kinds share
// every CU. Rows that receive a
// belt and a cap-pair contribution (belt rings near the belt edge) are zeroed beforehand and get
// exactly two atomic adds, which is order-independent: fl(0 + a + b) = fl(0 + b + a).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kFold = 4;   // ring pairs per FP32 -> FP64 fold
constexpr int kNKMax = convreal::kBeltBlockChunks;  // largest K-chunk count of a belt weight block

// ---------------------------------------------------------------- shared helpers
using convreal::buffer_resource;
using convreal::kNoLoad;
using convreal::ldu;
using convreal::ldu_record;

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
__global__ void zero_state_kernel(unsigned* amax, int n, unsigned* counter, int ncounters) {
  const int t = threadIdx.x;
  if (t < n) amax[t] = 0u;
  if (t < ncounters) counter[t] = 0u;
}

// per slot: |x| maximum (atomicMax on the bit pattern: non-negative floats order like their bits),
// and (zero_rows) zero of the rows that will receive two atomic adds. 16-byte loads where the map is
// 16-byte aligned (N_pix = 12 N^2 is a multiple of 4), a plain loop otherwise.
__global__ __launch_bounds__(256) void prep_kernel(convreal::Slots S, unsigned* __restrict__ amax, int zero_rows) {
  const int slot = blockIdx.y;
  const convreal::MixedDesc* d = S.desc[slot];
  const long long npix = d->npix;
  const float* x = S.x[slot];
  float* y = S.y[slot];
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  const long long t0 = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  float v = 0.0f;
  if ((reinterpret_cast<unsigned long long>(x) & 15) == 0) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const long long n4 = npix >> 2;
    for (long long i = t0; i < n4; i += stride) {
      const float4 q = x4[i];
      v = fmaxf(v, fmaxf(fmaxf(fabsf(q.x), fabsf(q.y)), fmaxf(fabsf(q.z), fabsf(q.w))));
    }
    for (long long i = (n4 << 2) + t0; i < npix; i += stride) v = fmaxf(v, fabsf(x[i]));
  } else {
    for (long long i = t0; i < npix; i += stride) v = fmaxf(v, fabsf(x[i]));
  }
  // one atomic per workgroup: atomics on one address serialise
  __shared__ float wmax[256 / 64];
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = wmax[0];
    for (int k = 1; k < 256 / 64; ++k) m = fmaxf(m, wmax[k]);
    atomicMax(amax + slot, __float_as_uint(m));
  }
  for (int z = 0; z < 2 && zero_rows; ++z) {
    const long long z0 = d->zero_lo[z], z1 = d->zero_hi[z];
    for (long long i = z0 + t0; i < z1; i += stride) y[i] = 0.0f;
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
// Belt staging, software-pipelined AHEAD input rings ahead: while the matrix cores work on ring j,
// every thread holds its share of the input windows (PX pixels) and of the weight fragments (2 half8)
// of the next rings in registers; after the products ring j+1 goes to the other LDS buffer.
template <int SEG>
struct BeltPrefetch {
  static constexpr int PX = (SEG + 32 * kNKMax + kBlock - 1) / kBlock;
  float x[PX];
  half8 w[2];
  int len;     // window pixels
  int nwv;     // weight half8 of the ring (128 per K-chunk)

  // Every thread issues the same PX + 2 loads whatever the window's length (elements past it read
  // the window's last pixel or the first fragment and are not stored), so that the compiler can
  // count the loads in flight and wait for the oldest ring only.
  __device__ __forceinline__ void load(const float* __restrict__ xj, int start_px, int len_, int ring_n,
                                       const half8* __restrict__ wsrc, int nwv_) {
    len = len_;
    nwv = nwv_;
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int u = min(static_cast<int>(threadIdx.x) + i * kBlock, len - 1);
      int p = start_px + u;   // start_px > -ring_n and the window is shorter than the ring
      p = p < 0 ? p + ring_n : p;
      p = p >= ring_n ? p - ring_n : p;
      x[i] = xj[p];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int v = static_cast<int>(threadIdx.x) + i * kBlock;
      w[i] = wsrc[v < nwv ? v : 0];
    }
  }

  // 8 copies of the window shifted by one pixel, split into FP16 pairs; weights as they are
  __device__ __forceinline__ void store(_Float16* __restrict__ S, half8* __restrict__ W, float sx) const {
    using BL = BeltLayout<SEG>;
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int u = threadIdx.x + i * kBlock;
      if (u < len) {
        const float xs = x[i] * sx;
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
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int v = threadIdx.x + i * kBlock;
      if (v < nwv) W[v] = w[i];
    }
  }
};

template <int SEG, int AHEAD>
__device__ __forceinline__ void belt_item(const convreal::MixedDesc* __restrict__ d, int idx, const float* __restrict__ xm,
                          float* __restrict__ ym, float sx, _Float16* __restrict__ S) {
  using BL = BeltLayout<SEG>;
  constexpr int NB = SEG / (16 * kWaves);  // 16-pixel blocks per wave
  half8* Wbuf = reinterpret_cast<half8*>(S + 2 * BL::BUF);   // 2 x kNKMax x 128 weight fragments
  const int ring_n = ldu(d->ring_n);
  const int nsegs = (ring_n + SEG - 1) / SEG;
  const int band = idx / nsegs;
  const int seg = idx % nsegs;
  const int a0 = seg * SEG;
  const int nj = ldu(d->band_nj[band]);
  const int woff = ldu(d->band_woff[band]);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15;
  const int g = lane >> 4;
  const int cpy = n & 7;
  const int lane_off = cpy * BL::CS + 16 * (NB * wave) + (n - cpy) + 8 * g;
  const half8* wt = reinterpret_cast<const half8*>(ldu(d->wt));
  const long long* rstart = ldu(d->rstart);
  const int* blk_mlo = ldu(d->blk_mlo);
  const int* blk_j = ldu(d->blk_j);
  const int* blk_nk = ldu(d->blk_nk);
  const int* blk_koff = ldu(d->blk_koff);

  floatx4 acc[NB];
  double accd[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) accd[b][r] = 0.0;
  }

  // Ring r's window and weights travel through register slot r % AHEAD: at iteration jj the
  // loads of ring jj + AHEAD are issued before the products of ring jj, and ring jj + 1 goes to
  // LDS after them, so a ring's loads have AHEAD - 1 rings of work to arrive. The loop is
  // unrolled by AHEAD so that the slots are registers.
  BeltPrefetch<SEG> pf[AHEAD];
  auto load_ring = [&](int jj, BeltPrefetch<SEG>& slot) {
    const int nk1 = ldu(blk_nk[woff + jj]);
    slot.load(xm + ldu(rstart[ldu(blk_j[woff + jj])]), a0 + ldu(blk_mlo[woff + jj]), SEG + 32 * nk1, ring_n,
              wt + static_cast<long long>(ldu(blk_koff[woff + jj])) * 128, nk1 * 128);
  };
  load_ring(0, pf[0]);
  pf[0].store(S, Wbuf, sx);
  // rings past the band's last reload that one (not stored): the same loads on every path
#pragma unroll
  for (int u = 1; u < AHEAD; ++u) load_ring(min(u, nj - 1), pf[u]);
  __syncthreads();
  for (int jb = 0; jb < nj; jb += AHEAD) {
#pragma unroll
    for (int u = 0; u < AHEAD; ++u) {
      const int jj = jb + u;
      if (jj >= nj) break;
      const int buf = jj & 1;
      load_ring(min(jj + AHEAD, nj - 1), pf[u]);
      const int nk = ldu(blk_nk[woff + jj]);
      const half8* wblk = Wbuf + buf * (kNKMax * 128);
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
      // the other buffers were last read in ring jj - 1, before the previous barrier
      if (jj + 1 < nj)
        pf[(u + 1) % AHEAD].store(S + (buf ^ 1) * BL::BUF, Wbuf + (buf ^ 1) * (kNKMax * 128), sx);
      __syncthreads();
    }
  }

  const double inv = static_cast<double>(ldu(d->inv_sw)) / static_cast<double>(sx);
  const int belt_lo = ldu(d->belt_lo), belt_hi = ldu(d->belt_hi);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int px = a0 + 16 * (NB * wave + b) + n;
    if (px >= ring_n) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ring = belt_lo + 16 * band + 4 * g + r;
      if (ring <= belt_hi) put(ym + rstart[ring] + px, accd[b][r] * inv, ldu(d->ring_add)[ring] != 0);
    }
  }
}

// ---------------------------------------------------------------- cap item
// sin^2(al) / al^2 as a polynomial in t = al^2 (al = half the azimuth difference). Each ring pair
// scales the coefficients by B_ij, so that d^2 = A_ij + t * poly(t).
//   short form, |al| <= 0.2 (t <= 0.04): relative error below 3e-12
//   long form, |al| <= 1.61 (t <= 2.6): relative error below 1e-11
// Either error moves d by far less than the 1e-7-pixel slack of the pair windows.
constexpr double kShortAlpha = 0.2;
constexpr double kSinShort[4] = {0.9999999999971675, -0.33333333107313623, 0.04444416233415409,
                                 -0.0031633255222186167};
constexpr double kSinLong[8] = {0.9999999999970449,     -0.3333333332512937,     0.04444444389087041,
                                -0.0031746016082493094, 0.00014109120522641625,  -4.273732374386684e-06,
                                9.31392155360743e-08,   -1.366547170656072e-09};

// Omega s_w Ktilde(d) is evaluated from q = (d / h)^2, the squared chord in units of the table
// spacing (0 beyond the cut q > qcut). t = d / h comes from a single-precision reciprocal square
// root refined by one Newton step in FP64 (relative error ~1e-14); segment floor(t), local
// coordinate frac(t). Lanes beyond the cut clamp the segment so that they stay inside the
// coefficient table; inside the cut t <= (n_tab - 3)(1 + 1e-9), so the clamp never moves a kept pair.
__device__ __forceinline__ void locate(double q, int seg_max, int& sg, float& f) {
  const float y0 = __builtin_amdgcn_rsqf(fmaxf(static_cast<float>(q), 1e-30f));
  const double y = static_cast<double>(y0);
  const double t0 = q * y;
  const double r = fma(-t0, t0, q);
  const double t = fma(r, 0.5 * y, t0);
  sg = min(static_cast<int>(t), seg_max);
  f = static_cast<float>(__builtin_amdgcn_fract(t));
}

// the E weights of one lane's A-operand entries, in phases (all chords, all table reads, all
// cubics) so that the LDS reads are issued together and their latency overlaps
template <int E>
__device__ __forceinline__ void weights_of(const double (&q)[E], double qcut, int seg_max,
                                           const float4* __restrict__ s_coef, float (&w)[E]) {
  int sg[E];
  float f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) locate(q[e], seg_max, sg[e], f[e]);
  float4 c[E];
#pragma unroll
  for (int e = 0; e < E; ++e) c[e] = s_coef[sg[e]];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const float v = fmaf(fmaf(fmaf(c[e].w, f[e], c[e].z), f[e], c[e].y), f[e], c[e].x);
    w[e] = q[e] <= qcut ? v : 0.0f;
  }
}

// v mod n for |v| < 2^24, n > 0 (reciprocal-based quotient, corrected by one step either way)
__device__ __forceinline__ int mod_any(int v, int n, float rcp_n) {
  const int q = static_cast<int>(floorf(static_cast<float>(v) * rcp_n));
  int m = v - q * n;
  m = m < 0 ? m + n : m;
  return m >= n ? m - n : m;
}

template <int E, typename HV>
__device__ __forceinline__ void split_fp16(const float (&v)[E], HV& hi, HV& lo) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const _Float16 h = static_cast<_Float16>(v[e]);
    hi[e] = h;
    lo[e] = static_cast<_Float16>(v[e] - static_cast<float>(h));
  }
}

// B operand of one K-step: image col of inputs b = bA .. bA + E - 1, i.e. pixels pofs + dir * b
// (mod nj) of the lane's ring, scaled by sx. Lanes read E consecutive pixels (reversed for reflected
// images); the wave takes the no-wrap branch when no lane crosses the ring's start. Needs nj >= E.
template <int E, typename HV>
__device__ __forceinline__ void load_inputs(const float* __restrict__ xj, int pofs, int dir, int bA, int nj,
                                            float rcp_n, float sx, HV& xhi, HV& xlo) {
  const int p0 = mod_any(pofs + dir * bA, nj, rcp_n);
  const int s = dir > 0 ? p0 : p0 - (E - 1);   // lowest pixel index read by this lane
  float v[E];
  if (__all(s >= 0 && s + E - 1 < nj)) {
    const float* xp = xj + s;
    float L[E];
#pragma unroll
    for (int e = 0; e < E; ++e) L[e] = xp[e];
    // forward lanes keep the order, reflected lanes reverse it (a bitwise select per element)
    const unsigned fwd = dir > 0 ? 0xffffffffu : 0u;
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = __uint_as_float((fwd & __float_as_uint(L[e])) | (~fwd & __float_as_uint(L[E - 1 - e]))) * sx;
  } else {
    int ix[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int idx = p0 + dir * e;
      idx = idx < 0 ? idx + nj : idx;
      ix[e] = idx >= nj ? idx - nj : idx;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xj[ix[e]];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] *= sx;
  }
  split_fp16<E>(v, xhi, xlo);
}

// window [lo, hi] of ring j for the output pixel with azimuth numerator u: the per-pair path's rule
// (centre (u n_j - c_j n_i) / 2 n_i, half-width hw plus 1e-7 pixel; a whole ring: n_j pixels).
// inv_2ni = 1 / (2 n_i): the centre is off by an ulp at most, far inside the 1e-7-pixel slack, and
// every caller (fill, apply, on-the-fly path) forms it the same way.
__device__ __forceinline__ void row_window(const convreal::CapPair& P, int u, int ni, double inv_2ni, int& lo,
                                           int& hi) {
  const double bc = static_cast<double>(u * P.nj - P.cj * ni) * inv_2ni;
  if (P.whole) {
    lo = static_cast<int>(floor(bc)) - P.nj / 2;
    hi = lo + P.nj - 1;
  } else {
    lo = static_cast<int>(ceil(bc - P.hw - 1e-7));
    hi = static_cast<int>(floor(bc + P.hw + 1e-7));
  }
}

// exclusive prefix sum of v over each 16-lane row of the wave (DPP row shifts: lanes without a
// source in their row read 0); total: the sum over the first row (callers pass values that depend
// on the lane's row of the tile only, so every 16-lane row agrees)
__device__ __forceinline__ int scan16(int v, int& total) {
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
  total = __builtin_amdgcn_readlane(x, 15);
  return x - v;
}

// union [b0, bend] of the windows of ring j over a tile's 16 rows (the centres increase with a, so
// the first row gives the start and the last row the end)
__device__ __forceinline__ void tile_union(const convreal::CapPair& P, int u_first, int u_last, int ni,
                                           double inv_2ni, int& b0, int& bend) {
  const double bc0 = static_cast<double>(u_first * P.nj - P.cj * ni) * inv_2ni;
  const double bc1 = static_cast<double>(u_last * P.nj - P.cj * ni) * inv_2ni;
  if (P.whole) {
    b0 = static_cast<int>(floor(bc0)) - P.nj / 2;
    bend = static_cast<int>(floor(bc1)) - P.nj / 2 + P.nj - 1;
  } else {
    b0 = static_cast<int>(ceil(bc0 - P.hw - 1e-7));
    bend = static_cast<int>(floor(bc1 + P.hw + 1e-7));
  }
}

// long-form weights of output pixel u and inputs bA .. bA + E - 1 (any ring pair): numerator reduced
// to [-M, M], degree-7 sin^2 polynomial, q = d^2 / h^2
struct LongForm {
  double Ah;
  double cl[8];
  double Md, twoM, inv_twoM, two_ni, scale;
  __device__ __forceinline__ LongForm(const convreal::CapPair& P, int ni, double ih2) {
    const double Bh = P.B * ih2;
    Ah = P.A * ih2;
#pragma unroll
    for (int u = 0; u < 8; ++u) cl[u] = Bh * kSinLong[u];
    Md = static_cast<double>(ni) * static_cast<double>(P.nj);
    twoM = 2.0 * Md;
    inv_twoM = 1.0 / twoM;
    two_ni = 2.0 * static_cast<double>(ni);
    scale = P.scale;
  }
  template <int E>
  __device__ __forceinline__ void q(int u, int bA, int ni, int nj, int cj, double (&qv)[E]) const {
    double nd = static_cast<double>(u * nj - (2 * bA + cj) * ni);
    nd = fma(-rint(nd * inv_twoM), twoM, nd);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double ne = nd - static_cast<double>(e) * two_ni;
      ne = ne < -Md ? ne + twoM : ne;
      ne = ne < -Md ? ne + twoM : ne;
      const double al = ne * scale;
      const double tq = al * al;
      double bp = cl[7];
#pragma unroll
      for (int k = 6; k >= 0; --k) bp = fma(bp, tq, cl[k]);
      qv[e] = fma(tq, bp, Ah);
    }
  }
};

// one short-form K-step of E inputs per lane (E = 8: 32 inputs on v_mfma_f32_16x16x32_f16; E = 4:
// 16 inputs on v_mfma_f32_16x16x16_f16, for the last step of a window)
template <int E>
__device__ __forceinline__ void short_step(floatx4& acc, int bA, int u_row, int ni, int nj, int cj, double scale,
                                           double delta, double Ah, double c0, double c1, double c2, double c3,
                                           double qcut, int seg_max, const float4* __restrict__ s_coef,
                                           const float* __restrict__ xj, int pofs, int dir, float rcp_n, float sx) {
  using HV = typename std::conditional<E == 8, half8, half4>::type;
  HV xhi, xlo;
  load_inputs<E>(xj, pofs, dir, bA, nj, rcp_n, sx, xhi, xlo);
  double al = static_cast<double>(u_row * nj - (2 * bA + cj) * ni) * scale;
  double qv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double tq = al * al;
    const double bp = fma(fma(fma(c3, tq, c2), tq, c1), tq, c0);
    qv[e] = fma(tq, bp, Ah);
    al -= delta;
  }
  float w[E];
  weights_of<E>(qv, qcut, seg_max, s_coef, w);
  HV whi, wlo;
  split_fp16<E>(w, whi, wlo);
  if constexpr (E == 8) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, xhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xlo, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(whi, xhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(wlo, xhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(whi, xlo, acc, 0, 0, 0);
  }
}

// What one lane of a cap tile is: tile t covers output pixels a0 .. a0 + rows - 1 of the fundamental
// domain [0, F) of north-half ring r, in blocks of 16. A operand: row = output pixel a0 + 16 blk + row
// of block blk, k-group kgrp; B operand and result: column col = image (hemisphere ch, reflection cf,
// quarter turn cq).
struct CapLane {
  int r, a0, ni, ci, F;
  int row, kgrp, col, ch, cf, cq, dir;
  int u_row, u_first, u_last;   // azimuth numerators of the lane's row in block 0, the tile's first and last row
  double inv_2ni;
  __device__ __forceinline__ CapLane(const convreal::MixedDesc* __restrict__ d, int t, int rows) {
    r = ldu(ldu(d->citem_ring)[t]);
    a0 = ldu(ldu(d->citem_a0)[t]);
    ni = ldu(ldu(d->rn)[r]);
    ci = ldu(ldu(d->rc)[r]);
    F = ((ni >> 2) - ci) / 2 + 1;
    const int lane = threadIdx.x & 63;
    row = lane & 15;
    kgrp = lane >> 4;
    col = lane & 15;
    ch = col >> 3;
    cf = (col >> 2) & 1;
    cq = col & 3;
    dir = cf ? -1 : 1;
    u_row = 2 * (a0 + row) + ci;
    u_first = 2 * a0 + ci;
    u_last = 2 * (a0 + rows - 1) + ci;
    inv_2ni = 1.0 / (2.0 * ni);
  }
  // first pixel of the lane's image of pixel 0 of ring j, relative to the ring (or its mirror)
  __device__ __forceinline__ int pofs(int nj, int cj) const {
    return cf ? (nj - cj + cq * (nj >> 2)) : cq * (nj >> 2);
  }
};

// ---------------------------------------------------------------- cap weight store
// Store tiles are kStoreBlocks blocks of 16 rows (one wave each). A row of the tile keeps, per
// cap-touching ring pair, the groups of 4 inputs that meet its window [lo, hi] (group g covers inputs
// b0 + 4g .. b0 + 4g + 3 of ring j, b0: start of the tile's union window), 16 bytes each: the 4
// weights x s_w rounded to FP16 (hi), then the FP16 residues (lo), zeros inside a group outside the
// window. Layout, per store tile: per ring pair (in list order), per 32-input step and per half of
// the step (the two load instructions of the apply, see the K order below), the stored groups of
// the lanes in lane order. Every load instruction of the apply thus reads one contiguous run of at
// most 1 KB. Nothing about the layout is stored besides the first group of every tile: the apply
// recomputes the same windows, and a ballot of the lanes whose group is stored, counted below each
// lane, gives every lane its offset. Weights are read through a buffer resource over the tile's
// block: a lane whose group is not stored gives an offset past the resource's range, which the
// hardware answers with zeros without a memory access, so every load instruction is issued
// unconditionally (and lands in the register that the matrix cores read later) while only stored
// groups move through the caches; addresses are 32-bit offsets from the tile's block and from the
// map. The blocks of a tile share each step's inputs: loaded, reversed, scaled and split once.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

constexpr int kStoreBlocks = convreal::kStoreBlocks;
constexpr int kStoreRows = 16 * kStoreBlocks;

// K order of a step: lane kgrp holds inputs 4 kgrp + [0, 4) (half 0) and 16 + 4 kgrp + [0, 4)
// (half 1) of the step's 32, i.e. weight groups 8q + kgrp and 8q + 4 + kgrp, so that each load
// instruction reads 64 contiguous bytes per row of weights and per image of inputs.
struct StorePair {
  int glo[kStoreBlocks];     // the lane's row stores groups glo .. glo + gn - 1 (gn = 0: none)
  int gn[kStoreBlocks];
  unsigned xofs;             // map index of the lowest pixel of the lane's step-0 half-0 inputs
  int nk;                    // 32-input steps over the union window (uniform)
};

// One step's operands as loaded (software-pipelined: the loads of later steps are in flight while
// the matrix cores work on this one).
struct StoreStep {
  u32x4 wa[kStoreBlocks], wb[kStoreBlocks];   // weight groups of each block's row, both halves
  float v[8];     // the lane's inputs, each half in memory order from its lowest pixel
  int blocks;     // bit b: block b has stored groups in this step (uniform)
  bool live;      // a step of the tile (false: the sequence has ended; the loads are not used)
  bool last;      // last step of its ring pair
};

// number of lanes below this one whose bit is set in the wave mask m
__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(m), 0u));
}

// Byte offsets in the tile's block of the lane's two groups of step q of block b (kNoLoad where not
// stored); pos: the step's first group, advanced past the step's groups. Uniform control flow only
// (a ballot).
__device__ __forceinline__ bool step_offsets(const StorePair& S, int b, int q, int kgrp, int& pos, unsigned& oa,
                                             unsigned& ob) {
  const bool fa = static_cast<unsigned>(8 * q + kgrp - S.glo[b]) < static_cast<unsigned>(S.gn[b]);
  const bool fb = static_cast<unsigned>(8 * q + 4 + kgrp - S.glo[b]) < static_cast<unsigned>(S.gn[b]);
  const unsigned long long ma = __builtin_amdgcn_ballot_w64(fa);
  const unsigned long long mb = __builtin_amdgcn_ballot_w64(fb);
  const int na = __builtin_popcountll(ma);
  unsigned ra = static_cast<unsigned>(pos) + lanes_below(ma);
  unsigned rb = static_cast<unsigned>(pos + na) + lanes_below(mb);
  // counted in every lane: an empty asm keeps the compiler from moving the counts into
  // exec-masked branches of their own (selects are cheaper than the branching)
  asm volatile("" : "+v"(ra), "+v"(rb));
  oa = fa ? ra * 16u : kNoLoad;
  ob = fb ? rb * 16u : kNoLoad;
  pos += na + __builtin_popcountll(mb);
  return (ma | mb) != 0ull;
}

__device__ __forceinline__ u32x4 load_group(__amdgpu_buffer_rsrc_t tile, unsigned off) {
  return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(tile, off, 0, 0));
}

// Ring pair P over a store tile: the union window [b0, bend] of its rows (steps of 32 inputs from
// b0), each lane's stored groups per block (S.glo, S.gn) and the pair's stored group count. The
// fill, the count and both apply paths take the layout from here.
struct PairWin {
  int b0, nk, stored;
};
__device__ __forceinline__ PairWin pair_windows(const convreal::CapPair& P, const CapLane& L, StorePair& S,
                                                int (&lo)[kStoreBlocks], int (&hi)[kStoreBlocks]) {
  PairWin w;
  int bend;
  tile_union(P, L.u_first, L.u_last, L.ni, L.inv_2ni, w.b0, bend);
  w.stored = 0;
  w.nk = bend < w.b0 ? 0 : (bend - w.b0 + 32) >> 5;
  if (w.nk == 0) return w;
#pragma unroll
  for (int b = 0; b < kStoreBlocks; ++b) {
    row_window(P, L.u_row + 32 * b, L.ni, L.inv_2ni, lo[b], hi[b]);
    const bool in = L.a0 + 16 * b + L.row < L.F && hi[b] >= lo[b];
    S.glo[b] = (lo[b] - w.b0) >> 2;
    S.gn[b] = in ? ((hi[b] - w.b0) >> 2) - S.glo[b] + 1 : 0;
    int total;
    scan16(S.gn[b], total);
    w.stored += total;
  }
  return w;
}

// The lane's inputs of the pair over all its steps lie in b0 + 4 kgrp + [0, span), pixels
// pofs + dir b (mod nj) of ring j (half h of step q starts at b0 + 4 kgrp + 32 q + 16 h). Returns
// whether they cross the ring's start; low: the lowest pixel (mod nj).
__device__ __forceinline__ bool pair_wraps(const convreal::CapPair& P, const CapLane& L, int b0, int nk, int& low) {
  const int nj = P.nj;
  const int pofs = L.pofs(nj, P.cj);
  const float rcp_n = __builtin_amdgcn_rcpf(static_cast<float>(nj));
  const int first = b0 + 4 * L.kgrp, span = 32 * (nk - 1) + 20;
  low = mod_any(L.dir > 0 ? pofs + first : pofs - (first + span - 1), nj, rcp_n);
  return low + span > nj;
}

// w_hi x_hi + w_lo x_hi + w_hi x_lo of one block on the step's split inputs
__device__ __forceinline__ void block_mfma(floatx4& acc, const half8& xhi, const half8& xlo, const u32x4& wa,
                                           const u32x4& wb) {
  const half8 whi = __builtin_bit_cast(half8, u32x4{wa.x, wa.y, wb.x, wb.y});
  const half8 wlo = __builtin_bit_cast(half8, u32x4{wa.z, wa.w, wb.z, wb.w});
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, xhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xlo, acc, 0, 0, 0);
}

// FP32 accumulators of the blocks, folded into FP64 every kFold ring pairs
struct CapAcc {
  floatx4 acc[kStoreBlocks];
  double accd[kStoreBlocks][4];
  int nfold;
  __device__ __forceinline__ void pair_done() {
    if (++nfold == kFold) {
      nfold = 0;
#pragma unroll
      for (int b = 0; b < kStoreBlocks; ++b) {
#pragma unroll
        for (int u = 0; u < 4; ++u) accd[b][u] += static_cast<double>(acc[b][u]);
        acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
};

__device__ __forceinline__ void store_compute(CapAcc& A, const StoreStep& R, int dir, float sx) {
  // forward lanes keep the memory order, reflected lanes reverse each half (a bitwise select per
  // element)
  const unsigned fwd = dir > 0 ? 0xffffffffu : 0u;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int r = (e & 4) + 3 - (e & 3);
    v[e] = __uint_as_float((fwd & __float_as_uint(R.v[e])) | (~fwd & __float_as_uint(R.v[r]))) * sx;
  }
  half8 xhi, xlo;
  split_fp16<8>(v, xhi, xlo);
#pragma unroll
  for (int b = 0; b < kStoreBlocks; ++b)
    if (R.blocks & (1 << b)) block_mfma(A.acc[b], xhi, xlo, R.wa[b], R.wb[b]);
}

// The tile's steps, ring pair after ring pair, as one sequence.
struct StoreIter {
  __amdgpu_buffer_rsrc_t tile;   // over the tile's block
  convreal::CapPair Pn;        // record kk, loaded one pair ahead of its use
  int kk, k1;                  // ring pair indices (below 2^31: at most (4 N)^2 ring pairs)
  int pos;                     // next step's first group, from the tile's block
  int q;
  StorePair S;

  // Set up ring pair P. Returns the pair's step count, 0 if it has no stored weight for the tile.
  // Tiles where some pair's inputs wrap around ring j never come here.
  __device__ __forceinline__ int setup(const convreal::CapPair& P, const CapLane& L) {
    int lo[kStoreBlocks], hi[kStoreBlocks];
    const PairWin w = pair_windows(P, L, S, lo, hi);
    if (w.stored == 0) return 0;
    int low;
    (void)pair_wraps(P, L, w.b0, w.nk, low);
    const long long xoff = L.ch ? P.xoff_m : P.xoff;
    S.xofs = static_cast<unsigned>(xoff + (L.dir > 0 ? low : low + 32 * (w.nk - 1) + 16));
    return w.nk;
  }

  // Load the next step into R (R.live = false once the tile has no step left). Every call issues
  // the same loads, an ended sequence reading no weight (zeros) and the map's first pixels, so that
  // the compiler can count the loads in flight and wait for the oldest only.
  __device__ __forceinline__ void next(const convreal::CapPair* __restrict__ cpair, const CapLane& L,
                                       const float* __restrict__ xm, StoreStep& R) {
    bool ok = true;
    while (q >= S.nk) {
      if (kk >= k1) {
        ok = false;
        break;
      }
      const convreal::CapPair P = Pn;
      ++kk;
      if (kk < k1) Pn = ldu_record(cpair[kk]);
      q = 0;
      S.nk = setup(P, L);
    }
    unsigned oa[kStoreBlocks], ob[kStoreBlocks], xa = 0, xc = 0;
    int blocks = 0;
    bool last = false;
#pragma unroll
    for (int b = 0; b < kStoreBlocks; ++b) oa[b] = ob[b] = kNoLoad;
    if (ok) {
#pragma unroll
      for (int b = 0; b < kStoreBlocks; ++b)
        if (step_offsets(S, b, q, L.kgrp, pos, oa[b], ob[b])) blocks |= 1 << b;
      xa = S.xofs + static_cast<unsigned>(L.dir * 32 * q);
      xc = xa + static_cast<unsigned>(L.dir * 16);
      ++q;
      last = q >= S.nk;
    }
#pragma unroll
    for (int b = 0; b < kStoreBlocks; ++b) {
      R.wa[b] = load_group(tile, oa[b]);
      R.wb[b] = load_group(tile, ob[b]);
    }
    // 32-bit byte offsets (maps hold at most 12 * 8192^2 pixels) on the map's base address
    const float* x0 = reinterpret_cast<const float*>(reinterpret_cast<const unsigned char*>(xm) + xa * 4u);
    const float* x1 = reinterpret_cast<const float*>(reinterpret_cast<const unsigned char*>(xm) + xc * 4u);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      R.v[e] = x0[e];
      R.v[4 + e] = x1[e];
    }
    R.blocks = blocks;
    R.live = ok;
    R.last = last;
  }
};

constexpr int kStoreSlots = 3;   // steps in flight per wave

// A store tile where some ring pair's inputs wrap around ring j for some lane (the first tile of a
// ring, rings of a few pixels near the poles): every pair at once, step after step, the inputs
// gathered pixel by pixel (ring indices mod n_j).
__device__ __forceinline__ void cap_rows_wrap(__amdgpu_buffer_rsrc_t tile, long long k0, long long k1,
                                              const convreal::CapPair* __restrict__ cpair, const CapLane& L,
                                              const float* __restrict__ xm, float sx, CapAcc& A) {
  int pos = 0;
  for (long long kk = k0; kk < k1; ++kk) {
    const convreal::CapPair P = ldu_record(cpair[kk]);
    StorePair S;
    int lo[kStoreBlocks], hi[kStoreBlocks];
    const PairWin w = pair_windows(P, L, S, lo, hi);
    if (w.stored == 0) continue;
    const int nj = P.nj;
    const float* xj = xm + (L.ch ? P.xoff_m : P.xoff);
    const int pofs = L.pofs(nj, P.cj);
    const float rcp_n = __builtin_amdgcn_rcpf(static_cast<float>(nj));
    const int first = w.b0 + 4 * L.kgrp;
    for (int q = 0; q < w.nk; ++q) {
      // indices first, then all loads, then the scaling; the scheduling barrier keeps the compiler
      // from pairing each load with its use, so that the 8 loads are in flight together
      int ix[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) ix[e] = mod_any(pofs + L.dir * (first + 32 * q + 16 * (e >> 2) + (e & 3)), nj, rcp_n);
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = xj[ix[e]];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] *= sx;
      half8 xhi, xlo;
      split_fp16<8>(v, xhi, xlo);
#pragma unroll
      for (int b = 0; b < kStoreBlocks; ++b) {
        unsigned oa, ob;
        if (!step_offsets(S, b, q, L.kgrp, pos, oa, ob)) continue;
        const u32x4 wa = load_group(tile, oa);
        const u32x4 wb = load_group(tile, ob);
        block_mfma(A.acc[b], xhi, xlo, wa, wb);
      }
    }
    A.pair_done();
  }
}

// all cap-touching pairs of a store tile, all blocks
__device__ __forceinline__ void cap_rows_store(const convreal::MixedDesc* __restrict__ d, int t, const CapLane& L,
                                               const float* __restrict__ xm, float sx,
                                               double (&accd)[kStoreBlocks][4]) {
  // the tile's first group, and whether some pair wraps (set by the count pass)
  const long long wo = ldu(ldu(d->wtile_off)[t]);
  const __amdgpu_buffer_rsrc_t tile =
      buffer_resource(reinterpret_cast<const unsigned char*>(ldu(d->wstore)) + 16 * (wo & convreal::kTileOffsetMask));
  const long long k0 = ldu(ldu(d->rest_off)[L.r]);
  const long long k1 = ldu(ldu(d->rest_off)[L.r + 1]);
  const convreal::CapPair* cpair = ldu(d->cpair);
  CapAcc A;
#pragma unroll
  for (int b = 0; b < kStoreBlocks; ++b) {
    A.acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 4; ++u) A.accd[b][u] = 0.0;
  }
  A.nfold = 0;
  if (wo & convreal::kTileWraps) {
    cap_rows_wrap(tile, k0, k1, cpair, L, xm, sx, A);
  } else {
    StoreIter it;
    it.tile = tile;
    it.kk = static_cast<int>(k0);
    it.k1 = static_cast<int>(k1);
    it.pos = 0;
    it.q = 0;
    it.S.nk = 0;
    if (it.kk < it.k1) it.Pn = ldu_record(cpair[it.kk]);
    StoreStep R[kStoreSlots];
#pragma unroll
    for (int s = 0; s < kStoreSlots; ++s) it.next(cpair, L, xm, R[s]);
    // Rounds over the slots: slot s holds step n + s; each live slot is used and every slot is
    // refilled at once, so the oldest slot is live exactly while steps remain.
    while (R[0].live) {
#pragma unroll
      for (int s = 0; s < kStoreSlots; ++s) {
        if (R[s].live) {
          store_compute(A, R[s], L.dir, sx);
          if (R[s].last) A.pair_done();
        }
        it.next(cpair, L, xm, R[s]);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < kStoreBlocks; ++b)
#pragma unroll
    for (int u = 0; u < 4; ++u) accd[b][u] = A.accd[b][u] + static_cast<double>(A.acc[b][u]);
}

// all cap-touching pairs of a tile with weights evaluated on the fly
__device__ __forceinline__ void cap_rows_fly(const convreal::MixedDesc* __restrict__ d, const CapLane& L,
                                             const float* __restrict__ xm, float sx,
                                             const float4* __restrict__ s_coef, double (&accd)[4]) {
  // squared chords are formed directly in units of the table spacing: q = d^2 / h^2
  const double inv_h = ldu(d->inv_h);
  const double ih2 = inv_h * inv_h;
  const double qcut = ldu(d->dcut2) * ih2;
  const int seg_max = ldu(d->nseg) - 1;
  const int ni = L.ni;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const long long* rest_off = ldu(d->rest_off);
  const convreal::CapPair* cpair = ldu(d->cpair);
  const long long k0 = ldu(rest_off[L.r]);
  const long long k1 = ldu(rest_off[L.r + 1]);
  int nfold = 0;
  for (long long kk = k0; kk < k1; ++kk) {
    const convreal::CapPair P = ldu_record(cpair[kk]);
    const int nj = P.nj;
    const int cj = P.cj;
    int b0, bend;
    tile_union(P, L.u_first, L.u_last, ni, L.inv_2ni, b0, bend);
    const int K = bend - b0 + 1;
    if (K <= 0) continue;
    const int nk = (K + 31) >> 5;
    const int blast = b0 + 32 * nk - 1;
    const float* xj = xm + (L.ch ? P.xoff_m : P.xoff);
    const int pofs = L.pofs(nj, cj);
    const float rcp_n = __builtin_amdgcn_rcpf(static_cast<float>(nj));
    // largest |numerator| over the tile's rows and padded inputs: the numerator grows with a and
    // falls with b, so the extremes sit at (last row, b0) and (first row, blast)
    const double lim = kShortAlpha / P.scale;
    const bool shortform = static_cast<double>(L.u_last * nj - (2 * b0 + cj) * ni) <= lim &&
                           -static_cast<double>(L.u_first * nj - (2 * blast + cj) * ni) <= lim;
    if (shortform) {
      // |al| <= 0.2 on every (row, input) of the tile: no wrap of the numerator, and every padded
      // input lies outside the cut (d^2 > d_cut^2 decides), so no per-row window test is needed
      const double Bh = P.B * ih2;
      const double Ah = P.A * ih2;
      const double c0 = Bh * kSinShort[0], c1 = Bh * kSinShort[1], c2 = Bh * kSinShort[2], c3 = Bh * kSinShort[3];
      const double delta = 2.0 * static_cast<double>(ni) * P.scale;   // al step per input pixel
      // steps of 32 inputs; a remainder of at most 16 takes one 16-input step
      const int nfull = (K & 31) > 0 && (K & 31) <= 16 ? nk - 1 : nk;
      for (int q = 0; q < nfull; ++q)
        short_step<8>(acc, b0 + 32 * q + 8 * L.kgrp, L.u_row, ni, nj, cj, P.scale, delta, Ah, c0, c1, c2, c3, qcut,
                      seg_max, s_coef, xj, pofs, L.dir, rcp_n, sx);
      if (nfull < nk)
        short_step<4>(acc, b0 + 32 * nfull + 4 * L.kgrp, L.u_row, ni, nj, cj, P.scale, delta, Ah, c0, c1, c2, c3,
                      qcut, seg_max, s_coef, xj, pofs, L.dir, rcp_n, sx);
    } else {
      // general form (rings near a pole): numerator reduced to [-M, M], the long polynomial, and
      // the lane's own window [lo_r, hi_r], which also keeps a pixel from entering twice when the
      // union is wider than the ring
      const LongForm lf(P, ni, ih2);
      int lo_r, hi_r;
      row_window(P, L.u_row, ni, L.inv_2ni, lo_r, hi_r);
      for (int q = 0; q < nk; ++q) {
        const int bA = b0 + 32 * q + 8 * L.kgrp;
        half8 xhi, xlo;
        {
          int ix[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) ix[e] = mod_any(pofs + L.dir * (bA + e), nj, rcp_n);
          float v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = xj[ix[e]];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] *= sx;
          split_fp16<8>(v, xhi, xlo);
        }
        double qv[8];
        lf.q<8>(L.u_row, bA, ni, nj, cj, qv);
        float w[8];
        weights_of<8>(qv, qcut, seg_max, s_coef, w);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int b = bA + e;
          w[e] = (b >= lo_r && b <= hi_r) ? w[e] : 0.0f;
        }
        half8 whi, wlo;
        split_fp16<8>(w, whi, wlo);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xhi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, xhi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, xlo, acc, 0, 0, 0);
      }
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
}

// store D rows 4 kgrp + u (output pixel a0 + 4 kgrp + u), column col (image) of one 16-row block
// starting at a0; each output pixel once: rows beyond the fundamental domain [0, F), reflections of
// pixels on a reflection axis and the mirror of the equator ring are skipped
__device__ __forceinline__ void cap_put(const convreal::MixedDesc* __restrict__ d, const CapLane& L, int a0,
                                        const double (&accd)[4], float* __restrict__ ym, float sx) {
  const int mr = ldu(d->nrings) - 1 - L.r;
  if (L.ch && mr == L.r) return;
  const int rr = L.ch ? mr : L.r;
  const double inv = static_cast<double>(ldu(d->inv_sw)) / static_cast<double>(sx);
  float* yr = ym + ldu(ldu(d->rstart)[rr]);
  const bool add = ldu(ldu(d->ring_add)[rr]) != 0;
  const int ni = L.ni, ci = L.ci;
  const int quarter = ni >> 2;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ao = a0 + 4 * L.kgrp + u;
    if (ao >= L.F) continue;
    if (L.cf && ((2 * ao + ci) % quarter) == 0) continue;
    int Pp = L.cf ? (ni - ao - ci + L.cq * quarter) : (ao + L.cq * quarter);
    Pp %= ni;
    if (Pp < 0) Pp += ni;
    put(yr + Pp, accd[u] * inv, add);
  }
}

// one wave: cap tile t of the plan's tile list and its 16 images. A plan with a weight store lists
// store tiles of kStoreRows rows; one without lists tiles of 16 rows, evaluated on the fly.
// FLY = false: every slot holds a weight store, so only the store path is compiled in.
template <bool FLY>
__device__ __forceinline__ void cap_tile(const convreal::MixedDesc* __restrict__ d, int t,
                                         const float* __restrict__ xm, float* __restrict__ ym, float sx,
                                         const float4* __restrict__ s_coef) {
  if (!FLY || ldu(d->wstore) != nullptr) {
    const CapLane L(d, t, kStoreRows);
    double accd[kStoreBlocks][4];
    cap_rows_store(d, t, L, xm, sx, accd);
#pragma unroll
    for (int b = 0; b < kStoreBlocks; ++b) cap_put(d, L, L.a0 + 16 * b, accd[b], ym, sx);
  } else if constexpr (FLY) {
    const CapLane L(d, t, 16);
    double accd[4] = {0.0, 0.0, 0.0, 0.0};
    cap_rows_fly(d, L, xm, sx, s_coef, accd);
    cap_put(d, L, L.a0, accd, ym, sx);
  }
}

// ---------------------------------------------------------------- cap weight store (set-up)
// One wave per store tile, the same tiles, ring pairs, union windows and row windows as the apply.
// FILL = false: the number of 16-byte groups of each tile; FILL = true: the groups (long form, any
// ring pair), tile t's block starting at group offsets[t].
template <bool FILL>
__global__ __launch_bounds__(kBlock) void cap_store_kernel(const convreal::MixedDesc* __restrict__ d,
                                                           long long* __restrict__ offsets,
                                                           u32x4* __restrict__ store) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  float4* s_coef = reinterpret_cast<float4*>(lds);
  if (FILL) {
    const float4* coef = reinterpret_cast<const float4*>(ldu(d->coef));
    const int nseg = ldu(d->nseg);
    for (int k = threadIdx.x; k < nseg; k += kBlock) s_coef[k] = coef[k];
    __syncthreads();
  }
  const int t = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  if (t >= ldu(d->n_citems)) return;
  const CapLane L(d, t, kStoreRows);
  const double inv_h = ldu(d->inv_h);
  const double ih2 = inv_h * inv_h;
  const double qcut = ldu(d->dcut2) * ih2;
  const int seg_max = ldu(d->nseg) - 1;
  const long long* rest_off = ldu(d->rest_off);
  const convreal::CapPair* cpair = ldu(d->cpair);
  const long long k0 = ldu(rest_off[L.r]);
  const long long k1 = ldu(rest_off[L.r + 1]);
  u32x4* tile = FILL ? store + (offsets[t] & convreal::kTileOffsetMask) : nullptr;
  int pos = 0;
  bool wraps = false;
  for (long long kk = k0; kk < k1; ++kk) {
    const convreal::CapPair P = ldu_record(cpair[kk]);
    StorePair S;
    int lo[kStoreBlocks], hi[kStoreBlocks];
    const PairWin w = pair_windows(P, L, S, lo, hi);
    if (w.stored == 0) continue;
    if (!FILL) {
      int low;
      wraps = wraps || __any(pair_wraps(P, L, w.b0, w.nk, low));
      pos += w.stored;
      continue;
    }
    // the apply's order: step, block, half, lanes in lane order
    const LongForm lf(P, L.ni, ih2);
    for (int q = 0; q < w.nk; ++q) {
#pragma unroll
      for (int b = 0; b < kStoreBlocks; ++b) {
        unsigned oa, ob;
        step_offsets(S, b, q, L.kgrp, pos, oa, ob);
        for (int h = 0; h < 2; ++h) {
          const unsigned o = h ? ob : oa;
          if (o == kNoLoad) continue;
          const int bA = w.b0 + 4 * (8 * q + 4 * h + L.kgrp);
          double qv[4];
          lf.q<4>(L.u_row + 32 * b, bA, L.ni, P.nj, P.cj, qv);
          float wv[4];
          weights_of<4>(qv, qcut, seg_max, s_coef, wv);
#pragma unroll
          for (int e = 0; e < 4; ++e) wv[e] = (bA + e >= lo[b] && bA + e <= hi[b]) ? wv[e] : 0.0f;
          half4 wh, wl;
          split_fp16<4>(wv, wh, wl);
          const u32x2 ph = __builtin_bit_cast(u32x2, wh), pl = __builtin_bit_cast(u32x2, wl);
          tile[o / 16u] = u32x4{ph.x, ph.y, pl.x, pl.y};
        }
      }
    }
  }
  if (!FILL && (threadIdx.x & 63) == 0) offsets[t] = pos | (wraps ? convreal::kTileWraps : 0);
}

// ---------------------------------------------------------------- persistent queue kernel
// WAVES: resident waves per SIMD the registers are sized for (= workgroups per compute unit); at
// least two, so that belt and cap items share a SIMD; three where the LDS allows it (256-pixel belt
// items and no coefficient table), at the price of a few spilled registers
// The queue is split into n_chunks chunks of items (chunk c: items chunk_off[c] .. chunk_off[c+1]
// - 1, each for nrep maps), one counter each. A workgroup takes items from its home chunk
// (see home below) first and then from the others, until every chunk is empty.
// home_div = 1 with one chunk per XCD: workgroups are spread over the XCDs in turn, so the items of
// a chunk share one L2. home_div = number of CUs with a belt chunk and two cap chunks: the first
// workgroups fill one slot on every CU, so each CU starts with one workgroup on belt items (matrix
// cores, LDS) beside two on cap items (the vector memory path).
template <int SEG, bool FLY, int WAVES>
__global__ __launch_bounds__(kBlock, WAVES) void mixed_persistent_kernel(convreal::Slots S,
                                                                  const int2* __restrict__ items,
                                                                  int n_items, int nrep,
                                                                  const int* __restrict__ chunk_off,
                                                                  int n_chunks, int home_div,
                                                                  const unsigned* __restrict__ amax,
                                                                  unsigned* __restrict__ counter,
                                                                  int coef_offset_bytes) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ int s_item;
  __shared__ const convreal::MixedDesc* s_coef_owner;
  _Float16* stage = reinterpret_cast<_Float16*>(lds);
  float4* s_coef = reinterpret_cast<float4*>(lds + coef_offset_bytes);
  if (threadIdx.x == 0) s_coef_owner = nullptr;
  // home_div > 0: chunk (block / home_div) mod n_chunks; home_div < 0 (roles with per-XCD cap
  // chunks): the first -home_div workgroups take chunk 0, the others chunk 1 + their XCD
  const int home =
      home_div > 0 ? static_cast<int>((blockIdx.x / static_cast<unsigned>(home_div)) % static_cast<unsigned>(n_chunks))
      : (static_cast<int>(blockIdx.x) < -home_div || n_chunks < 2)
          ? 0
          : 1 + static_cast<int>(blockIdx.x % static_cast<unsigned>(convreal::kXcds)) % (n_chunks - 1);
  unsigned empty = 0u;   // chunks this workgroup found empty (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      int got = -1;   // map repetition x n_items + item (the host keeps n_items x nrep below 2^31)
      for (int k = 0; k < n_chunks && got < 0; ++k) {
        const int c = home + k < n_chunks ? home + k : home + k - n_chunks;
        if (empty & (1u << c)) continue;
        const int c0 = chunk_off[c], len = chunk_off[c + 1] - c0;
        const unsigned v = len > 0 ? atomicAdd(counter + c, 1u) : 0u;
        if (len > 0 && v < static_cast<unsigned>(len) * static_cast<unsigned>(nrep))
          got = static_cast<int>(v / len) * n_items + c0 + static_cast<int>(v % len);
        else
          empty |= 1u << c;
      }
      s_item = got;
    }
    __syncthreads();
    // values read from LDS are the same in every lane; readfirstlane tells the compiler so, which
    // keeps the item's descriptor and its pointers in scalar registers and their loads scalar
    const int gi = __builtin_amdgcn_readfirstlane(s_item);
    const unsigned long long ow = reinterpret_cast<unsigned long long>(s_coef_owner);
    const unsigned long long ow_u =
        static_cast<unsigned long long>(static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(ow)))) |
        (static_cast<unsigned long long>(static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(ow >> 32))))
         << 32);
    const convreal::MixedDesc* owner = reinterpret_cast<const convreal::MixedDesc*>(ow_u);
    __syncthreads();
    if (gi < 0) break;
    const int2 it = ldu_record(items[gi % n_items]);
    const int slot = it.x + static_cast<int>(gi / n_items);
    const int kind = it.y >> 30;
    const int idx = it.y & 0x3fffffff;
    const convreal::MixedDesc* d = S.desc[slot];
    const float sx = map_scale(ldu(amax[slot]));
    if (kind == 0) {
      // three rings in flight, two where the registers are sized for three waves per SIMD
      belt_item<SEG, (WAVES >= 3 ? 2 : 3)>(d, idx, S.x[slot], S.y[slot], sx, stage);
      // a coefficient table inside the belt stage is gone (read again by the next cap item)
      if (FLY && coef_offset_bytes == 0 && threadIdx.x == 0) s_coef_owner = nullptr;
    } else {
      if (FLY && owner != d) {
        const float4* coef = reinterpret_cast<const float4*>(ldu(d->coef));
        const int nseg = ldu(d->nseg);
        for (int k = threadIdx.x; k < nseg; k += kBlock) s_coef[k] = coef[k];
        __syncthreads();
        if (threadIdx.x == 0) s_coef_owner = d;
      }
      const int t = idx * kWaves + __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
      if (t < ldu(d->n_citems))
        cap_tile<FLY>(d, t, S.x[slot], S.y[slot], sx, s_coef);
    }
    __syncthreads();
  }
}

}  // namespace

// Device scratch of conv_real_apply_noalloc (one copy per device; see noalloc_scratch_resolve).
static __device__ __align__(256) unsigned scratch[convreal::kNoallocScratchWords];

namespace convreal {

// belt stage: two window buffers (8 shifted copies, hi and lo planes) and two weight-fragment buffers
size_t belt_stage_bytes(int seg) {
  const size_t wbytes = 2 * kNKMax * 128 * sizeof(half8);
  return (seg == 512 ? static_cast<size_t>(BeltLayout<512>::BYTES) : static_cast<size_t>(BeltLayout<256>::BYTES)) +
         wbytes;
}

// Dynamic LDS of the persistent kernel: the belt stage, then the coefficient table.
size_t persistent_lds_bytes(int seg, int nseg) {
  const size_t coef_off = (belt_stage_bytes(seg) + 15) / 16 * 16;
  return coef_off + sizeof(float4) * static_cast<size_t>(nseg > 0 ? nseg : 1);
}

// Dynamic LDS with the coefficient table inside the 256-pixel belt stage (read again after every
// belt item): the larger of the two.
size_t shared_lds_bytes(int nseg) {
  const size_t stage = belt_stage_bytes(256), coef = sizeof(float4) * static_cast<size_t>(nseg > 0 ? nseg : 1);
  return stage > coef ? stage : coef;
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
                              int n_items, int nrep, const int* chunk_off, int n_chunks, unsigned* amax,
                              unsigned* counter, const Tuning& tune, int max_nseg, long long npix_max,
                              long long pairs, bool fly, hipStream_t st, bool zero_rows) {
  if (n_chunks < 1 || n_chunks > kMaxChunks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_state_kernel, dim3(1), dim3(kMaxSlots), 0, st, amax, nslots, counter, n_chunks);
  mark(mark_plan, st, "zero_state_kernel", 0);
  // at least 8 float4 per thread, at most 1024 workgroups (and atomics) per map
  const long long want = (npix_max / 4 + 2047) / 2048;
  const unsigned gx = static_cast<unsigned>(want < 1 ? 1 : (want < 1024 ? want : 1024));
  hipLaunchKernelGGL(prep_kernel, dim3(gx, nslots), dim3(256), 0, st, S, amax, zero_rows ? 1 : 0);
  mark(mark_plan, st, "prep_kernel", 0);
  if (n_items > 0 && nrep > 0) {
    // the coefficient table is only read when some slot evaluates cap weights on the fly; three
    // workgroups per CU fit when it shares the belt stage's LDS (a workgroup uses one at a time)
    const bool fly3 = fly && tune.seg == 256 && tune.wg_per_cu >= 3;
    const size_t coef_off = fly3 ? 0 : (belt_stage_bytes(tune.seg) + 15) / 16 * 16;
    const size_t lds = fly3 ? shared_lds_bytes(max_nseg) : persistent_lds_bytes(tune.seg, fly ? max_nseg : 0);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    long long total = static_cast<long long>(n_items) * nrep;
    if (total >= (1LL << 31)) return hipErrorInvalidValue;   // item counter is 32-bit
    long long grid = static_cast<long long>(ncu) * (tune.wg_per_cu > 0 ? tune.wg_per_cu : 2);
    if (grid > total) grid = total;
    const dim3 g(static_cast<unsigned>(grid)), blk(kBlock);
    // the role order hands out home chunks by workgroup slot on a CU (the first ncu workgroups fill
    // one slot on every CU), the others by workgroup (workgroups go round the XCDs in turn)
    const int home_div = tune.order == 3 ? ncu : (tune.order == 4 ? -ncu : 1);
    const int co = static_cast<int>(coef_off);
    if (tune.seg == 512 && fly)
      hipLaunchKernelGGL((mixed_persistent_kernel<512, true, 2>), g, blk, lds, st, S, items, n_items, nrep, chunk_off, n_chunks, home_div, amax, counter, co);
    else if (tune.seg == 512)
      hipLaunchKernelGGL((mixed_persistent_kernel<512, false, 2>), g, blk, lds, st, S, items, n_items, nrep, chunk_off, n_chunks, home_div, amax, counter, co);
    else if (fly3)
      hipLaunchKernelGGL((mixed_persistent_kernel<256, true, 3>), g, blk, lds, st, S, items, n_items, nrep, chunk_off, n_chunks, home_div, amax, counter, co);
    else if (fly)
      hipLaunchKernelGGL((mixed_persistent_kernel<256, true, 2>), g, blk, lds, st, S, items, n_items, nrep, chunk_off, n_chunks, home_div, amax, counter, co);
    else if (tune.wg_per_cu >= 3)
      hipLaunchKernelGGL((mixed_persistent_kernel<256, false, 3>), g, blk, lds, st, S, items, n_items, nrep, chunk_off, n_chunks, home_div, amax, counter, co);
    else
      hipLaunchKernelGGL((mixed_persistent_kernel<256, false, 2>), g, blk, lds, st, S, items, n_items, nrep, chunk_off, n_chunks, home_div, amax, counter, co);
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
  const void* fns[] = {reinterpret_cast<const void*>(&mixed_persistent_kernel<256, true, 2>),
                       reinterpret_cast<const void*>(&mixed_persistent_kernel<256, true, 3>),
                       reinterpret_cast<const void*>(&mixed_persistent_kernel<256, false, 2>),
                       reinterpret_cast<const void*>(&mixed_persistent_kernel<256, false, 3>),
                       reinterpret_cast<const void*>(&mixed_persistent_kernel<512, true, 2>),
                       reinterpret_cast<const void*>(&mixed_persistent_kernel<512, false, 2>)};
  for (const void* f : fns) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t cap_store_count(const conv_real_plan* p, long long* counts_dev) {
  const unsigned grid = static_cast<unsigned>((p->n_citems + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(cap_store_kernel<false>, dim3(grid), dim3(kBlock), 0, nullptr, p->d_desc, counts_dev,
                     static_cast<u32x4*>(nullptr));
  return hipGetLastError();
}

hipError_t cap_store_fill(const conv_real_plan* p) {
  const unsigned grid = static_cast<unsigned>((p->n_citems + kWaves - 1) / kWaves);
  const size_t lds = sizeof(float4) * static_cast<size_t>(p->cap_nseg > 0 ? p->cap_nseg : 1);
  hipLaunchKernelGGL(cap_store_kernel<true>, dim3(grid), dim3(kBlock), lds, nullptr, p->d_desc, p->d_wtile_off,
                     reinterpret_cast<u32x4*>(p->d_wstore));
  return hipGetLastError();
}

hipError_t launch_mixed(const conv_real_plan* p, const float* x, float* y, int nmaps, hipStream_t st) {
  return launch_mixed(p, x, y, nmaps, st, p->d_amax, p->d_counter);
}

hipError_t launch_mixed(const conv_real_plan* p, const float* x, float* y, int nmaps, hipStream_t st,
                        unsigned* amax, unsigned* counter) {
  // ring-FFT method: the belt rings of each map are written by the ring FFTs first; the queue then
  // holds the cap items only, and rows with cap contributions add to what the FFTs wrote (so the
  // prep pass zeroes nothing)
  const bool fft = p->method == CONV_REAL_METHOD_RING_FFT;
  for (int m0 = 0; m0 < nmaps; m0 += kMaxSlots) {
    const int nm = nmaps - m0 < kMaxSlots ? nmaps - m0 : kMaxSlots;
    for (int k = 0; k < nm && fft; ++k) {
      const size_t off = static_cast<size_t>(m0 + k) * p->npix;
      const hipError_t e = ring_fft_belt_f32(p, x + off, y + off, st);
      if (e != hipSuccess) return e;
    }
    Slots S;
    for (int k = 0; k < nm; ++k) {
      S.desc[k] = p->d_desc;
      S.x[k] = x + static_cast<size_t>(m0 + k) * p->npix;
      S.y[k] = y + static_cast<size_t>(m0 + k) * p->npix;
    }
    hipError_t e = launch_mixed_queue(p, S, nm, p->d_items, p->n_items, nm, p->d_qchunk_off, p->n_qchunks, amax,
                                      counter, p->tune, p->cap_nseg, p->npix,
                                      (fft ? p->pairs_rest : p->pairs) * nm, p->cap_mode && !p->d_wstore, st, !fft);
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


// Scratch of the apply that allocates nothing: one array per device, holding the per-slot max |x|
// words and the work-queue counters that zero_state_kernel clears at the start of every launch.
// Host code never passes the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the address hipGetSymbolAddress returns for the current device.
static_assert(kMaxSlots + kMaxChunks <= kNoallocScratchWords, "no-alloc scratch too small");

static std::mutex g_scratch_mu;
static unsigned* g_scratch_ptr[kNoallocMaxDevices] = {};

hipError_t noalloc_scratch_resolve(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = static_cast<unsigned*>(ptr);
  return hipSuccess;
}

unsigned* noalloc_scratch(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace convreal
