// pair_accumulate: every pixel pair evaluated and accumulated in FP64.
//
//   y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) x_q
//
// One thread per output pixel a of ring i; 256 threads own a tile of up to 256 consecutive pixels
// of one ring. For each listed neighbour ring j (from the ring_window pass) the thread walks the
// candidate pixels b of its azimuthal window. The half-angle alpha = (phi_a - phi_b) / 2 =
// (pi / 2) * num / (n_i n_j) has the exact integer numerator num = (2a + c_i) n_j - (2b + c_j) n_i;
// sin(alpha) is seeded from that numerator and advanced by the rotation alpha -> alpha - pi / n_j
// from one pixel to the next (re-seeded every 64 steps). The chord is d^2 = A_ij + B_ij sin^2(alpha);
// pairs with d^2 <= d_cut^2 are interpolated from the table and accumulated in FP64.
//
// The accumulate kernel is persistent: a workgroup of kGroups x 256 threads stages the kernel table
// in LDS once and its groups of 256 threads take tiles in turn. The table is staged as the
// per-segment coefficients of the interpolating cubic (4 doubles per segment, evaluated in Horner
// form) when they fit in 64 KB, else as the nodes themselves (4-point Lagrange weights per pair).
// t = d / h comes from the hardware reciprocal square root of (d / h)^2 refined by two Newton
// steps. The ring-pair tables are read with scalar loads (one tile = one ring, so every lane of a
// wave reads the same entries), and the azimuth numerator is reduced in exact FP64 arithmetic rather
// than by 64-bit integer division. Inputs are read straight from the map (neighbouring lanes read
// neighbouring pixels of ring j, through the L1): the loop is bound by its FP64 arithmetic, about 32
// vector instructions per pair, and staging the windows in LDS would add work without removing any.
//
// The same loop serves two callers:
//   * the plain path (CONV_REAL_F64 / F32): every ring pair of every output ring, stored;
//   * the mixed path's remainder: only ring pairs that touch a polar cap, listed by index; the
//     result is stored for cap output rings and added to the matrix-core result for belt rings.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace {

constexpr int kTile = 256;
constexpr int kGroups = 3;   // tiles in flight per workgroup of the accumulate kernel (two fit a CU)

struct PairArgs {
  const double* table;
  const double* coef;     // per segment c0..c3 of the cubic in f = t - k (nullptr: node form)
  const int* rn;
  const int* rc;
  const long long* rstart;
  const double* rcd;
  const double* rsd;
  const long long* off;   // per ring: CSR offsets into the (listed) ring pairs
  const long long* idx;   // listed pair -> ring-pair index, or nullptr for the identity
  const int* pj;          // per ring pair: neighbour ring
  const double* pA;
  const double* pB;
  const double* phw;
  const int* tile_ring;
  const int* tile_a0;
  const convreal::CapPair64* cpair;   // per listed pair (the FP64 cap kernel), else nullptr
  int ntiles;
  int n_tab;
  int belt_lo;            // rings [belt_lo, belt_hi] get y += (remainder mode); others y =
  int belt_hi;
  int accumulate_belt;
  double inv_h;
  double dcut2;
  double omega;
  long long npix;
};

// The candidate pixels b of neighbour ring j (ring pair k) for output pixel a of ring i: the window
// [blo, blo + nb) in ring j's pixel indices (unwrapped, blo in (-n_j, n_j)), and the pair's chord
// constants. Every table value is the same for all lanes of a tile (one ring i, one list of ring
// pairs) and comes through scalar loads.
struct RingWalk {
  int blo;
  int nb;
  int nj;
  int cj;
  long long sj;   // first pixel of ring j in the map
  double A, B;    // d^2 = A + B sin^2(alpha)
  double cd, sd;  // cos and sin of pi / n_j (one step of alpha)
};

__device__ __forceinline__ bool ring_walk(const PairArgs& a, long long k, int ni, int twoa_ci, RingWalk& w) {
  using convreal::ldu;
  const int j = ldu(ldu(a.pj)[k]);
  w.nj = ldu(ldu(a.rn)[j]);
  w.cj = ldu(ldu(a.rc)[j]);
  const double hw = ldu(ldu(a.phw)[k]);
  // window centre in pixels of ring j: b_c = ((2a + c_i) n_j / n_i - c_j) / 2, in [-1/2, n_j)
  const double bc2 = static_cast<double>(twoa_ci) * w.nj - static_cast<double>(w.cj) * ni;   // exact
  const double bc = bc2 / (2.0 * ni);
  int nb;
  if (2.0 * hw >= static_cast<double>(w.nj)) {
    w.blo = static_cast<int>(floor(bc)) - w.nj / 2;
    nb = w.nj;
  } else {
    w.blo = static_cast<int>(ceil(bc - hw - 1e-7));
    nb = static_cast<int>(floor(bc + hw + 1e-7)) - w.blo + 1;
    if (nb > w.nj) nb = w.nj;
  }
  if (nb <= 0) return false;
  w.nb = nb;
  w.A = ldu(ldu(a.pA)[k]);
  w.B = ldu(ldu(a.pB)[k]);
  w.sj = ldu(ldu(a.rstart)[j]);
  w.cd = ldu(ldu(a.rcd)[j]);
  w.sd = ldu(ldu(a.rsd)[j]);
  return true;
}

// sin and cos of alpha = (pi / 2) num / (n_i n_j) at window step t, from the exact numerator
// num = (2a + c_i) n_j - (2b + c_j) n_i, reduced modulo 2 n_i n_j (a shift of alpha by a multiple of
// pi, which leaves sin^2 alpha and the rotation unchanged). Every integer here is below 2^53, so the
// products, the difference and the fused reduction are exact in FP64.
__device__ __forceinline__ void seed_alpha(const RingWalk& w, int twoa_ci, int ni, int t, double& sa, double& ca) {
  const double num = static_cast<double>(twoa_ci) * w.nj - static_cast<double>(2 * (w.blo + t) + w.cj) * ni;
  const double m2 = 2.0 * static_cast<double>(ni) * static_cast<double>(w.nj);
  const double r = fma(-rint(num / m2), m2, num);
  sincospi(r / m2, &sa, &ca);
}

// first window pixel as an index into ring j
__device__ __forceinline__ int first_index(const RingWalk& w) { return w.blo < 0 ? w.blo + w.nj : w.blo; }

// number of pairs with d^2 <= d_cut^2 of output pixel ai of ring r (alpha advanced by rotation,
// re-seeded every 64 steps)
__device__ __forceinline__ unsigned long long count_pixel(const PairArgs& a, int r, int ai) {
  using convreal::ldu;
  const int ni = ldu(ldu(a.rn)[r]);
  const int twoa_ci = 2 * ai + ldu(ldu(a.rc)[r]);
  const long long k0 = ldu(ldu(a.off)[r]), k1 = ldu(ldu(a.off)[r + 1]);
  const long long* idx = ldu(a.idx);
  unsigned long long cnt = 0;
  for (long long kk = k0; kk < k1; ++kk) {
    RingWalk w;
    if (!ring_walk(a, idx ? ldu(idx[kk]) : kk, ni, twoa_ci, w)) continue;
    double sa = 0.0, ca = 1.0;
    for (int t = 0; t < w.nb; ++t) {
      if ((t & 63) == 0) seed_alpha(w, twoa_ci, ni, t, sa, ca);
      if (fma(w.B, sa * sa, w.A) <= a.dcut2) ++cnt;
      const double sa2 = sa * w.cd - ca * w.sd;
      ca = ca * w.cd + sa * w.sd;
      sa = sa2;
    }
  }
  return cnt;
}

// t = sqrt(q) for q > 0: hardware reciprocal square root refined by two Newton steps on t^2 = q
__device__ __forceinline__ double sqrt_refined(double q) {
  const double y = __builtin_amdgcn_rsq(q);
  const double hy = 0.5 * y;
  double t = q * y;
  t = fma(fma(-t, t, q), hy, t);
  return fma(fma(-t, t, q), hy, t);
}

// (d / h)^2 plus the smallest normal, so that the pixel itself (d = 0) gets t ~ 1e-154 (segment 0,
// the value at d = 0) and every other pair its own value: q is at least ~1e-30 there, far above the
// addend
__device__ __forceinline__ double scaled_q(double d2, double ih2) { return fma(d2, ih2, 2.2250738585072014e-308); }

// Ktilde at t = d / h, t in [0, n_tab - 3] (clamped there otherwise)
template <bool kCoef>
__device__ __forceinline__ double table_value(const double* __restrict__ s_tab, int n_tab, double t) {
  // f = t - k: t never exceeds n_tab - 3 (+ rounding) for a pair inside the cut; the clamp only keeps
  // other lanes' reads inside the table
  const int k = min(static_cast<int>(t), n_tab - 3);
  const double f = __builtin_amdgcn_fract(t);
  if constexpr (kCoef) {
    const double4 c = reinterpret_cast<const double4*>(s_tab)[k];
    return fma(fma(fma(c.w, f, c.z), f, c.y), f, c.x);
  } else {
    const double tm1 = s_tab[k == 0 ? 1 : k - 1];
    const double t0 = s_tab[k];
    const double t1 = s_tab[k + 1];
    const double t2 = s_tab[k + 2];
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
}

// sum over the listed neighbour rings of output pixel ai of ring r: acc[m] += Ktilde(d) x_m(q), in
// window order (alpha as in count_pixel)
template <bool kCoef, int kMaxMaps, typename T>
__device__ __forceinline__ void accumulate_pixel(const PairArgs& a, const double* __restrict__ s_tab, int r, int ai,
                                                 const T* __restrict__ x, int nm, double* acc) {
  using convreal::ldu;
  const int ni = ldu(ldu(a.rn)[r]);
  const int twoa_ci = 2 * ai + ldu(ldu(a.rc)[r]);
  const long long k0 = ldu(ldu(a.off)[r]), k1 = ldu(ldu(a.off)[r + 1]);
  const long long* idx = ldu(a.idx);
  const double ih2 = a.inv_h * a.inv_h;
  for (long long kk = k0; kk < k1; ++kk) {
    RingWalk w;
    if (!ring_walk(a, idx ? ldu(idx[kk]) : kk, ni, twoa_ci, w)) continue;
    const T* xj = x + w.sj;
    int bm = first_index(w);
    double sa = 0.0, ca = 1.0;
    for (int t = 0; t < w.nb; ++t) {
      if ((t & 63) == 0) seed_alpha(w, twoa_ci, ni, t, sa, ca);
      const double d2 = fma(w.B, sa * sa, w.A);
      if (d2 <= a.dcut2) {
        const double kt = table_value<kCoef>(s_tab, a.n_tab, sqrt_refined(scaled_q(d2, ih2)));
#pragma unroll
        for (int m = 0; m < kMaxMaps; ++m)
          if (m < nm) acc[m] = fma(kt, static_cast<double>(xj[m * a.npix + bm]), acc[m]);
      }
      const double sa2 = sa * w.cd - ca * w.sd;
      ca = ca * w.cd + sa * w.sd;
      sa = sa2;
      if (++bm == w.nj) bm = 0;
    }
  }
}

template <bool kCoef, int kMaxMaps, typename T>
__global__ __launch_bounds__(kTile * kGroups) void pair_accumulate_kernel(PairArgs a, const T* __restrict__ x,
                                                                          T* __restrict__ y, int nm) {
  extern __shared__ double s_tab[];
  const int nwords = kCoef ? 4 * (a.n_tab - 2) : a.n_tab;
  const double* src = kCoef ? a.coef : a.table;
  for (int k = threadIdx.x; k < nwords; k += blockDim.x) s_tab[k] = src[k];
  __syncthreads();
  using convreal::ldu;
  // the group (and so its tile, ring and ring-pair list) is the same in every lane of a wave
  const int grp = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kTile);
  const int lane = static_cast<int>(threadIdx.x) % kTile;
  for (int tile = blockIdx.x * kGroups + grp; tile < a.ntiles; tile += gridDim.x * kGroups) {
    const int r = ldu(ldu(a.tile_ring)[tile]);
    const int ai = ldu(ldu(a.tile_a0)[tile]) + lane;
    if (ai >= ldu(ldu(a.rn)[r])) continue;
    double acc[kMaxMaps];
#pragma unroll
    for (int m = 0; m < kMaxMaps; ++m) acc[m] = 0.0;
    accumulate_pixel<kCoef, kMaxMaps, T>(a, s_tab, r, ai, x, nm, acc);
    const long long out = a.rstart[r] + ai;
    const bool add = a.accumulate_belt && r >= a.belt_lo && r <= a.belt_hi;
#pragma unroll
    for (int m = 0; m < kMaxMaps; ++m) {
      if (m < nm) {
        T* yp = y + m * a.npix + out;
        const double v = a.omega * acc[m];
        *yp = add ? static_cast<T>(static_cast<double>(*yp) + v) : static_cast<T>(v);
      }
    }
  }
}

// Ring pairs that touch a polar cap, over the fundamental domain of the pixelization's symmetry
// group (quarter turns, the reflection phi -> -phi, the north/south mirror: 16 elements that map
// every ring onto itself or its mirror and keep every chord), on the FP64 matrix cores: each weight
// Ktilde(d(a, b)) is evaluated once and applied to the 16 images of input pixel b, which give the 16
// images of output pixel a. One wave per 16 consecutive domain pixels (rows) of a north-half ring.
// Per ring pair the 16 rows' windows are joined and walked 4 inputs at a time, each step one
// v_mfma_f64_16x16x4 of W[row][k] (weight of row pixel a and input pixel b0 + 4s + k in lane
// row + 16 k, zero outside the row's own window or the cut) by X[k][image] (input pixel b0 + 4s + k
// mapped by image = lane & 15, loaded once for all 16 rows). Lane l's results are rows 4 i + (l >> 4)
// of image l & 15 (the FP64 instruction's output order: register i of lanes 16 q .. 16 q + 15 holds
// row 4 i + q). Weights: alpha seeded from the exact numerator every 16 steps and rotated by 4 pixels
// between; the same membership test and interpolation as accumulate_pixel. Images that coincide
// (pixels on a reflection axis, the equator ring's mirror) are written once; belt rings get y +=,
// cap rings y =. One FP64 map per launch.
typedef double doublex4 __attribute__((ext_vector_type(4)));
// tiles per workgroup (the table is staged once for all of them): the 64 KB table allows two
// workgroups per CU, so 8 waves each give 4 waves per SIMD (register budget 128, 102 used, no spills;
// 12 waves at 6 per SIMD spilled 20-26 registers and took 4.5% longer at Nside 2048 / 30', 14
// spilled more and lost 19%)
constexpr int kMfmaWaves = 8;

template <bool kCoef>
__global__ __launch_bounds__(64 * kMfmaWaves, kMfmaWaves / 2) void cap_mfma64_kernel(PairArgs a, const double* __restrict__ x,
                                                           double* __restrict__ y, int nrings) {
  extern __shared__ double s_tab[];
  const int nwords = kCoef ? 4 * (a.n_tab - 2) : a.n_tab;
  const double* src = kCoef ? a.coef : a.table;
  for (int k = threadIdx.x; k < nwords; k += blockDim.x) s_tab[k] = src[k];
  __syncthreads();
  using convreal::ldu;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int tile = static_cast<int>(blockIdx.x) * kMfmaWaves + wave;
  if (tile >= a.ntiles) return;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int row = lane & 15, kq = lane >> 4;
  const int r = ldu(ldu(a.tile_ring)[tile]);
  const int a0 = ldu(ldu(a.tile_a0)[tile]);
  const int ni = ldu(ldu(a.rn)[r]);
  const int ci = ldu(ldu(a.rc)[r]);
  const int F = (ni / 4 - ci) / 2 + 1;
  const int ai = a0 + row;                  // this lane's row pixel (a weight row when ai < F)
  const int twoa_ci = 2 * ai + ci;
  const double ih2 = a.inv_h * a.inv_h;
  const double inv_2ni = 1.0 / (2.0 * ni);
  // B operand: this lane's image of the input pixels
  const int img = lane & 15, ih = img >> 3, ifl = (img >> 2) & 1, iq = img & 3;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  const long long k0 = ldu(ldu(a.off)[r]), k1 = ldu(ldu(a.off)[r + 1]);
  const convreal::CapPair64* cpair = ldu(a.cpair);
  convreal::CapPair64 Pn;   // record kk, loaded one pair ahead of its use
  if (k0 < k1) Pn = convreal::ldu_record(cpair[k0]);
  for (long long kk = k0; kk < k1; ++kk) {
    const convreal::CapPair64 P = Pn;
    if (kk + 1 < k1) Pn = convreal::ldu_record(cpair[kk + 1]);
    const int nj = P.nj;
    const int cj = P.cj;
    const double hw = P.hw;
    // this row's window [blo, blo + nb) of ring j: the bounds of ring_walk, the centre through the
    // tile's reciprocal of 2 n_i (the window keeps its 1e-7 margin; the cut test decides membership)
    int blo = 0, nb = 0;
    if (ai < F) {
      const double bc = (static_cast<double>(twoa_ci) * nj - static_cast<double>(cj) * ni) * inv_2ni;
      if (2.0 * hw >= static_cast<double>(nj)) {
        blo = static_cast<int>(floor(bc)) - nj / 2;
        nb = nj;
      } else {
        blo = static_cast<int>(ceil(bc - hw - 1e-7));
        nb = min(static_cast<int>(floor(bc + hw + 1e-7)) - blo + 1, nj);
      }
    }
    const bool has = nb > 0;
    int lo = has ? blo : 0x3fffffff, hi = has ? blo + nb - 1 : -0x3fffffff;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      lo = min(lo, __shfl_xor(lo, o));
      hi = max(hi, __shfl_xor(hi, o));
    }
    const int b0 = __builtin_amdgcn_readfirstlane(lo), bend = __builtin_amdgcn_readfirstlane(hi);
    if (bend < b0) continue;
    const double A = P.A, B = P.B;
    const double* xs = x + (ih ? P.xoff_m : P.xoff);
    // rotation by 4 input pixels (alpha -> alpha - 4 pi / n_j) from the ring's sin and cos of pi / n_j
    // by two angle doublings
    const double sd = P.sd, cd = P.cd;
    const double s2 = 2.0 * sd * cd, c2 = fma(-2.0 * sd, sd, 1.0);
    const double s4 = 2.0 * s2 * c2, c4 = fma(-2.0 * s2, s2, 1.0);
    // alpha seeds: numerator (2a + c_i) n_j - (2b + c_j) n_i reduced modulo m2 = 2 n_i n_j (exact
    // integers in FP64), sin and cos of pi num / m2
    const double m2 = 2.0 * static_cast<double>(ni) * static_cast<double>(nj);
    const double inv_m2 = 1.0 / m2;
    const double num0 = static_cast<double>(twoa_ci) * nj - static_cast<double>(2 * (b0 + kq) + cj) * ni;
    const double dnum = 8.0 * static_cast<double>(ni);   // numerator step per matrix step (4 pixels)
    const int ns = (bend - b0 + 4) >> 2;
    // step state: rel = b - blo of this lane's input b = b0 + 4 st + kq (outside the row's window when
    // unsigned rel > span; a row with no window never matches), iw = index in ring j of b's image
    const unsigned span = has ? static_cast<unsigned>(nb - 1) : 0u;
    int rel = has ? b0 + kq - blo : -0x40000000;
    int bw = b0 + kq;   // in (-n_j, n_j + 3): windows start above -n_j and below n_j
    bw = bw < 0 ? bw + nj : bw;
    bw = bw >= nj ? bw - nj : bw;
    int iw = (ifl ? nj - bw - cj : bw) + iq * (nj / 4);
    iw = iw >= nj ? iw - nj : iw;
    const int d4 = ifl ? -4 : 4, wrap = ifl ? -nj : nj;
    auto next_input = [&]() {
      const double v = xs[iw];
      iw += d4;
      iw -= static_cast<unsigned>(iw) >= static_cast<unsigned>(nj) ? wrap : 0;
      return v;
    };
    // weight of this lane's row and input at alpha's sine sa, zeroed outside the window or the cut
    auto next_weight = [&](double sa) {
      const double d2 = fma(B, sa * sa, A);
      const double kv = table_value<kCoef>(s_tab, a.n_tab, sqrt_refined(scaled_q(d2, ih2)));
      const bool in = static_cast<unsigned>(rel) <= span && d2 <= a.dcut2;
      rel += 4;
      return in ? kv : 0.0;
    };
    auto seed = [&](int st, double& sa, double& ca) {
      const double num = fma(-dnum, static_cast<double>(st), num0);
      const double rr = fma(-rint(num * inv_m2), m2, num);
      sincospi(rr * inv_m2, &sa, &ca);
    };
    double sa = 0.0, ca = 1.0;
    int st = 0;
    // two steps per iteration (seeds fall on even steps), so that their arithmetic overlaps
    for (; st + 1 < ns; st += 2) {
      if ((st & 15) == 0) seed(st, sa, ca);
      const double sb = sa * c4 - ca * s4, cb = ca * c4 + sa * s4;
      const double x0 = next_input(), x1 = next_input();
      const double w0 = next_weight(sa), w1 = next_weight(sb);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(w0, x0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(w1, x1, acc, 0, 0, 0);
      sa = sb * c4 - cb * s4;
      ca = cb * c4 + sb * s4;
    }
    if (st < ns) {
      if ((st & 15) == 0) seed(st, sa, ca);
      const double x0 = next_input();
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(next_weight(sa), x0, acc, 0, 0, 0);
    }
  }
  // lane holds rows 4 u + kq of image img
  const int quarter = ni / 4;
  const int rr = ih ? nrings - 1 - r : r;
  if (ih && rr == r) return;
  double* yr = y + ldu(ldu(a.rstart)[rr]);
  const bool add = rr >= a.belt_lo && rr <= a.belt_hi;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ao = a0 + 4 * u + kq;
    if (ao >= F) continue;
    if (ifl && ((2 * ao + ci) % quarter) == 0) continue;   // reflected image repeats a rotated one
    int P = ifl ? (ni - ao - ci + iq * quarter) : (ao + iq * quarter);
    P %= ni;
    if (P < 0) P += ni;
    const double v = a.omega * acc[u];
    yr[P] = add ? yr[P] + v : v;
  }
}

__global__ __launch_bounds__(kTile) void pair_count_kernel(PairArgs a,
                                                           unsigned long long* __restrict__ total) {
  __shared__ unsigned long long s_red[kTile];
  using convreal::ldu;
  const int tile = convreal::xcd_remap(blockIdx.x, a.ntiles);
  const int r = ldu(ldu(a.tile_ring)[tile]);
  const int ai = ldu(ldu(a.tile_a0)[tile]) + static_cast<int>(threadIdx.x);
  unsigned long long cnt = 0;
  if (ai < ldu(ldu(a.rn)[r])) cnt = count_pixel(a, r, ai);
  s_red[threadIdx.x] = cnt;
  __syncthreads();
  for (int w = kTile / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(total, s_red[0]);
}

PairArgs make_args(const conv_real_plan* p, bool remainder) {
  PairArgs a;
  a.table = p->d_table;
  a.coef = p->d_coef64;
  a.rn = p->d_rn;
  a.rc = p->d_rc;
  a.rstart = p->d_rstart;
  a.rcd = p->d_rcd;
  a.rsd = p->d_rsd;
  a.pj = p->d_pj;
  a.pA = p->d_pA;
  a.pB = p->d_pB;
  a.phw = p->d_phw;
  a.cpair = nullptr;
  if (remainder) {
    a.off = p->d_rest_off;
    a.idx = p->d_rest_idx;
    a.tile_ring = p->d_rtile_ring;
    a.tile_a0 = p->d_rtile_a0;
    a.ntiles = p->n_rtiles;
    a.accumulate_belt = 1;
  } else {
    a.off = p->d_poff;
    a.idx = nullptr;
    a.tile_ring = p->d_tile_ring;
    a.tile_a0 = p->d_tile_a0;
    a.ntiles = p->ntiles;
    a.accumulate_belt = 0;
  }
  a.belt_lo = p->belt_lo;
  a.belt_hi = p->belt_hi;
  a.n_tab = p->n_tab;
  a.inv_h = p->inv_h;
  a.dcut2 = p->dcut2;
  a.omega = p->omega;
  a.npix = p->npix;
  return a;
}

// One launch of the accumulate kernel over up to kMaxMaps maps: as many workgroups as can be
// resident at once (each stages the table once), at most one per kGroups tiles.
template <bool kCoef, int kMaxMaps, typename T>
hipError_t launch_accumulate(const PairArgs& a, const T* x, T* y, int nm, size_t lds, hipStream_t st) {
  const auto kern = pair_accumulate_kernel<kCoef, kMaxMaps, T>;
  int dev = 0, ncu = 256, per = 1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kTile * kGroups, lds)) != hipSuccess) return e;
  if (per < 1) per = 1;
  const long long want = (static_cast<long long>(a.ntiles) + kGroups - 1) / kGroups;
  const long long grid = want < static_cast<long long>(ncu) * per ? want : static_cast<long long>(ncu) * per;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(kTile * kGroups), lds, st, a, x, y, nm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loop(const conv_real_plan* p, const PairArgs& a, const T* x, T* y, int nmaps, hipStream_t st,
                       const char* name, long long pairs_per_map) {
  constexpr int kChunk = 4;
  if (a.ntiles == 0) return hipSuccess;
  // the coefficient form when the plan holds it (n_tab - 2 <= kCoefMaxSegs), else the nodes
  const bool coef = a.coef != nullptr;
  const size_t lds = coef ? sizeof(double) * 4 * static_cast<size_t>(a.n_tab - 2)
                          : sizeof(double) * static_cast<size_t>(a.n_tab);
  for (int m0 = 0; m0 < nmaps; m0 += kChunk) {
    const int nm = nmaps - m0 < kChunk ? nmaps - m0 : kChunk;
    const T* xi = x + static_cast<size_t>(m0) * p->npix;
    T* yo = y + static_cast<size_t>(m0) * p->npix;
    hipError_t e;
    if (coef)
      e = nm == 1 ? launch_accumulate<true, 1, T>(a, xi, yo, nm, lds, st)
                  : launch_accumulate<true, kChunk, T>(a, xi, yo, nm, lds, st);
    else
      e = nm == 1 ? launch_accumulate<false, 1, T>(a, xi, yo, nm, lds, st)
                  : launch_accumulate<false, kChunk, T>(a, xi, yo, nm, lds, st);
    if (e != hipSuccess) return e;
    convreal::mark(p, st, name, pairs_per_map * nm);
  }
  return hipSuccess;
}

}  // namespace

namespace convreal {

hipError_t launch_pair_count(const conv_real_plan* p, bool remainder, hipStream_t st) {
  const PairArgs a = make_args(p, remainder);
  if (a.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(pair_count_kernel, dim3(a.ntiles), dim3(kTile), 0, st, a, p->d_count);
  return hipGetLastError();
}

hipError_t launch_pair_accumulate(const conv_real_plan* p, const void* x, void* y, int nmaps,
                                  hipStream_t st) {
  const PairArgs a = make_args(p, false);
  if (p->precision == CONV_REAL_F64)
    return launch_loop(p, a, static_cast<const double*>(x), static_cast<double*>(y), nmaps, st,
                       "pair_accumulate_kernel<double>", p->pairs);
  return launch_loop(p, a, static_cast<const float*>(x), static_cast<float*>(y), nmaps, st,
                     "pair_accumulate_kernel<float>", p->pairs);
}

hipError_t launch_remainder_f64(const conv_real_plan* p, const double* x, double* y, int nmaps, hipStream_t st) {
  const PairArgs a = make_args(p, true);
  return launch_loop(p, a, x, y, nmaps, st, "pair_accumulate_kernel<double> (cap-touching pairs)", p->pairs_rest);
}

hipError_t launch_cap_mfma64(const conv_real_plan* p, const double* x, double* y, int nmaps, hipStream_t st) {
  PairArgs a = make_args(p, true);
  a.tile_ring = p->d_mtile_ring;
  a.tile_a0 = p->d_mtile_a0;
  a.cpair = p->d_fft_cpair;
  a.ntiles = p->n_mtiles;
  if (a.ntiles == 0) return hipSuccess;
  const bool coef = a.coef != nullptr;
  const size_t lds = coef ? sizeof(double) * 4 * static_cast<size_t>(a.n_tab - 2) : sizeof(double) * static_cast<size_t>(a.n_tab);
  const unsigned grid = static_cast<unsigned>((a.ntiles + kMfmaWaves - 1) / kMfmaWaves);
  for (int m = 0; m < nmaps; ++m) {
    const size_t off = static_cast<size_t>(m) * static_cast<size_t>(p->npix);
    if (coef)
      hipLaunchKernelGGL(cap_mfma64_kernel<true>, dim3(grid), dim3(64 * kMfmaWaves), lds, st, a, x + off, y + off,
                         p->nrings);
    else
      hipLaunchKernelGGL(cap_mfma64_kernel<false>, dim3(grid), dim3(64 * kMfmaWaves), lds, st, a, x + off, y + off,
                         p->nrings);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    convreal::mark(p, st, "cap_mfma64_kernel (cap-touching pairs, FP64 matrix cores)", p->pairs_rest);
  }
  return hipSuccess;
}

hipError_t launch_remainder(const conv_real_plan* p, const float* x, float* y, int nmaps,
                            hipStream_t st) {
  const PairArgs a = make_args(p, true);
  return launch_loop(p, a, x, y, nmaps, st, "pair_accumulate_kernel<float> (cap pairs)", p->pairs_rest);
}

}  // namespace convreal
