// pair_accumulate: every pixel pair evaluated and accumulated in FP64.
//
//   y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) x_q
//
// One thread per output pixel a of ring i; a workgroup owns a tile of up to 256 consecutive pixels
// of one ring, and the kernel table sits in LDS. For each listed neighbour ring j (from the
// ring_window pass) the thread walks the candidate pixels b of its azimuthal window. The
// half-angle alpha = (phi_a - phi_b) / 2 = (pi / 2) * num / (n_i n_j) has the exact integer
// numerator num = (2a + c_i) n_j - (2b + c_j) n_i; sin(alpha) is seeded from that numerator and
// advanced by the rotation alpha -> alpha - pi / n_j from one pixel to the next (re-seeded every
// 64 steps). The chord is d^2 = A_ij + B_ij sin^2(alpha); pairs with d^2 <= d_cut^2 are
// interpolated from the table and accumulated in FP64.
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

struct PairArgs {
  const double* table;
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

template <bool kCount, int kMaxMaps, typename T>
__device__ __forceinline__ void pair_loop(const PairArgs& a, const double* __restrict__ s_tab, int r,
                                          int ai, const T* __restrict__ x, int nm, double* acc,
                                          unsigned long long* cnt) {
  const int ni = a.rn[r];
  const long long twoa_ci = 2LL * ai + a.rc[r];
  const long long k0 = a.off[r];
  const long long k1 = a.off[r + 1];
  for (long long kk = k0; kk < k1; ++kk) {
    const long long k = a.idx ? a.idx[kk] : kk;
    const int j = a.pj[k];
    const int nj = a.rn[j];
    const long long cj = a.rc[j];
    const long long sj = a.rstart[j];
    const double A = a.pA[k];
    const double B = a.pB[k];
    const double hw = a.phw[k];
    // window centre in pixels of ring j: b_c = ((2a + c_i) n_j / n_i - c_j) / 2
    const long long bc2 = twoa_ci * nj - cj * ni;
    const double bc = static_cast<double>(bc2) / (2.0 * ni);
    long long blo, nb;
    if (2.0 * hw >= static_cast<double>(nj)) {
      blo = static_cast<long long>(floor(bc)) - nj / 2;
      nb = nj;
    } else {
      blo = static_cast<long long>(ceil(bc - hw - 1e-7));
      const long long bhi = static_cast<long long>(floor(bc + hw + 1e-7));
      nb = bhi - blo + 1;
      if (nb > nj) nb = nj;
    }
    if (nb <= 0) continue;
    const long long M = static_cast<long long>(ni) * nj;
    const double cd = a.rcd[j];
    const double sd = a.rsd[j];
    int bm = static_cast<int>(((blo % nj) + nj) % nj);
    double sa = 0.0, ca = 1.0;
    for (long long t = 0; t < nb; ++t) {
      if ((t & 63) == 0) {
        long long num = twoa_ci * nj - (2 * (blo + t) + cj) * ni;
        const long long m2 = 2 * M;
        num %= m2;
        if (num > M) num -= m2;
        else if (num <= -M) num += m2;
        sincos(static_cast<double>(num) * (M_PI / 2.0) / static_cast<double>(M), &sa, &ca);
      }
      const double d2 = fma(B, sa * sa, A);
      if (d2 <= a.dcut2) {
        if constexpr (kCount) {
          *cnt += 1;
        } else {
          const double kt = convreal::interp_f64(s_tab, a.n_tab, sqrt(d2), a.inv_h);
          const T* xp = x + sj + bm;
#pragma unroll
          for (int m = 0; m < kMaxMaps; ++m)
            if (m < nm) acc[m] = fma(kt, static_cast<double>(xp[m * a.npix]), acc[m]);
        }
      }
      const double sa2 = sa * cd - ca * sd;
      ca = ca * cd + sa * sd;
      sa = sa2;
      if (++bm == nj) bm = 0;
    }
  }
}

template <int kMaxMaps, typename T>
__global__ __launch_bounds__(kTile) void pair_accumulate_kernel(PairArgs a, const T* __restrict__ x,
                                                                T* __restrict__ y, int nm) {
  extern __shared__ double s_tab[];
  const int tile = convreal::xcd_remap(blockIdx.x, a.ntiles);
  for (int k = threadIdx.x; k < a.n_tab; k += blockDim.x) s_tab[k] = a.table[k];
  __syncthreads();
  const int r = a.tile_ring[tile];
  const int ai = a.tile_a0[tile] + threadIdx.x;
  if (ai >= a.rn[r]) return;
  double acc[kMaxMaps];
#pragma unroll
  for (int m = 0; m < kMaxMaps; ++m) acc[m] = 0.0;
  pair_loop<false, kMaxMaps, T>(a, s_tab, r, ai, x, nm, acc, nullptr);
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

__global__ __launch_bounds__(kTile) void pair_count_kernel(PairArgs a,
                                                           unsigned long long* __restrict__ total) {
  __shared__ unsigned long long s_red[kTile];
  const int tile = convreal::xcd_remap(blockIdx.x, a.ntiles);
  const int r = a.tile_ring[tile];
  const int ai = a.tile_a0[tile] + threadIdx.x;
  unsigned long long cnt = 0;
  if (ai < a.rn[r]) pair_loop<true, 1, float>(a, nullptr, r, ai, nullptr, 0, nullptr, &cnt);
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
  a.rn = p->d_rn;
  a.rc = p->d_rc;
  a.rstart = p->d_rstart;
  a.rcd = p->d_rcd;
  a.rsd = p->d_rsd;
  a.pj = p->d_pj;
  a.pA = p->d_pA;
  a.pB = p->d_pB;
  a.phw = p->d_phw;
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

template <typename T>
hipError_t launch_loop(const conv_real_plan* p, const PairArgs& a, const T* x, T* y, int nmaps,
                       size_t lds, hipStream_t st, const char* name, long long pairs_per_map) {
  constexpr int kChunk = 4;
  if (a.ntiles == 0) return hipSuccess;
  for (int m0 = 0; m0 < nmaps; m0 += kChunk) {
    const int nm = nmaps - m0 < kChunk ? nmaps - m0 : kChunk;
    const T* xi = x + static_cast<size_t>(m0) * p->npix;
    T* yo = y + static_cast<size_t>(m0) * p->npix;
    if (nm == 1)
      hipLaunchKernelGGL((pair_accumulate_kernel<1, T>), dim3(a.ntiles), dim3(kTile), lds, st, a, xi, yo, nm);
    else
      hipLaunchKernelGGL((pair_accumulate_kernel<kChunk, T>), dim3(a.ntiles), dim3(kTile), lds, st, a, xi, yo, nm);
    hipError_t e = hipGetLastError();
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
  const size_t lds = sizeof(double) * static_cast<size_t>(p->n_tab);
  if (p->precision == CONV_REAL_F64)
    return launch_loop(p, a, static_cast<const double*>(x), static_cast<double*>(y), nmaps, lds, st,
                       "pair_accumulate_kernel<double>", p->pairs);
  return launch_loop(p, a, static_cast<const float*>(x), static_cast<float*>(y), nmaps, lds, st,
                     "pair_accumulate_kernel<float>", p->pairs);
}

hipError_t launch_remainder(const conv_real_plan* p, const float* x, float* y, int nmaps,
                            hipStream_t st) {
  const PairArgs a = make_args(p, true);
  const size_t lds = sizeof(double) * static_cast<size_t>(p->n_tab);
  return launch_loop(p, a, x, y, nmaps, lds, st, "pair_accumulate_kernel<float> (cap pairs)",
                     p->pairs_rest);
}

}  // namespace convreal
