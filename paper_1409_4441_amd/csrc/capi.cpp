// C entry points of libconvreal: validation, plan construction, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace convreal {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

// HEALPix ring scheme with integer numerators (Gorski et al. 2005; library ordering):
//   caps, ring k from the nearer pole: 4k pixels, |z| = 1 - k^2/(3N^2), phi = (pi/2k)(a + 1/2)
//   belt, ring i = N..3N: 4N pixels, z = (2N - i) 2/(3N), phi = (pi/2N)(a + s/2), s = (i-N+1) mod 2
RingGrid make_ring_grid(int nside) {
  RingGrid g;
  const long long N = nside;
  const long long q = 3 * N * N;
  g.nside = nside;
  g.nrings = static_cast<int>(4 * N - 1);
  g.Z.resize(g.nrings);
  g.z.resize(g.nrings);
  g.s.resize(g.nrings);
  g.n.resize(g.nrings);
  g.c.resize(g.nrings);
  g.start.resize(g.nrings);
  long long pos = 0;
  for (long long i = 1; i <= 4 * N - 1; ++i) {
    long long Z;
    int n, c;
    if (i < N) {
      Z = q - i * i;
      n = static_cast<int>(4 * i);
      c = 1;
    } else if (i <= 3 * N) {
      Z = 2 * N * (2 * N - i);
      n = static_cast<int>(4 * N);
      c = static_cast<int>((i - N + 1) & 1);
    } else {
      const long long k = 4 * N - i;
      Z = -(q - k * k);
      n = static_cast<int>(4 * k);
      c = 1;
    }
    const int r = static_cast<int>(i - 1);
    g.Z[r] = Z;
    g.z[r] = static_cast<double>(Z) / static_cast<double>(q);
    // (q - Z)(q + Z) is exact in 64-bit integers for nside <= 8192.
    const long long S = (q - Z) * (q + Z);
    g.s[r] = std::sqrt(static_cast<double>(S)) / static_cast<double>(q);
    g.n[r] = n;
    g.c[r] = c;
    g.start[r] = pos;
    pos += n;
  }
  g.npix = pos;
  return g;
}

// Squared chord between rings r and t at equal azimuth: (z_r - z_t)^2 + (s_r - s_t)^2,
// with both differences formed from exact integer numerators.
static double ring_gap2(const RingGrid& g, int r, int t) {
  const double q = 3.0 * g.nside * static_cast<double>(g.nside);
  const long long dZ = g.Z[r] - g.Z[t];
  const long long sZ = g.Z[r] + g.Z[t];
  const double dz = static_cast<double>(dZ) / q;
  // s_r - s_t = (s_r^2 - s_t^2) / (s_r + s_t) = -(Z_r - Z_t)(Z_r + Z_t) / (q^2 (s_r + s_t))
  const double ds = -(static_cast<double>(dZ) * static_cast<double>(sZ)) / (q * q * (g.s[r] + g.s[t]));
  return dz * dz + ds * ds;
}

void neighbour_rings(const RingGrid& g, double dcut2, std::vector<int>& jlo, std::vector<int>& jhi) {
  // Slack so that rounding never drops a ring; the per-pair chord test is exact.
  const double lim = dcut2 * (1.0 + 1e-9) + 1e-300;
  jlo.assign(g.nrings, 0);
  jhi.assign(g.nrings, 0);
  for (int r = 0; r < g.nrings; ++r) {
    int lo = r, hi = r;
    while (lo - 1 >= 0 && ring_gap2(g, r, lo - 1) <= lim) --lo;
    while (hi + 1 < g.nrings && ring_gap2(g, r, hi + 1) <= lim) ++hi;
    jlo[r] = lo;
    jhi[r] = hi;
  }
}

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  (void)hipGetLastError();  // clear the runtime's sticky error so that later calls are not blamed
  return e == hipErrorOutOfMemory ? CONV_REAL_ENOMEM : CONV_REAL_EHIP;
}

int check_device(int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
    return CONV_REAL_ENODEV;
  }
  *dev_out = dev;
  return CONV_REAL_OK;
}

}  // namespace convreal

using convreal::set_error;
using convreal::check_device;
using convreal::DeviceGuard;
using convreal::hip_fail;

namespace {

constexpr int kMagic = 0x43565231;  // "CVR1"
constexpr int kTile = 256;          // output pixels per workgroup of the plain kernel

bool finite_all(const double* v, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}


template <typename T>
hipError_t dev_alloc(conv_real_plan* p, T** out, size_t count) {
  *out = nullptr;
  if (count == 0) count = 1;
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, count * sizeof(T));
  if (e != hipSuccess) return e;
  p->owned.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return hipSuccess;
}

template <typename T>
hipError_t dev_upload(conv_real_plan* p, T** out, const std::vector<T>& host) {
  hipError_t e = dev_alloc(p, out, host.size());
  if (e != hipSuccess) return e;
  if (host.empty()) return hipSuccess;
  return hipMemcpy(*out, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
}

void free_plan(conv_real_plan* p) {
  for (void* ptr : p->owned) (void)hipFree(ptr);
  p->owned.clear();
  p->magic = 0;
  delete p;
}

// Work items of one map for the persistent kernel, in the order the tuning asks for. An item is
// (slot, kind << 30 | index): kind 0 = belt (band x pixel segment), kind 1 = cap (4 tiles).
struct QueueItem {
  double cost;
  int kind;
  int idx;
};

// The plan's belt items (band-major) and cap items (ring-major, 4 tiles each) with their costs.
// with_belt = false: cap items only (a mixed plan on the ring-FFT method, whose belt ring pairs go
// through the ring FFTs).
void plan_items(const conv_real_plan* p, const convreal::Tuning& t, std::vector<QueueItem>& belt,
                std::vector<QueueItem>& cap, bool with_belt = true) {
  if (p->belt_enabled && with_belt) {
    const int nsegs = (4 * p->nside + t.seg - 1) / t.seg;
    for (int b = 0; b < p->belt_nbands; ++b)
      for (int s = 0; s < nsegs; ++s) belt.push_back({p->cost_belt[b] * (t.seg / 64), 0, b * nsegs + s});
  }
  // a stored weight is a load, about a third of the work of evaluating it
  const double cap_scale = p->d_wstore ? 0.35 : 1.0;
  if (p->cap_mode)
    for (int k = 0; k < static_cast<int>(p->cost_cap.size()); ++k) cap.push_back({p->cost_cap[k] * cap_scale, 1, k});
}

// Launch order of a queue and its chunk offsets. Orders 0 and 1: one chunk, all items by
// decreasing cost (0) or belt and cap items alternating, each by decreasing cost (1). Order 2: one
// chunk per XCD, each holding a contiguous, cost-balanced range of the belt items and one of the cap
// items in the order given (neighbouring bands and rings, whose input rings overlap, share an L2),
// alternating as in order 1. Orders 3 and 4: roles (see below).
template <typename E, typename Cost, typename Kind>
std::vector<int> order_queue(const std::vector<E>& belt_in, const std::vector<E>& cap_in, int order, Cost cost,
                             Kind kind, std::vector<E>& out) {
  auto desc = [&](const E& a, const E& b) { return cost(a) > cost(b); };
  out.clear();
  if (order == 2) {
    const int nc = convreal::kXcds;
    std::vector<std::vector<E>> ch(nc);
    for (const std::vector<E>* v : {&belt_in, &cap_in}) {
      double total = 0.0, acc = 0.0;
      for (const E& e : *v) total += cost(e);
      for (const E& e : *v) {
        const int c = total > 0.0 ? std::min(nc - 1, static_cast<int>(acc / total * nc)) : 0;
        ch[c].push_back(e);
        acc += cost(e);
      }
    }
    // within a chunk, belt and cap items alternate (each kind by decreasing cost), so that both
    // kinds share every CU of the XCD
    std::vector<int> off(1, 0);
    for (std::vector<E>& c : ch) {
      std::vector<E> bl, cp;
      for (const E& e : c) (kind(e) == 0 ? bl : cp).push_back(e);
      std::stable_sort(bl.begin(), bl.end(), desc);
      std::stable_sort(cp.begin(), cp.end(), desc);
      size_t i = 0, j = 0;
      while (i < bl.size() || j < cp.size()) {
        if (i < bl.size()) out.push_back(bl[i++]);
        if (j < cp.size()) out.push_back(cp[j++]);
      }
      off.push_back(static_cast<int>(out.size()));
    }
    return off;
  }
  std::vector<E> belt = belt_in, cap = cap_in;
  std::stable_sort(belt.begin(), belt.end(), desc);
  if (order == 4) {
    // roles as in order 3 for the belt (chunk 0), the cap items in ring order split into one
    // cost-balanced run of neighbouring rings per XCD (chunks 1..8): the cap workgroups of an XCD
    // start on rings whose input rings overlap, so their re-reads stay in that XCD's L2
    const int nc = convreal::kXcds;
    double total = 0.0, acc = 0.0;
    for (const E& e : cap) total += cost(e);
    std::vector<std::vector<E>> ch(nc);
    for (const E& e : cap) {
      const int c = total > 0.0 ? std::min(nc - 1, static_cast<int>(acc / total * nc)) : 0;
      ch[c].push_back(e);
      acc += cost(e);
    }
    out = belt;
    std::vector<int> off{0, static_cast<int>(out.size())};
    for (const std::vector<E>& c : ch) {
      out.insert(out.end(), c.begin(), c.end());
      off.push_back(static_cast<int>(out.size()));
    }
    return off;
  }
  std::stable_sort(cap.begin(), cap.end(), desc);
  if (order == 3) {
    // roles: chunk 0 holds the belt items by decreasing cost, chunks 1 and 2 the cap items dealt
    // alternately; the kernel gives the first workgroup of every CU chunk 0 and the other two chunks
    // 1 and 2 to start with
    std::vector<E> c1, c2;
    for (size_t k = 0; k < cap.size(); ++k) (k % 2 ? c2 : c1).push_back(cap[k]);
    out = belt;
    out.insert(out.end(), c1.begin(), c1.end());
    out.insert(out.end(), c2.begin(), c2.end());
    return std::vector<int>{0, static_cast<int>(belt.size()), static_cast<int>(belt.size() + c1.size()),
                            static_cast<int>(out.size())};
  }
  if (order == 1) {
    size_t i = 0, j = 0;
    while (i < belt.size() || j < cap.size()) {
      if (i < belt.size()) out.push_back(belt[i++]);
      if (j < cap.size()) out.push_back(cap[j++]);
    }
  } else {
    out = belt;
    out.insert(out.end(), cap.begin(), cap.end());
    std::stable_sort(out.begin(), out.end(), desc);
  }
  return std::vector<int>{0, static_cast<int>(out.size())};
}

// The kernel maps every counter value of chunk c to an item of chunk_off[c] .. chunk_off[c+1] - 1
// and reads that item and its map slot, so the offsets must cover exactly the uploaded items.
bool queue_ok(const std::vector<int>& off, size_t n_items) {
  if (off.size() < 2 || off.size() - 1 > static_cast<size_t>(convreal::kMaxChunks) || off.front() != 0) return false;
  for (size_t c = 1; c < off.size(); ++c)
    if (off[c] < off[c - 1]) return false;
  return static_cast<size_t>(off.back()) == n_items;
}

void release(conv_real_plan* p, void* ptr) {
  if (!ptr) return;
  for (auto it = p->owned.begin(); it != p->owned.end(); ++it)
    if (*it == ptr) {
      (void)hipFree(ptr);
      p->owned.erase(it);
      return;
    }
}

hipError_t build_items(conv_real_plan* p) {
  std::vector<QueueItem> belt, cap, q;
  plan_items(p, p->tune, belt, cap, p->method == CONV_REAL_METHOD_DIRECT);
  const std::vector<int> off = order_queue(belt, cap, p->tune.order, [](const QueueItem& e) { return e.cost; },
                                           [](const QueueItem& e) { return e.kind; }, q);
  std::vector<int2> items(q.size());
  for (size_t k = 0; k < q.size(); ++k) items[k] = make_int2(0, (q[k].kind << 30) | q[k].idx);
  if (!queue_ok(off, items.size())) return hipErrorInvalidValue;
  release(p, p->d_items);
  release(p, p->d_qchunk_off);
  p->d_items = nullptr;
  p->d_qchunk_off = nullptr;
  p->n_items = static_cast<int>(items.size());
  p->n_qchunks = static_cast<int>(off.size()) - 1;
  hipError_t e = dev_upload(p, &p->d_qchunk_off, off);
  if (e != hipSuccess || items.empty()) return e;
  return dev_upload(p, &p->d_items, items);
}

// The cap tile list for tiles of `rows` output pixels (16 on the fly, 16 kStoreBlocks with a store):
// tiles, per-item costs (4 tiles per item, one per wave), device copies and the host descriptor.
hipError_t build_cap_tiles(conv_real_plan* p, int rows) {
  std::vector<int> ring, a0s;
  for (int r = 0; r < static_cast<int>(p->cap_F.size()); ++r)
    for (int a0 = 0; a0 < p->cap_F[r]; a0 += rows) {
      ring.push_back(r);
      a0s.push_back(a0);
    }
  release(p, p->d_citem_ring);
  release(p, p->d_citem_a0);
  p->d_citem_ring = nullptr;
  p->d_citem_a0 = nullptr;
  p->n_citems = static_cast<int>(ring.size());
  p->cap_rows = rows;
  p->cost_cap.clear();
  for (int t = 0; t < p->n_citems; t += 4) {
    double c = 0.0;
    for (int u = t; u < std::min(t + 4, p->n_citems); ++u) c = std::max(c, p->cap_ring_cost[ring[u]]);
    p->cost_cap.push_back(c * (rows / 16));
  }
  hipError_t e = hipSuccess;
  if (!ring.empty() && ((e = dev_upload(p, &p->d_citem_ring, ring)) != hipSuccess ||
                        (e = dev_upload(p, &p->d_citem_a0, a0s)) != hipSuccess))
    return e;
  p->h_desc.n_citems = p->n_citems;
  p->h_desc.citem_ring = p->d_citem_ring;
  p->h_desc.citem_a0 = p->d_citem_a0;
  return hipSuccess;
}

// Mixed path set-up: belt bands, window width, split-FP16 weight blocks, and the list of ring
// pairs left to the per-pair kernel (every pair touching a polar cap).
hipError_t setup_mixed(conv_real_plan* p, const convreal::RingGrid& g, const std::vector<int>& jlo,
                       const std::vector<int>& jhi, const std::vector<long long>& poff,
                       const std::vector<int>& pj) {
  hipError_t e;
  const int N = p->nside;
  const int blo = N - 1, bhi = 3 * N - 1;  // belt rings, 0-based
  std::vector<double> hw(p->npairs_ring);
  if ((e = hipMemcpy(hw.data(), p->d_phw, sizeof(double) * hw.size(), hipMemcpyDeviceToHost)) != hipSuccess)
    return e;
  // Bands of 16 belt output rings; per (band, input ring j) the tight range of window offsets
  // m = b - a over the band's rows, from the same windows the per-pair kernel walks:
  // m in [ceil(delta/2 - hw - eps), floor(delta/2 + hw + eps)], delta = c_i - c_j.
  const int nbelt = bhi - blo + 1;
  const int nbands = (nbelt + 15) / 16;
  std::vector<int> band_nj(nbands), band_woff(nbands);
  std::vector<int> blk_j, blk_koff, blk_nk, blk_mlo, chunk_band, chunk_j, chunk_m0;
  bool ok = true;
  int nk_max = 1;
  for (int b = 0; b < nbands && ok; ++b) {
    const int r0 = blo + 16 * b;
    const int r1 = std::min(r0 + 15, bhi);
    int lo = jlo[r0], hi = jhi[r0];
    for (int r = r0; r <= r1; ++r) {
      lo = std::min(lo, jlo[r]);
      hi = std::max(hi, jhi[r]);
    }
    lo = std::max(lo, blo);
    hi = std::min(hi, bhi);
    band_woff[b] = static_cast<int>(blk_nk.size());
    for (int j = lo; j <= hi && ok; ++j) {
      int mmin = 1 << 30, mmax = -(1 << 30);
      for (int r = r0; r <= r1; ++r) {
        if (j < jlo[r] || j > jhi[r]) continue;
        const long long k = poff[r] + (j - jlo[r]);
        if (2.0 * hw[k] >= 4.0 * N) { ok = false; break; }  // window wraps the whole ring
        const double half_delta = 0.5 * (g.c[r] - g.c[j]);
        mmin = std::min(mmin, static_cast<int>(std::ceil(half_delta - hw[k] - 1e-7)));
        mmax = std::max(mmax, static_cast<int>(std::floor(half_delta + hw[k] + 1e-7)));
      }
      if (!ok) break;
      if (mmax < mmin) { mmin = 0; mmax = 0; }
      const int nk = (mmax - mmin + 1 + 31) / 32;
      if (32 * nk > 4 * N) { ok = false; break; }
      // a window of more than kBeltBlockChunks K-chunks goes in consecutive sub-blocks of the same
      // input ring, each staged and multiplied like a ring of its own (the LDS stage holds one)
      for (int q0 = 0; q0 < nk; q0 += convreal::kBeltBlockChunks) {
        const int nks = std::min(convreal::kBeltBlockChunks, nk - q0);
        const int m0 = mmin + 32 * q0;
        nk_max = std::max(nk_max, nks);
        blk_j.push_back(j);
        blk_koff.push_back(static_cast<int>(chunk_band.size()));
        blk_nk.push_back(nks);
        blk_mlo.push_back(m0);
        for (int q = 0; q < nks; ++q) {
          chunk_band.push_back(b);
          chunk_j.push_back(j);
          chunk_m0.push_back(m0 + 32 * q);
        }
      }
    }
    band_nj[b] = static_cast<int>(blk_nk.size()) - band_woff[b];
  }
  p->belt_enabled = ok ? 1 : 0;

  // weight scale: power of two with Omega * max|T| * s_w < 2^12 (interpolation overshoot stays
  // far below the FP16 maximum)
  std::vector<double> tab(p->n_tab);
  if ((e = hipMemcpy(tab.data(), p->d_table, sizeof(double) * p->n_tab, hipMemcpyDeviceToHost)) != hipSuccess)
    return e;
  double tmax = 0.0;
  for (double v : tab) tmax = std::max(tmax, std::fabs(v));
  int ex = 0;
  std::frexp(std::max(tmax * p->omega, 1e-300), &ex);
  p->belt_sw = std::ldexp(1.0, 12 - ex);

  if (p->belt_enabled) {
    p->belt_lo = blo;
    p->belt_hi = bhi;
    p->belt_nk = nk_max;
    p->belt_nbands = nbands;
    p->belt_nsegs = (4 * N + 255) / 256;
    p->n_wblk = static_cast<long long>(blk_nk.size());
    p->n_chunks = static_cast<long long>(chunk_band.size());
    if ((e = dev_upload(p, &p->d_blk_j, blk_j)) != hipSuccess ||
        (e = dev_upload(p, &p->d_band_nj, band_nj)) != hipSuccess ||
        (e = dev_upload(p, &p->d_band_woff, band_woff)) != hipSuccess ||
        (e = dev_upload(p, &p->d_blk_koff, blk_koff)) != hipSuccess ||
        (e = dev_upload(p, &p->d_blk_nk, blk_nk)) != hipSuccess ||
        (e = dev_upload(p, &p->d_blk_mlo, blk_mlo)) != hipSuccess ||
        (e = dev_upload(p, &p->d_chunk_band, chunk_band)) != hipSuccess ||
        (e = dev_upload(p, &p->d_chunk_j, chunk_j)) != hipSuccess ||
        (e = dev_upload(p, &p->d_chunk_m0, chunk_m0)) != hipSuccess ||
        (e = dev_alloc(p, &p->d_wt, static_cast<size_t>(p->n_chunks) * 1024)) != hipSuccess ||
        (e = convreal::build_belt_weights(p)) != hipSuccess)
      return e;
  } else {
    p->belt_lo = 1;
    p->belt_hi = 0;
  }
  if ((e = dev_alloc(p, &p->d_amax, convreal::kMaxMixedMaps)) != hipSuccess) return e;

  std::vector<long long> roff(g.nrings + 1, 0), ridx;
  std::vector<int> rtile_ring, rtile_a0;
  for (int r = 0; r < g.nrings; ++r) {
    const bool belt_row = p->belt_enabled && r >= blo && r <= bhi;
    for (long long k = poff[r]; k < poff[r + 1]; ++k)
      if (!belt_row || pj[k] < blo || pj[k] > bhi) ridx.push_back(k);
    roff[r + 1] = static_cast<long long>(ridx.size());
    if (roff[r + 1] > roff[r])
      for (int a0 = 0; a0 < g.n[r]; a0 += kTile) {
        rtile_ring.push_back(r);
        rtile_a0.push_back(a0);
      }
  }
  p->n_rtiles = static_cast<int>(rtile_ring.size());
  if ((e = dev_upload(p, &p->d_rest_off, roff)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rest_idx, ridx)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rtile_ring, rtile_ring)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rtile_a0, rtile_a0)) != hipSuccess)
    return e;

  // Cap-touching pairs on the matrix cores when the coefficient table fits in 64 KB of LDS.
  p->cap_mode = (p->n_tab - 2) * 16 <= 65536 ? 1 : 0;
  std::vector<int> ring_add(g.nrings, 0);
  if (p->cap_mode) {
    // 4-point Lagrange interpolant of segment k (nodes k-1..k+2, ghost T[-1] = T[1]) in the
    // monomial basis of the local coordinate f, scaled by Omega s_w.
    const int nseg = p->n_tab - 2;
    std::vector<float> coef(4 * static_cast<size_t>(nseg));
    const double sc = p->omega * p->belt_sw;
    for (int k = 0; k < nseg; ++k) {
      const double tm1 = tab[k == 0 ? 1 : k - 1], t0 = tab[k], t1 = tab[k + 1], t2 = tab[k + 2];
      coef[4 * k + 0] = static_cast<float>(sc * t0);
      coef[4 * k + 1] = static_cast<float>(sc * (-tm1 / 3.0 - t0 / 2.0 + t1 - t2 / 6.0));
      coef[4 * k + 2] = static_cast<float>(sc * (tm1 / 2.0 - t0 + t1 / 2.0));
      coef[4 * k + 3] = static_cast<float>(sc * (-tm1 / 6.0 + t0 / 2.0 - t1 / 2.0 + t2 / 6.0));
    }
    // cap tiles cover the symmetry group's fundamental domain [0, F) of every north-half output
    // ring that has cap-touching pairs (its mirror ring is produced alongside)
    std::vector<double>& ring_cost = p->cap_ring_cost;
    ring_cost.assign(g.nrings, 0.0);
    p->cap_F.assign(g.nrings, 0);
    for (int r = 0; r <= (g.nrings - 1) / 2; ++r) {
      if (roff[r + 1] == roff[r]) continue;
      p->cap_F[r] = (g.n[r] / 4 - g.c[r]) / 2 + 1;
      // estimated cycles of one 16-row tile: per neighbour ring, K-chunks x (weights + inputs) work
      double c = 0.0;
      for (long long kk = roff[r]; kk < roff[r + 1]; ++kk) {
        const long long k = ridx[kk];
        const int nj = g.n[pj[k]];
        const double K = std::min(static_cast<double>(nj) + 16.0 * nj / g.n[r], 16.0 * nj / g.n[r] + 2.0 * hw[k] + 2.0);
        c += std::ceil(K / 32.0) * 1200.0 + 150.0;
      }
      ring_cost[r] = c;
    }
    for (int r = 0; r < g.nrings; ++r)
      ring_add[r] = (p->belt_enabled && r >= blo && r <= bhi && roff[r + 1] > roff[r]) ? 1 : 0;
    // one record per cap-touching ring pair, in the order of the rest list
    std::vector<double> pA(p->npairs_ring), pB(p->npairs_ring);
    if ((e = hipMemcpy(pA.data(), p->d_pA, sizeof(double) * pA.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(pB.data(), p->d_pB, sizeof(double) * pB.size(), hipMemcpyDeviceToHost)) != hipSuccess)
      return e;
    std::vector<convreal::CapPair> cpair(ridx.size());
    for (int r = 0; r < g.nrings; ++r) {
      for (long long kk = roff[r]; kk < roff[r + 1]; ++kk) {
        const long long k = ridx[kk];
        const int j = pj[k];
        convreal::CapPair& c = cpair[kk];
        c.A = pA[k];
        c.B = pB[k];
        c.hw = hw[k];
        c.scale = M_PI / (2.0 * static_cast<double>(g.n[r]) * static_cast<double>(g.n[j]));
        c.xoff = g.start[j];
        c.xoff_m = g.start[g.nrings - 1 - j];
        c.nj = g.n[j];
        c.cj = g.c[j];
        c.whole = 2.0 * hw[k] >= static_cast<double>(g.n[j]) ? 1 : 0;
        c.pad = 0;
      }
    }
    if (!cpair.empty() && (e = dev_upload(p, &p->d_cpair, cpair)) != hipSuccess) return e;
    p->cap_nseg = nseg;
    if ((e = dev_upload(p, &p->d_coef, coef)) != hipSuccess || (e = build_cap_tiles(p, 16)) != hipSuccess) return e;
  }
  if ((e = dev_upload(p, &p->d_ring_add, ring_add)) != hipSuccess) return e;

  // belt band costs: per 16-pixel column block, K-chunks x 3 products x 16 cycles plus staging
  p->cost_belt.assign(p->belt_enabled ? p->belt_nbands : 0, 0.0);
  for (int b = 0; b < static_cast<int>(p->cost_belt.size()); ++b) {
    double c = 0.0;
    for (int jj = 0; jj < band_nj[b]; ++jj) c += blk_nk[band_woff[b] + jj] * 48.0 + 12.0;
    p->cost_belt[b] = c;
  }

  // rows receiving both contributions: one contiguous run of rings in each hemisphere
  convreal::MixedDesc d{};
  d.zero_lo[0] = d.zero_hi[0] = d.zero_lo[1] = d.zero_hi[1] = 0;
  int half = 0;
  for (int r = 0; r < g.nrings && half < 2; ++r) {
    if (!ring_add[r]) continue;
    int r1 = r;
    while (r1 + 1 < g.nrings && ring_add[r1 + 1]) ++r1;
    d.zero_lo[half] = g.start[r];
    d.zero_hi[half] = g.start[r1] + g.n[r1];
    ++half;
    r = r1;
  }
  d.rn = p->d_rn;
  d.rc = p->d_rc;
  d.rstart = p->d_rstart;
  d.nrings = g.nrings;
  d.ring_n = 4 * N;
  d.npix = p->npix;
  d.wt = p->d_wt;
  d.blk_j = p->d_blk_j;
  d.band_nj = p->d_band_nj;
  d.band_woff = p->d_band_woff;
  d.blk_koff = p->d_blk_koff;
  d.blk_nk = p->d_blk_nk;
  d.blk_mlo = p->d_blk_mlo;
  d.belt_lo = p->belt_lo;
  d.belt_hi = p->belt_hi;
  d.ring_add = p->d_ring_add;
  d.coef = p->d_coef;
  d.nseg = p->cap_nseg;
  d.n_citems = p->n_citems;
  d.citem_ring = p->d_citem_ring;
  d.citem_a0 = p->d_citem_a0;
  d.rest_off = p->d_rest_off;
  d.cpair = p->d_cpair;
  d.inv_h = p->inv_h;
  d.dcut2 = p->dcut2;
  d.inv_sw = static_cast<float>(1.0 / p->belt_sw);
  d.wstore = nullptr;
  d.wtile_off = nullptr;
  p->h_desc = d;
  std::vector<convreal::MixedDesc> dv(1, d);
  if ((e = dev_upload(p, &p->d_desc, dv)) != hipSuccess ||
      (e = dev_alloc(p, &p->d_counter, convreal::kMaxChunks)) != hipSuccess ||
      (e = convreal::set_lds_limits(p->cap_nseg)) != hipSuccess)
    return e;
  return build_items(p);
}

// Build (or drop) the cap weight store for `mode` (CONV_REAL_STORE_*), re-upload the descriptor and
// the work queue. Synchronous.
int set_weight_store(conv_real_plan* p, int mode) {
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "weight store: synchronise");
  release(p, p->d_wstore);
  release(p, p->d_wtile_off);
  p->d_wstore = nullptr;
  p->d_wtile_off = nullptr;
  p->wstore_groups = 0;
  p->h_desc.wstore = nullptr;
  p->h_desc.wtile_off = nullptr;
  p->wstore_mode = mode;
  int rc = CONV_REAL_OK;
  bool built = false;
  if (mode != CONV_REAL_STORE_OFF && p->cap_mode && !p->cap_F.empty()) {
    // the store is laid out over tiles of kStoreBlocks x 16 rows
    if ((e = build_cap_tiles(p, 16 * convreal::kStoreBlocks)) != hipSuccess) return hip_fail(e, "weight store: tiles");
  }
  if (mode != CONV_REAL_STORE_OFF && p->cap_mode && p->n_citems > 0) {
    long long* counts = nullptr;
    std::vector<long long> off(static_cast<size_t>(p->n_citems) + 1, 0);
    if ((e = hipMemcpy(p->d_desc, &p->h_desc, sizeof(p->h_desc), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = dev_alloc(p, &counts, static_cast<size_t>(p->n_citems))) != hipSuccess ||
        (e = convreal::cap_store_count(p, counts)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(off.data() + 1, counts, sizeof(long long) * p->n_citems, hipMemcpyDeviceToHost)) !=
            hipSuccess) {
      release(p, counts);
      return hip_fail(e, "weight store: count");
    }
    release(p, counts);
    // the count pass flags tiles whose inputs wrap around a ring in the high bits; the offsets keep
    // the flag beside the first group
    std::vector<long long> wraps(static_cast<size_t>(p->n_citems));
    for (int t = 0; t < p->n_citems; ++t) {
      wraps[t] = off[t + 1] & convreal::kTileWraps;
      off[t + 1] &= convreal::kTileOffsetMask;
    }
    for (int t = 0; t < p->n_citems; ++t) off[t + 1] += off[t];
    const long long n = off[p->n_citems];
    // 16-byte groups, every one written by the fill (at least one, so that the store is never empty)
    const size_t bytes = sizeof(uint4) * static_cast<size_t>(std::max(n, 1LL));
    bool build = true;
    if (mode == CONV_REAL_STORE_AUTO) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
      const double budget = std::min(64.0 * (1ull << 30), 0.4 * static_cast<double>(free_b));
      build = static_cast<double>(bytes) <= budget;
    }
    if (build) {
      off.pop_back();
      for (int t = 0; t < p->n_citems; ++t) off[t] |= wraps[t];
      if ((e = dev_alloc(p, &p->d_wstore, static_cast<size_t>(std::max(n, 1LL)))) != hipSuccess) {
        // the automatic mode falls back to evaluating on the fly
        if (mode == CONV_REAL_STORE_AUTO)
          (void)hipGetLastError();
        else
          rc = hip_fail(e, "weight store: allocation");
      } else if ((e = dev_upload(p, &p->d_wtile_off, off)) != hipSuccess ||
                 (e = convreal::cap_store_fill(p)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
        rc = hip_fail(e, "weight store: fill");
      } else {
        p->wstore_groups = n;
        p->h_desc.wstore = p->d_wstore;
        p->h_desc.wtile_off = p->d_wtile_off;
        built = true;
      }
      if (rc != CONV_REAL_OK) {
        release(p, p->d_wstore);
        release(p, p->d_wtile_off);
        p->d_wstore = nullptr;
        p->d_wtile_off = nullptr;
      }
    }
  }
  // without a store the weights are evaluated on the fly, over tiles of 16 rows
  if (!built && p->cap_mode && p->cap_rows != 16 && (e = build_cap_tiles(p, 16)) != hipSuccess)
    return hip_fail(e, "weight store: tiles");
  // Unless the caller chose the launch configuration: with a store the kernel needs no coefficient
  // table in LDS, so three workgroups with 256-pixel belt items fit a compute unit (and the kernel
  // is built for three waves per SIMD), one of them starting on belt items and two on cap items so
  // that every CU runs both kinds (at Nside 2048 7% faster than alternating the kinds in one queue,
  // 14% faster than by cost alone). Without a store the cap items need the coefficient table in
  // LDS; with three workgroups per CU it shares the belt stage's LDS (a workgroup reads it again after
  // a belt item), which keeps three workgroups per CU for tables up to 3413 segments and two up to
  // 4096 (after the stage, the table leaves room for two up to 2416 segments and one beyond): at
  // Nside 2048 with a 4096-node table, 30' 4.3 ms against 7.5 ms, 240' 109 ms against 171 ms.
  if (!p->tune_user) {
    p->tune.seg = 256;
    p->tune.wg_per_cu = 3;
    p->tune.order = 3;
  }
  if ((e = hipMemcpy(p->d_desc, &p->h_desc, sizeof(p->h_desc), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = build_items(p)) != hipSuccess)
    return hip_fail(e, "weight store: descriptor");
  return rc;
}

}  // namespace

extern "C" {

const char* conv_real_strerror(int code) {
  switch (code) {
    case CONV_REAL_OK: return "success";
    case CONV_REAL_EINVAL: return "invalid argument";
    case CONV_REAL_ENOMEM: return "out of memory";
    case CONV_REAL_EHIP: return "HIP runtime error";
    case CONV_REAL_EALIAS: return "input and output maps overlap";
    case CONV_REAL_ENODEV: return "no usable gfx950 device";
    default: return "unknown error";
  }
}

const char* conv_real_last_error(void) { return convreal::g_last_error.c_str(); }

int conv_real_tabulate(const double* k_ell, int lmax, double theta_cut, int n_tab, double* table) {
  if (!k_ell || !table) { set_error("conv_real_tabulate: NULL pointer"); return CONV_REAL_EINVAL; }
  if (lmax < 0 || lmax > CONV_REAL_MAX_LMAX) { set_error("conv_real_tabulate: lmax out of range"); return CONV_REAL_EINVAL; }
  if (!(theta_cut > 0.0) || !(theta_cut <= M_PI)) { set_error("conv_real_tabulate: theta_cut must be in (0, pi]"); return CONV_REAL_EINVAL; }
  if (n_tab < 4 || n_tab > CONV_REAL_MAX_NTAB) { set_error("conv_real_tabulate: n_tab out of range"); return CONV_REAL_EINVAL; }
  if (!finite_all(k_ell, lmax + 1)) { set_error("conv_real_tabulate: non-finite k_ell"); return CONV_REAL_EINVAL; }
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != CONV_REAL_OK) return rc;
  const double dcut = 2.0 * std::sin(0.5 * theta_cut);
  const double h = dcut / (n_tab - 3);
  hipError_t e = convreal::tabulate_device(k_ell, lmax, h, n_tab, table);
  if (e != hipSuccess) return hip_fail(e, "conv_real_tabulate");
  return CONV_REAL_OK;
}

int conv_real_init(conv_real_plan** plan, int nside, const double* table, int n_tab,
                   double theta_cut, int precision) {
  if (!plan) { set_error("conv_real_init: NULL plan pointer"); return CONV_REAL_EINVAL; }
  *plan = nullptr;
  if (!table) { set_error("conv_real_init: NULL table"); return CONV_REAL_EINVAL; }
  if (nside < 1 || nside > CONV_REAL_MAX_NSIDE) { set_error("conv_real_init: nside out of range"); return CONV_REAL_EINVAL; }
  if (n_tab < 4 || n_tab > CONV_REAL_MAX_NTAB) { set_error("conv_real_init: n_tab out of range"); return CONV_REAL_EINVAL; }
  if (!(theta_cut > 0.0) || !(theta_cut <= M_PI)) { set_error("conv_real_init: theta_cut must be in (0, pi]"); return CONV_REAL_EINVAL; }
  if (precision != CONV_REAL_F64 && precision != CONV_REAL_F32 && precision != CONV_REAL_MIXED) {
    set_error("conv_real_init: unknown precision"); return CONV_REAL_EINVAL;
  }
  if (!finite_all(table, n_tab)) { set_error("conv_real_init: non-finite table entry"); return CONV_REAL_EINVAL; }

  int dev = 0;
  int rc = check_device(&dev);
  if (rc != CONV_REAL_OK) return rc;
  // the fixed scratch of conv_real_apply_noalloc, located once per device (this device is current)
  hipError_t es = convreal::noalloc_scratch_resolve(dev);
  if (es != hipSuccess) return hip_fail(es, "conv_real_init: hipGetSymbolAddress of the no-alloc scratch");

  auto* p = new (std::nothrow) conv_real_plan();
  if (!p) { set_error("conv_real_init: host allocation failed"); return CONV_REAL_ENOMEM; }
  p->magic = kMagic;
  p->device = dev;
  p->nside = nside;
  p->precision = precision;
  p->n_tab = n_tab;
  p->theta_cut = theta_cut;
  p->dcut = 2.0 * std::sin(0.5 * theta_cut);
  // A cut of pi keeps every pair: no chord exceeds 2, and antipodal pairs must not be lost to
  // rounding of d^2 (or the sin^2 polynomial of the mixed path) at the tie d = d_cut = 2.
  p->dcut2 = theta_cut >= M_PI ? 4.0 * (1.0 + 1e-9) : p->dcut * p->dcut;
  p->h = p->dcut / (n_tab - 3);
  p->inv_h = 1.0 / p->h;
  p->npix = 12LL * nside * nside;
  p->omega = 4.0 * M_PI / static_cast<double>(p->npix);

  const convreal::RingGrid g = convreal::make_ring_grid(nside);
  p->nrings = g.nrings;
  std::vector<int> jlo, jhi;
  convreal::neighbour_rings(g, p->dcut2, jlo, jhi);

  std::vector<long long> poff(g.nrings + 1, 0);
  for (int r = 0; r < g.nrings; ++r) poff[r + 1] = poff[r] + (jhi[r] - jlo[r] + 1);
  p->npairs_ring = poff[g.nrings];
  std::vector<int> pi(p->npairs_ring), pj(p->npairs_ring);
  for (int r = 0; r < g.nrings; ++r)
    for (long long k = poff[r]; k < poff[r + 1]; ++k) {
      pi[k] = r;
      pj[k] = jlo[r] + static_cast<int>(k - poff[r]);
    }
  std::vector<double> rcd(g.nrings), rsd(g.nrings);
  for (int r = 0; r < g.nrings; ++r) {
    rcd[r] = std::cos(M_PI / g.n[r]);
    rsd[r] = std::sin(M_PI / g.n[r]);
  }
  std::vector<int> tile_ring, tile_a0;
  for (int r = 0; r < g.nrings; ++r)
    for (int a0 = 0; a0 < g.n[r]; a0 += kTile) {
      tile_ring.push_back(r);
      tile_a0.push_back(a0);
    }
  p->ntiles = static_cast<int>(tile_ring.size());
  std::vector<double> tab(table, table + n_tab);
  // per-segment coefficients of the interpolating cubic in f = t - k (nodes k-1..k+2, ghost node
  // T[-1] = T[1]) for the per-pair kernel, when they fit in 64 KB of LDS
  std::vector<double> coef64;
  if (n_tab - 2 <= convreal::kCoefMaxSegs) {
    coef64.resize(4 * static_cast<size_t>(n_tab - 2));
    for (int k = 0; k + 2 < n_tab; ++k) {
      const double tm1 = tab[k == 0 ? 1 : k - 1], t0 = tab[k], t1 = tab[k + 1], t2 = tab[k + 2];
      coef64[4 * k + 0] = t0;
      coef64[4 * k + 1] = -tm1 / 3.0 - t0 / 2.0 + t1 - t2 / 6.0;
      coef64[4 * k + 2] = tm1 / 2.0 - t0 + t1 / 2.0;
      coef64[4 * k + 3] = -tm1 / 6.0 + t0 / 2.0 - t1 / 2.0 + t2 / 6.0;
    }
  }

  hipError_t e = hipSuccess;
  if ((e = dev_upload(p, &p->d_table, tab)) != hipSuccess ||
      (!coef64.empty() && (e = dev_upload(p, &p->d_coef64, coef64)) != hipSuccess) ||
      (e = dev_upload(p, &p->d_rn, g.n)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rc, g.c)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rstart, g.start)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rcd, rcd)) != hipSuccess ||
      (e = dev_upload(p, &p->d_rsd, rsd)) != hipSuccess ||
      (e = dev_upload(p, &p->d_Z, g.Z)) != hipSuccess ||
      (e = dev_upload(p, &p->d_s, g.s)) != hipSuccess ||
      (e = dev_upload(p, &p->d_poff, poff)) != hipSuccess ||
      (e = dev_upload(p, &p->d_jlo, jlo)) != hipSuccess ||
      (e = dev_upload(p, &p->d_pi, pi)) != hipSuccess ||
      (e = dev_upload(p, &p->d_pj, pj)) != hipSuccess ||
      (e = dev_alloc(p, &p->d_pA, p->npairs_ring)) != hipSuccess ||
      (e = dev_alloc(p, &p->d_pB, p->npairs_ring)) != hipSuccess ||
      (e = dev_alloc(p, &p->d_phw, p->npairs_ring)) != hipSuccess ||
      (e = dev_upload(p, &p->d_tile_ring, tile_ring)) != hipSuccess ||
      (e = dev_upload(p, &p->d_tile_a0, tile_a0)) != hipSuccess ||
      (e = dev_alloc(p, &p->d_count, 1)) != hipSuccess) {
    rc = hip_fail(e, "conv_real_init: device allocation/upload");
    free_plan(p);
    return rc;
  }
  if ((e = convreal::launch_ring_window(p, nullptr)) != hipSuccess ||
      (e = hipMemset(p->d_count, 0, sizeof(unsigned long long))) != hipSuccess ||
      (e = convreal::launch_pair_count(p, false, nullptr)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    rc = hip_fail(e, "conv_real_init: window/count kernels");
    free_plan(p);
    return rc;
  }
  unsigned long long cnt = 0;
  if ((e = hipMemcpy(&cnt, p->d_count, sizeof(cnt), hipMemcpyDeviceToHost)) != hipSuccess) {
    rc = hip_fail(e, "conv_real_init: count readback");
    free_plan(p);
    return rc;
  }
  p->pairs = static_cast<long long>(cnt);
  if (precision == CONV_REAL_MIXED) {
    if ((e = setup_mixed(p, g, jlo, jhi, poff, pj)) != hipSuccess ||
        (e = hipMemset(p->d_count, 0, sizeof(unsigned long long))) != hipSuccess ||
        (e = convreal::launch_pair_count(p, true, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(&cnt, p->d_count, sizeof(cnt), hipMemcpyDeviceToHost)) != hipSuccess) {
      rc = hip_fail(e, "conv_real_init: mixed-precision set-up");
      free_plan(p);
      return rc;
    }
    p->pairs_rest = static_cast<long long>(cnt);
    if ((rc = set_weight_store(p, CONV_REAL_STORE_AUTO)) != CONV_REAL_OK) {
      free_plan(p);
      return rc;
    }
  }
  *plan = p;
  return CONV_REAL_OK;
}

int conv_real_set_weight_store(conv_real_plan* plan, int mode) {
  if (!plan || plan->magic != kMagic) { set_error("conv_real_set_weight_store: invalid plan"); return CONV_REAL_EINVAL; }
  if (plan->precision != CONV_REAL_MIXED) {
    set_error("conv_real_set_weight_store: mixed plans only");
    return CONV_REAL_EINVAL;
  }
  if (mode != CONV_REAL_STORE_OFF && mode != CONV_REAL_STORE_ON && mode != CONV_REAL_STORE_AUTO) {
    set_error("conv_real_set_weight_store: mode must be CONV_REAL_STORE_OFF, _ON or _AUTO");
    return CONV_REAL_EINVAL;
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_set_weight_store: hipSetDevice");
  return set_weight_store(plan, mode);
}

int conv_real_get_weight_store(const conv_real_plan* plan, int* active, long long* bytes) {
  if (!plan || plan->magic != kMagic || !active || !bytes) {
    set_error("conv_real_get_weight_store: invalid plan or NULL output");
    return CONV_REAL_EINVAL;
  }
  *active = plan->d_wstore ? 1 : 0;
  *bytes = plan->d_wstore ? static_cast<long long>(sizeof(uint4)) * plan->wstore_groups : 0;
  return CONV_REAL_OK;
}

namespace {

void release_ring_fft(conv_real_plan* p) {
  for (void* ptr : {static_cast<void*>(p->d_fft_tw), static_cast<void*>(p->d_fft_pi), static_cast<void*>(p->d_fft_pj),
                    static_cast<void*>(p->d_fft_pA), static_cast<void*>(p->d_fft_pB), static_cast<void*>(p->d_fft_boff),
                    static_cast<void*>(p->d_fft_K), static_cast<void*>(p->d_fft_X), static_cast<void*>(p->d_fft_Y),
                    static_cast<void*>(p->d_mtile_ring), static_cast<void*>(p->d_mtile_a0),
                    static_cast<void*>(p->d_fft_cpair)})
    release(p, ptr);
  p->d_fft_cpair = nullptr;
  p->d_mtile_ring = p->d_mtile_a0 = nullptr;
  p->n_mtiles = 0;
  p->d_fft_tw = nullptr;
  p->d_fft_pi = p->d_fft_pj = nullptr;
  p->d_fft_pA = p->d_fft_pB = nullptr;
  p->d_fft_boff = nullptr;
  p->d_fft_K = nullptr;
  p->d_fft_X = nullptr;
  p->d_fft_Y = nullptr;
  p->fft_work_bytes = 0;
  p->fft_npairs = 0;
}

// Ring-FFT set-up: the belt ring pairs (output ring major), twiddles, workspace, and the spectra of
// the belt pairs' kernels; for an FP64 plan also the list of the other ring pairs and their records
// for the FP64 cap kernel (a mixed plan keeps its own cap tiles for them).
hipError_t build_ring_fft(conv_real_plan* p) {
  const bool f64 = p->precision == CONV_REAL_F64;
  const int N = p->nside;
  const convreal::RingGrid g = convreal::make_ring_grid(N);
  std::vector<int> jlo, jhi;
  convreal::neighbour_rings(g, p->dcut2, jlo, jhi);
  std::vector<long long> poff(g.nrings + 1, 0);
  for (int r = 0; r < g.nrings; ++r) poff[r + 1] = poff[r] + (jhi[r] - jlo[r] + 1);
  std::vector<double> pA(p->npairs_ring), pB(p->npairs_ring), phw(p->npairs_ring);
  hipError_t e;
  if ((e = hipMemcpy(pA.data(), p->d_pA, sizeof(double) * pA.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(pB.data(), p->d_pB, sizeof(double) * pB.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(phw.data(), p->d_phw, sizeof(double) * phw.size(), hipMemcpyDeviceToHost)) != hipSuccess)
    return e;
  const int blo = N - 1, bhi = 3 * N - 1;   // belt rings (0-based): 4 N pixels each
  // kernel spectra of the north belt output rings through the equator; a south ring uses its
  // mirror's (same chord constants and azimuth offsets, input rings mirrored)
  std::vector<int> fi, fj;
  std::vector<double> fA, fB;
  std::vector<long long> boff(1, 0);
  // per output ring: the input rings with its own azimuth offset first, then those with the other one
  // (whose spectra carry the same half-pixel phase, applied once per frequency)
  for (int i = blo; i <= (g.nrings - 1) / 2; ++i) {
    for (int same = 1; same >= 0; --same) {
      for (int j = std::max(jlo[i], blo); j <= std::min(jhi[i], bhi); ++j) {
        if ((g.c[j] == g.c[i]) != (same == 1)) continue;
        const long long k = poff[i] + (j - jlo[i]);
        fi.push_back(i);
        fj.push_back(j);
        fA.push_back(pA[k]);
        fB.push_back(pB[k]);
      }
      boff.push_back(static_cast<long long>(fi.size()));
    }
  }
  // the apply kernels walk each offset group as j, j + 2, ... and take the belt offsets to alternate
  for (size_t t = 0; t + 1 < boff.size(); ++t)
    for (long long q = boff[t]; q + 1 < boff[t + 1]; ++q)
      if (fj[q + 1] != fj[q] + 2) return hipErrorInvalidValue;
  for (int r = blo; r < bhi; ++r)
    if (g.c[r + 1] + g.c[r] != 1) return hipErrorInvalidValue;
  std::vector<long long> roff(g.nrings + 1, 0), ridx;
  std::vector<convreal::CapPair64> rrec;   // the listed pairs as the FP64 cap kernel reads them
  std::vector<int> rtile_ring, rtile_a0;
  for (int r = 0; r < g.nrings && f64; ++r) {
    const bool belt_row = r >= blo && r <= bhi;
    for (long long k = poff[r]; k < poff[r + 1]; ++k) {
      const int j = jlo[r] + static_cast<int>(k - poff[r]);
      if (belt_row && j >= blo && j <= bhi) continue;
      ridx.push_back(k);
      convreal::CapPair64 c{};
      c.A = pA[k];
      c.B = pB[k];
      c.hw = phw[k];
      c.sd = std::sin(M_PI / g.n[j]);   // the per-ring tables' values
      c.cd = std::cos(M_PI / g.n[j]);
      c.nj = g.n[j];
      c.cj = g.c[j];
      c.xoff = static_cast<int>(g.start[j]);
      c.xoff_m = static_cast<int>(g.start[g.nrings - 1 - j]);
      rrec.push_back(c);
    }
    roff[r + 1] = static_cast<long long>(ridx.size());
    if (roff[r + 1] > roff[r])
      for (int a0 = 0; a0 < g.n[r]; a0 += kTile) {
        rtile_ring.push_back(r);
        rtile_a0.push_back(a0);
      }
  }
  // the cap-touching pairs by symmetry: fundamental domains of the north-half rings that have them
  std::vector<int> mtile_ring, mtile_a0;
  for (int r = 0; r <= (g.nrings - 1) / 2 && f64; ++r) {
    if (roff[r + 1] == roff[r]) continue;
    const int F = (g.n[r] / 4 - g.c[r]) / 2 + 1;
    for (int a0 = 0; a0 < F; a0 += 16) {
      mtile_ring.push_back(r);
      mtile_a0.push_back(a0);
    }
  }
  const int n = 4 * N;
  int logn = 0;
  while ((1 << logn) < n) ++logn;
  std::vector<double2> tw(static_cast<size_t>(n / 2));
  for (int m = 0; m < n / 2; ++m) {
    const double ang = 2.0 * M_PI * static_cast<double>(m) / static_cast<double>(n);
    tw[m] = make_double2(std::cos(ang), -std::sin(ang));
  }
  const size_t nbins = static_cast<size_t>(n / 2 + 1);
  p->belt_lo = blo;
  p->belt_hi = bhi;
  p->fft_n = n;
  p->fft_logn = logn;
  p->fft_npairs = static_cast<long long>(fi.size());
  if (f64) {
    release(p, p->d_rest_off);
    release(p, p->d_rest_idx);
    release(p, p->d_rtile_ring);
    release(p, p->d_rtile_a0);
    p->n_rtiles = static_cast<int>(rtile_ring.size());
    p->n_mtiles = static_cast<int>(mtile_ring.size());
    if ((e = dev_upload(p, &p->d_rest_off, roff)) != hipSuccess ||
        (e = dev_upload(p, &p->d_rest_idx, ridx)) != hipSuccess ||
        (e = dev_upload(p, &p->d_fft_cpair, rrec)) != hipSuccess ||
        (e = dev_upload(p, &p->d_rtile_ring, rtile_ring)) != hipSuccess ||
        (e = dev_upload(p, &p->d_rtile_a0, rtile_a0)) != hipSuccess ||
        (e = dev_upload(p, &p->d_mtile_ring, mtile_ring)) != hipSuccess ||
        (e = dev_upload(p, &p->d_mtile_a0, mtile_a0)) != hipSuccess)
      return e;
  }
  if ((e = dev_upload(p, &p->d_fft_tw, tw)) != hipSuccess || (e = dev_upload(p, &p->d_fft_pi, fi)) != hipSuccess ||
      (e = dev_upload(p, &p->d_fft_pj, fj)) != hipSuccess || (e = dev_upload(p, &p->d_fft_pA, fA)) != hipSuccess ||
      (e = dev_upload(p, &p->d_fft_pB, fB)) != hipSuccess || (e = dev_upload(p, &p->d_fft_boff, boff)) != hipSuccess ||
      (e = dev_alloc(p, &p->d_fft_K, nbins * fi.size())) != hipSuccess ||
      (e = dev_alloc(p, &p->d_fft_X, nbins * static_cast<size_t>(bhi - blo + 1))) != hipSuccess ||
      (e = dev_alloc(p, &p->d_fft_Y, nbins * static_cast<size_t>(bhi - blo + 1))) != hipSuccess ||
      (e = convreal::ring_fft_spectra(p)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
    return e;
  p->fft_work_bytes = static_cast<long long>(2 * sizeof(double2) * nbins * static_cast<size_t>(bhi - blo + 1));
  if (!f64) return hipSuccess;   // the mixed plan counted its cap-touching pairs at set-up
  if ((e = hipMemset(p->d_count, 0, sizeof(unsigned long long))) != hipSuccess ||
      (e = convreal::launch_pair_count(p, true, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
    return e;
  unsigned long long cnt = 0;
  if ((e = hipMemcpy(&cnt, p->d_count, sizeof(cnt), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  p->pairs_rest = static_cast<long long>(cnt);
  return hipSuccess;
}

}  // namespace

int conv_real_set_method(conv_real_plan* plan, int method) {
  if (!plan || plan->magic != kMagic) { set_error("conv_real_set_method: invalid plan"); return CONV_REAL_EINVAL; }
  if (plan->precision == CONV_REAL_F32) {
    set_error("conv_real_set_method: FP64 and mixed plans only");
    return CONV_REAL_EINVAL;
  }
  if (method != CONV_REAL_METHOD_DIRECT && method != CONV_REAL_METHOD_RING_FFT) {
    set_error("conv_real_set_method: method must be CONV_REAL_METHOD_DIRECT or _RING_FFT");
    return CONV_REAL_EINVAL;
  }
  const int N = plan->nside;
  if (method == CONV_REAL_METHOD_RING_FFT && ((N & (N - 1)) != 0 || N > 2048)) {
    set_error("conv_real_set_method: the ring FFTs need a power-of-two nside <= 2048");
    return CONV_REAL_EINVAL;
  }
  const bool mixed = plan->precision == CONV_REAL_MIXED;
  if (mixed && method == CONV_REAL_METHOD_RING_FFT && (!plan->belt_enabled || !plan->cap_mode)) {
    set_error("conv_real_set_method: this mixed plan has no belt ring pairs on the matrix cores (windows that "
              "cover whole belt rings) or no cap tiles (kernel table over 4098 nodes)");
    return CONV_REAL_EINVAL;
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_set_method: hipSetDevice");
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "conv_real_set_method: synchronise");
  if (method == CONV_REAL_METHOD_DIRECT) {
    release_ring_fft(plan);
    plan->method = method;
    // a mixed plan's queue takes its belt items back
    if (mixed && (e = build_items(plan)) != hipSuccess) return hip_fail(e, "conv_real_set_method: work queue");
    return CONV_REAL_OK;
  }
  if (!plan->d_fft_K && (e = build_ring_fft(plan)) != hipSuccess) {
    release_ring_fft(plan);
    plan->method = CONV_REAL_METHOD_DIRECT;
    return hip_fail(e, "conv_real_set_method: ring-FFT set-up");
  }
  plan->method = method;
  // a mixed plan's queue keeps only the cap items: the ring FFTs do the belt ring pairs
  if (mixed && (e = build_items(plan)) != hipSuccess) {
    release_ring_fft(plan);
    plan->method = CONV_REAL_METHOD_DIRECT;
    (void)build_items(plan);
    return hip_fail(e, "conv_real_set_method: work queue");
  }
  return CONV_REAL_OK;
}

int conv_real_get_method(const conv_real_plan* plan, int* method) {
  if (!plan || plan->magic != kMagic || !method) { set_error("conv_real_get_method: invalid argument"); return CONV_REAL_EINVAL; }
  *method = plan->method;
  return CONV_REAL_OK;
}

int conv_real_apply(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps, void* stream) {
  if (!plan || plan->magic != kMagic) { set_error("conv_real_apply: invalid plan"); return CONV_REAL_EINVAL; }
  if (!maps_in || !maps_out) { set_error("conv_real_apply: NULL map pointer"); return CONV_REAL_EINVAL; }
  if (nmaps < 1) { set_error("conv_real_apply: nmaps must be >= 1"); return CONV_REAL_EINVAL; }
  const size_t elem = plan->precision == CONV_REAL_F64 ? sizeof(double) : sizeof(float);
  const size_t bytes = static_cast<size_t>(nmaps) * static_cast<size_t>(plan->npix) * elem;
  const char* in0 = static_cast<const char*>(maps_in);
  const char* out0 = static_cast<const char*>(maps_out);
  if (in0 < out0 + bytes && out0 < in0 + bytes) {
    set_error("conv_real_apply: maps_in and maps_out overlap");
    return CONV_REAL_EALIAS;
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_apply: hipSetDevice");
  if (plan->precision == CONV_REAL_MIXED)
    e = convreal::launch_mixed(plan, static_cast<const float*>(maps_in), static_cast<float*>(maps_out), nmaps,
                               static_cast<hipStream_t>(stream));
  else if (plan->method == CONV_REAL_METHOD_RING_FFT)
    e = convreal::launch_ring_fft(plan, maps_in, maps_out, nmaps, static_cast<hipStream_t>(stream));
  else
    e = convreal::launch_pair_accumulate(plan, maps_in, maps_out, nmaps, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "conv_real_apply: launch");
  return CONV_REAL_OK;
}

int conv_real_apply_noalloc(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps, void* stream) {
  if (!plan || plan->magic != kMagic) { set_error("conv_real_apply_noalloc: invalid plan"); return CONV_REAL_EINVAL; }
  if (!maps_in || !maps_out) { set_error("conv_real_apply_noalloc: NULL map pointer"); return CONV_REAL_EINVAL; }
  if (nmaps < 1) { set_error("conv_real_apply_noalloc: nmaps must be >= 1"); return CONV_REAL_EINVAL; }
  if (plan->method == CONV_REAL_METHOD_RING_FFT) {
    set_error("conv_real_apply_noalloc: the ring-FFT method needs " + std::to_string(plan->fft_work_bytes) +
              " bytes of spectrum workspace, beyond the " +
              std::to_string(sizeof(unsigned) * convreal::kNoallocScratchWords) +
              "-byte fixed scratch; use conv_real_apply or the direct method");
    return CONV_REAL_EINVAL;
  }
  const size_t elem = plan->precision == CONV_REAL_F64 ? sizeof(double) : sizeof(float);
  const size_t bytes = static_cast<size_t>(nmaps) * static_cast<size_t>(plan->npix) * elem;
  const char* in0 = static_cast<const char*>(maps_in);
  const char* out0 = static_cast<const char*>(maps_out);
  if (in0 < out0 + bytes && out0 < in0 + bytes) {
    set_error("conv_real_apply_noalloc: maps_in and maps_out overlap");
    return CONV_REAL_EALIAS;
  }
  unsigned* scr = convreal::noalloc_scratch(plan->device);
  if (!scr) { set_error("conv_real_apply_noalloc: fixed scratch not located on the plan's device"); return CONV_REAL_EHIP; }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_apply_noalloc: hipSetDevice");
  if (plan->precision == CONV_REAL_MIXED)
    e = convreal::launch_mixed(plan, static_cast<const float*>(maps_in), static_cast<float*>(maps_out), nmaps,
                               static_cast<hipStream_t>(stream), scr, scr + convreal::kMaxSlots);
  else  // the direct per-pair kernels use no memory beyond the maps and the plan's tables
    e = convreal::launch_pair_accumulate(plan, maps_in, maps_out, nmaps, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "conv_real_apply_noalloc: launch");
  return CONV_REAL_OK;
}

int conv_real_profile(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps,
                      void* stream, const char** names, float* ms, long long* work, int* nstages) {
  if (!names || !ms || !work || !nstages || *nstages < 1) {
    set_error("conv_real_profile: NULL output or zero capacity");
    return CONV_REAL_EINVAL;
  }
  if (!plan || plan->magic != kMagic) { set_error("conv_real_profile: invalid plan"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_profile: hipSetDevice");
  convreal::Recorder rec;
  int made = 0;
  for (; made <= convreal::Recorder::kMax; ++made)
    if ((e = hipEventCreate(&rec.ev[made])) != hipSuccess) break;
  int rc = CONV_REAL_OK;
  if (e != hipSuccess) {
    rc = hip_fail(e, "conv_real_profile: hipEventCreate");
  } else {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((e = hipEventRecord(rec.ev[0], st)) != hipSuccess) {
      rc = hip_fail(e, "conv_real_profile: hipEventRecord");
    } else {
      plan->rec = &rec;
      rc = conv_real_apply(plan, maps_in, maps_out, nmaps, stream);
      plan->rec = nullptr;
      if (rc == CONV_REAL_OK && (e = hipStreamSynchronize(st)) != hipSuccess)
        rc = hip_fail(e, "conv_real_profile: hipStreamSynchronize");
    }
    if (rc == CONV_REAL_OK) {
      int out = 0;
      for (int k = 0; k < rec.n; ++k) {
        float t = 0.0f;
        if ((e = hipEventElapsedTime(&t, rec.ev[k], rec.ev[k + 1])) != hipSuccess) {
          rc = hip_fail(e, "conv_real_profile: hipEventElapsedTime");
          break;
        }
        if (out > 0 && std::strcmp(names[out - 1], rec.name[k]) == 0) {
          ms[out - 1] += t;
          work[out - 1] += rec.work[k];
        } else if (out < *nstages) {
          names[out] = rec.name[k];
          ms[out] = t;
          work[out] = rec.work[k];
          ++out;
        }
      }
      *nstages = out;
    }
  }
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(rec.ev[k]);
  return rc;
}

int conv_real_pairs(const conv_real_plan* plan, long long* pairs) {
  if (!plan || plan->magic != kMagic || !pairs) { set_error("conv_real_pairs: invalid argument"); return CONV_REAL_EINVAL; }
  *pairs = plan->pairs;
  return CONV_REAL_OK;
}

int conv_real_destroy(conv_real_plan* plan) {
  if (!plan) return CONV_REAL_OK;
  if (plan->magic != kMagic) { set_error("conv_real_destroy: invalid plan"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  (void)guard.enter(plan->device);
  free_plan(plan);
  return CONV_REAL_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning, autotune, batches
struct conv_real_batch {
  int magic = 0;
  int device = 0;
  int count = 0;
  conv_real_plan* plans[convreal::kMaxSlots] = {};
  convreal::Tuning tune;
  int2* d_items = nullptr;
  int n_items = 0;
  int* d_qchunk_off = nullptr;   // n_qchunks + 1 offsets into d_items
  int n_qchunks = 1;
  unsigned* d_amax = nullptr;
  unsigned* d_counter = nullptr;   // kMaxChunks counters
  int max_nseg = 0;
  long long npix_max = 0;
  long long pairs = 0;
};

namespace {

constexpr int kBatchMagic = 0x43564231;  // "CVB1"

bool tuning_ok(const conv_real_tuning* t) {
  return t && (t->seg == 256 || t->seg == 512) && t->wg_per_cu >= 1 && t->wg_per_cu <= 4 &&
         (t->order >= 0 && t->order <= 4);
}

convreal::Tuning to_internal(const conv_real_tuning* t) {
  convreal::Tuning r;
  r.seg = t->seg;
  r.wg_per_cu = t->wg_per_cu;
  r.order = t->order;
  return r;
}

void to_public(const convreal::Tuning& r, conv_real_tuning* t) {
  t->seg = r.seg;
  t->wg_per_cu = r.wg_per_cu;
  t->order = r.order;
}

std::vector<conv_real_tuning> candidate_tunings() {
  std::vector<conv_real_tuning> c;
  for (int seg : {256, 512})
    for (int wg : {1, 2, 3})
      for (int order : {0, 1, 2, 3, 4}) c.push_back({seg, wg, order});
  return c;
}

hipError_t build_batch_items(conv_real_batch* b) {
  using E = std::pair<QueueItem, int>;
  std::vector<E> belt, cap, ordered;
  for (int k = 0; k < b->count; ++k) {
    std::vector<QueueItem> bl, cp;
    plan_items(b->plans[k], b->tune, bl, cp);
    for (const QueueItem& q : bl) belt.push_back({q, k});
    for (const QueueItem& q : cp) cap.push_back({q, k});
  }
  const std::vector<int> off = order_queue(belt, cap, b->tune.order, [](const E& e) { return e.first.cost; },
                                           [](const E& e) { return e.first.kind; }, ordered);
  std::vector<int2> items(ordered.size());
  for (size_t k = 0; k < ordered.size(); ++k)
    items[k] = make_int2(ordered[k].second, (ordered[k].first.kind << 30) | ordered[k].first.idx);
  if (!queue_ok(off, items.size())) return hipErrorInvalidValue;
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_qchunk_off) (void)hipFree(b->d_qchunk_off);
  b->d_items = nullptr;
  b->d_qchunk_off = nullptr;
  b->n_items = static_cast<int>(items.size());
  b->n_qchunks = static_cast<int>(off.size()) - 1;
  hipError_t e = hipMalloc(&b->d_items, sizeof(int2) * std::max<size_t>(items.size(), 1));
  if (e != hipSuccess) return e;
  if (!items.empty()) e = hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  if ((e = hipMalloc(&b->d_qchunk_off, sizeof(int) * off.size())) != hipSuccess) return e;
  return hipMemcpy(b->d_qchunk_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice);
}

hipError_t batch_launch(conv_real_batch* b, const float* const* in, float* const* out, hipStream_t st) {
  convreal::Slots S;
  bool fly = false;   // some plan evaluates its cap weights on the fly
  for (int k = 0; k < b->count; ++k) {
    S.desc[k] = b->plans[k]->d_desc;
    S.x[k] = in[k];
    S.y[k] = out[k];
    fly = fly || (b->plans[k]->cap_mode && !b->plans[k]->d_wstore);
  }
  return convreal::launch_mixed_queue(b->plans[0], S, b->count, b->d_items, b->n_items, 1, b->d_qchunk_off, b->n_qchunks,
                                      b->d_amax, b->d_counter, b->tune, b->max_nseg, b->npix_max, b->pairs, fly, st);
}

// Mean milliseconds of `reps` runs of fn() on st, after one untimed run.
template <typename F>
int time_runs(F fn, hipStream_t st, int reps, float* ms_out) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return hip_fail(e, "autotune: hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "autotune: hipEventCreate");
  }
  int rc = fn();
  if (rc == CONV_REAL_OK && (e = hipEventRecord(e0, st)) != hipSuccess) rc = hip_fail(e, "autotune: record");
  for (int r = 0; r < reps && rc == CONV_REAL_OK; ++r) rc = fn();
  if (rc == CONV_REAL_OK && (e = hipEventRecord(e1, st)) != hipSuccess) rc = hip_fail(e, "autotune: record");
  if (rc == CONV_REAL_OK && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "autotune: sync");
  float ms = 0.0f;
  if (rc == CONV_REAL_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = hip_fail(e, "autotune: elapsed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = ms / reps;
  return rc;
}

}  // namespace

extern "C" {

int conv_real_set_tuning(conv_real_plan* plan, const conv_real_tuning* t) {
  if (!plan || plan->magic != kMagic) { set_error("conv_real_set_tuning: invalid plan"); return CONV_REAL_EINVAL; }
  if (plan->precision != CONV_REAL_MIXED) { set_error("conv_real_set_tuning: mixed plans only"); return CONV_REAL_EINVAL; }
  if (!tuning_ok(t)) { set_error("conv_real_set_tuning: field out of range"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  hipError_t e = guard.enter(plan->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_set_tuning: hipSetDevice");
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "conv_real_set_tuning: sync");
  plan->tune = to_internal(t);
  plan->tune_user = 1;
  if ((e = build_items(plan)) != hipSuccess) return hip_fail(e, "conv_real_set_tuning: work queue");
  return CONV_REAL_OK;
}

int conv_real_get_tuning(const conv_real_plan* plan, conv_real_tuning* t) {
  if (!plan || plan->magic != kMagic || !t) { set_error("conv_real_get_tuning: invalid argument"); return CONV_REAL_EINVAL; }
  to_public(plan->tune, t);
  return CONV_REAL_OK;
}

int conv_real_autotune(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps, void* stream,
                       conv_real_tuning* best) {
  if (!plan || plan->magic != kMagic || !best) { set_error("conv_real_autotune: invalid argument"); return CONV_REAL_EINVAL; }
  if (plan->precision != CONV_REAL_MIXED) { set_error("conv_real_autotune: mixed plans only"); return CONV_REAL_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  float best_ms = 1e30f;
  conv_real_tuning chosen;
  to_public(plan->tune, &chosen);
  for (const conv_real_tuning& c : candidate_tunings()) {
    int rc = conv_real_set_tuning(plan, &c);
    if (rc != CONV_REAL_OK) return rc;
    float ms = 0.0f;
    rc = time_runs([&]() { return conv_real_apply(plan, maps_in, maps_out, nmaps, stream); }, st, 3, &ms);
    if (rc != CONV_REAL_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      chosen = c;
    }
  }
  *best = chosen;
  return conv_real_set_tuning(plan, &chosen);
}

int conv_real_batch_create(conv_real_batch** batch, conv_real_plan* const* plans, int count) {
  if (!batch) { set_error("conv_real_batch_create: NULL batch pointer"); return CONV_REAL_EINVAL; }
  *batch = nullptr;
  if (!plans || count < 1 || count > convreal::kMaxSlots) {
    set_error("conv_real_batch_create: need 1..64 plans");
    return CONV_REAL_EINVAL;
  }
  for (int k = 0; k < count; ++k) {
    const conv_real_plan* p = plans[k];
    if (!p || p->magic != kMagic || p->precision != CONV_REAL_MIXED || !p->cap_mode || p->device != plans[0]->device) {
      set_error("conv_real_batch_create: every plan must be a mixed plan on one device with n_tab <= 4098");
      return CONV_REAL_EINVAL;
    }
    if (p->method != CONV_REAL_METHOD_DIRECT) {
      set_error("conv_real_batch_create: a batch applies the direct method; set it on every plan first");
      return CONV_REAL_EINVAL;
    }
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(plans[0]->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_batch_create: hipSetDevice");
  auto* b = new (std::nothrow) conv_real_batch();
  if (!b) { set_error("conv_real_batch_create: host allocation failed"); return CONV_REAL_ENOMEM; }
  b->magic = kBatchMagic;
  b->device = plans[0]->device;
  b->count = count;
  for (int k = 0; k < count; ++k) {
    b->plans[k] = plans[k];
    b->max_nseg = std::max(b->max_nseg, plans[k]->cap_nseg);
    b->npix_max = std::max(b->npix_max, plans[k]->npix);
    b->pairs += plans[k]->pairs;
  }
  if ((e = hipMalloc(&b->d_amax, sizeof(unsigned) * convreal::kMaxSlots)) != hipSuccess ||
      (e = hipMalloc(&b->d_counter, sizeof(unsigned) * convreal::kMaxChunks)) != hipSuccess ||
      (e = build_batch_items(b)) != hipSuccess) {
    const int rc = hip_fail(e, "conv_real_batch_create");
    if (b->d_amax) (void)hipFree(b->d_amax);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_qchunk_off) (void)hipFree(b->d_qchunk_off);
    delete b;
    return rc;
  }
  *batch = b;
  return CONV_REAL_OK;
}

int conv_real_batch_apply(conv_real_batch* batch, const float* const* maps_in, float* const* maps_out, void* stream) {
  if (!batch || batch->magic != kBatchMagic) { set_error("conv_real_batch_apply: invalid batch"); return CONV_REAL_EINVAL; }
  if (!maps_in || !maps_out) { set_error("conv_real_batch_apply: NULL map arrays"); return CONV_REAL_EINVAL; }
  for (int k = 0; k < batch->count; ++k) {
    if (!maps_in[k] || !maps_out[k]) { set_error("conv_real_batch_apply: NULL map pointer"); return CONV_REAL_EINVAL; }
  }
  for (int k = 0; k < batch->count; ++k) {
    const char* o0 = reinterpret_cast<const char*>(maps_out[k]);
    const char* o1 = o0 + sizeof(float) * batch->plans[k]->npix;
    for (int m = 0; m < batch->count; ++m) {
      const char* i0 = reinterpret_cast<const char*>(maps_in[m]);
      const char* i1 = i0 + sizeof(float) * batch->plans[m]->npix;
      if (i0 < o1 && o0 < i1) { set_error("conv_real_batch_apply: an output overlaps an input"); return CONV_REAL_EALIAS; }
      if (m != k) {
        const char* p0 = reinterpret_cast<const char*>(maps_out[m]);
        const char* p1 = p0 + sizeof(float) * batch->plans[m]->npix;
        if (p0 < o1 && o0 < p1) { set_error("conv_real_batch_apply: outputs overlap"); return CONV_REAL_EALIAS; }
      }
    }
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(batch->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_batch_apply: hipSetDevice");
  if ((e = batch_launch(batch, maps_in, maps_out, static_cast<hipStream_t>(stream))) != hipSuccess)
    return hip_fail(e, "conv_real_batch_apply: launch");
  return CONV_REAL_OK;
}

int conv_real_batch_set_tuning(conv_real_batch* batch, const conv_real_tuning* t) {
  if (!batch || batch->magic != kBatchMagic) { set_error("conv_real_batch_set_tuning: invalid batch"); return CONV_REAL_EINVAL; }
  if (!tuning_ok(t)) { set_error("conv_real_batch_set_tuning: field out of range"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  hipError_t e = guard.enter(batch->device);
  if (e != hipSuccess) return hip_fail(e, "conv_real_batch_set_tuning: hipSetDevice");
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "conv_real_batch_set_tuning: sync");
  batch->tune = to_internal(t);
  if ((e = build_batch_items(batch)) != hipSuccess) return hip_fail(e, "conv_real_batch_set_tuning: work queue");
  return CONV_REAL_OK;
}

int conv_real_batch_autotune(conv_real_batch* batch, const float* const* maps_in, float* const* maps_out,
                             void* stream, conv_real_tuning* best) {
  if (!batch || batch->magic != kBatchMagic || !best) { set_error("conv_real_batch_autotune: invalid argument"); return CONV_REAL_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  float best_ms = 1e30f;
  conv_real_tuning chosen;
  to_public(batch->tune, &chosen);
  for (const conv_real_tuning& c : candidate_tunings()) {
    int rc = conv_real_batch_set_tuning(batch, &c);
    if (rc != CONV_REAL_OK) return rc;
    float ms = 0.0f;
    rc = time_runs([&]() { return conv_real_batch_apply(batch, maps_in, maps_out, stream); }, st, 3, &ms);
    if (rc != CONV_REAL_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      chosen = c;
    }
  }
  *best = chosen;
  return conv_real_batch_set_tuning(batch, &chosen);
}

int conv_real_batch_pairs(const conv_real_batch* batch, long long* pairs) {
  if (!batch || batch->magic != kBatchMagic || !pairs) { set_error("conv_real_batch_pairs: invalid argument"); return CONV_REAL_EINVAL; }
  *pairs = batch->pairs;
  return CONV_REAL_OK;
}

int conv_real_batch_destroy(conv_real_batch* batch) {
  if (!batch) return CONV_REAL_OK;
  if (batch->magic != kBatchMagic) { set_error("conv_real_batch_destroy: invalid batch"); return CONV_REAL_EINVAL; }
  DeviceGuard guard;
  (void)guard.enter(batch->device);
  if (batch->d_items) (void)hipFree(batch->d_items);
  if (batch->d_qchunk_off) (void)hipFree(batch->d_qchunk_off);
  if (batch->d_amax) (void)hipFree(batch->d_amax);
  if (batch->d_counter) (void)hipFree(batch->d_counter);
  batch->magic = 0;
  delete batch;
  return CONV_REAL_OK;
}

}  // extern "C"

int convreal::plan_info(const conv_real_plan* p, int* nside, int* precision, int* device) {
  if (!p || p->magic != kMagic) {
    set_error("invalid conv_real plan");
    return CONV_REAL_EINVAL;
  }
  *nside = p->nside;
  *precision = p->precision;
  *device = p->device;
  return CONV_REAL_OK;
}
