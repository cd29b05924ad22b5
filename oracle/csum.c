/* Plain FP64 sums of the truncated real-space convolution at listed output pixels (oracle, C).
 *
 * Test infrastructure: called by the tests and by the benchmark's CPU baseline only, never by the
 * library. It computes the same definition as oracle/convolve.py (Eq. 1's real-space part on the
 * pixelized sphere):
 *
 *     y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) * x_q,   Omega = 4 pi / Npix,
 *
 * with d_pq = |v_p - v_q| from the pixel-centre unit vectors component by component, pairs at
 * d = d_cut included and every pair kept for a cut of pi, and Ktilde the 4-point Lagrange
 * interpolant on the uniform chord grid (node k at k h, h = d_cut / (n_tab - 3), ghost node
 * T[-1] = T[1]).
 *
 * Pixel centres follow the ring scheme of the equal-area iso-latitude grid the paper assumes
 * (HEALPix, ring order): north cap rings i = 1..N-1 with 4i pixels at z = 1 - i^2/(3N^2),
 * phi = (pi / 2i)(a + 1/2); belt rings i = N..3N with 4N pixels at z = 4/3 - 2i/(3N),
 * phi = (pi / 2N)(a + s/2), s = (i - N + 1) mod 2; south cap rings mirror the north.
 *
 * Candidates: for output pixel p on ring i, every ring j with |z_j - z_p| <= d_cut (necessary,
 * since |z_p - z_q| <= d_pq); on ring j the azimuths within the exact bound
 *     cos(dphi) >= (dz^2 + s_p^2 + s_j^2 - d_cut^2) / (2 s_p s_j)
 * widened by two pixels on each side (so rounding of the bound cannot lose a pair), and then the
 * exact chord test on every candidate. The pair set is therefore the same as that of the
 * ring-exhaustive search, at a cost proportional to the pairs instead of the ring lengths.
 * Sampled output pixels are spread over OpenMP threads; each sample's sum runs in one thread in a
 * fixed order. At most 64 maps per call.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double z;      /* cos(theta) */
  double s;      /* sin(theta) */
  double phi0;   /* azimuth of pixel 0 */
  double dphi;   /* 2 pi / n */
  int64_t n;     /* pixels */
  int64_t start; /* first pixel index */
} ring_t;

static void ring_table(int N, ring_t* r) {
  int64_t pos = 0;
  for (int i = 1; i < 4 * N; ++i) {
    ring_t* q = &r[i - 1];
    if (i < N || i > 3 * N) {
      const int k = i < N ? i : 4 * N - i; /* ring counted from the nearer pole */
      const double om = (double)k * k / (3.0 * N * N); /* 1 - |z| */
      q->z = i < N ? 1.0 - om : -(1.0 - om);
      q->s = sqrt(om * (2.0 - om));
      q->n = 4 * (int64_t)k;
      q->phi0 = M_PI / (2.0 * k) * 0.5;
    } else {
      q->z = (2.0 * N - i) * 2.0 / (3.0 * N);
      q->s = sqrt(((2.0 * i - N) / (3.0 * N)) * ((7.0 * N - 2.0 * i) / (3.0 * N)));
      q->n = 4 * (int64_t)N;
      q->phi0 = M_PI / (2.0 * N) * (0.5 * ((i - N + 1) % 2));
    }
    q->dphi = 2.0 * M_PI / (double)q->n;
    q->start = pos;
    pos += q->n;
  }
}

static int ring_of(const ring_t* r, int nr, int64_t p) {
  int lo = 0, hi = nr - 1; /* last ring with start <= p */
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (r[mid].start <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

static double interp(const double* T, int n, double h, double d) {
  const double t = d / h;
  int64_t k = (int64_t)floor(t);
  if (k < 0) k = 0;
  if (k > n - 3) k = n - 3;
  const double f = t - (double)k;
  const double tm1 = T[k == 0 ? 1 : k - 1], t0 = T[k], t1 = T[k + 1], t2 = T[k + 2];
  const double wm1 = -f * (f - 1.0) * (f - 2.0) / 6.0;
  const double w0 = (f + 1.0) * (f - 1.0) * (f - 2.0) / 2.0;
  const double w1 = -(f + 1.0) * f * (f - 2.0) / 2.0;
  const double w2 = (f + 1.0) * f * (f - 1.0) / 6.0;
  return wm1 * tm1 + w0 * t0 + w1 * t1 + w2 * t2;
}

/* y[m * npts + k] = the sum at pixel pix[k] of map m (x[m * npix + q], 1 <= nmaps <= 64); pairs[k] =
 * its pair count (may be NULL). nthreads <= 0: the OpenMP default. Returns 0, or -1 for bad
 * arguments. */
int oracle_convolve_sampled(int nside, const double* table, int n_tab, double theta_cut, const double* x,
                            int nmaps, const int64_t* pix, int64_t npts, double* y, int64_t* pairs, int nthreads) {
  if (nside < 1 || n_tab < 4 || !table || !x || !pix || !y || nmaps < 1 || nmaps > 64 || npts < 0 ||
      !(theta_cut > 0.0))
    return -1;
  const int N = nside, nr = 4 * N - 1;
  const int64_t npix = 12 * (int64_t)N * N;
  ring_t* r = (ring_t*)malloc(sizeof(ring_t) * (size_t)nr);
  if (!r) return -1;
  ring_table(N, r);
  const int all = theta_cut >= M_PI;
  const double dcut = 2.0 * sin(0.5 * theta_cut);
  const double h = dcut / (n_tab - 3);
  const double omega = 4.0 * M_PI / (double)npix;
  int bad = 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads) reduction(| : bad)
#endif
  for (int64_t k = 0; k < npts; ++k) {
    const int64_t p = pix[k];
    if (p < 0 || p >= npix) {
      bad = 1;
      continue;
    }
    const int i = ring_of(r, nr, p);
    const double php = r[i].phi0 + (double)(p - r[i].start) * r[i].dphi;
    const double zp = r[i].z, sp = r[i].s;
    const double xp = sp * cos(php), yp = sp * sin(php);
    double acc[64];
    for (int m = 0; m < nmaps; ++m) acc[m] = 0.0;
    int64_t cnt = 0;
    for (int j = 0; j < nr; ++j) {
      const double dz = r[j].z - zp;
      if (!all && fabs(dz) > dcut) continue;
      int64_t b0 = 0, nb = r[j].n;
      if (!all) {
        const double c = (dz * dz + sp * sp + r[j].s * r[j].s - dcut * dcut) / (2.0 * sp * r[j].s);
        if (c > -1.0) {
          const double dmax = acos(c > 1.0 ? 1.0 : c);
          const double t0 = (php - dmax - r[j].phi0) / r[j].dphi;
          const double t1 = (php + dmax - r[j].phi0) / r[j].dphi;
          b0 = (int64_t)floor(t0) - 2;
          const int64_t b1 = (int64_t)ceil(t1) + 2;
          if (b1 - b0 + 1 < r[j].n) nb = b1 - b0 + 1;
          else b0 = 0;
        }
      }
      for (int64_t t = 0; t < nb; ++t) {
        int64_t b = (b0 + t) % r[j].n;
        if (b < 0) b += r[j].n;
        const double phq = r[j].phi0 + (double)b * r[j].dphi;
        const double vx = r[j].s * cos(phq) - xp;
        const double vy = r[j].s * sin(phq) - yp;
        const double d = sqrt(vx * vx + vy * vy + dz * dz);
        if (!all && !(d <= dcut)) continue;
        const double w = interp(table, n_tab, h, d);
        const int64_t q = r[j].start + b;
        for (int m = 0; m < nmaps; ++m) acc[m] += w * x[(int64_t)m * npix + q];
        ++cnt;
      }
    }
    for (int m = 0; m < nmaps; ++m) y[(int64_t)m * npts + k] = omega * acc[m];
    if (pairs) pairs[k] = cnt;
  }
  free(r);
  return bad ? -1 : 0;
}
