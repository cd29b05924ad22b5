/*
 * Spherical-harmonic synthesis on iso-latitude rings, for drawing Gaussian random fields.
 *
 * For every ring (given by z = cos theta and sin theta) and every order m, computes
 *     F_m = sum_{l=m}^{lmax} a_lm lambda_lm(z)
 * where Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m phi} are the orthonormal spherical
 * harmonics. lambda_lm is produced by the standard stable recurrence in l at fixed m:
 *     lambda_mm     = (-1)^m sqrt((2m+1)/(4 pi) prod_{k=1}^m (2k-1)/(2k)) sin^m theta
 *     lambda_{m+1,m} = sqrt(2m+3) z lambda_mm
 *     lambda_lm     = a_lm (z lambda_{l-1,m} - lambda_{l-2,m} / a_{l-1,m}),
 *     a_lm          = sqrt((4 l^2 - 1) / (l^2 - m^2)).
 * Values that underflow double precision near the poles are carried with a separate power-of-2
 * exponent (multiples of 2^-256) and contribute only once they are back in range.
 *
 * Rings are processed in pairs (z, -z): lambda_lm(-z) = (-1)^(l+m) lambda_lm(z), so the sums over
 * even and odd l+m give both rings' coefficients.
 */
#include <math.h>
#include <stdlib.h>

#define SCALE_BITS 256

/* alm_re/alm_im: packed m-major (m = 0..lmax, l = m..lmax).
 * zn, sn: north-side rings (z >= 0), count nr.
 * out_north/out_south: [nr][lmax+1] complex as (re, im) pairs.
 * For z == 0 the south output equals the north one. */
void synth_ring_pairs(int lmax, const double* alm_re, const double* alm_im, int nr, const double* zn,
                      const double* sn, double* out_north, double* out_south) {
  const double big = ldexp(1.0, SCALE_BITS);
  const double small = ldexp(1.0, -SCALE_BITS);
  double* logmm = (double*)malloc(sizeof(double) * (lmax + 1));
  double acc = 0.0;
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) acc += log((2.0 * m - 1.0) / (2.0 * m));
    logmm[m] = 0.5 * (log((2.0 * m + 1.0) / (4.0 * M_PI)) + acc);
  }
  long long* moff = (long long*)malloc(sizeof(long long) * (lmax + 2));
  moff[0] = 0;
  for (int m = 0; m <= lmax; ++m) moff[m + 1] = moff[m] + (lmax - m + 1);

#pragma omp parallel
  {
    double* lp = (double*)malloc(sizeof(double) * nr);
    double* lc = (double*)malloc(sizeof(double) * nr);
    int* ex = (int*)malloc(sizeof(int) * nr);
    double* er = (double*)malloc(sizeof(double) * nr);
    double* ei = (double*)malloc(sizeof(double) * nr);
    double* orr = (double*)malloc(sizeof(double) * nr);
    double* oi = (double*)malloc(sizeof(double) * nr);
#pragma omp for schedule(dynamic, 4)
    for (int m = 0; m <= lmax; ++m) {
      const double* are = alm_re + moff[m];
      const double* aim = alm_im + moff[m];
      const double sign = (m & 1) ? -1.0 : 1.0;
      for (int r = 0; r < nr; ++r) {
        const double lg = logmm[m] + (m > 0 ? m * log(sn[r]) : 0.0);  /* natural log of |lambda_mm| */
        const double l2 = lg / log(2.0);
        int e = 0;
        double v;
        if (l2 < -900.0) {
          e = (int)floor(l2 / SCALE_BITS);
          v = sign * exp2(l2 - (double)e * SCALE_BITS);
        } else {
          v = sign * exp2(l2);
        }
        lp[r] = 0.0;
        lc[r] = v;
        ex[r] = e;
        er[r] = (e == 0) ? are[0] * v : 0.0;
        ei[r] = (e == 0) ? aim[0] * v : 0.0;
        orr[r] = 0.0;
        oi[r] = 0.0;
      }
      double amprev = 0.0;  /* a_{l-1,m} */
      for (int l = m + 1; l <= lmax; ++l) {
        const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double binv = (l == m + 1) ? 0.0 : 1.0 / amprev;
        const double cre = are[l - m], cim = aim[l - m];
        const int odd = (l - m) & 1;
        for (int r = 0; r < nr; ++r) {
          double nv = a * (zn[r] * lc[r] - binv * lp[r]);
          double pv = lc[r];
          if (ex[r] < 0 && fabs(nv) > 1.0) {
            nv *= small;
            pv *= small;
            ex[r] += 1;
          }
          lp[r] = pv;
          lc[r] = nv;
          const double w = (ex[r] == 0) ? nv : 0.0;
          if (odd) {
            orr[r] += cre * w;
            oi[r] += cim * w;
          } else {
            er[r] += cre * w;
            ei[r] += cim * w;
          }
        }
        amprev = a;
      }
      (void)big;
      for (int r = 0; r < nr; ++r) {
        double* on = out_north + 2 * ((long long)r * (lmax + 1) + m);
        double* os = out_south + 2 * ((long long)r * (lmax + 1) + m);
        on[0] = er[r] + orr[r];
        on[1] = ei[r] + oi[r];
        os[0] = er[r] - orr[r];
        os[1] = ei[r] - oi[r];
      }
    }
    free(lp);
    free(lc);
    free(ex);
    free(er);
    free(ei);
    free(orr);
    free(oi);
  }
  free(logmm);
  free(moff);
}
