/*
 * convsht.h - C ABI of the harmonic half of a split spherical convolution and of the hybrid apply,
 * in libconvreal (AMD Instinct MI355X, gfx950).
 *
 * The paper (Sutter, Wandelt & Elsner, "Using hybrid GPU/CPU kernel splitting to accelerate
 * spherical convolutions") splits a radially symmetric kernel K_l into a truncated harmonic part
 * K^_l (l <= l_cut) and a truncated real-space part K^_theta (Estimating Errors section, Eq. 1). The
 * harmonic part is applied by spherical-harmonic transforms, the real-space part by the real-space
 * sum of convreal.h, both at the same time, and the two output maps are summed (Fig. 1). Here both
 * halves run on the GPU, on two streams.
 *
 * Transforms, for a real map x on the ring grid of convreal.h (Npix = 12 nside^2 pixels, ring order):
 *
 *   analysis     a_lm = Omega * sum_p x_p conj(Y_lm(v_p)),   Omega = 4 pi / Npix (equal weights)
 *   synthesis    y_p  = sum_{l <= L} sum_{|m| <= l} b_lm Y_lm(v_p)
 *   convolution  y    = synthesis(k_l * analysis(x))
 *
 * Y_lm(theta, phi) = lambda_lm(cos theta) exp(i m phi): orthonormal spherical harmonics with the
 * Condon-Shortley phase. Real maps have a_{l,-m} = (-1)^m conj(a_lm), so only m >= 0 is stored,
 * m-major: index(l, m) = m (2L + 3 - m) / 2 + (l - m), (L + 1)(L + 2) / 2 complex values
 * (interleaved FP64 real, imaginary). The analysis is the equal-weight pixel quadrature (no ring
 * weights, no iteration); it is exact only up to the grid's quadrature error.
 *
 * Arithmetic: FP64 throughout. lambda_lm by the three-term recurrence in l at fixed m from
 * lambda_mm, started with a power-of-two exponent carried beside values below the FP64 range (so that
 * polar rings at large m neither underflow nor lose accuracy); contributions below about 2^-600 are
 * dropped. Ring sums as DFTs of the ring's n = 4k pixels, folded by quarter rings.
 *
 * Error behaviour: every entry point returns CONV_REAL_OK (0) or a negative CONV_REAL_* code
 * (convreal.h); arguments are validated on the host before any device call; conv_real_last_error()
 * gives the message. Device pointers are caller-owned; the plan owns its workspaces until
 * conv_sht_destroy. Calls on one plan must not overlap in time (the workspaces are per plan).
 */
#ifndef CONVSHT_H
#define CONVSHT_H

#include "convreal.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct conv_sht_plan conv_sht_plan;

#define CONV_SHT_MAX_NSIDE 2048
#define CONV_SHT_MAX_LMAX  8192

/* Map element types. */
#define CONV_SHT_F64 0
#define CONV_SHT_F32 1

/*
 * conv_sht_init - plan for one grid and band limit on the current device.
 *   nside  1..CONV_SHT_MAX_NSIDE;  lmax  0..CONV_SHT_MAX_LMAX
 * Allocates the recurrence coefficients ((L+1)(L+2)/2 x 16 bytes), a ring-by-order workspace
 * ((L + 1)(4 nside - 1) x 16 bytes), one alm workspace and the chirp-z tables of the rings with at
 * least 16 pixels per quarter that no power-of-two FFT takes (per ring length k: k + M values of 16 bytes, M the power of two at
 * least k + ceil(min(4k, L + 1) / 4) - 1; 99 MB at nside 2048 / L 1500), which it fills with a kernel,
 * and per order m the number of leading polar ring chunks that the Legendre sums leave out (L + 1
 * ints; a second set-up kernel). Synchronous.
 */
int conv_sht_init(conv_sht_plan** plan, int nside, int lmax);

/* conv_sht_alm_size - (lmax + 1)(lmax + 2) / 2 into *n (EINVAL for lmax < 0). */
int conv_sht_alm_size(int lmax, long long* n);

/*
 * conv_sht_analysis - alm (device, complex FP64, m-major) of one map (device, dtype CONV_SHT_F64 or
 * CONV_SHT_F32, 12 nside^2 values). Asynchronous on stream.
 */
int conv_sht_analysis(conv_sht_plan* plan, const void* map, int dtype, void* alm, void* stream);

/*
 * conv_sht_synthesis - map (device, dtype) from alm (device). accumulate = 0: the map is written;
 * 1: the synthesis is added to it. Asynchronous on stream.
 */
int conv_sht_synthesis(conv_sht_plan* plan, const void* alm, void* map, int dtype, int accumulate,
                       void* stream);

/* conv_sht_almxfl - alm_out[l, m] = fl[l] * alm_in[l, m] (device pointers; fl: lmax + 1 doubles;
 * alm_out may equal alm_in). Asynchronous. */
int conv_sht_almxfl(conv_sht_plan* plan, const void* alm_in, const double* fl, void* alm_out, void* stream);

/*
 * conv_sht_convolve - map_out (+)= synthesis(k_ell * analysis(map_in)): the radial kernel k_l
 * (device, lmax + 1 doubles) applied in harmonic space. map_in and map_out: device, dtype, one map
 * each, not overlapping. Uses the plan's alm workspace. Asynchronous.
 */
int conv_sht_convolve(conv_sht_plan* plan, const void* map_in, const double* k_ell, void* map_out,
                      int dtype, int accumulate, void* stream);

/* conv_sht_power_spectrum - cl[l] = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1), l = 0..lmax
 * (device pointers). Asynchronous. */
int conv_sht_power_spectrum(conv_sht_plan* plan, const void* alm, double* cl, void* stream);

/*
 * conv_hybrid_apply - the whole split convolution of Eq. 1 and Fig. 1:
 *     maps_out = real-space part (conv_real_apply of `real`) + synthesis(k_hat * analysis(maps_in))
 * for nmaps maps. `real` and `sht` must be on the same device and grid; the map type is FP64 for a
 * CONV_REAL_F64 real-space plan and FP32 otherwise. k_hat: device, sht lmax + 1 doubles (the
 * truncated harmonic kernel, zero above l_cut). The real-space part runs on `stream`; the analysis,
 * the product and the Legendre half of the synthesis run at the same time on `stream_sht`, whose
 * last kernel (the ring sums, adding into maps_out) waits for the real-space part; `stream` then
 * waits for it, so the result is complete in `stream` order. stream_sht NULL or equal to stream: all
 * on `stream`, one after the other. Asynchronous, no allocation, no host synchronisation.
 */
int conv_hybrid_apply(conv_real_plan* real, conv_sht_plan* sht, const double* k_hat, const void* maps_in,
                      void* maps_out, int nmaps, void* stream, void* stream_sht);

/* conv_sht_destroy - free a plan. NULL is accepted. */
int conv_sht_destroy(conv_sht_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* CONVSHT_H */
