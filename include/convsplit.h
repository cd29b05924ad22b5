/* convsplit.h - error and cost model of a kernel split, the least-squares split, and the split
 * search (libconvreal.so).
 *
 * A radial kernel with Legendre coefficients K_l (l = 0..lmax) is split into a harmonic part
 * K^_l kept for l <= l_cut and a real-space part truncated at theta_cut (paper, "Estimating
 * Errors": Eq. 1). The split is chosen by weighted least squares (Eqs. 3-5), its error is Eq. 2
 * (rms) and Eq. 6 (fractional, with the empirical factor alpha), and the cost of a split is the
 * slower of the two convolutions, which run concurrently (the cost section, Eqs. 7-8 and Fig. 1),
 * with the constants measured on this hardware instead of the paper's fits.
 *
 * Everything here is host-side FP64 on caller-owned host arrays. Functions return CONV_REAL_OK
 * (0) or a negative CONV_REAL_E* code (convreal.h); conv_real_last_error() gives the reason.
 * A context is not thread-safe for concurrent calls, except conv_split_search_many, which runs its
 * own worker threads on one context.
 */
#ifndef CONVSPLIT_H
#define CONVSPLIT_H

#include "convreal.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Returned (positive, not an error) by the search when no split meets the bound. */
#define CONV_SPLIT_INFEASIBLE 1

typedef struct conv_split_ctx conv_split_ctx;

/* Context for one band limit and input weighting (Eqs. 2-5).
 *   lmax       band limit, 1 <= lmax <= CONV_REAL_MAX_LMAX
 *   c_in       lmax + 1 values of the input spectrum C^in_l (host, copied); NULL means C^in = 1,
 *              the paper's choice
 *   theta_max  largest theta_cut that will be asked about, 0 < theta_max <= pi (radians)
 *   sv_cut     singular-value cutoff of the least-squares solve, relative to the largest (the
 *              paper drops singular values below 1e-6); 0 < sv_cut < 1
 * Computes the (lmax + 1)-point Gauss-Legendre nodes with z > cos(theta_max) (the real-space
 * samples) and the Legendre operator P_{l,k} = 2 pi w_k P_l(z_k). */
int conv_split_create(conv_split_ctx** ctx, int lmax, const double* c_in, double theta_max, double sv_cut);

/* Frees a context; NULL is accepted. */
int conv_split_destroy(conv_split_ctx* ctx);

/* Number of real-space samples inside theta_cut: nodes with z_k > cos(theta_cut).
 * theta_cut must be in (0, theta_max]. */
int conv_split_nodes(const conv_split_ctx* ctx, double theta_cut, int* z_cut);

/* The least-squares split of k_ell (lmax + 1 values) for (ell_cut, theta_cut) (Eqs. 3-5).
 * The identity block of the design matrix makes every row l <= ell_cut exact, so the solve is
 * the reduced problem: minimise sum_{l > ell_cut} (2l+1) C^in_l (K_l - (P x)_l)^2 over the
 * z_cut real-space samples x, through the singular value decomposition of the weighted matrix
 * B = W_r^1/2 P_r (rows l > ell_cut, W_l = (2l+1) C^in_l; Householder QR, then one-sided Jacobi on R),
 * dropping singular values below sv_cut times the largest; then K^_l = K_l - (P x)_l for l <= ell_cut.
 * Outputs (host, any may be NULL):
 *   k_hat    ell_cut + 1 values, the harmonic part K^_l
 *   k_theta  z_cut values, the real-space samples at the nodes in decreasing z
 *   k_real   lmax + 1 values, (P x)_l: Legendre coefficients of the real-space part (input to
 *            conv_real_tabulate for the real-space convolution)
 *   k_tilde  lmax + 1 values, K~_l of Eq. 1
 * 0 <= ell_cut <= lmax; ell_cut = lmax gives x = 0 (all harmonic). */
int conv_split_lsq(conv_split_ctx* ctx, const double* k_ell, int ell_cut, double theta_cut, double* k_hat,
                   double* k_theta, double* k_real, double* k_tilde);

/* Errors of that split: sigma_rms of Eq. 2 and sigma = alpha sigma_rms / sqrt(sum (2l+1) C^in_l K_l^2
 * / 4pi), Eq. 6 with its normalisation weighted like the error (the fractional rms error of the output
 * map; the printed Eq. 6 for C^in = 1, and independent of the scale of C^in). Either output may be NULL. */
int conv_split_error(conv_split_ctx* ctx, const double* k_ell, int ell_cut, double theta_cut, double alpha,
                     double* sigma_rms, double* sigma);

/* Cost model of a split (the paper's Eqs. 7-8 in form, constants measured here, with two terms that
 * Eq. 8 does not carry: the transforms' fixed launch cost and their ring sums, which grow with the
 * pixel count rather than with ell_cut; c0 = c1 = 0 is Eq. 8's form):
 *   t_real = a + b * pairs(nside, theta_cut)                   real-space convolution of one map
 *   t_sht  = c0 + c1 * 12 nside^2 + c * ell_cut^2 * lmax       harmonic-space convolution of one map
 *   wall   = max(t_real, t_sht)                                the two run concurrently */
typedef struct conv_cost_model {
  double a;  /* seconds */
  double b;  /* seconds per pixel pair */
  double c;  /* seconds per ell_cut^2 lmax */
  double c0; /* seconds per harmonic convolution */
  double c1; /* seconds per map pixel of a harmonic convolution */
} conv_cost_model;

/* Estimated pixel pairs of one map: Npix^2 (1 - cos theta_cut) / 2 (each pixel sees the fraction
 * of the sphere inside the cap of radius theta_cut). */
double conv_cost_pairs(int nside, double theta_cut);

/* Least-squares fit of (a, b) to n_real measured real-space times t_real[k] at pairs[k] (n_real >= 2;
 * with one point a = 0), and of (c0, c1, c) to n_sht harmonic times t_sht[k] at npix_sht[k] map pixels
 * and work_sht[k] = ell_cut^2 lmax, both on relative residuals (model / t - 1), so that runs of very
 * different length weigh alike. The harmonic coefficients are kept non-negative: every non-empty subset
 * of the three terms with no more terms than points is fitted, and the one with all coefficients >= 0
 * and the smallest residual wins (the others are 0; a subset with more terms must lower the residual
 * by more than 1e-9 relative and 1e-20 absolute). Times must be > 0, work > 0.
 * Inputs are host arrays. */
int conv_cost_fit(const double* pairs, const double* t_real, int n_real, const double* npix_sht,
                  const double* work_sht, const double* t_sht, int n_sht, conv_cost_model* m);

/* The model's times for one split; outputs may be NULL. */
int conv_cost_eval(const conv_cost_model* m, int nside, int lmax, double theta_cut, int ell_cut, double* t_real,
                   double* t_sht, double* wall);

/* Compensation of a split: max_{l <= ell_cut} |(P x)_l| / max_l |K_l|, the part of the kernel's scale
 * that the harmonic part must cancel at low l (the paper's fits need percent-level adjustments,
 * Results section, discussion of Fig. 3). Splits with few real-space samples inside the cut give
 * large, oscillating samples whose low-l content the pixel-grid sum reproduces far worse than the error
 * model assumes. */
int conv_split_compensation(conv_split_ctx* ctx, const double* k_ell, int ell_cut, double theta_cut, double* comp);

/* Largest compensation the search accepts (max_comp >= 0; 0, the default, accepts any). */
int conv_split_set_max_compensation(conv_split_ctx* ctx, double max_comp);

/* Largest l_cut / lmax the search accepts for a split with a real-space part (0 < frac <= 1; 1, the
 * default, accepts any): a real-space part that carries only multipoles near the grid's resolution
 * meets the error model on paper but not on the pixel grid (measured errors 7-100x the Eq. 6 estimate
 * above l_cut = 0.5 lmax, at most 4.6x below 0.45 lmax). */
int conv_split_set_max_ell_fraction(conv_split_ctx* ctx, double frac);

/* The split search (the paper's scan): for each theta in theta_grid (n_theta values in
 * (0, theta_max]), the smallest ell_cut in {0, s, 2s, ..., lmax} (s = ell_step >= 1) whose Eq. 6
 * error is <= bound, found by bisection (the error falls as ell_cut grows); if it exceeds the
 * context's l_cut limit or its compensation exceeds the context's compensation limit, that theta keeps
 * only ell_cut = lmax (all harmonic, error 0); among
 * these, the pair of least modelled wall time (ties: the smaller theta). Returns CONV_REAL_OK with
 * the pair, or CONV_SPLIT_INFEASIBLE (outputs untouched). Outputs may be NULL. */
int conv_split_search(conv_split_ctx* ctx, const double* k_ell, int nside, double bound, double alpha,
                      const double* theta_grid, int n_theta, int ell_step, const conv_cost_model* m,
                      double* theta_cut, int* ell_cut, double* wall, double* sigma);

/* The search for n kernels at once on worker threads (nthreads <= 0: hardware threads):
 * k_ells is n x (lmax + 1) row-major, bounds[n], theta_grids n x n_theta row-major (one scan grid
 * per kernel); outputs are n-arrays, theta_cut[k] < 0 marks an infeasible kernel. */
int conv_split_search_many(conv_split_ctx* ctx, const double* k_ells, int n, int nside, const double* bounds,
                           double alpha, const double* theta_grids, int n_theta, int ell_step,
                           const conv_cost_model* m, int nthreads, double* theta_cut, int* ell_cut, double* wall,
                           double* sigma);

#ifdef __cplusplus
}
#endif

#endif /* CONVSPLIT_H */
