"""Kernel splitting: error estimate, weighted least-squares split, cost model, split search (oracle).

Test infrastructure (see the package docstring). Follows the paper's Estimating Errors section:

* Eq. 1   K~_l = K^_l + P_{l theta} K^_theta: the approximate kernel is the truncated harmonic part
          (l <= l_cut) plus the Legendre transform of the truncated real-space part.
* Eq. 2   sigma_rms^2 = (1 / 4 pi) sum_{l=0}^{lmax} (K_l - K~_l)^2 C_l^in (2l + 1).
* Eq. 3-5 A^T W A x = A^T W K_l with x = [K^_l (l <= l_cut); K^_theta (z_cut samples)],
          A = [delta_{l,j} for the harmonic columns | P_{l,k} for the real-space columns],
          W = diag((2l + 1) C_l^in), solved by SVD dropping singular values below 1e-6.
* Eq. 6   sigma^2 = alpha^2 sigma_rms^2 / ((1 / 4 pi) sum (2l + 1) C_l^in K_l^2)  (C^in = 1 as printed).
* Eq. 7-8 cost models (the paper's GTX 480 / one-core fits, seconds, theta_cut in arcmin).
* Search  linear scan over theta_cut; for each, binary search for the smallest l_cut meeting the
          error bound; keep the cheapest pair, the wall time being that of the slower of the two
          convolutions that run in parallel (Fig. 1).

Readings (the paper is silent or garbled on these):
* the Legendre operator acts on the real-space kernel sampled at Gauss-Legendre nodes of an
  (lmax + 1)-point rule: P_{l,k} = 2 pi w_k P_l(z_k), for the nodes with z_k > cos(theta_cut)
  (their count is z_cut; the printed definition "lmax - l_cos(theta_cut)" is garbled);
* A has lmax + 1 rows (l = 0..lmax, as in the sums of Eqs. 2 and 6) and l_cut + 1 harmonic columns;
* W includes C_l^in (the printed W omits it; identical for the flat C_l^in = 1 the paper uses), and so
  does Eq. 6's normalisation (the output's power), so that sigma stays a fractional error for a Wiener
  weighting C^in = C^2 / (C + N);
* the singular-value cutoff is relative to the largest singular value; in the reduced solve (the
  identity block eliminated) it applies to the singular values of the weighted reduced matrix
  W_r^1/2 P_r. Applied to its normal matrix's eigenvalues (the squares) it removes far more and makes
  the Results section's Table 1 cuts miss the 1e-5 bound they were chosen to meet.
"""
from __future__ import annotations

import functools
import itertools
import math

import numpy as np

from . import kernel


@functools.lru_cache(maxsize=8)
def _leggauss(n: int):
    z, w = np.polynomial.legendre.leggauss(n)
    z.setflags(write=False)
    w.setflags(write=False)
    return z, w


def gauss_legendre(lmax: int):
    """Nodes and weights of the (lmax + 1)-point Gauss-Legendre rule on [-1, 1] (kept for reuse:
    the rule costs seconds at lmax 4096)."""
    return _leggauss(lmax + 1)


def real_space_nodes(lmax: int, theta_cut: float):
    """The Gauss-Legendre nodes inside the cut (z > cos theta_cut) and their weights."""
    z, w = gauss_legendre(lmax)
    sel = z > math.cos(theta_cut)
    return z[sel], w[sel]


def legendre_operator(lmax: int, z: np.ndarray, w: np.ndarray) -> np.ndarray:
    """P_{l,k} = 2 pi w_k P_l(z_k), shape [lmax + 1, len(z)]."""
    return 2.0 * math.pi * kernel.legendre_p(lmax, z) * w[None, :]


def design_matrix(lmax: int, ell_cut: int, theta_cut: float):
    """A of Eq. 5: identity block for l <= l_cut, Legendre operator for the real-space samples."""
    z, w = real_space_nodes(lmax, theta_cut)
    P = legendre_operator(lmax, z, w)
    A = np.zeros((lmax + 1, ell_cut + 1 + len(z)))
    A[: ell_cut + 1, : ell_cut + 1] = np.eye(ell_cut + 1)
    A[:, ell_cut + 1:] = P
    return A, z, w


def lsq_split(K_ell: np.ndarray, C_in: np.ndarray, ell_cut: int, theta_cut: float,
              sv_cut: float = 1e-6):
    """Solve A^T W A x = A^T W K (Eq. 3) by SVD, dropping singular values below sv_cut times the
    largest. Returns (K_hat_ell, K_hat_theta, z_nodes, K_tilde_ell)."""
    lmax = len(K_ell) - 1
    A, z, w = design_matrix(lmax, ell_cut, theta_cut)
    Wd = (2.0 * np.arange(lmax + 1) + 1.0) * C_in
    M = A.T @ (Wd[:, None] * A)
    rhs = A.T @ (Wd * K_ell)
    U, s, Vt = np.linalg.svd(M)
    keep = s >= sv_cut * s[0]
    x = Vt[keep].T @ ((U[:, keep].T @ rhs) / s[keep])
    K_tilde = A @ x
    return x[: ell_cut + 1], x[ell_cut + 1:], z, K_tilde


def lsq_split_reduced(K_ell: np.ndarray, C_in: np.ndarray, ell_cut: int, theta_cut: float,
                      sv_cut: float = 1e-6):
    """Eq. 3 with the identity block eliminated. Rows l <= l_cut of A are [e_l | P_l]: K^_l is free
    there, so those residuals vanish at the optimum and x minimises the remaining rows alone,
        sum_{l > l_cut} (2l + 1) C_l (K_l - (P x)_l)^2 = |W_r^1/2 K_r - W_r^1/2 P_r x|^2,
    solved by the SVD of the weighted matrix B = W_r^1/2 P_r, dropping singular values below sv_cut
    times the largest (the cutoff is applied to this problem's singular values, not to the full
    matrix of Eq. 3). Then K^_l = K_l - (P x)_l for l <= l_cut. Returns (K_hat_ell, x, z_nodes, K_tilde)."""
    lmax = len(K_ell) - 1
    z, w = real_space_nodes(lmax, theta_cut)
    P = legendre_operator(lmax, z, w)
    Wd = (2.0 * np.arange(lmax + 1) + 1.0) * C_in
    x = np.zeros(len(z))
    if len(z) > 0 and ell_cut < lmax:
        sw = np.sqrt(Wd[ell_cut + 1:])
        B = sw[:, None] * P[ell_cut + 1:]
        b = sw * K_ell[ell_cut + 1:]
        U, s, Vt = np.linalg.svd(B, full_matrices=False)
        keep = (s >= sv_cut * s.max()) & (s > 0)
        x = Vt[keep].T @ ((U[:, keep].T @ b) / s[keep])
    k_real = P @ x
    K_tilde = np.where(np.arange(lmax + 1) <= ell_cut, K_ell, k_real)
    return K_ell[: ell_cut + 1] - k_real[: ell_cut + 1], x, z, K_tilde


def rms_error(K_ell, K_tilde, C_in) -> float:
    """sigma_rms of Eq. 2."""
    ell = np.arange(len(K_ell))
    return math.sqrt(np.sum((K_ell - K_tilde) ** 2 * C_in * (2 * ell + 1)) / (4.0 * math.pi))


def fractional_error(K_ell, K_tilde, C_in, alpha: float = 5.0) -> float:
    """sigma of Eq. 6. The normalisation carries the input weights of Eq. 2, (1 / 4 pi) sum (2l + 1)
    C^in_l K_l^2 (the output map's power), so that sigma is the fractional rms error of the output; for
    the flat C^in = 1 of the Results section this is the printed Eq. 6."""
    ell = np.arange(len(K_ell))
    norm = np.sum((2 * ell + 1) * np.asarray(C_in, dtype=np.float64) * K_ell ** 2) / (4.0 * math.pi)
    return alpha * rms_error(K_ell, K_tilde, C_in) / math.sqrt(norm)


def wiener_weights(C_ell, N_ell):
    """Input weights for a Wiener-filter convolution (text after Eq. 2): C^in_l = C_l^2 / (C_l + N_l),
    signal power C_l, noise power N_l (zero where both vanish)."""
    C = np.asarray(C_ell, dtype=np.float64)
    N = np.asarray(N_ell, dtype=np.float64) * np.ones_like(C)
    den = C + N
    return np.where(den > 0, C * C / np.where(den > 0, den, 1.0), 0.0)


def cost_gpu_paper(theta_cut_arcmin: float) -> float:
    """Eq. 7: real-space GPU convolution, seconds (GTX 480, Nside 2048, lmax 4096)."""
    return 0.0232 * theta_cut_arcmin + 2.428


def cost_cpu_paper(ell_cut: float, lmax: int = 4096) -> float:
    """Eq. 8: harmonic-space convolution on one CPU core, seconds."""
    return 160.0 * ell_cut ** 2 * lmax / 4096.0 ** 3


def wall_time(t_gpu: float, t_cpu: float) -> float:
    """The two convolutions run concurrently (Fig. 1): the slower one sets the wall time."""
    return max(t_gpu, t_cpu)


def pairs_estimate(nside: int, theta_cut: float) -> float:
    """Pixel pairs of one map within theta_cut, estimated: every one of the Npix pixels sees the
    fraction (1 - cos theta_cut) / 2 of the sphere, i.e. of the Npix pixels."""
    npix = 12.0 * nside * nside
    return npix * npix * (1.0 - math.cos(theta_cut)) / 2.0


def cost_fit(pairs, t_real, npix_sht, work_sht, t_sht):
    """Measured-constant cost model: t_real = a + b pairs (the form of Eq. 7) and t_sht = c0 + c1 npix +
    c ell_cut^2 lmax (Eq. 8's term plus a fixed and a per-pixel term), each fitted by least squares on
    relative residuals (model / t - 1; a = 0 from a single point). The harmonic coefficients must not
    be negative: every non-empty subset of the three terms with no more terms than points is fitted,
    and the subset whose coefficients are all >= 0 with the smallest residual is kept (fewer terms unless
    more lower the residual beyond rounding). Returns (a, b, c, c0, c1)."""
    pairs, t_real = np.asarray(pairs, float), np.asarray(t_real, float)
    npix, work_sht, t_sht = np.asarray(npix_sht, float), np.asarray(work_sht, float), np.asarray(t_sht, float)
    if len(pairs) == 1:
        a, b = 0.0, t_real[0] / pairs[0]
    else:
        # minimise sum ((a + b p_k) / t_k - 1)^2: ordinary least squares on rows [1/t_k, p_k/t_k]
        M = np.stack([1.0 / t_real, pairs / t_real], axis=1)
        (a, b), *_ = np.linalg.lstsq(M, np.ones(len(pairs)), rcond=None)
    R = np.stack([np.ones_like(t_sht), npix, work_sht], axis=1) / t_sht[:, None]   # columns c0, c1, c
    best = None
    for size in (1, 2, 3):
        for cols in itertools.combinations(range(3), size):
            if size > len(t_sht):
                continue
            x, *_ = np.linalg.lstsq(R[:, cols], np.ones(len(t_sht)), rcond=None)
            if np.any(x < 0) or not np.all(np.isfinite(x)):
                continue
            res = float(np.sum((R[:, cols] @ x - 1.0) ** 2))
            # a subset with more terms must lower the residual by more than rounding (1e-9 relative,
            # 1e-20 absolute: an exact fit of fewer terms stays)
            if best is None or res < best[0] * (1.0 - 1e-9) - 1e-20:
                coef = np.zeros(3)
                coef[list(cols)] = x
                best = (res, coef)
    c0, c1, c = best[1]
    return float(a), float(b), float(c), float(c0), float(c1)


def compensation(K_ell, K_hat, K_tilde) -> float:
    """What the harmonic part cancels of the real-space part at low l: by Eq. 1, (P K^_theta)_l =
    K~_l - K^_l for l <= l_cut; its largest magnitude over the largest |K_l|."""
    lc = len(K_hat) - 1
    return float(np.max(np.abs(np.asarray(K_tilde)[: lc + 1] - np.asarray(K_hat))) / np.max(np.abs(K_ell)))


def split_search(K_ell, C_in, bound: float, theta_grid, t_gpu, t_cpu, alpha: float = 5.0,
                 sv_cut: float = 1e-6, solver=None, max_comp: float = 0.0, max_ell_frac: float = 1.0):
    """Scan theta_cut; binary-search the smallest feasible l_cut for each; keep the cheapest.
    solver is the least-squares split to use (default: the full solve of Eq. 3). A theta whose
    smallest feasible l_cut below lmax exceeds max_ell_frac lmax, or (max_comp > 0) whose split has a
    compensation above max_comp, keeps only l_cut = lmax.
    Returns (theta_cut, ell_cut, wall, error) or None if no pair meets the bound."""
    lmax = len(K_ell) - 1
    solve = lsq_split if solver is None else solver

    def err(lc, tc):
        _, _, _, kt = solve(K_ell, C_in, lc, tc, sv_cut)
        return fractional_error(K_ell, kt, C_in, alpha)

    def comp(lc, tc):
        kh, _, _, kt = solve(K_ell, C_in, lc, tc, sv_cut)
        return compensation(K_ell, kh, kt)

    best = None
    for tc in theta_grid:
        if err(lmax, tc) > bound:
            continue
        lo, hi = 0, lmax
        if err(lo, tc) <= bound:
            hi = lo
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if err(mid, tc) <= bound:
                hi = mid
            else:
                lo = mid
        if hi < lmax and (hi > max_ell_frac * lmax or (max_comp > 0 and comp(hi, tc) > max_comp)):
            hi = lmax
        wall = wall_time(t_gpu(tc), t_cpu(hi))
        if best is None or wall < best[2]:
            best = (tc, hi, wall, err(hi, tc))
    return best
