// Kernel-split model of libconvreal: Gauss-Legendre real-space samples, the Legendre operator,
// the reduced least-squares split (Eqs. 3-5), its errors (Eqs. 2 and 6), the cost model and the
// split search. Host-side FP64.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/convsplit.h"
#include "internal.h"

using convreal::set_error;

namespace {

// Singular values and right singular vectors of an m x n matrix B (column-major, destroyed),
// m >= n: Householder QR, B = Q R, then one-sided Jacobi (Hestenes) rotations on the columns of R,
// R V = U diag(s). Both steps keep small singular values to high relative accuracy (forming B^T B
// would square the condition number), which the relative cutoff of the split relies on.
// Outputs: s[n] (column norms, unsorted) and V (n x n row-major, columns are the vectors).
void householder_jacobi_svd(int m, int n, std::vector<double>& B, std::vector<double>& s, std::vector<double>& V) {
  auto b = [&](int i, int j) -> double& { return B[static_cast<size_t>(j) * m + i]; };
  for (int k = 0; k < n; ++k) {
    double tail2 = 0.0;
    for (int i = k + 1; i < m; ++i) tail2 += b(i, k) * b(i, k);
    const double norm = std::sqrt(b(k, k) * b(k, k) + tail2);
    if (norm == 0.0) continue;
    const double alpha = b(k, k) > 0.0 ? -norm : norm;  // reflect onto -sign(b_kk) |x| e_k
    const double v0 = b(k, k) - alpha;                  // no cancellation: opposite signs
    // reflector H = I - 2 v v^T / (v^T v), v = (v0, b(k+1..m-1, k))
    const double vtv = v0 * v0 + tail2;
    b(k, k) = alpha;
    if (vtv == 0.0) continue;
    for (int j = k + 1; j < n; ++j) {
      double d = v0 * b(k, j);
      for (int i = k + 1; i < m; ++i) d += b(i, k) * b(i, j);
      const double f = 2.0 * d / vtv;
      b(k, j) -= f * v0;
      for (int i = k + 1; i < m; ++i) b(i, j) -= f * b(i, k);
    }
  }
  // R: upper triangle of the first n rows, stored column-major n x n
  std::vector<double> R(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) R[static_cast<size_t>(j) * n + i] = b(i, j);
  V.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[static_cast<size_t>(i) * n + i] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double* cp = R.data() + static_cast<size_t>(p) * n;
        double* cq = R.data() + static_cast<size_t>(q) * n;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = 0; i < n; ++i) {
          al += cp[i] * cp[i];
          be += cq[i] * cq[i];
          ga += cp[i] * cq[i];
        }
        if (!(std::fabs(ga) > tol * std::sqrt(al * be))) continue;
        rotated = true;
        // rotation that makes columns p and q orthogonal: tan(2 phi) = 2 ga / (be - al), smaller root
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double sn = c * t;
        for (int i = 0; i < n; ++i) {
          const double x = cp[i], y = cq[i];
          cp[i] = c * x - sn * y;
          cq[i] = sn * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          double& vkp = V[static_cast<size_t>(k) * n + p];
          double& vkq = V[static_cast<size_t>(k) * n + q];
          const double x = vkp, y = vkq;
          vkp = c * x - sn * y;
          vkq = sn * x + c * y;
        }
      }
    }
    if (!rotated) break;
  }
  s.resize(n);
  for (int j = 0; j < n; ++j) {
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += R[static_cast<size_t>(j) * n + i] * R[static_cast<size_t>(j) * n + i];
    s[j] = std::sqrt(a);
  }
}

// Nodes z_k and weights w_k of the n-point Gauss-Legendre rule with z_k > zmin, in decreasing z:
// Newton's method on P_n from the usual asymptotic first guesses.
void gauss_legendre_above(int n, double zmin, std::vector<double>& z, std::vector<double>& w) {
  z.clear();
  w.clear();
  for (int k = 1; k <= n; ++k) {
    double x = std::cos(M_PI * (k - 0.25) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int l = 1; l < n; ++l) {
        const double p2 = ((2.0 * l + 1.0) * x * p1 - l * p0) / (l + 1.0);
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(x), p0 = P_{n-1}(x); P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1)
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) <= 1e-16 * std::max(1.0, std::fabs(x))) {
        // derivative at the converged node for the weight
        p0 = 1.0;
        p1 = x;
        for (int l = 1; l < n; ++l) {
          const double p2 = ((2.0 * l + 1.0) * x * p1 - l * p0) / (l + 1.0);
          p0 = p1;
          p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        break;
      }
    }
    if (!(x > zmin)) break;
    z.push_back(x);
    w.push_back(2.0 / ((1.0 - x * x) * dp * dp));
  }
}

constexpr size_t kCacheBytes = size_t(512) << 20;  // decompositions kept per context

// Singular values s_k and right singular vectors of the reduced weighted problem W_r^1/2 P_r
struct Svd {
  std::vector<double> s;  // n
  std::vector<double> V;  // n x n row-major, columns are the vectors
};

}  // namespace

struct conv_split_ctx {
  int lmax = 0;
  double theta_max = 0.0;
  double sv_cut = 1e-6;
  double max_comp = 0.0;   // search: largest accepted max_{l <= l_cut} |(P x)_l| / max_l |K_l| (0: no limit)
  double max_ell_frac = 1.0;  // search: largest accepted l_cut / lmax below lmax itself (1: no limit)
  std::vector<double> W;   // (2l + 1) C_l
  std::vector<double> z, w;
  int nmax = 0;
  std::vector<double> P;   // (lmax + 1) x nmax row-major: 2 pi w_k P_l(z_k)
  std::mutex mu;
  // (z_cut, ell_cut) -> singular values and vectors of the reduced problem; shared so that a worker
  // keeps its entry alive when another one clears the cache
  std::map<std::pair<int, int>, std::shared_ptr<const Svd>> cache;
  size_t cache_bytes = 0;
};

namespace {

int count_nodes(const conv_split_ctx* c, double theta_cut) {
  const double zc = std::cos(theta_cut);
  int n = 0;
  while (n < c->nmax && c->z[n] > zc) ++n;
  return n;
}

// SVD of the reduced problem's matrix B = W_r^1/2 P_r: rows l = ell_cut + 1..lmax, columns the
// first n samples. It does not depend on the kernel, so it is cached per (n, ell_cut).
std::shared_ptr<const Svd> reduced_svd(conv_split_ctx* c, int n, int ell_cut) {
  {
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->cache.find({n, ell_cut});
    if (it != c->cache.end()) return it->second;
  }
  const int rows = c->lmax - ell_cut;
  const int m = std::max(rows, n);  // zero rows past the problem's own leave its singular values as they are
  std::vector<double> B(static_cast<size_t>(m) * n, 0.0);
  for (int r = 0; r < rows; ++r) {
    const int l = ell_cut + 1 + r;
    const double* p = c->P.data() + static_cast<size_t>(l) * c->nmax;
    const double sw = std::sqrt(c->W[l]);
    for (int k = 0; k < n; ++k) B[static_cast<size_t>(k) * m + r] = sw * p[k];
  }
  auto e = std::make_shared<Svd>();
  householder_jacobi_svd(m, n, B, e->s, e->V);
  std::lock_guard<std::mutex> g(c->mu);
  const size_t bytes = sizeof(double) * (static_cast<size_t>(n) * n + n);
  if (c->cache_bytes + bytes > kCacheBytes) {
    c->cache.clear();
    c->cache_bytes = 0;
  }
  auto res = c->cache.emplace(std::make_pair(n, ell_cut), e);
  if (res.second) c->cache_bytes += bytes;
  return res.first->second;
}

// Solve the reduced problem; x has n entries (n = 0: nothing to solve). With B = U diag(s) V^T,
// x = sum over kept k of v_k (u_k . W_r^1/2 K_r) / s_k = sum v_k (v_k . P_r^T W_r K_r) / s_k^2, keeping
// s_k >= sv_cut * max s.
void solve_reduced(conv_split_ctx* c, const double* K, int ell_cut, int n, std::vector<double>& x) {
  x.assign(n, 0.0);
  if (n == 0 || ell_cut >= c->lmax) return;
  std::vector<double> rhs(n, 0.0);
  for (int l = ell_cut + 1; l <= c->lmax; ++l) {
    const double* p = c->P.data() + static_cast<size_t>(l) * c->nmax;
    const double f = c->W[l] * K[l];
    for (int k = 0; k < n; ++k) rhs[k] += p[k] * f;
  }
  const std::shared_ptr<const Svd> ep = reduced_svd(c, n, ell_cut);
  const Svd& e = *ep;
  double smax = 0.0;
  for (double v : e.s) smax = std::max(smax, v);
  for (int i = 0; i < n; ++i) {
    if (!(e.s[i] >= c->sv_cut * smax) || !(e.s[i] > 0.0)) continue;
    double proj = 0.0;
    for (int k = 0; k < n; ++k) proj += e.V[static_cast<size_t>(k) * n + i] * rhs[k];
    proj /= e.s[i] * e.s[i];
    for (int k = 0; k < n; ++k) x[k] += e.V[static_cast<size_t>(k) * n + i] * proj;
  }
}

// Eq. 2 sigma_rms^2 * 4 pi and the Eq. 6 normalisation * 4 pi for the split with samples x. The
// normalisation carries the same input weights C^in_l as the error (the output map's power), which is
// the printed Eq. 6 for the flat C^in = 1.
void split_sums(const conv_split_ctx* c, const double* K, int ell_cut, int n, const std::vector<double>& x,
                double* err_sum, double* norm_sum) {
  double es = 0.0, ns = 0.0;
  for (int l = 0; l <= c->lmax; ++l) {
    ns += c->W[l] * K[l] * K[l];
    if (l <= ell_cut) continue;
    const double* p = c->P.data() + static_cast<size_t>(l) * c->nmax;
    double kr = 0.0;
    for (int k = 0; k < n; ++k) kr += p[k] * x[k];
    const double r = K[l] - kr;
    es += c->W[l] * r * r;
  }
  *err_sum = es;
  *norm_sum = ns;
}

int check_ctx(const conv_split_ctx* c, const char* who) {
  if (!c) {
    set_error(std::string(who) + ": NULL context");
    return CONV_REAL_EINVAL;
  }
  return CONV_REAL_OK;
}

int check_split(const conv_split_ctx* c, const double* k_ell, int ell_cut, double theta_cut, const char* who) {
  if (int e = check_ctx(c, who)) return e;
  if (!k_ell) {
    set_error(std::string(who) + ": NULL k_ell");
    return CONV_REAL_EINVAL;
  }
  if (ell_cut < 0 || ell_cut > c->lmax) {
    set_error(std::string(who) + ": ell_cut must be in [0, lmax]");
    return CONV_REAL_EINVAL;
  }
  if (!(theta_cut > 0.0) || !(theta_cut <= c->theta_max * (1.0 + 1e-12))) {
    set_error(std::string(who) + ": theta_cut must be in (0, theta_max]");
    return CONV_REAL_EINVAL;
  }
  return CONV_REAL_OK;
}

// Compensation of a split: the largest |(P x)_l| for l <= ell_cut (what the harmonic part must cancel
// of the real-space part's low-l content) over the largest |K_l|.
double compensation_of(conv_split_ctx* c, const double* K, int ell_cut, double theta_cut) {
  const int n = count_nodes(c, theta_cut);
  std::vector<double> x;
  solve_reduced(c, K, ell_cut, n, x);
  double kmax = 0.0, cmax = 0.0;
  for (int l = 0; l <= c->lmax; ++l) kmax = std::max(kmax, std::fabs(K[l]));
  for (int l = 0; l <= ell_cut; ++l) {
    const double* p = c->P.data() + static_cast<size_t>(l) * c->nmax;
    double kr = 0.0;
    for (int k = 0; k < n; ++k) kr += p[k] * x[k];
    cmax = std::max(cmax, std::fabs(kr));
  }
  return kmax > 0.0 ? cmax / kmax : 0.0;
}

double sigma_of(conv_split_ctx* c, const double* K, int ell_cut, double theta_cut, double alpha) {
  const int n = count_nodes(c, theta_cut);
  std::vector<double> x;
  solve_reduced(c, K, ell_cut, n, x);
  double es, ns;
  split_sums(c, K, ell_cut, n, x, &es, &ns);
  return ns > 0.0 ? alpha * std::sqrt(es / ns) : 0.0;
}

// the scan for one kernel; returns true if some pair meets the bound
bool search_one(conv_split_ctx* c, const double* K, int nside, double bound, double alpha, const double* grid,
                int n_theta, int step, const conv_cost_model* m, double* th_out, int* lc_out, double* wall_out,
                double* sig_out) {
  bool found = false;
  double best_wall = 0.0, best_th = 0.0, best_sig = 0.0;
  int best_lc = 0;
  const int lmax = c->lmax;
  const int nsteps = lmax / step;  // candidates s * k for k = 0..nsteps, then lmax itself
  auto cand = [&](int k) { return k > nsteps ? lmax : std::min(lmax, k * step); };
  for (int g = 0; g < n_theta; ++g) {
    const double th = grid[g];
    // smallest feasible candidate index: the error falls as ell_cut grows; lmax is always exact
    int hi = nsteps + 1;               // lmax: error 0
    double sig_hi = 0.0;
    if (!(sigma_of(c, K, lmax, th, alpha) <= bound)) continue;
    int lo = -1;                       // index known infeasible (virtual)
    const double s0 = sigma_of(c, K, cand(0), th, alpha);
    if (s0 <= bound) {
      hi = 0;
      sig_hi = s0;
    } else {
      lo = 0;
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        const double s = sigma_of(c, K, cand(mid), th, alpha);
        if (s <= bound) {
          hi = mid;
          sig_hi = s;
        } else {
          lo = mid;
        }
      }
      if (hi == nsteps + 1) sig_hi = 0.0;
    }
    int lc = cand(hi);
    // a split whose harmonic part must cancel more than max_comp of the kernel's scale at low l is not
    // trusted (the pixel-grid sum cannot reproduce such large low-l content to the error model's
    // precision): this theta then keeps only the all-harmonic split
    if (lc < lmax && (static_cast<double>(lc) > c->max_ell_frac * lmax ||
                      (c->max_comp > 0.0 && compensation_of(c, K, lc, th) > c->max_comp))) {
      lc = lmax;
      sig_hi = 0.0;
    }
    double w = 0.0;
    conv_cost_eval(m, nside, lmax, th, lc, nullptr, nullptr, &w);
    if (!found || w < best_wall) {
      found = true;
      best_wall = w;
      best_th = th;
      best_lc = lc;
      best_sig = sig_hi;
    }
  }
  if (found) {
    if (th_out) *th_out = best_th;
    if (lc_out) *lc_out = best_lc;
    if (wall_out) *wall_out = best_wall;
    if (sig_out) *sig_out = best_sig;
  }
  return found;
}

int check_search(const conv_split_ctx* c, int nside, double alpha, const double* grid, int n_theta, int step,
                 const conv_cost_model* m, const char* who) {
  if (int e = check_ctx(c, who)) return e;
  if (!grid || n_theta <= 0 || !m) {
    set_error(std::string(who) + ": NULL grid or model, or empty grid");
    return CONV_REAL_EINVAL;
  }
  if (nside < 1 || nside > CONV_REAL_MAX_NSIDE || step < 1 || !(alpha > 0.0)) {
    set_error(std::string(who) + ": bad nside, ell_step or alpha");
    return CONV_REAL_EINVAL;
  }
  for (int g = 0; g < n_theta; ++g) {
    if (!(grid[g] > 0.0) || !(grid[g] <= c->theta_max * (1.0 + 1e-12))) {
      set_error(std::string(who) + ": theta_grid values must be in (0, theta_max]");
      return CONV_REAL_EINVAL;
    }
  }
  return CONV_REAL_OK;
}

// Harmonic cost t = c0 + c1 npix + c work on relative residuals, coefficients >= 0: every non-empty
// subset of the three terms with no more terms than points, by weighted least squares (normal equations
// of the rows r_j / t_k, columns scaled to unit maximum); the feasible subset with the smallest residual
// wins (fewer terms unless more lower the residual beyond rounding). coef = {c0, c1, c}.
bool fit_harmonic(const double* npix, const double* work, const double* t, int n, double (&coef)[3]) {
  auto reg = [&](int k, int j) { return j == 0 ? 1.0 : (j == 1 ? npix[k] : work[k]); };
  double scale[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < 3; ++j) scale[j] = std::max(scale[j], reg(k, j) / t[k]);
  bool found = false;
  double best = 0.0;
  // subsets in order of size, then by mask
  static const int kMasks[7] = {1, 2, 4, 3, 5, 6, 7};
  for (int mask : kMasks) {
    int idx[3], p = 0;
    for (int j = 0; j < 3; ++j)
      if (mask & (1 << j)) idx[p++] = j;
    if (p > n) continue;
    // normal equations N y = v for y_q = x_idx[q] * scale[idx[q]]
    double N[3][3] = {}, v[3] = {};
    for (int k = 0; k < n; ++k) {
      double row[3];
      for (int q = 0; q < p; ++q) row[q] = reg(k, idx[q]) / t[k] / scale[idx[q]];
      for (int q = 0; q < p; ++q) {
        v[q] += row[q];
        for (int r = 0; r < p; ++r) N[q][r] += row[q] * row[r];
      }
    }
    // Gaussian elimination with partial pivoting
    bool ok = true;
    for (int c = 0; c < p && ok; ++c) {
      int piv = c;
      for (int r = c + 1; r < p; ++r)
        if (std::fabs(N[r][c]) > std::fabs(N[piv][c])) piv = r;
      if (!(std::fabs(N[piv][c]) > 1e-300)) {
        ok = false;
        break;
      }
      if (piv != c) {
        for (int q = 0; q < p; ++q) std::swap(N[c][q], N[piv][q]);
        std::swap(v[c], v[piv]);
      }
      for (int r = c + 1; r < p; ++r) {
        const double f = N[r][c] / N[c][c];
        for (int q = c; q < p; ++q) N[r][q] -= f * N[c][q];
        v[r] -= f * v[c];
      }
    }
    if (!ok) continue;
    double y[3] = {0.0, 0.0, 0.0};
    for (int c = p - 1; c >= 0; --c) {
      double acc = v[c];
      for (int q = c + 1; q < p; ++q) acc -= N[c][q] * y[q];
      y[c] = acc / N[c][c];
    }
    double x[3] = {0.0, 0.0, 0.0};
    bool feasible = true;
    for (int q = 0; q < p; ++q) {
      x[idx[q]] = y[q] / scale[idx[q]];
      if (!(x[idx[q]] >= 0.0) || !std::isfinite(x[idx[q]])) feasible = false;
    }
    if (!feasible) continue;
    double res = 0.0;
    for (int k = 0; k < n; ++k) {
      const double d = (x[0] + x[1] * npix[k] + x[2] * work[k]) / t[k] - 1.0;
      res += d * d;
    }
    // subsets come in order of size: a larger one must lower the residual beyond rounding (1e-9
    // relative, 1e-20 absolute), so that an exact fit of fewer terms stays
    if (!found || res < best * (1.0 - 1e-9) - 1e-20) {
      found = true;
      best = res;
      for (int j = 0; j < 3; ++j) coef[j] = x[j];
    }
  }
  return found;
}

}  // namespace

extern "C" {

int conv_split_create(conv_split_ctx** ctx, int lmax, const double* c_in, double theta_max, double sv_cut) {
  if (!ctx) {
    set_error("conv_split_create: NULL ctx");
    return CONV_REAL_EINVAL;
  }
  if (lmax < 1 || lmax > CONV_REAL_MAX_LMAX || !(theta_max > 0.0) || !(theta_max <= M_PI) || !(sv_cut > 0.0) ||
      !(sv_cut < 1.0)) {
    set_error("conv_split_create: need 1 <= lmax <= CONV_REAL_MAX_LMAX, theta_max in (0, pi], sv_cut in (0, 1)");
    return CONV_REAL_EINVAL;
  }
  conv_split_ctx* c = new (std::nothrow) conv_split_ctx;
  if (!c) {
    set_error("conv_split_create: out of memory");
    return CONV_REAL_ENOMEM;
  }
  c->lmax = lmax;
  c->theta_max = theta_max;
  c->sv_cut = sv_cut;
  c->W.resize(lmax + 1);
  for (int l = 0; l <= lmax; ++l) {
    const double cl = c_in ? c_in[l] : 1.0;
    if (!(cl >= 0.0) || !std::isfinite(cl)) {
      delete c;
      set_error("conv_split_create: c_in must be finite and >= 0");
      return CONV_REAL_EINVAL;
    }
    c->W[l] = (2.0 * l + 1.0) * cl;
  }
  gauss_legendre_above(lmax + 1, std::cos(theta_max), c->z, c->w);
  c->nmax = static_cast<int>(c->z.size());
  c->P.assign(static_cast<size_t>(lmax + 1) * std::max(c->nmax, 1), 0.0);
  for (int k = 0; k < c->nmax; ++k) {
    const double x = c->z[k], f = 2.0 * M_PI * c->w[k];
    double p0 = 1.0, p1 = x;
    c->P[k] = f;
    if (lmax >= 1) c->P[static_cast<size_t>(c->nmax) + k] = f * x;
    for (int l = 1; l < lmax; ++l) {
      const double p2 = ((2.0 * l + 1.0) * x * p1 - l * p0) / (l + 1.0);
      p0 = p1;
      p1 = p2;
      c->P[static_cast<size_t>(l + 1) * c->nmax + k] = f * p2;
    }
  }
  *ctx = c;
  return CONV_REAL_OK;
}

int conv_split_destroy(conv_split_ctx* ctx) {
  delete ctx;
  return CONV_REAL_OK;
}

int conv_split_nodes(const conv_split_ctx* ctx, double theta_cut, int* z_cut) {
  if (int e = check_ctx(ctx, "conv_split_nodes")) return e;
  if (!z_cut || !(theta_cut > 0.0) || !(theta_cut <= ctx->theta_max * (1.0 + 1e-12))) {
    set_error("conv_split_nodes: NULL z_cut or theta_cut outside (0, theta_max]");
    return CONV_REAL_EINVAL;
  }
  *z_cut = count_nodes(ctx, theta_cut);
  return CONV_REAL_OK;
}

int conv_split_lsq(conv_split_ctx* ctx, const double* k_ell, int ell_cut, double theta_cut, double* k_hat,
                   double* k_theta, double* k_real, double* k_tilde) {
  if (int e = check_split(ctx, k_ell, ell_cut, theta_cut, "conv_split_lsq")) return e;
  const int n = count_nodes(ctx, theta_cut);
  std::vector<double> x;
  solve_reduced(ctx, k_ell, ell_cut, n, x);
  const int lmax = ctx->lmax;
  std::vector<double> kr(lmax + 1, 0.0);
  for (int l = 0; l <= lmax; ++l) {
    const double* p = ctx->P.data() + static_cast<size_t>(l) * ctx->nmax;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += p[k] * x[k];
    kr[l] = s;
  }
  if (k_hat)
    for (int l = 0; l <= ell_cut; ++l) k_hat[l] = k_ell[l] - kr[l];
  if (k_theta)
    for (int k = 0; k < n; ++k) k_theta[k] = x[k];
  if (k_real)
    for (int l = 0; l <= lmax; ++l) k_real[l] = kr[l];
  if (k_tilde)
    for (int l = 0; l <= lmax; ++l) k_tilde[l] = l <= ell_cut ? k_ell[l] : kr[l];
  return CONV_REAL_OK;
}

int conv_split_error(conv_split_ctx* ctx, const double* k_ell, int ell_cut, double theta_cut, double alpha,
                     double* sigma_rms, double* sigma) {
  if (int e = check_split(ctx, k_ell, ell_cut, theta_cut, "conv_split_error")) return e;
  const int n = count_nodes(ctx, theta_cut);
  std::vector<double> x;
  solve_reduced(ctx, k_ell, ell_cut, n, x);
  double es, ns;
  split_sums(ctx, k_ell, ell_cut, n, x, &es, &ns);
  if (sigma_rms) *sigma_rms = std::sqrt(es / (4.0 * M_PI));
  if (sigma) *sigma = ns > 0.0 ? alpha * std::sqrt(es / ns) : 0.0;
  return CONV_REAL_OK;
}

double conv_cost_pairs(int nside, double theta_cut) {
  const double npix = 12.0 * static_cast<double>(nside) * static_cast<double>(nside);
  const double th = std::min(std::max(theta_cut, 0.0), M_PI);
  // 1 - cos(theta) = 2 sin^2(theta / 2), without cancellation at small theta
  const double s = std::sin(0.5 * th);
  return npix * npix * s * s;
}

int conv_cost_fit(const double* pairs, const double* t_real, int n_real, const double* npix_sht,
                  const double* work_sht, const double* t_sht, int n_sht, conv_cost_model* m) {
  if (!pairs || !t_real || !npix_sht || !work_sht || !t_sht || !m || n_real < 1 || n_sht < 1) {
    set_error("conv_cost_fit: NULL argument or empty measurement set");
    return CONV_REAL_EINVAL;
  }
  // relative residuals: every measured point weighs by 1 / t^2, so that millisecond and
  // second-scale runs count alike
  for (int k = 0; k < n_real; ++k)
    if (!(t_real[k] > 0.0)) {
      set_error("conv_cost_fit: real-space times must be > 0");
      return CONV_REAL_EINVAL;
    }
  for (int k = 0; k < n_sht; ++k)
    if (!(t_sht[k] > 0.0)) {
      set_error("conv_cost_fit: harmonic times must be > 0");
      return CONV_REAL_EINVAL;
    }
  double a = 0.0, b = 0.0;
  if (n_real == 1) {
    if (!(pairs[0] > 0.0)) {
      set_error("conv_cost_fit: pairs must be > 0");
      return CONV_REAL_EINVAL;
    }
    b = t_real[0] / pairs[0];
  } else {
    double s0 = 0, sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (int k = 0; k < n_real; ++k) {
      const double w = 1.0 / (t_real[k] * t_real[k]);
      s0 += w;
      sx += w * pairs[k];
      sy += w * t_real[k];
      sxx += w * pairs[k] * pairs[k];
      sxy += w * pairs[k] * t_real[k];
    }
    const double den = s0 * sxx - sx * sx;
    if (!(std::fabs(den) > 1e-12 * s0 * sxx)) {
      set_error("conv_cost_fit: the pair counts must not all be equal");
      return CONV_REAL_EINVAL;
    }
    b = (s0 * sxy - sx * sy) / den;
    a = (sy - b * sx) / s0;
  }
  for (int k = 0; k < n_sht; ++k)
    if (!(work_sht[k] > 0.0) || !(npix_sht[k] > 0.0)) {
      set_error("conv_cost_fit: harmonic work and pixel counts must be > 0");
      return CONV_REAL_EINVAL;
    }
  double coef[3];
  if (!fit_harmonic(npix_sht, work_sht, t_sht, n_sht, coef)) {
    set_error("conv_cost_fit: no non-negative fit of the harmonic times");
    return CONV_REAL_EINVAL;
  }
  m->a = a;
  m->b = b;
  m->c0 = coef[0];
  m->c1 = coef[1];
  m->c = coef[2];
  return CONV_REAL_OK;
}

int conv_cost_eval(const conv_cost_model* m, int nside, int lmax, double theta_cut, int ell_cut, double* t_real,
                   double* t_sht, double* wall) {
  if (!m || nside < 1 || lmax < 0 || ell_cut < 0 || !(theta_cut >= 0.0)) {
    set_error("conv_cost_eval: bad argument");
    return CONV_REAL_EINVAL;
  }
  const double tr = m->a + m->b * conv_cost_pairs(nside, theta_cut);
  const double npix = 12.0 * static_cast<double>(nside) * static_cast<double>(nside);
  const double ts = m->c0 + m->c1 * npix +
                    m->c * static_cast<double>(ell_cut) * static_cast<double>(ell_cut) * static_cast<double>(lmax);
  if (t_real) *t_real = tr;
  if (t_sht) *t_sht = ts;
  if (wall) *wall = std::max(tr, ts);
  return CONV_REAL_OK;
}

int conv_split_set_max_compensation(conv_split_ctx* ctx, double max_comp) {
  if (int e = check_ctx(ctx, "conv_split_set_max_compensation")) return e;
  if (!(max_comp >= 0.0) || !std::isfinite(max_comp)) {
    set_error("conv_split_set_max_compensation: max_comp must be finite and >= 0");
    return CONV_REAL_EINVAL;
  }
  ctx->max_comp = max_comp;
  return CONV_REAL_OK;
}

int conv_split_set_max_ell_fraction(conv_split_ctx* ctx, double frac) {
  if (int e = check_ctx(ctx, "conv_split_set_max_ell_fraction")) return e;
  if (!(frac > 0.0) || !(frac <= 1.0)) {
    set_error("conv_split_set_max_ell_fraction: frac must be in (0, 1]");
    return CONV_REAL_EINVAL;
  }
  ctx->max_ell_frac = frac;
  return CONV_REAL_OK;
}

int conv_split_compensation(conv_split_ctx* ctx, const double* k_ell, int ell_cut, double theta_cut, double* comp) {
  if (int e = check_split(ctx, k_ell, ell_cut, theta_cut, "conv_split_compensation")) return e;
  if (!comp) {
    set_error("conv_split_compensation: NULL output");
    return CONV_REAL_EINVAL;
  }
  *comp = compensation_of(ctx, k_ell, ell_cut, theta_cut);
  return CONV_REAL_OK;
}

int conv_split_search(conv_split_ctx* ctx, const double* k_ell, int nside, double bound, double alpha,
                      const double* theta_grid, int n_theta, int ell_step, const conv_cost_model* m,
                      double* theta_cut, int* ell_cut, double* wall, double* sigma) {
  if (int e = check_search(ctx, nside, alpha, theta_grid, n_theta, ell_step, m, "conv_split_search")) return e;
  if (!k_ell || !(bound > 0.0)) {
    set_error("conv_split_search: NULL k_ell or bound <= 0");
    return CONV_REAL_EINVAL;
  }
  return search_one(ctx, k_ell, nside, bound, alpha, theta_grid, n_theta, ell_step, m, theta_cut, ell_cut, wall,
                    sigma)
             ? CONV_REAL_OK
             : CONV_SPLIT_INFEASIBLE;
}

int conv_split_search_many(conv_split_ctx* ctx, const double* k_ells, int n, int nside, const double* bounds,
                           double alpha, const double* theta_grids, int n_theta, int ell_step,
                           const conv_cost_model* m, int nthreads, double* theta_cut, int* ell_cut, double* wall,
                           double* sigma) {
  if (!k_ells || !bounds || n < 0 || !theta_cut || !ell_cut || !wall || !sigma) {
    set_error("conv_split_search_many: NULL argument or n < 0");
    return CONV_REAL_EINVAL;
  }
  for (int k = 0; k < n; ++k) {
    if (int e = check_search(ctx, nside, alpha, theta_grids + static_cast<size_t>(k) * n_theta, n_theta, ell_step, m,
                             "conv_split_search_many"))
      return e;
    if (!(bounds[k] > 0.0)) {
      set_error("conv_split_search_many: bounds must be > 0");
      return CONV_REAL_EINVAL;
    }
  }
  int nt = nthreads > 0 ? nthreads : static_cast<int>(std::thread::hardware_concurrency());
  nt = std::max(1, std::min(nt, std::max(n, 1)));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const double* K = k_ells + static_cast<size_t>(k) * (ctx->lmax + 1);
      if (!search_one(ctx, K, nside, bounds[k], alpha, theta_grids + static_cast<size_t>(k) * n_theta, n_theta,
                      ell_step, m, &theta_cut[k], &ell_cut[k], &wall[k], &sigma[k])) {
        theta_cut[k] = -1.0;
        ell_cut[k] = -1;
        wall[k] = 0.0;
        sigma[k] = 0.0;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  return CONV_REAL_OK;
}

}  // extern "C"
