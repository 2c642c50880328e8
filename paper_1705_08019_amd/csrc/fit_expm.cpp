// C ABI of the operator, matrix-exponential and ParaExp building blocks
// (Sec. III-A, Sec. III): apply B, estimate ||A||_2, exp(tB) by scaling and a
// truncated Taylor recurrence, the half-step h transform, axpy.
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "fit_host.hpp"

namespace fit {

// ---------------------------------------------------------------- (m, s)
// For a normal operator with spectrum in [-i rho, i rho] one Taylor sub-step
// h = t / s misses exp(hA) by at most delta = (rho h)^(m+1) / (m+1)! (the
// Lagrange remainder on the imaginary axis) and has norm <= 1 + delta, so s
// sub-steps are within s delta (1 + delta)^(s-1) relative.  The terms of a
// sub-step sum to at most e^(rho h) in norm against a result of norm 1, so
// rounding with unit roundoff u adds about s (m + 2) u e^(rho h).  The pair
// with the fewest operator applications m s whose sum of both stays within
// tol is taken (ties: fewer sub-steps).
static double taylor_bound(double theta, int m, int64_t s, double u) {
  if (theta == 0.0) return 0.0;
  const double log_delta = (m + 1) * std::log(theta / (double)s) - std::lgamma(m + 2.0);
  if (log_delta > 50.0 || theta / (double)s > 700.0) return INFINITY;
  const double delta = std::exp(log_delta);
  const double log_trunc = std::log((double)s) + log_delta + (double)(s - 1) * std::log1p(delta);
  const double log_round = std::log((double)s * (m + 2) * u) + theta / (double)s;
  if (std::max(log_trunc, log_round) > 700.0) return INFINITY;
  return std::exp(log_trunc) + std::exp(log_round);
}

// Smallest s with bound(s) <= tol, or -1, for a bound that falls with s on
// s <= theta (bisection there); beyond, s* (3/2)^q, q = 1..6, are tried and
// the first feasible one is bisected down to the previous sample.
template <typename F>
static int64_t first_feasible_s(double theta, double tol, F bound) {
  const int64_t s_star = std::max<int64_t>(1, (int64_t)std::ceil(theta));
  int64_t lo = -1, hi = -1;
  if (bound(s_star) <= tol) {
    lo = 1;
    hi = s_star;
  } else {
    int64_t prev = s_star;
    for (int q = 1; q <= 6; ++q) {
      const int64_t cand = (int64_t)std::ceil((double)s_star * std::pow(1.5, q));
      if (bound(cand) <= tol) {
        lo = prev + 1;
        hi = cand;
        break;
      }
      prev = cand;
    }
  }
  if (lo < 0) return -1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (bound(mid) <= tol) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

static int64_t first_feasible(double theta, int m, double tol, double u) {
  return first_feasible_s(theta, tol, [&](int64_t s) { return taylor_bound(theta, m, s, u); });
}

static bool taylor_params(double theta, double tol, double u, int* m_out, int64_t* s_out) {
  if (theta == 0.0) {
    *m_out = 0;
    *s_out = 1;
    return true;
  }
  int64_t best_cost = -1, best_s = 1;
  int best_m = 1;
  for (int m = 1; m <= 60; ++m) {
    const int64_t s = first_feasible(theta, m, tol, u);
    if (s < 0) continue;
    const int64_t cost = (int64_t)m * s;
    if (best_cost < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best_cost = cost;
      best_m = m;
      best_s = s;
    }
  }
  if (best_cost < 0) return false;
  *m_out = best_m;
  *s_out = best_s;
  return true;
}

// ---------------------------------------------------------------- Leja
// Newton interpolation of exp at conjugate pairs +-i c a_j of points on the
// imaginary interval i[-c, c] (Sec. III-A).  The squares x_j = a_j^2 form a
// Leja sequence of [0, 1] on the grid (1 - cos(pi i / 4000)) / 2: x_0 = 1,
// then each point maximises the product of distances to the previous ones
// (first index on ties).  In the basis of pair factors,
//   p(z) = sum_k (alpha_k + beta_k z) prod_{j<k} (z^2 + c^2 x_j),
// alpha_k = d_2k - d_2k+1 (i c a_k), beta_k = d_2k+1 with d the divided
// differences of exp at (i c a_0, -i c a_0, i c a_1, ...), real for such
// symmetric points.  The divided differences are exp(Z) e_0 for the lower
// bidiagonal Z (points on the diagonal, ones below), computed by repeated
// Taylor steps of Z / n_s on the vector.  Remainder on the imaginary axis:
// prod |z - z_j| / (2K)!, so one step misses exp(hA) by at most
// delta = max_{tau in [0, c^2]} prod_j |tau - c^2 x_j| / (2K)! (maximum over
// 4001 Chebyshev points of the interval, raised by 0.1 %), c = rho h; s steps
// by s delta (1 + delta)^(s-1); rounding adds about s (2K + 1) u S with
// S = max(1, sum_k (|alpha_k| + c |beta_k|) N_k), N_k the same maximum over
// the first k factors.  (K, s) minimise (2K - 1) s, the applications of B.
constexpr int kLejaCand = 4000;
constexpr int kLejaKMax = 30;

static const std::vector<double>& leja_cand() {
  static const std::vector<double> c = [] {
    std::vector<double> v(kLejaCand + 1);
    for (int i = 0; i <= kLejaCand; ++i) v[i] = 0.5 * (1.0 - std::cos(M_PI * i / kLejaCand));
    return v;
  }();
  return c;
}

static const std::vector<double>& leja_squares() {
  static const std::vector<double> xs = [] {
    const std::vector<double>& cand = leja_cand();
    std::vector<double> lp(cand.size()), out{1.0};
    for (size_t i = 0; i < cand.size(); ++i) lp[i] = std::log(std::fabs(cand[i] - 1.0));
    while ((int)out.size() < kLejaKMax) {
      size_t best = 0;
      for (size_t i = 1; i < cand.size(); ++i)
        if (lp[i] > lp[best]) best = i;
      const double xb = cand[best];
      out.push_back(xb);
      for (size_t i = 0; i < cand.size(); ++i) lp[i] += std::log(std::fabs(cand[i] - xb));
    }
    return out;
  }();
  return xs;
}

// Unscaled pair coefficients of the K-pair interpolant on i[-c, c].
static void leja_pairs(int K, double c, double* alpha, double* beta, double* a2) {
  typedef std::complex<double> cd;
  const std::vector<double>& x = leja_squares();
  const int n = 2 * K;
  std::vector<cd> z(n), d(n, cd(0.0)), term(n), nxt(n), acc(n);
  double zmax = 0.0;
  for (int k = 0; k < K; ++k) {
    const double a = c * std::sqrt(x[k]);
    z[2 * k] = cd(0.0, a);
    z[2 * k + 1] = cd(0.0, -a);
    zmax = std::max(zmax, a);
  }
  // exp(Z) e_0 by n_s Taylor steps of Z / n_s (||Z / n_s|| <= 1/2)
  const int ns = std::max(1, (int)std::ceil(2.0 * (zmax + 1.0)));
  d[0] = 1.0;
  for (int st = 0; st < ns; ++st) {
    term = d;
    acc = d;
    for (int p = 1; p <= 60; ++p) {
      const double f = 1.0 / ((double)ns * p);
      for (int k = n - 1; k >= 0; --k) nxt[k] = (z[k] * term[k] + (k ? term[k - 1] : cd(0.0))) * f;
      term.swap(nxt);
      for (int k = 0; k < n; ++k) acc[k] += term[k];
    }
    d = acc;
  }
  for (int k = 0; k < K; ++k) {
    alpha[k] = (d[2 * k] - d[2 * k + 1] * z[2 * k]).real();
    beta[k] = d[2 * k + 1].real();
    a2[k] = c * c * x[k];
  }
}

// N_k, k = 0..K: max over tau in [0, c^2] of prod_{j<k} |tau - a2_j| (x 1.001).
static void leja_basis_max(const double* a2, double c, int K, double* N) {
  const std::vector<double>& cand = leja_cand();
  std::vector<double> prod(cand.size(), 1.0);
  N[0] = 1.0;
  for (int k = 0; k < K; ++k) {
    double mx = 0.0;
    for (size_t i = 0; i < cand.size(); ++i) {
      prod[i] = prod[i] * std::fabs((c * c) * cand[i] - a2[k]);
      mx = std::max(mx, prod[i]);
    }
    N[k + 1] = mx * 1.001;
  }
}

static double leja_bound(double theta, int K, int64_t s, double u) {
  if (theta == 0.0) return 0.0;
  const double th = theta / (double)s;
  if (th > 700.0) return INFINITY;
  double al[kLejaKMax], be[kLejaKMax], a2[kLejaKMax], N[kLejaKMax + 1];
  leja_pairs(K, th, al, be, a2);
  leja_basis_max(a2, th, K, N);
  const double log_delta = N[K] > 0.0 ? std::log(N[K]) - std::lgamma(2.0 * K + 1.0) : -INFINITY;
  if (log_delta > 50.0) return INFINITY;
  const double delta = std::exp(log_delta);
  const double log_trunc = std::log((double)s) + log_delta + (double)(s - 1) * std::log1p(delta);
  double S = 0.0;
  for (int k = 0; k < K; ++k) S += (std::fabs(al[k]) + th * std::fabs(be[k])) * N[k];
  S = std::max(1.0, S);
  const double rnd = (double)s * (2 * K + 1) * u * S;
  if (log_trunc > 700.0) return INFINITY;
  return std::exp(log_trunc) + rnd;
}

static bool leja_search(double theta, double tol, double u, int* K_out, int64_t* s_out);

// Process-wide memo of the parameter search (it takes ~0.1 s per call and
// ParaExp asks for the same few (theta, tol, u) many times).
static bool leja_params(double theta, double tol, double u, int* K_out, int64_t* s_out) {
  struct Entry {
    double theta, tol, u;
    int K;
    int64_t s;
    bool ok;
  };
  static std::mutex mu;
  static std::vector<Entry> memo;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (const Entry& e : memo)
      if (e.theta == theta && e.tol == tol && e.u == u) {
        *K_out = e.K;
        *s_out = e.s;
        return e.ok;
      }
  }
  int K = 0;
  int64_t s = 1;
  const bool ok = leja_search(theta, tol, u, &K, &s);
  std::lock_guard<std::mutex> lk(mu);
  if (memo.size() >= 256) memo.erase(memo.begin());
  memo.push_back({theta, tol, u, K, s, ok});
  *K_out = K;
  *s_out = s;
  return ok;
}

static bool leja_search(double theta, double tol, double u, int* K_out, int64_t* s_out) {
  if (theta == 0.0) {
    *K_out = 0;
    *s_out = 1;
    return true;
  }
  int64_t best_cost = -1, best_s = 1;
  int best_K = 1;
  for (int K = 1; K <= kLejaKMax; ++K) {
    const int64_t s = first_feasible_s(theta, tol,
                                       [&](int64_t q) { return leja_bound(theta, K, q, u); });
    if (s < 0) continue;
    const int64_t cost = (int64_t)(2 * K - 1) * s;
    if (best_cost < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best_cost = cost;
      best_K = K;
      best_s = s;
    }
  }
  if (best_cost < 0) return false;
  *K_out = best_K;
  *s_out = best_s;
  return true;
}

// Scaled coefficients for the evaluation with the basis divided by g^(2k),
// g = max(c / 2, 1): alpha g^2k, beta g^2k, c^2 x_k / g^2 and g^2.
static void leja_scaled(int K, double c, double* alpha, double* beta, double* a2, double* g2) {
  leja_pairs(K, c, alpha, beta, a2);
  const double g = std::max(0.5 * c, 1.0);
  *g2 = g * g;
  double w = 1.0;
  for (int k = 0; k < K; ++k) {
    alpha[k] *= w;
    beta[k] *= w;
    a2[k] /= *g2;
    w *= *g2;
  }
}

// ---------------------------------------------------------------- helpers
static int ensure_xw(fit_grid* g) {
  if (g->xw) return FIT_OK;
  return dev_alloc(&g->xw, 6 * 3 * (size_t)g->d.n * g->esz, "operator workspace");
}

template <typename T>
static T* xw_vec(fit_grid* g, int v) {   // v = 0..5: (e, h) of three vectors
  return static_cast<T*>(g->xw) + (size_t)v * 3 * g->d.n;
}

static void op_coeffs(const fit_grid* g, double c, double ce[3], double ch[3]) {
  for (int a = 0; a < 3; ++a) {
    ce[a] = c / (g->gedge[a] / 4.0);
    ch[a] = -c * g->gf2[a] * 2.0 * g->imu_u;
  }
}

template <typename T>
static int apply_t(fit_grid* g, double c, const T* ein, const T* hin, T* eout, T* hout, T* eacc,
                   T* hacc, int mode) {
  double ce[3], ch[3];
  op_coeffs(g, c, ce, ch);
  hipError_t e;
  {
    ProfScope ps(g, FIT_PROF_OTHER);
    e = launch_opb<T>(ein, hin, eout, hout, eacc, hacc, mode, static_cast<const T*>(g->eps), g->d,
                      make_tiling(g->d, g->ty, g->kc), ce, ch, g->s);
  }
  if (e != hipSuccess) return hip_fail(e, "operator launch");
  g->smvp += 2;
  return FIT_OK;
}

// <a, b>_M of two (e, h) vectors: out[0] = e part, out[1] = h part (host).
template <typename T>
static int mdot_t(fit_grid* g, const T* ae, const T* ah, const T* be, const T* bh, double out[2]) {
  const int64_t nblk = std::min<int64_t>((g->d.n + 255) / 256, 2048);
  if (int rc = ensure_part(g, nblk)) return rc;
  double ge[3], mm[3];
  for (int a = 0; a < 3; ++a) {
    ge[a] = g->gedge[a] / 4.0;
    mm[a] = 1.0 / (g->gf2[a] * 2.0 * g->imu_u);
  }
  hipError_t e = launch_mdot<T>(ae, ah, be, bh, static_cast<const T*>(g->eps), g->d, ge, mm,
                                g->part, nblk, g->s);
  const int cols[kPartTerms] = {0, 1, -1, -1, -1, -1, -1, -1, -1, -1};
  if (e == hipSuccess)
    e = launch_reduce(g->part, nblk, g->jacc + 2, cols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, g->jacc + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, g->s);
  if (e == hipSuccess) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "M inner product");
  return FIT_OK;
}

static int need_op(const fit_grid* g) {
  if (g->nu) return fail(FIT_E_INVALID, "the operator needs a uniform spacing");
  if (!g->mu_uniform) return fail(FIT_E_INVALID, "the operator needs a uniform mu");
  if (g->lossy) return fail(FIT_E_INVALID, "the exponential needs a lossless grid (sigma = 0)");
  return FIT_OK;
}

template <typename T>
static int norm_t(fit_grid* g, int iters, uint64_t seed, double* rho) {
  if (int rc = ensure_xw(g)) return rc;
  T* xe = xw_vec<T>(g, 0);
  T* xh = xw_vec<T>(g, 1);
  T* ye = xw_vec<T>(g, 2);
  T* yh = xw_vec<T>(g, 3);
  hipError_t e = launch_seed<T>(xe, xh, g->d, seed, g->s);
  if (e != hipSuccess) return hip_fail(e, "power iteration start");
  double q = 0.0;
  for (int it = 0; it < iters; ++it) {
    // y = B x;  q = <y, y>_M / <x, x>_M  -> ||A||_2^2 (B is M-skew);  x <- -B y / q
    if (int rc = apply_t<T>(g, 1.0, xe, xh, ye, yh, nullptr, nullptr, 0)) return rc;
    double nx[2], ny[2];
    if (int rc = mdot_t<T>(g, xe, xh, xe, xh, nx)) return rc;
    if (int rc = mdot_t<T>(g, ye, yh, ye, yh, ny)) return rc;
    const double den = nx[0] + nx[1];
    if (!(den > 0.0)) return fail(FIT_E_DIVERGED, "power iteration vector vanished");
    q = (ny[0] + ny[1]) / den;
    if (!(q > 0.0) || !std::isfinite(q)) {
      if (q == 0.0) break;
      return fail(FIT_E_DIVERGED, "power iteration diverged");
    }
    if (it + 1 < iters)
      if (int rc = apply_t<T>(g, -1.0 / q, ye, yh, xe, xh, nullptr, nullptr, 0)) return rc;
  }
  *rho = std::sqrt(q);
  return FIT_OK;
}

template <typename T>
static int expm_t(fit_grid* g, double t, double tol, double rho, const T* ein, const T* hin,
                  T* eout, T* hout, int* m_out, int64_t* s_out) {
  int m;
  int64_t s;
  const double u = std::ldexp(1.0, sizeof(T) == 8 ? -53 : -24);
  if (!taylor_params(std::fabs(t) * rho, tol, u, &m, &s))
    return fail(FIT_E_INVALID, "tolerance below the rounding floor of the field dtype");
  if (m_out) *m_out = m;
  if (s_out) *s_out = s;
  const size_t bytes = 3 * (size_t)g->d.n * sizeof(T);
  if (m == 0) {
    hipError_t e = hipSuccess;
    if (eout != ein) e = hipMemcpyAsync(eout, ein, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e == hipSuccess && hout != hin) e = hipMemcpyAsync(hout, hin, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e != hipSuccess) return hip_fail(e, "exponential copy");
    return FIT_OK;
  }
  if (int rc = ensure_xw(g)) return rc;
  T* te[2] = {xw_vec<T>(g, 0), xw_vec<T>(g, 2)};
  T* th[2] = {xw_vec<T>(g, 1), xw_vec<T>(g, 3)};
  T* ae[2] = {eout, xw_vec<T>(g, 4)};
  T* ah[2] = {hout, xw_vec<T>(g, 5)};
  const double h = t / (double)s;
  const T* xe = ein;
  const T* xh = hin;
  int cur = (s % 2 == 1) ? 0 : 1;   // accumulator of the last sub-step lands in the output
  if (ein == eout || hin == hout) cur = 1;   // never accumulate over the input of sub-step 0
  for (int64_t sub = 0; sub < s; ++sub) {
    T* acc_e = ae[cur];
    T* acc_h = ah[cur];
    // term_1 = h B x, acc = x + term_1; term_k = (h / k) B term_(k-1), acc += term_k
    if (int rc = apply_t<T>(g, h, xe, xh, te[0], th[0], acc_e, acc_h, 2)) return rc;
    for (int k = 2; k <= m; ++k) {
      // term_k lives in buffer (k - 1) & 1: k = 2 reads buffer 0, writes buffer 1
      const int src = (k - 2) & 1, dst = (k - 1) & 1;
      if (int rc = apply_t<T>(g, h / k, te[src], th[src], te[dst], th[dst], acc_e, acc_h, 1))
        return rc;
    }
    xe = acc_e;
    xh = acc_h;
    cur ^= 1;
  }
  if (xe != eout) {
    hipError_t e = hipMemcpyAsync(eout, xe, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e == hipSuccess) e = hipMemcpyAsync(hout, xh, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e != hipSuccess) return hip_fail(e, "exponential copy");
  }
  return FIT_OK;
}

// Five (e, h) vectors for the Leja recurrence.
static int ensure_lw(fit_grid* g) {
  if (g->lw) return FIT_OK;
  return dev_alloc(&g->lw, 10 * 3 * (size_t)g->d.n * g->esz, "Leja workspace");
}

template <typename T>
static T* lw_vec(fit_grid* g, int v, int part) {   // v = 0..4, part 0: e, 1: h
  return static_cast<T*>(g->lw) + (size_t)(2 * v + part) * 3 * g->d.n;
}

// exp(tB) x by s steps of the K-pair Leja interpolant of exp(hB), h = t / s:
// per step q_0 = x, r_k = |h| B q_k, q_(k+1) = (|h| / g^2) B r_k + a2'_k q_k,
// x <- sum_k alpha'_k q_k + sign(h) beta'_k r_k (scaled coefficients).  The
// last pair updates the sum without forming q_K (2K - 1 applications).
template <typename T>
static int expm_leja_t(fit_grid* g, double t, double tol, double rho, const T* ein, const T* hin,
                       T* eout, T* hout, int* K_out, int64_t* s_out) {
  int K;
  int64_t s;
  const double u = std::ldexp(1.0, sizeof(T) == 8 ? -53 : -24);
  const double theta = std::fabs(t) * rho;
  if (!leja_params(theta, tol, u, &K, &s))
    return fail(FIT_E_INVALID, "tolerance below the rounding floor of the field dtype");
  if (K_out) *K_out = K;
  if (s_out) *s_out = s;
  const size_t bytes = 3 * (size_t)g->d.n * sizeof(T);
  const int64_t n3 = 3 * g->d.n;
  if (K == 0) {
    hipError_t e = hipSuccess;
    if (eout != ein) e = hipMemcpyAsync(eout, ein, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e == hipSuccess && hout != hin) e = hipMemcpyAsync(hout, hin, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e != hipSuccess) return hip_fail(e, "exponential copy");
    return FIT_OK;
  }
  if (int rc = ensure_lw(g)) return rc;
  const double h = t / (double)s, ha = std::fabs(h), sg = h < 0.0 ? -1.0 : 1.0;
  double al[kLejaKMax], be[kLejaKMax], a2[kLejaKMax], g2;
  leja_scaled(K, ha * rho, al, be, a2, &g2);
  double ce1[3], ch1[3], ce2[3], ch2[3];
  op_coeffs(g, ha, ce1, ch1);
  op_coeffs(g, ha / g2, ce2, ch2);
  const Tiling tl = make_tiling(g->d, g->ty, g->kc);
  const T* eps = static_cast<const T*>(g->eps);
  T* Re = lw_vec<T>(g, 0, 0);
  T* Rh = lw_vec<T>(g, 0, 1);
  T* Qe[2] = {lw_vec<T>(g, 1, 0), lw_vec<T>(g, 2, 0)};
  T* Qh[2] = {lw_vec<T>(g, 1, 1), lw_vec<T>(g, 2, 1)};
  T* Ae[2] = {lw_vec<T>(g, 3, 0), lw_vec<T>(g, 4, 0)};
  T* Ah[2] = {lw_vec<T>(g, 3, 1), lw_vec<T>(g, 4, 1)};
  const bool out_free = eout != ein && hout != hin && eout != hin && hout != ein;
  const T* xe = ein;
  const T* xh = hin;
  hipError_t err = hipSuccess;
  for (int64_t sub = 0; sub < s && err == hipSuccess; ++sub) {
    T* acce = (sub == s - 1 && out_free) ? eout : Ae[sub & 1];
    T* acch = (sub == s - 1 && out_free) ? hout : Ah[sub & 1];
    const T* qe = xe;
    const T* qh = xh;
    int qn = 0;
    for (int k = 0; k < K && err == hipSuccess; ++k) {
      {
        ProfScope ps(g, FIT_PROF_OTHER);
        err = launch_opb<T>(qe, qh, Re, Rh, nullptr, nullptr, 0, eps, g->d, tl, ce1, ch1, g->s);
      }
      g->smvp += 2;
      if (err != hipSuccess) break;
      if (k + 1 < K || K == 1) {
        // q_(k+1) = (|h| / g^2) B r_k + a2'_k q_k, acc (+)= alpha'_k q_k + beta'_k r_k
        ProfScope ps(g, FIT_PROF_OTHER);
        err = launch_opb<T>(Re, Rh, Qe[qn], Qh[qn], acce, acch, k == 0 ? 4 : 3, eps, g->d, tl,
                            ce2, ch2, g->s, qe, qh, a2[k], al[k], sg * be[k]);
        g->smvp += 2;
        qe = Qe[qn];
        qh = Qh[qn];
        qn ^= 1;
      } else {
        // last pair: acc += alpha'_K-1 q + beta'_K-1 r
        err = launch_axpy<T>((T)al[k], qe, qh, acce, acch, n3, g->s);
        if (err == hipSuccess) err = launch_axpy<T>((T)(sg * be[k]), Re, Rh, acce, acch, n3, g->s);
      }
    }
    xe = acce;
    xh = acch;
  }
  if (err != hipSuccess) return hip_fail(err, "Leja launch");
  if (xe != eout) {
    hipError_t e = hipMemcpyAsync(eout, xe, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e == hipSuccess) e = hipMemcpyAsync(hout, xh, bytes, hipMemcpyDeviceToDevice, g->s);
    if (e != hipSuccess) return hip_fail(e, "exponential copy");
  }
  return FIT_OK;
}

template <typename T>
static int shift_h_t(fit_grid* g, double c, const T* e, const T* hin, T* hout) {
  const Dims& d = g->d;
  HArgs<T> a;
  for (int k = 0; k < 3; ++k) {
    a.e[k] = e + k * d.n;
    a.hin[k] = hin + k * d.n;
    a.hout[k] = hout + k * d.n;
    a.kd[k] = (T)(c * g->gf2[k]);
    a.gf2[k] = g->gf2[k];
  }
  a.imu = g->mu_uniform ? nullptr : static_cast<const T*>(g->imu);
  a.imu_u = (T)g->imu_u;
  a.d = d;
  a.t = make_tiling(d, g->ty, g->kc);
  a.part = nullptr;
  set_metric(g, a.sq);
  a.kds = c;
  hipError_t err;
  {
    ProfScope ps(g, FIT_PROF_HPASS);
    err = launch_hpass<T>(a, g->mu_uniform, false, g->s);
  }
  if (err != hipSuccess) return hip_fail(err, "h shift launch");
  g->smvp += 1;
  return FIT_OK;
}

}  // namespace fit

using namespace fit;

extern "C" {

int fit_expm_params(double theta, double tol, double unit_roundoff, int* m, int64_t* s) {
  if (!m || !s) return fail(FIT_E_INVALID, "null argument");
  if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(FIT_E_INVALID, "theta must be >= 0");
  if (!(tol > 0.0) || tol >= 1.0) return fail(FIT_E_INVALID, "tol must be in (0, 1)");
  if (!(unit_roundoff > 0.0) || unit_roundoff >= 1.0)
    return fail(FIT_E_INVALID, "unit_roundoff must be in (0, 1)");
  if (!taylor_params(theta, tol, unit_roundoff, m, s))
    return fail(FIT_E_INVALID, "tolerance below the rounding floor");
  return FIT_OK;
}

int fit_expm_tolerance(double beta, double dt, double rho, double* tol) {
  if (!tol) return fail(FIT_E_INVALID, "null argument");
  if (!(beta > 0.0) || !std::isfinite(beta) || !(dt > 0.0) || !std::isfinite(dt) ||
      !(rho > 0.0) || !std::isfinite(rho))
    return fail(FIT_E_INVALID, "beta, dt and rho must be positive and finite");
  *tol = beta * dt * dt / rho;
  return FIT_OK;
}

int fit_op_apply(fit_grid* g, double alpha, const void* e_in, const void* h_in, void* e_out,
                 void* h_out) {
  if (!g || !e_in || !h_in || !e_out || !h_out) return fail(FIT_E_INVALID, "null argument");
  if (g->nu) return fail(FIT_E_INVALID, "the operator needs a uniform spacing");
  if (!g->mu_uniform) return fail(FIT_E_INVALID, "the operator needs a uniform mu");
  if (e_in == e_out || h_in == h_out || e_in == h_out || h_in == e_out)
    return fail(FIT_E_INVALID, "input and output must be distinct buffers");
  return g->f64 ? apply_t<double>(g, alpha, static_cast<const double*>(e_in),
                                  static_cast<const double*>(h_in), static_cast<double*>(e_out),
                                  static_cast<double*>(h_out), nullptr, nullptr, 0)
                : apply_t<float>(g, alpha, static_cast<const float*>(e_in),
                                 static_cast<const float*>(h_in), static_cast<float*>(e_out),
                                 static_cast<float*>(h_out), nullptr, nullptr, 0);
}

int fit_op_norm(fit_grid* g, int iters, uint64_t seed, double* rho) {
  if (!g || !rho) return fail(FIT_E_INVALID, "null argument");
  if (iters < 1 || iters > 100000) return fail(FIT_E_INVALID, "iters must be in [1, 100000]");
  if (int rc = need_op(g)) return rc;
  return g->f64 ? norm_t<double>(g, iters, seed, rho) : norm_t<float>(g, iters, seed, rho);
}

int fit_expm(fit_grid* g, double t, double tol, double rho, const void* e_in, const void* h_in,
             void* e_out, void* h_out, int* m, int64_t* s) {
  if (!g || !e_in || !h_in || !e_out || !h_out) return fail(FIT_E_INVALID, "null argument");
  if (!std::isfinite(t)) return fail(FIT_E_INVALID, "t must be finite");
  if (!(tol > 0.0) || tol >= 1.0) return fail(FIT_E_INVALID, "tol must be in (0, 1)");
  if (!(rho >= 0.0) || !std::isfinite(rho)) return fail(FIT_E_INVALID, "rho must be >= 0");
  if (int rc = need_op(g)) return rc;
  return g->f64 ? expm_t<double>(g, t, tol, rho, static_cast<const double*>(e_in),
                                 static_cast<const double*>(h_in), static_cast<double*>(e_out),
                                 static_cast<double*>(h_out), m, s)
                : expm_t<float>(g, t, tol, rho, static_cast<const float*>(e_in),
                                static_cast<const float*>(h_in), static_cast<float*>(e_out),
                                static_cast<float*>(h_out), m, s);
}

int fit_leja_params(double theta, double tol, double unit_roundoff, int* K, int64_t* s) {
  if (!K || !s) return fail(FIT_E_INVALID, "null argument");
  if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(FIT_E_INVALID, "theta must be >= 0");
  if (!(tol > 0.0) || tol >= 1.0) return fail(FIT_E_INVALID, "tol must be in (0, 1)");
  if (!(unit_roundoff > 0.0) || unit_roundoff >= 1.0)
    return fail(FIT_E_INVALID, "unit_roundoff must be in (0, 1)");
  if (!leja_params(theta, tol, unit_roundoff, K, s))
    return fail(FIT_E_INVALID, "tolerance below the rounding floor");
  return FIT_OK;
}

int fit_leja_coefficients(int K, double c, double* alpha, double* beta, double* a2, double* g2) {
  if (!alpha || !beta || !a2 || !g2) return fail(FIT_E_INVALID, "null argument");
  if (K < 1 || K > kLejaKMax) return fail(FIT_E_INVALID, "K must be in [1, 30]");
  if (!(c >= 0.0) || !std::isfinite(c)) return fail(FIT_E_INVALID, "c must be >= 0");
  leja_scaled(K, c, alpha, beta, a2, g2);
  return FIT_OK;
}

int fit_expm_leja(fit_grid* g, double t, double tol, double rho, const void* e_in,
                  const void* h_in, void* e_out, void* h_out, int* K, int64_t* s) {
  if (!g || !e_in || !h_in || !e_out || !h_out) return fail(FIT_E_INVALID, "null argument");
  if (!std::isfinite(t)) return fail(FIT_E_INVALID, "t must be finite");
  if (!(tol > 0.0) || tol >= 1.0) return fail(FIT_E_INVALID, "tol must be in (0, 1)");
  if (!(rho >= 0.0) || !std::isfinite(rho)) return fail(FIT_E_INVALID, "rho must be >= 0");
  if (int rc = need_op(g)) return rc;
  return g->f64 ? expm_leja_t<double>(g, t, tol, rho, static_cast<const double*>(e_in),
                                      static_cast<const double*>(h_in), static_cast<double*>(e_out),
                                      static_cast<double*>(h_out), K, s)
                : expm_leja_t<float>(g, t, tol, rho, static_cast<const float*>(e_in),
                                     static_cast<const float*>(h_in), static_cast<float*>(e_out),
                                     static_cast<float*>(h_out), K, s);
}

int fit_shift_h(fit_grid* g, double c, const void* e, const void* h_in, void* h_out) {
  if (!g || !e || !h_in || !h_out) return fail(FIT_E_INVALID, "null argument");
  if (!std::isfinite(c)) return fail(FIT_E_INVALID, "c must be finite");
  return g->f64 ? shift_h_t<double>(g, c, static_cast<const double*>(e),
                                    static_cast<const double*>(h_in), static_cast<double*>(h_out))
                : shift_h_t<float>(g, c, static_cast<const float*>(e),
                                   static_cast<const float*>(h_in), static_cast<float*>(h_out));
}

int fit_axpy(fit_grid* g, double a, const void* x_e, const void* x_h, void* y_e, void* y_h) {
  if (!g || !x_e || !x_h || !y_e || !y_h) return fail(FIT_E_INVALID, "null argument");
  const int64_t n3 = 3 * g->d.n;
  hipError_t e = g->f64 ? launch_axpy<double>(a, static_cast<const double*>(x_e),
                                              static_cast<const double*>(x_h),
                                              static_cast<double*>(y_e), static_cast<double*>(y_h),
                                              n3, g->s)
                        : launch_axpy<float>((float)a, static_cast<const float*>(x_e),
                                             static_cast<const float*>(x_h),
                                             static_cast<float*>(y_e), static_cast<float*>(y_h), n3,
                                             g->s);
  if (e != hipSuccess) return hip_fail(e, "axpy launch");
  return FIT_OK;
}

}  // extern "C"
