// C ABI of the operator, matrix-exponential and ParaExp building blocks
// (Sec. III-A, Sec. III): apply B, estimate ||A||_2, exp(tB) by scaling and a
// truncated Taylor recurrence, the half-step h transform, axpy.
#include <algorithm>
#include <cmath>
#include <string>

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

// Smallest s meeting tol for this m, or -1.  On s <= theta both parts fall
// with s (bisection is exact there); beyond, s* (3/2)^q, q = 1..6, are tried
// and the first feasible one is bisected down to the previous sample.
static int64_t first_feasible(double theta, int m, double tol, double u) {
  const int64_t s_star = std::max<int64_t>(1, (int64_t)std::ceil(theta));
  int64_t lo = -1, hi = -1;
  if (taylor_bound(theta, m, s_star, u) <= tol) {
    lo = 1;
    hi = s_star;
  } else {
    int64_t prev = s_star;
    for (int q = 1; q <= 6; ++q) {
      const int64_t cand = (int64_t)std::ceil((double)s_star * std::pow(1.5, q));
      if (taylor_bound(theta, m, cand, u) <= tol) {
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
    if (taylor_bound(theta, m, mid, u) <= tol) hi = mid;
    else lo = mid + 1;
  }
  return lo;
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
