// Adjoint (reverse-time leapfrog) and recording entry points of the C ABI,
// and release of the optional per-handle workspaces.
#include <algorithm>
#include <cmath>
#include <string>

#include "fit_host.hpp"

namespace fit {

void grid_release_extras(fit_grid* g) {
  if (!g->adj) return;
  fit_adjoint_ws* w = g->adj;
  dev_free(w->lam);
  dev_free(w->mu);
  dev_free(w->tau);
  dev_free(reinterpret_cast<void*&>(w->gMe));
  dev_free(reinterpret_cast<void*&>(w->gMs));
  dev_free(reinterpret_cast<void*&>(w->gcell));
  delete w;
  g->adj = nullptr;
}

template <typename T>
static int adjoint_step_t(fit_grid* g, int64_t m, const void* e_m, const void* e_m1,
                          const void* h_mh) {
  fit_adjoint_ws* w = g->adj;
  const Dims& d = g->d;
  AdjArgs<T> a;
  const T* h = static_cast<const T*>(h_mh);
  T* mu = static_cast<T*>(w->mu);
  for (int c = 0; c < 3; ++c) {
    a.h[c] = h + c * d.n;
    a.mu[c] = mu + c * d.n;
    a.kb[c] = (T)(4.0 * w->dt / g->gedge[c]);
    a.dmu[c] = (T)(w->dt * g->gf2[c]) * ((T)g->imu_u + (T)g->imu_u);
    a.ge[c] = g->gedge[c] / 4.0;
  }
  a.lam = static_cast<T*>(w->lam);
  a.tau = static_cast<T*>(w->tau);
  a.em = static_cast<const T*>(e_m);
  a.em1 = static_cast<const T*>(e_m1);
  a.eps = static_cast<const T*>(g->eps);
  a.sig = static_cast<const T*>(g->sig);
  a.gMe = w->gMe;
  a.gMs = w->gMs;
  a.d = d;
  a.t = make_tiling(d, g->ty, g->kc);
  a.hs = (T)(0.5 * w->dt);
  a.dt = w->dt;
  a.hdt = 0.5 * w->dt;
  a.src_comp = g->src_axis;
  a.src_idx = g->src_axis >= 0 ? g->src_idx : -1;
  a.src_val = (T)(g->src_axis >= 0 ? source_value(g, w->dt, m) : 0.0);
  a.probe = g->probe;
  hipError_t e;
  {
    ProfScope ps(g, FIT_PROF_ADJOINT);
    e = launch_adjoint_step<T>(a, g->lossy, g->s);
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint step launch");
  g->smvp += 2;
  return FIT_OK;
}

template <typename T>
static int record_t(fit_grid* g, int64_t nsteps, double dt, void* e_rec, void* h_rec) {
  const Dims& d = g->d;
  const size_t bytes = 3 * (size_t)d.n * sizeof(T);
  T* er = static_cast<T*>(e_rec);
  T* hr = static_cast<T*>(h_rec);
  hipError_t e = hipMemcpyAsync(er, g->e, bytes, hipMemcpyDeviceToDevice, g->s);
  if (e == hipSuccess) e = hipMemcpyAsync(hr, g->h, bytes, hipMemcpyDeviceToDevice, g->s);
  if (e != hipSuccess) return hip_fail(e, "record copy");
  // recording does not trace energies or accumulate the probe objective
  const int64_t save_every = g->trace_every;
  const Probe save_probe = g->probe;
  g->trace_every = 0;
  g->probe.on = 0;
  int rc = FIT_OK;
  const bool fused = use_fused(g);
  for (int64_t s = 0; s < nsteps && !rc; ++s) {
    const T* e0 = er + s * 3 * d.n;
    const T* h0 = hr + s * 3 * d.n;
    T* e1 = er + (s + 1) * 3 * d.n;
    T* h1 = hr + (s + 1) * 3 * d.n;
    rc = fused ? step_fused_io<T>(g, dt, e0, h0, e1, h1) : step_once<T>(g, dt, e0, e1, h0, h1);
  }
  g->trace_every = save_every;
  g->probe = save_probe;
  if (rc) return rc;
  e = hipMemcpyAsync(g->e, er + nsteps * 3 * d.n, bytes, hipMemcpyDeviceToDevice, g->s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->h, hr + nsteps * 3 * d.n, bytes, hipMemcpyDeviceToDevice, g->s);
  if (e != hipSuccess) return hip_fail(e, "record copy");
  return FIT_OK;
}

}  // namespace fit

using namespace fit;

extern "C" {

int fit_step_record(fit_grid* g, int64_t nsteps, double dt, void* e_rec, void* h_rec) {
  if (!g || !e_rec || !h_rec) return fail(FIT_E_INVALID, "null argument");
  if (nsteps < 0) return fail(FIT_E_INVALID, "nsteps must be >= 0");
  if (int rc = check_dt(g, dt)) return rc;
  return g->f64 ? record_t<double>(g, nsteps, dt, e_rec, h_rec)
                : record_t<float>(g, nsteps, dt, e_rec, h_rec);
}

int fit_adjoint_begin(fit_grid* g, int64_t nsteps, double dt) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (nsteps < 1) return fail(FIT_E_INVALID, "nsteps must be >= 1");
  if (!g->probe.on) return fail(FIT_E_STATE, "the adjoint needs a probe (fit_set_probe)");
  if (!g->mu_uniform) return fail(FIT_E_INVALID, "the adjoint needs a uniform mu");
  if (int rc = check_dt(g, dt)) return rc;
  if (!g->adj) {
    g->adj = new (std::nothrow) fit_adjoint_ws();
    if (!g->adj) return fail(FIT_E_OOM, "host allocation failed");
    fit_adjoint_ws* w = g->adj;
    const size_t fb = 3 * (size_t)g->d.n * g->esz, db = 3 * (size_t)g->d.n * sizeof(double);
    int rc = dev_alloc(&w->lam, fb, "adjoint lambda");
    if (!rc) rc = dev_alloc(&w->mu, fb, "adjoint mu");
    if (!rc) rc = dev_alloc(&w->tau, fb, "adjoint tau");
    if (!rc) rc = dev_alloc(reinterpret_cast<void**>(&w->gMe), db, "dJ/dM_eps");
    if (!rc) rc = dev_alloc(reinterpret_cast<void**>(&w->gMs), db, "dJ/dM_sigma");
    if (!rc)
      rc = dev_alloc(reinterpret_cast<void**>(&w->gcell), 2 * (size_t)g->d.n * sizeof(double),
                     "cell gradients");
    if (rc) {
      grid_release_extras(g);
      return rc;
    }
  }
  fit_adjoint_ws* w = g->adj;
  const size_t fb = 3 * (size_t)g->d.n * g->esz, db = 3 * (size_t)g->d.n * sizeof(double);
  hipError_t e = hipMemsetAsync(w->lam, 0, fb, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(w->mu, 0, fb, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(w->tau, 0, fb, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(w->gMe, 0, db, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(w->gMs, 0, db, g->s);
  if (e != hipSuccess) return hip_fail(e, "adjoint clear");
  w->N = nsteps;
  w->dt = dt;
  w->next_m = nsteps - 1;
  return FIT_OK;
}

int fit_adjoint_step(fit_grid* g, int64_t m, const void* e_m, const void* e_m1, const void* h_mh) {
  if (!g || !e_m || !e_m1 || !h_mh) return fail(FIT_E_INVALID, "null argument");
  if (!g->adj || g->adj->next_m < 0) return fail(FIT_E_STATE, "no adjoint sweep in progress");
  if (m != g->adj->next_m)
    return fail(FIT_E_STATE, "adjoint steps must run m = N-1 down to 0 (expected " +
                                 std::to_string(g->adj->next_m) + ")");
  int rc = g->f64 ? adjoint_step_t<double>(g, m, e_m, e_m1, h_mh)
                  : adjoint_step_t<float>(g, m, e_m, e_m1, h_mh);
  if (rc) return rc;
  g->adj->next_m = m - 1;
  return FIT_OK;
}

int fit_adjoint_segment(fit_grid* g, int64_t m0, int64_t nsteps, const void* e_rec,
                        const void* h_rec) {
  if (!g || !e_rec || !h_rec) return fail(FIT_E_INVALID, "null argument");
  if (nsteps < 1) return fail(FIT_E_INVALID, "nsteps must be >= 1");
  const size_t st = 3 * (size_t)g->d.n * g->esz;
  const char* er = static_cast<const char*>(e_rec);
  const char* hr = static_cast<const char*>(h_rec);
  for (int64_t s = nsteps - 1; s >= 0; --s) {
    int rc = fit_adjoint_step(g, m0 + s, er + s * st, er + (s + 1) * st, hr + s * st);
    if (rc) return rc;
  }
  return FIT_OK;
}

int fit_adjoint_grad(fit_grid* g, double* deps, double* dsigma, int on_device) {
  if (!g || !deps || !dsigma) return fail(FIT_E_INVALID, "null argument");
  if (!g->adj) return fail(FIT_E_STATE, "no adjoint sweep");
  fit_adjoint_ws* w = g->adj;
  double gq[3];
  for (int a = 0; a < 3; ++a) gq[a] = g->gedge[a] / 4.0;
  hipError_t e = launch_adjoint_gather(w->gMe, w->gMs, g->d, gq, g->desc.eps0, w->gcell,
                                       w->gcell + g->d.n, g->s);
  if (e != hipSuccess) return hip_fail(e, "gradient gather");
  const size_t b = (size_t)g->d.n * sizeof(double);
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  e = hipMemcpyAsync(deps, w->gcell, b, k, g->s);
  if (e == hipSuccess) e = hipMemcpyAsync(dsigma, w->gcell + g->d.n, b, k, g->s);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "gradient copy");
  return FIT_OK;
}

}  // extern "C"
