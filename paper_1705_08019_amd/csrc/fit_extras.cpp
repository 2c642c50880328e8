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
  if (!w->borrowed) {
    for (int q = 0; q < 2; ++q) {
      dev_free(w->lam[q]);
      dev_free(w->mu[q]);
    }
    dev_free(reinterpret_cast<void*&>(w->gcell));
  }
  delete w;
  g->adj = nullptr;
}

// Tile of the reverse-step kernel: the width (32, 64 or 128) that wastes the
// fewest lanes on the x extent (ties: the wider), as many rows as fit 512
// threads (FP32; 256 for FP64) together with the tw + ty + 1 halo threads,
// and z-chunks sized so that one round of resident workgroups covers the grid.
static Tiling adjoint_tiling(const fit_grid* g) {
  const Dims& d = g->d;
  const int nt = g->f64 ? 256 : 512;
  int tw = 32, best = 1 << 30;
  for (int w : {128, 64, 32}) {
    if ((nt - w - 1) / (w + 1) < 2) continue;
    const int waste = ((d.nx + w - 1) / w) * w - d.nx;
    if (waste < best) {
      best = waste;
      tw = w;
    }
  }
  int ty = (nt - tw - 1) / (tw + 1);
  ty = std::max(1, std::min(ty, d.ny));
  if (g->atw > 0) {
    tw = g->atw;
    ty = g->aty;
  }
  if (g->akc > 0) return make_tiling(d, ty, std::min(g->akc, d.nz), tw);
  int per_cu = adjoint_blocks_per_cu(tw, ty, g->esz, g->lossy);
  if (per_cu < 1) per_cu = 1;
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  (void)hipGetLastError();
  const int64_t tiles = (int64_t)((d.nx + tw - 1) / tw) * ((d.ny + ty - 1) / ty);
  const int64_t nkc = std::max<int64_t>(1, (int64_t)cus * per_cu / tiles);
  int kc = (int)((d.nz + nkc - 1) / nkc);
  // at least 4 planes per chunk (the march re-reads one plane below it)
  kc = std::min(d.nz, std::max(kc, std::min(4, d.nz)));
  return make_tiling(d, ty, kc, tw);
}

template <typename T>
static int adjoint_step_t(fit_grid* g, int64_t m, const void* e_m, const void* e_m1,
                          const void* h_mh) {
  fit_adjoint_ws* w = g->adj;
  const Dims& d = g->d;
  AdjArgs<T> a;
  const T* h = static_cast<const T*>(h_mh);
  const T* em = static_cast<const T*>(e_m);
  const T* em1 = static_cast<const T*>(e_m1);
  const T* l0 = static_cast<const T*>(w->lam[w->cur]);
  const T* u0 = static_cast<const T*>(w->mu[w->cur]);
  T* l1 = static_cast<T*>(w->lam[w->cur ^ 1]);
  T* u1 = static_cast<T*>(w->mu[w->cur ^ 1]);
  a.h = h;
  a.em = em;
  a.em1 = em1;
  a.lam0 = l0;
  a.mu0 = u0;
  a.lam1 = l1;
  a.mu1 = u1;
  for (int c = 0; c < 3; ++c) {
    a.kb[c] = (T)(4.0 * w->dt / g->gedge[c]);
    a.dmu[c] = (T)(w->dt * g->gf2[c]) * ((T)g->imu_u + (T)g->imu_u);
    a.ge[c] = g->gedge[c] / 4.0;
  }
  a.eps0 = g->desc.eps0;
  a.eps = static_cast<const T*>(g->eps);
  a.sig = static_cast<const T*>(g->sig);
  a.geps = w->gcell;
  a.gsig = w->gcell + d.n;
  a.d = d;
  a.t = w->t;
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
  w->cur ^= 1;
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
  dt = step_dt(g, dt);
  if (nsteps > 0) g->last_dt = dt;
  return g->f64 ? record_t<double>(g, nsteps, dt, e_rec, h_rec)
                : record_t<float>(g, nsteps, dt, e_rec, h_rec);
}

int fit_adjoint_get_tuning(const fit_grid* g, int* tw, int* ty, int* kc) {
  if (!g || !tw || !ty || !kc) return fail(FIT_E_INVALID, "null argument");
  const Tiling t = adjoint_tiling(g);
  *tw = t.tw;
  *ty = t.ty;
  *kc = t.kc;
  return FIT_OK;
}

int fit_adjoint_set_tuning(fit_grid* g, int tw, int ty, int kc) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if ((tw == 0) != (ty == 0)) return fail(FIT_E_INVALID, "give both tw and ty, or neither");
  if (tw < 0 || ty < 0 || kc < 0) return fail(FIT_E_INVALID, "negative tile size");
  if (tw > 0) {
    if (tw > 256) return fail(FIT_E_INVALID, "tw must be <= 256");
    const int nt = adjoint_threads(tw, ty);
    if (nt > 512 || (int64_t)(tw + 2) * (ty + 2) > kAdjRing * (int64_t)nt ||
        adjoint_lds_bytes(tw, ty, g->esz) > 160 * 1024)
      return fail(FIT_E_INVALID, "adjoint tile does not fit a workgroup (tw ty + tw + ty + 1 <= 512)");
  }
  g->atw = tw;
  g->aty = ty;
  g->akc = kc;
  return FIT_OK;
}

int fit_adjoint_bind(fit_grid* g, void* lam0, void* lam1, void* mu0, void* mu1, double* gcell) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  void* p[5] = {lam0, lam1, mu0, mu1, gcell};
  int nn = 0;
  for (void* q : p) nn += q == nullptr;
  if (nn != 0 && nn != 5) return fail(FIT_E_INVALID, "give all five adjoint buffers or none");
  const size_t fb = 3 * (size_t)g->d.n * g->esz;
  const size_t gb = 2 * (size_t)g->d.n * sizeof(double);
  if (nn == 0) {
    const void* f[7] = {g->e, g->h, g->e_alt, g->h_alt, g->eps, g->sig, g->imu};
    for (int a = 0; a < 5; ++a) {
      if (reinterpret_cast<uintptr_t>(p[a]) % 16 != 0)
        return fail(FIT_E_INVALID, "bound buffers must be aligned to 16 bytes");
      for (const void* o : f)
        if (o && o == p[a]) return fail(FIT_E_INVALID, "an adjoint buffer is a field or cell buffer");
      const char* x = static_cast<const char*>(p[a]);
      const size_t xa = a == 4 ? gb : fb;
      for (int b = 0; b < a; ++b) {
        const char* y = static_cast<const char*>(p[b]);
        if (x < y + fb && y < x + xa) return fail(FIT_E_INVALID, "adjoint buffers must not overlap");
      }
    }
  }
  hipError_t e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "bind sync");
  grid_release_extras(g);   // any sweep in progress ends here
  if (nn == 5) return FIT_OK;   // allocated by the library at the next fit_adjoint_begin
  g->adj = new (std::nothrow) fit_adjoint_ws();
  if (!g->adj) return fail(FIT_E_OOM, "host allocation failed");
  fit_adjoint_ws* w = g->adj;
  w->lam[0] = lam0;
  w->lam[1] = lam1;
  w->mu[0] = mu0;
  w->mu[1] = mu1;
  w->gcell = gcell;
  w->borrowed = true;
  return FIT_OK;
}

int fit_adjoint_begin(fit_grid* g, int64_t nsteps, double dt) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (nsteps < 1) return fail(FIT_E_INVALID, "nsteps must be >= 1");
  if (!g->probe.on) return fail(FIT_E_STATE, "the adjoint needs a probe (fit_set_probe)");
  if (g->nu) return fail(FIT_E_INVALID, "the adjoint needs a uniform spacing");
  if (!g->mu_uniform) return fail(FIT_E_INVALID, "the adjoint needs a uniform mu");
  if (int rc = check_dt(g, dt)) return rc;
  dt = step_dt(g, dt);
  if (!g->adj) {
    g->adj = new (std::nothrow) fit_adjoint_ws();
    if (!g->adj) return fail(FIT_E_OOM, "host allocation failed");
    fit_adjoint_ws* w = g->adj;
    const size_t fb = 3 * (size_t)g->d.n * g->esz;
    int rc = FIT_OK;
    for (int q = 0; q < 2 && !rc; ++q) {
      rc = dev_alloc(&w->lam[q], fb, "adjoint lambda");
      if (!rc) rc = dev_alloc(&w->mu[q], fb, "adjoint mu");
    }
    if (!rc)
      rc = dev_alloc(reinterpret_cast<void**>(&w->gcell), 2 * (size_t)g->d.n * sizeof(double),
                     "cell gradients");
    if (rc) {
      grid_release_extras(g);
      return rc;
    }
  }
  fit_adjoint_ws* w = g->adj;
  w->t = adjoint_tiling(g);
  if ((uint64_t)g->d.sxy * sizeof(double) > (uint64_t)UINT32_MAX)
    return fail(FIT_E_INVALID, "a z-plane of the grid spans more than 4 GiB of FP64 values "
                               "(the reverse-step kernel addresses a plane with 32-bit offsets)");
  {
    const int nt = adjoint_threads(w->t.tw, w->t.ty);
    if ((int64_t)(w->t.tw + 2) * (w->t.ty + 2) > kAdjRing * (int64_t)nt || nt > 512 ||
        adjoint_lds_bytes(w->t.tw, w->t.ty, g->esz) > 160 * 1024)
      return fail(FIT_E_INVALID, "adjoint tile does not fit a workgroup");
  }
  const size_t fb = 3 * (size_t)g->d.n * g->esz;
  w->cur = 0;
  hipError_t e = hipMemsetAsync(w->lam[0], 0, fb, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(w->mu[0], 0, fb, g->s);
  if (e == hipSuccess)
    e = hipMemsetAsync(w->gcell, 0, 2 * (size_t)g->d.n * sizeof(double), g->s);
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
  const size_t b = (size_t)g->d.n * sizeof(double);
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipError_t e = hipMemcpyAsync(deps, w->gcell, b, k, g->s);
  if (e == hipSuccess) e = hipMemcpyAsync(dsigma, w->gcell + g->d.n, b, k, g->s);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "gradient copy");
  return FIT_OK;
}

}  // extern "C"
