// C-ABI host code of libfit: handle management, material upload, the
// leapfrog time loop (two kernel launches per step, eq. cost_LF), energy
// trace bookkeeping and the probe objective.  All arithmetic of the method
// runs in the HIP kernels; this file only validates, allocates, launches.
#include "fit.h"
#include "fit_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace fit {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FIT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return FIT_OK;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(FIT_E_OOM, std::string("hipMalloc failed for ") + what + " (" +
                               std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
  }
  return FIT_OK;
}

void dev_free(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Probe accumulator rows for `rows` workgroups; on growth the rows so far
// are first folded into the probe total.
int ensure_pacc(fit_grid* g, int64_t rows) {
  if (rows <= g->pacc_rows) return FIT_OK;
  if (g->pacc) {
    hipError_t e = launch_pacc_flush(g->pacc, g->pacc_rows, g->jacc, g->s);
    if (e == hipSuccess) e = hipStreamSynchronize(g->s);
    if (e != hipSuccess) return hip_fail(e, "probe rows flush");
    dev_free(reinterpret_cast<void*&>(g->pacc));
  }
  g->pacc_rows = 0;
  int rc = dev_alloc(reinterpret_cast<void**>(&g->pacc), (size_t)rows * 2 * sizeof(double),
                     "probe rows");
  if (rc) return rc;
  hipError_t e = hipMemsetAsync(g->pacc, 0, (size_t)rows * 2 * sizeof(double), g->s);
  if (e != hipSuccess) return hip_fail(e, "probe rows clear");
  g->pacc_rows = rows;
  return FIT_OK;
}

int ensure_part(fit_grid* g, int64_t rows) {
  if (rows <= g->part_rows) return FIT_OK;
  if (g->part) {
    (void)hipStreamSynchronize(g->s);
    dev_free(reinterpret_cast<void*&>(g->part));
  }
  int rc = dev_alloc(reinterpret_cast<void**>(&g->part), (size_t)rows * kPartTerms * sizeof(double),
                     "partial sums");
  if (rc) {
    g->part_rows = 0;
    return rc;
  }
  g->part_rows = rows;
  return FIT_OK;
}

void default_tiling(const Dims& d, int* ty, int* kc) {
  const int ntx = (d.nx + 63) / 64;
  const int t = 4;
  const int nty = (d.ny + t - 1) / t;
  const int64_t target = 2048;
  int64_t nkc = (target + (int64_t)ntx * nty - 1) / ((int64_t)ntx * nty);
  int k = (int)((d.nz + nkc - 1) / nkc);
  k = std::max(k, 8);
  *ty = t;
  *kc = std::min(k, d.nz);
}

// Fused-kernel tiling: pick the z-chunk so that one round of resident
// workgroups (LDS- and wave-limited) covers the grid once.
void default_step_tiling(const Dims& d, size_t esz, bool lossy, int* ty, int* kc, int* tw) {
  // 1024 threads (FP32) or 256 (FP64, LDS) in a tile whose width (128, 64
  // or 32) wastes the fewest lanes on the x extent (ties: the wider); the
  // autotuner refines this
  const int nthr = esz == 8 ? 256 : 1024;
  int w = 64, best = 1 << 30;
  for (int c : {128, 64, 32}) {
    if (nthr / c < 2) continue;
    const int waste = ((d.nx + c - 1) / c) * c - d.nx;
    if (waste < best) {
      best = waste;
      w = c;
    }
  }
  const int t = std::min(16, nthr / w);
  int per_cu = step_blocks_per_cu(t, esz, lossy, w);
  if (per_cu <= 0) {   // no device information: estimate from LDS and waves
    const size_t lds = step_lds_bytes(t, esz, lossy, w) + 2048;
    per_cu = (int)std::min<size_t>((160 * 1024) / lds, 2048 / (w * t));
  }
  per_cu = std::max(per_cu, 1);
  int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  (void)hipGetLastError();
  const int64_t resident = (int64_t)cus * per_cu;
  const int64_t tiles = (int64_t)((d.nx + w - 1) / w) * ((d.ny + t - 1) / t);
  // one round of resident workgroups covers the grid
  const int64_t nkc = std::max<int64_t>(1, resident / tiles);
  int k = (int)((d.nz + nkc - 1) / nkc);
  k = std::max(k, std::min(8, d.nz));
  *ty = t;
  *kc = std::min(k, d.nz);
  *tw = w;
}

// Tile widths of the fused step: 32, 64, 128 or 256 lanes.
static bool valid_tw(int tw) { return tw == 32 || tw == 64 || tw == 128 || tw == 256; }

// The fused kernel takes a uniform mu (in value; on a tensor grid too).
static bool fused_ok(const fit_grid* g) { return g->mu_uniform || (g->nu && g->mu_value_uniform); }

bool use_fused(const fit_grid* g) {
  if (g->path == 1) return false;
  return fused_ok(g);
}

// Host-side mirror of the probe membership of a direction-a edge (used only
// for argument validation).
static bool valid_box(const int32_t lo[3], const int32_t hi[3]) {
  for (int a = 0; a < 3; ++a)
    if (lo[a] > hi[a]) return false;
  return true;
}

void set_metric(const fit_grid* g, const double* sq[3]) {
  sq[0] = g->nu ? g->sq : nullptr;
  sq[1] = g->nu ? g->sq + g->d.nx : nullptr;
  sq[2] = g->nu ? g->sq + g->d.nx + g->d.ny : nullptr;
}

template <typename T>
static void fill_eargs(fit_grid* g, EArgs<T>& a, const T* ein, T* eout, const T* h, double dt,
                       int64_t m) {
  const Dims& d = g->d;
  for (int c = 0; c < 3; ++c) {
    a.ein[c] = ein + c * d.n;
    a.eout[c] = eout + c * d.n;
    a.h[c] = h + c * d.n;
    a.kb[c] = (T)(4.0 * dt / g->gedge[c]);
    a.ge[c] = g->gedge[c] / 4.0;
  }
  a.eps = static_cast<const T*>(g->eps);
  a.sig = static_cast<const T*>(g->sig);
  a.d = d;
  a.t = make_tiling(d, g->ty, g->kc);
  a.hs = (T)(0.5 * dt);
  set_metric(g, a.sq);
  a.kbs = 4.0 * dt;
  a.src_comp = g->src_axis;
  a.src_idx = g->src_axis >= 0 ? g->src_idx : -1;
  const double val = g->src_axis >= 0 ? source_value(g, dt, m) : 0.0;
  a.src_val = (T)val;
  a.src_val_d = (double)(T)val;
  a.probe = g->probe;
  a.part = g->part;
  a.pacc = g->pacc;
  a.pscale = dt;
}

template <typename T>
static void fill_hargs(fit_grid* g, HArgs<T>& a, const T* e, const T* hin, T* hout, double dt) {
  const Dims& d = g->d;
  for (int c = 0; c < 3; ++c) {
    a.e[c] = e + c * d.n;
    a.hin[c] = hin + c * d.n;
    a.hout[c] = hout + c * d.n;
    a.kd[c] = (T)(dt * g->gf2[c]);
    a.gf2[c] = g->gf2[c];
  }
  a.imu = g->mu_uniform ? nullptr : static_cast<const T*>(g->imu);
  a.imu_u = (T)g->imu_u;
  a.d = d;
  a.t = make_tiling(d, g->ty, g->kc);
  a.part = g->part;
  set_metric(g, a.sq);
  a.kds = dt;
}

ProfScope::ProfScope(fit_grid* g_, int kind) : g(g_), slot(-1) {
  if (!g->prof_on || g->prof_used >= (int64_t)g->prof_kind.size()) return;
  slot = g->prof_used++;
  g->prof_kind[slot] = kind;
  (void)hipEventRecord(g->prof_ev[2 * slot], g->s);
}

ProfScope::~ProfScope() {
  if (slot >= 0) (void)hipEventRecord(g->prof_ev[2 * slot + 1], g->s);
}

bool trace_at(const fit_grid* g, int64_t m) {
  const int64_t te = g->trace_every;
  if (te <= 0) return false;
  const int64_t r = (m - g->trace_m0) % te;
  return r == 0;
}

double source_value(const fit_grid* g, double dt, int64_t m) {
  const double t = ((double)m + 0.5) * dt;
  const double x = (t - g->sigma_t) / g->sigma_t;
  return g->i_max * std::exp(-4.0 * x * x);
}

// One leapfrog step m -> m+1 with separate e and h passes.  ein/eout and
// hin/hout may alias (in-place) or not (recording).  Energy partials and the
// trace rows are produced as configured on the handle.
template <typename T>
int step_once(fit_grid* g, double dt, const T* ein, T* eout, const T* hin, T* hout) {
  const int64_t m = g->m;
  const bool tr_this = trace_at(g, m);
  const bool tr_next = trace_at(g, m + 1);
  const bool have_row = tr_this && g->trace_rows < g->trace_cap;
  if (tr_this && !have_row) g->trace_dropped++;
  const bool probe = g->probe.on != 0;
  const Tiling t = make_tiling(g->d, g->ty, g->kc);
  const int64_t nb = t.blocks();
  if ((have_row || tr_next || probe) && ensure_part(g, nb)) return FIT_E_OOM;
  if (probe) {
    if (int rc = ensure_pacc(g, nb)) return rc;
  }
  double* row = have_row ? g->trace + g->trace_rows * FIT_TRACE_COLS : nullptr;
  hipError_t e;

  EArgs<T> ea;
  fill_eargs<T>(g, ea, ein, eout, hin, dt, m);
  {
    ProfScope ps(g, FIT_PROF_EPASS);
    e = launch_epass<T>(ea, g->lossy, have_row, probe, g->s);
  }
  if (e != hipSuccess) return hip_fail(e, "e-update launch");
  if (have_row) {
    const int cols[kPartTerms] = {1, 2, 3, 8, 9, -1, -1, -1, -1, -1};
    const bool prev_ok = g->pend_m == m;
    ProfScope ps(g, FIT_PROF_REDUCE);
    e = launch_reduce(g->part, nb, row, cols, -1, 0.0, nullptr, !prev_ok ? 4 : -1, m,
                      prev_ok ? g->pend : nullptr, 4, g->s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
  }

  HArgs<T> ha;
  fill_hargs<T>(g, ha, eout, hin, hout, dt);
  const bool henergy = have_row || tr_next;
  {
    ProfScope ps(g, FIT_PROF_HPASS);
    e = launch_hpass<T>(ha, g->mu_uniform, henergy, g->s);
  }
  if (e != hipSuccess) return hip_fail(e, "h-update launch");
  if (have_row) {
    const int cols[kPartTerms] = {5, 6, 7, -1, -1, -1, -1, -1, -1, -1};
    ProfScope ps(g, FIT_PROF_REDUCE);
    e = launch_reduce(g->part, nb, row, cols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
  }
  if (tr_next) {
    // <h^(m+1/2), h^(m+3/2)> is the h cross term of row m+1.
    const int cols[kPartTerms] = {-1, 0, -1, -1, -1, -1, -1, -1, -1, -1};
    ProfScope ps(g, FIT_PROF_REDUCE);
    e = launch_reduce(g->part, nb, g->pend, cols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    g->pend_m = m + 1;
  }
  if (have_row) g->trace_rows++;
  g->m = m + 1;
  g->smvp += 2;
  return FIT_OK;
}

template int step_once<float>(fit_grid*, double, const float*, float*, const float*, float*);
template int step_once<double>(fit_grid*, double, const double*, double*, const double*, double*);

// One fused leapfrog step m -> m+1: state read from (e, h), written to
// (e_alt, h_alt), then the two sets swap roles.
// Tensor-grid metric of the fused kernels: the per-axis arrays (squared
// widths, widths, dual widths, reciprocal widths) and the dt scales.
template <class Args>
static void set_nu_args(const fit_grid* g, double dt, Args& a) {
  const Dims& d = g->d;
  const int nn[3] = {d.nx, d.ny, d.nz};
  const int64_t tot = (int64_t)nn[0] + nn[1] + nn[2];
  int64_t off = 0;
  for (int c = 0; c < 3; ++c) {
    a.nsq[c] = g->sq + off;
    a.ndl[c] = g->sq + 2 * tot + off;
    a.nrw[c] = g->sq + 3 * tot + off;
    off += nn[c];
  }
  a.kbs = 4.0 * dt;
  a.kds = dt;
}

template <typename T>
int step_fused_io(fit_grid* g, double dt, const T* e0, const T* h0, T* e1, T* h1) {
  const int64_t m = g->m;
  const bool tr_this = trace_at(g, m);
  const bool tr_next = trace_at(g, m + 1);
  const bool have_row = tr_this && g->trace_rows < g->trace_cap;
  if (tr_this && !have_row) g->trace_dropped++;
  const bool probe = g->probe.on != 0;
  // the step before a trace row forms only the h cross term of that row
  const int energy = have_row ? kEnergyAll : tr_next ? kEnergyHCross : kEnergyNone;
  const Dims& d = g->d;
  SArgs<T> a;
  for (int c = 0; c < 3; ++c) {
    a.e0[c] = e0 + c * d.n;
    a.h0[c] = h0 + c * d.n;
    a.e1[c] = e1 + c * d.n;
    a.h1[c] = h1 + c * d.n;
    a.kb[c] = (T)(4.0 * dt / g->gedge[c]);
    a.kd[c] = (T)(dt * g->gf2[c]);
    a.ge[c] = g->gedge[c] / 4.0;
    a.gf2[c] = g->gf2[c];
  }
  a.eps = static_cast<const T*>(g->eps);
  a.sig = static_cast<const T*>(g->sig);
  a.d = d;
  a.t = make_tiling(d, g->sty, g->skc, g->stw);
  a.hs = (T)(0.5 * dt);
  a.imu2 = (T)g->imu_value + (T)g->imu_value;
  if (g->nu) {
    set_nu_args(g, dt, a);
    const int64_t tot = (int64_t)d.nx + d.ny + d.nz;
    a.nw[0] = g->sq + tot;
    a.nw[1] = a.nw[0] + d.nx;
    a.nw[2] = a.nw[1] + d.ny;
  }
  a.src_comp = g->src_axis;
  a.src_idx = g->src_axis >= 0 ? g->src_idx : -1;
  const double val = g->src_axis >= 0 ? source_value(g, dt, m) : 0.0;
  a.src_val = (T)val;
  a.src_val_d = (double)(T)val;
  a.probe = g->probe;
  const int64_t nb = a.t.blocks();
  if (energy && ensure_part(g, nb)) return FIT_E_OOM;
  if (probe) {
    if (int rc = ensure_pacc(g, nb)) return rc;
  }
  a.part = g->part;
  a.pacc = g->pacc;
  a.pscale = dt;
  hipError_t e;
  {
    ProfScope ps(g, FIT_PROF_STEP);
    e = launch_step<T>(a, g->lossy, energy, probe, g->s);
  }
  if (e != hipSuccess) return hip_fail(e, "fused step launch");
  if (have_row) {
    double* row = g->trace + g->trace_rows * FIT_TRACE_COLS;
    const int cols[kPartTerms] = {1, 2, 3, 8, 9, -1, 5, 6, 7, -1};
    const bool prev_ok = g->pend_m == m;
    ProfScope ps(g, FIT_PROF_REDUCE);
    e = launch_reduce(g->part, nb, row, cols, -1, 0.0, nullptr, !prev_ok ? 4 : -1, m,
                      prev_ok ? g->pend : nullptr, 4, g->s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
  }
  if (tr_next) {
    const int cols[kPartTerms] = {-1, -1, -1, -1, -1, -1, -1, 0, -1, -1};
    ProfScope ps(g, FIT_PROF_REDUCE);
    e = launch_reduce(g->part, nb, g->pend, cols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    g->pend_m = m + 1;
  }
  if (have_row) g->trace_rows++;
  g->m = m + 1;
  g->smvp += 2;
  return FIT_OK;
}

int ensure_alt(fit_grid* g) {
  if (g->e_alt) return FIT_OK;
  int rc = dev_alloc(&g->e_alt, 3 * g->d.n * g->esz, "e (second buffer)");
  if (!rc) rc = dev_alloc(&g->h_alt, 3 * g->d.n * g->esz, "h (second buffer)");
  if (rc) {
    dev_free(g->e_alt);
    dev_free(g->h_alt);
  }
  g->bor_ealt = g->bor_halt = false;
  g->storage_version++;
  return rc;
}

void swap_sets(fit_grid* g) {
  std::swap(g->e, g->e_alt);
  std::swap(g->h, g->h_alt);
  std::swap(g->bor_e, g->bor_ealt);
  std::swap(g->bor_h, g->bor_halt);
}

template <typename T>
int step_fused(fit_grid* g, double dt) {
  int rc = ensure_alt(g);
  if (rc) return rc;
  rc = step_fused_io<T>(g, dt, static_cast<const T*>(g->e), static_cast<const T*>(g->h),
                        static_cast<T*>(g->e_alt), static_cast<T*>(g->h_alt));
  if (rc) return rc;
  swap_sets(g);
  return FIT_OK;
}

// ---------------------------------------------------------------- step pairs
static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 256;
  }
  return cus;
}

// Planes per chunk for one round of resident pair workgroups.
static int pair_kc(const fit_grid* g, int tw, int ty) {
  const size_t lds = step2_lds_bytes(tw, ty, g->esz, g->lossy, g->nu);
  const int per_cu = std::max(1, std::min((int)((160 * 1024) / std::max<size_t>(lds, 1)),
                                          2048 / step2_threads(tw, ty)));
  const int64_t tiles = (int64_t)((g->d.nx + tw - 1) / tw) * ((g->d.ny + ty - 1) / ty);
  const int64_t nkc = std::max<int64_t>(1, (int64_t)device_cus() * per_cu / tiles);
  const int k = (int)((g->d.nz + nkc - 1) / nkc);
  return std::min(g->d.nz, std::max(k, std::min(8, g->d.nz)));
}

// How steps m, m+1 run: kPairNone (singly), kPairPlain (a pair; no trace
// row at m, m+1 or m+2 -- a row at m+2 needs step m+1's h cross term), or
// kPairEnergy (a pair whose second step records the row at m+1, its first
// step the row's pending h cross term; uniform grids, one-point tiles).
enum { kPairNone = 0, kPairPlain = 1, kPairEnergy = 2 };
static int pair_now(const fit_grid* g, int64_t nleft) {
  if (nleft < 2 || !g->pair_on || !use_fused(g) || g->probe.on) return kPairNone;
  if (!step2_plane_ok(g->d, g->esz)) return kPairNone;
  // the tile may no longer fit after the materials or spacing changed
  // (lossless -> lossy, uniform -> tensor grid)
  if (!step2_shape_ok(g->ptw, g->pty, g->esz, g->lossy, g->nu)) return kPairNone;
  const int64_t m = g->m;
  if (trace_at(g, m) || trace_at(g, m + 2)) return kPairNone;
  if (!trace_at(g, m + 1)) return kPairPlain;
  return step2_energy_ok(g->ptw, g->pty, g->nu) ? kPairEnergy : kPairNone;
}

// Two fused steps m -> m+2 in one launch: state read from (e, h), written to
// (e_alt, h_alt), then the two sets swap roles.  energy: the trace row of
// step m+1 is recorded from the launch's partial sums (dropped, and the pair
// run plainly, when the trace is full).
template <typename T>
static int step_pair(fit_grid* g, double dt, bool energy = false) {
  int rc = ensure_alt(g);
  if (rc) return rc;
  const Dims& d = g->d;
  const T* e0 = static_cast<const T*>(g->e);
  const T* h0 = static_cast<const T*>(g->h);
  T* e2 = static_cast<T*>(g->e_alt);
  T* h2 = static_cast<T*>(g->h_alt);
  S2Args<T> a;
  for (int c = 0; c < 3; ++c) {
    a.e0[c] = e0 + c * d.n;
    a.h0[c] = h0 + c * d.n;
    a.e2[c] = e2 + c * d.n;
    a.h2[c] = h2 + c * d.n;
    a.kb[c] = (T)(4.0 * dt / g->gedge[c]);
    a.kd[c] = (T)(dt * g->gf2[c]);
  }
  a.eps = static_cast<const T*>(g->eps);
  a.sig = static_cast<const T*>(g->sig);
  a.d = d;
  a.t = make_tiling(d, g->pty, g->pkc > 0 ? g->pkc : pair_kc(g, g->ptw, g->pty), g->ptw);
  a.hs = (T)(0.5 * dt);
  a.imu2 = (T)g->imu_value + (T)g->imu_value;
  a.src_comp = g->src_axis;
  a.src_idx = g->src_axis >= 0 ? g->src_idx : -1;
  a.src_val[0] = (T)(g->src_axis >= 0 ? source_value(g, dt, g->m) : 0.0);
  a.src_val[1] = (T)(g->src_axis >= 0 ? source_value(g, dt, g->m + 1) : 0.0);
  if (g->nu) set_nu_args(g, dt, a);
  if (energy && g->trace_rows >= g->trace_cap) {
    g->trace_dropped++;
    energy = false;
  }
  const int64_t nb = a.t.blocks();
  if (energy) {
    if (ensure_part(g, nb)) return FIT_E_OOM;
    for (int c = 0; c < 3; ++c) {
      a.ge[c] = g->gedge[c] / 4.0;
      a.gf2[c] = g->gf2[c];
    }
    a.part = g->part;
  }
  hipError_t e;
  {
    ProfScope ps(g, energy ? FIT_PROF_PAIR_ENERGY : FIT_PROF_PAIR);
    e = energy ? launch_step2_energy<T>(a, g->lossy, g->s) : launch_step2<T>(a, g->lossy, g->s);
  }
  if (e != hipSuccess) return hip_fail(e, "step pair launch");
  if (energy) {
    // the row of step m+1: its terms, and the first step's h cross term in
    // the pending column
    double* row = g->trace + g->trace_rows * FIT_TRACE_COLS;
    const int cols[kPartTerms] = {1, 2, 3, 8, 9, -1, 5, 6, 7, 4};
    ProfScope ps(g, FIT_PROF_REDUCE);
    e = launch_reduce(g->part, nb, row, cols, -1, 0.0, nullptr, -1, g->m + 1, nullptr, -1, g->s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    g->trace_rows++;
  }
  swap_sets(g);
  g->m += 2;
  g->smvp += 4;
  return FIT_OK;
}

// Time `reps` pair launches of one tile on the current state (out of place,
// swapped back: the state, step counter and pair setting are unchanged);
// *ms = time per pair.
template <typename T>
static int time_pair(fit_grid* g, double dt, int tw, int ty, int kc, int reps, float* ms) {
  const int s_on = g->pair_on, s_tw = g->ptw, s_ty = g->pty, s_kc = g->pkc;
  const int64_t s_m = g->m, s_smvp = g->smvp;
  g->ptw = tw;
  g->pty = ty;
  g->pkc = kc;
  hipEvent_t ev[2];
  (void)hipEventCreate(&ev[0]);
  (void)hipEventCreate(&ev[1]);
  auto one = [&]() -> int {
    int r = step_pair<T>(g, dt);
    swap_sets(g);
    return r;
  };
  int rc = FIT_OK;
  for (int w = 0; w < 2 && !rc; ++w) rc = one();
  if (!rc) {
    (void)hipEventRecord(ev[0], g->s);
    for (int r = 0; r < reps && !rc; ++r) rc = one();
    (void)hipEventRecord(ev[1], g->s);
    hipError_t e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
    if (e != hipSuccess && !rc) rc = hip_fail(e, "pair timing");
    *ms /= (float)std::max(reps, 1);
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  g->pair_on = s_on;
  g->ptw = s_tw;
  g->pty = s_ty;
  g->pkc = s_kc;
  g->m = s_m;
  g->smvp = s_smvp;
  return rc;
}

template int step_fused<float>(fit_grid*, double);
template int step_fused<double>(fit_grid*, double);
template int step_fused_io<float>(fit_grid*, double, const float*, const float*, float*, float*);
template int step_fused_io<double>(fit_grid*, double, const double*, const double*, double*,
                                   double*);

double step_dt(const fit_grid* g, double dt) {
  if (g->f64) return dt;
  float f = (float)dt;
  if ((double)f > dt) f = std::nextafter(f, 0.0f);
  return (double)f;
}

int check_dt(const fit_grid* g, double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FIT_E_INVALID, "dt must be positive and finite");
  if (!(g->desc.flags & FIT_ALLOW_UNSTABLE) && dt > g->cfl * (1.0 + 1e-12))
    return fail(FIT_E_UNSTABLE, "dt = " + std::to_string(dt) + " exceeds the CFL bound " +
                                    std::to_string(g->cfl));
  return FIT_OK;
}

template <typename T>
int upload_cells(fit_grid* g, void** dst, const std::vector<double>& v, const char* what) {
  if (!*dst) {
    int rc = dev_alloc(dst, v.size() * sizeof(T), what);
    if (rc) return rc;
  }
  std::vector<T> tmp(v.begin(), v.end());
  hipError_t e = hipMemcpyAsync(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, g->s);
  if (e == hipSuccess) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "material upload");
  return FIT_OK;
}

// Time `reps` launches of one candidate on fixed inputs: the fused kernel
// reads (e, h) and writes the second buffer set; the split kernels run out of
// place into the second set.  The handle's state is left untouched.
template <typename T>
int time_candidate(fit_grid* g, double dt, int path, int tw, int ty, int kc, int reps, float* ms) {
  const int save_path = g->path, save_ty = g->ty, save_kc = g->kc, save_sty = g->sty,
            save_skc = g->skc, save_stw = g->stw;
  const int64_t save_m = g->m, save_smvp = g->smvp, save_tr = g->trace_every;
  const int64_t save_pend = g->pend_m;
  const fit::Probe save_probe = g->probe;
  g->trace_every = 0;
  g->probe.on = 0;
  if (path == 2) {
    g->sty = ty;
    g->skc = kc;
    g->stw = tw;
  } else {
    g->ty = ty;
    g->kc = kc;
  }
  hipEvent_t ev[2];
  (void)hipEventCreate(&ev[0]);
  (void)hipEventCreate(&ev[1]);
  int rc = FIT_OK;
  auto one = [&]() -> int {
    if (path == 2) {
      // run the fused step, then swap back so the inputs stay the same
      int r = step_fused<T>(g, dt);
      swap_sets(g);
      return r;
    }
    if (int r = ensure_alt(g)) return r;
    return step_once<T>(g, dt, static_cast<const T*>(g->e), static_cast<T*>(g->e_alt),
                        static_cast<const T*>(g->h), static_cast<T*>(g->h_alt));
  };
  for (int w = 0; w < 2 && !rc; ++w) rc = one();
  if (!rc) {
    (void)hipEventRecord(ev[0], g->s);
    for (int r = 0; r < reps && !rc; ++r) rc = one();
    (void)hipEventRecord(ev[1], g->s);
    hipError_t e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
    if (e != hipSuccess && !rc) rc = hip_fail(e, "autotune timing");
    *ms /= (float)std::max(reps, 1);
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  g->path = save_path;
  g->ty = save_ty;
  g->kc = save_kc;
  g->sty = save_sty;
  g->skc = save_skc;
  g->stw = save_stw;
  g->m = save_m;
  g->smvp = save_smvp;
  g->trace_every = save_tr;
  g->pend_m = save_pend;
  g->probe = save_probe;
  return rc;
}

// Inner products of the step that starts at the current state (e^m,
// h^(m+1/2)), for fit_energy: the e-update runs out of place into the second
// buffer set (e^(m+1), with the trace terms <e^m,e^m>, <e^m,e^(m+1)>, loss and
// source), then the h-update with -dt turns h^(m+1/2) back into h^(m-1/2)
// (<h^(m+1/2),h^(m+1/2)> and <h^(m+1/2),h^(m-1/2)>).  row: device, 10
// doubles in the trace-row layout; part: partial rows of the split tiling.
template <typename T>
static int state_terms(fit_grid* g, double dt, double* part, double* row) {
  const Tiling t = make_tiling(g->d, g->ty, g->kc);
  const int64_t nb = t.blocks();
  const T* e = static_cast<const T*>(g->e);
  const T* h = static_cast<const T*>(g->h);
  EArgs<T> ea;
  fill_eargs<T>(g, ea, e, static_cast<T*>(g->e_alt), h, dt, g->m);
  ea.part = part;
  hipError_t er = launch_epass<T>(ea, g->lossy, true, false, g->s);
  if (er != hipSuccess) return hip_fail(er, "e-update launch");
  const int ecols[kPartTerms] = {1, 2, 3, 8, 9, -1, -1, -1, -1, -1};
  er = launch_reduce(part, nb, row, ecols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
  if (er != hipSuccess) return hip_fail(er, "reduce launch");
  HArgs<T> ha;
  fill_hargs<T>(g, ha, e, h, static_cast<T*>(g->h_alt), -dt);
  ha.part = part;
  er = launch_hpass<T>(ha, g->mu_uniform, true, g->s);
  if (er != hipSuccess) return hip_fail(er, "h-update launch");
  const int hcols[kPartTerms] = {5, 4, -1, -1, -1, -1, -1, -1, -1, -1};
  er = launch_reduce(part, nb, row, hcols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
  if (er != hipSuccess) return hip_fail(er, "reduce launch");
  return FIT_OK;
}

// Partial-sum rows the energy entry points need (standalone energy kernel and
// the split tiling of state_terms).
int64_t energy_rows(const fit_grid* g) {
  const Tiling t = make_tiling(g->d, g->ty, g->kc);
  return std::max<int64_t>(std::min<int64_t>((g->d.n + 255) / 256, kEnergyBlocks), t.blocks());
}

// Enqueue the five energies of the current state into out (device, 5
// doubles): the standalone <e,e>, <h,h> kernel, then (once a step has fixed
// dt) the inner products of state_terms, combined on the device.  part: at
// least energy_rows(g) rows; work: 12 doubles of device scratch.  The second
// field buffer set must exist.  Allocates nothing.
int energy_enqueue(fit_grid* g, double* part, double* work, double* out) {
  double ge[3], gf2[3];
  for (int a = 0; a < 3; ++a) {
    ge[a] = g->gedge[a] / 4.0;
    gf2[a] = g->gf2[a];
  }
  int64_t nblk = 0;
  hipError_t e;
  if (g->f64)
    e = launch_energy<double>(static_cast<const double*>(g->e), static_cast<const double*>(g->h),
                              static_cast<const double*>(g->eps),
                              g->mu_uniform ? nullptr : static_cast<const double*>(g->imu),
                              g->imu_u, g->d, ge, gf2, g->nu ? g->sq : nullptr, part, &nblk,
                              g->s);
  else
    e = launch_energy<float>(static_cast<const float*>(g->e), static_cast<const float*>(g->h),
                             static_cast<const float*>(g->eps),
                             g->mu_uniform ? nullptr : static_cast<const float*>(g->imu),
                             (float)g->imu_u, g->d, ge, gf2, g->nu ? g->sq : nullptr, part,
                             &nblk, g->s);
  if (e != hipSuccess) return hip_fail(e, "energy launch");
  const int cols[kPartTerms] = {0, 1, -1, -1, -1, -1, -1, -1, -1, -1};
  e = launch_reduce(part, nblk, work, cols, -1, 0.0, nullptr, -1, -1, nullptr, -1, g->s);
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  const double dt = g->last_dt;
  if (dt > 0.0) {
    int rc = g->f64 ? state_terms<double>(g, dt, part, work + 2)
                    : state_terms<float>(g, dt, part, work + 2);
    if (rc) return rc;
  }
  e = launch_energy_combine(work, dt, out, g->s);
  if (e != hipSuccess) return hip_fail(e, "energy combine launch");
  return FIT_OK;
}

}  // namespace fit

using namespace fit;

extern "C" {

const char* fit_version(void) { return "fitmi 0.1 (gfx950)"; }

const char* fit_last_error(void) { return g_err.c_str(); }

int fit_grid_create(const fit_grid_desc* desc, void* stream, fit_grid** out) {
  if (!desc || !out) return fail(FIT_E_INVALID, "null argument");
  *out = nullptr;
  if (desc->nx < 1 || desc->ny < 1 || desc->nz < 1)
    return fail(FIT_E_INVALID, "need at least one cell per axis");
  if (desc->dtype != FIT_F32 && desc->dtype != FIT_F64) return fail(FIT_E_INVALID, "bad dtype");
  const double sp[3] = {desc->dx, desc->dy, desc->dz};
  for (double v : sp)
    if (!(v >= 0.0) || !std::isfinite(v)) return fail(FIT_E_INVALID, "spacings must be >= 0");
  if (!(desc->eps0 >= 0.0) || !(desc->mu0 >= 0.0) || !std::isfinite(desc->eps0) ||
      !std::isfinite(desc->mu0))
    return fail(FIT_E_INVALID, "eps0, mu0 must be >= 0");
  const int64_t n = (int64_t)desc->nx * desc->ny * desc->nz;
  if (n > (int64_t)1 << 40) return fail(FIT_E_INVALID, "grid too large");
  fit_grid* g = new (std::nothrow) fit_grid();
  if (!g) return fail(FIT_E_OOM, "host allocation failed");
  g->desc = *desc;
  double* dd[3] = {&g->desc.dx, &g->desc.dy, &g->desc.dz};
  for (double* v : dd)
    if (*v == 0.0) *v = 1.0;
  if (g->desc.eps0 == 0.0) g->desc.eps0 = 1.0;
  if (g->desc.mu0 == 0.0) g->desc.mu0 = 1.0;
  g->s = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&g->dev) != hipSuccess) {
    (void)hipGetLastError();
    g->dev = 0;
  }
  g->f64 = desc->dtype == FIT_F64;
  g->esz = g->f64 ? 8 : 4;
  g->d.nx = desc->nx;
  g->d.ny = desc->ny;
  g->d.nz = desc->nz;
  g->d.sx = desc->nx;
  g->d.sxy = (int64_t)desc->nx * desc->ny;
  g->d.n = n;
  const double s3[3] = {g->desc.dx, g->desc.dy, g->desc.dz};
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    g->gedge[a] = s3[b] * s3[c] / s3[a];          // M_eps = eps * g_a
    g->gf2[a] = s3[a] / (s3[b] * s3[c]) / 2.0;    // M_mu^{-1} = gf2 (imu_1 + imu_2)
  }
  default_tiling(g->d, &g->ty, &g->kc);
  default_step_tiling(g->d, g->esz, false, &g->sty, &g->skc, &g->stw);
  int rc = dev_alloc(&g->e, 3 * n * g->esz, "e");
  if (!rc) rc = dev_alloc(&g->h, 3 * n * g->esz, "h");
  if (!rc) rc = dev_alloc(&g->eps, n * g->esz, "eps");
  if (!rc) rc = dev_alloc(reinterpret_cast<void**>(&g->jacc), kJaccLen * sizeof(double), "probe sum");
  if (!rc) rc = dev_alloc(reinterpret_cast<void**>(&g->pend), sizeof(double), "pending term");
  if (rc) {
    fit_grid_destroy(g);
    return rc;
  }
  hipError_t e = hipMemsetAsync(g->e, 0, 3 * n * g->esz, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(g->h, 0, 3 * n * g->esz, g->s);
  if (e == hipSuccess) e = hipMemsetAsync(g->jacc, 0, kJaccLen * sizeof(double), g->s);
  if (e != hipSuccess) {
    fit_grid_destroy(g);
    return hip_fail(e, "initial clear");
  }
  // vacuum materials
  std::vector<double> ones((size_t)n, 1.0);
  rc = fit_set_materials(g, ones.data(), nullptr, nullptr);
  if (rc) {
    fit_grid_destroy(g);
    return rc;
  }
  *out = g;
  return FIT_OK;
}

int fit_grid_destroy(fit_grid* g) {
  if (!g) return FIT_OK;
  (void)hipStreamSynchronize(g->s);
  for (hipEvent_t ev : g->prof_ev) (void)hipEventDestroy(ev);
  g->prof_ev.clear();
  grid_release_extras(g);
  if (!g->bor_e) dev_free(g->e);
  if (!g->bor_h) dev_free(g->h);
  if (!g->bor_ealt) dev_free(g->e_alt);
  if (!g->bor_halt) dev_free(g->h_alt);
  if (!g->bor_mat) {
    dev_free(g->eps);
    dev_free(g->sig);
    dev_free(g->imu);
  }
  dev_free(reinterpret_cast<void*&>(g->sq));
  dev_free(reinterpret_cast<void*&>(g->part));
  dev_free(reinterpret_cast<void*&>(g->trace));
  dev_free(reinterpret_cast<void*&>(g->jacc));
  dev_free(reinterpret_cast<void*&>(g->pend));
  dev_free(reinterpret_cast<void*&>(g->pacc));
  dev_free(g->xw);
  dev_free(g->lw);
  dev_free(reinterpret_cast<void*&>(g->gram_part));
  dev_free(reinterpret_cast<void*&>(g->gram_G));
  dev_free(reinterpret_cast<void*&>(g->gram_w[0]));
  dev_free(reinterpret_cast<void*&>(g->gram_w[1]));
  delete g;
  return FIT_OK;
}

// Uploads the per-cell device arrays from the stored inputs (g->in_*) and
// the current spacing.  On a tensor grid the arrays hold the cell values
// times the cell volume and imu is always per cell.
static int apply_materials(fit_grid* g) {
  g->gram_w_ok[0] = g->gram_w_ok[1] = false;
  const int64_t n = g->d.n;
  const int nx = g->d.nx, ny = g->d.ny;
  const bool has_mu = !g->in_mu.empty(), has_sig = !g->in_sig.empty();
  // imu per cell only where it can vary (per-cell mu or a tensor grid)
  const bool per_cell_mu = has_mu || g->nu;
  std::vector<double> eps((size_t)n), imu(per_cell_mu ? (size_t)n : 1), sig;
  bool lossy = false;
  double ratio = INFINITY;   // min over cells of eps mu / (dx^-2 + dy^-2 + dz^-2)
  const double inv_u = 1.0 / (g->desc.dx * g->desc.dx) + 1.0 / (g->desc.dy * g->desc.dy) +
                       1.0 / (g->desc.dz * g->desc.dz);
  const double eps0 = g->desc.eps0, mu0 = g->desc.mu0;
  bool mu_uni = !g->nu;
  bool mu_val_uni = true;
  if (!per_cell_mu) imu[0] = 1.0 / mu0;
  if (has_sig) sig.resize((size_t)n);
  for (int64_t c = 0; c < n; ++c) {
    const double er = g->in_eps[c];
    const double mr = has_mu ? g->in_mu[c] : 1.0;
    double vol = 1.0, inv = inv_u;
    if (g->nu) {
      const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((int64_t)nx * ny));
      const double wx = g->wd[0][i], wy = g->wd[1][j], wz = g->wd[2][k];
      vol = wx * wy * wz;
      inv = 1.0 / (wx * wx) + 1.0 / (wy * wy) + 1.0 / (wz * wz);
    }
    eps[c] = eps0 * er * vol;
    if (per_cell_mu) {
      imu[c] = vol / (mu0 * mr);
      if (imu[c] != imu[0]) mu_uni = false;
      if (has_mu && mr != g->in_mu[0]) mu_val_uni = false;
    }
    ratio = std::min(ratio, eps0 * er * (mu0 * mr) / inv);
    if (has_sig) {
      sig[c] = g->in_sig[c] * vol;
      if (g->in_sig[c] != 0.0) lossy = true;
    }
  }
  const double cfl = std::sqrt(ratio);   // sqrt is monotone: the min of the roots
  int rc = g->f64 ? upload_cells<double>(g, &g->eps, eps, "eps") : upload_cells<float>(g, &g->eps, eps, "eps");
  if (rc) return rc;
  if (lossy) {
    rc = g->f64 ? upload_cells<double>(g, &g->sig, sig, "sigma")
                : upload_cells<float>(g, &g->sig, sig, "sigma");
    if (rc) return rc;
  }
  if (!mu_uni) {
    rc = g->f64 ? upload_cells<double>(g, &g->imu, imu, "1/mu")
                : upload_cells<float>(g, &g->imu, imu, "1/mu");
    if (rc) return rc;
  }
  g->lossy = lossy;
  g->mu_uniform = mu_uni;
  if (!g->tile_explicit) default_step_tiling(g->d, g->esz, lossy, &g->sty, &g->skc, &g->stw);
  g->imu_u = imu[0];
  g->mu_value_uniform = mu_val_uni;
  g->imu_value = 1.0 / (mu0 * (has_mu ? g->in_mu[0] : 1.0));
  g->cfl = cfl;
  g->materials_version++;
  return FIT_OK;
}

int fit_set_materials(fit_grid* g, const double* eps_r, const double* mu_r, const double* sigma) {
  if (!g || !eps_r) return fail(FIT_E_INVALID, "null argument");
  const int64_t n = g->d.n;
  for (int64_t c = 0; c < n; ++c) {
    if (!(eps_r[c] > 0.0) || !std::isfinite(eps_r[c]))
      return fail(FIT_E_INVALID, "eps_r must be > 0 and finite");
    if (mu_r && (!(mu_r[c] > 0.0) || !std::isfinite(mu_r[c])))
      return fail(FIT_E_INVALID, "mu_r must be > 0 and finite");
    if (sigma && (!(sigma[c] >= 0.0) || !std::isfinite(sigma[c])))
      return fail(FIT_E_INVALID, "sigma must be >= 0 and finite");
  }
  g->in_eps.assign(eps_r, eps_r + n);
  if (mu_r) g->in_mu.assign(mu_r, mu_r + n);
  else g->in_mu.clear();
  if (sigma) g->in_sig.assign(sigma, sigma + n);
  else g->in_sig.clear();
  return apply_materials(g);
}

int fit_set_spacing(fit_grid* g, const double* dx, const double* dy, const double* dz) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  const double* w[3] = {dx, dy, dz};
  const int nn[3] = {g->d.nx, g->d.ny, g->d.nz};
  const int nnull = (dx == nullptr) + (dy == nullptr) + (dz == nullptr);
  if (nnull == 3) {
    g->nu = false;
    for (auto& v : g->wd) v.clear();
    return apply_materials(g);
  }
  if (nnull != 0) return fail(FIT_E_INVALID, "give all three width arrays or none");
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < nn[a]; ++i)
      if (!(w[a][i] > 0.0) || !std::isfinite(w[a][i]))
        return fail(FIT_E_INVALID, "cell widths must be > 0 and finite");
  if (!g->sq) {
    int rc = dev_alloc(reinterpret_cast<void**>(&g->sq),
                       4 * (size_t)(nn[0] + nn[1] + nn[2]) * sizeof(double), "cell widths");
    if (rc) return rc;
  }
  std::vector<double> q, wv, dl, rw;
  for (int a = 0; a < 3; ++a) {
    g->wd[a].assign(w[a], w[a] + nn[a]);
    for (int i = 0; i < nn[a]; ++i) {
      q.push_back(w[a][i] * w[a][i]);
      wv.push_back(w[a][i]);
      dl.push_back(0.5 * ((i > 0 ? w[a][i - 1] : 0.0) + w[a][i]));
      rw.push_back(1.0 / w[a][i]);
    }
  }
  q.insert(q.end(), wv.begin(), wv.end());
  q.insert(q.end(), dl.begin(), dl.end());
  q.insert(q.end(), rw.begin(), rw.end());
  hipError_t e = hipMemcpyAsync(g->sq, q.data(), q.size() * sizeof(double),
                                hipMemcpyHostToDevice, g->s);
  if (e == hipSuccess) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "cell widths upload");
  g->nu = true;
  return apply_materials(g);
}

int fit_set_source(fit_grid* g, int axis, int i, int j, int k, double i_max, double sigma_t) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (axis == -1) {
    g->src_axis = -1;
    g->src_idx = -1;
    return FIT_OK;
  }
  if (axis < 0 || axis > 2) return fail(FIT_E_INVALID, "axis must be 0, 1, 2 or -1");
  if (!(sigma_t > 0.0) || !std::isfinite(sigma_t) || !std::isfinite(i_max))
    return fail(FIT_E_INVALID, "sigma_t must be > 0");
  const int p[3] = {i, j, k};
  const int nn[3] = {g->d.nx, g->d.ny, g->d.nz};
  for (int a = 0; a < 3; ++a) {
    const int lo = (a == axis) ? 0 : 1;
    const int hi = (a == axis) ? nn[a] - 1 : nn[a] - 1;
    if (p[a] < lo || p[a] > hi)
      return fail(FIT_E_INVALID, "source edge lies outside the grid or in a PEC wall");
  }
  g->src_axis = axis;
  g->src_idx = (int64_t)i + g->d.sx * j + g->d.sxy * (int64_t)k;
  g->i_max = i_max;
  g->sigma_t = sigma_t;
  return FIT_OK;
}

int fit_step_dt(const fit_grid* g, double dt, double* dt_used) {
  if (!g || !dt_used) return fail(FIT_E_INVALID, "null argument");
  *dt_used = step_dt(g, dt);
  return FIT_OK;
}

int fit_cfl_dt(const fit_grid* g, double* dt_cfl) {
  if (!g || !dt_cfl) return fail(FIT_E_INVALID, "null argument");
  *dt_cfl = g->cfl;
  return FIT_OK;
}

static int copy_field(fit_grid* g, void* dst, const void* src, int dir_in, int on_device) {
  const size_t bytes = 3 * (size_t)g->d.n * g->esz;
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice
                                 : (dir_in ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, g->s);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "field copy");
  return FIT_OK;
}

// Caller-provided device buffers: aligned to 16 bytes, pairwise disjoint
// (each `bytes` long) and none of them a buffer the library owns.
static int check_borrowed(const fit_grid* g, void* const* p, int np, size_t bytes) {
  const void* owned[7] = {g->bor_e ? nullptr : g->e,        g->bor_h ? nullptr : g->h,
                          g->bor_ealt ? nullptr : g->e_alt, g->bor_halt ? nullptr : g->h_alt,
                          g->bor_mat ? nullptr : g->eps,    g->bor_mat ? nullptr : g->sig,
                          g->bor_mat ? nullptr : g->imu};
  for (int a = 0; a < np; ++a) {
    if (!p[a]) continue;
    if (reinterpret_cast<uintptr_t>(p[a]) % 16 != 0)
      return fail(FIT_E_INVALID, "bound buffers must be aligned to 16 bytes");
    for (const void* o : owned)
      if (o && o == p[a]) return fail(FIT_E_INVALID, "a bound buffer is library-owned storage");
    const char* x = static_cast<const char*>(p[a]);
    for (int b = 0; b < a; ++b) {
      const char* y = static_cast<const char*>(p[b]);
      if (y && x < y + bytes && y < x + bytes)
        return fail(FIT_E_INVALID, "bound buffers must not overlap");
    }
  }
  return FIT_OK;
}

int fit_bind_fields(fit_grid* g, void* e, void* h, void* e_alt, void* h_alt) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  const size_t fb = 3 * (size_t)g->d.n * g->esz;
  const bool unbind = !e && !h && !e_alt && !h_alt;
  if (!unbind) {
    if (!e || !h) return fail(FIT_E_INVALID, "e and h are both required");
    if ((e_alt == nullptr) != (h_alt == nullptr))
      return fail(FIT_E_INVALID, "give both second-set buffers or neither");
    void* p[4] = {e, h, e_alt, h_alt};
    if (int rc = check_borrowed(g, p, 4, fb)) return rc;
  }
  hipError_t er = hipStreamSynchronize(g->s);   // no launch may still use the old buffers
  if (er != hipSuccess) return hip_fail(er, "bind sync");
  void* ne = e;
  void* nh = h;
  if (unbind) {   // the state moves back into library-owned buffers
    ne = g->bor_e ? nullptr : g->e;
    nh = g->bor_h ? nullptr : g->h;
    if (!ne) {
      if (int rc = dev_alloc(&ne, fb, "e")) return rc;
    }
    if (!nh) {
      if (int rc = dev_alloc(&nh, fb, "h")) {
        if (g->bor_e) dev_free(ne);
        return rc;
      }
    }
  }
  if (ne != g->e) er = hipMemcpyAsync(ne, g->e, fb, hipMemcpyDeviceToDevice, g->s);
  if (er == hipSuccess && nh != g->h) er = hipMemcpyAsync(nh, g->h, fb, hipMemcpyDeviceToDevice, g->s);
  if (er == hipSuccess) er = hipStreamSynchronize(g->s);
  if (er != hipSuccess) return hip_fail(er, "state copy into the bound buffers");
  if (!g->bor_e && g->e != ne) dev_free(g->e);
  if (!g->bor_h && g->h != nh) dev_free(g->h);
  g->e = ne;
  g->h = nh;
  g->bor_e = g->bor_h = !unbind;
  if (e_alt) {
    if (!g->bor_ealt) dev_free(g->e_alt);
    if (!g->bor_halt) dev_free(g->h_alt);
    g->e_alt = e_alt;
    g->h_alt = h_alt;
    g->bor_ealt = g->bor_halt = true;
  } else if (g->bor_ealt || g->bor_halt) {   // allocated again on first use
    if (!g->bor_ealt) dev_free(g->e_alt);
    if (!g->bor_halt) dev_free(g->h_alt);
    g->e_alt = g->h_alt = nullptr;
    g->bor_ealt = g->bor_halt = false;
  }
  g->storage_version++;
  return FIT_OK;
}

int fit_bind_materials(fit_grid* g, void* eps, void* sigma, void* imu) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  const size_t cb = (size_t)g->d.n * g->esz;
  const bool unbind = !eps && !sigma && !imu;
  if (!unbind) {
    if (!eps || !sigma || !imu) return fail(FIT_E_INVALID, "give all three cell buffers or none");
    void* p[3] = {eps, sigma, imu};
    if (int rc = check_borrowed(g, p, 3, cb)) return rc;
    const void* f[4] = {g->e, g->h, g->e_alt, g->h_alt};
    for (void* q : p)
      for (const void* o : f)
        if (o && q == o) return fail(FIT_E_INVALID, "a cell buffer is a field buffer");
  }
  hipError_t er = hipStreamSynchronize(g->s);
  if (er != hipSuccess) return hip_fail(er, "bind sync");
  if (!g->bor_mat) {
    dev_free(g->eps);
    dev_free(g->sig);
    dev_free(g->imu);
  }
  g->eps = eps;
  g->sig = sigma;
  g->imu = imu;
  g->bor_mat = !unbind;
  g->storage_version++;
  return apply_materials(g);   // writes the current materials into the new buffers
}

int fit_get_state(const fit_grid* g, void** e, void** h) {
  if (!g || !e || !h) return fail(FIT_E_INVALID, "null argument");
  *e = g->e;
  *h = g->h;
  return FIT_OK;
}

int fit_set_fields(fit_grid* g, const void* e, const void* h, int64_t step, int on_device) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (step < 0) return fail(FIT_E_INVALID, "step must be >= 0");
  const size_t bytes = 3 * (size_t)g->d.n * g->esz;
  hipError_t er;
  int rc;
  if (e) {
    if ((rc = copy_field(g, g->e, e, 1, on_device))) return rc;
  } else if ((er = hipMemsetAsync(g->e, 0, bytes, g->s)) != hipSuccess) {
    return hip_fail(er, "clear e");
  }
  if (h) {
    if ((rc = copy_field(g, g->h, h, 1, on_device))) return rc;
  } else if ((er = hipMemsetAsync(g->h, 0, bytes, g->s)) != hipSuccess) {
    return hip_fail(er, "clear h");
  }
  if (g->f64) {
    er = launch_mask<double>(static_cast<double*>(g->e), g->d, 0, g->s);
    if (er == hipSuccess) er = launch_mask<double>(static_cast<double*>(g->h), g->d, 1, g->s);
  } else {
    er = launch_mask<float>(static_cast<float*>(g->e), g->d, 0, g->s);
    if (er == hipSuccess) er = launch_mask<float>(static_cast<float*>(g->h), g->d, 1, g->s);
  }
  if (er != hipSuccess) return hip_fail(er, "PEC mask");
  g->m = step;
  g->pend_m = -1;
  return FIT_OK;
}

int fit_get_fields(fit_grid* g, void* e, void* h, int on_device) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  int rc;
  if (e && (rc = copy_field(g, e, g->e, 0, on_device))) return rc;
  if (h && (rc = copy_field(g, h, g->h, 0, on_device))) return rc;
  return FIT_OK;
}

int fit_get_step(const fit_grid* g, int64_t* step) {
  if (!g || !step) return fail(FIT_E_INVALID, "null argument");
  *step = g->m;
  return FIT_OK;
}

int fit_apply_curl(fit_grid* g, int which, const void* in, void* out) {
  if (!g || !in || !out) return fail(FIT_E_INVALID, "null argument");
  if (which != 0 && which != 1) return fail(FIT_E_INVALID, "which must be 0 (C) or 1 (C~)");
  if (in == out) return fail(FIT_E_INVALID, "in and out must differ");
  hipError_t e = g->f64 ? launch_curl<double>(static_cast<const double*>(in), static_cast<double*>(out), g->d, which, g->s)
                        : launch_curl<float>(static_cast<const float*>(in), static_cast<float*>(out), g->d, which, g->s);
  if (e != hipSuccess) return hip_fail(e, "curl launch");
  return FIT_OK;
}

int fit_step(fit_grid* g, int64_t nsteps, double dt) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (nsteps < 0) return fail(FIT_E_INVALID, "nsteps must be >= 0");
  int rc = check_dt(g, dt);
  if (rc) return rc;
  dt = step_dt(g, dt);
  if (nsteps > 0) g->last_dt = dt;
  const bool fused = use_fused(g);
  for (int64_t s = 0; s < nsteps; ++s) {
    const int pm = fused ? pair_now(g, nsteps - s) : kPairNone;
    if (pm != kPairNone) {
      const bool en = pm == kPairEnergy;
      rc = g->f64 ? step_pair<double>(g, dt, en) : step_pair<float>(g, dt, en);
      ++s;
    } else if (fused) {
      rc = g->f64 ? step_fused<double>(g, dt) : step_fused<float>(g, dt);
    } else {
      rc = g->f64 ? step_once<double>(g, dt, static_cast<const double*>(g->e), static_cast<double*>(g->e),
                                      static_cast<const double*>(g->h), static_cast<double*>(g->h))
                  : step_once<float>(g, dt, static_cast<const float*>(g->e), static_cast<float*>(g->e),
                                     static_cast<const float*>(g->h), static_cast<float*>(g->h));
    }
    if (rc) return rc;
  }
  return FIT_OK;
}

int fit_energy(fit_grid* g, double out[5]) {
  if (!g || !out) return fail(FIT_E_INVALID, "null argument");
  int rc = ensure_alt(g);
  if (!rc) rc = ensure_part(g, energy_rows(g));
  if (!rc) rc = energy_enqueue(g, g->part, g->jacc + kJaccWork, g->jacc + kJaccOut);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(out, g->jacc + kJaccOut, 5 * sizeof(double),
                                hipMemcpyDeviceToHost, g->s);
  if (e == hipSuccess) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "energy readback");
  if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
    return fail(FIT_E_DIVERGED, "energy is not finite");
  return FIT_OK;
}

int fit_trace_config(fit_grid* g, int64_t every, int64_t capacity) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (every < 0 || capacity < 0) return fail(FIT_E_INVALID, "every, capacity must be >= 0");
  (void)hipStreamSynchronize(g->s);
  dev_free(reinterpret_cast<void*&>(g->trace));
  g->trace_every = 0;
  g->trace_cap = 0;
  g->trace_rows = 0;
  g->trace_dropped = 0;
  g->pend_m = -1;
  g->trace_m0 = g->m;
  if (every > 0 && capacity > 0) {
    int rc = dev_alloc(reinterpret_cast<void**>(&g->trace),
                       (size_t)capacity * FIT_TRACE_COLS * sizeof(double), "trace");
    if (rc) return rc;
    g->trace_every = every;
    g->trace_cap = capacity;
  }
  return FIT_OK;
}

int fit_trace_read(fit_grid* g, double* out, int64_t max_rows, int64_t* nrows, int64_t* dropped) {
  if (!g || !nrows || (max_rows > 0 && !out)) return fail(FIT_E_INVALID, "null argument");
  const int64_t n = std::min<int64_t>(std::max<int64_t>(max_rows, 0), g->trace_rows);
  if (n > 0) {
    hipError_t e = hipMemcpyAsync(out, g->trace, (size_t)n * FIT_TRACE_COLS * sizeof(double),
                                  hipMemcpyDeviceToHost, g->s);
    if (e != hipSuccess) return hip_fail(e, "trace readback");
  }
  hipError_t e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "trace readback");
  *nrows = n;
  if (dropped) *dropped = g->trace_dropped + (g->trace_rows - n);
  g->trace_rows = 0;
  g->trace_dropped = 0;
  for (int64_t r = 0; r < n; ++r)
    if (!std::isfinite(out[r * FIT_TRACE_COLS + 1]) || !std::isfinite(out[r * FIT_TRACE_COLS + 5]))
      return fail(FIT_E_DIVERGED, "traced energy is not finite");
  return FIT_OK;
}

int fit_set_probe(fit_grid* g, const int32_t lo[3], const int32_t hi[3]) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (!lo && !hi) {
    g->probe.on = 0;
  } else {
    if (!lo || !hi || !valid_box(lo, hi)) return fail(FIT_E_INVALID, "bad probe box");
    for (int a = 0; a < 3; ++a) {
      g->probe.lo[a] = lo[a];
      g->probe.hi[a] = hi[a];
    }
    g->probe.on = 1;
  }
  return fit_probe_reset(g);
}

int fit_probe_value(fit_grid* g, double* J) {
  if (!g || !J) return fail(FIT_E_INVALID, "null argument");
  double v[2];
  hipError_t e = hipSuccess;
  if (g->pacc) e = launch_pacc_flush(g->pacc, g->pacc_rows, g->jacc, g->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(v, g->jacc, 2 * sizeof(double), hipMemcpyDeviceToHost, g->s);
  if (e == hipSuccess) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "probe readback");
  *J = v[0] + v[1];
  return FIT_OK;
}

int fit_probe_reset(fit_grid* g) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  hipError_t e = hipMemsetAsync(g->jacc, 0, 2 * sizeof(double), g->s);
  if (e == hipSuccess && g->pacc)
    e = hipMemsetAsync(g->pacc, 0, (size_t)g->pacc_rows * 2 * sizeof(double), g->s);
  if (e != hipSuccess) return hip_fail(e, "probe reset");
  return FIT_OK;
}

int fit_profile_begin(fit_grid* g, int64_t max_launches) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (max_launches < 0 || max_launches > (1 << 22)) return fail(FIT_E_INVALID, "bad max_launches");
  const size_t need = 2 * (size_t)max_launches;
  while (g->prof_ev.size() < need) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    g->prof_ev.push_back(ev);
  }
  g->prof_kind.assign((size_t)max_launches, FIT_PROF_OTHER);
  g->prof_used = 0;
  g->prof_on = true;
  return FIT_OK;
}

int fit_profile_end(fit_grid* g, double ms[FIT_PROF_N], int64_t count[FIT_PROF_N]) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (!g->prof_on) return fail(FIT_E_STATE, "profiling was not started");
  g->prof_on = false;
  hipError_t e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "profile sync");
  double acc[FIT_PROF_N] = {0};
  int64_t cnt[FIT_PROF_N] = {0};
  for (int64_t i = 0; i < g->prof_used; ++i) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, g->prof_ev[2 * i], g->prof_ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    acc[g->prof_kind[i]] += t;
    cnt[g->prof_kind[i]]++;
  }
  for (int k = 0; k < FIT_PROF_N; ++k) {
    if (ms) ms[k] = acc[k];
    if (count) count[k] = cnt[k];
  }
  return FIT_OK;
}

int fit_gram(fit_grid* g, const void* X, int64_t ld, int K, int which, double* G) {
  if (!g || !X || !G) return fail(FIT_E_INVALID, "null argument");
  if (K < 1 || K > 4096) return fail(FIT_E_INVALID, "K must be in [1, 4096]");
  if (which != 0 && which != 1) return fail(FIT_E_INVALID, "which must be 0 (e, M_eps) or 1 (h, M_mu)");
  if (ld < 3 * g->d.n) return fail(FIT_E_INVALID, "ld must be >= 3 nx ny nz");
  const int64_t cap_blocks = 1024;
  int rc = FIT_OK;
  if (!g->gram_part)
    rc = dev_alloc(reinterpret_cast<void**>(&g->gram_part),
                   (size_t)cap_blocks * 64 * 64 * sizeof(double), "Gram partials");
  if (rc) return rc;
  if (g->gram_G_cap < (int64_t)K * K) {
    dev_free(reinterpret_cast<void*&>(g->gram_G));
    g->gram_G_cap = 0;
    rc = dev_alloc(reinterpret_cast<void**>(&g->gram_G), (size_t)K * K * sizeof(double), "Gram");
    if (rc) return rc;
    g->gram_G_cap = (int64_t)K * K;
  }
  hipError_t e;
  if (!g->gram_w_ok[which]) {
    if (!g->gram_w[which]) {
      rc = dev_alloc(reinterpret_cast<void**>(&g->gram_w[which]), (size_t)(3 * g->d.n) * sizeof(double),
                     "Gram weights");
      if (rc) return rc;
    }
    double gw[3];
    for (int a = 0; a < 3; ++a) gw[a] = which == 0 ? g->gedge[a] / 4.0 : g->gf2[a];
    if (g->f64)
      e = launch_gram_weights<double>(g->gram_w[which], which, static_cast<const double*>(g->eps),
                                      g->mu_uniform ? nullptr : static_cast<const double*>(g->imu),
                                      g->imu_u, g->d, gw, g->nu ? g->sq : nullptr, g->s);
    else
      e = launch_gram_weights<float>(g->gram_w[which], which, static_cast<const float*>(g->eps),
                                     g->mu_uniform ? nullptr : static_cast<const float*>(g->imu),
                                     (float)g->imu_u, g->d, gw, g->nu ? g->sq : nullptr, g->s);
    if (e != hipSuccess) return hip_fail(e, "Gram weights");
    g->gram_w_ok[which] = true;
  }
  int64_t nwg = 0;
  {
    ProfScope ps(g, FIT_PROF_OTHER);
    if (g->f64)
      e = launch_gram<double>(static_cast<const double*>(X), ld, K, g->gram_w[which], g->d,
                              g->gram_part, cap_blocks, g->gram_G, g->s, &nwg);
    else
      e = launch_gram<float>(static_cast<const float*>(X), ld, K, g->gram_w[which], g->d,
                             g->gram_part, cap_blocks, g->gram_G, g->s, &nwg);
  }
  if (e != hipSuccess) return hip_fail(e, "Gram launch");
  e = hipMemcpyAsync(G, g->gram_G, (size_t)K * K * sizeof(double), hipMemcpyDeviceToHost, g->s);
  if (e == hipSuccess) e = hipStreamSynchronize(g->s);
  if (e != hipSuccess) return hip_fail(e, "Gram readback");
  return FIT_OK;
}

int fit_set_tuning(fit_grid* g, int path, int tw, int ty, int kc) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (path < 0 || path > 2) return fail(FIT_E_INVALID, "path must be 0 (auto), 1 (split), 2 (fused)");
  if (path == 2 && !fused_ok(g)) return fail(FIT_E_INVALID, "the fused step needs a uniform mu");
  const bool fused = path == 2 || (path == 0 && fused_ok(g));
  const bool expl = tw != 0 || ty != 0 || kc != 0;
  if (expl && tw == 0) tw = 64;
  if (expl) {
    if (fused) {
      if (!valid_tw(tw)) return fail(FIT_E_INVALID, "tw must be 32, 64, 128 or 256 for the fused step");
      if (ty < 2 || ty > 16 || (ty & (ty - 1)) != 0 || tw * ty > 1024)
        return fail(FIT_E_INVALID, "ty must be a power of two in [2, 16] with tw * ty <= 1024");
      if (step_lds_bytes(ty, g->esz, g->lossy, tw, g->nu ? g->d.nz + 1 : 0) > 160 * 1024)
        return fail(FIT_E_INVALID, "tile needs more LDS than a CU has");
    } else {
      if (tw != 64) return fail(FIT_E_INVALID, "the split kernels use tw = 64");
      if (ty < 1 || ty > 8 || (ty & (ty - 1)) != 0)
        return fail(FIT_E_INVALID, "ty must be a power of two in [1, 8] for the split path");
    }
    if (kc < 1) return fail(FIT_E_INVALID, "kc must be >= 1");
  }
  g->path = path;
  g->tile_explicit = expl;
  if (expl) {
    if (fused) {
      g->stw = tw;
      g->sty = ty;
      g->skc = std::min(kc, g->d.nz);
    } else {
      g->ty = ty;
      g->kc = std::min(kc, g->d.nz);
    }
  } else {
    default_tiling(g->d, &g->ty, &g->kc);
    default_step_tiling(g->d, g->esz, g->lossy, &g->sty, &g->skc, &g->stw);
  }
  return FIT_OK;
}

int fit_autotune(fit_grid* g, double dt, int reps, int* path, int* tw, int* ty, int* kc,
                 float* ms_best) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (reps < 1 || reps > 1000) return fail(FIT_E_INVALID, "reps must be in [1, 1000]");
  int rc = check_dt(g, dt);
  if (rc) return rc;
  dt = step_dt(g, dt);
  struct Cand { int path, tw, ty, kc; };
  std::vector<Cand> cands;
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  if (fused_ok(g)) {
    const int widths[4] = {32, 64, 128, 256};
    const int heights[4] = {2, 4, 8, 16};
    for (int w : widths) {
      if (w > 2 * g->d.nx && w > 32) continue;        // mostly empty lanes
      for (int t : heights) {
        if (w * t > 1024 || w * t < 128) continue;
        if (step_lds_bytes(t, g->esz, g->lossy, w, g->nu ? g->d.nz + 1 : 0) > 160 * 1024) continue;
        const int per_cu = step_blocks_per_cu(t, g->esz, g->lossy, w);
        if (per_cu <= 0) continue;
        const int64_t tiles = (int64_t)((g->d.nx + w - 1) / w) * ((g->d.ny + t - 1) / t);
        for (int mult = 1; mult <= 2; ++mult) {
          const int64_t nkc = std::max<int64_t>(1, mult * (int64_t)cus * per_cu / tiles);
          const int k = std::min<int>(g->d.nz, std::max<int>(std::min(8, g->d.nz),
                                                           (int)((g->d.nz + nkc - 1) / nkc)));
          bool dup = false;
          for (const Cand& c : cands) dup |= (c.path == 2 && c.tw == w && c.ty == t && c.kc == k);
          if (!dup) cands.push_back({2, w, t, k});
        }
      }
    }
  }
  {
    int t, k;
    default_tiling(g->d, &t, &k);
    cands.push_back({1, 64, t, k});
    cands.push_back({1, 64, t, std::min(g->d.nz, 4 * k)});
  }
  float best = 1e30f;
  Cand bc = cands[0];
  for (const Cand& c : cands) {
    float ms = 0.f;
    rc = g->f64 ? time_candidate<double>(g, dt, c.path, c.tw, c.ty, c.kc, reps, &ms)
                : time_candidate<float>(g, dt, c.path, c.tw, c.ty, c.kc, reps, &ms);
    if (rc) return rc;
    if (ms < best) {
      best = ms;
      bc = c;
    }
  }
  rc = fit_set_tuning(g, bc.path, bc.tw, bc.ty, bc.kc);
  if (rc) return rc;
  // two steps per launch: take it when a pair beats two single steps
  g->pair_on = 0;
  if (use_fused(g) && g->d.nz >= 2) {
    const int shapes[5][2] = {{32, 16}, {64, 8}, {32, 8}, {48, 8}, {64, 16}};
    float best_pair = 1e30f;
    int bw = 0, bt = 0, bk = 0;
    for (const auto& sh : shapes) {
      const int k0 = pair_kc(g, sh[0], sh[1]);
      if (!step2_shape_ok(sh[0], sh[1], g->esz, g->lossy, g->nu)) continue;
      const int kcs[2] = {k0, std::max(std::min(8, g->d.nz), k0 / 2)};
      for (int q = 0; q < 2; ++q) {
        if (q == 1 && kcs[1] == kcs[0]) continue;
        float ms = 0.f;
        rc = g->f64 ? time_pair<double>(g, dt, sh[0], sh[1], kcs[q], reps, &ms)
                    : time_pair<float>(g, dt, sh[0], sh[1], kcs[q], reps, &ms);
        if (rc) return rc;
        if (ms < best_pair) {
          best_pair = ms;
          bw = sh[0];
          bt = sh[1];
          bk = kcs[q];
        }
      }
    }
    if (bw > 0 && 0.5f * best_pair < 0.98f * best) {
      g->pair_on = 1;
      g->ptw = bw;
      g->pty = bt;
      g->pkc = bk;
      best = 0.5f * best_pair;
    }
  }
  if (path) *path = bc.path;
  if (tw) *tw = bc.tw;
  if (ty) *ty = bc.ty;
  if (kc) *kc = bc.kc;
  if (ms_best) *ms_best = best;
  return FIT_OK;
}

int fit_set_pair_tuning(fit_grid* g, int enable, int tw, int ty, int kc) {
  if (!g) return fail(FIT_E_INVALID, "null handle");
  if (enable != 0 && enable != 1) return fail(FIT_E_INVALID, "enable must be 0 or 1");
  if (kc < 0) return fail(FIT_E_INVALID, "kc must be >= 0");
  if (tw == 0 && ty == 0) {   // the first default tile that fits this dtype
    const int shapes[4][2] = {{64, 8}, {32, 16}, {32, 8}, {16, 8}};
    tw = 64;
    ty = 16;
    for (const auto& sh : shapes)
      if (step2_shape_ok(sh[0], sh[1], g->esz, g->lossy)) {
        tw = sh[0];
        ty = sh[1];
        break;
      }
  }
  if (!step2_shape_ok(tw, ty, g->esz, g->lossy))
    return fail(FIT_E_INVALID, "unsupported tile for the step pair (tw >= 8, ty >= 2, at most 1024 "
                               "threads with one point each or 768 with two, LDS <= 160 KiB)");
  g->pair_on = enable;
  g->ptw = tw;
  g->pty = ty;
  g->pkc = std::min(kc, g->d.nz);
  return FIT_OK;
}

int fit_get_pair_tuning(const fit_grid* g, int* enable, int* tw, int* ty, int* kc) {
  if (!g || !enable || !tw || !ty || !kc) return fail(FIT_E_INVALID, "null argument");
  *enable = g->pair_on;
  *tw = g->ptw;
  *ty = g->pty;
  *kc = g->pkc > 0 ? g->pkc : pair_kc(g, g->ptw, g->pty);
  return FIT_OK;
}

int fit_get_tuning(const fit_grid* g, int* path, int* tw, int* ty, int* kc) {
  if (!g || !path || !tw || !ty || !kc) return fail(FIT_E_INVALID, "null argument");
  const bool fused = use_fused(g);
  *path = fused ? 2 : 1;
  *tw = fused ? g->stw : 64;
  *ty = fused ? g->sty : g->ty;
  *kc = fused ? g->skc : g->kc;
  return FIT_OK;
}

int fit_smvp_count(const fit_grid* g, int64_t* count) {
  if (!g || !count) return fail(FIT_E_INVALID, "null argument");
  *count = g->smvp;
  return FIT_OK;
}

}  // extern "C"
