// Host-side handle definition and helpers shared by the C-ABI source files.
#pragma once

#include <string>
#include <vector>

#include "fit.h"
#include "fit_internal.hpp"

// Adjoint workspace: reverse state and per-edge FP64 sensitivities.
struct fit_adjoint_ws {
  int64_t N = 0;          // forward horizon (steps)
  double dt = 0.0;
  int64_t next_m = -1;    // reverse step expected next (N-1 down to 0)
  void* lam[2] = {nullptr, nullptr};   // 3n each, grid dtype; ping-pong
  void* mu[2] = {nullptr, nullptr};
  bool borrowed = false;  // lam, mu and gcell come from fit_adjoint_bind
  int cur = 0;            // buffer set holding lambda^(m+2), mu^(m+3/2)
  double* gcell = nullptr;  // 2n: per-cell dJ/deps_r, dJ/dsigma accumulators
  fit::Tiling t{};        // tile of the reverse-step kernel
};

struct fit_grid {
  fit_grid_desc desc{};
  fit::Dims d{};
  hipStream_t s = nullptr;
  int dev = 0;                   // HIP device current at creation
  bool f64 = false;
  size_t esz = 4;
  void* e = nullptr;     // 3 * n field values, slot layout
  void* h = nullptr;
  void* eps = nullptr;   // eps0 * eps_r per cell (field dtype)
  void* sig = nullptr;   // sigma per cell, allocated when some sigma != 0
  void* imu = nullptr;   // 1/(mu0 mu_r) per cell, allocated when mu is not uniform
  // storage borrowed from the caller (fit_bind_fields, fit_bind_materials):
  // never freed by the library.  The flags travel with the pointers when the
  // two field buffer sets swap roles.
  bool bor_e = false, bor_h = false, bor_ealt = false, bor_halt = false;
  bool bor_mat = false;          // eps, sig and imu all borrowed
  int64_t storage_version = 0;   // bumped whenever a buffer pointer changes
  double last_dt = 0.0;          // dt of the last fit_step / fit_step_record (0: none)
  bool lossy = false;
  bool mu_uniform = true;
  double imu_u = 1.0;
  double cfl = 0.0;
  // the caller's per-cell inputs (re-applied when the cell widths change)
  std::vector<double> in_eps, in_mu, in_sig;
  // tensor grid with per-axis cell widths (fit_set_spacing)
  bool nu = false;
  std::vector<double> wd[3];
  // device, 4 (nx + ny + nz) doubles: squared widths [x | y | z], then the
  // widths, the dual half-sums (d[i-1] + d[i]) / 2 (d[0] / 2 at i = 0) and the
  // reciprocal widths
  double* sq = nullptr;
  bool mu_value_uniform = true;  // all mu_r equal (also on a tensor grid)
  // two steps per pass (fit_set_pair_tuning)
  int pair_on = 0;
  int ptw = 64, pty = 16, pkc = 0;
  double imu_value = 1.0;        // 1 / (mu0 mu_r) of the first cell
  int64_t materials_version = 0;
  double gedge[3] = {1, 1, 1};   // d_b d_c / d_a
  double gf2[3] = {0.5, 0.5, 0.5};
  int src_axis = -1;
  int64_t src_idx = -1;
  double i_max = 0.0, sigma_t = 1.0;
  int64_t m = 0;
  int64_t smvp = 0;              // curl applications performed (2 per step)
  double* part = nullptr;
  int64_t part_rows = 0;
  double* trace = nullptr;
  int64_t trace_every = 0, trace_cap = 0, trace_rows = 0, trace_dropped = 0;
  int64_t trace_m0 = 0;          // step counter when the trace was configured
  double* pend = nullptr;        // h cross term waiting for the next trace row
  int64_t pend_m = -1;
  double* jacc = nullptr;        // [0..1] probe (sum, comp), [2..3] energy scratch
  fit::Probe probe{};
  int ty = 4, kc = 64;          // split half-step kernels
  int sty = 8, skc = 64;        // fused step kernel
  int stw = 64;                 // fused step tile width
  int path = 0;                 // FIT_PATH_*: 0 auto, 1 split, 2 fused
  bool tile_explicit = false;   // tile shape set by fit_set_tuning
  void* e_alt = nullptr;        // second buffer set of the fused (ping-pong) step
  void* h_alt = nullptr;
  fit_adjoint_ws* adj = nullptr;
  int atw = 0, aty = 0, akc = 0;   // reverse-step tile (0: default)
  double* pacc = nullptr;       // probe objective: per-workgroup (sum, compensation) rows
  int64_t pacc_rows = 0;
  void* xw = nullptr;            // operator / exponential workspace: 3 (e, h) vectors
  void* lw = nullptr;            // Leja workspace: 5 (e, h) vectors
  double* gram_part = nullptr;  // per-workgroup Gram blocks
  double* gram_G = nullptr;     // device K x K result
  int64_t gram_G_cap = 0;
  double* gram_w[2] = {nullptr, nullptr};   // Gram row weights (M_eps, M_mu), 3 n each
  bool gram_w_ok[2] = {false, false};       // weights match the current materials
  // kernel timing (fit_profile_begin/end)
  std::vector<hipEvent_t> prof_ev;   // 2 per timed launch
  std::vector<int> prof_kind;
  int64_t prof_used = 0;
  bool prof_on = false;
};

namespace fit {

// Device scratch g->jacc: [0..1] probe objective (sum, compensation),
// [kJaccWork, +12) the inner products fit_energy combines, [kJaccOut, +5) its
// five results.
constexpr int kJaccWork = 2;
constexpr int kJaccOut = 14;
constexpr int kJaccLen = 24;
// Energy entry points (fit_api.cpp): partial rows needed, and the enqueue of
// the five energies into device `out` (part: energy_rows rows; work: 12
// doubles; the second field buffer set must exist; allocates nothing).
int64_t energy_rows(const fit_grid* g);
int energy_enqueue(fit_grid* g, double* part, double* work, double* out);

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
int dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void*& p);
int ensure_part(fit_grid* g, int64_t rows);
int ensure_pacc(fit_grid* g, int64_t rows);
// The per-axis squared-width pointers of a tensor grid, or nulls.
void set_metric(const fit_grid* g, const double* sq[3]);
double source_value(const fit_grid* g, double dt, int64_t m);
// Step m records a trace row: m - m0 is a multiple of the trace interval
// (m0: the step counter when the trace was configured).
bool trace_at(const fit_grid* g, int64_t m);
int check_dt(const fit_grid* g, double dt);
// The step a grid advances with: dt itself for FP64 grids; for FP32 grids
// the largest FP32 value <= dt, so that the stencil coefficients (exact
// multiples of it on a uniform unit grid) and the source times describe one
// and the same leapfrog step.
double step_dt(const fit_grid* g, double dt);
template <typename T>
int step_once(fit_grid* g, double dt, const T* ein, T* eout, const T* hin, T* hout);
// Frees adjoint/other optional workspaces (defined with those features).
void grid_release_extras(fit_grid* g);
bool use_fused(const fit_grid* g);
void default_step_tiling(const Dims& d, size_t esz, bool lossy, int* ty, int* kc, int* tw);
template <typename T>
int step_fused(fit_grid* g, double dt);
template <typename T>
int step_fused_io(fit_grid* g, double dt, const T* e0, const T* h0, T* e1, T* h1);
int ensure_alt(fit_grid* g);
// Swap the roles of the two field buffer sets (and their borrowed flags).
void swap_sets(fit_grid* g);
void default_tiling(const Dims& d, int* ty, int* kc);

// Bracket one kernel launch with timing events when profiling is on.
struct ProfScope {
  fit_grid* g;
  int64_t slot;
  ProfScope(fit_grid* g_, int kind);
  ~ProfScope();
};

}  // namespace fit
