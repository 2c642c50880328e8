/*
 * fit.h -- C ABI of the MI355X FIT leapfrog library (libfit.so).
 *
 * The library advances the semi-discrete Maxwell system obtained by the
 * Finite Integration Technique on a staggered hexahedral grid pair with the
 * leapfrog scheme, and evaluates the discrete energy inner products
 * (Merkel, Niyonzima, Schoeps, "ParaExp using Leapfrog as Integrator for
 * High-Frequency Electromagnetic Simulations", Sec. II and II-A).
 *
 * Conventions common to every call
 * --------------------------------
 * Grid.   nx, ny, nz count primal CELLS (the paper counts grid points; points
 *         = cells + 1 per axis).  Node (i, j, k) has 0 <= i <= nx, etc.
 *         Spacings dx, dy, dz are uniform per axis.
 * Units.  eps0 and mu0 scale the per-cell relative values (0 selects 1, i.e.
 *         normalised units with c = 1).
 * Field layout ("slot layout").  A field is 3 component arrays, each of
 *         nx*ny*nz elements, stored back to back: element [a][k][j][i]
 *         (i fastest) holds the voltage of the direction-a primal edge (for e)
 *         or of the dual edge crossing the direction-a primal facet (for h)
 *         anchored at node (i, j, k).  Every edge and facet that is not in a
 *         PEC wall has a slot; all other slots are zero.  The step kernels
 *         (single, pair, split, batched) write them as zero and, like the
 *         energies and the Gram matrix, never read them as data: values a
 *         caller leaves there, NaN included, reach none of these results.
 *         e lives on edges with (for a = x) 1 <= j <= ny-1, 1 <= k <= nz-1
 *         (cyclically for y, z); h on facets with 1 <= i <= nx-1 (for a = x).
 * Boundary. Perfect electric conductor on all six faces (tangential e = 0,
 *         normal b = 0), the only boundary used in the paper.
 * Dtype.  Fields and stencils run in FIT_F32 or FIT_F64; every reduction
 *         (energies, probe objective, Gram entries, adjoint gradients)
 *         accumulates in FP64 with compensated summation.
 * Memory. The large device buffers -- both field buffer sets, the per-cell
 *         material arrays and the adjoint state -- can be storage of the
 *         caller's (e.g. PyTorch tensors) that the library borrows by pointer
 *         (fit_bind_fields, fit_bind_materials, fit_adjoint_bind) and never
 *         frees; the caller keeps them alive until they are unbound or the
 *         handle is destroyed.  Unbound roles are allocated (hipMalloc) and
 *         owned by the library, as are the small reduction scratch (partial
 *         sums, trace rows, probe rows) and the optional workspaces of the
 *         Gram and exponential entry points.  Other pointers passed in are
 *         borrowed for the duration of the call only.  "device" pointers must
 *         be device memory of the current HIP device; "host" pointers
 *         ordinary host memory.
 * Streams. All work is enqueued on the stream given at creation (NULL =
 *         the default stream).  Calls that return host data synchronise that
 *         stream; the others return once the work is enqueued.
 * Errors. Every call returns a fit_status; nothing throws across the ABI.
 *         fit_last_error() returns a thread-local message for the last
 *         non-OK status.  A HIP failure (launch error, sticky device error)
 *         surfaces as FIT_E_HIP on the call that observes it.
 * Threads. A handle must not be used from two threads at once.
 */
#ifndef FIT_H
#define FIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FIT_OK = 0,
  FIT_E_INVALID = -1,   /* bad argument (sizes, pointers, non-SPD material, ...) */
  FIT_E_OOM = -2,       /* device allocation failed */
  FIT_E_HIP = -3,       /* HIP runtime / kernel error */
  FIT_E_UNSTABLE = -4,  /* dt above the CFL bound without FIT_ALLOW_UNSTABLE */
  FIT_E_DIVERGED = -5,  /* energy watchdog: non-finite energy */
  FIT_E_STATE = -6      /* call not valid in the handle's current state */
} fit_status;

typedef enum { FIT_F32 = 0, FIT_F64 = 1 } fit_dtype;

enum { FIT_ALLOW_UNSTABLE = 1u };

typedef struct fit_grid fit_grid;   /* opaque handle */

typedef struct {
  int32_t nx, ny, nz;     /* cells per axis, each >= 1 */
  double dx, dy, dz;      /* uniform spacings, > 0 (0 selects 1) */
  double eps0, mu0;       /* vacuum constants, >= 0 (0 selects 1) */
  int32_t dtype;          /* fit_dtype */
  uint32_t flags;         /* FIT_ALLOW_UNSTABLE */
} fit_grid_desc;

/* Number of doubles per energy-trace row; see fit_trace_read. */
#define FIT_TRACE_COLS 10

/* Library version string (static storage). */
const char* fit_version(void);

/* Thread-local message describing the last non-OK status. */
const char* fit_last_error(void);

/* Create a grid: staggered primal/dual grid of nx*ny*nz cells (Sec. II).
 * Fields start at zero, materials at vacuum (eps_r = mu_r = 1, sigma = 0),
 * no source, step counter 0.  `stream` is a hipStream_t or NULL.
 * Errors: FIT_E_INVALID (sizes/spacings), FIT_E_OOM. */
int fit_grid_create(const fit_grid_desc* desc, void* stream, fit_grid** out);

/* Destroy a grid and free its device memory (synchronises its stream).
 * NULL is accepted. */
int fit_grid_destroy(fit_grid* g);

/* Per-cell materials -> the diagonal material matrices M_eps, M_sigma, M_mu
 * (eq. maxwell_grid3).  Host FP64 arrays of nx*ny*nz values, layout
 * [k][j][i].  mu_r may be NULL (all 1), sigma may be NULL (all 0).
 * The edge/facet averages are formed inside the kernels: M_eps of an edge is
 * eps0 times the mean eps_r of the (up to 4) cells around it times
 * d_b d_c / d_a; M_sigma likewise; M_mu^{-1} of a facet is the mean of
 * 1/(mu0 mu_r) over the 2 cells on its dual edge times d_a / (d_b d_c).
 * Errors: FIT_E_INVALID if eps_r <= 0, mu_r <= 0, sigma < 0 or non-finite. */
int fit_set_materials(fit_grid* g, const double* eps_r, const double* mu_r,
                      const double* sigma);

/* Per-axis cell widths of a tensor grid (non-uniform spacing; Sec. II with
 * the per-cell dimensions of eq. cfl): dx[nx], dy[ny], dz[nz] host FP64
 * arrays of positive finite widths, replacing the descriptor's uniform
 * spacing.  All three NULL returns to the descriptor's spacing.  The current
 * materials are re-applied: an a-edge with index i along a gets M_eps =
 * eps0 sum_c eps_r[c] (d_b[c] d_c[c] / 4) / d_a[i] over its <= 4 cells, an
 * a-facet M_mu^{-1} = sum_c (d_a[c] / 2) / (mu0 mu_r[c]) / (d_b d_c) over its
 * 2 cells, and dt_CFL takes each cell's own widths.  On such a grid the
 * device arrays hold cell values times the cell volume; the step runs fused
 * when mu_r is uniform and on the split kernels otherwise; batches, the
 * adjoint and the exponential entry points reject it with FIT_E_INVALID.
 * Errors: FIT_E_INVALID (a width <= 0 or non-finite, some but not all NULL),
 * FIT_E_OOM. */
int fit_set_spacing(fit_grid* g, const double* dx, const double* dy, const double* dz);

/* Gaussian line-current source (Sec. IV-A, eq. line_current):
 * i(t) = i_max exp(-4 ((t - sigma_t) / sigma_t)^2) on the single primal edge
 * of direction `axis` (0, 1, 2) leaving node (i, j, k), flowing in +axis,
 * sampled at t_{m+1/2} = (m + 1/2) dt.  It enters the e-update with a minus
 * sign (M_eps de/dt = C~ h - j).  axis = -1 removes the source.
 * Errors: FIT_E_INVALID if the edge lies in a PEC wall or sigma_t <= 0. */
int fit_set_source(fit_grid* g, int axis, int i, int j, int k, double i_max,
                   double sigma_t);

/* CFL step bound (eq. cfl): min over cells of
 * sqrt(eps mu / (dx^-2 + dy^-2 + dz^-2)).  Writes *dt_cfl. */
int fit_cfl_dt(const fit_grid* g, double* dt_cfl);

/* Borrow caller-owned device storage for the fields (initial values and the
 * leapfrog recurrence of Sec. II-A live there).  e, h: the buffers of the
 * state (e^(m), h^(m+1/2)); e_alt, h_alt: the second buffer set the fused and
 * two-step kernels write (both NULL: the library allocates its own on first
 * use).  Each is 3*nx*ny*nz elements of the grid's dtype in the slot layout,
 * 16-byte aligned, and no two overlap.  The current state is copied into
 * (e, h), so binding does not change it.  The two sets swap roles as steps
 * run: fit_get_state tells which buffers hold the state; the other set's
 * contents are scratch between calls.  All four NULL returns the state to
 * library-owned buffers (do this before freeing bound storage while the
 * handle lives).  Synchronises.  Errors: FIT_E_INVALID (only one of e, h or
 * of e_alt, h_alt given, misaligned or overlapping buffers, a buffer the
 * library owns), FIT_E_OOM. */
int fit_bind_fields(fit_grid* g, void* e, void* h, void* e_alt, void* h_alt);

/* Borrow caller-owned device storage for the per-cell material arrays the
 * kernels read (M_eps, M_sigma, M_mu^{-1} are formed from them, eq.
 * maxwell_grid3): eps, sigma and imu, each nx*ny*nz elements of the grid's
 * dtype, 16-byte aligned, disjoint.  The current materials are written into
 * them now and by every later fit_set_materials / fit_set_spacing (eps0 eps_r,
 * sigma and 1/(mu0 mu_r) per cell, times the cell volume on a tensor grid;
 * sigma and imu are written only when some sigma != 0 or mu varies).  All
 * three NULL returns to library-owned arrays.  Synchronises.
 * Errors: FIT_E_INVALID, FIT_E_OOM. */
int fit_bind_materials(fit_grid* g, void* eps, void* sigma, void* imu);

/* Device pointers of the buffers holding the current state e^(m),
 * h^(m+1/2) (bound or library-owned; valid until the next call that steps
 * or rebinds). */
int fit_get_state(const fit_grid* g, void** e, void** h);

/* The step the grid advances with when asked for dt (fit_step): dt itself
 * for FP64 grids, the largest FP32 value <= dt for FP32 grids.  Host only. */
int fit_step_dt(const fit_grid* g, double dt, double* dt_used);

/* Set the state e^(m), h^(m+1/2) and the step counter m.  e, h: 3*nx*ny*nz
 * values each in the slot layout and the grid's dtype; on_device != 0 means
 * device pointers, else host pointers.  Either pointer may be NULL (that
 * field is zeroed).  Slots of PEC-wall edges/facets are forced to zero. */
int fit_set_fields(fit_grid* g, const void* e, const void* h, int64_t step, int on_device);

/* Copy the current state out (layouts as fit_set_fields).  Either pointer
 * may be NULL.  Host destinations synchronise. */
int fit_get_fields(fit_grid* g, void* e, void* h, int on_device);

/* Current step counter m (the state holds e^(m), h^(m+1/2)). */
int fit_get_step(const fit_grid* g, int64_t* step);

/* Apply one PEC-restricted discrete curl: which = 0 applies the primal curl
 * C (edge voltages -> facet fluxes, eq. maxwell_grid1: C e = -d_t b); which =
 * 1 applies the dual curl C~ (dual-edge voltages -> dual-facet quantities,
 * C~ h = d_t d + j).  in/out: device pointers, slot layout, grid dtype;
 * in != out.  Output slots in PEC walls are zero. */
int fit_apply_curl(fit_grid* g, int which, const void* in, void* out);

/* Advance nsteps leapfrog steps (Sec. II-A):
 *   (M_eps + dt/2 M_sigma) e^(m+1) = (M_eps - dt/2 M_sigma) e^m + dt (C~ h^(m+1/2) - j_s(t_{m+1/2}))
 *   h^(m+3/2) = h^(m+1/2) - dt M_mu^{-1} C e^(m+1)
 * (the loss current is taken at the interpolated e^(m+1/2) = (e^m + e^(m+1))/2;
 * for sigma = 0 this is the paper's update).  Cost: 2 curl applications per
 * step (eq. cost_LF).  dt must be > 0 and <= fit_cfl_dt unless the grid was
 * created with FIT_ALLOW_UNSTABLE (else FIT_E_UNSTABLE).  An FP32 grid
 * advances with dt rounded down to the nearest FP32 value: its stencil
 * coefficients are FP32, and the source times t_(m+1/2) use the same step,
 * so the run is the leapfrog recurrence of that step (an unrepresented
 * remainder of dt would otherwise act as a systematic time-step error whose
 * phase drift grows linearly with the step count).  The same holds for
 * fit_step_record, fit_adjoint_begin, fit_autotune and batched steps.
 * Energies are traced as configured by fit_trace_config; the probe objective
 * is accumulated when a probe is set.  Asynchronous. */
int fit_step(fit_grid* g, int64_t nsteps, double dt);

/* Energies of the current state e^m, h^(m+1/2) (eq. energy), FP64:
 *   out[0] = <e^m, e^m>_eps,   out[1] = <h^(m+1/2), h^(m+1/2)>_mu,
 *   out[2] = W^m = <e^m, (e^m + e^(m+1))/2>_eps + <(h^(m-1/2) + h^(m+1/2))/2, h^(m+1/2)>_mu,
 *            the energy the lossless, source-free recurrence conserves,
 *   out[3] = Q^m = <e^m, e^m>_eps + <h^(m-1/2), h^(m+1/2)>_mu,
 *   out[4] = Q^(m+1) - Q^m = -2 dt ebar . (M_sigma ebar + j_s(t_(m+1/2))),
 *            ebar = (e^m + e^(m+1))/2: the exact discrete energy balance of
 *            the step that starts at the current state (0 when lossless and
 *            source-free).
 * e^(m+1) is the e-update of the current state and h^(m-1/2) the h-update run
 * backwards (h^(m+1/2) + dt M_mu^{-1} C e^m), both formed in the second field
 * buffer set with dt of the handle's last fit_step or fit_step_record; before
 * any step out[2..4] are NaN.  Synchronises.  Returns FIT_E_DIVERGED (with out
 * filled) if out[0] or out[1] is not finite. */
int fit_energy(fit_grid* g, double out[5]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the five
 * values of fit_energy written to out (a DEVICE pointer to 5 doubles) on the
 * handle's stream, with no allocation, no memset and no synchronisation.
 * The partial sums go to a fixed array of the library on the handle's
 * device (640 KiB, held until the process ends, shared by every call on that
 * device: calls that overlap on one device race).  Limits: the grid's
 * partial-sum rows (at most 4096 for the energy kernel, and the workgroups of
 * the half-step kernels' tiling) must not exceed 8192 (else FIT_E_INVALID);
 * the second field buffer set must already exist (bound with
 * fit_bind_fields or allocated by an earlier step; else FIT_E_STATE).
 * Values equal fit_energy's bitwise.  The first call on a device looks up the
 * array's device address. */
int fit_energy_noalloc(fit_grid* g, double* out);

/* Energy trace.  every > 0 records one row for each step m with
 * (m - m0) % every == 0, m0 the step counter at this call (every = 0
 * disables); up to `capacity` rows are kept
 * (later rows are dropped and counted).  The row of step m holds the inner
 * products available around that step (FP64):
 *   [0] m
 *   [1] <e^m, e^m>_eps        [2] <e^m, e^(m+1)>_eps     [3] <e^(m+1), e^(m+1)>_eps
 *   [4] <h^(m-1/2), h^(m+1/2)>_mu (NaN if step m-1 was not run in this handle)
 *   [5] <h^(m+1/2), h^(m+1/2)>_mu   [6] <h^(m+1/2), h^(m+3/2)>_mu   [7] <h^(m+3/2), h^(m+3/2)>_mu
 *   [8] ebar^T M_sigma ebar   [9] ebar . j_s,   ebar = (e^m + e^(m+1))/2.
 * From these, the paper's conserved energy is W^m = ([1]+[2]+[4]+[5])/2, and
 * Q^(m+1) - Q^m = -2 dt ([8] + [9]) with Q^m = [1] + [4], Q^(m+1) = [3] + [6].
 * Reconfiguring clears recorded rows. */
int fit_trace_config(fit_grid* g, int64_t every, int64_t capacity);

/* Copy up to max_rows recorded rows (FIT_TRACE_COLS doubles each) to host
 * `out`, write the number copied to *nrows and the number dropped for lack of
 * capacity to *dropped (may be NULL), then clear the record.  Synchronises. */
int fit_trace_read(fit_grid* g, double* out, int64_t max_rows, int64_t* nrows,
                   int64_t* dropped);

/* Probe objective J = dt * sum over steps m >= 1 of sum_{edges i in probe}
 * M_eps,i (e_i^m)^2, accumulated by fit_step (FP64, compensated).  The probe
 * holds the edges whose midpoints lie in the closed node-coordinate box
 * [lo[a], hi[a]] for a = x, y, z.  Setting the probe resets J to 0;
 * lo = hi = NULL removes it. */
int fit_set_probe(fit_grid* g, const int32_t lo[3], const int32_t hi[3]);

/* Read the probe objective accumulated so far (synchronises). */
int fit_probe_value(fit_grid* g, double* J);

/* Reset the probe objective to 0. */
int fit_probe_reset(fit_grid* g);

/* Mode-Gram energy matrix (the bilinear form of eq. energy over snapshots):
 * G[a][b] = sum_r M_rr x_a[r] x_b[r] for K snapshots x_0 .. x_{K-1}, with
 * M = M_eps (which = 0, x are e-fields) or M = M_mu (which = 1, h-fields)
 * of this grid's materials.  X: device pointer, snapshot a at X + a * ld
 * elements, each in the slot layout and the grid's dtype (ld >= 3 nx ny nz);
 * PEC-wall and phantom slots carry weight 0 and their values are ignored
 * (non-finite values there do not reach G).  Computed on the FP64 matrix cores with
 * FP64 accumulation inside a workgroup and compensated summation across
 * workgroups.  G: host, K * K doubles row-major, exactly symmetric.
 * 1 <= K <= 4096.  Synchronises. */
int fit_gram(fit_grid* g, const void* X, int64_t ld, int K, int which, double* G);

/* ---- Differentiation: discrete reverse-time adjoint of fit_step ----------
 * The objective is the probe energy J of fit_set_probe accumulated over a
 * forward run of N steps from step 0.  The adjoint recursion (lambda = dJ/de,
 * mu = dJ/dh, zero beyond the horizon), for m = N-1 down to 0:
 *   lambda^(m+1) = a lambda^(m+2) - C~ (dt M_mu^{-1} mu^(m+3/2)) + 2 dt w M_eps e^(m+1)
 *   mu^(m+1/2)   = mu^(m+3/2) + C (b lambda^(m+1))
 * with a, b the e-update coefficients of fit_step; it differentiates the
 * leapfrog updates of Sec. II-A exactly (dt held fixed).  Each reverse step
 * is one fused pass; its edge sensitivities to M_eps and M_sigma go straight
 * onto the per-cell eps_r and sigma gradients (FP64 accumulators), read by
 * fit_adjoint_grad.  Needs a uniform mu and a probe. */

/* Advance nsteps leapfrog steps like fit_step, recording every state:
 * e_rec + s * 3n holds e^(m0+s) and h_rec + s * 3n holds h^(m0+s+1/2) for
 * s = 0 .. nsteps (device pointers, (nsteps+1) * 3 * nx*ny*nz elements each,
 * grid dtype, slot layout); m0 is the step counter on entry.  The handle ends
 * in state m0 + nsteps.  No energy trace and no probe accumulation. */
int fit_step_record(fit_grid* g, int64_t nsteps, double dt, void* e_rec, void* h_rec);

/* Tile of the reverse-step kernel, used from the next fit_adjoint_begin:
 * tw x ty columns (tw ty + tw + ty + 1 <= 512 threads: the tile and its halo
 * points), kc z-planes per workgroup; tw = ty = 0 and kc = 0 select the
 * defaults (a width that wastes the fewest lanes, chunks for one round of
 * resident workgroups).  Errors: FIT_E_INVALID. */
int fit_adjoint_set_tuning(fit_grid* g, int tw, int ty, int kc);

/* The reverse-step tile the next fit_adjoint_begin will use (the one set, or
 * the defaults for this grid and device).  Errors: FIT_E_INVALID. */
int fit_adjoint_get_tuning(const fit_grid* g, int* tw, int* ty, int* kc);

/* Borrow caller-owned device storage for the adjoint state: lam0, lam1,
 * mu0, mu1 (3*nx*ny*nz elements of the grid's dtype each, the ping-pong
 * buffers of lambda and mu) and gcell (2*nx*ny*nz doubles: the per-cell
 * dJ/deps_r and dJ/dsigma accumulators), 16-byte aligned and disjoint.  Ends
 * any reverse sweep in progress; all five NULL returns to library-owned
 * storage at the next fit_adjoint_begin.  Synchronises.
 * Errors: FIT_E_INVALID, FIT_E_OOM. */
int fit_adjoint_bind(fit_grid* g, void* lam0, void* lam1, void* mu0, void* mu1, double* gcell);

/* Start a reverse sweep over a forward horizon of nsteps steps taken with dt:
 * clears lambda, mu and the accumulated sensitivities.  Errors: FIT_E_STATE
 * without a probe, FIT_E_INVALID for a non-uniform mu. */
int fit_adjoint_begin(fit_grid* g, int64_t nsteps, double dt);

/* One reverse step m (must be called for m = N-1, N-2, ..., 0 in order, else
 * FIT_E_STATE) given the forward states e^m, e^(m+1) and h^(m+1/2) (device
 * pointers, slot layout, grid dtype), e.g. recomputed from a checkpoint with
 * fit_step_record.  Asynchronous. */
int fit_adjoint_step(fit_grid* g, int64_t m, const void* e_m, const void* e_m1, const void* h_mh);

/* Reverse steps m0 + nsteps - 1 down to m0 over a recorded segment
 * (e_rec, h_rec as written by fit_step_record starting at m0). */
int fit_adjoint_segment(fit_grid* g, int64_t m0, int64_t nsteps, const void* e_rec,
                        const void* h_rec);

/* Per-cell gradients dJ/deps_r and dJ/dsigma (FP64, nx*ny*nz values each,
 * layout [k][j][i]) of the sensitivities accumulated so far; device or host
 * destinations.  Host destinations synchronise. */
int fit_adjoint_grad(fit_grid* g, double* deps, double* dsigma, int on_device);

/* ---- Matrix exponential and ParaExp building blocks (Sec. III) ----------
 * On the voltages x = (e, h) of a lossless grid with uniform mu the
 * semi-discrete system (eq. FIT_ode_1 without source) is dx/dt = B x,
 *   B (e, h) = ( M_eps^{-1} C~ h ,  -M_mu^{-1} C e ),
 * the similarity transform of the skew matrix A of eq. FIT_ode_2, so
 * exp(tB) x = T^{-1} exp(tA) T x and ||A||_2 is the M-norm of B.  All field
 * arguments are device pointers to 3-component slot-layout arrays of the
 * grid's dtype.  Asynchronous on the grid's stream unless stated. */

/* Taylor parameters (m terms, s sub-steps) for theta = |t| ||A||_2, a
 * relative tolerance tol in (0, 1) and the unit roundoff u of the
 * arithmetic: the fewest applications m s with
 *   s delta (1 + delta)^(s-1) + s (m + 2) u e^(theta / s) <= tol,
 *   delta = (theta / s)^(m+1) / (m+1)!
 * (the Taylor remainder on an imaginary spectrum plus a rounding estimate).
 * FIT_E_INVALID if tol is below what u allows.  Host only. */
int fit_expm_params(double theta, double tol, double unit_roundoff, int* m, int64_t* s);

/* Tolerance of the exponential that balances its backward error against the
 * O(dt^2) leapfrog error of the particular solutions (Sec. III-D, eq.
 * tolerance_leja_2): tol = beta dt^2 / kappa_exp(A), with kappa_exp(A) =
 * ||A||_2 = rho for the normal A of eq. FIT_ode_2.  beta > 0 is the
 * caller's constant of the leapfrog error (the paper leaves it open).
 * FIT_E_INVALID unless beta, dt, rho are positive and finite.  Host only. */
int fit_expm_tolerance(double beta, double dt, double rho, double* tol);

/* out = alpha B in (two curl applications).  Needs a uniform mu; inputs
 * and outputs must be distinct buffers.  Errors: FIT_E_INVALID. */
int fit_op_apply(fit_grid* g, double alpha, const void* e_in, const void* h_in, void* e_out,
                 void* h_out);

/* ||A||_2 estimated by `iters` power iterations on -B^2 in the M inner
 * product from a seeded pseudo-random start (Rayleigh quotients approach the
 * norm from below).  Lossless grids with uniform mu.  Synchronises. */
int fit_op_norm(fit_grid* g, int iters, uint64_t seed, double* rho);

/* (e_out, h_out) = exp(t B) (e_in, h_in) by (T_m(tB/s))^s with (m, s) from
 * fit_expm_params(|t| rho, tol, u) and u the unit roundoff of the grid's
 * dtype (2^-53, 2^-24); rho = ||A||_2 or a bound on it.  m and s (may be
 * null) receive the parameters used (m s applications of B).  In-place
 * (out == in) is allowed.  Lossless grids with uniform mu. */
int fit_expm(fit_grid* g, double t, double tol, double rho, const void* e_in, const void* h_in,
             void* e_out, void* h_out, int* m, int64_t* s);

/* Leja interpolation of exp (Sec. III-A): the interpolant of exp at K
 * conjugate pairs of points +-i c a_j on the imaginary interval i[-c, c],
 * a_j^2 a Leja sequence of [0, 1] (x_0 = 1, then greedy on the grid
 * (1 - cos(pi i / 4000)) / 2), degree 2K - 1.  One step of length h misses
 * exp(hA) by at most delta = max_{tau in [0, c^2]} prod_j |tau - c^2 a_j^2|
 * / (2K)! (remainder on the imaginary axis; c = rho h); (K, s) minimise the
 * applications (2K - 1) s subject to s delta (1 + delta)^(s-1) plus the
 * rounding estimate s (2K + 1) u S <= tol (S from the coefficients and the
 * basis bounds).  K <= 30.  FIT_E_INVALID if tol is below what u allows.
 * Host only. */
int fit_leja_params(double theta, double tol, double unit_roundoff, int* K, int64_t* s);

/* The evaluation coefficients of the K-pair interpolant on i[-c, c] in the
 * basis q_0 = 1, q_(k+1) = (z^2 / g2 + a2[k]) q_k (g2 = max(c/2, 1)^2):
 * p(z) = sum_k (alpha[k] + beta[k] z) q_k.  Arrays of K doubles.  Host only. */
int fit_leja_coefficients(int K, double c, double* alpha, double* beta, double* a2, double* g2);

/* (e_out, h_out) = exp(t B) (e_in, h_in) by s steps of the K-pair Leja
 * interpolant with (K, s) from fit_leja_params(|t| rho, tol, u), u the unit
 * roundoff of the grid's dtype (the parameter search is memoised per
 * process).  In place allowed.  Lossless grids with uniform mu and
 * spacing.  K, s may be null.  Allocates a workspace of five field pairs on
 * first use. */
int fit_expm_leja(fit_grid* g, double t, double tol, double rho, const void* e_in,
                  const void* h_in, void* e_out, void* h_out, int* K, int64_t* s);

/* h_out = h_in - c M_mu^{-1} C e (the h-update with step c; c = -dt/2 turns
 * h^(m+1/2) into the collocated h(t_m) = (h^(m-1/2) + h^(m+1/2))/2 given e^m,
 * c = +dt/2 turns it back).  h_out may equal h_in. */
int fit_shift_h(fit_grid* g, double c, const void* e, const void* h_in, void* h_out);

/* y += a x for two-field vectors (e, h). */
int fit_axpy(fit_grid* g, double a, const void* x_e, const void* x_h, void* y_e, void* y_h);

/* ---- Batched grids: many independent grids advanced together ------------
 * A batch advances nb grids (same dtype, uniform mu each; sizes, materials,
 * sources and dt may all differ) together.  Each launch covers one step of
 * every grid: one workgroup per fused-step tile of every grid (no workgroup
 * waits on another; the kernel boundary orders the steps).  Chunks of S
 * steps are captured once in a hipGraph and replayed.  Each grid's result is
 * bitwise identical to fit_step on that grid alone.  The grids stay usable on
 * their own between batch calls; a batch references them and must be
 * destroyed before them.  Batched steps record no energy trace; a grid with a
 * probe is rejected. */
typedef struct fit_batch fit_batch;

/* Build a batch over nb >= 1 distinct grids; `stream` is the caller's
 * hipStream_t (NULL = default stream); work is ordered after and before it. */
int fit_batch_create(fit_grid* const* grids, int nb, void* stream, fit_batch** out);

/* Destroy a batch (not its grids).  NULL is accepted. */
int fit_batch_destroy(fit_batch* b);

/* Tile of every grid: tw x ty columns with tw in {32, 64, 128, 256} and ty a
 * power of two in [2, 16] (64 <= tw ty <= 1024); or tw = FIT_TW_ROWS:
 * row-packed tiles, ty = threads per workgroup (a multiple of 64 in
 * [128, 1024]) and each grid's tile as wide as its x extent when that fits
 * (else 32..256 wide) with its rows splitting the y extent evenly.  0 keeps
 * tw / ty.  kc: z-planes per item (0 = whole columns); steps per captured
 * launch (0 keeps; default 16).  FIT_E_INVALID (tuning unchanged) if a tile
 * needs more LDS than a workgroup can have. */
enum { FIT_TW_ROWS = -1 };
int fit_batch_set_tuning(fit_batch* b, int tw, int ty, int kc, int steps_per_graph);
int fit_batch_get_tuning(const fit_batch* b, int* tw, int* ty, int* kc, int* steps_per_graph,
                         int* nwg);

/* Two steps of every grid per launch (temporal blocking of the Sec. II-A
 * recurrence, as fit_set_pair_tuning for one grid): with enable = 1 the
 * batch advances pairs of steps with one launch over tiles of every grid;
 * an odd last step runs singly.  Each grid takes the tile shape of a fixed
 * set (32 x 16, 32 x 18, 40 x 14, 24 x 24) that stages the fewest points
 * for its x / y extent, and its columns are cut into ceil(nz / kc) z-chunks
 * of even length (kc = 0: whole columns); the tiles of one z-chunk of one
 * grid are launched onto one XCD (their shared halo rows stay in its L2), the
 * longest first, with the work balanced over the XCDs.  Each grid's result stays bitwise identical to fit_step on
 * that grid alone.  FIT_E_INVALID if no pair tile fits the batch's dtype and
 * materials, or a z-plane of a grid spans more than 4 GiB. */
int fit_batch_set_pair(fit_batch* b, int enable, int kc);
int fit_batch_get_pair(const fit_batch* b, int* enable, int* kc);

/* The pair tile of grid g (0-based, in the order given to fit_batch_create)
 * in the current layout: tw x ty columns, kc planes per z-chunk.
 * FIT_E_INVALID for a bad index, FIT_E_STATE when pairs are off. */
int fit_batch_get_pair_tile(const fit_batch* b, int g, int* tw, int* ty, int* kc);

/* Persistent form of the batch (Sec. III, Alg. 1: the p independent leapfrog
 * runs): with enable = 1, S steps of every grid run in ONE cooperative launch
 * (S = steps_per_graph of fit_batch_set_tuning) whose workgroups -- as many
 * as the device holds at once, at most one per item -- each take items w,
 * w + G, w + 2G, ... of a step's tile table and then meet the whole launch
 * at a grid-wide barrier before the next step.  The S-step launch is
 * captured in a hipGraph and replayed for whole chunks (use_graph != 0; if
 * the runtime cannot capture a cooperative launch, chunks are launched
 * directly), the remainder runs as one launch.  With step pairs on
 * (fit_batch_set_pair), a launch runs S / 2 pairs instead: its workgroups (a
 * multiple of 8, as many as the device holds at once) take entries w,
 * w + G, ... of the pair item table, whose entry r lies on the XCD of
 * workgroup r, and meet at the barrier after every pair; an odd last step
 * runs through the single-step launch.  Each grid's result stays bitwise
 * identical to fit_step on that grid alone.  The barrier polls a device counter; a
 * poll that waits longer than about half a second gives up and flags the
 * call (the launch then ends with wrong fields instead of hanging).  get:
 * enable, the workgroups of the launch, whether the launch is captured, and
 * (synchronising) whether a barrier of the last fit_batch_step gave up; any
 * output may be NULL.  Errors: FIT_E_INVALID if the device cannot launch
 * cooperatively or the tile does not fit. */
int fit_batch_set_persistent(fit_batch* b, int enable);
int fit_batch_get_persistent(const fit_batch* b, int* enable, int* workgroups, int* captured,
                             int* barrier_failed);

/* Autotuner: time candidate (tw, ty, kc), row-packed ones included, with
 * `reps` single-step launches each (state unchanged) and keep the fastest;
 * then time step pairs (kc 6, 8, 12, 16, 24, 32 and whole columns) and
 * switch them on when a pair takes
 * less than 98 % of two single steps (ms_best is then half a pair).
 * dt: host array of nb step sizes. */
int fit_batch_autotune(fit_batch* b, const double* dt, int reps, int* tw, int* ty, int* kc,
                       float* ms_best);

/* Advance every grid of the batch by nsteps steps; dt: host array of nb step
 * sizes (each <= its grid's CFL bound unless that grid allows instability).
 * use_graph != 0 replays the captured S-step graph for whole chunks (the
 * remainder runs as direct launches); 0 launches directly.  Asynchronous with
 * respect to the host; ordered after and before the caller's stream.
 * get_tuning's last output is the number of workgroups per step launch. */
int fit_batch_step(fit_batch* b, int64_t nsteps, const double* dt, int use_graph);

/* Kernel timing.  Between fit_profile_begin and fit_profile_end every
 * kernel launch made by this handle is bracketed by a pair of hipEvents on
 * the handle's stream (at most max_launches launches are timed; later ones
 * run untimed).  fit_profile_end synchronises and writes, per kernel class
 * (FIT_PROF_* index), the summed launch duration in milliseconds to
 * ms[FIT_PROF_N] and the number of timed launches to count[FIT_PROF_N]
 * (either may be NULL); FIT_PROF_PAIR counts step pairs, FIT_PROF_PAIR_ENERGY
 * the pairs that also record a trace row.  This is instrumentation for the paper's cost
 * measure (curl applications, eq. cost_LF) in wall-clock form. */
enum { FIT_PROF_EPASS = 0, FIT_PROF_HPASS = 1, FIT_PROF_REDUCE = 2, FIT_PROF_STEP = 3,
       FIT_PROF_ADJOINT = 4, FIT_PROF_OTHER = 5, FIT_PROF_PAIR = 6, FIT_PROF_PAIR_ENERGY = 7,
       FIT_PROF_N = 8 };
int fit_profile_begin(fit_grid* g, int64_t max_launches);
int fit_profile_end(fit_grid* g, double ms[FIT_PROF_N], int64_t count[FIT_PROF_N]);

/* Streaming probe for the measured HBM ceiling (instrumentation; no step of
 * the method uses it).  mode 0: copy `bytes` from src to dst; mode 1: read
 * src (dst receives blocks * 256 floats of per-lane sums, which keeps the
 * loads alive); mode 2: fill dst.  16-byte accesses by consecutive lanes,
 * four in flight per lane, `blocks` workgroups of 256 threads striding over
 * the buffer, non-temporal loads and stores.  bytes: a positive multiple of
 * 16; device pointers, 16-byte aligned, src and dst disjoint.  Enqueued on
 * `stream` (a hipStream_t or NULL).  Errors: FIT_E_INVALID, FIT_E_HIP. */
int fit_stream_probe(int mode, void* dst, const void* src, int64_t bytes, int blocks,
                     void* stream);

/* Kernel path and tile shape of fit_step.  path: FIT_PATH_AUTO (fused
 * single-pass kernel when mu is uniform, else the two half-step kernels),
 * FIT_PATH_SPLIT (e-update and h-update kernels, in place) or FIT_PATH_FUSED
 * (one kernel per step, state ping-pongs between two buffer sets; needs a
 * uniform mu).  tw x ty: column tile (fused: tw in {32, 64, 128, 256}, ty a
 * power of two in [2, 16], tw ty <= 1024; split: tw = 64, ty in {1..8});
 * kc: z-planes per workgroup; tw = ty = kc = 0 selects the path's default.
 * Every path and tile computes the same values (bitwise: the per-node
 * arithmetic is shared).  Errors: FIT_E_INVALID. */
enum { FIT_PATH_AUTO = 0, FIT_PATH_SPLIT = 1, FIT_PATH_FUSED = 2 };
int fit_set_tuning(fit_grid* g, int path, int tw, int ty, int kc);

/* The path fit_step will take and its tile shape. */
int fit_get_tuning(const fit_grid* g, int* path, int* tw, int* ty, int* kc);

/* Two leapfrog steps per pass (temporal blocking of the Sec. II-A
 * recurrence): with enable = 1, fit_step advances pairs of steps with one
 * launch that reads the state and the materials once and keeps the
 * intermediate state on chip, whenever the fused path is active (uniform
 * mu; uniform or tensor-product spacing), no probe is set, the first step
 * of the pair is no trace row and the step after it needs no h cross term
 * for one (a trace row m+2), the tile fits the grid's materials and a
 * z-plane of the grid spans at most 4 GiB (other steps run singly).  A pair
 * whose second step is a trace row records the row itself (uniform spacing,
 * tiles of one point per thread: the FP64 compensated energy terms of eq.
 * energy formed in the pair, the row's pending h cross term from its first
 * step), equal to the single-step row up to the summation order; on a
 * tensor grid or a two-point tile that step runs singly.
 * The fields are bitwise those of single fused steps.  tw x ty: tile (tw >= 8,
 * ty >= 2; a workgroup has (tw + 4)(ty + 3) threads rounded up to a multiple
 * of 64, at most 1024; LDS within 160 KiB), kc: planes per chunk (0 = one
 * round of resident workgroups); tw = ty = 0 takes the first of 64 x 8,
 * 32 x 16, 32 x 8, 16 x 8 that fits the dtype.
 * Errors: FIT_E_INVALID for an unsupported tile. */
int fit_set_pair_tuning(fit_grid* g, int enable, int tw, int ty, int kc);
/* The pair setting in effect (kc: the chunk a launch would use). */
int fit_get_pair_tuning(const fit_grid* g, int* enable, int* tw, int* ty, int* kc);

/* Autotuner: time candidate kernel paths and tile shapes (tile heights,
 * z-chunks sized to one or two rounds of resident workgroups, from the
 * runtime's occupancy query) with `reps` timed launches each, on the current
 * state and dt, and keep the fastest (as fit_set_tuning).  The state, step
 * counter, trace and probe are left unchanged (candidates run out of place
 * into the second buffer set).  On the fused path it also times step pairs
 * (fit_set_pair_tuning) for a few tiles and z-chunks and switches them on
 * when a pair takes less than 98 % of two single steps.  Any output pointer
 * may be NULL; *ms_best is the per-step time of the winner.  Synchronises. */
int fit_autotune(fit_grid* g, double dt, int reps, int* path, int* tw, int* ty, int* kc,
                 float* ms_best);

/* Number of curl applications (sparse matrix-vector products of the paper's
 * cost model, eq. cost_LF: 2 per leapfrog step) performed by this handle. */
int fit_smvp_count(const fit_grid* g, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* FIT_H */
