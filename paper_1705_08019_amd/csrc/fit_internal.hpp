// Internal declarations shared by the HIP kernel files and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fit {

// Grid geometry in the slot layout: component arrays of n = nx*ny*nz
// elements, x fastest.  sx = nx, sxy = nx*ny.
struct Dims {
  int nx, ny, nz;
  int64_t sx, sxy, n;
};

// Tiling of a z-marching launch: blockDim = (tw, ty); each thread owns one
// (i, j) column of a tw x ty tile and marches over a chunk of kc planes.
// The half-step kernels use tw = 64; the fused step takes tw in {32, 64,
// 128, 256} (a row of tw lanes spans tw / 64 waves, or two rows share one).
struct Tiling {
  int ty, kc;
  int ntx, nty, nkc;
  int tw;
  int64_t blocks() const { return (int64_t)ntx * nty * nkc; }
};

Tiling make_tiling(const Dims& d, int ty, int kc, int tw = 64);

// Closed probe box in node coordinates; a direction-a edge at node p is in
// the probe when lo[a] <= p_a and p_a + 1 <= hi[a] and lo[b] <= p_b <= hi[b]
// for the two other axes.
struct Probe {
  int lo[3], hi[3];
  int on;
};

// Number of FP64 partial terms written per block by the energy variants.
// Workgroups are dispatched round-robin over the 8 XCDs of the chip: give
// each XCD a contiguous range of logical work items (tiles in x-fastest, then
// y, then z-chunk order) so that halo rows shared by neighbouring tiles stay
// in one XCD's L2.  bid = hardware workgroup index, nb = grid size.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t q = nb / kXcds, r = nb % kXcds;
  const int64_t x = bid % kXcds, l = bid / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

constexpr int kPartTerms = 10;
// Workgroups of the standalone energy kernel (grid-stride beyond that).
constexpr int64_t kEnergyBlocks = 4096;
// E-pass partial term slots
enum { PE_EE_MM = 0, PE_EE_MM1 = 1, PE_EE_M1M1 = 2, PE_LOSS = 3, PE_SRC = 4, PE_PROBE = 5 };
// H-pass partial term slots
enum { PH_HH_CC = 0, PH_HH_CN = 1, PH_HH_NN = 2 };
// Fused-step partial term slots: the E slots above, then the H terms.
enum { PS_HH_CC = 6, PS_HH_CN = 7, PS_HH_NN = 8 };
// Energy pairs: the first step's h cross term <h^(m+1/2), h^(m+3/2)> (the
// pending term of the row the second step records).
constexpr int kPairHCross = 9;
// Energy modes of the fused step: none, every term, or only the h cross
// term <h^(m+1/2), h^(m+3/2)> (the step before a trace row needs no other).
enum { kEnergyNone = 0, kEnergyAll = 1, kEnergyHCross = 2 };

template <typename T>
struct EArgs {
  const T* ein[3];
  T* eout[3];
  const T* h[3];
  const T* eps;      // eps0 * eps_r per cell
  const T* sig;      // sigma per cell (lossy variant only)
  Dims d;
  Tiling t;
  T kb[3];           // 4 dt / g_a with g_a = d_b d_c / d_a  (cb = kb / (S4eps + hs S4sig))
  T hs;              // dt / 2
  double ge[3];      // g_a / 4: M_eps = ge * S4eps,  M_sigma = ge * S4sig
  // Tensor grid with per-axis cell widths (null on a uniform grid): sq[a][i]
  // is the square of the a-width of cell index i, and eps, sig hold the cell
  // values times the cell volume V.  An a-edge with index i along a then has
  // M_eps = S4eps / (4 sq[a][i]) (its 4 cells share that width), so
  // kb = kbs sq[a][i] with kbs = 4 dt and ge = 1 / (4 sq[a][i]).
  const double* sq[3] = {nullptr, nullptr, nullptr};
  double kbs = 0.0;
  int src_comp;      // -1: no source
  int64_t src_idx;
  T src_val;         // i(t_{m+1/2})
  double src_val_d;
  Probe probe;
  double* part;      // [blocks][kPartTerms] or null
  double* pacc;      // probe objective: per-workgroup (sum, compensation) rows
  double pscale;     // dt: weight of this step's probe term
};

template <typename T>
struct HArgs {
  const T* e[3];
  const T* hin[3];
  T* hout[3];
  const T* imu;      // 1 / (mu0 mu_r) per cell, or null when uniform
  T imu_u;           // uniform 1 / (mu0 mu_r)
  Dims d;
  Tiling t;
  T kd[3];           // dt * d_a / (d_b d_c) / 2  (cd = kd * (imu_1 + imu_2))
  double gf2[3];     // d_a / (d_b d_c) / 2: M_mu^{-1} = gf2 * (imu_1 + imu_2)
  double* part;
  // Tensor grid (null on a uniform grid; needs the per-cell imu array, which
  // then holds imu times the cell volume): an a-facet with indices j, k
  // along the two other axes b, c has M_mu^{-1} = (imu_1 + imu_2) gf with
  // gf = 1 / (2 sq[b][j] sq[c][k]) (its 2 cells share those widths), and
  // kd = kds gf.
  const double* sq[3] = {nullptr, nullptr, nullptr};
  double kds = 0.0;
};

// Fused single-pass leapfrog step: reads state m from (e0, h0), writes state
// m+1 to (e1, h1) (distinct buffers).  Uniform mu only.
template <typename T>
struct SArgs {
  const T* e0[3];
  const T* h0[3];
  T* e1[3];
  T* h1[3];
  const T* eps;
  const T* sig;
  Dims d;
  Tiling t;
  T kb[3];
  T hs;
  T kd[3];
  T imu2;            // imu_u + imu_u
  double ge[3];
  double gf2[3];
  int src_comp;
  int64_t src_idx;
  T src_val;
  double src_val_d;
  Probe probe;
  double* part;      // [blocks][kPartTerms] (energy steps) or null
  double* pacc;      // probe objective: per-workgroup (sum, compensation) rows
  double pscale;     // dt: weight of this step's probe term
  // Tensor grid (per-axis cell widths; null otherwise).  eps and sig hold the
  // cell values times the cell volume; mu is uniform in value (imu2).
  // nsq: squared widths, nw: widths, ndl: dual half-sums (d[i-1] + d[i]) / 2
  // per axis.  An a-edge with index i along a: kb = kbs nsq[a][i], M_eps =
  // S4eps / (4 nsq[a][i]).  An x-facet at (i, j, k): M_mu^{-1} = (imu + imu)
  // ndl[0][i] / (2 nw[1][j] nw[2][k]), kd = kds times the factor of imu2
  // (cyclic for y, z facets).
  const double* nsq[3] = {nullptr, nullptr, nullptr};
  const double* nw[3] = {nullptr, nullptr, nullptr};
  const double* ndl[3] = {nullptr, nullptr, nullptr};
  const double* nrw[3] = {nullptr, nullptr, nullptr};   // 1 / widths
  double kbs = 0.0, kds = 0.0;
};

// Dynamic LDS bytes of the fused kernel for a tw x ty tile, and the number
// of its workgroups a CU holds at once (0 if the runtime cannot tell).
// Two fused steps per pass (fit_step2.hip): reads (e0, h0) = state m and
// writes (e2, h2) = state m+2 (distinct buffers).  Uniform mu and spacing,
// no energies or probe.  src_val: i(t_{m+1/2}), i(t_{m+3/2}).
constexpr int kS2Per = 2;   // staged X4 / R1 entries per thread
template <typename T>
struct S2Args {
  const T* e0[3];
  const T* h0[3];
  T* e2[3];
  T* h2[3];
  const T* eps;
  const T* sig;
  Dims d;
  Tiling t;
  T kb[3];
  T hs;
  T kd[3];
  T imu2;
  int src_comp;
  int64_t src_idx;
  T src_val[2];
  // energy pairs (uniform grids): edge and facet metrics as in SArgs, and
  // the launch's partial-sum rows (kPartTerms per workgroup)
  double ge[3] = {0.0, 0.0, 0.0};
  double gf2[3] = {0.0, 0.0, 0.0};
  double* part = nullptr;
  // tensor grid (null otherwise): as in SArgs
  const double* nsq[3] = {nullptr, nullptr, nullptr};
  const double* ndl[3] = {nullptr, nullptr, nullptr};
  const double* nrw[3] = {nullptr, nullptr, nullptr};
  double kbs = 0.0, kds = 0.0;
};
// Planes of per-plane metric factors held in LDS by the two-step kernel on a
// tensor grid (a ring; a power of two).
constexpr int kS2ZRing = 4;
// nu: tensor grid (per-plane metric ring in LDS).
size_t step2_lds_bytes(int tw, int ty, size_t esz, bool lossy, bool nu);
// Points of the (tw + 4) x (ty + 3) thread grid (the e^(m+1) region with its
// row stride) per thread of a pair workgroup: 1, or 2 where the grid has more
// than 1024 points.
int step2_points(int tw, int ty);
// Threads of a pair workgroup: the thread grid's points over step2_points,
// at least the staged (tw + 4) x (ty + 4) plane over kS2Per, rounded up to a
// multiple of 64.
int step2_threads(int tw, int ty);
// Tile shapes the two-step kernel takes: tw >= 8, ty >= 2, at most 1024
// threads with one point per thread (768 with two, FP32 only), LDS <= 160 KiB.
bool step2_shape_ok(int tw, int ty, size_t esz, bool lossy, bool nu = false);
// In-plane byte offsets of the two-step kernel are 32-bit: a plane of the
// slot layout must span at most 4 GiB.
bool step2_plane_ok(const Dims& d, size_t esz);
template <typename T>
hipError_t launch_step2(const S2Args<T>& a, bool lossy, hipStream_t s);
// A pair whose second step is a trace row (uniform grids, tiles of one point
// per thread): as launch_step2, and every workgroup writes its kPartTerms
// partial sums to a.part: the terms of the fused step with every energy term
// for the second step (slots PE_* and PS_*), the h cross term of the first
// step in slot kPairHCross.  hipErrorInvalidValue for other grids or tiles.
template <typename T>
hipError_t launch_step2_energy(const S2Args<T>& a, bool lossy, hipStream_t s);
bool step2_energy_ok(int tw, int ty, bool nu);

// nu_planes: planes of per-plane metric staged on a tensor grid (0 otherwise).
size_t step_lds_bytes(int ty, size_t esz, bool lossy, int tw = 64, int nu_planes = 0);
int step_blocks_per_cu(int ty, size_t esz, bool lossy, int tw = 64);

template <typename T>
hipError_t launch_step(const SArgs<T>& a, bool lossy, int energy, bool probe, hipStream_t s);

// Row weights W (3 n doubles) of the Gram form: M_eps of the edges (which 0,
// gw = g_a / 4) or M_mu of the facets (which 1, gw = gf2_a) (fit_gram.hip).
// sq: null, or the squared cell widths [x (nx) | y (ny) | z (nz)] of a tensor
// grid (then eps and imu hold cell values times the cell volume, gw unused).
template <typename T>
hipError_t launch_gram_weights(double* W, int which, const T* eps, const T* imu, T imu_u,
                               const Dims& d, const double gw[3], const double* sq,
                               hipStream_t s);

// Gram matrix G = X^T diag(W) X over K snapshots (fit_gram.hip); part must
// hold part_cap_blocks * 64 * 64 doubles, G (device) K * K doubles.
template <typename T>
hipError_t launch_gram(const T* X, int64_t ld, int K, const double* W, const Dims& d, double* part,
                       int64_t part_cap_blocks, double* G, hipStream_t s, int64_t* nwg_used);

// Reverse-time adjoint step (fit_adjoint.hip): one fused pass per reverse
// step.  All field arrays are slot-layout components; lambda and mu
// ping-pong (read *0, write *1).  geps / gsig: per-cell FP64 accumulators of
// dJ/deps_r and dJ/dsigma.
template <typename T>
struct AdjArgs {
  // 3-component slot-layout fields (component c at offset c n)
  const T* h;         // h^(m+1/2)
  const T* em;        // e^m
  const T* em1;       // e^(m+1)
  const T* lam0;      // lambda^(m+2)
  const T* mu0;       // mu^(m+3/2)
  T* lam1;            // lambda^(m+1)
  T* mu1;             // mu^(m+1/2)
  const T* eps;
  const T* sig;
  double* geps;
  double* gsig;
  Dims d;
  Tiling t;
  T kb[3];
  T hs;
  T dmu[3];           // dt M_mu^{-1} per facet direction (uniform mu)
  double ge[3];       // M_eps = ge E4 = (g_a / 4) E4; dM_sigma / d sigma(cell) = ge
  double eps0;        // dM_eps / d eps_r(cell) = eps0 ge
  double dt, hdt;
  int src_comp;
  int64_t src_idx;
  T src_val;
  Probe probe;
};

size_t adjoint_lds_bytes(int tw, int ty, size_t esz);
// Ring entries of a plane staged per thread by the reverse-step kernel:
// (tw + 2)(ty + 2) <= 2 (tw + 1)(ty + 1) <= 2 nthr whenever tw ty >= 2.
constexpr int kAdjRing = 2;
int adjoint_threads(int tw, int ty);   // tw ty column threads + tw + ty + 1 halo threads
int adjoint_blocks_per_cu(int tw, int ty, size_t esz, bool lossy);
template <typename T>
hipError_t launch_adjoint_step(const AdjArgs<T>& a, bool lossy, hipStream_t s);

// Batched leapfrog, one launch per step of all grids (fit_batch.hip).
struct BatchCtl {
  int64_t step_base;   // index of the next step within the current call
  int error;           // set by the persistent kernel when a barrier gave up
  int flip;            // buffer-set swaps so far in the call
  unsigned bar_count;  // persistent kernel: workgroups arrived at the barrier
  unsigned bar_gen;    // persistent kernel: barriers completed in this launch
};

template <typename T>
struct BatchGrid {
  T* e[2];             // the two state buffer sets
  T* h[2];
  const T* eps;
  const T* sig;
  Dims d;
  Tiling t;
  T kb[3];
  T hs;
  T kd[3];
  T imu2;
  int lossy;
  int src_comp;
  int64_t src_idx;
  const T* src_tab;    // source current of each step of the call, or null
  int par0;            // buffer set holding the state at the start of the call
  int ntiles;          // tiles per step
  int tile_off;        // offset of this grid's tiles within one step's items
  Tiling t2;           // step pairs: this grid's pair tiling (tw x ty, kc planes)
  int s2shape;         // its tile: index into kBatchPairShapes
};
// Tiles of the batched two-steps-per-launch kernel (compile-time variants of
// the pair tile body, at most 768 threads each); every grid takes the one
// that stages the fewest points for its x / y extent.
constexpr int kBatchPairShapes[4][2] = {{32, 16}, {32, 18}, {40, 14}, {24, 24}};
constexpr int kBatchPairNShapes = 4;
// One work item of a pair launch: tile `tile` (x fastest, then y, then
// z-chunk) of grid `grid`.
struct BatchItem {
  int grid, tile;
};

template <typename T>
struct BatchArgs {
  const BatchGrid<T>* grids;
  const int* item_grid;   // grid of each item of a step (P entries)
  const BatchItem* items2; // pair launches: the items, XCD-interleaved (P entries)
  BatchCtl* ctl;
  int nb;
  int P;                  // items (workgroups) per step
  int nthreads;           // threads per workgroup (1-D; >= tw ty of every grid's tile)
  int lds;                // dynamic LDS bytes (the largest grid tile's)
  int fixed_parity;       // autotuning: read par0, step index 0, no counter
  int launch_off;         // pair launches: index of the launch since the counters
                          // were last advanced (steps 2 launch_off, as many flips)
};

// Allow the batched kernel the largest dynamic LDS a workgroup can have and
// return its resident workgroups per CU for this shape (0 if unknown).
int batch_prepare(size_t esz, int nthreads, size_t lds);
template <typename T>
hipError_t launch_batch(const BatchArgs<T>& b, hipStream_t s);
// Two steps of every grid per launch (b.items2: the pair item table, b.P
// its length, b.lds the pair LDS, b.launch_off the launch's place since the
// last counter advance).  The counters are not advanced here.
template <typename T>
hipError_t launch_batch2(const BatchArgs<T>& b, hipStream_t s);
hipError_t launch_batch_set_base(BatchCtl* ctl, int64_t base, hipStream_t s);
// Advance the step index by `steps` and the buffer-set flips by `flips`.
hipError_t launch_batch_advance(BatchCtl* ctl, int steps, int flips, hipStream_t s);
// S steps of every grid in one cooperative launch of nwg resident workgroups
// (single-step items of b.item_grid; grid-wide barrier between steps); the
// step index and parity come from and go back to b.ctl.
template <typename T>
hipError_t launch_batch_persist(const BatchArgs<T>& b, int nwg, int S, hipStream_t s);
// Resident workgroups per CU of the persistent kernel (0 if unknown).
int batch_persist_blocks_per_cu(size_t esz, int nthreads, size_t lds);
// Persistent pairs: npairs pairs of steps of every grid in one cooperative
// launch of nwg resident workgroups (a multiple of 8; the pair item table of
// b, its threads and LDS), then the counters advanced by 2 npairs steps and
// npairs flips.
template <typename T>
hipError_t launch_batch2_persist(const BatchArgs<T>& b, int nwg, int npairs, hipStream_t s);
int batch2_persist_blocks_per_cu(size_t esz, int nthreads, size_t lds);

// Launch wrappers (fit_kernels.hip).  Return hipError_t of the launch.
template <typename T>
hipError_t launch_epass(const EArgs<T>& a, bool lossy, bool energy, bool probe, hipStream_t s);
template <typename T>
hipError_t launch_hpass(const HArgs<T>& a, bool mu_uniform, bool energy, hipStream_t s);

// Reduce `nblk` rows of kPartTerms partial sums (FP64, Neumaier) and scatter
// term t to dst[cols[t]] (cols[t] < 0: skip).  If jacc != null, term
// probe_term times jscale is added to the compensated pair jacc[0..1].
// If nan_col >= 0, dst[nan_col] is set to NaN; if row_m >= 0, dst[0] = row_m.
// If pend != null, dst[pend_col] = *pend (a term reduced by an earlier launch).
hipError_t launch_reduce(const double* part, int64_t nblk, double* dst, const int* cols,
                         int probe_term, double jscale, double* jacc, int nan_col,
                         int64_t row_m, const double* pend, int pend_col, hipStream_t s);

// out[0..4] = <e,e>, <h,h>, W, Q, Q^(m+1) - Q^m from work[0..1] (<e,e>,
// <h,h>) and work[2..11] (the trace-row terms of the step from the current
// state); with dt <= 0 the last three are NaN.
hipError_t launch_energy_combine(const double* work, double dt, double* out, hipStream_t s);

// Add the per-workgroup probe rows (sum, compensation) pacc[0 .. nrows) into
// the compensated pair jacc[0..1] in a fixed order, then clear the rows.
hipError_t launch_pacc_flush(double* pacc, int64_t nrows, double* jacc, hipStream_t s);

// Semi-discrete operator B (e, h) = (M_eps^{-1} C~ h, -M_mu^{-1} C e) of a
// lossless grid with uniform mu (fit_expm.hip): out = c B in with per-axis
// coefficients ce = c / (g_a / 4), ch = -c gf2_a (imu + imu); mode 1 also
// adds out to acc, mode 2 sets acc = in + out; modes 3 and 4 (Leja pair
// step) set out = c B in + gam y and acc += (3) or = (4) al y + be in.
// in, out, acc, y distinct.
template <typename T>
hipError_t launch_opb(const T* ein, const T* hin, T* eout, T* hout, T* eacc, T* hacc, int mode,
                      const T* eps, const Dims& d, const Tiling& t, const double ce[3],
                      const double ch[3], hipStream_t s, const T* ye = nullptr,
                      const T* yh = nullptr, double gam = 0.0, double al = 0.0, double be = 0.0);
// Per-workgroup rows (terms 0, 1) of <a, b>_M: sum M_eps a_e b_e and
// sum M_mu a_h b_h (mm = M_mu per facet direction); nblk rows of part.
template <typename T>
hipError_t launch_mdot(const T* ae, const T* ah, const T* be, const T* bh, const T* eps,
                       const Dims& d, const double ge[3], const double mm[3], double* part,
                       int64_t nblk, hipStream_t s);
template <typename T>
hipError_t launch_axpy(T a, const T* xe, const T* xh, T* ye, T* yh, int64_t n3, hipStream_t s);
template <typename T>
hipError_t launch_seed(T* xe, T* xh, const Dims& d, uint64_t seed, hipStream_t s);

// Zero the slots of PEC-wall edges (which = 0) or facets (which = 1).
template <typename T>
hipError_t launch_mask(T* f, const Dims& d, int which, hipStream_t s);

// out = C in (which = 0, edges -> facets) or C~ in (which = 1, facets -> edges).
template <typename T>
hipError_t launch_curl(const T* in, T* out, const Dims& d, int which, hipStream_t s);

// Standalone energies <e,e>_eps and <h,h>_mu of a state -> part rows 0, 1.
// sq as for launch_gram_weights.
template <typename T>
hipError_t launch_energy(const T* e, const T* h, const T* eps, const T* imu, T imu_u,
                         const Dims& d, const double ge[3], const double gf2[3],
                         const double* sq, double* part, int64_t* nblk, hipStream_t s);

}  // namespace fit
