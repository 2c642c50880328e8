// Batched leapfrog: many independent grids of uneven size, each with its own
// materials, source and dt, advanced together (the paper's independent
// leapfrog runs of Sec. III / Alg. 1 form such a batch).
//
// One launch covers one step of EVERY grid: workgroup r of the launch runs
// item r of the step's item table, i.e. one fused-step tile (the tile body of
// fit_step_tile.hpp) of one grid.  Consecutive steps are ordered by the
// kernel boundary alone: no workgroup ever waits on another, and no atomics
// are used.  The index of the step within a call lives in device memory and
// is advanced by a one-thread kernel after every step, so a captured chain of
// S (step, advance) launches can be replayed as a hipGraph.
#include "fit_step2_tile.hpp"
#include "fit_step_tile.hpp"

namespace fit {

__global__ void k_batch_set_base(BatchCtl* ctl, int64_t base) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->step_base = base;
    ctl->error = 0;
    ctl->flip = 0;
  }
}

// after a launch of `steps` steps: the step index and the buffer-set flips
__global__ void k_batch_advance(BatchCtl* ctl, int steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->step_base += steps;
    ctl->flip += 1;
  }
}

template <typename T>
__device__ __forceinline__ void batch_args(const BatchGrid<T>& G, int p, T src, SArgs<T>& a) {
  const int64_t n = G.d.n;
  for (int c = 0; c < 3; ++c) {
    a.e0[c] = G.e[p] + c * n;
    a.h0[c] = G.h[p] + c * n;
    a.e1[c] = G.e[1 - p] + c * n;
    a.h1[c] = G.h[1 - p] + c * n;
    a.kb[c] = G.kb[c];
    a.kd[c] = G.kd[c];
    a.ge[c] = 0.0;
    a.gf2[c] = 0.0;
  }
  a.eps = G.eps;
  a.sig = G.sig;
  a.d = G.d;
  a.t = G.t;
  a.hs = G.hs;
  a.imu2 = G.imu2;
  a.src_comp = G.src_comp;
  a.src_idx = G.src_idx;
  a.src_val = src;
  a.src_val_d = 0.0;
  a.probe.on = 0;
  a.part = nullptr;
  a.pacc = nullptr;
  a.pscale = 0.0;
}

// One step of every grid: one workgroup per item of the step's item table.
template <typename T>
__global__ __launch_bounds__(1024) void k_batch(BatchArgs<T> B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int r = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int g = B.item_grid[r];
  const BatchGrid<T>& G = B.grids[g];
  const int t = r - G.tile_off;
  const int64_t sg = B.fixed_parity ? 0 : B.ctl->step_base;   // step index within the call
  const int p = (int)((G.par0 + (B.fixed_parity ? 0 : B.ctl->flip)) & 1);
  SArgs<T> a;
  batch_args<T>(G, p, G.src_tab ? G.src_tab[sg] : T(0), a);
  const int tx = t % G.t.ntx;
  const int rr = t / G.t.ntx;
  const int tyi = rr % G.t.nty;
  const int kz = rr / G.t.nty;
  if (G.lossy)
    step_tile<T, true, false, false>(a, tx, tyi, kz, sm, nullptr, nullptr);
  else
    step_tile<T, false, false, false>(a, tx, tyi, kz, sm, nullptr, nullptr);
}

// Two steps of every grid: one workgroup per item of the pair item table,
// i.e. one 32 x 16 tile (with its z-chunk) of one grid, run by the tile body
// of the single-grid two-step kernel.  Budgets as that kernel's 32 x 16
// variant.
template <typename T>
__global__ __launch_bounds__(sizeof(T) == 8 ? 768 : 1024)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 3))) void k_batch2(BatchArgs<T> B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int r = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int g = B.item_grid[r];
  const BatchGrid<T>& G = B.grids[g];
  const int t = r - G.tile_off2;
  const int64_t sg = B.fixed_parity ? 0 : B.ctl->step_base;
  const int p = (int)((G.par0 + (B.fixed_parity ? 0 : B.ctl->flip)) & 1);
  S2Args<T> a;
  const int64_t n = G.d.n;
  for (int c = 0; c < 3; ++c) {
    a.e0[c] = G.e[p] + c * n;
    a.h0[c] = G.h[p] + c * n;
    a.e2[c] = G.e[1 - p] + c * n;
    a.h2[c] = G.h[1 - p] + c * n;
    a.kb[c] = G.kb[c];
    a.kd[c] = G.kd[c];
  }
  a.eps = G.eps;
  a.sig = G.sig;
  a.d = G.d;
  a.t = G.t2;
  a.hs = G.hs;
  a.imu2 = G.imu2;
  a.src_comp = G.src_comp;
  a.src_idx = G.src_idx;
  a.src_val[0] = G.src_tab ? G.src_tab[sg] : T(0);
  a.src_val[1] = G.src_tab ? G.src_tab[sg + 1] : T(0);
  const int tx = t % G.t2.ntx;
  const int rr = t / G.t2.ntx;
  if (G.lossy)
    step2_tile<T, true, false, kBatchPairTw, kBatchPairTy>(a, tx, rr % G.t2.nty, rr / G.t2.nty, sm);
  else
    step2_tile<T, false, false, kBatchPairTw, kBatchPairTy>(a, tx, rr % G.t2.nty, rr / G.t2.nty, sm);
}

template <typename T>
static int batch_occupancy(int nthreads, size_t lds) {
  int nb = 0;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_batch<T>),
                                                   nthreads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

int batch_prepare(size_t esz, int nthreads, size_t lds) {
  return esz == 8 ? batch_occupancy<double>(nthreads, lds) : batch_occupancy<float>(nthreads, lds);
}

// One step of every grid, then the step counter (fixed_parity: no counter).
template <typename T>
hipError_t launch_batch(const BatchArgs<T>& b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch<T>, dim3((unsigned)b.P), dim3(b.nthreads), (size_t)b.lds, s, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.fixed_parity) return e;
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, b.ctl, 1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch2(const BatchArgs<T>& b, hipStream_t s) {
  if (b.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch2<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, b.lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_batch2<T>, dim3((unsigned)b.P), dim3(b.nthreads), (size_t)b.lds, s, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.fixed_parity) return e;
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, b.ctl, 2);
  return hipGetLastError();
}

hipError_t launch_batch_set_base(BatchCtl* ctl, int64_t base, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_set_base, dim3(1), dim3(64), 0, s, ctl, base);
  return hipGetLastError();
}

template hipError_t launch_batch<float>(const BatchArgs<float>&, hipStream_t);
template hipError_t launch_batch<double>(const BatchArgs<double>&, hipStream_t);
template hipError_t launch_batch2<float>(const BatchArgs<float>&, hipStream_t);
template hipError_t launch_batch2<double>(const BatchArgs<double>&, hipStream_t);

}  // namespace fit
