// Batched leapfrog: many independent grids of uneven size, each with its own
// materials, source and dt, advanced together (the paper's independent
// leapfrog runs of Sec. III / Alg. 1 form such a batch).
//
// One launch covers one step of EVERY grid: workgroup r of the launch runs
// item r of the step's item table, i.e. one fused-step tile (the tile body of
// fit_step_tile.hpp) of one grid.  Consecutive steps are ordered by the
// kernel boundary alone: no workgroup ever waits on another, and no atomics
// are used.  The index of the step within a call lives in device memory and
// is advanced by a one-thread kernel after every single step, so a captured
// chain of S (step, advance) launches can be replayed as a hipGraph; a chain
// of pair launches (k_batch2) reads the counters plus each launch's offset in
// the chain and advances them once per chain.  The persistent form
// (k_batch_persist) runs S steps in one cooperative launch instead, with a
// grid-wide barrier between the steps.
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

// after launches of `steps` steps in all: the step index and the buffer-set
// flips (one per launch)
__global__ void k_batch_advance(BatchCtl* ctl, int steps, int flips) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->step_base += steps;
    ctl->flip += flips;
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
    step_tile<T, true, kEnergyNone, false>(a, tx, tyi, kz, sm, nullptr, nullptr);
  else
    step_tile<T, false, kEnergyNone, false>(a, tx, tyi, kz, sm, nullptr, nullptr);
}

// Two steps of every grid: one workgroup per item of the pair item table,
// i.e. one tile (with its z-chunk) of one grid, run by the tile body of the
// single-grid two-step kernel in the grid's compile-time tile shape.  The
// table is read in launch order: it is laid out so that the dispatcher's
// round-robin over the XCDs gives each XCD whole groups of neighbouring
// tiles, longest first (entries of grid -1 are padding).  The step index and buffer set of launch
// launch_off of a captured chain come from the counters plus its offset, so
// the counters are advanced once per chain.  Budgets as the single-grid
// kernel's one-point compile-time variants (at most 768 threads).  The
// outputs go out by ordinary stores: most grids' row segments straddle L2
// lines, and the neighbouring tiles of a group, running together on one
// XCD, complete those lines in L2 before they are written back.
template <typename T, bool LOSSY>
__device__ __forceinline__ void batch2_tile(const S2Args<T>& a, int shape, int t, T* sm) {
  const int tx = t % a.t.ntx;
  const int rr = t / a.t.ntx;
  const int tyi = rr % a.t.nty, kz = rr / a.t.nty;
  static_assert(kBatchPairNShapes == 4, "one case per shape");
  switch (shape) {
    case 0:
      step2_tile<T, LOSSY, false, kBatchPairShapes[0][0], kBatchPairShapes[0][1], 1, false,
                 false>(a, tx, tyi, kz, sm);
      break;
    case 1:
      step2_tile<T, LOSSY, false, kBatchPairShapes[1][0], kBatchPairShapes[1][1], 1, false,
                 false>(a, tx, tyi, kz, sm);
      break;
    case 2:
      step2_tile<T, LOSSY, false, kBatchPairShapes[2][0], kBatchPairShapes[2][1], 1, false,
                 false>(a, tx, tyi, kz, sm);
      break;
    default:
      step2_tile<T, LOSSY, false, kBatchPairShapes[3][0], kBatchPairShapes[3][1], 1, false,
                 false>(a, tx, tyi, kz, sm);
      break;
  }
}

// Two steps of item `it` (not padding) from step index sg with buffer-set
// offset flip (the grid's own parity added).
template <typename T>
__device__ __forceinline__ void batch2_item(const BatchArgs<T>& B, const BatchItem it, int64_t sg,
                                            int flip, T* sm) {
  const BatchGrid<T>& G = B.grids[it.grid];
  const int p = (int)((G.par0 + flip) & 1);
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
  if (G.lossy)
    batch2_tile<T, true>(a, G.s2shape, it.tile, sm);
  else
    batch2_tile<T, false>(a, G.s2shape, it.tile, sm);
}

template <typename T>
__global__ __launch_bounds__(768)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 3))) void k_batch2(BatchArgs<T> B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const BatchItem it = B.items2[blockIdx.x];
  if (it.grid < 0) return;   // padding of a shorter XCD list
  const int64_t sg = B.fixed_parity ? 0 : B.ctl->step_base + 2 * (int64_t)B.launch_off;
  const int flip = B.fixed_parity ? 0 : B.ctl->flip + B.launch_off;
  batch2_item<T>(B, it, sg, flip, sm);
}

// Persistent form: S steps of every grid in ONE launch.  Workgroup w runs
// items w, w + G, w + 2G, ... of each step's item table (G = gridDim.x; the
// loop bounds are the same for every thread of a workgroup, so every thread
// reaches every barrier), then the whole launch meets at a grid-wide barrier
// before the next step.  The launch is cooperative when launched directly
// (the runtime starts it only if every workgroup can be resident at once)
// and G never exceeds the resident capacity.
//
// The barrier lives in the control block (bar_count, bar_gen), cleared by
// k_batch_bar_reset before every launch: barrier s of the launch waits for
// bar_gen >= s + 1.  Each workgroup's first thread, after the workgroup has
// finished the step (every wave has waited for its stores to complete) and
// released the workgroup's writes at agent scope (the XCD's L2 written back,
// so the other XCDs see them), adds the workgroup to bar_count
// (agent-scope atomic),
// and either -- as the last to arrive -- clears the count and publishes the
// new generation with a release store, or polls bar_gen with agent-scope
// loads (which go to the device's coherence point, not the XCD's L2),
// sleeping between polls, and acquires at agent scope (the CU's L1 and the
// XCD's L2 drop lines another XCD may have rewritten) before the workgroup
// goes on.  One release and one acquire per workgroup and step: making every
// wave fence cost 1.6x the step time on the 64-grid workload.  A poll gives
// up after kBarSpins tries and sets ctl->error, so a launch whose workgroups
// could not all be resident ends (with wrong fields and the error flag)
// instead of hanging.
constexpr uint64_t kBarSpins = 1ull << 23;   // x >= 128 cycles: about 0.5 s

__global__ void k_batch_bar_reset(BatchCtl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->bar_count = 0u;
    ctl->bar_gen = 0u;
  }
}

__device__ __forceinline__ void grid_barrier(BatchCtl* ctl, unsigned target, unsigned nwg) {
  // every wave: its stores complete (acknowledged by the L2); then one
  // thread writes the XCD's L2 back at agent scope (the workgroup's stores
  // are all in it by now)
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned arrived =
        __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == nwg) {
      __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->bar_gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint64_t spins = 0;
      while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins >= kBarSpins) {
          __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    // acquire: the CU's L1 and the XCD's L2 drop their lines; the other
    // waves of the workgroup (same CU) read only after the barrier below
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_batch_persist(BatchArgs<T> B, int S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int w = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int64_t base = B.ctl->step_base;
  const int flip = B.ctl->flip;
  for (int s = 0; s < S; ++s) {
    for (int r = w; r < B.P; r += (int)gridDim.x) {
      const int g = B.item_grid[r];
      const BatchGrid<T>& G = B.grids[g];
      const int t = r - G.tile_off;
      const int p = (G.par0 + flip + s) & 1;
      SArgs<T> a;
      batch_args<T>(G, p, G.src_tab ? G.src_tab[base + s] : T(0), a);
      const int tx = t % G.t.ntx;
      const int rr = t / G.t.ntx;
      if (G.lossy)
        step_tile<T, true, kEnergyNone, false>(a, tx, rr % G.t.nty, rr / G.t.nty, sm, nullptr, nullptr);
      else
        step_tile<T, false, kEnergyNone, false>(a, tx, rr % G.t.nty, rr / G.t.nty, sm, nullptr, nullptr);
      __syncthreads();   // the next item restages the LDS
    }
    grid_barrier(B.ctl, (unsigned)s + 1u, gridDim.x);
  }
  // every workgroup has read step_base and flip before the last barrier
  if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    B.ctl->step_base = base + S;
    B.ctl->flip = flip + S;
  }
}

// Persistent pairs: npairs pairs of steps of every grid in one cooperative
// launch of G = gridDim.x resident workgroups (a multiple of 8).  Workgroup w
// runs entries w, w + G, w + 2G, ... of the pair item table, whose entry r
// belongs to XCD r mod 8 -- the XCD the dispatcher puts workgroup r on -- so
// each XCD's workgroups walk its own list (the tiles of a z-chunk of a grid
// together, longest first); empty entries are skipped.  The launch meets at
// the grid barrier after every pair (same barrier, bounds and error flag as
// the single-step form).
template <typename T>
__global__ __launch_bounds__(768)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 3))) void k_batch2_persist(BatchArgs<T> B,
                                                                                   int npairs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int64_t base = B.ctl->step_base;
  const int flip = B.ctl->flip;
  for (int j = 0; j < npairs; ++j) {
    for (int r = (int)blockIdx.x; r < B.P; r += (int)gridDim.x) {
      const BatchItem it = B.items2[r];
      if (it.grid < 0) continue;
      batch2_item<T>(B, it, base + 2 * (int64_t)j, flip + j, sm);
      __syncthreads();   // the next item restages the LDS
    }
    grid_barrier(B.ctl, (unsigned)j + 1u, gridDim.x);
  }
  // every workgroup has read step_base and flip before the last barrier
  if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    B.ctl->step_base = base + 2 * (int64_t)npairs;
    B.ctl->flip = flip + npairs;
  }
}

template <typename T>
static int persist2_occupancy(int nthreads, size_t lds) {
  int nb = 0;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch2_persist<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&k_batch2_persist<T>), nthreads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

int batch2_persist_blocks_per_cu(size_t esz, int nthreads, size_t lds) {
  return esz == 8 ? persist2_occupancy<double>(nthreads, lds)
                  : persist2_occupancy<float>(nthreads, lds);
}

template <typename T>
hipError_t launch_batch2_persist(const BatchArgs<T>& b, int nwg, int npairs, hipStream_t s) {
  if (nwg <= 0 || nwg % kXcds != 0 || npairs <= 0) return hipErrorInvalidValue;
  BatchArgs<T> a = b;
  int n = npairs;
  void* args[2] = {&a, &n};
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch2_persist<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, b.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_bar_reset, dim3(1), dim3(64), 0, s, b.ctl);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch2_persist<T>),
                                    dim3((unsigned)nwg), dim3((unsigned)b.nthreads), args,
                                    (unsigned)b.lds, s);
}

template hipError_t launch_batch2_persist<float>(const BatchArgs<float>&, int, int, hipStream_t);
template hipError_t launch_batch2_persist<double>(const BatchArgs<double>&, int, int, hipStream_t);

template <typename T>
static int persist_occupancy(int nthreads, size_t lds) {
  int nb = 0;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_persist<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&k_batch_persist<T>), nthreads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

int batch_persist_blocks_per_cu(size_t esz, int nthreads, size_t lds) {
  return esz == 8 ? persist_occupancy<double>(nthreads, lds)
                  : persist_occupancy<float>(nthreads, lds);
}

template <typename T>
hipError_t launch_batch_persist(const BatchArgs<T>& b, int nwg, int S, hipStream_t s) {
  BatchArgs<T> a = b;
  int steps = S;
  void* args[2] = {&a, &steps};
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_persist<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, b.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_bar_reset, dim3(1), dim3(64), 0, s, b.ctl);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch_persist<T>),
                                    dim3((unsigned)nwg), dim3((unsigned)b.nthreads), args,
                                    (unsigned)b.lds, s);
}

template hipError_t launch_batch_persist<float>(const BatchArgs<float>&, int, int, hipStream_t);
template hipError_t launch_batch_persist<double>(const BatchArgs<double>&, int, int, hipStream_t);

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
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, b.ctl, 1, 1);
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
  return hipGetLastError();
}

hipError_t launch_batch_advance(BatchCtl* ctl, int steps, int flips, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, ctl, steps, flips);
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
