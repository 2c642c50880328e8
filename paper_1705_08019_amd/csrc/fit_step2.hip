// Launchers and shape rules of the two-steps-per-pass kernel (the tile
// body is in fit_step2_tile.hpp).
#include <algorithm>

#include "fit_step2_tile.hpp"

namespace fit {

size_t step2_lds_bytes(int tw, int ty, size_t esz, bool lossy, bool nu) {
  const S2Geom g = s2_geom(tw, ty);
  const size_t n = 3 * (size_t)g.N4 + (size_t)g.N4 + (lossy ? (size_t)g.N4 : 0) +
                   6 * (size_t)g.N1 + 3 * (size_t)g.N2 + 6 * (size_t)g.N3 +
                   (nu ? 3 * (size_t)kS2ZRing : 0);
  return esz * n;
}

bool step2_plane_ok(const Dims& d, size_t esz) {
  return (uint64_t)d.sxy * esz <= (uint64_t)UINT32_MAX;
}

int step2_points(int tw, int ty) { return s2_geom(tw, ty).N1 > 1024 ? 2 : 1; }

// Streaming output stores only where every tile row segment starts and ends
// on a 128-byte line (rows and tile width whole lines) and the launch's
// state does not fit the 256 MiB Infinity Cache: there they keep the outputs
// from evicting the halos neighbouring tiles still read.  Where the segments
// straddle lines, ordinary stores let L2 join the parts neighbouring tiles
// write (a 250 x 256 x 512 FP32 grid: 0.47 against 0.59 ms per launch);
// where the state fits the Infinity Cache, ordinary stores keep the outputs
// there for the next launch, which streaming stores do not (128^3 FP32:
// 15.9 against 18.6 us per step).
constexpr uint64_t kInfinityCacheBytes = 256ull << 20;
static bool step2_streaming(const Dims& d, int tw, size_t esz) {
  // e and h read and written, eps and sigma read: 14 values per cell
  const uint64_t state = (uint64_t)d.n * esz * 14;
  return ((size_t)d.nx * esz) % 128 == 0 && ((size_t)tw * esz) % 128 == 0 &&
         state > kInfinityCacheBytes;
}

int step2_threads(int tw, int ty) {
  const S2Geom g = s2_geom(tw, ty);
  const int np = step2_points(tw, ty);
  // every point of R1 owned (np per thread), the staged X4 plane within
  // kS2Per entries per thread
  const int n = std::max((g.N1 + np - 1) / np, (g.N4 + kS2Per - 1) / kS2Per);
  return (n + 63) / 64 * 64;
}

bool step2_shape_ok(int tw, int ty, size_t esz, bool lossy, bool nu) {
  if (tw < 8 || ty < 2) return false;
  const int nthr = step2_threads(tw, ty);
  // one point per thread up to 1024 threads; two points per thread up to 768,
  // FP32 only (FP64 two-point tiles spill registers, and the useful ones
  // exceed the LDS)
  if (step2_points(tw, ty) > 1 && esz != 4) return false;
  if (nthr > (step2_points(tw, ty) == 1 ? 1024 : 768)) return false;
  return step2_lds_bytes(tw, ty, esz, lossy, nu) <= 160 * 1024;
}

// Register budgets: the FP32 compile-time one-point tiles at most 80 VGPRs
// (6 waves per SIMD: two 11- or 12-wave workgroups per CU); the FP64 ones at
// most 168 (3 waves per SIMD: one workgroup of up to 768 threads, no
// spills); two-point tiles 168 (one workgroup of up to 12 waves per CU: their
// LDS leaves room for no second); generic one-point tiles 128 (up to 1024
// threads).  (A 16-wave 64 x 12 tile would need 64 VGPRs for two workgroups
// per CU and spills there.)
template <typename T, int CTW, int CTY, int NP>
constexpr int s2_waves() {
  if (NP > 1) return 3;
  // one 16-wave workgroup per CU (4 waves per SIMD) for tiles of more than
  // 12 waves, else two workgroups per CU
  return CTW == 0 ? 4 : ((CTW + 4) * (CTY + 3) + 63) / 64 > 12 ? 4 : sizeof(T) == 8 ? 3 : 6;
}
template <typename T, int CTW, int NP>
constexpr int s2_max_threads() { return NP > 1 || (CTW > 0 && sizeof(T) == 8) ? 768 : 1024; }

template <typename T, bool LOSSY, bool NU, int CTW, int CTY, int NP, bool NTS>
__global__ __launch_bounds__((s2_max_threads<T, CTW, NP>()))
__attribute__((amdgpu_waves_per_eu((s2_waves<T, CTW, CTY, NP>())))) void k_step2(S2Args<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr = lt / A.t.ntx;
  step2_tile<T, LOSSY, NU, CTW, CTY, NP, false, NTS>(A, tx, (int)(rr % A.t.nty),
                                                     (int)(rr / A.t.nty),
                                                     reinterpret_cast<T*>(smem_raw));
}

template <typename T, bool L, bool N, int CW, int CY, int NP, bool NTS>
static hipError_t go_step2_k(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step2<T, L, N, CW, CY, NP, NTS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_step2<T, L, N, CW, CY, NP, NTS>), grd, blk, lds, s, a);
  return hipGetLastError();
}

template <typename T, bool L, bool N, int CW, int CY, int NP>
static hipError_t go_step2_t(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  return step2_streaming(a.d, a.t.tw, sizeof(T))
             ? go_step2_k<T, L, N, CW, CY, NP, true>(a, grd, blk, lds, s)
             : go_step2_k<T, L, N, CW, CY, NP, false>(a, grd, blk, lds, s);
}

// the 64 x 8 and 32 x 16 tiles (the fastest one-point tiles on 256 x 256 x
// 512 grids) and, in FP32, the two-point 64 x 16 tile have compile-time
// variants; other tiles take the generic ones
template <typename T, bool L, bool N>
static hipError_t go_step2(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  const int tw = a.t.tw, ty = a.t.ty;
  if (step2_points(tw, ty) > 1) {
    if constexpr (sizeof(T) == 4) {
      if (tw == 64 && ty == 16) return go_step2_t<T, L, N, 64, 16, 2>(a, grd, blk, lds, s);
      return go_step2_t<T, L, N, 0, 0, 2>(a, grd, blk, lds, s);
    }
    return hipErrorInvalidValue;   // not reached: step2_shape_ok rejects FP64 two-point tiles
  }
  if (tw == 32 && ty == 16) return go_step2_t<T, L, N, 32, 16, 1>(a, grd, blk, lds, s);
  if (tw == 64 && ty == 8) return go_step2_t<T, L, N, 64, 8, 1>(a, grd, blk, lds, s);
  if constexpr (sizeof(T) == 4)   // 1024 threads: FP32 only
    if (tw == 64 && ty == 12) return go_step2_t<T, L, N, 64, 12, 1>(a, grd, blk, lds, s);
  return go_step2_t<T, L, N, 0, 0, 1>(a, grd, blk, lds, s);
}

template <typename T>
hipError_t launch_step2(const S2Args<T>& a, bool lossy, hipStream_t s) {
  const bool nu = a.nsq[0] != nullptr;
  if (!step2_shape_ok(a.t.tw, a.t.ty, sizeof(T), lossy, nu)) return hipErrorInvalidValue;
  if (!step2_plane_ok(a.d, sizeof(T))) return hipErrorInvalidValue;
  const dim3 blk(step2_threads(a.t.tw, a.t.ty)), grd((unsigned)a.t.blocks());
  const size_t lds = step2_lds_bytes(a.t.tw, a.t.ty, sizeof(T), lossy, nu);
  if (lossy) return nu ? go_step2<T, true, true>(a, grd, blk, lds, s)
                       : go_step2<T, true, false>(a, grd, blk, lds, s);
  return nu ? go_step2<T, false, true>(a, grd, blk, lds, s)
            : go_step2<T, false, false>(a, grd, blk, lds, s);
}

template hipError_t launch_step2<float>(const S2Args<float>&, bool, hipStream_t);
template hipError_t launch_step2<double>(const S2Args<double>&, bool, hipStream_t);

// Energy pairs: the same tile body with the FP64 energy sums; its nine
// compensated accumulators do not fit the two-workgroups-per-CU budget, so
// one workgroup per CU (3 or 4 waves per SIMD).
bool step2_energy_ok(int tw, int ty, bool nu) { return !nu && step2_points(tw, ty) == 1; }

// the compile-time tile's own thread count (step2_threads), 1024 for generic tiles
template <int CTW, int CTY>
constexpr int s2e_threads() {
  if (CTW == 0) return 1024;
  const int n1 = (CTW + 4) * (CTY + 3), n4 = ((CTW + 4) * (CTY + 4) + kS2Per - 1) / kS2Per;
  return ((n1 > n4 ? n1 : n4) + 63) / 64 * 64;
}

template <typename T, bool LOSSY, int CTW, int CTY, bool NTS>
__global__ __launch_bounds__((s2e_threads<CTW, CTY>()))
__attribute__((amdgpu_waves_per_eu((s2e_threads<CTW, CTY>() > 768 ? 4 : 3)))) void k_step2e(
    S2Args<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr = lt / A.t.ntx;
  step2_tile<T, LOSSY, false, CTW, CTY, 1, true, NTS>(A, tx, (int)(rr % A.t.nty),
                                                      (int)(rr / A.t.nty),
                                                      reinterpret_cast<T*>(smem_raw),
                                                      A.part + (int64_t)blockIdx.x * kPartTerms);
}

template <typename T, bool L, int CW, int CY, bool NTS>
static hipError_t go_step2e_k(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step2e<T, L, CW, CY, NTS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_step2e<T, L, CW, CY, NTS>), grd, blk, lds, s, a);
  return hipGetLastError();
}

template <typename T, bool L, int CW, int CY>
static hipError_t go_step2e_t(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  return step2_streaming(a.d, a.t.tw, sizeof(T))
             ? go_step2e_k<T, L, CW, CY, true>(a, grd, blk, lds, s)
             : go_step2e_k<T, L, CW, CY, false>(a, grd, blk, lds, s);
}

template <typename T, bool L>
static hipError_t go_step2e(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  const int tw = a.t.tw, ty = a.t.ty;
  if (tw == 32 && ty == 16) return go_step2e_t<T, L, 32, 16>(a, grd, blk, lds, s);
  if (tw == 64 && ty == 8) return go_step2e_t<T, L, 64, 8>(a, grd, blk, lds, s);
  if constexpr (sizeof(T) == 4)
    if (tw == 64 && ty == 12) return go_step2e_t<T, L, 64, 12>(a, grd, blk, lds, s);
  return go_step2e_t<T, L, 0, 0>(a, grd, blk, lds, s);
}

template <typename T>
hipError_t launch_step2_energy(const S2Args<T>& a, bool lossy, hipStream_t s) {
  const bool nu = a.nsq[0] != nullptr;
  if (!step2_energy_ok(a.t.tw, a.t.ty, nu) || !a.part) return hipErrorInvalidValue;
  if (!step2_shape_ok(a.t.tw, a.t.ty, sizeof(T), lossy, nu)) return hipErrorInvalidValue;
  if (!step2_plane_ok(a.d, sizeof(T))) return hipErrorInvalidValue;
  const dim3 blk(step2_threads(a.t.tw, a.t.ty)), grd((unsigned)a.t.blocks());
  const size_t lds = step2_lds_bytes(a.t.tw, a.t.ty, sizeof(T), lossy, nu);
  return lossy ? go_step2e<T, true>(a, grd, blk, lds, s) : go_step2e<T, false>(a, grd, blk, lds, s);
}

template hipError_t launch_step2_energy<float>(const S2Args<float>&, bool, hipStream_t);
template hipError_t launch_step2_energy<double>(const S2Args<double>&, bool, hipStream_t);

}  // namespace fit
