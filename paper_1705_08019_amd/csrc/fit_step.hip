// Fused single-pass leapfrog step for gfx950 (Sec. II-A): one launch reads
// the state (e^m, h^(m+1/2)) once and writes (e^(m+1), h^(m+3/2)) to a second
// buffer set, so a step moves 6 field values + the per-cell materials per
// cell instead of the 9 + materials of two separate half-step passes.
//
// Tiling.  A workgroup owns a tw (x) x ty (y) column tile and marches a chunk
// of z-planes.  For each plane k it stages h^(m+1/2), eps and sigma of the
// tile plus a one-cell ring in LDS (double-buffered: planes k and k-1), forms
// e^(m+1) on the tile plus its +x column and +y row (the halo values the
// h-update needs are recomputed here, bitwise equal to what the neighbouring
// tile stores, since both use the same contraction-pinned point function),
// then forms h^(m+3/2) of plane k-1 from e^(m+1) of planes k-1 and k.  A
// chunk [k0, k1) recomputes e^(m+1) of plane k1 (not stored) to finish h of
// plane k1-1.  Reads and writes never touch the same buffer, so tiles and
// chunks need no ordering between them.
#include "fit_step_tile.hpp"

namespace fit {

size_t step_lds_bytes(int ty, size_t esz, bool lossy, int tw, int nu_planes) {
  const size_t RP = (size_t)(tw + 2) * (size_t)(ty + 2);   // ring plane: x in [-1, tw], y in [-1, ty]
  const size_t EP = (size_t)(tw + 1) * (size_t)(ty + 1);   // ext plane: x in [0, tw], y in [0, ty]
  return esz * (3 * 3 * RP + 3 * RP + (lossy ? 3 * RP : 0) + 2 * 3 * EP + 3 * (size_t)nu_planes);
}

template <typename T, bool LOSSY, int ENERGY, bool PROBE, bool NU>
__global__ __launch_bounds__(1024) void k_step(SArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr = lt / A.t.ntx;
  const int tyi = (int)(rr % A.t.nty);
  const int kz = (int)(rr / A.t.nty);
  step_tile<T, LOSSY, ENERGY, PROBE, NU>(A, tx, tyi, kz, reinterpret_cast<T*>(smem_raw),
                                         ENERGY != kEnergyNone
                                             ? A.part + (int64_t)blockIdx.x * kPartTerms
                                                : nullptr,
                                         PROBE ? A.pacc + 2 * (int64_t)blockIdx.x : nullptr);
}

template <typename T, bool LOSSY>
static int occupancy_of(int ty, int tw) {
  int nb = 0;
  const size_t lds = step_lds_bytes(ty, sizeof(T), LOSSY, tw);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step<T, LOSSY, kEnergyNone, false, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&k_step<T, LOSSY, kEnergyNone, false, false>), tw * ty, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

int step_blocks_per_cu(int ty, size_t esz, bool lossy, int tw) {
  if (esz == 8)
    return lossy ? occupancy_of<double, true>(ty, tw) : occupancy_of<double, false>(ty, tw);
  return lossy ? occupancy_of<float, true>(ty, tw) : occupancy_of<float, false>(ty, tw);
}

template <typename T>
hipError_t launch_step(const SArgs<T>& a, bool lossy, int energy, bool probe, hipStream_t s) {
  const dim3 blk(a.t.tw, a.t.ty), grd((unsigned)a.t.blocks());
  const bool nu = a.nsq[0] != nullptr;
  const size_t lds = step_lds_bytes(a.t.ty, sizeof(T), lossy, a.t.tw, nu ? a.t.kc + 1 : 0);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
#define FIT_S(L, E, P, N)                                                                 \
  do {                                                                                   \
    if (lds > 64 * 1024) {                                                               \
      hipError_t ea = hipFuncSetAttribute(                                               \
          reinterpret_cast<const void*>(&k_step<T, L, E, P, N>),                         \
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                         \
      if (ea != hipSuccess) return ea;                                                   \
    }                                                                                    \
    hipLaunchKernelGGL((k_step<T, L, E, P, N>), grd, blk, lds, s, a);                     \
  } while (0)
#define FIT_SN(L, E, P)              \
  do {                               \
    if (nu) FIT_S(L, E, P, true);    \
    else FIT_S(L, E, P, false);      \
  } while (0)
#define FIT_SP(L, E)                  \
  do {                                \
    if (probe) FIT_SN(L, E, true);    \
    else FIT_SN(L, E, false);         \
  } while (0)
#define FIT_SE(L)                                        \
  do {                                                   \
    if (energy == kEnergyAll) FIT_SP(L, kEnergyAll);     \
    else if (energy == kEnergyHCross) FIT_SP(L, kEnergyHCross); \
    else FIT_SP(L, kEnergyNone);                         \
  } while (0)
  if (energy != kEnergyNone && energy != kEnergyAll && energy != kEnergyHCross)
    return hipErrorInvalidValue;
  if (lossy) FIT_SE(true);
  else FIT_SE(false);
#undef FIT_SE
#undef FIT_SP
#undef FIT_SN
#undef FIT_S
  return hipGetLastError();
}

template hipError_t launch_step<float>(const SArgs<float>&, bool, int, bool, hipStream_t);
template hipError_t launch_step<double>(const SArgs<double>&, bool, int, bool, hipStream_t);

}  // namespace fit
