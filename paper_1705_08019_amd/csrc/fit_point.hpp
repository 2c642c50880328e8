// Per-node update arithmetic shared by every kernel that advances the
// leapfrog (split half-step kernels, the fused single-pass kernel, the
// batched kernel).  Floating-point contraction is pinned (explicit fma, no
// compiler contraction) so that a value recomputed redundantly in a halo is
// bitwise identical to the value its owner computes and stores.
#pragma once

#include <hip/hip_runtime.h>

namespace fit {

// Quotient a / b of the e-update coefficients (b > 0, a normal number).
// FP32: the hardware reciprocal (1 ulp) and one Newton correction of the
// quotient, q = a r, q + r (a - b q) (Markstein's refinement): within 1 ulp
// of a / b in 4 instructions, against about 10 for the IEEE sequence with
// its scaling and denormal-mode switches.  FP64: the IEEE division.
template <typename T>
__device__ __forceinline__ T qdiv(T a, T b) {
  return a / b;
}
template <>
__device__ __forceinline__ float qdiv<float>(float a, float b) {
#pragma clang fp contract(off)
  const float r = __builtin_amdgcn_rcpf(b);
  const float q = a * r;
  return fmaf(fmaf(-b, q, a), r, q);
}

// e-update of the three primal edges leaving one node (Sec. II-A):
//   e^(m+1) = ca e^m + cb (C~ h^(m+1/2) - j_s)
// with S4eps (E4*) and S4sig (S4*) the sums over the 4 cells around each edge,
//   ca = (E4 - hs S4) / (E4 + hs S4),  cb = kb / (E4 + hs S4),  hs = dt/2,
// and the dual curl by backward differences:
//   (C~ h)_x = [h_z(j) - h_z(j-1)] - [h_y(k) - h_y(k-1)]   (cyclic for y, z).
// The l* flags select edges that are not in a PEC wall; others become 0.
template <typename T, bool LOSSY>
__device__ __forceinline__ void e_point(T hxc, T hyc, T hzc, T hxp, T hyp, T hx_jm, T hy_im,
                                        T hz_jm, T hz_im, T E4x, T E4y, T E4z, T S4x, T S4y,
                                        T S4z, T exo, T eyo, T ezo, T jx, T jy, T jz, bool lx,
                                        bool ly, bool lz, T kbx, T kby, T kbz, T hs, T& exn,
                                        T& eyn, T& ezn) {
#pragma clang fp contract(off)
  const T cx = ((hzc - hz_jm) - (hyc - hyp)) - jx;
  const T cy = ((hxc - hxp) - (hzc - hz_im)) - jy;
  const T cz = ((hyc - hy_im) - (hxc - hx_jm)) - jz;
  T nx_, ny_, nz_;
  if (LOSSY) {
    const T dpx = fma(hs, S4x, E4x), dmx = fma(-hs, S4x, E4x);
    const T dpy = fma(hs, S4y, E4y), dmy = fma(-hs, S4y, E4y);
    const T dpz = fma(hs, S4z, E4z), dmz = fma(-hs, S4z, E4z);
    nx_ = qdiv(fma(dmx, exo, kbx * cx), dpx);
    ny_ = qdiv(fma(dmy, eyo, kby * cy), dpy);
    nz_ = qdiv(fma(dmz, ezo, kbz * cz), dpz);
  } else {
    nx_ = exo + qdiv(kbx * cx, E4x);
    ny_ = eyo + qdiv(kby * cy, E4y);
    nz_ = ezo + qdiv(kbz * cz, E4z);
  }
  exn = lx ? nx_ : T(0);
  eyn = ly ? ny_ : T(0);
  ezn = lz ? nz_ : T(0);
}

// h-update of the three primal facets anchored at one node (Sec. II-A, with
// the primal curl C acting on e):
//   h^(m+3/2) = h^(m+1/2) - kd (imu_1 + imu_2) (C e^(m+1))
//   (C e)_x = [e_z(j+1) - e_z(j)] - [e_y(k+1) - e_y(k)]   (cyclic for y, z).
// m* = imu_1 + imu_2 per facet; l* select facets not in a PEC wall.
template <typename T>
__device__ __forceinline__ void h_point(T exc, T eyc, T ezc, T exn, T eyn, T ez_jn, T ez_in,
                                        T ey_in, T ex_jn, T hxo, T hyo, T hzo, T mx, T my, T mz,
                                        bool lx, bool ly, bool lz, T kdx, T kdy, T kdz, T& hxn,
                                        T& hyn, T& hzn) {
#pragma clang fp contract(off)
  const T cx = (ez_jn - ezc) - (eyn - eyc);
  const T cy = (exn - exc) - (ez_in - ezc);
  const T cz = (ey_in - eyc) - (ex_jn - exc);
  const T ax = kdx * mx, ay = kdy * my, az = kdz * mz;
  hxn = lx ? fma(-ax, cx, hxo) : T(0);
  hyn = ly ? fma(-ay, cy, hyo) : T(0);
  hzn = lz ? fma(-az, cz, hzo) : T(0);
}

}  // namespace fit
