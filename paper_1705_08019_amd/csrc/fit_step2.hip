// Two leapfrog steps per pass (temporal blocking of the Sec. II-A
// recurrence): one launch reads (e^m, h^(m+1/2)) and the materials once and
// writes (e^(m+2), h^(m+5/2)); the intermediate state (e^(m+1), h^(m+3/2))
// lives only in LDS.  Per cell and pair of steps this moves the 56 B of one
// fused step instead of 112 B.
//
// A workgroup (as many threads as the e^(m+1) region has points, up to
// 1024, numbered linearly) owns a TW x TY column tile and marches a chunk [k0, k1) of
// z-planes with a lag of two planes between what it reads and what it
// stores.  In local coordinates (x along i, y along j) the regions are
//   X4: x in [-2, TW+1], y in [-2, TY+1]  staged h^(m+1/2), eps, sigma
//   R1: x in [-1, TW+1], y in [-1, TY+1]  e^(m+1)       (needs X4)
//   R2: x in [-1, TW],   y in [-1, TY]    h^(m+3/2)     (needs R1, X4)
//   R3: x in [0, TW],    y in [0, TY]     e^(m+2)       (needs R2, R1, X4)
//   tile                                  h^(m+5/2)     (needs R3, R2)
// Iteration k forms e^(m+1) of plane k, h^(m+3/2) of plane k-1, e^(m+2) of
// plane k-1 and h^(m+5/2) of plane k-2, for k = k0-1 .. k1+1; the halo rows
// and columns are recomputed by every tile that needs them with the same
// contraction-pinned point functions as the single-step kernels, so the
// result is bitwise that of two single steps.  Values outside the grid and
// on planes outside [0, nz) are zero (PEC), as in the single-step kernels.
#include <algorithm>

#include "fit_step_tile.hpp"

namespace fit {

struct S2Geom {
  int W4, N4, W1, N1, W2, N2, W3, N3;
};

__host__ __device__ inline S2Geom s2_geom(int tw, int ty) {
  S2Geom g;
  g.W4 = tw + 4;
  g.N4 = (tw + 4) * (ty + 4);
  g.W1 = tw + 3;
  g.N1 = (tw + 3) * (ty + 3);
  g.W2 = tw + 2;
  g.N2 = (tw + 2) * (ty + 2);
  g.W3 = tw + 1;
  g.N3 = (tw + 1) * (ty + 1);
  return g;
}

size_t step2_lds_bytes(int tw, int ty, size_t esz, bool lossy, int nu_planes) {
  const S2Geom g = s2_geom(tw, ty);
  const size_t n = 6 * (size_t)g.N4 + 3 * (size_t)g.N4 + (lossy ? 3 * (size_t)g.N4 : 0) +
                   6 * (size_t)g.N1 + 6 * (size_t)g.N2 + 6 * (size_t)g.N3 +
                   3 * (size_t)nu_planes;
  return esz * n;
}

bool step2_plane_ok(const Dims& d, size_t esz) {
  return (uint64_t)d.sxy * esz <= (uint64_t)UINT32_MAX;
}

int step2_threads(int tw, int ty) {
  const S2Geom g = s2_geom(tw, ty);
  return (g.N1 + 63) / 64 * 64;
}

bool step2_shape_ok(int tw, int ty, size_t esz, bool lossy, int nu_planes) {
  if (tw < 8 || ty < 2) return false;
  const S2Geom g = s2_geom(tw, ty);
  const int nthr = step2_threads(tw, ty);   // one thread per point of the largest computed region
  if (nthr > 1024 || g.N4 > kS2Per * nthr) return false;
  return step2_lds_bytes(tw, ty, esz, lossy, nu_planes) <= 160 * 1024;
}

// Global access at a wave-uniform plane base plus a per-thread 32-bit byte
// offset within the plane (the launchers check that a plane spans < 4 GiB):
// the scalar-base + 32-bit-offset addressing of the global instructions, so
// that no 64-bit vector address is formed per access.  `fresh` marks a
// loop-invariant offset as redefined inside the z-march (an empty asm, once
// per plane); otherwise its zero-extension is hoisted out of the loop and the
// 64-bit form returns.
__device__ __forceinline__ uint32_t fresh(uint32_t off) {
  asm volatile("" : "+v"(off));
  return off;
}
template <typename T>
__device__ __forceinline__ T pld(const T* base, uint32_t off) {
  using C1 = const __attribute__((address_space(1))) char;
  using T1 = const __attribute__((address_space(1))) T;
  return *(T1*)((C1*)base + off);
}
template <typename T>
__device__ __forceinline__ void pst(T* base, uint32_t off, T v) {
  using C1 = __attribute__((address_space(1))) char;
  using T1 = __attribute__((address_space(1))) T;
  *(T1*)((C1*)base + off) = v;
}

// FP32: at most 80 VGPRs (6 waves per SIMD), so that two workgroups of the
// 32 x 16 tile (11 waves each) are resident per CU.  CTW, CTY > 0 fix the
// tile at compile time (every LDS offset an immediate), 0 takes it from the
// tiling.
template <typename T, bool LOSSY, bool NU, int CTW, int CTY>
__global__ __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 4))) void k_step2(S2Args<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const Dims d = A.d;
  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr = lt / A.t.ntx;
  const int tyi = (int)(rr % A.t.nty);
  const int kz = (int)(rr / A.t.nty);
  const int TW = CTW > 0 ? CTW : A.t.tw, TY = CTY > 0 ? CTY : A.t.ty;
  const S2Geom G = s2_geom(TW, TY);
  T* h0L = sm;                                // [2][3][N4]   h^(m+1/2), planes k, k-1
  T* cL = h0L + 6 * G.N4;                     // [3][N4]      eps0 eps_r, planes k, k-1, k-2
  T* sL = cL + 3 * G.N4;                      // [3][N4]      sigma (lossy)
  T* e1L = sL + (LOSSY ? 3 * G.N4 : 0);       // [2][3][N1]   e^(m+1), planes k, k-1
  T* h1L = e1L + 6 * G.N1;                    // [2][3][N2]   h^(m+3/2), planes k-1, k-2
  T* e2L = h1L + 6 * G.N2;                    // [2][3][N3]   e^(m+2), planes k-1, k-2
  T* zL = e2L + 6 * G.N3;                     // tensor grid: [3][kc + 3] per-plane factors

  const int i0 = tx * TW, j0 = tyi * TY;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  const int tid = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int nthr = (int)(blockDim.x * blockDim.y);   // >= N1 >= N2 >= N3 >= TW TY
  const int64_t sx = d.sx, sxy = d.sxy;

  auto hb = [](int k) { return k & 1; };                 // h0 / e1 / h1 / e2 buffer of plane k
  auto cb = [](int k) { return ((k % 3) + 3) % 3; };     // eps / sigma buffer of plane k
  auto i4 = [&](int x, int y) { return (y + 2) * G.W4 + (x + 2); };
  auto i1 = [&](int x, int y) { return (y + 1) * G.W1 + (x + 1); };
  auto i2 = [&](int x, int y) { return (y + 1) * G.W2 + (x + 1); };
  auto i3 = [&](int x, int y) { return y * G.W3 + x; };
  auto in_grid = [&](int gx, int gy) { return gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny; };

  // ---- per-thread points of every region (fixed over the z-march); grid
  // points as in-plane element indices p (gx + sx gy); LDS neighbours as
  // constant offsets from the point's own index (-1: x - 1, -W: y - 1)
  // source point: plane sk, in-plane index sp (none: sk = -1)
  const int64_t sk = A.src_idx >= 0 ? A.src_idx / sxy : -100;   // k >= -1 in the march
  const uint32_t sp = (uint32_t)(A.src_idx - (sk >= 0 ? sk * sxy : A.src_idx));
  constexpr uint32_t ES = sizeof(T);
  // X4 staging entries (up to kS2Per per thread)
  uint32_t o4[kS2Per];
  bool in4[kS2Per];
#pragma unroll
  for (int r = 0; r < kS2Per; ++r) {
    const int q = tid + r * nthr;
    const int gx = i0 + (q % G.W4) - 2, gy = j0 + (q / G.W4) - 2;
    in4[r] = q < G.N4 && in_grid(gx, gy);
    o4[r] = in4[r] ? (uint32_t)(gx + sx * gy) * ES : 0u;
  }
  // R1 point (e^(m+1)): one per thread
  const bool a1 = tid < G.N1;
  const int x1 = tid % G.W1 - 1, y1 = tid / G.W1 - 1;
  const int gx1 = i0 + x1, gy1 = j0 + y1;
  const bool in1 = a1 && in_grid(gx1, gy1);
  const uint32_t p1 = in1 ? (uint32_t)(gx1 + sx * gy1) : 0u;
  const bool s1 = in1 && p1 == sp;
  const int r1 = i4(x1, y1), r1im = r1 - 1, r1jm = r1 - G.W4, r1ijm = r1jm - 1;
  // R2 point (h^(m+3/2))
  const bool a2 = tid < G.N2;
  const int x2 = tid % G.W2 - 1, y2 = tid / G.W2 - 1;
  const bool in2 = a2 && in_grid(i0 + x2, j0 + y2);
  const bool px2 = in2 && i0 + x2 > 0, py2 = in2 && j0 + y2 > 0;
  const int e2c = i1(x2, y2), e2in = e2c + 1, e2jn = e2c + G.W1, r2h = i4(x2, y2);
  // R3 point (e^(m+2))
  const bool a3 = tid < G.N3;
  const int x3 = tid % G.W3, y3 = tid / G.W3;
  const int gx3 = i0 + x3, gy3 = j0 + y3;
  const bool in3 = a3 && in_grid(gx3, gy3);
  const bool own3 = in3 && x3 < TW && y3 < TY;
  const uint32_t p3 = in3 ? (uint32_t)(gx3 + sx * gy3) : 0u;
  const bool s3 = in3 && p3 == sp;
  const int r3 = i4(x3, y3), r3im = r3 - 1, r3jm = r3 - G.W4, r3ijm = r3jm - 1;
  const int h3 = i2(x3, y3), h3im = h3 - 1, h3jm = h3 - G.W2, o3 = i1(x3, y3);
  // tile point (h^(m+5/2))
  const int x5 = tid % TW, y5 = tid / TW;
  const bool own5 = tid < TW * TY && in_grid(i0 + x5, j0 + y5);
  const uint32_t p5 = own5 ? (uint32_t)((i0 + x5) + sx * (j0 + y5)) : 0u;
  const int e5 = i3(x5, y5), e5in = e5 + 1, e5jn = e5 + G.W3, h5 = i2(x5, y5);

  // ---- tensor-grid metric (as in the single fused step): x / y factors of
  // each thread's points, z factors of planes k0 - 1 .. k1 + 1 staged in LDS
  T kb1x = A.kb[0], kb1y = A.kb[1], kb3x = A.kb[0], kb3y = A.kb[1];
  T kd2x = 0, kd2y = 0, kd2z = 0, kd5x = 0, kd5y = 0, kd5z = 0;
  const int zp = A.t.kc + 3;
  if (NU) {
    auto cx = [&](int gx) { return min(max(gx, 0), d.nx - 1); };
    auto cy = [&](int gy) { return min(max(gy, 0), d.ny - 1); };
    kb1x = (T)(A.kbs * A.nsq[0][cx(gx1)]);
    kb1y = (T)(A.kbs * A.nsq[1][cy(gy1)]);
    kb3x = (T)(A.kbs * A.nsq[0][cx(gx3)]);
    kb3y = (T)(A.kbs * A.nsq[1][cy(gy3)]);
    const int ix2 = cx(i0 + x2), jy2 = cy(j0 + y2), ix5 = cx(i0 + x5), jy5 = cy(j0 + y5);
    kd2x = (T)(A.kds * (0.5 * A.ndl[0][ix2] * A.nrw[1][jy2]));
    kd2y = (T)(A.kds * (0.5 * A.ndl[1][jy2] * A.nrw[0][ix2]));
    kd2z = (T)(A.kds * (0.5 * A.nrw[0][ix2] * A.nrw[1][jy2]));
    kd5x = (T)(A.kds * (0.5 * A.ndl[0][ix5] * A.nrw[1][jy5]));
    kd5y = (T)(A.kds * (0.5 * A.ndl[1][jy5] * A.nrw[0][ix5]));
    kd5z = (T)(A.kds * (0.5 * A.nrw[0][ix5] * A.nrw[1][jy5]));
    for (int q = tid; q < zp; q += nthr) {
      const int kk = k0 - 1 + q;
      const bool in = kk >= 0 && kk < d.nz;
      zL[q] = in ? (T)(A.kbs * A.nsq[2][kk]) : T(0);
      zL[zp + q] = in ? (T)A.nrw[2][kk] : T(0);
      zL[2 * zp + q] = in ? (T)A.ndl[2][kk] : T(0);
    }
  }
  auto zi = [&](int k) { return k - (k0 - 1); };   // z-factor slot of plane k

  // ---- register staging of plane k: X4 entries (h x3, eps, sigma), R1 entry (e x3)
  T ph[kS2Per][5];
  T pe[3];
  auto fetch = [&](int k) {
    const bool plane = k >= 0 && k < d.nz;
    const int64_t gk = plane ? sxy * (int64_t)k : 0;
    const T *bh0 = A.h0[0] + gk, *bh1 = A.h0[1] + gk, *bh2 = A.h0[2] + gk;
    const T *bc = A.eps + gk, *bs = LOSSY ? A.sig + gk : nullptr;
#pragma unroll
    for (int r = 0; r < kS2Per; ++r) {
      const bool in = plane && in4[r];
      const uint32_t o = fresh(o4[r]);
      ph[r][0] = in ? pld(bh0, o) : T(0);
      ph[r][1] = in ? pld(bh1, o) : T(0);
      ph[r][2] = in ? pld(bh2, o) : T(0);
      ph[r][3] = in ? pld(bc, o) : T(0);
      ph[r][4] = (LOSSY && in) ? pld(bs, o) : T(0);
    }
    const bool in = plane && in1;
    const uint32_t o = fresh(p1 * ES);
    pe[0] = in ? pld(A.e0[0] + gk, o) : T(0);
    pe[1] = in ? pld(A.e0[1] + gk, o) : T(0);
    pe[2] = in ? pld(A.e0[2] + gk, o) : T(0);
  };
  auto stage = [&](int k) {
    T* h = h0L + hb(k) * 3 * G.N4;
    T* c = cL + cb(k) * G.N4;
    T* s = sL + cb(k) * G.N4;
#pragma unroll
    for (int r = 0; r < kS2Per; ++r) {
      const int q = tid + r * nthr;
      if (q < G.N4) {
        h[q] = ph[r][0];
        h[G.N4 + q] = ph[r][1];
        h[2 * G.N4 + q] = ph[r][2];
        c[q] = ph[r][3];
        if (LOSSY) s[q] = ph[r][4];
      }
    }
  };

  // e-update of one point of plane k: h planes k (hp) and k-1 (hq) with row
  // stride NH and indices (rh, rh_im, rh_jm); materials of planes k, k-1 in
  // the X4 layout at (r, rim, rjm, rijm); same operand order as the
  // single-step kernels.
  auto e_upd = [&](bool valid, int gi, int gj, bool at_src, int k, const T* hp, const T* hq, int NH,
                   int rh, int rh_im, int rh_jm, int r, int rim, int rjm, int rijm, const T* cp,
                   const T* cq, const T* sp, const T* sq, T exo, T eyo, T ezo, T src, T kbx_,
                   T kby_, T kbz_, T& exn, T& eyn, T& ezn) {
    const T c = cp[r], c_im = cp[rim], c_jm = cp[rjm], c_ijm = cp[rijm];
    const T Sx = c + c_im, Sy = c + c_jm, Sxj = c_jm + c_ijm;
    const T pc = cq[r];
    const T sye = pc + cq[rjm], sxe = pc + cq[rim];
    T E4x = sye + Sy, E4y = sxe + Sx, E4z = Sx + Sxj;
    T S4x = 0, S4y = 0, S4z = 0;
    if (LOSSY) {
      const T s = sp[r], s_im = sp[rim], s_jm = sp[rjm], s_ijm = sp[rijm];
      const T Sxs = s + s_im, Sys = s + s_jm;
      const T ps = sq[r];
      const T sys = ps + sq[rjm], sxs = ps + sq[rim];
      S4x = sys + Sys;
      S4y = sxs + Sxs;
      S4z = Sxs + (s_jm + s_ijm);
    }
    T jx = 0, jy = 0, jz = 0;
    if (valid && at_src) {
      if (A.src_comp == 0) jx = src;
      if (A.src_comp == 1) jy = src;
      if (A.src_comp == 2) jz = src;
    }
    if (!valid) E4x = E4y = E4z = T(1);
    e_point<T, LOSSY>(hp[rh], hp[NH + rh], hp[2 * NH + rh], hq[rh], hq[NH + rh], hp[rh_jm],
                      hp[NH + rh_im], hp[2 * NH + rh_jm], hp[2 * NH + rh_im], E4x, E4y, E4z,
                      S4x, S4y, S4z, exo, eyo, ezo, jx, jy, jz, valid && gj > 0 && k > 0,
                      valid && gi > 0 && k > 0, valid && gi > 0 && gj > 0, kbx_, kby_, kbz_,
                      A.hs, exn, eyn, ezn);
  };

  // prologue: plane k0 - 2 staged, plane k0 - 1 in flight
  fetch(k0 - 2);
  stage(k0 - 2);
  fetch(k0 - 1);

  for (int k = k0 - 1; k <= k1 + 1; ++k) {
    stage(k);
    const T e0x = pe[0], e0y = pe[1], e0z = pe[2];
    if (k + 1 <= k1 + 1) fetch(k + 1);
    __syncthreads();

    // ---- e^(m+1) of plane k on R1
    if (a1) {
      const bool kin = k >= 0 && k < d.nz;
      T exn, eyn, ezn;
      e_upd(in1 && kin, gx1, gy1, s1 && k == sk, k, h0L + hb(k) * 3 * G.N4,
            h0L + hb(k - 1) * 3 * G.N4, G.N4, r1, r1im, r1jm, r1, r1im, r1jm, r1ijm,
            cL + cb(k) * G.N4, cL + cb(k - 1) * G.N4, sL + cb(k) * G.N4, sL + cb(k - 1) * G.N4,
            e0x, e0y, e0z, A.src_val[0], kb1x, kb1y, NU ? zL[zi(k)] : A.kb[2], exn, eyn, ezn);
      T* out = e1L + hb(k) * 3 * G.N1;
      out[tid] = exn;
      out[G.N1 + tid] = eyn;
      out[2 * G.N1 + tid] = ezn;
    }
    __syncthreads();

    // ---- h^(m+3/2) of plane km = k - 1 on R2 (from e^(m+1) of planes km, k)
    const int km = k - 1;
    if (km >= k0 - 1 && a2) {
      const T* nq = e1L + hb(km) * 3 * G.N1;
      const T* np_ = e1L + hb(k) * 3 * G.N1;
      const T* ho = h0L + hb(km) * 3 * G.N4;
      const bool valid = in2 && km >= 0 && km < d.nz;
      T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
      if (NU) {
        const T rz = zL[zp + zi(km)];
        kdx = kd2x * rz;
        kdy = kd2y * rz;
        kdz = kd2z * zL[2 * zp + zi(km)];
      }
      T hxn, hyn, hzn;
      h_point<T>(nq[e2c], nq[G.N1 + e2c], nq[2 * G.N1 + e2c], np_[e2c], np_[G.N1 + e2c],
                 nq[2 * G.N1 + e2jn], nq[2 * G.N1 + e2in], nq[G.N1 + e2in], nq[e2jn], ho[r2h],
                 ho[G.N4 + r2h], ho[2 * G.N4 + r2h], A.imu2, A.imu2, A.imu2, valid && px2,
                 valid && py2, valid && km > 0, kdx, kdy, kdz, hxn, hyn, hzn);
      T* out = h1L + hb(km) * 3 * G.N2;
      out[tid] = hxn;
      out[G.N2 + tid] = hyn;
      out[2 * G.N2 + tid] = hzn;
    }
    __syncthreads();

    // ---- e^(m+2) of plane km on R3 (from h^(m+3/2) of planes km, km - 1 and
    // e^(m+1) of plane km); the tile part of planes [k0, k1) is stored
    if (km >= k0 && a3) {
      const T* eo = e1L + hb(km) * 3 * G.N1;
      const bool kin = km >= 0 && km < d.nz;
      T exn, eyn, ezn;
      e_upd(in3 && kin, gx3, gy3, s3 && km == sk, km, h1L + hb(km) * 3 * G.N2, h1L + hb(km - 1) * 3 * G.N2,
            G.N2, h3, h3im, h3jm, r3, r3im, r3jm, r3ijm, cL + cb(km) * G.N4,
            cL + cb(km - 1) * G.N4, sL + cb(km) * G.N4, sL + cb(km - 1) * G.N4, eo[o3],
            eo[G.N1 + o3], eo[2 * G.N1 + o3], A.src_val[1], kb3x, kb3y,
            NU ? zL[zi(km)] : A.kb[2], exn, eyn, ezn);
      T* out = e2L + hb(km) * 3 * G.N3;
      out[tid] = exn;
      out[G.N3 + tid] = eyn;
      out[2 * G.N3 + tid] = ezn;
      if (own3 && km < k1) {
        const int64_t gk = sxy * (int64_t)km;
        const uint32_t o = fresh(p3 * ES);
        pst(A.e2[0] + gk, o, exn);
        pst(A.e2[1] + gk, o, eyn);
        pst(A.e2[2] + gk, o, ezn);
      }
    }
    __syncthreads();

    // ---- h^(m+5/2) of plane kh = k - 2 on the tile (from e^(m+2) of planes kh, kh + 1)
    const int kh = k - 2;
    if (kh >= k0 && kh < k1 && own5) {
      const T* nq = e2L + hb(kh) * 3 * G.N3;
      const T* np_ = e2L + hb(kh + 1) * 3 * G.N3;
      const T* ho = h1L + hb(kh) * 3 * G.N2;
      T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
      if (NU) {
        const T rz = zL[zp + zi(kh)];
        kdx = kd5x * rz;
        kdy = kd5y * rz;
        kdz = kd5z * zL[2 * zp + zi(kh)];
      }
      T hxn, hyn, hzn;
      h_point<T>(nq[e5], nq[G.N3 + e5], nq[2 * G.N3 + e5], np_[e5], np_[G.N3 + e5],
                 nq[2 * G.N3 + e5jn], nq[2 * G.N3 + e5in], nq[G.N3 + e5in], nq[e5jn], ho[h5],
                 ho[G.N2 + h5], ho[2 * G.N2 + h5], A.imu2, A.imu2, A.imu2, i0 + x5 > 0,
                 j0 + y5 > 0, kh > 0, kdx, kdy, kdz, hxn, hyn, hzn);
      const int64_t gk = sxy * (int64_t)kh;
      const uint32_t o = fresh(p5 * ES);
      pst(A.h2[0] + gk, o, hxn);
      pst(A.h2[1] + gk, o, hyn);
      pst(A.h2[2] + gk, o, hzn);
    }
  }
}

template <typename T, bool L, bool N, int CW, int CY>
static hipError_t go_step2_t(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step2<T, L, N, CW, CY>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_step2<T, L, N, CW, CY>), grd, blk, lds, s, a);
  return hipGetLastError();
}

// the 32 x 16 tile (the fastest on 256 x 256 x 512 grids) has its own
// compile-time variant; other tiles take the generic one
template <typename T, bool L, bool N>
static hipError_t go_step2(const S2Args<T>& a, dim3 grd, dim3 blk, size_t lds, hipStream_t s) {
  if (a.t.tw == 32 && a.t.ty == 16) return go_step2_t<T, L, N, 32, 16>(a, grd, blk, lds, s);
  return go_step2_t<T, L, N, 0, 0>(a, grd, blk, lds, s);
}

template <typename T>
hipError_t launch_step2(const S2Args<T>& a, bool lossy, hipStream_t s) {
  const bool nu = a.nsq[0] != nullptr;
  const int nup = nu ? a.t.kc + 3 : 0;
  if (!step2_shape_ok(a.t.tw, a.t.ty, sizeof(T), lossy, nup)) return hipErrorInvalidValue;
  if (!step2_plane_ok(a.d, sizeof(T))) return hipErrorInvalidValue;
  const dim3 blk(step2_threads(a.t.tw, a.t.ty)), grd((unsigned)a.t.blocks());
  const size_t lds = step2_lds_bytes(a.t.tw, a.t.ty, sizeof(T), lossy, nup);
  if (lossy) return nu ? go_step2<T, true, true>(a, grd, blk, lds, s)
                       : go_step2<T, true, false>(a, grd, blk, lds, s);
  return nu ? go_step2<T, false, true>(a, grd, blk, lds, s)
            : go_step2<T, false, false>(a, grd, blk, lds, s);
}

template hipError_t launch_step2<float>(const S2Args<float>&, bool, hipStream_t);
template hipError_t launch_step2<double>(const S2Args<double>&, bool, hipStream_t);

}  // namespace fit
