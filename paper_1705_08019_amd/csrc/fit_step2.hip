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
// Every LDS array has the row stride W = TW + 4 of X4 (a region keeps only
// its own rows), and in every phase thread t sits at column t % W (x = t % W
// - 2) of row t / W of the region it computes, so that each LDS access is t
// plus a constant: the lanes of a wave touch consecutive words (no bank
// conflicts where a packed region row would wrap inside a wave) and no
// per-point LDS index is held in registers.
// Iteration k forms e^(m+1) of plane k, h^(m+3/2) of plane k-1, e^(m+2) of
// plane k-1 and h^(m+5/2) of plane k-2, for k = k0-1 .. k1+1; the halo rows
// and columns are recomputed by every tile that needs them with the same
// contraction-pinned point functions as the single-step kernels, so the
// result is bitwise that of two single steps.  Values outside the grid and
// on planes outside [0, nz) are zero (PEC), as in the single-step kernels.
#include <algorithm>

#include "fit_step_tile.hpp"

namespace fit {

// Row stride W of every region; N4, N1, N2, N3: entries of X4 (ty + 4 rows),
// R1 (ty + 3), R2 (ty + 2), R3 (ty + 1).
struct S2Geom {
  int W, N4, N1, N2, N3;
};

__host__ __device__ inline S2Geom s2_geom(int tw, int ty) {
  S2Geom g;
  g.W = tw + 4;
  g.N4 = g.W * (ty + 4);
  g.N1 = g.W * (ty + 3);
  g.N2 = g.W * (ty + 2);
  g.N3 = g.W * (ty + 1);
  return g;
}

size_t step2_lds_bytes(int tw, int ty, size_t esz, bool lossy, bool nu) {
  const S2Geom g = s2_geom(tw, ty);
  const size_t n = 6 * (size_t)g.N4 + 3 * (size_t)g.N4 + (lossy ? 3 * (size_t)g.N4 : 0) +
                   6 * (size_t)g.N1 + 6 * (size_t)g.N2 + 6 * (size_t)g.N3 +
                   (nu ? 3 * (size_t)kS2ZRing : 0);
  return esz * n;
}

bool step2_plane_ok(const Dims& d, size_t esz) {
  return (uint64_t)d.sxy * esz <= (uint64_t)UINT32_MAX;
}

int step2_threads(int tw, int ty) {
  const S2Geom g = s2_geom(tw, ty);
  return (g.N1 + 63) / 64 * 64;
}

bool step2_shape_ok(int tw, int ty, size_t esz, bool lossy, bool nu) {
  if (tw < 8 || ty < 2) return false;
  const S2Geom g = s2_geom(tw, ty);
  const int nthr = step2_threads(tw, ty);   // one thread per point of the largest computed region
  if (nthr > 1024 || g.N4 > kS2Per * nthr) return false;
  return step2_lds_bytes(tw, ty, esz, lossy, nu) <= 160 * 1024;
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
  T* zL = e2L + 6 * G.N3;                     // tensor grid: [3][kS2ZRing] per-plane factors

  const int i0 = tx * TW, j0 = tyi * TY;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  const int tid = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int nthr = (int)(blockDim.x * blockDim.y);   // >= N1 >= N2 >= N3 >= TW TY
  const int64_t sx = d.sx, sxy = d.sxy;

  auto hb = [](int k) { return k & 1; };                 // h0 / e1 / h1 / e2 buffer of plane k
  auto cb = [](int k) { return ((k % 3) + 3) % 3; };     // eps / sigma buffer of plane k
  auto in_grid = [&](int gx, int gy) { return gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny; };

  // ---- per-thread points (fixed over the z-march); grid points as in-plane
  // element indices p (gx + sx gy)
  // source point: plane sk, in-plane index src_p (none: sk < -1)
  const int64_t sk = A.src_idx >= 0 ? A.src_idx / sxy : -100;   // k >= -1 in the march
  const uint32_t src_p = (uint32_t)(A.src_idx - (sk >= 0 ? sk * sxy : A.src_idx));
  constexpr uint32_t ES = sizeof(T);
  const int W = G.W;
  // X4 staging entries (up to kS2Per per thread)
  uint32_t o4[kS2Per];
  bool in4[kS2Per];
#pragma unroll
  for (int r = 0; r < kS2Per; ++r) {
    const int q = tid + r * nthr;
    const int gx = i0 + (q % W) - 2, gy = j0 + (q / W) - 2;
    in4[r] = q < G.N4 && in_grid(gx, gy);
    o4[r] = in4[r] ? (uint32_t)(gx + sx * gy) * ES : 0u;
  }
  // the thread's column x (all phases) and rows: y = row - 1 in R1 / R2,
  // y = row in R3 / the tile
  const int row = tid / W, x = tid % W - 2;
  const int gx = i0 + x, gyA = j0 + row - 1, gyB = j0 + row;
  // R1 point (e^(m+1)); LDS: R1 index t, its X4 index t + W
  const bool a1 = row < TY + 3 && x >= -1;
  const bool in1 = a1 && in_grid(gx, gyA);
  const uint32_t p1 = in1 ? (uint32_t)(gx + sx * gyA) : 0u;
  const bool s1 = in1 && p1 == src_p;
  // R2 point (h^(m+3/2)); LDS: R2 / R1 index t, X4 index t + W
  const bool a2 = row < TY + 2 && x >= -1 && x <= TW;
  const bool in2 = a2 && in_grid(gx, gyA);
  const bool px2 = in2 && gx > 0, py2 = in2 && gyA > 0;
  // R3 point (e^(m+2)); LDS: R3 index t, R2 / R1 index t + W, X4 index t + 2W
  const bool a3 = row < TY + 1 && x >= 0 && x <= TW;
  const bool in3 = a3 && in_grid(gx, gyB);
  const uint32_t p3 = in3 ? (uint32_t)(gx + sx * gyB) : 0u;
  const bool s3 = in3 && p3 == src_p;
  // tile point (h^(m+5/2)) = the R3 point when it lies in the tile; LDS: R3
  // index t, R2 index t + W
  const bool own = in3 && x < TW && row < TY;

  // ---- tensor-grid metric (as in the single fused step): x / y factors of
  // each thread's points, z factors of planes k0 - 1 .. k1 + 1 staged in LDS
  T kbx = A.kb[0], kb1y = A.kb[1], kb3y = A.kb[1];
  T kd2x = 0, kd2y = 0, kd2z = 0, kd5x = 0, kd5y = 0, kd5z = 0;
  if (NU) {
    const int ix = min(max(gx, 0), d.nx - 1);
    const int jA = min(max(gyA, 0), d.ny - 1), jB = min(max(gyB, 0), d.ny - 1);
    kbx = (T)(A.kbs * A.nsq[0][ix]);
    kb1y = (T)(A.kbs * A.nsq[1][jA]);
    kb3y = (T)(A.kbs * A.nsq[1][jB]);
    kd2x = (T)(A.kds * (0.5 * A.ndl[0][ix] * A.nrw[1][jA]));
    kd2y = (T)(A.kds * (0.5 * A.ndl[1][jA] * A.nrw[0][ix]));
    kd2z = (T)(A.kds * (0.5 * A.nrw[0][ix] * A.nrw[1][jA]));
    kd5x = (T)(A.kds * (0.5 * A.ndl[0][ix] * A.nrw[1][jB]));
    kd5y = (T)(A.kds * (0.5 * A.ndl[1][jB] * A.nrw[0][ix]));
    kd5z = (T)(A.kds * (0.5 * A.nrw[0][ix] * A.nrw[1][jB]));
  }
  // the z factors of plane k sit in ring slot k mod kS2ZRing of zL (kb_z,
  // 1 / w_z, dual width): thread 0 fetches them with the plane and stages
  // them with it; a slot is rewritten three planes after its last reader
  // (the tile h-update of plane k - 2 may still run while plane k + 1 is
  // staged, so the ring holds four planes)
  constexpr int ZR = kS2ZRing;
  auto zs = [](int k) { return k & (ZR - 1); };
  double zraw[3] = {0.0, 0.0, 0.0};

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
    if (NU && tid == 0) {
      zraw[0] = plane ? A.nsq[2][k] : 0.0;
      zraw[1] = plane ? A.nrw[2][k] : 0.0;
      zraw[2] = plane ? A.ndl[2][k] : 0.0;
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
    if (NU && tid == 0) {
      zL[zs(k)] = (T)(A.kbs * zraw[0]);
      zL[ZR + zs(k)] = (T)zraw[1];
      zL[2 * ZR + zs(k)] = (T)zraw[2];
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
      e_upd(in1 && kin, gx, gyA, s1 && k == sk, k, h0L + hb(k) * 3 * G.N4,
            h0L + hb(k - 1) * 3 * G.N4, G.N4, tid + W, tid + W - 1, tid, tid + W, tid + W - 1,
            tid, tid - 1, cL + cb(k) * G.N4, cL + cb(k - 1) * G.N4, sL + cb(k) * G.N4,
            sL + cb(k - 1) * G.N4, e0x, e0y, e0z, A.src_val[0], kbx, kb1y,
            NU ? zL[zs(k)] : A.kb[2], exn, eyn, ezn);
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
        const T rz = zL[ZR + zs(km)];
        kdx = kd2x * rz;
        kdy = kd2y * rz;
        kdz = kd2z * zL[2 * ZR + zs(km)];
      }
      T hxn, hyn, hzn;
      const int c = tid, cin = tid + 1, cjn = tid + W, rh = tid + W;
      h_point<T>(nq[c], nq[G.N1 + c], nq[2 * G.N1 + c], np_[c], np_[G.N1 + c],
                 nq[2 * G.N1 + cjn], nq[2 * G.N1 + cin], nq[G.N1 + cin], nq[cjn], ho[rh],
                 ho[G.N4 + rh], ho[2 * G.N4 + rh], A.imu2, A.imu2, A.imu2, valid && px2,
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
      const int o = tid + W;
      e_upd(in3 && kin, gx, gyB, s3 && km == sk, km, h1L + hb(km) * 3 * G.N2,
            h1L + hb(km - 1) * 3 * G.N2, G.N2, tid + W, tid + W - 1, tid, tid + 2 * W,
            tid + 2 * W - 1, tid + W, tid + W - 1, cL + cb(km) * G.N4, cL + cb(km - 1) * G.N4,
            sL + cb(km) * G.N4, sL + cb(km - 1) * G.N4, eo[o], eo[G.N1 + o], eo[2 * G.N1 + o],
            A.src_val[1], kbx, kb3y, NU ? zL[zs(km)] : A.kb[2], exn, eyn, ezn);
      T* out = e2L + hb(km) * 3 * G.N3;
      out[tid] = exn;
      out[G.N3 + tid] = eyn;
      out[2 * G.N3 + tid] = ezn;
      if (own && km < k1) {
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
    if (kh >= k0 && kh < k1 && own) {
      const T* nq = e2L + hb(kh) * 3 * G.N3;
      const T* np_ = e2L + hb(kh + 1) * 3 * G.N3;
      const T* ho = h1L + hb(kh) * 3 * G.N2;
      T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
      if (NU) {
        const T rz = zL[ZR + zs(kh)];
        kdx = kd5x * rz;
        kdy = kd5y * rz;
        kdz = kd5z * zL[2 * ZR + zs(kh)];
      }
      T hxn, hyn, hzn;
      const int c = tid, cin = tid + 1, cjn = tid + W, rh = tid + W;
      h_point<T>(nq[c], nq[G.N3 + c], nq[2 * G.N3 + c], np_[c], np_[G.N3 + c],
                 nq[2 * G.N3 + cjn], nq[2 * G.N3 + cin], nq[G.N3 + cin], nq[cjn], ho[rh],
                 ho[G.N2 + rh], ho[2 * G.N2 + rh], A.imu2, A.imu2, A.imu2, gx > 0, gyB > 0,
                 kh > 0, kdx, kdy, kdz, hxn, hyn, hzn);
      const int64_t gk = sxy * (int64_t)kh;
      const uint32_t o = fresh(p3 * ES);
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

}  // namespace fit
