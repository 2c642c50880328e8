// Two leapfrog steps per pass (temporal blocking of the Sec. II-A
// recurrence): one launch reads (e^m, h^(m+1/2)) and the materials once and
// writes (e^(m+2), h^(m+5/2)); the intermediate state (e^(m+1), h^(m+3/2))
// lives only in LDS.  Per cell and pair of steps this moves the 56 B of one
// fused step instead of 112 B.
//
// A workgroup (threads numbered linearly; one per point of the (TW + 4) x
// (TY + 3) thread grid, or one per two points for larger tiles) owns a
// TW x TY column tile and marches a
// chunk [k0, k1) of z-planes with a lag of two planes between what it reads
// and what it stores.  In local coordinates (x along i, y along j) the regions are
//   X4: x in [-2, TW+1], y in [-2, TY+1]  staged h^(m+1/2), eps, sigma
//   R1: x in [-1, TW+1], y in [-1, TY+1]  e^(m+1)       (needs X4)
//   R2: x in [-1, TW],   y in [-1, TY]    h^(m+3/2)     (needs R1, X4)
//   R3: x in [0, TW],    y in [0, TY]     e^(m+2)       (needs R2, R1, X4)
//   tile                                  h^(m+5/2)     (needs R3, R2)
// Point q of the thread grid is (x, y) = (q % W - 2, q / W - 1), W = TW + 4;
// a thread owns the same points in every phase (each phase runs on the
// points that lie in its region), and every LDS array has the row stride W
// (a region keeps only its own rows), so each LDS access is q plus a
// constant: the lanes of a wave touch consecutive words.
// Because the points are the same in every phase, what a phase needs of a
// point itself comes from registers: the thread carries its own h^(m+1/2),
// e^(m+1), the 4-cell material sums, h^(m+3/2) and e^(m+2) of the latest
// planes, and reads only the +-x / +-y neighbours from LDS.  The materials
// are needed by the first e-update alone (the second reuses its sums), so
// h^(m+1/2), eps and sigma are staged for one plane.
// Iteration k forms e^(m+1) of plane k, h^(m+3/2) of plane k-1, e^(m+2) of
// plane k-1 and h^(m+5/2) of plane k-2, for k = k0-1 .. k1+1, with two
// barriers: one after staging, one before the second e-update.  Each
// h-update reads from LDS only the e plane formed one iteration earlier
// (double-buffered; the newer plane comes from the point's own registers),
// so neither follows its e-update with a barrier.
// The halo rows and columns are recomputed by every tile that needs them
// with the same contraction-pinned point functions and operand order as the
// single-step kernels, so the result is bitwise that of two single steps.
// Values outside the grid and on planes outside [0, nz) are zero (PEC), as
// in the single-step kernels.
#pragma once

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
// NTS: streaming store.  The outputs are not read again by the launch, so
// on large grids they should not take L2 lines from the staged planes the
// neighbouring tiles still read (their halos).  Ordinary stores let L2
// merge the parts of one line that neighbouring tiles write, which matters
// where a tile's row segments straddle lines (grids whose x extent is not
// a multiple of the line's cells: the batched grids).
template <bool NTS, typename T>
__device__ __forceinline__ void pst(T* base, uint32_t off, T v) {
  using C1 = __attribute__((address_space(1))) char;
  using T1 = __attribute__((address_space(1))) T;
  if constexpr (NTS)
    __builtin_nontemporal_store(v, (T1*)((C1*)base + off));
  else
    *(T1*)((C1*)base + off) = v;
}

// Two fused steps of tile (tx, tyi) and z-chunk kz of the tiling A.t;
// sm: the workgroup's dynamic LDS (step2_lds_bytes).  CTW, CTY > 0 fix the
// tile at compile time (every LDS offset an immediate), 0 takes it from the
// tiling.  NP: points per thread -- thread t owns the points q = t + p nthr,
// p < NP, of the thread grid (tiles whose R1 region has more than 1024
// points, e.g. 64 x 16, take NP = 2); each point keeps its own carried
// values, and every phase runs over the thread's points in turn.  EN
// (uniform grids, NP = 1): also form the energy terms of a trace row at the
// second step -- the e terms where the second e-update stores its point,
// the h terms where the second h-update does, and the row's pending h cross
// term where the first h-update forms an own point of [k0, k1) -- in FP64
// with the compensated sums of the single step, and write the workgroup's
// block sums (kPartTerms) to part.  NTS: the outputs by streaming stores
// (see pst).
template <typename T, bool LOSSY, bool NU, int CTW, int CTY, int NP = 1, bool EN = false,
          bool NTS = true>
__device__ __forceinline__ void step2_tile(const S2Args<T>& A, int tx, int tyi, int kz, T* sm,
                                           double* part = nullptr) {
  static_assert(!EN || (NP == 1 && !NU), "energy pairs: uniform grids, one point per thread");
  const Dims d = A.d;
  const int TW = CTW > 0 ? CTW : A.t.tw, TY = CTY > 0 ? CTY : A.t.ty;
  const S2Geom G = s2_geom(TW, TY);
  T* h0L = sm;                                // [3][N4]      h^(m+1/2) of plane k
  T* cL = h0L + 3 * G.N4;                     // [N4]         eps0 eps_r V of plane k
  T* sL = cL + G.N4;                          // [N4]         sigma V of plane k (lossy)
  T* e1L = sL + (LOSSY ? G.N4 : 0);           // [2][3][N1]   e^(m+1), planes k, k-1
  T* h1L = e1L + 6 * G.N1;                    // [3][N2]      h^(m+3/2) of plane k-1
  T* e2L = h1L + 3 * G.N2;                    // [2][3][N3]   e^(m+2), planes k-1, k-2
  T* zL = e2L + 6 * G.N3;                     // tensor grid: [3][kS2ZRing] per-plane factors

  const int i0 = tx * TW, j0 = tyi * TY;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  const int tid = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int nthr = (int)(blockDim.x * blockDim.y);   // NP nthr >= N1
  const int64_t sx = d.sx, sxy = d.sxy;

  auto hb = [](int k) { return k & 1; };   // e1 / e2 buffer of plane k
  auto in_grid = [&](int gx, int gy) { return gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny; };

  // ---- the thread's points (x, y) = (q % W - 2, q / W - 1), the same in
  // every phase; grid points as in-plane element indices p (gx + sx gy)
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
  int gxp[NP], gyp[NP], i4[NP], i1[NP], i3[NP];
  uint32_t pg[NP];
  bool at_s[NP], a1[NP], in1[NP], a2[NP], in2[NP], a3[NP], in3[NP], own[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int q = tid + p * nthr;
    const int row = q / W, x = q % W - 2, y = row - 1;
    const int gx = i0 + x, gy = j0 + y;
    gxp[p] = gx;
    gyp[p] = gy;
    const bool ing = in_grid(gx, gy);
    pg[p] = ing ? (uint32_t)(gx + sx * gy) : 0u;
    at_s[p] = ing && pg[p] == src_p;
    // R1 (e^(m+1)): x in [-1, TW+1], y in [-1, TY+1]
    a1[p] = row < TY + 3 && x >= -1;
    in1[p] = a1[p] && ing;
    // R2 (h^(m+3/2)): x in [-1, TW], y in [-1, TY]
    a2[p] = row < TY + 2 && x >= -1 && x <= TW;
    in2[p] = a2[p] && ing;
    // R3 (e^(m+2)): x in [0, TW], y in [0, TY]
    a3[p] = row >= 1 && row < TY + 2 && x >= 0 && x <= TW;
    in3[p] = a3[p] && ing;
    // the tile (h^(m+5/2), stored)
    own[p] = in3[p] && x < TW && y < TY;
    // LDS indices of the point: X4 q + W (neighbours -1: x - 1, -W: y - 1),
    // R1 and R2 q (+1: x + 1, +W: y + 1), R3 q - W
    i4[p] = q + W;
    i1[p] = q;
    i3[p] = q - W;
  }

  // ---- tensor-grid metric (as in the single fused step): x / y factors of
  // the points, z factors of planes k0 - 2 .. k1 + 1 in an LDS ring
  T kbx[NP], kby[NP], kdxb[NP], kdyb[NP], kdzb[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    kbx[p] = A.kb[0];
    kby[p] = A.kb[1];
    kdxb[p] = kdyb[p] = kdzb[p] = T(0);
    if (NU) {
      const int ix = min(max(gxp[p], 0), d.nx - 1), jy = min(max(gyp[p], 0), d.ny - 1);
      kbx[p] = (T)(A.kbs * A.nsq[0][ix]);
      kby[p] = (T)(A.kbs * A.nsq[1][jy]);
      kdxb[p] = (T)(A.kds * (0.5 * A.ndl[0][ix] * A.nrw[1][jy]));
      kdyb[p] = (T)(A.kds * (0.5 * A.ndl[1][jy] * A.nrw[0][ix]));
      kdzb[p] = (T)(A.kds * (0.5 * A.nrw[0][ix] * A.nrw[1][jy]));
    }
  }
  // the z factors of plane k sit in ring slot k mod kS2ZRing of zL (kb_z,
  // 1 / w_z, dual width): thread 0 fetches them with the plane and stages
  // them with it; a slot is rewritten three planes after its last reader
  // (the tile h-update of plane k - 2 may still run while plane k + 1 is
  // staged, so the ring holds four planes)
  constexpr int ZR = kS2ZRing;
  auto zs = [](int k) { return k & (ZR - 1); };
  double zraw[3] = {0.0, 0.0, 0.0};

  // ---- register staging of plane k: X4 entries (h x3, eps, sigma), the
  // points' e^m
  T ph[kS2Per][5];
  T pe[NP][3];
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
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const bool in = plane && in1[p];
      const uint32_t o = fresh(pg[p] * ES);
      pe[p][0] = in ? pld(A.e0[0] + gk, o) : T(0);
      pe[p][1] = in ? pld(A.e0[1] + gk, o) : T(0);
      pe[p][2] = in ? pld(A.e0[2] + gk, o) : T(0);
    }
  };
  auto stage = [&](int k) {
#pragma unroll
    for (int r = 0; r < kS2Per; ++r) {
      const int q = tid + r * nthr;
      if (q < G.N4) {
        h0L[q] = ph[r][0];
        h0L[G.N4 + q] = ph[r][1];
        h0L[2 * G.N4 + q] = ph[r][2];
        cL[q] = ph[r][3];
        if (LOSSY) sL[q] = ph[r][4];
      }
    }
    if (NU && tid == 0) {
      zL[zs(k)] = (T)(A.kbs * zraw[0]);
      zL[ZR + zs(k)] = (T)zraw[1];
      zL[2 * ZR + zs(k)] = (T)zraw[2];
    }
  };

  // ---- values of each point carried from plane to plane (zero below the
  // chunk's first planes until they are formed):
  // h^(m+1/2) of the previous plane; the 2-cell sums of eps (sigma) along
  // x and y of the previous plane (the lower half of the next plane's x / y
  // edge sums); e^(m+1), its 4-cell sums E4 (S4), h^(m+3/2) and e^(m+2) of
  // the latest planes formed
  T hq[NP][3], Sxq[NP], Syq[NP], Sxsq[NP], Sysq[NP];
  T e1p[NP][3], E4p[NP][3], S4p[NP][3], h1p[NP][3], e2p[NP][3];
  // the values formed in an iteration: assigned only where a point takes
  // part in a phase (its region and the plane range), and read only there
  // or, carried, by the same point's later phases, which run on a subset of
  // the same condition -- so they are initialised once, not per plane (a
  // per-plane reset cost a register move for every value and plane)
  T e1c[NP][3], E4c[NP][3], S4c[NP][3], hc[NP][3];
  T Sxc[NP], Syc[NP], Sxsc[NP], Sysc[NP];
  T h1c[NP][3], e2c[NP][3];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    Sxq[p] = Syq[p] = Sxsq[p] = Sysq[p] = T(0);
    Sxc[p] = Syc[p] = Sxsc[p] = Sysc[p] = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      hq[p][c] = e1p[p][c] = S4p[p][c] = h1p[p][c] = e2p[p][c] = T(0);
      E4p[p][c] = T(1);
      e1c[p][c] = S4c[p][c] = hc[p][c] = h1c[p][c] = e2c[p][c] = T(0);
      E4c[p][c] = T(1);
    }
  }

  // energy pairs: FP64 compensated sums of the tile's own points on planes
  // [k0, k1), the terms of the fused single step (same selects of dead
  // slots and operand order)
  double acc[kPartTerms] = {};
  double cmp[kPartTerms] = {};

  // prologue: plane k0 - 2 staged for its carried values, plane k0 - 1 in flight
  fetch(k0 - 2);
  stage(k0 - 2);
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (a1[p]) {
      const int j4 = i4[p];
      hq[p][0] = h0L[j4];
      hq[p][1] = h0L[G.N4 + j4];
      hq[p][2] = h0L[2 * G.N4 + j4];
      const T c = cL[j4];
      Sxq[p] = c + cL[j4 - 1];
      Syq[p] = c + cL[j4 - W];
      if (LOSSY) {
        const T s = sL[j4];
        Sxsq[p] = s + sL[j4 - 1];
        Sysq[p] = s + sL[j4 - W];
      }
    }
  }
  fetch(k0 - 1);
  __syncthreads();   // the single staging buffer is read before it is reused

  for (int k = k0 - 1; k <= k1 + 1; ++k) {
    stage(k);
    T e0[NP][3];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      e0[p][0] = pe[p][0];
      e0[p][1] = pe[p][1];
      e0[p][2] = pe[p][2];
    }
    if (k + 1 <= k1 + 1) fetch(k + 1);
    __syncthreads();

    // ---- e^(m+1) of plane k on R1 (same operand order as the single step)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (a1[p]) {
        const int j4 = i4[p];
        const bool valid = in1[p] && k >= 0 && k < d.nz;
        hc[p][0] = h0L[j4];
        hc[p][1] = h0L[G.N4 + j4];
        hc[p][2] = h0L[2 * G.N4 + j4];
        const T c = cL[j4], c_im = cL[j4 - 1], c_jm = cL[j4 - W], c_ijm = cL[j4 - W - 1];
        Sxc[p] = c + c_im;
        Syc[p] = c + c_jm;
        const T Sxj = c_jm + c_ijm;
        E4c[p][0] = Syq[p] + Syc[p];
        E4c[p][1] = Sxq[p] + Sxc[p];
        E4c[p][2] = Sxc[p] + Sxj;
        if (LOSSY) {
          const T s = sL[j4], s_im = sL[j4 - 1], s_jm = sL[j4 - W], s_ijm = sL[j4 - W - 1];
          Sxsc[p] = s + s_im;
          Sysc[p] = s + s_jm;
          S4c[p][0] = Sysq[p] + Sysc[p];
          S4c[p][1] = Sxsq[p] + Sxsc[p];
          S4c[p][2] = Sxsc[p] + (s_jm + s_ijm);
        }
        if (!valid) E4c[p][0] = E4c[p][1] = E4c[p][2] = T(1);
        T jx = 0, jy = 0, jz = 0;
        if (valid && at_s[p] && k == sk) {
          if (A.src_comp == 0) jx = A.src_val[0];
          if (A.src_comp == 1) jy = A.src_val[0];
          if (A.src_comp == 2) jz = A.src_val[0];
        }
        e_point<T, LOSSY>(hc[p][0], hc[p][1], hc[p][2], hq[p][0], hq[p][1], h0L[j4 - W],
                          h0L[G.N4 + j4 - 1], h0L[2 * G.N4 + j4 - W], h0L[2 * G.N4 + j4 - 1],
                          E4c[p][0], E4c[p][1], E4c[p][2], S4c[p][0], S4c[p][1], S4c[p][2],
                          e0[p][0], e0[p][1], e0[p][2], jx, jy, jz,
                          valid && gyp[p] > 0 && k > 0, valid && gxp[p] > 0 && k > 0,
                          valid && gxp[p] > 0 && gyp[p] > 0, kbx[p], kby[p],
                          NU ? zL[zs(k)] : A.kb[2], A.hs, e1c[p][0], e1c[p][1], e1c[p][2]);
        T* out = e1L + hb(k) * 3 * G.N1;
        out[i1[p]] = e1c[p][0];
        out[G.N1 + i1[p]] = e1c[p][1];
        out[2 * G.N1 + i1[p]] = e1c[p][2];
      }
    }
    // (no barrier: the h-update below reads e^(m+1) of plane k - 1 alone from
    // LDS, the other buffer, written before the barriers of the previous
    // iteration; plane k enters through the point's own registers)

    // ---- h^(m+3/2) of plane km = k - 1 on R2: e^(m+1) of planes km (the
    // point from registers, its +x / +y neighbours from LDS) and k
    const int km = k - 1;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (km >= k0 - 1 && a2[p]) {
        const T* nq = e1L + hb(km) * 3 * G.N1;
        const int j1 = i1[p];
        const bool valid = in2[p] && km >= 0 && km < d.nz;
        T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
        if (NU) {
          const T rz = zL[ZR + zs(km)];
          kdx = kdxb[p] * rz;
          kdy = kdyb[p] * rz;
          kdz = kdzb[p] * zL[2 * ZR + zs(km)];
        }
        h_point<T>(e1p[p][0], e1p[p][1], e1p[p][2], e1c[p][0], e1c[p][1], nq[2 * G.N1 + j1 + W],
                   nq[2 * G.N1 + j1 + 1], nq[G.N1 + j1 + 1], nq[j1 + W], hq[p][0], hq[p][1],
                   hq[p][2], A.imu2, A.imu2, A.imu2, valid && gxp[p] > 0, valid && gyp[p] > 0,
                   valid && km > 0, kdx, kdy, kdz, h1c[p][0], h1c[p][1], h1c[p][2]);
        h1L[j1] = h1c[p][0];
        h1L[G.N2 + j1] = h1c[p][1];
        h1L[2 * G.N2 + j1] = h1c[p][2];
        if (EN && own[p] && km >= k0 && km < k1) {
          // <h^(m+1/2), h^(m+3/2)> of the first step
          const double wx = gxp[p] > 0 ? 1.0 / (A.gf2[0] * (double)A.imu2) : 0.0;
          const double wy = gyp[p] > 0 ? 1.0 / (A.gf2[1] * (double)A.imu2) : 0.0;
          const double wz = km > 0 ? 1.0 / (A.gf2[2] * (double)A.imu2) : 0.0;
          const double ox = gxp[p] > 0 ? (double)hq[p][0] : 0.0;
          const double oy = gyp[p] > 0 ? (double)hq[p][1] : 0.0;
          const double oz = km > 0 ? (double)hq[p][2] : 0.0;
          const double nx_ = h1c[p][0], ny_ = h1c[p][1], nz_ = h1c[p][2];
          nadd_s(acc[kPairHCross], cmp[kPairHCross], wx * ox * nx_ + wy * oy * ny_ + wz * oz * nz_);
        }
      }
    }
    __syncthreads();

    // ---- e^(m+2) of plane km on R3: h^(m+3/2) of planes km (the point from
    // registers, its -x / -y neighbours from LDS) and km - 1, e^(m+1) and
    // the 4-cell sums of plane km from registers; the tile part of planes
    // [k0, k1) is stored
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (km >= k0 && a3[p]) {
        const int j1 = i1[p];
        const bool valid = in3[p] && km >= 0 && km < d.nz;
        T jx = 0, jy = 0, jz = 0;
        if (valid && at_s[p] && km == sk) {
          if (A.src_comp == 0) jx = A.src_val[1];
          if (A.src_comp == 1) jy = A.src_val[1];
          if (A.src_comp == 2) jz = A.src_val[1];
        }
        e_point<T, LOSSY>(h1c[p][0], h1c[p][1], h1c[p][2], h1p[p][0], h1p[p][1], h1L[j1 - W],
                          h1L[G.N2 + j1 - 1], h1L[2 * G.N2 + j1 - W], h1L[2 * G.N2 + j1 - 1],
                          E4p[p][0], E4p[p][1], E4p[p][2], S4p[p][0], S4p[p][1], S4p[p][2],
                          e1p[p][0], e1p[p][1], e1p[p][2], jx, jy, jz,
                          valid && gyp[p] > 0 && km > 0, valid && gxp[p] > 0 && km > 0,
                          valid && gxp[p] > 0 && gyp[p] > 0, kbx[p], kby[p],
                          NU ? zL[zs(km)] : A.kb[2], A.hs, e2c[p][0], e2c[p][1], e2c[p][2]);
        T* out = e2L + hb(km) * 3 * G.N3;
        out[i3[p]] = e2c[p][0];
        out[G.N3 + i3[p]] = e2c[p][1];
        out[2 * G.N3 + i3[p]] = e2c[p][2];
        if (own[p] && km < k1) {
          const int64_t gk = sxy * (int64_t)km;
          const uint32_t o = fresh(pg[p] * ES);
          pst<NTS>(A.e2[0] + gk, o, e2c[p][0]);
          pst<NTS>(A.e2[1] + gk, o, e2c[p][1]);
          pst<NTS>(A.e2[2] + gk, o, e2c[p][2]);
          if (EN) {
            // the second step's e terms: e^(m+1) (old), e^(m+2) (new)
            const double mx = A.ge[0] * (double)E4p[p][0], my = A.ge[1] * (double)E4p[p][1],
                         mz = A.ge[2] * (double)E4p[p][2];
            const double ox = gyp[p] > 0 && km > 0 ? (double)e1p[p][0] : 0.0;
            const double oy = gxp[p] > 0 && km > 0 ? (double)e1p[p][1] : 0.0;
            const double oz = gxp[p] > 0 && gyp[p] > 0 ? (double)e1p[p][2] : 0.0;
            const double nx_ = e2c[p][0], ny_ = e2c[p][1], nz_ = e2c[p][2];
            nadd_s(acc[PE_EE_MM], cmp[PE_EE_MM], mx * ox * ox + my * oy * oy + mz * oz * oz);
            nadd_s(acc[PE_EE_MM1], cmp[PE_EE_MM1], mx * ox * nx_ + my * oy * ny_ + mz * oz * nz_);
            nadd_s(acc[PE_EE_M1M1], cmp[PE_EE_M1M1],
                   mx * nx_ * nx_ + my * ny_ * ny_ + mz * nz_ * nz_);
            if (LOSSY) {
              const double bx = 0.5 * (ox + nx_), by = 0.5 * (oy + ny_), bz = 0.5 * (oz + nz_);
              nadd_s(acc[PE_LOSS], cmp[PE_LOSS],
                     A.ge[0] * (double)S4p[p][0] * bx * bx + A.ge[1] * (double)S4p[p][1] * by * by +
                         A.ge[2] * (double)S4p[p][2] * bz * bz);
            }
            const double bs = A.src_comp == 0 ? 0.5 * (ox + nx_)
                            : A.src_comp == 1 ? 0.5 * (oy + ny_) : 0.5 * (oz + nz_);
            nadd_s(acc[PE_SRC], cmp[PE_SRC],
                   at_s[p] && km == sk ? bs * (double)A.src_val[1] : 0.0);
          }
        }
      }
    }

    // ---- h^(m+5/2) of plane kh = k - 2 on the tile: e^(m+2) of planes kh
    // (the point from registers, its +x / +y neighbours from LDS, written one
    // iteration earlier) and kh + 1 (registers), h^(m+3/2) of plane kh
    const int kh = k - 2;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (kh >= k0 && kh < k1 && own[p]) {
        const T* nq = e2L + hb(kh) * 3 * G.N3;
        const int j3 = i3[p];
        T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
        if (NU) {
          const T rz = zL[ZR + zs(kh)];
          kdx = kdxb[p] * rz;
          kdy = kdyb[p] * rz;
          kdz = kdzb[p] * zL[2 * ZR + zs(kh)];
        }
        T hxn, hyn, hzn;
        h_point<T>(e2p[p][0], e2p[p][1], e2p[p][2], e2c[p][0], e2c[p][1], nq[2 * G.N3 + j3 + W],
                   nq[2 * G.N3 + j3 + 1], nq[G.N3 + j3 + 1], nq[j3 + W], h1p[p][0], h1p[p][1],
                   h1p[p][2], A.imu2, A.imu2, A.imu2, gxp[p] > 0, gyp[p] > 0, kh > 0, kdx, kdy,
                   kdz, hxn, hyn, hzn);
        const int64_t gk = sxy * (int64_t)kh;
        const uint32_t o = fresh(pg[p] * ES);
        pst<NTS>(A.h2[0] + gk, o, hxn);
        pst<NTS>(A.h2[1] + gk, o, hyn);
        pst<NTS>(A.h2[2] + gk, o, hzn);
        if (EN) {
          // the second step's h terms: h^(m+3/2) (old), h^(m+5/2) (new)
          const double wx = gxp[p] > 0 ? 1.0 / (A.gf2[0] * (double)A.imu2) : 0.0;
          const double wy = gyp[p] > 0 ? 1.0 / (A.gf2[1] * (double)A.imu2) : 0.0;
          const double wz = kh > 0 ? 1.0 / (A.gf2[2] * (double)A.imu2) : 0.0;
          const double ox = gxp[p] > 0 ? (double)h1p[p][0] : 0.0;
          const double oy = gyp[p] > 0 ? (double)h1p[p][1] : 0.0;
          const double oz = kh > 0 ? (double)h1p[p][2] : 0.0;
          const double nx_ = hxn, ny_ = hyn, nz_ = hzn;
          nadd_s(acc[PS_HH_CC], cmp[PS_HH_CC], wx * ox * ox + wy * oy * oy + wz * oz * oz);
          nadd_s(acc[PS_HH_CN], cmp[PS_HH_CN], wx * ox * nx_ + wy * oy * ny_ + wz * oz * nz_);
          nadd_s(acc[PS_HH_NN], cmp[PS_HH_NN], wx * nx_ * nx_ + wy * ny_ * ny_ + wz * nz_ * nz_);
        }
      }
    }

    // ---- carry the points' values to the next plane
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        hq[p][c] = hc[p][c];
        e1p[p][c] = e1c[p][c];
        E4p[p][c] = E4c[p][c];
        S4p[p][c] = S4c[p][c];
        h1p[p][c] = h1c[p][c];
        e2p[p][c] = e2c[p][c];
      }
      Sxq[p] = Sxc[p];
      Syq[p] = Syc[p];
      Sxsq[p] = Sxsc[p];
      Sysq[p] = Sysc[p];
    }
  }

  if constexpr (EN) {
    // block sums of the terms in a fixed order: per wave, then over waves
    __shared__ double red[16][kPartTerms];
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    double v[kPartTerms];
#pragma unroll
    for (int t = 0; t < kPartTerms; ++t) {
      double x = acc[t] + cmp[t];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      v[t] = x;
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < kPartTerms; ++t) red[wave][t] = v[t];
    }
    __syncthreads();
    if (tid < kPartTerms) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w][tid];
      part[tid] = s;
    }
  }
}

}  // namespace fit
