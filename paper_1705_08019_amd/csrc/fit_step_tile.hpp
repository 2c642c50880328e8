// Tile body of the fused single-pass leapfrog step, shared by the per-grid
// kernel (fit_step.hip) and the batched multi-grid kernel (fit_batch.hip).
// See fit_step.hip for the algorithm.
#pragma once

#include "fit_internal.hpp"
#include "fit_point.hpp"

namespace fit {

__device__ __forceinline__ void nadd_s(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// Global-memory access through address-space-1 pointers: the batched kernel
// reads its field pointers from a device table, where the compiler cannot
// prove them global and would emit flat accesses (which share the LDS wait
// counter and so stall every LDS wait on the plane prefetch).
template <typename T>
__device__ __forceinline__ T gld(const T* p, int64_t i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}
template <typename T>
__device__ __forceinline__ void gst(T* p, int64_t i, T v) {
  ((__attribute__((address_space(1))) T*)p)[i] = v;
}

// Ring entries of one plane staged per thread: RP = (tw+2)(ty+2) <= 3 nthr
// whenever tw ty <= nthr and tw + ty + 2 <= nthr (the launchers check both).
constexpr int kRingPerThread = 3;

// One tw x ty column tile of one z-chunk: tile coordinates (tx, tyi, kz);
// sm = dynamic LDS of step_lds_bytes(); part = this tile's partial-sum row
// (ENERGY: kEnergyAll every term, kEnergyHCross only the h cross term); prow = this workgroup's probe accumulator row (PROBE only),
// to which the step adds pscale times its probe term.  The workgroup's threads (any 2-D shape, a multiple
// of 64 and at least tw ty of them, also at least tw + ty + 1) are numbered
// linearly; thread t < tw ty owns column (t mod tw, t div tw) of the tile, the
// rest only help to stage planes (row-packed tiles of the batched kernel,
// whose tile width is a grid's whole x extent, leave such threads over).
template <typename T, bool LOSSY, int ENERGY, bool PROBE, bool NU = false>
__device__ __forceinline__ void step_tile(const SArgs<T>& A, int tx, int tyi, int kz, T* sm,
                                          double* part, double* prow) {
  const Dims d = A.d;
  const int TY = A.t.ty;
  const int TW = A.t.tw;                 // tile width (x) = blockDim.x
  const int RW = TW + 2, RP = RW * (TY + 2);
  const int EW = TW + 1, EP = EW * (TY + 1);
  T* hL = sm;                          // [3][3][RP]  h^(m+1/2), planes k, k-1, k-2 rotating
  T* cL = hL + 9 * RP;                 // [3][RP]     eps0 eps_r
  T* sL = cL + 3 * RP;                 // [3][RP]     sigma (lossy only)
  T* nL = sL + (LOSSY ? 3 * RP : 0);   // [2][3][EP]  e^(m+1), planes k, k-1
  T* zL = nL + 2 * 3 * EP;             // tensor grid: [3][kc + 1] per-plane factors

  const int i0 = tx * TW, j0 = tyi * TY;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  const int tid = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int nthr = (int)(blockDim.x * blockDim.y);
  const bool act = tid < TW * TY;      // owns a column of the tile
  const int lx = tid % TW, ly = tid / TW;
  const int i = i0 + lx, j = j0 + ly;
  const bool own = act && (i < d.nx) && (j < d.ny);
  const int64_t sx = d.sx, sxy = d.sxy;

  // one extra e^(m+1) point per thread for the +y halo row / +x halo column
  const int nhalo = TW + TY + 1;
  const bool has_h = tid < nhalo;
  const int hx_ = tid < TW ? tid : TW;
  const int hy_ = tid < TW ? TY : tid - TW;
  const int hi = i0 + hx_, hj = j0 + hy_;
  const bool hvalid = has_h && hi < d.nx && hj < d.ny;

  auto ring = [&](int x, int y) { return (y + 1) * RW + (x + 1); };
  auto ext = [&](int x, int y) { return y * EW + x; };

  // metric: uniform constants, or (tensor grid) the own and halo point's
  // x / y factors, fixed over the z-march (indices clamped into the grid;
  // out-of-grid points are discarded anyway)
  // (the per-plane z factors below are products with precomputed per-axis
  // arrays: no division in the march)
  T kbox = A.kb[0], kboy = A.kb[1], kbhx = A.kb[0], kbhy = A.kb[1];
  double gex = A.ge[0], gey = A.ge[1];
  double hfx = 0.0, hfy = 0.0, hfz = 0.0;
  T kdxb = 0, kdyb = 0, kdzb = 0;
  if (NU) {
    const int ci = min(i, d.nx - 1), cj = min(j, d.ny - 1);
    const int chi = min(hi, d.nx - 1), chj = min(hj, d.ny - 1);
    kbox = (T)(A.kbs * A.nsq[0][ci]);
    kboy = (T)(A.kbs * A.nsq[1][cj]);
    kbhx = (T)(A.kbs * A.nsq[0][chi]);
    kbhy = (T)(A.kbs * A.nsq[1][chj]);
    gex = 0.25 / A.nsq[0][ci];
    gey = 0.25 / A.nsq[1][cj];
    hfx = 0.5 * A.ndl[0][ci] * A.nrw[1][cj];
    hfy = 0.5 * A.ndl[1][cj] * A.nrw[0][ci];
    hfz = 0.5 * A.nrw[0][ci] * A.nrw[1][cj];
    kdxb = (T)(A.kds * hfx);
    kdyb = (T)(A.kds * hfy);
    kdzb = (T)(A.kds * hfz);
    // per-plane z factors of planes k0 .. k1 (read after the first barrier)
    const int zp = A.t.kc + 1;
    for (int q = tid; q <= k1 - k0 && k0 + q < d.nz; q += nthr) {
      const int kk = k0 + q;
      zL[q] = (T)(A.kbs * A.nsq[2][kk]);
      zL[zp + q] = (T)A.nrw[2][kk];
      zL[2 * zp + q] = (T)A.ndl[2][kk];
    }
  }

  // ---- register staging of one plane: ring entries q = tid + r * nthr
  T pre[kRingPerThread][5];
  T eo[3], ho[3];
  auto fetch = [&](int k) {
#pragma unroll
    for (int r = 0; r < kRingPerThread; ++r) {
      const int q = tid + r * nthr;
      const int gx = i0 + (q % RW) - 1, gy = j0 + (q / RW) - 1;
      const bool in = q < RP && k >= 0 && k < d.nz && gx >= 0 && gx < d.nx && gy >= 0 &&
                      gy < d.ny;
      const int64_t g = gx + sx * gy + sxy * (int64_t)k;
      pre[r][0] = in ? gld(A.h0[0], g) : T(0);
      pre[r][1] = in ? gld(A.h0[1], g) : T(0);
      pre[r][2] = in ? gld(A.h0[2], g) : T(0);
      pre[r][3] = in ? gld(A.eps, g) : T(0);
      pre[r][4] = (LOSSY && in) ? gld(A.sig, g) : T(0);
    }
    const bool plane = k >= 0 && k < d.nz;
    const int64_t g = i + sx * j + sxy * (int64_t)k;
    const int64_t gh = hi + sx * hj + sxy * (int64_t)k;
    const bool lo = plane && own, lh = plane && hvalid;
    eo[0] = lo ? gld(A.e0[0], g) : T(0);
    eo[1] = lo ? gld(A.e0[1], g) : T(0);
    eo[2] = lo ? gld(A.e0[2], g) : T(0);
    ho[0] = lh ? gld(A.e0[0], gh) : T(0);
    ho[1] = lh ? gld(A.e0[1], gh) : T(0);
    ho[2] = lh ? gld(A.e0[2], gh) : T(0);
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int r = 0; r < kRingPerThread; ++r) {
      const int q = tid + r * nthr;
      if (q < RP) {
        hL[(buf * 3 + 0) * RP + q] = pre[r][0];
        hL[(buf * 3 + 1) * RP + q] = pre[r][1];
        hL[(buf * 3 + 2) * RP + q] = pre[r][2];
        cL[buf * RP + q] = pre[r][3];
        if (LOSSY) sL[buf * RP + q] = pre[r][4];
      }
    }
  };

  // e^(m+1) at ext point (x, y) of plane k; p = ring buffer of plane k, q of k-1.
  auto enew = [&](int x, int y, int k, int p, int q, T exo, T eyo, T ezo, bool valid, T& exn,
                  T& eyn, T& ezn, T& E4x, T& E4y, T& E4z, T& S4x, T& S4y, T& S4z, T kbx_,
                  T kby_, T kbz_) {
    const int r = ring(x, y), rim = ring(x - 1, y), rjm = ring(x, y - 1), rijm = ring(x - 1, y - 1);
    const T* hp = hL + p * 3 * RP;
    const T* hq = hL + q * 3 * RP;
    const T* cp = cL + p * RP;
    const T* cq = cL + q * RP;
    const T c = cp[r], c_im = cp[rim], c_jm = cp[rjm], c_ijm = cp[rijm];
    const T Sx = c + c_im, Sy = c + c_jm, Sxj = c_jm + c_ijm;
    const T pc = cq[r];
    const T sye = pc + cq[rjm], sxe = pc + cq[rim];
    E4x = sye + Sy;
    E4y = sxe + Sx;
    E4z = Sx + Sxj;
    S4x = S4y = S4z = T(0);
    if (LOSSY) {
      const T* sp = sL + p * RP;
      const T* sq = sL + q * RP;
      const T s = sp[r], s_im = sp[rim], s_jm = sp[rjm], s_ijm = sp[rijm];
      const T Sxs = s + s_im, Sys = s + s_jm;
      const T ps = sq[r];
      const T sys = ps + sq[rjm], sxs = ps + sq[rim];
      S4x = sys + Sys;
      S4y = sxs + Sxs;
      S4z = Sxs + (s_jm + s_ijm);
    }
    const int gi = i0 + x, gj = j0 + y;
    const int64_t g = gi + sx * gj + sxy * (int64_t)k;
    T jx = 0, jy = 0, jz = 0;
    if (valid && g == A.src_idx) {
      if (A.src_comp == 0) jx = A.src_val;
      if (A.src_comp == 1) jy = A.src_val;
      if (A.src_comp == 2) jz = A.src_val;
    }
    // keep denominators of out-of-grid points finite (their result is discarded)
    if (!valid) {
      E4x = E4y = E4z = T(1);
    }
    e_point<T, LOSSY>(hp[r], hp[RP + r], hp[2 * RP + r], hq[r], hq[RP + r], hp[rjm],
                      hp[RP + rim], hp[2 * RP + rjm], hp[2 * RP + rim], E4x, E4y, E4z, S4x, S4y,
                      S4z, exo, eyo, ezo, jx, jy, jz, valid && gj > 0 && k > 0,
                      valid && gi > 0 && k > 0, valid && gi > 0 && gj > 0, kbx_, kby_, kbz_,
                      A.hs, exn, eyn, ezn);
  };

  double acc[kPartTerms] = {0};
  double cmp[kPartTerms] = {0};
  bool pi_x = false, pi_yz = false, pj_y = false, pj_xz = false;
  if (PROBE) {
    pi_x = i >= A.probe.lo[0] && i + 1 <= A.probe.hi[0];
    pi_yz = i >= A.probe.lo[0] && i <= A.probe.hi[0];
    pj_y = j >= A.probe.lo[1] && j + 1 <= A.probe.hi[1];
    pj_xz = j >= A.probe.lo[1] && j <= A.probe.hi[1];
  }

  // prologue: plane k0 - 1 (zeros below the grid) into ring buffer 2, prefetch plane k0
  int bp = 2;          // ring buffer of plane k - 1
  int bc = 0;          // ring buffer of plane k
  fetch(k0 - 1);
  stage(bp);
  fetch(k0);

  for (int k = k0; k <= k1; ++k) {
    const bool plane = k < d.nz;
    const int ep = k & 1;          // ext buffer of plane k (k-1 in ep ^ 1)
    // plane k: registers -> LDS; keep e^m of the own / halo point
    stage(bc);
    const T eo0 = eo[0], eo1 = eo[1], eo2 = eo[2];
    const T ho0 = ho[0], ho1 = ho[1], ho2 = ho[2];
    // prefetch plane k+1 (in flight during the compute below)
    if (k + 1 <= k1) fetch(k + 1);
    __syncthreads();
    T* np_ = nL + ep * 3 * EP;
    const int64_t g = i + sx * j + sxy * (int64_t)k;
    T kbz = A.kb[2];
    double gez = A.ge[2];
    if (NU && plane) {
      kbz = zL[k - k0];
      if (ENERGY == kEnergyAll || PROBE) gez = 0.25 / A.nsq[2][k];
    }
    if (act) {
      T exn = 0, eyn = 0, ezn = 0, E4x, E4y, E4z, S4x, S4y, S4z;
      if (plane) enew(lx, ly, k, bc, bp, eo0, eo1, eo2, own, exn, eyn, ezn, E4x, E4y, E4z, S4x,
                      S4y, S4z, kbox, kboy, kbz);
      const int e = ext(lx, ly);
      np_[e] = exn;
      np_[EP + e] = eyn;
      np_[2 * EP + e] = ezn;
      if (plane && own && k < k1) {
        gst(A.e1[0], g, exn);
        gst(A.e1[1], g, eyn);
        gst(A.e1[2], g, ezn);
        if (ENERGY == kEnergyAll) {
          const double mx = gex * (double)E4x, my = gey * (double)E4y, mz = gez * (double)E4z;
          // e^m of dead edges (PEC walls, phantom slots) is selected away, not
          // multiplied by a zero weight: whatever such a slot holds stays out
          const double ox = j > 0 && k > 0 ? (double)eo0 : 0.0;
          const double oy = i > 0 && k > 0 ? (double)eo1 : 0.0;
          const double oz = i > 0 && j > 0 ? (double)eo2 : 0.0;
          const double nx_ = exn, ny_ = eyn, nz_ = ezn;
          nadd_s(acc[PE_EE_MM], cmp[PE_EE_MM], mx * ox * ox + my * oy * oy + mz * oz * oz);
          nadd_s(acc[PE_EE_MM1], cmp[PE_EE_MM1], mx * ox * nx_ + my * oy * ny_ + mz * oz * nz_);
          nadd_s(acc[PE_EE_M1M1], cmp[PE_EE_M1M1],
                 mx * nx_ * nx_ + my * ny_ * ny_ + mz * nz_ * nz_);
          if (LOSSY) {
            const double bx = 0.5 * (ox + nx_), by = 0.5 * (oy + ny_), bz = 0.5 * (oz + nz_);
            nadd_s(acc[PE_LOSS], cmp[PE_LOSS],
                   gex * (double)S4x * bx * bx + gey * (double)S4y * by * by +
                       gez * (double)S4z * bz * bz);
          }
          // The source term is selected, not branched to: every lane adds
          // (exactly) 0 except the source edge's.  A branch here left the
          // block divergent on one lane, and under the register pressure of
          // the FP32 lossy energy+probe variant the gfx950 code generator
          // placed register copies (of the h-update coefficient among
          // others) inside that one-lane block, before the exec mask was
          // restored, so every other lane later read stale registers.
          const double bs = A.src_comp == 0 ? 0.5 * (ox + nx_)
                          : A.src_comp == 1 ? 0.5 * (oy + ny_) : 0.5 * (oz + nz_);
          nadd_s(acc[PE_SRC], cmp[PE_SRC], g == A.src_idx ? bs * A.src_val_d : 0.0);
        }
        if (PROBE) {
          const bool kx = k >= A.probe.lo[2] && k <= A.probe.hi[2];
          const bool kz_ = k >= A.probe.lo[2] && k + 1 <= A.probe.hi[2];
          const double nx_ = exn, ny_ = eyn, nz_ = ezn;
          double pv = 0.0;
          if (pi_x && pj_xz && kx) pv += gex * (double)E4x * nx_ * nx_;
          if (pi_yz && pj_y && kx) pv += gey * (double)E4y * ny_ * ny_;
          if (pi_yz && pj_xz && kz_) pv += gez * (double)E4z * nz_ * nz_;
          nadd_s(acc[PE_PROBE], cmp[PE_PROBE], pv);
        }
      }
    }
    if (has_h) {
      T exn = 0, eyn = 0, ezn = 0, E4x, E4y, E4z, S4x, S4y, S4z;
      if (plane) enew(hx_, hy_, k, bc, bp, ho0, ho1, ho2, hvalid, exn, eyn, ezn, E4x, E4y, E4z,
                      S4x, S4y, S4z, kbhx, kbhy, kbz);
      const int e = ext(hx_, hy_);
      np_[e] = exn;
      np_[EP + e] = eyn;
      np_[2 * EP + e] = ezn;
    }
    __syncthreads();
    // h^(m+3/2) of plane k-1 from e^(m+1) of planes k-1 (nq) and k (np_)
    const int km = k - 1;
    if (k > k0 && own) {
      const T* nq = nL + (ep ^ 1) * 3 * EP;
      const int e = ext(lx, ly), e_in = ext(lx + 1, ly), e_jn = ext(lx, ly + 1);
      const int r = ring(lx, ly);
      const T* hq = hL + bp * 3 * RP;
      const T hxo = hq[r], hyo = hq[RP + r], hzo = hq[2 * RP + r];
      T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
      double gfx = A.gf2[0], gfy = A.gf2[1], gfz = A.gf2[2];
      if (NU) {
        const int zp = A.t.kc + 1;
        const T rz = zL[zp + km - k0];
        kdx = kdxb * rz;
        kdy = kdyb * rz;
        kdz = kdzb * zL[2 * zp + km - k0];
        if (ENERGY != kEnergyNone) {
          gfx = hfx * A.nrw[2][km];
          gfy = hfy * A.nrw[2][km];
          gfz = hfz * A.ndl[2][km];
        }
      }
      T hxn, hyn, hzn;
      h_point<T>(nq[e], nq[EP + e], nq[2 * EP + e], np_[e], np_[EP + e], nq[2 * EP + e_jn],
                 nq[2 * EP + e_in], nq[EP + e_in], nq[e_jn], hxo, hyo, hzo, A.imu2, A.imu2,
                 A.imu2, i > 0, j > 0, km > 0, kdx, kdy, kdz, hxn, hyn, hzn);
      const int64_t gm = i + sx * j + sxy * (int64_t)km;
      gst(A.h1[0], gm, hxn);
      gst(A.h1[1], gm, hyn);
      gst(A.h1[2], gm, hzn);
      if (ENERGY != kEnergyNone) {
        const double wx = i > 0 ? 1.0 / (gfx * (double)A.imu2) : 0.0;
        const double wy = j > 0 ? 1.0 / (gfy * (double)A.imu2) : 0.0;
        const double wz = km > 0 ? 1.0 / (gfz * (double)A.imu2) : 0.0;
        const double ox = i > 0 ? (double)hxo : 0.0, oy = j > 0 ? (double)hyo : 0.0;
        const double oz = km > 0 ? (double)hzo : 0.0, nx_ = hxn, ny_ = hyn, nz_ = hzn;
        if (ENERGY == kEnergyAll)
          nadd_s(acc[PS_HH_CC], cmp[PS_HH_CC], wx * ox * ox + wy * oy * oy + wz * oz * oz);
        nadd_s(acc[PS_HH_CN], cmp[PS_HH_CN], wx * ox * nx_ + wy * oy * ny_ + wz * oz * nz_);
        if (ENERGY == kEnergyAll)
          nadd_s(acc[PS_HH_NN], cmp[PS_HH_NN], wx * nx_ * nx_ + wy * ny_ * ny_ + wz * nz_ * nz_);
      }
    }
    // rotate ring buffers: plane k becomes k-1; the oldest buffer takes k+1
    const int nb_ = 3 - bc - bp;
    bp = bc;
    bc = nb_;
  }

  if (ENERGY != kEnergyNone || PROBE) {
    // block sum of the 9 terms, fixed order: per wave, then over waves (the
    // terms a mode does not form are zero)
    __shared__ double red[16][9];
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    double v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      double x = acc[t] + cmp[t];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      v[t] = x;
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < 9; ++t) red[wave][t] = v[t];
    }
    __syncthreads();
    if (tid < 9) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w][tid];
      if (ENERGY != kEnergyNone) part[tid] = s;
      if (PROBE && tid == PE_PROBE) {
        double ps = prow[0], pc = prow[1];
        nadd_s(ps, pc, A.pscale * s);
        prow[0] = ps;
        prow[1] = pc;
      }
    }
  }
}


}  // namespace fit
