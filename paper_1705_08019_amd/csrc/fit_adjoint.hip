// Discrete adjoint of the leapfrog (reverse time) and the per-cell gradient of
// the probe objective J = dt sum_{m>=1} sum_probe M_eps (e^m)^2.
//
// Forward step (Sec. II-A, loss at e^(m+1/2)):  e^(m+1) = a e^m + b s^m with
// s^m = C~ h^(m+1/2) - j_s, a = (M_eps - dt/2 M_sigma) / D, b = dt / D,
// D = M_eps + dt/2 M_sigma;  h^(m+3/2) = h^(m+1/2) - d C e^(m+1), d = dt M_mu^{-1}.
// Reverse step m (lambda = dJ/de, mu = dJ/dh, both zero beyond the horizon):
//   lambda^(m+1) = a lambda^(m+2) - C~ (d mu^(m+3/2)) + 2 dt w M_eps e^(m+1)
//   mu^(m+1/2)   = mu^(m+3/2) + C (b lambda^(m+1))
//   dJ/dM_eps(edge) += lambda^(m+1) (da/dM_eps e^m + db/dM_eps s^m) + dt w (e^(m+1))^2
//   dJ/dM_sig(edge) += lambda^(m+1) (da/dM_sig e^m + db/dM_sig s^m)
// and, since M_eps of an edge is (g_a / 4) times the sum of its 4 cells'
// eps0 eps_r (M_sigma likewise without eps0), each step's edge sensitivities
// go straight onto the cells: dJ/deps_r(c) += eps0 (g_a / 4) dJ/dM_eps summed
// over the 12 edges of cell c (FP64 accumulators, one per cell and quantity).
//
// Because C~ = C^T the reverse step has the shape of the forward one (the
// dual curl with backward differences feeds lambda, the primal curl with
// forward differences feeds mu), so it runs as one fused z-march per step
// like k_step: a tw x ty column tile walks its z-chunk; per plane k it stages
// h^(m+1/2), mu^(m+3/2), eps and sigma of plane k in LDS (double-buffered;
// the z neighbours below are carried in registers), forms lambda^(m+1),
// tau = b lambda^(m+1) and the FP64 edge sensitivities of plane k on the tile
// and on a +x / +y halo (recomputed, so tiles need no ordering; the halo points
// have threads of their own, so no wave does two points), then mu^(m+1/2) of
// plane k-1 from tau of planes k-1 (LDS) and k (registers), and adds the
// sensitivities of the 12 edges of each cell of plane k-1 to the per-cell
// accumulators.  lambda and mu ping-pong between two buffer sets.
// mu (permeability) must be uniform here.
#include <algorithm>

#include "fit_internal.hpp"
#include "fit_point.hpp"

namespace fit {

// Global access at a wave-uniform plane base (scalar registers) plus a
// per-thread 32-bit byte offset within the plane (fit_adjoint_begin checks
// that a plane of FP64 values spans < 4 GiB): no 64-bit vector address per
// access.  `afresh` marks the loop-invariant offset as redefined at each
// access (an empty asm) so that its zero-extension stays next to the access
// instead of being hoisted and shared, which brings the 64-bit form back.
__device__ __forceinline__ uint32_t afresh(uint32_t off) {
  asm volatile("" : "+v"(off));
  return off;
}
template <typename T>
__device__ __forceinline__ T ald(const T* base, uint32_t off) {
  using C1 = const __attribute__((address_space(1))) char;
  using T1 = const __attribute__((address_space(1))) T;
  return *(T1*)((C1*)base + afresh(off));
}
template <typename T>
__device__ __forceinline__ void ast(T* base, uint32_t off, T v) {
  using C1 = __attribute__((address_space(1))) char;
  using T1 = __attribute__((address_space(1))) T;
  *(T1*)((C1*)base + afresh(off)) = v;
}

// 1 / x for x > 0 in FP64: the hardware estimate refined by two Newton steps
// (error a few ulp; the FP64 divide sequence costs several times more).
__device__ __forceinline__ double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// z-neighbour (plane k-1) values of one point, carried between iterations.
template <typename T>
struct AdjPrev {
  T hx, hy, ux, uy, uz, Sx, Sy, Sxs, Sys;
};

// Threads: t < tw ty own tile column (t mod tw, t div tw); the next
// tw + ty + 1 threads own one halo point each (the +y row, then the +x
// column with the corner); the rest only stage planes.
// FP32: at most 128 VGPRs (4 waves per SIMD), so that two 512-thread
// workgroups are resident per CU.
template <typename T, bool LOSSY>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_adj(AdjArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Dims d = A.d;
  const int TW = A.t.tw, TY = A.t.ty;
  const int RW = TW + 2, RP = RW * (TY + 2);
  const int EW = TW + 1, EP = EW * (TY + 1);
  double* qL = reinterpret_cast<double*>(smem_raw);   // [6][EP] scaled sensitivities of plane k
  T* rL0 = reinterpret_cast<T*>(qL + 6 * EP);         // [2][8][RP] h xyz, mu xyz, eps, sigma
  T* tL = rL0 + 16 * RP;                              // [2][3][EP] tau of planes k, k-1

  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr_ = lt / A.t.ntx;
  const int tyi = (int)(rr_ % A.t.nty);
  const int kz = (int)(rr_ / A.t.nty);
  const int i0 = tx * TW, j0 = tyi * TY;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  const int tid = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int nthr = (int)(blockDim.x * blockDim.y);
  const int NO = TW * TY;
  const bool act = tid < NO;                                // owns a tile column
  const bool hal = tid >= NO && tid < NO + TW + TY + 1;     // owns a halo point
  const int hq = tid - NO;
  // this thread's point (tile coordinates)
  const int px = act ? tid % TW : (hq < TW ? hq : TW);
  const int py = act ? tid / TW : (hq < TW ? TY : hq - TW);
  const int pi = i0 + px, pj = j0 + py;
  const bool pvalid = (act || hal) && pi < d.nx && pj < d.ny;
  const bool own = act && pvalid;
  const int64_t sx = d.sx, sxy = d.sxy, n = d.n;
  constexpr uint32_t ES = sizeof(T);
  // in-plane element index of the point (0 outside the grid)
  const uint32_t pp = pvalid ? (uint32_t)(pi + sx * pj) : 0u;

  auto ring = [&](int x, int y) { return (y + 1) * RW + (x + 1); };
  auto ext = [&](int x, int y) { return y * EW + x; };

  // ---- register prefetch: the ring entries of a plane, and this thread's
  // point values lambda^(m+2) xyz, e^m xyz, e^(m+1) xyz
  T pre[kAdjRing][8];
  T pv[9];
  // ring entries of this thread: in-plane byte offsets (fixed over the march)
  uint32_t oring[kAdjRing];
  bool inring[kAdjRing];
#pragma unroll
  for (int r = 0; r < kAdjRing; ++r) {
    const int q = tid + r * nthr;
    const int gx = i0 + (q % RW) - 1, gy = j0 + (q / RW) - 1;
    inring[r] = q < RP && gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny;
    oring[r] = inring[r] ? (uint32_t)(gx + sx * gy) * ES : 0u;
  }
  auto fetch_ring = [&](int k) {
    const bool plane = k >= 0 && k < d.nz;
    const int64_t gk = plane ? sxy * (int64_t)k : 0;
#pragma unroll
    for (int r = 0; r < kAdjRing; ++r) {
      const bool in = plane && inring[r];
      const uint32_t o = afresh(oring[r]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pre[r][c] = in ? ald(A.h + c * n + gk, o) : T(0);
        pre[r][3 + c] = in ? ald(A.mu0 + c * n + gk, o) : T(0);
      }
      pre[r][6] = in ? ald(A.eps + gk, o) : T(0);
      pre[r][7] = (LOSSY && in) ? ald(A.sig + gk, o) : T(0);
    }
  };
  auto fetch_pt = [&](int k) {
    const bool lo = k >= 0 && k < d.nz && pvalid;
    const int64_t gk = lo ? sxy * (int64_t)k : 0;
    const uint32_t o = afresh(pp * ES);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv[c] = lo ? ald(A.lam0 + c * n + gk, o) : T(0);
      pv[3 + c] = lo ? ald(A.em + c * n + gk, o) : T(0);
      pv[6 + c] = lo ? ald(A.em1 + c * n + gk, o) : T(0);
    }
  };
  auto stage = [&](T* rL) {
#pragma unroll
    for (int r = 0; r < kAdjRing; ++r) {
      const int q = tid + r * nthr;
      if (q < RP) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (LOSSY || c < 7) rL[c * RP + q] = pre[r][c];
      }
    }
  };
  // plane-(k-1) values of point (x, y), read from a staged ring
  auto take_prev = [&](const T* rL, int x, int y, AdjPrev<T>& p) {
    const int r = ring(x, y), rim = ring(x - 1, y), rjm = ring(x, y - 1);
    p.hx = rL[0 * RP + r];
    p.hy = rL[1 * RP + r];
    p.ux = rL[3 * RP + r];
    p.uy = rL[4 * RP + r];
    p.uz = rL[5 * RP + r];
    const T c = rL[6 * RP + r];
    p.Sx = c + rL[6 * RP + rim];
    p.Sy = c + rL[6 * RP + rjm];
    p.Sxs = p.Sys = T(0);
    if (LOSSY) {
      const T s = rL[7 * RP + r];
      p.Sxs = s + rL[7 * RP + rim];
      p.Sys = s + rL[7 * RP + rjm];
    }
  };

  // lambda^(m+1), tau and the scaled edge sensitivities at point (x, y) of
  // plane k (ring rL); v = lambda^(m+2), e^m, e^(m+1) there; p = its
  // plane-(k-1) values (replaced by those of plane k on return).
  auto lam_point = [&](const T* rL, int x, int y, int k, bool valid, const T* v, AdjPrev<T>& p,
                       T* lam, T* tau, double* qe, double* qs) {
    const int r = ring(x, y), rim = ring(x - 1, y), rjm = ring(x, y - 1), rijm = ring(x - 1, y - 1);
    const T hxc = rL[0 * RP + r], hyc = rL[1 * RP + r], hzc = rL[2 * RP + r];
    const T hz_jm = rL[2 * RP + rjm], hx_jm = rL[0 * RP + rjm];
    const T hy_im = rL[1 * RP + rim], hz_im = rL[2 * RP + rim];
    const T uxc = rL[3 * RP + r], uyc = rL[4 * RP + r], uzc = rL[5 * RP + r];
    const T uz_jm = rL[5 * RP + rjm], ux_jm = rL[3 * RP + rjm];
    const T uy_im = rL[4 * RP + rim], uz_im = rL[5 * RP + rim];
    const int gi = i0 + x, gj = j0 + y;
    const int64_t g = gi + sx * gj + sxy * (int64_t)k;
    // s^m = C~ h^(m+1/2) - j_s
    T s0 = (hzc - hz_jm) - (hyc - p.hy);
    T s1 = (hxc - p.hx) - (hzc - hz_im);
    T s2 = (hyc - hy_im) - (hxc - hx_jm);
    if (valid && g == A.src_idx) {
      if (A.src_comp == 0) s0 -= A.src_val;
      if (A.src_comp == 1) s1 -= A.src_val;
      if (A.src_comp == 2) s2 -= A.src_val;
    }
    const T sv[3] = {s0, s1, s2};
    // C~ (d mu^(m+3/2))
    const T gv[3] = {A.dmu[2] * (uzc - uz_jm) - A.dmu[1] * (uyc - p.uy),
                     A.dmu[0] * (uxc - p.ux) - A.dmu[2] * (uzc - uz_im),
                     A.dmu[1] * (uyc - uy_im) - A.dmu[0] * (uxc - ux_jm)};
    // materials: sums of the 4 cells around each edge
    const T c = rL[6 * RP + r], c_im = rL[6 * RP + rim], c_jm = rL[6 * RP + rjm],
            c_ijm = rL[6 * RP + rijm];
    const T Sx = c + c_im, Sy = c + c_jm;
    const T E4[3] = {p.Sy + Sy, p.Sx + Sx, Sx + (c_jm + c_ijm)};
    T S4[3] = {T(0), T(0), T(0)};
    T Sxs = T(0), Sys = T(0);
    if (LOSSY) {
      const T s = rL[7 * RP + r], s_im = rL[7 * RP + rim], s_jm = rL[7 * RP + rjm],
              s_ijm = rL[7 * RP + rijm];
      Sxs = s + s_im;
      Sys = s + s_jm;
      S4[0] = p.Sys + Sys;
      S4[1] = p.Sxs + Sxs;
      S4[2] = Sxs + (s_jm + s_ijm);
    }
    const bool live[3] = {valid && gj > 0 && k > 0, valid && gi > 0 && k > 0,
                          valid && gi > 0 && gj > 0};
    const bool pi_x = gi >= A.probe.lo[0] && gi + 1 <= A.probe.hi[0];
    const bool pi_yz = gi >= A.probe.lo[0] && gi <= A.probe.hi[0];
    const bool pj_y = gj >= A.probe.lo[1] && gj + 1 <= A.probe.hi[1];
    const bool pj_xz = gj >= A.probe.lo[1] && gj <= A.probe.hi[1];
    const bool kx = k >= A.probe.lo[2] && k <= A.probe.hi[2];
    const bool kz_ = k >= A.probe.lo[2] && k + 1 <= A.probe.hi[2];
    const bool inp[3] = {pi_x && pj_xz && kx, pi_yz && pj_y && kx, pi_yz && pj_xz && kz_};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T E = live[a] ? E4[a] : T(1);   // finite denominators on dead / outside points
      const double Me = A.ge[a] * (double)E;
      const double Ms = A.ge[a] * (double)S4[a];
      const T Dt = E + A.hs * S4[a];
      const T ca = LOSSY ? qdiv(E - A.hs * S4[a], Dt) : T(1);
      const T cb = qdiv(A.kb[a], Dt);
      const T em = v[3 + a], em1 = v[6 + a];
      T ln = ca * v[a] - gv[a];
      double probe_e2 = 0.0;
      if (inp[a]) {
        probe_e2 = (double)em1 * (double)em1;
        ln += (T)(2.0 * A.dt * Me * (double)em1);
      }
      ln = live[a] ? ln : T(0);
      lam[a] = ln;
      tau[a] = cb * ln;
      // da/dM_eps = dt M_sig / D^2, db/dM_eps = -dt / D^2,
      // da/dM_sig = -dt M_eps / D^2, db/dM_sig = -dt^2 / (2 D^2)
      const double Dd = Me + A.hdt * Ms;
      // FP64 grids: the IEEE quotient (the FP64 path is held to the oracle at
      // rounding level); FP32 grids: the refined hardware reciprocal
      const double f = sizeof(T) == 8 ? (double)ln * A.dt / (Dd * Dd)
                                      : (double)ln * A.dt * rcp_d(Dd * Dd);
      qe[a] = A.eps0 * A.ge[a] * (f * (Ms * (double)em - (double)sv[a]) + A.dt * probe_e2);
      qs[a] = A.ge[a] * (-f * (Me * (double)em + A.hdt * (double)sv[a]));
      if (!live[a]) qe[a] = qs[a] = 0.0;
    }
    p.hx = hxc;
    p.hy = hyc;
    p.ux = uxc;
    p.uy = uyc;
    p.uz = uzc;
    p.Sx = Sx;
    p.Sy = Sy;
    p.Sxs = Sxs;
    p.Sys = Sys;
  };

  // prologue: plane k0 - 1 (zeros below the grid) gives the carried values
  AdjPrev<T> pvp{};
  fetch_ring(k0 - 1);
  fetch_pt(k0);   // in flight together with the ring of plane k0 - 1
  stage(rL0 + 8 * RP);
  __syncthreads();
  if (act || hal) take_prev(rL0 + 8 * RP, px, py, pvp);
  fetch_ring(k0);
  double Ae = 0.0, Ze = 0.0, As = 0.0, Zs = 0.0;   // own cell: partial sums of plane k-1

  for (int k = k0; k <= k1; ++k) {
    const bool plane = k < d.nz;
    // the accumulators of cell (i, j, k-1), updated at the end of this iteration
    const bool cell = own && k > k0;
    const int64_t ck = cell ? sxy * (int64_t)(k - 1) : 0;   // plane of the cell
    const uint32_t oc = afresh(pp * 8u);
    const double ge0 = cell ? ald(A.geps + ck, oc) : 0.0;
    const double gs0 = cell ? ald(A.gsig + ck, oc) : 0.0;
    // ring of plane k: buffer k & 1 (the other one may still be read for k-1)
    T* rL = rL0 + (k & 1) * 8 * RP;
    stage(rL);
    if (k + 1 <= k1) fetch_ring(k + 1);   // in flight during the compute below
    __syncthreads();   // ring k staged; every read of qL from iteration k-1 is done
    T* tk = tL + (k & 1) * 3 * EP;               // tau of plane k
    const T* tq = tL + ((k & 1) ^ 1) * 3 * EP;   // tau of plane k-1
    const T mux = pvp.ux, muy = pvp.uy, muz = pvp.uz;   // mu^(m+3/2) of plane k-1
    T tau_o[3] = {T(0), T(0), T(0)};
    if (act || hal) {
      T lam[3];
      double qe[3], qs[3];
      lam_point(rL, px, py, k, plane && pvalid, pv, pvp, lam, tau_o, qe, qs);
      const int e = ext(px, py);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        tau_o[a] = plane ? tau_o[a] : T(0);
        tk[a * EP + e] = tau_o[a];
        qL[a * EP + e] = plane ? qe[a] : 0.0;
        qL[(3 + a) * EP + e] = plane ? qs[a] : 0.0;
      }
      if (plane && own && k < k1) {
        const int64_t gk = sxy * (int64_t)k;
        const uint32_t o = afresh(pp * ES);
#pragma unroll
        for (int a = 0; a < 3; ++a) ast(A.lam1 + a * n + gk, o, lam[a]);
      }
    }
    if (k + 1 <= k1) fetch_pt(k + 1);   // in flight during the mu update and the cell sums
    // mu^(m+1/2) of plane k-1 = mu^(m+3/2) + C tau (forward differences)
    if (k > k0 && own) {
      const int km = k - 1;
      const int e = ext(px, py), e_in = ext(px + 1, py), e_jn = ext(px, py + 1);
      const T txc = tq[e], tyc = tq[EP + e], tzc = tq[2 * EP + e];
      const T cx = (tq[2 * EP + e_jn] - tzc) - (tau_o[1] - tyc);
      const T cy = (tau_o[0] - txc) - (tq[2 * EP + e_in] - tzc);
      const T cz = (tq[EP + e_in] - tyc) - (tq[e_jn] - txc);
      const int64_t gk = sxy * (int64_t)km;
      const uint32_t o = afresh(pp * ES);
      ast(A.mu1 + gk, o, pi > 0 ? mux + cx : T(0));
      ast(A.mu1 + n + gk, o, pj > 0 ? muy + cy : T(0));
      ast(A.mu1 + 2 * n + gk, o, km > 0 ? muz + cz : T(0));
    }
    __syncthreads();
    // the 12 edges of cell (i, j, k-1): x-edges (i, j..j+1) and y-edges
    // (i..i+1, j) of planes k-1 and k, z-edges (i..i+1, j..j+1) of plane k-1
    if (own) {
      const int e = ext(px, py), e_in = ext(px + 1, py), e_jn = ext(px, py + 1),
                e_ijn = ext(px + 1, py + 1);
      const double Ae_k = (qL[e] + qL[e_jn]) + (qL[EP + e] + qL[EP + e_in]);
      const double Ze_k =
          (qL[2 * EP + e] + qL[2 * EP + e_in]) + (qL[2 * EP + e_jn] + qL[2 * EP + e_ijn]);
      const double As_k = (qL[3 * EP + e] + qL[3 * EP + e_jn]) + (qL[4 * EP + e] + qL[4 * EP + e_in]);
      const double Zs_k =
          (qL[5 * EP + e] + qL[5 * EP + e_in]) + (qL[5 * EP + e_jn] + qL[5 * EP + e_ijn]);
      if (cell) {
        ast(A.geps + ck, oc, ge0 + ((Ae + Ze) + Ae_k));
        ast(A.gsig + ck, oc, gs0 + ((As + Zs) + As_k));
      }
      Ae = Ae_k;
      Ze = Ze_k;
      As = As_k;
      Zs = Zs_k;
    }
  }
}

size_t adjoint_lds_bytes(int tw, int ty, size_t esz) {
  const size_t RP = (size_t)(tw + 2) * (ty + 2), EP = (size_t)(tw + 1) * (ty + 1);
  return 6 * EP * sizeof(double) + (16 * RP + 6 * EP) * esz;
}

int adjoint_threads(int tw, int ty) { return ((tw * ty + tw + ty + 1 + 63) / 64) * 64; }

// Resident workgroups per CU: the waves per SIMD that the kernel's
// waves-per-EU attribute guarantees (FP32 4, i.e. <= 128 VGPRs; FP64 2),
// 4 SIMDs, and 160 KiB of LDS.
int adjoint_blocks_per_cu(int tw, int ty, size_t esz, bool lossy) {
  (void)lossy;
  const int nt = adjoint_threads(tw, ty);
  const size_t lds = adjoint_lds_bytes(tw, ty, esz);
  const int waves_simd = esz == 8 ? 2 : 4;
  const int by_waves = 4 * waves_simd / ((nt + 63) / 64);
  const int by_lds = (int)((160 * 1024) / std::max<size_t>(lds, 1));
  return std::min(by_waves, by_lds);
}

template <typename T>
hipError_t launch_adjoint_step(const AdjArgs<T>& a, bool lossy, hipStream_t s) {
  const int nt = adjoint_threads(a.t.tw, a.t.ty);
  const size_t lds = adjoint_lds_bytes(a.t.tw, a.t.ty, sizeof(T));
  const void* fn = lossy ? reinterpret_cast<const void*>(&k_adj<T, true>)
                         : reinterpret_cast<const void*>(&k_adj<T, false>);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (lossy)
    hipLaunchKernelGGL((k_adj<T, true>), dim3((unsigned)a.t.blocks()), dim3(nt), lds, s, a);
  else
    hipLaunchKernelGGL((k_adj<T, false>), dim3((unsigned)a.t.blocks()), dim3(nt), lds, s, a);
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjArgs<float>&, bool, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjArgs<double>&, bool, hipStream_t);

}  // namespace fit
