// Discrete adjoint of the leapfrog (reverse time) and the per-cell gradient of
// the probe objective J = dt sum_{m>=1} sum_probe M_eps (e^m)^2.
//
// Forward step (Sec. II-A, loss at e^(m+1/2)):  e^(m+1) = a e^m + b s^m with
// s^m = C~ h^(m+1/2) - j_s, a = (M_eps - dt/2 M_sigma) / D, b = dt / D,
// D = M_eps + dt/2 M_sigma;  h^(m+3/2) = h^(m+1/2) - d C e^(m+1), d = dt M_mu^{-1}.
// Reverse step m (lambda = dJ/de, mu = dJ/dh, both zero beyond the horizon):
//   lambda^(m+1) = a lambda^(m+2) - C~ (d mu^(m+3/2)) + 2 dt w M_eps e^(m+1)
//   mu^(m+1/2)   = mu^(m+3/2) + C (b lambda^(m+1))
//   dJ/dM_eps += lambda^(m+1) (da/dM_eps e^m + db/dM_eps s^m) + dt w (e^(m+1))^2
//   dJ/dM_sig += lambda^(m+1) (da/dM_sig e^m + db/dM_sig s^m)
// Because C~ = C^T, the two reverse passes are the forward stencils with the
// roles swapped: k_adj_e applies the dual curl (backward differences) to
// d mu, k_adj_h the primal curl (forward differences) to tau = b lambda.
// The last kernel gathers the per-edge sensitivities onto the cells
// (M_eps of an edge is eps0 g_a / 4 times the sum of its 4 cells' eps_r).
// mu (permeability) must be uniform here.
#include "fit_internal.hpp"

namespace fit {

template <typename T, bool LOSSY>
__global__ __launch_bounds__(512) void k_adj_e(AdjArgs<T> A) {
  const Dims d = A.d;
  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr = lt / A.t.ntx;
  const int tyi = (int)(rr % A.t.nty);
  const int kz = (int)(rr / A.t.nty);
  const int i = tx * 64 + (int)threadIdx.x;
  const int j = tyi * A.t.ty + (int)threadIdx.y;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  if (i >= d.nx || j >= d.ny) return;
  const bool ip = i > 0, jp = j > 0;
  const int64_t sx = d.sx, sxy = d.sxy;
  const T* __restrict__ hx = A.h[0];
  const T* __restrict__ hy = A.h[1];
  const T* __restrict__ hz = A.h[2];
  const T* __restrict__ ux = A.mu[0];
  const T* __restrict__ uy = A.mu[1];
  const T* __restrict__ uz = A.mu[2];
  const T* __restrict__ eps = A.eps;
  const T* __restrict__ sig = A.sig;
  int64_t idx = i + sx * j + sxy * (int64_t)k0;
  T hyp = 0, hxp = 0, uyp = 0, uxp = 0, sxe = 0, sye = 0, sxs = 0, sys = 0;
  if (k0 > 0) {
    const int64_t q = idx - sxy;
    hyp = hy[q];
    hxp = hx[q];
    uyp = uy[q];
    uxp = ux[q];
    const T c = eps[q];
    sxe = c + (ip ? eps[q - 1] : T(0));
    sye = c + (jp ? eps[q - sx] : T(0));
    if (LOSSY) {
      const T s = sig[q];
      sxs = s + (ip ? sig[q - 1] : T(0));
      sys = s + (jp ? sig[q - sx] : T(0));
    }
  }
  const bool pi_x = i >= A.probe.lo[0] && i + 1 <= A.probe.hi[0];
  const bool pi_yz = i >= A.probe.lo[0] && i <= A.probe.hi[0];
  const bool pj_y = j >= A.probe.lo[1] && j + 1 <= A.probe.hi[1];
  const bool pj_xz = j >= A.probe.lo[1] && j <= A.probe.hi[1];
  for (int k = k0; k < k1; ++k, idx += sxy) {
    // dual curl of h (for s^m) and of d mu
    const T hxc = hx[idx], hyc = hy[idx], hzc = hz[idx];
    const T hz_jm = jp ? hz[idx - sx] : T(0), hx_jm = jp ? hx[idx - sx] : T(0);
    const T hy_im = ip ? hy[idx - 1] : T(0), hz_im = ip ? hz[idx - 1] : T(0);
    const T uxc = ux[idx], uyc = uy[idx], uzc = uz[idx];
    const T uz_jm = jp ? uz[idx - sx] : T(0), ux_jm = jp ? ux[idx - sx] : T(0);
    const T uy_im = ip ? uy[idx - 1] : T(0), uz_im = ip ? uz[idx - 1] : T(0);
    T sx_ = (hzc - hz_jm) - (hyc - hyp);
    T sy_ = (hxc - hxp) - (hzc - hz_im);
    T sz_ = (hyc - hy_im) - (hxc - hx_jm);
    if (idx == A.src_idx) {
      if (A.src_comp == 0) sx_ -= A.src_val;
      if (A.src_comp == 1) sy_ -= A.src_val;
      if (A.src_comp == 2) sz_ -= A.src_val;
    }
    const T gx = A.dmu[2] * (uzc - uz_jm) - A.dmu[1] * (uyc - uyp);
    const T gy = A.dmu[0] * (uxc - uxp) - A.dmu[2] * (uzc - uz_im);
    const T gz = A.dmu[1] * (uyc - uy_im) - A.dmu[0] * (uxc - ux_jm);
    // materials
    const T c = eps[idx];
    const T c_im = ip ? eps[idx - 1] : T(0);
    const T c_jm = jp ? eps[idx - sx] : T(0);
    const T c_ijm = (ip && jp) ? eps[idx - sx - 1] : T(0);
    const T Sx = c + c_im, Sy = c + c_jm, Sxj = c_jm + c_ijm;
    const T E4[3] = {sye + Sy, sxe + Sx, Sx + Sxj};
    T S4[3] = {0, 0, 0};
    T Sxs = 0, Sys = 0;
    if (LOSSY) {
      const T s = sig[idx];
      const T s_im = ip ? sig[idx - 1] : T(0);
      const T s_jm = jp ? sig[idx - sx] : T(0);
      const T s_ijm = (ip && jp) ? sig[idx - sx - 1] : T(0);
      Sxs = s + s_im;
      Sys = s + s_jm;
      S4[0] = sys + Sys;
      S4[1] = sxs + Sxs;
      S4[2] = Sxs + (s_jm + s_ijm);
    }
    const bool live[3] = {jp && k > 0, ip && k > 0, ip && jp};
    const bool kx = k >= A.probe.lo[2] && k <= A.probe.hi[2];
    const bool kz_ = k >= A.probe.lo[2] && k + 1 <= A.probe.hi[2];
    const bool inp[3] = {pi_x && pj_xz && kx, pi_yz && pj_y && kx, pi_yz && pj_xz && kz_};
    const T sv[3] = {sx_, sy_, sz_};
    const T gv[3] = {gx, gy, gz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t o = a * d.n + idx;
      const double Me = A.ge[a] * (double)E4[a];
      const double Ms = A.ge[a] * (double)S4[a];
      const double Dd = Me + A.hdt * Ms;
      const T em = A.em[o], em1 = A.em1[o], lo = A.lam[o];
      const T Dt = E4[a] + A.hs * S4[a];
      const T ca = LOSSY ? (E4[a] - A.hs * S4[a]) / Dt : T(1);
      const T cb = A.kb[a] / Dt;
      T ln = ca * lo - gv[a];
      double probe_e2 = 0.0;
      if (inp[a]) {
        probe_e2 = (double)em1 * (double)em1;
        ln += (T)(2.0 * A.dt * Me * (double)em1);
      }
      ln = live[a] ? ln : T(0);
      A.lam[o] = ln;
      A.tau[o] = live[a] ? cb * ln : T(0);
      if (live[a]) {
        const double l = ln;
        const double inv2 = 1.0 / (Dd * Dd);
        const double da_dMe = A.dt * Ms * inv2, db_dMe = -A.dt * inv2;
        const double da_dMs = -A.dt * Me * inv2, db_dMs = -0.5 * A.dt * A.dt * inv2;
        A.gMe[o] += l * (da_dMe * (double)em + db_dMe * (double)sv[a]) + A.dt * probe_e2;
        A.gMs[o] += l * (da_dMs * (double)em + db_dMs * (double)sv[a]);
      }
    }
    hyp = hyc;
    hxp = hxc;
    uyp = uyc;
    uxp = uxc;
    sxe = Sx;
    sye = Sy;
    if (LOSSY) {
      sxs = Sxs;
      sys = Sys;
    }
  }
}

// mu^(m+1/2) = mu^(m+3/2) + C tau   (in place; C by forward differences)
template <typename T>
__global__ __launch_bounds__(512) void k_adj_h(AdjArgs<T> A) {
  const Dims d = A.d;
  const int64_t lt = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(lt % A.t.ntx);
  const int64_t rr = lt / A.t.ntx;
  const int tyi = (int)(rr % A.t.nty);
  const int kz = (int)(rr / A.t.nty);
  const int i = tx * 64 + (int)threadIdx.x;
  const int j = tyi * A.t.ty + (int)threadIdx.y;
  const int k0 = kz * A.t.kc;
  const int k1 = min(k0 + A.t.kc, d.nz);
  if (i >= d.nx || j >= d.ny) return;
  const int64_t sx = d.sx, sxy = d.sxy;
  const T* __restrict__ tx_ = A.tau;
  const T* __restrict__ ty_ = A.tau + d.n;
  const T* __restrict__ tz_ = A.tau + 2 * d.n;
  const bool in_ = i + 1 < d.nx, jn = j + 1 < d.ny;
  int64_t idx = i + sx * j + sxy * (int64_t)k0;
  T txc = tx_[idx], tyc = ty_[idx];
  for (int k = k0; k < k1; ++k, idx += sxy) {
    const bool kn = k + 1 < d.nz;
    const T txn = kn ? tx_[idx + sxy] : T(0);
    const T tyn = kn ? ty_[idx + sxy] : T(0);
    const T tzc = tz_[idx];
    const T tz_jn = jn ? tz_[idx + sx] : T(0);
    const T tz_in = in_ ? tz_[idx + 1] : T(0);
    const T ty_in = in_ ? ty_[idx + 1] : T(0);
    const T tx_jn = jn ? tx_[idx + sx] : T(0);
    const T cx = (tz_jn - tzc) - (tyn - tyc);
    const T cy = (txn - txc) - (tz_in - tzc);
    const T cz = (ty_in - tyc) - (tx_jn - txc);
    T* ux = A.mu[0];
    T* uy = A.mu[1];
    T* uz = A.mu[2];
    ux[idx] = i > 0 ? ux[idx] + cx : T(0);
    uy[idx] = j > 0 ? uy[idx] + cy : T(0);
    uz[idx] = k > 0 ? uz[idx] + cz : T(0);
    txc = txn;
    tyc = tyn;
  }
}

// dJ/deps_r[c] = eps0 sum over the 12 edges of cell c of (g_a / 4) dJ/dM_eps;
// dJ/dsigma[c] likewise with dJ/dM_sigma (no eps0).
__global__ __launch_bounds__(256) void k_adj_gather(const double* gMe, const double* gMs, Dims d,
                                                    double gq0, double gq1, double gq2,
                                                    double eps0, double* deps, double* dsig) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  const int i = (int)(c % d.nx);
  const int64_t r = c / d.nx;
  const int j = (int)(r % d.ny);
  const int k = (int)(r / d.ny);
  const double gq[3] = {gq0, gq1, gq2};
  double se = 0.0, ss = 0.0;
  // edges of direction a around the cell: its two transverse node indices are
  // (p_b, p_b + 1) x (p_c, p_c + 1); slots beyond the grid are PEC walls (0)
  const int p[3] = {i, j, k};
  const int nn[3] = {d.nx, d.ny, d.nz};
  const int64_t st[3] = {1, d.sx, d.sxy};
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, cc = (a + 2) % 3;
    for (int db = 0; db < 2; ++db) {
      for (int dc = 0; dc < 2; ++dc) {
        const int qb = p[b] + db, qc = p[cc] + dc;
        if (qb >= nn[b] || qc >= nn[cc]) continue;
        const int64_t o = a * d.n + c + db * st[b] + dc * st[cc];
        se += gq[a] * gMe[o];
        ss += gq[a] * gMs[o];
      }
    }
  }
  deps[c] = eps0 * se;
  dsig[c] = ss;
}

template <typename T>
hipError_t launch_adjoint_step(const AdjArgs<T>& a, bool lossy, hipStream_t s) {
  const dim3 blk(64, a.t.ty), grd((unsigned)a.t.blocks());
  if (lossy) hipLaunchKernelGGL((k_adj_e<T, true>), grd, blk, 0, s, a);
  else hipLaunchKernelGGL((k_adj_e<T, false>), grd, blk, 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_h<T>, grd, blk, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_gather(const double* gMe, const double* gMs, const Dims& d,
                                 const double gq[3], double eps0, double* deps, double* dsig,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, gMe, gMs,
                     d, gq[0], gq[1], gq[2], eps0, deps, dsig);
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjArgs<float>&, bool, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjArgs<double>&, bool, hipStream_t);

}  // namespace fit
