// Leapfrog half-step kernels for gfx950: the e-update (dual curl C~ of h with
// M_eps, M_sigma and the source) and the h-update (primal curl C of e with
// M_mu^{-1}), Sec. II-A; fused FP64 energy partials (eq. energy); a
// deterministic compensated reduction; PEC masking; a standalone curl and a
// standalone energy kernel.
//
// Data layout: every field component is an nx*ny*nz array, x fastest (slot
// layout of fit.h).  A launch tiles the x-y plane into 64 x ty column tiles
// (one wavefront per tile row, x along lanes so every load/store is a
// coalesced 256 B (FP32) row segment) and marches each column through a chunk
// of kc z-planes, carrying the values of plane k-1 that the next plane needs
// (h_x, h_y and two partial material sums) in registers.  In-plane -1 / +1
// neighbours are loaded from global memory; they hit L1/L2 because the
// neighbouring lane or row of the same workgroup loads the same lines.
// Material matrices are never stored: each edge's M_eps, M_sigma (mean of the
// 4 surrounding cells) and each facet's M_mu^{-1} (mean of 2 cells) are
// formed in registers from the per-cell arrays, so the e-update moves 8 B of
// material data per cell (FP32) instead of 24 B of per-edge coefficients.
#include "fit_internal.hpp"
#include "fit_point.hpp"

#include <algorithm>
#include <cmath>

namespace fit {

Tiling make_tiling(const Dims& d, int ty, int kc, int tw) {
  Tiling t;
  t.ty = ty;
  t.tw = tw;
  t.kc = kc < 1 ? 1 : (kc > d.nz ? d.nz : kc);
  t.ntx = (d.nx + tw - 1) / tw;
  t.nty = (d.ny + ty - 1) / ty;
  t.nkc = (d.nz + t.kc - 1) / t.kc;
  return t;
}

// Neumaier compensated accumulation.
__device__ __forceinline__ void nadd(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// Sum NT per-thread values over the (64 x blockDim.y) workgroup and write the
// NT totals to out (fixed order: deterministic).
// Returns the total of term threadIdx.x to the threads that store it (0 elsewhere).
template <int NT>
__device__ __forceinline__ double block_sum_store(double (&v)[NT], double* out) {
  __shared__ double sh[8][NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double x = v[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[t] = x;
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t) sh[threadIdx.y][t] = v[t];
  }
  __syncthreads();
  double s = 0.0;
  if (threadIdx.y == 0 && threadIdx.x < NT) {
    for (int w = 0; w < (int)blockDim.y; ++w) s += sh[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
  return s;
}

// --------------------------------------------------------------------------- e-update
// e^(m+1) = ca e^m + cb (C~ h^(m+1/2) - j_s),  with, per edge,
//   S4eps, S4sig = sums of the 4 cell values around the edge,
//   ca = (S4eps - hs S4sig) / (S4eps + hs S4sig),  cb = kb / (S4eps + hs S4sig).
// (C~ h)_x = [h_z(j) - h_z(j-1)] - [h_y(k) - h_y(k-1)]  (cyclic for y, z).
template <typename T, bool LOSSY, bool ENERGY, bool PROBE>
__global__ __launch_bounds__(512) void k_epass(EArgs<T> A) {
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
  const bool act = (i < d.nx) && (j < d.ny);

  double acc[kPartTerms] = {0};
  double cmp[kPartTerms] = {0};

  if (act) {
    const bool ip = i > 0, jp = j > 0;
    // metric of this column (tensor grid) or the uniform constants
    const bool nu = A.sq[0] != nullptr;
    T kbx = A.kb[0], kby = A.kb[1], kbz = A.kb[2];
    double gex = A.ge[0], gey = A.ge[1], gez = A.ge[2];
    if (nu) {
      const double qx = A.sq[0][i], qy = A.sq[1][j];
      kbx = (T)(A.kbs * qx);
      kby = (T)(A.kbs * qy);
      gex = 0.25 / qx;
      gey = 0.25 / qy;
    }
    const T* __restrict__ hx = A.h[0];
    const T* __restrict__ hy = A.h[1];
    const T* __restrict__ hz = A.h[2];
    const T* __restrict__ eps = A.eps;
    const T* __restrict__ sig = A.sig;
    const int64_t sx = d.sx, sxy = d.sxy;
    int64_t idx = i + sx * j + sxy * (int64_t)k0;
    // carried values of plane k-1
    T hyp = 0, hxp = 0, sxe = 0, sye = 0, sxs = 0, sys = 0;
    if (k0 > 0) {
      const int64_t q = idx - sxy;
      hyp = hy[q];
      hxp = hx[q];
      const T c = eps[q];
      sxe = c + (ip ? eps[q - 1] : T(0));
      sye = c + (jp ? eps[q - sx] : T(0));
      if (LOSSY) {
        const T s = sig[q];
        sxs = s + (ip ? sig[q - 1] : T(0));
        sys = s + (jp ? sig[q - sx] : T(0));
      }
    }
    bool pi_x = false, pi_yz = false, pj_y = false, pj_xz = false;
    if (PROBE) {
      pi_x = i >= A.probe.lo[0] && i + 1 <= A.probe.hi[0];
      pi_yz = i >= A.probe.lo[0] && i <= A.probe.hi[0];
      pj_y = j >= A.probe.lo[1] && j + 1 <= A.probe.hi[1];
      pj_xz = j >= A.probe.lo[1] && j <= A.probe.hi[1];
    }
    for (int k = k0; k < k1; ++k, idx += sxy) {
      if (nu) {
        const double qz = A.sq[2][k];
        kbz = (T)(A.kbs * qz);
        gez = 0.25 / qz;
      }
      const T hxc = hx[idx], hyc = hy[idx], hzc = hz[idx];
      const T hz_jm = jp ? hz[idx - sx] : T(0);
      const T hx_jm = jp ? hx[idx - sx] : T(0);
      const T hy_im = ip ? hy[idx - 1] : T(0);
      const T hz_im = ip ? hz[idx - 1] : T(0);
      const T c = eps[idx];
      const T c_im = ip ? eps[idx - 1] : T(0);
      const T c_jm = jp ? eps[idx - sx] : T(0);
      const T c_ijm = (ip && jp) ? eps[idx - sx - 1] : T(0);
      const T Sx = c + c_im, Sy = c + c_jm, Sxj = c_jm + c_ijm;
      const T E4x = sye + Sy, E4y = sxe + Sx, E4z = Sx + Sxj;
      T S4x = 0, S4y = 0, S4z = 0, Sxs = 0, Sys = 0;
      if (LOSSY) {
        const T s = sig[idx];
        const T s_im = ip ? sig[idx - 1] : T(0);
        const T s_jm = jp ? sig[idx - sx] : T(0);
        const T s_ijm = (ip && jp) ? sig[idx - sx - 1] : T(0);
        Sxs = s + s_im;
        Sys = s + s_jm;
        S4x = sys + Sys;
        S4y = sxs + Sxs;
        S4z = Sxs + (s_jm + s_ijm);
      }
      T jx = 0, jy = 0, jz = 0;
      if (idx == A.src_idx) {
        if (A.src_comp == 0) jx = A.src_val;
        if (A.src_comp == 1) jy = A.src_val;
        if (A.src_comp == 2) jz = A.src_val;
      }
      const bool lx = jp && k > 0, ly = ip && k > 0, lz = ip && jp;
      const T exo = A.ein[0][idx], eyo = A.ein[1][idx], ezo = A.ein[2][idx];
      T exn, eyn, ezn;
      e_point<T, LOSSY>(hxc, hyc, hzc, hxp, hyp, hx_jm, hy_im, hz_jm, hz_im, E4x, E4y, E4z, S4x,
                        S4y, S4z, exo, eyo, ezo, jx, jy, jz, lx, ly, lz, kbx, kby, kbz, A.hs,
                        exn, eyn, ezn);
      A.eout[0][idx] = exn;
      A.eout[1][idx] = eyn;
      A.eout[2][idx] = ezn;
      if (ENERGY) {
        const double mx = gex * (double)E4x, my = gey * (double)E4y, mz = gez * (double)E4z;
        // dead edges' e^m is selected away (not multiplied by a zero weight)
        const double ox = lx ? (double)exo : 0.0, oy = ly ? (double)eyo : 0.0;
        const double oz = lz ? (double)ezo : 0.0, nx_ = exn, ny_ = eyn, nz_ = ezn;
        nadd(acc[PE_EE_MM], cmp[PE_EE_MM], mx * ox * ox + my * oy * oy + mz * oz * oz);
        nadd(acc[PE_EE_MM1], cmp[PE_EE_MM1], mx * ox * nx_ + my * oy * ny_ + mz * oz * nz_);
        nadd(acc[PE_EE_M1M1], cmp[PE_EE_M1M1], mx * nx_ * nx_ + my * ny_ * ny_ + mz * nz_ * nz_);
        if (LOSSY) {
          const double bx = 0.5 * (ox + nx_), by = 0.5 * (oy + ny_), bz = 0.5 * (oz + nz_);
          nadd(acc[PE_LOSS], cmp[PE_LOSS],
               gex * (double)S4x * bx * bx + gey * (double)S4y * by * by +
                   gez * (double)S4z * bz * bz);
        }
        if (idx == A.src_idx) {
          const double bs = A.src_comp == 0 ? 0.5 * (ox + nx_)
                          : A.src_comp == 1 ? 0.5 * (oy + ny_) : 0.5 * (oz + nz_);
          nadd(acc[PE_SRC], cmp[PE_SRC], bs * A.src_val_d);
        }
      }
      if (PROBE) {
        const bool kx = k >= A.probe.lo[2] && k <= A.probe.hi[2];
        const bool kz_ = k >= A.probe.lo[2] && k + 1 <= A.probe.hi[2];
        double p = 0.0;
        const double nx_ = exn, ny_ = eyn, nz_ = ezn;
        if (pi_x && pj_xz && kx) p += gex * (double)E4x * nx_ * nx_;
        if (pi_yz && pj_y && kx) p += gey * (double)E4y * ny_ * ny_;
        if (pi_yz && pj_xz && kz_) p += gez * (double)E4z * nz_ * nz_;
        nadd(acc[PE_PROBE], cmp[PE_PROBE], p);
      }
      hyp = hyc;
      hxp = hxc;
      sxe = Sx;
      sye = Sy;
      if (LOSSY) {
        sxs = Sxs;
        sys = Sys;
      }
    }
  }
  if (ENERGY || PROBE) {
    double v[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) v[t] = acc[t] + cmp[t];
    const double tot = block_sum_store<6>(v, A.part + (int64_t)blockIdx.x * kPartTerms);
    if (PROBE && threadIdx.y == 0 && threadIdx.x == PE_PROBE) {
      double* prow = A.pacc + 2 * (int64_t)blockIdx.x;
      double ps = prow[0], pc = prow[1];
      nadd(ps, pc, A.pscale * tot);
      prow[0] = ps;
      prow[1] = pc;
    }
  }
}

// --------------------------------------------------------------------------- h-update
// h^(m+3/2) = h^(m+1/2) - cd (C e^(m+1)),  cd = kd * (imu_1 + imu_2) per facet.
// (C e)_x = [e_z(j+1) - e_z(j)] - [e_y(k+1) - e_y(k)]  (cyclic for y, z);
// e in a boundary plane (index n) is zero.
template <typename T, bool MU_UNIFORM, bool ENERGY>
__global__ __launch_bounds__(512) void k_hpass(HArgs<T> A) {
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
  const bool act = (i < d.nx) && (j < d.ny);

  double acc[3] = {0, 0, 0};
  double cmp[3] = {0, 0, 0};

  if (act) {
    const T* __restrict__ ex = A.e[0];
    const T* __restrict__ ey = A.e[1];
    const T* __restrict__ ez = A.e[2];
    const T* __restrict__ imu = A.imu;
    const int64_t sx = d.sx, sxy = d.sxy;
    const bool ip = i > 0, jp = j > 0;
    const bool in_ = i + 1 < d.nx, jn = j + 1 < d.ny;
    int64_t idx = i + sx * j + sxy * (int64_t)k0;
    T exc = ex[idx], eyc = ey[idx];
    T imp = 0;
    if (!MU_UNIFORM && k0 > 0) imp = imu[idx - sxy];
    // metric (tensor grid: per-cell imu times volume, see HArgs) or constants
    const bool nu = !MU_UNIFORM && A.sq[0] != nullptr;
    T kdx = A.kd[0], kdy = A.kd[1], kdz = A.kd[2];
    double gfx = A.gf2[0], gfy = A.gf2[1], gfz = A.gf2[2];
    double rqx = 0.0, rqy = 0.0;
    if (nu) {
      rqx = 1.0 / A.sq[0][i];
      rqy = 1.0 / A.sq[1][j];
      gfz = 0.5 * rqx * rqy;
      kdz = (T)(A.kds * gfz);
    }
    for (int k = k0; k < k1; ++k, idx += sxy) {
      if (nu) {
        const double rqz = 1.0 / A.sq[2][k];
        gfx = 0.5 * rqy * rqz;
        gfy = 0.5 * rqx * rqz;
        kdx = (T)(A.kds * gfx);
        kdy = (T)(A.kds * gfy);
      }
      const bool kn = k + 1 < d.nz;
      const T exn = kn ? ex[idx + sxy] : T(0);
      const T eyn = kn ? ey[idx + sxy] : T(0);
      const T ezc = ez[idx];
      const T ez_jn = jn ? ez[idx + sx] : T(0);
      const T ez_in = in_ ? ez[idx + 1] : T(0);
      const T ey_in = in_ ? ey[idx + 1] : T(0);
      const T ex_jn = jn ? ex[idx + sx] : T(0);
      T mx, my, mz;  // imu_1 + imu_2 per facet
      T imc = 0;
      if (MU_UNIFORM) {
        mx = my = mz = A.imu_u + A.imu_u;
      } else {
        imc = imu[idx];
        mx = imc + (ip ? imu[idx - 1] : T(0));
        my = imc + (jp ? imu[idx - sx] : T(0));
        mz = imc + imp;
      }
      const T hxo = A.hin[0][idx], hyo = A.hin[1][idx], hzo = A.hin[2][idx];
      T hxn, hyn, hzn;
      h_point<T>(exc, eyc, ezc, exn, eyn, ez_jn, ez_in, ey_in, ex_jn, hxo, hyo, hzo, mx, my, mz,
                 ip, jp, k > 0, kdx, kdy, kdz, hxn, hyn, hzn);
      A.hout[0][idx] = hxn;
      A.hout[1][idx] = hyn;
      A.hout[2][idx] = hzn;
      if (ENERGY) {
        // M_mu = 1 / (gf2 * (imu_1 + imu_2)); dead facets contribute 0.
        const double wx = ip ? 1.0 / (gfx * (double)mx) : 0.0;
        const double wy = jp ? 1.0 / (gfy * (double)my) : 0.0;
        const double wz = k > 0 ? 1.0 / (gfz * (double)mz) : 0.0;
        const double ox = ip ? (double)hxo : 0.0, oy = jp ? (double)hyo : 0.0;
        const double oz = k > 0 ? (double)hzo : 0.0, nx_ = hxn, ny_ = hyn, nz_ = hzn;
        nadd(acc[PH_HH_CC], cmp[PH_HH_CC], wx * ox * ox + wy * oy * oy + wz * oz * oz);
        nadd(acc[PH_HH_CN], cmp[PH_HH_CN], wx * ox * nx_ + wy * oy * ny_ + wz * oz * nz_);
        nadd(acc[PH_HH_NN], cmp[PH_HH_NN], wx * nx_ * nx_ + wy * ny_ * ny_ + wz * nz_ * nz_);
      }
      exc = exn;
      eyc = eyn;
      if (!MU_UNIFORM) imp = imc;
    }
  }
  if (ENERGY) {
    double v[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) v[t] = acc[t] + cmp[t];
    (void)block_sum_store<3>(v, A.part + (int64_t)blockIdx.x * kPartTerms);
  }
}

// --------------------------------------------------------------------------- energy combination
// out[0..4] from work (see launch_energy_combine): eq. energy's W^m, Q^m and
// the Poynting balance Q^(m+1) - Q^m = -2 dt ebar . (M_sigma ebar + j_s).
__global__ void k_energy_combine(const double* __restrict__ work, double dt,
                                 double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  out[0] = work[0];
  out[1] = work[1];
  if (dt > 0.0) {
    const double* r = work + 2;
    out[2] = 0.5 * (r[1] + r[2] + r[4] + r[5]);
    out[3] = r[1] + r[4];
    out[4] = -2.0 * dt * (r[8] + r[9]);
  } else {
    out[2] = out[3] = out[4] = __builtin_nan("");
  }
}

hipError_t launch_energy_combine(const double* work, double dt, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_combine, dim3(1), dim3(64), 0, s, work, dt, out);
  return hipGetLastError();
}

// --------------------------------------------------------------------------- probe rows
// One workgroup: thread t sums rows t, t + 256, ... (Neumaier over sum and
// compensation), the partial totals are combined in thread order, and the
// total is added to jacc.  Rows are cleared.
__global__ __launch_bounds__(256) void k_pacc_flush(double* pacc, int64_t nrows, double* jacc) {
  __shared__ double sh[2][256];
  double s = 0.0, c = 0.0;
  for (int64_t r = threadIdx.x; r < nrows; r += 256) {
    nadd(s, c, pacc[2 * r]);
    nadd(s, c, pacc[2 * r + 1]);
    pacc[2 * r] = 0.0;
    pacc[2 * r + 1] = 0.0;
  }
  sh[0][threadIdx.x] = s;
  sh[1][threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double js = jacc[0], jc = jacc[1];
    for (int t = 0; t < 256; ++t) {
      nadd(js, jc, sh[0][t]);
      nadd(js, jc, sh[1][t]);
    }
    jacc[0] = js;
    jacc[1] = jc;
  }
}

hipError_t launch_pacc_flush(double* pacc, int64_t nrows, double* jacc, hipStream_t s) {
  hipLaunchKernelGGL(k_pacc_flush, dim3(1), dim3(256), 0, s, pacc, nrows, jacc);
  return hipGetLastError();
}

// --------------------------------------------------------------------------- reduction
struct ReduceArgs {
  const double* part;
  int64_t nblk;
  double* dst;
  int cols[kPartTerms];
  int probe_term;
  double jscale;
  double* jacc;
  int nan_col;
  int64_t row_m;
  const double* pend;
  int pend_col;
};

// One workgroup of 256 threads: per-thread Neumaier over a strided subset of
// the block rows, then a fixed-order pairwise combination of (sum, comp).
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs R) {
  __shared__ double ss[256][kPartTerms];
  __shared__ double sc[256][kPartTerms];
  const int tid = threadIdx.x;
  double s[kPartTerms], c[kPartTerms];
#pragma unroll
  for (int t = 0; t < kPartTerms; ++t) s[t] = c[t] = 0.0;
  for (int64_t b = tid; b < R.nblk; b += 256) {
#pragma unroll
    for (int t = 0; t < kPartTerms; ++t) nadd(s[t], c[t], R.part[b * kPartTerms + t]);
  }
#pragma unroll
  for (int t = 0; t < kPartTerms; ++t) {
    ss[tid][t] = s[t];
    sc[tid][t] = c[t];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int t = 0; t < kPartTerms; ++t) {
        double a = ss[tid][t], ca = sc[tid][t];
        nadd(a, ca, ss[tid + w][t]);
        ss[tid][t] = a;
        sc[tid][t] = ca + sc[tid + w][t];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int t = 0; t < kPartTerms; ++t) {
      const double tot = ss[0][t] + sc[0][t];
      if (R.dst && R.cols[t] >= 0) R.dst[R.cols[t]] = tot;
      if (R.jacc && t == R.probe_term) {
        double js = R.jacc[0], jc = R.jacc[1];
        nadd(js, jc, tot * R.jscale);
        R.jacc[0] = js;
        R.jacc[1] = jc;
      }
    }
    if (R.dst && R.nan_col >= 0) R.dst[R.nan_col] = __builtin_nan("");
    if (R.dst && R.pend) R.dst[R.pend_col] = *R.pend;
    if (R.dst && R.row_m >= 0) R.dst[0] = (double)R.row_m;
  }
}

hipError_t launch_reduce(const double* part, int64_t nblk, double* dst, const int* cols,
                         int probe_term, double jscale, double* jacc, int nan_col,
                         int64_t row_m, const double* pend, int pend_col, hipStream_t s) {
  ReduceArgs R;
  R.pend = pend;
  R.pend_col = pend_col;
  R.part = part;
  R.nblk = nblk;
  R.dst = dst;
  for (int t = 0; t < kPartTerms; ++t) R.cols[t] = cols ? cols[t] : -1;
  R.probe_term = probe_term;
  R.jscale = jscale;
  R.jacc = jacc;
  R.nan_col = nan_col;
  R.row_m = row_m;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, R);
  return hipGetLastError();
}

// --------------------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_epass(const EArgs<T>& a, bool lossy, bool energy, bool probe, hipStream_t s) {
  const dim3 blk(64, a.t.ty), grd((unsigned)a.t.blocks());
#define FIT_E(L, E, P) hipLaunchKernelGGL((k_epass<T, L, E, P>), grd, blk, 0, s, a)
  if (lossy) {
    if (energy) { if (probe) FIT_E(true, true, true); else FIT_E(true, true, false); }
    else { if (probe) FIT_E(true, false, true); else FIT_E(true, false, false); }
  } else {
    if (energy) { if (probe) FIT_E(false, true, true); else FIT_E(false, true, false); }
    else { if (probe) FIT_E(false, false, true); else FIT_E(false, false, false); }
  }
#undef FIT_E
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hpass(const HArgs<T>& a, bool mu_uniform, bool energy, hipStream_t s) {
  const dim3 blk(64, a.t.ty), grd((unsigned)a.t.blocks());
  if (mu_uniform) {
    if (energy) hipLaunchKernelGGL((k_hpass<T, true, true>), grd, blk, 0, s, a);
    else hipLaunchKernelGGL((k_hpass<T, true, false>), grd, blk, 0, s, a);
  } else {
    if (energy) hipLaunchKernelGGL((k_hpass<T, false, true>), grd, blk, 0, s, a);
    else hipLaunchKernelGGL((k_hpass<T, false, false>), grd, blk, 0, s, a);
  }
  return hipGetLastError();
}

template hipError_t launch_epass<float>(const EArgs<float>&, bool, bool, bool, hipStream_t);
template hipError_t launch_epass<double>(const EArgs<double>&, bool, bool, bool, hipStream_t);
template hipError_t launch_hpass<float>(const HArgs<float>&, bool, bool, hipStream_t);
template hipError_t launch_hpass<double>(const HArgs<double>&, bool, bool, hipStream_t);

// --------------------------------------------------------------------------- PEC mask
__device__ __forceinline__ void decode(int64_t idx, const Dims& d, int& i, int& j, int& k) {
  i = (int)(idx % d.nx);
  const int64_t r = idx / d.nx;
  j = (int)(r % d.ny);
  k = (int)(r / d.ny);
}

// A direction-a edge slot is live when its two transverse node indices are
// >= 1 (slots only exist for indices < n, so the upper wall is never stored);
// a direction-a facet slot is live when its own index is >= 1.
__device__ __forceinline__ bool edge_live(int a, int i, int j, int k) {
  return a == 0 ? (j > 0 && k > 0) : a == 1 ? (i > 0 && k > 0) : (i > 0 && j > 0);
}
__device__ __forceinline__ bool facet_live(int a, int i, int j, int k) {
  return a == 0 ? i > 0 : a == 1 ? j > 0 : k > 0;
}

template <typename T>
__global__ void k_mask(T* f, Dims d, int which) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * d.n) return;
  const int a = (int)(g / d.n);
  int i, j, k;
  decode(g - a * d.n, d, i, j, k);
  const bool live = which == 0 ? edge_live(a, i, j, k) : facet_live(a, i, j, k);
  if (!live) f[g] = T(0);
}

template <typename T>
hipError_t launch_mask(T* f, const Dims& d, int which, hipStream_t s) {
  const int64_t n = 3 * d.n;
  hipLaunchKernelGGL(k_mask<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, d, which);
  return hipGetLastError();
}
template hipError_t launch_mask<float>(float*, const Dims&, int, hipStream_t);
template hipError_t launch_mask<double>(double*, const Dims&, int, hipStream_t);

// --------------------------------------------------------------------------- standalone curl
// Every input read is gated by the liveness of its slot, so garbage in
// PEC-wall slots of the input cannot leak into the result.
template <typename T>
__global__ void k_curl(const T* __restrict__ in, T* __restrict__ out, Dims d, int which) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.n) return;
  int i, j, k;
  decode(idx, d, i, j, k);
  const T* x = in;
  const T* y = in + d.n;
  const T* z = in + 2 * d.n;
  auto rd = [&](const T* p, int a, int ii, int jj, int kk) -> T {
    if (ii < 0 || jj < 0 || kk < 0 || ii >= d.nx || jj >= d.ny || kk >= d.nz) return T(0);
    const bool live = which == 0 ? edge_live(a, ii, jj, kk) : facet_live(a, ii, jj, kk);
    return live ? p[ii + d.sx * jj + d.sxy * (int64_t)kk] : T(0);
  };
  T cx, cy, cz;
  if (which == 0) {  // C e, forward differences
    cx = (rd(z, 2, i, j + 1, k) - rd(z, 2, i, j, k)) - (rd(y, 1, i, j, k + 1) - rd(y, 1, i, j, k));
    cy = (rd(x, 0, i, j, k + 1) - rd(x, 0, i, j, k)) - (rd(z, 2, i + 1, j, k) - rd(z, 2, i, j, k));
    cz = (rd(y, 1, i + 1, j, k) - rd(y, 1, i, j, k)) - (rd(x, 0, i, j + 1, k) - rd(x, 0, i, j, k));
    out[idx] = facet_live(0, i, j, k) ? cx : T(0);
    out[idx + d.n] = facet_live(1, i, j, k) ? cy : T(0);
    out[idx + 2 * d.n] = facet_live(2, i, j, k) ? cz : T(0);
  } else {  // C~ h, backward differences
    cx = (rd(z, 2, i, j, k) - rd(z, 2, i, j - 1, k)) - (rd(y, 1, i, j, k) - rd(y, 1, i, j, k - 1));
    cy = (rd(x, 0, i, j, k) - rd(x, 0, i, j, k - 1)) - (rd(z, 2, i, j, k) - rd(z, 2, i - 1, j, k));
    cz = (rd(y, 1, i, j, k) - rd(y, 1, i - 1, j, k)) - (rd(x, 0, i, j, k) - rd(x, 0, i, j - 1, k));
    out[idx] = edge_live(0, i, j, k) ? cx : T(0);
    out[idx + d.n] = edge_live(1, i, j, k) ? cy : T(0);
    out[idx + 2 * d.n] = edge_live(2, i, j, k) ? cz : T(0);
  }
}

template <typename T>
hipError_t launch_curl(const T* in, T* out, const Dims& d, int which, hipStream_t s) {
  hipLaunchKernelGGL(k_curl<T>, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, in, out, d,
                     which);
  return hipGetLastError();
}
template hipError_t launch_curl<float>(const float*, float*, const Dims&, int, hipStream_t);
template hipError_t launch_curl<double>(const double*, double*, const Dims&, int, hipStream_t);

// --------------------------------------------------------------------------- standalone energy
// <e,e>_eps and <h,h>_mu of one state; one thread per cell slot, block
// partials in part rows (term 0: electric, term 1: magnetic).
template <typename T>
__global__ __launch_bounds__(256) void k_energy(const T* __restrict__ e, const T* __restrict__ h,
                                                const T* __restrict__ eps,
                                                const T* __restrict__ imu, T imu_u, Dims d,
                                                double gex, double gey, double gez, double gfx,
                                                double gfy, double gfz, const double* sq,
                                                double* part) {
  // grid-stride over the cell slots (at most kEnergyBlocks workgroups), FP64
  // Neumaier accumulation per thread
  double v[2] = {0.0, 0.0};
  double cv[2] = {0.0, 0.0};
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.y * 64 + threadIdx.x; idx < d.n;
       idx += (int64_t)gridDim.x * 256) {
    double ve = 0.0, vh = 0.0;
    int i, j, k;
    decode(idx, d, i, j, k);
    auto ce = [&](int ii, int jj, int kk) -> double {
      if (ii < 0 || jj < 0 || kk < 0) return 0.0;
      return (double)eps[ii + d.sx * jj + d.sxy * (int64_t)kk];
    };
    auto cm = [&](int ii, int jj, int kk) -> double {
      if (ii < 0 || jj < 0 || kk < 0) return 0.0;
      return imu ? (double)imu[ii + d.sx * jj + d.sxy * (int64_t)kk] : (double)imu_u;
    };
    const double ex = e[idx], ey = e[idx + d.n], ez = e[idx + 2 * d.n];
    const double hx = h[idx], hy = h[idx + d.n], hz = h[idx + 2 * d.n];
    double gx = gex, gy = gey, gz = gez, fx = gfx, fy = gfy, fz = gfz;
    if (sq) {   // tensor grid: eps, imu hold cell values times the cell volume
      const double qx = sq[i], qy = sq[d.nx + j], qz = sq[d.nx + d.ny + k];
      gx = 0.25 / qx;
      gy = 0.25 / qy;
      gz = 0.25 / qz;
      fx = 0.5 / (qy * qz);
      fy = 0.5 / (qx * qz);
      fz = 0.5 / (qx * qy);
    }
    if (edge_live(0, i, j, k))
      ve += gx * (ce(i, j, k) + ce(i, j - 1, k) + ce(i, j, k - 1) + ce(i, j - 1, k - 1)) * ex * ex;
    if (edge_live(1, i, j, k))
      ve += gy * (ce(i, j, k) + ce(i - 1, j, k) + ce(i, j, k - 1) + ce(i - 1, j, k - 1)) * ey * ey;
    if (edge_live(2, i, j, k))
      ve += gz * (ce(i, j, k) + ce(i - 1, j, k) + ce(i, j - 1, k) + ce(i - 1, j - 1, k)) * ez * ez;
    if (facet_live(0, i, j, k)) vh += hx * hx / (fx * (cm(i, j, k) + cm(i - 1, j, k)));
    if (facet_live(1, i, j, k)) vh += hy * hy / (fy * (cm(i, j, k) + cm(i, j - 1, k)));
    if (facet_live(2, i, j, k)) vh += hz * hz / (fz * (cm(i, j, k) + cm(i, j, k - 1)));
    nadd(v[0], cv[0], ve);
    nadd(v[1], cv[1], vh);
  }
  v[0] += cv[0];
  v[1] += cv[1];
  // blockDim = (64, 4) viewed as 256 threads: reuse the 2-D block sum
  block_sum_store<2>(v, part + (int64_t)blockIdx.x * kPartTerms);
}

template <typename T>
hipError_t launch_energy(const T* e, const T* h, const T* eps, const T* imu, T imu_u,
                         const Dims& d, const double ge[3], const double gf2[3], const double* sq,
                         double* part, int64_t* nblk, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((d.n + 255) / 256, kEnergyBlocks);
  *nblk = nb;
  hipLaunchKernelGGL(k_energy<T>, dim3((unsigned)nb), dim3(64, 4), 0, s, e, h, eps, imu, imu_u, d,
                     ge[0], ge[1], ge[2], gf2[0], gf2[1], gf2[2], sq, part);
  return hipGetLastError();
}
template hipError_t launch_energy<float>(const float*, const float*, const float*, const float*,
                                         float, const Dims&, const double*, const double*,
                                         const double*, double*, int64_t*, hipStream_t);
template hipError_t launch_energy<double>(const double*, const double*, const double*,
                                          const double*, double, const Dims&, const double*,
                                          const double*, const double*, double*, int64_t*,
                                          hipStream_t);

}  // namespace fit
