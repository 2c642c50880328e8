// The semi-discrete FIT operator and the pieces of the matrix-exponential
// action (Sec. III-A) and of ParaExp (Sec. III) built on it.
//
// In the voltages x = (e, h) the lossless system of eq. FIT_ode_1 reads
// dx/dt = B x with
//   B (e, h) = ( M_eps^{-1} C~ h ,  -M_mu^{-1} C e ),
// the similarity transform of A in eq. FIT_ode_2 (A = T B T^{-1}, T =
// blkdiag(M_mu^{1/2}, M_eps^{1/2}) in [h; e] order), so exp(tA) acts on the
// transformed unknowns exactly as exp(tB) acts on the voltages, and
// ||A||_2 is the M-norm of B.
//
// k_opb: one application out = c B in (two curls, 2 SMVPs in the paper's
// count), optionally accumulated (acc += out, or acc = in + out for the
// first Taylor term).  A z-marching column kernel: each thread owns one
// (i, j) column of its tile and walks its z-chunk, carrying the h values of
// plane k-1 (backward differences of C~) and reading e of plane k+1 (forward
// differences of C).  M_eps of an edge is (g_a / 4) times the sum of its 4
// cells' eps0 eps_r; M_mu^{-1} of a facet is gf2_a (imu + imu) for a
// uniform mu.  PEC: dead edges and facets get 0.
#include "fit_internal.hpp"

namespace fit {

template <typename T>
struct OpArgs {
  const T* ein;       // 3-component fields, component c at offset c n
  const T* hin;
  T* eout;
  T* hout;
  T* eacc;            // accumulators (modes 1, 2)
  T* hacc;
  const T* eps;       // eps0 eps_r per cell
  Dims d;
  Tiling t;
  T ce[3];            // c / (g_a / 4): out_e = ce (C~ h) / E4
  T ch[3];            // -c gf2_a (imu + imu): out_h = ch (C e)
  const T* ye;        // second input (modes 3, 4)
  const T* yh;
  T gam, al, be;      // modes 3, 4: out += gam y, acc (+)= al y + be in
};

// MODE 0: out = c B in.  MODE 1: also acc += out.  MODE 2: also acc = in + out.
// MODE 3: out = c B in + gam y and acc += al y + be in (one pair step of the
// Leja recurrence: in = r_k, y = q_k, out = q_(k+1)).  MODE 4: as 3 with
// acc = al y + be in (the first pair).
template <typename T, int MODE>
__global__ __launch_bounds__(512) void k_opb(OpArgs<T> A) {
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
  const bool in_ = i + 1 < d.nx, jn = j + 1 < d.ny;
  const int64_t sx = d.sx, sxy = d.sxy, n = d.n;
  const T* __restrict__ ex = A.ein;
  const T* __restrict__ ey = A.ein + n;
  const T* __restrict__ ez = A.ein + 2 * n;
  const T* __restrict__ hx = A.hin;
  const T* __restrict__ hy = A.hin + n;
  const T* __restrict__ hz = A.hin + 2 * n;
  const T* __restrict__ eps = A.eps;
  int64_t idx = i + sx * j + sxy * (int64_t)k0;
  // carried: h of plane k-1 (x, y components), 2-cell eps sums of plane k-1,
  // and e of plane k (x, y components; read one plane ahead)
  T hyp = 0, hxp = 0, sxe = 0, sye = 0;
  if (k0 > 0) {
    const int64_t q = idx - sxy;
    hyp = hy[q];
    hxp = hx[q];
    const T c = eps[q];
    sxe = c + (ip ? eps[q - 1] : T(0));
    sye = c + (jp ? eps[q - sx] : T(0));
  }
  T exc = ex[idx], eyc = ey[idx];
  for (int k = k0; k < k1; ++k, idx += sxy) {
    // ---- e part: ce (C~ h) / E4 on live edges
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
    const bool lx = jp && k > 0, ly = ip && k > 0, lz = ip && jp;
    const T E4x = lx ? sye + Sy : T(1), E4y = ly ? sxe + Sx : T(1), E4z = lz ? Sx + Sxj : T(1);
    const T oex = lx ? A.ce[0] * ((hzc - hz_jm) - (hyc - hyp)) / E4x : T(0);
    const T oey = ly ? A.ce[1] * ((hxc - hxp) - (hzc - hz_im)) / E4y : T(0);
    const T oez = lz ? A.ce[2] * ((hyc - hy_im) - (hxc - hx_jm)) / E4z : T(0);
    // ---- h part: ch (C e) on live facets; e beyond the grid is 0
    const bool kn = k + 1 < d.nz;
    const T exn = kn ? ex[idx + sxy] : T(0);
    const T eyn = kn ? ey[idx + sxy] : T(0);
    const T ezc = ez[idx];
    const T ez_jn = jn ? ez[idx + sx] : T(0);
    const T ez_in = in_ ? ez[idx + 1] : T(0);
    const T ey_in = in_ ? ey[idx + 1] : T(0);
    const T ex_jn = jn ? ex[idx + sx] : T(0);
    const T ohx = ip ? A.ch[0] * ((ez_jn - ezc) - (eyn - eyc)) : T(0);
    const T ohy = jp ? A.ch[1] * ((exn - exc) - (ez_in - ezc)) : T(0);
    const T ohz = k > 0 ? A.ch[2] * ((ey_in - eyc) - (ex_jn - exc)) : T(0);
    if (MODE == 3 || MODE == 4) {
      // y and in are zero on dead slots, so out and acc stay zero there
      const T yex = A.ye[idx], yey = A.ye[n + idx], yez = A.ye[2 * n + idx];
      const T yhx = A.yh[idx], yhy = A.yh[n + idx], yhz = A.yh[2 * n + idx];
      A.eout[idx] = oex + A.gam * yex;
      A.eout[n + idx] = oey + A.gam * yey;
      A.eout[2 * n + idx] = oez + A.gam * yez;
      A.hout[idx] = ohx + A.gam * yhx;
      A.hout[n + idx] = ohy + A.gam * yhy;
      A.hout[2 * n + idx] = ohz + A.gam * yhz;
      const T bex = A.al * yex + A.be * exc, bey = A.al * yey + A.be * eyc,
              bez = A.al * yez + A.be * ezc;
      const T bhx = A.al * yhx + A.be * hxc, bhy = A.al * yhy + A.be * hyc,
              bhz = A.al * yhz + A.be * hzc;
      if (MODE == 3) {
        A.eacc[idx] += bex;
        A.eacc[n + idx] += bey;
        A.eacc[2 * n + idx] += bez;
        A.hacc[idx] += bhx;
        A.hacc[n + idx] += bhy;
        A.hacc[2 * n + idx] += bhz;
      } else {
        A.eacc[idx] = bex;
        A.eacc[n + idx] = bey;
        A.eacc[2 * n + idx] = bez;
        A.hacc[idx] = bhx;
        A.hacc[n + idx] = bhy;
        A.hacc[2 * n + idx] = bhz;
      }
    } else {
      A.eout[idx] = oex;
      A.eout[n + idx] = oey;
      A.eout[2 * n + idx] = oez;
      A.hout[idx] = ohx;
      A.hout[n + idx] = ohy;
      A.hout[2 * n + idx] = ohz;
    }
    if (MODE == 1) {
      A.eacc[idx] += oex;
      A.eacc[n + idx] += oey;
      A.eacc[2 * n + idx] += oez;
      A.hacc[idx] += ohx;
      A.hacc[n + idx] += ohy;
      A.hacc[2 * n + idx] += ohz;
    } else if (MODE == 2) {
      A.eacc[idx] = exc + oex;
      A.eacc[n + idx] = eyc + oey;
      A.eacc[2 * n + idx] = ezc + oez;
      A.hacc[idx] = hxc + ohx;
      A.hacc[n + idx] = hyc + ohy;
      A.hacc[2 * n + idx] = hzc + ohz;
    }
    hyp = hyc;
    hxp = hxc;
    sxe = Sx;
    sye = Sy;
    exc = exn;
    eyc = eyn;
  }
}

__device__ __forceinline__ void nadd_m(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// M-inner product partials: term 0 = sum M_eps a_e b_e, term 1 = sum M_mu
// a_h b_h over live slots (M_mu of a facet = 1 / (gf2_a (imu + imu))),
// FP64 per workgroup row of part (Neumaier within a thread).
template <typename T>
__global__ __launch_bounds__(256) void k_mdot(const T* ae, const T* ah, const T* be, const T* bh,
                                              const T* eps, Dims d, double ge0, double ge1,
                                              double ge2, double mm0, double mm1, double mm2,
                                              double* part) {
  const int64_t n = d.n;
  double se = 0.0, ce = 0.0, sh = 0.0, chh = 0.0;
  const double ge[3] = {ge0, ge1, ge2}, mm[3] = {mm0, mm1, mm2};
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % d.nx);
    const int64_t r = idx / d.nx;
    const int j = (int)(r % d.ny);
    const int k = (int)(r / d.ny);
    const bool ip = i > 0, jp = j > 0, kp = k > 0;
    // edges: the 4 cells around each
    const T c = eps[idx];
    const T c_im = ip ? eps[idx - 1] : T(0), c_jm = jp ? eps[idx - d.sx] : T(0);
    const T c_km = kp ? eps[idx - d.sxy] : T(0);
    const T c_ijm = (ip && jp) ? eps[idx - d.sx - 1] : T(0);
    const T c_ikm = (ip && kp) ? eps[idx - d.sxy - 1] : T(0);
    const T c_jkm = (jp && kp) ? eps[idx - d.sxy - d.sx] : T(0);
    const double E4[3] = {(double)c + (double)c_jm + (double)c_km + (double)c_jkm,
                          (double)c + (double)c_im + (double)c_km + (double)c_ikm,
                          (double)c + (double)c_im + (double)c_jm + (double)c_ijm};
    const bool le[3] = {jp && kp, ip && kp, ip && jp};
    const bool lh[3] = {ip, jp, kp};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t o = a * n + idx;
      if (le[a]) nadd_m(se, ce, ge[a] * E4[a] * (double)ae[o] * (double)be[o]);
      if (lh[a]) nadd_m(sh, chh, mm[a] * (double)ah[o] * (double)bh[o]);
    }
  }
  double v[2] = {se + ce, sh + chh};
  __shared__ double red[4][2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    double x = v[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[t] = x;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[wave][0] = v[0];
    red[wave][1] = v[1];
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += red[w][threadIdx.x];
    part[(int64_t)blockIdx.x * kPartTerms + threadIdx.x] = s;
  }
}

// y += a x over the two fields (6 n values each side).
template <typename T>
__global__ __launch_bounds__(256) void k_axpy(T a, const T* xe, const T* xh, T* ye, T* yh,
                                              int64_t n3) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n3; q += (int64_t)gridDim.x * 256) {
    ye[q] += a * xe[q];
    yh[q] += a * xh[q];
  }
}

// Pseudo-random start vector of the power iteration: uniform in [-1, 1]
// from a 64-bit mix of (seed, slot, field), zero on dead slots.
__device__ __forceinline__ double seed_value(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_seed(T* xe, T* xh, Dims d, uint64_t seed) {
  const int64_t n = d.n;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % d.nx);
    const int64_t r = idx / d.nx;
    const int j = (int)(r % d.ny);
    const int k = (int)(r / d.ny);
    const bool le[3] = {j > 0 && k > 0, i > 0 && k > 0, i > 0 && j > 0};
    const bool lh[3] = {i > 0, j > 0, k > 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t o = a * n + idx;
      xe[o] = le[a] ? (T)seed_value(seed * 0x100000001b3ull + 2 * (uint64_t)o) : T(0);
      xh[o] = lh[a] ? (T)seed_value(seed * 0x100000001b3ull + 2 * (uint64_t)o + 1) : T(0);
    }
  }
}

template <typename T>
hipError_t launch_opb(const T* ein, const T* hin, T* eout, T* hout, T* eacc, T* hacc, int mode,
                      const T* eps, const Dims& d, const Tiling& t, const double ce[3],
                      const double ch[3], hipStream_t s, const T* ye, const T* yh, double gam,
                      double al, double be) {
  OpArgs<T> A;
  A.ye = ye;
  A.yh = yh;
  A.gam = (T)gam;
  A.al = (T)al;
  A.be = (T)be;
  A.ein = ein;
  A.hin = hin;
  A.eout = eout;
  A.hout = hout;
  A.eacc = eacc;
  A.hacc = hacc;
  A.eps = eps;
  A.d = d;
  A.t = t;
  for (int c = 0; c < 3; ++c) {
    A.ce[c] = (T)ce[c];
    A.ch[c] = (T)ch[c];
  }
  const dim3 blk(64, t.ty), grd((unsigned)t.blocks());
  if (mode == 0) hipLaunchKernelGGL((k_opb<T, 0>), grd, blk, 0, s, A);
  else if (mode == 1) hipLaunchKernelGGL((k_opb<T, 1>), grd, blk, 0, s, A);
  else if (mode == 2) hipLaunchKernelGGL((k_opb<T, 2>), grd, blk, 0, s, A);
  else if (mode == 3) hipLaunchKernelGGL((k_opb<T, 3>), grd, blk, 0, s, A);
  else hipLaunchKernelGGL((k_opb<T, 4>), grd, blk, 0, s, A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mdot(const T* ae, const T* ah, const T* be, const T* bh, const T* eps,
                       const Dims& d, const double ge[3], const double mm[3], double* part,
                       int64_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot<T>, dim3((unsigned)nblk), dim3(256), 0, s, ae, ah, be, bh, eps, d,
                     ge[0], ge[1], ge[2], mm[0], mm[1], mm[2], part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy(T a, const T* xe, const T* xh, T* ye, T* yh, int64_t n3, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((n3 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_axpy<T>, dim3((unsigned)nb), dim3(256), 0, s, a, xe, xh, ye, yh, n3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_seed(T* xe, T* xh, const Dims& d, uint64_t seed, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((d.n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_seed<T>, dim3((unsigned)nb), dim3(256), 0, s, xe, xh, d, seed);
  return hipGetLastError();
}

#define FIT_EXPM_INST(T)                                                                        \
  template hipError_t launch_opb<T>(const T*, const T*, T*, T*, T*, T*, int, const T*,          \
                                    const Dims&, const Tiling&, const double*, const double*,  \
                                    hipStream_t, const T*, const T*, double, double, double);  \
  template hipError_t launch_mdot<T>(const T*, const T*, const T*, const T*, const T*,         \
                                     const Dims&, const double*, const double*, double*,       \
                                     int64_t, hipStream_t);                                    \
  template hipError_t launch_axpy<T>(T, const T*, const T*, T*, T*, int64_t, hipStream_t);     \
  template hipError_t launch_seed<T>(T*, T*, const Dims&, uint64_t, hipStream_t);
FIT_EXPM_INST(float)
FIT_EXPM_INST(double)
#undef FIT_EXPM_INST

}  // namespace fit
