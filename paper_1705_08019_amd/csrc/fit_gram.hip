// Mode-Gram energy matrix G[a][b] = sum_r M_rr x_a[r] x_b[r] for K snapshots
// (the bilinear energy form <x^(a), x^(b)>_M of Sec. II-A; M = M_eps for
// e-snapshots, M_mu for h-snapshots).  A dense contraction over the long row
// axis, so it runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Decomposition: the 3n rows are split into contiguous chunks, one per
// workgroup; a workgroup stages 32 rows x (up to 64) snapshots of its chunk in
// LDS as FP64 (FP32 snapshots are widened on load), forms the M weights of
// those 32 rows from the per-cell materials, and accumulates a 64 x 64 output
// block with 16 x 16 MFMA tiles (wave w owns output rows 16w..16w+15).  Each
// workgroup writes its FP64 block; a second kernel sums the blocks per entry
// with Neumaier compensation.  Larger K is covered block pair by block pair.
#include "fit_internal.hpp"

namespace fit {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramRows = 32;     // rows staged per LDS round
constexpr int kGramBlk = 64;      // snapshots per output block side

__device__ __forceinline__ bool g_edge_live(int a, int i, int j, int k) {
  return a == 0 ? (j > 0 && k > 0) : a == 1 ? (i > 0 && k > 0) : (i > 0 && j > 0);
}
__device__ __forceinline__ bool g_facet_live(int a, int i, int j, int k) {
  return a == 0 ? i > 0 : a == 1 ? j > 0 : k > 0;
}

template <typename T>
struct GramArgs {
  const T* X;          // snapshot s starts at X + s * ld
  int64_t ld;
  int a0, na, b0, nb;  // snapshot ranges of the output block (na, nb <= 64)
  int which;           // 0: e with M_eps, 1: h with M_mu
  const T* eps;
  const T* imu;        // null: uniform imu_u
  T imu_u;
  Dims d;
  double gw[3];        // ge (which 0) or gf2 (which 1)
  int64_t rows;        // 3 n
  int64_t chunk;       // rows per workgroup (multiple of kGramRows)
  double* part;        // [nwg][64][64]
};

template <typename T>
__device__ __forceinline__ double g_weight(const GramArgs<T>& A, int64_t r) {
  const int a = (int)(r / A.d.n);
  const int64_t idx = r - (int64_t)a * A.d.n;
  const int i = (int)(idx % A.d.nx);
  const int64_t t = idx / A.d.nx;
  const int j = (int)(t % A.d.ny);
  const int k = (int)(t / A.d.ny);
  const int64_t sx = A.d.sx, sxy = A.d.sxy;
  if (A.which == 0) {
    if (!g_edge_live(a, i, j, k)) return 0.0;
    // the 4 cells around the edge: the two transverse axes step back by one
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const int64_t st[3] = {1, sx, sxy};
    const T* e = A.eps;
    const double s = (double)e[idx] + (double)e[idx - st[b]] + (double)e[idx - st[c]] +
                     (double)e[idx - st[b] - st[c]];
    return A.gw[a] * s;
  }
  if (!g_facet_live(a, i, j, k)) return 0.0;
  const int64_t st[3] = {1, sx, sxy};
  const double m = A.imu ? (double)A.imu[idx] + (double)A.imu[idx - st[a]]
                         : 2.0 * (double)A.imu_u;
  return 1.0 / (A.gw[a] * m);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gram(GramArgs<T> A) {
  __shared__ double LA[kGramRows][kGramBlk + 1];
  __shared__ double LB[kGramRows][kGramBlk + 1];
  __shared__ double LW[kGramRows];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const bool same = A.a0 == A.b0 && A.na == A.nb;
  const int64_t r_begin = (int64_t)blockIdx.x * A.chunk;
  const int64_t r_end = min(r_begin + A.chunk, A.rows);
  d4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};

  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramRows) {
    __syncthreads();
    // stage: thread -> (snapshot s = tid / 4, rows 8 * (tid % 4) .. +8)
    {
      const int s = tid >> 2, rb = (tid & 3) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t r = r0 + rb + q;
        const bool in = r < r_end;
        double va = 0.0, vb = 0.0;
        if (in && s < A.na) va = (double)A.X[(int64_t)(A.a0 + s) * A.ld + r];
        if (!same && in && s < A.nb) vb = (double)A.X[(int64_t)(A.b0 + s) * A.ld + r];
        LA[rb + q][s] = va;
        if (!same) LB[rb + q][s] = vb;
      }
      if (tid < kGramRows) {
        const int64_t r = r0 + tid;
        LW[tid] = r < r_end ? g_weight<T>(A, r) : 0.0;
      }
    }
    __syncthreads();
    const double(*Bsrc)[kGramBlk + 1] = same ? LA : LB;
    // wave owns output rows 16*wave .. +15 (snapshots a0 + ...), all 4 column tiles
#pragma unroll
    for (int kk = 0; kk < kGramRows / 4; ++kk) {
      const int rr = kk * 4 + (lane >> 4);
      const double a = LW[rr] * LA[rr][16 * wave + (lane & 15)];
#pragma unroll
      for (int tb = 0; tb < 4; ++tb) {
        const double b = Bsrc[rr][16 * tb + (lane & 15)];
        acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[tb], 0, 0, 0);
      }
    }
  }
  // D[i][j] of tile (wave, tb): register v of a lane holds row lane / 16 + 4 v,
  // column lane % 16 (the FP64 output layout of this instruction)
  double* out = A.part + (int64_t)blockIdx.x * kGramBlk * kGramBlk;
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * wave + (lane >> 4) + 4 * v;
      const int jcol = 16 * tb + (lane & 15);
      out[i * kGramBlk + jcol] = acc[tb][v];
    }
  }
}

// Sum the per-workgroup blocks entry by entry (Neumaier), write G rows
// a0.. and columns b0.. of the K x K output (and the mirrored entries).
__global__ __launch_bounds__(256) void k_gram_reduce(const double* part, int64_t nwg, double* G,
                                                     int K, int a0, int na, int b0, int nb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kGramBlk * kGramBlk) return;
  const int i = e / kGramBlk, j = e % kGramBlk;
  if (i >= na || j >= nb) return;
  double s = 0.0, c = 0.0;
  for (int64_t w = 0; w < nwg; ++w) {
    const double x = part[w * kGramBlk * kGramBlk + e];
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
  }
  const double v = s + c;
  // in a diagonal block only the upper triangle writes (and mirrors), so
  // every entry has exactly one writer
  if (a0 == b0 && i > j) return;
  G[(int64_t)(a0 + i) * K + (b0 + j)] = v;
  G[(int64_t)(b0 + j) * K + (a0 + i)] = v;
}

template <typename T>
hipError_t launch_gram(const T* X, int64_t ld, int K, int which, const T* eps, const T* imu,
                       T imu_u, const Dims& d, const double gw[3], double* part,
                       int64_t part_cap_blocks, double* G, hipStream_t s, int64_t* nwg_used) {
  const int64_t rows = 3 * d.n;
  int64_t nwg = std::min<int64_t>(part_cap_blocks, 1024);
  int64_t chunk = (rows + nwg - 1) / nwg;
  chunk = ((chunk + kGramRows - 1) / kGramRows) * kGramRows;
  nwg = (rows + chunk - 1) / chunk;
  *nwg_used = nwg;
  for (int a0 = 0; a0 < K; a0 += kGramBlk) {
    for (int b0 = a0; b0 < K; b0 += kGramBlk) {
      GramArgs<T> A;
      A.X = X;
      A.ld = ld;
      A.a0 = a0;
      A.na = std::min(kGramBlk, K - a0);
      A.b0 = b0;
      A.nb = std::min(kGramBlk, K - b0);
      A.which = which;
      A.eps = eps;
      A.imu = imu;
      A.imu_u = imu_u;
      A.d = d;
      for (int c = 0; c < 3; ++c) A.gw[c] = gw[c];
      A.rows = rows;
      A.chunk = chunk;
      A.part = part;
      hipLaunchKernelGGL(k_gram<T>, dim3((unsigned)nwg), dim3(256), 0, s, A);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_gram_reduce, dim3(kGramBlk * kGramBlk / 256), dim3(256), 0, s, part,
                         nwg, G, K, a0, A.na, b0, A.nb);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template hipError_t launch_gram<float>(const float*, int64_t, int, int, const float*, const float*,
                                       float, const Dims&, const double*, double*, int64_t,
                                       double*, hipStream_t, int64_t*);
template hipError_t launch_gram<double>(const double*, int64_t, int, int, const double*,
                                        const double*, double, const Dims&, const double*, double*,
                                        int64_t, double*, hipStream_t, int64_t*);

}  // namespace fit
