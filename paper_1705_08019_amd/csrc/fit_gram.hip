// Mode-Gram energy matrix G[a][b] = sum_r M_rr x_a[r] x_b[r] for K snapshots
// (the bilinear energy form <x^(a), x^(b)>_M of Sec. II-A; M = M_eps for
// e-snapshots, M_mu for h-snapshots).  A dense contraction over the long row
// axis, so it runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// The M weights of the 3n rows are formed once per grid and kind from the
// per-cell materials (k_gram_weights) and kept until the materials change.
//
// Decomposition: the rows are split into contiguous chunks, one per
// workgroup; a workgroup stages slabs of R rows x C snapshots of its chunk in
// LDS as FP64 (R C = 4096: 64 x 64 for full blocks, 256 x 16 for K <= 16;
// FP32 snapshots are widened on load; each wave load instruction reads 64
// consecutive rows of one snapshot) and accumulates the 16 x 16
// MFMA tiles of a 64 x 64 output block that hold output: tiles past the
// snapshot count are never formed and, in a diagonal block, only the upper
// tile triangle is (G is symmetric).  The 4 waves split the rows of each
// staged slab (and, for a full 4 x 4 off-diagonal block, the tiles in two
// halves), so every wave has the same work for any K; their partial tiles are
// summed in LDS at the end.  The next slab is loaded into registers while the
// current one is multiplied.  Each workgroup writes its FP64 block; a second
// kernel sums the blocks per entry with Neumaier compensation.  Larger K is
// covered block pair by block pair.
#include "fit_internal.hpp"

namespace fit {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramBlk = 64;         // snapshots per output block side
constexpr int kGramChunkAlign = 256; // workgroup row chunks: a multiple of every slab height

__device__ __forceinline__ bool g_edge_live(int a, int i, int j, int k) {
  return a == 0 ? (j > 0 && k > 0) : a == 1 ? (i > 0 && k > 0) : (i > 0 && j > 0);
}
__device__ __forceinline__ bool g_facet_live(int a, int i, int j, int k) {
  return a == 0 ? i > 0 : a == 1 ? j > 0 : k > 0;
}

// ---------------------------------------------------------------- weights
template <typename T>
struct WeightArgs {
  double* W;           // 3 n
  int which;           // 0: M_eps of the edges, 1: M_mu of the facets
  const T* eps;
  const T* imu;        // null: uniform imu_u
  T imu_u;
  Dims d;
  double gw[3];        // g_a / 4 (which 0) or gf2_a (which 1)
  const double* sq;    // tensor grid: squared widths [x | y | z], or null
};

// M_eps of an edge is (g_a / 4) times the sum of its 4 cells' eps0 eps_r;
// M_mu of a facet is 1 / (gf2_a (imu + imu of the cell behind)); dead slots
// (PEC walls, phantoms) weigh 0.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_weights(WeightArgs<T> A) {
  const int64_t n = A.d.n;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * n) return;
  const int a = (int)(r / n);
  const int64_t idx = r - a * n;
  const int i = (int)(idx % A.d.nx);
  const int64_t t = idx / A.d.nx;
  const int j = (int)(t % A.d.ny);
  const int k = (int)(t / A.d.ny);
  const int64_t st[3] = {1, A.d.sx, A.d.sxy};
  // tensor grid: the squared widths of this slot's cell indices per axis
  double q[3] = {0.0, 0.0, 0.0};
  if (A.sq) {
    q[0] = A.sq[i];
    q[1] = A.sq[A.d.nx + j];
    q[2] = A.sq[A.d.nx + A.d.ny + k];
  }
  double w = 0.0;
  if (A.which == 0) {
    if (g_edge_live(a, i, j, k)) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      const T* e = A.eps;
      const double s = (double)e[idx] + (double)e[idx - st[b]] + (double)e[idx - st[c]] +
                       (double)e[idx - st[b] - st[c]];
      w = (A.sq ? 0.25 / q[a] : A.gw[a]) * s;
    }
  } else if (g_facet_live(a, i, j, k)) {
    const double m = A.imu ? (double)A.imu[idx] + (double)A.imu[idx - st[a]]
                           : 2.0 * (double)A.imu_u;
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    w = 1.0 / ((A.sq ? 0.5 / (q[b] * q[c]) : A.gw[a]) * m);
  }
  A.W[r] = w;
}

template <typename T>
hipError_t launch_gram_weights(double* W, int which, const T* eps, const T* imu, T imu_u,
                               const Dims& d, const double gw[3], const double* sq,
                               hipStream_t s) {
  WeightArgs<T> A;
  A.W = W;
  A.which = which;
  A.eps = eps;
  A.imu = imu;
  A.imu_u = imu_u;
  A.d = d;
  A.sq = sq;
  for (int c = 0; c < 3; ++c) A.gw[c] = gw[c];
  const int64_t rows = 3 * d.n;
  hipLaunchKernelGGL(k_gram_weights<T>, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Gram
template <typename T>
struct GramArgs {
  const T* X;          // snapshot s starts at X + s * ld
  int64_t ld;
  int a0, na, b0, nb;  // snapshot ranges of the output block (na, nb <= 64)
  const double* W;     // row weights
  int64_t rows;        // 3 n
  int64_t chunk;       // rows per workgroup (multiple of kGramChunkAlign)
  double* part;        // [nwg][64][64]
};

// Tile q of a block with NTA x NTB tiles, row-major; upper triangle only if DIAG.
template <int NTA, int NTB, bool DIAG>
struct TileSet {
  static constexpr int count = DIAG ? NTA * (NTA + 1) / 2 : NTA * NTB;
  static constexpr int ta(int q) {
    if (!DIAG) return q / NTB;
    int a = 0;
    while (q >= NTA - a) {
      q -= NTA - a;
      ++a;
    }
    return a;
  }
  static constexpr int tb(int q) {
    if (!DIAG) return q % NTB;
    int a = 0;
    while (q >= NTA - a) {
      q -= NTA - a;
      ++a;
    }
    return a + q;
  }
};

// MFMAs of one wave over the staged slab: the row quads kk = phase, phase + P,
// ... and the tiles q = GRP, GRP + G, ... of the block.
template <int NTA, int NTB, bool DIAG, int P, int GRP, int R, int C>
__device__ __forceinline__ void gram_slab(const double (*LA)[C + 1], const double (*LB)[C + 1],
                                          const double* LW, int phase, int lane, d4_t* acc) {
  using TS = TileSet<NTA, NTB, DIAG>;
  constexpr int G = 4 / P;
  const int col = lane & 15;
#pragma unroll
  for (int kk0 = 0; kk0 < R / 4; kk0 += P) {
    const int rr = 4 * (kk0 + phase) + (lane >> 4);
    const double w = LW[rr];
    double av[NTA], bv[NTB];
#pragma unroll
    for (int ta = 0; ta < NTA; ++ta) av[ta] = w * LA[rr][16 * ta + col];
#pragma unroll
    for (int tb = 0; tb < NTB; ++tb) bv[tb] = LB[rr][16 * tb + col];
#pragma unroll
    for (int u = 0; GRP + G * u < TS::count; ++u) {
      const int q = GRP + G * u;
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[TS::ta(q)], bv[TS::tb(q)], acc[u], 0, 0,
                                                    0);
    }
  }
}

// Add this wave's tiles into the LDS block O ((16 NTA) x (16 NTB), row-major).
template <int NTA, int NTB, bool DIAG, int P, int GRP>
__device__ __forceinline__ void gram_store(double* O, int lane, const d4_t* acc, bool first) {
  using TS = TileSet<NTA, NTB, DIAG>;
  constexpr int G = 4 / P;
#pragma unroll
  for (int u = 0; GRP + G * u < TS::count; ++u) {
    const int q = GRP + G * u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // register v of a lane holds row lane / 16 + 4 v, column lane % 16
      const int i = 16 * TS::ta(q) + (lane >> 4) + 4 * v;
      const int j = 16 * TS::tb(q) + (lane & 15);
      O[i * (16 * NTB) + j] = first ? acc[u][v] : O[i * (16 * NTB) + j] + acc[u][v];
    }
  }
}

// Waves per SIMD the register allocation must leave room for: 3 for the
// diagonal FP32 blocks (their accumulators then live in VGPRs, no spills);
// the FP64 and off-diagonal variants take what their registers allow.
template <typename T, bool DIAG>
constexpr int gram_min_waves() { return (DIAG && sizeof(T) == 4) ? 3 : 1; }

template <typename T, int NTA, int NTB, bool DIAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gram_min_waves<T, DIAG>())))
void k_gram(GramArgs<T> A) {
  using TS = TileSet<NTA, NTB, DIAG>;
  // row phases: every wave forms all tiles when their accumulators fit the
  // registers, else two tile halves x two row phases
  constexpr int P = TS::count <= 10 ? 4 : 2;
  constexpr int G = 4 / P;
  constexpr int NTW = (TS::count + G - 1) / G;
  // slab: R rows x C snapshot columns (R C = 4096: narrow blocks stage more
  // rows per round, so every round moves the same bytes)
  constexpr int NT = NTA > NTB ? NTA : NTB;
  constexpr int C = 16 * NT;
  constexpr int R = NT == 1 ? 256 : NT == 2 ? 128 : 64;
  constexpr int SS = 256 / R;                  // snapshot stride between a thread's loads
  constexpr int NQ = (C + SS - 1) / SS;        // loads per thread per operand
  __shared__ double LA[R][C + 1];
  __shared__ double LB[DIAG ? 1 : R][C + 1];
  __shared__ double LW[R];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int phase = wave % P, grp = wave / P;
  const int64_t r_begin = (int64_t)blockIdx.x * A.chunk;
  const int64_t r_end = min(r_begin + A.chunk, A.rows);

  d4_t acc[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) acc[u] = d4_t{0.0, 0.0, 0.0, 0.0};

  // staging: thread -> row r0 + tid % R of the snapshots tid / R + SS q:
  // every load instruction of a wave reads 64 consecutive rows of one snapshot
  const int row = tid % R, s0 = tid / R;
  constexpr int NB = DIAG ? 1 : NQ;
  T pa[NQ], pb[NB];
#pragma unroll
  for (int q = 0; q < NQ; ++q) pa[q] = T(0);
#pragma unroll
  for (int q = 0; q < NB; ++q) pb[q] = T(0);
  double pw = 0.0;
  // loads clamp the row to the chunk (in bounds); rows past it are zeroed on staging
  auto fetch = [&](int64_t r0) {
    const int64_t r = min(r0 + row, r_end - 1);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (s0 + SS * q < A.na) pa[q] = A.X[(int64_t)(A.a0 + s0 + SS * q) * A.ld + r];
    if (!DIAG) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (s0 + SS * q < A.nb) pb[q] = A.X[(int64_t)(A.b0 + s0 + SS * q) * A.ld + r];
    }
    if (tid < R) pw = A.W[r];
  };

  fetch(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += R) {
    __syncthreads();   // the previous slab's reads of LA / LB / LW are done
    const bool in = r0 + row < r_end;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int sq = s0 + SS * q;
      if (sq < C) LA[row][sq] = (in && sq < A.na) ? (double)pa[q] : 0.0;
    }
    if (!DIAG) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int sq = s0 + SS * q;
        if (sq < C) LB[DIAG ? 0 : row][sq] = (in && sq < A.nb) ? (double)pb[q] : 0.0;
      }
    }
    if (tid < R) LW[tid] = in ? pw : 0.0;
    __syncthreads();
    if (r0 + R < r_end) fetch(r0 + R);   // in flight during the MFMAs
    const double(*Bsrc)[C + 1] = DIAG ? LA : LB;
    if (G == 1 || grp == 0)
      gram_slab<NTA, NTB, DIAG, P, 0, R, C>(LA, Bsrc, LW, phase, lane, acc);
    else
      gram_slab<NTA, NTB, DIAG, P, (G > 1 ? 1 : 0), R, C>(LA, Bsrc, LW, phase, lane, acc);
  }

  // sum the row phases' partial tiles in LDS (LA reused as the output block)
  double* O = &LA[0][0];
  constexpr int OR = 16 * NTA, OC = 16 * NTB;
  static_assert(R * (C + 1) >= OR * OC, "LDS block too small");
  for (int ph = 0; ph < P; ++ph) {
    __syncthreads();
    if (phase == ph) {
      if (G == 1 || grp == 0)
        gram_store<NTA, NTB, DIAG, P, 0>(O, lane, acc, ph == 0);
      else
        gram_store<NTA, NTB, DIAG, P, (G > 1 ? 1 : 0)>(O, lane, acc, ph == 0);
    }
  }
  __syncthreads();
  double* out = A.part + (int64_t)blockIdx.x * kGramBlk * kGramBlk;
  for (int e = tid; e < OR * OC; e += 256) out[(e / OC) * kGramBlk + e % OC] = O[e];
}

// Sum the per-workgroup blocks entry by entry (Neumaier), write G rows
// a0.. and columns b0.. of the K x K output (and the mirrored entries).
// One workgroup per row i of the block; lane j of every wave holds entry
// (i, j), and wave v sums the blocks v, v + 16, v + 32, ... (each load of a
// wave reads 64 consecutive doubles of one block); the 16 wave sums are then
// combined in wave order, so the result does not depend on timing.  Entries
// of tiles the Gram kernel did not form (beyond na / nb, below the tile
// diagonal of a diagonal block) are never read.
constexpr int kGramRedWaves = 16;
__global__ __launch_bounds__(64 * kGramRedWaves) void k_gram_reduce(const double* part,
                                                                   int64_t nwg, double* G, int K,
                                                                   int a0, int na, int b0,
                                                                   int nb) {
  __shared__ double rs[kGramRedWaves][kGramBlk], rc[kGramRedWaves][kGramBlk];
  const int i = blockIdx.x;            // < na
  const int j = threadIdx.x & 63;
  const int v = threadIdx.x >> 6;
  const bool live = j < nb && !(a0 == b0 && (i / 16) > (j / 16));
  const int e = i * kGramBlk + j;
  double s = 0.0, c = 0.0;
  if (live) {
    int64_t w = v;
    for (; w + 7 * kGramRedWaves < nwg; w += 8 * kGramRedWaves) {
      double x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = part[(w + q * kGramRedWaves) * kGramBlk * kGramBlk + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double t = s + x[q];
        c += (fabs(s) >= fabs(x[q])) ? ((s - t) + x[q]) : ((x[q] - t) + s);
        s = t;
      }
    }
    for (; w < nwg; w += kGramRedWaves) {
      const double x = part[w * kGramBlk * kGramBlk + e];
      const double t = s + x;
      c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
      s = t;
    }
  }
  rs[v][j] = s;
  rc[v][j] = c;
  __syncthreads();
  if (v != 0 || !live) return;
  for (int u = 1; u < kGramRedWaves; ++u) {
    const double x = rs[u][j];
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
    c += rc[u][j];
  }
  const double val = s + c;
  // in a diagonal block only the upper triangle writes (and mirrors), so
  // every entry has exactly one writer
  if (a0 == b0 && i > j) return;
  G[(int64_t)(a0 + i) * K + (b0 + j)] = val;
  G[(int64_t)(b0 + j) * K + (a0 + i)] = val;
}

// One launch of a block pair: as many workgroups as are resident at once
// (one round, no tail), at most part_cap; returns the count used.
template <typename T, int NTA, int NTB, bool DIAG>
static hipError_t gram_go(GramArgs<T> A, int64_t part_cap, hipStream_t s, int64_t* nwg_used) {
  const void* fn = reinterpret_cast<const void*>(&k_gram<T, NTA, NTB, DIAG>);
  int per_cu = 0, cus = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1)
    per_cu = 2;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  (void)hipGetLastError();
  int64_t nwg = std::min<int64_t>(part_cap, (int64_t)per_cu * cus);
  int64_t chunk = (A.rows + nwg - 1) / nwg;
  chunk = ((chunk + kGramChunkAlign - 1) / kGramChunkAlign) * kGramChunkAlign;
  nwg = (A.rows + chunk - 1) / chunk;
  A.chunk = chunk;
  *nwg_used = nwg;
  hipLaunchKernelGGL((k_gram<T, NTA, NTB, DIAG>), dim3((unsigned)nwg), dim3(256), 0, s, A);
  return hipGetLastError();
}

template <typename T, int NTA>
static hipError_t gram_go_b(const GramArgs<T>& A, int ntb, bool diag, int64_t cap, hipStream_t s,
                            int64_t* nwg) {
  if (diag) return gram_go<T, NTA, NTA, true>(A, cap, s, nwg);
  switch (ntb) {
    case 1: return gram_go<T, NTA, 1, false>(A, cap, s, nwg);
    case 2: return gram_go<T, NTA, 2, false>(A, cap, s, nwg);
    case 3: return gram_go<T, NTA, 3, false>(A, cap, s, nwg);
    default: return gram_go<T, NTA, 4, false>(A, cap, s, nwg);
  }
}

template <typename T>
hipError_t launch_gram(const T* X, int64_t ld, int K, const double* W, const Dims& d, double* part,
                       int64_t part_cap_blocks, double* G, hipStream_t s, int64_t* nwg_used) {
  const int64_t rows = 3 * d.n;
  *nwg_used = 0;
  for (int a0 = 0; a0 < K; a0 += kGramBlk) {
    for (int b0 = a0; b0 < K; b0 += kGramBlk) {
      GramArgs<T> A;
      A.X = X;
      A.ld = ld;
      A.a0 = a0;
      A.na = std::min(kGramBlk, K - a0);
      A.b0 = b0;
      A.nb = std::min(kGramBlk, K - b0);
      A.W = W;
      A.rows = rows;
      A.chunk = 0;
      A.part = part;
      const int nta = (A.na + 15) / 16, ntb = (A.nb + 15) / 16;
      const bool diag = a0 == b0;
      int64_t nwg = 0;
      hipError_t e;
      switch (nta) {
        case 1: e = gram_go_b<T, 1>(A, ntb, diag, part_cap_blocks, s, &nwg); break;
        case 2: e = gram_go_b<T, 2>(A, ntb, diag, part_cap_blocks, s, &nwg); break;
        case 3: e = gram_go_b<T, 3>(A, ntb, diag, part_cap_blocks, s, &nwg); break;
        default: e = gram_go_b<T, 4>(A, ntb, diag, part_cap_blocks, s, &nwg); break;
      }
      if (e != hipSuccess) return e;
      *nwg_used = std::max(*nwg_used, nwg);
      hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)A.na), dim3(64 * kGramRedWaves), 0, s,
                         part, nwg, G, K, a0, A.na, b0, A.nb);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template hipError_t launch_gram_weights<float>(double*, int, const float*, const float*, float,
                                               const Dims&, const double*, const double*,
                                               hipStream_t);
template hipError_t launch_gram_weights<double>(double*, int, const double*, const double*, double,
                                                const Dims&, const double*, const double*,
                                                hipStream_t);
template hipError_t launch_gram<float>(const float*, int64_t, int, const double*, const Dims&,
                                       double*, int64_t, double*, hipStream_t, int64_t*);
template hipError_t launch_gram<double>(const double*, int64_t, int, const double*, const Dims&,
                                        double*, int64_t, double*, hipStream_t, int64_t*);

}  // namespace fit
