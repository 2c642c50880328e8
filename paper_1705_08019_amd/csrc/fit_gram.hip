// Mode-Gram energy matrix G[a][b] = sum_r M_rr x_a[r] x_b[r] for K snapshots
// (the bilinear energy form <x^(a), x^(b)>_M of Sec. II-A; M = M_eps for
// e-snapshots, M_mu for h-snapshots).  A dense contraction over the long row
// axis, so it runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// The M weights of the 3n rows are formed once per grid and kind from the
// per-cell materials (k_gram_weights) and kept until the materials change.
//
// Decomposition: the rows are split into contiguous chunks, one per
// workgroup.  A workgroup forms the 16 x 16 MFMA tiles of one output block
// (up to 64 x 64: 4 x 4 tiles; tiles past the snapshot count are never
// formed and, in a diagonal block, only the upper tile triangle is, G being
// symmetric) over its chunk, streaming the snapshots from HBM straight into
// the MFMA operands: no LDS staging and no barrier in the row loop (k_gram
// below gives the lane layout).  Its waves take consecutive row steps, each
// with the next step's loads in flight while the current one is multiplied;
// their partial tiles are summed in LDS at the end and the workgroup writes
// its FP64 block.  A second kernel sums the blocks per entry with Neumaier
// compensation.  Larger K is covered block pair by block pair.
#include <type_traits>

#include "fit_internal.hpp"

namespace fit {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramBlk = 64;         // snapshots per output block side
constexpr int kGramChunkAlign = 256; // workgroup row chunks: a multiple of every workgroup step

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
  double* part;        // [nwg][16 NTA][16 NTB] packed blocks
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

// f(integral_constant<int, I>) for I = B .. E-1: the tile loops must see
// their tile indices as constants (a runtime loop over the tile list leaves
// index searches and operand selects in the MFMA stream).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Row layout of a wave step (base r0, lane group g = lane / 16): the lane's
// row offset c < RL is row r0 + 16 (c / 4) + 4 g + c % 4, so the four lane
// groups read 4 consecutive rows each and one 16-byte load of every lane
// covers 16 consecutive rows of each snapshot; a wave step spans 4 RL rows.
__device__ __forceinline__ int gram_row(int g, int c) { return 16 * (c / 4) + 4 * g + c % 4; }

// The lane's RL rows of one snapshot (p = the snapshot at the step base plus
// 4 g): 16-byte loads when VEC (p 16-byte aligned), else element by element.
template <typename T, int RL, bool VEC>
__device__ __forceinline__ void gram_rows(const T* p, T (&v)[RL]) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int u = 0; u < RL / 4; ++u) {
    const T* q = p + 16 * u;
    if constexpr (VEC && sizeof(T) == 4) {
      const f4 x = *reinterpret_cast<const f4*>(q);
      v[4 * u] = x.x;
      v[4 * u + 1] = x.y;
      v[4 * u + 2] = x.z;
      v[4 * u + 3] = x.w;
    } else if constexpr (VEC) {
      const d2 x0 = *reinterpret_cast<const d2*>(q);
      const d2 x1 = *reinterpret_cast<const d2*>(q + 2);
      v[4 * u] = x0.x;
      v[4 * u + 1] = x0.y;
      v[4 * u + 2] = x1.x;
      v[4 * u + 3] = x1.y;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[4 * u + c] = q[c];
    }
  }
}

// Lane c of the lane's 16-lane row (DPP row broadcast, both halves of the
// double): the row weight of row offset c, which lane c of each group holds.
template <int C>
__device__ __forceinline__ double gram_bcast(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + C, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + C, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// The operands of one wave step: RL rows per lane of the NTA (and, off the
// diagonal, NB) snapshot tiles, and one row weight per lane (lane i of group
// g holds the weight of its group's row offset i % RL).
template <typename T, int NTA, int NB, int RL>
struct GramStage {
  T a[NTA][RL];
  T b[NB][RL];
  double w;
};

// G block (a0.., b0..) over the workgroup's row chunk, streamed straight
// from HBM into the MFMA operands (no LDS staging, no barriers in the row
// loop).  Lane l of a wave holds snapshot a0 + 16 ta + l % 16 (and b0 + 16 tb
// + l % 16) and its lane group g = l / 16 takes RL rows of the step: the
// MFMA's 4-long inner dimension runs over the 4 lane groups, so one MFMA per
// row offset c < RL and tile adds 4 rows of w x_a x_b, with the A operand
// w x_a and the B operand x_b taken from the lane's own registers (the
// weight broadcast within the group's 16-lane DPP row).  A wave step covers
// 4 RL rows (whole 128-byte lines of every snapshot for RL >= 8 in FP32, 4 in FP64); the
// NWV waves of the workgroup take consecutive steps, and each step's loads
// are in flight while the previous step is multiplied (two register stages,
// alternating).  Full rounds of the NWV waves load unconditionally; the
// chunk's last, partial round reads element by element (rows past the chunk
// as zero).  The waves' partial tiles are summed in LDS at the end and the
// workgroup writes its FP64 block.
template <typename T, int NTA, int NTB, bool DIAG, int RL, bool VEC, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_gram(GramArgs<T> A) {
  static_assert(RL % 4 == 0 && RL <= 16, "RL: a multiple of 4, at most one 16-lane row");
  using TS = TileSet<NTA, NTB, DIAG>;
  constexpr int NB = DIAG ? 1 : NTB;   // B operands of their own (off the diagonal)
  constexpr int NQ = TS::count;
  constexpr int OR = 16 * NTA, OC = 16 * NTB;
  using Stage = GramStage<T, NTA, NB, RL>;
  __shared__ double O[OR * OC];
  const int tid = threadIdx.x;
  const int lane = tid & 63, i = lane & 15, grp = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t r_begin = (int64_t)blockIdx.x * A.chunk;
  const int64_t r_end = min(r_begin + A.chunk, A.rows);

  // snapshot rows of the lane; a lane past na (nb) reads snapshot a0 (b0)
  // instead: its operand values only reach the output rows (columns) past
  // na (nb), which the reduction never reads (each MFMA output entry is
  // formed from its own A row and B column alone)
  const T* pa[NTA];
  const T* pb[NB];
#pragma unroll
  for (int ta = 0; ta < NTA; ++ta)
    pa[ta] = A.X + (int64_t)(16 * ta + i < A.na ? A.a0 + 16 * ta + i : A.a0) * A.ld + 4 * grp;
#pragma unroll
  for (int tb = 0; tb < NB; ++tb)
    pb[tb] = A.X + (int64_t)(!DIAG && 16 * tb + i < A.nb ? A.b0 + 16 * tb + i : A.b0) * A.ld +
             4 * grp;
  const int wrow = gram_row(grp, i % RL);   // the row whose weight the lane holds

  d4_t acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};

  auto load_full = [&](int64_t r0, Stage& st) {
#pragma unroll
    for (int ta = 0; ta < NTA; ++ta) gram_rows<T, RL, VEC>(pa[ta] + r0, st.a[ta]);
    if (!DIAG) {
#pragma unroll
      for (int tb = 0; tb < NB; ++tb) gram_rows<T, RL, VEC>(pb[tb] + r0, st.b[tb]);
    }
    st.w = A.W[r0 + wrow];
  };
  auto load_tail = [&](int64_t r0, Stage& st) {
#pragma unroll
    for (int c = 0; c < RL; ++c) {
      const int64_t r = r0 + gram_row(grp, c);
      const int o = 16 * (c / 4) + c % 4;   // from the lane's base (which includes 4 g)
      const bool in = r < r_end;
#pragma unroll
      for (int ta = 0; ta < NTA; ++ta) st.a[ta][c] = in ? pa[ta][r0 + o] : T(0);
      if (!DIAG) {
#pragma unroll
        for (int tb = 0; tb < NB; ++tb) st.b[tb][c] = in ? pb[tb][r0 + o] : T(0);
      }
    }
    st.w = r0 + wrow < r_end ? A.W[r0 + wrow] : 0.0;
  };
  auto multiply = [&](const Stage& st) {
    static_for<0, RL>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const double w = gram_bcast<c>(st.w);
      // a dead row (weight 0: PEC-wall or phantom slot) contributes exactly
      // 0 whatever the snapshots hold there: its values are selected away
      const bool live = w != 0.0;
      double av[NTA], bv[NTB];
#pragma unroll
      for (int ta = 0; ta < NTA; ++ta) av[ta] = w * (double)(live ? st.a[ta][c] : T(0));
#pragma unroll
      for (int tb = 0; tb < NTB; ++tb)
        bv[tb] = (double)(live ? (DIAG ? st.a[tb][c] : st.b[tb < NB ? tb : 0][c]) : T(0));
      static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int ta = TS::ta(q), tb = TS::tb(q);
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ta], bv[tb], acc[q], 0, 0, 0);
      });
    });
  };

  constexpr int64_t kStep = 4 * RL;          // rows of one wave step
  constexpr int64_t kRound = NWV * kStep;    // rows of one step of all the waves
  const int64_t full = (r_end - r_begin) / kRound;
  int64_t r0 = r_begin + wave * kStep;
  Stage s0, s1;
  int64_t k = 0;
  if (full > 0) load_full(r0, s0);
  // two rounds per pass, the stages alternate; every load in the loop is
  // unconditional, so each multiply waits only for its own stage's loads.
  // The scheduling barriers keep the compiler from hoisting the next
  // stage's loads above the multiply (which would need a third stage of
  // registers and wait for both stages at once).
  for (; k + 2 < full; k += 2) {
    load_full(r0 + kRound, s1);
    __builtin_amdgcn_sched_barrier(0);
    multiply(s0);
    __builtin_amdgcn_sched_barrier(0);
    load_full(r0 + 2 * kRound, s0);
    __builtin_amdgcn_sched_barrier(0);
    multiply(s1);
    __builtin_amdgcn_sched_barrier(0);
    r0 += 2 * kRound;
  }
  if (full - k == 2) {              // the last two full rounds (the first in s0)
    load_full(r0 + kRound, s1);
    multiply(s0);
    multiply(s1);
    r0 += 2 * kRound;
  } else if (full - k == 1) {       // the last full round (in s0)
    multiply(s0);
    r0 += kRound;
  }
  if (r_begin + full * kRound < r_end) {   // the partial round
    load_tail(r0, s1);
    multiply(s1);
  }

  // sum the waves' tiles in LDS, in wave order
  for (int w = 0; w < NWV; ++w) {
    if (wave == w) {
      static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int ta = TS::ta(q), tb = TS::tb(q);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // register v of a lane holds row lane / 16 + 4 v, column lane % 16
          const int e = (16 * ta + grp + 4 * v) * OC + 16 * tb + i;
          O[e] = w == 0 ? acc[q][v] : O[e] + acc[q][v];
        }
      });
    }
    __syncthreads();
  }
  // the block, packed (OR x OC, row-major) at its workgroup's slot
  double* out = A.part + (int64_t)blockIdx.x * (OR * OC);
  for (int e = tid; e < OR * OC; e += 64 * NWV) out[e] = O[e];
}

// Sum the per-workgroup blocks entry by entry (Neumaier), write G rows
// a0.. and columns b0.. of the K x K output (and the mirrored entries).
// One workgroup of 1024 threads per row i of the block: thread t holds
// column j = t % NBP (NBP = nb rounded up to 16, 32 or 64) and sums the
// blocks v, v + V, v + 2V, ... for its set v = t / NBP (V = 1024 / NBP sets,
// so narrow blocks keep every lane busy; each load of a set reads NBP
// consecutive doubles of one block); the V set sums are then combined in set
// order, so the result does not depend on timing.  Entries of tiles the Gram
// kernel did not form (beyond na / nb, below the tile diagonal of a diagonal
// block) are never read.
constexpr int kGramRedThreads = 1024;
__global__ __launch_bounds__(kGramRedThreads) void k_gram_reduce(const double* part, int64_t nwg,
                                                                 int64_t blk, int oc, double* G,
                                                                 int K, int a0, int na, int b0,
                                                                 int nb) {
  __shared__ double rs[kGramRedThreads], rc[kGramRedThreads];
  const int i = blockIdx.x;            // < na
  const int NBP = nb <= 16 ? 16 : nb <= 32 ? 32 : 64;
  const int V = kGramRedThreads / NBP;
  const int j = threadIdx.x % NBP;
  const int v = threadIdx.x / NBP;
  const bool live = j < nb && !(a0 == b0 && (i / 16) > (j / 16));
  const int e = i * oc + j;   // entry (i, j) of a packed block (blk doubles, row stride oc)
  double s = 0.0, c = 0.0;
  auto add = [&](double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
  };
  if (live) {
    int64_t w = v;
    for (; w + 3 * V < nwg; w += 4 * V) {
      double x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = part[(w + q * V) * blk + e];
#pragma unroll
      for (int q = 0; q < 4; ++q) add(x[q]);
    }
    for (; w < nwg; w += V) add(part[w * blk + e]);
  }
  rs[threadIdx.x] = s;
  rc[threadIdx.x] = c;
  __syncthreads();
  if (v != 0 || !live) return;
  for (int u = 1; u < V; ++u) {
    add(rs[u * NBP + j]);
    c += rc[u * NBP + j];
  }
  const double val = s + c;
  // in a diagonal block only the upper triangle writes (and mirrors), so
  // every entry has exactly one writer
  if (a0 == b0 && i > j) return;
  G[(int64_t)(a0 + i) * K + (b0 + j)] = val;
  G[(int64_t)(b0 + j) * K + (a0 + i)] = val;
}

// One launch of a block pair: as many workgroups as are resident at once
// (one round, no tail), at most part_cap; returns the count used.  Rows per
// lane: 16 for single-tile blocks (K <= 16: more bytes in flight for the
// memory-bound case), else the fewest for which a wave step reads whole
// 128-byte lines (8 FP32, 4 FP64 rows), except 4 for off-diagonal FP32
// blocks of more than 8 tiles (their two operand stages would not fit the
// registers beside the accumulators).
template <typename T, int NTA, int NTB, bool DIAG, bool VEC>
static hipError_t gram_go(GramArgs<T> A, int64_t part_cap, hipStream_t s, int64_t* nwg_used) {
  // part_cap: the partials buffer in 64 x 64 blocks; a workgroup writes a
  // packed (16 NTA) x (16 NTB) block
  part_cap = part_cap * kGramBlk * kGramBlk / (256 * NTA * NTB);
  constexpr int RL = NTA == 1 && NTB == 1                      ? 16
                     : sizeof(T) == 8 || (!DIAG && NTA * NTB > 8) ? 4
                                                                  : 8;
  // waves per workgroup: 8 for single-tile blocks (K <= 16, read-bound), at
  // most two workgroups per CU -- the same waves per CU as four 4-wave
  // workgroups, half the concurrent snapshot streams, each workgroup reading
  // twice the rows of every snapshot per round (0.0983-0.0995 -> 0.0970 ms
  // per K = 16 call); 4 otherwise
  constexpr int NWV = NTA == 1 && NTB == 1 ? 8 : 4;
  const void* fn = reinterpret_cast<const void*>(&k_gram<T, NTA, NTB, DIAG, RL, VEC, NWV>);
  int per_cu = 0, cus = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * NWV, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 2;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  (void)hipGetLastError();
  // single-tile blocks: more workgroups per CU only add concurrent snapshot
  // streams and partial blocks (4-wave workgroups: 0.100 ms per call at 4
  // per CU, 0.106 at 8; 8-wave ones: 0.097 at 2, 0.099 at 4)
  if (NTA == 1 && NTB == 1) per_cu = std::min(per_cu, 2);
  int64_t nwg = std::min<int64_t>(part_cap, (int64_t)per_cu * cus);
  int64_t chunk = (A.rows + nwg - 1) / nwg;
  chunk = ((chunk + kGramChunkAlign - 1) / kGramChunkAlign) * kGramChunkAlign;
  nwg = (A.rows + chunk - 1) / chunk;
  A.chunk = chunk;
  *nwg_used = nwg;
  hipLaunchKernelGGL((k_gram<T, NTA, NTB, DIAG, RL, VEC, NWV>), dim3((unsigned)nwg),
                     dim3(64 * NWV), 0, s, A);
  return hipGetLastError();
}

template <typename T, int NTA, bool VEC>
static hipError_t gram_go_b(const GramArgs<T>& A, int ntb, bool diag, int64_t cap, hipStream_t s,
                            int64_t* nwg) {
  if (diag) return gram_go<T, NTA, NTA, true, VEC>(A, cap, s, nwg);
  switch (ntb) {
    case 1: return gram_go<T, NTA, 1, false, VEC>(A, cap, s, nwg);
    case 2: return gram_go<T, NTA, 2, false, VEC>(A, cap, s, nwg);
    case 3: return gram_go<T, NTA, 3, false, VEC>(A, cap, s, nwg);
    default: return gram_go<T, NTA, 4, false, VEC>(A, cap, s, nwg);
  }
}

template <typename T, bool VEC>
static hipError_t gram_go_a(const GramArgs<T>& A, int nta, int ntb, bool diag, int64_t cap,
                            hipStream_t s, int64_t* nwg) {
  switch (nta) {
    case 1: return gram_go_b<T, 1, VEC>(A, ntb, diag, cap, s, nwg);
    case 2: return gram_go_b<T, 2, VEC>(A, ntb, diag, cap, s, nwg);
    case 3: return gram_go_b<T, 3, VEC>(A, ntb, diag, cap, s, nwg);
    default: return gram_go_b<T, 4, VEC>(A, ntb, diag, cap, s, nwg);
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
      // 16-byte loads need a 16-byte aligned base and snapshot stride
      const bool vec = (reinterpret_cast<uintptr_t>(X) % 16) == 0 && (ld * sizeof(T)) % 16 == 0;
      hipError_t e = vec ? gram_go_a<T, true>(A, nta, ntb, diag, part_cap_blocks, s, &nwg)
                         : gram_go_a<T, false>(A, nta, ntb, diag, part_cap_blocks, s, &nwg);
      if (e != hipSuccess) return e;
      *nwg_used = std::max(*nwg_used, nwg);
      hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)A.na), dim3(kGramRedThreads), 0, s,
                         part, nwg, (int64_t)256 * nta * ntb, 16 * ntb, G, K, a0, A.na, b0, A.nb);
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
