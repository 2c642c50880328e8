// C-ABI of the batched leapfrog: descriptor tables, source tables, graph
// capture/replay of S-step chunks (one launch per step of all grids) and the
// batch autotuner.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fit_host.hpp"

struct fit_batch {
  std::vector<fit_grid*> grids;
  int nb = 0;
  bool f64 = false;
  bool lossy_any = false;
  hipStream_t user = nullptr;    // caller's stream
  hipStream_t s = nullptr;       // private stream (graph capture needs a non-default stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  void* desc = nullptr;          // device BatchGrid<T>[nb]
  int* item_grid = nullptr;      // device, P entries
  fit::BatchCtl* ctl = nullptr;  // device
  void* src_tab = nullptr;       // device [nb][src_cap]
  int64_t src_cap = 0;
  int P = 0;
  // tile: tw x ty for every grid (tw > 0), or row-packed (tw = FIT_TW_ROWS):
  // ty threads per workgroup, each grid's tile shaped to its own extent
  int tw = 64, ty = 8;
  int kc = 0;                    // z-planes per item; 0: whole columns
  int nthreads = 512;            // threads per workgroup of the current layout
  size_t lds = 0;                // dynamic LDS of the current layout
  int steps_per_graph = 16;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_S = 0;
  bool graph_pairs = false;      // the captured chunk holds pair launches
  // two steps per launch: each grid in its own pair tile shape, its columns
  // cut into even z-chunks of at most pkc planes (0: whole columns)
  bool pair_on = false;
  int pkc = 0;
  fit::BatchItem* items2 = nullptr;   // device, P2 entries, XCD-interleaved
  int P2 = 0;
  size_t lds2 = 0;
  int nthreads2 = 0;
  std::vector<int> pshape;            // per grid: index into kBatchPairShapes
  std::vector<fit::Tiling> pt2;       // per grid: its pair tiling
  // persistent form: S steps per cooperative launch of persist_nwg resident
  // workgroups (fit_batch_set_persistent); persist_graph: the S-step launch
  // could be captured (else chunks are launched directly)
  bool persist = false;
  int persist_nwg = 0;
  bool persist_graph = true;
};

namespace fit {

static void batch_drop_graph(fit_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_S = 0;
  b->graph_pairs = false;
}

// Row-packed tile of one grid for `nt` threads: the tile width is the grid's
// whole x extent when it fits (no x halo at all), else a 32..256-wide power of
// two; the rows split the y extent evenly.  Picks the shape that leaves the
// fewest idle threads (ties: the wider tile).
static void rows_shape(const Dims& d, int nt, int* tw_out, int* ty_out) {
  const int cand[5] = {d.nx, 256, 128, 64, 32};
  double best = -1.0;
  *tw_out = 32;
  *ty_out = std::max(1, std::min(d.ny, nt / 32));
  for (int w : cand) {
    if (w < 1 || w > 256 || 2 * w > nt) continue;
    const int rows = nt / w;
    const int nty = (d.ny + rows - 1) / rows;
    const int t = (d.ny + nty - 1) / nty;
    if (w + t + 2 > nt) continue;
    const int ntx = (d.nx + w - 1) / w;
    const double util = (double)d.nx * d.ny / ((double)ntx * nty * nt);
    if (util > best * (1.0 + 1e-9)) {
      best = util;
      *tw_out = w;
      *ty_out = t;
    }
  }
}

// Tile of grid d under the batch's current tuning.
static Tiling batch_tiling(const fit_batch* b, const Dims& d) {
  const int kc = b->kc > 0 ? std::min(b->kc, d.nz) : d.nz;
  if (b->tw > 0) return make_tiling(d, b->ty, kc, b->tw);
  int tw = 0, ty = 0;
  rows_shape(d, b->ty, &tw, &ty);
  return make_tiling(d, ty, kc, tw);
}

// Resident workgroups of the persistent kernel for the current layout
// (at most one per item), 0 if it cannot run.
static int persist_workgroups(const fit_batch* b) {
  const size_t esz = b->f64 ? 8 : 4;
  const int per_cu = batch_persist_blocks_per_cu(esz, b->nthreads, b->lds);
  if (per_cu <= 0) return 0;
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  (void)hipGetLastError();
  return (int)std::min<int64_t>((int64_t)per_cu * cus, b->P);
}

// Resident workgroups of the persistent pair kernel for the pair layout, a
// multiple of 8 (entry r of the pair item table belongs to XCD r mod 8, and
// so does workgroup r of a launch) and at most the table's length; 0 if it
// cannot run.
static int persist2_workgroups(const fit_batch* b) {
  const size_t esz = b->f64 ? 8 : 4;
  const int per_cu = batch2_persist_blocks_per_cu(esz, b->nthreads2, b->lds2);
  if (per_cu <= 0 || b->P2 <= 0) return 0;
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  (void)hipGetLastError();
  const int64_t n = std::min<int64_t>((int64_t)per_cu * cus, b->P2);
  return (int)(n / kXcds * kXcds);
}

// Build the item table, the workgroup shape and the LDS size for the current
// tiling.  FIT_E_INVALID (nothing changed) if a grid's tile needs more LDS
// than a workgroup can have.
static int batch_layout(fit_batch* b) {
  const int nt = b->tw > 0 ? b->tw * b->ty : b->ty;
  const size_t esz = b->f64 ? 8 : 4;
  size_t lds = 0;
  std::vector<int> items;
  for (int g = 0; g < b->nb; ++g) {
    const Tiling t = batch_tiling(b, b->grids[g]->d);
    if (t.tw * t.ty > nt || t.tw + t.ty + 2 > nt)
      return fail(FIT_E_INVALID, "tile does not fit the workgroup");
    lds = std::max(lds, step_lds_bytes(t.ty, esz, b->lossy_any, t.tw));
    for (int64_t q = 0; q < t.blocks(); ++q) items.push_back(g);
  }
  if (lds > 160 * 1024) return fail(FIT_E_INVALID, "tile needs more LDS than a workgroup can have");
  if (items.size() > (size_t)0x7fffffff) return fail(FIT_E_INVALID, "too many work items");
  dev_free(reinterpret_cast<void*&>(b->item_grid));
  b->P = 0;
  int rc = dev_alloc(reinterpret_cast<void**>(&b->item_grid), items.size() * sizeof(int), "item table");
  if (rc) return rc;
  hipError_t e = hipMemcpy(b->item_grid, items.data(), items.size() * sizeof(int),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "item table upload");
  b->P = (int)items.size();
  b->nthreads = nt;
  b->lds = lds;
  (void)batch_prepare(esz, nt, lds);
  batch_drop_graph(b);
  if (b->persist) {   // the persistent launch's resident workgroups for this layout
    b->persist_nwg = persist_workgroups(b);
    if (b->persist_nwg <= 0)
      return fail(FIT_E_INVALID, "the persistent kernel cannot hold a workgroup of this tile");
  }
  return FIT_OK;
}

// Staged points per z-plane of grid d in pair tile shape q: the tiles'
// staging regions ((tw + 4) x (ty + 4) points of h, eps and, lossy, sigma)
// and e-update regions ((tw + 4) x (ty + 3) points of e).
static double pair_plane_cost(const Dims& d, int q, bool lossy) {
  const int tw = kBatchPairShapes[q][0], ty = kBatchPairShapes[q][1];
  const double tiles = (double)((d.nx + tw - 1) / tw) * ((d.ny + ty - 1) / ty);
  return tiles * ((tw + 4.0) * (ty + 4.0) * (lossy ? 5 : 4) + (tw + 4.0) * (ty + 3.0) * 3);
}

// The pair layout: each grid's tile shape (the one of kBatchPairShapes that
// fits the dtype and stages the fewest points for its x / y extent; ties go
// to the earlier, wider shape) and its z-chunks (the column cut into
// ceil(nz / pkc) chunks of even length, pkc = 0: whole columns).  An item's
// work grows with its chunk length plus the two planes of lag and one of
// halo, times its tile's staged points.
// The item table is laid out for the dispatcher, which hands workgroup b to
// XCD b mod 8: the tiles of one z-chunk of one grid (a group, cut into runs
// of consecutive tiles when it would exceed a 32nd of the whole work) go to
// one XCD, so the halo rows neighbouring tiles share are read once into that
// XCD's L2; groups are dealt largest first to the least loaded XCD, and each
// XCD takes its items largest first, so the short ones fill its tail.  The
// XCD lists are interleaved into the table (entry 8 i + x = item i of XCD
// x), the shorter ones padded with empty entries (grid -1).
// The kernel's threads and LDS are the largest any used shape needs.
// FIT_E_INVALID if no shape fits the dtype or a grid's plane is too large.
static int batch_layout2(fit_batch* b) {
  const size_t esz = b->f64 ? 8 : 4;
  std::vector<int> shape((size_t)b->nb);
  std::vector<Tiling> til((size_t)b->nb);
  struct Run {
    double cost, item_cost;
    int grid, t0, n;
  };
  std::vector<Run> groups;
  size_t lds = 0;
  int nthreads = 64;
  double total = 0.0;
  for (int g = 0; g < b->nb; ++g) {
    const fit_grid* gr = b->grids[g];
    const Dims& d = gr->d;
    if (!step2_plane_ok(d, esz))
      return fail(FIT_E_INVALID, "a z-plane of a grid spans more than 4 GiB");
    int best = -1;
    double best_cost = 0.0;
    for (int q = 0; q < kBatchPairNShapes; ++q) {
      const int tw = kBatchPairShapes[q][0], ty = kBatchPairShapes[q][1];
      if (!step2_shape_ok(tw, ty, esz, b->lossy_any, false) || step2_threads(tw, ty) > 768)
        continue;
      const double c = pair_plane_cost(d, q, gr->lossy);
      if (best < 0 || c < best_cost) {
        best = q;
        best_cost = c;
      }
    }
    if (best < 0) return fail(FIT_E_INVALID, "no pair tile fits a workgroup for this dtype");
    const int tw = kBatchPairShapes[best][0], ty = kBatchPairShapes[best][1];
    const int nch = b->pkc > 0 ? (d.nz + b->pkc - 1) / b->pkc : 1;
    const int kc = (d.nz + nch - 1) / nch;
    shape[g] = best;
    til[g] = make_tiling(d, ty, kc, tw);
    lds = std::max(lds, step2_lds_bytes(tw, ty, esz, b->lossy_any, false));
    nthreads = std::max(nthreads, step2_threads(tw, ty));
    const int per = til[g].ntx * til[g].nty;
    const double per_plane = best_cost / per;
    for (int kz = 0; kz < til[g].nkc; ++kz) {
      const int planes = std::min(kc, d.nz - kz * kc);
      const double ic = (planes + 3) * per_plane;
      groups.push_back({ic * per, ic, g, kz * per, per});
      total += ic * per;
    }
  }
  // cut the groups into runs of at most a 32nd of the work (at least one tile)
  std::vector<Run> runs;
  const double cap = total / (kXcds * 4);
  for (const Run& r : groups) {
    const int np = std::min(r.n, std::max(1, (int)std::ceil(r.cost / cap - 1e-9)));
    for (int k = 0, t = r.t0; k < np; ++k) {
      const int n = r.n / np + (k < r.n % np ? 1 : 0);
      runs.push_back({n * r.item_cost, r.item_cost, r.grid, t, n});
      t += n;
    }
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) {
    return x.item_cost != y.item_cost ? x.item_cost > y.item_cost : x.cost > y.cost;
  });
  std::vector<std::vector<BatchItem>> xl(kXcds);
  double load[kXcds] = {};
  for (const Run& r : runs) {
    int x = 0;
    for (int k = 1; k < kXcds; ++k)
      if (load[k] < load[x]) x = k;
    load[x] += r.cost;
    for (int t = r.t0; t < r.t0 + r.n; ++t) xl[x].push_back(BatchItem{r.grid, t});
  }
  size_t len = 0;
  for (const auto& l : xl) len = std::max(len, l.size());
  if (len * kXcds > (size_t)0x7fffffff) return fail(FIT_E_INVALID, "too many work items");
  std::vector<BatchItem> table(len * kXcds, BatchItem{-1, 0});
  for (int x = 0; x < kXcds; ++x)
    for (size_t i = 0; i < xl[x].size(); ++i) table[i * kXcds + x] = xl[x][i];
  dev_free(reinterpret_cast<void*&>(b->items2));
  b->P2 = 0;
  int rc = dev_alloc(reinterpret_cast<void**>(&b->items2), table.size() * sizeof(BatchItem),
                     "pair item table");
  if (rc) return rc;
  hipError_t e = hipMemcpy(b->items2, table.data(), table.size() * sizeof(BatchItem),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "pair item table upload");
  b->P2 = (int)table.size();
  b->lds2 = lds;
  b->nthreads2 = nthreads;
  b->pshape = shape;
  b->pt2 = til;
  batch_drop_graph(b);
  return FIT_OK;
}

// Set a tuning and lay the batch out for it; on failure the previous tuning
// (and layout) is restored.
static int batch_retune(fit_batch* b, int tw, int ty, int kc) {
  const int otw = b->tw, oty = b->ty, okc = b->kc;
  b->tw = tw;
  b->ty = ty;
  b->kc = kc;
  int rc = batch_layout(b);
  if (rc) {
    const std::string msg = fit_last_error();
    b->tw = otw;
    b->ty = oty;
    b->kc = okc;
    (void)batch_layout(b);
    return fail(rc, msg);
  }
  return FIT_OK;
}

// Fill and upload the per-grid descriptors for a call starting now.
template <typename T>
static int batch_desc(fit_batch* b, const double* dt, int64_t nsteps, bool with_src) {
  std::vector<BatchGrid<T>> desc((size_t)b->nb);
  if (with_src && nsteps > b->src_cap) {
    dev_free(b->src_tab);
    b->src_cap = 0;
    int rc = dev_alloc(&b->src_tab, (size_t)b->nb * (size_t)nsteps * sizeof(T), "source table");
    if (rc) return rc;
    b->src_cap = nsteps;
  }
  std::vector<T> tab;
  if (with_src) tab.assign((size_t)b->nb * (size_t)b->src_cap, T(0));
  int off = 0;
  for (int g = 0; g < b->nb; ++g) {
    fit_grid* gr = b->grids[g];
    BatchGrid<T>& D = desc[g];
    D.e[0] = static_cast<T*>(gr->e);
    D.e[1] = static_cast<T*>(gr->e_alt);
    D.h[0] = static_cast<T*>(gr->h);
    D.h[1] = static_cast<T*>(gr->h_alt);
    D.eps = static_cast<const T*>(gr->eps);
    D.sig = static_cast<const T*>(gr->sig);
    D.d = gr->d;
    D.t = batch_tiling(b, gr->d);
    for (int c = 0; c < 3; ++c) {
      D.kb[c] = (T)(4.0 * dt[g] / gr->gedge[c]);
      D.kd[c] = (T)(dt[g] * gr->gf2[c]);
    }
    D.hs = (T)(0.5 * dt[g]);
    D.imu2 = (T)gr->imu_u + (T)gr->imu_u;
    D.lossy = gr->lossy ? 1 : 0;
    D.src_comp = gr->src_axis;
    D.src_idx = gr->src_axis >= 0 ? gr->src_idx : -1;
    D.src_tab = nullptr;
    if (with_src && gr->src_axis >= 0) {
      T* row = tab.data() + (size_t)g * b->src_cap;
      for (int64_t s = 0; s < nsteps; ++s) row[s] = (T)source_value(gr, dt[g], gr->m + s);
      D.src_tab = static_cast<const T*>(b->src_tab) + (size_t)g * b->src_cap;
    }
    D.par0 = 0;
    D.ntiles = (int)D.t.blocks();
    D.tile_off = off;
    off += D.ntiles;
    if (g < (int)b->pt2.size()) {   // the pair layout (empty until pairs are laid out)
      D.t2 = b->pt2[g];
      D.s2shape = b->pshape[g];
    } else {
      D.t2 = Tiling{};
      D.s2shape = 0;
    }
  }
  hipError_t e = hipSuccess;
  if (with_src)
    e = hipMemcpyAsync(b->src_tab, tab.data(), tab.size() * sizeof(T), hipMemcpyHostToDevice, b->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->desc, desc.data(), desc.size() * sizeof(BatchGrid<T>),
                       hipMemcpyHostToDevice, b->s);
  // the host vectors die at return: wait for the copies
  if (e == hipSuccess) e = hipStreamSynchronize(b->s);
  if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
  return FIT_OK;
}

template <typename T>
static BatchArgs<T> batch_args_host(fit_batch* b, int fixed) {
  BatchArgs<T> a;
  a.grids = static_cast<const BatchGrid<T>*>(b->desc);
  a.item_grid = b->item_grid;
  a.items2 = nullptr;
  a.launch_off = 0;
  a.ctl = b->ctl;
  a.nb = b->nb;
  a.P = b->P;
  a.nthreads = b->nthreads;
  a.lds = (int)b->lds;
  a.fixed_parity = fixed;
  return a;
}

// the same for pair launches
template <typename T>
static BatchArgs<T> batch_args_pair(fit_batch* b, int fixed) {
  BatchArgs<T> a = batch_args_host<T>(b, fixed);
  a.item_grid = nullptr;
  a.items2 = b->items2;
  a.P = b->P2;
  a.nthreads = b->nthreads2;
  a.lds = (int)b->lds2;
  return a;
}

// nsteps steps of every grid through the persistent kernels: with step pairs
// on, launches of S / 2 pairs (S = steps per graph) and an odd last step
// through the single-step kernel; else S-step launches.  A captured launch
// is replayed per chunk when the graph is wanted and capture works, then one
// launch takes the remainder.
template <typename T>
static int batch_run_persist_pairs(fit_batch* b, int64_t nsteps, int use_graph) {
  const BatchArgs<T> a2 = batch_args_pair<T>(b, 0);
  const int nwg2 = persist2_workgroups(b);
  if (nwg2 <= 0)
    return fail(FIT_E_INVALID, "the persistent pair kernel cannot hold a workgroup of this tile");
  hipError_t e = launch_batch_set_base(b->ctl, 0, b->s);
  if (e != hipSuccess) return hip_fail(e, "batch step counter");
  const int64_t npair = nsteps / 2, nsingle = nsteps & 1;
  const int S2 = std::max(1, b->steps_per_graph / 2);
  int64_t done = 0;
  if (use_graph && b->persist_graph && npair >= S2) {
    if (!b->exec || b->graph_S != S2 || !b->graph_pairs) {
      batch_drop_graph(b);
      e = hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "graph capture begin");
      const hipError_t el = launch_batch2_persist<T>(a2, nwg2, S2, b->s);
      e = hipStreamEndCapture(b->s, &b->graph);
      if (el == hipSuccess && e == hipSuccess)
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (el != hipSuccess || e != hipSuccess) {   // capture of the cooperative launch failed
        (void)hipGetLastError();
        batch_drop_graph(b);
        b->persist_graph = false;
      } else {
        b->graph_S = S2;
        b->graph_pairs = true;
      }
    }
    if (b->exec) {
      for (; done + S2 <= npair; done += S2) {
        e = hipGraphLaunch(b->exec, b->s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
      }
    }
  }
  while (done < npair) {
    const int n = (int)std::min<int64_t>(npair - done, use_graph ? S2 : (int64_t)1 << 30);
    e = launch_batch2_persist<T>(a2, nwg2, n, b->s);
    if (e != hipSuccess) return hip_fail(e, "persistent pair launch");
    done += n;
  }
  if (nsingle) {
    e = launch_batch_persist<T>(batch_args_host<T>(b, 0), b->persist_nwg, 1, b->s);
    if (e != hipSuccess) return hip_fail(e, "persistent batch launch");
  }
  for (int g = 0; g < b->nb; ++g) {
    fit_grid* gr = b->grids[g];
    if ((npair + nsingle) & 1) swap_sets(gr);
    gr->m += nsteps;
    gr->smvp += 2 * nsteps;
  }
  return FIT_OK;
}

template <typename T>
static int batch_run_persist(fit_batch* b, int64_t nsteps, int use_graph) {
  if (b->pair_on && b->P2 > 0 && nsteps >= 2) return batch_run_persist_pairs<T>(b, nsteps, use_graph);
  const BatchArgs<T> a = batch_args_host<T>(b, 0);
  const int nwg = b->persist_nwg;
  hipError_t e = launch_batch_set_base(b->ctl, 0, b->s);
  if (e != hipSuccess) return hip_fail(e, "batch step counter");
  const int S = std::max(1, b->steps_per_graph);
  int64_t done = 0;
  if (use_graph && b->persist_graph && nsteps >= S) {
    if (!b->exec || b->graph_S != S || b->graph_pairs) {
      batch_drop_graph(b);
      e = hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "graph capture begin");
      const hipError_t el = launch_batch_persist<T>(a, nwg, S, b->s);
      e = hipStreamEndCapture(b->s, &b->graph);
      if (el == hipSuccess && e == hipSuccess)
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (el != hipSuccess || e != hipSuccess) {   // capture of the cooperative launch failed
        (void)hipGetLastError();
        batch_drop_graph(b);
        b->persist_graph = false;
      } else {
        b->graph_S = S;
        b->graph_pairs = false;
      }
    }
    if (b->exec) {
      for (; done + S <= nsteps; done += S) {
        e = hipGraphLaunch(b->exec, b->s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
      }
    }
  }
  while (done < nsteps) {
    const int n = (int)std::min<int64_t>(nsteps - done, use_graph ? S : (int64_t)1 << 30);
    e = launch_batch_persist<T>(a, nwg, n, b->s);
    if (e != hipSuccess) return hip_fail(e, "persistent batch launch");
    done += n;
  }
  for (int g = 0; g < b->nb; ++g) {
    fit_grid* gr = b->grids[g];
    if (nsteps & 1) swap_sets(gr);
    gr->m += nsteps;
    gr->smvp += 2 * nsteps;
  }
  return FIT_OK;
}

template <typename T>
static int batch_run(fit_batch* b, int64_t nsteps, const double* dt, int use_graph) {
  int rc = batch_desc<T>(b, dt, nsteps, true);
  if (rc) return rc;
  if (b->persist) return batch_run_persist<T>(b, nsteps, use_graph);
  // launches: pairs of steps when enabled (an odd last step runs singly)
  const bool pairs = b->pair_on && b->P2 > 0 && nsteps >= 2;
  const int64_t npair = pairs ? nsteps / 2 : 0;
  const int64_t nsingle = nsteps - 2 * npair;
  const int64_t nlaunch = pairs ? npair : nsteps;   // launches of the graphed kind
  const int S = std::max(1, pairs ? b->steps_per_graph / 2 : b->steps_per_graph);
  const int64_t chunks = use_graph ? nlaunch / S : 0;
  const int64_t rem = nlaunch - chunks * S;
  const BatchArgs<T> a = batch_args_host<T>(b, 0);
  const BatchArgs<T> a2 = batch_args_pair<T>(b, 0);
  // a single step advances the counters itself; a pair launch reads them
  // plus its offset within the chunk, and the chunk advances them once
  auto one = [&]() {
    if (!pairs) return launch_batch<T>(a, b->s);
    hipError_t el = launch_batch2<T>(a2, b->s);
    return el == hipSuccess ? launch_batch_advance(b->ctl, 2, 1, b->s) : el;
  };
  auto chunk_of_pairs = [&]() {
    hipError_t el = hipSuccess;
    BatchArgs<T> ak = a2;
    for (int q = 0; q < S && el == hipSuccess; ++q) {
      ak.launch_off = q;
      el = launch_batch2<T>(ak, b->s);
    }
    return el == hipSuccess ? launch_batch_advance(b->ctl, 2 * S, S, b->s) : el;
  };
  hipError_t e = launch_batch_set_base(b->ctl, 0, b->s);
  if (e != hipSuccess) return hip_fail(e, "batch step counter");
  if (chunks > 0) {
    if (!b->exec || b->graph_S != S || b->graph_pairs != pairs) {
      batch_drop_graph(b);
      e = hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "graph capture begin");
      hipError_t el = hipSuccess;
      if (pairs)
        el = chunk_of_pairs();
      else
        for (int q = 0; q < S && el == hipSuccess; ++q) el = one();
      e = hipStreamEndCapture(b->s, &b->graph);
      if (el != hipSuccess) {
        batch_drop_graph(b);
        return hip_fail(el, "batch launch in capture");
      }
      if (e != hipSuccess) {
        batch_drop_graph(b);
        return hip_fail(e, "graph capture end");
      }
      e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        batch_drop_graph(b);
        return hip_fail(e, "graph instantiate");
      }
      b->graph_S = S;
      b->graph_pairs = pairs;
    }
    for (int64_t c = 0; c < chunks; ++c) {
      e = hipGraphLaunch(b->exec, b->s);
      if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
  }
  for (int64_t q = 0; q < rem; ++q) {
    e = one();
    if (e != hipSuccess) return hip_fail(e, "batch launch");
  }
  if (pairs && nsingle > 0) {
    e = launch_batch<T>(a, b->s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
  }
  // every launch writes the other buffer set
  const int64_t launches = pairs ? npair + nsingle : nsteps;
  for (int g = 0; g < b->nb; ++g) {
    fit_grid* gr = b->grids[g];
    if (launches & 1) {
      swap_sets(gr);
    }
    gr->m += nsteps;
    gr->smvp += 2 * nsteps;
  }
  return FIT_OK;
}

// Time `reps` pair launches (every launch reads the same state).
template <typename T>
static int batch_time2(fit_batch* b, const double* dt, int reps, float* ms) {
  int rc = batch_desc<T>(b, dt, 2, true);
  if (rc) return rc;
  const BatchArgs<T> a = batch_args_pair<T>(b, 1);
  hipEvent_t ev[2];
  (void)hipEventCreate(&ev[0]);
  (void)hipEventCreate(&ev[1]);
  hipError_t e = launch_batch2<T>(a, b->s);
  if (e == hipSuccess) e = hipEventRecord(ev[0], b->s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_batch2<T>(a, b->s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], b->s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return hip_fail(e, "batch pair timing");
  *ms /= (float)reps;
  return FIT_OK;
}

// Time `reps` single steps (every step reads the same state) for the current tiling.
template <typename T>
static int batch_time(fit_batch* b, const double* dt, int reps, float* ms) {
  int rc = batch_desc<T>(b, dt, 1, true);
  if (rc) return rc;
  const BatchArgs<T> a = batch_args_host<T>(b, 1);
  hipEvent_t ev[2];
  (void)hipEventCreate(&ev[0]);
  (void)hipEventCreate(&ev[1]);
  hipError_t e = launch_batch<T>(a, b->s);
  if (e == hipSuccess) e = hipEventRecord(ev[0], b->s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_batch<T>(a, b->s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], b->s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return hip_fail(e, "batch autotune timing");
  *ms /= (float)reps;
  return FIT_OK;
}

}  // namespace fit

using namespace fit;

extern "C" {

int fit_batch_destroy(fit_batch* b);

int fit_batch_create(fit_grid* const* grids, int nb, void* stream, fit_batch** out) {
  if (!grids || !out || nb < 1) return fail(FIT_E_INVALID, "need at least one grid");
  *out = nullptr;
  fit_batch* b = new (std::nothrow) fit_batch();
  if (!b) return fail(FIT_E_OOM, "host allocation failed");
  b->nb = nb;
  b->user = static_cast<hipStream_t>(stream);
  for (int g = 0; g < nb; ++g) {
    fit_grid* gr = grids[g];
    if (!gr) {
      delete b;
      return fail(FIT_E_INVALID, "null grid in batch");
    }
    for (int q = 0; q < g; ++q)
      if (grids[q] == gr) {
        delete b;
        return fail(FIT_E_INVALID, "a grid appears twice in the batch");
      }
    if (g > 0 && gr->f64 != grids[0]->f64) {
      delete b;
      return fail(FIT_E_INVALID, "all grids of a batch need the same dtype");
    }
    if (gr->nu) {
      delete b;
      return fail(FIT_E_INVALID, "batched grids need a uniform spacing");
    }
    if (!gr->mu_uniform) {
      delete b;
      return fail(FIT_E_INVALID, "batched grids need a uniform mu");
    }
    b->grids.push_back(gr);
    b->lossy_any |= gr->lossy;
  }
  b->f64 = grids[0]->f64;
  b->tw = 64;
  b->ty = b->f64 ? 4 : 8;

  int rc = FIT_OK;
  for (fit_grid* gr : b->grids)
    if (!rc) rc = ensure_alt(gr);
  hipError_t e = hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess && !rc) rc = hip_fail(e, "batch stream");
  const size_t dsz = b->f64 ? sizeof(BatchGrid<double>) : sizeof(BatchGrid<float>);
  if (!rc) rc = dev_alloc(&b->desc, dsz * nb, "batch descriptors");
  if (!rc) rc = dev_alloc(reinterpret_cast<void**>(&b->ctl), sizeof(BatchCtl), "batch control");
  if (!rc) {
    e = hipMemset(b->ctl, 0, sizeof(BatchCtl));
    if (e != hipSuccess) rc = hip_fail(e, "batch control clear");
  }
  if (!rc) rc = batch_layout(b);
  if (rc) {
    fit_batch_destroy(b);
    return rc;
  }
  *out = b;
  return FIT_OK;
}

int fit_batch_destroy(fit_batch* b) {
  if (!b) return FIT_OK;
  if (b->s) (void)hipStreamSynchronize(b->s);
  batch_drop_graph(b);
  dev_free(b->desc);
  dev_free(reinterpret_cast<void*&>(b->item_grid));
  dev_free(reinterpret_cast<void*&>(b->items2));
  dev_free(reinterpret_cast<void*&>(b->ctl));
  dev_free(b->src_tab);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->s) (void)hipStreamDestroy(b->s);
  delete b;
  return FIT_OK;
}

int fit_batch_set_tuning(fit_batch* b, int tw, int ty, int kc, int steps_per_graph) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  const int ntw = tw != 0 ? tw : b->tw;
  int nty = ty != 0 ? ty : b->ty;
  if (ntw == FIT_TW_ROWS) {
    if (ty == 0 && b->tw != FIT_TW_ROWS) nty = 512;
    if (nty < 128 || nty > 1024 || nty % 64 != 0)
      return fail(FIT_E_INVALID, "row-packed tiles: ty = threads per workgroup, a multiple of 64 in [128, 1024]");
  } else {
    if (!(ntw == 32 || ntw == 64 || ntw == 128 || ntw == 256))
      return fail(FIT_E_INVALID, "tw must be 32, 64, 128, 256 or FIT_TW_ROWS");
    if (ty == 0 && b->tw == FIT_TW_ROWS) nty = std::max(2, 512 / ntw);
    if (nty < 2 || nty > 16 || (nty & (nty - 1)) != 0 || ntw * nty > 1024 || ntw * nty < 64)
      return fail(FIT_E_INVALID, "ty must be a power of two in [2, 16] with 64 <= tw * ty <= 1024");
  }
  if (kc < 0) return fail(FIT_E_INVALID, "kc must be >= 0 (0: whole columns)");
  if (steps_per_graph < 0 || steps_per_graph > 1 << 20)
    return fail(FIT_E_INVALID, "bad steps_per_graph");
  int rc = batch_retune(b, ntw, nty, kc);
  if (rc) return rc;
  if (steps_per_graph > 0) b->steps_per_graph = steps_per_graph;
  return FIT_OK;
}

int fit_batch_get_tuning(const fit_batch* b, int* tw, int* ty, int* kc, int* steps_per_graph,
                         int* nwg) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (tw) *tw = b->tw;
  if (ty) *ty = b->ty;
  if (kc) *kc = b->kc;
  if (steps_per_graph) *steps_per_graph = b->steps_per_graph;
  if (nwg) *nwg = b->P;
  return FIT_OK;
}

int fit_batch_set_pair(fit_batch* b, int enable, int kc) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (enable != 0 && enable != 1) return fail(FIT_E_INVALID, "enable must be 0 or 1");
  if (kc < 0) return fail(FIT_E_INVALID, "kc must be >= 0 (0: whole columns)");
  const int okc = b->pkc;
  b->pkc = kc;
  if (enable) {
    int rc = batch_layout2(b);
    if (rc) {
      b->pkc = okc;
      return rc;
    }
  }
  b->pair_on = enable != 0;
  batch_drop_graph(b);
  return FIT_OK;
}

int fit_batch_set_persistent(fit_batch* b, int enable) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (enable != 0 && enable != 1) return fail(FIT_E_INVALID, "enable must be 0 or 1");
  if (enable) {
    int dev = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        !coop) {
      (void)hipGetLastError();
      return fail(FIT_E_INVALID, "the device does not support cooperative launches");
    }
    const int nwg = persist_workgroups(b);
    if (nwg <= 0)
      return fail(FIT_E_INVALID, "the persistent kernel cannot hold a workgroup of this tile on a CU");
    b->persist_nwg = nwg;
    b->persist_graph = true;
  }
  b->persist = enable != 0;
  batch_drop_graph(b);
  return FIT_OK;
}

int fit_batch_get_persistent(const fit_batch* b, int* enable, int* workgroups, int* captured,
                             int* barrier_failed) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (enable) *enable = b->persist ? 1 : 0;
  if (workgroups)
    *workgroups = !b->persist ? 0 : (b->pair_on && b->P2 > 0) ? persist2_workgroups(b) : b->persist_nwg;
  if (captured) *captured = (b->persist && b->persist_graph) ? 1 : 0;
  if (barrier_failed) {
    BatchCtl c{};
    hipError_t e = hipMemcpyAsync(&c, b->ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, b->s);
    if (e == hipSuccess) e = hipStreamSynchronize(b->s);
    if (e != hipSuccess) return hip_fail(e, "batch control readback");
    *barrier_failed = c.error;
  }
  return FIT_OK;
}

int fit_batch_get_pair(const fit_batch* b, int* enable, int* kc) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (enable) *enable = b->pair_on ? 1 : 0;
  if (kc) *kc = b->pkc;
  return FIT_OK;
}

int fit_batch_get_pair_tile(const fit_batch* b, int g, int* tw, int* ty, int* kc) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (g < 0 || g >= b->nb) return fail(FIT_E_INVALID, "grid index out of range");
  if (!b->pair_on || g >= (int)b->pt2.size())
    return fail(FIT_E_STATE, "step pairs are not enabled for this batch");
  const fit::Tiling& t = b->pt2[(size_t)g];
  if (tw) *tw = t.tw;
  if (ty) *ty = t.ty;
  if (kc) *kc = t.kc;
  return FIT_OK;
}

// Checks made before every batched call: each grid's dt, and the grid
// properties the batch was laid out for, which fit_set_materials,
// fit_set_spacing, fit_set_probe or fit_bind_fields may have changed since.
// A grid that became lossy re-lays the batch out for the lossy tile body
// (its LDS holds the sigma planes); a non-uniform mu or spacing or a probe is
// rejected; a second buffer set dropped by a rebind is allocated again.
static int batch_check_dt(fit_batch* b, const double* dt) {
  if (!dt) return fail(FIT_E_INVALID, "dt array is null");
  bool lossy = false;
  for (int g = 0; g < b->nb; ++g) {
    fit_grid* gr = b->grids[g];
    if (int rc = check_dt(gr, dt[g])) return rc;
    if (gr->probe.on)
      return fail(FIT_E_STATE, "batched steps do not accumulate a probe objective; clear the probe");
    if (gr->nu) return fail(FIT_E_STATE, "a grid of the batch now has a non-uniform spacing");
    if (!gr->mu_uniform) return fail(FIT_E_STATE, "a grid of the batch now has a non-uniform mu");
    if (int rc = ensure_alt(gr)) return rc;
    lossy |= gr->lossy;
  }
  if (lossy != b->lossy_any) {
    const bool old = b->lossy_any;
    b->lossy_any = lossy;
    int rc = batch_layout(b);
    if (!rc && b->pair_on) rc = batch_layout2(b);
    if (rc) {
      const std::string msg = fit_last_error();
      b->lossy_any = old;
      (void)batch_layout(b);
      if (b->pair_on) (void)batch_layout2(b);
      return fail(rc, msg);
    }
  }
  return FIT_OK;
}

// join: the private stream waits for the caller's stream, and vice versa at the end
static int batch_enter(fit_batch* b) {
  hipError_t e = hipEventRecord(b->ev_in, b->user);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->s, b->ev_in, 0);
  if (e != hipSuccess) return hip_fail(e, "batch stream join");
  return FIT_OK;
}
static int batch_leave(fit_batch* b) {
  hipError_t e = hipEventRecord(b->ev_out, b->s);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->user, b->ev_out, 0);
  if (e != hipSuccess) return hip_fail(e, "batch stream join");
  return FIT_OK;
}

// The steps the grids advance with (FP32 grids: rounded down to FP32).
static std::vector<double> batch_dts(const fit_batch* b, const double* dt) {
  std::vector<double> v((size_t)b->nb);
  for (int g = 0; g < b->nb; ++g) v[g] = step_dt(b->grids[g], dt[g]);
  return v;
}

int fit_batch_step(fit_batch* b, int64_t nsteps, const double* dt_in, int use_graph) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (nsteps < 0) return fail(FIT_E_INVALID, "nsteps must be >= 0");
  if (int rc = batch_check_dt(b, dt_in)) return rc;
  if (nsteps == 0) return FIT_OK;
  const std::vector<double> dtv = batch_dts(b, dt_in);
  const double* dt = dtv.data();
  if (int rc = batch_enter(b)) return rc;
  int rc = b->f64 ? batch_run<double>(b, nsteps, dt, use_graph) : batch_run<float>(b, nsteps, dt, use_graph);
  int rc2 = batch_leave(b);
  if (!rc)
    for (int g = 0; g < b->nb; ++g) b->grids[g]->last_dt = dt[g];
  return rc ? rc : rc2;
}

int fit_batch_autotune(fit_batch* b, const double* dt_in, int reps, int* tw, int* ty, int* kc,
                       float* ms_best) {
  if (!b) return fail(FIT_E_INVALID, "null batch");
  if (reps < 1 || reps > 1000) return fail(FIT_E_INVALID, "reps must be in [1, 1000]");
  if (int rc = batch_check_dt(b, dt_in)) return rc;
  const std::vector<double> dtv = batch_dts(b, dt_in);
  const double* dt = dtv.data();
  if (int rc = batch_enter(b)) return rc;
  struct Cand { int tw, ty; };
  std::vector<Cand> shapes;
  for (int nt : {256, 512, 1024}) shapes.push_back({FIT_TW_ROWS, nt});
  for (int w : {32, 64, 128})
    for (int t : {2, 4, 8, 16})
      if (w * t >= 128 && w * t <= 1024) shapes.push_back({w, t});
  const int kcs[5] = {0, 48, 32, 24, 16};
  float best = 1e30f;
  int btw = b->tw, bty = b->ty, bkc = b->kc;
  int rc = FIT_OK;
  for (const Cand& c : shapes) {
    for (int q = 0; q < 5 && !rc; ++q) {
      b->tw = c.tw;
      b->ty = c.ty;
      b->kc = kcs[q];
      if (batch_layout(b) != FIT_OK) continue;   // e.g. tile over the LDS limit
      float ms = 0.f;
      rc = b->f64 ? batch_time<double>(b, dt, reps, &ms) : batch_time<float>(b, dt, reps, &ms);
      if (!rc && ms < best) {
        best = ms;
        btw = c.tw;
        bty = c.ty;
        bkc = kcs[q];
      }
    }
  }
  b->tw = btw;
  b->ty = bty;
  b->kc = bkc;
  int rc2 = batch_layout(b);
  // two steps per launch: taken when a pair beats two single steps by 2 %
  // (short z-chunks: the grids are small, so many items are needed to fill
  // the device)
  b->pair_on = false;
  const int pkc_prev = b->pkc;
  if (!rc && !rc2) {   // (timed as dispatcher-fed launches; the persistent form follows)
    float best_pair = 1e30f;
    int bpkc = -1;
    for (int pk : {6, 8, 12, 16, 24, 32, 0}) {
      b->pkc = pk;
      if (batch_layout2(b) != FIT_OK) break;   // the pair tile does not fit this batch
      float ms = 0.f;
      rc = b->f64 ? batch_time2<double>(b, dt, reps, &ms) : batch_time2<float>(b, dt, reps, &ms);
      if (rc) break;
      if (ms < best_pair) {
        best_pair = ms;
        bpkc = pk;
      }
    }
    if (!rc && bpkc >= 0 && 0.5f * best_pair < 0.98f * best) {
      b->pkc = bpkc;
      rc2 = batch_layout2(b);
      if (!rc2) {
        b->pair_on = true;
        best = 0.5f * best_pair;
      }
    }
  }
  if (!b->pair_on) b->pkc = pkc_prev;
  int rc3 = batch_leave(b);
  if (rc) return rc;
  if (rc2) return rc2;
  if (tw) *tw = btw;
  if (ty) *ty = bty;
  if (kc) *kc = bkc;
  if (ms_best) *ms_best = best;
  return rc3;
}

}  // extern "C"
