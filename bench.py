#!/usr/bin/env python3
"""Benchmark: FIT leapfrog throughput on one MI355X.

Workload (one "step" = one full leapfrog step, e-update + h-update, of the
whole grid): 256 x 256 x 512 cells, FP32 fields, 64 seeded dielectric blocks
(eps_r ~ U[1, 10]), sigma = 0.05 slabs of 8 cells at both z faces, Gaussian
z-current at the centre node (time width 20 steps), dt = 0.9 dt_CFL, FP64
energies every 50 steps.  Inputs are synthetic and resident in HBM before
the timed region starts.

The autotuner picks the kernel path and tile and, on the fused path, whether
pairs of steps run as one launch (bitwise the same fields).  Prints ONE JSON
line with the throughput (Gcell-updates/s), the roofline of the dominant
kernel (algorithmic bytes / measured launch duration, HIP events on the
library's stream), the oracle's CPU throughput on a bounded sample, and the
batched / adjoint / Gram / ParaExp / graded-grid forms.

Usage: python bench.py [--gpus 1] [--steps 2000] [--warmup 50]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FIT leapfrog Gcell-updates/s + % HBM roofline; batched/adjoint vs plain"
PEAK_FP64_MFMA = 78.6     # TFLOP/s, dense FP64 matrix
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E spec
# Algorithmic bytes per cell and step (FP32 fields, per-cell eps_r and sigma,
# no temporal blocking): e-update reads e, h and the 2 material values and
# writes e; h-update reads h, e and writes h.
B_EPASS = 4 * (3 + 3 + 3 + 2)   # 44
B_HPASS = 4 * (3 + 3 + 3)       # 36
B_STEP = B_EPASS + B_HPASS      # 80: the per-cell-step figure with no fusion at all
# Compulsory bytes of one launch of a fused kernel, per cell: read the state
# (e, h) and the per-cell eps and sigma once, write the new state once.  The
# same 56 B hold for a single fused step and for a two-step launch (whose
# intermediate state never leaves the chip), so the roofline fraction of a
# launch cannot exceed 1.
B_LAUNCH = 4 * (6 + 2 + 6)      # 56
# reverse (adjoint) step, FP32 fields: lambda and mu read + written, e^m,
# e^(m+1) and h^(m+1/2) read, eps and sigma read, and the two per-cell FP64
# gradient accumulators read + written
B_ADJ = 4 * (6 + 6 + 9 + 2) + 8 * 2 * 2    # 124


KERNEL_SOURCES = {"step": ("fit_step.hip", "fit_step_tile.hpp", "fit_point.hpp"),
                  "pair": ("fit_step2.hip", "fit_step2_tile.hpp", "fit_step_tile.hpp", "fit_point.hpp"),
                  "epass": ("fit_kernels.hip", "fit_point.hpp"),
                  "hpass": ("fit_kernels.hip", "fit_point.hpp"),
                  "batch_pair": ("fit_batch.hip", "fit_step2_tile.hpp", "fit_step_tile.hpp",
                                 "fit_point.hpp")}


def kernel_source_hash(tag: str) -> str:
    """Hash of the code a kernel is compiled from, comments and blank space
    left out (its counters go stale when the code changes, not when a
    comment does)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_08019_amd", "csrc")
    for f in KERNEL_SOURCES[tag]:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    the counters were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_c3.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get("kernels", {}).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec


def c3_inputs():
    from fit_workloads import c3
    return c3()


def run_plain(spec, steps: int, warmup: int, profile: bool = True, tile=None, pair=None):
    import torch
    from paper_1705_08019_amd import FitGrid
    g = FitGrid(spec.nx, spec.ny, spec.nz, spec.dtype)
    g.set_materials(spec.eps_r, spec.mu_r, spec.sigma)
    dt = spec.cfl_frac * g.cfl_dt()
    s = spec.source
    g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
    every = spec.energy_every
    if tile is None:
        tuned = g.autotune(dt, reps=10)
    else:
        tw = int(tile[3]) if len(tile) > 3 else 64
        g.set_tuning(tile[0], int(tile[1]), int(tile[2]), tw)
        p_, ty_, kc_, tw_ = g.get_tuning()
        tuned = (p_, ty_, kc_, float("nan"), tw_)
    if pair is not None:      # "off" or (tw, ty, kc): overrides the autotuner's choice
        if pair == "off":
            g.set_pair(False)
        else:
            g.set_pair(True, *map(int, pair))
    g.step(warmup, dt)
    # the trace starts with the timed steps: the timed window holds a row at
    # its first step and one every `every` steps (ceil(steps / every) rows)
    g.trace_config(every, steps // every + 4)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    if profile:
        g.profile_begin(steps * 6)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    g.step(steps, dt)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    prof = g.profile_end() if profile else None
    tr, dropped = g.trace_read()
    e_tot = tr[:, 1] + tr[:, 5]
    assert np.all(np.isfinite(e_tot)), "energy trace is not finite"
    out = dict(ms=ms, wall_s=wall, prof=prof, trace_rows=int(tr.shape[0]), tuned=tuned,
               energy_last=float(e_tot[-1]), smvp=g.smvp_count(), grid=g)
    return out


def measure_stream(nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """The measured HBM ceiling: the library's streaming copy / read / fill
    kernels (fit_stream_probe) over 1 GiB buffers, best over grid sizes and
    repetitions; GB/s counts the bytes read plus written."""
    import ctypes as C
    import torch
    from paper_1705_08019_amd._lib import call
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    for mode, name, moved in ((0, "copy", 2 * nbytes), (1, "read", nbytes), (2, "fill", nbytes)):
        best = (1e30, 0)
        for blocks in (1024, 2048, 4096, 8192):
            for _ in range(reps):
                ev[0].record()
                call("fit_stream_probe", mode, C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()),
                     nbytes, blocks, stream)
                ev[1].record()
                torch.cuda.synchronize()
                best = min(best, (ev[0].elapsed_time(ev[1]), blocks))
        out[name + "_GBs"] = round(moved / (best[0] / 1e3) / 1e9, 1)
        out[name + "_blocks"] = best[1]
    del a, b
    out["kernel"] = "fit_stream_probe: 16-byte non-temporal accesses, 4 in flight per lane"
    return out


def cpu_baseline():
    """The oracle (FP64 CSR leapfrog, single thread) on a bounded sample of the
    same recipe: 64 x 64 x 128 cells, 64 blocks, 8-cell lossy slabs, centre
    source; the step count is sized from a 10-step probe to about 15 s of CPU
    work."""
    from threadpoolctl import threadpool_limits
    from fit_workloads import dielectric_blocks, lossy_slab
    from oracle.topology import Topology
    from oracle.materials import Materials
    from oracle.leapfrog import Operators, run
    from oracle.stability import cfl_dt
    nx, ny, nz = 64, 64, 128
    eps = dielectric_blocks(nx, ny, nz, 64, 3)
    sig = lossy_slab(nx, ny, nz, 8)
    t = Topology(nx, ny, nz)
    ops = Operators(t, Materials(t, eps, sigma=sig))
    dt = 0.9 * cfl_dt(eps)
    src = dict(axis=2, i=nx // 2, j=ny // 2, k=nz // 2, i_max=1.0, sigma_t=20 * dt)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, 10, source=src)
        probe = time.perf_counter() - t0
        steps = int(min(2000, max(20, 15.0 / max(probe / 10, 1e-6))))
        t0 = time.perf_counter()
        run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, steps, source=src)
        sec = time.perf_counter() - t0
    return {"value": nx * ny * nz * steps / sec / 1e9, "unit": "Gcell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{nx}x{ny}x{nz} cells of the same recipe, {steps} steps, FP64 CSR "
                      f"leapfrog with per-step energies, {sec:.1f} s on 1 thread "
                      f"({cpu_model()}, {os.cpu_count()} logical CPUs visible)"}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def measure_copy(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Bandwidth of a plain 1 GiB device copy (read + write bytes / time),
    the practical HBM ceiling on this machine; context for the roofline."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = 1e30
    for _ in range(reps):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    del src, dst
    return round(2 * nbytes / (best / 1e3) / 1e9, 1)


def form_batched(plain_steps: int = 400, persistent: bool = True):
    """64 FP32 grids, per-axis sizes ~ U{32..96}, 8 dielectric blocks each,
    lossless, random interior source each, 4000 steps: batched launches
    (graph-captured, autotuned: single steps or step pairs) against plain
    per-grid launches of the same grids (plain timed over `plain_steps`
    steps)."""
    import torch
    from fit_workloads import c4
    from paper_1705_08019_amd import FitGrid, FitBatch
    specs = c4()
    nsteps = specs[0].nsteps

    def make():
        grids, dts = [], []
        for sp in specs:
            g = FitGrid(sp.nx, sp.ny, sp.nz, "f32")
            g.set_materials(sp.eps_r, None, None)
            dt = 0.9 * g.cfl_dt()
            s = sp.source
            g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
            grids.append(g)
            dts.append(dt)
        return grids, np.array(dts)

    cells = sum(sp.cells for sp in specs)
    grids, dts = make()
    b = FitBatch(grids)
    ty, kc, _, tw = b.autotune(dts, reps=5)
    pair_on, pair_kc = b.get_pair()
    b.step(32, dts)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    b.step(nsteps, dts)
    ev[1].record()
    torch.cuda.synchronize()
    ms_b = ev[0].elapsed_time(ev[1])
    # the persistent form: 16 steps of every grid per cooperative launch with a
    # grid-wide barrier between the steps (single steps) or between the pairs
    # of steps (8 pairs per launch), the launch replayed from a hipGraph
    def persistent_form(pairs):
        try:
            if not persistent:
                raise RuntimeError("skipped (--no-persistent)")
            b.set_persistent(False)
            if pairs:
                b.set_pair(True, pair_kc if pair_on else 6)
            else:
                b.set_pair(False)
            ty_, kc_, _, _, tw_ = b.get_tuning()
            b.set_tuning(ty_, kc_, 16, tw_)           # the autotuned tile, 16 steps per launch
            b.set_persistent(True)
            b.step(32, dts)
            torch.cuda.synchronize()
            ev[0].record()
            b.step(nsteps, dts)
            ev[1].record()
            torch.cuda.synchronize()
            ms_ps = ev[0].elapsed_time(ev[1])
            on, nwg, cap, failed = b.get_persistent()
            gps = cells * nsteps / (ms_ps / 1e3) / 1e9
            bcs = B_LAUNCH / 2 if pairs else B_LAUNCH
            out = {"Gcell_updates_per_s": round(gps, 3), "workgroups": nwg,
                   "steps_per_launch": 16, "captured_in_graph": cap, "barrier_gave_up": failed,
                   "alg_bytes_per_cell_update": bcs,
                   "alg_GBs": round(bcs * gps, 1), "frac": round(bcs * gps / PEAK_HBM_GBS, 4)}
            if pairs:
                out["pair_kc"] = b.get_pair()[1]
                out["launch"] = ("8 pairs of steps of all grids per cooperative launch, grid "
                                 "barrier after every pair, each XCD's workgroups walking its "
                                 "own list of the pair item table")
            else:
                out.update({"items_per_step": b.get_tuning()[3], "tile": [tw_, ty_, kc_]})
            return out
        except Exception as ex:   # reported, not hidden
            return {"error": f"{type(ex).__name__}: {ex}"}

    persist = persistent_form(False)
    persist_pairs = persistent_form(True)
    b.close()
    for g in grids:
        g.close()
    grids, dts = make()
    for g, dt in zip(grids, dts):
        g.autotune(dt, reps=3)
        g.step(4, dt)
    torch.cuda.synchronize()
    ev[0].record()
    for g, dt in zip(grids, dts):
        g.step(plain_steps, dt)
    ev[1].record()
    torch.cuda.synchronize()
    ms_p = ev[0].elapsed_time(ev[1])
    for g in grids:
        g.close()
    gb = cells * nsteps / (ms_b / 1e3) / 1e9
    gp = cells * plain_steps / (ms_p / 1e3) / 1e9
    # compulsory bytes per cell-update: 56 B per launch, one or two steps per launch
    bcs = B_LAUNCH / 2 if pair_on else B_LAUNCH
    # counted memory bytes of the pair launch (committed request-size counters
    # of the pairs alone, 16-plane chunks), while they match the kernel's code
    tr = load_traffic("batch_pair") if pair_on else None
    traffic = None
    if tr and tr.get("cells") == cells:
        traffic = {"bytes_per_launch": tr["bytes_per_launch"],
                   "bytes_per_cell": tr["bytes_per_cell"], "pair_kc_counted": 16,
                   "summary": "profiles/batch_pairs_c4.md"}
    return {"workload": "c4: 64 FP32 grids, sizes ~U{32..96}^3, 8 blocks each, 4000 steps",
            "cells_total": cells, "steps": nsteps, "Gcell_updates_per_s": round(gb, 3),
            "alg_bytes_per_cell_update": bcs,
            "alg_GBs": round(bcs * gb, 1), "frac": round(bcs * gb / PEAK_HBM_GBS, 4),
            "plain_per_grid_Gcell_updates_per_s": round(gp, 3),
            "plain_steps_timed": plain_steps, "batched_over_plain": round(gb / gp, 3),
            "tile": [tw, ty, kc], "pair_kc": pair_kc if pair_on else None,
            "pair_traffic": traffic,
            "persistent": persist, "persistent_pairs": persist_pairs,
            "launch": ("one launch per pair of steps of all grids (per-grid pair tiles, the tiles of one z-chunk of a grid on one XCD, longest first), hipGraph "
                       "chunks of 8 pairs" if pair_on else
                       "one launch per step of all grids, hipGraph chunks of 16")}


def form_adjoint():
    """96^3 FP32, materials as the 128^3 workload, 4096 steps, checkpoints
    every 64, probe [64, 80]^3: forward (with checkpoints) and backward
    (segment recompute + reverse sweep) throughput through the autograd
    Function (after one short warm-up run), and the per-step device times of
    the forward step, the recording recompute and the reverse-step kernel."""
    import torch
    from fit_workloads import c5
    from paper_1705_08019_amd import FitGrid, ProbeProblem, probe_energy
    sp = c5()
    box = sp.probe

    def problem(nsteps):
        return ProbeProblem(nx=sp.nx, ny=sp.ny, nz=sp.nz, nsteps=nsteps,
                            probe_lo=tuple(x[0] for x in box), probe_hi=tuple(x[1] for x in box),
                            dtype="f32", checkpoint_every=sp.checkpoint_every, source=sp.source)

    eps = torch.tensor(sp.eps_r, requires_grad=True)
    sig = torch.tensor(sp.sigma, requires_grad=True)
    probe_energy(eps, sig, problem(128)).backward()          # warm-up
    eps.grad = None
    sig.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = probe_energy(eps, sig, problem(sp.nsteps))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cs = sp.cells * sp.nsteps
    fwd = cs / (t1 - t0) / 1e9
    bwd = cs / (t2 - t1) / 1e9

    # per-step device times on the same grid
    g = FitGrid(sp.nx, sp.ny, sp.nz, "f32")
    g.set_materials(sp.eps_r, None, sp.sigma)
    dt = 0.9 * g.cfl_dt()
    s = sp.source
    g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
    g.set_probe([x[0] for x in box], [x[1] for x in box])
    g.autotune(dt, reps=3)
    K = sp.checkpoint_every
    shape = (K + 1, 3, sp.nz, sp.ny, sp.nx)
    er = torch.empty(shape, dtype=torch.float32, device="cuda")
    hr = torch.empty(shape, dtype=torch.float32, device="cuda")
    g.step(64, dt)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    g.step(4 * K, dt)
    ev[1].record()
    torch.cuda.synchronize()
    us_fwd = ev[0].elapsed_time(ev[1]) / (4 * K) * 1e3
    ev[0].record()
    g.step_record(K, dt, er, hr)
    ev[1].record()
    torch.cuda.synchronize()
    us_rec = ev[0].elapsed_time(ev[1]) / K * 1e3
    m0 = g.step_index - K
    best = None
    for _ in range(3):
        g.adjoint_begin(g.step_index, dt)
        torch.cuda.synchronize()
        ev[0].record()
        g.adjoint_segment(m0, K, er, hr)
        ev[1].record()
        torch.cuda.synchronize()
        us = ev[0].elapsed_time(ev[1]) / K * 1e3
        best = us if best is None else min(best, us)
    g.close()
    del er, hr
    ach = B_ADJ * sp.cells / (best * 1e-6) / 1e9
    return {"workload": "c5: 96^3 FP32, 4096 steps, checkpoints every 64, probe 16^3",
            "forward_Gcell_steps_per_s": round(fwd, 3), "adjoint_Gcell_steps_per_s": round(bwd, 3),
            "adjoint_over_forward": round(bwd / fwd, 3), "forward_s": round(t1 - t0, 4),
            "backward_s": round(t2 - t1, 4), "J": float(J.detach()),
            "note": "wall time incl. Python checkpoint bookkeeping; backward = recompute + reverse",
            "step_us": {"forward_with_probe": round(us_fwd, 2), "recompute_recording": round(us_rec, 2),
                        "reverse_k_adj": round(best, 2)},
            "reverse_roofline": {"kernel": "k_adj (fused reverse step + per-cell FP64 gradients)",
                                 "alg_bytes_per_cell": B_ADJ, "achieved": round(ach, 1),
                                 "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": round(ach / PEAK_HBM_GBS, 4),
                                 "note": "96^3 state (21 MB per field set) is largely resident in the 256 MB Infinity Cache"}}


def form_c2(steps: int = 10_000, warmup: int = 100):
    """The 128^3 workload (FP32, 32 blocks, sigma slabs, centre source) over
    its full 10 000 steps, autotuned; its 2.1 M cells (51 MB of state) stay
    resident in the 256 MB Infinity Cache, so its fraction is of the HBM
    roofline but the data mostly come from the cache."""
    import torch
    from fit_workloads import c2
    from paper_1705_08019_amd import FitGrid
    sp = c2()
    g = FitGrid(sp.nx, sp.ny, sp.nz, "f32")
    g.set_materials(sp.eps_r, None, sp.sigma)
    dt = 0.9 * g.cfl_dt()
    s = sp.source
    g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
    p_, ty_, kc_, _, tw_ = g.autotune(dt, reps=10)
    pon, ptw, pty, pkc = g.get_pair()
    g.step(warmup, dt)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    # the rate: the full run without per-launch events (an event pair around
    # each 40 us launch keeps the next launch from starting under the tail of
    # the previous one: about a sixth slower at this size)
    ev[0].record()
    g.step(steps, dt)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    ee, hh = g.energy()
    # the kernel time: a second run of the same length with per-launch events
    g.profile_begin(2 * steps + 16)
    ev[0].record()
    g.step(steps, dt)
    ev[1].record()
    torch.cuda.synchronize()
    prof = g.profile_end()
    ms_prof = ev[0].elapsed_time(ev[1])
    nlaunch = prof["step"][1] + prof["pair"][1] + prof["pair_energy"][1]
    kms = prof["step"][0] + prof["pair"][0] + prof["pair_energy"][0]
    gbs = B_LAUNCH * sp.cells * nlaunch / (kms * 1e-3) / 1e9
    g.close()
    return {"workload": "c2: 128^3 FP32, 32 blocks, sigma=0.05 z-slabs, centre source, "
                        f"{steps} steps (after {warmup} warm-up steps)",
            "Gcell_updates_per_s": round(sp.cells * steps / (ms / 1e3) / 1e9, 2),
            "ms_per_step": round(ms / steps, 5), "tile": [p_, tw_, ty_, kc_],
            "pair_tile": [ptw, pty, pkc] if pon else None,
            "launches": nlaunch, "kernel_ms_per_step": round(kms / steps, 5),
            "ms_per_step_with_launch_events": round(ms_prof / steps, 5),
            "alg_GBs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4),
            "residency": "LLC-resident (51 MB of state in the 256 MB Infinity Cache)",
            "energy_end": [ee, hh]}


def form_graded(steps: int = 300, warmup: int = 20):
    """The bandwidth workload on a tensor grid (per-axis widths ~U[0.5, 1.5]):
    the fused step with per-column / per-plane metric (autotuned tile, single
    steps or step pairs; 80 B algorithmic per cell-update) against the same grid with uniform spacing,
    and both on the split kernels.  Split algorithmic bytes: e-pass 44 B/cell
    (e, h, eps V, sigma V read, e written), h-pass 40 B/cell (e, h, imu V read,
    h written; the uniform split h-pass reads no imu: 36 B)."""
    import torch
    from fit_workloads import c3_graded
    from paper_1705_08019_amd import FitGrid
    spec = c3_graded()
    out = {"workload": "256x256x512 FP32 c3 materials, per-axis cell widths ~U[0.5, 1.5] "
                       f"(seed 103), {steps} steps; fused (autotuned) and split paths"}
    for name, spacing, path in (("graded_fused", spec.spacing, "fused"),
                                ("uniform_fused", (1.0, 1.0, 1.0), "fused"),
                                ("graded", spec.spacing, "split"),
                                ("uniform_split", (1.0, 1.0, 1.0), "split")):
        g = FitGrid(spec.nx, spec.ny, spec.nz, "f32", spacing=spacing)
        g.set_materials(spec.eps_r, None, spec.sigma)
        dt = 0.9 * g.cfl_dt()
        s = spec.source
        g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
        if path == "fused":
            p_, ty_, kc_, _, tw_ = g.autotune(dt, reps=5)
            assert p_ == "fused"
        else:
            g.set_tuning("split")
        g.step(warmup, dt)
        torch.cuda.synchronize()
        g.profile_begin(4 * steps)
        t0 = time.perf_counter()
        g.step(steps, dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = g.profile_end()
        if path == "fused":
            # per-step kernel time over single fused steps and step pairs
            # (two steps per launch, when the autotuner enabled them)
            npair = prof["pair"][1] + prof["pair_energy"][1]
            nstep = prof["step"][1] + 2 * npair
            nlaunch = prof["step"][1] + npair
            kms = prof["step"][0] + prof["pair"][0] + prof["pair_energy"][0]
            st = kms / max(nstep, 1)
            pon, ptw, pty, pkc = g.get_pair()
            # compulsory bytes (56 B per cell and launch) over the kernels' time
            gbs = B_LAUNCH * spec.cells * nlaunch / (kms * 1e-3) / 1e9
            out[name] = {"Gcell_updates_per_s": round(spec.cells * steps / wall / 1e9, 2),
                         "step_ms": round(st, 4), "tile": [tw_, ty_, kc_],
                         "pair_tile": [ptw, pty, pkc] if pon else None,
                         "alg_GBs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
            g.close()
            continue
        ep = prof["epass"][0] / max(prof["epass"][1], 1)
        hp = prof["hpass"][0] / max(prof["hpass"][1], 1)
        hb = 40 if name == "graded" else 36
        out[name] = {"Gcell_updates_per_s": round(spec.cells * steps / wall / 1e9, 2),
                     "epass_ms": round(ep, 4), "hpass_ms": round(hp, 4),
                     "epass_alg_GBs": round(44 * spec.cells / (ep * 1e-3) / 1e9, 1),
                     "hpass_alg_GBs": round(hb * spec.cells / (hp * 1e-3) / 1e9, 1),
                     "dt_cfl": g.cfl_dt()}
        out[name]["epass_frac"] = round(out[name]["epass_alg_GBs"] / PEAK_HBM_GBS, 4)
        out[name]["hpass_frac"] = round(out[name]["hpass_alg_GBs"] / PEAK_HBM_GBS, 4)
        g.close()
    return out


def form_paraexp(p: int = 8, nsteps: int = 1024, tol: float = 3e-3):
    """ParaExp (Alg. 1) on the 128^3 dielectric-block grid without the lossy
    slab (the exponential needs a lossless grid), FP32, p sub-intervals, the
    particular solutions as one batch, Taylor exponentials; against one plain
    leapfrog run of the same N steps.  Also the device time of one
    application of B (k_opb, accumulating mode) and its bytes per cell."""
    import torch
    from fit_workloads import c2
    from paper_1705_08019_amd import FitGrid
    from paper_1705_08019_amd.paraexp import paraexp
    sp = c2()
    g = FitGrid(sp.nx, sp.ny, sp.nz, "f32")
    g.set_materials(sp.eps_r)
    dt = 0.9 * g.cfl_dt()
    s = sp.source
    src = dict(axis=s["axis"], i=s["i"], j=s["j"], k=s["k"], i_max=s["i_max"],
               sigma_t=s["sigma_t_steps"] * dt)
    g.set_source(src["axis"], src["i"], src["j"], src["k"], src["i_max"], src["sigma_t"])
    rho = g.op_norm(60) * 1.02
    g.autotune(dt, reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(nsteps, dt)
    torch.cuda.synchronize()
    t_lf = time.perf_counter() - t0
    e_lf, _ = g.get_fields()
    # one application of B in the accumulating mode, timed with events
    e, h = g.get_fields()
    oe, oh = g.new_field(), g.new_field()
    ae, ah = g.new_field(), g.new_field()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 20
    g.expm(1e-3, e, h, rho, 1e-6, out=(ae, ah))   # warm-up
    torch.cuda.synchronize()
    g.profile_begin(4 * reps)
    for _ in range(reps):
        g.op_apply(e, h)
    prof = g.profile_end()
    us_apply = prof["other"][0] / max(prof["other"][1], 1) * 1e3
    g.close()
    # warm-up with the same arguments: the timed runs find their exponential
    # parameters in the process-wide memo (the search is timed separately)
    paraexp(sp.nx, sp.ny, sp.nz, sp.eps_r, dt, nsteps, p, src, tol=tol, rho=rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = paraexp(sp.nx, sp.ny, sp.nz, sp.eps_r, dt, nsteps, p, src, tol=tol, rho=rho)
    torch.cuda.synchronize()
    t_px = time.perf_counter() - t0
    diff = float(torch.linalg.vector_norm((res.e - e_lf).double()) /
                 torch.linalg.vector_norm(e_lf.double()))
    L = nsteps // p
    t0 = time.perf_counter()
    for th in (rho * L * dt, rho * 0.5 * dt, rho * (nsteps - L) * dt):
        FitGrid.leja_params(th, tol, FitGrid.UNIT_ROUNDOFF["f32"])
    t_search = time.perf_counter() - t0
    paraexp(sp.nx, sp.ny, sp.nz, sp.eps_r, dt, nsteps, p, src, tol=tol, rho=rho, method="leja")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rl = paraexp(sp.nx, sp.ny, sp.nz, sp.eps_r, dt, nsteps, p, src, tol=tol, rho=rho,
                 method="leja")
    torch.cuda.synchronize()
    t_lj = time.perf_counter() - t0
    diff_lj = float(torch.linalg.vector_norm((rl.e - e_lf).double()) /
                    torch.linalg.vector_norm(e_lf.double()))
    diff_tl = float(torch.linalg.vector_norm((rl.e - res.e).double()) /
                    torch.linalg.vector_norm(res.e.double()))
    b_apply = 4 * (6 + 1 + 6)      # read e, h, eps; write the image (mode 0)
    return {"workload": f"128^3 dielectric blocks (seed 2), lossless, FP32, {nsteps} steps, p = {p}, "
                        f"tol {tol:g}",
            "paraexp_s": round(t_px, 4), "leapfrog_s": round(t_lf, 4),
            "paraexp_over_leapfrog_time": round(t_px / t_lf, 2),
            "rel_l2_e_vs_leapfrog": diff, "rho": round(res.rho, 5),
            "expm_params": res.expm_params, "A_applications": res.A_applications,
            "C_proc_parallel_form": res.C_proc, "C_LF": 2 * nsteps,
            "leja": {"paraexp_s": round(t_lj, 4), "paraexp_over_leapfrog_time": round(t_lj / t_lf, 2),
                     "parameter_search_s": round(t_search, 4),
                     "expm_params_K_s": rl.expm_params, "A_applications": rl.A_applications,
                     "C_proc_parallel_form": rl.C_proc, "rel_l2_e_vs_leapfrog": diff_lj,
                     "rel_l2_e_vs_taylor": diff_tl},
            "apply_B_us": round(us_apply, 2),
            "apply_B_alg_GBs": round(b_apply * sp.cells / (us_apply * 1e-6) / 1e9, 1),
            "note": "one GPU: the p particular solutions run as one batch, the homogeneous "
                    "propagations as a chain of exponentials; 128^3 is LLC-resident"}


def gram_mfma_tiles(K: int) -> int:
    """16x16 output tiles the Gram kernel multiplies for K snapshots: per 64x64
    block pair (a0 <= b0) the tiles holding output, upper tile triangle only in
    diagonal blocks."""
    n = 0
    for a0 in range(0, K, 64):
        for b0 in range(a0, K, 64):
            ta = (min(64, K - a0) + 15) // 16
            tb = (min(64, K - b0) + 15) // 16
            n += ta * (ta + 1) // 2 if a0 == b0 else ta * tb
    return n


def form_gram(Ks=(64, 16), reps: int = 5):
    """Gram matrix of K FP32 snapshots of the 128^3 e-field (6.29 M rows) on
    the FP64 matrix cores.  Device time from HIP events around the launches
    (the Gram kernel and its cross-workgroup sum).  `TFLOPs` is the
    dense-product rate 2 rows K^2 / t (the cost G has as a plain product);
    `unique_TFLOPs` counts the K(K+1)/2 distinct entries; `mfma_TFLOPs` counts
    the MFMA work actually issued (whole 16 x 16 tiles of the upper tile
    triangle) and `frac` is that against the FP64 MFMA peak; `read_frac` is
    the snapshots and row weights read once, against the 8 TB/s HBM peak."""
    import torch
    from fit_workloads import c2
    from paper_1705_08019_amd import FitGrid
    sp = c2()
    g = FitGrid(sp.nx, sp.ny, sp.nz, "f32")
    g.set_materials(sp.eps_r, None, sp.sigma)
    rows = 3 * sp.cells
    out = []
    for K in Ks:
        X = torch.randn((K, rows), dtype=torch.float32, device="cuda")
        g.gram(X, 0)
        torch.cuda.synchronize()
        g.profile_begin(64 * reps)
        t0 = time.perf_counter()
        for _ in range(reps):
            g.gram(X, 0)
        sec_wall = (time.perf_counter() - t0) / reps
        ms_dev, n = g.profile_end()["other"]
        ms = ms_dev / reps
        dense = 2.0 * rows * K * K
        unique = 1.0 * rows * K * (K + 1)      # the K(K+1)/2 distinct entries, 2 flop per row each
        mfma = 2.0 * 16 * 16 * rows * gram_mfma_tiles(K)
        nbytes = K * rows * 4 + rows * 8       # the snapshots and the FP64 row weights, read once
        out.append({"workload": f"K={K} FP32 snapshots of the 128^3 e-field ({rows} rows)", "K": K,
                    "ms": round(ms, 4), "ms_wall_incl_readback": round(sec_wall * 1e3, 3),
                    "TFLOPs": round(dense / ms / 1e9, 2),
                    "unique_TFLOPs": round(unique / ms / 1e9, 2),
                    "unique_frac": round(unique / ms / 1e9 / PEAK_FP64_MFMA, 4),
                    "mfma_TFLOPs": round(mfma / ms / 1e9, 2),
                    "peak_fp64_mfma_TFLOPs": PEAK_FP64_MFMA,
                    "frac": round(mfma / ms / 1e9 / PEAK_FP64_MFMA, 4),
                    "read_GBs": round(nbytes / ms / 1e6, 1),
                    "read_frac": round(nbytes / ms / 1e6 / 8000.0, 4)})
        del X
    g.close()
    res = out[0]
    res["others"] = out[1:]
    return res


def calib_copy(nbytes: int = 1 << 30, reps: int = 3):
    """Copies of known size for checking the HBM byte counters: the library's
    streaming copy (k_stream_copy) and torch's copy_, each reading and
    writing exactly nbytes per launch."""
    import ctypes as C
    import torch
    from paper_1705_08019_amd._lib import call
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    res = {}
    for name in ("k_stream_copy", "torch_copy"):
        ms = []
        for _ in range(reps):
            ev[0].record()
            if name == "torch_copy":
                dst.copy_(src)
            else:
                call("fit_stream_probe", 0, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                     nbytes, 8192, stream)
            ev[1].record()
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        res[name] = {"best_ms": round(min(ms), 4),
                     "GBs_read_plus_write": round(2 * nbytes / (min(ms) / 1e3) / 1e9, 1)}
    print(json.dumps({"calib_copy_bytes_each_way": nbytes, "reps": reps, **res}), flush=True)


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _counter_by_launch(d, counter):
    """{(kernel, grid, wg): [values KiB per dispatch]} from a --pmc run."""
    out = {}
    for r in _csv_rows(d, "_counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Kernel_Name"], int(r["Grid_Size"]), int(r["Workgroup_Size"]))
        out.setdefault(key, []).append(float(r["Counter_Value"]))
    return out


def summarize_kernels(kt, out_md, cmd_note, title):
    """Kernel durations of one rocprofv3 --kernel-trace --stats run as
    profiles/<name>.md (every kernel, by total time)."""
    # one row per kernel, merged over the runs found below `kt` (one run per
    # form when the forms are profiled separately)
    merged = {}
    for r in _csv_rows(kt, "_kernel_stats.csv"):
        m = merged.setdefault(r["Name"], {"Name": r["Name"], "Calls": 0, "TotalDurationNs": 0.0,
                                          "MinNs": float("inf"), "MaxNs": 0.0})
        m["Calls"] += int(r["Calls"])
        m["TotalDurationNs"] += float(r["TotalDurationNs"])
        m["MinNs"] = min(m["MinNs"], float(r["MinNs"]))
        m["MaxNs"] = max(m["MaxNs"], float(r["MaxNs"]))
    for m in merged.values():
        m["AverageNs"] = m["TotalDurationNs"] / max(m["Calls"], 1)
    stats = sorted(merged.values(), key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 summary: " + os.path.basename(out_md).replace(".md", ""), "", title, "",
             "Commands (run from the repository root on the MI355X box):", "", "```"]
    lines += cmd_note + ["```", "", "## Kernel durations (--kernel-trace --stats)", "",
                         "| kernel | calls | total ms | avg us | min us | max us |",
                         "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.2f} | "
                     f"{float(r['AverageNs'])/1e3:.2f} | {float(r['MinNs'])/1e3:.2f} | "
                     f"{float(r['MaxNs'])/1e3:.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


# Request-size counters of the L2 (TCC) to memory (EA) interface: reads of
# 32, 64 and 128 bytes, writes of 64 bytes (the rest 32 bytes).  Bytes per
# dispatch = sum(size x count); no scale factor: a copy of known size checks
# them (its counted bytes over the bytes it must move are reported).
RD_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
               "TCC_EA0_RDREQ_128B_sum")
WR_COUNTERS = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_RDREQ_DRAM_sum",
               "TCC_EA0_WRREQ_DRAM_sum")


def _counters(dirs):
    """{(kernel, grid, wg): {counter: [per-dispatch values]}} over --pmc runs."""
    out = {}
    for d in dirs:
        for r in _csv_rows(d, "_counter_collection.csv"):
            key = (r["Kernel_Name"], int(r["Grid_Size"]), int(r["Workgroup_Size"]))
            out.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    return out


def request_bytes(c):
    """(read bytes, write bytes, read requests unaccounted) per dispatch from
    the request-size counters (averages over the dispatches)."""
    def avg(name):
        v = c.get(name) or c.get(name.replace("_sum", ""))
        return sum(v) / len(v) if v else 0.0
    n, n32, n64, n128 = (avg(x) for x in RD_COUNTERS)
    w, w64 = avg("TCC_EA0_WRREQ_sum"), avg("TCC_EA0_WRREQ_64B_sum")
    rd = 32 * n32 + 64 * n64 + 128 * n128
    wr = 64 * w64 + 32 * (w - w64)
    return rd, wr, n - (n32 + n64 + n128)


def summarize(kt, rd_dir, wr_dir, out_md, cells, cmd_note):
    """Kernel durations and request-counted memory bytes of the bandwidth
    workload -> profiles/<name>.md and profiles/traffic_c3.json."""
    stats = _csv_rows(kt, "_kernel_stats.csv")
    cnt = _counters([rd_dir, wr_dir])
    lines = ["# rocprofv3 summary: " + os.path.basename(out_md).replace(".md", ""), "",
             "Commands (run from the repository root on the MI355X box):", "", "```"]
    lines += cmd_note + ["```", "", "## Kernel durations (--kernel-trace --stats)", "",
                         "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.2f} | "
                     f"{float(r['MinNs'])/1e3:.2f} | {float(r['MaxNs'])/1e3:.2f} |")
    lines += ["", "## Memory bytes per dispatch (request-size counters)", "",
              "read = 32 RDREQ_32B + 64 RDREQ_64B + 128 RDREQ_128B, write = 64 WRREQ_64B + "
              "32 (WRREQ - WRREQ_64B), all summed over the TCC instances (L2-miss traffic to "
              "the memory side: Infinity Cache or HBM).  `unaccounted` = RDREQ minus the three "
              "sized counts.  DRAM columns: requests of either size the TCC sends to DRAM.", "",
              "| kernel | grid | wg | dispatches | read MB | write MB | B/cell | "
              "unaccounted reqs | RDREQ_DRAM | WRREQ_DRAM |", "|---|---|---|---|---|---|---|---|---|---|"]
    kernels = {}
    for key in sorted(cnt):
        c = cnt[key]
        rd, wr, lost = request_bytes(c)
        nd = max(len(v) for v in c.values())
        bpc = (rd + wr) / cells
        dram = [sum(c.get(x, [0.0])) / max(len(c.get(x, [0.0])), 1)
                for x in ("TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_WRREQ_DRAM_sum")]
        lines.append(f"| `{key[0][:70]}` | {key[1]} | {key[2]} | {nd} | {rd/1e6:.1f} | "
                     f"{wr/1e6:.1f} | {bpc:.2f} | {lost:.0f} | {dram[0]:.0f} | {dram[1]:.0f} |")
        name = key[0]
        tag = ("pair" if "k_step2<float, true, false" in name
               else "step" if "k_step<float, true, 0, false, false" in name
               else "epass" if "k_epass<float, true, false, false>" in name
               else "hpass" if "k_hpass<float, true, false>" in name
               else "batch_pair" if "k_batch2<float>" in name
               else "stream_copy" if "k_stream_copy" in name else None)
        if tag and (tag not in kernels or nd > kernels[tag]["dispatches"]):
            kernels[tag] = {"source_hash": kernel_source_hash(tag) if tag in KERNEL_SOURCES
                            else None,
                            "bytes_per_launch": round(rd + wr), "read_bytes": round(rd),
                            "write_bytes": round(wr), "bytes_per_cell": round(bpc, 2),
                            "dispatches": nd, "grid": key[1], "wg": key[2], "cells": cells,
                            "method": "request-size counters (no scale factor)"}
    if "stream_copy" in kernels:
        k = kernels["stream_copy"]
        lines += ["", f"Check: the streaming copy of 1 GiB each way counts "
                      f"{k['read_bytes'] / 2**30:.4f} GiB read and {k['write_bytes'] / 2**30:.4f} "
                      f"GiB written per dispatch."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if not kernels:       # no kernel of the bandwidth workload in this summary
        return
    # merge into the traffic record: this summary's kernels replace their own
    # entries, the other kernels' entries (other summaries) stay
    tpath = os.path.join(os.path.dirname(out_md), "traffic_c3.json")
    try:
        with open(tpath) as fh:
            old = json.load(fh)
    except (OSError, ValueError):
        old = {}
    merged = dict(old.get("kernels", {}))
    merged.update(kernels)
    summaries = sorted(set(old.get("summaries", [])) | {os.path.basename(out_md)})
    rec = {"kernels": merged, "summaries": summaries,
           "method": "request-size counters: 32/64/128 B reads, 64/32 B writes"}
    with open(tpath, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def form_batched_pairs(kc: int = 16, steps: int = 200):
    """The batched form's pair launches alone, at a fixed z-chunk length and
    no autotuner or per-grid comparison: a short run for counter passes
    (not part of the default forms)."""
    import torch
    from fit_workloads import c4
    from paper_1705_08019_amd import FitGrid, FitBatch
    specs = c4()
    grids, dts = [], []
    for sp in specs:
        g = FitGrid(sp.nx, sp.ny, sp.nz, "f32")
        g.set_materials(sp.eps_r, None, None)
        dt = 0.9 * g.cfl_dt()
        s = sp.source
        g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t_steps"] * dt)
        grids.append(g)
        dts.append(dt)
    dts = np.array(dts)
    cells = sum(sp.cells for sp in specs)
    b = FitBatch(grids)
    b.set_pair(True, kc)
    b.step(32, dts)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    b.step(steps, dts)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    b.close()
    for g in grids:
        g.close()
    gps = cells * steps / (ms / 1e3) / 1e9
    return {"workload": "c4 grids, step pairs only", "cells_total": cells, "pair_kc": kc,
            "steps": steps, "ms_per_pair_launch": round(2 * ms / steps, 4),
            "Gcell_updates_per_s": round(gps, 2),
            "frac": round(B_LAUNCH / 2 * gps / PEAK_HBM_GBS, 4)}


def run_forms(only=None, persistent=True) -> dict:
    """The batched, adjoint, Gram, ParaExp and graded-grid forms (or those
    named in `only`); a failing form is reported, not hidden."""
    out = {}
    batched = lambda: form_batched(persistent=persistent)
    for name, fn in (("c2", form_c2), ("batched", batched), ("adjoint", form_adjoint),
                     ("gram", form_gram), ("paraexp", form_paraexp), ("graded", form_graded),
                     ("batched_pairs", form_batched_pairs)):
        if (only and name not in only) or (not only and name == "batched_pairs"):
            continue
        try:
            out[name] = fn()
        except Exception as ex:
            out[name] = {"error": f"{type(ex).__name__}: {ex}"}
        print(f"form {name} done", file=sys.stderr, flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip batched/adjoint/Gram forms")
    ap.add_argument("--no-profile", action="store_true", help="no per-launch timing events")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--pair", default=None,
                    help="tw,ty,kc of the two-steps-per-launch kernel, or off (default: autotuner)")
    ap.add_argument("--tile", default=None,
                    help="path,ty,kc[,tw] (e.g. fused,16,128,64): skip the autotuner, use this tile")
    ap.add_argument("--summarize-kernels", nargs=2, metavar=("DIR", "TITLE"), default=None,
                    help="write --summary-out from one rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--forms-only", action="store_true",
                    help="run only the batched / adjoint / Gram / ParaExp / graded forms")
    ap.add_argument("--no-persistent", action="store_true",
                    help="batched form without its persistent sub-form (rocprofv3's kernel "
                         "trace of a process that ran the cooperative launch ends before "
                         "writing its results)")
    ap.add_argument("--form", action="append", default=[],
                    choices=["c2", "batched", "adjoint", "gram", "paraexp", "graded", "batched_pairs"],
                    help="with --forms-only: run only this form (repeatable)")
    ap.add_argument("--summarize", nargs=3, metavar="DIR", default=None,
                    help="kernel-trace, read-counter and write-counter rocprofv3 output dirs "
                         "-> profiles/")
    ap.add_argument("--summary-out", default=os.path.join(ROOT, "profiles", "fused_step_c3.md"))
    ap.add_argument("--summary-cmd", action="append", default=[])
    ap.add_argument("--cells", type=int, default=256 * 256 * 512,
                    help="with --summarize: cells per launch for the B/cell column")
    args = ap.parse_args(argv)
    if args.summarize_kernels:
        summarize_kernels(args.summarize_kernels[0], args.summary_out, args.summary_cmd,
                          args.summarize_kernels[1])
        return
    if args.summarize:
        summarize(*args.summarize, args.summary_out, args.cells, args.summary_cmd)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "layout (z-slab halo exchange) is a design note, not a measured path.",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.calib_copy:
        calib_copy()
        return 0
    if args.forms_only:
        print(json.dumps({"forms": run_forms(args.form, not args.no_persistent)}), flush=True)
        return 0
    spec = c3_inputs()
    cells = spec.cells
    tile = args.tile.split(",") if args.tile else None
    pair = None if args.pair is None else ("off" if args.pair == "off" else args.pair.split(","))
    r = run_plain(spec, args.steps, args.warmup, profile=not args.no_profile, tile=tile, pair=pair)
    ms_step = r["ms"] / args.steps
    value = cells * args.steps / (r["ms"] / 1e3) / 1e9
    roof = None
    path, ty, kc, tw = r["grid"].get_tuning()
    pon, ptw, pty, pkc = r["grid"].get_pair()
    ceiling = measure_stream()
    if r["prof"] is not None:
        st_ms, st_n = r["prof"]["step"]
        pr_ms, pr_n = r["prof"]["pair"]
        if pr_n > 0:   # two fused steps per launch: the dominant kernel
            avg = pr_ms / pr_n
            kname, kb, tkey, steps_per_launch = (
                "k_step2 (two fused leapfrog steps per launch, intermediate state in LDS)",
                B_LAUNCH, "pair", 2)
            st_n = pr_n
        elif st_n > 0:   # fused single-pass step kernel: one launch = one full step
            avg = st_ms / st_n
            kname, kb, tkey, steps_per_launch = (
                "k_step (fused leapfrog step: dual curl + M_eps/M_sigma + source, primal curl "
                "+ M_mu, energies)", B_LAUNCH, "step", 1)
        else:          # split half-step kernels: the e-update is the larger one
            pe_ms, pe_n = r["prof"]["epass"]
            avg = pe_ms / max(pe_n, 1)
            st_n = pe_n
            kname, kb, tkey, steps_per_launch = (
                "k_epass (e-update: dual curl + M_eps/M_sigma + source)", B_EPASS, "epass", 1)
        ach = kb * cells / (avg / 1e3) / 1e9
        tr = load_traffic(tkey)
        eq = B_STEP * steps_per_launch * cells / (avg / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                "traffic": None if tr is None else tr["bytes_per_launch"],
                "alg_bytes_per_cell": kb, "alg_bytes_per_launch": kb * cells,
                "alg_bytes_note": ("compulsory bytes of one launch: the state (e, h) and the "
                                   "per-cell eps, sigma read once, the new state written once"),
                "avg_launch_ms": round(avg, 5), "launches_timed": st_n,
                "steps_per_launch": steps_per_launch,
                "frac_of_measured_copy": round(ach / ceiling["copy_GBs"], 4),
                "measured_ceiling": ceiling,
                "traffic_GBs": None if tr is None else round(
                    tr["bytes_per_launch"] / (avg / 1e3) / 1e9, 1),
                "traffic_frac": None if tr is None else round(
                    tr["bytes_per_launch"] / (avg / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                "traffic_bytes_per_cell": None if tr is None else tr["bytes_per_cell"],
                "traffic_method": None if tr is None else tr.get("method"),
                "unfused_equivalent": {
                    "bytes_per_cell_step": B_STEP, "GBs": round(eq, 1),
                    "note": "80 B per cell-update (e-update and h-update as separate passes, "
                            "no temporal blocking) over this launch's steps; not a fraction "
                            "of the roofline: the fused launch moves fewer bytes"},
                "path": path, "tile": [ptw, pty, pkc] if pr_n > 0 else [tw, ty, kc],
                "single_tile": [path, ty, kc, tw], "pair_tile": [ptw, pty, pkc] if pon else None,
                "energy_pair_launches": r["prof"]["pair_energy"][1],
                "energy_pair_avg_ms": (round(r["prof"]["pair_energy"][0] /
                                             r["prof"]["pair_energy"][1], 5)
                                       if r["prof"]["pair_energy"][1] else None),
                "single_step_launches": r["prof"]["step"][1],
                "single_step_avg_ms": (round(r["prof"]["step"][0] / r["prof"]["step"][1], 5)
                                       if r["prof"]["step"][1] else None),
                "autotune_ms_per_step": (None if r["tuned"][3] != r["tuned"][3]
                                         else round(r["tuned"][3], 5))}
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3: 256x256x512-cell PEC cavity, FP32 fields, 64 dielectric "
                               "blocks, sigma=0.05 z-slabs, Gaussian centre source, FP64 energies "
                               "every 50 steps, dt=0.9 dt_CFL",
                   "cells": cells, "energy_every": spec.energy_every,
                   "trace_rows_timed": r["trace_rows"], "smvp": r["smvp"]},
        "roofline": roof,
    }
    r["grid"].close()
    line["config"]["torch_copy_GBs_read_plus_write"] = measure_copy()
    if not args.no_forms:
        line["forms"] = run_forms()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
