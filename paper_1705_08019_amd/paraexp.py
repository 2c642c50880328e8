"""ParaExp (Sec. III, Alg. 1) on one GPU: the p particular solutions advance
together as one batch (one launch per step of all p grids), the homogeneous
propagations use the library's matrix-exponential action.

The interval (0, T], T = N dt, is split into p sub-intervals of L = N / p
steps.  Grid j (0-based) starts at step j L with zero fields and runs L
leapfrog steps under the source at the global time: its end state is the
particular solution v_(j+1)(T_(j+1)) on the staggered grid.  The homogeneous
part sum_i w_i(T) = exp(T B) x_0 + sum_(j<p) exp((T - T_j) B) v_j(T_j) is
evaluated as the chain y <- exp(L dt B) y + v_j (the same sum by linearity),
with each v_j first collocated at T_j (h(T_j) from h^(m+1/2) and e^m by
the half h-update, one curl application).  The result follows the staggered
reconstruction of Sec. III-B: e^(N) = e_p^(N) + y_e(T) and
h^(N+1/2) = h_p^(N+1/2) + [exp(dt/2 B) y(T)]_h.  B is the operator of
``FitGrid.op_apply``.  This module only orchestrates library calls: every
arithmetic step runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from .batch import FitBatch
from ._lib import FitError
from .grid import FitGrid

__all__ = ["ParaExpResult", "paraexp"]


@dataclasses.dataclass
class ParaExpResult:
    e: torch.Tensor                 # e^(N)
    h: torch.Tensor                 # h^(N+1/2)
    rho: float                      # ||A||_2 used for the Taylor parameters
    tol: float                      # tolerance of every exponential
    expm_params: list               # (m, s) (Taylor) or (K, s) (Leja) of every exponential
    A_applications: int             # applications of B (2 curl products each)
    smvp_leapfrog: int              # curl products of the p particular runs
    C_proc: Optional[int]           # eq. tot_cost with the longest propagation


def paraexp(nx: int, ny: int, nz: int, eps_r, dt: float, nsteps: int, p: int,
            source: Optional[dict] = None, dtype: str = "f32", tol: float = 1e-8,
            rho: Optional[float] = None, norm_iters: int = 60, norm_margin: float = 1.02,
            spacing=(1.0, 1.0, 1.0), e0=None, h0=None, use_graph: bool = True,
            batch_tuning=None, beta: Optional[float] = None,
            method: str = "taylor") -> ParaExpResult:
    """Alg. 1 for a lossless grid with uniform mu.  ``source``: dict(axis, i, j,
    k, i_max, sigma_t) in time units (or sigma_t_steps).  ``rho``: ||A||_2 or a
    bound; by default the power-iteration estimate times ``norm_margin``
    (the Rayleigh quotients approach the norm from below).  ``e0``, ``h0``:
    initial e^(0), h^(1/2) (default zero).  ``beta``: if given, ``tol`` is
    replaced by beta dt^2 / rho (eq. tolerance_leja_2).  ``method``: the
    exponential, "taylor" (scaled truncated Taylor) or "leja" (Leja
    interpolation)."""
    if nsteps % p:
        raise ValueError("nsteps must be divisible by p")
    L = nsteps // p
    grids = []
    for j in range(p):
        g = FitGrid(nx, ny, nz, dtype, spacing=spacing)
        g.set_materials(eps_r)
        if source is not None:
            st = source["sigma_t"] if "sigma_t" in source else source["sigma_t_steps"] * dt
            g.set_source(source["axis"], source["i"], source["j"], source["k"],
                         source.get("i_max", 1.0), st)
        g.set_fields(None, None, j * L)
        grids.append(g)
    dt = grids[0].step_dt(dt)   # the step the leapfrog runs take (FP32: rounded down)
    b = FitBatch(grids)
    if batch_tuning is not None:
        b.set_tuning(*batch_tuning)
    b.step(L, np.full(p, dt), use_graph=use_graph)
    b.close()
    g0 = grids[0]
    if rho is None:
        rho = g0.op_norm(norm_iters) * norm_margin
    if beta is not None:
        tol = FitGrid.expm_tolerance(beta, dt, rho)
    params = []
    ye, yh = g0.new_field(), g0.new_field()
    started = False
    if e0 is not None or h0 is not None:
        xe = torch.as_tensor(e0, dtype=g0.tdtype).to(g0.device).reshape(g0.shape).contiguous() \
            if e0 is not None else g0.new_field()
        xh = torch.as_tensor(h0, dtype=g0.tdtype).to(g0.device).reshape(g0.shape).contiguous() \
            if h0 is not None else g0.new_field()
        g0.axpy(1.0, xe, g0.shift_h(-0.5 * dt, xe, xh), ye, yh)
        started = True
    for j in range(p - 1):
        if started:
            ye, yh, ms = g0.expm(L * dt, ye, yh, rho, tol, method=method)
            params.append(ms)
        ve, vh = grids[j].get_fields()
        g0.axpy(1.0, ve, grids[j].shift_h(-0.5 * dt, ve, vh), ye, yh)   # + v_(j+1)(T_(j+1))
        started = True
    ep, hp = grids[-1].get_fields()
    if started:
        ye, yh, ms = g0.expm(L * dt, ye, yh, rho, tol, method=method)
        params.append(ms)
        he, hh, ms = g0.expm(0.5 * dt, ye, yh, rho, tol, method=method)
        params.append(ms)
        g0.axpy(1.0, ye, hh, ep, hp)       # e^(N) += y_e(T), h^(N+1/2) += y_h(T + dt/2)
    apps = (lambda m, s: m * s) if method == "taylor" else \
        (lambda K, s: (2 * K - 1) * s if K > 0 else 0)
    n_a = sum(apps(m, s) for m, s in params)
    # eq. tot_cost: the longest propagation of the parallel form is (T - T_1);
    # None when that exponential cannot meet ``tol`` in this dtype (its
    # rounding floor grows with the length of the propagation)
    try:
        pick = FitGrid.expm_params if method == "taylor" else FitGrid.leja_params
        m1, s1 = (pick(rho * (nsteps - L) * dt, tol, FitGrid.UNIT_ROUNDOFF[dtype])
                  if p > 1 else (0, 1))
        c_proc = 2 * L + apps(m1, s1) + 2
    except FitError:
        c_proc = None
    res = ParaExpResult(e=ep, h=hp, rho=rho, tol=tol, expm_params=params, A_applications=n_a,
                        smvp_leapfrog=2 * nsteps, C_proc=c_proc)
    for g in grids:
        g.close()
    return res
