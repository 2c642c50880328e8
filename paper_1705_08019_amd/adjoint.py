"""Differentiable probe-energy objective of a FIT leapfrog run.

``probe_energy(eps_r, sigma, problem)`` returns
J = dt * sum_{m=1..N} sum_{probe edges} M_eps (e^m)^2 as a 0-d FP64 tensor; its
backward gives dJ/deps_r and dJ/dsigma per cell through the library's
reverse-time adjoint kernels.  The forward run keeps a checkpoint of
(e^m, h^(m+1/2)) every K steps; the backward pass recomputes each K-step
segment from its checkpoint into a recording buffer (fit_step_record) and
runs the reverse steps over it (fit_adjoint_segment), last segment first.
Memory: N/K checkpoints + one (K+1)-state segment buffer.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from .grid import FitGrid

__all__ = ["ProbeProblem", "probe_energy", "ProbeEnergyFunction"]


@dataclasses.dataclass
class ProbeProblem:
    nx: int
    ny: int
    nz: int
    nsteps: int
    probe_lo: tuple
    probe_hi: tuple
    dtype: str = "f32"
    dt: Optional[float] = None          # None: cfl_frac * dt_CFL of the materials
    cfl_frac: float = 0.9
    checkpoint_every: int = 64
    source: Optional[dict] = None       # axis, i, j, k, i_max, sigma_t (time units) or sigma_t_steps
    spacing: tuple = (1.0, 1.0, 1.0)
    e0: Optional[torch.Tensor] = None   # initial e^0 (slot layout), default 0
    h0: Optional[torch.Tensor] = None   # initial h^(1/2), default 0
    autotune: bool = True               # time the forward step's tiles once before the run
    adjoint_tile: Optional[tuple] = None   # (tw, ty, kc) of the reverse step, None: default


def _setup(problem: ProbeProblem, eps_r, sigma) -> tuple:
    g = FitGrid(problem.nx, problem.ny, problem.nz, problem.dtype, spacing=problem.spacing)
    er = eps_r.detach().to("cpu", torch.float64).numpy()
    sg = None if sigma is None else sigma.detach().to("cpu", torch.float64).numpy()
    g.set_materials(er, None, sg)
    dt = problem.dt if problem.dt is not None else problem.cfl_frac * g.cfl_dt()
    s = problem.source
    if s is not None:
        st = s["sigma_t"] if "sigma_t" in s else s["sigma_t_steps"] * dt
        g.set_source(s["axis"], s["i"], s["j"], s["k"], s.get("i_max", 1.0), st)
    g.set_probe(problem.probe_lo, problem.probe_hi)
    if problem.autotune:
        g.autotune(dt, reps=3)
    if problem.adjoint_tile is not None:
        g.adjoint_set_tuning(*problem.adjoint_tile)
    return g, dt


class ProbeEnergyFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, sigma, problem: ProbeProblem):
        g, dt = _setup(problem, eps_r, sigma)
        g.set_fields(problem.e0, problem.h0, 0)
        K = max(1, int(problem.checkpoint_every))
        ckpts = []
        m = 0
        while m < problem.nsteps:
            e, h = g.get_fields()
            ckpts.append((m, e, h))
            n = min(K, problem.nsteps - m)
            g.step(n, dt)
            m += n
        J = g.probe_value()
        ctx.g, ctx.dt, ctx.ckpts, ctx.K, ctx.problem = g, dt, ckpts, K, problem
        ctx.has_sigma = sigma is not None
        ctx.in_device = eps_r.device
        return torch.tensor(J, dtype=torch.float64, device=eps_r.device)

    @staticmethod
    def backward(ctx, gJ):
        g, dt, K, problem = ctx.g, ctx.dt, ctx.K, ctx.problem
        g.adjoint_begin(problem.nsteps, dt)
        shape = (K + 1, 3, g.nz, g.ny, g.nx)
        e_rec = torch.empty(shape, dtype=g.tdtype, device=g.device)
        h_rec = torch.empty(shape, dtype=g.tdtype, device=g.device)
        for m0, e, h in reversed(ctx.ckpts):
            n = min(K, problem.nsteps - m0)
            g.set_fields(e, h, m0)
            g.step_record(n, dt, e_rec, h_rec)
            g.adjoint_segment(m0, n, e_rec, h_rec)
        de, ds = g.adjoint_grad()
        scale = gJ.to(torch.float64)
        d_eps = scale * de
        d_sig = scale * ds if ctx.has_sigma else None
        ctx.g = None
        ctx.ckpts = None
        g.close()
        shp = (problem.nz, problem.ny, problem.nx)
        dev = ctx.in_device
        return d_eps.reshape(shp).to(dev), \
            (None if d_sig is None else d_sig.reshape(shp).to(dev)), None


def probe_energy(eps_r: torch.Tensor, sigma: Optional[torch.Tensor],
                 problem: ProbeProblem) -> torch.Tensor:
    """J(eps_r, sigma) with gradients through the adjoint (see module docstring)."""
    return ProbeEnergyFunction.apply(eps_r, sigma, problem)
