"""Test glue: build oracle problems from workload specs, compare slot arrays.

Only tests import this module.  It translates between the seeded inputs of
fit_workloads, the oracle's entity numbering and the slot layout used by the
HIP library; it contains no method arithmetic of its own.
"""
from __future__ import annotations

import numpy as np

from oracle.topology import Topology
from oracle.materials import Materials
from oracle.leapfrog import Operators
from oracle.stability import cfl_dt
from oracle import layout


def oracle_ops(spec_or_dims, eps=None, sigma=None, mu=None, spacing=(1.0, 1.0, 1.0)):
    if hasattr(spec_or_dims, "nx"):
        s = spec_or_dims
        t = Topology(s.nx, s.ny, s.nz)
        return Operators(t, Materials(t, s.eps_r, sigma=s.sigma, mu_r=s.mu_r,
                                      spacing=s.spacing, eps0=s.eps0, mu0=s.mu0))
    nx, ny, nz = spec_or_dims
    t = Topology(nx, ny, nz)
    eps = np.ones((nz, ny, nx)) if eps is None else eps
    return Operators(t, Materials(t, eps, sigma=sigma, mu_r=mu, spacing=spacing))


def spec_dt(spec) -> float:
    return spec.cfl_frac * cfl_dt(spec.eps_r, spec.mu_r, spec.spacing, spec.eps0, spec.mu0)


def oracle_source(spec, dt):
    if spec.source is None:
        return None
    s = dict(spec.source)
    if "sigma_t_steps" in s:
        s["sigma_t"] = s.pop("sigma_t_steps") * dt
    return s


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def to_np(x):
    try:
        import torch
        if isinstance(x, torch.Tensor):
            return x.detach().to("cpu", dtype=torch.float64).numpy()
    except ImportError:
        pass
    return np.asarray(x, dtype=np.float64)


edges_from_slots = layout.edges_from_slots
facets_from_slots = layout.facets_from_slots
edges_to_slots = layout.edges_to_slots
facets_to_slots = layout.facets_to_slots


def state_errors(ops, e, h, e_ref, h_ref) -> dict:
    """Errors of e and h (kept-entity vectors) against the reference: each
    relative to its own L2 norm, and each in the energy norm relative to the
    energy norm of the whole reference state, sqrt(<e,e>_eps + <h,h>_mu)."""
    de, dh = np.asarray(e) - e_ref, np.asarray(h) - h_ref
    scale = np.sqrt(e_ref @ (ops.M_eps * e_ref) + h_ref @ (ops.M_mu * h_ref))
    return dict(e_own=rel_l2(e, e_ref), h_own=rel_l2(h, h_ref),
                e_state=float(np.sqrt(de @ (ops.M_eps * de)) / scale),
                h_state=float(np.sqrt(dh @ (ops.M_mu * dh)) / scale))
