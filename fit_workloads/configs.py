"""Seeded workload recipes (cavity sizes, material maps, sources, probes).

Everything here is input data.  The five named workloads are:

* ``c1``  16x12x8 cells, FP64, vacuum, lossless PEC cavity, 1000 steps,
  initial e = (dual curl of) a seeded random facet potential, h = 0.
* ``c2``  128^3 cells, FP32, 32 dielectric blocks, sigma = 0.05 slabs of 8
  cells at both z faces, Gaussian z-current at the centre node, 10 000 steps.
* ``c3``  256x256x512 cells, FP32, 64 blocks, slabs and source as c2,
  2000 steps, energies every 50 steps (the bandwidth workload).
* ``c4``  64 independent FP32 grids with per-axis sizes ~ U{32..96}, 8 blocks
  each, lossless, random interior source node each, 4000 steps.
* ``c5``  96^3 FP32 adjoint workload: materials as c2, 4096 steps,
  checkpoints every 64 steps, probe box [64, 80]^3.
* ``x1``  the paper's two-dimensional cylindrical wave (Sec. IV-A): a
  20 m x 20 m x 1 m PEC box of vacuum, 41 (or 121) grid points per side in x
  and y and 2 in z, SI constants, the Gaussian line current of eq.
  line_current (1 A, 2e-8 s) on the z edge at the centre, T = 2e-7 s.
  ``x1_graded(points, k)`` is the same box with one element shrunk so that
  the largest over the smallest cell width is k (Sec. IV-A, eq.
  ration-costs): on a tensor grid that element's column in x and row in y
  get width s and all others k s, s = 20 / ((n - 1) k + 1).

Reduced copies (``*_small``) regenerate the same recipe at a smaller size for
parity runs against the oracle.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "WorkloadSpec", "dielectric_blocks", "lossy_slab", "facet_potential",
    "centre_source", "random_source", "batch_sizes", "probe_box",
    "c1", "c2", "c3", "c4", "c5", "c2_small", "c4_small", "c5_small", "scaled",
    "EPS0_SI", "MU0_SI", "x1", "x1_graded", "steps_for", "c3_graded",
]

EPS0_SI = 8.8541878128e-12      # vacuum permittivity [F/m] (CODATA 2018)
MU0_SI = 1.25663706212e-6       # vacuum permeability [H/m] (CODATA 2018)


@dataclasses.dataclass
class WorkloadSpec:
    """A single-grid workload: sizes, per-cell materials and excitation."""
    name: str
    nx: int
    ny: int
    nz: int
    dtype: str                      # "f32" or "f64": field precision
    nsteps: int
    eps_r: np.ndarray               # (nz, ny, nx) float64, > 0
    sigma: Optional[np.ndarray]     # (nz, ny, nx) float64, >= 0, or None (lossless)
    mu_r: Optional[np.ndarray] = None   # (nz, ny, nx) or None (mu_r = 1)
    cfl_frac: float = 0.9           # dt = cfl_frac * dt_CFL
    source: Optional[dict] = None   # see centre_source()
    init_potential_seed: Optional[int] = None  # e0 = dual curl of facet_potential(seed)
    energy_every: int = 0
    probe: Optional[tuple] = None   # ((lo_x, hi_x), (lo_y, hi_y), (lo_z, hi_z)) node coords
    checkpoint_every: int = 0
    spacing: tuple = (1.0, 1.0, 1.0)
    eps0: float = 1.0               # eps = eps0 eps_r, mu = mu0 mu_r
    mu0: float = 1.0
    t_end: Optional[float] = None   # end time; then dt = t_end / ceil(t_end / dt_CFL)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


def dielectric_blocks(nx: int, ny: int, nz: int, nblocks: int, seed: int,
                      lo: float = 1.0, hi: float = 10.0) -> np.ndarray:
    """Per-cell relative permittivity: background 1, ``nblocks`` axis-aligned
    boxes painted in draw order (later blocks overwrite earlier ones).

    Per block and axis the extent is ~ U{ceil(n/16), ceil(n/4)} cells, the
    origin ~ U{0, n - extent}; the value ~ U[lo, hi].
    """
    rng = np.random.default_rng(seed)
    eps = np.ones((nz, ny, nx), dtype=np.float64)
    dims = (nx, ny, nz)
    for _ in range(nblocks):
        ext = [int(rng.integers(math.ceil(n / 16), math.ceil(n / 4) + 1)) for n in dims]
        org = [int(rng.integers(0, n - e + 1)) for n, e in zip(dims, ext)]
        val = float(rng.uniform(lo, hi))
        eps[org[2]:org[2] + ext[2], org[1]:org[1] + ext[1], org[0]:org[0] + ext[0]] = val
    return eps


def lossy_slab(nx: int, ny: int, nz: int, thickness: int, value: float = 0.05) -> np.ndarray:
    """Per-cell conductivity: ``value`` in cells with k < thickness or
    k >= nz - thickness, zero elsewhere."""
    sig = np.zeros((nz, ny, nx), dtype=np.float64)
    t = max(0, min(thickness, nz))
    sig[:t] = value
    sig[nz - t:] = value
    return sig


def facet_potential(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Seeded U[-1, 1] values, one per facet slot, shape (3, nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(3, nz, ny, nx))


def centre_source(nx: int, ny: int, nz: int, sigma_t_steps: float = 20.0,
                  i_max: float = 1.0) -> dict:
    """Gaussian line current on the +z primal edge leaving node
    (nx//2, ny//2, nz//2).  The time width is given in steps; each side
    multiplies it by its own dt."""
    return dict(axis=2, i=nx // 2, j=ny // 2, k=nz // 2,
                i_max=i_max, sigma_t_steps=sigma_t_steps)


def random_source(nx: int, ny: int, nz: int, rng: np.random.Generator,
                  sigma_t_steps: float = 20.0, i_max: float = 1.0) -> dict:
    """Gaussian z-current on an edge leaving a random interior node."""
    i = int(rng.integers(1, nx))
    j = int(rng.integers(1, ny))
    k = int(rng.integers(0, nz))
    return dict(axis=2, i=i, j=j, k=k, i_max=i_max, sigma_t_steps=sigma_t_steps)


def batch_sizes(count: int = 64, lo: int = 32, hi: int = 96, seed: int = 4) -> list:
    """Per-grid (nx, ny, nz), each axis ~ U{lo..hi} independently."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(lo, hi + 1, size=3)) for _ in range(count)]


def probe_box(n: int, size: int) -> tuple:
    """Closed node-coordinate interval [3n/4 - size/2, 3n/4 + size/2]."""
    lo = 3 * n // 4 - size // 2
    return (lo, lo + size)


def scaled(n_big: int, n: int, v: int) -> int:
    return max(1, int(round(v * n / n_big)))


# --------------------------------------------------------------------------- named workloads

def c1() -> WorkloadSpec:
    nx, ny, nz = 16, 12, 8
    return WorkloadSpec(name="c1_cavity_16x12x8_f64", nx=nx, ny=ny, nz=nz, dtype="f64",
                        nsteps=1000, eps_r=np.ones((nz, ny, nx)), sigma=None,
                        init_potential_seed=1, energy_every=1)


def _block_grid(name, nx, ny, nz, dtype, nsteps, nblocks, seed, slab, **kw) -> WorkloadSpec:
    eps = dielectric_blocks(nx, ny, nz, nblocks, seed)
    sig = lossy_slab(nx, ny, nz, slab) if slab > 0 else None
    return WorkloadSpec(name=name, nx=nx, ny=ny, nz=nz, dtype=dtype, nsteps=nsteps,
                        eps_r=eps, sigma=sig, source=centre_source(nx, ny, nz), **kw)


def c2() -> WorkloadSpec:
    return _block_grid("c2_128cube_f32", 128, 128, 128, "f32", 10_000, 32, 2, 8)


def c2_small(n: int = 32, nsteps: int = 1000, dtype: str = "f32") -> WorkloadSpec:
    return _block_grid(f"c2_small_{n}cube_{dtype}", n, n, n, dtype, nsteps, 32, 2,
                       scaled(128, n, 8), energy_every=50)


def c3() -> WorkloadSpec:
    return _block_grid("c3_256x256x512_f32", 256, 256, 512, "f32", 2000, 64, 3, 8,
                       energy_every=50)


def c3_graded() -> WorkloadSpec:
    """c3 on a tensor grid: per-axis cell widths ~ U[0.5, 1.5] (seed 103)."""
    spec = c3()
    rng = np.random.default_rng(103)
    spec.name = "c3_graded_256x256x512_f32"
    spec.spacing = tuple(rng.uniform(0.5, 1.5, n) for n in (spec.nx, spec.ny, spec.nz))
    return spec


def c4(count: int = 64, nsteps: int = 4000, lo: int = 32, hi: int = 96,
       seed: int = 4) -> list:
    sizes = batch_sizes(count, lo, hi, seed)
    rng = np.random.default_rng(seed)
    out = []
    for b, (nx, ny, nz) in enumerate(sizes):
        eps = dielectric_blocks(nx, ny, nz, 8, 4000 + b)
        out.append(WorkloadSpec(name=f"c4_grid{b}_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                                dtype="f32", nsteps=nsteps, eps_r=eps, sigma=None,
                                source=random_source(nx, ny, nz, rng)))
    return out


def c4_small(count: int = 6, nsteps: int = 200) -> list:
    return c4(count=count, nsteps=nsteps, lo=6, hi=20, seed=44)


def c5() -> WorkloadSpec:
    n = 96
    box = probe_box(n, 16)
    return _block_grid("c5_adjoint_96cube_f32", n, n, n, "f32", 4096, 32, 5, 8,
                       probe=(box, box, box), checkpoint_every=64)


def c5_small(n: int = 24, nsteps: int = 4096, dtype: str = "f32") -> WorkloadSpec:
    box = probe_box(n, scaled(96, n, 16))
    return _block_grid(f"c5_small_{n}cube_{dtype}", n, n, n, dtype, nsteps, 32, 5,
                       scaled(96, n, 8), probe=(box, box, box), checkpoint_every=64)


def x1(points: int = 41, dtype: str = "f64") -> WorkloadSpec:
    """Cylindrical wave: ``points`` grid points per side in x, y (so points - 1
    cells of 20 / (points - 1) m), 2 in z (one 1 m cell).  The source is the
    +z edge at the centre node, sigma_t given in seconds (``sigma_t``)."""
    n = points - 1
    d = 20.0 / n
    return WorkloadSpec(name=f"x1_cylindrical_wave_{points}pt_{dtype}", nx=n, ny=n, nz=1,
                        dtype=dtype, nsteps=0, eps_r=np.ones((1, n, n)), sigma=None,
                        cfl_frac=1.0, source=dict(axis=2, i=n // 2, j=n // 2, k=0, i_max=1.0,
                                                  sigma_t=2e-8),
                        spacing=(d, d, 1.0), eps0=EPS0_SI, mu0=MU0_SI, t_end=2e-7)


def x1_graded(points: int = 41, k: float = 1.0, dtype: str = "f64") -> WorkloadSpec:
    """x1 with per-axis cell widths: the cells with x index (points - 1) // 4
    and y index (points - 1) // 4 are k times narrower than all others, the
    box stays 20 m wide."""
    spec = x1(points, dtype)
    n = spec.nx
    small = 20.0 / ((n - 1) * k + 1.0)
    w = np.full(n, k * small)
    w[n // 4] = small
    spec.name = f"x1_graded_k{k:g}_{points}pt_{dtype}"
    spec.spacing = (w.copy(), w.copy(), np.array([1.0]))
    return spec


def steps_for(t_end: float, dt_cfl: float) -> tuple:
    """(n_t, dt): the fewest equal steps of at most dt_cfl that reach t_end."""
    nt = int(math.ceil(t_end / dt_cfl))
    return nt, t_end / nt
