"""fit_energy_noalloc (the allocation-free entry point) against fit_energy on
the GPU: two calls in a row, the second on a smaller grid, each bitwise equal
to fit_energy's five values of the same state."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import dielectric_blocks, lossy_slab

pytestmark = pytest.mark.gpu


def _grid(n, seed, lossy):
    from paper_1705_08019_amd import FitGrid
    nx, ny, nz = n
    g = FitGrid(nx, ny, nz, "f32")
    g.set_materials(dielectric_blocks(nx, ny, nz, 6, seed),
                    None, lossy_slab(nx, ny, nz, 2, 0.1) if lossy else None)
    rng = np.random.default_rng(seed)
    g.set_fields(rng.standard_normal((3, nz, ny, nx)), None, 0)
    dt = 0.9 * g.cfl_dt()
    g.set_source(2, nx // 2, ny // 2, nz // 2, 1.0, 5 * dt)
    g.step(13, dt)
    return g


def test_noalloc_energy_equals_fit_energy_twice():
    from paper_1705_08019_amd._lib import call
    out = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    for n, seed, lossy in (((97, 61, 45), 3, True), ((23, 17, 11), 4, False)):
        g = _grid(n, seed, lossy)
        call("fit_energy_noalloc", g.handle, C.c_void_p(out.data_ptr()))
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        want = g.energies()
        ref = np.array([want[k] for k in ("ee", "hh", "W", "Q", "dQ")])
        print(f"{n}: noalloc {got} fit_energy {ref}", flush=True)
        assert np.array_equal(got, ref)
        g.close()


def test_noalloc_limits():
    from paper_1705_08019_amd import FitGrid
    from paper_1705_08019_amd._lib import FitError, call
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    g = FitGrid(8, 8, 8, "f64")
    call("fit_bind_fields", g.handle, None, None, None, None)   # no second buffer set yet
    with pytest.raises(FitError, match="STATE"):
        call("fit_energy_noalloc", g.handle, C.c_void_p(out.data_ptr()))
    g.close()
    g = FitGrid(2048, 2048, 2, "f32")        # more partial rows than the fixed scratch holds
    with pytest.raises(FitError, match="INVALID"):
        call("fit_energy_noalloc", g.handle, C.c_void_p(out.data_ptr()))
    g.close()
