"""FP32 over the long horizon of the 128^3 workload's recipe: 10 000 leapfrog
steps (Sec. II-A) of a 32^3 copy against the FP64 oracle run with the same
step (an FP32 grid advances with dt rounded down to FP32).

Bars: e and h within 1e-4 relative L2, each measured in the energy norm
against the whole state's energy norm sqrt(<e,e>_eps + <h,h>_mu); the
discrete Poynting balance of every traced step holds on the GPU's own trace
to 1e-6 of the energy scale; in a lossless, source-free copy W, Q and R
(eq. energy) stay at the oracle's conserved values to 1e-6 of the energy
scale and e, h are within 1e-4 of their own norms too.  Individual inner
products <e,e>_eps and <h,h>_mu follow the fields' phase error (at most
twice the field tolerance, 2e-4).  Every achieved error is printed, the
error of h against its own norm included: once the pulse has passed, the
charge it left holds the state's energy in a static e and h decays to a
small fraction of the state; FP32 then loses the e increments below half an
ulp of that static field, and h collects the curl of the frozen rounding
residue, so h's error against its own (small) norm grows to ~1e-3 while the
state's error stays ~1e-6.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fit_workloads import c2_small
from oracle.leapfrog import run, trace_derived
from _glue import oracle_ops, spec_dt, oracle_source, rel_l2, to_np, edges_from_slots, \
    facets_from_slots, edges_to_slots, state_errors

pytestmark = pytest.mark.gpu

N = 10_000
EVERY = 50


def _gpu_run(spec, e0=None):
    from paper_1705_08019_amd import FitGrid
    g = FitGrid(spec.nx, spec.ny, spec.nz, "f32")
    g.set_materials(spec.eps_r, None, spec.sigma)
    dt = spec_dt(spec)
    if spec.source is not None:
        s = oracle_source(spec, dt)
        g.set_source(s["axis"], s["i"], s["j"], s["k"], s["i_max"], s["sigma_t"])
    if e0 is not None:
        g.set_fields(e0, None, 0)
    g.set_pair(True)
    g.trace_config(EVERY, N // EVERY + 1)
    g.step(N, dt)
    e, h = g.get_fields()
    tr, dropped = g.trace_read()
    assert dropped == 0 and len(tr) == N // EVERY
    dt_used = g.step_dt(dt)
    assert dt_used <= dt and np.float32(dt_used) == dt_used
    g.close()
    return to_np(e), to_np(h), tr, dt_used


def test_c2_recipe_10k_steps_fp32():
    spec = c2_small(32, N)
    print(f"c2 recipe 32^3 FP32, {N} steps (GPU)", flush=True)
    e, h, tr, dt = _gpu_run(spec)
    ops = oracle_ops(spec)
    print("oracle run", flush=True)
    e_r, h_r, tr_r = run(ops, np.zeros(ops.n_e), np.zeros(ops.n_h), dt, N,
                         source=oracle_source(spec, dt))
    err = state_errors(ops, edges_from_slots(ops, e), facets_from_slots(ops, h), e_r, h_r)
    rows = tr_r[::EVERY]
    scale = np.nanmax(np.abs(rows[:, 1]) + np.abs(rows[:, 5]))
    d_ee = np.max(np.abs(tr[:, 1] - rows[:, 1])) / scale
    d_hh = np.max(np.abs(tr[:, 5] - rows[:, 5])) / scale
    # Poynting balance on the GPU's own rows: Q^(m+1) - Q^m = -2 dt (loss + source)
    q_m, q_next = tr[1:, 1] + tr[1:, 4], tr[1:, 3] + tr[1:, 6]
    bal = np.max(np.abs((q_next - q_m) + 2 * dt * (tr[1:, 8] + tr[1:, 9]))) / scale
    print(f"fields (state norm) e {err['e_state']:.2e} h {err['h_state']:.2e}; own norms "
          f"e {err['e_own']:.2e} h {err['h_own']:.2e}; <e,e> {d_ee:.2e} <h,h> {d_hh:.2e} of "
          f"the energy scale; balance residual {bal:.2e}", flush=True)
    assert err["e_state"] <= 1e-4 and err["h_state"] <= 1e-4
    assert err["e_own"] <= 1e-4
    assert bal <= 1e-6
    assert d_ee <= 2e-4 and d_hh <= 2e-4


def test_lossless_blocks_10k_steps_fp32_conserve_energy():
    spec = c2_small(32, N)
    spec.sigma = None
    spec.source = None
    rng = np.random.default_rng(21)
    ops = oracle_ops(spec)
    e0_or = rng.standard_normal(ops.n_e)
    e0 = edges_to_slots(ops, e0_or).astype(np.float32)
    e0_or = edges_from_slots(ops, e0.astype(np.float64))   # the FP32 start exactly
    print(f"lossless blocks 32^3 FP32, {N} steps (GPU)", flush=True)
    e, h, tr, dt = _gpu_run(spec, e0)
    print("oracle run", flush=True)
    e_r, h_r, tr_r = run(ops, e0_or, np.zeros(ops.n_h), dt, N)
    ferr = state_errors(ops, edges_from_slots(ops, e), facets_from_slots(ops, h), e_r, h_r)
    d = trace_derived(tr[1:])
    want = trace_derived(tr_r[1:2])          # the conserved values (m = 1)
    scale = abs(want["ee"][0]) + abs(want["hh"][0])
    err = {k: np.max(np.abs(d[k] - want[k][0])) / scale for k in ("W", "Q", "R")}
    print(f"fields own norms e {ferr['e_own']:.2e} h {ferr['h_own']:.2e}, state norm "
          f"e {ferr['e_state']:.2e} h {ferr['h_state']:.2e}; W {err['W']:.2e} Q {err['Q']:.2e} "
          f"R {err['R']:.2e} of the energy scale", flush=True)
    assert max(ferr.values()) <= 1e-4
    assert max(err.values()) <= 1e-6
