"""The C ABI on the CPU (no device work): libfit.so loads, exports every
function include/fit.h declares, the binding's ctypes table matches the
header, every entry point rejects a null handle before touching the device,
and the host-only parameter routines of the exponentials (Sec. III-A, eq.
tolerance_leja_2) agree with the oracle."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fit.h")


def _declared():
    """Names and parameter lists of the functions the header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(fit_[a-z0-9_]+)\s*\(([^)]*)\)\s*;",
                         text, flags=re.M):
        out[m.group(1)] = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
    return out


@pytest.fixture(scope="module")
def lib():
    from paper_1705_08019_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfit.so is not built (run the build first)")
    return _lib.lib()


def test_header_declares_the_scope_entry_points():
    names = _declared()
    assert len(names) > 50
    for n in ("fit_grid_create", "fit_set_materials", "fit_step", "fit_energy", "fit_adjoint_step"):
        assert n in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_table_matches_the_header(lib):
    from paper_1705_08019_amd import _lib
    decl = _declared()
    bound = dict(_lib.SIGNATURES)
    bound.update(_lib._CHAR)
    assert set(bound) == set(decl), (set(decl) ^ set(bound))
    for name, args in bound.items():
        assert len(args) == len(decl[name]), name


def _zero(t):
    if t in (C.c_double, C.c_float):
        return t(0.0)
    if t in (C.c_int, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64):
        return t(0)
    return None    # pointers and handles


def test_null_handles_are_rejected(lib):
    """Every entry point whose first parameter is a handle returns
    FIT_E_INVALID for a null one (destroy calls accept it) and records a
    message, without any device work."""
    from paper_1705_08019_amd import _lib
    decl = _declared()
    checked = 0
    for name, args in _lib.SIGNATURES.items():
        first = decl[name][0] if decl[name] else ""
        if not re.match(r"(const\s+)?fit_(grid|batch)\s*\*", first):
            continue
        if "* const*" in first:
            continue
        vals = [None] + [_zero(t) for t in args[1:]]
        rc = getattr(lib, name)(*vals)
        if name.endswith("_destroy"):
            assert rc == 0, name
        else:
            assert rc == -1, (name, rc)
            assert lib.fit_last_error(), name
        checked += 1
    assert checked > 40


def test_version_string(lib):
    assert lib.fit_version().decode().startswith("fitmi")


@pytest.mark.parametrize("theta,tol,u", [(3.0, 1e-12, 2.0 ** -53), (40.0, 1e-8, 2.0 ** -53),
                                         (300.0, 1e-6, 2.0 ** -53), (40.0, 3e-3, 2.0 ** -24),
                                         (1e-3, 1e-10, 2.0 ** -53)])
def test_host_parameter_searches_equal_the_oracle(lib, theta, tol, u):
    from oracle import expm, leja
    K, s = C.c_int(), C.c_int64()
    assert lib.fit_leja_params(theta, tol, u, C.byref(K), C.byref(s)) == 0
    assert (K.value, s.value) == leja.leja_parameters(theta, tol, u)
    m, s2 = C.c_int(), C.c_int64()
    assert lib.fit_expm_params(theta, tol, u, C.byref(m), C.byref(s2)) == 0
    assert (m.value, s2.value) == expm.taylor_parameters(theta, tol, u)


@pytest.mark.parametrize("K,c", [(1, 0.5), (6, 3.0), (19, 25.0), (30, 40.0)])
def test_host_leja_coefficients_equal_the_oracle(lib, K, c):
    import numpy as np
    from oracle import leja
    al, be, a2 = (np.zeros(K) for _ in range(3))
    g2 = C.c_double()
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.fit_leja_coefficients(K, c, ptr(al), ptr(be), ptr(a2), C.byref(g2)) == 0
    ra, rb, ra2, rg2 = leja.scaled_pairs(K, c)
    assert math.isclose(g2.value, rg2, rel_tol=1e-15)
    for x, y in ((al, ra), (be, rb), (a2, ra2)):
        np.testing.assert_allclose(x, y, rtol=1e-11, atol=1e-14 * np.abs(y).max())


def test_host_tolerance_equals_the_oracle(lib):
    from oracle import expm
    t = C.c_double()
    for beta, dt, rho in ((1.0, 0.5, 3.5), (0.2, 1e-12, 3e11)):
        assert lib.fit_expm_tolerance(beta, dt, rho, C.byref(t)) == 0
        assert math.isclose(t.value, expm.optimal_tolerance(beta, dt, rho), rel_tol=1e-15)
    assert lib.fit_expm_tolerance(-1.0, 0.5, 3.5, C.byref(t)) == -1
    assert lib.fit_expm_tolerance(1.0, 0.5, float("nan"), C.byref(t)) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libfit.so the binding raises at the first call: there is no
    fallback path that would compute anything elsewhere."""
    from paper_1705_08019_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libfit.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()
    with pytest.raises(RuntimeError, match="missing"):
        _lib.call("fit_version")
