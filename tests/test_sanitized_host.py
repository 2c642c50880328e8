"""The host side of libfit under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no device work): the library is rebuilt with the sanitizers on
its host code, loaded into a fresh Python process with the ASan runtime
preloaded, and driven through the entry points that run on the host alone --
argument validation and null handles of every call, the grid constructor's
failure and cleanup path when no device memory can be had, the descriptor
checks, the parameter searches of the exponentials (Taylor and Leja) and the
Leja coefficients over their whole range.  Any sanitizer report aborts the
process and fails the test."""
import glob
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_08019_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(not (os.path.exists(HIPCC) and ASAN_RT),
                                 reason="hipcc or the ASan runtime is not available")]

# Sanitizers on the host pass only (each -fsanitize= behind -Xarch_host).
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

DRIVER = r'''
import ctypes as C, importlib.util, math, re, sys
spec = importlib.util.spec_from_file_location("fit_lib", sys.argv[2])
L = importlib.util.module_from_spec(spec)
spec.loader.exec_module(L)
L.LIB_PATH = sys.argv[1]
lib = L.lib()
text = re.sub(r"/\*.*?\*/", " ", open(sys.argv[3]).read(), flags=re.S)
decl = {m.group(1): [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_]\w*\s*\**\s*(fit_\w+)\s*\(([^)]*)\)\s*;",
                             text, flags=re.M)}
zero = lambda t: t(0.0) if t in (C.c_double, C.c_float) else (t(0) if t in (
    C.c_int, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64) else None)
n = 0
for name, args in L.SIGNATURES.items():          # null handles everywhere
    first = decl[name][0] if decl[name] else ""
    if re.match(r"(const\s+)?fit_(grid|batch)\s*\*", first) and "* const*" not in first:
        rc = getattr(lib, name)(*([None] + [zero(t) for t in args[1:]]))
        assert rc == (0 if name.endswith("_destroy") else -1), (name, rc)
        assert lib.fit_last_error() is not None
        n += 1
assert n > 40, n
# descriptor checks and the constructor's failure / cleanup path
g = C.c_void_p()
for d in ((0, 4, 4, 0), (4, 4, 4, 7), (4, 4, 4, 0)):
    desc = L.GridDesc(d[0], d[1], d[2], 1.0, 1.0, 1.0, 1.0, 1.0, d[3], 0)
    rc = lib.fit_grid_create(C.byref(desc), None, C.byref(g))
    if rc == 0:
        lib.fit_grid_destroy(g)
    else:
        assert lib.fit_last_error(), rc
bad = L.GridDesc(4, 4, 4, -1.0, 1.0, 1.0, 1.0, 1.0, 0, 0)
assert lib.fit_grid_create(C.byref(bad), None, C.byref(g)) == -1
assert lib.fit_grid_create(None, None, C.byref(g)) == -1
# streaming probe argument checks (rejected before any launch)
assert lib.fit_stream_probe(5, None, None, 16, 1, None) == -1
assert lib.fit_stream_probe(0, C.c_void_p(16), C.c_void_p(32), 17, 1, None) == -1
assert lib.fit_stream_probe(0, C.c_void_p(64), C.c_void_p(64), 64, 1, None) == -1
# host parameter searches and coefficients over their range
m, s, K = C.c_int(), C.c_int64(), C.c_int()
for theta in (1e-6, 1e-3, 0.3, 3.0, 40.0, 300.0, 5e3):
    for tol in (1e-14, 1e-10, 1e-6, 3e-3, 0.5):
        for u in (2.0 ** -53, 2.0 ** -24):
            lib.fit_expm_params(theta, tol, u, C.byref(m), C.byref(s))
            lib.fit_leja_params(theta, tol, u, C.byref(K), C.byref(s))
for Kc in range(1, 31):
    for c in (1e-3, 0.5, 3.0, 25.0, 60.0):
        a = (C.c_double * Kc)(); b = (C.c_double * Kc)(); a2 = (C.c_double * Kc)()
        g2 = C.c_double()
        assert lib.fit_leja_coefficients(Kc, c, a, b, a2, C.byref(g2)) == 0
assert lib.fit_leja_coefficients(0, 1.0, None, None, None, None) == -1
assert lib.fit_leja_coefficients(31, 1.0, None, None, None, None) == -1
t = C.c_double()
assert lib.fit_expm_tolerance(1.0, 0.5, 3.5, C.byref(t)) == 0
assert lib.fit_expm_tolerance(1.0, float("inf"), 3.5, C.byref(t)) == -1
print("SANITIZED-HOST-OK", n)
'''


def test_host_code_is_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        objs, procs = [], []
        for src in sorted(glob.glob(os.path.join(CSRC, "*.hip")) +
                          glob.glob(os.path.join(CSRC, "*.cpp"))):
            obj = os.path.join(d, os.path.basename(src) + ".o")
            cmd = [HIPCC] + (["-x", "hip"] if src.endswith(".cpp") else []) + FLAGS + SAN + [
                "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj]
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                          text=True))
            objs.append(obj)
        for p in procs:
            out, _ = p.communicate()
            assert p.returncode == 0, out
        so = os.path.join(d, "libfit_san.so")
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", so, *objs],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, r.stdout
        env = dict(os.environ, LD_PRELOAD=ASAN_RT[-1],
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
                   HIP_VISIBLE_DEVICES="")
        r = subprocess.run([sys.executable, "-c", DRIVER, so,
                            os.path.join(ROOT, "paper_1705_08019_amd", "_lib.py"),
                            os.path.join(ROOT, "include", "fit.h")],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env,
                           timeout=600)
        assert r.returncode == 0 and "SANITIZED-HOST-OK" in r.stdout, r.stdout[-4000:]
