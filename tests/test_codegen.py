"""Generated gfx950 code of the kernels that share the fused tile body.

A vector register copy placed at a branch join but before the exec mask is
restored (``s_or_b64 exec, exec, ...``) runs only for the lanes that took the
branch; if the copied register is read afterwards by every lane, the other
lanes read stale values.  The FP32 lossy energy+probe variant of the fused
step once got exactly such copies (inside the one-lane block of the source
edge's energy term), which corrupted the h-update coefficient on every other
lane.  This test compiles the kernel sources to AMD assembly (hipcc, no GPU)
and asserts that no join block of any kernel starts with such copies.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_08019_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def join_copies(asm: str) -> dict:
    """{kernel: [label line, ...]} of join labels whose first instructions are
    v_mov copies followed by the exec restore."""
    lines = asm.splitlines()
    fn, hits = None, {}
    for n, l in enumerate(lines):
        if re.match(r"^_Z\w+:", l):
            fn = l.split(":")[0]
        if not re.match(r"^\.LBB\d+_\d+:", l):
            continue
        movs = 0
        for t in (x.strip() for x in lines[n + 1:n + 40]):
            if not t or t.startswith(";"):
                continue
            if t.startswith("s_or_b64 exec, exec"):
                if movs:
                    hits.setdefault(fn, []).append(n + 1)
                break
            if t.startswith(("v_mov_b32", "v_mov_b64")):
                movs += 1
                continue
            break
    return hits


@pytest.mark.parametrize("src", ["fit_step.hip", "fit_batch.hip", "fit_step2.hip"])
def test_no_register_copies_under_a_narrowed_exec_mask(src):
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        r = subprocess.run([HIPCC, *flags, os.path.join(CSRC, src), "-o", out],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, r.stdout
        hits = join_copies(open(out).read())
    assert not hits, hits
