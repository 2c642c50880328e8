"""Host logic of the benchmark's counter summaries (no GPU): request-size
bytes, the per-kernel traffic record and its merge across summaries, and
the source-hash guard that drops stale counters."""
import csv
import json
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PAIR = "void fit::k_step2<float, true, false, 64, 8, 1, true>(fit::S2Args<float>)"
BATCH = "void fit::k_batch2<float>(fit::BatchArgs<float>)"


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _run_dirs(tmp, name, kernel, grid, counters):
    """kernel-trace stats and two counter passes for one kernel, two dispatches."""
    kt, rd, wr = (os.path.join(tmp, name, d) for d in ("kt", "rd", "wr"))
    _write(os.path.join(kt, "x_kernel_stats.csv"),
           [{"Name": kernel, "Calls": 2, "TotalDurationNs": 1000, "AverageNs": 500,
             "MinNs": 490, "MaxNs": 510}])
    for d, names in ((rd, bench.RD_COUNTERS),
                     (wr, ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum"))):
        rows = [{"Kernel_Name": kernel, "Grid_Size": grid, "Workgroup_Size": 768,
                 "Counter_Name": c, "Counter_Value": counters[c]}
                for _ in range(2) for c in names]
        _write(os.path.join(d, "x_counter_collection.csv"), rows)
    return kt, rd, wr


def test_request_bytes_sizes_each_request_class():
    c = {"TCC_EA0_RDREQ_sum": [10.0], "TCC_EA0_RDREQ_32B_sum": [1.0],
         "TCC_EA0_RDREQ_64B_sum": [2.0], "TCC_EA0_RDREQ_128B_sum": [6.0],
         "TCC_EA0_WRREQ_sum": [5.0], "TCC_EA0_WRREQ_64B_sum": [3.0]}
    rd, wr, lost = bench.request_bytes(c)
    assert rd == 32 * 1 + 64 * 2 + 128 * 6
    assert wr == 64 * 3 + 32 * 2
    assert lost == 1


def test_summaries_merge_per_kernel_records_with_their_own_cells(tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    cnt = {"TCC_EA0_RDREQ_sum": 100.0, "TCC_EA0_RDREQ_32B_sum": 0.0,
           "TCC_EA0_RDREQ_64B_sum": 0.0, "TCC_EA0_RDREQ_128B_sum": 100.0,
           "TCC_EA0_WRREQ_sum": 50.0, "TCC_EA0_WRREQ_64B_sum": 50.0}
    a = _run_dirs(str(tmp_path), "a", PAIR, 393216, cnt)
    b = _run_dirs(str(tmp_path), "b", BATCH, 1959936, cnt)
    bench.summarize(*a, str(prof / "one.md"), 1000, ["cmd a"])
    bench.summarize(*b, str(prof / "two.md"), 500, ["cmd b"])
    rec = json.loads((prof / "traffic_c3.json").read_text())
    assert rec["summaries"] == ["one.md", "two.md"]
    pair, batch = rec["kernels"]["pair"], rec["kernels"]["batch_pair"]
    per_launch = 128 * 100 + 64 * 50
    assert pair["bytes_per_launch"] == batch["bytes_per_launch"] == per_launch
    assert pair["cells"] == 1000 and batch["cells"] == 500
    assert pair["bytes_per_cell"] == round(per_launch / 1000, 2)
    assert batch["bytes_per_cell"] == round(per_launch / 500, 2)
    assert pair["source_hash"] == bench.kernel_source_hash("pair")
    assert "cmd b" in (prof / "two.md").read_text()
    # a summary with none of the tagged kernels leaves the record alone
    c = _run_dirs(str(tmp_path), "c", "void other_kernel()", 64, cnt)
    before = (prof / "traffic_c3.json").read_text()
    bench.summarize(*c, str(prof / "three.md"), 10, [])
    assert (prof / "traffic_c3.json").read_text() == before


def test_stale_counters_are_not_reported(tmp_path, monkeypatch):
    """load_traffic returns an entry only while the kernel's sources hash to
    the value recorded with it; a change outside comments drops it."""
    root = tmp_path / "repo"
    csrc = root / "paper_1705_08019_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES["pair"]:
        shutil.copy(os.path.join(ROOT, "paper_1705_08019_amd", "csrc", f), csrc / f)
    (root / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.kernel_source_hash("pair")
    (root / "profiles" / "traffic_c3.json").write_text(json.dumps(
        {"kernels": {"pair": {"source_hash": h, "bytes_per_launch": 7, "cells": 1}}}))
    assert bench.load_traffic("pair")["bytes_per_launch"] == 7
    f = csrc / bench.KERNEL_SOURCES["pair"][0]
    f.write_text(f.read_text() + "\n// a comment does not make the counters stale\n")
    assert bench.load_traffic("pair") is not None
    f.write_text(f.read_text() + "\nstatic int extra_symbol = 0;\n")
    assert bench.load_traffic("pair") is None


@pytest.mark.parametrize("tag", sorted(bench.KERNEL_SOURCES))
def test_every_traced_kernel_has_its_sources(tag):
    for f in bench.KERNEL_SOURCES[tag]:
        assert os.path.exists(os.path.join(ROOT, "paper_1705_08019_amd", "csrc", f)), f
