"""Host logic of bench.py (CPU): the HBM traffic it reports comes from
rocprofv3 counters scaled by a plain copy's reading, and is reported only for
the sources and cell size it was taken on; runs on more than one GPU are
refused."""
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

import bench

_HEADER = "Kernel_Name,Counter_Name,Counter_Value\n"


def _csv(path, rows):
    with open(path, "w") as f:
        f.write(_HEADER)
        for name, counter, value in rows:
            f.write(f'"{name}",{counter},{value}\n')
    return str(path)


def _counter_files(tmp_path):
    main = "void sphjet::k_main<float>(sphjet::EvalView<float>)"
    colour = "void sphjet::k_colour<float>(sphjet::EvalView<float>)"
    rescan = "void sphjet::k_main_rescan<float>(sphjet::EvalView<float>)"
    fetch = _csv(tmp_path / "fetch.csv", [(main, "FETCH_SIZE", 100.0), (main, "FETCH_SIZE", 120.0),
                                          (main, "FETCH_SIZE", 110.0), (colour, "FETCH_SIZE", 40.0),
                                          (rescan, "FETCH_SIZE", 9.0), (main, "OTHER", 1e9)])
    write = _csv(tmp_path / "write.csv", [(main, "WRITE_SIZE", 50.0), (main, "WRITE_SIZE", 50.0),
                                          (main, "WRITE_SIZE", 70.0), (colour, "WRITE_SIZE", 10.0)])
    # a 1 GiB copy read as 0.5 GiB and written as 1 GiB (KiB per dispatch)
    cfetch = _csv(tmp_path / "cfetch.csv", [("copy_kernel", "FETCH_SIZE", 1024.0),
                                            ("copy_kernel", "FETCH_SIZE", 524288.0)])
    cwrite = _csv(tmp_path / "cwrite.csv", [("copy_kernel", "WRITE_SIZE", 1048576.0)])
    return fetch, write, cfetch, cwrite


def test_counters_scale_by_the_copy_and_take_medians(tmp_path, monkeypatch):
    out = tmp_path / "traffic_t.json"
    monkeypatch.setattr(bench, "traffic_path", lambda w: str(out))
    args = SimpleNamespace(traffic_from=_counter_files(tmp_path), workload="t", cell_factor=1.05, block_sweep=256)
    bench.write_traffic(args)
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    m = t["kernels"]["main"]
    assert m["dispatches"] == 3
    assert m["fetch_bytes"] == pytest.approx(110.0 * 1024 * 2.0)   # median of 100, 110, 120 KiB
    assert m["write_bytes"] == pytest.approx(50.0 * 1024 * 1.0)    # median of 50, 50, 70 KiB
    assert t["kernels"]["colour"]["fetch_bytes"] == pytest.approx(40.0 * 1024 * 2.0)
    # kernels outside the profiler's names (the rescans) are not reported
    assert set(t["kernels"]) == {"main", "colour"}
    assert t["sources_sha256"] == bench.sources_digest()


def test_traffic_is_reported_only_for_its_sources_and_cell_size(tmp_path, monkeypatch):
    out = tmp_path / "traffic_t.json"
    monkeypatch.setattr(bench, "traffic_path", lambda w: str(out))
    bench.write_traffic(SimpleNamespace(traffic_from=_counter_files(tmp_path), workload="t", cell_factor=1.05,
                                        block_sweep=256))
    b, shape = bench.measured_traffic("t", 1.05, 128, "main")
    assert b == pytest.approx(110.0 * 1024 * 2.0 + 50.0 * 1024)
    assert shape == "cell size 1.05 h, 256-thread sweep blocks"
    assert bench.measured_traffic("t", 2.2, 256, "main") == (None, None)       # other cells
    assert bench.measured_traffic("t", 1.05, 256, "surface") == (None, None)   # not measured
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 64)               # changed kernels
    assert bench.measured_traffic("t", 1.05, 256, "main") == (None, None)
    monkeypatch.setattr(bench, "traffic_path", lambda w: str(tmp_path / "missing.json"))
    assert bench.measured_traffic("t", 1.05, 256, "main") == (None, None)


def test_source_digest_covers_every_hip_source(tmp_path, monkeypatch):
    import shutil
    csrc = tmp_path / "paper_1603_02421_amd" / "csrc"
    shutil.copytree(os.path.join(bench.ROOT, "paper_1603_02421_amd", "csrc"), csrc)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.sources_digest()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            p = csrc / f
            text = p.read_text()
            p.write_text(text + "\n")
            assert bench.sources_digest() != d0, f
            p.write_text(text)
    assert bench.sources_digest() == d0


def test_method_bytes_add_up_to_the_step_model():
    m = bench.METHOD_BYTES
    neighbour_structure = 8 + 4 + 4 + 1.2 + 8 + 2 * 24
    per_step = 2 * (m["colour"] + m["main"] + m["surface"]) + m["predict"] + m["correct"] + neighbour_structure
    assert per_step == pytest.approx(393.2)
    assert per_step <= bench.METHOD_BYTES_PER_STEP < 1.05 * per_step


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
