"""Host logic of bench.py that needs no GPU: the one-GPU contract, the
roofline record and the launch shapes it names."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in out and out["n_gpus"] == 2


def test_roofline_record():
    import bench

    r = bench.roofline(100.0, 1_000_000, 1, None, dict(vec=1, overlap=1), 0.2)
    assert r["kernel"].startswith("lattice_traction_vkernel")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    # 72 B per node (FP32) over 100 us
    assert r["achieved"] == pytest.approx(1e6 * 72 / 100e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["whole_step"]["frac"] == pytest.approx(1e6 * 72 / 0.2e-3 / 1e9 / 8000.0)
    assert bench.roofline(1.0, 10, 2, None, dict(vec=1), None)["kernel"] == "lattice_vkernel"
    assert bench.roofline(1.0, 10, 0, None, {}, None)["kernel"] == "lattice_kernel"
    assert bench.BYTES_PER_LUP == {0: 144, 1: 72, 2: 36}


@pytest.mark.parametrize("name", ["couette", "sedimentation", "ensemble", "large", "large16", "huge", "huge16"])
def test_benchmark_shapes_are_valid(name):
    """Every launch shape the benchmark uses passes the library's own
    checks (no GPU call: the shapes are checked against the rules of
    lbm_set_tuning restated here, and against the storage form)."""
    import bench

    t = dict(bench.WORKLOAD_TUNING.get(name) or bench.VARIANT_TUNING[name])
    storage = 2 if name.endswith("16") else (0 if name == "sedimentation" else 1)
    elem = {0: 8, 1: 4, 2: 2}[storage]
    if t.get("vec"):
        nv = t["tile_w"] // 64
        assert t["tile_w"] % 64 == 0 and nv in (1, 2, 4, 8) and nv * elem <= 16
        assert t.get("rows_per_thread", 1) in (1, 2)
        if t.get("overlap"):
            assert t.get("rows_per_thread", 1) == 1 and t.get("persistent_wgs", 0) == 0
    else:
        assert t["tile_w"] in (64, 128, 256)
        assert not t.get("nt_store")
        if t.get("overlap"):
            assert t["tile_w"] == 64 and t.get("persistent_wgs", 0) == 0
