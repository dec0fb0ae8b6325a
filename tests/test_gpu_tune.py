"""The launch-shape autotuner: it times every candidate on whole steps of the
caller's solver, applies the fastest, leaves the simulation state as it was
(it works from a checkpoint it restores), and caches its choice per workload
shape."""
import json

import numpy as np
import pytest

from paper_1606_01805_amd import Solver
from paper_1606_01805_amd.tune import autotune
from workloads import configs as C

pytestmark = pytest.mark.gpu

CANDS = [dict(tile_w=64, rows_per_thread=1, persistent_wgs=0, xcd_remap=0, overlap=0),
         dict(tile_w=256, rows_per_thread=2, persistent_wgs=0, xcd_remap=1, overlap=0),
         dict(tile_w=64, rows_per_thread=2, persistent_wgs=0, xcd_remap=1, overlap=1)]


def _state(s):
    return s.populations(0), s.particles(), s.steps_done


def test_autotune_picks_a_candidate_and_leaves_the_state(tmp_path):
    wl = C.couette(storage=C.STORE_F32)
    s = Solver(wl.channels)
    s.step(30, record=False)
    f0, p0, n0 = _state(s)
    cache = str(tmp_path / "tuning.json")
    best, res = autotune(s, steps=20, cands=CANDS, cache=cache)
    assert best in CANDS
    assert len(res) == len(CANDS) and all(v > 0 for v in res.values())
    assert min(res, key=res.get) == json.dumps(best, sort_keys=True)
    t = s.tuning()
    assert all(t[k] == v for k, v in best.items())
    f1, p1, n1 = _state(s)
    assert n1 == n0
    assert np.array_equal(f1, f0) and np.array_equal(p1, p0)

    # the tuned run continues exactly as an untuned one (every launch shape
    # gives the same bits)
    ref = Solver(wl.channels)
    ref.step(30, record=False)
    assert np.array_equal(s.step(40), ref.step(40))
    ref.close()

    # the same workload shape reuses the cached choice without timing
    s2 = Solver(wl.channels)
    best2, res2 = autotune(s2, steps=20, cands=CANDS, cache=cache)
    assert best2 == best and res2 == {}
    s.close()
    s2.close()
