"""Limits of the boundary, on the GPU path: a particle of the largest marker
count (32 rounds of 64, a force patch near the per-particle cap) against the
oracle, the errors just past each limit, and the zero-step call."""
import numpy as np
import pytest

from paper_1606_01805_amd import Solver, _lib
from workloads import configs as C
from workloads import shapes

from gpu_util import body_size, run_oracle, series_errors

pytestmark = pytest.mark.gpu

MAX_MARKERS = 2048      # per particle (include/lbm.h)
MAX_CELLS = 32768       # force-patch cells per particle


def _err(fn):
    with pytest.raises(_lib.LBMError) as e:
        fn()
    return e.value.code


def test_largest_particle_fp64_matches_oracle():
    """2048 markers on a circle of diameter 160 (off the centre line, so that
    it moves): 32 rounds, each spread into its own partial patch of
    (ceil(2 rb) + 6)^2 = 167^2 = 27 889 cells (rb rounds to just above 80),
    within the cap of 32 768."""
    cfg = C.couette_config(256, 200, storage=C.STORE_F64)
    p = C.particle(shapes.circle(160.0, n_markers=MAX_MARKERS), 128.0, 110.0, 0.2)
    s = Solver([(cfg, [p])])
    g = s.step(120)
    s.close()
    _, r = run_oracle(cfg, [p], 120)
    errs = series_errors(g[:, 0], r[:, 0], body_size(p))
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


def test_particle_limits_rejected():
    cfg = C.couette_config(256, 256, storage=C.STORE_F32)
    s = Solver([(cfg, [])])
    ok = C.particle(shapes.circle(20.0, n_markers=64), 128.0, 128.0)
    # one marker past the per-particle maximum, and too few markers
    too_many = C.particle(shapes.circle(100.0, n_markers=MAX_MARKERS + 1), 128.0, 128.0)
    assert _err(lambda: s.add_particle(0, too_many)) == _lib.LBM_EINVAL
    too_few = C.particle(shapes.circle(20.0, n_markers=2), 128.0, 128.0)
    assert _err(lambda: s.add_particle(0, too_few)) == _lib.LBM_EINVAL
    # a body whose patch, (ceil(2 rb) + 6)^2 = 187^2 cells, exceeds the cap
    big = C.particle(shapes.circle(180.0, n_markers=600), 128.0, 128.0)
    assert 187 ** 2 > MAX_CELLS
    assert _err(lambda: s.add_particle(0, big)) == _lib.LBM_ECAPACITY
    # within 3 nodes of a wall (rb = 10: centre at y = 12 leaves 2 nodes)
    near = C.particle(shapes.circle(20.0, n_markers=64), 128.0, 12.0)
    assert _err(lambda: s.add_particle(0, near)) == _lib.LBM_EINVAL
    # a normal that is not a unit vector
    bad = dict(ok)
    bad["nrm"] = 2.0 * np.asarray(ok["nrm"])
    assert _err(lambda: s.add_particle(0, bad)) == _lib.LBM_EINVAL
    # none of the rejected particles was added; the valid one still is
    assert s.add_particle(0, ok) == 0
    assert s.n_particles == 1
    s.close()


def test_zero_steps_change_nothing():
    wl = C.couette(storage=C.STORE_F32)
    s = Solver(wl.channels)
    s.step(5)
    f = s.populations(0)
    p = s.particles()
    tr = s.step(0)
    assert tr.shape == (0, 1, 10)
    assert s.steps_done == 5
    assert np.array_equal(s.populations(0), f)
    assert np.array_equal(s.particles(), p)
    s.close()
