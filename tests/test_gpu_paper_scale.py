"""The paper's own experiments at full size, in the configuration the
experiment drivers run (paper_1606_01805_amd/experiments.py), against the
oracle on their first steps (FP64): the Re = 20 Couette channel of 1000 x 401
with the circle, the square and the AR-10 rectangle at 0.3 marker spacing
(17 to 21 rounds of 64 markers), the closed sedimentation box of the mesh
refinement at N = 40, and the 401 x 3001 box of the kernel comparison with
the polynomial kernel."""
import os

import numpy as np
import pytest

import oracle
from workloads import configs as C

from gpu_util import body_size, series_errors

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def _pair(channel, steps):
    from paper_1606_01805_amd import Solver

    cfg, parts = channel
    s = Solver([(cfg, parts)])
    g = s.step(steps)
    s.close()
    o = oracle.Oracle(cfg)
    o.set_threads(THREADS)
    for p in parts:
        o.add_particle(p)
    r = o.step(steps)
    return series_errors(g[:, 0], r[:, 0], body_size(parts[0]))


@pytest.mark.parametrize("family,y0", [("circle", 0.25), ("square", 0.5), ("rectangle", 0.25)])
def test_paper_couette_channel(family, y0):
    wl = C.paper_couette([(family, y0, 0.0)], storage=C.STORE_F64)
    errs = _pair(wl.channels[0], 20)
    print(family, {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


def test_paper_refinement_box():
    """The flow is at rest to begin with: the sedimentation bars of
    tests/test_gpu_coupled.py (the pressure is a small difference of
    densities near 1)."""
    ch, _ = C.paper_sedimentation_circle(40, storage=C.STORE_F64)
    errs = _pair(ch, 60)
    print({k: f"{v:.1e}" for k, v in errs.items()})
    for k in ("x", "y", "theta", "u", "v", "omega"):
        assert errs[k] < 5e-11, (k, errs)
    for k in ("Fx", "Fy", "M"):
        assert errs[k] < 1e-9, (k, errs)


def test_paper_kernel_box_polynomial():
    ch, _ = C.paper_sedimentation_ellipse(4, storage=C.STORE_F64)
    errs = _pair(ch, 12)
    print({k: f"{v:.1e}" for k, v in errs.items()})
    for k in ("x", "y", "theta", "u", "v", "omega"):
        assert errs[k] < 5e-11, (k, errs)
    for k in ("Fx", "Fy", "M"):
        assert errs[k] < 1e-9, (k, errs)
