"""lbm_time_kernels, which the benchmark's roofline figures come from: one
time per kernel phase (force and spreading, lattice pass, surface stress),
measured on real steps, so the step count advances by the repetitions."""
import numpy as np
import pytest

from paper_1606_01805_amd import Solver, _lib
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tuning", [dict(tile_w=128, rows_per_thread=2, xcd_remap=1, overlap=0),
                                    dict(tile_w=64, rows_per_thread=1, xcd_remap=1, overlap=1)])
def test_phase_times(tuning):
    wl = C.couette(storage=C.STORE_F32)
    s = Solver(wl.channels, tuning=tuning)
    s.step(4, record=False)
    us = s.time_kernels(6)
    assert us.shape == (3,) and np.all(np.isfinite(us)) and np.all(us > 0), us
    assert s.steps_done == 4 + 6
    assert np.all(np.isfinite(s.particles()))
    s.close()


def test_phase_times_without_particles_and_bad_reps():
    cfg, _ = C.couette(storage=C.STORE_F32).channels[0]
    s = Solver([(cfg, [])])
    us = s.time_kernels(3)
    assert us[1] > 0 and us[2] == 0.0, us
    with pytest.raises(_lib.LBMError) as e:
        s.time_kernels(0)
    assert e.value.code == _lib.LBM_EINVAL
    s.close()
