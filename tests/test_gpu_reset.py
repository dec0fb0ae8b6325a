"""lbm_reset: a handle returned to its initial state runs a new particle set
exactly as a fresh handle with the same channels does (bitwise: same kernels,
same inputs, same launch shapes), and drops what the earlier run held
(checkpoints, the particle set, the step count) while keeping its tuning."""
import numpy as np
import pytest

from paper_1606_01805_amd import Solver, _lib
from workloads import configs as C
from workloads import shapes

pytestmark = pytest.mark.gpu


def _case():
    wl = C.couette(storage=C.STORE_F32)           # 400 x 100, ellipse of 64 markers
    cfg, parts = wl.channels[0]
    other = C.particle(shapes.circle(12.0), 150.0, 40.0, 0.3)  # another marker count and box
    return cfg, parts[0], other


@pytest.mark.parametrize("storage", [C.STORE_F64, C.STORE_F32])
def test_reset_then_new_particle_matches_fresh_handle(storage):
    cfg, p1, p2 = _case()
    s = Solver([(cfg, [p1])], storage=storage, tuning=dict(overlap=1, tile_w=64, rows_per_thread=1))
    tun = s.tuning()
    s.step(37)                                    # graph replays and an eager step
    s.checkpoint_save(0)
    s.reset()
    assert s.steps_done == 0
    assert s.tuning() == tun
    s.add_particle(0, p2)
    t_reset = s.step(50)
    f_reset = s.populations(0)

    fresh = Solver([(cfg, [p2])], storage=storage, tuning=dict(overlap=1, tile_w=64, rows_per_thread=1))
    t_fresh = fresh.step(50)
    f_fresh = fresh.populations(0)
    fresh.close()
    assert np.array_equal(t_reset, t_fresh)
    assert np.array_equal(f_reset, f_fresh)

    # the earlier run's checkpoint is gone, and particles are closed again
    with pytest.raises(_lib.LBMError) as e:
        s.checkpoint_restore(0)
    assert e.value.code == _lib.LBM_ESTATE
    with pytest.raises(_lib.LBMError) as e:
        s.add_particle(0, p1)
    assert e.value.code == _lib.LBM_ESTATE
    s.close()


def test_reset_restores_initial_populations():
    cfg, p1, _ = _case()
    fresh = Solver([(cfg, [])])
    f0 = fresh.populations(0)
    fresh.close()
    s = Solver([(cfg, [p1])])
    s.step(20)
    assert not np.array_equal(s.populations(0), f0)
    s.reset()
    assert np.array_equal(s.populations(0), f0)
    assert s.particles().shape[0] == 0
    s.step(4)                                     # a particle-free run after the reset
    assert s.steps_done == 4
    s.close()
