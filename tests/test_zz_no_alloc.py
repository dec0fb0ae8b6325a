"""lbm_get_fields_noalloc (the entry point for callers that cannot allocate
device memory) against lbm_get_fields, through the C ABI: bitwise equal on
two calls in a row, the second on a smaller channel, and a channel above
the staging limit rejected with LBM_ECAPACITY."""
import ctypes

import numpy as np
import pytest

from workloads import configs as C
from workloads import shapes

pytestmark = pytest.mark.gpu


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _noalloc(L, h, ch, nx, ny, with_ux=True):
    r, u, v = (np.full((ny, nx), np.nan) for _ in range(3))
    rc = L.lbm_get_fields_noalloc(h, ch, _p(r), _p(u) if with_ux else None, _p(v))
    return rc, r, u, v


@pytest.mark.parametrize("storage", [C.STORE_F32, C.STORE_F64])
def test_noalloc_fields_equal_allocating_call(storage):
    from paper_1606_01805_amd import Solver, _lib

    L = _lib.lib()
    big = C.couette_config(400, 150, storage=storage)           # 60 000 nodes
    small = C.base_config(37, 23, tau=0.9, body_force=[1e-5, 0.0], storage=storage)
    p = C.particle(shapes.ellipse(20.0, 2.0, n_markers=48), 200.0, 70.3, 0.4)
    s = Solver([(big, [p]), (small, [])])
    s.step(51, record=False)
    for ch, (nx, ny) in ((0, (400, 150)), (1, (37, 23))):      # the second call is smaller
        rc, r, u, v = _noalloc(L, s._h, ch, nx, ny)
        assert rc == _lib.LBM_OK, L.lbm_last_error(s._h)
        ref = s.fields(ch)
        for a, b in zip((r, u, v), ref):
            assert np.array_equal(a, b)
    # an output left NULL is skipped; the others are still written
    rc, r, u, v = _noalloc(L, s._h, 1, 37, 23, with_ux=False)
    assert rc == _lib.LBM_OK and np.isnan(u).all()
    assert np.array_equal(r, s.fields(1)[0]) and np.array_equal(v, s.fields(1)[2])
    s.close()


def test_noalloc_fields_reject_channels_above_the_limit():
    from paper_1606_01805_amd import Solver, _lib

    L = _lib.lib()
    s = Solver([(C.base_config(600, 500, storage=C.STORE_F32), []),   # 300 000 nodes > 262 144
                (C.base_config(512, 512, storage=C.STORE_F32), [])])  # exactly the limit
    rc, r, _, _ = _noalloc(L, s._h, 0, 600, 500)
    assert rc == _lib.LBM_ECAPACITY and np.isnan(r).all()
    assert b"262144" in L.lbm_last_error(s._h)
    rc, r, u, v = _noalloc(L, s._h, 1, 512, 512)
    assert rc == _lib.LBM_OK
    assert np.array_equal(r, s.fields(1)[0])
    assert L.lbm_get_fields_noalloc(s._h, 2, None, None, None) == _lib.LBM_EINVAL
    s.close()
