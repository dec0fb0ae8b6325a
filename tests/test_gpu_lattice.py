"""GPU lattice pass vs the oracle (Sec. 1.1): the FP64 form performs the same
IEEE operations as the oracle and must match it bit for bit; the reduced
forms within their storage precision."""
import numpy as np
import pytest

import oracle
from workloads import configs as C

from gpu_util import run_gpu

pytestmark = pytest.mark.gpu
RNG = np.random.default_rng(42)


def _lattice_pair(cfg, steps, f=None, storage=None, tuning=None):
    from paper_1606_01805_amd import Solver

    s = Solver([(cfg, [])], storage=storage, tuning=tuning)
    o = oracle.Oracle(cfg)
    if f is not None:
        s.set_populations(f)
        o.set_populations(f)
    s.step(steps, record=False)
    o.step(steps, record=False)
    a, b = s.populations(), o.populations()
    s.close()
    return a, b


def _noisy(ny, nx, amp=0.05):
    _, w = oracle.lattice()
    return w[:, None, None] * (1 + amp * RNG.standard_normal((9, ny, nx)))


@pytest.mark.parametrize("nx,ny", [(70, 37), (3, 3), (64, 4), (257, 9)])
def test_periodic_box_bitwise(nx, ny):
    cfg = C.base_config(nx, ny, tau=0.9, body_force=[1e-5, -2e-6])
    a, b = _lattice_pair(cfg, 25, _noisy(ny, nx))
    assert np.array_equal(a, b)


def test_couette_bitwise():
    a, b = _lattice_pair(C.couette_config(100, 33), 200)
    assert np.array_equal(a, b)


def test_couette_from_rest_bitwise():
    cfg = C.couette_config(65, 17, tau=0.8)
    cfg["init"] = 0
    a, b = _lattice_pair(cfg, 500)
    assert np.array_equal(a, b)


def test_poiseuille_bitwise():
    a, b = _lattice_pair(C.base_config(40, 17, tau=0.8, bc_y=1, body_force=[1e-6, 0.0]), 300)
    assert np.array_equal(a, b)


def test_side_walls_bitwise():
    cfg = C.base_config(19, 30, tau=0.7, bc_x=1, body_force=[0.0, 2e-6],
                        u_wall=[[0.0, 0.01], [0.0, -0.02], [0, 0], [0, 0]])
    a, b = _lattice_pair(cfg, 300)
    assert np.array_equal(a, b)


def _bump(nx, ny, amp=0.01, cfg=None):
    """Equilibrium populations of a density bump at rest.  With cfg, the
    oracle's populations after one step from it, which satisfy that
    channel's wall and corner closures (the GPU applies the closures on the
    load after lbm_set_populations, the oracle only after streaming)."""
    f = np.zeros((9, ny, nx))
    for y in range(ny):
        for x in range(nx):
            dx, dy = x - 0.37 * nx, y - 0.61 * ny
            f[:, y, x] = oracle.equilibrium(1.0 + amp * np.exp(-(dx * dx + dy * dy) / 6.0), 0.0, 0.0)
    if cfg is not None:
        o = oracle.Oracle(cfg)
        o.set_populations(f)
        o.step(1, record=False)
        f = o.populations()
    return f


@pytest.mark.parametrize("nx,ny", [(23, 17), (3, 3), (70, 4)])
def test_closed_box_bitwise(nx, ny):
    """Walls on both axes: the corner closure of reading R23 (each corner
    takes its diagonal interior neighbour's density) matches the oracle bit
    for bit."""
    cfg = C.base_config(nx, ny, tau=0.8, bc_x=1, bc_y=1)
    a, b = _lattice_pair(cfg, 60, _bump(nx, ny, cfg=cfg))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("storage,tol", [(C.STORE_F32, 2e-8), (C.STORE_F16S, 3e-5)])
def test_closed_box_reduced_forms(storage, tol):
    cfg = C.base_config(31, 22, tau=0.8, bc_x=1, bc_y=1)
    f = _bump(31, 22, cfg=cfg)
    a, b = _lattice_pair(cfg, 60, f, storage=storage)
    assert np.abs(a - b).max() < tol


@pytest.mark.parametrize("tile_w,npt,pers,ov", [(64, 1, 0, 0), (128, 2, 0, 0), (256, 4, 0, 0), (64, 4, 7, 0),
                                                (256, 1, 3, 0), (64, 1, 0, 1), (64, 2, 0, 1), (64, 4, 0, 1)])
def test_launch_shapes_do_not_change_results(tile_w, npt, pers, ov):
    """Tile shape, persistent grid and the combined lattice / surface-stress
    launch (ov = 1, 64 x 9*npt tiles) give bitwise the same populations."""
    cfg = C.base_config(130, 45, tau=0.8, bc_y=1, body_force=[1e-6, 0.0])
    f = None
    a, _ = _lattice_pair(cfg, 40, f, tuning=dict(tile_w=tile_w, rows_per_thread=npt, persistent_wgs=pers,
                                                 overlap=ov))
    b, _ = _lattice_pair(cfg, 40, f)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("storage,tol", [(C.STORE_F32, 2e-8), (C.STORE_F16S, 3e-5)])
def test_reduced_forms_on_couette(storage, tol):
    """FP32 / FP16S storage of f - w_i with FP32 arithmetic: fields stay
    within the storage precision of the FP64 reference."""
    cfg = C.couette_config(100, 33)
    a, b = _lattice_pair(cfg, 300, storage=storage)
    assert np.abs(a - b).max() < tol


@pytest.mark.parametrize("storage,tol", [(C.STORE_F32, 1e-4), (C.STORE_F16S, 5e-2)])
def test_poiseuille_reduced(storage, tol):
    """Force-driven Poiseuille at u_max ~ 0.03 (the Mach range of the Couette
    workloads): relative error of the steady profile.  Each collision rounds
    the stored deviation d ~ w (3 e.u) ~ 1e-2 to its storage precision (2^-24
    in FP32, 2^-11 in FP16); the slowest viscous mode relaxes at nu k^2 ~ 4e-3
    per step (k = pi / 16), so the steady profile may sit ~ulp(d) / (nu k^2)
    away from the exact one: ~1e-5 (FP32) and ~3e-2 (FP16) of u_max."""
    ny, tau, g = 17, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    from paper_1606_01805_amd import Solver

    s = Solver([(C.base_config(8, ny, tau=tau, bc_y=1, body_force=[g, 0.0]), [])], storage=storage)
    s.step(20000, record=False)
    _, ux, _ = s.fields()
    y = np.arange(ny)
    exact = g / (2 * nu) * y * (ny - 1 - y)
    err = np.abs(ux - exact[:, None]).max() / exact.max()
    print(storage, err)
    assert err < tol


def test_set_get_populations_roundtrip():
    from paper_1606_01805_amd import Solver

    cfg = C.base_config(33, 20)
    f = _noisy(20, 33)
    for st, tol in ((C.STORE_F64, 0.0), (C.STORE_F32, 1e-8), (C.STORE_F16S, 2e-5)):
        s = Solver([(cfg, [])], storage=st)
        s.set_populations(f)
        assert np.abs(s.populations() - f).max() <= tol
        s.close()


def test_fields_match_oracle_definition():
    cfg = C.couette_config(50, 21, body_force=[1e-5, 0.0])
    cfg["bc_x"] = 0
    from paper_1606_01805_amd import Solver

    s = Solver([(cfg, [])])
    o = oracle.Oracle(cfg)
    s.step(30, record=False)
    o.step(30, record=False)
    for a, b in zip(s.fields(), o.fields()):
        assert np.array_equal(a, b)


F16S_SHAPES = [dict(tile_w=128, rows_per_thread=2), dict(tile_w=256, rows_per_thread=4),
               dict(tile_w=128, rows_per_thread=4, xcd_remap=1), dict(tile_w=256, rows_per_thread=2, persistent_wgs=5)]


def _f16s_run(channels, steps, tuning, f=None):
    from paper_1606_01805_amd import Solver

    s = Solver(channels, storage=C.STORE_F16S, tuning=tuning)
    if f is not None:
        s.set_populations(f)
    tr = s.step(steps)
    pops = [s.populations(k) for k in range(len(channels))]
    s.close()
    return tr, pops


@pytest.mark.parametrize("case", ["couette_ragged", "side_walls", "periodic_noisy", "tiny"])
def test_f16s_launch_shapes_bitwise(case):
    """F16S storage: tiles of width 128 and 256, more rows per thread, the
    XCD tile order and a persistent grid give bitwise the populations of
    64-wide tiles, with wrap, walls on either axis and ragged right edges."""
    f = None
    if case == "couette_ragged":
        cfg = C.couette_config(131, 37)                  # odd width, ragged against 128 and 256
    elif case == "side_walls":
        cfg = C.base_config(67, 40, tau=0.7, bc_x=1, body_force=[0.0, 2e-6],
                            u_wall=[[0.0, 0.01], [0.0, -0.02], [0, 0], [0, 0]])
    elif case == "periodic_noisy":
        cfg = C.base_config(258, 21, tau=0.9, body_force=[1e-5, -2e-6])
        f = _noisy(21, 258)
    else:
        cfg = C.base_config(3, 3, tau=0.9, body_force=[1e-5, -2e-6])
        f = _noisy(3, 3)
    _, ref = _f16s_run([(cfg, [])], 60, dict(tile_w=64, rows_per_thread=2), f)
    for tun in F16S_SHAPES:
        _, got = _f16s_run([(cfg, [])], 60, tun, f)
        assert np.array_equal(got[0], ref[0]), tun


def test_f16s_launch_shapes_with_particles_bitwise():
    """The same with force patches in the tiles: a particle crossing the
    periodic seam in a Couette channel, batched with a second channel."""
    from workloads import shapes

    c1 = C.couette_config(261, 64)
    p1 = C.particle(shapes.ellipse(20.0, 2.0, n_markers=50), 2.5, 30.0, 0.4)
    c2 = C.couette_config(140, 48)
    p2 = C.particle(shapes.circle(10.0, n_markers=32), 70.0, 20.0, 0.0)
    chans = [(c1, [p1]), (c2, [p2])]
    tr_ref, ref = _f16s_run(chans, 80, dict(tile_w=64, rows_per_thread=2))
    for tun in F16S_SHAPES:
        tr, got = _f16s_run(chans, 80, tun)
        assert np.array_equal(tr, tr_ref), tun
        for k in range(2):
            assert np.array_equal(got[k], ref[k]), (tun, k)


VEC_SHAPES = {C.STORE_F64: [(64, 1), (128, 1), (128, 2)],
              C.STORE_F32: [(128, 1), (256, 1), (256, 2)],
              C.STORE_F16S: [(256, 1), (512, 1), (512, 2), (128, 2)]}


@pytest.mark.parametrize("storage", [C.STORE_F64, C.STORE_F32, C.STORE_F16S])
@pytest.mark.parametrize("case", ["couette_ragged", "side_walls", "periodic_noisy", "box", "tiny", "wide"])
def test_vector_form_bitwise(storage, case):
    """The vector form of the lattice pass (vec = 1: tile_w / 64 nodes per
    lane, one chunk load per population plane, the x shift from the chunk and
    one extra element) gives bitwise the populations of the per-node form,
    with periodic wrap, walls on either axis, closed-box corners and ragged
    widths against every chunk size."""
    f = None
    if case == "couette_ragged":
        cfg = C.couette_config(131, 37)
    elif case == "side_walls":
        cfg = C.base_config(67, 40, tau=0.7, bc_x=1, body_force=[0.0, 2e-6],
                            u_wall=[[0.0, 0.01], [0.0, -0.02], [0, 0], [0, 0]])
    elif case == "periodic_noisy":
        cfg = C.base_config(70, 37, tau=0.9, body_force=[1e-5, -2e-6])
        f = _noisy(37, 70)
    elif case == "box":
        cfg = C.base_config(45, 30, tau=0.8, bc_x=1, bc_y=1)
        f = _bump(45, 30, cfg=cfg)
    elif case == "tiny":
        cfg = C.base_config(3, 3, tau=0.9)
        f = _noisy(3, 3)
    else:
        cfg = C.couette_config(1100, 9)  # several vector tiles per row, ragged at the end
    ref, _ = _lattice_pair(cfg, 30, f, storage=storage)
    for k, (tw, rows) in enumerate(VEC_SHAPES[storage]):
        got, _ = _lattice_pair(cfg, 30, f, storage=storage,
                               tuning=dict(vec=1, tile_w=tw, rows_per_thread=rows, xcd_remap=tw % 256 == 0,
                                           nt_store=k % 2))
        assert np.array_equal(got, ref), (tw, rows)


def test_vector_form_rejects_bad_shapes():
    from paper_1606_01805_amd import LBMError, Solver

    s = Solver([(C.couette_config(100, 20), [])], storage=C.STORE_F32)
    for bad in (dict(vec=1, tile_w=512), dict(vec=1, tile_w=256, rows_per_thread=4),
                dict(vec=1, tile_w=256, overlap=1, persistent_wgs=64),
                dict(vec=1, tile_w=256, rows_per_thread=2, overlap=1),
                dict(vec=2), dict(vec=0, nt_store=1), dict(adj_fused=3), dict(adj_fused=-1)):
        with pytest.raises(LBMError, match="EINVAL"):
            s.set_tuning(**bad)
    s.close()
