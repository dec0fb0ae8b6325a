"""Pins of the oracle's Zou-He walls (Sec. 1.1) and of the forced lattice
against the exact Couette and Poiseuille solutions."""
import math
import os

import numpy as np
import pytest

import oracle
from workloads import configs as C

RNG = np.random.default_rng(777)
UNKNOWN = {oracle.SIDE_YLO: (2, 5, 6), oracle.SIDE_YHI: (4, 7, 8),
           oracle.SIDE_XLO: (1, 5, 8), oracle.SIDE_XHI: (3, 6, 7)}
OPP = {1: 3, 2: 4, 3: 1, 4: 2}
NORMAL_IN = {oracle.SIDE_YLO: 2, oracle.SIDE_YHI: 4, oracle.SIDE_XLO: 1, oracle.SIDE_XHI: 3}


@pytest.mark.parametrize("side", [0, 1, 2, 3])
@pytest.mark.parametrize("with_force", [False, True])
def test_zouhe_moments(side, with_force):
    """After the reconstruction the node carries the wall velocity: the
    populations' momentum is rho u_w - g/2 and the unknowns alone were changed."""
    e, w = oracle.lattice()
    for _ in range(5):
        f = w * (1 + 0.1 * RNG.standard_normal(9))
        uw = 0.05 * RNG.standard_normal(2)
        g = 1e-3 * RNG.standard_normal(2) if with_force else np.zeros(2)
        f2 = oracle.zouhe(side, f, uw, g)
        known = [i for i in range(9) if i not in UNKNOWN[side]]
        assert np.array_equal(f2[known], f[known])
        rho = f2.sum()
        assert np.allclose(f2 @ e, rho * uw - 0.5 * g, atol=1e-16)


@pytest.mark.parametrize("side", [0, 1, 2, 3])
def test_zouhe_normal_nonequilibrium_bounce_back(side):
    """The wall-normal unknown bounces back the non-equilibrium part of its
    opposite: f_in - f_in^eq = f_out - f_out^eq (Zou and He)."""
    _, w = oracle.lattice()
    f = w * (1 + 0.1 * RNG.standard_normal(9))
    uw = np.array([0.04, -0.01])
    f2 = oracle.zouhe(side, f, uw)
    rho = f2.sum()
    feq = oracle.equilibrium(rho, uw[0], uw[1])
    i = NORMAL_IN[side]
    assert math.isclose(f2[i] - feq[i], f2[OPP[i]] - feq[OPP[i]], abs_tol=1e-16)


def test_couette_linear_profile_is_exact():
    """Moving walls at -U and +U: LBGK with on-node Zou-He walls holds the
    linear Couette profile (an exact discrete solution)."""
    ny = 17
    cfg = C.couette_config(4, ny, tau=1.0)
    cfg["init"] = oracle.INIT_REST  # start from rest; converge to the profile
    o = oracle.Oracle(cfg)
    o.step(20000, record=False)
    r, ux, uy = o.fields()
    U = cfg["u_wall"][3][0]
    exact = -U + 2 * U * np.arange(ny) / (ny - 1)
    assert np.abs(ux - exact[:, None]).max() <= 1e-10 * U
    assert np.abs(uy).max() <= 1e-12 * U


def test_couette_start_is_steady():
    """Initialised on the Couette profile the channel stays there."""
    cfg = C.couette_config(6, 21, tau=0.9)
    o = oracle.Oracle(cfg)
    r0, u0, _ = o.fields()
    o.step(200, record=False)
    r1, u1, _ = o.fields()
    assert np.abs(u1 - u0).max() < 1e-15 and np.abs(r1 - 1).max() < 1e-14


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_force_driven_poiseuille(tau):
    """Uniform body force g between resting walls: u(y) = g/(2 nu) y (H - y),
    H = NY - 1 (walls on the first and last rows), nu = (tau - 1/2)/3."""
    ny = 17
    nu = (tau - 0.5) / 3
    g = 1e-6
    o = oracle.Oracle(C.base_config(4, ny, tau=tau, bc_y=oracle.ZOUHE, body_force=[g, 0.0]))
    o.step(40000, record=False)
    _, ux, uy = o.fields()
    y = np.arange(ny)
    exact = g / (2 * nu) * y * (ny - 1 - y)
    assert np.abs(ux - exact[:, None]).max() <= 1e-9 * exact.max()
    assert np.abs(uy).max() <= 1e-14  # rounding level


def test_side_walls_poiseuille_along_y():
    """Same closed form with the walls on the x sides and the force along y."""
    nx = 13
    tau, g = 0.9, 2e-6
    nu = (tau - 0.5) / 3
    o = oracle.Oracle(C.base_config(nx, 4, tau=tau, bc_x=oracle.ZOUHE, body_force=[0.0, g]))
    o.step(30000, record=False)
    _, ux, uy = o.fields()
    x = np.arange(nx)
    exact = g / (2 * nu) * x * (nx - 1 - x)
    assert np.abs(uy - exact[None, :]).max() <= 1e-8 * exact.max()


def test_couette_mass_drift_small():
    """Zou-He walls are not exactly conservative: the 400 x 100 Couette
    channel with its ellipse keeps its mass to 1e-6 over 5000 steps."""
    wl = C.couette(storage=0)
    cfg, parts = wl.channels[0]
    o = oracle.Oracle(cfg)
    o.set_threads(os.cpu_count() or 1)
    o.add_particle(parts[0])
    m0 = o.populations().sum()
    o.step(5000, record=False)
    assert abs(o.populations().sum() / m0 - 1) < 1e-6


def _box_with_bump(nx, ny, tau=0.8, amp=0.01):
    """A closed box (Zou-He walls at rest on both axes, reading R23) holding
    a density bump that is mirror symmetric in x and in y."""
    o = oracle.Oracle(C.base_config(nx, ny, tau=tau, bc_x=oracle.ZOUHE, bc_y=oracle.ZOUHE))
    f = np.zeros((9, ny, nx))
    for y in range(ny):
        for x in range(nx):
            dx, dy = x - (nx - 1) / 2, y - (ny - 1) / 2
            f[:, y, x] = oracle.equilibrium(1.0 + amp * math.exp(-(dx * dx + dy * dy) / 8.0), 0.0, 0.0)
    o.set_populations(f)
    return o


def test_closed_box_corners_take_the_neighbour_density_at_rest():
    """Reading R23: each corner node carries the density of its diagonal
    interior neighbour and no momentum (walls at rest), and its three
    populations that point into the fluid are the bounce-back of their
    opposites."""
    nx, ny = 14, 11
    o = _box_with_bump(nx, ny)
    o.step(37, record=False)
    f = o.populations()
    e, _ = oracle.lattice()
    for (x, y, sx, sy) in ((0, 0, 1, 1), (nx - 1, 0, -1, 1), (0, ny - 1, 1, -1), (nx - 1, ny - 1, -1, -1)):
        fc = f[:, y, x]
        assert math.isclose(fc.sum(), f[:, y + sy, x + sx].sum(), rel_tol=0, abs_tol=4e-16)
        assert np.abs(fc @ e).max() < 4e-17
        for i in range(1, 9):
            if e[i][0] in (0, sx) and e[i][1] in (0, sy):  # points into the fluid
                j = [k for k in range(9) if (e[k] == -e[i]).all()][0]
                assert fc[i] == fc[j]


def test_closed_box_keeps_both_mirror_symmetries():
    """A bump that is symmetric under x -> nx-1-x and y -> ny-1-y stays so: the
    four corner closures and the four walls are each other's mirror images.
    A wrong index in one corner's closure breaks this."""
    nx, ny = 15, 12
    o = _box_with_bump(nx, ny)
    o.step(300, record=False)
    f = o.populations()
    mx = [0, 3, 2, 1, 4, 6, 5, 8, 7]  # mirror x: e_x -> -e_x
    my = [0, 1, 4, 3, 2, 8, 7, 6, 5]  # mirror y: e_y -> -e_y
    dev = f - oracle.lattice()[1][:, None, None]
    scale = np.abs(dev).max()
    assert np.abs(dev - dev[mx][:, :, ::-1]).max() < 1e-12 * scale
    assert np.abs(dev - dev[my][:, ::-1, :]).max() < 1e-12 * scale
    # the bump spreads: it is not trivially static
    assert scale > 1e-4


def test_closed_box_mass_settles():
    """Zou-He walls fix velocities, not mass: while the bump's pressure waves
    reach the walls the box's mass changes by a fraction of the bump's excess
    mass, and once the flow is at rest it stays constant."""
    o = _box_with_bump(20, 16)
    m0 = o.populations().sum()
    excess = m0 - 20 * 16
    o.step(1500, record=False)
    m1 = o.populations().sum()
    o.step(1500, record=False)
    m2 = o.populations().sum()
    assert abs(m1 - m0) < 0.2 * excess
    assert abs(m2 / m1 - 1) < 1e-12


def test_closed_box_rejects_moving_walls_and_body_force():
    base = dict(bc_x=oracle.ZOUHE, bc_y=oracle.ZOUHE)
    with pytest.raises(ValueError):
        oracle.Oracle(C.base_config(10, 10, u_wall=[[0, 0], [0, 0], [0.01, 0], [0, 0]], **base))
    with pytest.raises(ValueError):
        oracle.Oracle(C.base_config(10, 10, body_force=[1e-6, 0.0], **base))
