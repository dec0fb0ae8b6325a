"""Pins of the oracle's Zou-He walls (Sec. 1.1) and of the forced lattice
against the exact Couette and Poiseuille solutions."""
import math

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
    wl = C.couette(storage=0)
    cfg, parts = wl.channels[0]
    o = oracle.Oracle(cfg)
    o.add_particle(parts[0])
    m0 = o.populations().sum()
    o.step(300, record=False)
    assert abs(o.populations().sum() / m0 - 1) < 1e-6
