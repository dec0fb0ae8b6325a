"""Pins of the oracle's rigid-body update (Sec. 1.3, Eqs. (15), (16)) and of
whole-step invariants of the coupled method."""
import math
import os

import numpy as np
import pytest

import oracle
from workloads import configs as C
from workloads import shapes


def test_bdf2_constant_acceleration_closed_form():
    """From rest with history equal to the initial state:
    V^n = a (n - (1 - 3^-n)/2)."""
    a = 1.7e-3
    v = vm = 0.0
    x = xm = 0.0
    for n in range(1, 40):
        vn, xn = oracle.bdf2(v, vm, a, x, xm)
        assert math.isclose(vn, a * (n - 0.5 * (1 - 3.0 ** (-n))), rel_tol=1e-13)
        vm, v, xm, x = v, vn, x, xn


def test_bdf2_constant_velocity_position_closed_form():
    """Constant V0 and history X^-1 = X^0: X^n = X0 + V0 (n - (1 - 3^-n)/2)."""
    V0, X0 = 0.013, 5.0
    x = xm = X0
    for n in range(1, 40):
        vn, xn = oracle.bdf2(V0, V0, 0.0, x, xm)
        assert vn == V0
        assert math.isclose(xn, X0 + V0 * (n - 0.5 * (1 - 3.0 ** (-n))), rel_tol=1e-14)
        xm, x = x, xn


def test_particle_at_rest_in_fluid_at_rest_stays():
    o = oracle.Oracle(C.base_config(40, 40))
    o.add_particle(C.particle(shapes.triangle(10.0), 20.3, 19.6, 0.4, 1.2))
    tr = o.step(20)
    # the rest state f = w_i carries rounding of sum w_i - 1 only
    assert np.abs(tr[:, 0, 3:9]).max() < 1e-15


def test_first_step_is_buoyant_free_fall():
    """Fluid and particle at rest: F^0 = 0, so V^1 = (2/3)(1 - 1/ratio) g
    (BDF2 start-up with the buoyancy-reduced gravity on the particle only)."""
    g = np.array([0.0, -1e-5])
    ratio = 1.25
    o = oracle.Oracle(C.base_config(40, 60, tau=0.8, bc_x=oracle.ZOUHE, gravity=list(g)))
    o.add_particle(C.particle(shapes.circle(8.0, n_markers=28), 20.0, 30.0, 0.0, ratio))
    tr = o.step(1)
    assert np.abs(tr[0, 0, 6:9]).max() < 1e-15  # rounding of sum w_i - 1 only
    assert np.allclose(tr[0, 0, 3:5], 2 / 3 * (1 - 1 / ratio) * g, rtol=1e-9, atol=1e-17)
    assert np.allclose(tr[0, 0, 0:2], [20.0, 30.0 + 2 / 3 * tr[0, 0, 4]], rtol=1e-15, atol=1e-16)


def test_sedimentation_reaches_force_balance():
    """Terminal settling: as dV/dt -> 0 the hydrodynamic force balances the
    buoyancy-reduced weight, F_y -> (rho_s - rho_f) A |g|."""
    nx, ny, D, ratio, g = 32, 64, 6.0, 2.0, 2e-5
    o = oracle.Oracle(C.base_config(nx, ny, tau=1.0, bc_x=oracle.ZOUHE, gravity=[0.0, -g]))
    sh = shapes.circle(D, n_markers=20)
    xc = (nx - 1) / 2  # walls on columns 0 and nx - 1
    # turned by half a marker spacing: the set stays mirror-symmetric about
    # x = xc and no marker or probe sits on a round-half-up tie
    o.add_particle(C.particle(sh, xc, ny / 2, math.pi / 20, ratio))
    tr = o.step(4000)
    target = (ratio - 1) * float(sh["area"]) * g
    assert abs(tr[-1, 0, 7] / target - 1) < 2e-3
    dv = abs(tr[-1, 0, 4] - tr[-2, 0, 4])
    assert dv < 1e-3 * (1 - 1 / ratio) * g
    assert tr[-1, 0, 4] < 0  # it falls
    assert abs(tr[-1, 0, 0] - xc) < 1e-9  # and stays on the centre line


def test_centred_circle_in_couette_has_no_lift():
    """A circle at the centre of a -U/+U Couette channel: the problem is
    point-symmetric about the centre, so the lateral force vanishes and the
    particle spins against the shear."""
    nx, ny = 60, 41
    cfg = C.couette_config(nx, ny, tau=1.0)
    o = oracle.Oracle(cfg)
    o.add_particle(C.particle(shapes.circle(10.0, n_markers=32), 30.0, 20.0))
    o.set_threads(os.cpu_count() or 1)
    tr = o.step(5000)
    assert np.abs(tr[:, 0, 1] - 20.0).max() < 1e-9
    assert np.abs(tr[:, 0, 0] - 30.0).max() < 1e-9
    U = cfg["u_wall"][3][0]
    shear = 2 * U / (ny - 1)
    assert -0.6 * shear < tr[-1, 0, 5] < -0.3 * shear  # near the fluid's -gamma/2


def test_determinism():
    wl = C.couette(storage=0)
    cfg, parts = wl.channels[0]
    a, b = oracle.Oracle(cfg), oracle.Oracle(cfg)
    a.add_particle(parts[0])
    b.add_particle(parts[0])
    assert np.array_equal(a.step(30), b.step(30))


def test_unstable_configuration_is_reported():
    """Weak coupling is not stable for large velocity jumps (Sec. 1.3): a
    particle launched at 5 lattice units per step blows up, and the oracle
    reports the step."""
    o = oracle.Oracle(C.base_config(40, 24, tau=0.51, bc_y=oracle.ZOUHE))
    o.add_particle(C.particle(shapes.circle(6.0, n_markers=20), 20.0, 12.0, 0.0, 1.0, u=5.0))
    with pytest.raises(FloatingPointError, match="step 2"):
        o.step(100, record=False)
