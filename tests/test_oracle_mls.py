"""Pins of the oracle's MLS transfer operator and immersed-boundary coupling
(Sec. 1.2, Eqs. (8)-(12)) against reproduction properties, special cases and
adjointness, none of which the oracle computes itself."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads import configs as C
from workloads import shapes

RNG = np.random.default_rng(2024)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _coords(nodes_unwrapped):
    return nodes_unwrapped


def _unwrapped_nodes(x, y):
    i0, j0 = math.floor(x + 0.5), math.floor(y + 0.5)
    return np.array([(i0 + a, j0 + b) for b in (-1, 0, 1) for a in (-1, 0, 1)], dtype=float)


@pytest.mark.parametrize("trial", range(20))
def test_partition_of_unity_and_linear_reproduction(trial):
    cfg = C.base_config(64, 48)
    x, y = RNG.uniform(5, 59), RNG.uniform(5, 43)
    nodes, ok, phi, dx, dy = oracle.mls(cfg, x, y)
    assert ok.all()
    xk = _unwrapped_nodes(x, y)
    assert math.isclose(phi.sum(), 1.0, abs_tol=1e-14)
    assert np.allclose(phi @ xk, [x, y], atol=1e-13)
    # derivative weights reproduce the gradient of constants and linear fields
    assert abs(dx.sum()) < 1e-13 and abs(dy.sum()) < 1e-13
    assert np.allclose(dx @ xk, [1.0, 0.0], atol=1e-13)
    assert np.allclose(dy @ xk, [0.0, 1.0], atol=1e-13)
    # a linear field is reproduced exactly at the point (Eq. (8))
    a, b, c = RNG.standard_normal(3)
    u = a + b * xk[:, 0] + c * xk[:, 1]
    assert math.isclose(phi @ u, a + b * x + c * y, rel_tol=1e-12, abs_tol=1e-12)
    assert math.isclose(dx @ u, b, rel_tol=1e-11, abs_tol=1e-12)


def test_node_centred_values_match_golden():
    """Marker exactly on a node: A is diagonal and phi_k = W_k / sum W
    (Eq. (10) with alpha = 0.3, r_w = 2.6)."""
    g = json.load(open(os.path.join(GOLDEN, "mls_node_centred.json")))
    cfg = C.base_config(20, 20)
    _, ok, phi, dx, dy = oracle.mls(cfg, 10.0, 7.0)
    assert math.isclose(phi[4], g["centre"], rel_tol=0, abs_tol=5e-7)
    for k in (1, 3, 5, 7):
        assert math.isclose(phi[k], g["edge"], abs_tol=5e-7)
    for k in (0, 2, 6, 8):
        assert math.isclose(phi[k], g["corner"], abs_tol=5e-7)
    # symmetric stencil: the derivative weights are odd
    assert abs(dx[4]) < 1e-15 and math.isclose(dx[5], -dx[3], rel_tol=1e-14)


def test_kernel_special_values():
    """Eq. (10): W(0) = 1, W(alpha) = 1/e, W(r > 1) = 0, decreasing."""
    assert oracle.kernel_weight(oracle.W_EXP, 0.0) == 1.0
    assert math.isclose(oracle.kernel_weight(oracle.W_EXP, 0.3), math.exp(-1.0), rel_tol=1e-15)
    assert oracle.kernel_weight(oracle.W_EXP, 1.0001) == 0.0
    r = np.linspace(0, 1, 50)
    w = [oracle.kernel_weight(oracle.W_EXP, v) for v in r]
    assert np.all(np.diff(w) < 0)
    # cubic / quartic / cosine kernels (Eqs. (17)-(19)) at r = 0 and r = 1
    assert math.isclose(oracle.kernel_weight(oracle.W_CUBIC, 0.0), 2 / 3)
    assert math.isclose(oracle.kernel_weight(oracle.W_CUBIC, 1.0), 2 / 3, abs_tol=1e-15)
    assert oracle.kernel_weight(oracle.W_QUARTIC, 0.0) == 1.0
    assert abs(oracle.kernel_weight(oracle.W_QUARTIC, 1.0)) < 1e-15
    assert oracle.kernel_weight(oracle.W_COSINE, 0.0) == 0.5


def test_wall_drops_nodes_and_keeps_reproduction():
    cfg = C.base_config(40, 30, bc_y=oracle.ZOUHE)
    x, y = 12.3, 0.2  # anchor row 0: the row below is beyond the wall
    nodes, ok, phi, dx, dy = oracle.mls(cfg, x, y)
    assert ok.sum() == 6 and not ok[:3].any()
    xk = _unwrapped_nodes(x, y)
    assert math.isclose(phi.sum(), 1.0, abs_tol=1e-14)
    assert np.allclose(phi[ok] @ xk[ok], [x, y], atol=1e-13)
    assert np.all(phi[~ok] == 0)


def test_periodic_wrap_is_translation_invariant():
    cfg = C.base_config(40, 30)
    n1, ok1, p1, _, _ = oracle.mls(cfg, 0.3, 11.7)
    n2, ok2, p2, _, _ = oracle.mls(cfg, 40.3, 11.7)
    assert np.array_equal(n1, n2) and ok1.all() and ok2.all()
    assert np.allclose(p1, p2, atol=1e-14)
    assert (n1[:, 0] == 39).sum() == 3  # the column left of x = 0 wraps to 39


def _uniform_state(o, nx, ny, fun):
    f = np.zeros((9, ny, nx))
    for y in range(ny):
        for x in range(nx):
            r, ux, uy = fun(x, y)
            f[:, y, x] = oracle.equilibrium(r, ux, uy)
    o.set_populations(f)


def test_uniform_flow_matching_particle_gives_zero_force():
    """Fluid moving uniformly with the particle: U_l = U_b (linear reproduction)
    so every Lagrangian force, and the spread force, vanishes."""
    nx, ny = 48, 40
    o = oracle.Oracle(C.base_config(nx, ny))
    u0 = (0.02, -0.013)
    _uniform_state(o, nx, ny, lambda x, y: (1.0, *u0))
    sh = shapes.ellipse(12.0, 2.0, n_markers=40)
    o.add_particle(C.particle(sh, 23.4, 19.1, 0.3, u=u0[0], v=u0[1]))
    o.step(1)
    rec = o.marker_record(0)
    assert np.abs(rec[:, 6:8]).max() < 1e-15
    fx, fy = o.last_force()
    assert np.abs(fx).max() < 1e-15 and np.abs(fy).max() < 1e-15


def test_rigid_rotation_matching_particle_gives_zero_force():
    nx, ny = 48, 40
    o = oracle.Oracle(C.base_config(nx, ny))
    X, Y, Om = 23.7, 20.2, 0.004
    _uniform_state(o, nx, ny, lambda x, y: (1.0, -Om * (y - Y), Om * (x - X)))
    sh = shapes.circle(10.0, n_markers=32)
    o.add_particle(C.particle(sh, X, Y, 0.0, omega=Om))
    o.step(1)
    rec = o.marker_record(0)
    assert np.abs(rec[:, 6:8]).max() < 1e-16 * 1e3


def test_spread_conserves_force_and_is_transpose_of_interpolation():
    """Eq. (12) with c_l = S_l: sum_k f_lb(x_k) = sum_l S_l F_l (partition of
    unity), and <I u, c F> = <u, S F> (interpolation and spreading are
    transposes)."""
    nx, ny = 60, 50
    cfg = C.base_config(nx, ny)
    o = oracle.Oracle(cfg)
    _uniform_state(o, nx, ny, lambda x, y: (1.0 + 0.01 * math.sin(0.3 * x),
                                            0.02 * math.sin(0.2 * y + 0.1 * x), 0.01 * math.cos(0.15 * x)))
    r0, ux0, uy0 = o.fields()
    sh = shapes.make("triangle", 16.0)
    o.add_particle(C.particle(sh, 30.3, 24.8, 0.7, u=0.01, omega=0.002))
    o.step(1)
    rec = o.marker_record(0)
    ds = sh["ds"].numpy()
    F = rec[:, 6:8]
    U = rec[:, 4:6]
    fx, fy = o.last_force()
    tot = np.array([fx.sum(), fy.sum()])
    assert np.allclose(tot, (ds[:, None] * F).sum(0), rtol=1e-13, atol=1e-17)
    lhs = (ds[:, None] * F * U).sum()
    rhs = (fx * ux0).sum() + (fy * uy0).sum()
    assert math.isclose(lhs, rhs, rel_tol=1e-12)


def test_unit_spread_scale_reading():
    nx, ny = 40, 40
    cfg = C.base_config(nx, ny, spread_scale=1)
    o = oracle.Oracle(cfg)
    sh = shapes.circle(8.0, n_markers=20)
    o.add_particle(C.particle(sh, 20.2, 19.6, 0.0, u=0.01))
    o.step(1)
    F = o.marker_record(0)[:, 6:8]
    fx, fy = o.last_force()
    assert np.allclose([fx.sum(), fy.sum()], F.sum(0), rtol=1e-13)


def test_cosine_kernel_interior_values():
    """Eq. (19) away from r = 0: W = (1 + cos(pi r / 2)) / 4 takes the closed
    forms 3/8 at r = 2/3, (2 + sqrt 2)/8 at r = 1/2 and 1/4 at r = 1; a slip
    in the argument scale (cos(pi r) for cos(pi r / 2)) fails every one."""
    W = lambda r: oracle.kernel_weight(oracle.W_COSINE, r)  # noqa: E731
    assert math.isclose(W(2.0 / 3.0), 0.375, rel_tol=0, abs_tol=2e-16)
    assert math.isclose(W(0.5), (2.0 + math.sqrt(2.0)) / 8.0, rel_tol=0, abs_tol=2e-16)
    assert math.isclose(W(1.0), 0.25, rel_tol=0, abs_tol=2e-16)
    assert W(1.0 + 1e-12) == 0.0


def _peskin_sums(W, q):
    """For the polynomial kernel read as phi(q) = W(q / 2) (reading R14):
    the four lattice-point values around a point at offset q in [0, 1] and
    their even / odd sums."""
    v = [W(q / 2.0), W((1.0 - q) / 2.0), W((1.0 + q) / 2.0), W((2.0 - q) / 2.0)]
    return sum(v), v[0] + v[3], v[1] + v[2]


def test_polynomial_kernel_reading():
    """Eq. (20) under reading R14 (the branches evaluated at q = 2 r): W(0) =
    1/2, both branches give 1/4 at r = 1/2, W(1) = 0.  The function is the
    four-point delta function, so at every offset its four lattice values sum
    to 1 and the even and odd pairs to 1/2 each; a wrong sign, coefficient or
    branch point in either branch breaks these sums."""
    W = lambda r: oracle.kernel_weight(oracle.W_POLY, r)  # noqa: E731
    assert W(0.0) == 0.5
    assert W(0.5) == 0.25
    assert math.isclose(W(0.5 + 1e-13), 0.25, abs_tol=1e-12)
    assert math.isclose(W(1.0), 0.0, abs_tol=1e-16)
    assert W(1.0 + 1e-12) == 0.0
    for q in np.linspace(0.0, 1.0, 41):
        tot, even, odd = _peskin_sums(W, q)
        assert math.isclose(tot, 1.0, abs_tol=2e-15), q
        assert math.isclose(even, 0.5, abs_tol=2e-15), q
        assert math.isclose(odd, 0.5, abs_tol=2e-15), q
    r = np.linspace(0, 1, 60)
    assert np.all(np.diff([W(v) for v in r]) < 0)


@pytest.mark.parametrize("kernel", [1, 2, 3, 4])
def test_alternative_kernels_reproduce_linear_fields(kernel):
    """Every kernel of Sec. 2.2 gives an MLS operator with partition of unity
    and linear reproduction (Eqs. (8), (9))."""
    cfg = C.base_config(64, 48, mls_kernel=kernel)
    rng = np.random.default_rng(100 + kernel)
    for _ in range(5):
        x, y = rng.uniform(5, 59), rng.uniform(5, 43)
        _, ok, phi, dx, dy = oracle.mls(cfg, x, y)
        xk = _unwrapped_nodes(x, y)
        assert ok.all() and np.all(phi[[4]] > 0)
        assert math.isclose(phi.sum(), 1.0, abs_tol=1e-14)
        assert np.allclose(phi @ xk, [x, y], atol=1e-13)
        assert np.allclose(dx @ xk, [1.0, 0.0], atol=1e-12)
        assert np.allclose(dy @ xk, [0.0, 1.0], atol=1e-12)


def _spread_alone(cfg, state, parts):
    nx, ny = cfg["nx"], cfg["ny"]
    o = oracle.Oracle(cfg)
    _uniform_state(o, nx, ny, state)
    for p in parts:
        o.add_particle(p)
    o.step(1)
    return o.last_force()


def test_spread_order_adds_particle_sums():
    """Reading R20 (Eq. (12) fixes no order): each particle's terms at a node
    are summed on their own and the particle sums are added in ascending
    particle order.  Two particles whose stencils share nodes therefore give
    exactly (bitwise) the sum of their spreads alone; summing the second
    particle's terms onto the first's running sum would not."""
    nx, ny = 70, 50
    cfg = C.base_config(nx, ny)
    state = lambda x, y: (1.0 + 0.01 * math.sin(0.3 * x), 0.02 * math.sin(0.2 * y), 0.01 * math.cos(0.15 * x))  # noqa: E731
    a = C.particle(shapes.circle(10.0, n_markers=32), 30.2, 25.1, 0.0, u=0.013)
    b = C.particle(shapes.square(9.0), 39.7, 26.4, 0.3, v=-0.011, omega=0.003)
    fa = _spread_alone(cfg, state, [a])
    fb = _spread_alone(cfg, state, [b])
    fab = _spread_alone(cfg, state, [a, b])
    shared = (fa[0] != 0) & (fb[0] != 0)
    assert shared.sum() > 5
    for k in range(2):
        assert np.array_equal(fab[k], fa[k] + fb[k])


def test_spread_order_adds_round_sums():
    """Reading R20: a particle of more than 64 markers sums each round of 64
    consecutive markers on its own and adds the round sums in order, so its
    spread is exactly the sum of the spreads of two particles made of its
    first and its last 64 markers."""
    nx, ny = 70, 60
    cfg = C.base_config(nx, ny)
    state = lambda x, y: (1.0, 0.02 * math.sin(0.2 * y + 0.1 * x), 0.01 * math.cos(0.15 * x))  # noqa: E731
    p = C.particle(shapes.circle(16.0, n_markers=128), 34.6, 29.3, 0.2, u=0.01, omega=0.002)
    halves = []
    for lo in (0, 64):
        q = dict(p)
        for key in ("xi", "nrm", "ds"):
            q[key] = np.asarray(p[key])[lo:lo + 64].copy()
        halves.append(q)
    f1 = _spread_alone(cfg, state, [halves[0]])
    f2 = _spread_alone(cfg, state, [halves[1]])
    f = _spread_alone(cfg, state, [p])
    assert ((f1[0] != 0) & (f2[0] != 0)).sum() > 5
    for k in range(2):
        assert np.array_equal(f[k], f1[k] + f2[k])
