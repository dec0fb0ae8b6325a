"""Pins of the oracle's surface-stress force and moment (Sec. 1.3, Eqs. (13),
(14)) on synthetic level-n fields with closed-form answers."""
import math

import numpy as np
import pytest
import torch

import oracle
from workloads import configs as C
from workloads import shapes

NX, NY = 64, 64
X0, Y0 = 31.37, 32.21
DN = 1.2
TAU = 0.8
NU = (TAU - 0.5) / 3


def _cfg():
    return C.base_config(NX, NY, tau=TAU)


def _fields(rho_fun, u_fun):
    y, x = np.mgrid[0:NY, 0:NX].astype(float)
    rho = rho_fun(x, y) * np.ones((NY, NX))
    ux, uy = u_fun(x, y)
    return rho, ux * np.ones((NY, NX)), uy * np.ones((NY, NX))


def _body(shape, theta=0.0, omega=0.0):
    return C.particle(shape, X0, Y0, theta, omega=omega)


def _segment(length, normal, offset, n=8):
    """An open marker set along one straight face (any marker set is allowed)."""
    nrm = np.asarray(normal, float)
    t = np.array([-nrm[1], nrm[0]])
    s = (np.arange(n) + 0.5) / n * length - length / 2
    xi = offset[None, :] + s[:, None] * t[None, :]
    return dict(xi=torch.tensor(xi), nrm=torch.tensor(np.tile(nrm, (n, 1))),
                ds=torch.full((n,), length / n, dtype=torch.float64), area=1.0, polar_moment=1.0)


@pytest.mark.parametrize("fam", ["square", "triangle", "rectangle", "circle"])
def test_uniform_pressure_gives_no_load(fam):
    rho, ux, uy = _fields(lambda x, y: 1.03, lambda x, y: (0.0, 0.0))
    sh = shapes.make(fam, 14.0, aspect_ratio=3.0)
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(sh, 0.4))
    assert np.abs(F).max() < 1e-14


def test_pressure_gauge_on_one_face():
    """p = c_s^2 (rho - rho0): rho = 1.3 gives p = 0.1, load -p n L on a face."""
    rho, ux, uy = _fields(lambda x, y: 1.3, lambda x, y: (0.0, 0.0))
    seg = _segment(6.0, (0.0, 1.0), np.array([0.0, 4.0]))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(seg))
    assert np.allclose(F[:2], [0.0, -0.1 * 6.0], atol=1e-14)


@pytest.mark.parametrize("theta", [0.0, 0.37])
def test_linear_pressure_on_square(theta):
    """p = G . (x - X): the probe pressure adds dn G.n, so
    F = -G A - dn (sum n n^T S) G = -G (L^2 + 2 dn L) for a square, M = 0."""
    G = np.array([2e-4, -1e-4])
    L = 12.0
    rho, ux, uy = _fields(lambda x, y: 1 + 3 * (G[0] * (x - X0) + G[1] * (y - Y0)),
                          lambda x, y: (0.0, 0.0))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(shapes.square(L), theta))
    assert np.allclose(F[:2], -G * (L * L + 2 * DN * L), rtol=1e-11, atol=1e-16)
    assert abs(F[2]) < 1e-13


def test_linear_pressure_on_triangle():
    """Equilateral triangle: sum n n^T S = (3L/2) I, area sqrt(3)/4 L^2."""
    G = np.array([-1e-4, 3e-4])
    L = 15.0
    rho, ux, uy = _fields(lambda x, y: 1 + 3 * (G[0] * (x - X0) + G[1] * (y - Y0)),
                          lambda x, y: (0.0, 0.0))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(shapes.triangle(L), 0.2))
    A = math.sqrt(3) / 4 * L * L
    assert np.allclose(F[:2], -G * (A + DN * 1.5 * L), rtol=1e-11)
    assert abs(F[2]) < 1e-13


def test_acceleration_correction_of_marker_pressure():
    """Fluid at rest, lagged acceleration a: p_l = dn a.n_l so F = -dn (sum n n^T S) a."""
    rho, ux, uy = _fields(lambda x, y: 1.0, lambda x, y: (0.0, 0.0))
    a = np.array([3e-5, -2e-5])
    L = 10.0
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(shapes.square(L)), (a[0], a[1], 0.0))
    assert np.allclose(F[:2], -DN * 2 * L * a, rtol=1e-12)


def test_angular_acceleration_correction():
    """Fluid at rest, angular acceleration alpha on a square of edge L with
    markers at the centres of h-long sub-segments: p_l = dn alpha (r_l x n_l),
    M = -dn alpha sum (r x n)^2 S = -4 dn alpha (L^3/12 - L h^2/12)."""
    rho, ux, uy = _fields(lambda x, y: 1.0, lambda x, y: (0.0, 0.0))
    L, h, alpha = 12.0, 1.0, 4e-6
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(shapes.square(L, spacing=h)), (0, 0, alpha))
    expect = -4 * DN * alpha * (L ** 3 / 12 - L * h * h / 12)
    assert math.isclose(F[2], expect, rel_tol=1e-11)
    assert np.abs(F[:2]).max() < 1e-14  # rounding of sum phi_k - 1 at the probes


def test_centripetal_term_on_square():
    """Rotation Omega: a_l = -Omega^2 r_l, r.n = L/2 on every face: uniform
    marker pressure, no net load."""
    rho, ux, uy = _fields(lambda x, y: 1.0, lambda x, y: (0.0, 0.0))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(shapes.square(10.0), omega=0.01))
    scale = DN * 0.01 ** 2 * 5.0 * 40.0  # |p_l| times the perimeter
    assert np.abs(F[:2]).max() < 1e-12 * scale and abs(F[2]) < 1e-12 * scale * 5.0


def test_simple_shear_traction_on_faces():
    """u = (gamma (y - Y), 0): tau_xy = nu gamma.  A face with n = (0, 1)
    feels (nu gamma L, 0); a face with n = (1, 0) feels (0, nu gamma L)."""
    gam = 1e-3
    rho, ux, uy = _fields(lambda x, y: 1.0, lambda x, y: (gam * (y - Y0), 0.0 * x))
    L = 7.0
    top = _segment(L, (0.0, 1.0), np.array([0.0, 5.0]))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(top))
    assert np.allclose(F[:2], [NU * gam * L, 0.0], rtol=1e-11, atol=1e-12 * NU * gam * L)
    assert math.isclose(F[2], -5.0 * NU * gam * L, rel_tol=1e-11)
    right = _segment(L, (1.0, 0.0), np.array([5.0, 0.0]))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(right))
    assert np.allclose(F[:2], [0.0, NU * gam * L], rtol=1e-11, atol=1e-12 * NU * gam * L)
    assert math.isclose(F[2], 5.0 * NU * gam * L, rel_tol=1e-11)


def test_extensional_normal_stress_factor_two():
    """u = (eps x, -eps y): tau_yy = -2 nu eps on a face with n = (0, 1)."""
    eps = 2e-4
    rho, ux, uy = _fields(lambda x, y: 1.0, lambda x, y: (eps * (x - X0), -eps * (y - Y0)))
    L = 6.0
    top = _segment(L, (0.0, 1.0), np.array([0.0, 4.0]))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(top))
    assert np.allclose(F[:2], [0.0, -2 * NU * eps * L], rtol=1e-11, atol=1e-12 * NU * eps * L)


@pytest.mark.parametrize("fam", ["square", "triangle", "rectangle"])
def test_uniform_viscous_stress_gives_no_load_on_closed_polygons(fam):
    """Constant symmetric stress on a closed polygon: F = 0 and M = 0 (the
    midpoint rule is exact on straight faces)."""
    gam, eps = 1e-3, 3e-4
    rho, ux, uy = _fields(lambda x, y: 1.0,
                          lambda x, y: (gam * (y - Y0) + eps * (x - X0), -eps * (y - Y0)))
    sh = shapes.make(fam, 14.0, aspect_ratio=2.5)
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(sh, 0.3))
    scale = NU * gam * 14.0  # one face's load; the moment scale is that times 14
    assert np.abs(F[:2]).max() < 1e-11 * scale and abs(F[2]) < 1e-11 * scale * 14.0
    # a non-symmetric stress (nu grad u, no transpose) would leave a moment
    # -nu gamma A; the symmetric one leaves none


def test_rigid_rotation_field_has_no_viscous_load():
    Om = 2e-3
    rho, ux, uy = _fields(lambda x, y: 1.0, lambda x, y: (-Om * (y - Y0), Om * (x - X0)))
    F = oracle.surface_force(_cfg(), rho, ux, uy, _body(shapes.triangle(12.0)))
    scale = NU * Om * 12.0
    assert np.abs(F[:2]).max() < 1e-11 * scale and abs(F[2]) < 1e-11 * scale * 12.0
