"""Pins of the particle shapes (input preparation, Sec. 3.1)."""
import json
import math
import os

import numpy as np
import pytest
import torch

from workloads import shapes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_printed_area_ratios():
    g = json.load(open(os.path.join(GOLDEN, "area_ratios.json")))
    L = 100.0
    circ = float(shapes.circle(L)["area"])
    got = dict(ellipse=float(shapes.ellipse(L, 2.0)["area"]) / circ,
               square=float(shapes.square(L)["area"]) / circ,
               triangle=float(shapes.triangle(L)["area"]) / circ)
    for k, v in g["printed_digits"].items():
        assert abs(got[k] - v) <= g["tolerance"][k], (k, got[k])


def _poly_area_and_J(xi_vertices):
    """Shoelace area and polar moment about the origin of a closed polygon."""
    x, y = xi_vertices[:, 0], xi_vertices[:, 1]
    x1, y1 = np.roll(x, -1), np.roll(y, -1)
    cr = x * y1 - x1 * y
    A = cr.sum() / 2
    Ix = ((y * y + y * y1 + y1 * y1) * cr).sum() / 12
    Iy = ((x * x + x * x1 + x1 * x1) * cr).sum() / 12
    return A, Ix + Iy


@pytest.mark.parametrize("fam,args", [("square", (9.0,)), ("triangle", (12.0,)),
                                      ("rectangle", (20.0, 4.0))])
def test_polygon_area_and_polar_moment(fam, args):
    sh = getattr(shapes, fam)(*args)
    # recover the vertices from the edges: consecutive markers on an edge are
    # collinear; rebuild from the closed-form vertex list instead
    if fam == "square":
        a = args[0]
        V = np.array([[-a / 2, -a / 2], [a / 2, -a / 2], [a / 2, a / 2], [-a / 2, a / 2]])
    elif fam == "rectangle":
        w, h = args[0], args[0] / args[1]
        V = np.array([[-w / 2, -h / 2], [w / 2, -h / 2], [w / 2, h / 2], [-w / 2, h / 2]])
    else:
        R = args[0] / math.sqrt(3)
        V = np.array([[R * math.cos(t), R * math.sin(t)]
                      for t in (math.pi / 2, math.pi / 2 + 2 * math.pi / 3, math.pi / 2 + 4 * math.pi / 3)])
    A, J = _poly_area_and_J(V)
    assert math.isclose(float(sh["area"]), A, rel_tol=1e-12)
    assert math.isclose(float(sh["polar_moment"]), J, rel_tol=1e-12)
    # centroid at the origin and the boundary length equals the perimeter
    assert np.allclose(V.mean(0), 0, atol=1e-12)
    per = np.sqrt(((np.roll(V, -1, 0) - V) ** 2).sum(1)).sum()
    assert math.isclose(float(sh["ds"].sum()), per, rel_tol=1e-12)


def test_smooth_shapes_polar_moment_by_quadrature():
    """Circle m R^2/2 and ellipse m (a^2 + b^2)/4, checked by polar quadrature."""
    for sh, (a, b) in ((shapes.circle(10.0), (5.0, 5.0)), (shapes.ellipse(16.0, 2.0), (8.0, 4.0))):
        t = np.linspace(0, 2 * np.pi, 200001)[:-1]
        # J = integral over the boundary of r^4/4 dtheta for a star-shaped body
        r = a * b / np.sqrt((b * np.cos(t)) ** 2 + (a * np.sin(t)) ** 2)
        J = (r ** 4 / 4).mean() * 2 * np.pi
        A = (r ** 2 / 2).mean() * 2 * np.pi
        assert math.isclose(float(sh["polar_moment"]), J, rel_tol=1e-9)
        assert math.isclose(float(sh["area"]), A, rel_tol=1e-9)


@pytest.mark.parametrize("fam", shapes.FAMILIES)
def test_closed_boundary_and_outward_unit_normals(fam):
    sh = shapes.make(fam, 24.0, aspect_ratio=2.5)
    xi, nrm, ds = sh["xi"].numpy(), sh["nrm"].numpy(), sh["ds"].numpy()
    assert np.allclose((nrm * nrm).sum(1), 1.0, atol=1e-14)
    # closed curve: sum n S = 0 (exact for polygons; the arc-equispaced
    # ellipse integrates it by the midpoint rule, O(1/M^2))
    tol = 1e-10 if fam != "ellipse" else 2e-3 * float(ds.sum()) / len(ds) ** 1
    assert np.abs((nrm * ds[:, None]).sum(0)).max() < tol
    assert np.all((xi * nrm).sum(1) > 0)  # convex, centroid inside: outward
    assert np.all(ds > 0)


def test_marker_spacing():
    e = shapes.ellipse(25.0, 2.0, n_markers=64)
    xi = e["xi"].numpy()
    d = np.sqrt(((np.roll(xi, -1, 0) - xi) ** 2).sum(1))
    assert d.max() / d.min() < 1.01  # arc-length equispaced
    assert math.isclose(float(e["ds"].sum()), shapes.ellipse_perimeter(12.5, 6.25), rel_tol=1e-9)
    r = shapes.rectangle(16.0, 4.0, spacing=1.0)
    assert len(r["ds"]) == 2 * 16 + 2 * 4


def test_parameter_ellipse_is_differentiable_in_aspect_ratio():
    ar = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    e = shapes.ellipse(16.0, ar, n_markers=40, mode="param")
    (e["xi"][:, 1].abs().sum() + e["area"]).backward()
    b = 8.0 / 2.0
    # d/dAR of sum |b sin t| + pi a b with b = a/AR: -(b/AR) (sum|sin t| + pi a)
    t = 2 * np.pi * np.arange(40) / 40
    expect = -(b / 2.0) * (np.abs(np.sin(t)).sum() + np.pi * 8.0)
    assert math.isclose(float(ar.grad), expect, rel_tol=1e-12)
