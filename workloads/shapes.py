"""Particle shapes as Lagrangian marker sets (input preparation).

The paper transports circles, ellipses, squares, equilateral triangles and
rectangles (Sec. 3.1), with the reference length L_ref being the diameter, the
major axis, the edge, the edge and the long edge respectively; it fixes L_ref
through the printed area ratios 0.5 (ellipse of aspect ratio 2), 1.27 (square)
and 0.55 (triangle) against the circle.

Markers sit on segment centres and S_l is the segment length per unit depth (the
2-D reading of the paper's surface "triangles", Sec. 1.3).  Smooth shapes use
arc-length-equispaced markers with analytic normals and S_l = perimeter / M;
polygons split each edge into round(length / spacing) equal sub-segments with
the edge normal.  An ellipse may instead use parameter-equispaced markers
(S_l = local arc element x 2 pi / M), which are smooth in the aspect ratio and so
can be differentiated.

Everything is torch float64 on the CPU so the shape parameters can carry
gradients.  Each function returns a dict with
  xi  [M, 2]  body-frame marker positions about the centroid
  nrm [M, 2]  body-frame outward unit normals
  ds  [M]     segment lengths S_l
  area        body area
  polar_moment  integral of |r|^2 over the body (unit density)
This module holds no part of the flow solver's arithmetic.
"""
import math

import torch

DT = torch.float64


def _t(v):
    return v if torch.is_tensor(v) else torch.tensor(float(v), dtype=DT)


def circle(diameter, n_markers=None, spacing=1.0):
    R = _t(diameter) / 2
    M = int(n_markers) if n_markers else max(8, int(round(math.pi * float(diameter) / spacing)))
    t = 2 * math.pi * torch.arange(M, dtype=DT) / M
    c, s = torch.cos(t), torch.sin(t)
    return dict(
        xi=torch.stack([R * c, R * s], 1),
        nrm=torch.stack([c, s], 1),
        ds=(2 * math.pi * R / M) * torch.ones(M, dtype=DT),
        area=math.pi * R * R,
        polar_moment=math.pi * R ** 4 / 2,
        family="circle",
    )


def _ellipse_param(a, b, t):
    xi = torch.stack([a * torch.cos(t), b * torch.sin(t)], 1)
    tx, ty = -a * torch.sin(t), b * torch.cos(t)
    speed = torch.sqrt(tx * tx + ty * ty)
    nrm = torch.stack([ty / speed, -tx / speed], 1)
    return xi, nrm, speed


def ellipse_perimeter(a, b, n=200000):
    t = 2 * math.pi * torch.arange(n, dtype=DT) / n
    _, _, sp = _ellipse_param(_t(a), _t(b), t)
    return float(sp.detach().sum() * 2 * math.pi / n)


def ellipse(major_axis, aspect_ratio, n_markers=None, spacing=1.0, mode="arc"):
    """Ellipse with semi-axes a = major/2 along x and b = a / aspect_ratio."""
    a = _t(major_axis) / 2
    b = a / _t(aspect_ratio)
    P = ellipse_perimeter(a, b)
    M = int(n_markers) if n_markers else max(8, int(round(P / spacing)))
    if mode == "param":
        t = 2 * math.pi * torch.arange(M, dtype=DT) / M
        xi, nrm, speed = _ellipse_param(a, b, t)
        ds = speed * (2 * math.pi / M)
    else:
        with torch.no_grad():
            n = 200000
            tt = 2 * math.pi * torch.arange(n + 1, dtype=DT) / n
            _, _, sp = _ellipse_param(a, b, tt)
            # cumulative arc length by the trapezoidal rule
            s = torch.cat([torch.zeros(1, dtype=DT), torch.cumsum((sp[1:] + sp[:-1]) * math.pi / n, 0)])
            P = float(s[-1])
            target = P * torch.arange(M, dtype=DT) / M
            j = torch.searchsorted(s, target).clamp(1, n)
            t = tt[j - 1] + (target - s[j - 1]) / (s[j] - s[j - 1]) * (tt[j] - tt[j - 1])
        xi, nrm, _ = _ellipse_param(a, b, t)
        ds = (P / M) * torch.ones(M, dtype=DT)
    return dict(
        xi=xi, nrm=nrm, ds=ds, area=math.pi * a * b,
        polar_moment=math.pi * a * b * (a * a + b * b) / 4, family="ellipse",
    )


def _polygon(vertices, spacing):
    """Counter-clockwise polygon; markers at the centres of equal sub-segments."""
    xs, ns, dss = [], [], []
    V = len(vertices)
    for k in range(V):
        p0, p1 = vertices[k], vertices[(k + 1) % V]
        d = p1 - p0
        L = torch.sqrt((d * d).sum())
        m = max(1, int(round(float(L) / spacing)))
        tpar = (torch.arange(m, dtype=DT) + 0.5) / m
        xs.append(p0[None, :] + tpar[:, None] * d[None, :])
        nout = torch.stack([d[1], -d[0]]) / L
        ns.append(nout[None, :].expand(m, 2))
        dss.append((L / m) * torch.ones(m, dtype=DT))
    return torch.cat(xs, 0), torch.cat(ns, 0), torch.cat(dss, 0)


def rectangle(long_edge, aspect_ratio, spacing=1.0):
    w = _t(long_edge)
    h = w / _t(aspect_ratio)
    z = torch.zeros((), dtype=DT)
    verts = [torch.stack([-w / 2 + z, -h / 2]), torch.stack([w / 2 + z, -h / 2]),
             torch.stack([w / 2 + z, h / 2]), torch.stack([-w / 2 + z, h / 2])]
    xi, nrm, ds = _polygon(verts, spacing)
    return dict(xi=xi, nrm=nrm, ds=ds, area=w * h, polar_moment=w * h * (w * w + h * h) / 12,
                family="rectangle")


def square(edge, spacing=1.0):
    d = rectangle(edge, 1.0, spacing)
    d["family"] = "square"
    return d


def triangle(edge, spacing=1.0):
    """Equilateral triangle with its centroid at the origin, one vertex up."""
    a = _t(edge)
    Rc = a / math.sqrt(3.0)
    verts = [torch.stack([Rc * math.cos(t), Rc * math.sin(t)])
             for t in (math.pi / 2, math.pi / 2 + 2 * math.pi / 3, math.pi / 2 + 4 * math.pi / 3)]
    xi, nrm, ds = _polygon(verts, spacing)
    area = math.sqrt(3.0) / 4 * a * a
    return dict(xi=xi, nrm=nrm, ds=ds, area=area, polar_moment=area * a * a / 12,
                family="triangle")


def bounding_radius(shape) -> float:
    return float(torch.sqrt((shape["xi"] ** 2).sum(1)).max())


FAMILIES = ("circle", "ellipse", "rectangle", "square", "triangle")


def make(family, size, aspect_ratio=2.0, spacing=1.0, n_markers=None):
    """Shape of the given family with reference length L_ref = size."""
    if family == "circle":
        return circle(size, n_markers, spacing)
    if family == "ellipse":
        return ellipse(size, aspect_ratio, n_markers, spacing)
    if family == "rectangle":
        return rectangle(size, aspect_ratio, spacing)
    if family == "square":
        return square(size, spacing)
    if family == "triangle":
        return triangle(size, spacing)
    raise ValueError(family)
