"""Central finite differences of the oracle for the adjoint tests.

J = c . (x, y, theta, u, v, omega) of the particle after T steps.  A
parameter is perturbed through the inputs (configuration, particle
descriptor, initial populations); the derivative is the Richardson
combination (4 D(h/2) - D(h)) / 3 of two central differences, valid only when
the -h, -h/2, +h/2, +h runs used the same MLS anchors at every step (the
oracle's anchor hash): the step map is only piecewise smooth in the particle
state.  Returns None where the anchors differ for every h tried.
"""
import copy

import numpy as np

import oracle


def objective(cfg, parts, T, c, f0=None):
    o = oracle.Oracle(cfg)
    for p in parts:
        o.add_particle(p)
    if f0 is not None:
        o.set_populations(f0)
    o.step(T, record=False)
    st = o.particles()
    return float(np.dot(c, st[0, :6])), o.anchor_hash()


def derivative(cfg, parts, T, c, perturb, hs=(1e-3, 1e-4, 1e-5, 1e-6)):
    """perturb(cfg, parts, eps) modifies copies in place and returns f0 or
    None.  Returns (derivative, h) for the largest valid h, or (None, None)."""
    def J(eps):
        cf, pp = copy.deepcopy(cfg), copy.deepcopy(parts)
        f0 = perturb(cf, pp, eps)
        return objective(cf, pp, T, c, f0)

    for h in hs:
        vals = [J(e) for e in (-h, -h / 2, h / 2, h)]
        if len({v[1] for v in vals}) != 1:
            continue
        d1 = (vals[3][0] - vals[0][0]) / (2 * h)
        d2 = (vals[2][0] - vals[1][0]) / h
        return (4 * d2 - d1) / 3, h
    return None, None


def particle_field(key, idx=None):
    def m(cf, pp, eps):
        if idx is None:
            pp[0][key] = float(pp[0][key]) + eps
        else:
            a = np.array(pp[0][key], dtype=np.float64).copy()
            a.flat[idx] += eps
            pp[0][key] = a
        return None
    return m


def wall_speed(side, comp):
    def m(cf, pp, eps):
        uw = [list(map(float, v)) for v in cf["u_wall"]]
        uw[side][comp] += eps
        cf["u_wall"] = uw
        return None
    return m
