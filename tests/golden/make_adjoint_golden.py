"""Writes tests/golden/adjoint_couette_256x64_fd.json: central finite
differences, on the FP64 oracle only, of the final lateral position y(T) and
angular velocity omega(T) of the 256x64 Couette case (ellipse with major axis
16 and aspect ratio 2, 40 parameter-equispaced markers at (128, 15.75),
theta0 = pi/4, walls at -U and +U with Re = U H / nu = 20, T = 2000) with
respect to y0, theta0, the aspect ratio AR (major axis held) and U.

The MLS anchors make the step map piecewise smooth in the particle state, so
a difference quotient is a derivative only when the perturbed runs use the
same anchors at every step (the oracle hashes every marker and probe
anchor).  For each parameter the largest h in 1e-4, 1e-5, ... 1e-10 for which
the -h, -h/2, 0, +h/2, +h runs share the hash is used, with the Richardson
combination (4 D(h/2) - D(h)) / 3.

Run from the repository root: python tests/golden/make_adjoint_golden.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs as C  # noqa: E402

T = 2000
BASE = dict(y0=15.75, theta0=math.pi / 4, AR=2.0, U=C.couette_speed(64))
HS = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10)


def case(y0, theta0, AR, U):
    wl = C.adjoint_case(storage=C.STORE_F64, y0=y0, theta0=theta0, aspect_ratio=AR)
    cfg, parts = wl.channels[0]
    cfg = dict(cfg)
    cfg["u_wall"] = [[0.0, 0.0], [0.0, 0.0], [-U, 0.0], [U, 0.0]]
    return cfg, parts


def run(**kw):
    cfg, parts = case(**kw)
    o = oracle.Oracle(cfg)
    for p in parts:
        o.add_particle(p)
    o.step(T, record=False)
    st = o.particles()[0]
    return st[1], st[5], o.anchor_hash()


def main():
    y, om, h0 = run(**BASE)
    out = dict(source=__doc__.strip().splitlines()[0], steps=T, base=BASE, y=y, omega=om, grad={})
    for name in ("y0", "theta0", "AR", "U"):
        for h in HS:
            vals = []
            for e in (-h, -h / 2, h / 2, h):
                kw = dict(BASE)
                kw[name] += e
                vals.append(run(**kw))
            if any(v[2] != h0 for v in vals):
                print(name, h, "anchors differ", flush=True)
                continue
            g = {}
            for k, key in ((0, "y"), (1, "omega")):
                d1 = (vals[3][k] - vals[0][k]) / (2 * h)
                d2 = (vals[2][k] - vals[1][k]) / h
                g[key] = (4 * d2 - d1) / 3
                g[key + "_central_h"] = d1
            g["h"] = h
            out["grad"][name] = g
            print(name, g, flush=True)
            break
        else:
            out["grad"][name] = None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_couette_256x64_fd.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
