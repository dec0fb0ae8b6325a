"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same
seeded inputs and compare them."""
import numpy as np

import oracle

SERIES = ["x", "y", "theta", "u", "v", "omega", "Fx", "Fy", "M"]


def run_gpu(channels, steps, storage=None, tuning=None, record=True):
    from paper_1606_01805_amd import Solver

    s = Solver(channels, storage=storage, tuning=tuning)
    tr = s.step(steps, record=record)
    return s, tr


def run_oracle(cfg, parts, steps):
    o = oracle.Oracle(cfg)
    for p in parts:
        o.add_particle(p)
    return o, o.step(steps)


def motion_scales(ref, size):
    """Natural scales of a particle's motion, from the reference trajectory
    [n, 10] and the body size: displacement, angle, velocity, angular
    velocity, force, moment."""
    disp = np.abs(ref[:, 0:2] - ref[0, 0:2]).max()
    vel = np.abs(ref[:, 3:5]).max()
    frc = np.abs(ref[:, 6:8]).max()
    return dict(x=disp, y=disp, theta=disp / size, u=vel, v=vel, omega=vel / size,
                Fx=frc, Fy=frc, M=frc * size)


def series_errors(gpu, ref, size, x0=None):
    """Per-series error of one particle's record [n, 10] against the
    oracle's, each normalised by the motion scale of its group (displacements
    use the initial position x0 of the oracle trajectory's start)."""
    sc = motion_scales(ref, size)
    out = {}
    for k, nm in enumerate(SERIES):
        d = np.abs(gpu[:, k] - ref[:, k]).max()
        out[nm] = d / max(sc[nm], 1e-300)
    return out


def body_size(p):
    xi = np.asarray(p["xi"]).reshape(-1, 2)
    return float(np.sqrt((xi ** 2).sum(1)).max())
