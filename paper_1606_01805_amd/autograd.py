"""torch.autograd binding of the library's discrete adjoint.

`LBMIBMFunction` runs the coupled LBM / MLS-IBM solver forward on the GPU
(checkpointing every `segment` steps) and returns the particle records after
the last step; its backward pass calls the hand-written adjoint kernels
(lbm_adjoint_*): every segment is recomputed from its checkpoint into a tape
and reversed.  All arithmetic runs in the HIP library; this module only moves
arguments.  Inputs that carry gradients:

  pose    [n_particles, 6]  initial x, y, theta, u, v, omega
  xi      [n_markers, 2]    body-frame marker positions (all particles, in order)
  nrm     [n_markers, 2]    body-frame outward normals
  ds      [n_markers]       segment lengths S_l
  area    [n_particles]     body areas (m = density_ratio * area)
  polar   [n_particles]     polar moments (I = density_ratio * polar)
  u_wall  [n_channels, 4, 2] wall velocities

The output is [n_particles, 9]: x, y, theta, u, v, omega, Fx, Fy, M after the
last step (force and moment of that step).  Tensors are float64 on the CPU.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from .solver import Solver


@dataclass
class RunSpec:
    """The non-differentiable part of a run."""
    configs: List[dict]                 # channel configs (u_wall is replaced)
    density_ratio: List[float]          # per particle
    n_markers: List[int]                # per particle
    channel: List[int]                  # per particle
    steps: int
    segment: int = 100                  # checkpoint interval = tape length
    storage: Optional[int] = None
    tuning: Optional[dict] = None
    solver: Optional[Solver] = field(default=None, repr=False)  # last forward's solver


def _channels(spec, pose, xi, nrm, ds, area, polar, u_wall):
    chans = []
    for ci, cfg in enumerate(spec.configs):
        cfg = dict(cfg)
        cfg["u_wall"] = [[float(u_wall[ci, s, 0]), float(u_wall[ci, s, 1])] for s in range(4)]
        chans.append((cfg, []))
    off = 0
    for p, m in enumerate(spec.n_markers):
        chans[spec.channel[p]][1].append(dict(
            x=float(pose[p, 0]), y=float(pose[p, 1]), theta=float(pose[p, 2]), u=float(pose[p, 3]),
            v=float(pose[p, 4]), omega=float(pose[p, 5]), density_ratio=float(spec.density_ratio[p]),
            area=float(area[p]), polar_moment=float(polar[p]),
            xi=xi[off:off + m].numpy(), nrm=nrm[off:off + m].numpy(), ds=ds[off:off + m].numpy()))
        off += m
    return chans


class LBMIBMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pose, xi, nrm, ds, area, polar, u_wall, spec: RunSpec):
        if spec.steps % spec.segment != 0:
            raise ValueError("steps must be a multiple of segment")
        nseg = spec.steps // spec.segment
        if nseg > 63:
            raise ValueError("at most 63 segments (raise segment)")
        args = [t.detach().to("cpu", torch.float64) for t in (pose, xi, nrm, ds, area, polar, u_wall)]
        chans = _channels(spec, *args)
        # particles are added channel by channel; keep the caller's order
        order = sorted(range(len(spec.channel)), key=lambda p: (spec.channel[p], p))
        s = Solver(chans, storage=spec.storage, tuning=spec.tuning)
        for k in range(nseg):
            s.checkpoint_save(k)
            s.step(spec.segment, record=False)
        s.checkpoint_save(nseg)  # the final state, for repeated backward passes
        rec = s.particles()
        out = np.zeros((len(order), 9))
        for j, p in enumerate(order):
            out[p] = rec[j, :9]
        ctx.solver = s
        ctx.spec = spec
        ctx.order = order
        spec.solver = s
        return torch.from_numpy(out)

    @staticmethod
    def backward(ctx, g):
        s, spec, order = ctx.solver, ctx.spec, ctx.order
        npart = len(order)
        s.checkpoint_restore(spec.steps // spec.segment)
        seed = np.zeros((npart, 10))
        gn = g.detach().to("cpu", torch.float64).numpy()
        for j, p in enumerate(order):
            seed[j, :9] = gn[p]
        s.adjoint_begin(seed, spec.segment)
        s.adjoint_sweep(list(reversed(range(spec.steps // spec.segment))), spec.segment)
        part, mk, wall = s.adjoint_gradients()
        g_pose = np.zeros((npart, 6))
        g_area = np.zeros(npart)
        g_polar = np.zeros(npart)
        mks = [None] * npart
        for j, p in enumerate(order):
            # entries 17..24: initial pose and velocities, area, polar moment
            g_pose[p] = part[j, 17:23]
            g_area[p] = part[j, 23]
            g_polar[p] = part[j, 24]
            mks[p] = mk[j]
        mk = np.concatenate(mks, 0)
        t = lambda v: torch.from_numpy(np.ascontiguousarray(v))
        return (t(g_pose), t(mk[:, 0:2]), t(mk[:, 2:4]), t(mk[:, 4]), t(g_area), t(g_polar), t(wall), None)


def run_particles(pose, xi, nrm, ds, area, polar, u_wall, spec: RunSpec):
    """Differentiable final particle records [n_particles, 9]."""
    return LBMIBMFunction.apply(pose, xi, nrm, ds, area, polar, u_wall, spec)
