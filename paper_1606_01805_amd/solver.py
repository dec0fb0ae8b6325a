"""Python face of the C ABI: a Solver owns one lbm_handle.

Configuration and particle descriptions are plain dicts with the field names
of lbm_channel_config and lbm_particle_desc.  The population workspace is a
torch uint8 tensor on the current GPU and the work runs on torch's current
stream; nothing here computes any part of the method.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import AGRAD, PSTATE, check, lib

_CFG_DEFAULTS = dict(
    tau=1.0, bc_x=0, bc_y=0, u_wall=((0.0, 0.0),) * 4, init=0, body_force=(0.0, 0.0),
    gravity=(0.0, 0.0), storage=_lib.STORE_F64, fp16_exp=14, mls_rw=2.6, mls_alpha=0.3,
    probe_dn=1.2, mls_kernel=0, spread_scale=0,
)


def channel_config(cfg: dict) -> _lib.ChannelConfig:
    c = dict(_CFG_DEFAULTS)
    c.update(cfg)
    s = _lib.ChannelConfig()
    s.nx, s.ny, s.tau = int(c["nx"]), int(c["ny"]), float(c["tau"])
    s.bc_x, s.bc_y = int(c["bc_x"]), int(c["bc_y"])
    for i in range(4):
        for j in range(2):
            s.u_wall[i][j] = float(c["u_wall"][i][j])
    s.init = int(c["init"])
    for j in range(2):
        s.body_force[j] = float(c["body_force"][j])
        s.gravity[j] = float(c["gravity"][j])
    s.storage, s.fp16_exp = int(c["storage"]), int(c["fp16_exp"])
    s.mls_rw, s.mls_alpha, s.probe_dn = float(c["mls_rw"]), float(c["mls_alpha"]), float(c["probe_dn"])
    s.mls_kernel, s.spread_scale = int(c["mls_kernel"]), int(c["spread_scale"])
    return s


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _p(a):
    return a.ctypes.data_as(_lib._dp)


class Solver:
    """Channels advanced together by the HIP library (batched when > 1).

    channels: list of (config dict, [particle dicts]).  storage overrides the
    configs' storage when given.  tuning: dict of lbm_tuning fields.
    """

    def __init__(self, channels, storage=None, tuning=None, device=None, use_workspace=True):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (no CPU fallback exists)")
        self._L = lib()
        self.device = torch.device(device if device is not None else "cuda")
        cfgs = []
        for cfg, _ in channels:
            cfg = dict(cfg)
            if storage is not None:
                cfg["storage"] = storage
            cfgs.append(cfg)
        self.cfgs = cfgs
        n = len(cfgs)
        arr = (_lib.ChannelConfig * n)(*[channel_config(c) for c in cfgs])
        self._arr = arr
        nbytes = self._L.lbm_workspace_bytes(arr, n)
        if nbytes == 0:
            check(_lib.LBM_EINVAL, None)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.workspace = (torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                              if use_workspace else None)
        h = ctypes.c_void_p()
        ws = self.workspace.data_ptr() if self.workspace is not None else None
        check(self._L.lbm_init(arr, n, ctypes.c_void_p(self.stream.cuda_stream), ws, nbytes,
                               ctypes.byref(h)), None)
        self._h = h
        self.n_particles = 0
        self.particle_channel = []
        self._nmarkers = []
        for ci, (_, parts) in enumerate(channels):
            for p in parts:
                self.add_particle(ci, p)
        if tuning:
            self.set_tuning(**tuning)

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code):
        check(code, self._h)

    # -- particles --
    def add_particle(self, channel, d: dict) -> int:
        xi, nrm, ds = _f64(d["xi"], (-1, 2)), _f64(d["nrm"], (-1, 2)), _f64(d["ds"]).ravel()
        desc = _lib.ParticleDesc(float(d["x"]), float(d["y"]), float(d.get("theta", 0.0)),
                                 float(d.get("u", 0.0)), float(d.get("v", 0.0)), float(d.get("omega", 0.0)),
                                 float(d["density_ratio"]), float(d["area"]), float(d["polar_moment"]),
                                 int(xi.shape[0]), _p(xi), _p(nrm), _p(ds))
        pid = ctypes.c_int32()
        self._chk(self._L.lbm_add_particle(self._h, int(channel), ctypes.byref(desc), ctypes.byref(pid)))
        self.n_particles += 1
        self.particle_channel.append(channel)
        self._nmarkers.append(int(xi.shape[0]))
        return pid.value

    def reset(self):
        """Initial populations again, no particles, step 0 (lbm_reset)."""
        self._chk(self._L.lbm_reset(self._h))
        self.n_particles = 0
        self.particle_channel = []
        self._nmarkers = []

    # -- stepping --
    def step(self, n: int, record: bool = True):
        """Advance n steps; returns the [n, n_particles, 10] record or None."""
        traj = np.zeros((n, self.n_particles, PSTATE)) if (record and self.n_particles) else None
        self._chk(self._L.lbm_step(self._h, int(n), _p(traj) if traj is not None else None))
        return traj

    def particles(self):
        out = np.zeros((max(self.n_particles, 1), PSTATE))
        n = ctypes.c_int32()
        self._chk(self._L.lbm_get_particles(self._h, _p(out), out.shape[0], ctypes.byref(n)))
        return out[: n.value]

    def fields(self, channel=0):
        c = self.cfgs[channel]
        r, u, v = (np.zeros((c["ny"], c["nx"])) for _ in range(3))
        self._chk(self._L.lbm_get_fields(self._h, channel, _p(r), _p(u), _p(v)))
        return r, u, v

    def populations(self, channel=0):
        c = self.cfgs[channel]
        f = np.zeros((9, c["ny"], c["nx"]))
        self._chk(self._L.lbm_get_populations(self._h, channel, _p(f)))
        return f

    def set_populations(self, f, channel=0):
        c = self.cfgs[channel]
        f = _f64(f, (9, c["ny"], c["nx"]))
        self._chk(self._L.lbm_set_populations(self._h, channel, _p(f)))

    def checkpoint_save(self, slot=0):
        self._chk(self._L.lbm_checkpoint_save(self._h, slot))

    def checkpoint_restore(self, slot=0):
        self._chk(self._L.lbm_checkpoint_restore(self._h, slot))

    def set_tuning(self, **kw):
        t = _lib.Tuning()
        self._chk(self._L.lbm_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        self._chk(self._L.lbm_set_tuning(self._h, ctypes.byref(t)))

    def tuning(self):
        t = _lib.Tuning()
        self._chk(self._L.lbm_get_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in _lib.Tuning._fields_}

    def time_kernels(self, reps=100):
        out = np.zeros(3)
        self._chk(self._L.lbm_time_kernels(self._h, int(reps), _p(out)))
        return out

    @property
    def steps_done(self):
        return int(self._L.lbm_steps_done(self._h))

    # -- adjoint --
    def adjoint_begin(self, seed, max_segment):
        """Start reverse mode at the current step; seed [n_particles, 10] is
        dJ/d(last particle records)."""
        seed = _f64(seed, (self.n_particles, PSTATE)) if self.n_particles else np.zeros((1, PSTATE))
        self._chk(self._L.lbm_adjoint_begin(self._h, _p(seed), int(max_segment)))

    def adjoint_segment(self, slot, n):
        """Reverse the n steps that start at checkpoint `slot`."""
        self._chk(self._L.lbm_adjoint_segment(self._h, int(slot), int(n)))

    def adjoint_sweep(self, slots, n):
        """Reverse len(slots) segments of n steps, the last one first: slots[j]
        is the checkpoint of the j-th segment reversed (bitwise the results
        of adjoint_segment on each slot in turn; the recomputation of the
        next segment runs beside the reversal of the current one)."""
        arr = np.ascontiguousarray(np.asarray(slots, dtype=np.int32))
        self._chk(self._L.lbm_adjoint_sweep(self._h, arr.ctypes.data_as(ctypes.c_void_p), int(arr.size), int(n)))

    @property
    def adjoint_position(self):
        return int(self._L.lbm_adjoint_position(self._h))

    def adjoint_gradients(self):
        """(part [n_particles, 25] in the layout of LBM_AGRAD, markers: list
        of [n_markers, 5] per particle, wall [n_channels, 4, 2])."""
        npart = self.n_particles
        part = np.zeros((max(npart, 1), AGRAD))
        nmk = sum(self._nmarkers)
        mk = np.zeros((max(nmk, 1), 5))
        wall = np.zeros((len(self.cfgs), 4, 2))
        self._chk(self._L.lbm_adjoint_gradients(self._h, _p(part), _p(mk), _p(wall)))
        out, o = [], 0
        for m in self._nmarkers:
            out.append(mk[o:o + m].copy())
            o += m
        return part[:npart], out, wall

    def adjoint_field(self, channel=0):
        c = self.cfgs[channel]
        f = np.zeros((9, c["ny"], c["nx"]))
        self._chk(self._L.lbm_adjoint_field(self._h, channel, _p(f)))
        return f
