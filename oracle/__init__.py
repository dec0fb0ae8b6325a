"""Python access to the FP64 CPU oracle (test infrastructure only).

The oracle is the plain, serial, FP64 transcription of the coupled
lattice-Boltzmann / MLS immersed-boundary method of Coclite et al.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares nothing with the GPU library: its own C source, its own header, its own
structures here.

Configuration and particle descriptions are plain dicts (see workloads/), the
same dicts the GPU binding accepts.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PSTATE = 10
PERIODIC, ZOUHE = 0, 1
INIT_REST, INIT_COUETTE = 0, 1
SIDE_XLO, SIDE_XHI, SIDE_YLO, SIDE_YHI = 0, 1, 2, 3
W_EXP, W_CUBIC, W_QUARTIC, W_COSINE, W_POLY = 0, 1, 2, 3, 4

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class _Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("u_wall", (ctypes.c_double * 2) * 4), ("init", ctypes.c_int32),
        ("body_force", ctypes.c_double * 2), ("gravity", ctypes.c_double * 2),
        ("mls_rw", ctypes.c_double), ("mls_alpha", ctypes.c_double),
        ("probe_dn", ctypes.c_double), ("mls_kernel", ctypes.c_int32),
        ("spread_scale", ctypes.c_int32),
    ]


class _Particle(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_double), ("y", ctypes.c_double), ("theta", ctypes.c_double),
        ("u", ctypes.c_double), ("v", ctypes.c_double), ("omega", ctypes.c_double),
        ("density_ratio", ctypes.c_double), ("area", ctypes.c_double),
        ("polar_moment", ctypes.c_double), ("n_markers", ctypes.c_int32),
        ("xi", _dp), ("nrm", _dp), ("ds", _dp),
    ]


_lib = None


def lib():
    """Load (building if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Config)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_add_particle.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Particle)]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp]
        L.orc_n_particles.argtypes = [ctypes.c_void_p]
        L.orc_get_particles.argtypes = [ctypes.c_void_p, _dp]
        L.orc_get_populations.argtypes = [ctypes.c_void_p, _dp]
        L.orc_set_populations.argtypes = [ctypes.c_void_p, _dp]
        L.orc_get_fields.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_get_last_force.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_get_last_velocity.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_get_marker_record.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp, ctypes.c_int32]
        L.orc_anchor_hash.restype = ctypes.c_uint64
        L.orc_anchor_hash.argtypes = [ctypes.c_void_p]
        L.orc_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc_lattice.argtypes = [_dp, _dp]
        L.orc_equilibrium.argtypes = [ctypes.c_double] * 3 + [_dp]
        L.orc_collide_node.argtypes = [_dp] + [ctypes.c_double] * 5 + [_dp, _dp, _dp, _dp]
        L.orc_zouhe.argtypes = [ctypes.c_int, _dp] + [ctypes.c_double] * 4
        L.orc_mls.restype = ctypes.c_int
        L.orc_mls.argtypes = [ctypes.POINTER(_Config), ctypes.c_double, ctypes.c_double,
                              _ip, _ip, _ip, _dp, _dp, _dp]
        L.orc_kernel_weight.restype = ctypes.c_double
        L.orc_kernel_weight.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_bdf2.argtypes = [ctypes.c_double] * 5 + [_dp, _dp]
        L.orc_surface_force.argtypes = [ctypes.POINTER(_Config), _dp, _dp, _dp,
                                        ctypes.POINTER(_Particle), _dp, _dp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


DEFAULTS = dict(
    tau=1.0, bc_x=PERIODIC, bc_y=PERIODIC, u_wall=((0.0, 0.0),) * 4, init=INIT_REST,
    body_force=(0.0, 0.0), gravity=(0.0, 0.0), mls_rw=2.6, mls_alpha=0.3, probe_dn=1.2,
    mls_kernel=W_EXP, spread_scale=0,
)


def make_config(cfg: dict) -> _Config:
    c = dict(DEFAULTS)
    c.update({k: v for k, v in cfg.items() if k in DEFAULTS or k in ("nx", "ny")})
    s = _Config()
    s.nx, s.ny = int(c["nx"]), int(c["ny"])
    s.tau = float(c["tau"])
    s.bc_x, s.bc_y = int(c["bc_x"]), int(c["bc_y"])
    for i in range(4):
        for j in range(2):
            s.u_wall[i][j] = float(c["u_wall"][i][j])
    s.init = int(c["init"])
    for j in range(2):
        s.body_force[j] = float(c["body_force"][j])
        s.gravity[j] = float(c["gravity"][j])
    s.mls_rw, s.mls_alpha, s.probe_dn = float(c["mls_rw"]), float(c["mls_alpha"]), float(c["probe_dn"])
    s.mls_kernel, s.spread_scale = int(c["mls_kernel"]), int(c["spread_scale"])
    return s


def _particle_struct(d: dict):
    xi, nrm, ds = _f64(d["xi"], (-1, 2)), _f64(d["nrm"], (-1, 2)), _f64(d["ds"]).ravel()
    p = _Particle(float(d["x"]), float(d["y"]), float(d.get("theta", 0.0)),
                  float(d.get("u", 0.0)), float(d.get("v", 0.0)), float(d.get("omega", 0.0)),
                  float(d["density_ratio"]), float(d["area"]), float(d["polar_moment"]),
                  int(xi.shape[0]), _ptr(xi), _ptr(nrm), _ptr(ds))
    return p, (xi, nrm, ds)


class Oracle:
    """One oracle lattice (a single channel) with its particles."""

    def __init__(self, cfg: dict):
        self._L = lib()
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self.nx, self.ny = self._c.nx, self._c.ny
        self._h = self._L.orc_create(ctypes.byref(self._c))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self._keep = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    def add_particle(self, d: dict) -> int:
        p, keep = _particle_struct(d)
        pid = self._L.orc_add_particle(self._h, ctypes.byref(p))
        if pid < 0:
            raise ValueError("oracle rejected the particle")
        return pid

    @property
    def n_particles(self) -> int:
        return self._L.orc_n_particles(self._h)

    def step(self, n: int, record: bool = True):
        """Advance n steps; returns the [n, np, 10] trajectory (or None)."""
        np_ = self.n_particles
        traj = np.zeros((n, np_, PSTATE)) if (record and np_ > 0) else None
        bad = self._L.orc_step(self._h, int(n), _ptr(traj) if traj is not None else None)
        if bad:
            raise FloatingPointError(f"oracle state became invalid at step {bad}")
        return traj

    def particles(self):
        out = np.zeros((self.n_particles, PSTATE))
        if out.size:
            self._L.orc_get_particles(self._h, _ptr(out))
        return out

    def populations(self):
        f = np.zeros((9, self.ny, self.nx))
        self._L.orc_get_populations(self._h, _ptr(f))
        return f

    def set_populations(self, f):
        f = _f64(f, (9, self.ny, self.nx))
        self._L.orc_set_populations(self._h, _ptr(f))

    def fields(self):
        r, u, v = (np.zeros((self.ny, self.nx)) for _ in range(3))
        self._L.orc_get_fields(self._h, _ptr(r), _ptr(u), _ptr(v))
        return r, u, v

    def last_force(self):
        fx, fy = np.zeros((self.ny, self.nx)), np.zeros((self.ny, self.nx))
        self._L.orc_get_last_force(self._h, _ptr(fx), _ptr(fy))
        return fx, fy

    def last_velocity(self):
        ux, uy = np.zeros((self.ny, self.nx)), np.zeros((self.ny, self.nx))
        self._L.orc_get_last_velocity(self._h, _ptr(ux), _ptr(uy))
        return ux, uy

    def marker_record(self, p: int):
        n = self._L.orc_get_marker_record(self._h, p, None, 0)
        out = np.zeros((n, 8))
        self._L.orc_get_marker_record(self._h, p, _ptr(out), n)
        return out

    def anchor_hash(self) -> int:
        return int(self._L.orc_anchor_hash(self._h))

    def set_threads(self, n: int):
        """Threads for the node loops (results do not depend on it)."""
        self._L.orc_set_threads(self._h, int(n))


# ---- stage functions (closed-form tests) ----

def lattice():
    e, w = np.zeros((9, 2)), np.zeros(9)
    lib().orc_lattice(_ptr(e), _ptr(w))
    return e, w


def equilibrium(rho, ux, uy):
    f = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, _ptr(f))
    return f


def collide_node(f, g, flb, tau):
    f = _f64(f)
    out = np.zeros(9)
    r, ux, uy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_collide_node(_ptr(f), g[0], g[1], flb[0], flb[1], tau, _ptr(out),
                           ctypes.byref(r), ctypes.byref(ux), ctypes.byref(uy))
    return out, r.value, np.array([ux.value, uy.value])


def zouhe(side, f, uw, g=(0.0, 0.0)):
    f = _f64(f).copy()
    lib().orc_zouhe(side, _ptr(f), uw[0], uw[1], g[0], g[1])
    return f


def mls(cfg: dict, x: float, y: float):
    """MLS shape functions at (x, y): (nodes[9,2], valid[9], phi, dphi_dx, dphi_dy)."""
    c = make_config(cfg)
    ni, nj, ok = (np.zeros(9, dtype=np.int32) for _ in range(3))
    phi, dx, dy = np.zeros(9), np.zeros(9), np.zeros(9)
    ip = lambda a: a.ctypes.data_as(_ip)  # noqa: E731
    lib().orc_mls(ctypes.byref(c), x, y, ip(ni), ip(nj), ip(ok), _ptr(phi), _ptr(dx), _ptr(dy))
    return np.stack([ni, nj], 1), ok.astype(bool), phi, dx, dy


def kernel_weight(kind, r, alpha=0.3):
    return lib().orc_kernel_weight(kind, r, alpha)


def bdf2(v, vm, acc, x, xm):
    vn, xn = ctypes.c_double(), ctypes.c_double()
    lib().orc_bdf2(v, vm, acc, x, xm, ctypes.byref(vn), ctypes.byref(xn))
    return vn.value, xn.value


def surface_force(cfg: dict, rho, ux, uy, particle: dict, acc=(0.0, 0.0, 0.0)):
    """Force and moment (Fx, Fy, M) of Eqs. (13), (14) on given level-n fields."""
    c = make_config(cfg)
    shp = (c.ny, c.nx)
    rho, ux, uy = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
    p, keep = _particle_struct(particle)
    a = _f64(acc)
    out = np.zeros(3)
    lib().orc_surface_force(ctypes.byref(c), _ptr(rho), _ptr(ux), _ptr(uy), ctypes.byref(p),
                            _ptr(a), _ptr(out))
    return out
