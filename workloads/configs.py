"""Seeded synthetic workloads shaped like the paper's experiments (inputs only).

The paper's own cases are a sedimenting circle and ellipse in a narrow channel
(Sec. 2) and neutrally buoyant particles of five shapes in a Re = 20 Couette
flow (Sec. 3).  The workloads below keep those shapes, sizes, boundary
conditions and value ranges, scaled to the lattice sizes used for measurement:

  sedimentation  80x240, Zou-He side walls (u = 0), periodic in y, tau = 0.8,
                 fluid at rest, circle D = 10 at (40, 180), 32 markers,
                 density ratio 1.01, gravity 1e-5 along -y
  couette        400x100, periodic x, walls at y = 0 and y = NY-1 moving at
                 -U and +U with Re = U H / nu = 20 (H = NY nodes, tau = 1),
                 one neutrally buoyant ellipse (AR 2, major axis 25, 64 markers),
                 y0 ~ U[0.2, 0.8] (NY-1), theta0 ~ U[0, pi), seed 1606
  ensemble       256 independent Couette channels, H in {64, 96, 128, 192, 256},
                 L = 4H, one particle each of size 0.25 H from the five families,
                 markers 1 lu apart, random pose, seed 1606 + channel
  large          4096x1024 Couette, 64 non-overlapping particles of size
                 U[24, 48] from the five families, random poses, seed 1607
  adjoint        256x64 Couette, ellipse AR 2, major axis 16, 40
                 parameter-equispaced markers at (128, 15.75), theta0 = pi/4

Each channel is a config dict (the keys of the C structure lbm_channel_config)
and a list of particle dicts (the keys of lbm_particle_desc).  The kinematic
viscosity used to pick the wall speed is nu = (tau - 1/2)/3.
"""
import math

import numpy as np

from . import shapes

PERIODIC, ZOUHE = 0, 1
INIT_REST, INIT_COUETTE = 0, 1
STORE_F64, STORE_F32, STORE_F16S = 0, 1, 2


def base_config(nx, ny, tau=1.0, **kw):
    c = dict(nx=int(nx), ny=int(ny), tau=float(tau), bc_x=PERIODIC, bc_y=PERIODIC,
             u_wall=[[0.0, 0.0] for _ in range(4)], init=INIT_REST, body_force=[0.0, 0.0],
             gravity=[0.0, 0.0], storage=STORE_F64, fp16_exp=14, mls_rw=2.6, mls_alpha=0.3,
             probe_dn=1.2, mls_kernel=0, spread_scale=0)
    c.update(kw)
    return c


def couette_speed(ny, tau=1.0, re=20.0):
    """Wall speed U with Re = U H / nu, H = NY nodes, wall gap NY - 1."""
    nu = (tau - 0.5) / 3.0
    return re * nu / (ny - 1)


def couette_config(nx, ny, tau=1.0, re=20.0, **kw):
    U = couette_speed(ny, tau, re)
    uw = [[0.0, 0.0], [0.0, 0.0], [-U, 0.0], [U, 0.0]]
    return base_config(nx, ny, tau, bc_y=ZOUHE, u_wall=uw, init=INIT_COUETTE, **kw)


def particle(shape, x, y, theta=0.0, density_ratio=1.0, u=0.0, v=0.0, omega=0.0):
    return dict(
        x=float(x), y=float(y), theta=float(theta), u=float(u), v=float(v), omega=float(omega),
        density_ratio=float(density_ratio), area=float(shape["area"]),
        polar_moment=float(shape["polar_moment"]),
        xi=shape["xi"].detach().numpy().astype(np.float64).copy(),
        nrm=shape["nrm"].detach().numpy().astype(np.float64).copy(),
        ds=shape["ds"].detach().numpy().astype(np.float64).copy(),
        family=shape.get("family", ""),
    )


class Workload:
    def __init__(self, name, channels, steps, storage):
        self.name = name
        self.channels = channels  # list of (config dict, [particle dicts])
        self.steps = steps
        self.storage = storage

    @property
    def nodes(self):
        return sum(c["nx"] * c["ny"] for c, _ in self.channels)

    @property
    def n_particles(self):
        return sum(len(p) for _, p in self.channels)

    def with_storage(self, storage):
        chans = []
        for c, ps in self.channels:
            c = dict(c)
            c["storage"] = storage
            chans.append((c, ps))
        return Workload(self.name, chans, self.steps, storage)


def sedimentation(storage=STORE_F64):
    cfg = base_config(80, 240, tau=0.8, bc_x=ZOUHE, gravity=[0.0, -1e-5], storage=storage)
    sh = shapes.circle(10.0, n_markers=32)
    return Workload("sedimentation 80x240 circle D10", [(cfg, [particle(sh, 40.0, 180.0, 0.0, 1.01)])],
                    2000, storage)


def couette(storage=STORE_F32, seed=1606, nx=400, ny=100):
    rng = np.random.default_rng(seed)
    cfg = couette_config(nx, ny, storage=storage)
    y0 = rng.uniform(0.2, 0.8) * (ny - 1)
    th0 = rng.uniform(0.0, math.pi)
    sh = shapes.ellipse(25.0, 2.0, n_markers=64)
    return Workload(f"couette Re20 {nx}x{ny} ellipse AR2", [(cfg, [particle(sh, nx / 2, y0, th0)])],
                    50000, storage)


def random_shape(rng, size, spacing=1.0):
    fam = shapes.FAMILIES[int(rng.integers(0, 5))]
    ar = float(rng.uniform(1.5, 4.0)) if fam in ("ellipse", "rectangle") else 1.0
    return shapes.make(fam, size, aspect_ratio=ar, spacing=spacing)


def ensemble(storage=STORE_F32, n_channels=256, seed=1606):
    chans = []
    for c in range(n_channels):
        rng = np.random.default_rng(seed + c)
        H = int(rng.choice([64, 96, 128, 192, 256]))
        cfg = couette_config(4 * H, H, storage=storage)
        sh = random_shape(rng, 0.25 * H)
        rb = shapes.bounding_radius(sh)
        x = rng.uniform(0.0, 4 * H)
        y = rng.uniform(0.2, 0.8) * (H - 1)
        y = min(max(y, rb + 6.0), H - 1 - rb - 6.0)
        th = rng.uniform(0.0, 2 * math.pi)
        chans.append((cfg, [particle(sh, x, y, th)]))
    return Workload(f"ensemble {n_channels} Couette channels", chans, 1000, storage)


def large(storage=STORE_F32, n_particles=64, seed=1607, nx=4096, ny=1024):
    rng = np.random.default_rng(seed)
    cfg = couette_config(nx, ny, storage=storage)
    placed = []
    parts = []
    tries = 0
    while len(parts) < n_particles:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place particles")
        size = rng.uniform(24.0, 48.0)
        sh = random_shape(rng, size)
        rb = shapes.bounding_radius(sh)
        x = rng.uniform(0.0, nx)
        y = rng.uniform(rb + 6.0, ny - 1 - rb - 6.0)
        th = rng.uniform(0.0, 2 * math.pi)
        ok = True
        for (px, py, pr) in placed:
            dx = abs(x - px)
            dx = min(dx, nx - dx)
            if math.hypot(dx, y - py) < rb + pr + 6.0:
                ok = False
                break
        if not ok:
            continue
        placed.append((x, y, rb))
        parts.append(particle(sh, x, y, th))
    return Workload(f"large {nx}x{ny} {n_particles} particles", [(cfg, parts)], 10000, storage)


def adjoint_case(storage=STORE_F32, y0=15.75, theta0=math.pi / 4, aspect_ratio=2.0, re=20.0):
    cfg = couette_config(256, 64, re=re, storage=storage)
    sh = shapes.ellipse(16.0, aspect_ratio, n_markers=40, mode="param")
    return Workload("adjoint 256x64 ellipse AR2", [(cfg, [particle(sh, 128.0, y0, theta0)])],
                    2000, storage)


# ---- the paper's own experiments at full scale (Secs. 2 and 3) ----

PAPER_SPACING = 0.3  # marker spacing over the lattice spacing (Secs. 2.1, 2.2, 3.1)


def paper_couette_config(L=100, re=20.0, u_wall=0.01, storage=STORE_F32):
    """Sec. 3.1: a channel of 10 L x 4 L (periodic in x), bottom wall fixed,
    top wall at u_wall, Re = u_wall H / nu = 20 with H = 4 L the wall gap,
    started on the planar Couette profile.  With u_wall = 0.01 and L = 100
    (so that dt u_wall / L = 1e-4): nu = 0.2, tau = 1.1."""
    H = 4 * L
    nu = u_wall * H / re
    tau = 3.0 * nu + 0.5
    uw = [[0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [u_wall, 0.0]]
    return base_config(10 * L, H + 1, tau, bc_y=ZOUHE, u_wall=uw, init=INIT_COUETTE, storage=storage)


def paper_couette_shape(family, L=100, spacing=PAPER_SPACING):
    """The particle families of Sec. 3 with L_ref = L: circle (diameter),
    ellipse of aspect ratio 2 (major axis), square (edge), equilateral
    triangle (edge) and the rectangle of aspect ratio 10 (long edge)."""
    if family == "rectangle":
        return shapes.rectangle(L, 10.0, spacing)
    return shapes.make(family, L, aspect_ratio=2.0, spacing=spacing)


def paper_couette(cases, L=100, storage=STORE_F32):
    """One channel per (family, release height y0/H, initial x velocity over
    u_wall) of Sec. 3: neutrally buoyant, at rest (or at the given x
    velocity), released at x = 5 L."""
    chans = []
    for fam, yfrac, u0 in cases:
        cfg = paper_couette_config(L, storage=storage)
        H = cfg["ny"] - 1
        uw = cfg["u_wall"][3][0]
        sh = paper_couette_shape(fam, L)
        chans.append((cfg, [particle(sh, 5.0 * L, yfrac * H, 0.0, 1.0, u=u0 * uw)]))
    return Workload(f"paper Couette transport {10 * L}x{4 * L + 1}, {len(cases)} channels", chans, 0, storage)


def paper_sedimentation_circle(N, storage=STORE_F32, spacing=PAPER_SPACING, re=0.1):
    """Sec. 2.1 at resolution N (points per diameter): a closed box of
    4 N x 30 N lattice spacings, tau = 1, a circle of diameter N released at
    rest at (2 N, 28 N), density ratio 1.2, and the terminal Reynolds number
    Re = U N / nu = 0.1 of the paper.  The printed Froude number cannot hold
    with it in this channel (g = U^2 / (1398.3 N) gives a terminal Re near
    6e-8), so gravity is set from the wall-corrected Stokes drag of a
    cylinder midway between plane walls (Faxen): with k = D / W = 1/4,
    F / (mu U) = 4 pi / (ln(1/k) - 0.9157 + 1.7244 k^2 - 1.7302 k^4), and
    (rho_s - rho_f) A g = F.  The terminal velocity actually reached is
    measured, not assumed.  Returns the channel and U."""
    tau = 1.0
    nu = (tau - 0.5) / 3.0
    U = re * nu / N
    k = 0.25
    lam = 4.0 * math.pi / (math.log(1.0 / k) - 0.9157 + 1.7244 * k ** 2 - 1.7302 * k ** 4)
    area = math.pi * N * N / 4.0
    g = lam * nu * U / ((1.2 - 1.0) * area)
    cfg = base_config(4 * N + 1, 30 * N + 1, tau, bc_x=ZOUHE, bc_y=ZOUHE, gravity=[0.0, -g],
                      storage=storage)
    sh = shapes.circle(N, spacing=spacing)
    return (cfg, [particle(sh, 2.0 * N, 28.0 * N, 0.0, 1.2)]), U


def paper_sedimentation_ellipse(kernel=0, L=100, storage=STORE_F64, spacing=PAPER_SPACING):
    """Sec. 2.2: a closed box of 4 L x 30 L, tau = 1, an ellipse of major axis
    L and aspect ratio 2 released at rest at (2 L, 24 L) with theta0 = pi/4,
    density ratio 1.1, Re = u L / nu = 12.5, Fr = u / sqrt(L g) = 0.126,
    interpolation kernel `kernel`."""
    tau = 1.0
    nu = (tau - 0.5) / 3.0
    u = 12.5 * nu / L
    g = u * u / (0.126 ** 2 * L)
    cfg = base_config(4 * L + 1, 30 * L + 1, tau, bc_x=ZOUHE, bc_y=ZOUHE, gravity=[0.0, -g],
                      storage=storage, mls_kernel=kernel)
    sh = shapes.ellipse(L, 2.0, spacing=spacing)
    return (cfg, [particle(sh, 2.0 * L, 24.0 * L, math.pi / 4, 1.1)]), u


BY_NAME = dict(sedimentation=sedimentation, couette=couette, ensemble=ensemble, large=large,
               adjoint=adjoint_case)
