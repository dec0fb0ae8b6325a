"""Discrete adjoint of the coupled step on the GPU, through the C ABI, against
central finite differences of the FP64 oracle.

J = c . (x, y, theta, u, v, omega) after T steps, c random.  Every gradient
the library returns is checked: initial pose and velocities (the BDF2
history starts equal to them, so each is the sum of its current and previous
slots at step 0), marker positions, normals and segment lengths, area and
polar moment (through m = ratio * area, I = ratio * polar moment), wall
velocities (Zou-He closure and Couette start) and, through the adjoint
populations, a random interior perturbation of the initial populations.
The finite differences are Richardson-extrapolated and taken only where the
MLS anchors of all perturbed runs agree (tests/adjoint_fd.py); their
accuracy is ~1e-10 relative, so the FP64 bar is 1e-6 relative plus 5e-11
absolute (J is of order 10: 5e-12 of it).
"""
import numpy as np
import pytest

from workloads import configs as C
from workloads import shapes

import adjoint_fd as FD

pytestmark = pytest.mark.gpu

TOL_R, TOL_A = 1e-6, 5e-11


def _case(kind):
    if kind == "couette":
        cfg = C.couette_config(32, 24, tau=0.8, storage=0)
    elif kind == "sidewall":
        cfg = C.base_config(24, 32, tau=0.8, bc_x=1, u_wall=[[0.0, 0.01], [0.0, -0.02], [0.0, 0.0], [0.0, 0.0]],
                            body_force=[0.0, 1e-5], storage=0)
    elif kind == "cosine-unit":
        cfg = C.couette_config(32, 24, tau=0.8, storage=0, mls_kernel=3, spread_scale=1)
    else:
        raise ValueError(kind)
    cfg["gravity"] = [0.0, -1e-5]
    sh = shapes.ellipse(8.0, 2.0, n_markers=20, mode="param")
    p = C.particle(sh, 15.3, 11.1, 0.3, density_ratio=1.3, u=0.002, v=-0.001, omega=0.001)
    return cfg, [p]


def gpu_adjoint(cfg, parts, T, c, seg=None, storage=None, tuning=None, sweep=False, all_parts=False):
    from paper_1606_01805_amd import Solver

    seg = seg or T
    s = Solver([(cfg, parts)], storage=storage, tuning=tuning)
    for k in range(T // seg):
        s.checkpoint_save(k)
        s.step(seg, record=False)
    seed = np.zeros((len(parts), 10))
    seed[:, :6] = c
    s.adjoint_begin(seed, seg)
    if sweep:
        s.adjoint_sweep(list(reversed(range(T // seg))), seg)
    else:
        for k in reversed(range(T // seg)):
            s.adjoint_segment(k, seg)
    assert s.adjoint_position == 0
    part, mk, wall = s.adjoint_gradients()
    lam = s.adjoint_field(0)
    pops = s.populations()
    s.close()
    if all_parts:
        return part, mk, wall, lam, pops
    return part[0], mk[0], wall[0], lam


def _params(cfg, parts, part, mk, wall):
    ratio = parts[0]["density_ratio"]
    # the library's derived entries are the slot sums and scaled mass terms
    assert np.array_equal(part[17:23], [part[0] + part[2], part[1] + part[3], part[4] + part[5],
                                        part[6] + part[8], part[7] + part[9], part[10] + part[11]])
    assert part[23] == part[15] * ratio and part[24] == part[16] * ratio
    rows = [("x0", part[17], FD.particle_field("x")),
            ("y0", part[18], FD.particle_field("y")),
            ("theta0", part[19], FD.particle_field("theta")),
            ("u0", part[20], FD.particle_field("u")),
            ("v0", part[21], FD.particle_field("v")),
            ("omega0", part[22], FD.particle_field("omega")),
            ("area", part[23], FD.particle_field("area")),
            ("polar", part[24], FD.particle_field("polar_moment"))]
    for l in (0, 7, 13):
        rows += [(f"xi[{l}].x", mk[l, 0], FD.particle_field("xi", 2 * l)),
                 (f"xi[{l}].y", mk[l, 1], FD.particle_field("xi", 2 * l + 1)),
                 (f"nrm[{l}].x", mk[l, 2], FD.particle_field("nrm", 2 * l)),
                 (f"nrm[{l}].y", mk[l, 3], FD.particle_field("nrm", 2 * l + 1)),
                 (f"ds[{l}]", mk[l, 4], FD.particle_field("ds", l))]
    sides = (2, 3) if cfg["bc_y"] == 1 else ((0, 1) if cfg["bc_x"] == 1 else ())
    for sd in sides:
        for comp in (0, 1):
            rows.append((f"u_wall[{sd}][{comp}]", wall[sd, comp], FD.wall_speed(sd, comp)))
    return rows


@pytest.mark.parametrize("kind", ["couette", "sidewall", "cosine-unit"])
def test_adjoint_matches_oracle_finite_differences(kind):
    cfg, parts = _case(kind)
    T = 12
    c = np.random.default_rng(11).standard_normal(6)
    part, mk, wall, lam = gpu_adjoint(cfg, parts, T, c)
    bad = []
    for name, g, pert in _params(cfg, parts, part, mk, wall):
        fd, h = FD.derivative(cfg, parts, T, c, pert)
        assert fd is not None, f"{name}: anchors change for every step size"
        err = abs(g - fd)
        print(f"{kind} {name:14s} adjoint {g: .12e} fd {fd: .12e} (h={h:g}) err {err:.2e}")
        if err > TOL_R * abs(fd) + TOL_A:
            bad.append((name, g, fd))
    # dJ/d(initial populations) along an interior direction
    o_f0 = _oracle_f0(cfg, parts)
    d = np.random.default_rng(3).standard_normal(o_f0.shape) * 1e-2
    if cfg["bc_y"] == 1:
        d[:, 0, :] = d[:, -1, :] = 0.0
    if cfg["bc_x"] == 1:
        d[:, :, 0] = d[:, :, -1] = 0.0

    def pert_f(cf, pp, eps):
        return o_f0 + eps * d

    fd, h = FD.derivative(cfg, parts, T, c, pert_f)
    g = float((lam * d).sum())
    print(f"{kind} {'f0 direction':14s} adjoint {g: .12e} fd {fd: .12e} (h={h:g})")
    if abs(g - fd) > TOL_R * abs(fd) + TOL_A:
        bad.append(("f0", g, fd))
    assert not bad, bad


def _oracle_f0(cfg, parts):
    import oracle

    o = oracle.Oracle(cfg)
    for p in parts:
        o.add_particle(p)
    return o.populations()


def test_segments_reproduce_single_sweep_bitwise():
    cfg, parts = _case("couette")
    c = np.random.default_rng(5).standard_normal(6)
    a = gpu_adjoint(cfg, parts, 12, c)
    b = gpu_adjoint(cfg, parts, 12, c, seg=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_adjoint_launch_shape_independent():
    cfg, parts = _case("couette")
    c = np.random.default_rng(6).standard_normal(6)
    a = gpu_adjoint(cfg, parts, 8, c)
    b = gpu_adjoint(cfg, parts, 8, c, tuning=dict(tile_w=64, rows_per_thread=2))
    d = gpu_adjoint(cfg, parts, 8, c, tuning=dict(tile_w=64, rows_per_thread=2, overlap=1))
    for x, y, z in zip(a, b, d):
        assert np.array_equal(x, y)
        assert np.array_equal(x, z)


@pytest.mark.parametrize("storage,tol", [(C.STORE_F32, 1e-3), (C.STORE_F16S, 3e-2)])
def test_reduced_forms_close_to_fp64_adjoint(storage, tol):
    """FP32 / FP16S populations (FP32 adjoint populations): each gradient
    group within tol of the FP64 adjoint, relative to the group's largest
    entry."""
    cfg, parts = _case("couette")
    c = np.random.default_rng(7).standard_normal(6)
    ref = gpu_adjoint(cfg, parts, 12, c)
    red = gpu_adjoint(cfg, parts, 12, c, storage=storage)
    for name, x, y in zip(("particle", "markers", "walls", "populations"), ref, red):
        e = np.abs(x - y).max() / np.abs(x).max()
        print(storage, name, e)
        assert e < tol, (name, e)


# ---------------------------------------------------------------------------
# The 256x64 Couette case through torch.autograd, against the committed
# finite differences of the FP64 oracle (tests/golden/make_adjoint_golden.py).
# ---------------------------------------------------------------------------
def _couette_256x64(storage):
    import json
    import os

    import torch

    from paper_1606_01805_amd.autograd import RunSpec, run_particles

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "adjoint_couette_256x64_fd.json")))
    b = gold["base"]
    f64 = torch.float64
    y0, th0, AR, U = (torch.tensor(b[k], dtype=f64, requires_grad=True) for k in ("y0", "theta0", "AR", "U"))
    sh = shapes.ellipse(16.0, AR, n_markers=40, mode="param")
    z = torch.zeros((), dtype=f64)
    pose = torch.stack([torch.tensor(128.0, dtype=f64), y0, th0, z, z, z])[None]
    u_wall = torch.stack([torch.stack([z, z]), torch.stack([z, z]), torch.stack([-U, z]), torch.stack([U, z])])[None]
    cfg = C.adjoint_case(storage=storage).channels[0][0]
    spec = RunSpec(configs=[cfg], density_ratio=[1.0], n_markers=[40], channel=[0], steps=gold["steps"],
                   segment=100, storage=storage)
    out = run_particles(pose, sh["xi"], sh["nrm"], sh["ds"], sh["area"].reshape(1), sh["polar_moment"].reshape(1),
                        u_wall, spec)
    gy = torch.autograd.grad(out[0, 1], [y0, th0, AR, U], retain_graph=True)
    gw = torch.autograd.grad(out[0, 5], [y0, th0, AR, U])
    spec.solver.close()
    return gold, out.detach().numpy(), [float(v) for v in gy], [float(v) for v in gw]


@pytest.mark.parametrize("storage,tol", [(C.STORE_F64, 1e-5), (C.STORE_F32, 5e-3)])
def test_couette_256x64_gradients_match_oracle_fd(storage, tol):
    """d y(T) and d omega(T) (T = 2000, 20 checkpointed segments of 100) with
    respect to y0, theta0, aspect ratio and wall speed.

    Bar: tol relative plus twice the finite difference's own error estimate
    |D(h) - D(h/2)| = 3/4 |D(h) - R| (R the Richardson value): over 2000
    steps the rounding noise of J divided by the small h the anchors allow
    reaches ~1e-5 of the smaller derivatives.  tol = 1e-5 for FP64
    populations; 5e-3 for FP32 populations (measured worst 3.9e-3 for
    d omega / d U and 2.2e-3 for d omega / d y0).  The FP32 gap comes from
    the FP32 forward states the tape holds, around which the step map is
    linearised: holding the adjoint populations in FP64 instead of FP32
    leaves both errors unchanged (measured)."""
    gold, out, gy, gw = _couette_256x64(storage)
    print("final", out[0, :6], "oracle y", gold["y"], "omega", gold["omega"])
    bad = []
    for k, name in enumerate(("y0", "theta0", "AR", "U")):
        g = gold["grad"][name]
        assert g is not None, name
        for key, val in (("y", gy[k]), ("omega", gw[k])):
            ref = g[key]
            unc = 0.75 * abs(g[key + "_central_h"] - ref)
            err = abs(val - ref) / abs(ref)
            print(f"{storage} d{key}/d{name}: adjoint {val: .10e} fd {ref: .10e} (h={g['h']:g}) rel {err:.2e}"
                  f" fd-unc {unc / abs(ref):.1e}")
            if abs(val - ref) > tol * abs(ref) + 2 * unc:
                bad.append((key, name, val, ref, err))
    assert not bad, bad


# ---------------------------------------------------------------------------
# Several particles and channels: neighbour lists (overlapping adjoint
# patches), shared tiles, batched channels.
# ---------------------------------------------------------------------------
def _multi():
    ch0 = C.couette_config(48, 30, tau=0.8, storage=0)
    ch0["gravity"] = [0.0, -2e-6]
    e = shapes.ellipse(8.0, 2.0, n_markers=20, mode="param")
    ci = shapes.circle(6.0, n_markers=18)
    # bodies 4 lu apart: the probe stencils of each reach the other's patch
    p0 = [C.particle(e, 15.2, 14.3, 0.2, density_ratio=1.2, u=0.001),
          C.particle(ci, 26.1, 15.6, 0.0, density_ratio=1.1, v=0.0005)]
    ch1 = C.base_config(24, 32, tau=0.8, bc_x=1, u_wall=[[0.0, 0.01], [0.0, -0.02], [0.0, 0.0], [0.0, 0.0]],
                        body_force=[0.0, 1e-5], storage=0)
    p1 = [C.particle(shapes.square(7.0), 11.7, 16.4, 0.1, density_ratio=1.3, omega=0.001)]
    return [(ch0, p0), (ch1, p1)]


def _gpu_adjoint_channels(chans, T, seeds):
    from paper_1606_01805_amd import Solver

    s = Solver(chans)
    s.checkpoint_save(0)
    s.step(T, record=False)
    s.adjoint_begin(seeds, T)
    s.adjoint_segment(0, T)
    part, mk, wall = s.adjoint_gradients()
    lam = [s.adjoint_field(ci) for ci in range(len(chans))]
    s.close()
    return part, mk, wall, lam


def test_batched_multi_particle_adjoint_matches_fd_and_alone():
    chans = _multi()
    T = 10
    rng = np.random.default_rng(21)
    npart = sum(len(p) for _, p in chans)
    seeds = np.zeros((npart, 10))
    seeds[:, :6] = rng.standard_normal((npart, 6))
    part, mk, wall, lam = _gpu_adjoint_channels(chans, T, seeds)
    # batched == each channel alone, bitwise
    o = 0
    for ci, (cfg, ps) in enumerate(chans):
        pa, mka, wa, la = _gpu_adjoint_channels([(cfg, ps)], T, seeds[o:o + len(ps)])
        assert np.array_equal(pa, part[o:o + len(ps)])
        for j in range(len(ps)):
            assert np.array_equal(mka[j], mk[o + j])
        assert np.array_equal(wa[0], wall[ci])
        assert np.array_equal(la[0], lam[ci])
        o += len(ps)
    # against the oracle, channel by channel (the channels are independent;
    # J of a channel is the seed-weighted sum over its particles)
    bad = []
    o = 0
    for ci, (cfg, ps) in enumerate(chans):
        c = seeds[o:o + len(ps), :6]

        def objective(cf, pp, f0=None):
            import oracle

            orc = oracle.Oracle(cf)
            for p in pp:
                orc.add_particle(p)
            orc.step(T, record=False)
            return float((c * orc.particles()[:, :6]).sum()), orc.anchor_hash()

        def deriv(perturb):
            import copy

            for h in (1e-3, 1e-4, 1e-5, 1e-6):
                vals = []
                for e in (-h, -h / 2, h / 2, h):
                    cf, pp = copy.deepcopy(cfg), copy.deepcopy(ps)
                    perturb(cf, pp, e)
                    vals.append(objective(cf, pp))
                if len({v[1] for v in vals}) == 1:
                    d1 = (vals[3][0] - vals[0][0]) / (2 * h)
                    d2 = (vals[2][0] - vals[1][0]) / h
                    return (4 * d2 - d1) / 3
            return None

        for j in range(len(ps)):
            g = part[o + j]
            for name, key, val in (("x0", "x", g[0] + g[2]), ("y0", "y", g[1] + g[3]),
                                   ("theta0", "theta", g[4] + g[5]), ("omega0", "omega", g[10] + g[11])):
                def pert(cf, pp, e, j=j, key=key):
                    pp[j][key] = float(pp[j][key]) + e
                fd = deriv(pert)
                assert fd is not None, (ci, j, name)
                print(f"ch{ci} p{j} {name:7s} adjoint {val: .10e} fd {fd: .10e}")
                if abs(val - fd) > TOL_R * abs(fd) + TOL_A:
                    bad.append((ci, j, name, val, fd))

            def pert_xi(cf, pp, e, j=j):
                a = np.array(pp[j]["xi"], dtype=np.float64).copy()
                a[3, 1] += e
                pp[j]["xi"] = a
            fd = deriv(pert_xi)
            print(f"ch{ci} p{j} xi[3].y  adjoint {mk[o + j][3, 1]: .10e} fd {fd: .10e}")
            if abs(mk[o + j][3, 1] - fd) > TOL_R * abs(fd) + TOL_A:
                bad.append((ci, j, "xi[3].y", mk[o + j][3, 1], fd))
        o += len(ps)
    assert not bad, bad


@pytest.mark.parametrize("storage", [C.STORE_F64, C.STORE_F32, C.STORE_F16S])
def test_fused_adjoint_launches_bitwise(storage):
    """When no channel holds more than one particle, a reversed step runs its
    two particle kernels as one launch (adj_fused = 1), or the whole step,
    lattice included, as one launch (adj_fused = 2, the default, used when
    its workgroups fit the device at once, as here).  Gradients and adjoint
    populations are bitwise those of the three launches (adj_fused = 0):
    four channels of one particle each, one of them of 120 markers (three
    rounds of 56 in the adjoint kernels), one with side walls, gravity and a
    body force, one whose particle straddles the periodic seam (its adjoint
    box wraps)."""
    from paper_1606_01805_amd import Solver

    ch0 = C.couette_config(64, 40, tau=0.8, storage=0)
    ch0["gravity"] = [0.0, -2e-6]
    ch1 = C.couette_config(48, 30, tau=0.7, storage=0)
    ch2 = C.base_config(24, 32, tau=0.8, bc_x=1, u_wall=[[0.0, 0.01], [0.0, -0.02], [0.0, 0.0], [0.0, 0.0]],
                        body_force=[0.0, 1e-5], storage=0)
    ch3 = C.couette_config(40, 28, tau=0.9, storage=0)
    chans = [(ch0, [C.particle(shapes.ellipse(16.0, 2.0, n_markers=120, mode="param"), 30.3, 19.6, 0.4,
                               density_ratio=1.2, u=0.001)]),
             (ch1, [C.particle(shapes.circle(8.0, n_markers=30), 20.6, 15.2, 0.0, density_ratio=1.1, v=0.0005)]),
             (ch2, [C.particle(shapes.square(7.0), 11.7, 16.4, 0.1, density_ratio=1.3, omega=0.001)]),
             (ch3, [C.particle(shapes.ellipse(8.0, 2.0, n_markers=20, mode="param"), 1.4, 13.8, 0.3,
                               density_ratio=1.1, u=0.002)])]
    T = 12
    seeds = np.zeros((len(chans), 10))
    seeds[:, :6] = np.random.default_rng(31).standard_normal((len(chans), 6))

    def run(mode):
        s = Solver(chans, storage=storage, tuning=dict(adj_fused=mode))
        assert s.tuning()["adj_fused"] == mode
        s.checkpoint_save(0)
        s.step(T, record=False)
        s.adjoint_begin(seeds, T)
        s.adjoint_segment(0, T)
        part, mk, wall = s.adjoint_gradients()
        lam = [s.adjoint_field(ci) for ci in range(len(chans))]
        s.close()
        return part, mk, wall, lam

    ref = run(0)
    assert np.all(np.isfinite(ref[0])) and np.any(ref[0] != 0.0)
    for mode in (1, 2):
        got = run(mode)
        assert np.array_equal(got[0], ref[0]), mode
        for j in range(len(chans)):
            assert np.array_equal(got[1][j], ref[1][j]), (mode, j)
            assert np.array_equal(got[2][j], ref[2][j]), (mode, j)
            assert np.array_equal(got[3][j], ref[3][j]), (mode, j)


def test_fused_adjoint_launch_forms_edge_cases():
    """The launch forms of a reversed step stay bitwise equal with a channel
    that holds no particle (its lattice is updated by the lattice
    workgroups alone) and on a lattice too large for the whole step to fit
    the device in one pass (adj_fused = 2 then runs as 1)."""
    from paper_1606_01805_amd import Solver

    ch0 = C.couette_config(48, 30, tau=0.7, storage=0)
    ch1 = C.couette_config(40, 24, tau=0.9, storage=0)
    small = [(ch0, [C.particle(shapes.circle(8.0, n_markers=30), 20.6, 15.2, 0.0, density_ratio=1.1)]),
             (ch1, [])]
    big = [(C.couette_config(1024, 300, tau=0.8, storage=0),
            [C.particle(shapes.ellipse(16.0, 2.0, n_markers=60, mode="param"), 500.3, 150.6, 0.2)])]
    for chans, T in ((small, 10), (big, 4)):
        npart = sum(len(p) for _, p in chans)
        seeds = np.zeros((npart, 10))
        seeds[:, :6] = np.random.default_rng(41).standard_normal((npart, 6))

        def run(mode):
            s = Solver(chans, storage=C.STORE_F32, tuning=dict(adj_fused=mode))
            s.checkpoint_save(0)
            s.step(T, record=False)
            s.adjoint_begin(seeds, T)
            s.adjoint_segment(0, T)
            part, mk, wall = s.adjoint_gradients()
            lam = [s.adjoint_field(ci) for ci in range(len(chans))]
            s.close()
            return part, mk, wall, lam

        ref = run(0)
        assert np.any(ref[0] != 0.0)
        for mode in (1, 2):
            got = run(mode)
            assert np.array_equal(got[0], ref[0]), mode
            for j in range(len(ref[1])):
                assert np.array_equal(got[1][j], ref[1][j]), mode
            for ci in range(len(chans)):
                assert np.array_equal(got[2][ci], ref[2][ci]), mode
                assert np.array_equal(got[3][ci], ref[3][ci]), mode


@pytest.mark.parametrize("storage,overlap", [(C.STORE_F32, 0), (C.STORE_F32, 1), (C.STORE_F64, 0)])
def test_adjoint_sweep_equals_segments(storage, overlap):
    """lbm_adjoint_sweep (the next segment recomputed on a second stream
    beside the reversal of the current one, two tapes) gives bitwise the
    gradients, adjoint populations and final forward state of
    lbm_adjoint_segment called segment by segment: five segments, two
    particles, with and without the combined forward launch."""
    cfg = C.couette_config(96, 40, storage=storage)
    parts = [C.particle(shapes.ellipse(10.0, 2.0, n_markers=40), 30.2, 20.4, 0.7),
             C.particle(shapes.circle(8.0, n_markers=30), 66.8, 17.9, 0.0)]
    tun = dict(tile_w=64, rows_per_thread=1, overlap=1) if overlap else None
    c = [0.3, 1.0, 0.2, 0.5, -0.4, 1.0]
    a = gpu_adjoint(cfg, parts, 150, c, seg=30, storage=storage, tuning=tun, sweep=False, all_parts=True)
    b = gpu_adjoint(cfg, parts, 150, c, seg=30, storage=storage, tuning=tun, sweep=True, all_parts=True)
    for x, y in zip(a, b):
        if isinstance(x, list):
            for u, v in zip(x, y):
                assert np.array_equal(u, v)
        else:
            assert np.array_equal(x, y)


def test_repeated_adjoints_on_one_handle_bitwise():
    """A second adjoint of the same length on one handle keeps the first's
    tapes; one of another length allocates new ones.  Every run from the
    same checkpoints gives bitwise the same gradients and adjoint
    populations, with the sweep and segment by segment."""
    from paper_1606_01805_amd import Solver

    cfg = C.couette_config(96, 40, storage=C.STORE_F32)
    parts = [C.particle(shapes.ellipse(10.0, 2.0, n_markers=40), 30.2, 20.4, 0.7)]
    s = Solver([(cfg, parts)])
    for k in range(4):
        s.checkpoint_save(k)
        s.step(15, record=False)
    s.checkpoint_save(4)
    seed = np.zeros((1, 10))
    seed[0, :6] = [0.3, 1.0, 0.2, 0.5, -0.4, 1.0]

    def grad(seg, sweep):
        s.checkpoint_restore(4)
        s.adjoint_begin(seed, seg)
        if seg == 15:
            slots = [3, 2, 1, 0]
            if sweep:
                s.adjoint_sweep(slots, 15)
            else:
                for k in slots:
                    s.adjoint_segment(k, 15)
        else:
            s.adjoint_segment(0, 60)
        part, mk, wall = s.adjoint_gradients()
        return part, mk[0], wall[0], s.adjoint_field(0)

    runs = [grad(15, True), grad(15, True), grad(15, False), grad(60, False), grad(15, True)]
    s.close()
    for r in runs[1:]:
        for x, y in zip(runs[0], r):
            assert np.array_equal(x, y)


def test_adjoint_sweep_rejects_bad_schedules():
    """lbm_adjoint_sweep checks the whole chain of checkpoints before any
    work: an empty list, a slot out of order or a segment longer than the
    tape are rejected and leave the adjoint where it was."""
    from paper_1606_01805_amd import LBMError, Solver

    cfg = C.couette_config(64, 32)
    parts = [C.particle(shapes.circle(8.0, n_markers=30), 30.2, 15.4, 0.0)]
    s = Solver([(cfg, parts)])
    for k in range(3):
        s.checkpoint_save(k)
        s.step(10, record=False)
    s.adjoint_begin(np.ones((1, 10)), 10)
    with pytest.raises(LBMError, match="EINVAL"):
        s.adjoint_sweep([], 10)
    with pytest.raises(LBMError, match="ESTATE"):
        s.adjoint_sweep([2, 0, 1], 10)  # slot 0 does not end where slot 2 starts
    with pytest.raises(LBMError, match="EINVAL"):
        s.adjoint_sweep([2, 1, 0], 11)  # longer than the tape
    assert s.adjoint_position == 30
    s.adjoint_sweep([2, 1, 0], 10)
    assert s.adjoint_position == 0
    s.close()
