"""GPU coupled step (lattice + MLS-IBM + surface stress + BDF2) vs the oracle.

Comparison metric: for every series of the particle record (x, y, theta, u,
v, omega, Fx, Fy, M) the largest absolute difference over the run, divided by
the natural scale of its group in the oracle run (largest displacement for
x, y; displacement / size for theta; largest speed for u, v; speed / size for
omega; largest force for Fx, Fy; force x size for M).  Dividing a series by
its own maximum would make symmetric-zero series (e.g. the sideways motion of
a sedimenting circle) pure rounding noise.

FP64 bar: 1e-12 (the Couette, periodic-seam, polygon, overlapping-particle,
multi-round and alternative-kernel cases; both sides sum the spread in the
order of reading R20, so only the device's exp/cos/sin, which may differ
from the host's by one ulp, separate them).  The sedimentation case is
ill-conditioned in that respect: the fluid is nearly at rest, every
population near w_i carries absolute rounding noise of ~3e-17, so the density
near 1 that gives the pressure (rho - 1)/3 is held to ~1e-16 absolute against
pressure variations of ~1e-7, and a one-ulp change of a single kernel weight
anywhere moves the surface force by ~3e-10 of itself.  Measured on the oracle
alone (every exponential weight nudged by one ulp, 2000 steps): force 2.7e-10,
velocity 1.5e-11, position 7.4e-12.  The sedimentation bars are 1e-9 for
forces and 5e-11 for kinematics.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import configs as C
from workloads import shapes

from gpu_util import body_size, run_gpu, run_oracle, series_errors

pytestmark = pytest.mark.gpu


def _compare(wl_channels, steps, storage=None, tuning=None):
    s, g = run_gpu(wl_channels, steps, storage=storage, tuning=tuning)
    errs = []
    pid = 0
    for cfg, parts in wl_channels:
        cfg = dict(cfg)
        if storage is not None:
            cfg["storage"] = storage
        _, r = run_oracle(cfg, parts, steps)
        for k, p in enumerate(parts):
            errs.append(series_errors(g[:, pid + k], r[:, k], body_size(p)))
        pid += len(parts)
    s.close()
    return errs


def test_couette_fp64_parity():
    wl = C.couette(storage=C.STORE_F64)
    errs = _compare(wl.channels, 2000)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


def test_sedimentation_fp64_parity():
    wl = C.sedimentation()
    errs = _compare(wl.channels, 2000)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    for k in ("x", "y", "theta", "u", "v", "omega"):
        assert errs[k] < 5e-11, (k, errs)
    for k in ("Fx", "Fy", "M"):
        assert errs[k] < 1e-9, (k, errs)


def test_particle_across_periodic_edge_fp64():
    """A particle straddling x = 0 of a periodic channel: stencils, probes and
    the force patch wrap."""
    cfg = C.couette_config(90, 40, storage=C.STORE_F64)
    sh = shapes.ellipse(12.0, 2.0, n_markers=36)
    p = C.particle(sh, 1.3, 13.0, 0.7, u=-0.02)
    errs = _compare([(cfg, [p])], 600)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


def test_three_particles_with_overlapping_patches_fp64():
    cfg = C.couette_config(120, 60, storage=C.STORE_F64)
    a = C.particle(shapes.circle(10.0, n_markers=32), 40.2, 30.1, 0.0)
    b = C.particle(shapes.square(9.0), 53.7, 31.4, 0.3)       # patch overlaps a's
    c = C.particle(shapes.triangle(10.0), 90.0, 22.0, 1.0)
    errs = _compare([(cfg, [a, b, c])], 400)
    print([{k: f"{v:.1e}" for k, v in e.items()} for e in errs])
    for e in errs:
        assert max(e.values()) < 1e-12, errs


@pytest.mark.parametrize("fam", ["square", "triangle", "rectangle"])
def test_polygon_shapes_fp64(fam):
    cfg = C.couette_config(100, 48, storage=C.STORE_F64)
    sh = shapes.make(fam, 14.0, aspect_ratio=3.0)
    errs = _compare([(cfg, [C.particle(sh, 50.0, 21.3, 0.4)])], 500)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


def test_dense_markers_fp64():
    """Markers 0.3 lattice units apart, as in the paper (Sec. 2.1): each node
    receives force from many markers."""
    cfg = C.couette_config(80, 40, storage=C.STORE_F64)
    sh = shapes.circle(10.0, n_markers=105)
    errs = _compare([(cfg, [C.particle(sh, 40.0, 19.2, 0.0)])], 300)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


@pytest.mark.parametrize("kernel", [1, 2, 3, 4])
def test_alternative_kernels_fp64(kernel):
    """Cubic, quartic, cosine and polynomial weights (Sec. 2.2, Eqs. (17)-(20))."""
    cfg = C.couette_config(80, 40, storage=C.STORE_F64, mls_kernel=kernel)
    sh = shapes.ellipse(14.0, 2.0, n_markers=40)
    errs = _compare([(cfg, [C.particle(sh, 40.0, 19.2, 0.5)])], 300)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs


def _traj_errors(g, r, ny):
    """Trajectory error of a reduced form: positions over the wall gap,
    angle in radians, angular velocity over the shear rate."""
    shear = 2 * couette_u(ny) / (ny - 1)
    e_pos = np.abs(g[..., 0:2] - r[..., 0:2]).max() / (ny - 1)
    e_th = np.abs(g[..., 2] - r[..., 2]).max()
    e_om = np.abs(g[..., 5] - r[..., 5]).max() / shear
    return e_pos, e_th, e_om


def couette_u(ny):
    return C.couette_speed(ny)


def _bench_tuning(name):
    from bench import WORKLOAD_TUNING

    return WORKLOAD_TUNING[name]


@pytest.mark.parametrize("storage,tol,launch", [(C.STORE_F32, 1e-4, "default"), (C.STORE_F16S, 1e-2, "default"),
                                                (C.STORE_F32, 1e-4, "bench")])
def test_couette_reduced_forms_trajectory_error(storage, tol, launch):
    """The benchmark workload (400x100 Couette, Re 20, one ellipse) over 5000
    steps against the FP64 oracle, in the library's default launch shape and
    in the one bench.py times (lattice pass and surface stress combined)."""
    wl = C.couette(storage=storage)
    cfg, parts = wl.channels[0]
    steps = 5000
    s, g = run_gpu(wl.channels, steps, tuning=_bench_tuning("couette") if launch == "bench" else None)
    s.close()
    cfg64 = dict(cfg, storage=C.STORE_F64)
    _, r = run_oracle(cfg64, parts, steps)
    e = _traj_errors(g, r, cfg["ny"])
    print(storage, e)
    assert max(e) < tol, e


def test_determinism_and_graph_vs_eager():
    """Runs are bitwise reproducible, and neither graph replay nor the
    combined lattice / surface-stress launch (any rows, either tile order)
    changes a bit."""
    wl = C.couette(storage=C.STORE_F32)
    _, a = run_gpu(wl.channels, 301)
    _, b = run_gpu(wl.channels, 301)
    _, c = run_gpu(wl.channels, 301, tuning=dict(use_graph=0))
    xs = [b, c]
    for rows in (1, 2, 4):
        for remap in (0, 1):
            xs.append(run_gpu(wl.channels, 301, tuning=dict(overlap=1, tile_w=64, rows_per_thread=rows,
                                                            xcd_remap=remap))[1])
    xs.append(run_gpu(wl.channels, 301, tuning=dict(overlap=1, tile_w=64, use_graph=0))[1])
    for x in xs:
        assert np.array_equal(a, x)


def test_combined_launch_fp64_parity_with_overlapping_patches():
    """The combined lattice / surface-stress launch with three particles, two
    of them with overlapping patches (FP64): oracle parity, and bitwise the
    records of the separate launches."""
    cfg = C.couette_config(120, 60, storage=C.STORE_F64)
    a = C.particle(shapes.circle(10.0, n_markers=32), 40.2, 30.1, 0.0)
    b = C.particle(shapes.square(9.0), 53.7, 31.4, 0.3)
    c = C.particle(shapes.triangle(10.0), 90.0, 22.0, 1.0)
    chans = [(cfg, [a, b, c])]
    tun = dict(overlap=1, tile_w=64, rows_per_thread=2)
    errs = _compare(chans, 400, tuning=tun)
    print([{k: f"{v:.1e}" for k, v in e.items()} for e in errs])
    for e in errs:
        assert max(e.values()) < 1e-12, errs
    _, g = run_gpu(chans, 200, tuning=tun)
    _, h = run_gpu(chans, 200)
    assert np.array_equal(g, h)


def test_wide_rounds_spread_in_groups_fp64():
    """A 120-unit square rotated by 45 degrees with markers 3 apart (160
    markers, 3 rounds): the stencil anchors of each round of 64 markers span
    more than the 3072-cell mask box, so every round spreads in several
    marker groups.  FP64 against the oracle, and FP32 bitwise equal whether
    the channel runs alone or beside another."""
    cfg = C.couette_config(400, 240, storage=C.STORE_F64)
    p = C.particle(shapes.square(120.0, spacing=3.0), 200.3, 120.6, 0.785)
    errs = _compare([(cfg, [p])], 20)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-12, errs
    cfg32 = dict(cfg, storage=C.STORE_F32)
    other = (C.couette_config(96, 48, storage=C.STORE_F32), [C.particle(shapes.circle(10.0), 40.0, 23.4, 0.0)])
    _, g = run_gpu([other, (cfg32, [p])], 20)
    _, h = run_gpu([(cfg32, [p])], 20)
    assert np.array_equal(g[:, 1, :9], h[:, 0, :9])


def test_combined_launch_rejects_other_shapes():
    from paper_1606_01805_amd import Solver

    wl = C.couette(storage=C.STORE_F32)
    s = Solver(wl.channels)
    with pytest.raises(RuntimeError, match="overlap"):
        s.set_tuning(overlap=1, tile_w=256)
    with pytest.raises(RuntimeError, match="overlap"):
        s.set_tuning(overlap=1, tile_w=64, persistent_wgs=16)
    s.set_tuning(overlap=1, tile_w=64)
    s.step(3)
    s.close()


def test_checkpoint_restore_replays_bitwise():
    from paper_1606_01805_amd import Solver

    wl = C.couette(storage=C.STORE_F32)
    s = Solver(wl.channels)
    s.step(50)
    s.checkpoint_save(3)
    a = s.step(120)
    pa = s.populations()
    s.checkpoint_restore(3)
    b = s.step(120)
    assert np.array_equal(a, b) and np.array_equal(pa, s.populations())


def test_unstable_run_is_reported_at_the_oracle_step():
    from paper_1606_01805_amd import LBMError, Solver

    cfg = C.base_config(40, 24, tau=0.51, bc_y=1)
    p = C.particle(shapes.circle(6.0, n_markers=20), 20.0, 12.0, 0.0, 1.0, u=5.0)
    s = Solver([(cfg, [p])])
    with pytest.raises(LBMError, match="LBM_EUNSTABLE.*step 2 "):
        s.step(100)
    o = oracle.Oracle(cfg)
    o.add_particle(p)
    with pytest.raises(FloatingPointError, match="step 2"):
        o.step(100)


def test_closed_box_sedimentation_fp64():
    """A circle settling in a closed box (walls on both axes, the corner
    closure of reading R23): FP64 parity over 1500 steps at the sedimentation
    bars (the flow is nearly at rest, see the module docstring)."""
    cfg = C.base_config(40, 90, tau=0.8, bc_x=1, bc_y=1, gravity=[0.0, -2e-5])
    p = C.particle(shapes.circle(10.0, n_markers=32), 20.0, 60.0, 0.0, 1.05)
    errs = _compare([(cfg, [p])], 1500)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    for k in ("x", "y", "theta", "u", "v", "omega"):
        assert errs[k] < 5e-11, (k, errs)
    for k in ("Fx", "Fy", "M"):
        assert errs[k] < 1e-9, (k, errs)


def test_particle_near_box_corner_fp64():
    """A particle thrown toward a corner of a closed box: its probe stencils
    reach the wall column (the particle kernels apply the wall and corner
    closures to the nodes they pull)."""
    cfg = C.base_config(36, 30, tau=0.9, bc_x=1, bc_y=1, gravity=[-3e-5, -3e-5])
    p = C.particle(shapes.circle(8.0, n_markers=26), 7.05, 7.1, 0.0, 1.2, u=-0.04, v=-0.04)
    errs = _compare([(cfg, [p])], 200)[0]
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-11, errs
