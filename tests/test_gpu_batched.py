"""Batched form: many uneven channels advanced by single launches per kernel
phase.  Each channel must equal the same channel run alone, bit for bit, and
the oracle within the FP64 bar; full-size workloads are checked on sampled
outputs."""
import numpy as np
import pytest

import oracle
from workloads import configs as C
from workloads import shapes

from gpu_util import body_size, run_gpu, run_oracle, series_errors

pytestmark = pytest.mark.gpu


def _small_ensemble(storage, n=6):
    wl = C.ensemble(storage=storage, n_channels=n, seed=99)
    # shrink to test sizes: keep the particle, scale the channel to H = 48..96
    chans = []
    rng = np.random.default_rng(5)
    for k, (cfg, parts) in enumerate(wl.channels):
        H = int(rng.choice([32, 40, 48, 56]))
        c = C.couette_config(4 * H + k, H, storage=storage)  # ragged widths
        sh = C.random_shape(rng, 0.25 * H)
        rb = shapes.bounding_radius(sh)
        y = float(np.clip(rng.uniform(0.2, 0.8) * (H - 1), rb + 6, H - 1 - rb - 6))
        chans.append((c, [C.particle(sh, rng.uniform(0, 4 * H), y, rng.uniform(0, 6.28))]))
    chans.append((C.couette_config(70, 20, storage=storage), []))  # a channel with no particle
    return chans


@pytest.mark.parametrize("storage", [C.STORE_F32, C.STORE_F16S, C.STORE_F64])
def test_batched_equals_each_channel_alone(storage):
    chans = _small_ensemble(storage)
    s, g = run_gpu(chans, 200)
    s.close()
    pid = 0
    for cfg, parts in chans:
        if not parts:
            continue
        s1, g1 = run_gpu([(cfg, parts)], 200)
        s1.close()
        # identical except the channel-index column of the record
        assert np.array_equal(g[:, pid, :9], g1[:, 0, :9])
        assert np.all(g[:, pid, 9] == chans.index((cfg, parts)))
        pid += 1


def test_batched_fp64_matches_oracle():
    chans = _small_ensemble(C.STORE_F64, n=4)
    s, g = run_gpu(chans, 300)
    s.close()
    pid = 0
    for cfg, parts in chans:
        if not parts:
            continue
        _, r = run_oracle(cfg, parts, 300)
        e = series_errors(g[:, pid], r[:, 0], body_size(parts[0]))
        assert max(e.values()) < 1e-12, e
        pid += 1


def _multi_round_channels(storage):
    """Particles of 2 to 4 rounds of 64 markers (dense circles and ellipses),
    one or two per channel, so the particle kernels run several workgroups
    per particle and workgroup and particle indices differ."""
    chans = []
    specs = [(48, [(shapes.circle(12.0, n_markers=150), 40.3, 23.6, 0.0)]),
             (40, [(shapes.ellipse(14.0, 2.0, n_markers=70), 25.2, 19.1, 0.6),
                   (shapes.circle(10.0, n_markers=201), 90.7, 20.4, 0.0)]),
             (36, [(shapes.circle(8.0, n_markers=64), 60.0, 17.2, 0.0)]),
             (44, [(shapes.ellipse(16.0, 2.5, n_markers=256), 100.5, 22.3, 1.1)])]
    for k, (H, ps) in enumerate(specs):
        cfg = C.couette_config(4 * H + 3 * k, H, storage=storage)
        chans.append((cfg, [C.particle(sh, x, y, th) for sh, x, y, th in ps]))
    return chans


@pytest.mark.parametrize("storage", [C.STORE_F32, C.STORE_F64])
def test_batched_multi_round_particles(storage):
    """Several particles of several rounds in one handle: bitwise each channel
    alone (FP32, FP64) and bitwise with the combined launch, and the oracle
    within the FP64 bar."""
    chans = _multi_round_channels(storage)
    s, g = run_gpu(chans, 120)
    s.close()
    # the surface stress beside the lattice pass in one launch: bitwise the
    # same, in the per-node form (576-thread workgroups) and in the vector
    # form (256-thread workgroups: each thread takes three probe pairs in
    # turn, and the last round's workgroup sums the published terms in
    # stages of 85 markers)
    s2, g2 = run_gpu(chans, 120, tuning=dict(overlap=1, tile_w=64, rows_per_thread=2))
    s2.close()
    assert np.array_equal(g, g2)
    tw = 128 if storage == C.STORE_F64 else 256
    s3, g3 = run_gpu(chans, 120, tuning=dict(overlap=1, vec=1, tile_w=tw, rows_per_thread=1))
    s3.close()
    assert np.array_equal(g, g3)
    pid = 0
    for ci, (cfg, parts) in enumerate(chans):
        s1, g1 = run_gpu([(cfg, parts)], 120)
        s1.close()
        n = len(parts)
        assert np.array_equal(g[:, pid:pid + n, :9], g1[:, :, :9]), ci
        if storage == C.STORE_F64:
            _, r = run_oracle(cfg, parts, 120)
            for k in range(n):
                e = series_errors(g[:, pid + k], r[:, k], body_size(parts[k]))
                assert max(e.values()) < 1e-12, (ci, k, e)
        pid += n


def test_batched_persistent_grid_bitwise():
    chans = _small_ensemble(C.STORE_F32)
    _, a = run_gpu(chans, 120)
    _, b = run_gpu(chans, 120, tuning=dict(persistent_wgs=64, tile_w=128, rows_per_thread=2))
    assert np.array_equal(a, b)


def test_batched_combined_launch_bitwise():
    """Channels of uneven size with the lattice pass and the surface stress in
    one launch: bitwise the separate launches."""
    chans = _small_ensemble(C.STORE_F32)
    _, a = run_gpu(chans, 120)
    for remap in (0, 1):
        _, b = run_gpu(chans, 120, tuning=dict(overlap=1, tile_w=64, rows_per_thread=1, xcd_remap=remap))
        assert np.array_equal(a, b)


def test_full_ensemble_sampled_channels():
    """The 256-channel ensemble at full size, in the launch configuration of
    the benchmark: every particle record is finite, and 4 sampled channels
    match the oracle over the first 20 steps (FP32 vs FP64 oracle)."""
    from bench import VARIANT_TUNING

    wl = C.ensemble(storage=C.STORE_F32)
    steps = 20
    s, g = run_gpu(wl.channels, steps, tuning=VARIANT_TUNING["ensemble"])
    s.close()
    assert np.isfinite(g).all()
    for ch in (0, 77, 150, 255):
        cfg, parts = wl.channels[ch]
        _, r = run_oracle(dict(cfg, storage=C.STORE_F64), parts, steps)
        e_pos = np.abs(g[:, ch, 0:2] - r[:, 0, 0:2]).max() / (cfg["ny"] - 1)
        assert e_pos < 1e-6, (ch, e_pos)
        assert np.abs(g[:, ch, 9] - ch).max() == 0


def test_full_ensemble_equals_its_halves():
    """The full ensemble at full size in the benchmark's launch shape: its
    566 rounds of 64 markers take more than the 512 workgroups that two per
    CU hold on a 256-CU part, so its particle kernels run in two batches,
    while each half of it (under 512 rounds) runs in one.  The particle
    records of every channel are bitwise those of the half it belongs to."""
    from bench import VARIANT_TUNING

    wl = C.ensemble(storage=C.STORE_F32)
    rounds = sum((len(p["xi"]) + 63) // 64 for _, ps in wl.channels for p in ps)
    assert rounds > 512, rounds
    steps = 30
    s, g = run_gpu(wl.channels, steps, tuning=VARIANT_TUNING["ensemble"])
    s.close()
    for lo, hi in ((0, 128), (128, 256)):
        half = wl.channels[lo:hi]
        assert sum((len(p["xi"]) + 63) // 64 for _, ps in half for p in ps) <= 512
        s, h = run_gpu(half, steps, tuning=VARIANT_TUNING["ensemble"])
        s.close()
        assert np.array_equal(g[:, lo:hi, :9], h[:, :, :9]), (lo, hi)


# FP16S keeps about 11 bits of each scaled deviation: velocities carry a
# relative error of order 1e-5 (|u| <= 0.05), i.e. about 1e-6 lattice units
# of displacement over 3 steps, against 1e-8 for FP32.
@pytest.mark.parametrize("storage,key,tol_pos,tol_f",
                         [(C.STORE_F32, "large", 1e-8, 1e-4), (C.STORE_F16S, "large16", 1e-6, 1e-2)])
def test_full_large_domain_sampled_steps(storage, key, tol_pos, tol_f):
    """4096 x 1024 with 64 particles in the benchmark's launch configuration
    (FP32 and FP16S storage): 3 steps against the FP64 oracle, every
    particle."""
    from bench import VARIANT_TUNING

    wl = C.large(storage=storage)
    cfg, parts = wl.channels[0]
    steps = 3
    s, g = run_gpu(wl.channels, steps, tuning=VARIANT_TUNING[key])
    s.close()
    _, r = run_oracle(dict(cfg, storage=C.STORE_F64), parts, steps)
    e_pos = np.abs(g[..., 0:2] - r[..., 0:2]).max()
    e_F = np.abs(g[..., 6:8] - r[..., 6:8]).max() / np.abs(r[..., 6:8]).max()
    assert e_pos < tol_pos and e_F < tol_f, (e_pos, e_F)


@pytest.mark.parametrize("storage,tw,overlap", [(C.STORE_F32, 256, 0), (C.STORE_F16S, 512, 0), (C.STORE_F64, 128, 0),
                                                (C.STORE_F32, 256, 1), (C.STORE_F16S, 256, 1), (C.STORE_F64, 128, 1),
                                                (C.STORE_F32, 64, 1), (C.STORE_F16S, 512, 1)])
def test_vector_form_coupled_bitwise(storage, tw, overlap):
    """Batched uneven channels with particles: the vector form of the lattice
    pass gives bitwise the trajectories and populations of the per-node
    form (the IB force added per node, several particles per tile), also in
    the combined launch with the surface stress (overlap = 1: the same tiles
    in 256-thread workgroups, a round's 576 probe pairs on 256 threads)."""
    chans = _small_ensemble(storage)
    s0, g0 = run_gpu(chans, 120)
    p0 = [s0.populations(k) for k in range(len(chans))]
    s0.close()
    rows = 1 if overlap else 2
    s1, g1 = run_gpu(chans, 120, tuning=dict(vec=1, tile_w=tw, rows_per_thread=rows, nt_store=1, overlap=overlap))
    p1 = [s1.populations(k) for k in range(len(chans))]
    s1.close()
    assert np.array_equal(g0, g1)
    for a, b in zip(p0, p1):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("storage,key", [(C.STORE_F32, "huge"), (C.STORE_F16S, "huge16")])
def test_full_huge_domain_launch_shape_bitwise(storage, key):
    """The 8192 x 4096 domain with 64 particles in the benchmark's launch
    shape (vector tiles, nontemporal stores, the surface stress in the same
    launch) gives bitwise the particle records of the library's default
    shape (per-node tiles, separate launches) over 10 steps."""
    from bench import VARIANT_TUNING, make_workload

    wl = make_workload("huge", storage)
    s, g = run_gpu(wl.channels, 10, tuning=VARIANT_TUNING[key])
    s.close()
    s, h = run_gpu(wl.channels, 10)
    s.close()
    assert np.isfinite(g).all()
    assert np.array_equal(g, h)
