#!/usr/bin/env python3
"""Throughput of the fused D2Q9 + MLS-IBM step on one MI355X.

A step is one pass of the whole hot path: immersed-boundary force and
spreading, the lattice pass (streaming, walls, forced collision) and the
surface-stress / rigid-body update, for every channel of the workload.

Default workload: the batched ensemble of 256 independent Re = 20 Couette
channels of uneven size (H in {64, 96, 128, 192, 256}, L = 4H, 27.76 M nodes,
one particle of one of the five shape families each), FP32 storage, one
handle replayed from HIP graphs.  Other workloads of the same family:
--workload couette | sedimentation | large | huge | adjoint.

Prints one JSON line: the metric over exactly --steps timed steps, the median
of five more timed repeats, a roofline object for the lattice pass (HIP-event
timing of that kernel alone on the library's stream) and for the whole step,
the library's own copy-kernel ceiling, comparison variants (the plain
single-channel and per-channel forms, FP16S storage, a domain too large for
the Infinity Cache), the adjoint/forward cost, the trajectory errors of the
reduced forms at their workloads' full lengths, and a CPU baseline from the
FP64 oracle on a bounded sample of the workload.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS fused D2Q9+MLS-IBM step (plain vs batched/FP16); adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {0: 144, 1: 72, 2: 36}  # 9 reads + 9 writes per node
STORAGE = {"f64": 0, "f32": 1, "f16s": 2}
STORE_NAME = ["F64", "F32", "F16S"]
DTYPE = {0: "f64", 1: "f32", 2: "f32 (f16 storage)"}
REPEATS = 5

# Launch shapes picked by the autotuner (paper_1606_01805_amd/tune.py) per
# workload and storage form.
WORKLOAD_TUNING = {"couette": dict(tile_w=64, rows_per_thread=1, xcd_remap=0, overlap=1),
                   "sedimentation": dict(tile_w=64, rows_per_thread=1, xcd_remap=0, overlap=1),
                   "ensemble": dict(tile_w=256, rows_per_thread=1, xcd_remap=0, vec=1, nt_store=1, overlap=1)}
VARIANT_TUNING = {"ensemble": dict(tile_w=256, rows_per_thread=1, xcd_remap=0, vec=1, nt_store=1, overlap=1),
                  "large": dict(tile_w=256, rows_per_thread=1, xcd_remap=1, vec=1, overlap=1),
                  "large16": dict(tile_w=256, rows_per_thread=1, xcd_remap=1, vec=1, overlap=1),
                  "huge": dict(tile_w=256, rows_per_thread=1, xcd_remap=0, vec=1, nt_store=1, overlap=1),
                  "huge16": dict(tile_w=512, rows_per_thread=1, xcd_remap=0, vec=1, nt_store=1, overlap=1)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="ensemble",
                    choices=["ensemble", "couette", "sedimentation", "large", "huge", "adjoint"])
    ap.add_argument("--storage", default=None, choices=list(STORAGE))
    ap.add_argument("--plain", action="store_true",
                    help="ensemble only: one handle per channel (per-channel launches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--cpu-channels", type=int, default=8)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--repeats", type=int, default=REPEATS)
    ap.add_argument("--tile-w", type=int, default=None)
    ap.add_argument("--rows", type=int, default=None)
    ap.add_argument("--persistent", type=int, default=None)
    ap.add_argument("--xcd-remap", type=int, default=None)
    ap.add_argument("--overlap", type=int, default=None,
                    help="1: lattice pass and surface stress in one launch (needs --tile-w 64)")
    ap.add_argument("--vec", type=int, default=None,
                    help="1: vector form of the lattice pass (tile_w / 64 nodes per lane)")
    ap.add_argument("--nt-store", type=int, default=None,
                    help="1: nontemporal stores in the vector form")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the lattice launch shape with the project autotuner first")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the comparison workloads, the adjoint leg and the trajectory errors")
    return ap.parse_args()


def default_steps(name):
    return {"ensemble": (1000, 100), "couette": (20000, 2000), "sedimentation": (2000, 200),
            "large": (2000, 200), "huge": (200, 20), "adjoint": (2000, 200)}[name]


def make_workload(name, storage):
    from workloads import configs as C

    if name == "huge":
        return C.large(storage=storage, nx=8192, ny=4096)
    return C.BY_NAME[name](storage=storage)


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def cpu_baseline(wl, n_channels, steps):
    """The FP64 oracle as it stands on the first n_channels channels of the
    workload for `steps` steps: once on one host thread (the form the parity
    tests use), once with its node loops on every host thread available to
    this process (OMP_NUM_THREADS if set, else the CPU count).  The
    immersed-boundary and particle stages of the oracle stay serial."""
    import oracle

    chans = wl.channels[:n_channels]
    nodes = sum(c["nx"] * c["ny"] for c, _ in chans)
    nparts = sum(len(p) for _, p in chans)
    avail = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
    runs = {}
    for th in (1, threads):
        t0 = time.perf_counter()
        for cfg, parts in chans:
            o = oracle.Oracle(dict(cfg, storage=0))
            o.set_threads(th)
            for p in parts:
                o.add_particle(p)
            o.step(steps, record=False)
        runs[th] = time.perf_counter() - t0
    out = {"value": nodes * steps / runs[threads] / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{steps} steps of the first {len(chans)} channels ({nodes} nodes, {nparts} particles) in "
                     f"FP64, node loops on {threads} threads: {runs[threads]:.1f} s",
           "single_thread": {"value": nodes * steps / runs[1] / 1e6, "unit": "MLUPS", "cores": 1,
                             "seconds": runs[1]},
           "host": {"cpu_model": host_cpu(), "os_cpu_count": avail, "threads_used": threads}}
    return out


def kernel_source_sha():
    import hashlib

    h = hashlib.sha1()
    for f in ("lbm_kernels.hip", "lbm_device.h", "lbm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1606_01805_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def measured_traffic(key):
    """HBM bytes per lattice launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a plain
    copy), or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(key)
    if not e or e.get("kernel_source_sha") != kernel_source_sha():
        return None
    return e["bytes_per_launch"]


def roofline(us_lattice, nodes, storage, traffic_key=None, tuning=None, ms_step=None):
    b = nodes * BYTES_PER_LUP[storage]
    ach = b / (us_lattice * 1e-6) / 1e9
    vec = bool(tuning and tuning.get("vec"))
    if tuning and tuning.get("overlap"):
        name = ("lattice_traction_vkernel" if vec else "lattice_traction_kernel") + " (lattice workgroups only)"
    else:
        name = "lattice_vkernel" if vec else "lattice_kernel"
    out = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
           "traffic": measured_traffic(traffic_key) if traffic_key else None,
           "bytes_per_launch": b, "us_per_launch": us_lattice,
           "timing": "HIP events on the library stream around back-to-back launches of the "
                     "kernel alone on a step's tile lists, right after the timed steps (lbm_time_kernels)"}
    if ms_step:
        step_gbs = b / (ms_step * 1e-3) / 1e9
        out["whole_step"] = {"achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS, "ms_per_step": ms_step,
                             "note": "the step's algorithmic bytes over the median step time (all kernels)"}
    return out


def timed_steps(solvers, steps):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps, record=False)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def copy_ceiling(nbytes=1 << 30, reps=20):
    """GB/s of the library's hand-written copy kernel (read + write) over two
    buffers of nbytes: the practical ceiling of an HBM-bound pass."""
    import ctypes

    import torch

    from paper_1606_01805_amd import _lib

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    g = ctypes.c_double()
    st = torch.cuda.current_stream().cuda_stream
    _lib.check(_lib.lib().lbm_measure_copy(b.data_ptr(), a.data_ptr(), nbytes, reps, ctypes.c_void_p(st),
                                           ctypes.byref(g)))
    del a, b
    torch.cuda.synchronize()
    return {"GB/s": g.value, "frac_of_peak": g.value / HBM_PEAK_GBS,
            "what": f"lbm_measure_copy: 16-byte loads/stores, {nbytes >> 20} MiB read + written per launch, "
                    f"average of {reps} launches"}


def run_variant(name, storage, steps, warm, plain=False, tuning=None, traffic_key=None):
    """MLUPS of one comparison workload plus its lattice-kernel roofline."""
    from paper_1606_01805_amd import Solver

    wl = make_workload(name, storage)
    solvers = ([Solver([ch], tuning=tuning) for ch in wl.channels] if plain
               else [Solver(wl.channels, tuning=tuning)])
    for sv in solvers:
        sv.step(warm, record=False)
    dt = timed_steps(solvers, steps)
    out = {"workload": wl.name, "nodes": wl.nodes, "storage": STORE_NAME[storage],
           "launch": "plain (one handle per channel)" if plain else "single handle, HIP graph",
           "steps": steps, "MLUPS": wl.nodes * steps / dt / 1e6, "us_per_step": dt / steps * 1e6}
    if not plain:
        s0 = solvers[0]
        s0.checkpoint_save(7)
        us = s0.time_kernels(200 if wl.nodes < 1_000_000 else 20)
        s0.checkpoint_restore(7)
        out["kernel_us"] = dict(zip(["ibm_force", "lattice", "traction"], [float(v) for v in us]))
        out["tuning"] = s0.tuning()
        out["roofline"] = roofline(float(us[1]), wl.nodes, storage, traffic_key, out["tuning"], dt / steps * 1e3)
    for sv in solvers:
        sv.close()
    return out


def adjoint_leg(storage=1, steps=2000, seg=100, tuning=None):
    """Cost of one reverse-mode gradient on the 256x64 Couette case: the
    checkpointed forward (graph replay, a checkpoint every `seg` steps) and
    the adjoint sweep (every segment recomputed into the tape and reversed),
    per step, and their ratio, with the library's default launch shape or
    `tuning` for both."""
    import torch

    from paper_1606_01805_amd import Solver
    from workloads import configs as C

    wl = C.adjoint_case(storage=storage)
    s = Solver(wl.channels, tuning=tuning)
    nseg = steps // seg
    s.checkpoint_save(nseg + 1)
    s.step(200, record=False)  # warm-up (graphs built)
    s.checkpoint_restore(nseg + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, record=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    seed = [[0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0]]

    def forward_and_adjoint(sweep):
        # the checkpointed forward run, then the gradient: every segment
        # recomputed into a tape and reversed, either one after the other or
        # with the next segment's recomputation beside the current reversal
        s.checkpoint_restore(nseg + 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(nseg):
            s.checkpoint_save(k)
            s.step(seg, record=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.adjoint_begin(seed, seg)
        if sweep:
            s.adjoint_sweep(list(reversed(range(nseg))), seg)
        else:
            for k in reversed(range(nseg)):
                s.adjoint_segment(k, seg)
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1

    forward_and_adjoint(True)  # allocates the second tape
    t_fwd, t_adj = forward_and_adjoint(True)
    _, t_seq = forward_and_adjoint(False)
    s_tuning = s.tuning()
    s.close()
    return {"workload": wl.name, "storage": STORE_NAME[storage], "steps": steps, "segment": seg,
            "tuning": s_tuning,
            "forward_us_per_step": t_plain / steps * 1e6,
            "forward_checkpointed_us_per_step": t_fwd / steps * 1e6,
            "adjoint_us_per_step": t_adj / steps * 1e6,
            "adjoint_over_forward": t_adj / t_plain,
            "adjoint_segments_one_by_one_us_per_step": t_seq / steps * 1e6,
            "adjoint_segments_one_by_one_over_forward": t_seq / t_plain,
            "note": "adjoint time includes recomputing each segment from its checkpoint (lbm_adjoint_sweep: "
                    "the next segment's recomputation beside the current reversal; also timed with "
                    "lbm_adjoint_segment one segment after the other)"}


def trajectory_errors():
    """Trajectory error of FP32 and FP16S storage against the FP64 oracle
    trajectories of tests/golden (written by make_trajectory_golden.py, oracle
    only) over the workloads' full lengths: positions over the wall gap, angle
    in radians, angular velocity over the wall shear rate."""
    from paper_1606_01805_amd import Solver
    from workloads import configs as C

    out = {"metrics": "pos/(NY-1), theta [rad], omega/shear rate; max over kept steps and particles"}
    cases = [("couette_400x100_50k_fp64.npz", "couette", {1: WORKLOAD_TUNING["couette"], 2: WORKLOAD_TUNING["couette"]}),
             ("large_4096x1024_10k_fp64.npz", "large", {1: VARIANT_TUNING["large"], 2: VARIANT_TUNING["large16"]})]
    for fname, name, tun in cases:
        path = os.path.join(ROOT, "tests", "golden", fname)
        if not os.path.exists(path):
            continue
        g = np.load(path)
        steps, ref, total = g["steps"], g["rec"], int(g["total_steps"])
        res = {"steps": total}
        for st in (1, 2):
            wl = C.BY_NAME[name](storage=st)
            cfg = wl.channels[0][0]
            s = Solver(wl.channels, tuning=tun[st])
            tr = s.step(total, record=True)
            s.close()
            run = tr[steps - 1][..., [0, 1, 2, 5]]
            gap = cfg["ny"] - 1
            shear = abs(cfg["u_wall"][3][0] - cfg["u_wall"][2][0]) / gap
            res[STORE_NAME[st]] = {"pos": float(np.abs(run[..., 0:2] - ref[..., 0:2]).max() / gap),
                                   "theta": float(np.abs(run[..., 2] - ref[..., 2]).max()),
                                   "omega": float(np.abs(run[..., 3] - ref[..., 3]).max() / shear)}
        out[name] = res
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the benchmark has no multi-GPU path "
                                   "(the sharding design is described in the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1606_01805_amd import Solver

    steps, warm = default_steps(args.workload)
    steps = args.steps if args.steps is not None else steps
    warm = args.warmup if args.warmup is not None else warm
    storage = STORAGE[args.storage] if args.storage else (0 if args.workload == "sedimentation" else 1)
    wl = make_workload(args.workload, storage)
    tuning = {}
    if args.tile_w:
        tuning["tile_w"] = args.tile_w
    if args.rows:
        tuning["rows_per_thread"] = args.rows
    if args.persistent is not None:
        tuning["persistent_wgs"] = args.persistent
    if args.xcd_remap is not None:
        tuning["xcd_remap"] = args.xcd_remap
    if args.overlap is not None:
        tuning["overlap"] = args.overlap
    if args.vec is not None:
        tuning["vec"] = args.vec
    if args.nt_store is not None:
        tuning["nt_store"] = args.nt_store
    if not tuning and not args.autotune and not args.plain:
        key = args.workload + ("16" if storage == 2 and args.workload in ("large", "huge") else "")
        tuning = dict(WORKLOAD_TUNING.get(args.workload, VARIANT_TUNING.get(key, {})))

    solvers = ([Solver([ch], tuning=tuning) for ch in wl.channels] if args.plain
               else [Solver(wl.channels, tuning=tuning)])
    tune_report = None
    if args.autotune:
        from paper_1606_01805_amd.tune import autotune

        best, res = autotune(solvers[0], cache=None)
        for s in solvers[1:]:
            s.set_tuning(**best)
        tune_report = {k: v * 1e6 for k, v in res.items()}
    # warm-up: graphs of both step parities are captured on the first
    # multi-step call, so no capture falls in the timed region
    for s in solvers:
        s.step(warm, record=False)
    dt = timed_steps(solvers, steps)
    nodes = wl.nodes
    mlups = nodes * steps / dt / 1e6
    reps = [timed_steps(solvers, steps) / steps * 1e3 for _ in range(args.repeats)]
    med = statistics.median(reps) if reps else dt / steps * 1e3

    # Per-kernel device time, HIP events around back-to-back launches of each
    # kernel alone on the library's stream (after the timed region).
    s0 = solvers[0]
    s0.checkpoint_save(7)
    us = s0.time_kernels(args.kernel_reps)
    s0.checkpoint_restore(7)
    names = ["ibm_force", "lattice", "traction"]
    nodes0 = sum(c["nx"] * c["ny"] for c in s0.cfgs)
    key = {("couette", 1): "couette_f32", ("ensemble", 1): "ensemble_f32", ("large", 1): "large_f32",
           ("large", 2): "large_f16s", ("huge", 1): "huge_f32", ("huge", 2): "huge_f16s"}.get((args.workload, storage))
    roof = roofline(float(us[1]), nodes0, storage, key if not args.plain else None, s0.tuning(),
                    med if not args.plain else None)
    k = int(max(range(3), key=lambda i: us[i]))
    if k != 1:
        roof["dominant_by_time"] = names[k]
    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": dt / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[storage], "data": "synthetic",
        "config": {"workload": wl.name, "nodes": nodes, "channels": len(wl.channels),
                   "particles": wl.n_particles, "storage": STORE_NAME[storage],
                   "launch": "plain (per channel)" if args.plain else "single handle, HIP graph",
                   "tuning": s0.tuning()},
        "repeats": {"n": len(reps), "steps_each": steps, "ms_per_step": reps, "median_ms_per_step": med,
                    "median_MLUPS": nodes / (med * 1e-3) / 1e6},
        "kernel_us": dict(zip(names, [float(v) for v in us])),
        "roofline": roof,
    }
    if tune_report:
        out["autotune_us_per_step"] = tune_report
    for sv in solvers:
        sv.close()
    torch.cuda.synchronize()
    out["copy_ceiling"] = copy_ceiling()
    out["roofline"]["frac_of_copy_ceiling"] = roof["achieved"] / out["copy_ceiling"]["GB/s"]
    if not args.no_variants and args.workload == "ensemble":
        # plain vs batched, FP32 vs FP16S, a domain that does not fit the
        # 256 MB Infinity Cache, and the small latency-bound cases
        out["variants"] = [
            run_variant("ensemble", 1, 30, 6, plain=True),
            run_variant("couette", 1, 4000, 400, tuning=WORKLOAD_TUNING["couette"], traffic_key="couette_f32"),
            run_variant("sedimentation", 0, 2000, 200, tuning=WORKLOAD_TUNING["sedimentation"]),
            run_variant("large", 1, 500, 50, tuning=VARIANT_TUNING["large"], traffic_key="large_f32"),
            run_variant("large", 2, 500, 50, tuning=VARIANT_TUNING["large16"], traffic_key="large_f16s"),
            run_variant("huge", 1, 100, 10, tuning=VARIANT_TUNING["huge"], traffic_key="huge_f32"),
            run_variant("huge", 2, 100, 10, tuning=VARIANT_TUNING["huge16"], traffic_key="huge_f16s"),
        ]
        out["adjoint"] = adjoint_leg()
        # the same with the forward step in its fastest launch shape (the
        # surface stress beside the lattice pass), which the recomputation
        # uses too: the adjoint kernels do not change, the forward step does
        out["adjoint_fast_forward"] = adjoint_leg(tuning=WORKLOAD_TUNING["couette"])
        out["trajectory_error"] = trajectory_errors()
    if args.workload == "adjoint":
        out["adjoint"] = adjoint_leg(storage=storage)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_channels, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
