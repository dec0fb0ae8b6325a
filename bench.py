#!/usr/bin/env python3
"""Throughput of the fused D2Q9 + MLS-IBM step on one MI355X.

A step is one pass of the whole hot path: immersed-boundary force and
spreading, the lattice pass (streaming, walls, forced collision) and the
surface-stress / rigid-body update, for every channel of the workload.

Default workload: the Re = 20 Couette channel (400 x 100 lattice, periodic
in x, walls moving at -U/+U, one neutrally buoyant ellipse of aspect ratio 2
and major axis 25 with 64 markers), FP32 storage.  Other workloads of the
same family: --workload sedimentation | ensemble | large | adjoint.

Prints one JSON line with the metric, a roofline object for the dominant
kernel (HIP-event timing of that kernel alone on the library's stream) and a
CPU baseline from the FP64 oracle run on a bounded sample of the workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS fused D2Q9+MLS-IBM step (plain vs batched/FP16); adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {0: 144, 1: 72, 2: 36}  # 9 reads + 9 writes per node
STORAGE = {"f64": 0, "f32": 1, "f16s": 2}
DTYPE = {0: "f64", 1: "f32", 2: "f32 (f16 storage)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="couette",
                    choices=["couette", "sedimentation", "ensemble", "large", "adjoint"])
    ap.add_argument("--storage", default=None, choices=list(STORAGE))
    ap.add_argument("--plain", action="store_true",
                    help="ensemble only: one handle per channel (per-channel launches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB (counter calibration)")
    ap.add_argument("--tile-w", type=int, default=None)
    ap.add_argument("--rows", type=int, default=None)
    ap.add_argument("--persistent", type=int, default=None)
    ap.add_argument("--xcd-remap", type=int, default=None)
    ap.add_argument("--overlap", type=int, default=None,
                    help="1: lattice pass and surface stress in one launch (needs --tile-w 64)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the lattice launch shape with the project autotuner first")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the batched / plain / FP16S comparison runs")
    return ap.parse_args()


def default_steps(name):
    return {"couette": (50000, 2000), "sedimentation": (2000, 200), "ensemble": (1000, 100),
            "large": (2000, 200), "adjoint": (2000, 200)}[name]


def cpu_baseline(wl, seconds):
    """The FP64 oracle as it stands, one host thread, on the first channel of
    the workload for as many steps as fit in about `seconds`.  Its trajectory
    then serves as the reference for the trajectory error of the reduced
    storage forms, run on the GPU for the same steps from the same state."""
    import oracle

    cfg, parts = wl.channels[0]
    cfg = dict(cfg, storage=0)
    o = oracle.Oracle(cfg)
    for p in parts:
        o.add_particle(p)
    nodes = cfg["nx"] * cfg["ny"]
    t0 = time.perf_counter()
    first = o.step(2, record=True)
    per = (time.perf_counter() - t0) / 2
    n = max(2, int(seconds / max(per, 1e-9)))
    t0 = time.perf_counter()
    rest = o.step(n, record=True)
    dt = time.perf_counter() - t0
    out = {"value": nodes * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
           "sample": f"{n} steps of channel 0 ({cfg['nx']}x{cfg['ny']}, {len(parts)} particle(s)) "
                     f"in FP64 on one host thread, {dt:.1f} s"}
    if parts:
        ref = np.concatenate([first, rest], 0)
        out["trajectory_error"] = trajectory_errors(cfg, parts, ref)
    return out


def trajectory_errors(cfg, parts, ref):
    """Largest deviation from the oracle trajectory ref [n, particles, 10]
    over the run, per storage form: positions over the wall gap (or the
    channel height), angle in radians, angular velocity over the wall shear
    rate (or over the largest |omega| of the reference when the walls are at
    rest)."""
    import torch

    from paper_1606_01805_amd import Solver

    steps = ref.shape[0]
    gap = cfg["ny"] - 1
    shear = abs(cfg["u_wall"][3][0] - cfg["u_wall"][2][0]) / gap
    om_scale = shear if shear > 0 else max(np.abs(ref[..., 5]).max(), 1e-300)
    res = {"steps": steps, "metrics": "pos/(NY-1), theta [rad], omega/shear rate"}
    for name, st in (("F32", 1), ("F16S", 2), ("F64", 0)):
        s = Solver([(dict(cfg, storage=st), parts)])
        g = s.step(steps, record=True)
        torch.cuda.synchronize()
        s.close()
        res[name] = {"pos": float(np.abs(g[..., 0:2] - ref[..., 0:2]).max() / gap),
                     "theta": float(np.abs(g[..., 2] - ref[..., 2]).max()),
                     "omega": float(np.abs(g[..., 5] - ref[..., 5]).max() / om_scale)}
    return res


# Launch shapes picked by the autotuner: the main workload's default (used
# when no launch flag is given) and the comparison workloads.
WORKLOAD_TUNING = {"couette": dict(tile_w=64, rows_per_thread=1, xcd_remap=0, overlap=1)}
VARIANT_TUNING = {"ensemble": dict(tile_w=256, rows_per_thread=2, xcd_remap=0),
                  "large": dict(tile_w=128, rows_per_thread=2, xcd_remap=1),
                  "large16": dict(tile_w=64, rows_per_thread=4, xcd_remap=1)}


def kernel_source_sha():
    import hashlib

    h = hashlib.sha1()
    for f in ("lbm_kernels.hip", "lbm_device.h", "lbm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1606_01805_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def measured_traffic(key):
    """HBM bytes per lattice launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a plain
    256 MiB copy), or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(key)
    if not e or e.get("kernel_source_sha") != kernel_source_sha():
        return None
    return e["bytes_per_launch"]


def roofline(us_lattice, nodes, storage, traffic_key=None, tuning=None):
    b = nodes * BYTES_PER_LUP[storage]
    ach = b / (us_lattice * 1e-6) / 1e9
    # with the combined launch the lattice pass is timed as that kernel
    # without its particle workgroups
    name = ("lattice_traction_kernel (lattice workgroups only)" if tuning and tuning.get("overlap")
            else "lattice_kernel")
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(traffic_key) if traffic_key else None,
            "bytes_per_launch": b, "us_per_launch": us_lattice,
            "timing": "HIP events on the library stream around back-to-back launches of the "
                      "kernel alone, right after the timed steps (lbm_time_kernels)"}


def run_variant(name, storage, steps, warm, plain=False, tuning=None):
    """MLUPS of one comparison workload plus its lattice-kernel roofline."""
    import torch

    from paper_1606_01805_amd import Solver
    from workloads import configs as C

    wl = C.BY_NAME[name](storage=storage)
    solvers = ([Solver([ch], tuning=tuning) for ch in wl.channels] if plain
               else [Solver(wl.channels, tuning=tuning)])
    for sv in solvers:
        sv.step(warm, record=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sv in solvers:
        sv.step(steps, record=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": wl.name, "storage": ["F64", "F32", "F16S"][storage],
           "launch": "plain (one handle per channel)" if plain else "single handle, HIP graph",
           "steps": steps, "MLUPS": wl.nodes * steps / dt / 1e6, "ms_per_step": dt / steps * 1e3}
    if not plain:
        s0 = solvers[0]
        s0.checkpoint_save(7)
        us = s0.time_kernels(20)
        s0.checkpoint_restore(7)
        out["kernel_us"] = dict(zip(["ibm_force", "lattice", "traction"], [float(v) for v in us]))
        key = {("ensemble", 1): "ensemble_f32", ("large", 1): "large_f32", ("large", 2): "large_f16s"}.get((name, storage))
        out["tuning"] = s0.tuning()
        out["roofline"] = roofline(float(us[1]), wl.nodes, storage, key, out["tuning"])
    for sv in solvers:
        sv.close()
    return out


def adjoint_leg(storage=1, steps=2000, seg=100):
    """Cost of one reverse-mode gradient on the 256x64 Couette case: the
    checkpointed forward (graph replay, a checkpoint every `seg` steps) and
    the adjoint sweep (every segment recomputed into the tape and reversed),
    per step, and their ratio."""
    import torch

    from paper_1606_01805_amd import Solver
    from workloads import configs as C

    wl = C.adjoint_case(storage=storage)
    s = Solver(wl.channels)
    nseg = steps // seg
    s.checkpoint_save(nseg + 1)
    s.step(200, record=False)  # warm-up (graphs built)
    s.checkpoint_restore(nseg + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, record=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    s.checkpoint_restore(nseg + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nseg):
        s.checkpoint_save(k)
        s.step(seg, record=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    seed = [[0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0]]
    t0 = time.perf_counter()
    s.adjoint_begin(seed, seg)
    for k in reversed(range(nseg)):
        s.adjoint_segment(k, seg)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    s.close()
    return {"workload": wl.name, "storage": ["F64", "F32", "F16S"][storage], "steps": steps, "segment": seg,
            "forward_us_per_step": t_plain / steps * 1e6,
            "forward_checkpointed_us_per_step": t_fwd / steps * 1e6,
            "adjoint_us_per_step": t_adj / steps * 1e6,
            "adjoint_over_forward": t_adj / t_plain,
            "note": "adjoint time includes recomputing each segment from its checkpoint"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: the coupled step has no multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1606_01805_amd import Solver
    from workloads import configs as C

    steps, warm = default_steps(args.workload)
    steps = args.steps if args.steps is not None else steps
    warm = args.warmup if args.warmup is not None else warm
    storage = STORAGE[args.storage] if args.storage else (0 if args.workload == "sedimentation" else 1)
    wl = C.BY_NAME[args.workload](storage=storage)
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
    if not tuning and not args.autotune and not args.plain:
        tuning = dict(WORKLOAD_TUNING.get(args.workload, {}))

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    solvers = ([Solver([ch], tuning=tuning) for ch in wl.channels] if args.plain
               else [Solver(wl.channels, tuning=tuning)])
    tune_report = None
    if args.autotune:
        from paper_1606_01805_amd.tune import autotune

        best, res = autotune(solvers[0], cache=None)
        for s in solvers[1:]:
            s.set_tuning(**best)
        tune_report = {k: v * 1e6 for k, v in res.items()}
    for s in solvers:
        s.step(warm, record=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps, record=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nodes = wl.nodes
    mlups = nodes * steps / dt / 1e6

    # Per-kernel device time, HIP events around back-to-back launches of each
    # kernel alone on the library's stream (after the timed region).
    s0 = solvers[0]
    s0.checkpoint_save(7)
    us = s0.time_kernels(args.kernel_reps)
    s0.checkpoint_restore(7)
    names = ["ibm_force", "lattice", "traction"]
    k = int(max(range(3), key=lambda i: us[i]))
    nodes0 = sum(c["nx"] * c["ny"] for c in s0.cfgs)
    key = {("couette", 1): "couette_f32", ("ensemble", 1): "ensemble_f32", ("large", 1): "large_f32",
           ("large", 2): "large_f16s"}.get((args.workload, storage))
    roof = roofline(float(us[1]), nodes0, storage, key if not args.plain else None, s0.tuning())
    if k != 1:
        # the particle kernels (one workgroup per particle) are latency bound;
        # the lattice pass is the kernel that moves the step's bytes
        roof["dominant_by_time"] = names[k]
    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": dt / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[storage], "data": "synthetic",
        "config": {"workload": wl.name, "nodes": nodes, "channels": len(wl.channels),
                   "particles": wl.n_particles, "storage": ["F64", "F32", "F16S"][storage],
                   "launch": "plain (per channel)" if args.plain else "single handle, HIP graph",
                   "tuning": s0.tuning()},
        "kernel_us": dict(zip(names, [float(v) for v in us])),
        "roofline": roof,
    }
    if tune_report:
        out["autotune_us_per_step"] = tune_report
    for sv in solvers:
        sv.close()
    if not args.no_variants and args.workload == "couette":
        # plain vs batched (256 uneven channels) and FP32 vs FP16S storage
        out["variants"] = [
            run_variant("ensemble", 1, 300, 30, tuning=VARIANT_TUNING["ensemble"]),
            run_variant("ensemble", 1, 30, 5, plain=True),
            run_variant("large", 1, 500, 50, tuning=VARIANT_TUNING["large"]),
            run_variant("large", 2, 500, 50, tuning=VARIANT_TUNING["large16"]),
        ]
        out["adjoint"] = adjoint_leg()
    if args.workload == "adjoint":
        out["adjoint"] = adjoint_leg(storage=storage)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
