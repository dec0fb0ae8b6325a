"""Writes the FP64 oracle trajectories that the reduced storage forms (FP32,
FP16S) are measured against at the full run lengths of their workloads:

  couette_400x100_50k_fp64.npz   the Re = 20 Couette channel, 400 x 100, one
                                 ellipse (AR 2, major axis 25, 64 markers,
                                 seed 1606), 50 000 steps, every 10th step
  large_4096x1024_10k_fp64.npz   the 4096 x 1024 Couette channel with 64
                                 particles of the five families (seed 1607),
                                 10 000 steps, every 50th step

Each file holds `steps` (the 1-based step numbers kept), `rec` [kept steps,
particles, 4] with x, y, theta, omega after each kept step, and the run's
length and sampling.  Only the oracle is called.  The node loops of the
oracle run on several threads (results do not depend on the count).

Run from the repository root: python tests/golden/make_trajectory_golden.py
[couette|large] [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs as C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = {
    "couette": dict(file="couette_400x100_50k_fp64.npz", make=lambda: C.couette(storage=C.STORE_F64),
                    steps=50000, every=10, chunk=1000),
    "large": dict(file="large_4096x1024_10k_fp64.npz", make=lambda: C.large(storage=C.STORE_F64),
                  steps=10000, every=50, chunk=50),
}
COLS = [0, 1, 2, 5]  # x, y, theta, omega of the particle record


def run(name, threads):
    spec = CASES[name]
    wl = spec["make"]()
    cfg, parts = wl.channels[0]
    o = oracle.Oracle(cfg)
    o.set_threads(threads)
    for p in parts:
        o.add_particle(p)
    kept, rec = [], []
    done, t0 = 0, time.time()
    while done < spec["steps"]:
        n = min(spec["chunk"], spec["steps"] - done)
        tr = o.step(n, record=True)
        for j in range(n):
            s = done + j + 1
            if s % spec["every"] == 0:
                kept.append(s)
                rec.append(tr[j][:, COLS])
        done += n
        print(f"{name}: {done}/{spec['steps']} steps, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, spec["file"])
    np.savez_compressed(out, steps=np.array(kept, dtype=np.int32), rec=np.array(rec),
                        total_steps=spec["steps"], every=spec["every"])
    print("wrote", out)


if __name__ == "__main__":
    names = [sys.argv[1]] if len(sys.argv) > 1 else list(CASES)
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    for nm in names:
        run(nm, threads)
