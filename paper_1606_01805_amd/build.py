"""Build the gfx950 HIP library libpaper_lbm.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpaper_lbm.so")
SOURCES = ["csrc/lbm_kernels.hip", "csrc/lbm_adjoint.hip", "csrc/lbm_api.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: no FMA contraction, so the FP64 form performs exactly
# the IEEE operations written in the source.  The packed-FP32 feature is
# disabled for all device code.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep the per-node population arrays in registers: sinking the stores of
    # the four wall branches into one store with a computed index would move
    # the whole array to scratch memory
    "-mllvm", "-simplifycfg-sink-common=false",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compiles the three sources in parallel into objects under _build/, then
    links the shared library."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    compile_flags = [f for f in FLAGS if f != "-shared"]

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed ({r.returncode}):\n{msgs}")
        if verbose and msgs.strip():
            print(msgs)

    objs = [os.path.join(obj_dir, os.path.basename(src).replace(".hip", ".o")) for src in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(run, [[hipcc, *compile_flags, *inc, "-c", os.path.join(HERE, src), "-o", o]
                          for src, o in zip(SOURCES, objs)]))
    run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
