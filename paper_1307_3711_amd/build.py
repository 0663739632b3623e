"""Build liblcmd.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed FP32 instructions disabled and FP
contraction off outside the explicit fused multiply-adds of the Coulomb kernel (the push,
ionization and diagnostics kernels then round exactly as written).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblcmd.so")
SOURCES = ["api.hip", "force.hip", "step.hip", "mlp.hip"]
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17",
    "-ffp-contract=off", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature; that is expected
    errs = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        sys.stderr.write("\n".join(errs) + "\n")
        raise RuntimeError(f"hipcc failed building {what}")
    if verbose and errs:
        sys.stderr.write("\n".join(errs) + "\n")


def build(verbose=False):
    """Compile every source to an object in parallel (one hipcc per file), then link."""
    from concurrent.futures import ThreadPoolExecutor
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    objs = [os.path.join(obj_dir, os.path.splitext(s)[0] + ".o") for s in srcs]
    cflags = [f for f in FLAGS if f != "-shared"]
    jobs = [(["hipcc"] + cflags + ["-c", "-o", o, os.path.join(CSRC, s)], s) for s, o in zip(srcs, objs)]
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_run, cmd, what, verbose) for cmd, what in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    _run(["hipcc"] + FLAGS + ["-o", tmp] + objs, "liblcmd.so", verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
