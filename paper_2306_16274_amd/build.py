"""Compile the HIP library (liblbm_hip.so) for gfx950 in-tree with hipcc.

Each translation unit under csrc/ (the C ABI, the batched step and one unit per lattice and
storage type holding that pair's step kernels) is compiled to an object in parallel, then
the objects are linked into one shared library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["api.hip", "batch.hip"] + [f"step_q{q}_{t}.hip" for q in (19, 27)
                                      for t in ("fp64", "fp32", "fp16")]
HEADERS = ["ctx.h", "step_ops.h", "lattice.h", "common.h", "kernels.h", "misc_kernels.h",
           "fused.h", "../../include/lbm.h"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    # fuse a*b+c only where the source writes it in one expression: the rounding of a node
    # update then does not depend on the kernel it is inlined into (tile shape, batching)
    "-ffp-contract=on",
    "--offload-arch=gfx950",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    objs, pending, failed = [], list(SOURCES), []
    running = []
    while pending or running:
        while pending and len(running) < jobs:
            src = pending.pop(0)
            obj = os.path.join(OBJ, src.replace(".hip", ".o"))
            cmd = [_hipcc()] + HIPCC_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                  stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        src, proc = running.pop(0)
        out, _ = proc.communicate()
        if proc.returncode != 0:
            failed.append((src, out))
        elif out and verbose:
            sys.stderr.write(out)
    if failed:
        for src, out in failed:
            sys.stderr.write(f"---- {src}\n{out}")
        raise RuntimeError("hipcc failed building " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking " + LIB)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
