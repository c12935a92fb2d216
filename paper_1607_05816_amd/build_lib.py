"""Compile libuot.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is built with packed-FP32 instruction selection disabled
(-target-feature -packed-fp32-ops) and -O3; the shared library lands next to
this file so that the package loads it from the source tree.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libuot.so")
SOURCES = ["uot_kernels.hip", "uot_grid_tf.hip", "uot_dense_mf.hip", "uot_api.hip", "uot_net.hip"]
ARCH = os.environ.get("UOT_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# per-source additions: the matrix-core dense product keeps its MFMA operands
# and results in VGPRs, so the exp2 reads them without AGPR copies, and runs
# with the IEEE mode bit off (its maxima then need no NaN quieting; no NaN
# reaches them)
EXTRA = {"uot_dense_mf.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form", "-mno-amdgpu-ieee", "-fno-honor-nans"]}


def build(verbose: bool = False, jobs: int = 3) -> str:
    """Compile each source to an object, then link libuot.so; returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def _wait(item):
    p, src = item
    out, _ = p.communicate()
    if p.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, out.decode()))
    msg = out.decode().strip()
    if msg:
        # hipcc's host pass does not know the packed-fp32 feature flag; keep other output
        lines = [l for l in msg.splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l]
        if lines:
            print("\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    print(build(verbose=True))
