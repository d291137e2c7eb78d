"""Builds libhsf.so in-tree for gfx950 with hipcc (no JIT, no torch extension).

    python -m paper_2502_06959_amd.build [--jobs N]
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libhsf.so")
OBJ = os.path.join(HERE, "_build")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INC, "-I", SRC,
             # packed FP32 instructions stay off (see the design notes)
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-pthread", "-Wno-unused-command-line-argument"]
# Per-file additions.  The sweep kernels and the adjoint's tile passes branch
# on uniform plan-record fields inside their op loops; by default LLVM
# structurizes uniform regions too, which inserts register copies of the
# amplitude arrays at every merge.
_SKIP_UNIFORM = ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
FILE_FLAGS = {"sweep.hip": _SKIP_UNIFORM, "backward.hip": _SKIP_UNIFORM}
# complex products and quotients without the C99 inf/NaN recovery (the
# planner's values are O(1)): inline arithmetic, 2.3x faster host SVDs
CXX_FLAGS = ["-O3", "-fcx-limited-range", "-std=c++17", "-pthread", "-fPIC", "-I", INC, "-I", SRC, "-D__HIP_PLATFORM_AMD__",
             "-I", "/opt/rocm/include", "-Wall", "-Wno-unused-result"]


def sources():
    hip = sorted(f for f in os.listdir(SRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(SRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(args):
    cmd, obj = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=None, verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    hip, cpp = sources()
    tasks = []
    for f in hip:
        obj = os.path.join(OBJ, f + ".o")
        tasks.append((["hipcc", *HIP_FLAGS, *FILE_FLAGS.get(f, []), "-c", os.path.join(SRC, f), "-o", obj], obj))
    for f in cpp:
        obj = os.path.join(OBJ, f + ".o")
        tasks.append((["g++", *CXX_FLAGS, "-c", os.path.join(SRC, f), "-o", obj], obj))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, tasks))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
