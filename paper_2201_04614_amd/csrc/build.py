"""Build libdq.so (HIP, gfx950) in-tree.

    python paper_2201_04614_amd/csrc/build.py

Each .hip translation unit is compiled with hipcc in parallel, then linked
into paper_2201_04614_amd/libdq.so. Floating point is strict: no fast-math
and no contraction, so every fp64 step rounds exactly as written; packed fp32
instruction selection is disabled.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libdq.so")
# (source, object, extra flags): the encode and decode kernels are compiled
# once per dimensionality so their instantiations build in parallel
UNITS = [("dq_api.hip", "dq_api.o", []), ("dq_aux.hip", "dq_aux.o", []), ("dq_select.hip", "dq_select.o", []),
                                                                          ("dq_batch.hip", "dq_batch.o", []),
                                                                          ("dq_mixed.hip", "dq_mixed.o", []),
                                                                          ("dq_huffman.hip", "dq_huffman.o", [])] + [
    (f"dq_{k}.hip", f"dq_{k}_{d}d.o", [f"-DDQ_DIM={d}"]) for k in ("encode", "decode") for d in (1, 2, 3)]
ARCH = os.environ.get("DQ_OFFLOAD_ARCH", "gfx950")

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
          "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]


def _compile(src, obj, extra, verbose):
    cmd = ["hipcc", "-c", *CFLAGS, *extra, "-o", obj, os.path.join(HERE, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose=False, jobs=None):
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, o) for _, o, _ in UNITS]
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda u: _compile(u[0], os.path.join(objdir, u[1]), u[2], verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
