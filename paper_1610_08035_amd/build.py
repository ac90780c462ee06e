"""Build the gfx950 shared library ``libspingp.so`` in this folder with hipcc.

    python -m paper_1610_08035_amd.build
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspingp.so")
# The C-ABI unit, one object per compiled tile shape (R points per lane, L lanes per
# work-group; the list must match spg::tile_ops() in spingp_api.hip) and one wide-state unit
# per state dimension (spg::wide::ops()).
SOURCES = ["spingp_api.hip"]
TILES = [(8, 128), (8, 64), (8, 256), (4, 128), (4, 256), (16, 128)]
WIDE_B = list(range(2, 17))
HEADERS = ["spingp_device.hpp", "spingp_kernels.hpp", "spingp_host.hpp", "spingp_wide_host.hpp", "spingp_series.hpp",
           "spingp_wide.hpp", "spingp_sumdesc.hpp", "spingp_sqexp_tables.hpp"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed fp32 arithmetic stays off; all arithmetic here is fp64 anyway
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _compile(args):
    cmd, out = args
    res = subprocess.run(cmd, capture_output=True, text=True)
    return out, res.returncode, res.stdout + res.stderr


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(os.path.dirname(HERE), "include")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        jobs.append(([hipcc()] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    for r, l in TILES:
        obj = os.path.join(objdir, f"spingp_tile_R{r}_L{l}.o")
        jobs.append(([hipcc()] + HIPCC_FLAGS + inc + [f"-DSPG_TILE_R={r}", f"-DSPG_TILE_L={l}", "-c",
                                                       os.path.join(CSRC, "spingp_tile.hip"), "-o", obj], obj))
    for b in WIDE_B:
        obj = os.path.join(objdir, f"spingp_wide_b{b}.o")
        jobs.append(([hipcc()] + HIPCC_FLAGS + inc + [f"-DSPG_WIDE_B={b}", "-c", os.path.join(CSRC, "spingp_wide.hip"),
                                                       "-o", obj], obj))
    # the wide units take longest: start them first
    jobs.sort(key=lambda j: 0 if "wide_b" in j[1] else 1)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(_compile, jobs))
    for out, rc, log in results:
        if rc != 0:
            sys.stderr.write(log)
            raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
        if verbose:
            sys.stderr.write(log)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _, _ in results]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libspingp.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
