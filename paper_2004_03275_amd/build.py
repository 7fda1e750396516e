"""Build libamrv.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled to an object of its own, in parallel, and the
objects are linked into the shared library."""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libamrv.so")

SOURCES = ["kernels.hip", "mlp.hip", "multigrid.hip", "fmg.hip", "gridcopy.hip", "forest.cpp", "regrid.cpp", "api.cpp"]

# binary64 results are reproducible bit for bit only without contraction;
# packed-FP32 instructions are kept out of every HIP build
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]

# extra flags per unit: the combined-variant stage kernels, which run two
# waves per SIMD (register-bound), gain ~3% per launch from the
# ILP-maximising scheduler (the other stage kernels lose)
UNITS = {"stage_ilp.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
         # the same kernels in fast arithmetic: contraction on (the flag after
         # the common -ffp-contract=off wins)
         "stage_fast.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp", "-ffp-contract=fast"],
         # the two-launch 3D MHD stage update (default scheduler), exact and fast
         "stage_zsplit.hip": [],
         "stage_zsplit_fast.hip": ["-ffp-contract=fast"]}


def _jobs() -> int:
    env = os.environ.get("MAX_JOBS")
    if env and env.isdigit():
        return max(1, int(env))
    return max(1, min(16, os.cpu_count() or 1))


CACHE = os.path.join(os.path.dirname(HERE), "_build")


def _key(src: str, cmd: list) -> str:
    """Hash of a unit's compile command, its source and every header it may include."""
    h = hashlib.sha256(" ".join(cmd).encode())
    inc = os.path.join(os.path.dirname(HERE), "include")
    for d in (CSRC, inc):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hpp", ".h")) or name == src:
                with open(os.path.join(d, name), "rb") as fh:
                    h.update(name.encode() + fh.read())
    if src in UNITS:  # units that include another source
        with open(os.path.join(CSRC, "kernels.hip"), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:24]


def build(verbose: bool = False, extra: list | None = None, cache: bool = False) -> str:
    """Compile every unit and link libamrv.so.  cache=True reuses objects of
    unchanged units from _build/ (development only; the default compiles all)."""
    t0 = time.time()
    units = [(s, []) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    units += [(u, f) for u, f in UNITS.items()]
    if cache:
        os.makedirs(CACHE, exist_ok=True)
    with tempfile.TemporaryDirectory(dir=HERE, prefix="_build_") as tmpdir:
        def compile_one(unit):
            src, flags = unit
            obj = os.path.join(tmpdir, src + ".o")
            cmd = ["hipcc", *HIPFLAGS, *flags, *(extra or []), "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj]
            cached = os.path.join(CACHE, f"{src}.{_key(src, cmd[:-2])}.o") if cache else None
            if cached and os.path.exists(cached):
                return cached
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            if cached:
                shutil.copyfile(obj, cached)
            return obj

        with ThreadPoolExecutor(max_workers=_jobs()) as ex:
            objs = list(ex.map(compile_one, units))
        tmp = LIB + ".tmp"
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, cache="--cache" in sys.argv)
