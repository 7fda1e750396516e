#!/usr/bin/env python3
"""Benchmark of the block-forest finite-volume update on one MI355X.

Workload (default): the 3D spherical blast on a 4-level octree forest of 16^3
leaves (19,384 leaves, 79.4M cells, HLLC + van Leer + SSP-RK3, FP64).  A timed
step is one pass of the whole hot path: the Courant reduction (max_dt), one
full SSP-RK3 step (coarse-fine ghost slabs, stage kernels) and, every
--flag-every steps, the Loehner refinement flags.

Prints ONE JSON line: MCUPS of the batched path (interior cells x steps / s),
the stage kernel's HBM roofline fraction (algorithmic bytes / event-timed
launch duration), the one-launch-per-block path, full-size parity of one step
against the CPU oracle, the oracle's own throughput on the host cores, and
(object "reaction_diffusion") the paper's timed reaction-diffusion workload:
Schnakenberg on 256^2 with IMEX, split and explicit steps through the
multigrid solver; (object "reaction_diffusion_amr") Gray-Scott on the
paper's three-level AMR setup through the forest multigrid.  --workload rd2d
/ rd3d / gsamr2d print that workload's own line (ms per IMEX step on 256^2 /
128^3 / the 128^2-512^2 forest).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MCUPS (cell-updates/s) per full RK step, batched vs per-block, at 1e-10 L1"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


COUNTER_SOURCES = ("kernels.hip", "stage_ilp.hip", "stage_fast.hip", "stage_common.hpp", "bf16.hpp", "physics.hpp",
                   "internal.hpp")


def counter_sources_sha256() -> str:
    """sha256 of the stage kernel's sources and its compile flags (the common
    hipcc flags and the per-unit flags of paper_2004_03275_amd/build.py)."""
    import hashlib

    from paper_2004_03275_amd import build as B

    csrc = os.path.join(ROOT, "paper_2004_03275_amd", "csrc")
    data = b"".join(open(os.path.join(csrc, f), "rb").read() for f in COUNTER_SOURCES)
    return hashlib.sha256(data + repr(B.HIPFLAGS).encode() + repr(sorted(B.UNITS.items())).encode()).hexdigest()


def measured_counters(workload: str, limiter: str = "vanleer", variant: int = 0, arithmetic: str = "fast") -> dict:
    """HBM bytes per stage-kernel launch and the VALU / FP64 issue fractions
    from the committed counter summary, if it was taken on this workload and
    stage kernel (van Leer slopes, combined variant, fast arithmetic) with the
    current kernel sources and build flags (else an empty dict)."""
    if workload != "blast" or limiter != "vanleer" or variant != 0 or arithmetic != "fast":
        return {}
    prof = os.path.join(ROOT, "profiles", "hbm_counters_3d_amr_blast.md")
    try:
        text = open(prof).read()
        h = counter_sources_sha256()
    except OSError:
        return {}
    keys = ("kernel_source_sha256", "traffic_bytes_per_launch", "valu_issue_frac", "fp64_issue_frac")
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(keys))
    if vals.get("kernel_source_sha256", "").strip() != h:
        return {}
    return {k: float(vals[k]) for k in keys[1:] if k in vals}


def make_workload(name: str):
    import workloads as W

    if name == "blast":
        s = W.blast_scheme()
        f, U = W.blast(s, forest=W.blast_lohner_forest(s))
        desc = "3d_amr_blast"
    elif name == "kh":
        f, U = W.kh(16)
        desc = "2d_kelvin_helmholtz"
    elif name == "ot":
        f, U = W.orszag_tang(32)
        desc = "2d_mhd_orszag_tang"
    elif name == "sod":
        f, U = W.sod(1024)
        desc = "1d_sod"
    elif name == "mhdblast2d":
        f, U = W.mhd_blast(2, base=4, max_level=4)
        desc = "2d_amr_mhd_blast"
    elif name == "mhdblast3d":
        f, U = W.mhd_blast(3, base=4, max_level=3)
        desc = "3d_amr_mhd_blast"
    elif name == "dambreak2d":
        f, U = W.dam_break()
        desc = "2d_amr_shallow_water_dam_break"
    else:
        raise SystemExit(f"unknown workload {name}")
    return desc, f, U


RD_PAPER_MS = {"imex": 7.7, "split": 7.2, "explicit": 1.1}  # Sec. 2.5.2: 256^2 Schnakenberg, 4 CPU cores


def rd_vcycle_bytes(nd: int, n: int, nfields: int = 2) -> float:
    """Algorithmic HBM bytes of one V-cycle: per field and level above the
    LDS-resident tail (levels of more than 4,096 cells), the down launch reads
    phi and f and writes phi and the coarse f and phi (24 + 16/2^d bytes per
    cell), the up launch reads phi, f and the coarse correction and writes
    phi (24 + 8/2^d bytes per cell); the tail's own levels never leave LDS."""
    total = 0.0
    m = n
    while m ** nd > 4096:
        c = m ** nd
        total += c * (24 + 16 / 2 ** nd) + c * (24 + 8 / 2 ** nd)
        m //= 2
    return nfields * total


def rd_measure(nd: int, n: int, steps: int, warmup: int, log, cpu: bool = True, dt: float = 1e-3,
               tol: float = 1e-7) -> dict:
    """The paper's reaction-diffusion workload (Sec. 2.5.2): Schnakenberg on an
    n^nd uniform grid with zero Neumann boundaries, dt = 1e-3, multigrid to
    max residual <= tol max|f|; IMEX, split and explicit Euler steps timed
    with the state resident in HBM, one IMEX step checked against the oracle
    (exact solves), the oracle's IMEX step timed on the host."""
    import numpy as np
    import torch

    from paper_2004_03275_amd import multigrid as M
    import workloads as W

    params = {"model": M.SCHNAKENBERG, "Du": 0.05, "Dv": 1.0, "p1": 100.0, "p2": 0.1305, "p3": 0.7695}
    u0, v0, L = W.schnakenberg_initial(nd, n)
    mg = M.GpuMultigrid(nd, n, M.NEUMANN, L, nfields=2)
    res = {}
    for name, scheme, sdt, k in (("imex", M.IMEX, dt, steps), ("split", M.SPLIT, dt, steps),
                                 ("explicit", M.EULER, 1e-6, steps * 10)):
        u = torch.tensor(u0, device="cuda:0").contiguous()
        v = torch.tensor(v0, device="cuda:0").contiguous()
        mg.rd_step(u, v, sdt, scheme, params, nsteps=warmup, tol=tol)
        torch.cuda.synchronize()
        mg.profile(True)
        mg.profile_read()
        mg.profile(False)
        t0 = time.perf_counter()
        cyc, _ = mg.rd_step(u, v, sdt, scheme, params, nsteps=k, tol=tol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[name] = {"ms_per_step": 1e3 * el / k, "steps": k, "vcycles_per_step": cyc / k}
    # V-cycle time from HIP events (separate run, same work)
    u = torch.tensor(u0, device="cuda:0").contiguous()
    v = torch.tensor(v0, device="cuda:0").contiguous()
    mg.profile(True)
    mg.rd_step(u, v, dt, M.IMEX, params, nsteps=steps, tol=tol)
    vms, vcyc = mg.profile_read()
    mg.profile(False)
    vcycle_us = 1e3 * vms / max(vcyc, 1)
    vbytes = rd_vcycle_bytes(nd, n)
    achieved = vbytes / (vcycle_us * 1e-6) / 1e9
    out = {"workload": f"schnakenberg_{nd}d_{n}", "cells": n ** nd, "dt": dt, "tol": tol,
           "imex_ms_per_step": res["imex"]["ms_per_step"], "split_ms_per_step": res["split"]["ms_per_step"],
           "explicit_euler_ms_per_step": res["explicit"]["ms_per_step"],
           "imex_vcycles_per_step": res["imex"]["vcycles_per_step"],
           "split_vcycles_per_step": res["split"]["vcycles_per_step"],
           "vcycle_us": vcycle_us,
           "roofline": {"bound": "hbm", "kernel": "one V-cycle (all its launches)", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "algorithmic_bytes_per_vcycle": vbytes,
                        "note": "latency-bound: the levels are cache-resident and each V-cycle is a chain of "
                                "dependent launches"},
           "paper_cpu_ms_per_step": dict(RD_PAPER_MS) if (nd, n) == (2, 256) else None}
    log(f"rd {nd}D {n}: IMEX {out['imex_ms_per_step']:.3f} ms/step ({out['imex_vcycles_per_step']:.2f} cycles), "
        f"split {out['split_ms_per_step']:.3f} ms, explicit {out['explicit_euler_ms_per_step']:.4f} ms, "
        f"V-cycle {vcycle_us:.1f} us")
    if cpu:
        from oracle import rd as R

        u = torch.tensor(u0, device="cuda:0").contiguous()
        v = torch.tensor(v0, device="cuda:0").contiguous()
        mg.rd_step(u, v, dt, M.IMEX, params, nsteps=1, tol=1e-12, max_cycles=80)
        t0 = time.perf_counter()
        ru, rv = R.step(u0, v0, dt, R.IMEX, R.SCHNAKENBERG_PARAMS, L, R.NEUMANN)
        ocpu = time.perf_counter() - t0
        diff = max(np.abs(u.cpu().numpy() - ru).max() / np.abs(ru).max(),
                   np.abs(v.cpu().numpy() - rv).max() / np.abs(rv).max())
        out["parity"] = {"steps": 1, "scheme": "imex", "tol": 1e-12, "rel_max_diff": float(diff),
                         "bar": 1e-8}
        out["cpu_baseline"] = {"value": 1e3 * ocpu, "unit": "ms per IMEX step", "cores": 1, "kind": "oracle",
                               "sample": "one IMEX step of the same grid with exact (FFT/DCT) solves"}
        log(f"rd parity: rel max diff {diff:.2e}; oracle {1e3 * ocpu:.1f} ms per IMEX step")
    mg.close()
    return out


def fmg_vcycle_bytes(levels: list, base_cells: int) -> float:
    """Algorithmic HBM bytes of one forest V-cycle: on every level above the
    base, each block's 256 cells are read and written once on the way down
    (state and right-hand side in, state, parent state and right-hand side
    out: 24 + 16/4 bytes per cell) and once on the way up (state, right-hand
    side and parent change in, state out: 24 + 8/4), as rd_vcycle_bytes
    counts a uniform level; plus the level-1 correction's uniform V-cycles
    (one field), counted once."""
    total = 0.0
    for nblk in levels[1:]:
        c = 256 * nblk
        total += c * (24 + 16 / 4) + c * (24 + 8 / 4)
    return total + rd_vcycle_bytes(2, base_cells, nfields=1)


def fmg3d_vcycle_bytes(levels: list, base_cells: int) -> float:
    """fmg_vcycle_bytes in 3D: 24 + 16/8 bytes per cell down, 24 + 8/8 up, on
    every level above the base, plus one uniform V-cycle of the base grid."""
    total = 0.0
    for nblk in levels[1:]:
        c = 4096 * nblk
        total += c * (24 + 16 / 8) + c * (24 + 8 / 8)
    return total + rd_vcycle_bytes(3, base_cells, nfields=1)


def fmg3d_measure(log, reps: int = 3) -> dict:
    """Helmholtz solves on a four-level octree forest refined around a sphere
    (base 4^3 blocks of 16^3, levels 2-4 holding leaves, 14.5M cells; a
    Gaussian right-hand side with seeded noise): lambda = 1e4 (an IMEX-like
    step) and lambda = 10 (near Poisson), from zero to max residual <= 1e-7
    max |f|, state resident in HBM."""
    import numpy as np
    import torch

    from paper_2004_03275_amd import multigrid as M
    import workloads as W

    f = W.fmg_forest(W.fmg_scheme(base=4, max_level=4, bc=M.PERIODIC, ndim=3), centre=(0.5, 0.5, 0.5), radius=0.2)
    x, y, z = W.cell_centres(f)
    rhs = np.exp(-40 * ((x - 0.45) ** 2 + (y - 0.55) ** 2 + (z - 0.5) ** 2))
    rhs = rhs + 0.1 * W.uniform01(21, rhs.size).reshape(rhs.shape)
    mg = M.GpuForestMultigrid(f, 1.0, M.PERIODIC)
    levels = mg.levels()
    F = torch.tensor(rhs, device="cuda:0")
    out = {"workload": "helmholtz_3d_amr", "leaves": f.n, "cells": f.n * 4096,
           "levels": {str(k): v for k, v in f.level_counts().items()}, "blocks_per_tree_level": levels, "tol": 1e-7}
    vbytes = fmg3d_vcycle_bytes(levels, 64)
    for lam in (1e4, 10.0):
        U = torch.zeros_like(F)
        mg.solve(F, U, lam, tol=1e-7)  # warm-up (also sets the batch of unchecked cycles)
        ts, cs = [], []
        for _ in range(reps):
            U.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cyc, _, _ = mg.solve(F, U, lam, tol=1e-7)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            cs.append(cyc)
        ms = 1e3 * float(np.median(ts))
        vus = 1e3 * ms / max(cs[-1], 1)
        out[f"lambda_{lam:g}"] = {"ms_per_solve": ms, "vcycles": cs[-1], "vcycle_us": vus,
                                  "achieved_gbs": vbytes / (vus * 1e-6) / 1e9}
        log(f"3D AMR Helmholtz {f.level_counts()} lambda {lam:g}: {ms:.2f} ms per solve, {cs[-1]} cycles, "
            f"V-cycle {vus:.0f} us ({vbytes / (vus * 1e-6) / 1e9:.0f} GB/s algorithmic)")
    out["algorithmic_bytes_per_vcycle"] = vbytes
    mg.close()
    return out


def gsamr_measure(steps: int, warmup: int, log, cpu: bool = True, tol: float = 1e-7) -> dict:
    """Gray-Scott on the paper's three-level AMR setup (Sec. 2.5.2; periodic
    side 2, 128^2 to 512^2, a static forest refined around the initial
    perturbations): IMEX and split steps (dt = 0.5, the forest multigrid to
    max residual <= tol max|f|) and explicit midpoint steps (dt = 0.05, within
    the explicit limit of the finest level), state resident in HBM; one IMEX
    step checked against the oracle (exact composite solves), the oracle's
    IMEX step timed on the host."""
    import numpy as np
    import torch

    from paper_2004_03275_amd import multigrid as M
    import workloads as W

    params = {"model": M.GRAY_SCOTT, "Du": 2e-5, "Dv": 1e-5, "p1": 0.046, "p2": 0.063, "p3": 0.0}
    f, u0, v0, L = W.gray_scott_amr()
    mg = M.GpuForestMultigrid(f, L, M.PERIODIC)
    levels = mg.levels()
    res = {}
    for name, scheme, sdt in (("imex", M.IMEX, 0.5), ("split", M.SPLIT, 0.5), ("midpoint", M.MIDPOINT, 0.05)):
        u = torch.tensor(u0, device="cuda:0").contiguous()
        v = torch.tensor(v0, device="cuda:0").contiguous()
        mg.rd_step(u, v, sdt, scheme, params, nsteps=warmup, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc, _ = mg.rd_step(u, v, sdt, scheme, params, nsteps=steps, tol=tol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[name] = {"ms_per_step": 1e3 * el / steps, "vcycles_per_step": cyc / steps}
    # the V-cycle's share: the IMEX step time over its cycles (each cycle ends
    # in a host read of its residual, which this includes)
    vcycle_us = 1e3 * res["imex"]["ms_per_step"] / max(res["imex"]["vcycles_per_step"], 1e-9)
    vbytes = fmg_vcycle_bytes(levels, 16 * f.scheme.base_blocks[0])
    achieved = vbytes / (vcycle_us * 1e-6) / 1e9
    cells = f.n * 256
    out = {"workload": "gray_scott_amr_2d", "leaves": f.n, "cells": cells,
           "levels": {str(k): v for k, v in f.level_counts().items()}, "blocks_per_tree_level": levels,
           "dt": {"imex": 0.5, "split": 0.5, "midpoint": 0.05}, "tol": tol,
           "imex_ms_per_step": res["imex"]["ms_per_step"], "split_ms_per_step": res["split"]["ms_per_step"],
           "midpoint_ms_per_step": res["midpoint"]["ms_per_step"],
           "imex_vcycles_per_step": res["imex"]["vcycles_per_step"],
           "split_vcycles_per_step": res["split"]["vcycles_per_step"],
           "vcycle_us": vcycle_us,
           "roofline": {"bound": "hbm", "kernel": "one forest V-cycle (all its launches)", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "algorithmic_bytes_per_vcycle": vbytes,
                        "note": "latency-bound: about 50 dependent launches per cycle over cache-resident "
                                "levels, and a host read of the residual after each cycle"}}
    log(f"gray-scott AMR {f.level_counts()}: IMEX {out['imex_ms_per_step']:.2f} ms/step "
        f"({out['imex_vcycles_per_step']:.2f} cycles per step, both species), split {out['split_ms_per_step']:.2f} ms, "
        f"midpoint {out['midpoint_ms_per_step']:.3f} ms, V-cycle {vcycle_us:.0f} us")
    if cpu:
        from oracle import fmg as O
        from oracle import rd as R

        u = torch.tensor(u0, device="cuda:0").contiguous()
        v = torch.tensor(v0, device="cuda:0").contiguous()
        mg.rd_step(u, v, 0.5, M.IMEX, params, nsteps=1, tol=1e-12, max_cycles=80)
        t0 = time.perf_counter()
        ru, rv = O.rd_step(f, u0, v0, 0.5, R.IMEX, R.GRAY_SCOTT_PARAMS, L, O.PERIODIC)
        ocpu = time.perf_counter() - t0
        diff = max(np.abs(u.cpu().numpy() - ru).max() / np.abs(ru).max(),
                   np.abs(v.cpu().numpy() - rv).max() / np.abs(rv).max())
        out["parity"] = {"steps": 1, "scheme": "imex", "tol": 1e-12, "rel_max_diff": float(diff), "bar": 1e-8}
        out["cpu_baseline"] = {"value": 1e3 * ocpu, "unit": "ms per IMEX step", "cores": 1, "kind": "oracle",
                               "sample": "one IMEX step of the same forest with exact (sparse LU) composite solves"}
        log(f"gray-scott AMR parity: rel max diff {diff:.2e}; oracle {1e3 * ocpu:.0f} ms per IMEX step")
    mg.close()
    out["helmholtz_3d_amr"] = fmg3d_measure(log)
    return out


def gsamr_main(args, log):
    r = gsamr_measure(args.steps, args.warmup, log, cpu=not args.no_cpu_baseline)
    ms = r["imex_ms_per_step"]
    out = {
        "metric": "ms per IMEX Gray-Scott step on the three-level forest (multigrid to max residual <= 1e-7 max|f|)",
        "value": ms,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "leaves": r["leaves"], "cells": r["cells"], "levels": r["levels"],
                   "dt": r["dt"]["imex"], "tol": r["tol"], "model": "gray_scott", "bc": "periodic",
                   "cycle": "FAS V(2,2) over the block tree, uniform V-cycles on level 1"},
        "roofline": r["roofline"],
        "cpu_baseline": r.get("cpu_baseline"),
        "parity": r.get("parity"),
        "reaction_diffusion_amr": r,
    }
    print(json.dumps(out), flush=True)


def rd_main(args, log):
    nd, n = (2, 256) if args.workload == "rd2d" else (3, 128)
    r = rd_measure(nd, n, args.steps, args.warmup, log, cpu=not args.no_cpu_baseline)
    ms = r["imex_ms_per_step"]
    paper = RD_PAPER_MS["imex"] if (nd, n) == (2, 256) else None
    out = {
        "metric": "ms per IMEX reaction-diffusion step (multigrid to max residual <= 1e-7 max|f|)",
        "value": ms,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": ms / paper if paper else None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "cells": r["cells"], "dt": r["dt"], "tol": r["tol"],
                   "model": "schnakenberg", "bc": "neumann", "smoother": "tiled 2D" if nd == 2 else "per-colour",
                   "cycle": "V(2,2)", "launch": "direct (no graph)"},
        "roofline": r["roofline"],
        "cpu_baseline": r.get("cpu_baseline"),
        "parity": r.get("parity"),
        "reaction_diffusion": r,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="blast", choices=["blast", "kh", "ot", "sod", "mhdblast2d", "mhdblast3d",
                                                             "dambreak2d", "rd2d", "rd3d", "gsamr2d"])
    ap.add_argument("--flag-every", type=int, default=10)
    ap.add_argument("--per-block-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay each step as a HIP graph")
    ap.add_argument("--schedule", default=None,
                    help="fixed schedule instead of autotuning: grid, grid-noremap or persistent:<workgroups>")
    ap.add_argument("--variant", type=int, default=None, help="force the stage-kernel variant (0, 1, or 2 for 3D MHD)")
    ap.add_argument("--arithmetic", default="fast", choices=["fast", "exact"],
                    help="stage-kernel arithmetic: fast (FMA, refined reciprocal estimates; within the 1e-10 bar) "
                         "or exact (correctly rounded, bit for bit with the oracle)")
    ap.add_argument("--tune-reps", type=int, default=5)
    ap.add_argument("--host-dt", action="store_true",
                    help="time steps as amrv_max_dt + amrv_advance (host-side dt) instead of amrv_advance_cfl")
    ap.add_argument("--limiter", default=None, choices=["minmod", "vanleer", "mc", "koren", "cada"],
                    help="override the workload's limiter")
    ap.add_argument("--cada-radius", type=float, default=None,
                    help="radius of Cada's smoothness switch (with --limiter cada)")
    ap.add_argument("--adaptive-steps", type=int, default=None,
                    help="also run this many steps from the initial state with regridding (default 20 on the "
                         "3D blast, 0 elsewhere)")
    ap.add_argument("--regrid-every", type=int, default=5)
    ap.add_argument("--adaptive-flagger", default="lohner", choices=["lohner", "mlp"],
                    help="flags of the adaptive run: Loehner, or the learned flagger with Loehner fallback "
                         "(compared with full Loehner flags every second regrid)")
    ap.add_argument("--no-rd", action="store_true",
                    help="skip the reaction-diffusion measurement that the default run adds")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_03275_amd import _native as N
    from paper_2004_03275_amd import forest as F
    import workloads as W

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload in ("rd2d", "rd3d"):
        rd_main(args, log)
        return
    if args.workload == "gsamr2d":
        gsamr_main(args, log)
        return

    desc, f, U0 = make_workload(args.workload)
    s = f.scheme
    if args.limiter:
        s.limiter = {"minmod": W.MINMOD, "vanleer": W.VANLEER, "mc": W.MC, "koren": W.KOREN,
                      "cada": W.CADA}[args.limiter]
    if args.cada_radius is not None:
        s.cada_radius = args.cada_radius
    cells = f.n * s.cells_per_block
    log(f"workload {desc}: {f.n} leaves {f.level_counts()}, {cells} cells")

    g = F.GpuForest(f, device="cuda:0")
    g.set_arithmetic(N.ARITH_FAST if args.arithmetic == "fast" else N.ARITH_EXACT)
    g.set_state(U0)
    dt0 = g.max_dt()

    # -- full-size parity of one step against the oracle (same dt), and the
    #    oracle's throughput on the host cores
    parity = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        g.advance(dt0)
        G1 = g.get_state()
        o = oracle.OracleForest(f)
        o.set_state(U0)
        o.max_dt()
        threads = oracle.get_threads()
        t0 = time.perf_counter()
        o.advance(dt0)
        el = time.perf_counter() - t0
        R1 = o.get_state()
        o.close()
        e = W.relative_l1(G1, R1, f)
        parity = {"steps": 1, "rel_l1_max": float(e.max()), "bitwise_equal": bool(np.array_equal(G1, R1)),
                  "tolerance": 1e-10}
        cpu = {"value": cells / el / 1e6, "unit": "MCUPS", "cores": threads, "kind": "oracle",
               "sample": f"one full SSP-RK step of the same {desc} forest ({cells} cells) from its initial state, "
                         f"{el:.1f} s"}
        log(f"parity 1 step: rel L1 {e.max():.3e}, bitwise {parity['bitwise_equal']}; oracle {cpu['value']:.2f} "
            f"MCUPS on {threads} threads")
        del G1, R1
        g.set_state(U0)
        if args.workload == "blast":
            # the oracle on one thread, on a bounded sample of the same workload:
            # one step of the blast on the 8^3-base forest (the same sphere and levels)
            s8 = W.blast_scheme(base=8, max_level=s.max_level)
            f8, U8 = W.blast(s8)
            c8 = f8.n * s8.cells_per_block
            oracle.set_threads(1)
            try:
                o = oracle.OracleForest(f8)
                o.set_state(U8)
                dt8 = o.max_dt()
                t0 = time.perf_counter()
                o.advance(dt8)
                el1 = time.perf_counter() - t0
                o.close()
            finally:
                oracle.set_threads(threads)
            cpu["one_thread"] = {"value": c8 / el1 / 1e6, "unit": "MCUPS", "cores": 1,
                                 "sample": f"one full SSP-RK step of the 3d_amr_blast on the 8^3-base forest "
                                           f"({f8.n} leaves, {c8} cells) from its initial state, {el1:.1f} s"}
            log(f"oracle on 1 thread: {cpu['one_thread']['value']:.2f} MCUPS ({el1:.1f} s, {f8.n} leaves)")

    if args.copy_calibration_mib > 0:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration_mib} MiB read + written")
        del src, dst

    sched = None
    if args.schedule:
        if args.schedule == "grid":
            g.set_schedule(N.SCHED_GRID, 1, 0)
        elif args.schedule == "grid-noremap":
            g.set_schedule(N.SCHED_GRID, 0, 0)
        elif args.schedule.startswith("persistent"):
            wgs = int(args.schedule.split(":")[1]) if ":" in args.schedule else 0
            g.set_schedule(N.SCHED_PERSISTENT, 0, wgs)
        else:
            raise SystemExit(f"unknown schedule {args.schedule}")
        sched = (*g.get_schedule(), g.get_variant())
    elif not args.no_autotune:
        sched = g.autotune(args.tune_reps)
        log(f"autotuned schedule {sched}\n" + g.autotune_report())
    else:
        sched = (*g.get_schedule(), g.get_variant())
    if args.variant is not None:
        g.set_variant(args.variant)
        sched = (*sched[:3], args.variant)
    if args.graph:
        g.use_graph(True)

    def host_step(i):
        dt = g.max_dt()
        g.advance(dt)
        if args.flag_every and (i + 1) % args.flag_every == 0:
            g.flag_blocks()

    def device_steps(k, t):
        # k steps with device-computed dt, Loehner flags every flag_every steps
        done = 0
        while done < k:
            m = k - done
            if args.flag_every:
                m = min(m, args.flag_every - (done % args.flag_every))
            t, _ = g.advance_cfl(m, float("inf"), t)
            done += m
            if args.flag_every and done % args.flag_every == 0:
                g.flag_blocks()
        return t

    t_sim = 0.0
    if args.host_dt:
        for i in range(args.warmup):
            host_step(i)
    else:
        t_sim = device_steps(args.warmup, t_sim)
    g.synchronize()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    if args.host_dt:
        for i in range(args.steps):
            host_step(i)
    else:
        t_sim = device_steps(args.steps, t_sim)
    g.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    mcups = cells * args.steps / el / 1e6
    ms_step = el / args.steps * 1e3

    # stage-kernel roofline: HIP events around each stage launch (separate pass)
    g.profile(True)
    nprof = max(1, min(args.steps, 6))
    if args.host_dt:
        for i in range(nprof):
            host_step(i)
    else:
        t_sim = device_steps(nprof, t_sim)
    kms, launches, kbytes = g.profile_read()
    g.profile(False)
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms / 1e3) / 1e9 if launches else 0.0
    log(f"batched: {mcups:.1f} MCUPS, {ms_step:.3f} ms/step; stage kernel {avg_ms:.3f} ms/launch, "
        f"{achieved:.0f} GB/s algorithmic")

    per_block = None
    if args.per_block_steps > 0:
        g.use_graph(False)
        g.set_schedule(N.SCHED_PER_BLOCK)
        g.synchronize()
        t0 = time.perf_counter()
        for i in range(args.per_block_steps):
            dt = g.max_dt()
            g.advance(dt)
        g.synchronize()
        pel = time.perf_counter() - t0
        pb = cells * args.per_block_steps / pel / 1e6
        per_block = {"value": pb, "unit": "MCUPS", "steps": args.per_block_steps,
                     "ms_per_step": pel / args.per_block_steps * 1e3, "batched_over_per_block": mcups / pb}
        log(f"per-block: {pb:.1f} MCUPS ({mcups / pb:.1f}x slower)")

    # learned flagger against Loehner on the evolved state (config 5 on this forest)
    flagger = None
    if s.ndim > 1:
        from paper_2004_03275_amd import mlp as MLP

        try:
            wts = MLP.trained_weights()
            margin = MLP.trained_margin()
        except (OSError, ValueError, KeyError):
            wts = None
        if wts is not None:
            g.set_schedule(*sched[:3])
            g.mlp_set_weights(wts)
            g.mlp_set_margin(margin)
            fl, emax = g.flag_blocks(with_emax=True)
            fm = g.flag_blocks(mode=N.FLAG_MLP)
            ff = g.flag_blocks(mode=N.FLAG_MLP_FALLBACK)
            z = g.mlp_logits()

            def tflag(mode, reps=5):
                g.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    g.flag_blocks(mode=mode)
                return (time.perf_counter() - t0) / reps * 1e3

            tl, tm, tf = tflag(N.FLAG_LOHNER), tflag(N.FLAG_MLP), tflag(N.FLAG_MLP_FALLBACK)
            conf = np.zeros((3, 3), dtype=np.int64)
            np.add.at(conf, (fl.astype(np.int64) + 1, fm.astype(np.int64) + 1), 1)
            flagger = {"lohner_ms": tl, "mlp_ms": tm, "mlp_fallback_ms": tf,
                       "flag_disagreement": float(np.mean(fm != fl)),
                       "fallback_flag_disagreement": float(np.mean(ff != fl)),
                       "fallback_fraction": float(np.mean((np.abs(z[:, 0]) < margin) | (np.abs(z[:, 1]) < margin))),
                       "margin": margin, "refine_flags_lohner": int(np.sum(fl == 1)),
                       "coarsen_flags_lohner": int(np.sum(fl == -1)), "confusion_lohner_by_mlp": conf.tolist()}
            # features pooled in the last stage of the step (amrv_mlp_fuse_features):
            # the flagging that follows runs the network only
            if s.ndim == 3:
                # the cost of pooling: 5 device-timed steps (graph replay) with
                # and without it, each after one step that captures its graph
                step_ms = {}
                for fuse in (False, True):
                    g.mlp_fuse_features(fuse)
                    t_sim, _ = g.advance_cfl(1, float("inf"), t_sim)
                    g.synchronize()
                    t0 = time.perf_counter()
                    t_sim, _ = g.advance_cfl(5, float("inf"), t_sim)
                    g.synchronize()
                    step_ms[fuse] = (time.perf_counter() - t0) * 1e3 / 5
                g.synchronize()
                # the flagging after the fused step (network only; the
                # features stay valid until the state changes): median of 5
                tz = []
                for _ in range(5):
                    t0 = time.perf_counter()
                    fused = g.flag_blocks(mode=N.FLAG_MLP)
                    tz.append((time.perf_counter() - t0) * 1e3)
                tfz = float(np.median(tz))
                g.mlp_fuse_features(False)
                fsep = g.flag_blocks(mode=N.FLAG_MLP)
                flagger.update({"mlp_fused_ms": tfz, "fused_equal_separate": bool(np.array_equal(fused, fsep)),
                                "step_ms_with_fused_features": step_ms[True],
                                "step_ms_without_features": step_ms[False]})
            log(f"flagger: Loehner {tl:.2f} ms, MLP {tm:.2f} ms, fallback {tf:.2f} ms, fused "
                f"{flagger.get('mlp_fused_ms', float('nan')):.3f} ms; disagreement {flagger['flag_disagreement']:.4f} "
                f"(fallback {flagger['fallback_flag_disagreement']:.4f}); Loehner +1/-1: "
                f"{flagger['refine_flags_lohner']}/{flagger['coarsen_flags_lohner']}")

    # adaptive run: Loehner flags and a regrid (plan, new forest, transfer)
    # every regrid_every steps, from the initial state, timed as a whole
    adaptive = None
    nad = args.adaptive_steps if args.adaptive_steps is not None else (20 if args.workload == "blast" else 0)
    if nad > 0:
        g.use_graph(False)
        g.set_schedule(*sched[:3])
        g.set_variant(sched[3])
        g.set_state(U0)
        ga = g
        t_ad, done, updates, regrid_ms, regrids, counts = 0.0, 0, 0, 0.0, 0, []
        use_mlp = args.adaptive_flagger == "mlp" and s.ndim > 1
        vs_lohner = []
        if use_mlp:
            from paper_2004_03275_amd import mlp as MLP

            wts = MLP.trained_weights()
            g.mlp_set_weights(wts)
            g.mlp_set_margin(2.0)
        g.synchronize()
        t0 = time.perf_counter()
        while done < nad:
            m = min(args.regrid_every, nad - done)
            t_ad, _ = ga.advance_cfl(m, float("inf"), t_ad)
            updates += ga.forest.n * s.cells_per_block * m
            done += m
            if done < nad:
                ga.synchronize()
                r0 = time.perf_counter()
                if use_mlp:
                    flags = ga.flag_blocks(mode=N.FLAG_MLP_FALLBACK)
                    if regrids % 2 == 1:
                        ref = ga.flag_blocks()
                        vs_lohner.append(float(np.mean((flags == 1) != (ref == 1))))
                else:
                    flags = ga.flag_blocks()
                nxt = ga.regrid(flags)
                if use_mlp:
                    nxt.mlp_set_weights(wts)
                    nxt.mlp_set_margin(2.0)
                if ga is not g:
                    ga.close()
                ga = nxt
                regrid_ms += (time.perf_counter() - r0) * 1e3
                regrids += 1
                counts.append(ga.forest.n)
        ga.synchronize()
        ael = time.perf_counter() - t0
        adaptive = {"value": updates / ael / 1e6, "unit": "MCUPS", "steps": nad, "regrid_every": args.regrid_every,
                     "regrids": regrids, "regrid_ms_avg": regrid_ms / max(regrids, 1),
                     "leaves_after_each_regrid": counts, "final_levels": {str(k): v for k, v in
                                                                           ga.forest.level_counts().items()},
                     "flagger": "mlp_fallback" if use_mlp else "lohner",
                     "refine_disagreement_vs_lohner": vs_lohner if use_mlp else None,
                     "note": "cell updates of the current forest per step; regrid = flags, plan, new "
                             "forest (workspace, tables), transfer"}
        log(f"adaptive: {adaptive['value']:.1f} MCUPS over {nad} steps, {regrids} regrids of "
            f"{adaptive['regrid_ms_avg']:.1f} ms, leaves {counts}")
        if ga is not g:
            ga.close()

    rd = rd_amr = None
    if args.workload == "blast" and not args.no_rd:
        rd = rd_measure(2, 256, 20, 3, log, cpu=not args.no_cpu_baseline)
        rd_amr = gsamr_measure(10, 2, log, cpu=not args.no_cpu_baseline)

    counters = measured_counters(args.workload, ["minmod", "vanleer", "mc", "koren", "cada"][s.limiter], sched[3],
                                 args.arithmetic)
    names = {0: "per_block", 1: "grid", 2: "persistent"}
    bytes_per_cell_step = (2 + 3 * (s.rk_stages - 1)) * s.nvar * 8
    out = {
        "metric": METRIC,
        "value": mcups,
        "unit": "MCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "leaves": f.n,
            "levels": {str(k): v for k, v in f.level_counts().items()},
            "cells": cells,
            "block": list(s.block_nx[: s.ndim]),
            "nvar": s.nvar,
            "physics": ["euler", "mhd_glm", "polytrope"][s.physics],
            "flux": ["tvdlf", "hll", "hllc"][s.flux],
            "limiter": ["minmod", "vanleer", "mc", "koren", "cada"][s.limiter],
            "cada_radius": s.cada_radius,
            "rk_stages": s.rk_stages,
            "gamma": s.gamma,
            "cfl": s.cfl,
            "flag_every": args.flag_every,
            "schedule": {"mode": names[sched[0]], "xcd_remap": sched[1], "persistent_wgs": sched[2],
                         "stage_kernel_variant": ["combined_xy", "split_xy", "z_then_xy"][sched[3]]},
            "arithmetic": args.arithmetic,
            "graph": bool(args.graph) or not args.host_dt,
            "time_step": "host (amrv_max_dt + amrv_advance)" if args.host_dt else "device (amrv_advance_cfl)",
        },
        "step_roofline": {
            "bound": "hbm",
            "achieved": bytes_per_cell_step * cells / (ms_step / 1e3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": bytes_per_cell_step * cells / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_step": bytes_per_cell_step * cells,
            "note": "whole step (all launches, the timed region's flaggings included) against the interior-state "
                    "passes of the SSP stages",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_stage_zcol + k_stage_xy (stage update, two launches)" if sched[3] == 2
                       else "k_stage_tile (stage update)"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counters.get("traffic_bytes_per_launch"),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": kbytes / max(launches, 1),
            "avg_launch_ms": avg_ms,
            "launches": launches,
            "algorithmic_bytes_per_cell_step": bytes_per_cell_step,
            "valu_issue_frac": counters.get("valu_issue_frac"),
            "fp64_issue_frac": counters.get("fp64_issue_frac"),
            "counters": "profiles/hbm_counters_3d_amr_blast.md" if counters else None,
        },
        "cpu_baseline": cpu,
        "per_block": per_block,
        "parity": parity,
        "learned_flagger": flagger,
        "adaptive": adaptive,
        "reaction_diffusion": rd,
        "reaction_diffusion_amr": rd_amr,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
