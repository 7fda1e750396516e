"""Parity at the workloads' full sizes, in the bench's launch configuration
(autotuned schedule), GPU against the oracle.

* KH: 256 leaves of 16^2, 1000 SSP-RK3 steps with each side's own Courant
  dt, compared every 100 steps;
* Orszag-Tang: 1024 leaves of 16^2, MHD + GLM, to t = 0.5, compared every
  200 steps and at the end;
* 3D AMR blast: 19,384 leaves of 16^3 on 4 levels, 2 steps, then identical
  Loehner flags and regrid;
* 3D AMR blast on the path bench.py times: autotuned schedule, HIP-graph
  replay, 20 steps of amrv_advance_cfl (device-computed dt) in chunks of 5,
  Loehner flags after steps 10 and 20 as in the timed region;
* the paper's 3D MHD blast (512 leaves of 16^3, 9 variables) through the
  two-launch stage update (variant 2), exact and fast arithmetic, 8 steps with
  the Courant ramp.
The bar is relative L1 <= 1e-10 per variable; the runs are in fact equal
bit for bit, which is asserted too.
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _pair(f, U, tune=True):
    from paper_2004_03275_amd.forest import GpuForest

    g = GpuForest(f)
    g.set_state(U)
    if tune:
        g.autotune(2)
    o = oracle.OracleForest(f)
    o.set_state(U)
    return g, o


def _check(name, g, o, f, step):
    G = g.get_state()
    R = o.get_state()
    e = W.relative_l1(G, R, f).max()
    print(f"[full] {name} step {step}: rel L1 {e:.3e}, bitwise {np.array_equal(G, R)}", flush=True)
    assert e <= TOL, (name, step, e)


def test_kh_full_1000_steps():
    f, U = W.kh(16)
    g, o = _pair(f, U)
    t0 = time.time()
    for step in range(1, 1001):
        dg, do = g.max_dt(), o.max_dt()
        assert dg == do, (step, dg, do)
        g.advance(dg)
        o.advance(do)
        if step % 100 == 0:
            _check("kh", g, o, f, step)
    print(f"[full] kh done in {time.time() - t0:.1f} s", flush=True)


def test_orszag_tang_full_to_t05():
    f, U = W.orszag_tang(32)
    g, o = _pair(f, U)
    t, step = 0.0, 0
    t0 = time.time()
    while t < 0.5:
        dg, do = g.max_dt(), o.max_dt()
        assert dg == do and g.glm_ch == o.glm_ch, (step, dg, do)
        dt = min(dg, 0.5 - t)
        g.advance(dt)
        o.advance(dt)
        t += dt
        step += 1
        if step % 200 == 0:
            _check("ot", g, o, f, step)
    _check("ot", g, o, f, step)
    print(f"[full] ot: {step} steps to t = 0.5 in {time.time() - t0:.1f} s", flush=True)


def test_blast_full_size_two_steps_and_flags():
    s = W.blast_scheme()
    f, U = W.blast(s, forest=W.blast_lohner_forest(s))
    g, o = _pair(f, U)
    for step in (1, 2):
        dg, do = g.max_dt(), o.max_dt()
        assert dg == do
        g.advance(dg)
        o.advance(do)
        _check("blast", g, o, f, step)
    fg, eg = g.flag_blocks(with_emax=True)
    fo, eo = o.flag_blocks(with_emax=True)
    print(f"[full] blast flags: refine {int(np.sum(fo == 1))}, keep {int(np.sum(fo == 0))}, "
          f"coarsen {int(np.sum(fo == -1))}; identical {np.array_equal(fg, fo)}", flush=True)
    assert np.array_equal(fg, fo)
    assert np.array_equal(eg, eo)
    # regrid on these flags: the same leaves and the same transferred state
    g2, o2 = g.regrid(fg), o.regrid(fo)
    assert np.array_equal(g2.forest.level, o2.forest.level) and np.array_equal(g2.forest.ijk, o2.forest.ijk)
    nbad = int(np.count_nonzero(g2.get_state() != o2.get_state()))
    print(f"[full] blast regrid: {f.n} -> {g2.forest.n} leaves {g2.forest.level_counts()}, differing values {nbad}",
          flush=True)
    assert nbad == 0


def test_blast_timed_path_20_steps():
    """The configuration the headline MCUPS is measured in, against the oracle,
    in both arithmetic modes: exact (bit for bit) and fast (the bench's mode,
    relative L1 <= 1e-10, identical flags)."""
    from paper_2004_03275_amd import _native as N
    from paper_2004_03275_amd.forest import GpuForest

    s = W.blast_scheme()
    f, U = W.blast(s, forest=W.blast_lohner_forest(s))
    gs = {}
    for mode in (N.ARITH_EXACT, N.ARITH_FAST):
        g = GpuForest(f)
        g.set_arithmetic(mode)
        g.set_state(U)
        sched = g.autotune(5)
        g.use_graph(True)
        gs[mode] = [g, 0.0]
        print(f"[full] timed path arithmetic {mode}: {f.n} leaves, schedule {sched}", flush=True)
    o = oracle.OracleForest(f)
    o.set_state(U)
    to = 0.0
    t0 = time.time()
    for chunk in range(1, 5):
        for mode, gt in gs.items():
            gt[1], taken = gt[0].advance_cfl(5, float("inf"), gt[1])
            assert taken == 5
        for _ in range(5):
            dt = o.max_dt()
            o.advance(dt)
            to += dt
        step = 5 * chunk
        R = o.get_state()
        for mode, (g, tg) in gs.items():
            G = g.get_state()
            e = W.relative_l1(G, R, f).max()
            same = bool(np.array_equal(G, R))
            print(f"[full] timed path arithmetic {mode} step {step}: t {tg:.15e} (oracle {to:.15e}), rel L1 {e:.3e}, "
                  f"bitwise {same} ({time.time() - t0:.0f} s)", flush=True)
            assert e <= TOL, (mode, step, e)
            if mode == N.ARITH_EXACT:
                assert tg == to and same, (step, e)
            else:
                assert abs(tg - to) <= 1e-12 * to
            del G
        del R
        if step % 10 == 0:
            fo, eo = o.flag_blocks(with_emax=True)
            for mode, (g, _) in gs.items():
                fg, eg = g.flag_blocks(with_emax=True)
                de = float(np.max(np.abs(eg - eo)))
                print(f"[full] timed path arithmetic {mode} flags at step {step}: refine {int(np.sum(fo == 1))}, "
                      f"coarsen {int(np.sum(fo == -1))}; identical {np.array_equal(fg, fo)}, max |emax diff| {de:.2e}",
                      flush=True)
                assert np.array_equal(fg, fo)
                if mode == N.ARITH_EXACT:
                    assert np.array_equal(eg, eo)
                else:
                    assert de <= 1e-10
    for g, _ in gs.values():
        g.close()
    o.close()


@pytest.mark.parametrize("arith", [0, 1])
def test_mhd_blast_3d_full_size_two_launch(arith):
    """The bench's 3D MHD workload through stage-kernel variant 2 with the
    grid schedule and graph replay, 8 steps with the host-chosen ramped dt:
    bit for bit in exact arithmetic, within the bar in fast arithmetic."""
    from paper_2004_03275_amd import _native as N
    from paper_2004_03275_amd import forest as F

    f, U = W.mhd_blast(3, base=4, max_level=3)
    t0 = time.time()
    R, dts = oracle.run(f, U, steps=8, ramp_steps=10)
    G, gdts = F.run(f, U, steps=8, ramp_steps=10, schedule=(N.SCHED_GRID, 1, 0), graph=True, variant=2,
                    arithmetic=N.ARITH_FAST if arith else N.ARITH_EXACT)
    e = W.relative_l1(G, R, f).max()
    print(f"[full] mhd blast 3D ({f.n} leaves) variant 2 arithmetic {arith}: rel L1 {e:.3e}, "
          f"bitwise {np.array_equal(G, R)}, dt equal {gdts == dts} ({time.time() - t0:.1f} s)", flush=True)
    if arith == 0:
        assert gdts == dts
        assert np.array_equal(G, R)
    else:
        assert e <= TOL
