"""GPU (HIP, gfx950) results against the CPU oracle, through the C-ABI.

Both sides get the same seeded inputs.  The bar is the relative L1 of every
conserved variable <= 1e-10 (sum |U_gpu - U_orc| dV over max(sum |U_orc| dV,
1e-6 sum |E_orc| dV)); the kernels evaluate every expression in the oracle's
order with contraction off, so most cases also match bit for bit, which is
asserted where it holds by construction (same dt sequence).  Refinement flags
must be identical.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gpu():
    from paper_2004_03275_amd import forest as F

    return F


def rel_l1(U, R, forest):
    return W.relative_l1(U, R, forest)


def _report(name, U, R, f):
    e = rel_l1(U, R, f)
    nbad = int(np.count_nonzero(U != R))
    print(f"[parity] {name}: max rel L1 {e.max():.3e}, differing values {nbad}/{U.size}", flush=True)
    return e


def _amr2d(flux=W.HLLC, physics=W.EULER, lim=W.VANLEER):
    s = W.Scheme(ndim=2, block_nx=(16, 16), base_blocks=(4, 4), max_level=3, physics=physics,
                 gamma=1.4 if physics == W.EULER else 5.0 / 3.0, flux=flux, limiter=lim, rk_stages=3, cfl=0.8,
                 bc=W.PERIODIC)

    def refine(l, c):
        nb = 4 << (l - 1)
        return abs((c[0] + 0.5) / nb - 0.5) < 0.2 and abs((c[1] + 0.5) / nb - 0.45) < 0.2

    return W.refined_forest(s, refine)


def _blast_small(base=2, max_level=3, radius=0.2, buffer_cells=2.0):
    s = W.blast_scheme(base=base, max_level=max_level)
    f = W.blast_forest(s, radius=radius, buffer_cells=buffer_cells)
    return W.blast(s, radius=radius, forest=f)


# ---------------------------------------------------------------------------


def test_device_division_and_sqrt_are_correctly_rounded():
    """The parity argument needs IEEE-correct binary64 / and sqrt on gfx950:
    a 1D free-stream state with random values exercises them through to_prim
    and the sound speed; compare the CFL result with the host's."""
    F = _gpu()
    rng = np.random.default_rng(7)
    f, U = W.sod(1024)
    rho = rng.uniform(0.1, 10.0, (1, 1024))
    p = rng.uniform(0.01, 100.0, (1, 1024))
    u = rng.uniform(-3, 3, (1, 1024))
    U = W.state_from_primitive(f, rho, [u], p)
    g = F.GpuForest(f)
    o = oracle.OracleForest(f)
    for trial in range(20):
        rho = rng.uniform(0.1, 10.0, (1, 1024))
        p = rng.uniform(0.01, 100.0, (1, 1024))
        u = rng.uniform(-3, 3, (1, 1024))
        U = W.state_from_primitive(f, rho, [u], p)
        g.set_state(U)
        o.set_state(U)
        assert g.max_dt() == o.max_dt()


def test_sod_cfl_closed_form_bitwise():
    F = _gpu()
    f, U = W.sod(1024)
    g = F.GpuForest(f)
    g.set_state(U)
    assert g.max_dt() == 0.8 / (1024 * math.sqrt(1.4))


def test_sod_full_run_matches_oracle():
    F = _gpu()
    f, U = W.sod(1024)
    R, dts = oracle.run(f, U, t_end=0.2)
    G, gdts = F.run(f, U, t_end=0.2)
    assert len(gdts) == len(dts)
    e = _report("sod t=0.2", G, R, f)
    assert e.max() <= TOL
    assert np.array_equal(G, R)


@pytest.mark.parametrize("flux,lim", [(W.HLLC, W.VANLEER), (W.HLL, W.MINMOD), (W.TVDLF, W.VANLEER), (W.HLLC, W.MC),
                                      (W.TVDLF, W.MC), (W.HLLC, W.KOREN), (W.HLL, W.KOREN),
                                      (W.HLLC, W.CADA), (W.TVDLF, W.CADA)])
def test_kh_small_matches_oracle(flux, lim):
    F = _gpu()
    s = W.kh_scheme(4)
    s.flux, s.limiter = flux, lim
    f, U = W.kh(scheme=s)
    R, dts = oracle.run(f, U, steps=30)
    G, _ = F.run(f, U, steps=30)
    e = _report(f"kh 4x4 flux={flux} lim={lim}", G, R, f)
    assert e.max() <= TOL
    assert np.array_equal(G, R)


def test_orszag_tang_small_matches_oracle():
    F = _gpu()
    f, U = W.orszag_tang(4)
    R, dts = oracle.run(f, U, steps=30)
    G, _ = F.run(f, U, steps=30)
    e = _report("ot 4x4", G, R, f)
    assert e.max() <= TOL
    assert np.array_equal(G, R)


@pytest.mark.parametrize("flux", [W.HLLC, W.HLL])
def test_amr2d_matches_oracle(flux):
    F = _gpu()
    f = _amr2d(flux=flux)
    xs = W.cell_centres(f)
    inner = np.abs(xs[1] - 0.5) < 0.25
    rho = np.where(inner, 2.0, 1.0)
    u = np.where(inner, 0.5, -0.5)
    v = 0.05 * np.sin(4 * np.pi * xs[0])
    U = W.state_from_primitive(f, rho, [u, v], np.full_like(rho, 2.5))
    R, dts = oracle.run(f, U, steps=12)
    G, _ = F.run(f, U, dts=dts)
    e = _report(f"amr2d flux={flux} ({f.level_counts()})", G, R, f)
    assert e.max() <= TOL
    assert np.array_equal(G, R)


def test_blast_small_amr_matches_oracle():
    F = _gpu()
    f, U = _blast_small()
    R, dts = oracle.run(f, U, steps=3)
    G, _ = F.run(f, U, dts=dts)
    e = _report(f"blast small ({f.level_counts()})", G, R, f)
    assert e.max() <= TOL
    assert np.array_equal(G, R)


@pytest.mark.parametrize("lim", [W.MC, W.MINMOD, W.KOREN, W.CADA])
def test_blast_small_other_limiters_match_oracle(lim):
    F = _gpu()
    f, U = _blast_small()
    f.scheme.limiter = lim
    R, dts = oracle.run(f, U, steps=3)
    G, _ = F.run(f, U, dts=dts)
    _report(f"blast small limiter {lim}", G, R, f)
    assert np.array_equal(G, R)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("lim", [W.KOREN, W.CADA])
def test_asymmetric_limiters_both_variants_match_oracle(lim, variant):
    """Koren and Cada in the combined variant (both face states formed in the
    flux phase, no slope phase) and in the split variant (two stored half
    slopes per cell): both bit for bit the oracle's, 3D AMR and 2D."""
    F = _gpu()
    for f, U in (_blast_small(), W.kh(4)):
        f.scheme.limiter = lim
        R, dts = oracle.run(f, U, steps=3)
        G, _ = F.run(f, U, dts=dts, variant=variant)
        _report(f"{f.scheme.ndim}D limiter {lim} variant {variant}", G, R, f)
        assert np.array_equal(G, R)


@pytest.mark.parametrize("n,nb,flux,lim", [(1000, 1, W.TVDLF, W.MINMOD), (900, 3, W.HLLC, W.VANLEER),
                                          (1000, 1, W.HLL, W.CADA), (68, 1, W.HLLC, W.KOREN)])
def test_ragged_1d_blocks_match_oracle(n, nb, flux, lim):
    """1D leaves whose length is not a multiple of the 256-cell chunk of a
    workgroup (1000 = 3*256 + 232, 300, 68): the last chunk is partial."""
    F = _gpu()
    f, U = W.sod(n, nblocks=nb)
    f.scheme.flux, f.scheme.limiter = flux, lim
    R, dts = oracle.run(f, U, t_end=0.1)
    G, used = F.run(f, U, t_end=0.1)
    assert len(used) == len(dts)
    _report(f"ragged 1D n={n} blocks={nb}", G, R, f)
    assert np.array_equal(G, R)


@pytest.mark.parametrize("case", ["blast3d", "kh2d", "sod1d", "mhd2d"])
def test_cada_switch_matches_oracle(case):
    """Cada's limiter with its smoothness switch (the radius scales with each
    level's cell size): exercised in the 3D, 2D, 1D and MHD kernels and in the
    fine-side fluxes of coarse-fine faces."""
    F = _gpu()
    if case == "blast3d":
        f, U = _blast_small()
        f.scheme.limiter, f.scheme.cada_radius = W.CADA, 0.5
        steps = 3
    elif case == "kh2d":
        f, U = W.kh(4)
        f.scheme.limiter, f.scheme.cada_radius = W.CADA, 0.3
        steps = 20
    elif case == "sod1d":
        f, U = W.sod(1000, nblocks=4)
        f.scheme.limiter, f.scheme.cada_radius = W.CADA, 0.5
        steps = 60
    else:
        s = W.mhd_blast_scheme(2, base=2, max_level=3)
        s.cada_radius = 0.2
        f, U = W.mhd_blast(2, scheme=s)
        steps = 6
    R, dts = oracle.run(f, U, steps=steps)
    G, _ = F.run(f, U, dts=dts)
    _report(f"cada switch {case}", G, R, f)
    assert np.array_equal(G, R)


@pytest.mark.parametrize("lim", [W.MC, W.KOREN, W.CADA])
def test_sod_other_limiters_match_oracle(lim):
    F = _gpu()
    f, U = W.sod(1024, nblocks=8)
    f.scheme.limiter = lim
    R, dts = oracle.run(f, U, t_end=0.2)
    G, gdts = F.run(f, U, t_end=0.2)
    assert len(gdts) == len(dts)
    assert np.array_equal(G, R)


def test_orszag_tang_hllc_matches_oracle():
    F = _gpu()
    f, U = W.orszag_tang(4)
    f.scheme.flux = W.HLLC
    R, dts = oracle.run(f, U, steps=20)
    G, _ = F.run(f, U, dts=dts)
    assert np.array_equal(G, R)


def test_orszag_tang_koren_matches_oracle():
    F = _gpu()
    f, U = W.orszag_tang(4)
    f.scheme.limiter = W.KOREN
    R, dts = oracle.run(f, U, steps=20)
    G, _ = F.run(f, U, dts=dts)
    assert np.array_equal(G, R)


@pytest.mark.parametrize("nd,flux", [(2, W.HLLC), (3, W.HLLC), (2, W.HLL), (3, W.HLL)])
def test_mhd_blast_matches_oracle(nd, flux):
    """The paper's MHD blast (Sec. 2.4) on a small AMR forest, with the
    Courant ramp: exercises the 2D and 3D MHD stage kernels."""
    F = _gpu()
    f, U = W.mhd_blast(nd, scheme=W.mhd_blast_scheme(nd, base=2, max_level=3, flux=flux))
    R, dts = oracle.run(f, U, steps=6, ramp_steps=10)
    G, gdts = F.run(f, U, steps=6, ramp_steps=10)
    assert gdts == dts
    _report(f"mhd blast {nd}D ({f.level_counts()})", G, R, f)
    assert np.array_equal(G, R)


@pytest.mark.parametrize("flux,lim", [(W.HLLC, W.CADA), (W.HLL, W.CADA), (W.HLLC, W.VANLEER), (W.TVDLF, W.MINMOD)])
def test_mhd_3d_two_launch_variant_matches_oracle(flux, lim):
    """Stage-kernel variant 2 of the 3D MHD forests (the z direction of every
    column in one launch, then the x/y planes with the face states formed in
    place) on the paper's MHD blast: bit for bit the oracle's under the grid
    (XCD remap), persistent and per-block schedules and with graph replay,
    and with a symmetric and an asymmetric limiter."""
    F = _gpu()
    f, U = W.mhd_blast(3, scheme=W.mhd_blast_scheme(3, base=2, max_level=3, flux=flux, limiter=lim))
    R, dts = oracle.run(f, U, steps=4, ramp_steps=10)
    for sched, graph in [((1, 1, 0), False), ((2, 0, 0), True), ((2, 1, 24), False), ((0, 0, 0), False)]:
        G, gdts = F.run(f, U, steps=4, ramp_steps=10, schedule=sched, graph=graph, variant=2)
        assert gdts == dts
        _report(f"mhd blast 3D variant 2 flux={flux} lim={lim} sched={sched} graph={graph}", G, R, f)
        assert np.array_equal(G, R)


def test_two_launch_variant_is_3d_mhd_only():
    from paper_2004_03275_amd import _native as N

    F = _gpu()
    for f, _ in (W.mhd_blast(2, scheme=W.mhd_blast_scheme(2, base=2, max_level=2)), _blast_small()):
        g = F.GpuForest(f)
        with pytest.raises(N.AmrvError):
            g.set_variant(2)
        g.close()


def test_flags_identical():
    F = _gpu()
    for name, (f, U) in {"kh": W.kh(4), "blast": _blast_small(), "ot": W.orszag_tang(4)}.items():
        o = oracle.OracleForest(f)
        o.set_state(U)
        g = F.GpuForest(f)
        g.set_state(U)
        fo, eo = o.flag_blocks(with_emax=True)
        fg, eg = g.flag_blocks(with_emax=True)
        print(f"[flags] {name}: {np.bincount(fo + 1, minlength=3)} max|de|={np.abs(eo - eg).max():.3e}", flush=True)
        assert np.array_equal(fo, fg), name
        assert np.array_equal(eo, eg), name


def test_schedules_and_graph_are_bitwise_equal():
    F = _gpu()
    f, U = _blast_small()
    dts = [1e-4, 1.2e-4]
    outs = []
    for sched, graph, var in [((0, 0, 0), False, 0), ((1, 0, 0), False, 0), ((1, 1, 0), False, 1),
                              ((2, 0, 64), False, 1), ((1, 1, 0), True, 0), ((2, 0, 0), True, 1),
                              ((0, 0, 0), False, 1), ((2, 1, 0), False, 0), ((2, 1, 24), True, 0),
                              ((2, 1, 0), False, 1)]:
        G, _ = F.run(f, U, dts=dts, schedule=sched, graph=graph, variant=var)
        outs.append(G)
    for G in outs[1:]:
        assert np.array_equal(G, outs[0])


def test_nonphysical_and_bad_dt_are_reported():
    F = _gpu()
    from paper_2004_03275_amd import _native as N

    f, U = W.kh(2)
    g = F.GpuForest(f)
    V = U.copy()
    V[0, 1, 3, 4] = -1.0
    g.set_state(V)
    with pytest.raises(N.AmrvError) as e:
        g.max_dt()
    assert e.value.code == N.ENONPHYSICAL
    V = U.copy()
    V[2, 0, 0, 0] = np.nan
    g.set_state(V)
    with pytest.raises(N.AmrvError) as e:
        g.max_dt()
    assert e.value.code == N.ENONPHYSICAL
    g.set_state(U)
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(N.AmrvError) as e:
            g.advance(dt)
        assert e.value.code == N.EINVAL


def test_device_timed_steps_match_oracle():
    """amrv_advance_cfl: time steps chosen on the device from the fused
    Courant reduction, many steps per host call (graph replay)."""
    F = _gpu()
    f, U = W.sod(1024)
    R, dts = oracle.run(f, U, t_end=0.2)
    G, used = F.run(f, U, t_end=0.2, device_dt=True, chunk=64)
    assert len(used) == len(dts)
    assert np.array_equal(G, R)
    f, U = W.kh(4)
    R, _ = oracle.run(f, U, steps=40)
    G, _ = F.run(f, U, steps=40, device_dt=True, chunk=16)
    assert np.array_equal(G, R)
    f, U = _blast_small()
    R, _ = oracle.run(f, U, steps=3)
    for sched in [(2, 0, 0), (1, 1, 0), (2, 1, 0)]:
        G, _ = F.run(f, U, steps=3, device_dt=True, schedule=sched)
        _report(f"blast device-dt sched {sched}", G, R, f)
        assert np.array_equal(G, R)
    # the step count reported by the device (every schedule), to an end time
    R, dts = oracle.run(f, U, t_end=2e-3)
    for sched in [(1, 1, 0), (2, 0, 0), (2, 1, 0)]:
        G, used = F.run(f, U, t_end=2e-3, device_dt=True, schedule=sched, chunk=4)
        assert len(used) == len(dts), (sched, len(used), len(dts))
        assert np.array_equal(G, R)
    f, U = W.orszag_tang(4)
    R, _ = oracle.run(f, U, steps=30)
    G, _ = F.run(f, U, steps=30, device_dt=True, chunk=10)
    e = _report("ot device-dt", G, R, f)
    assert e.max() <= TOL


def test_device_timed_calls_reuse_the_fold_only_while_valid():
    """Consecutive amrv_advance_cfl calls reuse the Courant reduction folded
    by the previous call's last step; set_state or a host-timed step in
    between forces a fresh one."""
    F = _gpu()
    f, U = W.kh(4)
    R, _ = oracle.run(f, U, steps=6)
    g = F.GpuForest(f)
    g.set_state(U)
    t, n = g.advance_cfl(3, float("inf"), 0.0)
    t, n2 = g.advance_cfl(3, float("inf"), t)
    assert n == n2 == 3 and np.array_equal(g.get_state(), R)
    # a new state: the stale fold must not be used
    g.set_state(U)
    g.advance_cfl(2, float("inf"), 0.0)
    g.set_state(U)
    t, _ = g.advance_cfl(6, float("inf"), 0.0)
    assert np.array_equal(g.get_state(), R)
    # a host-timed step in between
    R2, dts = oracle.run(f, U, steps=5)
    g.set_state(U)
    t, _ = g.advance_cfl(2, float("inf"), 0.0)
    dt = g.max_dt()
    g.advance(dt)
    t, _ = g.advance_cfl(2, float("inf"), t + dt)
    assert np.array_equal(g.get_state(), R2)
    g.close()


def test_device_timed_run_reports_nonphysical_state():
    """A non-physical state met during a device-timed run is reported, with
    every schedule (the per-step queue reset must not clear the flag)."""
    F = _gpu()
    from paper_2004_03275_amd import _native as N

    f, U = W.kh(2)
    V = U.copy()
    V[0, 1, 3, 4] = -1.0
    for sched in [(1, 1, 0), (2, 0, 0), (2, 1, 0)]:
        g = F.GpuForest(f)
        g.set_schedule(*sched)
        g.set_state(V)
        with pytest.raises(N.AmrvError) as e:
            g.advance_cfl(3, float("inf"), 0.0)
        assert e.value.code == N.ENONPHYSICAL, sched
        g.close()


def test_autotune_keeps_state_and_parity():
    F = _gpu()
    f, U = _blast_small()
    g = F.GpuForest(f)
    g.set_state(U)
    sched = g.autotune(2)
    rep = g.autotune_report()
    print(f"[tune] chose {sched}\n{rep}", flush=True)
    assert np.array_equal(g.get_state(), U)
    # every candidate did real work: no timing near launch overhead only
    times = [float(l.split("median")[1].split("ms")[0]) for l in rep.strip().splitlines()]
    assert min(times) > 0.02, times
    R, dts = oracle.run(f, U, steps=2)
    for dt in dts:
        g.max_dt()
        g.advance(dt)
    assert np.array_equal(g.get_state(), R)
