"""The fast-arithmetic stage kernels (AMRV_ARITH_FAST: FMA contraction,
reciprocal and reciprocal-square-root estimates refined by Newton steps)
against the oracle, through the C-ABI.

The bar is the relative L1 difference <= 1e-10 per conserved variable over
the run (not bit-for-bit equality, which holds for the exact mode only).
Each case also checks that the fast kernels really ran: their result is not
bitwise equal to the exact path's.  The full-size 3D blast in fast mode is
in test_gpu_fullsize.py (the timed path).
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _run_both(f, U, **kw):
    from paper_2004_03275_amd import _native as N
    from paper_2004_03275_amd import forest as F

    fast, _ = F.run(f, U, arithmetic=N.ARITH_FAST, **kw)
    exact, _ = F.run(f, U, arithmetic=N.ARITH_EXACT, **kw)
    return fast, exact


def _check(name, f, G, E, R):
    e = W.relative_l1(G, R, f)
    print(f"[fast] {name}: rel L1 vs oracle {e.max():.3e}, differing from exact {int(np.count_nonzero(G != E))}"
          f"/{G.size}", flush=True)
    assert e.max() <= TOL
    assert np.array_equal(E, R)
    assert not np.array_equal(G, E)


def test_blast_small_amr_fast():
    s = W.blast_scheme(base=2, max_level=3)
    f = W.blast_forest(s, radius=0.2, buffer_cells=2.0)
    _, U = W.blast(s, radius=0.2, forest=f)
    R, dts = oracle.run(f, U, steps=4)
    G, E = _run_both(f, U, dts=dts)
    _check(f"blast small ({f.level_counts()})", f, G, E, R)


@pytest.mark.parametrize("flux,lim", [(W.HLLC, W.VANLEER), (W.HLL, W.MINMOD), (W.TVDLF, W.MC), (W.HLLC, W.KOREN),
                                      (W.HLL, W.CADA)])
def test_kh_small_fast(flux, lim):
    s = W.kh_scheme(4)
    s.flux, s.limiter = flux, lim
    f, U = W.kh(scheme=s)
    R, dts = oracle.run(f, U, steps=30)
    G, E = _run_both(f, U, dts=dts)
    _check(f"kh 4x4 flux={flux} lim={lim}", f, G, E, R)


def test_kh_full_1000_steps_fast():
    """KH at full size, 1000 steps, each side with its own Courant steps."""
    from paper_2004_03275_amd import _native as N
    from paper_2004_03275_amd.forest import GpuForest

    f, U = W.kh(16)
    g = GpuForest(f)
    g.set_arithmetic(N.ARITH_FAST)
    g.set_state(U)
    g.autotune(2)
    o = oracle.OracleForest(f)
    o.set_state(U)
    worst = 0.0
    for step in range(1, 1001):
        g.advance(g.max_dt())
        o.advance(o.max_dt())
        if step % 100 == 0:
            e = W.relative_l1(g.get_state(), o.get_state(), f).max()
            worst = max(worst, e)
            print(f"[fast] kh full step {step}: rel L1 {e:.3e}", flush=True)
            assert e <= TOL, (step, e)
    assert worst > 0.0  # the fast kernels ran


def test_dam_break_poly_fast():
    """The polytrope (shallow water) with a symmetric limiter in fast mode."""
    f, U = W.dam_break()
    f.scheme.limiter = W.MC
    R, dts = oracle.run(f, U, steps=10)
    G, E = _run_both(f, U, dts=dts)
    _check(f"dam break poly MC ({f.level_counts()})", f, G, E, R)


@pytest.mark.parametrize("flux,lim", [(W.HLLC, W.CADA), (W.HLL, W.VANLEER)])
def test_mhd_3d_two_launch_fast(flux, lim):
    """The 3D MHD blast through stage-kernel variant 2 (z columns, then x/y
    planes) in fast arithmetic: MHD-HLLC / HLL with the GLM sub-solve, the
    fast magnetosonic speed and Cada's limiter from the refined estimates."""
    f, U = W.mhd_blast(3, scheme=W.mhd_blast_scheme(3, base=2, max_level=3, flux=flux, limiter=lim))
    R, dts = oracle.run(f, U, steps=6, ramp_steps=10)
    G, E = _run_both(f, U, dts=dts, variant=2)
    _check(f"mhd blast 3D variant 2 flux={flux} lim={lim} ({f.level_counts()})", f, G, E, R)


@pytest.mark.parametrize("lim", [W.KOREN, W.CADA])
def test_blast_3d_asymmetric_limiters_fast(lim):
    """The combined 3D kernel with an asymmetric limiter (face states formed
    in the flux phase) in fast arithmetic."""
    s = W.blast_scheme(base=2, max_level=3)
    s.limiter = lim
    f = W.blast_forest(s, radius=0.2, buffer_cells=2.0)
    _, U = W.blast(s, radius=0.2, forest=f)
    R, dts = oracle.run(f, U, steps=4)
    G, E = _run_both(f, U, dts=dts, variant=0)
    _check(f"blast small lim={lim}", f, G, E, R)
