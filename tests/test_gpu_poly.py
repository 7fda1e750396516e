"""GPU (HIP, gfx950) polytrope without energy equation (the paper's shallow
water runs, Sec. 2.2) against the CPU oracle, through the C-ABI.

With gamma = 2 (shallow water) every power is an exact product, so the
kernels match the oracle bit for bit; other exponents go through the device
pow and are held to the relative L1 bar of 1e-10.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gpu():
    from paper_2004_03275_amd import forest as F

    return F


def _report(name, G, R, f):
    e = W.relative_l1(G, R, f)
    print(f"[poly] {name}: max rel L1 {e.max():.3e}, differing {int(np.count_nonzero(G != R))}/{G.size}",
          flush=True)
    return e


def _dam_small(flux=W.HLL, lim=W.KOREN):
    s = W.dam_break_scheme(base=4, max_level=3, flux=flux)
    s.limiter = lim
    return W.dam_break(scheme=s, buffer_cells=2.0)


@pytest.mark.parametrize("flux,lim", [(W.HLL, W.KOREN), (W.TVDLF, W.MINMOD), (W.HLL, W.VANLEER),
                                      (W.HLL, W.CADA)])
def test_dam_break_amr_bitwise(flux, lim):
    F = _gpu()
    f, U = _dam_small(flux, lim)
    print(f"[poly] dam break levels {f.level_counts()}", flush=True)
    R, dts = oracle.run(f, U, steps=12)
    G, used = F.run(f, U, steps=12)
    assert used == dts
    _report(f"dam break flux={flux} lim={lim}", G, R, f)
    assert np.array_equal(G, R)


def test_dam_break_device_timed_steps_and_variants():
    F = _gpu()
    f, U = _dam_small()
    R, dts = oracle.run(f, U, t_end=1.0)
    G, used = F.run(f, U, t_end=1.0, device_dt=True, chunk=16)
    assert len(used) == len(dts)
    assert np.array_equal(G, R)
    for sched in [(1, 1, 0), (2, 0, 0), (2, 1, 0)]:
        G, _ = F.run(f, U, steps=6, schedule=sched)
        R6, _ = oracle.run(f, U, steps=6)
        assert np.array_equal(G, R6), sched


def test_lake_at_rest_bitwise():
    F = _gpu()
    f, _ = _dam_small()
    shape = W.cell_centres(f)[0].shape
    U = W.state_from_primitive(f, np.full(shape, 1.3), [np.zeros(shape)] * 2)
    G, _ = F.run(f, U, steps=10)
    assert np.array_equal(G, U)


@pytest.mark.parametrize("nd", [1, 2])
def test_pow_exponent_matches_oracle(nd):
    """gamma = 1.4, c_ad = 1: p and c through pow on both sides."""
    F = _gpu()
    if nd == 1:
        s = W.Scheme(ndim=1, block_nx=(128,), base_blocks=(8,), max_level=1, xmin=(-10.0,), xmax=(10.0,),
                     physics=W.POLY, gamma=1.4, cad=1.0, flux=W.HLL, limiter=W.KOREN, rk_stages=3, cfl=0.9,
                     bc=W.ZERO_GRADIENT)
        f = W.uniform_forest(s)
        (x,) = W.cell_centres(f)
        U = W.state_from_primitive(f, np.where(x < 0.0, 1.0, 0.2), [np.where(x < 0.0, 0.2, -0.1)])
    else:
        s = W.dam_break_scheme(base=4, max_level=3)
        s.gamma, s.cad = 1.4, 1.0
        f, U = W.dam_break(scheme=s, buffer_cells=2.0)
    R, dts = oracle.run(f, U, steps=20)
    G, _ = F.run(f, U, dts=dts)
    e = _report(f"pow exponent {nd}D", G, R, f)
    assert e.max() <= TOL


def test_flags_and_features_match_oracle():
    F = _gpu()
    f, U = _dam_small()
    R, dts = oracle.run(f, U, steps=5)
    o = oracle.OracleForest(f)
    o.set_state(R)
    g = F.GpuForest(f)
    g.set_state(R)
    fo, eo = o.flag_blocks(with_emax=True)
    fg, eg = g.flag_blocks(with_emax=True)
    print(f"[poly] flags refine {int((fo == 1).sum())} coarsen {int((fo == -1).sum())}", flush=True)
    assert np.array_equal(fo, fg)
    assert np.array_equal(eo, eg)
    Xg = g.mlp_features()
    Xo = M.features(R, 2, f.scheme.gamma, cad=f.scheme.cad)
    assert np.array_equal(Xg, Xo)


def test_rejects_hllc_and_nonphysical_state():
    F = _gpu()
    from paper_2004_03275_amd import _native as N

    s = W.dam_break_scheme(base=2, max_level=1)
    s.flux = W.HLLC
    with pytest.raises(N.AmrvError) as e:
        F.GpuForest(W.uniform_forest(s))
    assert e.value.code == -1
    f, U = _dam_small()
    g = F.GpuForest(f)
    V = U.copy()
    V[0, 3, 2, 2] = -0.1
    g.set_state(V)
    with pytest.raises(N.AmrvError) as e:
        g.max_dt()
    assert e.value.code == -3
