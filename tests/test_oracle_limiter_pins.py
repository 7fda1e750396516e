"""Pins of the oracle's slope limiters: minmod, van Leer, the monotonized
central ('woodward') limiter of the paper's Gresho vortex runs (Sec. 2.3.1)
and Koren's limiter of its shallow-water and Karman runs (Sec. 2.2, 2.3.2).
A limiter here takes the difference a on the side of the cell away from the
face and b toward it.  Values for hand-worked pairs, the symmetry and sign
properties of a TVD limiter (Koren's is deliberately asymmetric), the
central branch of the monotonized central limiter, the third-order branch
of Koren's, convergence of a smooth 1D entropy wave in the full scheme, and
mirror symmetry of a shock tube with the asymmetric limiter."""
import numpy as np
import pytest

import oracle
from paper_2004_03275_amd import workloads as W

MM, VL, MC, KO = W.MINMOD, W.VANLEER, W.MC, W.KOREN

# (a, b): difference away from and toward the face; expected slopes worked
# by hand.  minmod: smaller magnitude; van Leer: 2ab/(a+b); MC: min(|2a|,
# |a+b|/2, |2b|); Koren: min(|2a|, |a+2b|/3, |2b|), all with the common sign
TABLE = [
    ((1.0, 3.0), {MM: 1.0, VL: 1.5, MC: 2.0, KO: 2.0}),
    ((3.0, 1.0), {MM: 1.0, VL: 1.5, MC: 2.0, KO: 5.0 / 3.0}),
    ((4.0, 5.0), {MM: 4.0, VL: 40.0 / 9.0, MC: 4.5, KO: 14.0 / 3.0}),
    ((1.0, 10.0), {MM: 1.0, VL: 20.0 / 11.0, MC: 2.0, KO: 2.0}),
    ((2.0, 3.0), {KO: 8.0 / 3.0}),
    ((3.0, 2.0), {KO: 7.0 / 3.0}),
    ((1.0, 4.0), {KO: 2.0}),
    ((4.0, 1.0), {KO: 2.0}),
    ((2.0, 2.0), {MM: 2.0, VL: 2.0, MC: 2.0, KO: 2.0}),
    ((-1.0, -3.0), {MM: -1.0, VL: -1.5, MC: -2.0, KO: -2.0}),
    ((-6.0, -2.0), {MM: -2.0, VL: -3.0, MC: -4.0, KO: -10.0 / 3.0}),
    ((1.0, -1.0), {MM: 0.0, VL: 0.0, MC: 0.0, KO: 0.0}),
    ((0.0, 5.0), {MM: 0.0, VL: 0.0, MC: 0.0, KO: 0.0}),
    ((5.0, 0.0), {MM: 0.0, VL: 0.0, MC: 0.0, KO: 0.0}),
]


@pytest.mark.parametrize("ab,expect", TABLE)
def test_limiter_values(ab, expect):
    for kind, val in expect.items():
        got = oracle.limiter_value(kind, *ab)
        assert got == pytest.approx(val, rel=1e-15, abs=0.0), (kind, ab, got)


def test_limiter_properties():
    rng = np.random.default_rng(3)
    a = rng.normal(size=4000) * np.exp(rng.uniform(-8, 8, 4000))
    b = rng.normal(size=4000) * np.exp(rng.uniform(-8, 8, 4000))
    for kind in (MM, VL, MC, KO):
        for x, y in zip(a, b):
            p = oracle.limiter_value(kind, x, y)
            if kind != KO:
                assert p == oracle.limiter_value(kind, y, x)      # symmetric, bit for bit
            assert -p == oracle.limiter_value(kind, -x, -y)       # odd
            if x * y <= 0:
                assert p == 0.0
                continue
            lo, hi = min(abs(x), abs(y)), max(abs(x), abs(y))
            assert np.sign(p) == np.sign(x)
            assert abs(p) <= 2 * lo * (1 + 1e-15)                 # TVD region
            assert abs(p) <= hi * (1 + 1e-15) or kind in (MC, KO)
            if kind in (VL, MC):
                assert abs(p) >= lo * (1 - 1e-15)                 # second-order region
    # MC: the central difference whenever it is the smallest (1/3 <= a/b <= 3)
    for r in (1.0 / 3.0, 0.5, 1.0, 2.0, 3.0):
        assert oracle.limiter_value(MC, r, 1.0) == 0.5 * (r + 1.0)
    assert oracle.limiter_value(MC, 0.25, 1.0) == 0.5
    assert oracle.limiter_value(MC, 4.0, 1.0) == 2.0
    # Koren: the third-order combination (a + 2b)/3 while it is the smallest
    # (a/b between 2/5 and 4), i.e. the kappa = 1/3 face value; 2a below, 2b above
    for r in (0.5, 1.0, 2.0, 3.0, 4.0):
        assert oracle.limiter_value(KO, r, 1.0) == (r + 2.0) / 3.0
    assert oracle.limiter_value(KO, 0.25, 1.0) == 0.5
    assert oracle.limiter_value(KO, 0.1, 1.0) == 0.2
    assert oracle.limiter_value(KO, 5.0, 1.0) == 2.0


def _entropy_wave(n, lim, t_end=0.25):
    """rho = 1 + 0.2 sin(2 pi x), u = 1, p = 1 on a periodic [0, 1]: the exact
    solution is the profile shifted by t.  L1 error of rho at t_end."""
    s = W.Scheme(ndim=1, block_nx=(n // 4,), base_blocks=(4,), max_level=1, flux=W.HLLC, limiter=lim,
                 rk_stages=3, cfl=0.5, bc=W.PERIODIC)
    f = W.uniform_forest(s)
    (x,) = W.cell_centres(f)
    h = 1.0 / n
    # cell averages of the initial profile
    rho = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - h / 2)) - np.cos(2 * np.pi * (x + h / 2))) / (2 * np.pi * h)
    U = W.state_from_primitive(f, rho, [np.ones_like(rho)], np.ones_like(rho))
    R, dts = oracle.run(f, U, t_end=t_end)
    exact = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - t_end - h / 2)) - np.cos(2 * np.pi * (x - t_end + h / 2))) / (
        2 * np.pi * h)
    return float(np.abs(R[0] - exact).mean())


@pytest.mark.parametrize("lim", [VL, MC, KO])
def test_second_order_on_a_smooth_wave(lim):
    e = [_entropy_wave(n, lim) for n in (64, 128, 256)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 1.5, (e, orders)


def test_mc_sharper_than_minmod():
    assert _entropy_wave(128, MC) < 0.6 * _entropy_wave(128, MM)


def test_koren_sharper_than_van_leer():
    assert _entropy_wave(128, KO) < _entropy_wave(128, VL)


def test_mirrored_shock_tube_with_koren():
    """Sod tube and its mirror image (x -> 1 - x, u -> -u): with an
    asymmetric limiter the two faces of a cell take different slopes, and
    only the face-correct assignment keeps the mirror symmetry."""
    def run(mirror):
        f, U = W.sod(512, nblocks=8)
        f.scheme.limiter = KO
        if mirror:
            U = U[:, ::-1, ::-1].copy()
            U[1] = -U[1]
        R, _ = oracle.run(f, U, steps=60)
        return R
    A, B = run(False), run(True)
    Bm = B[:, ::-1, ::-1].copy()
    Bm[1] = -Bm[1]
    assert np.abs(A - Bm).max() <= 1e-12 * np.abs(A).max()
    assert oracle.limiter_value(KO, 1.0, 3.0) != oracle.limiter_value(KO, 3.0, 1.0)
