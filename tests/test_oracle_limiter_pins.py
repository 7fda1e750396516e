"""Pins of the oracle's slope limiters: minmod, van Leer, the monotonized
central ('woodward') limiter of the paper's Gresho vortex runs (Sec. 2.3.1),
Koren's limiter of its shallow-water and Karman runs (Sec. 2.2, 2.3.2) and
Cada's third-order limiter of its MHD blast runs (Sec. 2.4; the LimO3
function of Cada and Torrilhon 2009).
A limiter here takes the difference a on the side of the cell away from the
face and b toward it.  Values for hand-worked pairs, the symmetry and sign
properties of a TVD limiter (Koren's is deliberately asymmetric), the
central branch of the monotonized central limiter, the third-order branch
of Koren's, convergence of a smooth 1D entropy wave in the full scheme, and
mirror symmetry of a shock tube with the asymmetric limiters, the published
ratio form of Cada's limiter, exact face values of the third-order
limiters on a quadratic profile, and Cada's smoothness switch (the unlimited
third-order slope where both differences are small against a radius times
the cell size): its values, third-order convergence on the smooth wave and
limited shock tubes."""
import numpy as np
import pytest

import oracle
import workloads as W

MM, VL, MC, KO, CA = W.MINMOD, W.VANLEER, W.MC, W.KOREN, W.CADA

# (a, b): difference away from and toward the face; expected slopes worked
# by hand.  minmod: smaller magnitude; van Leer: 2ab/(a+b); MC: min(|2a|,
# |a+b|/2, |2b|); Koren: min(|2a|, |a+2b|/3, |2b|), all with the common sign;
# Cada (b > 0): max(0, min(p3, max(-a/2, min(2a, p3, 1.6 b)))), p3 = (a+2b)/3
TABLE = [
    ((1.0, 3.0), {MM: 1.0, VL: 1.5, MC: 2.0, KO: 2.0, CA: 2.0}),
    ((3.0, 1.0), {MM: 1.0, VL: 1.5, MC: 2.0, KO: 5.0 / 3.0, CA: 1.6}),
    ((4.0, 5.0), {MM: 4.0, VL: 40.0 / 9.0, MC: 4.5, KO: 14.0 / 3.0, CA: 14.0 / 3.0}),
    ((1.0, 10.0), {MM: 1.0, VL: 20.0 / 11.0, MC: 2.0, KO: 2.0, CA: 2.0}),
    ((2.0, 3.0), {KO: 8.0 / 3.0, CA: 8.0 / 3.0}),
    ((3.0, 2.0), {KO: 7.0 / 3.0, CA: 7.0 / 3.0}),
    ((1.0, 4.0), {KO: 2.0, CA: 2.0}),
    ((4.0, 1.0), {KO: 2.0, CA: 1.6}),
    ((2.0, 2.0), {MM: 2.0, VL: 2.0, MC: 2.0, KO: 2.0, CA: 2.0}),
    ((-1.0, -3.0), {MM: -1.0, VL: -1.5, MC: -2.0, KO: -2.0, CA: -2.0}),
    ((-6.0, -2.0), {MM: -2.0, VL: -3.0, MC: -4.0, KO: -10.0 / 3.0, CA: -3.2}),
    ((1.0, -1.0), {MM: 0.0, VL: 0.0, MC: 0.0, KO: 0.0, CA: -1.0 / 3.0}),
    ((-1.0, 1.0), {CA: 1.0 / 3.0}),
    ((-0.5, 1.0), {CA: 0.25}),
    ((-1.5, 1.0), {CA: 1.0 / 6.0}),
    ((-2.0, 1.0), {CA: 0.0}),
    ((-3.0, 1.0), {CA: 0.0}),
    ((0.0, 5.0), {MM: 0.0, VL: 0.0, MC: 0.0, KO: 0.0, CA: 0.0}),
    ((5.0, 0.0), {MM: 0.0, VL: 0.0, MC: 0.0, KO: 0.0, CA: 0.0}),
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


def _cada_ratio_form(a, b):
    """The published form: b H(theta), theta = a/b."""
    t = a / b
    p3 = (2.0 + t) / 3.0
    return b * max(0.0, min(p3, max(-0.5 * t, min(2.0 * t, p3, 1.6))))


def test_cada_properties():
    rng = np.random.default_rng(5)
    a = rng.normal(size=6000) * np.exp(rng.uniform(-6, 6, 6000))
    b = rng.normal(size=6000) * np.exp(rng.uniform(-6, 6, 6000))
    n_extremum = 0
    for x, y in zip(a, b):
        p = oracle.limiter_value(CA, x, y)
        assert -p == oracle.limiter_value(CA, -x, -y)                 # odd, bit for bit
        assert p == pytest.approx(_cada_ratio_form(x, y), rel=4e-16, abs=4e-16 * abs(y))
        assert p * y >= 0.0 and abs(p) <= 1.6 * abs(y)                # 0 <= H <= 1.6
        t = x / y
        if -2.0 <= t <= -0.8 or 0.4 <= t <= 2.8:                      # third-order branch
            assert p == (x + 2.0 * y) / 3.0
        elif -0.8 < t < 0.0:
            assert p == -0.5 * x
        elif t > 2.8:
            assert p == 1.6 * y
        elif 0.0 <= t < 0.4:
            assert p == 2.0 * x
        else:
            assert p == 0.0
        n_extremum += (x * y < 0) and p != 0.0
    assert n_extremum > 500          # keeps a slope at extrema, unlike the TVD limiters
    assert oracle.limiter_value(CA, 1.0, 3.0) != oracle.limiter_value(CA, 3.0, 1.0)


@pytest.mark.parametrize("lim", [KO, CA])
def test_third_order_limiters_exact_on_a_quadratic(lim):
    """Cell averages of x^2 on cells [ih, (i+1)h], i >= 1: the two
    differences are 2i h^2 and (2i+2) h^2, their ratio lies in the
    third-order branch, and the reconstructed face values are the exact
    point values i^2 h^2 and (i+1)^2 h^2."""
    h = 0.01
    avg = lambda i: h * h * (i * i + i + 1.0 / 3.0)
    for i in range(1, 60):
        dm, dp = avg(i) - avg(i - 1), avg(i + 1) - avg(i)
        hi = avg(i) + 0.5 * oracle.limiter_value(lim, dm, dp)
        lo = avg(i) - 0.5 * oracle.limiter_value(lim, dp, dm)
        assert hi == pytest.approx((i + 1) ** 2 * h * h, rel=1e-12)
        assert lo == pytest.approx(i * i * h * h, rel=1e-12)
    # a TVD second-order limiter is not exact there
    i = 5
    dm, dp = avg(i) - avg(i - 1), avg(i + 1) - avg(i)
    assert avg(i) + 0.5 * oracle.limiter_value(VL, dm, dp) != pytest.approx((i + 1) ** 2 * h * h, rel=1e-6)


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


@pytest.mark.parametrize("lim", [VL, MC, KO, CA])
def test_second_order_on_a_smooth_wave(lim):
    e = [_entropy_wave(n, lim) for n in (64, 128, 256)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 1.5, (e, orders)


def test_mc_sharper_than_minmod():
    assert _entropy_wave(128, MC) < 0.6 * _entropy_wave(128, MM)


def test_koren_sharper_than_van_leer():
    assert _entropy_wave(128, KO) < _entropy_wave(128, VL)


def test_third_order_limiters_beat_second_order_on_a_smooth_wave():
    e = {lim: [_entropy_wave(n, lim) for n in (64, 128, 256)] for lim in (KO, CA)}
    for lim in (KO, CA):
        assert np.log2(e[lim][1] / e[lim][2]) > 2.15, (lim, e[lim])
        assert e[lim][2] < 0.4 * _entropy_wave(256, VL)


@pytest.mark.parametrize("lim", [KO, CA])
def test_mirrored_shock_tube_with_asymmetric_limiters(lim):
    """Sod tube and its mirror image (x -> 1 - x, u -> -u): with an
    asymmetric limiter the two faces of a cell take different slopes, and
    only the face-correct assignment keeps the mirror symmetry."""
    def run(mirror):
        f, U = W.sod(512, nblocks=8)
        f.scheme.limiter = lim
        if mirror:
            U = U[:, ::-1, ::-1].copy()
            U[1] = -U[1]
        R, _ = oracle.run(f, U, steps=60)
        return R
    A, B = run(False), run(True)
    Bm = B[:, ::-1, ::-1].copy()
    Bm[1] = -Bm[1]
    assert np.abs(A - Bm).max() <= 1e-12 * np.abs(A).max()
    assert oracle.limiter_value(lim, 1.0, 3.0) != oracle.limiter_value(lim, 3.0, 1.0)


# ---------------------------------------------------------------------------
# Cada's smoothness switch: thr2 = (r dx)^2
# ---------------------------------------------------------------------------


def test_cada_switch_values():
    rng = np.random.default_rng(11)
    for _ in range(4000):
        a, b = rng.normal(size=2) * np.exp(rng.uniform(-4, 4, 2))
        thr2 = float(np.exp(rng.uniform(-8, 8)))
        p = oracle.limiter_value(CA, a, b, thr2)
        if a * a + b * b <= thr2:
            assert p == (a + 2.0 * b) / 3.0          # unlimited, also at extrema
        else:
            assert p == oracle.limiter_value(CA, a, b)
    # at an extremum the switch keeps the third-order slope, LimO3 a smaller one
    assert oracle.limiter_value(CA, -1.0, 2.0, 10.0) == 1.0
    assert oracle.limiter_value(CA, -1.0, 2.0) == 0.5
    assert oracle.limiter_value(CA, 0.0, 3.0, 10.0) == 2.0
    assert oracle.limiter_value(CA, 0.0, 3.0) == 0.0
    # other limiters ignore it
    for kind in (MM, VL, MC, KO):
        assert oracle.limiter_value(kind, -1.0, 2.0, 10.0) == oracle.limiter_value(kind, -1.0, 2.0)


def _entropy_wave_r(n, r, t_end=0.25):
    s = W.Scheme(ndim=1, block_nx=(n // 4,), base_blocks=(4,), max_level=1, flux=W.HLLC, limiter=CA,
                 rk_stages=3, cfl=0.5, bc=W.PERIODIC, cada_radius=r)
    f = W.uniform_forest(s)
    (x,) = W.cell_centres(f)
    h = 1.0 / n
    sav = lambda y: (np.cos(2 * np.pi * (y - h / 2)) - np.cos(2 * np.pi * (y + h / 2))) / (2 * np.pi * h)
    U = W.state_from_primitive(f, 1.0 + 0.2 * sav(x), [np.ones_like(x)], np.ones_like(x))
    R, _ = oracle.run(f, U, t_end=t_end)
    return float(np.abs(R[0] - (1.0 + 0.2 * sav(x - t_end))).mean())


def test_cada_switch_gives_third_order_on_a_smooth_wave():
    """The limited function clips the slopes next to the wave's extrema
    (about second order); with the switch the scheme is third order."""
    e = [_entropy_wave_r(n, 1.0) for n in (64, 128, 256)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 2.9, (e, orders)
    assert e[2] < 0.05 * _entropy_wave_r(256, 0.0)


def test_cada_switch_still_limits_a_shock_tube():
    """Across the Sod tube's jumps the differences exceed any small radius:
    the solution stays as close to the exact one as without the switch."""
    from oracle import exact_riemann as E

    def err(r):
        f, U = W.sod(512, nblocks=8)
        f.scheme.limiter, f.scheme.cada_radius = CA, r
        R, _ = oracle.run(f, U, t_end=0.2)
        (x,) = W.cell_centres(f)
        rho, _, _ = E.sod_profile(x.ravel(), 0.2)
        return float(np.abs(R[0].ravel() - rho).mean()), float(R[0].min())

    e0, m0 = err(0.0)
    e1, m1 = err(0.5)
    assert e1 < 1.1 * e0 and m1 > 0.1, (e0, e1, m1)
