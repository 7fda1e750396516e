"""Pins of the oracle's polytropic closure without energy equation (Sec. 2.2:
p = c_ad rho^gamma, c^2 = gamma c_ad rho^(gamma-1); with rho = h, c_ad = 1/2,
gamma = 2 the shallow water equations of the paper's dam break).

The exact two-wave Riemann solution (test infrastructure, written from the
jump conditions and Riemann invariants) pins fluxes and wave speeds through
the whole scheme, for the shallow-water exponent (exact squares) and for
gamma = 1.4 (the pow path).  A small simple wave travels at the closed-form
sound speed.  A lake at rest stays bitwise at rest across coarse-fine faces;
mass and momentum are conserved; the 2D dam break keeps the symmetries of
its setup; a 2D run aligned with x equals the 1D run bit for bit; bad
configurations and states are rejected with the documented codes."""
import numpy as np
import pytest

import oracle
from oracle import exact_riemann as E
import workloads as W


def _scheme_1d(n, nb=8, g=2.0, cad=0.5, flux=W.HLL, lim=W.KOREN, bc=W.ZERO_GRADIENT, x=(-10.0, 10.0)):
    return W.Scheme(ndim=1, block_nx=(n // nb,), base_blocks=(nb,), max_level=1, xmin=(x[0],), xmax=(x[1],),
                    physics=W.POLY, gamma=g, cad=cad, flux=flux, limiter=lim, rk_stages=3, cfl=0.9, bc=bc)


def _riemann_1d(n, left, right, g=2.0, cad=0.5, flux=W.HLL, lim=W.KOREN, t=2.0):
    """L1 errors of rho and momentum against the exact solution at t."""
    f = W.uniform_forest(_scheme_1d(n, g=g, cad=cad, flux=flux, lim=lim))
    (x,) = W.cell_centres(f)
    rho = np.where(x < 0.0, left[0], right[0])
    u = np.where(x < 0.0, left[1], right[1])
    R, _ = oracle.run(f, W.state_from_primitive(f, rho, [u]), t_end=t)
    re, ue = E.poly_profile(x.ravel(), t, 0.0, left, right, g, cad)
    return np.abs(R[0].ravel() - re).mean(), np.abs(R[1].ravel() - re * ue).mean()


def test_exact_solver_satisfies_its_jump_conditions():
    g, cad = 2.0, 0.5
    rs, us = E.poly_star(2.5, 0.0, 0.5, 0.0, g, cad)
    # right shock: mass and momentum conserved across it
    m = np.sqrt((cad * rs ** 2 - cad * 0.25) * rs * 0.5 / (rs - 0.5))
    s = m / 0.5
    assert 0.5 * (0.0 - s) == pytest.approx(rs * (us - s), rel=1e-12)
    assert cad * 0.25 == pytest.approx(rs * us * (us - s) + cad * rs ** 2, rel=1e-12)
    # left rarefaction: u + 2c/(gamma-1) carried from the left state
    assert us + 2.0 * np.sqrt(rs) == pytest.approx(2.0 * np.sqrt(2.5), rel=1e-14)


@pytest.mark.parametrize("flux,lim", [(W.HLL, W.KOREN), (W.TVDLF, W.MINMOD), (W.HLL, W.CADA)])
def test_dam_break_converges_to_the_exact_solution(flux, lim):
    """The paper's dam-break heights 2.5 | 0.5 as a 1D Riemann problem:
    left rarefaction, right shock; first order in L1 (a shock)."""
    e = [_riemann_1d(n, (2.5, 0.0), (0.5, 0.0), flux=flux, lim=lim) for n in (256, 1024)]
    assert e[1][0] < 0.0025 and e[1][1] < 0.003, e
    assert e[0][0] / e[1][0] > 2.8 and e[0][1] / e[1][1] > 2.8, e


def test_polytrope_with_pow_exponent_converges():
    """gamma = 1.4, c_ad = 1: the exponents gamma and gamma - 1 go through pow."""
    e = [_riemann_1d(n, (1.0, 0.2), (0.2, -0.1), g=1.4, cad=1.0, t=1.5) for n in (256, 1024)]
    assert e[1][0] < 1e-3 and e[1][1] < 1e-3, e
    assert e[0][0] / e[1][0] > 2.5, e


@pytest.mark.parametrize("g,cad", [(2.0, 0.5), (1.4, 1.0), (5.0 / 3.0, 0.3)])
def test_simple_wave_travels_at_the_sound_speed(g, cad):
    """A right-going acoustic wave rho = rho0 (1 + eps sin), u = c0 eps sin
    on a periodic domain: after t it is the profile shifted by c0 t (to
    O(eps^2)); the error converges at second order only with the right c0."""
    rho0, eps, t = 1.3, 1e-6, 0.5
    c0 = np.sqrt(g * cad * rho0 ** (g - 1.0))

    def err(n):
        f = W.uniform_forest(_scheme_1d(n, g=g, cad=cad, lim=W.VANLEER, bc=W.PERIODIC, x=(0.0, 1.0)))
        (x,) = W.cell_centres(f)
        h = 1.0 / n
        sav = lambda y: (np.cos(2 * np.pi * (y - h / 2)) - np.cos(2 * np.pi * (y + h / 2))) / (2 * np.pi * h)
        rho = rho0 * (1.0 + eps * sav(x))
        U = np.stack([rho, rho0 * c0 * eps * sav(x)])
        R, _ = oracle.run(f, U, t_end=t)
        exact = rho0 * (1.0 + eps * sav(x - c0 * t))
        return np.abs(R[0] - exact).mean() / (rho0 * eps)

    e = [err(n) for n in (64, 128, 256)]
    assert e[2] < 2e-3, e
    assert np.log2(e[1] / e[2]) > 1.6, e


def _dam_forest_uniform(h=1.3):
    """The dam-break forest (three levels around the wall) with a lake at rest."""
    f, _ = W.dam_break(base=4, max_level=3, buffer_cells=2.0)
    shape = W.cell_centres(f)[0].shape
    return f, W.state_from_primitive(f, np.full(shape, h), [np.zeros(shape)] * 2)


def test_lake_at_rest_stays_at_rest_bitwise():
    f, U = _dam_forest_uniform()
    assert len(set(f.level.tolist())) == 3
    R, _ = oracle.run(f, U, steps=8)
    assert np.array_equal(R, U)


def test_mass_and_momentum_conserved_on_amr():
    s = W.dam_break_scheme(base=2, max_level=3)
    s.bc = W.PERIODIC
    f = W.blast_forest(s, 2.5, (0.0, 0.0, 0.0), 2.0)
    x, y = W.cell_centres(f)
    h = 1.0 + 0.3 * np.exp(-((x - 1.0) ** 2 + y ** 2) / 8.0)
    u = 0.1 * np.sin(2 * np.pi * y / 40.0)
    v = 0.05 * np.cos(2 * np.pi * x / 40.0)
    U = W.state_from_primitive(f, h, [u, v])
    R, _ = oracle.run(f, U, steps=15)
    vol = np.array([(40.0 / (2 * 16 << (l - 1))) ** 2 for l in f.level])[:, None, None]
    for k in range(3):
        before, after = (U[k] * vol).sum(), (R[k] * vol).sum()
        scale = (np.abs(U[k]) * vol).sum()
        assert abs(after - before) <= 1e-13 * scale, (k, before, after)
    assert np.abs(R - U).max() > 1e-3


def _global_2d(f, U):
    s = f.scheme
    nb = s.block_nx[0]
    G = np.empty((U.shape[0], s.base_blocks[1] * nb, s.base_blocks[0] * nb))
    for b in range(f.n):
        i, j = int(f.ijk[b][0]), int(f.ijk[b][1])
        G[:, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = U[:, b]
    return G


def test_dam_break_keeps_its_symmetries():
    s = W.dam_break_scheme(base=4, max_level=1)
    f, U = W.dam_break(scheme=s, forest=W.uniform_forest(s), r_dam=8.0)
    R, _ = oracle.run(f, U, steps=30)
    G = _global_2d(f, R)
    P = G[:, ::-1, ::-1]
    T = np.transpose(G, (0, 2, 1))
    sc = np.abs(G).reshape(3, -1).max(axis=1)
    assert np.abs(G[0] - P[0]).max() <= 1e-12 * sc[0]
    assert np.abs(G[1] + P[1]).max() <= 1e-12 * sc[1]
    assert np.abs(G[0] - T[0]).max() <= 1e-12 * sc[0]
    assert np.abs(G[1] - T[2]).max() <= 1e-12 * sc[1]
    assert sc[1] > 0.1


def test_x_aligned_2d_equals_1d_bitwise():
    s1 = _scheme_1d(64, nb=4, x=(-10.0, 10.0))
    f1 = W.uniform_forest(s1)
    (x1,) = W.cell_centres(f1)
    h1 = np.where(x1 < 1.0, 2.5, 0.5)
    R1, d1 = oracle.run(f1, W.state_from_primitive(f1, h1, [np.zeros_like(h1)]), steps=20)
    s2 = W.Scheme(ndim=2, block_nx=(16, 16), base_blocks=(4, 2), max_level=1, xmin=(-10.0, 0.0), xmax=(10.0, 10.0),
                  physics=W.POLY, gamma=2.0, cad=0.5, flux=W.HLL, limiter=W.KOREN, rk_stages=3, cfl=0.9,
                  bc=W.ZERO_GRADIENT)
    f2 = W.uniform_forest(s2)
    x2, _ = W.cell_centres(f2)
    h2 = np.where(x2 < 1.0, 2.5, 0.5)
    R2, d2 = oracle.run(f2, W.state_from_primitive(f2, h2, [np.zeros_like(h2)] * 2), dts=d1)
    for b in range(f2.n):
        i = int(f2.ijk[b][0])
        for row in range(16):
            assert np.array_equal(R2[0, b, row], R1[0, i])
            assert np.array_equal(R2[1, b, row], R1[1, i])
            assert not np.any(R2[2, b, row])


def test_rejects_bad_configuration_and_state():
    s = W.dam_break_scheme(base=2, max_level=1)
    for change in ({"flux": W.HLLC}, {"cad": 0.0}, {"gamma": 0.9}):
        t = W.dam_break_scheme(base=2, max_level=1)
        for k, v in change.items():
            setattr(t, k, v)
        with pytest.raises(oracle.OracleError) as e:
            oracle.OracleForest(W.uniform_forest(t))
        assert e.value.code == -1, change
    f, U = W.dam_break(scheme=s, forest=W.uniform_forest(s))
    o = oracle.OracleForest(f)
    for bad in ("h", "nan"):
        V = U.copy()
        if bad == "h":
            V[0, 1, 3, 4] = 0.0
        else:
            V[2, 0, 5, 5] = np.nan
        o.set_state(V)
        with pytest.raises(oracle.OracleError) as e:
            o.max_dt()
        assert e.value.code == -3, bad
    o.set_state(U)
    dt = o.max_dt()
    # Courant step of the state at rest: cfl / max (c / dx), c = sqrt(h)
    assert dt == pytest.approx(0.9 / (np.sqrt(2.5) / (40.0 / 32) * 2), rel=1e-15)


def test_lohner_flags_the_dam_wall():
    f, U = W.dam_break(base=4, max_level=3, buffer_cells=2.0)
    o = oracle.OracleForest(f)
    o.set_state(U)
    flags = o.flag_blocks()
    xs = W.cell_centres(f)
    r = np.sqrt(xs[0] ** 2 + xs[1] ** 2)
    wall = (r.reshape(f.n, -1).min(axis=1) < 2.5) & (r.reshape(f.n, -1).max(axis=1) > 2.5)
    assert np.all(flags[wall & (f.level < 3)] == 1)
    assert np.all(flags[~wall] <= 0)
    assert np.any(flags == -1)
