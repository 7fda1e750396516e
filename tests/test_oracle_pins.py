"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test ties the oracle to something other than itself: the exact Riemann
solution and its textbook star values, conservation laws, closed forms,
symmetries, and special cases that reduce bitwise to simpler runs.  A
plausible slip anywhere in the oracle (a dropped flux term, a wrong sign or
index, a transposed operand, a wrong ghost layer) breaks one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as ER
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _totals(forest, U):
    s = forest.scheme
    vol = np.ones(forest.n)
    for d in range(s.ndim):
        ncell = s.base_blocks[d] * (2.0 ** (forest.level - 1)) * s.block_nx[d]
        vol = vol * ((s.xmax[d] - s.xmin[d]) / ncell)
    w = vol.reshape([forest.n] + [1] * s.ndim)
    return np.array([(U[v] * w).sum() for v in range(U.shape[0])])


# ---------------------------------------------------------------------------
# whole scheme on the Sod tube (C1)
# ---------------------------------------------------------------------------


def test_exact_solver_matches_textbook_star_state():
    g = _golden("sod_star_toro.txt")
    p, u = ER.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert abs(p - g["p_star"]) < 6e-6
    assert abs(u - g["u_star"]) < 6e-6
    # densities just left and right of the contact
    rl = ER.sample(u - 1e-9, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)[0]
    rr = ER.sample(u + 1e-9, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)[0]
    assert abs(rl - g["rho_starL"]) < 6e-6
    assert abs(rr - g["rho_starR"]) < 6e-6


def test_sod_l1_error_and_convergence():
    errs = []
    for n in (256, 512, 1024):
        f, U = W.sod(n)
        R, _ = oracle.run(f, U, t_end=0.2)
        x = (np.arange(n) + 0.5) / n
        ex = ER.sod_profile(x, 0.2)
        errs.append(np.abs(R[0, 0] - ex[0]).mean())
    # first run gave 1.48e-3 at 1024 cells; a wrong flux or limiter is far off
    assert errs[2] < 2.0e-3
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 0.6, orders
    # the plateau values of the exact solution are reproduced away from waves
    f, U = W.sod(1024)
    R, _ = oracle.run(f, U, t_end=0.2)
    x = (np.arange(1024) + 0.5) / 1024
    ex = ER.sod_profile(x, 0.2)
    pos = ER.wave_positions(0.2)
    plateau = (x > pos["tail"] + 0.03) & (x < pos["contact"] - 0.03)
    assert np.abs(R[0, 0][plateau] - ex[0][plateau]).max() < 2e-3


def test_sod_conservation_and_boundary_momentum():
    f, U = W.sod(1024)
    R, dts = oracle.run(f, U, t_end=0.2)
    t = sum(dts)
    assert abs(t - 0.2) < 1e-15
    T0 = _totals(f, U)
    T1 = _totals(f, R)
    # no mass or energy flux through zero-gradient ends of a resting gas
    assert abs(T1[0] - T0[0]) <= 1e-14 * abs(T0[0])
    assert abs(T1[2] - T0[2]) <= 1e-14 * abs(T0[2])
    # momentum grows by (p_left - p_right) t = 0.9 t
    assert abs(T1[1] - 0.9 * t) < 1e-13


def test_cfl_closed_form_bitwise():
    f, U = W.sod(1024)
    o = oracle.OracleForest(f)
    o.set_state(U)
    assert o.max_dt() == 0.8 / (1024 * math.sqrt(1.4))


# ---------------------------------------------------------------------------
# special cases that reduce bitwise to simpler runs
# ---------------------------------------------------------------------------


def _sod_nd(ndim, axis, n=128, scheme_kw=None):
    """Sod tube along `axis` of an ndim forest of 16-cell blocks."""
    kw = dict(ndim=ndim, block_nx=(16,) * ndim, base_blocks=tuple(n // 16 if d == axis else 1 for d in range(ndim)),
              max_level=1, physics=W.EULER, gamma=1.4, flux=W.TVDLF, limiter=W.MINMOD, rk_stages=2, cfl=0.8,
              bc=W.ZERO_GRADIENT)
    kw.update(scheme_kw or {})
    s = W.Scheme(**kw)
    f = W.uniform_forest(s)
    xs = W.cell_centres(f)
    left = xs[axis] < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    vel = [np.zeros_like(rho) for _ in range(ndim)]
    return f, W.state_from_primitive(f, rho, vel, p)


def _line(forest, U, axis):
    """Gather the 1D profile along `axis` (all other coordinates 0)."""
    s = forest.scheme
    nd = s.ndim
    n = s.base_blocks[axis] * s.block_nx[axis]
    out = np.empty((U.shape[0], n))
    for b in range(forest.n):
        start = forest.ijk[b, axis] * s.block_nx[axis]
        sl = [slice(None), b] + [0] * nd
        sl[2 + (nd - 1 - axis)] = slice(None)
        out[:, start:start + s.block_nx[axis]] = U[tuple(sl)]
    return out


@pytest.mark.parametrize("flux,lim,rk", [(W.TVDLF, W.MINMOD, 2), (W.HLLC, W.VANLEER, 3), (W.HLL, W.VANLEER, 3)])
def test_directional_embedding_bitwise(flux, lim, rk):
    kw = dict(flux=flux, limiter=lim, rk_stages=rk)
    f1, U1 = _sod_nd(1, 0, scheme_kw=kw)
    R1, dts = oracle.run(f1, U1, steps=12)
    # single 128-cell block gives the same bits as eight 16-cell blocks
    s = W.sod_scheme(128)
    s.flux, s.limiter, s.rk_stages = flux, lim, rk
    fs = W.uniform_forest(s)
    Rs, _ = oracle.run(fs, W.state_from_primitive(fs, np.where(W.cell_centres(fs)[0] < 0.5, 1.0, 0.125),
                                                  [np.zeros((1, 128))],
                                                  np.where(W.cell_centres(fs)[0] < 0.5, 1.0, 0.1)), dts=dts)
    assert np.array_equal(Rs[:, 0], _line(f1, R1, 0))
    ref = _line(f1, R1, 0)
    for nd, axis in [(2, 0), (2, 1), (3, 2)]:
        f, U = _sod_nd(nd, axis, scheme_kw=kw)
        R, _ = oracle.run(f, U, dts=dts)
        prof = _line(f, R, axis)
        # density, normal momentum, energy equal the 1D run bit for bit
        assert np.array_equal(prof[0], ref[0])
        assert np.array_equal(prof[1 + axis], ref[1])
        assert np.array_equal(prof[1 + nd], ref[2])
        for d in range(nd):
            if d != axis:
                assert np.all(R[1 + d] == 0.0)
        # and the state is uniform across the tube
        for b in range(f.n):
            blk = R[:, b]
            for ax in range(nd):
                if ax == axis:
                    continue
                a = nd - ax
                assert np.array_equal(blk, np.broadcast_to(np.take(blk, [0], axis=a), blk.shape))


def _amr2d(bc=W.PERIODIC, flux=W.HLLC, physics=W.EULER):
    s = W.Scheme(ndim=2, block_nx=(8, 8), base_blocks=(4, 4), max_level=3, physics=physics,
                 gamma=1.4 if physics == W.EULER else 5.0 / 3.0, flux=flux, limiter=W.VANLEER, rk_stages=3,
                 cfl=0.8, bc=bc)

    def refine(l, c):
        # refine around the domain centre
        nb = 4 << (l - 1)
        return abs((c[0] + 0.5) / nb - 0.5) < 0.2 and abs((c[1] + 0.5) / nb - 0.45) < 0.2

    return W.refined_forest(s, refine)


def _amr3d(flux=W.HLLC):
    s = W.Scheme(ndim=3, block_nx=(8, 8, 8), base_blocks=(2, 2, 2), max_level=3, xmin=(-0.5,) * 3,
                 xmax=(0.5,) * 3, flux=flux, limiter=W.VANLEER, rk_stages=3, cfl=0.8, bc=W.PERIODIC)
    return W.blast_forest(s, radius=0.2, buffer_cells=1.0)


def test_amr_forests_have_all_face_kinds():
    for f in (_amr2d(), _amr3d()):
        counts = f.level_counts()
        assert len(counts) >= 2
        o = oracle.OracleForest(f)
        kinds = np.concatenate([o.face_kinds(b) for b in range(f.n)])
        assert {0, 1, 2} <= set(kinds.tolist())


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_free_stream_bitwise_across_coarse_fine(which):
    f = _amr2d() if which == "2d" else _amr3d()
    nd = f.scheme.ndim
    shape = f.state_shape()[1:]
    rho = np.full(shape, 1.3)
    vel = [np.full(shape, 0.37 * (d + 1) * (-1) ** d) for d in range(nd)]
    U = W.state_from_primitive(f, rho, vel, np.full(shape, 0.9))
    R, _ = oracle.run(f, U, steps=4)
    for v in range(U.shape[0]):
        assert np.all(R[v] == R[v].flat[0]), v
        # the SSP combinations (e.g. u/3 + 2u/3) may round the common value
        assert abs(R[v].flat[0] - U[v].flat[0]) <= 8 * np.spacing(abs(U[v].flat[0]))


def test_uniform_forest_levels_bitwise():
    s1 = W.kh_scheme(4)
    s1.block_nx = (8, 8, 1)
    f1, U1 = W.kh(scheme=W.Scheme(**{**s1.as_dict(), "base_blocks": (8, 8, 1)}))
    s2 = W.Scheme(**{**s1.as_dict(), "base_blocks": (4, 4, 1), "max_level": 2})
    f2, U2 = W.kh(scheme=s2, level=2)
    # same cells in a different leaf order: map leaf by global position
    key1 = {tuple(f1.ijk[b, :2]): b for b in range(f1.n)}
    perm = [key1[tuple(f2.ijk[b, :2])] for b in range(f2.n)]
    assert np.array_equal(U2, U1[:, perm])
    R1, dts = oracle.run(f1, U1, steps=6)
    R2, _ = oracle.run(f2, U2, dts=dts)
    assert np.array_equal(R2, R1[:, perm])


def test_block_order_does_not_matter():
    f, U = W.kh(4)
    R, dts = oracle.run(f, U, steps=4)
    rng = np.random.default_rng(3)
    perm = rng.permutation(f.n)
    fp = W.Forest(f.scheme, f.level[perm].copy(), f.ijk[perm].copy())
    Rp, _ = oracle.run(fp, U[:, perm], dts=dts)
    assert np.array_equal(Rp, R[:, perm])


def test_thread_count_does_not_matter():
    f = _amr3d()
    shape = f.state_shape()[1:]
    _, U = W.blast(f.scheme, radius=0.2, forest=f)
    old = oracle.get_threads()
    try:
        oracle.set_threads(1)
        R1, dts = oracle.run(f, U, steps=2)
        oracle.set_threads(max(2, old))
        R2, _ = oracle.run(f, U, dts=dts)
    finally:
        oracle.set_threads(old)
    assert np.array_equal(R1, R2)


# ---------------------------------------------------------------------------
# ghost fill: restriction and prolongation
# ---------------------------------------------------------------------------


def _linear_state(f, coef):
    xs = W.cell_centres(f)
    shape = xs[0].shape
    lin = np.full(shape, 5.0)
    for d, c in enumerate(coef):
        lin = lin + c * xs[d]
    U = np.stack([lin + v for v in range(f.scheme.nvar)])
    return U


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_ghosts_of_linear_data_are_exact(which):
    """Copy, restriction and minmod prolongation all reproduce linear data:
    every face ghost equals the linear function at its own cell centre."""
    f = _amr2d() if which == "2d" else _amr3d()
    s = f.scheme
    nd = s.ndim
    coef = [0.25, -0.5, 0.125][:nd]
    # dyadic coefficients and cell centres keep every value exact
    U = _linear_state(f, coef)
    o = oracle.OracleForest(f)
    o.set_state(U)
    checked = 0
    for b in range(f.n):
        P = o.padded_block(b)
        kinds = o.face_kinds(b)
        ncell = [s.base_blocks[d] << (f.level[b] - 1) for d in range(nd)]
        dx = [(s.xmax[d] - s.xmin[d]) / (ncell[d] * s.block_nx[d]) for d in range(nd)]
        for fc in range(2 * nd):
            d, side = fc // 2, (1 if fc & 1 else -1)
            for layer in range(2):
                idx = [slice(2, 2 + s.block_nx[e]) if e < nd else slice(0, 1) for e in range(3)]
                gi = -1 - layer if side < 0 else s.block_nx[d] + layer
                idx[d] = gi + 2
                ghost = P[0][tuple(reversed(idx))]
                # expected linear values at the ghost centres (no wrap across the
                # periodic edge: skip ghosts outside the domain)
                cent = []
                for e in range(nd):
                    if e == d:
                        g = f.ijk[b, e] * s.block_nx[e] + gi
                        c = s.xmin[e] + (g + 0.5) * dx[e]
                    else:
                        g = f.ijk[b, e] * s.block_nx[e] + np.arange(s.block_nx[e])
                        c = s.xmin[e] + (g + 0.5) * dx[e]
                    cent.append(c)
                if not (s.xmin[d] < cent[d] < s.xmax[d]):
                    continue
                grids = np.meshgrid(*[np.atleast_1d(c) for c in cent], indexing="ij")
                exp = np.full(grids[0].shape, 5.0)
                for e in range(nd):
                    exp = exp + coef[e] * grids[e]
                # linear data jumps across the periodic edge: keep ghosts whose
                # source stencil (a coarse cell and its neighbours) stays inside
                inside = np.ones(grids[0].shape, dtype=bool)
                for e in range(nd):
                    margin = 3.0 * 2.0 * dx[e]
                    inside &= (grids[e] > s.xmin[e] + margin) & (grids[e] < s.xmax[e] - margin)
                exp = np.squeeze(np.transpose(exp, list(reversed(range(nd)))))
                inside = np.squeeze(np.transpose(inside, list(reversed(range(nd)))))
                got = np.squeeze(ghost)
                assert np.array_equal(got[inside], exp[inside]), (b, fc, layer, kinds[fc])
                checked += int(inside.sum())
    assert checked > 0


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_restrict_of_prolong_is_identity(which):
    """The 2^d fine ghosts prolonged from one coarse cell average back to it."""
    f = _amr2d() if which == "2d" else _amr3d()
    s = f.scheme
    nd = s.ndim
    xs = W.cell_centres(f)
    smooth = 1.0 + 0.3 * np.sin(2 * np.pi * xs[0]) * np.cos(2 * np.pi * xs[1] + 0.3)
    if nd == 3:
        smooth = smooth + 0.1 * np.sin(4 * np.pi * xs[2])
    U = np.stack([smooth * (v + 1) for v in range(s.nvar)])
    o = oracle.OracleForest(f)
    o.set_state(U)
    worst = 0.0
    hits = 0
    for b in range(f.n):
        kinds = o.face_kinds(b)
        if 1 not in kinds:
            continue
        P = o.padded_block(b)
        for fc in range(2 * nd):
            if kinds[fc] != 1:
                continue
            d, side = fc // 2, (1 if fc & 1 else -1)
            # fine ghost layers (-2,-1) or (n, n+1) form one coarse layer
            sl = [slice(2, 2 + s.block_nx[e]) if e < nd else slice(0, 1) for e in range(3)]
            sl[d] = slice(0, 2) if side < 0 else slice(2 + s.block_nx[d], 4 + s.block_nx[d])
            slab = P[:, sl[2], sl[1], sl[0]]
            # average 2x2(x2) fine cells
            axes = [3 - e for e in range(nd)]
            avg = slab
            for a in axes:
                shp = list(avg.shape)
                shp[a] //= 2
                shp.insert(a + 1, 2)
                avg = avg.reshape(shp).mean(axis=a + 1)
            # the coarse neighbour's cells
            k = np.nonzero([kinds[fc] == 1])[0]
            # locate coarse leaf and cells by position
            lvl = f.level[b] - 1
            cb = [f.ijk[b, e] * s.block_nx[e] for e in range(nd)]
            gidx = []
            for e in range(nd):
                if e == d:
                    g = (cb[e] - 1) // 2 if side < 0 else (cb[e] + s.block_nx[e]) // 2
                    gidx.append(np.array([g]))
                else:
                    gidx.append(np.arange(cb[e] // 2, (cb[e] + s.block_nx[e]) // 2))
            ncl = [(s.base_blocks[e] << (lvl - 1)) * s.block_nx[e] for e in range(nd)]
            gidx = [g % n for g, n in zip(gidx, ncl)]
            blk = [g // s.block_nx[e] for e, g in enumerate(gidx)]
            owner = [c for c in range(f.n) if f.level[c] == lvl and all(
                f.ijk[c, e] == blk[e][0] for e in range(nd))]
            assert len(owner) == 1
            c = owner[0]
            loc = [g % s.block_nx[e] for e, g in enumerate(gidx)]
            sub = U[:, c]
            for e in reversed(range(nd)):
                sub = np.take(sub, loc[e], axis=1 + (nd - 1 - e))
            rel = np.abs(avg.reshape(sub.shape) - sub) / np.abs(sub)
            worst = max(worst, float(rel.max()))
            hits += 1
    assert hits > 0
    assert worst <= 4 * np.finfo(float).eps, worst


# ---------------------------------------------------------------------------
# conservation, positivity, contact preservation, symmetry
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("case", ["kh", "ot", "blast_amr", "kh_amr"])
def test_conservation_to_rounding(case):
    if case == "kh":
        f, U = W.kh(4)
        steps = 20
    elif case == "ot":
        f, U = W.orszag_tang(4)
        steps = 20
    elif case == "blast_amr":
        f = _amr3d()
        _, U = W.blast(f.scheme, radius=0.2, forest=f)
        steps = 3
    else:
        f = _amr2d()
        xs = W.cell_centres(f)
        rho = 1.0 + 0.5 * (np.abs(xs[1] - 0.5) < 0.25)
        u = np.where(np.abs(xs[1] - 0.5) < 0.25, 0.5, -0.5)
        v = 0.05 * np.sin(4 * np.pi * xs[0])
        U = W.state_from_primitive(f, rho, [u, v], np.full_like(rho, 2.5))
        steps = 10
    T0 = _totals(f, U)
    R, _ = oracle.run(f, U, steps=steps)
    T1 = _totals(f, R)
    nd = f.scheme.ndim
    scale = np.abs(T0).max()
    ncons = f.scheme.nvar - (1 if f.scheme.physics == W.MHD else 0)  # psi is damped
    for v in range(ncons):
        assert abs(T1[v] - T0[v]) <= 5e-14 * max(scale, 1.0), (v, T0[v], T1[v])
    assert np.all(R[0] > 0)


def test_blast_positivity_every_step():
    f = _amr3d()
    _, U = W.blast(f.scheme, radius=0.2, forest=f)
    o = oracle.OracleForest(f)
    o.set_state(U)
    for _ in range(4):
        dt = o.max_dt()  # raises on rho <= 0, p <= 0 or NaN
        o.advance(dt)
    assert o.max_dt() > 0


def test_hllc_keeps_shear_layer_stationary_hll_does_not():
    f, U = W.kh(4, amplitude=0.0)
    R, dts = oracle.run(f, U, steps=20)
    assert np.abs(R - U).max() <= 1e-12 * np.abs(U).max()
    s = W.kh_scheme(4)
    s.flux = W.HLL
    fh = W.Forest(s, f.level, f.ijk)
    Rh, _ = oracle.run(fh, U, dts=dts)
    assert np.abs(Rh - U).max() > 1e-3


def test_orszag_tang_point_symmetry():
    f, U = W.orszag_tang(4)
    R, _ = oracle.run(f, U, steps=30)
    s = f.scheme
    n = 4 * 16

    def glob(A):
        G = np.empty((A.shape[0], n, n))
        for b in range(f.n):
            i0, j0 = f.ijk[b, 0] * 16, f.ijk[b, 1] * 16
            G[:, j0:j0 + 16, i0:i0 + 16] = A[:, b]
        return G

    G = glob(R)
    Gr = G[:, ::-1, ::-1]
    sign = np.array([1, -1, -1, 1, -1, -1, 1.0])[:, None, None]
    scale = np.abs(G).max(axis=(1, 2), keepdims=True)
    asym = np.abs(G - sign * Gr) / scale
    assert asym[:6].max() < 1e-11, asym.max(axis=(1, 2))
    assert np.abs(G[6]).max() > 0  # psi has been generated


def test_blast_mirror_symmetry():
    f = _amr3d()
    _, U = W.blast(f.scheme, radius=0.2, forest=f)
    R, _ = oracle.run(f, U, steps=2)
    s = f.scheme
    # leaf of the mirror image x -> -x
    pos = {(int(f.level[b]), *map(int, f.ijk[b])): b for b in range(f.n)}
    worst = 0.0
    for b in range(f.n):
        l = int(f.level[b])
        nb = s.base_blocks[0] << (l - 1)
        m = pos[(l, nb - 1 - int(f.ijk[b, 0]), int(f.ijk[b, 1]), int(f.ijk[b, 2]))]
        A = R[:, b]
        B = R[:, m][:, :, :, ::-1].copy()
        B[1] = -B[1]
        worst = max(worst, float(np.abs(A - B).max() / np.abs(R).max()))
    assert worst < 1e-12


# ---------------------------------------------------------------------------
# Loehner estimator closed forms
# ---------------------------------------------------------------------------


def _loh_1d(rho, p, bc=W.ZERO_GRADIENT):
    n = len(rho)
    s = W.Scheme(ndim=1, block_nx=(n,), base_blocks=(1,), max_level=2, physics=W.EULER, gamma=1.4,
                 flux=W.HLLC, limiter=W.VANLEER, rk_stages=3, bc=bc)
    f = W.uniform_forest(s)
    U = W.state_from_primitive(f, np.asarray(rho, float)[None], [np.zeros((1, n))], np.asarray(p, float)[None])
    o = oracle.OracleForest(f)
    o.set_state(U)
    return o, o.lohner_cells(0)


def test_lohner_linear_data_is_zero():
    rho = 10.0 + np.arange(16)
    _, E = _loh_1d(rho, np.full(16, 3.0), bc=W.PERIODIC)
    # periodic wrap creates a jump at the ends; interior cells see linear data
    assert np.all(E[2:-2] == 0.0)


@pytest.mark.parametrize("a,b", [(1.0, 3.0), (2.0, 0.5), (7.0, 7.5)])
def test_lohner_step_closed_form(a, b):
    rho = np.where(np.arange(16) < 8, a, b)
    _, E = _loh_1d(rho, np.full(16, 1.0))
    eps = 0.01
    ea = abs(b - a) / (abs(b - a) + eps * (abs(b) + 3 * abs(a)))
    eb = abs(a - b) / (abs(a - b) + eps * (abs(a) + 3 * abs(b)))
    assert E[7] == pytest.approx(0.5 * ea, rel=1e-14)
    assert E[8] == pytest.approx(0.5 * eb, rel=1e-14)
    assert np.all(E[:6] == 0.0) and np.all(E[10:] == 0.0)


def test_lohner_quadratic_closed_form():
    c = 2.0
    k = np.arange(16) - 8.0
    p = c + k * k
    _, E = _loh_1d(np.ones(16), p)
    eps = 0.01
    for i in range(2, 14):
        kk = k[i]
        exp = 2.0 / (abs(2 * kk + 1) + abs(2 * kk - 1) + eps * (4 * c + 4 * kk * kk + 2))
        assert E[i] == pytest.approx(0.5 * exp, rel=1e-12)


def test_lohner_flag_rule():
    # refine above tol, coarsen strictly below frac*tol, level limits respected
    n = 16
    s = W.Scheme(ndim=1, block_nx=(n,), base_blocks=(2,), max_level=3, physics=W.EULER, gamma=1.4,
                 flux=W.HLLC, limiter=W.VANLEER, rk_stages=3, bc=W.ZERO_GRADIENT)
    lev = np.array([1, 2, 2], dtype=np.int32)
    ijk = np.array([[0, 0, 0], [2, 0, 0], [3, 0, 0]], dtype=np.int32)
    f = W.Forest(s, lev, ijk)
    xs = W.cell_centres(f)[0]
    rho = np.where(xs < 0.25, 1.0, 1.0)
    rho = np.where((xs > 0.85) & (xs < 0.95), 2.0, rho)
    U = W.state_from_primitive(f, rho, [np.zeros_like(rho)], np.ones_like(rho))
    o = oracle.OracleForest(f)
    o.set_state(U)
    flags, emax = o.flag_blocks(with_emax=True)
    assert emax[0] == 0.0 and flags[0] == 0  # level 1 cannot coarsen
    assert flags[2] == 1 and emax[2] > 0.1
    assert emax[1] == 0.0 and flags[1] == -1


# ---------------------------------------------------------------------------
# ABI contract on the oracle (error codes, checkpoint / restore)
# ---------------------------------------------------------------------------


def test_rejects_unbalanced_and_non_covering_forests():
    s = W.Scheme(ndim=2, block_nx=(8, 8), base_blocks=(2, 2), max_level=3)
    # a level-3 leaf next to a level-1 leaf
    lev, ijk = [1, 1, 1], [[1, 0, 0], [0, 1, 0], [1, 1, 0]]
    for q in range(4):
        if q == 0:
            lev += [3] * 4
            ijk += [[0 + (a & 1), 0 + (a >> 1), 0] for a in range(4)]
        else:
            lev.append(2)
            ijk.append([q & 1, q >> 1, 0])
    f = W.Forest(s, np.array(lev, np.int32), np.array(ijk, np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleForest(f)
    assert e.value.code == -2
    # a gap
    f = W.Forest(s, np.array([1, 1, 1], np.int32), np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleForest(f)
    assert e.value.code == -2
    # an overlap
    f = W.Forest(s, np.array([1, 1, 1, 1, 2], np.int32),
                 np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0, 0, 0]], np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleForest(f)
    assert e.value.code == -2


def test_rejects_nonphysical_state_and_bad_dt():
    f, U = W.kh(2)
    o = oracle.OracleForest(f)
    for bad in ("rho", "nan", "p"):
        V = U.copy()
        if bad == "rho":
            V[0, 1, 3, 4] = -1.0
        elif bad == "nan":
            V[2, 0, 0, 0] = np.nan
        else:
            V[3, 2, 5, 5] = 0.0  # E = 0 with momentum: p < 0
        o.set_state(V)
        with pytest.raises(oracle.OracleError) as e:
            o.max_dt()
        assert e.value.code == -3
    o.set_state(U)
    for dt in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(oracle.OracleError) as e:
            o.advance(dt)
        assert e.value.code == -1
    with pytest.raises(ValueError):
        o.set_state(U[:, :2])


def test_checkpoint_restore_bitwise():
    f, U = W.kh(2)
    R, dts = oracle.run(f, U, steps=8)
    o = oracle.OracleForest(f)
    o.set_state(U)
    for dt in dts[:3]:
        o.advance(dt)
    ck = o.get_state()
    o.close()
    o2 = oracle.OracleForest(f)
    o2.set_state(ck)
    for dt in dts[3:]:
        o2.advance(dt)
    assert np.array_equal(o2.get_state(), R)
