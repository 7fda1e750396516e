"""Pins of the forest Helmholtz oracle (oracle/fmg.py) against what fixes it
from outside: the uniform-grid exact solve (oracle/rd.py, spectral), exact
reproduction of constants and linear functions by every ghost rule, mirror
and transposition symmetry, and second-order convergence to a smooth
solution across coarse-fine faces (Sec. 1.4)."""
import numpy as np
import pytest

import workloads as W
from oracle import fmg, rd


def _uniform_to_grid(forest, u):
    """Leaf layout [leaf][y][x] of a uniform forest -> [y][x] of the grid."""
    s = forest.scheme
    nb = s.block_nx[0]
    n = (s.base_blocks[0] << (int(forest.level[0]) - 1)) * nb
    out = np.zeros((n, n))
    for k in range(forest.n):
        i, j = forest.ijk[k, :2]
        out[j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = u[k]
    return out


@pytest.mark.parametrize("bc", [fmg.PERIODIC, fmg.NEUMANN])
def test_uniform_forest_is_the_uniform_grid(bc):
    """Every leaf at level 2: the composite problem is the 5-point problem on
    the 64^2 grid, which oracle/rd.py solves spectrally."""
    s = W.fmg_scheme(base=2, max_level=2, bc=bc)
    f = W.uniform_forest(s, level=2)
    x, y = fmg.cell_centres(f, 1.0)
    rhs = np.sin(2 * np.pi * x) * np.cos(4 * np.pi * y) + x * y
    lam = 37.0
    u = fmg.solve(f, rhs, lam, 1.0, bc)
    ref = rd.helmholtz_solve(_uniform_to_grid(f, rhs), lam, 1.0, bc)
    assert np.max(np.abs(_uniform_to_grid(f, u) - ref)) <= 1e-12 * np.max(np.abs(ref))


def _refined(bc, base=4, max_level=3):
    """A circle off the centre: levels 1, 2 and 3 for base >= 4."""
    return W.fmg_forest(W.fmg_scheme(base=base, max_level=max_level, bc=bc), centre=(0.27, 0.3), radius=0.15)


@pytest.mark.parametrize("bc", [fmg.PERIODIC, fmg.NEUMANN])
def test_constants_are_reproduced(bc):
    f = _refined(bc)
    assert len(np.unique(f.level)) == 3
    lam = 5.0
    u = fmg.solve(f, np.full((f.n, 16, 16), -lam * 2.5), lam, 1.0, bc)
    assert np.max(np.abs(u - 2.5)) <= 1e-12


def test_linear_functions_have_zero_laplacian_off_the_boundary():
    """Rules (1) and (3) interpolate linear data exactly, so lap(a x + b y +
    c) vanishes at every cell whose stencil stays inside the domain -- a wrong
    weight, offset sign, tangential half or restriction shows up here."""
    f = _refined(fmg.NEUMANN)
    x, y = fmg.cell_centres(f, 1.0)
    u = 0.7 * x - 1.3 * y + 0.2
    lap = fmg.apply(f, u, 0.0, 1.0, fmg.NEUMANN)
    n = (4 << (f.level.astype(np.int64) - 1)) * 16
    h = 1.0 / n[:, None, None]
    interior = (x > h) & (x < 1 - h) & (y > h) & (y < 1 - h)
    assert interior.sum() > 0.9 * u.size
    # lap is O(1/h^2) * rounding of O(1) values
    assert np.max(np.abs(lap[interior])) <= 1e-9 * np.max(1.0 / h ** 2)
    assert np.max(np.abs(lap[~interior])) > 1.0  # the Neumann faces do see the slope


def test_mirror_and_transpose_symmetry():
    """A forest symmetric under x -> 1 - x and x <-> y, with the data mirrored
    or transposed, has the mirrored or transposed solution."""
    s = W.fmg_scheme(base=8, max_level=3, bc=fmg.NEUMANN)
    f = W.fmg_forest(s, centre=(0.5, 0.5), radius=0.15)
    assert len(np.unique(f.level)) == 3
    x, y = fmg.cell_centres(f, 1.0)
    lam = 11.0

    def field(a, b):
        return np.exp(-30 * ((a - 0.3) ** 2 + (b - 0.6) ** 2)) + 0.3 * a

    u = fmg.solve(f, field(x, y), lam, 1.0, fmg.NEUMANN)
    key = {(int(l), int(i), int(j)): k for k, (l, (i, j, _)) in enumerate(zip(f.level, f.ijk))}
    um = fmg.solve(f, field(1 - x, y), lam, 1.0, fmg.NEUMANN)
    ut = fmg.solve(f, field(y, x), lam, 1.0, fmg.NEUMANN)
    for k in range(f.n):
        l, i, j = int(f.level[k]), int(f.ijk[k, 0]), int(f.ijk[k, 1])
        nbl = 8 << (l - 1)
        km = key[(l, nbl - 1 - i, j)]
        kt = key[(l, j, i)]
        assert np.allclose(um[km][:, ::-1], u[k], rtol=0, atol=1e-12)
        assert np.allclose(ut[kt].T, u[k], rtol=0, atol=1e-12)


def test_second_order_convergence_across_coarse_fine_faces():
    """A smooth Neumann-compatible solution u = cos(2 pi x) cos(4 pi y), f =
    -(20 pi^2 + lambda) u, on one three-level block forest with 8, 16, 32 and
    64 cells per block side: the maximum error falls at second order (a
    non-conservative coarse side, the mean of the children as its ghost,
    falls at first order on the same forests)."""
    lam = 3.0
    f0 = _refined(fmg.NEUMANN)
    assert len(np.unique(f0.level)) == 3
    errs = []
    for nb in (8, 16, 32, 64):
        s = W.fmg_scheme(base=4, max_level=3, bc=fmg.NEUMANN)
        s.block_nx = (nb, nb, 1)
        f = W.Forest(s, f0.level, f0.ijk)
        x, y = fmg.cell_centres(f, 1.0)
        ue = np.cos(2 * np.pi * x) * np.cos(4 * np.pi * y)
        u = fmg.solve(f, -(20 * np.pi ** 2 + lam) * ue, lam, 1.0, fmg.NEUMANN)
        errs.append(np.max(np.abs(u - ue)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders >= 1.9), (errs, orders)
    assert errs[1] < 5e-3


@pytest.mark.parametrize("bc", [fmg.PERIODIC, fmg.NEUMANN])
def test_discrete_conservation(bc):
    """Rule (4) makes the coarse flux through a coarse-fine face the mean of
    the fine fluxes: the area-weighted sum of lap(u) over all leaf cells is
    zero for any u on a periodic or Neumann domain."""
    f = _refined(bc)
    u = W.uniform01(7, f.n * 256).reshape(f.n, 16, 16)
    lap = fmg.apply(f, u, 0.0, 1.0, bc)
    area = (1.0 / ((4 << (f.level.astype(np.int64) - 1)) * 16)) ** 2
    total = np.sum(lap * area[:, None, None])
    assert abs(total) <= 1e-12 * np.sum(np.abs(lap) * area[:, None, None])


@pytest.mark.parametrize("scheme", [rd.EULER, rd.MIDPOINT, rd.SPLIT, rd.IMEX])
def test_rd_step_on_a_uniform_forest_is_the_grid_step(scheme):
    """Every leaf at level 2: one step of each scheme equals oracle/rd.py's
    step on the 64^2 grid (spectral solves, its own Laplacian)."""
    s = W.fmg_scheme(base=4, max_level=2, bc=fmg.PERIODIC, length=2.0)
    f = W.uniform_forest(s, level=2)
    x, y = fmg.cell_centres(f, 2.0)
    g = sum(0.5 * np.exp(-25.0 * ((x - cx) ** 2 + (y - cy) ** 2)) for cx, cy in ((0.5, 0.5), (0.55, 0.6)))
    u, v = 1.0 - g, g.copy()
    p = rd.GRAY_SCOTT_PARAMS
    dt = 0.5 if scheme in (rd.SPLIT, rd.IMEX) else 0.05
    u1, v1 = fmg.rd_step(f, u, v, dt, scheme, p, 2.0, fmg.PERIODIC)
    gu, gv = rd.step(_uniform_to_grid(f, u), _uniform_to_grid(f, v), dt, scheme, p, 2.0, rd.PERIODIC)
    for a, b in ((u1, gu), (v1, gv)):
        assert np.max(np.abs(_uniform_to_grid(f, a) - b)) <= 1e-12 * np.max(np.abs(b))


def test_split_diffusion_conserves_mass_on_a_refined_forest():
    """The split scheme's diffusion solve (I - dt D lap) w1 = w* keeps the
    area integral of w* (the conservative coarse-fine faces): the change of
    the integral over a step is dt times the integral of the reaction."""
    f = _refined(fmg.PERIODIC)
    x, y = fmg.cell_centres(f, 1.0)
    u = 1.0 - 0.5 * np.exp(-60 * ((x - 0.3) ** 2 + (y - 0.35) ** 2))
    v = 1.0 - u
    p = rd.GRAY_SCOTT_PARAMS
    dt = 0.5
    u1, v1 = fmg.rd_step(f, u, v, dt, rd.SPLIT, p, 1.0, fmg.PERIODIC)
    ru, rv = rd.reaction(u, v, p)
    area = ((1.0 / ((4 << (f.level.astype(np.int64) - 1)) * 16)) ** 2)[:, None, None]
    for w, w1, r in ((u, u1, ru), (v, v1, rv)):
        expect = np.sum(area * (w + dt * r))
        assert abs(np.sum(area * w1) - expect) <= 1e-12 * abs(expect)


def test_poisson_divergence_and_projection_on_a_uniform_forest():
    """Every leaf at level 2, periodic: the zero-mean Poisson solve, the
    central divergence and the projection equal oracle/rd.py's on the grid."""
    s = W.fmg_scheme(base=4, max_level=2, bc=fmg.PERIODIC)
    f = W.uniform_forest(s, level=2)
    x, y = fmg.cell_centres(f, 1.0)
    bx = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.3 * np.cos(4 * np.pi * y)
    by = np.cos(2 * np.pi * x + 0.4) * np.sin(6 * np.pi * y)
    G = lambda a: _uniform_to_grid(f, a)  # noqa: E731
    div = fmg.divergence(f, bx, by, 1.0, fmg.PERIODIC)
    ref = rd.central_div([G(bx), G(by)], 1.0, rd.PERIODIC)
    assert np.max(np.abs(G(div) - ref)) <= 1e-12 * np.max(np.abs(ref))
    phi = fmg.poisson(f, div, 1.0, fmg.PERIODIC)
    pref = rd.poisson_solve(ref, 1.0, rd.PERIODIC)
    assert np.max(np.abs(G(phi) - pref)) <= 1e-11 * np.max(np.abs(pref))
    bx1, by1, _ = fmg.divb_project(f, bx, by, 1.0, fmg.PERIODIC)
    (rx, ry), _ = rd.divb_project([G(bx), G(by)], 1.0, rd.PERIODIC)
    assert max(np.max(np.abs(G(bx1) - rx)), np.max(np.abs(G(by1) - ry))) <= 1e-11


def test_divergence_of_linear_fields_off_the_boundary():
    f = _refined(fmg.NEUMANN)
    x, y = fmg.cell_centres(f, 1.0)
    div = fmg.divergence(f, 0.7 * x - 0.4 * y + 0.1, 0.2 * x + 1.9 * y, 1.0, fmg.NEUMANN)
    n = (4 << (f.level.astype(np.int64) - 1)) * 16
    h = 1.0 / n[:, None, None]
    interior = (x > h) & (x < 1 - h) & (y > h) & (y < 1 - h)
    assert np.max(np.abs(div[interior] - 2.6)) <= 1e-10
    assert np.max(np.abs(div[~interior] - 2.6)) > 0.1  # the Neumann faces do not see the slope


def test_poisson_on_a_refined_forest():
    """Zero area-weighted mean; the residual of lap(phi) = f - mean(f) at
    rounding level; second order against phi = sin(2 pi x) sin(4 pi y) on a
    fixed three-level block forest with 8, 16 and 32 cells per block side."""
    f0 = _refined(fmg.PERIODIC)
    errs = []
    for nb in (8, 16, 32):
        s = W.fmg_scheme(base=4, max_level=3, bc=fmg.PERIODIC)
        s.block_nx = (nb, nb, 1)
        f = W.Forest(s, f0.level, f0.ijk)
        x, y = fmg.cell_centres(f, 1.0)
        pe = np.sin(2 * np.pi * x) * np.sin(4 * np.pi * y)
        rhs = -20 * np.pi ** 2 * pe + 0.5
        phi = fmg.poisson(f, rhs, 1.0, fmg.PERIODIC)
        area = fmg.cell_areas(f, 1.0)
        assert abs(np.sum(area * phi)) <= 1e-13
        mean = np.sum(area * rhs) / np.sum(area)
        res = fmg.apply(f, phi, 0.0, 1.0, fmg.PERIODIC) - (rhs - mean)
        assert np.max(np.abs(res)) <= 1e-8 * np.max(np.abs(rhs))
        errs.append(np.max(np.abs(phi - (pe - np.sum(area * pe) / np.sum(area)))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders >= 1.8), (errs, orders)


def test_projection_reduces_the_divergence_on_a_refined_forest():
    """The approximate projection on a three-level forest: the divergence left
    is what the compact lap and div(grad) disagree on -- O(h^2) on a uniform
    forest (0.2% of the initial divergence at 64^2 here), O(1) next to
    coarse-fine faces, where the residue concentrates (6%)."""
    f = _refined(fmg.PERIODIC)
    x, y = fmg.cell_centres(f, 1.0)
    bx = np.sin(2 * np.pi * x) + 0.2 * np.cos(2 * np.pi * y)
    by = np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
    d0 = np.max(np.abs(fmg.divergence(f, bx, by, 1.0, fmg.PERIODIC)))
    bx1, by1, _ = fmg.divb_project(f, bx, by, 1.0, fmg.PERIODIC)
    d1 = np.max(np.abs(fmg.divergence(f, bx1, by1, 1.0, fmg.PERIODIC)))
    assert d1 <= 0.1 * d0, (d0, d1)


# -- 3D (octree) ---------------------------------------------------------------

def _forest3(bc, nb=4, base=2, max_level=3, centre=(0.3, 0.35, 0.4), radius=0.2):
    s = W.fmg_scheme(base=base, max_level=max_level, bc=bc, ndim=3)
    f = W.fmg_forest(s, centre=centre, radius=radius)
    s.block_nx = (nb, nb, nb)
    return f


def test_3d_uniform_forest_is_the_uniform_grid():
    """Every leaf at level 2 (4^3 cells per block, 16^3 grid): the composite
    solve equals oracle/rd.py's spectral 3D solve, both boundary rules."""
    for bc in (fmg.PERIODIC, fmg.NEUMANN):
        s = W.fmg_scheme(base=2, max_level=2, bc=bc, ndim=3)
        s.block_nx = (4, 4, 4)
        f = W.uniform_forest(s, level=2)
        x, y, z = fmg.cell_centres(f, 1.0)
        rhs = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) * np.cos(4 * np.pi * z) + x * z
        u = fmg.solve(f, rhs, 13.0, 1.0, bc)
        grid = np.zeros((16, 16, 16))
        ug = np.zeros((16, 16, 16))
        for k in range(f.n):
            i, j, l = f.ijk[k]
            grid[4 * l:4 * l + 4, 4 * j:4 * j + 4, 4 * i:4 * i + 4] = rhs[k]
            ug[4 * l:4 * l + 4, 4 * j:4 * j + 4, 4 * i:4 * i + 4] = u[k]
        ref = rd.helmholtz_solve(grid, 13.0, 1.0, bc)
        assert np.max(np.abs(ug - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_3d_constants_linear_fields_and_conservation():
    for bc in (fmg.PERIODIC, fmg.NEUMANN):
        f = _forest3(bc)
        assert len(f.level_counts()) == 2 and min(f.level_counts()) == 2
        x, y, z = fmg.cell_centres(f, 1.0)
        # constants: lap(1) = 0
        assert np.max(np.abs(fmg.apply(f, np.ones_like(x), 0.0, 1.0, bc))) <= 1e-9
        # conservation: the volume-weighted sum of lap(u) vanishes for any u
        u = W.uniform01(9, x.size).reshape(x.shape)
        lap = fmg.apply(f, u, 0.0, 1.0, bc)
        vol = fmg.cell_areas(f, 1.0)
        assert abs(np.sum(vol * lap)) <= 1e-12 * np.sum(np.abs(lap) * vol)
    # linear data: lap vanishes off the Neumann domain boundary
    f = _forest3(fmg.NEUMANN)
    x, y, z = fmg.cell_centres(f, 1.0)
    lap = fmg.apply(f, 0.7 * x - 1.3 * y + 0.4 * z + 0.2, 0.0, 1.0, fmg.NEUMANN)
    n = (2 << (f.level.astype(np.int64) - 1)) * 4
    h = (1.0 / n).reshape(-1, 1, 1, 1)
    interior = np.ones(x.shape, dtype=bool)
    for c in (x, y, z):
        interior &= (c > h) & (c < 1 - h)
    assert interior.sum() > 0.3 * x.size
    assert np.max(np.abs(lap[interior])) <= 1e-9 * np.max(1.0 / h ** 2)
    assert np.max(np.abs(lap[~interior])) > 0.1


def test_3d_symmetry_and_second_order():
    """Mirror (x -> 1 - x) and axis-permutation symmetry on a forest symmetric
    under both, and the order of the maximum error on one block forest with 4
    and 6 cells per block side."""
    s = W.fmg_scheme(base=2, max_level=3, bc=fmg.NEUMANN, ndim=3)
    f = W.fmg_forest(s, centre=(0.5, 0.5, 0.5), radius=0.2)
    s.block_nx = (4, 4, 4)
    x, y, z = fmg.cell_centres(f, 1.0)

    def field(a, b, c):
        return np.exp(-30 * ((a - 0.3) ** 2 + (b - 0.6) ** 2 + (c - 0.45) ** 2)) + 0.3 * a

    lam = 11.0
    u = fmg.solve(f, field(x, y, z), lam, 1.0, fmg.NEUMANN)
    um = fmg.solve(f, field(1 - x, y, z), lam, 1.0, fmg.NEUMANN)
    up = fmg.solve(f, field(y, z, x), lam, 1.0, fmg.NEUMANN)
    key = {(int(l), int(i), int(j), int(k)): n for n, (l, (i, j, k)) in enumerate(zip(f.level, f.ijk))}
    for n in range(f.n):
        l, i, j, k = int(f.level[n]), *(int(v) for v in f.ijk[n])
        nbl = 2 << (l - 1)
        assert np.allclose(um[key[(l, nbl - 1 - i, j, k)]][:, :, ::-1], u[n], rtol=0, atol=1e-12)
        # up solves f(y, z, x), so up(x, y, z) = u(y, z, x): up's block
        # (i, j, k) is u's block (j, k, i) with its axes cycled
        assert np.allclose(up[n], u[key[(l, j, k, i)]].transpose(1, 2, 0), rtol=0, atol=1e-12)
    lam = 3.0
    f0 = _forest3(fmg.NEUMANN)
    errs = []
    for nb in (4, 6):
        s = W.fmg_scheme(base=2, max_level=3, bc=fmg.NEUMANN, ndim=3)
        s.block_nx = (nb, nb, nb)
        g = W.Forest(s, f0.level, f0.ijk)
        x, y, z = fmg.cell_centres(g, 1.0)
        ue = np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y) * np.cos(4 * np.pi * z)
        uu = fmg.solve(g, -(24 * np.pi ** 2 + lam) * ue, lam, 1.0, fmg.NEUMANN)
        errs.append(np.max(np.abs(uu - ue)))
    order = np.log(errs[0] / errs[1]) / np.log(6 / 4)
    assert order >= 1.7, (errs, order)


def test_3d_projection_on_a_uniform_forest_is_the_grid_projection():
    """Every leaf at level 2 of an octree (4^3 cells per block, periodic 16^3
    grid): divergence, zero-mean Poisson and projection equal oracle/rd.py's."""
    s = W.fmg_scheme(base=2, max_level=2, bc=fmg.PERIODIC, ndim=3)
    s.block_nx = (4, 4, 4)
    f = W.uniform_forest(s, level=2)
    x, y, z = fmg.cell_centres(f, 1.0)
    B = [np.sin(2 * np.pi * x) * np.cos(2 * np.pi * z), np.cos(2 * np.pi * y + 0.3) * np.sin(2 * np.pi * x),
         np.sin(4 * np.pi * z) + 0.2 * np.cos(2 * np.pi * y)]

    def G(a):
        out = np.zeros((16, 16, 16))
        for k in range(f.n):
            i, j, l = f.ijk[k]
            out[4 * l:4 * l + 4, 4 * j:4 * j + 4, 4 * i:4 * i + 4] = a[k]
        return out

    P, _ = fmg.divb_project_nd(f, B, 1.0, fmg.PERIODIC)
    R, _ = rd.divb_project([G(b) for b in B], 1.0, rd.PERIODIC)
    for d in range(3):
        assert np.max(np.abs(G(P[d]) - R[d])) <= 1e-11
