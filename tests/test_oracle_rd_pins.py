"""Pins of the oracle's elliptic solve and reaction-diffusion schemes
(Sec. 1.4 multigrid, Sec. 2.5 reaction-diffusion; oracle/rd.py).

* The discrete Laplacian is pinned on a whole basis: every Fourier mode
  (periodic) and every cosine mode (Neumann) of small grids is an
  eigenvector with the closed-form eigenvalue, and quadratics are
  differentiated exactly in the interior.
* The exact Helmholtz solve is checked against a dense solve of a matrix
  assembled from the stencil by index loops written here, against a
  manufactured continuum solution at second order, and by the mass
  identity lambda sum(phi) = -sum(f).
* The time schemes: Table 1's printed explicit limits; fixed points of both
  models; the steps against an accurate stiff integration (scipy Radau) of
  the semi-discrete system: Euler and split at first order, midpoint and
  IMEX at second order, matching the paper's IMEX-versus-split finding;
  conservation of each species' mass by the diffusion (Neumann) in the
  split and IMEX solves with the reaction switched off; and the mirror
  symmetry of the 2D Schnakenberg initial condition.
"""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import rd as R
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rd_table1_dt_limits.txt")


def _modes(nd, n, bc):
    """Eigenvectors (real arrays) and closed-form eigenvalues of the
    unit-spacing-free second difference, h = 1 (L = n)."""
    ks = np.array(np.meshgrid(*([np.arange(n)] * nd), indexing="ij")).reshape(nd, -1).T
    idx = np.arange(n)
    for k in ks:
        vec = np.ones([n] * nd)
        lam = 0.0
        for d in range(nd):
            kd = k[d]
            if bc == R.PERIODIC:
                lam += 2.0 * np.cos(2.0 * np.pi * kd / n) - 2.0
            else:
                lam += 2.0 * np.cos(np.pi * kd / n) - 2.0
            sh = [1] * nd
            sh[nd - 1 - d] = n
            vec = vec * (np.cos(2.0 * np.pi * kd * idx / n) if bc == R.PERIODIC
                         else np.cos(np.pi * kd * (idx + 0.5) / n)).reshape(sh)
        yield vec, lam
        if bc == R.PERIODIC:
            # the sine partner of each direction's cosine (one at a time)
            for d in range(nd):
                if k[d] == 0:
                    continue
                v2 = np.ones([n] * nd)
                for e in range(nd):
                    sh = [1] * nd
                    sh[nd - 1 - e] = n
                    fn = np.sin if e == d else np.cos
                    v2 = v2 * fn(2.0 * np.pi * k[e] * idx / n).reshape(sh)
                yield v2, lam


@pytest.mark.parametrize("nd,n", [(2, 8), (3, 4)])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_laplacian_on_every_eigenmode(nd, n, bc):
    count = 0
    for vec, lam in _modes(nd, n, bc):
        got = R.laplacian(vec, float(n), bc)  # h = 1
        assert np.abs(got - lam * vec).max() <= 1e-12 * max(1.0, np.abs(vec).max()), lam
        count += 1
    assert count >= n ** nd


def test_laplacian_of_quadratics_is_exact_inside():
    n, L = 16, 2.0
    x, y, z = W.rd_cell_centres(3, n, L)
    w = 3.0 * x * x - y * y + 0.5 * z * z + x * y
    lap = R.laplacian(w, L, R.NEUMANN)
    inner = lap[1:-1, 1:-1, 1:-1]
    assert np.abs(inner - (6.0 - 2.0 + 1.0)).max() < 1e-11


def _dense_matrix(nd, n, length, bc, lam):
    """A = lap - lambda I assembled cell by cell (index loops)."""
    N = n ** nd
    A = np.zeros((N, N))
    ih2 = (n / length) ** 2
    for c in range(N):
        ijk = [(c // n ** d) % n for d in range(nd)]  # x, y, z
        A[c, c] -= lam
        for d in range(nd):
            for s in (-1, 1):
                m = list(ijk)
                t = m[d] + s
                if bc == R.PERIODIC:
                    t %= n
                else:
                    t = min(max(t, 0), n - 1)
                m[d] = t
                A[c, sum(m[e] * n ** e for e in range(nd))] += ih2
                A[c, c] -= ih2
    return A


@pytest.mark.parametrize("nd,n", [(2, 8), (3, 4)])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
@pytest.mark.parametrize("lam", [0.3, 50.0])
def test_exact_solve_matches_a_dense_solve(nd, n, bc, lam):
    rng = np.random.default_rng(7 + nd + 10 * bc)
    f = rng.standard_normal([n] * nd)
    phi = R.helmholtz_solve(f, lam, 1.7, bc)
    ref = np.linalg.solve(_dense_matrix(nd, n, 1.7, bc, lam), f.ravel()).reshape(f.shape)
    assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()
    # and the residual through the stencil code
    r = f - R.helmholtz_apply(phi, lam, 1.7, bc)
    assert np.abs(r).max() <= 1e-10 * np.abs(f).max()
    # mass: every row of lap sums to zero
    assert lam * phi.sum() == pytest.approx(-f.sum(), abs=1e-11 * np.abs(f).sum())


@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_manufactured_solution_converges_at_second_order(bc):
    """phi = cos(2 pi x) cos(2 pi y) (periodic) or cos(pi x) cos(pi y)
    (Neumann) on the unit square solves the continuum equation with
    f = (-(k^2 + k^2) - lambda) phi."""
    lam = 10.0
    k = 2.0 * np.pi if bc == R.PERIODIC else np.pi
    errs = []
    for n in (32, 64, 128):
        x, y = W.rd_cell_centres(2, n, 1.0)
        exact = np.cos(k * x) * np.cos(k * y)
        f = (-2.0 * k * k - lam) * exact
        errs.append(np.abs(R.helmholtz_solve(f, lam, 1.0, bc) - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.95) and np.all(orders < 2.05), (errs, orders)


def test_table1_explicit_limits():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for name, dmax, *vals in rows:
        for h, printed in zip((1 / 128, 1 / 256, 1 / 512), vals):
            got = R.explicit_dt_limit(h, 2, float(dmax))
            p = float(printed)
            # two printed significant digits
            assert abs(got - p) <= 0.05 * p, (name, h, got, p)


@pytest.mark.parametrize("scheme", [R.EULER, R.MIDPOINT, R.SPLIT, R.IMEX])
def test_fixed_points(scheme):
    p = R.SCHNAKENBERG_PARAMS
    a, b = p["p2"], p["p3"]
    u = np.full((8, 8), a + b)
    v = np.full((8, 8), b / (a + b) ** 2)
    u1, v1 = R.run(u, v, 1e-3, 5, scheme, p, 1.0, R.NEUMANN)
    assert np.abs(u1 - u).max() < 1e-12 and np.abs(v1 - v).max() < 1e-12
    g = R.GRAY_SCOTT_PARAMS
    u, v = np.ones((8, 8)), np.zeros((8, 8))
    u1, v1 = R.run(u, v, 0.5, 3, scheme, g, 2.0, R.PERIODIC)
    if scheme in (R.EULER, R.MIDPOINT):
        assert np.array_equal(u1, u) and np.array_equal(v1, v)
    else:
        assert np.abs(u1 - 1.0).max() < 1e-13 and np.abs(v1).max() < 1e-13


def _semi_discrete_reference(u0, v0, p, L, bc, t):
    shape = u0.shape
    N = u0.size

    def F(_, y):
        fu, fv = R.rhs_full(y[:N].reshape(shape), y[N:].reshape(shape), p, L, bc)
        return np.concatenate([fu.ravel(), fv.ravel()])

    sol = solve_ivp(F, (0.0, t), np.concatenate([u0.ravel(), v0.ravel()]), method="Radau", rtol=1e-11,
                    atol=1e-13)
    assert sol.success
    y = sol.y[:, -1]
    return y[:N].reshape(shape), y[N:].reshape(shape)


@pytest.fixture(scope="module")
def schnakenberg_16():
    u0, v0, L = W.schnakenberg_initial(2, 16)
    p = R.SCHNAKENBERG_PARAMS
    t = 0.02
    return u0, v0, L, p, t, _semi_discrete_reference(u0, v0, p, L, R.NEUMANN, t)


@pytest.mark.parametrize("scheme,dts,lo,hi", [
    (R.IMEX, (2e-3, 1e-3, 5e-4), 1.8, 2.2),
    (R.SPLIT, (2e-3, 1e-3, 5e-4), 0.7, 1.15),
    (R.MIDPOINT, (4e-5, 2e-5, 1e-5), 1.8, 2.2),
    (R.EULER, (4e-5, 2e-5, 1e-5), 0.9, 1.1),
])
def test_time_order_against_a_stiff_integrator(schnakenberg_16, scheme, dts, lo, hi):
    """The paper's comparison (Sec. 2.5.2, Fig. schnakenberg-conv): IMEX
    second order, the split scheme at most first order."""
    u0, v0, L, p, t, (ur, vr) = schnakenberg_16
    errs = []
    for dt in dts:
        n = int(round(t / dt))
        u, v = R.run(u0, v0, dt, n, scheme, p, L, R.NEUMANN)
        errs.append(np.sqrt(np.mean((u - ur) ** 2) + np.mean((v - vr) ** 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > lo) and np.all(orders < hi), (errs, orders)


@pytest.mark.parametrize("scheme", [R.SPLIT, R.IMEX])
def test_diffusion_conserves_mass(scheme):
    p = dict(R.SCHNAKENBERG_PARAMS, p1=0.0)  # kappa = 0: pure diffusion
    u0, v0, L = W.schnakenberg_initial(2, 32)
    u, v = R.run(u0, v0, 1e-2, 4, scheme, p, L, R.NEUMANN)
    assert u.sum() == pytest.approx(u0.sum(), rel=1e-13)
    assert v.sum() == pytest.approx(v0.sum(), rel=1e-13)
    assert np.abs(u - u0).max() > 1e-3  # it did diffuse


def test_schnakenberg_2d_keeps_its_mirror_symmetry():
    u0, v0, L = W.schnakenberg_initial(2, 32)
    u, v = R.run(u0, v0, 1e-3, 10, R.IMEX, R.SCHNAKENBERG_PARAMS, L, R.NEUMANN)
    assert np.abs(u - u[::-1, :]).max() < 1e-12
    assert np.abs(v - v[::-1, :]).max() < 1e-12
    assert np.abs(u - u[:, ::-1]).max() > 1e-3


def test_rejects_nonpositive_lambda():
    with pytest.raises(ValueError):
        R.helmholtz_solve(np.zeros((4, 4)), 0.0, 1.0, R.PERIODIC)


# -- Poisson (lambda = 0) and the divergence control of Sec. 2.4 -------------

@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_poisson_solve_is_the_minimum_norm_solution(bc):
    """The dense singular system solved by least squares (numpy lstsq gives
    the minimum-norm solution, which for a symmetric matrix with the
    constants as null space is the zero-mean one)."""
    n = 8
    rng = np.random.default_rng(3 + bc)
    f = rng.standard_normal((n, n))
    f -= f.mean()
    phi = R.poisson_solve(f, 1.3, bc)
    A = _dense_matrix(2, n, 1.3, bc, 0.0)
    ref = np.linalg.lstsq(A, f.ravel(), rcond=None)[0].reshape(n, n)
    assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(phi.mean()) < 1e-14 * np.abs(phi).max()
    r = f - R.laplacian(phi, 1.3, bc)
    assert np.abs(r).max() <= 1e-10 * np.abs(f).max()


def test_poisson_manufactured_second_order():
    errs = []
    for n in (32, 64, 128):
        x, y = W.rd_cell_centres(2, n, 1.0)
        exact = np.cos(2 * np.pi * x) * np.sin(4 * np.pi * y)
        f = -(4 + 16) * np.pi ** 2 * exact
        got = R.poisson_solve(f, 1.0, R.PERIODIC)
        errs.append(np.abs(got - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.95) and np.all(orders < 2.05), (errs, orders)


def _curl_field(n, L=1.0, nd=2):
    """A field that is divergence-free under central differences: the
    central-difference curl of a smooth potential (central differences in
    different directions commute)."""
    xs = W.rd_cell_centres(nd, n, L)
    if nd == 2:
        x, y = xs
        A = np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L) + 0.3 * np.cos(4 * np.pi * x / L)
        return [R.central_diff(A, 1, L, R.PERIODIC), -R.central_diff(A, 0, L, R.PERIODIC)]
    x, y, z = xs
    Ax = np.sin(2 * np.pi * y / L) * np.cos(2 * np.pi * z / L)
    Ay = np.cos(2 * np.pi * x / L) * np.sin(4 * np.pi * z / L)
    Az = np.sin(2 * np.pi * (x + y) / L)
    cd = lambda w, d: R.central_diff(w, d, L, R.PERIODIC)
    return [cd(Az, 1) - cd(Ay, 2), cd(Ax, 2) - cd(Az, 0), cd(Ay, 0) - cd(Ax, 1)]


@pytest.mark.parametrize("nd", [2, 3])
def test_projection_leaves_a_discretely_solenoidal_field_alone(nd):
    n = 32 if nd == 2 else 16
    B = _curl_field(n, nd=nd)
    assert np.abs(R.central_div(B, 1.0, R.PERIODIC)).max() < 1e-11
    P, phi = R.divb_project(B, 1.0, R.PERIODIC)
    for d in range(nd):
        assert np.abs(P[d] - B[d]).max() < 1e-11


def test_projection_removes_a_smooth_gradient_at_second_order():
    """B* = B_sol + grad(psi) with psi smooth: the projection returns B_sol
    up to O(h^2), and the central divergence drops by orders of magnitude."""
    errs, ratios = [], []
    for n in (32, 64, 128):
        x, y = W.rd_cell_centres(2, n, 1.0)
        Bs = _curl_field(n)
        psi = np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y)
        gx = -2 * np.pi * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        gy = -2 * np.pi * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
        B = [Bs[0] + gx, Bs[1] + gy]
        P, _ = R.divb_project(B, 1.0, R.PERIODIC)
        errs.append(max(np.abs(P[0] - Bs[0]).max(), np.abs(P[1] - Bs[1]).max()))
        ratios.append(np.abs(R.central_div(P, 1.0, R.PERIODIC)).max() /
                      np.abs(R.central_div(B, 1.0, R.PERIODIC)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.9), (errs, orders)
    assert max(ratios) < 1e-2, ratios


# -- variable coefficient (Sec. 1.4) ------------------------------------------

def test_variable_coefficient_reduces_to_the_constant_one():
    rng = np.random.default_rng(11)
    for nd, n, bc in [(2, 16, R.PERIODIC), (2, 16, R.NEUMANN), (3, 8, R.NEUMANN)]:
        f = rng.standard_normal((n,) * nd)
        eps = np.ones_like(f)
        a = R.helmholtz_var_solve(f, eps, 3.0, 1.0, bc)
        b = R.helmholtz_solve(f, 3.0, 1.0, bc)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
        phi = rng.standard_normal(f.shape)
        assert np.abs(R.helmholtz_var_apply(phi, eps, 3.0, 1.0, bc) - R.helmholtz_apply(phi, 3.0, 1.0, bc)).max() \
            < 1e-9


@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_variable_coefficient_matrix_properties(bc):
    """Symmetric, an M-matrix (off-diagonals >= 0 in lap - lambda form, i.e.
    lambda I - A has non-positive off-diagonals) with row sums -lambda, so
    the residual bound |e| <= |r| / lambda holds as in the constant case;
    and the matrix applied to a vector equals the stencil code."""
    rng = np.random.default_rng(12)
    n = 8
    eps = 0.2 + rng.random((n, n))
    A = R.helmholtz_var_matrix(eps, 2.5, 1.0, bc).toarray()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    off = A - np.diag(np.diag(A))
    assert off.min() >= 0.0
    assert np.abs(A.sum(axis=1) + 2.5).max() < 1e-9 * np.abs(A).max()
    phi = rng.standard_normal((n, n))
    assert np.abs(A @ phi.ravel() - R.helmholtz_var_apply(phi, eps, 2.5, 1.0, bc).ravel()).max() \
        < 1e-12 * np.abs(A).max()


def test_variable_coefficient_manufactured_second_order():
    """phi = cos(pi x) cos(pi y) (zero normal derivative on the unit square),
    eps = 1 + 0.5 sin(pi x) sin(pi y)... with f = div(eps grad phi) - lambda phi
    computed from the continuum formulas."""
    lam = 5.0
    errs = []
    for n in (32, 64, 128):
        x, y = W.rd_cell_centres(2, n, 1.0)
        c, s_ = np.cos, np.sin
        phi = c(np.pi * x) * c(np.pi * y)
        eps = 1.0 + 0.5 * c(np.pi * x) ** 2 * c(np.pi * y) ** 2
        px = -np.pi * s_(np.pi * x) * c(np.pi * y)
        py = -np.pi * c(np.pi * x) * s_(np.pi * y)
        ex = 0.5 * 2 * c(np.pi * x) * (-np.pi * s_(np.pi * x)) * c(np.pi * y) ** 2
        ey = 0.5 * 2 * c(np.pi * y) * (-np.pi * s_(np.pi * y)) * c(np.pi * x) ** 2
        lap = -2 * np.pi ** 2 * phi
        f = ex * px + ey * py + eps * lap - lam * phi
        got = R.helmholtz_var_solve(f, eps, lam, 1.0, R.NEUMANN)
        errs.append(np.abs(got - phi).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), (errs, orders)
