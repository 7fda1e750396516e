"""GPU (HIP, gfx950) multigrid Helmholtz solver and reaction-diffusion steps
against the CPU oracle (oracle/rd.py), through the C-ABI (include/amrv_mg.h).

Bars:
* Helmholtz solve: lambda I - lap is an M-matrix whose rows sum to lambda,
  so max |phi_gpu - phi_exact| <= r / lambda, r the true max residual of the
  GPU's answer.  The GPU reports r computed in binary64; the test allows
  twice that plus 1e-12 of max |phi| for the rounding of both sides.
* Explicit Euler and midpoint steps: bitwise (same operation order, no
  contraction on either side).
* Split and IMEX steps: the solves run to tol = 1e-12, so w* is within
  1e-12 max|f| / lambda of the exact one; IMEX's second stage multiplies that
  by at most 1 + dt/2 (D 4 d / h^2 + reaction Lipschitz), a few hundred
  here; over a few steps the relative difference stays below 1e-8.
"""
import numpy as np
import pytest

from oracle import rd as R
import workloads as W

pytestmark = pytest.mark.gpu


def _mg():
    import torch

    from paper_2004_03275_amd import multigrid as M

    return torch, M


def _seeded(shape, seed):
    return W.uniform01(seed, int(np.prod(shape))).reshape(shape) * 2.0 - 1.0


@pytest.mark.parametrize("nd,n", [(2, 16), (2, 64), (2, 256), (3, 8), (3, 16), (3, 64)])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
@pytest.mark.parametrize("lam", [1.0, 4000.0])
def test_helmholtz_solve_within_the_residual_bound(nd, n, bc, lam):
    torch, M = _mg()
    L = 1.0
    shape = (n,) * nd
    f = _seeded(shape, 11 + n + nd) + np.cos(2 * np.pi * W.rd_cell_centres(nd, n, L)[0])
    exact = R.helmholtz_solve(f, lam, L, bc)
    mg = M.GpuMultigrid(nd, n, bc, L, nfields=1)
    ft = torch.tensor(f, device="cuda:0").contiguous()
    phi = torch.zeros_like(ft)
    cycles, res, fmax = mg.solve(ft, phi, lam, tol=1e-10, max_cycles=40)
    got = phi.cpu().numpy()
    err = np.abs(got - exact).max()
    bound = 2.0 * res[0] / lam + 1e-12 * np.abs(exact).max()
    print(f"[mg] {nd}D n={n} bc={bc} lam={lam}: {cycles} cycles, res {res[0]:.2e}, err {err:.2e}, "
          f"bound {bound:.2e}", flush=True)
    assert fmax[0] == np.abs(f).max()
    assert res[0] <= 1e-10 * fmax[0]
    assert err <= bound
    assert cycles <= 20  # V(2,2) reduces the max residual >= 3x per cycle (about 0.1 in 2D, 0.25 in 3D)
    mg.close()


@pytest.mark.parametrize("nd,n", [(2, 128), (3, 32)])
def test_two_fields_graph_and_direct_launches_agree(nd, n):
    """Both fields of one solve match separate one-field solves, and graph
    replay matches direct launches bit for bit."""
    torch, M = _mg()
    shape = (n,) * nd
    f = np.stack([_seeded(shape, 5), _seeded(shape, 6)])
    lam = np.array([30.0, 700.0])
    out = []
    for graph in (True, False):
        mg = M.GpuMultigrid(nd, n, R.NEUMANN, 2.0, nfields=2, graph=graph)
        ft = torch.tensor(f, device="cuda:0").contiguous()
        phi = torch.zeros_like(ft)
        c, res, _ = mg.solve(ft, phi, lam, tol=1e-9)
        out.append(phi.cpu().numpy())
        mg.close()
    assert np.array_equal(out[0], out[1])
    for k in range(2):
        exact = R.helmholtz_solve(f[k], lam[k], 2.0, R.NEUMANN)
        assert np.abs(out[0][k] - exact).max() <= 2e-9 * np.abs(f[k]).max() / lam[k] + 1e-12


def test_initial_guess_that_solves_takes_no_cycle():
    torch, M = _mg()
    n = 32
    exact = R.helmholtz_solve(_seeded((n, n), 3), 50.0, 1.0, R.PERIODIC)
    f = R.helmholtz_apply(exact, 50.0, 1.0, R.PERIODIC)
    mg = M.GpuMultigrid(2, n, R.PERIODIC, 1.0, nfields=1)
    phi = torch.tensor(exact, device="cuda:0").contiguous()
    c, res, _ = mg.solve(torch.tensor(f, device="cuda:0").contiguous(), phi, 50.0, tol=1e-7)
    assert c == 0
    assert np.array_equal(phi.cpu().numpy(), exact)


def _rd_case(model, nd, n):
    if model == R.SCHNAKENBERG:
        u, v, L = W.schnakenberg_initial(nd, n)
        return u, v, L, R.NEUMANN, R.SCHNAKENBERG_PARAMS
    u, v, L = W.gray_scott_initial(n)
    return u, v, L, R.PERIODIC, R.GRAY_SCOTT_PARAMS


@pytest.mark.parametrize("model,nd,n,dt,steps", [
    (R.SCHNAKENBERG, 2, 64, 5e-5, 8), (R.SCHNAKENBERG, 3, 16, 2e-4, 5), (R.GRAY_SCOTT, 2, 64, 0.5, 6)])
@pytest.mark.parametrize("scheme", [R.EULER, R.MIDPOINT])
def test_explicit_steps_bitwise(model, nd, n, dt, steps, scheme):
    torch, M = _mg()
    u0, v0, L, bc, p = _rd_case(model, nd, n)
    ru, rv = R.run(u0, v0, dt, steps, scheme, p, L, bc)
    mg = M.GpuMultigrid(nd, n, bc, L, nfields=2)
    u = torch.tensor(u0, device="cuda:0").contiguous()
    v = torch.tensor(v0, device="cuda:0").contiguous()
    mg.rd_step(u, v, dt, scheme, p, nsteps=steps)
    gu, gv = u.cpu().numpy(), v.cpu().numpy()
    print(f"[rd] explicit model={model} {nd}D n={n} scheme={scheme}: differing "
          f"{int(np.count_nonzero(gu != ru) + np.count_nonzero(gv != rv))}", flush=True)
    assert np.array_equal(gu, ru) and np.array_equal(gv, rv)
    mg.close()


@pytest.mark.parametrize("model,nd,n,dt,steps", [
    (R.SCHNAKENBERG, 2, 64, 1e-3, 4), (R.SCHNAKENBERG, 2, 256, 1e-3, 3), (R.SCHNAKENBERG, 3, 32, 1e-3, 3),
    (R.GRAY_SCOTT, 2, 128, 0.5, 4)])
@pytest.mark.parametrize("scheme", [R.SPLIT, R.IMEX])
def test_implicit_steps_match_the_exact_solves(model, nd, n, dt, steps, scheme):
    torch, M = _mg()
    u0, v0, L, bc, p = _rd_case(model, nd, n)
    ru, rv = R.run(u0, v0, dt, steps, scheme, p, L, bc)
    mg = M.GpuMultigrid(nd, n, bc, L, nfields=2)
    u = torch.tensor(u0, device="cuda:0").contiguous()
    v = torch.tensor(v0, device="cuda:0").contiguous()
    cycles, res = mg.rd_step(u, v, dt, scheme, p, nsteps=steps, tol=1e-12, max_cycles=60)
    gu, gv = u.cpu().numpy(), v.cpu().numpy()
    eu = np.abs(gu - ru).max() / np.abs(ru).max()
    ev = np.abs(gv - rv).max() / max(np.abs(rv).max(), 1e-300)
    print(f"[rd] model={model} {nd}D n={n} scheme={scheme}: {cycles} cycles over {steps} steps, "
          f"rel max diff u {eu:.2e} v {ev:.2e}", flush=True)
    assert eu <= 1e-8 and ev <= 1e-8
    assert np.abs(gu - u0).max() > 1e-6  # it moved
    mg.close()


def test_paper_tolerance_step_is_close_to_the_exact_step():
    """At the paper's tol = 1e-7 (Sec. 2.5.2) one IMEX step of the 256^2
    Schnakenberg run stays within the residual bound propagated through the
    second stage."""
    torch, M = _mg()
    u0, v0, L, bc, p = _rd_case(R.SCHNAKENBERG, 2, 256)
    dt = 1e-3
    ru, rv = R.step(u0, v0, dt, R.IMEX, p, L, bc)
    mg = M.GpuMultigrid(2, 256, bc, L, nfields=2)
    u = torch.tensor(u0, device="cuda:0").contiguous()
    v = torch.tensor(v0, device="cuda:0").contiguous()
    cycles, res = mg.rd_step(u, v, dt, R.IMEX, p, nsteps=1, tol=1e-7)
    lam = np.array([2.0 / (dt * p["Du"]), 2.0 / (dt * p["Dv"])])
    # w* is off by at most delta = max_k res_k / lambda_k in every cell; the
    # second stage adds dt/2 (F(w*) - F(w*_exact)), F's max-norm Lipschitz
    # constant being at most D_max 8/h^2 plus the reaction Jacobian's row
    # sums, kappa (1 + 2 u v + u^2) with u <= 2, v <= 1 here
    ih2 = 256.0 ** 2
    delta = max(res[0] / lam[0], res[1] / lam[1])
    amp = 0.5 * dt * (max(p["Du"], p["Dv"]) * 8.0 * ih2 + p["p1"] * (1.0 + 4.0 + 4.0))
    assert u0.max() < 2.0 and v0.max() < 1.0
    for k, (g, r) in enumerate(((u, ru), (v, rv))):
        err = np.abs(g.cpu().numpy() - r).max()
        assert err <= 2.0 * amp * delta + 1e-12, (k, err, res)
    print(f"[rd] paper tol: {cycles} cycles, residuals {res}", flush=True)
    mg.close()


def test_errors():
    torch, M = _mg()
    from paper_2004_03275_amd import _native as N

    mg = M.GpuMultigrid(2, 32, R.NEUMANN, 1.0, nfields=1)
    f = torch.ones(32 * 32, dtype=torch.float64, device="cuda:0")
    phi = torch.zeros_like(f)
    with pytest.raises(N.AmrvError) as e:
        mg.solve(f, phi, -1.0)
    assert e.value.code == N.EINVAL
    with pytest.raises(N.AmrvError) as e:  # lambda = 0 with a right-hand side that does not sum to zero
        mg.solve(f, phi, 0.0, tol=1e-9, max_cycles=20)
    assert e.value.code == N.ENOTCONVERGED
    with pytest.raises(N.AmrvError) as e:
        mg.solve(torch.tensor(_seeded((32, 32), 9), device="cuda:0").contiguous(), phi, 1.0, tol=1e-15,
                 max_cycles=1)
    assert e.value.code == N.ENOTCONVERGED
    u = torch.ones(32 * 32, dtype=torch.float64, device="cuda:0")
    with pytest.raises(N.AmrvError) as e:
        mg.rd_step(u, u.clone(), 1e-3, R.IMEX, R.SCHNAKENBERG_PARAMS)
    assert e.value.code == N.EINVAL  # implicit steps need two fields
    mg.close()
    mg = M.GpuMultigrid(2, 32, R.NEUMANN, 1.0, nfields=1)
    bad = torch.full((32 * 32,), float("nan"), dtype=torch.float64, device="cuda:0")
    with pytest.raises(N.AmrvError) as e:
        mg.solve(bad, torch.zeros_like(bad), 1.0)
    assert e.value.code == N.ENONPHYSICAL
    mg.close()


@pytest.mark.parametrize("n", [128, 256, 512, 2048])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_tiled_and_per_colour_smoothers_agree_bitwise(n, bc):
    """The tiled 2D level kernels (halo re-sweeps in LDS) reproduce the
    per-colour launches bit for bit: solve and IMEX steps.  At 2048^2 a
    level has 8,192 tile blocks, far more than are resident at once, so a
    block that stages late must still see its neighbours' old values."""
    torch, M = _mg()
    f = np.stack([_seeded((n, n), 21), _seeded((n, n), 22)])
    out = []
    for sm in (M.TILED, M.PER_COLOUR):
        mg = M.GpuMultigrid(2, n, bc, 1.0, nfields=2, smoother=sm)
        ft = torch.tensor(f, device="cuda:0").contiguous()
        phi = torch.zeros_like(ft)
        c, res, _ = mg.solve(ft, phi, [3.0, 900.0], tol=1e-11)
        u0, v0, L = W.schnakenberg_initial(2, n)
        u = torch.tensor(u0, device="cuda:0").contiguous()
        v = torch.tensor(v0, device="cuda:0").contiguous()
        c2, _ = mg.rd_step(u, v, 1e-3, M.IMEX, R.SCHNAKENBERG_PARAMS, nsteps=2)
        out.append((c, res.copy(), phi.cpu().numpy(), c2, u.cpu().numpy(), v.cpu().numpy()))
        mg.close()
    a, b = out
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert a[3] == b[3] and np.array_equal(a[4], b[4]) and np.array_equal(a[5], b[5])


@pytest.mark.parametrize("nd,n", [(2, 4), (3, 4), (2, 8)])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_smallest_grids(nd, n, bc):
    """n = 4: one level above the exact 2-per-side solve, all in the tail."""
    torch, M = _mg()
    f = _seeded((n,) * nd, 40 + n)
    lam = 7.0
    exact = R.helmholtz_solve(f, lam, 1.0, bc)
    mg = M.GpuMultigrid(nd, n, bc, 1.0, nfields=1)
    phi = torch.zeros(f.size, dtype=torch.float64, device="cuda:0")
    c, res, _ = mg.solve(torch.tensor(f.ravel(), device="cuda:0"), phi, lam, tol=1e-13, max_cycles=60)
    assert np.abs(phi.cpu().numpy().reshape(f.shape) - exact).max() <= 2.0 * res[0] / lam + 1e-14
    mg.close()


@pytest.mark.parametrize("pre,post", [(1, 1), (4, 4), (1, 3), (5, 5)])
def test_sweep_counts_tiled_and_fallback(pre, post):
    """Tiled halos for 1..4 sweeps; 5 sweeps exceed the largest halo and run
    per colour.  Either way the two smoother settings agree bit for bit and
    the answer meets the residual bound."""
    torch, M = _mg()
    n, lam = 256, 2.0
    f = _seeded((n, n), 50 + pre)
    exact = R.helmholtz_solve(f, lam, 1.0, R.NEUMANN)
    out = []
    for sm in (M.TILED, M.PER_COLOUR):
        mg = M.GpuMultigrid(2, n, R.NEUMANN, 1.0, nfields=1, pre=pre, post=post, smoother=sm)
        phi = torch.zeros(n * n, dtype=torch.float64, device="cuda:0")
        c, res, _ = mg.solve(torch.tensor(f.ravel(), device="cuda:0"), phi, lam, tol=1e-10, max_cycles=60)
        out.append((c, phi.cpu().numpy()))
        assert np.abs(out[-1][1].reshape(n, n) - exact).max() <= 2.0 * res[0] / lam + 1e-13
        mg.close()
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])


def test_periodic_3d_and_gray_scott_512():
    torch, M = _mg()
    # 3D periodic IMEX on a Schnakenberg state (periodic faces instead of Neumann)
    u0, v0, L = W.schnakenberg_initial(3, 32)
    p = R.SCHNAKENBERG_PARAMS
    ru, rv = R.run(u0, v0, 1e-3, 2, R.IMEX, p, L, R.PERIODIC)
    mg = M.GpuMultigrid(3, 32, R.PERIODIC, L, nfields=2)
    u = torch.tensor(u0, device="cuda:0").contiguous()
    v = torch.tensor(v0, device="cuda:0").contiguous()
    mg.rd_step(u, v, 1e-3, R.IMEX, p, nsteps=2, tol=1e-12, max_cycles=60)
    assert np.abs(u.cpu().numpy() - ru).max() / np.abs(ru).max() <= 1e-8
    assert np.abs(v.cpu().numpy() - rv).max() / np.abs(rv).max() <= 1e-8
    mg.close()
    # Gray-Scott split steps on 512^2 (the paper's finest Gray-Scott level)
    u0, v0, L = W.gray_scott_initial(512)
    g = R.GRAY_SCOTT_PARAMS
    ru, rv = R.run(u0, v0, 0.5, 2, R.SPLIT, g, L, R.PERIODIC)
    mg = M.GpuMultigrid(2, 512, R.PERIODIC, L, nfields=2)
    u = torch.tensor(u0, device="cuda:0").contiguous()
    v = torch.tensor(v0, device="cuda:0").contiguous()
    mg.rd_step(u, v, 0.5, R.SPLIT, g, nsteps=2, tol=1e-12, max_cycles=60)
    assert np.abs(u.cpu().numpy() - ru).max() / np.abs(ru).max() <= 1e-8
    assert np.abs(v.cpu().numpy() - rv).max() / np.abs(rv).max() <= 1e-8
    mg.close()


# -- Poisson (lambda = 0) and the divergence control of Sec. 2.4 -------------

def _mu1(n, L, bc):
    """Smallest non-zero eigenvalue magnitude of the discrete Laplacian."""
    theta = 2 * np.pi / n if bc == R.PERIODIC else np.pi / n
    return (2.0 - 2.0 * np.cos(theta)) * (n / L) ** 2


@pytest.mark.parametrize("nd,n", [(2, 64), (2, 256), (3, 32)])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
def test_poisson_solve_up_to_a_constant(nd, n, bc):
    """lambda = 0 with a right-hand side that sums to zero: the GPU answer
    minus its mean equals the oracle's zero-mean solution within
    sqrt(cells) max|r| / mu_1 (2-norm bound of the error orthogonal to the
    constants)."""
    torch, M = _mg()
    f = _seeded((n,) * nd, 70 + n) + np.cos(2 * np.pi * W.rd_cell_centres(nd, n, 1.0)[1])
    f -= f.mean()
    exact = R.poisson_solve(f, 1.0, bc)
    mg = M.GpuMultigrid(nd, n, bc, 1.0, nfields=1)
    phi = torch.zeros(f.size, dtype=torch.float64, device="cuda:0")
    c, res, fmax = mg.solve(torch.tensor(f.ravel(), device="cuda:0"), phi, 0.0, tol=1e-11, max_cycles=60)
    got = phi.cpu().numpy().reshape(f.shape)
    got -= got.mean()
    err = np.abs(got - exact).max()
    bound = 2.0 * np.sqrt(f.size) * (res[0] + abs(f.mean())) / _mu1(n, 1.0, bc) + 1e-12 * np.abs(exact).max()
    print(f"[mg] poisson {nd}D n={n} bc={bc}: {c} cycles, res {res[0]:.2e}, err {err:.2e}, bound {bound:.2e}",
          flush=True)
    assert err <= bound
    mg.close()


def _solenoidal_plus_gradient(nd, n):
    xs = W.rd_cell_centres(nd, n, 1.0)
    cd = lambda w, d: R.central_diff(w, d, 1.0, R.PERIODIC)
    if nd == 2:
        x, y = xs
        A = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.3 * np.cos(4 * np.pi * x)
        psi = np.cos(2 * np.pi * x) * np.cos(4 * np.pi * y)
        B = [cd(A, 1), -cd(A, 0)]
    else:
        x, y, z = xs
        Ax = np.sin(2 * np.pi * y) * np.cos(2 * np.pi * z)
        Ay = np.cos(2 * np.pi * x) * np.sin(4 * np.pi * z)
        Az = np.sin(2 * np.pi * (x + y))
        psi = np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.cos(2 * np.pi * z)
        B = [cd(Az, 1) - cd(Ay, 2), cd(Ax, 2) - cd(Az, 0), cd(Ay, 0) - cd(Ax, 1)]
    noise = [0.01 * _seeded((n,) * nd, 90 + d) for d in range(nd)]
    return [B[d] + cd(psi, d) + noise[d] for d in range(nd)]


@pytest.mark.parametrize("nd,n", [(2, 128), (3, 32)])
def test_divb_projection_matches_the_oracle(nd, n):
    torch, M = _mg()
    B = _solenoidal_plus_gradient(nd, n)
    ref, _ = R.divb_project(B, 1.0, R.PERIODIC)
    mg = M.GpuMultigrid(nd, n, M.PERIODIC, 1.0, nfields=1)
    Bt = [torch.tensor(b, device="cuda:0").contiguous() for b in B]
    c, before, after = mg.divb_project(Bt, tol=1e-12, max_cycles=80)
    assert before == np.abs(R.central_div(B, 1.0, R.PERIODIC)).max()  # same arithmetic, bit for bit
    assert after == np.abs(R.central_div([b.cpu().numpy() for b in Bt], 1.0, R.PERIODIC)).max()
    err = max(np.abs(Bt[d].cpu().numpy() - ref[d]).max() for d in range(nd))
    scale = max(np.abs(b).max() for b in B)
    print(f"[mg] divB {nd}D n={n}: {c} cycles, max|div| {before:.3e} -> {after:.3e}, vs oracle {err:.2e}",
          flush=True)
    assert err <= 1e-9 * scale
    assert after < 0.1 * before
    mg.close()


def test_divb_projection_rejects_unsupported_setups():
    torch, M = _mg()
    from paper_2004_03275_amd import _native as N

    B = [torch.zeros(64 * 64, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    for kw in ({"nfields": 2, "bc": M.PERIODIC}, {"nfields": 1, "bc": M.NEUMANN}):
        mg = M.GpuMultigrid(2, 64, kw["bc"], 1.0, nfields=kw["nfields"])
        with pytest.raises(N.AmrvError) as e:
            mg.divb_project(B)
        assert e.value.code == N.EINVAL
        mg.close()


# -- variable coefficient (Sec. 1.4) ------------------------------------------

def _eps_field(nd, n, kind):
    xs = W.rd_cell_centres(nd, n, 1.0)
    if kind == "smooth":
        e = 1.0 + 0.5 * np.cos(2 * np.pi * xs[0]) * np.sin(2 * np.pi * xs[1])
    else:  # a jump of 10x across x = 1/2
        e = np.where(xs[0] < 0.5, 1.0, 10.0)
    return np.ascontiguousarray(e)


@pytest.mark.parametrize("nd,n", [(2, 64), (2, 256), (3, 16), (3, 32)])
@pytest.mark.parametrize("bc", [R.PERIODIC, R.NEUMANN])
@pytest.mark.parametrize("kind", ["smooth", "jump"])
def test_variable_coefficient_solve_within_the_residual_bound(nd, n, bc, kind):
    """div(eps grad phi) - lambda phi = f against the oracle's sparse direct
    solve: still an M-matrix with row sums lambda, so max |phi - exact| <=
    max |r| / lambda."""
    torch, M = _mg()
    lam = 20.0
    f = _seeded((n,) * nd, 60 + n)
    eps = _eps_field(nd, n, kind)
    exact = R.helmholtz_var_solve(f, eps, lam, 1.0, bc)
    mg = M.GpuMultigrid(nd, n, bc, 1.0, nfields=1)
    mg.set_coefficient(torch.tensor(eps.ravel(), device="cuda:0"))
    phi = torch.zeros(f.size, dtype=torch.float64, device="cuda:0")
    c, res, _ = mg.solve(torch.tensor(f.ravel(), device="cuda:0"), phi, lam, tol=1e-11, max_cycles=80)
    err = np.abs(phi.cpu().numpy().reshape(f.shape) - exact).max()
    print(f"[mg] var {kind} {nd}D n={n} bc={bc}: {c} cycles, res {res[0]:.2e}, err {err:.2e}", flush=True)
    assert err <= 2.0 * res[0] / lam + 1e-12 * np.abs(exact).max()
    mg.close()


def test_coefficient_reset_and_rejections():
    torch, M = _mg()
    from paper_2004_03275_amd import _native as N

    n = 64
    f = torch.tensor(_seeded((n, n), 3).ravel(), device="cuda:0")
    ref = M.GpuMultigrid(2, n, R.NEUMANN, 1.0, nfields=1)
    p0 = torch.zeros_like(f)
    ref.solve(f, p0, 4.0, tol=1e-10)
    mg = M.GpuMultigrid(2, n, R.NEUMANN, 1.0, nfields=1)
    mg.set_coefficient(torch.full((n * n,), 2.0, dtype=torch.float64, device="cuda:0"))
    p1 = torch.zeros_like(f)
    with pytest.raises(N.AmrvError) as e:
        mg.solve(f, p1, 0.0)
    assert e.value.code == N.EINVAL
    mg.solve(f, p1, 4.0, tol=1e-10)
    exact2 = R.helmholtz_var_solve(f.cpu().numpy().reshape(n, n), np.full((n, n), 2.0), 4.0, 1.0, R.NEUMANN)
    assert np.abs(p1.cpu().numpy().reshape(n, n) - exact2).max() < 1e-9
    mg.set_coefficient(None)  # back to eps = 1: bit for bit the fresh solver's answer
    p2 = torch.zeros_like(f)
    mg.solve(f, p2, 4.0, tol=1e-10)
    assert torch.equal(p2, p0)
    mg.close()
    ref.close()
    m2 = M.GpuMultigrid(2, n, R.PERIODIC, 1.0, nfields=2)
    m2.set_coefficient(torch.ones(n * n, dtype=torch.float64, device="cuda:0"))
    u = torch.ones(n * n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(N.AmrvError) as e:
        m2.rd_step(u, u.clone(), 1e-3, M.IMEX, R.SCHNAKENBERG_PARAMS)
    assert e.value.code == N.EINVAL
    m2.close()


@pytest.mark.parametrize("nd,sizes", [(2, (64, 256, 1024)), (3, (16, 32, 64, 128))])
def test_cycle_count_does_not_grow_with_the_grid(nd, sizes):
    """Multigrid's defining property: the V-cycles needed for a fixed
    relative residual stay (nearly) constant as the grid is refined, where a
    smoother alone would need O(n^2) sweeps."""
    torch, M = _mg()
    counts = []
    for n in sizes:
        f = _seeded((n,) * nd, 80 + n)
        mg = M.GpuMultigrid(nd, n, R.NEUMANN, 1.0, nfields=1)
        phi = torch.zeros(f.size, dtype=torch.float64, device="cuda:0")
        c, res, fmax = mg.solve(torch.tensor(f.ravel(), device="cuda:0"), phi, 1.0, tol=1e-9, max_cycles=60)
        counts.append(c)
        mg.close()
    print(f"[mg] {nd}D cycles to 1e-9 for n = {sizes}: {counts}", flush=True)
    assert max(counts) - min(counts) <= 3, counts
