"""The Helmholtz solver on a 2D block-adaptive forest (amrv_fmg_*, Sec. 1.4)
against the oracle's exact composite solve (oracle/fmg.py, sparse LU).

The V-cycles stop at max residual <= tol max |f|; the solution is compared
with the oracle's element by element at 1e-8 of max |u| (the GPU's iterate
differs from the exact discrete solution by the inverse operator applied to
that residual)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fmg

pytestmark = pytest.mark.gpu


def _mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_03275_amd import multigrid as MG

    return MG


def _rhs(f, seed=3):
    x, y = fmg.cell_centres(f, 1.0)
    noise = W.uniform01(seed, f.n * 256).reshape(f.n, 16, 16)
    return np.exp(-40 * ((x - 0.3) ** 2 + (y - 0.6) ** 2)) - 0.5 * np.cos(2 * np.pi * x) + 0.1 * noise


CASES = [
    # base, max_level, bc, centre, radius
    (4, 3, fmg.PERIODIC, (0.27, 0.3), 0.15),
    (4, 3, fmg.NEUMANN, (0.27, 0.3), 0.15),
    (2, 4, fmg.PERIODIC, (0.5, 0.45), 0.2),
    (1, 3, fmg.NEUMANN, (0.1, 0.9), 0.12),
    (8, 4, fmg.NEUMANN, (0.6, 0.4), 0.21),
]


@pytest.mark.parametrize("lam", [10.0, 1.0e5])
@pytest.mark.parametrize("base,max_level,bc,centre,radius", CASES)
def test_forest_solve_matches_oracle(base, max_level, bc, centre, radius, lam):
    MG = _mg()
    f = W.fmg_forest(W.fmg_scheme(base=base, max_level=max_level, bc=bc), centre=centre, radius=radius)
    rhs = _rhs(f)
    ref = fmg.solve(f, rhs, lam, 1.0, bc)
    s = MG.GpuForestMultigrid(f, 1.0, bc)
    print(f"forest {f.level_counts()} bc {bc} lambda {lam} blocks/level {s.levels()}", flush=True)
    F = torch.tensor(rhs, device="cuda:0")
    U = torch.zeros_like(F)
    cyc, res, fmax = s.solve(F, U, lam, tol=1e-10, max_cycles=40)
    u = U.cpu().numpy()
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    print(f"  cycles {cyc} residual {res / fmax:.2e} of max|f|, max error {err:.2e} of max|u|", flush=True)
    assert res <= 1e-10 * fmax
    assert cyc <= 20
    assert err <= 1e-8
    s.close()


def test_uniform_forest_and_repeated_solves():
    """Every leaf at level 2 (the composite problem is the plain 64^2 grid
    problem); the same handle then solves again with another lambda and f,
    and from the solution as its initial guess (no cycle needed)."""
    MG = _mg()
    f = W.uniform_forest(W.fmg_scheme(base=4, max_level=2, bc=fmg.PERIODIC), level=2)
    s = MG.GpuForestMultigrid(f, 1.0, fmg.PERIODIC)
    for lam, seed in ((3.0, 1), (250.0, 2)):
        rhs = _rhs(f, seed)
        ref = fmg.solve(f, rhs, lam, 1.0, fmg.PERIODIC)
        F = torch.tensor(rhs, device="cuda:0")
        U = torch.zeros_like(F)
        cyc, res, fmax = s.solve(F, U, lam, tol=1e-10)
        assert np.max(np.abs(U.cpu().numpy() - ref)) <= 1e-8 * np.max(np.abs(ref))
        cyc2, res2, _ = s.solve(F, U, lam, tol=1e-10)
        assert cyc2 == 0 and res2 <= 1e-10 * fmax
    s.close()


def test_bad_lambda_is_rejected():
    MG = _mg()
    from paper_2004_03275_amd import _native as N

    f = W.fmg_forest(W.fmg_scheme(base=4, max_level=3, bc=fmg.PERIODIC), centre=(0.27, 0.3), radius=0.15)
    s = MG.GpuForestMultigrid(f, 1.0, fmg.PERIODIC)
    F = torch.zeros((f.n, 16, 16), dtype=torch.float64, device="cuda:0")
    with pytest.raises(N.AmrvError):
        s.solve(F, F.clone(), 0.0)
    s.close()


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_forest_rd_step_matches_oracle(scheme):
    """Two Gray-Scott steps (Sec. 2.5.2 parameters and initial spots, periodic
    side 2) on a three-level forest refined around the spots: explicit Euler
    and midpoint (the paper's AMR run), split and IMEX through the forest
    solver, against the oracle's steps with the exact composite solves."""
    MG = _mg()
    from oracle import rd

    s = W.fmg_scheme(base=4, max_level=3, bc=fmg.PERIODIC, length=2.0)
    f = W.fmg_forest(s, centre=(0.26, 0.28), radius=0.1)
    x, y = fmg.cell_centres(f, 2.0)
    g = sum(0.5 * np.exp(-25.0 * ((x - cx) ** 2 + (y - cy) ** 2)) for cx, cy in ((0.5, 0.5), (0.55, 0.6)))
    u, v = 1.0 - g, g.copy()
    p = rd.GRAY_SCOTT_PARAMS
    dt = 0.5 if scheme in (rd.SPLIT, rd.IMEX) else 0.05
    ru, rv = u, v
    for _ in range(2):
        ru, rv = fmg.rd_step(f, ru, rv, dt, scheme, p, 2.0, fmg.PERIODIC)
    solver = MG.GpuForestMultigrid(f, 2.0, fmg.PERIODIC)
    U = torch.tensor(u, device="cuda:0")
    V = torch.tensor(v, device="cuda:0")
    cyc, res = solver.rd_step(U, V, dt, scheme, p, nsteps=2, tol=1e-11)
    print(f"forest {f.level_counts()} scheme {scheme} cycles {cyc}", flush=True)
    for a, b in ((U.cpu().numpy(), ru), (V.cpu().numpy(), rv)):
        assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(b))
    solver.close()
