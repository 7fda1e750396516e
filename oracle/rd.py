"""CPU reference of the elliptic solve and the reaction-diffusion schemes.

TEST INFRASTRUCTURE ONLY (tests/, smoke, bench's CPU leg).  Written from the
paper's multigrid and reaction-diffusion sections (Sec. 1.4 on multigrid,
Sec. 2.4 on its divergence control of the MHD runs, Sec. 2.5 and 2.5.1: Eqs.
gray-scott, schnakenberg, diff-helmholtz and imex, Table 1), sharing nothing
with the HIP path.

Grid: a uniform cell-centred grid of n cells per side on [0, L]^d (d = 2, 3),
h = L / n, arrays indexed [z][y][x] with x fastest.  Boundaries: periodic, or
zero Neumann (the ghost value beyond a face equals the adjacent interior
cell).

Discrete Laplacian (the standard second-order discretisation the paper
names): per direction ((w_minus + w_plus) - 2 w) * (1/h^2), the directions
added in the order x, y, z, with 1/h^2 formed as (n/L) * (n/L).

Helmholtz problem (Eq. diff-helmholtz): lap(phi) - lambda phi = f, lambda > 0;
Poisson (lambda = 0) for the divergence control of the MHD runs (Sec. 2.4),
whose solution is fixed up to a constant (the zero-mean one here).  With a
variable coefficient (Sec. 1.4): div(eps grad phi) - lambda phi = f, eps > 0
per cell, face coefficients the arithmetic mean of the two cells, solved by
a sparse direct solve; still an M-matrix with row sums lambda.
This module solves it exactly (to rounding): the operator is diagonalised by
the discrete Fourier transform (periodic) or the type-II cosine transform
(Neumann), with eigenvalue sum_d (2 cos(theta_d) - 2) / h^2 - lambda,
theta = 2 pi k / n (periodic) or pi k / n (Neumann).  The GPU solves the same
system iteratively; its maximum residual r bounds the difference:
A = lambda I - lap is an M-matrix whose rows sum to lambda, so
max |phi_gpu - phi_exact| <= max |r| / lambda.

Reaction terms F0 (Eqs. gray-scott and schnakenberg), diffusion F1 = D lap(w):
  Schnakenberg: F0_u = kappa (a - u + u^2 v), F0_v = kappa (b - u^2 v)
  Gray-Scott:   F0_u = -u v^2 + F (1 - u),   F0_v = u v^2 - (F + k) v

Time schemes on (u, v), each species with its own D:
  EULER     w1 = w + dt (F0(w) + F1(w))
  MIDPOINT  wh = w + (dt/2) (F0(w) + F1(w)); w1 = w + dt (F0(wh) + F1(wh))
  SPLIT     w* = w + dt F0(w) (explicit Euler on the reaction), then the
            backward-Euler diffusion step w1 = w* + dt F1(w1): Helmholtz with
            lambda = 1/(dt D), f = -lambda w*
  IMEX      the trapezoidal pair of Eq. imex: w* from
            w* - (dt/2) F1(w*) = w + dt F0(w) + (dt/2) F1(w), i.e. Helmholtz
            with lambda = 2/(dt D), f = -lambda (w + dt F0(w) + (dt/2) F1(w));
            then w1 = w + (dt/2) (F(w) + F(w*)), F = F0 + F1, F1(w*) by the
            stencil.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

PERIODIC, NEUMANN = 0, 1
SCHNAKENBERG, GRAY_SCOTT = 0, 1
EULER, MIDPOINT, SPLIT, IMEX = 0, 1, 2, 3

# Sec. 2.5: Schnakenberg parameters (Du, Dv, kappa, a, b) and Gray-Scott
# (Du, Dv, F, k)
SCHNAKENBERG_PARAMS = dict(model=SCHNAKENBERG, Du=0.05, Dv=1.0, p1=100.0, p2=0.1305, p3=0.7695)
GRAY_SCOTT_PARAMS = dict(model=GRAY_SCOTT, Du=2e-5, Dv=1e-5, p1=0.046, p2=0.063, p3=0.0)


def inv_h2(n: int, length: float) -> float:
    r = n / length
    return r * r


def _shift(w, axis, step, bc):
    """w at the neighbour in +step (step = +-1) along axis, with the boundary
    rule: periodic wrap, or the mirrored interior cell (Neumann)."""
    if bc == PERIODIC:
        return np.roll(w, -step, axis=axis)
    n = w.shape[axis]
    idx = np.clip(np.arange(n) + step, 0, n - 1)
    return np.take(w, idx, axis=axis)


def laplacian(w, length: float, bc: int):
    """Second-order Laplacian of a [z][y][x] (or [y][x]) array."""
    nd = w.ndim
    ih2 = inv_h2(w.shape[-1], length)
    out = None
    for d in range(nd):  # x, y, z
        ax = nd - 1 - d
        term = ((_shift(w, ax, -1, bc) + _shift(w, ax, +1, bc)) - 2.0 * w) * ih2
        out = term if out is None else out + term
    return out


def helmholtz_apply(phi, lam: float, length: float, bc: int):
    """lap(phi) - lambda phi."""
    return laplacian(phi, length, bc) - lam * phi


def _eigenvalues(shape, length: float, bc: int, lam: float):
    n = shape[-1]
    ih2 = inv_h2(n, length)
    k = np.arange(n)
    theta = (2.0 * np.pi * k / n) if bc == PERIODIC else (np.pi * k / n)
    mu1 = (2.0 * np.cos(theta) - 2.0) * ih2
    mu = -lam * np.ones(shape)
    nd = len(shape)
    for d in range(nd):
        sh = [1] * nd
        sh[nd - 1 - d] = n
        mu = mu + mu1.reshape(sh)
    return mu


def helmholtz_solve(f, lam: float, length: float, bc: int):
    """Exact solution of lap(phi) - lambda phi = f (lambda > 0)."""
    if not lam > 0.0:
        raise ValueError("lambda must be positive")
    mu = _eigenvalues(f.shape, length, bc, lam)
    if bc == PERIODIC:
        return np.real(np.fft.ifftn(np.fft.fftn(f) / mu))
    return sfft.idctn(sfft.dctn(f, type=2, norm="ortho") / mu, type=2, norm="ortho")


def _face_sums(phi, eps, length: float, bc: int):
    """sum_d (e+ (phi+ - phi) - e- (phi - phi-)) / h^2 with face coefficients
    e+- the arithmetic means of the two cells' eps (a face beyond a Neumann
    boundary mirrors the cell, so its difference vanishes)."""
    nd = phi.ndim
    ih2 = inv_h2(phi.shape[-1], length)
    out = None
    for d in range(nd):
        ax = nd - 1 - d
        ep = 0.5 * (eps + _shift(eps, ax, +1, bc))
        em = 0.5 * (eps + _shift(eps, ax, -1, bc))
        term = (ep * (_shift(phi, ax, +1, bc) - phi) - em * (phi - _shift(phi, ax, -1, bc))) * ih2
        out = term if out is None else out + term
    return out


def helmholtz_var_apply(phi, eps, lam: float, length: float, bc: int):
    """div(eps grad phi) - lambda phi, the variable-coefficient Helmholtz
    operator of the multigrid (Sec. 1.4)."""
    return _face_sums(phi, eps, length, bc) - lam * phi


def helmholtz_var_matrix(eps, lam: float, length: float, bc: int):
    """The operator as a sparse matrix on the flattened [z][y][x] grid,
    assembled column by column from unit vectors' stencil neighbourhoods."""
    import scipy.sparse as sp

    shape = eps.shape
    N = eps.size
    nd = eps.ndim
    n = shape[-1]
    ih2 = inv_h2(n, length)
    idx = np.arange(N).reshape(shape)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [-lam * np.ones(N)]
    for d in range(nd):
        ax = nd - 1 - d
        for step in (+1, -1):
            nb_idx = _shift(idx, ax, step, bc)
            e = 0.5 * (eps + _shift(eps, ax, step, bc)) * ih2
            same = nb_idx == idx  # a Neumann face: the mirrored difference is zero
            e = np.where(same, 0.0, e)
            rows += [idx.ravel(), idx.ravel()]
            cols += [nb_idx.ravel(), idx.ravel()]
            vals += [e.ravel(), -e.ravel()]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def helmholtz_var_solve(f, eps, lam: float, length: float, bc: int):
    """Solution of div(eps grad phi) - lambda phi = f, lambda > 0, eps > 0:
    a sparse direct solve up to 20,000 unknowns; beyond, conjugate gradients
    on the symmetric positive definite -A to a relative residual of 1e-14
    (its error is then at most that residual / lambda, the M-matrix bound)."""
    import scipy.sparse.linalg as spl

    if not lam > 0.0:
        raise ValueError("lambda must be positive")
    A = helmholtz_var_matrix(eps, lam, length, bc)
    if f.size <= 20000:
        return spl.spsolve(A.tocsc(), f.ravel()).reshape(f.shape)
    x, info = spl.cg(-A, -f.ravel(), rtol=1e-14, atol=0.0, maxiter=20000)
    if info != 0:
        raise RuntimeError("conjugate gradients did not converge")
    return x.reshape(f.shape)


def poisson_solve(f, length: float, bc: int):
    """The zero-mean solution of lap(phi) = f - mean(f) (periodic or Neumann
    faces, where lap is singular: constants are its null space and a right-
    hand side is admissible when it sums to zero; the mean is the part no
    phi can produce)."""
    mu = _eigenvalues(f.shape, length, bc, 0.0)
    mu.flat[0] = 1.0  # the constant mode: dropped below
    if bc == PERIODIC:
        hat = np.fft.fftn(f)
        hat.flat[0] = 0.0
        return np.real(np.fft.ifftn(hat / mu))
    hat = sfft.dctn(f, type=2, norm="ortho")
    hat.flat[0] = 0.0
    return sfft.idctn(hat / mu, type=2, norm="ortho")


def central_diff(w, d: int, length: float, bc: int):
    """(w(+1) - w(-1)) * (n / (2L)) along direction d (0 = x)."""
    n = w.shape[-1]
    ax = w.ndim - 1 - d
    return (_shift(w, ax, +1, bc) - _shift(w, ax, -1, bc)) * (0.5 * n / length)


def central_div(B, length: float, bc: int):
    """sum_d of the central differences of B[d], added x, y, z."""
    out = central_diff(B[0], 0, length, bc)
    for d in range(1, len(B)):
        out = out + central_diff(B[d], d, length, bc)
    return out


def divb_project(B, length: float, bc: int):
    """The multigrid divergence control of the MHD runs (Sec. 2.4): solve
    lap(phi) = div B* and set B = B* - grad phi (central differences for div
    and grad, the 5/7-point Laplacian for lap: an approximate projection,
    which removes the divergence up to the difference between lap and
    div(grad)).  Returns (B, phi)."""
    phi = poisson_solve(central_div(B, length, bc), length, bc)
    return [B[d] - central_diff(phi, d, length, bc) for d in range(len(B))], phi


def reaction(u, v, p: dict):
    """(F0_u, F0_v) of Eqs. schnakenberg / gray-scott."""
    if p["model"] == SCHNAKENBERG:
        kappa, a, b = p["p1"], p["p2"], p["p3"]
        uuv = (u * u) * v
        return kappa * ((a - u) + uuv), kappa * (b - uuv)
    F, k = p["p1"], p["p2"]
    uvv = u * (v * v)
    return F * (1.0 - u) - uvv, uvv - (F + k) * v


def rhs_full(u, v, p: dict, length: float, bc: int):
    """F = F0 + F1 for both species."""
    ru, rv = reaction(u, v, p)
    return ru + p["Du"] * laplacian(u, length, bc), rv + p["Dv"] * laplacian(v, length, bc)


def step(u, v, dt: float, scheme: int, p: dict, length: float, bc: int):
    """One time step of the given scheme; returns (u1, v1)."""
    if scheme == EULER:
        fu, fv = rhs_full(u, v, p, length, bc)
        return u + dt * fu, v + dt * fv
    if scheme == MIDPOINT:
        fu, fv = rhs_full(u, v, p, length, bc)
        uh, vh = u + (0.5 * dt) * fu, v + (0.5 * dt) * fv
        gu, gv = rhs_full(uh, vh, p, length, bc)
        return u + dt * gu, v + dt * gv
    ru, rv = reaction(u, v, p)
    if scheme == SPLIT:
        out = []
        for w, r, D in ((u, ru, p["Du"]), (v, rv, p["Dv"])):
            lam = 1.0 / (dt * D)
            out.append(helmholtz_solve(-lam * (w + dt * r), lam, length, bc))
        return out[0], out[1]
    if scheme == IMEX:
        star = []
        for w, r, D in ((u, ru, p["Du"]), (v, rv, p["Dv"])):
            lam = 2.0 / (dt * D)
            rhs = w + dt * r + (0.5 * dt) * (D * laplacian(w, length, bc))
            star.append(helmholtz_solve(-lam * rhs, lam, length, bc))
        fu, fv = rhs_full(u, v, p, length, bc)
        su, sv = rhs_full(star[0], star[1], p, length, bc)
        return u + (0.5 * dt) * (fu + su), v + (0.5 * dt) * (fv + sv)
    raise ValueError(f"unknown scheme {scheme}")


def run(u, v, dt: float, nsteps: int, scheme: int, p: dict, length: float, bc: int):
    for _ in range(nsteps):
        u, v = step(u, v, dt, scheme, p, length, bc)
    return u, v


def explicit_dt_limit(h: float, ndim: int, d_max: float) -> float:
    """Stability bound of explicit diffusion (Sec. 2.5.1, Table 1): h^2 / (2 N_dim D_max)."""
    return h * h / (2.0 * ndim * d_max)
