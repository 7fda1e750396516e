"""CPU reference of the Helmholtz problem on a 2D block-adaptive forest.

TEST INFRASTRUCTURE ONLY (tests/, smoke, bench's CPU leg).  Written from the
paper's multigrid section (Sec. 1.4: a geometric multigrid on the block-
adaptive quadtree grid for Poisson and Helmholtz problems, used by the
reaction-diffusion schemes of Sec. 2.5 and the divergence control of
Sec. 2.4), sharing nothing with the HIP path.

Grid: the leaves of a 2:1-balanced quadtree forest (workloads.Forest) on the
square [0, L]^2, b x b base blocks at level 1, NB x NB cells per block, level
l cells of width h_l = L / (b NB 2^(l-1)).  A field is one value per leaf
cell, laid out [leaf][y][x] (x fastest), as the forest's state variables.

The discrete problem on the leaf cells: lap(u) - lambda u = f, lambda > 0,
lap of a cell the 5-point sum (u_W + u_E + u_S + u_N - 4 u) / h_l^2 at the
cell's own level.  The value across a face comes from:
  (1) a leaf cell at the same level: its unknown;
  (2) the zero-Neumann mirror (the cell itself) at a non-periodic domain
      face; periodic faces wrap;
  (3) a coarser leaf (the fine side of a coarse-fine face): with u_c the
      coarse cell across the face, moved a quarter coarse cell along the face
      toward the fine cell with the coarse block's own tangential difference
      (central, one-sided at the block's edges), the value is
      (u + 2 u_c) / 3 -- linear along the normal between the fine cell's
      centre and the coarse cell's, at the ghost's centre;
  (4) a refined block (the coarse side): the face's flux is the mean of the
      two fine fluxes through it, each from rule (3); the offsets of (3)
      cancel in the mean, which leaves the value u + (4/3) (m - u), m the
      mean of the two fine cells that touch the face.
Rules (3) and (4) are a reading: the paper defers the coarse-fine stencils
to its multigrid library.  With (4) the scheme is conservative (the cell
sums of lap(u) times cell area cancel for every u on a periodic or Neumann
domain) and second order; every rule reproduces constants and linear
functions, so lap of a linear function is zero at every cell off the domain
boundary.

The system is assembled as a sparse matrix and solved directly (sparse LU):
the exact discrete solution the GPU's V-cycles converge to.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PERIODIC, NEUMANN = 0, 1


class ForestGrid:
    """Leaf and block bookkeeping of a 2D forest (levels 1-based)."""

    def __init__(self, level, ijk, base: int, nb: int, length: float, bc: int):
        self.level = np.asarray(level, dtype=np.int64)
        self.ij = np.asarray(ijk, dtype=np.int64)[:, :2]
        self.base, self.nb, self.length, self.bc = int(base), int(nb), float(length), int(bc)
        self.leaf = {(int(l), int(i), int(j)): k for k, (l, (i, j)) in enumerate(zip(self.level, self.ij))}
        blocks = set(self.leaf)
        for (l, i, j) in list(self.leaf):
            while l > 1:
                l, i, j = l - 1, i >> 1, j >> 1
                blocks.add((l, i, j))
        self.blocks = blocks
        self.ncell = len(self.leaf) * nb * nb

    def cells_per_side(self, l: int) -> int:
        return self.base * self.nb << (l - 1)

    def index(self, k: int, x: int, y: int) -> int:
        return (k * self.nb + y) * self.nb + x

    def neighbour(self, k: int, x: int, y: int, dx: int, dy: int) -> dict:
        """{unknown: weight} of the value across the face (dx, dy) of leaf k's
        cell (x, y)."""
        l = int(self.level[k])
        n = self.cells_per_side(l)
        gx = int(self.ij[k, 0]) * self.nb + x
        gy = int(self.ij[k, 1]) * self.nb + y
        ngx, ngy = gx + dx, gy + dy
        if not (0 <= ngx < n and 0 <= ngy < n):
            if self.bc == NEUMANN:
                return {self.index(k, x, y): 1.0}
            ngx %= n
            ngy %= n
        key = (l, ngx // self.nb, ngy // self.nb)
        if key in self.leaf:  # rule (1)
            return {self.index(self.leaf[key], ngx % self.nb, ngy % self.nb): 1.0}
        if key in self.blocks:  # rule (4): the two fine leaf cells that touch the face
            out = {self.index(k, x, y): -1.0 / 3.0}
            for t in (0, 1):
                if dx != 0:
                    fx, fy = 2 * ngx + (1 if dx < 0 else 0), 2 * ngy + t
                else:
                    fx, fy = 2 * ngx + t, 2 * ngy + (1 if dy < 0 else 0)
                fk = self.leaf[(l + 1, fx // self.nb, fy // self.nb)]
                q = self.index(fk, fx % self.nb, fy % self.nb)
                out[q] = out.get(q, 0.0) + 2.0 / 3.0
            return out
        # rule (3): the coarse leaf across the face
        cx, cy = ngx >> 1, ngy >> 1
        ck = self.leaf[(l - 1, cx // self.nb, cy // self.nb)]
        X, Y = cx % self.nb, cy % self.nb
        if dx != 0:  # tangential direction y
            t, o = Y, (0.25 if gy & 1 else -0.25)
            at = lambda s: self.index(ck, X, s)  # noqa: E731
        else:
            t, o = X, (0.25 if gx & 1 else -0.25)
            at = lambda s: self.index(ck, s, Y)  # noqa: E731
        uc = {at(t): 1.0}
        if t == 0:
            slope = {at(1): 1.0, at(0): -1.0}
        elif t == self.nb - 1:
            slope = {at(t): 1.0, at(t - 1): -1.0}
        else:
            slope = {at(t + 1): 0.5, at(t - 1): -0.5}
        for q, w in slope.items():
            uc[q] = uc.get(q, 0.0) + o * w
        out = {self.index(k, x, y): 1.0 / 3.0}
        for q, w in uc.items():
            out[q] = out.get(q, 0.0) + 2.0 / 3.0 * w
        return out


def grid(forest, length: float, bc: int) -> ForestGrid:
    s = forest.scheme
    if s.ndim != 2 or s.base_blocks[0] != s.base_blocks[1] or s.block_nx[0] != s.block_nx[1]:
        raise ValueError("a 2D forest of square blocks on a square base grid")
    return ForestGrid(forest.level, forest.ijk, s.base_blocks[0], s.block_nx[0], length, bc)


def matrix(g: ForestGrid, lam: float) -> sp.csr_matrix:
    """The operator lap - lambda I on the leaf cells."""
    rows, cols, vals = [], [], []
    nb = g.nb
    for k in range(len(g.level)):
        l = int(g.level[k])
        ih2 = (g.cells_per_side(l) / g.length) * (g.cells_per_side(l) / g.length)
        for y in range(nb):
            for x in range(nb):
                r = g.index(k, x, y)
                acc = {r: -4.0 * ih2 - lam}
                for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                    if 0 <= x + dx < nb and 0 <= y + dy < nb:
                        nbr = {g.index(k, x + dx, y + dy): 1.0}
                    else:
                        nbr = g.neighbour(k, x, y, dx, dy)
                    for q, w in nbr.items():
                        acc[q] = acc.get(q, 0.0) + w * ih2
                for q, w in acc.items():
                    rows.append(r)
                    cols.append(q)
                    vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.ncell, g.ncell))


def apply(forest, u: np.ndarray, lam: float, length: float, bc: int) -> np.ndarray:
    """lap(u) - lambda u on the leaf cells (u, result: [leaf][y][x])."""
    g = grid(forest, length, bc)
    return (matrix(g, lam) @ np.asarray(u, dtype=np.float64).reshape(-1)).reshape(np.shape(u))


def solve(forest, f: np.ndarray, lam: float, length: float, bc: int) -> np.ndarray:
    """The exact discrete solution of lap(u) - lambda u = f (lambda > 0)."""
    if not lam > 0.0:
        raise ValueError("lambda > 0")
    g = grid(forest, length, bc)
    A = matrix(g, lam).tocsc()
    u = spla.spsolve(A, np.asarray(f, dtype=np.float64).reshape(-1))
    return u.reshape(np.shape(f))


def cell_centres(forest, length: float):
    """x, y of every leaf cell ([leaf][y][x]) on [0, L]^2."""
    s = forest.scheme
    nb = s.block_nx[0]
    n = (s.base_blocks[0] << (forest.level.astype(np.int64) - 1)) * nb
    h = length / n
    loc = np.arange(nb, dtype=np.float64)
    x = (forest.ijk[:, 0, None, None] * nb + loc[None, None, :] + 0.5) * h[:, None, None]
    y = (forest.ijk[:, 1, None, None] * nb + loc[None, :, None] + 0.5) * h[:, None, None]
    return np.broadcast_to(x, (forest.n, nb, nb)).copy(), np.broadcast_to(y, (forest.n, nb, nb)).copy()


# -- reaction-diffusion on the forest (Sec. 2.5: Eqs. gray-scott, schnakenberg,
# diff-helmholtz and imex; the schemes as oracle/rd.py writes them on a
# uniform grid, with this module's lap and solve) ----------------------------

def rd_step(forest, u, v, dt: float, scheme: int, p: dict, length: float, bc: int):
    """One step of a reaction-diffusion scheme on the leaf cells ([leaf][y][x]
    fields); scheme and parameters as in oracle/rd.py.  Returns (u1, v1)."""
    from . import rd

    def lap(w):
        return apply(forest, w, 0.0, length, bc)

    def full(a, b):
        ra, rb = rd.reaction(a, b, p)
        return ra + p["Du"] * lap(a), rb + p["Dv"] * lap(b)

    if scheme == rd.EULER:
        fu, fv = full(u, v)
        return u + dt * fu, v + dt * fv
    if scheme == rd.MIDPOINT:
        fu, fv = full(u, v)
        uh, vh = u + (0.5 * dt) * fu, v + (0.5 * dt) * fv
        gu, gv = full(uh, vh)
        return u + dt * gu, v + dt * gv
    ru, rv = rd.reaction(u, v, p)
    if scheme == rd.SPLIT:
        out = []
        for w, r, D in ((u, ru, p["Du"]), (v, rv, p["Dv"])):
            lam = 1.0 / (dt * D)
            out.append(solve(forest, -lam * (w + dt * r), lam, length, bc))
        return out[0], out[1]
    if scheme == rd.IMEX:
        star = []
        for w, r, D in ((u, ru, p["Du"]), (v, rv, p["Dv"])):
            lam = 2.0 / (dt * D)
            star.append(solve(forest, -lam * (w + dt * r + (0.5 * dt) * (D * lap(w))), lam, length, bc))
        fu, fv = full(u, v)
        su, sv = full(star[0], star[1])
        return u + (0.5 * dt) * (fu + su), v + (0.5 * dt) * (fv + sv)
    raise ValueError(f"unknown scheme {scheme}")


# -- Poisson and the divergence control on the forest (Sec. 2.4: solve
# lap(phi) = div B*, set B = B* - grad phi; Sec. 1.4: the multigrid on the
# block-adaptive grid) ---------------------------------------------------------

def _value(g: ForestGrid, k: int, x: int, y: int, dx: int, dy: int) -> dict:
    """{unknown: weight} of the value one cell over from leaf k's cell (x, y):
    the cell itself inside the block, else the ghost rules (1)-(4), each of
    which interpolates linear data exactly."""
    if 0 <= x + dx < g.nb and 0 <= y + dy < g.nb:
        return {g.index(k, x + dx, y + dy): 1.0}
    return g.neighbour(k, x, y, dx, dy)


def diff_matrix(g: ForestGrid, d: int) -> sp.csr_matrix:
    """Central difference along d (0 = x): (w(+1) - w(-1)) * (n_l / (2L))."""
    rows, cols, vals = [], [], []
    dx, dy = (1, 0) if d == 0 else (0, 1)
    for k in range(len(g.level)):
        s = 0.5 * g.cells_per_side(int(g.level[k])) / g.length
        for y in range(g.nb):
            for x in range(g.nb):
                r = g.index(k, x, y)
                acc: dict = {}
                for sgn in (1, -1):
                    for q, w in _value(g, k, x, y, sgn * dx, sgn * dy).items():
                        acc[q] = acc.get(q, 0.0) + sgn * w
                for q, w in acc.items():
                    rows.append(r)
                    cols.append(q)
                    vals.append(w * s)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.ncell, g.ncell))


def cell_areas(forest, length: float) -> np.ndarray:
    """Area of every leaf cell, [leaf][y][x]."""
    s = forest.scheme
    n = (s.base_blocks[0] << (forest.level.astype(np.int64) - 1)) * s.block_nx[0]
    a = (length / n) ** 2
    return np.broadcast_to(a[:, None, None], (forest.n, s.block_nx[0], s.block_nx[0])).copy()


def divergence(forest, bx, by, length: float, bc: int) -> np.ndarray:
    """Central-difference divergence at the leaf cells (x, then y)."""
    g = grid(forest, length, bc)
    shp = np.shape(bx)
    return ((diff_matrix(g, 0) @ np.ravel(bx)) + (diff_matrix(g, 1) @ np.ravel(by))).reshape(shp)


def gradient(forest, phi, length: float, bc: int):
    g = grid(forest, length, bc)
    shp = np.shape(phi)
    return (diff_matrix(g, 0) @ np.ravel(phi)).reshape(shp), (diff_matrix(g, 1) @ np.ravel(phi)).reshape(shp)


def poisson(forest, f, length: float, bc: int) -> np.ndarray:
    """The zero-mean (area-weighted) solution of lap(phi) = f - mean(f), mean
    area-weighted: lap is singular on a periodic or Neumann domain (constants
    are its null space, and the area-weighted sum of lap(phi) vanishes), so
    the bordered system [[lap, 1], [area^T, 0]] [phi; c] = [f; 0] is solved,
    whose c is the area-weighted mean of f."""
    g = grid(forest, length, bc)
    A = matrix(g, 0.0)
    a = cell_areas(forest, length).ravel()
    n = g.ncell
    M = sp.bmat([[A, sp.csr_matrix(np.ones((n, 1)))], [sp.csr_matrix(a.reshape(1, n)), None]]).tocsc()
    sol = spla.spsolve(M, np.concatenate([np.ravel(f), [0.0]]))
    return sol[:n].reshape(np.shape(f))


def divb_project(forest, bx, by, length: float, bc: int):
    """The divergence control of Sec. 2.4 on the leaf cells: phi = the
    zero-mean solution of lap(phi) = div B*, B = B* - grad phi (central
    differences for div and grad, the 5-point composite lap: an approximate
    projection).  Returns (bx, by, phi)."""
    phi = poisson(forest, divergence(forest, bx, by, length, bc), length, bc)
    gx, gy = gradient(forest, phi, length, bc)
    return bx - gx, by - gy, phi
