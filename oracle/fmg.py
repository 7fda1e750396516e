"""CPU reference of the Helmholtz problem on a 2D or 3D block-adaptive forest.

TEST INFRASTRUCTURE ONLY (tests/, smoke, bench's CPU leg).  Written from the
paper's multigrid section (Sec. 1.4: a geometric multigrid on the block-
adaptive quadtree grid for Poisson and Helmholtz problems, used by the
reaction-diffusion schemes of Sec. 2.5 and the divergence control of
Sec. 2.4), sharing nothing with the HIP path.

Grid: the leaves of a 2:1-balanced quadtree or octree forest
(workloads.Forest) on the square or cube [0, L]^d, b^d base blocks at level
1, NB^d cells per block, level l cells of width h_l = L / (b NB 2^(l-1)).  A
field is one value per leaf cell, laid out [leaf][(z)][y][x] (x fastest), as
the forest's state variables.

The discrete problem on the leaf cells: lap(u) - lambda u = f, lambda > 0,
lap of a cell the (2d+1)-point sum (sum of the 2d values across its faces -
2d u) / h_l^2 at the cell's own level.  The value across a face comes from:
  (1) a leaf cell at the same level: its unknown;
  (2) the zero-Neumann mirror (the cell itself) at a non-periodic domain
      face; periodic faces wrap;
  (3) a coarser leaf (the fine side of a coarse-fine face): with u_c the
      coarse cell across the face, moved a quarter coarse cell along the face
      toward the fine cell in each tangential direction with the coarse
      block's own difference there (central, one-sided at the block's
      edges), the value is (u + 2 u_c) / 3 -- linear along the normal
      between the fine cell's centre and the coarse cell's, at the ghost's
      centre;
  (4) a refined block (the coarse side): the face's flux is the mean of the
      2^(d-1) fine fluxes through it, each from rule (3); the offsets of (3)
      cancel in the mean, which leaves the value u + (4/3) (m - u), m the
      mean of the fine cells that touch the face.
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
    """Leaf and block bookkeeping of a 2D or 3D forest (levels 1-based); a
    cell is addressed by its leaf and its local coordinates (x, y[, z])."""

    def __init__(self, level, ijk, base: int, nb: int, length: float, bc: int, ndim: int = 2):
        self.nd = int(ndim)
        self.level = np.asarray(level, dtype=np.int64)
        self.ij = np.asarray(ijk, dtype=np.int64)[:, : self.nd]
        self.base, self.nb, self.length, self.bc = int(base), int(nb), float(length), int(bc)
        self.leaf = {(int(l),) + tuple(int(v) for v in c): k for k, (l, c) in enumerate(zip(self.level, self.ij))}
        blocks = set(self.leaf)
        for key in list(self.leaf):
            l, c = key[0], key[1:]
            while l > 1:
                l, c = l - 1, tuple(v >> 1 for v in c)
                blocks.add((l,) + c)
        self.blocks = blocks
        self.ncell = len(self.leaf) * nb ** self.nd

    def cells_per_side(self, l: int) -> int:
        return self.base * self.nb << (l - 1)

    def index(self, k: int, c) -> int:
        i = k
        for v in reversed(c):
            i = i * self.nb + v
        return i

    def neighbour(self, k: int, c, d: int, sgn: int) -> dict:
        """{unknown: weight} of the value across the face of leaf k's cell c
        in direction d (0 = x), side sgn (+1 or -1)."""
        nb, nd = self.nb, self.nd
        l = int(self.level[k])
        n = self.cells_per_side(l)
        g = [int(self.ij[k, e]) * nb + c[e] for e in range(nd)]
        ng = list(g)
        ng[d] += sgn
        if not 0 <= ng[d] < n:
            if self.bc == NEUMANN:
                return {self.index(k, c): 1.0}
            ng[d] %= n
        key = (l,) + tuple(v // nb for v in ng)
        if key in self.leaf:  # rule (1)
            return {self.index(self.leaf[key], tuple(v % nb for v in ng)): 1.0}
        if key in self.blocks:  # rule (4): the 2^(nd-1) fine leaf cells that touch the face
            out = {self.index(k, c): -1.0 / 3.0}
            w = (4.0 / 3.0) / 2 ** (nd - 1)
            others = [e for e in range(nd) if e != d]
            for t in range(2 ** (nd - 1)):
                fc = [0] * nd
                fc[d] = 2 * ng[d] + (1 if sgn < 0 else 0)
                for bit, e in enumerate(others):
                    fc[e] = 2 * ng[e] + ((t >> bit) & 1)
                fk = self.leaf[(l + 1,) + tuple(v // nb for v in fc)]
                q = self.index(fk, tuple(v % nb for v in fc))
                out[q] = out.get(q, 0.0) + w
            return out
        # rule (3): the coarse leaf across the face, its cell moved a quarter
        # cell toward the fine cell along each tangential direction
        cc = [v >> 1 for v in ng]
        ck = self.leaf[(l - 1,) + tuple(v // nb for v in cc)]
        C = [v % nb for v in cc]
        uc = {self.index(ck, tuple(C)): 1.0}
        for e in range(nd):
            if e == d:
                continue
            o = 0.25 if g[e] & 1 else -0.25
            t = C[e]

            def at(sv, e=e):
                cv = list(C)
                cv[e] = sv
                return self.index(ck, tuple(cv))

            if t == 0:
                slope = {at(1): 1.0, at(0): -1.0}
            elif t == nb - 1:
                slope = {at(t): 1.0, at(t - 1): -1.0}
            else:
                slope = {at(t + 1): 0.5, at(t - 1): -0.5}
            for q, wv in slope.items():
                uc[q] = uc.get(q, 0.0) + o * wv
        out = {self.index(k, c): 1.0 / 3.0}
        for q, wv in uc.items():
            out[q] = out.get(q, 0.0) + 2.0 / 3.0 * wv
        return out

    def cells(self):
        """Local coordinates (x, y[, z]) of a block's cells in storage order."""
        for r in np.ndindex(*([self.nb] * self.nd)):
            yield tuple(reversed(r))


def grid(forest, length: float, bc: int) -> ForestGrid:
    s = forest.scheme
    nd = s.ndim
    if nd not in (2, 3) or len(set(s.base_blocks[:nd])) != 1 or len(set(s.block_nx[:nd])) != 1:
        raise ValueError("a 2D or 3D forest of square / cubic blocks on a square / cubic base grid")
    return ForestGrid(forest.level, forest.ijk, s.base_blocks[0], s.block_nx[0], length, bc, nd)


def matrix(g: ForestGrid, lam: float) -> sp.csr_matrix:
    """The operator lap - lambda I on the leaf cells."""
    rows, cols, vals = [], [], []
    nb, nd = g.nb, g.nd
    for k in range(len(g.level)):
        l = int(g.level[k])
        ih2 = (g.cells_per_side(l) / g.length) * (g.cells_per_side(l) / g.length)
        for c in g.cells():
            r = g.index(k, c)
            acc = {r: -2.0 * nd * ih2 - lam}
            for d in range(nd):
                for sgn in (-1, 1):
                    if 0 <= c[d] + sgn < nb:
                        cn = list(c)
                        cn[d] += sgn
                        nbr = {g.index(k, tuple(cn)): 1.0}
                    else:
                        nbr = g.neighbour(k, c, d, sgn)
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
    """Coordinates of every leaf cell on [0, L]^d, one array per direction
    (x, y[, z]), each [leaf][(z)][y][x]."""
    s = forest.scheme
    nd = s.ndim
    nb = s.block_nx[0]
    n = (s.base_blocks[0] << (forest.level.astype(np.int64) - 1)) * nb
    h = length / n
    loc = np.arange(nb, dtype=np.float64)
    out = []
    for d in range(nd):
        shape = [forest.n] + [1] * nd
        lshape = [1] * (nd + 1)
        lshape[nd - d] = nb
        x = (forest.ijk[:, d].reshape(shape) * nb + loc.reshape(lshape) + 0.5) * h.reshape(shape)
        out.append(np.broadcast_to(x, (forest.n,) + (nb,) * nd).copy())
    return tuple(out)


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

def _value(g: ForestGrid, k: int, c, d: int, sgn: int) -> dict:
    """{unknown: weight} of the value one cell over from leaf k's cell c
    along d: the cell itself inside the block, else the ghost rules (1)-(4),
    each of which interpolates linear data exactly."""
    if 0 <= c[d] + sgn < g.nb:
        cn = list(c)
        cn[d] += sgn
        return {g.index(k, tuple(cn)): 1.0}
    return g.neighbour(k, c, d, sgn)


def diff_matrix(g: ForestGrid, d: int) -> sp.csr_matrix:
    """Central difference along d (0 = x): (w(+1) - w(-1)) * (n_l / (2L))."""
    rows, cols, vals = [], [], []
    for k in range(len(g.level)):
        s = 0.5 * g.cells_per_side(int(g.level[k])) / g.length
        for c in g.cells():
            r = g.index(k, c)
            acc: dict = {}
            for sgn in (1, -1):
                for q, w in _value(g, k, c, d, sgn).items():
                    acc[q] = acc.get(q, 0.0) + sgn * w
            for q, w in acc.items():
                rows.append(r)
                cols.append(q)
                vals.append(w * s)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.ncell, g.ncell))


def cell_areas(forest, length: float) -> np.ndarray:
    """Area (2D) or volume (3D) of every leaf cell, [leaf][(z)][y][x]."""
    s = forest.scheme
    nd = s.ndim
    n = (s.base_blocks[0] << (forest.level.astype(np.int64) - 1)) * s.block_nx[0]
    a = (length / n) ** nd
    return np.broadcast_to(a.reshape([forest.n] + [1] * nd), (forest.n,) + (s.block_nx[0],) * nd).copy()


def divergence(forest, bx, by, length: float, bc: int, bz=None) -> np.ndarray:
    """Central-difference divergence at the leaf cells (x, then y[, then z])."""
    g = grid(forest, length, bc)
    shp = np.shape(bx)
    out = (diff_matrix(g, 0) @ np.ravel(bx)) + (diff_matrix(g, 1) @ np.ravel(by))
    if g.nd == 3:
        out = out + (diff_matrix(g, 2) @ np.ravel(bz))
    return out.reshape(shp)


def gradient(forest, phi, length: float, bc: int):
    g = grid(forest, length, bc)
    shp = np.shape(phi)
    return tuple((diff_matrix(g, d) @ np.ravel(phi)).reshape(shp) for d in range(g.nd))


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


def divb_project_nd(forest, B, length: float, bc: int):
    """divb_project for a 2D or 3D forest: B a list of nd leaf fields.
    Returns (list of projected fields, phi)."""
    div = divergence(forest, B[0], B[1], length, bc, B[2] if len(B) > 2 else None)
    phi = poisson(forest, div, length, bc)
    G = gradient(forest, phi, length, bc)
    return [B[d] - G[d] for d in range(len(B))], phi


def divb_project(forest, bx, by, length: float, bc: int):
    """The divergence control of Sec. 2.4 on the leaf cells of a 2D forest:
    phi = the zero-mean solution of lap(phi) = div B*, B = B* - grad phi
    (central differences for div and grad, the 5-point composite lap: an
    approximate projection).  Returns (bx, by, phi)."""
    phi = poisson(forest, divergence(forest, bx, by, length, bc), length, bc)
    gx, gy = gradient(forest, phi, length, bc)
    return bx - gx, by - gy, phi
