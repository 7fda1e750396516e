"""Seeded synthetic inputs shared by the HIP path's callers and the oracle.

This package holds no step of the finite-volume method: it builds block
forests (leaf lists with 2:1 balance, Morton order) and initial conditions in
conserved variables, the scheme parameters of each workload, and the relative
L1 difference used to compare two states.  It imports neither the product
package nor the oracle: tests, the smoke check and the bench hand its forests
and states to both.  One stored input, the leaf list of the 3D AMR blast
refined by the Loehner estimator (data/blast_lohner_forest.npz), was written
by oracle/lohner_forest.py.

Workloads (the paper's MPI-AMRVAC, arXiv 2004.03275, runs the solver it names
on block forests, Sec. 1.3; the configurations below are synthetic stand-ins
with the shapes of the problems it measures):

* ``sod``   1D Euler Sod tube, 1024 cells, TVDLF + minmod + SSP-RK2, CFL 0.8.
* ``kh``    2D Kelvin-Helmholtz, 256 leaves of 16x16, HLLC + van Leer + SSP-RK3.
* ``ot``    2D MHD Orszag-Tang, 1024 leaves of 16x16, HLL + GLM + van Leer.
* ``blast`` 3D spherical blast on a 4-level octree forest of 16^3 leaves
            (the hydrodynamic analogue of the paper's 3D blast, Sec. 2.4).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Sequence

import numpy as np

PERIODIC = 0
ZERO_GRADIENT = 1

EULER = 0
MHD = 1
POLY = 2  # polytrope p = c_ad rho^gamma without energy equation (shallow water)

TVDLF = 0
HLL = 1
HLLC = 2

MINMOD = 0
VANLEER = 1
MC = 2  # monotonized central ('woodward')
KOREN = 3
CADA = 4


@dataclasses.dataclass
class Scheme:
    """Geometry and scheme parameters of one forest (par-file keys of Sec. 1.3)."""

    ndim: int
    block_nx: tuple = (16, 16, 16)
    base_blocks: tuple = (1, 1, 1)
    max_level: int = 1
    xmin: tuple = (0.0, 0.0, 0.0)
    xmax: tuple = (1.0, 1.0, 1.0)
    physics: int = EULER
    gamma: float = 1.4
    flux: int = HLLC
    limiter: int = VANLEER
    rk_stages: int = 3
    cfl: float = 0.8
    bc: int = PERIODIC
    nghost: int = 2
    lohner_tol: float = 0.1
    lohner_coarsen_frac: float = 0.125
    lohner_eps: float = 0.01
    lohner_w_rho: float = 0.5
    lohner_w_p: float = 0.5
    glm_cr: float = 0.18
    cad: float = 1.0  # c_ad of the polytrope
    cada_radius: float = 0.0  # r of Cada's smoothness switch (0: the limited function alone)

    def __post_init__(self):
        nd = self.ndim
        bn = list(self.block_nx) + [1] * 3
        bb = list(self.base_blocks) + [1] * 3
        self.block_nx = tuple(bn[d] if d < nd else 1 for d in range(3))
        self.base_blocks = tuple(bb[d] if d < nd else 1 for d in range(3))
        self.xmin = tuple(float(x) for x in (list(self.xmin) + [0.0] * 3)[:3])
        self.xmax = tuple(float(x) for x in (list(self.xmax) + [1.0] * 3)[:3])

    @property
    def nvar(self) -> int:
        if self.physics == POLY:
            return 1 + self.ndim
        return 2 + self.ndim if self.physics == EULER else 3 + 2 * self.ndim

    @property
    def cells_per_block(self) -> int:
        return int(np.prod(self.block_nx[: self.ndim]))

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Forest:
    """A leaf list: level (1-based) and block coordinates at that level."""

    scheme: Scheme
    level: np.ndarray  # int32 [n]
    ijk: np.ndarray  # int32 [n, 3]

    @property
    def n(self) -> int:
        return int(self.level.shape[0])

    def state_shape(self) -> tuple:
        s = self.scheme
        shp = [s.nvar, self.n]
        for d in reversed(range(s.ndim)):
            shp.append(s.block_nx[d])
        return tuple(shp)

    def level_counts(self) -> dict:
        u, c = np.unique(self.level, return_counts=True)
        return {int(a): int(b) for a, b in zip(u, c)}


# ---------------------------------------------------------------------------
# forests
# ---------------------------------------------------------------------------


def _morton_key(level: np.ndarray, ijk: np.ndarray, max_level: int, ndim: int) -> np.ndarray:
    """Interleave the bits of each leaf's lower corner at the finest level."""
    shift = (max_level - level).astype(np.int64)
    c = ijk.astype(np.int64) << shift[:, None]
    key = np.zeros(len(level), dtype=np.int64)
    for bit in range(21):
        for d in range(ndim):
            key |= ((c[:, d] >> bit) & 1) << (ndim * bit + d)
    return key


def _finish(scheme: Scheme, nodes: list) -> Forest:
    lev = np.array([n[0] for n in nodes], dtype=np.int32)
    ijk = np.array([n[1:] for n in nodes], dtype=np.int32).reshape(-1, 3)
    order = np.argsort(_morton_key(lev, ijk, scheme.max_level, scheme.ndim), kind="stable")
    return Forest(scheme, lev[order].copy(), ijk[order].copy())


def uniform_forest(scheme: Scheme, level: int = 1) -> Forest:
    """Every leaf at one level: a pure domain decomposition (Sec. 1.3)."""
    nd = scheme.ndim
    nb = [scheme.base_blocks[d] << (level - 1) if d < nd else 1 for d in range(3)]
    nodes = [(level, i, j, k) for k in range(nb[2]) for j in range(nb[1]) for i in range(nb[0])]
    return _finish(scheme, nodes)


def _offsets(ndim: int):
    rng = [(-1, 0, 1)] * ndim + [(0,)] * (3 - ndim)
    for a in rng[0]:
        for b in rng[1]:
            for c in rng[2]:
                if a or b or c:
                    yield (a, b, c)


def refined_forest(scheme: Scheme, refine: Callable[[int, tuple], bool]) -> Forest:
    """Refine level by level where ``refine(level, (i, j, k))`` holds, then
    enforce 2:1 balance across faces, edges and corners."""
    nd, L = scheme.ndim, scheme.max_level
    per = scheme.bc == PERIODIC

    def nblk(l, d):
        return scheme.base_blocks[d] << (l - 1) if d < nd else 1

    refined: set = set()
    level_nodes = [
        (1, i, j, k)
        for k in range(nblk(1, 2))
        for j in range(nblk(1, 1))
        for i in range(nblk(1, 0))
    ]
    for l in range(1, L):
        for node in level_nodes:
            if refine(l, node[1:]):
                refined.add(node)
        # balance: neighbours (same level) of every refined node must exist,
        # i.e. their parents must be refined; ripple from fine to coarse
        changed = True
        while changed:
            changed = False
            for node in sorted(refined, key=lambda t: -t[0]):
                lv = node[0]
                if lv < 2:
                    continue
                for o in _offsets(nd):
                    c = [node[1 + d] + o[d] for d in range(3)]
                    ok = True
                    for d in range(nd):
                        n = nblk(lv, d)
                        if c[d] < 0 or c[d] >= n:
                            if per:
                                c[d] %= n
                            else:
                                ok = False
                    if not ok:
                        continue
                    par = (lv - 1, c[0] >> 1, c[1] >> 1, c[2] >> 1)
                    if par not in refined:
                        refined.add(par)
                        changed = True
        nxt = []
        for node in refined:
            if node[0] == l:
                lv, i, j, k = node
                for q in range(1 << nd):
                    ch = [2 * i + (q & 1), 2 * j + ((q >> 1) & 1) if nd >= 2 else 0,
                          2 * k + ((q >> 2) & 1) if nd >= 3 else 0]
                    nxt.append((l + 1, *ch))
        level_nodes = nxt
    # collect leaves: existing nodes that are not refined
    leaves = []
    stack = [
        (1, i, j, k)
        for k in range(nblk(1, 2))
        for j in range(nblk(1, 1))
        for i in range(nblk(1, 0))
    ]
    while stack:
        node = stack.pop()
        if node in refined:
            lv, i, j, k = node
            for q in range(1 << nd):
                stack.append((lv + 1, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1) if nd >= 2 else 0,
                              2 * k + ((q >> 2) & 1) if nd >= 3 else 0))
        else:
            leaves.append(node)
    return _finish(scheme, leaves)


def cell_centres(forest: Forest) -> list:
    """Cell-centre coordinates per dimension, each shaped like one state
    variable ([n, nz, ny, nx] without unused axes)."""
    s = forest.scheme
    nd = s.ndim
    out = []
    for d in range(nd):
        ncell_dom = (np.asarray(s.base_blocks[d], dtype=np.int64) << (forest.level.astype(np.int64) - 1)) * s.block_nx[d]
        dx = (s.xmax[d] - s.xmin[d]) / ncell_dom.astype(np.float64)
        shape = [1] + [1] * nd
        ax = 1 + (nd - 1 - d)
        shape[ax] = s.block_nx[d]
        loc = np.arange(s.block_nx[d], dtype=np.float64).reshape(shape)
        g = forest.ijk[:, d].astype(np.float64).reshape([forest.n] + [1] * nd) * s.block_nx[d] + loc
        x = s.xmin[d] + (g + 0.5) * dx.reshape([forest.n] + [1] * nd)
        full = [forest.n] + [s.block_nx[e] for e in reversed(range(nd))]
        out.append(np.broadcast_to(x, full).copy())
    return out


def _box_shell_hit(lo: np.ndarray, hi: np.ndarray, centre, radius: float, pad: float) -> bool:
    """Does the box [lo, hi] grown by pad contain points both inside and
    outside the sphere (i.e. touch its surface)?"""
    lo = lo - pad
    hi = hi + pad
    c = np.asarray(centre)
    nearest = np.clip(c, lo, hi)
    dmin = float(np.sqrt(np.sum((nearest - c) ** 2)))
    far = np.where(np.abs(lo - c) > np.abs(hi - c), lo, hi)
    dmax = float(np.sqrt(np.sum((far - c) ** 2)))
    return dmin <= radius <= dmax


# ---------------------------------------------------------------------------
# pseudo-random numbers: splitmix64 (Steele, Lea, Flood 2014)
# ---------------------------------------------------------------------------

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """The first ``count`` outputs of splitmix64 started at ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---------------------------------------------------------------------------
# initial conditions (conserved variables U = (rho, rho v, E [, B, psi]),
# E = rho v^2 / 2 + p / (gamma - 1) [+ B^2 / 2], Sec. 1.1)
# ---------------------------------------------------------------------------


def _euler_state(s: Scheme, rho, vel: Sequence, p) -> np.ndarray:
    nd = s.ndim
    U = np.empty((s.nvar,) + rho.shape, dtype=np.float64)
    U[0] = rho
    kin = np.zeros_like(rho)
    for d in range(nd):
        U[1 + d] = rho * vel[d]
        kin = kin + vel[d] * vel[d]
    U[1 + nd] = p / (s.gamma - 1.0) + 0.5 * rho * kin
    return U


def _mhd_state(s: Scheme, rho, vel: Sequence, p, B: Sequence) -> np.ndarray:
    nd = s.ndim
    U = np.empty((s.nvar,) + rho.shape, dtype=np.float64)
    U[0] = rho
    kin = np.zeros_like(rho)
    mag = np.zeros_like(rho)
    for d in range(nd):
        U[1 + d] = rho * vel[d]
        kin = kin + vel[d] * vel[d]
        U[2 + nd + d] = B[d]
        mag = mag + B[d] * B[d]
    U[1 + nd] = p / (s.gamma - 1.0) + 0.5 * rho * kin + 0.5 * mag
    U[2 + 2 * nd] = 0.0
    return U


def _poly_state(s: Scheme, rho, vel: Sequence) -> np.ndarray:
    U = np.empty((s.nvar,) + rho.shape, dtype=np.float64)
    U[0] = rho
    for d in range(s.ndim):
        U[1 + d] = rho * vel[d]
    return U


def state_from_primitive(forest: Forest, rho, vel, p=None, B=None) -> np.ndarray:
    """Conserved state from rho, velocity components, pressure (ignored by
    the polytrope, whose pressure follows from rho) and field (MHD)."""
    s = forest.scheme
    if s.physics == POLY:
        return _poly_state(s, rho, vel)
    if s.physics == EULER:
        return _euler_state(s, rho, vel, p)
    return _mhd_state(s, rho, vel, p, B)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------


def sod_scheme(ncells: int = 1024) -> Scheme:
    return Scheme(ndim=1, block_nx=(ncells,), base_blocks=(1,), max_level=1, physics=EULER,
                  gamma=1.4, flux=TVDLF, limiter=MINMOD, rk_stages=2, cfl=0.8, bc=ZERO_GRADIENT)


def sod(ncells: int = 1024, nblocks: int = 1):
    """Sod tube on [0, 1]: (rho, u, p) = (1, 0, 1) left of 0.5, (0.125, 0, 0.1)
    right; zero-gradient ends; run to t = 0.2."""
    s = sod_scheme(ncells // nblocks)
    s.base_blocks = (nblocks, 1, 1)
    f = uniform_forest(s)
    (x,) = cell_centres(f)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return f, state_from_primitive(f, rho, [np.zeros_like(rho)], p)


def kh_scheme(nblk: int = 16) -> Scheme:
    return Scheme(ndim=2, block_nx=(16, 16), base_blocks=(nblk, nblk), max_level=1, physics=EULER,
                  gamma=1.4, flux=HLLC, limiter=VANLEER, rk_stages=3, cfl=0.8, bc=PERIODIC)


def kh(nblk: int = 16, seed: int = 1234, amplitude: float = 0.01, scheme: Scheme | None = None,
       level: int = 1):
    """Kelvin-Helmholtz shear layer on [0,1]^2: rho = 2, u = +0.5 where
    |y - 0.5| < 0.25, else rho = 1, u = -0.5; p = 2.5; v = amplitude (2 xi - 1)
    with xi from splitmix64(seed) in global row-major cell order."""
    s = scheme or kh_scheme(nblk)
    f = uniform_forest(s, level)
    x, y = cell_centres(f)
    inner = np.abs(y - 0.5) < 0.25
    rho = np.where(inner, 2.0, 1.0)
    u = np.where(inner, 0.5, -0.5)
    p = np.full_like(rho, 2.5)
    ncx = (s.base_blocks[0] << (level - 1)) * s.block_nx[0]
    ncy = (s.base_blocks[1] << (level - 1)) * s.block_nx[1]
    xi = uniform01(seed, ncx * ncy)
    gi = (f.ijk[:, 0][:, None, None] * s.block_nx[0] + np.arange(s.block_nx[0])[None, None, :])
    gj = (f.ijk[:, 1][:, None, None] * s.block_nx[1] + np.arange(s.block_nx[1])[None, :, None])
    gidx = (gj * ncx + gi).astype(np.int64)
    v = amplitude * (2.0 * xi[gidx] - 1.0)
    return f, state_from_primitive(f, rho, [u, v], p)


def ot_scheme(nblk: int = 32) -> Scheme:
    return Scheme(ndim=2, block_nx=(16, 16), base_blocks=(nblk, nblk), max_level=1, physics=MHD,
                  gamma=5.0 / 3.0, flux=HLL, limiter=VANLEER, rk_stages=3, cfl=0.8, bc=PERIODIC)


def orszag_tang(nblk: int = 32, scheme: Scheme | None = None):
    """Orszag-Tang vortex on [0,1]^2 (mu0 = 1): rho = 25/9, p = 5/3,
    v = (-sin 2 pi y, sin 2 pi x), B = (-sin 2 pi y, sin 4 pi x), psi = 0."""
    s = scheme or ot_scheme(nblk)
    f = uniform_forest(s)
    x, y = cell_centres(f)
    rho = np.full_like(x, 25.0 / 9.0)
    p = np.full_like(x, 5.0 / 3.0)
    vx = -np.sin(2.0 * math.pi * y)
    vy = np.sin(2.0 * math.pi * x)
    bx = -np.sin(2.0 * math.pi * y)
    by = np.sin(4.0 * math.pi * x)
    return f, state_from_primitive(f, rho, [vx, vy], p, [bx, by])


def blast_scheme(base: int = 16, max_level: int = 4) -> Scheme:
    return Scheme(ndim=3, block_nx=(16, 16, 16), base_blocks=(base, base, base), max_level=max_level,
                  xmin=(-0.5, -0.5, -0.5), xmax=(0.5, 0.5, 0.5), physics=EULER, gamma=1.4, flux=HLLC,
                  limiter=VANLEER, rk_stages=3, cfl=0.8, bc=PERIODIC)


def blast_forest(scheme: Scheme, radius: float = 0.1, centre=(0.0, 0.0, 0.0), buffer_cells: float = 8.0) -> Forest:
    """Octree forest refined around the surface of the over-pressured sphere:
    a block at level l is refined while l < max_level if its box, grown by
    ``buffer_cells`` cells of that level, touches the sphere surface.  For the
    step initial state this marks the blocks whose cells see the pressure
    jump (where the Loehner estimator of Sec. 1.3 is large), plus a buffer."""
    s = scheme
    nd = s.ndim
    ext = np.array(s.xmax[:nd]) - np.array(s.xmin[:nd])
    lo0 = np.array(s.xmin[:nd])

    def refine(l, c):
        nb = np.array([s.base_blocks[d] << (l - 1) for d in range(nd)], dtype=np.float64)
        h = ext / nb
        lo = lo0 + np.array(c[:nd], dtype=np.float64) * h
        dx = h / np.array(s.block_nx[:nd])
        return _box_shell_hit(lo, lo + h, centre[:nd], radius, float(buffer_cells * dx.max()))

    return refined_forest(s, refine)


DATA = __import__("os").path.join(__import__("os").path.dirname(__file__), "data")


def blast_lohner_forest(scheme: Scheme | None = None) -> Forest:
    """The 3D AMR blast's forest (16^3 base blocks of 16^3 cells, 4 levels)
    refined where the Loehner estimator flags its initial state, with an
    8-cell buffer and 2:1 balance: the stored leaf list written by
    oracle/lohner_forest.py (19,384 leaves)."""
    s = scheme or blast_scheme()
    if s.ndim != 3 or s.base_blocks != (16, 16, 16) or s.max_level != 4 or s.block_nx != (16, 16, 16):
        raise ValueError("the stored Loehner forest is the 16^3-base, 4-level blast")
    with np.load(__import__("os").path.join(DATA, "blast_lohner_forest.npz")) as d:
        return Forest(s, d["level"].astype(np.int32), d["ijk"].astype(np.int32))


def blast(scheme: Scheme | None = None, radius: float = 0.1, p_in: float = 100.0, p_out: float = 0.1,
          centre=(0.0, 0.0, 0.0), buffer_cells: float = 8.0, forest: Forest | None = None):
    """Spherical blast in [-0.5, 0.5]^3: rho = 1, v = 0, p = p_in where the
    cell centre lies within ``radius`` of ``centre``, else p_out."""
    s = scheme or blast_scheme()
    f = forest or blast_forest(s, radius, centre, buffer_cells)
    xs = cell_centres(f)
    r2 = np.zeros_like(xs[0])
    for d in range(s.ndim):
        r2 = r2 + (xs[d] - centre[d]) ** 2
    rho = np.ones_like(r2)
    p = np.where(r2 < radius * radius, p_in, p_out)
    vel = [np.zeros_like(r2) for _ in range(s.ndim)]
    return f, state_from_primitive(f, rho, vel, p)


def dam_break_scheme(base: int = 6, max_level: int = 3, flux: int = HLL) -> Scheme:
    """The paper's circular dam break on a Cartesian grid (Sec. 2.2): the
    shallow water equations as the polytrope rho = h, c_ad = 1/2, gamma = 2
    (dimensionless, lengths in metres), [-20, 20]^2 with zero-gradient
    borders, HLL, three-step Runge-Kutta, Koren's limiter, Courant number
    0.9, 3 levels.  16^2 blocks on a 96^2 base grid stand in for the paper's
    10^2 blocks on 100^2 (effective 384^2 against 400^2)."""
    return Scheme(ndim=2, block_nx=(16, 16), base_blocks=(base, base), max_level=max_level,
                  xmin=(-20.0, -20.0), xmax=(20.0, 20.0), physics=POLY, gamma=2.0, cad=0.5, flux=flux,
                  limiter=KOREN, rk_stages=3, cfl=0.9, bc=ZERO_GRADIENT)


def dam_break(base: int = 6, max_level: int = 3, r_dam: float = 2.5, h_in: float = 2.5, h_out: float = 0.5,
              buffer_cells: float = 4.0, scheme: Scheme | None = None, forest: Forest | None = None):
    """Water height h_in within r_dam of the origin (cell centres), h_out
    outside, at rest; the paper runs it to t = 15.  The forest is refined
    around the dam wall like the blasts' around their surfaces."""
    s = scheme or dam_break_scheme(base, max_level)
    f = forest or blast_forest(s, r_dam, (0.0, 0.0, 0.0), buffer_cells)
    xs = cell_centres(f)
    r2 = xs[0] ** 2 + xs[1] ** 2
    h = np.where(r2 < r_dam * r_dam, h_in, h_out)
    return f, state_from_primitive(f, h, [np.zeros_like(h), np.zeros_like(h)])


def mhd_blast_scheme(ndim: int = 2, base: int = 4, max_level: int = 4, limiter: int = CADA,
                     flux: int = HLLC) -> Scheme:
    """The paper's MHD blast (Sec. 2.4) on [-0.5, 0.5]^ndim: gamma 5/3,
    three-step Runge-Kutta, HLLC (the MHD form after Li 2005), Courant
    number 0.9 (the drivers ramp the first 10 steps), periodic sides,
    16-cell blocks on a 64-cell base grid, Cada's third-order limiter.  GLM
    cleaning stands in for the paper's multigrid div B control."""
    nd = ndim
    return Scheme(ndim=nd, block_nx=(16,) * nd, base_blocks=(base,) * nd, max_level=max_level,
                  xmin=(-0.5,) * nd, xmax=(0.5,) * nd, physics=MHD, gamma=5.0 / 3.0, flux=flux,
                  limiter=limiter, rk_stages=3, cfl=0.9, bc=PERIODIC)


def mhd_blast(ndim: int = 2, base: int = 4, max_level: int = 4, radius: float = 0.1, p_in: float = 10.0,
              p_out: float = 0.1, buffer_cells: float = 4.0, scheme: Scheme | None = None,
              forest: Forest | None = None):
    """rho = 1, v = 0, p = p_in within ``radius`` of the origin (cell
    centres) else p_out, uniform B = (1, 1[, 1])/sqrt(ndim), psi = 0: plasma
    beta 0.2 outside and 20 inside (mu0 = 1).  The forest is refined around
    the blast surface like the hydrodynamic blast's."""
    s = scheme or mhd_blast_scheme(ndim, base, max_level)
    f = forest or blast_forest(s, radius, (0.0, 0.0, 0.0), buffer_cells)
    xs = cell_centres(f)
    r2 = np.zeros_like(xs[0])
    for d in range(s.ndim):
        r2 = r2 + xs[d] ** 2
    rho = np.ones_like(r2)
    p = np.where(r2 < radius * radius, p_in, p_out)
    vel = [np.zeros_like(r2) for _ in range(s.ndim)]
    b0 = 1.0 / math.sqrt(s.ndim)
    B = [np.full_like(r2, b0) for _ in range(s.ndim)]
    return f, state_from_primitive(f, rho, vel, p, B)


def relative_l1(U: np.ndarray, R: np.ndarray, forest: Forest) -> np.ndarray:
    """Per conserved variable: sum |U - R| dV / max(sum |R| dV, 1e-6 sum |E_R| dV),
    with dV the cell volume of each leaf's level (the polytrope, which has no
    energy: 1e-6 sum |rho_R| dV)."""
    s = forest.scheme
    nd = s.ndim
    vol = np.ones(forest.n)
    for d in range(nd):
        ncell = (np.asarray(s.base_blocks[d], dtype=np.float64) * (2.0 ** (forest.level - 1))) * s.block_nx[d]
        vol = vol * ((s.xmax[d] - s.xmin[d]) / ncell)
    w = vol.reshape([forest.n] + [1] * nd)
    diff = np.abs(U - R) * w
    ref = np.abs(R) * w
    axes = tuple(range(1, U.ndim))
    num = diff.sum(axis=axes)
    den = ref.sum(axis=axes)
    floor = 1e-6 * ref[0 if s.physics == POLY else 1 + nd].sum()
    return num / np.maximum(den, floor)


# ---------------------------------------------------------------------------
# learned flagger: seeded initial weights and jittered blast parameters
# ---------------------------------------------------------------------------

MLP_NIN, MLP_NH, MLP_NOUT = 128, 64, 2
MLP_NPARAM = MLP_NH * MLP_NIN + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NOUT * MLP_NH + MLP_NOUT


def mlp_init(seed: int) -> np.ndarray:
    """He-uniform initial weights (bound sqrt(6 / fan_in)), zero biases, as the
    binary32 parameter vector W1 [64][128], b1, W2 [64][64], b2, W3 [2][64], b3 [2]."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (MLP_NH, MLP_NIN)) * np.sqrt(6.0 / MLP_NIN)
    W2 = rng.uniform(-1, 1, (MLP_NH, MLP_NH)) * np.sqrt(6.0 / MLP_NH)
    W3 = rng.uniform(-1, 1, (MLP_NOUT, MLP_NH)) * np.sqrt(6.0 / MLP_NH)
    z = np.zeros(MLP_NH)
    return np.concatenate([W1.ravel(), z, W2.ravel(), z, W3.ravel(), np.zeros(MLP_NOUT)]).astype(np.float32)


def jittered_blast(seed: int, base: int = 8, max_level: int = 3, coarse: bool = False):
    """A blast with seeded centre (|c_i| <= 0.1), radius in [0.08, 0.12] and
    inner pressure in [50, 200] on its own refined forest, or with coarse=True
    on the uniform level-1 forest (every leaf below the top level, so the
    blocks the blast crosses are ones a flagger would refine)."""
    rng = np.random.default_rng(seed)
    radius = float(rng.uniform(0.08, 0.12))
    centre = tuple(float(c) for c in rng.uniform(-0.1, 0.1, 3))
    p_in = float(rng.uniform(50.0, 200.0))
    s = blast_scheme(base=base, max_level=max_level)
    f = uniform_forest(s) if coarse else blast_forest(s, radius=radius, centre=centre, buffer_cells=4.0)
    return blast(s, radius=radius, p_in=p_in, centre=centre, forest=f)


def mlp_random_features(seed: int, n: int) -> np.ndarray:
    """Seeded synthetic feature rows [n, 128] (bfloat16 bit patterns of
    values in about [-1, 1]) and class labels (+1 with probability 0.3, -1
    with 0.3, else 0), for kernel parity checks."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((n, MLP_NIN)) * 0.5).astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    r = rng.uniform(size=n)
    y = np.where(r < 0.3, 1.0, np.where(r < 0.6, -1.0, 0.0)).astype(np.float32)
    return bits, y


# -- reaction-diffusion on uniform grids (Sec. 2.5) -------------------------

def rd_cell_centres(ndim: int, n: int, length: float) -> list:
    """Cell-centre coordinates (x, y[, z]) of an n^ndim grid on [0, L]^ndim,
    arrays indexed [z][y][x]."""
    c = (np.arange(n) + 0.5) * (length / n)
    grids = np.meshgrid(*([c] * ndim), indexing="ij")  # [x][y][z] order
    return [np.ascontiguousarray(np.transpose(g)) for g in grids]


def schnakenberg_initial(ndim: int = 2, n: int = 256, a: float = 0.1305, b: float = 0.7695):
    """Sec. 2.5.2: v = b/(a+b)^2, u = a + b + exp(-100 |r - r0|^2) on the unit
    square/cube, r0 = (1/3, 1/2[, 1/2]).  Returns (u, v, L = 1)."""
    xs = rd_cell_centres(ndim, n, 1.0)
    r0 = (1.0 / 3.0, 0.5, 0.5)
    r2 = sum((x - r0[d]) ** 2 for d, x in enumerate(xs))
    u = a + b + np.exp(-100.0 * r2)
    v = np.full_like(u, b / (a + b) ** 2)
    return u, v, 1.0


def gray_scott_initial(n: int = 256):
    """Sec. 2.5.2: the steady state u = 1, v = 0 with two Gaussians
    0.5 exp(-25 |r - r_i|^2), r_1 = (0.5, 0.5), r_2 = (0.55, 0.6),
    subtracted from u and added to v, on the periodic square of side 2.
    Returns (u, v, L = 2)."""
    x, y = rd_cell_centres(2, n, 2.0)
    g = sum(0.5 * np.exp(-25.0 * ((x - cx) ** 2 + (y - cy) ** 2)) for cx, cy in ((0.5, 0.5), (0.55, 0.6)))
    return 1.0 - g, g.copy(), 2.0


# -- elliptic problems on a 2D block-adaptive forest (Sec. 1.4) -------------

def fmg_scheme(base: int = 2, max_level: int = 3, bc: int = PERIODIC, length: float = 1.0, ndim: int = 2) -> Scheme:
    """A forest of 16^d blocks on [0, L]^d (d = 2, 3) with base^d blocks at level 1."""
    return Scheme(ndim=ndim, block_nx=(16, 16, 16), base_blocks=(base,) * ndim, max_level=max_level,
                  xmin=(0.0,) * ndim, xmax=(length,) * ndim, bc=bc)


def fmg_forest(scheme: Scheme, centre=(0.5, 0.5, 0.5), radius: float = 0.25, buffer_cells: float = 2.0) -> Forest:
    """Quadtree / octree forest refined around a circle / sphere (centre and
    radius relative to the side L): a block at level l is refined while l <
    max_level if its box, grown by ``buffer_cells`` cells of that level,
    touches the circle -- shells of levels whose coarse-fine faces run in
    every direction and orientation."""
    s = scheme
    nd = s.ndim
    side = s.xmax[0] - s.xmin[0]
    c = tuple(centre[d] * side for d in range(nd))

    def refine(l, ij):
        nb = s.base_blocks[0] << (l - 1)
        h = side / nb
        lo = np.array([s.xmin[d] + ij[d] * h for d in range(nd)])
        return _box_shell_hit(lo, lo + h, c, radius * side, float(buffer_cells * h / s.block_nx[0]))

    return refined_forest(s, refine)


def gray_scott_amr(base: int = 8, max_level: int = 3):
    """Sec. 2.5.2's Gray-Scott AMR setup on a static forest: the periodic
    square of side 2, base x base blocks of 16^2 cells at level 1 (128^2 for
    base 8) and max_level 3 (512^2 effective); a block at level l <
    max_level is refined while its box comes within 0.7 - 0.2 (l - 1) of a
    perturbation centre (the paper refines as the pattern grows; here the
    forest stays as it starts).  Initial state: u = 1, v = 0 with the two
    Gaussians 0.5 exp(-25 |r - r_i|^2), r_1 = (0.5, 0.5), r_2 = (0.55, 0.6),
    subtracted from u and added to v.  Returns (forest, u, v, L = 2), fields
    [leaf][y][x]."""
    s = fmg_scheme(base=base, max_level=max_level, bc=PERIODIC, length=2.0)
    centres = ((0.5, 0.5), (0.55, 0.6))

    def refine(l, ij):
        h = 2.0 / (base << (l - 1))
        lo = np.array([ij[0] * h, ij[1] * h])
        reach = 0.7 - 0.2 * (l - 1)
        for c in centres:
            c = np.asarray(c)
            if float(np.sqrt(np.sum((np.clip(c, lo, lo + h) - c) ** 2))) < reach:
                return True
        return False

    f = refined_forest(s, refine)
    x, y = cell_centres(f)
    g = sum(0.5 * np.exp(-25.0 * ((x - cx) ** 2 + (y - cy) ** 2)) for cx, cy in centres)
    return f, 1.0 - g, g.copy(), 2.0
