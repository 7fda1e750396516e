"""CPU oracle of the block-forest finite-volume update.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and bench.py's CPU-baseline
leg may import it; the product package never does.  It wraps liborc.so
(oracle/orc.c, plain C in binary64) and exposes the same operations as the
HIP library's C-ABI on host arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


class _Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("block_nx", ctypes.c_int32 * 3),
        ("nghost", ctypes.c_int32),
        ("base_blocks", ctypes.c_int32 * 3),
        ("max_level", ctypes.c_int32),
        ("physics", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("rk_stages", ctypes.c_int32),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("pad_", ctypes.c_int32),
        ("xmin", ctypes.c_double * 3),
        ("xmax", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("lohner_tol", ctypes.c_double),
        ("lohner_coarsen_frac", ctypes.c_double),
        ("lohner_eps", ctypes.c_double),
        ("lohner_w_rho", ctypes.c_double),
        ("lohner_w_p", ctypes.c_double),
        ("glm_cr", ctypes.c_double),
        ("cad", ctypes.c_double),
        ("cada_radius", ctypes.c_double),
    ]


def bind(path: str) -> ctypes.CDLL:
    """Load an oracle library build at `path` and declare its functions."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.orc_forest_create.argtypes = [ctypes.POINTER(_Config), ctypes.c_int64, P, P, ctypes.POINTER(P)]
    L.orc_forest_destroy.argtypes = [P]
    L.orc_nvar.argtypes = [P]
    L.orc_set_state.argtypes = [P, P, ctypes.c_int64]
    L.orc_get_state.argtypes = [P, P, ctypes.c_int64]
    L.orc_max_dt.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    L.orc_glm_ch.argtypes = [P]
    L.orc_glm_ch.restype = ctypes.c_double
    L.orc_advance.argtypes = [P, ctypes.c_double]
    L.orc_flag_blocks.argtypes = [P, P, P]
    L.orc_padded_block.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64]
    L.orc_face_kinds.argtypes = [P, ctypes.c_int64, P]
    L.orc_lohner_cells.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64]
    L.orc_face_flux.argtypes = [P, P, P, ctypes.c_int, P]
    L.orc_regrid_plan.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P, P]
    L.orc_regrid_transfer.argtypes = [P, P]
    L.orc_limiter_value.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.orc_limiter_value.restype = ctypes.c_double
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = None
    L.orc_get_threads.restype = ctypes.c_int
    L.orc_last_error.restype = ctypes.c_char_p
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = bind(_build.LIB)
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != 0:
        raise OracleError(rc, lib().orc_last_error().decode())


def make_config(s) -> _Config:
    c = _Config()
    c.ndim = s.ndim
    for d in range(3):
        c.block_nx[d] = s.block_nx[d]
        c.base_blocks[d] = s.base_blocks[d]
        c.xmin[d] = s.xmin[d]
        c.xmax[d] = s.xmax[d]
        c.bc[d][0] = s.bc
        c.bc[d][1] = s.bc
    c.nghost = s.nghost
    c.max_level = s.max_level
    c.physics = s.physics
    c.flux = s.flux
    c.limiter = s.limiter
    c.rk_stages = s.rk_stages
    c.gamma = s.gamma
    c.cfl = s.cfl
    c.lohner_tol = s.lohner_tol
    c.lohner_coarsen_frac = s.lohner_coarsen_frac
    c.lohner_eps = s.lohner_eps
    c.lohner_w_rho = s.lohner_w_rho
    c.lohner_w_p = s.lohner_w_p
    c.glm_cr = s.glm_cr
    c.cad = s.cad
    c.cada_radius = s.cada_radius
    return c


def limiter_value(kind: int, a: float, b: float, thr2: float = 0.0) -> float:
    """The oracle's limited slope for the differences a (away from the face)
    and b (toward it); thr2 = (r dx)^2 of Cada's smoothness switch."""
    return float(lib().orc_limiter_value(int(kind), float(a), float(b), float(thr2)))


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


class OracleForest:
    """The oracle's forest: the same operations as the HIP library on host arrays."""

    def __init__(self, forest, config=None):
        self.forest = forest
        self.scheme = forest.scheme
        cfg = config if config is not None else make_config(forest.scheme)
        self._h = ctypes.c_void_p()
        lev = np.ascontiguousarray(forest.level, dtype=np.int32)
        ijk = np.ascontiguousarray(forest.ijk, dtype=np.int32)
        _check(lib().orc_forest_create(ctypes.byref(cfg), forest.n, lev.ctypes.data, ijk.ctypes.data,
                                       ctypes.byref(self._h)))
        self.nvar = lib().orc_nvar(self._h)
        self.shape = forest.state_shape()

    def close(self):
        if self._h:
            lib().orc_forest_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, U: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float64)
        if U.shape != self.shape:
            raise ValueError(f"state shape {U.shape} != {self.shape}")
        _check(lib().orc_set_state(self._h, U.ctypes.data, U.size))

    def get_state(self) -> np.ndarray:
        U = np.empty(self.shape, dtype=np.float64)
        _check(lib().orc_get_state(self._h, U.ctypes.data, U.size))
        return U

    def max_dt(self) -> float:
        dt = ctypes.c_double()
        _check(lib().orc_max_dt(self._h, ctypes.byref(dt)))
        return dt.value

    @property
    def glm_ch(self) -> float:
        return float(lib().orc_glm_ch(self._h))

    def advance(self, dt: float):
        _check(lib().orc_advance(self._h, float(dt)))

    def flag_blocks(self, with_emax: bool = False):
        flags = np.empty(self.forest.n, dtype=np.int8)
        emax = np.empty(self.forest.n, dtype=np.float64)
        _check(lib().orc_flag_blocks(self._h, flags.ctypes.data, emax.ctypes.data))
        return (flags, emax) if with_emax else flags

    def padded_block(self, leaf: int) -> np.ndarray:
        s = self.scheme
        px = [s.block_nx[d] + 2 * s.nghost if d < s.ndim else 1 for d in range(3)]
        out = np.empty((self.nvar, px[2], px[1], px[0]), dtype=np.float64)
        _check(lib().orc_padded_block(self._h, int(leaf), out.ctypes.data, out.size))
        return out

    def lohner_cells(self, leaf: int) -> np.ndarray:
        s = self.scheme
        out = np.empty([s.block_nx[d] for d in reversed(range(s.ndim))], dtype=np.float64)
        _check(lib().orc_lohner_cells(self._h, int(leaf), out.ctypes.data, out.size))
        return out

    def face_flux(self, vl, vr, direction: int = 0) -> np.ndarray:
        """The scheme's Riemann flux across a face normal to `direction` for
        primitive face states vl, vr."""
        vl = np.ascontiguousarray(vl, dtype=np.float64)
        vr = np.ascontiguousarray(vr, dtype=np.float64)
        assert vl.shape == vr.shape == (self.nvar,)
        F = np.empty(self.nvar, dtype=np.float64)
        _check(lib().orc_face_flux(self._h, vl.ctypes.data, vr.ctypes.data, int(direction), F.ctypes.data))
        return F

    def face_kinds(self, leaf: int) -> np.ndarray:
        k = np.empty(2 * self.scheme.ndim, dtype=np.int32)
        _check(lib().orc_face_kinds(self._h, int(leaf), k.ctypes.data))
        return k


    def regrid_plan(self, flags) -> tuple:
        """(level [m], ijk [m, 3]) of the regridded forest for these flags."""
        flags = np.ascontiguousarray(flags, dtype=np.int8)
        assert flags.shape == (self.forest.n,)
        m = ctypes.c_int64()
        lib().orc_regrid_plan(self._h, flags.ctypes.data, 0, ctypes.byref(m), None, None)
        lev = np.empty(max(m.value, 1), dtype=np.int32)
        ijk = np.empty((max(m.value, 1), 3), dtype=np.int32)
        _check(lib().orc_regrid_plan(self._h, flags.ctypes.data, m.value, ctypes.byref(m), lev.ctypes.data,
                                     ijk.ctypes.data))
        return lev[:m.value], ijk[:m.value]

    def regrid(self, flags) -> "OracleForest":
        """A new oracle forest on the regridded leaves, holding the transferred state."""
        lev, ijk = self.regrid_plan(flags)
        g = OracleForest(type(self.forest)(self.scheme, lev, ijk))
        _check(lib().orc_regrid_transfer(self._h, g._h))
        return g

    def transfer_to(self, other: "OracleForest"):
        """Move this forest's state onto `other` (a one-level regrid of it)."""
        _check(lib().orc_regrid_transfer(self._h, other._h))


def courant_factor(n: int, nramp: int) -> float:
    """The reduced Courant step of the MHD blast's start (Sec. 2.4: the
    first 10 steps are lowered gradually; the paper gives no formula).
    Reading: step n (from 0) of the first nramp steps takes the fraction
    (n + 1) / nramp of the Courant step, later steps all of it."""
    if nramp > 0 and n < nramp:
        return (n + 1) / nramp
    return 1.0


def run(forest, U0: np.ndarray, *, t_end: float | None = None, steps: int | None = None,
        dts=None, ramp_steps: int = 0):
    """Drive the oracle: free Courant steps to t_end, a fixed step count, or a
    given dt sequence (lockstep runs); ramp_steps > 0 scales the Courant step
    of the first steps by courant_factor.  Returns (state, dts used)."""
    o = OracleForest(forest)
    o.set_state(U0)
    used = []
    if dts is not None:
        for dt in dts:
            o.max_dt()
            o.advance(dt)
            used.append(dt)
    else:
        t = 0.0
        n = 0
        while True:
            if steps is not None and n >= steps:
                break
            dt = o.max_dt() * courant_factor(n, ramp_steps)
            if t_end is not None:
                if t >= t_end:
                    break
                dt = min(dt, t_end - t)
            o.advance(dt)
            used.append(dt)
            t += dt
            n += 1
    U = o.get_state()
    o.close()
    return U, used
