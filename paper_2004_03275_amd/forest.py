"""Python face of libamrv: a block forest whose state lives in HBM.

PyTorch supplies the device workspace (one uint8 tensor) and the stream; every
operation is a call through the C-ABI into the HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N


class GpuForest:
    """A forest on one GPU.  ``forest`` is a leaf list with its scheme (e.g.
    a workloads.Forest); ``stream`` a torch.cuda.Stream (a new one by default)."""

    def __init__(self, forest, device: str | torch.device = "cuda:0", stream: torch.cuda.Stream | None = None,
                 config: N.Config | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("GpuForest needs a ROCm GPU (torch.cuda.is_available() is False)")
        L = N.lib()
        self.forest = forest
        self.scheme = forest.scheme
        self.device = torch.device(device)
        self.cfg = config if config is not None else N.make_config(forest.scheme)
        self._lev = np.ascontiguousarray(forest.level, dtype=np.int32)
        self._ijk = np.ascontiguousarray(forest.ijk, dtype=np.int32)
        nbytes = L.amrv_workspace_bytes(ctypes.byref(self.cfg), forest.n, self._lev.ctypes.data,
                                        self._ijk.ctypes.data)
        if nbytes == 0:
            raise N.AmrvError(N.EINVAL, L.amrv_last_error().decode())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        N.check(L.amrv_forest_create(ctypes.byref(self.cfg), forest.n, self._lev.ctypes.data, self._ijk.ctypes.data,
                                     ctypes.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))
        self.nvar = L.amrv_nvar(self._h)
        self.shape = forest.state_shape()
        self.n_doubles = int(L.amrv_state_doubles(self._h))

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            N.lib().amrv_forest_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state --------------------------------------------------------------
    def set_state(self, U):
        if isinstance(U, torch.Tensor) and U.is_cuda:
            t = U.contiguous()
            if t.dtype != torch.float64 or t.numel() != self.n_doubles:
                raise ValueError("device state must be float64 with the forest's size")
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            N.check(N.lib().amrv_set_state(self._h, ctypes.c_void_p(t.data_ptr()), self.n_doubles, 1))
            self.synchronize()
            return
        U = np.ascontiguousarray(U, dtype=np.float64)
        if U.shape != tuple(self.shape):
            raise ValueError(f"state shape {U.shape} != {tuple(self.shape)}")
        N.check(N.lib().amrv_set_state(self._h, U.ctypes.data, U.size, 0))

    def get_state(self) -> np.ndarray:
        U = np.empty(self.shape, dtype=np.float64)
        N.check(N.lib().amrv_get_state(self._h, U.ctypes.data, U.size, 0))
        return U

    def state_tensor(self) -> torch.Tensor:
        """A device copy of the current state (float64, shape of the state)."""
        t = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        N.check(N.lib().amrv_get_state(self._h, ctypes.c_void_p(t.data_ptr()), self.n_doubles, 1))
        self.synchronize()
        return t

    # -- the method ---------------------------------------------------------
    def max_dt(self) -> float:
        dt = ctypes.c_double()
        N.check(N.lib().amrv_max_dt(self._h, ctypes.byref(dt)))
        return dt.value

    @property
    def glm_ch(self) -> float:
        return float(N.lib().amrv_glm_ch(self._h))

    def advance(self, dt: float):
        N.check(N.lib().amrv_advance(self._h, float(dt)))

    def advance_cfl(self, nsteps: int, t_end: float = float("inf"), t: float = 0.0):
        """nsteps steps with device-computed Courant time steps (no host
        synchronisation between them).  Returns (t after, steps taken)."""
        tt = ctypes.c_double(t)
        n = ctypes.c_int32()
        N.check(N.lib().amrv_advance_cfl(self._h, int(nsteps), float(t_end), ctypes.byref(tt), ctypes.byref(n)))
        return tt.value, n.value

    def regrid_plan(self, flags) -> tuple:
        """(level [m], ijk [m, 3]) of the regridded leaf list for these flags."""
        flags = np.ascontiguousarray(flags, dtype=np.int8)
        if flags.shape != (self.forest.n,):
            raise ValueError("one flag per leaf")
        # at most every leaf splits: one call with room for that
        cap = self.forest.n << self.scheme.ndim
        m = ctypes.c_int64()
        lev = np.empty(cap, dtype=np.int32)
        ijk = np.empty((cap, 3), dtype=np.int32)
        N.check(N.lib().amrv_regrid_plan(self._h, flags.ctypes.data, cap, ctypes.byref(m), lev.ctypes.data,
                                         ijk.ctypes.data))
        return lev[:m.value].copy(), ijk[:m.value].copy()

    def regrid(self, flags) -> "GpuForest":
        """A new forest on the regridded leaves (same device and stream,
        schedule and variant), holding this forest's transferred state."""
        lev, ijk = self.regrid_plan(flags)
        g = GpuForest(type(self.forest)(self.scheme, lev, ijk), device=self.device, stream=self.stream,
                      config=self.cfg)
        g.set_schedule(*self.get_schedule())
        g.set_variant(self.get_variant())
        N.check(N.lib().amrv_regrid_transfer(self._h, g._h))
        return g

    def transfer_to(self, other: "GpuForest"):
        """Move this forest's state onto `other` (a one-level regrid of it)."""
        N.check(N.lib().amrv_regrid_transfer(self._h, other._h))

    def flag_blocks(self, with_emax: bool = False, mode: int = N.FLAG_LOHNER):
        """Refinement flags (+1/0/-1).  with_emax also returns, per leaf, the
        Loehner maximum (LOHNER mode) or the learned flagger's logit (MLP
        modes; Loehner maximum on the fallback leaves)."""
        flags = np.empty(self.forest.n, dtype=np.int8)
        emax = np.empty(self.forest.n, dtype=np.float64) if with_emax else None
        N.check(N.lib().amrv_flag_blocks(self._h, int(mode), flags.ctypes.data,
                                         emax.ctypes.data if with_emax else None))
        return (flags, emax) if with_emax else flags

    # -- learned flagger ----------------------------------------------------
    def mlp_set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != N.MLP_NPARAM:
            raise ValueError(f"expected {N.MLP_NPARAM} parameters")
        N.check(N.lib().amrv_mlp_set_weights(self._h, w.ctypes.data, w.size))

    def mlp_set_margin(self, margin: float):
        N.check(N.lib().amrv_mlp_set_margin(self._h, float(margin)))

    def mlp_features(self, device: bool = False):
        """[n, 128] bfloat16 bit patterns of the current state (numpy uint16,
        or a device int16 tensor with the same bits if device=True)."""
        if device:
            t = torch.empty((self.forest.n, N.MLP_NIN), dtype=torch.int16, device=self.device)
            N.check(N.lib().amrv_mlp_features(self._h, ctypes.c_void_p(t.data_ptr()), 1))
            self.synchronize()
            return t
        X = np.empty((self.forest.n, N.MLP_NIN), dtype=np.uint16)
        N.check(N.lib().amrv_mlp_features(self._h, X.ctypes.data, 0))
        return X

    def mlp_fuse_features(self, enable: bool = True):
        """Pool the flagger's features in the last stage of every step."""
        N.check(N.lib().amrv_mlp_fuse_features(self._h, 1 if enable else 0))

    def mlp_logits(self) -> np.ndarray:
        """[n, 2] binary32 refine and coarsen logits of the last MLP flagging."""
        z = np.empty((self.forest.n, 2), dtype=np.float32)
        N.check(N.lib().amrv_mlp_logits(self._h, z.ctypes.data))
        return z

    # -- scheduling ---------------------------------------------------------
    def set_schedule(self, sched: int, xcd_remap: int = 1, persistent_wgs: int = 0):
        N.check(N.lib().amrv_set_schedule(self._h, int(sched), int(xcd_remap), int(persistent_wgs)))

    def get_schedule(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        N.check(N.lib().amrv_get_schedule(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_variant(self, variant: int):
        N.check(N.lib().amrv_set_variant(self._h, int(variant)))

    def get_variant(self) -> int:
        v = ctypes.c_int32()
        N.check(N.lib().amrv_get_variant(self._h, ctypes.byref(v)))
        return v.value

    def set_arithmetic(self, mode: int):
        """N.ARITH_EXACT (bit-for-bit with the oracle) or N.ARITH_FAST."""
        N.check(N.lib().amrv_set_arithmetic(self._h, int(mode)))

    def get_arithmetic(self) -> int:
        v = ctypes.c_int32()
        N.check(N.lib().amrv_get_arithmetic(self._h, ctypes.byref(v)))
        return v.value

    def autotune(self, reps: int = 3):
        """Pick the fastest schedule and stage-kernel variant; returns
        (schedule, xcd_remap, persistent_wgs, variant)."""
        N.check(N.lib().amrv_autotune(self._h, int(reps)))
        return (*self.get_schedule(), self.get_variant())

    def autotune_report(self) -> str:
        return N.lib().amrv_autotune_report(self._h).decode()

    def use_graph(self, enable: bool = True):
        N.check(N.lib().amrv_use_graph(self._h, 1 if enable else 0))

    def profile(self, enable: bool = True):
        N.check(N.lib().amrv_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(summed stage-kernel ms, launches, algorithmic bytes) since the last read."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        N.check(N.lib().amrv_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def grid_shape(self) -> tuple:
        """[z][y][x] extents of the uniform grid the leaves tile (uniform forests)."""
        s = self.scheme
        lev = int(self.forest.level[0])
        ext = [s.base_blocks[d] * (1 << (lev - 1)) * s.block_nx[d] for d in range(s.ndim)]
        return tuple(reversed(ext))

    def to_grid(self, var: int) -> torch.Tensor:
        """State variable var of a uniform forest as a device grid array."""
        t = torch.empty(self.grid_shape(), dtype=torch.float64, device=self.device)
        N.check(N.lib().amrv_uniform_grid_copy(self._h, int(var), ctypes.c_void_p(t.data_ptr()), 1))
        return t

    def from_grid(self, var: int, grid: torch.Tensor):
        """Write state variable var of a uniform forest from a device grid array."""
        if not (grid.is_cuda and grid.dtype == torch.float64 and grid.is_contiguous()
                and tuple(grid.shape) == self.grid_shape()):
            raise ValueError(f"expected a contiguous float64 device tensor of shape {self.grid_shape()}")
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_uniform_grid_copy(self._h, int(var), ctypes.c_void_p(grid.data_ptr()), 0))

    def synchronize(self):
        N.check(N.lib().amrv_synchronize(self._h))


def courant_ramp(step: int, ramp_steps: int) -> float:
    """Factor on the Courant time step of step ``step`` (counted from 0):
    the paper lowers the first 10 time steps of its MHD blast gradually
    (Sec. 2.4) without a formula; read as the linear ramp (step + 1) /
    ramp_steps over the first ramp_steps steps, 1 after them."""
    if ramp_steps <= 0 or step >= ramp_steps:
        return 1.0
    return (step + 1) / ramp_steps


def run(forest, U0, *, t_end=None, steps=None, dts=None, schedule=None, graph=False, device="cuda:0",
        variant=None, device_dt=False, chunk=50, ramp_steps=0, arithmetic=None):
    """Drive the GPU forest like oracle.run: free Courant steps to t_end, a
    fixed step count, or a given dt sequence; ramp_steps > 0 scales the first
    Courant steps by courant_ramp (host-chosen steps only).
    Returns (state, dts used)."""
    g = GpuForest(forest, device=device)
    if arithmetic is not None:
        g.set_arithmetic(arithmetic)
    if schedule is not None:
        g.set_schedule(*schedule)
    if variant is not None:
        g.set_variant(variant)
    if graph:
        g.use_graph(True)
    g.set_state(U0)
    used = []
    if device_dt:
        if dts is not None or ramp_steps:
            raise ValueError("device_dt runs choose their own time steps (no ramp)")
        t, n = 0.0, 0
        tend = float("inf") if t_end is None else float(t_end)
        while True:
            k = chunk if steps is None else min(chunk, steps - n)
            if k <= 0:
                break
            t, taken = g.advance_cfl(k, tend, t)
            n += taken
            if taken < k:
                break
        U = g.get_state()
        g.close()
        return U, [None] * n
    if dts is not None:
        for dt in dts:
            g.max_dt()
            g.advance(dt)
            used.append(dt)
    else:
        t, n = 0.0, 0
        while True:
            if steps is not None and n >= steps:
                break
            dt = g.max_dt() * courant_ramp(n, ramp_steps)
            if t_end is not None:
                if t >= t_end:
                    break
                dt = min(dt, t_end - t)
            g.advance(dt)
            used.append(dt)
            t += dt
            n += 1
    U = g.get_state()
    g.close()
    return U, used
