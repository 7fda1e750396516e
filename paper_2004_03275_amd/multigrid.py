"""Python face of libamrv's multigrid Helmholtz solver and reaction-diffusion
steps (include/amrv_mg.h): argument marshalling only; every step runs in the
HIP kernels.  Fields are float64 device tensors of shape [n]*ndim (index
[z][y][x], x fastest)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N

PERIODIC, NEUMANN = 0, 1
SCHNAKENBERG, GRAY_SCOTT = 0, 1
EULER, MIDPOINT, SPLIT, IMEX = 0, 1, 2, 3
TILED, PER_COLOUR = 0, 1


def rd_params(model: int, Du: float, Dv: float, p1: float, p2: float, p3: float = 0.0) -> N.RdParams:
    return N.RdParams(model=model, pad=0, Du=Du, Dv=Dv, p1=p1, p2=p2, p3=p3)


class GpuMultigrid:
    """A solver for one grid shape on one GPU (workspace from torch).
    graph=True replays each V-cycle from a captured HIP graph; for the few
    launches of a 2D cycle direct launches measured faster, so they are the
    default."""

    def __init__(self, ndim: int, n: int, bc: int, length: float, nfields: int = 2, pre: int = 2, post: int = 2,
                 graph: bool = False, smoother: int = TILED, device: str | torch.device = "cuda:0",
                 stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("GpuMultigrid needs a ROCm GPU (torch.cuda.is_available() is False)")
        L = N.lib()
        self.cfg = N.MgConfig(ndim=ndim, n=n, bc=bc, nfields=nfields, pre_sweeps=pre, post_sweeps=post,
                              use_graph=1 if graph else 0, smoother=smoother, length=length)
        nbytes = L.amrv_mg_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise N.AmrvError(N.EINVAL, L.amrv_last_error().decode())
        self.device = torch.device(device)
        self.ndim, self.n, self.nfields = ndim, n, nfields
        self.shape = (n,) * ndim
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        N.check(L.amrv_mg_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None):
            N.lib().amrv_mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t: torch.Tensor, count: int) -> torch.Tensor:
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("expected a contiguous float64 device tensor")
        if t.numel() != count:
            raise ValueError(f"expected {count} values, got {t.numel()}")
        return t

    def solve(self, f: torch.Tensor, phi: torch.Tensor, lam, tol: float = 1e-7, max_cycles: int = 50):
        """lap(phi) - lam phi = f for the nfields fields stacked in f and phi
        (phi: initial guess in, solution out).  Returns (cycles, max
        residual per field, max |f| per field)."""
        cells = self.n ** self.ndim
        self._dev(f, cells * self.nfields)
        self._dev(phi, cells * self.nfields)
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (self.nfields,)))
        cyc = ctypes.c_int32()
        res = np.zeros(self.nfields)
        fmax = np.zeros(self.nfields)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_mg_solve(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                      lam.ctypes.data, float(tol), int(max_cycles), ctypes.byref(cyc),
                                      res.ctypes.data, fmax.ctypes.data))
        return cyc.value, res, fmax

    def rd_step(self, u: torch.Tensor, v: torch.Tensor, dt: float, scheme: int, params: dict, nsteps: int = 1,
                tol: float = 1e-7, max_cycles: int = 50):
        """nsteps reaction-diffusion steps on u, v in place.  params: dict
        with model, Du, Dv, p1, p2, p3 (the oracle's parameter dicts).
        Returns (V-cycles summed over the steps, last residuals)."""
        cells = self.n ** self.ndim
        self._dev(u, cells)
        self._dev(v, cells)
        p = rd_params(int(params["model"]), params["Du"], params["Dv"], params["p1"], params["p2"],
                      params.get("p3", 0.0))
        cyc = ctypes.c_int32()
        res = np.zeros(2)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_rd_step(self._h, ctypes.byref(p), int(scheme), float(dt), int(nsteps),
                                     ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()), float(tol),
                                     int(max_cycles), ctypes.byref(cyc), res.ctypes.data))
        return cyc.value, res

    def set_coefficient(self, eps: torch.Tensor | None):
        """Solve div(eps grad phi) - lambda phi = f from now on (eps: float64
        device tensor of the grid's size, > 0), or return to eps = 1 (None)."""
        if eps is None:
            N.check(N.lib().amrv_mg_set_coefficient(self._h, None))
            self._eps = None
            return
        self._eps = self._dev(eps, self.n ** self.ndim)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_mg_set_coefficient(self._h, ctypes.c_void_p(eps.data_ptr())))

    def divb_project(self, B, tol: float = 1e-10, max_cycles: int = 50):
        """The divergence control of Sec. 2.4 on the ndim device arrays B
        (updated in place).  Returns (cycles, max |div B| before, after)."""
        cells = self.n ** self.ndim
        if len(B) != self.ndim:
            raise ValueError("one array per dimension")
        for b in B:
            self._dev(b, cells)
        ptr = [ctypes.c_void_p(b.data_ptr()) for b in B] + ([ctypes.c_void_p(0)] if self.ndim == 2 else [])
        cyc = ctypes.c_int32()
        before, after = ctypes.c_double(), ctypes.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_mg_divb_project(self._h, ptr[0], ptr[1], ptr[2], float(tol), int(max_cycles),
                                             ctypes.byref(cyc), ctypes.byref(before), ctypes.byref(after)))
        return cyc.value, before.value, after.value

    def profile(self, enable: bool = True):
        N.check(N.lib().amrv_mg_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(summed V-cycle ms, cycles) since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        N.check(N.lib().amrv_mg_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def fmg_config(forest, length: float, bc: int, pre: int = 2, post: int = 2) -> N.FmgConfig:
    """amrv_fmg_config of a 2D or 3D forest (workloads.Forest: 16^d blocks,
    base^d blocks at level 1)."""
    s = forest.scheme
    nd = s.ndim
    if nd not in (2, 3) or len(set(s.base_blocks[:nd])) != 1 or tuple(s.block_nx[:nd]) != (16,) * nd:
        raise ValueError("a 2D or 3D forest of 16^d blocks on a square / cubic base grid")
    return N.FmgConfig(nleaves=forest.n, base=s.base_blocks[0], max_level=s.max_level, bc=bc, pre_sweeps=pre,
                       post_sweeps=post, ndim=nd, length=length)


def fmg_workspace_bytes(forest, length: float, bc: int) -> int:
    """Workspace bytes of the forest solver (host only; raises AmrvError for a
    bad configuration or leaf list)."""
    L = N.lib()
    cfg = fmg_config(forest, length, bc)
    lev = np.ascontiguousarray(forest.level, dtype=np.int32)
    ijk = np.ascontiguousarray(forest.ijk, dtype=np.int32)
    nbytes = L.amrv_fmg_workspace_bytes(ctypes.byref(cfg), lev.ctypes.data, ijk.ctypes.data)
    if nbytes == 0:
        err = L.amrv_last_error().decode()
        raise N.AmrvError(N.EUNBALANCED if "balance" in err or "overlap" in err or "cover" in err or "gap" in err
                          else N.EINVAL, err)
    return int(nbytes)


class GpuForestMultigrid:
    """The Helmholtz solver on a 2D or 3D block-adaptive forest (amrv_fmg_*):
    fields are float64 device tensors of nleaves * 16^d values ([nleaves,
    (16,) 16, 16], the forest's layout of one variable)."""

    def __init__(self, forest, length: float, bc: int, pre: int = 2, post: int = 2,
                 device: str | torch.device = "cuda:0", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("GpuForestMultigrid needs a ROCm GPU (torch.cuda.is_available() is False)")
        L = N.lib()
        self.cfg = fmg_config(forest, length, bc, pre, post)
        lev = np.ascontiguousarray(forest.level, dtype=np.int32)
        ijk = np.ascontiguousarray(forest.ijk, dtype=np.int32)
        nbytes = fmg_workspace_bytes(forest, length, bc)
        self.device = torch.device(device)
        self.nleaves = forest.n
        self.ndim = forest.scheme.ndim
        self.ncb = 16 ** self.ndim
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        N.check(L.amrv_fmg_create(ctypes.byref(self.cfg), lev.ctypes.data, ijk.ctypes.data,
                                  ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None):
            N.lib().amrv_fmg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levels(self) -> list:
        out = np.zeros(16, dtype=np.int32)
        N.check(N.lib().amrv_fmg_levels(self._h, out.ctypes.data))
        return [int(v) for v in out if v]

    def solve(self, f: torch.Tensor, phi: torch.Tensor, lam: float, tol: float = 1e-10, max_cycles: int = 50):
        """lap(phi) - lam phi = f on the leaf cells (phi: initial guess in,
        solution out).  Returns (cycles, max residual, max |f|)."""
        for t in (f, phi):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("expected contiguous float64 device tensors")
            if t.numel() != self.nleaves * self.ncb:
                raise ValueError(f"expected {self.nleaves * self.ncb} values, got {t.numel()}")
        cyc = ctypes.c_int32()
        res, fmax = ctypes.c_double(), ctypes.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_fmg_solve(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                       float(lam), float(tol), int(max_cycles), ctypes.byref(cyc),
                                       ctypes.byref(res), ctypes.byref(fmax)))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return cyc.value, res.value, fmax.value

    def rd_step(self, u: torch.Tensor, v: torch.Tensor, dt: float, scheme: int, params: dict, nsteps: int = 1,
                tol: float = 1e-10, max_cycles: int = 50):
        """nsteps reaction-diffusion steps on the leaf fields u, v in place
        (params: dict with model, Du, Dv, p1, p2, p3).  Returns (V-cycles
        summed over the solves, largest final residual)."""
        for t in (u, v):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("expected contiguous float64 device tensors")
            if t.numel() != self.nleaves * self.ncb:
                raise ValueError(f"expected {self.nleaves * self.ncb} values, got {t.numel()}")
        p = rd_params(int(params["model"]), params["Du"], params["Dv"], params["p1"], params["p2"],
                      params.get("p3", 0.0))
        cyc = ctypes.c_int32()
        res = ctypes.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().amrv_fmg_rd_step(self._h, ctypes.byref(p), int(scheme), float(dt), int(nsteps),
                                         ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()), float(tol),
                                         int(max_cycles), ctypes.byref(cyc), ctypes.byref(res)))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return cyc.value, res.value

    def divb_project(self, *B: torch.Tensor, tol: float = 1e-10, max_cycles: int = 50):
        """The divergence control of Sec. 2.4 on the ndim leaf fields B
        (updated in place).  Returns (cycles, max |div B| before, after)."""
        if len(B) != self.ndim:
            raise ValueError(f"expected {self.ndim} field components, got {len(B)}")
        for t in B:
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("expected contiguous float64 device tensors")
            if t.numel() != self.nleaves * self.ncb:
                raise ValueError(f"expected {self.nleaves * self.ncb} values, got {t.numel()}")
        cyc = ctypes.c_int32()
        before, after = ctypes.c_double(), ctypes.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        ptr = [ctypes.c_void_p(t.data_ptr()) for t in B] + [None]
        N.check(N.lib().amrv_fmg_divb_project(self._h, ptr[0], ptr[1], ptr[2],
                                              float(tol), int(max_cycles), ctypes.byref(cyc), ctypes.byref(before),
                                              ctypes.byref(after)))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return cyc.value, before.value, after.value


def project_forest_b(g, fm: GpuForestMultigrid, ib: int, tol: float = 1e-10, max_cycles: int = 50):
    """The divergence control of Sec. 2.4 on a forest's state: B (state
    variables ib .. ib + ndim - 1, each a [leaf] + [16] * ndim field) projected in place by
    the forest solver fm built on the same leaves (g: forest.GpuForest).  The
    state moves device to device only.  Returns (cycles, max |div B| before,
    after)."""
    U = g.state_tensor()
    out = fm.divb_project(*[U[ib + d] for d in range(fm.ndim)], tol=tol, max_cycles=max_cycles)
    g.set_state(U)
    return out
