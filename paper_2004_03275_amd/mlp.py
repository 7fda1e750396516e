"""Learned refinement flagger: data from the solver, training on the GPU.

The paper flags blocks with the Loehner estimator (Sec. 1.3).  The learned
flagger predicts the same refine decision (block maximum of the estimator
above the tolerance) from 128 pooled features per leaf with a 128-64-64-1
perceptron whose forward and backward passes are the library's bfloat16 MFMA
kernels (amrv_mlp_train, AMRV_FLAG_MLP); Loehner stays as the fallback for
low-confidence leaves and as the judge of the disagreement rate.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _native as N
from . import workloads as W
from .forest import GpuForest


def snapshots(forest, U0, steps, device="cuda:0"):
    """Run the solver from U0 and yield (step, GpuForest) at the given step
    counts (Courant time steps)."""
    g = GpuForest(forest, device=device)
    g.set_state(U0)
    done = 0
    for target in sorted(steps):
        while done < target:
            g.advance(g.max_dt())
            done += 1
        yield done, g
    g.close()


def collect(forest, U0, steps, device="cuda:0"):
    """Features, Loehner block maxima and levels at several snapshots."""
    Xs, E, L = [], [], []
    for _, g in snapshots(forest, U0, steps, device):
        Xs.append(g.mlp_features())
        _, emax = g.flag_blocks(with_emax=True)
        E.append(emax)
        L.append(np.asarray(forest.level))
    return np.concatenate(Xs), np.concatenate(E), np.concatenate(L)


def blast_dataset(seeds, base=8, max_level=3, steps=(0, 4, 8, 14, 20, 28), device="cuda:0"):
    Xs, E, L = [], [], []
    for sd in seeds:
        f, U = W.jittered_blast(sd, base=base, max_level=max_level)
        X, e, l = collect(f, U, steps, device)
        Xs.append(X)
        E.append(e)
        L.append(l)
    return np.concatenate(Xs), np.concatenate(E), np.concatenate(L)


def kh_dataset(seeds, nblk=16, steps=(0, 100, 200, 300, 400), device="cuda:0"):
    Xs, E, L = [], [], []
    for sd in seeds:
        s = W.kh_scheme(nblk)
        s.max_level = 2
        f, U = W.kh(scheme=s, seed=sd, amplitude=0.05)
        X, e, l = collect(f, U, steps, device)
        Xs.append(X)
        E.append(e)
        L.append(l)
    return np.concatenate(Xs), np.concatenate(E), np.concatenate(L)


class Trainer:
    """Adam training of the flagger on device-resident features and labels."""

    def __init__(self, X: np.ndarray, y: np.ndarray, *, batch=1024, seed=0, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, pos_weight=None, device="cuda:0"):
        self.dev = torch.device(device)
        self.n = int(X.shape[0])
        self.batch = int(batch)
        self.X = torch.from_numpy(np.ascontiguousarray(X).view(np.int16)).to(self.dev)
        self.y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(self.dev)
        npos = float(np.sum(y > 0.5))
        self.pos_weight = float(pos_weight) if pos_weight is not None else max(1.0, (self.n - npos) / max(npos, 1.0))
        self.w = torch.from_numpy(W.mlp_init(seed)).to(self.dev)
        self.m = torch.zeros(N.MLP_NPARAM, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros_like(self.m)
        self.hyper = dict(lr=lr, beta1=beta1, beta2=beta2, eps=eps)
        self.t = 0
        nbytes = N.lib().amrv_mlp_train_workspace_bytes(self.batch)
        if nbytes == 0:
            raise N.AmrvError(N.EINVAL, N.lib().amrv_last_error().decode())
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.dev)
        self.stream = torch.cuda.Stream(device=self.dev)
        self.nb = (self.n + self.batch - 1) // self.batch
        self.loss = torch.zeros(self.nb, dtype=torch.float32, device=self.dev)
        self.seed = seed

    def _cfg(self):
        return N.TrainCfg(self.hyper["lr"], self.hyper["beta1"], self.hyper["beta2"], self.hyper["eps"],
                          self.pos_weight, self.t)

    def epoch(self, e: int) -> float:
        order = np.random.default_rng(self.seed * 1000 + e).permutation(self.n).astype(np.int32)
        od = torch.from_numpy(order).to(self.dev)
        cfg = self._cfg()
        torch.cuda.current_stream(self.dev).synchronize()
        N.check(N.lib().amrv_mlp_train(
            ctypes.c_void_p(self.X.data_ptr()), ctypes.c_void_p(self.y.data_ptr()), ctypes.c_void_p(od.data_ptr()),
            self.n, self.batch, 0, self.nb, ctypes.c_void_p(self.w.data_ptr()), ctypes.c_void_p(self.m.data_ptr()),
            ctypes.c_void_p(self.v.data_ptr()), ctypes.byref(cfg), ctypes.c_void_p(self.ws.data_ptr()),
            self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream), ctypes.c_void_p(self.loss.data_ptr()), None))
        self.stream.synchronize()
        self.t += self.nb
        return float(self.loss.mean().item())

    def fit(self, epochs: int, log=None):
        hist = []
        t0 = time.perf_counter()
        for e in range(epochs):
            L = self.epoch(e)
            hist.append(L)
            if log:
                log(f"epoch {e}: loss {L:.4f} ({time.perf_counter() - t0:.1f} s)")
        return hist

    def weights(self) -> np.ndarray:
        return self.w.detach().cpu().numpy().copy()


def evaluate(w: np.ndarray, seeds, tol=0.1, base=8, max_level=3, steps=(0, 6, 12, 20, 30), margin=None,
             device="cuda:0"):
    """Disagreement of the learned refine decision with Loehner's on held-out
    jittered blasts: fraction of leaves where [logit > 0] != [Loehner max > tol]
    (and, with a margin, of the fallback flags against the Loehner flags)."""
    tot = dis = dis_fb = unc = 0
    for sd in seeds:
        f, U = W.jittered_blast(sd, base=base, max_level=max_level)
        for _, g in snapshots(f, U, steps, device):
            g.mlp_set_weights(w)
            fl, emax = g.flag_blocks(with_emax=True)
            fm, z = g.flag_blocks(with_emax=True, mode=N.FLAG_MLP)
            dis += int(np.sum((z > 0) != (emax > tol)))
            tot += f.n
            if margin is not None:
                g.mlp_set_margin(margin)
                ff = g.flag_blocks(mode=N.FLAG_MLP_FALLBACK)
                # the fallback agrees with Loehner's refine decision where used
                dis_fb += int(np.sum((ff == 1) != (fl == 1)))
                unc += int(np.sum(np.abs(z) < margin))
    out = {"leaves": tot, "disagreement": dis / tot}
    if margin is not None:
        out.update({"fallback_disagreement": dis_fb / tot, "fallback_fraction": unc / tot, "margin": margin})
    return out
