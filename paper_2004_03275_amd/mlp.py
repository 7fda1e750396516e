"""Learned refinement flagger: data from the solver, training on the GPU.

The paper flags blocks with the Loehner estimator (Sec. 1.3).  The learned
flagger predicts the same refine decision (block maximum of the estimator
above the tolerance) from 128 pooled features per leaf with a 128-64-64-1
perceptron whose forward and backward passes are the library's bfloat16 MFMA
kernels (amrv_mlp_train, AMRV_FLAG_MLP); Loehner stays as the fallback for
low-confidence leaves and as the reference its disagreement rate is measured against.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _native as N
import workloads as W
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
    """Agreement of the learned flagger with Loehner on held-out jittered
    blasts.  flag_disagreement: fraction of leaves whose refine flag (+1)
    differs between AMRV_FLAG_MLP and AMRV_FLAG_LOHNER (the flags that drive
    refinement; neither refines a finest-level leaf).  label_disagreement:
    [logit > 0] against [Loehner max > tol] on every leaf, finest level
    included.  With a margin, the same for AMRV_FLAG_MLP_FALLBACK and the
    fraction of leaves that fell back to Loehner."""
    tot = dis_flag = dis_label = dis_fb = unc = 0
    for sd in seeds:
        f, U = W.jittered_blast(sd, base=base, max_level=max_level)
        for _, g in snapshots(f, U, steps, device):
            g.mlp_set_weights(w)
            fl, emax = g.flag_blocks(with_emax=True)
            fm, z = g.flag_blocks(with_emax=True, mode=N.FLAG_MLP)
            dis_flag += int(np.sum((fm == 1) != (fl == 1)))
            dis_label += int(np.sum((z > 0) != (emax > tol)))
            tot += f.n
            if margin is not None:
                g.mlp_set_margin(margin)
                ff = g.flag_blocks(mode=N.FLAG_MLP_FALLBACK)
                dis_fb += int(np.sum((ff == 1) != (fl == 1)))
                unc += int(np.sum(np.abs(z) < margin))
    out = {"leaves": tot, "flag_disagreement": dis_flag / tot, "label_disagreement": dis_label / tot}
    if margin is not None:
        out.update({"fallback_flag_disagreement": dis_fb / tot, "fallback_fraction": unc / tot, "margin": margin})
    return out


DATA_WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__file__), "data", "flagger_weights.npy")


def trained_weights() -> np.ndarray:
    """The flagger weights trained by `python -m paper_2004_03275_amd.mlp --save`
    (binary32, 12,481 values)."""
    w = np.load(DATA_WEIGHTS, allow_pickle=False)
    if w.shape != (N.MLP_NPARAM,) or w.dtype != np.float32:
        raise ValueError("unexpected flagger weight file")
    return w


def _seeds(spec: str):
    out = []
    for part in spec.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        elif part:
            out.append(int(part))
    return out


def main(argv=None):
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="train the learned refinement flagger on solver data")
    ap.add_argument("--blast-seeds", default="1-24")
    ap.add_argument("--kh-seeds", default="1-8")
    ap.add_argument("--test-seeds", default="101-103")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--margin", type=float, default=2.0)
    ap.add_argument("--tol", type=float, default=0.1)
    ap.add_argument("--out", default=None, help="write the weights and the training record (.npz)")
    ap.add_argument("--save", action="store_true", help="store the weights as the package's trained flagger")
    args = ap.parse_args(argv)

    def log(m):
        print(f"[flagger] {m}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    X1, e1, l1 = blast_dataset(_seeds(args.blast_seeds))
    log(f"blast data: {len(e1)} leaves ({time.perf_counter() - t0:.1f} s)")
    X2, e2, l2 = kh_dataset(_seeds(args.kh_seeds))
    log(f"kh data: {len(e2)} leaves ({time.perf_counter() - t0:.1f} s)")
    X = np.concatenate([X1, X2])
    y = (np.concatenate([e1, e2]) > args.tol).astype(np.float32)
    log(f"dataset: {len(y)} samples, {int(y.sum())} refine labels")
    tr = Trainer(X, y, batch=args.batch, seed=args.seed, lr=args.lr)
    t1 = time.perf_counter()
    hist = tr.fit(args.epochs, log)
    train_s = time.perf_counter() - t1
    w = tr.weights()
    res = evaluate(w, _seeds(args.test_seeds), tol=args.tol, margin=args.margin)
    rec = {"samples": int(len(y)), "positives": int(y.sum()), "epochs": args.epochs, "batch": args.batch,
           "lr": args.lr, "train_seconds": train_s, "final_loss": hist[-1], "pos_weight": tr.pos_weight,
           "steps": tr.t, "samples_per_s": len(y) * args.epochs / train_s, **res}
    log(json.dumps(rec))
    if args.out:
        np.savez(args.out, weights=w, loss=np.array(hist), record=json.dumps(rec))
    if args.save:
        import os

        os.makedirs(os.path.dirname(DATA_WEIGHTS), exist_ok=True)
        np.save(DATA_WEIGHTS, w)
        with open(os.path.join(os.path.dirname(DATA_WEIGHTS), "flagger_record.json"), "w") as fh:
            fh.write(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec), flush=True)
    return rec


if __name__ == "__main__":
    main()
