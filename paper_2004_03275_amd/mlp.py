"""Learned refinement flagger: data from the solver, training on the GPU.

The paper flags blocks with the Loehner estimator (Sec. 1.3): refine where
the block maximum exceeds the tolerance, coarsen where it lies below a
fraction of it.  The learned flagger predicts both decisions from 128 pooled
features per leaf with a 128-64-64-2 perceptron (a refine and a coarsen
logit) whose forward and backward passes are the library's bfloat16 MFMA
kernels (amrv_mlp_train, AMRV_FLAG_MLP); Loehner stays as the fallback for
low-confidence leaves and as the reference its disagreement rate is measured
against.
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


def labels(emax: np.ndarray, tol: float = 0.1, frac: float = 0.125) -> np.ndarray:
    """Loehner class of each block from its estimator maximum: +1 above tol,
    -1 below frac * tol, else 0 (the flag rule without its level limits)."""
    return np.where(emax > tol, 1.0, np.where(emax < frac * tol, -1.0, 0.0)).astype(np.float32)


def collect(forest, U0, steps, device="cuda:0"):
    """Features, Loehner block maxima and levels at several snapshots."""
    Xs, E, L = [], [], []
    for _, g in snapshots(forest, U0, steps, device):
        Xs.append(g.mlp_features())
        _, emax = g.flag_blocks(with_emax=True)
        E.append(emax)
        L.append(np.asarray(forest.level))
    return np.concatenate(Xs), np.concatenate(E), np.concatenate(L)


def blast_dataset(seeds, base=8, max_level=3, steps=(0, 4, 8, 14, 20, 28), coarse=False, device="cuda:0"):
    Xs, E, L = [], [], []
    for sd in seeds:
        f, U = W.jittered_blast(sd, base=base, max_level=max_level, coarse=coarse)
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
    """Adam training of the flagger on device-resident features and class labels
    (+1 refine, -1 coarsen, 0 keep)."""

    def __init__(self, X: np.ndarray, y: np.ndarray, *, batch=1024, seed=0, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, pos_weight=None, pos_weight_c=None, device="cuda:0"):
        self.dev = torch.device(device)
        self.n = int(X.shape[0])
        self.batch = int(batch)
        self.X = torch.from_numpy(np.ascontiguousarray(X).view(np.int16)).to(self.dev)
        self.y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(self.dev)
        npos = float(np.sum(y > 0.5))
        nneg = float(np.sum(y < -0.5))
        self.pos_weight = float(pos_weight) if pos_weight is not None else max(1.0, (self.n - npos) / max(npos, 1.0))
        self.pos_weight_c = (float(pos_weight_c) if pos_weight_c is not None
                             else max(0.05, (self.n - nneg) / max(nneg, 1.0)))
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
                          self.pos_weight, self.pos_weight_c, self.t)

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


def evaluate(w: np.ndarray, seeds, tol=0.1, frac=0.125, base=8, max_level=3, steps=(0, 6, 12, 20, 30), margin=None,
             coarse_steps=(0, 4, 8, 12), device="cuda:0"):
    """Agreement of the learned flagger with Loehner on held-out jittered
    blasts, over all three flag values: each seed on its refined forest at
    `steps` and on the uniform level-1 forest at `coarse_steps` (there the
    blast's blocks are below the top level, so Loehner raises +1 flags).
    flag_disagreement: fraction of leaves whose AMRV_FLAG_MLP flag (+1, 0 or
    -1) differs from AMRV_FLAG_LOHNER's; confusion[i][j]: leaves with Loehner
    flag i - 1 and network flag j - 1.  label_disagreement: the network's
    class (+1 where z_r > 0, else -1 where z_c > 0, else 0) against Loehner's
    class of the block maximum, on every leaf, level limits left out.
    refine_flags / coarsen_flags: Loehner's +1 and -1 counts.  With a margin,
    the same flag comparison for AMRV_FLAG_MLP_FALLBACK and the fraction of
    leaves that fell back to Loehner."""
    tot = dis_flag = dis_label = dis_fb = unc = nref = ncoa = 0
    conf = np.zeros((3, 3), dtype=np.int64)
    runs = [(sd, False, steps) for sd in seeds] + [(sd, True, coarse_steps) for sd in seeds]
    for sd, coarse, stp in runs:
        f, U = W.jittered_blast(sd, base=base, max_level=max_level, coarse=coarse)
        for _, g in snapshots(f, U, stp, device):
            g.mlp_set_weights(w)
            fl, emax = g.flag_blocks(with_emax=True)
            fm = g.flag_blocks(mode=N.FLAG_MLP)
            z = g.mlp_logits()
            pred = np.where(z[:, 0] > 0, 1, np.where(z[:, 1] > 0, -1, 0))
            dis_flag += int(np.sum(fm != fl))
            np.add.at(conf, (fl.astype(np.int64) + 1, fm.astype(np.int64) + 1), 1)
            dis_label += int(np.sum(pred != labels(emax, tol, frac)))
            nref += int(np.sum(fl == 1))
            ncoa += int(np.sum(fl == -1))
            tot += f.n
            if margin is not None:
                g.mlp_set_margin(margin)
                ff = g.flag_blocks(mode=N.FLAG_MLP_FALLBACK)
                dis_fb += int(np.sum(ff != fl))
                unc += int(np.sum((np.abs(z[:, 0]) < margin) | (np.abs(z[:, 1]) < margin)))
    out = {"leaves": tot, "refine_flags": nref, "coarsen_flags": ncoa, "flag_disagreement": dis_flag / tot,
           "label_disagreement": dis_label / tot, "confusion": conf.tolist()}
    if margin is not None:
        out.update({"fallback_flag_disagreement": dis_fb / tot, "fallback_fraction": unc / tot, "margin": margin})
    return out


C4_STEPS = (0, 5, 10, 15, 20, 25)


def flags_from_logits(z: np.ndarray, level: np.ndarray, max_level, dr: float = 0.0, dc: float = 0.0):
    """The flag rule of AMRV_FLAG_MLP on logits shifted by (dr, dc)."""
    zr, zc = z[:, 0] - dr, z[:, 1] - dc
    return np.where((zr > 0) & (level < max_level), 1, np.where(~(zr > 0) & (zc > 0) & (level > 1), -1, 0))


def calibrate(w: np.ndarray, seeds, base=8, max_level=3, steps=(0, 4, 8, 14, 20, 28), coarse_steps=(0, 3, 6, 10, 14),
              device="cuda:0", grid=np.arange(-4.0, 4.0001, 0.05), max_fallback=0.05, c4_seeds=()):
    """Decision thresholds of the two outputs, fitted on training seeds: the
    shifts (dr, dc) of the refine and coarsen logits that minimise the flag
    disagreement with Loehner over the seeds' snapshots (refined and level-1
    forests), folded into the output biases, and the fallback margin that
    sends max_fallback of those leaves to Loehner.  Returns (weights, dr, dc,
    disagreement before, after, margin)."""
    Z, FL, LV, MX = [], [], [], []
    runs = [(sd, False, steps, base, max_level) for sd in seeds] + \
        [(sd, True, coarse_steps, base, max_level) for sd in seeds] + [(sd, False, C4_STEPS, 16, 4) for sd in c4_seeds]
    for sd, coarse, stp, bs, ml in runs:
        f, U = W.jittered_blast(sd, base=bs, max_level=ml, coarse=coarse)
        for _, g in snapshots(f, U, stp, device):
            g.mlp_set_weights(w)
            FL.append(g.flag_blocks())
            g.flag_blocks(mode=N.FLAG_MLP)
            Z.append(g.mlp_logits())
            LV.append(np.asarray(f.level))
            MX.append(np.full(f.n, ml))
    Z, FL, LV, MX = np.concatenate(Z), np.concatenate(FL), np.concatenate(LV), np.concatenate(MX)
    before = float(np.mean(flags_from_logits(Z, LV, MX) != FL))
    best = (before, 0.0, 0.0)
    # the refine threshold first (the coarsen flag depends on it), then the coarsen one
    for dr in grid:
        d = float(np.mean(flags_from_logits(Z, LV, MX, dr, 0.0) != FL))
        if d < best[0] - 1e-12:
            best = (d, float(dr), 0.0)
    dr = best[1]
    for dc in grid:
        d = float(np.mean(flags_from_logits(Z, LV, MX, dr, dc) != FL))
        if d < best[0] - 1e-12:
            best = (d, dr, float(dc))
    _, dr, dc = best
    w2 = np.array(w, dtype=np.float32, copy=True)
    w2[N.MLP_NPARAM - 2] -= np.float32(dr)
    w2[N.MLP_NPARAM - 1] -= np.float32(dc)
    # the fallback margin: the largest one that sends at most max_fallback of
    # the calibration leaves to Loehner
    zs = np.stack([Z[:, 0] - dr, Z[:, 1] - dc], axis=1)
    near = np.minimum(np.abs(zs[:, 0]), np.abs(zs[:, 1]))
    margin = float(np.quantile(near, max_fallback)) if len(near) else 0.0
    return w2, dr, dc, before, best[0], margin


DATA_WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__file__), "data", "flagger_weights.npy")


def trained_weights() -> np.ndarray:
    """The flagger weights trained by `python -m paper_2004_03275_amd.mlp --save`
    (binary32, 12,546 values: the output biases include the calibrated
    decision thresholds)."""
    w = np.load(DATA_WEIGHTS, allow_pickle=False)
    if w.shape != (N.MLP_NPARAM,) or w.dtype != np.float32:
        raise ValueError("unexpected flagger weight file")
    return w


def trained_margin() -> float:
    """The fallback margin fitted with the committed weights (flagger_record.json)."""
    import json
    import os

    with open(os.path.join(os.path.dirname(DATA_WEIGHTS), "flagger_record.json")) as fh:
        return float(json.load(fh)["margin"])


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
    ap.add_argument("--blast-seeds", default="1-48")
    ap.add_argument("--kh-seeds", default="1-8")
    ap.add_argument("--test-seeds", default="101-103")
    ap.add_argument("--calib-seeds", default="1-12", help="training seeds the decision thresholds are fitted on")
    ap.add_argument("--c4-seeds", default="",
                    help="also train and calibrate on blasts on 16^3-base, 4-level forests (the 3D AMR blast's size)")
    ap.add_argument("--c4-test-seed", type=int, default=101)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--margin", type=float, default=None, help="fallback margin (default: fitted in calibration)")
    ap.add_argument("--tol", type=float, default=0.1)
    ap.add_argument("--out", default=None, help="write the weights and the training record (.npz)")
    ap.add_argument("--save", action="store_true", help="store the weights as the package's trained flagger")
    args = ap.parse_args(argv)

    def log(m):
        print(f"[flagger] {m}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    X1, e1, l1 = blast_dataset(_seeds(args.blast_seeds))
    X0, e0, l0 = blast_dataset(_seeds(args.blast_seeds), steps=(0, 3, 6, 10, 14), coarse=True)
    parts = [(X1, e1, l1), (X0, e0, l0)]
    if args.c4_seeds:
        parts.append(blast_dataset(_seeds(args.c4_seeds), base=16, max_level=4, steps=C4_STEPS))
    X1, e1, l1 = (np.concatenate([p[i] for p in parts]) for i in range(3))
    log(f"blast data (refined, level-1 and 16^3-base forests): {len(e1)} leaves ({time.perf_counter() - t0:.1f} s)")
    X2, e2, l2 = kh_dataset(_seeds(args.kh_seeds))
    log(f"kh data: {len(e2)} leaves ({time.perf_counter() - t0:.1f} s)")
    X = np.concatenate([X1, X2])
    y = labels(np.concatenate([e1, e2]), args.tol)
    log(f"dataset: {len(y)} samples, {int(np.sum(y > 0))} refine and {int(np.sum(y < 0))} coarsen labels")
    tr = Trainer(X, y, batch=args.batch, seed=args.seed, lr=args.lr)
    t1 = time.perf_counter()
    hist = tr.fit(args.epochs, log)
    train_s = time.perf_counter() - t1
    w0 = tr.weights()
    w, dr, dc, d0, d1, margin = calibrate(w0, _seeds(args.calib_seeds), c4_seeds=_seeds(args.c4_seeds))
    log(f"calibration on seeds {args.calib_seeds}: logit shifts refine {dr:+.2f}, coarsen {dc:+.2f}; "
        f"flag disagreement {d0:.4f} -> {d1:.4f}; fallback margin {margin:.3f}")
    res = evaluate(w, _seeds(args.test_seeds), tol=args.tol, margin=margin if args.margin is None else args.margin)
    res_c4 = evaluate(w, [args.c4_test_seed], tol=args.tol, base=16, max_level=4, steps=C4_STEPS, coarse_steps=(),
                      margin=margin if args.margin is None else args.margin)
    res["c4_size"] = res_c4
    rec = {"samples": int(len(y)), "refine_labels": int(np.sum(y > 0)), "coarsen_labels": int(np.sum(y < 0)),
           "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "train_seconds": train_s,
           "final_loss": hist[-1], "pos_weight": tr.pos_weight, "pos_weight_c": tr.pos_weight_c,
           "calibration": {"seeds": args.calib_seeds, "refine_shift": dr, "coarsen_shift": dc,
                           "disagreement_before": d0, "disagreement_after": d1, "margin": margin},
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
