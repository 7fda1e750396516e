"""CPU reference of the learned refinement flagger.

TEST INFRASTRUCTURE ONLY (tests/, smoke, bench's CPU leg).  The paper refines
blocks with the Loehner estimator (Sec. 1.3); the learned flagger is not
in the paper: a 128-64-64-2 multilayer perceptron that predicts, from pooled
block features, whether Loehner's block maximum exceeds the refinement
tolerance (output 0) and whether it lies below the coarsening fraction of it
(output 1).  This module is written from the definitions below, not from the
HIP code, and shares nothing with it.

Features of a leaf (3D, 16^3 cells): the means of rho and of p over the 64
sub-blocks of 4^3 cells (sub-block index bx + 4 by + 16 bz; cells summed in
order z, y, x inside a sub-block, binary64), each divided by the leaf's mean
of the 64 sub-block means (summed in sub-block order) minus one, rounded to
binary32 and then to bfloat16 (round to nearest even).  2D leaves (16^2) use
8^2 sub-blocks of 2^2 cells.  Feature order: the 64 rho features, then the 64
p features.  p follows the solver's primitive conversion
p = (gamma-1) ((E - (0.5 m.m) (1/rho)) [- 0.5 B.B]).

Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3 (two
logits).  Parameter vector (12,546 binary32): W1 [64][128], b1 [64],
W2 [64][64], b2 [64], W3 [2][64], b3 [2].  Labels are Loehner's classes
(+1 refine, -1 coarsen, 0 keep); the targets are y_r = [label = +1] for
output 0 and y_c = [label = -1] for output 1.  Loss: mean over the batch of
the sum of both outputs' class-weighted binary cross-entropies with logits,
-(pw y log s(z) + (1-y) log(1-s(z))), with weights pw_r and pw_c.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 128, 64, 2
NPARAM = NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT  # 12,546

# ---------------------------------------------------------------------------
# bfloat16
# ---------------------------------------------------------------------------


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns, round to nearest even (NaN kept NaN)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    nan = np.isnan(x)
    out = rounded.astype(np.uint16)
    out[nan] = 0x7FC0
    return out


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> binary32 values."""
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round binary32 values to bfloat16 and return them as binary32."""
    return bf16_value(bf16_bits(x))


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------


def _pressure(U: np.ndarray, ndim: int, gamma: float, mhd: bool, cad=None) -> np.ndarray:
    rho = U[0]
    if cad is not None:  # polytrope: c_ad rho^gamma (rho^1, rho^2 exact)
        e = rho if gamma == 1.0 else rho * rho if gamma == 2.0 else np.power(rho, gamma)
        return cad * e
    inv = 1.0 / rho
    mm = U[1] * U[1]
    for d in range(1, ndim):
        mm = mm + U[1 + d] * U[1 + d]
    if not mhd:
        return (gamma - 1.0) * (U[1 + ndim] - 0.5 * mm * inv)
    bb = U[2 + ndim] * U[2 + ndim]
    for d in range(1, ndim):
        bb = bb + U[2 + ndim + d] * U[2 + ndim + d]
    return (gamma - 1.0) * (U[1 + ndim] - 0.5 * mm * inv - 0.5 * bb)


def _pool(q: np.ndarray, ndim: int) -> np.ndarray:
    """64 sub-block means of one leaf's field, summed in the fixed order."""
    out = np.empty(64, dtype=np.float64)
    if ndim == 3:
        for bz in range(4):
            for by in range(4):
                for bx in range(4):
                    s = 0.0
                    for k in range(4):
                        for j in range(4):
                            for i in range(4):
                                s = s + float(q[4 * bz + k, 4 * by + j, 4 * bx + i])
                    out[bx + 4 * by + 16 * bz] = s / 64.0
    else:
        for by in range(8):
            for bx in range(8):
                s = 0.0
                for j in range(2):
                    for i in range(2):
                        s = s + float(q[2 * by + j, 2 * bx + i])
                out[bx + 8 * by] = s / 4.0
    return out


def leaf_features(U_leaf: np.ndarray, ndim: int, gamma: float, mhd: bool = False, cad=None) -> np.ndarray:
    """bfloat16 bit patterns [128] of one leaf's conserved state [nvar, (nz,) ny, nx]
    (``cad`` given: the polytrope's state)."""
    rho = U_leaf[0]
    p = _pressure(U_leaf, ndim, gamma, mhd, cad)
    feats = np.empty(NIN, dtype=np.float32)
    for v, q in enumerate((rho, p)):
        means = _pool(q, ndim)
        m = 0.0
        for x in means:
            m = m + float(x)
        m = m / 64.0
        for i in range(64):
            feats[64 * v + i] = np.float32(means[i] / m - 1.0)
    return bf16_bits(feats)


def features(U: np.ndarray, ndim: int, gamma: float, mhd: bool = False, leaves=None, cad=None) -> np.ndarray:
    """[n, 128] bfloat16 bit patterns for the leaves of a state [nvar, n, ...]."""
    idx = range(U.shape[1]) if leaves is None else leaves
    return np.stack([leaf_features(U[:, b], ndim, gamma, mhd, cad) for b in idx])


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------


def unpack(params: np.ndarray):
    p = np.asarray(params)
    o = 0
    W1 = p[o:o + NH * NIN].reshape(NH, NIN)
    o += NH * NIN
    b1 = p[o:o + NH]
    o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH)
    o += NH * NH
    b2 = p[o:o + NH]
    o += NH
    W3 = p[o:o + NOUT * NH].reshape(NOUT, NH)
    o += NOUT * NH
    b3 = p[o:o + NOUT]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), b3])


def he_uniform_init(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6/fan_in)), zero biases, float32."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (NH, NIN)) * np.sqrt(6.0 / NIN)
    W2 = rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH)
    W3 = rng.uniform(-1, 1, (NOUT, NH)) * np.sqrt(6.0 / NH)
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), W3, np.zeros(NOUT)).astype(np.float32)


def targets(labels) -> np.ndarray:
    """[B, 2] targets (y_r, y_c) of Loehner class labels (+1, -1, 0)."""
    lab = np.asarray(labels, dtype=np.float64)
    return np.stack([(lab > 0.5).astype(np.float64), (lab < -0.5).astype(np.float64)], axis=1)


def decide(z: np.ndarray) -> np.ndarray:
    """Predicted class of logits [B, 2]: +1 where z_r > 0, else -1 where
    z_c > 0, else 0 (before the level limits of a flag)."""
    z = np.asarray(z)
    return np.where(z[:, 0] > 0, 1, np.where(z[:, 1] > 0, -1, 0)).astype(np.int8)


def forward64(params: np.ndarray, X: np.ndarray):
    """binary64 forward pass; X [B, 128] values.  Returns (z [B, 2], cache)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float64) for a in unpack(np.asarray(params, np.float64)))
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (X, a1, h1, a2, h2)


def bce_loss64(z, labels, pw, pw_c):
    """mean over rows of the two outputs' -(pw y log s(z) + (1-y) log(1-s(z)))."""
    z = np.asarray(z, dtype=np.float64)
    y = targets(labels)
    w = np.array([pw, pw_c], dtype=np.float64)
    log_s = -np.logaddexp(0.0, -z)
    log_1ms = -np.logaddexp(0.0, z)
    return float(np.mean(np.sum(-(w * y * log_s + (1.0 - y) * log_1ms), axis=1)))


def loss64(params, X, labels, pw, pw_c):
    z, _ = forward64(params, X)
    return bce_loss64(z, labels, pw, pw_c)


def grad64(params, X, labels, pw, pw_c) -> np.ndarray:
    """binary64 gradient of loss64 by backpropagation."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float64) for a in unpack(np.asarray(params, np.float64)))
    z, (X, a1, h1, a2, h2) = forward64(params, X)
    y = targets(labels)
    w = np.array([pw, pw_c], dtype=np.float64)
    B = len(z)
    s = 1.0 / (1.0 + np.exp(-z))
    dz = ((1.0 - y) * s - w * y * (1.0 - s)) / B
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    dh2 = (dz @ W3) * (a2 > 0)
    dW2 = dh2.T @ h1
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    dW1 = dh1.T @ X
    db1 = dh1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dW3, db3)


# ---------------------------------------------------------------------------
# emulation of the rounding points of the GPU kernels (bfloat16 operands of
# every matrix product, binary32 accumulation, activations rounded to bfloat16
# before the next product)
# ---------------------------------------------------------------------------


def forward_bf16(params: np.ndarray, Xbits: np.ndarray):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(params, np.float32))
    Xb = bf16_value(Xbits)
    a1 = Xb @ bf16(W1).T + b1.astype(np.float32)
    h1b = bf16(np.maximum(a1, 0.0).astype(np.float32))
    a2 = h1b @ bf16(W2).T + b2.astype(np.float32)
    h2b = bf16(np.maximum(a2, 0.0).astype(np.float32))
    z = (h2b @ bf16(W3).T).astype(np.float32) + b3.astype(np.float32)
    return z.astype(np.float32), (Xb, a1, h1b, a2, h2b)


def grad_bf16(params: np.ndarray, Xbits: np.ndarray, labels: np.ndarray, pw: float, pw_c: float, weight=None):
    """Gradient with the GPU's rounding points: dz in binary32; dh2 (the sum
    dz_r w3_r + dz_c w3_c in that order) and dh1 rounded to bfloat16 as
    operands of the weight-gradient products; bias and W3 gradients summed in
    binary32.  weight: per-sample 0/1 mask (padding)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(params, np.float32))
    z, (Xb, a1, h1b, a2, h2b) = forward_bf16(params, Xbits)
    y = targets(labels).astype(np.float32)
    wmask = np.ones(len(z), np.float32) if weight is None else np.asarray(weight, np.float32)
    B = np.float32(wmask.sum())
    wcls = np.array([pw, pw_c], dtype=np.float32)
    s = (1.0 / (1.0 + np.exp(-z.astype(np.float64)))).astype(np.float32)
    dz = (((1.0 - y) * s - wcls * y * (1.0 - s)) / B * wmask[:, None]).astype(np.float32)
    dW3 = (dz.T @ h2b).astype(np.float32)
    db3 = dz.sum(axis=0, dtype=np.float32)
    W3b = bf16(W3)
    dh2 = ((dz[:, :1] * W3b[0][None, :] + dz[:, 1:] * W3b[1][None, :]) * (a2 > 0)).astype(np.float32)
    dh2b = bf16(dh2)
    dW2 = (dh2b.T @ h1b).astype(np.float32)
    db2 = dh2.sum(axis=0, dtype=np.float32)
    dh1 = ((dh2b @ bf16(W2)) * (a1 > 0)).astype(np.float32)
    dh1b = bf16(dh1)
    dW1 = (dh1b.T @ Xb).astype(np.float32)
    db1 = dh1.sum(axis=0, dtype=np.float32)
    loss = bce_loss64(z, labels, pw, pw_c)
    return pack(dW1, db1, dW2, db2, dW3, db3).astype(np.float32), loss


def adam(params, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in binary32; t counts from 1."""
    params = np.asarray(params, np.float32)
    m = (np.float32(b1) * m + np.float32(1 - b1) * g).astype(np.float32)
    v = (np.float32(b2) * v + np.float32(1 - b2) * g * g).astype(np.float32)
    mh = m / np.float32(1 - b1 ** t)
    vh = v / np.float32(1 - b2 ** t)
    return (params - np.float32(lr) * mh / (np.sqrt(vh) + np.float32(eps))).astype(np.float32), m, v
