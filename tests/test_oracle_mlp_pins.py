"""Pins of the learned flagger's CPU reference (no GPU).

* bfloat16 round-to-nearest-even on hand-checked bit patterns (ties to even);
* features: exactly zero for a uniform leaf; closed form for a linear profile;
* binary64 backpropagation against central finite differences;
* the bfloat16-emulating gradient close to the binary64 one;
* the first Adam step equals lr * g / (|g| + eps) elementwise.
"""
import numpy as np
import pytest

from oracle import mlp as M
import workloads as W


def test_bf16_rounding_bit_patterns():
    vals = np.array([1.0, -2.0, 0.0, 3.0], dtype=np.float32)
    assert list(M.bf16_bits(vals)) == [0x3F80, 0xC000, 0x0000, 0x4040]
    # exactly halfway between 0x3F80 and 0x3F81: ties to the even pattern
    tie_down = np.array([0x3F808000], dtype=np.uint32).view(np.float32)
    tie_up = np.array([0x3F818000], dtype=np.uint32).view(np.float32)
    above = np.array([0x3F808001], dtype=np.uint32).view(np.float32)
    assert M.bf16_bits(tie_down)[0] == 0x3F80
    assert M.bf16_bits(tie_up)[0] == 0x3F82
    assert M.bf16_bits(above)[0] == 0x3F81
    assert M.bf16_value(np.array([0x3F80], np.uint16))[0] == 1.0


def _leaf(U3):
    return U3


def test_features_of_uniform_leaf_are_zero():
    s = W.blast_scheme(base=1, max_level=1)
    f = W.uniform_forest(s)
    shape = f.state_shape()[1:]
    U = W.state_from_primitive(f, np.full(shape, 1.7), [np.full(shape, 0.3)] * 3, np.full(shape, 2.2))
    X = M.features(U, 3, s.gamma)
    # sums of 64 equal non-dyadic values round, so only rounding-level values
    assert np.all(np.abs(M.bf16_value(X)) < 1e-14)
    rho = np.full(shape, 2.0)
    U = W.state_from_primitive(f, rho, [np.zeros(shape)] * 3, np.full(shape, 0.5))
    assert np.all(M.features(U, 3, s.gamma)[:, :64] == 0)  # dyadic density: exact


def test_features_of_linear_profile_closed_form():
    # rho = a + b i along x inside one 16^3 leaf, p uniform
    a, b = 3.0, 0.125
    i = np.arange(16, dtype=np.float64)
    rho = np.broadcast_to(a + b * i, (16, 16, 16)).copy()[None]
    s = W.blast_scheme(base=1, max_level=1)
    f = W.uniform_forest(s)
    zeros = np.zeros_like(rho)
    U = W.state_from_primitive(f, rho, [zeros, zeros, zeros], np.ones_like(rho))
    X = M.features(U, 3, s.gamma)[0]
    got = M.bf16_value(X[:64])
    for sb in range(64):
        bx = sb & 3
        exact = (a + b * (4 * bx + 1.5)) / (a + b * 7.5) - 1.0
        assert got[sb] == M.bf16(np.array([exact], np.float32))[0]
    assert np.all(X[64:] == 0)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    w = W.mlp_init(3).astype(np.float64)
    w[M.NH * M.NIN:M.NH * M.NIN + M.NH] = rng.uniform(0.05, 0.2, M.NH)  # positive b1: active units
    X = rng.standard_normal((32, M.NIN)) * 0.5
    r = rng.uniform(size=32)
    y = np.where(r < 0.4, 1.0, np.where(r < 0.7, -1.0, 0.0))
    g = M.grad64(w, X, y, 2.5, 1.5)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    # the last parameters: b3 of both outputs, a W3 entry of each output, a b1 entry
    o3 = M.NH * M.NIN + M.NH + M.NH * M.NH + M.NH
    idx = np.concatenate([idx, [M.NPARAM - 1, M.NPARAM - 2, o3 + 5, o3 + M.NH + 7, M.NH * M.NIN + 3]])
    h = 1e-6
    for k in idx:
        wp = w.copy()
        wm = w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (M.loss64(wp, X, y, 2.5, 1.5) - M.loss64(wm, X, y, 2.5, 1.5)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-8, (k, fd, g[k])


def test_outputs_train_on_their_own_class():
    """The refine output's gradient ignores coarsen labels and vice versa: with
    every label +1 the coarsen output is pushed down only, with every label -1
    the refine output is."""
    X, _ = W.mlp_random_features(9, 64)
    w = W.mlp_init(2).astype(np.float64)
    Xv = M.bf16_value(X).astype(np.float64)
    ob3 = M.NPARAM - 2
    g_up = M.grad64(w, Xv, np.ones(64), 2.0, 3.0)
    g_dn = M.grad64(w, Xv, -np.ones(64), 2.0, 3.0)
    z, _ = M.forward64(w, Xv)
    s = 1.0 / (1.0 + np.exp(-z))
    # db3 closed forms: mean of ((1 - y) s - pw y (1 - s)) per output
    assert np.isclose(g_up[ob3], np.mean(-2.0 * (1.0 - s[:, 0])), rtol=1e-12)
    assert np.isclose(g_up[ob3 + 1], np.mean(s[:, 1]), rtol=1e-12)
    assert np.isclose(g_dn[ob3], np.mean(s[:, 0]), rtol=1e-12)
    assert np.isclose(g_dn[ob3 + 1], np.mean(-3.0 * (1.0 - s[:, 1])), rtol=1e-12)
    assert list(M.decide(np.array([[1.0, 1.0], [-1.0, 2.0], [-1.0, -2.0], [0.0, 0.5]]))) == [1, -1, 0, -1]


def test_bf16_emulated_gradient_is_close_to_binary64():
    X, y = W.mlp_random_features(5, 256)
    w = W.mlp_init(7)
    g32, _ = M.grad_bf16(w, X, y, 2.0, 1.0)
    g64 = M.grad64(w.astype(np.float64), M.bf16_value(X).astype(np.float64), y, 2.0, 1.0)
    rel = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    assert rel < 3e-2, rel


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(1)
    p = rng.standard_normal(100).astype(np.float32)
    g = rng.standard_normal(100).astype(np.float32)
    z = np.zeros(100, np.float32)
    p1, m, v = M.adam(p, g, z, z, 1, lr=1e-3)
    expect = p - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, expect, rtol=0, atol=2e-7)
