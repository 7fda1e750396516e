"""The allocation-free training entry point (amrv_mlp_train_noalloc) against
the workspace one (amrv_mlp_train), through the C-ABI: the same weights, Adam
moments, per-batch losses and gradient, bit for bit, on two calls in a row
(the second with fewer samples and a smaller batch, so it runs on what the
first left in the library's scratch)."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _inputs(seed, n):
    import torch

    dev = torch.device("cuda:0")
    X, y = W.mlp_random_features(seed, n)
    order = np.random.default_rng(seed + 1).permutation(n).astype(np.int32)
    return (torch.from_numpy(X.view(np.int16)).to(dev), torch.from_numpy(y.astype(np.float32)).to(dev),
            torch.from_numpy(order).to(dev))


def _state(w0, nb):
    import torch

    dev = torch.device("cuda:0")
    w = torch.from_numpy(w0.copy()).to(dev)
    return w, torch.zeros_like(w), torch.zeros_like(w), torch.zeros(nb, dtype=torch.float32, device=dev), \
        torch.zeros_like(w)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _run(noalloc, Xd, yd, od, n, batch, nbatch, w0, cfg):
    import torch

    from paper_2004_03275_amd import _native as N

    nb = (n + batch - 1) // batch
    w, m, v, loss, grad = _state(w0, nb)
    torch.cuda.synchronize()
    if noalloc:
        rc = N.lib().amrv_mlp_train_noalloc(_p(Xd), _p(yd), _p(od), n, batch, 0, nbatch, _p(w), _p(m), _p(v),
                                            ctypes.byref(cfg), None, _p(loss), _p(grad))
    else:
        ws = torch.empty(int(N.lib().amrv_mlp_train_workspace_bytes(batch)), dtype=torch.uint8, device="cuda:0")
        rc = N.lib().amrv_mlp_train(_p(Xd), _p(yd), _p(od), n, batch, 0, nbatch, _p(w), _p(m), _p(v),
                                    ctypes.byref(cfg), _p(ws), ws.numel(), None, _p(loss), _p(grad))
    N.check(rc)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (w, m, v, loss, grad)]


@pytest.mark.parametrize("calls", [[(4000, 1024, 3), (700, 256, 2)], [(8192, 4096, 2), (96, 32, 3)]])
def test_noalloc_training_matches_workspace_training(calls):
    from paper_2004_03275_amd import _native as N

    cfg = N.TrainCfg(1e-3, 0.9, 0.999, 1e-8, 2.0, 1.5, 0)
    w0 = W.mlp_init(11)
    for i, (n, batch, nbatch) in enumerate(calls):
        Xd, yd, od = _inputs(31 + i, n)
        ref = _run(False, Xd, yd, od, n, batch, nbatch, w0, cfg)
        got = _run(True, Xd, yd, od, n, batch, nbatch, w0, cfg)
        names = ("w", "m", "v", "loss", "grad")
        for name, a, b in zip(names, ref, got):
            assert np.array_equal(a, b), (i, name, float(np.abs(a - b).max()))
        assert not np.array_equal(ref[0], w0)  # the weights moved
        print(f"[noalloc] call {i}: n {n}, batch {batch}, {nbatch} steps, loss {got[3][:nbatch]}", flush=True)


def test_noalloc_rejects_batches_beyond_its_scratch():
    from paper_2004_03275_amd import _native as N

    cfg = N.TrainCfg(1e-3, 0.9, 0.999, 1e-8, 2.0, 1.5, 0)
    Xd, yd, od = _inputs(41, 256)
    w, m, v, loss, grad = _state(W.mlp_init(1), 1)
    rc = N.lib().amrv_mlp_train_noalloc(_p(Xd), _p(yd), _p(od), 256, 8192, 0, 1, _p(w), _p(m), _p(v),
                                        ctypes.byref(cfg), None, _p(loss), _p(grad))
    assert rc == N.EINVAL
