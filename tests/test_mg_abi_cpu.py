"""Host-side checks of the multigrid entry points (no GPU): configuration
validation and workspace sizing through amrv_mg_workspace_bytes."""
import ctypes
import os

import pytest

from paper_2004_03275_amd import _native as N


def _cfg(**kw):
    base = dict(ndim=2, n=64, bc=1, nfields=2, pre_sweeps=2, post_sweeps=2, use_graph=1, smoother=0, length=1.0)
    base.update(kw)
    return N.MgConfig(**base)


def _bytes(cfg):
    return N.lib().amrv_mg_workspace_bytes(ctypes.byref(cfg)), N.lib().amrv_last_error().decode()


pytestmark = pytest.mark.skipif(not os.path.exists(N.LIB_PATH), reason="libamrv.so not built")


@pytest.mark.parametrize("change,msg", [
    ({"ndim": 1}, "ndim"), ({"ndim": 4}, "ndim"), ({"n": 48}, "power of two"), ({"n": 2}, "power of two"),
    ({"n": 16384}, "power of two"), ({"ndim": 3, "n": 1024}, "power of two"), ({"bc": 2}, "boundary"),
    ({"nfields": 0}, "nfields"), ({"nfields": 3}, "nfields"), ({"pre_sweeps": 0}, "sweeps"),
    ({"post_sweeps": 9}, "sweeps"), ({"smoother": 2}, "smoother"), ({"length": 0.0}, "length"), ({"length": float("inf")}, "length"),
])
def test_rejects_bad_configurations(change, msg):
    n, err = _bytes(_cfg(**change))
    assert n == 0
    assert msg in err


def test_workspace_size():
    """Per field and level a solution and a right-hand side of (n >> l)^d
    doubles (256-byte aligned; 2D levels above the LDS-resident tail also a
    second solution buffer), a cell coefficient per level, four temporaries
    of n^d doubles, and the parameter block."""
    up = lambda b: (b + 255) // 256 * 256
    for nd, n, nf in [(2, 256, 2), (3, 32, 1), (2, 4, 1)]:
        got, _ = _bytes(_cfg(ndim=nd, n=n, nfields=nf))
        levels = [n >> l for l in range(n.bit_length() - 1)]
        # 2D levels above the 4,096-cell tail carry a second solution buffer
        per = [(3 if nd == 2 and m ** nd > 4096 else 2) * up(8 * m ** nd) for m in levels]
        want = nf * sum(per) + sum(up(8 * m ** nd) for m in levels) + 4 * up(8 * n ** nd) + up(8 * 44)
        assert got == want, (nd, n, nf, got, want)


def test_create_rejects_null_and_small_workspace():
    h = ctypes.c_void_p()
    cfg = _cfg()
    assert N.lib().amrv_mg_create(ctypes.byref(cfg), None, 1 << 20, None, ctypes.byref(h)) == N.EINVAL
    buf = (ctypes.c_uint8 * 4096)()
    addr = (ctypes.addressof(buf) + 255) // 256 * 256
    assert N.lib().amrv_mg_create(ctypes.byref(cfg), ctypes.c_void_p(addr), 1024, None, ctypes.byref(h)) == N.ENOMEM
