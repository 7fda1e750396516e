"""MHD pins of the oracle (no GPU).

* A small-amplitude shear Alfven wave (B0 along x, perturbation in v_y and
  B_y with dB_y = -sqrt(rho) dv_y) travels at v_A = B0/sqrt(rho): the
  oracle converges to the exact translated profile, and the opposite
  polarisation travels the other way.  A sign slip in the Lorentz force or
  the induction flux stops or reverses the wave.
* GLM cleaning: a divergence error in B_x with psi = 0 obeys
  dB_x/dt + dpsi/dx = 0, dpsi/dt + c_h^2 dB_x/dx = 0 (decoupled from the rest
  of the system): B_x - B0 = d sin(2 pi x) cos(2 pi tau), psi = -c_h d
  cos(2 pi x) sin(2 pi tau), tau = sum c_h dt; and the once-per-step damping
  multiplies psi by exp(-dt c_h / c_r).
* The paper's MHD blast (Sec. 2.4; uniform B along the diagonal) stays
  point symmetric and symmetric under x <-> y with the components exchanged.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _line_mhd(n, cr=0.18, flux=W.HLL):
    s = W.Scheme(ndim=2, block_nx=(n, 4), base_blocks=(1, 1), max_level=1, xmin=(0.0, 0.0),
                 xmax=(1.0, 4.0 / n), physics=W.MHD, gamma=5.0 / 3.0, flux=flux, limiter=W.VANLEER, rk_stages=3,
                 cfl=0.8, bc=W.PERIODIC, glm_cr=cr)
    f = W.uniform_forest(s)
    x, _ = W.cell_centres(f)
    return s, f, x


def _alfven(n, direction=+1, amp=1e-3, t_end=0.25, flux=W.HLL):
    s, f, x = _line_mhd(n, flux=flux)
    one = np.ones_like(x)
    dv = amp * np.sin(2 * np.pi * x)
    U = W.state_from_primitive(f, one, [0 * one, dv], one, [one, -direction * dv])
    R, dts = oracle.run(f, U, t_end=t_end)
    t = sum(dts)
    vy = R[2] / R[0]
    exact = amp * np.sin(2 * np.pi * (x - direction * t))
    return float(np.mean(np.abs(vy - exact))) / amp


@pytest.mark.parametrize("flux", [W.HLL, W.HLLC])
def test_alfven_wave_converges_to_the_travelling_solution(flux):
    errs = [_alfven(n, flux=flux) for n in (32, 64, 128)]
    # second-order scheme with limiter clipping at extrema: order >= 1.3
    assert errs[2] < 0.02, errs
    assert errs[0] / errs[1] > 2.4 and errs[1] / errs[2] > 2.4, errs


def test_alfven_wave_opposite_polarisation_travels_backwards():
    assert _alfven(64, direction=-1) < 0.05
    # the wrong direction is far off: the exact profile moved by half a wavelength
    assert _alfven(64, direction=-1) < 0.2 * _line_error_wrong_way()


def _line_error_wrong_way(n=64, amp=1e-3):
    s, f, x = _line_mhd(n)
    one = np.ones_like(x)
    dv = amp * np.sin(2 * np.pi * x)
    U = W.state_from_primitive(f, one, [0 * one, dv], one, [one, dv])  # travels in -x
    R, dts = oracle.run(f, U, t_end=0.25)
    t = sum(dts)
    vy = R[2] / R[0]
    wrong = amp * np.sin(2 * np.pi * (x - t))
    return float(np.mean(np.abs(vy - wrong))) / amp


def _glm(n, cr, steps=None, t_end=None, d=1e-3):
    s, f, x = _line_mhd(n, cr=cr)
    one = np.ones_like(x)
    U = W.state_from_primitive(f, one, [0 * one, 0 * one], one, [one + d * np.sin(2 * np.pi * x), 0 * one])
    o = oracle.OracleForest(f)
    o.set_state(U)
    tau, t, damp = 0.0, 0.0, 1.0
    while (t_end is None or t < t_end) and (steps is None or steps > 0):
        dt = o.max_dt()
        if t_end is not None:
            dt = min(dt, t_end - t)
        ch = o.glm_ch
        o.advance(dt)
        tau += ch * dt
        damp *= math.exp(-(dt * ch) / cr)
        t += dt
        if steps is not None:
            steps -= 1
    R = o.get_state()
    return x, R, tau, ch, damp


def test_glm_divergence_wave_without_damping():
    errs = []
    for n in (32, 64, 128):
        x, R, tau, ch, _ = _glm(n, cr=1e30, t_end=0.1)
        d = 1e-3
        bx = R[4] - 1.0
        psi = R[6]
        eb = np.mean(np.abs(bx - d * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * tau))) / d
        ep = np.mean(np.abs(psi + ch * d * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * tau))) / (ch * d)
        errs.append(max(eb, ep))
    assert errs[2] < 0.02, errs
    assert errs[0] / errs[2] > 4.0, errs


def test_glm_damping_factor():
    """A uniform psi on a uniform state has no flux divergence, so only the
    once-per-step damping acts: psi_n = psi_0 prod exp(-dt c_h / c_r) (to
    rounding of the SSP combinations)."""
    n = 32
    s, f, x = _line_mhd(n, cr=0.18)
    one = np.ones_like(x)
    U = W.state_from_primitive(f, one, [0.3 * one, -0.2 * one], one, [one, 0.5 * one])
    U[6] = 0.7
    o = oracle.OracleForest(f)
    o.set_state(U)
    damp = 1.0
    for _ in range(5):
        dt = o.max_dt()
        damp *= math.exp(-(dt * o.glm_ch) / 0.18)
        o.advance(dt)
    R = o.get_state()
    assert np.all(R[6] == R[6].flat[0])
    assert abs(R[6].flat[0] / 0.7 - damp) < 1e-13
    assert 0.1 < damp < 0.95
    for v in range(6):  # the rest stays uniform and unchanged up to rounding
        assert np.allclose(R[v], U[v], rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# the paper's MHD blast (Sec. 2.4): symmetries of the setup
# ---------------------------------------------------------------------------


def _global_2d(f, U):
    """State of a uniform 2D forest as [var][y][x] over the whole domain."""
    s = f.scheme
    nb = s.block_nx[0]
    G = np.empty((U.shape[0], s.base_blocks[1] * nb, s.base_blocks[0] * nb))
    for b in range(f.n):
        i, j = int(f.ijk[b][0]), int(f.ijk[b][1])
        G[:, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = U[:, b]
    return G


def test_mhd_blast_point_and_diagonal_symmetry():
    """rho, p radial, v = 0, B uniform along the diagonal: the solution stays
    point symmetric (rho even, v odd, B even under x -> -x) and symmetric
    under x <-> y with the x and y components exchanged."""
    s = W.mhd_blast_scheme(2, base=4, max_level=1, flux=W.HLL)
    f, U = W.mhd_blast(2, scheme=s)
    R, dts = oracle.run(f, U, steps=25, ramp_steps=10)
    assert dts[0] * 10 == pytest.approx(dts[1] * 5, rel=0.5)  # the ramp is on
    G = _global_2d(f, R)
    scale = np.abs(G).reshape(G.shape[0], -1).max(axis=1)
    # point symmetry (the grid is symmetric about the origin)
    P = G[:, ::-1, ::-1]
    assert np.all(np.abs(G[0] - P[0]) <= 1e-11 * scale[0])
    for k in (1, 2):
        assert np.all(np.abs(G[k] + P[k]) <= 1e-11 * scale[k] + 1e-14)
    for k in (3, 4, 5):
        assert np.all(np.abs(G[k] - P[k]) <= 1e-11 * scale[k])
    # diagonal mirror: transpose, exchange x and y components
    T = np.transpose(G, (0, 2, 1))
    assert np.all(np.abs(G[0] - T[0]) <= 1e-11 * scale[0])
    assert np.all(np.abs(G[1] - T[2]) <= 1e-11 * scale[1] + 1e-14)
    assert np.all(np.abs(G[3] - T[3]) <= 1e-11 * scale[3])
    assert np.all(np.abs(G[4] - T[5]) <= 1e-11 * scale[4])
    # the blast has moved: not trivially symmetric because nothing happened
    assert np.abs(G[1]).max() > 0.1


def test_courant_ramp_reading():
    """The reading of the lowered first steps (Sec. 2.4 gives no formula):
    the oracle's run takes (n + 1)/10 of each of the first 10 Courant steps."""
    assert [oracle.courant_factor(n, 10) for n in range(12)] == [(n + 1) / 10 for n in range(10)] + [1.0, 1.0]
    assert oracle.courant_factor(0, 0) == 1.0
    f, U = W.mhd_blast(2, base=2, max_level=2)
    o = oracle.OracleForest(f)
    o.set_state(U)
    _, dts = oracle.run(f, U, steps=3, ramp_steps=10)
    assert dts[0] == o.max_dt() * 0.1


# ---------------------------------------------------------------------------
# HLLC for MHD (Li 2005, the flux of the paper's MHD blast)
# ---------------------------------------------------------------------------


def test_mhd_hllc_without_field_is_the_hydrodynamic_hllc():
    """B = 0, psi = 0: the MHD HLLC flux takes the B_n = 0 branch and must
    give the hydrodynamic HLLC solution (up to the rounding of the fast
    speed formula)."""
    s = W.kh_scheme(2)
    f, U = W.kh(scheme=s)
    Re, dts = oracle.run(f, U, steps=20)
    sm = W.Scheme(ndim=2, block_nx=(16, 16), base_blocks=(2, 2), max_level=1, physics=W.MHD, gamma=1.4,
                  flux=W.HLLC, limiter=W.VANLEER, rk_stages=3, cfl=0.8, bc=W.PERIODIC)
    fm = W.Forest(sm, f.level, f.ijk)
    rho = U[0]
    u, v = U[1] / rho, U[2] / rho
    p = 0.4 * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / rho)
    z = np.zeros_like(rho)
    Rm, _ = oracle.run(fm, W.state_from_primitive(fm, rho, [u, v], p, [z, z]), dts=dts)
    for k in range(4):
        assert np.abs(Re[k] - Rm[k]).max() <= 1e-12 * np.abs(Re[k]).max(), k
    assert np.abs(Rm[4:]).max() == 0.0


def _contact(flux, steps=20):
    """A stationary tangential discontinuity in x: density and v_y jump,
    B = (0, 0.8) tangential, total pressure continuous, B_n = 0."""
    s = W.Scheme(ndim=2, block_nx=(32, 4), base_blocks=(1, 1), max_level=1, xmin=(0.0, 0.0), xmax=(1.0, 0.125),
                 physics=W.MHD, gamma=5.0 / 3.0, flux=flux, limiter=W.VANLEER, rk_stages=3, cfl=0.8,
                 bc=W.PERIODIC)
    f = W.uniform_forest(s)
    x, _ = W.cell_centres(f)
    one = np.ones_like(x)
    inner = np.abs(x - 0.5) < 0.25
    rho = np.where(inner, 2.0, 1.0)
    vy = np.where(inner, 0.5, -0.5)
    U = W.state_from_primitive(f, rho, [0 * one, vy], one, [0 * one, 0.8 * one])
    R, _ = oracle.run(f, U, steps=steps)
    return U, R


def test_mhd_hllc_keeps_a_tangential_discontinuity():
    """The B_n = 0 branch keeps each side's transverse velocity and field: the
    discontinuity stays exact; HLL (and an HLL-averaged star state) smear it."""
    U, R = _contact(W.HLLC)
    assert np.abs(R[0] - U[0]).max() <= 1e-14
    assert np.abs(R[2] - U[2]).max() <= 1e-14
    U, R = _contact(W.HLL)
    assert np.abs(R[0] - U[0]).max() > 1e-3
    assert np.abs(R[2] - U[2]).max() > 1e-3


def test_mhd_blast_with_hllc_keeps_its_symmetries():
    s = W.mhd_blast_scheme(2, base=4, max_level=1, flux=W.HLLC)
    f, U = W.mhd_blast(2, scheme=s)
    R, _ = oracle.run(f, U, steps=25, ramp_steps=10)
    G = _global_2d(f, R)
    scale = np.abs(G).reshape(G.shape[0], -1).max(axis=1)
    P = G[:, ::-1, ::-1]
    T = np.transpose(G, (0, 2, 1))
    assert np.all(np.abs(G[0] - P[0]) <= 1e-11 * scale[0])
    assert np.all(np.abs(G[1] + P[1]) <= 1e-11 * scale[1] + 1e-14)
    assert np.all(np.abs(G[0] - T[0]) <= 1e-11 * scale[0])
    assert np.all(np.abs(G[4] - T[5]) <= 1e-11 * scale[4])
    assert np.abs(G[1]).max() > 0.1
