"""Pins of the oracle's hydrodynamic HLLC flux against exact Riemann solutions
(no GPU).

HLLC (the flux of the paper's HD and MHD blast runs, Sec. 2.4, from Toro's
textbook) is run with the van Leer limiter and SSP-RK3 (the combination of the
KH and 3D blast workloads) on three shock tubes whose exact solutions differ
in kind: Sod (rarefaction, contact, shock), Toro's test 3 (a pressure ratio of
1e5, a strong shock) and Toro's test 2 (two rarefactions around a near-vacuum
star region).  Each has p_L != p_R or u_L != u_R, so the acoustic terms of the
contact speed S_M and of the star pressure p* decide the result; the thresholds
were fixed from a first run (256/512/1024 cells) with a margin of about 40%.

A sharper pin reads the HLLC star states back from the flux of single faces:
the star state on the side of the contact that the face lies on must satisfy
the jump conditions of a contact (normal velocity S_M, pressure p* and
energy flux (E* + p*) S_M on it, Toro ch. 10) and p* must be the same when
reached from the other side's wave (the condition that defines S_M).  A
supersonic face must take the upwind side's physical flux.

The last tests plant a sign slip in S_M's pressure difference and in p*, in a
copy of the oracle's source compiled on the side, and show that the pins
catch each.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import build as orc_build
from oracle import exact_riemann as ER

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (name, left (rho, u, p), right (rho, u, p), t_end,
#  L1 bound on rho and on p at 1024 cells (first run: rho, p))
TUBES = [
    ("sod", (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2, 1.0e-3, 6.0e-4),       # 7.31e-4, 4.06e-4
    ("toro3", (1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), 0.012, 3.0e-2, 1.0),   # 2.02e-2, 0.717
    ("toro2", (1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.15, 1.5e-3, 5.5e-4),    # 1.09e-3, 3.82e-4
]


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _tube(n, left, right):
    s = W.Scheme(ndim=1, block_nx=(n,), base_blocks=(1,), max_level=1, physics=W.EULER, gamma=1.4, flux=W.HLLC,
                 limiter=W.VANLEER, rk_stages=3, cfl=0.8, bc=W.ZERO_GRADIENT)
    f = W.uniform_forest(s)
    (x,) = W.cell_centres(f)
    lt = x < 0.5
    rho = np.where(lt, left[0], right[0])
    u = np.where(lt, left[1], right[1])
    p = np.where(lt, left[2], right[2])
    return f, W.state_from_primitive(f, rho, [u], p), x[0]


def _errors(left, right, t_end, ns=(256, 512, 1024)):
    """L1 errors of density and pressure against the exact solution."""
    out = []
    for n in ns:
        f, U, x = _tube(n, left, right)
        R, dts = oracle.run(f, U, t_end=t_end)
        assert abs(sum(dts) - t_end) < 1e-15
        ex = ER.sod_profile(x, t_end, 0.5, left, right)
        rho = R[0, 0]
        p = 0.4 * (R[2, 0] - 0.5 * R[1, 0] * R[1, 0] / rho)
        assert rho.min() > 0.0 and p.min() > 0.0  # positivity
        out.append((np.abs(rho - ex[0]).mean(), np.abs(p - ex[2]).mean()))
    return np.array(out)


@pytest.mark.parametrize("fixture,left,right", [
    ("toro_test2_star.txt", (1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),
    ("toro_test3_star.txt", (1.0, 0.0, 1000.0), (1.0, 0.0, 0.01)),
])
def test_exact_solver_matches_textbook_star_states(fixture, left, right):
    """The exact solver the pins rest on reproduces the textbook's printed
    star values (to its printed digits) for the two extra tubes."""
    g = _golden(fixture)
    p, u = ER.star_state(*left, *right)
    rl = ER.sample(u - 1e-9, *left, *right)[0]
    rr = ER.sample(u + 1e-9, *left, *right)[0]
    assert abs(p - g["p_star"]) <= 6e-6 * max(1.0, abs(g["p_star"]))
    assert abs(u - g["u_star"]) <= 6e-6 * max(1.0, abs(g["u_star"]))
    assert abs(rl - g["rho_starL"]) < 6e-6
    assert abs(rr - g["rho_starR"]) < 6e-6


@pytest.mark.parametrize("name,left,right,t_end,brho,bp", TUBES, ids=[t[0] for t in TUBES])
def test_hllc_vanleer_rk3_converges_to_exact_solution(name, left, right, t_end, brho, bp):
    e = _errors(left, right, t_end)
    assert e[2, 0] < brho and e[2, 1] < bp, e
    orders = np.log2(e[:-1] / e[1:])
    assert orders.min() >= 0.6, orders


def test_hllc_conserves_on_shock_tube():
    """Mass and energy are unchanged through the zero-gradient ends while no
    wave has reached them; momentum grows by (p_L - p_R) t."""
    left, right = (1.0, 0.0, 1000.0), (1.0, 0.0, 0.01)
    f, U, _ = _tube(512, left, right)
    R, dts = oracle.run(f, U, t_end=0.012)
    t = sum(dts)
    dx = 1.0 / 512
    assert abs(R[0].sum() * dx - U[0].sum() * dx) <= 1e-14
    assert abs(R[2].sum() - U[2].sum()) <= 1e-13 * U[2].sum()
    assert abs(R[1].sum() * dx - (1000.0 - 0.01) * t) <= 1e-12 * 1000.0


GAMMA = 1.4


def _euler_flux(rho, u, p):
    E = p / (GAMMA - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, (E + p) * u]), E


def _contact_conditions(F, left, right):
    """Residuals of the contact jump conditions of the star state read back
    from the HLLC flux F of the face (left | right); None for a supersonic
    face (checked against the upwind flux instead)."""
    (rl, ul, pl), (rr, ur, pr) = left, right
    cl, cr = math.sqrt(GAMMA * pl / rl), math.sqrt(GAMMA * pr / rr)
    sl, sr = min(ul - cl, ur - cr), max(ul + cl, ur + cr)  # Davis speeds
    if sl >= 0.0 or sr <= 0.0:
        return None
    FL, EL = _euler_flux(rl, ul, pl)
    FR, ER_ = _euler_flux(rr, ur, pr)
    kl, kr = rl * (sl - ul), rr * (sr - ur)  # mass fluxes through the outer waves
    # the side of the contact the face lies on: the flux is F_K + S_K (U*_K - U_K)
    # with U*_K = (rho*, rho* S_M, E*); its mass flux rho* S_M gives S_M
    if F[0] >= 0.0:  # S_M >= 0: the face sees the left star state
        sk, kk, Fk, Ek = sl, kl, FL, EL
    else:
        sk, kk, Fk, Ek = sr, kr, FR, ER_
    sm = F[0] * sk / (kk + F[0])
    rs = kk / (sk - sm)
    ps = F[1] - rs * sm * sm               # momentum flux on the contact: rho* S_M^2 + p*
    es = Ek + (F[2] - Fk[2]) / sk          # energy of the star state (jump across S_K)
    scale = max(abs(F[2]), abs(Fk[2]), 1.0)
    r_energy = (F[2] - (es + ps) * sm) / scale
    # p* reached across the left wave and across the right wave must agree
    pstar_l = pl + kl * (sm - ul)
    pstar_r = pr + kr * (sm - ur)
    pscale = max(pl, pr)
    return r_energy, (ps - pstar_l) / pscale, (ps - pstar_r) / pscale


def _random_faces(seed, n):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 10.0, (n, 2))
    u = rng.uniform(-3.0, 3.0, (n, 2))
    p = np.exp(rng.uniform(np.log(0.05), np.log(200.0), (n, 2)))
    return [((rho[i, 0], u[i, 0], p[i, 0]), (rho[i, 1], u[i, 1], p[i, 1])) for i in range(n)]


def _face_oracle():
    s = W.Scheme(ndim=1, block_nx=(16,), base_blocks=(1,), max_level=1, physics=W.EULER, gamma=GAMMA, flux=W.HLLC,
                 limiter=W.VANLEER, rk_stages=3, cfl=0.8, bc=W.ZERO_GRADIENT)
    return oracle.OracleForest(W.uniform_forest(s))


def _jump_condition_residuals(seed=7, n=400):
    o = _face_oracle()
    worst = np.zeros(3)
    nsub = nsup = 0
    for left, right in _random_faces(seed, n):
        F = o.face_flux(np.array(left), np.array(right))
        res = _contact_conditions(F, left, right)
        if res is None:
            nsup += 1
            up = left if min(left[1] - math.sqrt(GAMMA * left[2] / left[0]),
                             right[1] - math.sqrt(GAMMA * right[2] / right[0])) >= 0.0 else right
            Fu, _ = _euler_flux(*up)
            assert np.array_equal(F, Fu) or np.abs(F - Fu).max() <= 1e-14 * np.abs(Fu).max()
            continue
        nsub += 1
        worst = np.maximum(worst, np.abs(res))
    o.close()
    return worst, nsub, nsup


def test_hllc_star_states_satisfy_contact_jump_conditions():
    worst, nsub, nsup = _jump_condition_residuals()
    assert nsub > 300 and nsup > 5  # both kinds of face are exercised
    assert worst.max() < 1e-9, worst


# ---------------------------------------------------------------------------
# planted mistakes: each must break a pin above
# ---------------------------------------------------------------------------

PLANTS = {
    # contact speed S_M with the pressure difference reversed
    "sm_pressure_sign": ("double sm = ((pr - pl) + unl * rl - unr * rr) / (rl - rr);",
                         "double sm = ((pl - pr) + unl * rl - unr * rr) / (rl - rr);"),
    # star pressure p* = p_K - rho_K (S_K - u_K)(S_M - u_K)
    "pstar_sign": ("double ps = pk + rk * (sm - unk);", "double ps = pk - rk * (sm - unk);"),
}


@pytest.fixture(scope="module")
def planted_libs(tmp_path_factory):
    src = open(orc_build.SRC).read()
    out = {}
    d = tmp_path_factory.mktemp("planted")
    for name, (good, bad) in PLANTS.items():
        assert src.count(good) == 1, f"the expression to plant {name} in is not unique in the oracle"
        path = os.path.join(str(d), f"orc_{name}.c")
        with open(path, "w") as fh:
            fh.write(src.replace(good, bad))
        out[name] = orc_build.build(src=path, out=os.path.join(str(d), f"liborc_{name}.so"))
    return out


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_hllc_slip_fails_a_pin(plant, planted_libs, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", oracle.bind(planted_libs[plant]))
    failed = []
    worst, _, _ = _jump_condition_residuals()
    if not worst.max() < 1e-9:
        failed.append("contact jump conditions")
    for name, left, right, t_end, brho, bp in TUBES:
        try:
            e = _errors(left, right, t_end)
        except (AssertionError, oracle.OracleError, FloatingPointError):
            failed.append(name)  # positivity or a non-physical state
            continue
        orders = np.log2(e[:-1] / e[1:])
        if not (e[2, 0] < brho and e[2, 1] < bp and orders.min() >= 0.6):
            failed.append(name)
    assert failed, f"planted {plant} passed every HLLC pin"
