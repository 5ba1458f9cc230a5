"""Pins of the oracle's EOS, prim->con and con->prim (paper Sec. II.C.3-4).

con2prim is pinned by what the mathematics fixes: the round trip
prim -> con -> prim, the definition of the root (sign change of the master
function at the returned z), closed forms (dust z = r, fluid at rest z = 0),
the Lorentz-factor cap, the cold recovery and the atmosphere, and the
prim->con map against the covariant definitions D = alpha rho u^t,
S_j = alpha T^0_j, E = alpha^2 T^00.
"""
import math

import numpy as np
import pytest

import spacetime as stt
import synth

C2P = dict(w_max=100.0, rho_atm=1e-12)


def hybrid3():
    # three cold pieces, continuous pressure (K_i from continuity), thermal 5/3
    G = [1.35, 3.0, 2.6]
    rb = [5e-4, 1.5e-3]
    K = [0.09]
    for i in (1, 2):
        K.append(K[i - 1] * rb[i - 1] ** (G[i - 1] - G[i]))
    return dict(kind="hybrid", K=K, G=G, rho_b=rb, Gth=5.0 / 3.0)


def test_ideal_eos_closed_forms(orc):
    e = synth.ideal_eos(5.0 / 3.0)
    for rho, eps in [(1.0, 0.3), (1e-6, 2.0), (7.0, 1e-8)]:
        P = orc.eos_press(e, rho, eps)
        assert P == pytest.approx((2.0 / 3.0) * rho * eps, rel=1e-15)
        h = 1 + eps + P / rho
        assert orc.eos_cs2(e, rho, eps, P) == pytest.approx(5.0 / 3.0 * P / (rho * h), rel=1e-14)
        assert orc.eos_eps_cold(e, rho) == 0.0


def test_hybrid_continuity_and_single_piece(orc):
    e = hybrid3()
    for rb in e["rho_b"]:
        lo, hi = rb * (1 - 1e-12), rb * (1 + 1e-12)
        assert orc.eos_press_cold(e, lo) == pytest.approx(orc.eos_press_cold(e, hi), rel=1e-9)
        assert orc.eos_eps_cold(e, lo) == pytest.approx(orc.eos_eps_cold(e, hi), rel=1e-9)
    # one piece with Gth = G is the gamma-law pressure for every eps
    one = dict(kind="hybrid", K=[100.0], G=[2.0], rho_b=[], Gth=2.0)
    ideal = synth.ideal_eos(2.0, K=100.0)
    for rho, eps in [(1e-3, 0.2), (1e-8, 1e-5)]:
        assert orc.eos_press(one, rho, eps) == pytest.approx(orc.eos_press(ideal, rho, eps), rel=1e-13)


@pytest.mark.parametrize("eos", ["ideal", "hybrid"])
def test_sound_speed_is_adiabatic_derivative(orc, eos):
    """c_s^2 h = dP/drho along an adiabat (d eps = P/rho^2 d rho)."""
    e = synth.ideal_eos(5.0 / 3.0) if eos == "ideal" else hybrid3()
    for rho, eps in [(3e-4, 0.05), (1e-3, 0.2), (2e-3, 0.4)]:
        P = orc.eos_press(e, rho, eps)
        h = 1 + eps + P / rho
        dr = rho * 1e-6
        Pp = orc.eos_press(e, rho + dr, eps + P / rho ** 2 * dr)
        Pm = orc.eos_press(e, rho - dr, eps - P / rho ** 2 * dr)
        dPdr = (Pp - Pm) / (2 * dr)
        assert orc.eos_cs2(e, rho, eps, P) * h == pytest.approx(dPdr, rel=1e-7)


def random_state(rng, wmax=10.0):
    rho = math.exp(rng.uniform(math.log(1e-8), math.log(1e-2)))
    eps = math.exp(rng.uniform(math.log(1e-4), math.log(2.0)))
    w = rng.uniform(1.0, wmax)
    v = math.sqrt(1 - 1 / w ** 2)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    return rho, eps, w * v * d   # contravariant-orthonormal direction, scaled below


def state_in_metric(g, rho, eps, uflat, eos, orc):
    """Covariant u_i with gamma^ij u_i u_j = |uflat|^2."""
    gam = stt.sym_from6(g[5:11]) / g[4] ** 2
    Lc = np.linalg.cholesky(gam)       # gamma = Lc Lc^T
    u = Lc @ uflat                     # gamma^ij u_i u_j = |uflat|^2
    P = orc.eos_press(eos, rho, eps)
    return np.array([rho, u[0], u[1], u[2], P, eps])


@pytest.mark.parametrize("geom", ["cart", "cyl"])
def test_prim2con_matches_covariant(orc, geom):
    rng = np.random.default_rng(5)
    eos = synth.ideal_eos(2.0, 100.0)
    for _ in range(20):
        g = stt.random_point_metric(rng)
        rho, eps, uf = random_state(rng)
        p = state_in_metric(g, rho, eps, uf, eos, orc)
        x = rng.uniform(0.1, 3.0)
        q = orc.prim2con_point(eos, g, x, geom, p)
        ref = stt.conserved_covariant(g, p)
        if geom == "cyl":
            ref[2] *= x
        assert np.allclose(q, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("eos_kind", ["ideal", "hybrid"])
def test_round_trip(orc, eos_kind):
    rng = np.random.default_rng(11)
    eos = synth.ideal_eos(2.0, 100.0) if eos_kind == "ideal" else hybrid3()
    n_checked = 0
    for _ in range(200):
        g = stt.random_point_metric(rng)
        rho, eps, uf = random_state(rng)
        if eos_kind == "hybrid":
            eps = eps + orc.eos_eps_cold(eos, rho)
        p = state_in_metric(g, rho, eps, uf, eos, orc)
        x = rng.uniform(0.1, 3.0)
        q = orc.prim2con_point(eos, g, x, "cyl", p)
        p2, q2, flags, z = orc.con2prim_point(eos, g, x, "cyl", C2P, q)
        assert flags == 0
        # conserved variables reproduced from the recovered primitives
        q3 = orc.prim2con_point(eos, g, x, "cyl", p2)
        assert np.allclose(q3, q, rtol=1e-12, atol=1e-300)
        # primitives to 1e-12 where the recovery is well conditioned
        E = q[4] * g[4] ** 3
        D = q[0] * g[4] ** 3
        kappa = (E / D) / eps
        if kappa <= 1e4:
            n_checked += 1
            assert p2[0] == pytest.approx(p[0], rel=1e-12)
            assert p2[5] == pytest.approx(p[5], rel=1e-12)
            assert p2[4] == pytest.approx(p[4], rel=1e-12)
            assert np.allclose(p2[1:4], p[1:4], rtol=1e-12, atol=1e-12 * np.abs(p[1:4]).max())
    assert n_checked > 100


def test_root_is_bracketed(orc):
    """The returned z is the root of the master function: f changes sign
    within a relative distance 1e-12 of it, and |f(z)| is at rounding level."""
    rng = np.random.default_rng(3)
    eos = synth.ideal_eos(5.0 / 3.0)
    g = stt.random_point_metric(rng) * 0 + np.array(
        [1, 0, 0, 0, 1, 1, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 0], dtype=float)
    for _ in range(50):
        rho, eps, uf = random_state(rng)
        p = np.array([rho, *uf, (2 / 3) * rho * eps, eps])
        q = orc.prim2con_point(eos, g, 1.0, "cart", p)
        _, _, _, z = orc.con2prim_point(eos, g, 1.0, "cart", C2P, q)
        D, E = q[0], q[4]
        r = np.linalg.norm(q[1:4]) / D
        qq = E / D - 1
        up, dn = z * (1 + 1e-12), z * (1 - 1e-12)
        assert orc.c2p_master(eos, D, qq, r, dn) < 0.0 < orc.c2p_master(eos, D, qq, r, up)
        assert abs(orc.c2p_master(eos, D, qq, r, z)) <= 1e-14 * (z + r)


def test_closed_forms(orc):
    eos = synth.ideal_eos(5.0 / 3.0)
    flat = stt.random_point_metric(np.random.default_rng(0)) * 0
    flat[[0, 4, 5, 8, 10]] = 1.0
    # fluid at rest: z = 0 and rho = D exactly
    q = np.array([0.7, 0.0, 0.0, 0.0, 0.7 * 1.25])
    p, _, flags, z = orc.con2prim_point(eos, flat, 1.0, "cart", C2P, q)
    assert z == 0.0 and p[0] == 0.7 and flags == 0
    assert p[5] == pytest.approx(0.25, rel=1e-15)
    # dust (P = eps = 0): h-hat = 1, so z = r
    rho, u = 0.3, np.array([0.4, -0.2, 1.1])
    w = math.sqrt(1 + u @ u)
    q = np.array([rho * w, *(rho * w * u), rho * w * w])
    p, _, flags, z = orc.con2prim_point(eos, flat, 1.0, "cart", C2P, q)
    r = np.linalg.norm(q[1:4]) / q[0]
    assert z == pytest.approx(r, rel=1e-14)
    assert p[0] == pytest.approx(rho, rel=1e-13)
    assert np.allclose(p[1:4], u, rtol=1e-13)


def test_lorentz_cap(orc):
    """k = |S|/E above k_max = 2 v_max/(1+v_max^2) (the largest k a state
    with v <= v_max can have) is rescaled to k_max; the recovered state then
    satisfies v <= k_max (the root bracket gives v <= k)."""
    eos = synth.ideal_eos(5.0 / 3.0)
    flat = np.zeros(17)
    flat[[0, 4, 5, 8, 10]] = 1.0
    vmax = math.sqrt(1 - 1 / C2P["w_max"] ** 2)
    kmax = 2 * vmax / (1 + vmax ** 2)
    for kin in (1.2, 1.0, 1 - 1e-12):
        E = 2.0
        q = np.array([1.0, kin * E * 0.6, kin * E * 0.8, 0.0, E])
        p2, q2, flags, _ = orc.con2prim_point(eos, flat, 1.0, "cart", C2P, q)
        assert flags & 1
        assert np.all(np.isfinite(p2))
        w = math.sqrt(1 + p2[1:4] @ p2[1:4])
        assert math.sqrt(1 - 1 / w ** 2) <= kmax * (1 + 1e-12)
        assert np.allclose(orc.prim2con_point(eos, flat, 1.0, "cart", p2), q2, rtol=1e-13)
    # below k_max nothing is rescaled
    u = np.array([math.sqrt(50.0 ** 2 - 1), 0, 0])
    q = orc.prim2con_point(eos, flat, 1.0, "cart", np.array([1.0, *u, (2 / 3) * 0.1, 0.1]))
    assert orc.con2prim_point(eos, flat, 1.0, "cart", C2P, q)[2] == 0


def test_cold_recovery_and_atmosphere(orc):
    eos = synth.ideal_eos(5.0 / 3.0)
    flat = np.zeros(17)
    flat[[0, 4, 5, 8, 10]] = 1.0
    # energy below the cold value: eps-hat < 0 at the root -> cold recovery
    rho, u = 1.0, np.array([0.5, 0.0, 0.0])
    w = math.sqrt(1 + u @ u)
    q = np.array([rho * w, *(rho * w * u), rho * w * w * (1 - 1e-3)])
    p, q2, flags, z = orc.con2prim_point(eos, flat, 1.0, "cart", C2P, q)
    assert flags & 2
    assert p[4] == 0.0 and p[5] == 0.0
    assert q2[4] == pytest.approx(rho * w * w, rel=1e-13)   # E reset from primitives
    assert np.all(np.isfinite(p))
    # density below the floor -> atmosphere state, q reset
    c2p = dict(w_max=100.0, rho_atm=1e-3)
    q = orc.prim2con_point(eos, flat, 1.0, "cart", np.array([1e-5, 0.1, 0, 0, 1e-6, 0.15]))
    p, q2, flags, _ = orc.con2prim_point(eos, flat, 1.0, "cart", c2p, q)
    assert flags & 4
    assert p[0] == 1e-3 and np.all(p[1:4] == 0.0)
    assert np.allclose(orc.prim2con_point(eos, flat, 1.0, "cart", p), q2, rtol=1e-15)


@pytest.mark.parametrize("bad", [
    [0.0, 0, 0, 0, 1.0], [-1.0, 0, 0, 0, 1.0], [1.0, 0, 0, 0, -1.0],
    [np.nan, 0, 0, 0, 1.0], [1.0, np.inf, 0, 0, 1.0], [1.0, 0, 0, 0, np.nan]])
def test_invalid_input_goes_to_atmosphere(orc, bad):
    eos = synth.ideal_eos(5.0 / 3.0)
    flat = np.zeros(17)
    flat[[0, 4, 5, 8, 10]] = 1.0
    p, q2, flags, _ = orc.con2prim_point(eos, flat, 1.0, "cart", C2P, np.array(bad))
    assert flags & 8 and flags & 4
    assert np.all(np.isfinite(p)) and np.all(np.isfinite(q2))
    assert p[0] == C2P["rho_atm"]
