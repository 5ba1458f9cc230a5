"""Pins of the oracle's zero-temperature ("adiabatic") recovery (paper Sec.
III.C.2: the thermal part is neglected and the energy equation discarded)
and of the multi-piece polytrope of Sec. II.C.3.

- a cold state (eps = eps_cold(rho), P = P_cold(rho)) is recovered exactly
  and its E is unchanged;
- a hot state is mapped to the cold state with the same D and S_i (rest
  mass and momentum kept), P = P_cold, eps = eps_cold, and E reset;
- for the gamma law the cold state is dust: z = r in closed form;
- the three-piece polytrope is continuous in P and eps at the transition
  densities (the Delta eps_i of Sec. II.C.3).
"""
import numpy as np
import pytest

# a user-given three-piece cold polytrope (the paper's MPA1 pieces are not
# available): pieces joined continuously in P at rho_b
G3 = [1.35692, 3.005, 2.988]
RB = [1.5e-4, 8.1e-4]
K0 = 8.95e-2


def three_piece():
    K = [K0]
    for i in range(2):
        K.append(K[-1] * RB[i] ** (G3[i] - G3[i + 1]))
    return dict(kind="hybrid", K=K, G=G3, rho_b=RB, Gth=1.75)


def test_three_piece_continuity(orc):
    eos = three_piece()
    for rb in RB:
        lo, hi = rb * (1 - 1e-12), rb * (1 + 1e-12)
        assert orc.eos_press_cold(eos, lo) == pytest.approx(orc.eos_press_cold(eos, hi), rel=1e-10)
        assert orc.eos_eps_cold(eos, lo) == pytest.approx(orc.eos_eps_cold(eos, hi), rel=1e-10)


@pytest.mark.parametrize("rho", [5e-5, 4e-4, 2e-3])
def test_adiabatic_cold_state_round_trip(orc, rho):
    eos = three_piece()
    g = orc.metric_point(dict(alp=0.8, W=0.9, bx=0.05, gxx=1.1, gyy=1.0 / 1.1))
    p = np.array([rho, 0.1, 0.05, -0.2, orc.eos_press_cold(eos, rho), orc.eos_eps_cold(eos, rho)])
    q = orc.prim2con_point(eos, g, 1.3, "cyl", p)
    c2p = dict(w_max=100.0, rho_atm=1e-14, adiabatic=True)
    pr, qr, fl, _ = orc.con2prim_point(eos, g, 1.3, "cyl", c2p, q.copy())
    assert np.allclose(pr, p, rtol=1e-12, atol=1e-15)
    assert qr[4] == pytest.approx(q[4], rel=1e-13)
    assert fl & 2


def test_adiabatic_hot_state_keeps_mass_and_momentum(orc):
    eos = three_piece()
    g = orc.metric_point({})
    rho = 6e-4
    p = np.array([rho, 0.3, 0.0, 0.1, 0.0, orc.eos_eps_cold(eos, rho) + 0.05])
    p[4] = orc.eos_press(eos, rho, p[5])
    q = orc.prim2con_point(eos, g, 1.0, "cart", p)
    pr, qr, fl, _ = orc.con2prim_point(eos, g, 1.0, "cart", dict(w_max=100.0, rho_atm=1e-14, adiabatic=True),
                                       q.copy())
    assert pr[4] == pytest.approx(orc.eos_press_cold(eos, pr[0]), rel=1e-14)
    assert pr[5] == pytest.approx(orc.eos_eps_cold(eos, pr[0]), rel=1e-14)
    assert np.allclose(qr[:4], q[:4], rtol=1e-12)
    assert qr[4] < q[4]


def test_adiabatic_gamma_law_is_dust(orc):
    eos = dict(kind="ideal", K=[100.0], G=[2.0], rho_b=[], Gth=2.0)
    g = orc.metric_point({})
    q = np.array([1.2, 0.5, 0.0, 0.0, 2.0])
    pr, qr, fl, z = orc.con2prim_point(eos, g, 1.0, "cart", dict(w_max=100.0, rho_atm=1e-14, adiabatic=True),
                                       q.copy())
    r = 0.5 / 1.2
    assert z == pytest.approx(r, rel=1e-15)
    assert pr[0] == pytest.approx(1.2 / np.sqrt(1 + r * r), rel=1e-15)
    assert pr[4] == 0.0 and pr[5] == 0.0
