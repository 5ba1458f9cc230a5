"""Pins of the oracle's exact special-relativistic Riemann solver.

The paper checks its shock tube against the exact solution (Sec. III.B.1);
the oracle's solver is pinned here by the paper's printed contact position,
by the Rankine-Hugoniot (Taub) jump conditions across every shock, by the
Riemann invariant and characteristic speeds across every rarefaction, by
mirror symmetry, and by the Newtonian limit against a textbook Newtonian
exact solver written in this file.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def sr_U_F(g, rho, p, v):
    W = 1.0 / math.sqrt(1 - v * v)
    h = 1 + g / (g - 1) * p / rho
    U = np.array([rho * W, rho * h * W * W * v, rho * h * W * W - p])
    F = np.array([rho * W * v, rho * h * W * W * v * v + p, rho * h * W * W * v])
    return U, F


def test_paper_contact_position(orc):
    st = PAPER["shock_tube"]
    sol = orc.riemann_solve(st["gamma"], st["left"], st["right"])
    xc = st["x_interface"] + sol[7] * st["t"]
    assert round(xc, st["digits"]) == pytest.approx(st["x_contact"], abs=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_jump_conditions(orc, seed):
    g = 5.0 / 3.0
    (L, R), = synth.riemann_states(seed, 1, g)
    sol = orc.riemann_solve(g, L, R)
    ps, vs = sol[6], sol[7]
    sides = [(L, sol[8], bool(sol[10]), sol[12], sol[13], -1),
             (R, sol[9], bool(sol[11]), sol[15], sol[14], +1)]
    for (st, rs, shock, head, tail, sgn) in sides:
        Ua, Fa = sr_U_F(g, *st)
        Ub, Fb = sr_U_F(g, rs, ps, vs)
        if shock:
            V = head
            res = (Fb - Fa) - V * (Ub - Ua)
            scale = np.abs(Fa) + np.abs(Fb) + np.abs(Ua) + np.abs(Ub)
            assert np.all(np.abs(res) <= 1e-11 * scale)
        else:
            # Riemann invariant and edge speeds of the fan
            def cs(rho, p):
                h = 1 + g / (g - 1) * p / rho
                return math.sqrt(g * p / (rho * h))

            def J(rho, p, v):
                s = math.sqrt(g - 1)
                c = cs(rho, p)
                Fc = math.log((s + c) / (s - c)) / s
                return math.atanh(v) - sgn * Fc
            ca, cb = cs(st[0], st[1]), cs(rs, ps)
            assert J(*st) == pytest.approx(J(rs, ps, vs), abs=1e-11)
            head_ref = (st[2] + sgn * ca) / (1 + sgn * st[2] * ca)
            tail_ref = (vs + sgn * cb) / (1 + sgn * vs * cb)
            assert head == pytest.approx(head_ref, abs=1e-13)
            assert tail == pytest.approx(tail_ref, abs=1e-12)
            # an interior fan point keeps the invariant and lies on the characteristic
            xi = 0.5 * (head + tail)
            r, p, v = orc.riemann_sample(g, sol, xi)
            assert J(r, p, v) == pytest.approx(J(*st), abs=1e-10)
            c = cs(r, p)
            assert (v + sgn * c) / (1 + sgn * v * c) == pytest.approx(xi, abs=1e-10)
            # isentropic
            assert p / r ** g == pytest.approx(st[1] / st[0] ** g, rel=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_mirror_symmetry(orc, seed):
    g = 5.0 / 3.0
    (L, R), = synth.riemann_states(100 + seed, 1, g)
    a = orc.riemann_solve(g, L, R)
    b = orc.riemann_solve(g, (R[0], R[1], -R[2]), (L[0], L[1], -L[2]))
    assert b[6] == pytest.approx(a[6], rel=1e-13)
    assert b[7] == pytest.approx(-a[7], abs=1e-13)
    assert b[8] == pytest.approx(a[9], rel=1e-12)


def newtonian_exact(g, L, R):
    """Textbook Newtonian exact Riemann solver (Toro, ch. 4): p*, u*."""
    def fK(p, rho, pk):
        c = math.sqrt(g * pk / rho)
        if p > pk:
            A = 2 / ((g + 1) * rho)
            B = (g - 1) / (g + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * c / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)
    lo, hi = 1e-30, 1e3 * max(L[1], R[1])
    for _ in range(300):
        mid = math.sqrt(lo * hi)
        val = fK(mid, L[0], L[1]) + fK(mid, R[0], R[1]) + R[2] - L[2]
        if val > 0:
            hi = mid
        else:
            lo = mid
    p = math.sqrt(lo * hi)
    u = 0.5 * (L[2] + R[2]) + 0.5 * (fK(p, R[0], R[1]) - fK(p, L[0], L[1]))
    return p, u


@pytest.mark.parametrize("seed", range(4))
def test_newtonian_limit(orc, seed):
    g = 5.0 / 3.0
    rng = np.random.default_rng(seed)
    eps = 1e-9  # p/rho ~ eps, |v| ~ sqrt(eps): relativistic corrections ~ eps
    L = (rng.uniform(0.5, 2), rng.uniform(0.5, 2) * eps, rng.uniform(-1, 1) * math.sqrt(eps))
    R = (rng.uniform(0.5, 2), rng.uniform(0.5, 2) * eps, rng.uniform(-1, 1) * math.sqrt(eps))
    sol = orc.riemann_solve(g, L, R)
    pn, un = newtonian_exact(g, L, R)
    assert sol[6] == pytest.approx(pn, rel=1e-6)
    assert sol[7] == pytest.approx(un, rel=1e-5, abs=1e-6 * math.sqrt(eps))


def test_vacuum_detected(orc):
    g = 5.0 / 3.0
    L, R = (1.0, 1e-3, -0.5), (1.0, 1e-3, 0.5)
    assert synth.riemann_has_vacuum(g, L, R)
    with pytest.raises(ValueError):
        orc.riemann_solve(g, L, R)
