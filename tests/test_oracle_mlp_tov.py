"""Pins of the oracle's MLP back-propagation and of the TOV input generator.

- MLP: the analytic gradient of the mean-squared loss equals central finite
  differences of the loss (relative 1e-7).
- TOV (Sec. III.C.2): the K = 100, Gamma = 2, rho_c = 8e-3 star has the
  same baryon mass as the stable star with rho_s = 1.346e-3 (4 printed
  digits); its radius is 6.31 km within the paper's finest grid spacing
  (isotropic radius, reading); the exterior metric is isotropic
  Schwarzschild in closed form.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def test_mlp_gradient_vs_finite_differences(orc):
    rng = np.random.default_rng(0)
    P = rng.normal(size=orc.NPARAM_MLP) * 0.3
    X = rng.normal(size=(16, 3))
    t = rng.normal(size=16)
    loss, g = orc.mlp_loss_grad(P, X, t)
    idx = rng.choice(orc.NPARAM_MLP, 80, replace=False)
    idx = np.concatenate((idx, [0, 191, 192, 255, 256, 4351, 4352, 4415, 4416, 4479, 4480]))
    for i in idx:
        h = 1e-6 * max(1.0, abs(P[i]))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (orc.mlp_loss_grad(Pp, X, t)[0] - orc.mlp_loss_grad(Pm, X, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    y = orc.mlp_forward(P, X)
    assert loss == pytest.approx(np.mean((y - t) ** 2), rel=1e-14)


def test_tov_stable_partner_and_radius():
    ref = PAPER["tov_migration"]
    from scipy.optimize import brentq
    u = synth.tov_solve(K=ref["K"], G=ref["Gamma"], rho_c=ref["rho_c"])
    rs = brentq(lambda rc: synth.tov_solve(K=ref["K"], G=ref["Gamma"], rho_c=rc)["Mb"] - u["Mb"],
                5e-4, 2.5e-3, xtol=1e-12)
    assert round(rs, 6) == pytest.approx(ref["rho_s"], abs=1e-12)
    R_km = u["Rbar"] * synth.MSUN_KM
    assert abs(R_km - ref["radius_km"]) < ref["finest_dx_km"]


def test_tov_exterior_and_profile():
    tov = synth.tov_solve()
    M = tov["M"]
    rb = np.array([1.2, 2.0, 5.0]) * tov["Rbar"]
    rho, alp, W = synth.tov_fields(tov, rb)
    psi = 1 + M / (2 * rb)
    assert np.all(rho == 0)
    assert np.allclose(alp, (1 - M / (2 * rb)) / psi, rtol=1e-14)
    assert np.allclose(W, psi ** -2, rtol=1e-14)
    # continuity at the surface and central density
    r_in, a_in, w_in = synth.tov_fields(tov, np.array([tov["Rbar"] * (1 - 1e-9)]))
    r_out, a_out, w_out = synth.tov_fields(tov, np.array([tov["Rbar"] * (1 + 1e-9)]))
    assert a_in[0] == pytest.approx(a_out[0], rel=1e-7)
    assert w_in[0] == pytest.approx(w_out[0], rel=1e-7)
    r0, _, _ = synth.tov_fields(tov, np.array([0.0]))
    assert r0[0] == pytest.approx(1.28e-3, rel=1e-10)
