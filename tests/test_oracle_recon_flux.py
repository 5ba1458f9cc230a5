"""Pins of the oracle's reconstruction, face interpolation, derivatives,
Riemann fluxes and source terms (paper Sec. II.C.1-2).

- PPM (CW84) reproduces cell averages of cubics where the limiters are
  inactive; the per-cell parabola (PPM3) reproduces quadratics and leaves
  a face jump of -c3 h^3 on a cubic (CW84's form none); minmod reproduces
  linear profiles; a monotone step stays
  monotone; 6-point interpolation is exact for quintics; the 6th-order
  derivative is exact for polynomials of degree 6.
- Valencia flux equals the covariant densitised flux sqrt(-g) T^n_j etc.
  built from the 4-metric; HLLC and TVDLF fluxes of equal states equal it on
  random curved metrics with shift (this pins the tetrad, its back-transform
  and the densitisation); supersonic states are upwinded exactly; a
  stationary contact is kept exactly by HLLC and diffused by TVDLF.
- The signal speeds of both solvers (the coordinate characteristic speeds
  of TVDLF and the face-tetrad speeds of HLLC, mapped back to coordinates)
  equal the sound-front speeds of the covariant characteristic condition
  on random curved metrics with lapse, shift and conformal metric, in both
  directions; so do the speeds both fluxes report.
- Momentum sources equal (1/2) sqrt(-g) T^ab d_j g_ab and the energy source
  equals alpha sqrt(gamma) (T^{0b} d_b alpha - alpha T^ab Gamma^0_ab) on
  random metrics with consistent time derivatives.
"""
import math

import numpy as np
import pytest

import spacetime as stt
import synth

EOS = synth.ideal_eos(5.0 / 3.0)


def cell_avg_poly(c, xl, xr):
    P = np.polynomial.polynomial.Polynomial(c).integ()
    return (P(xr) - P(xl)) / (xr - xl)


def test_ppm_exact_for_cubic(orc):
    c = [0.3, 1.0, 0.2, 0.05]  # monotone, gentle curvature on [0, 1]
    n = 40
    xf = np.linspace(0.0, 1.0, n + 1)
    a = cell_avg_poly(c, xf[:-1], xf[1:])
    aL, aR = orc.recon_line("ppm", a)
    faces = xf[3:n - 2]
    exact = np.polynomial.polynomial.polyval(faces, c)
    assert np.allclose(aL, exact, rtol=0, atol=1e-13)
    assert np.allclose(aR, exact, rtol=0, atol=1e-13)


def test_ppm3_exact_for_quadratic(orc):
    """The per-cell parabola reproduces a quadratic from its cell averages
    on both sides of every face (limiters inactive on a monotone, gently
    curved profile)."""
    c = [0.3, 1.0, 0.2]
    n = 40
    xf = np.linspace(0.0, 1.0, n + 1)
    a = cell_avg_poly(c, xf[:-1], xf[1:])
    aL, aR = orc.recon_line("ppm3", a)
    exact = np.polynomial.polynomial.polyval(xf[3:n - 2], c)
    assert np.allclose(aL, exact, rtol=0, atol=1e-13)
    assert np.allclose(aR, exact, rtol=0, atol=1e-13)


def test_ppm3_face_jump_of_a_cubic(orc):
    """On cell averages of a cubic c3 x^3 + ..., the per-cell parabolas of
    the two cells at a face miss the cubic by opposite amounts: the right
    state minus the left state is -c3 h^3 at every face.  CW84's form gives
    both sides the same interface value there (jump 0, no dissipation from
    the Riemann solver)."""
    c3 = 0.05
    c = [0.3, 1.0, 0.2, c3]
    n = 40
    h = 1.0 / n
    xf = np.linspace(0.0, 1.0, n + 1)
    a = cell_avg_poly(c, xf[:-1], xf[1:])
    aL, aR = orc.recon_line("ppm3", a)
    assert np.allclose(aR - aL, -c3 * h ** 3, rtol=1e-6, atol=1e-15)
    bL, bR = orc.recon_line("ppm", a)
    assert np.abs(bR - bL).max() <= 1e-15


def test_minmod_exact_for_linear(orc):
    xf = np.linspace(0.0, 1.0, 31)
    a = 2.0 - 3.0 * 0.5 * (xf[:-1] + xf[1:])
    aL, aR = orc.recon_line("minmod", a)
    exact = 2.0 - 3.0 * xf[3:28]
    assert np.allclose(aL, exact, atol=1e-14) and np.allclose(aR, exact, atol=1e-14)


@pytest.mark.parametrize("recon", ["ppm", "minmod", "ppm3"])
def test_monotone_step_stays_monotone(orc, recon):
    a = np.array([1.0] * 10 + [0.7, 0.3] + [0.1] * 10)
    aL, aR = orc.recon_line(recon, a)
    seq = np.empty(2 * aL.size)
    seq[0::2], seq[1::2] = aL, aR
    assert np.all(np.diff(seq) <= 1e-15)
    assert seq.max() <= 1.0 and seq.min() >= 0.1


def test_lagrange6_and_deriv6_exactness(orc):
    rng = np.random.default_rng(0)
    c5 = rng.normal(size=6)
    h = 0.37
    x6 = (np.arange(6) - 2.5) * h          # cells around the face at 0
    assert orc.lagrange6(np.polynomial.polynomial.polyval(x6, c5)) == pytest.approx(c5[0], abs=1e-13)
    c6 = rng.normal(size=7)
    x7 = (np.arange(7) - 3.0) * h
    assert orc.deriv6(np.polynomial.polynomial.polyval(x7, c6), h) == pytest.approx(c6[1], abs=1e-12)


def random_prim(rng, g, wmax=4.0):
    rho = math.exp(rng.uniform(-3, 1))
    eps = math.exp(rng.uniform(-4, 0.5))
    w = rng.uniform(1.0, wmax)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    gam = stt.sym_from6(g[5:11]) / g[4] ** 2
    u = np.linalg.cholesky(gam) @ (math.sqrt(w * w - 1) * d)
    return np.array([rho, u[0], u[1], u[2], (2.0 / 3.0) * rho * eps, eps])


@pytest.mark.parametrize("dirn", [0, 1])
def test_valencia_flux_is_covariant_flux(orc, dirn):
    rng = np.random.default_rng(10 + dirn)
    for _ in range(30):
        g = stt.random_point_metric(rng)
        p = random_prim(rng, g)
        F = orc.valencia_flux_point(EOS, g, dirn, p)
        ref = stt.valencia_flux_covariant(g, p, 0 if dirn == 0 else 2)
        scale = np.abs(ref).max()
        assert np.allclose(F, ref, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("riemann", ["hllc", "tvdlf"])
@pytest.mark.parametrize("dirn", [0, 1])
def test_flux_consistency_on_curved_metric(orc, riemann, dirn):
    """F(p, p) = f(p): pins the tetrad legs, the back-transform, the moving
    face (shift) and the alpha W^-3 densitisation."""
    rng = np.random.default_rng(20 + dirn)
    for _ in range(40):
        g = stt.random_point_metric(rng, shift=0.3)
        p = random_prim(rng, g)
        F, _ = orc.face_flux_point(EOS, g, dirn, riemann, p, p)
        ref = stt.valencia_flux_covariant(g, p, 0 if dirn == 0 else 2)
        scale = np.abs(ref).max()
        assert np.allclose(F, ref, rtol=0, atol=2e-13 * scale)


def flat():
    g = np.zeros(17)
    g[[0, 4, 5, 8, 10]] = 1.0
    return g


def test_supersonic_upwinding(orc):
    g = flat()
    # both states move right faster than any left-going wave
    pL = np.array([1.0, 3.0, 0.1, 0.0, 0.01, 0.015])
    pR = np.array([0.5, 2.5, 0.0, 0.2, 0.02, 0.06])
    F, _ = orc.face_flux_point(EOS, g, 0, "hllc", pL, pR)
    assert np.allclose(F, orc.valencia_flux_point(EOS, g, 0, pL), rtol=1e-14, atol=1e-15)


def test_stationary_contact(orc):
    g = flat()
    pL = np.array([1.0, 0.0, 0.3, -0.2, 0.5, 0.75])
    pR = np.array([0.1, 0.0, -0.1, 0.4, 0.5, 7.5])
    F, _ = orc.face_flux_point(EOS, g, 0, "hllc", pL, pR)
    assert F[0] == 0.0 and F[2] == 0.0 and F[3] == 0.0 and F[4] == 0.0
    assert F[1] == 0.5
    Ft, _ = orc.face_flux_point(EOS, g, 0, "tvdlf", pL, pR)
    assert abs(Ft[0]) > 1e-3   # TVDLF diffuses the contact


def test_transpose_symmetry(orc):
    g = flat()
    rng = np.random.default_rng(4)
    for _ in range(20):
        a = random_prim(rng, g)
        b = random_prim(rng, g)
        a[2] = b[2] = 0.0
        a[3] = b[3] = 0.0
        Fx, _ = orc.face_flux_point(EOS, g, 0, "hllc", a, b)
        at, bt = a.copy(), b.copy()
        at[1], at[3] = 0.0, a[1]
        bt[1], bt[3] = 0.0, b[1]
        Fz, _ = orc.face_flux_point(EOS, g, 1, "hllc", at, bt)
        assert Fz[0] == Fx[0] and Fz[3] == Fx[1] and Fz[4] == Fx[4]
        assert Fz[1] == 0.0 and Fx[3] == 0.0


def test_momentum_source_covariant_identity(orc):
    rng = np.random.default_rng(7)
    for _ in range(30):
        g, dg = stt.random_metric_with_derivs(rng)
        dg[1, 0] = 0.0  # scalars are y-independent at y = 0 (axisymmetry)
        dg[1, 4] = 0.0
        p = random_prim(rng, g)
        dgo = np.vstack((dg[0], dg[2]))
        s = orc.source_point(EOS, g, dgo, 1.0, "cart", p)
        T, ua, G = stt.stress_energy_up(g, p)
        D = stt.four_metric_derivs(g, dg, 0.0, np.zeros(3))
        sg = stt.sqrt_minus_g(g)
        for comp, d in ((1, 1), (3, 3)):
            ref = 0.5 * sg * np.einsum("ab,ab->", T, D[d])
            assert s[comp] == pytest.approx(ref, rel=1e-11, abs=1e-13)
        assert s[0] == 0.0 and s[2] == 0.0


def test_energy_source_covariant_identity(orc):
    rng = np.random.default_rng(8)
    for _ in range(30):
        g, dg = stt.random_metric_with_derivs(rng)
        dg[1, 0] = 0.0
        p = random_prim(rng, g)
        dgo = np.vstack((dg[0], dg[2]))
        s = orc.source_point(EOS, g, dgo, 1.0, "cart", p)
        dt_alp, dt_beta = rng.normal(), rng.normal(size=3)
        T, ua, G = stt.stress_energy_up(g, p)
        D = stt.four_metric_derivs(g, dg, dt_alp, dt_beta)
        Gam = stt.christoffel_first_index_up(G, D)
        dalp4 = np.concatenate(([dt_alp], dg[:, 0]))
        sq = g[4] ** -3
        ref = g[0] * sq * (T[0] @ dalp4 - g[0] * np.einsum("ab,ab->", T, Gam[0]))
        assert s[4] == pytest.approx(ref, rel=1e-10, abs=1e-13)


def test_geometric_source_balances_pressure(orc):
    """Uniform fluid at rest in flat cylindrical space: the hoop-stress term
    cancels the area-weighted divergence of the pressure flux."""
    grid = synth.make_grid(16, 6, 0.0, 0.0, 0.1, 0.1, "cyl",
                           ("axis", "outflow", "periodic", "periodic"))
    p = synth.empty_fields(grid, 6)
    p[0], p[4], p[5] = 2.0, 0.3, 0.225
    Fx, _ = orc.face_flux(grid, 0, "hllc", EOS, {}, *orc.reconstruct(grid, 0, "ppm", p))
    Fz, _ = orc.face_flux(grid, 1, "hllc", EOS, {}, *orc.reconstruct(grid, 1, "ppm", p))
    L = orc.rhs(grid, EOS, {}, p, Fx, Fz)
    assert np.abs(synth.interior(grid, L)).max() <= 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_signal_speeds_match_covariant_characteristics(orc, seed):
    """lambda-+ from the 3+1 formula (TVDLF, Courant number) and from the
    tetrad frame (HLLC) against the roots of (u.xi)^2 = c_s^2 h^ab xi_a xi_b
    with the front covector xi = (-lambda, delta^n_i) built from the
    4-metric; c_s^2 = Gamma P / (rho h) for the gamma-law gas.  States up
    to w ~ 3 in every direction; metrics with alpha in [0.6, 1.2], shift of
    order 0.3 and a non-flat conformal metric (det 1).  A dropped alpha,
    beta^n or gamma^nn factor fails by O(0.1)."""
    rng = np.random.default_rng(300 + seed)
    gam = EOS["Gth"]
    for _ in range(20):
        g = stt.random_point_metric(rng, scale=0.3, shift=0.3)
        rho = rng.uniform(0.1, 2.0)
        P = rng.uniform(0.01, 3.0)
        eps = P / ((gam - 1.0) * rho)
        prim = np.array([rho, *rng.normal(size=3) * 1.2, P, eps])
        cs2 = gam * P / (rho * (1.0 + eps + P / rho))
        for d, n in ((0, 0), (1, 2)):
            ex = stt.acoustic_speeds(g, prim, n, cs2)
            scale = max(1.0, abs(ex[0]), abs(ex[1]))
            for frame in ("coord", "tetrad"):
                lm, lp = orc.signal_speeds(EOS, g, d, prim, frame)
                assert abs(lm - ex[0]) <= 1e-12 * scale, (frame, d, lm, ex)
                assert abs(lp - ex[1]) <= 1e-12 * scale, (frame, d, lp, ex)
            vmax = max(abs(ex[0]), abs(ex[1]))
            for riemann in ("hllc", "tvdlf"):
                _, sp = orc.face_flux_point(EOS, g, d, riemann, prim, prim)
                assert abs(sp - vmax) <= 1e-12 * scale, (riemann, d, sp, vmax)
