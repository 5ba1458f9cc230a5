"""Pins of the oracle's fixed-mesh-refinement operators (paper Sec. II.A
grid structure, Sec. II.E FMR setting).

- restriction is the volume-weighted average: a hand-computed 2 x 2
  cylindrical block, constants are kept, and sum(q dV) over the child's
  footprint is unchanged;
- spatial prolongation reproduces linear data exactly (the minmod of two
  equal differences is that difference) and is flat at an extremum;
- time interpolation is exact for data quadratic in time, and falls back to
  the linear interpolant through (t^n, t^{n+1}) where the slices are not
  monotone (the limiter of Sec. II.E);
- the Berger-Oliger step with restriction and flux correction keeps the
  total mass and angular momentum of a closed box to round-off (the
  conservation across refinement boundaries the paper checks in Sec.
  III.D); without the flux correction they are not kept, so the pin sees a
  dropped or sign-flipped correction;
- with l_fix the levels up to l_fix take the parent's step, finer ones half
  of it;
- the (4+4) buffer schedule (Sec. II.E): its prolongation fills the inner
  buffer with the same exactness (linear in space, quadratic in time); the
  Berger-Oliger step keeps mass and angular momentum to round-off with it
  too and loses them without the flux correction; the stage mapping (the
  buffer and ghosts prolonged at t before stage 1, the ghosts at t + dt
  before stage 2, nothing before stage 3, which updates the own cells
  only) is what the driver does; a uniform state at rest stays uniform to
  round-off across the refinement boundaries under both schedules (the
  restriction's volume-weighted sum rounds).
"""
import math

import numpy as np
import pytest

import synth

OPTS = dict(recon="ppm", riemann="hllc", c2p=dict(w_max=100.0, rho_atm=1e-12))
GAM = 5.0 / 3.0


def test_restrict_hand_example(orc):
    """Cylindrical child cells x = 0.5, 1.5 (dx = dz = 1) under the parent
    cell x = 1 (dx = dz = 2): q_p = (1*0.5 + 2*1.5 + 3*0.5 + 4*1.5) / 4."""
    cg = synth.make_grid(6, 6, 0.0, 0.0, 1.0, 1.0, "cyl", ("axis", "external", "reflect", "external"))
    pg = synth.make_grid(6, 6, 0.0, 0.0, 2.0, 2.0, "cyl", ("axis", "outflow", "reflect", "outflow"))
    qc = synth.empty_fields(cg, 5)
    ng = cg["ng"]
    for c in range(5):
        qc[c, ng + 0, ng + 0] = 1.0 + c
        qc[c, ng + 0, ng + 1] = 2.0 + c
        qc[c, ng + 1, ng + 0] = 3.0 + c
        qc[c, ng + 1, ng + 1] = 4.0 + c
    qp = synth.empty_fields(pg, 5)
    orc.fmr_restrict(pg, qp, cg, qc)
    for c in range(5):
        want = ((1 + c) * 0.5 + (2 + c) * 1.5 + (3 + c) * 0.5 + (4 + c) * 1.5) / 4.0
        assert qp[c, ng, ng] == pytest.approx(want, rel=1e-15)
    assert qp[0, ng, ng] == pytest.approx(2.75, rel=1e-15)


@pytest.mark.parametrize("geom", ["cyl", "cart"])
def test_restrict_conserves_and_keeps_constants(orc, geom):
    pg, cg = synth.fmr_grids(2, 16, 1.0, geom=geom, outer="outflow")
    rng = np.random.default_rng(3)
    qc = synth.empty_fields(cg, 5)
    qc[:] = rng.uniform(0.5, 2.0, size=qc.shape)
    qp = synth.empty_fields(pg, 5)
    orc.fmr_restrict(pg, qp, cg, qc)
    Xc, _ = synth.cell_coords(cg)
    Xp, _ = synth.cell_coords(pg)
    vol = (lambda X, g: X * g["dx"] * g["dz"]) if geom == "cyl" else (lambda X, g: g["dx"] * g["dz"] + 0 * X)
    fine = (synth.interior(cg, qc) * synth.interior(cg, vol(Xc, cg))).sum(axis=(1, 2))
    coarse = (synth.interior(pg, qp)[:, :8, :8] * synth.interior(pg, vol(Xp, pg))[:8, :8]).sum(axis=(1, 2))
    assert np.allclose(coarse, fine, rtol=1e-14, atol=0)
    qc[:] = 0.7
    orc.fmr_restrict(pg, qp, cg, qc)
    assert np.allclose(synth.interior(pg, qp)[:, :8, :8], 0.7, rtol=1e-15, atol=0)


def child_ghosts(cg, nbuf=0):
    """Index arrays of the child's cross-shaped EXTERNAL halo (x-high,
    z-high sides) and of its nbuf interior rows/columns next to them."""
    ng, nx, nz = cg["ng"], cg["nx"], cg["nz"]
    ks, js = [], []
    for m in range(-nbuf, ng):
        for k in range(nz):
            ks.append(ng + k); js.append(ng + nx + m)
        for j in range(nx - nbuf if m < 0 else nx):
            ks.append(ng + nz + m); js.append(ng + j)
    return np.array(ks), np.array(js)


@pytest.mark.parametrize("geom,nbuf", [("cyl", 0), ("cart", 0), ("cyl", 4), ("cart", 4)])
def test_prolong_linear_exact_and_quadratic_in_time(orc, geom, nbuf):
    pg, cg = synth.fmr_grids(2, 16, 1.0, geom=geom, outer="outflow", nbuf=nbuf)
    eos = synth.ideal_eos(GAM)
    Xp, Zp = synth.cell_coords(pg)
    Xc, Zc = synth.cell_coords(cg)
    coef = np.array([[1.0, 0.3, 0.2], [0.01, 0.02, -0.03], [0.02, 0.01, 0.01],
                     [-0.01, 0.03, 0.02], [0.5, 0.1, 0.2], [0.75, -0.05, 0.1]])

    def field(X, Z, t):
        p = np.zeros((6,) + X.shape)
        for c in range(6):
            # linear in space, quadratic and monotone in time on [0, 2]
            p[c] = (coef[c, 0] + coef[c, 1] * X + coef[c, 2] * Z) * (1.0 + 0.1 * t + 0.02 * t * t)
        return p
    times = [0.0, 1.0, 2.0]
    slices = [np.ascontiguousarray(field(Xp, Zp, t)) for t in times]
    t = 1.37
    pc = synth.empty_fields(cg, 6)
    qc = synth.empty_fields(cg, 5)
    orc.fmr_prolong(pg, slices, times, t, cg, eos, {}, pc, qc, nbuf=nbuf)
    ks, js = child_ghosts(cg, nbuf)
    # nothing else is written
    touched = np.zeros(pc.shape[1:], dtype=bool)
    touched[ks, js] = True
    assert not np.any(pc[:, ~touched])
    # the parent's own ghosts across its low sides are mirror images, not
    # the linear continuation: keep child ghosts whose parent stencil stays
    # inside the parent (parent cell j, k >= 1, i.e. child j, k >= 2)
    ng = cg["ng"]
    keep = (js - ng >= 2) & (ks - ng >= 2)
    ks, js = ks[keep], js[keep]
    want = field(Xc, Zc, t)
    for c in range(6):
        got = pc[c][ks, js]
        ref = want[c][ks, js]
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-15), c
    # the conserved values are the prim->con map of the prolonged primitives
    for kk, jj in list(zip(ks, js))[:20]:
        x = Xc[kk, jj]
        q = orc.prim2con_point(eos, orc.metric_point({}), x, geom, pc[:, kk, jj])
        assert np.allclose(qc[:, kk, jj], q, rtol=1e-15, atol=0)


def test_prolong_time_limiter_and_extremum(orc):
    pg, cg = synth.fmr_grids(2, 16, 1.0, geom="cart", outer="outflow")
    eos = synth.ideal_eos(GAM)
    base = synth.empty_fields(pg, 6)
    base[0], base[4], base[5] = 1.0, 1.0, 1.5
    # non-monotone in time: rho goes 1.0 -> 1.2 -> 1.1
    s0, s1, s2 = base.copy(), base.copy(), base.copy()
    s1[0] = 1.2
    s2[0] = 1.1
    pc = synth.empty_fields(cg, 6)
    qc = synth.empty_fields(cg, 5)
    orc.fmr_prolong(pg, [s0, s1, s2], [0.0, 1.0, 2.0], 1.5, cg, eos, {}, pc, qc)
    ks, js = child_ghosts(cg)
    assert np.allclose(pc[0][ks, js], 1.15, rtol=1e-15)
    # monotone quadratic through (0, 1.0), (1, 1.2), (2, 1.5) at t = 1.5
    s2[0] = 1.5
    orc.fmr_prolong(pg, [s0, s1, s2], [0.0, 1.0, 2.0], 1.5, cg, eos, {}, pc, qc)
    assert np.allclose(pc[0][ks, js], 1.0 + 0.15 * 1.5 + 0.05 * 1.5 * 1.5, rtol=1e-15)
    # a single slice is used as it is; a local maximum in x gives a flat
    # prolongation in x
    one = base.copy()
    ng = pg["ng"]
    one[0, ng + 2, ng + 8] = 2.0      # parent cell (j=8, k=2) of ghosts (16..17, 4..5)
    orc.fmr_prolong(pg, [one], [0.0], 0.0, cg, eos, {}, pc, qc)
    for kf in (4, 5):
        for jf in (16, 17):
            assert pc[0][ng + kf, ng + jf] == pytest.approx(2.0, rel=1e-15)


def composite_totals(orc, drv):
    """sum(q_D dV) and sum(q_Sphi dV) over the composite grid: each level's
    own cells without the lower-left quarter its child covers."""
    M = J = 0.0
    n = len(drv.lev)
    for l, L in enumerate(drv.lev):
        g = drv.own(l)
        q = synth.interior(g, L["q"])
        X, _ = synth.cell_coords(g)
        x = synth.interior(g, X)
        dV = (2.0 * math.pi * x if g["geom"] == "cyl" else np.ones_like(x)) * g["dx"] * g["dz"]
        mask = np.ones_like(x, dtype=bool)
        if l + 1 < n:
            cg = drv.own(l + 1)
            mask[:cg["nz"] // 2, :cg["nx"] // 2] = False
        M += float((q[0] * dV)[mask].sum())
        J += float((q[2] * dV)[mask].sum())
    return M, J


def make_driver(orc, geom, nlev, l_fix=0, n=16, nbuf=0):
    grids = synth.fmr_grids(nlev, n, 1.0, geom=geom, outer="reflect", nbuf=nbuf)
    eos = synth.ideal_eos(GAM)
    levels = []
    for l, g in enumerate(grids):
        p = synth.blast_state(g, (0.3, 0.2), 0.15, 7)
        q = orc.prim2con(g, eos, {}, p, with_ghosts=True)
        levels.append(dict(grid=g, metric={}, q=q, nbuf=nbuf if l > 0 else 0))
    return orc.FmrDriver(levels, eos, OPTS, l_fix=l_fix), grids


@pytest.mark.parametrize("geom,nbuf", [("cart", 0), ("cyl", 0), ("cart", 4), ("cyl", 4)])
def test_bo_step_conserves_mass_and_angular_momentum(orc, geom, nbuf):
    drv, grids = make_driver(orc, geom, 3, nbuf=nbuf)
    M0, J0 = composite_totals(orc, drv)
    dt = 0.4 * grids[-1]["dx"] * 2 ** (len(grids) - 1)
    for _ in range(2):
        drv.step(dt)
    M1, J1 = composite_totals(orc, drv)
    assert abs(M1 - M0) <= 1e-13 * abs(M0), (M0, M1)
    assert abs(J1 - J0) <= 1e-13 * max(abs(J0), abs(M0)), (J0, J1)
    # the fine levels did evolve: the blast crosses the refinement boundary
    q2 = synth.interior(grids[2], drv.lev[2]["q"])
    assert np.abs(q2[1]).max() > 1e-3


@pytest.mark.parametrize("nbuf", [0, 4])
def test_bo_step_without_flux_correction_loses_mass(orc, monkeypatch, nbuf):
    drv, grids = make_driver(orc, "cart", 2, nbuf=nbuf)
    M0, _ = composite_totals(orc, drv)
    monkeypatch.setattr(orc, "fmr_reflux", lambda *a, **k: None)
    dt = 0.4 * grids[-1]["dx"] * 2
    for _ in range(2):
        drv.step(dt)
    M1, _ = composite_totals(orc, drv)
    assert abs(M1 - M0) > 1e-9 * abs(M0), (M0, M1)


@pytest.mark.parametrize("l_fix,want", [(0, [(0, 1), (1, 2), (2, 4)]), (1, [(0, 1), (1, 1), (2, 2)])])
def test_bo_schedule(orc, monkeypatch, l_fix, want):
    drv, grids = make_driver(orc, "cart", 3, l_fix=l_fix, n=8)
    calls = []
    real = drv._step

    def spy(l, t, dt):
        calls.append((l, t, dt))
        return real(l, t, dt)
    monkeypatch.setattr(drv, "_step", spy)
    drv.step(0.01)
    for l, count in want:
        mine = [c for c in calls if c[0] == l]
        assert len(mine) == count, (l, mine)
        assert all(c[2] == pytest.approx(0.01 / count) for c in mine)
        assert [c[1] for c in mine] == pytest.approx([i * 0.01 / count for i in range(count)])


def test_buffer_schedule_stage_mapping(orc, monkeypatch):
    """One coarse step of two levels under the buffer schedule: the child's
    two steps each prolong (buffer + ghosts at t, then ghosts at t + dt)
    and run two stages on the grid with its buffer and the last on its own
    cells; the parent's three stages run on its whole grid."""
    drv, grids = make_driver(orc, "cart", 2, n=8, nbuf=4)
    pro, sub = [], []
    real_pro, real_sub = orc.fmr_prolong, orc.rk_substep

    def spy_pro(pgrid, slices, times, t, cgrid, *a, nbuf=0):
        pro.append((round(t, 12), nbuf))
        return real_pro(pgrid, slices, times, t, cgrid, *a, nbuf=nbuf)

    def spy_sub(grid, *a, **k):
        sub.append((grid["nx"], grid["nz"]))
        return real_sub(grid, *a, **k)
    monkeypatch.setattr(orc, "fmr_prolong", spy_pro)
    monkeypatch.setattr(orc, "rk_substep", spy_sub)
    dt = 0.02
    drv.step(dt)
    h = dt / 2
    assert pro == [(0.0, 4), (round(h, 12), 0), (round(h, 12), 4), (round(2 * h, 12), 0)]
    assert sub == [(8, 8)] * 3 + [(12, 12), (12, 12), (8, 8)] * 2


@pytest.mark.parametrize("nbuf", [0, 4])
def test_uniform_state_stays_uniform(orc, nbuf):
    grids = synth.fmr_grids(3, 16, 1.0, geom="cart", outer="reflect", nbuf=nbuf)
    eos = synth.ideal_eos(GAM)
    levels = []
    for l, g in enumerate(grids):
        p = synth.empty_fields(g, 6)
        p[0], p[4] = 1.3, 0.7
        p[5] = p[4] / ((GAM - 1.0) * p[0])
        levels.append(dict(grid=g, metric={}, q=orc.prim2con(g, eos, {}, p, with_ghosts=True),
                           nbuf=nbuf if l > 0 else 0))
    drv = orc.FmrDriver(levels, eos, OPTS)
    q0 = [synth.interior(drv.own(l), L["q"]).copy() for l, L in enumerate(drv.lev)]
    for _ in range(2):
        drv.step(0.4 * grids[0]["dx"])
    for l, L in enumerate(drv.lev):
        q = synth.interior(drv.own(l), L["q"])
        for c in (0, 4):
            assert np.abs(q[c] - q0[l][c]).max() <= 1e-14 * q0[l][c].max(), (l, c)
        for c in (1, 2, 3):
            assert np.abs(q[c]).max() <= 1e-14, (l, c)
