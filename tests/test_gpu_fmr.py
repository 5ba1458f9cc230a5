"""GPU: the mesh-refinement calls against the oracle (Sec. II.A, II.E).

- prolongation: child ghost primitives bit for bit (the same operations in
  the same order on both sides), conserved values to 1e-14, for one, two
  and three parent slices and for flat, star and general child metrics;
- restriction and flux correction bit for bit;
- the Berger-Oliger driver: every level after two coarse steps within
  1e-12 of the oracle's driver (per field, normwise), with and without
  l_fix, on a blast crossing two refinement boundaries and on a star whose
  surface the finest boundary cuts; composite mass conserved to round-off
  in a closed box.  Both boundary schedules: the halo (ghost cells
  prolonged before every stage) and the paper's (4+4) buffer (nbuf = 4).
"""
import math

import numpy as np
import pytest

import synth
from cmp import percell_local

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_03223_amd import grhd  # noqa: E402

DEV = torch.device("cuda:0")
GAM = 5.0 / 3.0
OPTS = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=dict(w_max=100.0, rho_atm=1e-12))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def mdev(metric):
    return {k: dev(v) if isinstance(v, np.ndarray) else v for k, v in metric.items()}


def normwise(g, o):
    worst = 0.0
    for c in range(g.shape[0]):
        scale = np.abs(o[c]).max()
        d = np.abs(g[c] - o[c]).max()
        worst = max(worst, d if scale == 0.0 else d / scale)
    return worst


def parent_slices(pg, nslice, seed):
    rng = np.random.default_rng(seed)
    base = synth.blast_state(pg, (0.45, 0.3), 0.2, seed)
    out = []
    for s in range(nslice):
        p = base.copy()
        p[0] *= 1.0 + 0.05 * s + 0.01 * rng.uniform(-1, 1, size=p[0].shape)
        p[4] *= 1.0 + 0.03 * s + 0.01 * rng.uniform(-1, 1, size=p[0].shape)
        for c in (1, 2, 3):
            p[c] += 0.01 * rng.uniform(-1, 1, size=p[0].shape)
        p[5] = p[4] / ((GAM - 1.0) * p[0])
        out.append(np.ascontiguousarray(p))
    return out


@pytest.mark.parametrize("nslice", [1, 2, 3])
@pytest.mark.parametrize("case", ["flat_cart", "star_cyl", "general_cart"])
def test_prolong_parity(orc, nslice, case):
    geom = "cyl" if case == "star_cyl" else "cart"
    pg, cg = synth.fmr_grids(2, 24, 1.0, geom=geom, outer="outflow")
    eos = synth.ideal_eos(GAM)
    if case == "flat_cart":
        cm = {}
    elif case == "star_cyl":
        cm = dict(alp=0.8 + 0.1 * synth.cell_coords(cg)[0], W=0.9 + 0.05 * synth.cell_coords(cg)[1])
        cm = {k: np.ascontiguousarray(v) for k, v in cm.items()}
    else:
        cm = synth.general_metric(cg, 5, amp=0.05)
    sl = parent_slices(pg, nslice, 11 + nslice)
    times = [0.0, 0.7, 1.5][:nslice]
    t = 1.1 if nslice == 3 else (0.4 if nslice == 2 else 0.0)
    p_o = synth.empty_fields(cg, 6)
    q_o = synth.empty_fields(cg, 5)
    orc.fmr_prolong(pg, sl, times, t, cg, eos, cm, p_o, q_o)
    p_g = torch.zeros((6,) + p_o.shape[1:], dtype=torch.float64, device=DEV)
    q_g = torch.zeros((5,) + p_o.shape[1:], dtype=torch.float64, device=DEV)
    grhd.fmr_prolong(pg, [dev(s) for s in sl], times, t, cg, mdev(cm), eos, OPTS["c2p"]["rho_atm"], p_g, q_g)
    torch.cuda.synchronize()
    assert np.array_equal(p_g.cpu().numpy(), p_o)
    assert normwise(q_g.cpu().numpy(), q_o) <= 1e-14
    assert np.any(p_o[0] != 0.0)


@pytest.mark.parametrize("geom", ["cyl", "cart"])
def test_restrict_and_reflux_parity(orc, geom):
    pg, cg = synth.fmr_grids(2, 32, 1.0, geom=geom, outer="outflow")
    rng = np.random.default_rng(5)
    qc = synth.empty_fields(cg, 5)
    qc[:] = rng.uniform(0.5, 2.0, size=qc.shape)
    qp = synth.empty_fields(pg, 5)
    qp[:] = rng.uniform(0.5, 2.0, size=qp.shape)
    qp_o = qp.copy()
    orc.fmr_restrict(pg, qp_o, cg, qc)
    qp_g = dev(qp)
    grhd.fmr_restrict(pg, qp_g, cg, dev(qc))
    torch.cuda.synchronize()
    assert np.array_equal(qp_g.cpu().numpy(), qp_o)
    J, K = cg["nx"] // 2, cg["nz"] // 2
    preg = rng.normal(size=5 * (J + K))
    creg = rng.normal(size=5 * (cg["nx"] + cg["nz"]))
    orc.fmr_reflux(pg, qp_o, preg, cg, creg)
    grhd.fmr_reflux(pg, qp_g, dev(preg), cg, dev(creg))
    torch.cuda.synchronize()
    assert np.array_equal(qp_g.cpu().numpy(), qp_o)


def own(g, nbuf):
    return dict(g, nx=g["nx"] - nbuf, nz=g["nz"] - nbuf)


def composite_mass(levels_q, grids, nbuf=0):
    M = 0.0
    grids = [own(g, nbuf if l > 0 else 0) for l, g in enumerate(grids)]
    for l, (g, q) in enumerate(zip(grids, levels_q)):
        qi = synth.interior(g, q)
        X, _ = synth.cell_coords(g)
        x = synth.interior(g, X)
        dV = (2.0 * math.pi * x if g["geom"] == "cyl" else np.ones_like(x)) * g["dx"] * g["dz"]
        mask = np.ones_like(x, dtype=bool)
        if l + 1 < len(grids):
            mask[:grids[l + 1]["nz"] // 2, :grids[l + 1]["nx"] // 2] = False
        M += float((qi[0] * dV)[mask].sum())
    return M


def run_pair(orc, grids, eos, metrics, prims, l_fix, dt, nstep, nbuf=0, gpu_opts=None):
    qs = [orc.prim2con(g, eos, m, p, with_ghosts=True) for g, m, p in zip(grids, metrics, prims)]
    nb = [nbuf if l > 0 else 0 for l in range(len(grids))]
    drv = orc.FmrDriver([dict(grid=g, metric=m, q=q, nbuf=b) for g, m, q, b in zip(grids, metrics, qs, nb)],
                        eos, OPTS, l_fix=l_fix)
    lev_g = [dict(grid=g, metric=mdev(m), q=dev(q), nbuf=b) for g, m, q, b in zip(grids, metrics, qs, nb)]
    h = grhd.Hierarchy(lev_g, eos, gpu_opts or OPTS, l_fix=l_fix)
    M0 = composite_mass([L["q"] for L in drv.lev], grids, nbuf)
    for _ in range(nstep):
        drv.step(dt)
        h.step(dt)
    torch.cuda.synchronize()
    out_g = [L["q"].cpu().numpy() for L in lev_g]
    out_o = [L["q"] for L in drv.lev]
    h.close()
    return out_g, out_o, M0


def reach(level, l_fix, coarse_steps):
    """Cells the stencil reaches on a level over a run: 3 per Runge-Kutta
    stage, 3 stages per step, 2 steps per parent step below l_fix."""
    steps = coarse_steps
    for m in range(1, level + 1):
        steps *= 1 if m <= l_fix else 2
    return 9 * steps


@pytest.mark.parametrize("nbuf", [0, 4])
@pytest.mark.parametrize("l_fix", [0, 1])
@pytest.mark.parametrize("geom", ["cart", "cyl"])
def test_hierarchy_blast_parity_and_conservation(orc, geom, l_fix, nbuf):
    grids = synth.fmr_grids(3, 32, 1.0, geom=geom, outer="reflect", nbuf=nbuf)
    eos = synth.ideal_eos(GAM)
    prims = [synth.blast_state(g, (0.3, 0.2), 0.15, 7) for g in grids]
    # the finest level keeps a Courant factor of 0.4
    dt = 0.4 * grids[0]["dx"] / 2 ** min(l_fix, 2)
    out_g, out_o, M0 = run_pair(orc, grids, eos, [{}] * 3, prims, l_fix, dt, 2, nbuf)
    for l, g in enumerate(grids):
        e = normwise(synth.interior(g, out_g[l]), synth.interior(g, out_o[l]))
        assert e <= 1e-12, (l, e)
        e = percell_local(synth.interior(g, out_g[l]), synth.interior(g, out_o[l]), (0, 4),
                          radius=reach(l, l_fix, 2))
        assert e <= 1e-12, (l, e)
    M_g = composite_mass(out_g, grids, nbuf)
    assert abs(M_g - M0) <= 1e-13 * abs(M0), (M0, M_g)


@pytest.mark.parametrize("nbuf", [0, 4])
def test_hierarchy_star_parity(orc, nbuf):
    """The TOV star on three levels whose finest boundary cuts the star."""
    tov = synth.tov_solve()
    grids = synth.fmr_grids(3, 32, 40.0, geom="cyl", outer="outflow", nbuf=nbuf)
    prims, metrics = [], []
    eos = None
    for l, g in enumerate(grids):
        p, m, eos = synth.star_problem(g, seed=90 + l, tov=tov, vel=0.02)
        prims.append(p)
        metrics.append(m)
    opts_star = dict(OPTS, c2p=dict(w_max=100.0, rho_atm=1e-10))
    qs = [orc.prim2con(g, eos, m, p, with_ghosts=True) for g, m, p in zip(grids, metrics, prims)]
    nb = [nbuf if l > 0 else 0 for l in range(3)]
    drv = orc.FmrDriver([dict(grid=g, metric=m, q=q, nbuf=b) for g, m, q, b in zip(grids, metrics, qs, nb)],
                        eos, opts_star)
    lev_g = [dict(grid=g, metric=mdev(m), q=dev(q), nbuf=b) for g, m, q, b in zip(grids, metrics, qs, nb)]
    h = grhd.Hierarchy(lev_g, eos, opts_star)
    dt = 0.4 * grids[0]["dx"]
    for _ in range(2):
        drv.step(dt)
        h.step(dt)
    torch.cuda.synchronize()
    for l, g in enumerate(grids):
        e = normwise(synth.interior(g, lev_g[l]["q"].cpu().numpy()), synth.interior(g, drv.lev[l]["q"]))
        assert e <= 1e-12, (l, e)
        e = percell_local(synth.interior(g, lev_g[l]["q"].cpu().numpy()), synth.interior(g, drv.lev[l]["q"]),
                          (0, 4), radius=reach(l, 0, 2))
        assert e <= 1e-12, (l, e)
    assert h.time == pytest.approx(2 * dt)
    h.close()


@pytest.mark.parametrize("nbuf", [0, 4])
def test_hierarchy_with_learned_guess(orc, nbuf):
    """The blast on three cylindrical levels with every level's recovery
    seeded by the learned guess: the levels after two coarse steps equal the
    oracle's driver (which recovers from the bracket alone) to the bars of
    the unseeded driver, and composite mass is conserved to round-off (the
    guess moves only where each root search starts)."""
    from test_gpu_mlp import train
    net, _ = train(orc, n=100_000, epochs=4)
    grids = synth.fmr_grids(3, 32, 1.0, geom="cyl", outer="reflect", nbuf=nbuf)
    eos = synth.ideal_eos(GAM)
    prims = [synth.blast_state(g, (0.3, 0.2), 0.15, 7) for g in grids]
    dt = 0.4 * grids[0]["dx"]
    seeded = dict(OPTS, c2p=dict(OPTS["c2p"], mlp=net.buf))
    out_g, out_o, M0 = run_pair(orc, grids, eos, [{}] * 3, prims, 0, dt, 2, nbuf, gpu_opts=seeded)
    for l, g in enumerate(grids):
        e = normwise(synth.interior(g, out_g[l]), synth.interior(g, out_o[l]))
        assert e <= 1e-12, (l, e)
        e = percell_local(synth.interior(g, out_g[l]), synth.interior(g, out_o[l]), (0, 4),
                          radius=reach(l, 0, 2))
        assert e <= 1e-12, (l, e)
    M_g = composite_mass(out_g, grids, nbuf)
    assert abs(M_g - M0) <= 1e-13 * abs(M0), (M0, M_g)
