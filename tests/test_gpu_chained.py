"""GPU: the chained stage (grhd_rk_substep_chained) against the oracle.

A whole SSP-RK3 step runs as one recovery pass and three chained stages.
After each stage the stored q_out and its recovery flags must equal the
oracle's stage followed by the oracle's recovery of the result (per field
1e-12 normwise, and per cell on D and E against the largest value the
stencil reaches; flags exact), and the primitives must equal the oracle's
recovery of the stored q_out (1e-12 normwise and per cell on rho, on P
and eps scaled by the recovery's conditioning: the recovery on identical
input; the
primitives of a slowly moving cell amplify the 1e-16-level differences of
its conserved state, so the end-to-end comparison goes through q); the
boundary fluxes equal the oracle's; the diagnostics carry the stage's
Courant number, the recovery counts of q_out and the sums of the stored
state.
"""
import math

import numpy as np
import pytest

import synth
from cmp import normwise, percell, percell_cond, percell_local

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_03223_amd import grhd  # noqa: E402

DEV = torch.device("cuda:0")
C2P_STAR = dict(w_max=100.0, rho_atm=1e-10)
C2P_RIE = dict(w_max=100.0, rho_atm=1e-12)
TOL = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def mdev(metric):
    return {k: dev(v) if isinstance(v, np.ndarray) else v for k, v in metric.items()}


def sums(grid, q):
    """Sums of q_D dV and q_Sphi dV over the interior (cell volumes of the
    grid's geometry)."""
    qi = synth.interior(grid, q)
    nx = grid["nx"]
    x = grid["x0"] + (np.arange(nx) + 0.5) * grid["dx"]
    if grid["geom"] == "cyl":
        dV = 2.0 * math.pi * x * grid["dx"] * grid["dz"]
    else:
        dV = np.full(nx, grid["dx"] * grid["dz"])
    return float((qi[0] * dV).sum()), float((qi[2] * dV).sum())


def run_step(orc, grid, eos, metric, opts, q0, dt, acc=None):
    """One SSP-RK3 step (or the stages of `acc`) chained on the GPU and
    stage by stage in the oracle; checks after every stage."""
    I = lambda a: synth.interior(grid, a)  # noqa: E731
    c2p = opts["c2p"]
    sub = grhd.Substep(grid, eos, mdev(metric), opts)
    shp = q0.shape[1:]
    qg = [dev(q0)] + [torch.zeros_like(dev(q0)) for _ in range(3)]
    pg = [torch.zeros((6,) + shp, dtype=torch.float64, device=DEV) for _ in range(2)]
    fg = [torch.zeros(shp, dtype=torch.uint8, device=DEV) for _ in range(2)]
    nb = 2 * grid["nz"] + 2 * grid["nx"]
    freg = torch.zeros(5 * nb, dtype=torch.float64, device=DEV)
    grhd.con2prim(grid, eos, mdev(metric), c2p, qg[0], pg[0], flags=fg[0])
    # oracle: each stage recovers its raw q_s first
    r = orc.rk_substep(grid, eos, metric, opts, dict(grhd.SSPRK3[0], dt=dt), q0, q0)
    qn_o = r["qs"]
    qs_raw = q0
    stages = [dict(s, dt=dt) for s in grhd.SSPRK3] if acc is None else acc["stages"]
    cur = 0
    for i, st in enumerate(stages):
        dg = grhd.new_diag()
        ai = dev(acc["in"]) if acc is not None else None
        ao = torch.zeros_like(qg[0]) if acc is not None else None
        qs_g = qg[0] if i == 0 else qg[i]
        out = qg[i + 1]
        sub.chained(st, qg[0], qs_g, out, pg[cur], fg[cur], pg[1 - cur], fg[1 - cur],
                    acc_in=ai, acc_out=ao, flux_reg=freg, diag=dg)
        ref = orc.rk_substep(grid, eos, metric, opts, st, qn_o, qs_raw, acc_in=acc["in"] if acc else None,
                             want_acc=acc is not None)
        p_r, q_r, fl_r, d_r = orc.con2prim(grid, eos, metric, c2p, ref["qout"])
        torch.cuda.synchronize()
        cur = 1 - cur
        q_g = out.cpu().numpy()
        e_q = normwise(I(q_g), I(q_r))
        assert e_q <= TOL, (i, e_q)
        e_c = percell_local(I(q_g), I(q_r), (0, 4))
        assert e_c <= TOL, (i, e_c)
        # the recovery itself on identical input: the oracle recovers the
        # GPU's stored q_out (a recovery maps its own corrected output to
        # the same primitives up to rounding)
        p_same = orc.con2prim(grid, eos, metric, c2p, q_g)[0]
        e_p = normwise(I(pg[cur].cpu().numpy()), I(p_same))
        assert e_p <= TOL, (i, e_p)
        e_pc = percell(I(pg[cur].cpu().numpy()), I(p_same), (0,))
        assert e_pc <= TOL, (i, e_pc)
        e_pk = percell_cond(I(pg[cur].cpu().numpy()), I(p_same), I(q_g))
        assert e_pk <= TOL, (i, e_pk)
        assert np.array_equal(I(fg[cur].cpu().numpy()), I(fl_r)), i
        fr, fo = freg.cpu().numpy().reshape(5, nb), ref["flux_reg"]
        assert np.abs(fr - fo).max() <= TOL * np.abs(fo).max(), i
        if acc is not None:
            assert normwise(I(ao.cpu().numpy()), I(ref["acc"])) <= TOL
        d = grhd.read_diag(dg)
        assert d["max_courant"] == pytest.approx(ref["diag"]["max_courant"], rel=1e-12)
        mb, jm = sums(grid, q_r)
        assert d["Mb"] == pytest.approx(mb, rel=1e-12)
        assert d["J"] == pytest.approx(jm, rel=1e-12, abs=1e-12 * abs(mb))
        for k in ("n_rescale", "n_cold", "n_atm", "n_fail"):
            assert d[k] == d_r[k], (i, k)
        qs_raw = ref["qout"]


@pytest.fixture(scope="module")
def tov():
    return synth.tov_solve()


@pytest.mark.parametrize("n", [64, 93])
def test_chained_star_step(orc, tov, n):
    grid = synth.star_grid(n)
    p, metric, eos = synth.star_problem(grid, seed=70 + n, tov=tov, vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR)
    run_step(orc, grid, eos, metric, opts, q, 0.4 * grid["dx"])


@pytest.mark.parametrize("riemann", ["hllc", "tvdlf"])
def test_chained_riemann_step(orc, riemann):
    gam = 5.0 / 3.0
    (L, R), = synth.riemann_states(5, 1, gam)
    grid = synth.riemann_grid(400, nz=8)
    eos = synth.ideal_eos(gam)
    q = orc.prim2con(grid, eos, {}, synth.riemann_prims(grid, L, R), with_ghosts=True)
    opts = dict(recon="ppm", riemann=riemann, prec="fp64", c2p=C2P_RIE)
    run_step(orc, grid, eos, {}, opts, q, 0.4 * grid["dx"])


def test_chained_general_metric_hybrid(orc):
    """General metric (shift, conformal metric, curvature) and the
    two-piece hybrid EOS: the recovery instance of the other class."""
    grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
    metric = synth.general_metric(grid, 9)
    p = synth.smooth_state(grid, 10, vamp=0.5)
    eos = dict(kind="hybrid", K=[0.3, 0.3 * 0.9 ** (1.4 - 2.2)], G=[1.4, 2.2], rho_b=[0.9], Gth=5.0 / 3.0)
    rho = p[0]
    ecold = np.where(rho < 0.9, 0.3 / 0.4 * rho ** 0.4,
                     eos["K"][1] / 1.2 * rho ** 1.2 + (0.3 / 0.4 * 0.9 ** 0.4 - eos["K"][1] / 1.2 * 0.9 ** 1.2))
    p[5] = ecold + 0.2
    p[4] = np.array([orc.eos_press(eos, r, e) for r, e in zip(rho.ravel(), p[5].ravel())]).reshape(rho.shape)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_RIE)
    run_step(orc, grid, eos, metric, opts, q, 0.005)


def test_chained_rk4_accumulator(orc, tov):
    grid = synth.star_grid(40)
    p, metric, eos = synth.star_problem(grid, seed=81, tov=tov, vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    acc = orc.prim2con(grid, eos, metric, synth.star_problem(grid, seed=82, tov=tov, vel=0.05)[0],
                       with_ghosts=True) * 1e-3
    dt = 0.4 * grid["dx"]
    stages = [dict(a=1.0, b=0.0, c=0.5, dt=dt, g=0.0, d=1.0, e=1.0 / 3.0),
              dict(a=1.0, b=0.0, c=1.0 / 6.0, dt=dt, g=1.0, d=0.0, e=0.0)]
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR)
    run_step(orc, grid, eos, metric, opts, q, dt, acc=dict(stages=stages, **{"in": acc}))


def test_chained_equals_unchained(orc, tov):
    """Chained and unchained stages compute the same numbers: after one
    stage and one recovery they agree to rounding, in FP64 and in mixed
    precision."""
    grid = synth.star_grid(77)
    p, metric, eos = synth.star_problem(grid, seed=83, tov=tov, vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    md = mdev(metric)
    st = dict(grhd.SSPRK3[0], dt=0.4 * grid["dx"])
    shp = q.shape[1:]
    for prec in ("fp64", "mixed"):
        opts = dict(recon="ppm", riemann="hllc", prec=prec, c2p=C2P_STAR)
        sub = grhd.Substep(grid, eos, md, opts)
        # unchained: stage (with its own leading recovery), then recovery of q_out
        qa = dev(q)
        oa = torch.zeros_like(qa)
        pa = torch.zeros((6,) + shp, dtype=torch.float64, device=DEV)
        sub(st, qa, qa, oa, pa)
        pa2 = torch.zeros_like(pa)
        fa2 = torch.zeros(shp, dtype=torch.uint8, device=DEV)
        grhd.con2prim(grid, eos, md, C2P_STAR, oa, pa2, flags=fa2)
        # chained: recovery, then the stage with the recovery of q_out
        qb = dev(q)
        pb = torch.zeros_like(pa)
        fb = torch.zeros(shp, dtype=torch.uint8, device=DEV)
        grhd.con2prim(grid, eos, md, C2P_STAR, qb, pb, flags=fb)
        ob = torch.zeros_like(qb)
        pb2 = torch.zeros_like(pa)
        fb2 = torch.zeros(shp, dtype=torch.uint8, device=DEV)
        sub.chained(st, qb, qb, ob, pb, fb, pb2, fb2)
        torch.cuda.synchronize()
        I = lambda a: synth.interior(grid, a.cpu().numpy())  # noqa: E731
        assert normwise(I(ob), I(oa)) <= 1e-14, prec
        assert normwise(I(pb2), I(pa2)) <= 1e-14, prec
        assert np.array_equal(I(fb2), I(fa2)), prec
