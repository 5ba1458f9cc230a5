"""GPU parity: every C-ABI call of libgrhd.so against the FP64 oracle on the
same seeded inputs (run on an MI355X).

Bar (FP64 path): per field, max|gpu - oracle| <= 1e-12 max|oracle| (the
normwise reading of "1e-12 relative"), and per cell on the positive
fields, so a low-density or atmosphere cell cannot hide behind the stellar
scale: D and E of the stage output within 1e-12 of the largest value its
stencil reaches (tests/cmp.py), D and E of the corrected input and the
recovered rho within 1e-12 of the cell's own value, the recovered P and
eps within 1e-12 max(1, kappa 1e-2) of it (kappa = (E/D)^2 / eps: the
conditioning of eps at the root); reconstruction is
bitwise (both sides evaluate the limiters without fused multiply-add on
identical inputs); recovery flags are bit-exact.  Stage tests run the
paper's face states (every primitive reconstructed) and, where marked, the
EOS face variant.  Sizes span several tiles with ragged tails; full-size
star grids (512^2, 1024^2) are compared on every cell.
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


@pytest.fixture(scope="module")
def tov():
    return synth.tov_solve()


def star_case(n, seed, tov, vel=0.02, extent=20.0):
    grid = synth.star_grid(n, extent=extent)
    p, metric, eos = synth.star_problem(grid, seed=seed, tov=tov, vel=vel)
    return grid, p, metric, eos


# two-piece hybrid EOS (K != 1 in both pieces, so a misplaced K shows)
HYBRID = dict(kind="hybrid", K=[0.3, 0.3 * 0.9 ** (1.4 - 2.2)], G=[1.4, 2.2], rho_b=[0.9], Gth=5.0 / 3.0)


def hybrid_state(orc, p):
    """p with eps = eps_cold(rho) + 0.2 and P from the hybrid EOS."""
    rho = p[0]
    K1 = HYBRID["K"][1]
    ecold = np.where(rho < 0.9, 0.3 / 0.4 * rho ** 0.4,
                     K1 / 1.2 * rho ** 1.2 + (0.3 / 0.4 * 0.9 ** 0.4 - K1 / 1.2 * 0.9 ** 1.2))
    p[5] = ecold + 0.2
    p[4] = np.array([orc.eos_press(HYBRID, r, e) for r, e in zip(rho.ravel(), p[5].ravel())]).reshape(rho.shape)
    return p


# ------------------------------------------------------------ pointwise calls

@pytest.mark.parametrize("case", ["star", "general"])
def test_prim2con(orc, tov, case):
    if case == "star":
        grid, p, metric, eos = star_case(70, 3, tov)
    else:
        grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
        metric = synth.general_metric(grid, 1)
        p = synth.smooth_state(grid, 2)
        eos = synth.ideal_eos(5.0 / 3.0)
    q_o = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    q_g = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=DEV)
    grhd.prim2con(grid, eos, mdev(metric), dev(p), q_g, with_ghosts=True)
    assert normwise(q_g.cpu().numpy(), q_o) <= 1e-14


@pytest.mark.parametrize("case", ["star", "general", "hybrid"])
def test_con2prim(orc, tov, case):
    if case == "star":
        grid, p, metric, eos = star_case(70, 4, tov, vel=0.1)
        c2p = C2P_STAR
    else:
        grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
        metric = synth.general_metric(grid, 3)
        p = synth.smooth_state(grid, 4, vamp=0.8)
        eos = synth.ideal_eos(5.0 / 3.0)
        c2p = C2P_RIE
        if case == "hybrid":
            eos = HYBRID
            p = hybrid_state(orc, p)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    # a few pathological cells: invalid input, super-luminal momentum, cold
    qi = synth.interior(grid, q)
    qi[0, 1, 1] = -1.0
    qi[4, 2, 2] = np.nan
    qi[1, 3, 3] = 5.0 * qi[4, 3, 3]
    qi[4, 4, 4] = qi[0, 4, 4] * 0.5
    p_o, q_o, fl_o, d_o = orc.con2prim(grid, eos, metric, c2p, q)
    qg = dev(q)
    pg = torch.zeros((6,) + q.shape[1:], dtype=torch.float64, device=DEV)
    fl = torch.zeros(q.shape[1:], dtype=torch.uint8, device=DEV)
    dg = grhd.new_diag()
    grhd.con2prim(grid, eos, mdev(metric), c2p, qg, pg, flags=fl, diag=dg)
    torch.cuda.synchronize()
    assert np.array_equal(synth.interior(grid, fl.cpu().numpy()), synth.interior(grid, fl_o))
    pgi = synth.interior(grid, pg.cpu().numpy())
    assert np.all(np.isfinite(pgi))
    assert normwise(pgi, synth.interior(grid, p_o)) <= TOL
    assert percell(pgi, synth.interior(grid, p_o), (0,)) <= TOL
    assert percell_cond(pgi, synth.interior(grid, p_o), synth.interior(grid, q_o)) <= TOL
    assert normwise(synth.interior(grid, qg.cpu().numpy()), synth.interior(grid, q_o)) <= TOL
    d = grhd.read_diag(dg)
    for k in ("n_rescale", "n_cold", "n_atm", "n_fail"):
        assert d[k] == d_o[k], k


@pytest.mark.parametrize("recon", ["ppm", "minmod", "ppm3"])
@pytest.mark.parametrize("dirn", [0, 1])
def test_reconstruct_bitwise(orc, tov, recon, dirn):
    grid, p, metric, eos = star_case(70, 5, tov, vel=0.1)
    pf = orc.fill_ghosts(grid, p)
    L_o, R_o = orc.reconstruct(grid, dirn, recon, pf)
    pi = np.zeros_like(p)
    synth.interior(grid, pi)[...] = synth.interior(grid, p)
    L_g, R_g = grhd.reconstruct(grid, dirn, recon, dev(pi))
    assert np.array_equal(L_g.cpu().numpy(), L_o) and np.array_equal(R_g.cpu().numpy(), R_o)
    # FP32 path: same limiter algebra in single precision; a limiter branch
    # may flip on FP32 rounding, so require agreement on almost every face and
    # boundedness everywhere
    L_f, R_f = grhd.reconstruct(grid, dirn, recon, dev(pi), prec="mixed")
    for a, b in ((L_f.cpu().numpy(), L_o), (R_f.cpu().numpy(), R_o)):
        assert np.all(np.isfinite(a))
        close = np.abs(a - b) <= 2e-6 * np.abs(b) + 1e-30
        assert close.mean() >= 0.995


@pytest.mark.parametrize("riemann", ["hllc", "tvdlf"])
@pytest.mark.parametrize("dirn", [0, 1])
@pytest.mark.parametrize("case", ["star", "general", "hybrid"])
def test_flux(orc, tov, riemann, dirn, case):
    if case == "star":
        grid, p, metric, eos = star_case(70, 6, tov, vel=0.1)
    else:
        grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
        metric = synth.general_metric(grid, 5)
        p = synth.smooth_state(grid, 6, vamp=0.5)
        eos = synth.ideal_eos(5.0 / 3.0)
        if case == "hybrid":
            eos = HYBRID
            p = hybrid_state(orc, p)
    pf = orc.fill_ghosts(grid, p)
    L, R = orc.reconstruct(grid, dirn, "ppm", pf)
    F_o, s_o = orc.face_flux(grid, dirn, riemann, eos, metric, L, R)
    F_g, s_g = grhd.hllc_flux(grid, dirn, riemann, eos, mdev(metric), dev(L), dev(R))
    assert normwise(F_g.cpu().numpy(), F_o) <= 1e-13
    assert float(s_g.cpu()[0]) == pytest.approx(s_o, rel=1e-13)


# ------------------------------------------------------------ fused substep

def run_pair(orc, grid, eos, metric, opts, stage, qn, qs, acc_in=None, want_acc=False, tile=None):
    ref = orc.rk_substep(grid, eos, metric, opts, stage, qn, qs, acc_in=acc_in, want_acc=want_acc)
    o = dict(opts)
    if tile:
        o["tile"] = tile
    sub = grhd.Substep(grid, eos, mdev(metric), o)
    qs_g = dev(qs)
    qn_g = dev(qn) if qn is not None else qs_g
    qo = torch.zeros_like(qs_g)
    pg = torch.zeros((6,) + qs.shape[1:], dtype=torch.float64, device=DEV)
    nb = 2 * grid["nz"] + 2 * grid["nx"]
    freg = torch.zeros(5 * nb, dtype=torch.float64, device=DEV)
    fl = torch.zeros(qs.shape[1:], dtype=torch.uint8, device=DEV)
    dg = grhd.new_diag()
    ai = dev(acc_in) if acc_in is not None else None
    ao = torch.zeros_like(qs_g) if want_acc else None
    sub(stage, qn_g, qs_g, qo, pg, acc_in=ai, acc_out=ao, flux_reg=freg, flags=fl, diag=dg)
    torch.cuda.synchronize()
    out = dict(qout=qo.cpu().numpy(), qs=qs_g.cpu().numpy(), p=pg.cpu().numpy(),
               flux_reg=freg.cpu().numpy().reshape(5, nb), flags=fl.cpu().numpy(),
               diag=grhd.read_diag(dg), acc=ao.cpu().numpy() if want_acc else None)
    return ref, out


def check_pair(grid, ref, out, tol=TOL, flag_mask=0xFF):
    I = lambda a: synth.interior(grid, a)  # noqa: E731
    assert normwise(I(out["qout"]), I(ref["qout"])) <= tol
    assert normwise(I(out["qs"]), I(ref["qs"])) <= tol
    assert normwise(I(out["p"]), I(ref["p"])) <= tol
    # per cell on the positive fields: D, E; rho, P, eps
    assert percell_local(I(out["qout"]), I(ref["qout"]), (0, 4)) <= tol
    assert percell(I(out["qs"]), I(ref["qs"]), (0, 4)) <= tol
    assert percell(I(out["p"]), I(ref["p"]), (0,)) <= tol
    assert percell_cond(I(out["p"]), I(ref["p"]), I(ref["qs"])) <= tol
    assert np.array_equal(I(out["flags"]) & flag_mask, I(ref["flags"]) & flag_mask)
    # boundary fluxes: one scale for all components (the mass flux through
    # the axis and through a static atmosphere is rounding noise)
    fr, fo = out["flux_reg"], ref["flux_reg"]
    assert np.abs(fr - fo).max() <= tol * np.abs(fo).max()
    d, r = out["diag"], ref["diag"]
    assert d["max_courant"] == pytest.approx(r["max_courant"], rel=1e-12)
    assert d["Mb"] == pytest.approx(r["Mb"], rel=1e-12)
    assert d["J"] == pytest.approx(r["J"], rel=1e-12, abs=1e-12 * abs(r["Mb"]))
    for k in ("n_rescale", "n_cold", "n_atm", "n_fail"):
        assert d[k] == r[k], k
    if ref["acc"] is not None:
        assert normwise(I(out["acc"]), I(ref["acc"])) <= tol


@pytest.mark.parametrize("seed,face_eps", [(0, "recon"), (1, "recon"), (2, "recon"), (0, "eos")])
@pytest.mark.parametrize("riemann,recon", [("hllc", "ppm"), ("tvdlf", "ppm"), ("hllc", "minmod"),
                                           ("hllc", "ppm3")])
def test_substep_riemann(orc, seed, riemann, recon, face_eps):
    """Riemann problems on 400 x 8 (Cartesian, flat, periodic z), all three
    SSP-RK3 stages from oracle-evolved states."""
    gam = 5.0 / 3.0
    (L, R), = synth.riemann_states(seed, 1, gam)
    grid = synth.riemann_grid(400, nz=8)
    eos = synth.ideal_eos(gam)
    p = synth.riemann_prims(grid, L, R)
    q0 = orc.prim2con(grid, eos, {}, p, with_ghosts=True)
    opts = dict(recon=recon, riemann=riemann, prec="fp64", c2p=C2P_RIE, face_eps=face_eps)
    dt = 0.4 * grid["dx"]
    # evolve a few steps with the oracle so every stage starts from a
    # developed solution
    q = q0
    for _ in range(10):
        qn = q
        for st in grhd.SSPRK3:
            r = orc.rk_substep(grid, eos, {}, opts, dict(st, dt=dt), qn, q)
            qn = r["qs"] if st["a"] == 0.0 else qn
            q = r["qout"]
    qn = q
    for st in grhd.SSPRK3:
        ref, out = run_pair(orc, grid, eos, {}, opts, dict(st, dt=dt), qn, q)
        check_pair(grid, ref, out)
        q = ref["qout"]


def test_paper_shock_tube_substeps(orc):
    """The paper's problem at N = 800.  Its right state has P = 0 exactly:
    in the cells the shock is entering, whether the recovered specific
    energy is a rounding-level positive number or is clamped to the cold
    value (P = 0) is decided by rounding, and the sound speed
    c_s = sqrt(Gamma P / (rho h)) turns a pressure of order 1e-16 into a
    wave speed of order 1e-8; the local fluxes then differ at the 1e-6
    relative level, i.e. ~1e-11 against the largest state.  The bar for this
    degenerate state is 1e-9 normwise and the cold-recovery flag may differ;
    every other flag and every non-degenerate case keep 1e-12."""
    gam = 5.0 / 3.0
    L, R = synth.PAPER_SHOCK_TUBE
    grid = synth.riemann_grid(800, nz=1)
    eos = synth.ideal_eos(gam)
    q = orc.prim2con(grid, eos, {}, synth.riemann_prims(grid, L, R), with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_RIE)
    dt = 0.4 * grid["dx"]
    for i in range(6):
        st = grhd.SSPRK3[i % 3]
        ref, out = run_pair(orc, grid, eos, {}, opts, dict(st, dt=dt), q, q)
        check_pair(grid, ref, out, tol=1e-9, flag_mask=0xFF & ~2)
        q = ref["qout"]


@pytest.mark.parametrize("recon,face_eps", [("ppm", "recon"), ("ppm", "eos"), ("ppm3", "recon")])
@pytest.mark.parametrize("n", [64, 93])
@pytest.mark.parametrize("stage", [0, 1, 2])
def test_substep_star(orc, tov, n, stage, recon, face_eps):
    grid, p, metric, eos = star_case(n, 10 + n + stage, tov, vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    qn = orc.prim2con(grid, eos, metric, star_case(n, 99, tov, vel=0.05)[1], with_ghosts=True)
    opts = dict(recon=recon, riemann="hllc", prec="fp64", c2p=C2P_STAR, face_eps=face_eps)
    st = dict(grhd.SSPRK3[stage], dt=0.4 * grid["dx"])
    ref, out = run_pair(orc, grid, eos, metric, opts, st, qn, q)
    check_pair(grid, ref, out)


@pytest.mark.parametrize("face_eps", ["recon", "eos"])
@pytest.mark.parametrize("riemann,eos_kind", [("hllc", "ideal"), ("tvdlf", "ideal"), ("hllc", "hybrid")])
def test_substep_general_metric(orc, riemann, eos_kind, face_eps):
    grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
    metric = synth.general_metric(grid, 7)
    p = synth.smooth_state(grid, 8, vamp=0.5)
    eos = synth.ideal_eos(5.0 / 3.0)
    if eos_kind == "hybrid":
        eos = HYBRID
        p = hybrid_state(orc, p)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann=riemann, prec="fp64", c2p=C2P_RIE, face_eps=face_eps)
    ref, out = run_pair(orc, grid, eos, metric, opts, dict(grhd.SSPRK3[1], dt=0.005), q, q)
    check_pair(grid, ref, out)


def test_substep_general_metric_cylindrical(orc, tov):
    """Cylindrical grid with every metric field active (shift, conformal
    metric, curvature) on top of the star: exercises the tetrad legs, the
    moving face and the full source terms with the hoop-stress term."""
    grid, p, metric, eos = star_case(48, 21, tov, vel=0.05)
    gm = synth.general_metric(grid, 22, amp=0.02)
    gm["alp"] = metric["alp"] * (1.0 + 0.0 * gm["alp"])
    gm["W"] = metric["W"]
    q = orc.prim2con(grid, eos, gm, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR)
    ref, out = run_pair(orc, grid, eos, gm, opts, dict(grhd.SSPRK3[0], dt=0.4 * grid["dx"]), q, q)
    check_pair(grid, ref, out)


def test_substep_rk4_accumulator(orc, tov):
    grid, p, metric, eos = star_case(40, 31, tov, vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    acc = orc.prim2con(grid, eos, metric, star_case(40, 32, tov, vel=0.05)[1], with_ghosts=True) * 1e-3
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR)
    st = dict(a=1.0, b=0.0, c=0.5, dt=0.4 * grid["dx"], g=0.0, d=1.0, e=1.0 / 3.0)
    ref, out = run_pair(orc, grid, eos, metric, opts, st, q, q, acc_in=acc, want_acc=True)
    check_pair(grid, ref, out)
    st = dict(a=1.0, b=0.0, c=1.0 / 6.0, dt=0.4 * grid["dx"], g=1.0, d=0.0, e=0.0)
    ref, out = run_pair(orc, grid, eos, metric, opts, st, q, q, acc_in=acc, want_acc=True)
    check_pair(grid, ref, out)


def test_tile_shapes_bitwise(orc, tov):
    """The per-cell arithmetic does not depend on the tiling: every built
    tile shape gives identical bits, including ragged tails."""
    grid, p, metric, eos = star_case(77, 41, tov, vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR)
    st = dict(grhd.SSPRK3[1], dt=0.4 * grid["dx"])
    outs = []
    for tile in [(16, 15), (32, 8), (32, 16), (64, 8), (16, 16), (16, 8), (16, 7)]:
        ref, out = run_pair(orc, grid, eos, metric, opts, st, q, q, tile=tile)
        outs.append(out)
    check_pair(grid, ref, outs[0])
    for o in outs[1:]:
        assert np.array_equal(synth.interior(grid, o["qout"]), synth.interior(grid, outs[0]["qout"]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_general_metric_tile_shapes_bitwise(orc, prec):
    """The general class reads its geometry fields from LDS on 16 x 7 and
    16 x 8 tiles and from memory on larger ones: the same bits either way
    (cylindrical star with every metric field active, ragged tails)."""
    tov = synth.tov_solve()
    grid, p, metric, eos = star_case(77, 43, tov, vel=0.05)
    gm = synth.general_metric(grid, 44, amp=0.02)
    gm["alp"] = metric["alp"] * (1.0 + 0.0 * gm["alp"])
    gm["W"] = metric["W"]
    q = orc.prim2con(grid, eos, gm, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec=prec, c2p=C2P_STAR)
    st = dict(grhd.SSPRK3[1], dt=0.4 * grid["dx"])
    outs = []
    for tile in [(16, 7), (16, 8), (16, 15), (32, 8)]:
        ref, out = run_pair(orc, grid, eos, gm, opts, st, q, q, tile=tile)
        outs.append(out)
    if prec == "fp64":
        check_pair(grid, ref, outs[0])
    for o in outs[1:]:
        assert np.array_equal(synth.interior(grid, o["qout"]), synth.interior(grid, outs[0]["qout"]))


@pytest.mark.parametrize("n,face_eps", [(512, "recon"), (1024, "recon"), (512, "eos")])
def test_substep_full_size_star(orc, tov, n, face_eps):
    """Full star sizes in the benchmark's launch configuration, all cells."""
    grid, p, metric, eos = star_case(n, 50, tov, vel=0.02)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR, face_eps=face_eps)
    ref, out = run_pair(orc, grid, eos, metric, opts, dict(grhd.SSPRK3[2], dt=0.4 * grid["dx"]), q, q)
    check_pair(grid, ref, out)


def test_invalid_cells_never_nan(orc):
    grid = synth.riemann_grid(64, nz=4)
    eos = synth.ideal_eos(5.0 / 3.0)
    (L, R), = synth.riemann_states(3, 1)
    q = orc.prim2con(grid, eos, {}, synth.riemann_prims(grid, L, R), with_ghosts=True)
    qi = synth.interior(grid, q)
    qi[0, 0, 5] = -1.0
    qi[4, 1, 9] = np.nan
    qi[2, 2, 11] = np.inf
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_RIE)
    ref, out = run_pair(orc, grid, eos, {}, opts, dict(grhd.SSPRK3[0], dt=0.001), q, q)
    assert np.all(np.isfinite(synth.interior(grid, out["qout"])))
    check_pair(grid, ref, out)


def test_mixed_single_substep_close(orc, tov):
    """Mixed precision (FP32 reconstruction and flux) after one substep:
    within FP32 rounding of the flux term of the oracle."""
    grid, p, metric, eos = star_case(64, 61, tov, vel=0.02)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_STAR)
    st = dict(grhd.SSPRK3[0], dt=0.4 * grid["dx"])
    ref, _ = run_pair(orc, grid, eos, metric, opts, st, q, q)
    _, out = run_pair(orc, grid, eos, metric, dict(opts, prec="mixed"), st, q, q)
    I = lambda a: synth.interior(grid, a)  # noqa: E731
    dq_o = I(ref["qout"]) - I(q)
    dq_g = I(out["qout"]) - I(q)
    for c in (0, 1, 3, 4):
        assert np.abs(dq_g[c] - dq_o[c]).max() <= 1e-5 * np.abs(dq_o[c]).max() + 1e-16 * np.abs(I(q)[c]).max()


# ------------------------------------------------------------ zero temperature

THREE_PIECE = dict(kind="hybrid", K=[8.95e-2, 8.95e-2 * 1.5e-4 ** (1.35692 - 3.005),
                                     8.95e-2 * 1.5e-4 ** (1.35692 - 3.005) * 8.1e-4 ** (3.005 - 2.988)],
                   G=[1.35692, 3.005, 2.988], rho_b=[1.5e-4, 8.1e-4], Gth=1.75)


def test_con2prim_adiabatic_three_piece(orc):
    """The adiabatic recovery (cold root from D, S; E reset) on a general
    metric with a three-piece polytrope, hot and cold cells mixed."""
    grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
    metric = synth.general_metric(grid, 13)
    rng = np.random.default_rng(14)
    p = synth.smooth_state(grid, 15, vamp=0.3)
    p[0] = 10.0 ** rng.uniform(-5, -2.5, size=p[0].shape)
    ec = np.array([orc.eos_eps_cold(THREE_PIECE, r) for r in p[0].ravel()]).reshape(p[0].shape)
    p[5] = ec + np.where(rng.uniform(size=ec.shape) < 0.5, 0.0, 0.02)
    p[4] = np.array([orc.eos_press(THREE_PIECE, r, e) for r, e in zip(p[0].ravel(), p[5].ravel())]).reshape(ec.shape)
    q = orc.prim2con(grid, THREE_PIECE, metric, p, with_ghosts=True)
    c2p = dict(w_max=100.0, rho_atm=1e-12, adiabatic=True)
    p_o, q_o, fl_o, d_o = orc.con2prim(grid, THREE_PIECE, metric, c2p, q)
    qg = dev(q)
    pg = torch.zeros((6,) + q.shape[1:], dtype=torch.float64, device=DEV)
    fl = torch.zeros(q.shape[1:], dtype=torch.uint8, device=DEV)
    grhd.con2prim(grid, THREE_PIECE, mdev(metric), c2p, qg, pg, flags=fl)
    torch.cuda.synchronize()
    I = lambda a: synth.interior(grid, a)  # noqa: E731
    assert np.array_equal(I(fl.cpu().numpy()), I(fl_o))
    assert normwise(I(pg.cpu().numpy()), I(p_o)) <= TOL
    assert normwise(I(qg.cpu().numpy()), I(q_o)) <= TOL


def test_substep_star_adiabatic(orc, tov):
    """The star with the zero-temperature law P = K rho^Gamma (one-piece
    hybrid EOS, energy equation discarded), every stage."""
    grid, p, metric, _ = star_case(64, 71, tov, vel=0.05)
    eos = dict(kind="hybrid", K=[tov["K"]], G=[tov["G"]], rho_b=[], Gth=2.0)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=dict(C2P_STAR, adiabatic=True))
    qn = q
    for s in range(3):
        st = dict(grhd.SSPRK3[s], dt=0.4 * grid["dx"])
        ref, out = run_pair(orc, grid, eos, metric, opts, st, qn, q)
        check_pair(grid, ref, out)
        if s == 0:
            qn = ref["qs"]
        q = ref["qout"]


@pytest.mark.parametrize("nx,nz,bc", [(1, 1, "periodic"), (2, 1, "periodic"), (1, 2, "periodic"),
                                      (2, 2, "periodic"), (1, 21, "periodic"), (19, 1, "periodic"),
                                      (2, 37, "periodic"), (1, 1, "outflow"), (2, 3, "outflow"),
                                      (3, 1, "outflow")])
@pytest.mark.parametrize("recon,riemann", [("ppm", "hllc"), ("minmod", "tvdlf")])
def test_substep_tiny_grids(orc, nx, nz, bc, recon, riemann):
    """Degenerate grids: directions of 1 to 3 cells (periodic ones shorter
    than the 3-cell halo wrap onto themselves), one partial tile."""
    eos = synth.ideal_eos(5.0 / 3.0)
    grid = synth.make_grid(nx, nz, 0.0, 0.0, 0.1, 0.1, "cart", (bc,) * 4)
    rng = np.random.default_rng(100 * nx + nz)
    p = synth.empty_fields(grid, 6)
    b = rng.uniform(size=p.shape)              # ghosts too: the BCs overwrite them
    p[0] = 1.0 + 0.3 * b[0]
    p[1], p[2], p[3] = 0.3 * (b[1] - 0.5), 0.2 * (b[2] - 0.5), 0.3 * (b[3] - 0.5)
    p[4] = 0.5 + 0.3 * b[4]
    p[5] = p[4] / ((5.0 / 3.0 - 1.0) * p[0])
    q = orc.prim2con(grid, eos, {}, p, with_ghosts=True)
    opts = dict(recon=recon, riemann=riemann, c2p=C2P_RIE)
    ref, out = run_pair(orc, grid, eos, {}, opts, dict(grhd.SSPRK3[0], dt=0.01), q, q)
    check_pair(grid, ref, out)


def test_substep_at_the_size_limit(orc):
    """A field of exactly 2^29 cells (the 32-bit offset limit): 16378 x
    32762 interior cells, row pitch 16384, periodic, the state repeating
    with period 2 in z.  Every pair of rows must equal, bit for bit, the
    result on a 2-row periodic grid, which is itself checked against the
    oracle; a read or write at a wrong offset anywhere in the 4 GiB fields
    breaks the equality.  About 65 GiB of device arrays."""
    free, _ = torch.cuda.mem_get_info(DEV)
    if free < 80 * (1 << 30):
        pytest.skip("needs about 65 GiB of free device memory (%.1f GiB free)" % (free / (1 << 30)))
    eos = synth.ideal_eos(5.0 / 3.0)
    nx, nz = 16378, 32762
    gs = synth.make_grid(nx, 2, 0.0, 0.0, 0.1, 0.1, "cart", ("periodic",) * 4)
    gb = synth.make_grid(nx, nz, 0.0, 0.0, 0.1, 0.1, "cart", ("periodic",) * 4)
    pitch, ng = gb["pitch"], gb["ng"]
    assert pitch == gs["pitch"] == 16384 and (nz + 2 * ng) * pitch == 1 << 29
    rng = np.random.default_rng(29)
    p = synth.empty_fields(gs, 6)
    b = rng.uniform(size=p.shape)
    p[0] = 1.0 + 0.3 * b[0]
    p[1], p[2], p[3] = 0.3 * (b[1] - 0.5), 0.2 * (b[2] - 0.5), 0.3 * (b[3] - 0.5)
    p[4] = 0.5 + 0.3 * b[4]
    p[5] = p[4] / ((5.0 / 3.0 - 1.0) * p[0])
    q = orc.prim2con(gs, eos, {}, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P_RIE, tile=(16, 16))
    st = dict(grhd.SSPRK3[0], dt=0.01)
    ref, small = run_pair(orc, gs, eos, {}, opts, st, q, q, tile=(16, 16))
    check_pair(gs, ref, small)

    rows = nz + 2 * ng
    qb = torch.zeros((5, rows, pitch), dtype=torch.float64, device=DEV)
    qs_small = dev(q)[:, ng:ng + 2, :]
    qb[:, ng:ng + nz].view(5, nz // 2, 2, pitch).copy_(qs_small[:, None].expand(5, nz // 2, 2, pitch))
    qo = torch.zeros_like(qb)
    pb = torch.zeros((6, rows, pitch), dtype=torch.float64, device=DEV)
    fb = torch.zeros((rows, pitch), dtype=torch.uint8, device=DEV)
    dg = grhd.new_diag()
    sub = grhd.Substep(gb, eos, {}, opts)
    sub(st, qb, qb, qo, pb, flags=fb, diag=dg)
    torch.cuda.synchronize()

    def rows_equal(big, small_np, nf):
        s = torch.from_numpy(np.ascontiguousarray(small_np[..., ng:ng + 2, ng:ng + nx])).to(DEV)
        bv = big[..., ng:ng + nz, :].view(*big.shape[:-2], nz // 2, 2, pitch)[..., ng:ng + nx]
        if big.dtype == torch.float64:
            bv, s = bv.view(torch.int64), s.view(torch.int64)
        return bool((bv == s.unsqueeze(-3)).all())

    try:
        assert rows_equal(qo, small["qout"], 5)
        assert rows_equal(qb, small["qs"], 5)
        assert rows_equal(pb, small["p"], 6)
        assert rows_equal(fb, small["flags"], 1)
        d, r = grhd.read_diag(dg), small["diag"]
        assert d["max_courant"] == r["max_courant"]
        assert d["Mb"] == pytest.approx(r["Mb"] * (nz // 2), rel=1e-12)
        for k in ("n_rescale", "n_cold", "n_atm", "n_fail"):
            assert d[k] == r[k] * (nz // 2), k
    finally:
        del qb, qo, pb, fb
        torch.cuda.empty_cache()
