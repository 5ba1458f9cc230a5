"""GPU: Bondi accretion in the maximal trumpet slice (Sec. III.B.2), the
general-metric path (shift, lapse, extrinsic curvature, cylindrical).

- parity: every stage of an SSP-RK3 step against the oracle (1e-12
  normwise per field), with the inner region r < 0.4M held at the initial
  state by grhd_fix_cells on the GPU and by the same assignment in the
  oracle's loop;
- the flow stays stationary: the L1 density error of the paper's measure
  at t = 20M falls by at least 3x per doubling of the resolution (N = 64,
  128, 256 on [0, 16M]^2), the paper's second-order claim, with the
  per-cell third-order parabola (PPM3) under HLLC and under TVDLF, and with
  minmod.  CW84's PPM, whose two face states coincide wherever no limiter
  acts, leaves the grid-scale error seeded near the held region undamped
  and converges at about first order there (2.5x, 2.2x, 2.0x per doubling
  from N = 32 on the oracle); it is not pinned.
- the inner-region hold inside the stage (grhd_options.fix_mask) equals
  the separate grhd_fix_cells pass bit for bit.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_03223_amd import grhd  # noqa: E402

DEV = torch.device("cuda:0")
C2P = dict(w_max=100.0, rho_atm=1e-14)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def normwise(g, o):
    worst = 0.0
    for c in range(g.shape[0]):
        scale = np.abs(o[c]).max()
        d = np.abs(g[c] - o[c]).max()
        worst = max(worst, d if scale == 0.0 else d / scale)
    return worst


def bondi_case(n):
    d = 16.0 / n
    g = synth.make_grid(n, n, 0.0, 0.0, d, d, "cyl", ("axis", "external", "reflect", "external"))
    p, m, eos, frozen = synth.bondi_problem(g)
    return g, p, m, eos, frozen


@pytest.mark.parametrize("riemann,recon", [("hllc", "ppm"), ("tvdlf", "ppm"), ("hllc", "ppm3"),
                                           ("tvdlf", "ppm3")])
def test_bondi_step_parity(orc, riemann, recon):
    g, p, m, eos, frozen = bondi_case(64)
    opts = dict(recon=recon, riemann=riemann, prec="fp64", c2p=C2P)
    q0 = orc.prim2con(g, eos, m, p, with_ghosts=True)
    md = {k: dev(v) for k, v in m.items()}
    sub = grhd.Substep(g, eos, md, opts)
    mask = dev(frozen.astype(np.uint8))
    qfix = dev(q0)
    # the EXTERNAL ghosts of every stage buffer carry the exact flow (a
    # stage writes interior cells only)
    qg = [dev(q0), dev(q0), dev(q0)]
    pg = torch.zeros((6,) + q0.shape[1:], dtype=torch.float64, device=DEV)
    dt = 0.4 * g["dx"]
    qn_o, qs_o = q0, q0
    roles = [(0, 0, 1), (0, 1, 2), (0, 2, 1)]
    for s, st in enumerate(grhd.SSPRK3):
        stage = dict(st, dt=dt)
        a, b, c = roles[s]
        sub(stage, qg[a], qg[b], qg[c], pg)
        grhd.fix_cells(g, mask, qfix, qg[c])
        ref = orc.rk_substep(g, eos, m, opts, stage, qn_o, qs_o)
        out_o = ref["qout"].copy()
        out_o[:, frozen] = q0[:, frozen]
        if s == 0:
            qn_o = ref["qs"]
        torch.cuda.synchronize()
        I = lambda a_: synth.interior(g, a_)  # noqa: E731
        e = normwise(I(qg[c].cpu().numpy()), I(out_o))
        assert e <= 1e-12, (s, e)
        # the oracle's next stage reads the ghosts of its q_s: exact flow
        qs_o = out_o
        ng = g["ng"]
        ghost = np.ones(q0.shape[1:], dtype=bool)
        ghost[ng:ng + g["nz"], ng:ng + g["nx"]] = False
        qs_o[:, ghost] = q0[:, ghost]


def evolve_l1(n, t_end, riemann="hllc", recon="ppm"):
    g, p, m, eos, frozen = bondi_case(n)
    md = {k: dev(v) for k, v in m.items()}
    opts = dict(recon=recon, riemann=riemann, prec="fp64", c2p=C2P)
    sub = grhd.Substep(g, eos, md, opts)
    pd = dev(p)
    q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=DEV)
    grhd.prim2con(g, eos, md, pd, q, with_ghosts=True)
    qfix = q.clone()
    q1, q2 = q.clone(), q.clone()   # ghosts of every buffer: the exact flow
    mask = dev(frozen.astype(np.uint8))
    pw = torch.zeros_like(pd)
    dt = 0.4 * g["dx"]
    nsteps = int(round(t_end / dt))
    calls = [sub.bind(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, pw)
             for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)])]
    for _ in range(nsteps):
        for c, qo in zip(calls, (q1, q2, q)):
            c()
            grhd.fix_cells(g, mask, qfix, qo)
    grhd.con2prim(g, eos, md, C2P, q.clone(), pw)
    torch.cuda.synchronize()
    rho = synth.interior(g, pw.cpu().numpy()[0])
    rho0 = synth.interior(g, p[0])
    X, _ = synth.cell_coords(g)
    x = synth.interior(g, X)
    sg = synth.interior(g, m["alp"] * m["W"] ** -3) * x      # sqrt(-g) dV / (2 pi dx dz)
    return float((np.abs(rho - rho0) * sg).sum() / (np.abs(rho0) * sg).sum()), nsteps


@pytest.mark.parametrize("riemann", ["hllc", "tvdlf"])
def test_bondi_stationary_ppm3_second_order(riemann):
    """The paper's statement (Sec. III.B.2): the L1 density error of the
    stationary flow converges at second order with both Riemann solvers.
    Bar: at least 3x per doubling at t = 20M, N = 64, 128, 256."""
    errs = [evolve_l1(n, 20.0, riemann=riemann, recon="ppm3")[0] for n in (64, 128, 256)]
    assert errs[0] / errs[1] >= 3.0 and errs[1] / errs[2] >= 3.0, errs


def test_bondi_stationary_minmod_second_order():
    errs = [evolve_l1(n, 20.0, recon="minmod")[0] for n in (64, 128, 256)]
    assert errs[0] / errs[1] >= 3.0 and errs[1] / errs[2] >= 3.0, errs


def run_state(g, p, m, eos, frozen, opts, t_end):
    md = {k: dev(v) for k, v in m.items()}
    sub = grhd.Substep(g, eos, md, opts)
    pd = dev(p)
    q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=DEV)
    grhd.prim2con(g, eos, md, pd, q, with_ghosts=True)
    qfix, q1, q2 = q.clone(), q.clone(), q.clone()
    mask = dev(frozen.astype(np.uint8))
    pw = torch.zeros_like(pd)
    dt = 0.4 * g["dx"]
    calls = [sub.bind(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, pw)
             for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)])]
    for _ in range(int(round(t_end / dt))):
        for c, qo in zip(calls, (q1, q2, q)):
            c()
            grhd.fix_cells(g, mask, qfix, qo)
    grhd.con2prim(g, eos, md, opts["c2p"], q.clone(), pw)
    torch.cuda.synchronize()
    return pw.cpu().numpy()


def total_variation(g, rho):
    x = g["x0"] + (np.arange(g["nx"]) + 0.5) * g["dx"]
    xf = g["x0"] + np.arange(1, g["nx"]) * g["dx"]
    return float((np.abs(np.diff(rho, axis=1)) * xf).sum() * g["dz"] +
                 (np.abs(np.diff(rho, axis=0)) * x).sum() * g["dx"])


def test_hot_bubble_hllc_sharper_than_tvdlf():
    """Sec. III.B.3: the hot bubble in the Bondi flow keeps more structure
    (a larger total variation of the density) with HLLC than with TVDLF."""
    n = 256
    d = 16.0 / n
    g = synth.make_grid(n, n, 0.0, 0.0, d, d, "cyl", ("axis", "external", "reflect", "external"))
    p, m, eos, frozen = synth.modified_bondi_problem(g)
    tv = {}
    for riemann in ("hllc", "tvdlf"):
        pf = run_state(g, p, m, eos, frozen, dict(recon="ppm", riemann=riemann, prec="fp64", c2p=C2P), 5.0)
        rho = synth.interior(g, pf[0])
        assert np.all(np.isfinite(rho)) and rho.min() > 0.0
        tv[riemann] = total_variation(g, rho)
    assert tv["hllc"] > 1.02 * tv["tvdlf"], tv


def test_fixed_cells_in_the_stage_equal_a_separate_pass():
    """grhd_options.fix_mask/fix_q: the stage stores the fixed state on the
    masked cells; two SSP-RK3 steps equal the stage followed by
    grhd_fix_cells bit for bit, and the diagnostics then sum the stored
    state."""
    g, p, m, eos, frozen = bondi_case(64)
    md = {k: dev(v) for k, v in m.items()}
    pd = dev(p)
    q0 = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=DEV)
    grhd.prim2con(g, eos, md, pd, q0, with_ghosts=True)
    mask = dev(frozen.astype(np.uint8))
    qfix = q0.clone()
    dt = 0.4 * g["dx"]
    outs = []
    for fused in (False, True):
        opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=C2P)
        if fused:
            opts["fix"] = (mask, qfix)
        sub = grhd.Substep(g, eos, md, opts)
        q = q0.clone()
        q1, q2 = q.clone(), q.clone()
        pw = torch.zeros_like(pd)
        diag = grhd.new_diag()
        for _ in range(2):
            for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)]):
                sub(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, pw, diag=diag)
                if not fused:
                    grhd.fix_cells(g, mask, qfix, qo)
        torch.cuda.synchronize()
        outs.append((q.clone(), grhd.read_diag(diag)))
    assert torch.equal(outs[0][0].view(torch.int64), outs[1][0].view(torch.int64))
    qi = synth.interior(g, outs[1][0].cpu().numpy())
    X, _ = synth.cell_coords(g)
    x = synth.interior(g, X)
    mb = float((qi[0] * 2.0 * np.pi * x * g["dx"] * g["dz"]).sum())
    assert outs[1][1]["Mb"] == pytest.approx(mb, rel=1e-12)
