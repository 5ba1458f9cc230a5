"""GPU: the learned recovery guess.

- the matrix-core forward pass equals the oracle's FP64 forward pass with
  the same BF16-rounded weights, to BF16 activation rounding;
- the training gradient (FP32, BF16-rounded weights) equals the oracle's
  FP64 back-propagation with the same weights (per tensor, normwise 1e-4);
- training on (D, S, tau) -> P pairs that the oracle generates lowers the
  loss, and the recovery seeded by the trained network reaches the same
  root as the paper's Illinois recovery and as the oracle's bisection
  (1e-12 normwise on the primitives) with fewer master-function
  evaluations on the differentially rotating workload;
- the batched plan with the learned guess (star levels, a rotating-field
  patch and Riemann patches in one graph) lands every patch on the same
  state as the plan without it (1e-12 normwise, per cell on the positive
  fields) and as the oracle's stage.
"""
import numpy as np
import pytest

import synth
from cmp import normwise, percell, percell_cond

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_03223_amd import grhd  # noqa: E402

DEV = torch.device("cuda:0")


def bf16_round(a):
    t = torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32)
    return t.numpy().astype(np.float64)


def rounded_params(P):
    """FP64 copy of an FP32 parameter vector with W1 and W2 rounded to BF16
    (the matrices the GPU uses)."""
    Q = P.astype(np.float64).copy()
    Q[0:192] = bf16_round(P[0:192])
    Q[256:4352] = bf16_round(P[256:4352])
    return Q


def test_forward_matches_oracle(orc):
    P = grhd.mlp_init(3)
    scal = torch.tensor([0, 0, 0, 1, 1, 1, 0, 1], dtype=torch.float32, device=DEV)
    net = grhd.MLP(P, scal)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(1000, 3)).astype(np.float32)
    y = net.forward(torch.from_numpy(X).to(DEV)).cpu().numpy()
    ref = orc.mlp_forward(rounded_params(P.cpu().numpy()), bf16_round(X))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= 2e-2, err
    assert np.corrcoef(y, ref)[0, 1] > 0.9999


def test_gradient_matches_oracle(orc):
    P = grhd.mlp_init(4)
    rng = np.random.default_rng(1)
    n = 777  # several chunks and a ragged tail
    X = rng.normal(size=(n, 3)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    g, loss = grhd.mlp_grad(P, torch.from_numpy(X).to(DEV), torch.from_numpy(t).to(DEV))
    g = g.cpu().numpy()
    lo, go = orc.mlp_loss_grad(rounded_params(P.cpu().numpy()), X.astype(np.float64), t.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=1e-4)
    for a, b in [(0, 192), (192, 256), (256, 4352), (4352, 4416), (4416, 4480), (4480, 4481)]:
        err = np.abs(g[a:b] - go[a:b]).max() / np.abs(go[a:b]).max()
        assert err <= 1e-4, (a, b, err)


def test_features_match_definition():
    """grhd_mlp_features against the features written out in numpy:
    (log10 D, |S|/E, log10((E - D)/D)) and the target log10(P/D), on
    conserved values spanning the recovery samples' range."""
    rng = np.random.default_rng(5)
    n = 5000
    D = 10.0 ** rng.uniform(-10, -2, n)
    S = rng.normal(size=(3, n)) * D * rng.uniform(0, 3, n)
    E = D * (1.0 + 10.0 ** rng.uniform(-8, 1, n)) + np.sqrt((S ** 2).sum(0))
    P = D * 10.0 ** rng.uniform(-9, 0, n)
    q = torch.from_numpy(np.stack([D, S[0], S[1], S[2], E])).to(DEV)
    X, y = grhd.recovery_features(q, torch.from_numpy(P).to(DEV))
    X, y = X.cpu().numpy(), y.cpu().numpy()
    ref = np.stack([np.log10(D), np.sqrt((S ** 2).sum(0)) / E, np.log10((E - D) / D)], axis=1)
    # per element, relative to max(1, |value|): the logarithms cross zero
    for c in range(3):
        assert np.max(np.abs(X[:, c] - ref[:, c]) / np.maximum(np.abs(ref[:, c]), 1.0)) <= 1e-14, c
    t = np.log10(P / D)
    assert np.max(np.abs(y - t) / np.maximum(np.abs(t), 1.0)) <= 1e-14
    X0 = grhd.recovery_features(q)
    assert torch.equal(X0.cpu(), torch.from_numpy(X))


def training_pairs(orc, seed, n, sampler=None):
    """(D, S, tau) -> P pairs from the oracle's prim->con on seeded states."""
    prims = (sampler or synth.recovery_samples)(seed, n)
    grid = synth.make_grid(n, 1, 0.0, 0.0, 1.0, 1.0, "cart", ("outflow",) * 4)
    p = synth.empty_fields(grid, 6)
    synth.interior(grid, p)[:, 0, :] = prims.T
    q = orc.prim2con(grid, synth.ideal_eos(2.0, 100.0), {}, p)
    qi = synth.interior(grid, q)[:, 0, :]
    D, E = qi[0], qi[4]
    S = np.sqrt(qi[1] ** 2 + qi[2] ** 2 + qi[3] ** 2)
    X = np.stack([np.log10(D), S / E, np.log10((E - D) / D)], axis=1)
    y = np.log10(prims[:, 4] / D)
    return X, y


def train(orc, n=200_000, epochs=8, batch=8192, seed=11, sampler=None):
    X, y = training_pairs(orc, seed, n, sampler)
    xm, xs = X.mean(axis=0), X.std(axis=0)
    ym, ys = y.mean(), y.std()
    scal = torch.tensor(list(xm) + list(xs) + [ym, ys], dtype=torch.float32, device=DEV)
    Xs = torch.from_numpy(((X - xm) / xs).astype(np.float32)).to(DEV)
    ts = torch.from_numpy(((y - ym) / ys).astype(np.float32)).to(DEV)
    net = grhd.MLP(grhd.mlp_init(seed), scal)
    _, l0 = grhd.mlp_grad(net.params, Xs, ts)
    losses = [float(l0.cpu()[0])]
    g = torch.Generator(device=DEV).manual_seed(seed)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=DEV)
        lr = 3e-3 * (0.5 ** (ep // 3))
        for b in range(0, n, batch):
            idx = perm[b:b + batch]
            net.train_step(Xs[idx].contiguous(), ts[idx].contiguous(), lr)
        losses.append(float(net.loss.cpu()[0]))
    return net, losses


def test_training_and_gain(orc):
    net, losses = train(orc)
    # losses[0] is the untrained network's loss on the whole set
    assert losses[-1] < 0.02 * losses[0] and losses[-1] < 1e-2, losses
    # recovery on the rotating workload (flat metric), three ways
    grid = synth.make_grid(256, 64, 0.0, 0.0, 20.0 / 256, 20.0 / 256, "cart",
                           ("outflow", "outflow", "outflow", "outflow"))
    p = synth.rotating_field(grid, 7)
    eos = synth.ideal_eos(2.0, 100.0)
    q = orc.prim2con(grid, eos, {}, p)
    c2p = dict(w_max=100.0, rho_atm=1e-12)
    p_o, _, fl_o, _ = orc.con2prim(grid, eos, {}, c2p, q)
    res = {}
    for name, mlp in (("illinois", None), ("mlp", net.buf)):
        qg = torch.from_numpy(q).to(DEV)
        pg = torch.zeros((6,) + q.shape[1:], dtype=torch.float64, device=DEV)
        fl = torch.zeros(q.shape[1:], dtype=torch.uint8, device=DEV)
        dg = grhd.new_diag()
        grhd.con2prim(grid, eos, {}, dict(c2p, mlp=mlp), qg, pg, flags=fl, diag=dg)
        torch.cuda.synchronize()
        res[name] = (synth.interior(grid, pg.cpu().numpy()), grhd.read_diag(dg),
                     synth.interior(grid, fl.cpu().numpy()))
    ref = synth.interior(grid, p_o)
    for name, (pp, d, fl) in res.items():
        assert np.array_equal(fl, synth.interior(grid, fl_o)), name
        for c in range(6):
            scale = np.abs(ref[c]).max()
            assert np.abs(pp[c] - ref[c]).max() <= 1e-12 * scale, (name, c)
        # per cell on the positive fields: rho spans eight decades here
        e = percell(pp, ref, (0,))
        assert e <= 1e-12, (name, e)
        e = percell_cond(pp, ref, synth.interior(grid, q))
        assert e <= 1e-12, (name, e)
    it_ill = res["illinois"][1]["iter_sum"]
    it_mlp = res["mlp"][1]["iter_sum"]
    assert it_mlp < it_ill, (it_mlp, it_ill)


def test_batch_with_learned_guess(orc):
    """The batched recovery seeded by the network (star levels, a
    rotating-field patch, Riemann patches, FP64) against the same plan with
    the paper's Illinois recovery and against the oracle's stage."""
    def both(seed, n):
        a = synth.recovery_samples(seed, n // 2)
        b = synth.star_recovery_samples(seed + 1, n - n // 2)
        return np.concatenate([a, b])
    net, _ = train(orc, n=100_000, epochs=4, sampler=both)
    tov = synth.tov_solve()
    patches = []
    for lvl, grid in enumerate(synth.fmr_levels(2, 48, finest_extent=20.0)):
        p, metric, eos = synth.star_problem(grid, seed=40 + lvl, tov=tov, vel=0.05)
        patches.append(dict(grid=grid, metric=metric, p=p, eos_id=0))
    rg = synth.make_grid(96, 24, 0.0, 0.0, 20.0 / 96, 20.0 / 96, "cart", ("outflow",) * 4)
    patches.append(dict(grid=rg, metric={}, p=synth.rotating_field(rg, 8), eos_id=0))
    gam = 5.0 / 3.0
    for nxr, (L, R) in zip((77, 130), synth.riemann_states(9, 2, gam)):
        g = synth.riemann_grid(nxr, nz=8)
        patches.append(dict(grid=g, metric={}, p=synth.riemann_prims(g, L, R, gam), eos_id=1))
    eos_table = [synth.ideal_eos(2.0, 100.0), synth.ideal_eos(gam)]
    c2p = dict(w_max=100.0, rho_atm=1e-10)
    out = {}
    for name, mlp in (("illinois", None), ("mlp", net.buf)):
        opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=dict(c2p, mlp=mlp))
        bufs, descs = [], []
        for pt in patches:
            q0 = orc.prim2con(pt["grid"], eos_table[pt["eos_id"]], pt["metric"], pt["p"], with_ghosts=True)
            q = torch.from_numpy(q0).to(DEV)
            b = dict(q0=q0, q=q, q1=torch.zeros_like(q),
                     p=torch.zeros((6,) + q.shape[1:], dtype=torch.float64, device=DEV))
            bufs.append(b)
            descs.append(dict(grid=pt["grid"], metric={k: torch.from_numpy(v).to(DEV) for k, v in pt["metric"].items()},
                              qn=b["q"], qs=b["q"], qout=b["q1"], p=b["p"],
                              stage=dict(grhd.SSPRK3[0], dt=0.4 * pt["grid"]["dx"]), eos_id=pt["eos_id"]))
        plan = grhd.Plan(descs, eos_table, opts)
        for b in bufs:   # plan creation may have timed the batch on the buffers
            b["q"].copy_(torch.from_numpy(b["q0"]))
        dg = grhd.new_diag()
        plan(descs, diag=dg)
        torch.cuda.synchronize()
        out[name] = [dict(q1=b["q1"].cpu().numpy(), q=b["q"].cpu().numpy(), p=b["p"].cpu().numpy())
                     for b in bufs]
        out[name + "_diag"] = grhd.read_diag(dg)
        plan.close()
    for i, pt in enumerate(patches):
        g = pt["grid"]
        I = lambda a: synth.interior(g, a)  # noqa: E731
        ref = orc.rk_substep(g, eos_table[pt["eos_id"]], pt["metric"], dict(recon="ppm", riemann="hllc", c2p=c2p),
                             dict(grhd.SSPRK3[0], dt=0.4 * g["dx"]), bufs[i]["q0"], bufs[i]["q0"])
        for name in ("illinois", "mlp"):
            o = out[name][i]
            assert normwise(I(o["q1"]), I(ref["qout"])) <= 1e-12, (name, i)
            assert normwise(I(o["p"]), I(ref["p"])) <= 1e-12, (name, i)
            assert percell(I(o["p"]), I(ref["p"]), (0,)) <= 1e-12, (name, i)
            assert percell_cond(I(o["p"]), I(ref["p"]), I(ref["qs"])) <= 1e-12, (name, i)
        assert normwise(I(out["mlp"][i]["q1"]), I(out["illinois"][i]["q1"])) <= 1e-12, i
    assert out["mlp_diag"]["n_fail"] == out["illinois_diag"]["n_fail"] == 0


@pytest.mark.parametrize("case", ["rotating", "star", "general"])
def test_chained_with_learned_guess(orc, case):
    """grhd_rk_substep_chained seeded by the network: one SSP-RK3 step of
    chained stages with and without the guess.  After every stage the
    stored q_out and its flags equal the oracle's stage followed by its
    recovery, and its primitives the oracle's recovery of that same q_out
    (1e-12 normwise, per cell on rho, on P and eps by the recovery's
    conditioning); q_out equals the unseeded chained stage's (1e-12
    normwise; the primitives of the two runs come from slightly different
    q_out, so they are each compared with the recovery of their own); on
    a fast shear flow (every cell needs a real root search) the seeded
    recoveries take fewer master-function evaluations."""
    def both(seed, n):
        a = synth.recovery_samples(seed, n // 2)
        b = synth.star_recovery_samples(seed + 1, n - n // 2)
        return np.concatenate([a, b])
    net, _ = train(orc, n=100_000, epochs=4, sampler=both)
    if case == "rotating":
        # a smooth, fast shear flow (Lorentz factor 1 to 5 across the grid)
        # of the rotating workload's thermal state: every cell needs a root
        # search
        grid = synth.make_grid(256, 64, 0.0, 0.0, 20.0 / 256, 20.0 / 256, "cart", ("outflow",) * 4)
        X, Z = synth.cell_coords(grid)
        p = synth.empty_fields(grid, 6)
        p[0] = 1e-4 + 1e-3 * np.exp(-((X - 10.0) ** 2 + (Z - 2.5) ** 2) / 20.0)
        p[5] = 100.0 * p[0] * (1.0 + 0.5 * np.sin(X / 3.0))
        p[4] = (2.0 - 1.0) * p[0] * p[5]
        w = 1.0 + 4.0 * X / 20.0
        p[2] = np.sqrt(np.maximum(w * w - 1.0, 0.0))
        # every momentum component well above the pressure terms that
        # change it (R20's per-field scale)
        p[1] = 0.5 + 0.3 * np.sin(2.0 * np.pi * Z / 5.0)
        p[3] = 0.4 + 0.2 * np.cos(2.0 * np.pi * X / 20.0)
        metric, eos = {}, synth.ideal_eos(2.0, 100.0)
        c2p = dict(w_max=100.0, rho_atm=1e-12)
    elif case == "star":
        grid = synth.star_grid(64)
        p, metric, eos = synth.star_problem(grid, seed=61, tov=synth.tov_solve(), vel=0.05)
        c2p = dict(w_max=100.0, rho_atm=1e-10)
    else:
        grid = synth.make_grid(45, 38, 0.0, 0.0, 0.02, 0.025, "cart", ("periodic",) * 4)
        metric = synth.general_metric(grid, 7)
        p, eos = synth.smooth_state(grid, 8, vamp=0.5), synth.ideal_eos(5.0 / 3.0)
        c2p = dict(w_max=100.0, rho_atm=1e-12)
    q0 = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    md = {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in metric.items()}
    dt = 0.4 * min(grid["dx"], grid["dz"])
    I = lambda a: synth.interior(grid, a)  # noqa: E731
    runs = {}
    for name, mlp in (("illinois", None), ("mlp", net.buf)):
        opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=dict(c2p, mlp=mlp))
        sub = grhd.Substep(grid, eos, md, opts)
        shp = q0.shape[1:]
        qg = [torch.from_numpy(q0).to(DEV)] + [torch.zeros((5,) + shp, dtype=torch.float64, device=DEV)
                                              for _ in range(3)]
        pg = [torch.zeros((6,) + shp, dtype=torch.float64, device=DEV) for _ in range(2)]
        fg = [torch.zeros(shp, dtype=torch.uint8, device=DEV) for _ in range(2)]
        grhd.con2prim(grid, eos, md, dict(c2p, mlp=mlp), qg[0], pg[0], flags=fg[0])
        cur, outs = 0, []
        for i, st in enumerate(grhd.SSPRK3):
            dg = grhd.new_diag()
            sub.chained(dict(st, dt=dt), qg[0], qg[0] if i == 0 else qg[i], qg[i + 1], pg[cur], fg[cur],
                        pg[1 - cur], fg[1 - cur], diag=dg)
            cur = 1 - cur
            torch.cuda.synchronize()
            outs.append(dict(q=qg[i + 1].cpu().numpy(), p=pg[cur].cpu().numpy(), f=fg[cur].cpu().numpy(),
                             d=grhd.read_diag(dg)))
        runs[name] = outs
    # the oracle: each stage from the seeded run's own input (the recovery
    # of its stored q_s), then the recovery of the result
    opts_o = dict(recon="ppm", riemann="hllc", c2p=c2p)
    qn_o = orc.con2prim(grid, eos, metric, c2p, q0)[1]
    qs_in = qn_o
    for i, st in enumerate(grhd.SSPRK3):
        ref = orc.rk_substep(grid, eos, metric, opts_o, dict(st, dt=dt), qn_o, qs_in)
        p_r, q_r, fl_r, _ = orc.con2prim(grid, eos, metric, c2p, ref["qout"])
        g_, u_ = runs["mlp"][i], runs["illinois"][i]
        assert normwise(I(g_["q"]), I(q_r)) <= 1e-12, (case, i)
        assert np.array_equal(I(g_["f"]), I(fl_r)), (case, i)
        p_same = orc.con2prim(grid, eos, metric, c2p, g_["q"])[0]
        assert normwise(I(g_["p"]), I(p_same)) <= 1e-12, (case, i)
        assert percell(I(g_["p"]), I(p_same), (0,)) <= 1e-12, (case, i)
        assert percell_cond(I(g_["p"]), I(p_same), I(g_["q"])) <= 1e-12, (case, i)
        assert normwise(I(g_["q"]), I(u_["q"])) <= 1e-12, (case, i)
        assert g_["d"]["n_fail"] == u_["d"]["n_fail"] == 0
        qs_in = g_["q"]
    if case == "rotating":
        it_m = sum(o["d"]["iter_sum"] for o in runs["mlp"])
        it_i = sum(o["d"]["iter_sum"] for o in runs["illinois"])
        assert it_m < it_i, (it_m, it_i)
