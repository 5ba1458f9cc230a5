"""GPU: an SSP-RK3 step of grhd_rk_substep calls captured into a HIP graph
(torch.cuda.CUDAGraph on a side stream) replays bit for bit as the same
calls made eagerly, state and diagnostics, on every replay, with eager work
and synchronisations between the replays.  The library allocates nothing
on these calls: their scratch is the workspace the caller passes (here the
Substep's), so the captured graph holds the caller's addresses; an eager
call on a larger grid between the replays (its own workspace) changes
nothing."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_03223_amd import grhd  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_captured_step_replays_as_eager(prec):
    grid = synth.star_grid(128)
    p, metric_np, eos = synth.star_problem(grid, seed=131, tov=synth.tov_solve(), vel=0.02)
    metric = {k: torch.from_numpy(v).to(DEV) for k, v in metric_np.items()}
    sub = grhd.Substep(grid, eos, metric, dict(recon="ppm", riemann="hllc", prec=prec,
                                               c2p=dict(w_max=100.0, rho_atm=1e-10, reuse_atm=True)))
    st = [grhd.make_stage(dict(s, dt=0.4 * grid["dx"])) for s in grhd.SSPRK3]

    def state():
        pd = torch.from_numpy(np.ascontiguousarray(p)).to(DEV)
        q = torch.zeros((5,) + pd.shape[1:], dtype=torch.float64, device=DEV)
        grhd.prim2con(grid, eos, metric, pd, q, with_ghosts=True)
        return dict(q=q, q1=torch.zeros_like(q), q2=torch.zeros_like(q), p=torch.zeros_like(pd),
                    fl=torch.zeros(pd.shape[1:], dtype=torch.uint8, device=DEV), diag=grhd.new_diag())

    def step(S):
        for s, (a, b, c) in enumerate([("q", "q", "q1"), ("q", "q1", "q2"), ("q", "q2", "q")]):
            sub(st[s], S[a], S[b], S[c], S["p"], flags=S["fl"], diag=S["diag"])

    def same(x, y):
        return torch.equal(x.view(torch.int64), y.view(torch.int64))

    A, B = state(), state()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        step(B)                       # eager, on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            step(B)                   # captured, not run
    torch.cuda.current_stream().wait_stream(side)
    step(A)
    torch.cuda.synchronize()
    assert same(A["q"], B["q"])
    # a larger grid with its own Substep (and workspace), run eagerly
    # between the replays
    big = synth.star_grid(256)
    pb, mb_np, _ = synth.star_problem(big, seed=132, tov=synth.tov_solve(), vel=0.02)
    mb = {k: torch.from_numpy(v).to(DEV) for k, v in mb_np.items()}
    sub_big = grhd.Substep(big, eos, mb, dict(recon="ppm", riemann="hllc", prec=prec,
                                              c2p=dict(w_max=100.0, rho_atm=1e-10)))
    pbd = torch.from_numpy(np.ascontiguousarray(pb)).to(DEV)
    qb = torch.zeros((5,) + pbd.shape[1:], dtype=torch.float64, device=DEV)
    grhd.prim2con(big, eos, mb, pbd, qb, with_ghosts=True)
    qb1 = torch.zeros_like(qb)
    for _ in range(4):
        step(A)
        sub_big(st[0], qb, qb, qb1, torch.zeros_like(pbd), diag=grhd.new_diag())
        g.replay()
        torch.cuda.synchronize()
        x = A["q"].sum()              # eager work between the replays
        torch.cuda.synchronize()
        assert torch.isfinite(x)
        assert same(A["q"], B["q"]) and same(A["p"], B["p"]) and same(A["fl"], B["fl"])
        assert same(A["diag"], B["diag"])
