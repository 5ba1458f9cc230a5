"""GPU: recovery with reuse_atm (a cell that was and stays atmosphere keeps
the primitives the last recovery wrote) ends bit for bit as the recovery
that writes every cell.

- two SSP-RK3 steps of the star through grhd_rk_substep with caller flags
  (zero at the start), the chained stages and grhd_con2prim: q, p and the
  flags after every stage equal those of the same calls with reuse_atm = 0,
  in FP64 and in mixed precision;
- the mode does skip: primitives overwritten by the host at cells whose
  flag is ATM stay as they are after a recovery that resets those cells to
  the atmosphere again, and are rewritten with reuse_atm = 0;
- without caller flags grhd_rk_substep ignores the option (its flag
  scratch may come from another call).
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
C2P = dict(w_max=100.0, rho_atm=1e-10)
ATM = 4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def star(orc):
    grid = synth.star_grid(96)
    p, metric, eos = synth.star_problem(grid, seed=121, tov=synth.tov_solve(), vel=0.05)
    q = orc.prim2con(grid, eos, metric, p, with_ghosts=True)
    md = {k: dev(v) if isinstance(v, np.ndarray) else v for k, v in metric.items()}
    return grid, eos, md, q


def same(a, b):
    return torch.equal(a.view(torch.int64) if a.dtype == torch.float64 else a,
                       b.view(torch.int64) if b.dtype == torch.float64 else b)


def separate_run(grid, eos, md, q0, prec, reuse):
    opts = dict(recon="ppm", riemann="hllc", prec=prec, c2p=dict(C2P, reuse_atm=reuse))
    sub = grhd.Substep(grid, eos, md, opts)
    q = dev(q0)
    q1, q2 = torch.zeros_like(q), torch.zeros_like(q)
    shp = q.shape[1:]
    p = torch.zeros((6,) + shp, dtype=torch.float64, device=DEV)
    fl = torch.zeros(shp, dtype=torch.uint8, device=DEV)
    dt = 0.4 * grid["dx"]
    out = []
    for _ in range(2):
        for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)]):
            sub(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, p, flags=fl)
            out.append((qo.clone(), p.clone(), fl.clone()))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separate_stages_unchanged(star, prec):
    grid, eos, md, q0 = star
    a = separate_run(grid, eos, md, q0, prec, False)
    b = separate_run(grid, eos, md, q0, prec, True)
    stay = 0
    for i, ((qa, pa, fa), (qb, pb, fb)) in enumerate(zip(a, b)):
        assert same(qa, qb) and same(pa, pb) and same(fa, fb), i
        if i:
            stay += int(((a[i - 1][2] & ATM) & (fa & ATM)).count_nonzero())
    assert stay > 1000   # the skipped writes were exercised


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chained_stages_unchanged(star, prec):
    grid, eos, md, q0 = star
    outs = []
    for reuse in (False, True):
        c2p = dict(C2P, reuse_atm=reuse)
        sub = grhd.Substep(grid, eos, md, dict(recon="ppm", riemann="hllc", prec=prec, c2p=c2p))
        q = dev(q0)
        q1, q2 = torch.zeros_like(q), torch.zeros_like(q)
        shp = q.shape[1:]
        pp = [torch.zeros((6,) + shp, dtype=torch.float64, device=DEV) for _ in range(2)]
        ff = [torch.zeros(shp, dtype=torch.uint8, device=DEV) for _ in range(2)]
        grhd.con2prim(grid, eos, md, c2p, q, pp[0], flags=ff[0])
        dt = 0.4 * grid["dx"]
        cur, out = 0, []
        for _ in range(2):
            for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)]):
                sub.chained(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, pp[cur], ff[cur], pp[1 - cur], ff[1 - cur])
                cur = 1 - cur
                out.append((qo.clone(), pp[cur].clone(), ff[cur].clone()))
        torch.cuda.synchronize()
        outs.append(out)
    for i, ((qa, pa, fa), (qb, pb, fb)) in enumerate(zip(*outs)):
        assert same(qa, qb) and same(pa, pb) and same(fa, fb), i


def test_con2prim_skips_and_flagless_substep_ignores(star):
    """Every recovery below takes a fresh copy of the same q (a recovery
    corrects q in place), so all of them flag the same cells."""
    grid, eos, md, q0 = star
    shp = q0.shape[1:]
    p = torch.zeros((6,) + shp, dtype=torch.float64, device=DEV)
    fl = torch.zeros(shp, dtype=torch.uint8, device=DEV)
    grhd.con2prim(grid, eos, md, dict(C2P, reuse_atm=True), dev(q0), p, flags=fl)
    ref, fref = p.clone(), fl.clone()
    atm = (fl & ATM).bool()
    assert int(atm.count_nonzero()) > 1000
    # host-written marker at the atmosphere cells: kept with reuse_atm ...
    p[:, atm] = 7.0
    grhd.con2prim(grid, eos, md, dict(C2P, reuse_atm=True), dev(q0), p, flags=fl)
    torch.cuda.synchronize()
    assert same(fl, fref)
    assert bool((p[:, atm] == 7.0).all())
    assert same(p[:, ~atm], ref[:, ~atm])
    # ... and rewritten without it
    grhd.con2prim(grid, eos, md, dict(C2P, reuse_atm=False), dev(q0), p, flags=fl)
    torch.cuda.synchronize()
    assert same(p, ref)
    # grhd_rk_substep without caller flags writes every cell
    sub = grhd.Substep(grid, eos, md, dict(recon="ppm", riemann="hllc", prec="fp64",
                                            c2p=dict(C2P, reuse_atm=True)))
    st = dict(grhd.SSPRK3[0], dt=0.4 * grid["dx"])
    q = dev(q0)
    qo = torch.zeros_like(q)
    sub(st, q, q, qo, p)     # primes the flag scratch
    p[:, atm] = 7.0
    q = dev(q0)
    sub(st, q, q, qo, p)
    torch.cuda.synchronize()
    assert same(p, ref)
