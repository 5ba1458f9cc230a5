"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/grhd.h, and rejects invalid arguments before touching
the device (GRHD_ERR_INVALID with a message)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "grhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grhd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def G():
    from paper_2502_03223_amd import grhd
    if not os.path.exists(grhd.LIB_PATH):
        pytest.skip("library not built")
    return grhd


def test_exports_every_declared_symbol(G):
    lib = G.lib()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert G.lib().grhd_version().startswith(b"grhd-mi355x")


def grid_ok():
    import synth
    return synth.make_grid(16, 8, 0.0, 0.0, 0.1, 0.1, "cyl", ("axis", "outflow", "reflect", "outflow"))


def call_substep(G, grid=None, eos=None, opts=None, stage=None, null_q=False):
    import synth
    g = G.make_grid(grid or grid_ok())
    e = G.make_eos(eos or synth.ideal_eos(2.0, 100.0))
    m = G.make_metric({})
    o = G.make_options(opts or dict(c2p=dict(w_max=100.0, rho_atm=1e-10)))
    st = G.make_stage(stage or dict(a=0.0, b=1.0, c=1.0, dt=0.01))
    q = G.Cons()
    if not null_q:
        for c in range(5):
            q.q[c] = 0x1000 + 8 * c   # never dereferenced: validation fails first
    qo = G.Cons()
    for c in range(5):
        qo.q[c] = 0x2000 + 8 * c
    p = G.Prim()
    for c in range(6):
        p.p[c] = 0x3000 + 8 * c
    return G.lib().grhd_rk_substep(C.byref(g), C.byref(e), C.byref(m), C.byref(o), C.byref(st),
                                   C.byref(q), C.byref(q), C.byref(qo), C.byref(p), None, None,
                                   None, None, None, None, 0, None)


@pytest.mark.parametrize("bad", [
    dict(grid=dict(grid_ok(), nx=0)),
    dict(grid=dict(grid_ok(), ng=2)),
    dict(grid=dict(grid_ok(), dx=-1.0)),
    dict(grid=dict(grid_ok(), pitch=10)),
    dict(grid=dict(grid_ok(), nz=8192, pitch=65536)),     # more than 2^29 cells per field
    dict(grid=dict(grid_ok(), bc=("outflow", "axis", "reflect", "outflow"))),
    dict(grid=dict(grid_ok(), bc=("periodic", "outflow", "reflect", "outflow"))),
    dict(grid=dict(grid_ok(), x0=-1.0)),
    dict(eos=dict(kind="ideal", K=[1.0], G=[0.5], rho_b=[], Gth=2.0)),
    dict(opts=dict(c2p=dict(w_max=100.0, rho_atm=0.0))),
    dict(opts=dict(c2p=dict(w_max=0.5, rho_atm=1e-10))),
    dict(stage=dict(a=0.0, b=1.0, c=1.0, dt=float("nan"))),
    dict(null_q=True),
])
def test_invalid_arguments_rejected(G, bad):
    rc = call_substep(G, **bad)
    assert rc == -1
    assert len(G.lib().grhd_last_error()) > 0


def test_null_pointers_rejected(G):
    lib = G.lib()
    assert lib.grhd_rk_substep(*([None] * 15 + [0, None])) == -1
    assert lib.grhd_con2prim(*([None] * 9 + [0, None])) == -1
    assert lib.grhd_reconstruct(None, 0, 0, 0, None, None, None, None) == -1
    assert lib.grhd_hllc_flux(None, 0, 0, 0, None, None, None, None, None, None, None) == -1
    assert lib.grhd_mlp_features(None, 0, None, None, None, None) == -1


def call_chained(G, opts=None, grid=None, alias_p=False, alias_flags=False, null_flags_out=False):
    import synth
    g = G.make_grid(grid or grid_ok())
    e = G.make_eos(synth.ideal_eos(2.0, 100.0))
    m = G.make_metric({})
    o = G.make_options(opts or dict(c2p=dict(w_max=100.0, rho_atm=1e-10)))
    st = G.make_stage(dict(a=0.0, b=1.0, c=1.0, dt=0.01))
    q, qo, pi, po = G.Cons(), G.Cons(), G.Prim(), G.Prim()
    for c in range(5):
        q.q[c] = 0x1000 + 8 * c   # never dereferenced: validation fails first
        qo.q[c] = 0x2000 + 8 * c
    for c in range(6):
        pi.p[c] = 0x3000 + 8 * c
        po.p[c] = (0x3000 if alias_p and c == 2 else 0x4000) + 8 * c
    fi = C.c_void_p(0x5000)
    fo = None if null_flags_out else C.c_void_p(0x5000 if alias_flags else 0x6000)
    return G.lib().grhd_rk_substep_chained(C.byref(g), C.byref(e), C.byref(m), C.byref(o), C.byref(st),
                                           C.byref(q), C.byref(q), C.byref(qo), C.byref(pi), fi,
                                           C.byref(po), fo, None, None, None, None, None, 0, None)


@pytest.mark.parametrize("bad,rc", [
    (dict(alias_p=True), -1),
    (dict(alias_flags=True), -1),
    (dict(null_flags_out=True), -1),
    (dict(opts=dict(c2p=dict(w_max=100.0, rho_atm=1e-10), tile=(32, 8))), -3),
    (dict(grid=dict(grid_ok(), bc=("axis", "external", "reflect", "outflow"))), -3),
])
def test_chained_arguments_rejected(G, bad, rc):
    """The chained stage rejects aliased outputs (invalid) and what it is
    not built for (unsupported: other tiles, EXTERNAL sides) before
    touching the device."""
    assert call_chained(G, **bad) == rc
    assert len(G.lib().grhd_last_error()) > 0


def test_workspace_size_and_errors(G):
    """The size query covers every part a call can use, and a call whose
    parts do not fit its workspace returns GRHD_ERR_WORKSPACE before
    launching anything (here with fake device addresses that are never
    dereferenced)."""
    import synth
    lib = G.lib()
    g = G.make_grid(grid_ok())
    n = C.c_size_t(0)
    assert lib.grhd_workspace_bytes(C.byref(g), C.byref(n)) == 0
    # 16 x 8 grid: at most 1 x 1 stage tile, 8 recovery blocks, 14 x 64 flags
    assert n.value >= 14 * 64 and n.value % 256 == 0
    big = G.make_grid(synth.make_grid(1024, 1024, 0.0, 0.0, 0.1, 0.1, "cyl",
                                      ("axis", "outflow", "reflect", "outflow")))
    nb = C.c_size_t(0)
    assert lib.grhd_workspace_bytes(C.byref(big), C.byref(nb)) == 0
    assert nb.value > n.value
    assert lib.grhd_workspace_bytes(None, C.byref(n)) == -1

    e = G.make_eos(synth.ideal_eos(2.0, 100.0))
    m = G.make_metric({})
    o = G.make_options(dict(c2p=dict(w_max=100.0, rho_atm=1e-10)))
    st = G.make_stage(dict(a=0.0, b=1.0, c=1.0, dt=0.01))
    q, qo, p = G.Cons(), G.Cons(), G.Prim()
    for c in range(5):
        q.q[c] = 0x1000 + 8 * c
        qo.q[c] = 0x2000 + 8 * c
    for c in range(6):
        p.p[c] = 0x3000 + 8 * c
    diag = C.c_void_p(0x8000)
    # diagnostics and no caller flags, but no workspace
    rc = lib.grhd_rk_substep(C.byref(g), C.byref(e), C.byref(m), C.byref(o), C.byref(st), C.byref(q),
                             C.byref(q), C.byref(qo), C.byref(p), None, None, None, None, diag,
                             None, 0, None)
    assert rc == -4 and b"workspace" in lib.grhd_last_error()
    # a workspace one byte short
    rc = lib.grhd_rk_substep(C.byref(g), C.byref(e), C.byref(m), C.byref(o), C.byref(st), C.byref(q),
                             C.byref(q), C.byref(qo), C.byref(p), None, None, None, None, diag,
                             C.c_void_p(0x100000), n.value - 1, None)
    assert rc == -4
    rc = lib.grhd_con2prim(C.byref(g), C.byref(e), C.byref(m), C.byref(o.c2p), C.byref(q), C.byref(p),
                           None, diag, None, 0, None)
    assert rc == -4
