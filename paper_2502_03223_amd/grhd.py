"""Thin ctypes binding of libgrhd.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; this module
only converts plain Python descriptions and torch device tensors into the C
structs of include/grhd.h, calls the library on the current HIP stream and
raises on any non-zero status.  There is no CPU fallback: when the library
is missing, importing the product path raises.

Plain-data conventions (shared with the tests):
  grid   dict(nx, nz, ng, pitch, x0, z0, dx, dz, geom='cyl'|'cart',
              bc=(xlo, xhi, zlo, zhi))
  eos    dict(kind='ideal'|'hybrid', K=[..], G=[..], rho_b=[..], Gth=..)
  metric dict name -> device tensor (rows, pitch) float64, or float
  c2p    dict(w_max, rho_atm[, tol, max_iter])
Cell fields are float64 device tensors of shape (nfield, rows, pitch),
rows = nz + 2 ng.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrhd.so")

METRIC_NAMES = ["alp", "bx", "by", "bz", "W", "gxx", "gxy", "gxz", "gyy",
                "gyz", "gzz", "kxx", "kxy", "kxz", "kyy", "kyz", "kzz"]
FLAT = {"alp": 1.0, "W": 1.0, "gxx": 1.0, "gyy": 1.0, "gzz": 1.0}
BC = {"outflow": 0, "periodic": 1, "axis": 2, "reflect": 3, "external": 4}
GEOM = {"cyl": 0, "cart": 1}
RECON = {"ppm": 0, "minmod": 1, "ppm3": 2}
RIEMANN = {"hllc": 0, "tvdlf": 1}
PREC = {"fp64": 0, "mixed": 1}
FACE_EPS = {"recon": 0, "eos": 1}
EOS_KIND = {"ideal": 0, "hybrid": 1}


class GrhdError(RuntimeError):
    pass


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("ng", C.c_int),
                ("pitch", C.c_int64), ("x0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dz", C.c_double), ("geom", C.c_int),
                ("bc", C.c_int * 4)]


class Eos(C.Structure):
    _fields_ = [("kind", C.c_int), ("npieces", C.c_int), ("K", C.c_double * 8),
                ("Gamma", C.c_double * 8), ("rho_b", C.c_double * 8),
                ("Gamma_th", C.c_double)]


class Metric(C.Structure):
    _fields_ = [("f", C.c_void_p * 17), ("cval", C.c_double * 17)]


class Cons(C.Structure):
    _fields_ = [("q", C.c_void_p * 5)]


class Prim(C.Structure):
    _fields_ = [("p", C.c_void_p * 6)]


class C2PParams(C.Structure):
    _fields_ = [("w_max", C.c_double), ("rho_atm", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int), ("guess", C.c_int), ("mlp", C.c_void_p),
                ("adiabatic", C.c_int), ("reuse_atm", C.c_int)]


class Options(C.Structure):
    _fields_ = [("recon", C.c_int), ("riemann", C.c_int), ("prec", C.c_int),
                ("c2p", C2PParams), ("tile_x", C.c_int), ("tile_z", C.c_int),
                ("fix_mask", C.c_void_p), ("fix_q", Cons),
                ("ev_begin", C.c_void_p), ("ev_end", C.c_void_p), ("face_eps", C.c_int)]


class Stage(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("dt", C.c_double), ("g", C.c_double), ("d", C.c_double),
                ("e", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("max_courant", C.c_double), ("Mb", C.c_double), ("J", C.c_double),
                ("n_rescale", C.c_ulonglong), ("n_cold", C.c_ulonglong),
                ("n_atm", C.c_ulonglong), ("n_fail", C.c_ulonglong),
                ("iter_sum", C.c_ulonglong), ("iter_max", C.c_ulonglong)]


class Level(C.Structure):
    _fields_ = [("grid", Grid), ("metric", Metric), ("q", Cons), ("q1", Cons), ("q2", Cons),
                ("p", Prim), ("slice", Prim * 3), ("reg_child_bnd", C.c_void_p),
                ("reg_parent_int", C.c_void_p), ("nbuf", C.c_int)]


class Patch(C.Structure):
    _fields_ = [("grid", Grid), ("metric", Metric), ("qn", Cons), ("qs", Cons),
                ("qout", Cons), ("p", Prim), ("stage", Stage), ("eos_id", C.c_int),
                ("flux_reg", C.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GrhdError("libgrhd.so is not built (run __graft_entry__.build())")
        _lib = C.CDLL(LIB_PATH)
        p, i = C.c_void_p, C.c_int
        sig = {
            "grhd_con2prim": [p, p, p, p, p, p, p, p, p, C.c_size_t, p],
            "grhd_workspace_bytes": [p, p],
            "grhd_prim2con": [p, p, p, p, p, i, p],
            "grhd_reconstruct": [p, i, i, i, p, p, p, p],
            "grhd_hllc_flux": [p, i, i, i, p, p, p, p, p, p, p],
            "grhd_rk_substep": [p] * 14 + [p, C.c_size_t, p],
            "grhd_rk_substep_noalloc": [p] * 15,
            "grhd_rk_substep_chained": [p] * 16 + [p, C.c_size_t, p],
            "grhd_fix_cells": [p, p, p, p, p],
            "grhd_fmr_prolong": [p, p, i, p, C.c_double, p, p, p, C.c_double, p, p, p],
            "grhd_fmr_restrict": [p, p, p, p, p],
            "grhd_fmr_reflux": [p, p, p, p, p, p],
            "grhd_fmr_create": [p, i, p, p, i, C.c_double, p, p],
            "grhd_fmr_step": [p, C.c_double, p],
            "grhd_fmr_time": [p, p],
            "grhd_fmr_destroy": [p],
            "grhd_plan_create": [p, i, p, i, p, C.c_char_p, p],
            "grhd_batch_levels": [p, p, i, p, p],
            "grhd_plan_destroy": [p],
            "grhd_plan_tile": [p, p, p],
            "grhd_autotune": [p, i, p, i, p, C.c_char_p, p, p],
            "grhd_event_create": [p],
            "grhd_event_elapsed_ms": [p, p, p],
            "grhd_event_destroy": [p],
        }
        for name, args in sig.items():
            fn = getattr(_lib, name, None)
            if fn is None:
                continue
            fn.restype = C.c_int
            fn.argtypes = args
        _lib.grhd_last_error.restype = C.c_char_p
        _lib.grhd_version.restype = C.c_char_p
    return _lib


def exported_symbols():
    return [n for n in dir(lib()) if n.startswith("grhd_")]


def _check(rc, what):
    if rc != 0:
        msg = lib().grhd_last_error().decode()
        raise GrhdError("%s failed (%d): %s" % (what, rc, msg))


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------ marshalling

def make_grid(g):
    s = Grid()
    s.nx, s.nz, s.ng, s.pitch = g["nx"], g["nz"], g["ng"], g["pitch"]
    s.x0, s.z0, s.dx, s.dz = g["x0"], g["z0"], g["dx"], g["dz"]
    s.geom = GEOM[g["geom"]]
    for k in range(4):
        s.bc[k] = BC[g["bc"][k]]
    return s


def make_eos(e):
    s = Eos()
    s.kind = EOS_KIND[e["kind"]]
    s.npieces = len(e["K"])
    for k, (K, G) in enumerate(zip(e["K"], e["G"])):
        s.K[k], s.Gamma[k] = K, G
    for k, r in enumerate(e.get("rho_b", [])):
        s.rho_b[k] = r
    s.Gamma_th = e["Gth"]
    return s


def _dptr(t):
    assert t.is_cuda and t.dtype == torch.float64, "metric fields must be float64 device tensors"
    assert t.is_contiguous()
    return t.data_ptr()


def make_metric(m):
    s = Metric()
    for k, name in enumerate(METRIC_NAMES):
        v = m.get(name, FLAT.get(name, 0.0))
        if isinstance(v, torch.Tensor):
            s.f[k] = _dptr(v)
            s.cval[k] = 0.0
        else:
            s.f[k] = None
            s.cval[k] = float(v)
    return s


def _fields(t, nf, dtype=torch.float64):
    assert t is not None and t.is_cuda and t.dtype == dtype and t.is_contiguous()
    assert t.shape[0] == nf
    stride = t.stride(0) * t.element_size()
    return [t.data_ptr() + c * stride for c in range(nf)]


def make_cons(t):
    s = Cons()
    for c, ptr in enumerate(_fields(t, 5)):
        s.q[c] = ptr
    return s


def make_prim(t, dtype=torch.float64):
    s = Prim()
    for c, ptr in enumerate(_fields(t, 6, dtype)):
        s.p[c] = ptr
    return s


def make_c2p(c):
    s = C2PParams()
    s.w_max, s.rho_atm = c["w_max"], c["rho_atm"]
    s.tol = c.get("tol", 0.0)
    s.max_iter = c.get("max_iter", 0)
    s.guess = 1 if c.get("mlp") is not None else 0
    s.mlp = c["mlp"].data_ptr() if c.get("mlp") is not None else None
    s.adiabatic = 1 if c.get("adiabatic") else 0
    s.reuse_atm = 1 if c.get("reuse_atm") else 0
    return s


def make_stage(st):
    s = Stage()
    s.a, s.b, s.c, s.dt = st["a"], st["b"], st["c"], st["dt"]
    s.g, s.d, s.e = st.get("g", 0.0), st.get("d", 0.0), st.get("e", 0.0)
    return s


def make_options(o):
    s = Options()
    s.recon = RECON[o.get("recon", "ppm")]
    s.riemann = RIEMANN[o.get("riemann", "hllc")]
    s.prec = PREC[o.get("prec", "fp64")]
    s.face_eps = FACE_EPS[o.get("face_eps", "recon")]
    s.c2p = make_c2p(o["c2p"])
    tile = o.get("tile", (0, 0))
    s.tile_x, s.tile_z = tile
    fix = o.get("fix")
    if fix is not None:   # (mask uint8 cell tensor, q_fixed)
        s.fix_mask = fix[0].data_ptr()
        s.fix_q = make_cons(fix[1])
    ev = o.get("events")
    if ev is not None:
        s.ev_begin, s.ev_end = ev[0].handle, ev[1].handle
    return s


def new_diag(device="cuda"):
    return torch.zeros(16, dtype=torch.float64, device=device)  # >= sizeof(grhd_diag)


def read_diag(t):
    raw = t.cpu().numpy().tobytes()
    d = Diag.from_buffer_copy(raw[:C.sizeof(Diag)])
    return {k: getattr(d, k) for k, _ in Diag._fields_}


# ------------------------------------------------------------ calls

def workspace_bytes(grid):
    """Bytes of device workspace the single-patch calls need on this grid."""
    n = C.c_size_t(0)
    g = grid if isinstance(grid, Grid) else make_grid(grid)
    _check(lib().grhd_workspace_bytes(C.byref(g), C.byref(n)), "grhd_workspace_bytes")
    return n.value


def new_workspace(grid, device="cuda"):
    """A device workspace for the single-patch calls on this grid (torch
    allocations are 512-byte aligned)."""
    return torch.empty(max(workspace_bytes(grid), 256), dtype=torch.uint8, device=device)


def _ws_args(ws):
    if ws is None:
        return C.c_void_p(0), C.c_size_t(0)
    return C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel() * ws.element_size())


def con2prim(grid, eos, metric, c2p, q, p, flags=None, diag=None, workspace=None):
    """q (5,rows,pitch) in/out, p (6,rows,pitch) out.  With diag and no
    workspace, one is allocated for the call."""
    if diag is not None and workspace is None:
        workspace = new_workspace(grid, q.device)
    wp, wb = _ws_args(workspace)
    rc = lib().grhd_con2prim(
        C.byref(make_grid(grid)), C.byref(make_eos(eos)), C.byref(make_metric(metric)),
        C.byref(make_c2p(c2p)), C.byref(make_cons(q)), C.byref(make_prim(p)),
        C.c_void_p(flags.data_ptr() if flags is not None else 0),
        C.c_void_p(diag.data_ptr() if diag is not None else 0), wp, wb, _stream())
    _check(rc, "grhd_con2prim")


def prim2con(grid, eos, metric, p, q, with_ghosts=False):
    rc = lib().grhd_prim2con(C.byref(make_grid(grid)), C.byref(make_eos(eos)),
                             C.byref(make_metric(metric)), C.byref(make_prim(p)),
                             C.byref(make_cons(q)), 1 if with_ghosts else 0, _stream())
    _check(rc, "grhd_prim2con")


def face_shape(grid, dirn):
    nx, nz = grid["nx"], grid["nz"]
    return (nz, nx + 1) if dirn == 0 else (nz + 1, nx)


def reconstruct(grid, dirn, recon, p, prec="fp64"):
    dt = torch.float64 if prec == "fp64" else torch.float32
    shp = face_shape(grid, dirn)
    pL = torch.empty((6,) + shp, dtype=dt, device=p.device)
    pR = torch.empty((6,) + shp, dtype=dt, device=p.device)
    rc = lib().grhd_reconstruct(C.byref(make_grid(grid)), dirn, RECON[recon], PREC[prec],
                                C.byref(make_prim(p)), C.byref(make_prim(pL, dt)),
                                C.byref(make_prim(pR, dt)), _stream())
    _check(rc, "grhd_reconstruct")
    return pL, pR


def hllc_flux(grid, dirn, riemann, eos, metric, pL, pR, prec="fp64"):
    dt = torch.float64 if prec == "fp64" else torch.float32
    F = torch.empty((5,) + tuple(pL.shape[1:]), dtype=torch.float64, device=pL.device)
    sp = torch.zeros(1, dtype=torch.float64, device=pL.device)
    rc = lib().grhd_hllc_flux(C.byref(make_grid(grid)), dirn, RIEMANN[riemann], PREC[prec],
                              C.byref(make_eos(eos)), C.byref(make_metric(metric)),
                              C.byref(make_prim(pL, dt)), C.byref(make_prim(pR, dt)),
                              C.byref(make_cons(F)), C.c_void_p(sp.data_ptr()), _stream())
    _check(rc, "grhd_hllc_flux")
    return F, sp


class Substep:
    """Pre-marshalled arguments of repeated grhd_rk_substep calls (the
    structs are built once; only the stage and buffers change)."""

    def __init__(self, grid, eos, metric, opts, workspace=None):
        """workspace: device workspace of grhd_workspace_bytes(grid) bytes
        (allocated here when not given; calls through one Substep share it,
        so they must not run at the same time)."""
        self.grid = make_grid(grid)
        self.eos = make_eos(eos)
        self.metric = make_metric(metric)
        self.opts = make_options(opts)
        self._keep = (grid, eos, metric, opts)
        self.ws = workspace if workspace is not None else new_workspace(self.grid)
        self._wsa = _ws_args(self.ws)

    def __call__(self, stage, qn, qs, qout, p, acc_in=None, acc_out=None, flux_reg=None,
                 flags=None, diag=None, stream=None, events=None):
        """events: optional (begin, end) Event pair recorded around the fused
        stage kernel of this call."""
        st = make_stage(stage) if isinstance(stage, dict) else stage
        if events is not None:
            self.opts.ev_begin, self.opts.ev_end = events[0].handle, events[1].handle
        else:
            self.opts.ev_begin = self.opts.ev_end = None
        rc = lib().grhd_rk_substep(
            C.byref(self.grid), C.byref(self.eos), C.byref(self.metric), C.byref(self.opts),
            C.byref(st), C.byref(make_cons(qn if qn is not None else qs)),
            C.byref(make_cons(qs)), C.byref(make_cons(qout)), C.byref(make_prim(p)),
            C.byref(make_cons(acc_in)) if acc_in is not None else None,
            C.byref(make_cons(acc_out)) if acc_out is not None else None,
            C.c_void_p(flux_reg.data_ptr() if flux_reg is not None else 0),
            C.c_void_p(flags.data_ptr() if flags is not None else 0),
            C.c_void_p(diag.data_ptr() if diag is not None else 0), *self._wsa,
            C.c_void_p(stream) if stream is not None else _stream())
        _check(rc, "grhd_rk_substep")


    def bind(self, stage, qn, qs, qout, p, diag=None, stream=None, flags=None):
        """A call of this substep with every argument marshalled once (for
        loops that repeat the same calls)."""
        L = lib()
        st = make_stage(stage) if isinstance(stage, dict) else stage
        args = (C.byref(self.grid), C.byref(self.eos), C.byref(self.metric), C.byref(self.opts),
                C.byref(st), C.byref(make_cons(qn if qn is not None else qs)),
                C.byref(make_cons(qs)), C.byref(make_cons(qout)), C.byref(make_prim(p)), None, None,
                C.c_void_p(0), C.c_void_p(flags.data_ptr() if flags is not None else 0),
                C.c_void_p(diag.data_ptr() if diag is not None else 0), *self._wsa,
                C.c_void_p(stream) if stream is not None else _stream())
        keep = (st, qn, qs, qout, p, diag, flags, self.ws)

        def call():
            _check(L.grhd_rk_substep(*args), "grhd_rk_substep")
        call.keep = keep
        return call


    def _chained_args(self, stage, qn, qs, qout, p_in, flags_in, p_out, flags_out, acc_in, acc_out,
                      flux_reg, diag, stream):
        st = make_stage(stage) if isinstance(stage, dict) else stage
        args = (C.byref(self.grid), C.byref(self.eos), C.byref(self.metric), C.byref(self.opts),
                C.byref(st), C.byref(make_cons(qn if qn is not None else qs)),
                C.byref(make_cons(qs)), C.byref(make_cons(qout)), C.byref(make_prim(p_in)),
                C.c_void_p(flags_in.data_ptr() if flags_in is not None else 0),
                C.byref(make_prim(p_out)), C.c_void_p(flags_out.data_ptr()),
                C.byref(make_cons(acc_in)) if acc_in is not None else None,
                C.byref(make_cons(acc_out)) if acc_out is not None else None,
                C.c_void_p(flux_reg.data_ptr() if flux_reg is not None else 0),
                C.c_void_p(diag.data_ptr() if diag is not None else 0), *self._wsa,
                C.c_void_p(stream) if stream is not None else _stream())
        return st, args

    def chained(self, stage, qn, qs, qout, p_in, flags_in, p_out, flags_out, acc_in=None,
                acc_out=None, flux_reg=None, diag=None, stream=None, events=None):
        """grhd_rk_substep_chained: the stage with the recovery of q_out at
        its end; p_in/flags_in hold the recovery of q_s, p_out/flags_out
        receive that of q_out."""
        if events is not None:
            self.opts.ev_begin, self.opts.ev_end = events[0].handle, events[1].handle
        else:
            self.opts.ev_begin = self.opts.ev_end = None
        _, args = self._chained_args(stage, qn, qs, qout, p_in, flags_in, p_out, flags_out, acc_in,
                                     acc_out, flux_reg, diag, stream)
        _check(lib().grhd_rk_substep_chained(*args), "grhd_rk_substep_chained")

    def bind_chained(self, stage, qn, qs, qout, p_in, flags_in, p_out, flags_out, diag=None,
                     stream=None):
        """A chained call with every argument marshalled once."""
        L = lib()
        st, args = self._chained_args(stage, qn, qs, qout, p_in, flags_in, p_out, flags_out, None,
                                      None, None, diag, stream)
        keep = (st, qn, qs, qout, p_in, flags_in, p_out, flags_out, diag, self.ws)

        def call():
            _check(L.grhd_rk_substep_chained(*args), "grhd_rk_substep_chained")
        call.keep = keep
        return call


def rk_substep(grid, eos, metric, opts, stage, qn, qs, qout, p, **kw):
    Substep(grid, eos, metric, opts)(stage, qn, qs, qout, p, **kw)


SSPRK3 = [dict(a=0.0, b=1.0, c=1.0), dict(a=0.75, b=0.25, c=0.25),
          dict(a=1.0 / 3.0, b=2.0 / 3.0, c=2.0 / 3.0)]


# ------------------------------------------------------------ batched path

def make_patch(d):
    """d: dict(grid, metric, qn, qs, qout, p, stage, eos_id[, flux_reg])."""
    s = Patch()
    s.grid = make_grid(d["grid"])
    s.metric = make_metric(d["metric"])
    s.qn = make_cons(d["qn"] if d.get("qn") is not None else d["qs"])
    s.qs = make_cons(d["qs"])
    s.qout = make_cons(d["qout"])
    s.p = make_prim(d["p"])
    s.stage = make_stage(d["stage"])
    s.eos_id = d.get("eos_id", 0)
    fr = d.get("flux_reg")
    s.flux_reg = fr.data_ptr() if fr is not None else None
    return s


def autotune(patches, eos_table, opts, tune_cache=None):
    """grhd_autotune: the tile shapes a plan for these patches would use
    (may time the candidates on the patches' buffers)."""
    n = len(patches)
    arr = (Patch * n)(*[make_patch(d) for d in patches])
    eos_arr = (Eos * len(eos_table))(*[make_eos(e) for e in eos_table])
    o = make_options(opts)
    tx = (C.c_int * 2)()
    tz = (C.c_int * 2)()
    _check(lib().grhd_autotune(arr, n, eos_arr, len(eos_table), C.byref(o),
                               tune_cache.encode() if tune_cache else None, tx, tz), "grhd_autotune")
    return dict(square=(tx[0], tz[0]), thin=(tx[1], tz[1]))


class Plan:
    """A grhd_plan: one graph-captured substep over many patches.
    Creating it may run the batch on the given buffers to time candidate
    tile shapes (q_s corrected in place, q_out overwritten)."""

    def __init__(self, patches, eos_table, opts, tune_cache=None):
        lib()
        self.n = len(patches)
        arr = (Patch * self.n)(*[make_patch(d) for d in patches])
        eos_arr = (Eos * len(eos_table))(*[make_eos(e) for e in eos_table])
        self._opts = make_options(opts)
        self.handle = C.c_void_p()
        rc = lib().grhd_plan_create(arr, self.n, eos_arr, len(eos_table), C.byref(self._opts),
                                    tune_cache.encode() if tune_cache else None,
                                    C.byref(self.handle))
        _check(rc, "grhd_plan_create")

    def table(self, patches):
        """Marshalled patch table, reusable across calls with the same
        buffers and stages."""
        return (Patch * self.n)(*[make_patch(d) for d in patches])

    def __call__(self, patches, diag=None, stream=None):
        arr = patches if isinstance(patches, C.Array) else self.table(patches)
        rc = lib().grhd_batch_levels(self.handle, arr, self.n,
                                     C.c_void_p(diag.data_ptr() if diag is not None else 0),
                                     C.c_void_p(stream) if stream is not None else _stream())
        _check(rc, "grhd_batch_levels")

    def tiles(self):
        tx = (C.c_int * 2)()
        tz = (C.c_int * 2)()
        _check(lib().grhd_plan_tile(self.handle, tx, tz), "grhd_plan_tile")
        return dict(square=(tx[0], tz[0]), thin=(tx[1], tz[1]))

    def close(self):
        if self.handle:
            lib().grhd_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ timing

class Event:
    """HIP event (timing enabled) owned by the library's helpers."""

    def __init__(self):
        L = lib()
        h = C.c_void_p()
        _check(L.grhd_event_create(C.byref(h)), "grhd_event_create")
        self.handle = h

    def elapsed_ms(self, end):
        ms = C.c_float()
        _check(lib().grhd_event_elapsed_ms(self.handle, end.handle, C.byref(ms)),
               "grhd_event_elapsed_ms")
        return ms.value

    def __del__(self):
        try:
            lib().grhd_event_destroy(self.handle)
        except Exception:
            pass


def fix_cells(grid, mask, q_fixed, q):
    """grhd_fix_cells: q = q_fixed where mask (uint8 cell tensor) is set."""
    assert mask.is_cuda and mask.dtype == torch.uint8 and mask.is_contiguous()
    rc = lib().grhd_fix_cells(C.byref(make_grid(grid)), C.c_void_p(mask.data_ptr()),
                              C.byref(make_cons(q_fixed)), C.byref(make_cons(q)), _stream())
    _check(rc, "grhd_fix_cells")


# ------------------------------------------------------------ mesh refinement

def fmr_prolong(pgrid, slices, times, t, cgrid, cmetric, eos, rho_atm, p_child, q_child):
    """grhd_fmr_prolong: slices = list of 1-3 (6, rows, pitch) parent
    primitive tensors, oldest first, with their times."""
    arr = (Prim * len(slices))(*[make_prim(x) for x in slices])
    tm = (C.c_double * len(times))(*times)
    rc = lib().grhd_fmr_prolong(C.byref(make_grid(pgrid)), arr, len(slices), tm, float(t),
                                C.byref(make_grid(cgrid)), C.byref(make_metric(cmetric)),
                                C.byref(make_eos(eos)), float(rho_atm), C.byref(make_prim(p_child)),
                                C.byref(make_cons(q_child)), _stream())
    _check(rc, "grhd_fmr_prolong")


def fmr_restrict(pgrid, q_parent, cgrid, q_child):
    rc = lib().grhd_fmr_restrict(C.byref(make_grid(pgrid)), C.byref(make_cons(q_parent)),
                                 C.byref(make_grid(cgrid)), C.byref(make_cons(q_child)), _stream())
    _check(rc, "grhd_fmr_restrict")


def fmr_reflux(pgrid, q_parent, reg_parent, cgrid, reg_child):
    for r in (reg_parent, reg_child):
        assert r.is_cuda and r.dtype == torch.float64 and r.is_contiguous()
    rc = lib().grhd_fmr_reflux(C.byref(make_grid(pgrid)), C.byref(make_cons(q_parent)),
                               C.c_void_p(reg_parent.data_ptr()), C.byref(make_grid(cgrid)),
                               C.c_void_p(reg_child.data_ptr()), _stream())
    _check(rc, "grhd_fmr_reflux")


class Hierarchy:
    """A grhd_fmr driver over levels given as dicts (grid, metric, q, and
    nbuf: 0 for the halo schedule, the buffer width for the buffer
    schedule); the stage buffers, recovery workspace, slices and registers
    are allocated here as device tensors and handed to the library."""

    def __init__(self, levels, eos, opts, l_fix=0, t0=0.0):
        lib()
        n = len(levels)
        self.levels = levels
        self.bufs = []
        arr = (Level * n)()
        for l, d in enumerate(levels):
            q = d["q"]
            shp = q.shape[1:]
            b = dict(q1=torch.zeros_like(q), q2=torch.zeros_like(q),
                     p=torch.zeros((6,) + shp, dtype=torch.float64, device=q.device))
            b["slices"] = [torch.zeros((6,) + shp, dtype=torch.float64, device=q.device)
                           for _ in range(3 if l + 1 < n else 0)]
            g = d["grid"]
            nb = int(d.get("nbuf", 0))
            b["reg_child_bnd"] = (torch.zeros(5 * (g["nx"] + g["nz"] - 2 * nb), dtype=torch.float64,
                                              device=q.device) if l > 0 else None)
            if l + 1 < n:
                cg, cb = levels[l + 1]["grid"], int(levels[l + 1].get("nbuf", 0))
                b["reg_parent_int"] = torch.zeros(5 * ((cg["nx"] - cb) // 2 + (cg["nz"] - cb) // 2),
                                                  dtype=torch.float64, device=q.device)
            else:
                b["reg_parent_int"] = None
            L = arr[l]
            L.grid = make_grid(g)
            L.metric = make_metric(d["metric"])
            L.q = make_cons(q)
            L.q1 = make_cons(b["q1"])
            L.q2 = make_cons(b["q2"])
            L.p = make_prim(b["p"])
            for s_, t_ in enumerate(b["slices"]):
                L.slice[s_] = make_prim(t_)
            L.reg_child_bnd = b["reg_child_bnd"].data_ptr() if b["reg_child_bnd"] is not None else None
            L.reg_parent_int = b["reg_parent_int"].data_ptr() if b["reg_parent_int"] is not None else None
            L.nbuf = nb
            self.bufs.append(b)
        self._arr = arr
        self._opts = make_options(opts)
        self._eos = make_eos(eos)
        self.handle = C.c_void_p()
        _check(lib().grhd_fmr_create(arr, n, C.byref(self._eos), C.byref(self._opts), int(l_fix), float(t0),
                                     C.byref(self.handle), _stream()), "grhd_fmr_create")

    def step(self, dt0):
        _check(lib().grhd_fmr_step(self.handle, float(dt0), _stream()), "grhd_fmr_step")

    @property
    def time(self):
        t = C.c_double()
        _check(lib().grhd_fmr_time(self.handle, C.byref(t)), "grhd_fmr_time")
        return t.value

    def close(self):
        if self.handle:
            torch.cuda.synchronize()
            lib().grhd_fmr_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ learned guess

NPARAM_MLP = 4481


def _fptr(t):
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _mlp_sigs():
    L = lib()
    if getattr(L, "_mlp_sig", False):
        return L
    p, i, f = C.c_void_p, C.c_int, C.c_float
    L.grhd_mlp_bytes.restype = C.c_size_t
    L.grhd_mlp_bytes.argtypes = []
    L.grhd_mlp_features.restype = C.c_int
    L.grhd_mlp_features.argtypes = [C.POINTER(Cons), C.c_longlong, p, p, p, p]
    for name, args in {"grhd_mlp_pack": [p, p, p, p],
                       "grhd_mlp_forward": [p, p, p, i, p],
                       "grhd_mlp_grad": [p, p, p, p, i, p, p],
                       "grhd_mlp_train_step": [p, p, p, p, p, p, p, i, f, i, p, p]}.items():
        fn = getattr(L, name)
        fn.restype = C.c_int
        fn.argtypes = args
    L._mlp_sig = True
    return L


class MLP:
    """Device weight buffer of the learned recovery guess plus its FP32
    master parameters and Adam state.  scal: feature mean[3], std[3],
    target mean, std (float32 device tensor of 8)."""

    def __init__(self, params, scal):
        L = _mlp_sigs()
        dev = params.device
        self.buf = torch.zeros(int(L.grhd_mlp_bytes()), dtype=torch.uint8, device=dev)
        self.params = params.contiguous()
        self.scal = scal.contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step_no = 0
        self.pack()

    def pack(self):
        _check(_mlp_sigs().grhd_mlp_pack(C.c_void_p(self.buf.data_ptr()), _fptr(self.params),
                                         _fptr(self.scal), _stream()), "grhd_mlp_pack")

    def forward(self, X):
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(_mlp_sigs().grhd_mlp_forward(C.c_void_p(self.buf.data_ptr()), _fptr(X), _fptr(y),
                                            X.shape[0], _stream()), "grhd_mlp_forward")
        return y

    def train_step(self, X, t, lr):
        self.step_no += 1
        _check(_mlp_sigs().grhd_mlp_train_step(
            C.c_void_p(self.buf.data_ptr()), _fptr(self.params), _fptr(self.m), _fptr(self.v),
            _fptr(self.grad), _fptr(X), _fptr(t), X.shape[0], C.c_float(lr), self.step_no,
            _fptr(self.loss), _stream()), "grhd_mlp_train_step")
        return self.loss


def mlp_grad(params, X, t):
    grad = torch.empty_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=params.device)
    _check(_mlp_sigs().grhd_mlp_grad(_fptr(params), _fptr(grad), _fptr(X), _fptr(t), X.shape[0],
                                     _fptr(loss), _stream()), "grhd_mlp_grad")
    return grad, loss


def mlp_init(seed, device="cuda"):
    """He-initialised FP32 parameter vector (W1[64][3], b1, W2[64][64], b2, w3, b3)."""
    g = torch.Generator().manual_seed(seed)
    P = torch.zeros(NPARAM_MLP, dtype=torch.float32)
    P[0:192] = torch.randn(192, generator=g) * (2.0 / 3.0) ** 0.5
    P[256:4352] = torch.randn(4096, generator=g) * (2.0 / 64.0) ** 0.5
    P[4416:4480] = torch.randn(64, generator=g) * (1.0 / 64.0) ** 0.5
    return P.to(device)


def recovery_features(q, P=None):
    """Unscaled training features (log10 D, S/E, log10(tau/D)) of n samples
    of densitised conserved variables of a flat Cartesian metric (q: 5 x n
    float64 device tensor, each row contiguous), computed by
    grhd_mlp_features; with P (n float64, the samples' pressures) also the
    target log10(P/D).  Returns X (n x 3), or (X, y)."""
    assert q.is_cuda and q.dtype == torch.float64 and q.shape[0] == 5
    n = q.shape[1]
    s = Cons()
    for c in range(5):
        assert q[c].is_contiguous()
        s.q[c] = q[c].data_ptr()
    X = torch.empty((n, 3), dtype=torch.float64, device=q.device)
    y = None
    if P is not None:
        assert P.is_cuda and P.dtype == torch.float64 and P.is_contiguous() and P.shape[0] == n
        y = torch.empty(n, dtype=torch.float64, device=q.device)
    vp = lambda t: C.c_void_p(t.data_ptr() if t is not None else 0)  # noqa: E731
    _check(_mlp_sigs().grhd_mlp_features(C.byref(s), n, vp(P), vp(X), vp(y), _stream()),
           "grhd_mlp_features")
    return X if P is None else (X, y)
