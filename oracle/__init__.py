"""Plain FP64 CPU oracle of the GRHD Runge-Kutta substep (ctypes binding).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product package never does, and it never imports the product
package.  The C sources follow Lam & Shibata (arXiv 2502.03223) Sec. II.C;
see the header comments of ``or_hydro.c``, ``or_riemann.c`` and ``or_mlp.c``.

Plain-data conventions shared with the callers (data formats, not code):
  grid   dict(nx, nz, ng, pitch, x0, z0, dx, dz, geom='cyl'|'cart',
              bc=(xlo, xhi, zlo, zhi) names from BC_NAMES)
  eos    dict(kind='ideal'|'hybrid', K=[..], G=[..], rho_b=[..], Gth=..)
  metric dict name -> array (nz+2ng, pitch) or float; missing names take the
         flat-space value (alp=1, W=1, gxx=gyy=gzz=1, others 0)
  c2p    dict(w_max, rho_atm)
Cell fields are float64 arrays of shape (nfield, nz+2ng, pitch).
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = ["or_hydro.c", "or_riemann.c", "or_mlp.c", "or_fmr.c"]

METRIC_NAMES = ["alp", "bx", "by", "bz", "W", "gxx", "gxy", "gxz", "gyy",
                "gyz", "gzz", "kxx", "kxy", "kxz", "kyy", "kyz", "kzz"]
FLAT = {"alp": 1.0, "W": 1.0, "gxx": 1.0, "gyy": 1.0, "gzz": 1.0}
BC_NAMES = {"outflow": 0, "periodic": 1, "axis": 2, "reflect": 3, "external": 4}
RECON = {"ppm": 0, "minmod": 1, "ppm3": 2}
RIEMANN = {"hllc": 0, "tvdlf": 1}
# face states of the stage: "recon" reconstructs every primitive (Sec.
# II.C.2); "eos" takes eps from the EOS at the reconstructed (rho, P)
FACE_EPS = {"recon": 0, "eos": 1}
NPARAM_MLP = 4481


def build(force=True):
    """Compile the oracle with gcc -O3 (no FMA contraction, no fast-math:
    the optimisation level changes no result)."""
    srcs = [os.path.join(_HERE, s) for s in _SRCS]
    if not force and os.path.exists(_SO) and all(
            os.path.getmtime(_SO) >= os.path.getmtime(s) for s in srcs):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("ng", C.c_int),
                ("pitch", C.c_int64), ("x0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dz", C.c_double), ("geom", C.c_int),
                ("bc", C.c_int * 4)]


class Eos(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("K", C.c_double * 8),
                ("G", C.c_double * 8), ("rho_b", C.c_double * 8),
                ("Gth", C.c_double)]


class Metric(C.Structure):
    _fields_ = [("f", C.c_void_p * 17), ("c", C.c_double * 17)]


class C2P(C.Structure):
    _fields_ = [("w_max", C.c_double), ("rho_atm", C.c_double), ("adiabatic", C.c_int)]


class Stage(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("dt", C.c_double), ("g", C.c_double), ("d", C.c_double),
                ("e", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("max_courant", C.c_double), ("Mb", C.c_double),
                ("J", C.c_double), ("n_rescale", C.c_ulonglong),
                ("n_cold", C.c_ulonglong), ("n_atm", C.c_ulonglong),
                ("n_fail", C.c_ulonglong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        d, p, i = C.c_double, C.c_void_p, C.c_int
        sig = {
            "or_eos_press": (d, [p, d, d]),
            "or_eos_eps": (d, [p, d, d]),
            "or_eos_eps_cold": (d, [p, d]),
            "or_eos_press_cold": (d, [p, d]),
            "or_eos_cs2": (d, [p, d, d, d]),
            "or_prim2con_point": (None, [p, p, d, i, p, p]),
            "or_con2prim_point": (C.c_uint, [p, p, d, i, p, p, p, p]),
            "or_c2p_master": (d, [p, d, d, d, d]),
            "or_valencia_flux_point": (None, [p, p, i, p, p]),
            "or_face_flux_point": (None, [p, p, i, i, p, p, p, p]),
            "or_coord_speeds": (None, [p, p, i, p, p, p]),
            "or_tetrad_speeds": (None, [p, p, i, p, p, p]),
            "or_source_point": (None, [p, p, p, d, i, p, p]),
            "or_recon_line": (None, [i, i, p, p, p]),
            "or_lagrange6": (d, [p]),
            "or_deriv6": (d, [p, d]),
            "or_prim2con": (None, [p, p, p, p, p, i]),
            "or_con2prim": (None, [p, p, p, p, p, p, p, p]),
            "or_fill_ghosts": (None, [p, p]),
            "or_reconstruct": (None, [p, i, i, p, p, p]),
            "or_face_flux": (None, [p, i, i, p, p, p, p, p, p]),
            "or_rhs": (None, [p, p, p, p, p, p, p]),
            "or_rk_substep": (i, [p, p, p, i, i, i, p, p, p, p, p, p, p, p, p, p, p]),
            "or_rk_substep_reg": (i, [p, p, p, i, i, i, p, p, p, p, p, p, p, p, p, p, p, p, i, i, d,
                                      p, p]),
            "or_fmr_prolong": (None, [p, p, p, p, i, d, d, d, d, p, p, p, i, p, p]),
            "or_fmr_restrict": (None, [p, p, p, p]),
            "or_fmr_reflux": (None, [p, p, p, p, p]),
            "or_riemann_solve": (i, [d, d, d, d, d, d, d, p]),
            "or_riemann_sample": (None, [d, p, d, p, p, p]),
            "or_riemann_cellavg": (i, [d, d, d, d, d, d, d, d, d, i, p, i, p, p, p]),
            "or_mlp_forward": (None, [p, i, p, p]),
            "or_mlp_loss_grad": (d, [p, i, p, p, p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


# ---------------------------------------------------------------- marshalling

def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def make_grid(g):
    s = Grid()
    s.nx, s.nz, s.ng, s.pitch = g["nx"], g["nz"], g["ng"], g["pitch"]
    s.x0, s.z0, s.dx, s.dz = g["x0"], g["z0"], g["dx"], g["dz"]
    s.geom = 0 if g["geom"] == "cyl" else 1
    for k in range(4):
        s.bc[k] = BC_NAMES[g["bc"][k]]
    return s


def make_eos(e):
    s = Eos()
    s.kind = 0 if e["kind"] == "ideal" else 1
    K, G = list(e["K"]), list(e["G"])
    s.n = len(K)
    for k in range(len(K)):
        s.K[k], s.G[k] = K[k], G[k]
    for k, r in enumerate(e.get("rho_b", [])):
        s.rho_b[k] = r
    s.Gth = e["Gth"]
    return s


def make_metric(m, keep):
    """m: dict name -> array or float.  keep: list that holds array refs."""
    s = Metric()
    for k, name in enumerate(METRIC_NAMES):
        v = m.get(name, FLAT.get(name, 0.0))
        if isinstance(v, np.ndarray):
            a = _f64(v)
            keep.append(a)
            s.f[k] = a.ctypes.data
            s.c[k] = 0.0
        else:
            s.f[k] = None
            s.c[k] = float(v)
    return s


def metric_point(m):
    """17 metric values at a point from a dict of floats."""
    return np.array([float(m.get(n, FLAT.get(n, 0.0))) for n in METRIC_NAMES])


def make_c2p(c):
    s = C2P()
    s.w_max, s.rho_atm = c["w_max"], c["rho_atm"]
    s.adiabatic = 1 if c.get("adiabatic") else 0
    return s


def _fieldptrs(arr, nf):
    assert arr.dtype == np.float64 and arr.flags["C_CONTIGUOUS"]
    assert arr.shape[0] == nf
    ptrs = (C.c_void_p * nf)()
    for c in range(nf):
        ptrs[c] = arr[c].ctypes.data
    return ptrs


# ---------------------------------------------------------------- pointwise

def eos_press(eos, rho, eps):
    return lib().or_eos_press(C.byref(make_eos(eos)), rho, eps)


def eos_eps(eos, rho, P):
    return lib().or_eos_eps(C.byref(make_eos(eos)), rho, P)


def eos_cs2(eos, rho, eps, P):
    return lib().or_eos_cs2(C.byref(make_eos(eos)), rho, eps, P)


def eos_eps_cold(eos, rho):
    return lib().or_eos_eps_cold(C.byref(make_eos(eos)), rho)


def eos_press_cold(eos, rho):
    return lib().or_eos_press_cold(C.byref(make_eos(eos)), rho)


def prim2con_point(eos, g, x, geom, p):
    g, p = _f64(g), _f64(p)
    q = np.zeros(5)
    lib().or_prim2con_point(C.byref(make_eos(eos)), _ptr(g), x,
                            0 if geom == "cyl" else 1, _ptr(p), _ptr(q))
    return q


def con2prim_point(eos, g, x, geom, c2p, q):
    g = _f64(g)
    q = np.array(q, dtype=np.float64)
    p = np.zeros(6)
    z = np.zeros(1)
    f = lib().or_con2prim_point(C.byref(make_eos(eos)), _ptr(g), x,
                                0 if geom == "cyl" else 1,
                                C.byref(make_c2p(c2p)), _ptr(q), _ptr(p), _ptr(z))
    return p, q, int(f), float(z[0])


def c2p_master(eos, D, qq, r, z):
    return lib().or_c2p_master(C.byref(make_eos(eos)), D, qq, r, z)


def valencia_flux_point(eos, g, dirn, p):
    g, p = _f64(g), _f64(p)
    F = np.zeros(5)
    lib().or_valencia_flux_point(C.byref(make_eos(eos)), _ptr(g), dirn, _ptr(p), _ptr(F))
    return F


def face_flux_point(eos, g, dirn, riemann, pL, pR):
    g, pL, pR = _f64(g), _f64(pL), _f64(pR)
    F = np.zeros(5)
    sp = np.zeros(1)
    lib().or_face_flux_point(C.byref(make_eos(eos)), _ptr(g), dirn, RIEMANN[riemann],
                             _ptr(pL), _ptr(pR), _ptr(F), _ptr(sp))
    return F, float(sp[0])


def signal_speeds(eos, g, dirn, p, frame="coord"):
    """(lambda-, lambda+) of state p at a face of direction dirn as
    coordinate speeds: frame "coord" from the 3+1 characteristic formula
    (TVDLF), "tetrad" from the face tetrad frame (HLLC)."""
    g, p = _f64(g), _f64(p)
    lm, lp = C.c_double(), C.c_double()
    fn = lib().or_coord_speeds if frame == "coord" else lib().or_tetrad_speeds
    fn(C.byref(make_eos(eos)), _ptr(g), dirn, _ptr(p), C.byref(lm), C.byref(lp))
    return lm.value, lp.value


def source_point(eos, g, dg, x, geom, p):
    g, dg, p = _f64(g), _f64(dg), _f64(p)
    s = np.zeros(5)
    lib().or_source_point(C.byref(make_eos(eos)), _ptr(g), _ptr(dg), x,
                          0 if geom == "cyl" else 1, _ptr(p), _ptr(s))
    return s


def recon_line(recon, a):
    a = _f64(a)
    n = a.size
    aL = np.zeros(max(n - 5, 0))
    aR = np.zeros(max(n - 5, 0))
    lib().or_recon_line(RECON[recon], n, _ptr(a), _ptr(aL), _ptr(aR))
    return aL, aR


def lagrange6(a):
    a = _f64(a)
    return lib().or_lagrange6(_ptr(a))


def deriv6(a, h):
    a = _f64(a)
    return lib().or_deriv6(_ptr(a), h)


# ---------------------------------------------------------------- grid level

def prim2con(grid, eos, metric, p, with_ghosts=False):
    keep = []
    q = np.zeros((5,) + p.shape[1:])
    lib().or_prim2con(C.byref(make_grid(grid)), C.byref(make_eos(eos)),
                      C.byref(make_metric(metric, keep)), _fieldptrs(p, 6),
                      _fieldptrs(q, 5), 1 if with_ghosts else 0)
    return q


def con2prim(grid, eos, metric, c2p, q):
    """Returns (p, q_corrected, flags, diag).  q is not modified."""
    keep = []
    q = q.copy()
    p = np.zeros((6,) + q.shape[1:])
    flags = np.zeros(q.shape[1:], dtype=np.uint8)
    d = Diag()
    lib().or_con2prim(C.byref(make_grid(grid)), C.byref(make_eos(eos)),
                      C.byref(make_metric(metric, keep)), C.byref(make_c2p(c2p)),
                      _fieldptrs(q, 5), _fieldptrs(p, 6), _ptr(flags), C.byref(d))
    return p, q, flags, d.as_dict()


def fill_ghosts(grid, p):
    p = p.copy()
    lib().or_fill_ghosts(C.byref(make_grid(grid)), _fieldptrs(p, 6))
    return p


def face_shape(grid, dirn):
    nx, nz = grid["nx"], grid["nz"]
    return (nz, nx + 1) if dirn == 0 else (nz + 1, nx)


def reconstruct(grid, dirn, recon, p):
    shp = face_shape(grid, dirn)
    pL = np.zeros((6,) + shp)
    pR = np.zeros((6,) + shp)
    lib().or_reconstruct(C.byref(make_grid(grid)), dirn, RECON[recon],
                         _fieldptrs(p, 6), _fieldptrs(pL, 6), _fieldptrs(pR, 6))
    return pL, pR


def face_flux(grid, dirn, riemann, eos, metric, pL, pR):
    keep = []
    F = np.zeros((5,) + pL.shape[1:])
    sp = np.zeros(1)
    lib().or_face_flux(C.byref(make_grid(grid)), dirn, RIEMANN[riemann],
                       C.byref(make_eos(eos)), C.byref(make_metric(metric, keep)),
                       _fieldptrs(_f64(pL), 6), _fieldptrs(_f64(pR), 6),
                       _fieldptrs(F, 5), _ptr(sp))
    return F, float(sp[0])


def rhs(grid, eos, metric, p, Fx, Fz):
    keep = []
    L = np.zeros((5,) + p.shape[1:])
    lib().or_rhs(C.byref(make_grid(grid)), C.byref(make_eos(eos)),
                 C.byref(make_metric(metric, keep)), _fieldptrs(p, 6),
                 _fieldptrs(_f64(Fx), 5), _fieldptrs(_f64(Fz), 5), _fieldptrs(L, 5))
    return L


SSPRK3 = [dict(a=0.0, b=1.0, c=1.0), dict(a=0.75, b=0.25, c=0.25),
          dict(a=1.0 / 3.0, b=2.0 / 3.0, c=2.0 / 3.0)]


def rk_substep(grid, eos, metric, opts, stage, qn, qs, acc_in=None, want_acc=False, reg=None,
               want_faces=False):
    """One substep.  Returns dict(qout, qs (corrected), p, flags, diag,
    flux_reg, acc, Fx, Fz).  Inputs are not modified.  reg: optional (array,
    reg_j, reg_k, weight): the refinement-boundary register (5 x (reg_k +
    reg_j) float64, updated in place) gets weight dt F added on the face
    set {x faces j = reg_j, k < reg_k} + {z faces k = reg_k, j < reg_j}.
    want_faces: Fx (5, nz, nx + 1) and Fz (5, nz + 1, nx), every face flux."""
    keep = []
    qs = qs.copy()
    qout = np.zeros_like(qs)
    p = np.zeros((6,) + qs.shape[1:])
    flags = np.zeros(qs.shape[1:], dtype=np.uint8)
    nb = 2 * grid["nz"] + 2 * grid["nx"]
    freg = np.zeros(5 * nb)
    d = Diag()
    st = Stage()
    st.a, st.b, st.c, st.dt = stage["a"], stage["b"], stage["c"], stage["dt"]
    st.g, st.d, st.e = stage.get("g", 0.0), stage.get("d", 0.0), stage.get("e", 0.0)
    acc_out = np.zeros_like(qs) if want_acc else None
    qn_ptr = _fieldptrs(qn, 5) if qn is not None else None
    if reg is not None:
        assert reg[0].dtype == np.float64 and reg[0].flags.c_contiguous
    nx, nz = grid["nx"], grid["nz"]
    fx = np.zeros((5, nz, nx + 1)) if want_faces else None
    fz = np.zeros((5, nz + 1, nx)) if want_faces else None
    lib().or_rk_substep_reg(
        C.byref(make_grid(grid)), C.byref(make_eos(eos)),
        C.byref(make_metric(metric, keep)), RECON[opts.get("recon", "ppm")],
        RIEMANN[opts.get("riemann", "hllc")], FACE_EPS[opts.get("face_eps", "recon")],
        C.byref(make_c2p(opts["c2p"])),
        C.byref(st), qn_ptr if qn is not None else _fieldptrs(qs, 5),
        _fieldptrs(qs, 5), _fieldptrs(qout, 5), _fieldptrs(p, 6),
        _fieldptrs(acc_in, 5) if acc_in is not None else None,
        _fieldptrs(acc_out, 5) if acc_out is not None else None,
        _ptr(freg), _ptr(flags), C.byref(d),
        _ptr(reg[0]) if reg is not None else None,
        reg[1] if reg is not None else 0, reg[2] if reg is not None else 0,
        float(reg[3]) if reg is not None else 0.0,
        _fieldptrs(fx, 5) if want_faces else None, _fieldptrs(fz, 5) if want_faces else None)
    return dict(qout=qout, qs=qs, p=p, flags=flags, diag=d.as_dict(),
                flux_reg=freg.reshape(5, nb), acc=acc_out, Fx=fx, Fz=fz)


# ---------------------------------------------------------------- refinement

def fmr_prolong(pgrid, slices, times, t, cgrid, eos, cmetric, p_child, q_child, nbuf=0):
    """Fill the child's EXTERNAL ghost cells (p_child 6 and q_child 5 cell
    arrays, updated in place) from the parent's primitive slices (a list of
    1-3 arrays, oldest first, with their times) at time t; with nbuf > 0
    also the nbuf interior rows/columns next to each EXTERNAL side."""
    keep = []
    ns = len(slices)
    old = slices[0] if ns == 3 else None
    cur = slices[-2] if ns >= 2 else slices[0]
    new = slices[-1] if ns >= 2 else None
    t_old = times[0] if ns == 3 else 0.0
    t_cur = times[-2] if ns >= 2 else times[0]
    t_new = times[-1] if ns >= 2 else 0.0
    lib().or_fmr_prolong(C.byref(make_grid(pgrid)), _fieldptrs(old, 6) if old is not None else None,
                         _fieldptrs(cur, 6), _fieldptrs(new, 6) if new is not None else None, ns,
                         t_old, t_cur, t_new, t, C.byref(make_grid(cgrid)), C.byref(make_eos(eos)),
                         C.byref(make_metric(cmetric, keep)), int(nbuf), _fieldptrs(p_child, 6),
                         _fieldptrs(q_child, 5))


def fmr_restrict(pgrid, q_parent, cgrid, q_child):
    """q_parent (updated in place) over the child's footprint."""
    lib().or_fmr_restrict(C.byref(make_grid(pgrid)), _fieldptrs(q_parent, 5),
                          C.byref(make_grid(cgrid)), _fieldptrs(q_child, 5))


def fmr_reflux(pgrid, q_parent, preg, cgrid, creg):
    """Flux correction of the parent cells next to the child (in place)."""
    preg, creg = _f64(preg), _f64(creg)
    lib().or_fmr_reflux(C.byref(make_grid(pgrid)), _fieldptrs(q_parent, 5), _ptr(preg),
                        C.byref(make_grid(cgrid)), _ptr(creg))


class FmrDriver:
    """Berger-Oliger driver of the oracle (Sec. II.E): the same schedule as
    the library's (SSP-RK3 per level, levels l <= l_fix take the parent's
    step and finer ones half of it, restriction, flux correction and
    recovery of the parent after its child's steps), with every operation
    done by the oracle functions above.  levels: list of dict(grid, metric,
    q, nbuf=0) with numpy cell arrays (q is copied).

    Two schedules for a child's boundary, per level (nbuf):
    - nbuf = 0, the halo schedule: the 3 ghost cells beyond each EXTERNAL
      side are prolonged from the parent's slices before every stage, at
      the time of the stage's input state;
    - nbuf > 0, the buffer schedule of Sec. II.E (the paper's (4+4) with
      nbuf = 4): the level's grid holds nbuf cells beyond its own cells on
      each EXTERNAL side.  Before the first stage the buffer and the ghost
      cells beyond it are prolonged at t; the first two stages evolve own
      cells and buffer alike, the second after the ghost cells are
      prolonged at t + dt; the last stage updates the own cells only,
      reading the buffer as the second stage left it (the paper's RK4
      mapping, all stages but the last on the wider domain, taken to
      SSP-RK3 as a reading).  Restriction, registers and flux correction
      concern the own cells.
    """

    A = (0.0, 0.75, 1.0 / 3.0)
    B = (1.0, 0.25, 2.0 / 3.0)
    T = (0.0, 1.0, 0.5)          # stage times in units of dt
    W = (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0)   # weights of the stage fluxes in the step

    def __init__(self, levels, eos, opts, l_fix=0, t0=0.0):
        self.lev = [dict(grid=d["grid"], metric=d["metric"], q=np.array(d["q"], dtype=np.float64),
                         nbuf=int(d.get("nbuf", 0))) for d in levels]
        # the last stage reads the buffer as ghost cells: it must be at least
        # as wide as the ghost layers
        assert self.lev[0]["nbuf"] == 0
        assert all(L["nbuf"] == 0 or L["nbuf"] >= L["grid"]["ng"] for L in self.lev)
        self.eos, self.opts, self.l_fix, self.t = eos, opts, l_fix, t0
        n = len(self.lev)
        self.slices = [[] for _ in range(n)]
        for l, L in enumerate(self.lev):
            own = self.own(l)
            L["reg_bnd"] = np.zeros(5 * (own["nx"] + own["nz"])) if l > 0 else None
            if l + 1 < n:
                co = self.own(l + 1)
                L["reg_int"] = np.zeros(5 * (co["nx"] // 2 + co["nz"] // 2))
                self._push(l, t0)
            else:
                L["reg_int"] = None

    def own(self, l):
        """Level l's grid without its buffer (same arrays and pitch)."""
        g, b = self.lev[l]["grid"], self.lev[l]["nbuf"]
        return dict(g, nx=g["nx"] - b, nz=g["nz"] - b)

    def _recover(self, l):
        L = self.lev[l]
        p, q, _, _ = con2prim(L["grid"], self.eos, L["metric"], self.opts["c2p"], L["q"])
        L["q"] = q
        return p

    def _push(self, l, t):
        self.slices[l].append((t, self._recover(l)))
        self.slices[l] = self.slices[l][-3:]

    def _step(self, l, t, dt):
        n = len(self.lev)
        L = self.lev[l]
        g = L["grid"]
        own = self.own(l)
        nb = L["nbuf"]
        has_child, has_parent = l + 1 < n, l > 0
        if has_child:
            co = self.own(l + 1)
            J, K = co["nx"] // 2, co["nz"] // 2
            L["reg_int"][:] = 0.0
        bufs = {"q": L["q"], "q1": np.zeros_like(L["q"]), "q2": np.zeros_like(L["q"])}
        order = [("q", "q", "q1"), ("q", "q1", "q2"), ("q", "q2", "q")]
        for s in range(3):
            qn_name, qs_name, qo_name = order[s]
            last_on_own = nb > 0 and s == 2
            gs = own if last_on_own else g
            if has_parent and not last_on_own:
                P = self.lev[l - 1]
                ts = [x[0] for x in self.slices[l - 1]]
                sl = [x[1] for x in self.slices[l - 1]]
                p_scratch = np.zeros((6,) + L["q"].shape[1:])
                fmr_prolong(P["grid"], sl, ts, t + self.T[s] * dt, g, self.eos, L["metric"], p_scratch,
                            bufs[qs_name], nbuf=nb if s == 0 else 0)
            st = dict(a=self.A[s], b=self.B[s], c=self.B[s], dt=dt)
            reg = (L["reg_int"], J, K, self.W[s]) if has_child else None
            r = rk_substep(gs, self.eos, L["metric"], self.opts, st, bufs[qn_name], bufs[qs_name], reg=reg,
                           want_faces=has_parent and nb > 0)
            bufs[qs_name] = r["qs"]
            if qs_name == "q":
                bufs["q"] = r["qs"]
            if has_parent:
                w = self.W[s] * dt
                onx, onz = own["nx"], own["nz"]
                rb = L["reg_bnd"].reshape(5, onx + onz)
                if nb == 0:
                    fr = r["flux_reg"]
                    rb[:, :onz] += w * fr[:, onz:2 * onz]
                    rb[:, onz:] += w * fr[:, 2 * onz + onx:]
                else:
                    rb[:, :onz] += w * r["Fx"][:, :onz, onx]
                    rb[:, onz:] += w * r["Fz"][:, onz, :onx]
            out = np.array(bufs[qo_name]) if qo_name != "q" else bufs["q"]
            I = (slice(None), slice(gs["ng"], gs["ng"] + gs["nz"]), slice(gs["ng"], gs["ng"] + gs["nx"]))
            out[I] = r["qout"][I]
            bufs[qo_name] = out
        L["q"] = bufs["q"]
        if not has_child:
            return
        self._push(l, t + dt)
        nsub = 1 if l + 1 <= self.l_fix else 2
        for i in range(nsub):
            self._step(l + 1, t + i * (dt / nsub), dt / nsub)
        C_ = self.lev[l + 1]
        fmr_restrict(g, L["q"], co, C_["q"])
        fmr_reflux(g, L["q"], L["reg_int"], co, C_["reg_bnd"])
        C_["reg_bnd"][:] = 0.0
        self.slices[l][-1] = (t + dt, self._recover(l))

    def step(self, dt0):
        self._step(0, self.t, dt0)
        self.t += dt0


# ---------------------------------------------------------------- exact Riemann

def riemann_solve(gam, L, R):
    sol = np.zeros(16)
    rc = lib().or_riemann_solve(gam, L[0], L[1], L[2], R[0], R[1], R[2], _ptr(sol))
    if rc:
        raise ValueError("Riemann problem produces vacuum")
    return sol


def riemann_sample(gam, sol, xi):
    r, p, v = C.c_double(), C.c_double(), C.c_double()
    lib().or_riemann_sample(gam, _ptr(_f64(sol)), xi, C.byref(r), C.byref(p), C.byref(v))
    return r.value, p.value, v.value


def riemann_cellavg(gam, L, R, xint, t, xface, nsub=64):
    xface = _f64(xface)
    n = xface.size - 1
    rho, p, v = np.zeros(n), np.zeros(n), np.zeros(n)
    rc = lib().or_riemann_cellavg(gam, L[0], L[1], L[2], R[0], R[1], R[2], xint, t,
                                  n, _ptr(xface), nsub, _ptr(rho), _ptr(p), _ptr(v))
    if rc:
        raise ValueError("Riemann problem produces vacuum")
    return rho, p, v


# ---------------------------------------------------------------- MLP

def mlp_forward(params, X):
    params, X = _f64(params), _f64(X)
    y = np.zeros(X.shape[0])
    lib().or_mlp_forward(_ptr(params), X.shape[0], _ptr(X), _ptr(y))
    return y


def mlp_loss_grad(params, X, t):
    params, X, t = _f64(params), _f64(X), _f64(t)
    g = np.zeros(NPARAM_MLP)
    loss = lib().or_mlp_loss_grad(_ptr(params), X.shape[0], _ptr(X), _ptr(t), _ptr(g))
    return loss, g
