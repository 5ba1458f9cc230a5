"""Seeded synthetic inputs for the GRHD substep (shared by tests and bench).

This module holds no arithmetic of the hydro method itself: it only lays out
grids, draws seeded random states, integrates the TOV equations for the
initial star and the Cowling metric, and writes PRIMITIVE variables and
metric fields.  The conversion to conserved variables is done separately by
each side (the oracle's prim2con, the GPU's grhd_prim2con).

Workload recipes (all synthetic; the paper's own runs use external initial
data that is not available):
  * Riemann problems on a flat metric, ideal gas G = 5/3, x in [0, 1],
    interface at x = 0.5; states rho ~ logU[0.1, 10], p ~ logU[1e-3, 20],
    v_x ~ U[-0.5, 0.5], v_y = v_z = 0, redrawn when the exact solution
    contains vacuum (closed-form test below).
  * TOV polytrope K = 100, G = 2 (G = c = Msun = 1), rho_c = 1.28e-3, mapped
    onto a cylindrical (varpi, z) grid in isotropic coordinates; Cowling
    metric alpha(r), W = psi^-2; beta = 0, conformal metric = identity,
    K_ij = 0; atmosphere rho_atm = 1e-10; density perturbed by 1e-4 xi,
    xi ~ U[-1, 1] iid per cell; P = K rho^G, u_i = 0.
  * A differentially rotating field for the standalone recovery workload:
    rho ~ logU[1e-10, 1e-2], eps = 100 rho (1 + theta), theta ~ U[0, 1],
    Lorentz factor w(varpi) = 1 + 9 (varpi / 20)(1 + 0.05 xi) clipped to
    [1, 10], u_y = w v, u_x = u_z = 0; flat metric.
"""
import math

import numpy as np

NG = 3


def make_grid(nx, nz, x0, z0, dx, dz, geom, bc, ng=NG, pad=64):
    """Cell-centred grid with ng ghosts; the row pitch is padded to a
    multiple of `pad` doubles."""
    row = nx + 2 * ng
    pitch = ((row + pad - 1) // pad) * pad
    return dict(nx=nx, nz=nz, ng=ng, pitch=pitch, x0=float(x0), z0=float(z0),
                dx=float(dx), dz=float(dz), geom=geom, bc=tuple(bc))


def cell_coords(grid):
    """x and z of every stored cell (ghosts included), shape (rows, pitch);
    padding columns get the coordinate of a far-right ghost."""
    ng, pitch = grid["ng"], grid["pitch"]
    rows = grid["nz"] + 2 * ng
    j = np.arange(pitch) - ng
    k = np.arange(rows) - ng
    x = grid["x0"] + (j + 0.5) * grid["dx"]
    z = grid["z0"] + (k + 0.5) * grid["dz"]
    X, Z = np.meshgrid(x, z)
    return X, Z


def interior(grid, a):
    """View of the interior cells of a field array (..., rows, pitch)."""
    ng = grid["ng"]
    return a[..., ng:ng + grid["nz"], ng:ng + grid["nx"]]


def empty_fields(grid, nf):
    return np.zeros((nf, grid["nz"] + 2 * grid["ng"], grid["pitch"]))


# ------------------------------------------------------------------ EOS specs

def ideal_eos(gamma, K=1.0):
    """Gamma-law gas P = (G-1) rho eps; K is only used for the atmosphere."""
    return dict(kind="ideal", K=[K], G=[gamma], rho_b=[], Gth=gamma)


# ------------------------------------------------------------------ Riemann

def _rapid(v):
    return 0.5 * math.log((1 + v) / (1 - v))


def riemann_has_vacuum(gam, L, R):
    """Closed-form admissibility test: vacuum forms when the two
    rarefactions expanded to zero pressure do not meet."""
    def cs(rho, p):
        h = 1 + gam / (gam - 1) * p / rho
        return math.sqrt(gam * p / (rho * h))

    def Fc(c):
        s = math.sqrt(gam - 1)
        return math.log((s + c) / (s - c)) / s
    v0L = math.tanh(_rapid(L[2]) + Fc(cs(L[0], L[1])))
    v0R = math.tanh(_rapid(R[2]) - Fc(cs(R[0], R[1])))
    return v0L <= v0R


def riemann_states(seed, n=1, gam=5.0 / 3.0):
    """n seeded (L, R) states (rho, p, v_x), vacuum-free."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        rho = np.exp(rng.uniform(math.log(0.1), math.log(10.0), 2))
        p = np.exp(rng.uniform(math.log(1e-3), math.log(20.0), 2))
        v = rng.uniform(-0.5, 0.5, 2)
        L = (float(rho[0]), float(p[0]), float(v[0]))
        R = (float(rho[1]), float(p[1]), float(v[1]))
        if not riemann_has_vacuum(gam, L, R):
            out.append((L, R))
    return out


PAPER_SHOCK_TUBE = ((10.0, 40.0 / 3.0, 0.0), (1.0, 0.0, 0.0))


def riemann_grid(nx, nz=8, length=1.0, geom="cart", direction="x"):
    d = length / nx
    if direction == "x":
        return make_grid(nx, nz, 0.0, 0.0, d, d, geom,
                         ("outflow", "outflow", "periodic", "periodic"))
    return make_grid(nz, nx, 0.0, 0.0, d, d, geom,
                     ("periodic", "periodic", "outflow", "outflow"))


def riemann_prims(grid, L, R, gam=5.0 / 3.0, xint=0.5, direction="x"):
    """Primitive arrays (rho, u_x, u_y, u_z, P, eps) of a flat-space
    Riemann problem (covariant u_i = w v_i in flat space)."""
    X, Z = cell_coords(grid)
    s = X if direction == "x" else Z
    left = s < xint
    p = empty_fields(grid, 6)
    for (st, mask) in ((L, left), (R, ~left)):
        rho, pr, v = st
        w = 1.0 / math.sqrt(1.0 - v * v)
        p[0][mask] = rho
        p[1 if direction == "x" else 3][mask] = w * v
        p[4][mask] = pr
        p[5][mask] = pr / ((gam - 1.0) * rho)
    return p


# ------------------------------------------------------------------ TOV star

MSUN_KM = 1.476625


def tov_solve(K=100.0, G=2.0, rho_c=1.28e-3, npts=20001):
    """Spherical polytropic star: integrate the TOV equations in
    Schwarzschild r, then the isotropic radius, lapse and baryon mass.
    Returns a dict of tabulated profiles and the global numbers."""
    from scipy.integrate import solve_ivp

    # the density is integrated instead of the pressure (dP = G K rho^(G-1)
    # drho): for G = 2 it falls linearly at the surface, which keeps the
    # right-hand side smooth up to the surface.
    def rhs(r, y):
        m, rho, phi, ell, mb = y
        rho = max(rho, 0.0)
        P = K * rho ** G
        e = rho + P / (G - 1.0)
        f = 1.0 - 2.0 * m / r
        dm = 4 * math.pi * r * r * e
        dphi = (m + 4 * math.pi * r ** 3 * P) / (r * r * f)
        dP = -(e + P) * dphi
        drho = dP / (G * K * rho ** (G - 1.0)) if rho > 0 else 0.0
        dell = (1.0 / math.sqrt(f) - 1.0) / r
        dmb = 4 * math.pi * r * r * rho / math.sqrt(f)
        return [dm, drho, dphi, dell, dmb]

    Pc = K * rho_c ** G
    ec = rho_c + Pc / (G - 1.0)
    r0 = 1e-6
    m0 = 4.0 / 3.0 * math.pi * r0 ** 3 * ec
    y0 = [m0, rho_c, 0.0, 0.0, 4.0 / 3.0 * math.pi * r0 ** 3 * rho_c]

    def surf(r, y):
        return y[1]
    surf.terminal = True
    surf.direction = -1
    sol = solve_ivp(rhs, [r0, 200.0], y0, method="DOP853", rtol=1e-12,
                    atol=1e-16, events=surf, dense_output=True)
    R = float(sol.t_events[0][0])
    yR = sol.sol(R)
    M, phiR, ellR, Mb = float(yR[0]), float(yR[2]), float(yR[3]), float(yR[4])
    rbarR = 0.5 * (R - M + math.sqrt(R * R - 2 * M * R))
    r = np.linspace(r0, R, npts)
    Y = sol.sol(r)
    phi_shift = 0.5 * math.log(1.0 - 2.0 * M / R) - phiR
    ell_shift = math.log(rbarR / R) - ellR
    ell = Y[3] + ell_shift
    rbar = r * np.exp(ell)
    rho = np.maximum(Y[1], 0.0)
    alp = np.exp(Y[2] + phi_shift)
    W = np.exp(ell)          # W = psi^-2 = rbar / r
    return dict(K=K, G=G, rho_c=rho_c, R=R, M=M, Mb=Mb, Rbar=rbarR,
                rbar=rbar, rho=rho, alp=alp, W=W)


def tov_fields(tov, rbar):
    """rho, alpha, W at isotropic radius rbar (array); exterior is the
    isotropic Schwarzschild solution and rho = 0."""
    from scipy.interpolate import CubicSpline
    key = "_splines"
    if key not in tov:
        xs = np.concatenate(([0.0], tov["rbar"]))
        tov[key] = tuple(CubicSpline(xs, np.concatenate(([v[0]], v)))
                         for v in (tov["rho"], tov["alp"], tov["W"]))
    srho, salp, sW = tov[key]
    rb = np.asarray(rbar, dtype=np.float64)
    inside = rb < tov["Rbar"]
    M = tov["M"]
    rs = np.maximum(rb, 1e-300)
    psi = 1.0 + M / (2.0 * rs)
    alp_out = (1.0 - M / (2.0 * rs)) / psi
    W_out = 1.0 / (psi * psi)
    rho = np.where(inside, np.maximum(srho(np.minimum(rb, tov["Rbar"])), 0.0), 0.0)
    alp = np.where(inside, salp(np.minimum(rb, tov["Rbar"])), alp_out)
    W = np.where(inside, sW(np.minimum(rb, tov["Rbar"])), W_out)
    return rho, alp, W


def star_grid(n, extent=20.0):
    d = extent / n
    return make_grid(n, n, 0.0, 0.0, d, d, "cyl",
                     ("axis", "outflow", "reflect", "outflow"))


def star_problem(grid, seed, tov=None, rho_atm=1e-10, pert=1e-4, vel=0.0):
    """(prims, metric dict, eos) for the perturbed TOV star on `grid`.
    vel > 0 adds iid velocities u_i ~ vel U[-1, 1] inside the star (test
    states with active limiters and non-trivial recovery)."""
    if tov is None:
        tov = tov_solve()
    K, G = tov["K"], tov["G"]
    X, Z = cell_coords(grid)
    rbar = np.sqrt(X * X + Z * Z)
    rho0, alp, W = tov_fields(tov, rbar)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=rho0.shape)
    rho = rho0 * (1.0 + pert * xi)
    rho = np.maximum(rho, rho_atm)
    p = empty_fields(grid, 6)
    p[0] = rho
    p[4] = K * rho ** G
    p[5] = p[4] / ((G - 1.0) * rho)
    if vel > 0.0:
        inside = rho0 > 0.0
        for c in (1, 2, 3):
            p[c] = np.where(inside, vel * rng.uniform(-1.0, 1.0, size=rho0.shape), 0.0)
    metric = dict(alp=np.ascontiguousarray(alp), W=np.ascontiguousarray(W))
    eos = ideal_eos(G, K=K)
    return p, metric, eos


def fmr_levels(nlev=6, n=256, finest_extent=20.0, nbuf=0):
    """Nested levels anchored at the origin, 2:1 refinement; level l covers
    [0, finest_extent * 2^(nlev-1-l)]^2 with its own n x n cells; levels
    with a parent hold nbuf buffer cells beyond them on the high sides."""
    out = []
    for l in range(nlev):
        g = star_grid(n, finest_extent * 2 ** (nlev - 1 - l))
        if l > 0 and nbuf:
            g = make_grid(n + nbuf, n + nbuf, g["x0"], g["z0"], g["dx"], g["dz"], g["geom"], g["bc"])
        out.append(g)
    return out


def fmr_grids(nlev, n, extent, geom="cart", outer="reflect", nbuf=0):
    """Nested 2:1 levels anchored at the lower faces: level 0 covers
    [0, extent]^2 with n x n cells, every finer level n x n own cells over
    its parent's lower-left quarter (plus nbuf buffer cells beyond them on
    the high sides) with EXTERNAL high sides; level 0's high sides are
    `outer`; low sides: axis (cyl) or reflect (cart) in x, reflect in z."""
    lo_x = "axis" if geom == "cyl" else "reflect"
    out = []
    for l in range(nlev):
        d = extent / n / 2 ** l
        hi = outer if l == 0 else "external"
        m = n if l == 0 else n + nbuf
        out.append(make_grid(m, m, 0.0, 0.0, d, d, geom, (lo_x, hi, "reflect", hi)))
    return out


def blast_state(grid, center, width, seed, gamma=5.0 / 3.0, vamp=0.05):
    """Smooth over-dense, over-pressured Gaussian bump at `center` on a
    uniform background, with a small seeded velocity field."""
    rng = np.random.default_rng(seed)
    X, Z = cell_coords(grid)
    r2 = ((X - center[0]) ** 2 + (Z - center[1]) ** 2) / width ** 2
    bump = np.exp(-r2)
    ph = rng.uniform(0, 2 * math.pi, 3)
    p = empty_fields(grid, 6)
    p[0] = 1.0 + 0.5 * bump
    p[1] = vamp * bump * np.sin(X / width + ph[0])
    p[2] = 0.5 * vamp * bump * np.cos(Z / width + ph[1])
    p[3] = vamp * bump * np.sin((X + Z) / width + ph[2])
    p[4] = 0.1 + 1.0 * bump
    p[5] = p[4] / ((gamma - 1.0) * p[0])
    return p


def trumpet_r_of_R(R, M=1.0):
    """Isotropic radius of the maximal trumpet slice of Schwarzschild as a
    function of the areal radius R >= 3M/2 (closed form)."""
    R = np.asarray(R, dtype=np.float64)
    a = (2.0 * R + M + np.sqrt(4.0 * R * R + 4.0 * M * R + 3.0 * M * M)) / 4.0
    b = ((4.0 + 3.0 * math.sqrt(2.0)) * (2.0 * R - 3.0 * M)
         / (8.0 * R + 6.0 * M + 3.0 * np.sqrt(8.0 * R * R + 8.0 * M * R + 6.0 * M * M)))
    return a * np.maximum(b, 0.0) ** (1.0 / math.sqrt(2.0))


def trumpet_R_of_r(r, M=1.0):
    """Areal radius at isotropic radius r (inverse of trumpet_r_of_R, by
    bisection to the last bit; r(R) increases monotonically)."""
    r = np.asarray(r, dtype=np.float64)
    lo = np.full(r.shape, 1.5 * M)
    hi = np.maximum(r, 0.0) + 2.0 * M + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        up = trumpet_r_of_R(mid, M) < r
        lo = np.where(up, mid, lo)
        hi = np.where(up, hi, mid)
    return 0.5 * (lo + hi)


def trumpet_metric(grid, M=1.0):
    """The maximal trumpet slice of a Schwarzschild black hole of mass M in
    the cartoon plane y = 0: lapse, shift C x^i / R^3, W = r / R, flat
    conformal metric, K = 0 and K_ij = W^-2 C / R^3 (delta_ij - 3 x^i x^j /
    r^2), C = 3 sqrt(3) M^2 / 4 (every stored cell)."""
    X, Z = cell_coords(grid)
    r = np.sqrt(X * X + Z * Z)
    R = trumpet_R_of_r(r, M)
    C = 3.0 * math.sqrt(3.0) * M * M / 4.0
    c = C / R ** 3
    W = r / R
    iW2 = 1.0 / (W * W)
    out = dict(alp=np.sqrt(1.0 - 2.0 * M / R + C * C / R ** 4), bx=c * X, bz=c * Z, W=W,
               kxx=iW2 * c * (1.0 - 3.0 * X * X / (r * r)), kxz=iW2 * c * (-3.0 * X * Z / (r * r)),
               kyy=iW2 * c, kzz=iW2 * c * (1.0 - 3.0 * Z * Z / (r * r)))
    return {k: np.ascontiguousarray(v) for k, v in out.items()}


def bondi_profile(R, M=1.0, K=1.0, G=4.0 / 3.0, Rc=8.0):
    """Transonic Bondi (Michel) accretion in Schwarzschild areal radius:
    (rho, |u^R|) at R for the polytrope P = K rho^G with the sonic point at
    Rc.  The flux 4 pi R^2 rho |u^R| and the Bernoulli constant
    h^2 (1 - 2M/R + u^2) are those of the sonic point; subsonic branch
    outside Rc, supersonic inside.  Returns (rho, u, mdot)."""
    R = np.asarray(R, dtype=np.float64)
    uc2 = M / (2.0 * Rc)
    cs2c = uc2 / (1.0 - 3.0 * uc2)

    def hK(rho):
        return 1.0 + G / (G - 1.0) * K * rho ** (G - 1.0)
    # sonic density: cs2 = G K rho^(G-1) / h solved for rho in closed form
    x = cs2c / (G - cs2c * G / (G - 1.0))          # K rho^(G-1)
    rhoc = (x / K) ** (1.0 / (G - 1.0))
    uc = math.sqrt(uc2)
    mdot = 4.0 * math.pi * Rc * Rc * rhoc * uc
    B = hK(rhoc) ** 2 * (1.0 - 2.0 * M / Rc + uc2)

    def f(u, RR):
        rho = mdot / (4.0 * math.pi * RR * RR * u)
        return hK(rho) ** 2 * (1.0 - 2.0 * M / RR + u * u) - B
    # f is convex in log u with its minimum at the sonic speed of the
    # radius: bisection on each branch, vectorised over R
    lo_s, hi_s = np.full(R.shape, 1e-12), np.full(R.shape, 1.0)
    # the minimum of f over u (golden section in log u)
    a, b = np.log(lo_s), np.log(hi_s * 0.9999999)
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(200):
        c1 = b - g * (b - a)
        c2 = a + g * (b - a)
        left = f(np.exp(c1), R) < f(np.exp(c2), R)
        b = np.where(left, c2, b)
        a = np.where(left, a, c1)
    umin = np.exp(0.5 * (a + b))
    sub = R > Rc
    lo = np.where(sub, 1e-14, umin)
    hi = np.where(sub, umin, 0.9999999999)
    flo = f(lo, R)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = f(mid, R)
        same = np.sign(fm) == np.sign(flo)
        lo = np.where(same, mid, lo)
        flo = np.where(same, fm, flo)
        hi = np.where(same, hi, mid)
    u = 0.5 * (lo + hi)
    u = np.where(np.abs(R - Rc) < 1e-12, uc, u)
    rho = mdot / (4.0 * math.pi * R * R * u)
    return rho, u, mdot


def bondi_problem(grid, M=1.0, r_in=0.4):
    """(prims, metric, eos, frozen) for the Bondi flow in the maximal trumpet
    slice (every stored cell, so EXTERNAL ghosts carry the solution):
    rho, P = rho^(4/3), eps, and the covariant spatial four-velocity of the
    infalling flow on the trumpet slice; frozen marks the cells with
    r < r_in, which keep their initial state."""
    G, K = 4.0 / 3.0, 1.0
    metric = trumpet_metric(grid, M)
    X, Z = cell_coords(grid)
    r = np.sqrt(X * X + Z * Z)
    R = trumpet_R_of_r(r, M)
    rho, u, _ = bondi_profile(R, M, K, G, 8.0)
    C = 3.0 * math.sqrt(3.0) * M * M / 4.0
    alp = metric["alp"]
    s = np.sqrt(1.0 - 2.0 * M / R + u * u)
    a = C / (R * R * alp)
    # covariant radial component on the trumpet slice (T = t_S + h(R),
    # h' = C / (R^2 (1 - 2M/R) alpha)), written without the horizon's 0/0
    uR = (C * C / R ** 4 - u * u) / (alp * alp * (s * a + u))
    ur = uR * alp * R / r          # dR/dr = alpha R / r
    p = empty_fields(grid, 6)
    p[0] = rho
    p[1] = ur * X / r
    p[3] = ur * Z / r
    p[4] = K * rho ** G
    p[5] = p[4] / ((G - 1.0) * rho)
    return p, metric, ideal_eos(G, K=K), np.ascontiguousarray(r < r_in)


def modified_bondi_problem(grid, M=1.0, r_in=0.4):
    """The Bondi flow with a hot, light bubble (Sec. III.B.3): inside
    r < 3M [1 + 0.05 (cos(80 theta) + 1)] (theta the polar angle from the
    z axis) rho = 0.1 rho_bondi, P = 50 P_bondi, u = 0."""
    p, metric, eos, frozen = bondi_problem(grid, M, r_in)
    X, Z = cell_coords(grid)
    r = np.sqrt(X * X + Z * Z)
    theta = np.arctan2(np.abs(X), Z)
    inside = r < 3.0 * M * (1.0 + 0.05 * (np.cos(80.0 * theta) + 1.0))
    G = 4.0 / 3.0
    p[0] = np.where(inside, 0.1 * p[0], p[0])
    p[4] = np.where(inside, 50.0 * p[4], p[4])
    for c in (1, 2, 3):
        p[c] = np.where(inside, 0.0, p[c])
    p[5] = p[4] / ((G - 1.0) * p[0])
    return p, metric, eos, frozen


def riemann_patch_sizes(seed, npatch=64, lo=128, hi=2048):
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            for _ in range(npatch)]


# ------------------------------------------------------------------ recovery field

def rotating_field(grid, seed):
    """Primitive arrays of the differentially rotating recovery workload."""
    rng = np.random.default_rng(seed)
    X, Z = cell_coords(grid)
    shp = X.shape
    rho = np.exp(rng.uniform(math.log(1e-10), math.log(1e-2), shp))
    theta = rng.uniform(0.0, 1.0, shp)
    eps = 100.0 * rho * (1.0 + theta)
    xi = rng.uniform(-1.0, 1.0, shp)
    w = np.clip(1.0 + 9.0 * (np.abs(X) / 20.0) * (1.0 + 0.05 * xi), 1.0, 10.0)
    v = np.sqrt(1.0 - 1.0 / (w * w))
    p = empty_fields(grid, 6)
    p[0] = rho
    p[2] = w * v
    p[5] = eps
    p[4] = (2.0 - 1.0) * rho * eps   # gamma-law G = 2 pressure of (rho, eps)
    return p


def recovery_samples(seed, n):
    """n primitive states (rho, u_x, u_y, u_z, P, eps) drawn from the same
    distributions as the rotating field, flat metric (training inputs)."""
    rng = np.random.default_rng(seed)
    rho = np.exp(rng.uniform(math.log(1e-10), math.log(1e-2), n))
    theta = rng.uniform(0.0, 1.0, n)
    eps = 100.0 * rho * (1.0 + theta)
    w = rng.uniform(1.0, 10.0, n)
    v = np.sqrt(1.0 - 1.0 / (w * w))
    out = np.zeros((n, 6))
    out[:, 0] = rho
    out[:, 2] = w * v
    out[:, 5] = eps
    out[:, 4] = rho * eps
    return out


def star_recovery_samples(seed, n, K=100.0, rho_max=1.5e-3):
    """n primitive states (rho, u_x, u_y, u_z, P, eps) of the kind the star
    holds, flat metric (training inputs of the learned guess for the star):
    rho log-uniform in [1e-10, rho_max], eps = K rho (1 + 0.1 theta) with
    theta ~ U[0, 1] (the Gamma = 2 polytrope plus a small thermal part),
    u_x, u_z ~ N(0, 0.03), u_y = 0."""
    rng = np.random.default_rng(seed)
    rho = np.exp(rng.uniform(math.log(1e-10), math.log(rho_max), n))
    eps = K * rho * (1.0 + 0.1 * rng.uniform(0.0, 1.0, n))
    out = np.zeros((n, 6))
    out[:, 0] = rho
    out[:, 1] = rng.normal(0.0, 0.03, n)
    out[:, 3] = rng.normal(0.0, 0.03, n)
    out[:, 5] = eps
    out[:, 4] = rho * eps
    return out


def general_metric(grid, seed, amp=0.1):
    """Smooth random metric with every field active: lapse, shift, W,
    conformal metric with det = 1 (M / det(M)^(1/3)), extrinsic curvature;
    periodic in both directions of the grid (for Cartesian periodic tests)."""
    rng = np.random.default_rng(seed)
    X, Z = cell_coords(grid)
    Lx = grid["nx"] * grid["dx"]
    Lz = grid["nz"] * grid["dz"]

    def smooth():
        a, b, c, d = rng.uniform(0, 2 * math.pi, 4)
        return (np.sin(2 * math.pi * X / Lx + a) * np.cos(2 * math.pi * Z / Lz + b)
                + 0.5 * np.sin(2 * math.pi * (X / Lx + Z / Lz) + c) + 0.3 * np.cos(4 * math.pi * Z / Lz + d))
    m = {}
    m["alp"] = 0.8 + amp * smooth()
    m["bx"], m["by"], m["bz"] = (amp * smooth() for _ in range(3))
    m["W"] = 0.85 + amp * smooth()
    M = np.zeros(X.shape + (3, 3))
    for i in range(3):
        for j in range(i, 3):
            v = (1.0 if i == j else 0.0) + amp * smooth()
            M[..., i, j] = v
            M[..., j, i] = v
    det = np.linalg.det(M)
    M = M / np.cbrt(det)[..., None, None]
    names = ["gxx", "gxy", "gxz", "gyy", "gyz", "gzz"]
    for n, (i, j) in zip(names, [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        m[n] = np.ascontiguousarray(M[..., i, j])
    for n in ["kxx", "kxy", "kxz", "kyy", "kyz", "kzz"]:
        m[n] = 0.05 * smooth()
    return {k: np.ascontiguousarray(v) for k, v in m.items()}


def smooth_state(grid, seed, gamma=5.0 / 3.0, vamp=0.3):
    """Smooth periodic primitive state (covariant u_i small enough for any
    metric of general_metric)."""
    rng = np.random.default_rng(seed)
    X, Z = cell_coords(grid)
    Lx = grid["nx"] * grid["dx"]
    Lz = grid["nz"] * grid["dz"]
    kx, kz = 2 * math.pi / Lx, 2 * math.pi / Lz
    ph = rng.uniform(0, 2 * math.pi, 6)
    p = empty_fields(grid, 6)
    p[0] = 1.0 + 0.3 * np.sin(kx * X + ph[0]) * np.cos(kz * Z + ph[1])
    p[1] = vamp * np.sin(kx * X + ph[2])
    p[2] = 0.7 * vamp * np.cos(kz * Z + ph[3])
    p[3] = vamp * np.sin(kx * X + kz * Z + ph[4])
    p[4] = 0.5 + 0.2 * np.cos(kx * X - kz * Z + ph[5])
    p[5] = p[4] / ((gamma - 1.0) * p[0])
    return p
