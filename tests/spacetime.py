"""Test-side spacetime algebra, independent of the oracle and of the GPU code.

Everything here is built from the 4-metric g_ab and the stress-energy
tensor T^ab = rho h u^a u^b + P g^ab of a perfect fluid (the paper's
Sec. II.C.1 definitions), with numpy linear algebra, so that the oracle's
3+1 formulas (Valencia flux, tetrad HLLC, source terms) can be checked
against the covariant objects they are derived from.
"""
import numpy as np
from scipy.linalg import expm

NAMES = ["alp", "bx", "by", "bz", "W", "gxx", "gxy", "gxz", "gyy", "gyz",
         "gzz", "kxx", "kxy", "kxz", "kyy", "kyz", "kzz"]
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def sym_from6(v):
    m = np.zeros((3, 3), dtype=np.result_type(v[0], 1.0))
    for (i, j), x in zip(SYM, v):
        m[i, j] = x
        m[j, i] = x
    return m


def six_from_sym(m):
    return np.array([m[i, j] for (i, j) in SYM])


def random_traceless(rng, scale):
    A = rng.normal(size=(3, 3)) * scale
    A = 0.5 * (A + A.T)
    A -= np.trace(A) / 3.0 * np.eye(3)
    return A


def random_point_metric(rng, scale=0.2, shift=0.1, curv=0.1):
    """Metric values at a point: det(gt) = 1 exactly (matrix exponential of a
    traceless symmetric matrix), random lapse, shift, W, K_ij."""
    gt = expm(random_traceless(rng, scale))
    g = np.zeros(17)
    g[0] = rng.uniform(0.6, 1.2)
    g[1:4] = rng.normal(size=3) * shift
    g[4] = rng.uniform(0.7, 1.1)
    g[5:11] = six_from_sym(gt)
    g[11:17] = six_from_sym(sym_from6(rng.normal(size=6) * curv))
    return g


def random_metric_with_derivs(rng, scale=0.2, shift=0.1, curv=0.1):
    """Metric values g[17] and first derivatives dg[3][17] (x, y, z) at a
    point, with det(gt) = 1 along every direction (gt = expm(A0 + s A_d);
    derivative by the complex step, exact to rounding)."""
    A0 = random_traceless(rng, scale)
    g = random_point_metric(rng, scale, shift, curv)
    g[5:11] = six_from_sym(expm(A0))
    dg = np.zeros((3, 17))
    hs = 1e-30
    for d in range(3):
        Ad = random_traceless(rng, scale)
        dgt = np.imag(expm(A0 + 1j * hs * Ad)) / hs
        dg[d, 5:11] = six_from_sym(dgt)
        dg[d, 0] = rng.normal() * 0.1
        dg[d, 1:4] = rng.normal(size=3) * 0.1
        dg[d, 4] = rng.normal() * 0.1
        dg[d, 11:17] = rng.normal(size=6) * 0.05
    return g, dg


def four_metric(g):
    """g_ab from (alpha, beta^i, W, gt_ij): gamma_ij = W^-2 gt_ij."""
    alp, beta, W = g[0], g[1:4], g[4]
    gam = sym_from6(g[5:11]) / W ** 2
    bl = gam @ beta
    G = np.zeros((4, 4), dtype=np.result_type(g[0], 1.0))
    G[0, 0] = -alp ** 2 + bl @ beta
    G[0, 1:] = bl
    G[1:, 0] = bl
    G[1:, 1:] = gam
    return G


def four_velocity_up(g, u_low_spatial):
    """u^a from the covariant spatial components u_i (u_t from u^a u_a = -1)."""
    alp, beta, W = g[0], g[1:4], g[4]
    gam = sym_from6(g[5:11]) / W ** 2
    gi = np.linalg.inv(gam)
    w = np.sqrt(1.0 + u_low_spatial @ gi @ u_low_spatial)
    ut = w / alp
    ui = gi @ u_low_spatial - beta * ut
    return np.concatenate(([ut], ui))


def stress_energy_up(g, prim):
    rho, u, P, eps = prim[0], np.asarray(prim[1:4]), prim[4], prim[5]
    h = 1.0 + eps + P / rho
    G = four_metric(g)
    Gi = np.linalg.inv(G)
    ua = four_velocity_up(g, u)
    return rho * h * np.outer(ua, ua) + P * Gi, ua, G


def sqrt_minus_g(g):
    return g[0] * g[4] ** -3  # alpha * sqrt(gamma), det(gt) = 1


def valencia_flux_covariant(g, prim, n):
    """Densitised coordinate flux in direction n (spatial index 0..2) from
    the covariant definitions: rest-mass current sqrt(-g) rho u^n,
    momentum sqrt(-g) T^n_j, energy sqrt(-g)(alpha^2 T^{0n} ... ) written
    as the flux of E = alpha^2 T^00 : sqrt(gamma) alpha^2 T^{0n}."""
    T, ua, G = stress_energy_up(g, prim)
    sg = sqrt_minus_g(g)
    Tmix = T @ G  # T^a_b
    F = np.zeros(5)
    F[0] = sg * prim[0] * ua[1 + n]
    for j in range(3):
        F[1 + j] = sg * Tmix[1 + n, 1 + j]
    F[4] = sg * g[0] * T[0, 1 + n]
    return F


def conserved_covariant(g, prim):
    """Densitised (D, S_j, E) from the covariant objects:
    D = alpha rho u^t, S_j = -n_a T^a_j = alpha T^0_j, E = alpha^2 T^00."""
    T, ua, G = stress_energy_up(g, prim)
    sq = g[4] ** -3
    Tmix = T @ G
    q = np.zeros(5)
    q[0] = sq * g[0] * prim[0] * ua[0]
    for j in range(3):
        q[1 + j] = sq * g[0] * Tmix[0, 1 + j]
    q[4] = sq * g[0] ** 2 * T[0, 0]
    return q


def four_metric_derivs(g, dg, dt_alp, dt_beta):
    """d_c g_ab for c = t, x, y, z.  Spatial derivatives from dg (chain rule
    through gamma_ij = W^-2 gt_ij, beta_i = gamma_ij beta^j); the time
    derivative of gamma_ij from the ADM relation
    d_t gamma_ij = -2 alpha K_ij + beta^k d_k gamma_ij + gamma_kj d_i beta^k
    + gamma_ik d_j beta^k, with free d_t alpha, d_t beta^i."""
    alp, beta, W = g[0], g[1:4], g[4]
    gt = sym_from6(g[5:11])
    gam = gt / W ** 2
    K = sym_from6(g[11:17])
    dgam = np.zeros((3, 3, 3))
    for d in range(3):
        dgam[d] = sym_from6(dg[d, 5:11]) / W ** 2 - 2.0 * dg[d, 4] * gt / W ** 3
    dbeta = dg[:, 1:4]        # dbeta[d, k] = d_d beta^k
    dalp = dg[:, 0]
    dtgam = -2.0 * alp * K.copy()
    for i in range(3):
        for j in range(3):
            s = 0.0
            for k in range(3):
                s += beta[k] * dgam[k, i, j] + gam[k, j] * dbeta[i, k] + gam[i, k] * dbeta[j, k]
            dtgam[i, j] += s
    dalp4 = np.concatenate(([dt_alp], dalp))
    dbeta4 = np.vstack((dt_beta[None, :], dbeta))
    dgam4 = np.concatenate((dtgam[None], dgam))
    D = np.zeros((4, 4, 4))
    for c in range(4):
        bl = gam @ beta
        dbl = dgam4[c] @ beta + gam @ dbeta4[c]
        D[c, 0, 0] = -2 * alp * dalp4[c] + dbl @ beta + bl @ dbeta4[c]
        D[c, 0, 1:] = dbl
        D[c, 1:, 0] = dbl
        D[c, 1:, 1:] = dgam4[c]
    return D


def christoffel_first_index_up(G, D):
    """Gamma^c_ab = 1/2 g^cd (d_a g_db + d_b g_da - d_d g_ab); D[c,a,b] = d_c g_ab."""
    Gi = np.linalg.inv(G)
    low = 0.5 * (np.einsum("adb->dab", D) + np.einsum("bda->dab", D) - D)
    # low[d,a,b] = 1/2 (d_a g_db + d_b g_da - d_d g_ab)
    return np.einsum("cd,dab->cab", Gi, low)


def acoustic_speeds(g, prim, n, cs2):
    """Coordinate speeds lambda = dx^n/dt of the two sound fronts moving
    along spatial direction n, from the covariant characteristic condition
    of a perfect fluid, (u^a xi_a)^2 = c_s^2 h^ab xi_a xi_b with
    h^ab = g^ab + u^a u^b and the front covector xi = (-lambda, delta^n_i).
    Returns (lambda-, lambda+)."""
    G = four_metric(g)
    Gi = np.linalg.inv(G)
    ua = four_velocity_up(g, np.asarray(prim[1:4], dtype=float))
    c2 = cs2
    ut, un = ua[0], ua[1 + n]
    gtt, gtn, gnn = Gi[0, 0], Gi[0, 1 + n], Gi[1 + n, 1 + n]
    # (1 - c2)(u^n - lambda u^t)^2 - c2 (g^nn - 2 lambda g^tn + lambda^2 g^tt) = 0
    A = (1.0 - c2) * ut * ut - c2 * gtt
    B = -2.0 * ((1.0 - c2) * un * ut - c2 * gtn)
    C = (1.0 - c2) * un * un - c2 * gnn
    r = np.sqrt(B * B - 4.0 * A * C)
    return (-B - r) / (2.0 * A), (-B + r) / (2.0 * A)
