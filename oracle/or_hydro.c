/*
 * or_hydro.c -- plain FP64 CPU oracle of one GRHD Runge-Kutta substep.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may call it; the product path never does.
 *
 * Source of every formula: Lam & Shibata, "SACRA-2D" (arXiv 2502.03223),
 * Sec. II.C (GRHD).  Where the paper is silent or misprinted the reading
 * taken is stated next to the code (the same readings are listed in the
 * design notes of the repository).  Every step is done in the paper's order,
 * one array per intermediate, no fusion, no tiling.
 *
 * Parity pins live in tests/ (exact Riemann solution, uniform-state
 * preservation, conservation, con2prim round trip, polynomial exactness,
 * flux consistency against the stress-energy tensor, covariant source
 * identity, a uniform-pressure contact kept to round-off, smooth-wave
 * convergence).  Build: gcc -O3 -ffp-contract=off (no fused multiply-add, no
 * fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static int64_t cidx(const or_grid *g, int j, int k) {
  return (int64_t)(k + g->ng) * g->pitch + (j + g->ng);
}

static double mval(const or_metric *m, int f, int64_t i) {
  return m->f[f] ? m->f[f][i] : m->c[f];
}

/* inverse of the symmetric 3x3 matrix stored as (xx,xy,xz,yy,yz,zz) */
static void inv_sym3(const double *a, double *inv) {
  double cxx = a[3] * a[5] - a[4] * a[4];
  double cxy = a[2] * a[4] - a[1] * a[5];
  double cxz = a[1] * a[4] - a[2] * a[3];
  double cyy = a[0] * a[5] - a[2] * a[2];
  double cyz = a[1] * a[2] - a[0] * a[4];
  double czz = a[0] * a[3] - a[1] * a[1];
  double det = a[0] * cxx + a[1] * cxy + a[2] * cxz;
  inv[0] = cxx / det; inv[1] = cxy / det; inv[2] = cxz / det;
  inv[3] = cyy / det; inv[4] = cyz / det; inv[5] = czz / det;
}

/* element (i,j) of a symmetric matrix in (xx,xy,xz,yy,yz,zz) storage */
static double s3(const double *a, int i, int j) {
  static const int map[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return a[map[i][j]];
}

/* ------------------------------------------------------------------ */
/* Equation of state, Sec. II.C.3: cold piecewise polytrope + thermal   */
/* gamma-law part.  OR_EOS_IDEAL is the plain gamma-law P=(G-1) rho eps */
/* with eps_min = 0 (cold part identically zero).                       */
/* ------------------------------------------------------------------ */

static int eos_piece(const or_eos *e, double rho) {
  int i = 0;
  while (i < e->n - 1 && rho >= e->rho_b[i]) i++;
  return i;
}

/* Delta eps_i from continuity of the cold specific energy at rho_b */
static double eos_deps(const or_eos *e, int i) {
  double d = 0.0;
  for (int m = 1; m <= i; m++) {
    double rb = e->rho_b[m - 1];
    d += e->K[m - 1] / (e->G[m - 1] - 1.0) * pow(rb, e->G[m - 1] - 1.0) -
         e->K[m] / (e->G[m] - 1.0) * pow(rb, e->G[m] - 1.0);
  }
  return d;
}

double or_eos_press_cold(const or_eos *e, double rho) {
  if (e->kind == OR_EOS_IDEAL) return 0.0;
  int i = eos_piece(e, rho);
  return e->K[i] * pow(rho, e->G[i]);
}

double or_eos_eps_cold(const or_eos *e, double rho) {
  if (e->kind == OR_EOS_IDEAL) return 0.0;
  int i = eos_piece(e, rho);
  return e->K[i] / (e->G[i] - 1.0) * pow(rho, e->G[i] - 1.0) + eos_deps(e, i);
}

double or_eos_press(const or_eos *e, double rho, double eps) {
  if (e->kind == OR_EOS_IDEAL) return (e->Gth - 1.0) * rho * eps;
  double pc = or_eos_press_cold(e, rho);
  double ec = or_eos_eps_cold(e, rho);
  return pc + (e->Gth - 1.0) * rho * (eps - ec);
}

/* the inverse of or_eos_press in eps: the specific internal energy at
 * which the EOS gives pressure P at density rho */
double or_eos_eps(const or_eos *e, double rho, double P) {
  if (e->kind == OR_EOS_IDEAL) return P / ((e->Gth - 1.0) * rho);
  double pc = or_eos_press_cold(e, rho);
  double ec = or_eos_eps_cold(e, rho);
  return ec + (P - pc) / ((e->Gth - 1.0) * rho);
}

/* sound speed squared: c_s^2 h = dP/drho|_eps + (P/rho^2) dP/deps|_rho,
 * derivatives at (rho, eps), P as given (reconstructed states carry an
 * independent P); clamped to [0, 1). */
double or_eos_cs2(const or_eos *e, double rho, double eps, double P) {
  double chi, kap;
  if (e->kind == OR_EOS_IDEAL) {
    chi = (e->Gth - 1.0) * eps;
    kap = (e->Gth - 1.0) * rho;
  } else {
    int i = eos_piece(e, rho);
    double kr = e->K[i] * pow(rho, e->G[i] - 1.0);
    double ec = or_eos_eps_cold(e, rho);
    chi = e->G[i] * kr + (e->Gth - 1.0) * (eps - ec) - (e->Gth - 1.0) * kr;
    kap = (e->Gth - 1.0) * rho;
  }
  double h = 1.0 + eps + P / rho;
  double cs2 = (chi + P / (rho * rho) * kap) / h;
  if (!(cs2 > 0.0)) cs2 = 0.0;
  if (cs2 > 0.999999) cs2 = 0.999999;
  return cs2;
}

/* ------------------------------------------------------------------ */
/* prim -> con, eq. (cons_var): q = psi^6 (rho w, rho h w u_i,          */
/* rho h w^2 - P), psi^6 = W^-3, with q_Sphi = x q_Sy in cylindrical    */
/* geometry (u_phi = x u_y).                                            */
/* ------------------------------------------------------------------ */

void or_prim2con_point(const or_eos *e, const double *g, double x, int geom,
                       const double *p, double *q) {
  (void)e;
  double W = g[OR_W];
  double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
  double gtu[6];
  inv_sym3(gt, gtu);
  double u[3] = {p[1], p[2], p[3]};
  double usq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) usq += W * W * s3(gtu, i, j) * u[i] * u[j];
  double w = sqrt(1.0 + usq);
  double rho = p[0], P = p[4], eps = p[5];
  double h = 1.0 + eps + P / rho;
  double sg = 1.0 / (W * W * W);
  q[0] = sg * (rho * w);
  q[1] = sg * (rho * h * w * u[0]);
  q[2] = sg * (rho * h * w * u[1]);
  if (geom == OR_GEOM_CYL) q[2] = x * q[2];
  q[3] = sg * (rho * h * w * u[2]);
  q[4] = sg * (rho * h * w * w - P);
}

/* ------------------------------------------------------------------ */
/* con -> prim, Sec. II.C.4 (Galeazzi et al. master function).          */
/* The method converges to the unique root z* of f(z) in [z-, z+]; the  */
/* oracle finds that root by plain bisection to the last bit, which is  */
/* its definition.  Readings: k_max = 2 v_max/(1+v_max^2) for the S_i   */
/* rescaling; eps-hat clamped below by eps_min(rho-hat); cold recovery  */
/* when the unclamped eps(z*) < eps_min; atmosphere resets the whole    */
/* state (rho_atm, u = 0, cold P and eps) when rho < rho_atm.           */
/* ------------------------------------------------------------------ */

double or_c2p_master(const or_eos *e, double D, double qq, double r, double z) {
  double w = sqrt(1.0 + z * z);
  double rho = D / w;
  double eps = w * qq - z * r + z * z / (1.0 + w);
  double emin = or_eos_eps_cold(e, rho);
  if (eps < emin) eps = emin;
  double P = or_eos_press(e, rho, eps);
  double a = P / (rho * (1.0 + eps));
  double h = (1.0 + eps) * (1.0 + a);
  return z - r / h;
}

static double c2p_cold_fn(const or_eos *e, double D, double r, double z) {
  double w = sqrt(1.0 + z * z);
  double rho = D / w;
  double hc = 1.0 + or_eos_eps_cold(e, rho) + or_eos_press_cold(e, rho) / rho;
  return z - r / hc;
}

/* bisection on a bracket where fn(lo) <= 0 <= fn(hi), to the last bit */
static double bisect_root(const or_eos *e, double D, double qq, double r,
                          double lo, double hi, int cold) {
  double flo = cold ? c2p_cold_fn(e, D, r, lo) : or_c2p_master(e, D, qq, r, lo);
  double fhi = cold ? c2p_cold_fn(e, D, r, hi) : or_c2p_master(e, D, qq, r, hi);
  if (flo >= 0.0) return lo;
  if (fhi <= 0.0) return hi;
  for (int it = 0; it < 4000; it++) {
    double mid = lo + 0.5 * (hi - lo);
    if (!(mid > lo && mid < hi)) break;
    double fm = cold ? c2p_cold_fn(e, D, r, mid) : or_c2p_master(e, D, qq, r, mid);
    if (fm < 0.0) { lo = mid; flo = fm; }
    else { hi = mid; fhi = fm; }
  }
  return (-flo < fhi) ? lo : hi;
}

static void atmosphere_prim(const or_eos *e, const or_c2p *cp, double *p) {
  double ra = cp->rho_atm;
  double Pa, ea;
  if (e->kind == OR_EOS_IDEAL) {
    Pa = e->K[0] * pow(ra, e->G[0]);
    ea = Pa / ((e->Gth - 1.0) * ra);
  } else {
    Pa = or_eos_press_cold(e, ra);
    ea = or_eos_eps_cold(e, ra);
  }
  p[0] = ra; p[1] = 0.0; p[2] = 0.0; p[3] = 0.0; p[4] = Pa; p[5] = ea;
}

unsigned or_con2prim_point(const or_eos *e, const double *g, double x, int geom,
                           const or_c2p *cp, double *q, double *p, double *zroot) {
  unsigned flags = 0;
  double W = g[OR_W];
  double W3 = W * W * W;
  int ok = 1;
  for (int c = 0; c < 5; c++)
    if (!isfinite(q[c])) ok = 0;
  double D = W3 * q[0];
  double S[3];
  S[0] = W3 * q[1];
  S[1] = (geom == OR_GEOM_CYL) ? W3 * (q[2] / x) : W3 * q[2];
  S[2] = W3 * q[3];
  double E = W3 * q[4];
  if (!(D > 0.0) || !(E > 0.0)) ok = 0;
  double z = 0.0;
  if (ok) {
    double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
    double gtu[6];
    inv_sym3(gt, gtu);
    double S2 = 0.0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) S2 += W * W * s3(gtu, i, j) * S[i] * S[j];
    double r = sqrt(S2) / D;
    double qq = E / D - 1.0;
    double k = r / (1.0 + qq);
    double vmax = sqrt(1.0 - 1.0 / (cp->w_max * cp->w_max));
    double kmax = 2.0 * vmax / (1.0 + vmax * vmax);
    if (k > kmax) {
      double sc = kmax / k;
      S[0] *= sc; S[1] *= sc; S[2] *= sc;
      r = kmax * (1.0 + qq);
      k = kmax;
      flags |= OR_F_RESCALE;
    }
    double zm = 0.5 * k / sqrt(1.0 - 0.25 * k * k);
    double zp = k / sqrt(1.0 - k * k);
    /* the adiabatic mode (Sec. III.C.2) never uses the energy: only the
     * cold root below */
    z = (k > 0.0 && !cp->adiabatic) ? bisect_root(e, D, qq, r, zm, zp, 0) : 0.0;
    double w = sqrt(1.0 + z * z);
    double rho = D / w;
    double eps = w * qq - z * r + z * z / (1.0 + w);
    double P, h;
    if (cp->adiabatic || eps < or_eos_eps_cold(e, rho)) {
      /* zero-temperature recovery from (D, S_i) on [0, r] */
      z = (r > 0.0) ? bisect_root(e, D, qq, r, 0.0, r, 1) : 0.0;
      w = sqrt(1.0 + z * z);
      rho = D / w;
      eps = or_eos_eps_cold(e, rho);
      P = or_eos_press_cold(e, rho);
      flags |= OR_F_COLD;
    } else {
      P = or_eos_press(e, rho, eps);
    }
    h = 1.0 + eps + P / rho;
    p[0] = rho;
    p[1] = S[0] / (D * h);
    p[2] = S[1] / (D * h);
    p[3] = S[2] / (D * h);
    p[4] = P;
    p[5] = eps;
    if (!isfinite(rho) || !isfinite(P) || !isfinite(eps) || !isfinite(p[1]) ||
        !isfinite(p[2]) || !isfinite(p[3]))
      ok = 0;
  }
  /* a cell that ends as the atmosphere carries only the atmosphere flag
   * (plus the failure flag for invalid input) */
  if (!ok || p[0] < cp->rho_atm) {
    atmosphere_prim(e, cp, p);
    flags = ok ? OR_F_ATM : (OR_F_ATM | OR_F_FAIL);
    z = 0.0;
  }
  if (flags) or_prim2con_point(e, g, x, geom, p, q);
  if (zroot) *zroot = z;
  return flags;
}

/* ------------------------------------------------------------------ */
/* Reconstruction, Sec. II.C.2: third-order PPM (Colella & Woodward     */
/* 1984, interface values with monotonised slopes and the parabola      */
/* limiter; no steepening, no flattening) or minmod (the paper's        */
/* prolongation limiter).                                               */
/*                                                                      */
/* A second reading of "3rd-order PPM" (OR_RECON_PPM3): each cell's     */
/* parabola is the one whose averages over the cell and its two         */
/* neighbours are the three cell values; its edge values, held inside   */
/* the range of the two averages that meet at that edge, go through the */
/* same parabola limiter.  In CW84's form both sides of a face start    */
/* from one shared interface value, so where no limiter acts the two    */
/* face states are equal and the Riemann solver adds no dissipation;    */
/* here they differ by a sixth of the third difference across the face. */
/* ------------------------------------------------------------------ */

static double mono_slope(double am, double a0, double ap) {
  double d = 0.5 * (ap - am);
  if ((ap - a0) * (a0 - am) > 0.0) {
    double m = fabs(d);
    double l = 2.0 * fabs(a0 - am);
    double r = 2.0 * fabs(ap - a0);
    if (l < m) m = l;
    if (r < m) m = r;
    return copysign(m, d);
  }
  return 0.0;
}

static void ppm_cell(double a, double aL, double aR, double *oL, double *oR) {
  if ((aR - a) * (a - aL) <= 0.0) {
    aL = a;
    aR = a;
  } else {
    double dA = aR - aL;
    double a6 = 6.0 * (a - 0.5 * (aL + aR));
    if (dA * a6 > dA * dA) aL = 3.0 * a - 2.0 * aR;
    else if (-(dA * dA) > dA * a6) aR = 3.0 * a - 2.0 * aL;
  }
  *oL = aL;
  *oR = aR;
}

/* edge values of the parabola with averages am, a0, ap over three
 * neighbouring cells of equal width (left edge, right edge of the middle
 * cell), each clipped to the range of the two averages at that edge */
static void parabola3_edges(double am, double a0, double ap, double *eL, double *eR) {
  double l = (2.0 * am + 5.0 * a0 - ap) / 6.0;
  double r = (-am + 5.0 * a0 + 2.0 * ap) / 6.0;
  *eL = fmin(fmax(l, fmin(am, a0)), fmax(am, a0));
  *eR = fmin(fmax(r, fmin(a0, ap)), fmax(a0, ap));
}

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (fabs(a) < fabs(b)) ? a : b;
}

void or_recon_line(int recon, int n, const double *a, double *aL, double *aR) {
  if (n < 6) return;
  if (recon == OR_RECON_MINMOD) {
    for (int i = 2; i <= n - 4; i++) {
      double si = minmod(a[i] - a[i - 1], a[i + 1] - a[i]);
      double sj = minmod(a[i + 1] - a[i], a[i + 2] - a[i + 1]);
      aL[i - 2] = a[i] + 0.5 * si;
      aR[i - 2] = a[i + 1] - 0.5 * sj;
    }
    return;
  }
  if (recon == OR_RECON_PPM3) {
    for (int i = 2; i <= n - 4; i++) {
      double eL0, eR0, eL1, eR1, l0, r0, l1, r1;
      parabola3_edges(a[i - 1], a[i], a[i + 1], &eL0, &eR0);
      parabola3_edges(a[i], a[i + 1], a[i + 2], &eL1, &eR1);
      ppm_cell(a[i], eL0, eR0, &l0, &r0);
      ppm_cell(a[i + 1], eL1, eR1, &l1, &r1);
      aL[i - 2] = r0;
      aR[i - 2] = l1;
    }
    return;
  }
  double *dm = (double *)malloc(sizeof(double) * n);
  double *ai = (double *)malloc(sizeof(double) * n);
  for (int i = 1; i < n - 1; i++) dm[i] = mono_slope(a[i - 1], a[i], a[i + 1]);
  /* ai[i] = interface value a_{i+1/2} */
  for (int i = 1; i < n - 2; i++)
    ai[i] = a[i] + 0.5 * (a[i + 1] - a[i]) - (dm[i + 1] - dm[i]) / 6.0;
  for (int i = 2; i <= n - 4; i++) {
    double l0, r0, l1, r1;
    ppm_cell(a[i], ai[i - 1], ai[i], &l0, &r0);
    ppm_cell(a[i + 1], ai[i], ai[i + 1], &l1, &r1);
    aL[i - 2] = r0;  /* left state at face i+1/2: right edge of cell i */
    aR[i - 2] = l1;  /* right state: left edge of cell i+1 */
  }
  free(dm);
  free(ai);
}

/* metric at a face: centred 6-point Lagrange interpolation (reading of
 * "Lagrangian interpolation"), weights (3,-25,150,150,-25,3)/256 */
double or_lagrange6(const double *a) {
  return (3.0 * a[0] - 25.0 * a[1] + 150.0 * a[2] + 150.0 * a[3] - 25.0 * a[4] +
          3.0 * a[5]) / 256.0;
}

/* sixth-order centred first derivative (the paper's finite-difference
 * order), weights (-1,9,-45,0,45,-9,1)/60h */
double or_deriv6(const double *a, double h) {
  return (-a[0] + 9.0 * a[1] - 45.0 * a[2] + 45.0 * a[4] - 9.0 * a[5] + a[6]) /
         (60.0 * h);
}

/* ------------------------------------------------------------------ */
/* Fluxes, Sec. II.C.1-2.                                               */
/* Valencia flux (reading of the misprinted alpha factor):              */
/*   f^n = W^-3 [ (D, S_j, E)(alpha v^n - beta^n) + alpha P (0, d^n_j, v^n) ]  */
/* with v^n = gamma^{nj} u_j / w the Eulerian velocity.                 */
/* ------------------------------------------------------------------ */

struct fstate {
  double rho, u[3], P, eps;
};

void or_valencia_flux_point(const or_eos *e, const double *g, int dir,
                            const double *p, double *F) {
  (void)e;
  int n = (dir == 0) ? 0 : 2;
  double alp = g[OR_ALP], W = g[OR_W];
  double beta[3] = {g[OR_BX], g[OR_BY], g[OR_BZ]};
  double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
  double gtu[6];
  inv_sym3(gt, gtu);
  double u[3] = {p[1], p[2], p[3]};
  double usq = 0.0, un = 0.0;
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) usq += W * W * s3(gtu, i, j) * u[i] * u[j];
    un += W * W * s3(gtu, n, i) * u[i];
  }
  double w = sqrt(1.0 + usq);
  double rho = p[0], P = p[4], eps = p[5];
  double h = 1.0 + eps + P / rho;
  double vn = un / w;
  double D = rho * w, E = rho * h * w * w - P;
  double sg = 1.0 / (W * W * W);
  double tr = alp * vn - beta[n];
  F[0] = sg * (D * tr);
  for (int j = 0; j < 3; j++)
    F[1 + j] = sg * (rho * h * w * u[j] * tr + ((j == n) ? alp * P : 0.0));
  F[4] = sg * (E * tr + alp * P * vn);
}

/* densitised conserved vector in Cartesian components (no x factor) */
static void cons_cart(const double *g, const double *p, double *q) {
  double W = g[OR_W];
  double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
  double gtu[6];
  inv_sym3(gt, gtu);
  double usq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) usq += W * W * s3(gtu, i, j) * p[1 + i] * p[1 + j];
  double w = sqrt(1.0 + usq);
  double h = 1.0 + p[5] + p[4] / p[0];
  double sg = 1.0 / (W * W * W);
  q[0] = sg * (p[0] * w);
  for (int j = 0; j < 3; j++) q[1 + j] = sg * (p[0] * h * w * p[1 + j]);
  q[4] = sg * (p[0] * h * w * w - p[4]);
}

/* coordinate characteristic speeds (Banyuls et al. 1997) for TVDLF */
void or_coord_speeds(const or_eos *e, const double *g, int dir,
                     const double *p, double *lm, double *lp) {
  int n = (dir == 0) ? 0 : 2;
  double alp = g[OR_ALP], W = g[OR_W];
  double beta[3] = {g[OR_BX], g[OR_BY], g[OR_BZ]};
  double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
  double gtu[6];
  inv_sym3(gt, gtu);
  double usq = 0.0, un = 0.0;
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) usq += W * W * s3(gtu, i, j) * p[1 + i] * p[1 + j];
    un += W * W * s3(gtu, n, i) * p[1 + i];
  }
  double w = sqrt(1.0 + usq);
  double vn = un / w;
  double v2 = usq / (w * w);
  double gnn = W * W * s3(gtu, n, n);
  double cs2 = or_eos_cs2(e, p[0], p[5], p[4]);
  double cs = sqrt(cs2);
  double disc = (1.0 - v2) * (gnn * (1.0 - v2 * cs2) - vn * vn * (1.0 - cs2));
  if (disc < 0.0) disc = 0.0;
  double den = 1.0 - v2 * cs2;
  *lm = alp / den * (vn * (1.0 - cs2) - cs * sqrt(disc)) - beta[n];
  *lp = alp / den * (vn * (1.0 - cs2) + cs * sqrt(disc)) - beta[n];
}

/* tetrad-frame state (special-relativistic form), corrected readings:
 * E = rho h w^2 - P and S_(j) = rho h w u_(j) */
struct tstate {
  double q[5], f[5];  /* order: D, S_(n), S_(t1), S_(t2), E */
  double vn, P, lm, lp;
};

static void tetrad_state(const or_eos *e, const double *p, double E_leg[3][3],
                         struct tstate *s) {
  double ut[3];
  for (int a = 0; a < 3; a++) {
    ut[a] = 0.0;
    for (int i = 0; i < 3; i++) ut[a] += E_leg[a][i] * p[1 + i];
  }
  double w = sqrt(1.0 + ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
  double v[3] = {ut[0] / w, ut[1] / w, ut[2] / w};
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double rho = p[0], P = p[4], eps = p[5];
  double h = 1.0 + eps + P / rho;
  s->q[0] = rho * w;
  for (int a = 0; a < 3; a++) s->q[1 + a] = rho * h * w * ut[a];
  s->q[4] = rho * h * w * w - P;
  s->vn = v[0];
  s->P = P;
  s->f[0] = s->q[0] * v[0];
  s->f[1] = s->q[1] * v[0] + P;
  s->f[2] = s->q[2] * v[0];
  s->f[3] = s->q[3] * v[0];
  s->f[4] = (s->q[4] + P) * v[0];
  double cs2 = or_eos_cs2(e, rho, eps, P);
  double cs = sqrt(cs2);
  double disc = (1.0 - v2) * (1.0 - v2 * cs2 - (1.0 - cs2) * v[0] * v[0]);
  if (disc < 0.0) disc = 0.0;
  double den = 1.0 - v2 * cs2;
  s->lm = (v[0] * (1.0 - cs2) - cs * sqrt(disc)) / den;
  s->lp = (v[0] * (1.0 - cs2) + cs * sqrt(disc)) / den;
}

/* HLLC starred state of side s (Mignone & Bodo 2005 in the tetrad frame) */
static void hllc_star(const struct tstate *s, double lam, double lc, double Pc,
                      double *qc) {
  double dl = lam - s->vn;
  double den = lam - lc;
  qc[0] = s->q[0] * dl / den;
  qc[1] = (s->q[1] * dl + Pc - s->P) / den;
  qc[2] = s->q[2] * dl / den;
  qc[3] = s->q[3] * dl / den;
  qc[4] = (s->q[4] * dl + Pc * lc - s->P * s->vn) / den;
}

/* Tetrad of a face (Sec. II.C.2): contravariant spatial legs El (normal,
 * tangent 1, tangent 2; x/y/z components), covariant legs Ec, the normal
 * factor sqrt(gamma^nn) and the face speed v_int in the tetrad frame. */
static void face_tetrad(const double *g, int dir, double El[3][3], double Ec[3][3],
                        double *sqgnn_out, double *vint_out) {
  int n = (dir == 0) ? 0 : 2;
  double alp = g[OR_ALP], W = g[OR_W];
  double beta[3] = {g[OR_BX], g[OR_BY], g[OR_BZ]};
  double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
  double gtu[6];
  inv_sym3(gt, gtu);
  if (dir == 0) {
    double B = 1.0 / sqrt(gtu[0]);
    double C = 1.0 / sqrt(gt[5]);
    double Dh = B * C;
    El[0][0] = W * B * gtu[0]; El[0][1] = W * B * gtu[1]; El[0][2] = W * B * gtu[2];
    El[1][0] = 0.0; El[1][1] = W * Dh * gt[5]; El[1][2] = -(W * Dh * gt[4]);
    El[2][0] = 0.0; El[2][1] = 0.0; El[2][2] = W * C;
  } else {
    /* z faces: cyclic relabelling (n, t1, t2) = (z, x, y) */
    double B = 1.0 / sqrt(gtu[5]);
    double C = 1.0 / sqrt(gt[3]);
    double Dh = B * C;
    El[0][0] = W * B * gtu[2]; El[0][1] = W * B * gtu[4]; El[0][2] = W * B * gtu[5];
    El[1][0] = W * Dh * gt[3]; El[1][1] = -(W * Dh * gt[1]); El[1][2] = 0.0;
    El[2][0] = 0.0; El[2][1] = W * C; El[2][2] = 0.0;
  }
  /* covariant legs e_(a)_j = gamma_ji e_(a)^i, gamma_ij = W^-2 gt_ij */
  for (int a = 0; a < 3; a++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int i = 0; i < 3; i++) s += s3(gt, j, i) * El[a][i];
      Ec[a][j] = s / (W * W);
    }
  double sqgnn = W * sqrt(s3(gtu, n, n));
  *sqgnn_out = sqgnn;
  *vint_out = beta[n] / (alp * sqgnn);
}

/* the signal speeds lambda-, lambda+ of one state in the face tetrad
 * frame, mapped to coordinate speeds alpha sqrt(gamma^nn) lambda - beta^n */
void or_tetrad_speeds(const or_eos *e, const double *g, int dir, const double *p,
                      double *lm, double *lp) {
  double El[3][3], Ec[3][3], sqgnn, vint;
  face_tetrad(g, dir, El, Ec, &sqgnn, &vint);
  struct tstate s;
  tetrad_state(e, p, El, &s);
  double f = g[OR_ALP] * sqgnn;
  *lm = f * (s.lm - vint);
  *lp = f * (s.lp - vint);
}

void or_face_flux_point(const or_eos *e, const double *g, int dir, int riemann,
                        const double *pL, const double *pR, double *F,
                        double *speed) {
  double alp = g[OR_ALP], W = g[OR_W];
  double sg = 1.0 / (W * W * W);
  if (riemann == OR_RIEMANN_TVDLF) {
    /* local Lax-Friedrichs in the coordinate frame (reading of TVDLF) */
    double fL[5], fR[5], qL[5], qR[5], l1, l2, l3, l4;
    or_valencia_flux_point(e, g, dir, pL, fL);
    or_valencia_flux_point(e, g, dir, pR, fR);
    cons_cart(g, pL, qL);
    cons_cart(g, pR, qR);
    or_coord_speeds(e, g, dir, pL, &l1, &l2);
    or_coord_speeds(e, g, dir, pR, &l3, &l4);
    double c = fabs(l1);
    if (fabs(l2) > c) c = fabs(l2);
    if (fabs(l3) > c) c = fabs(l3);
    if (fabs(l4) > c) c = fabs(l4);
    for (int m = 0; m < 5; m++) F[m] = 0.5 * (fL[m] + fR[m] - c * (qR[m] - qL[m]));
    if (speed) *speed = c;
    return;
  }
  /* HLLC in the tetrad frame of the face */
  double El[3][3], Ec[3][3], sqgnn, vint;
  face_tetrad(g, dir, El, Ec, &sqgnn, &vint);

  struct tstate L, R;
  tetrad_state(e, pL, El, &L);
  tetrad_state(e, pR, El, &R);
  double lamL = (L.lm < R.lm) ? L.lm : R.lm;
  double lamR = (L.lp > R.lp) ? L.lp : R.lp;

  double G[5];
  if (!(lamR - lamL > 0.0)) {
    const struct tstate *s = (vint <= lamL) ? &L : &R;
    for (int m = 0; m < 5; m++) G[m] = s->f[m] - vint * s->q[m];
  } else {
    double qh[5], fh[5];
    double dlam = lamR - lamL;
    for (int m = 0; m < 5; m++) {
      qh[m] = (lamR * R.q[m] - lamL * L.q[m] + L.f[m] - R.f[m]) / dlam;
      fh[m] = (lamR * L.f[m] - lamL * R.f[m] + lamR * lamL * (R.q[m] - L.q[m])) / dlam;
    }
    /* contact speed: root of fh_E lc^2 - (E_h + fh_Sn) lc + Sn_h = 0,
     * the Mignone-Bodo root in cancellation-free form */
    double qa = fh[4];
    double qb = -(qh[4] + fh[1]);
    double qc = qh[1];
    double disc = qb * qb - 4.0 * qa * qc;
    if (disc < 0.0) disc = 0.0;
    double den = -qb + sqrt(disc);
    double lc = (den > 0.0) ? 2.0 * qc / den : 0.0;
    if (!(den > 0.0) || !(lc > lamL && lc < lamR)) {
      /* degenerate fan: HLL state */
      if (vint <= lamL) for (int m = 0; m < 5; m++) G[m] = L.f[m] - vint * L.q[m];
      else if (vint <= lamR) for (int m = 0; m < 5; m++) G[m] = fh[m] - vint * qh[m];
      else for (int m = 0; m < 5; m++) G[m] = R.f[m] - vint * R.q[m];
    } else {
      double Pc = -lc * fh[4] + fh[1];
      double qs[5], fs[5];
      if (vint <= lamL) {
        for (int m = 0; m < 5; m++) G[m] = L.f[m] - vint * L.q[m];
      } else if (vint <= lc) {
        hllc_star(&L, lamL, lc, Pc, qs);
        for (int m = 0; m < 5; m++) {
          fs[m] = L.f[m] + lamL * (qs[m] - L.q[m]);
          G[m] = fs[m] - vint * qs[m];
        }
      } else if (vint <= lamR) {
        hllc_star(&R, lamR, lc, Pc, qs);
        for (int m = 0; m < 5; m++) {
          fs[m] = R.f[m] + lamR * (qs[m] - R.q[m]);
          G[m] = fs[m] - vint * qs[m];
        }
      } else {
        for (int m = 0; m < 5; m++) G[m] = R.f[m] - vint * R.q[m];
      }
    }
  }
  /* back to the Eulerian coordinate frame, then densitise with alpha W^-3 */
  F[0] = alp * sg * (sqgnn * G[0]);
  for (int j = 0; j < 3; j++) {
    double s = Ec[0][j] * G[1] + Ec[1][j] * G[2] + Ec[2][j] * G[3];
    F[1 + j] = alp * sg * (sqgnn * s);
  }
  F[4] = alp * sg * (sqgnn * G[4]);
  if (speed) {
    double a1 = fabs(lamL - vint), a2 = fabs(lamR - vint);
    *speed = alp * sqgnn * ((a1 > a2) ? a1 : a2);
  }
}

/* ------------------------------------------------------------------ */
/* Source terms, Sec. II.C.1 (corrected reading):                       */
/*  s_Sj = P d_j(alpha W^-3) - W^-3 rho h w^2 [ d_j alpha - v_i d_j beta^i */
/*         + (W^2/2) alpha v_i v_k d_j gt^{ik} + (1/W) alpha v_i v^i d_j W ] */
/*         (+ the cylindrical term (f_Sphi)^phi / varpi for j = varpi)  */
/*  s_E  = W^-3 [ alpha K_ij S^ij - rho h w^2 v^i d_i alpha ]           */
/* with v_i = u_i / w the Eulerian velocity; d(alpha W^-3) by the       */
/* product rule and d gt^{ik} = -gt^{ia} gt^{kb} d gt_ab (readings).    */
/* ------------------------------------------------------------------ */

void or_source_point(const or_eos *e, const double *g, const double *dg,
                     double x, int geom, const double *p, double *s) {
  (void)e;
  double alp = g[OR_ALP], W = g[OR_W];
  double beta[3] = {g[OR_BX], g[OR_BY], g[OR_BZ]};
  double gt[6] = {g[OR_GXX], g[OR_GXY], g[OR_GXZ], g[OR_GYY], g[OR_GYZ], g[OR_GZZ]};
  double Kl[6] = {g[OR_KXX], g[OR_KXY], g[OR_KXZ], g[OR_KYY], g[OR_KYZ], g[OR_KZZ]};
  double gtu[6];
  inv_sym3(gt, gtu);
  double rho = p[0], P = p[4], eps = p[5];
  double u[3] = {p[1], p[2], p[3]};
  double usq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) usq += W * W * s3(gtu, i, j) * u[i] * u[j];
  double w = sqrt(1.0 + usq);
  double h = 1.0 + eps + P / rho;
  double vl[3], vu[3], vt[3];
  for (int i = 0; i < 3; i++) vl[i] = u[i] / w;
  for (int i = 0; i < 3; i++) {
    vu[i] = 0.0;
    vt[i] = 0.0;
    for (int j = 0; j < 3; j++) {
      vu[i] += W * W * s3(gtu, i, j) * vl[j];
      vt[i] += s3(gtu, i, j) * vl[j];
    }
  }
  double vsq = vl[0] * vu[0] + vl[1] * vu[1] + vl[2] * vu[2];
  double sg = 1.0 / (W * W * W);
  double rhw2 = rho * h * w * w;
  double sm[2];
  for (int d = 0; d < 2; d++) {
    const double *dd = dg + d * OR_NMET;
    double dalp = dd[OR_ALP], dW = dd[OR_W];
    double dsg = -3.0 * dW / (W * W * W * W);   /* d(W^-3) */
    double dasg = dalp * sg + alp * dsg;        /* d(alpha W^-3) */
    double vdb = vl[0] * dd[OR_BX] + vl[1] * dd[OR_BY] + vl[2] * dd[OR_BZ];
    double dgt[6] = {dd[OR_GXX], dd[OR_GXY], dd[OR_GXZ], dd[OR_GYY], dd[OR_GYZ], dd[OR_GZZ]};
    double vvdg = 0.0;  /* v_i v_k d gt^{ik} */
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) vvdg -= vt[a] * vt[b] * s3(dgt, a, b);
    double br = dalp - vdb + 0.5 * W * W * alp * vvdg + alp * vsq * dW / W;
    sm[d] = P * dasg - sg * rhw2 * br;
  }
  s[0] = 0.0;
  s[1] = sm[0];
  s[2] = 0.0;
  s[3] = sm[1];
  if (geom == OR_GEOM_CYL) {
    /* (f_Sphi)^phi / varpi = W^-3 [ S_y (alpha v^y - beta^y) + alpha P ] / x */
    double Sy = rho * h * w * u[1];
    s[1] += sg * (Sy * (alp * vu[1] - beta[1]) + alp * P) / x;
  }
  /* energy: K_ij S^ij = rho h w^2 v^i v^j K_ij + P gamma^ij K_ij */
  double KS = 0.0, trK = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      KS += vu[i] * vu[j] * s3(Kl, i, j);
      trK += W * W * s3(gtu, i, j) * s3(Kl, i, j);
    }
  KS = rhw2 * KS + P * trK;
  double vda = vu[0] * dg[OR_ALP] + vu[2] * dg[OR_NMET + OR_ALP];
  s[4] = sg * (alp * KS - rhw2 * vda);
}

/* ------------------------------------------------------------------ */
/* grid-level operations                                                */
/* ------------------------------------------------------------------ */

static double xc(const or_grid *g, int j) { return g->x0 + (j + 0.5) * g->dx; }
static double xf(const or_grid *g, int j) { return g->x0 + j * g->dx; }

static void metric_at(const or_metric *m, int64_t i, double *g) {
  for (int f = 0; f < OR_NMET; f++) g[f] = mval(m, f, i);
}

void or_prim2con(const or_grid *gr, const or_eos *e, const or_metric *m,
                 double *const *p, double *const *q, int with_ghosts) {
  int lo = with_ghosts ? -gr->ng : 0;
  for (int k = lo; k < gr->nz - lo; k++)
    for (int j = lo; j < gr->nx - lo; j++) {
      int64_t i = cidx(gr, j, k);
      double g[OR_NMET], pp[6], qq[5];
      metric_at(m, i, g);
      for (int c = 0; c < 6; c++) pp[c] = p[c][i];
      or_prim2con_point(e, g, xc(gr, j), gr->geom, pp, qq);
      for (int c = 0; c < 5; c++) q[c][i] = qq[c];
    }
}

static int ext_side(const or_grid *gr, int j, int k) {
  /* 1 if ghost cell (j,k) is supplied by the caller (external boundary) */
  if (j < 0 && k >= 0 && k < gr->nz) return gr->bc[0] == OR_BC_EXTERNAL;
  if (j >= gr->nx && k >= 0 && k < gr->nz) return gr->bc[1] == OR_BC_EXTERNAL;
  if (k < 0 && j >= 0 && j < gr->nx) return gr->bc[2] == OR_BC_EXTERNAL;
  if (k >= gr->nz && j >= 0 && j < gr->nx) return gr->bc[3] == OR_BC_EXTERNAL;
  return 0;
}

void or_con2prim(const or_grid *gr, const or_eos *e, const or_metric *m,
                 const or_c2p *cp, double *const *q, double *const *p,
                 uint8_t *flags, or_diag *diag) {
  int ng = gr->ng;
  for (int k = -ng; k < gr->nz + ng; k++)
    for (int j = -ng; j < gr->nx + ng; j++) {
      int interior = (j >= 0 && j < gr->nx && k >= 0 && k < gr->nz);
      if (!interior && !ext_side(gr, j, k)) continue;
      int64_t i = cidx(gr, j, k);
      double g[OR_NMET], pp[6], qq[5];
      metric_at(m, i, g);
      for (int c = 0; c < 5; c++) qq[c] = q[c][i];
      unsigned f = or_con2prim_point(e, g, xc(gr, j), gr->geom, cp, qq, pp, NULL);
      for (int c = 0; c < 5; c++) q[c][i] = qq[c];
      for (int c = 0; c < 6; c++) p[c][i] = pp[c];
      if (flags) flags[i] = (uint8_t)f;
      if (diag && interior) {
        if (f & OR_F_RESCALE) diag->n_rescale++;
        if (f & OR_F_COLD) diag->n_cold++;
        if (f & OR_F_ATM) diag->n_atm++;
        if (f & OR_F_FAIL) diag->n_fail++;
      }
    }
}

/* boundary conditions on primitives: axis parity (u_x, u_y odd),
 * mirror (normal velocity odd), periodic (the ghost at index j takes the
 * cell j mod n, so a direction of fewer than 3 cells wraps onto itself),
 * outflow copy, external (kept) */
void or_fill_ghosts(const or_grid *gr, double *const *p) {
  int ng = gr->ng, nx = gr->nx, nz = gr->nz;
  for (int k = 0; k < nz; k++)
    for (int side = 0; side < 2; side++) {
      int bc = gr->bc[side];
      if (bc == OR_BC_EXTERNAL) continue;
      for (int mm = 0; mm < ng; mm++) {
        int jg = side == 0 ? -1 - mm : nx + mm;
        int js;
        if (bc == OR_BC_PERIODIC) js = ((jg % nx) + nx) % nx;
        else if (bc == OR_BC_OUTFLOW) js = side == 0 ? 0 : nx - 1;
        else js = side == 0 ? mm : nx - 1 - mm;
        int64_t ig = cidx(gr, jg, k), is = cidx(gr, js, k);
        for (int c = 0; c < 6; c++) p[c][ig] = p[c][is];
        if (bc == OR_BC_AXIS) { p[1][ig] = -p[1][ig]; p[2][ig] = -p[2][ig]; }
        if (bc == OR_BC_REFLECT) p[1][ig] = -p[1][ig];
      }
    }
  for (int j = -ng; j < nx + ng; j++)
    for (int side = 0; side < 2; side++) {
      int bc = gr->bc[2 + side];
      if (bc == OR_BC_EXTERNAL) continue;
      for (int mm = 0; mm < ng; mm++) {
        int kg = side == 0 ? -1 - mm : nz + mm;
        int ks;
        if (bc == OR_BC_PERIODIC) ks = ((kg % nz) + nz) % nz;
        else if (bc == OR_BC_OUTFLOW) ks = side == 0 ? 0 : nz - 1;
        else ks = side == 0 ? mm : nz - 1 - mm;
        int64_t ig = cidx(gr, j, kg), is = cidx(gr, j, ks);
        for (int c = 0; c < 6; c++) p[c][ig] = p[c][is];
        if (bc == OR_BC_REFLECT || bc == OR_BC_AXIS) p[3][ig] = -p[3][ig];
      }
    }
}

/* x faces: index k*(nx+1) + j for face x_{j-1/2}, j = 0..nx, k = 0..nz-1;
 * z faces: index k*nx + j for face z_{k-1/2}, k = 0..nz, j = 0..nx-1 */
void or_reconstruct(const or_grid *gr, int dir, int recon, double *const *p,
                    double *const *pL, double *const *pR) {
  int ng = gr->ng, nx = gr->nx, nz = gr->nz;
  int nl = (dir == 0) ? nx + 2 * ng : nz + 2 * ng;
  int nlines = (dir == 0) ? nz : nx;
  double *line = (double *)malloc(sizeof(double) * nl);
  double *aL = (double *)malloc(sizeof(double) * nl);
  double *aR = (double *)malloc(sizeof(double) * nl);
  for (int l = 0; l < nlines; l++)
    for (int c = 0; c < 6; c++) {
      for (int s = 0; s < nl; s++) {
        int64_t i = (dir == 0) ? cidx(gr, s - ng, l) : cidx(gr, l, s - ng);
        line[s] = p[c][i];
      }
      or_recon_line(recon, nl, line, aL, aR);
      int nf = (dir == 0) ? nx + 1 : nz + 1;
      for (int f = 0; f < nf; f++) {
        /* face index f in line coordinates: face (f-1)+1/2 + ng shift */
        int64_t o = (dir == 0) ? (int64_t)l * (nx + 1) + f : (int64_t)f * nx + l;
        pL[c][o] = aL[f + ng - 3];
        pR[c][o] = aR[f + ng - 3];
      }
    }
  free(line);
  free(aL);
  free(aR);
}

/* face metric by 6-point interpolation along the face normal */
static void face_metric(const or_grid *gr, const or_metric *m, int dir, int j,
                        int k, double *g) {
  for (int f = 0; f < OR_NMET; f++) {
    if (!m->f[f]) { g[f] = m->c[f]; continue; }
    double a[6];
    for (int s = 0; s < 6; s++) {
      int64_t i = (dir == 0) ? cidx(gr, j - 3 + s, k) : cidx(gr, j, k - 3 + s);
      a[s] = m->f[f][i];
    }
    g[f] = or_lagrange6(a);
  }
}

void or_face_flux(const or_grid *gr, int dir, int riemann, const or_eos *e,
                  const or_metric *m, double *const *pL, double *const *pR,
                  double *const *F, double *max_speed) {
  int nx = gr->nx, nz = gr->nz;
  int nfx = (dir == 0) ? nx + 1 : nx;
  int nfz = (dir == 0) ? nz : nz + 1;
  double smax = 0.0;
  for (int k = 0; k < nfz; k++)
    for (int j = 0; j < nfx; j++) {
      int64_t o = (int64_t)k * nfx + j;
      double g[OR_NMET], a[6], b[6], ff[5], sp;
      face_metric(gr, m, dir, j, k, g);
      for (int c = 0; c < 6; c++) { a[c] = pL[c][o]; b[c] = pR[c][o]; }
      or_face_flux_point(e, g, dir, riemann, a, b, ff, &sp);
      if (sp > smax) smax = sp;
      if (gr->geom == OR_GEOM_CYL) {
        /* flux of q_Sphi = x q_Sy: x at the face (x faces) or centre */
        double xx = (dir == 0) ? xf(gr, j) : xc(gr, j);
        ff[2] = xx * ff[2];
      }
      for (int c = 0; c < 5; c++) F[c][o] = ff[c];
    }
  if (max_speed) *max_speed = smax;
}

/* L(q) = <s> - (1/dV) [area-weighted flux differences], Sec. II.C.1 */
void or_rhs(const or_grid *gr, const or_eos *e, const or_metric *m,
            double *const *p, double *const *Fx, double *const *Fz,
            double *const *L) {
  int nx = gr->nx, nz = gr->nz;
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < nx; j++) {
      int64_t i = cidx(gr, j, k);
      double g[OR_NMET], dg[2 * OR_NMET], pp[6], s[5];
      metric_at(m, i, g);
      for (int d = 0; d < 2; d++)
        for (int f = 0; f < OR_NMET; f++) {
          if (!m->f[f]) { dg[d * OR_NMET + f] = 0.0; continue; }
          double a[7];
          for (int t = 0; t < 7; t++) {
            int64_t ii = (d == 0) ? cidx(gr, j - 3 + t, k) : cidx(gr, j, k - 3 + t);
            a[t] = m->f[f][ii];
          }
          dg[d * OR_NMET + f] = or_deriv6(a, d == 0 ? gr->dx : gr->dz);
        }
      for (int c = 0; c < 6; c++) pp[c] = p[c][i];
      or_source_point(e, g, dg, xc(gr, j), gr->geom, pp, s);
      int64_t fxl = (int64_t)k * (nx + 1) + j, fxr = fxl + 1;
      int64_t fzl = (int64_t)k * nx + j, fzr = fzl + nx;
      for (int c = 0; c < 5; c++) {
        double divx, divz;
        if (gr->geom == OR_GEOM_CYL) {
          divx = (xf(gr, j + 1) * Fx[c][fxr] - xf(gr, j) * Fx[c][fxl]) /
                 (xc(gr, j) * gr->dx);
        } else {
          divx = (Fx[c][fxr] - Fx[c][fxl]) / gr->dx;
        }
        divz = (Fz[c][fzr] - Fz[c][fzl]) / gr->dz;
        L[c][i] = s[c] - divx - divz;
      }
    }
}

static double **alloc_fields(int nf, int64_t n) {
  double **a = (double **)malloc(sizeof(double *) * nf);
  for (int c = 0; c < nf; c++) a[c] = (double *)calloc((size_t)n, sizeof(double));
  return a;
}

static void free_fields(double **a, int nf) {
  for (int c = 0; c < nf; c++) free(a[c]);
  free(a);
}

/* Face states on the EOS: a variant of Sec. II.C.2, which names rho, u_i,
 * P and eps as the primitives taken to the faces.  In the variant rho, u_i
 * and P come from the reconstruction and eps from the EOS at the
 * reconstructed (rho, P), so the face states lie on the EOS. */
static void faces_on_eos(const or_eos *e, int64_t n, double *const *L, double *const *R) {
  for (int64_t o = 0; o < n; o++) {
    L[5][o] = or_eos_eps(e, L[0][o], L[4][o]);
    R[5][o] = or_eos_eps(e, R[0][o], R[4][o]);
  }
}

int or_rk_substep(const or_grid *gr, const or_eos *e, const or_metric *m,
                  int recon, int riemann, int face_eps, const or_c2p *cp,
                  const or_stage *st, double *const *qn, double *const *qs,
                  double *const *qout, double *const *p_out, double *const *acc_in,
                  double *const *acc_out, double *flux_reg, uint8_t *flags,
                  or_diag *diag) {
  return or_rk_substep_reg(gr, e, m, recon, riemann, face_eps, cp, st, qn, qs, qout, p_out,
                           acc_in, acc_out, flux_reg, flags, diag, NULL, 0, 0, 0.0, NULL, NULL);
}

int or_rk_substep_reg(const or_grid *gr, const or_eos *e, const or_metric *m,
                      int recon, int riemann, int face_eps, const or_c2p *cp,
                      const or_stage *st,
                      double *const *qn, double *const *qs, double *const *qout,
                      double *const *p_out, double *const *acc_in,
                      double *const *acc_out, double *flux_reg, uint8_t *flags,
                      or_diag *diag, double *reg, int reg_j, int reg_k, double reg_w,
                      double *const *fx_out, double *const *fz_out) {
  int nx = gr->nx, nz = gr->nz;
  int64_t ncell = (int64_t)(nz + 2 * gr->ng) * gr->pitch;
  int64_t nfxa = (int64_t)nz * (nx + 1), nfza = (int64_t)(nz + 1) * nx;
  double **p = alloc_fields(6, ncell);
  double **L = alloc_fields(5, ncell);
  double **xL = alloc_fields(6, nfxa), **xR = alloc_fields(6, nfxa);
  double **zL = alloc_fields(6, nfza), **zR = alloc_fields(6, nfza);
  double **Fx = alloc_fields(5, nfxa), **Fz = alloc_fields(5, nfza);
  or_diag dloc;
  memset(&dloc, 0, sizeof(dloc));

  /* 1. primitive recovery (q_s corrected in place) */
  or_con2prim(gr, e, m, cp, qs, p, flags, &dloc);
  /* 2. ghost cells on primitives */
  or_fill_ghosts(gr, p);
  /* 3. reconstruction of (rho, u_i, P, eps), 4. Riemann fluxes, in x then z */
  double sx, sz;
  or_reconstruct(gr, 0, recon, p, xL, xR);
  if (face_eps == OR_FACE_EPS_EOS) faces_on_eos(e, nfxa, xL, xR);
  or_face_flux(gr, 0, riemann, e, m, xL, xR, Fx, &sx);
  or_reconstruct(gr, 1, recon, p, zL, zR);
  if (face_eps == OR_FACE_EPS_EOS) faces_on_eos(e, nfza, zL, zR);
  or_face_flux(gr, 1, riemann, e, m, zL, zR, Fz, &sz);
  /* 5. divergence and sources */
  or_rhs(gr, e, m, p, Fx, Fz, L);
  /* 6. Runge-Kutta stage combination */
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < nx; j++) {
      int64_t i = cidx(gr, j, k);
      for (int c = 0; c < 5; c++) {
        double v = st->b * qs[c][i] + st->c * st->dt * L[c][i];
        if (st->a != 0.0) v += st->a * qn[c][i];
        if (acc_in && st->g != 0.0) v += st->g * st->dt * acc_in[c][i];
        qout[c][i] = v;
        if (acc_out) {
          double av = st->e * L[c][i];
          if (acc_in && st->d != 0.0) av += st->d * acc_in[c][i];
          acc_out[c][i] = av;
        }
      }
    }
  if (p_out)
    for (int k = 0; k < nz; k++)
      for (int j = 0; j < nx; j++) {
        int64_t i = cidx(gr, j, k);
        for (int c = 0; c < 6; c++) p_out[c][i] = p[c][i];
      }
  /* 7. boundary-face fluxes (flux register) */
  if (flux_reg) {
    int64_t nb = 2 * (int64_t)nz + 2 * (int64_t)nx;
    for (int c = 0; c < 5; c++) {
      for (int k = 0; k < nz; k++) {
        flux_reg[c * nb + k] = Fx[c][(int64_t)k * (nx + 1)];
        flux_reg[c * nb + nz + k] = Fx[c][(int64_t)k * (nx + 1) + nx];
      }
      for (int j = 0; j < nx; j++) {
        flux_reg[c * nb + 2 * nz + j] = Fz[c][j];
        flux_reg[c * nb + 2 * nz + nx + j] = Fz[c][(int64_t)nz * nx + j];
      }
    }
  }
  /* 7b. refinement-boundary flux register (Sec. II.E): the time integral
   * of the flux through the L-shaped face set {x faces j = reg_j, k <
   * reg_k} + {z faces k = reg_k, j < reg_j}, accumulated with the stage's
   * weight in the Runge-Kutta step */
  if (reg) {
    int64_t nr = (int64_t)reg_k + reg_j;
    for (int c = 0; c < 5; c++) {
      for (int k = 0; k < reg_k; k++)
        reg[c * nr + k] += reg_w * st->dt * Fx[c][(int64_t)k * (nx + 1) + reg_j];
      for (int j = 0; j < reg_j; j++)
        reg[c * nr + reg_k + j] += reg_w * st->dt * Fz[c][(int64_t)reg_k * nx + j];
    }
  }
  /* 7c. every face flux, for registers on other face sets */
  if (fx_out)
    for (int c = 0; c < 5; c++) memcpy(fx_out[c], Fx[c], sizeof(double) * (size_t)nfxa);
  if (fz_out)
    for (int c = 0; c < 5; c++) memcpy(fz_out[c], Fz[c], sizeof(double) * (size_t)nfza);
  /* 8. diagnostics on the stage output */
  if (diag) {
    double cx = sx * st->dt / gr->dx, cz = sz * st->dt / gr->dz;
    dloc.max_courant = cx > cz ? cx : cz;
    double Mb = 0.0, J = 0.0;
    for (int k = 0; k < nz; k++)
      for (int j = 0; j < nx; j++) {
        int64_t i = cidx(gr, j, k);
        double dV = (gr->geom == OR_GEOM_CYL) ? 2.0 * M_PI * xc(gr, j) * gr->dx * gr->dz
                                              : gr->dx * gr->dz;
        Mb += qout[0][i] * dV;
        J += qout[2][i] * dV;
      }
    dloc.Mb = Mb;
    dloc.J = J;
    *diag = dloc;
  }
  free_fields(p, 6); free_fields(L, 5);
  free_fields(xL, 6); free_fields(xR, 6); free_fields(zL, 6); free_fields(zR, 6);
  free_fields(Fx, 5); free_fields(Fz, 5);
  return 0;
}
