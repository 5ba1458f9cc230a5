/*
 * or_riemann.c -- exact solution of the 1-D special-relativistic Riemann
 * problem for an ideal gas with no tangential velocity.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle.h).
 *
 * The paper checks its shock-tube run against the exact solution (Sec.
 * III.B.1); this is an independent implementation written from the
 * published method of Marti & Mueller (J. Fluid Mech. 258, 1994; Living
 * Rev. Relativ. 2003): the star pressure p* is the zero of
 * v*_L(p) - v*_R(p), where each side is joined to the star region either
 * by a shock (Taub adiabat, mass flux j, shock speed V_s) or by a
 * rarefaction (the Riemann invariant atanh(v) +- F(c_s) constant along the
 * fan, F(c) = ln[(sqrt(G-1)+c)/(sqrt(G-1)-c)]/sqrt(G-1) for an ideal gas).
 * p* is found by plain bisection to machine precision.
 *
 * Solution vector `sol` (16 doubles): [0..5] rhoL pL vL rhoR pR vR,
 * [6] p*, [7] v*, [8] rho*_L, [9] rho*_R, [10] left wave is a shock,
 * [11] right wave is a shock, [12] left head speed, [13] left tail speed,
 * [14] right tail speed, [15] right head speed.
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

static double enth(double g, double rho, double p) {
  return 1.0 + g / (g - 1.0) * p / rho;
}

static double csound(double g, double rho, double p) {
  return sqrt(g * p / (rho * enth(g, rho, p)));
}

static double rapid(double v) { return 0.5 * log((1.0 + v) / (1.0 - v)); }

static double Fc(double g, double c) {
  double s = sqrt(g - 1.0);
  return log((s + c) / (s - c)) / s;
}

/* post-wave velocity and density for side state a (sgn = -1 left, +1
 * right) at star pressure p */
static void wave_curve(double g, double rho, double pa, double va, int sgn,
                       double p, double *vb, double *rhob, double *Vs) {
  if (p > pa) {
    /* shock: Taub adiabat for h_b, then mass flux and shock speed */
    double ha = enth(g, rho, pa);
    double dp = p - pa;
    double A = (p + (g - 1.0) * pa) / (g * p);
    double B = (g - 1.0) * dp / (g * p);
    double C = -ha * ha - ha / rho * dp;
    double hb = (-B + sqrt(B * B - 4.0 * A * C)) / (2.0 * A);
    double rb = g * p / ((g - 1.0) * (hb - 1.0));
    double j2 = dp / (ha / rho - hb / rb);
    double jm = sqrt(j2);
    double Wa = 1.0 / sqrt(1.0 - va * va);
    double r2W2 = rho * rho * Wa * Wa;
    double vs = (r2W2 * va + sgn * jm * sqrt(j2 + rho * rho)) / (r2W2 + j2);
    double Ws = 1.0 / sqrt(1.0 - vs * vs);
    double j = sgn * jm;
    *vb = (ha * Wa * va + Ws * dp / j) /
          (ha * Wa + dp * (Ws * va / j + 1.0 / (rho * Wa)));
    *rhob = rb;
    *Vs = vs;
  } else {
    /* rarefaction along the isentrope p/rho^G = const */
    double rb = rho * pow(p / pa, 1.0 / g);
    double ca = csound(g, rho, pa);
    double cb = (p > 0.0) ? csound(g, rb, p) : 0.0;
    double ra = rapid(va) - sgn * (Fc(g, ca) - Fc(g, cb));
    *vb = tanh(ra);
    *rhob = rb;
    *Vs = 0.0;
  }
}

int or_riemann_solve(double gam, double rhoL, double pL, double vL,
                     double rhoR, double pR, double vR, double *sol) {
  double vbL, vbR, rb, vs;
  sol[0] = rhoL; sol[1] = pL; sol[2] = vL;
  sol[3] = rhoR; sol[4] = pR; sol[5] = vR;
  /* vacuum check: both rarefactions down to p = 0 */
  double cL = csound(gam, rhoL, pL), cR = (pR > 0.0) ? csound(gam, rhoR, pR) : 0.0;
  double v0L = tanh(rapid(vL) + Fc(gam, cL));
  double v0R = tanh(rapid(vR) - Fc(gam, cR));
  if (v0L <= v0R) return 1;
  /* bracket p* */
  double lo = 0.0, hi = (pL > pR ? pL : pR);
  if (hi <= 0.0) hi = 1.0;
  for (int it = 0; it < 400; it++) {
    wave_curve(gam, rhoL, pL, vL, -1, hi, &vbL, &rb, &vs);
    wave_curve(gam, rhoR, pR, vR, +1, hi, &vbR, &rb, &vs);
    if (vbL - vbR < 0.0) break;
    lo = hi;
    hi *= 2.0;
  }
  for (int it = 0; it < 2000; it++) {
    double mid = (lo > 0.0 && hi / lo > 4.0) ? sqrt(lo * hi) : lo + 0.5 * (hi - lo);
    if (lo == 0.0) mid = 0.5 * hi;
    if (!(mid > lo && mid < hi)) break;
    wave_curve(gam, rhoL, pL, vL, -1, mid, &vbL, &rb, &vs);
    wave_curve(gam, rhoR, pR, vR, +1, mid, &vbR, &rb, &vs);
    if (vbL - vbR > 0.0) lo = mid;
    else hi = mid;
    if (lo > 0.0 && (hi - lo) <= 1e-16 * hi) break;
  }
  double ps = 0.5 * (lo + hi);
  double rsL, rsR, VsL, VsR;
  wave_curve(gam, rhoL, pL, vL, -1, ps, &vbL, &rsL, &VsL);
  wave_curve(gam, rhoR, pR, vR, +1, ps, &vbR, &rsR, &VsR);
  double vsx = 0.5 * (vbL + vbR);
  sol[6] = ps; sol[7] = vsx; sol[8] = rsL; sol[9] = rsR;
  sol[10] = (ps > pL) ? 1.0 : 0.0;
  sol[11] = (ps > pR) ? 1.0 : 0.0;
  if (ps > pL) {
    sol[12] = VsL; sol[13] = VsL;
  } else {
    double c1 = csound(gam, rsL, ps);
    sol[12] = (vL - cL) / (1.0 - vL * cL);
    sol[13] = (vsx - c1) / (1.0 - vsx * c1);
  }
  if (ps > pR) {
    sol[14] = VsR; sol[15] = VsR;
  } else {
    double c1 = csound(gam, rsR, ps);
    sol[14] = (vsx + c1) / (1.0 + vsx * c1);
    sol[15] = (vR + cR) / (1.0 + vR * cR);
  }
  return 0;
}

/* state inside a rarefaction fan at similarity coordinate xi */
static void fan_state(double g, double rho, double pa, double va, int sgn,
                      double xi, double *rr, double *pp, double *vv) {
  double ca = csound(g, rho, pa);
  double Jc = rapid(va) + (sgn < 0 ? Fc(g, ca) : -Fc(g, ca));
  double K = pa / pow(rho, g);
  double lo = 0.0, hi = ca, c = 0.5 * ca, v = va;
  for (int it = 0; it < 300; it++) {
    c = 0.5 * (lo + hi);
    v = (sgn < 0) ? (xi + c) / (1.0 + xi * c) : (xi - c) / (1.0 - xi * c);
    double res = rapid(v) + (sgn < 0 ? Fc(g, c) : -Fc(g, c)) - Jc;
    /* left fan: res increases with c; right fan: res decreases with c */
    if ((sgn < 0) ? (res > 0.0) : (res < 0.0)) hi = c;
    else lo = c;
    if (hi - lo <= 1e-17) break;
  }
  double y = c * c / (1.0 - c * c / (g - 1.0));
  double r = pow(y / (g * K), 1.0 / (g - 1.0));
  *rr = r;
  *pp = K * pow(r, g);
  *vv = v;
}

void or_riemann_sample(double gam, const double *sol, double xi, double *rho,
                       double *p, double *v) {
  if (xi < sol[12]) {
    *rho = sol[0]; *p = sol[1]; *v = sol[2];
  } else if (xi < sol[13]) {
    fan_state(gam, sol[0], sol[1], sol[2], -1, xi, rho, p, v);
  } else if (xi < sol[7]) {
    *rho = sol[8]; *p = sol[6]; *v = sol[7];
  } else if (xi < sol[14]) {
    *rho = sol[9]; *p = sol[6]; *v = sol[7];
  } else if (xi < sol[15]) {
    fan_state(gam, sol[3], sol[4], sol[5], +1, xi, rho, p, v);
  } else {
    *rho = sol[3]; *p = sol[4]; *v = sol[5];
  }
}

int or_riemann_cellavg(double gam, double rhoL, double pL, double vL,
                       double rhoR, double pR, double vR, double xint, double t,
                       int n, const double *xface, int nsub, double *rho,
                       double *p, double *v) {
  double sol[16];
  if (or_riemann_solve(gam, rhoL, pL, vL, rhoR, pR, vR, sol)) return 1;
  for (int i = 0; i < n; i++) {
    double a = xface[i], b = xface[i + 1];
    double sr = 0.0, sp = 0.0, sv = 0.0;
    for (int s = 0; s < nsub; s++) {
      double x = a + (s + 0.5) * (b - a) / nsub;
      double r, pp, vv;
      or_riemann_sample(gam, sol, (x - xint) / t, &r, &pp, &vv);
      sr += r; sp += pp; sv += vv;
    }
    rho[i] = sr / nsub;
    p[i] = sp / nsub;
    v[i] = sv / nsub;
  }
  return 0;
}
