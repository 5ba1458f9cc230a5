/*
 * or_fmr.c -- oracle of the fixed-mesh-refinement operators between two
 * levels (Lam & Shibata, SACRA-2D, Sec. II.A grid structure and Sec. II.E
 * FMR setting).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops in the order the
 * paper describes the operations; nothing is fused or reordered beyond
 * what the definitions state.
 *
 * Layout of a parent-child pair (the nested, mirror-symmetric boxes of
 * Sec. II.A): both levels start at the same lower faces, the child has
 * half the spacing, so child cell (jf, kf) lies in parent cell
 * (jf / 2, kf / 2) and the child covers parent cells [0, nx_c/2) x
 * [0, nz_c/2).  The child's low sides are the parent's low sides (axis,
 * equator); its high sides are EXTERNAL and filled by prolongation.
 *
 * Readings (the paper names the methods, not every detail):
 *  - spatial prolongation: per field, the minmod of the one-sided parent
 *    differences in x and in z, each applied over the quarter-cell offset
 *    of the child centre from the parent centre (dimension by dimension);
 *  - time interpolation: the second-order Lagrange polynomial through the
 *    three parent slices, replaced by the linear one through (t^n, t^{n+1})
 *    where (p^{n+1} - p^n)(p^n - p^{n-1}) < 0; with fewer slices, linear
 *    (two) or the current slice (one);
 *  - the parent's own boundary conditions supply its ghost primitives
 *    (axis and equator parities), exactly as in the substep;
 *  - flux correction: the registers hold the time integral of each face
 *    flux over the level's step (sum over Runge-Kutta stages of the stage
 *    weight times dt times the flux); the parent cell next to the interface
 *    takes the area-weighted child integral in place of its own;
 *  - the (4+4) buffer schedule: the band of nbuf interior cells next to
 *    the child's EXTERNAL sides is prolonged together with the halo (at
 *    the start of a child step) and then evolved by the child's own
 *    stages; the schedule itself lives in the driver.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int64_t gidx(const or_grid *g, int j, int k) {
  return (int64_t)(k + g->ng) * g->pitch + (j + g->ng);
}
static double cx(const or_grid *g, int j) { return g->x0 + (j + 0.5) * g->dx; }
static double fx(const or_grid *g, int j) { return g->x0 + j * g->dx; }
static double cz(const or_grid *g, int k) { return g->z0 + (k + 0.5) * g->dz; }

static double mm(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

static double cell_volume(const or_grid *g, int j) {
  return g->geom == OR_GEOM_CYL ? 2.0 * M_PI * cx(g, j) * g->dx * g->dz : g->dx * g->dz;
}

/* time interpolation of one value (reading above) */
static double time_interp(int nslice, double a_old, double a_cur, double a_new, double t_old,
                          double t_cur, double t_new, double t) {
  if (nslice <= 1) return a_cur;
  double lin = a_cur + (a_new - a_cur) * ((t - t_cur) / (t_new - t_cur));
  if (nslice == 2) return lin;
  if ((a_new - a_cur) * (a_cur - a_old) < 0.0) return lin;
  double l0 = (t - t_cur) * (t - t_new) / ((t_old - t_cur) * (t_old - t_new));
  double l1 = (t - t_old) * (t - t_new) / ((t_cur - t_old) * (t_cur - t_new));
  double l2 = (t - t_old) * (t - t_cur) / ((t_new - t_old) * (t_new - t_cur));
  return l0 * a_old + l1 * a_cur + l2 * a_new;
}

void or_fmr_prolong(const or_grid *pg, double *const *p_old, double *const *p_cur,
                    double *const *p_new, int nslice, double t_old, double t_cur,
                    double t_new, double t, const or_grid *cg, const or_eos *e,
                    const or_metric *cm, int nbuf, double *const *cp, double *const *cq) {
  int64_t n = (int64_t)(pg->nz + 2 * pg->ng) * pg->pitch;
  /* 1. the parent's primitives at time t, every stored cell */
  double *pt[6];
  for (int c = 0; c < 6; c++) {
    pt[c] = (double *)calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < n; i++)
      pt[c][i] = time_interp(nslice, p_old ? p_old[c][i] : 0.0, p_cur[c][i],
                             p_new ? p_new[c][i] : 0.0, t_old, t_cur, t_new, t);
  }
  /* 2. the parent's boundary conditions on those primitives */
  or_fill_ghosts(pg, pt);
  /* 3. every child ghost cell of the cross-shaped halo on an EXTERNAL
   * side, and every interior cell within nbuf cells of an EXTERNAL side */
  int ng = cg->ng;
  for (int kf = -ng; kf < cg->nz + ng; kf++)
    for (int jf = -ng; jf < cg->nx + ng; jf++) {
      int jin = jf >= 0 && jf < cg->nx, kin = kf >= 0 && kf < cg->nz;
      if (!jin && !kin) continue; /* corner */
      if (jin && kin) {
        int band = (cg->bc[0] == OR_BC_EXTERNAL && jf < nbuf) ||
                   (cg->bc[1] == OR_BC_EXTERNAL && jf >= cg->nx - nbuf) ||
                   (cg->bc[2] == OR_BC_EXTERNAL && kf < nbuf) ||
                   (cg->bc[3] == OR_BC_EXTERNAL && kf >= cg->nz - nbuf);
        if (!band) continue;
      } else {
        int side = !jin ? (jf < 0 ? 0 : 1) : (kf < 0 ? 2 : 3);
        if (cg->bc[side] != OR_BC_EXTERNAL) continue;
      }
      int jc = (jf >= 0) ? jf / 2 : -((1 - jf) / 2);
      int kc = (kf >= 0) ? kf / 2 : -((1 - kf) / 2);
      double ox = cx(cg, jf) - cx(pg, jc), oz = cz(cg, kf) - cz(pg, kc);
      double pf[6];
      for (int c = 0; c < 6; c++) {
        double a = pt[c][gidx(pg, jc, kc)];
        double sx = mm(pt[c][gidx(pg, jc + 1, kc)] - a, a - pt[c][gidx(pg, jc - 1, kc)]) / pg->dx;
        double sz = mm(pt[c][gidx(pg, jc, kc + 1)] - a, a - pt[c][gidx(pg, jc, kc - 1)]) / pg->dz;
        pf[c] = a + sx * ox + sz * oz;
      }
      int64_t i = gidx(cg, jf, kf);
      double g[OR_NMET], q[5];
      for (int f = 0; f < OR_NMET; f++) g[f] = cm->f[f] ? cm->f[f][i] : cm->c[f];
      or_prim2con_point(e, g, cx(cg, jf), cg->geom, pf, q);
      for (int c = 0; c < 6; c++) cp[c][i] = pf[c];
      for (int c = 0; c < 5; c++) cq[c][i] = q[c];
    }
  for (int c = 0; c < 6; c++) free(pt[c]);
}

void or_fmr_restrict(const or_grid *pg, double *const *pq, const or_grid *cg,
                     double *const *cq) {
  for (int kc = 0; kc < cg->nz / 2; kc++)
    for (int jc = 0; jc < cg->nx / 2; jc++) {
      double Vc = cell_volume(pg, jc);
      for (int c = 0; c < 5; c++) {
        double s = 0.0;
        for (int b = 0; b < 2; b++)
          for (int a = 0; a < 2; a++)
            s += cq[c][gidx(cg, 2 * jc + a, 2 * kc + b)] * cell_volume(cg, 2 * jc + a);
        pq[c][gidx(pg, jc, kc)] = s / Vc;
      }
    }
}

void or_fmr_reflux(const or_grid *pg, double *const *pq, const double *preg,
                   const or_grid *cg, const double *creg) {
  int J = cg->nx / 2, K = cg->nz / 2;
  int64_t np = (int64_t)K + J, nc = (int64_t)cg->nz + cg->nx;
  int cyl = pg->geom == OR_GEOM_CYL;
  /* parent cells (J, k), k < K: their low x face is the interface */
  for (int k = 0; k < K; k++) {
    double a = cyl ? fx(pg, J) / (cx(pg, J) * pg->dx) : 1.0 / pg->dx;
    for (int c = 0; c < 5; c++) {
      double fine = 0.5 * (creg[c * nc + 2 * k] + creg[c * nc + 2 * k + 1]);
      pq[c][gidx(pg, J, k)] += a * (fine - preg[c * np + k]);
    }
  }
  /* parent cells (j, K), j < J: their low z face is the interface */
  for (int j = 0; j < J; j++)
    for (int c = 0; c < 5; c++) {
      double fine = 0.0;
      for (int a = 0; a < 2; a++) {
        double w = cyl ? cx(cg, 2 * j + a) / (2.0 * cx(pg, j)) : 0.5;
        fine += w * creg[c * nc + cg->nz + 2 * j + a];
      }
      pq[c][gidx(pg, j, K)] += (fine - preg[c * np + K + j]) / pg->dz;
    }
}
