// grhd_host.hpp -- host-side helpers shared by the library's translation
// units: argument validation, conversion of the public descriptors into
// kernel launch structs, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "grhd.h"
#include "grhd_dev.hpp"

namespace grhd {

void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

struct Q5 { double *q[5]; };
struct P6 { double *p[6]; };

inline bool bc_ok(int b) { return b >= GRHD_BC_OUTFLOW && b <= GRHD_BC_EXTERNAL; }

inline int check_grid(const grhd_grid *g) {
  if (!g) return fail(GRHD_ERR_INVALID, "grid is NULL");
  if (g->nx < 1 || g->nz < 1) return fail(GRHD_ERR_INVALID, "nx, nz must be >= 1 (got %d, %d)", g->nx, g->nz);
  if (g->ng != 3) return fail(GRHD_ERR_INVALID, "ng must be 3 (got %d)", g->ng);
  if (g->pitch < (int64_t)g->nx + 2 * g->ng)
    return fail(GRHD_ERR_INVALID, "pitch %lld < nx + 2 ng", (long long)g->pitch);
  if ((int64_t)(g->nz + 2 * g->ng) * g->pitch > ((int64_t)1 << 29))
    return fail(GRHD_ERR_INVALID, "a field holds at most 2^29 cells ((nz + 2 ng) pitch = %lld)",
                (long long)((int64_t)(g->nz + 2 * g->ng) * g->pitch));
  if (!(g->dx > 0.0) || !(g->dz > 0.0) || !std::isfinite(g->dx) || !std::isfinite(g->dz))
    return fail(GRHD_ERR_INVALID, "dx, dz must be finite and > 0");
  if (g->geom != GRHD_GEOM_CYLINDRICAL && g->geom != GRHD_GEOM_CARTESIAN)
    return fail(GRHD_ERR_INVALID, "bad geometry %d", g->geom);
  if (g->geom == GRHD_GEOM_CYLINDRICAL && !(g->x0 >= 0.0))
    return fail(GRHD_ERR_INVALID, "cylindrical grid needs x0 >= 0");
  for (int s = 0; s < 4; s++) {
    if (!bc_ok(g->bc[s])) return fail(GRHD_ERR_INVALID, "bad boundary condition %d on side %d", g->bc[s], s);
    if (g->bc[s] == GRHD_BC_AXIS && s != 0) return fail(GRHD_ERR_INVALID, "AXIS boundary only at x-low");
    int n = (s < 2) ? g->nx : g->nz;
    if ((g->bc[s] == GRHD_BC_AXIS || g->bc[s] == GRHD_BC_REFLECT) && n < 3)
      return fail(GRHD_ERR_INVALID, "mirror boundaries need >= 3 cells");
  }
  if ((g->bc[0] == GRHD_BC_PERIODIC) != (g->bc[1] == GRHD_BC_PERIODIC) ||
      (g->bc[2] == GRHD_BC_PERIODIC) != (g->bc[3] == GRHD_BC_PERIODIC))
    return fail(GRHD_ERR_INVALID, "periodic boundaries must be paired");
  if (g->geom == GRHD_GEOM_CYLINDRICAL && g->bc[0] == GRHD_BC_PERIODIC)
    return fail(GRHD_ERR_INVALID, "cylindrical grid cannot be periodic in x");
  return GRHD_OK;
}

inline GridK to_gridk(const grhd_grid *g) {
  GridK k;
  k.nx = g->nx; k.nz = g->nz; k.ng = g->ng; k.pitch = g->pitch;
  k.x0 = g->x0; k.z0 = g->z0; k.dx = g->dx; k.dz = g->dz;
  k.geom = g->geom;
  for (int s = 0; s < 4; s++) k.bc[s] = g->bc[s];
  return k;
}

inline int check_eos(const grhd_eos *e) {
  if (!e) return fail(GRHD_ERR_INVALID, "eos is NULL");
  if (e->kind != GRHD_EOS_IDEAL && e->kind != GRHD_EOS_HYBRID)
    return fail(GRHD_ERR_INVALID, "bad eos kind %d", e->kind);
  if (e->npieces < 1 || e->npieces > 8) return fail(GRHD_ERR_INVALID, "npieces must be 1..8");
  if (!(e->Gamma_th > 1.0)) return fail(GRHD_ERR_INVALID, "Gamma_th must be > 1");
  for (int i = 0; i < e->npieces; i++)
    if (!(e->Gamma[i] > 1.0) || !(e->K[i] > 0.0))
      return fail(GRHD_ERR_INVALID, "piece %d needs K > 0, Gamma > 1", i);
  for (int i = 0; i + 1 < e->npieces; i++)
    if (!(e->rho_b[i] > 0.0) || (i > 0 && !(e->rho_b[i] > e->rho_b[i - 1])))
      return fail(GRHD_ERR_INVALID, "rho_b must be positive and increasing");
  return GRHD_OK;
}

// Kernel EOS: derived constants (energy offsets of the pieces, atmosphere)
inline EosK to_eosk(const grhd_eos *e, double rho_atm) {
  EosK k{};
  k.kind = e->kind;
  k.n = e->npieces;
  for (int i = 0; i < 8; i++) {
    k.K[i] = e->K[i]; k.G[i] = e->Gamma[i]; k.rho_b[i] = e->rho_b[i]; k.deps[i] = 0.0;
  }
  k.Gth = e->Gamma_th;
  for (int i = 1; i < e->npieces; i++) {
    double rb = e->rho_b[i - 1];
    k.deps[i] = k.deps[i - 1] + e->K[i - 1] / (e->Gamma[i - 1] - 1.0) * std::pow(rb, e->Gamma[i - 1] - 1.0) -
                e->K[i] / (e->Gamma[i] - 1.0) * std::pow(rb, e->Gamma[i] - 1.0);
  }
  k.rho_atm = rho_atm;
  if (e->kind == GRHD_EOS_IDEAL) {
    k.P_atm = e->K[0] * std::pow(rho_atm, e->Gamma[0]);
    k.eps_atm = k.P_atm / ((e->Gamma_th - 1.0) * rho_atm);
  } else {
    int i = 0;
    while (i < e->npieces - 1 && rho_atm >= e->rho_b[i]) i++;
    k.P_atm = e->K[i] * std::pow(rho_atm, e->Gamma[i]);
    k.eps_atm = e->K[i] / (e->Gamma[i] - 1.0) * std::pow(rho_atm, e->Gamma[i] - 1.0) + k.deps[i];
  }
  // c_s^2 of the atmosphere state, the same expression as the device EOS
  const double gm1 = k.Gth - 1.0;
  double chi;
  if (k.kind == GRHD_EOS_IDEAL) {
    chi = gm1 * k.eps_atm;
  } else {
    int i = 0;
    while (i < k.n - 1 && rho_atm >= k.rho_b[i]) i++;
    const double kr = k.K[i] * std::pow(rho_atm, k.G[i] - 1.0);
    const double ec = kr / (k.G[i] - 1.0) + k.deps[i];
    chi = k.G[i] * kr + gm1 * (k.eps_atm - ec) - gm1 * kr;
  }
  const double h = 1.0 + k.eps_atm + k.P_atm / rho_atm;
  double cs2 = (chi + k.P_atm / rho_atm * gm1) / h;
  if (!(cs2 > 0.0)) cs2 = 0.0;
  if (cs2 > 0.999999) cs2 = 0.999999;
  k.cs_atm = std::sqrt(cs2);
  k.rhw2_atm = rho_atm * h;
  return k;
}

inline int check_c2p(const grhd_c2p_params *c) {
  if (!c) return fail(GRHD_ERR_INVALID, "c2p params are NULL");
  if (!(c->w_max > 1.0)) return fail(GRHD_ERR_INVALID, "w_max must be > 1");
  if (!(c->rho_atm > 0.0)) return fail(GRHD_ERR_INVALID, "rho_atm must be > 0");
  if (c->guess != GRHD_GUESS_NONE && c->guess != GRHD_GUESS_MLP)
    return fail(GRHD_ERR_INVALID, "bad guess mode");
  if (c->guess == GRHD_GUESS_MLP && !c->mlp) return fail(GRHD_ERR_INVALID, "MLP guess needs weights");
  return GRHD_OK;
}

inline int check_face_eps(int face_eps) {
  if (face_eps != GRHD_FACE_EPS_RECON && face_eps != GRHD_FACE_EPS_EOS)
    return fail(GRHD_ERR_INVALID, "bad face_eps");
  return GRHD_OK;
}

inline C2PK to_c2pk(const grhd_c2p_params *c) {
  C2PK k;
  double vmax = std::sqrt(1.0 - 1.0 / (c->w_max * c->w_max));
  k.kmax = 2.0 * vmax / (1.0 + vmax * vmax);
  k.tol = (c->tol > 0.0) ? c->tol : 1e-15;
  k.max_iter = (c->max_iter > 0) ? c->max_iter : 100;
  k.guess = c->guess;
  k.mlp = c->mlp;
  k.adiabatic = c->adiabatic ? 1 : 0;
  k.reuse_atm = 0;  // set by the entry points that take it
  return k;
}

inline MetK to_metk(const grhd_metric *m) {
  MetK k;
  for (int i = 0; i < GRHD_NMET; i++) { k.f[i] = m->f[i]; k.c[i] = m->cval[i]; }
  return k;
}

// conformally flat static class: only alpha and W may vary; shift zero,
// conformal metric identity, extrinsic curvature zero
inline int metric_class(const grhd_metric *m) {
  for (int i = GRHD_M_BX; i <= GRHD_M_BZ; i++)
    if (m->f[i] || m->cval[i] != 0.0) return MC_GEN;
  for (int i = GRHD_M_GXX; i <= GRHD_M_GZZ; i++) {
    double id = (i == GRHD_M_GXX || i == GRHD_M_GYY || i == GRHD_M_GZZ) ? 1.0 : 0.0;
    if (m->f[i] || m->cval[i] != id) return MC_GEN;
  }
  for (int i = GRHD_M_KXX; i <= GRHD_M_KZZ; i++)
    if (m->f[i] || m->cval[i] != 0.0) return MC_GEN;
  return MC_CF;
}

inline int check_metric(const grhd_metric *m) {
  if (!m) return fail(GRHD_ERR_INVALID, "metric is NULL");
  if (!m->f[GRHD_M_ALP] && !(m->cval[GRHD_M_ALP] > 0.0))
    return fail(GRHD_ERR_INVALID, "uniform lapse must be > 0");
  if (!m->f[GRHD_M_W] && !(m->cval[GRHD_M_W] > 0.0))
    return fail(GRHD_ERR_INVALID, "uniform W must be > 0");
  return GRHD_OK;
}

inline int check_cons(const grhd_cons *q, const char *what) {
  if (!q) return fail(GRHD_ERR_INVALID, "%s is NULL", what);
  for (int c = 0; c < 5; c++)
    if (!q->q[c]) return fail(GRHD_ERR_INVALID, "%s field %d is NULL", what, c);
  return GRHD_OK;
}

inline int check_prim(const grhd_prim *p, const char *what) {
  if (!p) return fail(GRHD_ERR_INVALID, "%s is NULL", what);
  for (int c = 0; c < 6; c++)
    if (!p->p[c]) return fail(GRHD_ERR_INVALID, "%s field %d is NULL", what, c);
  return GRHD_OK;
}

inline int launch_status(const char *what) {
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(GRHD_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(err));
  return GRHD_OK;
}

}  // namespace grhd
