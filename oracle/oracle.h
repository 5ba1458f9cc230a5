/*
 * oracle.h -- declarations of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * for the GPU hydro substep.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may link, load or call it.  It shares no
 * code, header, table or helper with the HIP library: everything below is
 * written again from the paper (Lam & Shibata, SACRA-2D, arXiv 2502.03223).
 *
 * Conventions (all restated here, nothing is imported):
 *  - cell-centred arrays, one array per field (SoA), row-major [z][x] with x
 *    fastest; every array carries ng ghost layers on each side, so cell
 *    (j,k), j in [-ng, nx+ng), k in [-ng, nz+ng), lives at
 *    (k+ng)*pitch + (j+ng);
 *  - x_j = x0 + (j+1/2) dx, z_k = z0 + (k+1/2) dz (x0, z0 = lower faces);
 *  - velocities are the covariant spatial components u_i of the
 *    four-velocity in the Cartesian basis at y = 0 (u_phi = x u_y);
 *  - conserved variables are densitised by psi^6 = W^-3, eq. (cons_var).
 */
#ifndef GRHD_ORACLE_H
#define GRHD_ORACLE_H

#include <stdint.h>

#define OR_NMET 17
/* metric field order: lapse, shift^i, W = psi^-2, conformal metric
 * (det = 1, lower indices), extrinsic curvature K_ij (lower indices) */
enum {
  OR_ALP = 0, OR_BX, OR_BY, OR_BZ, OR_W,
  OR_GXX, OR_GXY, OR_GXZ, OR_GYY, OR_GYZ, OR_GZZ,
  OR_KXX, OR_KXY, OR_KXZ, OR_KYY, OR_KYZ, OR_KZZ
};

enum { OR_GEOM_CYL = 0, OR_GEOM_CART = 1 };
enum { OR_BC_OUTFLOW = 0, OR_BC_PERIODIC = 1, OR_BC_AXIS = 2,
       OR_BC_REFLECT = 3, OR_BC_EXTERNAL = 4 };
/* PPM: CW84's interface form; PPM3: per-cell three-average parabola */
enum { OR_RECON_PPM = 0, OR_RECON_MINMOD = 1, OR_RECON_PPM3 = 2 };
enum { OR_RIEMANN_HLLC = 0, OR_RIEMANN_TVDLF = 1 };
/* face states of the stage: every primitive reconstructed (Sec. II.C.2,
 * the default), or eps taken from the EOS at the reconstructed (rho, P)
 * (a variant, not the paper's) */
enum { OR_FACE_EPS_RECON = 0, OR_FACE_EPS_EOS = 1 };
enum { OR_EOS_IDEAL = 0, OR_EOS_HYBRID = 1 };

/* con2prim flag bits */
#define OR_F_RESCALE 1u
#define OR_F_COLD    2u
#define OR_F_ATM     4u
#define OR_F_FAIL    8u

typedef struct {
  int nx, nz, ng;
  int64_t pitch;
  double x0, z0, dx, dz;
  int geom;
  int bc[4];               /* x-low, x-high, z-low, z-high */
} or_grid;

typedef struct {
  int kind;                /* OR_EOS_IDEAL or OR_EOS_HYBRID */
  int n;                   /* number of cold polytropic pieces (>= 1) */
  double K[8], G[8];       /* piece constants and adiabatic indices */
  double rho_b[8];         /* rho_b[i] = upper density bound of piece i */
  double Gth;              /* thermal index (IDEAL: the gamma-law index) */
} or_eos;

typedef struct {
  const double *f[OR_NMET];  /* NULL => the field is the constant c[] */
  double c[OR_NMET];
} or_metric;

typedef struct {
  double w_max, rho_atm;
  int adiabatic;           /* 1: zero temperature, the energy equation is
                              discarded (the cold root from D and S) */
} or_c2p;

typedef struct {
  double a, b, c, dt;      /* q_out = a q^n + b q_s + c dt L(q_s) + g dt acc */
  double g, d, e;          /* acc_out = d acc + e L(q_s) */
} or_stage;

typedef struct {
  double max_courant, Mb, J;
  unsigned long long n_rescale, n_cold, n_atm, n_fail;
} or_diag;

#ifdef __cplusplus
extern "C" {
#endif

/* pointwise EOS */
double or_eos_press(const or_eos *e, double rho, double eps);
double or_eos_eps(const or_eos *e, double rho, double P);
double or_eos_eps_cold(const or_eos *e, double rho);
double or_eos_press_cold(const or_eos *e, double rho);
double or_eos_cs2(const or_eos *e, double rho, double eps, double P);

/* pointwise state conversions; metric values g[OR_NMET] at the point */
void or_prim2con_point(const or_eos *e, const double *g, double x, int geom,
                       const double *p /*6*/, double *q /*5*/);
unsigned or_con2prim_point(const or_eos *e, const double *g, double x, int geom,
                           const or_c2p *cp, double *q /*5 in/out*/,
                           double *p /*6 out*/, double *zroot);
double or_c2p_master(const or_eos *e, double D, double qq, double r, double z);

/* pointwise fluxes: direction dir (0 = x, 1 = z), face metric g[] */
void or_valencia_flux_point(const or_eos *e, const double *g, int dir,
                            const double *p, double *F /*5*/);
void or_face_flux_point(const or_eos *e, const double *g, int dir, int riemann,
                        const double *pL, const double *pR, double *F /*5*/,
                        double *speed /* max |coordinate speed| or NULL */);
/* signal speeds of one state in direction dir, as coordinate speeds
 * dx^n/dt: from the 3+1 characteristic formula (used by TVDLF), and from
 * the face tetrad frame (used by HLLC) mapped back to coordinates */
void or_coord_speeds(const or_eos *e, const double *g, int dir,
                     const double *p, double *lm, double *lp);
void or_tetrad_speeds(const or_eos *e, const double *g, int dir,
                      const double *p, double *lm, double *lp);
/* pointwise source: metric values g[], first derivatives dg[2][OR_NMET]
 * (d/dx, d/dz) at the cell; geometric term added when geom is cylindrical */
void or_source_point(const or_eos *e, const double *g, const double *dg,
                     double x, int geom, const double *p, double *s /*5*/);

/* 1-D limited reconstruction of n cell values a[] into the left/right
 * states at the n-5 faces that have a full stencil (face i+1/2 for
 * i = 2 .. n-4): aL[i-2], aR[i-2] */
void or_recon_line(int recon, int n, const double *a, double *aL, double *aR);
double or_lagrange6(const double *a /* 6 consecutive cells */);
double or_deriv6(const double *a /* 7 consecutive cells */, double h);

/* grid-level operations */
void or_prim2con(const or_grid *gr, const or_eos *e, const or_metric *m,
                 double *const *p /*6*/, double *const *q /*5*/, int with_ghosts);
void or_con2prim(const or_grid *gr, const or_eos *e, const or_metric *m,
                 const or_c2p *cp, double *const *q, double *const *p,
                 uint8_t *flags, or_diag *diag);
void or_fill_ghosts(const or_grid *gr, double *const *p);
void or_reconstruct(const or_grid *gr, int dir, int recon,
                    double *const *p, double *const *pL, double *const *pR);
void or_face_flux(const or_grid *gr, int dir, int riemann, const or_eos *e,
                  const or_metric *m, double *const *pL, double *const *pR,
                  double *const *F, double *max_speed);
void or_rhs(const or_grid *gr, const or_eos *e, const or_metric *m,
            double *const *p, double *const *Fx, double *const *Fz,
            double *const *L);
int or_rk_substep(const or_grid *gr, const or_eos *e, const or_metric *m,
                  int recon, int riemann, int face_eps, const or_c2p *cp,
                  const or_stage *st,
                  double *const *qn, double *const *qs, double *const *qout,
                  double *const *p_out, double *const *acc_in,
                  double *const *acc_out, double *flux_reg, uint8_t *flags,
                  or_diag *diag);

/* the same substep, also adding reg_w dt F on the refinement-boundary
 * face set {x faces j = reg_j, k < reg_k} + {z faces k = reg_k, j < reg_j}
 * into reg (5 x (reg_k + reg_j): x faces by k, then z faces by j) */
int or_rk_substep_reg(const or_grid *gr, const or_eos *e, const or_metric *m,
                      int recon, int riemann, int face_eps, const or_c2p *cp,
                      const or_stage *st,
                      double *const *qn, double *const *qs, double *const *qout,
                      double *const *p_out, double *const *acc_in,
                      double *const *acc_out, double *flux_reg, uint8_t *flags,
                      or_diag *diag, double *reg, int reg_j, int reg_k, double reg_w,
                      double *const *fx_out /* 5 x nz x (nx+1), nullable */,
                      double *const *fz_out /* 5 x (nz+1) x nx, nullable */);

/* fixed mesh refinement between a parent level and its child, which
 * covers the parent cells [0, nx_c/2) x [0, nz_c/2) with half the spacing
 * (Sec. II.A, II.E).
 * prolong: the child's ghost cells on EXTERNAL sides (the cross-shaped
 * halo) and, with nbuf > 0, the child's last nbuf rows/columns of interior
 * cells next to each EXTERNAL side (the inner buffer of the (4+4) buffer
 * schedule) from the parent's primitives: time interpolation of nslice parent
 * slices (1: p_cur; 2: linear between t_cur and t_new; 3: quadratic over
 * t_old, t_cur, t_new, linear where the slices are not monotone) at time t,
 * then minmod-limited linear prolongation in space, then the conserved
 * variables from the primitives with the child's metric.
 * restrict: q_parent = sum(q_child dV_child) / dV_parent over each 2 x 2
 * block.  reflux: the parent cells just outside the child get the
 * difference of the child's and the parent's time-integrated fluxes through
 * the shared faces. */
void or_fmr_prolong(const or_grid *pg, double *const *p_old, double *const *p_cur,
                    double *const *p_new, int nslice, double t_old, double t_cur,
                    double t_new, double t, const or_grid *cg, const or_eos *e,
                    const or_metric *cm, int nbuf, double *const *cp /*6*/,
                    double *const *cq /*5*/);
void or_fmr_restrict(const or_grid *pg, double *const *pq, const or_grid *cg,
                     double *const *cq);
void or_fmr_reflux(const or_grid *pg, double *const *pq, const double *preg,
                   const or_grid *cg, const double *creg);

/* exact special-relativistic Riemann solver (ideal gas, no tangential
 * velocity); returns 0 on success, 1 if the solution contains vacuum */
int or_riemann_solve(double gam, double rhoL, double pL, double vL,
                     double rhoR, double pR, double vR, double *out /*12*/);
void or_riemann_sample(double gam, const double *sol, double xi,
                       double *rho, double *p, double *v);
int or_riemann_cellavg(double gam, double rhoL, double pL, double vL,
                       double rhoR, double pR, double vR, double xint, double t,
                       int n, const double *xface, int nsub,
                       double *rho, double *p, double *v);

/* MLP 3-64-64-1 with ReLU hidden units, FP64 forward/backward */
void or_mlp_forward(const double *params, int n, const double *X, double *y);
double or_mlp_loss_grad(const double *params, int n, const double *X,
                        const double *t, double *grad);

#ifdef __cplusplus
}
#endif
#endif
