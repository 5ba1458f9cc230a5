/*
 * grhd.h -- C ABI of the MI355X GRHD substep library (libgrhd.so).
 *
 * The library advances the axisymmetric general-relativistic hydrodynamics
 * of Lam & Shibata, "SACRA-2D" (arXiv 2502.03223), Sec. II.C, by one
 * Runge-Kutta stage on a cylindrical (varpi, z) mesh at y = 0, with the
 * spacetime metric given as input fields (Cowling approximation).
 *
 * Conventions for every call:
 *  - All array pointers are DEVICE pointers owned by the caller.  The
 *    library never frees caller memory; the only library-owned objects are
 *    plans (explicit create/destroy).
 *  - Cell arrays: one FP64 array per field (SoA), row-major [z][x] with x
 *    fastest, ng ghost layers on every side: cell (j,k), j in [-ng, nx+ng),
 *    k in [-ng, nz+ng), is element (k+ng)*pitch + (j+ng).  ng must be 3.
 *    x_j = x0 + (j+1/2) dx, z_k = z0 + (k+1/2) dz (the paper's cell-centred
 *    grid, Sec. II.A).
 *  - Face arrays (x faces): element k*(nx+1) + j is the face x_{j-1/2},
 *    j = 0..nx, k = 0..nz-1.  (z faces): element k*nx + j is the face
 *    z_{k-1/2}, k = 0..nz, j = 0..nx-1.
 *  - Conserved variables (eq. cons_var) are densitised by psi^6 = W^-3:
 *    q = (D, S_x, S_phi, S_z, E), S_phi = x S_y in cylindrical geometry
 *    (S_y in Cartesian geometry).  Primitives p = (rho, u_x, u_y, u_z, P,
 *    eps) with u_i the covariant spatial four-velocity (Cartesian basis).
 *  - Calls are asynchronous on the caller's HIP stream (NULL = default
 *    stream); results are valid after the caller synchronises.  Every call
 *    validates its arguments before launching and returns a grhd_status; no
 *    exception or abort crosses the ABI.  grhd_last_error() explains the
 *    last failure of the calling thread.
 *  - Trouble in a single cell during primitive recovery is not a call
 *    error: it is reported through per-cell flags and the diag counters.
 *  - The single-patch calls never allocate: device scratch (the partial
 *    records of the diagnostics, and the recovery flags of a stage whose
 *    caller passes no flags array) lives in a caller-owned workspace, sized
 *    by grhd_workspace_bytes.  Calls that may run at the same time need
 *    separate workspaces.
 */
#ifndef GRHD_H
#define GRHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GRHD_OK = 0,
  GRHD_ERR_INVALID = -1,     /* bad argument: nothing was launched */
  GRHD_ERR_DEVICE = -2,      /* a HIP call or launch failed */
  GRHD_ERR_UNSUPPORTED = -3, /* valid but not implemented combination */
  GRHD_ERR_WORKSPACE = -4    /* the caller's workspace is missing or too
                                small for this call: nothing was launched */
} grhd_status;

enum { GRHD_GEOM_CYLINDRICAL = 0, GRHD_GEOM_CARTESIAN = 1 };
/* boundary conditions applied to primitives (AXIS only at x-low: u_x and
 * u_y odd; REFLECT: normal velocity odd; EXTERNAL: ghost cells of q are
 * supplied by the caller and recovered like interior cells) */
enum { GRHD_BC_OUTFLOW = 0, GRHD_BC_PERIODIC = 1, GRHD_BC_AXIS = 2,
       GRHD_BC_REFLECT = 3, GRHD_BC_EXTERNAL = 4 };
/* reconstruction of the face states (Sec. II.C.2, third-order PPM):
 * PPM    Colella & Woodward (1984): interface values from monotonised
 *        slopes, then the parabola limiter; no steepening or flattening.
 *        Where no limiter acts both sides of a face take the same value.
 * MINMOD linear slopes limited by minmod (the paper's prolongation limiter)
 * PPM3   each cell's parabola through its own and its two neighbours'
 *        averages (third order), edge values clipped to the range of the
 *        two averages meeting there, then the same parabola limiter; the
 *        two face states differ by a sixth of the third difference across
 *        the face, the upwind dissipation that PPM's shared interface
 *        value lacks on smooth flows (Sec. III.B.2's second-order Bondi
 *        convergence holds with PPM3, not with PPM) */
enum { GRHD_RECON_PPM = 0, GRHD_RECON_MINMOD = 1, GRHD_RECON_PPM3 = 2 };
enum { GRHD_RIEMANN_HLLC = 0, GRHD_RIEMANN_TVDLF = 1 };
enum { GRHD_PREC_FP64 = 0, GRHD_PREC_MIXED = 1 };
/* face states of the stage: every primitive reconstructed, eps included
 * (Sec. II.C.2; the default), or eps from the EOS at the face's
 * reconstructed (rho, P) (a variant that keeps the face states on the EOS) */
enum { GRHD_FACE_EPS_RECON = 0, GRHD_FACE_EPS_EOS = 1 };
enum { GRHD_EOS_IDEAL = 0, GRHD_EOS_HYBRID = 1 };
enum { GRHD_GUESS_NONE = 0, GRHD_GUESS_MLP = 1 };
/* per-cell recovery flags */
enum { GRHD_FLAG_RESCALE = 1, GRHD_FLAG_COLD = 2, GRHD_FLAG_ATM = 4,
       GRHD_FLAG_FAIL = 8 };
/* metric field indices of grhd_metric */
enum { GRHD_M_ALP = 0, GRHD_M_BX, GRHD_M_BY, GRHD_M_BZ, GRHD_M_W,
       GRHD_M_GXX, GRHD_M_GXY, GRHD_M_GXZ, GRHD_M_GYY, GRHD_M_GYZ, GRHD_M_GZZ,
       GRHD_M_KXX, GRHD_M_KXY, GRHD_M_KXZ, GRHD_M_KYY, GRHD_M_KYZ, GRHD_M_KZZ,
       GRHD_NMET };

/* Cell-centred grid of one patch (Sec. II.A). */
typedef struct {
  int nx, nz, ng;         /* interior cells; ghosts (must be 3) */
  int64_t pitch;          /* row pitch in elements, >= nx + 2 ng; a field
                             holds at most 2^29 cells:
                             (nz + 2 ng) pitch <= 2^29 */
  double x0, z0, dx, dz;  /* lower faces of cell (0,0); spacings > 0 */
  int geom;               /* GRHD_GEOM_*; cylindrical needs x0 >= 0 */
  int bc[4];              /* x-low, x-high, z-low, z-high: GRHD_BC_* */
} grhd_grid;

/* Hybrid EOS of Sec. II.C.3: piecewise-polytropic cold part plus a
 * Gamma_th thermal part.  GRHD_EOS_IDEAL: P = (Gamma_th - 1) rho eps,
 * eps_min = 0; K[0], Gamma[0] then only set the atmosphere pressure
 * K[0] rho_atm^Gamma[0].  rho_b[i] is the upper density of piece i. */
typedef struct {
  int kind, npieces;
  double K[8], Gamma[8], rho_b[8];
  double Gamma_th;
} grhd_eos;

/* Metric fields (cell arrays with ghosts, read only).  NULL means the
 * field is the uniform value cval[i].  Order: lapse, shift^x,y,z,
 * W = psi^-2, conformal metric gt_xx,xy,xz,yy,yz,zz (det = 1),
 * extrinsic curvature K_xx..K_zz.  Ghost values are the caller's (the axis
 * parity of vector and tensor components is the caller's to apply). */
typedef struct {
  const double *f[GRHD_NMET];
  double cval[GRHD_NMET];
} grhd_metric;

typedef struct { double *q[5]; } grhd_cons;      /* D, S_x, S_phi, S_z, E */
typedef struct { double *p[6]; } grhd_prim;      /* rho, u_x, u_y, u_z, P, eps */

/* Primitive recovery parameters (Sec. II.C.4). */
typedef struct {
  double w_max;           /* Lorentz-factor limit (100): sets k_max */
  double rho_atm;         /* atmosphere density floor, > 0 */
  double tol;             /* relative root tolerance (<= 0: 1e-15) */
  int max_iter;           /* root-solver iteration cap (<= 0: 100) */
  int guess;              /* GRHD_GUESS_* */
  const void *mlp;        /* device weights for GRHD_GUESS_MLP (layout in
                             grhd_mlp_forward) */
  int adiabatic;          /* nonzero: the zero-temperature mode of
                             Sec. III.C.2 -- the energy equation is
                             discarded: every cell takes the cold root from
                             (D, S_i), its E is reset from the cold state
                             and it carries GRHD_FLAG_COLD */
  int reuse_atm;          /* nonzero: a cell whose entry in the caller's
                             flags array already carries GRHD_FLAG_ATM and
                             that is reset to the atmosphere again does not
                             rewrite its primitives.  Precondition: p holds
                             what the last recovery with this flags array
                             wrote (for such cells the atmosphere state of
                             the same rho_atm and EOS), or the flags are
                             zero.  p then ends exactly as with 0.  Taken by
                             grhd_con2prim and grhd_rk_substep with caller
                             flags and by grhd_rk_substep_chained (pair
                             p_out, flags_out); ignored elsewhere */
} grhd_c2p_params;

typedef struct {
  int recon, riemann, prec;   /* GRHD_RECON_*, GRHD_RIEMANN_*, GRHD_PREC_* */
  grhd_c2p_params c2p;
  int tile_x, tile_z;         /* 0, 0 = library default (16 x 15; 16 x 7
                                 on grids of fewer than 1536 tiles of
                                 16 x 16, 128 for the general metric
                                 class, and for general metrics with at
                                 least 8 of the 11 lapse, shift, W and
                                 conformal-metric fields as arrays: the
                                 16 x 7 and 16 x 8 general instances stage
                                 those fields in LDS).  Built: 16 x 15,
                                 16 x 7, 16 x 16, 16 x 8, 32 x 8, 32 x 16,
                                 64 x 8 */
  const uint8_t *fix_mask;    /* optional interior boundary condition
                                 (nullable; grhd_rk_substep and
                                 grhd_rk_substep_chained): on interior
                                 cells whose mask byte (cell array, layout
                                 of q) is nonzero the stage stores
                                 fix_q instead of its update, as
                                 grhd_fix_cells after the stage would */
  grhd_cons fix_q;
  void *ev_begin, *ev_end;    /* optional events from grhd_event_create,
                                 recorded on the stream right before and
                                 right after the fused stage kernel of
                                 grhd_rk_substep, so that kernel can be timed
                                 alone; NULL = not recorded (ignored by the
                                 batched plan) */
  int face_eps;               /* GRHD_FACE_EPS_* (0: the paper's) */
} grhd_options;

/* One Runge-Kutta stage:
 *   q_out   = a q^n + b q_s + c dt L(q_s) + g dt acc_in
 *   acc_out = d acc_in + e L(q_s)
 * SSP-RK3: (a,b,c) = (0,1,1), (3/4,1/4,1/4), (1/3,2/3,2/3), g = d = e = 0.
 * Classical RK4 uses the accumulator (see the library notes). */
typedef struct { double a, b, c, dt, g, d, e; } grhd_rk_stage;

/* Device-resident diagnostics, overwritten by each call that takes one. */
typedef struct {
  double max_courant;     /* max |coordinate signal speed| dt / spacing */
  double Mb, J;           /* sum q_D dV, sum q_Sphi dV of the output */
  unsigned long long n_rescale, n_cold, n_atm, n_fail;  /* flagged cells */
  unsigned long long iter_sum, iter_max;  /* root-solver master-function
                                             evaluations: total, worst cell */
} grhd_diag;

/* ---------------------------------------------------------------- calls */

/* Device workspace (bytes) that grhd_con2prim, grhd_rk_substep and
 * grhd_rk_substep_chained need on this grid with every option (diagnostics
 * on, no caller flags).  The workspace must be 256-byte aligned device
 * memory owned by the caller; each call uses the parts it needs and
 * returns GRHD_ERR_WORKSPACE, launching nothing, when they do not fit.  A
 * call without diag (and, for grhd_rk_substep, with caller flags) needs
 * none and takes NULL, 0. */
int grhd_workspace_bytes(const grhd_grid *grid, size_t *bytes);

/* Conservative-to-primitive recovery, Sec. II.C.4 (Galeazzi master
 * function f(z) = z - r / h(z) on [z-, z+], Illinois bracketed root, k
 * rescaling for w_max, zero-temperature recovery when eps < eps_min,
 * atmosphere floor).  Interior cells (plus EXTERNAL ghost strips).
 * q: in; rewritten from the recovered primitives where a flag is set.
 * p: out.  flags: nullable uint8 cell array.  diag: nullable (counters). */
int grhd_con2prim(const grhd_grid *grid, const grhd_eos *eos,
                  const grhd_metric *metric, const grhd_c2p_params *c2p,
                  const grhd_cons *q, const grhd_prim *p, uint8_t *flags,
                  grhd_diag *diag, void *workspace, size_t workspace_bytes,
                  void *hip_stream);

/* Primitive-to-conservative map, eq. (cons_var).  with_ghosts != 0 also
 * converts every ghost cell. */
int grhd_prim2con(const grhd_grid *grid, const grhd_eos *eos,
                  const grhd_metric *metric, const grhd_prim *p,
                  const grhd_cons *q, int with_ghosts, void *hip_stream);

/* Limited reconstruction of the primitives to the faces of direction dir
 * (0 = varpi/x, 1 = z), Sec. II.C.2: third-order PPM or minmod.  p holds
 * interior primitives; ghost values come from the boundary conditions
 * (EXTERNAL: from p's ghost cells).  pL, pR: face arrays of 6 fields, FP64
 * (prec = FP64) or FP32 (prec = MIXED; pointers then address float).
 * Every field is reconstructed, eps included, as in the stage
 * (grhd_rk_substep) unless its options select the EOS face variant. */
int grhd_reconstruct(const grhd_grid *grid, int dir, int recon, int prec,
                     const grhd_prim *p, const grhd_prim *pL,
                     const grhd_prim *pR, void *hip_stream);

/* Riemann flux at the faces of direction dir, Sec. II.C.2: HLLC in the
 * face tetrad frame (Mignone & Bodo) with the back-transform to the
 * Eulerian frame, or TVD Lax-Friedrichs.  Face metric by 6-point
 * interpolation.  F: densitised face flux of q, 5 FP64 face arrays; the
 * S_phi component carries the x factor (x of the face for x faces, of the
 * cell centre for z faces) in cylindrical geometry.  max_speed: nullable
 * device double, receives the largest |coordinate signal speed|. */
int grhd_hllc_flux(const grhd_grid *grid, int dir, int riemann, int prec,
                   const grhd_eos *eos, const grhd_metric *metric,
                   const grhd_prim *pL, const grhd_prim *pR,
                   const grhd_cons *F, double *max_speed, void *hip_stream);

/* One Runge-Kutta stage of the whole hot path, Sec. II.C.1: recovery of
 * q_s (corrected in place), ghost handling, reconstruction of rho, u_i, P
 * and eps to the faces (opts->face_eps selects the EOS variant), Riemann
 * fluxes in both directions, area-weighted divergence with the cylindrical
 * and metric source terms, stage combination.
 * qn: q^n (read only when stage->a != 0; may alias qs).  qs: in/out.
 * qout: out (interior cells; must not alias qs; may alias qn, each cell
 * reads its own q^n before its q_out is written).
 * p: required workspace and output: primitives of q_s (interior cells).
 * acc_in / acc_out: nullable accumulator cell arrays (RK4).
 * flux_reg: nullable, 5 x (2 nz + 2 nx) doubles: the q fluxes on the
 * x-low, x-high, z-low, z-high boundary faces (refluxing hook).
 * flags: nullable uint8 cell array (the recovery flags of q_s; without it
 * they go to the workspace).  diag: nullable.  workspace: see
 * grhd_workspace_bytes. */
int grhd_rk_substep(const grhd_grid *grid, const grhd_eos *eos,
                    const grhd_metric *metric, const grhd_options *opts,
                    const grhd_rk_stage *stage, const grhd_cons *qn,
                    const grhd_cons *qs, const grhd_cons *qout,
                    const grhd_prim *p, const grhd_cons *acc_in,
                    const grhd_cons *acc_out, double *flux_reg,
                    uint8_t *flags, grhd_diag *diag, void *workspace,
                    size_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * stage of grhd_rk_substep, same arguments and results, without a
 * workspace.  Its scratch (the diagnostic records, and the recovery flags
 * of q_s when flags is NULL) is a fixed device array of
 * GRHD_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until
 * the process ends; the call allocates nothing.  A grid whose scratch
 * needs more (grhd_workspace_bytes is an upper bound) returns
 * GRHD_ERR_WORKSPACE before launching anything.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be ordered by the caller. */
#define GRHD_NOALLOC_SCRATCH_BYTES (8 << 20)
int grhd_rk_substep_noalloc(const grhd_grid *grid, const grhd_eos *eos,
                            const grhd_metric *metric, const grhd_options *opts,
                            const grhd_rk_stage *stage, const grhd_cons *qn,
                            const grhd_cons *qs, const grhd_cons *qout,
                            const grhd_prim *p, const grhd_cons *acc_in,
                            const grhd_cons *acc_out, double *flux_reg,
                            uint8_t *flags, grhd_diag *diag, void *hip_stream);

/* The same stage with the recovery moved to its end (Sec. II.C.1 and
 * II.C.4 in one pass): the call takes the recovery of q_s as input and
 * leaves the recovery of q_out as output, so a sequence of stages needs
 * one recovery pass in total (grhd_con2prim before the first stage) and
 * each stage is a single kernel.  The arithmetic equals grhd_rk_substep's;
 * only where the recovery runs differs.
 * p_in, flags_in: primitives and recovery flags of q_s, as grhd_con2prim
 * or the previous chained stage wrote them (q_s already corrected);
 * flags_in is nullable (the atmosphere test then compares primitives).
 * p_out, flags_out: written with the recovery of q_out (interior cells);
 * q_out is stored corrected, as a recovery corrects it in place.  p_out
 * must not alias p_in, flags_out not flags_in.
 * diag: the recovery counts refer to q_out; Mb and J are sums of the
 * stored (corrected) q_out.  With c2p.guess = GRHD_GUESS_MLP the recovery
 * of q_out starts from the learned guess (each wave evaluates the network
 * for its cells at the end of the tile), except in tiles whose cells and
 * halo are all atmosphere, which recover as without it; the root is the
 * same to the solver's tolerance.  Tile shapes other than 16 x 15 and
 * EXTERNAL sides (whose ghosts would need a recovery of their own) return
 * GRHD_ERR_UNSUPPORTED.  Other arguments as grhd_rk_substep; ev_begin/
 * ev_end bracket the one kernel of the call. */
int grhd_rk_substep_chained(const grhd_grid *grid, const grhd_eos *eos,
                            const grhd_metric *metric, const grhd_options *opts,
                            const grhd_rk_stage *stage, const grhd_cons *qn,
                            const grhd_cons *qs, const grhd_cons *qout,
                            const grhd_prim *p_in, const uint8_t *flags_in,
                            const grhd_prim *p_out, uint8_t *flags_out,
                            const grhd_cons *acc_in, const grhd_cons *acc_out,
                            double *flux_reg, grhd_diag *diag, void *workspace,
                            size_t workspace_bytes, void *hip_stream);

/* ------------------------------------------------------------ batched path */

/* One patch of a batch: any mixture of refinement levels and independent
 * instances; each patch carries its own grid, metric, state and stage. */
typedef struct {
  grhd_grid grid;
  grhd_metric metric;
  grhd_cons qn, qs, qout;
  grhd_prim p;               /* required workspace/output per patch */
  grhd_rk_stage stage;
  int eos_id;                /* index into the plan's EOS table */
  double *flux_reg;          /* nullable */
} grhd_patch;

typedef struct grhd_plan grhd_plan;   /* opaque, library-owned */

/* Build a plan for a fixed set of patch shapes: tile shape (from tune_cache
 * if given and present, else measured and stored there), device patch and
 * work tables, launch configuration and the captured graph.  The options'
 * recovery may take the learned guess (GRHD_GUESS_MLP): the batched
 * recovery then evaluates the network on the matrix cores, as
 * grhd_con2prim does. */
int grhd_plan_create(const grhd_patch *patches, int npatch,
                     const grhd_eos *eos_table, int neos,
                     const grhd_options *opts, const char *tune_cache,
                     grhd_plan **out);

/* One substep of every patch in one graph-captured launch sequence
 * (recovery, then one kernel over all (patch, tile) items).
 * The patch array must have the shapes given at plan creation; pointers
 * and stage coefficients may change between calls. */
int grhd_batch_levels(grhd_plan *plan, const grhd_patch *patches, int npatch,
                      grhd_diag *diag, void *hip_stream);

int grhd_plan_destroy(grhd_plan *plan);

/* Tile shapes chosen for a plan (for reporting): tile_x[0], tile_z[0] =
 * square-ish patches, tile_x[1], tile_z[1] = thin patches (nz <= 8);
 * both arrays hold 2 ints. */
int grhd_plan_tile(const grhd_plan *plan, int *tile_x, int *tile_z);

/* The batched autotuner on its own: the tile shapes a plan for these
 * patches would use -- taken from tune_cache when it holds this GPU,
 * option set and patch-shape set, else measured by timing the candidate
 * shapes on the patches (their q_s is corrected in place and q_out
 * overwritten, as by grhd_plan_create) and stored there.  tile_x, tile_z:
 * 2 ints each, laid out as for grhd_plan_tile.  Explicit tile_x/tile_z in
 * opts are returned as they are.  Synchronous (library streams). */
int grhd_autotune(const grhd_patch *patches, int npatch, const grhd_eos *eos_table, int neos,
                  const grhd_options *opts, const char *tune_cache, int *tile_x, int *tile_z);

/* Interior boundary condition (the inner region of the Bondi test of
 * Sec. III.B.2 keeps its initial state): q = q_fixed on every interior
 * cell whose mask byte (cell array, same layout as q) is nonzero. */
int grhd_fix_cells(const grhd_grid *grid, const uint8_t *mask,
                   const grhd_cons *q_fixed, const grhd_cons *q,
                   void *hip_stream);

/* ------------------------------------------------------- mesh refinement */

/* Fixed mesh refinement, Sec. II.A and II.E.  Levels are the nested,
 * mirror-symmetric boxes of Sec. II.A: a child starts at its parent's lower
 * faces with half the spacing (child cell (jf, kf) lies in parent cell
 * (jf/2, kf/2)), has even nx, nz, the parent's low-side boundary
 * conditions, EXTERNAL high sides, and its parent extends at least 3 cells
 * beyond it.  Registers hold time integrals of face fluxes (in the flux
 * register form of grhd_rk_substep: S_phi component times x, E flux).
 * reg_child_bnd (levels with a parent): 5 x (nx + nz): the x-high faces by
 * k, then the z-high faces by j.  reg_parent_int (levels with a child):
 * 5 x (K + J) with J = nx_child/2, K = nz_child/2: the x faces j = J,
 * k < K, then the z faces k = K, j < J. */
typedef struct {
  grhd_grid grid;
  grhd_metric metric;
  grhd_cons q;               /* state (in/out) */
  grhd_cons q1, q2;          /* Runge-Kutta stage buffers */
  grhd_prim p;               /* recovery workspace */
  grhd_prim slice[3];        /* primitive time slices (levels with a child) */
  double *reg_child_bnd;     /* levels with a parent */
  double *reg_parent_int;    /* levels with a child */
  int nbuf;                  /* levels with a parent: 0 = halo schedule;
                                3..8 = buffer schedule with this inner
                                buffer width (the paper's (4+4): 4) */
} grhd_level;

typedef struct grhd_fmr grhd_fmr;   /* opaque, library-owned */

/* Prolongation into the child's EXTERNAL ghost cells (the cross-shaped
 * halo), Sec. II.E: the parent's primitives at time t from nslice slices
 * (oldest first, increasing times: 1 = the slice itself, 2 = linear, 3 =
 * second-order Lagrange, first order through the last two slices where
 * (p^{n+1} - p^n)(p^n - p^{n-1}) < 0), the parent's boundary conditions on
 * them, minmod-limited linear prolongation in space (per field, x and z
 * slopes over the child centre's offset), then the conserved variables
 * from the primitives with the child's metric (no recovery).  Writes
 * p_child and q_child ghost cells only.  rho_atm: atmosphere floor of the
 * EOS constants. */
int grhd_fmr_prolong(const grhd_grid *parent, const grhd_prim *slices, int nslice,
                     const double *times, double t, const grhd_grid *child,
                     const grhd_metric *child_metric, const grhd_eos *eos,
                     double rho_atm, const grhd_prim *p_child,
                     const grhd_cons *q_child, void *hip_stream);

/* Conservative restriction, Sec. II.E: every parent cell under the child
 * takes sum(q_child dV_child) / dV_parent of its 2 x 2 child cells. */
int grhd_fmr_restrict(const grhd_grid *parent, const grhd_cons *q_parent,
                      const grhd_grid *child, const grhd_cons *q_child,
                      void *hip_stream);

/* Flux correction, Sec. II.E: the parent cells just outside the child
 * (x interface: cells (J, k < K); z interface: cells (j < J, K)) replace
 * the parent's time-integrated flux through their low face by the child's
 * (area-weighted over the two child faces). */
int grhd_fmr_reflux(const grhd_grid *parent, const grhd_cons *q_parent,
                    const double *reg_parent, const grhd_grid *child,
                    const double *reg_child, void *hip_stream);

/* Berger-Oliger driver (Sec. II.E) over nlev levels (level 0 coarsest):
 * a level steps with SSP-RK3; levels l <= l_fix take the parent's step,
 * finer levels half of it; after a child's steps its parent is
 * restricted, refluxed and recovered.  A child's boundary follows one of
 * two schedules, per level:
 *  - halo (nbuf = 0): before each stage the child's ghost cells are
 *    prolonged from its parent's slices at the time of the stage's input
 *    state (t, t + dt, t + dt/2);
 *  - buffer (nbuf > 0; the paper's (4+4) structure with nbuf = 4): the
 *    level's grid holds nbuf cells beyond its own nx - nbuf by nz - nbuf
 *    cells on the high sides.  Before the first stage the buffer and the
 *    ghost cells beyond it are prolonged at t; the first two stages evolve
 *    own cells and buffer, the second after the ghost cells are prolonged
 *    at t + dt; the last stage updates the own cells only and reads the
 *    buffer as the second stage left it (the paper's RK4 mapping, every
 *    stage but the last on the wider domain, taken to SSP-RK3).  The
 *    3 ghost cells are the outer buffer the hydro stencils read.  The
 *    level's low sides must not be EXTERNAL.
 * Restriction, registers (reg_child_bnd: 5 x (own nx + own nz);
 * reg_parent_int: from the child's own cells) and flux correction concern
 * own cells; the parent's own cells must reach (child nx + 3)/2 + 2 cells
 * (nx of the child's grid, buffer included).  create: copies
 * the level descriptors (device buffers stay the caller's), recovers every
 * level with a child into its first slice.  step: one step dt0 of level 0
 * (all finer levels follow).  Single path kernels on 16 x 15 tiles (16 x 7
 * on grids of fewer than 1536 tiles of 16 x 16).  With opts->c2p.guess =
 * GRHD_GUESS_MLP every level's recovery of its evolved cells starts from
 * the learned guess (the prolonged frame of a child is recovered without
 * it).
 * The driver owns one recovery flag array per level (device memory, freed
 * by destroy, which first waits for the device to finish queued work). */
int grhd_fmr_create(const grhd_level *levels, int nlev, const grhd_eos *eos,
                    const grhd_options *opts, int l_fix, double t0,
                    grhd_fmr **out, void *hip_stream);
int grhd_fmr_step(grhd_fmr *h, double dt0, void *hip_stream);
int grhd_fmr_time(const grhd_fmr *h, double *t);
int grhd_fmr_destroy(grhd_fmr *h);

/* ---------------------------------------------------------- learned guess */

/* An added initial-guess model for the recovery of Sec. II.C.4 (not part
 * of the paper, which starts the Illinois iteration from the bracket of
 * its eq. for z-/z+): an MLP 3 -> 64 -> 64 -> 1 with ReLU hidden units.
 *   features  x = ((log10 D, S/E, log10((E - D)/D)) - mean) / std, with the
 *             undensitised D, E, S = sqrt(gamma^ij S_i S_j) of the cell;
 *   output    y = (log10(P/D) - mean_y) / std_y, so P0 = D 10^(y std_y + mean_y)
 *             gives v0 = S/(E + P0) and the starting point z0 = v0 W(v0)
 *             of a Newton iteration on the paper's master function kept
 *             inside the bracket (Illinois from the bracket when it leaves
 *             it or does not converge in 8 steps).
 * The guess only changes where the root search starts, never the root.
 *
 * Parameter vector (GRHD_MLP_NPARAM FP32): W1[64][3], b1[64], W2[64][64]
 * (row = output unit), b2[64], w3[64], b3.  The device weight buffer
 * (grhd_mlp_bytes() bytes, device memory owned by the caller) holds W1 and
 * W2 in BF16 (for the matrix cores), the vectors in FP32 and the eight
 * scalers (feature mean[3], std[3], target mean, std).  Pass it as
 * grhd_c2p_params.mlp with guess = GRHD_GUESS_MLP. */
#define GRHD_MLP_HIDDEN 64
#define GRHD_MLP_NPARAM 4481
size_t grhd_mlp_bytes(void);

/* Fill a weight buffer from FP32 params (device, NPARAM) and scal (device,
 * 8 floats; NULL keeps the scalers already in the buffer). */
int grhd_mlp_pack(void *mlp, const float *params, const float *scal,
                  void *hip_stream);

/* Network output for n standardised feature rows: X device n x 3 FP32
 * (row-major), y device n FP32 (the standardised output).  BF16 matrix
 * products with FP32 accumulation, as inside the recovery kernel. */
int grhd_mlp_forward(const void *mlp, const float *X, float *y, int n,
                     void *hip_stream);

/* Training data of the network: for n samples of densitised conserved
 * values of a flat Cartesian metric (q: five device arrays of n doubles),
 * X (device n x 3 doubles, row-major) receives the unscaled features
 * (log10 D, S/E, log10((E - D)/D)), S = |S_i|, and, when P (device n
 * doubles, the samples' pressures) and y are given, y the unscaled target
 * log10(P/D).  n >= 0; errors: GRHD_ERR_INVALID for NULL q fields or X. */
int grhd_mlp_features(const grhd_cons *q, long long n, const double *P,
                      double *X, double *y, void *hip_stream);

/* Gradient of the loss mean_i (y_i - t_i)^2 over n >= 1 samples at the FP32
 * params (W1, W2 rounded to BF16 as in the forward kernel, FP32
 * arithmetic): grad device NPARAM floats (overwritten), loss device float
 * (nullable, overwritten).  X, t standardised, device. */
int grhd_mlp_grad(const float *params, float *grad, const float *X,
                  const float *t, int n, float *loss, void *hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr, step
 * number step >= 1 for the bias correction) on a batch: params, m, v are
 * the FP32 master parameters and moments (device, NPARAM each), grad a
 * device workspace of NPARAM floats; the BF16 weights in mlp are refreshed
 * from the updated params (scalers kept). */
int grhd_mlp_train_step(void *mlp, float *params, float *m, float *v,
                        float *grad, const float *X, const float *t, int n,
                        float lr, int step, float *loss, void *hip_stream);

/* ---------------------------------------------------------------- timing */

/* A HIP event with timing enabled, for grhd_options.ev_begin/ev_end. */
int grhd_event_create(void **ev);
/* Milliseconds between two recorded events; waits for `end`. */
int grhd_event_elapsed_ms(void *begin, void *end, float *ms);
int grhd_event_destroy(void *ev);

/* ---------------------------------------------------------------- misc */
const char *grhd_last_error(void);
const char *grhd_version(void);

#ifdef __cplusplus
}
#endif
#endif
