// grhd_fmr.hip -- fixed mesh refinement between levels (Sec. II.A grid
// structure, Sec. II.E FMR setting): prolongation of primitives into a
// child's EXTERNAL ghost cells (time interpolation of the parent's slices,
// minmod-limited in space, conserved values built from the primitives),
// conservative restriction, refluxing with the flux registers the stage
// kernel accumulates, and the Berger-Oliger driver with l_fix sub-cycling.
//
// Layout: the nested, mirror-symmetric boxes of Sec. II.A.  A child starts
// at its parent's lower faces with half the spacing, so child cell (jf, kf)
// lies in parent cell (jf / 2, kf / 2); the child's high sides are
// EXTERNAL, its low sides are the parent's.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <vector>

#include "grhd.h"
#include "grhd_dev.hpp"
#include "grhd_host.hpp"
#include "grhd_tile.hpp"

namespace grhd {

int fill_patch(const grhd_grid *grid, const grhd_metric *metric, const grhd_rk_stage *stage,
               const grhd_cons *qn, const grhd_cons *qs, const grhd_cons *qout, const grhd_prim *p,
               const grhd_cons *acc_in, const grhd_cons *acc_out, double *flux_reg, int recon,
               int riemann, PatchK &pk);
int launch_con2prim_mlp_rect(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                             const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part, int jlo, int jhi,
                             int klo, int khi, hipStream_t st);
int launch_con2prim(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                    const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *diag, hipStream_t st);
int launch_substep(const PatchK &pk, const EosK &e, int prec, int mc, int shape, FluxPart *part2,
                   hipStream_t st);
int shape_index(int tx, int tz);
void shape_of(int s, int *tx, int *tz);

// parent primitive slices, oldest first, with the interpolation weights
// at the target time (computed on the host)
struct SliceK {
  const double *p[3][6];
  int ns;
  double wl;          // linear weight of the newest slice, (t - t_cur) / (t_new - t_cur)
  double l[3];        // quadratic Lagrange weights of the three slices
};

// Time interpolation of one value (slices oldest first): the current slice
// (1 slice), linear between the last two (2 slices), or the quadratic
// Lagrange polynomial through three, replaced by the linear one where the
// slices are not monotone.
__device__ __forceinline__ double slice_interp(const SliceK &S, const double *a) {
#pragma clang fp contract(off)
  if (S.ns == 1) return a[0];
  const int c = S.ns - 2, n = S.ns - 1;  // current, newest
  const double lin = a[c] + (a[n] - a[c]) * S.wl;
  if (S.ns == 2) return lin;
  if ((a[2] - a[1]) * (a[1] - a[0]) < 0.0) return lin;
  return S.l[0] * a[0] + S.l[1] * a[1] + S.l[2] * a[2];
}

// the parent's primitive field f at cell (j, k), with the parent's boundary
// conditions (index map and velocity parities)
__device__ __forceinline__ double parent_prim(const GridK &pg, const SliceK &S, int f, int j, int k) {
  int js, ks;
  double sg[3];
  ghost_map(pg, j, k, js, ks, sg);
  const long long i = cell_index(pg, js, ks);
  double a[3];
#pragma unroll
  for (int s = 0; s < 3; s++) a[s] = (s < S.ns) ? S.p[s][f][i] : 0.0;
  double v = slice_interp(S, a);
  if (f >= 1 && f <= 3) v *= sg[f - 1];
  return v;
}

__device__ __forceinline__ double minmod2(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// Number of child ghost cells on EXTERNAL sides (cross-shaped halo).
__host__ __device__ inline long long prolong_count(const GridK &cg) {
  long long n = 0;
  for (int s = 0; s < 4; s++)
    if (cg.bc[s] == GRHD_BC_EXTERNAL) n += (long long)cg.ng * (s < 2 ? cg.nz : cg.nx);
  return n;
}

// child ghost cell number id of the cross-shaped EXTERNAL halo (sides in
// order x-low, x-high, z-low, z-high); false past the last one
__device__ __forceinline__ bool ghost_cell(const GridK &cg, long long id, int &jf, int &kf) {
  for (int s = 0; s < 4; s++) {
    if (cg.bc[s] != GRHD_BC_EXTERNAL) continue;
    const long long len = (s < 2) ? cg.nz : cg.nx;
    const long long n = (long long)cg.ng * len;
    if (id < n) {
      const int m = (int)(id / len), r = (int)(id % len);
      if (s == 0) { jf = -1 - m; kf = r; }
      else if (s == 1) { jf = cg.nx + m; kf = r; }
      else if (s == 2) { jf = r; kf = -1 - m; }
      else { jf = r; kf = cg.nz + m; }
      return true;
    }
    id -= n;
  }
  return false;
}

// Number of the child's interior cells within nbuf of its EXTERNAL high
// sides (the inner buffer of the buffer schedule).
__host__ __device__ inline long long band_count(const GridK &cg, int nbuf) {
  if (nbuf <= 0) return 0;
  const bool xh = cg.bc[1] == GRHD_BC_EXTERNAL, zh = cg.bc[3] == GRHD_BC_EXTERNAL;
  return (xh ? (long long)nbuf * cg.nz : 0) + (zh ? (long long)nbuf * (xh ? cg.nx - nbuf : cg.nx) : 0);
}

// buffer cell number id: the nbuf columns next to the x-high side (every
// row), then the nbuf rows next to the z-high side (left of those columns)
__device__ __forceinline__ bool band_cell(const GridK &cg, int nbuf, long long id, int &jf, int &kf) {
  const bool xh = cg.bc[1] == GRHD_BC_EXTERNAL, zh = cg.bc[3] == GRHD_BC_EXTERNAL;
  if (xh) {
    const long long n = (long long)nbuf * cg.nz;
    if (id < n) {
      jf = cg.nx - nbuf + (int)(id % nbuf);
      kf = (int)(id / nbuf);
      return true;
    }
    id -= n;
  }
  if (zh) {
    const int w = xh ? cg.nx - nbuf : cg.nx;
    if (id < (long long)nbuf * w) {
      jf = (int)(id % w);
      kf = cg.nz - nbuf + (int)(id / w);
      return true;
    }
  }
  return false;
}

// cell number id of the prolonged frame: the EXTERNAL halo (if halo), then
// the buffer band (nbuf > 0)
__device__ __forceinline__ bool frame_cell(const GridK &cg, int halo, int nbuf, long long id, int &jf,
                                           int &kf) {
  if (halo) {
    const long long n = prolong_count(cg);
    if (id < n) return ghost_cell(cg, id, jf, kf);
    id -= n;
  }
  return nbuf > 0 && band_cell(cg, nbuf, id, jf, kf);
}

// One workgroup: 32 ghost cells x 6 fields, one (field, cell) per thread;
// the prolonged primitives meet in LDS for the conserved variables.
constexpr int PRO_CELLS = 32;

template <int MC>
__global__ void __launch_bounds__(PRO_CELLS * 6)
k_fmr_prolong(GridK pg, SliceK S, GridK cg, MetK cm, EosK e, P6 cp, Q5 cq) {
#pragma clang fp contract(off)
  __shared__ double spf[6][PRO_CELLS];
  const int f = threadIdx.x / PRO_CELLS, cl = threadIdx.x % PRO_CELLS;
  int jf = 0, kf = 0;
  const bool act = ghost_cell(cg, (long long)blockIdx.x * PRO_CELLS + cl, jf, kf);
  if (act) {
    const int jc = (jf >= 0) ? jf / 2 : -((1 - jf) / 2);
    const int kc = (kf >= 0) ? kf / 2 : -((1 - kf) / 2);
    const double ox = (cg.x0 + (jf + 0.5) * cg.dx) - (pg.x0 + (jc + 0.5) * pg.dx);
    const double oz = (cg.z0 + (kf + 0.5) * cg.dz) - (pg.z0 + (kc + 0.5) * pg.dz);
    const double a = parent_prim(pg, S, f, jc, kc);
    const double xp = parent_prim(pg, S, f, jc + 1, kc), xm = parent_prim(pg, S, f, jc - 1, kc);
    const double zp = parent_prim(pg, S, f, jc, kc + 1), zm = parent_prim(pg, S, f, jc, kc - 1);
    const double sx = minmod2(xp - a, a - xm) / pg.dx;
    const double sz = minmod2(zp - a, a - zm) / pg.dz;
    const double v = a + sx * ox + sz * oz;
    spf[f][cl] = v;
    cp.p[f][cell_index(cg, jf, kf)] = v;
  }
  __syncthreads();
  if (f == 0 && act) {
    const long long i = cell_index(cg, jf, kf);
    double pf[6];
    for (int c = 0; c < 6; c++) pf[c] = spf[c][cl];
    const double W = mval(cm, GRHD_M_W, i);
    double gtu[6];
    if (MC == MC_GEN) {
      double gt[6];
      for (int s = 0; s < 6; s++) gt[s] = mval(cm, GRHD_M_GXX + s, i);
      inv_sym3(gt, gtu);
    }
    double q[5];
    prim2con_cell<MC>(W, gtu, cg.x0 + (jf + 0.5) * cg.dx, cg.geom, pf, q);
    for (int c = 0; c < 5; c++) cq.q[c][i] = q[c];
  }
}

// A level stage's recovery with the prolongation of the level's frame in
// one launch.  Workgroups [0, nrec) recover the interior cells j < rnx,
// k < rnz (rows of 256 cells, row k = b / segs); the others take 32 frame
// cells each (the EXTERNAL halo if halo, then the nbuf-wide buffer band;
// 8 x 32 threads, fields 0-5 on the first six groups), prolong them as
// k_fmr_prolong does, form the conserved values and recover them in
// registers as the recovery launch would from memory: the same results as
// the two launches, without the second one.  The two sets are disjoint.
constexpr int PREP_THREADS = 256;

template <int MC, int EK>
__global__ void __launch_bounds__(PREP_THREADS)
k_fmr_prep(GridK pg, SliceK S, GridK cg, MetK cm, EosK e, C2PK cp, P6 pp, Q5 qq, uint8_t *flags, int segs,
           int nrec, int rnx, int halo, int nbuf) {
#pragma clang fp contract(off)
  __shared__ double spf[6][PRO_CELLS];
  const int b = blockIdx.x;
  if (b < nrec) {
    const int k = b / segs;
    const int j = (b % segs) * PREP_THREADS + threadIdx.x;
    if (j >= rnx) return;
    const long long i = cell_index(cg, j, k);
    const double W = mval(cm, GRHD_M_W, i);
    double gtu[6];
    if (MC == MC_GEN) {
      double gt[6];
      for (int t = 0; t < 6; t++) gt[t] = mval(cm, GRHD_M_GXX + t, i);
      inv_sym3(gt, gtu);
    }
    double q[5], p[6];
    for (int c = 0; c < 5; c++) q[c] = qq.q[c][i];
    const double q0[5] = {q[0], q[1], q[2], q[3], q[4]};
    const C2PResult r = con2prim_cell<MC, EK>(e, cp, W, gtu, cg.x0 + (j + 0.5) * cg.dx, cg.geom, q, p, -1.0);
    if (r.flags) store_corrected(q, q0, qq.q, i);
    for (int c = 0; c < 6; c++) pp.p[c][i] = p[c];
    if (flags) flags[i] = (uint8_t)r.flags;
    return;
  }
  const int f = threadIdx.x / PRO_CELLS, cl = threadIdx.x % PRO_CELLS;
  int jf = 0, kf = 0;
  const bool act = frame_cell(cg, halo, nbuf, (long long)(b - nrec) * PRO_CELLS + cl, jf, kf);
  if (act && f < 6) {
    const int jc = (jf >= 0) ? jf / 2 : -((1 - jf) / 2);
    const int kc = (kf >= 0) ? kf / 2 : -((1 - kf) / 2);
    const double ox = (cg.x0 + (jf + 0.5) * cg.dx) - (pg.x0 + (jc + 0.5) * pg.dx);
    const double oz = (cg.z0 + (kf + 0.5) * cg.dz) - (pg.z0 + (kc + 0.5) * pg.dz);
    const double a = parent_prim(pg, S, f, jc, kc);
    const double xp = parent_prim(pg, S, f, jc + 1, kc), xm = parent_prim(pg, S, f, jc - 1, kc);
    const double zp = parent_prim(pg, S, f, jc, kc + 1), zm = parent_prim(pg, S, f, jc, kc - 1);
    const double sx = minmod2(xp - a, a - xm) / pg.dx;
    const double sz = minmod2(zp - a, a - zm) / pg.dz;
    spf[f][cl] = a + sx * ox + sz * oz;
  }
  __syncthreads();
  if (f == 0 && act) {
    const long long i = cell_index(cg, jf, kf);
    double pf[6];
    for (int c = 0; c < 6; c++) pf[c] = spf[c][cl];
    const double W = mval(cm, GRHD_M_W, i);
    double gtu[6];
    if (MC == MC_GEN) {
      double gt[6];
      for (int t = 0; t < 6; t++) gt[t] = mval(cm, GRHD_M_GXX + t, i);
      inv_sym3(gt, gtu);
    }
    const double x = cg.x0 + (jf + 0.5) * cg.dx;
    double q[5], p[6];
    prim2con_cell<MC>(W, gtu, x, cg.geom, pf, q);
    // q is now what the prolongation stores; the recovery corrects it
    const C2PResult r = con2prim_cell<MC, EK>(e, cp, W, gtu, x, cg.geom, q, p, -1.0);
    for (int c = 0; c < 5; c++) qq.q[c][i] = q[c];
    for (int c = 0; c < 6; c++) pp.p[c][i] = p[c];
    if (flags) flags[i] = (uint8_t)r.flags;
  }
}

__device__ __forceinline__ double cell_volume(const GridK &g, int j) {
  return (g.geom == GRHD_GEOM_CYLINDRICAL) ? 2.0 * M_PI * (g.x0 + (j + 0.5) * g.dx) * g.dx * g.dz
                                           : g.dx * g.dz;
}

// q_parent = sum(q_child dV_child) / dV_parent over each 2 x 2 block
__global__ void __launch_bounds__(256)
k_fmr_restrict(GridK pg, Q5 pq, GridK cg, Q5 cq) {
#pragma clang fp contract(off)
  const int J = cg.nx / 2, K = cg.nz / 2;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)J * K) return;
  const int jc = (int)(id % J), kc = (int)(id / J);
  const double Vc = cell_volume(pg, jc);
  const double V0 = cell_volume(cg, 2 * jc), V1 = cell_volume(cg, 2 * jc + 1);
  const long long i00 = cell_index(cg, 2 * jc, 2 * kc), i01 = cell_index(cg, 2 * jc, 2 * kc + 1);
  for (int c = 0; c < 5; c++) {
    double s = 0.0;
    s += cq.q[c][i00] * V0;
    s += cq.q[c][i00 + 1] * V1;
    s += cq.q[c][i01] * V0;
    s += cq.q[c][i01 + 1] * V1;
    pq.q[c][cell_index(pg, jc, kc)] = s / Vc;
  }
}

// parent cells next to the child: (J, k < K) across the x interface,
// (j < J, K) across the z interface
__global__ void __launch_bounds__(256)
k_fmr_reflux(GridK pg, Q5 pq, const double *preg, GridK cg, const double *creg) {
#pragma clang fp contract(off)
  const int J = cg.nx / 2, K = cg.nz / 2;
  const long long np = (long long)K + J, nc = (long long)cg.nz + cg.nx;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  const bool cyl = pg.geom == GRHD_GEOM_CYLINDRICAL;
  if (id < K) {
    const int k = id;
    const double a = cyl ? (pg.x0 + J * pg.dx) / ((pg.x0 + (J + 0.5) * pg.dx) * pg.dx) : 1.0 / pg.dx;
    const long long i = cell_index(pg, J, k);
    for (int c = 0; c < 5; c++) {
      const double fine = 0.5 * (creg[c * nc + 2 * k] + creg[c * nc + 2 * k + 1]);
      pq.q[c][i] += a * (fine - preg[c * np + k]);
    }
  } else if (id < K + J) {
    const int j = id - K;
    const long long i = cell_index(pg, j, K);
    const double xp = pg.x0 + (j + 0.5) * pg.dx;
    for (int c = 0; c < 5; c++) {
      double fine = 0.0;
      for (int a = 0; a < 2; a++) {
        const double w = cyl ? (cg.x0 + (2 * j + a + 0.5) * cg.dx) / (2.0 * xp) : 0.5;
        fine += w * creg[c * nc + cg.nz + 2 * j + a];
      }
      pq.q[c][i] += (fine - preg[c * np + K + j]) / pg.dz;
    }
  }
}

__global__ void k_fmr_zero(double *a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// ------------------------------------------------------------ host side

static int check_pair(const grhd_grid *pg, const grhd_grid *cg) {
  int rc;
  if ((rc = check_grid(pg)) || (rc = check_grid(cg))) return rc;
  if (pg->geom != cg->geom) return fail(GRHD_ERR_INVALID, "parent and child geometries differ");
  if ((cg->nx & 1) || (cg->nz & 1)) return fail(GRHD_ERR_INVALID, "child nx, nz must be even");
  if (std::fabs(cg->dx * 2.0 - pg->dx) > 1e-12 * pg->dx || std::fabs(cg->dz * 2.0 - pg->dz) > 1e-12 * pg->dz)
    return fail(GRHD_ERR_INVALID, "child spacing must be half the parent's");
  if (cg->x0 != pg->x0 || cg->z0 != pg->z0)
    return fail(GRHD_ERR_INVALID, "child must start at the parent's lower faces");
  if (pg->nx < cg->nx / 2 + 3 || pg->nz < cg->nz / 2 + 3)
    return fail(GRHD_ERR_INVALID, "parent must extend >= 3 cells beyond the child");
  if (cg->bc[0] != pg->bc[0] || cg->bc[2] != pg->bc[2])
    return fail(GRHD_ERR_INVALID, "child low sides must be the parent's low sides");
  if (cg->bc[1] != GRHD_BC_EXTERNAL || cg->bc[3] != GRHD_BC_EXTERNAL)
    return fail(GRHD_ERR_INVALID, "child high sides must be EXTERNAL");
  return GRHD_OK;
}

// the time-interpolation weights at t for slice times ts[0..ns) (oldest
// first): linear between the last two, quadratic Lagrange through three
static void slice_weights(SliceK &S, const double *ts, double t) {
  S.wl = 0.0;
  S.l[0] = S.l[1] = S.l[2] = 0.0;
  if (S.ns >= 2) {
    const double tc = ts[S.ns - 2], tn = ts[S.ns - 1];
    S.wl = (t - tc) / (tn - tc);
  }
  if (S.ns == 3) {
    const double t0 = ts[0], t1 = ts[1], t2 = ts[2];
    S.l[0] = (t - t1) * (t - t2) / ((t0 - t1) * (t0 - t2));
    S.l[1] = (t - t0) * (t - t2) / ((t1 - t0) * (t1 - t2));
    S.l[2] = (t - t0) * (t - t1) / ((t2 - t0) * (t2 - t1));
  }
}

static SliceK make_slices(const grhd_prim *slices, int ns, const double *times, double t) {
  SliceK S{};
  S.ns = ns;
  for (int s = 0; s < ns; s++)
    for (int f = 0; f < 6; f++) S.p[s][f] = slices[s].p[f];
  slice_weights(S, times, t);
  return S;
}

static int prolong(const grhd_grid *pg, const SliceK &S, const grhd_grid *cg,
                   const grhd_metric *cm, const grhd_eos *eos, double rho_atm, const grhd_prim *pc,
                   const grhd_cons *qc, hipStream_t st) {
  GridK P = to_gridk(pg), Cg = to_gridk(cg);
  long long n = prolong_count(Cg);
  if (n == 0) return GRHD_OK;
  P6 pp;
  Q5 qq;
  for (int f = 0; f < 6; f++) pp.p[f] = pc->p[f];
  for (int c = 0; c < 5; c++) qq.q[c] = qc->q[c];
  EosK e = to_eosk(eos, rho_atm);
  dim3 grid((unsigned)((n + PRO_CELLS - 1) / PRO_CELLS)), block(PRO_CELLS * 6);
  if (metric_class(cm) == MC_GEN)
    hipLaunchKernelGGL(k_fmr_prolong<MC_GEN>, grid, block, 0, st, P, S, Cg, to_metk(cm), e, pp, qq);
  else
    hipLaunchKernelGGL(k_fmr_prolong<MC_CF>, grid, block, 0, st, P, S, Cg, to_metk(cm), e, pp, qq);
  return launch_status("fmr prolong");
}

// recovery of a child level's q_s (cells j < rnx, k < rnz) with its frame
// prolonged from the parent slices S (the EXTERNAL halo if halo, the
// nbuf-wide buffer band if nbuf > 0) in one launch (k_fmr_prep).  With the
// learned guess the cells j < rnx, k < rnz are recovered by the seeded
// recovery kernel first and k_fmr_prep prolongs and recovers the frame only
// (the two sets of cells are disjoint).
static int prep(const grhd_grid *pg, const SliceK &S, const grhd_level &L, const EosK &e, const C2PK &cp,
                const Q5 &q, const P6 &p, uint8_t *flags, int mc, int rnx, int rnz, int halo, int nbuf,
                hipStream_t st) {
  const GridK P = to_gridk(pg), Cg = to_gridk(&L.grid);
  const MetK m = to_metk(&L.metric);
  const bool seeded = cp.guess == GRHD_GUESS_MLP;
  if (seeded) {
    const int rc = launch_con2prim_mlp_rect(Cg, e, cp, m, mc, q, p, flags, nullptr, 0, rnx, 0, rnz, st);
    if (rc) return rc;
  }
  const int segs = (rnx + PREP_THREADS - 1) / PREP_THREADS;
  const long long nrec = seeded ? 0 : (long long)segs * rnz;
  const long long nframe = (halo ? prolong_count(Cg) : 0) + band_count(Cg, nbuf);
  const long long npro = (nframe + PRO_CELLS - 1) / PRO_CELLS;
  if (nrec + npro >= (1LL << 31)) return fail(GRHD_ERR_UNSUPPORTED, "level too large");
  if (nrec + npro == 0) return GRHD_OK;
  const dim3 grid((unsigned)(nrec + npro)), block(PREP_THREADS);
  const bool ideal = e.kind == GRHD_EOS_IDEAL;
  if (mc == MC_GEN) {
    if (ideal)
      hipLaunchKernelGGL((k_fmr_prep<MC_GEN, GRHD_EOS_IDEAL>), grid, block, 0, st, P, S, Cg, m, e, cp, p, q, flags,
                         segs, (int)nrec, rnx, halo, nbuf);
    else
      hipLaunchKernelGGL((k_fmr_prep<MC_GEN, GRHD_EOS_HYBRID>), grid, block, 0, st, P, S, Cg, m, e, cp, p, q,
                         flags, segs, (int)nrec, rnx, halo, nbuf);
  } else {
    if (ideal)
      hipLaunchKernelGGL((k_fmr_prep<MC_CF, GRHD_EOS_IDEAL>), grid, block, 0, st, P, S, Cg, m, e, cp, p, q, flags,
                         segs, (int)nrec, rnx, halo, nbuf);
    else
      hipLaunchKernelGGL((k_fmr_prep<MC_CF, GRHD_EOS_HYBRID>), grid, block, 0, st, P, S, Cg, m, e, cp, p, q,
                         flags, segs, (int)nrec, rnx, halo, nbuf);
  }
  return launch_status("fmr stage recovery and prolongation");
}

static int restrict_(const grhd_grid *pg, const grhd_cons *qp, const grhd_grid *cg, const grhd_cons *qc,
                     hipStream_t st) {
  Q5 a, b;
  for (int c = 0; c < 5; c++) { a.q[c] = qp->q[c]; b.q[c] = qc->q[c]; }
  long long n = (long long)(cg->nx / 2) * (cg->nz / 2);
  hipLaunchKernelGGL(k_fmr_restrict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, to_gridk(pg), a,
                     to_gridk(cg), b);
  return launch_status("fmr restrict");
}

static int reflux(const grhd_grid *pg, const grhd_cons *qp, const double *preg, const grhd_grid *cg,
                  const double *creg, hipStream_t st) {
  Q5 a;
  for (int c = 0; c < 5; c++) a.q[c] = qp->q[c];
  int n = cg->nx / 2 + cg->nz / 2;
  hipLaunchKernelGGL(k_fmr_reflux, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, to_gridk(pg), a,
                     preg, to_gridk(cg), creg);
  return launch_status("fmr reflux");
}

static int zero(double *a, long long n, hipStream_t st) {
  if (n <= 0) return GRHD_OK;
  hipLaunchKernelGGL(k_fmr_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n);
  return launch_status("fmr zero");
}

}  // namespace grhd

using namespace grhd;

extern "C" int grhd_fmr_prolong(const grhd_grid *parent, const grhd_prim *slices, int nslice,
                                const double *times, double t, const grhd_grid *child,
                                const grhd_metric *child_metric, const grhd_eos *eos, double rho_atm,
                                const grhd_prim *p_child, const grhd_cons *q_child, void *hip_stream) {
  int rc;
  if ((rc = check_pair(parent, child)) || (rc = check_metric(child_metric)) || (rc = check_eos(eos)) ||
      (rc = check_prim(p_child, "p_child")) || (rc = check_cons(q_child, "q_child")))
    return rc;
  if (!slices || !times || nslice < 1 || nslice > 3) return fail(GRHD_ERR_INVALID, "need 1-3 slices and times");
  for (int s = 0; s < nslice; s++)
    if ((rc = check_prim(&slices[s], "slice"))) return rc;
  for (int s = 0; s + 1 < nslice; s++)
    if (!(times[s + 1] > times[s])) return fail(GRHD_ERR_INVALID, "slice times must increase");
  if (!(rho_atm > 0.0)) return fail(GRHD_ERR_INVALID, "rho_atm must be > 0");
  return prolong(parent, make_slices(slices, nslice, times, t), child, child_metric, eos, rho_atm, p_child,
                 q_child, (hipStream_t)hip_stream);
}

extern "C" int grhd_fmr_restrict(const grhd_grid *parent, const grhd_cons *q_parent, const grhd_grid *child,
                                 const grhd_cons *q_child, void *hip_stream) {
  int rc;
  if ((rc = check_pair(parent, child)) || (rc = check_cons(q_parent, "q_parent")) ||
      (rc = check_cons(q_child, "q_child")))
    return rc;
  return restrict_(parent, q_parent, child, q_child, (hipStream_t)hip_stream);
}

extern "C" int grhd_fmr_reflux(const grhd_grid *parent, const grhd_cons *q_parent, const double *reg_parent,
                               const grhd_grid *child, const double *reg_child, void *hip_stream) {
  int rc;
  if ((rc = check_pair(parent, child)) || (rc = check_cons(q_parent, "q_parent"))) return rc;
  if (!reg_parent || !reg_child) return fail(GRHD_ERR_INVALID, "registers are NULL");
  return reflux(parent, q_parent, reg_parent, child, reg_child, (hipStream_t)hip_stream);
}

// ------------------------------------------------------------ driver

struct grhd_fmr {
  std::vector<grhd_level> lev;
  grhd_eos eos;
  grhd_options opts;
  int l_fix = 0;
  double t = 0.0;
  // per level: slice buffers oldest..newest (indices into slice[]), count, times
  std::vector<std::array<int, 3>> order;
  std::vector<int> ns;
  std::vector<std::array<double, 3>> ts;
  int shape = 3;
  // per level: recovery flags of the stage recoveries (library-owned), so
  // the stage kernel takes its all-atmosphere tile path
  std::vector<uint8_t *> flags;
  ~grhd_fmr() {
    for (uint8_t *f : flags)
      if (f) (void)hipFree(f);
  }
};

namespace {

int recover(grhd_fmr *h, int l, const grhd_prim *dst, hipStream_t st) {
  const grhd_level &L = h->lev[l];
  Q5 q;
  P6 p;
  for (int c = 0; c < 5; c++) q.q[c] = L.q.q[c];
  for (int f = 0; f < 6; f++) p.p[f] = dst->p[f];
  return launch_con2prim(to_gridk(&L.grid), to_eosk(&h->eos, h->opts.c2p.rho_atm), to_c2pk(&h->opts.c2p),
                         to_metk(&L.metric), metric_class(&L.metric), q, p, nullptr, nullptr, st);
}

// a new newest slice of level l at time t (the oldest buffer is reused)
int push_slice(grhd_fmr *h, int l, double t, hipStream_t st) {
  auto &o = h->order[l];
  auto &T = h->ts[l];
  int &n = h->ns[l];
  int buf;
  if (n < 3) {
    buf = o[n];
    T[n] = t;
    n++;
  } else {
    buf = o[0];
    o[0] = o[1]; o[1] = o[2]; o[2] = buf;
    T[0] = T[1]; T[1] = T[2]; T[2] = t;
  }
  return recover(h, l, &h->lev[l].slice[buf], st);
}

// level l without its buffer (same arrays and pitch)
grhd_grid own_grid(const grhd_level &L) {
  grhd_grid g = L.grid;
  g.nx -= L.nbuf;
  g.nz -= L.nbuf;
  return g;
}

int step_level(grhd_fmr *h, int l, double t, double dt, hipStream_t st) {
  int rc;
  const int nlev = (int)h->lev.size();
  grhd_level &L = h->lev[l];
  const bool has_child = l + 1 < nlev, has_parent = l > 0;
  const int nb = L.nbuf;
  const grhd_grid own = own_grid(L);
  const grhd_grid cown = has_child ? own_grid(h->lev[l + 1]) : own;
  if (has_child && (rc = zero(L.reg_parent_int, 5LL * (cown.nx / 2 + cown.nz / 2), st))) return rc;
  // SSP-RK3: (q^n, q_s, q_out) = (q, q, q1), (q, q1, q2), (q, q2, q)
  static const double kA[3] = {0.0, 0.75, 1.0 / 3.0}, kB[3] = {1.0, 0.25, 2.0 / 3.0},
                      kC[3] = {1.0, 0.25, 2.0 / 3.0}, kT[3] = {0.0, 1.0, 0.5},
                      kW[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  const grhd_cons *qs_of[3] = {&L.q, &L.q1, &L.q2}, *qo_of[3] = {&L.q1, &L.q2, &L.q};
  EosK e = to_eosk(&h->eos, h->opts.c2p.rho_atm);
  const int mc = metric_class(&L.metric);
  for (int s = 0; s < 3; s++) {
    // buffer schedule: the last stage updates the own cells only
    const bool last_on_own = nb > 0 && s == 2;
    const grhd_grid &gs = last_on_own ? own : L.grid;
    // the parent's slices at the stage time (frame of this level)
    SliceK S{};
    if (has_parent) {
      const grhd_level &Pl = h->lev[l - 1];
      S.ns = h->ns[l - 1];
      for (int i = 0; i < S.ns; i++)
        for (int f = 0; f < 6; f++) S.p[i][f] = Pl.slice[h->order[l - 1][i]].p[f];
      slice_weights(S, h->ts[l - 1].data(), t + kT[s] * dt);
    }
    grhd_rk_stage stg{};
    stg.a = kA[s]; stg.b = kB[s]; stg.c = kC[s]; stg.dt = dt;
    PatchK pk;
    if ((rc = fill_patch(&gs, &L.metric, &stg, &L.q, qs_of[s], qo_of[s], &L.p, nullptr, nullptr, nullptr,
                         h->opts.recon, h->opts.riemann, pk)))
      return rc;
    pk.face_eos = h->opts.face_eps == GRHD_FACE_EPS_EOS ? 1 : 0;
    pk.flags = h->flags[l];
    if (has_parent) { pk.reg[0] = L.reg_child_bnd; pk.reg_j[0] = own.nx; pk.reg_k[0] = own.nz; }
    if (has_child) { pk.reg[1] = L.reg_parent_int; pk.reg_j[1] = cown.nx / 2; pk.reg_k[1] = cown.nz / 2; }
    pk.reg_w = kW[s];
    // grids of few 16 x 16 tiles (under two per workgroup slot of the
    // chip) take 16 x 7 tiles: twice the workgroups, half the latency of
    // the slowest (star) tile; larger ones 16 x 15
    const int shape = ((long long)((gs.nx + 15) / 16) * ((gs.nz + 15) / 16) < 1536)
                          ? shape_index(16, 7) : h->shape;
    int tx, tz;
    shape_of(shape, &tx, &tz);
    pk.xshift = tile_xshift(gs.ng, tx);
    pk.tiles_x = (gs.nx + pk.xshift + tx - 1) / tx;
    pk.tiles_z = (gs.nz + tz - 1) / tz;
    Q5 q;
    P6 p;
    for (int c = 0; c < 5; c++) q.q[c] = qs_of[s]->q[c];
    for (int f = 0; f < 6; f++) p.p[f] = L.p.p[f];
    // recovery of q_s; a child level's frame is prolonged in the same
    // launch: halo schedule, the ghost cells before every stage; buffer
    // schedule, buffer and ghost cells before the first stage (the own
    // cells recovered), the ghost cells before the second, nothing before
    // the last (the whole grid recovered: the own cells' stage reads the
    // buffer as its ghost cells)
    const int nx = L.grid.nx, nz = L.grid.nz;
    if (!has_parent)
      rc = launch_con2prim(pk.g, e, to_c2pk(&h->opts.c2p), pk.m, mc, q, p, h->flags[l], nullptr, st);
    else if (nb > 0 && s == 0)
      rc = prep(&h->lev[l - 1].grid, S, L, e, to_c2pk(&h->opts.c2p), q, p, h->flags[l], mc, own.nx, own.nz,
                1, nb, st);
    else
      rc = prep(&h->lev[l - 1].grid, S, L, e, to_c2pk(&h->opts.c2p), q, p, h->flags[l], mc, nx, nz,
                last_on_own ? 0 : 1, 0, st);
    if (rc) return rc;
    if ((rc = launch_substep(pk, e, h->opts.prec, mc, shape, nullptr, st))) return rc;
  }
  if (!has_child) return GRHD_OK;
  if ((rc = push_slice(h, l, t + dt, st))) return rc;
  const int nsub = (l + 1 <= h->l_fix) ? 1 : 2;
  for (int i = 0; i < nsub; i++)
    if ((rc = step_level(h, l + 1, t + i * (dt / nsub), dt / nsub, st))) return rc;
  grhd_level &C = h->lev[l + 1];
  if ((rc = restrict_(&L.grid, &L.q, &cown, &C.q, st))) return rc;
  if ((rc = reflux(&L.grid, &L.q, L.reg_parent_int, &cown, C.reg_child_bnd, st))) return rc;
  if ((rc = zero(C.reg_child_bnd, 5LL * (cown.nx + cown.nz), st))) return rc;
  // the newest slice is the corrected state at t + dt
  return recover(h, l, &L.slice[h->order[l][h->ns[l] - 1]], st);
}

}  // namespace

extern "C" int grhd_fmr_create(const grhd_level *levels, int nlev, const grhd_eos *eos, const grhd_options *opts,
                               int l_fix, double t0, grhd_fmr **out, void *hip_stream) {
  int rc;
  if (!out) return fail(GRHD_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!levels || nlev < 1) return fail(GRHD_ERR_INVALID, "need at least one level");
  if (!opts) return fail(GRHD_ERR_INVALID, "opts is NULL");
  if ((rc = check_eos(eos)) || (rc = check_c2p(&opts->c2p)) || (rc = check_face_eps(opts->face_eps)))
    return rc;
  if (opts->prec != GRHD_PREC_FP64 && opts->prec != GRHD_PREC_MIXED) return fail(GRHD_ERR_INVALID, "bad prec");
  if (l_fix < 0) return fail(GRHD_ERR_INVALID, "l_fix must be >= 0");
  for (int l = 0; l < nlev; l++) {
    const grhd_level &L = levels[l];
    if ((rc = check_grid(&L.grid)) || (rc = check_metric(&L.metric)) || (rc = check_cons(&L.q, "q")) ||
        (rc = check_cons(&L.q1, "q1")) || (rc = check_cons(&L.q2, "q2")) || (rc = check_prim(&L.p, "p")))
      return rc;
    if (l == 0 && L.nbuf != 0) return fail(GRHD_ERR_INVALID, "level 0 has no buffer (nbuf must be 0)");
    if (l > 0) {
      if (L.nbuf != 0 && (L.nbuf < L.grid.ng || L.nbuf > 8))
        return fail(GRHD_ERR_INVALID, "level %d: nbuf must be 0 or in [ng, 8]", l);
      if (L.nbuf != 0 && (L.grid.bc[0] == GRHD_BC_EXTERNAL || L.grid.bc[2] == GRHD_BC_EXTERNAL))
        return fail(GRHD_ERR_INVALID, "level %d: the buffer schedule needs non-EXTERNAL low sides", l);
      const grhd_grid po = own_grid(levels[l - 1]), co = own_grid(L);
      if (co.nx < 2 || co.nz < 2) return fail(GRHD_ERR_INVALID, "level %d: no own cells", l);
      // the own cells pair with the parent as a halo-schedule child; the
      // parent's own cells also cover the buffer's and ghosts' stencils
      if ((rc = check_pair(&po, &co))) return rc;
      if (po.nx < (L.grid.nx + L.grid.ng) / 2 + 2 || po.nz < (L.grid.nz + L.grid.ng) / 2 + 2)
        return fail(GRHD_ERR_INVALID, "level %d: the parent's own cells must cover the child's buffer", l);
      if (!L.reg_child_bnd) return fail(GRHD_ERR_INVALID, "level %d needs reg_child_bnd", l);
    }
    if (l + 1 < nlev) {
      for (int s = 0; s < 3; s++)
        if ((rc = check_prim(&L.slice[s], "slice"))) return rc;
      if (!L.reg_parent_int) return fail(GRHD_ERR_INVALID, "level %d needs reg_parent_int", l);
    }
  }
  grhd_fmr *h = new grhd_fmr();
  h->lev.assign(levels, levels + nlev);
  h->eos = *eos;
  h->opts = *opts;
  h->l_fix = l_fix;
  h->t = t0;
  h->order.assign(nlev, {0, 1, 2});
  h->ns.assign(nlev, 0);
  h->ts.assign(nlev, {0.0, 0.0, 0.0});
  h->shape = shape_index(16, 15);
  h->flags.assign(nlev, nullptr);
  for (int l = 0; l < nlev; l++) {
    const size_t fb = (size_t)(levels[l].grid.nz + 2 * levels[l].grid.ng) * (size_t)levels[l].grid.pitch;
    if (hipMalloc(&h->flags[l], fb) != hipSuccess || hipMemset(h->flags[l], 0, fb) != hipSuccess) {
      delete h;
      return fail(GRHD_ERR_DEVICE, "flag allocation failed");
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  for (int l = 0; l < nlev; l++) {
    if (l + 1 < nlev && (rc = push_slice(h, l, t0, st))) { delete h; return rc; }
    if (l > 0 && (rc = zero(levels[l].reg_child_bnd,
                            5LL * (levels[l].grid.nx + levels[l].grid.nz - 2 * levels[l].nbuf), st))) {
      delete h;
      return rc;
    }
  }
  *out = h;
  return GRHD_OK;
}

extern "C" int grhd_fmr_step(grhd_fmr *h, double dt0, void *hip_stream) {
  if (!h) return fail(GRHD_ERR_INVALID, "hierarchy is NULL");
  if (!(dt0 > 0.0) || !std::isfinite(dt0)) return fail(GRHD_ERR_INVALID, "dt must be finite and > 0");
  int rc = step_level(h, 0, h->t, dt0, (hipStream_t)hip_stream);
  if (rc) return rc;
  h->t += dt0;
  return GRHD_OK;
}

extern "C" int grhd_fmr_time(const grhd_fmr *h, double *t) {
  if (!h || !t) return fail(GRHD_ERR_INVALID, "NULL argument");
  *t = h->t;
  return GRHD_OK;
}

extern "C" int grhd_fmr_destroy(grhd_fmr *h) {
  if (!h) return fail(GRHD_ERR_INVALID, "hierarchy is NULL");
  // queued steps may still read the level flags
  if (hipDeviceSynchronize() != hipSuccess) return fail(GRHD_ERR_DEVICE, "hipDeviceSynchronize failed");
  delete h;
  return GRHD_OK;
}
