// grhd_kernels.hip -- gfx950 kernels and the C ABI of the single-patch
// calls: primitive recovery, prim->con, reconstruction, Riemann flux and
// the fused Runge-Kutta stage.  Physics in grhd_dev.hpp, tile pipeline in
// grhd_tile.hpp.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "grhd.h"
#include "grhd_dev.hpp"
#include "grhd_host.hpp"
#include "grhd_tile.hpp"
#include "grhd_diag.hpp"

namespace grhd {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

// ------------------------------------------------------------ small kernels

// Fold of the diagnostic records into *diag.  Workgroup b of the first
// kernel folds the b-th contiguous chunk of each record array; one wave of
// the second folds the chunk results in a fixed order.  The chunk count
// is a function of the record counts, so the result depends on nothing
// else.
__device__ __forceinline__ void fold_chunk(int n, int nchunk, int b, int &lo, int &m) {
  const int c = (n + nchunk - 1) / nchunk;
  lo = b * c < n ? b * c : n;
  m = n - lo < c ? n - lo : c;
}

__global__ void __launch_bounds__(256)
k_diag_chunks(const C2PPart *p1, int n1, const FluxPart *p2, int n2, FoldPart *lvl) {
  __shared__ unsigned long long red[4][9];
  int lo1, m1, lo2, m2;
  fold_chunk(n1, gridDim.x, blockIdx.x, lo1, m1);
  fold_chunk(n2, gridDim.x, blockIdx.x, lo2, m2);
  FoldPart f = fold_records<256>(p1 + lo1, m1, p2 + lo2, m2, red);
  if (threadIdx.x == 0) lvl[blockIdx.x] = f;
}

__global__ void __launch_bounds__(64) k_diag_final(const FoldPart *lvl, int nchunk, grhd_diag *diag) {
  FoldPart f = fold_wave(lvl, nchunk);
  if (threadIdx.x == 0) {
    diag->max_courant = f.cmax;
    diag->Mb = f.mb;
    diag->J = f.jm;
    diag->n_rescale = f.n[0];
    diag->n_cold = f.n[1];
    diag->n_atm = f.n[2];
    diag->n_fail = f.n[3];
    diag->iter_sum = f.n[4];
    diag->iter_max = f.n[5];
  }
}

int launch_diag_final(const C2PPart *p1, int n1, const FluxPart *p2, int n2, FoldPart *lvl,
                      grhd_diag *diag, hipStream_t st) {
  // about one record of each array per thread, at most kFoldMax chunks
  const int n = n1 > n2 ? n1 : n2;
  int nchunk = (n + 255) / 256;
  nchunk = nchunk < 1 ? 1 : (nchunk > kFoldMax ? kFoldMax : nchunk);
  hipLaunchKernelGGL(k_diag_chunks, dim3(nchunk), dim3(256), 0, st, p1, n1, p2, n2, lvl);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, lvl, nchunk, diag);
  return launch_status("diag final");
}

__global__ void k_zero_double(double *d) {
  if (threadIdx.x == 0) *d = 0.0;
}

// The gamma-law, conformally flat recovery fits six waves per SIMD in
// registers without spilling (one more than unconstrained); the other
// instances would spill there.
template <int MC, int EK>
constexpr int con2prim_waves() {
  return (MC == MC_CF && EK == GRHD_EOS_IDEAL) ? 6 : 1;
}

// Recovery of one cell per thread over [jlo, jhi) x [klo, khi); cells
// outside the interior are processed only on EXTERNAL sides (corners never).
template <int MC, int EK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(con2prim_waves<MC, EK>())))
k_con2prim(GridK g, EosK e, C2PK cp, MetK m, Q5 q, P6 p, uint8_t *flags, C2PPart *part,
           int jlo, int jhi, int klo) {
  __shared__ unsigned long long red[4][6];
  int j = jlo + blockIdx.x * blockDim.x + threadIdx.x;
  int k = klo + blockIdx.y;
  bool act = j < jhi;
  bool jin = (j >= 0 && j < g.nx), kin = (k >= 0 && k < g.nz);
  if (!jin || !kin) {
    if (!jin && !kin) act = false;
    else if (!jin) act = act && g.bc[j < 0 ? 0 : 1] == GRHD_BC_EXTERNAL;
    else act = act && g.bc[k < 0 ? 2 : 3] == GRHD_BC_EXTERNAL;
  }
  unsigned fl = 0;
  int iters = 0;
  if (act) {
    const unsigned i = cell_idx32(g, j, k);
    double W = mval32(m, GRHD_M_W, i);
    double gtu[6];
    if (MC == MC_GEN) {
      double gt[6];
      for (int t = 0; t < 6; t++) gt[t] = mval32(m, GRHD_M_GXX + t, i);
      inv_sym3(gt, gtu);
    }
    double qq[5], pp[6];
    for (int c = 0; c < 5; c++) qq[c] = ld32(q.q[c], i);
    // flag of the last recovery into p (reuse_atm implies caller flags)
    const unsigned old = cp.reuse_atm ? (unsigned)ld32(flags, i) : 0u;
    double q0[5] = {qq[0], qq[1], qq[2], qq[3], qq[4]};
    double x = g.x0 + (j + 0.5) * g.dx;
    C2PResult r = con2prim_cell<MC, EK>(e, cp, W, gtu, x, g.geom, qq, pp, -1.0);
    fl = r.flags;
    iters = r.iters;
    if (fl) store_corrected(qq, q0, q.q, i);
    // a cell that was and stays atmosphere already holds its primitives
    if (!(old & fl & GRHD_FLAG_ATM))
      for (int c = 0; c < 6; c++) st32(p.p[c], i, pp[c]);
    if (flags) st32(flags, i, (uint8_t)fl);
  }
  if (part)
    c2p_block_partial<256>(act && jin && kin, fl, iters, &part[blockIdx.y * gridDim.x + blockIdx.x], red);
}

template <int MC>
__global__ void __launch_bounds__(256)
k_prim2con(GridK g, MetK m, P6 p, Q5 q, int lo) {
  int j = lo + blockIdx.x * blockDim.x + threadIdx.x;
  int k = lo + blockIdx.y;
  if (j >= g.nx - lo) return;
  long long i = cell_index(g, j, k);
  double W = mval(m, GRHD_M_W, i);
  double gtu[6];
  if (MC == MC_GEN) {
    double gt[6];
    for (int t = 0; t < 6; t++) gt[t] = mval(m, GRHD_M_GXX + t, i);
    inv_sym3(gt, gtu);
  }
  double pp[6], qq[5];
  for (int c = 0; c < 6; c++) pp[c] = p.p[c][i];
  prim2con_cell<MC>(W, gtu, g.x0 + (j + 0.5) * g.dx, g.geom, pp, qq);
  for (int c = 0; c < 5; c++) q.q[c][i] = qq[c];
}

template <class T> struct Ptr6 { T *a[6]; };

// Reconstruction at every face of one direction (one thread per face).
template <class T>
__global__ void __launch_bounds__(256)
k_reconstruct(GridK g, int dir, int recon, P6 p, Ptr6<T> L, Ptr6<T> R) {
  int nfx = (dir == 0) ? g.nx + 1 : g.nx;
  int nfz = (dir == 0) ? g.nz : g.nz + 1;
  long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= (long long)nfx * nfz) return;
  int j = (int)(f % nfx), k = (int)(f / nfx);
  T st[6][6];
  for (int i = 0; i < 6; i++) {
    int jj = (dir == 0) ? j - 3 + i : j;
    int kk = (dir == 0) ? k : k - 3 + i;
    int js, ks;
    double sg[3];
    ghost_map(g, jj, kk, js, ks, sg);
    long long is = cell_index(g, js, ks);
    st[0][i] = (T)p.p[0][is];
    st[1][i] = (T)(sg[0] * p.p[1][is]);
    st[2][i] = (T)(sg[1] * p.p[2][is]);
    st[3][i] = (T)(sg[2] * p.p[3][is]);
    st[4][i] = (T)p.p[4][is];
    st[5][i] = (T)p.p[5][is];
  }
  for (int c = 0; c < 6; c++) {
    T a, b;
    recon_face(recon, st[c], a, b);
    L.a[c][f] = a;
    R.a[c][f] = b;
  }
}

template <class T, int MC>
__global__ void __launch_bounds__(256)
k_flux(GridK g, EosK e, MetK m, int dir, int riemann, Ptr6<T> Lp, Ptr6<T> Rp, Q5 F,
       double *max_speed) {
  int nfx = (dir == 0) ? g.nx + 1 : g.nx;
  int nfz = (dir == 0) ? g.nz : g.nz + 1;
  long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double sp = 0.0;
  if (f < (long long)nfx * nfz) {
    int j = (int)(f % nfx), k = (int)(f / nfx);
    PrimT<T> L, R;
    L.rho = Lp.a[0][f]; L.u[0] = Lp.a[1][f]; L.u[1] = Lp.a[2][f]; L.u[2] = Lp.a[3][f];
    L.P = Lp.a[4][f]; L.eps = Lp.a[5][f];
    R.rho = Rp.a[0][f]; R.u[0] = Rp.a[1][f]; R.u[1] = Rp.a[2][f]; R.u[2] = Rp.a[3][f];
    R.P = Rp.a[4][f]; R.eps = Rp.a[5][f];
    FaceMet<T> fm;
    T t6[6];
    for (int fld = 0; fld < 11; fld++) {
      const double *src = m.f[fld];
      T v;
      if (src) {
        for (int i = 0; i < 6; i++) {
          long long ii = (dir == 0) ? cell_index(g, j - 3 + i, k) : cell_index(g, j, k - 3 + i);
          t6[i] = (T)src[ii];
        }
        v = lagrange6(t6);
      } else {
        v = (T)m.c[fld];
      }
      if (fld == 0) fm.alp = v;
      else if (fld < 4) fm.beta[fld - 1] = v;
      else if (fld == 4) fm.W = v;
      else fm.gt[fld - 5] = v;
    }
    FluxT<T> out;
    face_flux<T, MC>(e, fm, dir, riemann, L, R, out);
    double fv[5] = {(double)out.f[0], (double)out.f[1], (double)out.f[2], (double)out.f[3],
                    (double)out.f[0] + (double)out.f[4]};
    if (g.geom == GRHD_GEOM_CYLINDRICAL)
      fv[2] *= (dir == 0) ? g.x0 + j * g.dx : g.x0 + (j + 0.5) * g.dx;
    for (int c = 0; c < 5; c++) F.q[c][f] = fv[c];
    sp = (double)out.speed;
  }
  if (max_speed) {
    sp = wave_max(sp);
    if ((threadIdx.x & 63) == 0)
      atomicMax((unsigned long long *)max_speed, (unsigned long long)__double_as_longlong(sp));
  }
}

// Fused stage: one workgroup per tile, tile = workgroup index.  The
// hardware deals workgroups to the 8 XCDs round-robin by index, so each XCD
// takes every 8th tile of a tile row: any spatially smooth distribution of
// heavy tiles (stellar interior, shocks) spreads evenly over the XCDs, and
// when the tile row length is a multiple of 8 the tiles above and below a
// tile run on the same XCD (its z halo is then shared in that XCD's L2).
// Each tile writes one diagnostic record part2[tile]; a one-workgroup
// kernel folds the records afterwards.  (Handing tiles out through a global
// counter costs two same-address atomics per workgroup, which serialise
// across the XCDs and cost more than the imbalance they remove.)
// Waves per SIMD the register allocation must allow: the FP64 16-wide
// instances of the conformally flat class fit at least three workgroups per
// CU in LDS, so their registers are held to three waves; the FP32 16 x 16
// and 16 x 15 instances fit four (31 KB of LDS) and are held to four.
template <class T, int MC, int TX, int TZ>
constexpr int substep_waves() {
  return (sizeof(T) == 8 && MC == MC_CF && TX == 16 && TZ >= 7) ? 3
         : (sizeof(T) == 4 && MC == MC_CF && TX == 16 && TZ >= 15) ? 4
                                                                   : 1;
}

constexpr int CHAIN_TZ = 15;  // tiles of the chained stage: 16 x 15

// The chained instances: as above, except that the FP32 hybrid-EOS
// recovery would spill at four waves and stays unconstrained, the FP32
// ideal-gas instance takes three waves (at four it spills 56 B per lane;
// measured on the 1024^2 star 67.1 against 69.2 us per stage), and the
// instances with the learned guess take three waves (conformally flat) or
// two (general metric): unbounded, the compiler kept the network's operand
// fragments in 36-48 AGPRs on top of the VGPRs, a wave per SIMD less;
// bounded, the same work fits without spilling (the mixed chained form with
// the guess on the 1024^2 star: 1.25e10 against 1.0e10 zone-updates/s).
template <class T, int MC, int EK, bool ML>
constexpr int chain_waves() {
  return (sizeof(T) == 4 && EK != GRHD_EOS_IDEAL) ? 1
         : (ML && MC == MC_CF)                     ? 3
         : ML                                      ? 2
         : (sizeof(T) == 4 && MC == MC_CF)         ? 3
                                                   : substep_waves<T, MC, 16, CHAIN_TZ>();
}

template <class T, int MC, int TX, int TZ>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(substep_waves<T, MC, TX, TZ>())))
k_substep(PatchK P, EosK e, FluxPart *part2) {
  __shared__ TileSmem<T, MC, TX, TZ> sm;
  __shared__ double red[NT / 64][3];
  const int t = blockIdx.x;
  double cm, mb, jm;
  C2PAcc acc{};
  int tx, tz;
  tile_of(t, P.tiles_x, P.tiles_z, tx, tz);
  substep_tile<T, MC, TX, TZ>(P, e, tx, tz, sm, cm, mb, jm, acc);
  if (part2) flux_block_partial<NT>(cm, mb, jm, &part2[t], red);
}

// The chained stage: the same tile work on 16 x CHAIN_TZ tiles, ending with the
// recovery of q_out for the next stage (ML: seeded by the learned guess).
// Records: part1[tile] (recovery of q_out), part2[tile] (stage
// diagnostics).
template <class T, int MC, int EK, bool ML>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(chain_waves<T, MC, EK, ML>())))
k_substep_chain(PatchK P, EosK e, C2PPart *part1, FluxPart *part2) {
  __shared__ TileSmem<T, MC, 16, CHAIN_TZ> sm;
  __shared__ double red[NT / 64][3];
  __shared__ unsigned long long red1[NT / 64][6];
  const int t = blockIdx.x;
  double cm, mb, jm;
  C2PAcc acc{};
  int tx, tz;
  tile_of(t, P.tiles_x, P.tiles_z, tx, tz);
  substep_tile<T, MC, 16, CHAIN_TZ, true, EK, ML>(P, e, tx, tz, sm, cm, mb, jm, acc);
  if (part2) {
    flux_block_partial<NT>(cm, mb, jm, &part2[t], red);
    c2p_counts_partial<NT>(acc.n, &part1[t], red1);
  }
}

// ------------------------------------------------------------ dispatch

using SubstepFn = void (*)(PatchK, EosK, FluxPart *);

struct TileShape { int tx, tz; };
// 16 x 15 and 16 x 7 tiles have 511 and 247 faces: two (one) full passes of
// the 256 threads over the faces, where 16 x 16 (544) and 16 x 8 (280) leave
// a third (second) pass for a few faces
static const TileShape kShapes[] = {{32, 8}, {32, 16}, {64, 8}, {16, 16}, {16, 8}, {16, 15}, {16, 7}};
constexpr int kNumShapes = 7;

template <class T, int MC>
static SubstepFn pick_shape(int s) {
  switch (s) {
    case 0: return k_substep<T, MC, 32, 8>;
    case 1: return k_substep<T, MC, 32, 16>;
    case 2: return k_substep<T, MC, 64, 8>;
    case 4: return k_substep<T, MC, 16, 8>;
    case 5: return k_substep<T, MC, 16, 15>;
    case 6: return k_substep<T, MC, 16, 7>;
    default: return k_substep<T, MC, 16, 16>;
  }
}

static SubstepFn substep_kernel(int prec, int mc, int shape) {
  if (prec == GRHD_PREC_MIXED)
    return mc == MC_GEN ? pick_shape<float, MC_GEN>(shape) : pick_shape<float, MC_CF>(shape);
  return mc == MC_GEN ? pick_shape<double, MC_GEN>(shape) : pick_shape<double, MC_CF>(shape);
}

// The caller's device workspace of the single-patch calls, in 256-byte
// aligned parts: the fold's chunk results, the recovery records, the stage
// records and, for a stage whose caller passes no flags array, the recovery
// flags of q_s.  The library never allocates on these paths; a call whose
// parts do not fit the workspace it is given launches nothing and returns
// GRHD_ERR_WORKSPACE.
struct Workspace {
  FoldPart *lvl;
  C2PPart *p1;
  FluxPart *p2;
  uint8_t *flags;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of the parts: n1 recovery records, n2 stage records (both with the
// fold's chunk results when either is nonzero), nflag flag bytes.
static size_t ws_need(size_t n1, size_t n2, size_t nflag) {
  size_t o = 0;
  if (n1 || n2) {
    o += align256(sizeof(FoldPart) * kFoldMax);
    o += align256(sizeof(C2PPart) * n1);
    o += align256(sizeof(FluxPart) * n2);
  }
  o += align256(nflag);
  return o;
}

int ws_carve(void *ws, size_t bytes, size_t n1, size_t n2, size_t nflag, Workspace &w) {
  w = Workspace{nullptr, nullptr, nullptr, nullptr};
  const size_t need = ws_need(n1, n2, nflag);
  if (need == 0) return GRHD_OK;
  if (!ws) return fail(GRHD_ERR_WORKSPACE, "this call needs a workspace of %zu bytes (workspace is NULL)", need);
  if ((uintptr_t)ws % 256) return fail(GRHD_ERR_INVALID, "workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(GRHD_ERR_WORKSPACE, "workspace of %zu bytes is too small: this call needs %zu", bytes, need);
  char *c = (char *)ws;
  if (n1 || n2) {
    w.lvl = (FoldPart *)c;
    c += align256(sizeof(FoldPart) * kFoldMax);
    w.p1 = (C2PPart *)c;
    c += align256(sizeof(C2PPart) * n1);
    w.p2 = (FluxPart *)c;
    c += align256(sizeof(FluxPart) * n2);
  }
  if (nflag) w.flags = (uint8_t *)c;
  return GRHD_OK;
}

int shape_index(int tx, int tz) {
  for (int s = 0; s < kNumShapes; s++)
    if (kShapes[s].tx == tx && kShapes[s].tz == tz) return s;
  return -1;
}

int num_shapes() { return kNumShapes; }
void shape_of(int s, int *tx, int *tz) { *tx = kShapes[s].tx; *tz = kShapes[s].tz; }

template <int MC, int EK>
static void con2prim_launch(dim3 grid, hipStream_t st, const GridK &g, const EosK &e, const C2PK &cp,
                            const MetK &m, const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part,
                            int jlo, int jhi, int klo) {
  hipLaunchKernelGGL((k_con2prim<MC, EK>), grid, dim3(256), 0, st, g, e, cp, m, q, p, flags, part, jlo,
                     jhi, klo);
}

static int con2prim_blocks_of(const grhd_grid *g) {
  int jlo = (g->bc[0] == GRHD_BC_EXTERNAL) ? -g->ng : 0;
  int jhi = (g->bc[1] == GRHD_BC_EXTERNAL) ? g->nx + g->ng : g->nx;
  int klo = (g->bc[2] == GRHD_BC_EXTERNAL) ? -g->ng : 0;
  int khi = (g->bc[3] == GRHD_BC_EXTERNAL) ? g->nz + g->ng : g->nz;
  return ((jhi - jlo + 255) / 256) * (khi - klo);
}

// the most stage tiles any built shape makes of a grid
static long long max_stage_tiles(const grhd_grid *g) {
  long long m = 0;
  for (int s = 0; s < kNumShapes; s++) {
    const int tx = kShapes[s].tx, tz = kShapes[s].tz;
    const long long t = (long long)((g->nx + tile_xshift(g->ng, tx) + tx - 1) / tx) * ((g->nz + tz - 1) / tz);
    if (t > m) m = t;
  }
  return m;
}

int con2prim_blocks(const GridK &g) {
  int jlo = (g.bc[0] == GRHD_BC_EXTERNAL) ? -g.ng : 0;
  int jhi = (g.bc[1] == GRHD_BC_EXTERNAL) ? g.nx + g.ng : g.nx;
  int klo = (g.bc[2] == GRHD_BC_EXTERNAL) ? -g.ng : 0;
  int khi = (g.bc[3] == GRHD_BC_EXTERNAL) ? g.nz + g.ng : g.nz;
  return ((jhi - jlo + 255) / 256) * (khi - klo);
}

int launch_con2prim_mlp(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                        const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part, hipStream_t st);

int launch_con2prim(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                    const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *diag, hipStream_t st) {
  if (cp.guess == GRHD_GUESS_MLP) return launch_con2prim_mlp(g, e, cp, m, mc, q, p, flags, diag, st);
  int jlo = (g.bc[0] == GRHD_BC_EXTERNAL) ? -g.ng : 0;
  int jhi = (g.bc[1] == GRHD_BC_EXTERNAL) ? g.nx + g.ng : g.nx;
  int klo = (g.bc[2] == GRHD_BC_EXTERNAL) ? -g.ng : 0;
  int khi = (g.bc[3] == GRHD_BC_EXTERNAL) ? g.nz + g.ng : g.nz;
  dim3 grid((jhi - jlo + 255) / 256, khi - klo);
  bool ideal = e.kind == GRHD_EOS_IDEAL;
  if (mc == MC_GEN) {
    if (ideal) con2prim_launch<MC_GEN, GRHD_EOS_IDEAL>(grid, st, g, e, cp, m, q, p, flags, diag, jlo, jhi, klo);
    else con2prim_launch<MC_GEN, GRHD_EOS_HYBRID>(grid, st, g, e, cp, m, q, p, flags, diag, jlo, jhi, klo);
  } else {
    if (ideal) con2prim_launch<MC_CF, GRHD_EOS_IDEAL>(grid, st, g, e, cp, m, q, p, flags, diag, jlo, jhi, klo);
    else con2prim_launch<MC_CF, GRHD_EOS_HYBRID>(grid, st, g, e, cp, m, q, p, flags, diag, jlo, jhi, klo);
  }
  return launch_status("con2prim");
}

int launch_substep(const PatchK &pk, const EosK &e, int prec, int mc, int shape, FluxPart *part2,
                   hipStream_t st) {
  SubstepFn fn = substep_kernel(prec, mc, shape);
  long long nt = (long long)pk.tiles_x * pk.tiles_z;
  if (nt >= (1LL << 31)) return fail(GRHD_ERR_UNSUPPORTED, "more than 2^31 - 1 tiles");
  hipLaunchKernelGGL(fn, dim3((unsigned)nt), dim3(NT), 0, st, pk, e, part2);
  return launch_status("substep");
}

using ChainFn = void (*)(PatchK, EosK, C2PPart *, FluxPart *);

template <class T, bool ML>
static ChainFn chain_kernel_t(int mc, int ek) {
  if (mc == MC_GEN)
    return ek == GRHD_EOS_IDEAL ? k_substep_chain<T, MC_GEN, GRHD_EOS_IDEAL, ML>
                                : k_substep_chain<T, MC_GEN, GRHD_EOS_HYBRID, ML>;
  return ek == GRHD_EOS_IDEAL ? k_substep_chain<T, MC_CF, GRHD_EOS_IDEAL, ML>
                              : k_substep_chain<T, MC_CF, GRHD_EOS_HYBRID, ML>;
}

int launch_substep_chain(const PatchK &pk, const EosK &e, int prec, int mc, C2PPart *part1,
                         FluxPart *part2, hipStream_t st) {
  const bool ml = pk.cp.guess == GRHD_GUESS_MLP;
  ChainFn fn = (prec == GRHD_PREC_MIXED)
                   ? (ml ? chain_kernel_t<float, true>(mc, e.kind) : chain_kernel_t<float, false>(mc, e.kind))
                   : (ml ? chain_kernel_t<double, true>(mc, e.kind) : chain_kernel_t<double, false>(mc, e.kind));
  long long nt = (long long)pk.tiles_x * pk.tiles_z;
  if (nt >= (1LL << 31)) return fail(GRHD_ERR_UNSUPPORTED, "more than 2^31 - 1 tiles");
  hipLaunchKernelGGL(fn, dim3((unsigned)nt), dim3(NT), 0, st, pk, e, part1, part2);
  return launch_status("chained substep");
}

}  // namespace grhd

using namespace grhd;

// ------------------------------------------------------------ C ABI

extern "C" const char *grhd_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *grhd_version(void) { return "grhd-mi355x 0.1 (gfx950)"; }

extern "C" int grhd_workspace_bytes(const grhd_grid *grid, size_t *bytes) {
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if (!bytes) return fail(GRHD_ERR_INVALID, "bytes is NULL");
  const size_t n1 = (size_t)con2prim_blocks_of(grid);
  const size_t n2 = (size_t)max_stage_tiles(grid);
  const size_t nflag = (size_t)(grid->nz + 2 * grid->ng) * (size_t)grid->pitch;
  *bytes = ws_need(n1, n2, nflag);
  return GRHD_OK;
}

extern "C" int grhd_con2prim(const grhd_grid *grid, const grhd_eos *eos, const grhd_metric *metric,
                             const grhd_c2p_params *c2p, const grhd_cons *q, const grhd_prim *p,
                             uint8_t *flags, grhd_diag *diag, void *workspace, size_t workspace_bytes,
                             void *hip_stream) {
  int rc;
  if ((rc = check_grid(grid)) || (rc = check_eos(eos)) || (rc = check_metric(metric)) ||
      (rc = check_c2p(c2p)) || (rc = check_cons(q, "q")) || (rc = check_prim(p, "p")))
    return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  Q5 qq;
  P6 pp;
  for (int c = 0; c < 5; c++) qq.q[c] = q->q[c];
  for (int c = 0; c < 6; c++) pp.p[c] = p->p[c];
  GridK g = to_gridk(grid);
  int nb1 = con2prim_blocks(g);
  Workspace db;
  if ((rc = ws_carve(workspace, workspace_bytes, diag ? nb1 : 0, 0, 0, db))) return rc;
  C2PPart *p1 = db.p1;
  C2PK cp = to_c2pk(c2p);
  cp.reuse_atm = (c2p->reuse_atm && flags) ? 1 : 0;
  if ((rc = launch_con2prim(g, to_eosk(eos, c2p->rho_atm), cp, to_metk(metric),
                            metric_class(metric), qq, pp, flags, p1, st)))
    return rc;
  if (diag) {
    return launch_diag_final(p1, nb1, nullptr, 0, db.lvl, diag, st);
  }
  return GRHD_OK;
}

extern "C" int grhd_prim2con(const grhd_grid *grid, const grhd_eos *eos, const grhd_metric *metric,
                             const grhd_prim *p, const grhd_cons *q, int with_ghosts,
                             void *hip_stream) {
  int rc;
  if ((rc = check_grid(grid)) || (rc = check_eos(eos)) || (rc = check_metric(metric)) ||
      (rc = check_prim(p, "p")) || (rc = check_cons(q, "q")))
    return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  GridK g = to_gridk(grid);
  MetK m = to_metk(metric);
  Q5 qq;
  P6 pp;
  for (int c = 0; c < 5; c++) qq.q[c] = q->q[c];
  for (int c = 0; c < 6; c++) pp.p[c] = p->p[c];
  int lo = with_ghosts ? -g.ng : 0;
  int n = g.nx - 2 * lo;
  dim3 gd((n + 255) / 256, g.nz - 2 * lo);
  if (metric_class(metric) == MC_GEN)
    hipLaunchKernelGGL(k_prim2con<MC_GEN>, gd, dim3(256), 0, st, g, m, pp, qq, lo);
  else
    hipLaunchKernelGGL(k_prim2con<MC_CF>, gd, dim3(256), 0, st, g, m, pp, qq, lo);
  return launch_status("prim2con");
}

extern "C" int grhd_reconstruct(const grhd_grid *grid, int dir, int recon, int prec,
                                const grhd_prim *p, const grhd_prim *pL, const grhd_prim *pR,
                                void *hip_stream) {
  int rc;
  if ((rc = check_grid(grid)) || (rc = check_prim(p, "p")) || (rc = check_prim(pL, "pL")) ||
      (rc = check_prim(pR, "pR")))
    return rc;
  if (dir != 0 && dir != 1) return fail(GRHD_ERR_INVALID, "dir must be 0 or 1");
  if (recon != GRHD_RECON_PPM && recon != GRHD_RECON_MINMOD && recon != GRHD_RECON_PPM3)
    return fail(GRHD_ERR_INVALID, "bad recon");
  if (prec != GRHD_PREC_FP64 && prec != GRHD_PREC_MIXED) return fail(GRHD_ERR_INVALID, "bad prec");
  hipStream_t st = (hipStream_t)hip_stream;
  GridK g = to_gridk(grid);
  P6 pp;
  for (int c = 0; c < 6; c++) pp.p[c] = p->p[c];
  long long nf = (dir == 0) ? (long long)(g.nx + 1) * g.nz : (long long)g.nx * (g.nz + 1);
  int blocks = (int)((nf + 255) / 256);
  if (prec == GRHD_PREC_FP64) {
    Ptr6<double> L, R;
    for (int c = 0; c < 6; c++) { L.a[c] = pL->p[c]; R.a[c] = pR->p[c]; }
    hipLaunchKernelGGL(k_reconstruct<double>, dim3(blocks), dim3(256), 0, st, g, dir, recon, pp, L, R);
  } else {
    Ptr6<float> L, R;
    for (int c = 0; c < 6; c++) { L.a[c] = (float *)pL->p[c]; R.a[c] = (float *)pR->p[c]; }
    hipLaunchKernelGGL(k_reconstruct<float>, dim3(blocks), dim3(256), 0, st, g, dir, recon, pp, L, R);
  }
  return launch_status("reconstruct");
}

extern "C" int grhd_hllc_flux(const grhd_grid *grid, int dir, int riemann, int prec,
                              const grhd_eos *eos, const grhd_metric *metric, const grhd_prim *pL,
                              const grhd_prim *pR, const grhd_cons *F, double *max_speed,
                              void *hip_stream) {
  int rc;
  if ((rc = check_grid(grid)) || (rc = check_eos(eos)) || (rc = check_metric(metric)) ||
      (rc = check_prim(pL, "pL")) || (rc = check_prim(pR, "pR")) || (rc = check_cons(F, "F")))
    return rc;
  if (dir != 0 && dir != 1) return fail(GRHD_ERR_INVALID, "dir must be 0 or 1");
  if (riemann != GRHD_RIEMANN_HLLC && riemann != GRHD_RIEMANN_TVDLF) return fail(GRHD_ERR_INVALID, "bad riemann");
  if (prec != GRHD_PREC_FP64 && prec != GRHD_PREC_MIXED) return fail(GRHD_ERR_INVALID, "bad prec");
  hipStream_t st = (hipStream_t)hip_stream;
  GridK g = to_gridk(grid);
  EosK e = to_eosk(eos, 1.0);
  MetK m = to_metk(metric);
  int mc = metric_class(metric);
  Q5 FF;
  for (int c = 0; c < 5; c++) FF.q[c] = F->q[c];
  long long nf = (dir == 0) ? (long long)(g.nx + 1) * g.nz : (long long)g.nx * (g.nz + 1);
  int blocks = (int)((nf + 255) / 256);
  if (max_speed) {
    hipLaunchKernelGGL(k_zero_double, dim3(1), dim3(64), 0, st, max_speed);
    if ((rc = launch_status("max_speed reset"))) return rc;
  }
  if (prec == GRHD_PREC_FP64) {
    Ptr6<double> L, R;
    for (int c = 0; c < 6; c++) { L.a[c] = pL->p[c]; R.a[c] = pR->p[c]; }
    if (mc == MC_GEN)
      hipLaunchKernelGGL((k_flux<double, MC_GEN>), dim3(blocks), dim3(256), 0, st, g, e, m, dir, riemann, L, R, FF, max_speed);
    else
      hipLaunchKernelGGL((k_flux<double, MC_CF>), dim3(blocks), dim3(256), 0, st, g, e, m, dir, riemann, L, R, FF, max_speed);
  } else {
    Ptr6<float> L, R;
    for (int c = 0; c < 6; c++) { L.a[c] = (float *)pL->p[c]; R.a[c] = (float *)pR->p[c]; }
    if (mc == MC_GEN)
      hipLaunchKernelGGL((k_flux<float, MC_GEN>), dim3(blocks), dim3(256), 0, st, g, e, m, dir, riemann, L, R, FF, max_speed);
    else
      hipLaunchKernelGGL((k_flux<float, MC_CF>), dim3(blocks), dim3(256), 0, st, g, e, m, dir, riemann, L, R, FF, max_speed);
  }
  return launch_status("hllc_flux");
}

namespace grhd {
int fill_patch(const grhd_grid *grid, const grhd_metric *metric, const grhd_rk_stage *stage,
               const grhd_cons *qn, const grhd_cons *qs, const grhd_cons *qout, const grhd_prim *p,
               const grhd_cons *acc_in, const grhd_cons *acc_out, double *flux_reg, int recon,
               int riemann, PatchK &pk) {
  int rc;
  if ((rc = check_grid(grid)) || (rc = check_metric(metric)) || (rc = check_cons(qs, "qs")) ||
      (rc = check_cons(qout, "qout")) || (rc = check_prim(p, "p")))
    return rc;
  if (!stage) return fail(GRHD_ERR_INVALID, "stage is NULL");
  if (!std::isfinite(stage->dt) || !std::isfinite(stage->a) || !std::isfinite(stage->b) ||
      !std::isfinite(stage->c))
    return fail(GRHD_ERR_INVALID, "stage coefficients must be finite");
  if (stage->a != 0.0 && (rc = check_cons(qn, "qn"))) return rc;
  if (acc_in && (rc = check_cons(acc_in, "acc_in"))) return rc;
  if (acc_out && (rc = check_cons(acc_out, "acc_out"))) return rc;
  if (recon != GRHD_RECON_PPM && recon != GRHD_RECON_MINMOD && recon != GRHD_RECON_PPM3)
    return fail(GRHD_ERR_INVALID, "bad recon");
  if (riemann != GRHD_RIEMANN_HLLC && riemann != GRHD_RIEMANN_TVDLF) return fail(GRHD_ERR_INVALID, "bad riemann");
  // q_out may alias q^n (each cell reads its own q^n before writing
  // q_out), never q_s (whose halo other tiles read)
  for (int c = 0; c < 5; c++)
    if (qout->q[c] == qs->q[c]) return fail(GRHD_ERR_INVALID, "qout must not alias qs");
  pk.g = to_gridk(grid);
  pk.m = to_metk(metric);
  for (int c = 0; c < 5; c++) {
    pk.qn[c] = (stage->a != 0.0) ? qn->q[c] : nullptr;
    pk.qs[c] = qs->q[c];
    pk.qo[c] = qout->q[c];
    pk.acc_in[c] = acc_in ? acc_in->q[c] : nullptr;
    pk.acc_out[c] = acc_out ? acc_out->q[c] : nullptr;
  }
  for (int c = 0; c < 6; c++) pk.p[c] = p->p[c];
  pk.flux_reg = flux_reg;
  pk.fix_mask = nullptr;
  for (int c = 0; c < 5; c++) pk.fix_q[c] = nullptr;
  pk.a = stage->a; pk.b = stage->b; pk.cdt = stage->c * stage->dt;
  pk.gdt = stage->g * stage->dt; pk.d = stage->d; pk.e = stage->e; pk.dt = stage->dt;
  pk.cx = stage->dt / grid->dx; pk.cz = stage->dt / grid->dz;
  pk.idx = 1.0 / grid->dx; pk.idz = 1.0 / grid->dz;
  pk.i60dx = 1.0 / (60.0 * grid->dx); pk.i60dz = 1.0 / (60.0 * grid->dz);
  pk.use_qn = stage->a != 0.0;
  pk.use_acc_in = acc_in != nullptr && (stage->g != 0.0 || stage->d != 0.0);
  pk.use_acc_out = acc_out != nullptr;
  pk.recon = recon;
  pk.riemann = riemann;
  pk.face_eos = 0;
  pk.eos_id = 0;
  pk.tile_base = 0;
  pk.flags = nullptr;
  for (int c = 0; c < 6; c++) pk.po[c] = nullptr;
  pk.flags_out = nullptr;
  pk.cp = C2PK{};
  for (int s = 0; s < 2; s++) {
    pk.reg[s] = nullptr;
    pk.reg_j[s] = 0;
    pk.reg_k[s] = 0;
  }
  pk.reg_w = 0.0;
  return GRHD_OK;
}
}  // namespace grhd

// the optional interior boundary condition of grhd_options
static int set_fixed(const grhd_options *opts, PatchK &pk) {
  pk.face_eos = opts->face_eps == GRHD_FACE_EPS_EOS ? 1 : 0;
  if (!opts->fix_mask) return GRHD_OK;
  int rc;
  if ((rc = check_cons(&opts->fix_q, "fix_q"))) return rc;
  pk.fix_mask = opts->fix_mask;
  for (int c = 0; c < 5; c++) pk.fix_q[c] = opts->fix_q.q[c];
  return GRHD_OK;
}

namespace grhd {
// The whole stage on a given workspace (the caller's, or the static one of
// the variant that allocates nothing).
int rk_substep_ws(const grhd_grid *grid, const grhd_eos *eos, const grhd_metric *metric,
                  const grhd_options *opts, const grhd_rk_stage *stage, const grhd_cons *qn,
                  const grhd_cons *qs, const grhd_cons *qout, const grhd_prim *p,
                  const grhd_cons *acc_in, const grhd_cons *acc_out, double *flux_reg, uint8_t *flags,
                  grhd_diag *diag, void *workspace, size_t workspace_bytes, void *hip_stream) {
  int rc;
  if (!opts) return fail(GRHD_ERR_INVALID, "opts is NULL");
  if ((rc = check_eos(eos)) || (rc = check_c2p(&opts->c2p)) || (rc = check_face_eps(opts->face_eps)))
    return rc;
  if (opts->prec != GRHD_PREC_FP64 && opts->prec != GRHD_PREC_MIXED) return fail(GRHD_ERR_INVALID, "bad prec");
  PatchK pk;
  if ((rc = fill_patch(grid, metric, stage, qn, qs, qout, p, acc_in, acc_out, flux_reg, opts->recon,
                       opts->riemann, pk)))
    return rc;
  if ((rc = set_fixed(opts, pk))) return rc;
  // default 16 x 15: two full passes of the workgroup over the faces, a
  // small halo per cell, and the FP64 instance fits three workgroups per CU
  // in LDS; grids of few such tiles take 16 x 7 (twice the workgroups,
  // half the length of the slowest tile): under 1536 tiles of 16 x 16 for
  // the conformally flat class, under 128 for the general one
  int shape = shape_index(16, 15);
  if (opts->tile_x || opts->tile_z) {
    shape = shape_index(opts->tile_x, opts->tile_z);
    if (shape < 0) return fail(GRHD_ERR_UNSUPPORTED, "tile %dx%d not built", opts->tile_x, opts->tile_z);
  } else {
    const long long t16 = (long long)((grid->nx + 15) / 16) * ((grid->nz + 15) / 16);
    // a general metric with most geometry fields as arrays reads them from
    // LDS on 16 x 7 tiles (measured at 1024^2: 11 arrays, 316 against
    // 331 us per stage on 16 x 15; 4 arrays, 284 against 249 us)
    int geo = 0;
    if (metric)
      for (int f = 0; f < 11; f++) geo += metric->f[f] != nullptr;
    if (t16 < (metric_class(metric) == MC_CF ? 1536 : 128) || geo >= 8) shape = shape_index(16, 7);
  }
  int tx, tz;
  shape_of(shape, &tx, &tz);
  pk.xshift = tile_xshift(grid->ng, tx);
  pk.tiles_x = (grid->nx + pk.xshift + tx - 1) / tx;
  pk.tiles_z = (grid->nz + tz - 1) / tz;
  hipStream_t st = (hipStream_t)hip_stream;
  EosK e = to_eosk(eos, opts->c2p.rho_atm);
  int mc = metric_class(metric);
  Q5 q;
  P6 pp;
  for (int c = 0; c < 5; c++) q.q[c] = qs->q[c];
  for (int c = 0; c < 6; c++) pp.p[c] = p->p[c];
  int nb1 = con2prim_blocks(pk.g), nb2 = pk.tiles_x * pk.tiles_z;
  // the stage kernel reads the recovery flags (all-atmosphere tiles skip
  // their primitives); without caller flags they go to the workspace
  const size_t nflag = flags ? 0 : (size_t)(grid->nz + 2 * grid->ng) * (size_t)grid->pitch;
  Workspace db;
  if ((rc = ws_carve(workspace, workspace_bytes, diag ? nb1 : 0, diag ? nb2 : 0, nflag, db))) return rc;
  C2PPart *p1 = db.p1;
  FluxPart *p2 = db.p2;
  uint8_t *fl = flags ? flags : db.flags;
  pk.flags = fl;
  C2PK cp = to_c2pk(&opts->c2p);
  cp.reuse_atm = (opts->c2p.reuse_atm && flags) ? 1 : 0;  // never with workspace flags
  if ((rc = launch_con2prim(pk.g, e, cp, pk.m, mc, q, pp, fl, p1, st))) return rc;
  if (opts->ev_begin && hipEventRecord((hipEvent_t)opts->ev_begin, st) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "hipEventRecord failed");
  if ((rc = launch_substep(pk, e, opts->prec, mc, shape, p2, st))) return rc;
  if (opts->ev_end && hipEventRecord((hipEvent_t)opts->ev_end, st) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "hipEventRecord failed");
  if (diag) return launch_diag_final(p1, nb1, p2, nb2, db.lvl, diag, st);
  return GRHD_OK;
}
}  // namespace grhd

extern "C" int grhd_rk_substep(const grhd_grid *grid, const grhd_eos *eos, const grhd_metric *metric,
                               const grhd_options *opts, const grhd_rk_stage *stage,
                               const grhd_cons *qn, const grhd_cons *qs, const grhd_cons *qout,
                               const grhd_prim *p, const grhd_cons *acc_in, const grhd_cons *acc_out,
                               double *flux_reg, uint8_t *flags, grhd_diag *diag, void *workspace,
                               size_t workspace_bytes, void *hip_stream) {
  return rk_substep_ws(grid, eos, metric, opts, stage, qn, qs, qout, p, acc_in, acc_out, flux_reg, flags,
                       diag, workspace, workspace_bytes, hip_stream);
}

extern "C" int grhd_rk_substep_chained(const grhd_grid *grid, const grhd_eos *eos,
                                       const grhd_metric *metric, const grhd_options *opts,
                                       const grhd_rk_stage *stage, const grhd_cons *qn,
                                       const grhd_cons *qs, const grhd_cons *qout,
                                       const grhd_prim *p_in, const uint8_t *flags_in,
                                       const grhd_prim *p_out, uint8_t *flags_out,
                                       const grhd_cons *acc_in, const grhd_cons *acc_out,
                                       double *flux_reg, grhd_diag *diag, void *workspace,
                                       size_t workspace_bytes, void *hip_stream) {
  int rc;
  if (!opts) return fail(GRHD_ERR_INVALID, "opts is NULL");
  if ((rc = check_eos(eos)) || (rc = check_c2p(&opts->c2p)) || (rc = check_face_eps(opts->face_eps)))
    return rc;
  if (opts->prec != GRHD_PREC_FP64 && opts->prec != GRHD_PREC_MIXED) return fail(GRHD_ERR_INVALID, "bad prec");
  if ((opts->tile_x || opts->tile_z) && !(opts->tile_x == 16 && opts->tile_z == CHAIN_TZ))
    return fail(GRHD_ERR_UNSUPPORTED, "the chained stage is built for 16 x %d tiles only", CHAIN_TZ);
  PatchK pk;
  if ((rc = fill_patch(grid, metric, stage, qn, qs, qout, p_in, acc_in, acc_out, flux_reg, opts->recon,
                       opts->riemann, pk)))
    return rc;
  if ((rc = set_fixed(opts, pk))) return rc;
  if ((rc = check_prim(p_out, "p_out"))) return rc;
  if (!flags_out) return fail(GRHD_ERR_INVALID, "flags_out is NULL");
  if (flags_in && flags_in == flags_out) return fail(GRHD_ERR_INVALID, "flags_out must not alias flags_in");
  for (int a = 0; a < 6; a++)
    for (int b = 0; b < 6; b++)
      if (p_out->p[a] == p_in->p[b]) return fail(GRHD_ERR_INVALID, "p_out must not alias p_in");
  for (int s = 0; s < 4; s++)
    if (grid->bc[s] == GRHD_BC_EXTERNAL)
      return fail(GRHD_ERR_UNSUPPORTED, "the chained stage recovers interior cells only (no EXTERNAL sides)");
  pk.flags = const_cast<uint8_t *>(flags_in);
  for (int c = 0; c < 6; c++) pk.po[c] = p_out->p[c];
  pk.flags_out = flags_out;
  pk.cp = to_c2pk(&opts->c2p);
  pk.cp.reuse_atm = opts->c2p.reuse_atm ? 1 : 0;
  pk.xshift = tile_xshift(grid->ng, 16);
  pk.tiles_x = (grid->nx + pk.xshift + 15) / 16;
  pk.tiles_z = (grid->nz + CHAIN_TZ - 1) / CHAIN_TZ;
  hipStream_t st = (hipStream_t)hip_stream;
  EosK e = to_eosk(eos, opts->c2p.rho_atm);
  int mc = metric_class(metric);
  int nt = pk.tiles_x * pk.tiles_z;
  Workspace db;
  if ((rc = ws_carve(workspace, workspace_bytes, diag ? nt : 0, diag ? nt : 0, 0, db))) return rc;
  C2PPart *p1 = db.p1;
  FluxPart *p2 = db.p2;
  if (opts->ev_begin && hipEventRecord((hipEvent_t)opts->ev_begin, st) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "hipEventRecord failed");
  if ((rc = launch_substep_chain(pk, e, opts->prec, mc, p1, p2, st))) return rc;
  if (opts->ev_end && hipEventRecord((hipEvent_t)opts->ev_end, st) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "hipEventRecord failed");
  if (diag) return launch_diag_final(p1, nt, p2, nt, db.lvl, diag, st);
  return GRHD_OK;
}

namespace grhd {
// q = q_fixed on the interior cells where mask is set
__global__ void __launch_bounds__(256) k_fix_cells(GridK g, const uint8_t *mask, Q5 qf, Q5 q) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)g.nx * g.nz) return;
  const long long i = cell_index(g, (int)(id % g.nx), (int)(id / g.nx));
  if (!mask[i]) return;
  for (int c = 0; c < 5; c++) q.q[c][i] = qf.q[c][i];
}
}  // namespace grhd

extern "C" int grhd_fix_cells(const grhd_grid *grid, const uint8_t *mask, const grhd_cons *q_fixed,
                              const grhd_cons *q, void *hip_stream) {
  int rc;
  if ((rc = check_grid(grid)) || (rc = check_cons(q_fixed, "q_fixed")) || (rc = check_cons(q, "q")))
    return rc;
  if (!mask) return fail(GRHD_ERR_INVALID, "mask is NULL");
  Q5 a, b;
  for (int c = 0; c < 5; c++) { a.q[c] = q_fixed->q[c]; b.q[c] = q->q[c]; }
  long long n = (long long)grid->nx * grid->nz;
  hipLaunchKernelGGL(k_fix_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream,
                     to_gridk(grid), mask, a, b);
  return launch_status("fix cells");
}

extern "C" int grhd_event_create(void **ev) {
  if (!ev) return fail(GRHD_ERR_INVALID, "ev is NULL");
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return fail(GRHD_ERR_DEVICE, "hipEventCreate failed");
  *ev = (void *)e;
  return GRHD_OK;
}

extern "C" int grhd_event_elapsed_ms(void *begin, void *end, float *ms) {
  if (!begin || !end || !ms) return fail(GRHD_ERR_INVALID, "NULL argument");
  if (hipEventSynchronize((hipEvent_t)end) != hipSuccess) return fail(GRHD_ERR_DEVICE, "hipEventSynchronize failed");
  if (hipEventElapsedTime(ms, (hipEvent_t)begin, (hipEvent_t)end) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "hipEventElapsedTime failed");
  return GRHD_OK;
}

extern "C" int grhd_event_destroy(void *ev) {
  if (!ev) return GRHD_OK;
  return hipEventDestroy((hipEvent_t)ev) == hipSuccess ? GRHD_OK : fail(GRHD_ERR_DEVICE, "hipEventDestroy failed");
}
