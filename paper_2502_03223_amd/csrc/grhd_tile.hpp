// grhd_tile.hpp -- the fused per-tile work of one Runge-Kutta stage:
// LDS-staged primitives with a 3-cell halo (boundary conditions applied as
// an index map while loading), reconstruction + Riemann flux on every face
// of the tile in x then z (fluxes staged in LDS, one buffer reused for both
// directions), area-weighted divergence, cylindrical and metric sources,
// and the stage combination, all for one TX x TZ tile of one patch.
// Used by the single-patch kernels and by the batched kernel.
#pragma once

#include "grhd_dev.hpp"
#include "grhd_diag.hpp"
#include "grhd_mlp.hpp"

namespace grhd {

constexpr int NT = 256;  // threads per workgroup (4 wave64)

struct PatchK {
  GridK g;
  MetK m;
  double *qn[5], *qs[5], *qo[5], *p[6];
  double *acc_in[5], *acc_out[5];
  double *flux_reg;
  double a, b, cdt, gdt, d, e, dt;
  // grid and step constants, set on the host: dt/dx, dt/dz, 1/dx, 1/dz,
  // 1/(60 dx), 1/(60 dz)
  double cx, cz, idx, idz, i60dx, i60dz;
  int use_qn, use_acc_in, use_acc_out;
  int recon, riemann, eos_id;
  int face_eos;  // 1: face eps from the EOS at the face's (rho, P) (variant)
  uint8_t *flags;  // recovery flags of q_s (nullable)
  // chained stages only: recovery of q_out at the end of the stage
  double *po[6];       // primitives of q_out
  uint8_t *flags_out;  // recovery flags of q_out
  C2PK cp;
  // refinement-boundary flux registers (nullable): reg[s] accumulates
  // reg_w dt F over the face set {x faces j = reg_j[s], k < reg_k[s]} +
  // {z faces k = reg_k[s], j < reg_j[s]} (5 x (reg_k + reg_j) doubles)
  double *reg[2];
  int reg_j[2], reg_k[2];
  double reg_w;
  // interior boundary condition (nullable): cells with a nonzero mask
  // byte store fix_q instead of their update
  const uint8_t *fix_mask;
  const double *fix_q[5];
  int tiles_x, tiles_z;
  int xshift;  // tile tx covers cells j in [tx TX - xshift, (tx + 1) TX - xshift)
  long long tile_base;
};

// Tile layout of a patch: tiles start xshift = ng mod TX cells left of the
// interior, so with rows aligned to 128 bytes (pitch a multiple of 16
// doubles) every tile row segment starts on a line boundary.
__host__ __device__ inline int tile_xshift(int ng, int TX) { return ng % TX; }

// Order of the tiles of one patch over the workgroups: stripes of 8 tile
// columns, each stripe row by row.  Workgroups are dealt to the 8 XCDs
// round-robin, so in a full stripe each XCD owns one tile column: tiles
// above and below one another share their z halo in one L2, and any
// spatially compact heavy region spreads over all XCDs.
__host__ __device__ inline void tile_of(long long t, int tiles_x, int tiles_z, int &tx, int &tz) {
  long long per = 8LL * tiles_z;
  int s = (int)(t / per);
  int rem = (int)(t - per * s);
  int w = tiles_x - 8 * s;
  if (w > 8) w = 8;
  tz = rem / w;
  tx = 8 * s + rem % w;
}

template <class T, int MC, int TX, int TZ>
struct TileSmem {
  static constexpr int HX = TX + 6, HZ = TZ + 6, NC = HX * HZ;
  static constexpr int NFX = (TX + 1) * TZ, NFZ = TX * (TZ + 1);
  static constexpr int NF = NFX + NFZ;  // x faces, then z faces
  static constexpr int NM = (MC == MC_CF) ? NC : 1;
  // general class on tiles of at most 128 cells: the 11 geometry fields
  // (lapse, shift, W, conformal metric; the fields whose face values and
  // derivatives the stage takes) staged in LDS as well
  static constexpr bool MG = (MC == MC_GEN) && TX * TZ <= 128;
  static constexpr int NGM = 11;
  static constexpr int NGC = MG ? NC : 1;
  T p[6][NC];
  double ma[NM], mw[NM];
  double mg[NGM][NGC];
  T f[5][NF];
  uint8_t atm[NC];  // 1: the cell holds exactly the atmosphere state
};

// Source cell of ghost cell (j, k) under the boundary conditions, with the
// velocity parities; false for cells no stencil of the tile reads.
__device__ __forceinline__ bool ghost_map(const GridK &g, int j, int k, int &js, int &ks,
                                          double sg[3]) {
  sg[0] = sg[1] = sg[2] = 1.0;
  js = j;
  ks = k;
  bool jin = (j >= 0 && j < g.nx), kin = (k >= 0 && k < g.nz);
  if (jin && kin) return true;
  if (!jin && !kin) return false;
  if (!jin) {
    int side = (j < 0) ? 0 : 1;
    int bc = g.bc[side];
    if (bc == GRHD_BC_PERIODIC) js = ((j % g.nx) + g.nx) % g.nx;
    else if (bc == GRHD_BC_OUTFLOW) js = side ? g.nx - 1 : 0;
    else if (bc == GRHD_BC_AXIS || bc == GRHD_BC_REFLECT) {
      js = side ? 2 * g.nx - 1 - j : -1 - j;
      sg[0] = -1.0;
      if (bc == GRHD_BC_AXIS) sg[1] = -1.0;
    }
  } else {
    int side = (k < 0) ? 0 : 1;
    int bc = g.bc[2 + side];
    if (bc == GRHD_BC_PERIODIC) ks = ((k % g.nz) + g.nz) % g.nz;
    else if (bc == GRHD_BC_OUTFLOW) ks = side ? g.nz - 1 : 0;
    else if (bc == GRHD_BC_AXIS || bc == GRHD_BC_REFLECT) {
      ks = side ? 2 * g.nz - 1 - k : -1 - k;
      sg[2] = -1.0;
    }
  }
  return true;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Adds reg_w dt F of one face to the refinement-boundary registers that
// contain it.  A face on a tile edge is computed by both tiles: the tile
// holding the cell on its high side adds it (the last tile at the patch's
// high edge).  fv: the face flux in register form (S_phi component times
// x, E flux = D flux + tau flux).
template <int TX, int TZ>
__device__ __forceinline__ void fmr_reg_add(const PatchK &P, bool isx, int j, int k, int jj, int kk,
                                            const double *fv) {
  for (int s = 0; s < 2; s++) {
    double *r = P.reg[s];
    if (!r) continue;
    const int rj = P.reg_j[s], rk = P.reg_k[s];
    const bool on = isx ? (j == rj && k < rk && (jj < TX || j == P.g.nx))
                        : (k == rk && j < rj && (kk < TZ || k == P.g.nz));
    if (!on) continue;
    const long long nr = (long long)rk + rj;
    const long long o = isx ? k : rk + j;
    const double wdt = P.reg_w * P.dt;
    for (int m = 0; m < 5; m++) r[m * nr + o] += wdt * fv[m];
  }
}

// Recovery statistics of the cells one thread finished (rescale, cold,
// atmosphere, failed, iteration sum, iteration max).
struct C2PAcc {
  unsigned long long n[6];
};

// Chained stages: recovery of the stage result v of cell ic (Sec. II.C.4),
// v corrected where a flag is set, then q_out, the primitives and flags of
// q_out written, so that the next stage needs no recovery pass of its own.
// W, gt: metric at the cell.  Without CHAIN the caller stores v itself.
// fprev: the cell's flag byte in P.flags_out when the caller loaded it
// already, else -1.
template <int MC, int EK>
__device__ __forceinline__ void recover_store(const PatchK &P, const EosK &e, unsigned ic, double W,
                                              const double *gtu, double xc, double dV, double *v,
                                              double &mb, double &jm, C2PAcc &acc, double zg,
                                              int fprev = -1) {
  {
    double pp[6];
    C2PResult r = con2prim_cell<MC, EK>(e, P.cp, W, gtu, xc, P.g.geom, v, pp, zg);
    // a cell that was and stays atmosphere already holds its primitives
    const bool keep = P.cp.reuse_atm && (r.flags & GRHD_FLAG_ATM) &&
                      ((fprev >= 0 ? (uint8_t)fprev : ld32(P.flags_out, ic)) & GRHD_FLAG_ATM);
    if (!keep)
      for (int c = 0; c < 6; c++) st32(P.po[c], ic, pp[c]);
    st32(P.flags_out, ic, (uint8_t)r.flags);
    acc.n[0] += (r.flags & GRHD_FLAG_RESCALE) ? 1 : 0;
    acc.n[1] += (r.flags & GRHD_FLAG_COLD) ? 1 : 0;
    acc.n[2] += (r.flags & GRHD_FLAG_ATM) ? 1 : 0;
    acc.n[3] += (r.flags & GRHD_FLAG_FAIL) ? 1 : 0;
    acc.n[4] += (unsigned long long)r.iters;
    if ((unsigned long long)r.iters > acc.n[5]) acc.n[5] = (unsigned long long)r.iters;
  }
  for (int m = 0; m < 5; m++) st32(P.qo[m], ic, v[m]);
  mb += v[0] * dV;
  jm += v[2] * dV;
}

template <int MC, int EK, bool CHAIN>
__device__ __forceinline__ void finish_cell(const PatchK &P, const EosK &e, unsigned ic, double W,
                                            const double *gt, double xc, double dV, double *v,
                                            double &mb, double &jm, C2PAcc &acc, int fprev = -1) {
  if (!CHAIN) return;  // stored by the caller as they were computed
  double gtu[6];
  if (MC == MC_GEN) inv_sym3(gt, gtu);
  recover_store<MC, EK>(P, e, ic, W, gtu, xc, dV, v, mb, jm, acc, -1.0, fprev);
}

// Chained stages with the learned guess (GRHD_GUESS_MLP): the recovery of
// the stage result starts from the network's guess.  Every lane of the wave
// calls it (the network spans the wave); act marks the lanes holding a
// cell, the others pass W = 1, the identity metric and a zero state.
template <int MC, int EK>
__device__ __forceinline__ void finish_cell_mlp(const PatchK &P, const EosK &e, bool act, unsigned ic,
                                                double W, const double *gt, double xc, double dV,
                                                double *v, double &mb, double &jm, C2PAcc &acc) {
  double gtu[6];
  if (MC == MC_GEN) inv_sym3(gt, gtu);
  const double zg = mlp_guess_wave<MC>((const MlpDev *)P.cp.mlp, act, W, gtu, xc, P.g.geom, v);
  if (act) recover_store<MC, EK>(P, e, ic, W, gtu, xc, dV, v, mb, jm, acc, zg);
}

// Classification of an inner 16-wide tile (its halo inside the grid, rows
// 16-byte aligned in the flag array) from the recovery flags with wide
// loads: 16 flag bytes per tile row (one 16-byte load), the three bytes on
// each side of the row (one aligned 4-byte load each), and the six halo
// rows above and below.  Returns this thread's share: false when one of the
// bytes it loaded lacks GRHD_FLAG_ATM.  e0(k) = element of cell (j0, k).
template <int TZ>
__device__ __forceinline__ bool atm_flags16(const PatchK &P, int j0, int k0) {
  const int tid = threadIdx.x;
  constexpr int NL = 3 * TZ + 6;
  if (tid >= NL) return true;
  const GridK &g = P.g;
  const unsigned A = 0x04040404u;  // GRHD_FLAG_ATM in every byte
  int row, kind;                   // kind 0: 16 bytes, 1: left side, 2: right side
  if (tid < TZ) { row = tid; kind = 0; }
  else if (tid < 2 * TZ) { row = tid - TZ; kind = 1; }
  else if (tid < 3 * TZ) { row = tid - 2 * TZ; kind = 2; }
  else { const int h = tid - 3 * TZ; row = h < 3 ? h - 3 : TZ + h - 3; kind = 0; }
  const unsigned e0 = cell_idx32(g, j0, k0 + row);
  const uint8_t *f = P.flags;
  if (kind == 0) {
    const uint4 v = *reinterpret_cast<const uint4 *>(f + e0);
    return ((v.x & v.y & v.z & v.w) & A) == A;
  }
  if (kind == 1) {
    const unsigned v = *reinterpret_cast<const unsigned *>(f + e0 - 4);
    return ((v | 0xFFu) & A) == A;          // bytes 1..3: cells j0-3 .. j0-1
  }
  const unsigned v = *reinterpret_cast<const unsigned *>(f + e0 + 16);
  return ((v | 0xFF000000u) & A) == A;      // bytes 0..2: cells j0+16 .. j0+18
}

// The global loads of an inner tile that the all-atmosphere stage needs,
// one cell per thread: the cell's own states (q_s, q^n, accumulator) and
// lapse and W on its cross-shaped 7-point stencils (x: ax, wx at j-3..j+3;
// z: az, wz at k-3..k+3; the centre value is in both).  They are issued
// together with the classification's flag loads, so an all-atmosphere tile
// makes one memory round trip before its arithmetic.
template <int TX, int TZ>
struct LeanLoads {
  static constexpr int CPT = (TX * TZ + NT - 1) / NT;
  unsigned ic[CPT];
  double qs5[CPT][5], qn5[CPT][5], ai5[CPT][5];
  double ax[CPT][7], wx[CPT][7], az[CPT][7], wz[CPT][7];
  int fo[CPT];  // chained stages: the cell's byte in flags_out, or -1
};

// CHAIN: the byte of flags_out that the recovery at the end of a chained
// stage consults (reuse_atm) is loaded here too, so that no load waits
// behind the arithmetic.
template <int TX, int TZ, bool CHAIN>
__device__ __forceinline__ void lean_issue(const PatchK &P, int j0, int k0, LeanLoads<TX, TZ> &L) {
  using LL = LeanLoads<TX, TZ>;
  const GridK &g = P.g;
  const int tid = threadIdx.x;
  const unsigned pitch = (unsigned)g.pitch;
#pragma unroll
  for (int ci = 0; ci < LL::CPT; ci++) {
    const int c = tid + ci * NT;
    const int jj = c % TX, kk = c / TX;
    const unsigned ic = cell_idx32(g, j0 + jj, k0 + kk);
    L.ic[ci] = ic;
    if (c < TX * TZ) {
      for (int m = 0; m < 5; m++) L.qs5[ci][m] = ld32(P.qs[m], ic);
      if (P.use_qn)
        for (int m = 0; m < 5; m++) L.qn5[ci][m] = ld32(P.qn[m], ic);
      if (P.use_acc_in)
        for (int m = 0; m < 5; m++) L.ai5[ci][m] = ld32(P.acc_in[m], ic);
      L.fo[ci] = (CHAIN && P.cp.reuse_atm) ? (int)ld32(P.flags_out, ic) : -1;
      for (int i = 0; i < 7; i++) {
        const unsigned ix = ic - 3u + (unsigned)i, iz = ic + (unsigned)(i - 3) * pitch;
        L.ax[ci][i] = mval32(P.m, GRHD_M_ALP, ix);
        L.wx[ci][i] = mval32(P.m, GRHD_M_W, ix);
        L.az[ci][i] = mval32(P.m, GRHD_M_ALP, iz);
        L.wz[ci][i] = mval32(P.m, GRHD_M_W, iz);
      }
    }
  }
}

// Atmosphere face flux (conformally flat class): the normal-momentum flux
// alpha W^-3 P_atm and the signal speed alpha c_s W at the face whose
// 6-point stencil starts at a[0], w[0].  The expressions of the general
// path's atmosphere faces.
template <class T>
__device__ __forceinline__ T atm_face(const double *a, const double *w, T Pa, T cs_atm, T &sp) {
  T t6[6];
  for (int i = 0; i < 6; i++) t6[i] = (T)a[i];
  const T alp = lagrange6(t6);
  for (int i = 0; i < 6; i++) t6[i] = (T)w[i];
  const T W = lagrange6(t6);
  T sg = T(1) / (W * W * W);
  sp = alp * (cs_atm * W);
  return sg * (alp * Pa);
}

// The whole stage of an inner all-atmosphere tile of the conformally flat
// class (halo inside the grid, every cell of the halo flagged ATM by the
// recovery), one cell per thread and no shared memory: each thread
// evaluates the four faces of its cell from the stencils in registers (a
// face between two cells is evaluated by both, with the same operations on
// the same values, hence the same bits), the lapse and W derivatives, the
// divergence, sources and stage update.  Every value is computed with the
// same expressions in the same order as the atmosphere branch of the
// general tile code below, so a cell's result does not depend on the path
// its tile takes.  Inner tiles have no grid-boundary faces (no flux
// register entries); a refinement-register face is added by the cell on its
// high side, as in the general code.
template <class T, int TX, int TZ, bool CHAIN, int EK>
__device__ __forceinline__ void lean_atm_tile(const PatchK &P, const EosK &e, int j0, int k0,
                                              const LeanLoads<TX, TZ> &ld, double &cmax_out,
                                              double &mb_out, double &jm_out, C2PAcc &acc) {
  constexpr int CPT = LeanLoads<TX, TZ>::CPT;
  const GridK &g = P.g;
  const int tid = threadIdx.x;
  const bool cyl = (g.geom == GRHD_GEOM_CYLINDRICAL);
  const T Pa = (T)e.P_atm, cs_atm = (T)e.cs_atm;
  const double cx = P.cx, cz = P.cz;
  const bool regs = P.reg[0] || P.reg[1];
  const double rhw2_atm = e.rhw2_atm;
  const double i60dx = P.i60dx, i60dz = P.i60dz;
  double cmax = 0.0, mb = 0.0, jm = 0.0;
#pragma unroll
  for (int ci = 0; ci < CPT; ci++) {
#pragma clang fp contract(off)
    const int c = tid + ci * NT;
    if (!(c < TX * TZ)) continue;
    const int jj = c % TX, kk = c / TX;
    const int j = j0 + jj, k = k0 + kk;
    const unsigned ic = ld.ic[ci];
    // the four faces: left and right x faces, bottom and top z faces
    T sp;
    const T fxl = atm_face<T>(ld.ax[ci], ld.wx[ci], Pa, cs_atm, sp);
    cmax = fmax(cmax, (double)sp * cx);
    const T fxr = atm_face<T>(ld.ax[ci] + 1, ld.wx[ci] + 1, Pa, cs_atm, sp);
    cmax = fmax(cmax, (double)sp * cx);
    const T fzb = atm_face<T>(ld.az[ci], ld.wz[ci], Pa, cs_atm, sp);
    cmax = fmax(cmax, (double)sp * cz);
    const T fzt = atm_face<T>(ld.az[ci] + 1, ld.wz[ci] + 1, Pa, cs_atm, sp);
    cmax = fmax(cmax, (double)sp * cz);
    if (regs) {
      double fv[5] = {0.0, (double)fxl, 0.0, 0.0, 0.0};
      fmr_reg_add<TX, TZ>(P, true, j, k, jj, kk, fv);
      double fw[5] = {0.0, 0.0, 0.0, (double)fzb, 0.0};
      fmr_reg_add<TX, TZ>(P, false, j, k, jj, kk, fw);
    }
    double xc = g.x0 + (j + 0.5) * g.dx;
    const double xl = g.x0 + j * g.dx, xr = g.x0 + (j + 1) * g.dx;
    const double ivx = cyl ? 1.0 / (xc * g.dx) : P.idx, ivz = P.idz;
    double gm[GRHD_NMET], dg[2 * GRHD_NMET];
    for (int i = 0; i < GRHD_NMET; i++) { gm[i] = P.m.c[i]; dg[i] = 0.0; dg[GRHD_NMET + i] = 0.0; }
    gm[GRHD_M_ALP] = ld.ax[ci][3];
    gm[GRHD_M_W] = ld.wx[ci][3];
    if (P.m.f[GRHD_M_ALP]) {
      dg[GRHD_M_ALP] = deriv6(ld.ax[ci], i60dx);
      dg[GRHD_NMET + GRHD_M_ALP] = deriv6(ld.az[ci], i60dz);
    }
    if (P.m.f[GRHD_M_W]) {
      dg[GRHD_M_W] = deriv6(ld.wx[ci], i60dx);
      dg[GRHD_NMET + GRHD_M_W] = deriv6(ld.wz[ci], i60dz);
    }
    double L[5];
    {
      const double Fl = (double)fxl, Fr = (double)fxr;
      const double divx1 = cyl ? (xr * Fr - xl * Fl) * ivx : (Fr - Fl) * ivx;
      const double divz3 = ((double)fzt - (double)fzb) * ivz;
      double s[5];
      sources_atm_cf(gm, dg, xc, g.geom, e.P_atm, rhw2_atm, s);
      L[0] = 0.0; L[1] = s[1] - divx1; L[2] = 0.0; L[3] = s[3] - divz3; L[4] = 0.0;
    }
    double dV = cyl ? 2.0 * M_PI * xc * g.dx * g.dz : g.dx * g.dz;
    const bool fixed = P.fix_mask && ld32(P.fix_mask, ic);
    double v[5];
    for (int m = 0; m < 5; m++) {
      v[m] = P.b * ld.qs5[ci][m] + P.cdt * L[m];
      if (P.use_qn) v[m] += P.a * ld.qn5[ci][m];
      if (P.use_acc_in) v[m] += P.gdt * ld.ai5[ci][m];
      if (fixed) v[m] = ld32(P.fix_q[m], ic);
      if (!CHAIN) {
        st32(P.qo[m], ic, v[m]);
        if (m == 0) mb += v[m] * dV;
        if (m == 2) jm += v[m] * dV;
      }
      if (P.use_acc_out) {
        double av = P.e * L[m];
        if (P.use_acc_in) av += P.d * ld.ai5[ci][m];
        st32(P.acc_out[m], ic, av);
      }
    }
    finish_cell<MC_CF, EK, CHAIN>(P, e, ic, gm[GRHD_M_W], gm + GRHD_M_GXX, xc, dV, v, mb, jm, acc,
                                  ld.fo[ci]);
  }
  cmax_out = cmax;
  mb_out = mb;
  jm_out = jm;
}

// One tile of one patch.  cmax, mb, jm receive this thread's share of the
// tile's diagnostics (max Courant number, sums of q_D dV and q_Sphi dV of
// the stored q_out); with CHAIN, acc its recovery statistics.
// ML (chained stages only): the recovery at the end of the stage takes the
// learned guess; every cell's recovery then waits for the end of the cell
// loop, where the whole wave evaluates the network.  All-atmosphere tiles
// of the lean path recover without it.
template <class T, int MC, int TX, int TZ, bool CHAIN = false, int EK = 0, bool ML = false>
__device__ __forceinline__ void substep_tile(const PatchK &P, const EosK &e, int tx, int tz,
                                             TileSmem<T, MC, TX, TZ> &sm, double &cmax_out,
                                             double &mb_out, double &jm_out, C2PAcc &acc) {
  static_assert(!ML || CHAIN, "the learned guess belongs to the chained stage's recovery");
  using S = TileSmem<T, MC, TX, TZ>;
  constexpr int HX = S::HX;
  constexpr int CPT = (TX * TZ + NT - 1) / NT;
  constexpr int LPT = (S::NC + NT - 1) / NT;
  const GridK &g = P.g;
  const int tid = threadIdx.x;
  const int nx = g.nx, nz = g.nz;
  const int j0 = tx * TX - P.xshift, k0 = tz * TZ;
  const bool cyl = (g.geom == GRHD_GEOM_CYLINDRICAL);
  const T ra = (T)e.rho_atm, Pa = (T)e.P_atm, ea = (T)e.eps_atm;
  const T cs_atm = (T)e.cs_atm;
  __syncthreads();  // LDS of a previous use in this workgroup is free

  // ---- 1. stage the cross-shaped halo in LDS: lapse and W (conformally
  // flat class) and the atmosphere mask first, then the primitives unless
  // the whole halo is atmosphere.  With the recovery flags of q_s at hand
  // the mask comes from them (ATM: the recovery reset the cell to exactly
  // the atmosphere state) and an all-atmosphere tile needs no primitives at
  // all; without them the mask compares the primitive values.  Within each
  // part all addresses come first, then all loads, then all LDS stores.
  // Boundary conditions are an index map with velocity parities.
  bool tile_atm;
  // a tile whose halo lies inside the grid reads every cell where it is
  // (no boundary map, no parities)
  const bool inner = j0 >= 3 && j0 + TX + 3 <= nx && k0 >= 3 && k0 + TZ + 3 <= nz;
  // inner 16-wide tiles with 16-byte aligned flag rows are classified from
  // wide flag loads first; an all-atmosphere one of the conformally flat
  // class then stages only its lapse and W
  if constexpr (MC == MC_CF) {
    const bool fast_class = TX == 16 && inner && P.flags != nullptr && (g.pitch & 15) == 0 &&
                            ((uintptr_t)P.flags & 15) == 0;
    if (fast_class) {
      LeanLoads<TX, TZ> ld;
      lean_issue<TX, TZ, CHAIN>(P, j0, k0, ld);
      const bool mine = atm_flags16<TZ>(P, j0, k0);
      if (__syncthreads_and(mine) != 0) {
        lean_atm_tile<T, TX, TZ, CHAIN, EK>(P, e, j0, k0, ld, cmax_out, mb_out, jm_out, acc);
        return;
      }
    }
  }
  {
    const bool have_flags = P.flags != nullptr;
    unsigned src[LPT], im[LPT];
    bool use[LPT], fin[LPT];
    double s0[LPT], s1[LPT], s2[LPT];
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      int c = tid + i * NT;
      int jj = c % HX, kk = c / HX;
      int j = j0 - 3 + jj, k = k0 - 3 + kk;
      bool inx = (jj >= 3 && jj < 3 + TX), inz = (kk >= 3 && kk < 3 + TZ);
      int js = j, ks = k;
      double sg[3] = {1.0, 1.0, 1.0};
      bool need;
      if (inner) {
        need = c < S::NC && (inx || inz);
      } else {
        need = c < S::NC &&
               ((inx && j < nx && k >= -3 && k < nz + 3) || (inz && k < nz && j >= -3 && j < nx + 3));
        if (need) need = ghost_map(g, j, k, js, ks, sg);
      }
      use[i] = need;
      // recovery flags exist for grid cells only (an EXTERNAL ghost maps
      // to itself and counts as not atmosphere)
      fin[i] = inner || (js >= 0 && js < nx && ks >= 0 && ks < nz);
      src[i] = need ? cell_idx32(g, js, ks) : 0u;
      im[i] = need ? cell_idx32(g, j, k) : 0u;
      s0[i] = sg[0]; s1[i] = sg[1]; s2[i] = sg[2];
    }
    double va[LPT], vw[LPT];
    uint8_t fl[LPT];
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      if (use[i]) {
        fl[i] = (have_flags && fin[i]) ? ld32(P.flags, src[i]) : (uint8_t)0;
        if (MC == MC_CF) {
          va[i] = mval32(P.m, GRHD_M_ALP, im[i]);
          vw[i] = mval32(P.m, GRHD_M_W, im[i]);
        }
      }
    }
    if constexpr (S::MG) {
      // the geometry fields at every cell a face or derivative stencil
      // reads (metric ghost cells are the caller's, as in the face loop)
      double vg[LPT][S::NGM];
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (use[i])
          for (int fld = 0; fld < S::NGM; fld++) vg[i][fld] = mval32(P.m, fld, im[i]);
#pragma unroll
      for (int i = 0; i < LPT; i++) {
        const int c = tid + i * NT;
        if (use[i])
          for (int fld = 0; fld < S::NGM; fld++) sm.mg[fld][c] = vg[i][fld];
      }
    }
    int my_atm = have_flags ? 1 : 0;
#pragma unroll
    for (int i = 0; i < LPT; i++) {
      int c = tid + i * NT;
      if (use[i]) {
        uint8_t a = (fl[i] & GRHD_FLAG_ATM) ? 1 : 0;
        sm.atm[c] = a;
        my_atm &= a;
        if (MC == MC_CF) {
          sm.ma[c] = va[i];
          sm.mw[c] = vw[i];
        }
      }
    }
    tile_atm = __syncthreads_and(my_atm) != 0;
    if (!tile_atm) {
      double v[LPT][6];
#pragma unroll
      for (int i = 0; i < LPT; i++)
        if (use[i])
          for (int f = 0; f < 6; f++) v[i][f] = ld32(P.p[f], src[i]);
#pragma unroll
      for (int i = 0; i < LPT; i++) {
        int c = tid + i * NT;
        if (use[i]) {
          T r = (T)v[i][0], u0 = (T)(s0[i] * v[i][1]), u1 = (T)(s1[i] * v[i][2]),
            u2 = (T)(s2[i] * v[i][3]), pr = (T)v[i][4], ep = (T)v[i][5];
          sm.p[0][c] = r; sm.p[1][c] = u0; sm.p[2][c] = u1; sm.p[3][c] = u2;
          sm.p[4][c] = pr; sm.p[5][c] = ep;
          if (!have_flags)
            sm.atm[c] = (r == ra && u0 == T(0) && u1 == T(0) && u2 == T(0) && pr == Pa && ep == ea) ? 1 : 0;
        }
      }
      __syncthreads();
    }
  }

  const int nb = 2 * nz + 2 * nx;  // flux-register stride
  double cmax = 0.0;
  // rho h of the atmosphere state
  const double rhw2_atm = e.rhw2_atm;
  const double i60dx = P.i60dx, i60dz = P.i60dz;

  const bool atm_fast = (MC == MC_CF) && tile_atm;
  if (atm_fast) {
    // ---- all-atmosphere tile (conformally flat metric class): at every
    // face the atmosphere at rest has only alpha W^-3 P_atm in the normal
    // momentum (S_x at x faces, S_z at z faces) and the signal speeds
    // -+ alpha c_s W; D, S_phi and tau of the cells change only through
    // the stage weights.  The same values as the general path's uniform
    // faces and atmosphere sources, with the zero terms left out.
    const double cx = P.cx, cz = P.cz;
    for (int f = tid; f < S::NF; f += NT) {
      const bool isx = f < S::NFX;
      int jj, kk, base, stride;
      if (isx) {
        jj = f % (TX + 1); kk = f / (TX + 1);
        base = (kk + 3) * HX + jj; stride = 1;
      } else {
        int h = f - S::NFX;
        jj = h % TX; kk = h / TX;
        base = kk * HX + jj + 3; stride = HX;
      }
      const int j = j0 + jj, k = k0 + kk;
      const bool valid = isx ? (k < nz && j >= 0 && j <= nx) : (j >= 0 && j < nx && k <= nz);
      T fn = T(0);
      if (valid) {
        T t6[6];
        for (int i = 0; i < 6; i++) t6[i] = (T)sm.ma[base + i * stride];
        const T alp = lagrange6(t6);
        for (int i = 0; i < 6; i++) t6[i] = (T)sm.mw[base + i * stride];
        const T W = lagrange6(t6);
        T sg = T(1) / (W * W * W);
        fn = sg * (alp * Pa);
        const T sp = alp * (cs_atm * W);
        cmax = fmax(cmax, (double)sp * (isx ? cx : cz));
        if (P.flux_reg && (isx ? (j == 0 || j == nx) : (k == 0 || k == nz))) {
          int o = isx ? ((j == 0) ? k : nz + k) : 2 * nz + ((k == 0) ? j : nx + j);
          for (int m = 0; m < 5; m++) P.flux_reg[m * nb + o] = 0.0;
          P.flux_reg[(isx ? 1 : 3) * nb + o] = (double)fn;
        }
        if (P.reg[0] || P.reg[1]) {
          double fv[5] = {0.0, isx ? (double)fn : 0.0, 0.0, isx ? 0.0 : (double)fn, 0.0};
          fmr_reg_add<TX, TZ>(P, isx, j, k, jj, kk, fv);
        }
      }
      sm.f[0][f] = fn;
    }
  } else {
    // ---- 2. all faces of the tile in one balanced loop: x faces x_{j-1/2}
    // (j = j0..j0+TX) first, then z faces z_{k-1/2} (k = k0..k0+TZ); the
    // stencil is addressed by a base and a stride so x and z lanes of one
    // wave run the same instructions.
    for (int f = tid; f < S::NF; f += NT) {
      const bool isx = f < S::NFX;
      int jj, kk, base, stride;
      if (isx) {
        jj = f % (TX + 1); kk = f / (TX + 1);
        base = (kk + 3) * HX + jj; stride = 1;
      } else {
        int h = f - S::NFX;
        jj = h % TX; kk = h / TX;
        base = kk * HX + jj + 3; stride = HX;
      }
      const int j = j0 + jj, k = k0 + kk;
      const bool valid = isx ? (k < nz && j >= 0 && j <= nx) : (j >= 0 && j < nx && k <= nz);
      FluxT<T> out;
      for (int m = 0; m < 5; m++) out.f[m] = T(0);
      if (valid) {
        // a stencil of six atmosphere cells has equal left and right states,
        // and both solvers then return the physical flux of that state
        // exactly: evaluate it directly
        bool uni = tile_atm;
        if (!uni) {
          uni = true;
          for (int i = 0; i < 6; i++) uni = uni && sm.atm[base + i * stride];
        }
        PrimT<T> L, R;
        if (uni) {
          L.rho = ra;
          L.u[0] = T(0); L.u[1] = T(0); L.u[2] = T(0);
          L.P = Pa; L.eps = ea;
          R = L;
        } else {
          // rho, u_i, P and eps reconstructed (the paper's face states);
          // in the EOS variant eps comes from the EOS at the face's
          // (rho, P) instead
          T s[6], a, b;
          const int nrec = P.face_eos ? 5 : 6;
          for (int fld = 0; fld < nrec; fld++) {
            for (int i = 0; i < 6; i++) s[i] = sm.p[fld][base + i * stride];
            recon_face(P.recon, s, a, b);
            if (fld == 0) { L.rho = a; R.rho = b; }
            else if (fld < 4) { L.u[fld - 1] = a; R.u[fld - 1] = b; }
            else if (fld == 4) { L.P = a; R.P = b; }
            else { L.eps = a; R.eps = b; }
          }
          if (P.face_eos) {
            L.eps = eos_eps(e, L.rho, L.P);
            R.eps = eos_eps(e, R.rho, R.P);
          }
        }
        FaceMet<T> fm;
        T t6[6];
        if (MC == MC_CF) {
          for (int i = 0; i < 6; i++) t6[i] = (T)sm.ma[base + i * stride];
          fm.alp = lagrange6(t6);
          for (int i = 0; i < 6; i++) t6[i] = (T)sm.mw[base + i * stride];
          fm.W = lagrange6(t6);
        } else {
          long long g0 = isx ? cell_index(g, j - 3, k) : cell_index(g, j, k - 3);
          long long gs = isx ? 1 : g.pitch;
          for (int fld = 0; fld < 11; fld++) {
            const double *src = P.m.f[fld];
            T v;
            if (src) {
              if constexpr (S::MG) {
                for (int i = 0; i < 6; i++) t6[i] = (T)sm.mg[fld][base + i * stride];
              } else {
                for (int i = 0; i < 6; i++) t6[i] = (T)src[g0 + i * gs];
              }
              v = lagrange6(t6);
            } else {
              v = (T)P.m.c[fld];
            }
            if (fld == 0) fm.alp = v;
            else if (fld < 4) fm.beta[fld - 1] = v;
            else if (fld == 4) fm.W = v;
            else fm.gt[fld - 5] = v;
          }
        }
        if (uni && MC == MC_CF) {
          // the atmosphere at rest in a conformally flat metric without
          // shift: of the physical flux only alpha W^-3 P in the normal
          // momentum survives, and the signal speeds are -+ alpha c_s W
          // (the physical-flux evaluation below reduces to exactly these)
          T sg = T(1) / (fm.W * fm.W * fm.W);
          out.f[isx ? 1 : 3] = sg * (fm.alp * Pa);
          out.speed = fm.alp * (cs_atm * fm.W);
        } else if (uni) {
          T Q[5], lm, lp, gtu[6];
          if (MC == MC_GEN) inv_sym3<T, true>(fm.gt, gtu);
          valencia<T, MC>(e, fm, gtu, isx ? 0 : 2, L, out.f, Q, lm, lp);
          out.speed = fmax(fabs(lm), fabs(lp));
        } else {
          face_flux<T, MC>(e, fm, isx ? 0 : 1, P.riemann, L, R, out);
        }
        cmax = fmax(cmax, (double)out.speed * (isx ? P.cx : P.cz));
        const bool on_edge = isx ? (j == 0 || j == nx) : (k == 0 || k == nz);
        if ((P.flux_reg && on_edge) || P.reg[0] || P.reg[1]) {
          double xx = isx ? g.x0 + j * g.dx : g.x0 + (j + 0.5) * g.dx;
          double fv[5] = {(double)out.f[0], (double)out.f[1], (double)out.f[2], (double)out.f[3],
                          (double)out.f[0] + (double)out.f[4]};
          if (cyl) fv[2] *= xx;
          if (P.flux_reg && on_edge) {
            int o = isx ? ((j == 0) ? k : nz + k) : 2 * nz + ((k == 0) ? j : nx + j);
            for (int m = 0; m < 5; m++) P.flux_reg[m * nb + o] = fv[m];
          }
          fmr_reg_add<TX, TZ>(P, isx, j, k, jj, kk, fv);
        }
      }
      for (int m = 0; m < 5; m++) sm.f[m][f] = out.f[m];
    }
  }
  __syncthreads();

  // ---- 3. divergence, sources, stage combination, diagnostics
  double mb = 0.0, jm = 0.0;
  constexpr int ND = ML ? CPT : 1;  // deferred recoveries (ML)
  bool d_act[ND];
  unsigned d_ic[ND];
  double d_W[ND], d_xc[ND], d_dV[ND], d_v[ND][5], d_gt[ND][6];
  if constexpr (ML) {
    for (int ci = 0; ci < CPT; ci++) {
      d_act[ci] = false;
      d_ic[ci] = 0u;
      d_W[ci] = 1.0;
      d_xc[ci] = g.x0 + 0.5 * g.dx;
      d_dV[ci] = 0.0;
      for (int m = 0; m < 5; m++) d_v[ci][m] = 0.0;
      for (int s = 0; s < 6; s++) d_gt[ci][s] = (s == 0 || s == 3 || s == 5) ? 1.0 : 0.0;
    }
  }
#pragma unroll
  for (int ci = 0; ci < CPT; ci++) {
    // per-cell arithmetic evaluated without contraction, so that every
    // compiled instance (single patch, batch) rounds identically
#pragma clang fp contract(off)
    int c = tid + ci * NT;
    int jj = c % TX, kk = c / TX;
    int j = j0 + jj, k = k0 + kk;
    if (!(c < TX * TZ && j >= 0 && j < nx && k < nz)) continue;
    const unsigned ic = cell_idx32(g, j, k);
    // state loads first: their latency overlaps the flux arithmetic below
    double qs5[5], qn5[5], ai5[5];
    for (int m = 0; m < 5; m++) qs5[m] = ld32(P.qs[m], ic);
    if (P.use_qn)
      for (int m = 0; m < 5; m++) qn5[m] = ld32(P.qn[m], ic);
    if (P.use_acc_in)
      for (int m = 0; m < 5; m++) ai5[m] = ld32(P.acc_in[m], ic);
    const int lc = (kk + 3) * HX + (jj + 3);
    double xc = g.x0 + (j + 0.5) * g.dx;
    const double xl = g.x0 + j * g.dx, xr = g.x0 + (j + 1) * g.dx;
    const int fl = kk * (TX + 1) + jj, fr = fl + 1;
    const int fb = S::NFX + kk * TX + jj, ft = fb + TX;
    const double ivx = cyl ? 1.0 / (xc * g.dx) : P.idx, ivz = P.idz;
    // metric at the cell and its x, z derivatives
    double gm[GRHD_NMET], dg[2 * GRHD_NMET];
    if (MC == MC_CF) {
      for (int i = 0; i < GRHD_NMET; i++) { gm[i] = P.m.c[i]; dg[i] = 0.0; dg[GRHD_NMET + i] = 0.0; }
      gm[GRHD_M_ALP] = sm.ma[lc];
      gm[GRHD_M_W] = sm.mw[lc];
      double a7[7];
      if (P.m.f[GRHD_M_ALP]) {
        for (int i = 0; i < 7; i++) a7[i] = sm.ma[lc - 3 + i];
        dg[GRHD_M_ALP] = deriv6(a7, i60dx);
        for (int i = 0; i < 7; i++) a7[i] = sm.ma[lc + (i - 3) * HX];
        dg[GRHD_NMET + GRHD_M_ALP] = deriv6(a7, i60dz);
      }
      if (P.m.f[GRHD_M_W]) {
        for (int i = 0; i < 7; i++) a7[i] = sm.mw[lc - 3 + i];
        dg[GRHD_M_W] = deriv6(a7, i60dx);
        for (int i = 0; i < 7; i++) a7[i] = sm.mw[lc + (i - 3) * HX];
        dg[GRHD_NMET + GRHD_M_W] = deriv6(a7, i60dz);
      }
    } else {
      for (int i = 0; i < GRHD_NMET; i++) {
        const double *src = P.m.f[i];
        if (!src) { gm[i] = P.m.c[i]; dg[i] = 0.0; dg[GRHD_NMET + i] = 0.0; continue; }
        if constexpr (S::MG) {
          if (i < S::NGM) {
            double a7[7];
            gm[i] = sm.mg[i][lc];
            for (int t = 0; t < 7; t++) a7[t] = sm.mg[i][lc - 3 + t];
            dg[i] = deriv6(a7, i60dx);
            for (int t = 0; t < 7; t++) a7[t] = sm.mg[i][lc + (t - 3) * HX];
            dg[GRHD_NMET + i] = deriv6(a7, i60dz);
            continue;
          }
        }
        gm[i] = ld32(src, ic);
        double a7[7];
        for (int t = 0; t < 7; t++) a7[t] = ld32(src, ic - 3u + (unsigned)t);
        dg[i] = deriv6(a7, i60dx);
        for (int t = 0; t < 7; t++) a7[t] = ld32(src, ic + (unsigned)((t - 3) * (int)g.pitch));
        dg[GRHD_NMET + i] = deriv6(a7, i60dz);
      }
    }
    double L[5];
    if (atm_fast) {
      // all-atmosphere tile: only the normal momenta carry a flux, and
      // only S_x and S_z have sources
      const double Fl = (double)sm.f[0][fl], Fr = (double)sm.f[0][fr];
      const double divx1 = cyl ? (xr * Fr - xl * Fl) * ivx : (Fr - Fl) * ivx;
      const double divz3 = ((double)sm.f[0][ft] - (double)sm.f[0][fb]) * ivz;
      double s[5];
      sources_atm_cf(gm, dg, xc, g.geom, e.P_atm, rhw2_atm, s);
      L[0] = 0.0; L[1] = s[1] - divx1; L[2] = 0.0; L[3] = s[3] - divz3; L[4] = 0.0;
    } else {
      const bool catm = tile_atm || sm.atm[lc];
      double pc[6];
      if (tile_atm) {
        pc[0] = e.rho_atm; pc[1] = 0.0; pc[2] = 0.0; pc[3] = 0.0; pc[4] = e.P_atm; pc[5] = e.eps_atm;
      } else if (sizeof(T) == sizeof(double)) {
        for (int i = 0; i < 6; i++) pc[i] = (double)sm.p[i][lc];  // own cells: no parity flip
      } else {
        for (int i = 0; i < 6; i++) pc[i] = ld32(P.p[i], ic);
      }
      double divx[5], divz[5];
      for (int m = 0; m < 5; m++) {
        double Fl, Fr;
        if (m == 4) {
          Fl = (double)sm.f[0][fl] + (double)sm.f[4][fl];
          Fr = (double)sm.f[0][fr] + (double)sm.f[4][fr];
        } else {
          Fl = (double)sm.f[m][fl];
          Fr = (double)sm.f[m][fr];
        }
        if (cyl) {
          if (m == 2) { Fl *= xl; Fr *= xr; }
          divx[m] = (xr * Fr - xl * Fl) * ivx;
        } else {
          divx[m] = (Fr - Fl) * ivx;
        }
      }
      for (int m = 0; m < 5; m++) {
        double Fb, Ft;
        if (m == 4) {
          Fb = (double)sm.f[0][fb] + (double)sm.f[4][fb];
          Ft = (double)sm.f[0][ft] + (double)sm.f[4][ft];
        } else {
          Fb = (double)sm.f[m][fb];
          Ft = (double)sm.f[m][ft];
        }
        if (cyl && m == 2) { Fb *= xc; Ft *= xc; }
        divz[m] = (Ft - Fb) * ivz;
      }
      double s[5];
      if (MC == MC_CF && catm) sources_atm_cf(gm, dg, xc, g.geom, e.P_atm, rhw2_atm, s);
      else sources<MC>(gm, dg, xc, g.geom, pc, s);
      for (int m = 0; m < 5; m++) L[m] = s[m] - divx[m] - divz[m];
    }
    double dV = cyl ? 2.0 * M_PI * xc * g.dx * g.dz : g.dx * g.dz;
    const bool fixed = P.fix_mask && ld32(P.fix_mask, ic);
    double v[5];
    for (int m = 0; m < 5; m++) {
      v[m] = P.b * qs5[m] + P.cdt * L[m];
      if (P.use_qn) v[m] += P.a * qn5[m];
      if (P.use_acc_in) v[m] += P.gdt * ai5[m];
      if (fixed) v[m] = ld32(P.fix_q[m], ic);
      if (!CHAIN) {
        st32(P.qo[m], ic, v[m]);
        if (m == 0) mb += v[m] * dV;
        if (m == 2) jm += v[m] * dV;
      }
      if (P.use_acc_out) {
        double av = P.e * L[m];
        if (P.use_acc_in) av += P.d * ai5[m];
        st32(P.acc_out[m], ic, av);
      }
    }
    if constexpr (ML) {
      d_act[ci] = true;
      d_ic[ci] = ic;
      d_W[ci] = gm[GRHD_M_W];
      d_xc[ci] = xc;
      d_dV[ci] = dV;
      for (int m = 0; m < 5; m++) d_v[ci][m] = v[m];
      for (int s = 0; s < 6; s++) d_gt[ci][s] = gm[GRHD_M_GXX + s];
    } else {
      finish_cell<MC, EK, CHAIN>(P, e, ic, gm[GRHD_M_W], gm + GRHD_M_GXX, xc, dV, v, mb, jm, acc);
    }
  }
  if constexpr (ML) {
    // every lane of the wave is here: the network spans the wave
    for (int ci = 0; ci < CPT; ci++)
      finish_cell_mlp<MC, EK>(P, e, d_act[ci], d_ic[ci], d_W[ci], d_gt[ci], d_xc[ci], d_dV[ci], d_v[ci], mb, jm,
                              acc);
  }

  cmax_out = cmax;
  mb_out = mb;
  jm_out = jm;
}

}  // namespace grhd
