// grhd_batch.hip -- batched substep of many patches (fixed-mesh-refinement
// levels and independent instances of uneven sizes) in one graph-captured
// sequence: one recovery launch over all patches, one stage launch with a
// workgroup per (patch, tile) item, the diagnostic fold.  Two tile shapes
// are compiled into the stage kernel (thin patches with nz <= 8 and the
// rest); an autotuner measures the candidate shapes on the actual patches
// and caches the choice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "grhd.h"
#include "grhd_dev.hpp"
#include "grhd_host.hpp"
#include "grhd_tile.hpp"
#include "grhd_diag.hpp"

namespace grhd {

int launch_con2prim_batch_mlp(int mc, int ek, const PatchK *pt, const EosK *eos, const C2PK &cp,
                              const long long *item_prefix, int npatch, long long items, C2PPart *part,
                              hipStream_t st);
int fill_patch(const grhd_grid *grid, const grhd_metric *metric, const grhd_rk_stage *stage,
               const grhd_cons *qn, const grhd_cons *qs, const grhd_cons *qout, const grhd_prim *p,
               const grhd_cons *acc_in, const grhd_cons *acc_out, double *flux_reg, int recon,
               int riemann, PatchK &pk);

// ------------------------------------------------------------ kernels

// recovery over all patches: item = (patch, row, 256-cell segment)
template <int MC, int EK>
__global__ void __launch_bounds__(256)
k_con2prim_batch(const PatchK *__restrict__ pt, const EosK *__restrict__ eos, C2PK cp,
                 const long long *__restrict__ item_prefix, int npatch, C2PPart *part) {
  __shared__ unsigned long long red[4][6];
  long long b = blockIdx.x;
  int lo = 0, hi = npatch - 1;
  while (lo < hi) {  // last patch whose first item <= b
    int mid = (lo + hi + 1) >> 1;
    if (item_prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const PatchK &P = pt[lo];
  const EosK &e = eos[P.eos_id];
  long long li = b - item_prefix[lo];
  int segs = (P.g.nx + 255) / 256;
  int k = (int)(li / segs);
  int j = (int)(li % segs) * 256 + threadIdx.x;
  bool act = j < P.g.nx;
  unsigned fl = 0;
  int iters = 0;
  if (act) {
    long long i = cell_index(P.g, j, k);
    double W = mval(P.m, GRHD_M_W, i);
    double gtu[6];
    if (MC == MC_GEN) {
      double gt[6];
      for (int t = 0; t < 6; t++) gt[t] = mval(P.m, GRHD_M_GXX + t, i);
      inv_sym3(gt, gtu);
    }
    double qq[5], pp[6];
    for (int c = 0; c < 5; c++) qq[c] = P.qs[c][i];
    double q0[5] = {qq[0], qq[1], qq[2], qq[3], qq[4]};
    double x = P.g.x0 + (j + 0.5) * P.g.dx;
    C2PResult r = con2prim_cell<MC, EK>(e, cp, W, gtu, x, P.g.geom, qq, pp, -1.0);
    fl = r.flags;
    iters = r.iters;
    if (fl) store_corrected(qq, q0, P.qs, i);
    for (int c = 0; c < 6; c++) P.p[c][i] = pp[c];
    if (P.flags) P.flags[i] = (uint8_t)fl;
  }
  if (part) c2p_block_partial<256>(act, fl, iters, &part[blockIdx.x], red);
}

// Batched stage kernel: one workgroup per (patch, tile) item, item =
// workgroup index (patches in table order, tiles row-major), so the XCDs
// (dealt workgroups round-robin) each take every 8th item of every patch.
// Two tile shapes share the LDS: thin patches (nz <= 8) use AX x AZ, the
// others BX x BZ.  Each item writes one diagnostic record.
// Waves per SIMD the registers must allow: with both shapes 16 cells wide
// (16 x 16 or 16 x 8) the LDS of the conformally flat class fits three
// workgroups per CU in FP64 and four in FP32, as in the single-patch kernel.
template <class T, int MC, int AX, int AZ, int BX, int BZ>
constexpr int batch_waves() {
  constexpr bool narrow = AX == 16 && BX == 16 && (AZ == 8 || AZ == 16) && (BZ == 8 || BZ == 16);
  return (MC == MC_CF && narrow) ? (sizeof(T) == 8 ? 3 : 4) : 1;
}

template <class T, int MC, int AX, int AZ, int BX, int BZ>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(batch_waves<T, MC, AX, AZ, BX, BZ>())))
k_batch(const PatchK *__restrict__ pt, const EosK *__restrict__ eos,
        const long long *__restrict__ tile_prefix, int npatch, FluxPart *part2) {
  __shared__ double red[NT / 64][3];
  __shared__ union {
    TileSmem<T, MC, AX, AZ> a;
    TileSmem<T, MC, BX, BZ> b;
  } sm;
  const long long t = blockIdx.x;
  int lo = 0, hi = npatch - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tile_prefix[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const PatchK &P = pt[lo];
  int lt = (int)(t - tile_prefix[lo]);
  double cm, mb, jm;
  C2PAcc acc{};
  int tx, tz;
  tile_of(lt, P.tiles_x, P.tiles_z, tx, tz);
  if (P.g.nz <= 8)
    substep_tile<T, MC, AX, AZ>(P, eos[P.eos_id], tx, tz, sm.a, cm, mb, jm, acc);
  else
    substep_tile<T, MC, BX, BZ>(P, eos[P.eos_id], tx, tz, sm.b, cm, mb, jm, acc);
  flux_block_partial<NT>(cm, mb, jm, &part2[t], red);
}

using BatchFn = void (*)(const PatchK *, const EosK *, const long long *, int, FluxPart *);

// thin-patch shapes (nz <= 8) and square-patch shapes (indices are kept
// in tune caches: new shapes go at the end)
static const int kThin[3][2] = {{64, 8}, {32, 8}, {16, 8}};
static const int kSquare[5][2] = {{32, 8}, {32, 16}, {64, 8}, {16, 16}, {16, 8}};
static const int kNumThin = 3, kNumSquare = 5;

template <class T, int MC, int AX, int AZ>
static BatchFn pick_b(int b) {
  switch (b) {
    case 0: return k_batch<T, MC, AX, AZ, 32, 8>;
    case 1: return k_batch<T, MC, AX, AZ, 32, 16>;
    case 2: return k_batch<T, MC, AX, AZ, 64, 8>;
    case 3: return k_batch<T, MC, AX, AZ, 16, 16>;
    default: return k_batch<T, MC, AX, AZ, 16, 8>;
  }
}

template <class T, int MC>
static BatchFn pick_ab(int a, int b) {
  return a == 0 ? pick_b<T, MC, 64, 8>(b) : a == 1 ? pick_b<T, MC, 32, 8>(b) : pick_b<T, MC, 16, 8>(b);
}

static BatchFn batch_kernel(int prec, int mc, int a, int b) {
  if (prec == GRHD_PREC_MIXED)
    return mc == MC_GEN ? pick_ab<float, MC_GEN>(a, b) : pick_ab<float, MC_CF>(a, b);
  return mc == MC_GEN ? pick_ab<double, MC_GEN>(a, b) : pick_ab<double, MC_CF>(a, b);
}

}  // namespace grhd

using namespace grhd;

// ------------------------------------------------------------ plan

struct grhd_plan {
  int npatch = 0, neos = 0, prec = 0, mc = MC_CF, ek = GRHD_EOS_IDEAL;
  int shape_a = 0, shape_b = 0;
  grhd_options opts{};
  C2PK cp{};
  std::vector<int> nx, nz;
  std::vector<long long> tile_prefix, item_prefix;
  long long total_tiles = 0, total_items = 0;
  PatchK *d_patches = nullptr;
  EosK *d_eos = nullptr;
  long long *d_tile_prefix = nullptr, *d_item_prefix = nullptr;
  grhd_diag *d_diag = nullptr;      // used when the caller passes no diag
  static constexpr int kSlots = 4;
  PatchK *h_slots[kSlots] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t slot_ev[kSlots] = {};
  int slot = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  grhd_diag *graph_diag = nullptr;  // diag pointer baked into the graph
  C2PPart *d_part1 = nullptr;       // diagnostic records: recovery workgroups,
  FluxPart *d_part2 = nullptr;      // stage tiles
  FoldPart *d_lvl = nullptr;        // the fold's chunk results
  long long part2_cap = 0;
  uint8_t *d_flags = nullptr;       // recovery flags of every patch, read by
  std::vector<size_t> flag_off, flag_bytes;  // the stage (atmosphere tiles)
};

namespace {

int plan_tiles(grhd_plan *pl, int a, int b, std::vector<PatchK> &hp) {
  pl->tile_prefix.assign(pl->npatch, 0);
  long long acc = 0;
  for (int i = 0; i < pl->npatch; i++) {
    int tx, tz;
    if (hp[i].g.nz <= 8) { tx = kThin[a][0]; tz = kThin[a][1]; }
    else { tx = kSquare[b][0]; tz = kSquare[b][1]; }
    hp[i].xshift = tile_xshift(hp[i].g.ng, tx);
    hp[i].tiles_x = (hp[i].g.nx + hp[i].xshift + tx - 1) / tx;
    hp[i].tiles_z = (hp[i].g.nz + tz - 1) / tz;
    pl->tile_prefix[i] = acc;
    acc += (long long)hp[i].tiles_x * hp[i].tiles_z;
  }
  pl->total_tiles = acc;
  if (acc >= (1LL << 31)) return fail(GRHD_ERR_UNSUPPORTED, "more than 2^31 - 1 tiles in one plan");
  return GRHD_OK;
}

int build_patch_table(grhd_plan *pl, const grhd_patch *patches, std::vector<PatchK> &hp) {
  hp.resize(pl->npatch);
  for (int i = 0; i < pl->npatch; i++) {
    const grhd_patch &P = patches[i];
    if (P.eos_id < 0 || P.eos_id >= pl->neos) return fail(GRHD_ERR_INVALID, "patch %d: bad eos_id", i);
    if (P.grid.nx != pl->nx[i] || P.grid.nz != pl->nz[i])
      return fail(GRHD_ERR_INVALID, "patch %d shape differs from the plan", i);
    int rc = fill_patch(&P.grid, &P.metric, &P.stage, &P.qn, &P.qs, &P.qout, &P.p, nullptr, nullptr,
                        P.flux_reg, pl->opts.recon, pl->opts.riemann, hp[i]);
    if (rc) return rc;
    hp[i].face_eos = pl->opts.face_eps == GRHD_FACE_EPS_EOS ? 1 : 0;
    if (P.grid.bc[0] == GRHD_BC_EXTERNAL || P.grid.bc[1] == GRHD_BC_EXTERNAL ||
        P.grid.bc[2] == GRHD_BC_EXTERNAL || P.grid.bc[3] == GRHD_BC_EXTERNAL)
      return fail(GRHD_ERR_UNSUPPORTED, "patch %d: EXTERNAL boundaries are not batched", i);
    hp[i].eos_id = P.eos_id;
    size_t fb = (size_t)(P.grid.nz + 2 * P.grid.ng) * (size_t)P.grid.pitch;
    if (fb > pl->flag_bytes[i]) return fail(GRHD_ERR_INVALID, "patch %d layout differs from the plan", i);
    hp[i].flags = pl->d_flags ? pl->d_flags + pl->flag_off[i] : nullptr;
  }
  return GRHD_OK;
}

int capture_graph(grhd_plan *pl, grhd_diag *diag) {
  if (pl->exec) { hipGraphExecDestroy(pl->exec); pl->exec = nullptr; }
  if (pl->graph) { hipGraphDestroy(pl->graph); pl->graph = nullptr; }
  hipStream_t s = pl->cap_stream;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "graph capture begin failed");
  dim3 gi((unsigned)pl->total_items);
  C2PPart *p1 = pl->d_part1;
  if (pl->cp.guess == GRHD_GUESS_MLP)
    launch_con2prim_batch_mlp(pl->mc, pl->ek, pl->d_patches, pl->d_eos, pl->cp, pl->d_item_prefix, pl->npatch,
                              pl->total_items, p1, s);
  else if (pl->mc == MC_GEN && pl->ek == GRHD_EOS_IDEAL)
    hipLaunchKernelGGL((k_con2prim_batch<MC_GEN, GRHD_EOS_IDEAL>), gi, dim3(256), 0, s, pl->d_patches,
                       pl->d_eos, pl->cp, pl->d_item_prefix, pl->npatch, p1);
  else if (pl->mc == MC_GEN)
    hipLaunchKernelGGL((k_con2prim_batch<MC_GEN, GRHD_EOS_HYBRID>), gi, dim3(256), 0, s, pl->d_patches,
                       pl->d_eos, pl->cp, pl->d_item_prefix, pl->npatch, p1);
  else if (pl->ek == GRHD_EOS_IDEAL)
    hipLaunchKernelGGL((k_con2prim_batch<MC_CF, GRHD_EOS_IDEAL>), gi, dim3(256), 0, s, pl->d_patches,
                       pl->d_eos, pl->cp, pl->d_item_prefix, pl->npatch, p1);
  else
    hipLaunchKernelGGL((k_con2prim_batch<MC_CF, GRHD_EOS_HYBRID>), gi, dim3(256), 0, s, pl->d_patches,
                       pl->d_eos, pl->cp, pl->d_item_prefix, pl->npatch, p1);
  BatchFn fn = batch_kernel(pl->prec, pl->mc, pl->shape_a, pl->shape_b);
  hipLaunchKernelGGL(fn, dim3((unsigned)pl->total_tiles), dim3(NT), 0, s, pl->d_patches, pl->d_eos,
                     pl->d_tile_prefix, pl->npatch, pl->d_part2);
  launch_diag_final(pl->d_part1, (int)pl->total_items, pl->d_part2, (int)pl->total_tiles, pl->d_lvl, diag, s);
  hipError_t le = hipGetLastError();
  hipError_t err = hipStreamEndCapture(s, &pl->graph);
  if (le != hipSuccess || err != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : err));
  if (hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "graph instantiation failed");
  pl->graph_diag = diag;
  return GRHD_OK;
}

int upload_table(grhd_plan *pl, const std::vector<PatchK> &hp, hipStream_t st) {
  int s = pl->slot;
  pl->slot = (pl->slot + 1) % grhd_plan::kSlots;
  if (hipEventSynchronize(pl->slot_ev[s]) != hipSuccess) return fail(GRHD_ERR_DEVICE, "slot wait failed");
  std::memcpy(pl->h_slots[s], hp.data(), sizeof(PatchK) * pl->npatch);
  if (hipMemcpyAsync(pl->d_patches, pl->h_slots[s], sizeof(PatchK) * pl->npatch, hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "patch table upload failed");
  if (hipEventRecord(pl->slot_ev[s], st) != hipSuccess) return fail(GRHD_ERR_DEVICE, "event record failed");
  return GRHD_OK;
}

int set_shapes(grhd_plan *pl, int a, int b, const grhd_patch *patches) {
  std::vector<PatchK> hp;
  int rc = build_patch_table(pl, patches, hp);
  if (rc) return rc;
  pl->shape_a = a;
  pl->shape_b = b;
  if ((rc = plan_tiles(pl, a, b, hp))) return rc;
  if (hipMemcpy(pl->d_tile_prefix, pl->tile_prefix.data(), sizeof(long long) * pl->npatch,
                hipMemcpyHostToDevice) != hipSuccess)
    return fail(GRHD_ERR_DEVICE, "tile table upload failed");
  if (pl->total_tiles > pl->part2_cap) {
    hipFree(pl->d_part2);
    pl->d_part2 = nullptr;
    if (hipMalloc(&pl->d_part2, sizeof(FluxPart) * pl->total_tiles) != hipSuccess)
      return fail(GRHD_ERR_DEVICE, "plan allocation failed");
    pl->part2_cap = pl->total_tiles;
  }
  return capture_graph(pl, pl->d_diag);
}

double time_plan(grhd_plan *pl, const grhd_patch *patches, int reps) {
  std::vector<PatchK> hp;
  if (build_patch_table(pl, patches, hp)) return 1e30;
  plan_tiles(pl, pl->shape_a, pl->shape_b, hp);
  hipStream_t s = pl->cap_stream;
  if (upload_table(pl, hp, s)) return 1e30;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipGraphLaunch(pl->exec, s);  // warm
  hipEventRecord(e0, s);
  for (int r = 0; r < reps; r++) hipGraphLaunch(pl->exec, s);
  hipEventRecord(e1, s);
  hipEventSynchronize(e1);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms / reps;
}

std::string tune_key(const grhd_plan *pl) {
  hipDeviceProp_t prop;
  int dev = 0;
  hipGetDevice(&dev);
  hipGetDeviceProperties(&prop, dev);
  unsigned long long h = 1469598103934665603ull;
  for (int i = 0; i < pl->npatch; i++) {
    h = (h ^ (unsigned long long)pl->nx[i]) * 1099511628211ull;
    h = (h ^ (unsigned long long)pl->nz[i]) * 1099511628211ull;
  }
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|prec=%d|mc=%d|recon=%d|riemann=%d|face=%d|n=%d|%016llx",
           prop.gcnArchName, pl->prec, pl->mc, pl->opts.recon, pl->opts.riemann, pl->opts.face_eps,
           pl->npatch, h);
  return buf;
}

bool cache_lookup(const char *path, const std::string &key, int *a, int *b) {
  if (!path) return false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[400];
    int ia, ib;
    if (sscanf(line, "%399s %d %d", k, &ia, &ib) == 3 && key == k && ia >= 0 && ia < kNumThin && ib >= 0 &&
        ib < kNumSquare) {
      *a = ia;
      *b = ib;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char *path, const std::string &key, int a, int b, double ms) {
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %.6f\n", key.c_str(), a, b, ms);
  fclose(f);
}

void destroy_plan(grhd_plan *pl) {
  if (!pl) return;
  if (pl->exec) hipGraphExecDestroy(pl->exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  for (int s = 0; s < grhd_plan::kSlots; s++) {
    if (pl->slot_ev[s]) hipEventDestroy(pl->slot_ev[s]);
    if (pl->h_slots[s]) hipHostFree(pl->h_slots[s]);
  }
  if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
  hipFree(pl->d_patches);
  hipFree(pl->d_eos);
  hipFree(pl->d_tile_prefix);
  hipFree(pl->d_item_prefix);
  hipFree(pl->d_diag);
  hipFree(pl->d_part1);
  hipFree(pl->d_part2);
  hipFree(pl->d_lvl);
  hipFree(pl->d_flags);
  delete pl;
}

}  // namespace

extern "C" int grhd_plan_create(const grhd_patch *patches, int npatch, const grhd_eos *eos_table,
                                int neos, const grhd_options *opts, const char *tune_cache,
                                grhd_plan **out) {
  int rc;
  if (!out) return fail(GRHD_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!patches || npatch < 1) return fail(GRHD_ERR_INVALID, "need at least one patch");
  if (!eos_table || neos < 1) return fail(GRHD_ERR_INVALID, "need at least one EOS");
  if (!opts) return fail(GRHD_ERR_INVALID, "opts is NULL");
  if ((rc = check_c2p(&opts->c2p)) || (rc = check_face_eps(opts->face_eps))) return rc;
  if (opts->prec != GRHD_PREC_FP64 && opts->prec != GRHD_PREC_MIXED) return fail(GRHD_ERR_INVALID, "bad prec");
  for (int i = 0; i < neos; i++)
    if ((rc = check_eos(&eos_table[i]))) return rc;
  grhd_plan *pl = new grhd_plan();
  for (int i = 0; i < neos; i++)
    if (eos_table[i].kind == GRHD_EOS_HYBRID) pl->ek = GRHD_EOS_HYBRID;
  pl->npatch = npatch;
  pl->neos = neos;
  pl->prec = opts->prec;
  pl->opts = *opts;
  pl->cp = to_c2pk(&opts->c2p);
  pl->mc = MC_CF;
  size_t flag_total = 0;
  for (int i = 0; i < npatch; i++) {
    if ((rc = check_metric(&patches[i].metric))) { destroy_plan(pl); return rc; }
    if (metric_class(&patches[i].metric) == MC_GEN) pl->mc = MC_GEN;
    pl->nx.push_back(patches[i].grid.nx);
    pl->nz.push_back(patches[i].grid.nz);
    pl->flag_off.push_back(flag_total);
    size_t fb = (size_t)(patches[i].grid.nz + 2 * patches[i].grid.ng) * (size_t)patches[i].grid.pitch;
    pl->flag_bytes.push_back(fb);
    flag_total += (fb + 255) & ~(size_t)255;
  }
  std::vector<PatchK> hp;
  if ((rc = build_patch_table(pl, patches, hp))) { destroy_plan(pl); return rc; }
  // recovery items: (patch, row, 256-cell segment)
  pl->item_prefix.assign(npatch, 0);
  long long acc = 0;
  for (int i = 0; i < npatch; i++) {
    pl->item_prefix[i] = acc;
    acc += (long long)pl->nz[i] * ((pl->nx[i] + 255) / 256);
  }
  pl->total_items = acc;
  std::vector<EosK> he(neos);
  for (int i = 0; i < neos; i++) he[i] = to_eosk(&eos_table[i], opts->c2p.rho_atm);
  bool okm = hipMalloc(&pl->d_patches, sizeof(PatchK) * npatch) == hipSuccess &&
             hipMalloc(&pl->d_eos, sizeof(EosK) * neos) == hipSuccess &&
             hipMalloc(&pl->d_tile_prefix, sizeof(long long) * npatch) == hipSuccess &&
             hipMalloc(&pl->d_item_prefix, sizeof(long long) * npatch) == hipSuccess &&
             hipMalloc(&pl->d_diag, sizeof(grhd_diag)) == hipSuccess &&
             hipMalloc(&pl->d_part1, sizeof(C2PPart) * pl->total_items) == hipSuccess &&
             hipMalloc(&pl->d_lvl, sizeof(FoldPart) * kFoldMax) == hipSuccess &&
             hipMalloc(&pl->d_flags, flag_total) == hipSuccess &&
             hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) == hipSuccess;
  for (int s = 0; okm && s < grhd_plan::kSlots; s++)
    okm = hipHostMalloc((void **)&pl->h_slots[s], sizeof(PatchK) * npatch, hipHostMallocDefault) == hipSuccess &&
          hipEventCreateWithFlags(&pl->slot_ev[s], hipEventDisableTiming) == hipSuccess;
  if (!okm) { destroy_plan(pl); return fail(GRHD_ERR_DEVICE, "plan allocation failed"); }
  okm = hipMemcpy(pl->d_eos, he.data(), sizeof(EosK) * neos, hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(pl->d_item_prefix, pl->item_prefix.data(), sizeof(long long) * npatch,
                  hipMemcpyHostToDevice) == hipSuccess;
  if (!okm) { destroy_plan(pl); return fail(GRHD_ERR_DEVICE, "plan upload failed"); }

  // tile shapes: cache, explicit option, or measured on the given patches
  std::string key = tune_key(pl);
  int a = 0, b = 0;
  bool have_thin = false, have_sq = false;
  for (int i = 0; i < npatch; i++) (pl->nz[i] <= 8 ? have_thin : have_sq) = true;
  if (opts->tile_x || opts->tile_z) {
    for (int i = 0; i < kNumSquare; i++)
      if (kSquare[i][0] == opts->tile_x && kSquare[i][1] == opts->tile_z) b = i;
    for (int i = 0; i < kNumThin; i++)
      if (kThin[i][0] == opts->tile_x && kThin[i][1] == opts->tile_z) a = i;
  } else if (!cache_lookup(tune_cache, key, &a, &b)) {
    // every (thin, square) pair: the kernel's LDS and registers are those
    // of both shapes together, so one shape's best depends on the other
    double best = 1e30;
    int ba = 0, bb = 0;
    for (int ia = 0; ia < (have_thin ? kNumThin : 1); ia++)
      for (int ib = 0; ib < (have_sq ? kNumSquare : 1); ib++) {
        if ((rc = set_shapes(pl, ia, ib, patches))) { destroy_plan(pl); return rc; }
        double ms = time_plan(pl, patches, 5);
        if (ms < best) { best = ms; ba = ia; bb = ib; }
      }
    a = ba;
    b = bb;
    cache_store(tune_cache, key, a, b, best);
  }
  if ((rc = set_shapes(pl, a, b, patches))) { destroy_plan(pl); return rc; }
  if (hipStreamSynchronize(pl->cap_stream) != hipSuccess) {
    destroy_plan(pl);
    return fail(GRHD_ERR_DEVICE, "plan setup failed");
  }
  *out = pl;
  return GRHD_OK;
}

extern "C" int grhd_batch_levels(grhd_plan *pl, const grhd_patch *patches, int npatch, grhd_diag *diag,
                                 void *hip_stream) {
  int rc;
  if (!pl) return fail(GRHD_ERR_INVALID, "plan is NULL");
  if (!patches || npatch != pl->npatch) return fail(GRHD_ERR_INVALID, "patch count differs from the plan");
  std::vector<PatchK> hp;
  if ((rc = build_patch_table(pl, patches, hp))) return rc;
  plan_tiles(pl, pl->shape_a, pl->shape_b, hp);
  hipStream_t st = (hipStream_t)hip_stream;
  grhd_diag *d = diag ? diag : pl->d_diag;
  if (d != pl->graph_diag && (rc = capture_graph(pl, d))) return rc;
  if ((rc = upload_table(pl, hp, st))) return rc;
  if (hipGraphLaunch(pl->exec, st) != hipSuccess) return fail(GRHD_ERR_DEVICE, "graph launch failed");
  return GRHD_OK;
}

extern "C" int grhd_plan_destroy(grhd_plan *pl) {
  if (!pl) return fail(GRHD_ERR_INVALID, "plan is NULL");
  hipDeviceSynchronize();
  destroy_plan(pl);
  return GRHD_OK;
}

extern "C" int grhd_autotune(const grhd_patch *patches, int npatch, const grhd_eos *eos_table, int neos,
                             const grhd_options *opts, const char *tune_cache, int *tile_x, int *tile_z) {
  if (!tile_x || !tile_z) return fail(GRHD_ERR_INVALID, "NULL argument");
  grhd_plan *pl = nullptr;
  int rc = grhd_plan_create(patches, npatch, eos_table, neos, opts, tune_cache, &pl);
  if (rc) return rc;
  rc = grhd_plan_tile(pl, tile_x, tile_z);
  grhd_plan_destroy(pl);
  return rc;
}

extern "C" int grhd_plan_tile(const grhd_plan *pl, int *tile_x, int *tile_z) {
  if (!pl || !tile_x || !tile_z) return fail(GRHD_ERR_INVALID, "NULL argument");
  tile_x[0] = kSquare[pl->shape_b][0];
  tile_z[0] = kSquare[pl->shape_b][1];
  tile_x[1] = kThin[pl->shape_a][0];
  tile_z[1] = kThin[pl->shape_a][1];
  return GRHD_OK;
}
