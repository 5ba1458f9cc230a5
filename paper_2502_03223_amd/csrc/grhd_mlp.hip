// grhd_mlp.hip -- the learned initial guess of the primitive recovery:
// inference on the matrix cores inside the recovery kernel, and the
// training kernels (per-sample forward and backward in FP32 with the BF16
// weights of the inference path, gradient reduction, Adam, packing).
#include <hip/hip_runtime.h>

#include <cmath>

#include "grhd.h"
#include "grhd_dev.hpp"
#include "grhd_diag.hpp"
#include "grhd_host.hpp"
#include "grhd_mlp.hpp"
#include "grhd_tile.hpp"

namespace grhd {

// ------------------------------------------------------------ inference

// standalone forward: X holds standardised features (n x 3), y receives
// the network output
__global__ void __launch_bounds__(256) k_mlp_forward(const MlpDev *w, const float *X, float *y, int n) {
  __shared__ MlpDev sw;
  mlp_stage<256>(w, &sw);
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = i < n;
  float x0 = act ? X[3 * i] : 0.0f, x1 = act ? X[3 * i + 1] : 0.0f, x2 = act ? X[3 * i + 2] : 0.0f;
  float o = mlp_forward_wave(&sw, x0, x1, x2);
  if (act) y[i] = o;
}

// Recovery of cell (j, k) seeded by the network: features (log10 D, S/E,
// log10(tau/D)), output log10(P/D); the guess P0 gives v0 = S/(E + P0) and
// z0 = v0 / sqrt(1 - v0^2), from which a safeguarded Newton solve starts.
// Every lane of the wave calls it (the network spans the wave); act marks
// the lanes that hold a cell.  q: the conserved fields (in; corrected where
// a flag is set), p: the primitives (out), flags: nullable.
template <int MC, int EK>
__device__ __forceinline__ void mlp_recover_cell(const EosK &e, const C2PK &cp, const MlpDev *w,
                                                 const GridK &g, const MetK &m, double *const *q,
                                                 double *const *p, uint8_t *flags, bool act, int j,
                                                 int k, unsigned &fl, int &iters) {
  long long i = cell_index(g, act ? j : 0, act ? k : 0);
  double qq[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, W = 1.0, gtu[6];
  double x = g.x0 + (j + 0.5) * g.dx;
  if (act) {
    W = mval(m, GRHD_M_W, i);
    for (int c = 0; c < 5; c++) qq[c] = q[c][i];
  }
  const double q0[5] = {qq[0], qq[1], qq[2], qq[3], qq[4]};
  if (MC == MC_GEN) {
    double gt[6];
    for (int t = 0; t < 6; t++) gt[t] = act ? mval(m, GRHD_M_GXX + t, i) : (t == 0 || t == 3 || t == 5);
    inv_sym3(gt, gtu);
  }
  // the guess (all lanes take part in the network evaluation)
  const double zg = mlp_guess_wave<MC>(w, act, W, gtu, x, g.geom, qq);
  fl = 0;
  iters = 0;
  if (act) {
    double pp[6];
    C2PResult res = con2prim_cell<MC, EK>(e, cp, W, gtu, x, g.geom, qq, pp, zg);
    fl = res.flags;
    iters = res.iters;
    if (fl) store_corrected(qq, q0, q, i);
    for (int c = 0; c < 6; c++) p[c][i] = pp[c];
    if (flags) flags[i] = (uint8_t)fl;
  }
}

// The single-patch recovery with the learned guess.  The workgroup stages
// the weights in LDS once; its waves read their operand fragments from
// there.
template <int MC, int EK>
__global__ void __launch_bounds__(256)
k_con2prim_mlp(GridK g, EosK e, C2PK cp, MetK m, Q5 q, P6 p, uint8_t *flags, C2PPart *part,
               int jlo, int jhi, int klo) {
  __shared__ unsigned long long red[4][6];
  __shared__ MlpDev sw;
  mlp_stage<256>((const MlpDev *)cp.mlp, &sw);
  int j = jlo + blockIdx.x * blockDim.x + threadIdx.x;
  int k = klo + blockIdx.y;
  bool act = j < jhi;
  bool jin = (j >= 0 && j < g.nx), kin = (k >= 0 && k < g.nz);
  if (!jin || !kin) {
    if (!jin && !kin) act = false;
    else if (!jin) act = act && g.bc[j < 0 ? 0 : 1] == GRHD_BC_EXTERNAL;
    else act = act && g.bc[k < 0 ? 2 : 3] == GRHD_BC_EXTERNAL;
  }
  unsigned fl;
  int iters;
  mlp_recover_cell<MC, EK>(e, cp, &sw, g, m, q.q, p.p, flags, act, j, k, fl, iters);
  if (part)
    c2p_block_partial<256>(act && jin && kin, fl, iters, &part[blockIdx.y * gridDim.x + blockIdx.x], red);
}

// The batched recovery with the learned guess: item = (patch, row,
// 256-cell segment) of a patch table, as the batch's plain recovery.
template <int MC, int EK>
__global__ void __launch_bounds__(256)
k_con2prim_batch_mlp(const PatchK *__restrict__ pt, const EosK *__restrict__ eos, C2PK cp,
                     const long long *__restrict__ item_prefix, int npatch, C2PPart *part) {
  __shared__ unsigned long long red[4][6];
  __shared__ MlpDev sw;
  mlp_stage<256>((const MlpDev *)cp.mlp, &sw);
  long long b = blockIdx.x;
  int lo = 0, hi = npatch - 1;
  while (lo < hi) {  // last patch whose first item <= b
    int mid = (lo + hi + 1) >> 1;
    if (item_prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const PatchK &P = pt[lo];
  long long li = b - item_prefix[lo];
  int segs = (P.g.nx + 255) / 256;
  int k = (int)(li / segs);
  int j = (int)(li % segs) * 256 + threadIdx.x;
  bool act = j < P.g.nx;
  unsigned fl;
  int iters;
  mlp_recover_cell<MC, EK>(eos[P.eos_id], cp, &sw, P.g, P.m, P.qs, P.p, P.flags, act, j, k, fl, iters);
  if (part) c2p_block_partial<256>(act, fl, iters, &part[blockIdx.x], red);
}

int launch_con2prim_batch_mlp(int mc, int ek, const PatchK *pt, const EosK *eos, const C2PK &cp,
                              const long long *item_prefix, int npatch, long long items, C2PPart *part,
                              hipStream_t st) {
  dim3 gi((unsigned)items);
  if (mc == MC_GEN && ek == GRHD_EOS_IDEAL)
    hipLaunchKernelGGL((k_con2prim_batch_mlp<MC_GEN, GRHD_EOS_IDEAL>), gi, dim3(256), 0, st, pt, eos, cp,
                       item_prefix, npatch, part);
  else if (mc == MC_GEN)
    hipLaunchKernelGGL((k_con2prim_batch_mlp<MC_GEN, GRHD_EOS_HYBRID>), gi, dim3(256), 0, st, pt, eos, cp,
                       item_prefix, npatch, part);
  else if (ek == GRHD_EOS_IDEAL)
    hipLaunchKernelGGL((k_con2prim_batch_mlp<MC_CF, GRHD_EOS_IDEAL>), gi, dim3(256), 0, st, pt, eos, cp,
                       item_prefix, npatch, part);
  else
    hipLaunchKernelGGL((k_con2prim_batch_mlp<MC_CF, GRHD_EOS_HYBRID>), gi, dim3(256), 0, st, pt, eos, cp,
                       item_prefix, npatch, part);
  return GRHD_OK;
}

template <int MC, int EK>
static void launch_mlp(dim3 grid, hipStream_t st, const GridK &g, const EosK &e, const C2PK &cp,
                       const MetK &m, const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part, int jlo,
                       int jhi, int klo) {
  hipLaunchKernelGGL((k_con2prim_mlp<MC, EK>), grid, dim3(256), 0, st, g, e, cp, m, q, p, flags, part,
                     jlo, jhi, klo);
}

int launch_con2prim_mlp_rect(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                             const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part, int jlo, int jhi,
                             int klo, int khi, hipStream_t st);

int launch_con2prim_mlp(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                        const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part, hipStream_t st) {
  int jlo = (g.bc[0] == GRHD_BC_EXTERNAL) ? -g.ng : 0;
  int jhi = (g.bc[1] == GRHD_BC_EXTERNAL) ? g.nx + g.ng : g.nx;
  int klo = (g.bc[2] == GRHD_BC_EXTERNAL) ? -g.ng : 0;
  int khi = (g.bc[3] == GRHD_BC_EXTERNAL) ? g.nz + g.ng : g.nz;
  return launch_con2prim_mlp_rect(g, e, cp, m, mc, q, p, flags, part, jlo, jhi, klo, khi, st);
}

// The same recovery over the cells [jlo, jhi) x [klo, khi) of the grid
// (cells outside the interior only on EXTERNAL sides); part: one record
// per workgroup, nullable.
int launch_con2prim_mlp_rect(const GridK &g, const EosK &e, const C2PK &cp, const MetK &m, int mc,
                             const Q5 &q, const P6 &p, uint8_t *flags, C2PPart *part, int jlo, int jhi,
                             int klo, int khi, hipStream_t st) {
  if (jhi <= jlo || khi <= klo) return GRHD_OK;
  dim3 grid((jhi - jlo + 255) / 256, khi - klo);
  bool ideal = e.kind == GRHD_EOS_IDEAL;
  if (mc == MC_GEN) {
    if (ideal) launch_mlp<MC_GEN, GRHD_EOS_IDEAL>(grid, st, g, e, cp, m, q, p, flags, part, jlo, jhi, klo);
    else launch_mlp<MC_GEN, GRHD_EOS_HYBRID>(grid, st, g, e, cp, m, q, p, flags, part, jlo, jhi, klo);
  } else {
    if (ideal) launch_mlp<MC_CF, GRHD_EOS_IDEAL>(grid, st, g, e, cp, m, q, p, flags, part, jlo, jhi, klo);
    else launch_mlp<MC_CF, GRHD_EOS_HYBRID>(grid, st, g, e, cp, m, q, p, flags, part, jlo, jhi, klo);
  }
  return launch_status("con2prim (learned guess)");
}

// ------------------------------------------------------------ training

// FP32 matrix-core instruction v_mfma_f32_16x16x4_f32 (wave64; r = l % 16,
// g = l / 16): A lane l = A[r][g], B lane l = B[g][r], result lane l =
// D[4g + v][r], v < 4 (the layout of the BF16 16x16x16 instruction with one
// K value per lane).
__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int GC = 16;      // samples per chunk: one matrix-core column block
constexpr int GWAVES = 4;   // waves per workgroup
constexpr int W2P = MLP_H + 1;

// Gradient of the MSE loss with the BF16-rounded weights of the inference
// path, FP32 arithmetic on the FP32 matrix cores.  A wave takes chunks of
// 16 samples (the columns of a 16x16 block); the hidden layers are 4 blocks
// of 16 units (the rows):
//   layer 1   H1 = ReLU(W1 X + b1)           4 instructions (K = 3, padded)
//   layer 2   H2 = ReLU(W2 H1 + b2)          64 (K = 64 units)
//   output    y = w3 . H2 + b3, dy = 2 (y - t) / n
//   backward  dH2 = dy w3 [H2 > 0]; dH1 = (W2^T dH2) [H1 > 0]     64
//             dW2 += dH2 H1^T over the chunk's samples           64 (K = 16)
// A result block holds units 4g + v of lane l's group for sample r, which
// is the B operand of the next product if its K indices are taken as
// (units 4g + v, g = 0..3) for fixed v: a sum over K does not depend on its
// order, and the weights are read in that order.  dW2 sums over samples,
// so H1 and dH2 go through LDS once per chunk to put units in the rows.
// The vector gradients (b1, b2, w3, b3, W1) are accumulated per lane and
// summed at the end; each workgroup folds its gradient in LDS and adds it
// to grad with one atomic per parameter.
__global__ void __launch_bounds__(64 * GWAVES)
k_mlp_grad(const float *__restrict__ P, const float *__restrict__ X, const float *__restrict__ t, int n,
           float *grad, float *loss) {
  __shared__ float sW2[MLP_H][W2P];
  __shared__ float sW1[MLP_H][4];
  __shared__ float sb1[MLP_H], sb2[MLP_H], sw3[MLP_H];
  __shared__ float sT[GWAVES][2][MLP_H][GC + 1];  // per wave: H1, dH2 as [unit][sample]
  __shared__ float sG[MLP_NPARAM];
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, r = l & 15, g = l >> 4;
  for (int i = tid; i < MLP_H * MLP_H; i += blockDim.x) sW2[i / MLP_H][i % MLP_H] = bf2f(f2bf(P[OFF_W2 + i]));
  for (int i = tid; i < MLP_H * 4; i += blockDim.x) {
    const int u = i / 4, k = i % 4;
    sW1[u][k] = (k < 3) ? bf2f(f2bf(P[OFF_W1 + u * 3 + k])) : 0.0f;
  }
  for (int i = tid; i < MLP_H; i += blockDim.x) {
    sb1[i] = P[OFF_B1 + i];
    sb2[i] = P[OFF_B2 + i];
    sw3[i] = P[OFF_W3 + i];
  }
  for (int i = tid; i < MLP_NPARAM; i += blockDim.x) sG[i] = 0.0f;
  const float b3 = P[OFF_B3];
  __syncthreads();
  f32x4 gW2[4][4];  // [mo][mb]: lane holds dW2[16 mo + 4g + v][16 mb + r]
  float gw3[4][4], gb2[4][4], gb1[4][4], gW1[4][4][3];
  for (int a = 0; a < 4; a++)
    for (int v = 0; v < 4; v++) {
      for (int b = 0; b < 4; b++) gW2[a][b][v] = 0.0f;
      gw3[a][v] = gb2[a][v] = gb1[a][v] = 0.0f;
      for (int k = 0; k < 3; k++) gW1[a][v][k] = 0.0f;
    }
  float gb3 = 0.0f, lsum = 0.0f;
  const float inv_n = 1.0f / (float)n;
  const int nchunk = (n + GC - 1) / GC;
  float(*TH)[GC + 1] = sT[wv][0];
  float(*TD)[GC + 1] = sT[wv][1];
  for (int ch = blockIdx.x * GWAVES + wv; ch < nchunk; ch += gridDim.x * GWAVES) {
    const int s = ch * GC + r;
    const bool act = s < n;
    float x[3];
    for (int k = 0; k < 3; k++) x[k] = act ? X[3 * s + k] : 0.0f;
    const float xb = (g == 0) ? x[0] : (g == 1) ? x[1] : (g == 2) ? x[2] : 0.0f;
    float h1[4][4], h2[4][4], d2[4][4];
    for (int mb = 0; mb < 4; mb++) {
      f32x4 c = {sb1[16 * mb + 4 * g], sb1[16 * mb + 4 * g + 1], sb1[16 * mb + 4 * g + 2], sb1[16 * mb + 4 * g + 3]};
      c = mfma4(sW1[16 * mb + r][g], xb, c);
      for (int v = 0; v < 4; v++) h1[mb][v] = fmaxf(c[v], 0.0f);
    }
    for (int mo = 0; mo < 4; mo++) {
      f32x4 c = {sb2[16 * mo + 4 * g], sb2[16 * mo + 4 * g + 1], sb2[16 * mo + 4 * g + 2], sb2[16 * mo + 4 * g + 3]};
      for (int mb = 0; mb < 4; mb++)
        for (int v = 0; v < 4; v++) c = mfma4(sW2[16 * mo + r][16 * mb + 4 * g + v], h1[mb][v], c);
      for (int v = 0; v < 4; v++) h2[mo][v] = fmaxf(c[v], 0.0f);
    }
    float part = 0.0f;
    for (int mo = 0; mo < 4; mo++)
      for (int v = 0; v < 4; v++) part += sw3[16 * mo + 4 * g + v] * h2[mo][v];
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    const float res = act ? part + b3 - t[s] : 0.0f;
    const float dy = 2.0f * res * inv_n;
    if (g == 0) {
      lsum += res * res;
      gb3 += dy;
    }
    for (int mo = 0; mo < 4; mo++)
      for (int v = 0; v < 4; v++) {
        gw3[mo][v] += dy * h2[mo][v];
        d2[mo][v] = (h2[mo][v] > 0.0f) ? dy * sw3[16 * mo + 4 * g + v] : 0.0f;
        gb2[mo][v] += d2[mo][v];
      }
    for (int mb = 0; mb < 4; mb++) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int mo = 0; mo < 4; mo++)
        for (int v = 0; v < 4; v++) c = mfma4(sW2[16 * mo + 4 * g + v][16 * mb + r], d2[mo][v], c);
      for (int v = 0; v < 4; v++) {
        const float d1 = (h1[mb][v] > 0.0f) ? c[v] : 0.0f;
        gb1[mb][v] += d1;
        for (int k = 0; k < 3; k++) gW1[mb][v][k] += d1 * x[k];
      }
    }
    // this wave's LDS block: the previous chunk's reads are done before
    // these writes, and these writes before the reads below
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int mb = 0; mb < 4; mb++)
      for (int v = 0; v < 4; v++) {
        TH[16 * mb + 4 * g + v][r] = h1[mb][v];
        TD[16 * mb + 4 * g + v][r] = d2[mb][v];
      }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < GC / 4; j++)
      for (int mo = 0; mo < 4; mo++) {
        const float a = TD[16 * mo + r][4 * j + g];
        for (int mb = 0; mb < 4; mb++) gW2[mo][mb] = mfma4(a, TH[16 * mb + r][4 * j + g], gW2[mo][mb]);
      }
  }
  // the vector gradients are summed over the 16 sample lanes of each lane
  // group first: LDS atomics on one address from many lanes serialise
  auto rsum16 = [](float x) {
    x += __shfl_xor(x, 1, 64);
    x += __shfl_xor(x, 2, 64);
    x += __shfl_xor(x, 4, 64);
    x += __shfl_xor(x, 8, 64);
    return x;
  };
  for (int mo = 0; mo < 4; mo++)
    for (int v = 0; v < 4; v++) {
      const int u = 16 * mo + 4 * g + v;
      for (int mb = 0; mb < 4; mb++) atomicAdd(&sG[OFF_W2 + u * MLP_H + 16 * mb + r], gW2[mo][mb][v]);
      const float a = rsum16(gw3[mo][v]), b = rsum16(gb2[mo][v]), c = rsum16(gb1[mo][v]);
      float w[3];
      for (int k = 0; k < 3; k++) w[k] = rsum16(gW1[mo][v][k]);
      if (r == 0) {
        atomicAdd(&sG[OFF_W3 + u], a);
        atomicAdd(&sG[OFF_B2 + u], b);
        atomicAdd(&sG[OFF_B1 + u], c);
        for (int k = 0; k < 3; k++) atomicAdd(&sG[OFF_W1 + u * 3 + k], w[k]);
      }
    }
  {
    const float b = rsum16(gb3);
    if (l == 0) atomicAdd(&sG[OFF_B3], b);
  }
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  if (loss && l == 0) atomicAdd(loss, lsum * inv_n);
  __syncthreads();
  for (int i = tid; i < MLP_NPARAM; i += blockDim.x) atomicAdd(&grad[i], sG[i]);
}

__global__ void k_fill0(float *a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master parameters
__global__ void k_adam(float *P, float *m, float *v, const float *g, float lr, float bc1, float bc2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  float gi = g[i];
  float mi = 0.9f * m[i] + 0.1f * gi;
  float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// FP32 parameters -> device weight buffer (BF16 matrices, FP32 vectors);
// scal (nullable): feature mean[3], std[3], target mean, std
__global__ void k_mlp_pack(MlpDev *w, const float *P, const float *scal) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4 * 64 * 4) {  // W1op[mb][l][e]
    int mb = i / 256, l = (i / 4) % 64, el = i % 4;
    int u = mb * 16 + (l & 15), k = 4 * (l >> 4) + el;
    w->W1op[mb][l][el] = (k < 3) ? f2bf(P[OFF_W1 + u * 3 + k]) : (uint16_t)0;
  }
  if (i < 4 * 4 * 64 * 4) {  // W2op[mb][kb][l][e]
    int mb = i / 1024, kb = (i / 256) % 4, l = (i / 4) % 64, el = i % 4;
    int u = mb * 16 + (l & 15), k = 16 * kb + 4 * (l >> 4) + el;
    w->W2op[mb][kb][l][el] = f2bf(P[OFF_W2 + u * MLP_H + k]);
  }
  if (i < MLP_H) {
    w->b1[i] = P[OFF_B1 + i];
    w->b2[i] = P[OFF_B2 + i];
    w->w3[i] = P[OFF_W3 + i];
  }
  if (i == 0) {
    w->b3 = P[OFF_B3];
    if (scal) {
      for (int k = 0; k < 3; k++) {
        w->xm[k] = scal[k];
        w->xs[k] = scal[3 + k];
      }
      w->ym = scal[6];
      w->ys = scal[7];
    }
  }
}

}  // namespace grhd

using namespace grhd;

extern "C" size_t grhd_mlp_bytes(void) { return sizeof(MlpDev); }

extern "C" int grhd_mlp_pack(void *mlp, const float *params, const float *scal, void *hip_stream) {
  if (!mlp || !params) return fail(GRHD_ERR_INVALID, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_mlp_pack, dim3((MLP_H * MLP_H + 255) / 256), dim3(256), 0, st, (MlpDev *)mlp, params,
                     scal);
  return launch_status("mlp pack");
}

// Training data: the unscaled features of the network (the definition the
// recovery kernels standardise) and the target log10(P/D) of one sample
// per thread, in FP64.
__global__ void __launch_bounds__(256)
k_mlp_features(Q5 q, long long n, const double *P, double *X, double *y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double D = q.q[0][i], E = q.q[4][i];
  const double S = sqrt(q.q[1][i] * q.q[1][i] + q.q[2][i] * q.q[2][i] + q.q[3][i] * q.q[3][i]);
  X[3 * i] = log10(D);
  X[3 * i + 1] = S / E;
  X[3 * i + 2] = log10((E - D) / D);
  if (y) y[i] = log10(P[i] / D);
}

extern "C" int grhd_mlp_features(const grhd_cons *q, long long n, const double *P, double *X, double *y,
                                 void *hip_stream) {
  if (!q || !X) return fail(GRHD_ERR_INVALID, "NULL argument");
  for (int c = 0; c < 5; c++)
    if (!q->q[c]) return fail(GRHD_ERR_INVALID, "q field %d is NULL", c);
  if (n < 0) return fail(GRHD_ERR_INVALID, "n must be >= 0");
  if ((P == nullptr) != (y == nullptr)) return fail(GRHD_ERR_INVALID, "P and y go together");
  if (n == 0) return GRHD_OK;
  if (n > (1LL << 38)) return fail(GRHD_ERR_UNSUPPORTED, "too many samples");  // grid x < 2^31
  Q5 qq;
  for (int c = 0; c < 5; c++) qq.q[c] = q->q[c];
  hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream,
                     qq, n, P, X, y);
  return launch_status("mlp features");
}

extern "C" int grhd_mlp_forward(const void *mlp, const float *X, float *y, int n, void *hip_stream) {
  if (!mlp || !X || !y) return fail(GRHD_ERR_INVALID, "NULL argument");
  if (n < 0) return fail(GRHD_ERR_INVALID, "n must be >= 0");
  if (n == 0) return GRHD_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, st, (const MlpDev *)mlp, X, y, n);
  return launch_status("mlp forward");
}

static int mlp_grad_launch(const float *params, float *grad, const float *X, const float *t, int n,
                           float *loss, hipStream_t st) {
  hipLaunchKernelGGL(k_fill0, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, grad, MLP_NPARAM);
  if (loss) hipLaunchKernelGGL(k_fill0, dim3(1), dim3(64), 0, st, loss, 1);
  // about four chunks of 16 samples per wave, at most 256 workgroups
  const long long nchunk = ((long long)n + GC - 1) / GC;
  const long long want = (nchunk + 4 * GWAVES - 1) / (4 * GWAVES);
  const int blocks = (int)(want < 256 ? want : 256);
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(64 * GWAVES), 0, st, params, X, t, n, grad, loss);
  return launch_status("mlp gradient");
}

extern "C" int grhd_mlp_grad(const float *params, float *grad, const float *X, const float *t, int n,
                             float *loss, void *hip_stream) {
  if (!params || !grad || !X || !t) return fail(GRHD_ERR_INVALID, "NULL argument");
  if (n < 1) return fail(GRHD_ERR_INVALID, "n must be >= 1");
  return mlp_grad_launch(params, grad, X, t, n, loss, (hipStream_t)hip_stream);
}

extern "C" int grhd_mlp_train_step(void *mlp, float *params, float *m, float *v, float *grad, const float *X,
                                   const float *t, int n, float lr, int step, float *loss, void *hip_stream) {
  if (!mlp || !params || !m || !v || !grad || !X || !t) return fail(GRHD_ERR_INVALID, "NULL argument");
  if (n < 1 || step < 1 || !(lr > 0.0f)) return fail(GRHD_ERR_INVALID, "need n >= 1, step >= 1, lr > 0");
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = mlp_grad_launch(params, grad, X, t, n, loss, st);
  if (rc) return rc;
  float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, params, m, v, grad, lr, bc1, bc2);
  if ((rc = launch_status("adam"))) return rc;
  hipLaunchKernelGGL(k_mlp_pack, dim3((MLP_H * MLP_H + 255) / 256), dim3(256), 0, st, (MlpDev *)mlp, params,
                     (const float *)nullptr);
  return launch_status("mlp pack");
}
