// grhd_mlp.hpp -- the learned initial guess of the primitive recovery: a
// 3 -> 64 -> 64 -> 1 ReLU network with BF16 weights, evaluated per wave of
// 64 cells on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32
// accumulation).  The guess is never trusted: it only seeds a safeguarded
// FP64 Newton solve of the paper's master function, with the paper's
// Illinois bracketing as the fallback.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grhd.h"
#include "grhd_dev.hpp"

namespace grhd {

constexpr int MLP_H = 64;

// Device weight buffer (grhd_mlp_bytes() bytes), matrices in matrix-core
// operand order: the fragment that lane l (r = l % 16, g = l / 16) feeds to
// the 16x16x16 instruction for unit block mb (and input block kb) is four
// consecutive BF16 values, so a wave reads each operand as one contiguous
// 512-byte run.
//   W1op[mb][l][i] = W1[16 mb + r][4 g + i]   (inputs 3..15 are zero)
//   W2op[mb][kb][l][i] = W2[16 mb + r][16 kb + 4 g + i]
struct MlpDev {
  uint16_t W1op[4][64][4];
  uint16_t W2op[4][4][64][4];
  float b1[MLP_H], b2[MLP_H], w3[MLP_H];
  float b3;
  float xm[3], xs[3];         // feature standardisation (mean, std)
  float ym, ys;               // target scaling
  float pad[55];
};
static_assert(sizeof(MlpDev) % 16 == 0, "MlpDev is copied in 16-byte words");

// FP32 master parameter vector order (GRHD_MLP_NPARAM floats), same as the
// FP64 reference: W1[64][3], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 256, OFF_B2 = 4352, OFF_W3 = 4416, OFF_B3 = 4480;
constexpr int MLP_NPARAM = 4481;

__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ __forceinline__ float bf2f(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// four FP32 values to a BF16 operand fragment: two dwords, each a
// round-to-nearest-even pack of two values
__device__ __forceinline__ u32x2 pack4(float a, float b, float c, float d) {
  bf16x2v lo = {(__bf16)a, (__bf16)b}, hi = {(__bf16)c, (__bf16)d};
  return u32x2{__builtin_bit_cast(unsigned int, lo), __builtin_bit_cast(unsigned int, hi)};
}

__device__ __forceinline__ f32x4 mfma16(u32x2 a, u32x2 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, a), __builtin_bit_cast(bf16x4, b),
                                                   c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(u32x2 a_lo, u32x2 a_hi, u32x2 b_lo, u32x2 b_hi, f32x4 c) {
  u32x4 a = {a_lo.x, a_lo.y, a_hi.x, a_hi.y}, b = {b_lo.x, b_lo.y, b_hi.x, b_hi.y};
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a), __builtin_bit_cast(bf16v8, b), c,
                                                 0, 0, 0);
}

// Forward pass for the 64 lanes of a wave: lane l holds the standardised
// features (x0, x1, x2) of its cell and receives the network output.  All
// 64 lanes must execute this function (matrix-core operands span the wave).
// Layouts (wave64), r = l % 16, g = l / 16:
//   16x16x16: A lane l = A[r][4g+i], B lane l = B[4g+i][r], i < 4;
//   16x16x32: A lane l = A[r][8g+i], B lane l = B[8g+i][r], i < 8;
//   result (both): lane l = D[4g+i][r].
// With units as rows and cells as columns, a layer-1 result tile is, after
// ReLU, the 16x16x16 B operand of its 16 units.  Layer 2 uses the 16x16x32
// instruction (twice the rate on gfx950): its B operand is the pair of
// layer-1 tiles kb = 2p, 2p+1 side by side in each lane, which orders the
// 32 K indices of a lane group as (units 32p+4g..+3, units 32p+16+4g..+3);
// the W2 columns are loaded in that same order, and a sum over K does not
// depend on its order.  Biases enter as the accumulator's initial value.
// Operands are assembled from whole dwords (two BF16 each).
struct MlpRegs {
  u32x2 a1[4], a2[4][4];
  f32x4 c1[4], c2[4], o3[4];
  float b3;
};

// this lane's share of the weights, from a weight buffer in global memory
// or in LDS
__device__ __forceinline__ MlpRegs mlp_load(const MlpDev *__restrict__ w) {
  const int l = threadIdx.x & 63;
  const int g = l >> 4;
  MlpRegs R;
  for (int mb = 0; mb < 4; mb++) {
    R.a1[mb] = *(const u32x2 *)&w->W1op[mb][l][0];
    for (int kb = 0; kb < 4; kb++) R.a2[mb][kb] = *(const u32x2 *)&w->W2op[mb][kb][l][0];
    R.c1[mb] = *(const f32x4 *)&w->b1[mb * 16 + 4 * g];
    R.c2[mb] = *(const f32x4 *)&w->b2[mb * 16 + 4 * g];
    R.o3[mb] = *(const f32x4 *)&w->w3[mb * 16 + 4 * g];
  }
  R.b3 = w->b3;
  return R;
}

// copy of the weight buffer into LDS by a whole workgroup (every thread
// calls it; a barrier follows the copy)
template <int NTHR>
__device__ __forceinline__ void mlp_stage(const MlpDev *__restrict__ w, MlpDev *sw) {
  const u32x4 *src = (const u32x4 *)w;
  u32x4 *dst = (u32x4 *)sw;
  constexpr int N = sizeof(MlpDev) / 16;
  for (int i = threadIdx.x; i < N; i += NTHR) dst[i] = src[i];
  __syncthreads();
}

__device__ __forceinline__ float mlp_forward_regs(const MlpRegs &R, float x0, float x1, float x2) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, g = l >> 4;
  float y = 0.0f;
  for (int cb = 0; cb < 4; cb++) {
    // layer-1 input tile: inputs 0..2 of cells cb*16 + r live in lanes g = 0
    int src = cb * 16 + r;
    float f0 = __shfl(x0, src, 64), f1 = __shfl(x1, src, 64), f2 = __shfl(x2, src, 64);
    u32x2 xb = (g == 0) ? pack4(f0, f1, f2, 0.0f) : u32x2{0u, 0u};
    u32x2 h1[4];
    for (int mb = 0; mb < 4; mb++) {
      f32x4 acc = mfma16(R.a1[mb], xb, R.c1[mb]);
      h1[mb] = pack4(fmaxf(acc[0], 0.0f), fmaxf(acc[1], 0.0f), fmaxf(acc[2], 0.0f), fmaxf(acc[3], 0.0f));
    }
    float part = 0.0f;
    for (int mb = 0; mb < 4; mb++) {
      f32x4 acc = R.c2[mb];
      for (int p = 0; p < 2; p++)
        acc = mfma32(R.a2[mb][2 * p], R.a2[mb][2 * p + 1], h1[2 * p], h1[2 * p + 1], acc);
      for (int i = 0; i < 4; i++) part += R.o3[mb][i] * fmaxf(acc[i], 0.0f);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g == cb) y = part + R.b3;
  }
  return y;
}

__device__ __forceinline__ float mlp_forward_wave(const MlpDev *__restrict__ w, float x0, float x1,
                                                  float x2) {
  MlpRegs R = mlp_load(w);
  return mlp_forward_regs(R, x0, x1, x2);
}

// The learned guess for the cells of a wave: features (log10 D, S/E,
// log10(tau/D)) of the undensitised state (q densitised by W^-3; S_phi =
// x S_y on cylindrical grids), the network's log10(P/D), then
// z0 = v0 / sqrt(1 - v0^2) with v0 = S/(E + P0); -1 (no guess) where the
// state or the guess is out of range.  Every lane of the wave calls it; act
// marks the lanes that hold a cell (the others pass any finite values).
// W, gtu: conformal factor and inverse conformal metric at the cell (gtu
// used by the general class only), x: the cell's x.
template <int MC>
__device__ __forceinline__ double mlp_guess_wave(const MlpDev *__restrict__ w, bool act, double W,
                                                 const double *gtu, double x, int geom, const double *qq) {
  double W3 = W * W * W;
  double D = W3 * qq[0], E = W3 * qq[4];
  double Sx = W3 * qq[1], Sy = W3 * ((geom == GRHD_GEOM_CYLINDRICAL && act) ? qq[2] / x : qq[2]),
         Sz = W3 * qq[3];
  double S2;
  if (MC == MC_GEN) {
    double Sv[3] = {Sx, Sy, Sz};
    S2 = 0.0;
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) S2 += gtu[s3i(a, b)] * Sv[a] * Sv[b];
    S2 *= W * W;
  } else {
    S2 = W * W * (Sx * Sx + Sy * Sy + Sz * Sz);
  }
  const double tau = E - D;
  const bool good = act && D > 0.0 && E > 0.0 && tau > 0.0 && isfinite(S2) && isfinite(E);
  // features and guess in FP32 with the hardware's approximate log2, exp2,
  // reciprocal and square root: the guess only sets where the FP64 root
  // search starts
  const float Df = (float)D, Ef = (float)E, tauf = (float)tau;
  const float Sf = __builtin_amdgcn_sqrtf((float)S2);
  const float kLg = 0.30102999566f;  // log10(2)
  float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
  if (good) {
    const float iD = __builtin_amdgcn_rcpf(Df);
    f0 = (__builtin_amdgcn_logf(Df) * kLg - w->xm[0]) * __builtin_amdgcn_rcpf(w->xs[0]);
    f1 = (Sf * __builtin_amdgcn_rcpf(Ef) - w->xm[1]) * __builtin_amdgcn_rcpf(w->xs[1]);
    f2 = (__builtin_amdgcn_logf(tauf * iD) * kLg - w->xm[2]) * __builtin_amdgcn_rcpf(w->xs[2]);
  }
  float y = mlp_forward_wave(w, f0, f1, f2);
  double zg = -1.0;
  if (good) {
    const float P0 = Df * __builtin_amdgcn_exp2f((y * w->ys + w->ym) * 3.32192809489f);  // 10^x = 2^(x log2 10)
    const float v0 = Sf * __builtin_amdgcn_rcpf(Ef + P0);
    if (v0 >= 0.0f && v0 < 1.0f) zg = (double)(v0 * __builtin_amdgcn_rsqf(1.0f - v0 * v0));
  }
  return zg;
}

}  // namespace grhd
