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

namespace grhd {

constexpr int MLP_H = 64;

// Device weight buffer (grhd_mlp_bytes() bytes).  W1 is padded from 3 to
// 16 inputs so layer 1 is one MFMA K-step; rows are output units.
struct MlpDev {
  uint16_t W1[MLP_H * 16];    // bf16 [out][16], inputs 3..15 zero
  uint16_t W2[MLP_H * MLP_H]; // bf16 [out][in]
  float b1[MLP_H], b2[MLP_H], w3[MLP_H];
  float b3;
  float xm[3], xs[3];         // feature standardisation (mean, std)
  float ym, ys;               // target scaling
  float pad[53];
};

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
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// four FP32 values to a BF16 operand fragment (round to nearest even,
// hardware pack-converts)
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  __bf16 ha = (__bf16)a, hb = (__bf16)b, hc = (__bf16)c, hd = (__bf16)d;
  bf16x4 v;
  v[0] = __builtin_bit_cast(short, ha);
  v[1] = __builtin_bit_cast(short, hb);
  v[2] = __builtin_bit_cast(short, hc);
  v[3] = __builtin_bit_cast(short, hd);
  return v;
}

__device__ __forceinline__ bf16v8 cat8(bf16x4 lo, bf16x4 hi) {
  bf16v8 v;
  for (int i = 0; i < 4; i++) {
    v[i] = __builtin_bit_cast(__bf16, lo[i]);
    v[4 + i] = __builtin_bit_cast(__bf16, hi[i]);
  }
  return v;
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
__device__ __forceinline__ float mlp_forward_wave(const MlpDev *__restrict__ w, float x0, float x1,
                                                  float x2) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, g = l >> 4;
  bf16x4 a1[4];
  bf16v8 a2[4][2];
  f32x4 c1[4], c2[4], o3[4];
  for (int mb = 0; mb < 4; mb++) {
    const uint16_t *src = &w->W1[(mb * 16 + r) * 16 + 4 * g];
    a1[mb] = bf16x4{(short)src[0], (short)src[1], (short)src[2], (short)src[3]};
    for (int p = 0; p < 2; p++) {
      const uint16_t *lo = &w->W2[(mb * 16 + r) * MLP_H + 32 * p + 4 * g];
      const uint16_t *hi = lo + 16;
      a2[mb][p] = cat8(bf16x4{(short)lo[0], (short)lo[1], (short)lo[2], (short)lo[3]},
                       bf16x4{(short)hi[0], (short)hi[1], (short)hi[2], (short)hi[3]});
    }
    for (int i = 0; i < 4; i++) {
      int u = mb * 16 + 4 * g + i;
      c1[mb][i] = w->b1[u];
      c2[mb][i] = w->b2[u];
      o3[mb][i] = w->w3[u];
    }
  }
  const float b3 = w->b3;
  float y = 0.0f;
  for (int cb = 0; cb < 4; cb++) {
    // layer-1 input tile: inputs 0..2 of cells cb*16 + r live in lanes g = 0
    int src = cb * 16 + r;
    float f0 = __shfl(x0, src, 64), f1 = __shfl(x1, src, 64), f2 = __shfl(x2, src, 64);
    bf16x4 xb = (g == 0) ? pack4(f0, f1, f2, 0.0f) : bf16x4{0, 0, 0, 0};
    bf16x4 h1[4];
    for (int mb = 0; mb < 4; mb++) {
      f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[mb], xb, c1[mb], 0, 0, 0);
      h1[mb] = pack4(fmaxf(acc[0], 0.0f), fmaxf(acc[1], 0.0f), fmaxf(acc[2], 0.0f), fmaxf(acc[3], 0.0f));
    }
    bf16v8 hb[2] = {cat8(h1[0], h1[1]), cat8(h1[2], h1[3])};
    float part = 0.0f;
    for (int mb = 0; mb < 4; mb++) {
      f32x4 acc = c2[mb];
      for (int p = 0; p < 2; p++) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[mb][p], hb[p], acc, 0, 0, 0);
      for (int i = 0; i < 4; i++) part += o3[mb][i] * fmaxf(acc[i], 0.0f);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g == cb) y = part + b3;
  }
  return y;
}

}  // namespace grhd
