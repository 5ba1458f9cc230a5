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
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 v;
  v[0] = (short)f2bf(a);
  v[1] = (short)f2bf(b);
  v[2] = (short)f2bf(c);
  v[3] = (short)f2bf(d);
  return v;
}

// Forward pass for the 64 lanes of a wave: lane l holds the standardised
// features (x0, x1, x2) of its cell and receives the network output.  All
// 64 lanes must execute this function (matrix-core operands span the wave).
// MFMA 16x16x16 layouts (wave64): A operand lane l = A[l%16][4(l/16)+i],
// B operand lane l = B[4(l/16)+i][l%16], result lane l = D[4(l/16)+i][l%16].
// With units as rows and cells as columns, a layer's result tile is, after
// bias and ReLU, directly the B operand of the next layer.
__device__ __forceinline__ float mlp_forward_wave(const MlpDev *__restrict__ w, float x0, float x1,
                                                  float x2) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, g = l >> 4;
  // weights of both layers in operand layout (independent of the cells)
  bf16x4 a1[4], a2[4][4];
  for (int mb = 0; mb < 4; mb++) {
    const uint16_t *src = &w->W1[(mb * 16 + r) * 16 + 4 * g];
    a1[mb] = bf16x4{(short)src[0], (short)src[1], (short)src[2], (short)src[3]};
    for (int kb = 0; kb < 4; kb++) {
      const uint16_t *s2 = &w->W2[(mb * 16 + r) * MLP_H + kb * 16 + 4 * g];
      a2[mb][kb] = bf16x4{(short)s2[0], (short)s2[1], (short)s2[2], (short)s2[3]};
    }
  }
  float y = 0.0f;
  for (int cb = 0; cb < 4; cb++) {
    // layer-1 input tile: inputs 0..2 of cells cb*16 + r live in lanes g = 0
    int src = cb * 16 + r;
    float f0 = __shfl(x0, src, 64), f1 = __shfl(x1, src, 64), f2 = __shfl(x2, src, 64);
    bf16x4 xb = (g == 0) ? pack4(f0, f1, f2, 0.0f) : pack4(0.0f, 0.0f, 0.0f, 0.0f);
    bf16x4 h1[4];
    for (int mb = 0; mb < 4; mb++) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[mb], xb, acc, 0, 0, 0);
      float v[4];
      for (int i = 0; i < 4; i++) v[i] = fmaxf(acc[i] + w->b1[mb * 16 + 4 * g + i], 0.0f);
      h1[mb] = pack4(v[0], v[1], v[2], v[3]);
    }
    float part = 0.0f;
    for (int mb = 0; mb < 4; mb++) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int kb = 0; kb < 4; kb++)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[mb][kb], h1[kb], acc, 0, 0, 0);
      for (int i = 0; i < 4; i++) {
        int u = mb * 16 + 4 * g + i;
        part += w->w3[u] * fmaxf(acc[i] + w->b2[u], 0.0f);
      }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g == cb) y = part + w->b3;
  }
  return y;
}

}  // namespace grhd
