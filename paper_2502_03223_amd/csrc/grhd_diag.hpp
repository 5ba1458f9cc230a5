// grhd_diag.hpp -- diagnostics without contended atomics: every workgroup
// reduces its cells (wave shuffles, then LDS) and writes one partial record
// to a scratch array; one single-workgroup kernel folds the records in a
// fixed order and overwrites the caller's grhd_diag.
#pragma once

#include "grhd_dev.hpp"

namespace grhd {

struct C2PPart { unsigned long long n[6]; };   // rescale, cold, atm, fail, iter sum, iter max
struct FluxPart { double cmax, mb, jm, pad; };

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// workgroup partial of the recovery statistics; all threads must call it
template <int NTHR>
__device__ __forceinline__ void c2p_block_partial(bool act, unsigned fl, int iters, C2PPart *out,
                                                  unsigned long long (*red)[6]) {
  unsigned long long v[6];
  v[0] = __popcll(__ballot(act && (fl & GRHD_FLAG_RESCALE)));
  v[1] = __popcll(__ballot(act && (fl & GRHD_FLAG_COLD)));
  v[2] = __popcll(__ballot(act && (fl & GRHD_FLAG_ATM)));
  v[3] = __popcll(__ballot(act && (fl & GRHD_FLAG_FAIL)));
  unsigned long long it = act ? (unsigned long long)iters : 0ull;
  v[4] = wave_sum_u64(it);
  v[5] = wave_max_u64(it);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < 6; i++) red[w][i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    C2PPart p;
    for (int i = 0; i < 6; i++) p.n[i] = red[0][i];
    for (int ww = 1; ww < NTHR / 64; ww++) {
      for (int i = 0; i < 5; i++) p.n[i] += red[ww][i];
      p.n[5] = red[ww][5] > p.n[5] ? red[ww][5] : p.n[5];
    }
    *out = p;
  }
}

// workgroup partial of the stage diagnostics (max Courant number, sums of
// q_D dV and q_Sphi dV); all threads must call it
template <int NTHR>
__device__ __forceinline__ void flux_block_partial(double cmax, double mb, double jm, FluxPart *out,
                                                   double (*red)[3]) {
  for (int o = 32; o > 0; o >>= 1) {
    cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
    mb += __shfl_xor(mb, o, 64);
    jm += __shfl_xor(jm, o, 64);
  }
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = cmax;
    red[w][1] = mb;
    red[w][2] = jm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    FluxPart p{red[0][0], red[0][1], red[0][2], 0.0};
    for (int ww = 1; ww < NTHR / 64; ww++) {
      p.cmax = fmax(p.cmax, red[ww][0]);
      p.mb += red[ww][1];
      p.jm += red[ww][2];
    }
    *out = p;
  }
}

// fold n1 recovery records and n2 stage records into diag (fixed order);
// defined once in grhd_kernels.hip
int launch_diag_final(const C2PPart *p1, int n1, const FluxPart *p2, int n2, grhd_diag *diag,
                      hipStream_t st);

}  // namespace grhd
