// grhd_diag.hpp -- diagnostics without atomics: every workgroup of the
// recovery and every tile of the stage kernel reduces its cells (wave
// shuffles, then LDS) and writes one partial record to a scratch array; a
// first kernel folds contiguous chunks of the records in parallel, a
// second one wave folds the chunks in a fixed order and overwrites the
// caller's grhd_diag.
#pragma once

#include "grhd_dev.hpp"

namespace grhd {

struct C2PPart { unsigned long long n[6]; };   // rescale, cold, atm, fail, iter sum, iter max
struct FluxPart { double cmax, mb, jm, pad; };

// A 64-bit integer moved across lanes by one DPP pattern (both halves).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, true);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int lane) {
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)v, lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

constexpr int kDppQuad1032 = 0xB1, kDppQuad2301 = 0x4E, kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;

// Wave sum and maximum of 64-bit integers without LDS: within each row of
// 16 lanes by DPP (swap neighbours, swap pairs, mirror half rows, mirror
// rows), then the four row results.  All 64 lanes must be active; the
// result is uniform.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  v += dpp_u64<kDppQuad1032>(v);
  v += dpp_u64<kDppQuad2301>(v);
  v += dpp_u64<kDppRowHalfMirror>(v);
  v += dpp_u64<kDppRowMirror>(v);
  return lane_u64(v, 0) + lane_u64(v, 16) + lane_u64(v, 32) + lane_u64(v, 48);
}

__device__ __forceinline__ unsigned long long u64max(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  v = u64max(v, dpp_u64<kDppQuad1032>(v));
  v = u64max(v, dpp_u64<kDppQuad2301>(v));
  v = u64max(v, dpp_u64<kDppRowHalfMirror>(v));
  v = u64max(v, dpp_u64<kDppRowMirror>(v));
  return u64max(u64max(lane_u64(v, 0), lane_u64(v, 16)), u64max(lane_u64(v, 32), lane_u64(v, 48)));
}

// A double moved across lanes by one DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Wave sum and maximum of doubles in a fixed order, without LDS: within
// each row of 16 lanes by DPP (swap neighbours, swap pairs, mirror half
// rows, mirror rows: each step combines two equal-sized groups, so every
// lane of a row ends with the same bits), then the four row results in
// order.  All 64 lanes must be active; the result is uniform.
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<kDppQuad1032>(v);
  v += dpp_f64<kDppQuad2301>(v);
  v += dpp_f64<kDppRowHalfMirror>(v);
  v += dpp_f64<kDppRowMirror>(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<kDppQuad1032>(v));
  v = fmax(v, dpp_f64<kDppQuad2301>(v));
  v = fmax(v, dpp_f64<kDppRowHalfMirror>(v));
  v = fmax(v, dpp_f64<kDppRowMirror>(v));
  return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// Sum and maximum over the wave of small non-negative integers, exact, by
// bit planes: plane b contributes 2^b times the number of lanes with bit b
// set (a ballot and a bit count, no LDS traffic); the planes run while any
// lane has bits left, a loop that is uniform over the wave.
__device__ __forceinline__ unsigned long long wave_sum_small(unsigned long long v) {
  unsigned long long s = 0;
  for (int b = 0; b < 64 && __ballot((v >> b) != 0); b++)
    s += (unsigned long long)__popcll(__ballot((v >> b) & 1)) << b;
  return s;
}

__device__ __forceinline__ unsigned long long wave_max_small(unsigned long long v) {
  int top = 0;  // planes in use
  while (top < 64 && __ballot((v >> top) != 0)) top++;
  // from the highest plane down, keep the lanes that agree with the
  // maximum found so far
  bool alive = true;
  unsigned long long m = 0;
  for (int b = top - 1; b >= 0; b--) {
    const bool bit = ((v >> b) & 1) != 0;
    if (__ballot(alive && bit)) {
      m |= 1ull << b;
      alive = alive && bit;
    }
  }
  return m;
}

// workgroup partial of per-thread recovery statistics v[6] (counts and
// iteration sum are summed, the iteration maximum is maxed); all threads
// must call it
template <int NTHR>
__device__ __forceinline__ void c2p_counts_partial(const unsigned long long *v6, C2PPart *out,
                                                   unsigned long long (*red)[6]) {
  unsigned long long v[6];
  for (int i = 0; i < 5; i++) v[i] = wave_sum_small(v6[i]);
  v[5] = wave_max_small(v6[5]);
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

// workgroup partial of the recovery statistics, one cell per thread; all
// threads must call it
template <int NTHR>
__device__ __forceinline__ void c2p_block_partial(bool act, unsigned fl, int iters, C2PPart *out,
                                                  unsigned long long (*red)[6]) {
  unsigned long long v[6];
  v[0] = (act && (fl & GRHD_FLAG_RESCALE)) ? 1ull : 0ull;
  v[1] = (act && (fl & GRHD_FLAG_COLD)) ? 1ull : 0ull;
  v[2] = (act && (fl & GRHD_FLAG_ATM)) ? 1ull : 0ull;
  v[3] = (act && (fl & GRHD_FLAG_FAIL)) ? 1ull : 0ull;
  v[4] = act ? (unsigned long long)iters : 0ull;
  v[5] = v[4];
  c2p_counts_partial<NTHR>(v, out, red);
}

// workgroup partial of the stage diagnostics (max Courant number, sums of
// q_D dV and q_Sphi dV); all threads must call it
template <int NTHR>
__device__ __forceinline__ void flux_block_partial(double cmax, double mb, double jm, FluxPart *out,
                                                   double (*red)[3]) {
  cmax = wave_max_f64(cmax);
  mb = wave_sum_f64(mb);
  jm = wave_sum_f64(jm);
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

// A folded set of records.
struct FoldPart {
  unsigned long long n[6];
  double cmax, mb, jm;
};

// Fold records p1[0..n1) and p2[0..n2) by one whole workgroup of NTHR
// threads (every thread must call it); the result is valid in thread 0.
// red: NTHR/64 x 9 words of LDS.  Thread t folds records t, t + NTHR, ...
// of both arrays; the loads of up to four records of each array are
// issued together before any is used, so a small fold is one memory round
// trip.  The waves reduce by shuffles and thread 0 combines the wave
// results in wave order: the result depends only on the record counts.
template <int NTHR>
__device__ FoldPart fold_records(const C2PPart *p1, int n1, const FluxPart *p2, int n2,
                                 unsigned long long (*red)[9]) {
  int t = threadIdx.x;
  unsigned long long a[6] = {0, 0, 0, 0, 0, 0};
  double c = 0.0, mb = 0.0, jm = 0.0;
  const int nmax = n1 > n2 ? n1 : n2;
  for (int i0 = t; i0 < nmax; i0 += 4 * NTHR) {
    C2PPart r1[4];
    FluxPart r2[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if (i0 + u * NTHR < n1) r1[u] = p1[i0 + u * NTHR];
      if (i0 + u * NTHR < n2) r2[u] = p2[i0 + u * NTHR];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if (i0 + u * NTHR < n1) {
        for (int k = 0; k < 5; k++) a[k] += r1[u].n[k];
        a[5] = r1[u].n[5] > a[5] ? r1[u].n[5] : a[5];
      }
      if (i0 + u * NTHR < n2) {
        c = fmax(c, r2[u].cmax);
        mb += r2[u].mb;
        jm += r2[u].jm;
      }
    }
  }
  for (int k = 0; k < 5; k++) a[k] = wave_sum_u64(a[k]);
  a[5] = wave_max_u64(a[5]);
  c = wave_max_f64(c);
  mb = wave_sum_f64(mb);
  jm = wave_sum_f64(jm);
  int w = t >> 6;
  if ((t & 63) == 0) {
    for (int k = 0; k < 6; k++) red[w][k] = a[k];
    red[w][6] = (unsigned long long)__double_as_longlong(c);
    red[w][7] = (unsigned long long)__double_as_longlong(mb);
    red[w][8] = (unsigned long long)__double_as_longlong(jm);
  }
  __syncthreads();
  FoldPart f{};
  if (t == 0) {
    for (int k = 0; k < 6; k++) f.n[k] = red[0][k];
    f.cmax = __longlong_as_double((long long)red[0][6]);
    f.mb = __longlong_as_double((long long)red[0][7]);
    f.jm = __longlong_as_double((long long)red[0][8]);
    for (int ww = 1; ww < NTHR / 64; ww++) {
      for (int k = 0; k < 5; k++) f.n[k] += red[ww][k];
      f.n[5] = red[ww][5] > f.n[5] ? red[ww][5] : f.n[5];
      f.cmax = fmax(f.cmax, __longlong_as_double((long long)red[ww][6]));
      f.mb += __longlong_as_double((long long)red[ww][7]);
      f.jm += __longlong_as_double((long long)red[ww][8]);
    }
  }
  return f;
}

// Fold of the folded sets f[0..n) (n <= 64) by one wave in a fixed order;
// the result is valid in lane 0 and depends only on n.
__device__ __forceinline__ FoldPart fold_wave(const FoldPart *f, int n) {
  const int t = threadIdx.x;
  FoldPart a{};
  if (t < n) a = f[t];
  for (int k = 0; k < 5; k++) a.n[k] = wave_sum_u64(a.n[k]);
  a.n[5] = wave_max_u64(a.n[5]);
  a.cmax = wave_max_f64(a.cmax);
  a.mb = wave_sum_f64(a.mb);
  a.jm = wave_sum_f64(a.jm);
  return a;
}

// fold into *diag (two small launches: chunks of the records in parallel,
// then the chunks in order); defined once in grhd_kernels.hip
// lvl: kFoldMax folded sets of device scratch owned by the caller.
constexpr int kFoldMax = 64;
int launch_diag_final(const C2PPart *p1, int n1, const FluxPart *p2, int n2, FoldPart *lvl,
                      grhd_diag *diag, hipStream_t st);

}  // namespace grhd
