"""The exact quotient by six that the reconstruction kernels use in place of
a division (PPM interface values, PPM3 edge values): q = x * RN(1/6),
r = fma(-q, 6, x), q' = fma(r, RN(1/6), q) must round exactly as x / 6 does,
since the limiters downstream take decisions on those bits.  Checked here
on the host with the same three operations in C (IEEE double and float,
fused multiply-add from the C library), against the division, over
floats spread across every binade and random doubles with random and
low-bit-pattern significands; results below the normal range are left
out, as in the kernels' use."""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static double d6(double x) { const double z = 1.0 / 6.0; double q = x * z; double r = fma(-q, 6.0, x); return fma(r, z, q); }
static float f6(float x) { const float z = 1.0f / 6.0f; float q = x * z; float r = fmaf(-q, 6.0f, x); return fmaf(r, z, q); }
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
int main(void) {
  long bad = 0, n = 0;
  for (uint64_t u = 0x00800000ull; u < 0x7f800000ull; u += 61) {   /* positive normal floats, every binade */
    float x; uint32_t v = (uint32_t)u; memcpy(&x, &v, 4);
    for (int sg = 0; sg < 2; sg++, x = -x) {
      float a = x / 6.0f, b = f6(x);
      if (fabsf(a) < 1.1754944e-38f * 8) continue;
      if (memcmp(&a, &b, 4)) bad++;
      n++;
    }
  }
  for (long i = 0; i < 4000000L; i++) {
    uint64_t u = xr(), ex = 1 + (xr() % 2040);
    u = (u & 0x800fffffffffffffull) | (ex << 52);
    if (i & 1) u = (u & ~0xfffull) | (xr() & 7);
    double x; memcpy(&x, &u, 8);
    double a = x / 6.0, b = d6(x);
    if (fabs(a) < 2.2250738585072014e-308 * 8) continue;
    if (memcmp(&a, &b, 8)) bad++;
    n++;
  }
  printf("%ld %ld\n", n, bad);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_quotient_by_six_is_the_division(tmp_path):
    c = os.path.join(tmp_path, "d6.c")
    exe = os.path.join(tmp_path, "d6")
    open(c, "w").write(SRC)
    # no contraction: the products and sums are the written ones
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-o", exe, c, "-lm"])
    n, bad = (int(v) for v in subprocess.check_output([exe], timeout=120).split())
    assert n > 5_000_000
    assert bad == 0
