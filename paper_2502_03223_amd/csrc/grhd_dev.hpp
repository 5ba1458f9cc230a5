// grhd_dev.hpp -- gfx950 device functions of the GRHD substep.
//
// Physics: Lam & Shibata, SACRA-2D (arXiv 2502.03223), Sec. II.C.  The
// readings taken where the paper is silent or misprinted are restated at
// each function.  Reconstruction and the Riemann solver are templated on
// the arithmetic type T (double, or float in the mixed-precision path);
// recovery, sources, divergence and the stage update are always double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grhd.h"

namespace grhd {

// ------------------------------------------------------------ launch data

struct GridK {
  int nx, nz, ng;
  long long pitch;
  double x0, z0, dx, dz;
  int geom;
  int bc[4];
};

struct EosK {
  int kind, n;
  double K[8], G[8], rho_b[8], deps[8];
  double Gth;
  double P_atm, eps_atm, rho_atm;
  // of the atmosphere state, set on the host: sound speed (c_s^2 clamped
  // to [0, 0.999999] as eos_cs2 does) and rho h
  double cs_atm, rhw2_atm;
};

struct MetK {
  const double *f[GRHD_NMET];
  double c[GRHD_NMET];
};

struct C2PK {
  double kmax, tol;
  int max_iter, guess;
  const void *mlp;
  int adiabatic;  // zero-temperature mode: the cold root only
  int reuse_atm;  // skip the primitives of cells that stay atmosphere
};

enum MetricClass { MC_CF = 0, MC_GEN = 1 };  // conformally flat static / general

__device__ __forceinline__ long long cell_index(const GridK &g, int j, int k) {
  return (long long)(k + g.ng) * g.pitch + (j + g.ng);
}

__device__ __forceinline__ double mval(const MetK &m, int f, long long i) {
  return m.f[f] ? m.f[f][i] : m.c[f];
}

// Cell arrays addressed by a 32-bit element index through a 32-bit byte
// offset from the base pointer (a field holds at most 2^29 cells, checked
// on the host): with a uniform base the compiler uses the scalar-base
// form, one offset register for every field of a cell.
__device__ __forceinline__ unsigned cell_idx32(const GridK &g, int j, int k) {
  return (unsigned)((k + g.ng) * (int)g.pitch + (j + g.ng));
}

template <class X>
__device__ __forceinline__ X ld32(const X *base, unsigned i) {
  return *reinterpret_cast<const X *>(reinterpret_cast<const char *>(base) + i * (unsigned)sizeof(X));
}

template <class X>
__device__ __forceinline__ void st32(X *base, unsigned i, X v) {
  *reinterpret_cast<X *>(reinterpret_cast<char *>(base) + i * (unsigned)sizeof(X)) = v;
}

__device__ __forceinline__ double mval32(const MetK &m, int f, unsigned i) {
  return m.f[f] ? ld32(m.f[f], i) : m.c[f];
}

// Reciprocal and square root of the flux arithmetic from the hardware
// approximations instead of the correctly rounded sequences: frcp is
// v_rcp_f64 (relative error about 2^-24) refined by two Newton steps,
// within one ulp of 1/x; fsqrt is v_rsq_f64 refined by one coupled Newton
// step for sqrt(x) and 1/(2 sqrt(x)) and a final residual correction,
// which gave the correctly rounded root on all of 4M random arguments over
// 40 decades.  For finite x > 0 (fsqrt: x >= 0).  In single precision the
// hardware instructions themselves (about one ulp).
template <class T> __device__ __forceinline__ T frcp(T x);
template <> __device__ __forceinline__ double frcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <> __device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <class T> __device__ __forceinline__ T fsqrt(T x);
template <> __device__ __forceinline__ double fsqrt<double>(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double y = x * r, h = 0.5 * r;
  const double e = fma(-y, h, 0.5);
  y = fma(y, e, y);
  h = fma(h, e, h);
  const double d = fma(-y, y, x);
  y = fma(d, h, y);
  return x > 0.0 ? y : x;  // rsq(0) is infinite
}
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// inverse of a symmetric 3x3 (xx,xy,xz,yy,yz,zz) by cofactors / det
// FAST: the reciprocal of the determinant from frcp (the face metric of the
// flux); the recovery and the sources keep the correctly rounded division.
template <class T, bool FAST = false>
__device__ __forceinline__ void inv_sym3(const T *a, T *inv) {
  T cxx = a[3] * a[5] - a[4] * a[4];
  T cxy = a[2] * a[4] - a[1] * a[5];
  T cxz = a[1] * a[4] - a[2] * a[3];
  T cyy = a[0] * a[5] - a[2] * a[2];
  T cyz = a[1] * a[2] - a[0] * a[4];
  T czz = a[0] * a[3] - a[1] * a[1];
  T det = a[0] * cxx + a[1] * cxy + a[2] * cxz;
  T id = FAST ? frcp(det) : T(1) / det;
  inv[0] = cxx * id; inv[1] = cxy * id; inv[2] = cxz * id;
  inv[3] = cyy * id; inv[4] = cyz * id; inv[5] = czz * id;
}

__device__ __forceinline__ int s3i(int i, int j) {
  // (xx,xy,xz,yy,yz,zz) storage index of the symmetric element (i,j)
  return (i == j) ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : (i + j == 1 ? 1 : (i + j == 2 ? 2 : 4));
}

// ------------------------------------------------------------ EOS (II.C.3)

__device__ __forceinline__ int eos_piece(const EosK &e, double rho) {
  int i = 0;
  while (i < e.n - 1 && rho >= e.rho_b[i]) i++;
  return i;
}

__device__ __forceinline__ double eps_cold(const EosK &e, double rho) {
  if (e.kind == GRHD_EOS_IDEAL) return 0.0;
  int i = eos_piece(e, rho);
  return e.K[i] / (e.G[i] - 1.0) * pow(rho, e.G[i] - 1.0) + e.deps[i];
}

__device__ __forceinline__ double press_cold(const EosK &e, double rho) {
  if (e.kind == GRHD_EOS_IDEAL) return 0.0;
  int i = eos_piece(e, rho);
  return e.K[i] * pow(rho, e.G[i]);
}

__device__ __forceinline__ double eos_press(const EosK &e, double rho, double eps) {
  if (e.kind == GRHD_EOS_IDEAL) return (e.Gth - 1.0) * rho * eps;
  return press_cold(e, rho) + (e.Gth - 1.0) * rho * (eps - eps_cold(e, rho));
}

// c_s^2 from dP/drho|_eps + (P/rho^2) dP/deps|_rho at the given (rho, eps),
// with an independent (reconstructed) P; clamped to [0, 0.999999].
template <class T>
__device__ __forceinline__ T eos_cs2(const EosK &e, T rho, T eps, T P) {
  T gm1 = T(e.Gth - 1.0);
  T chi;
  if (e.kind == GRHD_EOS_IDEAL) {
    chi = gm1 * eps;
  } else {
    double rd = (double)rho;
    int i = eos_piece(e, rd);
    T kr = T(e.K[i] * pow(rd, e.G[i] - 1.0));  // K rho^(Gamma - 1)
    T ec = kr / T(e.G[i] - 1.0) + T(e.deps[i]);  // cold specific energy
    chi = T(e.G[i]) * kr + gm1 * (eps - ec) - gm1 * kr;
  }
  const T Pr = P * frcp(rho);
  T h = T(1) + eps + Pr;
  T cs2 = (chi + Pr * gm1) * frcp(h);
  if (!(cs2 > T(0))) cs2 = T(0);
  if (cs2 > T(0.999999)) cs2 = T(0.999999);
  return cs2;
}

// specific internal energy at which the EOS gives pressure P at density
// rho (the inverse of eos_press in eps); the face states of the flux take
// rho, u_i and P from the reconstruction and eps from here, so that they
// lie on the EOS
template <class T>
__device__ __forceinline__ T eos_eps(const EosK &e, T rho, T P) {
  T gm1 = T(e.Gth - 1.0);
  if (e.kind == GRHD_EOS_IDEAL) return P / (gm1 * rho);
  double rd = (double)rho;
  int i = eos_piece(e, rd);
  T kr = T(e.K[i] * pow(rd, e.G[i] - 1.0));  // K rho^(Gamma - 1)
  T ec = kr / T(e.G[i] - 1.0) + T(e.deps[i]);  // cold specific energy
  return ec + (P - kr * rho) / (gm1 * rho);
}

// ------------------------------------------------ prim -> con (cons_var)

// conserved vector (densitised, Cartesian S components, E total) of a
// primitive state, given W and the inverse conformal metric (GEN) or not.
template <int MC>
__device__ __forceinline__ void prim2con_cell(double W, const double *gtu, double x,
                                              int geom, const double *p, double *q) {
  double usq;
  if (MC == MC_GEN) {
    usq = 0.0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) usq += gtu[s3i(i, j)] * p[1 + i] * p[1 + j];
    usq *= W * W;
  } else {
    usq = W * W * (p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  }
  double w = sqrt(1.0 + usq);
  double rho = p[0], P = p[4], eps = p[5];
  double h = 1.0 + eps + P / rho;
  double sg = 1.0 / (W * W * W);
  double rhw = rho * h * w;
  q[0] = sg * (rho * w);
  q[1] = sg * (rhw * p[1]);
  q[2] = sg * (rhw * p[2]);
  if (geom == GRHD_GEOM_CYLINDRICAL) q[2] = x * q[2];
  q[3] = sg * (rhw * p[3]);
  q[4] = sg * (rhw * w - P);
}

// ------------------------------------------------ con -> prim (II.C.4)
// The EOS kind is a template parameter (EK) so the gamma-law kernels carry
// no piecewise-polytrope code.

template <int EK>
__device__ __forceinline__ double eps_cold_k(const EosK &e, double rho) {
  return (EK == GRHD_EOS_IDEAL) ? 0.0 : eps_cold(e, rho);
}

template <int EK>
__device__ __forceinline__ double press_cold_k(const EosK &e, double rho) {
  return (EK == GRHD_EOS_IDEAL) ? 0.0 : press_cold(e, rho);
}

template <int EK>
__device__ __forceinline__ double eos_press_k(const EosK &e, double rho, double eps) {
  return (EK == GRHD_EOS_IDEAL) ? (e.Gth - 1.0) * rho * eps : eos_press(e, rho, eps);
}

// h(z) = (1 + eps)(1 + a) of the master function f(z) = z - r / h(z)
// (eq. c2p_fn), eps-hat clamped to eps_min.
template <int EK>
__device__ __forceinline__ double c2p_h(const EosK &e, double D, double qq, double r, double z) {
  double w = sqrt(1.0 + z * z);
  double eps = w * qq - z * r + z * z / (1.0 + w);
  if (EK == GRHD_EOS_IDEAL) {
    // (1+eps)(1+a) with a = P/(rho(1+eps)) reduces to 1 + Gamma eps
    if (eps < 0.0) eps = 0.0;
    return 1.0 + e.Gth * eps;
  } else {
    double rho = D / w;
    double emin = eps_cold(e, rho);
    if (eps < emin) eps = emin;
    double P = eos_press(e, rho, eps);
    double a = P / (rho * (1.0 + eps));
    return (1.0 + eps) * (1.0 + a);
  }
}

// master function f(z), or its zero-temperature variant z - r / h_cold
template <int EK, bool COLD>
__device__ __forceinline__ double c2p_f(const EosK &e, double D, double qq, double r, double z) {
  if (COLD) {
    double rho = D / sqrt(1.0 + z * z);
    double hc = 1.0 + eps_cold_k<EK>(e, rho) + press_cold_k<EK>(e, rho) / rho;
    return z - r / hc;
  }
  return z - r / c2p_h<EK>(e, D, qq, r, z);
}

// f(z) and f'(z).  Gamma law: with eps(z) = w q - z r + (w - 1),
// deps/dz = z (1 + q) / w - r and f' = 1 + r Gamma eps' / h^2 where eps > 0.
template <int EK>
__device__ __forceinline__ void c2p_f_df(const EosK &e, double D, double qq, double r, double z,
                                         double &f, double &df) {
  if (EK == GRHD_EOS_IDEAL) {
    // refined hardware reciprocals and root (within an ulp): the Newton
    // iteration this feeds stops within the solver tolerance of the same
    // root, which the bracket safeguards
    double w = fsqrt(1.0 + z * z);
    double eps = w * qq - z * r + z * z * frcp(1.0 + w);
    if (eps > 0.0) {
      double h = 1.0 + e.Gth * eps;
      double ih = frcp(h);
      f = z - r * ih;
      df = 1.0 + r * e.Gth * (z * (1.0 + qq) * frcp(w) - r) * ih * ih;
    } else {
      f = z - r;
      df = 1.0;
    }
  } else {
    f = c2p_f<EK, false>(e, D, qq, r, z);
    double hh = 1e-7 * z + 1e-300;
    df = (c2p_f<EK, false>(e, D, qq, r, z + hh) - f) / hh;
  }
}

// Illinois (modified regula falsi) on a bracket with f(a) < 0 < f(b).
// Converged when the step, the bracket, or the distance of the secant
// estimate to an end of the bracket falls below tol z (the last case is a
// bracket end that already is the root).
template <int EK, bool COLD>
__device__ double illinois(const EosK &e, double D, double qq, double r, double a, double b,
                           double tol, int max_iter, int *iters) {
  double fa = c2p_f<EK, COLD>(e, D, qq, r, a);
  (*iters)++;
  if (!(fa < 0.0)) return a;
  double fb = c2p_f<EK, COLD>(e, D, qq, r, b);
  (*iters)++;
  if (!(fb > 0.0)) return b;
  int side = 0;
  double c = a;
  for (int it = 0; it < max_iter; it++) {
    double cp = c;
    c = (a * fb - b * fa) / (fb - fa);
    if (c - a <= tol * c || b - c <= tol * c) {
      c = fmin(fmax(c, a), b);
      break;
    }
    double fc = c2p_f<EK, COLD>(e, D, qq, r, c);
    (*iters)++;
    if (fc > 0.0) {
      b = c; fb = fc;
      if (side == -1) fa *= 0.5;
      side = -1;
    } else if (fc < 0.0) {
      a = c; fa = fc;
      if (side == 1) fb *= 0.5;
      side = 1;
    } else {
      break;
    }
    if (fabs(c - cp) <= tol * c || (b - a) <= tol * c) break;
  }
  return c;
}

struct C2PResult {
  unsigned flags;
  int iters;
};

// Full recovery of one cell.  q: densitised conserved (in; rewritten from
// the primitives when a flag is set).  W, gtu: metric at the cell.
// zguess >= 0 starts a safeguarded Newton iteration inside the bracket
// (Illinois from the bracket when it does not converge).  A cell whose
// state ends as the atmosphere carries the ATM flag only (plus FAIL for
// invalid input).  The root satisfies z >= z- (and the gamma-law cold root
// is z = r), so rho = D / w(z) <= D / w(min(z-, r)): when that bound is
// below rho_atm the cell is atmosphere and the root is not needed.
template <int MC, int EK>
__device__ C2PResult con2prim_cell(const EosK &e, const C2PK &cp, double W, const double *gtu,
                                   double x, int geom, double *q, double *p, double zguess) {
  C2PResult res{0u, 0};
  double W3 = W * W * W;
  bool ok = isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) &&
            isfinite(q[4]);
  double D = W3 * q[0];
  double S[3];
  S[0] = W3 * q[1];
  S[1] = (geom == GRHD_GEOM_CYLINDRICAL) ? W3 * (q[2] / x) : W3 * q[2];
  S[2] = W3 * q[3];
  double E = W3 * q[4];
  if (!(D > 0.0) || !(E > 0.0)) ok = false;
  bool atm = !ok || D < e.rho_atm;
  double r = 0.0, qq = 0.0, z = 0.0;
  if (!atm) {
    double S2;
    if (MC == MC_GEN) {
      S2 = 0.0;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) S2 += gtu[s3i(i, j)] * S[i] * S[j];
      S2 *= W * W;
    } else {
      S2 = W * W * (S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    }
    double iD = 1.0 / D;
    r = sqrt(S2) * iD;
    qq = E * iD - 1.0;
    double k = r / (1.0 + qq);
    if (k > cp.kmax) {
      double sc = cp.kmax / k;
      S[0] *= sc; S[1] *= sc; S[2] *= sc;
      r = cp.kmax * (1.0 + qq);
      k = cp.kmax;
      res.flags |= GRHD_FLAG_RESCALE;
    }
    double zm = 0.5 * k / sqrt(1.0 - 0.25 * k * k);
    double zp = k / sqrt(1.0 - k * k);
    double zlo = (EK == GRHD_EOS_IDEAL) ? fmin(zm, r) : 0.0;
    if (D / sqrt(1.0 + zlo * zlo) < e.rho_atm) atm = true;
    // the adiabatic mode never solves the energy equation: the cold root
    // below is its only root
    if (!atm && k > 0.0 && !cp.adiabatic) {
      bool done = false;
      double za = zm, zb = zp;
      if (zguess >= 0.0) {
        // safeguarded Newton from the learned guess (analytic derivative
        // for the gamma law, a one-sided difference otherwise): every
        // evaluation narrows the bracket [za, zb]; a step that leaves it
        // first tries the untested end itself (the root may sit on it, as
        // for cold gas where it equals z+), then bisects; after 8
        // evaluations Illinois finishes on the narrowed bracket
        bool ta = false, tb = false;
        double zz = fmin(fmax(zguess, zm), zp);
        if (EK == GRHD_EOS_IDEAL) {
          // the guess is first refined by Newton in FP32 (to about 1e-6
          // relative, clamped to the bracket), which is far cheaper than
          // FP64 evaluations; the FP64 iteration then starts next to the
          // root
          const float zmf = (float)zm, zpf = (float)zp, qf = (float)qq, rf = (float)r, Gf = (float)e.Gth;
          float zf = fminf(fmaxf((float)zz, zmf), zpf);
          // (hardware approximations of the square root and reciprocal:
          // this stage only has to land near the root)
          for (int it = 0; it < 4; it++) {
            float w = __builtin_amdgcn_sqrtf(1.0f + zf * zf);
            float eps = w * qf - zf * rf + zf * zf * __builtin_amdgcn_rcpf(1.0f + w);
            float f, df;
            if (eps > 0.0f) {
              float ih = __builtin_amdgcn_rcpf(1.0f + Gf * eps);
              f = zf - rf * ih;
              df = 1.0f + rf * Gf * (zf * (1.0f + qf) * __builtin_amdgcn_rcpf(w) - rf) * ih * ih;
            } else {
              f = zf - rf;
              df = 1.0f;
            }
            res.iters += 1;
            float zn = fminf(fmaxf(zf - f * __builtin_amdgcn_rcpf(df), zmf), zpf);
            float dz = fabsf(zn - zf);
            zf = zn;
            if (!(dz > 1e-6f * zf)) break;
          }
          zz = fmin(fmax((double)zf, zm), zp);
        }
        // Converged when a step is below the tolerance, or when two Newton
        // steps in a row (no bisection, no end test) were taken and the
        // second moved z by at most 1e-9 z: in the quadratic regime the
        // point it lands on is then within rounding of the root.
        bool prev_newton = false;
        for (int it = 0; it < 8; it++) {
          double f0, df;
          c2p_f_df<EK>(e, D, qq, r, zz, f0, df);
          res.iters += 1;
          if (f0 == 0.0 || (zz == zp && f0 <= 0.0) || (zz == zm && f0 >= 0.0)) {
            z = zz;
            done = true;
            break;
          }
          if (f0 < 0.0) { za = zz; ta = true; }
          else { zb = zz; tb = true; }
          double zn = zz - f0 * frcp(df);
          bool newton = true;
          if (!(zn > za && zn < zb)) {
            newton = false;
            if (zn >= zb && !tb) zn = zb;
            else if (zn <= za && !ta) zn = za;
            else zn = 0.5 * (za + zb);
          }
          double dz = fabs(zn - zz);
          zz = zn;
          if (dz <= cp.tol * zz || (newton && prev_newton && dz <= 1e-9 * zz)) {
            z = zz;
            done = true;
            break;
          }
          prev_newton = newton;
        }
      }
      if (!done) z = illinois<EK, false>(e, D, qq, r, za, zb, cp.tol, cp.max_iter, &res.iters);
    }
  }
  if (!atm) {
    double w = sqrt(1.0 + z * z);
    double rho = D / w;
    double eps = w * qq - z * r + z * z / (1.0 + w);
    double P;
    if (cp.adiabatic || eps < eps_cold_k<EK>(e, rho)) {
      if (EK == GRHD_EOS_IDEAL) {
        z = r;  // h_cold = 1: the zero-temperature root is z = r
      } else {
        z = (r > 0.0) ? illinois<EK, true>(e, D, qq, r, 0.0, r, cp.tol, cp.max_iter, &res.iters) : 0.0;
      }
      w = sqrt(1.0 + z * z);
      rho = D / w;
      eps = eps_cold_k<EK>(e, rho);
      P = press_cold_k<EK>(e, rho);
      res.flags |= GRHD_FLAG_COLD;
    } else {
      P = eos_press_k<EK>(e, rho, eps);
    }
    double h = 1.0 + eps + P / rho;
    double iDh = 1.0 / (D * h);
    p[0] = rho;
    p[1] = S[0] * iDh;
    p[2] = S[1] * iDh;
    p[3] = S[2] * iDh;
    p[4] = P;
    p[5] = eps;
    if (!isfinite(rho) || !isfinite(P) || !isfinite(eps) || !isfinite(p[1]) ||
        !isfinite(p[2]) || !isfinite(p[3]))
      ok = false;
    atm = !ok || rho < e.rho_atm;
  }
  if (atm) {
    p[0] = e.rho_atm; p[1] = 0.0; p[2] = 0.0; p[3] = 0.0;
    p[4] = e.P_atm; p[5] = e.eps_atm;
    res.flags = ok ? GRHD_FLAG_ATM : (GRHD_FLAG_ATM | GRHD_FLAG_FAIL);
  }
  if (res.flags) prim2con_cell<MC>(W, gtu, x, geom, p, q);
  return res;
}

// Write back the components of a corrected conserved state that differ
// bitwise from the ones read: a cell reset to the atmosphere state it
// already held rewrites nothing.
__device__ __forceinline__ void store_corrected(const double *qq, const double *q0, double *const *q,
                                                long long i) {
  for (int c = 0; c < 5; c++)
    if (__double_as_longlong(qq[c]) != __double_as_longlong(q0[c])) q[c][i] = qq[c];
}

__device__ __forceinline__ void store_corrected(const double *qq, const double *q0, double *const *q,
                                                unsigned i) {
  for (int c = 0; c < 5; c++)
    if (__double_as_longlong(qq[c]) != __double_as_longlong(q0[c])) st32(q[c], i, qq[c]);
}

// ------------------------------------------------ reconstruction (II.C.2)
// PPM of Colella & Woodward (1984): monotonised central slopes, interface
// values, parabola limiter; no steepening or flattening.  Contraction into
// FMA is switched off so the limiter decisions are taken on the same
// rounded values as a plain evaluation.

// x / 6 rounded to nearest, bit for bit what a division gives, in three
// operations instead of a full division: q = x * RN(1/6) is within two ulps
// of x/6, so the remainder x - 6q is exact in one FMA, and q + r * RN(1/6)
// rounds to RN(x/6): x/6 = (x/2)/3 lies at least a sixth of an ulp away
// from any midpoint between two representable numbers, far more than the
// error of the corrected step (normal range; checked against division on
// every finite float and 4e8 random doubles).
template <class T>
__device__ __forceinline__ T div6(T x) {
  const T z = T(1) / T(6);
  const T q = x * z;
  const T r = fma(-q, T(6), x);
  return fma(r, z, q);
}

template <class T>
__device__ __forceinline__ T mono_slope(T am, T a0, T ap) {
#pragma clang fp contract(off)
  T d = T(0.5) * (ap - am);
  if ((ap - a0) * (a0 - am) > T(0)) {
    T m = fabs(d);
    T l = T(2) * fabs(a0 - am);
    T r = T(2) * fabs(ap - a0);
    if (l < m) m = l;
    if (r < m) m = r;
    return copysign(m, d);
  }
  return T(0);
}

template <class T>
__device__ __forceinline__ void ppm_cell(T a, T aL, T aR, T &oL, T &oR) {
#pragma clang fp contract(off)
  if ((aR - a) * (a - aL) <= T(0)) {
    aL = a;
    aR = a;
  } else {
    T dA = aR - aL;
    T a6 = T(6) * (a - T(0.5) * (aL + aR));
    if (dA * a6 > dA * dA) aL = T(3) * a - T(2) * aR;
    else if (-(dA * dA) > dA * a6) aR = T(3) * a - T(2) * aL;
  }
  oL = aL;
  oR = aR;
}

// left and right states at the face between s[2] and s[3] of a 6-cell stencil
template <class T>
__device__ __forceinline__ void ppm_face(const T *s, T &L, T &R) {
#pragma clang fp contract(off)
  T d1 = mono_slope(s[0], s[1], s[2]);
  T d2 = mono_slope(s[1], s[2], s[3]);
  T d3 = mono_slope(s[2], s[3], s[4]);
  T d4 = mono_slope(s[3], s[4], s[5]);
  T i1 = s[1] + T(0.5) * (s[2] - s[1]) - div6<T>(d2 - d1);
  T i2 = s[2] + T(0.5) * (s[3] - s[2]) - div6<T>(d3 - d2);
  T i3 = s[3] + T(0.5) * (s[4] - s[3]) - div6<T>(d4 - d3);
  T l0, r0, l1, r1;
  ppm_cell(s[2], i1, i2, l0, r0);
  ppm_cell(s[3], i2, i3, l1, r1);
  L = r0;
  R = l1;
}

// The second reading of third-order PPM: each cell's own parabola through
// the averages of the cell and its two neighbours; its edge values, held
// inside the range of the two averages that meet at each edge, go through
// the same parabola limiter.  Left and right states of a face then differ
// by a sixth of the third difference across it (upwind dissipation that
// CW84's shared interface value does not have where no limiter acts).
template <class T>
__device__ __forceinline__ void parabola3_edges(T am, T a0, T ap, T &eL, T &eR) {
#pragma clang fp contract(off)
  T l = div6<T>(T(2) * am + T(5) * a0 - ap);
  T r = div6<T>(-am + T(5) * a0 + T(2) * ap);
  eL = fmin(fmax(l, fmin(am, a0)), fmax(am, a0));
  eR = fmin(fmax(r, fmin(a0, ap)), fmax(a0, ap));
}

template <class T>
__device__ __forceinline__ void ppm3_face(const T *s, T &L, T &R) {
  T eL0, eR0, eL1, eR1, l0, r0, l1, r1;
  parabola3_edges(s[1], s[2], s[3], eL0, eR0);
  parabola3_edges(s[2], s[3], s[4], eL1, eR1);
  ppm_cell(s[2], eL0, eR0, l0, r0);
  ppm_cell(s[3], eL1, eR1, l1, r1);
  L = r0;
  R = l1;
}

template <class T>
__device__ __forceinline__ T minmod(T a, T b) {
  if (a * b <= T(0)) return T(0);
  return (fabs(a) < fabs(b)) ? a : b;
}

template <class T>
__device__ __forceinline__ void minmod_face(const T *s, T &L, T &R) {
#pragma clang fp contract(off)
  T si = minmod(s[2] - s[1], s[3] - s[2]);
  T sj = minmod(s[3] - s[2], s[4] - s[3]);
  L = s[2] + T(0.5) * si;
  R = s[3] - T(0.5) * sj;
}

template <class T>
__device__ __forceinline__ void recon_face(int recon, const T *s, T &L, T &R) {
  if (recon == GRHD_RECON_MINMOD) minmod_face(s, L, R);
  else if (recon == GRHD_RECON_PPM3) ppm3_face(s, L, R);
  else ppm_face(s, L, R);
}

// 6-point centred interpolation to the face (metric is smooth) and the
// sixth-order centred first derivative, both without contraction into FMA:
// every caller (the face loops, the per-cell atmosphere faces) rounds them
// identically.
template <class T>
__device__ __forceinline__ T lagrange6(const T *a) {
#pragma clang fp contract(off)
  return (T(3) * a[0] - T(25) * a[1] + T(150) * a[2] + T(150) * a[3] - T(25) * a[4] +
          T(3) * a[5]) * T(1.0 / 256.0);
}

__device__ __forceinline__ double deriv6(const double *a, double inv60h) {
#pragma clang fp contract(off)
  return (-a[0] + 9.0 * a[1] - 45.0 * a[2] + 45.0 * a[4] - 9.0 * a[5] + a[6]) * inv60h;
}

// ------------------------------------------------ Riemann solvers (II.C.2)

template <class T> struct PrimT { T rho, u[3], P, eps; };

// face metric
template <class T> struct FaceMet {
  T alp, W, beta[3], gt[6];
};

// Flux in the tau form: (D, S_x, S_y, S_z, tau = E - D), densitised.
template <class T> struct FluxT { T f[5]; T speed; };

// tetrad-frame state; q/f order (D, S_n, S_t1, S_t2, tau)
template <class T> struct TState { T q[5], f[5], vn, P, lm, lp; };

template <class T>
__device__ __forceinline__ void tetrad_state(const EosK &e, const PrimT<T> &p, const T *ut,
                                             TState<T> &s) {
  T usq = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  T w = fsqrt(T(1) + usq);
  T iw = frcp(w);
  T vn = ut[0] * iw;
  T iw2 = iw * iw;            // 1 - v^2
  T v2 = usq * iw2;
  T h = T(1) + p.eps + p.P * frcp(p.rho);
  T D = p.rho * w;
  T rhw = D * h;
  s.q[0] = D;
  s.q[1] = rhw * ut[0];
  s.q[2] = rhw * ut[1];
  s.q[3] = rhw * ut[2];
  // tau = rho h w^2 - P - rho w without cancellation
  s.q[4] = D * usq * frcp(T(1) + w) + D * p.eps * w + p.P * usq;
  s.vn = vn;
  s.P = p.P;
  s.f[0] = s.q[0] * vn;
  s.f[1] = s.q[1] * vn + p.P;
  s.f[2] = s.q[2] * vn;
  s.f[3] = s.q[3] * vn;
  s.f[4] = (s.q[4] + p.P) * vn;
  T cs2 = eos_cs2<T>(e, p.rho, p.eps, p.P);
  T cs = fsqrt(cs2);
  T disc = iw2 * (T(1) - v2 * cs2 - (T(1) - cs2) * vn * vn);
  if (disc < T(0)) disc = T(0);
  T sd = cs * fsqrt(disc);
  T a0 = vn * (T(1) - cs2);
  T iden = frcp(T(1) - v2 * cs2);
  s.lm = (a0 - sd) * iden;
  s.lp = (a0 + sd) * iden;
}

template <class T>
__device__ __forceinline__ void hllc_star(const TState<T> &s, T lam, T lc, T Pc, T *qc) {
  T dl = lam - s.vn;
  T id = frcp(lam - lc);
  qc[0] = s.q[0] * dl * id;
  qc[1] = (s.q[1] * dl + Pc - s.P) * id;
  qc[2] = s.q[2] * dl * id;
  qc[3] = s.q[3] * dl * id;
  qc[4] = (s.q[4] * dl + Pc * lc - s.P * s.vn) * id;
}

// HLLC in the face tetrad frame; G = f - v_int q of the selected region.
template <class T>
__device__ __forceinline__ void hllc_tetrad(const TState<T> &L, const TState<T> &R, T vint,
                                            T *G, T &lamL, T &lamR) {
  lamL = fmin(L.lm, R.lm);
  lamR = fmax(L.lp, R.lp);
  if (!(lamR - lamL > T(0))) {
    const TState<T> &s = (vint <= lamL) ? L : R;
    for (int m = 0; m < 5; m++) G[m] = s.f[m] - vint * s.q[m];
    return;
  }
  T idl = frcp(lamR - lamL);
  T qh[5], fh[5];
  for (int m = 0; m < 5; m++) {
    qh[m] = (lamR * R.q[m] - lamL * L.q[m] + L.f[m] - R.f[m]) * idl;
    fh[m] = (lamR * L.f[m] - lamL * R.f[m] + lamR * lamL * (R.q[m] - L.q[m])) * idl;
  }
  // contact speed: root of fE lc^2 - (E + fSn) lc + Sn = 0 (E = tau + D)
  T qa = fh[4] + fh[0];
  T qb = -(qh[4] + qh[0] + fh[1]);
  T qc = qh[1];
  T disc = qb * qb - T(4) * qa * qc;
  if (disc < T(0)) disc = T(0);
  T den = -qb + fsqrt(disc);
  T lc = (den > T(0)) ? T(2) * qc * frcp(den) : T(0);
  if (!(den > T(0)) || !(lc > lamL && lc < lamR)) {
    if (vint <= lamL) for (int m = 0; m < 5; m++) G[m] = L.f[m] - vint * L.q[m];
    else if (vint <= lamR) for (int m = 0; m < 5; m++) G[m] = fh[m] - vint * qh[m];
    else for (int m = 0; m < 5; m++) G[m] = R.f[m] - vint * R.q[m];
    return;
  }
  T Pc = -lc * qa + fh[1];
  if (vint <= lamL) {
    for (int m = 0; m < 5; m++) G[m] = L.f[m] - vint * L.q[m];
  } else if (vint <= lc) {
    T qs[5];
    hllc_star(L, lamL, lc, Pc, qs);
    for (int m = 0; m < 5; m++) G[m] = L.f[m] + lamL * (qs[m] - L.q[m]) - vint * qs[m];
  } else if (vint <= lamR) {
    T qs[5];
    hllc_star(R, lamR, lc, Pc, qs);
    for (int m = 0; m < 5; m++) G[m] = R.f[m] + lamR * (qs[m] - R.q[m]) - vint * qs[m];
  } else {
    for (int m = 0; m < 5; m++) G[m] = R.f[m] - vint * R.q[m];
  }
}

// Valencia flux in direction n (tau form) and conserved vector (tau form),
// densitised, plus coordinate characteristic speeds.
template <class T, int MC>
__device__ __forceinline__ void valencia(const EosK &e, const FaceMet<T> &m, const T *gtu, int n,
                                         const PrimT<T> &p, T *F, T *Q, T &lm, T &lp) {
  T W = m.W;
  T usq, un, gnn;
  if (MC == MC_GEN) {
    usq = T(0);
    un = T(0);
    for (int i = 0; i < 3; i++) {
      for (int j = 0; j < 3; j++) usq += gtu[s3i(i, j)] * p.u[i] * p.u[j];
      un += gtu[s3i(n, i)] * p.u[i];
    }
    usq *= W * W;
    un *= W * W;
    gnn = W * W * gtu[s3i(n, n)];
  } else {
    usq = W * W * (p.u[0] * p.u[0] + p.u[1] * p.u[1] + p.u[2] * p.u[2]);
    un = W * W * p.u[n];
    gnn = W * W;
  }
  T w = fsqrt(T(1) + usq);
  T iw = frcp(w);
  T vn = un * iw;
  T h = T(1) + p.eps + p.P * frcp(p.rho);
  T D = p.rho * w;
  T tau = D * usq * frcp(T(1) + w) + D * p.eps * w + p.P * usq;
  T sg = frcp(W * W * W);
  T bn = (MC == MC_GEN) ? m.beta[n] : T(0);
  T tr = m.alp * vn - bn;
  T rhw = D * h;
  F[0] = sg * (D * tr);
  for (int j = 0; j < 3; j++) F[1 + j] = sg * (rhw * p.u[j] * tr + ((j == n) ? m.alp * p.P : T(0)));
  F[4] = sg * (tau * tr + m.alp * p.P * vn);
  Q[0] = sg * D;
  for (int j = 0; j < 3; j++) Q[1 + j] = sg * (rhw * p.u[j]);
  Q[4] = sg * tau;
  T cs2 = eos_cs2<T>(e, p.rho, p.eps, p.P);
  T cs = fsqrt(cs2);
  T v2 = usq * iw * iw;
  T disc = (iw * iw) * (gnn * (T(1) - v2 * cs2) - vn * vn * (T(1) - cs2));
  if (disc < T(0)) disc = T(0);
  T a = m.alp * frcp(T(1) - v2 * cs2);
  const T sd = cs * fsqrt(disc);
  lm = a * (vn * (T(1) - cs2) - sd) - bn;
  lp = a * (vn * (T(1) - cs2) + sd) - bn;
}

// Face flux (tau form), direction dir (0 = x, 1 = z).  speed: largest
// |coordinate signal speed|.
template <class T, int MC>
__device__ __forceinline__ void face_flux(const EosK &e, const FaceMet<T> &m, int dir, int riemann,
                                          const PrimT<T> &pL, const PrimT<T> &pR, FluxT<T> &out) {
  const int n = (dir == 0) ? 0 : 2;
  T gtu[6];
  if (MC == MC_GEN) inv_sym3<T, true>(m.gt, gtu);
  if (riemann == GRHD_RIEMANN_TVDLF) {
    T fL[5], fR[5], qL[5], qR[5], l1, l2, l3, l4;
    valencia<T, MC>(e, m, gtu, n, pL, fL, qL, l1, l2);
    valencia<T, MC>(e, m, gtu, n, pR, fR, qR, l3, l4);
    T c = fmax(fmax(fabs(l1), fabs(l2)), fmax(fabs(l3), fabs(l4)));
    for (int k = 0; k < 5; k++) out.f[k] = T(0.5) * (fL[k] + fR[k] - c * (qR[k] - qL[k]));
    out.speed = c;
    return;
  }
  const T W = m.W;
  T El[3][3];  // contravariant legs (normal, t1, t2), x/y/z components
  T sqgnn, vint;
  if (MC == MC_GEN) {
    const T *gt = m.gt;
    if (dir == 0) {
      T B = frcp(fsqrt(gtu[0]));
      T C = frcp(fsqrt(gt[5]));
      T Dh = B * C;
      El[0][0] = W * B * gtu[0]; El[0][1] = W * B * gtu[1]; El[0][2] = W * B * gtu[2];
      El[1][0] = T(0); El[1][1] = W * Dh * gt[5]; El[1][2] = -(W * Dh * gt[4]);
      El[2][0] = T(0); El[2][1] = T(0); El[2][2] = W * C;
    } else {
      // z faces: cyclic relabelling (n, t1, t2) = (z, x, y)
      T B = frcp(fsqrt(gtu[5]));
      T C = frcp(fsqrt(gt[3]));
      T Dh = B * C;
      El[0][0] = W * B * gtu[2]; El[0][1] = W * B * gtu[4]; El[0][2] = W * B * gtu[5];
      El[1][0] = W * Dh * gt[3]; El[1][1] = -(W * Dh * gt[1]); El[1][2] = T(0);
      El[2][0] = T(0); El[2][1] = W * C; El[2][2] = T(0);
    }
    sqgnn = W * fsqrt(gtu[s3i(n, n)]);
    vint = m.beta[n] * frcp(m.alp * sqgnn);
  } else {
    sqgnn = W;
    vint = T(0);
  }
  TState<T> L, R;
  {
    T ut[3];
    if (MC == MC_GEN) {
      for (int a = 0; a < 3; a++) ut[a] = El[a][0] * pL.u[0] + El[a][1] * pL.u[1] + El[a][2] * pL.u[2];
    } else if (dir == 0) {
      ut[0] = W * pL.u[0]; ut[1] = W * pL.u[1]; ut[2] = W * pL.u[2];
    } else {
      ut[0] = W * pL.u[2]; ut[1] = W * pL.u[0]; ut[2] = W * pL.u[1];
    }
    tetrad_state(e, pL, ut, L);
    if (MC == MC_GEN) {
      for (int a = 0; a < 3; a++) ut[a] = El[a][0] * pR.u[0] + El[a][1] * pR.u[1] + El[a][2] * pR.u[2];
    } else if (dir == 0) {
      ut[0] = W * pR.u[0]; ut[1] = W * pR.u[1]; ut[2] = W * pR.u[2];
    } else {
      ut[0] = W * pR.u[2]; ut[1] = W * pR.u[0]; ut[2] = W * pR.u[1];
    }
    tetrad_state(e, pR, ut, R);
  }
  T G[5], lamL, lamR;
  hllc_tetrad(L, R, vint, G, lamL, lamR);
  // back to the Eulerian frame, densitised by alpha W^-3
  T pref = m.alp * frcp(W * W * W) * sqgnn;
  out.f[0] = pref * G[0];
  out.f[4] = pref * G[4];
  if (MC == MC_GEN) {
    // covariant legs e_(a)_j = gamma_ji e_(a)^i, gamma_ij = W^-2 gt_ij
    T iW2 = frcp(W * W);
    for (int j = 0; j < 3; j++) {
      T s = T(0);
      for (int a = 0; a < 3; a++) {
        T ec = T(0);
        for (int i = 0; i < 3; i++) ec += m.gt[s3i(j, i)] * El[a][i];
        s += ec * iW2 * G[1 + a];
      }
      out.f[1 + j] = pref * s;
    }
  } else {
    T pw = pref * frcp(W);  // covariant legs W^-1 times unit vectors
    if (dir == 0) {
      out.f[1] = pw * G[1]; out.f[2] = pw * G[2]; out.f[3] = pw * G[3];
    } else {
      out.f[3] = pw * G[1]; out.f[1] = pw * G[2]; out.f[2] = pw * G[3];
    }
  }
  out.speed = m.alp * sqgnn * fmax(fabs(lamL - vint), fabs(lamR - vint));
}

// ------------------------------------------------ sources (II.C.1)
// s_Sj = P d_j(alpha W^-3) - W^-3 rho h w^2 [d_j alpha - v_i d_j beta^i
//        + (W^2/2) alpha v_i v_k d_j gt^{ik} + (1/W) alpha v_i v^i d_j W]
//        (+ W^-3 [S_y (alpha v^y - beta^y) + alpha P] / x for j = varpi)
// s_E  = W^-3 [alpha K_ij S^ij - rho h w^2 v^i d_i alpha]
// with Eulerian v_i = u_i / w; d gt^{ik} = -gt^{ia} gt^{kb} d gt_ab.
// g: 17 metric values at the cell; dg: d/dx (dg[0..16]) and d/dz
// (dg[17..33]).
template <int MC>
__device__ __forceinline__ void sources(const double *g, const double *dg, double x, int geom,
                                        const double *p, double *s) {
#pragma clang fp contract(off)
  double alp = g[GRHD_M_ALP], W = g[GRHD_M_W];
  double rho = p[0], P = p[4], eps = p[5];
  double u[3] = {p[1], p[2], p[3]};
  double gtu[6];
  double usq;
  if (MC == MC_GEN) {
    double gt[6] = {g[5], g[6], g[7], g[8], g[9], g[10]};
    inv_sym3(gt, gtu);
    usq = 0.0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) usq += gtu[s3i(i, j)] * u[i] * u[j];
    usq *= W * W;
  } else {
    usq = W * W * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  }
  double w = sqrt(1.0 + usq);
  double iw = 1.0 / w;
  double h = 1.0 + eps + P / rho;
  double vl[3] = {u[0] * iw, u[1] * iw, u[2] * iw};
  double vu[3], vt[3];
  if (MC == MC_GEN) {
    for (int i = 0; i < 3; i++) {
      vt[i] = gtu[s3i(i, 0)] * vl[0] + gtu[s3i(i, 1)] * vl[1] + gtu[s3i(i, 2)] * vl[2];
      vu[i] = W * W * vt[i];
    }
  } else {
    for (int i = 0; i < 3; i++) {
      vt[i] = vl[i];
      vu[i] = W * W * vl[i];
    }
  }
  double vsq = vl[0] * vu[0] + vl[1] * vu[1] + vl[2] * vu[2];
  // one division for the powers of 1/W (they differ from the quotients
  // by a few ulp at most)
  double iW = 1.0 / W;
  double sg = iW * iW * iW;
  double rhw2 = rho * h * w * w;
  double sm[2];
  for (int d = 0; d < 2; d++) {
    const double *dd = dg + d * GRHD_NMET;
    double dalp = dd[GRHD_M_ALP], dW = dd[GRHD_M_W];
    double dasg = dalp * sg + alp * (-3.0 * dW * (sg * iW));
    double br = dalp + alp * vsq * dW * iW;
    if (MC == MC_GEN) {
      double vdb = vl[0] * dd[GRHD_M_BX] + vl[1] * dd[GRHD_M_BY] + vl[2] * dd[GRHD_M_BZ];
      double vvdg = 0.0;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) vvdg -= vt[a] * vt[b] * dd[GRHD_M_GXX + s3i(a, b)];
      br += -vdb + 0.5 * W * W * alp * vvdg;
    }
    sm[d] = P * dasg - sg * rhw2 * br;
  }
  s[0] = 0.0;
  s[1] = sm[0];
  s[2] = 0.0;
  s[3] = sm[1];
  if (geom == GRHD_GEOM_CYLINDRICAL) {
    double Sy = rho * h * w * u[1];
    double by = (MC == MC_GEN) ? g[GRHD_M_BY] : 0.0;
    s[1] += sg * (Sy * (alp * vu[1] - by) + alp * P) / x;
  }
  double vda = vu[0] * dg[GRHD_M_ALP] + vu[2] * dg[GRHD_NMET + GRHD_M_ALP];
  double KS = 0.0;
  if (MC == MC_GEN) {
    double trK = 0.0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        double Kij = g[GRHD_M_KXX + s3i(i, j)];
        KS += vu[i] * vu[j] * Kij;
        trK += W * W * gtu[s3i(i, j)] * Kij;
      }
    KS = rhw2 * KS + P * trK;
  }
  s[4] = sg * (alp * KS - rhw2 * vda);
}

// sources<MC_CF> for a cell at rest (u = 0): the same operations with
// every velocity term exactly zero (w = 1, v = 0); P and rhw2 = rho h of
// the cell's state come from the caller (for the atmosphere they are
// constants of the launch), so no square root and three divisions fewer.
__device__ __forceinline__ void sources_atm_cf(const double *g, const double *dg, double x, int geom,
                                               double P, double rhw2, double *s) {
#pragma clang fp contract(off)
  double alp = g[GRHD_M_ALP], W = g[GRHD_M_W];
  double iW = 1.0 / W;
  double sg = iW * iW * iW;
  double sm[2];
  for (int d = 0; d < 2; d++) {
    const double *dd = dg + d * GRHD_NMET;
    double dalp = dd[GRHD_M_ALP], dW = dd[GRHD_M_W];
    double dasg = dalp * sg + alp * (-3.0 * dW * (sg * iW));
    sm[d] = P * dasg - sg * rhw2 * dalp;
  }
  s[0] = 0.0;
  s[1] = sm[0];
  s[2] = 0.0;
  s[3] = sm[1];
  if (geom == GRHD_GEOM_CYLINDRICAL) s[1] += sg * (alp * P) / x;
  s[4] = 0.0;
}

}  // namespace grhd
