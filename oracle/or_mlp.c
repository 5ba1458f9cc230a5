/*
 * or_mlp.c -- FP64 forward pass and back-propagation of the small MLP that
 * supplies the con2prim pressure guess: 3 -> 64 (ReLU) -> 64 (ReLU) -> 1.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle.h).
 *
 * The network is not part of the paper; it is an added initial-guess
 * model whose result is always refined by the paper's root solve.  This
 * file is the plain definition of the network and of the gradient of the
 * mean-squared loss, used to check the GPU training kernels.
 *
 * Parameter vector (4481 doubles): W1[64][3], b1[64], W2[64][64] (row =
 * output unit), b2[64], w3[64], b3.
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3
 *   loss = (1/n) sum (y - t)^2
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

#define H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + H * 3)
#define OFF_W2 (OFF_B1 + H)
#define OFF_B2 (OFF_W2 + H * H)
#define OFF_W3 (OFF_B2 + H)
#define OFF_B3 (OFF_W3 + H)
#define NPARAM (OFF_B3 + 1)

static double fwd_one(const double *P, const double *x, double *h1, double *h2) {
  for (int o = 0; o < H; o++) {
    double s = P[OFF_B1 + o];
    for (int i = 0; i < 3; i++) s += P[OFF_W1 + o * 3 + i] * x[i];
    h1[o] = s > 0.0 ? s : 0.0;
  }
  for (int o = 0; o < H; o++) {
    double s = P[OFF_B2 + o];
    for (int i = 0; i < H; i++) s += P[OFF_W2 + o * H + i] * h1[i];
    h2[o] = s > 0.0 ? s : 0.0;
  }
  double y = P[OFF_B3];
  for (int i = 0; i < H; i++) y += P[OFF_W3 + i] * h2[i];
  return y;
}

void or_mlp_forward(const double *params, int n, const double *X, double *y) {
  double h1[H], h2[H];
  for (int s = 0; s < n; s++) y[s] = fwd_one(params, X + 3 * s, h1, h2);
}

double or_mlp_loss_grad(const double *params, int n, const double *X,
                        const double *t, double *grad) {
  double h1[H], h2[H], d2[H], d1[H];
  memset(grad, 0, sizeof(double) * NPARAM);
  double loss = 0.0;
  for (int s = 0; s < n; s++) {
    const double *x = X + 3 * s;
    double y = fwd_one(params, x, h1, h2);
    double r = y - t[s];
    loss += r * r;
    double dy = 2.0 * r / n;
    grad[OFF_B3] += dy;
    for (int i = 0; i < H; i++) {
      grad[OFF_W3 + i] += dy * h2[i];
      d2[i] = (h2[i] > 0.0) ? dy * params[OFF_W3 + i] : 0.0;
    }
    for (int o = 0; o < H; o++) {
      grad[OFF_B2 + o] += d2[o];
      for (int i = 0; i < H; i++) grad[OFF_W2 + o * H + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < H; i++) {
      double a = 0.0;
      for (int o = 0; o < H; o++) a += params[OFF_W2 + o * H + i] * d2[o];
      d1[i] = (h1[i] > 0.0) ? a : 0.0;
    }
    for (int o = 0; o < H; o++) {
      grad[OFF_B1 + o] += d1[o];
      for (int i = 0; i < 3; i++) grad[OFF_W1 + o * 3 + i] += d1[o] * x[i];
    }
  }
  return loss / n;
}
