/*
 * mlp_oracle.c -- plain FP64 reference of the learned star-pressure guess
 * network.  TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark).
 *
 * Network (parameters flat, row-major): W1[32][6], b1[32], W2[32][32],
 * b2[32], W3[32], b3.
 *   z1 = W1 x + b1, a1 = relu(z1); z2 = W2 a1 + b2, a2 = relu(z2);
 *   y = W3 . a2 + b3
 * Loss over n samples L = (1/n) sum (y - t)^2, gradients by the chain rule.
 *
 * emulate = 1 rounds to bfloat16 (8 significant bits, nearest-even) where a
 * BF16 matrix unit would see its operands: the weights W1, W2, W3, the input
 * x, the activation a1, and in the backward pass the two error signals that
 * enter a matrix product (dL/dz2 for W2's gradient and for dL/da1, dL/dz1
 * for W1's gradient).  Everything else, including every sum, is FP64.
 *
 * Features of an interface: a = ln(rho_L/rho_bar), b = ln(p_L/p_bar),
 * w = asinh((u_L - u_bar)/c_bar), q = ln(p_ptr/p_bar),
 * x = (a, b, w, q, -a, -b), target ln(p_star / p_ptr),
 * with rho_bar, p_bar geometric means, u_bar the mean velocity,
 * c_bar = sqrt(gamma p_bar / rho_bar) and p_ptr the two-rarefaction guess of
 * the two states (oracle_ptr_guess): the network learns the correction to
 * the method's own starting guess.
 */
#include <math.h>
#include <string.h>

#include "hydro_oracle.h"

#define NH 32
#define NI 6
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NI)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH)
#define NPAR (OFF_B3 + 1)

int mlp_oracle_nparams(void) { return NPAR; }

/* nearest-even rounding to 8 significant bits (bfloat16 precision) */
double mlp_oracle_bf16(double v) {
  if (v == 0.0 || !isfinite(v)) return v;
  int e;
  double m = frexp(v, &e); /* |m| in [0.5, 1) */
  double s = rint(m * 256.0); /* nearest-even in the default rounding mode */
  return ldexp(s / 256.0, e);
}

static double bf(double v, int emulate) { return emulate ? mlp_oracle_bf16(v) : v; }
static double relu(double v) { return v > 0.0 ? v : 0.0; }

/* cache (may be NULL): xb[6], z1[32], a1[32], z2[32], a2[32] */
double mlp_oracle_forward(const double *P, const double *x, int emulate, double *cache) {
  double xb[NI], z1[NH], a1[NH], z2[NH], a2[NH];
  for (int k = 0; k < NI; k++) xb[k] = bf(x[k], emulate);
  for (int i = 0; i < NH; i++) {
    double s = P[OFF_B1 + i];
    for (int k = 0; k < NI; k++) s += bf(P[OFF_W1 + i * NI + k], emulate) * xb[k];
    z1[i] = s;
    a1[i] = bf(relu(s), emulate);
  }
  double y = P[OFF_B3];
  for (int i = 0; i < NH; i++) {
    double s = P[OFF_B2 + i];
    for (int k = 0; k < NH; k++) s += bf(P[OFF_W2 + i * NH + k], emulate) * a1[k];
    z2[i] = s;
    a2[i] = relu(s);
    y += bf(P[OFF_W3 + i], emulate) * a2[i];
  }
  if (cache) {
    memcpy(cache, xb, sizeof xb);
    memcpy(cache + NI, z1, sizeof z1);
    memcpy(cache + NI + NH, a1, sizeof a1);
    memcpy(cache + NI + 2 * NH, z2, sizeof z2);
    memcpy(cache + NI + 3 * NH, a2, sizeof a2);
  }
  return y;
}

/* grad[NPAR] and *loss of L = (1/n) sum_s (y_s - t_s)^2 over X[n][6], T[n] */
void mlp_oracle_loss_grad(const double *P, const double *X, const double *T, long n, int emulate,
                          double *grad, double *loss) {
  double cache[NI + 4 * NH];
  memset(grad, 0, sizeof(double) * NPAR);
  double L = 0.0;
  for (long s = 0; s < n; s++) {
    const double y = mlp_oracle_forward(P, X + 6 * s, emulate, cache);
    const double *xb = cache, *z1 = cache + NI, *a1 = cache + NI + NH;
    const double *z2 = cache + NI + 2 * NH, *a2 = cache + NI + 3 * NH;
    const double r = y - T[s];
    L += r * r / (double)n;
    const double gy = 2.0 * r / (double)n;
    grad[OFF_B3] += gy;
    double gz2[NH], ga1[NH];
    for (int i = 0; i < NH; i++) {
      grad[OFF_W3 + i] += gy * a2[i];
      gz2[i] = z2[i] > 0.0 ? gy * bf(P[OFF_W3 + i], emulate) : 0.0;
      grad[OFF_B2 + i] += gz2[i];
    }
    for (int k = 0; k < NH; k++) ga1[k] = 0.0;
    for (int i = 0; i < NH; i++) {
      const double g = bf(gz2[i], emulate);
      for (int k = 0; k < NH; k++) {
        grad[OFF_W2 + i * NH + k] += g * a1[k];
        ga1[k] += bf(P[OFF_W2 + i * NH + k], emulate) * g;
      }
    }
    for (int k = 0; k < NH; k++) {
      const double gz1 = z1[k] > 0.0 ? ga1[k] : 0.0;
      grad[OFF_B1 + k] += gz1;
      const double g = bf(gz1, emulate);
      for (int f = 0; f < NI; f++) grad[OFF_W1 + k * NI + f] += g * xb[f];
    }
  }
  if (loss) *loss = L;
}

/* record (rho_L, u_L, p_L, rho_R, u_R, p_R, p*, ...) -> features and target */
void mlp_oracle_features(const double *rec, double gamma, double *x, double *target) {
  const double rbar = sqrt(rec[0] * rec[3]);
  const double pbar = sqrt(rec[2] * rec[5]);
  const double ubar = 0.5 * (rec[1] + rec[4]);
  const double cbar = sqrt(gamma * pbar / rbar);
  const double qL[4] = {rec[0], rec[1], 0.0, rec[2]};
  const double qR[4] = {rec[3], rec[4], 0.0, rec[5]};
  const double p_ptr = oracle_ptr_guess(qL, qR, gamma);
  x[0] = log(rec[0] / rbar);
  x[1] = log(rec[2] / pbar);
  x[2] = asinh((rec[1] - ubar) / cbar);
  x[3] = log(p_ptr / pbar);
  x[4] = log(rec[3] / rbar);
  x[5] = log(rec[5] / pbar);
  if (target) *target = log(rec[6] / p_ptr);
}
