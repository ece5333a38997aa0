/*
 * hydro_oracle.c -- plain FP64 CPU oracle of the split second-order Godunov
 * sweep.  TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg).
 *
 * Built with gcc -O2 -ffp-contract=off: every operation below rounds once,
 * in the order written.  Nothing here is blocked, fused or reordered; each
 * function is one step of the method as the paper orders it (Figure 5:
 * primitive variables, Riemann problems at the interfaces, incoming fluxes,
 * update), with the numerical readings the paper leaves open stated where
 * they are taken.
 *
 * The state the two-shock solver's sampling takes inside a transonic
 * rarefaction fan (a reading: linear interpolation across the fan, in
 * oracle_riemann) is pinned against the exact fan: on families of weak
 * transonic rarefactions it must differ from the exact state by the
 * closed-form error of linear interpolation at x/t = 0, second order in the
 * fan width (tests/test_oracle_riemann.py).
 */
#include "hydro_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Primitive variables (Figure 5, COMPUTE: "compute primitive variables").    */
/* Ideal-gas equation of state p = (gamma-1) (E - rho |u|^2 / 2).             */
/* Reading: density floored at RHO_MIN, pressure at rho c_min^2 / gamma so    */
/* that the sound speed never drops below C_MIN.                              */
/* ------------------------------------------------------------------------ */
double oracle_p_floor(double rho, double gamma) {
  return rho * (ORACLE_C_MIN * ORACLE_C_MIN) / gamma;
}

void oracle_cons_to_prim(const double u[4], double gamma, double q[4]) {
  double rho = fmax(u[0], ORACLE_RHO_MIN);
  double un = u[1] / rho;
  double ut = u[2] / rho;
  double ekin = 0.5 * rho * (un * un + ut * ut);
  double p = (gamma - 1.0) * (u[3] - ekin);
  q[0] = rho;
  q[1] = un;
  q[2] = ut;
  q[3] = fmax(p, oracle_p_floor(rho, gamma));
}

double oracle_sound_speed(const double q[4], double gamma) {
  return sqrt(gamma * q[3] / q[0]);
}

/* ------------------------------------------------------------------------ */
/* Second-order reconstruction (Section 1: second-order Godunov scheme).      */
/* Reading: minmod-limited slopes of the primitive variables.                 */
/* ------------------------------------------------------------------------ */
double oracle_minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  if (a > 0.0) return fmin(a, b);
  return fmax(a, b);
}

/* Other limiters of van Leer's family, for the same one-sided differences:
 *   MC (monotonized central): sign(a) min(2|a|, 2|b|, |a+b|/2),
 *   van Leer: the harmonic mean 2ab/(a+b);
 * both 0 unless a and b have the same sign. */
double oracle_limit(double a, double b, int limiter) {
  if (limiter == ORACLE_LIMITER_MINMOD) return oracle_minmod(a, b);
  if (a * b <= 0.0) return 0.0;
  if (limiter == ORACLE_LIMITER_MC) {
    double m = fmin(2.0 * fabs(a), 2.0 * fabs(b));
    m = fmin(m, 0.5 * fabs(a + b));
    return a > 0.0 ? m : -m;
  }
  return 2.0 * a * b / (a + b);
}

/* MUSCL-Hancock half-step trace (reading; no characteristic projection).
 * The primitive 1D Euler system q_t + A(q) q_x = 0 advanced by half a step
 * with the limited slope as q_x gives the source S = -A(q) dq:
 *   S_rho = -(u drho + rho du)
 *   S_u   = -(u du + dp / rho)
 *   S_ut  = -(u dut)
 *   S_p   = -(u dp + gamma p du)
 * and the face states q -/+ dq/2 + (dt/h) S / 2, floored. */
void oracle_trace(const double q[4], const double dq[4], double gamma,
                  double lam, double qm[4], double qp[4]) {
  double rho = q[0], un = q[1], p = q[3];
  double S[4];
  S[0] = -(un * dq[0] + rho * dq[1]);
  S[1] = -(un * dq[1] + dq[3] / rho);
  S[2] = -(un * dq[2]);
  S[3] = -(un * dq[3] + gamma * p * dq[1]);
  for (int k = 0; k < 4; k++) {
    double half_step = 0.5 * lam * S[k];
    qm[k] = q[k] - 0.5 * dq[k] + half_step;
    qp[k] = q[k] + 0.5 * dq[k] + half_step;
  }
  qm[0] = fmax(qm[0], ORACLE_RHO_MIN);
  qp[0] = fmax(qp[0], ORACLE_RHO_MIN);
  qm[3] = fmax(qm[3], oracle_p_floor(qm[0], gamma));
  qp[3] = fmax(qp[3], oracle_p_floor(qp[0], gamma));
}

/* ------------------------------------------------------------------------ */
/* Riemann solver at a cell interface (Section 1, ref. [4]; Figure 5).        */
/* ------------------------------------------------------------------------ */

/* Smallest admissible star pressure for the pair (reading). */
static double pmin_of(const double qL[4], const double qR[4], double gamma) {
  return fmin(oracle_p_floor(qL[0], gamma), oracle_p_floor(qR[0], gamma));
}

/* Two-rarefaction guess: the star pressure when both waves are
 * rarefactions, p = [(cL + cR - (gamma-1)(uR-uL)/2) /
 *                    (cL pL^-z + cR pR^-z)]^(1/z),  z = (gamma-1)/(2 gamma);
 * a non-positive numerator means vacuum forms, and the guess is the floor. */
double oracle_ptr_guess(const double qL[4], const double qR[4], double gamma) {
  double z = (gamma - 1.0) / (2.0 * gamma);
  double cL = oracle_sound_speed(qL, gamma);
  double cR = oracle_sound_speed(qR, gamma);
  double pmin = pmin_of(qL, qR, gamma);
  double num = cL + cR - 0.5 * (gamma - 1.0) * (qR[1] - qL[1]);
  double p;
  if (num <= 0.0) {
    p = pmin;
  } else {
    double den = cL * pow(qL[3], -z) + cR * pow(qR[3], -z);
    p = pow(num / den, 1.0 / z);
  }
  return fmax(p, pmin);
}

/* Lagrangian wave speed of side K at pressure p under the two-shock
 * approximation: W_K^2 = C_K (1 + (gamma+1)/(2 gamma) (p - p_K)/p_K),
 * C_K = gamma p_K rho_K. */
static double shock_W(const double q[4], double gamma, double p) {
  double C = gamma * q[3] * q[0];
  double g = (gamma + 1.0) / (2.0 * gamma);
  return sqrt(C * (1.0 + g * (p - q[3]) / q[3]));
}

double oracle_two_shock_f(const double qL[4], const double qR[4], double gamma,
                          double p) {
  double WL = shock_W(qL, gamma, p);
  double WR = shock_W(qR, gamma, p);
  return (p - qL[3]) / WL + (p - qR[3]) / WR + (qR[1] - qL[1]);
}

int oracle_riemann(const double qL[4], const double qR[4], double gamma,
                   int niter, double tol, double qg[4], double *pstar_out,
                   double *ustar_out, int *converged) {
  double CL = gamma * qL[3] * qL[0];
  double CR = gamma * qR[3] * qR[0];
  double pmin = pmin_of(qL, qR, gamma);

  /* star pressure: Newton on f from the two-rarefaction guess.  With
   * z_K = 2 W_K^3 / (W_K^2 + C_K), f'(p) = 1/z_L + 1/z_R and
   * -f(p) = u*_L - u*_R, so the Newton step is
   * dp = z_L z_R / (z_L + z_R) (u*_L - u*_R). */
  double p = oracle_ptr_guess(qL, qR, gamma);
  int k = 0, conv = 0;
  while (k < niter) {
    k++;
    double WL = shock_W(qL, gamma, p);
    double WR = shock_W(qR, gamma, p);
    double zL = 2.0 * WL * WL * WL / (WL * WL + CL);
    double zR = 2.0 * WR * WR * WR / (WR * WR + CR);
    double usL = qL[1] - (p - qL[3]) / WL;
    double usR = qR[1] + (p - qR[3]) / WR;
    double dp = zL * zR / (zL + zR) * (usL - usR);
    /* on the floor with the step pointing below it: f(p_min) > 0 (f
     * increasing), the root lies under the floor and the floored star
     * pressure is the floor itself (reading) */
    int below_floor = p == pmin && p + dp < pmin;
    p = fmax(p + dp, pmin);
    if (fabs(dp) <= tol * p || below_floor) {
      conv = 1;
      break;
    }
  }

  /* star velocity at the final pressure (reading: the plain average of the
   * two sides' estimates) */
  double WL = shock_W(qL, gamma, p);
  double WR = shock_W(qR, gamma, p);
  double usL = qL[1] - (p - qL[3]) / WL;
  double usR = qR[1] + (p - qR[3]) / WR;
  double us = 0.5 * (usL + usR);

  /* upwind side of the contact (reading: u* = 0 goes to the left side) */
  const double *qo;
  double Wo, s;
  if (us >= 0.0) {
    qo = qL;
    Wo = WL;
    s = 1.0;
  } else {
    qo = qR;
    Wo = WR;
    s = -1.0;
  }
  double ro = qo[0], uo = qo[1], po = qo[3];
  double co = oracle_sound_speed(qo, gamma);

  /* star density on that side, from the Lagrangian jump
   * 1/rho* = 1/rho_o - (p* - p_o)/W_o^2 */
  double rs = ro / (1.0 + ro * (po - p) / (Wo * Wo));
  rs = fmax(rs, ORACLE_RHO_MIN);
  double cs = fmax(ORACLE_C_MIN, sqrt(gamma * p / rs));

  /* speeds of the outer and inner edge of the wave on that side, counted
   * positive when they move away from the interface */
  double sout, sin_;
  if (p >= po) { /* shock: both edges move with it */
    sout = Wo / ro - s * uo;
    sin_ = sout;
  } else { /* rarefaction: head and tail */
    sout = co - s * uo;
    sin_ = cs - s * us;
  }

  /* state at x/t = 0 (reading: linear interpolation across a fan) */
  if (sout < 0.0) {
    qg[0] = ro;
    qg[1] = uo;
    qg[3] = po;
  } else if (sin_ > 0.0) {
    qg[0] = rs;
    qg[1] = us;
    qg[3] = p;
  } else {
    double f = sout / fmax(sout - sin_, ORACLE_C_MIN);
    f = fmin(fmax(f, 0.0), 1.0);
    qg[0] = f * rs + (1.0 - f) * ro;
    qg[1] = f * us + (1.0 - f) * uo;
    qg[3] = f * p + (1.0 - f) * po;
  }
  qg[2] = qo[2]; /* transverse velocity is carried by the contact */

  if (pstar_out) *pstar_out = p;
  if (ustar_out) *ustar_out = us;
  if (converged) *converged = conv;
  return k;
}

/* Euler flux through an interface normal to the sweep direction
 * (Figure 5: "compute incoming fluxes"). */
void oracle_flux(const double qg[4], double gamma, double F[4]) {
  double rho = qg[0], un = qg[1], ut = qg[2], p = qg[3];
  double mass = rho * un;
  F[0] = mass;
  F[1] = mass * un + p;
  F[2] = mass * ut;
  F[3] = un * (gamma * p / (gamma - 1.0) + 0.5 * rho * (un * un + ut * ut));
}

/* ------------------------------------------------------------------------ */
/* Other interface solvers (options).  The paper names its Riemann solver     */
/* only by reference [4]; besides the two-shock reading above, the exact      */
/* solver of the Euler Riemann problem and the HLLC approximate flux.         */
/* ------------------------------------------------------------------------ */

/* Exact wave curve of side K and its derivative at pressure p:
 *   shock (p > p_K):       f_K = (p - p_K) sqrt(A_K / (p + B_K)),
 *                          A_K = 2 / ((gamma+1) rho_K),
 *                          B_K = (gamma-1)/(gamma+1) p_K,
 *                          f_K' = sqrt(A_K / (p + B_K)) (1 - (p - p_K) / (2 (p + B_K)))
 *   rarefaction (p <= p_K): f_K = 2 c_K/(gamma-1) ((p/p_K)^z - 1),
 *                          z = (gamma-1)/(2 gamma),
 *                          f_K' = (p/p_K)^(-(gamma+1)/(2 gamma)) / (rho_K c_K) */
static void exact_curve(const double q[4], double gamma, double p, double *f,
                        double *df) {
  double rho = q[0], pK = q[3];
  if (p > pK) {
    double A = 2.0 / ((gamma + 1.0) * rho);
    double B = (gamma - 1.0) / (gamma + 1.0) * pK;
    double s = sqrt(A / (p + B));
    *f = (p - pK) * s;
    *df = s * (1.0 - (p - pK) / (2.0 * (p + B)));
  } else {
    double c = oracle_sound_speed(q, gamma);
    double z = (gamma - 1.0) / (2.0 * gamma);
    *f = 2.0 * c / (gamma - 1.0) * (pow(p / pK, z) - 1.0);
    *df = pow(p / pK, -(gamma + 1.0) / (2.0 * gamma)) / (rho * c);
  }
}

double oracle_exact_f(const double qL[4], const double qR[4], double gamma,
                      double p) {
  double fL, dfL, fR, dfR;
  exact_curve(qL, gamma, p, &fL, &dfL);
  exact_curve(qR, gamma, p, &fR, &dfR);
  return fL + fR + (qR[1] - qL[1]);
}

int oracle_riemann_exact(const double qL[4], const double qR[4], double gamma,
                         int niter, double tol, double qg[4], double *pstar_out,
                         double *ustar_out, int *converged) {
  const double g = gamma;
  double pmin = pmin_of(qL, qR, g);

  /* star pressure: Newton on the exact f from the two-rarefaction guess,
   * with the same floor and stopping test as the two-shock solver */
  double p = oracle_ptr_guess(qL, qR, g);
  int k = 0, conv = 0;
  while (k < niter) {
    k++;
    double fL, dfL, fR, dfR;
    exact_curve(qL, g, p, &fL, &dfL);
    exact_curve(qR, g, p, &fR, &dfR);
    double dp = -(fL + fR + (qR[1] - qL[1])) / (dfL + dfR);
    int below_floor = p == pmin && p + dp < pmin; /* as in oracle_riemann */
    p = fmax(p + dp, pmin);
    if (fabs(dp) <= tol * p || below_floor) {
      conv = 1;
      break;
    }
  }

  /* star velocity u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2 */
  double fL, dfL, fR, dfR;
  exact_curve(qL, g, p, &fL, &dfL);
  exact_curve(qR, g, p, &fR, &dfR);
  double us = 0.5 * (qL[1] + qR[1]) + 0.5 * (fR - fL);

  /* the self-similar solution at x/t = 0; u* = 0 goes to the left side (the
   * tie reading of the two-shock solver) */
  double G6 = (g - 1.0) / (g + 1.0);
  double z = (g - 1.0) / (2.0 * g);
  double r, u, pr;
  const double *qo;
  if (us >= 0.0) { /* left of the contact */
    qo = qL;
    double rho = qL[0], uK = qL[1], pK = qL[3];
    double c = oracle_sound_speed(qL, g);
    if (p > pK) { /* left shock, speed u_L - c_L sqrt(...) */
      double S = uK - c * sqrt((g + 1.0) / (2.0 * g) * p / pK + z);
      if (S >= 0.0) {
        r = rho, u = uK, pr = pK;
      } else {
        r = rho * (p / pK + G6) / (G6 * p / pK + 1.0), u = us, pr = p;
      }
    } else { /* left rarefaction: head u_L - c_L, tail u* - c*_L */
      double head = uK - c;
      double tail = us - c * pow(p / pK, z);
      if (head >= 0.0) {
        r = rho, u = uK, pr = pK;
      } else if (tail < 0.0) {
        r = rho * pow(p / pK, 1.0 / g), u = us, pr = p;
      } else { /* inside the fan */
        double cf = 2.0 / (g + 1.0) * (c + 0.5 * (g - 1.0) * uK);
        r = rho * pow(cf / c, 2.0 / (g - 1.0));
        u = cf;
        pr = pK * pow(cf / c, 2.0 * g / (g - 1.0));
      }
    }
  } else { /* right of the contact */
    qo = qR;
    double rho = qR[0], uK = qR[1], pK = qR[3];
    double c = oracle_sound_speed(qR, g);
    if (p > pK) { /* right shock, speed u_R + c_R sqrt(...) */
      double S = uK + c * sqrt((g + 1.0) / (2.0 * g) * p / pK + z);
      if (S <= 0.0) {
        r = rho, u = uK, pr = pK;
      } else {
        r = rho * (p / pK + G6) / (G6 * p / pK + 1.0), u = us, pr = p;
      }
    } else { /* right rarefaction: head u_R + c_R, tail u* + c*_R */
      double head = uK + c;
      double tail = us + c * pow(p / pK, z);
      if (head <= 0.0) {
        r = rho, u = uK, pr = pK;
      } else if (tail > 0.0) {
        r = rho * pow(p / pK, 1.0 / g), u = us, pr = p;
      } else { /* inside the fan */
        double cf = 2.0 / (g + 1.0) * (c - 0.5 * (g - 1.0) * uK);
        r = rho * pow(cf / c, 2.0 / (g - 1.0));
        u = -cf;
        pr = pK * pow(cf / c, 2.0 * g / (g - 1.0));
      }
    }
  }
  qg[0] = fmax(r, ORACLE_RHO_MIN);
  qg[1] = u;
  qg[2] = qo[2]; /* transverse velocity is carried by the contact */
  qg[3] = pr;

  if (pstar_out) *pstar_out = p;
  if (ustar_out) *ustar_out = us;
  if (converged) *converged = conv;
  return k;
}

/* Wave-speed bounds of the HLLC flux: Einfeldt's, from the Roe averages
 *   w = sqrt(rho),  a~ = (w_L a_L + w_R a_R)/(w_L + w_R) for a = u, v, H,
 *   H = (E + p)/rho,  c~^2 = (gamma-1)(H~ - (u~^2 + v~^2)/2)  (floored at
 *   c_min^2, a reading),
 *   S_L = min(u_L - c_L, u~ - c~),  S_R = max(u_R + c_R, u~ + c~),
 * and the contact speed
 *   S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R)) /
 *        (rho_L (S_L - u_L) - rho_R (S_R - u_R)). */
void oracle_hllc_speeds(const double qL[4], const double qR[4], double gamma,
                        double S[3]) {
  double g = gamma;
  double cL = oracle_sound_speed(qL, g), cR = oracle_sound_speed(qR, g);
  double HL = (g / (g - 1.0) * qL[3] + 0.5 * qL[0] * (qL[1] * qL[1] + qL[2] * qL[2])) / qL[0];
  double HR = (g / (g - 1.0) * qR[3] + 0.5 * qR[0] * (qR[1] * qR[1] + qR[2] * qR[2])) / qR[0];
  double wL = sqrt(qL[0]), wR = sqrt(qR[0]);
  double ua = (wL * qL[1] + wR * qR[1]) / (wL + wR);
  double va = (wL * qL[2] + wR * qR[2]) / (wL + wR);
  double Ha = (wL * HL + wR * HR) / (wL + wR);
  double c2 = (g - 1.0) * (Ha - 0.5 * (ua * ua + va * va));
  double ca = sqrt(fmax(c2, ORACLE_C_MIN * ORACLE_C_MIN));
  double SL = fmin(qL[1] - cL, ua - ca);
  double SR = fmax(qR[1] + cR, ua + ca);
  double mL = qL[0] * (SL - qL[1]), mR = qR[0] * (SR - qR[1]);
  S[0] = SL;
  S[1] = (qR[3] - qL[3] + qL[1] * mL - qR[1] * mR) / (mL - mR);
  S[2] = SR;
}

/* HLLC flux (Toro, Spruce and Speares): with the speeds above and the star
 * states
 *   U*_K = rho_K (S_K - u_K)/(S_K - S*) (1, S*, v_K,
 *          E_K/rho_K + (S* - u_K)(S* + p_K / (rho_K (S_K - u_K)))),
 * the flux at x/t = 0 is F_L if 0 <= S_L, F_L + S_L (U*_L - U_L) if
 * S_L < 0 <= S*, F_R + S_R (U*_R - U_R) if S* < 0 < S_R, F_R if S_R <= 0
 * (S* = 0 takes the left star state, the tie reading of the other solvers). */
void oracle_hllc_flux(const double qL[4], const double qR[4], double gamma,
                      double F[4]) {
  double S[3];
  oracle_hllc_speeds(qL, qR, gamma, S);
  double SL = S[0], Ss = S[1], SR = S[2];
  if (SL >= 0.0) {
    oracle_flux(qL, gamma, F);
    return;
  }
  if (SR <= 0.0) {
    oracle_flux(qR, gamma, F);
    return;
  }
  const double *q = Ss >= 0.0 ? qL : qR;
  double SK = Ss >= 0.0 ? SL : SR;
  double rho = q[0], u = q[1], v = q[2], p = q[3];
  double E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
  double U[4] = {rho, rho * u, rho * v, E};
  double a = rho * (SK - u) / (SK - Ss);
  double Us[4] = {a, a * Ss, a * v, a * (E / rho + (Ss - u) * (Ss + p / (rho * (SK - u))))};
  oracle_flux(q, gamma, F);
  for (int k = 0; k < 4; k++) F[k] = F[k] + SK * (Us[k] - U[k]);
}

int oracle_hllc_left(const double qL[4], const double qR[4], double gamma) {
  double S[3];
  oracle_hllc_speeds(qL, qR, gamma, S);
  if (S[0] >= 0.0) return 1;
  if (S[2] <= 0.0) return 0;
  return S[1] >= 0.0;
}

/* ------------------------------------------------------------------------ */
/* One pencil (Figure 5: READ into a 1D buffer, COMPUTE, WRITE back).          */
/* ------------------------------------------------------------------------ */
void oracle_pencil(double *w, int n, double lam, const oracle_cfg *c,
                   long long *hist) {
  const double g = c->gamma;
  const int m = n + 4; /* cells -2 .. n+1 */
  const int ns = c->nscalars;
  double *q = (double *)malloc(sizeof(double) * 4 * (size_t)m);
  double *qm = (double *)malloc(sizeof(double) * 4 * (size_t)m);
  double *qp = (double *)malloc(sizeof(double) * 4 * (size_t)m);
  double *F = (double *)malloc(sizeof(double) * 4 * (size_t)m);
  int *left = (int *)malloc(sizeof(int) * (size_t)m);

  /* primitive variables of cells -2 .. n+1 */
  for (int j = 0; j < m; j++) {
    double u[4] = {w[0 * m + j], w[1 * m + j], w[2 * m + j], w[3 * m + j]};
    oracle_cons_to_prim(u, g, &q[4 * j]);
  }
  /* slopes and face states of cells -1 .. n */
  for (int j = 1; j < m - 1; j++) {
    double dq[4];
    for (int k = 0; k < 4; k++)
      dq[k] = oracle_limit(q[4 * j + k] - q[4 * (j - 1) + k],
                           q[4 * (j + 1) + k] - q[4 * j + k], c->limiter);
    oracle_trace(&q[4 * j], dq, g, lam, &qm[4 * j], &qp[4 * j]);
  }
  /* Riemann problem and flux at interfaces -1/2 .. n-1/2: interface between
   * pencil columns j and j+1 is stored at F[j]; left[j] says whether x/t = 0
   * lies on the left of the contact there */
  for (int j = 1; j < m - 2; j++) {
    if (c->riemann == ORACLE_RIEMANN_HLLC) { /* no iteration to count */
      oracle_hllc_flux(&qp[4 * j], &qm[4 * (j + 1)], g, &F[4 * j]);
      left[j] = oracle_hllc_left(&qp[4 * j], &qm[4 * (j + 1)], g);
      continue;
    }
    double qg[4], us;
    int conv;
    int it = c->riemann == ORACLE_RIEMANN_EXACT
                 ? oracle_riemann_exact(&qp[4 * j], &qm[4 * (j + 1)], g, c->niter,
                                        c->tol, qg, NULL, &us, &conv)
                 : oracle_riemann(&qp[4 * j], &qm[4 * (j + 1)], g, c->niter, c->tol,
                                  qg, NULL, &us, &conv);
    if (hist) hist[conv ? it : 0]++;
    oracle_flux(qg, g, &F[4 * j]);
    left[j] = us >= 0.0;
  }
  /* conservative update of cells 0 .. n-1 (columns 2 .. n+1) */
  for (int j = 2; j < m - 2; j++)
    for (int k = 0; k < 4; k++)
      w[k * m + j] = w[k * m + j] + lam * (F[4 * (j - 1) + k] - F[4 * j + k]);

  /* passive scalars (rows 4.. of w hold rho X): X = (rho X)/rho with the
   * floored density of the primitive variables, limited slopes, faces
   * X -/+ dX/2 + (dt/h) S_X/2 with the advective source S_X = -u dX, and the
   * flux of rho X = mass flux times the face value X on the side of the
   * contact that holds x/t = 0 (reading: the scalar is carried by the
   * contact, like the transverse velocity) */
  for (int s = 0; s < ns; s++) {
    double *ws = w + (size_t)(4 + s) * m;
    double *X = (double *)malloc(sizeof(double) * (size_t)m);
    double *Xm = (double *)malloc(sizeof(double) * (size_t)m);
    double *Xp = (double *)malloc(sizeof(double) * (size_t)m);
    double *FX = (double *)malloc(sizeof(double) * (size_t)m);
    for (int j = 0; j < m; j++) X[j] = ws[j] / q[4 * j];
    for (int j = 1; j < m - 1; j++) {
      double dX = oracle_limit(X[j] - X[j - 1], X[j + 1] - X[j], c->limiter);
      double half_step = 0.5 * lam * (-q[4 * j + 1] * dX);
      Xm[j] = X[j] - 0.5 * dX + half_step;
      Xp[j] = X[j] + 0.5 * dX + half_step;
    }
    for (int j = 1; j < m - 2; j++) FX[j] = F[4 * j] * (left[j] ? Xp[j] : Xm[j + 1]);
    for (int j = 2; j < m - 2; j++) ws[j] = ws[j] + lam * (FX[j - 1] - FX[j]);
    free(X);
    free(Xm);
    free(Xp);
    free(FX);
  }

  free(q);
  free(qm);
  free(qp);
  free(F);
  free(left);
}

/* ------------------------------------------------------------------------ */
/* Boundary conditions (Figure 5: "apply boundary conditions").  Reading:     */
/* two ghost cells per side (the stencil of Figures 1-2), filled before each  */
/* sweep along that sweep's direction from the current state:                 */
/*   periodic   ghost -g = cell n-g,  ghost n-1+g = cell g-1                  */
/*   reflective ghost -g = cell g-1,  ghost n-1+g = cell n-g, normal momentum */
/*              negated                                                        */
/*   outflow    ghost -g = cell 0,    ghost n-1+g = cell n-1                  */
/* ------------------------------------------------------------------------ */
static long cell_index(int nx, int dir, int line, int i) {
  /* offset of pencil cell i in one variable plane */
  return dir == ORACLE_DIR_X ? (long)line * nx + i : (long)i * nx + line;
}

/* grid plane of pencil variable k: rho, normal momentum, transverse
 * momentum, E, then the passive scalars in their own order */
static int pencil_plane(int dir, int k) {
  if (k == 1) return dir == ORACLE_DIR_X ? 1 : 2;
  if (k == 2) return dir == ORACLE_DIR_X ? 2 : 1;
  return k;
}

void oracle_load_pencil_n(const double *U, int nx, int ny, int nvars, int dir,
                          int line, int bc, double *w) {
  const int n = dir == ORACLE_DIR_X ? nx : ny;
  const int m = n + 4;
  const long plane = (long)nx * ny;
  for (int j = 0; j < m; j++) {
    int i = j - 2;
    double sign = 1.0;
    if (i < 0 || i >= n) {
      int g = i < 0 ? -i : i - (n - 1); /* 1 or 2 */
      if (bc == ORACLE_BC_PERIODIC) {
        i = i < 0 ? n - g : g - 1;
      } else if (bc == ORACLE_BC_REFLECT) {
        i = i < 0 ? g - 1 : n - g;
        sign = -1.0;
      } else {
        i = i < 0 ? 0 : n - 1;
      }
    }
    long off = cell_index(nx, dir, line, i);
    for (int k = 0; k < nvars; k++) {
      double v = U[pencil_plane(dir, k) * plane + off];
      w[k * m + j] = k == 1 ? sign * v : v;
    }
  }
}

void oracle_load_pencil(const double *U, int nx, int ny, int dir, int line,
                        int bc, double *w) {
  oracle_load_pencil_n(U, nx, ny, 4, dir, line, bc, w);
}

void oracle_sweep(double *U, int nx, int ny, int dir, double dt,
                  const oracle_cfg *c, long long *hist) {
  const int n = dir == ORACLE_DIR_X ? nx : ny;
  const int lines = dir == ORACLE_DIR_X ? ny : nx;
  const int m = n + 4;
  const int nv = 4 + c->nscalars;
  const long plane = (long)nx * ny;
  const double h = 1.0 / (double)(nx > ny ? nx : ny);
  const double lam = dt / h;

  /* Pencils are independent (Section 1), so they may run in any order;
   * the result does not depend on the thread count. */
#pragma omp parallel for schedule(static) if (hist == NULL)
  for (int line = 0; line < lines; line++) {
    double *w = (double *)malloc(sizeof(double) * (size_t)nv * (size_t)m);
    oracle_load_pencil_n(U, nx, ny, nv, dir, line, c->bc, w);
    oracle_pencil(w, n, lam, c, hist);
    for (int i = 0; i < n; i++) {
      long off = cell_index(nx, dir, line, i);
      for (int k = 0; k < nv; k++) U[pencil_plane(dir, k) * plane + off] = w[k * m + i + 2];
    }
    free(w);
  }
}

/* ------------------------------------------------------------------------ */
/* Time step (Figure 5: "for each time step n").  Reading: the CFL condition  */
/* for split sweeps, dt = cfl h / max_cells max(|u|+c, |v|+c), from U^n,       */
/* one dt for both sweeps.                                                     */
/* ------------------------------------------------------------------------ */
double oracle_max_speed(const double *U, int nx, int ny, double gamma) {
  const long plane = (long)nx * ny;
  double smax = 0.0;
  for (long off = 0; off < plane; off++) {
    double u[4] = {U[off], U[plane + off], U[2 * plane + off],
                   U[3 * plane + off]};
    double q[4];
    oracle_cons_to_prim(u, gamma, q);
    double c = oracle_sound_speed(q, gamma);
    double s = fmax(fabs(q[1]) + c, fabs(q[2]) + c);
    smax = fmax(smax, s);
  }
  return smax;
}

double oracle_compute_dt(const double *U, int nx, int ny, const oracle_cfg *c) {
  const double h = 1.0 / (double)(nx > ny ? nx : ny);
  return c->cfl * h / oracle_max_speed(U, nx, ny, c->gamma);
}

double oracle_step_n(double *U, int nx, int ny, const oracle_cfg *c,
                     long step_index, long long *hist) {
  double dt = oracle_compute_dt(U, nx, ny, c);
  const int yx = c->order == ORACLE_ORDER_ALTERNATE && (step_index & 1);
  oracle_sweep(U, nx, ny, yx ? ORACLE_DIR_Y : ORACLE_DIR_X, dt, c, hist);
  oracle_sweep(U, nx, ny, yx ? ORACLE_DIR_X : ORACLE_DIR_Y, dt, c, hist);
  return dt;
}

double oracle_step(double *U, int nx, int ny, const oracle_cfg *c,
                   long long *hist) {
  return oracle_step_n(U, nx, ny, c, 0, hist);
}

/* ------------------------------------------------------------------------ */
/* Conserved totals: sum of U_k h^2 over interior cells, Neumaier-compensated */
/* so that the oracle's own rounding stays a few ulp.                          */
/* ------------------------------------------------------------------------ */
void oracle_totals_n(const double *U, int nx, int ny, int nvars, double *out) {
  const long plane = (long)nx * ny;
  const double h = 1.0 / (double)(nx > ny ? nx : ny);
  for (int k = 0; k < nvars; k++) {
    double sum = 0.0, comp = 0.0;
    for (long off = 0; off < plane; off++) {
      double x = U[k * plane + off];
      double t = sum + x;
      if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
      else
        comp += (x - t) + sum;
      sum = t;
    }
    out[k] = (sum + comp) * (h * h);
  }
}

void oracle_totals(const double *U, int nx, int ny, double out[4]) {
  oracle_totals_n(U, nx, ny, 4, out);
}

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
