/*
 * oracle_driver.c -- a plain C program that runs every path of the CPU oracle
 * on small seeded states, for builds with the compiler's sanitizers (test
 * infrastructure: AddressSanitizer + UndefinedBehaviorSanitizer over the
 * solver, the network oracle and the three OpenMP schemes; ThreadSanitizer
 * over the coarse-grain scheme's neighbour barrier).
 *
 * Usage: oracle_driver all | threads
 *   all      every solver, limiter, boundary type, order and scalar count,
 *            the network oracle, and the three OpenMP schemes (fine grain,
 *            coarse grain, tasks) against the serial step;
 *   threads  the fine- and coarse-grain schemes on more threads and larger
 *            grids (the coarse-grain scheme's busy-wait barrier).
 * Exits 0 when every scheme's step equals the serial step bitwise and the
 * sanitizer reported nothing (the builds abort on the first report).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hydro_oracle.h"

double mlp_oracle_forward(const double *P, const double *x, int emulate, double *cache);
void mlp_oracle_loss_grad(const double *P, const double *X, const double *T, long n, int emulate,
                          double *grad, double *loss);
void mlp_oracle_features(const double *rec, double gamma, double *x, double *target);
int mlp_oracle_nparams(void);

/* SplitMix64 (Steele, Lea and Flood 2014) for seeded inputs */
static uint64_t sm_state;
static double uniform01(void) {
  uint64_t z = (sm_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

/* cell-wise random states with a few strong jumps: rho, p log-uniform, |u| < 1 */
static void random_state(double *U, int nx, int ny, int nv, double gamma) {
  const long plane = (long)nx * ny;
  for (long i = 0; i < plane; i++) {
    const double r = exp(-1.0 + 2.0 * uniform01());
    const double p = exp(-2.0 + 4.0 * uniform01());
    const double u = 2.0 * uniform01() - 1.0, v = 2.0 * uniform01() - 1.0;
    U[i] = r;
    U[plane + i] = r * u;
    U[2 * plane + i] = r * v;
    U[3 * plane + i] = p / (gamma - 1.0) + 0.5 * r * (u * u + v * v);
    for (int k = 4; k < nv; k++) U[k * plane + i] = r * uniform01();
  }
}

static oracle_cfg make_cfg(int bc, int limiter, int riemann, int order, int ns) {
  oracle_cfg c;
  c.gamma = 1.4;
  c.cfl = 0.8;
  c.bc = bc;
  c.niter = 10;
  c.tol = 1e-8;
  c.limiter = limiter;
  c.order = order;
  c.riemann = riemann;
  c.nscalars = ns;
  return c;
}

/* schemes: bit k set runs scheme k (ORACLE_SCHEME_*) on 1..maxthreads threads */
static int check_schemes(int nx, int ny, const oracle_cfg *c, int schemes, int maxthreads) {
  const int nv = 4 + c->nscalars;
  const size_t n = (size_t)nv * nx * ny;
  double *U0 = malloc(n * sizeof(double)), *A = malloc(n * sizeof(double));
  double *B = malloc(n * sizeof(double));
  random_state(U0, nx, ny, nv, c->gamma);
  memcpy(A, U0, n * sizeof(double));
  long long hist[11] = {0};
  oracle_step(A, nx, ny, c, hist);
  int bad = 0;
  for (int scheme = ORACLE_SCHEME_FINE; scheme <= ORACLE_SCHEME_TASKS; scheme++) {
    if (!(schemes & (1 << scheme))) continue;
    for (int t = 1; t <= maxthreads; t++) {
      memcpy(B, U0, n * sizeof(double));
      oracle_step_scheme(B, nx, ny, c, scheme, t);
      if (memcmp(A, B, n * sizeof(double)) != 0) {
        fprintf(stderr, "scheme %d, %d threads, %dx%d bc %d: differs from the serial step\n",
                scheme, t, nx, ny, c->bc);
        bad = 1;
      }
    }
  }
  free(U0);
  free(A);
  free(B);
  return bad;
}

static int run_all(void) {
  int bad = 0;
  /* every solver, limiter, boundary type, order and scalar count, two steps */
  for (int riemann = 0; riemann <= 2; riemann++)
    for (int limiter = 0; limiter <= 2; limiter++)
      for (int bc = 1; bc <= 3; bc++) {
        const int ns = (riemann + limiter + bc) % 2;
        const oracle_cfg c = make_cfg(bc, limiter, riemann, (bc + limiter) % 2, ns);
        const int nx = 7 + bc, ny = 5 + limiter;
        const int nv = 4 + ns;
        double *U = malloc(sizeof(double) * nv * nx * ny);
        random_state(U, nx, ny, nv, c.gamma);
        long long hist[11] = {0};
        for (long s = 0; s < 2; s++) oracle_step_n(U, nx, ny, &c, s, hist);
        double tot[8];
        oracle_totals_n(U, nx, ny, nv, tot);
        for (int k = 0; k < nv; k++)
          if (!isfinite(tot[k])) bad = 1;
        free(U);
      }
  /* the three OpenMP schemes against the serial step, ragged decompositions */
  const int shapes[][2] = {{13, 9}, {20, 3}, {4, 17}};
  for (int s = 0; s < 3; s++)
    for (int bc = 1; bc <= 3; bc++) {
      const oracle_cfg c = make_cfg(bc, 0, 0, 0, s == 2);
      bad |= check_schemes(shapes[s][0], shapes[s][1], &c, 7, 4);
    }
  /* the network oracle: forward (exact and emulated), loss gradient, features */
  const int np = mlp_oracle_nparams();
  double *P = malloc(sizeof(double) * np), *g = malloc(sizeof(double) * np);
  for (int i = 0; i < np; i++) P[i] = 0.4 * (2.0 * uniform01() - 1.0);
  double X[6 * 5], T[5], cache[6 + 4 * 32], loss = 0.0;
  for (int i = 0; i < 30; i++) X[i] = 2.0 * uniform01() - 1.0;
  for (int i = 0; i < 5; i++) T[i] = uniform01();
  for (int e = 0; e <= 1; e++) {
    (void)mlp_oracle_forward(P, X, e, cache);
    mlp_oracle_loss_grad(P, X, T, 5, e, g, &loss);
    if (!isfinite(loss)) bad = 1;
  }
  const double rec[8] = {1.0, 0.2, 1.0, 0.125, -0.1, 0.1, 0.3, 2.0};
  double x[6], tgt;
  mlp_oracle_features(rec, 1.4, x, &tgt);
  free(P);
  free(g);
  return bad;
}

static int run_threads(void) {
  int bad = 0;
  const int shapes[][2] = {{24, 18}, {31, 6}, {9, 40}};
  const int schemes = (1 << ORACLE_SCHEME_FINE) | (1 << ORACLE_SCHEME_COARSE);
  for (int s = 0; s < 3; s++)
    for (int bc = 1; bc <= 3; bc++) {
      const oracle_cfg c = make_cfg(bc, s % 3, 0, 0, s == 1);
      bad |= check_schemes(shapes[s][0], shapes[s][1], &c, schemes, 6);
    }
  return bad;
}

int main(int argc, char **argv) {
  sm_state = 2106;
  const int threads = argc > 1 && strcmp(argv[1], "threads") == 0;
  const int bad = threads ? run_threads() : run_all();
  printf("%s: %s\n", threads ? "threads" : "all", bad ? "MISMATCH" : "ok");
  return bad;
}
