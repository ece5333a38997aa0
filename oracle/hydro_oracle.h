/*
 * hydro_oracle.h -- plain, slow FP64 CPU oracle of the split second-order
 * Godunov sweep for the 2D compressible Euler equations.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no source,
 * header, table or helper with the HIP library; the two meet only through the
 * seeded input generators, which hold none of the method's arithmetic.
 *
 * What it computes follows the paper's statement of the method (Section 1):
 * a fixed rectangular 2D domain, conservative variables U = (rho, rho u,
 * rho v, E) on a uniform finite-volume grid, one 1D second-order Godunov
 * update per direction performed successively (directional splitting), a
 * Riemann problem at every cell interface, fluxes, and a conservative update.
 * Each 1D update of cell i reads the five cells i-2..i+2 of its pencil only
 * (Figures 1 and 2).  The per-pencil order READ -> COMPUTE (primitive
 * variables, Riemann problems, incoming fluxes) -> WRITE is Figure 5; the
 * column loop runs before the row loop, with boundary conditions applied in
 * every time step.
 *
 * The numerical details are not printed in the paper (they are delegated to
 * its references [3]-[5]); the readings taken here are the textbook ones
 * (minmod-limited slopes, MUSCL-Hancock half-step trace in primitive
 * variables, two-shock Riemann solver iterated by Newton from the
 * two-rarefaction guess, linear fan sampling, CFL time step).  Every reading
 * is listed next to the function that takes it.  Options beyond them: the
 * MC and van Leer limiters, and sweep orders that alternate x-y / y-x
 * between steps (Strang-type symmetrisation of the splitting), two other
 * interface solvers (the exact Riemann solver and the HLLC flux), and
 * passive scalars advected with the flow.
 *
 * Layout: a grid is double U[4 + nscalars][ny][nx] (x fastest), variables
 * (rho, rho*u, rho*v, E) and then rho*X for each passive scalar X.  Pencils are rows (x-sweep) or columns (y-sweep).
 * Cells are square, h = 1 / max(nx, ny).
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary types, one type for all four sides */
#define ORACLE_BC_REFLECT 1
#define ORACLE_BC_OUTFLOW 2
#define ORACLE_BC_PERIODIC 3

#define ORACLE_DIR_X 0
#define ORACLE_DIR_Y 1

/* floors (a reading: the paper states none) */
#define ORACLE_RHO_MIN 1e-10
#define ORACLE_C_MIN 1e-10

#define ORACLE_LIMITER_MINMOD 0
#define ORACLE_LIMITER_MC 1       /* monotonized central */
#define ORACLE_LIMITER_VANLEER 2

#define ORACLE_RIEMANN_TWO_SHOCK 0 /* Newton on the two-shock function */
#define ORACLE_RIEMANN_EXACT 1     /* Newton on the exact wave curves */
#define ORACLE_RIEMANN_HLLC 2      /* HLLC flux, Einfeldt wave speeds */

#define ORACLE_MAX_SCALARS 4

#define ORACLE_ORDER_XY 0         /* x-sweep then y-sweep every step */
#define ORACLE_ORDER_ALTERNATE 1  /* x then y on even steps, y then x on odd */

typedef struct {
  double gamma; /* ratio of specific heats, > 1 */
  double cfl;   /* Courant number, (0, 1] */
  int bc;       /* ORACLE_BC_* */
  int niter;    /* Newton iteration cap (10) */
  double tol;   /* convergence test |dp| <= tol * p (1e-8) */
  int limiter;  /* ORACLE_LIMITER_* (minmod) */
  int order;    /* ORACLE_ORDER_* (x then y) */
  int riemann;  /* ORACLE_RIEMANN_* (two-shock) */
  int nscalars; /* passive scalars carried after E (0..ORACLE_MAX_SCALARS) */
} oracle_cfg;

/* conservative (rho, m_n, m_t, E) -> primitive (rho, u_n, u_t, p), floored */
void oracle_cons_to_prim(const double u[4], double gamma, double q[4]);
/* pressure floor of a cell of density rho: rho * c_min^2 / gamma */
double oracle_p_floor(double rho, double gamma);
/* sound speed sqrt(gamma p / rho) */
double oracle_sound_speed(const double q[4], double gamma);

/* limited slope of one variable from its two one-sided differences */
double oracle_minmod(double a, double b);
/* the same for any ORACLE_LIMITER_* */
double oracle_limit(double a, double b, int limiter);

/* MUSCL-Hancock half-step trace of one cell: primitive state q, limited
 * slopes dq, lambda = dt/h.  qm is the state at the cell's left face
 * (x_{i-1/2}), qp at its right face (x_{i+1/2}). */
void oracle_trace(const double q[4], const double dq[4], double gamma,
                  double lam, double qm[4], double qp[4]);

/* two-rarefaction star-pressure guess for the left/right states */
double oracle_ptr_guess(const double qL[4], const double qR[4], double gamma);

/* two-shock wave function f(p) = sum_K (p - p_K)/W_K(p) + (u_R - u_L)
 * (its root is the two-shock star pressure) */
double oracle_two_shock_f(const double qL[4], const double qR[4], double gamma,
                          double p);

/* Riemann problem at one interface.  Star pressure by Newton on the
 * two-shock function from the two-rarefaction guess, floored at p_min,
 * stopped at |dp| <= tol*p, or when an iteration that starts on the floor
 * points below it (the root lies under the floor, so the star pressure is the
 * floor), or after niter iterations; then the Godunov state at x/t = 0.
 * Returns the number of iterations done; *converged says whether the test
 * was met.  qg receives (rho, u_n, u_t, p) at the interface; pstar/ustar may
 * be NULL. */
int oracle_riemann(const double qL[4], const double qR[4], double gamma,
                   int niter, double tol, double qg[4], double *pstar,
                   double *ustar, int *converged);

/* exact wave function f(p) = f_L(p) + f_R(p) + (u_R - u_L) with the shock
 * and rarefaction curves of each side (its root is the exact p*) */
double oracle_exact_f(const double qL[4], const double qR[4], double gamma,
                      double p);

/* Riemann problem solved exactly: Newton on the exact wave function from the
 * two-rarefaction guess (same cap, test and floor as oracle_riemann), then
 * the exact self-similar solution at x/t = 0, rarefaction fans included.
 * Same arguments and return value as oracle_riemann. */
int oracle_riemann_exact(const double qL[4], const double qR[4], double gamma,
                         int niter, double tol, double qg[4], double *pstar,
                         double *ustar, int *converged);

/* HLLC wave speeds S = (S_L, S*, S_R) (Einfeldt's bounds, contact speed) */
void oracle_hllc_speeds(const double qL[4], const double qR[4], double gamma,
                        double S[3]);

/* HLLC flux through the interface between primitive states qL and qR */
void oracle_hllc_flux(const double qL[4], const double qR[4], double gamma,
                      double F[4]);
/* 1 when x/t = 0 lies left of the HLLC contact (S_L >= 0, or S_R > 0 and
 * S* >= 0) */
int oracle_hllc_left(const double qL[4], const double qR[4], double gamma);

/* Euler flux normal to the interface from the Godunov state */
void oracle_flux(const double qg[4], double gamma, double F[4]);

/* 1D update of one pencil held with its ghost cells: w is [4+nscalars][n+4],
 * cell i of the pencil at column i+2 (ghosts at 0,1 and n+2,n+3), variables
 * (rho, m_n, m_t, E, rho X_1, ...).  Cells 0..n-1 are updated in place with
 * lambda = dt/h.  hist (may be NULL) has niter+1 slots: hist[k] counts
 * interfaces converged after k iterations, hist[0] the unconverged ones (the
 * HLLC flux iterates nothing and counts nothing). */
void oracle_pencil(double *w, int n, double lam, const oracle_cfg *c,
                   long long *hist);

/* copy pencil `line` of direction dir out of U into w ([4][n+4]) and fill
 * its two ghost cells per side by the boundary rule (scalars are copied like
 * density: only the normal momentum changes sign at a wall) */
void oracle_load_pencil(const double *U, int nx, int ny, int dir, int line,
                        int bc, double *w);
/* the same for nvars = 4 + nscalars planes, w [nvars][n+4] */
void oracle_load_pencil_n(const double *U, int nx, int ny, int nvars, int dir,
                          int line, int bc, double *w);

/* one directional sweep of the whole grid with time step dt */
void oracle_sweep(double *U, int nx, int ny, int dir, double dt,
                  const oracle_cfg *c, long long *hist);

/* max over interior cells of max(|u|+c, |v|+c) */
double oracle_max_speed(const double *U, int nx, int ny, double gamma);

/* dt = cfl * h / max speed */
double oracle_compute_dt(const double *U, int nx, int ny, const oracle_cfg *c);

/* one time step: dt from U, then the two sweeps (x then y, or with
 * ORACLE_ORDER_ALTERNATE y then x when step_index is odd).  Returns dt. */
double oracle_step(double *U, int nx, int ny, const oracle_cfg *c,
                   long long *hist);
double oracle_step_n(double *U, int nx, int ny, const oracle_cfg *c,
                     long step_index, long long *hist);

/* sum over interior cells of each conserved variable times h^2 */
void oracle_totals(const double *U, int nx, int ny, double out[4]);
/* the same for nvars planes (4 + passive scalars) */
void oracle_totals_n(const double *U, int nx, int ny, int nvars, double *out);

/* The paper's OpenMP parallelisations of a time step (openmp_schemes.c):
 * the pencil-parallel loop (fine grain), one subdomain per thread with a
 * neighbour busy-wait barrier (coarse grain), and subdomain tasks with
 * interface-buffer dependencies (tasks).  Each gives oracle_step bitwise.
 * Returns dt. */
#define ORACLE_SCHEME_FINE 0
#define ORACLE_SCHEME_COARSE 1
#define ORACLE_SCHEME_TASKS 2
double oracle_step_scheme(double *U, int nx, int ny, const oracle_cfg *c, int scheme,
                          int threads);
/* the px x py decomposition the coarse-grain and task schemes use */
void oracle_scheme_decomposition(int threads, int nx, int ny, int *px, int *py);

/* number of OpenMP threads the sweeps use (1 when built without OpenMP) */
int oracle_threads(void);
/* set that number (n > 0); results do not depend on it */
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
