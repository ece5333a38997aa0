/*
 * openmp_schemes.c -- the paper's three OpenMP parallelisations of a HYDRO
 * time step, applied to the oracle's pencil update.  TEST INFRASTRUCTURE ONLY
 * (the CPU-baseline leg of the benchmark and the tests): it times the
 * schemes the paper compares on the host, and every scheme must give the
 * serial oracle step bitwise, because a 1D update of a pencil segment reads
 * cells two beyond each end and nothing else (Figures 1 and 2), and every
 * scheme below computes each segment with the same arithmetic.
 *
 *   fine-grain   (Section 2): the loop over pencils of each sweep is an
 *                OpenMP parallel loop (the oracle's own sweep).
 *   coarse-grain (Section 3): a 2D decomposition, one subdomain per thread;
 *                a thread updates its subdomain one pencil segment at a time
 *                in place (READ into a buffer, COMPUTE, WRITE back), and
 *                before writing a segment it waits until its two neighbours
 *                along the sweep have READ the same pencil, through shared
 *                per-thread counters of pencils read (busy wait with flushes;
 *                the counters are sequentially consistent atomics).
 *   tasks        (Sections 5 and 6, Figure 10): one task per column of
 *                subdomains (subdomains that share a range of pencils); in
 *                it, one task per interface between consecutive subdomains
 *                copies the two cells on each side into a shared interface
 *                buffer (depend out), and one task per subdomain READs its
 *                interior, takes its ghost cells from the two interface
 *                buffers (depend in), COMPUTEs and WRITEs in place.
 *
 * Reading taken where the paper is silent: periodic boundaries make the
 * first and last subdomains along a sweep neighbours (one more interface,
 * one more synchronised pair); reflective and outflow ghosts at the domain
 * edges come from the subdomain's own cells.  The time step is the oracle's
 * (one max reduction, then the x and y sweeps); dt is the same for every
 * scheme.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#include "hydro_oracle.h"

/* grid plane of pencil variable k (rho, normal, transverse, E, scalars) */
static int plane_of(int dir, int k) {
  if (k == 1) return dir == ORACLE_DIR_X ? 1 : 2;
  if (k == 2) return dir == ORACLE_DIR_X ? 2 : 1;
  return k;
}

static long offset_of(int nx, int dir, int line, int i) {
  return dir == ORACLE_DIR_X ? (long)line * nx + i : (long)i * nx + line;
}

/* pencil cell i (may be outside 0..n-1) -> interior cell by the boundary
 * rule; *sign = -1 when the normal momentum changes sign (a wall) */
static int ghost_cell(int i, int n, int bc, double *sign) {
  *sign = 1.0;
  if (i >= 0 && i < n) return i;
  int g = i < 0 ? -i : i - (n - 1); /* 1 or 2 */
  if (bc == ORACLE_BC_PERIODIC) return i < 0 ? n - g : g - 1;
  if (bc == ORACLE_BC_REFLECT) {
    *sign = -1.0;
    return i < 0 ? g - 1 : n - g;
  }
  return i < 0 ? 0 : n - 1;
}

/* READ cells a-2 .. b+1 of pencil `line` straight from U into w
 * ([nv][b-a+4]); skip_lo / skip_hi leave the two ghost cells at that end
 * unread (the caller fills them) */
static void read_segment(const double *U, int nx, int ny, int nv, int dir, int line, int a,
                         int b, int bc, int skip_lo, int skip_hi, double *w) {
  const int n = dir == ORACLE_DIR_X ? nx : ny;
  const int m = b - a + 4;
  const long plane = (long)nx * ny;
  for (int j = skip_lo ? 2 : 0; j < (skip_hi ? m - 2 : m); j++) {
    double sign;
    int i = ghost_cell(a - 2 + j, n, bc, &sign);
    long off = offset_of(nx, dir, line, i);
    for (int k = 0; k < nv; k++) {
      double v = U[plane_of(dir, k) * plane + off];
      w[k * m + j] = k == 1 ? sign * v : v;
    }
  }
}

/* WRITE the updated cells a .. b-1 of w back into U */
static void write_segment(double *U, int nx, int ny, int nv, int dir, int line, int a, int b,
                          const double *w) {
  const int m = b - a + 4;
  const long plane = (long)nx * ny;
  for (int i = a; i < b; i++) {
    long off = offset_of(nx, dir, line, i);
    for (int k = 0; k < nv; k++) U[plane_of(dir, k) * plane + off] = w[k * m + (i - a) + 2];
  }
}

/* bounds of part p of 0..n-1 cut into P nearly equal parts */
static int part_lo(int n, int P, int p) { return (int)((long)n * p / P); }

/* a near-square decomposition px * py = T with px <= nx, py <= ny: the
 * divisor pair whose subdomains are closest to square (1 x T if none fits) */
static void decompose(int T, int nx, int ny, int *px, int *py) {
  int best = -1;
  double best_r = 0.0;
  for (int d = 1; d <= T; d++) {
    if (T % d) continue;
    const int e = T / d;
    if (d > nx || e > ny) continue;
    const double r = fabs(log(((double)nx / d) / ((double)ny / e)));
    if (best < 0 || r < best_r) {
      best = d;
      best_r = r;
    }
  }
  if (best < 0) best = 1;
  *px = best;
  *py = T / best;
}

/* ------------------------------------------------------------ coarse grain */
static void coarse_sweep(double *U, int nx, int ny, int dir, double lam, const oracle_cfg *c,
                         int px, int py, volatile int *nread) {
  const int nv = 4 + c->nscalars;
  const int n = dir == ORACLE_DIR_X ? nx : ny;
  const int P = dir == ORACLE_DIR_X ? px : py; /* subdomains along the sweep */
  const int periodic = c->bc == ORACLE_BC_PERIODIC;
#pragma omp parallel num_threads(px * py)
  {
    const int t = omp_get_thread_num();
    const int kx = t % px, ky = t / px;
    const int ks = dir == ORACLE_DIR_X ? kx : ky; /* position along the sweep */
    const int kl = dir == ORACLE_DIR_X ? ky : kx; /* position across it */
    const int Q = dir == ORACLE_DIR_X ? py : px;
    const int nl = dir == ORACLE_DIR_X ? ny : nx; /* pencils */
    const int a = part_lo(n, P, ks), b = part_lo(n, P, ks + 1);
    const int l0 = part_lo(nl, Q, kl), l1 = part_lo(nl, Q, kl + 1);
    /* neighbours along the sweep (thread ids), -1 at a non-periodic edge */
    int left = ks > 0 ? ks - 1 : (periodic ? P - 1 : -1);
    int right = ks < P - 1 ? ks + 1 : (periodic ? 0 : -1);
    if (left >= 0) left = dir == ORACLE_DIR_X ? ky * px + left : left * px + kx;
    if (right >= 0) right = dir == ORACLE_DIR_X ? ky * px + right : right * px + kx;
    double *w = (double *)malloc(sizeof(double) * (size_t)nv * (size_t)(b - a + 4));
    for (int line = l0; line < l1; line++) {
      const int r = line - l0 + 1; /* pencils read once this one is */
      /* (1) READ, then publish the count */
      read_segment(U, nx, ny, nv, dir, line, a, b, c->bc, 0, 0, w);
      /* The counter is a sequentially consistent atomic: its store releases
       * the READ above, and a neighbour's load that sees it acquires it, so
       * that READ happens before the neighbour's WRITE of the same cells.
       * The flushes alone (fences around relaxed atomics) order nothing
       * after the load that ends the wait. */
#pragma omp flush
#pragma omp atomic write seq_cst
      nread[t] = r;
#pragma omp flush
      /* (2) COMPUTE */
      oracle_pencil(w, b - a, lam, c, NULL);
      /* barrier of three: both neighbours have read this pencil */
      for (int nb = 0; nb < 2; nb++) {
        const int o = nb ? right : left;
        if (o < 0 || o == t) continue;
        for (;;) {
          int v;
#pragma omp flush
#pragma omp atomic read seq_cst
          v = nread[o];
          if (v >= r) break;
        }
      }
      /* (3) WRITE */
      write_segment(U, nx, ny, nv, dir, line, a, b, w);
    }
    free(w);
  }
}

/* ------------------------------------------------------------ tasks */
/* One column of subdomains: pencils l0..l1-1, P subdomains along the sweep.
 * iface[q] holds, for interface q (between subdomain q and q+1, cyclic when
 * periodic), cells e-2 .. e+1 of each pencil and variable, e = first cell of
 * subdomain q+1: [line][k][4]. */
static void tasks_column(double *U, int nx, int ny, int dir, double lam, const oracle_cfg *c,
                         int P, int l0, int l1) {
  const int nv = 4 + c->nscalars;
  const int n = dir == ORACLE_DIR_X ? nx : ny;
  const int periodic = c->bc == ORACLE_BC_PERIODIC;
  const int nif = periodic ? P : P - 1;
  const int nlines = l1 - l0;
  const long plane = (long)nx * ny;
  double *iface = (double *)malloc(sizeof(double) * (size_t)(nif > 0 ? nif : 1) * nlines * nv * 4);
  char *dep = (char *)malloc((size_t)(P + 1));

  for (int q = 0; q < nif; q++) {
#pragma omp task shared(U, iface, dep) firstprivate(q) depend(out : dep[q])
    {
      const int e = part_lo(n, P, (q + 1) % P); /* first cell of subdomain q+1 */
      for (int line = l0; line < l1; line++)
        for (int j = 0; j < 4; j++) {
          int i = ((e - 2 + j) % n + n) % n; /* periodic wrap of the first interface */
          long off = offset_of(nx, dir, line, i);
          for (int k = 0; k < nv; k++)
            iface[(((size_t)q * nlines + (line - l0)) * nv + k) * 4 + j] =
                U[plane_of(dir, k) * plane + off];
        }
    }
  }
  for (int p = 0; p < P; p++) {
    /* interfaces on each side (-1: a non-periodic domain edge) */
    const int qin = p > 0 ? p - 1 : (periodic ? P - 1 : -1);
    const int qout = p < P - 1 ? p : (periodic ? P - 1 : -1);
    const int ia = qin >= 0 ? qin : P, ib = qout >= 0 ? qout : P; /* P: a dummy slot */
#pragma omp task shared(U, iface, dep) firstprivate(p, qin, qout) depend(in : dep[ia], dep[ib])
    {
      const int a = part_lo(n, P, p), b = part_lo(n, P, p + 1);
      const int m = b - a + 4;
      double *w = (double *)malloc(sizeof(double) * (size_t)nv * (size_t)m);
      for (int line = l0; line < l1; line++) {
        /* READ: own cells from U (boundary rule at a non-periodic edge),
         * the neighbours' cells from the interface buffers */
        read_segment(U, nx, ny, nv, dir, line, a, b, c->bc, qin >= 0, qout >= 0, w);
        for (int k = 0; k < nv; k++) {
          if (qin >= 0)
            for (int j = 0; j < 2; j++)
              w[k * m + j] = iface[(((size_t)qin * nlines + (line - l0)) * nv + k) * 4 + j];
          if (qout >= 0)
            for (int j = 0; j < 2; j++)
              w[k * m + (b - a + 2) + j] =
                  iface[(((size_t)qout * nlines + (line - l0)) * nv + k) * 4 + 2 + j];
        }
        oracle_pencil(w, b - a, lam, c, NULL); /* COMPUTE */
        write_segment(U, nx, ny, nv, dir, line, a, b, w); /* WRITE */
      }
      free(w);
    }
  }
#pragma omp taskwait
  free(iface);
  free(dep);
}

static void tasks_sweep(double *U, int nx, int ny, int dir, double lam, const oracle_cfg *c,
                        int px, int py) {
  const int P = dir == ORACLE_DIR_X ? px : py;
  const int Q = dir == ORACLE_DIR_X ? py : px;
  const int nl = dir == ORACLE_DIR_X ? ny : nx;
#pragma omp parallel num_threads(px * py)
#pragma omp single
  {
    for (int kl = 0; kl < Q; kl++) {
#pragma omp task shared(U) firstprivate(kl)
      tasks_column(U, nx, ny, dir, lam, c, P, part_lo(nl, Q, kl), part_lo(nl, Q, kl + 1));
    }
#pragma omp taskwait
  }
}

/* ------------------------------------------------------------ one step */
double oracle_step_scheme(double *U, int nx, int ny, const oracle_cfg *c, int scheme,
                          int threads) {
  if (threads < 1) threads = 1;
  const int prev = omp_get_max_threads();
  omp_set_num_threads(threads);
  const double dt = oracle_compute_dt(U, nx, ny, c);
  const double lam = dt / (1.0 / (double)(nx > ny ? nx : ny));
  if (scheme == ORACLE_SCHEME_FINE) {
    oracle_sweep(U, nx, ny, ORACLE_DIR_X, dt, c, NULL);
    oracle_sweep(U, nx, ny, ORACLE_DIR_Y, dt, c, NULL);
  } else {
    int px, py;
    decompose(threads, nx, ny, &px, &py);
    if (scheme == ORACLE_SCHEME_COARSE) {
      volatile int *nread = (volatile int *)calloc((size_t)threads, sizeof(int));
      coarse_sweep(U, nx, ny, ORACLE_DIR_X, lam, c, px, py, nread);
      for (int t = 0; t < threads; t++) nread[t] = 0;
      coarse_sweep(U, nx, ny, ORACLE_DIR_Y, lam, c, px, py, nread);
      free((void *)nread);
    } else {
      tasks_sweep(U, nx, ny, ORACLE_DIR_X, lam, c, px, py);
      tasks_sweep(U, nx, ny, ORACLE_DIR_Y, lam, c, px, py);
    }
  }
  omp_set_num_threads(prev);
  return dt;
}

void oracle_scheme_decomposition(int threads, int nx, int ny, int *px, int *py) {
  decompose(threads < 1 ? 1 : threads, nx, ny, px, py);
}
