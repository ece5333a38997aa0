/* step_blast.c -- the C ABI used from plain C, without Python or PyTorch:
 * a 64x64 corner blast (reflective walls, gamma 1.4, CFL 0.8; the paper's
 * point-explosion test type, Section 7), 3 time steps in FP64 on the GPU.
 * Writes the final state [4][64][64] as raw doubles to argv[1] and prints the
 * conserved totals.  Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "hydro.h"

static int fail(const char *what) {
  fprintf(stderr, "%s: %s\n", what, hydro_last_error());
  return 1;
}

int main(int argc, char **argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: %s out.bin\n", argv[0]);
    return 2;
  }
  const int n = 64;
  const long pitch = 64;
  const size_t plane = (size_t)n * (size_t)pitch, elems = 4 * plane;
  double *host = (double *)calloc(elems, sizeof(double));
  if (!host) return 1;
  const double gamma = 1.4, hcell = 1.0 / n;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      host[j * pitch + i] = 1.0;                          /* rho */
      host[3 * plane + j * pitch + i] = 1e-5 / (gamma - 1.0); /* E of p = 1e-5 at rest */
    }
  host[3 * plane] = 1.0 / (hcell * hcell); /* unit energy deposit in the corner cell */

  void *dev = NULL;
  if (hipMalloc(&dev, elems * sizeof(double)) != hipSuccess) return 1;
  if (hipMemcpy(dev, host, elems * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 1;

  hydro_t *h = hydro_create(n, n, gamma, 0.8, HYDRO_BC_REFLECT);
  if (!h) return fail("hydro_create");
  if (hydro_bind(h, dev, pitch, HYDRO_F64, NULL) != HYDRO_OK) return fail("hydro_bind");
  for (int s = 0; s < 3; ++s)
    if (hydro_step(h) != HYDRO_OK) return fail("hydro_step");
  double tot[4];
  if (hydro_conserved_totals(h, tot) != HYDRO_OK) return fail("hydro_conserved_totals");
  if (hipMemcpy(host, dev, elems * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;
  hydro_destroy(h);
  hipFree(dev);

  FILE *f = fopen(argv[1], "wb");
  if (!f || fwrite(host, sizeof(double), elems, f) != elems) return 1;
  fclose(f);
  free(host);
  printf("totals %.17g %.17g %.17g %.17g\n", tot[0], tot[1], tot[2], tot[3]);
  return 0;
}
