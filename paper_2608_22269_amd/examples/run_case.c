/*
 * A plain C caller of libwbsph: no Python, no PyTorch.  It reads a case
 * file, allocates the workspace and a stream with the HIP runtime, creates a
 * context from host arrays, runs sph_step and writes the fields back.
 *
 *   run_case <case file> <output file>
 *
 * Case file (little endian):
 *   "WBSPHCS1"                          8 bytes
 *   uint64 params_bytes                 must equal sizeof(sph_params)
 *   sph_params                          params_bytes bytes, as declared in wbsph.h
 *   int64 n, int32 dim, int32 nsteps
 *   double x[n*dim], u[n*dim], phi[n]; uint8 kind[n]; double normal[n*dim]
 * Output file:
 *   "WBSPHOUT", int64 n, int32 dim, int32 steps done, double t,
 *   double x[n*dim], u[n*dim], phi[n]   (the caller's particle order)
 *
 * Every call's status is checked; on an error the program prints the
 * library's message and exits with status 1 (2 for a malformed file).
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "wbsph.h"

static void *read_all(FILE *f, size_t bytes, const char *what) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "run_case: cannot read %s (%zu bytes)\n", what, bytes);
    exit(2);
  }
  return p;
}

static int check(sph_status s, sph_ctx *ctx, const char *call) {
  if (s == SPH_OK) return 0;
  fprintf(stderr, "run_case: %s: %s (%s)\n", call, sph_status_string(s), ctx ? sph_last_error(ctx) : "");
  return 1;
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: run_case <case file> <output file>\n");
    return 2;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) {
    fprintf(stderr, "run_case: cannot open %s\n", argv[1]);
    return 2;
  }
  char magic[8];
  uint64_t pbytes = 0;
  if (fread(magic, 1, 8, f) != 8 || memcmp(magic, "WBSPHCS1", 8) != 0 || fread(&pbytes, 8, 1, f) != 1 ||
      pbytes != sizeof(sph_params)) {
    fprintf(stderr, "run_case: not a case file for this library (sph_params is %zu bytes)\n", sizeof(sph_params));
    return 2;
  }
  sph_params p;
  int64_t n = 0;
  int32_t dim = 0, nsteps = 0;
  if (fread(&p, sizeof p, 1, f) != 1 || fread(&n, 8, 1, f) != 1 || fread(&dim, 4, 1, f) != 1 ||
      fread(&nsteps, 4, 1, f) != 1 || n < 0 || (dim != 2 && dim != 3) || nsteps < 0) {
    fprintf(stderr, "run_case: malformed header\n");
    return 2;
  }
  const size_t nd = (size_t)n * (size_t)dim;
  double *x = read_all(f, nd * sizeof(double), "x");
  double *u = read_all(f, nd * sizeof(double), "u");
  double *phi = read_all(f, (size_t)n * sizeof(double), "phi");
  uint8_t *kind = read_all(f, (size_t)n, "kind");
  double *normal = read_all(f, nd * sizeof(double), "normal");
  fclose(f);

  int64_t nf = 0;
  for (int64_t k = 0; k < n; ++k) nf += kind[k] == 0;
  const size_t ws = sph_workspace_bytes(&p, nf, n - nf);
  if (ws == 0) {
    fprintf(stderr, "run_case: invalid parameters (%s)\n", sph_status_string(sph_validate(&p)));
    return 1;
  }
  void *wsp = NULL;
  hipStream_t stream = NULL;
  if (hipMalloc(&wsp, ws) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
    fprintf(stderr, "run_case: cannot allocate %zu bytes of workspace or a stream\n", ws);
    return 1;
  }
  sph_ctx *ctx = NULL;
  int bad = check(sph_init(&p, n, x, u, phi, NULL, kind, normal, 0, wsp, ws, (void *)stream, &ctx), ctx, "sph_init");
  if (!bad) bad = check(sph_step(ctx, nsteps, 0.0), ctx, "sph_step");
  double stats[20];
  if (!bad) bad = check(sph_fields(ctx, SPH_FIELD_X, x, 0), ctx, "sph_fields(X)");
  if (!bad) bad = check(sph_fields(ctx, SPH_FIELD_U, u, 0), ctx, "sph_fields(U)");
  if (!bad) bad = check(sph_fields(ctx, SPH_FIELD_PHI, phi, 0), ctx, "sph_fields(PHI)");
  if (!bad) bad = check(sph_stats(ctx, stats), ctx, "sph_stats");
  if (!bad) {
    FILE *o = fopen(argv[2], "wb");
    const int32_t done = (int32_t)stats[2];
    if (!o || fwrite("WBSPHOUT", 1, 8, o) != 8 || fwrite(&n, 8, 1, o) != 1 || fwrite(&dim, 4, 1, o) != 1 ||
        fwrite(&done, 4, 1, o) != 1 || fwrite(&stats[0], 8, 1, o) != 1 || fwrite(x, sizeof(double), nd, o) != nd ||
        fwrite(u, sizeof(double), nd, o) != nd || fwrite(phi, sizeof(double), (size_t)n, o) != (size_t)n) {
      fprintf(stderr, "run_case: cannot write %s\n", argv[2]);
      bad = 1;
    }
    if (o) fclose(o);
  }
  if (ctx) sph_destroy(ctx);
  (void)hipStreamDestroy(stream);
  (void)hipFree(wsp);
  free(x);
  free(u);
  free(phi);
  free(kind);
  free(normal);
  return bad;
}
