/*
 * Stand-alone driver of the CPU oracle for a sanitizer build.
 *
 * TEST INFRASTRUCTURE ONLY: the CPU test suite compiles this file together
 * with fslbm_oracle.c under -fsanitize=address,undefined, runs it on small
 * scenes and compares its output with the ordinary build.  Any
 * out-of-bounds access, leak or undefined behaviour in the oracle aborts
 * the run.
 *
 * Usage: sanitize_driver <scene file> <output file>
 *   scene file (little endian): int32 nx, ny, nz, periodic[3], collision,
 *   n_bubbles, steps; double tau, trt_lambda, sigma, g[3], p0, eps,
 *   inject_rate; then uint8 type[N], double phi[N], rho[N], u[3N],
 *   int32 id[N], int32 b_id[nb], int32 b_flags[nb], double b_vstar[nb],
 *   double b_pinit[nb].
 *   output file: uint8 type[N], double phi[N], mass[N], f[19N],
 *   int32 id[N], then int64 step, int32 next_id, double bucket,
 *   double total_mass, int32 n_bubbles, and per bubble (by ID) int32 id,
 *   double volume, v_star, pressure.
 */
#include <stdio.h>
#include <stdlib.h>

#include "fslbm_oracle.h"

static int rd(FILE *f, void *p, size_t sz, size_t n) { return fread(p, sz, n, f) == n; }
static int wr(FILE *f, const void *p, size_t sz, size_t n) { return fwrite(p, sz, n, f) == n; }

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s scene out\n", argv[0]);
    return 2;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[9];
  double dv[9];
  if (!rd(f, hdr, 4, 9) || !rd(f, dv, 8, 9)) return 3;
  orc_params p = {0};
  p.nx = hdr[0];
  p.ny = hdr[1];
  p.nz = hdr[2];
  for (int k = 0; k < 3; ++k) p.periodic[k] = hdr[3 + k];
  p.collision = hdr[6];
  const int32_t nb = hdr[7], steps = hdr[8];
  p.tau = dv[0];
  p.trt_lambda = dv[1];
  p.sigma = dv[2];
  for (int k = 0; k < 3; ++k) p.g[k] = dv[3 + k];
  p.p0 = dv[6];
  p.eps = dv[7];
  p.inject_rate = dv[8];
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  uint8_t *type = malloc(N);
  double *phi = malloc(8 * N), *rho = malloc(8 * N), *u = malloc(24 * N);
  int32_t *id = malloc(4 * N);
  int32_t *b_id = malloc(4 * (size_t)(nb > 0 ? nb : 1));
  int32_t *b_flags = malloc(4 * (size_t)(nb > 0 ? nb : 1));
  double *b_vstar = malloc(8 * (size_t)(nb > 0 ? nb : 1));
  double *b_pinit = malloc(8 * (size_t)(nb > 0 ? nb : 1));
  if (!rd(f, type, 1, N) || !rd(f, phi, 8, N) || !rd(f, rho, 8, N) || !rd(f, u, 8, 3 * N) ||
      !rd(f, id, 4, N) || !rd(f, b_id, 4, nb) || !rd(f, b_flags, 4, nb) ||
      !rd(f, b_vstar, 8, nb) || !rd(f, b_pinit, 8, nb))
    return 3;
  fclose(f);
  char err[256];
  orc *o = orc_create(&p, type, phi, rho, u, id, b_id, b_flags, b_vstar, b_pinit, nb, NULL,
                      NULL, 0, 0, 0.0, err, (int32_t)sizeof err);
  if (!o) {
    fprintf(stderr, "create: %s\n", err);
    return 4;
  }
  if (orc_step(o, steps) != 0) {
    fprintf(stderr, "step: %s\n", orc_error(o));
    return 5;
  }
  double *mass = malloc(8 * N), *fo = malloc(8 * 19 * N);
  orc_read(o, type, phi, mass, fo, id, NULL, NULL);
  int64_t step, ntop;
  int32_t next_id;
  double bucket, tm;
  orc_scalars(o, &step, &next_id, &bucket, &tm, &ntop);
  const int32_t n = orc_nbubbles(o);
  int32_t *bi = malloc(4 * (size_t)(n > 0 ? n : 1));
  double *bv = malloc(8 * (size_t)(n > 0 ? n : 1));
  double *bs = malloc(8 * (size_t)(n > 0 ? n : 1));
  double *bp = malloc(8 * (size_t)(n > 0 ? n : 1));
  orc_bubbles(o, bi, NULL, bv, bs, bp, NULL);
  FILE *g = fopen(argv[2], "wb");
  if (!g) return 6;
  int ok = wr(g, type, 1, N) && wr(g, phi, 8, N) && wr(g, mass, 8, N) && wr(g, fo, 8, 19 * N) &&
           wr(g, id, 4, N) && wr(g, &step, 8, 1) && wr(g, &next_id, 4, 1) &&
           wr(g, &bucket, 8, 1) && wr(g, &tm, 8, 1) && wr(g, &n, 4, 1);
  for (int32_t k = 0; ok && k < n; ++k)
    ok = wr(g, &bi[k], 4, 1) && wr(g, &bv[k], 8, 1) && wr(g, &bs[k], 8, 1) && wr(g, &bp[k], 8, 1);
  fclose(g);
  orc_destroy(o);
  free(type);
  free(phi);
  free(rho);
  free(u);
  free(id);
  free(b_id);
  free(b_flags);
  free(b_vstar);
  free(b_pinit);
  free(mass);
  free(fo);
  free(bi);
  free(bv);
  free(bs);
  free(bp);
  return ok ? 0 : 6;
}
