/*
 * The 40x10-cell parity channel driven through the C ABI alone: plain C, no HIP headers, the
 * library's own workspace and the default stream.  Writes (rho, U, V, T) of every cell after
 * the requested steps as raw doubles to the output file.
 *
 *   channel <steps> <output file>
 */
#include <stdio.h>
#include <stdlib.h>

#include "ugks.h"

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <steps> <output file>\n", argv[0]);
    return 2;
  }
  const int steps = atoi(argv[1]);
  ugks_mesh mesh = {40, 10, 4.0, 1.0};
  ugks_vgrid vgrid = {24, 24, 5.0, 5.0, 0};
  ugks_bc bc = {UGKS_BC_CHANNEL, 0, 2.0, 1.0, 1.0, 0.0, 0.0};
  ugks_opts opts = {0};
  opts.precision = UGKS_FP64;
  opts.cfl = 0.8;
  opts.rho0 = 1.0;
  opts.T0 = 1.0;
  opts.noise = 0.01;
  opts.seed = 1;
  ugks_handle* h = NULL;
  int rc = ugks_create(&mesh, &vgrid, 0.1, &bc, &opts, &h);
  if (rc != UGKS_OK) {
    fprintf(stderr, "ugks_create: %d %s\n", rc, ugks_last_error(NULL));
    return 1;
  }
  rc = ugks_step(h, steps);
  double* m = malloc(sizeof(double) * 4 * 40 * 10);
  if (rc == UGKS_OK) rc = ugks_moments(h, m);
  ugks_info info;
  if (rc == UGKS_OK) rc = ugks_get_info(h, &info);
  if (rc != UGKS_OK) {
    fprintf(stderr, "step/moments: %d %s\n", rc, ugks_last_error(h));
    ugks_destroy(h);
    free(m);
    return 1;
  }
  FILE* fp = fopen(argv[2], "wb");
  const size_t n = fp ? fwrite(m, sizeof(double), 4 * 40 * 10, fp) : 0;
  if (fp) fclose(fp);
  printf("steps %lld dt %.17g device bytes %zu\n", (long long)info.steps, info.dt,
         info.device_bytes);
  ugks_destroy(h);
  free(m);
  return n == 4 * 40 * 10 ? 0 : 1;
}
