/*
 * The oracle run under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): a few
 * steps of each case kind (channel, periodic, internal degrees of freedom, the Shakhov model,
 * the adaptive step, the collisionless limit), state and flux reads, set_state, and the
 * exported building blocks.  Exit status 0 when every call succeeds; the sanitizers abort on
 * the first fault they find.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ugks_oracle.h"

static ugks_ref_case base(void) {
  ugks_ref_case c = {0};
  c.nx = 9; c.ny = 5; c.lx = 2.0; c.ly = 1.0; c.nu = 8; c.nv = 7; c.umax = 4.0; c.vmax = 4.0;
  c.kn = 0.1; c.bc = 1; c.p_ratio = 2.0; c.T_in = 1.2; c.T_wall = 1.3; c.cfl = 0.8;
  c.rho0 = 1.0; c.T0 = 1.0; c.noise = 0.02; c.seed = 7; c.prandtl = 1.0;
  return c;
}

static int run(const char* what, ugks_ref_case c, int steps) {
  ugks_ref* s = ugks_ref_create(&c);
  if (!s) { fprintf(stderr, "%s: create failed\n", what); return 1; }
  if (ugks_ref_step(s, steps)) { fprintf(stderr, "%s: step failed\n", what); return 1; }
  const int nf = c.nu * c.nv * (c.dof > 0 ? 2 : 1);
  const size_t nc = (size_t)c.nx * c.ny;
  double* f = malloc(sizeof(double) * nc * nf);
  double* W = malloc(sizeof(double) * nc * 4);
  double* Fx = malloc(sizeof(double) * (c.nx + 1) * c.ny * 4);
  double* Fy = malloc(sizeof(double) * c.nx * (c.ny + 1) * 4);
  double* Ffx = malloc(sizeof(double) * (c.nx + 1) * c.ny * nf);
  double* Ffy = malloc(sizeof(double) * c.nx * (c.ny + 1) * nf);
  double* Wg = malloc(sizeof(double) * 2 * c.ny * 4);
  double* fg = malloc(sizeof(double) * 2 * c.ny * nf);
  ugks_ref_get_state(s, f, W);
  ugks_ref_get_face_flux(s, Fx, Fy);
  ugks_ref_get_micro_flux(s, Ffx, Ffy);
  ugks_ref_get_ghost(s, Wg, fg);
  ugks_ref_set_state(s, f, W);
  int bad = ugks_ref_step(s, 1) != 0;
  ugks_ref_get_state(s, f, W);
  for (size_t q = 0; q < nc * 4; ++q) bad |= !isfinite(W[q]);
  printf("%s: %d steps, dt %.6g, time %.6g, rho[0] %.6f\n", what, steps + 1, ugks_ref_dt(s),
         ugks_ref_time(s), W[0]);
  free(f); free(W); free(Fx); free(Fy); free(Ffx); free(Ffy); free(Wg); free(fg);
  ugks_ref_destroy(s);
  return bad;
}

int main(void) {
  int bad = 0;
  ugks_ref_case c = base();
  bad |= run("channel", c, 3);
  c = base(); c.bc = 0; bad |= run("periodic", c, 3);
  c = base(); c.dof = 1; bad |= run("internal dof", c, 2);
  c = base(); c.prandtl = 2.0 / 3.0; bad |= run("shakhov", c, 2);
  c = base(); c.adaptive_dt = 1; bad |= run("adaptive dt", c, 3);
  c = base(); c.kn = INFINITY; c.bc = 0; bad |= run("collisionless", c, 2);
  c = base(); c.nu = 9; c.nv = 9; c.ny = 1; bad |= run("one row, zero velocities", c, 2);
  /* building blocks */
  double x[9], w[9], full[7], pos[7], neg[7], Mt[5], prim[4], a[4];
  ugks_ref_nodes(9, 3.0, x, w);
  ugks_ref_moments_1d(0.2, 1.1, full, pos, neg);
  ugks_ref_time_weights(1e-3, 0.05, Mt);
  const double W4[4] = {1.0, 0.1, -0.2, 1.3};
  bad |= ugks_ref_prim(W4, prim, 0);
  const double sl[4] = {0.1, 0.0, 0.2, -0.1};
  ugks_ref_micro_slope(prim, sl, a, 0);
  const double q[2] = {0.01, -0.02};
  (void)ugks_ref_shakhov(prim, q, 2.0 / 3.0, 0.5, -0.3);
  (void)ugks_ref_vanleer(0.3, 0.1);
  (void)ugks_ref_splitmix64(1, 2);
  ugks_ref_case invalid = base(); invalid.nu = 1;
  bad |= ugks_ref_create(&invalid) != NULL;
  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
