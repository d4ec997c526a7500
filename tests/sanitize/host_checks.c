/*
 * The host side of the library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
 * only, no GPU needed): workspace sizing for every case kind and the argument checks of
 * ugks_create, ugks_step, ugks_moments, ugks_get_info and the batch calls, all of which return
 * before any device work.  Exit status 0 when every call returns what the header documents.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "ugks.h"

static int expect(const char* what, int rc, int want) {
  if (rc != want) {
    fprintf(stderr, "%s: got %d, want %d (%s)\n", what, rc, want, ugks_last_error(NULL));
    return 1;
  }
  return 0;
}

int main(void) {
  int bad = 0;
  ugks_mesh mesh = {400, 100, 4.0, 1.0};
  ugks_vgrid vg = {40, 40, 6.0, 6.0, 0};
  ugks_bc bc = {UGKS_BC_CHANNEL, 0, 2.0, 1.0, 1.0, 0.0, 0.0};
  ugks_opts o;
  memset(&o, 0, sizeof o);
  o.cfl = 0.8; o.rho0 = 1.0; o.T0 = 1.0; o.noise = 0.01; o.seed = 1;
  size_t n = 0;
  bad |= expect("required bytes", ugks_required_bytes(&mesh, &vg, &o, &n), UGKS_OK);
  o.precision = UGKS_FP32_STORE;
  bad |= expect("required bytes fp32", ugks_required_bytes(&mesh, &vg, &o, &n), UGKS_OK);
  vg.internal_dof = 1;
  bad |= expect("required bytes dof", ugks_required_bytes(&mesh, &vg, &o, &n), UGKS_OK);
  vg.internal_dof = 0; o.prandtl = 2.0 / 3.0;
  bad |= expect("required bytes shakhov", ugks_required_bytes(&mesh, &vg, &o, &n), UGKS_OK);
  o.prandtl = 0.0;
  for (int chunks = 0; chunks <= 16; chunks += 4) {
    o.velocity_chunks = chunks;
    bad |= expect("required bytes chunks", ugks_required_bytes(&mesh, &vg, &o, &n), UGKS_OK);
  }
  o.velocity_chunks = 0;
  ugks_vgrid big = {1024, 1024, 20.0, 20.0, 0};
  ugks_mesh one = {1, 1, 1.0, 1.0};
  bad |= expect("required bytes 1024^2", ugks_required_bytes(&one, &big, &o, &n), UGKS_OK);
  /* rejected arguments: each returns before any device call */
  ugks_handle* h = (ugks_handle*)0x1;
  bad |= expect("create NULL out", ugks_create(&mesh, &vg, 0.1, &bc, &o, NULL), UGKS_E_INVAL);
  ugks_mesh m0 = {0, 10, 1.0, 1.0};
  bad |= expect("create nx 0", ugks_create(&m0, &vg, 0.1, &bc, &o, &h), UGKS_E_INVAL);
  bad |= h != NULL;
  ugks_vgrid v1 = {1, 10, 5.0, 5.0, 0};
  bad |= expect("create nu 1", ugks_create(&mesh, &v1, 0.1, &bc, &o, &h), UGKS_E_INVAL);
  ugks_vgrid v2 = {10, 1025, 5.0, 5.0, 0};
  bad |= expect("create nv 1025", ugks_create(&mesh, &v2, 0.1, &bc, &o, &h), UGKS_E_INVAL);
  bad |= expect("create kn 0", ugks_create(&mesh, &vg, 0.0, &bc, &o, &h), UGKS_E_INVAL);
  bad |= expect("create kn nan", ugks_create(&mesh, &vg, NAN, &bc, &o, &h), UGKS_E_INVAL);
  ugks_bc b2 = bc; b2.p_ratio = -1.0;
  bad |= expect("create p_ratio", ugks_create(&mesh, &vg, 0.1, &b2, &o, &h), UGKS_E_INVAL);
  ugks_opts o2 = o; o2.adaptive_dt = 1; o2.dt_override = 1e-3;
  bad |= expect("create adaptive + override", ugks_create(&mesh, &vg, 0.1, &bc, &o2, &h),
                UGKS_E_INVAL);
  o2 = o; o2.prandtl = 0.5; ugks_vgrid v3 = vg; v3.internal_dof = 2;
  bad |= expect("create shakhov + dof", ugks_create(&mesh, &v3, 0.1, &bc, &o2, &h), UGKS_E_INVAL);
  o2 = o; o2.workspace = (void*)0x100; o2.workspace_bytes = 16;
  bad |= expect("create small workspace", ugks_create(&mesh, &vg, 0.1, &bc, &o2, &h),
                UGKS_E_NOMEM);
  bad |= expect("step NULL", ugks_step(NULL, 1), UGKS_E_INVAL);
  bad |= expect("step_static NULL", ugks_step_static(NULL, 1), UGKS_E_INVAL);
  bad |= expect("moments NULL", ugks_moments(NULL, NULL), UGKS_E_INVAL);
  bad |= expect("info NULL", ugks_get_info(NULL, NULL), UGKS_E_INVAL);
  bad |= expect("destroy NULL", ugks_destroy(NULL), UGKS_OK);
  bad |= expect("batch create 0", ugks_batch_create(NULL, 0, NULL), UGKS_E_INVAL);
  bad |= expect("batch destroy NULL", ugks_batch_destroy(NULL), UGKS_OK);
  printf("%s (last message: %s)\n", bad ? "FAILED" : "ok", ugks_last_error(NULL));
  return bad;
}
