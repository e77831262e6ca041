/* Host-only exercise of the C-ABI for the sanitizer test (tests/test_host_sanitizers.py):
 * plan creation over every supported size class and flag set, workspace sizes, the
 * FP64 step table, every tuning setter with valid and invalid values, tracing
 * switches, rejected configurations and the error strings.  Needs no GPU. */
#include <stdio.h>
#include <string.h>
#include <stdlib.h>
#include "cola.h"

static cola_config base(int np, int nm) {
  cola_config c;
  memset(&c, 0, sizeof c);
  c.np = np; c.nm = nm; c.box = 100.0; c.omega_m = 0.3; c.omega_l = 0.7; c.h = 0.7; c.n_s = 0.96; c.sigma8 = 0.8;
  c.a_init = 0.1; c.a_final = 1.0; c.n_steps = 10; c.n_lpt = -2.5; c.flags = 0;
  return c;
}

int main(void) {
  int bad = 0;
  const int sizes[][2] = {{16, 16}, {16, 32}, {16, 48}, {24, 48}, {32, 64}, {32, 96}, {64, 128}, {128, 256}, {256, 512}, {256, 768}, {512, 1024}};
  for (unsigned k = 0; k < sizeof sizes / sizeof sizes[0]; ++k) {
    for (unsigned flags = 0; flags < 16; ++flags) {
      cola_config c = base(sizes[k][0], sizes[k][1]);
      c.flags = flags;
      cola_plan p = NULL;
      if (cola_plan_create(&c, &p) != COLA_OK || !p) { printf("create failed %d %d %u\n", c.np, c.nm, flags); bad++; continue; }
      size_t b = 0, ba = 0, bt = 0;
      if (cola_workspace_bytes(p, &b) || cola_adjoint_workspace_bytes(p, &ba) || cola_tuning_workspace_bytes(p, &bt)) bad++;
      const size_t n = 13 * (c.n_steps + 1);
      double* tab = (double*)malloc(n * sizeof(double));
      if (cola_step_table(p, tab, n) != COLA_OK) bad++;
      if (cola_step_table(p, tab, n - 1) == COLA_OK) bad++;   /* too short */
      free(tab);
      for (int d = 0; d <= 64; d += 4) (void)cola_plan_set_bin_depth(p, d);
      (void)cola_plan_set_bin_depth(p, 32);
      for (int pass = -1; pass <= 2; ++pass)
        for (int w = -1; w <= 17; ++w) (void)cola_plan_set_fft_tile(p, pass, w);
      for (int r = -2; r <= 2; ++r) (void)cola_plan_set_fft_rotation(p, r);
      int32_t rows = -1, yw, xw, bd;
      if (cola_plan_get_fft_rotation(p, &rows) || cola_plan_get_tuning(p, &yw, &xw, &bd)) bad++;
      for (int r = -1; r <= 2; ++r) (void)cola_plan_set_resident_steps(p, r);
      for (int t = -1; t <= 3; ++t) (void)cola_trace_enable(p, t);
      (void)cola_trace_enable(p, 0);
      if (cola_workspace_bytes(p, &b)) bad++;
      if (cola_plan_destroy(p) != COLA_OK) bad++;
    }
  }
  /* invalid configurations are rejected without a plan */
  cola_config c = base(32, 64);
  cola_plan p = NULL;
  c.nm = 80;  if (cola_plan_create(&c, &p) == COLA_OK) bad++;
  c = base(32, 48); if (cola_plan_create(&c, &p) == COLA_OK) bad++;
  c = base(32, 64); c.n_lpt = 0; if (cola_plan_create(&c, &p) == COLA_OK) bad++;
  c = base(32, 64); c.n_steps = 0; if (cola_plan_create(&c, &p) == COLA_OK) bad++;
  c = base(32, 64); c.box = -1; if (cola_plan_create(&c, &p) == COLA_OK) bad++;
  c = base(32, 64); c.flags = 0x100; if (cola_plan_create(&c, &p) == COLA_OK) bad++;
  if (cola_plan_create(NULL, &p) == COLA_OK) bad++;
  if (cola_plan_destroy(NULL) != COLA_OK) bad++;
  /* error paths of the device entry points with null arguments: each must return an
     error status (on a machine without a GPU, possibly COLA_ERR_HIP) without touching
     memory */
  {
    cola_config cc = base(16, 32);
    cola_plan q = NULL;
    if (cola_plan_create(&cc, &q) != COLA_OK) bad++;
    cola_particles none = {NULL, NULL, NULL, NULL};
    size_t sz = 0;
    double dd[8];
    int32_t li[64];
    if (cola_step(NULL, 0, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_step(q, 0, &none, NULL, NULL) == COLA_OK) bad++;
    if (cola_step(q, 99, &none, NULL, NULL) == COLA_OK) bad++;
    if (cola_run(q, NULL, &none, NULL, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_finish(q, &none, NULL, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_density(q, NULL, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_density_noalloc(q, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_pm_force(q, NULL, 0.5, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_cross_power(q, NULL, NULL, dd, NULL, NULL) == COLA_OK) bad++;
    if (cola_fft_r2c(q, 17, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_run_adjoint(q, NULL, NULL, NULL, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_ensemble_create(0, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_run_batched(0, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == COLA_OK) bad++;
    if (cola_ensemble_launch(NULL, NULL) == COLA_OK) bad++;
    if (cola_ensemble_destroy(NULL) != COLA_OK) bad++;
    if (cola_autotune(q, &none, NULL, 0, NULL, NULL, li) == COLA_OK) bad++;
    if (cola_trace_read(q, dd, li, 1) == COLA_OK) bad++;   /* capacity below the stage count */
    if (cola_workspace_bytes(NULL, &sz) == COLA_OK) bad++;
    if (cola_plan_destroy(q) != COLA_OK) bad++;
  }
  for (int s = -10; s <= 1; ++s) if (!cola_strerror(s)) bad++;
  for (int k = -1; k <= cola_trace_stage_count(); ++k) (void)cola_trace_stage_name(k);
  printf(bad ? "FAIL %d\n" : "OK\n", bad);
  return bad != 0;
}
