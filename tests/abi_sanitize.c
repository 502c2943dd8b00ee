/* Host-side driver for the sanitizer build of libgp2s (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code only): exercises the context lifecycle,
 * option defaults, status strings and the scalar validation of every parameter, none
 * of which touches a GPU. Exits 0 when every check holds; a sanitizer report aborts. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "gp2s.h"

static int failures = 0;
#define CHECK(cond)                                                 \
  do {                                                              \
    if (!(cond)) {                                                  \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static gp2s_params base(double* centers, double* weights) {
  gp2s_params p;
  memset(&p, 0, sizeof(p));
  p.dim = 2;
  p.n_bumps = 2;
  p.radius = 0.05;
  p.bump_width = 0.6;
  p.noise_var = 1e-4;
  p.centers = centers;
  p.weights = weights;
  return p;
}

int main(void) {
  double centers[6] = {0.2, 0.3, 0.7, 0.6, 0.5, 0.5};
  double weights[2] = {1.0, -0.5};
  double radii[3] = {0.05, 0.02, 0.03};
  double ls[2] = {0.3, -0.2};
  int32_t groups[2] = {0, 1};
  CHECK(gp2s_abi_version() == GP2S_ABI_VERSION);
  gp2s_solve_opts o;
  gp2s_default_opts(&o);
  gp2s_default_opts(NULL);
  CHECK(o.n_probes == 64 && o.tol == 1e-8 && o.probe_tol == 1e-5 && o.precond == GP2S_PRECOND_BLOCK);
  for (int s = -1; s < 12; ++s) CHECK(gp2s_status_string(s) != NULL);
  CHECK(gp2s_create(NULL, NULL, NULL, NULL, NULL) == GP2S_E_INVALID);
  for (int round = 0; round < 3; ++round) {
    gp2s_ctx ctx = NULL;
    CHECK(gp2s_create(&ctx, NULL, NULL, NULL, NULL) == GP2S_OK);
    gp2s_params p = base(centers, weights);
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_OK);
    CHECK(gp2s_check_params(ctx, 0, &p) == GP2S_E_INVALID);
    CHECK(gp2s_check_params(ctx, (int64_t)1 << 31, &p) == GP2S_E_INVALID);
    CHECK(gp2s_check_params(ctx, 100, NULL) == GP2S_E_INVALID);
    p.dim = 5;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_INVALID);
    p = base(centers, weights);
    p.radius = NAN;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_NONFINITE);
    p = base(centers, weights);
    p.noise_var = -1.0;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_INVALID);
    p = base(centers, weights);
    p.n_bumps = 0;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_INVALID);
    p = base(centers, weights);
    p.n_bumps = 100000;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_INVALID);
    p = base(centers, weights);
    p.kernel = 7;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_INVALID);
    p = base(centers, weights);
    p.radii = radii;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_OK);
    p.dim = 3;
    p.n_bumps = 1;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_OK);
    p = base(centers, weights);
    p.ls_weights = ls;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_OK);
    p = base(centers, weights);
    p.ff_groups = groups;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_OK);
    p.radii = radii;
    CHECK(gp2s_check_params(ctx, 100, &p) == GP2S_E_INVALID);
    CHECK(strlen(gp2s_last_error(ctx)) > 0);
    /* entry points reject bad arguments before any device call */
    gp2s_matrix h = NULL;
    p = base(centers, weights);
    CHECK(gp2s_assemble(ctx, 10, NULL, &p, GP2S_MIXED, &h) == GP2S_E_INVALID);
    CHECK(gp2s_assemble(ctx, 10, centers, &p, 9, &h) == GP2S_E_INVALID);
    CHECK(gp2s_spmv(ctx, NULL, 1, NULL, NULL) == GP2S_E_INVALID);
    CHECK(gp2s_spmv_noalloc(ctx, NULL, 1, NULL, NULL) == GP2S_E_INVALID);
    gp2s_report rep;
    o.n_probes = 65;
    CHECK(gp2s_lml(ctx, NULL, NULL, &o, NULL, &rep) == GP2S_E_INVALID);
    o.n_probes = 64;
    CHECK(gp2s_matrix_set_block_product(NULL, 64, 1) == GP2S_E_INVALID);
    CHECK(gp2s_set_timing_mask(ctx, 0xffffffffu) == GP2S_OK);
    gp2s_stats stats;
    CHECK(gp2s_get_stats(ctx, &stats) == GP2S_OK);
    CHECK(gp2s_set_timing(ctx, 0) == GP2S_OK);
    CHECK(gp2s_destroy(ctx) == GP2S_OK);
  }
  CHECK(gp2s_destroy(NULL) == GP2S_E_INVALID);
  if (failures) fprintf(stderr, "%d checks failed\n", failures);
  else printf("sanitized host checks passed\n");
  return failures ? 1 : 0;
}
