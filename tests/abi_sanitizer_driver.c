/* Host-side checks of the C ABI, run against the checking build of the
 * library (AddressSanitizer + UndefinedBehaviorSanitizer on the host code,
 * CHEFSI_DEBUG table checks).  Every call below either fails argument
 * validation on the host or builds a plan (whose tables the debug build
 * verifies before any device upload); none dereferences a device pointer.
 * Without a GPU a valid plan stops at hipGetDevice with CHEFSI_ERR_HIP.
 * Exit status 0 when every result is as expected. */
#include <stdio.h>
#include <string.h>

#include "chefsi.h"

static int failures = 0, checks = 0;

static void expect(int got, int want, const char* what) {
  ++checks;
  if (got != want) {
    ++failures;
    printf("FAIL %s: got %d, want %d (%s)\n", what, got, want, chefsi_last_error());
  }
}

static void plan_case(int nx, int ny, int nz, int stencil, const int32_t* J, const char* what) {
  chefsi_plan p = NULL;
  const int rc = chefsi_plan_create(&p, nx, ny, nz, stencil, J);
  ++checks;
  if (rc == CHEFSI_OK) {
    chefsi_plan_destroy(p);
  } else if (rc != CHEFSI_ERR_HIP || strstr(chefsi_last_error(), "table check") != NULL) {
    ++failures;
    printf("FAIL plan %s: rc %d (%s)\n", what, rc, chefsi_last_error());
  }
}

int main(void) {
  int32_t J8[8], J12[12], J6[6], J27[27], J2[2];
  size_t bytes = 0;
  double fake[4];
  for (int i = 0; i < 8; ++i) J8[i] = 32;
  for (int i = 0; i < 6; ++i) J6[i] = 24;
  for (int i = 0; i < 27; ++i) J27[i] = 40;
  {
    const int32_t mix[12] = {8, 16, 13, 40, 64, 128, 200, 256, 129, 127, 56, 1};
    memcpy(J12, mix, sizeof(mix));
  }
  J2[0] = 1;
  J2[1] = 256;

  ++checks;
  if (chefsi_version() == NULL || strncmp(chefsi_version(), "chefsi", 6) != 0) {
    ++failures;
    printf("FAIL version\n");
  }

  /* plan arguments */
  expect(chefsi_plan_create(NULL, 2, 2, 2, 7, J8), CHEFSI_ERR_ARG, "plan out NULL");
  {
    chefsi_plan p = NULL;
    expect(chefsi_plan_create(&p, 0, 2, 2, 7, J8), CHEFSI_ERR_ARG, "plan nx 0");
    expect(chefsi_plan_create(&p, 2, 2, 2, 6, J8), CHEFSI_ERR_ARG, "plan stencil 6");
    expect(chefsi_plan_create(&p, 2, 2, 2, 7, NULL), CHEFSI_ERR_ARG, "plan counts NULL");
    J8[3] = 0;
    expect(chefsi_plan_create(&p, 2, 2, 2, 7, J8), CHEFSI_ERR_ARG, "plan J 0");
    J8[3] = 257;
    expect(chefsi_plan_create(&p, 2, 2, 2, 7, J8), CHEFSI_ERR_ARG, "plan J 257");
    J8[3] = 32;
    expect(chefsi_plan_create(&p, 4096, 4096, 4096, 7, J8), CHEFSI_ERR_ARG, "plan too many elements");
  }

  /* valid plans: the debug build checks every table before the upload */
  plan_case(2, 2, 2, 7, J8, "uniform 2x2x2");
  plan_case(4, 3, 1, 5, J12, "mixed sheet 4x3");
  plan_case(3, 2, 1, 7, J6, "length-1 z under the 7-point stencil");
  plan_case(3, 3, 3, 7, J27, "odd 3x3x3");
  plan_case(2, 1, 1, 7, J2, "extreme counts 1 and 256");
  plan_case(2, 1, 1, 5, J2, "extreme counts, 5-point");

  /* entry points that validate without a plan or before using it */
  expect(chefsi_workspace_bytes(NULL, CHEFSI_OP_FILTER, 8, 0, 1, 1, &bytes), CHEFSI_ERR_ARG, "ws NULL plan");
  expect(chefsi_orthonormalize_workspace_bytes(100, 10, 2, &bytes), CHEFSI_OK, "orth ws");
  ++checks;
  if (bytes == 0) {
    ++failures;
    printf("FAIL orth ws size 0\n");
  }
  expect(chefsi_orthonormalize_workspace_bytes(10, 100, 2, &bytes), CHEFSI_ERR_ARG, "orth ws ns > n");
  expect(chefsi_orthonormalize_workspace_bytes(100, 10, 3, &bytes), CHEFSI_ERR_ARG, "orth ws passes 3");
  expect(chefsi_orthonormalize_workspace_bytes(100, 10, 2, NULL), CHEFSI_ERR_ARG, "orth ws bytes NULL");
  expect(chefsi_orthonormalize_backward_workspace_bytes(100, 10, &bytes), CHEFSI_OK, "orth bwd ws");
  expect(chefsi_orthonormalize_backward_workspace_bytes(5, 10, &bytes), CHEFSI_ERR_ARG, "orth bwd ws ns > n");
  expect(chefsi_orthonormalize(0, 4, fake, 4, 2, NULL, NULL, 0, NULL), CHEFSI_ERR_ARG, "orth n 0");
  expect(chefsi_orthonormalize(100, 4, NULL, 4, 2, NULL, NULL, 0, NULL), CHEFSI_ERR_ARG, "orth Y NULL");
  expect(chefsi_orthonormalize(100, 4, fake, 2, 2, NULL, NULL, 0, NULL), CHEFSI_ERR_ARG, "orth ld < ns");
  expect(chefsi_orthonormalize_backward(100, 4, fake, 4, NULL, fake, 4, fake, 4, NULL, 0, NULL), CHEFSI_ERR_ARG,
         "orth bwd U NULL");
  expect(chefsi_orthonormalize_backward(100, 4, fake, 4, fake, fake, 4, fake, 4, NULL, 0, NULL), CHEFSI_ERR_ARG,
         "orth bwd output overlaps Yhat");
  expect(chefsi_occupations(0, fake, 1.0, 1e-3, fake, fake, NULL), CHEFSI_ERR_ARG, "occ ns 0");
  expect(chefsi_occupations(4, fake, 1.0, 0.0, fake + 1, fake + 2, NULL), CHEFSI_ERR_ARG, "occ kT 0");
  expect(chefsi_occupations(4, fake, 4.0, 1e-3, fake, fake, NULL), CHEFSI_ERR_ARG, "occ n_occ = ns");
  expect(chefsi_filter(NULL, fake, 4, 0.0, 1.0, -1.0, 0, fake, 4, fake, 4, 4, NULL, 0, NULL), CHEFSI_ERR_ARG,
         "filter NULL plan");
  expect(chefsi_filter_noalloc(NULL, fake, 4, 0.0, 1.0, -1.0, 0, fake, 4, fake, 4, 4, NULL), CHEFSI_ERR_ARG,
         "filter_noalloc NULL plan");
  expect(chefsi_bounds(NULL, fake, fake, 20, NULL, 4, NULL, NULL, NULL, 0, NULL), CHEFSI_ERR_ARG, "bounds NULL plan");
  expect(chefsi_rayleigh_ritz(NULL, fake, fake, 4, 4, fake, 4, fake, NULL, NULL, NULL, 0, NULL), CHEFSI_ERR_ARG,
         "rr NULL plan");
  expect(chefsi_sweep(NULL, fake, 4, 0, 0, 20, fake, NULL, 0, fake, 4, 4, fake, NULL, NULL, NULL, NULL, 0, NULL),
         CHEFSI_ERR_ARG, "sweep NULL plan");
  expect(chefsi_loss(NULL, fake, 4, 0.0, 1.0, -1.0, 2, 2, fake, 4, 4, fake, NULL, 0, NULL), CHEFSI_ERR_ARG,
         "loss NULL plan");
  expect(chefsi_rayleigh_ritz_backward(NULL, fake, fake, 4, 4, fake, fake, fake, 4, fake, 0, NULL, 0, NULL),
         CHEFSI_ERR_ARG, "rr bwd NULL plan");
  expect(chefsi_density_blocks(NULL, fake, 4, 4, fake, fake, NULL, 0, NULL), CHEFSI_ERR_ARG, "density NULL plan");
  expect(chefsi_realign(NULL, 8, fake, fake, fake, 4, 4, NULL, 0, NULL), CHEFSI_ERR_ARG, "realign NULL plan");
  expect(chefsi_plan_neighbour(NULL, 0, 0), -1, "neighbour NULL plan");
  chefsi_plan_destroy(NULL);

  printf("%d checks, %d failures\n", checks, failures);
  return failures == 0 ? 0 : 1;
}
