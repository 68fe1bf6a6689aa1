/* Host-only exercise of the C ABI's argument validation, options, footprints and status strings,
 * linked against a build of the library whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Every call here must return before any device work (no GPU is
 * needed); the sanitizers report any invalid host memory access or undefined behaviour on the way. */
#include <stdio.h>
#include <string.h>

#include "fossils.h"

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "expectation failed: %s (line %d)\n", #cond, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(void) {
  fs_options o;
  memset(&o, 0, sizeof o);
  EXPECT(fs_options_default(1000000, 1000, &o) == FS_OK);
  EXPECT(o.d == 12000 && o.zeta == 8 && o.kw_every == 5 && o.max_inner == 100);
  EXPECT(fs_options_default(5, 10, &o) == FS_ERR_SHAPE);
  EXPECT(fs_options_default(5, 0, &o) == FS_ERR_SHAPE);
  EXPECT(fs_options_default(5, 2, NULL) == FS_ERR_INVALID_ARG);
  for (int s = -10; s <= 4; ++s) {
    const char* str = fs_status_string((fs_status)s);
    EXPECT(str != NULL && strlen(str) > 3);
  }
  EXPECT(fs_last_error_detail() != NULL);
  /* null context / server / sketch handles */
  double dummy[4] = {0, 0, 0, 0};
  EXPECT(fossils_solve(NULL, 10, 2, dummy, 10, dummy, dummy, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(spir_solve(NULL, 10, 2, dummy, 10, dummy, dummy, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(spir_lsqr_solve(NULL, 10, 2, dummy, 10, dummy, dummy, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fossils_solve_complex(NULL, 10, 2, dummy, 10, dummy, dummy, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fossils_solve_multi(NULL, 10, 2, dummy, 10, 3, dummy, 10, dummy, 2, NULL, NULL) < 0);
  EXPECT(fossils_solve_mixed(NULL, 10, 2, dummy, 10, NULL, 0, dummy, dummy, NULL, NULL) < 0);
  EXPECT(fossils_solve_noalloc(NULL, 10, 2, dummy, 10, dummy, dummy, NULL, NULL) == FS_ERR_INVALID_ARG);
  {
    fs_problem pr = {10, 2, dummy, 10, dummy, dummy, FS_METHOD_FOSSILS};
    fs_status sts[1] = {FS_OK};
    EXPECT(fossils_solve_batched(NULL, 1, &pr, NULL, NULL, sts) == FS_ERR_INVALID_ARG);
    EXPECT(fossils_solve_batched(NULL, 0, &pr, NULL, NULL, sts) == FS_ERR_INVALID_ARG);
    EXPECT(fossils_solve_batched(NULL, 1, NULL, NULL, NULL, sts) == FS_ERR_INVALID_ARG);
  }
  EXPECT(fs_context_destroy(NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_context_create(0, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(sketch_create(NULL, 10, 5, 2, 1, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(sketch_destroy(NULL) == FS_ERR_INVALID_ARG);
  EXPECT(sketch_indices(NULL, 0, 1, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(sketch_apply(NULL, 2, dummy, 10, dummy, dummy, 10, NULL, 0) == FS_ERR_INVALID_ARG);
  EXPECT(fs_sketch_qr(NULL, 10, 2, dummy, 10) == FS_ERR_INVALID_ARG);
  EXPECT(fs_svd_triangular(NULL, 2, dummy, 2, dummy, dummy, 2, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_normal_pass(NULL, 10, 2, dummy, 10, dummy, dummy) == FS_ERR_INVALID_ARG);
  EXPECT(fs_residual_pass(NULL, 10, 2, dummy, 10, dummy, dummy, dummy, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_trsv(NULL, 2, dummy, 2, 0, dummy, dummy) == FS_ERR_INVALID_ARG);
  EXPECT(fs_triangular_inverse(NULL, 2, dummy, 2, dummy) == FS_ERR_INVALID_ARG);
  EXPECT(fs_time_normal_pass(NULL, 10, 2, dummy, 10, dummy, dummy, 1, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_tune_pass(NULL, 10, 2, dummy, 10, dummy, dummy, 1, NULL, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_set_pass_tuning(NULL, 10, 2, 16, 256) == FS_ERR_INVALID_ARG);
  EXPECT(fs_clear_pass_tuning(NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_to_fp32(NULL, 10, 2, dummy, 10, NULL, 10) == FS_ERR_INVALID_ARG);
  EXPECT(fs_context_workspace(NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_context_trim(NULL) == FS_ERR_INVALID_ARG);
  fs_server h = NULL;
  EXPECT(fs_server_create(NULL, 1u << 30, 2, &h) == FS_ERR_INVALID_ARG);
  EXPECT(fs_server_destroy(NULL) == FS_ERR_INVALID_ARG);
  EXPECT(batched_submit(NULL, NULL, NULL) == FS_ERR_INVALID_ARG);
  int32_t done = 0;
  EXPECT(batched_poll(NULL, 1, &done, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_server_wait(NULL, 1) == FS_ERR_INVALID_ARG);
  EXPECT(fs_server_ticket_times(NULL, 1, NULL, NULL, NULL) == FS_ERR_INVALID_ARG);
  EXPECT(fs_server_memory(NULL, NULL, NULL, NULL) == FS_ERR_INVALID_ARG);
  size_t bytes = 0;
  EXPECT(fs_server_request_footprint(NULL, 10, 2, NULL, &bytes) == FS_ERR_INVALID_ARG);
  /* workspace footprints over a sweep of shapes and options (integer arithmetic on large sizes) */
  size_t prev = 0;
  for (long long m = 1000; m <= 100000000LL; m *= 10) {
    const size_t f = fs_solve_footprint(m, 500, NULL);
    EXPECT(f > prev);
    prev = f;
  }
  EXPECT(fs_solve_footprint(10, 20, NULL) == 0);
  EXPECT(fs_options_default(2000000, 15000, &o) == FS_OK);
  EXPECT(fs_solve_footprint(2000000, 15000, &o) > (size_t)8 * 180000 * 15001);
  o.d = 60000;
  o.zeta = 64;
  EXPECT(fs_solve_footprint(2000000, 15000, &o) > 0);
  if (fails) {
    fprintf(stderr, "%d expectation(s) failed\n", fails);
    return 1;
  }
  printf("sanitized host checks passed\n");
  return 0;
}
