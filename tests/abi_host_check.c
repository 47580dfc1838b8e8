/*
 * Host-side argument validation of the C ABI, run under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  The library is compiled host-only (no device
 * code) with the sanitizers, and this driver calls every entry point whose
 * validation needs no device: NULL handles and buffers, out-of-range sizes,
 * precisions, tolerances and temperatures.  Each call must return its status
 * without touching the GPU; any invalid read, write, overflow or undefined
 * operation on the way aborts the program.
 *
 * Built and run by tests/test_abi_host.py (not part of the library).
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "ephw.h"

static int failures = 0;

static void expect(const char* what, ephw_status got, ephw_status want) {
  if (got != want) {
    fprintf(stderr, "FAIL %s: status %d (%s), expected %d; last error: %s\n", what, (int)got,
            ephw_status_string(got), (int)want, ephw_last_error());
    ++failures;
  }
}

int main(void) {
  /* status strings, including out-of-range codes */
  for (int s = -3; s < 100; ++s) {
    const char* t = ephw_status_string(s);
    if (!t || !t[0]) {
      fprintf(stderr, "FAIL empty status string for %d\n", s);
      ++failures;
    }
  }
  if (ephw_version() != 200) {
    fprintf(stderr, "FAIL version %d\n", (int)ephw_version());
    ++failures;
  }

  /* handles */
  expect("ctx_create out NULL", ephw_ctx_create(0, NULL), EPHW_EINVAL);
  expect("ctx_check NULL", ephw_ctx_check(NULL, NULL), EPHW_EINVAL);
  expect("ctx_set_limits NULL", ephw_ctx_set_limits(NULL, 0, 40), EPHW_EINVAL);
  expect("ctx_memory NULL", ephw_ctx_memory(NULL, NULL, NULL), EPHW_EINVAL);
  expect("system_load NULL", ephw_system_load(NULL, NULL, NULL), EPHW_EINVAL);
  expect("system_set_g NULL", ephw_system_set_g(NULL, NULL, NULL), EPHW_EINVAL);
  expect("system_bytes NULL", ephw_system_bytes(NULL, NULL), EPHW_EINVAL);
  expect("system_trim NULL", ephw_system_trim(NULL), EPHW_EINVAL);
  expect("window_pairs NULL",
         ephw_window_pairs(NULL, NULL, 4, 0.0, 1.0, EPHW_PAIRS_AUTO, NULL, NULL, NULL, NULL, 0, NULL, NULL),
         EPHW_EINVAL);
  expect("interpolate_pairs NULL",
         ephw_interpolate_pairs(NULL, NULL, 4, EPHW_PAIRS_BY_Q, NULL, NULL, NULL, 0, 1, EPHW_OUT_G, 0, 0, NULL, NULL,
                                NULL, 0, NULL),
         EPHW_EINVAL);
  expect("set_q_batch NULL", ephw_set_q_batch(NULL, 4), EPHW_EINVAL);
  expect("set_k_tile NULL", ephw_set_k_tile(NULL, 4), EPHW_EINVAL);
  expect("kset_create NULL", ephw_kset_create(NULL, NULL, 4, 0, NULL, NULL), EPHW_EINVAL);
  expect("kset_bands NULL", ephw_kset_bands(NULL, NULL, NULL, NULL), EPHW_EINVAL);
  expect("profile_enable NULL", ephw_profile_enable(NULL, 1), EPHW_EINVAL);
  expect("profile_read NULL", ephw_profile_read(NULL, NULL, NULL), EPHW_EINVAL);
  expect("batch_create NULL", ephw_batch_create(NULL, NULL, 0, NULL, NULL, NULL), EPHW_EINVAL);
  expect("batch_run NULL", ephw_batch_run(NULL, NULL), EPHW_EINVAL);
  expect("batch_shape NULL", ephw_batch_shape(NULL, 0, NULL, NULL, NULL, NULL), EPHW_EINVAL);
  expect("batch_stats NULL", ephw_batch_stats(NULL, NULL, NULL), EPHW_EINVAL);
  expect("batch_solo NULL", ephw_batch_solo(NULL, 0, NULL), EPHW_EINVAL);

  /* compute calls with NULL handles or buffers */
  expect("bands NULL", ephw_bands(NULL, NULL, 3, NULL, NULL, NULL), EPHW_EINVAL);
  expect("phonons NULL", ephw_phonons(NULL, NULL, 3, NULL, NULL, NULL, NULL), EPHW_EINVAL);
  expect("phase_sum_rp NULL", ephw_phase_sum_rp(NULL, NULL, 3, 0, NULL, NULL), EPHW_EINVAL);
  expect("interpolate NULL",
         ephw_interpolate(NULL, NULL, 1, NULL, 0, 0, EPHW_OUT_G, NULL, NULL, NULL, 0, NULL, NULL, NULL),
         EPHW_EINVAL);
  expect("interpolate_noalloc NULL",
         ephw_interpolate_noalloc(NULL, NULL, 1, NULL, 0, 0, EPHW_OUT_G, NULL, NULL, NULL, 0, NULL, NULL, NULL),
         EPHW_EINVAL);
  expect("interpolate_linewidth NULL",
         ephw_interpolate_linewidth(NULL, NULL, 1, NULL, 0.02, 0.0, 0.01, 0.0, 1, NULL, NULL), EPHW_EINVAL);
  expect("wannier_transform NULL", ephw_wannier_transform(NULL, NULL, 4, NULL, NULL, NULL, NULL), EPHW_EINVAL);
  expect("window_screen NULL",
         ephw_window_screen(NULL, NULL, 4, NULL, 0.0, 1.0, NULL, NULL, NULL, NULL, NULL, NULL, NULL), EPHW_EINVAL);
  expect("loss_backward NULL",
         ephw_loss_backward(NULL, NULL, 1, NULL, 0, 0, NULL, NULL, NULL, NULL, NULL), EPHW_EINVAL);

  /* degenerate-block sums: precision, sizes, tolerance and buffers */
  expect("degsums prec", ephw_degenerate_sums(7, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 1e-6, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums nw 0", ephw_degenerate_sums(0, NULL, 1, 1, 3, 0, NULL, NULL, NULL, 1e-6, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums nw huge", ephw_degenerate_sums(0, NULL, 1, 1, 3, 1 << 30, NULL, NULL, NULL, 1e-6, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums nq < 0", ephw_degenerate_sums(0, NULL, -1, 1, 3, 4, NULL, NULL, NULL, 1e-6, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums tol < 0", ephw_degenerate_sums(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, -1.0, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums tol nan", ephw_degenerate_sums(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, NAN, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums tol inf", ephw_degenerate_sums(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, INFINITY, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums NULL g", ephw_degenerate_sums(0, NULL, 2, 3, 3, 4, NULL, NULL, NULL, 1e-6, NULL, NULL),
         EPHW_EINVAL);
  expect("degsums empty", ephw_degenerate_sums(1, NULL, 0, 3, 3, 4, NULL, NULL, NULL, 1e-6, NULL, NULL), EPHW_OK);

  /* linewidth: temperature and width positive and finite, nq_total >= 1, buffers present */
  expect("lw T 0", ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.0, 0.0, 0.01, 0.0, 1, NULL, NULL),
         EPHW_EINVAL);
  expect("lw T nan", ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, NAN, 0.0, 0.01, 0.0, 1, NULL, NULL),
         EPHW_EINVAL);
  expect("lw sigma < 0",
         ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.02, 0.0, -1.0, 0.0, 1, NULL, NULL), EPHW_EINVAL);
  expect("lw mu inf",
         ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.02, INFINITY, 0.01, 0.0, 1, NULL, NULL),
         EPHW_EINVAL);
  expect("lw omega_min < 0",
         ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.02, 0.0, 0.01, -1.0, 1, NULL, NULL), EPHW_EINVAL);
  expect("lw nq_total 0",
         ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.02, 0.0, 0.01, 0.0, 0, NULL, NULL), EPHW_EINVAL);
  expect("lw NULL g", ephw_linewidth(0, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.02, 0.0, 0.01, 0.0, 1, NULL, NULL),
         EPHW_EINVAL);
  expect("lw prec", ephw_linewidth(9, NULL, 1, 1, 3, 4, NULL, NULL, NULL, 0.02, 0.0, 0.01, 0.0, 1, NULL, NULL),
         EPHW_EINVAL);
  expect("lw empty", ephw_linewidth(1, NULL, 0, 1, 3, 4, NULL, NULL, NULL, 0.02, 0.0, 0.01, 0.0, 1, NULL, NULL),
         EPHW_OK);

  /* freeing NULL handles is a no-op */
  expect("system_free NULL", ephw_system_free(NULL), EPHW_OK);
  expect("kset_free NULL", ephw_kset_free(NULL), EPHW_OK);
  expect("batch_free NULL", ephw_batch_free(NULL), EPHW_OK);
  expect("ctx_destroy NULL", ephw_ctx_destroy(NULL), EPHW_OK);

  /* the last error stays a readable string after all of the above */
  const char* e = ephw_last_error();
  if (!e || strlen(e) > 4096) {
    fprintf(stderr, "FAIL last error string\n");
    ++failures;
  }
  if (failures) return 1;
  printf("abi_host_check: ok\n");
  return 0;
}
