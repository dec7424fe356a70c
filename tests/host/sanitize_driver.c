/* Host-side checks of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer:
 * descriptor validation over valid, invalid and extreme descriptors, and every entry point
 * with missing arguments.  None of these calls reaches the device, so the driver runs on a
 * machine without a GPU.  Exit status 0 when every expectation holds; a sanitizer report
 * aborts the process. */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "bfly.h"

static int failures = 0;
#define EXPECT(c)                                               \
  do {                                                          \
    if (!(c)) {                                                 \
      printf("expectation failed (line %d): %s\n", __LINE__, #c); \
      ++failures;                                               \
    }                                                           \
  } while (0)

static bf_bank_desc base(int32_t precision, int32_t L) {
  bf_bank_desc d;
  memset(&d, 0, sizeof d);
  d.fs = 4096.0;
  d.L = L;
  d.n_f0 = 2880;
  d.n_fdot = 3000;
  d.shard_index = 0;
  d.shard_count = 12;
  d.precision = precision;
  d.f0_min = 50.0;
  d.f0_max = 2000.0;
  d.fdot_min = -2000.0;
  d.fdot_max = 2000.0;
  return d;
}

static int is_status(bf_status s) { return s <= 0 && s >= BF_ECANCELED; }

int main(void) {
  const int32_t precisions[] = {BF_FP32, BF_BF16X3, BF_FP8, BF_F16X2, BF_FFT, BF_F16F8, BF_F16F6};
  const int32_t lengths[] = {1, 2, 37, 64, 2000, 4095, 4096, 4097, 4224, 4225, 8192, 8193};
  for (size_t i = 0; i < sizeof precisions / sizeof precisions[0]; ++i)
    for (size_t j = 0; j < sizeof lengths / sizeof lengths[0]; ++j) {
      bf_bank_desc d = base(precisions[i], lengths[j]);
      size_t bytes = 0;
      const bf_status st = bf_bank_bytes(&d, &bytes);
      EXPECT(st == BF_OK || st == BF_EINVAL);
      if (st == BF_OK) EXPECT(bytes > 0 && bytes % 256 == 0);
      else EXPECT(strlen(bf_last_error()) > 0);
      if (lengths[j] > 8192) EXPECT(st == BF_EINVAL);
    }

  /* invalid and extreme descriptors: every one rejected, none overflows */
  const double bad_doubles[] = {0.0, -1.0, NAN, INFINITY, -INFINITY};
  for (size_t i = 0; i < sizeof bad_doubles / sizeof bad_doubles[0]; ++i) {
    bf_bank_desc d = base(BF_FP32, 2000);
    size_t bytes = 0;
    d.fs = bad_doubles[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_FP32, 2000);
    d.f0_max = bad_doubles[i] == 0.0 ? 10.0 : bad_doubles[i];   /* 10 < f0_min */
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_FP32, 2000);
    d.fdot_min = isfinite(bad_doubles[i]) ? 3000.0 : bad_doubles[i];   /* > fdot_max */
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
  }
  const int32_t bad_ints[] = {0, -1, INT32_MIN};
  for (size_t i = 0; i < sizeof bad_ints / sizeof bad_ints[0]; ++i) {
    size_t bytes = 0;
    bf_bank_desc d = base(BF_BF16X3, 2000);
    d.L = bad_ints[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_BF16X3, 2000);
    d.n_f0 = bad_ints[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_BF16X3, 2000);
    d.n_fdot = bad_ints[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_BF16X3, 2000);
    d.shard_count = bad_ints[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_BF16X3, 2000);
    d.shard_index = bad_ints[i] == 0 ? 12 : bad_ints[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
    d = base(BF_BF16X3, 2000);
    d.precision = bad_ints[i] == 0 ? 7 : bad_ints[i];
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);
  }
  {
    size_t bytes = 0;
    bf_bank_desc d = base(BF_FP32, 8192);
    d.n_f0 = INT32_MAX;
    d.n_fdot = INT32_MAX;
    d.shard_count = 1;
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);   /* too many templates */
    d.shard_count = INT32_MAX;
    d.shard_index = INT32_MAX - 1;
    d.n_fdot = 1;
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_OK);       /* one template per shard */
    d.n_f0 = 46341;
    d.n_fdot = 46341;
    d.shard_count = 1;
    d.shard_index = 0;
    EXPECT(bf_bank_bytes(&d, &bytes) == BF_EINVAL);   /* 2^31 templates */
  }

  /* missing arguments */
  {
    bf_bank_desc d = base(BF_FP32, 2000);
    size_t bytes = 0;
    int64_t n = 100000;
    bf_bank* bank = NULL;
    EXPECT(bf_bank_bytes(NULL, &bytes) == BF_EINVAL);
    EXPECT(bf_bank_bytes(&d, NULL) == BF_EINVAL);
    EXPECT(bf_bank_create(&d, NULL, 1u << 20, NULL, &bank) == BF_EINVAL && bank == NULL);
    EXPECT(bf_bank_create(&d, (void*)&bytes, 1u << 20, NULL, NULL) == BF_EINVAL);
    EXPECT(bf_bank_info(NULL, NULL, NULL, NULL, NULL, NULL) == BF_EINVAL);
    EXPECT(bf_workspace_bytes(NULL, &n, 1, NULL, &bytes) == BF_EINVAL);
    EXPECT(bf_tails_workspace_bytes(NULL, &n, 1, NULL, &bytes) == BF_EINVAL);
    EXPECT(bf_coincidence_workspace_bytes(NULL, n, 10, &bytes) == BF_EINVAL);
    EXPECT(bf_search_segment(NULL, NULL, n, NULL, NULL, NULL, 0, NULL) == BF_EINVAL);
    EXPECT(bf_search_batch(NULL, NULL, 1, NULL, NULL, 0, NULL) == BF_EINVAL);
    EXPECT(bf_search_tails(NULL, NULL, 1, 5.0f, NULL, NULL, 0, NULL) == BF_EINVAL);
    EXPECT(bf_coincidence(NULL, NULL, NULL, n, 0, 0.0, NULL, NULL, NULL, NULL, 0, NULL) ==
           BF_EINVAL);
    int32_t nr = 0;
    int64_t items = 0;
    EXPECT(bf_plan(NULL, &n, 1, &nr, &items) == BF_EINVAL);
    EXPECT(bf_server_create(NULL, NULL, NULL) == BF_EINVAL);
    EXPECT(bf_server_request_bytes(NULL, n, &bytes) == BF_EINVAL);
    uint64_t ticket = 0;
    EXPECT(bf_submit(NULL, NULL, n, &ticket) == BF_EINVAL);
    int32_t state = 0;
    EXPECT(is_status(bf_poll(NULL, 1, &state, NULL, NULL, NULL)));
    EXPECT(is_status(bf_cancel(NULL, 1)));
    EXPECT(is_status(bf_server_stats(NULL, NULL, NULL, NULL, NULL, NULL)));
    EXPECT(bf_server_destroy(NULL) == BF_OK || bf_server_destroy(NULL) == BF_EINVAL);
    EXPECT(bf_bank_destroy(NULL) == BF_OK || bf_bank_destroy(NULL) == BF_EINVAL);
    EXPECT(bf_kernel_times(NULL, NULL) == BF_EINVAL);
    EXPECT(bf_set_timing(1) == BF_OK);
    double ms[8];
    int32_t searches = -1;
    EXPECT(bf_kernel_times(ms, &searches) == BF_EAGAIN);   /* no timed search ran */
    EXPECT(bf_set_timing(0) == BF_OK);
    EXPECT(bf_last_error() != NULL);
  }
  printf("%d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
