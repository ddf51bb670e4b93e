// Host-side checks of the library's planning and validation code, built with
// AddressSanitizer on the host side only (the device code is built as usual
// and never launched).
// Every call below returns before any HIP call: workspace queries, argument
// rejection on every entry point, and batch planning into a host buffer with
// stand-in device addresses (the planner only stores them). Prints "all checks
// passed" and exits 0, or names the failed check and exits 1; a memory error
// aborts under the sanitizer.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "tucker.h"

static int failures = 0;
#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);  \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static tucker_shape shape_of(int d, const int64_t* dims) {
  tucker_shape s;
  memset(&s, 0, sizeof(s));
  s.order = d;
  for (int k = 0; k < d && k < TUCKER_MAX_ORDER; ++k) s.dims[k] = dims[k];
  return s;
}

// splitmix64: a fixed pseudo-random stream of test shapes
static uint64_t rng_state = 0x12345678u;
static uint64_t next_u64() {
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

int main() {
  void* const fake = (void*)(uintptr_t)0x100000;  // a stand-in device address (never dereferenced)

  // workspace queries over random shapes, orders 1..8, every precision and variant
  for (int it = 0; it < 400; ++it) {
    const int d = (int)uniform(1, 8);
    int64_t dims[TUCKER_MAX_ORDER], ranks[TUCKER_MAX_ORDER];
    for (int k = 0; k < d; ++k) {
      dims[k] = uniform(1, d <= 3 ? 300 : 12);
      ranks[k] = uniform(1, dims[k]);
    }
    const tucker_shape s = shape_of(d, dims);
    const int p = (int)uniform(0, 12), q = (int)uniform(0, 4);
    for (int prec = 0; prec < 3; ++prec)
      for (int seq = 0; seq < 2; ++seq) {
        const size_t w = tucker_workspace_bytes(&s, ranks, p, q, (tucker_precision)prec, seq);
        tucker_options opt;
        memset(&opt, 0, sizeof(opt));
        CHECK(tucker_workspace_bytes_ex(&s, ranks, p, q, (tucker_precision)prec, seq, &opt) == w);
        opt.order_kind = TUCKER_ORDER_DECREASING;
        (void)tucker_workspace_bytes_ex(&s, ranks, p, q, (tucker_precision)prec, seq, &opt);
        opt.order_kind = TUCKER_ORDER_NATURAL;
        opt.holistic = 1;
        (void)tucker_workspace_bytes_ex(&s, ranks, p, q, (tucker_precision)prec, seq, &opt);
        for (int k = 0; k < d; ++k)
          (void)tucker_op_workspace_bytes(&s, k, (int64_t)uniform(1, 64), (tucker_precision)prec);
      }
  }

  // argument rejection before any launch
  const int64_t d3[3] = {40, 36, 30};
  const tucker_shape s3 = shape_of(3, d3);
  int64_t r3[3] = {5, 6, 4};
  void* U[3] = {fake, fake, fake};
  CHECK(tucker_rsthosvd(nullptr, fake, r3, 4, 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, fake, 1 << 30,
                        nullptr) == TUCKER_EINVAL);
  CHECK(tucker_rsthosvd(&s3, nullptr, r3, 4, 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, fake, 1 << 30,
                        nullptr) == TUCKER_EINVAL);
  CHECK(tucker_rthosvd(&s3, fake, r3, -1, 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, fake, 1 << 30,
                       nullptr) == TUCKER_EINVAL);
  CHECK(tucker_rthosvd(&s3, fake, r3, 4, TUCKER_MAX_Q + 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr,
                       fake, 1 << 30, nullptr) == TUCKER_EINVAL);
  CHECK(tucker_rsthosvd(&s3, fake, r3, 4, 1, TUCKER_SHIFT_ADAPTIVE, 1, (tucker_precision)7, fake, U, nullptr, fake,
                        1 << 30, nullptr) == TUCKER_EINVAL);
  CHECK(tucker_rsthosvd(&s3, fake, r3, 4, 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, fake, 16,
                        nullptr) == TUCKER_EWORKSPACE);
  int64_t bad_r[3] = {5, 6, 31};  // r_3 > n_3
  CHECK(tucker_rsthosvd(&s3, fake, bad_r, 4, 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, fake, 1 << 30,
                        nullptr) == TUCKER_EINVAL);
  int64_t infeasible[3] = {2, 2, 5};  // r_3 > r_1 r_2 in ST-HOSVD
  CHECK(tucker_rsthosvd(&s3, fake, infeasible, 4, 1, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, fake,
                        1 << 30, nullptr) == TUCKER_EINVAL);
  const int64_t d9[9] = {2, 2, 2, 2, 2, 2, 2, 2, 2};
  tucker_shape s9 = shape_of(8, d9);
  s9.order = 9;
  CHECK(tucker_workspace_bytes(&s9, r3, 1, 1, TUCKER_FP32, 1) == 0);
  tucker_options opt;
  memset(&opt, 0, sizeof(opt));
  opt.fp32_products = 2;
  CHECK(tucker_workspace_bytes_ex(&s3, r3, 4, 1, TUCKER_FP32, 1, &opt) == 0);
  memset(&opt, 0, sizeof(opt));
  opt.order_kind = TUCKER_ORDER_GIVEN;
  opt.order[0] = 0;
  opt.order[1] = 0;
  opt.order[2] = 1;  // not a permutation
  CHECK(tucker_workspace_bytes_ex(&s3, r3, 4, 1, TUCKER_FP32, 1, &opt) == 0);
  memset(&opt, 0, sizeof(opt));
  opt.reserved[3] = 1;
  CHECK(tucker_workspace_bytes_ex(&s3, r3, 4, 1, TUCKER_FP32, 1, &opt) == 0);
  CHECK(tucker_sketch(&s3, 0, fake, 41, 1, TUCKER_FP32, fake, fake, 1 << 30, nullptr) == TUCKER_EINVAL);
  CHECK(tucker_sketch(&s3, 3, fake, 4, 1, TUCKER_FP32, fake, fake, 1 << 30, nullptr) == TUCKER_EINVAL);
  CHECK(tucker_shifted_power(&s3, 0, fake, 4, fake, nullptr, 0, TUCKER_FP32, fake, (double*)fake, fake, 1 << 30, nullptr) ==
        TUCKER_EINVAL);
  CHECK(tucker_core(&s3, 0, fake, fake, 65, TUCKER_FP32, fake, nullptr) == TUCKER_EINVAL);
  CHECK(tucker_orth(10, 11, (const double*)fake, TUCKER_FP64, fake, (double*)fake, fake, 1 << 20, nullptr) ==
        TUCKER_EINVAL);
  CHECK(tucker_norm2(fake, -1, TUCKER_FP32, (double*)fake, fake, 1 << 20, nullptr) == TUCKER_EINVAL);
  CHECK(tucker_fill_gaussian(1, 9, 0, 10, 10, TUCKER_FP64, fake, nullptr) == TUCKER_EINVAL);
  int32_t qused[3];
  CHECK(tucker_rsthosvd_pve(&s3, fake, r3, 4, 0, 0.5, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr, qused,
                            fake, 1 << 30, nullptr) == TUCKER_EINVAL);
  const int64_t big[3] = {1000, 1000, 1000};
  const tucker_shape sb = shape_of(3, big);
  int64_t rb[3] = {50, 50, 50};
  CHECK(tucker_rsthosvd_noalloc(&sb, fake, rb, 10, 3, TUCKER_SHIFT_ADAPTIVE, 1, TUCKER_FP32, fake, U, nullptr,
                                nullptr) == TUCKER_EWORKSPACE);
  for (int st = -5; st <= 0; ++st) CHECK(tucker_status_string(st) != nullptr);

  // batch planning into host memory: random items of the serving distribution
  for (int rep = 0; rep < 20; ++rep) {
    const int cap = (int)uniform(1, 64), q = (int)uniform(0, 2), p = 8;
    const int n = (int)uniform(0, cap);
    std::vector<tucker_batch_item> items((size_t)n);
    int lmax = 0;
    for (int b = 0; b < n; ++b) {
      tucker_batch_item& it = items[(size_t)b];
      memset(&it, 0, sizeof(it));
      int64_t dims[3];
      for (int k = 0; k < 3; ++k) dims[k] = uniform(8, 64);
      it.shape = shape_of(3, dims);
      // ranks 2..4 keep every r_k <= r_i r_j, so each item is feasible
      for (int k = 0; k < 3; ++k) it.ranks[k] = uniform(2, 4);
      it.seed = (uint64_t)b;
      it.A = fake;
      it.G = fake;
      for (int k = 0; k < 3; ++k) it.U[k] = fake;
      it.info = (b & 1) ? (tucker_info*)fake : nullptr;
      for (int k = 0; k < 3; ++k) {
        const int l = (int)(it.ranks[k] + p < dims[k] ? it.ranks[k] + p : dims[k]);
        lmax = l > lmax ? l : lmax;
      }
    }
    const int lclass = lmax <= 16 ? 16 : 32;
    size_t ws = tucker_batch_table_bytes(cap, 3, q);
    CHECK(ws > 0);
    for (int b = 0; b < n; ++b) {
      const size_t ib = tucker_batch_item_bytes(&items[(size_t)b], p, q);
      CHECK(ib > 0);
      ws += (ib + 255) / 256 * 256 + 256;
    }
    const size_t pb = tucker_batch_plan_bytes(cap, 3, q);
    CHECK(pb > 0);
    std::vector<unsigned char> plan(pb);
    const int rc = tucker_batch_plan(cap, 3, lclass, n, n ? items.data() : nullptr, p, q, TUCKER_SHIFT_ADAPTIVE, fake,
                                     ws, plan.data(), plan.size());
    if (rc != TUCKER_OK) fprintf(stderr, "batch plan: %s\n", tucker_status_string(rc));
    CHECK(rc == TUCKER_OK);
    // a plan buffer one byte short, a workspace too small
    if (pb > 0)
      CHECK(tucker_batch_plan(cap, 3, lclass, n, n ? items.data() : nullptr, p, q, TUCKER_SHIFT_ADAPTIVE, fake,
                              ws, plan.data(), plan.size() - 1) == TUCKER_EWORKSPACE);
    if (n > 0)
      CHECK(tucker_batch_plan(cap, 3, lclass, n, items.data(), p, q, TUCKER_SHIFT_ADAPTIVE, fake, 16, plan.data(),
                              plan.size()) == TUCKER_EWORKSPACE);
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("all checks passed\n");
  return 0;
}
