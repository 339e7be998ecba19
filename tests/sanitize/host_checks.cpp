// Host-side checks of libtsvd_rbk under AddressSanitizer and
// UndefinedBehaviorSanitizer (built with build_library(sanitize=True)):
// workspace planning over extreme and invalid shapes, the host generator of
// the test tensor, the pseudoinverse cut-off and the argument checks of every
// entry point.  Nothing here reaches the device: every call either plans
// sizes on the host or is rejected before any HIP call.  Exit status 0 and
// the line "host checks ok" mean no sanitizer report and every expectation met.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "tsvd_rbk.h"
#include "tsvd_rbk_diag.h"

static int g_fail = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                     \
    }                                                               \
  } while (0)

int main() {
  EXPECT(tsvd_version() > 0);

  // workspace planning over every operation, precision and a grid of
  // shapes with values at and beyond the documented limits
  const int64_t dims[] = {-1, 0, 1, 7, 64, 4096, 46341, (int64_t)1 << 31, (int64_t)1 << 40, INT64_MAX / 3, INT64_MAX};
  const int64_t small[] = {-1, 0, 1, 5, 110, 1024, 5000, (int64_t)1 << 40, INT64_MAX};
  const int precs[] = {-1, TSVD_PREC_F64, TSVD_PREC_F32, TSVD_PREC_BF16, TSVD_PREC_BF16X3, 99};
  size_t nonzero = 0, calls = 0;
  for (int op = -1; op <= 14; ++op)
    for (int prec : precs)
      for (int64_t n1 : dims)
        for (int64_t n2 : dims)
          for (int64_t n3 : {(int64_t)-1, (int64_t)1, (int64_t)8, (int64_t)4096, (int64_t)4097, INT64_MAX}) {
            const size_t w = tsvd_workspace_bytes(n1, n2, n3, 5, 8, 2, prec, op);
            ++calls;
            if (w) {
              ++nonzero;
              EXPECT(n1 >= 1 && n2 >= 1 && n3 >= 1 && n3 <= 4096);
            }
          }
  for (int64_t k : small)
    for (int64_t b : small)
      for (int64_t q : small)
        for (int op = 0; op <= 12; ++op) {
          (void)tsvd_workspace_bytes(512, 300, 16, k, b, q, TSVD_PREC_F32, op);
          ++calls;
        }
  EXPECT(nonzero > 0);
  EXPECT(tsvd_workspace_bytes(4096, 4096, 64, 100, 110, 3, TSVD_PREC_BF16X3, TSVD_OP_RBK) > 0);
  EXPECT(tsvd_workspace_bytes(4096, 4096, 64, 100, 110, 3, TSVD_PREC_F32, TSVD_OP_APPROX) > 0);

  // the host generator of Omega: deterministic, finite, argument checks
  {
    std::vector<double> a(3 * 5 * 7), b(3 * 5 * 7);
    EXPECT(tsvd_omega(3, 5, 7, 12345, a.data()) == TSVD_OK);
    EXPECT(tsvd_omega(3, 5, 7, 12345, b.data()) == TSVD_OK);
    EXPECT(memcmp(a.data(), b.data(), a.size() * sizeof(double)) == 0);
    bool finite = true;
    for (double v : a) finite = finite && isfinite(v);
    EXPECT(finite);
    EXPECT(tsvd_omega(0, 5, 7, 1, a.data()) == TSVD_EINVAL);
    EXPECT(tsvd_omega(3, 5, 7, 1, nullptr) == TSVD_EINVAL);
    EXPECT(tsvd_omega((int64_t)1 << 40, (int64_t)1 << 40, 1, 1, a.data()) == TSVD_EINVAL);
    EXPECT(tsvd_omega(INT64_MAX, INT64_MAX, INT64_MAX, 1, a.data()) == TSVD_EINVAL);
    EXPECT(strlen(tsvd_last_error()) > 0);
  }

  // pseudoinverse cut-off
  EXPECT(tsvd_tpinv_default_rtol(4096, 256, TSVD_PREC_F32) == 4096 * ldexp(1.0, -23));
  EXPECT(tsvd_tpinv_default_rtol(0, 5, TSVD_PREC_F32) == -1.0);
  EXPECT(tsvd_tpinv_default_rtol(INT64_MAX, INT64_MAX, TSVD_PREC_F64) > 0.0);

  // argument checks of the entry points: null, misaligned and oversized
  // arguments are rejected before anything is enqueued
  void* nul = nullptr;
  void* fake = (void*)(uintptr_t)(1 << 20);
  void* odd = (void*)(uintptr_t)((1 << 20) + 8);
  EXPECT(tsvd_rbk(nul, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, fake, fake, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_rbk(fake, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, odd, fake, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_rbk(fake, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, fake, fake, fake, fake, 16, nul) == TSVD_ENOMEM);
  EXPECT(tsvd_rbk(fake, INT64_MAX, INT64_MAX, 8, 5, 8, 2, 1, TSVD_PREC_F32, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_omega(fake, nul, 64, 64, 8, 5, 8, 2, TSVD_PREC_F32, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_approx(fake, 64, 64, 8, 9, 8, 2, 1, TSVD_PREC_F32, fake, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_power(fake, 64, 64, 8, 5, 8, 5000, 1, TSVD_PREC_F32, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_literal(fake, 64, 64, 8, 5, 8, -1, 1, TSVD_PREC_F32, fake, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_noalloc(nul, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, fake, fake, fake, nul) == TSVD_EINVAL);
  EXPECT(tsvd_tqr(fake, 64, 64, 8, TSVD_PREC_BF16, fake, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_tpinv(fake, 64, 64, 8, NAN, TSVD_PREC_F32, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_tpinv(fake, 64, 64, 8, 1e-15, TSVD_PREC_F32, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_complete(fake, nul, 64, 64, 8, 5, 8, 2, 1, 3, 2, TSVD_PREC_F32, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_proj(fake, 64, 64, 8, 0, 2, 1, TSVD_PREC_F32, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_proj_backward(fake, nul, 64, 64, 8, 8, 2, 1, TSVD_PREC_F32, fake, fake, 1 << 30, nul) == TSVD_EINVAL);
  EXPECT(tsvd_rbk_ritz(fake, 64, 64, 8, 9, 8, 2, 1, TSVD_PREC_F32, fake, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_ritz(fake, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, nul, fake, fake, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_ritz_omega(fake, nul, 64, 64, 8, 5, 8, 2, TSVD_PREC_F32, fake, fake, fake, fake, fake, 1 << 30,
                             nul) == TSVD_EINVAL);
  EXPECT(tsvd_rbk_approx_backward(fake, nul, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_approx_backward(fake, fake, 64, 64, 8, 0, 8, 2, 1, TSVD_PREC_F32, fake, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_rbk_approx_backward(fake, fake, 64, 64, 8, 5, 8, 2, 1, TSVD_PREC_F32, fake, fake, 16, nul) ==
         TSVD_ENOMEM);
  EXPECT(tsvd_rbk_approx_backward_omega(fake, nul, fake, 64, 64, 8, 5, 8, 2, TSVD_PREC_F32, fake, fake, 1 << 30,
                                        nul) == TSVD_EINVAL);
  EXPECT(tsvd_workspace_bytes(4096, 4096, 64, 100, 110, 3, TSVD_PREC_F32, TSVD_OP_APPROX_BWD) >
         tsvd_workspace_bytes(4096, 4096, 64, 100, 110, 3, TSVD_PREC_F32, TSVD_OP_PROJ_BWD));
  EXPECT(tsvd_workspace_bytes(64, 64, 8, 5, 8, 2, TSVD_PREC_F32, 13) == 0);
  EXPECT(tsvd_read_info(nul, nullptr, nul) == TSVD_EINVAL);
  EXPECT(strlen(tsvd_last_error()) > 0);

  // diagnostic entry points: sizes at and beyond their limits
  for (int64_t r : dims)
    for (int64_t c : dims)
      for (int mode = -1; mode <= 4; ++mode) {
        const size_t w = tsvd_diag_kgemm_ws_bytes(1, r, c, 110, 33, mode, 1);
        if (w) EXPECT(r >= 1 && c >= 1 && mode >= 0 && mode <= 3);
        ++calls;
      }
  EXPECT(tsvd_diag_kgemm(fake, 0, fake, fake, INT64_MAX, INT64_MAX, 110, 33, 2, 1, fake, 1 << 30, nul) ==
         TSVD_EINVAL);
  EXPECT(tsvd_diag_split_bf16x3(fake, fake, INT64_MAX, nul) == TSVD_EINVAL);
  EXPECT(tsvd_diag_heig_ws_bytes(2000, 10, 4) == 0);
  EXPECT(tsvd_diag_omega(fake, ((int64_t)1 << 40) + 1, 1, 0, nul) == TSVD_EINVAL);

  printf("%zu planning calls\n", calls);
  if (g_fail) {
    printf("%d expectations failed\n", g_fail);
    return 1;
  }
  printf("host checks ok\n");
  return 0;
}
