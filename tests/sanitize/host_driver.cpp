// Host-only driver of libptk for the sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code; no device code is built, and
// nothing here launches a kernel).  Exercises the code paths that run without
// a GPU: the self-test of the internal checks, the coefficient derivation for
// every kernel the library supports, argument validation, and context
// creation on a machine that may have no device.  Exit status 0 = all checks
// passed; a sanitizer finding aborts the run.
#include <cmath>
#include <cstdio>

#include "ptk.h"

static int failures = 0;
static void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

int main() {
  check(ptk_selftest() == PTK_OK, "self-test");
  // coefficient tables: partition of unity, sum_j beta_j(t) = 1 for every t,
  // i.e. the constant terms add up to 1 and every other power to 0
  const int kernels[][3] = {{PTK_LAGRANGE, 4, 0}, {PTK_LAGRANGE, 6, 0}, {PTK_LAGRANGE, 8, 0},
                            {PTK_SPLINE, 4, 1},   {PTK_SPLINE, 6, 1},   {PTK_SPLINE, 6, 2},
                            {PTK_SPLINE, 8, 1},   {PTK_SPLINE, 8, 2},   {PTK_SPLINE, 8, 3}};
  for (const auto& k : kernels) {
    ptk_kernel kk{k[0], k[1], k[2]};
    double val[64], der[64];
    check(ptk_kernel_table(&kk, val, der) == PTK_OK, "kernel table");
    for (int p = 0; p < kk.I; ++p) {
      double sum = 0.0;
      for (int j = 0; j < kk.I; ++j) sum += val[j * kk.I + p];
      check(std::fabs(sum - (p == 0 ? 1.0 : 0.0)) < 1e-12, "partition of unity");
    }
  }
  // argument validation
  ptk_kernel odd{PTK_SPLINE, 5, 1}, rough{PTK_SPLINE, 6, 3}, fam{7, 6, 1};
  double v[64];
  check(ptk_kernel_table(nullptr, v, nullptr) == PTK_EINVAL, "NULL kernel");
  check(ptk_kernel_table(&odd, v, nullptr) == PTK_EUNSUPPORTED, "odd I");
  check(ptk_kernel_table(&rough, v, nullptr) == PTK_EINVAL, "m too large");
  check(ptk_kernel_table(&fam, v, nullptr) == PTK_EINVAL, "bad family");
  check(ptk_create(nullptr, 0) == PTK_EINVAL, "create NULL");
  ptk_ctx* c = nullptr;
  check(ptk_create(&c, -1) == PTK_EINVAL && c == nullptr, "create bad device");
  check(ptk_set_field(nullptr, nullptr, 32, 0, 0, nullptr, nullptr) == PTK_EINVAL, "set_field NULL");
  check(ptk_interpolate(nullptr, nullptr, 0, nullptr, 0, nullptr) == PTK_EINVAL, "interpolate NULL");
  check(ptk_advance_particles(nullptr, nullptr, 0, nullptr, nullptr, PTK_HEUN, 1e-3, 1, nullptr, nullptr) ==
            PTK_EINVAL,
        "advance NULL");
  check(ptk_particles_advance(nullptr, PTK_HEUN, 1e-3, 1, nullptr, nullptr) == PTK_EINVAL, "particles NULL");
  check(ptk_particles_set_inertia(nullptr, nullptr, nullptr, nullptr, 0, 0.1, nullptr) == PTK_EINVAL,
        "set_inertia NULL");
  check(ptk_particles_get_inertia(nullptr, nullptr, nullptr, nullptr, nullptr) == PTK_EINVAL, "get_inertia NULL");
  ptk_destroy(nullptr);
  if (failures) return 1;
  std::printf("host driver: all checks passed\n");
  return 0;
}
