// Test infrastructure: the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (sanitizers on the host pass only).  Runs on a
// machine without a GPU: argument validation of every entry point, the
// launch-shape table and its queries, the error strings, and one call with
// valid arguments that must fail cleanly at device set-up.  Exit status 0:
// every call returned what it should; the sanitizers abort on any error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "pn.h"

#define EXPECT(cond)                                                          \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #cond); \
      return 1;                                                               \
    }                                                                         \
  } while (0)

int main() {
  const int kInval = PN_EINVAL;
  // aligned, never dereferenced: validation fails before any use
  double* d = reinterpret_cast<double*>(static_cast<uintptr_t>(4096));
  double* mis = reinterpret_cast<double*>(static_cast<uintptr_t>(4097));
  const double nan = std::nan(""), inf = INFINITY;

  EXPECT(pn_potential_accel(d, d, d, 1, 1.0, 30.0, 0.0, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(d, d, d, 16, 0.0, 30.0, 0.0, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(d, d, d, 16, 1.0, -1.0, 0.0, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(d, d, d, 16, 1.0, nan, 0.0, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(d, d, d, 16, 1.0, 30.0, -1e-3, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(d, d, d, 16, 1.0, 30.0, inf, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(nullptr, d, d, 16, 1.0, 30.0, 0.0, d, d, nullptr, 0) == kInval);
  EXPECT(pn_potential_accel(mis, d, d, 16, 1.0, 30.0, 0.0, d, d, nullptr, 0) == kInval);
  EXPECT(pn_correction(d, nullptr, d, 16, 1.0, 30.0, 0.0, d, d, d, nullptr, 0) == kInval);
  EXPECT(pn_step(d, d, d, 16, 1.0, 30.0, 0.0, nan, 1, 0, nullptr, 0) == kInval);
  EXPECT(pn_step(d, d, d, 16, 1.0, 30.0, 0.0, 1e-4, -1, 0, nullptr, 0) == kInval);
  EXPECT(pn_step(d, d, d, 16, 1.0, 30.0, 0.0, 1e-4, 1, 7, nullptr, 0) == kInval);
  EXPECT(pn_accel(d, d, d, 16, 1.0, 30.0, 0.0, 9, d, d, d, nullptr, 0) == kInval);
  EXPECT(pn_accel_eih(d, nullptr, d, 16, 1.0, 30.0, 0.0, 0, d, d, d, nullptr, 0) == kInval);
  EXPECT(pn_diagnostics(d, d, d, 16, 1.0, 30.0, 0.0, nullptr, nullptr, 0) == kInval);
  EXPECT(pn_encounters(d, d, d, 2, 1.0, 30.0, 0.1, d, nullptr, 0) == kInval);
  EXPECT(pn_encounters(d, d, d, 16, 1.0, 30.0, -0.1, d, nullptr, 0) == kInval);
  EXPECT(pn_jerk(d, d, d, 16, 1.0, 30.0, 0.0, nullptr, d, nullptr, 0) == kInval);
  EXPECT(pn_step_hermite(d, d, d, 16, 1.0, 30.0, 0.0, 0.0, 1, nullptr, 0) == kInval);
  EXPECT(pn_step_hermite(d, d, d, 1, 1.0, 30.0, 0.0, 1e-3, 1, nullptr, 0) == kInval);
  EXPECT(pn_last_timing(nullptr) == kInval);

  // batched: a one-body system, offsets not starting at 0, no systems
  int64_t off_bad[3] = {0, 10, 11}, off_start[3] = {1, 10, 20};
  double p2[2] = {1.0, 1.0};
  EXPECT(pn_step_batched(2, off_bad, p2, p2, p2, d, d, d, 1e-4, 1, 0, nullptr, 0) == kInval);
  EXPECT(pn_step_batched(2, off_start, p2, p2, p2, d, d, d, 1e-4, 1, 0, nullptr, 0) == kInval);
  EXPECT(pn_step_batched(0, off_start, p2, p2, p2, d, d, d, 1e-4, 1, 0, nullptr, 0) == kInval);

  // launch-shape table: install, query across sizes, clear
  EXPECT(pn_set_shape(0, 10, 5, 1, 4, 0) == kInval);
  EXPECT(pn_set_shape(0, 2, 5, 3, 4, 0) == kInval);
  EXPECT(pn_set_shape(0, 2, 1000, 1, 4, 8) == PN_OK);
  EXPECT(pn_set_shape(1, 1001, 1 << 20, 2, 1, 0) == PN_OK);
  int out4[4];
  for (int64_t N = 2; N <= (int64_t(1) << 28); N = N * 3 + 1) {
    for (int prec = 0; prec < 2; ++prec) {
      EXPECT(pn_query_shape(prec, N, out4) == PN_OK);
      EXPECT(out4[0] >= 1 && out4[1] >= 1 && out4[2] >= 1 && out4[3] >= 1);
    }
  }
  EXPECT(pn_query_shape(0, 1, out4) == kInval);
  EXPECT(pn_query_shape(7, 100, out4) == kInval);
  EXPECT(pn_query_shape(0, 100, nullptr) == kInval);
  EXPECT(pn_set_shape(-1, 0, 0, 0, 0, 0) == PN_OK);

  for (int code : {0, -1, -2, -3, -4, 99}) EXPECT(pn_strerror(code) != nullptr);

  // valid arguments (host arrays): must fail cleanly at device set-up, not crash
  const int64_t N = 64;
  double* pos = static_cast<double*>(std::aligned_alloc(256, 3 * N * sizeof(double)));
  double* vel = static_cast<double*>(std::aligned_alloc(256, 3 * N * sizeof(double)));
  double* mass = static_cast<double*>(std::aligned_alloc(256, N * sizeof(double)));
  double* acc = static_cast<double*>(std::aligned_alloc(256, 3 * N * sizeof(double)));
  for (int64_t k = 0; k < 3 * N; ++k) pos[k] = vel[k] = 0.01 * (double)k;
  for (int64_t k = 0; k < N; ++k) mass[k] = 1.0;
  EXPECT(pn_accel(pos, vel, mass, N, 1.0, 30.0, 1e-4, PN_FP64, acc, nullptr, nullptr, nullptr,
                  0) != PN_OK);
  std::free(pos), std::free(vel), std::free(mass), std::free(acc);
  (void)pn_release();
  std::printf("sanitized host driver: all calls ok\n");
  return 0;
}
