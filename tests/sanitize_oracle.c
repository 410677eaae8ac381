/* Test infrastructure: drives every entry point of the CPU oracle
 * (oracle/pnref.c) on small seeded systems and on invalid arguments, so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer checks the
 * oracle's memory accesses and arithmetic on every path.  Every array is
 * allocated at its exact size.  Exit status 0: all calls returned what they
 * should and every result is finite; the sanitizers abort on any error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef int64_t idx_t;

int pnref_newton(const double *, const double *, idx_t, double, double, double *, double *);
int pnref_correction(const double *, const double *, const double *, idx_t, double, double,
                     double, const double *, const double *, double *);
int pnref_accel(const double *, const double *, const double *, idx_t, double, double, double,
                double *, double *, double *);
int pnref_accel_rows(const double *, const double *, const double *, idx_t, double, double,
                     double, const idx_t *, idx_t, double *, double *, double *);
int pnref_literal(const double *, const double *, const double *, idx_t, double, double, double,
                  double *);
int pnref_eih(const double *, const double *, const double *, idx_t, double, double, double,
              double *, double *);
int pnref_eih2(const double *, const double *, const double *, idx_t, double, double, double,
               double *, double *, double *);
int pnref_twobody(const double *, const double *, double, double, double, double, double *,
                  double *);
int pnref_step(double *, double *, const double *, idx_t, double, double, double, double, idx_t);
int pnref_jerk(const double *, const double *, const double *, idx_t, double, double, double,
               double, double *, double *);
int pnref_hermite(double *, double *, const double *, idx_t, double, double, double, double,
                  idx_t, double);
int pnref_diagnostics(const double *, const double *, const double *, idx_t, double, double,
                      double, double *);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) * 0x1.0p-53;
}

static double *alloc(idx_t n) {
  double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

static int all_finite(const double *a, idx_t n) {
  for (idx_t k = 0; k < n; ++k)
    if (!isfinite(a[k])) return 0;
  return 1;
}

#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #cond); \
      return 1;                                                        \
    }                                                                  \
  } while (0)

/* Body 0 a massive object of mass 0.1 at rest at the origin, N - 1 stars of
 * total mass 1 in the unit cube around it, velocities recentred so that the
 * total momentum vanishes. */
static void make_system(idx_t N, double *pos, double *vel, double *mass) {
  double p[3] = {0.0, 0.0, 0.0};
  mass[0] = 0.1;
  for (int c = 0; c < 3; ++c) pos[c] = vel[c] = 0.0;
  for (idx_t s = 1; s < N; ++s) {
    mass[s] = 1.0 / (double)(N - 1);
    for (int c = 0; c < 3; ++c) {
      pos[3 * s + c] = urand() - 0.5;
      vel[3 * s + c] = 0.3 * (urand() - 0.5);
      p[c] += mass[s] * vel[3 * s + c];
    }
  }
  for (int c = 0; c < 3; ++c) vel[c] = -p[c] / mass[0];
}

static int run(idx_t N, double c, double eps) {
  const double G = 1.0;
  double *pos = alloc(3 * N), *vel = alloc(3 * N), *mass = alloc(N);
  double *aN = alloc(3 * N), *phi = alloc(N), *a1 = alloc(3 * N), *lit = alloc(3 * N);
  double *jerk = alloc(3 * N), *out8 = alloc(8);
  const idx_t nrows = N > 1 ? 2 : 1;
  idx_t *rows = (idx_t *)malloc(sizeof(idx_t) * (size_t)nrows);
  double *rN = alloc(3 * nrows), *rphi = alloc(nrows), *r1 = alloc(3 * nrows);
  make_system(N, pos, vel, mass);
  rows[0] = 0;
  if (nrows > 1) rows[1] = N - 1;

  EXPECT(pnref_newton(pos, mass, N, G, eps, aN, phi) == 0);
  EXPECT(all_finite(aN, 3 * N) && all_finite(phi, N));
  EXPECT(pnref_correction(pos, vel, mass, N, G, c, eps, phi, aN, a1) == 0);
  EXPECT(all_finite(a1, 3 * N));
  EXPECT(pnref_accel(pos, vel, mass, N, G, c, eps, aN, phi, a1) == 0);
  EXPECT(all_finite(aN, 3 * N) && all_finite(phi, N) && all_finite(a1, 3 * N));
  EXPECT(pnref_accel_rows(pos, vel, mass, N, G, c, eps, rows, nrows, rN, rphi, r1) == 0);
  EXPECT(all_finite(rN, 3 * nrows) && all_finite(r1, 3 * nrows));
  EXPECT(pnref_literal(pos, vel, mass, N, G, c, eps, lit) == 0);
  EXPECT(all_finite(lit, 3 * N));
  EXPECT(pnref_eih(pos, vel, mass, N, G, c, eps, aN, a1) == 0);
  EXPECT(all_finite(aN, 3 * N) && all_finite(a1, 3 * N));
  EXPECT(pnref_eih2(pos, vel, mass, N, G, c, eps, aN, phi, a1) == 0);
  EXPECT(all_finite(aN, 3 * N) && all_finite(a1, 3 * N));
  EXPECT(pnref_diagnostics(pos, vel, mass, N, G, c, eps, out8) == 0);
  EXPECT(all_finite(out8, 8));
  EXPECT(pnref_jerk(pos, vel, mass, N, G, c, eps, 1e-4, aN, jerk) == 0);
  EXPECT(all_finite(aN, 3 * N) && all_finite(jerk, 3 * N));
  EXPECT(pnref_step(pos, vel, mass, N, G, c, eps, 1e-4, 2) == 0);
  EXPECT(pnref_hermite(pos, vel, mass, N, G, c, eps, 1e-4, 2, 1e-4) == 0);
  EXPECT(all_finite(pos, 3 * N) && all_finite(vel, 3 * N));

  /* invalid arguments: an error code, no access past the arrays */
  EXPECT(pnref_accel(pos, vel, mass, 1, G, c, eps, aN, phi, a1) < 0);
  EXPECT(pnref_accel(NULL, vel, mass, N, G, c, eps, aN, phi, a1) < 0);
  EXPECT(pnref_accel(pos, vel, mass, N, G, 0.0, eps, aN, phi, a1) < 0);
  EXPECT(pnref_accel(pos, vel, mass, N, G, c, -1.0, aN, phi, a1) < 0);
  EXPECT(pnref_step(pos, vel, mass, N, G, c, eps, NAN, 1) < 0);
  rows[0] = N;
  EXPECT(pnref_accel_rows(pos, vel, mass, N, G, c, eps, rows, nrows, rN, rphi, r1) < 0);

  free(pos), free(vel), free(mass), free(aN), free(phi), free(a1), free(lit), free(jerk);
  free(out8), free(rows), free(rN), free(rphi), free(r1);
  return 0;
}

int main(void) {
  const idx_t sizes[] = {2, 3, 7, 33};
  const double cs[] = {30.0, INFINITY, 3.0};
  const double epss[] = {1e-4, 0.0, 1e-2};
  for (size_t a = 0; a < sizeof sizes / sizeof sizes[0]; ++a)
    for (size_t b = 0; b < sizeof cs / sizeof cs[0]; ++b)
      if (run(sizes[a], cs[b], epss[b])) {
        fprintf(stderr, "case N=%lld c=%g eps=%g\n", (long long)sizes[a], cs[b], epss[b]);
        return 1;
      }
  double x[3] = {0.3, -0.2, 0.1}, v[3] = {0.1, 0.2, -0.1}, an[3], a1[3];
  EXPECT(pnref_twobody(x, v, 0.1, 1e-3, 1.0, 30.0, an, a1) == 0);
  EXPECT(all_finite(an, 3) && all_finite(a1, 3));
  EXPECT(pnref_twobody(x, v, -1.0, 1e-3, 1.0, 30.0, an, a1) < 0);
  printf("sanitized oracle driver: all calls ok\n");
  return 0;
}
