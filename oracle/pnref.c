/*
 * pnref.c -- plain FP64 CPU oracle for the limited first-order
 * post-Newtonian (1PN) N-body equations of motion of
 *   T. Tatekawa, "Accelerating N-body simulation of self-gravitating systems
 *   with limited first-order post-Newtonian approximation" (arXiv:1801.07986).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or constant with the HIP library.
 *
 * Conventions (paper Sec. 2):
 *   - array index 0 is the massive object the paper labels #1 (mass M);
 *     indices 1..N-1 are the low-mass stars i, j, k.  Sums over j, k run over
 *     stars only.
 *   - pos, vel: [N][3] row-major doubles; mass: [N].
 *   - x_ab = x_a - x_b.  The paper's text defines x_1j = x_j - x_1, which would
 *     make Eq. (1) repulsive; the signs printed in Eqs. (1) and (4) are those of
 *     attraction with x_ab = x_a - x_b, which is the reading used throughout.
 *   - Plummer softening (Sec. 4, Eq. (10)): every pair distance r_ab becomes
 *     R_ab = sqrt(r_ab^2 + eps^2), and n_ab = x_ab / R_ab.
 *   - lambda = 1/c^2; c = +inf gives lambda = 0 (pure Newtonian).
 *
 * Equation numbers count the displayed equations of the paper in order:
 *   (1) BH equation of motion, (2) [a_1]_BH, (3) [a_1]_Cross, (4) star equation
 *   of motion, (5) [a_i]_BH, (6) [a_i]_Cross, (7) 1PN energy, (8) 1PN momentum,
 *   (9) sum of star masses, (10) Plummer softening.
 *
 * Compiled with -O2 -ffp-contract=off: every operation is a plain IEEE double
 * operation in source order.  OpenMP (when enabled) only distributes the outer
 * per-body loop; each body's sums run sequentially in index order.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PNREF_OK 0
#define PNREF_EINVAL (-1)
#define PNREF_ENOMEM (-4)

typedef int64_t idx_t;

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* d = xa - xb; returns the softened distance R = sqrt(|d|^2 + eps^2). */
static double sep(const double *xa, const double *xb, double eps2, double *d) {
  d[0] = xa[0] - xb[0];
  d[1] = xa[1] - xb[1];
  d[2] = xa[2] - xb[2];
  return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2);
}

static double lambda_of(double c) { return isinf(c) ? 0.0 : 1.0 / (c * c); }

static int check_common(const double *pos, const double *mass, idx_t N, double G,
                        double eps) {
  if (!pos || !mass || N < 2) return PNREF_EINVAL;
  if (!(G > 0.0) || !isfinite(G)) return PNREF_EINVAL;
  if (!(eps >= 0.0) || !isfinite(eps)) return PNREF_EINVAL;
  if (!(mass[0] > 0.0)) return PNREF_EINVAL;
  return PNREF_OK;
}

static int check_c(double c) {
  if (isnan(c) || !(c > 0.0)) return PNREF_EINVAL;
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* Newtonian acceleration and potential: the first terms of Eqs. (1)    */
/* and (4) (Eq. (4) printed with r_ij in place of r_ij^3; the cube is   */
/* what dimensions and the Newtonian limit require), softened by Eq.   */
/* (10).  phi_a = -sum_{b != a} G m_b / R_ab.                           */
/* ------------------------------------------------------------------ */
int pnref_newton(const double *pos, const double *mass, idx_t N, double G,
                 double eps, double *acc, double *phi) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc || !acc || !phi) return rc ? rc : PNREF_EINVAL;
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (idx_t a = 0; a < N; ++a) {
    double ax = 0.0, ay = 0.0, az = 0.0, p = 0.0, d[3];
    for (idx_t b = 0; b < N; ++b) {
      if (b == a) continue;
      double R = sep(pos + 3 * a, pos + 3 * b, eps2, d);
      double R3 = R * R * R;
      ax -= G * mass[b] * d[0] / R3;
      ay -= G * mass[b] * d[1] / R3;
      az -= G * mass[b] * d[2] / R3;
      p -= G * mass[b] / R;
    }
    acc[3 * a + 0] = ax;
    acc[3 * a + 1] = ay;
    acc[3 * a + 2] = az;
    phi[a] = p;
  }
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* Limited-1PN correction, all N bodies (Eqs. (1)-(6)).                 */
/*                                                                      */
/* The paper's Eqs. (2), (3), (5), (6) are the Einstein-Infeld-Hoffmann */
/* (EIH) 1PN equations it cites, kept to first order in the star masses */
/* relative to each equation's leading term.  Written in EIH layout,    */
/* with V_a = -phi_a the Newtonian potential magnitude at body a and    */
/* a^N_a the Newtonian acceleration of a, the terms kept are:           */
/*                                                                      */
/* star i, partner = massive object (index 0):                          */
/*   (G M/R^2) n_i0 [ -v_i^2 + 4 v_i.w + 4 V_i + V_0 + 1/2 x_i0.a^N_0 ] */
/*   + (G M/R^2) [ (n_i0.4v_i)(v_i - w) - 3 (n_i0.w) v_i ]              */
/*   + 7/2 (G M/R) a^N_0                                                */
/*   This holds Eq. (5) and the terms of Eq. (6) with factor G^2 m M    */
/*   carrying 1/r_i1 or 1/r_j1 (5 G^2 m_i M x_i1/r^4, the first j-sum,  */
/*   the 1/r_i1 half of the 7/2 sum) and its velocity terms (second and */
/*   sixth lines of Eq. (6)).                                           */
/* star i, partner = star j:                                            */
/*   (G m_j/R^2) n_ij [ -v_i^2 - 2 v_j^2 + 4 v_i.v_j + 3/2 (n_ij.v_j)^2 */
/*                      + 4 u_i + u_j + 1/2 x_ij.(-b_j) ]               */
/*   + (G m_j/R^2) [ n_ij.(4 v_i - 3 v_j) ] (v_i - v_j)                 */
/*   + 7/2 (G m_j/R_ij) (-b_j)                                          */
/*   with u_s = G M / R_s0 and -b_s = -G M x_s0 / R_s0^3 the massive    */
/*   object's potential and pull at star s.  This holds the second j-sum */
/*   of Eq. (6), the 1/r_ij half of its 7/2 sum and its last two lines. */
/* massive object (index 0), partner = star s:                          */
/*   (G m_s/R^2) n_0s [ -2 v_s^2 + 4 w.v_s + 3/2 (n_0s.v_s)^2 + 4 V_0   */
/*                      + V_s + 1/2 x_0s.a^N_s ]                        */
/*   + (G m_s/R^2) [ 3 (n_0s.v_s) v_s - 3 (n_0s.v_s) w - 4 (n_0s.w) v_s ]*/
/*   + 7/2 (G m_s/R_0s) a^N_s                                           */
/*   This is Eq. (2) plus Eq. (3): the 4 G^2 m_j^2 and 4/r_1k terms come */
/*   from 4 V_0, the 5/(4 r_jk) and r^2/(4 r_jk^3) terms from V_s and    */
/*   1/2 x_0s.a^N_s, the -7/2 sum from 7/2 (G m_s/R) a^N_s, and the last */
/*   line (with 1/M) from the w terms.                                  */
/*                                                                      */
/* The massive object's velocity never enters: Eqs. (2)-(6) contain no   */
/* v_1.  Its linear occurrences in EIH appear instead through           */
/* w = -P/M, P = sum_s m_s v_s (the velocity the massive object has in  */
/* the frame of zero Newtonian momentum); that substitution is exactly   */
/* the second line of Eq. (6), its sixth line and the last line of      */
/* Eq. (3).  Terms quadratic in w are of second order and dropped.      */
/*                                                                      */
/* Inputs phi and acc_newton are the Newtonian potential and            */
/* acceleration of all N bodies (pnref_newton).  Output acc_1pn is      */
/* lambda times the bracketed 1PN part, for all N bodies.               */
/* ------------------------------------------------------------------ */
int pnref_correction(const double *pos, const double *vel, const double *mass,
                     idx_t N, double G, double c, double eps, const double *phi,
                     const double *acc_newton, double *acc_1pn) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !phi || !acc_newton || !acc_1pn) return PNREF_EINVAL;
  const double lam = lambda_of(c);
  const double eps2 = eps * eps;
  const double M = mass[0];
  const double *x0 = pos;
  double *u = (double *)malloc(sizeof(double) * N);
  double *b = (double *)malloc(sizeof(double) * 3 * N);
  if (!u || !b) {
    free(u);
    free(b);
    return PNREF_ENOMEM;
  }
  /* the massive object's potential u_s and pull -b_s at each star */
  u[0] = 0.0;
  b[0] = b[1] = b[2] = 0.0;
  for (idx_t s = 1; s < N; ++s) {
    double d[3];
    double R = sep(pos + 3 * s, x0, eps2, d); /* x_s0 */
    u[s] = G * M / R;
    b[3 * s + 0] = G * M * d[0] / (R * R * R);
    b[3 * s + 1] = G * M * d[1] / (R * R * R);
    b[3 * s + 2] = G * M * d[2] / (R * R * R);
  }
  /* Newtonian star momentum P and w = -P/M */
  double P[3] = {0.0, 0.0, 0.0};
  for (idx_t s = 1; s < N; ++s) {
    P[0] += mass[s] * vel[3 * s + 0];
    P[1] += mass[s] * vel[3 * s + 1];
    P[2] += mass[s] * vel[3 * s + 2];
  }
  const double w[3] = {-P[0] / M, -P[1] / M, -P[2] / M};
  const double V0 = -phi[0];
  const double *aN0 = acc_newton;

  /* stars */
#pragma omp parallel for schedule(static)
  for (idx_t i = 1; i < N; ++i) {
    const double *xi = pos + 3 * i, *vi = vel + 3 * i;
    const double Vi = -phi[i];
    const double vi2 = dot3(vi, vi);
    double out[3] = {0.0, 0.0, 0.0};

    /* partner: massive object */
    {
      double d[3], n[3];
      double R = sep(xi, x0, eps2, d); /* x_i0 */
      n[0] = d[0] / R;
      n[1] = d[1] / R;
      n[2] = d[2] / R;
      double k = G * M / (R * R);
      double br = -vi2 + 4.0 * dot3(vi, w) + 4.0 * Vi + V0 + 0.5 * dot3(d, aN0);
      double n4v = 4.0 * dot3(n, vi);
      double nw = dot3(n, w);
      for (int q = 0; q < 3; ++q)
        out[q] += k * (br * n[q] + n4v * (vi[q] - w[q]) - 3.0 * nw * vi[q]) +
                  3.5 * (G * M / R) * aN0[q];
    }
    /* partners: stars j != i */
    for (idx_t j = 1; j < N; ++j) {
      if (j == i) continue;
      const double *xj = pos + 3 * j, *vj = vel + 3 * j, *bj = b + 3 * j;
      double d[3], n[3];
      double R = sep(xi, xj, eps2, d); /* x_ij */
      n[0] = d[0] / R;
      n[1] = d[1] / R;
      n[2] = d[2] / R;
      double k = G * mass[j] / (R * R);
      double nvj = dot3(n, vj);
      double S = -vi2 - 2.0 * dot3(vj, vj) + 4.0 * dot3(vi, vj) + 1.5 * nvj * nvj +
                 4.0 * u[i] + u[j] - 0.5 * dot3(d, bj);
      double D = 4.0 * dot3(n, vi) - 3.0 * nvj;
      for (int q = 0; q < 3; ++q)
        out[q] += k * (S * n[q] + D * (vi[q] - vj[q])) - 3.5 * (G * mass[j] / R) * bj[q];
    }
    acc_1pn[3 * i + 0] = lam * out[0];
    acc_1pn[3 * i + 1] = lam * out[1];
    acc_1pn[3 * i + 2] = lam * out[2];
  }

  /* massive object */
  {
    double out[3] = {0.0, 0.0, 0.0};
    for (idx_t s = 1; s < N; ++s) {
      const double *vs = vel + 3 * s, *aNs = acc_newton + 3 * s;
      double d[3], n[3];
      double R = sep(x0, pos + 3 * s, eps2, d); /* x_0s */
      n[0] = d[0] / R;
      n[1] = d[1] / R;
      n[2] = d[2] / R;
      double k = G * mass[s] / (R * R);
      double nvs = dot3(n, vs);
      double Vs = -phi[s];
      double br = -2.0 * dot3(vs, vs) + 4.0 * dot3(w, vs) + 1.5 * nvs * nvs + 4.0 * V0 +
                  Vs + 0.5 * dot3(d, aNs);
      double nw = dot3(n, w);
      for (int q = 0; q < 3; ++q)
        out[q] += k * (br * n[q] + 3.0 * nvs * vs[q] - 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +
                  3.5 * (G * mass[s] / R) * aNs[q];
    }
    acc_1pn[0] = lam * out[0];
    acc_1pn[1] = lam * out[1];
    acc_1pn[2] = lam * out[2];
  }
  free(u);
  free(b);
  return PNREF_OK;
}

/* Full evaluation: Newtonian acceleration, potential and 1PN part. */
int pnref_accel(const double *pos, const double *vel, const double *mass, idx_t N,
                double G, double c, double eps, double *acc_newton, double *phi,
                double *acc_1pn) {
  int rc = pnref_newton(pos, mass, N, G, eps, acc_newton, phi);
  if (rc) return rc;
  return pnref_correction(pos, vel, mass, N, G, c, eps, phi, acc_newton, acc_1pn);
}

/* ------------------------------------------------------------------ */
/* Same definition, evaluated for a subset of bodies only (for sizes   */
/* where the whole set is too slow on the CPU).  rows: nrows indices   */
/* into 0..N-1.  Outputs are [nrows] / [nrows][3] in the order given.  */
/* If row 0 (the massive object) is requested, every star's potential  */
/* and Newtonian acceleration is needed and an O(N^2) Newtonian pass   */
/* runs first; star rows alone cost O(N) each.                          */
/* ------------------------------------------------------------------ */
int pnref_accel_rows(const double *pos, const double *vel, const double *mass,
                     idx_t N, double G, double c, double eps, const idx_t *rows,
                     idx_t nrows, double *acc_newton, double *phi, double *acc_1pn) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !rows || nrows < 0 || !acc_newton || !phi || !acc_1pn)
    return PNREF_EINVAL;
  for (idx_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= N) return PNREF_EINVAL;
  const double eps2 = eps * eps;
  int need_bh = 0;
  for (idx_t r = 0; r < nrows; ++r) need_bh |= (rows[r] == 0);

  /* Newtonian potential/acceleration: all bodies if the massive object
     is requested, else only the massive object and the requested rows */
  double *aN = (double *)malloc(sizeof(double) * 3 * N);
  double *ph = (double *)malloc(sizeof(double) * N);
  char *want = (char *)calloc((size_t)N, 1);
  if (!aN || !ph || !want) {
    free(aN);
    free(ph);
    free(want);
    return PNREF_ENOMEM;
  }
  want[0] = 1;
  for (idx_t r = 0; r < nrows; ++r) want[rows[r]] = 1;
  if (need_bh) memset(want, 1, (size_t)N);
#pragma omp parallel for schedule(dynamic, 64)
  for (idx_t a = 0; a < N; ++a) {
    if (!want[a]) continue;
    double ax = 0.0, ay = 0.0, az = 0.0, p = 0.0, d[3];
    for (idx_t b = 0; b < N; ++b) {
      if (b == a) continue;
      double R = sep(pos + 3 * a, pos + 3 * b, eps2, d);
      double R3 = R * R * R;
      ax -= G * mass[b] * d[0] / R3;
      ay -= G * mass[b] * d[1] / R3;
      az -= G * mass[b] * d[2] / R3;
      p -= G * mass[b] / R;
    }
    aN[3 * a + 0] = ax;
    aN[3 * a + 1] = ay;
    aN[3 * a + 2] = az;
    ph[a] = p;
  }

  /* 1PN part: same arithmetic as pnref_correction, per requested row */
  const double lam = lambda_of(c);
  const double M = mass[0];
  const double *x0 = pos;
  double P[3] = {0.0, 0.0, 0.0};
  for (idx_t s = 1; s < N; ++s) {
    P[0] += mass[s] * vel[3 * s + 0];
    P[1] += mass[s] * vel[3 * s + 1];
    P[2] += mass[s] * vel[3 * s + 2];
  }
  const double w[3] = {-P[0] / M, -P[1] / M, -P[2] / M};
  const double V0 = -ph[0];
  const double *aN0 = aN;

#pragma omp parallel for schedule(dynamic, 1)
  for (idx_t r = 0; r < nrows; ++r) {
    idx_t i = rows[r];
    double out[3] = {0.0, 0.0, 0.0};
    if (i == 0) {
      for (idx_t s = 1; s < N; ++s) {
        const double *vs = vel + 3 * s, *aNs = aN + 3 * s;
        double d[3], n[3];
        double R = sep(x0, pos + 3 * s, eps2, d);
        n[0] = d[0] / R;
        n[1] = d[1] / R;
        n[2] = d[2] / R;
        double k = G * mass[s] / (R * R);
        double nvs = dot3(n, vs);
        double Vs = -ph[s];
        double br = -2.0 * dot3(vs, vs) + 4.0 * dot3(w, vs) + 1.5 * nvs * nvs + 4.0 * V0 +
                    Vs + 0.5 * dot3(d, aNs);
        double nw = dot3(n, w);
        for (int q = 0; q < 3; ++q)
          out[q] += k * (br * n[q] + 3.0 * nvs * vs[q] - 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +
                    3.5 * (G * mass[s] / R) * aNs[q];
      }
    } else {
      const double *xi = pos + 3 * i, *vi = vel + 3 * i;
      const double Vi = -ph[i];
      const double vi2 = dot3(vi, vi);
      double d0[3];
      double Ri0 = sep(xi, x0, eps2, d0);
      const double ui = G * M / Ri0;
      {
        double n[3] = {d0[0] / Ri0, d0[1] / Ri0, d0[2] / Ri0};
        double k = G * M / (Ri0 * Ri0);
        double br = -vi2 + 4.0 * dot3(vi, w) + 4.0 * Vi + V0 + 0.5 * dot3(d0, aN0);
        double n4v = 4.0 * dot3(n, vi);
        double nw = dot3(n, w);
        for (int q = 0; q < 3; ++q)
          out[q] += k * (br * n[q] + n4v * (vi[q] - w[q]) - 3.0 * nw * vi[q]) +
                    3.5 * (G * M / Ri0) * aN0[q];
      }
      for (idx_t j = 1; j < N; ++j) {
        if (j == i) continue;
        const double *xj = pos + 3 * j, *vj = vel + 3 * j;
        double dj0[3];
        double Rj0 = sep(xj, x0, eps2, dj0);
        double uj = G * M / Rj0;
        double bj[3] = {G * M * dj0[0] / (Rj0 * Rj0 * Rj0), G * M * dj0[1] / (Rj0 * Rj0 * Rj0),
                        G * M * dj0[2] / (Rj0 * Rj0 * Rj0)};
        double d[3], n[3];
        double R = sep(xi, xj, eps2, d);
        n[0] = d[0] / R;
        n[1] = d[1] / R;
        n[2] = d[2] / R;
        double k = G * mass[j] / (R * R);
        double nvj = dot3(n, vj);
        double S = -vi2 - 2.0 * dot3(vj, vj) + 4.0 * dot3(vi, vj) + 1.5 * nvj * nvj +
                   4.0 * ui + uj - 0.5 * dot3(d, bj);
        double D = 4.0 * dot3(n, vi) - 3.0 * nvj;
        for (int q = 0; q < 3; ++q)
          out[q] += k * (S * n[q] + D * (vi[q] - vj[q])) - 3.5 * (G * mass[j] / R) * bj[q];
      }
    }
    acc_1pn[3 * r + 0] = lam * out[0];
    acc_1pn[3 * r + 1] = lam * out[1];
    acc_1pn[3 * r + 2] = lam * out[2];
    acc_newton[3 * r + 0] = aN[3 * i + 0];
    acc_newton[3 * r + 1] = aN[3 * i + 1];
    acc_newton[3 * r + 2] = aN[3 * i + 2];
    phi[r] = ph[i];
  }
  free(aN);
  free(ph);
  free(want);
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* Eqs. (1)-(6) transcribed term by term as printed, with the readings */
/* x_ab = x_a - x_b, v_ij = v_i - v_j, r_ij^3 in Eq. (4), v_i for the   */
/* printed v_a of Eq. (5), (v_j.n_1j)^2 squared in Eq. (2), j != k in   */
/* the G^2 double sums of Eq. (3) and k = j included in its last line.  */
/* The double sums over j, k of Eq. (3) are evaluated as written        */
/* (O(N^2) for one body).  Distances use R everywhere; this form is     */
/* compared with pnref_accel at eps = 0, where the two are the same     */
/* equations.  Writes the total acceleration (Newtonian + lambda*1PN).  */
/* ------------------------------------------------------------------ */
int pnref_literal(const double *pos, const double *vel, const double *mass, idx_t N,
                  double G, double c, double eps, double *acc) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !acc) return PNREF_EINVAL;
  const double lam = lambda_of(c);
  const double eps2 = eps * eps;
  const double M = mass[0];
  const double *x1 = pos; /* the paper's body #1 */

  /* ---- Eq. (1): body #1 ---- */
  {
    double newt[3] = {0, 0, 0}, aBH[3] = {0, 0, 0}, aCr[3] = {0, 0, 0};
    for (idx_t j = 1; j < N; ++j) {
      const double *vj = vel + 3 * j;
      double x1j[3];
      double r1j = sep(x1, pos + 3 * j, eps2, x1j);
      double n1j[3] = {x1j[0] / r1j, x1j[1] / r1j, x1j[2] / r1j};
      double r3 = r1j * r1j * r1j;
      double vjn = dot3(vj, n1j);
      /* Newtonian term of Eq. (1) */
      for (int q = 0; q < 3; ++q) newt[q] += -G * mass[j] * x1j[q] / r3;
      /* Eq. (2) */
      double br = 5.0 * G * M / r1j - 2.0 * dot3(vj, vj) + 1.5 * vjn * vjn;
      double vx = dot3(vj, x1j);
      for (int q = 0; q < 3; ++q)
        aBH[q] += G * mass[j] * x1j[q] / r3 * br + 3.0 * G * mass[j] / r3 * vx * vj[q];
      /* Eq. (3), first line */
      double r4 = r3 * r1j;
      for (int q = 0; q < 3; ++q) aCr[q] += 4.0 * G * G * mass[j] * mass[j] * x1j[q] / r4;
      /* Eq. (3), double sums over k */
      for (idx_t k = 1; k < N; ++k) {
        const double *vk = vel + 3 * k;
        double x1k[3];
        double r1k = sep(x1, pos + 3 * k, eps2, x1k);
        if (k != j) {
          double xjk[3];
          double rjk = sep(pos + 3 * j, pos + 3 * k, eps2, xjk);
          double rjk3 = rjk * rjk * rjk;
          double f = 4.0 / r1k + 5.0 / (4.0 * rjk) - r1k * r1k / (4.0 * rjk3) +
                     r1j * r1j / (4.0 * rjk3);
          for (int q = 0; q < 3; ++q) {
            aCr[q] += G * G * mass[j] * mass[k] * x1j[q] / r3 * f;
            aCr[q] -= 3.5 * G * G * mass[j] * mass[k] * xjk[q] / (rjk3 * r1j);
          }
        }
        /* last line: k = j included */
        double vv = dot3(vj, vk), vjx = dot3(vj, x1j), vkx = dot3(vk, x1j);
        for (int q = 0; q < 3; ++q)
          aCr[q] -= G * mass[j] * mass[k] / (M * r3) *
                    (4.0 * vv * x1j[q] - 3.0 * vjx * vk[q] - 4.0 * vkx * vj[q]);
      }
    }
    for (int q = 0; q < 3; ++q) acc[q] = newt[q] + lam * aBH[q] + lam * aCr[q];
  }

  /* ---- Eq. (4): stars ---- */
#pragma omp parallel for schedule(static)
  for (idx_t i = 1; i < N; ++i) {
    const double *xi = pos + 3 * i, *vi = vel + 3 * i;
    double xi1[3];
    double ri1 = sep(xi, x1, eps2, xi1);
    double ri13 = ri1 * ri1 * ri1;
    double vi2 = dot3(vi, vi);
    double newt[3], aBH[3], aCr[3];
    /* Newtonian, massive object */
    for (int q = 0; q < 3; ++q) newt[q] = -G * M * xi1[q] / ri13;
    /* Eq. (5) */
    double vix = dot3(vi, xi1);
    for (int q = 0; q < 3; ++q)
      aBH[q] = G * M * xi1[q] / ri13 * (4.0 * G * M / ri1 - vi2) +
               4.0 * G * M / ri13 * vix * vi[q];
    /* Eq. (6), first line */
    for (int q = 0; q < 3; ++q)
      aCr[q] = 5.0 * G * G * mass[i] * M * xi1[q] / (ri13 * ri1) -
               G * mass[i] / ri13 * (4.0 * vi2 * xi1[q] - 7.0 * vix * vi[q]);
    for (idx_t j = 1; j < N; ++j) {
      if (j == i) continue;
      const double *xj = pos + 3 * j, *vj = vel + 3 * j;
      double xij[3], xj1[3];
      double rij = sep(xi, xj, eps2, xij);
      double rj1 = sep(xj, x1, eps2, xj1);
      double rij3 = rij * rij * rij, rj13 = rj1 * rj1 * rj1;
      double nij[3] = {xij[0] / rij, xij[1] / rij, xij[2] / rij};
      double vij[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
      /* Newtonian, stars (Eq. (4) with r_ij^3) */
      for (int q = 0; q < 3; ++q) newt[q] -= G * mass[j] * xij[q] / rij3;
      double f3 = 4.0 / rij + 5.0 / (4.0 * rj1) + ri1 * ri1 / (4.0 * rj13) -
                  rij * rij / (4.0 * rj13);
      double f4 = 4.0 / ri1 + 5.0 / (4.0 * rj1) - ri1 * ri1 / (4.0 * rj13) +
                  rij * rij / (4.0 * rj13);
      double vjn = dot3(vj, nij);
      double b7 = vi2 - 2.0 * dot3(vij, vij) + 1.5 * vjn * vjn;
      double x8 = 4.0 * dot3(xij, vi) - 3.0 * dot3(xij, vj);
      double vv = dot3(vi, vj), vjx = dot3(vj, xi1);
      for (int q = 0; q < 3; ++q) {
        aCr[q] += G * G * mass[j] * M * xi1[q] / ri13 * f3;          /* line 2 */
        aCr[q] += G * G * mass[j] * M * xij[q] / rij3 * f4;          /* line 3 */
        aCr[q] -= 3.5 * G * G * mass[j] * M * xj1[q] / rj13 *
                  (1.0 / rij - 1.0 / ri1);                           /* line 4 */
        aCr[q] -= G * mass[j] / ri13 *
                  (4.0 * vv * xi1[q] - 3.0 * vjx * vi[q] - 4.0 * vix * vj[q]); /* line 5 */
        aCr[q] += G * mass[j] * xij[q] / rij3 * b7;                  /* line 6 */
        aCr[q] += G * mass[j] / rij3 * x8 * vij[q];                  /* line 7 */
      }
    }
    for (int q = 0; q < 3; ++q) acc[3 * i + q] = newt[q] + lam * aBH[q] + lam * aCr[q];
  }
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* Unrestricted EIH 1PN equations for every body (the equations the    */
/* paper starts from, Sec. 1-2), by brute force: every potential and   */
/* Newtonian acceleration inside a pair term is itself summed in place */
/* (O(N^3)).  Uses each body's own velocity, the massive object's       */
/* included.  Writes the 1PN part (times lambda) and the Newtonian part */
/* separately.  For small N only.                                       */
/*                                                                      */
/*   a_a = sum_{b!=a} -G m_b n_ab / R_ab^2                              */
/*     + lambda sum_{b!=a} { (G m_b / R_ab^2) n_ab [ -v_a^2 - 2 v_b^2     */
/*          + 4 v_a.v_b + 3/2 (n_ab.v_b)^2 + 4 sum_{c!=a} G m_c / R_ac    */
/*          + sum_{c!=b} G m_c / R_bc + 1/2 x_ab . a^N_b ]                */
/*        + (G m_b / R_ab^2) [n_ab.(4 v_a - 3 v_b)] (v_a - v_b)           */
/*        + 7/2 (G m_b / R_ab) a^N_b },  a^N_b = -sum_{c!=b} G m_c x_bc/R^3 */
/* ------------------------------------------------------------------ */
int pnref_eih(const double *pos, const double *vel, const double *mass, idx_t N,
              double G, double c, double eps, double *acc_newton, double *acc_1pn) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !acc_newton || !acc_1pn) return PNREF_EINVAL;
  const double lam = lambda_of(c);
  const double eps2 = eps * eps;
  for (idx_t a = 0; a < N; ++a) {
    const double *xa = pos + 3 * a, *va = vel + 3 * a;
    double newt[3] = {0, 0, 0}, pn[3] = {0, 0, 0};
    for (idx_t b = 0; b < N; ++b) {
      if (b == a) continue;
      const double *xb = pos + 3 * b, *vb = vel + 3 * b;
      double xab[3];
      double R = sep(xa, xb, eps2, xab);
      double n[3] = {xab[0] / R, xab[1] / R, xab[2] / R};
      double Va = 0.0, Vb = 0.0, aNb[3] = {0, 0, 0}, t[3];
      for (idx_t cc = 0; cc < N; ++cc) {
        if (cc != a) Va += G * mass[cc] / sep(xa, pos + 3 * cc, eps2, t);
        if (cc != b) {
          double Rbc = sep(xb, pos + 3 * cc, eps2, t); /* x_bc */
          Vb += G * mass[cc] / Rbc;
          for (int q = 0; q < 3; ++q) aNb[q] -= G * mass[cc] * t[q] / (Rbc * Rbc * Rbc);
        }
      }
      double nvb = dot3(n, vb);
      double br = -dot3(va, va) - 2.0 * dot3(vb, vb) + 4.0 * dot3(va, vb) + 1.5 * nvb * nvb +
                  4.0 * Va + Vb + 0.5 * dot3(xab, aNb);
      double D = 4.0 * dot3(n, va) - 3.0 * nvb;
      double k = G * mass[b] / (R * R);
      for (int q = 0; q < 3; ++q) {
        newt[q] -= k * n[q];
        pn[q] += k * br * n[q] + k * D * (va[q] - vb[q]) + 3.5 * (G * mass[b] / R) * aNb[q];
      }
    }
    for (int q = 0; q < 3; ++q) {
      acc_newton[3 * a + q] = newt[q];
      acc_1pn[3 * a + q] = lam * pn[q];
    }
  }
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* The same unrestricted EIH equations with each body's potential V_b  */
/* and Newtonian acceleration a^N_b summed once beforehand (O(N^2)):    */
/* the definition above, not regrouped.  Writes a^N, phi = -V and the   */
/* 1PN part (times lambda) of every body.                               */
/* ------------------------------------------------------------------ */
/* 1PN part (without lambda) of body a from every body's Newtonian      */
/* potential phi = -V and acceleration aN: the EIH pair sum above.      */
static void eih_row(const double *pos, const double *vel, const double *mass, idx_t N,
                    double G, double eps2, const double *phi, const double *acc_newton,
                    idx_t a, double pn[3]) {
  const double *xa = pos + 3 * a, *va = vel + 3 * a;
  const double Va = -phi[a];
  pn[0] = pn[1] = pn[2] = 0.0;
  for (idx_t b = 0; b < N; ++b) {
    if (b == a) continue;
    const double *xb = pos + 3 * b, *vb = vel + 3 * b, *aNb = acc_newton + 3 * b;
    double xab[3];
    double R = sep(xa, xb, eps2, xab);
    double n[3] = {xab[0] / R, xab[1] / R, xab[2] / R};
    double nvb = dot3(n, vb);
    double br = -dot3(va, va) - 2.0 * dot3(vb, vb) + 4.0 * dot3(va, vb) + 1.5 * nvb * nvb +
                4.0 * Va - phi[b] + 0.5 * dot3(xab, aNb);
    double D = 4.0 * dot3(n, va) - 3.0 * nvb;
    double k = G * mass[b] / (R * R);
    for (int q = 0; q < 3; ++q)
      pn[q] += k * br * n[q] + k * D * (va[q] - vb[q]) + 3.5 * (G * mass[b] / R) * aNb[q];
  }
}

int pnref_eih2(const double *pos, const double *vel, const double *mass, idx_t N, double G,
               double c, double eps, double *acc_newton, double *phi, double *acc_1pn) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !acc_newton || !phi || !acc_1pn) return PNREF_EINVAL;
  rc = pnref_newton(pos, mass, N, G, eps, acc_newton, phi);
  if (rc) return rc;
  const double lam = lambda_of(c);
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (idx_t a = 0; a < N; ++a) {
    double pn[3];
    eih_row(pos, vel, mass, N, G, eps2, phi, acc_newton, a, pn);
    for (int q = 0; q < 3; ++q) acc_1pn[3 * a + q] = lam * pn[q];
  }
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* pnref_eih2 for the given bodies only: the Newtonian pass over every  */
/* body (O(N^2); every partner's potential and acceleration enters),    */
/* then the O(N) EIH sum of each requested row.  Outputs are [nrows] /  */
/* [nrows][3] in the order of rows.                                     */
/* ------------------------------------------------------------------ */
int pnref_eih2_rows(const double *pos, const double *vel, const double *mass, idx_t N,
                    double G, double c, double eps, const idx_t *rows, idx_t nrows,
                    double *acc_newton, double *phi, double *acc_1pn) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !rows || nrows < 0 || !acc_newton || !phi || !acc_1pn)
    return PNREF_EINVAL;
  for (idx_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= N) return PNREF_EINVAL;
  double *aN = (double *)malloc(sizeof(double) * 3 * N);
  double *ph = (double *)malloc(sizeof(double) * N);
  if (!aN || !ph) {
    free(aN);
    free(ph);
    return PNREF_ENOMEM;
  }
  rc = pnref_newton(pos, mass, N, G, eps, aN, ph);
  if (!rc) {
    const double lam = lambda_of(c);
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (idx_t r = 0; r < nrows; ++r) {
      const idx_t a = rows[r];
      double pn[3];
      eih_row(pos, vel, mass, N, G, eps2, ph, aN, a, pn);
      for (int q = 0; q < 3; ++q) {
        acc_newton[3 * r + q] = aN[3 * a + q];
        acc_1pn[3 * r + q] = lam * pn[q];
      }
      phi[r] = ph[a];
    }
  }
  free(aN);
  free(ph);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Textbook two-body 1PN relative acceleration in harmonic gauge (the  */
/* N = 2 case of the EIH equations the paper cites):                   */
/*   a = -(G m / r^2) [ (1 + lambda A) n + lambda B v ]                  */
/*   A = -3/2 nu rdot^2 + (1 + 3 nu) v^2 - 2 (2 + nu) G m / r           */
/*   B = -2 (2 - nu) rdot,  m = m1 + m2, nu = m1 m2 / m^2, rdot = n.v    */
/* x = x1 - x2, v = v1 - v2.  Unsoftened.  Writes Newtonian and 1PN     */
/* parts of the relative acceleration separately.                       */
/* ------------------------------------------------------------------ */
int pnref_twobody(const double *x, const double *v, double m1, double m2, double G,
                  double c, double *a_newton, double *a_1pn) {
  if (!x || !v || !a_newton || !a_1pn || !(m1 > 0.0) || !(m2 > 0.0)) return PNREF_EINVAL;
  if (check_c(c)) return PNREF_EINVAL;
  const double lam = lambda_of(c);
  double m = m1 + m2, nu = m1 * m2 / (m * m);
  double r = sqrt(dot3(x, x));
  double n[3] = {x[0] / r, x[1] / r, x[2] / r};
  double rdot = dot3(n, v), v2 = dot3(v, v);
  double A = -1.5 * nu * rdot * rdot + (1.0 + 3.0 * nu) * v2 - 2.0 * (2.0 + nu) * G * m / r;
  double B = -2.0 * (2.0 - nu) * rdot;
  double k = G * m / (r * r);
  for (int q = 0; q < 3; ++q) {
    a_newton[q] = -k * n[q];
    a_1pn[q] = -k * lam * (A * n[q] + B * v[q]);
  }
  return PNREF_OK;
}

/* ------------------------------------------------------------------ */
/* Classical fourth-order Runge-Kutta with fixed step (Sec. 3.2 and     */
/* Sec. 4) on y = (x, v) of all N bodies, the massive object included: */
/*   k1 = f(y), k2 = f(y + dt/2 k1), k3 = f(y + dt/2 k2),               */
/*   k4 = f(y + dt k3), y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4),           */
/* f(x, v) = (v, a^N(x) + a^1PN(x, v)).  pos, vel updated in place.    */
/* ------------------------------------------------------------------ */
static int deriv(const double *x, const double *v, const double *mass, idx_t N, double G,
                 double c, double eps, double *aN, double *ph, double *a1, double *a) {
  int rc = pnref_accel(x, v, mass, N, G, c, eps, aN, ph, a1);
  if (rc) return rc;
  for (idx_t t = 0; t < 3 * N; ++t) a[t] = aN[t] + a1[t];
  return PNREF_OK;
}

int pnref_step(double *pos, double *vel, const double *mass, idx_t N, double G, double c,
               double eps, double dt, idx_t nsteps) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !isfinite(dt) || nsteps < 0) return PNREF_EINVAL;
  const idx_t n3 = 3 * N;
  double *buf = (double *)malloc(sizeof(double) * (size_t)n3 * 14 + sizeof(double) * N);
  if (!buf) return PNREF_ENOMEM;
  double *kx1 = buf, *kv1 = kx1 + n3, *kx2 = kv1 + n3, *kv2 = kx2 + n3, *kx3 = kv2 + n3,
         *kv3 = kx3 + n3, *kx4 = kv3 + n3, *kv4 = kx4 + n3, *xs = kv4 + n3, *vs = xs + n3,
         *aN = vs + n3, *a1 = aN + n3, *a = a1 + n3, *ph = a + n3;
  (void)ph;
  for (idx_t step = 0; step < nsteps; ++step) {
    /* k1 */
    memcpy(kx1, vel, sizeof(double) * n3);
    if ((rc = deriv(pos, vel, mass, N, G, c, eps, aN, ph, a1, kv1))) break;
    /* k2 */
    for (idx_t t = 0; t < n3; ++t) {
      xs[t] = pos[t] + 0.5 * dt * kx1[t];
      vs[t] = vel[t] + 0.5 * dt * kv1[t];
    }
    memcpy(kx2, vs, sizeof(double) * n3);
    if ((rc = deriv(xs, vs, mass, N, G, c, eps, aN, ph, a1, kv2))) break;
    /* k3 */
    for (idx_t t = 0; t < n3; ++t) {
      xs[t] = pos[t] + 0.5 * dt * kx2[t];
      vs[t] = vel[t] + 0.5 * dt * kv2[t];
    }
    memcpy(kx3, vs, sizeof(double) * n3);
    if ((rc = deriv(xs, vs, mass, N, G, c, eps, aN, ph, a1, kv3))) break;
    /* k4 */
    for (idx_t t = 0; t < n3; ++t) {
      xs[t] = pos[t] + dt * kx3[t];
      vs[t] = vel[t] + dt * kv3[t];
    }
    memcpy(kx4, vs, sizeof(double) * n3);
    if ((rc = deriv(xs, vs, mass, N, G, c, eps, aN, ph, a1, kv4))) break;
    /* combine */
    for (idx_t t = 0; t < n3; ++t) {
      pos[t] += dt / 6.0 * (kx1[t] + 2.0 * kx2[t] + 2.0 * kx3[t] + kx4[t]);
      vel[t] += dt / 6.0 * (kv1[t] + 2.0 * kv2[t] + 2.0 * kv3[t] + kv4[t]);
    }
  }
  free(buf);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Jerk (time derivative of the acceleration along the motion, needed by */
/* the Hermite scheme the paper proposes in Sec. 5 / Appendix A):        */
/*   jerk = d/dh a(x + h v, v + h a) at h = 0,                          */
/* the derivative of the limited-1PN acceleration in the direction of   */
/* the flow, by Richardson-extrapolated central differences:            */
/*   [8 (a(h) - a(-h)) - (a(2h) - a(-2h))] / (12 h),  error O(h^4).     */
/* acc_out receives a itself.                                            */
/* ------------------------------------------------------------------ */
int pnref_jerk(const double *pos, const double *vel, const double *mass, idx_t N, double G,
               double c, double eps, double h, double *acc_out, double *jerk) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !acc_out || !jerk || !(h > 0.0)) return PNREF_EINVAL;
  const idx_t n3 = 3 * N;
  double *buf = (double *)malloc(sizeof(double) * (size_t)n3 * 6 + sizeof(double) * N);
  if (!buf) return PNREF_ENOMEM;
  double *xs = buf, *vs = xs + n3, *aN = vs + n3, *a1 = aN + n3, *ap = a1 + n3,
         *am = ap + n3, *ph = am + n3;
  if ((rc = pnref_accel(pos, vel, mass, N, G, c, eps, aN, ph, a1))) goto done;
  for (idx_t t = 0; t < n3; ++t) acc_out[t] = aN[t] + a1[t];
  for (idx_t t = 0; t < n3; ++t) jerk[t] = 0.0;
  for (int k = 1; k <= 2; ++k) {
    const double w = (k == 1) ? 8.0 : -1.0;
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      const double hh = sgn * k * h;
      for (idx_t t = 0; t < n3; ++t) {
        xs[t] = pos[t] + hh * vel[t];
        vs[t] = vel[t] + hh * acc_out[t];
      }
      if ((rc = pnref_accel(xs, vs, mass, N, G, c, eps, aN, ph, a1))) goto done;
      double *dst = (sgn > 0) ? ap : am;
      for (idx_t t = 0; t < n3; ++t) dst[t] = aN[t] + a1[t];
    }
    for (idx_t t = 0; t < n3; ++t) jerk[t] += w * (ap[t] - am[t]);
  }
  for (idx_t t = 0; t < n3; ++t) jerk[t] /= 12.0 * h;
done:
  free(buf);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Exact jerk by complex-step differentiation (Lyness & Moler 1967;     */
/* Squire & Trapp 1998).  For f analytic along the path,               */
/*   f(x + i h d) = f(x) + i h f'(x) d + O(h^2),                        */
/* so Re f = f(x) and Im f / h = f'(x) d to rounding: there is no       */
/* difference of nearby values, hence no cancellation, and with h tiny  */
/* (1e-20 here) the O(h^2) remainder is far below one ulp.  The limited-*/
/* 1PN acceleration (the definition of pnref_accel, written out again   */
/* below in complex arithmetic) is evaluated at positions x + i h v and */
/* velocities v + i h a, with a = pnref_accel's acceleration: this is    */
/* the derivative along the motion, jerk = (v.grad_x + a.grad_v) a.     */
/* Every operation is analytic -- sums, products, quotients and the     */
/* principal square root of numbers with positive real part -- and no  */
/* branch depends on a complex value.                                    */
/* ------------------------------------------------------------------ */
typedef double complex cpx;

static const double kCsH = 1e-20; /* complex step */

static cpx cdot3(const cpx *a, const cpx *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* d = xa - xb; returns R = sqrt(|d|^2 + eps^2) (principal root) */
static cpx csep(const cpx *xa, const cpx *xb, double eps2, cpx *d) {
  for (int q = 0; q < 3; ++q) d[q] = xa[q] - xb[q];
  return csqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2);
}

/* rows: nrows indices into 0..N-1; acc_out, jerk_out: [nrows][3] in that
   order.  Star rows cost O(N) each on top of one real evaluation of all
   bodies (the direction a); the massive object's row needs every star's
   potential and Newtonian acceleration, one more O(N^2) pass. */
int pnref_jerk_rows(const double *pos, const double *vel, const double *mass, idx_t N, double G,
                    double c, double eps, const idx_t *rows, idx_t nrows, double *acc_out,
                    double *jerk_out) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !rows || nrows < 0 || !acc_out || !jerk_out) return PNREF_EINVAL;
  for (idx_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= N) return PNREF_EINVAL;
  const idx_t n3 = 3 * N;
  const double lam = lambda_of(c), eps2 = eps * eps, M = mass[0], h = kCsH;
  double *ra = (double *)malloc(sizeof(double) * (size_t)(2 * n3 + N));
  cpx *X = (cpx *)malloc(sizeof(cpx) * (size_t)n3);
  cpx *W = (cpx *)malloc(sizeof(cpx) * (size_t)n3);
  cpx *u = (cpx *)malloc(sizeof(cpx) * (size_t)N);
  cpx *b = (cpx *)malloc(sizeof(cpx) * (size_t)n3);
  cpx *V = (cpx *)malloc(sizeof(cpx) * (size_t)N);
  cpx *aN = (cpx *)malloc(sizeof(cpx) * (size_t)n3);
  char *want = (char *)calloc((size_t)N, 1);
  if (!ra || !X || !W || !u || !b || !V || !aN || !want) {
    rc = PNREF_ENOMEM;
    goto done;
  }
  /* the direction of the velocities: the acceleration itself */
  {
    double *raN = ra, *ra1 = ra + n3, *rph = ra + 2 * n3;
    if ((rc = pnref_accel(pos, vel, mass, N, G, c, eps, raN, rph, ra1))) goto done;
    for (idx_t t = 0; t < n3; ++t) {
      X[t] = pos[t] + I * (h * vel[t]);
      W[t] = vel[t] + I * (h * (raN[t] + ra1[t]));
    }
  }
  /* massive object's potential u_s = G M / R_s0 and pull b_s at each star */
  u[0] = 0.0;
  b[0] = b[1] = b[2] = 0.0;
  for (idx_t s = 1; s < N; ++s) {
    cpx d[3];
    cpx R = csep(X + 3 * s, X, eps2, d);
    u[s] = G * M / R;
    for (int q = 0; q < 3; ++q) b[3 * s + q] = G * M * d[q] / (R * R * R);
  }
  /* w = -P/M, P = sum_s m_s v_s */
  cpx w[3] = {0.0, 0.0, 0.0};
  for (idx_t s = 1; s < N; ++s)
    for (int q = 0; q < 3; ++q) w[q] += mass[s] * W[3 * s + q];
  for (int q = 0; q < 3; ++q) w[q] = -w[q] / M;
  /* Newtonian potential magnitude V_a and acceleration aN_a: the massive
     object, the requested rows, and every body if the massive object's
     row is requested */
  want[0] = 1;
  for (idx_t r = 0; r < nrows; ++r) {
    want[rows[r]] = 1;
    if (rows[r] == 0) memset(want, 1, (size_t)N);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (idx_t a = 0; a < N; ++a) {
    if (!want[a]) continue;
    cpx Va = 0.0, g[3] = {0.0, 0.0, 0.0}, d[3];
    for (idx_t e = 0; e < N; ++e) {
      if (e == a) continue;
      cpx R = csep(X + 3 * a, X + 3 * e, eps2, d);
      Va += G * mass[e] / R;
      for (int q = 0; q < 3; ++q) g[q] -= G * mass[e] * d[q] / (R * R * R);
    }
    V[a] = Va;
    for (int q = 0; q < 3; ++q) aN[3 * a + q] = g[q];
  }
  const cpx *x0 = X, *aN0 = aN;
  const cpx V0 = V[0];
#pragma omp parallel for schedule(dynamic, 1)
  for (idx_t r = 0; r < nrows; ++r) {
    const idx_t i = rows[r];
    cpx pn[3] = {0.0, 0.0, 0.0};
    if (i == 0) {
      /* massive object: one term per star s */
      for (idx_t s = 1; s < N; ++s) {
        const cpx *vs = W + 3 * s, *as = aN + 3 * s;
        cpx d[3];
        cpx R = csep(x0, X + 3 * s, eps2, d);
        cpx n[3] = {d[0] / R, d[1] / R, d[2] / R};
        cpx k = G * mass[s] / (R * R), nv = cdot3(n, vs), nw = cdot3(n, w);
        cpx br = -2.0 * cdot3(vs, vs) + 4.0 * cdot3(w, vs) + 1.5 * nv * nv + 4.0 * V0 + V[s] +
                 0.5 * cdot3(d, as);
        for (int q = 0; q < 3; ++q)
          pn[q] += k * (br * n[q] + 3.0 * nv * vs[q] - 3.0 * nv * w[q] - 4.0 * nw * vs[q]) +
                   3.5 * (G * mass[s] / R) * as[q];
      }
    } else {
      const cpx *xi = X + 3 * i, *vi = W + 3 * i;
      const cpx vi2 = cdot3(vi, vi);
      /* partner: the massive object */
      {
        cpx d[3];
        cpx R = csep(xi, x0, eps2, d);
        cpx n[3] = {d[0] / R, d[1] / R, d[2] / R};
        cpx k = G * M / (R * R), nw = cdot3(n, w), n4v = 4.0 * cdot3(n, vi);
        cpx br = -vi2 + 4.0 * cdot3(vi, w) + 4.0 * V[i] + V0 + 0.5 * cdot3(d, aN0);
        for (int q = 0; q < 3; ++q)
          pn[q] += k * (br * n[q] + n4v * (vi[q] - w[q]) - 3.0 * nw * vi[q]) +
                   3.5 * (G * M / R) * aN0[q];
      }
      /* partners: stars j != i */
      for (idx_t j = 1; j < N; ++j) {
        if (j == i) continue;
        const cpx *vj = W + 3 * j, *bj = b + 3 * j;
        cpx d[3];
        cpx R = csep(xi, X + 3 * j, eps2, d);
        cpx n[3] = {d[0] / R, d[1] / R, d[2] / R};
        cpx k = G * mass[j] / (R * R), nv = cdot3(n, vj);
        cpx S = -vi2 - 2.0 * cdot3(vj, vj) + 4.0 * cdot3(vi, vj) + 1.5 * nv * nv + 4.0 * u[i] +
                u[j] - 0.5 * cdot3(d, bj);
        cpx D = 4.0 * cdot3(n, vi) - 3.0 * nv;
        for (int q = 0; q < 3; ++q)
          pn[q] += k * (S * n[q] + D * (vi[q] - vj[q])) - 3.5 * (G * mass[j] / R) * bj[q];
      }
    }
    for (int q = 0; q < 3; ++q) {
      cpx tot = aN[3 * i + q] + lam * pn[q];
      acc_out[3 * r + q] = creal(tot);
      jerk_out[3 * r + q] = cimag(tot) / h;
    }
  }
done:
  free(ra);
  free(X);
  free(W);
  free(u);
  free(b);
  free(V);
  free(aN);
  free(want);
  return rc;
}

/* All N bodies (rows 0..N-1). */
int pnref_jerk_exact(const double *pos, const double *vel, const double *mass, idx_t N, double G,
                     double c, double eps, double *acc_out, double *jerk_out) {
  if (N < 2) return PNREF_EINVAL;
  idx_t *rows = (idx_t *)malloc(sizeof(idx_t) * (size_t)N);
  if (!rows) return PNREF_ENOMEM;
  for (idx_t r = 0; r < N; ++r) rows[r] = r;
  int rc = pnref_jerk_rows(pos, vel, mass, N, G, c, eps, rows, N, acc_out, jerk_out);
  free(rows);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Fourth-order Hermite scheme with a fixed step (predict, evaluate,    */
/* correct), the scheme the paper names as the remedy for close          */
/* encounters (Sec. 4-5):                                               */
/*   x_p = x + v dt + a dt^2/2 + j dt^3/6 + s dt^4/24 + k dt^5/120       */
/*   v_p = v + a dt + j dt^2/2 + s dt^3/6 + k dt^4/24                    */
/*   (a_p, j_p) at (x_p, v_p)                                           */
/*   v' = v + (a + a_p) dt/2 + (j - j_p) dt^2/12                         */
/*   x' = x + (v + v') dt/2 + (a - a_p) dt^2/12                          */
/* s, k (snap, crackle) come from the step's Hermite interpolation of   */
/* a:  s_0 = (-6 (a - a_p) - dt (4 j + 2 j_p)) / dt^2,                   */
/*     k = (12 (a - a_p) + 6 dt (j + j_p)) / dt^3,  s <- s_0 + k dt,     */
/* and are zero before the first step.  The velocity-dependent 1PN force */
/* makes the predicted velocity matter: with the plain predictor         */
/* (a and j only) its O(dt^3) error would leave the scheme third order.  */
/* Jerks from pnref_jerk with difference step h, or, with h = 0, the    */
/* exact ones of pnref_jerk_exact.                                       */
/* ------------------------------------------------------------------ */
static int jerk_of(const double *pos, const double *vel, const double *mass, idx_t N, double G,
                   double c, double eps, double h, double *acc, double *jerk) {
  if (h == 0.0) return pnref_jerk_exact(pos, vel, mass, N, G, c, eps, acc, jerk);
  return pnref_jerk(pos, vel, mass, N, G, c, eps, h, acc, jerk);
}

int pnref_hermite(double *pos, double *vel, const double *mass, idx_t N, double G, double c,
                  double eps, double dt, idx_t nsteps, double h) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !isfinite(dt) || !(dt > 0.0) || nsteps < 0 || !(h >= 0.0) ||
      !isfinite(h))
    return PNREF_EINVAL;
  const idx_t n3 = 3 * N;
  double *buf = (double *)malloc(sizeof(double) * (size_t)n3 * 8);
  if (!buf) return PNREF_ENOMEM;
  double *a = buf, *j = a + n3, *sn = j + n3, *cr = sn + n3, *xp = cr + n3, *vp = xp + n3,
         *ap = vp + n3, *jp = ap + n3;
  const double dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
  if ((rc = jerk_of(pos, vel, mass, N, G, c, eps, h, a, j))) goto done;
  for (idx_t t = 0; t < n3; ++t) sn[t] = cr[t] = 0.0;
  for (idx_t step = 0; step < nsteps; ++step) {
    for (idx_t t = 0; t < n3; ++t) {
      xp[t] = pos[t] + dt * vel[t] + dt2 / 2.0 * a[t] + dt3 / 6.0 * j[t] + dt4 / 24.0 * sn[t] +
              dt5 / 120.0 * cr[t];
      vp[t] = vel[t] + dt * a[t] + dt2 / 2.0 * j[t] + dt3 / 6.0 * sn[t] + dt4 / 24.0 * cr[t];
    }
    if ((rc = jerk_of(xp, vp, mass, N, G, c, eps, h, ap, jp))) break;
    for (idx_t t = 0; t < n3; ++t) {
      double vn = vel[t] + dt / 2.0 * (a[t] + ap[t]) + dt2 / 12.0 * (j[t] - jp[t]);
      pos[t] = pos[t] + dt / 2.0 * (vel[t] + vn) + dt2 / 12.0 * (a[t] - ap[t]);
      vel[t] = vn;
      double s0 = (-6.0 * (a[t] - ap[t]) - dt * (4.0 * j[t] + 2.0 * jp[t])) / dt2;
      double k = (12.0 * (a[t] - ap[t]) + 6.0 * dt * (j[t] + jp[t])) / dt3;
      sn[t] = s0 + k * dt;
      cr[t] = k;
      a[t] = ap[t];
      j[t] = jp[t];
    }
  }
done:
  free(buf);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Conserved quantities, Eqs. (7) and (8), by direct summation as       */
/* printed.  Double sums over i, j run over ordered star pairs with     */
/* i != j wherever r_ij appears; the last term of Eq. (7),             */
/* 1/2 sum_{i,j} G^2 M m_i m_j / (r_1i r_1j), contains no r_ij and runs */
/* over all (i, j) including i = j (it is the three-body term of the    */
/* 1PN energy with both partners the same star).  v_1 is the massive    */
/* object's own velocity.                                               */
/* out[0] = Newtonian energy, out[1] = lambda * 1PN energy bracket,     */
/* out[2..4] = Newtonian momentum, out[5..7] = lambda * 1PN momentum    */
/* terms.  E = out[0] + out[1], P = out[2..4] + out[5..7].              */
/* ------------------------------------------------------------------ */
int pnref_diagnostics(const double *pos, const double *vel, const double *mass, idx_t N,
                      double G, double c, double eps, double *out) {
  int rc = check_common(pos, mass, N, G, eps);
  if (rc) return rc;
  if (check_c(c) || !vel || !out) return PNREF_EINVAL;
  const double lam = lambda_of(c);
  const double eps2 = eps * eps;
  const double M = mass[0];
  const double *x1 = pos, *v1 = vel;
  const double v12 = dot3(v1, v1);

  double EN = 0.5 * M * v12, E1 = 0.0;
  double PN[3] = {M * v1[0], M * v1[1], M * v1[2]}, P1[3] = {0, 0, 0};
  double sum_over_r1i = 0.0; /* sum_i G m_i / r_1i, for the i = j-inclusive term */

  for (idx_t i = 1; i < N; ++i) {
    const double *xi = pos + 3 * i, *vi = vel + 3 * i;
    double vi2 = dot3(vi, vi);
    double x1i[3];
    double r1i = sep(x1, xi, eps2, x1i);
    double n1i[3] = {x1i[0] / r1i, x1i[1] / r1i, x1i[2] / r1i};
    /* Newtonian: 1/2 m v^2 and -G M m_i / r_1i */
    EN += 0.5 * mass[i] * vi2;
    EN -= G * M * mass[i] / r1i;
    /* 1PN single sums of Eq. (7) */
    E1 += 0.375 * mass[i] * vi2 * vi2;
    E1 += 1.5 * G * M * mass[i] / r1i * vi2;
    E1 += 0.5 * G * G * M * M * mass[i] / (r1i * r1i);
    E1 += 0.5 * G * M * mass[i] / r1i *
          (3.0 * v12 - 7.0 * dot3(v1, vi) - dot3(n1i, v1) * dot3(n1i, vi));
    sum_over_r1i += G * mass[i] / r1i;
    /* Eq. (8) */
    double vin = dot3(vi, n1i), v1n = dot3(v1, n1i);
    for (int q = 0; q < 3; ++q) {
      PN[q] += mass[i] * vi[q];
      P1[q] += 0.5 * mass[i] * vi[q] * vi2;
      P1[q] -= 0.5 * G * M * mass[i] / r1i * (vi[q] + vin * n1i[q]);
      P1[q] -= 0.5 * G * M * mass[i] / r1i * (v1[q] + v1n * n1i[q]);
    }
    /* pair sums over j != i */
    for (idx_t j = 1; j < N; ++j) {
      if (j == i) continue;
      const double *xj = pos + 3 * j, *vj = vel + 3 * j;
      double xij[3];
      double rij = sep(xi, xj, eps2, xij);
      double nij[3] = {xij[0] / rij, xij[1] / rij, xij[2] / rij};
      double k = G * mass[i] * mass[j] / rij;
      EN -= 0.5 * k;
      E1 += 0.25 * k * (6.0 * vi2 - 7.0 * dot3(vi, vj) - dot3(nij, vi) * dot3(nij, vj));
      E1 += G * G * M * mass[i] * mass[j] / (rij * r1i);
      double vin2 = dot3(vi, nij);
      for (int q = 0; q < 3; ++q) P1[q] -= 0.5 * k * (vi[q] + vin2 * nij[q]);
    }
  }
  /* 1/2 sum_{i,j} G^2 M m_i m_j / (r_1i r_1j), i = j included */
  E1 += 0.5 * M * sum_over_r1i * sum_over_r1i;

  out[0] = EN;
  out[1] = lam * E1;
  for (int q = 0; q < 3; ++q) {
    out[2 + q] = PN[q];
    out[5 + q] = lam * P1[q];
  }
  return PNREF_OK;
}
