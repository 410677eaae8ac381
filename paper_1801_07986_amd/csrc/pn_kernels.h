// pn_kernels.h -- gfx950 device code of libpn (included once, by pn_api.hip).
//
// Notation (Sec. 2 of the paper): body 0 is the massive object (the paper's
// #1, mass M); stars are bodies 1..N-1, stored as "star k" = body k+1 in every
// star-indexed array (Ns = N-1 stars).  x_ab = x_a - x_b, R_ab = sqrt(r^2+eps^2)
// (Eq. (10)), lambda = 1/c^2.
//
// Per force evaluation the work is split into
//   k_prologue   O(N)   massive-object/star pair terms u_s = G M / R_s0 and
//                       b_s = G M x_s0 / R_s0^3, star packets for the pair
//                       sweep, block partials of sum m_s b_s, m_s u_s, m_s v_s;
//   k_pair       O(N^2) star-star sweep: per star i the sums
//                         U_i  = sum_j G m_j / R_ij                (potential)
//                         G_i  = sum_j G m_j x_ij / R_ij^3         (= -g_i)
//                         Q_i  = sum_j (G m_j/R^3)[S'_ij x_ij - D'_ij v_j]
//                         C2_i = sum_j (G m_j/R^3) D'_ij        (stored / sqrt(3/2))
//                         Q7_i = sum_j (G m_j/R) (-b_j / 2)
//                       with S'_ij = e_j + 4 v_i.v_j + 3/2 (x_ij.v_j/R)^2
//                       - x_ij.b_j/2, e_j = -2 v_j^2 + u_j, and
//                       D'_ij = x_ij.(4 v_i - 3 v_j); written per j-split;
//   k_epilogue   O(N)   per star: reduces the splits, assembles the Newtonian
//                       and 1PN accelerations (Eqs. (4)-(6)), the star's term
//                       of the massive object's 1PN sum (Eqs. (2)-(3)) as block
//                       partials, and the Runge-Kutta stage update;
//   k_bh_final   O(N)   one block: the massive object's acceleration (Eq. (1))
//                       and stage update.
// The star-star 1PN sum of Eq. (6) needs no pass-1 result of any other star
// (only x, v, m and the O(N) massive-object terms u_j, b_j), so the potential
// sweep and the 1PN sweep share one pass over j.
//
// Runge-Kutta steps chain their evaluations: k_epilogue_chain also performs
// the next stage's prologue (each star's next state is in its registers), and
// k_pair_bh is the sweep with one extra workgroup doing the previous stage's
// k_bh_final work (the sweep reads only star packets), so a step is eight
// kernels.  Massive-object block rows hold 64 stars in every kernel, summed
// in the same tree, so whichever kernel writes a row it holds the same sum.
// For small systems k_stage runs a whole stage in one launch (each workgroup
// sums all j for a few stars and runs their epilogue; every workgroup
// recomputes the massive object's pending update), four kernels per step.
// All reductions of the O(N) kernels are wavefront xor butterflies.
//
// The same four kernels instantiated on dual numbers (T = S = Dual) give the
// time derivative of the force along the motion (the jerk of the Hermite
// scheme), and their epilogue carries the Hermite corrector and predictor the
// way the FP64 one carries the Runge-Kutta stage update.  In a jerk
// evaluation the FP64 epilogue writes the dual packets (k_epilogue_chain<Dual>)
// and the dual epilogue carries the FP64 massive-object update
// (k_epilogue_dual_bh): six kernels.  Further down:
// Eqs. (7)-(8) diagnostics (k_diag_*), close-encounter search (k_enc_*),
// the unrestricted EIH equations (k_eih_*, reusing k_pair), and batched
// ensembles (k_*_batched: one launch per phase for many systems).
#pragma once

#include <hip/hip_runtime.h>
#include <climits>
#include <type_traits>
#include <stdint.h>

namespace pn {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)
constexpr int kProRows = kBlock / 64;  // prologue block rows per workgroup (one per 64 stars)
constexpr int kNF = 11;      // pair-sum fields: U, G(3), Q(3), C2, Q7(3)
enum Field { F_U = 0, F_G = 1, F_Q = 4, F_C2 = 7, F_Q7 = 8 };
enum PairMode { MODE_P1 = 1, MODE_P2 = 2, MODE_FUSED = 3 };

// Star packet read by the pair sweep.  Positions stay FP64 so that coordinate
// differences are formed in FP64 in both precisions.  The velocity is stored
// scaled, s = sqrt(3/2) v: then 3/2 (x.v_j / R)^2 = (x.s_j / R)^2, and with
// the per-i vector (4/sqrt(3/2)) v_i the other velocity products come out
// unscaled (4 v_i.v_j = [(4/sqrt(3/2)) v_i].s_j); D'_ij / sqrt(3/2) is
// accumulated and rescaled in the epilogue.  The FP64 packet holds s/2 (see
// PairScale below).
constexpr double kSqrt32 = 1.22474487139158904909864203735;    // sqrt(3/2)
constexpr double kInvSqrt32 = 0.816496580927726032732428024902; // 1/sqrt(3/2)

// Scalings of the pair sweep.  The FP64 sweep refines v_rsq_f64 by a Newton
// step written Y = y (3 - x y^2), which is 2/R (three instructions; the form
// that yields 1/R takes four), and carries the factor 2 through instead of
// removing it: its packets hold s/2, its i-vector is 2 (4/sqrt(3/2)) v_i, the
// D-term coefficient is -8, and a wavefront's sums come out as 2U, 8G, 8Q,
// 16 C2 and 2 Q7, scaled back when it flushes them.  Every factor is a power
// of two, so the FP64 sums are those of the unscaled terms bit for bit except
// for the reciprocal square root itself.  The FP32 and dual-number sweeps use
// 1/R as it is.
template <typename T> struct PairScale {
  static constexpr double sv = kSqrt32;         // packet velocity = sv v
  static constexpr double inv_sv = kInvSqrt32;  // v = inv_sv (packet velocity)
  static constexpr double k = 8.0 / 3.0;        // i-vector = k (packet velocity)
  static constexpr double d = -2.0;             // D term: d (x.s_j) + x.k_i
  static constexpr double u = 1.0, g = 1.0, q = 1.0, c2 = 1.0, q7 = 1.0;  // flush factors
};
template <> struct PairScale<double> {
  static constexpr double sv = 0.5 * kSqrt32;
  static constexpr double inv_sv = 2.0 * kInvSqrt32;
  static constexpr double k = 32.0 / 3.0;
  static constexpr double d = -8.0;
  static constexpr double u = 0.5, g = 0.125, q = 0.125, c2 = 0.0625, q7 = 0.5;
};

struct alignas(16) PkF64 {
  double x, y, z, gm, svx, svy, svz, e, hbx, hby, hbz, pad;
};
struct alignas(16) PkF32 {
  double x, y, z;
  float gm, svx, svy, svz, e, hbx, hby, hbz, pad0, pad1;
};
static_assert(sizeof(PkF64) == 96, "packet layout");
static_assert(sizeof(PkF32) == 64, "packet layout");

template <typename T> struct PkOf;
template <> struct PkOf<double> { using type = PkF64; };
template <> struct PkOf<float> { using type = PkF32; };

// ---------------------------------------------------------------------------
// Reciprocal square root in FP64.  The hardware estimate (v_rsq_f64) is good
// to about 2^-24 relative (measured: 5.2e-8 at worst); one step of the
// third-order series
//   1/sqrt(x) = y (1 - r)^(-1/2) = y (1 + r/2 + 3 r^2/8 + ...),  r = 1 - x y^2
// brings it to full double precision (residual ~ (5/16) r^3 < 2^-70).  The
// O(N) kernels (massive-object terms, epilogues) use this.
//
// The O(N^2) pair sweeps use one Newton step instead: y (1 + e) becomes
// y (1 + r/2) = y (1 - 3/2 e^2 - e^3/2), at most 4.1e-15 below the true value
// (the sweep's accuracy target is 1e-12; measured per-body errors stay at
// 1e-14).  Written y (3 - x y^2) it is twice that in three instructions, two
// fewer than the series.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double r = fma(-x * y, y, 1.0);
  double p = fma(0.375, r, 0.5);
  return fma(y * r, p, y);
}
__device__ __forceinline__ double rsqrt_f64_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double r = fma(-x * y, y, 1.0);
  return fma(y * r, 0.5, y);
}
// The same Newton step as 2/sqrt(x) = y (3 - x y^2): one instruction less.
__device__ __forceinline__ double rsqrt2_f64_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  return y * fma(-x * y, y, 3.0);
}
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt_f64(x); }

// a*b + c with c wavefront-uniform (held in SGPRs).  For doubles the compiler
// otherwise copies c into a VGPR pair (two v_mov) to use the accumulating
// v_fmac form; one VOP3 v_fma_f64 with a scalar addend is the same operation.
__device__ __forceinline__ double fma_uniform_c(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}
__device__ __forceinline__ float fma_uniform_c(float a, float b, float c) { return fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// Forward-mode dual number v + d e (e^2 = 0).  Evaluating the force with every
// input replaced by (value, time derivative along the motion) -- positions
// (x, v), velocities (v, a) -- yields the acceleration in .v and its exact
// time derivative, the jerk, in .d (the Hermite scheme of Sec. 4-5 needs
// both).  Operators are hidden friends, so they never shadow the scalar
// overloads of fma & co. for plain doubles.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() = default;
  __host__ __device__ constexpr Dual(double x) : v(x), d(0.0) {}
  __host__ __device__ constexpr Dual(double x, double y) : v(x), d(y) {}
  friend __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
  friend __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
  friend __device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
  friend __device__ __forceinline__ Dual operator*(Dual a, Dual b) {
    return {a.v * b.v, fma(a.v, b.d, a.d * b.v)};
  }
  friend __device__ __forceinline__ Dual operator*(double s, Dual b) { return {s * b.v, s * b.d}; }
  friend __device__ __forceinline__ Dual operator*(Dual b, double s) { return {b.v * s, b.d * s}; }
  friend __device__ __forceinline__ Dual operator/(Dual a, double s) { return {a.v / s, a.d / s}; }
  __device__ __forceinline__ Dual& operator+=(Dual b) {
    v += b.v;
    d += b.d;
    return *this;
  }
  __device__ __forceinline__ Dual& operator*=(double s) {
    v *= s;
    d *= s;
    return *this;
  }
  friend __device__ __forceinline__ Dual fma(Dual a, Dual b, Dual c) {
    return {fma(a.v, b.v, c.v), fma(a.v, b.d, fma(a.d, b.v, c.d))};
  }
};
// d(x^-1/2) = -x^-3/2 dx / 2
__device__ __forceinline__ Dual rsqrt_t(Dual x) {
  const double y = rsqrt_f64(x.v);
  return {y, -0.5 * y * y * y * x.d};
}
// the pair sweep's reciprocal square root (FP64: one Newton step, see rsqrt_f64,
// and 2/R rather than 1/R, see PairScale)
__device__ __forceinline__ float rsqrt_pair(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_pair(double x) { return rsqrt2_f64_newton(x); }
__device__ __forceinline__ Dual rsqrt_pair(Dual x) {
  const double y = rsqrt_f64_newton(x.v);
  return {y, -0.5 * y * y * y * x.d};
}
__device__ __forceinline__ Dual fma_uniform_c(Dual a, Dual b, Dual c) { return fma(a, b, c); }

// Helpers that let the O(N) stages run on double or Dual: a Dual quantity
// stored in a row of width 2K keeps its value in column k and its derivative
// in column K + k.
template <typename T> struct IsDual { static constexpr bool value = false; };
template <> struct IsDual<Dual> { static constexpr bool value = true; };
template <typename T> struct Width { static constexpr int n = IsDual<T>::value ? 2 : 1; };
template <typename T> struct ScalarOf { using type = double; };  // O(N) arithmetic of a sweep type
template <> struct ScalarOf<Dual> { using type = Dual; };
template <typename T> struct PosOf { using type = double; };     // position type of a sweep type
template <> struct PosOf<Dual> { using type = Dual; };

__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(Dual x) { return x.v; }
__device__ __forceinline__ bool finite_s(double x) { return isfinite(x); }
__device__ __forceinline__ bool finite_s(Dual x) { return isfinite(x.v) && isfinite(x.d); }

// element i of a value array (and, for Dual, of its derivative array)
template <typename S> __device__ __forceinline__ S ld(const double* v, const double* d, size_t i);
template <> __device__ __forceinline__ double ld<double>(const double* v, const double*, size_t i) {
  return v[i];
}
template <> __device__ __forceinline__ Dual ld<Dual>(const double* v, const double* d, size_t i) {
  return Dual(v[i], d[i]);
}
// column k of a row holding K quantities
__device__ __forceinline__ void put(double* row, int k, int, double x) { row[k] = x; }
__device__ __forceinline__ void put(double* row, int k, int K, Dual x) {
  row[k] = x.v;
  row[K + k] = x.d;
}
template <typename S> __device__ __forceinline__ S get(const double* row, int k, int K);
template <> __device__ __forceinline__ double get<double>(const double* row, int k, int) {
  return row[k];
}
template <> __device__ __forceinline__ Dual get<Dual>(const double* row, int k, int K) {
  return Dual(row[k], row[K + k]);
}

// Star packet of the jerk sweep: every field with its time derivative.
struct alignas(16) PkDual {
  Dual x, y, z, gm, svx, svy, svz, e, hbx, hby, hbz;
};
static_assert(sizeof(PkDual) == 176, "packet layout");
template <> struct PkOf<Dual> { using type = PkDual; };
__device__ __forceinline__ void clear_pad(PkF64& p) { p.pad = 0.0; }
__device__ __forceinline__ void clear_pad(PkF32& p) { p.pad0 = p.pad1 = 0.f; }
__device__ __forceinline__ void clear_pad(PkDual&) {}

// Fixed-order workgroup sum of K doubles per thread; result in lds[k*kBlock].
template <int K>
__device__ __forceinline__ void block_sum(const double (&v)[K], double* lds) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) lds[k * kBlock + t] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int k = 0; k < K; ++k) lds[k * kBlock + t] += lds[k * kBlock + t + s];
    }
    __syncthreads();
  }
}

// A double from another lane of the same row of 16 by a DPP move (two 32-bit
// halves); CTRL: 0x141 lane i <- 7 - i within 8, 0x140 i <- 15 - i within 16,
// 0xB1 / 0x4E (quad permutations) i <- i ^ 1 / i ^ 2.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, true);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wavefront by six exchanges: lane i with 7 - i
// (within 8), i ^ 1, i ^ 2, 15 - i (within 16), i ^ 16, i ^ 32.  Both lanes
// of every exchange add the same two values, so after each level the lanes it
// joined hold the same bits, and at the end every lane holds the same sum; no
// barrier.  The first four levels are DPP moves within a row, the last two
// go through the LDS crossbar (ds_bpermute).
template <int K>
__device__ __forceinline__ void wave_allsum(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x141>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x4E>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x140>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], 16, 64);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], 32, 64);
}

// Element col of a register array, chosen per lane without indexing the
// array at run time (a chain of selects).
template <int K>
__device__ __forceinline__ double pick(const double (&v)[K], int col) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) r = col == k ? v[k] : r;
  return r;
}

// Wave index as a scalar (so that loop bounds derived from it stay uniform
// and j packets keep coming through scalar loads).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Sum of `rows` partial rows of width `stride` (first K columns), fixed order:
// lane l of every wavefront sums rows l, l+64, ..., then wave_allsum.  Every
// thread of every workgroup ends with the same bits, without a barrier.
// Split in two so that a kernel can request the rows of several sums before
// waiting for any: rows_load (this lane's partial sums), then rows_sum.
// The lane's first row is loaded, not added, so that up to 64 rows (every
// system of up to 4096 stars) rows_load issues its loads and returns without
// waiting for them.
template <int K>
__device__ __forceinline__ void rows_load(const double* part, int rows, int stride,
                                          double (&v)[K]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  if (l < rows) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = part[(size_t)l * stride + k];
  }
  for (int r = l + 64; r < rows; r += 64) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += part[(size_t)r * stride + k];
  }
}
template <int K>
__device__ __forceinline__ void rows_sum(const double (&v)[K], double (&out)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = v[k];
  wave_allsum<K>(out);
}
template <int K>
__device__ __forceinline__ void reduce_rows(const double* part, int rows, int stride,
                                            double (&out)[K]) {
  double v[K];
  rows_load<K>(part, rows, stride, v);
  rows_sum<K>(v, out);
}

__global__ void k_reset_status(int* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) status[0] = 0;
}

// ---------------------------------------------------------------------------
// Prologue: massive-object/star pair terms and star packets (O(N), FP64).
// ---------------------------------------------------------------------------
struct ProArgs {
  const double* pos;  // [N][3] (state of this evaluation)
  const double* vel;  // [N][3] or nullptr (Newtonian-only evaluation)
  const double* mass; // [N]
  int Ns;
  double G, eps2;
  void* pk;       // [Ns] packets (PkOf<T>)
  double* ub;     // [Ns][4 W]: u_s, b_s(3)
  double* bpart;  // [gridDim.x * kProRows][8 W]: per 64 stars sum m b (3), sum m u, sum m v (3), 0
  int* status;
  // jerk sweep (T = Dual): time derivatives of pos and vel (the velocity and
  // the acceleration of the evaluation state)
  const double* pos_d = nullptr;
  const double* vel_d = nullptr;
};

// Prologue terms of star k (body k + 1) at position xs, velocity vs, with the
// massive object at x0: writes the packet pk[k] and the row ub[k] = (u, b),
// and returns the star's block-sum terms v = (m b, m u, m v).  Shared by the
// prologue and by the Runge-Kutta epilogue that prepares the next evaluation.
template <typename T, typename S>
__device__ __forceinline__ void star_terms(const S (&x0)[3], const S (&xs)[3], const S (&vs)[3],
                                           double m, double G, double gM, double eps2, void* pk,
                                           double* ub_rows, int k, S (&v)[7]) {
  constexpr int W = Width<T>::n;
  const S dx = xs[0] - x0[0], dy = xs[1] - x0[1], dz = xs[2] - x0[2];
  const S rinv = rsqrt_t(fma(dz, dz, fma(dy, dy, fma(dx, dx, S(eps2)))));
  const S u = gM * rinv;
  const S b3 = u * rinv * rinv;
  const S bx = b3 * dx, by = b3 * dy, bz = b3 * dz;
  const S vx = vs[0], vy = vs[1], vz = vs[2];
  const S v2 = fma(vz, vz, fma(vy, vy, vx * vx));
  using Pk = typename PkOf<T>::type;
  Pk p;
  p.x = xs[0];
  p.y = xs[1];
  p.z = xs[2];
  p.gm = (T)(G * m);
  p.svx = (T)(PairScale<T>::sv * vx);
  p.svy = (T)(PairScale<T>::sv * vy);
  p.svz = (T)(PairScale<T>::sv * vz);
  p.e = (T)fma(S(-2.0), v2, u);
  p.hbx = (T)(-0.5 * bx);
  p.hby = (T)(-0.5 * by);
  p.hbz = (T)(-0.5 * bz);
  clear_pad(p);
  static_cast<Pk*>(pk)[k] = p;
  double* ub = ub_rows + 4 * W * (size_t)k;
  put(ub, 0, 4, u);
  put(ub, 1, 4, bx);
  put(ub, 2, 4, by);
  put(ub, 3, 4, bz);
  v[0] = m * bx;
  v[1] = m * by;
  v[2] = m * bz;
  v[3] = m * u;
  v[4] = m * vx;
  v[5] = m * vy;
  v[6] = m * vz;
}

// W = Width<T>::n doubles per quantity (value, and derivative for Dual).
template <typename T>
__device__ __forceinline__ void prologue_block(const ProArgs& a, int blk) {
  using S = typename ScalarOf<T>::type;
  constexpr int W = Width<T>::n;
  const int k = blk * kBlock + threadIdx.x;
  S v[7] = {0, 0, 0, 0, 0, 0, 0};
  if (k < a.Ns) {
    const int s = k + 1;
    const S x0[3] = {ld<S>(a.pos, a.pos_d, 0), ld<S>(a.pos, a.pos_d, 1),
                     ld<S>(a.pos, a.pos_d, 2)};
    const S xs[3] = {ld<S>(a.pos, a.pos_d, 3 * s), ld<S>(a.pos, a.pos_d, 3 * s + 1),
                     ld<S>(a.pos, a.pos_d, 3 * s + 2)};
    S vs[3] = {0.0, 0.0, 0.0};
    if (a.vel) {
      vs[0] = ld<S>(a.vel, a.vel_d, 3 * s);
      vs[1] = ld<S>(a.vel, a.vel_d, 3 * s + 1);
      vs[2] = ld<S>(a.vel, a.vel_d, 3 * s + 2);
    }
    star_terms<T, S>(x0, xs, vs, a.mass[s], a.G, a.G * a.mass[0], a.eps2, a.pk, a.ub, k, v);
  }
  // a block row per wavefront (64 stars), summed by wave_allsum and written
  // from the wavefront's own registers
  double flat[7 * W];
#pragma unroll
  for (int q = 0; q < 7; ++q) put(flat, q, 7, v[q]);
  wave_allsum<7 * W>(flat);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l < 8 * W) {
    // row layout: value columns 0..7, derivative columns 8..15 (Dual)
    const int q = l & 7, h = l >> 3;
    a.bpart[((size_t)blk * kProRows + w) * 8 * W + l] = q < 7 ? pick(flat, h * 7 + q) : 0.0;
  }
  if (blk == 0 && threadIdx.x == 0) {
    const double M = a.mass[0];
    if (!(M > 0.0) || !isfinite(M)) atomicOr(a.status, 2);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prologue(ProArgs a) {
  prologue_block<T>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Star-star sweep.  i-bodies live in registers (IPT per lane); every lane of a
// wavefront visits the same j at the same time, so the j packet is uniform and
// is read through the scalar unit into SGPRs (no LDS traffic, no per-lane
// broadcast).  A workgroup owns the i-range [ilo, ihi) and the j-range of one
// split (gridDim.y splits); with WS = 4 its four wavefronts share the i-range
// and divide the split's j-range into four pieces, reduced in LDS in fixed
// order at the end.  Partial sums go to part[split][field][star].
// T = double: FP64 throughout.  T = float: FP64 coordinate differences, FP32
// pair arithmetic, FP32 partial sums over tiles of kTile j added into FP64
// accumulators after each tile.  T = Dual: the FP64 sweep on dual numbers,
// 2 kNF fields per star (values, then their time derivatives).
// ---------------------------------------------------------------------------
struct PairArgs {
  const void* pk;
  int Ns;
  int jchunk;  // j per split
  double eps2;
  double* part;  // [gridDim.y][kNF W][Ns]
};

constexpr int kTile = 64;  // j per FP32 partial-sum tile (mixed precision)

template <typename T, int IPT>
struct PairAcc {
  T U[IPT], Gx[IPT], Gy[IPT], Gz[IPT], Qx[IPT], Qy[IPT], Qz[IPT], C2[IPT], Q7x[IPT], Q7y[IPT],
      Q7z[IPT];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      U[i] = Gx[i] = Gy[i] = Gz[i] = Qx[i] = Qy[i] = Qz[i] = C2[i] = Q7x[i] = Q7y[i] = Q7z[i] = T(0);
    }
  }
};

template <typename T, int IPT>
struct PairI {  // the i-side operands of one lane
  typename PosOf<T>::type x[IPT], y[IPT], z[IPT];
  T kx[IPT], ky[IPT], kz[IPT];  // (4/sqrt(3/2)) v_i
  int idx[IPT];
};

template <typename T, int MODE, int IPT, bool MASK>
__device__ __forceinline__ void pair_one(const typename PkOf<T>::type& p, int j, T eps2,
                                         const PairI<T, IPT>& I, PairAcc<T, IPT>& A) {
  using P = typename PosOf<T>::type;
  const P xj = p.x, yj = p.y, zj = p.z;
  const T gm = p.gm;
#pragma unroll
  for (int ii = 0; ii < IPT; ++ii) {
    const T dx = (T)(I.x[ii] - xj), dy = (T)(I.y[ii] - yj), dz = (T)(I.z[ii] - zj);
    T rinv = rsqrt_pair(fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2))));
    if (MASK) rinv = (j == I.idx[ii]) ? T(0) : rinv;
    const T rinv2 = rinv * rinv;
    const T mr = gm * rinv;
    const T mr3 = mr * rinv2;
    if (MODE & MODE_P1) A.U[ii] += mr;
    A.Gx[ii] = fma(mr3, dx, A.Gx[ii]);
    A.Gy[ii] = fma(mr3, dy, A.Gy[ii]);
    A.Gz[ii] = fma(mr3, dz, A.Gz[ii]);
    if (MODE & MODE_P2) {
      const T sx = p.svx, sy = p.svy, sz = p.svz;  // sqrt(3/2) v_j
      const T xs = fma(dz, sz, fma(dy, sy, dx * sx));
      const T t = xs * rinv;
      T s = fma_uniform_c(t, t, (T)p.e);           // e_j + 3/2 (x.v_j/R)^2
      s = fma(I.kz[ii], sz, fma(I.ky[ii], sy, fma(I.kx[ii], sx, s)));  // + 4 v_i.v_j
      s = fma(dz, (T)p.hbz, fma(dy, (T)p.hby, fma(dx, (T)p.hbx, s)));  // - x.b_j / 2
      const T x4 = fma(dz, I.kz[ii], fma(dy, I.ky[ii], dx * I.kx[ii]));
      const T D = fma(T(PairScale<T>::d), xs, x4);  // x.(4 v_i - 3 v_j) / sqrt(3/2)
      const T c1 = mr3 * s, c2 = mr3 * D;
      A.Qx[ii] = fma(-c2, sx, fma(c1, dx, A.Qx[ii]));
      A.Qy[ii] = fma(-c2, sy, fma(c1, dy, A.Qy[ii]));
      A.Qz[ii] = fma(-c2, sz, fma(c1, dz, A.Qz[ii]));
      A.C2[ii] += c2;
      A.Q7x[ii] = fma(mr, (T)p.hbx, A.Q7x[ii]);
      A.Q7y[ii] = fma(mr, (T)p.hby, A.Q7y[ii]);
      A.Q7z[ii] = fma(mr, (T)p.hbz, A.Q7z[ii]);
    }
  }
}

// j loop over [j0, j1).
template <typename T, int MODE, int IPT, bool MASK>
__device__ __forceinline__ void pair_range(const typename PkOf<T>::type* __restrict__ pk, int j0,
                                           int j1, T eps2, const PairI<T, IPT>& I,
                                           PairAcc<T, IPT>& A) {
  using Pk = typename PkOf<T>::type;
  int j = j0;
  // FP64: four j per iteration (the same order of additions, 1-2 % faster
  // than two); FP32 keeps two, where four cost occupancy
  if constexpr (sizeof(T) == 8) {
    for (; j + 3 < j1; j += 4) {
      const Pk p0 = pk[j];
      const Pk p1 = pk[j + 1];
      const Pk p2 = pk[j + 2];
      const Pk p3 = pk[j + 3];
      pair_one<T, MODE, IPT, MASK>(p0, j, eps2, I, A);
      pair_one<T, MODE, IPT, MASK>(p1, j + 1, eps2, I, A);
      pair_one<T, MODE, IPT, MASK>(p2, j + 2, eps2, I, A);
      pair_one<T, MODE, IPT, MASK>(p3, j + 3, eps2, I, A);
    }
  }
  // two j per iteration: two independent dependency chains per wavefront
  for (; j + 1 < j1; j += 2) {
    const Pk p0 = pk[j];
    const Pk p1 = pk[j + 1];
    pair_one<T, MODE, IPT, MASK>(p0, j, eps2, I, A);
    pair_one<T, MODE, IPT, MASK>(p1, j + 1, eps2, I, A);
  }
  if (j < j1) pair_one<T, MODE, IPT, MASK>(pk[j], j, eps2, I, A);
}

template <typename T, int MODE, int IPT>
__device__ __forceinline__ void pair_segment(const typename PkOf<T>::type* __restrict__ pk, int j0,
                                             int j1, int ilo, int ihi, T eps2,
                                             const PairI<T, IPT>& I, PairAcc<T, IPT>& A) {
  // the diagonal j == i can only occur for j in [ilo, ihi)
  const int m0 = max(j0, ilo), m1 = min(j1, ihi);
  if (m0 < m1) {
    pair_range<T, MODE, IPT, false>(pk, j0, m0, eps2, I, A);
    pair_range<T, MODE, IPT, true>(pk, m0, m1, eps2, I, A);
    pair_range<T, MODE, IPT, false>(pk, m1, j1, eps2, I, A);
  } else {
    pair_range<T, MODE, IPT, false>(pk, j0, j1, eps2, I, A);
  }
}

// acc[f] += s x (and acc[kNF + f] += s dx/dt for Dual); s is a PairScale
// factor, a power of two (1 outside the FP64 sweep)
template <int NFO, int IPT>
__device__ __forceinline__ void acc_add(double (&acc)[NFO][IPT], int f, int ii, float x, double s) {
  acc[f][ii] += (double)x * s;
}
template <int NFO, int IPT>
__device__ __forceinline__ void acc_add(double (&acc)[NFO][IPT], int f, int ii, double x,
                                        double s) {
  acc[f][ii] += x * s;
}
template <int NFO, int IPT>
__device__ __forceinline__ void acc_add(double (&acc)[NFO][IPT], int f, int ii, Dual x, double s) {
  acc[f][ii] += x.v * s;
  acc[kNF + f][ii] += x.d * s;
}

template <typename T, int IPT, int NFO>
__device__ __forceinline__ void acc_flush(const PairAcc<T, IPT>& A, double (&acc)[NFO][IPT]) {
#pragma unroll
  for (int ii = 0; ii < IPT; ++ii) {
    using SC = PairScale<T>;
    acc_add(acc, F_U, ii, A.U[ii], SC::u);
    acc_add(acc, F_G, ii, A.Gx[ii], SC::g);
    acc_add(acc, F_G + 1, ii, A.Gy[ii], SC::g);
    acc_add(acc, F_G + 2, ii, A.Gz[ii], SC::g);
    acc_add(acc, F_Q, ii, A.Qx[ii], SC::q);
    acc_add(acc, F_Q + 1, ii, A.Qy[ii], SC::q);
    acc_add(acc, F_Q + 2, ii, A.Qz[ii], SC::q);
    acc_add(acc, F_C2, ii, A.C2[ii], SC::c2);
    acc_add(acc, F_Q7, ii, A.Q7x[ii], SC::q7);
    acc_add(acc, F_Q7 + 1, ii, A.Q7y[ii], SC::q7);
    acc_add(acc, F_Q7 + 2, ii, A.Q7z[ii], SC::q7);
  }
}

__device__ __forceinline__ bool field_written(int f, int mode) {
  f %= kNF;  // derivative fields of the jerk sweep follow the value fields
  if (f == F_U) return (mode & MODE_P1) != 0;
  if (f < F_Q) return true;
  return (mode & MODE_P2) != 0;
}

// Threads of a sweep workgroup: WS wavefronts sharing one i-range of 64 IPT
// lanes (WS = 4 or 8), or 256 lanes (WS = 1).
template <int WS>
constexpr int pair_threads() {
  return WS == 8 ? 2 * kBlock : kBlock;
}

// LDS of pair_block's wavefront reduction: WS = 4, waves 1-3 park their sums;
// WS = 8, waves 4-7 then waves 1-3 (the same four regions).
template <typename T, int IPT, int WS>
constexpr int pair_red_doubles() {
  return WS > 1 ? (WS == 8 ? 4 : WS - 1) * kNF * Width<T>::n * IPT * 64 : 1;
}

// red: pair_red_doubles<T, IPT, WS>() doubles of LDS
template <typename T, int MODE, int IPT, int WS>
__device__ __forceinline__ void pair_block(const PairArgs& a, int ib, int sp, double* red) {
  using Pk = typename PkOf<T>::type;
  constexpr int NFO = kNF * Width<T>::n;  // output fields per star
  static_assert(WS == 1 || WS == 4 || WS == 8, "wavefronts per i-range");
  constexpr int LANES = pair_threads<WS>() / WS;  // distinct i-lanes per workgroup
  constexpr int IB = LANES * IPT;     // i-bodies per workgroup
  const Pk* __restrict__ pk = static_cast<const Pk*>(a.pk);
  const int wave = WS > 1 ? wave_id() : 0;
  const int lane = WS > 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int ilo = ib * IB;
  const int ihi = min(a.Ns, ilo + IB);
  PairI<T, IPT> I;
#pragma unroll
  for (int ii = 0; ii < IPT; ++ii) {
    I.idx[ii] = ilo + lane + ii * LANES;
    const int il = min(I.idx[ii], a.Ns - 1);  // lanes past the end compute on a copy, never stored
    const Pk& p = pk[il];
    I.x[ii] = p.x;
    I.y[ii] = p.y;
    I.z[ii] = p.z;
    // (4/sqrt(3/2)) v_i = (8/3) s_i (times 2 in FP64, see PairScale)
    I.kx[ii] = T(PairScale<T>::k) * (T)p.svx;
    I.ky[ii] = T(PairScale<T>::k) * (T)p.svy;
    I.kz[ii] = T(PairScale<T>::k) * (T)p.svz;
  }
  // j-range of this wavefront
  int j0 = sp * a.jchunk;
  int j1 = min(a.Ns, j0 + a.jchunk);
  if (WS > 1) {
    const int q = (j1 - j0 + WS - 1) / WS;
    const int w0 = min(j1, j0 + wave * q);
    j1 = min(j1, w0 + q);
    j0 = w0;
  }
  const T eps2 = (T)a.eps2;

  double acc[NFO][IPT];
#pragma unroll
  for (int f = 0; f < NFO; ++f)
#pragma unroll
    for (int ii = 0; ii < IPT; ++ii) acc[f][ii] = 0.0;

  PairAcc<T, IPT> A;
  if constexpr (sizeof(T) != 4) {
    A.zero();
    pair_segment<T, MODE, IPT>(pk, j0, j1, ilo, ihi, eps2, I, A);
    acc_flush(A, acc);
  } else {
    for (int t0 = j0; t0 < j1; t0 += kTile) {
      const int t1 = min(j1, t0 + kTile);
      A.zero();
      pair_segment<T, MODE, IPT>(pk, t0, t1, ilo, ihi, eps2, I, A);
      acc_flush(A, acc);
    }
  }

  const size_t plane = (size_t)a.Ns;
  double* out = a.part + (size_t)sp * NFO * plane;
  if constexpr (WS == 1) {
#pragma unroll
    for (int ii = 0; ii < IPT; ++ii) {
      if (I.idx[ii] < a.Ns) {
#pragma unroll
        for (int f = 0; f < NFO; ++f)
          if (field_written(f, MODE)) out[f * plane + I.idx[ii]] = acc[f][ii];
      }
    }
  } else {
    // fixed-order reduction over the WS wavefronts: waves 1..WS-1 park their
    // sums in LDS, wave 0 adds them to its own in wave order and stores
    // (LDS of WS-1 waves only, so it does not cap the occupancy).  WS = 8:
    // first wave w < 4 adds wave w + 4's sums to its own.
    if constexpr (WS == 8) {
      if (wave >= 4) {
#pragma unroll
        for (int f = 0; f < NFO; ++f)
#pragma unroll
          for (int ii = 0; ii < IPT; ++ii)
            red[(((wave - 4) * NFO + f) * IPT + ii) * 64 + lane] = acc[f][ii];
      }
      __syncthreads();
      if (wave < 4) {
#pragma unroll
        for (int f = 0; f < NFO; ++f)
#pragma unroll
          for (int ii = 0; ii < IPT; ++ii)
            acc[f][ii] += red[((wave * NFO + f) * IPT + ii) * 64 + lane];
      }
      __syncthreads();
    }
    if (wave > 0 && wave < 4) {
#pragma unroll
      for (int f = 0; f < NFO; ++f)
#pragma unroll
        for (int ii = 0; ii < IPT; ++ii)
          red[(((wave - 1) * NFO + f) * IPT + ii) * 64 + lane] = acc[f][ii];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int ii = 0; ii < IPT; ++ii) {
        const int idx = ilo + lane + ii * 64;
        if (idx < a.Ns) {
#pragma unroll
          for (int f = 0; f < NFO; ++f) {
            if (field_written(f, MODE)) {
              double sum = acc[f][ii];
#pragma unroll
              for (int w = 1; w < 4; ++w) sum += red[(((w - 1) * NFO + f) * IPT + ii) * 64 + lane];
              out[f * plane + idx] = sum;
            }
          }
        }
      }
    }
  }
}

template <typename T, int MODE, int IPT, int WS>
__global__ __launch_bounds__(pair_threads<WS>()) void k_pair(PairArgs a) {
  __shared__ double red[pair_red_doubles<T, IPT, WS>()];
  pair_block<T, MODE, IPT, WS>(a, blockIdx.x, blockIdx.y, red);
}

// ---------------------------------------------------------------------------
// Epilogue (per star) and final step (massive object).
// ---------------------------------------------------------------------------
struct EpiArgs {
  const double* pos;  // [N][3] state of this evaluation
  const double* vel;  // [N][3] (may be nullptr when newton_only)
  const double* mass;
  int Ns;
  double G, lam, eps2;
  const double* ub;     // [Ns][4 W]
  const double* bpart;  // prologue partials [nbpro][8 W]
  int nbpro;
  const double* part;  // pair partials [nsplit][kNF W][Ns]
  int nsplit;
  int newton_only;      // skip every 1PN term
  const double* phi_in; // correction mode: Newtonian potential of all N bodies (else nullptr)
  const double* accN_in;// correction mode: Newtonian acceleration of all N bodies
  double* acc_newton;   // outputs, [N][3] / [N] (any may be nullptr)
  double* phi;
  double* acc_1pn;
  double* bhpart;  // [gridDim.x][4 W]: the massive object's 1PN sum, block partials
  int nbepi;       // (k_bh_final) number of bhpart rows
  int* status;
  // Runge-Kutta stage update (stage < 0: none)
  int stage;
  double dt;
  double *X, *V, *Xs, *Vs, *KX, *KV;  // [N][3]
  double* acc_tot = nullptr;  // total acceleration [N][3] (optional)
  // jerk evaluation (S = Dual): derivatives of pos and vel, and the jerk [N][3]
  const double* pos_d = nullptr;
  const double* vel_d = nullptr;
  double* jerk = nullptr;
  // Hermite update (herm < 0: none, 0: first evaluation, 1: evaluation at
  // the predicted state): acceleration and jerk kept between steps, and the
  // next predicted state, all [N][3]
  int herm = -1;
  double *HA = nullptr, *HJ = nullptr, *XP = nullptr, *VP = nullptr;
  // chained Runge-Kutta stages (k_epilogue_chain): the next evaluation's
  // packets, u/b rows and block-sum rows (one per epilogue workgroup)
  void* pk_next = nullptr;
  double* ub_next = nullptr;
  double* bpart_next = nullptr;
};

// Classical RK4 bookkeeping for one body component.  The evaluation state of
// stage 0 is (X, V); of stages 1-3 it is (Xs, Vs).  KX/KV accumulate
// k1 + 2 k2 + 2 k3; stage 3 applies y += dt/6 (k1 + 2 k2 + 2 k3 + k4).
// rk4_next gives the component of the next evaluation state (stage 3: the new
// step's state) from the stage derivative k and the step-start value Y; the
// same function serves position and velocity, and the epilogue uses it for
// the massive object's next position too, so that every thread derives that
// position bit for bit as k_bh_final does.
__device__ __forceinline__ double rk4_next(int stage, double dt, double Y, double K, double k) {
  switch (stage) {
    case 0:
    case 1:
      return Y + 0.5 * dt * k;
    case 2:
      return Y + dt * k;
    default:
      return Y + dt / 6.0 * (K + k);
  }
}
// A kernel-argument pointer the compiler may not trace back to its field:
// otherwise it merges stores through X or Xs into one store through a pointer
// selected from a copy of the arguments in scratch memory.
__device__ __forceinline__ double* uniform_ptr(double* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// The step-start state (X, V) and the accumulated stage sums (KX, KV) of one
// body component, read ahead of their use (a kernel requests all its global
// reads up front so that their latencies overlap).
struct Rk4In {
  double X = 0.0, V = 0.0, KX = 0.0, KV = 0.0;
};
__device__ __forceinline__ Rk4In rk4_load(const EpiArgs& a, size_t o) {
  Rk4In r;
  if (a.stage < 0 || a.stage > 3) return r;
  r.X = a.X[o];
  r.V = a.V[o];
  if (a.stage > 0) {
    r.KX = a.KX[o];
    r.KV = a.KV[o];
  }
  return r;
}
// xv: velocity of the evaluation state (the position derivative k_x); returns
// the next evaluation state's position and velocity component in xn, vn.
__device__ __forceinline__ void rk4_update(const EpiArgs& a, size_t o, const Rk4In& in,
                                           double xv, double acc, double& xn, double& vn) {
  if (a.stage < 0 || a.stage > 3) return;
  const double KX = in.KX, KV = in.KV;
  xn = rk4_next(a.stage, a.dt, in.X, KX, xv);
  vn = rk4_next(a.stage, a.dt, in.V, KV, acc);
  if (a.stage < 3) {
    a.KX[o] = a.stage == 0 ? xv : KX + 2.0 * xv;
    a.KV[o] = a.stage == 0 ? acc : KV + 2.0 * acc;
    uniform_ptr(a.Xs)[o] = xn;
    uniform_ptr(a.Vs)[o] = vn;
  } else {
    uniform_ptr(a.X)[o] = xn;
    uniform_ptr(a.V)[o] = vn;
  }
}

// Fourth-order Hermite bookkeeping for one body component, from the
// acceleration ap and jerk jp of the evaluation state.  herm 0 (state
// (X, V)): keeps a = ap, j = jp; snap and crackle are zero.  herm 1 (state
// (XP, VP), the prediction): corrector
//   v' = v + (a + ap) dt/2 + (j - jp) dt^2/12,
//   x' = x + (v + v') dt/2 + (a - ap) dt^2/12,
// snap and crackle at the step's end from the Hermite interpolant of a,
//   k = (12 (a - ap) + 6 dt (j + jp)) / dt^3,
//   s = (-6 (a - ap) - dt (4 j + 2 jp)) / dt^2 + k dt,
// then a = ap, j = jp.  Both cases predict the next evaluation state
//   XP = x + v dt + a dt^2/2 + j dt^3/6 + s dt^4/24 + k dt^5/120,
//   VP = v + a dt + j dt^2/2 + s dt^3/6 + k dt^4/24.
// (The velocity-dependent 1PN force is why the predictor carries s and k: a
// velocity predicted to O(dt^3) only would cap the scheme at third order.)
__device__ __forceinline__ void hermite_update(const EpiArgs& a, size_t o, double ap, double jp) {
  const double dt = a.dt, dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
  double x = a.X[o], v = a.V[o], sn = 0.0, cr = 0.0;
  if (a.herm == 1) {
    const double a0 = a.HA[o], j0 = a.HJ[o];
    const double vn = v + dt / 2.0 * (a0 + ap) + dt2 / 12.0 * (j0 - jp);
    x = x + dt / 2.0 * (v + vn) + dt2 / 12.0 * (a0 - ap);
    v = vn;
    cr = (12.0 * (a0 - ap) + 6.0 * dt * (j0 + jp)) / dt3;
    sn = (-6.0 * (a0 - ap) - dt * (4.0 * j0 + 2.0 * jp)) / dt2 + cr * dt;
    a.X[o] = x;
    a.V[o] = v;
  }
  a.HA[o] = ap;
  a.HJ[o] = jp;
  a.XP[o] = x + dt * v + dt2 / 2.0 * ap + dt3 / 6.0 * jp + dt4 / 24.0 * sn + dt5 / 120.0 * cr;
  a.VP[o] = v + dt * ap + dt2 / 2.0 * jp + dt3 / 6.0 * sn + dt4 / 24.0 * cr;
}

// The massive object's acceleration A0 = a^N_0, potential magnitude V0 = -phi_0
// and the star momentum P, from the prologue partials (or the caller's inputs).
template <typename S>
constexpr int bh_cols() { return IsDual<S>::value ? 16 : 7; }  // columns read per prologue row

// rows: this thread's partial sums of the prologue rows (rows_load)
template <typename S>
__device__ __forceinline__ void bh_quantities(const EpiArgs& a,
                                              const double (&rows)[bh_cols<S>()], S (&A0)[3],
                                              S& V0, S (&P)[3]) {
  constexpr int K = bh_cols<S>();
  double r[K];
  rows_sum<K>(rows, r);
  const double iM = 1.0 / a.mass[0];  // one division for the four quotients
  A0[0] = get<S>(r, 0, 8) * iM;
  A0[1] = get<S>(r, 1, 8) * iM;
  A0[2] = get<S>(r, 2, 8) * iM;
  V0 = get<S>(r, 3, 8) * iM;
  P[0] = get<S>(r, 4, 8);
  P[1] = get<S>(r, 5, 8);
  P[2] = get<S>(r, 6, 8);
  if constexpr (!IsDual<S>::value) {
    if (a.phi_in) {
      V0 = -a.phi_in[0];
      A0[0] = a.accN_in[0];
      A0[1] = a.accN_in[1];
      A0[2] = a.accN_in[2];
    }
  }
}

constexpr int kEpiStars = 64;  // stars per epilogue workgroup (4 threads per star reduce the splits)

__device__ __forceinline__ bool epi_field_used(int f, const EpiArgs& a) {
  f %= kNF;
  if (f == F_U) return a.phi_in == nullptr;  // correction mode: U is not computed
  if (f < F_Q) return true;
  return !a.newton_only;
}

// S = double: the evaluation; S = Dual: the same arithmetic on dual numbers
// (acceleration and jerk).  PkT (S = double only): also the next sweep's
// prologue into pk_next, ub_next and bpart_next (packets of PkOf<PkT>):
// double / float, a Runge-Kutta stage's, from each star's next state and the
// massive object's next position; Dual, the jerk sweep's at this state, with
// the derivatives (v, a) of (x, v) from the acceleration just computed.
// void: none.
// The massive object's state at an evaluation, for an epilogue whose kernel
// computes it (the one-launch Runge-Kutta stage) instead of reading it.
struct BhStage {
  double x0[3];  // evaluation position
  double X[3];   // step-start position
  double KX[3];  // stage sum of its velocities through the previous stage
  double v[3];   // evaluation velocity
};

// The epilogue of NSTAR stars (blk * NSTAR ...), from the prologue rows `rows`
// (this thread's rows_load).  OWNBH = false: the stars' pair sums are the
// nsplit partials in a.part, the massive object's state is read from a.pos,
// a.X, a.KX, a.vel.  OWNBH = true (S = double only): the caller has put the
// pair sums in fsum[field][NSTAR] and passes the massive object's state in own.
template <typename S, typename PkT, int NSTAR, bool OWNBH>
__device__ __forceinline__ void epilogue_rows(const EpiArgs& a, int blk, double* lds,
                                              double* fsum, const double (&rows)[bh_cols<S>()],
                                              const BhStage& own) {
  constexpr bool DUAL = IsDual<S>::value;
  constexpr int W = DUAL ? 2 : 1;
  constexpr int NFO = kNF * W;
  static_assert(NSTAR <= 64, "the stars of a workgroup are in its first wavefront");
  static_assert(OWNBH || NSTAR == kEpiStars, "the split reduction takes 4 threads per star");
  static_assert(!OWNBH || (!DUAL && !std::is_void<PkT>::value), "own state: chained FP64 epilogue");
  // Every global read of the workgroup is requested before the first wait:
  // the prologue rows (by the caller), the pair partials, the star's own
  // inputs and Runge-Kutta state, the massive object's state.  (At small N
  // this kernel is a chain of memory latencies; issued in order, they added
  // up.)
  const double M = a.mass[0];
  S x0, y0, z0;
  if constexpr (OWNBH) {
    x0 = own.x0[0];
    y0 = own.x0[1];
    z0 = own.x0[2];
  } else {
    x0 = ld<S>(a.pos, a.pos_d, 0);
    y0 = ld<S>(a.pos, a.pos_d, 1);
    z0 = ld<S>(a.pos, a.pos_d, 2);
  }
  const int k = blk * NSTAR + threadIdx.x;
  const bool star = threadIdx.x < NSTAR && k < a.Ns;
  const int i = k + 1;
  S ui = 0.0, bx = 0.0, by = 0.0, bz = 0.0, xi = 0.0, yi = 0.0, zi = 0.0;
  S vi[3] = {0.0, 0.0, 0.0};
  double m_s = 0.0;  // the star's mass (G m is formed where it is used, after the loads)
  Rk4In rk[3];
  // the massive object's step-start position, stage sum and velocity (uniform:
  // scalar loads)
  double bh_x[3] = {0.0, 0.0, 0.0}, bh_kx[3] = {0.0, 0.0, 0.0}, bh_v[3] = {0.0, 0.0, 0.0};
  if constexpr (OWNBH) {
    for (int c = 0; c < 3; ++c) {
      bh_x[c] = own.X[c];
      bh_kx[c] = a.stage == 0 ? 0.0 : own.KX[c];
      bh_v[c] = own.v[c];
    }
  } else if constexpr (!DUAL && !std::is_void<PkT>::value) {
    if (a.stage >= 0) {
      for (int c = 0; c < 3; ++c) {
        bh_x[c] = a.X[c];
        bh_kx[c] = a.stage == 0 ? 0.0 : a.KX[c];
        bh_v[c] = a.vel[c];
      }
    }
  }
  if (star) {
    const double* ub = a.ub + 4 * W * (size_t)k;
    ui = get<S>(ub, 0, 4);
    bx = get<S>(ub, 1, 4);
    by = get<S>(ub, 2, 4);
    bz = get<S>(ub, 3, 4);
    xi = ld<S>(a.pos, a.pos_d, 3 * i);
    yi = ld<S>(a.pos, a.pos_d, 3 * i + 1);
    zi = ld<S>(a.pos, a.pos_d, 3 * i + 2);
    if (!a.newton_only) {
      vi[0] = ld<S>(a.vel, a.vel_d, 3 * i);
      vi[1] = ld<S>(a.vel, a.vel_d, 3 * i + 1);
      vi[2] = ld<S>(a.vel, a.vel_d, 3 * i + 2);
      m_s = a.mass[i];
    }
    if constexpr (!DUAL) {
      for (int c = 0; c < 3; ++c) rk[c] = rk4_load(a, 3 * (size_t)i + c);
    }
  }

  // split reduction: thread (g, l) sums fields g, g+4, g+8, ... of star l, in
  // split order; the loads of up to 8 (dual: 4) splits of all its fields are
  // issued together, then added in order
  if constexpr (!OWNBH) {
    constexpr int FPT = (NFO + 3) / 4;      // fields per thread
    constexpr int BATCH = DUAL ? 4 : 8;     // splits per batch of loads
    const int g = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int kk = blk * kEpiStars + l;
    if (kk < a.Ns) {
      const size_t plane = (size_t)a.Ns;
      const size_t sstride = (size_t)NFO * plane;
      double sum[FPT];
      bool use[FPT];
#pragma unroll
      for (int fi = 0; fi < FPT; ++fi) {
        const int f = g + 4 * fi;
        sum[fi] = 0.0;
        use[fi] = f < NFO && epi_field_used(f, a);
      }
      const double* src = a.part + (size_t)g * plane + kk;
      int sp = 0;
      for (; sp + BATCH <= a.nsplit; sp += BATCH) {
        double v[FPT][BATCH];
#pragma unroll
        for (int fi = 0; fi < FPT; ++fi)
#pragma unroll
          for (int q = 0; q < BATCH; ++q)
            v[fi][q] = use[fi] ? src[(size_t)4 * fi * plane + (size_t)(sp + q) * sstride] : 0.0;
#pragma unroll
        for (int fi = 0; fi < FPT; ++fi)
#pragma unroll
          for (int q = 0; q < BATCH; ++q) sum[fi] += v[fi][q];
      }
      if (sp < a.nsplit) {  // the remaining splits, also in one batch
        double v[FPT][BATCH];
#pragma unroll
        for (int fi = 0; fi < FPT; ++fi)
#pragma unroll
          for (int q = 0; q < BATCH; ++q)
            v[fi][q] = (use[fi] && sp + q < a.nsplit)
                           ? src[(size_t)4 * fi * plane + (size_t)(sp + q) * sstride]
                           : 0.0;
#pragma unroll
        for (int fi = 0; fi < FPT; ++fi)
#pragma unroll
          for (int q = 0; q < BATCH; ++q)
            if (sp + q < a.nsplit) sum[fi] += v[fi][q];
      }
#pragma unroll
      for (int fi = 0; fi < FPT; ++fi)
        if (g + 4 * fi < NFO) fsum[(g + 4 * fi) * kEpiStars + l] = sum[fi];
    }
  }
  if constexpr (!OWNBH) __syncthreads();  // fsum complete (the caller orders its own)
  S A0[3], V0, P[3];
  bh_quantities<S>(a, rows, A0, V0, P);
  const double gM = a.G * M;
  const double iM = 1.0 / M;
  const S w[3] = {-(P[0] * iM), -(P[1] * iM), -(P[2] * iM)};

  constexpr bool CHAIN = !std::is_void<PkT>::value;
  constexpr bool JNEXT = std::is_same<PkT, Dual>::value;  // the jerk sweep's packets
  constexpr int NP = JNEXT ? 14 : 7;  // block-sum terms of the next prologue
  static_assert(!CHAIN || !DUAL, "chained epilogues are FP64 evaluations");
  S bh[3] = {0.0, 0.0, 0.0};
  double pro[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) pro[q] = 0.0;
  if (star) {
    const int t = threadIdx.x;
    S sum[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) {
      if constexpr (DUAL) sum[f] = S(fsum[f * NSTAR + t], fsum[(kNF + f) * NSTAR + t]);
      else sum[f] = fsum[f * NSTAR + t];
    }
    sum[F_C2] *= kSqrt32;  // the sweep accumulates D'/sqrt(3/2)
    // Newtonian part: g_i - b_i with g_i = -G_i
    const S aN[3] = {-sum[F_G] - bx, -sum[F_G + 1] - by, -sum[F_G + 2] - bz};
    S Vi = sum[F_U] + ui;  // -phi_i
    S a1[3] = {0.0, 0.0, 0.0};
    if (!a.newton_only) {
      const S vi2 = vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2];
      S Vphi = Vi;
      S aNs[3] = {aN[0], aN[1], aN[2]};
      if constexpr (!DUAL) {
        if (a.phi_in) {  // correction mode: the caller's potential and Newtonian acceleration
          Vphi = -a.phi_in[i];
          aNs[0] = a.accN_in[3 * i];
          aNs[1] = a.accN_in[3 * i + 1];
          aNs[2] = a.accN_in[3 * i + 2];
        }
      }
      // Eq. (6) star-star terms: S_i0 G_i + Q_i + C2_i v_i + 7 Q7_i, S_i0 = -v_i^2 + 4 u_i
      const S Si0 = -vi2 + 4.0 * ui;
      S q[3];
      for (int c = 0; c < 3; ++c)
        q[c] = Si0 * sum[F_G + c] + sum[F_Q + c] + sum[F_C2] * vi[c] + 7.0 * sum[F_Q7 + c];
      // massive-object partner (Eq. (5) and the G^2 m M / velocity terms of Eq. (6))
      const S d0[3] = {xi - x0, yi - y0, zi - z0};
      const S rinv0 = rsqrt_t(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2] + a.eps2);
      const S n0[3] = {d0[0] * rinv0, d0[1] * rinv0, d0[2] * rinv0};
      const S kk = gM * rinv0 * rinv0;
      const S vw = vi[0] * w[0] + vi[1] * w[1] + vi[2] * w[2];
      const S dA = d0[0] * A0[0] + d0[1] * A0[1] + d0[2] * A0[2];
      const S br = -vi2 + 4.0 * vw + 4.0 * Vphi + V0 + 0.5 * dA;
      const S n4v = 4.0 * (n0[0] * vi[0] + n0[1] * vi[1] + n0[2] * vi[2]);
      const S nw = n0[0] * w[0] + n0[1] * w[1] + n0[2] * w[2];
      const S g7 = 3.5 * gM * rinv0;
      for (int c = 0; c < 3; ++c) {
        const S B = kk * (br * n0[c] + n4v * (vi[c] - w[c]) - 3.0 * nw * vi[c]) + g7 * A0[c];
        a1[c] = a.lam * (B + q[c]);
      }
      // this star's term of the massive object's 1PN sum (Eqs. (2)-(3))
      const S Vs = Vphi;
      const double gm_s = a.G * m_s;
      const S ks = gm_s * rinv0 * rinv0;
      const S n0s[3] = {-n0[0], -n0[1], -n0[2]};
      const S d0s[3] = {-d0[0], -d0[1], -d0[2]};
      const S nvs = n0s[0] * vi[0] + n0s[1] * vi[1] + n0s[2] * vi[2];
      const S dAs = d0s[0] * aNs[0] + d0s[1] * aNs[1] + d0s[2] * aNs[2];
      const S brs = -2.0 * vi2 + 4.0 * vw + 1.5 * nvs * nvs + 4.0 * V0 + Vs + 0.5 * dAs;
      const S nws = n0s[0] * w[0] + n0s[1] * w[1] + n0s[2] * w[2];
      const S g7s = 3.5 * gm_s * rinv0;
      for (int c = 0; c < 3; ++c)
        bh[c] = ks * (brs * n0s[c] + 3.0 * nvs * vi[c] - 3.0 * nvs * w[c] - 4.0 * nws * vi[c]) +
                g7s * aNs[c];
    }
    if (a.acc_newton) {
      a.acc_newton[3 * i] = val(aN[0]);
      a.acc_newton[3 * i + 1] = val(aN[1]);
      a.acc_newton[3 * i + 2] = val(aN[2]);
    }
    if (a.phi) a.phi[i] = -val(Vi);
    if (a.acc_1pn) {
      a.acc_1pn[3 * i] = val(a1[0]);
      a.acc_1pn[3 * i + 1] = val(a1[1]);
      a.acc_1pn[3 * i + 2] = val(a1[2]);
    }
    const S at[3] = {aN[0] + a1[0], aN[1] + a1[1], aN[2] + a1[2]};
    if (a.acc_tot) {
      for (int c = 0; c < 3; ++c) a.acc_tot[3 * i + c] = val(at[c]);
    }
    if (!finite_s(at[0]) || !finite_s(at[1]) || !finite_s(at[2])) atomicOr(a.status, 1);
    if constexpr (DUAL) {
      if (a.jerk) {
        for (int c = 0; c < 3; ++c) a.jerk[3 * i + c] = at[c].d;
      }
      if (a.herm >= 0) {
        for (int c = 0; c < 3; ++c) hermite_update(a, 3 * (size_t)i + c, at[c].v, at[c].d);
      }
    } else {
      if constexpr (JNEXT) {
        // the jerk sweep's prologue terms of this star (as k_prologue<Dual>
        // computes them from pos_d = vel, vel_d = the acceleration)
        const Dual x0d[3] = {Dual(x0, a.vel[0]), Dual(y0, a.vel[1]), Dual(z0, a.vel[2])};
        const Dual xsd[3] = {Dual(xi, vi[0]), Dual(yi, vi[1]), Dual(zi, vi[2])};
        const Dual vsd[3] = {Dual(vi[0], at[0]), Dual(vi[1], at[1]), Dual(vi[2], at[2])};
        Dual pd[7];
        star_terms<Dual, Dual>(x0d, xsd, vsd, a.mass[i], a.G, gM, a.eps2, a.pk_next, a.ub_next, k,
                               pd);
#pragma unroll
        for (int q = 0; q < 7; ++q) {
          pro[q] = pd[q].v;
          pro[7 + q] = pd[q].d;
        }
      }
      if (a.stage >= 0) {
        double xn[3] = {0.0, 0.0, 0.0}, vn[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 3; ++c)
          rk4_update(a, 3 * (size_t)i + c, rk[c], vi[c], at[c], xn[c], vn[c]);
        if constexpr (CHAIN && !JNEXT) {
          // the massive object's next position, as k_bh_final will compute it
          double x0n[3];
          for (int c = 0; c < 3; ++c) x0n[c] = rk4_next(a.stage, a.dt, bh_x[c], bh_kx[c], bh_v[c]);
          star_terms<PkT, double>(x0n, xn, vn, a.mass[i], a.G, gM, a.eps2, a.pk_next, a.ub_next,
                                  k, pro);
        }
      }
    }
  }
  constexpr int NB = CHAIN ? 3 + NP : 3 * W;
  double bhs[NB];
#pragma unroll
  for (int c = 0; c < 3; ++c) put(bhs, c, 3, bh[c]);
  if constexpr (CHAIN) {
#pragma unroll
    for (int q = 0; q < NP; ++q) bhs[3 + q] = pro[q];
  }
  // the stars are in wavefront 0: it sums its rows (wave_allsum, every lane
  // then holds every sum) and writes them from its registers
  if (wave_id() == 0) {
    wave_allsum<NB>(bhs);
    const int l = threadIdx.x;
    if (l < 4 * W) {
      // row layout: values in columns 0..2, derivatives in 4..6 (Dual)
      const int q = l & 3, h = l >> 2;
      a.bhpart[(size_t)blk * 4 * W + l] = q < 3 ? pick(bhs, h * 3 + q) : 0.0;
    }
    if constexpr (CHAIN) {
      // the prologue's row layout: sum m b (3), sum m u, sum m v (3), 0 (and
      // the same 8 columns of derivatives for the jerk sweep)
      constexpr int RW = JNEXT ? 16 : 8;
      if (l >= 32 && l < 32 + RW) {
        const int c = l - 32, q = c & 7, h = c >> 3;
        a.bpart_next[(size_t)blk * RW + c] = q < 7 ? pick(bhs, 3 + h * 7 + q) : 0.0;
      }
    }
  }
}

template <typename S, typename PkT = void>
__device__ __forceinline__ void epilogue_block(const EpiArgs& a, int blk, double* lds,
                                               double* fsum) {
  double rows[bh_cols<S>()];
  rows_load<bh_cols<S>()>(a.bpart, a.nbpro, IsDual<S>::value ? 16 : 8, rows);
  epilogue_rows<S, PkT, kEpiStars, false>(a, blk, lds, fsum, rows, BhStage{});
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_epilogue(EpiArgs a) {
  __shared__ double lds[(IsDual<S>::value ? 16 : 7) * kBlock];
  __shared__ double fsum[kNF * Width<S>::n * kEpiStars];
  epilogue_block<S>(a, blockIdx.x, lds, fsum);
}

// FP64 epilogue that also performs the next sweep's prologue (packets of
// PkOf<T>; T = Dual: the jerk sweep at this state), saving that kernel.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_epilogue_chain(EpiArgs a) {
  __shared__ double lds[(std::is_same<T, Dual>::value ? 17 : 10) * kBlock];
  __shared__ double fsum[kNF * kEpiStars];
  epilogue_block<double, T>(a, blockIdx.x, lds, fsum);
}

template <typename S>
__device__ __forceinline__ void bh_final_block(const EpiArgs& a, double* lds) {
  constexpr bool DUAL = IsDual<S>::value;
  constexpr int W = DUAL ? 2 : 1;
  // both row sets and the massive object's own state are requested before
  // the first wait (see epilogue_block)
  double rows[bh_cols<S>()], rows1[4 * W - 1];  // 1PN rows: columns 0..2 (4..6: derivatives)
  rows_load<bh_cols<S>()>(a.bpart, a.nbpro, DUAL ? 16 : 8, rows);
  if (!a.newton_only) rows_load<4 * W - 1>(a.bhpart, a.nbepi, 4 * W, rows1);
  // thread c < 3 finishes component c: its velocity and Runge-Kutta state
  const int cc = threadIdx.x;
  S v0c = 0.0;
  Rk4In rkc;
  if (cc < 3) {
    if (!a.newton_only) v0c = ld<S>(a.vel, a.vel_d, cc);
    if constexpr (!DUAL) rkc = rk4_load(a, (size_t)cc);
  }
  S A0[3], V0, P[3];
  bh_quantities<S>(a, rows, A0, V0, P);
  S T[3] = {0.0, 0.0, 0.0};
  if (!a.newton_only) {
    double r[4 * W - 1];
    rows_sum<4 * W - 1>(rows1, r);
    for (int c = 0; c < 3; ++c) T[c] = get<S>(r, c, 4);
  }
  // component c of the massive object's outputs and update (c a constant in
  // each call below, so that nothing is indexed at run time)
  auto finish = [&](int c, const S& A0c, const S& Tc) {
    const S a1c = a.lam * Tc;
    const S atc = A0c + a1c;
    if (a.acc_newton) a.acc_newton[c] = val(A0c);
    if (a.phi && c == 0) a.phi[0] = -val(V0);
    if (a.acc_1pn) a.acc_1pn[c] = val(a1c);
    if (a.acc_tot) a.acc_tot[c] = val(atc);
    if (!finite_s(atc)) atomicOr(a.status, 1);
    if constexpr (DUAL) {
      if (a.jerk) a.jerk[c] = atc.d;
      if (a.herm >= 0) hermite_update(a, (size_t)c, atc.v, atc.d);
    } else {
      if (a.stage >= 0) {
        double xn, vn;
        rk4_update(a, (size_t)c, rkc, v0c, atc, xn, vn);
      }
    }
  };
  if (cc == 0) finish(0, A0[0], T[0]);
  else if (cc == 1) finish(1, A0[1], T[1]);
  else if (cc == 2) finish(2, A0[2], T[2]);
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_bh_final(EpiArgs a) {
  __shared__ double lds[(IsDual<S>::value ? 16 : 7) * kBlock];
  bh_final_block<S>(a, lds);
}

// The jerk evaluation's dual epilogue with the FP64 pass's massive-object
// update (k_bh_final<double>'s work) in one extra workgroup: the dual
// epilogue reads neither the massive object's FP64 acceleration nor the FP64
// partial rows (its own rows are in separate buffers).
__global__ __launch_bounds__(kBlock) void k_epilogue_dual_bh(EpiArgs a, EpiArgs e) {
  __shared__ double lds[16 * kBlock];
  __shared__ double fsum[kNF * 2 * kEpiStars];
  if (blockIdx.x == gridDim.x - 1) {
    bh_final_block<double>(e, lds);
    return;
  }
  epilogue_block<Dual>(a, blockIdx.x, lds, fsum);
}

// The sweep of a chained Runge-Kutta stage with the previous stage's
// massive-object update (k_bh_final's work) in one extra workgroup: the sweep
// reads only star packets, which the previous epilogue has written, so the
// two are independent and the stage saves a kernel boundary.  Grid: the
// sweep's (iblocks + 1) x nsplit; column iblocks, split 0 runs the update
// (sharing the sweep's LDS), the rest of that column exits.
template <typename T, int MODE, int IPT, int WS>
__global__ __launch_bounds__(pair_threads<WS>()) void k_pair_bh(PairArgs a, EpiArgs e) {
  constexpr int L = pair_red_doubles<T, IPT, WS>() > 7 * kBlock ? pair_red_doubles<T, IPT, WS>()
                                                                : 7 * kBlock;
  __shared__ double lds[L];
  if (blockIdx.x == gridDim.x - 1) {
    if (blockIdx.y == 0) bh_final_block<double>(e, lds);
    return;
  }
  pair_block<T, MODE, IPT, WS>(a, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// Small systems: one launch per Runge-Kutta stage.  With a few hundred bodies
// a stage is a chain of latencies (launch, loads, reductions, dependent FP64
// arithmetic) rather than work, and one kernel per stage saves a launch and
// the split partials' trip through memory: a workgroup owns NS stars and
// sums all their j in its own 256 lanes (lane sl + NS q takes star sl and
// j = q, q + 256/NS, ...), reduces them in fixed order (a butterfly within
// each wavefront, then the four wavefronts) and runs those stars' epilogue.  No other workgroup's partials are needed, so
// nothing waits across workgroups.  The massive object's update of the
// previous stage needs every epilogue's rows; each workgroup computes it
// itself from the rows the previous launch wrote (the same sums in the same
// order, so the same bits everywhere), and workgroup 0 stores it.  Every
// buffer a stage reads is one no workgroup of that stage writes: packets, u/b
// rows and massive-object 1PN rows alternate between two buffers, block rows
// rotate through four (a stage reads its own and the previous stage's), and
// the massive object's state alternates between two copies of
// (X, V, Xs, Vs, KX, KV).
// ---------------------------------------------------------------------------
constexpr int kStageFirst = 0;  // the first stage of a call: no pending update
constexpr int kStageFull = 1;   // pending update, sweep and epilogue
constexpr int kStageFinal = 2;  // the last pending update only (one workgroup)

struct StageArgs {
  EpiArgs e;             // this stage's epilogue; e.nbpro rows in every row buffer
  const void* pk;        // this stage's packets (PkOf<T>)
  int mode;
  int pstage;            // stage of the pending massive-object update
  const double* prow;    // its block rows [e.nbpro][8]
  const double* phrow;   // its massive-object 1PN rows [e.nbpro][4]
  const double* bhs_in;  // the massive object's X, V, Xs, Vs, KX, KV before that update
  double* bhs_out;       // ... after it
};

// The stars' pair sums of one workgroup (lanes of star sl: sl + NS q).
template <typename T, int NS>
__device__ __forceinline__ void stage_sweep(const StageArgs& sa, double (&acc)[kNF][1]) {
  using Pk = typename PkOf<T>::type;
  constexpr int Q = kBlock / NS;
  const Pk* __restrict__ pk = static_cast<const Pk*>(sa.pk);
  const int Ns = sa.e.Ns;
  const int sl = threadIdx.x % NS, q = threadIdx.x / NS;
  PairI<T, 1> I;
  I.idx[0] = blockIdx.x * NS + sl;
  {
    const Pk& p = pk[min(I.idx[0], Ns - 1)];  // lanes past the end compute on a copy, never stored
    I.x[0] = p.x;
    I.y[0] = p.y;
    I.z[0] = p.z;
    I.kx[0] = T(PairScale<T>::k) * (T)p.svx;
    I.ky[0] = T(PairScale<T>::k) * (T)p.svy;
    I.kz[0] = T(PairScale<T>::k) * (T)p.svz;
  }
  const T eps2 = (T)sa.e.eps2;
#pragma unroll
  for (int f = 0; f < kNF; ++f) acc[f][0] = 0.0;
  PairAcc<T, 1> A;
  int j = q;
  while (j < Ns) {
    // FP32: partial sums over kTile of this lane's terms, then into FP64
    const int jend = sizeof(T) == 4 ? min(Ns, j + kTile * Q) : Ns;
    A.zero();
    for (; j + Q < jend; j += 2 * Q) {
      const Pk p0 = pk[j];
      const Pk p1 = pk[j + Q];
      pair_one<T, MODE_FUSED, 1, true>(p0, j, eps2, I, A);
      pair_one<T, MODE_FUSED, 1, true>(p1, j + Q, eps2, I, A);
    }
    if (j < jend) {
      pair_one<T, MODE_FUSED, 1, true>(pk[j], j, eps2, I, A);
      j += Q;
    }
    acc_flush(A, acc);
  }
}

// The pending update: the massive object's acceleration at stage sa.pstage
// from that stage's rows (as k_bh_final), then its Runge-Kutta bookkeeping (as
// rk4_update) on the state in bi.  Every thread ends with the result in out
// and the state of this stage's evaluation in own; workgroup 0 stores out (and
// the new step-start state after stage 3).
__device__ __forceinline__ void stage_bh_update(const StageArgs& sa, const double (&prows)[7],
                                                const double (&phrows)[3], const double (&bi)[18],
                                                double (&out)[18], BhStage& own) {
  const EpiArgs& a = sa.e;
  double A0[3], V0, P[3], r[3];
  bh_quantities<double>(a, prows, A0, V0, P);
  rows_sum<3>(phrows, r);
  const int ps = sa.pstage;
  bool finite = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double atc = A0[c] + a.lam * r[c];
    finite = finite && isfinite(atc);
    const double X = bi[c], V = bi[3 + c], vs = bi[9 + c], KX = bi[12 + c], KV = bi[15 + c];
    const double xn = rk4_next(ps, a.dt, X, KX, vs);
    const double vn = rk4_next(ps, a.dt, V, KV, atc);
    if (ps < 3) {
      out[c] = X;
      out[3 + c] = V;
      out[12 + c] = ps == 0 ? vs : KX + 2.0 * vs;
      out[15 + c] = ps == 0 ? atc : KV + 2.0 * atc;
    } else {
      out[c] = xn;
      out[3 + c] = vn;
      out[12 + c] = 0.0;
      out[15 + c] = 0.0;
    }
    out[6 + c] = xn;
    out[9 + c] = vn;
    own.x0[c] = xn;
    own.X[c] = out[c];
    own.KX[c] = out[12 + c];
    own.v[c] = vn;
  }
  if (blockIdx.x == 0) {
    const int t = threadIdx.x;
    if (t == 0 && !finite) atomicOr(a.status, 1);
#pragma unroll
    for (int c = 0; c < 18; ++c)
      if (t == c) sa.bhs_out[c] = out[c];
    if (ps == 3) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (t == 32 + c) uniform_ptr(a.X)[c] = out[c];
        if (t == 40 + c) uniform_ptr(a.V)[c] = out[3 + c];
      }
    }
  }
}

template <typename T, int NS>
__global__ __launch_bounds__(kBlock) void k_stage(StageArgs sa) {
  static_assert(kBlock == 256 && 64 % NS == 0 && NS * kNF <= kBlock, "stars per workgroup");
  __shared__ double red[kNF * 4 * NS];
  __shared__ double lds[10 * kBlock];
  __shared__ double fsum[kNF * NS];
  const EpiArgs& a = sa.e;
  const int t = threadIdx.x;
  const bool pend = sa.mode != kStageFirst;
  const bool eval = sa.mode != kStageFinal;
  // reads first: the pending update's rows and state, this stage's rows
  double prows[7], phrows[3], rows[7], bi[18];
  if (pend) {
    rows_load<7>(sa.prow, a.nbpro, 8, prows);
    rows_load<3>(sa.phrow, a.nbpro, 4, phrows);
#pragma unroll
    for (int c = 0; c < 18; ++c) bi[c] = sa.bhs_in[c];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bi[c] = bi[6 + c] = a.X[c];
      bi[3 + c] = bi[9 + c] = a.V[c];
      bi[12 + c] = bi[15 + c] = 0.0;
    }
  }
  if (eval) {
    rows_load<7>(a.bpart, a.nbpro, 8, rows);
    double acc[kNF][1];
    stage_sweep<T, NS>(sa, acc);
    // a star's lanes within a wavefront are NS apart: an xor butterfly over
    // distances NS ... 32 sums them (the same bits in each), and lane sl < NS
    // of wavefront w parks star sl's partial
#pragma unroll
    for (int m = NS; m < 64; m <<= 1) {
#pragma unroll
      for (int f = 0; f < kNF; ++f) acc[f][0] += __shfl_xor(acc[f][0], m, 64);
    }
    if ((t & 63) < NS) {
#pragma unroll
      for (int f = 0; f < kNF; ++f) red[(f * 4 + (t >> 6)) * NS + (t & 63)] = acc[f][0];
    }
  }
  BhStage own;
  if (pend) {
    double out[18];
    stage_bh_update(sa, prows, phrows, bi, out, own);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      own.x0[c] = own.X[c] = bi[c];
      own.KX[c] = 0.0;
      own.v[c] = bi[3 + c];
    }
    if (blockIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < 18; ++c)
        if (t == c) sa.bhs_out[c] = bi[c];
    }
  }
  if (!eval) return;
  __syncthreads();
  if (t < NS * kNF) {  // star sl, field f: the four wavefronts' partials in order
    const int sl = t % NS, f = t / NS;
    fsum[f * NS + sl] = ((red[(f * 4) * NS + sl] + red[(f * 4 + 1) * NS + sl]) +
                         red[(f * 4 + 2) * NS + sl]) + red[(f * 4 + 3) * NS + sl];
  }
  __syncthreads();
  epilogue_rows<double, T, NS, true>(a, blockIdx.x, lds, fsum, rows, own);
}

// A call's first packets, u/b rows and block rows in the stage kernel's
// layout (a block row per NS stars, reduced as its epilogue reduces them, so
// that a run resumed from a saved state repeats the continuous run bit for bit).
template <typename T, int NS>
__global__ __launch_bounds__(kBlock) void k_stage_head(EpiArgs a) {
  const int t = threadIdx.x, k = blockIdx.x * NS + t;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  if (t < NS && k < a.Ns) {
    const int s = k + 1;
    const double x0[3] = {a.pos[0], a.pos[1], a.pos[2]};
    const double xs[3] = {a.pos[3 * s], a.pos[3 * s + 1], a.pos[3 * s + 2]};
    const double vs[3] = {a.vel[3 * s], a.vel[3 * s + 1], a.vel[3 * s + 2]};
    star_terms<T, double>(x0, xs, vs, a.mass[s], a.G, a.G * a.mass[0], a.eps2, a.pk_next,
                          a.ub_next, k, v);
  }
  if (t < 64) {  // the stars are in wavefront 0 (as in the stage's epilogue)
    wave_allsum<7>(v);
    if (t < 8) a.bpart_next[(size_t)blockIdx.x * 8 + t] = t < 7 ? pick(v, t) : 0.0;
  }
  if (blockIdx.x == 0 && t == 0) {
    const double M = a.mass[0];
    if (!(M > 0.0) || !isfinite(M)) atomicOr(a.status, 2);
  }
}

// ---------------------------------------------------------------------------
// Diagnostics (Eqs. (7)-(8)).  Star-star pair sums per star i:
//   U_i = sum_j G m_j / R_ij
//   W_i = sum_j (G m_j / R_ij) [-7 v_i.v_j - (n_ij.v_i)(n_ij.v_j)]
//   Y_i = sum_j (G m_j / R_ij) (v_i.n_ij) n_ij
// then O(N) terms per star and fixed-order reductions.
// ---------------------------------------------------------------------------
constexpr int kND = 5;  // U, W, Y(3)

struct DiagPairArgs {
  const PkF64* pk;
  int Ns, jchunk;
  double eps2;
  double* part;  // [gridDim.y][kND][Ns]
};

__global__ __launch_bounds__(kBlock) void k_diag_pair(DiagPairArgs a) {
  const PkF64* __restrict__ pk = a.pk;
  const int ilo = blockIdx.x * kBlock;
  const int ihi = min(a.Ns, ilo + kBlock);
  const int i = ilo + threadIdx.x;
  const PkF64& pi = pk[min(i, a.Ns - 1)];
  const double xi = pi.x, yi = pi.y, zi = pi.z;
  constexpr double iv = PairScale<double>::inv_sv;
  const double vxi = iv * pi.svx, vyi = iv * pi.svy, vzi = iv * pi.svz;
  const int j0 = blockIdx.y * a.jchunk, j1 = min(a.Ns, j0 + a.jchunk);
  double U = 0.0, W = 0.0, Yx = 0.0, Yy = 0.0, Yz = 0.0;
  for (int j = j0; j < j1; ++j) {
    const PkF64& p = pk[j];
    const double dx = xi - p.x, dy = yi - p.y, dz = zi - p.z;
    double rinv = rsqrt_f64(fma(dz, dz, fma(dy, dy, fma(dx, dx, a.eps2))));
    if (j >= ilo && j < ihi) rinv = (j == i) ? 0.0 : rinv;
    const double mr = p.gm * rinv;
    const double rinv2 = rinv * rinv;
    const double vxj = iv * p.svx, vyj = iv * p.svy, vzj = iv * p.svz;
    const double vv = fma(vzi, vzj, fma(vyi, vyj, vxi * vxj));
    const double xvi = fma(dz, vzi, fma(dy, vyi, dx * vxi));
    const double xvj = fma(dz, vzj, fma(dy, vyj, dx * vxj));
    U += mr;
    W = fma(mr, fma(-xvi * xvj, rinv2, -7.0 * vv), W);
    const double cy = mr * xvi * rinv2;
    Yx = fma(cy, dx, Yx);
    Yy = fma(cy, dy, Yy);
    Yz = fma(cy, dz, Yz);
  }
  if (i < a.Ns) {
    const size_t plane = (size_t)a.Ns;
    double* out = a.part + (size_t)blockIdx.y * kND * plane + i;
    out[0] = U;
    out[plane] = W;
    out[2 * plane] = Yx;
    out[3 * plane] = Yy;
    out[4 * plane] = Yz;
  }
}

struct DiagEpiArgs {
  const double* pos;
  const double* vel;
  const double* mass;
  int Ns;
  double G, lam, eps2;
  const double* ub;
  const double* part;
  int nsplit;
  double* dpart;  // [gridDim.x][10]
  int ndpart;     // (k_diag_final) rows of dpart
  double* out8;   // (k_diag_final)
};

// Per-star contributions, columns of dpart:
//  0: 1/2 m v^2 - 1/2 m U - m u          (Newtonian energy, stars)
//  1: 1PN energy bracket, star terms
//  2: m u / M  (sum = U0 = sum_i G m_i / R_1i)
//  3-5: m v                               (Newtonian momentum, stars)
//  6-8: 1PN momentum bracket, star terms
__global__ __launch_bounds__(kBlock) void k_diag_epi(DiagEpiArgs a) {
  __shared__ double lds[9 * kBlock];
  const int k = blockIdx.x * kBlock + threadIdx.x;
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (k < a.Ns) {
    const int i = k + 1;
    const size_t plane = (size_t)a.Ns;
    double U = 0.0, W = 0.0, Y[3] = {0.0, 0.0, 0.0};
    for (int sp = 0; sp < a.nsplit; ++sp) {
      const double* pp = a.part + (size_t)sp * kND * plane + k;
      U += pp[0];
      W += pp[plane];
      Y[0] += pp[2 * plane];
      Y[1] += pp[3 * plane];
      Y[2] += pp[4 * plane];
    }
    const double M = a.mass[0], m = a.mass[i];
    const double u = a.ub[4 * (size_t)k];
    const double* vi = a.vel + 3 * i;
    const double* v1 = a.vel;
    const double d[3] = {a.pos[0] - a.pos[3 * i], a.pos[1] - a.pos[3 * i + 1],
                         a.pos[2] - a.pos[3 * i + 2]};  // x_1i
    const double rinv = rsqrt_f64(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + a.eps2);
    const double n[3] = {d[0] * rinv, d[1] * rinv, d[2] * rinv};
    const double vi2 = vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2];
    const double v12 = v1[0] * v1[0] + v1[1] * v1[1] + v1[2] * v1[2];
    const double v1vi = v1[0] * vi[0] + v1[1] * vi[1] + v1[2] * vi[2];
    const double nv1 = n[0] * v1[0] + n[1] * v1[1] + n[2] * v1[2];
    const double nvi = n[0] * vi[0] + n[1] * vi[1] + n[2] * vi[2];
    v[0] = 0.5 * m * vi2 - 0.5 * m * U - m * u;
    v[1] = 0.375 * m * vi2 * vi2 + 1.5 * m * u * vi2 + 0.5 * m * u * u +
           0.25 * m * (6.0 * vi2 * U + W) + 0.5 * m * u * (3.0 * v12 - 7.0 * v1vi - nv1 * nvi) +
           m * u * U;
    v[2] = m * u / M;
    for (int c = 0; c < 3; ++c) {
      v[3 + c] = m * vi[c];
      v[6 + c] = 0.5 * m * vi2 * vi[c] - 0.5 * m * u * (vi[c] + nvi * n[c]) -
                 0.5 * m * u * (v1[c] + nv1 * n[c]) - 0.5 * m * (U * vi[c] + Y[c]);
    }
  }
  block_sum<9>(v, lds);
  if (threadIdx.x < 10)
    a.dpart[(size_t)blockIdx.x * 10 + threadIdx.x] = threadIdx.x < 9 ? lds[threadIdx.x * kBlock] : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_diag_final(DiagEpiArgs a) {
  double r[9];
  reduce_rows<9>(a.dpart, a.ndpart, 10, r);
  if (threadIdx.x == 0) {
    const double M = a.mass[0];
    const double* v1 = a.vel;
    const double v12 = v1[0] * v1[0] + v1[1] * v1[1] + v1[2] * v1[2];
    const double U0 = r[2];
    a.out8[0] = 0.5 * M * v12 + r[0];
    a.out8[1] = a.lam * (r[1] + 0.5 * M * U0 * U0);
    for (int c = 0; c < 3; ++c) {
      a.out8[2 + c] = M * v1[c] + r[3 + c];
      a.out8[5 + c] = a.lam * r[6 + c];
    }
  }
}

// ---------------------------------------------------------------------------
// Close-encounter diagnostics (what the paper's test-model figures follow,
// Sec. 4): the star nearest to the massive object, how many stars lie within
// a given radius of it, and the nearest star-star pair.  Unsoftened
// distances.  Minima carry the smaller index on ties, so results are exact
// and order independent.
// ---------------------------------------------------------------------------
struct EncArgs {
  const double* pos;
  const double* vel;
  const PkF64* pk;  // star packets (positions)
  int Ns, jchunk;
  double r_close2;  // squared radius for the count
  const double* mass;
  double G, lam;    // gravitational constant, 1/c^2
  double* part;     // [gridDim.y][2][Ns]: per-star nearest r^2 and partner (as double)
  int nsplit;
  double* bpart;    // [blocks][6]: nearest BH r^2, its star, close count, nearest pair r^2,
                    //              largest 1PN/Newton ratio of a BH pair, its star
  long long* bpair; // [blocks][2]: nearest pair (i, j)
  int nb;
  double* out;      // [8] final
};

// Strength of the 1PN term of a star's pair with the massive object: the
// lambda-part of Eq. (5), (G M / r^2) lambda [(4 G M / r - v^2) n + 4 (n.v) v],
// over the Newtonian pull G M / r^2 (unsoftened r, the star's own velocity).
__device__ __forceinline__ double bh_pair_ratio(double dx, double dy, double dz, double r2,
                                                double vx, double vy, double vz, double gM,
                                                double lam) {
  const double r = sqrt(r2);
  const double nx = dx / r, ny = dy / r, nz = dz / r;
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double nv = nx * vx + ny * vy + nz * vz;
  const double k = 4.0 * gM / r - v2;
  const double tx = k * nx + 4.0 * nv * vx, ty = k * ny + 4.0 * nv * vy,
               tz = k * nz + 4.0 * nv * vz;
  return lam * sqrt(tx * tx + ty * ty + tz * tz);
}

__device__ __forceinline__ bool enc_less(double r2a, long long ia, double r2b, long long ib) {
  return r2a < r2b || (r2a == r2b && ia < ib);
}

__global__ __launch_bounds__(kBlock) void k_enc_pair(EncArgs a) {
  const PkF64* __restrict__ pk = a.pk;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const PkF64& pi = pk[min(i, a.Ns - 1)];
  const double xi = pi.x, yi = pi.y, zi = pi.z;
  const int j0 = blockIdx.y * a.jchunk, j1 = min(a.Ns, j0 + a.jchunk);
  double best = INFINITY;
  int bj = -1;
  for (int j = j0; j < j1; ++j) {
    const PkF64& p = pk[j];
    const double dx = xi - p.x, dy = yi - p.y, dz = zi - p.z;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (j != i && r2 < best) {  // strict: the first (smallest) j wins ties
      best = r2;
      bj = j;
    }
  }
  if (i < a.Ns) {
    double* out = a.part + (size_t)blockIdx.y * 2 * a.Ns + i;
    out[0] = best;
    out[a.Ns] = (double)bj;
  }
}

__global__ __launch_bounds__(kBlock) void k_enc_star(EncArgs a) {
  __shared__ double s_r2[kBlock], s_pr2[kBlock], s_cnt[kBlock], s_z[kBlock];
  __shared__ long long s_i[kBlock], s_pi[kBlock], s_pj[kBlock], s_zi[kBlock];
  const int k = blockIdx.x * kBlock + threadIdx.x;
  double r2 = INFINITY, pr2 = INFINITY, cnt = 0.0, z = -1.0;
  long long idx = LLONG_MAX, pi_ = LLONG_MAX, pj_ = LLONG_MAX, zi = LLONG_MAX;
  if (k < a.Ns) {
    const double dx = a.pos[3 * (k + 1)] - a.pos[0], dy = a.pos[3 * (k + 1) + 1] - a.pos[1],
                 dz = a.pos[3 * (k + 1) + 2] - a.pos[2];
    r2 = dx * dx + dy * dy + dz * dz;
    idx = k + 1;
    cnt = r2 < a.r_close2 ? 1.0 : 0.0;
    z = bh_pair_ratio(dx, dy, dz, r2, a.vel[3 * (k + 1)], a.vel[3 * (k + 1) + 1],
                      a.vel[3 * (k + 1) + 2], a.G * a.mass[0], a.lam);
    zi = k + 1;
    for (int sp = 0; sp < a.nsplit; ++sp) {
      const double* p = a.part + (size_t)sp * 2 * a.Ns + k;
      const long long j = (long long)p[a.Ns];
      if (j >= 0 && enc_less(p[0], j, pr2, pj_)) {
        pr2 = p[0];
        pj_ = j;
      }
    }
    if (pj_ != LLONG_MAX) {  // the pair as (smaller, larger) body index
      const long long bi = k + 1, bj = pj_ + 1;
      pi_ = bi < bj ? bi : bj;
      pj_ = bi < bj ? bj : bi;
    }
  }
  s_r2[threadIdx.x] = r2;
  s_i[threadIdx.x] = idx;
  s_cnt[threadIdx.x] = cnt;
  s_pr2[threadIdx.x] = pr2;
  s_pi[threadIdx.x] = pi_;
  s_pj[threadIdx.x] = pj_;
  s_z[threadIdx.x] = z;
  s_zi[threadIdx.x] = zi;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    const int t = threadIdx.x;
    if (t < s) {
      if (enc_less(s_r2[t + s], s_i[t + s], s_r2[t], s_i[t])) {
        s_r2[t] = s_r2[t + s];
        s_i[t] = s_i[t + s];
      }
      s_cnt[t] += s_cnt[t + s];
      const bool take = s_pr2[t + s] < s_pr2[t] ||
                        (s_pr2[t + s] == s_pr2[t] &&
                         (s_pi[t + s] < s_pi[t] || (s_pi[t + s] == s_pi[t] && s_pj[t + s] < s_pj[t])));
      if (take) {
        s_pr2[t] = s_pr2[t + s];
        s_pi[t] = s_pi[t + s];
        s_pj[t] = s_pj[t + s];
      }
      // largest ratio, ties to the smaller index (NaN ratios never win)
      if (s_z[t + s] > s_z[t] || (s_z[t + s] == s_z[t] && s_zi[t + s] < s_zi[t])) {
        s_z[t] = s_z[t + s];
        s_zi[t] = s_zi[t + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* b = a.bpart + 6 * (size_t)blockIdx.x;
    b[0] = s_r2[0];
    b[1] = (double)s_i[0];
    b[2] = s_cnt[0];
    b[3] = s_pr2[0];
    b[4] = s_z[0];
    b[5] = (double)s_zi[0];
    a.bpair[2 * (size_t)blockIdx.x] = s_pi[0];
    a.bpair[2 * (size_t)blockIdx.x + 1] = s_pj[0];
  }
}

__global__ void k_enc_final(EncArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r2 = INFINITY, cnt = 0.0, pr2 = INFINITY, z = -1.0;
  long long idx = LLONG_MAX, pi_ = LLONG_MAX, pj_ = LLONG_MAX, zi = LLONG_MAX;
  for (int b = 0; b < a.nb; ++b) {
    const double* p = a.bpart + 6 * (size_t)b;
    const long long bz = (long long)p[5];
    if (p[4] > z || (p[4] == z && bz < zi)) {
      z = p[4];
      zi = bz;
    }
    const long long bi = (long long)p[1];
    if (enc_less(p[0], bi, r2, idx)) {
      r2 = p[0];
      idx = bi;
    }
    cnt += p[2];
    const long long qi = a.bpair[2 * (size_t)b], qj = a.bpair[2 * (size_t)b + 1];
    if (p[3] < pr2 || (p[3] == pr2 && (qi < pi_ || (qi == pi_ && qj < pj_)))) {
      pr2 = p[3];
      pi_ = qi;
      pj_ = qj;
    }
  }
  a.out[0] = sqrt(r2);
  a.out[1] = (double)idx;
  a.out[2] = cnt;
  a.out[3] = sqrt(pr2);
  a.out[4] = (double)pi_;
  a.out[5] = (double)pj_;
  a.out[6] = z;
  a.out[7] = (double)zi;
}

// ---------------------------------------------------------------------------
// Unrestricted EIH equations for every pair (no massive-object truncation).
// In EIH layout the full 1PN pair term of body a with partner b is
//   (G m_b/R^2) n_ab [-v_a^2 - 2 v_b^2 + 4 v_a.v_b + 3/2 (n_ab.v_b)^2
//                     + 4 V_a + V_b + 1/2 x_ab.a^N_b]
//   + (G m_b/R^2) [n_ab.(4 v_a - 3 v_b)] (v_a - v_b) + 7/2 (G m_b/R) a^N_b,
// the limited star-star term with u_b -> V_b (the full potential) and
// -b_b -> a^N_b (the full Newtonian acceleration).  So it takes two sweeps
// over all N bodies with the same pair kernel: pass 1 (MODE_P1) gives V and
// a^N of every body; k_eih_mid writes them into the packets
// (e = -2 v^2 + V, hb = a^N / 2); pass 2 (MODE_P2) sums the 1PN terms.
// ---------------------------------------------------------------------------
struct EihArgs {
  const double* pos;
  const double* vel;
  const double* mass;
  int N;
  double G, lam;
  void* pk;           // [N] packets of all bodies
  double* va;         // [N][4]: V, a^N (3)
  const double* part; // [nsplit][kNF][N]
  int nsplit;
  double* acc_newton; // outputs (any may be nullptr)
  double* phi;
  double* acc_1pn;
  int* status;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eih_packets(EihArgs a) {
  using Pk = typename PkOf<T>::type;
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b < a.N) {
    Pk p;
    p.x = a.pos[3 * b];
    p.y = a.pos[3 * b + 1];
    p.z = a.pos[3 * b + 2];
    p.gm = (T)(a.G * a.mass[b]);
    p.svx = (T)(PairScale<T>::sv * a.vel[3 * b]);
    p.svy = (T)(PairScale<T>::sv * a.vel[3 * b + 1]);
    p.svz = (T)(PairScale<T>::sv * a.vel[3 * b + 2]);
    p.e = T(0);
    p.hbx = T(0);
    p.hby = T(0);
    p.hbz = T(0);
    if constexpr (sizeof(T) == 8) {
      p.pad = 0.0;
    } else {
      p.pad0 = 0.f;
      p.pad1 = 0.f;
    }
    static_cast<Pk*>(a.pk)[b] = p;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eih_mid(EihArgs a) {
  using Pk = typename PkOf<T>::type;
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b < a.N) {
    const size_t plane = (size_t)a.N;
    double U = 0.0, Gx = 0.0, Gy = 0.0, Gz = 0.0;
    for (int sp = 0; sp < a.nsplit; ++sp) {
      const double* pp = a.part + (size_t)sp * kNF * plane + b;
      U += pp[F_U * plane];
      Gx += pp[F_G * plane];
      Gy += pp[(F_G + 1) * plane];
      Gz += pp[(F_G + 2) * plane];
    }
    const double aN[3] = {-Gx, -Gy, -Gz};
    const double vx = a.vel[3 * b], vy = a.vel[3 * b + 1], vz = a.vel[3 * b + 2];
    Pk& p = static_cast<Pk*>(a.pk)[b];
    p.e = (T)(-2.0 * (vx * vx + vy * vy + vz * vz) + U);
    p.hbx = (T)(0.5 * aN[0]);
    p.hby = (T)(0.5 * aN[1]);
    p.hbz = (T)(0.5 * aN[2]);
    double* v4 = a.va + 4 * (size_t)b;
    v4[0] = U;
    v4[1] = aN[0];
    v4[2] = aN[1];
    v4[3] = aN[2];
    if (a.phi) a.phi[b] = -U;
    if (a.acc_newton) {
      a.acc_newton[3 * b] = aN[0];
      a.acc_newton[3 * b + 1] = aN[1];
      a.acc_newton[3 * b + 2] = aN[2];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_eih_final(EihArgs a) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b < a.N) {
    const size_t plane = (size_t)a.N;
    double sum[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) sum[f] = 0.0;
    for (int sp = 0; sp < a.nsplit; ++sp) {
      const double* pp = a.part + (size_t)sp * kNF * plane + b;
#pragma unroll
      for (int f = F_G; f < kNF; ++f) sum[f] += pp[f * plane];
    }
    sum[F_C2] *= kSqrt32;
    const double* v4 = a.va + 4 * (size_t)b;
    const double vx = a.vel[3 * b], vy = a.vel[3 * b + 1], vz = a.vel[3 * b + 2];
    const double v[3] = {vx, vy, vz};
    const double S0 = -(vx * vx + vy * vy + vz * vz) + 4.0 * v4[0];
    double a1[3];
    for (int c = 0; c < 3; ++c)
      a1[c] = a.lam * (S0 * sum[F_G + c] + sum[F_Q + c] + sum[F_C2] * v[c] + 7.0 * sum[F_Q7 + c]);
    if (a.acc_1pn) {
      a.acc_1pn[3 * b] = a1[0];
      a.acc_1pn[3 * b + 1] = a1[1];
      a.acc_1pn[3 * b + 2] = a1[2];
    }
    bool bad = false;
    for (int c = 0; c < 3; ++c) bad |= !isfinite(v4[1 + c] + a1[c]);
    if (bad) atomicOr(a.status, 1);
  }
}

// ---------------------------------------------------------------------------
// Batched ensemble: many independent systems in one launch per phase.
// Every phase's workgroups are numbered system after system in the order
// `order` (systems by decreasing cost, so the dispatcher, which starts
// workgroups in index order, hands out the largest systems first);
// `pre_*[r]` is the first workgroup of the r-th system in that order.  A
// workgroup finds its system by binary search over pre_* (scalar loads) and
// runs the same per-block code as the single-system kernels on that system's
// slices of the concatenated arrays.
// ---------------------------------------------------------------------------
struct SysDev {
  int64_t body0;  // first body (the massive object) in the concatenated body arrays
  int64_t star0;  // first star in the concatenated star arrays (packets, u/b)
  int64_t part0;  // first double of the system's pair partials
  int Ns, nsplit, jchunk, iblocks;
  int pro0, epi0;  // first row of the system's prologue / epilogue partials
  int npro, nepi;  // number of those rows
  double G, lam, eps2;
};

struct BatchArgs {
  const SysDev* sys;
  const int* order;
  const int* pre;  // prefix of this phase's workgroups over `order`, n_sys+1 entries
  int n_sys;
  const double* pos;  // evaluation state, concatenated [sum N][3]
  const double* vel;
  const double* mass;
  void* pk;  // packets of all stars
  double* ub;
  double* bpart;
  double* part;
  double* bhpart;
  int* status;
  int stage;
  double dt;
  double *X, *V, *Xs, *Vs, *KX, *KV;
};

// rank r of the system owning workgroup blk: pre[r] <= blk < pre[r+1]
__device__ __forceinline__ int batch_rank(const int* pre, int n, int blk) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ ProArgs batch_pro_args(const BatchArgs& b, const SysDev& S) {
  using Pk = typename PkOf<T>::type;
  ProArgs a;
  a.pos = b.pos + 3 * S.body0;
  a.vel = b.vel + 3 * S.body0;
  a.mass = b.mass + S.body0;
  a.Ns = S.Ns;
  a.G = S.G;
  a.eps2 = S.eps2;
  a.pk = static_cast<Pk*>(b.pk) + S.star0;
  a.ub = b.ub + 4 * S.star0;
  a.bpart = b.bpart + 8 * kProRows * (int64_t)S.pro0;
  a.status = b.status;
  return a;
}

__device__ __forceinline__ EpiArgs batch_epi_args(const BatchArgs& b, const SysDev& S) {
  EpiArgs a;
  const int64_t o3 = 3 * S.body0;
  a.pos = b.pos + o3;
  a.vel = b.vel + o3;
  a.mass = b.mass + S.body0;
  a.Ns = S.Ns;
  a.G = S.G;
  a.lam = S.lam;
  a.eps2 = S.eps2;
  a.ub = b.ub + 4 * S.star0;
  a.bpart = b.bpart + 8 * kProRows * (int64_t)S.pro0;
  a.nbpro = S.nepi;  // one prologue row per 64 stars
  a.part = b.part + S.part0;
  a.nsplit = S.nsplit;
  a.newton_only = 0;
  a.phi_in = nullptr;
  a.accN_in = nullptr;
  a.acc_newton = nullptr;
  a.phi = nullptr;
  a.acc_1pn = nullptr;
  a.bhpart = b.bhpart + 4 * (int64_t)S.epi0;
  a.nbepi = S.nepi;
  a.status = b.status;
  a.stage = b.stage;
  a.dt = b.dt;
  a.X = b.X + o3;
  a.V = b.V + o3;
  a.Xs = b.Xs + o3;
  a.Vs = b.Vs + o3;
  a.KX = b.KX + o3;
  a.KV = b.KV + o3;
  return a;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prologue_batched(BatchArgs b) {
  const int r = batch_rank(b.pre, b.n_sys, blockIdx.x);
  const SysDev S = b.sys[b.order[r]];
  prologue_block<T>(batch_pro_args<T>(b, S), blockIdx.x - b.pre[r]);
}

// IPT i-bodies per lane for every system of the ensemble (the plan's shape)
template <typename T, int IPT>
__global__ __launch_bounds__(kBlock) void k_pair_batched(BatchArgs b) {
  using Pk = typename PkOf<T>::type;
  const int r = batch_rank(b.pre, b.n_sys, blockIdx.x);
  const SysDev S = b.sys[b.order[r]];
  const int local = blockIdx.x - b.pre[r];
  PairArgs a;
  a.pk = static_cast<const Pk*>(b.pk) + S.star0;
  a.Ns = S.Ns;
  a.jchunk = S.jchunk;
  a.eps2 = S.eps2;
  a.part = b.part + S.part0;
  __shared__ double red[pair_red_doubles<T, IPT, 4>()];
  pair_block<T, MODE_FUSED, IPT, 4>(a, local % S.iblocks, local / S.iblocks, red);
}

__global__ __launch_bounds__(kBlock) void k_epilogue_batched(BatchArgs b) {
  __shared__ double lds[7 * kBlock];
  __shared__ double fsum[kNF * kEpiStars];
  const int r = batch_rank(b.pre, b.n_sys, blockIdx.x);
  const SysDev S = b.sys[b.order[r]];
  epilogue_block<double>(batch_epi_args(b, S), blockIdx.x - b.pre[r], lds, fsum);
}

__global__ __launch_bounds__(kBlock) void k_bh_final_batched(BatchArgs b) {
  __shared__ double lds[7 * kBlock];
  const SysDev S = b.sys[b.order[blockIdx.x]];
  bh_final_block<double>(batch_epi_args(b, S), lds);
}

}  // namespace pn
