/*
 * pn.h -- C ABI of libpn, the MI355X (gfx950) implementation of the
 * limited first-order post-Newtonian direct N-body hot path of
 *   T. Tatekawa, "Accelerating N-body simulation of self-gravitating systems
 *   with limited first-order post-Newtonian approximation" (arXiv:1801.07986).
 *
 * System: one massive object (the paper's body #1, here index 0, mass M) and
 * N-1 low-mass stars (Sec. 2).  N counts the massive object.
 *
 * Common conventions for every entry point
 * ----------------------------------------
 * - Array arguments are DEVICE pointers (e.g. torch.Tensor.data_ptr() of a
 *   CUDA/HIP tensor) to float64, C-contiguous, 8-byte aligned, unless marked
 *   "host".  pos, vel, acc_*: [N][3] row-major (x, y, z of body b at
 *   3b..3b+2); mass, phi: [N].  Inputs and outputs must not overlap, except
 *   where stated.
 * - Units are the caller's; G > 0.  c is the speed of light: lambda = 1/c^2
 *   multiplies every 1PN term; c = +INFINITY is allowed and gives the
 *   Newtonian equations exactly.
 * - eps >= 0 is the Plummer softening length of Sec. 4, Eq. (10): every pair
 *   distance r_ab (massive object included) is replaced by
 *   R_ab = sqrt(r_ab^2 + eps^2) in every term, and n_ab = x_ab / R_ab.
 * - stream: a hipStream_t, or NULL for the library's own stream (which, like
 *   every default-flag stream, is ordered after the legacy default stream).
 * - flags: 0 = synchronous: the call returns after the device work finished
 *   and reports device-detected errors.  PN_ASYNC = enqueue only: returns after
 *   launching; device-detected errors (PN_ENONFINITE, an invalid mass[0]) are
 *   then not reported.
 * - Ownership: the caller owns every argument buffer.  The library owns only
 *   internal scratch, kept per device and grown on demand, and (pn_step) cached
 *   HIP graphs; pn_release() frees both.  No argument pointer is kept after the
 *   call returns, except inside the cached step graphs of pn_step,
 *   pn_step_hermite (one step, and 16 steps per replay for long runs) and
 *   pn_step_batched, which are re-captured when any pointer or parameter
 *   changes.
 * - Return codes: PN_OK, or one of the negative codes below.  No C++ exception
 *   crosses the ABI.  Outputs are unspecified after an error, except
 *   PN_ENONFINITE, where all outputs are written.
 * - Determinism: identical inputs, sizes and schedule give bitwise-identical
 *   outputs (fixed-order reductions, no floating-point atomics).
 * - Thread safety: calls may come from several host threads; the library
 *   serialises them internally.  Calls on one stream run in call order; a
 *   call on a different stream than the previous call first makes its stream
 *   wait for the previous call's device work (all calls share the library's
 *   scratch), so the device work of two calls never overlaps, PN_ASYNC or not.
 */
#ifndef PN_H_
#define PN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PN_OK 0
#define PN_EINVAL (-1)     /* bad argument (null/misaligned pointer, N < 2, G <= 0, c <= 0 or
                              NaN, eps < 0, non-finite dt, nsteps < 0, unknown precision,
                              mass[0] <= 0 detected on the device) */
#define PN_ENONFINITE (-2) /* a non-finite acceleration was produced (outputs written) */
#define PN_EDEVICE (-3)    /* HIP runtime error (text: pn_strerror(PN_EDEVICE)) */
#define PN_ENOMEM (-4)     /* device allocation failed */

/* precision of the O(N^2) star-star pair sums */
#define PN_FP64 0  /* everything in FP64 */
#define PN_MIXED 1 /* pair arithmetic in FP32 with FP64 coordinate differences and FP32
                      partial sums carried in FP64 between j-tiles; black-hole terms,
                      potentials, reductions and integrator state in FP64 */

/* flags */
#define PN_ASYNC 1   /* see above */
#define PN_NOGRAPH 2 /* pn_step: launch kernels directly instead of replaying a graph */
#define PN_TIMING 4  /* pn_step / pn_accel: time every pair-kernel launch with HIP events
                        (implies PN_NOGRAPH); read with pn_last_timing() */

/*
 * Newtonian acceleration and potential of all N bodies: the first terms of
 * Eq. (1) (massive object) and Eq. (4) (stars; printed with r_ij where r_ij^3
 * is meant), softened per Eq. (10):
 *   acc_newton[a] = -sum_{b != a} G m_b x_ab / R_ab^3,
 *   phi[a]        = -sum_{b != a} G m_b / R_ab.
 * vel and c are not used (kept so every call takes the same system
 * description); vel may be NULL.  c must still be valid.
 */
int pn_potential_accel(const double* pos, const double* vel, const double* mass, int64_t N,
                       double G, double c, double eps, double* acc_newton, double* phi,
                       void* stream, int flags);

/*
 * Limited-1PN acceleration of all N bodies, lambda times the bracketed terms of
 * Eqs. (1)-(6): Eqs. (2)+(3) for the massive object, (5)+(6) for the stars.
 * phi and acc_newton are the Newtonian potential and acceleration of all bodies
 * at the same positions (normally pn_potential_accel's outputs); they supply
 * the potentials and Newtonian accelerations inside the 1PN brackets.  The
 * massive object's own velocity vel[0] is not used: Eqs. (2)-(6) contain no
 * v_1; its linear occurrences in the underlying EIH equations appear through
 * w = -sum_s m_s v_s / M (second and sixth lines of Eq. (6), last line of
 * Eq. (3)).  Output acc_1pn: [N][3]; total acceleration = acc_newton + acc_1pn.
 */
int pn_correction(const double* pos, const double* vel, const double* mass, int64_t N,
                  double G, double c, double eps, const double* phi, const double* acc_newton,
                  double* acc_1pn, void* stream, int flags);

/*
 * One full force evaluation as pn_step performs it (one fused star-star
 * sweep in the given precision): Newtonian acceleration, potential and 1PN
 * part of all N bodies.  Any of the three outputs may be NULL.
 */
int pn_accel(const double* pos, const double* vel, const double* mass, int64_t N, double G,
             double c, double eps, int precision, double* acc_newton, double* phi,
             double* acc_1pn, void* stream, int flags);

/*
 * pn_accel for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, outputs and error codes as pn_accel, and the same kernels; the
 * call makes no device allocation and no hipFree.  Its scratch (star packets,
 * the sweep's per-split partial sums, block rows, the status word) is a fixed
 * 64 MiB device array that the library's code object holds on every GPU it
 * is loaded on, until the process ends.
 * - Limit: the partial sums take 88 bytes per star and j-split; where
 *   pn_accel's split count would not fit, fewer splits are used (results then
 *   differ from pn_accel's by rounding only), and N whose scratch exceeds
 *   64 MiB even with one split (about N > 300000) is rejected with PN_EINVAL
 *   before any device work (pn_strerror(PN_EINVAL) names the sizes).
 * - Calls on one GPU share that array and it keeps the last call's contents
 *   (each call rewrites everything it reads, its status word included): calls
 *   that overlap on one GPU, from different streams or host threads racing
 *   with PN_ASYNC, race.  Calls of the other entry points use their own
 *   scratch and do not race with it.
 * - The first call of the library on a device (any entry point) sets the
 *   device up: it creates the library's stream and looks up the array's
 *   device address.  Make one such call before capturing.  Under capture pass
 *   the capturing stream and PN_ASYNC (a synchronous call waits for the
 *   stream).  PN_TIMING is rejected (it would create events).
 */
int pn_accel_noalloc(const double* pos, const double* vel, const double* mass, int64_t N,
                     double G, double c, double eps, int precision, double* acc_newton,
                     double* phi, double* acc_1pn, void* stream, int flags);

/*
 * Unrestricted EIH 1PN accelerations of all N bodies: every pair at full 1PN
 * order, with no body singled out (the general N-body 1PN equations the paper
 * starts from in Sec. 2 and names as its next step in Sec. 5).  Evaluated in
 * two O(N^2) sweeps: the Newtonian potential and acceleration of every body,
 * then the 1PN pair sum, which uses them.  Same softening reading and output
 * layout as pn_accel; every body's own velocity enters (vel[0] included).
 */
int pn_accel_eih(const double* pos, const double* vel, const double* mass, int64_t N, double G,
                 double c, double eps, int precision, double* acc_newton, double* phi,
                 double* acc_1pn, void* stream, int flags);

/*
 * Advance (pos, vel) of all N bodies, massive object included, by nsteps
 * fixed steps of the classical fourth-order Runge-Kutta method (Sec. 3.2 and
 * Sec. 4): four force evaluations per step, f(x, v) = (v, a^N + a^1PN).
 * pos and vel are read and overwritten in place; mass is read only.
 * nsteps = 0 is a no-op.  precision: PN_FP64 or PN_MIXED.
 */
int pn_step(double* pos, double* vel, const double* mass, int64_t N, double G, double c,
            double eps, double dt, int64_t nsteps, int precision, void* stream, int flags);

/*
 * Total acceleration a = a^N + a^1PN of all N bodies and its time derivative
 * along the motion, the jerk j = (d/dt) a(x(t), v(t)) = (v . grad_x) a +
 * (a . grad_v) a, which the fourth-order Hermite scheme the paper proposes
 * for close encounters (Sec. 4, Sec. 5, Appendix) needs.  Computed exactly
 * (to rounding) in FP64 by forward-mode differentiation of the evaluation:
 * one FP64 evaluation gives a, then the same sweep on dual numbers (value,
 * derivative) with positions (x, v) and velocities (v, a).  Outputs acc, jerk:
 * [N][3] device arrays, both required.  vel[0] is used here (the massive
 * object moves with it, so it enters the derivative of every distance to it),
 * unlike in pn_accel.  FP64 only.
 */
int pn_jerk(const double* pos, const double* vel, const double* mass, int64_t N, double G,
            double c, double eps, double* acc, double* jerk, void* stream, int flags);

/*
 * Advance (pos, vel) of all N bodies by nsteps fixed steps of the
 * fourth-order Hermite scheme (Sec. 4-5, Appendix), FP64:
 *   predict  x_p = x + v dt + a dt^2/2 + j dt^3/6 + s dt^4/24 + k dt^5/120,
 *            v_p = v + a dt + j dt^2/2 + s dt^3/6 + k dt^4/24,
 *   evaluate (a_p, j_p) at (x_p, v_p) as pn_jerk does,
 *   correct  v' = v + (a + a_p) dt/2 + (j - j_p) dt^2/12,
 *            x' = x + (v + v') dt/2 + (a - a_p) dt^2/12,
 * with snap s and crackle k from the step's Hermite interpolant of a
 * (k = (12 (a - a_p) + 6 dt (j + j_p))/dt^3, s = (-6 (a - a_p) -
 * dt (4 j + 2 j_p))/dt^2 + k dt), both zero before the first step.  Each call
 * starts afresh from (a, j) at the given state; one call of n1 + n2 steps
 * therefore differs (at O(dt^5)) from two calls of n1 and n2.  Two sweeps per
 * step (the FP64 one and the dual one).  dt > 0; nsteps = 0 is a no-op.
 */
int pn_step_hermite(double* pos, double* vel, const double* mass, int64_t N, double G, double c,
                    double eps, double dt, int64_t nsteps, void* stream, int flags);

/*
 * Conserved quantities of Sec. 2: 1PN total energy (Eq. (7)) and momentum
 * (Eq. (8)), by the sum conventions of those equations (ordered star pairs
 * i != j where r_ij appears; the last sum of Eq. (7) includes i = j).
 * out8 (HOST pointer, 8 doubles): [E_N, lambda*E_1PN, P_N(3), lambda*P_1PN(3)],
 * E = out8[0] + out8[1], P = out8[2..4] + out8[5..7].
 */
int pn_diagnostics(const double* pos, const double* vel, const double* mass, int64_t N,
                   double G, double c, double eps, double* out8, void* stream, int flags);

/*
 * Close-encounter diagnostics of the kind the paper's test-model figures
 * follow (Sec. 4): distance of the star nearest to the massive object, the
 * number of stars closer to it than r_close (e.g. a multiple of the
 * Schwarzschild radius 2GM/c^2), the nearest star-star pair, and how
 * relativistic the most relativistic massive-object/star pair is: the ratio
 * of the lambda-term of Eq. (5) to the Newtonian pull,
 * |(4GM/r - v_s^2) n + 4 (n.v_s) v_s| / c^2 (v_s the star's velocity).
 * Unsoftened distances; N >= 3; c = inf gives ratio 0.  out8 (HOST, 8
 * doubles): [min r_0s, its body index, count with r_0s < r_close, min r_ij,
 * i, j, max ratio, its body index] (i < j, body indices; ties go to the
 * smallest indices).  Always synchronous.
 */
int pn_encounters(const double* pos, const double* vel, const double* mass, int64_t N, double G,
                  double c, double r_close, double* out8, void* stream, int flags);

/*
 * Many independent systems advanced together (each as pn_step would).
 * System b occupies bodies offsets[b] .. offsets[b+1]-1 of the concatenated
 * pos/vel/mass arrays, its massive object at offsets[b]; offsets (HOST, n_sys+1
 * entries) starts at 0 and increases by at least 2 per system.  G, c, eps
 * (HOST, n_sys entries each) are per-system parameters; dt is common.
 */
int pn_step_batched(int32_t n_sys, const int64_t* offsets, const double* G, const double* c,
                    const double* eps, double* pos, double* vel, const double* mass, double dt,
                    int64_t nsteps, int precision, void* stream, int flags);

/*
 * Sweep shape of pn_step_batched in the given precision (searched by the
 * autotuner over whole ensemble steps): ipt i-bodies per lane (1 or 2) for
 * every system, and the ensemble's common j-split count (1..64; 0 = the
 * default rule, about 16k sweep workgroups in all), which each system caps so
 * that a wavefront keeps at least 32 j.  precision < 0 restores the defaults
 * (1 i per lane, the rule).  Like pn_set_shape, it changes speed only.
 */
int pn_set_batch_shape(int precision, int ipt, int nsplit);

/*
 * The shape pn_step_batched would use for this ensemble (HOST offsets as
 * pn_step_batched takes them): out (HOST, n_sys + 1 ints) = [i-bodies per
 * lane, then each system's j-split count].  Host only.
 */
int pn_query_batch_shape(int precision, int32_t n_sys, const int64_t* offsets, int* out);

/*
 * One launch per Runge-Kutta stage for small systems (the integrator of
 * Sec. 3.2 / Sec. 4 as pn_step runs it, Eqs. (1)-(6) per stage): pn_step in
 * the given precision advances systems of n_min <= N <= n_max bodies with one
 * kernel per stage.  In that kernel each workgroup sums all j for ns stars
 * (ns = 2, 4, 8 or 16) and runs their epilogue; every workgroup recomputes
 * the massive object's pending update.  Sizes no entry covers keep the
 * chained two-kernel stages.  Entries are searched in the order given;
 * precision < 0 clears them.  Searched by the autotuner.  The choice changes
 * speed only: both forms meet the same accuracy, each is deterministic, and
 * a run split over several calls equals one call in either.  The two forms
 * sum in different orders, so they differ from each other by rounding.  Host
 * only; PN_EINVAL for a bad precision, n_min < 2, n_max < n_min or ns outside
 * {2, 4, 8, 16}.
 */
int pn_set_stage_kernel(int precision, int64_t n_min, int64_t n_max, int ns);

/*
 * Stars per workgroup of the one-launch stage that pn_step would use for an
 * N-body system in the given precision, 0 for the chained two-kernel stages;
 * PN_EINVAL for a bad precision or N.  Host only.
 */
int pn_query_stage_kernel(int precision, int64_t N);

/*
 * Launch shape of the star-star sweep for systems with n_min <= N <= n_max in
 * the given precision (searched by the autotuner; later entries never override
 * earlier ones that match).  ipt: i-bodies per lane (1 or 2); ws: wavefronts
 * sharing one i-range (1, 4, or 8 in workgroups of 512 threads); nsplit: j-range
 * splits (0 = default rule).
 * precision < 0 clears the table.  Shapes change speed only: results of a
 * given shape are deterministic and every shape meets the same accuracy.
 */
int pn_set_shape(int precision, int64_t n_min, int64_t n_max, int ipt, int ws, int nsplit);

/*
 * The launch shape the evaluation of an N-body system would use in the given
 * precision (tuned table, PN_SHAPE override or default rule; the shape
 * changes only speed, never the sums): out4 (HOST, 4 ints) = [i-bodies per
 * lane, wavefronts per i-range, j-splits, i-blocks].  Lets a caller name the
 * exact sweep kernel it measured.
 */
int pn_query_shape(int precision, int64_t N, int* out4);

/* Text for a return code (PN_EDEVICE: the last HIP error seen).  Never NULL. */
const char* pn_strerror(int code);

/*
 * After a call made with PN_TIMING: out (HOST, 3 doubles) receives
 * [number of pair-kernel launches, their total duration in ms, pairs per launch].
 * A pn_step in one-launch stages (pn_set_stage_kernel) times those stage
 * kernels, which also run the epilogue.
 */
int pn_last_timing(double* out);

/* Frees the library's scratch memory and cached graphs on every device. */
int pn_release(void);

#ifdef __cplusplus
}
#endif

#endif /* PN_H_ */
