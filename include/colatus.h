/*
 * colatus.h -- C ABI of the MI355X (gfx950) COLATUS hot path.
 *
 * Paper: Stalder et al., "A new gravitational N-body simulation algorithm
 * for investigation of cosmological chaotic advection" (arXiv:1208.3444).
 *
 * What the library computes
 *   - the direct-summation (particle-particle) softened acceleration of
 *     Eq. (1) in comoving coordinates, with the attractive sign,
 *         acc_k = a^-3 G sum_{j != k} m_j (x_j - x_k) / (|x_j - x_k|^2 + eps^2)^{3/2}
 *     (Section II; the GPU force loop of Appendix A);
 *   - the expansion-aware kick-drift-kick step built from the drift and kick
 *     operators of Eq. (9), with a(t) from the Friedmann equation, Eq. (2);
 *   - the discrete adjoint (vector-Jacobian product) of that step, used for
 *     trajectory sensitivities and finite-time Lyapunov exponents of the
 *     chaotic-advection study the paper motivates (Sections I and IV);
 *   - optionally the deformation term of Eq. (10), a fixed attractor, in
 *     the forces, the run and the adjoint (with its parameter gradients),
 *     and the background term of Eq. (6) (the mean density's pull removed);
 *   - the paper's own difference equations, Eqs. (3)-(5), as a second
 *     scheme (colatus_run_he);
 *   - tracer tracks (the state of chosen particles at every step) and each
 *     tracer's velocity power spectrum (Section I's stated goal).
 *
 * Conventions shared by every entry point
 *   - Arrays named x, v, acc, lam_*, grad_* are structure-of-arrays float64
 *     planes of shape [3][N]: x[0..N) holds the x components, x[N..2N) the
 *     y components, x[2N..3N) the z components.  m and phi are [N] float64.
 *     All of them are DEVICE pointers on the current HIP device, contiguous,
 *     owned by the caller; the library never frees or retains them beyond
 *     the call's queued work.
 *   - x is the comoving position, v = dx/dt the comoving velocity (Eq. (1)),
 *     m the particle mass, eps the Plummer softening in comoving units, G the
 *     gravitational constant, H0 and Om_R, Om_M, Om_K, Om_L the parameters
 *     of Eq. (2) (no renormalisation of their sum), a the scale factor.
 *   - stream is a hipStream_t (NULL = the default stream).  Work is queued
 *     on it and the call returns without waiting, except where a host
 *     output (diagnostics) is requested, or where the library grows one of
 *     its scratch buffers (the old buffer is freed after the device is idle)
 *     or reads back a coefficient table it needs on the host (the adjoint).
 *   - Every argument check runs on the host before any HIP call; on an error
 *     nothing has been queued.  Return value 0 on success, else one of the
 *     negative COLATUS_E* codes; colatus_strerror() names it.
 *   - Internal scratch (split-j partial sums, coefficient tables, work lists,
 *     checkpoints) is allocated by the library per (device, stream), kept for
 *     reuse and released by colatus_release() or at process exit.  Calls on
 *     one stream are serialised by the stream; concurrent calls from
 *     different host threads on the SAME stream are not supported.
 *   - Results are deterministic: the split over source slices is summed in a
 *     fixed order, with no atomics in any reduction, so a repeated call on the
 *     same input gives bitwise the same output.
 *   - Limits: 1 <= N <= 2^28 particles (per call, all boxes together).
 *
 * Readings of the paper taken by this library
 *   - Eq. (1) prints the pair term as m_j (x_k - x_j), which is repulsive;
 *     the attractive m_j (x_j - x_k) is used.  The self pair j == k is
 *     excluded.  Open box; the background term of Eq. (6) only when a
 *     colatus_background is passed.
 *   - The step is the symplectic kick-drift-kick of Eq. (9) with canonical
 *     momentum p = a^2 v (per unit mass): kick p += g int dt/a, drift
 *     x += p int dt/a^2, where g = G sum m_j (x_j - x_k) r^-3.  Steps are
 *     uniform in ln a; the half-step point is the midpoint in ln a.
 *   - Static limit: H0 == 0 holds a fixed; see colatus_step / colatus_run.
 */
#ifndef COLATUS_H
#define COLATUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define COLATUS_OK          0
#define COLATUS_EINVAL     -1  /* invalid argument (shape, range, NULL, non-finite scalar) */
#define COLATUS_EFRIEDMANN -2  /* H^2(a) <= 0 somewhere on the requested range of a      */
#define COLATUS_ENODEV     -3  /* no HIP device available                                 */
#define COLATUS_ENOMEM     -4  /* device scratch allocation failed                        */
#define COLATUS_EHIP       -5  /* a HIP runtime call failed                               */
#define COLATUS_ENONFINITE -6  /* diagnostics found a NaN or Inf in the state             */
#define COLATUS_ESCRATCH   -7  /* problem too large for the allocation-free entry point's
                                  fixed scratch (colatus_forces_noalloc: N > 16384)      */

/* ---- pair arithmetic --------------------------------------------------- */
/* The FP32 forms evaluate each pair in FP32 on coordinates taken relative to
 * the centre of the target tile (FP64 subtraction, then rounding), sum the
 * pair terms of one tile in FP32 (a tile: a part of at most 256 sources in
 * the default symmetric loop, 256 sources in the ordered loop), and then
 * accumulate the tiles' FP32 partials per target as follows.               */
#define COLATUS_FP64         0  /* FP64 pairs, FP64 running sums                            */
#define COLATUS_MIXED_TWOSUM 1  /* FP32 pairs; tile partials accumulated by TwoSum into an
                                   unevaluated (hi, lo) FP32 pair (compensated)            */
#define COLATUS_MIXED_F64ACC 2  /* FP32 pairs; tile partials accumulated in FP64           */
#define COLATUS_FP32         3  /* FP32 pairs; tile partials accumulated in one FP32
                                   running sum (no compensation)                           */

/* ---- ensembles of independent boxes ------------------------------------ */
/* Particles of box b are [box_offsets[b], box_offsets[b+1]) of the [3][N]
 * arrays; particles of different boxes do not interact, and box b uses
 * softening eps[b] (the scalar eps argument is then ignored).  Both arrays
 * are HOST pointers, read during the call only.  box_offsets[0] == 0,
 * non-decreasing, box_offsets[n_boxes] == N, every box non-empty.
 * A NULL batch pointer means one box holding all N particles.             */
typedef struct {
    int32_t n_boxes;
    const int64_t *box_offsets; /* host, n_boxes + 1 */
    const double *eps;          /* host, n_boxes     */
} colatus_batch;

/* ---- deformation attractor (Eq. (10)) --------------------------------- */
/* The deformation term of Eq. (10): a fixed point at comoving x_psi that
 * pulls every particle like a mass S/G would, S = C psi (C and psi enter
 * only as their product).  It adds to the comoving sum g of particle k
 *     S (x_psi - x_k) / (|x_psi - x_k|^2 + eps^2)^{3/2}
 * (attractive, as the pair term of Eq. (1) is read; eps is the particle's
 * box softening), and -S / sqrt(|x_psi - x_k|^2 + eps^2) to its potential;
 * the diagnostics count this external energy once (not halved).  x_psi is
 * the same comoving point in every box of a batch.  HOST pointer, read
 * during the call only; NULL means Eq. (1) alone.  strength and x must be
 * finite (strength 0 adds nothing but still yields d/dS in colatus_adjoint).
 * A particle exactly at x_psi with eps == 0 gives Inf/NaN.                 */
typedef struct {
    double strength; /* S = C psi */
    double x[3];     /* x_psi, comoving */
} colatus_attractor;

/* ---- background term (Eq. (6)) ------------------------------------------ */
/* The background term of the comoving potential of Eq. (6): with it the
 * pull of the mean matter density is removed, so that an unperturbed
 * distribution at that density follows the expansion a(t) of Eq. (2)
 * instead of collapsing under its own mean density (Eq. (1) alone, in an
 * open box).  It adds to the comoving sum g of particle k
 *     b (x_k - c)
 * and -b |x_k - c|^2 / 2 to its potential (an external field: counted once
 * in the diagnostics).  b = Om_M H0^2 / 2 is the value consistent with
 * Eq. (2) (Lambda and radiation act on every particle alike, so only the
 * matter term remains once they are included); c is the centre of the
 * region the particles sample (the box centre).  Scales with a like the
 * pair sum.  HOST pointer, read during the call; NULL: no background term.
 * coefficient and centre must be finite.  The same b and c for every box
 * of a batch.                                                              */
typedef struct {
    double coefficient; /* b */
    double centre[3];   /* c, comoving */
} colatus_background;

/* ---- tracer tracks ----------------------------------------------------- */
/* The state of chosen particles at every grid point a run visits, so that
 * a single particle's velocity can be followed step by step (Section I and
 * Section IV give this as the method's purpose).
 *   index: HOST array of n_tracers distinct particle indices in [0, N)
 *          (global indices when a batch is given), read during the call.
 *   out:   DEVICE array [rows][2][3][n_tracers], rows = last_step -
 *          first_step + 1, written by the call: out[r][0][c][t] = x_c and
 *          out[r][1][c][t] = v_c (= dx/dt, comoving) of particle index[t] at
 *          grid point first_step + r; row 0 is the start state as given.
 * 1 <= n_tracers <= 65536, else COLATUS_EINVAL (as for a repeated or
 * out-of-range index, or a NULL pointer).  Recording adds no launch per
 * step (the step kernels write the rows).                                 */
typedef struct {
    int32_t n_tracers;
    const int64_t *index; /* host, n_tracers */
    double *out;          /* device, [rows][2][3][n_tracers] */
} colatus_tracks;

/* ---- diagnostics row --------------------------------------------------- */
/* One row per integer grid point a_n visited by a run (first row: the start
 * state).  With p = a^2 v:
 *   K  = 1/2 sum m |p|^2 / a^2            U = (1/(2a)) sum_k m_k phi_k
 *   LI = K + U - (K + U)_first + sum of trapezoids of (2K + U) over ln a,
 *        the residual of the Layzer-Irvine equation dE/d ln a = -(2K + U)
 *        that this Hamiltonian system obeys (zero for exact integration);
 *        in the static limit LI = E - E_first.
 *   P  = sum m p,   L = sum m x cross p   (conserved by central forces)
 *   t  = cosmic time elapsed since the run's first row.
 * flags bit 0: a NaN or Inf was seen in this row's sums.                  */
typedef struct {
    double a, t, K, U, LI;
    double P[3];
    double L[3];
    uint32_t flags;
    uint32_t reserved;
} colatus_diag;

/* ---- entry points ------------------------------------------------------ */

/* Pair sum of Eq. (1) (Section II) for every particle.
 *   x    [3][N] device, m [N] device.
 *   acc  [3][N] device, out: a^-3 G sum_{j != k} m_j (x_j - x_k) r^-3,
 *        r = sqrt(|x_j - x_k|^2 + eps^2).
 *   phi  [N] device, out, or NULL: phi_k = -G sum_{j != k} m_j / r (comoving,
 *        no a factor); its negative gradient is the comoving pair sum.
 *   precision: COLATUS_FP64 / _MIXED_TWOSUM / _MIXED_F64ACC / _FP32.
 *   eps >= 0 (eps == 0 with two coincident particles gives Inf/NaN), G finite,
 *   a > 0.  batch: see colatus_batch, or NULL.
 *   attractor: see colatus_attractor, or NULL; its field (times a^-3) and
 *   potential are added to acc and phi, in FP64 for every precision.
 *   background: see colatus_background, or NULL; added the same way.       */
int colatus_forces(const double *x, const double *m, int64_t N, double eps,
                   double G, double a, int precision, double *acc, double *phi,
                   const colatus_batch *batch, const colatus_attractor *attractor,
                   const colatus_background *background, void *stream);

/* One kick-drift-kick step (Eq. (9) operators, Section II) from a to a_next,
 * in place on x and v (comoving position and dx/dt):
 *   p = a^2 v;  p += K(a, a_h) g(x);  x += D(a, a_next) p;
 *   p += K(a_h, a_next) g(x);  v = p / a_next^2,
 * with a_h = sqrt(a a_next), K(a1,a2) = int_{a1}^{a2} da/(a^2 H),
 * D(a1,a2) = int_{a1}^{a2} da/(a^3 H), H from Eq. (2).
 * Static limit H0 == 0: a stays fixed and a_next is read as the time step
 * dt (K = dt/(2a) each, D = dt/a^2).  With an attractor or a background
 * term (or NULL) g includes the Eq. (10) / Eq. (6) terms.
 *   g_cache: NULL, or a DEVICE [3][N] array holding g(x) at the entry
 *            positions (the comoving sum without a^-3, external terms
 *            included: what colatus_forces returns with a = 1, or what the
 *            previous colatus_step left there); the step uses it for the
 *            opening kick and overwrites it with g(x) at the new positions,
 *            so a sequence of steps costs one force evaluation each (NULL:
 *            two per step).  Must not alias x or v (COLATUS_EINVAL).
 * colatus_run makes many steps in one call (one evaluation per step).     */
int colatus_step(double *x, double *v, const double *m, int64_t N, double eps,
                 double G, double H0, double Om_R, double Om_M, double Om_K,
                 double Om_L, double a, double a_next, int precision, double *g_cache,
                 const colatus_batch *batch, const colatus_attractor *attractor,
                 const colatus_background *background, void *stream);

/* Steps first_step .. last_step-1 of the global grid a_n = a_begin
 * exp(n ln(a_end/a_begin)/n_steps), a_{n_steps} = a_end, in place on x, v.
 * Running [0, k) then [k, n_steps) matches one [0, n_steps) run up to the
 * rounding of the p <-> v conversion at the seam.
 * Static limit H0 == 0: a stays at a_begin and a_end is read as the total
 * elapsed time (dt = a_end / n_steps).
 *   diag: HOST array of (last_step - first_step + 1) rows, or NULL.  When
 *         non-NULL the call synchronises the stream and returns
 *         COLATUS_ENONFINITE if any row saw a NaN/Inf.  With a batch, diag
 *         holds n_boxes consecutive blocks of rows (box-major).
 * Requires n_steps >= 1, 0 <= first_step < last_step <= n_steps, a_begin > 0,
 * a_end > 0 (or > 0 elapsed time in the static limit), H^2 > 0 on the range
 * (else COLATUS_EFRIEDMANN).  The steps are launched on the stream as they
 * are queued; with COLATUS_OPT_GRAPH = 1, a call of 256 steps or more also
 * captures 16 steps in a graph that this and later calls with the same
 * arguments and buffers replay (the same kernels and arguments, so the same
 * bits).  attractor (or NULL): the Eq. (10) term joins g
 * at every kick and its energy joins U; so does the Eq. (6) background
 * term (or NULL).  tracks (or NULL): see colatus_tracks; rows r >= 1 hold
 * v = p / a^2 as the final v does.                                          */
int colatus_run(double *x, double *v, const double *m, int64_t N, double eps,
                double G, double H0, double Om_R, double Om_M, double Om_K,
                double Om_L, double a_begin, double a_end, int64_t n_steps,
                int64_t first_step, int64_t last_step, int precision,
                colatus_diag *diag, const colatus_batch *batch,
                const colatus_attractor *attractor,
                const colatus_background *background, const colatus_tracks *tracks,
                void *stream);

/* The paper's own difference equations, Eqs. (3)-(5) (after Hockney and
 * Eastwood), on the grid of colatus_run, in place on x and v:
 *   x^{n+1/2} = x^n + tau v^n / 2
 *   v^{n+1}   = v^n (1 - H tau)/(1 + H tau) + g(x^{n+1/2}) tau / (a^3 (1 + H tau))
 *   x^{n+1}   = x^{n+1/2} + tau v^{n+1} / 2
 * with g the comoving sum of Eq. (1) (attractive sign; plus the attractor if
 * given), tau the cosmic time of the step and H, a at its half time
 * t^n + tau/2.  The paper notes this scheme is not symplectic; it is offered
 * beside the kick-drift-kick step for that comparison (diagnostics rows as in
 * colatus_run; each row costs one more pair sweep with the potential, at the
 * integer-point positions).  One pair sweep per step, launched without
 * graph capture.  Arguments, limits and errors as colatus_run (tracks: the
 * state at the integer points, x^n and v^n).                              */
int colatus_run_he(double *x, double *v, const double *m, int64_t N, double eps,
                   double G, double H0, double Om_R, double Om_M, double Om_K,
                   double Om_L, double a_begin, double a_end, int64_t n_steps,
                   int64_t first_step, int64_t last_step, int precision,
                   colatus_diag *diag, const colatus_batch *batch,
                   const colatus_attractor *attractor,
                   const colatus_background *background, const colatus_tracks *tracks,
                   void *stream);

/* Periodic boundaries (Section II solves the motion equations in a periodic
 * box; the printed force loop is an open all-pairs sum, so the method is
 * not given there): the periodic comoving field by Ewald summation, for one
 * box of side `box` (comoving) holding all N particles, its images filling
 * space and the mean density removed (the field of the density contrast):
 *   acc_k = a^-3 G sum_{j != k} m_j E(x_j - x_k),
 *   E(d)  = sum_n (d + nL) C(alpha |d + nL|) / |d + nL|^3
 *           + (4 pi / L^3) sum_{q != 0} q / q^2 exp(-q^2 / 4 alpha^2) sin(q . d),
 *   C(u)  = erfc(u) + (2u / sqrt(pi)) exp(-u^2),  q = 2 pi n / L,
 * which does not depend on alpha; the nearest image d* of each pair takes
 * the Plummer law of Eq. (1): + d* [(|d*|^2 + eps^2)^{-3/2} - |d*|^{-3}]
 * (0 at d* = 0; at an exact half-box tie the image rint() picks).
 *   phi_k = -G [sum_{j != k} m_j Psi(x_j - x_k) + m_k Psi_self], with Psi the
 * matching potential (real part erfc(alpha r)/r, the nearest image's
 * Plummer correction, reciprocal part exp(-q^2/4 alpha^2)/q^2 cos(q . d),
 * constant -pi / (alpha^2 L^3)) and Psi_self the particle's own images and
 * background (-2.8372974794806 / L for one particle: the simple cubic
 * Madelung constant).  The library takes alpha and the cutoffs so that the
 * neglected real-space images and reciprocal terms fall below 1e-15 (FP64)
 * or 3e-9 (FP32 forms) of the kernel: real space on the nearest image only
 * (the pair sweep's symmetric loop, in the given precision; FP32 pairs
 * take coordinates rounded to multiples of L / 2^32 and the nearest image
 * of those, an exact tie along an axis giving -L/2), reciprocal
 * space in FP64 by structure factors.  No external terms; one box; 1 <= N
 * <= 262144; box > 0 finite, else COLATUS_EINVAL.  Other arguments as
 * colatus_forces.                                                         */
int colatus_forces_periodic(const double *x, const double *m, int64_t N, double eps,
                            double G, double a, double box, int precision, double *acc,
                            double *phi, void *stream);

/* Kick-drift-kick steps [first_step, last_step) of colatus_run's grid with
 * the periodic field of colatus_forces_periodic; after every drift each
 * coordinate is wrapped into [0, box).  diag: as colatus_run (U from the
 * periodic potential; P is conserved, L is not, with periodic boundaries).
 * Launched eagerly (one real-space sweep and the reciprocal-space kernels
 * per step).  Arguments, limits and errors as colatus_run and
 * colatus_forces_periodic.                                                 */
int colatus_run_periodic(double *x, double *v, const double *m, int64_t N, double eps,
                         double G, double H0, double Om_R, double Om_M, double Om_K,
                         double Om_L, double box, double a_begin, double a_end,
                         int64_t n_steps, int64_t first_step, int64_t last_step,
                         int precision, colatus_diag *diag, void *stream);

/* Velocity power spectrum of each tracer of a track (the power spectrum of
 * a single particle's velocity series that Section I names as the method's
 * goal): the periodogram over the track's rows,
 *   out[t][k] = (1/rows) sum_c | sum_{n < rows} w_c[n] exp(-2 pi i k n / rows) |^2,
 *   k = 0 .. rows/2,  w_c[n] = v_c of tracer t at row n, less its mean over
 *   the rows if remove_mean != 0.
 * The rows are grid points uniform in ln a, so k counts cycles per `rows`
 * grid steps.  Parseval: out[t][0] + 2 sum_{0<k<rows/2} out[t][k]
 * (+ out[t][rows/2] for even rows) = sum_n |w[n]|^2.
 *   track: DEVICE [rows][2][3][n_tracers] (as colatus_tracks.out).
 *   out:   DEVICE [n_tracers][rows/2 + 1], written.
 * FP64 throughout; the phase k n is reduced modulo rows exactly before the
 * twiddle factor is formed.  A direct transform: cost ~ rows^2 n_tracers.
 * 1 <= rows <= 131072 and 1 <= n_tracers <= 65536, else COLATUS_EINVAL.   */
int colatus_velocity_spectrum(const double *track, int64_t rows, int32_t n_tracers,
                              int remove_mean, double *out, void *stream);

/* Reverse-mode derivative of the full run [0, n_steps) of colatus_run
 * (discretise-then-differentiate: the exact gradient of the computed map).
 * For each of n_cot cotangent pairs (lam_xN[c], lam_vN[c]), each [3][N],
 * on the end state (x_N, v_N), writes grad_x0[c] = d<lam, state_N>/dx_0 and
 * grad_v0[c] = d<lam, state_N>/dv_0, each [3][N]; arrays are [n_cot][3][N]
 * device.  x0, v0 are not modified; xN, vN ([3][N] device, or NULL) receive
 * the forward end state.  The forward run stores (x, p) every
 * checkpoint_every steps and recomputes each segment, bitwise, during the
 * reverse sweep (one more force sweep per step); checkpoint_every == 0
 * keeps every position of the forward run instead (24 B x N x (n_steps + 1)
 * of device memory, 158 MB for 200 steps at N = 32768) and recomputes
 * nothing: the same bits, one force sweep per step fewer; -1 chooses: every
 * position if they take at most a quarter of the free device memory, else
 * segments of ceil(sqrt(n_steps)) steps.  checkpoint_every < -1 is
 * COLATUS_EINVAL.  The transpose Jacobian of the pair sum,
 *   (J^T lam)_k = G sum_{j != k} M(d)(m_k lam_j - m_j lam_k),
 *   M(d) = r^-3 I - 3 r^-5 d d^T,  d = x_j - x_k,
 * is evaluated by its own O(N^2) pair sweep in the given precision, once
 * per step for all cotangents together.  1 <= n_cot <= 4096.  batch: see
 * colatus_batch, or NULL (the boxes do not interact, so each box's
 * cotangents move only its own particles' gradients).
 * With an attractor (Eq. (10), or NULL) the run is the attractor's run; its
 * transpose Jacobian -S M(d) (d = x_psi - x_k) joins the pair sum's, and
 * grad_attractor ([n_cot][4] device, or NULL; requires an attractor)
 * receives d<lam, state_N>/dS and d<lam, state_N>/dx_psi per cotangent,
 * accumulated in a fixed order (deterministic).  With a background term
 * (Eq. (6), or NULL) its transpose Jacobian b I joins as well.              */
int colatus_adjoint(const double *x0, const double *v0, const double *m,
                    int64_t N, double eps, double G, double H0, double Om_R,
                    double Om_M, double Om_K, double Om_L, double a_begin,
                    double a_end, int64_t n_steps, int64_t checkpoint_every,
                    int32_t n_cot, const double *lam_xN, const double *lam_vN,
                    double *grad_x0, double *grad_v0, double *xN, double *vN,
                    double *grad_attractor, int precision,
                    const colatus_batch *batch, const colatus_attractor *attractor,
                    const colatus_background *background, void *stream);

/* colatus_forces without any allocation, for callers that cannot allocate
 * device memory: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and results as colatus_forces with
 * batch == NULL (one box).  It always runs the symmetric pair loop in 2x2
 * groups: with COLATUS_OPT_PAIR_FORM = 2 (and the other options at their
 * defaults) the two give the same bits; at the default pair form, boxes
 * too small to fill the GPU with symmetric items (up to about 11 000
 * particles) take the ordered loop in colatus_forces, and the two agree to
 * the precision's rounding.  The call allocates nothing and copies nothing from the host: its
 * scratch (work items, blocks, the box's common mass, the partial-sum slots)
 * is one fixed device array of about 17.4 MB, which every device the library
 * runs on holds from the library's load until the process ends.  Limit:
 * 1 <= N <= 16384 in every precision (N > 16384: COLATUS_ESCRATCH, nothing
 * queued).  Every call on a device shares that device's array, which keeps
 * the last call's contents: calls that overlap in time on one device (other
 * streams, other host threads) race and give undefined results; calls on
 * one stream are ordered and safe.                                          */
int colatus_forces_noalloc(const double *x, const double *m, int64_t N, double eps,
                           double G, double a, int precision, double *acc, double *phi,
                           const colatus_attractor *attractor,
                           const colatus_background *background, void *stream);

/* Finite-time Lyapunov exponents of tracer particles, the measure of the
 * chaotic advection that Sections I and IV motivate the method with.  For
 * tracer t (HOST array tracers[n_tracers] of particle indices, global with a
 * batch), the 3x3 block B_t = d x_t(a_end) / d x_t(a_begin) of the run's
 * flow map is read off the discrete adjoint of colatus_run [0, n_steps)
 * seeded with the unit vectors on x_t(a_end) (3 cotangents per tracer, all
 * tracers in one adjoint pass); then, in the library, in FP64:
 *   sigma_t = largest singular value of B_t (square root of the largest
 *             eigenvalue of B_t^T B_t, cyclic Jacobi rotations),
 *   lambda_t[t]   = ln sigma_t / (t(a_end) - t(a_begin)),
 *   lambda_lna[t] = ln sigma_t / ln(a_end / a_begin)   (NaN if H0 == 0),
 *   blocks[t][i][j] = (B_t)_{ij}.
 * The cosmic time span is the sum of the run's step times in grid order
 * (what the diagnostics' t reports; a_end itself in the static limit).
 *   lambda_t: DEVICE [n_tracers], written; lambda_lna, blocks: DEVICE
 *   [n_tracers] and [n_tracers][3][3], or NULL.
 * Other arguments, precision, checkpointing and the external terms as in
 * colatus_adjoint.  1 <= n_tracers <= 1365 and every index in [0, N), else
 * COLATUS_EINVAL.  Device scratch: the adjoint's, with 3 n_tracers
 * cotangents (about 0.45 GB at N = 32768 and 64 tracers).                  */
int colatus_ftle(const double *x0, const double *v0, const double *m, int64_t N,
                 double eps, double G, double H0, double Om_R, double Om_M,
                 double Om_K, double Om_L, double a_begin, double a_end, int64_t n_steps,
                 int64_t checkpoint_every, int32_t n_tracers, const int64_t *tracers,
                 double *lambda_t, double *lambda_lna, double *blocks, int precision,
                 const colatus_batch *batch, const colatus_attractor *attractor,
                 const colatus_background *background, void *stream);

/* Cosmic time elapsed over the grid of colatus_run, t(a_end) - t(a_begin) =
 * sum over steps of int dt (Eq. (2), Gauss-Legendre in ln a per step, the
 * same arithmetic as the run's coefficients), summed in grid order: the
 * value the last diagnostics row's t holds after a full run.  Static limit
 * H0 == 0: a_end (the elapsed time as given).  *t: HOST, written.  The call
 * synchronises the stream.  Arguments as colatus_run.                      */
int colatus_cosmic_time(double a_begin, double a_end, int64_t n_steps, double H0,
                        double Om_R, double Om_M, double Om_K, double Om_L, double *t,
                        void *stream);

/* Transpose-Jacobian product of the comoving sum g (Eq. (1) without a^-3,
 * plus the Eq. (10) attractor's field and the Eq. (6) background term when
 * given):
 * out[c] = J(x)^T lam[c] for n_cot cotangents, arrays [n_cot][3][N]
 * device.  The building block of colatus_adjoint.                         */
int colatus_force_vjp(const double *x, const double *m, int64_t N, double eps,
                      double G, int32_t n_cot, const double *lam, double *out,
                      int precision, const colatus_attractor *attractor,
                      const colatus_background *background, void *stream);

/* Hubble rate of Eq. (2) at scale factor a, on the host.  Returns
 * COLATUS_EFRIEDMANN if H^2 < 0 there.                                    */
int colatus_hubble(double a, double H0, double Om_R, double Om_M, double Om_K,
                   double Om_L, double *H);

/* Human-readable name of a return code (static string).                  */
const char *colatus_strerror(int code);

/* ---- tuning, timing and housekeeping ----------------------------------- */
#define COLATUS_OPT_GRAPH      1  /* 1: colatus_run calls of 256 steps or more capture
                                     16 steps in a hipGraph, kept per (stream, kernel
                                     arguments) and replayed by later calls of 16
                                     steps or more; 0 (default): every step launched
                                     eagerly (replay measured no faster on gfx950,
                                     and the first capture costs a few ms)           */
#define COLATUS_OPT_TIMER      2  /* 1: bracket every pair-sweep and integrator launch
                                     with hipEvents on its stream (default 0; the run
                                     then launches eagerly instead of from a graph)  */
#define COLATUS_OPT_AUTOTUNE   3  /* 1: time candidate tile shapes on first use of an
                                     (N bucket, precision) and keep the fastest
                                     (default 0: built-in heuristic)                 */
#define COLATUS_OPT_TILE_R     4  /* >0: force targets per lane of the forward sweep
                                     (forms 0, 1: 1, 2, 4; form 2: 4 or 8 with 64
                                     threads, or 4 with 128 for FP32 pairs; 4 with
                                     64, or 2 with 128 for FP64); 0 = auto          */
#define COLATUS_OPT_TILE_TPB   5  /* >0: force threads per block of the forward sweep
                                     (forms 0, 1: 128, 256; form 2: see TILE_R);
                                     0 = auto.  An unsupported combination makes
                                     the forward calls return COLATUS_EINVAL         */
#define COLATUS_OPT_TILE_SLICES 6 /* >0: force the number of source slices (forms 0,
                                     1; form 2 derives its slots from the parts);
                                     0 = auto                                        */
#define COLATUS_OPT_PERSISTENT 7  /* 1: persistent pair-sweep grid (about one resident
                                     round of workgroups) pulling LPT-ordered work
                                     items from a device counter; 0 (default): one
                                     workgroup per work item, in the same LPT order,
                                     left to the hardware dispatcher (measured
                                     faster on gfx950)                               */
#define COLATUS_OPT_PAIR_FORM  8  /* pair loop: 0 = ordered pairs, weight
                                     m r^-1 (r^-1)^2; 1 = ordered pairs, weight
                                     m r^-1 rcp(r^2) (one VALU multiply fewer, one
                                     more transcendental; the adjoint treats 1 as 0);
                                     2 = symmetric: each unordered pair once,
                                     applied to both particles (the forward and
                                     adjoint pair terms change sign when the two
                                     particles swap), boxes cut into parts of
                                     R x threads particles; -1 (default) = the
                                     heuristic's or the autotuner's choice (2 for
                                     the forward up to 2^18 particles per box and
                                     for the adjoint with up to 3 cotangents, else
                                     0).  FP64 pairs: 1 means 0                      */
#define COLATUS_OPT_ROCTX      9  /* 1: a roctx range around every call, named after
                                     the entry point, and one per step of the
                                     eagerly launched loops (graph-replayed steps
                                     fall inside their call's range), for
                                     rocprofv3 --marker-trace; 0 (default): none */
#define COLATUS_OPT_PAIR_GROUP 10 /* 1 (default): the forward symmetric loop with 4
                                     targets per lane and 64 threads runs 2x2 blocks
                                     of part pairs in one workgroup of four waves,
                                     adding the two partial sums of each target
                                     part and of each source part before writing,
                                     so every particle gets ceil(P/2) + 1 partial-sum
                                     slots instead of P (P parts of 256 in its box);
                                     0: one item per workgroup, P slots.  The sums
                                     differ by the rounding of those additions  */
int colatus_set_option(int key, int64_t value);
int colatus_get_option(int key, int64_t *value);

/* Kernel timer: sum of hipEvent durations (on the launching stream) of the
 * forward pair-sweep (kind 0), adjoint pair-sweep (kind 1) or run
 * integrator (kind 2) launches recorded since the last reset, and their
 * count.  Synchronises the recorded events.  reset != 0 clears.           */
int colatus_timer_read(int kind, double *total_ms, int64_t *launches, int reset);

/* Tile shape the library would use (or has tuned) for N particles in one
 * box at the given precision: out[0] = targets per lane R, out[1] = threads
 * per block, out[2] = source slices (form 2: the parts P of R x threads
 * particles), out[3] = pair-loop form (see COLATUS_OPT_PAIR_FORM).  kind 0 =
 * forward, 1 = adjoint.  A forward form 2 with R = 4 and 64 threads runs in
 * 2x2 groups of part pairs while COLATUS_OPT_PAIR_GROUP is 1, and then
 * writes ceil(P/2) + 1 partial-sum slots per particle (P = 1: one) instead
 * of P.                                                                    */
int colatus_tile_config(int64_t N, int precision, int kind, int32_t out[4]);

/* Release all cached device scratch of every (device, stream) workspace,
 * after synchronising each of those streams, and the pooled timer events.
 * Tuned tile shapes, options and unread timer records are kept.  The next
 * call on a stream allocates its scratch again.  The calling thread's
 * current device is restored before return.  Always returns COLATUS_OK
 * (cleanup errors are ignored); with no HIP device it does nothing.        */
int colatus_release(void);

/* Library version, major*10000 + minor*100 + patch.                      */
int colatus_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COLATUS_H */
