// Internal declarations shared by the HIP translation units of libcolatus.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "colatus.h"

namespace colatus {

// One unit of the O(N^2) pair sweep: a block of target particles of one box
// against a contiguous slice of that box's source particles.  The sweep
// writes its partial sums into slot `slice` of the partial-sum buffer.  In
// the symmetric form (form 2) a box is cut into parts; kind 0 pairs part p
// (targets) with part q > p (sources): p's partial from q goes to slot
// `slice`, q's reaction from p to slot `rslice`; kind 1 is a piece of one
// part's targets against that whole part (no reaction).  One item per
// workgroup: slice = q, rslice = p, diagonal slot p.  Grouped (four waves
// per workgroup): slots numbered by super-part (build_symmetric_groups).
struct WorkItem {
    int64_t i0, i1;   // targets [i0, i1)
    int64_t j0, j1;   // sources [j0, j1)
    double eps2;      // squared softening of the box
    int32_t slice;    // partial-sum slot of the targets
    int32_t box;
    int32_t rslice;   // partial-sum slot of the sources' reaction (form 2)
    int16_t kind;     // form 2: 0 = pair of parts, 1 = piece of a diagonal,
                      // -1 = padding of a group (grouped form)
    int8_t tmate;     // grouped form: 1 if the targets' partial sums are added
                      // to those of wave (this wave ^ 1) of the group
    int8_t rmate;     // grouped form: 1 if the reactions are added to those of
                      // wave (this wave ^ 2) of the group
};

// Up to kIntBlock particles of one box, for the O(N) kernels (finalise,
// kick/drift, diagnostics).  Blocks never straddle a box boundary.
constexpr int kIntBlock = 64;
struct IntBlock {
    int64_t i0, i1;
    double eps;       // softening of the box (self-term of the potential)
    int32_t box;
    int32_t n_slices; // partial-sum slots written for this box
};

// Coefficients of step n of a run (Eq. (9) integrals), and of the paper's
// difference equations, Eqs. (3)-(5), on the same grid.
struct StepCoef {
    double k1;   // int_{a_n}^{a_n+1/2} dt / a
    double d;    // int_{a_n}^{a_n+1} dt / a^2
    double k2;   // int_{a_n+1/2}^{a_n+1} dt / a
    double dt;   // cosmic time of the step (tau of Eqs. (3)-(5))
    double a0;   // a_n
    double a1;   // a_{n+1}
    double ah;   // a at the half time t_n + dt/2 (Eqs. (3)-(5))
    double Hh;   // H(ah)
};

enum Precision { kFP64 = 0, kMixedTwoSum = 1, kMixedF64Acc = 2, kFP32 = 3 };

// How the O(N) readers add a particle's partial-sum slots (one slot per part
// or source slice):
//   kSlotF64        FP64 slots (already scaled by the box's common mass),
//                   summed in FP64;
//   kSlotF32Fold64  FP32 slots (one FP32 sum of at most 256 pair terms each,
//                   without the mass), summed in FP64;
//   kSlotF32TwoSum  FP32 slots, summed in an unevaluated FP32 pair (hi, lo)
//                   by TwoSum (compensated FP32 accumulation);
//   kSlotF32Direct  FP32 slots, summed in one FP32 running sum.
enum SlotMode { kSlotF64 = 0, kSlotF32Fold64 = 1, kSlotF32TwoSum = 2, kSlotF32Direct = 3 };

// hi + lo += v with the rounding error of hi + v carried into lo (TwoSum,
// Knuth): hi + lo then holds the running sum to about twice FP32 precision.
__device__ __forceinline__ void two_sum_add(float &hi, float &lo, float v)
{
    float s = hi + v;
    float bp = s - hi;
    float err = (hi - (s - bp)) + (v - bp);
    hi = s;
    lo += err;
}

// FP64 1/sqrt(s) for s > 0 finite: the hardware estimate (v_rsq_f64, about
// 5e-8 relative on gfx950) refined by one Newton step,
//   y1 = y0 + (y0 / 2) (1 - s y0^2),
// which squares the error (measured maximum 4e-15 relative over 2^-60..2^20).
// Every FP64 kernel that must reproduce another's r^-1 bit for bit uses this.
__device__ __forceinline__ double rsqrt_refined(double s)
{
    const double y0 = __builtin_amdgcn_rsq(s);
    const double e = fma(-s * y0, y0, 1.0);
    return fma(0.5 * y0, e, y0);
}

// External terms added to the comoving sum g of every particle, each with
// its potential counted once in the energy:
// * the deformation attractor of Eq. (10) (on != 0): a fixed point of
//   strength S = C psi at comoving (x, y, z) adding S d (|d|^2 + eps^2)^{-3/2},
//   d = x_psi - x_k (eps: the particle's box softening), potential
//   -S / sqrt(|d|^2 + eps^2);
// * the background term of Eq. (6) (bg != 0): b (x_k - c), potential
//   -b |x_k - c|^2 / 2 (the mean matter density's pull removed about the
//   centre c; b = Om_M H0^2 / 2 makes it consistent with Eq. (2)).
// Both scale with a like the pair sum.
struct ExtField {
    int on;
    double S, x, y, z;
    int bg;
    double b, cx, cy, cz;
};

// Host checks of the Eq. (10) attractor and Eq. (6) background arguments of
// an entry point (NULL: none); COLATUS_EINVAL on a non-finite value.
int resolve_external(const colatus_attractor *a, const colatus_background *bg, ExtField &out);

// Shape of one pair-sweep launch.
struct TileCfg {
    int R;        // targets per lane
    int tpb;      // threads per block (= sources per LDS tile in forms 0, 1)
    int slices;   // source slices per box (form 2: parts of R * tpb particles)
    int form;     // FP32 pair-loop form (see launch_pair_sweep); 0 for FP64
    int group = 0; // form 2 with R = 4, tpb = 64: 2x2 groups of part pairs
                   // per workgroup of four waves (pair_sweep_sym_grp_kernel)
};

// How the readers add the slots a sweep of this shape writes (SlotMode).
// The symmetric form with FP32 pairs and parts of at most 256 particles
// writes FP32 slots (each one FP32 sum of at most 256 terms), and the
// precision then chooses the accumulation over the slots: TwoSum
// (MIXED_TWOSUM), FP64 (MIXED_F64ACC) or plain FP32 (FP32); every other
// sweep writes FP64 slots, summed in FP64.
inline int slot_mode_for(const TileCfg &cfg, int precision)
{
    if (!(cfg.form == 2 && precision != kFP64 && cfg.R * cfg.tpb <= 256))
        return kSlotF64;
    if (precision == kMixedTwoSum)
        return kSlotF32TwoSum;
    if (precision == kFP32)
        return kSlotF32Direct;
    return kSlotF32Fold64;
}

// Diagnostics partial row written per IntBlock: K*a^2*2, sum m phi, P[3], L[3],
// non-finite flag (as a double), padding.
constexpr int kDiagW = 10;

// ---- launchers (each returns the launch's hipError_t) -------------------

// Forward pair sweep: part[s][3][N] = sum over the item's sources of
// m_j (x_j - x_k) r^-3, and part_phi[s][N] = sum m_j / r when with_phi.
// form 0: w = m r^-1 (r^-1)^2; form 1: w = m r^-1 rcp(s) (FP32 only);
// form 2: symmetric items (FP32 only; R in {4, 8}, tpb in {64, 128}), each
// unordered pair evaluated once and applied to both particles.
// box_mass[b]: common mass of box b or NaN (see launch_box_mass), or null.
// step_inc: if non-null, the sweep's first thread adds 1 to *step_inc (the
// run's step counter; nothing in the sweep reads it).
hipError_t launch_pair_sweep(int precision, int form, const TileCfg &cfg, bool with_phi,
                             bool mask_self, const double *x, const double *m,
                             int64_t N, const WorkItem *items, int n_items,
                             int *counter, bool persistent, const double *box_mass,
                             double *part, double *part_phi, int64_t *step_inc,
                             hipStream_t stream);

// box_mass[b] = m of box b if all its masses are equal and positive, else NaN
// (box_offsets: device, n_boxes + 1 entries ending at N).
hipError_t launch_box_mass(const double *m, const int64_t *box_offsets, int n_boxes, int64_t N,
                           double *box_mass, hipStream_t stream);

// Adjoint pair sweep for n_cot cotangents lam [n_cot][3][N]:
// part[s][c][3][N] = sum over the item's sources of M(d)(m_k lam_j - m_j lam_k).
hipError_t launch_adjoint_sweep(int precision, const TileCfg &cfg, bool mask_self,
                                const double *x, const double *m, int64_t N,
                                int n_cot, const double *lam,
                                const WorkItem *items, int n_items, int *counter,
                                bool persistent, const double *box_mass, double *part,
                                hipStream_t stream);

// Sets *counter = 0 (graph-safe replacement for a memset node).
hipError_t launch_zero_counter(int *counter, hipStream_t stream);

// Partial-sum slots: FP64, already multiplied by the box's common mass, or
// (slot_mode != kSlotF64: the symmetric loop with FP32 pairs and parts of at
// most 256) FP32 without it, the buffer then read as float; readers add the
// slots as the SlotMode slot_mode says and apply the mass in FP64.

// acc = scale * sum_s part[s] + inv_a3 f_att(x), phi = -G (sum_s part_phi[s] -
// m/eps) + phi_att(x).  With kick_v: also the closing half kick of a cached
// step from that acc, kick_v = (kick_p + k2 acc) / a1^2 (kick_coef[0]).
hipError_t launch_forces_finalize(int precision, const double *box_mass,
                                  const IntBlock *blocks, int n_blocks,
                                  const double *part, const double *part_phi, int slot_mode,
                                  const double *x, const double *m, int64_t N, double G,
                                  double scale, const ExtField &ext, double inv_a3,
                                  double *acc, double *phi, hipStream_t stream,
                                  const double *kick_p = nullptr, double *kick_v = nullptr,
                                  const StepCoef *kick_coef = nullptr);

// out = G * sum_s part[s] - S M(d) lam (attractor) for n_cot cotangents
// ([n_cot][3][N]).
hipError_t launch_vjp_finalize(const IntBlock *blocks, int n_blocks, const double *part,
                               int slot_mode, const double *box_mass, const double *x,
                               const double *lam, const ExtField &ext, int64_t N, int n_cot,
                               double G, double *out, hipStream_t stream);

// Step coefficients of steps [first, last) of the global grid.  half_time:
// also solve the half-time point (ah, Hh) of Eqs. (3)-(5), else leave it NaN.
hipError_t launch_coefficients(double H0, double OmR, double OmM, double OmK, double OmL,
                               double a_begin, double a_end, int64_t n_steps,
                               int64_t first, int64_t last, int half_time, StepCoef *coef,
                               hipStream_t stream);

// p = a_first^2 v (mode 0) or v = p / a^2 (mode 1) over all particles.
hipError_t launch_convert(int mode, const double *src, double *dst, int64_t N,
                          const StepCoef *coef, int64_t idx, hipStream_t stream);

struct IntegrateArgs {
    double *x;             // [3][N], in/out
    double *p;             // [3][N], in/out (canonical momentum a^2 v)
    const double *m;
    const double *part;    // [S][3][N]
    const double *part_phi;// [S][N] or null
    const IntBlock *blocks;
    int n_blocks;
    int64_t N;
    double G;
    const StepCoef *coef;  // indexed by (n - first)
    const int64_t *step;   // device run descriptor {n, first, last}: the
                           // absolute step counter n (advanced by the next
                           // pair sweep or a tick kernel) and the call's step
                           // range; kept in device memory so that a captured
                           // step graph does not depend on the range
    int *work_counter;     // pair-sweep work counter, re-armed here (or null)
    double *diag_part;     // [rows][n_blocks][kDiagW] or null
    int precision;         // pair arithmetic of the sweep that wrote part_phi
    const double *box_mass;// per-box common mass or NaN (as given to the sweep)
    int slot_mode;          // SlotMode of the slots (see above)
    ExtField ext;          // external terms added to g (Eqs. (10), (6))
    const int32_t *track_slot = nullptr; // [N]: tracer number of each particle or -1
    double *track = nullptr;   // [rows][2][3][n_tracers]: rows n > first are written here
    int32_t n_tracers = 0;
    // periodic boundaries: the reciprocal-space field [3][N] and potential
    // part [N] at x_n (launch_ewald_kspace), added to the slots' sums; after
    // the drift every coordinate is wrapped into [0, box) (box > 0)
    const double *ewald_g = nullptr;
    const double *ewald_p = nullptr;
    double box = 0.0;
};
// Finalise g(x_n) from the partials, then kick by k2_{n-1} (n > first),
// record diagnostics of the state at a_n, and (n < last) kick by k1_n and
// drift by d_n.  Reads n from *step and re-arms the pair-sweep work counter
// for the sweep that follows (graph-safe, no memset).
hipError_t launch_integrate(const IntegrateArgs &args, hipStream_t stream);

// *step += 1; *counter = 0.
hipError_t launch_tick(int64_t *step, int *counter, hipStream_t stream);

// ---- the paper's difference equations, Eqs. (3)-(5) ------------------------
// x += f * coef[idx].dt * v over all particles (the opening half drift).
hipError_t launch_he_drift(double *x, const double *v, int64_t N, const StepCoef *coef,
                           int64_t idx, double f, hipStream_t stream);

struct HEArgs {
    double *x;             // [3][N]: x^{n+1/2} in; x^{n+3/2} (or x^{n+1} at the end) out
    double *v;             // [3][N]: v^n in, v^{n+1} out
    double *xi;            // [3][N] or null: receives x^{n+1}
    const double *part;    // slots of the sweep at x^{n+1/2}
    int slot_mode;
    const IntBlock *blocks;
    int n_blocks;
    int64_t N;
    double G;
    const StepCoef *coef;  // indexed by row
    int64_t row;           // n - first
    int last;              // n + 1 == last step of the call
    const double *box_mass;
    ExtField ext;
    const int32_t *track_slot = nullptr; // as in IntegrateArgs: row + 1 (x^{n+1}, v^{n+1})
    double *track = nullptr;
    int32_t n_tracers = 0;
};
// v = v (1 - H tau)/(1 + H tau) + g(x^{n+1/2}) tau / (a^3 (1 + H tau)) with H, a
// at the half time; x^{n+1} = x^{n+1/2} + tau v / 2; then the next step's
// opening half drift unless last.
hipError_t launch_he_step(const HEArgs &args, hipStream_t stream);

// One step with a cached force g (colatus_step with g_cache), coefficients
// coef[0]: mode 0 = opening kick and drift (p from v), mode 1 = closing kick
// and v from p.
hipError_t launch_cached_kick(int mode, double *x, double *v, double *p, const double *g,
                              int64_t N, const StepCoef *coef, hipStream_t stream);

// ---- tracer tracks ---------------------------------------------------------
// slot[i] = -1 for all N particles, then slot[idx[t]] = t.
hipError_t launch_track_slots(int32_t *slot, int64_t N, const int64_t *idx, int32_t T,
                              hipStream_t stream);
// One track row [2][3][T] from x and v (the start state): row[c][t] = x[c][idx[t]],
// row[3 + c][t] = v[c][idx[t]].
hipError_t launch_track_gather(const double *x, const double *v, int64_t N,
                               const int64_t *idx, int32_t T, double *row, hipStream_t stream);

// Velocity periodogram of each tracer over M track rows (spectrum.hip):
// out[t][k] = (1/M) sum_c |sum_n w_c[n] e^{-2 pi i k n / M}|^2, k <= M/2,
// w = v (less its mean if remove_mean).  twiddle: [M] double2 scratch.
hipError_t launch_velocity_spectrum(const double *track, int64_t M, int32_t T, int remove_mean,
                                    double *twiddle, double *out, hipStream_t stream);

// Diagnostics row `row` of the state (x, v) at scale factor a_of(row):
// row 0 -> coef[0].a0, row r > 0 -> coef[r - 1].a1; p = a^2 v; the potential
// from the PHI slots of a sweep at x (plus the attractor).
hipError_t launch_state_diag(const double *x, const double *v, const double *m,
                             const double *part_phi, int slot_mode, const IntBlock *blocks,
                             int n_blocks, int64_t N, double G, const StepCoef *coef,
                             int64_t row, int precision, const double *box_mass,
                             const ExtField &ext, double *diag_part, hipStream_t stream);

// Reduce per-block diagnostics rows per box and accumulate LI / t.
// out: [n_boxes][rows] rows of colatus_diag layout (as doubles, 14 each).
hipError_t launch_diag_reduce(const double *diag_part, int rows, const IntBlock *blocks,
                              int n_blocks, int n_boxes, const int32_t *box_first_block,
                              const StepCoef *coef, double H0, double *out,
                              hipStream_t stream);

// Adjoint update after a VJP sweep at x_n (all cotangents):
//   w = G sum_s part - S M(d) lam_p;  lam_x += cw * w;
//   then if do_drift: lam_p += dnext * lam_x.
// With the attractor on and att_acc non-null, block b also adds
// cw * (sum_k lam_p . f_k / S, sum_k S M(d_k) lam_p) over its particles to
// att_acc[b][c][0..4) (its own row only: deterministic, no atomics).
hipError_t launch_adjoint_update(const IntBlock *blocks, int n_blocks, const double *part,
                                 int slot_mode, const double *box_mass, const double *x,
                                 const ExtField &ext, double *att_acc, int64_t N, int n_cot,
                                 double G, double cw, double *lam_x, double *lam_p,
                                 int do_drift, double dnext, hipStream_t stream);

// out[c][q] = sum over blocks b (in order) of att_acc[b][c][q], q < 4.
hipError_t launch_att_grad_reduce(const double *att_acc, int n_blocks, int n_cot, double *out,
                                  hipStream_t stream);

// FTLE cotangents: lam[0..n) = 0, then for tracer t < T, component i < 3,
// lam[(3 t + i)][i][idx[t]] = 1 (lam is [3T][3][N]).
hipError_t launch_ftle_seed(double *lam, int64_t n, const int64_t *idx, int T, int64_t N,
                            hipStream_t stream);

// Finite-time Lyapunov exponents from the adjoint's position gradients
// grad [3T][3][N] (row 3t + i holds d x_i(end) of tracer idx[t] / d x_0):
// the tracer's block B[i][j] = grad[3t + i][j][idx[t]], sigma = its largest
// singular value (square root of the largest eigenvalue of B^T B, cyclic
// Jacobi in FP64), lam_t[t] = ln sigma / span_t, lam_lna[t] = ln sigma /
// span_lna (or null), blocks[t][i][j] = B[i][j] (or null).
hipError_t launch_ftle(const double *grad, const int64_t *idx, int T, int64_t N, double span_t,
                       double span_lna, double *lam_t, double *lam_lna, double *blocks,
                       hipStream_t stream);

// ---- periodic boundaries (Ewald summation) -------------------------------
// Real-space part: the symmetric work items (parts of 256, R = 4, one wave),
// each pair's nearest image, Plummer pair less the smooth long-range part
// (see pair_sweep.hip); slots as the symmetric loop's (FP32 for FP32 pairs,
// FP64 otherwise), masses included (readers take no common mass).
hipError_t launch_ewald_real(int precision, bool with_phi, const double *x, const double *m,
                             int64_t N, const WorkItem *items, int n_items, double *part,
                             double *part_phi, int64_t *step_inc, double L, double alpha,
                             hipStream_t stream);

// A run of consecutive n_z of one reciprocal-space column (nx, ny), its k
// values stored from k0 on.
constexpr int kEwaldSegLen = 16;
struct EwaldSeg {
    int nx, ny, z0, cnt, k0;
};

struct EwaldArgs {
    const double *x, *m;
    int64_t N;
    double L, alpha;
    const EwaldSeg *segs;  // [n_segs], k0 consecutive
    const EwaldSeg *segs_sk;  // [n_segs] the same segments, longest first (structure factors)
    int n_segs, K;
    const double *coef;    // [K]: 2 (4 pi / L^3) exp(-k^2 / 4 alpha^2) / k^2
    double2 *sk_part;      // [n_sk_chunks][K]
    int n_sk_chunks;
    double2 *S;            // [K]: W(k) = coef(k) S(k), the weighted structure factor
    int n_k_chunks;        // ranges of segments for the per-particle sums
    double *kpart_g;       // [n_k_chunks][3][N]
    double *kpart_p;       // [n_k_chunks][N]
    double *msum;          // [1]: total mass
    bool mass_ready;       // msum already holds the masses' sum (a run's later steps)
    double *gk;            // [3][N] out: reciprocal field (no G)
    double *pk;            // [N] out: reciprocal potential part + self and background terms
};
// The reciprocal-space field and potential part of every particle, with the
// self and background constants (ewald.hip).
hipError_t launch_ewald_kspace(const EwaldArgs &args, hipStream_t stream);

// acc += G inv_a3 gk; phi += -G pk (phi may be null).
hipError_t launch_ewald_add(const double *gk, const double *pk, int64_t N, double G,
                            double inv_a3, double *acc, double *phi, hipStream_t stream);

// p[0..n) = value (a fill kernel; graph-safe).
hipError_t launch_fill(double *p, int64_t n, double value, hipStream_t stream);

// lam_p = lam_v / aN^2 (mode 0) or grad_v = a0^2 lam_p (mode 1); n values.
hipError_t launch_scale(const double *src, double *dst, int64_t n, double factor,
                        hipStream_t stream);

}  // namespace colatus
