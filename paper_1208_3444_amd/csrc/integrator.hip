// O(N) kernels around the pair sweep: Friedmann step coefficients, the
// kick-drift-kick update in canonical momentum, diagnostics, and the
// finalisation of split-source partial sums.  All of them are bound by HBM
// traffic (or launch latency at small N): each reads and writes each
// particle's FP64 state once, coalesced, in structure-of-arrays planes.
#include "colatus_internal.h"

#include "colatus.h"

#include <math.h>

namespace colatus {
namespace {

// ---------------------------------------------------------------------------
// Friedmann equation (Eq. (2)) and the time integrals of the kick and drift
// operators (Eq. (9)), evaluated in s = ln a by composite 8-point
// Gauss-Legendre quadrature (sub-intervals of at most 0.05 in ln a):
//   cosmic time   int dt       = int ds / H
//   kick          int dt / a   = int e^-s  ds / H
//   drift         int dt / a^2 = int e^-2s ds / H
// ---------------------------------------------------------------------------
__constant__ double kGLx[4] = {0.18343464249564978, 0.52553240991632899, 0.79666647741362673,
                               0.96028985649753618};
__constant__ double kGLw[4] = {0.36268378337836177, 0.31370664587788705, 0.22238103445337434,
                               0.10122853629037669};

struct Cosmo {
    double H0, OmR, OmM, OmK, OmL;
};

__device__ double hubble(const Cosmo &c, double a)
{
    const double ia = 1.0 / a;
    const double ia2 = ia * ia;
    const double e2 = c.OmR * ia2 * ia2 + c.OmM * ia2 * ia + c.OmK * ia2 + c.OmL;
    return c.H0 * sqrt(e2);  // NaN when e2 < 0; the host rejects such ranges
}

// int_{s0}^{s1} e^{-q s} / H(e^s) ds for q = 0, 1, 2 at once.
__device__ void time_integrals(const Cosmo &c, double s0, double s1, double out[3])
{
    const double span = s1 - s0;
    int nsub = (int)ceil(fabs(span) / 0.05);
    if (nsub < 1)
        nsub = 1;
    const double h = span / nsub;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nsub; ++k) {
        const double mid = s0 + (k + 0.5) * h;
        for (int q = 0; q < 4; ++q) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double s = mid + sgn * 0.5 * h * kGLx[q];
                const double a = exp(s);
                const double wH = kGLw[q] / hubble(c, a);
                const double ia = 1.0 / a;
                acc[0] += wH;
                acc[1] += wH * ia;
                acc[2] += wH * ia * ia;
            }
        }
    }
    for (int q = 0; q < 3; ++q)
        out[q] = 0.5 * h * acc[q];
}

__global__ void coefficients_kernel(Cosmo c, double a_begin, double a_end, int64_t n_steps,
                                    int64_t first, int64_t last, int half_time, StepCoef *coef)
{
    const int64_t n = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= last)
        return;
    StepCoef s;
    if (c.H0 == 0.0) {
        const double dt = a_end / (double)n_steps;
        const double a = a_begin;
        s.k1 = 0.5 * dt / a;
        s.k2 = 0.5 * dt / a;
        s.d = dt / (a * a);
        s.dt = dt;
        s.a0 = a;
        s.a1 = a;
        s.ah = a;
        s.Hh = 0.0;
    } else {
        const double delta = log(a_end / a_begin) / (double)n_steps;
        const double a0 = a_begin * exp((double)n * delta);
        const double ah = a_begin * exp(((double)n + 0.5) * delta);
        const double a1 = (n + 1 == n_steps) ? a_end : a_begin * exp((double)(n + 1) * delta);
        const double s0 = log(a0), sh = log(ah), s1 = log(a1);
        double lo[3], hi[3];
        time_integrals(c, s0, sh, lo);
        time_integrals(c, sh, s1, hi);
        s.k1 = lo[1];
        s.k2 = hi[1];
        s.d = lo[2] + hi[2];
        s.dt = lo[0] + hi[0];
        s.a0 = a0;
        s.a1 = a1;
        // only the Eqs. (3)-(5) scheme reads ah and Hh
        s.ah = NAN;
        s.Hh = NAN;
        if (!half_time) {
            coef[n - first] = s;
            return;
        }
        // half time of Eqs. (3)-(5): solve int_{s0}^{u} ds / H = dt / 2 for
        // u = ln a by Newton's method (derivative 1/H), from the ln-a midpoint
        double u = sh;
        for (int it = 0; it < 8; ++it) {
            double t[3];
            time_integrals(c, s0, u, t);
            const double du = (t[0] - 0.5 * s.dt) * hubble(c, exp(u));
            u -= du;
            if (fabs(du) <= 1e-15 * fabs(u) + 1e-300)
                break;
        }
        s.ah = exp(u);
        s.Hh = hubble(c, s.ah);
    }
    coef[n - first] = s;
}

__global__ void convert_kernel(int mode, const double *__restrict__ src, double *__restrict__ dst,
                               int64_t n3, const StepCoef *__restrict__ coef, int64_t idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3)
        return;
    if (mode == 0) {
        const double a = coef[idx].a0;
        dst[i] = a * a * src[i];
    } else {
        const double a = coef[idx].a1;
        dst[i] = src[i] / (a * a);
    }
}

// One kick-drift-kick step with the force at its start given (the step
// with a cached force): mode 0, p = a_n^2 v, p += k1 g, x += d p; mode 1,
// p += k2 g, v = p / a_{n+1}^2.  The same operations, in the same order, as
// the conversion and integrate kernels of a run.  Elementwise over [3][N].
__global__ void cached_kick_kernel(int mode, double *__restrict__ x, double *__restrict__ v,
                                   double *__restrict__ p, const double *__restrict__ g,
                                   int64_t n3, const StepCoef *__restrict__ coef)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3)
        return;
    const StepCoef cf = coef[0];
    // explicit FMAs: the run's kernels contract their updates the same way
    if (mode == 0) {
        const double p0 = cf.a0 * cf.a0 * v[i];
        const double pi = fma(cf.k1, g[i], p0);
        x[i] = fma(cf.d, pi, x[i]);
        p[i] = pi;
    } else {
        const double pi = fma(cf.k2, g[i], p[i]);
        v[i] = pi / (cf.a1 * cf.a1);
    }
}

// Deterministic tree sum of kDiagW values over the first kIntBlock threads
// (every thread of the block calls it; the others contribute nothing).
__device__ void block_sum_rows(double (&v)[kDiagW], double (*sh)[kIntBlock])
{
    const int tid = threadIdx.x;
    if (tid < kIntBlock)
        for (int q = 0; q < kDiagW; ++q)
            sh[q][tid] = v[q];
    __syncthreads();
    for (int w = kIntBlock / 2; w > 0; w >>= 1) {
        if (tid < w) {
            for (int q = 0; q < kDiagW; ++q) {
                if (q == kDiagW - 1)
                    sh[q][tid] = fmax(sh[q][tid], sh[q][tid + w]);
                else
                    sh[q][tid] += sh[q][tid + w];
            }
        }
        __syncthreads();
    }
    for (int q = 0; q < kDiagW; ++q)
        v[q] = sh[q][0];
}

__device__ __forceinline__ bool finite3(double a, double b, double c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// The potential sweep includes the self pair j == k, whose term is exactly
// m_k * rsqrt(eps^2) as the sweep computed it (zero separation); subtract
// that same value, rounded the same way, so no FP32-vs-FP64 residue of a
// large self term is left in phi.  Equal-mass boxes (mbox not NaN) were
// summed without m and scaled by mbox in FP64.  With eps == 0 the sweep
// masks the self pair.
__device__ __forceinline__ double self_potential(int precision, double m, double eps,
                                                 double mbox)
{
    if (!(eps > 0.0))
        return 0.0;
    const double eps2 = eps * eps;
    if (precision == kFP64)
        return m * rsqrt_refined(eps2);
    const float r = __builtin_amdgcn_rsqf((float)eps2);
    if (!isnan(mbox))
        return mbox * (double)r;
    return (double)((float)m * r);
}

__device__ __forceinline__ double box_mass_of(const double *box_mass, int box)
{
    return box_mass ? box_mass[box] : NAN;
}

// Eq. (10) attractor at particle position (px, py, pz), softening eps: adds
// its field S d r^-3 (d = x_psi - x, r^2 = |d|^2 + eps^2) to f and returns
// its potential -S / r.  FP64 with IEEE square root and division.
__device__ __forceinline__ double attractor_pull(const ExtField &A, double px, double py,
                                                 double pz, double eps, double (&f)[3])
{
    const double dx = A.x - px, dy = A.y - py, dz = A.z - pz;
    const double s = dx * dx + dy * dy + dz * dz + eps * eps;
    const double r = sqrt(s);
    const double r3 = 1.0 / (s * r);
    f[0] += A.S * dx * r3;
    f[1] += A.S * dy * r3;
    f[2] += A.S * dz * r3;
    return -A.S / r;
}

// Background term of Eq. (6): adds b (x - c) to f and returns its potential
// -b |x - c|^2 / 2.
__device__ __forceinline__ double background_pull(const ExtField &E, double px, double py,
                                                  double pz, double (&f)[3])
{
    const double dx = px - E.cx, dy = py - E.cy, dz = pz - E.cz;
    f[0] += E.b * dx;
    f[1] += E.b * dy;
    f[2] += E.b * dz;
    return -0.5 * E.b * (dx * dx + dy * dy + dz * dz);
}

// Every external term present: field added to f, potential returned.
__device__ __forceinline__ double ext_pull(const ExtField &E, double px, double py, double pz,
                                           double eps, double (&f)[3])
{
    double ph = 0.0;
    if (E.on)
        ph += attractor_pull(E, px, py, pz, eps, f);
    if (E.bg)
        ph += background_pull(E, px, py, pz, f);
    return ph;
}

// M(d) l with M(d) = r^-3 I - 3 r^-5 d d^T (the attractor's field derivative
// is -S M(d) with respect to the particle, +S M(d) with respect to x_psi);
// also returns l . d r^-3 (= l . f / S).
__device__ __forceinline__ double attractor_m(const ExtField &A, double px, double py,
                                              double pz, double eps, const double (&l)[3],
                                              double (&mv)[3])
{
    const double dx = A.x - px, dy = A.y - py, dz = A.z - pz;
    const double s = dx * dx + dy * dy + dz * dz + eps * eps;
    const double rinv = 1.0 / sqrt(s);
    const double r3 = rinv * rinv * rinv;
    const double r5 = r3 * rinv * rinv;
    const double dl = dx * l[0] + dy * l[1] + dz * l[2];
    mv[0] = r3 * l[0] - 3.0 * r5 * dl * dx;
    mv[1] = r3 * l[1] - 3.0 * r5 * dl * dy;
    mv[2] = r3 * l[2] - 3.0 * r5 * dl * dz;
    return dl * r3;
}

// Kick-drift-kick in canonical momentum p = a^2 v (Eq. (9) with the kick
// factor int dt/a acting on g = G sum m_j (x_j - x_k) r^-3 and the drift
// factor int dt/a^2 acting on p).  One launch per grid point n:
//   g = G sum_s part[s]                       (finalise split partials)
//   p += k2_{n-1} g                           (closing half kick, n > first)
//   diagnostics of (x_n, p_n)                 (optional)
//   p += k1_n g;  x += d_n p                  (opening half kick + drift, n < last)
// The split-source partials of one 64-particle block are summed by
// kSliceGroups waves in parallel (wave q takes slices q, q + G, q + 2G, ...
// in order) and combined in LDS in the fixed order q = 0, 1, ..., G-1, so the
// result is deterministic; this keeps enough loads in flight to stream the
// partials at cache/HBM bandwidth instead of one latency-bound thread per
// particle.
constexpr int kSliceGroups = 4;
constexpr int kFinalizeThreads = kIntBlock * kSliceGroups;

// Sum of NC strided planes (k * stride + c * N) over this thread's slice
// group, then the fixed-order combine of the groups; valid in wave 0
// afterwards.  The accumulation follows the slot mode:
//   kSlotF64, kSlotF32Fold64: FP64 running sums, FP64 combine;
//   kSlotF32TwoSum: an unevaluated FP32 pair (hi, lo), each slot added by
//     TwoSum, the groups' pairs combined by TwoSum, hi + lo taken in FP64;
//   kSlotF32Direct: one FP32 running sum, FP32 combine.
template <int NC, int MODE, typename P>
__device__ __forceinline__ void grouped_slice_sum(const P *__restrict__ base, int S,
                                                  int64_t stride, int64_t N, bool valid,
                                                  double (*sh)[kSliceGroups][kIntBlock],
                                                  double (&out)[NC])
{
    const int p = threadIdx.x & (kIntBlock - 1), q = threadIdx.x / kIntBlock;
    if constexpr (MODE == kSlotF32TwoSum) {
        float hi[NC], lo[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            hi[c] = lo[c] = 0.0f;
        if (valid) {
#pragma unroll 4
            for (int k = q; k < S; k += kSliceGroups) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    two_sum_add(hi[c], lo[c], base[(int64_t)k * stride + (int64_t)c * N]);
            }
        }
        // (hi, lo) travel through LDS as the two halves of one 8-byte word
#pragma unroll
        for (int c = 0; c < NC; ++c)
            sh[c][q][p] = __builtin_bit_cast(double, make_float2(hi[c], lo[c]));
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            float2 h = __builtin_bit_cast(float2, sh[c][0][p]);
            float H = h.x, L = h.y;
#pragma unroll
            for (int g = 1; g < kSliceGroups; ++g) {
                const float2 o = __builtin_bit_cast(float2, sh[c][g][p]);
                two_sum_add(H, L, o.x);
                L += o.y;
            }
            out[c] = (double)H + (double)L;
        }
    } else if constexpr (MODE == kSlotF32Direct) {
        float acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = 0.0f;
        if (valid) {
#pragma unroll 4
            for (int k = q; k < S; k += kSliceGroups) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[c] += base[(int64_t)k * stride + (int64_t)c * N];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            sh[c][q][p] = (double)acc[c];
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            float t = (float)sh[c][0][p];
#pragma unroll
            for (int g = 1; g < kSliceGroups; ++g)
                t += (float)sh[c][g][p];
            out[c] = (double)t;
        }
    } else {
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = 0.0;
        if (valid) {
#pragma unroll 4
            for (int k = q; k < S; k += kSliceGroups) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[c] += (double)base[(int64_t)k * stride + (int64_t)c * N];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            sh[c][q][p] = acc[c];
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double t = sh[c][0][p];
#pragma unroll
            for (int g = 1; g < kSliceGroups; ++g)
                t += sh[c][g][p];
            out[c] = t;
        }
    }
}

// Slot sums at element offset `off`.  FP64 slots (mode kSlotF64) hold
// partial sums already multiplied by the box's common mass; FP32 slots (the
// symmetric loop with FP32 pairs: one FP32 sum of at most 256 terms per
// slot) hold them without it, and the mass (1 when the masses differ)
// multiplies the total here in FP64.
template <int NC>
__device__ __forceinline__ void slot_sum(const double *part, int mode, int64_t off, int S,
                                         int64_t stride, int64_t N, bool valid,
                                         double (*sh)[kSliceGroups][kIntBlock], double mbox,
                                         double (&out)[NC])
{
    const float *pf = reinterpret_cast<const float *>(part) + off;
    switch (mode) {
    case kSlotF64:
        grouped_slice_sum<NC, kSlotF64>(part + off, S, stride, N, valid, sh, out);
        return;
    case kSlotF32TwoSum:
        grouped_slice_sum<NC, kSlotF32TwoSum>(pf, S, stride, N, valid, sh, out);
        break;
    case kSlotF32Direct:
        grouped_slice_sum<NC, kSlotF32Direct>(pf, S, stride, N, valid, sh, out);
        break;
    default:
        grouped_slice_sum<NC, kSlotF32Fold64>(pf, S, stride, N, valid, sh, out);
        break;
    }
    const double f = isnan(mbox) ? 1.0 : mbox;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        out[c] *= f;
}

__global__ __launch_bounds__(kFinalizeThreads) void integrate_kernel(IntegrateArgs A)
{
    __shared__ double shs[4][kSliceGroups][kIntBlock];
    __shared__ double sh[kDiagW][kIntBlock];
    const IntBlock blk = A.blocks[blockIdx.x];
    const int pl = threadIdx.x & (kIntBlock - 1);
    const bool lead = threadIdx.x < kIntBlock;
    const int64_t i = blk.i0 + pl;
    const bool valid = i < blk.i1;
    const int64_t n = A.step[0], first = A.step[1], last = A.step[2];
    const int64_t row = n - first;
    const int64_t N = A.N;
    const int S = blk.n_slices;

    const double mbox = box_mass_of(A.box_mass, blk.box);
    double gs[3];
    slot_sum<3>(A.part, A.slot_mode, i, S, 3 * N, N, valid, shs, mbox, gs);
    double phs = 0.0;
    if (A.diag_part) {
        __syncthreads();
        double t[1];
        slot_sum<1>(A.part_phi, A.slot_mode, i, S, N, N, valid, shs, mbox, t);
        phs = t[0];
    }

    double v[kDiagW];
    for (int q = 0; q < kDiagW; ++q)
        v[q] = 0.0;
    if (lead && valid) {
        if (A.ewald_g) {
            for (int c = 0; c < 3; ++c)
                gs[c] += A.ewald_g[c * N + i];
            if (A.diag_part)
                phs += A.ewald_p[i];
        }
        double g[3] = {A.G * gs[0], A.G * gs[1], A.G * gs[2]};
        double p[3] = {A.p[i], A.p[N + i], A.p[2 * N + i]};
        double xx[3] = {A.x[i], A.x[N + i], A.x[2 * N + i]};
        // external potential (attractor, background: counted once)
        const double phe = ext_pull(A.ext, xx[0], xx[1], xx[2], blk.eps, g);
        if (n > first) {
            const StepCoef cp = A.coef[row - 1];
            for (int c = 0; c < 3; ++c)
                p[c] += cp.k2 * g[c];
            // tracer row at a_n: v = p / a^2, the final conversion's formula
            const int32_t t = A.track_slot ? A.track_slot[i] : -1;
            if (t >= 0) {
                const int64_t T = A.n_tracers;
                double *out = A.track + row * 6 * T + t;
                for (int c = 0; c < 3; ++c) {
                    out[c * T] = xx[c];
                    out[(3 + c) * T] = p[c] / (cp.a1 * cp.a1);
                }
            }
        }
        if (A.diag_part) {
            const double mi = A.m[i];
            phs -= self_potential(A.precision, mi, blk.eps, mbox);
            // U = (1/2a) sum m (phi_pair + 2 phi_att): the pair potential is
            // shared by two particles, the attractor's belongs to one
            const double phi = -A.G * phs + 2.0 * phe;
            v[0] = mi * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
            v[1] = mi * phi;
            v[2] = mi * p[0];
            v[3] = mi * p[1];
            v[4] = mi * p[2];
            v[5] = mi * (xx[1] * p[2] - xx[2] * p[1]);
            v[6] = mi * (xx[2] * p[0] - xx[0] * p[2]);
            v[7] = mi * (xx[0] * p[1] - xx[1] * p[0]);
            v[8] = 0.0;
            v[9] = (finite3(xx[0], xx[1], xx[2]) && finite3(p[0], p[1], p[2]) && isfinite(phi))
                       ? 0.0
                       : 1.0;
        }
        if (n < last) {
            const StepCoef cf = A.coef[row];
            for (int c = 0; c < 3; ++c) {
                p[c] += cf.k1 * g[c];
                xx[c] += cf.d * p[c];
                if (A.box > 0.0)
                    xx[c] -= A.box * floor(xx[c] / A.box);
            }
            A.x[i] = xx[0];
            A.x[N + i] = xx[1];
            A.x[2 * N + i] = xx[2];
        }
        A.p[i] = p[0];
        A.p[N + i] = p[1];
        A.p[2 * N + i] = p[2];
    }
    if (A.diag_part) {
        block_sum_rows(v, sh);
        if (threadIdx.x == 0) {
            double *out = A.diag_part + (row * A.n_blocks + blockIdx.x) * kDiagW;
            for (int q = 0; q < kDiagW; ++q)
                out[q] = v[q];
        }
    }
    if (A.work_counter && blockIdx.x == 0 && threadIdx.x == 0)
        *A.work_counter = 0;
}

__global__ void tick_kernel(int64_t *step, int *counter)
{
    *step += 1;
    *counter = 0;
}

// One block per box: sum the per-block rows in block order, then the
// Layzer-Irvine residual and elapsed time by a sequential pass.
// Diagnostics rows: one thread per (box, row) sums the row's block partials
// over the box's blocks in block order (the order, and so the bits, do not
// depend on the launch shape); the grid is flattened over (box, row chunk).
constexpr int kDiagRowThreads = 64;

__global__ __launch_bounds__(kDiagRowThreads) void diag_rows_kernel(
    const double *__restrict__ diag_part, int rows, int chunks, int n_blocks,
    const int32_t *__restrict__ box_first_block, const StepCoef *__restrict__ coef,
    colatus_diag *__restrict__ out)
{
    const int box = (int)(blockIdx.x / (unsigned)chunks);
    const int r = (int)(blockIdx.x % (unsigned)chunks) * kDiagRowThreads + (int)threadIdx.x;
    if (r >= rows)
        return;
    const int b0 = box_first_block[box], b1 = box_first_block[box + 1];
    double s[kDiagW];
    for (int q = 0; q < kDiagW; ++q)
        s[q] = 0.0;
    for (int b = b0; b < b1; ++b) {
        const double *d = diag_part + ((int64_t)r * n_blocks + b) * kDiagW;
        for (int q = 0; q < kDiagW - 1; ++q)
            s[q] += d[q];
        s[kDiagW - 1] = fmax(s[kDiagW - 1], d[kDiagW - 1]);
    }
    const double a = (r < rows - 1) ? coef[r].a0 : coef[r - 1].a1;
    colatus_diag row;
    row.a = a;
    row.t = 0.0;
    row.K = 0.5 * s[0] / (a * a);
    row.U = 0.5 * s[1] / a;
    row.LI = 0.0;
    row.P[0] = s[2];
    row.P[1] = s[3];
    row.P[2] = s[4];
    row.L[0] = s[5];
    row.L[1] = s[6];
    row.L[2] = s[7];
    const bool bad = s[kDiagW - 1] != 0.0 || !isfinite(row.K) || !isfinite(row.U);
    row.flags = bad ? 1u : 0u;
    row.reserved = 0u;
    out[(int64_t)box * rows + r] = row;
}

// Cosmic time and the Layzer-Irvine residual along each box's rows
// (trapezoid in ln a), one thread per box, rows in order.
__global__ void diag_prefix_kernel(int rows, int n_boxes, const StepCoef *__restrict__ coef,
                                   double H0, colatus_diag *__restrict__ out)
{
    const int box = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (box >= n_boxes)
        return;
    colatus_diag *o = out + (int64_t)box * rows;
    const double E0 = o[0].K + o[0].U;
    double t = 0.0, li = 0.0;
    double prev = 2.0 * o[0].K + o[0].U;
    for (int r = 1; r < rows; ++r) {
        t += coef[r - 1].dt;
        const double src = 2.0 * o[r].K + o[r].U;
        const double dlna = (H0 == 0.0) ? 0.0 : log(o[r].a) - log(o[r - 1].a);
        li += 0.5 * (prev + src) * dlna;
        prev = src;
        o[r].t = t;
        o[r].LI = o[r].K + o[r].U - E0 + li;
    }
}

// acc = scale * sum_s part[s];  phi = -G (sum_s part_phi[s] - self term).
__global__ __launch_bounds__(kFinalizeThreads) void forces_finalize_kernel(
    int precision, const double *__restrict__ box_mass, const IntBlock *__restrict__ blocks,
    const double *__restrict__ part, const double *__restrict__ part_phi, int slot_mode,
    const double *__restrict__ x, const double *__restrict__ m, int64_t N, double G,
    double scale, ExtField ext, double inv_a3, double *__restrict__ acc,
    double *__restrict__ phi, const double *__restrict__ kick_p, double *__restrict__ kick_v,
    const StepCoef *__restrict__ kick_coef)
{
    __shared__ double shs[4][kSliceGroups][kIntBlock];
    const IntBlock blk = blocks[blockIdx.x];
    const int64_t i = blk.i0 + (threadIdx.x & (kIntBlock - 1));
    const bool valid = i < blk.i1;
    const bool lead = threadIdx.x < kIntBlock;
    const double mbox = box_mass_of(box_mass, blk.box);
    double g[3];
    slot_sum<3>(part, slot_mode, i, blk.n_slices, 3 * N, N, valid, shs, mbox, g);
    double f[3] = {0.0, 0.0, 0.0}, phe = 0.0;
    if (lead && valid)
        phe = ext_pull(ext, x[i], x[N + i], x[2 * N + i], blk.eps, f);
    if (lead && valid)
        for (int c = 0; c < 3; ++c) {
            const double gc = scale * g[c] + inv_a3 * f[c];
            acc[(int64_t)c * N + i] = gc;
            if (kick_v) {
                // closing half kick of a cached step: v = (p + k2 g) / a1^2,
                // the same operations on the same g as the separate kick
                const StepCoef cf = kick_coef[0];
                const double pi = fma(cf.k2, gc, kick_p[(int64_t)c * N + i]);
                kick_v[(int64_t)c * N + i] = pi / (cf.a1 * cf.a1);
            }
        }
    if (phi) {
        __syncthreads();
        double t[1];
        slot_sum<1>(part_phi, slot_mode, i, blk.n_slices, N, N, valid, shs, mbox, t);
        if (lead && valid)
            phi[i] = -G * (t[0] - self_potential(precision, m[i], blk.eps, mbox)) + phe;
    }
}

// out[c] = G * sum_s part[s][c]  (part [S][n_cot][3][N]).
__global__ __launch_bounds__(kFinalizeThreads) void vjp_finalize_kernel(
    const IntBlock *__restrict__ blocks, const double *__restrict__ part, int slot_mode,
    const double *__restrict__ box_mass, const double *__restrict__ x,
    const double *__restrict__ lam, ExtField ext, int64_t N, int n_cot, double G,
    double *__restrict__ out)
{
    __shared__ double shs[4][kSliceGroups][kIntBlock];
    const IntBlock blk = blocks[blockIdx.x];
    const int64_t i = blk.i0 + (threadIdx.x & (kIntBlock - 1));
    const bool valid = i < blk.i1;
    const bool lead = threadIdx.x < kIntBlock;
    const double mbox = box_mass_of(box_mass, blk.box);
    for (int c = 0; c < n_cot; ++c) {
        double w[3];
        slot_sum<3>(part, slot_mode, (int64_t)c * 3 * N + i, blk.n_slices,
                    (int64_t)n_cot * 3 * N, N, valid, shs, mbox, w);
        if (lead && valid) {
            double o[3] = {G * w[0], G * w[1], G * w[2]};
            if (ext.on || ext.bg) {
                const double l[3] = {lam[((int64_t)c * 3 + 0) * N + i],
                                     lam[((int64_t)c * 3 + 1) * N + i],
                                     lam[((int64_t)c * 3 + 2) * N + i]};
                if (ext.on) {
                    double mv[3];
                    (void)attractor_m(ext, x[i], x[N + i], x[2 * N + i], blk.eps, l, mv);
                    for (int q = 0; q < 3; ++q)
                        o[q] -= ext.S * mv[q];
                }
                if (ext.bg)  // the background field's Jacobian is b I
                    for (int q = 0; q < 3; ++q)
                        o[q] += ext.b * l[q];
            }
            for (int q = 0; q < 3; ++q)
                out[((int64_t)c * 3 + q) * N + i] = o[q];
        }
        __syncthreads();
    }
}

// lam_x += cw * G sum_s part[s];  then (do_drift) lam_p += dnext * lam_x.
__global__ __launch_bounds__(kFinalizeThreads) void adjoint_update_kernel(
    const IntBlock *__restrict__ blocks, const double *__restrict__ part, int slot_mode,
    const double *__restrict__ box_mass, const double *__restrict__ x, ExtField ext,
    double *__restrict__ att_acc, int64_t N, int n_cot, double G, double cw,
    double *__restrict__ lam_x, double *__restrict__ lam_p, int do_drift, double dnext)
{
    __shared__ double shs[4][kSliceGroups][kIntBlock];
    __shared__ double sg[4][kIntBlock];
    const IntBlock blk = blocks[blockIdx.x];
    const int pl = threadIdx.x & (kIntBlock - 1);
    const int64_t i = blk.i0 + pl;
    const bool valid = i < blk.i1;
    const bool lead = threadIdx.x < kIntBlock;
    const double mbox = box_mass_of(box_mass, blk.box);
    for (int c = 0; c < n_cot; ++c) {
        double w[3];
        slot_sum<3>(part, slot_mode, (int64_t)c * 3 * N + i, blk.n_slices,
                    (int64_t)n_cot * 3 * N, N, valid, shs, mbox, w);
        double gp[4] = {0.0, 0.0, 0.0, 0.0};
        if (lead && valid) {
            double o[3] = {G * w[0], G * w[1], G * w[2]};
            if (ext.on || ext.bg) {
                // lam_p as the sweep saw it (before this update's drift)
                const double l[3] = {lam_p[((int64_t)c * 3 + 0) * N + i],
                                     lam_p[((int64_t)c * 3 + 1) * N + i],
                                     lam_p[((int64_t)c * 3 + 2) * N + i]};
                if (ext.on) {
                    double mv[3];
                    gp[0] = attractor_m(ext, x[i], x[N + i], x[2 * N + i], blk.eps, l, mv);
                    for (int q = 0; q < 3; ++q) {
                        o[q] -= ext.S * mv[q];
                        gp[1 + q] = ext.S * mv[q];
                    }
                }
                if (ext.bg)
                    for (int q = 0; q < 3; ++q)
                        o[q] += ext.b * l[q];
            }
            for (int q = 0; q < 3; ++q) {
                const int64_t k = ((int64_t)c * 3 + q) * N + i;
                const double lx = lam_x[k] + cw * o[q];
                lam_x[k] = lx;
                if (do_drift)
                    lam_p[k] += dnext * lx;
            }
        }
        if (ext.on && att_acc) {
            // this block's parameter derivatives, summed in particle order
            if (lead)
                for (int q = 0; q < 4; ++q)
                    sg[q][pl] = gp[q];
            __syncthreads();
            if (threadIdx.x < 4) {
                double t = 0.0;
                for (int k = 0; k < kIntBlock; ++k)
                    t += sg[threadIdx.x][k];
                att_acc[((int64_t)blockIdx.x * n_cot + c) * 4 + threadIdx.x] += cw * t;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// The paper's difference equations, Eqs. (3)-(5), in the comoving velocity v:
// one sweep per step at the half-step positions, this O(N) update after it.
// ---------------------------------------------------------------------------
__global__ void he_drift_kernel(double *__restrict__ x, const double *__restrict__ v,
                                int64_t n3, const StepCoef *__restrict__ coef, int64_t idx,
                                double f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3)
        x[i] += f * coef[idx].dt * v[i];
}

__global__ __launch_bounds__(kFinalizeThreads) void he_step_kernel(HEArgs A)
{
    __shared__ double shs[4][kSliceGroups][kIntBlock];
    const IntBlock blk = A.blocks[blockIdx.x];
    const int64_t i = blk.i0 + (threadIdx.x & (kIntBlock - 1));
    const bool valid = i < blk.i1;
    const bool lead = threadIdx.x < kIntBlock;
    const int64_t N = A.N;
    const double mbox = box_mass_of(A.box_mass, blk.box);
    double gs[3];
    slot_sum<3>(A.part, A.slot_mode, i, blk.n_slices, 3 * N, N, valid, shs, mbox, gs);
    if (!(lead && valid))
        return;
    const StepCoef cf = A.coef[A.row];
    double g[3] = {A.G * gs[0], A.G * gs[1], A.G * gs[2]};
    double xx[3] = {A.x[i], A.x[N + i], A.x[2 * N + i]};
    double vv[3] = {A.v[i], A.v[N + i], A.v[2 * N + i]};
    (void)ext_pull(A.ext, xx[0], xx[1], xx[2], blk.eps, g);
    const double tau = cf.dt, Ht = cf.Hh * tau;
    const double drag = (1.0 - Ht) / (1.0 + Ht);
    const double kick = tau / (cf.ah * cf.ah * cf.ah * (1.0 + Ht));
    const double tnext = A.last ? 0.0 : A.coef[A.row + 1].dt;
    const int32_t t = A.track_slot ? A.track_slot[i] : -1;
    const int64_t T = A.n_tracers;
    double *out = t >= 0 ? A.track + (A.row + 1) * 6 * T + t : nullptr;
    for (int c = 0; c < 3; ++c) {
        vv[c] = vv[c] * drag + g[c] * kick;
        const double xi = xx[c] + 0.5 * tau * vv[c];
        if (A.xi)
            A.xi[(int64_t)c * N + i] = xi;
        if (out) {
            out[c * T] = xi;
            out[(3 + c) * T] = vv[c];
        }
        A.x[(int64_t)c * N + i] = A.last ? xi : xi + 0.5 * tnext * vv[c];
        A.v[(int64_t)c * N + i] = vv[c];
    }
}

// ---------------------------------------------------------------------------
// Tracer tracks: the particle -> tracer map read by the step kernels, and the
// start-state row.
// ---------------------------------------------------------------------------
__global__ void track_slots_fill_kernel(int32_t *__restrict__ slot, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N)
        slot[i] = -1;
}

__global__ void track_slots_set_kernel(int32_t *__restrict__ slot,
                                       const int64_t *__restrict__ idx, int32_t T)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T)
        slot[idx[t]] = t;
}

__global__ void track_gather_kernel(const double *__restrict__ x, const double *__restrict__ v,
                                    int64_t N, const int64_t *__restrict__ idx, int32_t T,
                                    double *__restrict__ row)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T)
        return;
    const int64_t k = idx[t];
    for (int c = 0; c < 3; ++c) {
        row[(int64_t)c * T + t] = x[c * N + k];
        row[(int64_t)(3 + c) * T + t] = v[c * N + k];
    }
}

__global__ __launch_bounds__(kFinalizeThreads) void state_diag_kernel(
    const double *__restrict__ x, const double *__restrict__ v, const double *__restrict__ m,
    const double *__restrict__ part_phi, int slot_mode, const IntBlock *__restrict__ blocks,
    int n_blocks, int64_t N, double G, const StepCoef *__restrict__ coef, int64_t row,
    int precision, const double *__restrict__ box_mass, ExtField ext,
    double *__restrict__ diag_part)
{
    __shared__ double shs[4][kSliceGroups][kIntBlock];
    __shared__ double sh[kDiagW][kIntBlock];
    const IntBlock blk = blocks[blockIdx.x];
    const int64_t i = blk.i0 + (threadIdx.x & (kIntBlock - 1));
    const bool valid = i < blk.i1;
    const bool lead = threadIdx.x < kIntBlock;
    const double mbox = box_mass_of(box_mass, blk.box);
    double t[1];
    slot_sum<1>(part_phi, slot_mode, i, blk.n_slices, N, N, valid, shs, mbox, t);
    double w[kDiagW];
    for (int q = 0; q < kDiagW; ++q)
        w[q] = 0.0;
    if (lead && valid) {
        const double a = row == 0 ? coef[0].a0 : coef[row - 1].a1;
        const double mi = m[i];
        const double xx[3] = {x[i], x[N + i], x[2 * N + i]};
        const double p[3] = {a * a * v[i], a * a * v[N + i], a * a * v[2 * N + i]};
        double f[3] = {0.0, 0.0, 0.0};
        const double phe = ext_pull(ext, xx[0], xx[1], xx[2], blk.eps, f);
        const double phi = -G * (t[0] - self_potential(precision, mi, blk.eps, mbox)) + 2.0 * phe;
        w[0] = mi * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        w[1] = mi * phi;
        w[2] = mi * p[0];
        w[3] = mi * p[1];
        w[4] = mi * p[2];
        w[5] = mi * (xx[1] * p[2] - xx[2] * p[1]);
        w[6] = mi * (xx[2] * p[0] - xx[0] * p[2]);
        w[7] = mi * (xx[0] * p[1] - xx[1] * p[0]);
        w[9] = (finite3(xx[0], xx[1], xx[2]) && finite3(p[0], p[1], p[2]) && isfinite(phi))
                   ? 0.0
                   : 1.0;
    }
    block_sum_rows(w, sh);
    if (threadIdx.x == 0) {
        double *out = diag_part + (row * n_blocks + blockIdx.x) * kDiagW;
        for (int q = 0; q < kDiagW; ++q)
            out[q] = w[q];
    }
}

// out[c][q] = sum_b att_acc[b][c][q] over blocks in order.
__global__ void att_grad_reduce_kernel(const double *__restrict__ att_acc, int n_blocks,
                                       int n_cot, double *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)n_cot * 4)
        return;
    double t = 0.0;
    for (int b = 0; b < n_blocks; ++b)
        t += att_acc[(int64_t)b * n_cot * 4 + k];
    out[k] = t;
}

__global__ void fill_kernel(double *__restrict__ p, int64_t n, double value)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n)
        p[k] = value;
}

__global__ void scale_kernel(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                             double f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = f * src[i];
}

inline unsigned blocks_for(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

// ---------------------------------------------------------------------------
// Finite-time Lyapunov exponents (the chaotic-advection diagnostic of
// Sections I and IV): lambda = ln sigma_max(d x_t(end) / d x_t(0)) / span.
// ---------------------------------------------------------------------------
__global__ void ftle_seed_kernel(double *__restrict__ lam, const int64_t *__restrict__ idx,
                                 int T, int64_t N)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= 3 * T)
        return;
    const int t = k / 3, i = k - 3 * t;
    lam[((int64_t)k * 3 + i) * N + idx[t]] = 1.0;
}

// Largest eigenvalue of the symmetric 3x3 matrix c (overwritten) by cyclic
// Jacobi rotations (Rutishauser's form of each rotation), which converge
// quadratically; the sweep stops once the off-diagonal entries are below
// 1e-17 of the diagonal's size.
__device__ double sym3_max_eigenvalue(double c[3][3])
{
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = c[0][1] * c[0][1] + c[0][2] * c[0][2] + c[1][2] * c[1][2];
        const double dia = c[0][0] * c[0][0] + c[1][1] * c[1][1] + c[2][2] * c[2][2];
        if (!(off > 1e-34 * dia))
            break;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                const double apq = c[p][q];
                if (apq == 0.0)
                    continue;
                const double theta = (c[q][q] - c[p][p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                                 (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                // A' = R^T A R with R the rotation in the (p, q) plane
                for (int k = 0; k < 3; ++k) {
                    const double akp = c[k][p], akq = c[k][q];
                    c[k][p] = cs * akp - sn * akq;
                    c[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = c[p][k], aqk = c[q][k];
                    c[p][k] = cs * apk - sn * aqk;
                    c[q][k] = sn * apk + cs * aqk;
                }
                c[p][q] = c[q][p] = 0.0;
            }
        }
    }
    return fmax(c[0][0], fmax(c[1][1], c[2][2]));
}

__global__ void ftle_kernel(const double *__restrict__ grad, const int64_t *__restrict__ idx,
                            int T, int64_t N, double span_t, double span_lna,
                            double *__restrict__ lam_t, double *__restrict__ lam_lna,
                            double *__restrict__ blocks)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= T)
        return;
    const int64_t k = idx[t];
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            B[i][j] = grad[((int64_t)(3 * t + i) * 3 + j) * N + k];
    double C[3][3];  // B^T B
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[i][j] = B[0][i] * B[0][j] + B[1][i] * B[1][j] + B[2][i] * B[2][j];
    const double ln_sigma = 0.5 * log(sym3_max_eigenvalue(C));
    lam_t[t] = ln_sigma / span_t;
    if (lam_lna)
        lam_lna[t] = ln_sigma / span_lna;
    if (blocks)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                blocks[(int64_t)t * 9 + i * 3 + j] = B[i][j];
}

}  // namespace

hipError_t launch_coefficients(double H0, double OmR, double OmM, double OmK, double OmL,
                               double a_begin, double a_end, int64_t n_steps, int64_t first,
                               int64_t last, int half_time, StepCoef *coef, hipStream_t stream)
{
    Cosmo c{H0, OmR, OmM, OmK, OmL};
    const int64_t n = last - first;
    hipLaunchKernelGGL(coefficients_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, stream, c,
                       a_begin, a_end, n_steps, first, last, half_time, coef);
    return hipGetLastError();
}

hipError_t launch_convert(int mode, const double *src, double *dst, int64_t N,
                          const StepCoef *coef, int64_t idx, hipStream_t stream)
{
    hipLaunchKernelGGL(convert_kernel, dim3(blocks_for(3 * N, 256)), dim3(256), 0, stream, mode,
                       src, dst, 3 * N, coef, idx);
    return hipGetLastError();
}

hipError_t launch_integrate(const IntegrateArgs &args, hipStream_t stream)
{
    hipLaunchKernelGGL(integrate_kernel, dim3(args.n_blocks), dim3(kFinalizeThreads), 0, stream,
                       args);
    return hipGetLastError();
}

hipError_t launch_tick(int64_t *step, int *counter, hipStream_t stream)
{
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, stream, step, counter);
    return hipGetLastError();
}

hipError_t launch_diag_reduce(const double *diag_part, int rows, const IntBlock *blocks,
                              int n_blocks, int n_boxes, const int32_t *box_first_block,
                              const StepCoef *coef, double H0, double *out, hipStream_t stream)
{
    (void)blocks;
    if (rows < 2 || n_boxes < 1)  // a run has at least its start and end rows
        return hipErrorInvalidValue;
    const int64_t chunks = (rows + kDiagRowThreads - 1) / kDiagRowThreads;
    const int64_t grid = chunks * (int64_t)n_boxes;
    if (grid > 0x7fffffff)
        return hipErrorInvalidValue;
    colatus_diag *o = reinterpret_cast<colatus_diag *>(out);
    hipLaunchKernelGGL(diag_rows_kernel, dim3((unsigned)grid), dim3(kDiagRowThreads), 0, stream,
                       diag_part, rows, (int)chunks, n_blocks, box_first_block, coef, o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(diag_prefix_kernel, dim3((unsigned)((n_boxes + 63) / 64)), dim3(64), 0,
                       stream, rows, n_boxes, coef, H0, o);
    return hipGetLastError();
}

hipError_t launch_forces_finalize(int precision, const double *box_mass, const IntBlock *blocks,
                                  int n_blocks, const double *part, const double *part_phi,
                                  int slot_mode, const double *x, const double *m, int64_t N,
                                  double G, double scale, const ExtField &ext, double inv_a3,
                                  double *acc, double *phi, hipStream_t stream,
                                  const double *kick_p, double *kick_v, const StepCoef *kick_coef)
{
    hipLaunchKernelGGL(forces_finalize_kernel, dim3(n_blocks), dim3(kFinalizeThreads), 0, stream,
                       precision, box_mass, blocks, part, part_phi, slot_mode, x, m, N, G, scale,
                       ext, inv_a3, acc, phi, kick_p, kick_v, kick_coef);
    return hipGetLastError();
}

hipError_t launch_vjp_finalize(const IntBlock *blocks, int n_blocks, const double *part,
                               int slot_mode, const double *box_mass, const double *x,
                               const double *lam, const ExtField &ext, int64_t N, int n_cot,
                               double G, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(vjp_finalize_kernel, dim3(n_blocks), dim3(kFinalizeThreads), 0, stream,
                       blocks, part, slot_mode, box_mass, x, lam, ext, N, n_cot, G, out);
    return hipGetLastError();
}

hipError_t launch_adjoint_update(const IntBlock *blocks, int n_blocks, const double *part,
                                 int slot_mode, const double *box_mass, const double *x,
                                 const ExtField &ext, double *att_acc, int64_t N, int n_cot,
                                 double G, double cw, double *lam_x, double *lam_p,
                                 int do_drift, double dnext, hipStream_t stream)
{
    hipLaunchKernelGGL(adjoint_update_kernel, dim3(n_blocks), dim3(kFinalizeThreads), 0, stream,
                       blocks, part, slot_mode, box_mass, x, ext, att_acc, N, n_cot, G, cw, lam_x,
                       lam_p, do_drift, dnext);
    return hipGetLastError();
}

hipError_t launch_att_grad_reduce(const double *att_acc, int n_blocks, int n_cot, double *out,
                                  hipStream_t stream)
{
    const int64_t n = (int64_t)n_cot * 4;
    hipLaunchKernelGGL(att_grad_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream,
                       att_acc, n_blocks, n_cot, out);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double value, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p, n, value);
    return hipGetLastError();
}

hipError_t launch_ftle_seed(double *lam, int64_t n, const int64_t *idx, int T, int64_t N,
                            hipStream_t stream)
{
    hipError_t e = launch_fill(lam, n, 0.0, stream);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(ftle_seed_kernel, dim3(blocks_for(3 * (int64_t)T, 64)), dim3(64), 0, stream,
                       lam, idx, T, N);
    return hipGetLastError();
}

hipError_t launch_ftle(const double *grad, const int64_t *idx, int T, int64_t N, double span_t,
                       double span_lna, double *lam_t, double *lam_lna, double *blocks,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(ftle_kernel, dim3(blocks_for(T, 64)), dim3(64), 0, stream, grad, idx, T, N,
                       span_t, span_lna, lam_t, lam_lna, blocks);
    return hipGetLastError();
}

hipError_t launch_he_drift(double *x, const double *v, int64_t N, const StepCoef *coef,
                           int64_t idx, double f, hipStream_t stream)
{
    hipLaunchKernelGGL(he_drift_kernel, dim3(blocks_for(3 * N, 256)), dim3(256), 0, stream, x, v,
                       3 * N, coef, idx, f);
    return hipGetLastError();
}

hipError_t launch_cached_kick(int mode, double *x, double *v, double *p, const double *g,
                              int64_t N, const StepCoef *coef, hipStream_t stream)
{
    const int64_t n3 = 3 * N;
    hipLaunchKernelGGL(cached_kick_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0,
                       stream, mode, x, v, p, g, n3, coef);
    return hipGetLastError();
}

hipError_t launch_track_slots(int32_t *slot, int64_t N, const int64_t *idx, int32_t T,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(track_slots_fill_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                       stream, slot, N);
    hipLaunchKernelGGL(track_slots_set_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0,
                       stream, slot, idx, T);
    return hipGetLastError();
}

hipError_t launch_track_gather(const double *x, const double *v, int64_t N, const int64_t *idx,
                               int32_t T, double *row, hipStream_t stream)
{
    hipLaunchKernelGGL(track_gather_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0,
                       stream, x, v, N, idx, T, row);
    return hipGetLastError();
}

hipError_t launch_he_step(const HEArgs &args, hipStream_t stream)
{
    hipLaunchKernelGGL(he_step_kernel, dim3(args.n_blocks), dim3(kFinalizeThreads), 0, stream,
                       args);
    return hipGetLastError();
}

hipError_t launch_state_diag(const double *x, const double *v, const double *m,
                             const double *part_phi, int slot_mode, const IntBlock *blocks,
                             int n_blocks, int64_t N, double G, const StepCoef *coef,
                             int64_t row, int precision, const double *box_mass,
                             const ExtField &ext, double *diag_part, hipStream_t stream)
{
    hipLaunchKernelGGL(state_diag_kernel, dim3(n_blocks), dim3(kFinalizeThreads), 0, stream, x,
                       v, m, part_phi, slot_mode, blocks, n_blocks, N, G, coef, row, precision,
                       box_mass, ext, diag_part);
    return hipGetLastError();
}

hipError_t launch_scale(const double *src, double *dst, int64_t n, double factor,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, src, dst, n,
                       factor);
    return hipGetLastError();
}

}  // namespace colatus
