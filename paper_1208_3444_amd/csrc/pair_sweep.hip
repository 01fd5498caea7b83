// Pair sweeps of the direct-summation (particle-particle) scheme: the O(N^2)
// hot loop of the method (Section II: the force computation dominates the
// cost; Appendix A: one GPU thread per target particle looping over every
// source).  Gfx950 design, not a translation of the paper's kernel.
//
// Symmetric loops (form 2, the default up to 2^18 particles per box): the
// pair terms of the forward sum and of its adjoint change sign when the two
// particles swap, so each unordered pair is evaluated once.  A box is cut
// into parts of 256; a work item (one wave) holds part p's targets in
// registers, four per lane, while part q's sources pass around the wave one
// lane per step (DPP rotation) carrying their reaction accumulators.  Each
// partial-sum slot (part p's pull on a particle) is written once; an O(N)
// kernel adds the slots in a fixed order, so results are deterministic.  The
// forward loop runs 2x2 blocks of part pairs in workgroups of four waves
// that add the partial sums of a shared part in LDS before writing, halving
// the slots.
//
// Ordered loops (forms 0 and 1; larger boxes, many-cotangent adjoints):
//   * a work item is (block of target particles) x (slice of sources); the
//     slices of one target block write separate partial sums;
//   * each lane keeps R targets in registers; sources are staged tile by tile
//     into LDS (one source per thread) and read back as wave-uniform
//     broadcasts, so one LDS read feeds R pair interactions;
//   * per-tile FP32 partial sums are folded into FP64 or an unevaluated FP32
//     (hi, lo) pair with TwoSum (Knuth), bounding the accumulation error.
//
// Both: FP32 pairs use coordinates relative to the centre of the target
// block's (part's) bounding box (FP64 subtract, then round to FP32), so the
// FP32 pair arithmetic keeps the relative accuracy of the separation itself;
// rsqrt is the hardware v_rsq_f32 in FP32 and v_rsq_f64 refined by one Newton
// step in FP64; no MFMA: the pair interaction is not a dense contraction.
//
// The persistent variant launches about one grid of resident workgroups and
// pulls work items from a device counter until none are left (every
// workgroup's last fetch sees the counter past the end and exits).
#include "colatus_internal.h"

#include <math.h>
#include <type_traits>

namespace colatus {
namespace {

enum AccMode { kDirect = 0, kTwoSum = 1, kFold64 = 2 };

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

__device__ __forceinline__ float rsqrt_t(float s) { return __builtin_amdgcn_rsqf(s); }
__device__ __forceinline__ double rsqrt_t(double s) { return rsqrt_refined(s); }

// s^{-3/2} for FP64 pairs that do not need s^{-1/2} itself: with
// y = v_rsq_f64(s) (relative error below 6e-8) and e = 1 - s y^2,
// s^{-3/2} = y^3 (1 - e)^{-3/2} = y^3 (1 + 3e/2 + O(e^2)).  The first-order
// correction applied to y^3 leaves about (15/8) e^2 < 3e-14 relative, one
// operation fewer than refining y (rsqrt_refined) and cubing it.
__device__ __forceinline__ double rinv3_fp64(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    const double y2 = y * y;
    const double e = fma(-s, y2, 1.0);
    const double y3 = y2 * y;
    return fma(1.5 * e, y3, y3);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }


// Centre of the bounding box of the block's valid targets, for every thread.
template <int TPB, int R>
__device__ __forceinline__ void block_centre(const double (&tx)[R], const double (&ty)[R],
                                             const double (&tz)[R], const bool (&valid)[R],
                                             double (*red)[6], double &cx, double &cy,
                                             double &cz)
{
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (valid[r]) {
            v[0] = fmin(v[0], tx[r]);
            v[1] = fmin(v[1], ty[r]);
            v[2] = fmin(v[2], tz[r]);
            v[3] = fmax(v[3], tx[r]);
            v[4] = fmax(v[4], ty[r]);
            v[5] = fmax(v[5], tz[r]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            v[q] = fmin(v[q], __shfl_xor(v[q], off, 64));
            v[q + 3] = fmax(v[q + 3], __shfl_xor(v[q + 3], off, 64));
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            red[wave][q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 6; ++q)
        v[q] = red[0][q];
#pragma unroll
    for (int w = 1; w < TPB / 64; ++w) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            v[q] = fmin(v[q], red[w][q]);
            v[q + 3] = fmax(v[q + 3], red[w][q + 3]);
        }
    }
    cx = 0.5 * (v[0] + v[3]);
    cy = 0.5 * (v[1] + v[4]);
    cz = 0.5 * (v[2] + v[5]);
}

// Fetch the next work item index (persistent) or this block's (one-shot).
__device__ __forceinline__ int next_item(int persistent, int *counter, int *s_item, int iter)
{
    if (!persistent)
        return iter == 0 ? (int)blockIdx.x : 0x7fffffff;
    if (threadIdx.x == 0)
        *s_item = atomicAdd(counter, 1);
    __syncthreads();
    int it = *s_item;
    __syncthreads();
    return it;
}

// ---------------------------------------------------------------------------
// Forward sweep: sum_j m_j (x_j - x_k) r^-3 (and sum_j m_j r^-1 with PHI).
//
// Per pair: 3 subtractions, 3 FMAs for s = |d|^2 + eps^2, one v_rsq, then
// the weight w = m_j r^-3 and 3 FMAs into the accumulators.  The weight is
// formed either as m r^-1 (r^-1 r^-1) (FORM 0) or as (m r^-1) rcp(s)
// (FORM 1, one VALU multiply fewer, one more transcendental, which gfx950
// issues beside the VALU stream).  When every mass of the box is equal
// (EQM), m_j leaves the loop and multiplies the slice's partial sum once.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T pad_coord();
template <> __device__ __forceinline__ float pad_coord<float>() { return 1e30f; }
template <> __device__ __forceinline__ double pad_coord<double>() { return 1e150; }

template <typename T> __device__ __forceinline__ T rcp_t(T s);
template <> __device__ __forceinline__ float rcp_t<float>(float s) { return __builtin_amdgcn_rcpf(s); }
template <> __device__ __forceinline__ double rcp_t<double>(double s) { return 1.0 / s; }

template <typename T, int R, bool PHI, bool MASK, bool EQM, int FORM, typename V>
__device__ __forceinline__ void sweep_tile(const V *__restrict__ tile, int nt4, const T (&xi)[R],
                                           const T (&yi)[R], const T (&zi)[R], T eps2,
                                           T (&ax)[R], T (&ay)[R], T (&az)[R], T (&ph)[R])
{
    for (int jj = 0; jj < nt4; jj += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const V pj = tile[jj + u];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T dx = pj.x - xi[r];
                const T dy = pj.y - yi[r];
                const T dz = pj.z - zi[r];
                T s = fma_t(dx, dx, eps2);
                s = fma_t(dy, dy, s);
                s = fma_t(dz, dz, s);
                const T rinv = rsqrt_t(s);
                T mr = EQM ? rinv : pj.w * rinv;
                T w3;
                if constexpr (FORM == 1)
                    w3 = mr * rcp_t<T>(s);
                else
                    w3 = mr * (rinv * rinv);
                if constexpr (MASK) {
                    w3 = s > (T)0 ? w3 : (T)0;
                    mr = s > (T)0 ? mr : (T)0;
                }
                ax[r] = fma_t(w3, dx, ax[r]);
                ay[r] = fma_t(w3, dy, ay[r]);
                az[r] = fma_t(w3, dz, az[r]);
                if constexpr (PHI)
                    ph[r] += mr;
            }
        }
    }
}

template <typename T, int ACC, int R, int TPB, bool PHI, bool MASK, int FORM>
__global__ __launch_bounds__(TPB) void pair_sweep_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N,
    const WorkItem *__restrict__ items, int n_items, int *__restrict__ counter,
    int persistent, const double *__restrict__ box_mass, double *__restrict__ part,
    double *__restrict__ part_phi, int64_t *__restrict__ step_inc)
{
    using V = typename V4<T>::type;
    __shared__ V tile[TPB];
    __shared__ double red[TPB / 64][6];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const double *X = x, *Y = x + N, *Z = x + 2 * N;
    if (step_inc && blockIdx.x == 0 && tid == 0)
        *step_inc += 1;

    for (int iter = 0;; ++iter) {
        const int it = next_item(persistent, counter, &s_item, iter);
        if (it >= n_items)
            break;
        const WorkItem w = items[it];
        // common mass of the box, or NaN when the masses differ
        const double mbox = box_mass ? box_mass[w.box] : NAN;
        const bool eqm = !isnan(mbox);

        double tx[R], ty[R], tz[R];
        bool valid[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = w.i0 + tid + (int64_t)r * TPB;
            valid[r] = i < w.i1;
            const int64_t ii = valid[r] ? i : w.i0;
            tx[r] = X[ii];
            ty[r] = Y[ii];
            tz[r] = Z[ii];
        }
        double cx, cy, cz;
        block_centre<TPB, R>(tx, ty, tz, valid, red, cx, cy, cz);

        T xi[R], yi[R], zi[R];
        T ax[R], ay[R], az[R], ph[R];
        T hx[R], hy[R], hz[R], hp[R];      // TwoSum hi
        T lx[R], ly[R], lz[R], lp[R];      // TwoSum lo
        double bx[R], by[R], bz[R], bp[R]; // FP64 fold
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xi[r] = (T)(tx[r] - cx);
            yi[r] = (T)(ty[r] - cy);
            zi[r] = (T)(tz[r] - cz);
            ax[r] = ay[r] = az[r] = ph[r] = (T)0;
            hx[r] = hy[r] = hz[r] = hp[r] = (T)0;
            lx[r] = ly[r] = lz[r] = lp[r] = (T)0;
            bx[r] = by[r] = bz[r] = bp[r] = 0.0;
        }
        const T eps2 = (T)w.eps2;

        for (int64_t jt = w.j0; jt < w.j1; jt += TPB) {
            const int64_t j = jt + tid;
            V v;
            if (j < w.j1) {
                v.x = (T)(X[j] - cx);
                v.y = (T)(Y[j] - cy);
                v.z = (T)(Z[j] - cz);
                v.w = (T)m[j];
            } else {
                // padding: so far away that the pair adds nothing (FP32: s
                // overflows to +inf and r^-1 = 0; FP64: r^-3 underflows to 0)
                v.x = v.y = v.z = pad_coord<T>();
                v.w = (T)0;
            }
            __syncthreads();
            tile[tid] = v;
            __syncthreads();
            const int nt = (int)((w.j1 - jt) < TPB ? (w.j1 - jt) : TPB);
            const int nt4 = (nt + 3) & ~3;
            if (eqm)
                sweep_tile<T, R, PHI, MASK, true, FORM>(tile, nt4, xi, yi, zi, eps2, ax, ay, az,
                                                        ph);
            else
                sweep_tile<T, R, PHI, MASK, false, FORM>(tile, nt4, xi, yi, zi, eps2, ax, ay, az,
                                                         ph);
            if constexpr (ACC == kTwoSum) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    two_sum_add(hx[r], lx[r], (float)ax[r]);
                    two_sum_add(hy[r], ly[r], (float)ay[r]);
                    two_sum_add(hz[r], lz[r], (float)az[r]);
                    if constexpr (PHI)
                        two_sum_add(hp[r], lp[r], (float)ph[r]);
                    ax[r] = ay[r] = az[r] = ph[r] = (T)0;
                }
            } else if constexpr (ACC == kFold64) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    bx[r] += (double)ax[r];
                    by[r] += (double)ay[r];
                    bz[r] += (double)az[r];
                    if constexpr (PHI)
                        bp[r] += (double)ph[r];
                    ax[r] = ay[r] = az[r] = ph[r] = (T)0;
                }
            }
        }

        const int64_t slot = (int64_t)w.slice;
        const double scale = eqm ? mbox : 1.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!valid[r])
                continue;
            const int64_t i = w.i0 + tid + (int64_t)r * TPB;
            double ox, oy, oz, op;
            if constexpr (ACC == kTwoSum) {
                ox = (double)hx[r] + (double)lx[r];
                oy = (double)hy[r] + (double)ly[r];
                oz = (double)hz[r] + (double)lz[r];
                op = (double)hp[r] + (double)lp[r];
            } else if constexpr (ACC == kFold64) {
                ox = bx[r];
                oy = by[r];
                oz = bz[r];
                op = bp[r];
            } else {
                ox = (double)ax[r];
                oy = (double)ay[r];
                oz = (double)az[r];
                op = (double)ph[r];
            }
            part[(slot * 3 + 0) * N + i] = scale * ox;
            part[(slot * 3 + 1) * N + i] = scale * oy;
            part[(slot * 3 + 2) * N + i] = scale * oz;
            if constexpr (PHI)
                part_phi[slot * N + i] = scale * op;
        }
    }
}

// ---------------------------------------------------------------------------
// Symmetric forward sweep (form 2, FP32 pairs).  The pair term of Eq. (1) is
// antisymmetric: the pull of j on k, m_j d r^-3 with d = x_j - x_k, and the
// pull of k on j, -m_k d r^-3, share d, s = |d|^2 + eps^2 and r^-3.  Each
// unordered pair is therefore evaluated once and applied to both particles.
//
// A work item is a pair of parts (p, q), p < q, of one partition of a box.
// The W waves of the workgroup hold part p's U = 64 R W targets in registers
// (R per lane).  Part q's sources pass through in chunks of 64, one per lane;
// after every step each source moves one lane on (a DPP rotation of the whole
// wave) and carries the accumulator of its reaction with it, so after 64
// steps every source has met every target of the wave and is back in its
// lane with its reaction complete.  The waves' reactions are added in a fixed
// order.  Part p's partial sum from part q goes to the item's target slot
// and part q's reaction from part p to its reaction slot (with one item per
// workgroup slots q and p; the grouped form below numbers them by
// super-part): each (slot, particle) is written once, and the O(N) kernels
// add the slots in a fixed order.  The diagonal item (p, p) evaluates the
// ordered pairs of its part with the same loop and no reaction.
//
// Per unordered pair with equal masses: 3 subtractions, 3 FMAs, one v_rsq,
// 2 multiplies, 3 + 3 FMAs; per step and lane 6 rotations shared by R pairs.
// ---------------------------------------------------------------------------
// A value known to be equal in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// lane l receives the value lane (l - 1) mod 64 held (DPP wave_ror:1); every
// lane of the wave must be active.
__device__ __forceinline__ float wave_rotate(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x13C, 0xF, 0xF, true));
}
__device__ __forceinline__ double wave_rotate(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x13C, 0xF, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x13C, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Far-away coordinate of a missing target or source of the symmetric loops.
// Forward: s overflows (FP32) or r^-3 underflows (FP64) and the pair adds 0.
// Adjoint: s must stay finite so that d.u does (r^-3 underflows to 0).
template <typename T> __device__ __forceinline__ T sym_pad();
template <> __device__ __forceinline__ float sym_pad<float>() { return 1e30f; }
template <> __device__ __forceinline__ double sym_pad<double>() { return 1e150; }
template <typename T> __device__ __forceinline__ T adj_pad();
template <> __device__ __forceinline__ float adj_pad<float>() { return 1e18f; }
template <> __device__ __forceinline__ double adj_pad<double>() { return 1e150; }

// 64 steps of one source chunk against the lane's R targets.  REACT: also
// accumulate the reaction on the travelling source (q*); EQM: the box's common
// mass leaves the loop (weights r^-3 and r^-1 only).
template <typename T, int R, bool REACT, bool EQM, bool PHI, bool MASK>
__device__ __forceinline__ void sym_chunk(T sx, T sy, T sz, T sm, T &qx, T &qy, T &qz, T &qp,
                                          const T (&xi)[R], const T (&yi)[R], const T (&zi)[R],
                                          const T (&mi)[R], T eps2, T (&ax)[R], T (&ay)[R],
                                          T (&az)[R], T (&ap)[R])
{
#pragma unroll 2
    for (int k = 0; k < 64; ++k) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T dx = sx - xi[r];
            const T dy = sy - yi[r];
            const T dz = sz - zi[r];
            T s = fma_t(dx, dx, eps2);
            s = fma_t(dy, dy, s);
            s = fma_t(dz, dz, s);
            T rinv, w;
            if constexpr (sizeof(T) == 8 && !PHI) {
                w = rinv3_fp64(s);
                if constexpr (MASK)
                    w = s > (T)0.0 ? w : (T)0.0;
            } else {
                rinv = rsqrt_t(s);
                if constexpr (MASK)
                    rinv = s > (T)0.0 ? rinv : (T)0.0;
                w = rinv * (rinv * rinv);
            }
            const T wt = EQM ? w : sm * w;
            ax[r] = fma_t(wt, dx, ax[r]);
            ay[r] = fma_t(wt, dy, ay[r]);
            az[r] = fma_t(wt, dz, az[r]);
            if constexpr (PHI)
                ap[r] += EQM ? rinv : sm * rinv;
            if constexpr (REACT) {
                const T ws = EQM ? w : mi[r] * w;
                qx = fma_t(-ws, dx, qx);
                qy = fma_t(-ws, dy, qy);
                qz = fma_t(-ws, dz, qz);
                if constexpr (PHI)
                    qp += EQM ? rinv : mi[r] * rinv;
            }
        }
        sx = wave_rotate(sx);
        sy = wave_rotate(sy);
        sz = wave_rotate(sz);
        if constexpr (!EQM)
            sm = wave_rotate(sm);
        if constexpr (REACT) {
            qx = wave_rotate(qx);
            qy = wave_rotate(qy);
            qz = wave_rotate(qz);
            if constexpr (PHI)
                qp = wave_rotate(qp);
        }
    }
}

// One work item of the symmetric sweep.  REACT: a pair of parts (p < q),
// R targets per lane, with the reaction on the sources; otherwise a piece of
// a diagonal item: one target per lane against the whole part, no reaction
// (every unordered pair inside the part is met twice, once from each side).
// FOLD: the sources of a part exceed 256 and the targets' FP32 partial sums
// are folded every 256 sources; with at most 256 every partial sum (a
// target's from one part, a source's reaction from one part) is a single
// FP32 sum of at most 256 terms, like the ordered loop's per-tile partials.
template <typename T, int ACC, int R, int W, bool FOLD, bool REACT, bool PHI, bool MASK>
__device__ __forceinline__ void sym_item(const WorkItem &w, const double *__restrict__ X,
                                         const double *__restrict__ Y,
                                         const double *__restrict__ Z,
                                         const double *__restrict__ m, int64_t N,
                                         const double *__restrict__ box_mass,
                                         double *__restrict__ part,
                                         double *__restrict__ part_phi, double (*red)[6],
                                         T (*react)[W][PHI ? 4 : 3][64])
{
    constexpr int TPB = 64 * W;
    constexpr int NQ = PHI ? 4 : 3;
    // FP32 pairs without folding: every slot is one FP32 sum, stored as FP32
    // without the box mass (the readers apply it in FP64)
    constexpr bool F32OUT = sizeof(T) == 4 && !FOLD;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double mbox = box_mass ? box_mass[w.box] : NAN;
    const bool eqm = !isnan(mbox);

    double tx[R], ty[R], tz[R];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(wave * 64 * R + r * 64 + lane);
        valid[r] = i < w.i1;
        const int64_t ii = valid[r] ? i : w.i0;
        tx[r] = X[ii];
        ty[r] = Y[ii];
        tz[r] = Z[ii];
    }
    double cx, cy, cz;
    block_centre<TPB, R>(tx, ty, tz, valid, red, cx, cy, cz);
    cx = uniform(cx);
    cy = uniform(cy);
    cz = uniform(cz);

    // Missing targets sit far away with zero mass: they neither pull nor are
    // pulled (FP32 s overflows to +inf, r^-1 = 0).
    T xi[R], yi[R], zi[R], mi[R];
    T ax[R], ay[R], az[R], ap[R];
    float hx[R], hy[R], hz[R], hp[R];  // TwoSum (FP32 pairs only)
    float lx[R], ly[R], lz[R], lp[R];
    double bx[R], by[R], bz[R], bp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(wave * 64 * R + r * 64 + lane);
        if (valid[r]) {
            xi[r] = (T)(tx[r] - cx);
            yi[r] = (T)(ty[r] - cy);
            zi[r] = (T)(tz[r] - cz);
            mi[r] = (T)m[i];
        } else {
            xi[r] = yi[r] = zi[r] = sym_pad<T>();
            mi[r] = (T)0.0;
        }
        ax[r] = ay[r] = az[r] = ap[r] = (T)0.0;
        if constexpr (FOLD) {
            hx[r] = hy[r] = hz[r] = hp[r] = (T)0.0;
            lx[r] = ly[r] = lz[r] = lp[r] = (T)0.0;
            bx[r] = by[r] = bz[r] = bp[r] = 0.0;
        }
    }
    const T eps2 = uniform((T)w.eps2);
    const double scale = eqm ? mbox : 1.0;
    const int n_chunks = (int)((w.j1 - w.j0 + 63) / 64);

    for (int c = 0; c < n_chunks; ++c) {
        const int64_t j = w.j0 + (int64_t)c * 64 + lane;
        const bool jv = j < w.j1;
        T sx = sym_pad<T>(), sy = sym_pad<T>(), sz = sym_pad<T>(), sm = (T)0.0;
        if (jv) {
            sx = (T)(X[j] - cx);
            sy = (T)(Y[j] - cy);
            sz = (T)(Z[j] - cz);
            sm = (T)m[j];
        }
        T qx = (T)0.0, qy = (T)0.0, qz = (T)0.0, qp = (T)0.0;
        if (eqm)
            sym_chunk<T, R, REACT, true, PHI, MASK>(sx, sy, sz, sm, qx, qy, qz, qp, xi, yi, zi, mi,
                                                 eps2, ax, ay, az, ap);
        else
            sym_chunk<T, R, REACT, false, PHI, MASK>(sx, sy, sz, sm, qx, qy, qz, qp, xi, yi, zi, mi,
                                                  eps2, ax, ay, az, ap);
        if constexpr (FOLD) {
            if ((c & 3) == 3 || c == n_chunks - 1) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (ACC == kTwoSum) {
                        two_sum_add(hx[r], lx[r], ax[r]);
                        two_sum_add(hy[r], ly[r], ay[r]);
                        two_sum_add(hz[r], lz[r], az[r]);
                        if constexpr (PHI)
                            two_sum_add(hp[r], lp[r], ap[r]);
                        ax[r] = ay[r] = az[r] = ap[r] = (T)0.0;
                    } else if constexpr (ACC == kFold64) {
                        bx[r] += (double)ax[r];
                        by[r] += (double)ay[r];
                        bz[r] += (double)az[r];
                        if constexpr (PHI)
                            bp[r] += (double)ap[r];
                        ax[r] = ay[r] = az[r] = ap[r] = (T)0.0;
                    }
                }
            }
        }
        if constexpr (REACT) {
            // reaction on this chunk's sources: the waves' sums in a fixed order
            double o[NQ];
            if constexpr (W == 1) {
                o[0] = (double)qx;
                o[1] = (double)qy;
                o[2] = (double)qz;
                if constexpr (PHI)
                    o[NQ - 1] = (double)qp;
            } else {
                T(*buf)[NQ][64] = react[c & 1];
                buf[wave][0][lane] = qx;
                buf[wave][1][lane] = qy;
                buf[wave][2][lane] = qz;
                if constexpr (PHI)
                    buf[wave][NQ - 1][lane] = qp;
                __syncthreads();
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if constexpr (ACC == kTwoSum) {
                        float hi = (float)buf[0][q][lane], lo = 0.0f;
#pragma unroll
                        for (int v = 1; v < W; ++v)
                            two_sum_add(hi, lo, buf[v][q][lane]);
                        o[q] = (double)hi + (double)lo;
                    } else if constexpr (ACC == kFold64) {
                        double t = 0.0;
#pragma unroll
                        for (int v = 0; v < W; ++v)
                            t += (double)buf[v][q][lane];
                        o[q] = t;
                    } else {
                        T t = buf[0][q][lane];
#pragma unroll
                        for (int v = 1; v < W; ++v)
                            t += buf[v][q][lane];
                        o[q] = (double)t;
                    }
                }
            }
            if (wave == 0 && jv) {
                const int64_t rs = (int64_t)w.rslice;
                if constexpr (F32OUT) {
                    float *pf = reinterpret_cast<float *>(part);
                    pf[(rs * 3 + 0) * N + j] = qx;
                    pf[(rs * 3 + 1) * N + j] = qy;
                    pf[(rs * 3 + 2) * N + j] = qz;
                    if constexpr (PHI)
                        reinterpret_cast<float *>(part_phi)[rs * N + j] = qp;
                } else {
                    part[(rs * 3 + 0) * N + j] = scale * o[0];
                    part[(rs * 3 + 1) * N + j] = scale * o[1];
                    part[(rs * 3 + 2) * N + j] = scale * o[2];
                    if constexpr (PHI)
                        part_phi[rs * N + j] = scale * o[NQ - 1];
                }
            }
        }
    }

    const int64_t slot = (int64_t)w.slice;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!valid[r])
            continue;
        const int64_t i = w.i0 + (int64_t)(wave * 64 * R + r * 64 + lane);
        if constexpr (F32OUT) {
            float *pf = reinterpret_cast<float *>(part);
            pf[(slot * 3 + 0) * N + i] = ax[r];
            pf[(slot * 3 + 1) * N + i] = ay[r];
            pf[(slot * 3 + 2) * N + i] = az[r];
            if constexpr (PHI)
                reinterpret_cast<float *>(part_phi)[slot * N + i] = ap[r];
            continue;
        }
        double ox, oy, oz, op;
        if constexpr (FOLD && ACC == kTwoSum) {
            ox = (double)hx[r] + (double)lx[r];
            oy = (double)hy[r] + (double)ly[r];
            oz = (double)hz[r] + (double)lz[r];
            op = (double)hp[r] + (double)lp[r];
        } else if constexpr (FOLD && ACC == kFold64) {
            ox = bx[r];
            oy = by[r];
            oz = bz[r];
            op = bp[r];
        } else {
            ox = (double)ax[r];
            oy = (double)ay[r];
            oz = (double)az[r];
            op = (double)ap[r];
        }
        part[(slot * 3 + 0) * N + i] = scale * ox;
        part[(slot * 3 + 1) * N + i] = scale * oy;
        part[(slot * 3 + 2) * N + i] = scale * oz;
        if constexpr (PHI)
            part_phi[slot * N + i] = scale * op;
    }
}

// One wave per workgroup with four targets per lane is held to 80 VGPRs so
// that six waves share each SIMD (measured 10 % faster than four at 32^3;
// two 8-byte values of the item loop spill, outside the pair loop).
template <typename T, int ACC, int R, int W, bool PHI, bool MASK>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && R * W == 4 ? 6 : 1))) void
pair_sweep_sym_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N,
    const WorkItem *__restrict__ items, int n_items, int *__restrict__ counter,
    int persistent, const double *__restrict__ box_mass, double *__restrict__ part,
    double *__restrict__ part_phi, int64_t *__restrict__ step_inc)
{
    constexpr bool FOLD = 64 * R * W > 256;
    __shared__ double red[W][6];
    __shared__ T react[W > 1 ? 2 : 1][W][PHI ? 4 : 3][64];
    __shared__ int s_item;
    const double *X = x, *Y = x + N, *Z = x + 2 * N;
    if (step_inc && blockIdx.x == 0 && threadIdx.x == 0)
        *step_inc += 1;

    for (int iter = 0;; ++iter) {
        const int it = next_item(persistent, counter, &s_item, iter);
        if (it >= n_items)
            break;
        const WorkItem w = items[it];
        if (w.kind == 0)
            sym_item<T, ACC, R, W, FOLD, true, PHI, MASK>(w, X, Y, Z, m, N, box_mass, part,
                                                       part_phi, red, react);
        else
            sym_item<T, ACC, 1, W, FOLD, false, PHI, MASK>(w, X, Y, Z, m, N, box_mass, part,
                                                        part_phi, red, react);
    }
}

// ---------------------------------------------------------------------------
// Grouped symmetric sweep: four waves per workgroup, each on its own work
// item.  Parts pair up into super-parts {2A, 2A+1}; the group of two
// super-parts A < B is the 2x2 block of part pairs {p0, p1} x {q0, q1}
// (wave 2a + b: targets p_a, sources q_b).  The two waves with the same
// target part add their targets' partial sums (wave 2a's + wave 2a+1's), the
// two with the same source part their reactions (wave b's + wave b+2's),
// through LDS, so the block writes one slot per particle where the single
// items wrote two: a particle of a box of P parts gets ceil(P/2) + 1 slots
// instead of P (slot B for super-part B != A, slot A for the pair inside
// its super-part, the last for its diagonal; a part alone in its super-part
// puts its diagonal in slot A).  Items without a partner (tmate / rmate 0),
// and the groups of unrelated items (pairs inside super-parts, diagonal
// pieces), write their slots directly; padding items (kind -1) only take
// part in the barriers.  A combined slot is one addition (FP32 with FP32
// pairs, FP64 with FP64 pairs) of two partial sums of at most 256 terms.
// ---------------------------------------------------------------------------
constexpr int kGroupWaves = 4;

// Centre of the bounding box of one wave's valid targets, in every lane.
template <int R>
__device__ __forceinline__ void wave_centre(const double (&tx)[R], const double (&ty)[R],
                                            const double (&tz)[R], const bool (&valid)[R],
                                            double &cx, double &cy, double &cz)
{
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (valid[r]) {
            v[0] = fmin(v[0], tx[r]);
            v[1] = fmin(v[1], ty[r]);
            v[2] = fmin(v[2], tz[r]);
            v[3] = fmax(v[3], tx[r]);
            v[4] = fmax(v[4], ty[r]);
            v[5] = fmax(v[5], tz[r]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            v[q] = fmin(v[q], __shfl_xor(v[q], off, 64));
            v[q + 3] = fmax(v[q + 3], __shfl_xor(v[q + 3], off, 64));
        }
    }
    cx = uniform(0.5 * (v[0] + v[3]));
    cy = uniform(0.5 * (v[1] + v[4]));
    cz = uniform(0.5 * (v[2] + v[5]));
}

// One slot value of particle i: FP32 sums stored as FP32 without the box
// mass; FP64 sums stored multiplied by it (scale, 1 when the masses differ).
template <typename T, bool PHI>
__device__ __forceinline__ void grp_store(double *__restrict__ part, double *__restrict__ part_phi,
                                          int64_t N, int64_t slot, int64_t i, T vx, T vy, T vz,
                                          T vp, double scale)
{
    if constexpr (sizeof(T) == 4) {
        float *pf = reinterpret_cast<float *>(part);
        pf[(slot * 3 + 0) * N + i] = vx;
        pf[(slot * 3 + 1) * N + i] = vy;
        pf[(slot * 3 + 2) * N + i] = vz;
        if constexpr (PHI)
            reinterpret_cast<float *>(part_phi)[slot * N + i] = vp;
    } else {
        part[(slot * 3 + 0) * N + i] = scale * vx;
        part[(slot * 3 + 1) * N + i] = scale * vy;
        part[(slot * 3 + 2) * N + i] = scale * vz;
        if constexpr (PHI)
            part_phi[slot * N + i] = scale * vp;
    }
}

// The pair loop of one wave's item (R targets per lane; REACT: a pair of
// parts with the reaction on the sources, else a diagonal piece).  The
// targets' partial sums are left in (ax, ay, az, ap); the reactions go to
// rst[NQ][256] (LDS, chunk c at 64 c + lane) when the item has a reaction
// partner, else straight to slot rslice.
template <typename T, int R, bool REACT, bool PHI, bool MASK>
__device__ __forceinline__ void grp_item(const WorkItem &w, const double *__restrict__ X,
                                         const double *__restrict__ Y,
                                         const double *__restrict__ Z,
                                         const double *__restrict__ m, int64_t N, double mbox,
                                         double *__restrict__ part, double *__restrict__ part_phi,
                                         T (*rst)[256], T (&ax)[R], T (&ay)[R], T (&az)[R],
                                         T (&ap)[R], bool (&valid)[R])
{
    const int lane = threadIdx.x & 63;
    const bool eqm = !isnan(mbox);
    double tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        valid[r] = i < w.i1;
        const int64_t ii = valid[r] ? i : w.i0;
        tx[r] = X[ii];
        ty[r] = Y[ii];
        tz[r] = Z[ii];
    }
    double cx, cy, cz;
    wave_centre<R>(tx, ty, tz, valid, cx, cy, cz);
    T xi[R], yi[R], zi[R], mi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        if (valid[r]) {
            xi[r] = (T)(tx[r] - cx);
            yi[r] = (T)(ty[r] - cy);
            zi[r] = (T)(tz[r] - cz);
            mi[r] = (T)m[i];
        } else {
            xi[r] = yi[r] = zi[r] = sym_pad<T>();
            mi[r] = (T)0.0;
        }
        ax[r] = ay[r] = az[r] = ap[r] = (T)0.0;
    }
    const T eps2 = uniform((T)w.eps2);
    const double scale = eqm ? mbox : 1.0;
    const int n_chunks = (int)((w.j1 - w.j0 + 63) / 64);
    for (int c = 0; c < n_chunks; ++c) {
        const int64_t j = w.j0 + (int64_t)c * 64 + lane;
        const bool jv = j < w.j1;
        T sx = sym_pad<T>(), sy = sym_pad<T>(), sz = sym_pad<T>(), sm = (T)0.0;
        if (jv) {
            sx = (T)(X[j] - cx);
            sy = (T)(Y[j] - cy);
            sz = (T)(Z[j] - cz);
            sm = (T)m[j];
        }
        T qx = (T)0.0, qy = (T)0.0, qz = (T)0.0, qp = (T)0.0;
        if (eqm)
            sym_chunk<T, R, REACT, true, PHI, MASK>(sx, sy, sz, sm, qx, qy, qz, qp, xi, yi, zi, mi,
                                                 eps2, ax, ay, az, ap);
        else
            sym_chunk<T, R, REACT, false, PHI, MASK>(sx, sy, sz, sm, qx, qy, qz, qp, xi, yi, zi,
                                                  mi, eps2, ax, ay, az, ap);
        if constexpr (REACT) {
            if (rst) {
                rst[0][c * 64 + lane] = qx;
                rst[1][c * 64 + lane] = qy;
                rst[2][c * 64 + lane] = qz;
                if constexpr (PHI)
                    rst[3][c * 64 + lane] = qp;
            } else if (jv) {
                grp_store<T, PHI>(part, part_phi, N, (int64_t)w.rslice, j, qx, qy, qz, qp, scale);
            }
        }
    }
}

template <typename T, bool PHI, bool MASK>
__global__ __launch_bounds__(64 * kGroupWaves)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 3))) void
pair_sweep_sym_grp_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N,
    const WorkItem *__restrict__ items, int n_groups, int *__restrict__ counter,
    int persistent, const double *__restrict__ box_mass, double *__restrict__ part,
    double *__restrict__ part_phi, int64_t *__restrict__ step_inc)
{
    constexpr int NQ = PHI ? 4 : 3;
    // targets exported by the odd waves of a target pair; reactions of the
    // waves with a reaction partner
    __shared__ T tbuf[kGroupWaves / 2][NQ][256];
    __shared__ T rbuf[kGroupWaves][NQ][256];
    __shared__ int s_item;
    const double *X = x, *Y = x + N, *Z = x + 2 * N;
    // the wave index is uniform in the wave: the item loads to scalar registers
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (step_inc && blockIdx.x == 0 && threadIdx.x == 0)
        *step_inc += 1;

    for (int iter = 0;; ++iter) {
        const int g = next_item(persistent, counter, &s_item, iter);
        if (g >= n_groups)
            break;
        const WorkItem w = items[(int64_t)g * kGroupWaves + wave];
        const double mbox = (w.kind >= 0 && box_mass) ? box_mass[w.box] : NAN;
        const double scale = isnan(mbox) ? 1.0 : mbox;
        T ax[4], ay[4], az[4], ap[4];
        bool valid[4] = {false, false, false, false};
        if (w.kind == 0) {
            grp_item<T, 4, true, PHI, MASK>(w, X, Y, Z, m, N, mbox, part, part_phi,
                                            w.rmate ? rbuf[wave] : nullptr, ax, ay, az, ap,
                                            valid);
            if (!w.tmate) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (valid[r])
                        grp_store<T, PHI>(part, part_phi, N, (int64_t)w.slice,
                                          w.i0 + (int64_t)(r * 64 + lane), ax[r], ay[r], az[r],
                                          ap[r], scale);
            } else if (wave & 1) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    tbuf[wave >> 1][0][r * 64 + lane] = ax[r];
                    tbuf[wave >> 1][1][r * 64 + lane] = ay[r];
                    tbuf[wave >> 1][2][r * 64 + lane] = az[r];
                    if constexpr (PHI)
                        tbuf[wave >> 1][3][r * 64 + lane] = ap[r];
                }
            }
        } else if (w.kind == 1) {
            T bx[1], by[1], bz[1], bp[1];
            bool v1[1];
            grp_item<T, 1, false, PHI, MASK>(w, X, Y, Z, m, N, mbox, part, part_phi, nullptr, bx,
                                             by, bz, bp, v1);
            if (v1[0])
                grp_store<T, PHI>(part, part_phi, N, (int64_t)w.slice, w.i0 + lane, bx[0], by[0],
                                  bz[0], bp[0], scale);
        }
        __syncthreads();
        if (w.kind == 0 && w.tmate && !(wave & 1)) {
            // targets: this wave's (sources q0) + the odd wave's (sources q1)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (valid[r]) {
                    const int e = r * 64 + lane;
                    T vp = (T)0.0;
                    if constexpr (PHI)
                        vp = ap[r] + tbuf[wave >> 1][3][e];
                    grp_store<T, PHI>(part, part_phi, N, (int64_t)w.slice, w.i0 + e,
                                      ax[r] + tbuf[wave >> 1][0][e], ay[r] + tbuf[wave >> 1][1][e],
                                      az[r] + tbuf[wave >> 1][2][e], vp, scale);
                }
        }
        if (w.kind == 0 && w.rmate && wave < 2) {
            // reactions on sources q_b: from targets p0 (wave b) + p1 (wave b + 2)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int e = c * 64 + lane;
                const int64_t j = w.j0 + e;
                if (j < w.j1) {
                    T vp = (T)0.0;
                    if constexpr (PHI)
                        vp = rbuf[wave][3][e] + rbuf[wave + 2][3][e];
                    grp_store<T, PHI>(part, part_phi, N, (int64_t)w.rslice, j,
                                      rbuf[wave][0][e] + rbuf[wave + 2][0][e],
                                      rbuf[wave][1][e] + rbuf[wave + 2][1][e],
                                      rbuf[wave][2][e] + rbuf[wave + 2][2][e], vp, scale);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Symmetric adjoint sweep (form 2, FP32 pairs, one cotangent per launch).
// The adjoint pair term M(d)(m_k lam_j - m_j lam_k), M(d) = r^-3 I -
// 3 r^-5 d d^T, changes sign when k and j swap (M(-d) = M(d)), so each
// unordered pair is evaluated once, with the work items, slots and DPP
// rotation of the symmetric forward sweep; the travelling source carries
// its position, cotangent (and mass) and the accumulator of its reaction.
// Missing sources and targets sit at 1e18 with zero mass and cotangent: s
// stays finite in FP32 (3e36) while r^-3 underflows to 0, so d.u stays
// finite and the pair adds exactly 0.
//
// FULL chunks (every target and source lane holds a particle, so no padding
// position enters) apply r^-3 inside the accumulation instead:
// v = r^-3 (u - 3 r^-2 (d.u) d), added as fma(r^-3, ., acc) to the target
// and fma(-r^-3, ., q) to the reaction: three multiplies fewer per pair.
// There d.u is formed from the unscaled u, which against a padding position
// (|d| ~ 1e18) would overflow FP32 for |u| above ~1e20; chunks with padding
// therefore keep the scaled form.
// ---------------------------------------------------------------------------
template <typename T, int R, bool REACT, bool EQM, bool MASK, bool FULL>
__device__ __forceinline__ void sym_adj_chunk(T sx, T sy, T sz, T sm, T slx, T sly, T slz,
                                              T &qx, T &qy, T &qz, const T (&xi)[R],
                                              const T (&yi)[R], const T (&zi)[R],
                                              const T (&mk)[R], const T (&lkx)[R],
                                              const T (&lky)[R], const T (&lkz)[R], T eps2,
                                              T (&ax)[R], T (&ay)[R], T (&az)[R])
{
#pragma unroll 1
    for (int k = 0; k < 64; ++k) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T dx = sx - xi[r];
            const T dy = sy - yi[r];
            const T dz = sz - zi[r];
            T s = fma_t(dx, dx, eps2);
            s = fma_t(dy, dy, s);
            s = fma_t(dz, dz, s);
            T rinv = rsqrt_t(s);
            if constexpr (MASK)
                rinv = s > (T)0.0 ? rinv : (T)0.0;
            // M(d) u = r^-3 u - 3 r^-5 (d.u) d = u' - 3 r^-2 (d.u') d with
            // u' = r^-3 u (one multiply fewer per pair than scaling t)
            const T r2 = rinv * rinv;
            const T r3 = r2 * rinv;
            const T m3r2 = -(T)3.0 * r2;
            T ux, uy, uz;
            if constexpr (EQM) {
                ux = slx - lkx[r];
                uy = sly - lky[r];
                uz = slz - lkz[r];
            } else {
                // both products rounded before the difference, so that the
                // self pair (j = k, inside a diagonal part) gives u = 0
                // exactly; a fused m_k lam_j - m_j lam_k would leave the
                // product's rounding error, which r^-3 = eps^-3 amplifies
#pragma clang fp contract(off)
                ux = mk[r] * slx - sm * lkx[r];
                uy = mk[r] * sly - sm * lky[r];
                uz = mk[r] * slz - sm * lkz[r];
            }
            if constexpr (FULL) {
                const T du = fma_t(dx, ux, fma_t(dy, uy, dz * uz));
                const T t = m3r2 * du;
                const T vx = fma_t(t, dx, ux);
                const T vy = fma_t(t, dy, uy);
                const T vz = fma_t(t, dz, uz);
                ax[r] = fma_t(r3, vx, ax[r]);
                ay[r] = fma_t(r3, vy, ay[r]);
                az[r] = fma_t(r3, vz, az[r]);
                if constexpr (REACT) {
                    qx = fma_t(-r3, vx, qx);
                    qy = fma_t(-r3, vy, qy);
                    qz = fma_t(-r3, vz, qz);
                }
            } else {
                ux *= r3;
                uy *= r3;
                uz *= r3;
                const T du = fma_t(dx, ux, fma_t(dy, uy, dz * uz));
                const T t = m3r2 * du;
                const T vx = fma_t(t, dx, ux);
                const T vy = fma_t(t, dy, uy);
                const T vz = fma_t(t, dz, uz);
                ax[r] += vx;
                ay[r] += vy;
                az[r] += vz;
                if constexpr (REACT) {
                    qx -= vx;
                    qy -= vy;
                    qz -= vz;
                }
            }
        }
        sx = wave_rotate(sx);
        sy = wave_rotate(sy);
        sz = wave_rotate(sz);
        slx = wave_rotate(slx);
        sly = wave_rotate(sly);
        slz = wave_rotate(slz);
        if constexpr (!EQM)
            sm = wave_rotate(sm);
        if constexpr (REACT) {
            qx = wave_rotate(qx);
            qy = wave_rotate(qy);
            qz = wave_rotate(qz);
        }
    }
}

// A slot value of the symmetric adjoint: FP32 pairs store the FP32 sum as it
// is (the readers apply the box mass), FP64 pairs the scaled FP64 value.
__device__ __forceinline__ void store_slot(double *part, int64_t k, float v, double)
{
    reinterpret_cast<float *>(part)[k] = v;
}
__device__ __forceinline__ void store_slot(double *part, int64_t k, double v, double scale)
{
    part[k] = scale * v;
}

// One work item of the symmetric adjoint sweep, cotangent c of n_cot; parts
// of at most 256 particles (one FP32 partial per slot, as in the forward).
template <typename T, int R, bool REACT, bool MASK>
__device__ __forceinline__ void sym_adj_item(const WorkItem &w, const double *__restrict__ X,
                                             const double *__restrict__ Y,
                                             const double *__restrict__ Z,
                                             const double *__restrict__ m,
                                             const double *__restrict__ lam, int n_cot, int c,
                                             int64_t N, const double *__restrict__ box_mass,
                                             double *__restrict__ part, double (*red)[6])
{
    const int lane = threadIdx.x & 63;
    const double mbox = box_mass ? box_mass[w.box] : NAN;
    const bool eqm = !isnan(mbox);
    const double *LX = lam + ((int64_t)c * 3 + 0) * N;
    const double *LY = lam + ((int64_t)c * 3 + 1) * N;
    const double *LZ = lam + ((int64_t)c * 3 + 2) * N;

    double tx[R], ty[R], tz[R];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        valid[r] = i < w.i1;
        const int64_t ii = valid[r] ? i : w.i0;
        tx[r] = X[ii];
        ty[r] = Y[ii];
        tz[r] = Z[ii];
    }
    double cx, cy, cz;
    block_centre<64, R>(tx, ty, tz, valid, red, cx, cy, cz);
    cx = uniform(cx);
    cy = uniform(cy);
    cz = uniform(cz);

    T xi[R], yi[R], zi[R], mk[R], lkx[R], lky[R], lkz[R];
    T ax[R], ay[R], az[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        if (valid[r]) {
            xi[r] = (T)(tx[r] - cx);
            yi[r] = (T)(ty[r] - cy);
            zi[r] = (T)(tz[r] - cz);
            mk[r] = (T)m[i];
            lkx[r] = (T)LX[i];
            lky[r] = (T)LY[i];
            lkz[r] = (T)LZ[i];
        } else {
            xi[r] = yi[r] = zi[r] = adj_pad<T>();
            mk[r] = lkx[r] = lky[r] = lkz[r] = (T)0.0;
        }
        ax[r] = ay[r] = az[r] = (T)0.0;
    }
    const T eps2 = uniform((T)w.eps2);
    const double scale = eqm ? mbox : 1.0;
    const int n_chunks = (int)((w.j1 - w.j0 + 63) / 64);
    const bool full_t = w.i1 - w.i0 == (int64_t)(64 * R);

    for (int ch = 0; ch < n_chunks; ++ch) {
        const int64_t j = w.j0 + (int64_t)ch * 64 + lane;
        const bool jv = j < w.j1;
        T sx = adj_pad<T>(), sy = adj_pad<T>(), sz = adj_pad<T>(), sm = (T)0.0;
        T slx = (T)0.0, sly = (T)0.0, slz = (T)0.0;
        if (jv) {
            sx = (T)(X[j] - cx);
            sy = (T)(Y[j] - cy);
            sz = (T)(Z[j] - cz);
            sm = (T)m[j];
            slx = (T)LX[j];
            sly = (T)LY[j];
            slz = (T)LZ[j];
        }
        T qx = (T)0.0, qy = (T)0.0, qz = (T)0.0;
        const bool full = full_t && w.j0 + (int64_t)(ch + 1) * 64 <= w.j1;
        if (eqm && full)
            sym_adj_chunk<T, R, REACT, true, MASK, true>(sx, sy, sz, sm, slx, sly, slz, qx, qy, qz,
                                                      xi, yi, zi, mk, lkx, lky, lkz, eps2, ax,
                                                      ay, az);
        else if (eqm)
            sym_adj_chunk<T, R, REACT, true, MASK, false>(sx, sy, sz, sm, slx, sly, slz, qx, qy, qz,
                                                       xi, yi, zi, mk, lkx, lky, lkz, eps2, ax,
                                                       ay, az);
        else if (full)
            sym_adj_chunk<T, R, REACT, false, MASK, true>(sx, sy, sz, sm, slx, sly, slz, qx, qy,
                                                       qz, xi, yi, zi, mk, lkx, lky, lkz, eps2,
                                                       ax, ay, az);
        else
            sym_adj_chunk<T, R, REACT, false, MASK, false>(sx, sy, sz, sm, slx, sly, slz, qx, qy,
                                                        qz, xi, yi, zi, mk, lkx, lky, lkz, eps2,
                                                        ax, ay, az);
        if constexpr (REACT) {
            if (jv) {
                const int64_t rs = (int64_t)w.rslice;
                store_slot(part, ((rs * n_cot + c) * 3 + 0) * N + j, qx, scale);
                store_slot(part, ((rs * n_cot + c) * 3 + 1) * N + j, qy, scale);
                store_slot(part, ((rs * n_cot + c) * 3 + 2) * N + j, qz, scale);
            }
        }
    }
    const int64_t slot = (int64_t)w.slice;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!valid[r])
            continue;
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        store_slot(part, ((slot * n_cot + c) * 3 + 0) * N + i, ax[r], scale);
        store_slot(part, ((slot * n_cot + c) * 3 + 1) * N + i, ay[r], scale);
        store_slot(part, ((slot * n_cot + c) * 3 + 2) * N + i, az[r], scale);
    }
}

template <typename T, int R, bool MASK>
__global__ __launch_bounds__(64) void adjoint_sweep_sym_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N,
    const double *__restrict__ lam, int n_cot, int c, const WorkItem *__restrict__ items,
    int n_items, int *__restrict__ counter, int persistent, const double *__restrict__ box_mass,
    double *__restrict__ part)
{
    __shared__ double red[1][6];
    __shared__ int s_item;
    const double *X = x, *Y = x + N, *Z = x + 2 * N;
    for (int iter = 0;; ++iter) {
        const int it = next_item(persistent, counter, &s_item, iter);
        if (it >= n_items)
            break;
        const WorkItem w = items[it];
        if (w.kind == 0)
            sym_adj_item<T, R, true, MASK>(w, X, Y, Z, m, lam, n_cot, c, N, box_mass, part, red);
        else
            sym_adj_item<T, 1, false, MASK>(w, X, Y, Z, m, lam, n_cot, c, N, box_mass, part, red);
    }
}

// ---------------------------------------------------------------------------
// Adjoint sweep: sum_j M(d)(m_k lam_j - m_j lam_k), M(d) = r^-3 I - 3 r^-5 d d^T,
// for C cotangents sharing the geometry.  lam is [n_cot][3][N]; this launch
// handles cotangents [c0, c0 + C).  part is [slices][n_cot][3][N].
// ---------------------------------------------------------------------------
// Pair loop of the adjoint sweep over one LDS tile.  With equal masses
// (EQM) the bracket m_k lam_j - m_j lam_k is m (lam_j - lam_k); the common
// m multiplies the slice's partial sum once instead.
template <typename T, int R, int C, bool MASK, bool EQM, typename V>
__device__ __forceinline__ void adjoint_tile(const V *__restrict__ tile,
                                             const T *__restrict__ ltile, int nt,
                                             const T (&xi)[R], const T (&yi)[R],
                                             const T (&zi)[R], const T (&mk)[R],
                                             const T (&lk)[R][3 * C], T eps2,
                                             T (&acc)[R][3 * C])
{
    constexpr int LW = 3 * C;
    for (int jj = 0; jj < nt; ++jj) {
        const V pj = tile[jj];
        T lt[LW];
#pragma unroll
        for (int q = 0; q < LW; ++q)
            lt[q] = ltile[jj * LW + q];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T dx = pj.x - xi[r];
            const T dy = pj.y - yi[r];
            const T dz = pj.z - zi[r];
            T s = fma_t(dx, dx, eps2);
            s = fma_t(dy, dy, s);
            s = fma_t(dz, dz, s);
            T rinv = rsqrt_t(s);
            if constexpr (MASK)
                rinv = s > (T)0 ? rinv : (T)0;
            const T r2 = rinv * rinv;
            const T r3 = r2 * rinv;
            const T m3r5 = (T)(-3) * (r3 * r2);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T ux, uy, uz;
                if constexpr (EQM) {
                    ux = lt[3 * c + 0] - lk[r][3 * c + 0];
                    uy = lt[3 * c + 1] - lk[r][3 * c + 1];
                    uz = lt[3 * c + 2] - lk[r][3 * c + 2];
                } else {
                    // rounded products, then the difference: u = 0 exactly
                    // for the self pair (see the symmetric loop)
#pragma clang fp contract(off)
                    ux = mk[r] * lt[3 * c + 0] - pj.w * lk[r][3 * c + 0];
                    uy = mk[r] * lt[3 * c + 1] - pj.w * lk[r][3 * c + 1];
                    uz = mk[r] * lt[3 * c + 2] - pj.w * lk[r][3 * c + 2];
                }
                const T du = fma_t(dx, ux, fma_t(dy, uy, dz * uz));
                const T t = m3r5 * du;
                acc[r][3 * c + 0] = fma_t(t, dx, fma_t(r3, ux, acc[r][3 * c + 0]));
                acc[r][3 * c + 1] = fma_t(t, dy, fma_t(r3, uy, acc[r][3 * c + 1]));
                acc[r][3 * c + 2] = fma_t(t, dz, fma_t(r3, uz, acc[r][3 * c + 2]));
            }
        }
    }
}

template <typename T, int ACC, int R, int TPB, int C, bool MASK>
__global__ __launch_bounds__(TPB) void adjoint_sweep_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N,
    const double *__restrict__ lam, int n_cot, int c0,
    const WorkItem *__restrict__ items, int n_items, int *__restrict__ counter,
    int persistent, const double *__restrict__ box_mass, double *__restrict__ part)
{
    using V = typename V4<T>::type;
    constexpr int LW = 3 * C;
    __shared__ V tile[TPB];
    __shared__ T ltile[TPB * LW];
    __shared__ double red[TPB / 64][6];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const double *X = x, *Y = x + N, *Z = x + 2 * N;

    for (int iter = 0;; ++iter) {
        const int it = next_item(persistent, counter, &s_item, iter);
        if (it >= n_items)
            break;
        const WorkItem w = items[it];
        const double mbox = box_mass ? box_mass[w.box] : NAN;
        const bool eqm = !isnan(mbox);

        double tx[R], ty[R], tz[R];
        bool valid[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = w.i0 + tid + (int64_t)r * TPB;
            valid[r] = i < w.i1;
            const int64_t ii = valid[r] ? i : w.i0;
            tx[r] = X[ii];
            ty[r] = Y[ii];
            tz[r] = Z[ii];
        }
        double cx, cy, cz;
        block_centre<TPB, R>(tx, ty, tz, valid, red, cx, cy, cz);

        T xi[R], yi[R], zi[R], mk[R];
        T lk[R][LW];    // lam_k
        T acc[R][LW];   // tile partial / direct sum
        double fold[R][LW];
        T hi[R][LW], lo[R][LW];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = w.i0 + tid + (int64_t)r * TPB;
            const int64_t ii = valid[r] ? i : w.i0;
            xi[r] = (T)(tx[r] - cx);
            yi[r] = (T)(ty[r] - cy);
            zi[r] = (T)(tz[r] - cz);
            mk[r] = (T)m[ii];
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    lk[r][3 * c + q] = (T)lam[((int64_t)(c0 + c) * 3 + q) * N + ii];
                    acc[r][3 * c + q] = (T)0;
                    fold[r][3 * c + q] = 0.0;
                    hi[r][3 * c + q] = (T)0;
                    lo[r][3 * c + q] = (T)0;
                }
        }
        const T eps2 = (T)w.eps2;

        for (int64_t jt = w.j0; jt < w.j1; jt += TPB) {
            const int64_t j = jt + tid;
            V v;
            T lj[LW];
            if (j < w.j1) {
                v.x = (T)(X[j] - cx);
                v.y = (T)(Y[j] - cy);
                v.z = (T)(Z[j] - cz);
                v.w = (T)m[j];
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        lj[3 * c + q] = (T)lam[((int64_t)(c0 + c) * 3 + q) * N + j];
            } else {
                v.x = v.y = v.z = v.w = (T)0;
#pragma unroll
                for (int q = 0; q < LW; ++q)
                    lj[q] = (T)0;
            }
            __syncthreads();
            tile[tid] = v;
#pragma unroll
            for (int q = 0; q < LW; ++q)
                ltile[tid * LW + q] = lj[q];
            __syncthreads();
            const int nt = (int)((w.j1 - jt) < TPB ? (w.j1 - jt) : TPB);
            if (eqm)
                adjoint_tile<T, R, C, MASK, true>(tile, ltile, nt, xi, yi, zi, mk, lk, eps2, acc);
            else
                adjoint_tile<T, R, C, MASK, false>(tile, ltile, nt, xi, yi, zi, mk, lk, eps2, acc);
            if constexpr (ACC != kDirect) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int q = 0; q < LW; ++q) {
                        if constexpr (ACC == kTwoSum)
                            two_sum_add(hi[r][q], lo[r][q], (float)acc[r][q]);
                        else
                            fold[r][q] += (double)acc[r][q];
                        acc[r][q] = (T)0;
                    }
            }
        }

        const int64_t slot = (int64_t)w.slice;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!valid[r])
                continue;
            const int64_t i = w.i0 + tid + (int64_t)r * TPB;
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    double o;
                    if constexpr (ACC == kTwoSum)
                        o = (double)hi[r][3 * c + q] + (double)lo[r][3 * c + q];
                    else if constexpr (ACC == kFold64)
                        o = fold[r][3 * c + q];
                    else
                        o = (double)acc[r][3 * c + q];
                    part[((slot * n_cot + (c0 + c)) * 3 + q) * N + i] = eqm ? mbox * o : o;
                }
        }
    }
}

__global__ void zero_counter_kernel(int *counter) { *counter = 0; }

// ---------------------------------------------------------------------------
// Host-side dispatch over the template instantiations.
// ---------------------------------------------------------------------------
struct LaunchShape {
    int grid;
};

int device_cu_count()
{
    static int cached = -1;
    if (cached > 0)
        return cached;
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        n = 256;
    cached = n;
    return n;
}

template <typename K>
int persistent_grid(K kernel, int tpb, size_t dyn_lds, int n_items)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, tpb, dyn_lds) !=
            hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    long g = (long)per_cu * device_cu_count();
    return (int)(g < n_items ? g : n_items);
}

template <typename T, int ACC, int R, int TPB, bool PHI, bool MASK, int FORM>
hipError_t launch_fwd(const double *x, const double *m, int64_t N, const WorkItem *items,
                      int n_items, int *counter, bool persistent, const double *box_mass,
                      double *part, double *part_phi, int64_t *step_inc, hipStream_t stream)
{
    auto k = pair_sweep_kernel<T, ACC, R, TPB, PHI, MASK, FORM>;
    int grid = persistent ? persistent_grid(k, TPB, 0, n_items) : n_items;
    if (grid <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(TPB), 0, stream, x, m, N, items, n_items, counter,
                       persistent ? 1 : 0, box_mass, part, part_phi, step_inc);
    return hipGetLastError();
}

struct FwdArgs {
    const double *x, *m;
    int64_t N;
    const WorkItem *items;
    int n_items;
    int *counter;
    bool persistent;
    const double *box_mass;
    double *part, *part_phi;
    int64_t *step_inc;
    hipStream_t s;
};

template <typename T, int ACC, int R, int W, bool PHI, bool MASK>
hipError_t launch_sym(const FwdArgs &a)
{
    auto k = pair_sweep_sym_kernel<T, ACC, R, W, PHI, MASK>;
    int grid = a.persistent ? persistent_grid(k, 64 * W, 0, a.n_items) : a.n_items;
    if (grid <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * W), 0, a.s, a.x, a.m, a.N, a.items, a.n_items,
                       a.counter, a.persistent ? 1 : 0, a.box_mass, a.part, a.part_phi,
                       a.step_inc);
    return hipGetLastError();
}

template <typename T, int ACC, int R, int W>
hipError_t dispatch_sym_flags(bool phi, bool mask, const FwdArgs &a)
{
    if (phi)
        return mask ? launch_sym<T, ACC, R, W, true, true>(a)
                    : launch_sym<T, ACC, R, W, true, false>(a);
    return mask ? launch_sym<T, ACC, R, W, false, true>(a)
                : launch_sym<T, ACC, R, W, false, false>(a);
}

// Grouped symmetric sweep: a.items holds kGroupWaves items per group.
template <typename T, bool PHI, bool MASK>
hipError_t launch_sym_grp(const FwdArgs &a)
{
    auto k = pair_sweep_sym_grp_kernel<T, PHI, MASK>;
    const int n_groups = a.n_items / kGroupWaves;
    const int tpb = 64 * kGroupWaves;
    int grid = a.persistent ? persistent_grid(k, tpb, 0, n_groups) : n_groups;
    if (grid <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(tpb), 0, a.s, a.x, a.m, a.N, a.items, n_groups,
                       a.counter, a.persistent ? 1 : 0, a.box_mass, a.part, a.part_phi,
                       a.step_inc);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_sym_grp(bool phi, bool mask, const FwdArgs &a)
{
    if (a.n_items % kGroupWaves != 0)
        return hipErrorInvalidValue;
    if (phi)
        return mask ? launch_sym_grp<T, true, true>(a) : launch_sym_grp<T, true, false>(a);
    return mask ? launch_sym_grp<T, false, true>(a) : launch_sym_grp<T, false, false>(a);
}

template <typename T, int ACC>
hipError_t dispatch_sym(const TileCfg &cfg, bool phi, bool mask, const FwdArgs &a)
{
    if (cfg.group) {
        if (cfg.R != 4 || cfg.tpb != 64)
            return hipErrorInvalidValue;
        return dispatch_sym_grp<T>(phi, mask, a);
    }
    if constexpr (sizeof(T) == 4) {
        if (cfg.R == 4 && cfg.tpb == 64)
            return dispatch_sym_flags<T, ACC, 4, 1>(phi, mask, a);
        if (cfg.R == 8 && cfg.tpb == 64)
            return dispatch_sym_flags<T, ACC, 8, 1>(phi, mask, a);
        if (cfg.R == 4 && cfg.tpb == 128)
            return dispatch_sym_flags<T, ACC, 4, 2>(phi, mask, a);
    } else {
        if (cfg.R == 4 && cfg.tpb == 64)
            return dispatch_sym_flags<T, ACC, 4, 1>(phi, mask, a);
        if (cfg.R == 2 && cfg.tpb == 128)
            return dispatch_sym_flags<T, ACC, 2, 2>(phi, mask, a);
    }
    return hipErrorInvalidValue;
}

template <typename T, int ACC, int R, int TPB, int FORM>
hipError_t dispatch_fwd_flags(bool phi, bool mask, const FwdArgs &a)
{
#define COLATUS_FWD_F(P, M)                                                                   \
    return launch_fwd<T, ACC, R, TPB, P, M, FORM>(a.x, a.m, a.N, a.items, a.n_items, a.counter, \
                                                  a.persistent, a.box_mass, a.part, a.part_phi, \
                                                  a.step_inc, a.s);
    if (phi) {
        if (mask) {
            COLATUS_FWD_F(true, true)
        }
        COLATUS_FWD_F(true, false)
    }
    if (mask) {
        COLATUS_FWD_F(false, true)
    }
    COLATUS_FWD_F(false, false)
#undef COLATUS_FWD_F
}

template <typename T, int ACC, int FORM>
hipError_t dispatch_fwd_shape(const TileCfg &cfg, bool phi, bool mask, const FwdArgs &a)
{
#define COLATUS_FWD(RR, TT)                                                                  \
    if (cfg.R == RR && cfg.tpb == TT)                                                        \
        return dispatch_fwd_flags<T, ACC, RR, TT, FORM>(phi, mask, a);
    COLATUS_FWD(1, 256)
    COLATUS_FWD(2, 256)
    COLATUS_FWD(4, 256)
    COLATUS_FWD(1, 128)
    COLATUS_FWD(2, 128)
    COLATUS_FWD(4, 128)
#undef COLATUS_FWD
    return hipErrorInvalidValue;
}

template <typename T, int ACC>
hipError_t dispatch_fwd_form(int form, const TileCfg &cfg, bool phi, bool mask, const FwdArgs &a)
{
    if (form == 2)
        return dispatch_sym<T, ACC>(cfg, phi, mask, a);
    if (form == 1)
        return dispatch_fwd_shape<T, ACC, 1>(cfg, phi, mask, a);
    return dispatch_fwd_shape<T, ACC, 0>(cfg, phi, mask, a);
}

template <typename T, int ACC, int R, int TPB, int C>
hipError_t launch_adj(bool mask, const double *x, const double *m, int64_t N, const double *lam,
                      int n_cot, int c0, const WorkItem *items, int n_items, int *counter,
                      bool persistent, const double *box_mass, double *part, hipStream_t stream)
{
    if (mask) {
        auto k = adjoint_sweep_kernel<T, ACC, R, TPB, C, true>;
        int grid = persistent ? persistent_grid(k, TPB, 0, n_items) : n_items;
        hipLaunchKernelGGL(k, dim3(grid), dim3(TPB), 0, stream, x, m, N, lam, n_cot, c0, items,
                           n_items, counter, persistent ? 1 : 0, box_mass, part);
    } else {
        auto k = adjoint_sweep_kernel<T, ACC, R, TPB, C, false>;
        int grid = persistent ? persistent_grid(k, TPB, 0, n_items) : n_items;
        hipLaunchKernelGGL(k, dim3(grid), dim3(TPB), 0, stream, x, m, N, lam, n_cot, c0, items,
                           n_items, counter, persistent ? 1 : 0, box_mass, part);
    }
    return hipGetLastError();
}

template <typename T, int R, bool MASK>
hipError_t launch_adj_sym(const double *x, const double *m, int64_t N, const double *lam,
                          int n_cot, const WorkItem *items, int n_items, int *counter,
                          bool persistent, const double *box_mass, double *part, hipStream_t s)
{
    auto k = adjoint_sweep_sym_kernel<T, R, MASK>;
    const int grid = persistent ? persistent_grid(k, 64, 0, n_items) : n_items;
    for (int c = 0; c < n_cot; ++c) {
        if (c > 0 && persistent)
            hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, counter);
        hipLaunchKernelGGL(k, dim3(grid), dim3(64), 0, s, x, m, N, lam, n_cot, c, items, n_items,
                           counter, persistent ? 1 : 0, box_mass, part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename T, int ACC>
hipError_t dispatch_adj(const TileCfg &cfg, bool mask, const double *x, const double *m,
                        int64_t N, int n_cot, const double *lam, const WorkItem *items,
                        int n_items, int *counter, bool persistent, const double *box_mass,
                        double *part, hipStream_t s)
{
    if (cfg.form == 2) {
        if (cfg.R != 4 || cfg.tpb != 64)
            return hipErrorInvalidValue;
        return mask ? launch_adj_sym<T, 4, true>(x, m, N, lam, n_cot, items, n_items, counter,
                                                 persistent, box_mass, part, s)
                    : launch_adj_sym<T, 4, false>(x, m, N, lam, n_cot, items, n_items, counter,
                                                  persistent, box_mass, part, s);
    }
    // Cotangents in chunks of 8, then 4, then 1; the work counter is re-armed
    // before every chunk after the first.
    int c0 = 0;
    bool first = true;
    while (c0 < n_cot) {
        const int left = n_cot - c0;
        if (!first && persistent) {
            hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, counter);
        }
        first = false;
        hipError_t e;
        const bool r2 = cfg.R >= 2;
        if (left >= 8) {
            // eight cotangents keep 24 accumulators per target: one target per lane
            e = launch_adj<T, ACC, 1, 256, 8>(mask, x, m, N, lam, n_cot, c0, items, n_items,
                                              counter, persistent, box_mass, part, s);
            c0 += 8;
        } else if (left >= 4) {
            e = r2 ? launch_adj<T, ACC, 2, 256, 4>(mask, x, m, N, lam, n_cot, c0, items, n_items,
                                                    counter, persistent, box_mass, part, s)
                   : launch_adj<T, ACC, 1, 256, 4>(mask, x, m, N, lam, n_cot, c0, items, n_items,
                                                    counter, persistent, box_mass, part, s);
            c0 += 4;
        } else {
            e = r2 ? launch_adj<T, ACC, 2, 256, 1>(mask, x, m, N, lam, n_cot, c0, items, n_items,
                                                    counter, persistent, box_mass, part, s)
                   : launch_adj<T, ACC, 1, 256, 1>(mask, x, m, N, lam, n_cot, c0, items, n_items,
                                                    counter, persistent, box_mass, part, s);
            c0 += 1;
        }
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Periodic boundaries: the real-space part of the Ewald sum, on the work
// items of the symmetric loop (parts of 256, four targets per lane, one wave;
// each unordered pair evaluated once and applied to both particles: the
// term changes sign when the two particles swap).  Per pair, with d the
// nearest image of x_j - x_k, r = |d|:
//   w   = (r^2 + eps^2)^{-3/2} - P(alpha r) r^{-3},  P(u) = erf(u) - (2u / sqrt(pi)) e^{-u^2}
//   psi = (r^2 + eps^2)^{-1/2} - erf(alpha r) / r
// i.e. the Plummer pair of Eq. (1) less the smooth long-range part that the
// reciprocal-space sum carries; the other images are negligible (alpha is
// chosen so that the real-space kernel is below the precision's resolution
// at half the box).  r == 0 (a part's own particle, or coincident
// particles): w = 0 and psi = (eps^2)^{-1/2} (0 at eps == 0), the value the
// open-box loop gives its self pair and the O(N) kernels remove.
// FP64 pairs take coordinates relative to the item's first target, each
// wrapped to its nearest image before the subtraction, and wrap the pair's
// separation once more.  FP32 pairs take 32-bit fixed-point coordinates
// (below).  Masses multiply every term (missing particles have mass 0), and
// the slots hold them: readers are given no common mass.
// ---------------------------------------------------------------------------
template <typename T> struct EwaldReal {
    T L, invL, alpha, c2;  // c2 = 2 / sqrt(pi)
};

__device__ __forceinline__ float rint_t(float u) { return rintf(u); }
__device__ __forceinline__ double rint_t(double u) { return rint(u); }

// erf(u) and exp(-u^2) for u >= 0 (FP64 pairs): the math library's.
__device__ __forceinline__ void erf_gauss(double u, double &erf_u, double &gauss)
{
    erf_u = erf(u);
    gauss = exp(-u * u);
}

template <typename T, bool PHI>
__device__ __forceinline__ void ewald_pair(T dx, T dy, T dz, T eps2, const EwaldReal<T> &E,
                                           T &w, T &psi)
{
    const T r2 = fma_t(dx, dx, fma_t(dy, dy, dz * dz));
    const T rs = rsqrt_t(r2 + eps2);
    if (r2 > (T)0.0) {
        const T ri = rsqrt_t(r2);
        const T u = E.alpha * (r2 * ri);
        T erf_u, gauss;
        erf_gauss(u, erf_u, gauss);
        const T P = erf_u - E.c2 * u * gauss;
        w = rs * (rs * rs) - P * (ri * (ri * ri));
        if constexpr (PHI)
            psi = rs - erf_u * ri;
    } else {
        w = (T)0.0;
        if constexpr (PHI)
            psi = eps2 > (T)0.0 ? rs : (T)0.0;
    }
}

__device__ __forceinline__ double wrap_image(double d, double L)
{
    return d - L * rint(d / L);
}

// 64 steps of one source chunk (sources travel around the wave as in
// sym_chunk) against the lane's R targets.
template <typename T, int R, bool REACT, bool PHI>
__device__ __forceinline__ void ewald_chunk(T sx, T sy, T sz, T sm, T &qx, T &qy, T &qz, T &qp,
                                            const T (&xi)[R], const T (&yi)[R],
                                            const T (&zi)[R], const T (&mi)[R], T eps2,
                                            const EwaldReal<T> &E, T (&ax)[R], T (&ay)[R],
                                            T (&az)[R], T (&ap)[R])
{
    for (int k = 0; k < 64; ++k) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            T dx = sx - xi[r], dy = sy - yi[r], dz = sz - zi[r];
            dx = fma_t(-E.L, rint_t(dx * E.invL), dx);
            dy = fma_t(-E.L, rint_t(dy * E.invL), dy);
            dz = fma_t(-E.L, rint_t(dz * E.invL), dz);
            T w, psi;
            ewald_pair<T, PHI>(dx, dy, dz, eps2, E, w, psi);
            const T wt = sm * w;
            ax[r] = fma_t(wt, dx, ax[r]);
            ay[r] = fma_t(wt, dy, ay[r]);
            az[r] = fma_t(wt, dz, az[r]);
            if constexpr (PHI)
                ap[r] = fma_t(sm, psi, ap[r]);
            if constexpr (REACT) {
                const T ws = mi[r] * w;
                qx = fma_t(-ws, dx, qx);
                qy = fma_t(-ws, dy, qy);
                qz = fma_t(-ws, dz, qz);
                if constexpr (PHI)
                    qp = fma_t(mi[r], psi, qp);
            }
        }
        sx = wave_rotate(sx);
        sy = wave_rotate(sy);
        sz = wave_rotate(sz);
        sm = wave_rotate(sm);
        if constexpr (REACT) {
            qx = wave_rotate(qx);
            qy = wave_rotate(qy);
            qz = wave_rotate(qz);
            if constexpr (PHI)
                qp = wave_rotate(qp);
        }
    }
}

// One work item of FP64 pairs (kind 0: a pair of parts with the reaction;
// kind 1: a 64-target piece of a diagonal part).  Slots as the symmetric
// loop's, FP64, masses included.
template <typename T, int R, bool REACT, bool PHI>
__device__ __forceinline__ void ewald_item(const WorkItem &w, const double *__restrict__ X,
                                           const double *__restrict__ Y,
                                           const double *__restrict__ Z,
                                           const double *__restrict__ m, int64_t N,
                                           double *__restrict__ part,
                                           double *__restrict__ part_phi, const double L,
                                           const EwaldReal<T> &E)
{
    static_assert(sizeof(T) == 8, "FP32 pairs take ewald_item_fx");
    const int lane = threadIdx.x & 63;
    // reference point: the item's first target (wave-uniform)
    const double cx = X[w.i0], cy = Y[w.i0], cz = Z[w.i0];
    T xi[R], yi[R], zi[R], mi[R];
    T ax[R], ay[R], az[R], ap[R];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        valid[r] = i < w.i1;
        if (valid[r]) {
            xi[r] = (T)wrap_image(X[i] - cx, L);
            yi[r] = (T)wrap_image(Y[i] - cy, L);
            zi[r] = (T)wrap_image(Z[i] - cz, L);
            mi[r] = (T)m[i];
        } else {
            xi[r] = yi[r] = zi[r] = mi[r] = (T)0.0;
        }
        ax[r] = ay[r] = az[r] = ap[r] = (T)0.0;
    }
    const T eps2 = (T)w.eps2;
    const int n_chunks = (int)((w.j1 - w.j0 + 63) / 64);
    for (int c = 0; c < n_chunks; ++c) {
        const int64_t j = w.j0 + (int64_t)c * 64 + lane;
        const bool jv = j < w.j1;
        T sx = (T)0.0, sy = (T)0.0, sz = (T)0.0, sm = (T)0.0;
        if (jv) {
            sx = (T)wrap_image(X[j] - cx, L);
            sy = (T)wrap_image(Y[j] - cy, L);
            sz = (T)wrap_image(Z[j] - cz, L);
            sm = (T)m[j];
        }
        T qx = (T)0.0, qy = (T)0.0, qz = (T)0.0, qp = (T)0.0;
        ewald_chunk<T, R, REACT, PHI>(sx, sy, sz, sm, qx, qy, qz, qp, xi, yi, zi, mi, eps2, E,
                                      ax, ay, az, ap);
        if constexpr (REACT) {
            if (jv) {
                const int64_t rs = (int64_t)w.rslice;
                part[(rs * 3 + 0) * N + j] = qx;
                part[(rs * 3 + 1) * N + j] = qy;
                part[(rs * 3 + 2) * N + j] = qz;
                if constexpr (PHI)
                    part_phi[rs * N + j] = qp;
            }
        }
    }
    const int64_t slot = (int64_t)w.slice;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!valid[r])
            continue;
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        part[(slot * 3 + 0) * N + i] = ax[r];
        part[(slot * 3 + 1) * N + i] = ay[r];
        part[(slot * 3 + 2) * N + i] = az[r];
        if constexpr (PHI)
            part_phi[slot * N + i] = ap[r];
    }
}

// FP32 pairs on fixed-point coordinates.  Each coordinate is stored as
// round(x 2^32 / L) modulo 2^32 (FP64 arithmetic, exact for |x| below
// 2^21 L); the difference
// of two such values, read as a signed 32-bit integer, is the nearest image
// of the separation to 2^-32 L, with no wrap arithmetic, and one conversion
// gives it in FP32.  Inside the loop lengths are in units of L / 2^32; the
// stores scale the sums back (the force by (2^32 / L)^2, the potential by
// 2^32 / L).
struct EwaldFx {
    float eps2;      // eps^2 in those units
    float c_exp;     // -alpha^2 log2(e): exp(-alpha^2 r^2) = 2^(c_exp r^2)
    float c_t;       // 0.3275911 alpha
    float c_g;       // (2 / sqrt(pi)) alpha
    float phi_self;  // the r = 0 potential term: (eps^2)^{-1/2}, 0 at eps = 0
};

__device__ __forceinline__ uint32_t fx_coord(double x, double scale)
{
    double q = rint(x * scale);  // an integer; exact below 2^53
    q -= 4294967296.0 * floor(q * 2.3283064365386963e-10);  // mod 2^32
    // a non-finite coordinate (or one beyond 2^21 L) takes 0 here, a defined
    // conversion; a NaN still reaches every field through the reciprocal sums
    return q >= 0.0 && q < 4294967296.0 ? (uint32_t)q : 0u;
}

__device__ __forceinline__ uint32_t wave_rotate_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x13C, 0xF, 0xF, true);
}

// One FP32 pair.  With u = alpha r, Hastings' approximation (Abramowitz and
// Stegun 7.1.26; absolute error at most 1.5e-7, a few FP32 units of the
// kernel it enters) gives erf(u) = 1 - t p(t) g, t = 1 / (1 + 0.3275911 u),
// g = exp(-u^2), p of fourth degree, so that
// P(u) = erf(u) - (2 / sqrt(pi)) u g = 1 - g (t p + c_g r).  (Folding c_g
// into the exponent as 2^(c_exp r^2 + log2 c_g) would save the product c_g r
// but raises the exponent's rounding error sixfold.)  At r = 0 the pair's
// terms are selected (w = 0, psi = phi_self), not branched to, so that the
// target rows interleave.
template <bool PHI>
__device__ __forceinline__ void ewald_pair_fx(float dx, float dy, float dz, const EwaldFx &E,
                                              float &w, float &psi)
{
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float rs = __builtin_amdgcn_rsqf(r2 + E.eps2);
    const float ri = __builtin_amdgcn_rsqf(r2);  // +inf at r = 0: not selected
    const float r = r2 * ri;
    const float g = __builtin_amdgcn_exp2f(E.c_exp * r2);
    const float t = __builtin_amdgcn_rcpf(fmaf(E.c_t, r, 1.0f));
    const float p =
        fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f),
                     -0.284496736f),
             0.254829592f);
    const float P = fmaf(-g, fmaf(t, p, E.c_g * r), 1.0f);
    const bool nz = r2 > 0.0f;
    w = nz ? fmaf(-P, ri * (ri * ri), rs * (rs * rs)) : 0.0f;
    if constexpr (PHI) {
        const float erf_u = fmaf(-t * p, g, 1.0f);
        psi = nz ? fmaf(-erf_u, ri, rs) : E.phi_self;
    }
}

template <int R, bool REACT, bool PHI>
__device__ __forceinline__ void ewald_chunk_fx(uint32_t sx, uint32_t sy, uint32_t sz, float sm,
                                               float &qx, float &qy, float &qz, float &qp,
                                               const uint32_t (&xi)[R], const uint32_t (&yi)[R],
                                               const uint32_t (&zi)[R], const float (&mi)[R],
                                               const EwaldFx &E, float (&ax)[R], float (&ay)[R],
                                               float (&az)[R], float (&ap)[R])
{
    for (int k = 0; k < 64; ++k) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float dx = (float)(int32_t)(sx - xi[r]);
            const float dy = (float)(int32_t)(sy - yi[r]);
            const float dz = (float)(int32_t)(sz - zi[r]);
            float w, psi;
            ewald_pair_fx<PHI>(dx, dy, dz, E, w, psi);
            const float wt = sm * w;
            ax[r] = fmaf(wt, dx, ax[r]);
            ay[r] = fmaf(wt, dy, ay[r]);
            az[r] = fmaf(wt, dz, az[r]);
            if constexpr (PHI)
                ap[r] = fmaf(sm, psi, ap[r]);
            if constexpr (REACT) {
                const float ws = mi[r] * w;
                qx = fmaf(-ws, dx, qx);
                qy = fmaf(-ws, dy, qy);
                qz = fmaf(-ws, dz, qz);
                if constexpr (PHI)
                    qp = fmaf(mi[r], psi, qp);
            }
        }
        sx = wave_rotate_u(sx);
        sy = wave_rotate_u(sy);
        sz = wave_rotate_u(sz);
        sm = wave_rotate(sm);
        if constexpr (REACT) {
            qx = wave_rotate(qx);
            qy = wave_rotate(qy);
            qz = wave_rotate(qz);
            if constexpr (PHI)
                qp = wave_rotate(qp);
        }
    }
}

template <int R, bool REACT, bool PHI>
__device__ __forceinline__ void ewald_item_fx(const WorkItem &w, const double *__restrict__ X,
                                              const double *__restrict__ Y,
                                              const double *__restrict__ Z,
                                              const double *__restrict__ m, int64_t N,
                                              double *__restrict__ part,
                                              double *__restrict__ part_phi, const double L,
                                              const double alpha)
{
    const int lane = threadIdx.x & 63;
    const double sc = 4294967296.0 / L;  // fixed-point units per length
    const double a_fx = alpha / sc;      // alpha in those units
    EwaldFx E;
    E.eps2 = (float)(w.eps2 * sc * sc);
    E.c_exp = (float)(-a_fx * a_fx * 1.4426950408889634);
    E.c_t = (float)(0.3275911 * a_fx);
    E.c_g = (float)(1.1283791670955126 * a_fx);
    E.phi_self = E.eps2 > 0.0f ? __builtin_amdgcn_rsqf(E.eps2) : 0.0f;
    const double sf = sc * sc;  // force sums back to lengths
    uint32_t xi[R], yi[R], zi[R];
    float mi[R], ax[R], ay[R], az[R], ap[R];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        valid[r] = i < w.i1;
        if (valid[r]) {
            xi[r] = fx_coord(X[i], sc);
            yi[r] = fx_coord(Y[i], sc);
            zi[r] = fx_coord(Z[i], sc);
            mi[r] = (float)m[i];
        } else {
            xi[r] = yi[r] = zi[r] = 0u;
            mi[r] = 0.0f;
        }
        ax[r] = ay[r] = az[r] = ap[r] = 0.0f;
    }
    float *pf = reinterpret_cast<float *>(part);
    float *pp = reinterpret_cast<float *>(part_phi);
    const int n_chunks = (int)((w.j1 - w.j0 + 63) / 64);
    for (int c = 0; c < n_chunks; ++c) {
        const int64_t j = w.j0 + (int64_t)c * 64 + lane;
        const bool jv = j < w.j1;
        uint32_t sx = 0u, sy = 0u, sz = 0u;
        float sm = 0.0f;
        if (jv) {
            sx = fx_coord(X[j], sc);
            sy = fx_coord(Y[j], sc);
            sz = fx_coord(Z[j], sc);
            sm = (float)m[j];
        }
        float qx = 0.0f, qy = 0.0f, qz = 0.0f, qp = 0.0f;
        ewald_chunk_fx<R, REACT, PHI>(sx, sy, sz, sm, qx, qy, qz, qp, xi, yi, zi, mi, E, ax, ay,
                                      az, ap);
        if constexpr (REACT) {
            if (jv) {
                const int64_t rs = (int64_t)w.rslice;
                pf[(rs * 3 + 0) * N + j] = (float)(sf * (double)qx);
                pf[(rs * 3 + 1) * N + j] = (float)(sf * (double)qy);
                pf[(rs * 3 + 2) * N + j] = (float)(sf * (double)qz);
                if constexpr (PHI)
                    pp[rs * N + j] = (float)(sc * (double)qp);
            }
        }
    }
    const int64_t slot = (int64_t)w.slice;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!valid[r])
            continue;
        const int64_t i = w.i0 + (int64_t)(r * 64 + lane);
        pf[(slot * 3 + 0) * N + i] = (float)(sf * (double)ax[r]);
        pf[(slot * 3 + 1) * N + i] = (float)(sf * (double)ay[r]);
        pf[(slot * 3 + 2) * N + i] = (float)(sf * (double)az[r]);
        if constexpr (PHI)
            pp[slot * N + i] = (float)(sc * (double)ap[r]);
    }
}

template <typename T, bool PHI>
__global__ __launch_bounds__(64) void ewald_real_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N,
    const WorkItem *__restrict__ items, int n_items, double *__restrict__ part,
    double *__restrict__ part_phi, int64_t *__restrict__ step_inc, double L, double alpha)
{
    const double *X = x, *Y = x + N, *Z = x + 2 * N;
    if (step_inc && blockIdx.x == 0 && threadIdx.x == 0)
        *step_inc += 1;
    const int it = (int)blockIdx.x;
    if (it >= n_items)
        return;
    const WorkItem w = items[it];
    if constexpr (sizeof(T) == 4) {
        if (w.kind == 0)
            ewald_item_fx<4, true, PHI>(w, X, Y, Z, m, N, part, part_phi, L, alpha);
        else
            ewald_item_fx<1, false, PHI>(w, X, Y, Z, m, N, part, part_phi, L, alpha);
    } else {
        EwaldReal<T> E;
        E.L = (T)L;
        E.invL = (T)(1.0 / L);
        E.alpha = (T)alpha;
        E.c2 = (T)1.1283791670955126;  // 2 / sqrt(pi)
        if (w.kind == 0)
            ewald_item<T, 4, true, PHI>(w, X, Y, Z, m, N, part, part_phi, L, E);
        else
            ewald_item<T, 1, false, PHI>(w, X, Y, Z, m, N, part, part_phi, L, E);
    }
}

template <typename T, bool PHI>
hipError_t launch_ewald_real_t(const double *x, const double *m, int64_t N,
                               const WorkItem *items, int n_items, double *part,
                               double *part_phi, int64_t *step_inc, double L, double alpha,
                               hipStream_t stream)
{
    hipLaunchKernelGGL((ewald_real_kernel<T, PHI>), dim3(n_items), dim3(64), 0, stream, x, m, N,
                       items, n_items, part, part_phi, step_inc, L, alpha);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_counter(int *counter, hipStream_t stream)
{
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
    return hipGetLastError();
}

hipError_t launch_pair_sweep(int precision, int form, const TileCfg &cfg, bool with_phi,
                             bool mask_self, const double *x, const double *m, int64_t N,
                             const WorkItem *items, int n_items, int *counter, bool persistent,
                             const double *box_mass, double *part, double *part_phi,
                             int64_t *step_inc, hipStream_t stream)
{
    if (n_items <= 0)
        return hipSuccess;
    const FwdArgs a{x, m, N, items, n_items, counter, persistent, box_mass, part, part_phi,
                    step_inc, stream};
    switch (precision) {
    case kFP64:
        if (form == 2)
            return dispatch_sym<double, kDirect>(cfg, with_phi, mask_self, a);
        return dispatch_fwd_shape<double, kDirect, 0>(cfg, with_phi, mask_self, a);
    case kMixedTwoSum:
        return dispatch_fwd_form<float, kTwoSum>(form, cfg, with_phi, mask_self, a);
    case kMixedF64Acc:
        return dispatch_fwd_form<float, kFold64>(form, cfg, with_phi, mask_self, a);
    case kFP32:
        return dispatch_fwd_form<float, kDirect>(form, cfg, with_phi, mask_self, a);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ewald_real(int precision, bool with_phi, const double *x, const double *m,
                             int64_t N, const WorkItem *items, int n_items, double *part,
                             double *part_phi, int64_t *step_inc, double L, double alpha,
                             hipStream_t stream)
{
    if (n_items <= 0)
        return hipSuccess;
    if (precision == kFP64)
        return with_phi ? launch_ewald_real_t<double, true>(x, m, N, items, n_items, part,
                                                            part_phi, step_inc, L, alpha, stream)
                        : launch_ewald_real_t<double, false>(x, m, N, items, n_items, part,
                                                             part_phi, step_inc, L, alpha,
                                                             stream);
    return with_phi ? launch_ewald_real_t<float, true>(x, m, N, items, n_items, part, part_phi,
                                                       step_inc, L, alpha, stream)
                    : launch_ewald_real_t<float, false>(x, m, N, items, n_items, part, part_phi,
                                                        step_inc, L, alpha, stream);
}

// box_mass[b] = the common mass of box b, or NaN if its masses differ (or one
// is not positive).  Two passes over the whole grid: every box takes its first
// mass, then every particle whose mass differs from its box's first marks the
// box NaN.  Those marks all store the same value, so the result does not
// depend on their order.
__global__ void box_mass_seed_kernel(const double *__restrict__ m,
                                     const int64_t *__restrict__ off, int n_boxes,
                                     double *__restrict__ box_mass)
{
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= n_boxes)
        return;
    const double m0 = m[off[b]];
    box_mass[b] = m0 > 0.0 ? m0 : NAN;
}

__global__ void box_mass_check_kernel(const double *__restrict__ m,
                                      const int64_t *__restrict__ off, int n_boxes, int64_t N,
                                      double *__restrict__ box_mass)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    // the box holding particle i: the last b with off[b] <= i
    int lo = 0, hi = n_boxes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const double mi = m[i];
    if (mi != m[off[lo]] || !(mi > 0.0))
        box_mass[lo] = NAN;
}

hipError_t launch_box_mass(const double *m, const int64_t *box_offsets, int n_boxes, int64_t N,
                           double *box_mass, hipStream_t stream)
{
    if (n_boxes < 1 || N < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(box_mass_seed_kernel, dim3((unsigned)((n_boxes + 63) / 64)), dim3(64), 0,
                       stream, m, box_offsets, n_boxes, box_mass);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(box_mass_check_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                       stream, m, box_offsets, n_boxes, N, box_mass);
    return hipGetLastError();
}

hipError_t launch_adjoint_sweep(int precision, const TileCfg &cfg, bool mask_self,
                                const double *x, const double *m, int64_t N, int n_cot,
                                const double *lam, const WorkItem *items, int n_items,
                                int *counter, bool persistent, const double *box_mass,
                                double *part, hipStream_t stream)
{
    if (n_items <= 0)
        return hipSuccess;
    switch (precision) {
    case kFP64:
        return dispatch_adj<double, kDirect>(cfg, mask_self, x, m, N, n_cot, lam, items,
                                             n_items, counter, persistent, box_mass, part, stream);
    case kMixedTwoSum:
        return dispatch_adj<float, kTwoSum>(cfg, mask_self, x, m, N, n_cot, lam, items,
                                            n_items, counter, persistent, box_mass, part, stream);
    case kMixedF64Acc:
        return dispatch_adj<float, kFold64>(cfg, mask_self, x, m, N, n_cot, lam, items,
                                            n_items, counter, persistent, box_mass, part, stream);
    case kFP32:
        return dispatch_adj<float, kDirect>(cfg, mask_self, x, m, N, n_cot, lam, items,
                                            n_items, counter, persistent, box_mass, part, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace colatus
