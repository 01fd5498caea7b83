// Periodic boundaries (Section II solves the motion equations in a periodic
// box): the reciprocal-space part of the Ewald sum, its constants, and the
// O(N) epilogue that adds them to the real-space part the pair sweep
// computes (pair_sweep.hip, ewald_real_kernel).
//
// With the box side L, splitting parameter alpha and reciprocal vectors
// k = 2 pi n / L, n != 0, |n| <= n_max, taken over half of k-space (each k
// stands for k and -k, hence the factor 2 in its weight):
//   S(k)   = sum_j m_j exp(i k . x_j)                       (structure factor)
//   c(k)   = 2 (4 pi / L^3) exp(-k^2 / (4 alpha^2)) / k^2
//   W(k)   = c(k) S(k)
//   g_k^K  = sum_k k Im(exp(-i k . x_i) W(k))                (field, no G)
//   psi^K  = sum_k Re(exp(-i k . x_i) W(k))                  (potential part)
// Phases start from sincospi of the exact phase at the first k of a short
// run of consecutive n_z (a column segment) and advance by multiplying with
// exp(+-i 2 pi z / L): at most fifteen FP64 products per segment.
#include "colatus_internal.h"

#include <math.h>

namespace colatus {
namespace {

constexpr int kSegThreads = 64;  // segments per block, one per lane
constexpr int kSkWaves = 4;      // waves per block, each on a quarter of a particle tile
constexpr int kSkTile = 256;     // particles staged in LDS at a time

// Partial structure factors: block (segments b*64.., particle chunk c):
// out[c][k] = sum over the chunk's particles j of m_j exp(i k . x_j), for
// every k of each lane's segment.  The four waves of a block share the
// segments and split every staged tile of 256 particles into quarters (in
// index order within each); their sums are added in wave order, so the
// result is fixed.  The split keeps four times as many waves in flight as
// one wave per block would, for the same partial-sum buffer.
__global__ __launch_bounds__(kSegThreads * kSkWaves) void ewald_sk_kernel(
    const double *__restrict__ x, const double *__restrict__ m, int64_t N, int64_t chunk,
    const EwaldSeg *__restrict__ segs, int n_segs, int K, double inv_L,
    double2 *__restrict__ part)
{
    __shared__ double sx[kSkTile], sy[kSkTile], sz[kSkTile], sm[kSkTile], scz[kSkTile],
        ssz[kSkTile];
    __shared__ double2 red[kSkWaves][4][kSegThreads];
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int s = (int)(blockIdx.x * kSegThreads) + lane;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
    EwaldSeg g = {0, 0, 0, 0, 0};
    if (s < n_segs)
        g = segs[s];
    double re[kEwaldSegLen], im[kEwaldSegLen];
#pragma unroll
    for (int q = 0; q < kEwaldSegLen; ++q)
        re[q] = im[q] = 0.0;
    for (int64_t t0 = j0; t0 < j1; t0 += kSkTile) {
        __syncthreads();
        for (int u = (int)threadIdx.x; u < kSkTile; u += kSegThreads * kSkWaves) {
            const int64_t j = t0 + u;
            if (j < j1) {
                sx[u] = x[j];
                sy[u] = x[N + j];
                sz[u] = x[2 * N + j];
                sm[u] = m[j];
                double c, sn;
                sincospi(2.0 * x[2 * N + j] * inv_L, &sn, &c);
                scz[u] = c;
                ssz[u] = sn;
            }
        }
        __syncthreads();
        const int nt = (int)((j1 - t0) < kSkTile ? (j1 - t0) : kSkTile);
        const int per = kSkTile / kSkWaves;
        const int u0 = wave * per, u1 = u0 + per < nt ? u0 + per : nt;
        if (s < n_segs) {
            for (int u = u0; u < u1; ++u) {
                double c, sn;
                sincospi(2.0 * (g.nx * sx[u] + g.ny * sy[u] + g.z0 * sz[u]) * inv_L, &sn, &c);
                double er = sm[u] * c, ei = sm[u] * sn;
                const double zr = scz[u], zi = ssz[u];
#pragma unroll
                for (int q = 0; q < kEwaldSegLen; ++q) {
                    if (q < g.cnt) {
                        re[q] += er;
                        im[q] += ei;
                        const double tr = er * zr - ei * zi;
                        ei = er * zi + ei * zr;
                        er = tr;
                    }
                }
            }
        }
    }
    // the waves' sums, four k at a time, added in wave order by wave 0
#pragma unroll
    for (int q0 = 0; q0 < kEwaldSegLen; q0 += 4) {
#pragma unroll
        for (int dq = 0; dq < 4; ++dq)
            red[wave][dq][lane] = make_double2(re[q0 + dq], im[q0 + dq]);
        __syncthreads();
        if (wave == 0 && s < n_segs) {
#pragma unroll
            for (int dq = 0; dq < 4; ++dq) {
                if (q0 + dq < g.cnt) {
                    double2 v = red[0][dq][lane];
#pragma unroll
                    for (int w = 1; w < kSkWaves; ++w) {
                        v.x += red[w][dq][lane].x;
                        v.y += red[w][dq][lane].y;
                    }
                    part[(int64_t)blockIdx.y * K + g.k0 + q0 + dq] = v;
                }
            }
        }
        __syncthreads();
    }
}

// W(k) = c(k) S(k), S(k) the sum over the chunks: a block takes 32
// consecutive k, its eight thread groups every eighth chunk each (in chunk
// order), and the groups' sums are added in group order.
constexpr int kRedK = 32, kRedGroups = 8;
__global__ __launch_bounds__(kRedK * kRedGroups) void ewald_sk_reduce_kernel(
    const double2 *__restrict__ part, int n_chunks, int K, const double *__restrict__ coef,
    double2 *__restrict__ W)
{
    __shared__ double2 red[kRedGroups][kRedK];
    const int kl = (int)(threadIdx.x % kRedK), grp = (int)(threadIdx.x / kRedK);
    const int k = (int)blockIdx.x * kRedK + kl;
    double r = 0.0, i = 0.0;
    if (k < K) {
        for (int c = grp; c < n_chunks; c += kRedGroups) {
            const double2 v = part[(int64_t)c * K + k];
            r += v.x;
            i += v.y;
        }
    }
    red[grp][kl] = make_double2(r, i);
    __syncthreads();
    if (grp == 0 && k < K) {
        for (int g = 1; g < kRedGroups; ++g) {
            r += red[g][kl].x;
            i += red[g][kl].y;
        }
        W[k] = make_double2(coef[k] * r, coef[k] * i);
    }
}

// Per particle i and range of segments (blockIdx.y): partial sums of the
// reciprocal-space field (no G) and potential part,
//   pg[kc][c][i] = sum_k k_c Im(exp(-i k.x_i) W(k)),
//   pp[kc][i]    = sum_k Re(exp(-i k.x_i) W(k)),
// over the segments of range kc, in segment order.  Within a segment of n
// consecutive n_z = z0 + q the terms w_q = Im(exp(-i k.x_i) W(k)) enter the
// field as (2 pi / L) (n_x, n_y, z0 + q) w_q; the running sums T_q =
// sum_{r <= q} w_r and U = sum_q T_q give sum_q q w_q = n T - U, so each k
// costs two complex multiply-adds and the phase step.  Four waves (256
// particles) share each staged run of segments.
constexpr int kKfThreads = 256;
__global__ __launch_bounds__(kKfThreads) void ewald_kforce_kernel(
    const double *__restrict__ x, int64_t N, const EwaldSeg *__restrict__ segs, int n_segs,
    int segs_per_chunk, const double2 *__restrict__ W, double inv_L, double *__restrict__ pg,
    double *__restrict__ pp)
{
    __shared__ EwaldSeg sseg[64];
    __shared__ double2 sW[64 * kEwaldSegLen];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < N;
    const double xi = valid ? x[i] : 0.0, yi = valid ? x[N + i] : 0.0,
                 zi = valid ? x[2 * N + i] : 0.0;
    double cz, sz;
    sincospi(2.0 * zi * inv_L, &sz, &cz);
    const double two_pi_L = 2.0 * 3.14159265358979323846 * inv_L;
    const int sb = (int)blockIdx.y * segs_per_chunk;
    const int se = sb + segs_per_chunk < n_segs ? sb + segs_per_chunk : n_segs;
    double fx = 0.0, fy = 0.0, fz = 0.0, fp = 0.0;
    for (int s0 = sb; s0 < se; s0 += 64) {
        const int ns = se - s0 < 64 ? se - s0 : 64;
        __syncthreads();
        for (int u = threadIdx.x; u < ns; u += blockDim.x)
            sseg[u] = segs[s0 + u];
        __syncthreads();
        // the k of consecutive segments are consecutive from sseg[0].k0
        const int kb = sseg[0].k0;
        const int kn = sseg[ns - 1].k0 + sseg[ns - 1].cnt - kb;
        for (int u = threadIdx.x; u < kn; u += blockDim.x)
            sW[u] = W[kb + u];
        __syncthreads();
        for (int t = 0; t < ns; ++t) {
            const EwaldSeg g = sseg[t];
            double c, sn;
            // exp(-i k.x_i) at the segment's first k, then exp(-i 2 pi z / L) steps
            sincospi(2.0 * (g.nx * xi + g.ny * yi + g.z0 * zi) * inv_L, &sn, &c);
            double er = c, ei = -sn;
            double P = 0.0, T = 0.0, U = 0.0;
            const double2 *wk = sW + (g.k0 - kb);
            for (int q = 0; q < g.cnt; ++q) {
                const double2 w = wk[q];
                P = fma(er, w.x, P);
                P = fma(-ei, w.y, P);
                T = fma(er, w.y, T);
                T = fma(ei, w.x, T);
                U += T;
                const double tr = er * cz + ei * sz;
                ei = ei * cz - er * sz;
                er = tr;
            }
            fp += P;
            fx = fma(two_pi_L * g.nx, T, fx);
            fy = fma(two_pi_L * g.ny, T, fy);
            fz = fma(two_pi_L, (double)(g.z0 + g.cnt) * T - U, fz);
        }
    }
    if (valid) {
        const int64_t kc = blockIdx.y;
        pg[(kc * 3 + 0) * N + i] = fx;
        pg[(kc * 3 + 1) * N + i] = fy;
        pg[(kc * 3 + 2) * N + i] = fz;
        pp[kc * N + i] = fp;
    }
}

// gk[c][i] = sum over ranges kc (in order) of pg; pk[i] likewise plus
// m_i self_c + bg_c M, with self_c = -2 alpha / sqrt(pi) (the real-space
// self term; the particle's other images are below resolution) and
// bg_c = -pi / (alpha^2 L^3) (the removed background).
__global__ void ewald_kreduce_kernel(const double *__restrict__ pg, const double *__restrict__ pp,
                                     int n_kc, int64_t N, const double *__restrict__ m,
                                     double self_c, const double *__restrict__ msum, double bg_c,
                                     double *__restrict__ gk, double *__restrict__ pk)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    double f[3] = {0.0, 0.0, 0.0}, p = 0.0;
    for (int kc = 0; kc < n_kc; ++kc) {
        for (int c = 0; c < 3; ++c)
            f[c] += pg[((int64_t)kc * 3 + c) * N + i];
        p += pp[(int64_t)kc * N + i];
    }
    for (int c = 0; c < 3; ++c)
        gk[c * N + i] = f[c];
    pk[i] = p + m[i] * self_c + bg_c * msum[0];
}

// Total mass, one block, fixed order (for the background constant).
__global__ __launch_bounds__(1024) void ewald_mass_kernel(const double *__restrict__ m, int64_t N,
                                                          double *__restrict__ out)
{
    __shared__ double sh[1024];
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += 1024)
        t += m[i];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = sh[0];
}

// acc += (G / a^3) g^K; phi += -G psi^K (colatus_forces_periodic's epilogue).
__global__ void ewald_add_kernel(const double *__restrict__ gk, const double *__restrict__ pk,
                                 int64_t N, double G, double inv_a3, double *__restrict__ acc,
                                 double *__restrict__ phi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    for (int c = 0; c < 3; ++c)
        acc[c * N + i] += G * inv_a3 * gk[c * N + i];
    if (phi)
        phi[i] += -G * pk[i];
}

}  // namespace

hipError_t launch_ewald_kspace(const EwaldArgs &A, hipStream_t stream)
{
    const double inv_L = 1.0 / A.L;
    const int64_t N = A.N;
    const int64_t chunk = (N + A.n_sk_chunks - 1) / A.n_sk_chunks;
    hipError_t e = hipSuccess;
    if (!A.mass_ready) {
        hipLaunchKernelGGL(ewald_mass_kernel, dim3(1), dim3(1024), 0, stream, A.m, N, A.msum);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const double pi = 3.14159265358979323846;
    const double self_c = -2.0 * A.alpha / sqrt(pi);
    const double bg_c = -pi / (A.alpha * A.alpha * A.L * A.L * A.L);
    if (A.n_segs > 0) {
        hipLaunchKernelGGL(ewald_sk_kernel,
                           dim3((unsigned)((A.n_segs + kSegThreads - 1) / kSegThreads),
                                (unsigned)A.n_sk_chunks),
                           dim3(kSegThreads * kSkWaves), 0, stream, A.x, A.m, N, chunk,
                           A.segs_sk, A.n_segs, A.K, inv_L, A.sk_part);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(ewald_sk_reduce_kernel, dim3((unsigned)((A.K + kRedK - 1) / kRedK)),
                           dim3(kRedK * kRedGroups), 0, stream, A.sk_part, A.n_sk_chunks, A.K,
                           A.coef, A.S);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const int spc = (A.n_segs + A.n_k_chunks - 1) / A.n_k_chunks;
    const int n_kc = A.n_segs > 0 ? (A.n_segs + spc - 1) / spc : 0;
    if (n_kc > 0) {
        hipLaunchKernelGGL(ewald_kforce_kernel,
                           dim3((unsigned)((N + kKfThreads - 1) / kKfThreads), (unsigned)n_kc),
                           dim3(kKfThreads), 0, stream, A.x, N, A.segs, A.n_segs, spc, A.S, inv_L,
                           A.kpart_g, A.kpart_p);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(ewald_kreduce_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                       stream, A.kpart_g, A.kpart_p, n_kc, N, A.m, self_c, A.msum, bg_c, A.gk,
                       A.pk);
    return hipGetLastError();
}

hipError_t launch_ewald_add(const double *gk, const double *pk, int64_t N, double G,
                            double inv_a3, double *acc, double *phi, hipStream_t stream)
{
    hipLaunchKernelGGL(ewald_add_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream,
                       gk, pk, N, G, inv_a3, acc, phi);
    return hipGetLastError();
}

}  // namespace colatus
