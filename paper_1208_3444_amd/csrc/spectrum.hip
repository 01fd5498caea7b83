// Velocity power spectrum of tracer tracks: for each tracer, the periodogram
// of its velocity series over the track's rows (the power spectrum of a
// single particle's velocity that Section I names as the method's goal),
//   E(k) = (1/M) sum_c | sum_{n<M} w_c[n] exp(-2 pi i k n / M) |^2,  k <= M/2.
//
// A direct transform in FP64: M is the number of grid points of a run (about
// a thousand), so the O(M^2) sum per tracer is microseconds and keeps every
// bin an independent, fixed-order sum.  One thread per (tracer, k); a block
// covers 256 consecutive k of one tracer and stages the tracer's three
// velocity columns through LDS in chunks, every lane then reading the same
// LDS word (a broadcast).  The twiddle factors come from a table of the M
// roots of unity, indexed by k n reduced modulo M exactly (an integer
// recurrence), so no angle is ever formed from a large product.
#include "colatus_internal.h"

#include <hip/hip_runtime.h>

namespace colatus {

namespace {

constexpr int kSpecThreads = 256;
constexpr int kSpecChunk = 1024;  // rows staged per LDS pass (24 KB)

// W[j] = exp(-2 pi i j / M) as (cos, -sin), j < M.
__global__ void twiddle_kernel(double2 *__restrict__ W, int64_t M)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M)
        return;
    double s, c;
    sincospi(2.0 * ((double)j / (double)M), &s, &c);
    W[j] = make_double2(c, -s);
}

__global__ __launch_bounds__(kSpecThreads) void spectrum_kernel(
    const double *__restrict__ track, int64_t M, int32_t T, int remove_mean,
    const double2 *__restrict__ W, int64_t K, int64_t k_blocks, double *__restrict__ out)
{
    __shared__ double wv[3][kSpecChunk];
    __shared__ double red[3][kSpecThreads];
    const int64_t t = blockIdx.x / k_blocks;
    const int64_t k = (blockIdx.x % k_blocks) * kSpecThreads + threadIdx.x;
    const int tid = threadIdx.x;
    const int64_t row = 6 * (int64_t)T;
    const double *v0 = track + 3 * (int64_t)T + t;  // v_c of tracer t at row n: v0[n row + c T]

    double mu[3] = {0.0, 0.0, 0.0};
    if (remove_mean) {
        // fixed-order block sum: strided partial per thread, then a tree
        double s[3] = {0.0, 0.0, 0.0};
        for (int64_t n = tid; n < M; n += kSpecThreads)
            for (int c = 0; c < 3; ++c)
                s[c] += v0[n * row + c * (int64_t)T];
        for (int c = 0; c < 3; ++c)
            red[c][tid] = s[c];
        __syncthreads();
        for (int h = kSpecThreads / 2; h > 0; h >>= 1) {
            if (tid < h)
                for (int c = 0; c < 3; ++c)
                    red[c][tid] += red[c][tid + h];
            __syncthreads();
        }
        for (int c = 0; c < 3; ++c)
            mu[c] = red[c][0] / (double)M;
    }

    double re[3] = {0.0, 0.0, 0.0}, im[3] = {0.0, 0.0, 0.0};
    const int64_t kk = k < K ? k : 0;  // idle lanes still stage and sync
    int64_t j = 0;                     // k n mod M
    for (int64_t n0 = 0; n0 < M; n0 += kSpecChunk) {
        const int len = (int)(M - n0 < kSpecChunk ? M - n0 : kSpecChunk);
        __syncthreads();
        for (int q = tid; q < len; q += kSpecThreads)
            for (int c = 0; c < 3; ++c)
                wv[c][q] = v0[(n0 + q) * row + c * (int64_t)T] - mu[c];
        __syncthreads();
        for (int q = 0; q < len; ++q) {
            const double2 w = W[j];
            for (int c = 0; c < 3; ++c) {
                re[c] = fma(wv[c][q], w.x, re[c]);
                im[c] = fma(wv[c][q], w.y, im[c]);
            }
            j += kk;
            if (j >= M)
                j -= M;
        }
    }
    if (k < K) {
        double e = 0.0;
        for (int c = 0; c < 3; ++c)
            e += re[c] * re[c] + im[c] * im[c];
        out[t * K + k] = e / (double)M;
    }
}

}  // namespace

hipError_t launch_velocity_spectrum(const double *track, int64_t M, int32_t T, int remove_mean,
                                    double *twiddle, double *out, hipStream_t stream)
{
    double2 *W = reinterpret_cast<double2 *>(twiddle);
    hipLaunchKernelGGL(twiddle_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, stream,
                       W, M);
    const int64_t K = M / 2 + 1;
    const int64_t kb = (K + kSpecThreads - 1) / kSpecThreads;
    hipLaunchKernelGGL(spectrum_kernel, dim3((unsigned)(kb * T)), dim3(kSpecThreads), 0, stream,
                       track, M, T, remove_mean, W, K, kb, out);
    return hipGetLastError();
}

}  // namespace colatus
