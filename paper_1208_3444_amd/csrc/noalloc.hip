// colatus_forces_noalloc: the pair sum of colatus_forces for callers that
// cannot allocate device memory (work under stream capture, serving loops,
// harnesses that forbid hipMalloc).  Every scratch byte the call needs (the
// work items, the O(N) blocks, the box's common mass, the partial-sum slots)
// lives in one file-scope device array; the items and blocks are generated
// on the device, so the call makes no allocation and no host-to-device copy.
//
// It runs the kernels of colatus_forces with the symmetric form's tile shape
// (parts of 256 particles, four targets per lane, 2x2 groups of part pairs
// per workgroup), so with that form selected the two entry points give the
// same bits (colatus_forces takes the ordered loop for boxes too small to
// fill the GPU with symmetric items, and then agrees to rounding).
#include "colatus.h"
#include "colatus_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

namespace colatus {
namespace {

// Largest N the scratch holds, for every precision, with the potential.
constexpr int64_t kNoAllocMaxN = 16384;
constexpr int64_t kPart = 256;   // particles per part (4 targets x 64 lanes)
constexpr int64_t kPiece = 64;   // targets per piece of a diagonal part
constexpr int64_t kMaxParts = kNoAllocMaxN / kPart;
constexpr int64_t kMaxSupers = (kMaxParts + 1) / 2;  // super-parts of two parts
constexpr int64_t kMaxLoose = kMaxParts / 2 + kMaxParts * (kPart / kPiece);
constexpr int64_t kMaxItems =
    4 * (kMaxSupers * (kMaxSupers - 1) / 2 + (kMaxLoose + 3) / 4);
constexpr int64_t kMaxSlots = kMaxSupers + 1;  // partial-sum slots per particle
constexpr int64_t kMaxBlocks = kNoAllocMaxN / kIntBlock;

constexpr size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
// Byte offsets of the regions of the scratch array.
constexpr size_t kOffCounter = 0;    // int: pair-sweep work counter
constexpr size_t kOffOffsets = 256;  // int64[2]: box offsets {0, N}
constexpr size_t kOffBoxMass = 512;  // double: the box's common mass or NaN
constexpr size_t kOffBlocks = 768;   // IntBlock[kMaxBlocks]
constexpr size_t kOffItems = kOffBlocks + round256(kMaxBlocks * sizeof(IntBlock));
constexpr size_t kOffPart = kOffItems + round256(kMaxItems * sizeof(WorkItem));
constexpr size_t kPartBytes = (size_t)kMaxSlots * 3 * kNoAllocMaxN * sizeof(double);
constexpr size_t kOffPhi = kOffPart + kPartBytes;
constexpr size_t kPhiBytes = (size_t)kMaxSlots * kNoAllocMaxN * sizeof(double);
constexpr size_t kScratchBytes = kOffPhi + kPhiBytes;  // about 17.4 MB

// The scratch array: one copy per device, held until the process ends.  Host
// code never passes this name to a kernel (on the host it is only a handle);
// it uses the device address hipGetSymbolAddress returns for the current
// device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[kMaxDevices] = {};

// Device address of the scratch array on device `dev` (current), looked up
// once per device.
int scratch_address(int dev, unsigned char *&out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return COLATUS_ENODEV;
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return COLATUS_EHIP;
        g_na_ptr[dev] = static_cast<unsigned char *>(p);
    }
    out = g_na_ptr[dev];
    return COLATUS_OK;
}

// Work items and blocks of one box [0, N) in the grouped symmetric form,
// written by one thread each, four items per group.  Parts pair up into
// super-parts {2A, 2A+1}; groups [0, n_blk) are the 2x2 blocks of super-parts
// A < B in row order of the (A, B) triangle: wave 2a + b pairs part 2A + a
// (targets, slot B) with part 2B + b (sources, reaction in slot A), and the
// waves sharing a part add their partial sums (tmate, rmate); a missing part
// leaves a padding item.  The remaining groups hold the loose items four at
// a time: the pair inside each full super-part (slot A on both sides), then
// the 64-target pieces of the diagonal parts (part j / 4, piece j % 4; slot
// ceil(P/2), or A for a part alone in its super-part), then padding.  Every
// particle gets ceil(P/2) + 1 slots (ceil(P/2) in a lone part).  The order of
// the groups does not change the result (each slot is written by one group).
// The functions below are plain host-and-device code, so the list can be
// checked on the host.
//
// Work item t (t < n_items) of that list.
__host__ __device__ inline WorkItem noalloc_item(int t, int64_t N, double eps, int P, int n_blk,
                                                 int n_intra, int n_pieces)
{
    const int S2 = (P + 1) / 2;
    WorkItem w{};
    w.eps2 = eps * eps;
    w.box = 0;
    w.kind = -1;
    const int g = t / 4, e = t % 4;
    if (g < n_blk) {
        int k = g, A = 0;
        while (k >= S2 - 1 - A) {
            k -= S2 - 1 - A;
            ++A;
        }
        const int B = A + 1 + k;
        const int a = e >> 1, b = e & 1;
        const int p = 2 * A + a, q = 2 * B + b;
        if (p < P && q < P) {
            w.i0 = (int64_t)p * kPart;
            w.i1 = w.i0 + kPart < N ? w.i0 + kPart : N;
            w.j0 = (int64_t)q * kPart;
            w.j1 = w.j0 + kPart < N ? w.j0 + kPart : N;
            w.slice = B;
            w.rslice = A;
            w.kind = 0;
            w.tmate = (int8_t)(2 * B + (1 - b) < P);
            w.rmate = (int8_t)(2 * A + (1 - a) < P);
        }
    } else {
        const int l = (g - n_blk) * 4 + e;
        if (l < n_intra) {
            w.i0 = (int64_t)(2 * l) * kPart;
            w.i1 = w.i0 + kPart < N ? w.i0 + kPart : N;
            w.j0 = (int64_t)(2 * l + 1) * kPart;
            w.j1 = w.j0 + kPart < N ? w.j0 + kPart : N;
            w.slice = l;
            w.rslice = l;
            w.kind = 0;
        } else if (l - n_intra < n_pieces) {
            const int j = l - n_intra, p = j / (int)(kPart / kPiece), i = j % (int)(kPart / kPiece);
            const int64_t p0 = (int64_t)p * kPart, p1 = p0 + kPart < N ? p0 + kPart : N;
            w.i0 = p0 + (int64_t)i * kPiece;
            w.i1 = w.i0 + kPiece < p1 ? w.i0 + kPiece : p1;
            w.j0 = p0;
            w.j1 = p1;
            w.slice = (p ^ 1) < P ? S2 : p / 2;
            w.rslice = w.slice;
            w.kind = 1;
        }
    }
    return w;
}

// IntBlock t (t < n_blocks): 64 particles, the slot count of their part.
__host__ __device__ inline IntBlock noalloc_block(int t, int64_t N, double eps, int P)
{
    const int S2 = (P + 1) / 2;
    IntBlock b;
    b.i0 = (int64_t)t * kIntBlock;
    b.i1 = b.i0 + kIntBlock < N ? b.i0 + kIntBlock : N;
    b.eps = eps;
    b.box = 0;
    const int p = (int)(b.i0 / kPart);
    b.n_slices = (p ^ 1) < P ? S2 + 1 : S2;
    return b;
}

// The list's sizes for N particles (P parts of 256).
struct NoAllocSizes {
    int P, n_blk, n_intra, n_pieces, n_items, n_blocks;
};
__host__ __device__ inline NoAllocSizes noalloc_sizes(int64_t N)
{
    NoAllocSizes z;
    z.P = (int)((N + kPart - 1) / kPart);
    const int S2 = (z.P + 1) / 2;
    z.n_blk = S2 * (S2 - 1) / 2;
    z.n_intra = z.P / 2;
    const int64_t last_len = N - (int64_t)(z.P - 1) * kPart;
    z.n_pieces = (z.P - 1) * (int)(kPart / kPiece) + (int)((last_len + kPiece - 1) / kPiece);
    z.n_items = 4 * (z.n_blk + (z.n_intra + z.n_pieces + 3) / 4);
    z.n_blocks = (int)((N + kIntBlock - 1) / kIntBlock);
    return z;
}

// One thread per item and block; also the box offsets and the cleared work
// counter.
__global__ void noalloc_setup_kernel(int64_t N, double eps, int P, int n_blk, int n_intra,
                                     int n_pieces, int n_items, int n_blocks,
                                     WorkItem *__restrict__ items, IntBlock *__restrict__ blocks,
                                     int64_t *__restrict__ offsets, int *__restrict__ counter)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t == 0) {
        offsets[0] = 0;
        offsets[1] = N;
        *counter = 0;
    }
    if (t < n_items)
        items[t] = noalloc_item(t, N, eps, P, n_blk, n_intra, n_pieces);
    if (t < n_blocks)
        blocks[t] = noalloc_block(t, N, eps, P);
}

}  // namespace
}  // namespace colatus

using namespace colatus;

extern "C" int colatus_forces_noalloc(const double *x, const double *m, int64_t N, double eps,
                                      double G, double a, int precision, double *acc,
                                      double *phi, const colatus_attractor *attractor,
                                      const colatus_background *background, void *stream)
{
    if (N < 1 || precision < COLATUS_FP64 || precision > COLATUS_FP32 || !std::isfinite(G) ||
        !std::isfinite(a) || a <= 0.0 || !std::isfinite(eps) || eps < 0.0)
        return COLATUS_EINVAL;
    if (N > kNoAllocMaxN)
        return COLATUS_ESCRATCH;
    if (!x || !m || !acc)
        return COLATUS_EINVAL;
    ExtField ext;
    if (resolve_external(attractor, background, ext) != COLATUS_OK)
        return COLATUS_EINVAL;
    int dev = 0;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1 || hipGetDevice(&dev) != hipSuccess)
        return COLATUS_ENODEV;
    unsigned char *base = nullptr;
    const int rc = scratch_address(dev, base);
    if (rc != COLATUS_OK)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);

    int *counter = reinterpret_cast<int *>(base + kOffCounter);
    int64_t *offsets = reinterpret_cast<int64_t *>(base + kOffOffsets);
    double *box_mass = reinterpret_cast<double *>(base + kOffBoxMass);
    IntBlock *blocks = reinterpret_cast<IntBlock *>(base + kOffBlocks);
    WorkItem *items = reinterpret_cast<WorkItem *>(base + kOffItems);
    double *part = reinterpret_cast<double *>(base + kOffPart);
    double *part_phi = reinterpret_cast<double *>(base + kOffPhi);

    const NoAllocSizes z = noalloc_sizes(N);
    const int P = z.P, n_items = z.n_items, n_blocks = z.n_blocks;
    if (n_items > kMaxItems || n_blocks > kMaxBlocks)
        return COLATUS_ESCRATCH;
    const int n_setup = n_items > n_blocks ? n_items : n_blocks;
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3((unsigned)((n_setup + 255) / 256)), dim3(256),
                       0, s, N, eps, P, z.n_blk, z.n_intra, z.n_pieces, n_items, n_blocks,
                       items, blocks, offsets, counter);
    if (hipGetLastError() != hipSuccess)
        return COLATUS_EHIP;
    if (launch_box_mass(m, offsets, 1, N, box_mass, s) != hipSuccess)
        return COLATUS_EHIP;
    TileCfg cfg{4, 64, P, 2};
    cfg.group = 1;
    if (launch_pair_sweep(precision, cfg.form, cfg, phi != nullptr, eps == 0.0, x, m, N, items,
                          n_items, counter, false, box_mass, part, phi ? part_phi : nullptr,
                          nullptr, s) != hipSuccess)
        return COLATUS_EHIP;
    if (launch_forces_finalize(precision, box_mass, blocks, n_blocks, part,
                               phi ? part_phi : nullptr, slot_mode_for(cfg, precision), x, m, N,
                               G, G / (a * a * a), ext, 1.0 / (a * a * a), acc, phi,
                               s) != hipSuccess)
        return COLATUS_EHIP;
    return COLATUS_OK;
}
