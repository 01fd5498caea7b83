// C ABI of libcolatus: argument validation, scratch management, work lists,
// tile-shape selection (heuristic or autotuned), hipGraph replay of the run's
// repeated step, pair-sweep timers, and the drivers of colatus_forces,
// colatus_step, colatus_run, colatus_adjoint and colatus_force_vjp.
#include "colatus.h"
#include "colatus_internal.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

using namespace colatus;

namespace {

constexpr int64_t kMaxN = (int64_t)1 << 28;
constexpr int kMaxCot = 4096;

// ---------------------------------------------------------------------------
// Options.
// ---------------------------------------------------------------------------
// Atomic: the roctx switch is read before an entry point takes the lock.
struct Options {
    std::atomic<int64_t> graph{0};  // measured no faster than eager launches
    std::atomic<int64_t> timer{0};
    std::atomic<int64_t> autotune{0};
    std::atomic<int64_t> tile_r{0};
    std::atomic<int64_t> tile_tpb{0};
    std::atomic<int64_t> tile_slices{0};
    std::atomic<int64_t> persistent{0};  // one-shot grid measured faster on gfx950
    std::atomic<int64_t> pair_form{-1};  // -1: heuristic or tuned
    std::atomic<int64_t> roctx{0};       // 1: roctx ranges around calls and eager steps
    std::atomic<int64_t> pair_group{1};  // 1: 2x2 groups of part pairs (forward, form 2)
};
Options g_opt;
std::mutex g_mu;  // guards the workspace map, tuned shapes and timers

// A roctx range for the lifetime of the object, when COLATUS_OPT_ROCTX is on
// (host-side marks for rocprofv3's marker trace; names are static strings).
struct TraceRange {
    bool on;
    explicit TraceRange(const char *name) : on(g_opt.roctx != 0)
    {
        if (on)
            roctxRangePush(name);
    }
    ~TraceRange()
    {
        if (on)
            roctxRangePop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// ---------------------------------------------------------------------------
// Validation helpers (host only; nothing touches HIP before they pass).
// ---------------------------------------------------------------------------
bool is_fin(double v) { return std::isfinite(v); }

struct Boxes {
    std::vector<int64_t> off;  // n_boxes + 1
    std::vector<double> eps;   // n_boxes
    int64_t max_n = 0;
};

int resolve_boxes(int64_t N, double eps, const colatus_batch *batch, Boxes &b)
{
    if (!batch) {
        if (!is_fin(eps) || eps < 0.0)
            return COLATUS_EINVAL;
        b.off = {0, N};
        b.eps = {eps};
        b.max_n = N;
        return COLATUS_OK;
    }
    if (batch->n_boxes < 1 || !batch->box_offsets || !batch->eps)
        return COLATUS_EINVAL;
    b.off.assign(batch->box_offsets, batch->box_offsets + batch->n_boxes + 1);
    b.eps.assign(batch->eps, batch->eps + batch->n_boxes);
    if (b.off[0] != 0 || b.off.back() != N)
        return COLATUS_EINVAL;
    for (int i = 0; i < batch->n_boxes; ++i) {
        if (b.off[i + 1] <= b.off[i])
            return COLATUS_EINVAL;
        if (!is_fin(b.eps[i]) || b.eps[i] < 0.0)
            return COLATUS_EINVAL;
        b.max_n = std::max(b.max_n, b.off[i + 1] - b.off[i]);
    }
    return COLATUS_OK;
}

bool valid_precision(int p) { return p >= COLATUS_FP64 && p <= COLATUS_FP32; }

// a^4 H^2 / H0^2 = Om_R + Om_M a + Om_K a^2 + Om_L a^4 must stay > 0 on
// [lo, hi].  Checked at 4096 points and at the critical points of the
// quartic located by bisection between sign changes of its derivative.
bool friedmann_positive(double OmR, double OmM, double OmK, double OmL, double lo, double hi)
{
    auto f = [&](double a) { return OmR + a * (OmM + a * (OmK + a * a * OmL)); };
    auto df = [&](double a) { return OmM + a * (2.0 * OmK + 4.0 * OmL * a * a); };
    const int n = 4096;
    double prev_a = lo, prev_d = df(lo);
    if (!(f(lo) > 0.0) || !(f(hi) > 0.0))
        return false;
    for (int i = 1; i <= n; ++i) {
        const double a = lo + (hi - lo) * i / n;
        if (!(f(a) > 0.0))
            return false;
        const double d = df(a);
        if ((prev_d < 0.0) != (d < 0.0)) {
            double l = prev_a, r = a;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (l + r);
                if ((df(mid) < 0.0) == (prev_d < 0.0))
                    l = mid;
                else
                    r = mid;
            }
            if (!(f(0.5 * (l + r)) > 0.0))
                return false;
        }
        prev_a = a;
        prev_d = d;
    }
    return true;
}

int validate_cosmology(double H0, double OmR, double OmM, double OmK, double OmL,
                       double a_begin, double a_end)
{
    if (!is_fin(H0) || H0 < 0.0 || !is_fin(OmR) || !is_fin(OmM) || !is_fin(OmK) || !is_fin(OmL))
        return COLATUS_EINVAL;
    if (!is_fin(a_begin) || !is_fin(a_end) || a_begin <= 0.0 || a_end <= 0.0)
        return COLATUS_EINVAL;
    if (H0 == 0.0)
        return COLATUS_OK;
    if (a_begin == a_end)
        return COLATUS_EINVAL;
    const double lo = std::min(a_begin, a_end), hi = std::max(a_begin, a_end);
    if (!friedmann_positive(OmR, OmM, OmK, OmL, lo, hi))
        return COLATUS_EFRIEDMANN;
    return COLATUS_OK;
}

// ---------------------------------------------------------------------------
// Device scratch, one workspace per (device, stream).
// ---------------------------------------------------------------------------
struct Buffer {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct WorkList {
    // key
    int64_t N = -1;
    std::vector<int64_t> off;
    std::vector<double> eps;
    TileCfg cfg{0, 0, 0, 0};
    // content
    std::vector<WorkItem> items;
    std::vector<IntBlock> blocks;
    std::vector<int32_t> box_first_block;
    int max_slices = 0;
    Buffer d_items, d_blocks, d_box_first, d_off;
    uint64_t used = 0;  // last use (workspace clock), for eviction
    bool matches(const std::vector<int64_t> &o, const std::vector<double> &e, int64_t n,
                 const TileCfg &c) const
    {
        return N == n && off == o && eps == e && cfg.R == c.R && cfg.tpb == c.tpb &&
               cfg.slices == c.slices && cfg.form == c.form && cfg.group == c.group;
    }
};

// A captured run step graph: kStepsPerGraph iterations of (integrate, pair
// sweep), valid for exactly the kernel arguments and launch shapes in `key`
// (pointers, sizes, scalars, tile shape).  Everything that changes from call
// to call without changing those (the step range, the coefficients, the work
// items' contents) is read from device memory, so a key match means the
// graph launches the same kernels with the same arguments an eager loop would.
struct StepGraph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};

// Work lists and step graphs kept per workspace (least recently used evicted).
constexpr size_t kMaxWorkLists = 1024;
constexpr size_t kMaxStepGraphs = 8;
constexpr int64_t kStepsPerGraph = 16;
// A call captures a new step graph only when it is this long: measured on
// gfx950, replaying the captured steps runs no faster than launching them
// (0.2289 against 0.2285 ms per 32^3 step, 0.0452 against 0.0457 ms at 16^3),
// while capturing and instantiating one costs about 4 ms of host time.
constexpr int64_t kGraphCaptureSteps = 256;

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    Buffer part, part_phi, coef, p, diag_part, diag_out, counters, lam_x, lam_p, ckpt, seg,
        box_mass, att_acc, he_x, track_idx, track_slot, twiddle, ftle_idx;
    // periodic boundaries: the reciprocal-space plan (vectors and weights for
    // one box side and precision) and its work buffers
    Buffer ew_segs, ew_segs_sk, ew_coef, ew_skp, ew_S, ew_kpg, ew_kpp, ew_msum, ew_g, ew_p;
    double ew_L = 0.0, ew_alpha = 0.0;
    int ew_nmax = -1, ew_nsegs = 0, ew_K = 0;
    // work lists by (N, boxes, softenings, tile shape); fwd / adj: the lists
    // selected by the current call's forward and adjoint set-up
    std::vector<WorkList *> lists;
    WorkList *fwd = nullptr, *adj = nullptr;
    std::vector<StepGraph> graphs;
    uint64_t clock = 0;
    std::vector<int64_t> track_host;  // tracer list being uploaded
    hipEvent_t track_ev = nullptr;    // recorded after its upload
    std::vector<int64_t> ftle_host;   // FTLE tracer list being uploaded
    hipEvent_t ftle_ev = nullptr;     // recorded after its upload
    // every device allocation the workspace owns, work lists aside
    std::vector<Buffer *> buffers()
    {
        return {&part,     &part_phi,   &coef,  &p,        &diag_part,  &diag_out,
                &counters, &lam_x,      &lam_p, &ckpt,     &seg,        &box_mass,
                &att_acc,  &he_x,       &track_idx, &track_slot, &twiddle, &ftle_idx,
                &ew_segs,  &ew_segs_sk, &ew_coef, &ew_skp, &ew_S, &ew_kpg, &ew_kpp, &ew_msum,
                &ew_g,     &ew_p};
    }
};

void free_worklist_buffers(WorkList &wl)
{
    for (Buffer *bb : {&wl.d_items, &wl.d_blocks, &wl.d_box_first, &wl.d_off})
        if (bb->ptr) {
            (void)hipFree(bb->ptr);
            bb->ptr = nullptr;
            bb->cap = 0;
        }
}

std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

int hip_err(hipError_t e)
{
    if (e == hipSuccess)
        return COLATUS_OK;
    if (e == hipErrorOutOfMemory)
        return COLATUS_ENOMEM;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice)
        return COLATUS_ENODEV;
    return COLATUS_EHIP;
}

#define CHECK_HIP(expr)                                                                       \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            return hip_err(_e);                                                               \
    } while (0)

#define CHECK_RC(expr)                                                                        \
    do {                                                                                      \
        int _rc = (expr);                                                                     \
        if (_rc != COLATUS_OK)                                                                \
            return _rc;                                                                       \
    } while (0)

int ensure(Buffer &b, size_t bytes)
{
    if (bytes == 0)
        bytes = 256;
    if (b.cap >= bytes)
        return COLATUS_OK;
    if (b.ptr) {
        CHECK_HIP(hipDeviceSynchronize());
        CHECK_HIP(hipFree(b.ptr));
        b.ptr = nullptr;
        b.cap = 0;
    }
    const size_t rounded = (bytes + 4095) & ~(size_t)4095;
    CHECK_HIP(hipMalloc(&b.ptr, rounded));
    b.cap = rounded;
    return COLATUS_OK;
}

// Tracer tracks: validated host index list and the caller's device output.
constexpr int32_t kMaxTracers = 65536;
constexpr int64_t kMaxSpectrumRows = (int64_t)1 << 17;

struct Tracks {
    int32_t n = 0;
    const int64_t *index = nullptr;
    double *out = nullptr;
};

int resolve_tracks(const colatus_tracks *t, int64_t N, Tracks &out)
{
    out = Tracks{};
    if (!t)
        return COLATUS_OK;
    if (t->n_tracers < 1 || t->n_tracers > kMaxTracers || !t->index || !t->out)
        return COLATUS_EINVAL;
    std::vector<int64_t> idx(t->index, t->index + t->n_tracers);
    std::sort(idx.begin(), idx.end());
    if (idx.front() < 0 || idx.back() >= N)
        return COLATUS_EINVAL;
    for (size_t k = 1; k < idx.size(); ++k)
        if (idx[k] == idx[k - 1])
            return COLATUS_EINVAL;
    out.n = t->n_tracers;
    out.index = t->index;
    out.out = t->out;
    return COLATUS_OK;
}

int device_ready(int &dev)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return COLATUS_ENODEV;
    if (hipGetDevice(&dev) != hipSuccess)
        return COLATUS_ENODEV;
    return COLATUS_OK;
}

int get_workspace(hipStream_t stream, Workspace *&ws)
{
    int dev = 0;
    CHECK_RC(device_ready(dev));
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        ws = it->second;
        return COLATUS_OK;
    }
    // registered only once its counters exist, so that a failed set-up is
    // retried by the next call instead of leaving a workspace without them
    Workspace *fresh = new Workspace();
    fresh->device = dev;
    fresh->stream = stream;
    // counters: [0] work-item counter (int), [64..88) run descriptor
    // {n, first, last} (int64), [128] completion counter (int)
    int rc = ensure(fresh->counters, 256);
    if (rc == COLATUS_OK)
        rc = hip_err(launch_zero_counter(static_cast<int *>(fresh->counters.ptr), stream));
    if (rc != COLATUS_OK) {
        if (fresh->counters.ptr)
            (void)hipFree(fresh->counters.ptr);
        delete fresh;
        return rc;
    }
    g_ws[key] = fresh;
    ws = fresh;
    return COLATUS_OK;
}

int *work_counter(Workspace *ws) { return static_cast<int *>(ws->counters.ptr); }
int *done_counter(Workspace *ws)
{
    return reinterpret_cast<int *>(static_cast<char *>(ws->counters.ptr) + 128);
}
int64_t *step_counter(Workspace *ws)
{
    return reinterpret_cast<int64_t *>(static_cast<char *>(ws->counters.ptr) + 64);
}

// The run descriptor {n, first, last} (see IntegrateArgs::step) and the
// sweep counters, written by a kernel (graph-safe; no memset node).
__global__ void set_step_kernel(int64_t *step, int64_t value, int64_t first, int64_t last,
                                int *counter, int *done)
{
    step[0] = value;
    step[1] = first;
    step[2] = last;
    *counter = 0;
    *done = 0;
}

int set_step(Workspace *ws, int64_t value, int64_t first, int64_t last, hipStream_t s)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(1), 0, s, step_counter(ws), value, first,
                       last, work_counter(ws), done_counter(ws));
    CHECK_HIP(hipGetLastError());
    return COLATUS_OK;
}

// ---------------------------------------------------------------------------
// Tile shapes.
// ---------------------------------------------------------------------------
struct TuneKey {
    int64_t nbucket;
    int nboxes_bucket;
    int precision;
    int kind;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(nbucket, nboxes_bucket, precision, kind) <
               std::tie(o.nbucket, o.nboxes_bucket, o.precision, o.kind);
    }
};
std::map<TuneKey, TileCfg> g_tuned;

int64_t pow2_ceil(int64_t n)
{
    int64_t p = 1;
    while (p < n)
        p <<= 1;
    return p;
}

int cu_count(int dev)
{
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        n = 256;
    return n;
}

int n_target_blocks(const Boxes &b, int ti)
{
    int64_t t = 0;
    for (size_t i = 0; i + 1 < b.off.size(); ++i)
        t += (b.off[i + 1] - b.off[i] + ti - 1) / ti;
    return (int)t;
}

// Ordered forms (0, 1): enough (target block, source slice) items to give
// every CU several resident workgroups, with at least two source tiles per
// slice so the LDS staging stays amortised.
TileCfg ordered_cfg(const Boxes &b, int precision, int kind, int n_cu)
{
    TileCfg c;
    int per_cu = 8;
    if (kind == 0) {
        if (precision == COLATUS_FP64) {
            c.R = 2;
            c.tpb = 256;
            per_cu = 16;
        } else {
            // one target per lane and many small items measured fastest with
            // the one-shot grid (32^3: 128 target blocks x 64 slices)
            c.R = 1;
            c.tpb = 256;
            per_cu = 32;
        }
    } else {
        c.R = 1;
        c.tpb = 256;
    }
    const int tb = n_target_blocks(b, c.R * c.tpb);
    const int want = per_cu * n_cu;
    int s = (want + tb - 1) / tb;
    const int64_t max_s = std::max<int64_t>(1, b.max_n / (2 * c.tpb));
    s = (int)std::max<int64_t>(1, std::min<int64_t>(s, max_s));
    c.slices = s;
    c.form = 0;
    return c;
}

TileCfg symmetric_cfg(const Boxes &b, int R, int tpb);

// Largest box for the symmetric form: its partial-sum buffer holds one slot
// per part of 256 particles, ceil(n / 256) x n x 12 bytes with FP32 pairs
// (24 with FP64): 3.2 GB (6.4 GB) at 2^18.  Larger boxes use the ordered
// form, whose slot count stays near 64.
constexpr int64_t kSymMaxN = 262144;

// Cotangents up to which the adjoint uses the symmetric form (one launch per
// cotangent); more share the geometry in the ordered form's chunks of 8.
constexpr int kSymMaxCot = 3;

// The forward symmetric form in 2x2 groups of part pairs (four waves per
// workgroup), when COLATUS_OPT_PAIR_GROUP allows it.
TileCfg grouped_cfg(const Boxes &b)
{
    TileCfg c = symmetric_cfg(b, 4, 64);
    c.group = g_opt.pair_group != 0 ? 1 : 0;
    return c;
}

// Waves of a symmetric sweep over the boxes (parts of 256: the pairs of
// parts, and four 64-target pieces per diagonal part).
int64_t symmetric_waves(const Boxes &b)
{
    int64_t w = 0;
    for (size_t k = 0; k + 1 < b.off.size(); ++k) {
        const int64_t P = (b.off[k + 1] - b.off[k] + 255) / 256;
        w += P * (P - 1) / 2 + 4 * P;
    }
    return w;
}

// Sweeps whose symmetric items would give fewer waves than this in all
// leave most of the GPU idle (one wave per CU at 16^3); they take the
// ordered loop with one target per lane and one source tile per slice
// (small_boxes_cfg).  Measured per step of a run: the forward 2.8x faster
// in both precisions at 16^3 (4096 particles, 200 symmetric waves) and
// 1.37x (1.19x in FP64) at 20^3 (8000, 656 waves); an adjoint step (its
// forward and adjoint sweeps) 1.6x at 16^3 and 1.2x (1.06x) at 20^3; both
// slower from 24^3 (13824, 1701 waves).
constexpr int64_t kSmallSymWaves = 1024;

TileCfg small_boxes_cfg(const Boxes &b, int kind)
{
    // the adjoint's ordered loop runs 256 threads per block
    const int tpb = kind == 0 && b.max_n <= 6144 ? 128 : 256;
    return TileCfg{1, tpb, (int)std::max<int64_t>(1, (b.max_n + tpb - 1) / tpb), 0};
}

// Built-in heuristic: forward sweeps use the symmetric form (each unordered
// pair once, one wave per item, four targets per lane), measured at 32^3
// 1.36x (FP32 pairs) and 1.41x (FP64) faster than the ordered form, in 2x2
// groups of part pairs that halve the slots per particle; the adjoint with
// few cotangents uses the single-item symmetric form (1.27x and 1.84x);
// both unless the boxes are too small to fill the GPU with its items.
TileCfg heuristic_cfg(const Boxes &b, int precision, int kind, int n_cu, int n_cot = 1)
{
    if (symmetric_waves(b) < kSmallSymWaves)
        return small_boxes_cfg(b, kind);
    if (b.max_n <= kSymMaxN && kind == 0)
        return grouped_cfg(b);
    if (b.max_n <= kSymMaxN && n_cot <= kSymMaxCot)
        return symmetric_cfg(b, 4, 64);
    return ordered_cfg(b, precision, kind, n_cu);
}

// Number of source slices giving about `per_cu` work items per CU.
int slices_for(const Boxes &b, int R, int tpb, int per_cu, int n_cu)
{
    const int tb = n_target_blocks(b, R * tpb);
    const int s = (per_cu * n_cu + tb - 1) / tb;
    const int64_t max_s = std::max<int64_t>(1, b.max_n / (2 * tpb));
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, max_s));
}

// Symmetric form (form 2): R targets per lane, tpb threads, parts of R * tpb.
TileCfg symmetric_cfg(const Boxes &b, int R, int tpb)
{
    TileCfg c{R, tpb, 1, 2};
    const int64_t U = (int64_t)R * tpb;
    c.slices = (int)std::max<int64_t>(1, (b.max_n + U - 1) / U);
    return c;
}

TileCfg apply_overrides(TileCfg c, int kind, int precision, const Boxes &b, int n_cu)
{
    // the adjoint and FP64 have one ordered loop: form 1 means form 0 there
    int want = (int)g_opt.pair_form;
    if (want == 1 && (kind == 1 || precision == COLATUS_FP64))
        want = 0;
    if (want >= 0 && want != c.form) {
        if (want == 2) {
            c = kind == 0 ? grouped_cfg(b) : symmetric_cfg(b, 4, 64);
        } else {
            if (c.form == 2)
                c = ordered_cfg(b, precision, kind, n_cu);
            c.form = want;
        }
    }
    if (g_opt.tile_r > 0 && kind == 0)
        c.R = (int)g_opt.tile_r;
    if (g_opt.tile_tpb > 0 && kind == 0)
        c.tpb = (int)g_opt.tile_tpb;
    if (c.form == 2)
        c.slices = symmetric_cfg(b, c.R, c.tpb).slices;
    else if (g_opt.tile_slices > 0)
        c.slices = (int)g_opt.tile_slices;
    // groups: the forward symmetric form with 4 targets per lane and 64
    // threads only, and not when the option turns them off
    if (kind != 0 || c.form != 2 || c.R != 4 || c.tpb != 64)
        c.group = 0;
    else if (g_opt.pair_group == 0)
        c.group = 0;
    return c;
}

bool cfg_supported(const TileCfg &c, int kind, int precision)
{
    const bool fp64 = precision == COLATUS_FP64;
    if (c.group)
        return kind == 0 && c.form == 2 && c.R == 4 && c.tpb == 64;
    if (kind == 0 && c.form == 2 && fp64)
        return (c.R == 4 && c.tpb == 64) || (c.R == 2 && c.tpb == 128);
    if (kind == 0 && c.form == 2)
        return ((c.R == 4 || c.R == 8) && c.tpb == 64) || (c.R == 4 && c.tpb == 128);
    if (kind == 1 && c.form == 2)
        return c.R == 4 && c.tpb == 64;
    if (kind == 0)
        return (c.R == 1 || c.R == 2 || c.R == 4) && (c.tpb == 128 || c.tpb == 256) &&
               c.slices >= 1 && (c.form == 0 || c.form == 1);
    return (c.R == 1 || c.R == 2) && c.tpb == 256 && c.slices >= 1;
}

// ---------------------------------------------------------------------------
// Work lists.
// ---------------------------------------------------------------------------
// Symmetric items (form 2): every box is cut into parts of U = R * tpb
// particles.  Kind 0 item (p, q), p < q, pairs part p (targets, slot q) with
// part q (sources, reaction in slot p); the diagonal (p, p) is cut into
// pieces of tpb targets (one per lane) against the whole part (slot p).
// Every particle of a box with P parts gets exactly P slots.  The pieces are
// a quarter of a pair's work (or less): sorted last, they fill the final
// round of workgroups that equal-sized pairs would leave half empty.
void build_symmetric_items(const Boxes &b, const TileCfg &cfg, WorkList &wl)
{
    const int64_t U = (int64_t)cfg.R * cfg.tpb;
    const int nb = (int)b.eps.size();
    for (int box = 0; box < nb; ++box) {
        const int64_t o0 = b.off[box], o1 = b.off[box + 1];
        const int64_t P = (o1 - o0 + U - 1) / U;
        wl.max_slices = std::max<int>(wl.max_slices, (int)P);
        const double eps2 = b.eps[box] * b.eps[box];
        for (int64_t p = 0; p < P; ++p) {
            const int64_t p0 = o0 + p * U, p1 = std::min(o0 + (p + 1) * U, o1);
            for (int64_t q = p + 1; q < P; ++q) {
                WorkItem w{};
                w.i0 = p0;
                w.i1 = p1;
                w.j0 = o0 + q * U;
                w.j1 = std::min(o0 + (q + 1) * U, o1);
                w.eps2 = eps2;
                w.slice = (int32_t)q;
                w.rslice = (int32_t)p;
                w.box = box;
                w.kind = 0;
                wl.items.push_back(w);
            }
            for (int64_t t0 = p0; t0 < p1; t0 += cfg.tpb) {
                WorkItem w{};
                w.i0 = t0;
                w.i1 = std::min<int64_t>(t0 + cfg.tpb, p1);
                w.j0 = p0;
                w.j1 = p1;
                w.eps2 = eps2;
                w.slice = (int32_t)p;
                w.rslice = (int32_t)p;
                w.box = box;
                w.kind = 1;
                wl.items.push_back(w);
            }
        }
        wl.box_first_block.push_back((int32_t)wl.blocks.size());
        for (int64_t i0 = o0; i0 < o1; i0 += kIntBlock) {
            IntBlock ib;
            ib.i0 = i0;
            ib.i1 = std::min<int64_t>(i0 + kIntBlock, o1);
            ib.eps = b.eps[box];
            ib.box = box;
            ib.n_slices = (int32_t)P;
            wl.blocks.push_back(ib);
        }
    }
    wl.box_first_block.push_back((int32_t)wl.blocks.size());
    // largest first: every lane of a workgroup runs, missing targets
    // included, so a pair costs (R * tpb target slots) x (sources), plus
    // about a third for the reaction; a piece costs tpb x (sources)
    const int64_t slots = U;
    auto cost = [slots, &cfg](const WorkItem &w) {
        const int64_t ns = w.j1 - w.j0;
        return w.kind == 0 ? 4 * slots * ns / 3 : (int64_t)cfg.tpb * ns;
    };
    std::stable_sort(wl.items.begin(), wl.items.end(),
                     [&cost](const WorkItem &a, const WorkItem &c) { return cost(a) > cost(c); });
}

// Grouped symmetric items (form 2, parts of 256, four waves per group).
// Parts pair up into super-parts {2A, 2A+1} (the last alone when P is odd).
// For super-parts A < B the group holds the 2x2 block of items (2A + a,
// 2B + b) in wave 2a + b: targets in slot B, reactions in slot A; the two
// waves with the same target part (or source part) add their partial sums
// before the one write (tmate, rmate).  The pairs inside super-parts
// (2A, 2A+1: slot A on both sides) and the diagonal pieces (slot
// ceil(P/2), or slot A for a part alone in its super-part) have no partner
// and are packed four to a group.  Every particle of a paired part gets
// ceil(P/2) + 1 slots, one of a lone part ceil(P/2), each written exactly
// once.  Groups are ordered by their longest item, largest first.
void build_symmetric_groups(const Boxes &b, const TileCfg &cfg, WorkList &wl)
{
    const int64_t U = (int64_t)cfg.R * cfg.tpb;
    const int nb = (int)b.eps.size();
    struct Group {
        WorkItem w[4];
        int64_t cost;
    };
    auto cost = [U, &cfg](const WorkItem &w) -> int64_t {
        if (w.kind < 0)
            return 0;
        const int64_t ns = w.j1 - w.j0;
        return w.kind == 0 ? 4 * U * ns / 3 : (int64_t)cfg.tpb * ns;
    };
    WorkItem pad{};
    pad.kind = -1;
    std::vector<Group> groups;
    std::vector<WorkItem> loose;
    for (int box = 0; box < nb; ++box) {
        const int64_t o0 = b.off[box], o1 = b.off[box + 1];
        const int64_t P = (o1 - o0 + U - 1) / U;
        const int64_t S2 = (P + 1) / 2;
        const double eps2 = b.eps[box] * b.eps[box];
        auto lo = [&](int64_t p) { return o0 + p * U; };
        auto hi = [&](int64_t p) { return std::min(o0 + (p + 1) * U, o1); };
        auto paired = [&](int64_t p) { return (p ^ 1) < P; };
        wl.max_slices = std::max<int>(wl.max_slices, (int)(P > 1 ? S2 + 1 : S2));
        for (int64_t A = 0; A < S2; ++A)
            for (int64_t B = A + 1; B < S2; ++B) {
                Group g;
                for (WorkItem &w : g.w)
                    w = pad;
                g.cost = 0;
                for (int a = 0; a < 2; ++a)
                    for (int bb = 0; bb < 2; ++bb) {
                        const int64_t p = 2 * A + a, q = 2 * B + bb;
                        if (p >= P || q >= P)
                            continue;
                        WorkItem &w = g.w[2 * a + bb];
                        w.i0 = lo(p);
                        w.i1 = hi(p);
                        w.j0 = lo(q);
                        w.j1 = hi(q);
                        w.eps2 = eps2;
                        w.slice = (int32_t)B;
                        w.rslice = (int32_t)A;
                        w.box = box;
                        w.kind = 0;
                        w.tmate = (int8_t)(2 * B + (1 - bb) < P);
                        w.rmate = (int8_t)(2 * A + (1 - a) < P);
                        g.cost = std::max(g.cost, cost(w));
                    }
                groups.push_back(g);
            }
        for (int64_t p = 0; p < P; ++p) {
            if ((p & 1) == 0 && paired(p)) {
                WorkItem w{};
                w.i0 = lo(p);
                w.i1 = hi(p);
                w.j0 = lo(p + 1);
                w.j1 = hi(p + 1);
                w.eps2 = eps2;
                w.slice = (int32_t)(p / 2);
                w.rslice = (int32_t)(p / 2);
                w.box = box;
                w.kind = 0;
                loose.push_back(w);
            }
            const int32_t dslot = (int32_t)(paired(p) ? S2 : p / 2);
            for (int64_t t0 = lo(p); t0 < hi(p); t0 += cfg.tpb) {
                WorkItem w{};
                w.i0 = t0;
                w.i1 = std::min<int64_t>(t0 + cfg.tpb, hi(p));
                w.j0 = lo(p);
                w.j1 = hi(p);
                w.eps2 = eps2;
                w.slice = dslot;
                w.rslice = dslot;
                w.box = box;
                w.kind = 1;
                loose.push_back(w);
            }
        }
        wl.box_first_block.push_back((int32_t)wl.blocks.size());
        for (int64_t i0 = o0; i0 < o1; i0 += kIntBlock) {
            const int64_t p = (i0 - o0) / U;
            IntBlock ib;
            ib.i0 = i0;
            ib.i1 = std::min<int64_t>(i0 + kIntBlock, o1);
            ib.eps = b.eps[box];
            ib.box = box;
            ib.n_slices = (int32_t)(paired(p) ? S2 + 1 : S2);
            wl.blocks.push_back(ib);
        }
    }
    wl.box_first_block.push_back((int32_t)wl.blocks.size());
    std::stable_sort(loose.begin(), loose.end(), [&cost](const WorkItem &a, const WorkItem &c) {
        return cost(a) > cost(c);
    });
    for (size_t k = 0; k < loose.size(); k += 4) {
        Group g;
        g.cost = 0;
        for (size_t e = 0; e < 4; ++e) {
            g.w[e] = k + e < loose.size() ? loose[k + e] : pad;
            g.cost = std::max(g.cost, cost(g.w[e]));
        }
        groups.push_back(g);
    }
    std::stable_sort(groups.begin(), groups.end(),
                     [](const Group &a, const Group &c) { return a.cost > c.cost; });
    wl.items.reserve(groups.size() * 4);
    for (const Group &g : groups)
        for (const WorkItem &w : g.w)
            wl.items.push_back(w);
}

void build_worklist(const Boxes &b, int64_t N, const TileCfg &cfg, WorkList &wl)
{
    wl.items.clear();
    wl.blocks.clear();
    wl.box_first_block.clear();
    wl.max_slices = 0;
    if (cfg.form == 2 && cfg.group) {
        build_symmetric_groups(b, cfg, wl);
        return;
    }
    if (cfg.form == 2) {
        build_symmetric_items(b, cfg, wl);
        return;
    }
    const int ti = cfg.R * cfg.tpb;
    const int nb = (int)b.eps.size();
    for (int box = 0; box < nb; ++box) {
        const int64_t o0 = b.off[box], o1 = b.off[box + 1], nbx = o1 - o0;
        const int64_t tiles = (nbx + cfg.tpb - 1) / cfg.tpb;
        int64_t s = std::min<int64_t>(cfg.slices, tiles);
        const int64_t tiles_per_slice = (tiles + s - 1) / s;
        const int64_t js = tiles_per_slice * cfg.tpb;
        s = (nbx + js - 1) / js;
        wl.max_slices = std::max<int>(wl.max_slices, (int)s);
        const double eps2 = b.eps[box] * b.eps[box];
        for (int64_t i0 = o0; i0 < o1; i0 += ti) {
            const int64_t i1 = std::min(i0 + ti, o1);
            for (int64_t q = 0; q < s; ++q) {
                WorkItem w{};
                w.i0 = i0;
                w.i1 = i1;
                w.j0 = o0 + q * js;
                w.j1 = std::min(o0 + (q + 1) * js, o1);
                w.eps2 = eps2;
                w.slice = (int32_t)q;
                w.box = box;
                wl.items.push_back(w);
            }
        }
        wl.box_first_block.push_back((int32_t)wl.blocks.size());
        for (int64_t i0 = o0; i0 < o1; i0 += kIntBlock) {
            IntBlock ib;
            ib.i0 = i0;
            ib.i1 = std::min<int64_t>(i0 + kIntBlock, o1);
            ib.eps = b.eps[box];
            ib.box = box;
            ib.n_slices = (int32_t)s;
            wl.blocks.push_back(ib);
        }
    }
    wl.box_first_block.push_back((int32_t)wl.blocks.size());
    // Longest-processing-time-first order for the persistent grid: an item's
    // cost is its source count (every lane of the block runs).
    std::stable_sort(wl.items.begin(), wl.items.end(), [](const WorkItem &a, const WorkItem &c) {
        return (a.j1 - a.j0) > (c.j1 - c.j0);
    });
}

// Build the list for (b, N, cfg) and upload it into wl's device buffers.
// wl must hold no list that queued work may still read (a fresh list, or a
// temporary one after a synchronisation).  The host vectors stay with the
// list, so the asynchronous uploads never read freed or changed memory.
int upload_worklist(WorkList &wl, const Boxes &b, int64_t N, const TileCfg &cfg, hipStream_t s)
{
    // the key is recorded last: a list whose upload failed is rebuilt
    wl.N = -1;
    build_worklist(b, N, cfg, wl);
    CHECK_RC(ensure(wl.d_items, wl.items.size() * sizeof(WorkItem)));
    CHECK_RC(ensure(wl.d_blocks, wl.blocks.size() * sizeof(IntBlock)));
    CHECK_RC(ensure(wl.d_box_first, wl.box_first_block.size() * sizeof(int32_t)));
    CHECK_RC(ensure(wl.d_off, b.off.size() * sizeof(int64_t)));
    CHECK_HIP(hipMemcpyAsync(wl.d_items.ptr, wl.items.data(), wl.items.size() * sizeof(WorkItem),
                             hipMemcpyHostToDevice, s));
    CHECK_HIP(hipMemcpyAsync(wl.d_blocks.ptr, wl.blocks.data(),
                             wl.blocks.size() * sizeof(IntBlock), hipMemcpyHostToDevice, s));
    CHECK_HIP(hipMemcpyAsync(wl.d_box_first.ptr, wl.box_first_block.data(),
                             wl.box_first_block.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             s));
    wl.off = b.off;
    CHECK_HIP(hipMemcpyAsync(wl.d_off.ptr, wl.off.data(), wl.off.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    wl.N = N;
    wl.eps = b.eps;
    wl.cfg = cfg;
    return COLATUS_OK;
}

// The workspace's list for (b, N, cfg): a cached one if it exists, else a
// new one (no synchronisation: the lists in use keep their buffers).  When
// the cache is full the least recently used list, other than the ones the
// current call has selected, is freed after the stream's queued work.
int select_worklist(Workspace *ws, const Boxes &b, int64_t N, const TileCfg &cfg, hipStream_t s,
                    WorkList *&out)
{
    const uint64_t now = ++ws->clock;
    for (WorkList *wl : ws->lists)
        if (wl->matches(b.off, b.eps, N, cfg)) {
            wl->used = now;
            out = wl;
            return COLATUS_OK;
        }
    if (ws->lists.size() >= kMaxWorkLists) {
        size_t victim = ws->lists.size();
        for (size_t k = 0; k < ws->lists.size(); ++k) {
            WorkList *wl = ws->lists[k];
            if (wl == ws->fwd || wl == ws->adj)
                continue;
            if (victim == ws->lists.size() || wl->used < ws->lists[victim]->used)
                victim = k;
        }
        if (victim < ws->lists.size()) {
            CHECK_HIP(hipStreamSynchronize(s));
            free_worklist_buffers(*ws->lists[victim]);
            delete ws->lists[victim];
            ws->lists.erase(ws->lists.begin() + (std::ptrdiff_t)victim);
        }
    }
    WorkList *wl = new WorkList();
    const int rc = upload_worklist(*wl, b, N, cfg, s);
    if (rc != COLATUS_OK) {
        // nothing was queued that reads the buffers unless an upload was
        (void)hipStreamSynchronize(s);
        free_worklist_buffers(*wl);
        delete wl;
        return rc;
    }
    wl->used = now;
    ws->lists.push_back(wl);
    out = wl;
    return COLATUS_OK;
}

// ---------------------------------------------------------------------------
// Pair-sweep timers (hipEvents around each launch on its stream).
// ---------------------------------------------------------------------------
struct TimerRec {
    hipEvent_t start, stop;
};
std::vector<TimerRec> g_timer[3];  // forward sweep, adjoint sweep, integrator
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Integrator launch, bracketed by hipEvents when the timer is enabled.
int run_integrate(const IntegrateArgs &A, hipStream_t s)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_opt.timer) {
        e0 = take_event();
        e1 = take_event();
    }
    if (e0)
        CHECK_HIP(hipEventRecord(e0, s));
    CHECK_HIP(launch_integrate(A, s));
    if (e1) {
        CHECK_HIP(hipEventRecord(e1, s));
        g_timer[2].push_back({e0, e1});
    }
    return COLATUS_OK;
}

// Forward pair sweep on the workspace's buffers, with the timer if enabled.
int run_forward_sweep(Workspace *ws, const WorkList &wl, int precision, bool phi,
                      bool mask, const double *x, const double *m, int64_t N, hipStream_t s,
                      bool zero_counter, int64_t *step_inc = nullptr)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_opt.timer) {
        e0 = take_event();
        e1 = take_event();
    }
    if (zero_counter && g_opt.persistent)
        CHECK_HIP(launch_zero_counter(work_counter(ws), s));
    if (e0)
        CHECK_HIP(hipEventRecord(e0, s));
    CHECK_HIP(launch_pair_sweep(precision, wl.cfg.form, wl.cfg, phi, mask, x, m, N,
                                static_cast<const WorkItem *>(wl.d_items.ptr),
                                (int)wl.items.size(), work_counter(ws), g_opt.persistent != 0,
                                static_cast<const double *>(ws->box_mass.ptr),
                                static_cast<double *>(ws->part.ptr),
                                phi ? static_cast<double *>(ws->part_phi.ptr) : nullptr,
                                step_inc, s));
    if (e1) {
        CHECK_HIP(hipEventRecord(e1, s));
        g_timer[0].push_back({e0, e1});
    }
    return COLATUS_OK;
}

int run_adjoint_sweep(Workspace *ws, const WorkList &wl, int precision, bool mask,
                      const double *x, const double *m, int64_t N, int n_cot,
                      const double *lam, hipStream_t s)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_opt.timer) {
        e0 = take_event();
        e1 = take_event();
    }
    if (g_opt.persistent)
        CHECK_HIP(launch_zero_counter(work_counter(ws), s));
    if (e0)
        CHECK_HIP(hipEventRecord(e0, s));
    CHECK_HIP(launch_adjoint_sweep(precision, wl.cfg, mask, x, m, N, n_cot, lam,
                                   static_cast<const WorkItem *>(wl.d_items.ptr),
                                   (int)wl.items.size(), work_counter(ws),
                                   g_opt.persistent != 0,
                                   static_cast<const double *>(ws->box_mass.ptr),
                                   static_cast<double *>(ws->part.ptr), s));
    if (e1) {
        CHECK_HIP(hipEventRecord(e1, s));
        g_timer[1].push_back({e0, e1});
    }
    return COLATUS_OK;
}

int prepare_box_mass(Workspace *ws, const WorkList &wl, const double *m, hipStream_t s);

// How the readers add the slots of this list's sweeps (SlotMode).
int slot_mode_of(const WorkList &wl, int precision) { return slot_mode_for(wl.cfg, precision); }

// Choose (and if asked, autotune) the tile shape, then make the work list.
int prepare_worklist(Workspace *ws, int kind, const Boxes &b, int64_t N, int precision,
                     const double *x, const double *m, int n_cot, hipStream_t s)
{
    const int n_cu = cu_count(ws->device);
    TuneKey key{pow2_ceil(b.max_n), (int)std::min<size_t>(pow2_ceil(b.eps.size()), 1 << 20),
                precision, kind};
    TileCfg cfg;
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
        cfg = it->second;
    } else {
        cfg = heuristic_cfg(b, precision, kind, n_cu, n_cot);
        if (g_opt.autotune && x && m) {
            // time candidates on the live data; scratch outputs only
            std::vector<TileCfg> cand;
            if (kind == 0) {
                const bool fp32 = precision != COLATUS_FP64;
                if (b.max_n <= kSymMaxN) {
                    if (g_opt.pair_group != 0)
                        cand.push_back(grouped_cfg(b));
                    cand.push_back(small_boxes_cfg(b, 0));
                    if (fp32)
                        for (auto rt : {std::make_pair(4, 64), std::make_pair(8, 64),
                                        std::make_pair(4, 128)})
                            cand.push_back(symmetric_cfg(b, rt.first, rt.second));
                    else
                        for (auto rt : {std::make_pair(4, 64), std::make_pair(2, 128)})
                            cand.push_back(symmetric_cfg(b, rt.first, rt.second));
                }
                for (int form : {0, 1}) {
                    if (form == 1 && !fp32)
                        continue;
                    for (int r : {1, 2, 4})
                        for (int t : {128, 256})
                            for (int per_cu : {4, 8, 16}) {
                                TileCfg c{r, t, slices_for(b, r, t, per_cu, n_cu), form};
                                cand.push_back(c);
                            }
                }
            } else {
                if (b.max_n <= kSymMaxN && n_cot <= kSymMaxCot)
                    cand.push_back(symmetric_cfg(b, 4, 64));
                for (int r : {1, 2})
                    for (int per_cu : {4, 8, 16}) {
                        TileCfg c{r, 256, slices_for(b, r, 256, per_cu, n_cu), 0};
                        cand.push_back(c);
                    }
            }
            hipEvent_t e0 = take_event(), e1 = take_event();
            float best = 1e30f;
            for (const TileCfg &c : cand) {
                WorkList tmp;
                CHECK_RC(upload_worklist(tmp, b, N, c, s));
                CHECK_RC(prepare_box_mass(ws, tmp, m, s));
                const size_t need = (size_t)tmp.max_slices * 3 * (size_t)N * sizeof(double) *
                                    (kind == 0 ? 1 : (size_t)std::max(1, n_cot));
                CHECK_RC(ensure(ws->part, need));
                CHECK_RC(ensure(ws->part_phi, (size_t)tmp.max_slices * N * sizeof(double)));
                float ms_total = 0.0f;
                for (int rep = 0; rep < 4; ++rep) {
                    CHECK_HIP(launch_zero_counter(work_counter(ws), s));
                    CHECK_HIP(hipEventRecord(e0, s));
                    if (kind == 0)
                        CHECK_HIP(launch_pair_sweep(
                            precision, c.form, c, false, false, x, m, N,
                            static_cast<const WorkItem *>(tmp.d_items.ptr), (int)tmp.items.size(),
                            work_counter(ws), g_opt.persistent != 0,
                            static_cast<const double *>(ws->box_mass.ptr),
                            static_cast<double *>(ws->part.ptr), nullptr, nullptr, s));
                    else
                        CHECK_HIP(launch_adjoint_sweep(
                            precision, c, false, x, m, N, 1, x,
                            static_cast<const WorkItem *>(tmp.d_items.ptr), (int)tmp.items.size(),
                            work_counter(ws), g_opt.persistent != 0,
                            static_cast<const double *>(ws->box_mass.ptr),
                            static_cast<double *>(ws->part.ptr), s));
                    CHECK_HIP(hipEventRecord(e1, s));
                    CHECK_HIP(hipEventSynchronize(e1));
                    float ms = 0.0f;
                    CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (rep > 0)
                        ms_total += ms;
                }
                for (Buffer *bb : {&tmp.d_items, &tmp.d_blocks, &tmp.d_box_first, &tmp.d_off})
                    if (bb->ptr)
                        (void)hipFree(bb->ptr);
                if (ms_total < best) {
                    best = ms_total;
                    cfg = c;
                }
            }
            g_event_pool.push_back(e0);
            g_event_pool.push_back(e1);
            g_tuned[key] = cfg;
        }
    }
    cfg = apply_overrides(cfg, kind, precision, b, n_cu);
    if (!cfg_supported(cfg, kind, precision))
        return COLATUS_EINVAL;
    WorkList *wl = nullptr;
    CHECK_RC(select_worklist(ws, b, N, cfg, s, wl));
    (kind == 0 ? ws->fwd : ws->adj) = wl;
    return COLATUS_OK;
}

// Per-box common mass (NaN where the masses of a box differ), for the
// equal-mass form of the pair loop.  Queued on the stream; the masses are
// read as they are when this runs.
int prepare_box_mass(Workspace *ws, const WorkList &wl, const double *m, hipStream_t s)
{
    const int n_boxes = (int)wl.off.size() - 1;
    CHECK_RC(ensure(ws->box_mass, (size_t)n_boxes * sizeof(double)));
    CHECK_HIP(launch_box_mass(m, static_cast<const int64_t *>(wl.d_off.ptr), n_boxes,
                              wl.off.back(), static_cast<double *>(ws->box_mass.ptr), s));
    return COLATUS_OK;
}

int check_ptrs(std::initializer_list<const void *> ps)
{
    for (const void *p : ps)
        if (!p)
            return COLATUS_EINVAL;
    return COLATUS_OK;
}

// ---------------------------------------------------------------------------
// The run driver (shared by colatus_step and colatus_run).
// ---------------------------------------------------------------------------
struct RunParams {
    double *x, *v;
    const double *m;
    int64_t N;
    double G, H0, OmR, OmM, OmK, OmL, a_begin, a_end;
    int64_t n_steps, first, last;
    int precision;
    colatus_diag *diag;
    hipStream_t stream;
    ExtField ext;
    Tracks trk;
};

// Upload the tracer list, build the particle -> tracer map and write the
// start-state row of the track (x and v as given).
int prepare_tracks(Workspace *ws, const RunParams &P)
{
    if (P.trk.n == 0)
        return COLATUS_OK;
    hipStream_t s = P.stream;
    CHECK_RC(ensure(ws->track_idx, (size_t)P.trk.n * sizeof(int64_t)));
    CHECK_RC(ensure(ws->track_slot, (size_t)P.N * sizeof(int32_t)));
    const int64_t *didx = static_cast<const int64_t *>(ws->track_idx.ptr);
    // the caller's host list is copied into the workspace's own, which the
    // asynchronous upload reads; the previous upload from it must be done
    // before it is overwritten
    if (!ws->track_ev)
        CHECK_HIP(hipEventCreateWithFlags(&ws->track_ev, hipEventDisableTiming));
    else
        CHECK_HIP(hipEventSynchronize(ws->track_ev));
    ws->track_host.assign(P.trk.index, P.trk.index + P.trk.n);
    CHECK_HIP(hipMemcpyAsync(ws->track_idx.ptr, ws->track_host.data(),
                             (size_t)P.trk.n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    CHECK_HIP(hipEventRecord(ws->track_ev, s));
    CHECK_HIP(launch_track_slots(static_cast<int32_t *>(ws->track_slot.ptr), P.N, didx, P.trk.n,
                                 s));
    CHECK_HIP(launch_track_gather(P.x, P.v, P.N, didx, P.trk.n, P.trk.out, s));
    return COLATUS_OK;
}

// Flat key of every kernel argument and launch shape a captured step uses.
struct KeyBuilder {
    std::vector<uint64_t> v;
    void add(const void *p) { v.push_back((uint64_t)(uintptr_t)p); }
    void add(int64_t i) { v.push_back((uint64_t)i); }
    void add(double d)
    {
        uint64_t u;
        std::memcpy(&u, &d, sizeof u);
        v.push_back(u);
    }
};

std::vector<uint64_t> step_graph_key(const Workspace *ws, const RunParams &P,
                                     const IntegrateArgs &A, bool mask)
{
    const WorkList &wl = *ws->fwd;
    KeyBuilder k;
    // integrate_kernel
    k.add(A.x); k.add(A.p); k.add(A.m); k.add(A.part); k.add(A.part_phi); k.add(A.blocks);
    k.add((int64_t)A.n_blocks); k.add(A.N); k.add(A.G); k.add(A.coef); k.add(A.step);
    k.add(A.work_counter); k.add(A.diag_part); k.add((int64_t)A.precision); k.add(A.box_mass);
    k.add((int64_t)A.slot_mode);
    k.add((int64_t)A.ext.on); k.add(A.ext.S); k.add(A.ext.x); k.add(A.ext.y); k.add(A.ext.z);
    k.add((int64_t)A.ext.bg); k.add(A.ext.b); k.add(A.ext.cx); k.add(A.ext.cy); k.add(A.ext.cz);
    k.add(A.track_slot); k.add(A.track); k.add((int64_t)A.n_tracers);
    k.add(A.ewald_g); k.add(A.ewald_p); k.add(A.box);
    // pair sweep
    k.add((int64_t)P.precision); k.add((int64_t)wl.cfg.R); k.add((int64_t)wl.cfg.tpb);
    k.add((int64_t)wl.cfg.slices); k.add((int64_t)wl.cfg.form); k.add((int64_t)(P.diag != nullptr));
    k.add((int64_t)mask); k.add(P.x); k.add(P.m); k.add(P.N); k.add(wl.d_items.ptr);
    k.add((int64_t)wl.items.size()); k.add((int64_t)g_opt.persistent); k.add(ws->part.ptr);
    k.add(ws->part_phi.ptr); k.add(ws->counters.ptr);
    k.add(kStepsPerGraph);
    return k.v;
}

// Runs n_iter iterations of (integrate(n), pair sweep(x_{n+1})).  Calls of at
// least kGraphCaptureSteps steps capture kStepsPerGraph iterations in a graph,
// kept for later calls with the same arguments; a cached graph is replayed
// whenever the call is long enough for one.  Shorter calls, and the steps
// left over, are launched eagerly.  Nothing here waits for the device.
int enqueue_steps(Workspace *ws, const RunParams &P, const IntegrateArgs &base, bool mask,
                  int64_t n_iter)
{
    hipStream_t s = P.stream;
    const bool phi = P.diag != nullptr;
    auto body = [&](hipStream_t st) -> int {
        CHECK_RC(run_integrate(base, st));  // re-arms the work counter
        CHECK_RC(run_forward_sweep(ws, *ws->fwd, P.precision, phi, mask, P.x, P.m, P.N, st,
                                   false, step_counter(ws)));  // advances the step
        return COLATUS_OK;
    };
    StepGraph *g = nullptr;
    if (g_opt.graph && !g_opt.timer && n_iter >= kStepsPerGraph) {
        std::vector<uint64_t> key = step_graph_key(ws, P, base, mask);
        for (StepGraph &sg : ws->graphs)
            if (sg.key == key)
                g = &sg;
        if (!g && n_iter >= kGraphCaptureSteps) {
            if (!ws->cap_stream)
                CHECK_HIP(hipStreamCreateWithFlags(&ws->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            CHECK_HIP(hipStreamBeginCapture(ws->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = COLATUS_OK;
            for (int64_t k = 0; k < kStepsPerGraph && rc == COLATUS_OK; ++k)
                rc = body(ws->cap_stream);
            hipError_t ec = hipStreamEndCapture(ws->cap_stream, &graph);
            if (rc != COLATUS_OK) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return rc;
            }
            CHECK_HIP(ec);
            hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            CHECK_HIP(ei);
            if (ws->graphs.size() >= kMaxStepGraphs) {
                // the least recently used graph may still be queued: wait first
                size_t victim = 0;
                for (size_t k = 1; k < ws->graphs.size(); ++k)
                    if (ws->graphs[k].used < ws->graphs[victim].used)
                        victim = k;
                hipError_t es = hipStreamSynchronize(s);
                if (es != hipSuccess) {
                    (void)hipGraphExecDestroy(exec);
                    return hip_err(es);
                }
                (void)hipGraphExecDestroy(ws->graphs[victim].exec);
                ws->graphs.erase(ws->graphs.begin() + (std::ptrdiff_t)victim);
            }
            StepGraph fresh;
            fresh.key = std::move(key);
            fresh.exec = exec;
            ws->graphs.push_back(std::move(fresh));
            g = &ws->graphs.back();
        }
    }
    int64_t done = 0;
    if (g) {
        g->used = ++ws->clock;
        for (; done + kStepsPerGraph <= n_iter; done += kStepsPerGraph)
            CHECK_HIP(hipGraphLaunch(g->exec, s));
    }
    for (; done < n_iter; ++done) {
        TraceRange step("step");
        CHECK_RC(body(s));
    }
    return COLATUS_OK;
}

int run_impl(const RunParams &P, const Boxes &b)
{
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(P.stream, ws));
    hipStream_t s = P.stream;
    CHECK_RC(prepare_worklist(ws, 0, b, P.N, P.precision, P.x, P.m, 1, s));
    const WorkList &wl = *ws->fwd;
    CHECK_RC(prepare_box_mass(ws, wl, P.m, s));
    const int64_t nsteps = P.last - P.first;
    const int64_t rows = nsteps + 1;
    const int n_boxes = (int)b.eps.size();
    const size_t n3 = 3 * (size_t)P.N;
    CHECK_RC(ensure(ws->coef, (size_t)nsteps * sizeof(StepCoef)));
    CHECK_RC(ensure(ws->p, n3 * sizeof(double)));
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * n3 * sizeof(double)));
    const bool diag = P.diag != nullptr;
    if (diag) {
        CHECK_RC(ensure(ws->part_phi, (size_t)wl.max_slices * P.N * sizeof(double)));
        CHECK_RC(ensure(ws->diag_part, (size_t)rows * wl.blocks.size() * kDiagW * sizeof(double)));
        CHECK_RC(ensure(ws->diag_out, (size_t)n_boxes * rows * sizeof(colatus_diag)));
    }
    bool mask = false;
    for (double e : b.eps)
        mask = mask || e == 0.0;

    StepCoef *coef = static_cast<StepCoef *>(ws->coef.ptr);
    double *p = static_cast<double *>(ws->p.ptr);
    CHECK_HIP(launch_coefficients(P.H0, P.OmR, P.OmM, P.OmK, P.OmL, P.a_begin, P.a_end,
                                  P.n_steps, P.first, P.last, 0, coef, s));
    CHECK_HIP(launch_convert(0, P.v, p, P.N, coef, 0, s));
    CHECK_RC(set_step(ws, P.first, P.first, P.last, s));
    CHECK_RC(run_forward_sweep(ws, wl, P.precision, diag, mask, P.x, P.m, P.N, s, false));

    IntegrateArgs A;
    A.x = P.x;
    A.p = p;
    A.m = P.m;
    A.part = static_cast<const double *>(ws->part.ptr);
    A.part_phi = diag ? static_cast<const double *>(ws->part_phi.ptr) : nullptr;
    A.blocks = static_cast<const IntBlock *>(wl.d_blocks.ptr);
    A.n_blocks = (int)wl.blocks.size();
    A.N = P.N;
    A.G = P.G;
    A.coef = coef;
    A.step = step_counter(ws);
    A.work_counter = work_counter(ws);
    A.diag_part = diag ? static_cast<double *>(ws->diag_part.ptr) : nullptr;
    A.precision = P.precision;
    A.box_mass = static_cast<const double *>(ws->box_mass.ptr);
    A.slot_mode = slot_mode_of(wl, P.precision);
    A.ext = P.ext;
    CHECK_RC(prepare_tracks(ws, P));
    A.track_slot = P.trk.n ? static_cast<const int32_t *>(ws->track_slot.ptr) : nullptr;
    A.track = P.trk.out;
    A.n_tracers = P.trk.n;

    CHECK_RC(enqueue_steps(ws, P, A, mask, nsteps));
    CHECK_RC(run_integrate(A, s));  // closing half kick at a_last (+ diagnostics)
    CHECK_HIP(launch_convert(1, p, P.v, P.N, coef, nsteps - 1, s));
    if (diag) {
        CHECK_HIP(launch_diag_reduce(static_cast<const double *>(ws->diag_part.ptr), (int)rows,
                                     A.blocks, A.n_blocks, n_boxes,
                                     static_cast<const int32_t *>(wl.d_box_first.ptr), coef,
                                     P.H0, static_cast<double *>(ws->diag_out.ptr), s));
        CHECK_HIP(hipMemcpyAsync(P.diag, ws->diag_out.ptr,
                                 (size_t)n_boxes * rows * sizeof(colatus_diag),
                                 hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        for (int64_t r = 0; r < (int64_t)n_boxes * rows; ++r)
            if (P.diag[r].flags & 1u)
                return COLATUS_ENONFINITE;
    }
    return COLATUS_OK;
}

}  // namespace

namespace colatus {

// Host checks of the Eq. (10) attractor and Eq. (6) background arguments
// (NULL: none), copied into the kernels' ExtField.
int resolve_external(const colatus_attractor *a, const colatus_background *bg, ExtField &out)
{
    out = ExtField{};
    if (a) {
        if (!std::isfinite(a->strength) || !std::isfinite(a->x[0]) || !std::isfinite(a->x[1]) || !std::isfinite(a->x[2]))
            return COLATUS_EINVAL;
        out.on = 1;
        out.S = a->strength;
        out.x = a->x[0];
        out.y = a->x[1];
        out.z = a->x[2];
    }
    if (bg) {
        if (!std::isfinite(bg->coefficient) || !std::isfinite(bg->centre[0]) || !std::isfinite(bg->centre[1]) ||
            !std::isfinite(bg->centre[2]))
            return COLATUS_EINVAL;
        out.bg = 1;
        out.b = bg->coefficient;
        out.cx = bg->centre[0];
        out.cy = bg->centre[1];
        out.cz = bg->centre[2];
    }
    return COLATUS_OK;
}

}  // namespace colatus

namespace {

// ---------------------------------------------------------------------------
// Periodic boundaries (Ewald summation).
// ---------------------------------------------------------------------------
// The Ewald kernel's real-space part C(u) = erfc(u) + (2u/sqrt(pi)) e^{-u^2}
// (u = alpha r) and the reciprocal weights exp(-pi^2 n^2 / (alpha L)^2)
// both fall below the precision's resolution tol: alpha from C(alpha L / 2)
// = tol (the nearest image is the only real-space term kept; the others lie
// at least L / 2 away), n_max from the weight at tol.
constexpr double kEwaldTolFP64 = 1e-15;
constexpr double kEwaldTolFP32 = 3e-9;

void ewald_parameters(double L, int precision, double &alpha, int &nmax)
{
    const double tol = precision == COLATUS_FP64 ? kEwaldTolFP64 : kEwaldTolFP32;
    auto C = [](double u) { return std::erfc(u) + 1.1283791670955126 * u * std::exp(-u * u); };
    double lo = 0.0, hi = 12.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (C(mid) > tol)
            lo = mid;
        else
            hi = mid;
    }
    alpha = 2.0 * hi / L;
    nmax = (int)std::ceil(alpha * L / M_PI * std::sqrt(std::log(1.0 / tol)));
}

// The half-space reciprocal vectors n != 0, |n| <= nmax (n_x > 0, or n_x = 0
// and n_y > 0, or n_x = n_y = 0 and n_z > 0), as column segments of up to
// kEwaldSegLen consecutive n_z, with their weights 2 (4 pi / L^3)
// exp(-k^2 / 4 alpha^2) / k^2; uploaded once per (L, precision).  A second
// copy of the segments, longest first, feeds the structure-factor kernel,
// whose lanes each take a segment: a wave of equal counts runs its loop over
// the k without idle lanes (its sums are stored by k, so the order changes
// no result).
int ensure_ewald_plan(Workspace *ws, double L, int precision, hipStream_t s)
{
    double alpha = 0.0;
    int nmax = 0;
    ewald_parameters(L, precision, alpha, nmax);
    if (ws->ew_L == L && ws->ew_alpha == alpha && ws->ew_nmax == nmax)
        return COLATUS_OK;
    ws->ew_nmax = -1;
    std::vector<EwaldSeg> segs;
    std::vector<double> coef;
    const double vol = L * L * L;
    for (int nx = 0; nx <= nmax; ++nx)
        for (int ny = -nmax; ny <= nmax; ++ny) {
            const int r2 = nx * nx + ny * ny;
            if (r2 > nmax * nmax)
                continue;
            const int zm = (int)std::floor(std::sqrt((double)(nmax * nmax - r2)));
            int z0 = -zm;
            if (nx == 0 && ny < 0)
                continue;
            if (nx == 0 && ny == 0)
                z0 = 1;
            for (int zb = z0; zb <= zm; zb += kEwaldSegLen) {
                EwaldSeg g;
                g.nx = nx;
                g.ny = ny;
                g.z0 = zb;
                g.cnt = std::min(kEwaldSegLen, zm - zb + 1);
                g.k0 = (int)coef.size();
                for (int q = 0; q < g.cnt; ++q) {
                    const double kx = 2.0 * M_PI * nx / L, ky = 2.0 * M_PI * ny / L,
                                 kz = 2.0 * M_PI * (zb + q) / L;
                    const double k2 = kx * kx + ky * ky + kz * kz;
                    coef.push_back(2.0 * 4.0 * M_PI / vol * std::exp(-k2 / (4.0 * alpha * alpha)) /
                                   k2);
                }
                segs.push_back(g);
            }
        }
    std::vector<EwaldSeg> segs_sk = segs;
    std::stable_sort(segs_sk.begin(), segs_sk.end(),
                     [](const EwaldSeg &a, const EwaldSeg &b) { return a.cnt > b.cnt; });
    // the previous plan's buffers may still be read by queued work
    CHECK_HIP(hipStreamSynchronize(s));
    CHECK_RC(ensure(ws->ew_segs, std::max<size_t>(1, segs.size()) * sizeof(EwaldSeg)));
    CHECK_RC(ensure(ws->ew_segs_sk, std::max<size_t>(1, segs.size()) * sizeof(EwaldSeg)));
    CHECK_RC(ensure(ws->ew_coef, std::max<size_t>(1, coef.size()) * sizeof(double)));
    if (!segs.empty()) {
        CHECK_HIP(hipMemcpyAsync(ws->ew_segs.ptr, segs.data(), segs.size() * sizeof(EwaldSeg),
                                 hipMemcpyHostToDevice, s));
        CHECK_HIP(hipMemcpyAsync(ws->ew_segs_sk.ptr, segs_sk.data(),
                                 segs_sk.size() * sizeof(EwaldSeg), hipMemcpyHostToDevice, s));
        CHECK_HIP(hipMemcpyAsync(ws->ew_coef.ptr, coef.data(), coef.size() * sizeof(double),
                                 hipMemcpyHostToDevice, s));
        CHECK_HIP(hipStreamSynchronize(s));  // the host tables are local
    }
    ws->ew_L = L;
    ws->ew_alpha = alpha;
    ws->ew_nsegs = (int)segs.size();
    ws->ew_K = (int)coef.size();
    ws->ew_nmax = nmax;
    return COLATUS_OK;
}

// Work buffers of the reciprocal-space sums for N particles, and the
// launch arguments.
int ewald_args(Workspace *ws, const double *x, const double *m, int64_t N, EwaldArgs &A)
{
    const int n_sk = (int)std::max<int64_t>(1, std::min<int64_t>(256, N / 256));
    const int64_t blocks = (N + 63) / 64;
    const int n_kc = (int)std::max<int64_t>(1, std::min<int64_t>(64, (8192 + blocks - 1) / blocks));
    const size_t K = (size_t)std::max(1, ws->ew_K);
    CHECK_RC(ensure(ws->ew_skp, (size_t)n_sk * K * 2 * sizeof(double)));
    CHECK_RC(ensure(ws->ew_S, K * 2 * sizeof(double)));
    CHECK_RC(ensure(ws->ew_kpg, (size_t)n_kc * 3 * (size_t)N * sizeof(double)));
    CHECK_RC(ensure(ws->ew_kpp, (size_t)n_kc * (size_t)N * sizeof(double)));
    CHECK_RC(ensure(ws->ew_msum, sizeof(double)));
    CHECK_RC(ensure(ws->ew_g, 3 * (size_t)N * sizeof(double)));
    CHECK_RC(ensure(ws->ew_p, (size_t)N * sizeof(double)));
    A.x = x;
    A.m = m;
    A.N = N;
    A.L = ws->ew_L;
    A.alpha = ws->ew_alpha;
    A.segs = static_cast<const EwaldSeg *>(ws->ew_segs.ptr);
    A.segs_sk = static_cast<const EwaldSeg *>(ws->ew_segs_sk.ptr);
    A.n_segs = ws->ew_nsegs;
    A.K = ws->ew_K;
    A.coef = static_cast<const double *>(ws->ew_coef.ptr);
    A.sk_part = static_cast<double2 *>(ws->ew_skp.ptr);
    A.n_sk_chunks = n_sk;
    A.S = static_cast<double2 *>(ws->ew_S.ptr);
    A.n_k_chunks = n_kc;
    A.kpart_g = static_cast<double *>(ws->ew_kpg.ptr);
    A.kpart_p = static_cast<double *>(ws->ew_kpp.ptr);
    A.msum = static_cast<double *>(ws->ew_msum.ptr);
    A.gk = static_cast<double *>(ws->ew_g.ptr);
    A.pk = static_cast<double *>(ws->ew_p.ptr);
    A.mass_ready = false;
    return COLATUS_OK;
}

// The symmetric work list (parts of 256) of one box, whatever the tile
// options say: the periodic real-space loop runs on it.
int prepare_periodic_worklist(Workspace *ws, int64_t N, double eps, hipStream_t s)
{
    Boxes b;
    b.off = {0, N};
    b.eps = {eps};
    b.max_n = N;
    WorkList *wl = nullptr;
    CHECK_RC(select_worklist(ws, b, N, symmetric_cfg(b, 4, 64), s, wl));
    ws->fwd = wl;
    return COLATUS_OK;
}

bool valid_box(double box) { return is_fin(box) && box > 0.0; }

// The discrete adjoint of a kick-drift-kick run (colatus_adjoint and
// colatus_ftle), on the calling entry point's workspace, lock held.
struct AdjointParams {
    const double *x0, *v0, *m;
    int64_t N;
    double G, H0, OmR, OmM, OmK, OmL, a_begin, a_end;
    int64_t n_steps, checkpoint_every;
    int32_t n_cot;
    const double *lam_xN, *lam_vN;  // the caller's cotangents, or lam_xN null:
    const int64_t *seed_idx;        // unit cotangents e_i on x of these
                                    // n_cot / 3 particles (device), none on v
    double *grad_x0, *grad_v0;      // outputs, or null (left in lam_x / lam_p)
    double *xN, *vN, *grad_attractor;
    int precision;
    ExtField ext;
    hipStream_t stream;
    std::vector<StepCoef> *coef_host;  // receives the coefficient table, or null
};

int adjoint_impl(Workspace *ws, const AdjointParams &P, const Boxes &b)
{
    const double *x0 = P.x0, *v0 = P.v0, *m = P.m, *lam_xN = P.lam_xN, *lam_vN = P.lam_vN;
    const int64_t N = P.N, n_steps = P.n_steps;
    int64_t checkpoint_every = P.checkpoint_every;
    const int32_t n_cot = P.n_cot;
    const double G = P.G;
    double *grad_x0 = P.grad_x0, *grad_v0 = P.grad_v0, *xN = P.xN, *vN = P.vN,
           *grad_attractor = P.grad_attractor;
    const int precision = P.precision;
    const ExtField &ext = P.ext;
    hipStream_t s = P.stream;
    bool mask = false;
    for (double e : b.eps)
        mask = mask || e == 0.0;
    CHECK_RC(prepare_worklist(ws, 0, b, N, precision, x0, m, 1, s));
    CHECK_RC(prepare_worklist(ws, 1, b, N, precision, x0, m, n_cot, s));
    const WorkList &wf = *ws->fwd;
    const WorkList &wa = *ws->adj;
    CHECK_RC(prepare_box_mass(ws, wf, m, s));
    const size_t n3 = 3 * (size_t)N;
    if (checkpoint_every < 0) {
        // automatic: every position when they take at most a quarter of the
        // free device memory, else segments of ceil(sqrt(n_steps)) steps
        // (the least checkpoint + segment memory; the compute is the same for
        // every segment length)
        size_t free_b = 0, total_b = 0;
        CHECK_HIP(hipMemGetInfo(&free_b, &total_b));
        const double need = (double)(n_steps + 1) * (double)n3 * sizeof(double);
        checkpoint_every = need <= 0.25 * (double)free_b
                               ? 0
                               : (int64_t)std::ceil(std::sqrt((double)n_steps));
    }
    // checkpoint_every == 0: every position of the forward run is kept (one
    // segment spanning the run, filled by the forward pass itself)
    const bool keep_all = checkpoint_every == 0;
    const int64_t K = keep_all ? n_steps : checkpoint_every;
    const int64_t n_seg = (n_steps + K - 1) / K;
    CHECK_RC(ensure(ws->coef, (size_t)n_steps * sizeof(StepCoef)));
    CHECK_RC(ensure(ws->p, n3 * sizeof(double)));
    const size_t part_fwd = (size_t)wf.max_slices * n3;
    const size_t part_adj = (size_t)wa.max_slices * n3 * (size_t)n_cot;
    CHECK_RC(ensure(ws->part, std::max(part_fwd, part_adj) * sizeof(double)));
    CHECK_RC(ensure(ws->lam_x, (size_t)n_cot * n3 * sizeof(double)));
    CHECK_RC(ensure(ws->lam_p, (size_t)n_cot * n3 * sizeof(double)));
    // checkpoints: (x, p) at n = 0, K, 2K, ... ; segment states: K + 1 positions
    CHECK_RC(ensure(ws->ckpt, (size_t)n_seg * 2 * n3 * sizeof(double)));
    CHECK_RC(ensure(ws->seg, (size_t)(K + 1) * n3 * sizeof(double)));

    StepCoef *coef = static_cast<StepCoef *>(ws->coef.ptr);
    double *p = static_cast<double *>(ws->p.ptr);
    double *ck = static_cast<double *>(ws->ckpt.ptr);
    double *seg = static_cast<double *>(ws->seg.ptr);
    double *lx = static_cast<double *>(ws->lam_x.ptr);
    double *lp = static_cast<double *>(ws->lam_p.ptr);
    // the working position buffer is the first segment slot
    double *xw = seg;

    CHECK_HIP(launch_coefficients(P.H0, P.OmR, P.OmM, P.OmK, P.OmL, P.a_begin, P.a_end, n_steps, 0,
                                  n_steps, 0, coef, s));
    std::vector<StepCoef> hc((size_t)n_steps);
    CHECK_HIP(hipMemcpyAsync(hc.data(), coef, hc.size() * sizeof(StepCoef), hipMemcpyDeviceToHost,
                             s));
    CHECK_HIP(hipStreamSynchronize(s));

    IntegrateArgs A;
    A.p = p;
    A.m = m;
    A.part = static_cast<const double *>(ws->part.ptr);
    A.part_phi = nullptr;
    A.blocks = static_cast<const IntBlock *>(wf.d_blocks.ptr);
    A.n_blocks = (int)wf.blocks.size();
    A.N = N;
    A.G = G;
    A.coef = coef;
    A.step = step_counter(ws);
    A.work_counter = work_counter(ws);
    A.diag_part = nullptr;
    A.precision = precision;
    A.box_mass = static_cast<const double *>(ws->box_mass.ptr);
    A.slot_mode = slot_mode_of(wf, precision);
    A.ext = ext;
    // per-block accumulators of the attractor's parameter derivatives
    double *acc_att = nullptr;
    const int n_ablk = (int)wa.blocks.size();
    if (grad_attractor) {
        const size_t n_acc = (size_t)n_ablk * (size_t)n_cot * 4;
        CHECK_RC(ensure(ws->att_acc, n_acc * sizeof(double)));
        acc_att = static_cast<double *>(ws->att_acc.ptr);
        CHECK_HIP(launch_fill(acc_att, (int64_t)n_acc, 0.0, s));
    }

    // ---- forward with checkpoints --------------------------------------
    CHECK_HIP(hipMemcpyAsync(xw, x0, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    CHECK_HIP(launch_convert(0, v0, p, N, coef, 0, s));
    CHECK_RC(set_step(ws, 0, 0, n_steps, s));
    A.x = xw;
    for (int64_t n = 0; n < n_steps; ++n) {
        TraceRange step("adjoint forward step");
        if (keep_all) {
            // x_n stays in slot n; the step writes x_{n+1} into slot n + 1
            double *xs = seg + (size_t)n * n3;
            double *xn = xs + n3;
            CHECK_RC(run_forward_sweep(ws, wf, precision, false, mask, xs, m, N, s, true));
            CHECK_HIP(hipMemcpyAsync(xn, xs, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            A.x = xn;
            CHECK_HIP(launch_integrate(A, s));
            CHECK_HIP(launch_tick(step_counter(ws), work_counter(ws), s));
            continue;
        }
        CHECK_RC(run_forward_sweep(ws, wf, precision, false, mask, xw, m, N, s, true));
        if (n % K == 0) {
            double *cx = ck + (size_t)(n / K) * 2 * n3;
            CHECK_HIP(hipMemcpyAsync(cx, xw, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            CHECK_HIP(hipMemcpyAsync(cx + n3, p, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        CHECK_HIP(launch_integrate(A, s));
        CHECK_HIP(launch_tick(step_counter(ws), work_counter(ws), s));
    }
    if (keep_all)
        xw = seg + (size_t)n_steps * n3;  // x_N
    if (xN || vN) {
        CHECK_RC(run_forward_sweep(ws, wf, precision, false, mask, xw, m, N, s, true));
        A.x = xw;
        CHECK_HIP(launch_integrate(A, s));  // closing half kick at a_end
        if (xN)
            CHECK_HIP(hipMemcpyAsync(xN, xw, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (vN)
            CHECK_HIP(launch_convert(1, p, vN, N, coef, n_steps - 1, s));
    }

    // ---- reverse sweep ---------------------------------------------------
    const double aN = hc[(size_t)n_steps - 1].a1, a0 = hc[0].a0;
    if (lam_xN) {
        CHECK_HIP(hipMemcpyAsync(lx, lam_xN, (size_t)n_cot * n3 * sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
        CHECK_HIP(launch_scale(lam_vN, lp, (int64_t)n_cot * (int64_t)n3, 1.0 / (aN * aN), s));
    } else {
        // unit cotangents on the tracers' final positions, none on velocities
        CHECK_HIP(launch_fill(lp, (int64_t)n_cot * (int64_t)n3, 0.0, s));
        CHECK_HIP(launch_ftle_seed(lx, (int64_t)n_cot * (int64_t)n3, P.seed_idx, n_cot / 3, N,
                                   s));
    }
    for (int64_t sg = n_seg - 1; sg >= 0; --sg) {
        const int64_t lo = sg * K, hi = std::min(lo + K, n_steps);
        // recompute positions x_lo .. x_hi from the checkpoint (bitwise: same
        // kernels), unless the forward pass kept them all
        const double *cx = ck + (size_t)sg * 2 * n3;
        if (!keep_all) {
            CHECK_HIP(hipMemcpyAsync(seg, cx, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            CHECK_HIP(hipMemcpyAsync(p, cx + n3, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            CHECK_RC(set_step(ws, lo, 0, n_steps, s));
        }
        for (int64_t n = lo; n < hi && !keep_all; ++n) {
            double *xs = seg + (size_t)(n - lo) * n3;
            double *xn = seg + (size_t)(n - lo + 1) * n3;
            CHECK_RC(run_forward_sweep(ws, wf, precision, false, mask, xs, m, N, s, true));
            CHECK_HIP(hipMemcpyAsync(xn, xs, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
            IntegrateArgs B = A;
            B.x = xn;
            CHECK_HIP(launch_integrate(B, s));
            CHECK_HIP(launch_tick(step_counter(ws), work_counter(ws), s));
        }
        // visit x_n for n = hi .. lo+1 (and lo itself in segment 0): every grid
        // point is visited once, x_hi being the unvisited bottom of the segment above
        const int64_t top = hi;
        const int64_t bottom = (sg == 0) ? lo : lo + 1;
        for (int64_t n = top; n >= bottom; --n) {
            TraceRange step("adjoint reverse step");
            const double *xs = seg + (size_t)(n - lo) * n3;
            CHECK_RC(run_adjoint_sweep(ws, wa, precision, mask, xs, m, N, n_cot, lp, s));
            const double cw = (n < n_steps ? hc[(size_t)n].k1 : 0.0) +
                              (n > 0 ? hc[(size_t)n - 1].k2 : 0.0);
            const double dnext = n > 0 ? hc[(size_t)n - 1].d : 0.0;
            CHECK_HIP(launch_adjoint_update(static_cast<const IntBlock *>(wa.d_blocks.ptr),
                                            n_ablk, static_cast<const double *>(ws->part.ptr),
                                            slot_mode_of(wa, precision),
                                            static_cast<const double *>(ws->box_mass.ptr), xs,
                                            ext, acc_att, N, n_cot, G, cw, lx, lp,
                                            n > 0 ? 1 : 0, dnext, s));
        }
    }
    if (grad_x0)
        CHECK_HIP(hipMemcpyAsync(grad_x0, lx, (size_t)n_cot * n3 * sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
    if (grad_v0)
        CHECK_HIP(launch_scale(lp, grad_v0, (int64_t)n_cot * (int64_t)n3, a0 * a0, s));
    if (P.coef_host)
        *P.coef_host = std::move(hc);
    if (grad_attractor)
        CHECK_HIP(launch_att_grad_reduce(acc_att, n_ablk, n_cot, grad_attractor, s));
        return COLATUS_OK;
}

}  // namespace

// ===========================================================================
// Exported entry points.
// ===========================================================================
extern "C" {

int colatus_version(void) { return 10400; }

const char *colatus_strerror(int code)
{
    switch (code) {
    case COLATUS_OK: return "success";
    case COLATUS_EINVAL: return "invalid argument";
    case COLATUS_EFRIEDMANN: return "H^2(a) <= 0 on the requested range of a";
    case COLATUS_ENODEV: return "no HIP device available";
    case COLATUS_ENOMEM: return "device memory allocation failed";
    case COLATUS_EHIP: return "HIP runtime error";
    case COLATUS_ENONFINITE: return "non-finite value in the state";
    case COLATUS_ESCRATCH:
        return "problem too large for the fixed scratch of the allocation-free entry point";
    default: return "unknown error code";
    }
}

int colatus_hubble(double a, double H0, double Om_R, double Om_M, double Om_K, double Om_L,
                   double *H)
{
    if (!H || !is_fin(a) || a <= 0.0 || !is_fin(H0) || H0 < 0.0 || !is_fin(Om_R) ||
        !is_fin(Om_M) || !is_fin(Om_K) || !is_fin(Om_L))
        return COLATUS_EINVAL;
    const double e2 = Om_R / (a * a * a * a) + Om_M / (a * a * a) + Om_K / (a * a) + Om_L;
    if (e2 < 0.0)
        return COLATUS_EFRIEDMANN;
    *H = H0 * std::sqrt(e2);
    return COLATUS_OK;
}

int colatus_set_option(int key, int64_t value)
{
    std::lock_guard<std::mutex> lock(g_mu);
    switch (key) {
    case COLATUS_OPT_GRAPH: g_opt.graph = value != 0; return COLATUS_OK;
    case COLATUS_OPT_TIMER: g_opt.timer = value != 0; return COLATUS_OK;
    case COLATUS_OPT_AUTOTUNE: g_opt.autotune = value != 0; return COLATUS_OK;
    case COLATUS_OPT_TILE_R:
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
            return COLATUS_EINVAL;
        g_opt.tile_r = value;
        return COLATUS_OK;
    case COLATUS_OPT_TILE_TPB:
        if (value != 0 && value != 64 && value != 128 && value != 256)
            return COLATUS_EINVAL;
        g_opt.tile_tpb = value;
        return COLATUS_OK;
    case COLATUS_OPT_TILE_SLICES:
        if (value < 0 || value > 4096)
            return COLATUS_EINVAL;
        g_opt.tile_slices = value;
        return COLATUS_OK;
    case COLATUS_OPT_PERSISTENT: g_opt.persistent = value != 0; return COLATUS_OK;
    case COLATUS_OPT_ROCTX: g_opt.roctx = value != 0; return COLATUS_OK;
    case COLATUS_OPT_PAIR_FORM:
        if (value < -1 || value > 2)
            return COLATUS_EINVAL;
        g_opt.pair_form = value;
        return COLATUS_OK;
    case COLATUS_OPT_PAIR_GROUP:
        if (value != 0 && value != 1)
            return COLATUS_EINVAL;
        g_opt.pair_group = value;
        return COLATUS_OK;
    }
    return COLATUS_EINVAL;
}

int colatus_get_option(int key, int64_t *value)
{
    if (!value)
        return COLATUS_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    switch (key) {
    case COLATUS_OPT_GRAPH: *value = g_opt.graph; return COLATUS_OK;
    case COLATUS_OPT_TIMER: *value = g_opt.timer; return COLATUS_OK;
    case COLATUS_OPT_AUTOTUNE: *value = g_opt.autotune; return COLATUS_OK;
    case COLATUS_OPT_TILE_R: *value = g_opt.tile_r; return COLATUS_OK;
    case COLATUS_OPT_TILE_TPB: *value = g_opt.tile_tpb; return COLATUS_OK;
    case COLATUS_OPT_TILE_SLICES: *value = g_opt.tile_slices; return COLATUS_OK;
    case COLATUS_OPT_PERSISTENT: *value = g_opt.persistent; return COLATUS_OK;
    case COLATUS_OPT_PAIR_FORM: *value = g_opt.pair_form; return COLATUS_OK;
    case COLATUS_OPT_ROCTX: *value = g_opt.roctx; return COLATUS_OK;
    case COLATUS_OPT_PAIR_GROUP: *value = g_opt.pair_group; return COLATUS_OK;
    }
    return COLATUS_EINVAL;
}

int colatus_timer_read(int kind, double *total_ms, int64_t *launches, int reset)
{
    if (kind < 0 || kind > 2 || !total_ms || !launches)
        return COLATUS_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    double tot = 0.0;
    for (const TimerRec &r : g_timer[kind]) {
        CHECK_HIP(hipEventSynchronize(r.stop));
        float ms = 0.0f;
        CHECK_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)g_timer[kind].size();
    if (reset) {
        for (const TimerRec &r : g_timer[kind]) {
            g_event_pool.push_back(r.start);
            g_event_pool.push_back(r.stop);
        }
        g_timer[kind].clear();
    }
    return COLATUS_OK;
}

int colatus_tile_config(int64_t N, int precision, int kind, int32_t out[4])
{
    if (!out || N < 1 || N > kMaxN || !valid_precision(precision) || kind < 0 || kind > 1)
        return COLATUS_EINVAL;
    int dev = 0;
    int n_cu = 256;
    if (device_ready(dev) == COLATUS_OK)
        n_cu = cu_count(dev);
    Boxes b;
    b.off = {0, N};
    b.eps = {0.0};
    b.max_n = N;
    std::lock_guard<std::mutex> lock(g_mu);
    TuneKey key{pow2_ceil(N), 1, precision, kind};
    auto it = g_tuned.find(key);
    TileCfg c = it != g_tuned.end() ? it->second : heuristic_cfg(b, precision, kind, n_cu);
    c = apply_overrides(c, kind, precision, b, n_cu);
    out[0] = c.R;
    out[1] = c.tpb;
    out[2] = c.slices;
    out[3] = c.form;
    return COLATUS_OK;
}

int colatus_release(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return COLATUS_OK;
    int current = 0;
    const bool restore = hipGetDevice(&current) == hipSuccess;
    for (auto &kv : g_ws) {
        Workspace *ws = kv.second;
        (void)hipSetDevice(ws->device);
        (void)hipStreamSynchronize(ws->stream);
        for (Buffer *bb : ws->buffers())
            if (bb->ptr)
                (void)hipFree(bb->ptr);
        for (WorkList *wl : ws->lists) {
            free_worklist_buffers(*wl);
            delete wl;
        }
        for (StepGraph &sg : ws->graphs)
            (void)hipGraphExecDestroy(sg.exec);
        if (ws->track_ev)
            (void)hipEventDestroy(ws->track_ev);
        if (ws->ftle_ev)
            (void)hipEventDestroy(ws->ftle_ev);
        if (ws->cap_stream)
            (void)hipStreamDestroy(ws->cap_stream);
        delete ws;
    }
    g_ws.clear();
    // pooled timer events (those still held by unread timers stay valid)
    for (hipEvent_t e : g_event_pool)
        (void)hipEventDestroy(e);
    g_event_pool.clear();
    if (restore)
        (void)hipSetDevice(current);
    return COLATUS_OK;
}

int colatus_forces(const double *x, const double *m, int64_t N, double eps, double G, double a,
                   int precision, double *acc, double *phi, const colatus_batch *batch,
                   const colatus_attractor *attractor, const colatus_background *background,
                   void *stream)
{
    TraceRange trace("colatus_forces");
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G) || !is_fin(a) || a <= 0.0)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, m, acc}));
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, batch, b));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(prepare_worklist(ws, 0, b, N, precision, x, m, 1, s));
    const WorkList &wl = *ws->fwd;
    CHECK_RC(prepare_box_mass(ws, wl, m, s));
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * 3 * N * sizeof(double)));
    if (phi)
        CHECK_RC(ensure(ws->part_phi, (size_t)wl.max_slices * N * sizeof(double)));
    bool mask = false;
    for (double e : b.eps)
        mask = mask || e == 0.0;
    CHECK_RC(run_forward_sweep(ws, wl, precision, phi != nullptr, mask, x, m, N, s, true));
    CHECK_HIP(launch_forces_finalize(precision, static_cast<const double *>(ws->box_mass.ptr),
                                     static_cast<const IntBlock *>(wl.d_blocks.ptr),
                                     (int)wl.blocks.size(), static_cast<const double *>(ws->part.ptr),
                                     phi ? static_cast<const double *>(ws->part_phi.ptr) : nullptr,
                                     slot_mode_of(wl, precision), x, m, N, G, G / (a * a * a), ext,
                                     1.0 / (a * a * a), acc, phi, s));
    return COLATUS_OK;
}

// The paper's difference equations, Eqs. (3)-(5): per step one sweep at the
// half-step positions and one O(N) update (kick with drag, the two half
// drifts fused across steps); with diagnostics, a potential sweep at the
// integer-point positions as well.  Launched eagerly.
int run_he_impl(const RunParams &P, const Boxes &b)
{
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(P.stream, ws));
    hipStream_t s = P.stream;
    CHECK_RC(prepare_worklist(ws, 0, b, P.N, P.precision, P.x, P.m, 1, s));
    const WorkList &wl = *ws->fwd;
    CHECK_RC(prepare_box_mass(ws, wl, P.m, s));
    const int64_t nsteps = P.last - P.first;
    const int64_t rows = nsteps + 1;
    const int n_boxes = (int)b.eps.size();
    const size_t n3 = 3 * (size_t)P.N;
    CHECK_RC(ensure(ws->coef, (size_t)nsteps * sizeof(StepCoef)));
    CHECK_RC(ensure(ws->p, n3 * sizeof(double)));
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * n3 * sizeof(double)));
    const bool diag = P.diag != nullptr;
    if (diag) {
        CHECK_RC(ensure(ws->he_x, n3 * sizeof(double)));
        CHECK_RC(ensure(ws->part_phi, (size_t)wl.max_slices * P.N * sizeof(double)));
        CHECK_RC(ensure(ws->diag_part, (size_t)rows * wl.blocks.size() * kDiagW * sizeof(double)));
        CHECK_RC(ensure(ws->diag_out, (size_t)n_boxes * rows * sizeof(colatus_diag)));
    }
    bool mask = false;
    for (double e : b.eps)
        mask = mask || e == 0.0;

    StepCoef *coef = static_cast<StepCoef *>(ws->coef.ptr);
    double *vw = static_cast<double *>(ws->p.ptr);  // the velocity, updated in place
    double *xi = diag ? static_cast<double *>(ws->he_x.ptr) : nullptr;
    const IntBlock *blocks = static_cast<const IntBlock *>(wl.d_blocks.ptr);
    const int n_blocks = (int)wl.blocks.size();
    const int smode = slot_mode_of(wl, P.precision);
    const double *bm = static_cast<const double *>(ws->box_mass.ptr);
    double *dpart = diag ? static_cast<double *>(ws->diag_part.ptr) : nullptr;
    const double *pphi = static_cast<const double *>(ws->part_phi.ptr);
    CHECK_HIP(launch_coefficients(P.H0, P.OmR, P.OmM, P.OmK, P.OmL, P.a_begin, P.a_end,
                                  P.n_steps, P.first, P.last, 1, coef, s));
    CHECK_HIP(hipMemcpyAsync(vw, P.v, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    CHECK_RC(prepare_tracks(ws, P));
    if (diag) {
        CHECK_RC(run_forward_sweep(ws, wl, P.precision, true, mask, P.x, P.m, P.N, s, true));
        CHECK_HIP(launch_state_diag(P.x, vw, P.m, pphi, smode, blocks, n_blocks, P.N, P.G, coef,
                                    0, P.precision, bm, P.ext, dpart, s));
    }
    CHECK_HIP(launch_he_drift(P.x, vw, P.N, coef, 0, 0.5, s));
    HEArgs H;
    H.x = P.x;
    H.v = vw;
    H.xi = xi;
    H.part = static_cast<const double *>(ws->part.ptr);
    H.slot_mode = smode;
    H.blocks = blocks;
    H.n_blocks = n_blocks;
    H.N = P.N;
    H.G = P.G;
    H.coef = coef;
    H.box_mass = bm;
    H.ext = P.ext;
    H.track_slot = P.trk.n ? static_cast<const int32_t *>(ws->track_slot.ptr) : nullptr;
    H.track = P.trk.out;
    H.n_tracers = P.trk.n;
    for (int64_t r = 0; r < nsteps; ++r) {
        TraceRange step("step");
        CHECK_RC(run_forward_sweep(ws, wl, P.precision, false, mask, P.x, P.m, P.N, s, true));
        H.row = r;
        H.last = r + 1 == nsteps ? 1 : 0;
        CHECK_HIP(launch_he_step(H, s));
        if (diag) {
            CHECK_RC(run_forward_sweep(ws, wl, P.precision, true, mask, xi, P.m, P.N, s, true));
            CHECK_HIP(launch_state_diag(xi, vw, P.m, pphi, smode, blocks, n_blocks, P.N, P.G, coef,
                                        r + 1, P.precision, bm, P.ext, dpart, s));
        }
    }
    CHECK_HIP(hipMemcpyAsync(P.v, vw, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (diag) {
        CHECK_HIP(launch_diag_reduce(dpart, (int)rows, blocks, n_blocks, n_boxes,
                                     static_cast<const int32_t *>(wl.d_box_first.ptr), coef,
                                     P.H0, static_cast<double *>(ws->diag_out.ptr), s));
        CHECK_HIP(hipMemcpyAsync(P.diag, ws->diag_out.ptr,
                                 (size_t)n_boxes * rows * sizeof(colatus_diag),
                                 hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        for (int64_t q = 0; q < (int64_t)n_boxes * rows; ++q)
            if (P.diag[q].flags & 1u)
                return COLATUS_ENONFINITE;
    }
    return COLATUS_OK;
}

int colatus_run_he(double *x, double *v, const double *m, int64_t N, double eps, double G,
                   double H0, double Om_R, double Om_M, double Om_K, double Om_L,
                   double a_begin, double a_end, int64_t n_steps, int64_t first_step,
                   int64_t last_step, int precision, colatus_diag *diag,
                   const colatus_batch *batch, const colatus_attractor *attractor,
                   const colatus_background *background, const colatus_tracks *tracks,
                   void *stream)
{
    TraceRange trace("colatus_run_he");
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G))
        return COLATUS_EINVAL;
    if (n_steps < 1 || first_step < 0 || last_step <= first_step || last_step > n_steps)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, v, m}));
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, batch, b));
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    Tracks trk;
    CHECK_RC(resolve_tracks(tracks, N, trk));
    RunParams P{x, v, m, N, G, H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end, n_steps,
                first_step, last_step, precision, diag, static_cast<hipStream_t>(stream), ext,
                trk};
    return run_he_impl(P, b);
}

int colatus_run(double *x, double *v, const double *m, int64_t N, double eps, double G,
                double H0, double Om_R, double Om_M, double Om_K, double Om_L, double a_begin,
                double a_end, int64_t n_steps, int64_t first_step, int64_t last_step,
                int precision, colatus_diag *diag, const colatus_batch *batch,
                const colatus_attractor *attractor, const colatus_background *background,
                const colatus_tracks *tracks,
                void *stream)
{
    TraceRange trace("colatus_run");
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G))
        return COLATUS_EINVAL;
    if (n_steps < 1 || first_step < 0 || last_step <= first_step || last_step > n_steps)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, v, m}));
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, batch, b));
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    Tracks trk;
    CHECK_RC(resolve_tracks(tracks, N, trk));
    RunParams P{x, v, m, N, G, H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end, n_steps,
                first_step, last_step, precision, diag, static_cast<hipStream_t>(stream), ext,
                trk};
    return run_impl(P, b);
}

int colatus_step(double *x, double *v, const double *m, int64_t N, double eps, double G,
                 double H0, double Om_R, double Om_M, double Om_K, double Om_L, double a,
                 double a_next, int precision, double *g_cache, const colatus_batch *batch,
                 const colatus_attractor *attractor, const colatus_background *background,
                 void *stream)
{
    TraceRange trace("colatus_step");
    if (!g_cache)
        return colatus_run(x, v, m, N, eps, G, H0, Om_R, Om_M, Om_K, Om_L, a, a_next, 1, 0, 1,
                           precision, nullptr, batch, attractor, background, nullptr, stream);
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G))
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, v, m}));
    if (g_cache == x || g_cache == v)
        return COLATUS_EINVAL;
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, batch, b));
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a, a_next));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(prepare_worklist(ws, 0, b, N, precision, x, m, 1, s));
    const WorkList &wl = *ws->fwd;
    CHECK_RC(prepare_box_mass(ws, wl, m, s));
    const size_t n3 = 3 * (size_t)N;
    CHECK_RC(ensure(ws->coef, sizeof(StepCoef)));
    CHECK_RC(ensure(ws->p, n3 * sizeof(double)));
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * n3 * sizeof(double)));
    bool mask = false;
    for (double e : b.eps)
        mask = mask || e == 0.0;
    StepCoef *coef = static_cast<StepCoef *>(ws->coef.ptr);
    double *p = static_cast<double *>(ws->p.ptr);
    CHECK_HIP(launch_coefficients(H0, Om_R, Om_M, Om_K, Om_L, a, a_next, 1, 0, 1, 0, coef, s));
    CHECK_HIP(launch_cached_kick(0, x, v, p, g_cache, N, coef, s));
    CHECK_RC(run_forward_sweep(ws, wl, precision, false, mask, x, m, N, s, true));
    // g at the new positions into the cache (the comoving sum: a = 1), and
    // the closing half kick from it in the same kernel
    CHECK_HIP(launch_forces_finalize(precision, static_cast<const double *>(ws->box_mass.ptr),
                                     static_cast<const IntBlock *>(wl.d_blocks.ptr),
                                     (int)wl.blocks.size(), static_cast<const double *>(ws->part.ptr),
                                     nullptr, slot_mode_of(wl, precision), x, m, N, G, G, ext, 1.0,
                                     g_cache, nullptr, s, p, v, coef));
    return COLATUS_OK;
}

int colatus_forces_periodic(const double *x, const double *m, int64_t N, double eps, double G,
                            double a, double box, int precision, double *acc, double *phi,
                            void *stream)
{
    TraceRange trace("colatus_forces_periodic");
    if (N < 1 || N > kSymMaxN || !valid_precision(precision) || !is_fin(G) || !is_fin(a) ||
        a <= 0.0 || !is_fin(eps) || eps < 0.0 || !valid_box(box))
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, m, acc}));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(ensure_ewald_plan(ws, box, precision, s));
    CHECK_RC(prepare_periodic_worklist(ws, N, eps, s));
    const WorkList &wl = *ws->fwd;
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * 3 * N * sizeof(double)));
    if (phi)
        CHECK_RC(ensure(ws->part_phi, (size_t)wl.max_slices * N * sizeof(double)));
    EwaldArgs E;
    CHECK_RC(ewald_args(ws, x, m, N, E));
    CHECK_HIP(launch_ewald_real(precision, phi != nullptr, x, m, N,
                                static_cast<const WorkItem *>(wl.d_items.ptr), (int)wl.items.size(),
                                static_cast<double *>(ws->part.ptr),
                                phi ? static_cast<double *>(ws->part_phi.ptr) : nullptr, nullptr,
                                box, ws->ew_alpha, s));
    const ExtField none{};
    CHECK_HIP(launch_forces_finalize(precision, nullptr,
                                     static_cast<const IntBlock *>(wl.d_blocks.ptr),
                                     (int)wl.blocks.size(), static_cast<const double *>(ws->part.ptr),
                                     phi ? static_cast<const double *>(ws->part_phi.ptr) : nullptr,
                                     slot_mode_of(wl, precision), x, m, N, G, G / (a * a * a),
                                     none, 1.0 / (a * a * a), acc, phi, s));
    CHECK_HIP(launch_ewald_kspace(E, s));
    CHECK_HIP(launch_ewald_add(E.gk, E.pk, N, G, 1.0 / (a * a * a), acc, phi, s));
    return COLATUS_OK;
}

int colatus_run_periodic(double *x, double *v, const double *m, int64_t N, double eps, double G,
                         double H0, double Om_R, double Om_M, double Om_K, double Om_L,
                         double box, double a_begin, double a_end, int64_t n_steps,
                         int64_t first_step, int64_t last_step, int precision,
                         colatus_diag *diag, void *stream)
{
    TraceRange trace("colatus_run_periodic");
    if (N < 1 || N > kSymMaxN || !valid_precision(precision) || !is_fin(G) || !is_fin(eps) ||
        eps < 0.0 || !valid_box(box))
        return COLATUS_EINVAL;
    if (n_steps < 1 || first_step < 0 || last_step <= first_step || last_step > n_steps)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, v, m}));
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(ensure_ewald_plan(ws, box, precision, s));
    CHECK_RC(prepare_periodic_worklist(ws, N, eps, s));
    const WorkList &wl = *ws->fwd;
    const int64_t nsteps = last_step - first_step;
    const int64_t rows = nsteps + 1;
    const size_t n3 = 3 * (size_t)N;
    const bool with_diag = diag != nullptr;
    CHECK_RC(ensure(ws->coef, (size_t)nsteps * sizeof(StepCoef)));
    CHECK_RC(ensure(ws->p, n3 * sizeof(double)));
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * n3 * sizeof(double)));
    if (with_diag) {
        CHECK_RC(ensure(ws->part_phi, (size_t)wl.max_slices * N * sizeof(double)));
        CHECK_RC(ensure(ws->diag_part, (size_t)rows * wl.blocks.size() * kDiagW * sizeof(double)));
        CHECK_RC(ensure(ws->diag_out, (size_t)rows * sizeof(colatus_diag)));
    }
    EwaldArgs E;
    CHECK_RC(ewald_args(ws, x, m, N, E));
    StepCoef *coef = static_cast<StepCoef *>(ws->coef.ptr);
    double *p = static_cast<double *>(ws->p.ptr);
    CHECK_HIP(launch_coefficients(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end, n_steps, first_step,
                                  last_step, 0, coef, s));
    CHECK_HIP(launch_convert(0, v, p, N, coef, 0, s));
    CHECK_RC(set_step(ws, first_step, first_step, last_step, s));
    auto sweep = [&](int64_t *step_inc) -> int {
        CHECK_HIP(launch_ewald_real(precision, with_diag, x, m, N,
                                    static_cast<const WorkItem *>(wl.d_items.ptr),
                                    (int)wl.items.size(), static_cast<double *>(ws->part.ptr),
                                    with_diag ? static_cast<double *>(ws->part_phi.ptr) : nullptr,
                                    step_inc, box, ws->ew_alpha, s));
        CHECK_HIP(launch_ewald_kspace(E, s));
        return COLATUS_OK;
    };
    CHECK_RC(sweep(nullptr));
    E.mass_ready = true;  // the masses do not change during the run
    IntegrateArgs A;
    A.x = x;
    A.p = p;
    A.m = m;
    A.part = static_cast<const double *>(ws->part.ptr);
    A.part_phi = with_diag ? static_cast<const double *>(ws->part_phi.ptr) : nullptr;
    A.blocks = static_cast<const IntBlock *>(wl.d_blocks.ptr);
    A.n_blocks = (int)wl.blocks.size();
    A.N = N;
    A.G = G;
    A.coef = coef;
    A.step = step_counter(ws);
    A.work_counter = work_counter(ws);
    A.diag_part = with_diag ? static_cast<double *>(ws->diag_part.ptr) : nullptr;
    A.precision = precision;
    A.box_mass = nullptr;  // the periodic slots hold their masses
    A.slot_mode = slot_mode_of(wl, precision);
    A.ext = ExtField{};
    A.ewald_g = E.gk;
    A.ewald_p = E.pk;
    A.box = box;
    for (int64_t k = 0; k < nsteps; ++k) {
        TraceRange step("step");
        CHECK_RC(run_integrate(A, s));
        CHECK_RC(sweep(step_counter(ws)));  // advances the step
    }
    CHECK_RC(run_integrate(A, s));  // closing half kick at a_last (+ diagnostics)
    CHECK_HIP(launch_convert(1, p, v, N, coef, nsteps - 1, s));
    if (with_diag) {
        CHECK_HIP(launch_diag_reduce(static_cast<const double *>(ws->diag_part.ptr), (int)rows,
                                     A.blocks, A.n_blocks, 1,
                                     static_cast<const int32_t *>(wl.d_box_first.ptr), coef, H0,
                                     static_cast<double *>(ws->diag_out.ptr), s));
        CHECK_HIP(hipMemcpyAsync(diag, ws->diag_out.ptr, (size_t)rows * sizeof(colatus_diag),
                                 hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        for (int64_t r = 0; r < rows; ++r)
            if (diag[r].flags & 1u)
                return COLATUS_ENONFINITE;
    }
    return COLATUS_OK;
}

int colatus_velocity_spectrum(const double *track, int64_t rows, int32_t n_tracers,
                              int remove_mean, double *out, void *stream)
{
    TraceRange trace("colatus_velocity_spectrum");
    if (rows < 1 || rows > kMaxSpectrumRows || n_tracers < 1 || n_tracers > kMaxTracers)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({track, out}));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(ensure(ws->twiddle, (size_t)rows * 2 * sizeof(double)));
    CHECK_HIP(launch_velocity_spectrum(track, rows, n_tracers, remove_mean ? 1 : 0,
                                       static_cast<double *>(ws->twiddle.ptr), out, s));
    return COLATUS_OK;
}

int colatus_force_vjp(const double *x, const double *m, int64_t N, double eps, double G,
                      int32_t n_cot, const double *lam, double *out, int precision,
                      const colatus_attractor *attractor,
                      const colatus_background *background, void *stream)
{
    TraceRange trace("colatus_force_vjp");
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G) || n_cot < 1 ||
        n_cot > kMaxCot)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x, m, lam, out}));
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, nullptr, b));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(prepare_worklist(ws, 1, b, N, precision, x, m, n_cot, s));
    const WorkList &wl = *ws->adj;
    CHECK_RC(prepare_box_mass(ws, wl, m, s));
    CHECK_RC(ensure(ws->part, (size_t)wl.max_slices * n_cot * 3 * N * sizeof(double)));
    const bool mask = eps == 0.0;
    CHECK_RC(run_adjoint_sweep(ws, wl, precision, mask, x, m, N, n_cot, lam, s));
    CHECK_HIP(launch_vjp_finalize(static_cast<const IntBlock *>(wl.d_blocks.ptr),
                                  (int)wl.blocks.size(), static_cast<const double *>(ws->part.ptr),
                                  slot_mode_of(wl, precision),
                                  static_cast<const double *>(ws->box_mass.ptr), x, lam, ext, N,
                                  n_cot, G, out, s));
    return COLATUS_OK;
}

int colatus_adjoint(const double *x0, const double *v0, const double *m, int64_t N, double eps,
                    double G, double H0, double Om_R, double Om_M, double Om_K, double Om_L,
                    double a_begin, double a_end, int64_t n_steps, int64_t checkpoint_every,
                    int32_t n_cot, const double *lam_xN, const double *lam_vN, double *grad_x0,
                    double *grad_v0, double *xN, double *vN, double *grad_attractor,
                    int precision, const colatus_batch *batch,
                    const colatus_attractor *attractor,
                    const colatus_background *background, void *stream)
{
    TraceRange trace("colatus_adjoint");
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G) || n_steps < 1 ||
        checkpoint_every < -1 || n_cot < 1 || n_cot > kMaxCot)
        return COLATUS_EINVAL;
    if (grad_attractor && !attractor)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x0, v0, m, lam_xN, lam_vN, grad_x0, grad_v0}));
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, batch, b));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    AdjointParams P{x0, v0, m, N, G, H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end, n_steps,
                    checkpoint_every, n_cot, lam_xN, lam_vN, nullptr, grad_x0, grad_v0, xN, vN,
                    grad_attractor, precision, ext, s, nullptr};
    return adjoint_impl(ws, P, b);
}

int colatus_ftle(const double *x0, const double *v0, const double *m, int64_t N, double eps,
                 double G, double H0, double Om_R, double Om_M, double Om_K, double Om_L,
                 double a_begin, double a_end, int64_t n_steps, int64_t checkpoint_every,
                 int32_t n_tracers, const int64_t *tracers, double *lambda_t,
                 double *lambda_lna, double *blocks, int precision,
                 const colatus_batch *batch, const colatus_attractor *attractor,
                 const colatus_background *background, void *stream)
{
    TraceRange trace("colatus_ftle");
    if (N < 1 || N > kMaxN || !valid_precision(precision) || !is_fin(G) || n_steps < 1 ||
        checkpoint_every < -1 || n_tracers < 1 || n_tracers > kMaxCot / 3)
        return COLATUS_EINVAL;
    CHECK_RC(check_ptrs({x0, v0, m, tracers, lambda_t}));
    for (int32_t t = 0; t < n_tracers; ++t)
        if (tracers[t] < 0 || tracers[t] >= N)
            return COLATUS_EINVAL;
    Boxes b;
    CHECK_RC(resolve_boxes(N, eps, batch, b));
    ExtField ext;
    CHECK_RC(resolve_external(attractor, background, ext));
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    // the tracer list, uploaded from the workspace's own host copy
    CHECK_RC(ensure(ws->ftle_idx, (size_t)n_tracers * sizeof(int64_t)));
    if (!ws->ftle_ev)
        CHECK_HIP(hipEventCreateWithFlags(&ws->ftle_ev, hipEventDisableTiming));
    else
        CHECK_HIP(hipEventSynchronize(ws->ftle_ev));
    ws->ftle_host.assign(tracers, tracers + n_tracers);
    CHECK_HIP(hipMemcpyAsync(ws->ftle_idx.ptr, ws->ftle_host.data(),
                             (size_t)n_tracers * sizeof(int64_t), hipMemcpyHostToDevice, s));
    CHECK_HIP(hipEventRecord(ws->ftle_ev, s));
    const int64_t *didx = static_cast<const int64_t *>(ws->ftle_idx.ptr);
    std::vector<StepCoef> hc;
    AdjointParams P{x0, v0, m, N, G, H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end, n_steps,
                    checkpoint_every, 3 * n_tracers, nullptr, nullptr, didx, nullptr, nullptr,
                    nullptr, nullptr, nullptr, precision, ext, s, &hc};
    CHECK_RC(adjoint_impl(ws, P, b));
    // elapsed cosmic time: the step times summed in grid order, as the
    // diagnostics rows do; per unit ln a unless a is held fixed
    double span_t = 0.0;
    for (const StepCoef &c : hc)
        span_t += c.dt;
    const double span_lna = H0 == 0.0 ? NAN : std::log(a_end / a_begin);
    CHECK_HIP(launch_ftle(static_cast<const double *>(ws->lam_x.ptr), didx, n_tracers, N, span_t,
                          span_lna, lambda_t, lambda_lna, blocks, s));
    return COLATUS_OK;
}

int colatus_cosmic_time(double a_begin, double a_end, int64_t n_steps, double H0, double Om_R,
                        double Om_M, double Om_K, double Om_L, double *t, void *stream)
{
    TraceRange trace("colatus_cosmic_time");
    if (!t || n_steps < 1)
        return COLATUS_EINVAL;
    CHECK_RC(validate_cosmology(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    CHECK_RC(get_workspace(s, ws));
    CHECK_RC(ensure(ws->coef, (size_t)n_steps * sizeof(StepCoef)));
    StepCoef *coef = static_cast<StepCoef *>(ws->coef.ptr);
    CHECK_HIP(launch_coefficients(H0, Om_R, Om_M, Om_K, Om_L, a_begin, a_end, n_steps, 0,
                                  n_steps, 0, coef, s));
    std::vector<StepCoef> hc((size_t)n_steps);
    CHECK_HIP(hipMemcpyAsync(hc.data(), coef, hc.size() * sizeof(StepCoef), hipMemcpyDeviceToHost,
                             s));
    CHECK_HIP(hipStreamSynchronize(s));
    double span = 0.0;
    for (const StepCoef &c : hc)
        span += c.dt;
    *t = span;
    return COLATUS_OK;
}

}  // extern "C"
