// Host check of the pair sweeps' work lists (no GPU calls): builds the
// library's lists with its own builder (the translation unit of the C ABI is
// included whole) for many box layouts and checks, by simulating which
// (particle, slot) each item writes:
//   * grouped symmetric lists (2x2 groups of part pairs): four items per
//     group; every unordered pair of parts of a box met by exactly one
//     item; every diagonal part covered by pieces of at most 64 targets;
//     partners (tmate: wave ^ 1, rmate: wave ^ 2) on the same part and slot;
//     every slot 0 .. n_slices - 1 of every particle written exactly once
//     (a combined partial sum counted once, by its writing wave);
//   * single-item symmetric lists: the same with P slots per particle;
//   * ordered lists: every (target, source slice) once, the slices of a box
//     tiling its sources;
//   * the allocation-free call's list (generated on the device by the
//     functions noalloc_list.cpp runs here): the grouped checks above for
//     every N it accepts (all N to 1100, then a stride), within its fixed
//     scratch, and the same items and partner pairings as the builder's
//     grouped list for that box, so the two calls give the same sums.
#include "api.cpp"

#include <cstdio>
#include <map>
#include <random>

bool noalloc_host_list(int64_t N, double eps, std::vector<colatus::WorkItem> &items,
                       std::vector<colatus::IntBlock> &blocks, int &max_slots);

namespace {

int fail(const char *what, long a = 0, long b = 0)
{
    std::printf("FAIL: %s (%ld, %ld)\n", what, a, b);
    return 1;
}

Boxes make_boxes(const std::vector<int64_t> &sizes)
{
    Boxes b;
    b.off = {0};
    for (int64_t n : sizes) {
        b.off.push_back(b.off.back() + n);
        b.eps.push_back(0.01);
        b.max_n = std::max(b.max_n, n);
    }
    return b;
}

// Simulated writes of a symmetric list (grouped or not) against its blocks.
int check_list(const Boxes &b, const WorkList &wl, bool grouped)
{
    const std::vector<int64_t> sizes = [&b] {
        std::vector<int64_t> v;
        for (size_t k = 0; k + 1 < b.off.size(); ++k)
            v.push_back(b.off[k + 1] - b.off[k]);
        return v;
    }();
    const int64_t N = b.off.back();
    const int64_t U = 256;
    const size_t G = grouped ? 4 : 1;
    if (wl.items.size() % G)
        return fail("items not a multiple of the group size", (long)wl.items.size());
    std::vector<std::vector<int32_t>> writes((size_t)N);
    std::map<std::pair<int64_t, int64_t>, int> met;
    std::vector<int> diag((size_t)N, 0);
    for (size_t g = 0; g < wl.items.size() / G; ++g)
        for (size_t e = 0; e < G; ++e) {
            const WorkItem &w = wl.items[g * G + e];
            if (w.kind < 0)
                continue;
            const int64_t o0 = b.off[w.box], o1 = b.off[w.box + 1];
            if (w.kind == 0) {
                const int64_t p = (w.i0 - o0) / U, q = (w.j0 - o0) / U;
                if (p == q || w.i1 - w.i0 > U || w.j1 - w.j0 > U || w.i1 > o1 || w.j1 > o1)
                    return fail("bad pair item", (long)p, (long)q);
                ++met[{(int64_t)w.box * (1 << 20) + std::min(p, q), std::max(p, q)}];
                const bool tm = grouped && w.tmate, rm = grouped && w.rmate;
                if (tm) {
                    const WorkItem &o = wl.items[g * G + (e ^ 1)];
                    if (o.kind != 0 || !o.tmate || o.i0 != w.i0 || o.i1 != w.i1 ||
                        o.slice != w.slice || o.box != w.box)
                        return fail("target partners differ", (long)g, (long)e);
                }
                if (rm) {
                    const WorkItem &o = wl.items[g * G + (e ^ 2)];
                    if (o.kind != 0 || !o.rmate || o.j0 != w.j0 || o.j1 != w.j1 ||
                        o.rslice != w.rslice || o.box != w.box)
                        return fail("reaction partners differ", (long)g, (long)e);
                }
                if (!tm || !(e & 1))
                    for (int64_t i = w.i0; i < w.i1; ++i)
                        writes[(size_t)i].push_back(w.slice);
                if (!rm || e < 2)
                    for (int64_t j = w.j0; j < w.j1; ++j)
                        writes[(size_t)j].push_back(w.rslice);
            } else {
                const int64_t p = (w.i0 - o0) / U;
                if (w.i1 - w.i0 > 64 || w.j0 != o0 + p * U || w.j1 != std::min(o0 + (p + 1) * U, o1))
                    return fail("bad diagonal piece", (long)w.i0, (long)w.j0);
                for (int64_t i = w.i0; i < w.i1; ++i) {
                    writes[(size_t)i].push_back(w.slice);
                    ++diag[(size_t)i];
                }
            }
        }
    size_t n_pairs = 0, want = 0;
    for (size_t bx = 0; bx < sizes.size(); ++bx) {
        const int64_t P = (sizes[bx] + U - 1) / U;
        want += (size_t)(P * (P - 1) / 2);
        for (int64_t p = 0; p < P; ++p)
            for (int64_t q = p + 1; q < P; ++q) {
                auto it = met.find({(int64_t)bx * (1 << 20) + p, q});
                if (it == met.end() || it->second != 1)
                    return fail("pair of parts not met once", (long)p, (long)q);
            }
    }
    for (auto &kv : met)
        n_pairs += (size_t)kv.second;
    if (n_pairs != want)
        return fail("extra pair items", (long)n_pairs, (long)want);
    int64_t covered = 0;
    for (const IntBlock &ib : wl.blocks) {
        if (ib.n_slices > wl.max_slices)
            return fail("n_slices above max_slices", (long)ib.n_slices, wl.max_slices);
        for (int64_t i = ib.i0; i < ib.i1; ++i) {
            if (diag[(size_t)i] != 1)
                return fail("diagonal coverage", (long)i, diag[(size_t)i]);
            std::vector<int32_t> s = writes[(size_t)i];
            std::sort(s.begin(), s.end());
            if ((int)s.size() != ib.n_slices)
                return fail("slots written", (long)i, (long)s.size());
            for (int k = 0; k < ib.n_slices; ++k)
                if (s[(size_t)k] != k)
                    return fail("slot missing or written twice", (long)i, k);
            ++covered;
        }
    }
    if (covered != N)
        return fail("blocks do not cover the particles", (long)covered, (long)N);
    return 0;
}

int check_symmetric(const std::vector<int64_t> &sizes, bool grouped)
{
    const Boxes b = make_boxes(sizes);
    TileCfg cfg{4, 64, 1, 2};
    cfg.group = grouped ? 1 : 0;
    WorkList wl;
    build_worklist(b, b.off.back(), cfg, wl);
    return check_list(b, wl, grouped);
}

// The combining structure of a grouped list: every pair item with its
// partner flags, and the diagonal pieces, as a sorted multiset.
std::vector<std::vector<int64_t>> signature(const std::vector<WorkItem> &items)
{
    std::vector<std::vector<int64_t>> sig;
    for (size_t g = 0; g < items.size() / 4; ++g)
        for (size_t e = 0; e < 4; ++e) {
            const WorkItem &w = items[g * 4 + e];
            if (w.kind < 0)
                continue;
            // a partner's part: the other target part of the group for a
            // reaction partner, the other source part for a target partner
            const int64_t tm = w.tmate ? items[g * 4 + (e ^ 1)].j0 : -1;
            const int64_t rm = w.rmate ? items[g * 4 + (e ^ 2)].i0 : -1;
            sig.push_back({w.kind, w.i0, w.i1, w.j0, w.j1, w.slice, w.rslice, tm, rm});
        }
    std::sort(sig.begin(), sig.end());
    return sig;
}

int check_noalloc(int64_t N)
{
    std::vector<WorkItem> items;
    std::vector<IntBlock> blocks;
    int max_slots = 0;
    if (!noalloc_host_list(N, 0.01, items, blocks, max_slots))
        return fail("allocation-free list beyond its scratch", (long)N);
    Boxes b = make_boxes({N});
    WorkList wl;
    wl.items = items;
    wl.blocks = blocks;
    wl.max_slices = max_slots;
    if (check_list(b, wl, true))
        return fail("allocation-free list", (long)N);
    WorkList ref;
    TileCfg cfg{4, 64, 1, 2};
    cfg.group = 1;
    build_worklist(b, N, cfg, ref);
    if (signature(items) != signature(ref.items))
        return fail("allocation-free list differs from the builder's", (long)N);
    for (size_t k = 0; k < blocks.size(); ++k)
        if (blocks[k].i0 != ref.blocks[k].i0 || blocks[k].i1 != ref.blocks[k].i1 ||
            blocks[k].n_slices != ref.blocks[k].n_slices)
            return fail("allocation-free blocks differ from the builder's", (long)N, (long)k);
    return 0;
}

int check_ordered(const std::vector<int64_t> &sizes, int R, int tpb, int slices)
{
    const Boxes b = make_boxes(sizes);
    const int64_t N = b.off.back();
    const TileCfg cfg{R, tpb, slices, 0};
    WorkList wl;
    build_worklist(b, N, cfg, wl);
    std::map<std::pair<int64_t, int32_t>, int> seen;  // (target block start, slice)
    std::vector<int64_t> src((size_t)N, 0);
    for (const WorkItem &w : wl.items) {
        const int64_t o0 = b.off[w.box], o1 = b.off[w.box + 1];
        if (w.i0 < o0 || w.i1 > o1 || w.j0 < o0 || w.j1 > o1 || w.i1 - w.i0 > R * tpb)
            return fail("ordered item outside its box", (long)w.i0, (long)w.j0);
        ++seen[{w.i0, w.slice}];
        if (w.i0 == o0)
            for (int64_t j = w.j0; j < w.j1; ++j)
                ++src[(size_t)j];
    }
    for (auto &kv : seen)
        if (kv.second != 1)
            return fail("(target block, slice) twice", (long)kv.first.first, kv.first.second);
    for (int64_t j = 0; j < N; ++j)
        if (src[(size_t)j] != 1)
            return fail("source slices do not tile the box", (long)j, (long)src[(size_t)j]);
    for (const IntBlock &ib : wl.blocks)
        for (int32_t s = 0; s < ib.n_slices; ++s)
            if (!seen.count({b.off[ib.box] + ((ib.i0 - b.off[ib.box]) / (R * tpb)) * (R * tpb), s}))
                return fail("slot never written", (long)ib.i0, s);
    return 0;
}

}  // namespace

int main()
{
    int bad = 0, cases = 0;
    const std::vector<int64_t> singles = {1,    2,    63,   64,   65,    100,   255,  256,
                                          257,  511,  512,  513,  700,   768,   769,  1000,
                                          1024, 1025, 1300, 4096, 30000, 32768, 65536};
    for (int64_t n : singles)
        for (bool grouped : {true, false}) {
            bad |= check_symmetric({n}, grouped);
            ++cases;
        }
    std::mt19937_64 rng(7);
    for (int t = 0; t < 20; ++t) {
        std::vector<int64_t> sz;
        const int nb = 1 + (int)(rng() % 40);
        for (int k = 0; k < nb; ++k)
            sz.push_back(1 + (int64_t)(rng() % 9000));
        for (bool grouped : {true, false}) {
            bad |= check_symmetric(sz, grouped);
            ++cases;
        }
        bad |= check_ordered(sz, 2, 128, 1 + (int)(rng() % 8));
        ++cases;
    }
    std::vector<int64_t> ens;
    for (int k = 0; k < 256; ++k)
        ens.push_back(512 + (int64_t)((k * 7919) % 7681));
    bad |= check_symmetric(ens, true);
    bad |= check_symmetric(ens, false);
    bad |= check_ordered(ens, 4, 256, 5);
    cases += 3;
    bad |= check_ordered({32768}, 1, 256, 64);
    bad |= check_ordered({1000, 3, 70000}, 4, 128, 9);
    cases += 2;
    for (int64_t n = 1; n <= 16384 && !bad; n += (n < 1100 ? 1 : 97)) {
        bad |= check_noalloc(n);
        ++cases;
    }
    bad |= check_noalloc(16384);
    ++cases;
    std::printf(bad ? "FAILED (%d cases)\n" : "all ok (%d cases)\n", cases);
    return bad;
}
