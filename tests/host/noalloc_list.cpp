// The allocation-free call's work list, generated on the host with the same
// functions its setup kernel runs (noalloc.hip is included whole), for
// worklist_check.cpp.
#include "noalloc.hip"

#include <vector>

// Items and blocks for N particles in one box; returns false if the list
// would not fit the fixed scratch.
bool noalloc_host_list(int64_t N, double eps, std::vector<colatus::WorkItem> &items,
                       std::vector<colatus::IntBlock> &blocks, int &max_slots)
{
    const NoAllocSizes z = noalloc_sizes(N);
    if (z.n_items > kMaxItems || z.n_blocks > kMaxBlocks)
        return false;
    items.clear();
    blocks.clear();
    for (int t = 0; t < z.n_items; ++t)
        items.push_back(noalloc_item(t, N, eps, z.P, z.n_blk, z.n_intra, z.n_pieces));
    for (int t = 0; t < z.n_blocks; ++t)
        blocks.push_back(noalloc_block(t, N, eps, z.P));
    max_slots = (int)kMaxSlots;
    return true;
}
