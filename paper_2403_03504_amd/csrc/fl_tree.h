// Quadtree, neighbour/interaction lists and expansion storage shared by the
// FMM kernels.  Layout (all structure-of-arrays in HBM, sized by provable
// capacities so no kernel can overflow and nothing is read back to the host
// inside an iteration):
//
//   systems     K independent systems (components) handled together: system
//               k owns nodes [coff[k], coff[k+1]); every system has its own
//               root square and its own tree (a forest), and no list ever
//               joins two systems.  Reductions run over tiles of SEG_TILE
//               nodes that never straddle two systems, so a system's results
//               do not depend on what else is in the batch.
//
//   part[n]     float4 (x, y, mass, original index as int bits), Morton order
//   skey[n]     uint32 Morton keys, sorted
//   cells       depth-first pre-order (sorted by (begin, level)); per cell:
//               level, ixy (ix | iy << 16), begin, end, parent, child (int4,
//               -1 = empty quadrant), leafidx (-1 for internal cells), skip
//               (first cell after its subtree: a subtree is [id, skip))
//   leaves      leaf_cell[nleaves] in Morton order (a leaf's index = the
//               index of its first particle among the "cell-start" particles)
//   hash        (system, level, ix, iy) -> cell id, open addressing,
//               epoch-tagged (cleared only when the epoch wraps)
//   lists       V (M2L) and X (P2L) per cell; U (P2P) and W (M2P) per leaf;
//               offsets are packed int64 pairs (lo = first list, hi = second);
//               U is stored as the leaves' particle ranges, sorted and with
//               touching ranges merged (a leaf's 3x3 block is a few Morton runs)
//   M, Lp       outgoing / partial incoming expansions, (p+1) float2 per
//               cell, scaled by the cell width (coefficient k of an outgoing
//               expansion holds a_k / w^k, of an incoming one b_k * w^k)
#pragma once

#include <vector>

#include "fl_common.h"

namespace fl {

constexpr int SEG_TILE = 2048;

// K independent systems over n nodes (device arrays, see the layout notes).
struct Segs {
    int K = 1, n = 0;
    const int32_t *coff = nullptr;      // [K+1] first node of each system
    const int32_t *ncomp = nullptr;     // [n] system of each node; null when K == 1
    const int2 *tiles = nullptr;        // [ntiles] (system, first node), SEG_TILE nodes at most
    const int32_t *tile_off = nullptr;  // [K+1] first tile of each system
    int ntiles = 0;
    int cbits = 0;                      // bits of the system id in hash keys (0 when K == 1)
    RsSegs sort;                        // system-aligned sort tiles (K > 1 only)
};

// One system of n nodes (device arrays cached per context).
Segs segs_single(fl_ctx *c, int32_t n);
// K systems with host offsets coff[0..K] (coff[0] = 0, strictly increasing);
// uploads to workspace buffers named after `tag` and synchronises.
Segs make_segs(fl_ctx *c, const std::vector<int32_t> &coff, const char *tag);

struct TreeBufs {
    int n = 0, bits = 16, leaf = 64;
    Segs s;
    int64_t cells_cap = 0, leaves_cap = 0, hash_cap = 0;
    double *root = nullptr;      // [4 K] per system: xmin, ymin, L, S
    int32_t *ccomp = nullptr;    // [cells_cap] system of each cell (null when K == 1)
    float4 *part = nullptr;      // [n]
    uint32_t *skey = nullptr;    // [n]
    int32_t *lvl = nullptr;      // [cells_cap]
    uint32_t *ixy = nullptr;
    int32_t *beg = nullptr, *end = nullptr, *par = nullptr, *leafidx = nullptr;
    int32_t *skip = nullptr;       // [cells_cap] first cell after the cell's subtree (pre-order)
    int4 *child = nullptr;
    int32_t *leaf_cell = nullptr;  // [leaves_cap]
    uint64_t *start_key = nullptr;  // system << 32 | Morton key of each cell-start particle
    int32_t *start_pos = nullptr, *start_D = nullptr;
    int32_t *counts = nullptr;     // [0] cells, [1] leaves, [2] max level, [3] error bits
    uint64_t *hslot = nullptr;     // 2 words per slot: key, cell id (one 16-byte read per probe)
    uint32_t *epoch = nullptr;     // device epoch of the hash table
    int64_t *off2 = nullptr;       // per particle (cells, starts) packed prefix
    int32_t *pack = nullptr;       // per particle (D+1) | lambda << 8
};

struct ListBufs {
    int64_t v_cap = 0, x_cap = 0, u_cap = 0, w_cap = 0;
    int64_t *offVX = nullptr;  // [cells_cap + 1]
    int64_t *offUW = nullptr;  // [leaves_cap + 1]
    int32_t *V = nullptr, *X = nullptr, *W = nullptr;
    int2 *U = nullptr;         // near-field particle ranges [begin, end), sorted and merged
    int32_t *nU = nullptr;     // [leaves_cap] merged range count of each leaf
    unsigned long long *block_pairs = nullptr;  // near-field pair counts per fill block
    int fill_blocks = 0;
};

// Device view used by the kernels.
struct TreeView {
    int n, bits, leaf, K, cbits;
    const int32_t *coff;
    const int32_t *ccomp;
    const double *root;
    const float4 *part;
    const int32_t *lvl;
    const uint32_t *ixy;
    const int32_t *beg, *end, *par, *leafidx, *skip;
    const int4 *child;
    const int32_t *leaf_cell;
    const int32_t *counts;
    const uint64_t *hslot;
    const uint32_t *epoch;
    int64_t hash_cap;
};

inline TreeView view(const TreeBufs &t)
{
    return TreeView{t.n,       t.bits,  t.leaf,      t.s.K,    t.s.cbits, t.s.coff, t.ccomp,
                    t.root,    t.part,  t.lvl,       t.ixy,    t.beg,     t.end,    t.par,
                    t.leafidx, t.skip,  t.child,     t.leaf_cell, t.counts, t.hslot,
                    t.epoch,   t.hash_cap};
}

// Capacities that no input can exceed (see the capacity notes in fl_tree.hip).
int64_t cells_capacity(int64_t n, int leaf, int bits, int K = 1);

// Per system: bbox -> Morton keys; then one stable sort by (system, key) ->
// sorted particles -> forest.  deg may be null (unit masses).  All on the
// context stream, no host synchronisation.
// xy_out (optional, n float2): the (x, y) pairs as well, for the attraction.
// Extrema of the positions per tile, already known (the ForceAtlas2 update
// writes them for the next iteration): `per` float4 (min x, max x, min y,
// max y) per tile of the Segs, in tile order.  Null: computed by the build.
struct BBoxIn {
    const float4 *part = nullptr;
    int per = 1;
};
void build_tree(fl_ctx *c, TreeBufs &t, const Segs &s, const float *x, const float *y, const int32_t *deg, int bits,
                int leaf, float2 *xy_out = nullptr, BBoxIn bb = {});
// lanes: lanes per cell of the list kernels, 1 or 8 (the same lists either way)
void build_lists(fl_ctx *c, const TreeBufs &t, ListBufs &L, int lanes);
// The lists' statistics (counts, near pairs) into the context's counters;
// nothing of the passes reads them, so the caller launches this off the
// critical path (on a branch stream `s`, or the context's stream if null).
void lists_stats(fl_ctx *c, const TreeBufs &t, const ListBufs &L, hipStream_t s = nullptr);
// lanes per cell when the caller leaves the choice open (0)
int default_list_lanes(int64_t n);
// Deepest level of the last tree into the statistics block.
void tree_max_level(fl_ctx *c);
// Sticky capacity-guard bits of the tree/list kernels (synchronises).
int32_t tree_error_bits(fl_ctx *c, bool clear);

void fill_i32(fl_ctx *c, int32_t *p, int64_t n, int32_t v);
int32_t read_i32(fl_ctx *c, const int32_t *dp);
int64_t read_i64(fl_ctx *c, const int64_t *dp);

// ---- geometry helpers (device) ---------------------------------------------
__device__ __forceinline__ int cell_ix(uint32_t v) { return (int)(v & 0xFFFFu); }
__device__ __forceinline__ int cell_iy(uint32_t v) { return (int)(v >> 16); }

__device__ __forceinline__ bool is_leaf4(int4 ch) { return ch.x < 0 && ch.y < 0 && ch.z < 0 && ch.w < 0; }

// Closed squares of two distinct, non-nested cells touch.
__device__ __forceinline__ bool cells_adjacent(int la, uint32_t a, int lb, uint32_t b)
{
    int L = la > lb ? la : lb;
    int sa = 1 << (L - la), sb = 1 << (L - lb);
    int ax0 = cell_ix(a) * sa, ay0 = cell_iy(a) * sa;
    int bx0 = cell_ix(b) * sb, by0 = cell_iy(b) * sb;
    return ax0 <= bx0 + sb && bx0 <= ax0 + sa && ay0 <= by0 + sb && by0 <= ay0 + sa;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ull;
    z ^= z >> 33;
    return z;
}

__device__ __forceinline__ int cell_comp(const TreeView &t, int c) { return t.ccomp ? t.ccomp[c] : 0; }

// key bits: iy [0,16) ix [16,32) level [32,37) system [37,37+cbits) epoch above
constexpr int HASH_BASE_BITS = 37;
constexpr int HASH_TAG_BITS = 27;  // system + epoch bits

__device__ __forceinline__ uint64_t hash_key(int comp, int level, int ix, int iy)
{
    return ((uint64_t)(uint32_t)comp << HASH_BASE_BITS) | ((uint64_t)level << 32) | ((uint64_t)(uint32_t)ix << 16) |
           (uint64_t)(uint32_t)iy;
}

__device__ __forceinline__ int64_t hash_size(int ncells, int64_t cap)
{
    int64_t h = 64;
    while (h < 2 * (int64_t)ncells) h <<= 1;
    return h < cap ? h : cap;
}

// cell id of region (comp, level, ix, iy), or -1 if no cell of that exact region
__device__ __forceinline__ int hash_find(const TreeView &t, int64_t H, uint64_t ep, int comp, int level, int ix,
                                         int iy)
{
    const int sh = HASH_BASE_BITS + t.cbits;
    uint64_t k = hash_key(comp, level, ix, iy) | (ep << sh);
    int64_t h = (int64_t)(mix64(k & ((1ull << sh) - 1)) & (uint64_t)(H - 1));
    for (int64_t probe = 0; probe < H; ++probe) {
        const ulonglong2 e = reinterpret_cast<const ulonglong2 *>(t.hslot)[h];  // key and cell id together
        if ((e.x >> sh) != ep) return -1;
        if (e.x == k) return (int)e.y;
        h = (h + 1) & (H - 1);
    }
    return -1;
}

// Deepest cell on the path to region (comp, level, ix, iy): the region's own
// cell, else the leaf that covers it; -1 when the region holds no particle.
__device__ __forceinline__ int lookup_region(const TreeView &t, int64_t H, uint64_t ep, int comp, int level, int ix,
                                             int iy)
{
    for (int l = level; l >= 0; --l, ix >>= 1, iy >>= 1) {
        int id = hash_find(t, H, ep, comp, l, ix, iy);
        if (id < 0) continue;
        if (l == level) return id;
        return is_leaf4(t.child[id]) ? id : -1;
    }
    return -1;
}

}  // namespace fl
