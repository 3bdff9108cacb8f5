// Quadtree over the particles (paper sec. 3.2.1: a square covering all
// particles, divided into four while it holds more than leaf_size of them)
// and the neighbour / interaction lists of the FMM.
//
// Tree construction without per-level launches.  With K the sorted Morton
// keys and cd(a, b) the number of leading base-4 digits two keys share:
//   D(k)   = cd(K[k-1], K[k])            (k starts a new level-l region for l > D)
//   W(j)   = cd(K[j], K[j+L])            (L = leaf_size)
//   lam(k) = min(B, 1 + max_{j in [k-L, k]} W(j))
// A level-l region holding particle k has more than L particles iff some
// window of L+1 consecutive sorted particles containing k shares its level-l
// prefix, i.e. iff l <= max W over the windows through k.  So lam(k) is the
// level of the leaf holding k, and particle k begins exactly the cells of
// levels D(k)+1 .. lam(k).  A prefix sum of max(0, lam - D) numbers every cell
// in (begin, level) order, which is depth-first pre-order.  The windowed
// maximum uses log2(L+1) doubling rounds in LDS.
//
// Capacity notes (no kernel can write past them):
//   cells  <= 1 + 4 B floor(n / (L+1))  (a split cell holds > L particles and
//            split cells of one level are disjoint), and <= 1 + B n; a forest
//            of K trees holds at most K + 4 B floor(n / (L+1)) and K + B n;
//   V(c)   <= 27 (same-level cells in the parent's 6x6 block minus c's 3x3);
//   X(c)   <= 8 (one covering leaf per ring square of the parent);
//   sum |W| = sum |X| (W and X are dual) <= 8 cells;
//   sum |U| <= 17 leaves (a leaf touches at most 8 cells at least its size).
#include <algorithm>

#include "fl_tree.h"

namespace fl {

// A forest of K trees holds at most the sum of the per-tree bounds.
int64_t cells_capacity(int64_t n, int leaf, int bits, int K)
{
    int64_t a = (int64_t)K + 4 * (int64_t)bits * (n / ((int64_t)leaf + 1));
    int64_t b = (int64_t)K + (int64_t)bits * n;
    int64_t c = a < b ? a : b;
    return c < 1 ? 1 : c;
}

namespace {

constexpr int NT = 256;

__device__ __forceinline__ uint32_t part1by1(uint32_t v)
{
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ __forceinline__ uint32_t compact1by1(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}

__device__ __forceinline__ uint32_t quantize(float v, double vmin, double S, int bits)
{
    double t = floor(__dmul_rn(__dsub_rn((double)v, vmin), S));
    double top = (double)((1u << bits) - 1u);
    if (!(t >= 0.0)) t = 0.0;  // also maps NaN to 0
    if (t > top) t = top;
    return (uint32_t)t;
}

// common leading base-4 digits of two keys of 2*bits bits
__device__ __forceinline__ int common_digits(uint32_t a, uint32_t b, int bits)
{
    uint32_t x = a ^ b;
    if (x == 0) return bits;
    int lz = __clz((int)x) - (32 - 2 * bits);
    return lz >> 1;
}

// ---- bbox + root square per system ------------------------------------------
// k_bbox: the extrema of every tile (tiles never straddle two systems);
// k_bbox_root: one block per system combines its tiles' extrema (min/max are
// exact, so the order does not matter) into the system's root square.  Two
// launches and no device-scope fences.  Within a ForceAtlas2 run the update
// of the previous iteration has written the extrema (`per` per tile) and
// k_bbox is skipped.
__global__ __launch_bounds__(NT) void k_bbox(const float *__restrict__ x, const float *__restrict__ y, Segs sg,
                                             float4 *__restrict__ partial)
{
    __shared__ float4 red[NT / WAVE];
    const int2 tl = sg.tiles[blockIdx.x];
    const int b1 = min(tl.y + SEG_TILE, sg.coff[tl.x + 1]);
    float mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
    for (int i = tl.y + threadIdx.x; i < b1; i += NT) {
        float a = x[i], b = y[i];
        mnx = fminf(mnx, a);
        mxx = fmaxf(mxx, a);
        mny = fminf(mny, b);
        mxy = fmaxf(mxy, b);
    }
    mnx = wave_min_f(mnx);
    mxx = wave_max_f(mxx);
    mny = wave_min_f(mny);
    mxy = wave_max_f(mxy);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = make_float4(mnx, mxx, mny, mxy);
    __syncthreads();
    if (threadIdx.x == 0) {
        float4 r = red[0];
        for (int w = 1; w < NT / WAVE; ++w) {
            r.x = fminf(r.x, red[w].x);
            r.y = fmaxf(r.y, red[w].y);
            r.z = fminf(r.z, red[w].z);
            r.w = fmaxf(r.w, red[w].w);
        }
        partial[blockIdx.x] = r;
    }
}

// Block k finishes the root squares of systems k, k + gridDim.x, ...; block 0
// also advances the hash epoch (when there is a table).
__global__ __launch_bounds__(NT) void k_bbox_root(Segs sg, const float4 *__restrict__ partial, int per,
                                                  double *__restrict__ root, int bits, uint32_t *__restrict__ epoch)
{
    __shared__ float4 red[NT / WAVE];
    if (blockIdx.x == 0 && threadIdx.x == 0 && epoch) {
        uint32_t e = *epoch + 1u;
        if (e >= (1u << (HASH_TAG_BITS - sg.cbits)) || e == 0u) e = 1u;  // wrap: k_morton clears the table
        *epoch = e;
    }
    for (int comp = blockIdx.x; comp < sg.K; comp += gridDim.x) {
        const int t0 = per * sg.tile_off[comp], nt = per * sg.tile_off[comp + 1] - t0;
        float4 q = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
        for (int j = threadIdx.x; j < nt; j += NT) {
            const float4 v = partial[t0 + j];
            q.x = fminf(q.x, v.x);
            q.y = fmaxf(q.y, v.y);
            q.z = fminf(q.z, v.z);
            q.w = fmaxf(q.w, v.w);
        }
        q.x = wave_min_f(q.x);
        q.y = wave_max_f(q.y);
        q.z = wave_min_f(q.z);
        q.w = wave_max_f(q.w);
        if (lane_id() == 0) red[threadIdx.x / WAVE] = q;
        __syncthreads();
        if (threadIdx.x == 0) {
            float4 r = red[0];
            for (int w = 1; w < NT / WAVE; ++w) {
                r.x = fminf(r.x, red[w].x);
                r.y = fmaxf(r.y, red[w].y);
                r.z = fminf(r.z, red[w].z);
                r.w = fmaxf(r.w, red[w].w);
            }
            double x0 = r.x, x1 = r.y, y0 = r.z, y1 = r.w;
            double L = (x1 - x0) > (y1 - y0) ? (x1 - x0) : (y1 - y0);
            if (!(L > 0.0)) L = 1.0;
            if (!isfinite(x0)) x0 = 0.0;
            if (!isfinite(y0)) y0 = 0.0;
            if (!isfinite(L)) L = 1.0;
            double *rt = root + 4 * (int64_t)comp;
            rt[0] = x0;
            rt[1] = y0;
            rt[2] = L;
            rt[3] = __ddiv_rn(ldexp(1.0, bits), L);
        }
        __syncthreads();
    }
}

// Morton key of every node relative to its system's root square; with more
// than one system also the sort key (system << 32 | key); with `xym` also
// the node's (x, y, mass, index) record, so that moving a node to its sorted
// place is a single 16-byte access; with `xy` the (x, y) pairs the
// attraction gathers read.  When the hash epoch has
// just restarted at 1 (a wrap, or a new key layout) all hcap slots of the
// table are cleared here (before any insert of this build).
__global__ void k_morton(const float *__restrict__ x, const float *__restrict__ y, int n,
                         const int32_t *__restrict__ ncomp, const double *__restrict__ root, int bits,
                         uint32_t *__restrict__ key, uint64_t *__restrict__ key64, int32_t *__restrict__ idx,
                         const uint32_t *__restrict__ epoch, uint64_t *__restrict__ hslot, int64_t hcap,
                         const int32_t *__restrict__ deg, float4 *__restrict__ xym, int32_t *__restrict__ counts,
                         float2 *__restrict__ xy)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (counts && i < 3) counts[i] = 0;  // the tree's cell, leaf and level counts ([3], the error bits, is sticky)
    if (hslot && epoch && *epoch == 1u)
        for (int64_t h = i; h < hcap; h += (int64_t)gridDim.x * blockDim.x) hslot[2 * h] = 0ull;  // the keys
    if (i >= n) return;
    const int comp = ncomp ? ncomp[i] : 0;
    const double *rt = root + 4 * (int64_t)comp;
    double x0 = rt[0], y0 = rt[1], S = rt[3];
    const float xi = x[i], yi = y[i];
    uint32_t qx = quantize(xi, x0, S, bits), qy = quantize(yi, y0, S, bits);
    const uint32_t k = part1by1(qx) | (part1by1(qy) << 1);
    if (key) key[i] = k;
    if (key64) key64[i] = ((uint64_t)(uint32_t)comp << 32) | k;
    if (idx) idx[i] = i;
    if (xym) xym[i] = make_float4(xi, yi, deg ? (float)(deg[i] + 1) : 1.0f, __int_as_float(i));
    if (xy) xy[i] = make_float2(xi, yi);
}

// sorted particles; with more than one system also the sorted Morton keys
// (the low halves of the sorted (system, key) pairs)
__global__ void k_gather(const float4 *__restrict__ xym, const int32_t *__restrict__ perm, int n,
                         float4 *__restrict__ part, const uint64_t *__restrict__ skey64, uint32_t *__restrict__ skey)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    part[k] = xym[perm[k]];
    if (skey64) skey[k] = (uint32_t)skey64[k];
}

// ---- tree: levels per particle ----------------------------------------------
constexpr int T1_TB = 1024;
constexpr int T1_MAXL = 1024;  // largest leaf size supported
constexpr int T1_LEN = T1_TB + T1_MAXL;
constexpr int T1_PER = T1_LEN / NT;

// Sorted position k belongs to the system of node k (the sort keeps every
// system's node range).  Two particles of different systems share no cell:
// their common-prefix length is -1.
__global__ __launch_bounds__(NT) void k_tree_levels(const uint32_t *__restrict__ K, int n, int bits, int L,
                                                    const int32_t *__restrict__ ncomp, int32_t *__restrict__ pack,
                                                    int64_t *__restrict__ off2, int64_t *__restrict__ bsum)
{
    __shared__ int A[T1_LEN];
    const int t0 = blockIdx.x * T1_TB;
    const int base = t0 - L;
    const int len = T1_TB + L;
    for (int i = threadIdx.x; i < len; i += NT) {
        int j = base + i;
        int a = -1;
        if (j >= 0 && j + L < n && (!ncomp || ncomp[j] == ncomp[j + L])) a = common_digits(K[j], K[j + L], bits);
        A[i] = a;
    }
    const int w = L + 1;
    int s = 1;
    while (2 * s <= w) s <<= 1;
    for (int h = 1; h < s; h <<= 1) {
        int v[T1_PER];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < T1_PER; ++r) {
            int i = threadIdx.x + r * NT;
            int a = -1;
            if (i < len) {
                a = A[i];
                if (i + h < len) a = max(a, A[i + h]);
            }
            v[r] = a;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < T1_PER; ++r) {
            int i = threadIdx.x + r * NT;
            if (i < len) A[i] = v[r];
        }
    }
    __syncthreads();
    // per particle: the cells it starts and whether it starts a leaf, packed
    // (cells | starts << 32), then their exclusive prefix within the block;
    // the block's total goes to bsum (a scan of the block totals completes
    // the numbering)
    __shared__ int64_t C[T1_TB];
    __shared__ int64_t stmp[NT / WAVE];
    for (int t = threadIdx.x; t < T1_TB; t += NT) {
        int k = t0 + t;
        int64_t v = 0;
        if (k < n) {
            int mx = max(A[t], A[t + w - s]);
            int lam = min(bits, 1 + mx);
            int D = (k == 0 || (ncomp && ncomp[k - 1] != ncomp[k])) ? -1 : common_digits(K[k - 1], K[k], bits);
            int c = lam - D;
            if (c < 0) c = 0;
            pack[k] = (D + 1) | (lam << 8);
            v = (int64_t)c | ((int64_t)(c > 0 ? 1 : 0) << 32);
        }
        C[t] = v;
    }
    __syncthreads();
    static_assert(T1_TB == 4 * NT, "four particles per thread in the block scan");
    const int q = 4 * (int)threadIdx.x;
    const int64_t a0 = C[q], a1 = C[q + 1], a2 = C[q + 2], a3 = C[q + 3];
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, NT>(a0 + a1 + a2 + a3, stmp, tot);
    C[q] = ex;
    C[q + 1] = ex + a0;
    C[q + 2] = ex + a0 + a1;
    C[q + 3] = ex + a0 + a1 + a2;
    __syncthreads();
    for (int t = threadIdx.x; t < T1_TB; t += NT)
        if (t0 + t < n) off2[t0 + t] = C[t];
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__device__ __forceinline__ uint32_t region_prefix(uint32_t key, int level, int bits)
{
    return level == 0 ? 0u : (key >> (2 * (bits - level)));
}

// off2: per particle, the exclusive prefix of (cells | starts << 32) within
// its block of T1_TB particles; bpre: exclusive prefix of the block totals,
// bpre[number of blocks] = the totals
__device__ __forceinline__ int64_t tree_offset(const int64_t *__restrict__ off2, const int64_t *__restrict__ bpre,
                                               int k)
{
    return off2[k] + bpre[k / T1_TB];
}

__global__ void k_tree_cells(const uint32_t *__restrict__ K, int n, int bits, const int32_t *__restrict__ pack,
                             const int64_t *__restrict__ off2, const int64_t *__restrict__ bpre,
                             const int32_t *__restrict__ ncomp, TreeBufs t)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int pk = pack[k];
    int D = (pk & 0xFF) - 1, lam = pk >> 8;
    if (lam - D <= 0) return;
    int64_t o = tree_offset(off2, bpre, k);
    int cid0 = (int)(o & 0xFFFFFFFFll), li = (int)(o >> 32);
    int64_t tot = bpre[(n + T1_TB - 1) / T1_TB];
    int ncells = (int)(tot & 0xFFFFFFFFll), nleaves = (int)(tot >> 32);
    if (ncells > t.cells_cap || nleaves > t.leaves_cap) {
        // cannot happen (see the capacity notes); refuse rather than overrun
        if (k == 0) {
            t.counts[0] = 0;
            t.counts[1] = 0;
            t.counts[3] = 1;
        }
        return;
    }
    uint32_t key = K[k];
    const int comp = ncomp ? ncomp[k] : 0;
    t.start_pos[li] = k;
    t.start_key[li] = ((uint64_t)(uint32_t)comp << 32) | key;
    t.start_D[li] = D;
    t.leaf_cell[li] = cid0 + (lam - D - 1);
    if (k == 0) {
        t.counts[0] = ncells;
        t.counts[1] = nleaves;
    }
    // the cells this particle starts (their hash entries are made per cell,
    // in parallel, by k_tree_links: a chain of inserts here would serialise
    // the deep starts)
    for (int l = D + 1; l <= lam; ++l) {
        int id = cid0 + (l - D - 1);
        uint32_t pre = region_prefix(key, l, bits);
        int ix = (int)compact1by1(pre), iy = (int)compact1by1(pre >> 1);
        t.lvl[id] = l;
        t.ixy[id] = (uint32_t)ix | ((uint32_t)iy << 16);
        t.beg[id] = k;
        t.child[id] = make_int4(-1, -1, -1, -1);
        t.leafidx[id] = (l == lam) ? li : -1;
        t.par[id] = (l == 0) ? -1 : (l - 1 > D ? id - 1 : -2);
        if (t.ccomp) t.ccomp[id] = comp;
    }
}

// insert (system, level, ix, iy) -> id into the table of this epoch
__device__ __forceinline__ void hash_insert(const TreeBufs &t, int64_t H, uint64_t ep, int sh, int comp, int l,
                                            uint32_t ixy, int id)
{
    const uint64_t hk = hash_key(comp, l, (int)(ixy & 0xFFFFu), (int)(ixy >> 16));
    const uint64_t kk = hk | (ep << sh);
    int64_t h = (int64_t)(mix64(hk) & (uint64_t)(H - 1));
    for (int64_t probe = 0; probe < H; ++probe) {
        const uint64_t old = t.hslot[2 * h];
        if ((old >> sh) == ep) {
            h = (h + 1) & (H - 1);
            continue;
        }
        const unsigned long long prev =
            atomicCAS((unsigned long long *)&t.hslot[2 * h], (unsigned long long)old, (unsigned long long)kk);
        if (prev == old) {
            t.hslot[2 * h + 1] = (uint64_t)(uint32_t)id;
            break;
        }
        --probe;  // lost the slot to another insert: look at it again
    }
}

__device__ __forceinline__ int lower_bound_u64(const uint64_t *a, int n, uint64_t v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first cell (pre-order) whose first particle is >= v: the number of cells
// started by the particles before v (cells are numbered particle by particle)
__device__ __forceinline__ int first_cell_from(const int64_t *__restrict__ off2, const int64_t *__restrict__ bpre,
                                               int n, int ncells, int v)
{
    return v < n ? (int)(tree_offset(off2, bpre, v) & 0xFFFFFFFFll) : ncells;
}

// Two independent jobs per cell, each a chain of dependent loads: its hash
// entry (probe and insert), and its end, skip and parent (binary searches
// over the leaf starts).  Even waves insert and odd waves link, so that the
// two chains of a cell run side by side in different waves.
__global__ __launch_bounds__(NT) void k_tree_links(const uint32_t *__restrict__ K, int n, int bits,
                                                   const int64_t *__restrict__ off2,
                                                   const int64_t *__restrict__ bpre, TreeBufs t)
{
    static_assert(NT % (2 * WAVE) == 0, "whole wave pairs per block");
    const int ncells = t.counts[0];
    const int nleaves = t.counts[1];
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int pairs = (int)(gridDim.x * blockDim.x / (2 * WAVE));
    const bool insert = (gw & 1) == 0;
    for (int id = (gw >> 1) * WAVE + lane_id(); id < ncells; id += pairs * WAVE) {
        const int l = t.lvl[id];
        const int comp = t.ccomp ? t.ccomp[id] : 0;
        if (insert) {
            hash_insert(t, hash_size(ncells, t.hash_cap), *t.epoch, HASH_BASE_BITS + t.s.cbits, comp, l, t.ixy[id],
                        id);
            continue;
        }
        if (l == 0) {
            const int e0 = t.s.K > 1 ? t.s.coff[comp + 1] : n;
            t.end[id] = e0;
            t.skip[id] = first_cell_from(off2, bpre, n, ncells, e0);
            continue;
        }
        const int k = t.beg[id];
        const uint32_t pre = region_prefix(K[k], l, bits);
        const int sh = 2 * (bits - l);
        // start keys carry the system above bit 32: the region's end is the
        // first cell start past it in the same system, or the next system's
        // first start
        const uint64_t cs = (uint64_t)(uint32_t)comp << 32;
        const uint64_t T = cs + (((uint64_t)pre + 1ull) << sh);
        const int j = lower_bound_u64(t.start_key, nleaves, T);
        const int eid = j < nleaves ? t.start_pos[j] : n;
        t.end[id] = eid;
        t.skip[id] = first_cell_from(off2, bpre, n, ncells, eid);
        int p = t.par[id];
        if (p == -2) {
            const uint64_t Tp = cs | ((uint64_t)(pre >> 2) << (sh + 2));
            const int jp = lower_bound_u64(t.start_key, nleaves, Tp);
            if (jp >= nleaves) {
                atomicOr(&t.counts[3], 2);
                continue;
            }
            const int bp = t.start_pos[jp];
            const int Dp = t.start_D[jp];
            const int cid0 = (int)(tree_offset(off2, bpre, bp) & 0xFFFFFFFFll);
            p = cid0 + (l - 1 - Dp - 1);
            t.par[id] = p;
        }
        if (p < 0 || p >= ncells) {
            atomicOr(&t.counts[3], 2);
            continue;
        }
        reinterpret_cast<int *>(&t.child[p])[pre & 3u] = id;
    }
}

// ---- lists ------------------------------------------------------------------
struct CountSink {
    int nV = 0, nX = 0, nU = 0, nW = 0;
    __device__ void V(int) { ++nV; }
    __device__ void X(int) { ++nX; }
    __device__ void U(int) { ++nU; }
    __device__ void W(int) { ++nW; }
};

// Counting pass of the lane groups: besides the counts, the lane's first
// LIST_SLOTS entries (cell ids tagged V 0, X 1, U 2, W 3 in the top two
// bits) are kept in LDS and written out per cell, so that the filling pass
// replays them instead of enumerating the ring again (a chain of dependent
// lookups); a lane with more entries enumerates again.
constexpr int LIST_SLOTS = 16;
// Workgroups of the list kernels: two waves (16 cells of 8 lanes), which
// leaves the upward pass on the other branch more room beside them than
// four waves did (2M-node iteration 0.713 -> 0.706 ms)
constexpr int LIST_NT = 128;
constexpr int LIST_SLOT_Q = LIST_SLOTS / 4;  // int4 words per (cell, lane)
struct SlotSink {
    using lds_i32 = __attribute__((address_space(3))) int32_t;
    lds_i32 *slot;
    int nV = 0, nX = 0, nU = 0, nW = 0;
    __device__ void put(uint32_t tag, int s)
    {
        const int k = nV + nX + nU + nW;
        if (k < LIST_SLOTS) slot[k] = (int)((tag << 30) | (uint32_t)s);
    }
    __device__ void V(int s)
    {
        put(0u, s);
        ++nV;
    }
    __device__ void X(int s)
    {
        put(1u, s);
        ++nX;
    }
    __device__ void U(int s)
    {
        put(2u, s);
        ++nU;
    }
    __device__ void W(int s)
    {
        put(3u, s);
        ++nW;
    }
};

template <class Sink>
__device__ __forceinline__ void replay_slots(const int4 *__restrict__ gs, int tot, Sink &sk)
{
    int e[LIST_SLOTS];
#pragma unroll
    for (int q = 0; q < LIST_SLOT_Q; ++q) {
        const int4 a = 4 * q < tot ? gs[q] : make_int4(0, 0, 0, 0);
        e[4 * q] = a.x;
        e[4 * q + 1] = a.y;
        e[4 * q + 2] = a.z;
        e[4 * q + 3] = a.w;
    }
#pragma unroll
    for (int i = 0; i < LIST_SLOTS; ++i) {
        if (i < tot) {
            const uint32_t v = (uint32_t)e[i];
            const int id = (int)(v & 0x3FFFFFFFu);
            switch (v >> 30) {
            case 0: sk.V(id); break;
            case 1: sk.X(id); break;
            case 2: sk.U(id); break;
            default: sk.W(id); break;
            }
        }
    }
}

struct FillSink {
    int32_t *pV, *pX;
    int2 *pU;
    int32_t *pW;
    const int32_t *beg, *end;
    bool ids;  // U entries as (cell, 0), resolved to particle ranges later
    int nV = 0, nX = 0, nU = 0, nW = 0;
    __device__ void V(int s) { pV[nV++] = s; }
    __device__ void X(int s) { pX[nX++] = s; }
    __device__ void U(int s) { pU[nU++] = ids ? make_int2(s, 0) : make_int2(beg[s], end[s]); }
    __device__ void W(int s) { pW[nW++] = s; }
};

// A coarse leaf N can cover several squares of a cell's ring; it is listed
// once, at the first ring square (in scan order) that it covers.  Squares of
// the ring at level l around (cx, cy), scanned dy-major from (-1, -1).
__device__ __forceinline__ bool ring_seen_before(const TreeView &t, int N, int l, int cx, int cy, int side, int dx,
                                                 int dy)
{
    const int ln = t.lvl[N];
    if (ln >= l) return false;  // same-level cells cover one square only
    const int sh = l - ln;
    const uint32_t nxy = t.ixy[N];
    const int nx = cell_ix(nxy), ny = cell_iy(nxy);
    for (int ey = -1; ey <= dy; ++ey)
        for (int ex = -1; ex <= 1; ++ex) {
            if (ey == dy && ex >= dx) return false;
            if (!ex && !ey) continue;
            const int rx = cx + ex, ry = cy + ey;
            if (rx < 0 || ry < 0 || rx >= side || ry >= side) continue;
            if ((rx >> sh) == nx && (ry >> sh) == ny) return true;
        }
    return false;
}

// The lists of cell c are enumerated by LANES lanes (1 or 8): lane q takes
// squares q, q + LANES, ... of the 3x3 ring (numbered dy-major from (-1, -1)
// without the centre), the V and X entries coming from that square of the
// parent's ring and the U and W entries from that square of c's own ring
// (leaves only).  Concatenating the lanes' entries in lane order gives each
// list in the order of one scan of the ring, whatever LANES is, so the lists
// (and every result) do not depend on the launch shape.  One lane per cell
// suits large trees (many cells, throughput-bound); eight suit small ones
// (few cells, bound by the chains of dependent hash lookups).
__device__ __forceinline__ void ring_square(int q, int &dx, int &dy)
{
    const int r = q < 4 ? q : q + 1;  // skip the centre (index 4 of the 3x3 block)
    dx = r % 3 - 1;
    dy = r / 3 - 1;
}

template <class Sink>
__device__ void vx_square(const TreeView &t, int64_t H, uint64_t ep, int c, int comp, int l, uint32_t cxy, int q,
                          Sink &sk)
{
    if (l < 2) return;
    int dx, dy;
    ring_square(q, dx, dy);
    const int pl = l - 1, px = cell_ix(cxy) >> 1, py = cell_iy(cxy) >> 1, pside = 1 << pl;
    const int rx = px + dx, ry = py + dy;
    if (rx < 0 || ry < 0 || rx >= pside || ry >= pside) return;
    const int N = lookup_region(t, H, ep, comp, pl, rx, ry);
    if (N < 0) return;
    const int4 ch = t.child[N];
    if (!is_leaf4(ch)) {
        // N is the same-level neighbour of the parent, subdivided
        const int cc[4] = {ch.x, ch.y, ch.z, ch.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int s = cc[k];
            if (s >= 0 && !cells_adjacent(l, t.ixy[s], l, cxy)) sk.V(s);
        }
    } else if (!ring_seen_before(t, N, pl, px, py, pside, dx, dy) && !cells_adjacent(t.lvl[N], t.ixy[N], l, cxy)) {
        sk.X(N);
    }
}

template <class Sink>
__device__ void uw_square(const TreeView &t, int64_t H, uint64_t ep, int comp, int l, uint32_t cxy, int q, Sink &sk)
{
    int dx, dy;
    ring_square(q, dx, dy);
    const int cx = cell_ix(cxy), cy = cell_iy(cxy), side = 1 << l;
    const int rx = cx + dx, ry = cy + dy;
    if (rx < 0 || ry < 0 || rx >= side || ry >= side) return;
    const int N = lookup_region(t, H, ep, comp, l, rx, ry);
    if (N < 0) return;
    if (is_leaf4(t.child[N])) {
        if (!ring_seen_before(t, N, l, cx, cy, side, dx, dy)) sk.U(N);
        return;
    }
    // walk N's subtree in pre-order: a descendant adjacent to the cell is
    // entered (or listed in U if it is a leaf); one that is not goes to W and
    // its subtree is skipped
    for (int s = N + 1, e = t.skip[N]; s < e;) {
        if (cells_adjacent(t.lvl[s], t.ixy[s], l, cxy)) {
            if (is_leaf4(t.child[s])) {
                sk.U(s);
                s = t.skip[s];
            } else {
                ++s;
            }
        } else {
            sk.W(s);
            s = t.skip[s];
        }
    }
}

template <int LANES, class Sink>
__device__ void enumerate_part(const TreeView &t, int64_t H, uint64_t ep, int c, int q, Sink &sk)
{
    const int l = t.lvl[c];
    const uint32_t cxy = t.ixy[c];
    const int comp = cell_comp(t, c);  // lists never leave the cell's system
    for (int s = q; s < 8; s += LANES) vx_square(t, H, ep, c, comp, l, cxy, s, sk);
    if (!is_leaf4(t.child[c])) return;
    for (int s = q; s < 8; s += LANES) uw_square(t, H, ep, comp, l, cxy, s, sk);
}

template <int LANES>
__device__ __forceinline__ int group_sum(int v)
{
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LANES);
    return v;
}

template <int LANES>
__device__ __forceinline__ int group_excl(int v)
{
    const int q = lane_id() & (LANES - 1);
    int inc = v;
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const int u = __shfl_up(inc, o, LANES);
        if (q >= o) inc += u;
    }
    return inc - v;
}

// Grid-stride over cells, one LANES-lane group per cell; the trip count is
// uniform over the wave (the shuffles need all lanes of a group).  With
// `slots` each lane also stores its first LIST_SLOTS entries there.
template <int LANES>
__global__ __launch_bounds__(LIST_NT) void k_lists_count(TreeView t, int64_t *__restrict__ cntVX,
                                                     int64_t *__restrict__ cntUW, int64_t *__restrict__ lanecnt,
                                                     int4 *__restrict__ slots)
{
    __shared__ int32_t slot_lds[LANES > 1 ? LIST_NT : 1][LANES > 1 ? LIST_SLOTS : 1];
    const int ncells = t.counts[0];
    const int64_t H = hash_size(ncells, t.hash_cap);
    const uint64_t ep = *t.epoch;
    const int q = lane_id() & (LANES - 1);
    const int gpw = WAVE / LANES;
    const int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int nw = gridDim.x * (blockDim.x / WAVE);
    for (int c0 = wid * gpw; c0 < ncells; c0 += nw * gpw) {
        const int c = c0 + lane_id() / LANES;
        int cV = 0, cX = 0, cU = 0, cW = 0;
        if constexpr (LANES > 1) {
            SlotSink sk{(SlotSink::lds_i32 *)slot_lds[threadIdx.x]};
            if (c < ncells) enumerate_part<LANES>(t, H, ep, c, q, sk);
            cV = sk.nV;
            cX = sk.nX;
            cU = sk.nU;
            cW = sk.nW;
            if (c < ncells) {
                lanecnt[(int64_t)c * LANES + q] =
                    (int64_t)cV | ((int64_t)cX << 8) | ((int64_t)cU << 16) | ((int64_t)cW << 40);
                const int tot = cV + cX + cU + cW;
                if (slots && tot > 0) {  // the lane's own LDS row: no synchronisation needed
                    const int32_t *r = slot_lds[threadIdx.x];
                    int4 *gs = slots + ((int64_t)c * LANES + q) * LIST_SLOT_Q;
#pragma unroll
                    for (int w4 = 0; w4 < LIST_SLOT_Q; ++w4)
                        if (4 * w4 < tot) gs[w4] = make_int4(r[4 * w4], r[4 * w4 + 1], r[4 * w4 + 2], r[4 * w4 + 3]);
                }
            }
        } else {
            CountSink sk;
            if (c < ncells) enumerate_part<LANES>(t, H, ep, c, q, sk);
            cV = sk.nV;
            cX = sk.nX;
            cU = sk.nU;
            cW = sk.nW;
        }
        const int nV = group_sum<LANES>(cV), nX = group_sum<LANES>(cX);
        const int nU = group_sum<LANES>(cU), nW = group_sum<LANES>(cW);
        if (c < ncells && q == 0) {
            cntVX[c] = (int64_t)nV | ((int64_t)nX << 32);
            const int li = t.leafidx[c];
            if (li >= 0) cntUW[li] = (int64_t)(nU + 1) | ((int64_t)nW << 32);  // + the leaf itself
        }
    }
}

// LDS writes of any lane of a wave visible to the wave's other lanes (LDS
// operations of a wave complete in order; no wait for global stores).
__device__ __forceinline__ void lds_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Near-field ranges of a leaf are sorted by start and touching ones merged.
// Up to FILL_STAGE of them are gathered in LDS and sorted there by lane 0 of
// the cell's group (a handful of LDS operations per range); larger lists
// (rare: a coarse leaf beside many small ones) are sorted in place in global
// memory.
constexpr int FILL_STAGE = 48;

__device__ __forceinline__ int sort_merge_ranges(int2 *r, int k, int64_t &src)
{
    for (int a = 1; a < k; ++a) {
        const int2 v = r[a];
        int b = a - 1;
        while (b >= 0 && r[b].x > v.x) {
            r[b + 1] = r[b];
            --b;
        }
        r[b + 1] = v;
    }
    int m = 0;
    src = 0;
    for (int a = 0; a < k; ++a) {
        src += r[a].y - r[a].x;
        if (m > 0 && r[m - 1].y == r[a].x) r[m - 1].y = r[a].y;
        else r[m++] = r[a];
    }
    return m;
}

template <int LANES>
__global__ __launch_bounds__(LIST_NT) void k_lists_fill(TreeView t, const int64_t *__restrict__ offVX,
                                                    const int64_t *__restrict__ offUW, int32_t *__restrict__ V,
                                                    int32_t *__restrict__ X, int2 *__restrict__ U,
                                                    int32_t *__restrict__ nU, int32_t *__restrict__ W,
                                                    unsigned long long *__restrict__ block_pairs, int64_t cap,
                                                    int64_t lcap, int64_t v_cap, int64_t x_cap, int64_t u_cap,
                                                    int64_t w_cap, int32_t *__restrict__ err,
                                                    const int64_t *__restrict__ lanecnt,
                                                    const int4 *__restrict__ slots)
{
    constexpr int STG = LANES > 1 ? FILL_STAGE : 1;  // one lane per cell: no staging
    __shared__ int2 stage[LIST_NT / LANES][STG];
    __shared__ int2 sorted[LIST_NT / LANES][STG];
    const int ncells = t.counts[0];
    const int64_t tvx = offVX[ncells], tuw = offUW[t.counts[1]];
    const bool fits = (tvx & 0xFFFFFFFFll) <= v_cap && (tvx >> 32) <= x_cap && (tuw & 0xFFFFFFFFll) <= u_cap &&
                      (tuw >> 32) <= w_cap;
    if (!fits) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, 4);
        if (threadIdx.x == 0) block_pairs[blockIdx.x] = 0ull;
        return;
    }
    const int64_t H = hash_size(ncells, t.hash_cap);
    const uint64_t ep = *t.epoch;
    const int q = lane_id() & (LANES - 1);
    const int gpw = WAVE / LANES;
    const int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int nw = gridDim.x * (blockDim.x / WAVE);
    int2 *st = stage[threadIdx.x / LANES];
    int2 *so = sorted[threadIdx.x / LANES];
    unsigned long long pairs = 0;
    for (int c0 = wid * gpw; c0 < ncells; c0 += nw * gpw) {
        const int c = c0 + lane_id() / LANES;
        const bool live = c < ncells;
        const int li = live ? t.leafidx[c] : -1;
        const int64_t ou = li >= 0 ? offUW[li] : 0;
        int2 *u0 = U + (ou & 0xFFFFFFFFll);
        // the leaf's range count, itself included (from the counting pass)
        const int k = li >= 0 ? (int)((offUW[li + 1] - ou) & 0xFFFFFFFFll) : 0;
        int pV = 0, pX = 0, pU = 0, pW = 0, tot = LIST_SLOTS + 1;
        if (LANES > 1) {  // each lane's offsets within its group's lists
            const int64_t lc = live ? lanecnt[(int64_t)c * LANES + q] : 0;
            const int cV = (int)(lc & 0xFF), cX = (int)((lc >> 8) & 0xFF);
            const int cU = (int)((lc >> 16) & 0xFFFFFF), cW = (int)((lc >> 40) & 0xFFFFFF);
            pV = group_excl<LANES>(cV);
            pX = group_excl<LANES>(cX);
            pU = group_excl<LANES>(cU);
            pW = group_excl<LANES>(cW);
            if (slots) tot = cV + cX + cU + cW;
        }
        const bool staged = LANES > 1 && li >= 0 && k <= STG;
        if (live) {
            const int64_t o = offVX[c];
            FillSink sk{V + (o & 0xFFFFFFFFll) + pV, X + (o >> 32) + pX, (staged ? st : u0) + 1 + pU,
                        W + (ou >> 32) + pW, t.beg, t.end, staged};
            if (LANES > 1 && tot <= LIST_SLOTS) {
                if (tot > 0) replay_slots(slots + ((int64_t)c * LANES + q) * LIST_SLOT_Q, tot, sk);
            } else {
                enumerate_part<LANES>(t, H, ep, c, q, sk);
            }
            if (li >= 0 && q == 0) (staged ? st : u0)[0] = staged ? make_int2(c, 0) : make_int2(t.beg[c], t.end[c]);
        }
        // the group's U entries were written by its lanes: make them visible
        // to the group.  Staged lists are in LDS (a wave-level sync suffices);
        // only when some list of the wave went to global memory does the
        // wave wait for its global stores
        if (__ballot(li >= 0 && !staged) != 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        } else {
            lds_wave_sync();
        }
        if (staged) {
            // staged entries are cell ids: their particle ranges, loaded by
            // the group's lanes together (one memory round trip)
            for (int a = q; a < k; a += LANES) {
                const int s = st[a].x;
                st[a] = make_int2(t.beg[s], t.end[s]);
            }
        }
        lds_wave_sync();
        if (staged) {
            // rank sort by the group's lanes: entry a goes to the number of
            // entries ordered before it (by start, ties by position, so the
            // ranks are a permutation of 0..k-1)
            for (int a = q; a < k; a += LANES) {
                const int2 v = st[a];
                int r = 0;
                for (int b2 = 0; b2 < k; ++b2) {
                    const int x = st[b2].x;
                    r += (x < v.x || (x == v.x && b2 < a)) ? 1 : 0;
                }
                so[r] = v;
            }
        }
        lds_wave_sync();
        if (li >= 0 && q == 0) {
            int64_t src = 0;
            int m = 0;
            if (staged) {
                // merge touching ranges (already sorted)
                int2 cur = so[0];
                src = cur.y - cur.x;
                for (int a = 1; a < k; ++a) {
                    const int2 v = so[a];
                    src += v.y - v.x;
                    if (cur.y == v.x) {
                        cur.y = v.y;
                    } else {
                        u0[m++] = cur;
                        cur = v;
                    }
                }
                u0[m++] = cur;
            } else {
                m = sort_merge_ranges(u0, k, src);
            }
            nU[li] = m;
            pairs += (unsigned long long)src * (unsigned long long)(t.end[c] - t.beg[c]);
        }
        // lane 0 is done with the stage before the next cell's lanes write it
        lds_wave_sync();
    }
    // one partial per block, summed by k_lists_stats: thousands of waves
    // adding to one global counter serialise at the memory side and stall
    // the loads of every wave queued behind them
    __shared__ unsigned long long red[LIST_NT / WAVE];
    pairs = block_sum<unsigned long long, LIST_NT>(pairs, red);
    if (threadIdx.x == 0) block_pairs[blockIdx.x] = pairs;
}

__global__ __launch_bounds__(256) void k_lists_stats(const int32_t *__restrict__ counts,
                                                     const int64_t *__restrict__ offVX,
                                                     const int64_t *__restrict__ offUW,
                                                     const unsigned long long *__restrict__ block_pairs, int nblocks,
                                                     int64_t *__restrict__ st, int n)
{
    __shared__ unsigned long long red[256 / WAVE];
    unsigned long long p = 0;
    for (int i = threadIdx.x; i < nblocks; i += 256) p += block_pairs[i];
    p = block_sum<unsigned long long, 256>(p, red);
    if (threadIdx.x != 0) return;
    const int64_t tvx = offVX[counts[0]], tuw = offUW[counts[1]];
    st[0] = counts[0];
    st[1] = counts[1];
    st[2] = (int64_t)p;
    st[3] = tvx & 0xFFFFFFFFll;
    st[5] = tvx >> 32;
    st[7] = tuw & 0xFFFFFFFFll;
    st[4] = tuw >> 32;
    st[8] += st[2];
    st[9] += st[3];
    st[10] += 1;
    st[11] += n;
}

__global__ void k_export_cells(TreeView t, int32_t *__restrict__ out, int cap)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= t.counts[0] || c >= cap) return;
    int32_t *o = out + 10 * (int64_t)c;
    uint32_t v = t.ixy[c];
    int4 ch = t.child[c];
    o[0] = t.lvl[c];
    o[1] = cell_ix(v);
    o[2] = cell_iy(v);
    o[3] = t.beg[c];
    o[4] = t.end[c];
    o[5] = t.par[c];
    o[6] = ch.x;
    o[7] = ch.y;
    o[8] = ch.z;
    o[9] = ch.w;
}

__global__ void k_fill_ncomp(const int32_t *__restrict__ coff, int K, int n, int32_t *__restrict__ ncomp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = K;  // last system whose first node is <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (coff[mid] <= i) lo = mid;
        else hi = mid;
    }
    ncomp[i] = lo;
}

}  // namespace

static Segs upload_segs(fl_ctx *c, const std::vector<int32_t> &coff, const std::string &tag)
{
    const int K = (int)coff.size() - 1;
    FL_REQUIRE(K >= 1 && K <= (1 << 20), "between 1 and 2^20 systems per batch");
    FL_REQUIRE(coff[0] == 0, "system offsets must start at 0");
    std::vector<int2> tiles;
    std::vector<int32_t> toff(K + 1);
    for (int k = 0; k < K; ++k) {
        FL_REQUIRE(coff[k + 1] > coff[k], "every system needs at least one node");
        toff[k] = (int32_t)tiles.size();
        for (int64_t b = coff[k]; b < coff[k + 1]; b += SEG_TILE) tiles.push_back(make_int2(k, (int)b));
    }
    toff[K] = (int32_t)tiles.size();
    std::vector<int2> stiles;  // sort tiles
    std::vector<int32_t> stoff(K + 1);
    const int stile = radix_sort_tile(coff[K]);
    if (K > 1) {
        for (int k = 0; k < K; ++k) {
            stoff[k] = (int32_t)stiles.size();
            for (int64_t b = coff[k]; b < coff[k + 1]; b += stile) stiles.push_back(make_int2(k, (int)b));
        }
        stoff[K] = (int32_t)stiles.size();
    }
    Segs sg;
    sg.K = K;
    sg.n = coff[K];
    sg.ntiles = (int)tiles.size();
    int cb = 0;
    while ((1 << cb) < K) ++cb;
    sg.cbits = cb;
    int32_t *d_coff = ws<int32_t>(c, (tag + "_coff").c_str(), (size_t)K + 1);
    int32_t *d_toff = ws<int32_t>(c, (tag + "_toff").c_str(), (size_t)K + 1);
    int2 *d_tiles = ws<int2>(c, (tag + "_tiles").c_str(), tiles.size());
    FL_CHECK_HIP(hipMemcpyAsync(d_coff, coff.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(d_toff, toff.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(
        hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice, c->stream));
    sg.coff = d_coff;
    sg.tile_off = d_toff;
    sg.tiles = d_tiles;
    if (K > 1) {
        int2 *d_st = ws<int2>(c, (tag + "_stiles").c_str(), stiles.size());
        int32_t *d_stoff = ws<int32_t>(c, (tag + "_stoff").c_str(), (size_t)K + 1);
        FL_CHECK_HIP(hipMemcpyAsync(d_st, stiles.data(), sizeof(int2) * stiles.size(), hipMemcpyHostToDevice,
                                    c->stream));
        FL_CHECK_HIP(
            hipMemcpyAsync(d_stoff, stoff.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice, c->stream));
        sg.sort.K = K;
        sg.sort.ntiles = (int)stiles.size();
        sg.sort.tile = stile;
        sg.sort.coff = d_coff;
        sg.sort.tiles = d_st;
        sg.sort.toff = d_stoff;
        int32_t *nc = ws<int32_t>(c, (tag + "_ncomp").c_str(), (size_t)sg.n);
        hipLaunchKernelGGL(k_fill_ncomp, dim3(grid_for(sg.n, NT)), dim3(NT), 0, c->stream, (const int32_t *)d_coff, K,
                           sg.n, nc);
        FL_LAUNCH_CHECK();
        sg.ncomp = nc;
    }
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));  // the host vectors go out of scope
    return sg;
}

Segs segs_single(fl_ctx *c, int32_t n)
{
    FL_REQUIRE(n >= 1, "need n >= 1");
    if (c->seg1_n != n) {
        c->seg1_n = -1;
        upload_segs(c, std::vector<int32_t>{0, n}, "seg1");
        c->seg1_n = n;
    }
    Segs sg;
    sg.K = 1;
    sg.n = n;
    sg.ntiles = (n + SEG_TILE - 1) / SEG_TILE;
    sg.coff = ws<int32_t>(c, "seg1_coff", 2);
    sg.tile_off = ws<int32_t>(c, "seg1_toff", 2);
    sg.tiles = ws<int2>(c, "seg1_tiles", (size_t)sg.ntiles);
    return sg;
}

Segs make_segs(fl_ctx *c, const std::vector<int32_t> &coff, const char *tag) { return upload_segs(c, coff, tag); }

namespace {

void build_tree_impl(fl_ctx *c, TreeBufs &t, const Segs &s, const float *x, const float *y, const int32_t *deg,
                     int bits, int leaf, float2 *xy_out, BBoxIn bb)
{
    const int n = s.n;
    t.n = n;
    t.s = s;
    t.bits = bits;
    t.leaf = leaf;
    t.cells_cap = cells_capacity(n, leaf, bits, s.K);
    t.leaves_cap = t.cells_cap < n ? t.cells_cap : n;
    int64_t hc = 64;
    while (hc < 2 * t.cells_cap) hc <<= 1;
    t.hash_cap = hc;
    const int64_t cap = t.cells_cap, lcap = t.leaves_cap;

    t.root = ws<double>(c, "t_root", 4 * (size_t)s.K);
    float4 *bpart = ws<float4>(c, "t_bbox_part", (size_t)s.ntiles);
    t.epoch = ws_zeroed<uint32_t>(c, "t_epoch", 4);
    uint32_t *k0 = ws<uint32_t>(c, "t_key0", n);
    uint32_t *k1 = ws<uint32_t>(c, "t_key1", n);
    int32_t *i0 = ws<int32_t>(c, "t_idx0", n);
    int32_t *i1 = ws<int32_t>(c, "t_idx1", n);
    uint64_t *q0 = nullptr, *q1 = nullptr;
    // several systems: a segmented sort of the 32-bit keys when its tiles
    // pad the input little (systems of a few keys each take the sort of
    // (system, key) pairs instead); both give the same order
    const int64_t min_tiles = s.sort.tile > 0 ? ((int64_t)n + s.sort.tile - 1) / s.sort.tile : 0;
    const bool seg = s.K > 1 && s.sort.tiles && s.sort.ntiles <= 2 * min_tiles + 8 &&
                     radix_sort_seg_fits(n, s.sort.ntiles);
    if (s.K > 1 && !seg) {
        q0 = ws<uint64_t>(c, "t_qkey0", n);
        q1 = ws<uint64_t>(c, "t_qkey1", n);
    }
    t.part = ws<float4>(c, "t_part", n);
    t.ccomp = s.K > 1 ? ws<int32_t>(c, "t_ccomp", cap) : nullptr;
    t.lvl = ws<int32_t>(c, "t_lvl", cap);
    t.ixy = ws<uint32_t>(c, "t_ixy", cap);
    t.beg = ws<int32_t>(c, "t_beg", cap);
    t.end = ws<int32_t>(c, "t_end", cap);
    t.par = ws<int32_t>(c, "t_par", cap);
    t.leafidx = ws<int32_t>(c, "t_leafidx", cap);
    t.skip = ws<int32_t>(c, "t_skip", cap);
    t.child = ws<int4>(c, "t_child", cap);
    t.leaf_cell = ws<int32_t>(c, "t_leafcell", lcap);
    t.start_key = ws<uint64_t>(c, "t_skey_start", lcap);
    t.start_pos = ws<int32_t>(c, "t_spos", lcap);
    t.start_D = ws<int32_t>(c, "t_sD", lcap);
    t.counts = ws_zeroed<int32_t>(c, "t_counts", 4);
    t.hslot = ws_zeroed<uint64_t>(c, "t_hslot", 2 * (size_t)hc);
    t.pack = ws<int32_t>(c, "t_pack", n);
    t.off2 = ws<int64_t>(c, "t_off2", (size_t)n);
    const size_t nblk_t = (size_t)grid_for(n, T1_TB);
    int64_t *bsum = ws<int64_t>(c, "t_bsum", nblk_t);
    int64_t *bpre = ws<int64_t>(c, "t_bpre", nblk_t + 1);
    if (c->tree_cbits != s.cbits) {
        // the key layout changes: restart the epoch, so that this build
        // clears the table before inserting
        fill_i32(c, (int32_t *)t.epoch, 1, 0);
        c->tree_cbits = s.cbits;
    }

    if (!bb.part) {
        hipLaunchKernelGGL(k_bbox, dim3(s.ntiles), dim3(NT), 0, c->stream, x, y, s, bpart);
        bb = BBoxIn{bpart, 1};
    }
    hipLaunchKernelGGL(k_bbox_root, dim3(std::min(s.K, 1024)), dim3(NT), 0, c->stream, s, bb.part, bb.per, t.root,
                       bits, t.epoch);
    float4 *xym = ws<float4>(c, "t_xym", n);
    // a restarted epoch clears every slot the table holds, not only this
    // build's: a later, larger build probes slots past this one's range, and
    // words left there under another key layout could pass its epoch test
    const int64_t hkey_slots = (int64_t)(c->bufs["t_hslot"].cap / (2 * sizeof(uint64_t)));
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, x, y, n, s.ncomp,
                       (const double *)t.root, bits, s.K > 1 && !seg ? nullptr : k0, q0, q0 ? i0 : nullptr,
                       (const uint32_t *)t.epoch,
                       t.hslot, hkey_slots, deg, xym, t.counts, xy_out);
    FL_LAUNCH_CHECK();
    uint32_t *sk;
    if (seg) {
        // the last pass also moves every node's record to its sorted place
        const bool alt = radix_sort_u32_seg(c, k0, i0, k1, i1, n, 2 * bits, t.counts + 3, s.sort,
                                            (const float4 *)xym, t.part, true);
        sk = alt ? k1 : k0;
    } else if (s.K > 1) {
        const bool alt = radix_sort_u64v(c, q0, i0, q1, i1, n, 32 + s.cbits, t.counts + 3);
        const uint64_t *sq = alt ? q1 : q0;
        const int32_t *perm = alt ? i1 : i0;
        sk = k0;  // written by k_gather
        hipLaunchKernelGGL(k_gather, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, (const float4 *)xym, perm, n,
                           t.part, sq, sk);
    } else {
        // the last pass also moves every node's record to its sorted place
        const bool alt =
            radix_sort_u32(c, k0, i0, k1, i1, n, 2 * bits, t.counts + 3, (const float4 *)xym, t.part, true);
        sk = alt ? k1 : k0;
    }
    t.skey = sk;
    const unsigned nblk = grid_for(n, T1_TB);
    hipLaunchKernelGGL(k_tree_levels, dim3(nblk), dim3(NT), 0, c->stream, (const uint32_t *)sk, n, bits, leaf, s.ncomp,
                       t.pack, t.off2, bsum);
    FL_LAUNCH_CHECK();
    scan_excl_i64(c, bsum, bpre, nblk);
    hipLaunchKernelGGL(k_tree_cells, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, (const uint32_t *)sk, n, bits,
                       (const int32_t *)t.pack, (const int64_t *)t.off2, (const int64_t *)bpre, s.ncomp, t);
    // a pair of waves per 64 cells (the grid loops past 2048 blocks)
    hipLaunchKernelGGL(k_tree_links, dim3(grid_for(2 * cap, NT, 2048)), dim3(NT), 0, c->stream, (const uint32_t *)sk,
                       n, bits, (const int64_t *)t.off2, (const int64_t *)bpre, t);
    FL_LAUNCH_CHECK();
}

}  // namespace

void build_tree(fl_ctx *c, TreeBufs &t, const Segs &s, const float *x, const float *y, const int32_t *deg, int bits,
                int leaf, float2 *xy_out, BBoxIn bb)
{
    build_tree_impl(c, t, s, x, y, deg, bits, leaf, xy_out, bb);
}

// eight lanes measured faster at every size tried (15k-node components up to
// a 2M-node system); one lane per cell stays available to the tuner
int default_list_lanes(int64_t) { return 8; }

void build_lists(fl_ctx *c, const TreeBufs &t, ListBufs &L, int lanes)
{
    FL_REQUIRE(lanes == 1 || lanes == 8, "list building takes 1 or 8 lanes per cell");
    const int64_t cap = t.cells_cap, lcap = t.leaves_cap;
    L.v_cap = 27 * cap;
    L.x_cap = 8 * cap;
    L.w_cap = 8 * cap;
    L.u_cap = 17 * lcap;
    int64_t *cntVX = ws<int64_t>(c, "l_cntVX", cap);
    int64_t *cntUW = ws<int64_t>(c, "l_cntUW", lcap);
    L.offVX = ws<int64_t>(c, "l_offVX", cap + 1);
    L.offUW = ws<int64_t>(c, "l_offUW", lcap + 1);
    L.V = ws<int32_t>(c, "l_V", L.v_cap);
    L.X = ws<int32_t>(c, "l_X", L.x_cap);
    L.U = ws<int2>(c, "l_U", L.u_cap);
    L.nU = ws<int32_t>(c, "l_nU", lcap);
    L.W = ws<int32_t>(c, "l_W", L.w_cap);
    TreeView tv = view(t);
    // grid-stride over the cells (their number is known on the device only)
    const bool wide = lanes == 8;
    const unsigned lg = grid_for(cap, wide ? LIST_NT / 8 : LIST_NT, 4096 * 256 / LIST_NT);
    int64_t *lanecnt = wide ? ws<int64_t>(c, "l_lanecnt", (size_t)cap * 8) : nullptr;
    // entry slots: LIST_SLOT_Q int4 per (cell, lane); cell ids must leave the tag bits free
    int4 *slots = wide && cap < (int64_t(1) << 30) ? ws<int4>(c, "l_slots", (size_t)cap * 8 * LIST_SLOT_Q) : nullptr;
    if (wide)
        hipLaunchKernelGGL(k_lists_count<8>, dim3(lg), dim3(LIST_NT), 0, c->stream, tv, cntVX, cntUW, lanecnt, slots);
    else
        hipLaunchKernelGGL(k_lists_count<1>, dim3(lg), dim3(LIST_NT), 0, c->stream, tv, cntVX, cntUW, lanecnt,
                           (int4 *)nullptr);
    FL_LAUNCH_CHECK();
    scan_excl_i64_pair(c, cntVX, L.offVX, cap, t.counts, cntUW, L.offUW, lcap, t.counts + 1);
    auto fill = wide ? k_lists_fill<8> : k_lists_fill<1>;
    L.block_pairs = ws<unsigned long long>(c, "l_block_pairs", (size_t)lg);
    L.fill_blocks = (int)lg;
    hipLaunchKernelGGL(fill, dim3(lg), dim3(LIST_NT), 0, c->stream, tv, (const int64_t *)L.offVX,
                       (const int64_t *)L.offUW, L.V, L.X, L.U, L.nU, L.W, L.block_pairs, cap, lcap, L.v_cap,
                       L.x_cap, L.u_cap, L.w_cap, t.counts + 3, (const int64_t *)lanecnt, (const int4 *)slots);
    FL_LAUNCH_CHECK();
}

void lists_stats(fl_ctx *c, const TreeBufs &t, const ListBufs &L, hipStream_t s)
{
    hipLaunchKernelGGL(k_lists_stats, dim3(1), dim3(256), 0, s ? s : c->stream, t.counts, (const int64_t *)L.offVX,
                       (const int64_t *)L.offUW, (const unsigned long long *)L.block_pairs, L.fill_blocks,
                       c->d_stats, t.n);
    FL_LAUNCH_CHECK();
}

__global__ void k_max_level(const int32_t *__restrict__ counts, const int32_t *__restrict__ lvl,
                            int64_t *__restrict__ st)
{
    __shared__ int lds[4];
    int m = 0;
    for (int i = threadIdx.x; i < counts[0]; i += blockDim.x) m = max(m, lvl[i]);
    m = wave_max_i(m);
    if (lane_id() == 0) lds[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) st[6] = max(max(lds[0], lds[1]), max(lds[2], lds[3]));
}

// deepest level of the last tree into the statistics block (for fl_fmm_stats)
void tree_max_level(fl_ctx *c)
{
    auto it = c->bufs.find("t_lvl");
    if (it == c->bufs.end() || !it->second.p) return;
    int32_t *counts = ws_zeroed<int32_t>(c, "t_counts", 4);
    hipLaunchKernelGGL(k_max_level, dim3(1), dim3(256), 0, c->stream, counts, (const int32_t *)it->second.p,
                       c->d_stats);
    FL_LAUNCH_CHECK();
}

int32_t tree_error_bits(fl_ctx *c, bool clear)
{
    int32_t *counts = ws_zeroed<int32_t>(c, "t_counts", 4);
    int32_t v = read_i32(c, counts + 3);
    if (clear) FL_CHECK_HIP(hipMemsetAsync(counts + 3, 0, sizeof(int32_t), c->stream));
    return v;
}

void morton_keys(fl_ctx *c, int32_t n, const float *x, const float *y, int bits, uint32_t *key, double *root_out)
{
    const Segs sg = segs_single(c, n);
    double *root = root_out ? root_out : ws<double>(c, "t_root", 4);
    float4 *bpart = ws<float4>(c, "t_bbox_part", (size_t)sg.ntiles);
    // no tree is built: leave the hash epoch alone
    hipLaunchKernelGGL(k_bbox, dim3(sg.ntiles), dim3(NT), 0, c->stream, x, y, sg, bpart);
    hipLaunchKernelGGL(k_bbox_root, dim3(1), dim3(NT), 0, c->stream, sg, (const float4 *)bpart, 1, root, bits,
                       (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, x, y, n, (const int32_t *)nullptr,
                       (const double *)root, bits, key, (uint64_t *)nullptr, (int32_t *)nullptr,
                       (const uint32_t *)nullptr, (uint64_t *)nullptr, (int64_t)0, (const int32_t *)nullptr,
                       (float4 *)nullptr, (int32_t *)nullptr, (float2 *)nullptr);
    FL_LAUNCH_CHECK();
}

}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_morton(fl_ctx *c, int32_t n, const float *x, const float *y, int32_t bits, uint32_t *key, double *root4)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1 && x && y && key, "fl_morton: need n >= 1 and non-null arrays");
    FL_REQUIRE(bits >= 1 && bits <= 16, "fl_morton: bits must be in [1, 16]");
    morton_keys(c, n, x, y, bits, key, root4);
    FL_API_END(c)
}

fl_status fl_sort_keys(fl_ctx *c, int32_t n, const uint32_t *key, int32_t bits, uint32_t *key_out, int32_t *perm)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1 && key && key_out && perm, "fl_sort_keys: need n >= 1 and non-null arrays");
    FL_REQUIRE(bits >= 1 && bits <= 16, "fl_sort_keys: bits must be in [1, 16]");
    uint32_t *kt = ws<uint32_t>(c, "sk_kt", n);
    int32_t *vt = ws<int32_t>(c, "sk_vt", n);
    FL_CHECK_HIP(hipMemcpyAsync(key_out, key, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c->stream));
    int32_t *err = ws_zeroed<int32_t>(c, "sk_err", 1);
    // bits >= 1: at least one pass, which writes every payload (the indices)
    bool alt = radix_sort_u32(c, key_out, perm, kt, vt, n, 2 * bits, err, nullptr, nullptr, true);
    if (read_i32(c, err)) {
        FL_CHECK_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), c->stream));
        throw Error(FL_EHIP, "fl_sort_keys: the sort's look-back gave up");
    }
    if (alt) {
        FL_CHECK_HIP(hipMemcpyAsync(key_out, kt, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c->stream));
        FL_CHECK_HIP(hipMemcpyAsync(perm, vt, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c->stream));
    }
    FL_API_END(c)
}

fl_status fl_tree(fl_ctx *c, int32_t n, const float *x, const float *y, int32_t bits, int32_t leaf_size,
                  int32_t *cells, int32_t cap, int32_t *n_cells_out)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1 && x && y && cells && cap >= 0, "fl_tree: need n >= 1 and non-null arrays");
    FL_REQUIRE(bits >= 1 && bits <= 16, "fl_tree: bits must be in [1, 16]");
    FL_REQUIRE(leaf_size >= 1 && leaf_size <= 1024, "fl_tree: leaf_size must be in [1, 1024]");
    TreeBufs t;
    build_tree(c, t, segs_single(c, n), x, y, nullptr, bits, leaf_size);
    TreeView tv = view(t);
    hipLaunchKernelGGL(k_export_cells, dim3(grid_for(t.cells_cap, 256)), dim3(256), 0, c->stream, tv, cells, cap);
    FL_LAUNCH_CHECK();
    int32_t nc = read_i32(c, t.counts);
    if (tree_error_bits(c, true)) throw Error(FL_EHIP, "fl_tree: capacity guard tripped");
    if (n_cells_out) *n_cells_out = nc;
    FL_REQUIRE(nc <= cap, "fl_tree: output capacity too small");
    FL_API_END(c)
}

}  // extern "C"
