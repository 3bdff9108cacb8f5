// The FMM passes of the paper's sec. 3.2.1 on the quadtree of fl_tree.hip,
// with the expansion operators of Greengard & Rokhlin (1987) for the
// potential phi(z) = sum_j m_j log(z - z_j), whose conjugate derivative gives
// the repulsion: F_i = kr m_i conj(phi'(z_i)).
//
// Every expansion is stored scaled by its cell width w so FP32 cannot
// overflow for any order or extent: outgoing coefficient k holds a_k / w^k
// (|.| <= Q 0.71^k / k), incoming coefficient l holds b_l w^l.
//
//   k_p2m     leaves: outgoing expansion from the particles (P2M).
//   k_m2m_*   each internal cell shifts its children's expansions to its
//             centre and adds them (M2M), deepest level first: one workgroup
//             per level-4 subtree (levels ordered by workgroup barriers),
//             then one workgroup for the levels above.
//   k_m2l     every cell: interacting cells' outgoing expansions converted to
//             an incoming one (M2L, V list) plus particles of coarser
//             separated leaves (P2L, X list); one lane per source cell.
//   k_l2l     every leaf: incoming expansions of the leaf and all its
//             ancestors shifted to the leaf centre.  Shifts compose exactly,
//             so this is the paper's parent-to-child recursion unrolled along
//             each leaf's ancestor chain (one launch instead of one per level).
//   k_p2p     one wave per leaf: the direct near field over the U list
//             (P2P), written per particle in sorted order.  Lanes hold
//             targets; sources are read at wave-uniform addresses (scalar
//             loads, SGPR operands: no per-lane memory traffic in the pair
//             loop).  Leaves of at most 32 (16) targets run 2 (4) lane groups
//             on interleaved sources, staged 64 at a time in LDS and read
//             there by each group (no per-pair selects); the groups are
//             combined with xor shuffles (fixed order).
//   k_far     one thread per particle: far field from its leaf's incoming
//             expansion (L2P) and the W list's outgoing expansions (M2P),
//             added to the near field; the force goes to the node's
//             original index.
//
// Launch shapes: P2M, M2L and the evaluations launch about one wave per leaf
// (or pair of cells) instead of a fixed stride of several per wave; the cost
// per leaf varies a lot, and the dispatcher balances short waves better.
#include <algorithm>

#include "fl_fmm.h"

namespace fl {
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 crecip(float2 a)
{
    float inv = 1.0f / (a.x * a.x + a.y * a.y);
    return make_float2(a.x * inv, -a.y * inv);
}

constexpr float binomf(int n, int k)
{
    if (k < 0 || k > n) return 0.0f;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return (float)r;
}

// Centre, width w = L 2^-l and its reciprocal.  The root record holds
// 2^bits / L correctly rounded, so 2^(l - bits) times it is 1 / w correctly
// rounded (a power-of-two scaling is exact): the same bits as the FP64
// division, without one.
struct CellGeo {
    double cx, cy, w, iw;
};

__device__ __forceinline__ CellGeo geo(const TreeView &t, int c)
{
    const double *rt = t.root + 4 * (int64_t)cell_comp(t, c);
    const double x0 = rt[0], y0 = rt[1], L = rt[2];
    const int l = t.lvl[c];
    const uint32_t v = t.ixy[c];
    const double w = ldexp(L, -l);
    return CellGeo{x0 + ((double)cell_ix(v) + 0.5) * w, y0 + ((double)cell_iy(v) + 0.5) * w, w,
                   ldexp(rt[3], l - t.bits)};
}

__device__ __forceinline__ float2 rel(float x, float y, const CellGeo &g)
{
    return make_float2((float)(((double)x - g.cx) / g.w), (float)(((double)y - g.cy) / g.w));
}

// ---------------------------------------------------------------------------
// Lanes of one wave exchanging data through LDS: make every lane's LDS writes
// visible to the other lanes of the wave (no block barrier: the waves of a
// block work on different leaves and must not wait for each other).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P>
struct P2MLds {
    float2 buf[4][P + 1][WAVE + 1];  // per-wave P2M contributions, transposed (padded rows)
};

// k_p2m: one wave per leaf.  Each lane takes particles of the leaf and writes
// its P+1 terms (Q contribution and -q u^k / k) to LDS; lane k then sums
// column k in lane order, over the rows that hold particles.
template <int P>
__global__ __launch_bounds__(256) void k_p2m(TreeView t, const float4 *__restrict__ part,
                                             const int32_t *__restrict__ leaf_cell, float2 *__restrict__ M)
{
    __shared__ P2MLds<P> sh;
    const int nleaves = t.counts[1];
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    const int wpb = blockDim.x / WAVE;
    for (int li = blockIdx.x * wpb + w; li < nleaves; li += gridDim.x * wpb) {
        const int c = leaf_cell[li];
        const CellGeo g = geo(t, c);
        const double inv_w = g.iw;
        const int b = t.beg[c], e = t.end[c];
        float2 acc = make_float2(0.f, 0.f);
        for (int t0 = b; t0 < e; t0 += WAVE) {
            const int j = t0 + lane;
            float q = 0.f;
            float2 u = make_float2(0.f, 0.f);
            if (j < e) {
                const float4 p = part[j];
                q = p.z;
                u = make_float2((float)(((double)p.x - g.cx) * inv_w), (float)(((double)p.y - g.cy) * inv_w));
            }
            sh.buf[w][0][lane] = make_float2(q, 0.f);
            float2 pw = u;
#pragma unroll
            for (int k = 1; k <= P; ++k) {
                sh.buf[w][k][lane] = cscale(pw, -q * (1.0f / (float)k));
                pw = cmul(pw, u);
            }
            wave_lds_sync();
            if (lane <= P) {
                const int nl = min(WAVE, e - t0);  // rows past the leaf's particles hold zeros
#pragma unroll 8
                for (int i = 0; i < nl; ++i) acc = cadd(acc, sh.buf[w][lane][i]);
            }
            wave_lds_sync();
        }
        if (lane <= P) M[(int64_t)c * (P + 1) + lane] = acc;
    }
}

// Child-to-parent shift of outgoing expansions (M2M, Greengard & Rokhlin
// Lemma 2.3) in scaled form: child centre at (+-1/4, +-1/4) parent widths,
// child width 1/2, so each quadrant has a constant operator
//   A_l = sum_k T_q[l][k] A^q_k,  T_q[0][0] = 1,  T_q[l][0] = -z^l / l,
//   T_q[l][k] = 2^-k z^(l-k) C(l-1, k-1) (1 <= k <= l).
template <int P>
__global__ void k_m2m_table(float2 *__restrict__ T)
{
    for (int idx = threadIdx.x; idx < 4 * (P + 1) * (P + 1); idx += blockDim.x) {
        const int q = idx / ((P + 1) * (P + 1)), l = (idx / (P + 1)) % (P + 1), k = idx % (P + 1);
        const double zx = (q & 1) ? 0.25 : -0.25, zy = (q >> 1) ? 0.25 : -0.25;
        double vx = 0.0, vy = 0.0;
        if (l == 0) {
            vx = k == 0 ? 1.0 : 0.0;
        } else if (k <= l) {
            double px = 1.0, py = 0.0;  // z^(l-k)
            for (int i = 0; i < l - k; ++i) {
                const double nx = px * zx - py * zy, ny = px * zy + py * zx;
                px = nx;
                py = ny;
            }
            double f;
            if (k == 0) {
                f = -1.0 / (double)l;
            } else {
                f = ldexp(1.0, -k);
                for (int i = 1; i <= k - 1; ++i) f = f * (double)(l - k + i) / (double)i;
            }
            vx = f * px;
            vy = f * py;
        }
        T[idx] = make_float2((float)vx, (float)vy);
    }
}

template <int P>
__device__ __forceinline__ void m2m_cell(const TreeView &t, const float2 *__restrict__ T, float2 *M, int c)
{
    const int4 ch = t.child[c];
    float2 B[P + 1];
#pragma unroll
    for (int l = 0; l <= P; ++l) B[l] = make_float2(0.f, 0.f);
    const int cc[4] = {ch.x, ch.y, ch.z, ch.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cid = cc[q];
        if (cid < 0) continue;
        float2 A[P + 1];
        const float2 *Mq = M + (int64_t)cid * (P + 1);
#pragma unroll
        for (int k = 0; k <= P; ++k) A[k] = Mq[k];
        const float2 *Tq = T + q * (P + 1) * (P + 1);
#pragma unroll
        for (int l = 0; l <= P; ++l) {
#pragma unroll
            for (int k = 0; k <= l; ++k) {
                const float2 tq = Tq[l * (P + 1) + k];
                B[l].x += tq.x * A[k].x - tq.y * A[k].y;
                B[l].y += tq.x * A[k].y + tq.y * A[k].x;
            }
        }
    }
    float2 *Mc = M + (int64_t)c * (P + 1);
#pragma unroll
    for (int l = 0; l <= P; ++l) Mc[l] = B[l];
}

// first cell id whose first particle is >= v (cells are sorted by begin)
__device__ __forceinline__ int first_cell_at(const TreeView &t, int ncells, int v)
{
    int lo = 0, hi = ncells;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t.beg[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int M2M_CUT = 4;  // subtrees rooted at level 4: 256 workgroups

// k_m2m_sub: a workgroup owns the subtree of one level-4 square of one
// system (a contiguous range of the pre-order) at a time; its internal cells
// are shifted level by level, deepest first, with a workgroup barrier
// between levels.  Subtree r is square r % 256 of system r / 256.
template <int P>
__global__ __launch_bounds__(256) void k_m2m_sub(TreeView t, const float2 *__restrict__ T, float2 *M)
{
    const int ncells = t.counts[0];
    const int side = 1 << M2M_CUT;
    if (ncells <= 1 || M2M_CUT >= t.bits) return;
    const int64_t H = hash_size(ncells, t.hash_cap);
    const uint64_t ep = *t.epoch;
    __shared__ int sm[4];
    const int64_t nsub = (int64_t)t.K * side * side;
    for (int64_t r = blockIdx.x; r < nsub; r += gridDim.x) {
        const int comp = (int)(r >> (2 * M2M_CUT)), sq = (int)(r & (side * side - 1));
        const int root = hash_find(t, H, ep, comp, M2M_CUT, sq % side, sq / side);
        if (root < 0 || is_leaf4(t.child[root])) continue;  // uniform over the workgroup
        const int c0 = root, c1 = first_cell_at(t, ncells, t.end[root]);
        int maxl = M2M_CUT;
        for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) maxl = max(maxl, t.lvl[c]);
        maxl = wave_max_i(maxl);
        if (lane_id() == 0) sm[threadIdx.x / WAVE] = maxl;
        __syncthreads();
        maxl = max(max(sm[0], sm[1]), max(sm[2], sm[3]));
        __syncthreads();
        for (int lev = maxl - 1; lev >= M2M_CUT; --lev) {
            for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x)
                if (t.lvl[c] == lev && !is_leaf4(t.child[c])) m2m_cell<P>(t, T, M, c);
            __syncthreads();
        }
    }
}

// k_m2m_top: the internal cells above level 4 (at most 85 squares per
// system, found by their (system, level, ix, iy) key), a workgroup per system.
template <int P>
__global__ __launch_bounds__(256) void k_m2m_top(TreeView t, const float2 *__restrict__ T, float2 *M)
{
    // a short chain of dependent levels that M2L waits for, started as the
    // near field fills the GPU: its waves issue first (a 2M-node iteration
    // 0.6853-0.6859 -> 0.6832-0.6840 ms together with L2L's; priority for the
    // whole upward/M2L branch, or for M2L, was slower)
    __builtin_amdgcn_s_setprio(3);
    const int ncells = t.counts[0];
    if (ncells <= 1) return;
    const int64_t H = hash_size(ncells, t.hash_cap);
    const uint64_t ep = *t.epoch;
    const int top = min(M2M_CUT, t.bits) - 1;
    for (int comp = blockIdx.x; comp < t.K; comp += gridDim.x) {
        for (int lev = top; lev >= 0; --lev) {
            const int side = 1 << lev;
            for (int r = threadIdx.x; r < side * side; r += blockDim.x) {
                const int c = hash_find(t, H, ep, comp, lev, r % side, r / side);
                if (c >= 0 && !is_leaf4(t.child[c])) m2m_cell<P>(t, T, M, c);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// k_m2l: two target cells per wave (one per half-wave).  Lane j of a half
// converts source V[j] of its cell (a V list holds at most 27 cells) with the
// whole M2L of Greengard & Rokhlin's Lemma 2.4 in scaled form, rho = w / z0:
//   B_l += rho^l [ -Q/l + sum_k C(l+k-1, k-1) (-rho)^k A_k ],
// and the half's lanes are summed through LDS in lane order (fixed order).
// The X list (P2L: particles of coarser separated leaves) is spread over the
// same lanes, particle by particle, before the sum.
template <int P>
__global__ __launch_bounds__(256) void k_m2l(TreeView t, const float4 *__restrict__ part,
                                             const float2 *__restrict__ M, const int64_t *__restrict__ offVX,
                                             const int32_t *__restrict__ V, const int32_t *__restrict__ X,
                                             float2 *__restrict__ Lp)
{
    constexpr int ROW = 2 * P + 1;  // floats per lane row (odd: no bank conflicts down a column)
    __shared__ float rows_all[4][WAVE * ROW];
    // rho^k (k = 1..P) of every offset (dx, dy) a V entry can have: a child
    // of a same-level neighbour of the parent lies at most 3 cells away on
    // each axis, so 7 x 7 offsets (the centre is never used)
    __shared__ float2 rpow[P][49];
    if (threadIdx.x < 49) {
        const int dx = (int)threadIdx.x / 7 - 3, dy = (int)threadIdx.x % 7 - 3;
        const float2 rho = (dx | dy) ? crecip(make_float2((float)dx, (float)dy)) : make_float2(0.f, 0.f);
        float2 pw = rho;
        for (int k = 0; k < P; ++k) {
            rpow[k][threadIdx.x] = pw;
            pw = cmul(pw, rho);
        }
    }
    __syncthreads();
    float *rows = rows_all[threadIdx.x / WAVE];
    const int ncells = t.counts[0];
    const int lane = lane_id();
    const int half = lane >> 5, j = lane & 31;
    const int wpb = blockDim.x / WAVE;
    for (int c0 = 2 * (blockIdx.x * wpb + (int)threadIdx.x / WAVE); c0 < ncells; c0 += 2 * gridDim.x * wpb) {
        const int c = c0 + half;
        const bool live = c < ncells;
        float2 B[P + 1];
#pragma unroll
        for (int l = 0; l <= P; ++l) B[l] = make_float2(0.f, 0.f);
        int x0 = 0, x1 = 0;
        if (live) {
            const int64_t o0 = offVX[c], o1 = offVX[c + 1];
            const int v0 = (int)(o0 & 0xFFFFFFFFll), v1 = (int)(o1 & 0xFFFFFFFFll);
            x0 = (int)(o0 >> 32);
            x1 = (int)(o1 >> 32);
            const uint32_t cxy = t.ixy[c];
            for (int ei = v0 + j; ei < v1; ei += 32) {
                const int s = V[ei];
                const uint32_t sxy = t.ixy[s];
                // same level: source centre - target centre = w (dx + i dy),
                // rho = w / (source - target) from the offset table
                const int o = (cell_ix(sxy) - cell_ix(cxy) + 3) * 7 + (cell_iy(sxy) - cell_iy(cxy) + 3);
                const float2 *Ms = M + (int64_t)s * (P + 1);
                const float Q = Ms[0].x;
                float2 ap[P + 1];  // rho^k a_k; the sign of (-rho)^k goes into the coefficient
#pragma unroll
                for (int k = 1; k <= P; ++k) ap[k] = cmul(rpow[k - 1][o], Ms[k]);
#pragma unroll
                for (int l = 1; l <= P; ++l) {
                    float2 in = make_float2(-Q * (1.0f / (float)l), 0.f);
#pragma unroll
                    for (int k = 1; k <= P; ++k) {
                        const float bc = (k & 1 ? -1.0f : 1.0f) * binomf(l + k - 1, k - 1);
                        in.x = fmaf(bc, ap[k].x, in.x);
                        in.y = fmaf(bc, ap[k].y, in.y);
                    }
                    const float2 rl = rpow[l - 1][o];
                    B[l].x = fmaf(rl.x, in.x, fmaf(-rl.y, in.y, B[l].x));
                    B[l].y = fmaf(rl.x, in.y, fmaf(rl.y, in.x, B[l].y));
                }
            }
        }
        const bool anyx = __ballot(live && x1 > x0) != 0;
        if (anyx && live && x1 > x0) {
            const CellGeo g = geo(t, c);
            const double inv_w = g.iw;
            for (int e = x0; e < x1; ++e) {
                const int s = X[e];
                const int sb = t.beg[s], se = t.end[s];
                for (int jj = sb + j; jj < se; jj += 32) {
                    const float4 p = part[jj];
                    const float2 zn = make_float2((float)(((double)p.x - g.cx) * inv_w),
                                                  (float)(((double)p.y - g.cy) * inv_w));
                    const float2 rho = crecip(zn);  // w / (z_j - z_c)
                    float2 pw = rho;
#pragma unroll
                    for (int l = 1; l <= P; ++l) {
                        const float s2 = p.z * (1.0f / (float)l);
                        B[l].x -= s2 * pw.x;
                        B[l].y -= s2 * pw.y;
                        pw = cmul(pw, rho);
                    }
                }
            }
        }
        // sum over the half's 32 lanes through LDS: each lane stores its 2P
        // components, then lane q < 2P of the half adds component q over the
        // 32 rows in lane order (a transposed reduction: 2P stores and 32
        // loads per lane instead of an xor butterfly of 5 x 2P shuffles)
        wave_lds_sync();  // the previous cell's rows have been read
#pragma unroll
        for (int l = 1; l <= P; ++l) {
            rows[lane * ROW + 2 * (l - 1)] = B[l].x;
            rows[lane * ROW + 2 * (l - 1) + 1] = B[l].y;
        }
        wave_lds_sync();
        if (live) {
            float *Lc = reinterpret_cast<float *>(Lp + (int64_t)c * (P + 1));
            if (j < 2 * P) {
                const float *col = rows + half * 32 * ROW + j;
                float acc = 0.f;
#pragma unroll 8
                for (int r = 0; r < 32; ++r) acc += col[r * ROW];
                Lc[2 + j] = acc;
            }
            if (j == 0) {
                Lc[0] = 0.f;  // B_0 is never accumulated (the potential's constant)
                Lc[1] = 0.f;
            }
        }
    }
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_l2l(TreeView t, const float2 *__restrict__ Lp, float2 *__restrict__ Lleaf)
{
    // between M2L and the far field on the critical path: issue first
    __builtin_amdgcn_s_setprio(3);
    const int nleaves = t.counts[1];
    for (int li = blockIdx.x * blockDim.x + threadIdx.x; li < nleaves; li += gridDim.x * blockDim.x) {
        const int c = t.leaf_cell[li];
        const int lc = t.lvl[c];
        const uint32_t cxy = t.ixy[c];
        float2 C[P + 1];
        const float2 *Lc = Lp + (int64_t)c * (P + 1);
#pragma unroll
        for (int l = 0; l <= P; ++l) C[l] = Lc[l];
        for (int a = t.par[c]; a >= 0; a = t.par[a]) {
            const int la = t.lvl[a];
            const uint32_t axy = t.ixy[a];
            const float r = ldexpf(1.0f, la - lc);
            const float2 tau = make_float2(((float)cell_ix(cxy) + 0.5f) * r - ((float)cell_ix(axy) + 0.5f),
                                           ((float)cell_iy(cxy) + 0.5f) * r - ((float)cell_iy(axy) + 0.5f));
            float2 d[P + 1];
            const float2 *La = Lp + (int64_t)a * (P + 1);
#pragma unroll
            for (int l = 0; l <= P; ++l) d[l] = La[l];
            // Taylor shift: d_m <- sum_{l >= m} C(l, m) tau^(l-m) d_l
#pragma unroll
            for (int k = 0; k < P; ++k) {
#pragma unroll
                for (int j = P - 1; j >= k; --j) d[j] = cadd(d[j], cmul(tau, d[j + 1]));
            }
            float rm = 1.0f;
#pragma unroll
            for (int m = 0; m <= P; ++m) {
                C[m].x += rm * d[m].x;
                C[m].y += rm * d[m].y;
                rm *= r;
            }
        }
        float2 *Lo = Lleaf + (int64_t)li * (P + 1);
#pragma unroll
        for (int l = 0; l <= P; ++l) Lo[l] = C[l];
    }
}

// ---------------------------------------------------------------------------
// near-field pair: source (sx, sy, sm) at a wave-uniform address, so the
// compiler keeps it in scalar registers and the VALU reads it directly
#define FL_P2P_PAIR(SX, SY, SM)                                                                                     \
    {                                                                                                               \
        const float dx = me.x - (SX), dy = me.y - (SY);                                                             \
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));                                                        \
        const float sm = (SM) * __builtin_amdgcn_rcpf(r2);                                                          \
        fx = fmaf(sm, dx, fx);                                                                                      \
        fy = fmaf(sm, dy, fy);                                                                                      \
    }

constexpr int P2P_GMAX = 16;            // lane groups at most
constexpr int P2P_TMAX = 8;             // targets per lane at most
constexpr int P2P_STAGE = WAVE + P2P_GMAX;  // staged sources plus zero-mass padding
// per wave, the staged sources (float4) during the source loop and the lane
// groups' partial sums (float2, T per lane) after it share one LDS area
constexpr int P2P_WAVE_LDS = (P2P_STAGE * 16 > WAVE * P2P_TMAX * 8 ? P2P_STAGE * 16 : WAVE * P2P_TMAX * 8);

// Lane-group shape of the near field for a leaf chunk of n targets: T
// targets per lane, groups of L = ceil(n / T) lanes, G = 64 / L groups on
// sources interleaved mod G.  A round of G sources costs 64 T lane slots and
// does G n pairs; the shape with the most pairs per slot wins (the smaller
// T on a tie).  G = 1 is the plain one-target-per-lane wave.
// The shapes of all chunk sizes 1..64, fixed at compile time (T | L << 8 |
// G << 16 | S << 24, with S = G floor(64 / G) the sources a stage takes, so
// that only a range's last stage ends in a partial round): a chunk reads its
// shape with one scalar load instead of dividing.
struct P2PShapes {
    uint32_t v[WAVE + 1];
};

constexpr P2PShapes p2p_shape_table()
{
    P2PShapes s{};
    for (int n = 1; n <= WAVE; ++n) {
        int T = 1, L = n, G = WAVE / n < P2P_GMAX ? WAVE / n : P2P_GMAX;
        int best = G * n * 840;  // pairs per round x 840 / T (840: a common multiple of 1..8)
        for (int t = 2; t <= P2P_TMAX; ++t) {
            const int l = (n + t - 1) / t, g = WAVE / l < P2P_GMAX ? WAVE / l : P2P_GMAX;
            const int v = g * n * 840 / t;
            if (v > best) {
                best = v;
                T = t;
                L = l;
                G = g;
            }
        }
        const int S = G * (WAVE / G);
        s.v[n] = (uint32_t)T | ((uint32_t)L << 8) | ((uint32_t)G << 16) | ((uint32_t)S << 24);
    }
    return s;
}

__constant__ P2PShapes P2P_SHAPE = p2p_shape_table();

__device__ __forceinline__ void p2p_shape(int n, int &T, int &L, int &G, int &S)
{
    const uint32_t v = P2P_SHAPE.v[n];
    T = (int)(v & 0xFFu);
    L = (int)((v >> 8) & 0xFFu);
    G = (int)((v >> 16) & 0xFFu);
    S = (int)(v >> 24);
}

// One chunk of a leaf's targets (t0 .. t0 + n) in lane groups: lane (g, r)
// holds targets r, r + L, ..., takes sources k = g mod G from an LDS stage of
// S <= 64 sources (a multiple of G), and the groups' sums are added in group
// order through LDS.  Lanes past G L compute on group 0's sources and their
// sums are never read.
template <int T>
__device__ __forceinline__ void p2p_groups(const float4 *__restrict__ part, const int2 *__restrict__ U, int u0,
                                           int u1, int t0, int n, int L, int G, int S, float4 *sw, float2 *rw,
                                           float2 *__restrict__ near, int32_t *__restrict__ pleaf, int li)
{
    const int lane = lane_id();
    // lane / L through FP32: lane + 0.5 is at least 0.5 / L away from every
    // multiple of L, far more than the rounding of the product
    const int grp = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)L)), r = lane - grp * L;
    const int gr = grp < G ? grp : 0;
    // the targets' (x, y) only: the mass and id are not needed here
    const float2 *pxy = reinterpret_cast<const float2 *>(part);
    float2 me[T];
    float fx[T], fy[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        me[u] = pxy[2 * (t0 + min(r + u * L, n - 1))];
        fx[u] = 0.f;
        fy[u] = 0.f;
    }
    for (int ue = u0; ue < u1; ++ue) {
        const int2 rg = U[ue];
        for (int j0 = rg.x; j0 < rg.y; j0 += S) {
            const int ns = min(S, rg.y - j0);
            const bool in = lane < ns;
            const float4 v = part[j0 + (in ? lane : 0)];
            // lanes past the chunk hold a source of mass 0 (adds 0); the
            // select is per component (a whole-float4 select went through
            // scratch memory)
            const float4 sv = make_float4(v.x, v.y, in ? v.z : 0.f, in ? v.w : 0.f);
            wave_lds_sync();  // the previous chunk has been read
            sw[lane] = sv;
            if (lane < P2P_GMAX) sw[WAVE + lane] = make_float4(v.x, v.y, 0.f, 0.f);
            wave_lds_sync();
            // k + gr <= ns - 1 + G - 1 < P2P_STAGE; past ns the stage holds mass 0
            for (int k = 0; k < ns; k += G) {
                const float4 s0 = sw[k + gr];
#pragma unroll
                for (int u = 0; u < T; ++u) {
                    const float dx = me[u].x - s0.x, dy = me[u].y - s0.y;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
                    const float sm = s0.z * __builtin_amdgcn_rcpf(r2);
                    fx[u] = fmaf(sm, dx, fx[u]);
                    fy[u] = fmaf(sm, dy, fy[u]);
                }
            }
        }
    }
    wave_lds_sync();  // the previous chunk's sums have been read
#pragma unroll
    for (int u = 0; u < T; ++u) rw[lane * T + u] = make_float2(fx[u], fy[u]);
    wave_lds_sync();
    // one target per lane: target k = r' + u' L is lane k, which adds the
    // groups' sums of lane (g, r') slot u' in group order (u' = k / L as above)
    if (lane < n) {
        const int uk = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)L)), rk = lane - uk * L;
        float2 a = rw[rk * T + uk];
        for (int g = 1; g < G; ++g) {
            const float2 q = rw[(g * L + rk) * T + uk];
            a.x += q.x;
            a.y += q.y;
        }
        near[t0 + lane] = a;
        pleaf[t0 + lane] = li;
    }
}

// k_p2p: the near field of every particle over its leaf's U list (sorted
// particle order, one float2 per particle).  It needs only the lists, so it
// runs beside the upward pass and M2L.  Eight waves per SIMD: the bound
// keeps the registers at 64 (the eight-target lane groups would take 95 and
// leave five waves in flight).
__global__ __launch_bounds__(256, 8) void k_p2p(TreeView t, const float4 *__restrict__ part,
                                                const int64_t *__restrict__ offUW, const int2 *__restrict__ U,
                                                const int32_t *__restrict__ nU, const int32_t *__restrict__ cbeg,
                                                const int32_t *__restrict__ cend,
                                                const int32_t *__restrict__ leaf_cell, float2 *__restrict__ near,
                                                int32_t *__restrict__ pleaf)
{
    // per wave: the sources of the lane-group path (zero-mass padded), then
    // the lane groups' partial sums
    __shared__ __align__(16) unsigned char lds[4][P2P_WAVE_LDS];
    const int nleaves = t.counts[1];
    const int lane = lane_id();
    const int wpb = blockDim.x / WAVE;
    float4 *sw = reinterpret_cast<float4 *>(lds[threadIdx.x / WAVE]);
    float2 *rw = reinterpret_cast<float2 *>(lds[threadIdx.x / WAVE]);
    const int first = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (int)threadIdx.x / WAVE);
    for (int li = first; li < nleaves; li += gridDim.x * wpb) {
        const int c = leaf_cell[li];
        const int b = cbeg[c], e = cend[c];
        const int64_t ou0 = offUW[li];
        const int u0 = (int)(ou0 & 0xFFFFFFFFll), u1 = u0 + nU[li];
        for (int t0 = b; t0 < e; t0 += WAVE) {
            const int ntc = min(WAVE, e - t0);
            int T, L, G, S;
            p2p_shape(ntc, T, L, G, S);
            if (G > 1) {
                switch (T) {
                case 1: p2p_groups<1>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                case 2: p2p_groups<2>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                case 3: p2p_groups<3>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                case 4: p2p_groups<4>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                case 5: p2p_groups<5>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                case 6: p2p_groups<6>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                case 7: p2p_groups<7>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                default: p2p_groups<8>(part, U, u0, u1, t0, ntc, L, G, S, sw, rw, near, pleaf, li); break;
                }
                continue;
            }
            // one target per lane, the whole wave on each source: sources at
            // wave-uniform addresses (scalar loads, SGPR operands)
            const bool valid = lane < ntc;
            const float4 me = part[t0 + (valid ? lane : 0)];
            float fx = 0.f, fy = 0.f;
            for (int ue = u0; ue < u1; ++ue) {
                const int2 rg = U[ue];
                const int sb = rg.x, se = rg.y;
                int j = sb;
                for (; j + 4 <= se; j += 4) {
                    const float4 s0 = part[j], s1 = part[j + 1], s2 = part[j + 2], s3 = part[j + 3];
                    FL_P2P_PAIR(s0.x, s0.y, s0.z)
                    FL_P2P_PAIR(s1.x, s1.y, s1.z)
                    FL_P2P_PAIR(s2.x, s2.y, s2.z)
                    FL_P2P_PAIR(s3.x, s3.y, s3.z)
                }
                for (; j < se; ++j) {
                    const float4 s0 = part[j];
                    FL_P2P_PAIR(s0.x, s0.y, s0.z)
                }
            }
            if (valid) {
                near[t0 + lane] = make_float2(fx, fy);
                pleaf[t0 + lane] = li;
            }
        }
    }
}

// k_far: far field of every particle from its leaf's incoming expansion
// (L2P) and the W list's outgoing expansions (M2P), added to the near field;
// one thread per particle (sorted order), its leaf from the near-field pass.
// A wave then holds 64 particles of one or two leaves, so every lane works
// and the leaf data it shares arrives once through the caches.
template <int P>
__global__ __launch_bounds__(256) void k_far(TreeView t, int n, const float4 *__restrict__ part,
                                             const float2 *__restrict__ M, const float2 *__restrict__ Lleaf,
                                             const int64_t *__restrict__ offUW, const int32_t *__restrict__ W,
                                             const int32_t *__restrict__ leaf_cell, const int32_t *__restrict__ pleaf,
                                             const float2 *__restrict__ near, float kr, float2 *__restrict__ fr)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int li = pleaf[k];
        const int c = leaf_cell[li];
        const float4 me = part[k];
        const float2 nf = near[k];
        const int w0 = (int)(offUW[li] >> 32), w1 = (int)(offUW[li + 1] >> 32);
        const CellGeo g = geo(t, c);
        const double inv_w = g.iw;
        const float2 *Lc = Lleaf + (int64_t)li * (P + 1);
        // far field: incoming expansion of the leaf (Horner in the scaled variable)
        const float2 v =
            make_float2((float)(((double)me.x - g.cx) * inv_w), (float)(((double)me.y - g.cy) * inv_w));
        float2 acc = cscale(Lc[P], (float)P);
#pragma unroll
        for (int l = P - 1; l >= 1; --l) acc = cadd(cmul(acc, v), cscale(Lc[l], (float)l));
        float2 dphi = cscale(acc, (float)inv_w);
        // W list: outgoing expansions of small separated cells at the particle
        for (int we = w0; we < w1; ++we) {
            const int s = W[we];
            const CellGeo gs = geo(t, s);
            const double inv_ws = gs.iw;
            const float2 tt = crecip(make_float2((float)(((double)me.x - gs.cx) * inv_ws),
                                                 (float)(((double)me.y - gs.cy) * inv_ws)));
            const float2 *Ms = M + (int64_t)s * (P + 1);
            float2 sum = make_float2(Ms[0].x, 0.f);
            float2 pw = tt;
#pragma unroll
            for (int q = 1; q <= P; ++q) {
                const float2 tk = cmul(Ms[q], pw);
                sum.x -= (float)q * tk.x;
                sum.y -= (float)q * tk.y;
                pw = cmul(pw, tt);
            }
            dphi = cadd(dphi, cscale(cmul(tt, sum), (float)inv_ws));
        }
        // F = kr m_i (conj(phi'_far) + near field)
        const float km = kr * me.z;
        const int orig = __float_as_int(me.w);
        fr[orig] = make_float2(km * (dphi.x + nf.x), km * (nf.y - dphi.y));  // one 8-byte store per node
    }
}
#undef FL_P2P_PAIR

template <int P>
struct FmmBufs {
    float2 *M, *Lp, *Ll, *T;
    bool fresh;  // the M2M table still has to be written
};

template <int P>
FmmBufs<P> fmm_bufs(fl_ctx *c, const TreeBufs &t)
{
    FmmBufs<P> b;
    b.M = ws<float2>(c, "f_M", (size_t)t.cells_cap * (P + 1));
    b.Lp = ws<float2>(c, "f_Lp", (size_t)t.cells_cap * (P + 1));
    b.Ll = ws<float2>(c, "f_Lleaf", (size_t)t.leaves_cap * (P + 1));
    std::string tn = "f_m2m_T" + std::to_string(P);
    auto it = c->bufs.find(tn);
    b.fresh = it == c->bufs.end() || !it->second.p;
    b.T = ws<float2>(c, tn.c_str(), 4 * (P + 1) * (P + 1));
    return b;
}

// upward pass: outgoing expansions of the leaves, shifted up to the root
template <int P>
void upward_p(fl_ctx *c, hipStream_t s, const TreeBufs &t, const FmmBufs<P> &b)
{
    TreeView tv = view(t);
    if (b.fresh) hipLaunchKernelGGL(k_m2m_table<P>, dim3(1), dim3(256), 0, s, b.T);
    hipLaunchKernelGGL(k_p2m<P>, dim3(grid_for(t.leaves_cap, 4, 16384)), dim3(256), 0, s, tv, (const float4 *)t.part,
                       (const int32_t *)t.leaf_cell, b.M);
    const int64_t nsub = (int64_t)t.s.K << (2 * M2M_CUT);
    hipLaunchKernelGGL(k_m2m_sub<P>, dim3((unsigned)std::min<int64_t>(nsub, 2048)), dim3(256), 0, s, tv,
                       (const float2 *)b.T, b.M);
    hipLaunchKernelGGL(k_m2m_top<P>, dim3((unsigned)std::min(t.s.K, 1024)), dim3(256), 0, s, tv, (const float2 *)b.T,
                       b.M);
    FL_LAUNCH_CHECK();
}

// incoming expansions: M2L and P2L into every cell, L2L down to the leaves
template <int P>
void m2l_p(fl_ctx *c, hipStream_t s, const TreeBufs &t, const ListBufs &L, const FmmBufs<P> &b)
{
    TreeView tv = view(t);
    hipLaunchKernelGGL(k_m2l<P>, dim3(grid_for(t.cells_cap, 8, 16384)), dim3(256), 0, s, tv, (const float4 *)t.part,
                       b.M, L.offVX, L.V, L.X, b.Lp);
    hipLaunchKernelGGL(k_l2l<P>, dim3(grid_for(t.leaves_cap, 256, 2048)), dim3(256), 0, s, tv, b.Lp, b.Ll);
    FL_LAUNCH_CHECK();
}

// near field (P2P) of every particle: about one wave per leaf (4 waves per
// block): leaves differ a lot in cost, and the dispatcher balances
// single-leaf waves far better than a fixed stride of several per wave
void near_p(fl_ctx *c, const TreeBufs &t, const ListBufs &L, float2 *near, int32_t *pleaf)
{
    TreeView tv = view(t);
    hipLaunchKernelGGL(k_p2p, dim3(grid_for(t.leaves_cap, 4, 16384)), dim3(256), 0, c->stream, tv,
                       (const float4 *)t.part, L.offUW, (const int2 *)L.U, (const int32_t *)L.nU,
                       (const int32_t *)t.beg, (const int32_t *)t.end, (const int32_t *)t.leaf_cell, near, pleaf);
    FL_LAUNCH_CHECK();
}

template <int P>
void far_p(fl_ctx *c, const TreeBufs &t, const ListBufs &L, const FmmBufs<P> &b, const float2 *near,
           const int32_t *pleaf, float kr, float2 *fr)
{
    TreeView tv = view(t);
    hipLaunchKernelGGL(k_far<P>, dim3(grid_for(t.n, 256, 16384)), dim3(256), 0, c->stream, tv, t.n,
                       (const float4 *)t.part,
                       (const float2 *)b.M, (const float2 *)b.Ll, L.offUW, (const int32_t *)L.W,
                       (const int32_t *)t.leaf_cell, pleaf, near, kr, fr);
    FL_LAUNCH_CHECK();
}

// The lists and the upward pass need only the tree; the near field needs
// only the lists, M2L both.  Unless phases are being timed (or the
// context's branches are off), the upward pass, then M2L and L2L, run on a
// branch stream while the main stream builds the lists and evaluates the
// near field; the far field joins the two (events; recorded as parallel
// branches under capture).
template <int P>
void fmm_passes(fl_ctx *c, const TreeBufs &t, int lanes, float kr, float2 *fr,
                const ListsHook *on_lists)
{
    ListBufs L;
    const FmmBufs<P> b = fmm_bufs<P>(c, t);
    float2 *near = ws<float2>(c, "f_near", (size_t)t.n);
    int32_t *pleaf = ws<int32_t>(c, "f_pleaf", (size_t)t.n);
    if (c->timing || !c->branches) {
        {
            PhaseTimer pt(c, FL_PH_LISTS);
            build_lists(c, t, L, lanes);
            lists_stats(c, t, L);
        }
        if (on_lists) {
            if (!c->ev_lists) FL_CHECK_HIP(hipEventCreateWithFlags(&c->ev_lists, hipEventDisableTiming));
            FL_CHECK_HIP(hipEventRecord(c->ev_lists, c->stream));
            (*on_lists)(c->ev_lists, [](hipStream_t) {});
        }
        {
            PhaseTimer pt(c, FL_PH_UPWARD);
            upward_p<P>(c, c->stream, t, b);
        }
        {
            PhaseTimer pt(c, FL_PH_M2L);
            m2l_p<P>(c, c->stream, t, L, b);
        }
        {
            PhaseTimer pt(c, FL_PH_EVAL);
            near_p(c, t, L, near, pleaf);
        }
    } else {
        hipStream_t us = aux_stream(c, 3);
        for (hipEvent_t *e : {&c->ev_fork2, &c->ev_join2, &c->ev_lists})
            if (!*e) FL_CHECK_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
        FL_CHECK_HIP(hipEventRecord(c->ev_fork2, c->stream));
        FL_CHECK_HIP(hipStreamWaitEvent(us, c->ev_fork2, 0));
        upward_p<P>(c, us, t, b);
        build_lists(c, t, L, lanes);
        FL_CHECK_HIP(hipEventRecord(c->ev_lists, c->stream));
        // the near field is enqueued (recorded) first among the list build's
        // successors: graph replay dispatched it after M2L and L2L otherwise
        near_p(c, t, L, near, pleaf);
        FL_CHECK_HIP(hipStreamWaitEvent(us, c->ev_lists, 0));
        // the statistics (for the host only) on the other branch when there
        // is one: ahead of M2L they delayed the far field, which waits for
        // M2L and L2L; else ahead of M2L rather than between the near field
        // and the far field
        if (on_lists)
            (*on_lists)(c->ev_lists, [&](hipStream_t s) { lists_stats(c, t, L, s); });
        else
            lists_stats(c, t, L, us);
        m2l_p<P>(c, us, t, L, b);
        FL_CHECK_HIP(hipEventRecord(c->ev_join2, us));
        FL_CHECK_HIP(hipStreamWaitEvent(c->stream, c->ev_join2, 0));
    }
    PhaseTimer pt(c, FL_PH_FAR);
    far_p<P>(c, t, L, b, near, pleaf, kr, fr);
}

}  // namespace

bool fmm_order_supported(int p) { return p == 4 || p == 6 || p == 8 || p == 10 || p == 12 || p == 16; }

void fmm_repulsion(fl_ctx *c, const Segs &s, const float *x, const float *y, const int32_t *deg, int p, int leaf,
                   int bits, int lanes, float kr, float2 *fr, const ListsHook *on_lists,
                   float2 *xy_out, BBoxIn bb)
{
    TreeBufs t;
    {
        PhaseTimer pt(c, FL_PH_TREE);
        build_tree(c, t, s, x, y, deg, bits, leaf, xy_out, bb);
    }
    switch (p) {
    case 4: fmm_passes<4>(c, t, lanes, kr, fr, on_lists); break;
    case 6: fmm_passes<6>(c, t, lanes, kr, fr, on_lists); break;
    case 8: fmm_passes<8>(c, t, lanes, kr, fr, on_lists); break;
    case 10: fmm_passes<10>(c, t, lanes, kr, fr, on_lists); break;
    case 12: fmm_passes<12>(c, t, lanes, kr, fr, on_lists); break;
    case 16: fmm_passes<16>(c, t, lanes, kr, fr, on_lists); break;
    default: throw Error(FL_EUNSUPPORTED, "FMM expansion order not built (use 4, 6, 8, 10, 12 or 16)");
    }
}

}  // namespace fl
