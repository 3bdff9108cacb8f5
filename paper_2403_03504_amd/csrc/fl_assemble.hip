// Assembly of the component layouts into one drawing (paper sec. 4): rescale
// every component to a common density, link the components into a tree (the
// meta-graph), lay the tree out by Kamada-Kawai, and, when it is too large for
// one layout, cut it into groups that are laid out separately and assembled
// again one level up.
//
//   k_asm_sums     one wave per tile (<= ASM_TILE nodes of one component):
//                  FP64 sums of x and y
//   k_asm_centre   one thread per component: its centroid from its tiles
//   k_asm_moments  one wave per tile: FP64 sum and maximum of |p - c|^2
//   k_asm_frames   one thread per component: scale and radius, written into
//                  the component's slot of the first level (its place in the
//                  random order)
//   k_asm_level    one workgroup per group of <= 256 items (one wave per 64):
//                  meta-graph links by a prefix maximum, path lengths in
//                  closed form, the starting layout, sequential majorization
//                  sweeps, then the group's node count, centre and radius as
//                  an item of the next level
//   k_asm_shift    one thread per item, top level first: its translation
//   k_asm_place    one wave per tile: p -> s (p - c) + shift
//   k_asm_export   one thread per component: frames and first-level links
//
// The meta-graph of a group is a chain of "records" (items with more nodes
// than every earlier item, each linked to the record before it) with every
// other item hanging off the record current when it arrives.  The path length
// between items i != j is therefore L_i + L_j + |h_i - h_j|, where L is the
// length of the item's own edge if it hangs off a record (0 for a record) and
// h the chain length from the group's first item to the item's record, so no
// distance matrix is stored: each lane keeps one item in registers, the
// moving item is read from LDS, and a sweep is g sequential item moves, each
// one reduction over the workgroup.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "fl_fa2.h"

namespace fl {
namespace {

constexpr int ASM_TILE = 2048;
constexpr int ASM_MAX = 256;
constexpr int ASM_Q = ASM_MAX / WAVE;
constexpr int ASM_WPB = 4;  // waves per block of the per-tile kernels

__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ float read_lane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double read_lane(double v, int l)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xFFFFFFFFull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(256) void k_asm_label_check(const int32_t *__restrict__ label, int n,
                                                         int32_t *__restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (label[i] < 0 || label[i] >= n)) atomicOr(err, 1);
}

__global__ __launch_bounds__(256) void k_asm_sums(const int2 *__restrict__ tiles, int ntiles,
                                                  const int32_t *__restrict__ coff, const float *__restrict__ x,
                                                  const float *__restrict__ y, double2 *__restrict__ part)
{
    const int t = blockIdx.x * ASM_WPB + (int)(threadIdx.x / WAVE);
    if (t >= ntiles) return;  // wave-uniform
    const int2 tl = tiles[t];
    const int e = min(tl.y + ASM_TILE, coff[tl.x + 1]);
    double sx = 0.0, sy = 0.0;
    for (int i = tl.y + lane_id(); i < e; i += WAVE) {
        sx += (double)x[i];
        sy += (double)y[i];
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane_id() == 0) part[t] = make_double2(sx, sy);
}

__global__ __launch_bounds__(256) void k_asm_centre(int K, const int32_t *__restrict__ coff,
                                                    const int32_t *__restrict__ toff,
                                                    const double2 *__restrict__ part, double2 *__restrict__ cen)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double sx = 0.0, sy = 0.0;
    for (int t = toff[k]; t < toff[k + 1]; ++t) {
        sx += part[t].x;
        sy += part[t].y;
    }
    const double n = (double)(coff[k + 1] - coff[k]);
    cen[k] = make_double2(sx / n, sy / n);
}

__global__ __launch_bounds__(256) void k_asm_moments(const int2 *__restrict__ tiles, int ntiles,
                                                     const int32_t *__restrict__ coff, const float *__restrict__ x,
                                                     const float *__restrict__ y, const double2 *__restrict__ cen,
                                                     double2 *__restrict__ part)
{
    const int t = blockIdx.x * ASM_WPB + (int)(threadIdx.x / WAVE);
    if (t >= ntiles) return;
    const int2 tl = tiles[t];
    const int e = min(tl.y + ASM_TILE, coff[tl.x + 1]);
    const double2 c = cen[tl.x];
    double s2 = 0.0, m2 = 0.0;
    for (int i = tl.y + lane_id(); i < e; i += WAVE) {
        const double dx = (double)x[i] - c.x, dy = (double)y[i] - c.y;
        const double r2 = dx * dx + dy * dy;
        s2 += r2;
        m2 = fmax(m2, r2);
    }
    s2 = wave_sum(s2);
    m2 = wave_max_d(m2);
    if (lane_id() == 0) part[t] = make_double2(s2, m2);
}

__global__ __launch_bounds__(256) void k_asm_frames(int K, const int32_t *__restrict__ coff,
                                                    const int32_t *__restrict__ toff,
                                                    const double2 *__restrict__ part, const int32_t *__restrict__ inv,
                                                    double density, double *__restrict__ scale,
                                                    double *__restrict__ rad, int32_t *__restrict__ iw,
                                                    double *__restrict__ ir)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double s2 = 0.0, m2 = 0.0;
    for (int t = toff[k]; t < toff[k + 1]; ++t) {
        s2 += part[t].x;
        m2 = fmax(m2, part[t].y);
    }
    const int nk = coff[k + 1] - coff[k];
    const double rho = sqrt(s2 / (double)nk);
    const double s = rho > 0.0 ? sqrt((double)nk / (2.0 * M_PI * density)) / rho : 1.0;
    const double R = s * sqrt(m2);
    scale[k] = s;
    rad[k] = R;
    const int slot = inv[k];
    iw[slot] = nk;
    ir[slot] = R;
}

// Wave total of v by DPP: inclusive sums inside rows of 16 lanes (row_shr 1,
// 2, 4, 8; lanes shifted in from outside the row add 0), then the totals of
// the rows before by row_bcast 15 and 31.  Only lane 63 holds the total.
__device__ __forceinline__ float dpp_total_in_lane63(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return v;
}

// One group: items [a, a + g) of the level, g <= ASM_MAX, NW waves (item j
// lives on lane j % 64 of wave j / 64).  Wave 0 builds the meta-graph and the
// starting layout into LDS; then every item move is one step of all waves:
// partial sums over their items, a DPP wave total, and (NW > 1) the wave
// totals exchanged through LDS and added in wave order, so every wave gets
// the same new position.
template <int NW>
__global__ __launch_bounds__(NW * WAVE) void k_asm_level(int m, int M, const int32_t *__restrict__ iw,
                                                         const double *__restrict__ ir, double gap, int sweeps,
                                                         double2 *__restrict__ P, int32_t *__restrict__ par_out,
                                                         int32_t *__restrict__ nw, double2 *__restrict__ nc,
                                                         double *__restrict__ nr)
{
    __shared__ double Rs[ASM_MAX];
    __shared__ double hs[ASM_MAX];
    __shared__ float Ls[ASM_MAX];
    __shared__ float2 pos[ASM_MAX];
    __shared__ int32_t ps[ASM_MAX];
    __shared__ float part[2][NW][2];
    const int grp = blockIdx.x;
    const int a = grp * M;
    const int g = min(M, m - a);
    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / WAVE);

    for (int t = (int)threadIdx.x; t < g; t += NW * WAVE) Rs[t] = ir[a + t];
    __syncthreads();
    if (wv == 0) {
        int wq[ASM_Q];
        double Rq[ASM_Q];
#pragma unroll
        for (int q = 0; q < ASM_Q; ++q) {
            const int t = lane + WAVE * q;
            wq[q] = t < g ? iw[a + t] : 0;
            Rq[q] = t < g ? Rs[t] : 0.0;
        }
        // links: the largest earlier item (first on a tie) is the maximum of
        // key = nodes << 32 | ~t over the items before t
        int parq[ASM_Q];
        bool recq[ASM_Q];
        unsigned long long kcarry = 0ull;
#pragma unroll
        for (int q = 0; q < ASM_Q; ++q) {
            const int t = lane + WAVE * q;
            const unsigned long long key =
                t < g ? (((unsigned long long)(unsigned)wq[q] << 32) | (unsigned long long)(~(unsigned)t)) : 0ull;
            unsigned long long inc = key;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const unsigned long long v = __shfl_up(inc, o, WAVE);
                if (lane >= o) inc = inc > v ? inc : v;
            }
            unsigned long long exc = __shfl_up(inc, 1, WAVE);
            if (lane == 0) exc = 0ull;
            exc = exc > kcarry ? exc : kcarry;
            const unsigned long long last = __shfl(inc, WAVE - 1, WAVE);
            kcarry = kcarry > last ? kcarry : last;
            parq[q] = t == 0 ? -1 : (int)(~(unsigned)(exc & 0xFFFFFFFFull));
            recq[q] = t == 0 || key > exc;
        }
        // edge lengths, leg lengths L, chain positions h (FP64 prefix sum),
        // starting layout
        double hcarry = 0.0;
#pragma unroll
        for (int q = 0; q < ASM_Q; ++q) {
            const int t = lane + WAVE * q;
            const double e = (t < g && t > 0) ? Rq[q] + Rs[parq[q]] + gap : 0.0;
            const double inc = wave_incl_scan(recq[q] ? e : 0.0);
            const double h = hcarry + inc;
            hcarry += __shfl(inc, WAVE - 1, WAVE);
            const double leg = recq[q] ? 0.0 : e;
            const double d0 = leg + h;  // path length from item 0
            double sn, cs;
            sincos(2.0 * M_PI * (double)t / (double)g, &sn, &cs);
            if (t < g) {
                hs[t] = h;
                Ls[t] = (float)leg;
                pos[t] = make_float2((float)(d0 * cs), (float)(d0 * sn));
                ps[t] = parq[q];
            }
        }
    }
    __syncthreads();

    // sequential majorization sweeps.  Lane j holds item j; the moving item
    // i comes from registers (one wave) or LDS (several waves), fetched one
    // move ahead (item i + 1 does not move during move i).  1 / sum_j w_ij is
    // fixed over the sweeps and computed once.
    const int j = wv * WAVE + lane;
    const bool live = j < g;
    float xj = 0.f, yj = 0.f, Lj = 0.f;
    double hj = 0.0;
    if (live) {
        xj = pos[j].x;
        yj = pos[j].y;
        Lj = Ls[j];
        hj = hs[j];
    }
    float rswj = 0.f;  // 1 / sum_k w_jk of item j
    if (g > 1 && sweeps > 0) {
        for (int i = 0; i < g; ++i) {
            float Li;
            double hi;
            if constexpr (NW == 1) {
                Li = read_lane(Lj, i);
                hi = read_lane(hj, i);
            } else {
                Li = Ls[i];
                hi = hs[i];
            }
            float sw = 0.f;
            if (live && j != i) {
                const float D = Li + Lj + (float)fabs(hi - hj);
                sw = __builtin_amdgcn_rcpf(D * D);
            }
            sw = dpp_total_in_lane63(sw);
            if constexpr (NW == 1) {
                sw = read_lane(sw, WAVE - 1);
            } else {
                const int b = i & 1;
                if (lane == WAVE - 1) part[b][wv][0] = sw;
                __syncthreads();
                sw = part[b][0][0];
#pragma unroll
                for (int u = 1; u < NW; ++u) sw += part[b][u][0];
            }
            if (j == i) rswj = 1.0f / sw;
        }
    }
    for (int s = 0; s < sweeps && g > 1; ++s) {
        float2 pn;
        float Ln;
        double hn;
        if constexpr (NW > 1) {
            pn = pos[0];
            Ln = Ls[0];
            hn = hs[0];
        }
        for (int i = 0; i < g; ++i) {
            float2 pi;
            float Li;
            double hi;
            if constexpr (NW == 1) {
                pi = make_float2(read_lane(xj, i), read_lane(yj, i));
                Li = read_lane(Lj, i);
                hi = read_lane(hj, i);
            } else {
                pi = pn;
                Li = Ln;
                hi = hn;
                const int i1 = i + 1 < g ? i + 1 : 0;
                pn = pos[i1];
                Ln = Ls[i1];
                hn = hs[i1];
            }
            float ax = 0.f, ay = 0.f;
            if (live && j != i) {
                const float D = Li + Lj + (float)fabs(hi - hj);
                const float w = __builtin_amdgcn_rcpf(D * D);
                const float dx = pi.x - xj, dy = pi.y - yj;
                const float r2 = dx * dx + dy * dy;
                const float rinv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
                const float wd = w * D * rinv;
                ax = w * xj + wd * dx;
                ay = w * yj + wd * dy;
            }
            ax = dpp_total_in_lane63(ax);
            ay = dpp_total_in_lane63(ay);
            if constexpr (NW == 1) {
                ax = read_lane(ax, WAVE - 1);
                ay = read_lane(ay, WAVE - 1);
            } else {
                const int b = i & 1;
                if (lane == WAVE - 1) {
                    part[b][wv][0] = ax;
                    part[b][wv][1] = ay;
                }
                __syncthreads();
                if (j == i) {
                    ax = part[b][0][0];
                    ay = part[b][0][1];
#pragma unroll
                    for (int u = 1; u < NW; ++u) {
                        ax += part[b][u][0];
                        ay += part[b][u][1];
                    }
                }
            }
            if (j == i) {
                xj = ax * rswj;
                yj = ay * rswj;
                if constexpr (NW > 1) pos[i] = make_float2(xj, yj);
            }
        }
    }
    if constexpr (NW == 1) {
        if (live) pos[j] = make_float2(xj, yj);
    }
    __syncthreads();

    // placements, first-level links, and the group as a next-level item
    if (wv != 0) return;
    long long W = 0;
    double cx = 0.0, cy = 0.0;
    float2 pq[ASM_Q];
    double Rq[ASM_Q];
#pragma unroll
    for (int q = 0; q < ASM_Q; ++q) {
        const int t = lane + WAVE * q;
        pq[q] = t < g ? pos[t] : make_float2(0.f, 0.f);
        Rq[q] = t < g ? Rs[t] : 0.0;
        if (t < g) {
            const int wt = iw[a + t];
            P[a + t] = make_double2((double)pq[q].x, (double)pq[q].y);
            if (par_out) par_out[a + t] = ps[t] < 0 ? -1 : a + ps[t];
            W += wt;
            cx += (double)wt * (double)pq[q].x;
            cy += (double)wt * (double)pq[q].y;
        }
    }
    W = wave_sum(W);
    cx = wave_sum(cx) / (double)W;
    cy = wave_sum(cy) / (double)W;
    double rg = 0.0;
#pragma unroll
    for (int q = 0; q < ASM_Q; ++q) {
        const int t = lane + WAVE * q;
        if (t < g) {
            const double dx = (double)pq[q].x - cx, dy = (double)pq[q].y - cy;
            rg = fmax(rg, sqrt(dx * dx + dy * dy) + Rq[q]);
        }
    }
    rg = wave_max_d(rg);
    if (lane == 0) {
        nw[grp] = (int32_t)W;
        nc[grp] = make_double2(cx, cy);
        nr[grp] = rg;
    }
}

// F[t] = P[t] - C[t] + (translation of the group holding t); the top level's
// group is moved by minus its centre, so the drawing is centred.
__global__ __launch_bounds__(256) void k_asm_shift(int m, int M, const double2 *__restrict__ P,
                                                   const double2 *__restrict__ C, const double2 *__restrict__ Fup,
                                                   const double2 *__restrict__ ctop, double2 *__restrict__ F)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    double2 f = P[t];
    if (C) {
        f.x -= C[t].x;
        f.y -= C[t].y;
    }
    if (ctop) {
        f.x -= ctop[0].x;
        f.y -= ctop[0].y;
    } else {
        const double2 u = Fup[t / M];
        f.x += u.x;
        f.y += u.y;
    }
    F[t] = f;
}

__global__ __launch_bounds__(256) void k_asm_place(const int2 *__restrict__ tiles, int ntiles,
                                                   const int32_t *__restrict__ coff, const double2 *__restrict__ cen,
                                                   const double *__restrict__ scale, const int32_t *__restrict__ inv,
                                                   const double2 *__restrict__ F, float *__restrict__ x,
                                                   float *__restrict__ y)
{
    const int t = blockIdx.x * ASM_WPB + (int)(threadIdx.x / WAVE);
    if (t >= ntiles) return;
    const int2 tl = tiles[t];
    const int e = min(tl.y + ASM_TILE, coff[tl.x + 1]);
    const double2 c = cen[tl.x];
    const double s = scale[tl.x];
    const double2 f = F[inv[tl.x]];
    for (int i = tl.y + lane_id(); i < e; i += WAVE) {
        x[i] = (float)(s * ((double)x[i] - c.x) + f.x);
        y[i] = (float)(s * ((double)y[i] - c.y) + f.y);
    }
}

__global__ __launch_bounds__(256) void k_asm_export(int K, const double2 *__restrict__ cen,
                                                    const double *__restrict__ scale, const double *__restrict__ rad,
                                                    const int32_t *__restrict__ inv, const int32_t *__restrict__ order,
                                                    const double2 *__restrict__ F, const int32_t *__restrict__ par0,
                                                    double *__restrict__ frame, int32_t *__restrict__ parent)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int slot = inv[k];
    if (frame) {
        double *o = frame + 6 * (int64_t)k;
        o[0] = cen[k].x;
        o[1] = cen[k].y;
        o[2] = scale[k];
        o[3] = rad[k];
        o[4] = F[slot].x;
        o[5] = F[slot].y;
    }
    if (parent) {
        const int p = par0[slot];
        parent[k] = p < 0 ? -1 : order[p];
    }
}

__global__ __launch_bounds__(256) void k_asm_gather(const int32_t *__restrict__ perm, int n, const float *__restrict__ x,
                                                    const float *__restrict__ y, float *__restrict__ xs,
                                                    float *__restrict__ ys)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    xs[r] = x[perm[r]];
    ys[r] = y[perm[r]];
}

__global__ __launch_bounds__(256) void k_asm_scatter(const int32_t *__restrict__ perm, int n,
                                                     const float *__restrict__ xs, const float *__restrict__ ys,
                                                     float *__restrict__ x, float *__restrict__ y)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    x[perm[r]] = xs[r];
    y[perm[r]] = ys[r];
}

void check_params(const fl_assemble_params *p)
{
    FL_REQUIRE(p, "fl_assemble: parameters missing");
    FL_REQUIRE(std::isfinite(p->density) && p->density > 0.0, "fl_assemble: density must be > 0");
    FL_REQUIRE(std::isfinite(p->gap) && p->gap > 0.0, "fl_assemble: gap must be > 0");
    FL_REQUIRE(p->max_group >= 2 && p->max_group <= ASM_MAX, "fl_assemble: max_group must be in [2, 256]");
    FL_REQUIRE(p->sweeps >= 0, "fl_assemble: sweeps must be >= 0");
}

}  // namespace

// Components are the node ranges [off[k], off[k+1]) of x, y (device copy
// d_off); order [host] is the random order.  Synchronises.
void assemble_ranges(fl_ctx *c, const std::vector<int32_t> &off, const int32_t *d_off, float *x, float *y,
                     const std::vector<int32_t> &order, const fl_assemble_params &prm, double *frame,
                     int32_t *parent, fl_assemble_stats *st)
{
    const int K = (int)off.size() - 1;
    FL_REQUIRE(K >= 1 && (int)order.size() == K, "fl_assemble: order must have one entry per component");
    std::vector<int32_t> inv(K, -1);
    for (int t = 0; t < K; ++t) {
        const int k = order[t];
        FL_REQUIRE(k >= 0 && k < K && inv[k] < 0, "fl_assemble: order must be a permutation of 0..n_comp-1");
        inv[k] = t;
    }
    std::vector<int2> tiles;
    std::vector<int32_t> toff(K + 1);
    for (int k = 0; k < K; ++k) {
        FL_REQUIRE(off[k + 1] > off[k], "fl_assemble: empty component");
        toff[k] = (int32_t)tiles.size();
        for (int64_t b = off[k]; b < off[k + 1]; b += ASM_TILE) tiles.push_back(make_int2(k, (int)b));
    }
    toff[K] = (int32_t)tiles.size();
    const int ntiles = (int)tiles.size();
    const int M = prm.max_group;
    std::vector<int64_t> m{K};
    while (m.back() > M) m.push_back((m.back() + M - 1) / M);
    const int L = (int)m.size();
    std::vector<int64_t> lo(L + 2, 0);
    for (int l = 0; l < L; ++l) lo[l + 1] = lo[l] + m[l];
    lo[L + 1] = lo[L] + 1;  // the top group as an item
    const int64_t tot = lo[L + 1];
    int64_t groups = 0;
    for (int l = 0; l < L; ++l) groups += (m[l] + M - 1) / M;

    int2 *d_tiles = ws<int2>(c, "asm_tiles", (size_t)ntiles);
    int32_t *d_toff = ws<int32_t>(c, "asm_toff", (size_t)K + 1);
    int32_t *d_order = ws<int32_t>(c, "asm_order", (size_t)K);
    int32_t *d_inv = ws<int32_t>(c, "asm_inv", (size_t)K);
    double2 *part = ws<double2>(c, "asm_part", (size_t)ntiles);
    double2 *cen = ws<double2>(c, "asm_cen", (size_t)K);
    double *scale = ws<double>(c, "asm_scale", (size_t)K);
    double *rad = ws<double>(c, "asm_rad", (size_t)K);
    int32_t *iw = ws<int32_t>(c, "asm_iw", (size_t)tot);
    double *ir = ws<double>(c, "asm_ir", (size_t)tot);
    double2 *ic = ws<double2>(c, "asm_ic", (size_t)tot);
    double2 *P = ws<double2>(c, "asm_P", (size_t)tot);
    double2 *F = ws<double2>(c, "asm_F", (size_t)tot);
    int32_t *par0 = ws<int32_t>(c, "asm_par0", (size_t)K);
    FL_CHECK_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int2) * ntiles, hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(d_toff, toff.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(d_inv, inv.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, c->stream));

    const unsigned gt = grid_for(ntiles, ASM_WPB);
    const unsigned gk = grid_for(K, 256);
    hipLaunchKernelGGL(k_asm_sums, dim3(gt), dim3(256), 0, c->stream, (const int2 *)d_tiles, ntiles, d_off,
                       (const float *)x, (const float *)y, part);
    hipLaunchKernelGGL(k_asm_centre, dim3(gk), dim3(256), 0, c->stream, K, d_off, (const int32_t *)d_toff,
                       (const double2 *)part, cen);
    hipLaunchKernelGGL(k_asm_moments, dim3(gt), dim3(256), 0, c->stream, (const int2 *)d_tiles, ntiles, d_off,
                       (const float *)x, (const float *)y, (const double2 *)cen, part);
    hipLaunchKernelGGL(k_asm_frames, dim3(gk), dim3(256), 0, c->stream, K, d_off, (const int32_t *)d_toff,
                       (const double2 *)part, (const int32_t *)d_inv, prm.density, scale, rad, iw, ir);
    FL_LAUNCH_CHECK();
    for (int l = 0; l < L; ++l) {
        const unsigned ng = (unsigned)((m[l] + M - 1) / M);
        const int gmax = (int)std::min<int64_t>(M, m[l]);
        auto kern = gmax <= WAVE ? k_asm_level<1> : (gmax <= 2 * WAVE ? k_asm_level<2> : k_asm_level<4>);
        const int nwv = gmax <= WAVE ? 1 : (gmax <= 2 * WAVE ? 2 : 4);
        hipLaunchKernelGGL(kern, dim3(ng), dim3(nwv * WAVE), 0, c->stream, (int)m[l], M,
                           (const int32_t *)(iw + lo[l]), (const double *)(ir + lo[l]), prm.gap, prm.sweeps,
                           P + lo[l], l == 0 ? par0 : (int32_t *)nullptr, iw + lo[l + 1], ic + lo[l + 1],
                           ir + lo[l + 1]);
        FL_LAUNCH_CHECK();
    }
    for (int l = L - 1; l >= 0; --l) {
        const bool top = l == L - 1;
        hipLaunchKernelGGL(k_asm_shift, dim3(grid_for(m[l], 256)), dim3(256), 0, c->stream, (int)m[l], M,
                           (const double2 *)(P + lo[l]), l == 0 ? (const double2 *)nullptr : (const double2 *)(ic + lo[l]),
                           top ? (const double2 *)nullptr : (const double2 *)(F + lo[l + 1]),
                           top ? (const double2 *)(ic + lo[L]) : (const double2 *)nullptr, F + lo[l]);
        FL_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_asm_place, dim3(gt), dim3(256), 0, c->stream, (const int2 *)d_tiles, ntiles, d_off,
                       (const double2 *)cen, (const double *)scale, (const int32_t *)d_inv, (const double2 *)F, x, y);
    FL_LAUNCH_CHECK();
    if (frame || parent) {
        hipLaunchKernelGGL(k_asm_export, dim3(gk), dim3(256), 0, c->stream, K, (const double2 *)cen,
                           (const double *)scale, (const double *)rad, (const int32_t *)d_inv,
                           (const int32_t *)d_order, (const double2 *)F, (const int32_t *)par0, frame, parent);
        FL_LAUNCH_CHECK();
    }
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));  // host vectors outlive the async copies
    if (st) {
        st->n_comp = K;
        st->levels = L;
        st->groups = (int32_t)groups;
    }
}

}  // namespace fl

using namespace fl;

extern "C" {

void fl_assemble_default_params(fl_assemble_params *p)
{
    if (!p) return;
    p->density = 1.0;
    p->gap = 1.0;
    p->max_group = 256;
    p->sweeps = 100;
}

fl_status fl_assemble(fl_ctx *c, int32_t n, const int32_t *label, int32_t n_comp, const int32_t *order, float *x,
                      float *y, const fl_assemble_params *prm, double *frame, int32_t *parent,
                      fl_assemble_stats *stats)
{
    FL_API_BEGIN(c)
    const auto t0 = std::chrono::steady_clock::now();
    FL_REQUIRE(n >= 1 && label && order && x && y, "fl_assemble: bad arguments");
    FL_REQUIRE(n_comp >= 1 && n_comp <= n, "fl_assemble: need 1 <= n_comp <= n");
    check_params(prm);
    std::vector<int32_t> ord(order, order + n_comp);
    int32_t *err = ws<int32_t>(c, "asm_err", 1);
    fill_i32(c, err, 1, 0);
    hipLaunchKernelGGL(k_asm_label_check, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, label, n, err);
    FL_LAUNCH_CHECK();
    FL_REQUIRE(read_i32(c, err) == 0, "fl_assemble: a label lies outside [0, n)");
    LabelSort ls = sort_by_label(c, n, label, n_comp);
    float *xs = ws<float>(c, "asm_xs", n), *ys = ws<float>(c, "asm_ys", n);
    const unsigned g = grid_for(n, 256);
    hipLaunchKernelGGL(k_asm_gather, dim3(g), dim3(256), 0, c->stream, ls.perm, n, (const float *)x,
                       (const float *)y, xs, ys);
    FL_LAUNCH_CHECK();
    assemble_ranges(c, ls.off, ls.d_off, xs, ys, ord, *prm, frame, parent, stats);
    hipLaunchKernelGGL(k_asm_scatter, dim3(g), dim3(256), 0, c->stream, ls.perm, n, (const float *)xs,
                       (const float *)ys, x, y);
    FL_LAUNCH_CHECK();
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    if (stats) stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    FL_API_END(c)
}

}  // extern "C"
