// Kamada-Kawai for the small components (paper sec. 3.1, sec. 4).
//
//   k_kk_bfs    hop distances d_ij of one component (<= 256 nodes) per
//               workgroup: breadth-first search from every source at once.
//               Each node keeps bitsets over sources (visited, frontier) in
//               LDS; one level is next(v) = OR_{u in N(v)} frontier(u) minus
//               visited(v), and every source bit newly set in next(v) is the
//               distance d+1 of (source, v).  Unit weights, so this equals the
//               paper's Floyd-Warshall distances (exact integers).
//   k_kk_steps  localized stress majorization of the energy
//               E = sum_{i<j} d_ij^-2 (|p_i - p_j| - l d_ij)^2, all nodes of a
//               component updated together from the previous positions:
//                 p_i' = sum_{j!=i} w_ij (p_j + l d_ij u_ij) / sum_{j!=i} w_ij,
//               w_ij = d_ij^-2, u_ij the unit vector from p_j to p_i (0 if the
//               two coincide).  One workgroup runs every step for a batch of
//               components (at most 256 nodes in total, one thread per node),
//               with positions and the batch's distances (uint8) in LDS.
#include <algorithm>
#include <string>

#include "fl_common.h"
#include "fl_tree.h"

namespace fl {
namespace {

constexpr int KK_MAX = 256;
constexpr int KK_WORDS = KK_MAX / 32;

__global__ __launch_bounds__(256) void k_kk_bfs(const int32_t *__restrict__ comp_off, const int32_t *__restrict__ ids,
                                                const int64_t *__restrict__ dist_off,
                                                const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                int32_t *__restrict__ dist, int32_t *__restrict__ err)
{
    __shared__ uint32_t vis[KK_MAX][KK_WORDS];
    __shared__ uint32_t fr[KK_MAX][KK_WORDS];
    __shared__ uint32_t nx[KK_MAX][KK_WORDS];
    __shared__ int any;
    const int c = ids[blockIdx.x];
    const int cb = comp_off[c], n = comp_off[c + 1] - cb;
    int32_t *D = dist + dist_off[blockIdx.x];
    const int nw = (n + 31) / 32;
    for (int i = threadIdx.x; i < n * nw; i += blockDim.x) {
        const int v = i / nw, w = i % nw;
        const uint32_t self = (v / 32 == w) ? (1u << (v % 32)) : 0u;
        vis[v][w] = self;
        fr[v][w] = self;
    }
    for (int v = threadIdx.x; v < n; v += blockDim.x) D[(int64_t)v * n + v] = 0;
    __syncthreads();
    for (int d = 0; d < n; ++d) {
        if (threadIdx.x == 0) any = 0;
        for (int i = threadIdx.x; i < n * nw; i += blockDim.x) {
            const int v = i / nw, w = i % nw;
            uint32_t acc = 0;
            for (int e = row_ptr[cb + v]; e < row_ptr[cb + v + 1]; ++e) {
                const int u = col[e] - cb;
                if (u < 0 || u >= n) {
                    atomicOr(err, 1);  // edge leaves the component
                    continue;
                }
                acc |= fr[u][w];
            }
            nx[v][w] = acc & ~vis[v][w];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n * nw; i += blockDim.x) {
            const int v = i / nw, w = i % nw;
            uint32_t m = nx[v][w];
            fr[v][w] = m;
            vis[v][w] |= m;
            if (m) any = 1;
            while (m) {
                const int b = __ffs((int)m) - 1;
                m &= m - 1;
                D[(int64_t)(w * 32 + b) * n + v] = d + 1;
            }
        }
        __syncthreads();
        if (!any) break;
        __syncthreads();
    }
    // a pair never reached means the "component" was not connected
    for (int i = threadIdx.x; i < n * nw; i += blockDim.x) {
        const int v = i / nw, w = i % nw;
        const int lim = min(32, n - w * 32);
        const uint32_t full = lim == 32 ? 0xFFFFFFFFu : ((1u << lim) - 1u);
        if ((vis[v][w] & full) != full) atomicOr(err, 2);
    }
}

struct KKBatch {
    int32_t c0, c1;  // components [c0, c1) of the full list: consecutive node ranges
    int32_t k0;      // index of c0 in the subset (for the distance offsets)
    int32_t pad;
};

__global__ __launch_bounds__(256) void k_kk_steps(const KKBatch *__restrict__ batches,
                                                  const int32_t *__restrict__ comp_off,
                                                  const int64_t *__restrict__ dist_off,
                                                  const int32_t *__restrict__ dist, float *__restrict__ x,
                                                  float *__restrict__ y, float l, int steps)
{
    __shared__ float2 pos[KK_MAX];
    __shared__ uint8_t D8[KK_MAX * KK_MAX];
    __shared__ int cstart[KK_MAX + 1];  // batch-local node offsets of the components
    __shared__ int dbase[KK_MAX];       // batch-local distance offsets
    const KKBatch bt = batches[blockIdx.x];
    const int ncomp = bt.c1 - bt.c0;
    const int nb = comp_off[bt.c0];
    const int nnodes = comp_off[bt.c1] - nb;
    if (threadIdx.x == 0) {
        int s = 0, db = 0;
        for (int k = 0; k < ncomp; ++k) {
            const int nk = comp_off[bt.c0 + k + 1] - comp_off[bt.c0 + k];
            cstart[k] = s;
            dbase[k] = db;
            s += nk;
            db += nk * nk;
        }
        cstart[ncomp] = s;
    }
    __syncthreads();
    // stage distances as bytes (components of <= 256 nodes have d <= 255)
    for (int k = 0; k < ncomp; ++k) {
        const int nk = cstart[k + 1] - cstart[k];
        const int32_t *Dk = dist + dist_off[bt.k0 + k];
        for (int i = threadIdx.x; i < nk * nk; i += blockDim.x) D8[dbase[k] + i] = (uint8_t)Dk[i];
    }
    const int t = threadIdx.x;
    int k = 0;
    if (t < nnodes) {
        while (cstart[k + 1] <= t) ++k;
        pos[t] = make_float2(x[nb + t], y[nb + t]);
    }
    __syncthreads();
    const int s0 = t < nnodes ? cstart[k] : 0;
    const int nk = t < nnodes ? cstart[k + 1] - s0 : 0;
    const int li = t - s0;
    const uint8_t *Drow = D8 + (t < nnodes ? dbase[k] + li * nk : 0);
    for (int st = 0; st < steps; ++st) {
        float2 np = make_float2(0.f, 0.f);
        if (t < nnodes) {
            const float2 pi = pos[t];
            float sw = 0.f, ax = 0.f, ay = 0.f;
            for (int j = 0; j < nk; ++j) {
                if (j == li) continue;
                const float2 pj = pos[s0 + j];
                const float d = (float)Drow[j];
                const float w = 1.0f / (d * d);
                const float dx = pi.x - pj.x, dy = pi.y - pj.y;
                const float r2 = dx * dx + dy * dy;
                const float rinv = r2 > 0.f ? rsqrtf(r2) : 0.f;
                const float ld = l * d * w;  // w l d
                sw += w;
                ax += w * pj.x + ld * dx * rinv;
                ay += w * pj.y + ld * dy * rinv;
            }
            np = sw > 0.f ? make_float2(ax / sw, ay / sw) : pi;
            // a pair: the update reflects its distance r to |2l - r|; half
            // way lands it at distance l about its midpoint
            if (nk == 2) np = make_float2(0.5f * (pi.x + np.x), 0.5f * (pi.y + np.y));
        }
        __syncthreads();
        if (t < nnodes) pos[t] = np;
        __syncthreads();
    }
    if (t < nnodes) {
        x[nb + t] = pos[t].x;
        y[nb + t] = pos[t].y;
    }
}

// ---- Newton-Raphson (the paper's minimiser) --------------------------------
// One wave per component (<= 256 nodes, node j on lane j % 64, slot j / 64),
// the largest components first: the distance matrix in LDS (as bytes); each
// lane's nodes (position, gradient, sum_j w_ij) in registers.  A move:
//   1. the node m with the largest |g| (lowest index on a tie) by a wave
//      maximum over (|g|^2 bits << 32 | ~index);
//   2. Newton-Raphson steps on p_m: one wave reduction gives the gradient
//      and the Hessian at p_m; the 2x2 solve when the Hessian is
//      positive definite, else -g / (2 sum w); the step is halved until E_m
//      decreases (one more reduction per trial, of per-pair energy changes);
//   3. every other node's gradient is corrected for p_m's move (old term out,
//      new term in), and m's own is the last one computed.
constexpr int KKN_Q = KK_MAX / WAVE;
constexpr int KKN_INNER = 16;

__device__ __forceinline__ float kkn_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), WAVE - 1));
}

// Wave maximum of a 64-bit key by DPP, the same row pattern as kkn_sum
// (lanes shifted in from outside a row read 0, the identity of unsigned max)
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ unsigned long long kkn_max_step(unsigned long long v)
{
    const unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    const unsigned lo2 = (unsigned)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, ROWS, 0xF, BOUND);
    const unsigned hi2 = (unsigned)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, ROWS, 0xF, BOUND);
    const unsigned long long u = ((unsigned long long)hi2 << 32) | lo2;
    return u > v ? u : v;
}

__device__ __forceinline__ unsigned long long kkn_max_u64(unsigned long long v)
{
    v = kkn_max_step<0x111, 0xF, true>(v);
    v = kkn_max_step<0x112, 0xF, true>(v);
    v = kkn_max_step<0x114, 0xF, true>(v);
    v = kkn_max_step<0x118, 0xF, true>(v);
    v = kkn_max_step<0x142, 0xA, false>(v);
    v = kkn_max_step<0x143, 0xC, false>(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, WAVE - 1);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), WAVE - 1);
    return ((unsigned long long)hi << 32) | lo;
}

// gradient and Hessian terms of the pair (node at p, other node at q) in
// p; nothing for coincident points
struct KKTerm {
    float gx, gy, hxx, hxy, hyy;
};

__device__ __forceinline__ KKTerm kkn_term(float px, float py, float qx, float qy, float w, float L)
{
    KKTerm t{0.f, 0.f, 0.f, 0.f, 0.f};
    const float dx = px - qx, dy = py - qy;
    const float r2 = dx * dx + dy * dy;
    if (r2 > 0.f) {
        const float ir = __builtin_amdgcn_rsqf(r2);
        const float ir3 = ir * ir * ir;
        const float w2 = 2.f * w;
        t.gx = w2 * (dx - L * dx * ir);
        t.gy = w2 * (dy - L * dy * ir);
        t.hxx = w2 * (1.f - L * dy * dy * ir3);
        t.hxy = w2 * L * dx * dy * ir3;
        t.hyy = w2 * (1.f - L * dx * dx * ir3);
    }
    return t;
}

// gradient term only (the corrections after a move and the first gradients)
__device__ __forceinline__ float2 kkn_grad(float px, float py, float qx, float qy, float w, float L)
{
    const float dx = px - qx, dy = py - qy;
    const float r2 = dx * dx + dy * dy;
    if (!(r2 > 0.f)) return make_float2(0.f, 0.f);
    const float f = 2.f * w * (1.f - L * __builtin_amdgcn_rsqf(r2));
    return make_float2(f * dx, f * dy);
}

__device__ __forceinline__ float read_lane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ float kkn_pick(const float (&a)[KK_MAX / WAVE], int q)
{
    return q == 0 ? a[0] : q == 1 ? a[1] : q == 2 ? a[2] : a[3];
}

__global__ __launch_bounds__(WAVE) void k_kk_newton(const int32_t *__restrict__ comp_off,
                                                    const int32_t *__restrict__ ids,
                                                    const int64_t *__restrict__ dist_off,
                                                    const int32_t *__restrict__ sched,
                                                    const int32_t *__restrict__ dist, float *__restrict__ x,
                                                    float *__restrict__ y, float l, float tol, int moves_per_node)
{
    extern __shared__ float2 lds_kkn[];  // positions [KK_MAX], then the distances as bytes
    float2 *pos = lds_kkn;
    uint8_t *D8 = reinterpret_cast<uint8_t *>(lds_kkn + KK_MAX);
    const int k = sched[blockIdx.x];
    const int lane = lane_id();
    const int c = ids[k];
    const int cb = comp_off[c], n = comp_off[c + 1] - cb;
    const int32_t *Dg = dist + dist_off[k];
    for (int j = lane; j < n; j += WAVE) pos[j] = make_float2(x[cb + j], y[cb + j]);
    for (int e = lane; e < n * n; e += WAVE) D8[e] = (uint8_t)Dg[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // own nodes in registers: positions, gradients, sum_j w_ij
    float xq[KKN_Q], yq[KKN_Q], gx[KKN_Q], gy[KKN_Q], swq[KKN_Q];
#pragma unroll
    for (int q = 0; q < KKN_Q; ++q) {
        gx[q] = 0.f;
        gy[q] = 0.f;
        swq[q] = 0.f;
        xq[q] = 0.f;
        yq[q] = 0.f;
        const int i = lane + WAVE * q;
        if (i < n) {
            const float2 pi = pos[i];
            xq[q] = pi.x;
            yq[q] = pi.y;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                const float2 pj = pos[j];
                const float d = (float)D8[i * n + j];
                const float w = __builtin_amdgcn_rcpf(d * d);
                const float2 t = kkn_grad(pi.x, pi.y, pj.x, pj.y, w, l * d);
                gx[q] += t.x;
                gy[q] += t.y;
                swq[q] += w;
            }
        }
    }

    const float tol2 = tol * tol;
    const int64_t budget = (int64_t)moves_per_node * n;
    for (int64_t mv = 0; mv < budget; ++mv) {
        // 1. the node with the largest gradient norm
        unsigned long long key = 0ull;
#pragma unroll
        for (int q = 0; q < KKN_Q; ++q) {
            const int i = lane + WAVE * q;
            if (i < n) {
                const float g2 = gx[q] * gx[q] + gy[q] * gy[q];
                const unsigned long long kq =
                    ((unsigned long long)__float_as_uint(g2) << 32) | (unsigned long long)(~(unsigned)i);
                key = kq > key ? kq : key;
            }
        }
        key = kkn_max_u64(key);
        const float g2max = __uint_as_float((unsigned)(key >> 32));
        if (!(g2max >= tol2)) break;  // also ends on a NaN gradient
        const int m = (int)(~(unsigned)(key & 0xFFFFFFFFull));
        const int qm = m / WAVE, lm = m & (WAVE - 1);
        const uint8_t *Dm = D8 + m * n;
        float wq[KKN_Q], Lq[KKN_Q];
        bool other[KKN_Q];
#pragma unroll
        for (int q = 0; q < KKN_Q; ++q) {
            const int j = lane + WAVE * q;
            other[q] = j < n && j != m;
            const float d = j < n ? (float)Dm[j] : 1.f;
            wq[q] = __builtin_amdgcn_rcpf(d * d);
            Lq[q] = l * d;
        }
        const float ox = read_lane_f(kkn_pick(xq, qm), lm), oy = read_lane_f(kkn_pick(yq, qm), lm);
        const float swm = read_lane_f(kkn_pick(swq, qm), lm);
        float mx = ox, my = oy;
        float Gx = 0.f, Gy = 0.f;
        // 2. Newton-Raphson steps on p_m
        for (int s = 0; s <= KKN_INNER; ++s) {
            float a[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // gx gy hxx hxy hyy
#pragma unroll
            for (int q = 0; q < KKN_Q; ++q) {
                if (other[q]) {
                    const KKTerm t = kkn_term(mx, my, xq[q], yq[q], wq[q], Lq[q]);
                    a[0] += t.gx;
                    a[1] += t.gy;
                    a[2] += t.hxx;
                    a[3] += t.hxy;
                    a[4] += t.hyy;
                }
            }
            Gx = kkn_sum(a[0]);
            Gy = kkn_sum(a[1]);
            if (Gx * Gx + Gy * Gy < tol2 || s == KKN_INNER) break;
            const float hxx = kkn_sum(a[2]), hxy = kkn_sum(a[3]), hyy = kkn_sum(a[4]);
            const float det = hxx * hyy - hxy * hxy;
            float sx, sy;
            if (hxx > 0.f && det > 0.f) {
                sx = -(hyy * Gx - hxy * Gy) / det;
                sy = -(hxx * Gy - hxy * Gx) / det;
            } else {
                sx = -Gx / (2.f * swm);
                sy = -Gy / (2.f * swm);
            }
            // E_m(trial) < E_m(p_m), evaluated as a sum of per-pair changes
            // w ((r1 - L)^2 - (r0 - L)^2) = w (r1 - r0)(r1 + r0 - 2L) with
            // r1 - r0 = (2 s.e + s.s) / (r1 + r0), e = p_m - p_j: no
            // difference of nearly equal numbers, so FP32 resolves the
            // decrease of a small step
            float exq[KKN_Q], eyq[KKN_Q], r0q[KKN_Q];
#pragma unroll
            for (int q = 0; q < KKN_Q; ++q) {
                exq[q] = other[q] ? mx - xq[q] : 0.f;
                eyq[q] = other[q] ? my - yq[q] : 0.f;
                r0q[q] = __builtin_amdgcn_sqrtf(exq[q] * exq[q] + eyq[q] * eyq[q]);
            }
            bool moved = false;
            for (int h = 0; h <= 30; ++h) {
                float de = 0.f;
#pragma unroll
                for (int q = 0; q < KKN_Q; ++q) {
                    if (other[q]) {
                        const float ux = exq[q] + sx, uy = eyq[q] + sy;
                        const float rs = __builtin_amdgcn_sqrtf(ux * ux + uy * uy) + r0q[q];
                        const float dr = rs > 0.f ? (2.f * (sx * exq[q] + sy * eyq[q]) + sx * sx + sy * sy) *
                                                        __builtin_amdgcn_rcpf(rs)
                                                  : 0.f;
                        de += dr * (rs - 2.f * Lq[q]) * wq[q];
                    }
                }
                if (kkn_sum(de) < 0.f) {
                    mx += sx;
                    my += sy;
                    moved = true;
                    break;
                }
                sx *= 0.5f;
                sy *= 0.5f;
            }
            if (!moved) break;
        }
        // 3. p_m's move in every other gradient; m keeps the last one computed
#pragma unroll
        for (int q = 0; q < KKN_Q; ++q) {
            if (other[q]) {
                const float2 to = kkn_grad(xq[q], yq[q], ox, oy, wq[q], Lq[q]);
                const float2 tn = kkn_grad(xq[q], yq[q], mx, my, wq[q], Lq[q]);
                gx[q] += tn.x - to.x;
                gy[q] += tn.y - to.y;
            }
            if (q == qm && lane == lm) {
                xq[q] = mx;
                yq[q] = my;
                gx[q] = Gx;
                gy[q] = Gy;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KKN_Q; ++q) {
        const int i = lane + WAVE * q;
        if (i < n) {
            x[cb + i] = xq[q];
            y[cb + i] = yq[q];
        }
    }
}

// ---- cluster / decluster (sec. 3.1) ------------------------------------------
// Per node of a component (global id), what the reductions did with it:
//   rec = (kind, a, b, i), rec_k = k, kidx = index among the kept nodes or -1
//   kind 0: kept;  kind 1: i-th of k nodes of a removed chain from end a to
//   end b (a < b);  kind 2: a contracted leaf of node a, j = i-th of k.
// One workgroup per component (<= 256 nodes, node v on thread v).
__global__ __launch_bounds__(KK_MAX) void k_kk_reduce(const int32_t *__restrict__ comp_off,
                                                      const int32_t *__restrict__ ids,
                                                      const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, int flags,
                                                      int4 *__restrict__ rec, int32_t *__restrict__ rec_k,
                                                      int32_t *__restrict__ kidx, int32_t *__restrict__ kcount)
{
    __shared__ int deg[KK_MAX];
    __shared__ uint8_t leaf[KK_MAX], mid[KK_MAX];
    __shared__ int4 chains[KK_MAX];  // (a, b, smallest node id) of every candidate chain
    __shared__ int nch;
    __shared__ int lds_scan[KK_MAX / WAVE];
    const int c = ids[blockIdx.x];
    const int cb = comp_off[c], n = comp_off[c + 1] - cb;
    const int v = threadIdx.x;
    const bool valid = v < n;
    const int r0 = valid ? row_ptr[cb + v] : 0, r1 = valid ? row_ptr[cb + v + 1] : 0;
    if (valid) deg[v] = r1 - r0;
    if (v == 0) nch = 0;
    __syncthreads();
    if (valid) leaf[v] = (flags & FL_KK_REDUCE_LEAVES) && deg[v] == 1 && deg[col[r0] - cb] >= 2;
    __syncthreads();
    int rest = 0;
    if (valid && !leaf[v])
        for (int e = r0; e < r1; ++e) rest += leaf[col[e] - cb] ? 0 : 1;
    if (valid) mid[v] = (flags & FL_KK_REDUCE_CHAINS) && !leaf[v] && rest == 2;
    __syncthreads();

    int kind = 0, a = -1, b = -1, ii = 0, kk = 0, minid = v;
    bool cand = false;
    if (valid && mid[v]) {
        int nb[2], q = 0;
        for (int e = r0; e < r1 && q < 2; ++e)
            if (!leaf[col[e] - cb]) nb[q++] = col[e] - cb;
        int len[2], end[2];
        for (int s = 0; s < 2; ++s) {
            int prev = v, cur = nb[s], steps = 0;
            while (mid[cur] && cur != v && steps < n) {
                ++steps;
                minid = min(minid, cur);
                int nxt = -1;
                for (int e = row_ptr[cb + cur]; e < row_ptr[cb + cur + 1]; ++e) {
                    const int u = col[e] - cb;
                    if (!leaf[u] && u != prev) {
                        nxt = u;
                        break;
                    }
                }
                prev = cur;
                cur = nxt < 0 ? v : nxt;
            }
            len[s] = steps;
            end[s] = cur;
        }
        if (end[0] != v && end[1] != v && end[0] != end[1]) {
            a = min(end[0], end[1]);
            b = max(end[0], end[1]);
            ii = (a == end[0] ? len[0] : len[1]) + 1;
            kk = len[0] + len[1] + 1;
            cand = true;
            if (v == minid) {
                const int slot = atomicAdd(&nch, 1);
                chains[slot] = make_int4(a, b, minid, 0);
            }
        }
    }
    __syncthreads();
    if (cand) {
        // of the chains between the same two ends, only the one with the
        // smallest node id is removed
        const int m = nch;
        for (int t = 0; t < m; ++t) {
            const int4 o = chains[t];
            if (o.x == a && o.y == b && o.z < minid) cand = false;
        }
    }
    if (cand) kind = 1;
    if (valid && leaf[v]) {
        kind = 2;
        a = col[r0] - cb;
        int rank = 0, tot = 0;
        for (int e = row_ptr[cb + a]; e < row_ptr[cb + a + 1]; ++e) {
            const int u = col[e] - cb;
            if (leaf[u]) {
                ++tot;
                rank += u < v ? 1 : 0;
            }
        }
        ii = rank;
        kk = tot;
    }
    const int kept = valid && kind == 0 ? 1 : 0;
    int total;
    const int pos = block_excl_scan<int, KK_MAX>(kept, lds_scan, total);
    if (valid) {
        rec[cb + v] = make_int4(kind, a, b, ii);
        rec_k[cb + v] = kk;
        kidx[cb + v] = kept ? pos : -1;
    }
    if (v == 0) kcount[blockIdx.x] = total;
}

// The kept nodes of each component into consecutive slots of the reduced
// batch: positions, and the rows and columns of their hop distances.
__global__ __launch_bounds__(KK_MAX) void k_kk_gather_reduced(
    const int32_t *__restrict__ comp_off, const int32_t *__restrict__ ids, const int64_t *__restrict__ doff,
    const int32_t *__restrict__ roff, const int64_t *__restrict__ rdoff, const int32_t *__restrict__ kidx,
    const int32_t *__restrict__ dist, const float *__restrict__ x, const float *__restrict__ y,
    int32_t *__restrict__ rdist, float *__restrict__ rx, float *__restrict__ ry)
{
    __shared__ int klist[KK_MAX];
    const int k = blockIdx.x;
    const int c = ids[k];
    const int cb = comp_off[c], n = comp_off[c + 1] - cb;
    const int kc = roff[k + 1] - roff[k];
    const int v = threadIdx.x;
    if (v < n && kidx[cb + v] >= 0) klist[kidx[cb + v]] = v;
    __syncthreads();
    if (v < kc) {
        rx[roff[k] + v] = x[cb + klist[v]];
        ry[roff[k] + v] = y[cb + klist[v]];
    }
    const int32_t *D = dist + doff[k];
    int32_t *R = rdist + rdoff[k];
    for (int e = v; e < kc * kc; e += blockDim.x) {
        const int i = e / kc, j = e - i * kc;
        R[e] = D[klist[i] * n + klist[j]];
    }
}

// Kept nodes from the reduced layout, then removed chains on the segments
// between their ends, then contracted leaves at distance l from their node.
__global__ __launch_bounds__(KK_MAX) void k_kk_decluster(const int32_t *__restrict__ comp_off,
                                                         const int32_t *__restrict__ ids,
                                                         const int32_t *__restrict__ roff,
                                                         const int4 *__restrict__ rec,
                                                         const int32_t *__restrict__ rec_k,
                                                         const int32_t *__restrict__ kidx,
                                                         const float *__restrict__ rx, const float *__restrict__ ry,
                                                         double l, float *__restrict__ x, float *__restrict__ y)
{
    __shared__ float2 p[KK_MAX];
    __shared__ double lds_sum[KK_MAX / WAVE];
    const int k = blockIdx.x;
    const int c = ids[k];
    const int cb = comp_off[c], n = comp_off[c + 1] - cb;
    const int v = threadIdx.x;
    const bool valid = v < n;
    int4 r = make_int4(-1, 0, 0, 0);
    int rk = 0;
    if (valid) {
        r = rec[cb + v];
        rk = rec_k[cb + v];
        if (r.x == 0) p[v] = make_float2(rx[roff[k] + kidx[cb + v]], ry[roff[k] + kidx[cb + v]]);
    }
    __syncthreads();
    if (r.x == 1) {
        const double t = (double)r.w / (double)(rk + 1);
        const float2 pa = p[r.y], pb = p[r.z];
        p[v] = make_float2((float)((double)pa.x + t * ((double)pb.x - (double)pa.x)),
                           (float)((double)pa.y + t * ((double)pb.y - (double)pa.y)));
    }
    __syncthreads();
    const bool placed = valid && r.x != 2;
    const double cnt = block_sum<double, KK_MAX>(placed ? 1.0 : 0.0, lds_sum);
    const double cx = block_sum<double, KK_MAX>(placed ? (double)p[v].x : 0.0, lds_sum) / cnt;
    const double cy = block_sum<double, KK_MAX>(placed ? (double)p[v].y : 0.0, lds_sum) / cnt;
    // R: the largest distance of a placed node from the centre; p_v within
    // 1e-4 (R + l) of the centre counts as the centre (rounding must not
    // decide a symmetric case)
    double rr = placed ? hypot((double)p[v].x - cx, (double)p[v].y - cy) : 0.0;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) rr = fmax(rr, __shfl_xor(rr, o, WAVE));
    if (lane_id() == 0) lds_sum[v / WAVE] = rr;
    __syncthreads();
    double R = 0.0;
#pragma unroll
    for (int u = 0; u < KK_MAX / WAVE; ++u) R = fmax(R, lds_sum[u]);
    if (r.x == 2) {
        const float2 pv = p[r.y];
        const double dx = (double)pv.x - cx, dy = (double)pv.y - cy;
        const double ang = hypot(dx, dy) <= 1e-4 * (R + l)
                               ? 2.0 * M_PI * (double)r.w / (double)rk
                               : atan2(dy, dx) + ((double)r.w - 0.5 * (double)(rk - 1)) * M_PI / (double)rk;
        double sn, cs;
        sincos(ang, &sn, &cs);
        p[v] = make_float2((float)((double)pv.x + l * cs), (float)((double)pv.y + l * sn));
    }
    if (valid) {
        x[cb + v] = p[v].x;
        y[cb + v] = p[v].y;
    }
}

}  // namespace

// Components taken by Kamada-Kawai: `ids` (ascending) index the full offset
// list.  Batches join runs of consecutive ids (adjacent node ranges) up to
// KK_MAX nodes; dist_off[k] = sum of n^2 over ids[0..k).
struct KKPlan {
    std::vector<int32_t> ids;
    std::vector<int64_t> doff;
    std::vector<KKBatch> batches;
    int32_t *d_off = nullptr, *d_ids = nullptr;
    int64_t *d_doff = nullptr;
    KKBatch *d_batches = nullptr;
};

static KKPlan kk_plan(fl_ctx *c, int n_all, const int32_t *off, const std::vector<int32_t> &ids,
                      const std::string &tag = "kk")
{
    KKPlan p;
    p.ids = ids;
    const int m = (int)ids.size();
    p.doff.resize(m + 1);
    p.doff[0] = 0;
    for (int k = 0; k < m; ++k) {
        const int cid = ids[k];
        FL_REQUIRE(cid >= 0 && cid < n_all && (k == 0 || cid > ids[k - 1]), "component ids must be ascending");
        const int64_t nk = off[cid + 1] - off[cid];
        FL_REQUIRE(nk >= 1, "component offsets must be increasing");
        FL_REQUIRE(nk <= KK_MAX, "Kamada-Kawai components are limited to 256 nodes");
        p.doff[k + 1] = p.doff[k] + nk * nk;
    }
    int k = 0;
    while (k < m) {
        int e = k, tot = 0;
        while (e < m && (e == k || ids[e] == ids[e - 1] + 1) && tot + (off[ids[e] + 1] - off[ids[e]]) <= KK_MAX) {
            tot += off[ids[e] + 1] - off[ids[e]];
            ++e;
        }
        p.batches.push_back(KKBatch{ids[k], ids[e - 1] + 1, k, 0});
        k = e;
    }
    p.d_off = ws<int32_t>(c, (tag + "_off").c_str(), n_all + 1);
    p.d_ids = ws<int32_t>(c, (tag + "_ids").c_str(), m > 0 ? m : 1);
    p.d_doff = ws<int64_t>(c, (tag + "_doff").c_str(), m + 1);
    p.d_batches = ws<KKBatch>(c, (tag + "_batches").c_str(), p.batches.size() + 1);
    FL_CHECK_HIP(hipMemcpyAsync(p.d_off, off, sizeof(int32_t) * (n_all + 1), hipMemcpyHostToDevice, c->stream));
    if (m > 0) FL_CHECK_HIP(hipMemcpyAsync(p.d_ids, p.ids.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(p.d_doff, p.doff.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, c->stream));
    if (!p.batches.empty())
        FL_CHECK_HIP(hipMemcpyAsync(p.d_batches, p.batches.data(), sizeof(KKBatch) * p.batches.size(),
                                    hipMemcpyHostToDevice, c->stream));
    return p;
}

static void kk_bfs(fl_ctx *c, const KKPlan &p, const int32_t *row_ptr, const int32_t *col, int32_t *dist)
{
    if (p.ids.empty()) return;
    int32_t *err = ws<int32_t>(c, "kk_err", 1);
    FL_CHECK_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_kk_bfs, dim3((unsigned)p.ids.size()), dim3(256), 0, c->stream, p.d_off, p.d_ids, p.d_doff,
                       row_ptr, col, dist, err);
    FL_LAUNCH_CHECK();
    int32_t e = read_i32(c, err);  // also keeps the plan's host vectors alive until the copies are done
    if (e & 1) throw Error(FL_EINVAL, "an edge leaves its component's id range");
    if (e & 2) throw Error(FL_EINVAL, "a component is not connected");
}

static void kk_run_steps(fl_ctx *c, const KKPlan &p, const int32_t *dist, float *x, float *y,
                         const fl_kk_params &prm)
{
    if (p.batches.empty()) return;
    if (prm.minimiser == FL_KK_NEWTON) {
        // one wave per component, the largest first (they set the time)
        const int nc = (int)p.ids.size();
        std::vector<int32_t> sched(nc);
        int64_t n2max = 1;
        for (int k = 0; k < nc; ++k) {
            sched[k] = k;
            n2max = std::max<int64_t>(n2max, p.doff[k + 1] - p.doff[k]);
        }
        std::stable_sort(sched.begin(), sched.end(), [&](int a, int b) {
            return p.doff[a + 1] - p.doff[a] > p.doff[b + 1] - p.doff[b];
        });
        int32_t *d_sched = ws<int32_t>(c, "kk_sched", (size_t)nc);
        FL_CHECK_HIP(hipMemcpyAsync(d_sched, sched.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, c->stream));
        const size_t lds = sizeof(float2) * KK_MAX + (size_t)n2max;  // positions, then n^2 distance bytes
        FL_CHECK_HIP(hipFuncSetAttribute((const void *)k_kk_newton, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds));
        hipLaunchKernelGGL(k_kk_newton, dim3((unsigned)nc), dim3(WAVE), lds, c->stream, p.d_off, p.d_ids, p.d_doff,
                           (const int32_t *)d_sched, dist, x, y, (float)prm.l, (float)(prm.eps * prm.l), prm.steps);
    } else {
        hipLaunchKernelGGL(k_kk_steps, dim3((unsigned)p.batches.size()), dim3(256), 0, c->stream, p.d_batches,
                           p.d_off, p.d_doff, dist, x, y, (float)prm.l, prm.steps);
    }
    FL_LAUNCH_CHECK();
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));  // host plan vectors outlive the async copies
}

// Kamada-Kawai for the components `ids` of a graph whose components are the
// node ranges [off[k], off[k+1]); distances in the context workspace.
void kk_layout_subset(fl_ctx *c, int n_all, const int32_t *off, const std::vector<int32_t> &ids,
                      const int32_t *row_ptr, const int32_t *col, float *x, float *y, const fl_kk_params &prm)
{
    if (ids.empty()) return;
    KKPlan p = kk_plan(c, n_all, off, ids);
    int32_t *dist = ws<int32_t>(c, "kk_dist", p.doff.back() > 0 ? p.doff.back() : 1);
    kk_bfs(c, p, row_ptr, col, dist);
    if (!prm.reduce) {
        kk_run_steps(c, p, dist, x, y, prm);
        return;
    }
    // cluster: which nodes stay; lay out the kept nodes with their hop
    // distances in the full component (the reductions keep them); decluster
    const int m = (int)ids.size();
    const int64_t nodes = off[n_all];
    int4 *rec = ws<int4>(c, "kkr_rec", (size_t)nodes);
    int32_t *rec_k = ws<int32_t>(c, "kkr_reck", (size_t)nodes);
    int32_t *kidx = ws<int32_t>(c, "kkr_kidx", (size_t)nodes);
    int32_t *kcount = ws<int32_t>(c, "kkr_kcount", (size_t)m);
    hipLaunchKernelGGL(k_kk_reduce, dim3((unsigned)m), dim3(KK_MAX), 0, c->stream, (const int32_t *)p.d_off,
                       (const int32_t *)p.d_ids, row_ptr, col, (int)prm.reduce, rec, rec_k, kidx, kcount);
    FL_LAUNCH_CHECK();
    std::vector<int32_t> kc(m), roff(m + 1, 0);
    FL_CHECK_HIP(hipMemcpyAsync(kc.data(), kcount, sizeof(int32_t) * m, hipMemcpyDeviceToHost, c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    for (int k = 0; k < m; ++k) {
        FL_REQUIRE(kc[k] >= 1, "Kamada-Kawai reduction removed every node of a component");
        roff[k + 1] = roff[k] + kc[k];
    }
    std::vector<int32_t> rids(m);
    for (int k = 0; k < m; ++k) rids[k] = k;
    KKPlan rp = kk_plan(c, m, roff.data(), rids, "kkr");
    int32_t *rdist = ws<int32_t>(c, "kkr_dist", rp.doff.back() > 0 ? rp.doff.back() : 1);
    float *rx = ws<float>(c, "kkr_x", (size_t)roff[m]), *ry = ws<float>(c, "kkr_y", (size_t)roff[m]);
    hipLaunchKernelGGL(k_kk_gather_reduced, dim3((unsigned)m), dim3(KK_MAX), 0, c->stream, (const int32_t *)p.d_off,
                       (const int32_t *)p.d_ids, (const int64_t *)p.d_doff, (const int32_t *)rp.d_off,
                       (const int64_t *)rp.d_doff, (const int32_t *)kidx, (const int32_t *)dist, (const float *)x,
                       (const float *)y, rdist, rx, ry);
    FL_LAUNCH_CHECK();
    kk_run_steps(c, rp, rdist, rx, ry, prm);
    hipLaunchKernelGGL(k_kk_decluster, dim3((unsigned)m), dim3(KK_MAX), 0, c->stream, (const int32_t *)p.d_off,
                       (const int32_t *)p.d_ids, (const int32_t *)rp.d_off, (const int4 *)rec, (const int32_t *)rec_k,
                       (const int32_t *)kidx, (const float *)rx, (const float *)ry, prm.l, x, y);
    FL_LAUNCH_CHECK();
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
}

void check_kk_params(const fl_kk_params *p)
{
    FL_REQUIRE(p, "null Kamada-Kawai parameters");
    FL_REQUIRE(p->l > 0.0 && std::isfinite(p->l), "Kamada-Kawai: need a finite l > 0");
    FL_REQUIRE(p->steps >= 0, "Kamada-Kawai: need steps >= 0");
    FL_REQUIRE(p->minimiser == FL_KK_MAJORIZATION || p->minimiser == FL_KK_NEWTON,
               "Kamada-Kawai: unknown minimiser");
    FL_REQUIRE(std::isfinite(p->eps) && p->eps >= 0.0, "Kamada-Kawai: need a finite eps >= 0");
    FL_REQUIRE((p->reduce & ~(FL_KK_REDUCE_LEAVES | FL_KK_REDUCE_CHAINS)) == 0, "Kamada-Kawai: unknown reduce flags");
}

static std::vector<int32_t> iota_ids(int n)
{
    std::vector<int32_t> v(n);
    for (int i = 0; i < n; ++i) v[i] = i;
    return v;
}

}  // namespace fl

using namespace fl;

extern "C" {

void fl_kk_default_params(fl_kk_params *p)
{
    if (!p) return;
    p->l = 1.0;
    p->steps = 200;
    p->minimiser = FL_KK_MAJORIZATION;
    p->eps = 1e-3;
    p->reduce = 0;
}

fl_status fl_hop_distances(fl_ctx *c, int32_t n_comp, const int32_t *comp_offsets, const int32_t *row_ptr,
                           const int32_t *col_idx, int32_t *dist, int64_t *dist_offsets)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n_comp >= 1 && comp_offsets && row_ptr && col_idx && dist, "fl_hop_distances: bad arguments");
    KKPlan p = kk_plan(c, n_comp, comp_offsets, iota_ids(n_comp));
    kk_bfs(c, p, row_ptr, col_idx, dist);
    if (dist_offsets) std::memcpy(dist_offsets, p.doff.data(), sizeof(int64_t) * (n_comp + 1));
    FL_API_END(c)
}

fl_status fl_kk_steps(fl_ctx *c, int32_t n_comp, const int32_t *comp_offsets, const int32_t *dist, float *x, float *y,
                      const fl_kk_params *prm)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n_comp >= 1 && comp_offsets && dist && x && y, "fl_kk_steps: bad arguments");
    check_kk_params(prm);
    FL_REQUIRE(prm->reduce == 0, "fl_kk_steps: the reductions need the graph (use fl_kk_layout)");
    KKPlan p = kk_plan(c, n_comp, comp_offsets, iota_ids(n_comp));
    kk_run_steps(c, p, dist, x, y, *prm);
    FL_API_END(c)
}

fl_status fl_kk_layout(fl_ctx *c, int32_t n_comp, const int32_t *comp_offsets, const int32_t *row_ptr,
                       const int32_t *col_idx, float *x, float *y, const fl_kk_params *prm)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n_comp >= 1 && comp_offsets && row_ptr && col_idx && x && y, "fl_kk_layout: bad arguments");
    check_kk_params(prm);
    kk_layout_subset(c, n_comp, comp_offsets, iota_ids(n_comp), row_ptr, col_idx, x, y, *prm);
    FL_API_END(c)
}

}  // extern "C"
