// Kamada-Kawai for the small components (paper sec. 3.1, sec. 4).
//
//   k_kk_bfs    hop distances d_ij of one component (<= 256 nodes) per
//               workgroup: breadth-first search from every source at once.
//               Each node keeps bitsets over sources (visited, frontier) in
//               LDS; one level is next(v) = OR_{u in N(v)} frontier(u) minus
//               visited(v), and every source bit newly set in next(v) is the
//               distance d+1 of (source, v).  Unit weights, so this equals the
//               paper's Floyd-Warshall distances (exact integers).
//   k_kk_major  localized stress majorization of the energy
//               E = sum_{i<j} d_ij^-2 (|p_i - p_j| - l d_ij)^2, all nodes of a
//               component updated together from the previous positions:
//                 p_i' = sum_{j!=i} w_ij (p_j + l d_ij u_ij) / sum_{j!=i} w_ij,
//               w_ij = d_ij^-2, u_ij the unit vector from p_j to p_i (0 if the
//               two coincide).  One workgroup runs every step of one
//               component, each node's sum split over several lanes, with
//               positions, the distances (uint8) and a table of the weights
//               in LDS.
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

// Localized stress majorization with each node's sum split over s lanes: a
// workgroup takes one component of nk nodes; node i is summed by lanes
// i*s .. i*s + s - 1, lane `sub` taking the block of B = ceil(nk / s)
// consecutive j from sub * B (rounded up to a multiple of four); the s
// partial sums are added by a butterfly inside the lane group (a fixed order,
// so a component's result does not depend on anything else in the launch).
// The distances sit in LDS as bytes, rows padded to four so that one 32-bit
// read brings four; the weights w = 1/d^2 and l d w come from a table over
// the integer hop distances (d = 0, the node itself or a padding slot, weighs
// 0), computed once per workgroup; sum_j w_ij is fixed over the steps.  A
// coincident pair gets no unit vector: r^2 carries 1e-30, so its direction
// term is 0 * (finite).  s: about eight pairs per lane, at most 16 lanes per
// node and blockDim threads in all.
__device__ __forceinline__ int kk_lanes_per_node(int nk, int threads)
{
    int s = 1;
    while (s < 16 && 2 * s * 8 <= nk && 2 * s * nk <= threads) s *= 2;
    return s;
}

__device__ __forceinline__ int kk_row_stride(int nk) { return (nk + 3) & ~3; }

__global__ __launch_bounds__(1024) void k_kk_major(const int32_t *__restrict__ comp_off,
                                                   const int32_t *__restrict__ ids,
                                                   const int64_t *__restrict__ dist_off,
                                                   const int32_t *__restrict__ order,
                                                   const int32_t *__restrict__ dist, float *__restrict__ x,
                                                   float *__restrict__ y, float l, int steps)
{
    extern __shared__ float4 kk_lds[];
    const int k = order[blockIdx.x];
    const int cb = comp_off[ids[k]];
    const int nk = comp_off[ids[k] + 1] - cb;
    const int rs = kk_row_stride(nk);
    float2 *pos = reinterpret_cast<float2 *>(kk_lds);              // [rs]: past nk, copies of node nk-1
    float2 *wq = pos + rs;                                          // [256]: (1/d^2, l d / d^2)
    uint32_t *D4 = reinterpret_cast<uint32_t *>(wq + KK_MAX);       // [nk][rs / 4]: four distance bytes per word
    const int32_t *Dk = dist + dist_off[k];
    const int wpr = rs >> 2;
    for (int b = threadIdx.x; b < nk * wpr; b += blockDim.x) {
        const int r = b / wpr, c0 = 4 * (b - r * wpr);
        int32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = c0 + u < nk ? Dk[(int64_t)r * nk + c0 + u] : 0;
        D4[b] = (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
    }
    for (int d = threadIdx.x; d < KK_MAX; d += blockDim.x) {
        const float fd = (float)d;
        const float w = d > 0 ? 1.0f / (fd * fd) : 0.f;
        wq[d] = make_float2(w, l * fd * w);
    }
    for (int i = threadIdx.x; i < rs; i += blockDim.x) {
        const int g = cb + min(i, nk - 1);
        pos[i] = make_float2(x[g], y[g]);
    }
    __syncthreads();
    const int s = kk_lanes_per_node(nk, blockDim.x);
    const int t = threadIdx.x;
    const int i = t / s, sub = t - i * s;
    const bool live = i < nk;
    const int B = ((nk + s - 1) / s + 3) & ~3;  // a multiple of four
    const int j0 = live ? min(rs, sub * B) : rs, j1 = live ? min(rs, j0 + B) : rs;
    const uint32_t *Drow = D4 + (live ? i * wpr : 0);
    float sw = 0.f;
    for (int j = j0; j < j1; j += 4) {
        const uint32_t d4 = Drow[j >> 2];
#pragma unroll
        for (int u = 0; u < 4; ++u) sw += wq[(d4 >> (8 * u)) & 0xFFu].x;
    }
    for (int o = s >> 1; o > 0; o >>= 1) sw += __shfl_xor(sw, o, WAVE);
    for (int st = 0; st < steps; ++st) {
        const float2 pi = live ? pos[i] : make_float2(0.f, 0.f);
        float ax = 0.f, ay = 0.f;
        for (int j = j0; j < j1; j += 4) {
            const uint32_t d4 = Drow[j >> 2];
            float2 pj[4], c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pj[u] = pos[j + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = wq[(d4 >> (8 * u)) & 0xFFu];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float dx = pi.x - pj[u].x, dy = pi.y - pj[u].y;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
                const float q = c[u].y * __builtin_amdgcn_rsqf(r2);
                ax = fmaf(c[u].x, pj[u].x, ax);
                ay = fmaf(c[u].x, pj[u].y, ay);
                ax = fmaf(q, dx, ax);
                ay = fmaf(q, dy, ay);
            }
        }
        for (int o = s >> 1; o > 0; o >>= 1) {
            ax += __shfl_xor(ax, o, WAVE);
            ay += __shfl_xor(ay, o, WAVE);
        }
        float2 np = pi;
        if (live) {
            np = sw > 0.f ? make_float2(ax / sw, ay / sw) : pi;
            // a pair: the update reflects its distance r to |2l - r|; half
            // way lands it at distance l about its midpoint
            if (nk == 2) np = make_float2(0.5f * (pi.x + np.x), 0.5f * (pi.y + np.y));
        }
        __syncthreads();
        if (live && sub == 0) {
            pos[i] = np;
            if (i == nk - 1)
                for (int pad = nk; pad < rs; ++pad) pos[pad] = np;  // padding slots weigh 0 but stay finite
        }
        __syncthreads();
    }
    for (int i2 = threadIdx.x; i2 < nk; i2 += blockDim.x) {
        x[cb + i2] = pos[i2].x;
        y[cb + i2] = pos[i2].y;
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
// list; dist_off[k] = sum of n^2 over ids[0..k).
struct KKPlan {
    std::vector<int32_t> ids;
    std::vector<int64_t> doff;
    int32_t *d_off = nullptr, *d_ids = nullptr;
    int64_t *d_doff = nullptr;
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
    p.d_off = ws<int32_t>(c, (tag + "_off").c_str(), n_all + 1);
    p.d_ids = ws<int32_t>(c, (tag + "_ids").c_str(), m > 0 ? m : 1);
    p.d_doff = ws<int64_t>(c, (tag + "_doff").c_str(), m + 1);
    FL_CHECK_HIP(hipMemcpyAsync(p.d_off, off, sizeof(int32_t) * (n_all + 1), hipMemcpyHostToDevice, c->stream));
    if (m > 0) FL_CHECK_HIP(hipMemcpyAsync(p.d_ids, p.ids.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(p.d_doff, p.doff.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, c->stream));
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
    if (p.ids.empty()) return;
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
        // one workgroup per component, in three size classes with their own
        // launch (the workgroup width and the LDS size follow the class):
        // up to 16 nodes one wave, up to 64 nodes four, larger ones sixteen,
        // each class largest first
        const int nc = (int)p.ids.size();
        const int cls_max[3] = {16, 64, KK_MAX}, cls_threads[3] = {WAVE, 256, 1024};
        std::vector<int32_t> cls[3];
        for (int k = 0; k < nc; ++k) {
            const int64_t n2 = p.doff[k + 1] - p.doff[k];
            int q = 0;
            while ((int64_t)cls_max[q] * cls_max[q] < n2) ++q;
            cls[q].push_back(k);
        }
        std::vector<int32_t> order;
        for (auto &v : cls) {
            std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
                return p.doff[a + 1] - p.doff[a] > p.doff[b + 1] - p.doff[b];
            });
            order.insert(order.end(), v.begin(), v.end());
        }
        int32_t *d_order = ws<int32_t>(c, "kk_order", (size_t)nc);
        FL_CHECK_HIP(hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, c->stream));
        // the classes run side by side: the large components, one workgroup
        // each, leave most compute units free while they run
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        for (auto &e : ev) FL_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        FL_CHECK_HIP(hipEventRecord(ev[0], c->stream));
        const hipStream_t cs[3] = {aux_stream(c, 3), aux_stream(c, 2), c->stream};
        const size_t first_of[3] = {0, cls[0].size(), cls[0].size() + cls[1].size()};
        for (int q = 2; q >= 0; --q) {  // the large components first, so that their groups are placed first
            const size_t first = first_of[q];
            if (q < 2) FL_CHECK_HIP(hipStreamWaitEvent(cs[q], ev[0], 0));
            if (cls[q].empty()) continue;
            int64_t nk = 1;
            while (nk * nk < p.doff[cls[q][0] + 1] - p.doff[cls[q][0]]) ++nk;  // the class's largest
            const int64_t rs = (nk + 3) & ~3;
            // positions, the weight table, the distance bytes
            const size_t lds = sizeof(float2) * (size_t)(rs + KK_MAX) + (size_t)(nk * rs);
            if (lds > 64 * 1024)
                FL_CHECK_HIP(hipFuncSetAttribute((const void *)k_kk_major,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(k_kk_major, dim3((unsigned)cls[q].size()), dim3(cls_threads[q]), lds, cs[q],
                               p.d_off, p.d_ids, p.d_doff, (const int32_t *)(d_order + first), dist, x, y,
                               (float)prm.l, prm.steps);
            FL_LAUNCH_CHECK();
        }
        for (int q = 0; q < 2; ++q) {
            FL_CHECK_HIP(hipEventRecord(ev[q + 1], cs[q]));
            FL_CHECK_HIP(hipStreamWaitEvent(c->stream, ev[q + 1], 0));
        }
        FL_CHECK_HIP(hipStreamSynchronize(c->stream));
        for (auto &e : ev) (void)hipEventDestroy(e);
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
