// The FMM passes of the paper's sec. 3.2.1 on the quadtree of fl_tree.hip,
// with the expansion operators of Greengard & Rokhlin (1987) for the
// potential phi(z) = sum_j m_j log(z - z_j), whose conjugate derivative gives
// the repulsion: F_i = kr m_i conj(phi'(z_i)).
//
// Every expansion is stored scaled by its cell width w so FP32 cannot
// overflow for any order or extent: outgoing coefficient k holds a_k / w^k
// (|.| <= Q 0.71^k / k), incoming coefficient l holds b_l w^l.
//
//   k_upward  leaves: outgoing expansion from the particles (P2M); then each
//             thread climbs while it is the last child to finish, shifting
//             the four children's expansions to the parent centre (M2M).  The
//             arrival counters reset themselves; nobody waits for anybody.
//   k_m2l     every cell: interacting cells' outgoing expansions converted to
//             an incoming one (M2L, V list) plus particles of coarser
//             separated leaves (P2L, X list).
//   k_l2l     every leaf: incoming expansions of the leaf and all its
//             ancestors shifted to the leaf centre.  Shifts compose exactly,
//             so this is the paper's parent-to-child recursion unrolled along
//             each leaf's ancestor chain (one launch instead of one per level).
//   k_eval    one wave per leaf: far field from the incoming expansion (L2P),
//             W-list outgoing expansions at the particles (M2P), and the
//             direct near field over the U list (P2P).  Lanes are split into
//             groups that stride over the sources so small leaves still fill
//             the wave; groups are combined with xor shuffles (fixed order).
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

struct CellGeo {
    double cx, cy, w;
};

__device__ __forceinline__ CellGeo geo(const TreeView &t, int c)
{
    const double x0 = t.root[0], y0 = t.root[1], L = t.root[2];
    const int l = t.lvl[c];
    const uint32_t v = t.ixy[c];
    const double w = ldexp(L, -l);
    return CellGeo{x0 + ((double)cell_ix(v) + 0.5) * w, y0 + ((double)cell_iy(v) + 0.5) * w, w};
}

__device__ __forceinline__ float2 rel(float x, float y, const CellGeo &g)
{
    return make_float2((float)(((double)x - g.cx) / g.w), (float)(((double)y - g.cy) / g.w));
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_upward(TreeView t, float2 *__restrict__ M, int32_t *arrive)
{
    const int nleaves = t.counts[1];
    for (int li = blockIdx.x * blockDim.x + threadIdx.x; li < nleaves; li += gridDim.x * blockDim.x) {
        const int c = t.leaf_cell[li];
        const CellGeo g = geo(t, c);
        float2 a[P + 1];
#pragma unroll
        for (int k = 0; k <= P; ++k) a[k] = make_float2(0.f, 0.f);
        const int b = t.beg[c], e = t.end[c];
        for (int j = b; j < e; ++j) {
            const float4 p = t.part[j];
            const float2 u = rel(p.x, p.y, g);
            a[0].x += p.z;
            float2 pw = u;
#pragma unroll
            for (int k = 1; k <= P; ++k) {
                const float s = p.z / (float)k;
                a[k].x -= s * pw.x;
                a[k].y -= s * pw.y;
                pw = cmul(pw, u);
            }
        }
        float2 *Mc = M + (int64_t)c * (P + 1);
#pragma unroll
        for (int k = 0; k <= P; ++k) Mc[k] = a[k];

        // climb: shift the children of each completed parent (M2M)
        int cur = c;
        while (true) {
            const int par = t.par[cur];
            if (par < 0) break;
            const int4 ch = t.child[par];
            const int nch = (ch.x >= 0) + (ch.y >= 0) + (ch.z >= 0) + (ch.w >= 0);
            __threadfence();
            const int old = atomicAdd(&arrive[par], 1);
            if (old != nch - 1) break;
            __threadfence();
            arrive[par] = 0;
            float2 bsum[P + 1];
#pragma unroll
            for (int l = 0; l <= P; ++l) bsum[l] = make_float2(0.f, 0.f);
            const int cc[4] = {ch.x, ch.y, ch.z, ch.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cid = cc[q];
                if (cid < 0) continue;
                // child centre relative to the parent centre, in parent widths
                const float2 z = make_float2((q & 1) ? 0.25f : -0.25f, (q >> 1) ? 0.25f : -0.25f);
                float2 A[P + 1];
                const float2 *Mq = M + (int64_t)cid * (P + 1);
#pragma unroll
                for (int k = 0; k <= P; ++k) A[k] = Mq[k];
                float2 zp[P + 1];
                zp[0] = make_float2(1.f, 0.f);
#pragma unroll
                for (int k = 1; k <= P; ++k) zp[k] = cmul(zp[k - 1], z);
                const float Q = A[0].x;
                bsum[0].x += Q;
#pragma unroll
                for (int l = 1; l <= P; ++l) {
                    float2 s = cscale(zp[l], -Q / (float)l);
                    float half = 1.0f;
#pragma unroll
                    for (int k = 1; k <= l; ++k) {
                        half *= 0.5f;
                        const float2 tz = cmul(A[k], zp[l - k]);
                        const float f = half * binomf(l - 1, k - 1);
                        s.x += f * tz.x;
                        s.y += f * tz.y;
                    }
                    bsum[l] = cadd(bsum[l], s);
                }
            }
            float2 *Mp = M + (int64_t)par * (P + 1);
#pragma unroll
            for (int l = 0; l <= P; ++l) Mp[l] = bsum[l];
            cur = par;
        }
    }
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_m2l(TreeView t, const float2 *__restrict__ M,
                                             const int64_t *__restrict__ offVX, const int32_t *__restrict__ V,
                                             const int32_t *__restrict__ X, float2 *__restrict__ Lp)
{
    const int ncells = t.counts[0];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += gridDim.x * blockDim.x) {
        float2 B[P + 1];
#pragma unroll
        for (int l = 0; l <= P; ++l) B[l] = make_float2(0.f, 0.f);
        const int64_t o0 = offVX[c], o1 = offVX[c + 1];
        const int v0 = (int)(o0 & 0xFFFFFFFFll), v1 = (int)(o1 & 0xFFFFFFFFll);
        const int x0 = (int)(o0 >> 32), x1 = (int)(o1 >> 32);
        const uint32_t cxy = t.ixy[c];
        const int cx = cell_ix(cxy), cy = cell_iy(cxy);
        for (int e = v0; e < v1; ++e) {
            const int s = V[e];
            const uint32_t sxy = t.ixy[s];
            // same level: source centre - target centre = w (dx + i dy)
            const float dx = (float)(cell_ix(sxy) - cx), dy = (float)(cell_iy(sxy) - cy);
            const float2 rho = crecip(make_float2(dx, dy));  // w / z0
            const float2 mr = make_float2(-rho.x, -rho.y);
            const float2 *Ms = M + (int64_t)s * (P + 1);
            const float Q = Ms[0].x;
            float2 ap[P + 1];
            float2 pw = mr;
#pragma unroll
            for (int k = 1; k <= P; ++k) {
                ap[k] = cmul(pw, Ms[k]);
                pw = cmul(pw, mr);
            }
            float2 rl = rho;
#pragma unroll
            for (int l = 1; l <= P; ++l) {
                float2 in = make_float2(-Q / (float)l, 0.f);
#pragma unroll
                for (int k = 1; k <= P; ++k) {
                    const float bc = binomf(l + k - 1, k - 1);
                    in.x += bc * ap[k].x;
                    in.y += bc * ap[k].y;
                }
                B[l] = cadd(B[l], cmul(rl, in));
                rl = cmul(rl, rho);
            }
        }
        if (x1 > x0) {
            const CellGeo g = geo(t, c);
            for (int e = x0; e < x1; ++e) {
                const int s = X[e];
                const int sb = t.beg[s], se = t.end[s];
                for (int j = sb; j < se; ++j) {
                    const float4 p = t.part[j];
                    const float2 rho = crecip(rel(p.x, p.y, g));  // w / (z_j - z_c)
                    float2 pw = rho;
#pragma unroll
                    for (int l = 1; l <= P; ++l) {
                        const float s2 = p.z / (float)l;
                        B[l].x -= s2 * pw.x;
                        B[l].y -= s2 * pw.y;
                        pw = cmul(pw, rho);
                    }
                }
            }
        }
        float2 *Lc = Lp + (int64_t)c * (P + 1);
#pragma unroll
        for (int l = 0; l <= P; ++l) Lc[l] = B[l];
    }
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_l2l(TreeView t, const float2 *__restrict__ Lp, float2 *__restrict__ Lleaf)
{
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
template <int P>
__global__ __launch_bounds__(256) void k_eval(TreeView t, const float2 *__restrict__ M,
                                              const float2 *__restrict__ Lleaf, const int64_t *__restrict__ offUW,
                                              const int32_t *__restrict__ U, const int32_t *__restrict__ W, float kr,
                                              float *__restrict__ frx, float *__restrict__ fry)
{
    const int nleaves = t.counts[1];
    const int lane = lane_id();
    const int waves_total = gridDim.x * (blockDim.x / WAVE);
    for (int li = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; li < nleaves; li += waves_total) {
        const int c = t.leaf_cell[li];
        const int b = t.beg[c], e = t.end[c];
        const int64_t ou0 = offUW[li], ou1 = offUW[li + 1];
        const int u0 = (int)(ou0 & 0xFFFFFFFFll), u1 = (int)(ou1 & 0xFFFFFFFFll);
        const int w0 = (int)(ou0 >> 32), w1 = (int)(ou1 >> 32);
        const CellGeo g = geo(t, c);
        const float2 *Lc = Lleaf + (int64_t)li * (P + 1);
        for (int t0 = b; t0 < e; t0 += WAVE) {
            const int ntc = min(WAVE, e - t0);
            const int lg = ntc <= 4 ? 2 : ntc <= 8 ? 3 : ntc <= 16 ? 4 : ntc <= 32 ? 5 : 6;
            const int tp = 1 << lg;
            const int G = WAVE >> lg;
            const int ti = lane & (tp - 1), grp = lane >> lg;
            const bool valid = ti < ntc;
            const float4 me = t.part[t0 + (valid ? ti : 0)];
            float fx = 0.f, fy = 0.f;
            for (int ue = u0; ue < u1; ++ue) {
                const int s = U[ue];
                const int sb = t.beg[s], se = t.end[s];
                int j = sb + grp;
                for (; j + 3 * G < se; j += 4 * G) {
                    const float4 s0 = t.part[j], s1 = t.part[j + G], s2 = t.part[j + 2 * G], s3 = t.part[j + 3 * G];
#define FL_P2P_PAIR(S)                                                                                              \
    {                                                                                                               \
        const float dx = me.x - S.x, dy = me.y - S.y;                                                               \
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));                                                        \
        const float sm = S.z * __builtin_amdgcn_rcpf(r2);                                                           \
        fx = fmaf(sm, dx, fx);                                                                                      \
        fy = fmaf(sm, dy, fy);                                                                                      \
    }
                    FL_P2P_PAIR(s0)
                    FL_P2P_PAIR(s1)
                    FL_P2P_PAIR(s2)
                    FL_P2P_PAIR(s3)
                }
                for (; j < se; j += G) {
                    const float4 s0 = t.part[j];
                    FL_P2P_PAIR(s0)
                }
#undef FL_P2P_PAIR
            }
            for (int o = tp; o < WAVE; o <<= 1) {
                fx += __shfl_xor(fx, o, WAVE);
                fy += __shfl_xor(fy, o, WAVE);
            }
            if (grp == 0 && valid) {
                // far field: incoming expansion of the leaf (Horner in the scaled variable)
                const float2 v = rel(me.x, me.y, g);
                float2 acc = cscale(Lc[P], (float)P);
#pragma unroll
                for (int l = P - 1; l >= 1; --l) acc = cadd(cmul(acc, v), cscale(Lc[l], (float)l));
                const float invw = (float)(1.0 / g.w);
                float2 dphi = cscale(acc, invw);
                // W list: outgoing expansions of small separated cells at the particle
                for (int we = w0; we < w1; ++we) {
                    const int s = W[we];
                    const CellGeo gs = geo(t, s);
                    const float2 tt = crecip(rel(me.x, me.y, gs));  // w_s / (z - z_s)
                    const float2 *Ms = M + (int64_t)s * (P + 1);
                    float2 sum = make_float2(Ms[0].x, 0.f);
                    float2 pw = tt;
#pragma unroll
                    for (int k = 1; k <= P; ++k) {
                        const float2 tk = cmul(Ms[k], pw);
                        sum.x -= (float)k * tk.x;
                        sum.y -= (float)k * tk.y;
                        pw = cmul(pw, tt);
                    }
                    dphi = cadd(dphi, cscale(cmul(tt, sum), (float)(1.0 / gs.w)));
                }
                // F = kr m_i (conj(phi'_far) + near field)
                const float km = kr * me.z;
                const int orig = __float_as_int(me.w);
                frx[orig] = km * (dphi.x + fx);
                fry[orig] = km * (fy - dphi.y);
            }
        }
    }
}

template <int P>
void run_fmm_p(fl_ctx *c, const TreeBufs &t, const ListBufs &L, float kr, float *frx, float *fry)
{
    const int64_t cap = t.cells_cap, lcap = t.leaves_cap;
    float2 *M = ws<float2>(c, "f_M", (size_t)cap * (P + 1));
    float2 *Lp = ws<float2>(c, "f_Lp", (size_t)cap * (P + 1));
    float2 *Ll = ws<float2>(c, "f_Lleaf", (size_t)lcap * (P + 1));
    int32_t *arrive = ws_zeroed<int32_t>(c, "f_arrive", cap);
    TreeView tv = view(t);
    const unsigned gl = grid_for(lcap, 256, 2048);
    const unsigned gc = grid_for(cap, 256, 2048);
    {
        PhaseTimer pt(c, FL_PH_UPWARD);
        hipLaunchKernelGGL(k_upward<P>, dim3(gl), dim3(256), 0, c->stream, tv, M, arrive);
        FL_LAUNCH_CHECK();
    }
    {
        PhaseTimer pt(c, FL_PH_M2L);
        hipLaunchKernelGGL(k_m2l<P>, dim3(gc), dim3(256), 0, c->stream, tv, M, L.offVX, L.V, L.X, Lp);
        hipLaunchKernelGGL(k_l2l<P>, dim3(gl), dim3(256), 0, c->stream, tv, Lp, Ll);
        FL_LAUNCH_CHECK();
    }
    {
        PhaseTimer pt(c, FL_PH_EVAL);
        const unsigned ge = grid_for(lcap, 4, 2048);  // 4 waves per block
        hipLaunchKernelGGL(k_eval<P>, dim3(ge), dim3(256), 0, c->stream, tv, M, Ll, L.offUW, L.U, L.W, kr, frx, fry);
        FL_LAUNCH_CHECK();
    }
}

}  // namespace

bool fmm_order_supported(int p) { return p == 4 || p == 6 || p == 8 || p == 10 || p == 12 || p == 16; }

void fmm_repulsion(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, int p, int leaf,
                   int bits, float kr, float *frx, float *fry)
{
    TreeBufs t;
    ListBufs L;
    {
        PhaseTimer pt(c, FL_PH_TREE);
        build_tree(c, t, n, x, y, deg, bits, leaf);
    }
    {
        PhaseTimer pt(c, FL_PH_LISTS);
        build_lists(c, t, L);
    }
    switch (p) {
    case 4: run_fmm_p<4>(c, t, L, kr, frx, fry); break;
    case 6: run_fmm_p<6>(c, t, L, kr, frx, fry); break;
    case 8: run_fmm_p<8>(c, t, L, kr, frx, fry); break;
    case 10: run_fmm_p<10>(c, t, L, kr, frx, fry); break;
    case 12: run_fmm_p<12>(c, t, L, kr, frx, fry); break;
    case 16: run_fmm_p<16>(c, t, L, kr, frx, fry); break;
    default: throw Error(FL_EUNSUPPORTED, "FMM expansion order not built (use 4, 6, 8, 10, 12 or 16)");
    }
}

}  // namespace fl
