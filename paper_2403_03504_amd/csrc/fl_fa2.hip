// ForceAtlas2 iteration of the paper's sec. 3.2 on one GPU:
//   repulsion  exact O(n^2) (LDS-tiled) or FMM (fl_fmm.hip)
//   attraction linear CSR attraction in FP64 sums (rows longer than 32
//              entries are cut into 256-entry chunks summed by one wave each
//              and added in chunk order); in an iteration these gathers
//              (k_attract_chunks, k_attract_rows) run on a branch stream
//              beside the repulsion and k_combine reads their sums
//   k_combine  gravity, F = F_r + F_a + F_g, per-node swing |F - F'| and
//              traction |F + F'| in FP64, per-tile partial sums; k_speed adds
//              each system's partials in a fixed order and sets its global
//              speed s_G (no host round trip)
//   k_update   per-node speed and move p += s_i F, F' <- F
// There are no floating-point atomics: a run is bitwise reproducible.
#include <algorithm>
#include <exception>
#include <functional>
#include <vector>

#include "fl_fa2.h"
#include "fl_fmm.h"

namespace fl {
namespace {

constexpr int NT = 256;
constexpr int HEAVY = 32;
// the per-node passes (combine, update) take a quarter tile per block: more
// blocks in flight for what is a chain of independent loads per node (an
// eighth was no better); the combine's FP64 partials are per quarter tile
constexpr int TILE_SUB = 4;

struct StepConsts {
    double ka, kg, tau, ks, ksmax, max_rise;
    int gravity_mode, swing_mode;
};

// ---- exact repulsion ------------------------------------------------------------
// Block b takes targets [tile + 256 (b % 8), +256) of system tile b / 8; every
// target sums its own system's sources in 256-source tiles counted from the
// system's first node (FP32 within a tile, FP64 across tiles), so a system's
// forces do not depend on the other systems of the batch.
constexpr int EXACT_SUB = SEG_TILE / NT;

__global__ __launch_bounds__(NT) void k_rep_exact(Segs sg, const float *__restrict__ x, const float *__restrict__ y,
                                                  const int32_t *__restrict__ deg, float kr, float2 *__restrict__ fr)
{
    __shared__ float4 tile[NT];
    const int2 tl = sg.tiles[blockIdx.x / EXACT_SUB];
    const int comp = tl.x;
    const int cb = sg.coff[comp], ce = sg.coff[comp + 1];
    const int t0 = tl.y + (int)(blockIdx.x % EXACT_SUB) * NT;
    const int tend = min(tl.y + SEG_TILE, ce);
    if (t0 >= tend) return;  // the whole block
    const int i = t0 + threadIdx.x;
    const bool live = i < tend;
    const float xi = live ? x[i] : 0.f, yi = live ? y[i] : 0.f;
    double ax = 0.0, ay = 0.0;
    for (int s0 = cb; s0 < ce; s0 += NT) {
        const int j = s0 + threadIdx.x;
        tile[threadIdx.x] = j < ce ? make_float4(x[j], y[j], (float)(deg[j] + 1), 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        float sx = 0.f, sy = 0.f;
#pragma unroll 8
        for (int k = 0; k < NT; ++k) {
            const float4 s = tile[k];
            const float dx = xi - s.x, dy = yi - s.y;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
            const float sm = s.z * __builtin_amdgcn_rcpf(r2);
            sx = fmaf(sm, dx, sx);
            sy = fmaf(sm, dy, sy);
        }
        ax += sx;
        ay += sy;
        __syncthreads();
    }
    if (live) {
        const double km = (double)kr * (double)(deg[i] + 1);
        fr[i] = make_float2((float)(km * ax), (float)(km * ay));
    }
}

// ---- attraction plan: rows longer than HEAVY are cut into CHUNK-entry pieces,
// each summed by one wave; the owning row adds its pieces in order ---------------
constexpr int CHUNK = 256;

__global__ void k_chunk_count(int n, const int32_t *__restrict__ row_ptr, int32_t *__restrict__ nch)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int d = row_ptr[i + 1] - row_ptr[i];
    nch[i] = d > HEAVY ? (d + CHUNK - 1) / CHUNK : 0;
}

__global__ void k_chunk_fill(int n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ choff,
                             int2 *__restrict__ chunks)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int rb = row_ptr[i], re = row_ptr[i + 1];
    for (int c = choff[i], e = rb; c < choff[i + 1]; ++c, e += CHUNK) chunks[c] = make_int2(i, e);
}

__global__ void k_pack_xy(const float *__restrict__ x, const float *__restrict__ y, int n, float2 *__restrict__ xy)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xy[i] = make_float2(x[i], y[i]);
}

__global__ __launch_bounds__(NT) void k_attract_chunks(const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col, const float2 *__restrict__ xy,
                                                       const int2 *__restrict__ chunks,
                                                       const int32_t *__restrict__ nchunks, double2 *__restrict__ csum)
{
    const int nc = *nchunks;
    const int lane = lane_id();
    for (int c = blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE; c < nc; c += gridDim.x * (NT / WAVE)) {
        const int2 ch = chunks[c];
        const int r = ch.x;
        const int e1 = min(ch.y + CHUNK, row_ptr[r + 1]);
        const float2 pr = xy[r];
        const double rx = pr.x, ry = pr.y;
        double sx = 0.0, sy = 0.0;
        for (int e = ch.y + lane; e < e1; e += WAVE) {
            const float2 pj = xy[col[e]];
            sx += (double)pj.x - rx;
            sy += (double)pj.y - ry;
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (lane == 0) csum[c] = make_double2(sx, sy);
    }
}

// The attraction sum of every row (the same arithmetic, in the same order,
// as k_combine's own): light rows by their gathers, heavy rows from their
// chunk sums.  Lets the gathers run on a branch stream beside the repulsion,
// in eight-wave workgroups: beside the near field they held up its waves
// less than four-wave ones (2M-node iteration 0.704 -> 0.695 ms; two waves
// 0.744 ms, sixteen 0.738 ms)
constexpr int ROWS_NT = 512;
__global__ __launch_bounds__(ROWS_NT) void k_attract_rows(int n, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float2 *__restrict__ xy,
                                                     const int32_t *__restrict__ choff,
                                                     const double2 *__restrict__ csum, double2 *__restrict__ asum)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ax = 0.0, ay = 0.0;
    const float2 pi = xy[i];
    const double xi = pi.x, yi = pi.y;
    const int rb = row_ptr[i], re = row_ptr[i + 1];
    if (re - rb <= HEAVY) {
        int e = rb;
        for (; e + 4 <= re; e += 4) {  // four gathers in flight
            const int j0 = col[e], j1 = col[e + 1], j2 = col[e + 2], j3 = col[e + 3];
            const float2 p0 = xy[j0], p1 = xy[j1], p2 = xy[j2], p3 = xy[j3];
            ax += (double)p0.x - xi;
            ay += (double)p0.y - yi;
            ax += (double)p1.x - xi;
            ay += (double)p1.y - yi;
            ax += (double)p2.x - xi;
            ay += (double)p2.y - yi;
            ax += (double)p3.x - xi;
            ay += (double)p3.y - yi;
        }
        for (; e < re; ++e) {
            const float2 pj = xy[col[e]];
            ax += (double)pj.x - xi;
            ay += (double)pj.y - yi;
        }
    } else {
        for (int c = choff[i]; c < choff[i + 1]; ++c) {
            const double2 v = csum[c];
            ax += v.x;
            ay += v.y;
        }
    }
    asum[i] = make_double2(ax, ay);
}

// ---- attraction + gravity + combine + swing/traction ---------------------------
// One block per system tile: forces, and per-tile FP64 partial sums of swing
// and traction.  k_speed then adds each system's tile partials in tile order
// (fixed, so runs are bitwise reproducible and a system's result does not
// depend on the batch) and sets that system's global speed.
__global__ __launch_bounds__(NT) void k_combine(Segs sg, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col, const int32_t *__restrict__ deg,
                                                const float2 *__restrict__ xy,
                                                const float2 *__restrict__ fr,
                                                StepConsts k, const float *__restrict__ fpx,
                                                const float *__restrict__ fpy, int first, float *__restrict__ fx,
                                                float *__restrict__ fy, float *__restrict__ fax,
                                                float *__restrict__ fay, float *__restrict__ fgx,
                                                float *__restrict__ fgy, double2 *__restrict__ part,
                                                int32_t *__restrict__ flags, const int32_t *__restrict__ choff,
                                                const double2 *__restrict__ csum, const double2 *__restrict__ asum)
{
    __shared__ double lds[NT / WAVE];
    const int2 tl = sg.tiles[blockIdx.x / TILE_SUB];
    const int comp = tl.x;
    const int b0 = tl.y + (int)(blockIdx.x % TILE_SUB) * (SEG_TILE / TILE_SUB);
    const int b1 = min(b0 + SEG_TILE / TILE_SUB, sg.coff[comp + 1]);
    double wswg = 0.0, wtra = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += NT) {
        double ax = 0.0, ay = 0.0;
        const float2 pi = xy[i];
        const double xi = pi.x, yi = pi.y;
        const int rb = row_ptr[i], re = row_ptr[i + 1];
        if (asum) {
            const double2 a = asum[i];
            ax = a.x;
            ay = a.y;
        } else if (re - rb <= HEAVY) {
            int e = rb;
            for (; e + 4 <= re; e += 4) {  // four gathers in flight
                const int j0 = col[e], j1 = col[e + 1], j2 = col[e + 2], j3 = col[e + 3];
                const float2 p0 = xy[j0], p1 = xy[j1], p2 = xy[j2], p3 = xy[j3];
                ax += (double)p0.x - xi;
                ay += (double)p0.y - yi;
                ax += (double)p1.x - xi;
                ay += (double)p1.y - yi;
                ax += (double)p2.x - xi;
                ay += (double)p2.y - yi;
                ax += (double)p3.x - xi;
                ay += (double)p3.y - yi;
            }
            for (; e < re; ++e) {
                const float2 pj = xy[col[e]];
                ax += (double)pj.x - xi;
                ay += (double)pj.y - yi;
            }
        } else {
            for (int c = choff[i]; c < choff[i + 1]; ++c) {
                const double2 v = csum[c];
                ax += v.x;
                ay += v.y;
            }
        }
        const double m = (double)(deg[i] + 1);
        const double Fax = k.ka * ax, Fay = k.ka * ay;
        double Fgx, Fgy;
        if (k.gravity_mode == FL_GRAV_STRONG_UNIT) {
            Fgx = -k.kg * xi;
            Fgy = -k.kg * yi;
        } else if (k.gravity_mode == FL_GRAV_FA2_CONST) {
            const double r = sqrt(xi * xi + yi * yi);
            const double s = r > 0.0 ? -k.kg * m / r : 0.0;
            Fgx = s * xi;
            Fgy = s * yi;
        } else {
            Fgx = -k.kg * m * xi;
            Fgy = -k.kg * m * yi;
        }
        const float2 fri = fr ? fr[i] : make_float2(0.f, 0.f);
        const double Frx = fri.x, Fry = fri.y;
        const float Fx = (float)(Frx + Fax + Fgx), Fy = (float)(Fry + Fay + Fgy);
        if (fx) {
            fx[i] = Fx;
            fy[i] = Fy;
        }
        if (fax) {
            fax[i] = (float)Fax;
            fay[i] = (float)Fay;
        }
        if (fgx) {
            fgx[i] = (float)Fgx;
            fgy[i] = (float)Fgy;
        }
        if (!isfinite(Fx) || !isfinite(Fy)) atomicOr(flags + comp, 1);
        if (part) {
            const double px = first ? 0.0 : (double)fpx[i], py = first ? 0.0 : (double)fpy[i];
            const double dxs = (double)Fx - px, dys = (double)Fy - py;
            const double dxt = (double)Fx + px, dyt = (double)Fy + py;
            const double w = (k.swing_mode == FL_SWING_FA2) ? m : 1.0;
            wswg += w * sqrt(dxs * dxs + dys * dys);
            wtra += w * sqrt(dxt * dxt + dyt * dyt);
        }
    }
    if (!part) return;
    wswg = block_sum<double, NT>(wswg, lds);
    wtra = block_sum<double, NT>(wtra, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(wswg, wtra);
}

// Block k: systems k, k + gridDim.x, ...: SWG, TRA (fixed-order sums of the
// tile partials) and the global speed.
__global__ __launch_bounds__(NT) void k_speed(Segs sg, const double2 *__restrict__ part, StepConsts k, int first,
                                              double *__restrict__ scalars, double *__restrict__ ring, int ring_it)
{
    __shared__ double lds[NT / WAVE];
    for (int comp = blockIdx.x; comp < sg.K; comp += gridDim.x) {
        const int t0 = TILE_SUB * sg.tile_off[comp], nt = TILE_SUB * sg.tile_off[comp + 1] - t0;
        double s0 = 0.0, s1 = 0.0;
        for (int b = threadIdx.x; b < nt; b += NT) {
            const double2 v = part[t0 + b];
            s0 += v.x;
            s1 += v.y;
        }
        s0 = block_sum<double, NT>(s0, lds);
        s1 = block_sum<double, NT>(s1, lds);
        if (threadIdx.x == 0) {
            double *sc = scalars + 4 * (int64_t)comp;
            const double SWG = s0;
            const double TRA = (k.swing_mode == FL_SWING_FA2) ? s1 / 2.0 : s1;
            const double sprev = sc[0];
            double sG;
            if (SWG > 0.0) {
                sG = k.tau * TRA / SWG;
                if (!first) sG = fmin(sG, (1.0 + k.max_rise) * sprev);
            } else {
                sG = first ? 1.0 : (1.0 + k.max_rise) * sprev;
            }
            sc[0] = sG;
            sc[1] = SWG;
            sc[2] = TRA;
            if (ring && comp == 0) {  // the per-iteration record is system 0's
                ring[3 * ring_it + 0] = SWG;
                ring[3 * ring_it + 1] = TRA;
                ring[3 * ring_it + 2] = sG;
            }
        }
    }
}

// With `bpart` every block also writes the extrema of its nodes' new
// positions (min x, max x, min y, max y): the next iteration's bounding
// square, so that the tree build need not read the positions again.
__global__ __launch_bounds__(NT) void k_update(Segs sg, float *__restrict__ x, float *__restrict__ y,
                                               const float *__restrict__ fx, const float *__restrict__ fy,
                                               float *__restrict__ fpx, float *__restrict__ fpy, int first,
                                               const double *__restrict__ scalars, double ks, double ksmax,
                                               int32_t *__restrict__ flags, float4 *__restrict__ bpart)
{
    const int2 tl = sg.tiles[blockIdx.x / TILE_SUB];
    const int comp = tl.x;
    const int b0 = tl.y + (int)(blockIdx.x % TILE_SUB) * (SEG_TILE / TILE_SUB);
    const int b1 = min(b0 + SEG_TILE / TILE_SUB, sg.coff[comp + 1]);
    float mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
    if (flags[comp] & 1) {  // non-finite forces: this system stays as it was
        if (bpart)
            for (int i = b0 + threadIdx.x; i < b1; i += NT) {
                const float px = x[i], py = y[i];
                mnx = fminf(mnx, px);
                mxx = fmaxf(mxx, px);
                mny = fminf(mny, py);
                mxy = fmaxf(mxy, py);
            }
    } else {
    const double sG = scalars[4 * (int64_t)comp];
    for (int i = b0 + threadIdx.x; i < b1; i += NT) {
        const float Fx = fx[i], Fy = fy[i];
        const double px = first ? 0.0 : (double)fpx[i], py = first ? 0.0 : (double)fpy[i];
        const double dx = (double)Fx - px, dy = (double)Fy - py;
        const double swg = sqrt(dx * dx + dy * dy);
        double s = ks * sG / (1.0 + sG * sqrt(swg));
        const double fn = sqrt((double)Fx * Fx + (double)Fy * Fy);
        if (fn > 0.0) s = fmin(s, ksmax / fn);
        const float nx = (float)((double)x[i] + s * (double)Fx);
        const float ny = (float)((double)y[i] + s * (double)Fy);
        x[i] = nx;
        y[i] = ny;
        fpx[i] = Fx;
        fpy[i] = Fy;
        if (!isfinite(nx) || !isfinite(ny)) atomicOr(flags + comp, 2);
        mnx = fminf(mnx, nx);
        mxx = fmaxf(mxx, nx);
        mny = fminf(mny, ny);
        mxy = fmaxf(mxy, ny);
    }
    }
    if (!bpart) return;
    __shared__ float4 red[NT / WAVE];
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
        bpart[blockIdx.x] = r;
    }
}

__global__ void k_split(const float2 *__restrict__ v, int n, float *__restrict__ a, float *__restrict__ b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 q = v[i];
    a[i] = q.x;
    b[i] = q.y;
}

__global__ void k_validate_rows(int n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
                                int32_t *__restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == 0 && row_ptr[0] != 0) atomicOr(bad, 1);
    if (i == n) return;
    const int rb = row_ptr[i], re = row_ptr[i + 1];
    if (re < rb) atomicOr(bad, 2);
    else if (deg && deg[i] != re - rb) atomicOr(bad, 4);
}

__global__ void k_validate_cols(int n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                int32_t *__restrict__ bad)
{
    const int nnz = row_ptr[n];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
        const int j = col[e];
        if (j < 0 || j >= n) {
            atomicOr(bad, 8);
            return;
        }
    }
}

// every edge stays inside its system (sys: system of each node)
__global__ void k_validate_systems(int n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                   const int32_t *__restrict__ sys, int32_t *__restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int si = sys[i];
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
        if (sys[col[e]] != si) {
            atomicOr(bad, 1);
            return;
        }
}

__global__ void k_check_finite(int n, const float *__restrict__ x, const float *__restrict__ y,
                               int32_t *__restrict__ flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (!isfinite(x[i]) || !isfinite(y[i]))) atomicOr(flags, 4);
}

// the systems' status words of a batch OR-ed into the caller's word
__global__ void k_flags_or(const int32_t *__restrict__ f, int K, int32_t *__restrict__ dst)
{
    int v = 0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) v |= f[k];
    for (int o = WAVE / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, WAVE);
    if (lane_id() == 0 && v) atomicOr(dst, v);
}

}  // namespace

struct GraphArgs {
    int32_t n;
    const int32_t *row_ptr, *col, *deg;
};

static void validate_params(const fl_fa2_params *p)
{
    FL_REQUIRE(p != nullptr, "null FA2 parameters");
    FL_REQUIRE(std::isfinite(p->kr) && std::isfinite(p->kg) && std::isfinite(p->ka), "kr, kg, ka must be finite");
    FL_REQUIRE(p->gravity_mode >= 0 && p->gravity_mode <= 2, "unknown gravity_mode");
    FL_REQUIRE(p->swing_mode == FL_SWING_PAPER || p->swing_mode == FL_SWING_FA2, "unknown swing_mode");
    FL_REQUIRE(p->tau > 0.0 && std::isfinite(p->tau), "tau must be > 0");
    FL_REQUIRE(p->ks >= 0.0 && std::isfinite(p->ks), "ks must be >= 0");
    FL_REQUIRE(p->ksmax > 0.0, "ksmax must be > 0");
    FL_REQUIRE(p->max_rise >= 0.0 && std::isfinite(p->max_rise), "max_rise must be >= 0");
    FL_REQUIRE(p->repulsion == FL_REP_EXACT || p->repulsion == FL_REP_FMM || p->repulsion == FL_REP_AUTO,
               "unknown repulsion mode");
    if (p->repulsion == FL_REP_FMM) {
        FL_REQUIRE(p->leaf_size >= 1 && p->leaf_size <= 1024, "leaf_size must be in [1, 1024]");
        FL_REQUIRE(p->morton_bits >= 1 && p->morton_bits <= 16, "morton_bits must be in [1, 16]");
        FL_REQUIRE(p->list_lanes == 0 || p->list_lanes == 1 || p->list_lanes == 8, "list_lanes must be 0, 1 or 8");
        if (!fmm_order_supported(p->p))
            throw Error(p->p >= 1 && p->p <= 20 ? FL_EUNSUPPORTED : FL_EINVAL,
                        "FMM expansion order must be one of 4, 6, 8, 10, 12, 16");
    }
}

static void validate_graph(fl_ctx *c, const GraphArgs &g)
{
    FL_REQUIRE(g.n >= 1, "need n >= 1");
    FL_REQUIRE(g.row_ptr && g.col && g.deg, "null graph array");
    int32_t *bad = ws<int32_t>(c, "fa2_bad", 1);
    FL_CHECK_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_validate_rows, dim3(grid_for((int64_t)g.n + 1, NT)), dim3(NT), 0, c->stream, g.n, g.row_ptr,
                       g.deg, bad);
    FL_LAUNCH_CHECK();
    int32_t b = read_i32(c, bad);
    if (b == 0) {
        hipLaunchKernelGGL(k_validate_cols, dim3(2048), dim3(NT), 0, c->stream, g.n, g.row_ptr, g.col, bad);
        FL_LAUNCH_CHECK();
        b = read_i32(c, bad);
    }
    if (b & 1) throw Error(FL_EINVAL, "row_ptr[0] must be 0");
    if (b & 2) throw Error(FL_EINVAL, "row_ptr must be non-decreasing");
    if (b & 4) throw Error(FL_EINVAL, "deg[i] must equal row_ptr[i+1] - row_ptr[i]");
    if (b & 8) throw Error(FL_EINVAL, "column index outside [0, n)");
}

struct AttractPlan {
    int32_t *choff = nullptr;   // [n+1] first chunk of each row (heavy rows only)
    int2 *chunks = nullptr;     // (row, first entry)
    int64_t cap = 0;            // chunk capacity; per-chunk sums live in workspace "at_csum"
};

static int64_t attract_cap(int64_t nnz) { return nnz / (HEAVY + 1) + nnz / CHUNK + 2; }

// Chunks of the rows longer than HEAVY; depends on the graph only.  The plan
// goes to the given arrays (choff [n+1], chunks [attract_cap(nnz)]) or, when
// they are null, to the context's workspace.
static AttractPlan attract_plan(fl_ctx *c, const GraphArgs &g, int32_t *choff = nullptr, int2 *chunks = nullptr,
                                int64_t nnz = -1)
{
    AttractPlan a;
    const int n = g.n;
    if (nnz < 0) nnz = read_i32(c, g.row_ptr + n);
    a.cap = attract_cap(nnz);
    int32_t *nch = ws<int32_t>(c, "at_nch", n);
    a.choff = choff ? choff : ws<int32_t>(c, "at_choff", (size_t)n + 1);
    a.chunks = chunks ? chunks : ws<int2>(c, "at_chunks", a.cap);
    hipLaunchKernelGGL(k_chunk_count, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, n, g.row_ptr, nch);
    FL_LAUNCH_CHECK();
    scan_excl_i32(c, nch, a.choff, n);
    hipLaunchKernelGGL(k_chunk_fill, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, n, g.row_ptr, a.choff, a.chunks);
    FL_LAUNCH_CHECK();
    return a;
}

// positions interleaved (x, y) so each neighbour is one 8-byte gather
// packed: the (x, y) pairs are already in the "at_xy" buffer (written by the
// tree build)
static const float2 *attract_chunks(fl_ctx *c, const GraphArgs &g, const AttractPlan &a, const float *x,
                                    const float *y, double2 *csum, hipStream_t s = nullptr, bool packed = false)
{
    if (!s) s = c->stream;
    float2 *xy = ws<float2>(c, "at_xy", g.n);
    if (!packed) hipLaunchKernelGGL(k_pack_xy, dim3(grid_for(g.n, NT)), dim3(NT), 0, s, x, y, g.n, xy);
    // one wave per chunk, grid-strided: 4096 blocks (16 per CU) keep enough
    // gathers in flight; 1024 and 2048 blocks were 1.2% and 0.5% slower per
    // 2M-node iteration, 8192 no faster.  Small graphs launch no more blocks
    // than their chunk capacity needs.
    const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (a.cap + NT / WAVE - 1) / (NT / WAVE)));
    hipLaunchKernelGGL(k_attract_chunks, dim3(blocks), dim3(NT), 0, s, g.row_ptr, g.col, (const float2 *)xy,
                       a.chunks, a.choff + g.n, csum);
    FL_LAUNCH_CHECK();
    return xy;
}

static void repulsion(fl_ctx *c, const Segs &sg, const GraphArgs &g, const float *x, const float *y,
                      const fl_fa2_params *p, float2 *fr, const ListsHook *on_lists = nullptr,
                      float2 *xy_out = nullptr, BBoxIn bb = {})
{
    if (p->repulsion == FL_REP_EXACT) {
        PhaseTimer pt(c, FL_PH_EXACT);
        hipLaunchKernelGGL(k_rep_exact, dim3(sg.ntiles * EXACT_SUB), dim3(NT), 0, c->stream, sg, x, y, g.deg,
                           (float)p->kr, fr);
        FL_LAUNCH_CHECK();
    } else {
        const int lanes = p->list_lanes ? p->list_lanes : default_list_lanes(sg.n);
        fmm_repulsion(c, sg, x, y, g.deg, p->p, p->leaf_size, p->morton_bits, lanes, (float)p->kr, fr, on_lists,
                      xy_out, bb);
    }
}

static StepConsts consts(const fl_fa2_params *p)
{
    return StepConsts{p->ka, p->kg, p->tau, p->ks, p->ksmax, p->max_rise, p->gravity_mode, p->swing_mode};
}

namespace {

// A batch of K independent systems sharing parameters (K = 1: one graph).
// The state's scalars hold 4 doubles per system.
struct Sys {
    fl_ctx *c;  // context (and stream) the batch runs on
    Segs sg;
    GraphArgs g;
    AttractPlan ap;
    float *x, *y;
    fl_fa2_state st;
    fl_fa2_params prm;
    // one status word per system (bit 0: a non-finite force, bit 1: a
    // non-finite position), cleared by the caller before the first iteration
    int32_t *flags;
    // the last iteration's update wrote the tile extrema of the positions
    // (FMM runs): the next tree build takes them instead of reading x, y
    bool bbox_ready = false;
};

// one iteration; b.flags must have been cleared by the caller.  Unless phases
// are being timed (or the context's branches are off), the attraction
// gathers run on a branch stream (fork and join by events, which graph
// capture records as parallel branches) beside the repulsion; the combine
// then reads their sums.  With the FMM the branch forks once the lists are
// built, so that the gathers (bound by memory latency) overlap the
// ALU-bound near field rather than the latency-bound tree build.
static void iteration(Sys &b, double *ring, int ring_it)
{
    fl_ctx *c = b.c;
    int32_t *flags = b.flags;
    const int n = b.g.n;
    float2 *fr = ws<float2>(c, "fa2_fr", n);
    float *fcx = ws<float>(c, "fa2_fcx", n);
    float *fcy = ws<float>(c, "fa2_fcy", n);
    double2 *part = ws<double2>(c, "fa2_part", (size_t)b.sg.ntiles * TILE_SUB);
    double2 *csum = ws<double2>(c, "at_csum", b.ap.cap);
    const int first = b.st.iter == 0 ? 1 : 0;
    // FMM: the update leaves the tile extrema of the new positions for the
    // next iteration's bounding square
    float4 *bpart = b.prm.repulsion != FL_REP_EXACT
                        ? ws<float4>(c, "fa2_bbox_part", (size_t)b.sg.ntiles * TILE_SUB)
                        : nullptr;
    const BBoxIn bb = b.bbox_ready ? BBoxIn{bpart, TILE_SUB} : BBoxIn{};
    const float2 *xy = nullptr;
    double2 *asum = nullptr;
    if (!c->timing && c->branches) {
        asum = ws<double2>(c, "fa2_asum", n);
        hipStream_t as = aux_stream(c, 2);
        if (!c->ev_fork) FL_CHECK_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        if (!c->ev_join) FL_CHECK_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
        const bool fmm = b.prm.repulsion != FL_REP_EXACT;  // the tree build then packs (x, y)
        const ListsHook side = [&](hipEvent_t after, const BranchTail &tail) {
            FL_CHECK_HIP(hipStreamWaitEvent(as, after, 0));
            xy = attract_chunks(c, b.g, b.ap, b.x, b.y, csum, as, fmm);
            hipLaunchKernelGGL(k_attract_rows, dim3(grid_for(n, ROWS_NT)), dim3(ROWS_NT), 0, as, n, b.g.row_ptr,
                               b.g.col, xy, (const int32_t *)b.ap.choff, (const double2 *)csum, asum);
            FL_LAUNCH_CHECK();
            tail(as);
            FL_CHECK_HIP(hipEventRecord(c->ev_join, as));
        };
        if (!fmm) {
            FL_CHECK_HIP(hipEventRecord(c->ev_fork, c->stream));
            side(c->ev_fork, [](hipStream_t) {});
            repulsion(c, b.sg, b.g, b.x, b.y, &b.prm, fr);
        } else {
            repulsion(c, b.sg, b.g, b.x, b.y, &b.prm, fr, &side, ws<float2>(c, "at_xy", n), bb);
        }
        if (!xy) throw Error(FL_EHIP, "iteration: the attraction branch was not forked");
        FL_CHECK_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    } else {
        repulsion(c, b.sg, b.g, b.x, b.y, &b.prm, fr, nullptr, nullptr, bb);
    }
    {
        PhaseTimer pt(c, FL_PH_ATTRACT);
        if (!xy) xy = attract_chunks(c, b.g, b.ap, b.x, b.y, csum);
        hipLaunchKernelGGL(k_combine, dim3(b.sg.ntiles * TILE_SUB), dim3(NT), 0, c->stream, b.sg, b.g.row_ptr,
                           b.g.col,
                           b.g.deg, xy, (const float2 *)fr, consts(&b.prm),
                           (const float *)b.st.fx_prev, (const float *)b.st.fy_prev, first, fcx, fcy,
                           (float *)nullptr, (float *)nullptr, (float *)nullptr, (float *)nullptr, part, flags,
                           (const int32_t *)b.ap.choff, (const double2 *)csum, (const double2 *)asum);
        hipLaunchKernelGGL(k_speed, dim3(std::min(b.sg.K, 1024)), dim3(NT), 0, c->stream, b.sg,
                           (const double2 *)part, consts(&b.prm), first, b.st.scalars, ring, ring_it);
        FL_LAUNCH_CHECK();
    }
    {
        PhaseTimer pt(c, FL_PH_UPDATE);
        hipLaunchKernelGGL(k_update, dim3(b.sg.ntiles * TILE_SUB), dim3(NT), 0, c->stream, b.sg, b.x, b.y,
                           (const float *)fcx, (const float *)fcy, b.st.fx_prev, b.st.fy_prev, first,
                           (const double *)b.st.scalars, b.prm.ks, b.prm.ksmax, flags, bpart);
        FL_LAUNCH_CHECK();
    }
    b.bbox_ready = bpart != nullptr;
    b.st.iter += 1;
}

// ---- graph replay ------------------------------------------------------------
// An iteration is a fixed sequence of launches whose sizes depend only on the
// systems and the parameters (every data-dependent count stays on the
// device), so after one eager iteration (which sizes the workspace and makes
// F' valid) one more is captured and the graph is replayed.  Captured
// iterations are bitwise the same as eager ones.
constexpr int GRAPH_MIN_ITERS = 4;

static void destroy_graph(hipGraph_t g, hipGraphExec_t e)
{
    AllocGuard guard;  // freeing a graph's memory may synchronise the device
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
}

// Iterations of batches, each on its own context and stream: one eager
// iteration of every batch, then per batch one graph holding one iteration,
// captured on and replayed iters-1 times on the batch's stream, so that
// batches run on separate hardware queues.  On return all work is enqueued
// and `main` is ordered after every batch.
static void run_graph(hipStream_t main, std::vector<Sys> &bs, int iters)
{
    for (auto &b : bs) iteration(b, nullptr, 0);
    const size_t nb = bs.size();
    std::vector<hipGraph_t> graphs(nb, nullptr);
    std::vector<hipGraphExec_t> execs(nb, nullptr);
    std::vector<hipEvent_t> ev(nb, nullptr);
    auto release = [&] {
        for (size_t k = 0; k < nb; ++k) destroy_graph(graphs[k], execs[k]);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    try {
        if (iters > 1) {
            for (size_t k = 0; k < nb; ++k) {
                hipStream_t s = bs[k].c->stream;
                const int64_t it0 = bs[k].st.iter;
                std::exception_ptr fail;
                hipGraph_t failed = nullptr;
                {
                    // no device allocation or free anywhere in the process while recording
                    CaptureGuard recording;
                    FL_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                    try {
                        iteration(bs[k], nullptr, 0);
                    } catch (...) {
                        fail = std::current_exception();
                    }
                    const hipError_t ec = hipStreamEndCapture(s, fail ? &failed : &graphs[k]);
                    bs[k].st.iter = it0;  // recorded, not run
                    if (!fail) FL_CHECK_HIP(ec);
                }
                if (fail) {
                    destroy_graph(failed, nullptr);
                    std::rethrow_exception(fail);
                }
                {
                    // instantiation allocates the graph's device resources:
                    // not while another thread records
                    AllocGuard guard;
                    FL_CHECK_HIP(hipGraphInstantiate(&execs[k], graphs[k], nullptr, nullptr, 0));
                }
            }
            for (int it = 1; it < iters; ++it)
                for (size_t k = 0; k < nb; ++k) FL_CHECK_HIP(hipGraphLaunch(execs[k], bs[k].c->stream));
            for (auto &b : bs) b.st.iter += iters - 1;
        }
        for (size_t k = 0; k < nb; ++k) {
            FL_CHECK_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
            FL_CHECK_HIP(hipEventRecord(ev[k], bs[k].c->stream));
            FL_CHECK_HIP(hipStreamWaitEvent(main, ev[k], 0));
        }
        FL_CHECK_HIP(hipStreamSynchronize(main));
    } catch (...) {
        for (auto &b : bs) (void)hipStreamSynchronize(b.c->stream);
        release();
        throw;
    }
    release();
}

}  // namespace

// Batches of independent systems (the large components of a layout), each
// `iters` iterations from a zero state.  Batch k runs on branch context k
// (own stream and workspace: tree, lists, state, attraction plan), all of
// its systems in the same launches; with graphs on, the batches' replayed
// graphs run concurrently, otherwise the batches run one after the other as
// eager launches on the caller's stream.
void fa2_run_batches(fl_ctx *c, const std::vector<FA2Batch> &in, int iters, int32_t *flags)
{
    if (in.empty() || iters <= 0) return;
    const bool graphs = c->use_graphs;
    hipEvent_t ready = nullptr;
    FL_CHECK_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    std::vector<Sys> bs;
    try {
        FL_CHECK_HIP(hipEventRecord(ready, c->stream));  // inputs were prepared on the caller's stream
        for (size_t k = 0; k < in.size(); ++k) {
            const FA2Batch &B = in[k];
            fl_ctx *bc = graphs ? sub_ctx(c, k) : c;
            if (graphs) {
                bc->timing = false;
                bc->branches = c->branches;
                FL_CHECK_HIP(hipStreamWaitEvent(bc->stream, ready, 0));
            }
            const std::string tag = "bt" + std::to_string(graphs ? 0 : k);
            Sys b;
            b.c = bc;
            b.sg = make_segs(bc, B.coff, tag.c_str());
            const int n = b.sg.n;
            b.g = GraphArgs{n, B.row_ptr, B.col, B.deg};
            int32_t *choff = ws<int32_t>(bc, (tag + "_choff").c_str(), (size_t)n + 1);
            int2 *chunks = ws<int2>(bc, (tag + "_chunks").c_str(), (size_t)attract_cap(B.nnz));
            b.ap = attract_plan(bc, b.g, choff, chunks, B.nnz);
            b.x = B.x;
            b.y = B.y;
            b.st = fl_fa2_state{ws<float>(bc, (tag + "_fpx").c_str(), n), ws<float>(bc, (tag + "_fpy").c_str(), n),
                                ws<double>(bc, (tag + "_sc").c_str(), 4 * (size_t)b.sg.K), 0};
            b.prm = B.prm;
            b.flags = ws<int32_t>(bc, (tag + "_flags").c_str(), (size_t)b.sg.K);
            fill_i32(bc, b.flags, b.sg.K, 0);
            bs.push_back(b);
        }
        if (graphs) {
            hipStream_t main = aux_stream(c, 1);
            run_graph(main, bs, iters);
            FL_CHECK_HIP(hipEventRecord(ready, main));
            FL_CHECK_HIP(hipStreamWaitEvent(c->stream, ready, 0));
        } else {
            for (auto &b : bs)
                for (int it = 0; it < iters; ++it) iteration(b, nullptr, 0);
        }
        for (auto &b : bs) {
            hipLaunchKernelGGL(k_flags_or, dim3(1), dim3(NT), 0, c->stream, (const int32_t *)b.flags, b.sg.K, flags);
            FL_LAUNCH_CHECK();
        }
        for (auto &b : bs)
            if (b.prm.repulsion != FL_REP_EXACT && tree_error_bits(b.c, true))
                throw Error(FL_EHIP, "FMM capacity guard tripped (tree or list sizes)");
    } catch (...) {
        if (graphs)
            for (auto &b : bs) (void)hipStreamSynchronize(b.c->stream);
        (void)hipEventDestroy(ready);
        throw;
    }
    (void)hipEventDestroy(ready);
}

void exact_repulsion(fl_ctx *c, const Segs &sg, const float *x, const float *y, const int32_t *deg, float kr,
                     float2 *fr)
{
    hipLaunchKernelGGL(k_rep_exact, dim3(sg.ntiles * EXACT_SUB), dim3(NT), 0, c->stream, sg, x, y, deg, kr, fr);
    FL_LAUNCH_CHECK();
}

void fa2_validate(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg,
                  const fl_fa2_params *prm)
{
    validate_params(prm);
    validate_graph(c, GraphArgs{n, row_ptr, col, deg});
}

}  // namespace fl

using namespace fl;

extern "C" {

void fl_fa2_default_params(fl_fa2_params *p)
{
    if (!p) return;
    p->kr = 1.0;
    p->kg = 1.0;
    p->ka = 1.0;
    p->gravity_mode = FL_GRAV_STRONG_MASS;
    p->swing_mode = FL_SWING_PAPER;
    p->tau = 1.0;
    p->ks = 0.1;
    p->ksmax = 10.0;
    p->max_rise = 0.5;
    p->repulsion = FL_REP_FMM;
    p->p = 8;
    p->leaf_size = 64;
    p->morton_bits = 16;
    p->list_lanes = 0;
}

fl_status fl_fa2_forces(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                        const float *x, const float *y, const fl_fa2_params *prm, float *frx, float *fry, float *fax,
                        float *fay, float *fgx, float *fgy)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(prm != nullptr, "null FA2 parameters");
    const fl_fa2_params rp = resolve_repulsion(c->tuning, n, *prm);
    prm = &rp;
    validate_params(prm);
    FL_REQUIRE(x && y, "null positions");
    FL_REQUIRE((!frx) == (!fry) && (!fax) == (!fay) && (!fgx) == (!fgy), "force outputs come in x/y pairs");
    GraphArgs g{n, row_ptr, col_idx, deg};
    validate_graph(c, g);
    const Segs sg = segs_single(c, n);
    float2 *fr = ws<float2>(c, "fa2_fr", n);
    repulsion(c, sg, g, x, y, prm, fr);
    if (frx) {
        hipLaunchKernelGGL(k_split, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, (const float2 *)fr, n, frx, fry);
        FL_LAUNCH_CHECK();
    }
    if (fax || fgx) {
        int32_t *flags = ws<int32_t>(c, "fa2_flags", 1);
        AttractPlan ap = attract_plan(c, g);
        double2 *csum = ws<double2>(c, "at_csum", ap.cap);
        const float2 *xy = attract_chunks(c, g, ap, x, y, csum);
        hipLaunchKernelGGL(k_combine, dim3(sg.ntiles * TILE_SUB), dim3(NT), 0, c->stream, sg, row_ptr, col_idx, deg, xy,
                           (const float2 *)nullptr, consts(prm), (const float *)nullptr,
                           (const float *)nullptr, 1, (float *)nullptr, (float *)nullptr, fax, fay, fgx, fgy,
                           (double2 *)nullptr, flags, (const int32_t *)ap.choff, (const double2 *)csum,
                           (const double2 *)nullptr);
        FL_LAUNCH_CHECK();
    }
    FL_API_END(c)
}

}  // extern "C"

fl_status fa2_run_impl(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                       float *x, float *y, fl_fa2_state *st, const fl_fa2_params *prm, int32_t iters,
                       fl_step_stats *per_iter, bool always_sync)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(prm != nullptr, "null FA2 parameters");
    FL_REQUIRE(x && y && st && st->fx_prev && st->fy_prev && st->scalars, "null positions or state");
    FL_REQUIRE(st->iter >= 0, "state iter must be >= 0");
    FL_REQUIRE(iters >= 0, "iters must be >= 0");
    // independent systems (components) given by the state: node ranges on
    // the host, each with its own repulsion and global speed
    const bool multi = st->n_comp > 1;
    std::vector<int32_t> coff;
    int32_t largest = n;
    if (multi) {
        FL_REQUIRE(st->comp_offsets != nullptr, "n_comp > 1 needs comp_offsets");
        coff.assign(st->comp_offsets, st->comp_offsets + st->n_comp + 1);
        FL_REQUIRE(coff[0] == 0 && coff[st->n_comp] == n, "comp_offsets must run from 0 to n");
        largest = 0;
        for (int k = 0; k < st->n_comp; ++k) {
            FL_REQUIRE(coff[k + 1] > coff[k], "comp_offsets must be strictly increasing");
            largest = std::max(largest, coff[k + 1] - coff[k]);
        }
    } else {
        FL_REQUIRE(st->n_comp >= 0, "n_comp must be >= 0");
    }
    const fl_fa2_params rp = resolve_repulsion(c->tuning, largest, *prm);
    prm = &rp;
    validate_params(prm);
    GraphArgs g{n, row_ptr, col_idx, deg};
    validate_graph(c, g);
    const Segs sg = multi ? make_segs(c, coff, "fa2_sys") : segs_single(c, n);
    if (multi) {
        int32_t *bad = ws<int32_t>(c, "fa2_bad", 1);
        fill_i32(c, bad, 1, 0);
        hipLaunchKernelGGL(k_validate_systems, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, n, row_ptr, col_idx,
                           sg.ncomp, bad);
        FL_LAUNCH_CHECK();
        if (read_i32(c, bad)) throw Error(FL_EINVAL, "an edge joins two systems of comp_offsets");
    }
    // one status word per system, and a summary word after them
    const int K = sg.K;
    int32_t *flags = ws<int32_t>(c, "fa2_flags", (size_t)K + 1);
    fill_i32(c, flags, K + 1, 0);
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n, NT)), dim3(NT), 0, c->stream, n, x, y, flags + K);
    FL_LAUNCH_CHECK();
    if (read_i32(c, flags + K) & 4) throw Error(FL_ENONFINITE, "non-finite initial position");
    double *ring = per_iter ? ws<double>(c, "fa2_ring", 3 * (size_t)(iters > 0 ? iters : 1)) : nullptr;
    Sys b{c, sg, g, attract_plan(c, g), x, y, *st, *prm, flags};
    if (!ring && !c->timing && iters >= GRAPH_MIN_ITERS && c->use_graphs) {
        // the caller's stream may be the null stream, which cannot be
        // captured: run on private streams ordered after it and before
        // anything enqueued on it later
        hipStream_t user = c->stream;
        hipEvent_t e = nullptr;
        FL_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        try {
            hipStream_t bs = aux_stream(c, 0), main = aux_stream(c, 1);
            FL_CHECK_HIP(hipEventRecord(e, user));
            FL_CHECK_HIP(hipStreamWaitEvent(bs, e, 0));
            c->stream = bs;
            std::vector<Sys> one{b};
            run_graph(main, one, iters);
            c->stream = user;
            FL_CHECK_HIP(hipEventRecord(e, main));
            FL_CHECK_HIP(hipStreamWaitEvent(user, e, 0));
            st->iter = one[0].st.iter;
        } catch (...) {
            if (c->stream != user) (void)hipStreamSynchronize(c->stream);
            c->stream = user;
            (void)hipEventDestroy(e);
            throw;
        }
        (void)hipEventDestroy(e);
    } else {
        for (int it = 0; it < iters; ++it) iteration(b, ring, it);
        st->iter = b.st.iter;
    }
    if (per_iter || always_sync) {
        hipLaunchKernelGGL(k_flags_or, dim3(1), dim3(NT), 0, c->stream, (const int32_t *)flags, K, flags + K);
        FL_LAUNCH_CHECK();
        int32_t f = read_i32(c, flags + K);
        if (per_iter && iters > 0) {
            std::vector<double> h(3 * (size_t)iters);
            FL_CHECK_HIP(hipMemcpyAsync(h.data(), ring, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
            FL_CHECK_HIP(hipStreamSynchronize(c->stream));
            for (int it = 0; it < iters; ++it) per_iter[it] = fl_step_stats{h[3 * it], h[3 * it + 1], h[3 * it + 2]};
        }
        if (prm->repulsion == FL_REP_FMM && tree_error_bits(c, true))
            throw Error(FL_EHIP, "FMM capacity guard tripped (tree or list sizes)");
        if (f & 1) throw Error(FL_ENONFINITE, "non-finite force");
        if (f & 2) throw Error(FL_ENONFINITE, "non-finite position after the update");
    }
    FL_API_END(c)
}

extern "C" {

fl_status fl_fa2_step(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                      float *x, float *y, fl_fa2_state *st, const fl_fa2_params *prm, fl_step_stats *stats)
{
    return fa2_run_impl(c, n, row_ptr, col_idx, deg, x, y, st, prm, 1, stats, true);
}

fl_status fl_fa2_run(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                     float *x, float *y, fl_fa2_state *st, const fl_fa2_params *prm, int32_t iters,
                     fl_step_stats *per_iter)
{
    return fa2_run_impl(c, n, row_ptr, col_idx, deg, x, y, st, prm, iters, per_iter, true);
}

}  // extern "C"
