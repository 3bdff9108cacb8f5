// Barnes-Hut repulsion on the FMM's quadtree, kept as a comparator (paper
// sec. 3.2.1 names it as the O(N log N) method the FMM improves on; Barnes &
// Hut 1986).
//
//   k_bh_leafsum  one wave per leaf: FP64 sums of m, m x and m y over its
//                 particles; three FP64 exclusive scans over the leaves follow
//   k_bh_cells    one thread per cell: a cell's leaves are a contiguous run
//                 (pre-order lists leaves in Morton order), from the first
//                 leaf of its subtree to the first leaf after it, so its mass
//                 and centre of mass are differences of the scanned sums;
//                 stored as one float4 (centre x, centre y, mass, side)
//   k_bh_walk     one wave per leaf of targets, 64 at a time.  The wave walks
//                 the cells in pre-order with one shared cursor; cell data is
//                 wave-uniform (scalar loads).  A lane that accepts a cell
//                 adds its monopole and sleeps until the end of the cell's
//                 subtree (skip).  The cursor descends while an awake lane
//                 opens the cell, sums an opened leaf directly for the lanes
//                 that opened it, jumps over a subtree every awake lane has
//                 accepted, and jumps to the earliest wake-up when all sleep.
//                 Every lane ends with the forces of its own per-target walk.
#include <climits>
#include <cmath>

#include "fl_tree.h"

namespace fl {
namespace {

__global__ __launch_bounds__(256) void k_bh_leafsum(TreeView t, double *__restrict__ sm, double *__restrict__ sx,
                                                    double *__restrict__ sy)
{
    const int nleaves = t.counts[1];
    const int wpb = blockDim.x / WAVE;
    const int lane = lane_id();
    const int first = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (int)threadIdx.x / WAVE);
    for (int li = first; li < nleaves; li += gridDim.x * wpb) {
        const int c = t.leaf_cell[li];
        double a = 0.0, b = 0.0, d = 0.0;
        for (int j = t.beg[c] + lane; j < t.end[c]; j += WAVE) {
            const float4 p = t.part[j];
            a += (double)p.z;
            b += (double)p.z * (double)p.x;
            d += (double)p.z * (double)p.y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        d = wave_sum(d);
        if (lane == 0) {
            sm[li] = a;
            sx[li] = b;
            sy[li] = d;
        }
    }
}

__global__ __launch_bounds__(256) void k_bh_cells(TreeView t, const double *__restrict__ Sm,
                                                  const double *__restrict__ Sx, const double *__restrict__ Sy,
                                                  float4 *__restrict__ mono)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell = t.counts[0], nleaves = t.counts[1];
    if (c >= ncell) return;
    int d = c;
    while (t.leafidx[d] < 0) ++d;  // first child follows its parent in pre-order
    const int l0 = t.leafidx[d];
    int l1 = nleaves;
    const int e = t.skip[c];
    if (e < ncell) {
        d = e;
        while (t.leafidx[d] < 0) ++d;
        l1 = t.leafidx[d];
    }
    const double m = Sm[l1] - Sm[l0];
    const double cx = (Sx[l1] - Sx[l0]) / m, cy = (Sy[l1] - Sy[l0]) / m;
    const double side = ldexp(t.root[2], -t.lvl[c]);
    mono[c] = make_float4((float)cx, (float)cy, (float)m, (float)side);
}

__global__ __launch_bounds__(256) void k_bh_walk(TreeView t, const float4 *__restrict__ mono, float th2, float kr,
                                                 float *__restrict__ frx, float *__restrict__ fry)
{
    const int nleaves = t.counts[1], ncell = t.counts[0];
    const int lane = lane_id();
    const int wpb = blockDim.x / WAVE;
    const int first = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (int)threadIdx.x / WAVE);
    for (int li = first; li < nleaves; li += gridDim.x * wpb) {
        const int lc = t.leaf_cell[li];
        const int b = t.beg[lc], e = t.end[lc];
        for (int t0 = b; t0 < e; t0 += WAVE) {
            const bool valid = t0 + lane < e;
            const float4 me = t.part[valid ? t0 + lane : t0];
            float fx = 0.f, fy = 0.f;
            int resume = valid ? 0 : INT_MAX;  // the lane sleeps while the cursor is below this cell
            int c = 0;
            while (c < ncell) {
                const bool awake = resume <= c;
                if (!__any(awake)) {
                    c = __builtin_amdgcn_readfirstlane(-wave_max_i(-resume));  // > c: all valid lanes sleep past c
                    continue;
                }
                const float4 mo = mono[c];
                const int sk = t.skip[c];
                const bool holds = c <= lc && lc < sk;  // an ancestor of (or) the targets' leaf
                bool acc = false;
                if (awake && !holds) {
                    const float dx = me.x - mo.x, dy = me.y - mo.y;
                    const float d2 = dx * dx + dy * dy;
                    if (mo.w * mo.w < th2 * d2) {
                        const float s = mo.z * __builtin_amdgcn_rcpf(d2);
                        fx = fmaf(s, dx, fx);
                        fy = fmaf(s, dy, fy);
                        resume = sk;
                        acc = true;
                    }
                }
                const bool open = awake && !acc;
                if (!__any(open)) {
                    c = sk;
                    continue;
                }
                if (t.leafidx[c] >= 0) {
                    if (open) {
                        const int je = t.end[c];
                        for (int j = t.beg[c]; j < je; ++j) {
                            const float4 s0 = t.part[j];
                            const float dx = me.x - s0.x, dy = me.y - s0.y;
                            const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
                            const float sm = s0.z * __builtin_amdgcn_rcpf(r2);
                            fx = fmaf(sm, dx, fx);
                            fy = fmaf(sm, dy, fy);
                        }
                    }
                    c = sk;
                } else {
                    c = c + 1;
                }
            }
            if (valid) {
                const float km = kr * me.z;
                const int orig = __float_as_int(me.w);
                frx[orig] = km * fx;
                fry[orig] = km * fy;
            }
        }
    }
}

}  // namespace

void bh_repulsion(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, float kr, float theta,
                  int leaf, int bits, float *frx, float *fry)
{
    const Segs s = segs_single(c, n);
    TreeBufs t;
    {
        PhaseTimer pt(c, FL_PH_TREE);
        build_tree(c, t, s, x, y, deg, bits, leaf);
    }
    PhaseTimer pt(c, FL_PH_BH);
    const TreeView tv = view(t);
    const int64_t lcap = t.leaves_cap;
    double *sm = ws<double>(c, "bh_sm", (size_t)lcap + 1), *sx = ws<double>(c, "bh_sx", (size_t)lcap + 1),
           *sy = ws<double>(c, "bh_sy", (size_t)lcap + 1);
    double *Sm = ws<double>(c, "bh_Sm", (size_t)lcap + 1), *Sx = ws<double>(c, "bh_Sx", (size_t)lcap + 1),
           *Sy = ws<double>(c, "bh_Sy", (size_t)lcap + 1);
    float4 *mono = ws<float4>(c, "bh_mono", (size_t)t.cells_cap);
    const unsigned gl = grid_for(lcap, 4, 16384);
    hipLaunchKernelGGL(k_bh_leafsum, dim3(gl), dim3(256), 0, c->stream, tv, sm, sx, sy);
    FL_LAUNCH_CHECK();
    scan_excl_f64(c, sm, Sm, lcap, t.counts + 1, "bhm");
    scan_excl_f64(c, sx, Sx, lcap, t.counts + 1, "bhx");
    scan_excl_f64(c, sy, Sy, lcap, t.counts + 1, "bhy");
    hipLaunchKernelGGL(k_bh_cells, dim3(grid_for(t.cells_cap, 256)), dim3(256), 0, c->stream, tv, (const double *)Sm,
                       (const double *)Sx, (const double *)Sy, mono);
    hipLaunchKernelGGL(k_bh_walk, dim3(gl), dim3(256), 0, c->stream, tv, (const float4 *)mono, theta * theta, kr, frx,
                       fry);
    FL_LAUNCH_CHECK();
}

}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_bh_repulsion(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, double kr,
                          double theta, int32_t leaf_size, int32_t morton_bits, float *frx, float *fry)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1 && x && y && deg && frx && fry, "fl_bh_repulsion: bad arguments");
    FL_REQUIRE(std::isfinite(kr), "fl_bh_repulsion: kr must be finite");
    FL_REQUIRE(std::isfinite(theta) && theta >= 0.0 && theta <= 10.0, "fl_bh_repulsion: theta must be in [0, 10]");
    FL_REQUIRE(leaf_size >= 1 && leaf_size <= 1024, "fl_bh_repulsion: leaf_size must be in [1, 1024]");
    FL_REQUIRE(morton_bits >= 1 && morton_bits <= 16, "fl_bh_repulsion: morton_bits must be in [1, 16]");
    bh_repulsion(c, n, x, y, deg, (float)kr, (float)theta, leaf_size, morton_bits, frx, fry);
    if (tree_error_bits(c, true)) throw Error(FL_EHIP, "fl_bh_repulsion: tree capacity guard tripped");
    FL_API_END(c)
}

}  // extern "C"
