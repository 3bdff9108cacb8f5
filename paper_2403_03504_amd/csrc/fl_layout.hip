// The paper's overall method (sec. 4): split the graph into its connected
// components (directions ignored), lay out components with few nodes by
// Kamada-Kawai and those with many by ForceAtlas2 with FMM repulsion.
//
// Nodes are renumbered so that every component is a contiguous id range
// (stable sort by component label, i.e. by smallest member id), the CSR is
// permuted accordingly, the small components run through the batched
// Kamada-Kawai kernels in one persistent launch, each large component runs
// its own ForceAtlas2 iterations on a local CSR, and the positions are put
// back in the caller's order.  Single nodes go to the origin.
#include <chrono>

#include "fl_fa2.h"
#include "fl_tree.h"

namespace fl {
namespace {

__global__ void k_label_keys(const int32_t *__restrict__ label, int n, uint32_t *__restrict__ key,
                             int32_t *__restrict__ idx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint32_t)label[i];
    idx[i] = i;
}

__global__ void k_comp_flags(const uint32_t *__restrict__ skey, int n, int32_t *__restrict__ flag)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    flag[r] = (r == 0 || skey[r] != skey[r - 1]) ? 1 : 0;
}

__global__ void k_comp_offsets(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int n,
                               int32_t *__restrict__ off)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (flag[r]) off[pos[r]] = r;
    if (r == 0) off[pos[n]] = n;
}

__global__ void k_permute_nodes(const int32_t *__restrict__ perm, int n, const int32_t *__restrict__ deg,
                                const float *__restrict__ x, const float *__restrict__ y, int32_t *__restrict__ inv,
                                int32_t *__restrict__ ndeg, float *__restrict__ xs, float *__restrict__ ys)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int o = perm[r];
    inv[o] = r;
    ndeg[r] = deg[o];
    xs[r] = x[o];
    ys[r] = y[o];
}

__global__ void k_permute_cols(const int32_t *__restrict__ perm, const int32_t *__restrict__ inv, int n,
                               const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                               const int32_t *__restrict__ nrow_ptr, int32_t *__restrict__ ncol)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int o = perm[r];
    int k = nrow_ptr[r];
    for (int e = row_ptr[o]; e < row_ptr[o + 1]; ++e) ncol[k++] = inv[col[e]];
}

__global__ void k_local_csr(const int32_t *__restrict__ nrow_ptr, const int32_t *__restrict__ ncol, int cb, int nc,
                            int32_t *__restrict__ lrp, int32_t *__restrict__ lcol)
{
    const int base = nrow_ptr[cb];
    const int nnz = nrow_ptr[cb + nc] - base;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= nc; i += gridDim.x * blockDim.x)
        lrp[i] = nrow_ptr[cb + i] - base;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x)
        lcol[e] = ncol[base + e] - cb;
}

// first CSR entry of each component (k in [0, ncomp]: the last is nnz)
__global__ void k_comp_rp(const int32_t *__restrict__ off, int ncomp, const int32_t *__restrict__ nrow_ptr,
                          int32_t *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= ncomp) out[k] = nrow_ptr[off[k]];
}

__global__ void k_zero_pos(float *__restrict__ xs, float *__restrict__ ys, const int32_t *__restrict__ idx, int m)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    xs[idx[i]] = 0.f;
    ys[idx[i]] = 0.f;
}

__global__ void k_unpermute_pos(const int32_t *__restrict__ perm, int n, const float *__restrict__ xs,
                                const float *__restrict__ ys, float *__restrict__ x, float *__restrict__ y)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    x[perm[r]] = xs[r];
    y[perm[r]] = ys[r];
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

void layout(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg, float *x, float *y,
            const fl_fa2_params *fa2, int32_t fa2_iters, const fl_kk_params *kk, int32_t kk_max_nodes,
            int32_t fmm_min_nodes, fl_layout_stats *stats)
{
    auto t0 = std::chrono::steady_clock::now();
    fa2_validate(c, n, row_ptr, col, deg, fa2);
    FL_REQUIRE(kk && kk->l > 0.0 && std::isfinite(kk->l) && kk->steps >= 0, "bad Kamada-Kawai parameters");
    FL_REQUIRE(kk_max_nodes >= 1 && kk_max_nodes <= 256, "kk_max_nodes must be in [1, 256]");
    FL_REQUIRE(fa2_iters >= 0, "fa2_iters must be >= 0");
    const unsigned g = grid_for(n, 256);
    int32_t *label = ws<int32_t>(c, "lay_label", n);
    const int32_t ncomp = components(c, n, row_ptr, col, label);
    uint32_t *k0 = ws<uint32_t>(c, "lay_k0", n), *k1 = ws<uint32_t>(c, "lay_k1", n);
    int32_t *i0 = ws<int32_t>(c, "lay_i0", n), *i1 = ws<int32_t>(c, "lay_i1", n);
    hipLaunchKernelGGL(k_label_keys, dim3(g), dim3(256), 0, c->stream, label, n, k0, i0);
    FL_LAUNCH_CHECK();
    int nbits = 1;
    while (nbits < 31 && ((int64_t)1 << nbits) < n) ++nbits;
    const bool alt = radix_sort_u32(c, k0, i0, k1, i1, n, nbits);
    const uint32_t *skey = alt ? k1 : k0;
    const int32_t *perm = alt ? i1 : i0;
    int32_t *flag = ws<int32_t>(c, "lay_flag", n);
    int32_t *pos = ws<int32_t>(c, "lay_pos", (size_t)n + 1);
    int32_t *d_off = ws<int32_t>(c, "lay_off", (size_t)ncomp + 1);
    hipLaunchKernelGGL(k_comp_flags, dim3(g), dim3(256), 0, c->stream, skey, n, flag);
    scan_excl_i32(c, flag, pos, n);
    hipLaunchKernelGGL(k_comp_offsets, dim3(g), dim3(256), 0, c->stream, flag, pos, n, d_off);
    int32_t *inv = ws<int32_t>(c, "lay_inv", n), *ndeg = ws<int32_t>(c, "lay_ndeg", n);
    float *xs = ws<float>(c, "lay_xs", n), *ys = ws<float>(c, "lay_ys", n);
    hipLaunchKernelGGL(k_permute_nodes, dim3(g), dim3(256), 0, c->stream, perm, n, deg, x, y, inv, ndeg, xs, ys);
    int32_t *nrow_ptr = ws<int32_t>(c, "lay_rp", (size_t)n + 1);
    scan_excl_i32(c, ndeg, nrow_ptr, n);
    const int32_t nnz = read_i32(c, row_ptr + n);
    int32_t *ncol = ws<int32_t>(c, "lay_col", nnz > 0 ? nnz : 1);
    hipLaunchKernelGGL(k_permute_cols, dim3(g), dim3(256), 0, c->stream, perm, inv, n, row_ptr, col, nrow_ptr, ncol);
    FL_LAUNCH_CHECK();
    int32_t *d_crp = ws<int32_t>(c, "lay_crp", (size_t)ncomp + 1);
    hipLaunchKernelGGL(k_comp_rp, dim3(grid_for((int64_t)ncomp + 1, 256)), dim3(256), 0, c->stream,
                       (const int32_t *)d_off, ncomp, (const int32_t *)nrow_ptr, d_crp);
    FL_LAUNCH_CHECK();
    std::vector<int32_t> off(ncomp + 1), crp(ncomp + 1);
    FL_CHECK_HIP(hipMemcpyAsync(off.data(), d_off, sizeof(int32_t) * (ncomp + 1), hipMemcpyDeviceToHost, c->stream));
    FL_CHECK_HIP(hipMemcpyAsync(crp.data(), d_crp, sizeof(int32_t) * (ncomp + 1), hipMemcpyDeviceToHost, c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));

    std::vector<int32_t> kk_ids, fa2_ids, single_nodes;
    int64_t kk_nodes = 0, fa2_nodes = 0;
    for (int k = 0; k < ncomp; ++k) {
        const int sz = off[k + 1] - off[k];
        if (sz == 1) single_nodes.push_back(off[k]);
        else if (sz <= kk_max_nodes) {
            kk_ids.push_back(k);
            kk_nodes += sz;
        } else {
            fa2_ids.push_back(k);
            fa2_nodes += sz;
        }
    }
    const double ms_setup = ms_since(t0);
    auto t1 = std::chrono::steady_clock::now();
    if (!single_nodes.empty()) {
        int32_t *d_single = ws<int32_t>(c, "lay_single", single_nodes.size());
        FL_CHECK_HIP(hipMemcpyAsync(d_single, single_nodes.data(), sizeof(int32_t) * single_nodes.size(),
                                    hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_zero_pos, dim3(grid_for((int64_t)single_nodes.size(), 256)), dim3(256), 0, c->stream, xs,
                           ys, (const int32_t *)d_single, (int)single_nodes.size());
        FL_LAUNCH_CHECK();
    }
    kk_layout_subset(c, ncomp, off.data(), kk_ids, nrow_ptr, ncol, xs, ys, kk->l, kk->steps);
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    const double ms_kk = ms_since(t1);
    auto t2 = std::chrono::steady_clock::now();
    int32_t *flags = ws<int32_t>(c, "lay_flags", 1);
    FL_CHECK_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t), c->stream));
    if (!fa2_ids.empty()) {
        // a local CSR per component, side by side: component j of the list
        // keeps rows [cb + j, cb + j + nc] and its own column range
        int32_t *lrp = ws<int32_t>(c, "lay_lrp", (size_t)n + fa2_ids.size() + 1);
        int32_t *lcol = ws<int32_t>(c, "lay_lcol", nnz > 0 ? nnz : 1);
        std::vector<FA2System> sys;
        for (size_t j = 0; j < fa2_ids.size(); ++j) {
            const int k = fa2_ids[j];
            const int cb = off[k], nc = off[k + 1] - off[k];
            int32_t *rp = lrp + cb + j, *cl = lcol + crp[k];
            hipLaunchKernelGGL(k_local_csr, dim3(grid_for(nc + 1, 256, 1024)), dim3(256), 0, c->stream,
                               (const int32_t *)nrow_ptr, (const int32_t *)ncol, cb, nc, rp, cl);
            FL_LAUNCH_CHECK();
            sys.push_back(FA2System{nc, (int64_t)crp[k + 1] - crp[k], rp, cl, ndeg + cb, xs + cb, ys + cb});
        }
        fa2_run_many(c, sys, fa2, fa2_iters, fmm_min_nodes, flags);
    }
    hipLaunchKernelGGL(k_unpermute_pos, dim3(g), dim3(256), 0, c->stream, perm, n, (const float *)xs,
                       (const float *)ys, x, y);
    FL_LAUNCH_CHECK();
    const int32_t f = read_i32(c, flags);
    const double ms_fa2 = ms_since(t2);
    if (f & 1) throw Error(FL_ENONFINITE, "non-finite force in a ForceAtlas2 component");
    if (f & 2) throw Error(FL_ENONFINITE, "non-finite position in a ForceAtlas2 component");
    if (stats) {
        stats->n_comp = ncomp;
        stats->n_single = (int32_t)single_nodes.size();
        stats->n_kk = (int32_t)kk_ids.size();
        stats->n_fa2 = (int32_t)fa2_ids.size();
        stats->kk_nodes = kk_nodes;
        stats->fa2_nodes = fa2_nodes;
        stats->ms_setup = ms_setup;
        stats->ms_kk = ms_kk;
        stats->ms_fa2 = ms_fa2;
    }
}

}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_layout(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                    float *x, float *y, const fl_fa2_params *fa2, int32_t fa2_iters, const fl_kk_params *kk,
                    int32_t kk_max_nodes, int32_t fmm_min_nodes, fl_layout_stats *stats)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1 && row_ptr && col_idx && deg && x && y && fa2 && kk, "fl_layout: bad arguments");
    layout(c, n, row_ptr, col_idx, deg, x, y, fa2, fa2_iters, kk, kk_max_nodes, fmm_min_nodes, stats);
    FL_API_END(c)
}

}  // extern "C"
