// The paper's overall method (sec. 4): split the graph into its connected
// components (directions ignored), lay out components with few nodes by
// Kamada-Kawai and those with many by ForceAtlas2 with FMM repulsion.
//
// Nodes are renumbered so that every component is a contiguous id range
// (stable sort by component label, i.e. by smallest member id), and the
// components are regrouped by method: the ForceAtlas2 components first, one
// group per repulsion configuration (exact, or FMM with its p and leaf size),
// then the Kamada-Kawai components, then single nodes (which go to the
// origin).  The CSR is permuted accordingly.  The small components run
// through the batched Kamada-Kawai kernels; every ForceAtlas2 group runs as
// one batch, all its components in the same launches; positions go back in
// the caller's order.
#include <chrono>
#include <map>

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

// New position of every node once the components are regrouped: the node
// at label-sorted position r (component comp(r) = pos[r] + flag[r] - 1)
// moves to newstart[comp] + (r - off[comp]).
__global__ void k_regroup(const int32_t *__restrict__ perm, const int32_t *__restrict__ flag,
                          const int32_t *__restrict__ pos, const int32_t *__restrict__ off,
                          const int32_t *__restrict__ newstart, int n, int32_t *__restrict__ perm2)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int k = pos[r] + flag[r] - 1;
    perm2[newstart[k] + (r - off[k])] = perm[r];
}

__global__ void k_zero_range(float *__restrict__ xs, float *__restrict__ ys, int b, int e)
{
    const int i = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= e) return;
    xs[i] = 0.f;
    ys[i] = 0.f;
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

LabelSort sort_by_label(fl_ctx *c, int32_t n, const int32_t *label, int32_t n_labels)
{
    const unsigned g = grid_for(n, 256);
    uint32_t *k0 = ws<uint32_t>(c, "lay_k0", n), *k1 = ws<uint32_t>(c, "lay_k1", n);
    int32_t *i0 = ws<int32_t>(c, "lay_i0", n), *i1 = ws<int32_t>(c, "lay_i1", n);
    hipLaunchKernelGGL(k_label_keys, dim3(g), dim3(256), 0, c->stream, label, n, k0, i0);
    FL_LAUNCH_CHECK();
    int nbits = 1;
    while (nbits < 31 && ((int64_t)1 << nbits) < n) ++nbits;
    int32_t *serr = ws_zeroed<int32_t>(c, "lay_sort_err", 1);
    const bool alt = radix_sort_u32(c, k0, i0, k1, i1, n, nbits, serr);
    const uint32_t *skey = alt ? k1 : k0;
    LabelSort r;
    r.perm = alt ? i1 : i0;
    int32_t *flag = ws<int32_t>(c, "lay_flag", n);
    int32_t *pos = ws<int32_t>(c, "lay_pos", (size_t)n + 1);
    int32_t *d_off = ws<int32_t>(c, "lay_off", (size_t)n_labels + 1);
    hipLaunchKernelGGL(k_comp_flags, dim3(g), dim3(256), 0, c->stream, skey, n, flag);
    scan_excl_i32(c, flag, pos, n);
    if (read_i32(c, serr)) {
        FL_CHECK_HIP(hipMemsetAsync(serr, 0, sizeof(int32_t), c->stream));
        throw Error(FL_EHIP, "layout: the label sort's look-back gave up");
    }
    FL_REQUIRE(read_i32(c, pos + n) == n_labels, "the number of distinct labels differs from the component count");
    hipLaunchKernelGGL(k_comp_offsets, dim3(g), dim3(256), 0, c->stream, flag, pos, n, d_off);
    FL_LAUNCH_CHECK();
    r.flag = flag;
    r.pos = pos;
    r.d_off = d_off;
    r.off.resize((size_t)n_labels + 1);
    FL_CHECK_HIP(hipMemcpyAsync(r.off.data(), d_off, sizeof(int32_t) * ((size_t)n_labels + 1), hipMemcpyDeviceToHost,
                                c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    return r;
}

void layout(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *deg, float *x, float *y,
            const fl_fa2_params *fa2, int32_t fa2_iters, const fl_kk_params *kk, int32_t kk_max_nodes,
            int32_t fmm_min_nodes, fl_layout_stats *stats)
{
    auto t0 = std::chrono::steady_clock::now();
    fa2_validate(c, n, row_ptr, col, deg, fa2);
    check_kk_params(kk);
    FL_REQUIRE(kk_max_nodes >= 1 && kk_max_nodes <= 256, "kk_max_nodes must be in [1, 256]");
    FL_REQUIRE(fa2_iters >= 0, "fa2_iters must be >= 0");
    const unsigned g = grid_for(n, 256);
    int32_t *label = ws<int32_t>(c, "lay_label", n);
    const int32_t ncomp = components(c, n, row_ptr, col, label);
    LabelSort ls = sort_by_label(c, n, label, ncomp);
    const int32_t *perm = ls.perm, *flag = ls.flag, *pos = ls.pos, *d_off = ls.d_off;
    const std::vector<int32_t> &off = ls.off;

    // classify, then regroup: ForceAtlas2 groups (one per distinct resolved
    // repulsion configuration) first, then the Kamada-Kawai components, then
    // single nodes; label order within each class
    struct Cfg {
        int rep, p, leaf;
        bool operator<(const Cfg &o) const
        {
            return rep != o.rep ? rep < o.rep : (p != o.p ? p < o.p : leaf < o.leaf);
        }
    };
    std::map<Cfg, std::vector<int32_t>> groups;
    std::map<Cfg, fl_fa2_params> group_prm;
    std::vector<int32_t> kk_list, single_list;
    int64_t kk_nodes = 0, fa2_nodes = 0;
    int32_t n_fa2 = 0;
    for (int k = 0; k < ncomp; ++k) {
        const int sz = off[k + 1] - off[k];
        if (sz == 1) {
            single_list.push_back(k);
        } else if (sz <= kk_max_nodes) {
            kk_list.push_back(k);
            kk_nodes += sz;
        } else {
            fl_fa2_params pr = resolve_repulsion(c->tuning, sz, *fa2);
            if (fa2->repulsion == FL_REP_FMM && sz < fmm_min_nodes) pr.repulsion = FL_REP_EXACT;
            pr.list_lanes = fa2->list_lanes;  // a batch's launch shape follows the batch's size
            const Cfg key = pr.repulsion == FL_REP_EXACT ? Cfg{FL_REP_EXACT, 0, 0}
                                                          : Cfg{FL_REP_FMM, pr.p, pr.leaf_size};
            groups[key].push_back(k);
            group_prm[key] = pr;
            fa2_nodes += sz;
            ++n_fa2;
        }
    }
    std::vector<int32_t> newstart(ncomp), neworder;
    neworder.reserve(ncomp);
    for (auto &kv : groups)
        for (int32_t k : kv.second) neworder.push_back(k);
    for (int32_t k : kk_list) neworder.push_back(k);
    for (int32_t k : single_list) neworder.push_back(k);
    std::vector<int32_t> newoff(ncomp + 1, 0);
    for (int j = 0; j < ncomp; ++j) {
        const int k = neworder[j];
        newstart[k] = newoff[j];
        newoff[j + 1] = newoff[j] + (off[k + 1] - off[k]);
    }
    int32_t *d_newstart = ws<int32_t>(c, "lay_newstart", (size_t)ncomp);
    FL_CHECK_HIP(hipMemcpyAsync(d_newstart, newstart.data(), sizeof(int32_t) * ncomp, hipMemcpyHostToDevice,
                                c->stream));
    int32_t *perm2 = ws<int32_t>(c, "lay_perm2", n);
    hipLaunchKernelGGL(k_regroup, dim3(g), dim3(256), 0, c->stream, perm, (const int32_t *)flag,
                       (const int32_t *)pos, (const int32_t *)d_off, (const int32_t *)d_newstart, n, perm2);
    FL_LAUNCH_CHECK();

    int32_t *inv = ws<int32_t>(c, "lay_inv", n), *ndeg = ws<int32_t>(c, "lay_ndeg", n);
    float *xs = ws<float>(c, "lay_xs", n), *ys = ws<float>(c, "lay_ys", n);
    hipLaunchKernelGGL(k_permute_nodes, dim3(g), dim3(256), 0, c->stream, (const int32_t *)perm2, n, deg, x, y, inv,
                       ndeg, xs, ys);
    int32_t *nrow_ptr = ws<int32_t>(c, "lay_rp", (size_t)n + 1);
    scan_excl_i32(c, ndeg, nrow_ptr, n);
    const int32_t nnz = read_i32(c, row_ptr + n);
    int32_t *ncol = ws<int32_t>(c, "lay_col", nnz > 0 ? nnz : 1);
    hipLaunchKernelGGL(k_permute_cols, dim3(g), dim3(256), 0, c->stream, (const int32_t *)perm2, inv, n, row_ptr,
                       col, nrow_ptr, ncol);
    FL_LAUNCH_CHECK();
    const double ms_setup = ms_since(t0);

    auto t1 = std::chrono::steady_clock::now();
    const int n_first_single = newoff[ncomp - (int)single_list.size()];  // single nodes come last
    if (!single_list.empty()) {
        hipLaunchKernelGGL(k_zero_range, dim3(grid_for(n - n_first_single, 256)), dim3(256), 0, c->stream, xs, ys,
                           n_first_single, n);
        FL_LAUNCH_CHECK();
    }
    {
        std::vector<int32_t> kk_ids;
        const int first_kk = ncomp - (int)single_list.size() - (int)kk_list.size();
        for (int j = 0; j < (int)kk_list.size(); ++j) kk_ids.push_back(first_kk + j);
        kk_layout_subset(c, ncomp, newoff.data(), kk_ids, nrow_ptr, ncol, xs, ys, *kk);
    }
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    const double ms_kk = ms_since(t1);

    auto t2 = std::chrono::steady_clock::now();
    int32_t *flags = ws<int32_t>(c, "lay_flags", 1);
    fill_i32(c, flags, 1, 0);
    if (!groups.empty()) {
        // one local CSR per group (rows [gs, ge) of the regrouped CSR, ids
        // shifted to the group), side by side: group j keeps rows
        // [gs + j, ge + j] of lrp
        int32_t *lrp = ws<int32_t>(c, "lay_lrp", (size_t)n + groups.size() + 1);
        int32_t *lcol = ws<int32_t>(c, "lay_lcol", nnz > 0 ? nnz : 1);
        std::vector<FA2Batch> batches;
        int j = 0, ci = 0;
        for (auto &kv : groups) {
            const int gs = newoff[ci], cnt = (int)kv.second.size();
            const int ge = newoff[ci + cnt];
            const int32_t e0 = read_i32(c, nrow_ptr + gs), e1 = read_i32(c, nrow_ptr + ge);
            int32_t *rp = lrp + gs + j, *cl = lcol + e0;
            hipLaunchKernelGGL(k_local_csr, dim3(grid_for((int64_t)(ge - gs) + 1, 256, 1024)), dim3(256), 0,
                               c->stream, (const int32_t *)nrow_ptr, (const int32_t *)ncol, gs, ge - gs, rp, cl);
            FL_LAUNCH_CHECK();
            FA2Batch b;
            b.coff.resize(cnt + 1);
            for (int q = 0; q <= cnt; ++q) b.coff[q] = newoff[ci + q] - gs;
            b.nnz = (int64_t)e1 - e0;
            b.row_ptr = rp;
            b.col = cl;
            b.deg = ndeg + gs;
            b.x = xs + gs;
            b.y = ys + gs;
            b.prm = group_prm[kv.first];
            batches.push_back(std::move(b));
            ci += cnt;
            ++j;
        }
        fa2_run_batches(c, batches, fa2_iters, flags);
    }
    hipLaunchKernelGGL(k_unpermute_pos, dim3(g), dim3(256), 0, c->stream, (const int32_t *)perm2, n,
                       (const float *)xs, (const float *)ys, x, y);
    FL_LAUNCH_CHECK();
    const int32_t f = read_i32(c, flags);
    const double ms_fa2 = ms_since(t2);
    if (f & 1) throw Error(FL_ENONFINITE, "non-finite force in a ForceAtlas2 component");
    if (f & 2) throw Error(FL_ENONFINITE, "non-finite position in a ForceAtlas2 component");
    if (stats) {
        stats->n_comp = ncomp;
        stats->n_single = (int32_t)single_list.size();
        stats->n_kk = (int32_t)kk_list.size();
        stats->n_fa2 = n_fa2;
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
