// Graph preparation (the paper's sec. 2 graph, sec. 4 component split):
//   * CSR of the simple undirected graph of a directed edge list, built by
//     sorting 64-bit (row, col) keys: bit-exact and independent of the order
//     in which equal pairs arrive;
//   * connected components by hooking roots onto smaller roots (atomicMin)
//     and full path compression, repeated until no edge joins two trees.  The
//     surviving root of every tree is its smallest node id, so the labels are
//     unique whatever the interleaving of the atomics.
#include "fl_common.h"

namespace fl {
namespace {

__global__ void k_csr_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m, int64_t n,
                           uint64_t *__restrict__ keys, int32_t *__restrict__ bad)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int64_t u = src[e], v = dst[e];
    const uint64_t sent = (uint64_t)n * (uint64_t)n;
    if (u < 0 || v < 0 || u >= n || v >= n) {
        *bad = 1;
        keys[2 * e] = keys[2 * e + 1] = sent;
        return;
    }
    if (u == v) {
        keys[2 * e] = keys[2 * e + 1] = sent;
    } else {
        keys[2 * e] = (uint64_t)u * (uint64_t)n + (uint64_t)v;
        keys[2 * e + 1] = (uint64_t)v * (uint64_t)n + (uint64_t)u;
    }
}

__global__ void k_csr_flags(const uint64_t *__restrict__ keys, int64_t len, uint64_t sent, int32_t *__restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    uint64_t k = keys[i];
    flag[i] = (k != sent && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
}

__global__ void k_csr_compact(const uint64_t *__restrict__ keys, const int32_t *__restrict__ flag,
                              const int32_t *__restrict__ pos, int64_t len, int64_t n, int32_t *__restrict__ col,
                              uint64_t *__restrict__ ukeys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len || !flag[i]) return;
    uint64_t k = keys[i];
    col[pos[i]] = (int32_t)(k % (uint64_t)n);
    ukeys[pos[i]] = k;
}

// row_ptr[u] = number of distinct pairs with row < u (binary search over the
// sorted distinct keys); no atomics, so hub rows cost nothing extra
__global__ void k_csr_rows(const uint64_t *__restrict__ ukeys, const int32_t *__restrict__ nnz_p, int64_t n,
                           int32_t *__restrict__ row_ptr, int32_t *__restrict__ deg)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    const int64_t nnz = nnz_p ? *nnz_p : 0;
    auto lb = [&](uint64_t v) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (ukeys[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    int64_t a = lb((uint64_t)u * (uint64_t)n);
    row_ptr[u] = (int32_t)a;
    if (u < n) deg[u] = (int32_t)(lb((uint64_t)(u + 1) * (uint64_t)n) - a);
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// components --------------------------------------------------------------
__global__ void k_cc_init(int32_t *__restrict__ parent, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = (int32_t)i;
}

__global__ void k_rows_of(const int32_t *__restrict__ row_ptr, int64_t n, int32_t *__restrict__ rows)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) rows[e] = (int32_t)v;
}

__device__ __forceinline__ int32_t cc_root(const int32_t *parent, int32_t x)
{
    int32_t p = __builtin_nontemporal_load(&parent[x]);
    while (p != x) {
        x = p;
        p = __builtin_nontemporal_load(&parent[x]);
    }
    return x;
}

__global__ void k_cc_hook(const int32_t *__restrict__ rows, const int32_t *__restrict__ col, int64_t nnz,
                          int32_t *parent, int32_t *__restrict__ changed)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int32_t u = rows[e], v = col[e];
    if (u >= v) return;  // each undirected edge once
    int32_t ru = cc_root(parent, u), rv = cc_root(parent, v);
    if (ru == rv) return;
    int32_t hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
    atomicMin(&parent[hi], lo);
    *changed = 1;
}

__global__ void k_cc_compress(int32_t *parent, int64_t n)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t r = cc_root(parent, (int32_t)v);
    parent[v] = r;
}

__global__ void k_cc_count(const int32_t *__restrict__ parent, int64_t n, int32_t *__restrict__ count)
{
    __shared__ int32_t lds[4];
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t c = (v < n && parent[v] == (int32_t)v) ? 1 : 0;
    c = block_sum<int32_t, 256>(c, lds);
    if (threadIdx.x == 0 && c) atomicAdd(count, c);
}

}  // namespace

// host helpers used by other translation units -------------------------------
void fill_i32(fl_ctx *c, int32_t *p, int64_t n, int32_t v)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, p, n, v);
    FL_LAUNCH_CHECK();
}

int32_t read_i32(fl_ctx *c, const int32_t *dp)
{
    FL_CHECK_HIP(hipMemcpyAsync(c->host_stage, dp, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    int32_t v;
    std::memcpy(&v, c->host_stage, sizeof(v));
    return v;
}

int64_t read_i64(fl_ctx *c, const int64_t *dp)
{
    FL_CHECK_HIP(hipMemcpyAsync(c->host_stage, dp, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    int64_t v;
    std::memcpy(&v, c->host_stage, sizeof(v));
    return v;
}

int64_t build_csr(fl_ctx *c, int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *row_ptr,
                  int32_t *col, int32_t *deg)
{
    int64_t len = 2 * m;
    int32_t *bad = ws<int32_t>(c, "csr_bad", 1);
    FL_CHECK_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), c->stream));
    const int32_t *nnz_p = nullptr;
    const uint64_t *ukeys = nullptr;
    if (m > 0) {
        uint64_t *keys = ws<uint64_t>(c, "csr_keys", (size_t)len);
        uint64_t *tmp = ws<uint64_t>(c, "csr_keys_tmp", (size_t)len);
        hipLaunchKernelGGL(k_csr_keys, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, src, dst, m, (int64_t)n, keys,
                           bad);
        FL_LAUNCH_CHECK();
        if (read_i32(c, bad)) throw Error(FL_EINVAL, "fl_build_csr: edge endpoint outside [0, n)");
        const uint64_t sent = (uint64_t)n * (uint64_t)n;
        int nbits = 64 - __builtin_clzll(sent | 1ull);
        int32_t *serr = ws_zeroed<int32_t>(c, "csr_sort_err", 1);
        bool alt = radix_sort_u64(c, keys, tmp, len, nbits, serr);
        uint64_t *sk = alt ? tmp : keys;
        int32_t *flag = ws<int32_t>(c, "csr_flag", (size_t)len);
        int32_t *pos = ws<int32_t>(c, "csr_pos", (size_t)len + 1);
        hipLaunchKernelGGL(k_csr_flags, dim3(grid_for(len, 256)), dim3(256), 0, c->stream, sk, len, sent, flag);
        scan_excl_i32(c, flag, pos, len);
        uint64_t *uk = alt ? keys : tmp;  // the free ping-pong buffer
        hipLaunchKernelGGL(k_csr_compact, dim3(grid_for(len, 256)), dim3(256), 0, c->stream, sk, flag, pos, len,
                           (int64_t)n, col, uk);
        FL_LAUNCH_CHECK();
        nnz_p = pos + len;
        ukeys = uk;
    }
    hipLaunchKernelGGL(k_csr_rows, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, c->stream, ukeys, nnz_p,
                       (int64_t)n, row_ptr, deg);
    FL_LAUNCH_CHECK();
    const int64_t nnz = (int64_t)read_i32(c, row_ptr + n);
    if (m > 0) {
        int32_t *serr = ws_zeroed<int32_t>(c, "csr_sort_err", 1);
        if (read_i32(c, serr)) {
            FL_CHECK_HIP(hipMemsetAsync(serr, 0, sizeof(int32_t), c->stream));
            throw Error(FL_EHIP, "fl_build_csr: the edge sort's look-back gave up");
        }
    }
    return nnz;
}

int32_t components(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *label)
{
    int32_t nnz = read_i32(c, row_ptr + n);
    int32_t *rows = ws<int32_t>(c, "cc_rows", (size_t)nnz + 1);
    int32_t *flag = ws<int32_t>(c, "cc_flag", 2);
    hipLaunchKernelGGL(k_cc_init, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, label, (int64_t)n);
    if (nnz > 0)
        hipLaunchKernelGGL(k_rows_of, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, row_ptr, (int64_t)n, rows);
    FL_LAUNCH_CHECK();
    for (int it = 0; nnz > 0; ++it) {
        FL_CHECK_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), c->stream));
        hipLaunchKernelGGL(k_cc_hook, dim3(grid_for(nnz, 256)), dim3(256), 0, c->stream, rows, col, (int64_t)nnz,
                           label, flag);
        hipLaunchKernelGGL(k_cc_compress, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, label, (int64_t)n);
        FL_LAUNCH_CHECK();
        if (!read_i32(c, flag)) break;
        if (it > 4 * 32 + 64) throw Error(FL_EHIP, "fl_components: no convergence");
    }
    FL_CHECK_HIP(hipMemsetAsync(flag + 1, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_cc_count, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, label, (int64_t)n, flag + 1);
    FL_LAUNCH_CHECK();
    return read_i32(c, flag + 1);
}

}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_build_csr(fl_ctx *c, int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *row_ptr,
                       int32_t *col_idx, int32_t *deg, int64_t *nnz_out)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1 && m >= 0, "fl_build_csr: need n >= 1 and m >= 0");
    FL_REQUIRE(2 * m < (int64_t)INT32_MAX, "fl_build_csr: too many edges for int32 CSR");
    FL_REQUIRE(row_ptr && deg && (m == 0 || (src && dst && col_idx)), "fl_build_csr: null pointer");
    int64_t nnz = build_csr(c, n, m, src, dst, row_ptr, col_idx, deg);
    if (nnz_out) *nnz_out = nnz;
    FL_API_END(c)
}

fl_status fl_components(fl_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t *label,
                        int32_t *n_comp_out)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(n >= 1, "fl_components: need n >= 1");
    FL_REQUIRE(row_ptr && col_idx && label, "fl_components: null pointer");
    int32_t k = components(c, n, row_ptr, col_idx, label);
    if (n_comp_out) *n_comp_out = k;
    FL_API_END(c)
}

}  // extern "C"
