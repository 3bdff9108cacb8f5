// Autotuning of the repulsion: exact or FMM per system size, and the FMM's
// expansion order and leaf size, chosen by measurement on the device.  The
// paper fixes none of these (it states only that the FMM is O(n), sec. 3.2.1),
// so the choice is the fastest configuration that keeps the force error
// under a caller's bound.
//
// Errors are measured against the exact O(n^2) repulsion on the same points
// (FP32 pair terms, FP64 sums: good to about 1e-7 relative), with an FP64
// device reduction of |F - F_exact|^2 and |F_exact|^2.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fl_fa2.h"
#include "fl_fmm.h"

namespace fl {
namespace {

constexpr int ERR_BLOCKS = 512;
constexpr int ERR_NT = 256;
const int TUNE_P[] = {4, 6, 8, 10, 12, 16};
const int TUNE_LEAF[] = {16, 24, 32, 48, 64, 96, 128};
const int TUNE_LANES[] = {1, 8};

// per-block partial sums of |a - b|^2 and |b|^2 in FP64
__global__ __launch_bounds__(ERR_NT) void k_err_partial(int n, const float2 *__restrict__ a,
                                                         const float2 *__restrict__ b, double2 *__restrict__ part)
{
    __shared__ double lds[ERR_NT / WAVE];
    double d = 0.0, r = 0.0;
    for (int i = blockIdx.x * ERR_NT + threadIdx.x; i < n; i += gridDim.x * ERR_NT) {
        const float2 av = a[i], bv = b[i];
        const double ex = (double)bv.x, ey = (double)bv.y;
        const double dx = (double)av.x - ex, dy = (double)av.y - ey;
        d += dx * dx + dy * dy;
        r += ex * ex + ey * ey;
    }
    d = block_sum<double, ERR_NT>(d, lds);
    r = block_sum<double, ERR_NT>(r, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(d, r);
}

double rel_err(fl_ctx *c, int n, const float2 *a, const float2 *b)
{
    double2 *part = ws<double2>(c, "tune_part", ERR_BLOCKS);
    hipLaunchKernelGGL(k_err_partial, dim3(ERR_BLOCKS), dim3(ERR_NT), 0, c->stream, n, a, b, part);
    FL_LAUNCH_CHECK();
    std::vector<double2> h(ERR_BLOCKS);
    FL_CHECK_HIP(hipMemcpyAsync(h.data(), part, sizeof(double2) * ERR_BLOCKS, hipMemcpyDeviceToHost, c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    double d = 0.0, r = 0.0;
    for (const auto &v : h) {
        d += v.x;
        r += v.y;
    }
    return r > 0.0 ? std::sqrt(d / r) : std::sqrt(d);
}

// median duration in ms of `reps` runs of f on the context's stream (after
// one untimed run that sizes the workspace)
template <class F>
double time_median(fl_ctx *c, int reps, F &&f)
{
    f();
    hipEvent_t a, b;
    FL_CHECK_HIP(hipEventCreate(&a));
    FL_CHECK_HIP(hipEventCreate(&b));
    std::vector<double> ms;
    try {
        for (int r = 0; r < reps; ++r) {
            FL_CHECK_HIP(hipEventRecord(a, c->stream));
            f();
            FL_CHECK_HIP(hipEventRecord(b, c->stream));
            FL_CHECK_HIP(hipEventSynchronize(b));
            float t = 0.f;
            FL_CHECK_HIP(hipEventElapsedTime(&t, a, b));
            ms.push_back(t);
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

}  // namespace

void check_tuning(const fl_tuning &t)
{
    FL_REQUIRE(t.fmm_min_nodes >= 1, "tuning: fmm_min_nodes must be >= 1");
    FL_REQUIRE(t.n_buckets >= 1 && t.n_buckets <= FL_TUNE_MAX_BUCKETS, "tuning: n_buckets must be in [1, 16]");
    for (int b = 0; b < t.n_buckets; ++b) {
        FL_REQUIRE(fmm_order_supported(t.p[b]), "tuning: p must be one of 4, 6, 8, 10, 12, 16");
        FL_REQUIRE(t.leaf_size[b] >= 1 && t.leaf_size[b] <= 1024, "tuning: leaf_size must be in [1, 1024]");
        FL_REQUIRE(t.list_lanes[b] == 0 || t.list_lanes[b] == 1 || t.list_lanes[b] == 8,
                   "tuning: list_lanes must be 0, 1 or 8");
        FL_REQUIRE(t.bucket_max[b] >= 1, "tuning: bucket_max must be >= 1");
        FL_REQUIRE(b == 0 || t.bucket_max[b] > t.bucket_max[b - 1], "tuning: bucket_max must be ascending");
    }
    FL_REQUIRE(std::isfinite(t.max_rel_err) && t.max_rel_err >= 0.0, "tuning: max_rel_err must be >= 0");
}

fl_fa2_params resolve_repulsion(const fl_tuning &t, int64_t n, const fl_fa2_params &p)
{
    if (p.repulsion != FL_REP_AUTO) return p;
    fl_fa2_params r = p;
    if (n < t.fmm_min_nodes) {
        r.repulsion = FL_REP_EXACT;
        return r;
    }
    int b = 0;
    while (b + 1 < t.n_buckets && n > t.bucket_max[b]) ++b;
    r.repulsion = FL_REP_FMM;
    r.p = t.p[b];
    r.leaf_size = t.leaf_size[b];
    if (p.list_lanes == 0) r.list_lanes = t.list_lanes[b];
    return r;
}

static void autotune(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, int32_t n_sizes,
                     const int32_t *sizes, double max_rel_err, int32_t reps, fl_tuning *out,
                     std::vector<fl_tune_sample> &samples)
{
    FL_REQUIRE(n >= 2 && x && y && deg && sizes && out, "fl_autotune: bad arguments");
    FL_REQUIRE(n_sizes >= 1 && n_sizes <= FL_TUNE_MAX_BUCKETS, "fl_autotune: n_sizes must be in [1, 16]");
    FL_REQUIRE(max_rel_err >= 1e-6 && max_rel_err <= 1.0, "fl_autotune: max_rel_err must be in [1e-6, 1]");
    FL_REQUIRE(reps >= 1 && reps <= 20, "fl_autotune: reps must be in [1, 20]");
    for (int k = 0; k < n_sizes; ++k) {
        FL_REQUIRE(sizes[k] >= 2 && sizes[k] <= n, "fl_autotune: sizes must be in [2, n]");
        FL_REQUIRE(k == 0 || sizes[k] > sizes[k - 1], "fl_autotune: sizes must be ascending");
    }
    float2 *ex = ws<float2>(c, "tune_ex", n);
    float2 *fx = ws<float2>(c, "tune_fx", n);
    const int bits = 16;
    std::vector<double> t_exact(n_sizes), t_fmm(n_sizes);
    fl_tuning t{};
    t.n_buckets = n_sizes;
    t.max_rel_err = max_rel_err;
    for (int k = 0; k < n_sizes; ++k) {
        const int s = sizes[k];
        const Segs sg = segs_single(c, s);
        t_exact[k] = time_median(c, reps, [&] { exact_repulsion(c, sg, x, y, deg, 1.f, ex); });
        samples.push_back(fl_tune_sample{s, 0, 0, 0, 1, t_exact[k], 0.0});
        double best = INFINITY, best_err = INFINITY, closest = INFINITY, closest_ms = INFINITY;
        int bp = 8, bl = 64, bn = 1, cp = 16, cl = 16, cn = 1;
        for (int p : TUNE_P) {
            for (int leaf : TUNE_LEAF) {
                for (int lanes : TUNE_LANES) {
                    const double ms = time_median(
                        c, reps, [&] { fmm_repulsion(c, sg, x, y, deg, p, leaf, bits, lanes, 1.f, fx); });
                    if (tree_error_bits(c, true)) throw Error(FL_EHIP, "FMM capacity guard tripped while tuning");
                    const double e = rel_err(c, s, fx, ex);
                    const int ok = e <= max_rel_err ? 1 : 0;
                    samples.push_back(fl_tune_sample{s, p, leaf, lanes, ok, ms, e});
                    if (ok && ms < best) {
                        best = ms;
                        best_err = e;
                        bp = p;
                        bl = leaf;
                        bn = lanes;
                    }
                    if (e < closest || (e == closest && ms < closest_ms)) {
                        closest = e;
                        closest_ms = ms;
                        cp = p;
                        cl = leaf;
                        cn = lanes;
                    }
                }
            }
        }
        if (!std::isfinite(best_err)) {  // no configuration meets the bound: the most accurate one
            bp = cp;
            bl = cl;
            bn = cn;
            best = closest_ms;
        }
        t_fmm[k] = best;
        t.p[k] = bp;
        t.leaf_size[k] = bl;
        t.list_lanes[k] = bn;
        t.bucket_max[k] = k + 1 < n_sizes ? (int32_t)std::floor(std::sqrt((double)s * sizes[k + 1])) : INT32_MAX;
    }
    // crossover: the FMM is faster from size index k0 on
    int k0 = n_sizes;
    while (k0 > 0 && t_fmm[k0 - 1] < t_exact[k0 - 1]) --k0;
    if (k0 == 0) t.fmm_min_nodes = sizes[0];
    else if (k0 == n_sizes) t.fmm_min_nodes = sizes[n_sizes - 1] + 1;
    else t.fmm_min_nodes = (int32_t)std::ceil(std::sqrt((double)sizes[k0 - 1] * sizes[k0]));
    check_tuning(t);
    *out = t;
}

}  // namespace fl

using namespace fl;

extern "C" {

void fl_default_tuning(fl_tuning *out)
{
    if (!out) return;
    *out = fl_tuning{};
    out->fmm_min_nodes = 4096;
    out->n_buckets = 1;
    out->bucket_max[0] = INT32_MAX;
    out->p[0] = 8;
    out->leaf_size[0] = 64;
    out->list_lanes[0] = 0;
    out->max_rel_err = 0.0;
}

fl_status fl_set_tuning(fl_ctx *c, const fl_tuning *tuning)
{
    FL_API_BEGIN(c)
    fl_tuning t;
    if (tuning) t = *tuning;
    else fl_default_tuning(&t);
    check_tuning(t);
    c->tuning = t;
    FL_API_END(c)
}

fl_status fl_get_tuning(fl_ctx *c, fl_tuning *out)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(out != nullptr, "null output");
    *out = c->tuning;
    FL_API_END(c)
}

fl_status fl_autotune(fl_ctx *c, int32_t n, const float *x, const float *y, const int32_t *deg, int32_t n_sizes,
                      const int32_t *sizes, double max_rel_err, int32_t reps, fl_tuning *out,
                      fl_tune_sample *samples, int32_t samples_cap, int32_t *n_samples)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(samples_cap >= 0 && (samples || samples_cap == 0), "fl_autotune: bad sample buffer");
    std::vector<fl_tune_sample> sm;
    fl_tuning t;
    autotune(c, n, x, y, deg, n_sizes, sizes, max_rel_err, reps, &t, sm);
    c->tuning = t;
    if (out) *out = t;
    for (int i = 0; i < (int)sm.size() && i < samples_cap; ++i) samples[i] = sm[i];
    if (n_samples) *n_samples = (int32_t)sm.size();
    FL_API_END(c)
}

}  // extern "C"
