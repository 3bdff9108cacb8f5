// Context management, error plumbing and per-phase timing of libfa2lay.
#include "fl_tree.h"

#include <cstdio>

namespace fl {

PhaseTimer::PhaseTimer(fl_ctx *ctx, int phase) : c(ctx), ph(phase)
{
    if (!c->timing) return;
    if (c->ev_free.empty()) {
        hipEvent_t e;
        FL_CHECK_HIP(hipEventCreate(&e));
        c->ev_free.push_back(e);
    }
    a = c->ev_free.back();
    c->ev_free.pop_back();
    FL_CHECK_HIP(hipEventRecord(a, c->stream));
}

PhaseTimer::~PhaseTimer() noexcept(false)
{
    if (!a) return;
    hipEvent_t b;
    if (c->ev_free.empty()) {
        if (hipEventCreate(&b) != hipSuccess) return;
    } else {
        b = c->ev_free.back();
        c->ev_free.pop_back();
    }
    if (hipEventRecord(b, c->stream) != hipSuccess) return;
    c->ev_pending.push_back({ph, {a, b}});
    // bound the number of outstanding events: fold the oldest ones once the
    // stream has passed them (this synchronises, so keep the window large)
    if (c->ev_pending.size() > 4096) flush_timing(c);
}

void flush_timing(fl_ctx *c)
{
    for (auto &pe : c->ev_pending) {
        FL_CHECK_HIP(hipEventSynchronize(pe.second.second));
        float ms = 0.f;
        FL_CHECK_HIP(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
        c->phase_ms[pe.first] += ms;
        c->phase_cnt[pe.first] += 1;
        c->ev_free.push_back(pe.second.first);
        c->ev_free.push_back(pe.second.second);
    }
    c->ev_pending.clear();
}

namespace {
thread_local bool t_recording = false;
}

std::shared_mutex &alloc_capture_mutex()
{
    static std::shared_mutex m;
    return m;
}

bool recording_thread() { return t_recording; }

CaptureGuard::CaptureGuard() : lk(alloc_capture_mutex()) { t_recording = true; }

CaptureGuard::~CaptureGuard() { t_recording = false; }

void free_retired(fl_ctx *c)
{
    if (c->retired.empty()) return;
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    for (auto s : c->aux)
        if (s) FL_CHECK_HIP(hipStreamSynchronize(s));
    AllocGuard guard;
    for (auto &r : c->retired) (void)hipFree(r.first);
    c->ws_bytes -= c->retired_bytes;
    c->retired.clear();
    c->retired_bytes = 0;
}

void *arena_carve(fl_ctx *c, size_t bytes, const char *name)
{
    const size_t off = (c->arena_used + 255) & ~size_t(255);
    const size_t len = (bytes + 255) & ~size_t(255);
    if (off > c->arena_cap || len > c->arena_cap - off)
        throw Error(FL_ENOMEM, std::string("the call needs more than the ") + std::to_string(c->arena_cap) +
                                   " bytes of its fixed scratch (at buffer " + name + ")");
    c->arena_used = off + len;
    return c->arena + off;
}

static size_t held_with_branches(const fl_ctx *o)
{
    size_t b = o->ws_bytes;
    for (const fl_ctx *sc : o->sub) b += sc->ws_bytes;
    return b;
}

void budget_check(fl_ctx *c, size_t bytes, const char *name)
{
    fl_ctx *o = c->owner ? c->owner : c;
    if (!o->budget || held_with_branches(o) + bytes <= o->budget) return;
    free_retired(o);
    for (fl_ctx *sc : o->sub) free_retired(sc);
    const size_t held = held_with_branches(o);
    if (held + bytes > o->budget)
        throw Error(FL_ENOMEM, std::string("workspace budget of ") + std::to_string(o->budget) +
                                   " bytes exceeded: " + std::to_string(held) + " held, " + std::to_string(bytes) +
                                   " more for " + name);
}

hipStream_t aux_stream(fl_ctx *c, int i)
{
    if (!c->aux[i]) FL_CHECK_HIP(hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking));
    return c->aux[i];
}

fl_ctx *sub_ctx(fl_ctx *c, size_t b)
{
    while (c->sub.size() <= b) {
        hipStream_t s = nullptr;
        FL_CHECK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        fl_ctx *sc = nullptr;
        if (fl_create(&sc, c->device, s, 0) != FL_OK) {
            (void)hipStreamDestroy(s);
            throw Error(FL_EHIP, "branch context creation failed");
        }
        sc->own_stream = true;
        sc->owner = c->owner ? c->owner : c;  // the budget is the owning context's
        c->sub.push_back(sc);
    }
    return c->sub[b];
}

}  // namespace fl

using namespace fl;

extern "C" {

const char *fl_version(void) { return "fa2lay 0.1 gfx950"; }

fl_status fl_create(fl_ctx **out, int device, void *stream, size_t workspace_budget_bytes)
{
    if (!out) return FL_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FL_EINVAL;
    fl_ctx *c = new (std::nothrow) fl_ctx();
    if (!c) return FL_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->budget = workspace_budget_bytes;
    fl_default_tuning(&c->tuning);
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return FL_EHIP;
    }
    AllocGuard guard;
    if (hipMalloc(&c->d_stats, 16 * sizeof(int64_t)) != hipSuccess) {
        delete c;
        return FL_ENOMEM;
    }
    if (hipMemset(c->d_stats, 0, 16 * sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc(&c->host_stage, 4096, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(c->d_stats);
        delete c;
        return FL_EHIP;
    }
    *out = c;
    return FL_OK;
}

void fl_destroy(fl_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto *s : c->sub) fl_destroy(s);
    for (auto s : c->aux)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    for (hipEvent_t e : {c->ev_fork, c->ev_join, c->ev_fork2, c->ev_join2, c->ev_lists})
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    AllocGuard guard;
    for (auto &r : c->retired) (void)hipFree(r.first);
    for (auto &kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    for (auto &pe : c->ev_pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    for (auto e : c->ev_free) (void)hipEventDestroy(e);
    if (c->d_stats) (void)hipFree(c->d_stats);
    if (c->host_stage) (void)hipHostFree(c->host_stage);
    delete c;
}

const char *fl_last_error(const fl_ctx *c) { return c ? c->err.c_str() : "null context"; }

fl_status fl_set_stream(fl_ctx *c, void *stream)
{
    FL_API_BEGIN(c)
    c->stream = (hipStream_t)stream;
    FL_API_END(c)
}

fl_status fl_synchronize(fl_ctx *c)
{
    FL_API_BEGIN(c)
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    // a quiet point: the stream has drained, and so have the branch
    // contexts (their work joins the context's stream)
    free_retired(c);
    for (auto *sc : c->sub) free_retired(sc);
    FL_API_END(c)
}

size_t fl_workspace_bytes(const fl_ctx *c) { return c ? c->ws_bytes : 0; }

fl_status fl_set_timing(fl_ctx *c, int enable)
{
    FL_API_BEGIN(c)
    c->timing = enable != 0;
    FL_API_END(c)
}

fl_status fl_set_graphs(fl_ctx *c, int enable)
{
    FL_API_BEGIN(c)
    c->use_graphs = enable != 0;
    FL_API_END(c)
}

fl_status fl_get_timing(fl_ctx *c, double *ms, int64_t *counts)
{
    FL_API_BEGIN(c)
    flush_timing(c);
    for (int i = 0; i < FL_NPHASE; ++i) {
        if (ms) ms[i] = c->phase_ms[i];
        if (counts) counts[i] = c->phase_cnt[i];
        c->phase_ms[i] = 0.0;
        c->phase_cnt[i] = 0;
    }
    FL_API_END(c)
}

fl_status fl_fmm_stats(fl_ctx *c, int64_t *out, int reset)
{
    FL_API_BEGIN(c)
    FL_REQUIRE(out != nullptr, "fl_fmm_stats: null output");
    tree_max_level(c);
    FL_CHECK_HIP(hipMemcpyAsync(c->host_stage, c->d_stats, FL_NSTATS * sizeof(int64_t), hipMemcpyDeviceToHost,
                                c->stream));
    FL_CHECK_HIP(hipStreamSynchronize(c->stream));
    std::memcpy(out, c->host_stage, FL_NSTATS * sizeof(int64_t));
    if (reset) FL_CHECK_HIP(hipMemsetAsync(c->d_stats + 8, 0, 4 * sizeof(int64_t), c->stream));
    FL_API_END(c)
}

}  // extern "C"
