// Internal header of libfa2lay: context, workspace, error plumbing and the
// wave64 device helpers shared by the kernels.  Written for gfx950 (CDNA4):
// 64-lane wavefronts, 256-thread workgroups unless a kernel says otherwise.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fa2lay.h"

namespace fl {

constexpr int WAVE = 64;

struct Error : std::runtime_error {
    fl_status code;
    Error(fl_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define FL_CHECK_HIP(expr)                                                                          \
    do {                                                                                            \
        hipError_t _e = (expr);                                                                     \
        if (_e != hipSuccess)                                                                       \
            throw ::fl::Error(FL_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));          \
    } while (0)

#define FL_REQUIRE(cond, msg)                                                                       \
    do {                                                                                            \
        if (!(cond)) throw ::fl::Error(FL_EINVAL, msg);                                             \
    } while (0)

#define FL_LAUNCH_CHECK() FL_CHECK_HIP(hipGetLastError())

// Entry points: validate, run, map exceptions to fl_status and the
// context's last-error text.  Nothing is thrown across the C ABI.
#define FL_API_BEGIN(c)                                                                             \
    if (!(c)) return FL_EINVAL;                                                                     \
    try {                                                                                           \
        FL_CHECK_HIP(hipSetDevice((c)->device));

#define FL_API_END(c)                                                                               \
    }                                                                                               \
    catch (const fl::Error &e) {                                                                    \
        (c)->err = e.what();                                                                        \
        return e.code;                                                                              \
    }                                                                                               \
    catch (const std::exception &e) {                                                               \
        (c)->err = e.what();                                                                        \
        return FL_EHIP;                                                                             \
    }                                                                                               \
    return FL_OK;

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

}  // namespace fl

struct fl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::map<std::string, fl::DevBuf> bufs;
    size_t ws_bytes = 0;  // workspace held, retired buffers included
    // workspace buffers replaced by larger ones, freed together once the
    // context's streams are idle (free_retired)
    std::vector<std::pair<void *, size_t>> retired;
    size_t retired_bytes = 0;
    // pinned host staging for small read-backs
    void *host_stage = nullptr;
    // timing
    bool timing = false;
    double phase_ms[FL_NPHASE] = {};
    int64_t phase_cnt[FL_NPHASE] = {};
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    // statistics of the last FMM evaluation live in device memory
    int64_t *d_stats = nullptr;  // [8]
    uint32_t epoch = 0;          // hash-table epoch, advanced per tree build
    bool use_graphs = true;      // fl_fa2_run replays a captured iteration
    fl_tuning tuning{};          // read by FL_REP_AUTO (set in fl_create)
    // private streams (created on first use, destroyed with the context) and
    // branch contexts for concurrent runs of independent systems
    hipStream_t aux[4] = {nullptr, nullptr, nullptr, nullptr};
    // fork/join of the branches of an iteration: the attraction gathers and
    // the FMM's upward pass (created on first use); `branches` off runs them
    // in line on the context's stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_fork2 = nullptr, ev_join2 = nullptr, ev_lists = nullptr;
    bool branches = true;
    std::vector<fl_ctx *> sub;
    bool own_stream = false;     // a branch context destroys its stream
    int32_t seg1_n = -1;         // n of the cached one-system descriptor
    int tree_cbits = 0;          // system-id width of the hash keys last inserted
    // a fixed device arena (the allocation-free entry point's scratch): while
    // set, workspace buffers are carved from it for the one call and nothing
    // is allocated or freed
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    // workspace bound of a context and its branch contexts (0: none); a
    // branch context points at the context that owns the bound
    size_t budget = 0;
    fl_ctx *owner = nullptr;
};

namespace fl {

// Device allocations and frees may synchronise the whole device, and that
// breaks a graph another thread is recording on one of its streams.  They
// hold AllocGuard (exclusive) and recordings hold CaptureGuard (shared), so
// the two never overlap in a process; a thread that is recording takes no
// AllocGuard (HIP refuses its own allocations then, with an error).
std::shared_mutex &alloc_capture_mutex();
bool recording_thread();
struct AllocGuard {
    std::unique_lock<std::shared_mutex> lk;
    AllocGuard()
    {
        if (!recording_thread()) lk = std::unique_lock<std::shared_mutex>(alloc_capture_mutex());
    }
};
struct CaptureGuard {
    std::shared_lock<std::shared_mutex> lk;
    CaptureGuard();   // marks the thread as recording
    ~CaptureGuard();  // clears the mark
};

// Frees the retired workspace buffers after synchronising the context's
// streams (a quiet point: the end of a job, the context's destruction).
void free_retired(fl_ctx *c);

// Grow-only named workspace buffer of at least `count` elements of T.
// The buffer it replaces may still be in use by enqueued work: it is retired
// rather than freed (a free may synchronise the whole device), and retired
// buffers are freed together once they would hold more than half of the
// context's workspace, or at the next quiet point.
// Carves `bytes` (rounded up to 256) from the context's arena; throws
// FL_ENOMEM past its end.
void *arena_carve(fl_ctx *c, size_t bytes, const char *name);
// Throws FL_ENOMEM unless `bytes` more of workspace keep the context (with
// its branch contexts) within its budget; frees retired buffers first when
// that makes the room.
void budget_check(fl_ctx *c, size_t bytes, const char *name);

template <class T>
T *ws(fl_ctx *c, const char *name, size_t count)
{
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    DevBuf &b = c->bufs[name];
    if (c->arena) {
        if (b.cap < bytes) {  // first request in this call, or a larger one: a new piece
            b.p = arena_carve(c, bytes, name);
            b.cap = (bytes + 255) & ~size_t(255);
        }
        return static_cast<T *>(b.p);
    }
    if (b.cap < bytes) {
        if (b.p) {
            c->retired.emplace_back(b.p, b.cap);
            c->retired_bytes += b.cap;
            b.p = nullptr;
            b.cap = 0;
            if (2 * c->retired_bytes > c->ws_bytes) free_retired(c);
        }
        size_t nb = bytes + bytes / 8 + 256;
        budget_check(c, nb, name);
        hipError_t e;
        {
            AllocGuard guard;
            e = hipMalloc(&b.p, nb);
        }
        if (e != hipSuccess && !c->retired.empty()) {  // the retired buffers may make the room
            (void)hipGetLastError();
            free_retired(c);
            AllocGuard guard;
            e = hipMalloc(&b.p, nb);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(FL_ENOMEM, std::string("workspace allocation of ") + std::to_string(nb) + " bytes for " +
                                       name + " failed");
        }
        b.cap = nb;
        c->ws_bytes += nb;
    }
    return static_cast<T *>(b.p);
}

// Zero-filled on first allocation (kept for buffers whose contents must start
// at zero and are kept clean by the kernels that use them).
void fill_i32(fl_ctx *c, int32_t *p, int64_t n, int32_t v);

template <class T>
T *ws_zeroed(fl_ctx *c, const char *name, size_t count)
{
    DevBuf &b = c->bufs[name];
    size_t before = b.cap;
    T *p = ws<T>(c, name, count);
    if (b.cap != before) {
        if (c->arena)  // a fill kernel (a caller may record the arena's calls into a graph)
            fill_i32(c, reinterpret_cast<int32_t *>(p), (int64_t)(b.cap / sizeof(int32_t)), 0);
        else
            FL_CHECK_HIP(hipMemsetAsync(p, 0, b.cap, c->stream));
    }
    return p;
}

// Parameters with FL_REP_AUTO replaced by the choice of `t` for a system of
// n nodes (other modes are returned unchanged).
fl_fa2_params resolve_repulsion(const fl_tuning &t, int64_t n, const fl_fa2_params &p);
// Throws FL_EINVAL unless t is a well-formed table.
void check_tuning(const fl_tuning &t);

// Private stream i (0..3) of the context, created on first use.
hipStream_t aux_stream(fl_ctx *c, int i);
// Branch context b (with its own stream), created on first use.
fl_ctx *sub_ctx(fl_ctx *c, size_t b);

inline unsigned grid_for(int64_t n, int threads, int64_t max_blocks = 1 << 20)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (unsigned)b;
}

// ---- timing helpers --------------------------------------------------------
struct PhaseTimer {
    fl_ctx *c;
    int ph;
    hipEvent_t a = nullptr;
    PhaseTimer(fl_ctx *ctx, int phase);
    ~PhaseTimer() noexcept(false);
};
void flush_timing(fl_ctx *c);

// ---- device helpers --------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ float wave_min_f(float v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ float wave_max_f(float v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Inclusive scan across the 64 lanes of a wave.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    int lane = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        T t = __shfl_up(v, o, WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan over a block of NT threads; returns the exclusive prefix and
// the block total.  `lds` holds NT/64 elements.  Contains __syncthreads.
template <class T, int NT>
__device__ __forceinline__ T block_excl_scan(T v, T *lds, T &total)
{
    constexpr int NW = NT / WAVE;
    int lane = lane_id(), w = threadIdx.x / WAVE;
    T inc = wave_incl_scan(v);
    if (lane == WAVE - 1) lds[w] = inc;
    __syncthreads();
    T wbase = T(0), tot = T(0);
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T s = lds[i];
        if (i < w) wbase += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wbase + inc - v;
}

// Sum over a block of NT threads (deterministic order); result valid in all
// threads.  `lds` holds NT/64 elements.
template <class T, int NT>
__device__ __forceinline__ T block_sum(T v, T *lds)
{
    constexpr int NW = NT / WAVE;
    T s = wave_sum(v);
    if (lane_id() == 0) lds[threadIdx.x / WAVE] = s;
    __syncthreads();
    T tot = T(0);
#pragma unroll
    for (int i = 0; i < NW; ++i) tot += lds[i];
    __syncthreads();
    return tot;
}

// ---- scans and sorts (fl_scan.hip) ----------------------------------------
// Exclusive scan of in[0..n) into out[0..n]; out[n] = total.  n is a host
// bound; when dn != nullptr the live length is *dn (<= n) and elements past it
// read as zero.  Three launches.
void scan_excl_i32(fl_ctx *c, const int32_t *in, int32_t *out, int64_t n, const int32_t *dn = nullptr);
void scan_excl_i64(fl_ctx *c, const int64_t *in, int64_t *out, int64_t n, const int32_t *dn = nullptr);
// Two such scans in the same two launches (separately when either is long
// enough to need the recursive form).
void scan_excl_i64_pair(fl_ctx *c, const int64_t *in0, int64_t *out0, int64_t n0, const int32_t *dn0,
                        const int64_t *in1, int64_t *out1, int64_t n1, const int32_t *dn1);
// FP64 scan, summed in a fixed order (deterministic); `tag` names its
// workspace, so scans whose results are used together need distinct tags.
void scan_excl_f64(fl_ctx *c, const double *in, double *out, int64_t n, const int32_t *dn, const char *tag);

// Stable LSD radix sort of 32-bit keys with int32 payload over bits
// [0, nbits).  Ping-pongs between (k, v) and (kt, vt); returns true when the
// sorted result ended in (kt, vt).  With gdst the last pass also writes
// gdst[i] = gsrc[sorted payload i] (payload values must index gsrc).  With
// vals_iota the payload of key i is i, and v is not read (only written).
// Device error bit 8 goes to *err when a look-back gives up.
bool radix_sort_u32(fl_ctx *c, uint32_t *k, int32_t *v, uint32_t *kt, int32_t *vt, int64_t n, int nbits,
                    int32_t *err = nullptr, const float4 *gsrc = nullptr, float4 *gdst = nullptr,
                    bool vals_iota = false);
bool radix_sort_u64(fl_ctx *c, uint64_t *k, uint64_t *kt, int64_t n, int nbits, int32_t *err = nullptr);

// Keys per tile of the sort of n keys (one block each).
int radix_sort_tile(int64_t n);
// Segmented sort: K independent key ranges [coff[s], coff[s+1]), each sorted
// on its own (stable), cut into system-aligned tiles of `tile` keys (that of
// radix_sort_tile for all the keys): tile t covers [tiles[t].y,
// min(tiles[t].y + tile, coff[tiles[t].x + 1])), the tiles of a system are
// consecutive and in system order.  The result equals one stable sort by
// (system, key), with no system bits in the keys.
struct RsSegs {
    int K = 0, ntiles = 0, tile = 0;
    const int32_t *coff = nullptr;  // [K+1], device
    const int2 *tiles = nullptr;    // [ntiles] (system, first key), device
    const int32_t *toff = nullptr;  // [K+1] first tile of each system, device
};
// whether the segmented one-launch-per-pass sort takes n keys in `ntiles` tiles
bool radix_sort_seg_fits(int64_t n, int ntiles);
bool radix_sort_u32_seg(fl_ctx *c, uint32_t *k, int32_t *v, uint32_t *kt, int32_t *vt, int64_t n, int nbits,
                        int32_t *err, const RsSegs &sg, const float4 *gsrc = nullptr, float4 *gdst = nullptr,
                        bool vals_iota = false);
bool radix_sort_u64v(fl_ctx *c, uint64_t *k, int32_t *v, uint64_t *kt, int32_t *vt, int64_t n, int nbits,
                     int32_t *err = nullptr);

}  // namespace fl
