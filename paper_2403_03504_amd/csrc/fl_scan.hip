// Device-wide exclusive scans and a stable LSD radix sort, written for wave64.
//
// Scan: reduce tiles -> rescan every tile with the sum of the tiles before it
// (two launches; the tile sums are scanned first only when there are many).
//
// Radix sort, 8-bit digits: two launches count the digits of every pass, then
// each pass is one launch in which a block ranks a tile of 4096 or 8192 keys
// (each wave ranks its keys step by step with ballot-built "same digit" lane
// masks, no atomics, so equal digits keep the input order) and finds the
// keys of each digit in the tiles before it by decoupled look-back.  Inputs
// of more than 1024 tiles take a three-launch pass instead (per-tile
// histograms, a scan of them, the scatter).
#include <algorithm>
#include <type_traits>

#include "fl_common.h"

namespace fl {

namespace {

constexpr int SC_NT = 256;
constexpr int SC_IPT = 8;
constexpr int SC_TILE = SC_NT * SC_IPT;  // 2048
constexpr int SC_TOP_NT = 1024;

template <class T>
__device__ __forceinline__ void scan_reduce_tile(const T *__restrict__ in, int64_t n, const int32_t *__restrict__ dn,
                                                 T *__restrict__ part, int64_t bx)
{
    __shared__ T lds[SC_NT / WAVE];
    int64_t live = dn ? (int64_t)*dn : n;
    if (live > n) live = n;
    int64_t base = bx * SC_TILE;
    T s = T(0);
#pragma unroll
    for (int i = 0; i < SC_IPT; ++i) {
        int64_t idx = base + (int64_t)i * SC_NT + threadIdx.x;
        if (idx < live) s += in[idx];
    }
    s = block_sum<T, SC_NT>(s, lds);
    if (threadIdx.x == 0) part[bx] = s;
}

template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_reduce(const T *__restrict__ in, int64_t n,
                                                        const int32_t *__restrict__ dn, T *__restrict__ part)
{
    scan_reduce_tile<T>(in, n, dn, part, blockIdx.x);
}

// Each block adds the sums of the tiles before it, then scans its own tile.
// With few tiles (<= SC_DIRECT) a block adds the raw tile sums itself in a
// fixed order; with more, they were scanned beforehand (part then holds the
// exclusive prefixes and part[ntiles] the total).  Block 0 also writes the
// total to out[live] and out[n].  Entries past `live` are only written inside
// the last live tile.
constexpr int64_t SC_DIRECT = 4096;

template <class T>
__device__ __forceinline__ void scan_down_tile(const T *__restrict__ in, T *__restrict__ out, int64_t n,
                                               const int32_t *__restrict__ dn, const T *__restrict__ part,
                                               int scanned, int64_t bx)
{
    __shared__ T lds[SC_NT / WAVE];
    int64_t live = dn ? (int64_t)*dn : n;
    if (live > n) live = n;
    const int64_t tile0 = bx * SC_TILE;
    const int64_t nlive_tiles = (live + SC_TILE - 1) / SC_TILE;
    if (bx == 0) {
        T tot = T(0);
        if (scanned) {
            tot = part[nlive_tiles];
        } else {
            for (int64_t b = threadIdx.x; b < nlive_tiles; b += SC_NT) tot += part[b];
            tot = block_sum<T, SC_NT>(tot, lds);
        }
        if (threadIdx.x == 0) {
            out[live] = tot;
            out[n] = tot;
        }
    }
    if (tile0 >= live) return;  // the whole block
    T carry = T(0);
    if (scanned) {
        carry = part[bx];
    } else {
        for (int64_t b = threadIdx.x; b < bx; b += SC_NT) carry += part[b];
        carry = block_sum<T, SC_NT>(carry, lds);
    }
    const int64_t base = tile0 + (int64_t)threadIdx.x * SC_IPT;
    T v[SC_IPT];
    T s = T(0);
#pragma unroll
    for (int i = 0; i < SC_IPT; ++i) {
        int64_t idx = base + i;
        v[i] = idx < live ? in[idx] : T(0);
        s += v[i];
    }
    T tot;
    T ex = block_excl_scan<T, SC_NT>(s, lds, tot);
    T run = carry + ex;
#pragma unroll
    for (int i = 0; i < SC_IPT; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
}

template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_down(const T *__restrict__ in, T *__restrict__ out, int64_t n,
                                                      const int32_t *__restrict__ dn, const T *__restrict__ part,
                                                      int scanned)
{
    scan_down_tile<T>(in, out, n, dn, part, scanned, blockIdx.x);
}

// An input of one tile, in one launch: the block's own total is the scan's
// (integer types only, where the order of the additions does not matter).
template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_single(const T *__restrict__ in, T *__restrict__ out, int64_t n,
                                                        const int32_t *__restrict__ dn)
{
    __shared__ T lds[SC_NT / WAVE];
    int64_t live = dn ? (int64_t)*dn : n;
    if (live > n) live = n;
    const int64_t base = (int64_t)threadIdx.x * SC_IPT;
    T v[SC_IPT];
    T s = T(0);
#pragma unroll
    for (int i = 0; i < SC_IPT; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < live ? in[idx] : T(0);
        s += v[i];
    }
    T tot;
    T run = block_excl_scan<T, SC_NT>(s, lds, tot);
    if (live > 0) {
#pragma unroll
        for (int i = 0; i < SC_IPT; ++i) {
            const int64_t idx = base + i;
            if (idx < n) out[idx] = run;
            run += v[i];
        }
    }
    if (threadIdx.x == 0) {
        out[live] = tot;
        out[n] = tot;
    }
}

// Two independent scans in the same launches: blockIdx.y picks the array
// (each with its own tiles; blocks past an array's tiles do nothing).
template <class T>
struct ScanJob {
    const T *in;
    T *out;
    int64_t n, ntiles;
    const int32_t *dn;
    T *part;
};

template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_reduce_pair(ScanJob<T> a, ScanJob<T> b)
{
    const ScanJob<T> &j = blockIdx.y ? b : a;
    if ((int64_t)blockIdx.x < j.ntiles) scan_reduce_tile<T>(j.in, j.n, j.dn, j.part, blockIdx.x);
}

template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_down_pair(ScanJob<T> a, ScanJob<T> b)
{
    const ScanJob<T> &j = blockIdx.y ? b : a;
    if ((int64_t)blockIdx.x < j.ntiles) scan_down_tile<T>(j.in, j.out, j.n, j.dn, j.part, 0, blockIdx.x);
}

template <class T>
void scan_excl(fl_ctx *c, const T *in, T *out, int64_t n, const int32_t *dn, const char *tag, int depth = 0)
{
    int64_t ntiles = (n + SC_TILE - 1) / SC_TILE;
    if (ntiles < 1) ntiles = 1;
    if (ntiles == 1 && std::is_integral<T>::value) {
        hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(SC_NT), 0, c->stream, in, out, n, dn);
        FL_LAUNCH_CHECK();
        return;
    }
    std::string nm = std::string("scan_part_") + tag + std::to_string(depth);
    T *part = ws<T>(c, nm.c_str(), (size_t)ntiles + 1);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)ntiles), dim3(SC_NT), 0, c->stream, in, n, dn, part);
    const bool scanned = ntiles > SC_DIRECT;
    if (scanned) {  // exclusive prefixes of the tile sums, total at part[ntiles]
        std::string nm2 = std::string("scan_pfx_") + tag + std::to_string(depth);
        T *pfx = ws<T>(c, nm2.c_str(), (size_t)ntiles + 1);
        scan_excl<T>(c, part, pfx, ntiles, nullptr, tag, depth + 1);
        part = pfx;
    }
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)ntiles), dim3(SC_NT), 0, c->stream, in, out, n, dn,
                       (const T *)part, scanned ? 1 : 0);
    FL_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// radix sort
constexpr int RS_NT = 1024;          // threads of every sort block
constexpr int RS_NW = RS_NT / WAVE;  // 16 waves
// The tile of one block: STEPS 64-key steps per wave.  4096 keys for up to
// RS_LARGE_FROM keys, 8192 above: a long input's passes then walk half as
// many tiles back, while a shorter one keeps more blocks in flight.
template <int STEPS_>
struct RsCfg {
    static constexpr int STEPS = STEPS_;
    static constexpr int WTILE = STEPS * WAVE;   // keys per wave
    static constexpr int TILE = RS_NW * WTILE;  // keys per block
};
using RsSmall = RsCfg<4>;
using RsLarge = RsCfg<8>;
constexpr int64_t RS_LARGE_FROM = 1536 * 1024;
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;  // digit d is thread d's in the per-digit steps
static_assert(RS_NT >= RS_BINS, "a thread per digit");
constexpr int RS_MAXPASS = 8;  // 64-bit keys

template <class K, class C>
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                    int32_t *__restrict__ hist, int nblocks)
{
    __shared__ int cnt[RS_BINS];
    if (threadIdx.x < RS_BINS) cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * C::TILE;
#pragma unroll 4
    for (int i = 0; i < C::TILE / RS_NT; ++i) {
        int64_t idx = base + (int64_t)i * RS_NT + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(int)((keys[idx] >> shift) & (RS_BINS - 1))], 1);
    }
    __syncthreads();
    if (threadIdx.x < RS_BINS) hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// The LDS of one scatter block.
template <class K, bool HasVal, class C>
struct RsShared {
    int wcnt[RS_NW][RS_BINS];
    int gbase[RS_BINS];
    int lstart[RS_BINS];
    int scan_tmp[RS_NT / WAVE];
    int tile;
    K skey[C::TILE];
    int32_t sval[HasVal ? C::TILE : 1];
};

// Loads tile `tile` and ranks its keys: each wave ranks its C::WTILE keys step
// by step with ballot masks of equal digits (no atomics, so equal digits keep
// the input order), then every digit gets its exclusive prefix over the
// waves (wcnt) and the block's count of the digit is returned to thread d.
template <class K, bool HasVal, class C>
__device__ __forceinline__ int rs_rank(RsShared<K, HasVal, C> &S, const K *__restrict__ kin,
                                       const int32_t *__restrict__ vin, int64_t t0, int64_t t1, int shift,
                                       K (&key)[C::STEPS], int32_t (&val)[C::STEPS], int (&off)[C::STEPS],
                                       int (&dig)[C::STEPS])
{
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    const int64_t wbase = t0 + (int64_t)w * C::WTILE;
#pragma unroll
    for (int st = 0; st < C::STEPS; ++st) {
        int64_t idx = wbase + (int64_t)st * WAVE + lane;
        bool ok = idx < t1;
        key[st] = ok ? kin[idx] : K(0);
        if (HasVal) val[st] = ok ? (vin ? vin[idx] : (int32_t)idx) : 0;  // no input payload: the index
        dig[st] = ok ? (int)((key[st] >> shift) & (RS_BINS - 1)) : -1;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
#pragma unroll
    for (int st = 0; st < C::STEPS; ++st) {
        const int d = dig[st];
        uint64_t mask = __ballot(d >= 0);
#pragma unroll
        for (int b = 0; b < RS_BITS; ++b) {
            uint64_t bal = __ballot((d >> b) & 1);
            mask &= ((d >> b) & 1) ? bal : ~bal;
        }
        int rank = __popcll(mask & lt);
        int cnt = __popcll(mask);
        int leader = mask ? __ffsll((long long)mask) - 1 : lane;
        int b0 = 0;
        if (d >= 0) b0 = S.wcnt[w][d];
        off[st] = b0 + rank;
        if (d >= 0 && lane == leader) S.wcnt[w][d] = b0 + cnt;
    }
    __syncthreads();
    const int t = threadIdx.x;
    int run = 0;
    if (t < RS_BINS) {
#pragma unroll
        for (int ww = 0; ww < RS_NW; ++ww) {
            int cnum = S.wcnt[ww][t];
            S.wcnt[ww][t] = run;
            run += cnum;
        }
    }
    int tot;
    const int ls = block_excl_scan<int, RS_NT>(run, S.scan_tmp, tot);  // the digit's start in the block's order
    if (t < RS_BINS) S.lstart[t] = ls;
    return run;
}

// Places the ranked keys of the tile [t0, t1) in LDS in digit order and
// writes every digit's run to its global position gbase[d] + rank within the
// digit (coalesced); positions at or past `lim` are dropped.
template <class K, bool HasVal, class C>
__device__ __forceinline__ void rs_place(RsShared<K, HasVal, C> &S, K *__restrict__ kout, int32_t *__restrict__ vout,
                                         int64_t t0, int64_t t1, int64_t lim, int shift, const K (&key)[C::STEPS],
                                         const int32_t (&val)[C::STEPS], const int (&off)[C::STEPS],
                                         const int (&dig)[C::STEPS], const float4 *__restrict__ gsrc,
                                         float4 *__restrict__ gdst)
{
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int st = 0; st < C::STEPS; ++st) {
        const int d = dig[st];
        if (d < 0) continue;
        const int lp = S.lstart[d] + S.wcnt[w][d] + off[st];
        S.skey[lp] = key[st];
        if (HasVal) S.sval[lp] = val[st];
    }
    __syncthreads();
    const int live = (int)(t1 - t0);
    for (int i = threadIdx.x; i < live; i += RS_NT) {
        const K k2 = S.skey[i];
        const int d = (int)((k2 >> shift) & (RS_BINS - 1));
        const int64_t pos = (int64_t)S.gbase[d] + (i - S.lstart[d]);
        if (pos < lim) {  // always true unless a look-back gave up (error flagged)
            kout[pos] = k2;
            if (HasVal) {
                const int32_t v = S.sval[i];
                vout[pos] = v;
                if (gdst) gdst[pos] = gsrc[v];  // last pass: the record of the value's index, moved along
            }
        }
    }
}

// Stable scatter of one pass with the per-tile digit histograms scanned
// beforehand (three launches per pass).
template <class K, bool HasVal, class C>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const K *__restrict__ kin, const int32_t *__restrict__ vin,
                                                       K *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
                                                       int shift, const int32_t *__restrict__ hscan, int nblocks,
                                                       const float4 *__restrict__ gsrc, float4 *__restrict__ gdst)
{
    __shared__ RsShared<K, HasVal, C> S;
    for (int i = threadIdx.x; i < RS_NW * RS_BINS; i += RS_NT) (&S.wcnt[0][0])[i] = 0;
    if (threadIdx.x < RS_BINS) S.gbase[threadIdx.x] = hscan[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    K key[C::STEPS];
    int32_t val[C::STEPS];
    int off[C::STEPS], dig[C::STEPS];
    const int64_t t0 = (int64_t)blockIdx.x * C::TILE, t1 = t0 + C::TILE < n ? t0 + C::TILE : n;
    rs_rank<K, HasVal, C>(S, kin, vin, t0, t1, shift, key, val, off, dig);
    __syncthreads();
    rs_place<K, HasVal, C>(S, kout, vout, t0, t1, n, shift, key, val, off, dig, gsrc, gdst);
}

// ---- one launch per pass: decoupled look-back --------------------------------
// Two launches count the digits of every pass over the whole input, per tile
// and then summed (the global digit offsets of a pass do not depend on the
// order of the keys).  Each pass is then one launch: a block takes the next
// tile in launch order from a ticket counter, ranks it, publishes its per-digit
// counts, and finds the number of keys of each digit in the tiles before it
// by walking back over their published words until one carries an inclusive
// prefix (Merrill & Garland 2016); the first pass reads its tiles' prefixes
// from the counting launches instead.  A tile waits only on tiles that were
// taken before it, by blocks that are running and publish their counts
// before they wait themselves, so every wait ends; a bounded spin guards the
// launch anyway and flags an error instead of hanging.
//
// Status word of (pass, tile, digit): flag in bits 30-31 (0 none yet,
// 1 count of this tile, 2 inclusive prefix up to this tile), value in bits
// 0-29.
constexpr uint32_t RS_AGG = 1u << 30, RS_PFX = 2u << 30, RS_VAL = (1u << 30) - 1u;
constexpr uint32_t RS_SPIN_LIMIT = 1u << 22;
constexpr int RS_LOOK = 8;  // tiles read per look-back step
// Larger inputs take the three-launch pass: their look-back chains grow with
// the tile count while launch overhead matters less (8M keys at most here,
// far below the 2^30 the status words hold).
constexpr int RS_LOOKBACK_TILES = 1024;

// Keys [t0, t1) of a tile; its positions lie in [base, lim) (its system's
// range, the whole input without segments); `first`: the first tile of its
// system, which publishes an inclusive prefix at once.
struct RsTile {
    int64_t t0, t1, base, lim;
    int sys;
    bool first;
};

template <class C>
__device__ __forceinline__ RsTile rs_tile(const RsSegs &sg, int64_t n, int tile)
{
    RsTile r;
    if (sg.tiles) {
        const int2 td = sg.tiles[tile];
        r.sys = td.x;
        r.t0 = td.y;
        r.base = sg.coff[td.x];
        r.lim = sg.coff[td.x + 1];
        r.first = tile == sg.toff[td.x];
    } else {
        r.sys = 0;
        r.t0 = (int64_t)tile * C::TILE;
        r.base = 0;
        r.lim = n;
        r.first = tile == 0;
    }
    r.t1 = r.t0 + C::TILE < r.lim ? r.t0 + C::TILE : r.lim;
    return r;
}

// Digit counts of all passes per tile (LDS counts, written out
// per tile), the clearing of every pass's status words, and (block 0) the
// zeroing of the summed counts and the tickets; the launches after this one
// on the stream see all of it.
template <class K, class C>
__global__ __launch_bounds__(RS_NT) void k_rs_hist_all(const K *__restrict__ keys, int64_t n, int passes,
                                                        uint32_t *__restrict__ part, uint32_t *__restrict__ status,
                                                        int64_t nstatus, uint32_t *__restrict__ gh, int ngh,
                                                        RsSegs sg)
{
    __shared__ uint32_t cnt[RS_MAXPASS][RS_BINS];
    for (int i = threadIdx.x; i < RS_MAXPASS * RS_BINS; i += RS_NT) (&cnt[0][0])[i] = 0u;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < ngh; i += RS_NT) gh[i] = 0u;
    const int64_t stride = (int64_t)gridDim.x * RS_NT;
    for (int64_t i = (int64_t)blockIdx.x * RS_NT + threadIdx.x; i < nstatus; i += stride) status[i] = 0u;
    __syncthreads();
    const RsTile tl = rs_tile<C>(sg, n, blockIdx.x);
    for (int64_t i = tl.t0 + threadIdx.x; i < tl.t1; i += RS_NT) {
        const K k = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&cnt[p][(int)((k >> (p * RS_BITS)) & (RS_BINS - 1))], 1u);
    }
    __syncthreads();
    if (threadIdx.x < RS_BINS)
        for (int p = 0; p < passes; ++p)
            part[((int64_t)blockIdx.x * passes + p) * RS_BINS + threadIdx.x] = cnt[p][threadIdx.x];
}

// Sums the per-tile counts: one block per (pass, digit) entry, its waves
// over consecutive runs of tiles, then the waves' totals in wave order
// (integers: the order does not matter).  The first pass's tiles are the
// input's own, so for it the block also writes every tile's exclusive prefix
// of the digit (pfx0[tile][digit]): that pass needs no look-back.
__global__ __launch_bounds__(RS_NT) void k_rs_hist_sum(const uint32_t *__restrict__ part, int ntiles, int passes,
                                                        uint32_t *__restrict__ gh, uint32_t *__restrict__ pfx0)
{
    __shared__ uint32_t wt[RS_NW];
    const int i = blockIdx.x;  // pass * 256 + digit
    const int64_t st = (int64_t)passes * RS_BINS;
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    const int per = ((ntiles + RS_NW - 1) / RS_NW + WAVE - 1) / WAVE * WAVE;  // tiles per wave
    const int tb = w * per, te = min(ntiles, tb + per);
    uint32_t sum = 0u;
    for (int b = tb + lane; b < te; b += WAVE) sum += part[(int64_t)b * st + i];
    sum = wave_sum(sum);
    if (lane == 0) wt[w] = sum;
    __syncthreads();
    uint32_t base = 0u, tot = 0u;
    for (int k = 0; k < RS_NW; ++k) {
        if (k < w) base += wt[k];
        tot += wt[k];
    }
    if (i < RS_BINS) {
        // the wave's tiles again (now in cache), as exclusive prefixes
        for (int b0 = tb; b0 < te; b0 += WAVE) {
            const int b = b0 + lane;
            const uint32_t v = b < te ? part[(int64_t)b * st + i] : 0u;
            const uint32_t inc = wave_incl_scan(v);
            if (b < te) pfx0[(int64_t)b * RS_BINS + i] = base + inc - v;
            base += __shfl(inc, WAVE - 1, WAVE);
        }
    }
    if (threadIdx.x == 0) gh[i] = tot;
}

// The same per system: one wave per (system, pass, digit) entry, its lanes
// over the system's tiles; gh[(system * passes + pass) * 256 + digit], and
// the first pass's tile prefixes within each system.
__global__ __launch_bounds__(RS_NT) void k_rs_hist_sum_seg(const uint32_t *__restrict__ part, int passes, RsSegs sg,
                                                            uint32_t *__restrict__ gh, uint32_t *__restrict__ pfx0)
{
    const int64_t i = (int64_t)blockIdx.x * RS_NW + threadIdx.x / WAVE;
    const int64_t per = (int64_t)passes * RS_BINS;
    if (i >= (int64_t)sg.K * per) return;
    const int sys = (int)(i / per), r = (int)(i - sys * per), ps = r / RS_BINS, d = r - ps * RS_BINS;
    const int tb = sg.toff[sys], te = sg.toff[sys + 1];
    const int lane = lane_id();
    uint32_t sum = 0u;
    if (ps == 0) {
        for (int b0 = tb; b0 < te; b0 += WAVE) {
            const int b = b0 + lane;
            const uint32_t v = b < te ? part[(int64_t)b * per + r] : 0u;
            const uint32_t inc = wave_incl_scan(v);
            if (b < te) pfx0[(int64_t)b * RS_BINS + d] = sum + inc - v;
            sum += __shfl(inc, WAVE - 1, WAVE);
        }
    } else {
        for (int b = tb + lane; b < te; b += WAVE) sum += part[(int64_t)b * per + r];
        sum = wave_sum(sum);
    }
    if (lane == 0) gh[i] = sum;
}

template <class K, bool HasVal, class C>
__global__ __launch_bounds__(RS_NT) void k_rs_onesweep(const K *__restrict__ kin, const int32_t *__restrict__ vin,
                                                        K *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
                                                        int shift, const uint32_t *__restrict__ gh, int ghstride,
                                                        uint32_t *__restrict__ status, uint32_t *__restrict__ ticket,
                                                        const uint32_t *__restrict__ pfx, int32_t *__restrict__ err,
                                                        const float4 *__restrict__ gsrc, float4 *__restrict__ gdst,
                                                        RsSegs sg)
{
    __shared__ RsShared<K, HasVal, C> S;
    for (int i = threadIdx.x; i < RS_NW * RS_BINS; i += RS_NT) (&S.wcnt[0][0])[i] = 0;
    // with the tiles' prefixes given (first pass) the tile is the block's own
    if (threadIdx.x == 0) S.tile = pfx ? (int)blockIdx.x : (int)atomicAdd(ticket, 1u);
    __syncthreads();
    const int tile = S.tile;
    K key[C::STEPS];
    int32_t val[C::STEPS];
    int off[C::STEPS], dig[C::STEPS];
    const int d = threadIdx.x;
    const bool dig_thread = d < RS_BINS;  // thread d handles digit d
    const RsTile tl = rs_tile<C>(sg, n, tile);
    const uint32_t cnt = (uint32_t)rs_rank<K, HasVal, C>(S, kin, vin, tl.t0, tl.t1, shift, key, val, off, dig);
    uint32_t *my = status + (int64_t)tile * RS_BINS + d;
    if (!pfx && dig_thread)
        __hip_atomic_store(my, (tl.first ? RS_PFX : RS_AGG) | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // start of the digit in the system: counts of the smaller digits
    int tot;
    const uint32_t dstart = (uint32_t)block_excl_scan<int, RS_NT>(
        dig_thread ? (int)gh[(int64_t)tl.sys * ghstride + d] : 0, S.scan_tmp, tot);
    uint32_t before = 0;
    if (!dig_thread) {
    } else if (pfx) {
        before = pfx[(int64_t)tile * RS_BINS + d];
    } else if (!tl.first) {
        // the walk ends at an inclusive prefix, at the latest on the first
        // tile of the system (it publishes one at once)
        // look back RS_LOOK tiles at a time (independent loads in flight),
        // consuming counts in order until an inclusive prefix; a tile that
        // has published nothing yet stops the window and is read again
        int j = tile - 1;
        uint32_t spins = 0;
        for (;;) {
            uint32_t v[RS_LOOK];
#pragma unroll
            for (int u = 0; u < RS_LOOK; ++u)
                v[u] = j - u >= 0 ? __hip_atomic_load(status + (int64_t)(j - u) * RS_BINS + d, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                                  : 0u;  // never consumed: a first tile publishes a prefix
            int used = 0;
            bool pfx = false;
#pragma unroll
            for (int u = 0; u < RS_LOOK; ++u) {
                const uint32_t f = v[u] & ~RS_VAL;
                if (f == 0u) break;
                before += v[u] & RS_VAL;
                used = u + 1;
                if (f == RS_PFX) {
                    pfx = true;
                    break;
                }
            }
            if (pfx) break;
            j -= used;
            if (used == 0) {
                if (++spins > RS_SPIN_LIMIT) {
                    atomicOr(err, 8);
                    before = (uint32_t)n;  // every write of this digit is then out of range and skipped
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(my, RS_PFX | ((before + cnt) & RS_VAL), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (dig_thread) S.gbase[d] = (int)(tl.base + dstart + before);
    __syncthreads();
    rs_place<K, HasVal, C>(S, kout, vout, tl.t0, tl.t1, tl.lim, shift, key, val, off, dig, gsrc, gdst);
}

template <class K, bool HasVal, class C>
bool radix_sort_c(fl_ctx *c, K *k, int32_t *v, K *kt, int32_t *vt, int64_t n, int nbits, const char *tag,
                  int32_t *err, const float4 *gsrc, float4 *gdst, bool vals_iota)
{
    if (n <= 0) return false;
    const int nblocks = (int)((n + C::TILE - 1) / C::TILE);
    const int passes = (nbits + RS_BITS - 1) / RS_BITS;
    K *ka = k, *kb = kt;
    int32_t *va = v, *vb = vt;
    if (nblocks <= RS_LOOKBACK_TILES && passes <= RS_MAXPASS) {
        // gh (passes x 256 digit counts) and the tickets share one buffer
        const int nz = passes * RS_BINS + passes;
        uint32_t *gh = ws<uint32_t>(c, (std::string("rs_gh_") + tag).c_str(), (size_t)nz);
        uint32_t *ticket = gh + passes * RS_BINS;
        uint32_t *part = ws<uint32_t>(c, (std::string("rs_part_") + tag).c_str(), (size_t)nblocks * passes * RS_BINS);
        const int64_t nstatus = (int64_t)passes * nblocks * RS_BINS;
        uint32_t *status = ws<uint32_t>(c, (std::string("rs_status_") + tag).c_str(), (size_t)nstatus);
        if (!err) err = ws_zeroed<int32_t>(c, "rs_err", 1);
        hipLaunchKernelGGL((k_rs_hist_all<K, C>), dim3(nblocks), dim3(RS_NT), 0, c->stream, (const K *)k, n, passes,
                           part, status, nstatus, gh, nz, RsSegs{});
        uint32_t *pfx0 = ws<uint32_t>(c, (std::string("rs_pfx0_") + tag).c_str(), (size_t)nblocks * RS_BINS);
        hipLaunchKernelGGL(k_rs_hist_sum, dim3(passes * RS_BINS), dim3(RS_NT), 0, c->stream,
                           (const uint32_t *)part, nblocks, passes, gh, pfx0);
        for (int ps = 0; ps < passes; ++ps) {
            hipLaunchKernelGGL((k_rs_onesweep<K, HasVal, C>), dim3(nblocks), dim3(RS_NT), 0, c->stream, (const K *)ka,
                               (const int32_t *)(ps == 0 && vals_iota ? nullptr : va), kb, vb, n, ps * RS_BITS,
                               (const uint32_t *)(gh + ps * RS_BINS), 0,
                               status + (int64_t)ps * nblocks * RS_BINS, ticket + ps,
                               ps == 0 ? (const uint32_t *)pfx0 : (const uint32_t *)nullptr, err,
                               ps == passes - 1 ? gsrc : nullptr, ps == passes - 1 ? gdst : nullptr, RsSegs{});
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        FL_LAUNCH_CHECK();
        return (passes & 1) != 0;
    }
    std::string hn = std::string("rs_hist_") + tag;
    int32_t *hist = ws<int32_t>(c, hn.c_str(), (size_t)RS_BINS * nblocks * 2 + 1);
    int32_t *hscan = hist + (size_t)RS_BINS * nblocks;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = ps * RS_BITS;
        hipLaunchKernelGGL((k_rs_hist<K, C>), dim3(nblocks), dim3(RS_NT), 0, c->stream, ka, n, shift, hist, nblocks);
        scan_excl<int32_t>(c, hist, hscan, (int64_t)RS_BINS * nblocks, nullptr, tag);
        hipLaunchKernelGGL((k_rs_scatter<K, HasVal, C>), dim3(nblocks), dim3(RS_NT), 0, c->stream, ka,
                           ps == 0 && vals_iota ? nullptr : va, kb, vb, n,
                           shift, hscan, nblocks, ps == passes - 1 ? gsrc : nullptr,
                           ps == passes - 1 ? gdst : nullptr);
        FL_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return (passes & 1) != 0;
}

template <class K, bool HasVal>
bool radix_sort(fl_ctx *c, K *k, int32_t *v, K *kt, int32_t *vt, int64_t n, int nbits, const char *tag,
                int32_t *err, const float4 *gsrc = nullptr, float4 *gdst = nullptr, bool vals_iota = false)
{
    return radix_sort_tile(n) == RsLarge::TILE
               ? radix_sort_c<K, HasVal, RsLarge>(c, k, v, kt, vt, n, nbits, tag, err, gsrc, gdst, vals_iota)
               : radix_sort_c<K, HasVal, RsSmall>(c, k, v, kt, vt, n, nbits, tag, err, gsrc, gdst, vals_iota);
}

template <class C>
void sort_seg_launches(fl_ctx *c, uint32_t *k, int32_t *v, uint32_t *kt, int32_t *vt, int64_t n, int passes,
                       int32_t *err, const RsSegs &sg, const float4 *gsrc, float4 *gdst, bool vals_iota)
{
    const int nt = sg.ntiles;
    const int64_t per = (int64_t)passes * RS_BINS;
    // per-system digit counts, then the tickets (the only words zeroed)
    uint32_t *gh = ws<uint32_t>(c, "rs_gh_seg", (size_t)(sg.K * per + passes));
    uint32_t *ticket = gh + sg.K * per;
    uint32_t *part = ws<uint32_t>(c, "rs_part_seg", (size_t)nt * per);
    const int64_t nstatus = (int64_t)nt * per;
    uint32_t *status = ws<uint32_t>(c, "rs_status_seg", (size_t)nstatus);
    if (!err) err = ws_zeroed<int32_t>(c, "rs_err", 1);
    hipLaunchKernelGGL((k_rs_hist_all<uint32_t, C>), dim3(nt), dim3(RS_NT), 0, c->stream, (const uint32_t *)k, n,
                       passes, part, status, nstatus, ticket, passes, sg);
    uint32_t *pfx0 = ws<uint32_t>(c, "rs_pfx0_seg", (size_t)nt * RS_BINS);
    hipLaunchKernelGGL(k_rs_hist_sum_seg, dim3((unsigned)((sg.K * per + RS_NW - 1) / RS_NW)), dim3(RS_NT), 0,
                       c->stream, (const uint32_t *)part, passes, sg, gh, pfx0);
    uint32_t *ka = k, *kb = kt;
    int32_t *va = v, *vb = vt;
    for (int ps = 0; ps < passes; ++ps) {
        hipLaunchKernelGGL((k_rs_onesweep<uint32_t, true, C>), dim3(nt), dim3(RS_NT), 0, c->stream,
                           (const uint32_t *)ka, (const int32_t *)(ps == 0 && vals_iota ? nullptr : va), kb, vb, n,
                           ps * RS_BITS,
                           (const uint32_t *)(gh + ps * RS_BINS), (int)per, status + (int64_t)ps * nt * RS_BINS,
                           ticket + ps, ps == 0 ? (const uint32_t *)pfx0 : (const uint32_t *)nullptr, err,
                           ps == passes - 1 ? gsrc : nullptr, ps == passes - 1 ? gdst : nullptr, sg);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    FL_LAUNCH_CHECK();
}

}  // namespace

int radix_sort_tile(int64_t n) { return n > RS_LARGE_FROM ? RsLarge::TILE : RsSmall::TILE; }

void scan_excl_i32(fl_ctx *c, const int32_t *in, int32_t *out, int64_t n, const int32_t *dn)
{
    scan_excl<int32_t>(c, in, out, n, dn, "i32");
}

void scan_excl_i64(fl_ctx *c, const int64_t *in, int64_t *out, int64_t n, const int32_t *dn)
{
    scan_excl<int64_t>(c, in, out, n, dn, "i64");
}

void scan_excl_i64_pair(fl_ctx *c, const int64_t *in0, int64_t *out0, int64_t n0, const int32_t *dn0,
                        const int64_t *in1, int64_t *out1, int64_t n1, const int32_t *dn1)
{
    const int64_t t0 = std::max<int64_t>(1, (n0 + SC_TILE - 1) / SC_TILE);
    const int64_t t1 = std::max<int64_t>(1, (n1 + SC_TILE - 1) / SC_TILE);
    if (t0 > SC_DIRECT || t1 > SC_DIRECT) {  // a recursive scan: one at a time
        scan_excl<int64_t>(c, in0, out0, n0, dn0, "i64");
        scan_excl<int64_t>(c, in1, out1, n1, dn1, "i64b");
        return;
    }
    ScanJob<int64_t> a{in0, out0, n0, t0, dn0, ws<int64_t>(c, "scan_pair_a", (size_t)t0 + 1)};
    ScanJob<int64_t> b{in1, out1, n1, t1, dn1, ws<int64_t>(c, "scan_pair_b", (size_t)t1 + 1)};
    const dim3 grid((unsigned)std::max(t0, t1), 2);
    hipLaunchKernelGGL(k_scan_reduce_pair<int64_t>, grid, dim3(SC_NT), 0, c->stream, a, b);
    hipLaunchKernelGGL(k_scan_down_pair<int64_t>, grid, dim3(SC_NT), 0, c->stream, a, b);
    FL_LAUNCH_CHECK();
}

void scan_excl_f64(fl_ctx *c, const double *in, double *out, int64_t n, const int32_t *dn, const char *tag)
{
    scan_excl<double>(c, in, out, n, dn, tag);
}

bool radix_sort_seg_fits(int64_t n, int ntiles) { return n > 0 && ntiles >= 1 && ntiles <= RS_LOOKBACK_TILES; }

bool radix_sort_u32_seg(fl_ctx *c, uint32_t *k, int32_t *v, uint32_t *kt, int32_t *vt, int64_t n, int nbits,
                        int32_t *err, const RsSegs &sg, const float4 *gsrc, float4 *gdst, bool vals_iota)
{
    if (n <= 0) return false;
    const int passes = (nbits + RS_BITS - 1) / RS_BITS;
    FL_REQUIRE(radix_sort_seg_fits(n, sg.ntiles) && passes <= RS_MAXPASS && sg.tiles && sg.K >= 1,
               "segmented sort: tiles out of range");
    FL_REQUIRE(sg.tile == RsSmall::TILE || sg.tile == RsLarge::TILE, "segmented sort: tiles of an unknown size");
    if (sg.tile == RsLarge::TILE)
        sort_seg_launches<RsLarge>(c, k, v, kt, vt, n, passes, err, sg, gsrc, gdst, vals_iota);
    else
        sort_seg_launches<RsSmall>(c, k, v, kt, vt, n, passes, err, sg, gsrc, gdst, vals_iota);
    return (passes & 1) != 0;
}

bool radix_sort_u32(fl_ctx *c, uint32_t *k, int32_t *v, uint32_t *kt, int32_t *vt, int64_t n, int nbits,
                    int32_t *err, const float4 *gsrc, float4 *gdst, bool vals_iota)
{
    return radix_sort<uint32_t, true>(c, k, v, kt, vt, n, nbits, "u32", err, gsrc, gdst, vals_iota);
}

bool radix_sort_u64(fl_ctx *c, uint64_t *k, uint64_t *kt, int64_t n, int nbits, int32_t *err)
{
    return radix_sort<uint64_t, false>(c, k, nullptr, kt, nullptr, n, nbits, "u64", err);
}

bool radix_sort_u64v(fl_ctx *c, uint64_t *k, int32_t *v, uint64_t *kt, int32_t *vt, int64_t n, int nbits,
                     int32_t *err)
{
    return radix_sort<uint64_t, true>(c, k, v, kt, vt, n, nbits, "u64v", err);
}

}  // namespace fl
