// Device-wide exclusive scans and a stable LSD radix sort, written for wave64.
//
// Scan: reduce tiles -> rescan every tile with the sum of the tiles before it
// (two launches; the tile sums are scanned first only when there are many).  Radix sort: per pass, a digit histogram per tile, a scan of the
// digit-major histogram, and a stable scatter in which each wave ranks its
// keys step by step with ballot-built "same digit" lane masks (no atomics in
// the ranking, so the order of equal digits is the input order).
#include "fl_common.h"

namespace fl {

namespace {

constexpr int SC_NT = 256;
constexpr int SC_IPT = 8;
constexpr int SC_TILE = SC_NT * SC_IPT;  // 2048
constexpr int SC_TOP_NT = 1024;

template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_reduce(const T *__restrict__ in, int64_t n,
                                                        const int32_t *__restrict__ dn, T *__restrict__ part)
{
    __shared__ T lds[SC_NT / WAVE];
    int64_t live = dn ? (int64_t)*dn : n;
    if (live > n) live = n;
    int64_t base = (int64_t)blockIdx.x * SC_TILE;
    T s = T(0);
#pragma unroll
    for (int i = 0; i < SC_IPT; ++i) {
        int64_t idx = base + (int64_t)i * SC_NT + threadIdx.x;
        if (idx < live) s += in[idx];
    }
    s = block_sum<T, SC_NT>(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Each block adds the sums of the tiles before it, then scans its own tile.
// With few tiles (<= SC_DIRECT) a block adds the raw tile sums itself in a
// fixed order; with more, they were scanned beforehand (part then holds the
// exclusive prefixes and part[ntiles] the total).  Block 0 also writes the
// total to out[live] and out[n].  Entries past `live` are only written inside
// the last live tile.
constexpr int64_t SC_DIRECT = 4096;

template <class T>
__global__ __launch_bounds__(SC_NT) void k_scan_down(const T *__restrict__ in, T *__restrict__ out, int64_t n,
                                                      const int32_t *__restrict__ dn, const T *__restrict__ part,
                                                      int scanned)
{
    __shared__ T lds[SC_NT / WAVE];
    int64_t live = dn ? (int64_t)*dn : n;
    if (live > n) live = n;
    const int64_t tile0 = (int64_t)blockIdx.x * SC_TILE;
    const int64_t nlive_tiles = (live + SC_TILE - 1) / SC_TILE;
    if (blockIdx.x == 0) {
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
        carry = part[blockIdx.x];
    } else {
        for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SC_NT) carry += part[b];
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
void scan_excl(fl_ctx *c, const T *in, T *out, int64_t n, const int32_t *dn, const char *tag, int depth = 0)
{
    int64_t ntiles = (n + SC_TILE - 1) / SC_TILE;
    if (ntiles < 1) ntiles = 1;
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
constexpr int RS_NT = 256;
constexpr int RS_NW = RS_NT / WAVE;  // 4 waves
constexpr int RS_STEPS = 16;         // 64-key steps per wave
constexpr int RS_WTILE = RS_STEPS * WAVE;  // 1024 keys per wave
constexpr int RS_TILE = RS_NW * RS_WTILE;  // 4096 keys per block
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;

template <class K>
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                    int32_t *__restrict__ hist, int nblocks)
{
    __shared__ int cnt[RS_BINS];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int i = 0; i < RS_TILE / RS_NT; ++i) {
        int64_t idx = base + (int64_t)i * RS_NT + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(int)((keys[idx] >> shift) & (RS_BINS - 1))], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one pass.  Each wave ranks its 1024 keys step by step
// (ballot masks of equal digits), the block then places its 4096 keys in LDS
// in digit order and writes every digit's run contiguously (coalesced).
template <class K, bool HasVal>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const K *__restrict__ kin, const int32_t *__restrict__ vin,
                                                       K *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
                                                       int shift, const int32_t *__restrict__ hscan, int nblocks)
{
    __shared__ int wcnt[RS_NW][RS_BINS];
    __shared__ int gbase[RS_BINS];
    __shared__ int lstart[RS_BINS];
    __shared__ int scan_tmp[RS_NT / WAVE];
    __shared__ K skey[RS_TILE];
    __shared__ int32_t sval[HasVal ? RS_TILE : 1];
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    for (int i = threadIdx.x; i < RS_NW * RS_BINS; i += RS_NT) (&wcnt[0][0])[i] = 0;
    gbase[threadIdx.x] = hscan[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();

    const int64_t wbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_WTILE;
    K key[RS_STEPS];
    int32_t val[RS_STEPS];
    int off[RS_STEPS];
    int dig[RS_STEPS];
#pragma unroll
    for (int s = 0; s < RS_STEPS; ++s) {
        int64_t idx = wbase + (int64_t)s * WAVE + lane;
        bool ok = idx < n;
        key[s] = ok ? kin[idx] : K(0);
        if (HasVal) val[s] = ok ? vin[idx] : 0;
        dig[s] = ok ? (int)((key[s] >> shift) & (RS_BINS - 1)) : -1;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
#pragma unroll
    for (int s = 0; s < RS_STEPS; ++s) {
        const int d = dig[s];
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
        if (d >= 0) b0 = wcnt[w][d];
        off[s] = b0 + rank;
        if (d >= 0 && lane == leader) wcnt[w][d] = b0 + cnt;
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves, and the digit's start in
    // the block's digit-sorted order
    {
        int t = threadIdx.x, run = 0;
#pragma unroll
        for (int ww = 0; ww < RS_NW; ++ww) {
            int cnum = wcnt[ww][t];
            wcnt[ww][t] = run;
            run += cnum;
        }
        int tot;
        int ex = block_excl_scan<int, RS_NT>(run, scan_tmp, tot);
        lstart[t] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RS_STEPS; ++s) {
        const int d = dig[s];
        if (d < 0) continue;
        const int lp = lstart[d] + wcnt[w][d] + off[s];
        skey[lp] = key[s];
        if (HasVal) sval[lp] = val[s];
    }
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    const int live = (int)((n - tile0) < RS_TILE ? (n - tile0) : RS_TILE);
    for (int i = threadIdx.x; i < live; i += RS_NT) {
        const K k2 = skey[i];
        const int d = (int)((k2 >> shift) & (RS_BINS - 1));
        const int64_t pos = (int64_t)gbase[d] + (i - lstart[d]);
        kout[pos] = k2;
        if (HasVal) vout[pos] = sval[i];
    }
}

template <class K, bool HasVal>
bool radix_sort(fl_ctx *c, K *k, int32_t *v, K *kt, int32_t *vt, int64_t n, int nbits, const char *tag)
{
    if (n <= 0) return false;
    int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    std::string hn = std::string("rs_hist_") + tag;
    int32_t *hist = ws<int32_t>(c, hn.c_str(), (size_t)RS_BINS * nblocks * 2 + 1);
    int32_t *hscan = hist + (size_t)RS_BINS * nblocks;
    int passes = (nbits + RS_BITS - 1) / RS_BITS;
    K *ka = k, *kb = kt;
    int32_t *va = v, *vb = vt;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = ps * RS_BITS;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3(nblocks), dim3(RS_NT), 0, c->stream, ka, n, shift, hist, nblocks);
        scan_excl<int32_t>(c, hist, hscan, (int64_t)RS_BINS * nblocks, nullptr, tag);
        hipLaunchKernelGGL((k_rs_scatter<K, HasVal>), dim3(nblocks), dim3(RS_NT), 0, c->stream, ka, va, kb, vb, n,
                           shift, hscan, nblocks);
        FL_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return (passes & 1) != 0;
}

}  // namespace

void scan_excl_i32(fl_ctx *c, const int32_t *in, int32_t *out, int64_t n, const int32_t *dn)
{
    scan_excl<int32_t>(c, in, out, n, dn, "i32");
}

void scan_excl_i64(fl_ctx *c, const int64_t *in, int64_t *out, int64_t n, const int32_t *dn)
{
    scan_excl<int64_t>(c, in, out, n, dn, "i64");
}

void scan_excl_f64(fl_ctx *c, const double *in, double *out, int64_t n, const int32_t *dn, const char *tag)
{
    scan_excl<double>(c, in, out, n, dn, tag);
}

bool radix_sort_u32(fl_ctx *c, uint32_t *k, int32_t *v, uint32_t *kt, int32_t *vt, int64_t n, int nbits)
{
    return radix_sort<uint32_t, true>(c, k, v, kt, vt, n, nbits, "u32");
}

bool radix_sort_u64(fl_ctx *c, uint64_t *k, uint64_t *kt, int64_t n, int nbits)
{
    return radix_sort<uint64_t, false>(c, k, nullptr, kt, nullptr, n, nbits, "u64");
}

bool radix_sort_u64v(fl_ctx *c, uint64_t *k, int32_t *v, uint64_t *kt, int32_t *vt, int64_t n, int nbits)
{
    return radix_sort<uint64_t, true>(c, k, v, kt, vt, n, nbits, "u64v");
}

}  // namespace fl
