// Index traversal on gfx950 (Algorithm 1, rounds i = K..1; sections 4 and 6.2).
//
// One launch sequence handles a batch of repetitions j0 .. j0+B-1 of round i
// for every dimension: B * D "segments" of n_s windows each.
//
//  * sort_prefixes  stable LSD radix sort of every segment by the length-i
//                   hash prefix of repetition j (left half-function j div m,
//                   right half-function j mod m; section 6.1), one byte per
//                   pass. Pass 0 builds the keys straight from the index; its
//                   histogram comes from the fingerprint-table kernel, which
//                   reads the same index words. Tiles of 4096 elements are
//                   ranked in LDS with wave ballots and written out digit by
//                   digit (coalesced).
//  * k_enum         windows with equal prefixes are adjacent and, the sort
//                   being stable, in increasing window order; each element
//                   walks the rest of its run. For every non-trivial pair it
//                   counts the dimensions where the pair collides (the weight
//                   W of Algorithm 1, computed on the fly as in section 6.2),
//                   emits the pair once (from the lowest colliding dimension)
//                   when W_i >= d, and skips it when it already had W >= d at
//                   prefix i+1 in the same repetition (section 6.2).
//  * k_verify       one wave per candidate: the D per-dimension z-normalised
//                   distances (Eq. zned) in FP64 with coalesced loads, the d
//                   smallest (ties to the lower dimension), dist_d and dist_max.
//  * k_filter/k_pool  the set of distinct verified pairs is kept as a sorted
//                   pool of its P best; TOP is the greedy non-overlapping top-k
//                   of the pool, recomputed after each repetition, with a
//                   snapshot per repetition for the host's stopping check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "internal.h"

namespace mm {

// ------------------------------------------------------------------ helpers
__device__ inline uint32_t lane_id() { return threadIdx.x & 63; }

__device__ inline uint32_t mbcnt64(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int l = (int)lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

// Exclusive scan over the block (NT threads); sh needs NT/64 words. Returns
// the exclusive prefix; *total gets the block sum. Contains barriers: every
// thread of the block must call it.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    const int wave = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane_id() == 63) sh[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) {
        uint32_t s = sh[q];
        if (q < wave) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Prefix of length i of the tensored key of section 6.1: the symbols of the
// left and right half-functions interleaved (l0 r0 l1 r1 ...), first symbol
// most significant. The prefix of length i' < i is this value shifted right by
// 8 (i - i') bits, so one sort by the longest prefix orders every shorter one.
__device__ inline uint64_t spread_bytes(uint32_t v)
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    return x;   // bytes b0 b1 b2 b3 (b0 most significant) -> 0 b0 0 b1 0 b2 0 b3
}

template <typename KT>
__device__ inline KT make_key(uint32_t L, uint32_t R, int i)
{
    const uint64_t full = (spread_bytes(L) << 8) | spread_bytes(R);
    return (KT)(full >> (8 * (8 - i)));
}

// Sort key of a segment element: the prefix itself, or (g.hashed) the top 24
// bits of its multiplicative (Fibonacci) hash
template <typename KT>
__device__ inline KT sort_key(uint32_t L, uint32_t R, const StepGeom& g)
{
    if (g.hashed) return (KT)((make_key<uint64_t>(L, R, g.i_lo) * 0x9E3779B97F4A7C15ull) >> 40);
    return make_key<KT>(L, R, g.i_lo);
}

__device__ inline uint32_t top_mask(int nbytes)
{
    return nbytes <= 0 ? 0u : (nbytes >= 4 ? 0xFFFFFFFFu : (0xFFFFFFFFu << (32 - 8 * nbytes)));
}

struct SegPtr {
    const uint32_t* Lw;
    const uint32_t* Rw;
};

__device__ inline SegPtr seg_words(const uint32_t* H, const StepGeom& g, int seg)
{
    const int jb = seg / g.Ds, f = seg - jb * g.Ds;
    const int j = g.j0 + jb, l = j / g.m, r = j - l * g.m;
    SegPtr p;
    p.Lw = H + ((int64_t)f * g.NF + l) * g.ns;
    p.Rw = H + ((int64_t)f * g.NF + g.NL + r) * g.ns;
    return p;
}

__global__ void k_zero64(unsigned long long* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ radix sort
template <typename KT, bool FIRST>
__global__ __launch_bounds__(256) void k_hist(const KT* __restrict__ kin, const uint32_t* __restrict__ H,
                                              StepGeom g, int pass, int64_t tiles,
                                              uint32_t* __restrict__ hist)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int seg = blockIdx.y;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kSortTile;
    const int64_t end = base + kSortTile < g.ns ? base + kSortTile : g.ns;
    SegPtr sp;
    if (FIRST) sp = seg_words(H, g, seg);
    const KT* ks = kin + (int64_t)seg * g.ns;
    // every load of the tile first, then the keys, then the counts: a loop
    // that counted each element as it arrived would wait out one memory
    // latency per element
    constexpr int ITEMS = kSortTile / 256;
    uint32_t dg[ITEMS];
    if constexpr (FIRST) {
        uint32_t lv[ITEMS], rv[ITEMS];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int64_t e = base + q * 256 + threadIdx.x;
            lv[q] = e < end ? sp.Lw[e] : 0u;
            rv[q] = e < end ? sp.Rw[e] : 0u;
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) dg[q] = (uint32_t)(sort_key<KT>(lv[q], rv[q], g) >> (8 * pass)) & 255u;
    } else {
        KT kv[ITEMS];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int64_t e = base + q * 256 + threadIdx.x;
            kv[q] = e < end ? ks[e] : (KT)0;
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) dg[q] = (uint32_t)(kv[q] >> (8 * pass)) & 255u;
    }
#pragma unroll
    for (int q = 0; q < ITEMS; ++q)
        if (base + q * 256 + threadIdx.x < end) atomicAdd(&cnt[dg[q]], 1u);
    __syncthreads();
    hist[((int64_t)seg * tiles + tile) * 256 + threadIdx.x] = cnt[threadIdx.x];
}

// Scatter offsets of one segment from its tile-major histogram [tile][digit]:
// offset(t, dg) = (elements of digits < dg) + (elements of digit dg in tiles
// < t), written in place. Four groups of 256 threads (one per digit) take a
// quarter of the tiles each; every row of 256 counts is one coalesced access.
__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ hist, int64_t tiles)
{
    __shared__ uint32_t part[4][256];
    __shared__ uint32_t sh[16];
    uint32_t* h = hist + (int64_t)blockIdx.x * tiles * 256;
    const int grp = threadIdx.x >> 8, dg = threadIdx.x & 255;
    const int64_t per = (tiles + 3) / 4;
    const int64_t t0 = grp * per, t1 = t0 + per < tiles ? t0 + per : tiles;
    // eight rows in flight per thread in both passes over the tiles
    uint32_t s = 0;
    int64_t t = t0;
    for (; t + 8 <= t1; t += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = h[(t + u) * 256 + dg];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; t < t1; ++t) s += h[t * 256 + dg];
    part[grp][dg] = s;
    __syncthreads();
    // per digit: total over the tiles, and the count before this group's tiles
    uint32_t before = 0, total = 0;
    for (int q = 0; q < 4; ++q) {
        const uint32_t v = part[q][dg];
        before += q < grp ? v : 0u;
        total += v;
    }
    // digit bases: exclusive scan of the totals over the 256 digits (group 0)
    uint32_t base = 0;
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(grp == 0 ? total : 0u, sh, &tot);
        __syncthreads();
        if (grp == 0) part[0][dg] = ex;
        __syncthreads();
        base = part[0][dg];
    }
    uint32_t run = base + before;
    for (t = t0; t + 8 <= t1; t += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = h[(t + u) * 256 + dg];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            h[(t + u) * 256 + dg] = run;
            run += v[u];
        }
    }
    for (; t < t1; ++t) {
        const uint32_t v = h[t * 256 + dg];
        h[t * 256 + dg] = run;
        run += v;
    }
}

// Work-groups are dealt to the 8 XCDs round-robin by linear id, so adjacent
// tiles, which write adjacent pieces of every digit's output range, would sit
// in different L2 caches. This bijection of the (segment, tile) grid gives
// each XCD one contiguous range of tiles instead.
__device__ inline void xcd_tile(int64_t tiles, int& seg, int64_t& tile)
{
    const int64_t total = tiles * gridDim.y;
    const int64_t lin = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    const int64_t q = total / 8, r = total % 8, k = lin % 8;
    const int64_t m = k * q + (k < r ? k : r) + lin / 8;
    seg = (int)(m / tiles);
    tile = m - (int64_t)seg * tiles;
}

template <typename KT, bool FIRST>
__global__ __launch_bounds__(256) void k_scatter(const KT* __restrict__ kin, const uint32_t* __restrict__ iin,
                                                 const uint32_t* __restrict__ H, StepGeom g, int pass,
                                                 int64_t tiles, const uint32_t* __restrict__ hist,
                                                 KT* __restrict__ kout, uint32_t* __restrict__ iout)
{
    constexpr int ITEMS = kSortTile / 256;   // 16 per thread
    __shared__ KT skey[kSortTile];
    __shared__ uint32_t sidx[kSortTile];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t dbase[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t scan_sh[4];

    int seg;
    int64_t tile;
    xcd_tile(tiles, seg, tile);
    const int64_t base = tile * kSortTile;
    const int count = (int)((g.ns - base) < kSortTile ? (g.ns - base) : kSortTile);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = threadIdx.x; q < 4 * 256; q += 256) (&wcnt[0][0])[q] = 0;
    gofs[threadIdx.x] = hist[((int64_t)seg * tiles + tile) * 256 + threadIdx.x];
    __syncthreads();

    SegPtr sp;
    if (FIRST) sp = seg_words(H, g, seg);
    const KT* ks = kin + (int64_t)seg * g.ns;
    const uint32_t* is = iin + (int64_t)seg * g.ns;
    KT k_[ITEMS];
    uint32_t i_[ITEMS], r_[ITEMS];
    // wave-contiguous blocks of the tile keep the order; every load is issued
    // before the first ranking step waits on one
    if constexpr (FIRST) {
        uint32_t lv[ITEMS], rv[ITEMS];
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) {
            const int e = wave * (kSortTile / 4) + s * 64 + lane;
            lv[s] = e < count ? sp.Lw[base + e] : 0u;
            rv[s] = e < count ? sp.Rw[base + e] : 0u;
        }
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) {
            const int e = wave * (kSortTile / 4) + s * 64 + lane;
            k_[s] = e < count ? sort_key<KT>(lv[s], rv[s], g) : (KT)0;
            i_[s] = e < count ? (uint32_t)(base + e) : 0u;
        }
    } else {
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) {
            const int e = wave * (kSortTile / 4) + s * 64 + lane;
            k_[s] = e < count ? ks[base + e] : (KT)0;
            i_[s] = e < count ? is[base + e] : 0u;
        }
    }
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const int e = wave * (kSortTile / 4) + s * 64 + lane;
        const bool valid = e < count;
        const KT key = k_[s];
        const uint32_t dg = (uint32_t)(key >> (8 * pass)) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = mbcnt64(peers);
        uint32_t before = 0;
        if (valid) before = wcnt[wave][dg];
        if (valid && rank == 0) wcnt[wave][dg] = before + (uint32_t)__popcll(peers);
        r_[s] = before + rank;
    }
    __syncthreads();
    {
        const int dgt = threadIdx.x;
        uint32_t c0 = wcnt[0][dgt], c1 = wcnt[1][dgt], c2 = wcnt[2][dgt], c3 = wcnt[3][dgt];
        uint32_t tot_all;
        uint32_t db = block_excl_scan<256>(c0 + c1 + c2 + c3, scan_sh, &tot_all);
        dbase[dgt] = db;
        wcnt[0][dgt] = 0;
        wcnt[1][dgt] = c0;
        wcnt[2][dgt] = c0 + c1;
        wcnt[3][dgt] = c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const int e = wave * (kSortTile / 4) + s * 64 + lane;
        if (e < count) {
            const uint32_t dg = (uint32_t)(k_[s] >> (8 * pass)) & 255u;
            const uint32_t pos = dbase[dg] + wcnt[wave][dg] + r_[s];
            skey[pos] = k_[s];
            sidx[pos] = i_[s];
        }
    }
    __syncthreads();
    KT* ko = kout + (int64_t)seg * g.ns;
    uint32_t* io = iout + (int64_t)seg * g.ns;
    for (int q = threadIdx.x; q < count; q += 256) {
        const KT key = skey[q];
        const uint32_t dg = (uint32_t)(key >> (8 * pass)) & 255u;
        const uint32_t dst = gofs[dg] + ((uint32_t)q - dbase[dg]);
        ko[dst] = key;
        io[dst] = sidx[q];
    }
}

// One LSD pass of the segmented sort, as three launches (histogram, scan,
// scatter); `cur` names the buffer holding the input keys of this pass.
hipError_t launch_hist(const StepGeom& g, const uint32_t* H, const SortBufs& b, int pass, int cur,
                       hipStream_t s)
{
    dim3 grid((unsigned)b.tiles, (unsigned)g.nseg);
    if (sort_keys_32(g)) {
        const uint32_t* kin = (const uint32_t*)b.keys[cur];
        if (pass == 0)
            hipLaunchKernelGGL((k_hist<uint32_t, true>), grid, dim3(256), 0, s, kin, H, g, pass, b.tiles, b.hist);
        else
            hipLaunchKernelGGL((k_hist<uint32_t, false>), grid, dim3(256), 0, s, kin, H, g, pass, b.tiles, b.hist);
    } else {
        const uint64_t* kin = (const uint64_t*)b.keys[cur];
        if (pass == 0)
            hipLaunchKernelGGL((k_hist<uint64_t, true>), grid, dim3(256), 0, s, kin, H, g, pass, b.tiles, b.hist);
        else
            hipLaunchKernelGGL((k_hist<uint64_t, false>), grid, dim3(256), 0, s, kin, H, g, pass, b.tiles, b.hist);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const StepGeom& g, const SortBufs& b, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3((unsigned)g.nseg), dim3(1024), 0, s, b.hist, b.tiles);
    return hipGetLastError();
}

hipError_t launch_scatter(const StepGeom& g, const uint32_t* H, const SortBufs& b, int pass, int cur,
                          hipStream_t s)
{
    dim3 grid((unsigned)b.tiles, (unsigned)g.nseg);
    if (sort_keys_32(g)) {
        const uint32_t* kin = (const uint32_t*)b.keys[cur];
        uint32_t* kout = (uint32_t*)b.keys[cur ^ 1];
        if (pass == 0)
            hipLaunchKernelGGL((k_scatter<uint32_t, true>), grid, dim3(256), 0, s, kin, b.idx[cur], H, g,
                               pass, b.tiles, b.hist, kout, b.idx[cur ^ 1]);
        else
            hipLaunchKernelGGL((k_scatter<uint32_t, false>), grid, dim3(256), 0, s, kin, b.idx[cur], H, g,
                               pass, b.tiles, b.hist, kout, b.idx[cur ^ 1]);
    } else {
        const uint64_t* kin = (const uint64_t*)b.keys[cur];
        uint64_t* kout = (uint64_t*)b.keys[cur ^ 1];
        if (pass == 0)
            hipLaunchKernelGGL((k_scatter<uint64_t, true>), grid, dim3(256), 0, s, kin, b.idx[cur], H, g,
                               pass, b.tiles, b.hist, kout, b.idx[cur ^ 1]);
        else
            hipLaunchKernelGGL((k_scatter<uint64_t, false>), grid, dim3(256), 0, s, kin, b.idx[cur], H, g,
                               pass, b.tiles, b.hist, kout, b.idx[cur ^ 1]);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ enumeration
// Fingerprint rows of a batch: for every repetition of the batch and every
// window, an 8-bit digest of each dimension's length-i_lo prefix (equal
// prefixes give equal digests), bit-sliced into 8 planes ([jb][a][fp_words]);
// and a second-stage row of 16-bit digests in 16 planes ([jb][a][fq_words]).
// The pairs of a run are screened with the first rows for >= d equal
// digests (OR of the XORed plane words, then a popcount); those that pass
// are screened again with the second rows, and the few left have their
// per-dimension prefixes rebuilt from the index and counted exactly.
__device__ inline uint32_t prefix_digest8(uint64_t prefix, int i_lo)
{
    // one symbol is its own digest; longer prefixes are mixed by a
    // multiplicative (Fibonacci) hash and the top byte kept
    return i_lo == 1 ? (uint32_t)(prefix & 0xFFu) : (uint32_t)((prefix * 0x9E3779B97F4A7C15ull) >> 56);
}
__device__ inline uint32_t prefix_digest16(uint64_t prefix, int i_lo)
{
    return i_lo <= 2 ? (uint32_t)(prefix & 0xFFFFu) : (uint32_t)((prefix * 0x9E3779B97F4A7C15ull) >> 48);
}

// Transpose of an 8 x 8 bit matrix held as 64 bits, row r in byte r and
// column c in bit c of it: afterwards byte c, bit r holds the old byte r,
// bit c (three rounds of masked delta swaps, Hacker's Delight section 7-3).
__host__ __device__ inline uint64_t transpose8(uint64_t x)
{
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    return x;
}

// Plane k (k < 8) of a chunk from its groups of 8 dimensions, transposed:
// group g's byte k holds plane k's bits for dimensions 8 g .. 8 g + 7.
__host__ __device__ inline uint32_t plane_of(const uint64_t (&t)[4], int k)
{
    return (uint32_t)((t[0] >> (8 * k)) & 0xFFu) | (uint32_t)((t[1] >> (8 * k)) & 0xFFu) << 8 |
           (uint32_t)((t[2] >> (8 * k)) & 0xFFu) << 16 | (uint32_t)((t[3] >> (8 * k)) & 0xFFu) << 24;
}

// Words of 8 planes (planes 8 h .. 8 h + 7 of a row) with DP-bit planes.
template <int DP>
__host__ __device__ inline void plane_words(const uint64_t (&t)[4], uint32_t* out)
{
    constexpr int G = 32 / DP;   // planes per word
#pragma unroll
    for (int q = 0; q < 8 / G; ++q) out[q] = 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k / G] |= plane_of(t, k) << ((k % G) * DP);
}

// Number of dimensions whose digests differ, from the OR of XORed words of
// DP-bit planes (32 / DP planes to the word folded onto the low DP bits).
template <int DP>
__host__ __device__ inline int fold_count(uint32_t o)
{
    if (DP <= 16) o |= o >> 16;
    if (DP <= 8) o |= o >> 8;
    if (DP <= 4) o |= o >> 4;
    return __builtin_popcount(DP == 32 ? o : (o & ((1u << DP) - 1u)));
}

// A chunk's first-stage words (DP / 4) and second-stage words (max(4, DP / 2):
// planes 0..7 from the low digest bytes, 8..15 from the high ones) from its
// transposed groups.
template <int DP>
__host__ __device__ inline void chunk_words(const uint64_t (&t8)[4], const uint64_t (&tl)[4], const uint64_t (&th)[4],
                                            uint32_t* o8, uint32_t* oq)
{
    plane_words<DP>(t8, o8);
    plane_words<DP>(tl, oq);
    if (DP == 4) {
        plane_words<DP>(th, oq + 1);
        oq[2] = oq[3] = 0u;
    } else {
        plane_words<DP>(th, oq + DP / 4);
    }
}

template <int DP>
__global__ __launch_bounds__(256) void k_fptable(const uint32_t* __restrict__ H, StepGeom g, int reps,
                                                 int64_t tiles, uint32_t* __restrict__ fps,
                                                 uint32_t* __restrict__ fq, uint32_t* __restrict__ hist)
{
    // work-group m = (sort tile) * reps + repetition, with each XCD taking
    // one contiguous range of m: the batch's repetitions of a tile run back
    // to back on one XCD, and the left half-function words they share (one
    // left function serves g.m consecutive repetitions) come from its L2.
    // A work-group walks its sort tile 256 windows at a time, one window per
    // thread, and also counts the tile's sort digits of pass 0 for every
    // segment dimension (f < Ds): the histogram the radix sort's first pass
    // would otherwise read the index words again for.
    __shared__ uint32_t cnt[32][256];
    const int64_t nb = (int64_t)gridDim.x;
    const int64_t q = nb / 8, rr = nb % 8, x = blockIdx.x % 8;
    const int64_t m = x * q + (x < rr ? x : rr) + blockIdx.x / 8;
    const int jb = (int)(m % reps);
    const int64_t tile = m / reps;
    const int64_t t0 = tile * kSortTile;
    const int j = g.j0 + jb, l = j / g.m, r = j - l * g.m;
    const int nw = fp_words(g.D), nq = fq_words(g.D);
    constexpr int CD = DP < 32 ? DP : 32;   // dimensions per chunk
    const int64_t lstep = (int64_t)g.NF * g.ns;
    // chunks of 32 dimensions (one chunk unless D > 32), each as four groups
    // of 8 whose digests are gathered byte by byte and then transposed. Every
    // index word of a chunk is loaded before the first is used (a dimension
    // past D reloads the last one and is masked out), so a thread waits out
    // one memory latency per chunk, not one per dimension.
    for (int c0 = 0; c0 < g.D; c0 += 32) {
        const int nh = g.Ds - c0 < CD ? (g.Ds - c0 > 0 ? g.Ds - c0 : 0) : CD;   // segment dimensions here
        for (int v = threadIdx.x; v < nh * 256; v += 256) (&cnt[0][0])[v] = 0;
        __syncthreads();
        for (int64_t a = t0 + threadIdx.x; a < t0 + kSortTile && a < g.ns; a += 256) {
            const int64_t gid = (int64_t)jb * g.ns + a;
            const uint32_t* Lb = H + (int64_t)l * g.ns + a;
            const uint32_t* Rb = H + (int64_t)(g.NL + r) * g.ns + a;
            uint32_t Lw[CD], Rw[CD];
#pragma unroll
            for (int u = 0; u < CD; ++u) {
                const int f = c0 + u < g.D ? c0 + u : g.D - 1;
                Lw[u] = Lb[f * lstep];
                Rw[u] = __builtin_nontemporal_load(Rb + f * lstep);
            }
            uint64_t t8[4], tl[4], th[4];
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                uint64_t b8 = 0, bl = 0, bh = 0;
                if (8 * gq < CD) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int uu = 8 * gq + u;
                        const uint64_t pre = make_key<uint64_t>(Lw[uu], Rw[uu], g.i_lo);
                        const uint32_t d16 = prefix_digest16(pre, g.i_lo);
                        const uint64_t keep = c0 + uu < g.D ? 0xFFull : 0ull;
                        b8 |= ((uint64_t)prefix_digest8(pre, g.i_lo) & keep) << (8 * u);
                        bl |= ((uint64_t)(d16 & 0xFFu) & keep) << (8 * u);
                        bh |= ((uint64_t)(d16 >> 8) & keep) << (8 * u);
                        // pass 0's digit: the low byte of the sort key
                        if (uu < nh) {
                            const uint32_t dg = g.hashed ? (uint32_t)((pre * 0x9E3779B97F4A7C15ull) >> 40) & 255u
                                                         : (uint32_t)pre & 255u;
                            atomicAdd(&cnt[uu][dg], 1u);
                        }
                    }
                }
                t8[gq] = transpose8(b8);
                tl[gq] = transpose8(bl);
                th[gq] = transpose8(bh);
            }
            // the chunk's words leave in whole 16-byte stores where rows allow
            constexpr int W8 = DP / 4, WQ = DP / 2 < 4 ? 4 : DP / 2;
            uint32_t o8[W8], oq[WQ];
            chunk_words<DP>(t8, tl, th, o8, oq);
            uint32_t* f8 = fps + gid * nw + (c0 / 32) * 8;
            if constexpr (W8 == 1)
                f8[0] = o8[0];
            else if constexpr (W8 == 2)
                *reinterpret_cast<uint2*>(f8) = make_uint2(o8[0], o8[1]);
            else {
#pragma unroll
                for (int v = 0; v < W8 / 4; ++v)
                    reinterpret_cast<uint4*>(f8)[v] = make_uint4(o8[4 * v], o8[4 * v + 1], o8[4 * v + 2], o8[4 * v + 3]);
            }
            if (g.fq) {
                uint4* q4 = reinterpret_cast<uint4*>(fq + gid * nq + (c0 / 32) * 16);
#pragma unroll
                for (int v = 0; v < WQ / 4; ++v) q4[v] = make_uint4(oq[4 * v], oq[4 * v + 1], oq[4 * v + 2], oq[4 * v + 3]);
            }
        }
        __syncthreads();
        // the tile's pass-0 counts of the chunk's segment dimensions: segment
        // jb * Ds + f, layout [segment][tile][digit]
        for (int u = 0; u < nh; ++u)
            hist[(((int64_t)jb * g.Ds + c0 + u) * tiles + tile) * 256 + threadIdx.x] = cnt[u][threadIdx.x];
        __syncthreads();
    }
}

hipError_t launch_fptable(const uint32_t* H, const StepGeom& g, int reps, uint32_t* fps, uint32_t* fq,
                          const SortBufs& b, hipStream_t s)
{
    const int64_t tiles = (g.ns + kSortTile - 1) / kSortTile;
    if (tiles != b.tiles) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(tiles * reps));   // (sort tile, repetition) pairs
    switch (plane_bits(g.D)) {
    case 4: hipLaunchKernelGGL(k_fptable<4>, grid, dim3(256), 0, s, H, g, reps, tiles, fps, fq, b.hist); break;
    case 8: hipLaunchKernelGGL(k_fptable<8>, grid, dim3(256), 0, s, H, g, reps, tiles, fps, fq, b.hist); break;
    case 16: hipLaunchKernelGGL(k_fptable<16>, grid, dim3(256), 0, s, H, g, reps, tiles, fps, fq, b.hist); break;
    default: hipLaunchKernelGGL(k_fptable<32>, grid, dim3(256), 0, s, H, g, reps, tiles, fps, fq, b.hist); break;
    }
    return hipGetLastError();
}

// Second stage: do the 16-bit digests of windows a and b agree in >= d
// dimensions? (Rows of 16 planes; with D > 32, one popcount per chunk.)
__host__ __device__ inline bool second_stage(const uint32_t* __restrict__ fq, int nq, int D, int d, uint32_t a,
                                             uint32_t b)
{
    const uint4* ra = reinterpret_cast<const uint4*>(fq + (int64_t)a * nq);
    const uint4* rb = reinterpret_cast<const uint4*>(fq + (int64_t)b * nq);
    int z = 0;
    if (D <= 32) {
        uint32_t o = 0;
        for (int c = 0; c < nq / 4; ++c) {
            const uint4 x = ra[c], y = rb[c];
            o |= (x.x ^ y.x) | (x.y ^ y.y) | (x.z ^ y.z) | (x.w ^ y.w);
        }
        const int dp = plane_bits(D);
        z = dp == 4 ? fold_count<4>(o) : dp == 8 ? fold_count<8>(o) : dp == 16 ? fold_count<16>(o) : fold_count<32>(o);
    } else {
        for (int c = 0; c < nq / 4; c += 4) {   // a chunk: 16 words
            uint32_t o = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint4 x = ra[c + v], y = rb[c + v];
                o |= (x.x ^ y.x) | (x.y ^ y.y) | (x.z ^ y.z) | (x.w ^ y.w);
            }
            z += __builtin_popcount(o);
        }
    }
    return z <= D - d;   // digests differ in at most D - d dimensions
}

constexpr int kFpRegs = 8;   // fingerprint words kept in registers (32 dimensions)

// NW consecutive words of a fingerprint row (at a multiple of NW words from
// an aligned base) in as few vector loads as possible; zeros when !take.
template <int NW>
__device__ inline void load_row(uint32_t (&o)[NW], const uint32_t* src, bool take)
{
    if constexpr (NW % 4 == 0) {
#pragma unroll
        for (int q = 0; q < NW / 4; ++q) {
            const uint4 v = take ? reinterpret_cast<const uint4*>(src)[q] : make_uint4(0u, 0u, 0u, 0u);
            o[4 * q] = v.x; o[4 * q + 1] = v.y; o[4 * q + 2] = v.z; o[4 * q + 3] = v.w;
        }
    } else if constexpr (NW == 2) {
        const uint2 v = take ? *reinterpret_cast<const uint2*>(src) : make_uint2(0u, 0u);
        o[0] = v.x; o[1] = v.y;
    } else {
#pragma unroll
        for (int wd = 0; wd < NW; ++wd) o[wd] = take ? src[wd] : 0u;
    }
}

// Words between consecutive fingerprint rows in LDS: nw rounded up to odd.
__host__ __device__ inline int lds_row_words(int nw) { return nw | 1; }
// LDS words per member of a tile: tile P (stored twice unless the rows are
// wider than the registers: then its circulant partners wrap explicitly),
// tile Q, and the two index arrays.
__host__ __device__ inline int tile_member_words(int nw)
{
    return (nw > kFpRegs ? 2 : 3) * lds_row_words(nw) + 2;
}

// Dimensions whose first-stage digests differ between the lane's own row
// (its first NW words in registers, the rest at own_tail, only when TAIL)
// and the partner's (pw). NW < 8 means D <= 16 and planes of 4 NW bits;
// NW = 8 is one 32-dimension chunk, and TAIL rows add a chunk per 8 words.
template <int NW, bool TAIL, typename GetW>
__host__ __device__ inline int screen(const uint32_t (&ofp)[NW], const uint32_t* own_tail, const GetW& pw, int nw)
{
    uint32_t o = 0;
#pragma unroll
    for (int wd = 0; wd < NW; ++wd) o |= ofp[wd] ^ pw(wd);
    int z = fold_count<4 * NW>(o);
    if (TAIL)
        for (int c = NW; c < nw; c += 8) {
            uint32_t t = 0;
#pragma unroll
            for (int wd = 0; wd < 8; ++wd) t |= own_tail[c + wd] ^ pw(c + wd);
            z += __builtin_popcount(t);
        }
    return z;
}

// Number of leading symbols two kt-symbol prefixes share.
__device__ inline int common_symbols(uint64_t x, uint64_t y, int kt)
{
    const uint64_t v = x ^ y;
    if (v == 0) return kt;
    return (__clzll((long long)v) - (64 - 8 * kt)) >> 3;
}

// Exact test of a pair (a < b) that passed the screen, in repetition j of a
// segment of dimension f. cp(f') = symbols shared by the two length-kt
// prefixes in dimension f' (kt = min(i_hi + 1, K)), so the pair collides at
// round i in f' iff cp(f') >= i. It is a candidate of step (i, j), for each
// round i of the group at which it collides in f, iff W_i = #{f' : cp >= i}
// >= d, no f' < f has cp >= i (it is reported once, from its lowest colliding
// dimension) and, below round K, W_{i+1} < d (section 6.2: pairs seen one
// symbol deeper are skipped).
constexpr int kMaxLev = 8;   // rounds of a group + 1 (a group spans at most 7 rounds)

__device__ inline void judge_pair(uint32_t a, uint32_t b, const uint32_t* __restrict__ H, const StepGeom& g,
                                  int f, int j, int kt, int d, Cand* __restrict__ cand, uint32_t cap,
                                  Counters* __restrict__ cnt)
{
    if (g.nparts > 1 && pair_part(a, b, g.nparts) != (uint32_t)g.part) return;   // another part's pair
    const int l = j / g.m, r = j - l * g.m;
    const int nlev = g.i - g.i_lo + 2;
    // per level lv (round i_lo + lv), byte lv counts the dimensions colliding
    // there (atl) and those among them below f (blw); D <= 128 fits a byte
    uint64_t atl = 0, blw = 0;
    int cpf = 0;
    for (int fp = 0; fp < g.D; ++fp) {
        const uint32_t* Hl = H + ((int64_t)fp * g.NF + l) * g.ns;
        const uint32_t* Hr = H + ((int64_t)fp * g.NF + g.NL + r) * g.ns;
        const int cp = common_symbols(make_key<uint64_t>(Hl[a], Hr[a], kt), make_key<uint64_t>(Hl[b], Hr[b], kt), kt);
        int nl = cp - g.i_lo + 1;   // levels 0 .. nl - 1 collide
        nl = nl < 0 ? 0 : (nl > nlev ? nlev : nl);
        const uint64_t ones = nl ? 0x0101010101010101ull & (~0ull >> (64 - 8 * nl)) : 0ull;
        atl += ones;
        if (fp < f) blw += ones;
        if (fp == f) cpf = cp;
    }
    if ((int)(atl & 0xFF) < d) return;   // the digests agreed by chance
    if (cpf < g.i_lo) return;            // equal sort-key hashes, different prefixes
    const int top = cpf < g.i ? cpf : g.i;
    for (int lv = nlev - 2; lv >= 0; --lv) {
        const int i = g.i_lo + lv;
        if (i > top) continue;   // rounds i_lo .. min(top, i_hi)
        const int Wi = (int)((atl >> (8 * lv)) & 0xFF);
        if (Wi < d || ((blw >> (8 * lv)) & 0xFF) != 0) continue;
        // below round K: skip a pair every dimensionality of (d .. dhi] it counts
        // for had already at prefix i + 1 (section 6.2)
        if (i < g.K && (int)((atl >> (8 * (lv + 1))) & 0xFF) >= (Wi < g.dhi ? Wi : g.dhi)) continue;
        const uint32_t pos = atomicAdd(&cnt->n_cand, 1u);
        if (pos < cap) cand[pos] = Cand{a, b, (uint32_t)j, (uint32_t)i | ((uint32_t)Wi << 8)};
    }
}

// Queue a wavefront's pending long runs (seg, start, len) as tile rows: one
// atomic reserves the rows of all of them, lane i writes run i's rows.
__device__ inline void flush_runs(const uint32_t (*pend)[3], int npend, int TS, int lane,
                                  Counters* __restrict__ cnt, RunRec* __restrict__ units, uint32_t ucap)
{
    wave_sync_lds();
    uint32_t seg = 0, start = 0, len = 0, T = 0;
    if (lane < npend) {
        seg = pend[lane][0];
        start = pend[lane][1];
        len = pend[lane][2];
        T = (len + (uint32_t)TS - 1) / (uint32_t)TS;
    }
    // inclusive prefix sum of T over the lanes
    uint32_t incl = T;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += v;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&cnt->n_units, total);
    base = (uint32_t)__shfl((int)base, 0, 64);
    const uint32_t first = base + incl - T;
    for (uint32_t tp = 0; tp < T; ++tp)
        if ((uint64_t)first + tp < ucap) units[first + tp] = RunRec{seg, start, len, tp};
    wave_sync_lds();
}

// Window scan: run detection and the runs that fit a window. Segments are
// sorted by their length-i_lo prefix (the group's lowest round), so every
// deeper round's runs lie inside its runs. Each wavefront owns 64 consecutive
// elements of one segment (four such windows at a time): ballots mark the
// heads of runs of length >= 2 that start there and the tails where runs end.
//  * Runs that close inside the window are enumerated all at once, lane by
//    lane: the member at position q of a run of n pairs with the members at
//    q + s (mod n), 1 <= s <= (n - 1) / 2, plus, for even n and q < n / 2, the
//    one at q + n / 2, which covers each unordered pair once; fingerprint
//    words reach the partner by cross-lane permutes.
//  * The one run that leaves the window has its end found 64 keys at a time
//    and is queued, as one unit per tile of TS members, for k_enum_tiles.
// Pairs that pass the screen and are not trivial matches go to judge_pair.
template <typename KT, int NW, bool TAIL>
__global__ __launch_bounds__(256, 4) void k_enum_runs(const KT* __restrict__ keys,
                                                   const uint32_t* __restrict__ idx,
                                                   const uint32_t* __restrict__ H,
                                                   const uint32_t* __restrict__ fps,
                                                   const uint32_t* __restrict__ fqs, StepGeom g, int kt,
                                                   int d, int w, int TS, Cand* __restrict__ cand,
                                                   uint32_t cap, Counters* __restrict__ cnt,
                                                   unsigned long long* __restrict__ coll_part,
                                                   RunRec* __restrict__ units, uint32_t ucap)
{
    __shared__ unsigned long long coll_sh[4], memb_sh[4], scr_sh[4];
    __shared__ uint32_t pend[4][64][3];   // per wavefront: long runs waiting to be queued
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = TAIL ? fp_words(g.D) : NW;   // NW = min(nw, kFpRegs); TAIL iff nw > NW
    const int nq = fq_words(g.D);
    const int zmax = g.D - d;   // digests may differ in at most D - d dimensions
    int npend = 0;   // uniform across the wavefront
    unsigned long long ncoll = 0, nmemb = 0, nscr = 0;
    uint32_t maxrun = 0;
    const int64_t wins_per_seg = (g.ns + 63) / 64;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const uint64_t lane_bit = 1ull << lane;
    const uint64_t le_mask = lane_bit | (lane_bit - 1);   // lanes <= this one
    const uint64_t ge_mask = ~(lane_bit - 1);             // lanes >= this one
    // persistent: each wavefront strides over groups of four consecutive
    // 64-element windows of all segments; the four windows' keys (and the
    // two keys beyond each window's edges) are loaded together, neighbours
    // inside a window come by lane shuffles
    const int64_t quads_per_seg = (wins_per_seg + 3) / 4;
    const int64_t total_quads = quads_per_seg * g.nseg;
    for (int64_t qd = (int64_t)blockIdx.x * 4 + wave; qd < total_quads; qd += nwaves) {
        const int seg = (int)(qd / quads_per_seg);
        const int64_t qstart = (qd - (int64_t)seg * quads_per_seg) * 256;
        const int jb = seg / g.Ds, f = seg - jb * g.Ds;
        const int j = g.j0 + jb;
        const KT* ks = keys + (int64_t)seg * g.ns;
        const uint32_t* is = idx + (int64_t)seg * g.ns;
        const uint32_t* fbase = fps + (int64_t)jb * g.ns * nw;
        const uint32_t* qbase = fqs + (int64_t)jb * g.ns * nq;
        // bit 2r: the lane's key in window r equals the one before it, bit
        // 2r + 1: the one after it; xr: the window indices of run members
        uint32_t sflags = 0;
        uint32_t xr[4];
        {
            // fast skip: most groups of windows hold no run at the lowest round
            // of the first round group
            KT kq[4], kedge[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t t = qstart + 64 * r + lane;
                // keys and indices stream through once: non-temporal loads leave
                // the caches to the fingerprint rows gathered below
                kq[r] = t < g.ns ? __builtin_nontemporal_load(ks + t) : (KT)0;
                // lane 0 holds the key before the window, lane 63 the one after it
                const int64_t te = lane == 0 ? t - 1 : t + 1;
                kedge[r] = ((lane == 0 || lane == 63) && te >= 0 && te < g.ns) ? ks[te] : (KT)0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t t = qstart + 64 * r + lane;
                // every lane takes part in both shuffles (a lane left out of one
                // would hand its neighbour 0 instead of its key), then selects
                const KT up = (KT)__shfl_up(kq[r], 1, 64);
                const KT dn = (KT)__shfl_down(kq[r], 1, 64);
                const KT kp = lane == 0 ? kedge[r] : up;
                const KT kn = lane == 63 ? kedge[r] : dn;
                const bool sp = t < g.ns && t > 0 && kp == kq[r];
                const bool sn = t < g.ns && t + 1 < g.ns && kn == kq[r];
                sflags |= ((sp ? 1u : 0u) | (sn ? 2u : 0u)) << (2 * r);
            }
            if (!__ballot(sflags != 0)) continue;
            // the four windows' indices in one round of loads
#pragma unroll
            for (int r = 0; r < 4; ++r)
                xr[r] = ((sflags >> (2 * r)) & 3u) ? __builtin_nontemporal_load(is + qstart + 64 * r + lane) : 0u;
        }
#pragma unroll 1
        for (int r = 0; r < 4; ++r) {
        const int64_t base = qstart + 64 * r;
        if (base >= g.ns) break;
        const int64_t t = base + lane;
        const bool valid = t < g.ns;
        const bool same_prev = ((sflags >> (2 * r)) & 1u) != 0;
        const bool same_next = ((sflags >> (2 * r)) & 2u) != 0;
        const bool head = valid && !same_prev && same_next;
        const uint64_t heads = __ballot(head);
        if (!heads) continue;
        const uint64_t tails = __ballot(valid && !same_next);

        // runs that close inside the window
        const uint64_t hb = heads & le_mask, tb = tails & ge_mask;
        const bool inner = valid && (head || same_prev) && hb && tb;
        const int h = 63 - __clzll((long long)(hb | 1ull));               // the run's head lane
        const int e = __ffsll((unsigned long long)(tb | (1ull << 63)));   // one past its tail lane
        const int L = e - h, q = lane - h;
        const int npart = inner ? (L - 1) / 2 + (((L & 1) == 0 && q < L / 2) ? 1 : 0) : 0;
        const uint64_t inner_bits = __ballot(inner);
        ncoll += (unsigned long long)npart;
        if (lane == 0) nmemb += (unsigned long long)__popcll(inner_bits);
        if (inner_bits) {
            const uint32_t xu = r == 0 ? xr[0] : r == 1 ? xr[1] : r == 2 ? xr[2] : xr[3];
            const uint32_t* ofw = fbase + (int64_t)xu * nw;
            uint32_t ofp[NW];
            load_row<NW>(ofp, ofw, inner);
            for (int s = 1;; ++s) {
                const bool act = s <= npart;
                if (!__ballot(act)) break;
                int qs = q + s;
                if (qs >= L) qs -= L;
                const int pl = act ? h + qs : lane;
                const uint32_t y = __shfl(xu, pl, 64);
                int z = 0;
                if (!TAIL) {
                    // every lane takes part in the permutes; only active lanes use them
                    z = screen<NW, false>(ofp, ofw, [&](int wd) { return (uint32_t)__shfl(ofp[wd], pl, 64); }, nw);
                } else if (act) {
                    const uint32_t* pfw = fbase + (int64_t)y * nw;
                    z = screen<NW, true>(ofp, ofw, [&](int wd) { return pfw[wd]; }, nw);
                }
                if (act && z <= zmax) {
                    const uint32_t a = xu < y ? xu : y, b = xu < y ? y : xu;
                    if (2 * (int64_t)(b - a) > (int64_t)w &&   // else a trivial match
                        (!g.fq || second_stage(qbase, nq, g.D, d, a, b))) {
                        ++nscr;
                        judge_pair(a, b, H, g, f, j, kt, d, cand, cap, cnt);
                    }
                }
            }
        }

        // the one run that leaves the window, if its head is here
        const uint64_t open = __ballot(head && !tb);
        if (!open) continue;
        const int hl = __ffsll((unsigned long long)open) - 1;
        const KT hk = ks[base + hl];
        int64_t pos = base + 64, end = -1;
        while (end < 0) {
            const int64_t ee = pos + lane;
            const bool stop = ee >= g.ns || ks[ee < g.ns ? ee : g.ns - 1] != hk;
            const uint64_t m = __ballot(stop);
            if (m) end = pos + __ffsll((unsigned long long)m) - 1;
            pos += 64;
        }
        const int64_t start = base + hl;
        const int len = (int)(end - start);
        if (lane == 0) {
            nmemb += (unsigned long long)len;
            ncoll += (unsigned long long)len * (len - 1) / 2;
            maxrun = maxrun > (uint32_t)len ? maxrun : (uint32_t)len;
        }
        // queued for k_enum_tiles, 64 runs at a time
        if (lane == 0) {
            pend[wave][npend][0] = (uint32_t)seg;
            pend[wave][npend][1] = (uint32_t)start;
            pend[wave][npend][2] = (uint32_t)len;
        }
        if (++npend == 64) {
            flush_runs(pend[wave], npend, TS, lane, cnt, units, ucap);
            npend = 0;
        }
        }
    }
    if (npend) flush_runs(pend[wave], npend, TS, lane, cnt, units, ucap);
    // pairs, run members and screened pairs: one triple of partial sums per
    // work-group, no atomics
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ncoll += __shfl_xor(ncoll, o, 64);
        nscr += __shfl_xor(nscr, o, 64);
    }
    if (lane == 0) {
        coll_sh[wave] = ncoll;
        memb_sh[wave] = nmemb;
        scr_sh[wave] = nscr;
    }
    if (lane == 0 && maxrun) atomicMax(&cnt->max_run, maxrun);   // one per wavefront
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t b = blockIdx.x;
        coll_part[3 * b] = coll_sh[0] + coll_sh[1] + coll_sh[2] + coll_sh[3];
        coll_part[3 * b + 1] = memb_sh[0] + memb_sh[1] + memb_sh[2] + memb_sh[3];
        coll_part[3 * b + 2] = scr_sh[0] + scr_sh[1] + scr_sh[2] + scr_sh[3];
    }
}

// Long runs, one tile row at a time: unit (segment, run start, run length,
// tp) pairs tile tp of the run with itself (circulant partners) and with
// every later tile of the run. Tiles are staged in the wave's LDS region:
// window indices and fingerprint rows at an odd stride (lanes reading
// consecutive rows hit distinct banks); tile P is stored twice so that the
// circulant partners u + 1 + v of member u need no wrap (once, with an
// explicit wrap, when the rows are wider than the registers). Lane u owns
// members u, u + 64, ... of P and walks their partners in tile Q >= P (all
// lanes read the same partner of Q at once: an LDS broadcast). Wavefronts
// take units in a fixed stride; a run's rows are consecutive units, so long
// runs spread over many wavefronts.
template <int NW, bool TAIL>
__global__ __launch_bounds__(256, 4) void k_enum_tiles(const uint32_t* __restrict__ idx,
                                                    const uint32_t* __restrict__ H,
                                                    const uint32_t* __restrict__ fps,
                                                    const uint32_t* __restrict__ fqs, StepGeom g, int kt,
                                                    int d, int w, int TS, const RunRec* __restrict__ units,
                                                    uint32_t ucap, Cand* __restrict__ cand, uint32_t cap,
                                                    Counters* __restrict__ cnt)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = TAIL ? fp_words(g.D) : NW;   // NW = min(nw, kFpRegs); TAIL iff nw > NW
    const int nq = fq_words(g.D);
    const int zmax = g.D - d;   // digests may differ in at most D - d dimensions
    // LDS rows of fingerprint words at an odd stride, so that lanes reading
    // consecutive rows hit distinct banks
    const int ldw = lds_row_words(nw);
    uint32_t* mine = reinterpret_cast<uint32_t*>(smem_raw) + (size_t)wave * TS * tile_member_words(nw);
    uint32_t* fpA = mine;                                    // tile P (twice unless TAIL)
    uint32_t* fpB = fpA + (size_t)(TAIL ? 1 : 2) * TS * ldw;   // TS rows: tile Q
    uint32_t* idA = fpB + (size_t)TS * ldw;
    uint32_t* idB = idA + TS;

    unsigned long long nscr = 0;
    const uint32_t nunits = min(cnt->n_units, ucap);
    const uint32_t nwaves = gridDim.x * 4;
    for (uint32_t uq = blockIdx.x * 4 + wave; uq < nunits; uq += nwaves) {
        const RunRec un = units[uq];
        const int seg = (int)un.seg, len = (int)un.len, tp = (int)un.tp;
        const int64_t start = un.start;
        const int jb = seg / g.Ds, f = seg - jb * g.Ds;
        const int j = g.j0 + jb;
        const uint32_t* is = idx + (int64_t)seg * g.ns;
        const uint32_t* fbase = fps + (int64_t)jb * g.ns * nw;
        const uint32_t* qbase = fqs + (int64_t)jb * g.ns * nq;
        const int T = (len + TS - 1) / TS;
        {
            const int nA = min(TS, len - tp * TS);
            wave_sync_lds();
            for (int r = lane; r < nA; r += 64) {
                const uint32_t a = is[start + tp * TS + r];
                idA[r] = a;
                for (int w0 = 0; w0 < nw; w0 += NW) {
                    uint32_t v[NW];
                    load_row<NW>(v, fbase + (int64_t)a * nw + w0, true);
#pragma unroll
                    for (int wd = 0; wd < NW; ++wd) {
                        fpA[(size_t)r * ldw + w0 + wd] = v[wd];
                        if (!TAIL) fpA[(size_t)(r + nA) * ldw + w0 + wd] = v[wd];
                    }
                }
            }
            for (int tq = tp; tq < T; ++tq) {
                const bool same = tq == tp;
                const int nB = min(TS, len - tq * TS);
                if (!same) {
                    wave_sync_lds();
                    for (int r = lane; r < nB; r += 64) {
                        const uint32_t b = is[start + tq * TS + r];
                        idB[r] = b;
                        for (int w0 = 0; w0 < nw; w0 += NW) {
                            uint32_t v[NW];
                            load_row<NW>(v, fbase + (int64_t)b * nw + w0, true);
#pragma unroll
                            for (int wd = 0; wd < NW; ++wd) fpB[(size_t)r * ldw + w0 + wd] = v[wd];
                        }
                    }
                }
                wave_sync_lds();
                for (int u = lane; u < nA; u += 64) {
                    const uint32_t* ofw = fpA + (size_t)u * ldw;
                    uint32_t ofp[NW];
#pragma unroll
                    for (int wd = 0; wd < NW; ++wd) ofp[wd] = ofw[wd];
                    // partners: u + 1 + v in P (v < nA / 2, the last one only for
                    // u < nA / 2 when nA is even), or every member v of Q
                    const uint32_t* P0 = same ? fpA + (size_t)(u + 1) * ldw : fpB;
                    const int nv = same ? ((nA & 1) == 0 && u >= nA / 2 ? nA / 2 - 1 : nA / 2) : nB;                    // row of partner v (tile P is stored once when TAIL: wrap)
                    auto prow = [&](int v) -> const uint32_t* {
                        if (!TAIL || !same) return P0 + (size_t)v * ldw;
                        int qq = u + 1 + v;
                        if (qq >= nA) qq -= nA;
                        return fpA + (size_t)qq * ldw;
                    };
                    auto check = [&](int v) {
                        int qq = same ? u + 1 + v : v;
                        if (same && qq >= nA) qq -= nA;
                        const uint32_t xu = idA[u], y = same ? idA[qq] : idB[qq];
                        const uint32_t a = xu < y ? xu : y, b = xu < y ? y : xu;
                        if (2 * (int64_t)(b - a) <= (int64_t)w) return;   // trivial match
                        if (!(!g.fq || second_stage(qbase, nq, g.D, d, a, b))) return;
                        ++nscr;
                        judge_pair(a, b, H, g, f, j, kt, d, cand, cap, cnt);
                    };
                    int v = 0;
                    // UP partners per step, their LDS reads issued together
                    // (two for rows of 8 words and more, to stay within 128 VGPRs)
                    constexpr int UP = NW >= 8 ? 2 : 4;
                    for (; v + UP <= nv; v += UP) {
                        const uint32_t* pr[UP];
#pragma unroll
                        for (int c = 0; c < UP; ++c) pr[c] = prow(v + c);
                        uint32_t pw[UP][NW];
#pragma unroll
                        for (int c = 0; c < UP; ++c)
#pragma unroll
                            for (int wd = 0; wd < NW; ++wd) pw[c][wd] = pr[c][wd];
                        int z[UP];
#pragma unroll
                        for (int c = 0; c < UP; ++c) {
                            uint32_t o = 0;
#pragma unroll
                            for (int wd = 0; wd < NW; ++wd) o |= ofp[wd] ^ pw[c][wd];
                            z[c] = fold_count<4 * NW>(o);
                        }
                        if (TAIL)
                            // the rest of the lane's own row is read once for the UP
                            // partners, a 32-dimension chunk (8 words) at a time
                            for (int c0 = NW; c0 < nw; c0 += 8) {
                                uint32_t t[UP];
#pragma unroll
                                for (int c = 0; c < UP; ++c) t[c] = 0u;
#pragma unroll
                                for (int wd = 0; wd < 8; ++wd) {
                                    const uint32_t o = ofw[c0 + wd];
#pragma unroll
                                    for (int c = 0; c < UP; ++c) t[c] |= o ^ pr[c][c0 + wd];
                                }
#pragma unroll
                                for (int c = 0; c < UP; ++c) z[c] += __popc(t[c]);
                            }
                        // most steps pass no partner: one test of the smallest count first
                        int zmin = z[0];
#pragma unroll
                        for (int c = 1; c < UP; ++c) zmin = min(zmin, z[c]);
                        if (zmin <= zmax) {
                            uint32_t hit = 0;
#pragma unroll
                            for (int c = 0; c < UP; ++c) hit |= (uint32_t)(z[c] <= zmax) << c;
                            while (hit) {
                                const int bit = __ffs(hit) - 1;
                                hit &= hit - 1;
                                check(v + bit);
                            }
                        }
                    }
                    for (; v < nv; ++v) {
                        const uint32_t* p = prow(v);
                        if (screen<NW, TAIL>(ofp, ofw, [&](int wd) { return p[wd]; }, nw) <= zmax) check(v);
                    }
                }
            }
        }
    }
    // screened pairs: one atomic per wavefront
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nscr += __shfl_xor(nscr, o, 64);
    if (lane == 0 && nscr) atomicAdd(&cnt->n_screen, nscr);
}

__global__ __launch_bounds__(1024) void k_sum_partials(const unsigned long long* __restrict__ part,
                                                       int64_t count, Counters* __restrict__ cnt)
{
    __shared__ unsigned long long sh[3][16];
    unsigned long long v[3] = {0, 0, 0};
    for (int64_t q = threadIdx.x; q < count; q += 1024)
        for (int c = 0; c < 3; ++c) v[c] += part[3 * q + c];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
        if ((threadIdx.x & 63) == 0) sh[c][threadIdx.x >> 6] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c)
            for (int q = 0; q < 16; ++q) t[c] += sh[c][q];
        cnt->n_coll += t[0];
        cnt->n_memb += t[1];
        cnt->n_screen += t[2];
    }
}

// Members per tile: a wave's region (tile P twice, tile Q, indices) stays
// within 13 KB, so that three work-groups (52 KB each) fit a CU's LDS; up to
// 128 members for rows of at most 2 words (fewer tile rows per run, each
// lane owning two members of P), 64 otherwise.
static int tile_size(int D)
{
    const int cap = fp_words(D) <= 2 ? 128 : 64;
    int ts = 13312 / (4 * tile_member_words(fp_words(D)));
    ts = ts > cap ? cap : ts;
    return ts < 16 ? 16 : (ts / 16) * 16;
}

constexpr int kEnumBlocks = 2048;   // persistent grid: at most 8 work-groups per CU
int64_t enum_partials(const StepGeom&) { return kEnumBlocks; }

static int resident_blocks_query(const void* fn, size_t lds)
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, lds) != hipSuccess || ncu < 1 || per < 1)
        return kEnumBlocks;
    return std::min(kEnumBlocks, ncu * std::min(per, 8));
}

// Work-groups that are resident at once (so that none waits for a slot):
// CUs times the occupancy of the kernel at this LDS size, capped.
static int resident_blocks(const void* fn, size_t lds)
{
    // cached per (kernel, LDS size); a stale entry only changes the grid size
    struct Entry {
        const void* fn;
        size_t lds;
        int nb;
    };
    static thread_local Entry cache[8] = {};
    static thread_local int next = 0;
    for (const Entry& e : cache)
        if (e.fn == fn && e.lds == lds) return e.nb;
    const int nb = resident_blocks_query(fn, lds);
    cache[next] = Entry{fn, lds, nb};
    next = (next + 1) & 7;
    return nb;
}


// The windows' short runs (queueing the long ones as tile rows), then the
// tile rows, then the sum of the first kernel's partial counts.
template <typename KT, int NW, bool TAIL>
static hipError_t go_enum(const StepGeom& g, const KT* keys, const uint32_t* idx, const uint32_t* H,
                          const uint32_t* fps, const uint32_t* fq, int kt, int d, int w, Cand* cand,
                          uint32_t cap, Counters* cnt, unsigned long long* part, RunRec* units,
                          uint32_t ucap, hipStream_t s)
{
    const int TS = tile_size(g.D);
    const void* fa = (const void*)k_enum_runs<KT, NW, TAIL>;
    const int nba = resident_blocks(fa, 0);
    hipLaunchKernelGGL((k_enum_runs<KT, NW, TAIL>), dim3(nba), dim3(256), 0, s, keys, idx, H, fps, fq, g, kt,
                       d, w, TS, cand, cap, cnt, part, units, ucap);
    const size_t lds = (size_t)4 * TS * tile_member_words(fp_words(g.D)) * 4;   // 4 waves
    const void* fb = (const void*)k_enum_tiles<NW, TAIL>;
    if (lds > 65536) (void)hipFuncSetAttribute(fb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int nbb = resident_blocks(fb, lds);
    hipLaunchKernelGGL((k_enum_tiles<NW, TAIL>), dim3(nbb), dim3(256), lds, s, idx, H, fps, fq, g, kt, d, w, TS,
                       units, ucap, cand, cap, cnt);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, part, (int64_t)nba, cnt);
    return hipGetLastError();
}

template <typename KT>
static hipError_t go_enum_nw(const StepGeom& g, const KT* k, const uint32_t* idx, const uint32_t* H,
                             const uint32_t* fps, const uint32_t* fq, int kt, int d, int w, Cand* cand,
                             uint32_t cap, Counters* cnt, unsigned long long* part, RunRec* u, uint32_t uc,
                             hipStream_t s)
{
    switch (fp_words(g.D)) {
    case 1: return go_enum<KT, 1, false>(g, k, idx, H, fps, fq, kt, d, w, cand, cap, cnt, part, u, uc, s);
    case 2: return go_enum<KT, 2, false>(g, k, idx, H, fps, fq, kt, d, w, cand, cap, cnt, part, u, uc, s);
    case 4: return go_enum<KT, 4, false>(g, k, idx, H, fps, fq, kt, d, w, cand, cap, cnt, part, u, uc, s);
    case 8: return go_enum<KT, 8, false>(g, k, idx, H, fps, fq, kt, d, w, cand, cap, cnt, part, u, uc, s);
    default: return go_enum<KT, kFpRegs, true>(g, k, idx, H, fps, fq, kt, d, w, cand, cap, cnt, part, u, uc, s);
    }
}

hipError_t launch_enum(const StepGeom& g, const SortBufs& b, int buf, const uint32_t* H,
                       const uint32_t* fps, const uint32_t* fq, int kt, int d, int w, Cand* cand,
                       uint32_t cap, Counters* cnt, unsigned long long* part, hipStream_t s)
{
    if (g.i - g.i_lo + 2 > kMaxLev) return hipErrorInvalidValue;
    if (sort_keys_32(g))
        return go_enum_nw<uint32_t>(g, (const uint32_t*)b.keys[buf], b.idx[buf], H, fps, fq, kt, d, w, cand,
                                    cap, cnt, part, b.units, b.ucap, s);
    return go_enum_nw<uint64_t>(g, (const uint64_t*)b.keys[buf], b.idx[buf], H, fps, fq, kt, d, w, cand, cap,
                                cnt, part, b.units, b.ucap, s);
}

// ------------------------------------------------------------------ probe
// Pairs of windows sharing their length-i prefix, for i = 1 .. kk, in
// segments sorted by their length-kk prefix (a shorter prefix's runs are
// unions of consecutive runs of the longer one). A run is followed for at
// most kProbeCap members: the counts are exact below that, lower bounds
// above it. out[i - 1] accumulates the count of level i.
constexpr int64_t kProbeCap = 1 << 16;

template <typename KT>
__global__ __launch_bounds__(256) void k_probe_levels(const KT* __restrict__ keys, int64_t ns, int nseg, int kk,
                                                      unsigned long long* __restrict__ out)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lane_bit = 1ull << lane;
    const uint64_t le_mask = lane_bit | (lane_bit - 1), ge_mask = ~(lane_bit - 1);
    unsigned long long acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t wins_per_seg = (ns + 63) / 64;
    const int64_t total_wins = wins_per_seg * nseg;
    for (int64_t win = (int64_t)blockIdx.x * 4 + wave; win < total_wins; win += (int64_t)gridDim.x * 4) {
        const int seg = (int)(win / wins_per_seg);
        const int64_t base = (win - (int64_t)seg * wins_per_seg) * 64;
        const KT* ks = keys + (int64_t)seg * ns;
        const int64_t t = base + lane;
        const bool valid = t < ns;
        const KT kf = valid ? ks[t] : (KT)0;
        const KT kp = valid && t > 0 ? ks[t - 1] : (KT)0;
        const KT kn = valid && t + 1 < ns ? ks[t + 1] : (KT)0;
#pragma unroll
        for (int lv = 0; lv < 8; ++lv) {
            if (lv >= kk) break;
            const int sh = 8 * (kk - 1 - lv);   // level lv + 1
            const KT k = kf >> sh;
            const bool same_prev = valid && t > 0 && (KT)(kp >> sh) == k;
            const bool same_next = valid && t + 1 < ns && (KT)(kn >> sh) == k;
            const bool head = valid && !same_prev && same_next;
            const uint64_t heads = __ballot(head);
            if (!heads) continue;
            const uint64_t tails = __ballot(valid && !same_next);
            const uint64_t hb = heads & le_mask, tb = tails & ge_mask;
            const bool inner = valid && (head || same_prev) && hb && tb;
            const int h = 63 - __clzll((long long)(hb | 1ull));
            const int e = __ffsll((unsigned long long)(tb | (1ull << 63)));
            const int L = e - h, q = lane - h;
            acc[lv] += inner ? (unsigned long long)((L - 1) / 2 + (((L & 1) == 0 && q < L / 2) ? 1 : 0)) : 0ull;
            const uint64_t open = __ballot(head && !tb);
            if (!open) continue;
            const int hl = __ffsll((unsigned long long)open) - 1;
            const KT hk = __shfl(k, hl, 64);
            const int64_t start = base + hl;
            int64_t pos = base + 64, end = -1;
            while (end < 0 && pos - start < kProbeCap) {
                const int64_t ee = pos + lane;
                const bool stop = ee >= ns || (KT)(ks[ee < ns ? ee : ns - 1] >> sh) != hk;
                const uint64_t m = __ballot(stop);
                if (m) end = pos + __ffsll((unsigned long long)m) - 1;
                pos += 64;
            }
            const int64_t len = end < 0 ? kProbeCap : end - start;
            if (lane == 0) acc[lv] += (unsigned long long)(len * (len - 1) / 2);
        }
    }
#pragma unroll
    for (int lv = 0; lv < 8; ++lv) {
        unsigned long long v = acc[lv];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0 && v) atomicAdd(&out[lv], v);
    }
}

hipError_t launch_probe(const StepGeom& g, const SortBufs& b, int buf, unsigned long long* out, hipStream_t s)
{
    if (g.i_lo < 1 || g.i_lo > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(64), 0, s, out, 8);
    if (sort_keys_32(g))
        hipLaunchKernelGGL(k_probe_levels<uint32_t>, dim3(512), dim3(256), 0, s, (const uint32_t*)b.keys[buf],
                           g.ns, g.nseg, g.i_lo, out);
    else
        hipLaunchKernelGGL(k_probe_levels<uint64_t>, dim3(512), dim3(256), 0, s, (const uint64_t*)b.keys[buf],
                           g.ns, g.nseg, g.i_lo, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ verification
template <typename T>
__global__ __launch_bounds__(256) void k_verify(const Cand* __restrict__ cand, uint32_t cap,
                                                const Counters* __restrict__ cnt,
                                                const T* __restrict__ x, int64_t n, int64_t ns,
                                                int D, int w, int d, const double* __restrict__ mu,
                                                const double* __restrict__ isig,
                                                VRec* __restrict__ out, int nd)
{
    __shared__ double sorted[4][kMaxD];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t nc = cnt->n_cand;
    if (nc > cap) return;   // overflow: the batch is re-run with more room
    for (uint32_t c = blockIdx.x * 4 + wave; c < nc; c += gridDim.x * 4) {
        const Cand cd = cand[c];
        double my0 = 0.0, my1 = 0.0;
        for (int f = 0; f < D; ++f) {
            const T* xa = x + (int64_t)f * n + cd.a;
            const T* xb = x + (int64_t)f * n + cd.b;
            const double ma = mu[(int64_t)f * ns + cd.a], sa = isig[(int64_t)f * ns + cd.a];
            const double mb = mu[(int64_t)f * ns + cd.b], sb = isig[(int64_t)f * ns + cd.b];
            double acc = 0.0;
            for (int t = lane; t < w; t += 64) {
                const double za = ((double)xa[t] - ma) * sa;
                const double zb = ((double)xb[t] - mb) * sb;
                const double dz = za - zb;
                acc = acc + dz * dz;
            }
            const double dist = sqrt(wave_sum(acc));
            if ((f & 63) == lane) {
                if (f < 64) my0 = dist; else my1 = dist;
            }
        }
        // rank of each dimension by (distance, index)
        int rank0 = 0, rank1 = 0;
        for (int fp = 0; fp < D; ++fp) {
            const double v = __shfl(fp < 64 ? my0 : my1, fp & 63, 64);
            rank0 += (v < my0) || (v == my0 && fp < lane);
            rank1 += (v < my1) || (v == my1 && fp < lane + 64);
        }
        // distances in rank order; for each dimensionality d' in [d, d + nd):
        // the d' smallest (ties to the lower dimension), their sum in rank
        // order and the largest of them
        const int dtop = d + nd - 1;
        if (lane < D && rank0 < dtop) sorted[wave][rank0] = my0;
        if (lane + 64 < D && rank1 < dtop) sorted[wave][rank1] = my1;
        wave_sync_lds();
        double s = 0.0;
        if (lane == 0)
            for (int q = 0; q < d - 1; ++q) s = s + sorted[wave][q];
        for (int dd = 0; dd < nd; ++dd) {
            const int dq = d + dd;
            const uint64_t m0 = __ballot(lane < D && rank0 < dq), m1 = __ballot(lane + 64 < D && rank1 < dq);
            if (lane == 0) {
                s = s + sorted[wave][dq - 1];
                VRec v;
                v.dist_d = s;
                v.dist_max = sorted[wave][dq - 1];
                v.a = cd.a;
                v.b = cd.b;
                v.j = cd.j;
                v.pad = cd.pad;
                v.dims[0] = m0;
                v.dims[1] = m1;
                out[(size_t)dd * cap + c] = v;
            }
        }
        wave_sync_lds();
    }
}

hipError_t launch_verify(const Cand* cand, uint32_t cap, const Counters* cnt, const void* x,
                         int dtype, int64_t n, int64_t ns, int D, int w, int d, const double* mu,
                         const double* isig, VRec* out, hipStream_t s, int nd)
{
    if (nd < 1 || d + nd - 1 > D) return hipErrorInvalidValue;
    dim3 grid(2048);
    if (dtype == 0)
        hipLaunchKernelGGL(k_verify<double>, grid, dim3(256), 0, s, cand, cap, cnt, (const double*)x,
                           n, ns, D, w, d, mu, isig, out, nd);
    else
        hipLaunchKernelGGL(k_verify<float>, grid, dim3(256), 0, s, cand, cap, cnt, (const float*)x,
                           n, ns, D, w, d, mu, isig, out, nd);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pool
__device__ inline bool key_less(double da, uint32_t aa, uint32_t ab, double db, uint32_t ba, uint32_t bb)
{
    if (da != db) return da < db;
    if (aa != ba) return aa < ba;
    return ab < bb;
}

// Step of a verified record inside a replay window starting at step s0:
// step = (K - i) L + j (rounds descending, repetitions ascending).
__device__ inline int rec_step(const VRec& r, int K, int L, int s0)
{
    return (K - tag_round(r.pad)) * L + (int)r.j - s0;
}

// Keep the records that can still enter the pool: all of them while it is
// not full, else those strictly better than its current worst entry.
__global__ __launch_bounds__(256) void k_filter(const VRec* __restrict__ rec, uint32_t count,
                                                const PoolState* __restrict__ ps,
                                                const VRec* __restrict__ pools, int P,
                                                uint32_t* __restrict__ keep, ReplayCtl* __restrict__ rc)
{
    const bool full = ps->n_pool >= P;
    VRec thr;
    if (full) thr = pools[(int64_t)ps->cur * P + P - 1];
    bool dropped = false;
    for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c < count; c += gridDim.x * 256) {
        const VRec& r = rec[c];
        const int st = rec_step(r, rc->K, rc->L, rc->s0);
        if (st < 0 || st >= rc->nsteps) continue;   // not a step of this window
        if (tag_weight(r.pad) < rc->wmin) continue;   // a pair this dimensionality does not count
        if (!full || key_less(r.dist_d, r.a, r.b, thr.dist_d, thr.a, thr.b)) {
            const uint32_t pos = atomicAdd(&rc->n_keep, 1u);
            keep[pos] = c;
            atomicAdd(&rc->step_count[st], 1u);
        } else {
            dropped = true;
        }
    }
    // a record left out makes the pool a truncated one (what TOP may need
    // could be missing while |TOP| < k): one atomic per wavefront
    if (__ballot(dropped) && (threadIdx.x & 63) == 0) atomicOr(&rc->dropped, 1);
}

// Exclusive scan of the per-step counts (one block): offsets and cursors.
__global__ __launch_bounds__(1024) void k_step_scan(ReplayCtl* __restrict__ rc)
{
    __shared__ uint32_t sh[16];
    const int nsteps = rc->nsteps;
    const int per = (nsteps + 1023) / 1024;
    const int lo = threadIdx.x * per;
    const int hi = lo + per < nsteps ? lo + per : nsteps;
    uint32_t s = 0;
    for (int q = lo; q < hi; ++q) s += rc->step_count[q];
    uint32_t tot;
    uint32_t run = block_excl_scan<1024>(s, sh, &tot);
    for (int q = lo; q < hi; ++q) {
        const uint32_t v = rc->step_count[q];
        rc->step_off[q] = run;
        rc->step_count[q] = run;   // becomes the scatter cursor
        run += v;
    }
    if (threadIdx.x == 0) rc->step_off[nsteps] = tot;
}

__global__ __launch_bounds__(256) void k_step_scatter(const VRec* __restrict__ rec,
                                                      const uint32_t* __restrict__ keep,
                                                      uint32_t* __restrict__ order,
                                                      ReplayCtl* __restrict__ rc)
{
    const uint32_t nk = rc->n_keep;
    for (uint32_t q = blockIdx.x * 256 + threadIdx.x; q < nk; q += gridDim.x * 256) {
        const uint32_t c = keep[q];
        const uint32_t pos = atomicAdd(&rc->step_count[rec_step(rec[c], rc->K, rc->L, rc->s0)], 1u);
        order[pos] = c;
    }
}

constexpr int kPoolThreads = 1024;
constexpr int kChunk = 1024;

// Single work-group: for each step of the replay window in order, merge the
// step's kept records into the pool (sorted by (dist_d, a, b), duplicates
// dropped, best P kept), recompute TOP greedily when it can change, and
// record a snapshot of |TOP|, the k-th dist_max and TOP itself.
__global__ __launch_bounds__(kPoolThreads) void k_pool(const VRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ order,
                                                       const ReplayCtl* __restrict__ rc,
                                                       PoolState* __restrict__ ps,
                                                       VRec* __restrict__ pools, int P,
                                                       VRec* __restrict__ top, int k, int w,
                                                       Snap* __restrict__ snaps,
                                                       VRec* __restrict__ snap_tops)
{
    __shared__ double cd[kChunk];
    __shared__ uint32_t ca[kChunk], cb[kChunk], ci[kChunk];
    __shared__ uint32_t ka[kChunk], kb2[kChunk], kidx[kChunk];
    __shared__ double kd[kChunk];
    __shared__ int klb[kChunk];
    __shared__ uint32_t scan_sh[kPoolThreads / 64];
    __shared__ int acc_list[4096];
    __shared__ int s_np, s_cur, s_trunc, s_topn, s_improved;

    const int tid = threadIdx.x;
    const int nsteps = rc->nsteps;
    if (tid == 0) {
        s_np = ps->n_pool;
        s_cur = ps->cur;
        s_trunc = ps->truncated | (rc->dropped ? 1 : 0);
        s_topn = ps->top_n;
    }
    __syncthreads();

    for (int st = 0; st < nsteps; ++st) {
        const uint32_t beg = rc->step_off[st], end = rc->step_off[st + 1];
        if (beg == end) {
            // nothing new: the pool and TOP stand, the snapshot repeats (no
            // shared state changes, so no barrier is needed)
            if (tid == 0) {
                Snap sn;
                sn.top_n = s_topn;
                sn.truncated = s_trunc;
                sn.dist_max = s_topn == k ? top[k - 1].dist_max : 0.0;
                snaps[st] = sn;
            }
            for (int q = tid; q < s_topn; q += kPoolThreads) snap_tops[(int64_t)st * k + q] = top[q];
            continue;
        }
        if (tid == 0) s_improved = 0;
        __syncthreads();
        for (uint32_t start = beg; start < end; start += kChunk) {
            const uint32_t cnum = min((uint32_t)kChunk, end - start);
            double my_d = __builtin_huge_val();
            uint32_t my_a = 0xFFFFFFFFu, my_b = 0xFFFFFFFFu, my_i = 0xFFFFFFFFu;
            if ((uint32_t)tid < cnum) {
                my_i = order[start + tid];
                const VRec& r = rec[my_i];
                my_d = r.dist_d;
                my_a = r.a;
                my_b = r.b;
            }
            if (cnum <= 256) {
                // small chunk: rank by counting (ties, i.e. the same pair met
                // twice, ordered by position), one scatter
                kd[tid] = my_d; ka[tid] = my_a; kb2[tid] = my_b;
                __syncthreads();
                if ((uint32_t)tid < cnum) {
                    int rank = 0;
                    for (int q = 0; q < (int)cnum; ++q) {
                        const bool less = key_less(kd[q], ka[q], kb2[q], my_d, my_a, my_b) ||
                                          (q < tid && kd[q] == my_d && ka[q] == my_a && kb2[q] == my_b);
                        rank += less;
                    }
                    cd[rank] = my_d; ca[rank] = my_a; cb[rank] = my_b; ci[rank] = my_i;
                }
                __syncthreads();
            } else {
                cd[tid] = my_d; ca[tid] = my_a; cb[tid] = my_b; ci[tid] = my_i;
                __syncthreads();
                // bitonic sort of the chunk by (dist_d, a, b)
                for (int size = 2; size <= kChunk; size <<= 1) {
                    for (int stride = size >> 1; stride > 0; stride >>= 1) {
                        const int pa = tid ^ stride;
                        if (pa > tid) {
                            const bool up = (tid & size) == 0;
                            const bool gt = key_less(cd[pa], ca[pa], cb[pa], cd[tid], ca[tid], cb[tid]);
                            if (gt == up) {
                                double td = cd[tid]; cd[tid] = cd[pa]; cd[pa] = td;
                                uint32_t t1 = ca[tid]; ca[tid] = ca[pa]; ca[pa] = t1;
                                uint32_t t2 = cb[tid]; cb[tid] = cb[pa]; cb[pa] = t2;
                                uint32_t t3 = ci[tid]; ci[tid] = ci[pa]; ci[pa] = t3;
                            }
                        }
                        __syncthreads();
                    }
                }
            }
            const int np = s_np;
            const VRec* pool = pools + (int64_t)s_cur * P;
            VRec* npool = pools + (int64_t)(s_cur ^ 1) * P;
            // drop chunk entries already in the pool (a pair always has the same key)
            uint32_t keepme = 0;
            int lb_pool = 0;
            if ((uint32_t)tid < cnum) {
                int lo = 0, hi = np;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const VRec& pm = pool[mid];
                    if (key_less(pm.dist_d, pm.a, pm.b, cd[tid], ca[tid], cb[tid])) lo = mid + 1; else hi = mid;
                }
                lb_pool = lo;
                const bool dup = lo < np && pool[lo].a == ca[tid] && pool[lo].b == cb[tid];
                const bool dup_in_chunk = tid > 0 && ca[tid - 1] == ca[tid] && cb[tid - 1] == cb[tid];
                keepme = (dup || dup_in_chunk) ? 0u : 1u;
            }
            uint32_t ctot;
            const uint32_t cpos = block_excl_scan<kPoolThreads>(keepme, scan_sh, &ctot);
            if (keepme) {
                kd[cpos] = cd[tid];
                ka[cpos] = ca[tid];
                kb2[cpos] = cb[tid];
                kidx[cpos] = ci[tid];
                klb[cpos] = lb_pool;
            }
            __syncthreads();
            // merge into the other buffer, keeping the best P
            for (int p = tid; p < np; p += kPoolThreads) {
                const VRec& pe = pool[p];
                int lo = 0, hi = (int)ctot;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (key_less(kd[mid], ka[mid], kb2[mid], pe.dist_d, pe.a, pe.b)) lo = mid + 1; else hi = mid;
                }
                const int pos = p + lo;
                if (pos < P) npool[pos] = pe;
            }
            if ((uint32_t)tid < ctot) {
                const int pos = tid + klb[tid];
                if (pos < P) npool[pos] = rec[kidx[tid]];
            }
            __syncthreads();
            if (tid == 0) {
                const int tot = np + (int)ctot;
                if (tot > P) s_trunc = 1;
                s_np = tot < P ? tot : P;
                s_cur ^= 1;
                // TOP can change only if a new entry beats the current k-th pick
                if (ctot > 0) {
                    if (s_topn < k) s_improved = 1;
                    else {
                        const VRec& tk = top[k - 1];
                        if (key_less(kd[0], ka[0], kb2[0], tk.dist_d, tk.a, tk.b)) s_improved = 1;
                    }
                }
            }
            __syncthreads();
        }
        // greedy non-overlapping selection (wave 0)
        if (s_improved && tid < 64) {
            const VRec* pool = pools + (int64_t)s_cur * P;
            const int np = s_np;
            int got = 0;
            for (int e = 0; e < np && got < k; ++e) {
                const int64_t ea = pool[e].a, eb = pool[e].b;
                bool clash = false;
                for (int q = tid; q < got; q += 64) {
                    const VRec& t = pool[acc_list[q]];
                    clash |= 2 * llabs(ea - (int64_t)t.a) <= (int64_t)w;
                    clash |= 2 * llabs(ea - (int64_t)t.b) <= (int64_t)w;
                    clash |= 2 * llabs(eb - (int64_t)t.a) <= (int64_t)w;
                    clash |= 2 * llabs(eb - (int64_t)t.b) <= (int64_t)w;
                }
                if (__ballot(clash) == 0) {
                    if (tid == 0) acc_list[got] = e;
                    ++got;
                    wave_sync_lds();
                }
            }
            wave_sync_lds();
            for (int q = tid; q < got; q += 64) top[q] = pool[acc_list[q]];
            if (tid == 0) s_topn = got;
        }
        __syncthreads();
        if (tid == 0) {
            Snap sn;
            sn.top_n = s_topn;
            sn.truncated = s_trunc;
            sn.dist_max = s_topn == k ? top[k - 1].dist_max : 0.0;
            snaps[st] = sn;
        }
        for (int q = tid; q < s_topn; q += kPoolThreads) snap_tops[(int64_t)st * k + q] = top[q];
        __syncthreads();
    }
    if (tid == 0) {
        ps->n_pool = s_np;
        ps->cur = s_cur;
        ps->truncated = s_trunc;
        ps->top_n = s_topn;
    }
}

hipError_t launch_replay(const VRec* rec, uint32_t count, uint32_t* keep, uint32_t* order,
                         ReplayCtl* rc, PoolState* ps, VRec* pools, int P, VRec* top, int k, int w,
                         Snap* snaps, VRec* snap_tops, hipStream_t s)
{
    if (k > 4096) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)(count == 0 ? 1 : (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_filter, dim3(blocks), dim3(256), 0, s, rec, count, ps, pools, P, keep, rc);
    hipLaunchKernelGGL(k_step_scan, dim3(1), dim3(1024), 0, s, rc);
    hipLaunchKernelGGL(k_step_scatter, dim3(blocks), dim3(256), 0, s, rec, keep, order, rc);
    hipLaunchKernelGGL(k_pool, dim3(1), dim3(kPoolThreads), 0, s, rec, order, rc, ps, pools, P, top,
                       k, w, snaps, snap_tops);
    return hipGetLastError();
}

__global__ void k_pool_reset(PoolState* ps)
{
    ps->n_pool = 0;
    ps->top_n = 0;
    ps->truncated = 0;
    ps->cur = 0;
    ps->skipped = 0;
}

hipError_t launch_pool_reset(PoolState* ps, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool_reset, dim3(1), dim3(1), 0, s, ps);
    return hipGetLastError();
}

__global__ void k_zero(uint32_t* p, size_t words)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < words; q += (size_t)gridDim.x * blockDim.x)
        p[q] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const size_t words = bytes / 4;
    const unsigned blocks = (unsigned)((words + 255) / 256 < 1024 ? (words + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_zero, dim3(blocks ? blocks : 1), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError();
}

// ------------------------------------------------------------------ exact fallback
// Every non-trivial pair (a, b), b >= a + floor(w/2) + 1, rows [row_lo, row_hi):
// row a holds M - a pairs (M = n_s - floor(w/2) - 1) for a < M, stored at
// offset(a) - base, offset(a) = a M - a (a - 1) / 2.
__global__ void k_allpairs(int64_t ns, int w, int64_t row_lo, int64_t row_hi, int64_t base,
                           Cand* __restrict__ cand)
{
    const int64_t M = ns - (w / 2) - 1;
    for (int64_t a = row_lo + blockIdx.x; a < row_hi; a += gridDim.x) {
        if (a >= M) continue;
        const int64_t off = a * M - a * (a - 1) / 2 - base;
        const int64_t first = a + (w / 2) + 1;
        for (int64_t b = first + threadIdx.x; b < ns; b += blockDim.x)
            cand[off + (b - first)] = Cand{(uint32_t)a, (uint32_t)b, 0u, 0u};
    }
}

__global__ void k_set_count(Counters* cnt, uint32_t v)
{
    cnt->n_cand = v;
}

hipError_t launch_set_count(Counters* cnt, uint32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, cnt, v);
    return hipGetLastError();
}

hipError_t launch_allpairs(int64_t ns, int w, int64_t row_lo, int64_t row_hi, int64_t base,
                           Cand* cand, Counters* cnt, hipStream_t s)
{
    const int64_t M = ns - (w / 2) - 1;
    auto off = [M](int64_t a) { int64_t aa = a < M ? a : M; return aa * M - aa * (aa - 1) / 2; };
    const int64_t count = off(row_hi) - off(row_lo);
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, cnt, (uint32_t)count);
    hipLaunchKernelGGL(k_allpairs, dim3(1024), dim3(256), 0, s, ns, w, row_lo, row_hi, base, cand);
    return hipGetLastError();
}

}  // namespace mm
