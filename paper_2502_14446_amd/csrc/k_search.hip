// Index traversal on gfx950 (Algorithm 1, rounds i = K..1; sections 4 and 6.2).
//
// One launch sequence handles a batch of repetitions j0 .. j0+B-1 of round i
// for every dimension: B * D "segments" of n_s windows each.
//
//  * sort_prefixes  stable LSD radix sort of every segment by the length-i
//                   hash prefix of repetition j (left half-function j div m,
//                   right half-function j mod m; section 6.1), one byte per
//                   pass. Pass 0 builds the keys straight from the index.
//                   Tiles of 4096 elements are ranked in LDS with wave ballots
//                   and written out digit by digit (coalesced).
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

// Prefix of length i of the tensored key: the first ceil(i/2) symbols of the
// left word and the first floor(i/2) of the right word. The interleaved key
// of section 6.1 has equal length-i prefixes exactly when both parts are
// equal, which is all the traversal needs (no order between runs is used).
template <typename KT>
__device__ inline KT make_key(uint32_t L, uint32_t R, int i)
{
    const int lb = (i + 1) >> 1, rb = i >> 1;
    uint64_t v = (uint64_t)(L >> (32 - 8 * lb));
    if (rb) v = (v << (8 * rb)) | (uint64_t)(R >> (32 - 8 * rb));
    return (KT)v;
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
    const int jb = seg / g.D, f = seg - jb * g.D;
    const int j = g.j0 + jb, l = j / g.m, r = j - l * g.m;
    SegPtr p;
    p.Lw = H + ((int64_t)f * g.NF + l) * g.ns;
    p.Rw = H + ((int64_t)f * g.NF + g.NL + r) * g.ns;
    return p;
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
    for (int64_t e = base + threadIdx.x; e < end; e += 256) {
        KT key = FIRST ? make_key<KT>(sp.Lw[e], sp.Rw[e], g.i) : ks[e];
        atomicAdd(&cnt[(uint32_t)(key >> (8 * pass)) & 255u], 1u);
    }
    __syncthreads();
    hist[((int64_t)seg * 256 + threadIdx.x) * tiles + tile] = cnt[threadIdx.x];
}

// Exclusive scan of one segment's digit-major histogram (digit, tile).
__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ hist, int64_t tiles)
{
    __shared__ uint32_t sh[16];
    uint32_t* h = hist + (int64_t)blockIdx.x * 256 * tiles;
    const int64_t total = 256 * tiles;
    const int64_t per = (total + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < total ? lo + per : total;
    uint32_t s = 0;
    for (int64_t q = lo; q < hi; ++q) s += h[q];
    uint32_t tot;
    uint32_t run = block_excl_scan<1024>(s, sh, &tot);
    for (int64_t q = lo; q < hi; ++q) {
        uint32_t v = h[q];
        h[q] = run;
        run += v;
    }
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

    const int seg = blockIdx.y;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kSortTile;
    const int count = (int)((g.ns - base) < kSortTile ? (g.ns - base) : kSortTile);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = threadIdx.x; q < 4 * 256; q += 256) (&wcnt[0][0])[q] = 0;
    gofs[threadIdx.x] = hist[((int64_t)seg * 256 + threadIdx.x) * tiles + tile];
    __syncthreads();

    SegPtr sp;
    if (FIRST) sp = seg_words(H, g, seg);
    const KT* ks = kin + (int64_t)seg * g.ns;
    const uint32_t* is = iin + (int64_t)seg * g.ns;
    KT k_[ITEMS];
    uint32_t i_[ITEMS], r_[ITEMS];
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const int e = wave * (kSortTile / 4) + s * 64 + lane;   // wave-contiguous blocks keep order
        const bool valid = e < count;
        KT key = 0;
        uint32_t id = 0;
        if (valid) {
            const int64_t ge = base + e;
            if (FIRST) {
                key = make_key<KT>(sp.Lw[ge], sp.Rw[ge], g.i);
                id = (uint32_t)ge;
            } else {
                key = ks[ge];
                id = is[ge];
            }
        }
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
        k_[s] = key;
        i_[s] = id;
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
    if (g.i <= 4) {
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
    if (g.i <= 4) {
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
// Does pair (a, b), colliding at prefix i in dimension f, enter the step's
// candidates? W_i over all dimensions must reach d, f must be the lowest
// colliding dimension, and (when i < K) W_{i+1} must stay below d.
__device__ inline bool pair_is_candidate(const uint32_t* __restrict__ H, const StepGeom& g, int f,
                                         int l, int r, uint32_t a, uint32_t b, int d)
{
    const int i = g.i;
    const uint32_t mL = top_mask((i + 1) >> 1), mR = top_mask(i >> 1);
    const bool deeper = i < g.K;
    const uint32_t mL1 = top_mask((i + 2) >> 1), mR1 = top_mask((i + 1) >> 1);
    int Wi = 0, Wi1 = 0;
    for (int fp = 0; fp < g.D; ++fp) {
        const uint32_t* Lw = H + ((int64_t)fp * g.NF + l) * g.ns;
        const uint32_t* Rw = H + ((int64_t)fp * g.NF + g.NL + r) * g.ns;
        const uint32_t xl = Lw[a] ^ Lw[b];
        const uint32_t xr = Rw[a] ^ Rw[b];
        const bool eq = ((xl & mL) | (xr & mR)) == 0u;
        if (fp < f && eq) return false;
        Wi += eq;
        if (deeper) {
            const bool eq1 = ((xl & mL1) | (xr & mR1)) == 0u;
            Wi1 += eq1;
            if (Wi1 >= d) return false;
        }
        if (Wi + (g.D - 1 - fp) < d) return false;
    }
    return Wi >= d;
}

template <typename KT>
__global__ __launch_bounds__(256) void k_enum(const KT* __restrict__ keys, const uint32_t* __restrict__ idx,
                                              const uint32_t* __restrict__ H, StepGeom g, int d, int w,
                                              Cand* __restrict__ cand, uint32_t cap,
                                              Counters* __restrict__ cnt)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)g.nseg * g.ns;
    unsigned long long ncoll = 0;
    if (gid < total) {
        const int seg = (int)(gid / g.ns);
        const int64_t t = gid - (int64_t)seg * g.ns;
        const KT* ks = keys + (int64_t)seg * g.ns;
        const uint32_t* is = idx + (int64_t)seg * g.ns;
        const KT key = ks[t];
        if (t + 1 < g.ns && ks[t + 1] == key) {
            const int jb = seg / g.D, f = seg - jb * g.D;
            const int j = g.j0 + jb, l = j / g.m, r = j - l * g.m;
            const uint32_t a = is[t];
            for (int64_t q = t + 1; q < g.ns && ks[q] == key; ++q) {
                const uint32_t b = is[q];
                if (2 * (int64_t)(b - a) <= (int64_t)w) continue;   // trivial match
                ++ncoll;
                if (pair_is_candidate(H, g, f, l, r, a, b, d)) {
                    const uint32_t pos = atomicAdd(&cnt->n_cand, 1u);
                    if (pos < cap) cand[pos] = Cand{a, b, (uint32_t)j, 0u};
                }
            }
        }
    }
    // one atomic per wave for the collision counter
    unsigned long long tot = ncoll;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if (lane_id() == 0 && tot) atomicAdd(&cnt->n_coll, tot);
}

hipError_t launch_enum(const StepGeom& g, const uint32_t* H, const SortBufs& b, int buf, int d,
                       int w, Cand* cand, uint32_t cap, Counters* cnt, hipStream_t s)
{
    const int64_t total = (int64_t)g.nseg * g.ns;
    dim3 grid((unsigned)((total + 255) / 256));
    if (g.i <= 4)
        hipLaunchKernelGGL(k_enum<uint32_t>, grid, dim3(256), 0, s, (const uint32_t*)b.keys[buf],
                           b.idx[buf], H, g, d, w, cand, cap, cnt);
    else
        hipLaunchKernelGGL(k_enum<uint64_t>, grid, dim3(256), 0, s, (const uint64_t*)b.keys[buf],
                           b.idx[buf], H, g, d, w, cand, cap, cnt);
    return hipGetLastError();
}

// ------------------------------------------------------------------ verification
template <typename T>
__global__ __launch_bounds__(256) void k_verify(const Cand* __restrict__ cand, uint32_t cap,
                                                const Counters* __restrict__ cnt,
                                                const T* __restrict__ x, int64_t n, int64_t ns,
                                                int D, int w, int d, const double* __restrict__ mu,
                                                const double* __restrict__ isig,
                                                VRec* __restrict__ out)
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
        const bool sel0 = lane < D && rank0 < d;
        const bool sel1 = lane + 64 < D && rank1 < d;
        if (sel0) sorted[wave][rank0] = my0;
        if (sel1) sorted[wave][rank1] = my1;
        const uint64_t m0 = __ballot(sel0), m1 = __ballot(sel1);
        wave_sync_lds();
        if (lane == 0) {
            double s = 0.0;
            for (int q = 0; q < d; ++q) s = s + sorted[wave][q];
            VRec v;
            v.dist_d = s;
            v.dist_max = sorted[wave][d - 1];
            v.a = cd.a;
            v.b = cd.b;
            v.j = cd.j;
            v.pad = 0;
            v.dims[0] = m0;
            v.dims[1] = m1;
            out[c] = v;
        }
        wave_sync_lds();
    }
}

hipError_t launch_verify(const Cand* cand, uint32_t cap, const Counters* cnt, const void* x,
                         int dtype, int64_t n, int64_t ns, int D, int w, int d, const double* mu,
                         const double* isig, VRec* out, hipStream_t s)
{
    dim3 grid(2048);
    if (dtype == 0)
        hipLaunchKernelGGL(k_verify<double>, grid, dim3(256), 0, s, cand, cap, cnt, (const double*)x,
                           n, ns, D, w, d, mu, isig, out);
    else
        hipLaunchKernelGGL(k_verify<float>, grid, dim3(256), 0, s, cand, cap, cnt, (const float*)x,
                           n, ns, D, w, d, mu, isig, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pool
__device__ inline bool key_less(double da, uint32_t aa, uint32_t ab, double db, uint32_t ba, uint32_t bb)
{
    if (da != db) return da < db;
    if (aa != ba) return aa < ba;
    return ab < bb;
}

__global__ __launch_bounds__(256) void k_filter(const VRec* __restrict__ rec, uint32_t cap,
                                                const Counters* __restrict__ cnt_in,
                                                const PoolState* __restrict__ ps,
                                                const VRec* __restrict__ pools, int P,
                                                uint32_t* __restrict__ keep, Counters* cnt_out)
{
    const uint32_t nc = cnt_in->n_cand;
    if (nc > cap) return;
    const bool full = ps->n_pool >= P;
    VRec thr;
    if (full) thr = pools[(int64_t)ps->cur * P + P - 1];
    for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c < nc; c += gridDim.x * 256) {
        const VRec& r = rec[c];
        if (!full || key_less(r.dist_d, r.a, r.b, thr.dist_d, thr.a, thr.b)) {
            const uint32_t pos = atomicAdd(&cnt_out->n_keep, 1u);
            keep[pos] = c;
        }
    }
}

hipError_t launch_filter(const VRec* rec, uint32_t cap, const Counters* cnt, const PoolState* ps,
                         const VRec* pools, int P, uint32_t* keep, Counters* cnt_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_filter, dim3(1024), dim3(256), 0, s, rec, cap, cnt, ps, pools, P, keep, cnt_out);
    return hipGetLastError();
}

constexpr int kPoolThreads = 1024;
constexpr int kChunk = 1024;
constexpr int kMaxBatch = 64;

// Single work-group: for each repetition of the batch in order, merge its
// kept candidates into the pool (sorted by (dist_d, a, b), duplicates
// dropped, best P kept), recompute TOP greedily when it can change, and
// record a snapshot.
__global__ __launch_bounds__(kPoolThreads) void k_pool(const VRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ keep,
                                                       uint32_t* __restrict__ order, uint32_t cap,
                                                       Counters* __restrict__ cnt,
                                                       PoolState* __restrict__ ps,
                                                       VRec* __restrict__ pools, int P,
                                                       VRec* __restrict__ top, int k, int w, int j0,
                                                       int B, Snap* __restrict__ snaps,
                                                       VRec* __restrict__ snap_tops)
{
    __shared__ uint32_t jcount[kMaxBatch + 1];
    __shared__ uint32_t joff[kMaxBatch + 1];
    __shared__ double cd[kChunk];
    __shared__ uint32_t ca[kChunk], cb[kChunk], ci[kChunk];
    __shared__ uint32_t scan_sh[kPoolThreads / 64];
    __shared__ int acc_list[4096];
    __shared__ int s_np, s_cur, s_trunc, s_topn, s_improved, s_cn;

    const int tid = threadIdx.x;
    if (cnt->n_cand > cap) {
        if (tid == 0) ps->skipped = 1;
        return;
    }
    const uint32_t nkeep = cnt->n_keep;
    if (tid == 0) {
        s_np = ps->n_pool;
        s_cur = ps->cur;
        s_trunc = ps->truncated;
        s_topn = ps->top_n;
        ps->skipped = 0;
    }
    if (tid <= kMaxBatch) jcount[tid] = 0;
    __syncthreads();
    // bucket the kept candidates by repetition
    for (uint32_t q = tid; q < nkeep; q += kPoolThreads) atomicAdd(&jcount[rec[keep[q]].j - j0], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t s = 0;
        for (int b = 0; b < B; ++b) {
            joff[b] = s;
            s += jcount[b];
            jcount[b] = joff[b];
        }
        joff[B] = s;
    }
    __syncthreads();
    for (uint32_t q = tid; q < nkeep; q += kPoolThreads) {
        const uint32_t c = keep[q];
        const uint32_t pos = atomicAdd(&jcount[rec[c].j - j0], 1u);
        order[pos] = c;
    }
    __syncthreads();

    for (int jb = 0; jb < B; ++jb) {
        if (tid == 0) s_improved = 0;
        __syncthreads();
        for (uint32_t start = joff[jb]; start < joff[jb + 1]; start += kChunk) {
            const uint32_t cnum = min((uint32_t)kChunk, joff[jb + 1] - start);
            // load the chunk, pad with +inf
            if ((uint32_t)tid < cnum) {
                const VRec& r = rec[order[start + tid]];
                cd[tid] = r.dist_d;
                ca[tid] = r.a;
                cb[tid] = r.b;
                ci[tid] = order[start + tid];
            } else {
                cd[tid] = __builtin_huge_val();
                ca[tid] = 0xFFFFFFFFu;
                cb[tid] = 0xFFFFFFFFu;
                ci[tid] = 0xFFFFFFFFu;
            }
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
            const int np = s_np;
            const VRec* pool = pools + (int64_t)s_cur * P;
            VRec* npool = pools + (int64_t)(s_cur ^ 1) * P;
            // drop chunk entries already in the pool
            uint32_t keepme = 0;
            int lb_pool = 0;
            if ((uint32_t)tid < cnum) {
                int lo = 0, hi = np;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    const VRec& pm = pool[mid];
                    if (key_less(pm.dist_d, pm.a, pm.b, cd[tid], ca[tid], cb[tid])) lo = mid + 1; else hi = mid;
                }
                lb_pool = lo;
                const bool dup = lo < np && pool[lo].a == ca[tid] && pool[lo].b == cb[tid];
                keepme = dup ? 0u : 1u;
            }
            uint32_t ctot;
            const uint32_t cpos = block_excl_scan<kPoolThreads>(keepme, scan_sh, &ctot);
            // compact kept chunk entries (their pool lower bounds travel along)
            __shared__ uint32_t ka[kChunk], kb2[kChunk], kidx[kChunk];
            __shared__ double kd[kChunk];
            __shared__ int klb[kChunk];
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
                    int mid = (lo + hi) >> 1;
                    if (key_less(kd[mid], ka[mid], kb2[mid], pe.dist_d, pe.a, pe.b)) lo = mid + 1; else hi = mid;
                }
                const int pos = p + lo;
                if (pos < P) npool[pos] = pe;
            }
            if ((uint32_t)tid < ctot) {
                const int pos = tid + klb[tid];
                if (pos < P) {
                    VRec v = rec[kidx[tid]];
                    npool[pos] = v;
                }
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
                const uint32_t ea = pool[e].a, eb = pool[e].b;
                bool clash = false;
                for (int s = tid; s < got; s += 64) {
                    const VRec& t = pool[acc_list[s]];
                    const int64_t h = w;
                    clash |= 2 * llabs((int64_t)ea - (int64_t)t.a) <= h;
                    clash |= 2 * llabs((int64_t)ea - (int64_t)t.b) <= h;
                    clash |= 2 * llabs((int64_t)eb - (int64_t)t.a) <= h;
                    clash |= 2 * llabs((int64_t)eb - (int64_t)t.b) <= h;
                }
                if (__ballot(clash) == 0) {
                    if (tid == 0) acc_list[got] = e;
                    ++got;
                    wave_sync_lds();
                }
            }
            wave_sync_lds();
            for (int s = tid; s < got; s += 64) top[s] = pool[acc_list[s]];
            if (tid == 0) s_topn = got;
        }
        __syncthreads();
        __threadfence_block();
        if (tid == 0) {
            Snap sn;
            sn.top_n = s_topn;
            sn.truncated = s_trunc;
            sn.dist_max = s_topn == k ? top[k - 1].dist_max : 0.0;
            snaps[jb] = sn;
        }
        for (int s = tid; s < s_topn; s += kPoolThreads) snap_tops[(int64_t)jb * k + s] = top[s];
        __syncthreads();
    }
    if (tid == 0) {
        ps->n_pool = s_np;
        ps->cur = s_cur;
        ps->truncated = s_trunc;
        ps->top_n = s_topn;
    }
}

hipError_t launch_pool(const VRec* rec, const uint32_t* keep, uint32_t cap, Counters* cnt,
                       PoolState* ps, VRec* pools, int P, VRec* top, int k, int w, int j0, int B,
                       Snap* snaps, VRec* snap_tops, hipStream_t s)
{
    if (B > kMaxBatch || k > 4096) return hipErrorInvalidValue;
    // the order scratch lives right after the keep list (same capacity)
    uint32_t* order = const_cast<uint32_t*>(keep) + cap;
    hipLaunchKernelGGL(k_pool, dim3(1), dim3(kPoolThreads), 0, s, rec, keep, order, cap, cnt, ps,
                       pools, P, top, k, w, j0, B, snaps, snap_tops);
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
    cnt->n_keep = 0;
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
