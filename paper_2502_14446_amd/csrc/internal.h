// Internal declarations shared by the translation units of libmomenti.
// Kernels live in k_hash.hip (index construction) and k_search.hip (index
// traversal); the C ABI and the host-side orchestration in momenti.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>

namespace mm {

// A candidate pair (a < b) emitted by the traversal, tagged with the
// repetition j, the round (prefix length) i that produced it and the number
// W of dimensions it collided in there.
struct Cand {
    uint32_t a, b, j, pad;   // pad: round i | W << 8
};
__host__ __device__ inline int tag_round(uint32_t pad) { return (int)(pad & 0xFFu); }
__host__ __device__ inline int tag_weight(uint32_t pad) { return (int)(pad >> 8); }

// A verified pair: dist_d (definition "d-dimensional distance"), dist_max
// (Eq. distdmax), the chosen dimensions and the repetition that produced it.
struct VRec {
    double dist_d, dist_max;
    uint32_t a, b, j, pad;   // pad: round i | W << 8 (as in Cand)
    uint64_t dims[2];
};
static_assert(sizeof(VRec) == 48, "VRec layout");

// State of the device-side pool of verified pairs and of TOP.
struct PoolState {
    int32_t n_pool;      // entries in the pool (sorted by (dist_d, a, b))
    int32_t top_n;       // |TOP|
    int32_t truncated;   // the pool dropped entries at some point (it holds the best P only)
    int32_t cur;         // which of the two pool buffers is current
    int32_t skipped;     // the pool step was skipped because candidates overflowed
    int32_t pad[3];
};

// Per-repetition result of one traversal step.
struct Snap {
    int32_t top_n;
    int32_t truncated;
    double dist_max;     // dist_max of TOP[k-1] when top_n == k
};

// Device counters of one batch of traversal steps.
struct Counters {
    uint32_t n_cand;             // candidates emitted (may exceed the buffer)
    uint32_t max_run;            // longest run that left its 64-element window
    unsigned long long n_coll;   // pairs of equal prefixes in the segments (trivial matches included)
    unsigned long long n_memb;   // elements in runs of >= 2
    unsigned long long n_screen; // non-trivial pairs that passed the fingerprint screen
    uint32_t n_units;            // tile rows of long runs queued for the tile kernel
    uint32_t pad_;
};

// One tile row of a run of equal prefixes inside a sorted segment: tile tp of
// the run is paired with itself and with every later tile.
struct RunRec {
    uint32_t seg, start, len, tp;
};
// Tile rows a batch of nseg segments can queue at most: a run is queued only
// when it leaves its 64-element window (at most one per window), and cut into
// tiles of at least 16 members.
inline int64_t units_bound(int64_t nseg, int64_t ns) { return nseg * ((ns + 15) / 16 + (ns + 63) / 64 + 1); }

// Control block of one replay of verified records in step order.
constexpr int kMaxSteps = 8 * 1024;
struct ReplayCtl {
    uint32_t n_keep;
    int32_t K, L, s0, nsteps;
    int32_t dropped;     // set by the filter when it left out a record (the pool was full)
    int32_t wmin;        // records with a weight W below this are not for this pool
    int32_t pad;
    uint32_t step_count[kMaxSteps];
    uint32_t step_off[kMaxSteps + 1];
};

constexpr int kMaxD = 128;
constexpr int kMaxW = 8192;
// Repetitions: L = 256 gives m = 16 and 16 + 16 half-functions, 4 (ceil(L / m)
// + min(L, m)) = 128 hash columns, the projection tile's width (4 MFMA blocks
// of 32); L = 257 would need 132.
constexpr int kMaxL = 256;
constexpr double kFlatRel = 1e-8;      // sigma <= kFlatRel * |mu|: flat window

// ---- index construction (k_hash.hip) ----
// *first = index (f n + t) of the first non-finite series value, left as set
// by the caller (~0) when there is none.
hipError_t launch_first_nonfinite(const void* x, int dtype, int64_t total, unsigned long long* first,
                                  hipStream_t s);
hipError_t launch_stats(const void* x, int dtype, int64_t n, int64_t ns, int D, int w,
                        double* mu, double* isig, hipStream_t s);
hipError_t launch_rsample(const void* x, int dtype, int64_t n, int D, int w, const int64_t* win,
                          int S, const double* vec, int nvec, double* dots, hipStream_t s);
// proj: 0 f64, 1 f32, 2 bf16, 3 fp8. R/U in the layout and type of that path.
hipError_t launch_proj(int proj, const void* x, int dtype, int64_t n, int64_t ns, int D, int w,
                       const double* mu, const double* isig, const void* R, const void* U,
                       int Cpad, int wpad, int NF, int K, double inv_r, uint32_t* H, hipStream_t s);
// LDS bytes one work-group of the BF16 (proj 2) or FP8 (proj 3) projection
// takes for Cpad columns and rows padded to wpad; at most kMaxLdsBytes fit a
// CU. (The FP64 and FP32 kernels stay far below it for any w <= kMaxW.)
size_t lowp_lds_bytes(int proj, int Cpad, int wpad);
constexpr size_t kMaxLdsBytes = 160 * 1024;

// ---- index traversal (k_search.hip) ----
struct SortBufs {
    void* keys[2];
    uint32_t* idx[2];
    uint32_t* hist;
    int64_t tiles;
    RunRec* units;       // tile rows of long runs, units_bound(nseg, ns) of them
    uint32_t ucap;
};
struct StepGeom {
    int64_t ns;
    int D, NF, NL, m;
    int j0, nseg;        // first repetition of the batch, segments = reps * Ds
    int Ds;              // dimensions that get segments: seg = rep * Ds + f, f < Ds
    int i, K;            // highest round of the group; K
    int i_lo;            // lowest round of the group: segments are sorted by this prefix length
    int hashed;          // 1: sorted by a 24-bit hash of that prefix instead (equal prefixes
                         // stay adjacent; the rare equal hashes of different prefixes only
                         // add members to a run, and the exact test rejects them)
    int dhi;             // highest dimensionality searched (several at once, section 6.3): a pair
                         // is emitted at round i < K while some d in (W_{i+1}, W_i] is at most
                         // dhi (d itself for one dimensionality); its W_i rides in Cand.pad
    int part, nparts;    // emit only the candidates (a, b) with pair_part(a, b, nparts) == part
                         // (nparts a power of two; 1 = all): a step whose candidates do not fit
                         // in memory at once is enumerated in parts
    int fq;              // 1: second-stage rows are built and screen the pairs (second_stage_pays)
};
// Does the second screen pay for its table? A pair passes the first one by
// chance when >= d - 1 of the other D - 1 dimensions have equal 8-bit digests
// without equal prefixes, about C(D - 1, d - 1) 2^(-8 (d - 1)) of the pairs
// (the digests of unequal prefixes agree with probability 2^-8). Below 2^-24
// those pairs go straight to the exact test: a few thousand per 10^11 pairs.
inline int second_stage_pays(int D, int d)
{
    if (d <= 1) return 0;   // every pair of a run passes both screens
    double lp = -8.0 * (d - 1) * 0.6931471805599453;
    for (int q = 0; q < d - 1; ++q) lp += std::log((double)(D - 1 - q) / (double)(q + 1));
    return lp > -24.0 * 0.6931471805599453 ? 1 : 0;
}
// Part of a candidate pair when a step is enumerated in parts.
__host__ __device__ inline uint32_t pair_part(uint32_t a, uint32_t b, int nparts)
{
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    return h & (uint32_t)(nparts - 1);
}
// Sort keys of a segment element: the length-i_lo prefix, or its 24-bit hash.
inline bool sort_keys_32(const StepGeom& g) { return g.hashed || g.i_lo <= 4; }
inline int sort_passes(const StepGeom& g) { return g.hashed ? 3 : g.i_lo; }
// Fingerprint rows are bit-sliced: a window's digest of dimension f (8 bits
// in the first-stage row, 16 in the second) is spread over planes, bit k of
// the digest being bit f of plane k. With D <= 32 a plane has Dp bits (D
// rounded up to 4, 8, 16 or 32), 32 / Dp planes to a word, plane k in word
// k / (32 / Dp) at bit (k mod (32 / Dp)) Dp; with D > 32 the dimensions come
// in chunks of 32, one word per plane, chunk q's plane k in word P q + k
// (P = 8 or 16 planes). Padding dimensions are zero bits. Two windows'
// digests differ in dimension f iff some plane differs at f, so the number
// of differing digests is the popcount of the OR of the XORed words, folded
// over the planes that share a word.
__host__ __device__ inline int plane_bits(int D) { return D <= 4 ? 4 : D <= 8 ? 8 : D <= 16 ? 16 : 32; }
// 32-bit words of a first-stage row (8 planes): 1, 2, 4, 8 or 8 per chunk
__host__ __device__ inline int fp_words(int D) { return D <= 32 ? plane_bits(D) / 4 : 8 * ((D + 31) / 32); }
// 32-bit words of a second-stage row (16 planes), in whole 16-byte pieces
__host__ __device__ inline int fq_words(int D)
{
    return D <= 32 ? (plane_bits(D) / 2 < 4 ? 4 : plane_bits(D) / 2) : 16 * ((D + 31) / 32);
}
constexpr int kSortTile = 4096;

// Stable LSD sort of every segment of the batch by its length-i hash prefix,
// one byte per pass (pass 0 reads the keys straight from the index); each
// pass is histogram + scan + scatter from buffer `cur` to buffer `cur ^ 1`,
// except that launch_fptable writes pass 0's histogram.
hipError_t launch_hist(const StepGeom& g, const uint32_t* H, const SortBufs& b, int pass, int cur,
                       hipStream_t s);
hipError_t launch_scan(const StepGeom& g, const SortBufs& b, hipStream_t s);
hipError_t launch_scatter(const StepGeom& g, const uint32_t* H, const SortBufs& b, int pass, int cur,
                          hipStream_t s);
// Fingerprint rows of the batch, fps[jb][a][fp_words(D)]: an 8-bit digest
// of every dimension's length-i_lo prefix (the prefix itself when i_lo = 1);
// and second-stage rows fq[jb][a][fq_words(D)] with a 16-bit digest per
// dimension (the prefix itself when i_lo <= 2); both bit-sliced. The same
// pass over the index words writes the histogram of the sort's pass 0 into
// b.hist (the batch's segments), so that pass starts from the scan.
hipError_t launch_fptable(const uint32_t* H, const StepGeom& g, int reps, uint32_t* fps, uint32_t* fq,
                          const SortBufs& b, hipStream_t s);
// Runs of >= 2 equal length-i_lo prefixes and the pairs of every run (one
// launch); `part` holds enum_partials(g) per-work-group triples of counts
// (pairs in runs, run members, screened pairs). kt = min(i_hi + 1, K).
int64_t enum_partials(const StepGeom& g);
hipError_t launch_enum(const StepGeom& g, const SortBufs& b, int buf, const uint32_t* H,
                       const uint32_t* fps, const uint32_t* fq, int kt, int d, int w, Cand* cand,
                       uint32_t cap, Counters* cnt, unsigned long long* part, hipStream_t s);
// Probe of one sorted batch: out[i - 1] = pairs of windows (in the batch's
// segments) that share their length-i prefix, i = 1 .. g.i_lo, for segments
// sorted by their length-g.i_lo prefix (8 counters, device memory).
hipError_t launch_probe(const StepGeom& g, const SortBufs& b, int buf, unsigned long long* out, hipStream_t s);
// Verification of the candidates: for every d in [d, d + nd), record
// c's dist_d, dist_max and dimensions at out[(d - d0) * cap + c].
hipError_t launch_verify(const Cand* cand, uint32_t cap, const Counters* cnt, const void* x,
                         int dtype, int64_t n, int64_t ns, int D, int w, int d, const double* mu,
                         const double* isig, VRec* out, hipStream_t s, int nd = 1);
// Replay `count` verified records (tagged with round and repetition) in step
// order through the pool: filter, bucket by step, then one work-group walks
// the steps of rc->[s0, s0 + nsteps) and writes a snapshot per step. rc must
// hold K, L, s0, nsteps and zeroed counts; keep and order hold count entries.
hipError_t launch_replay(const VRec* rec, uint32_t count, uint32_t* keep, uint32_t* order,
                         ReplayCtl* rc, PoolState* ps, VRec* pools, int P, VRec* top, int k, int w,
                         Snap* snaps, VRec* snap_tops, hipStream_t s);
hipError_t launch_pool_reset(PoolState* ps, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_allpairs(int64_t ns, int w, int64_t row_lo, int64_t row_hi, int64_t base,
                           Cand* cand, Counters* cnt, hipStream_t s);
// Set the candidate count (e.g. to the buffer's capacity after an overflow,
// so that the buffered candidates can be verified).
hipError_t launch_set_count(Counters* cnt, uint32_t v, hipStream_t s);

// ---- exact answer over every pair (k_exact.hip) ----
// One launch of the diagonal sweep: work items [item_lo, item_hi) of a grid
// of groups of G adjacent diagonals (the first at s_lo, group gr at
// s_lo + gr G) times chunks of Lc pairs along them (item = gr chunks + c).
// Pairs whose d smallest per-dimension distances sum below theta are
// appended to the candidates (a, b, 0, 0) for verification.
struct SweepArgs {
    int64_t n, ns;
    int64_t s_lo;          // first diagonal offset of group 0
    int64_t item_lo, item_hi;
    int64_t chunks;        // chunks per group
    int D, Dp, G, DL;      // dimensions, lanes per diagonal, diagonals per wave, dimensions per lane
    int w, d, Lc;
    int part, nparts;      // emit only pair_part(a, b, nparts) == part (nparts 1: all)
    double theta, th2, low2;   // theta, theta^2, (theta / d)^2
};
hipError_t launch_sweep(const void* x, int dtype, const double* mu, const double* isig, const SweepArgs& g,
                        Cand* cand, uint32_t cap, Counters* cnt, hipStream_t s);

}  // namespace mm
