// C ABI and host orchestration of the MOMENTI motif search on gfx950.
//
// Host responsibilities: argument checks, the memory cap on the number of
// repetitions, the seeded random projections (Philox4x32-10 + Box-Muller),
// the r estimate from device-computed sample projections, the round /
// repetition loop of Algorithm 1 with the stopping rule of Algorithm 2
// (Lemma 6.1 for the tensored index), and the exact fallback. Every step of
// the data path itself runs in the kernels of k_hash.hip and k_search.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/momenti.h"
#include "internal.h"

using namespace mm;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(MOMENTI_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
    } while (0)

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// multiply-xor round with Weyl key increments.
static void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t prod0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t prod1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)prod1;
        x3 = (uint32_t)prod0;
        x0 = y0;
        x2 = y2;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// Stream identifiers (the last counter word).
enum : uint32_t { kStreamProj = 0, kStreamOffset = 1, kStreamRVec = 2, kStreamRWin = 3 };

static inline double unit53(uint32_t hi, uint32_t lo)
{
    return (double)((((uint64_t)hi << 32) | lo) >> 11) * 0x1.0p-53;
}

static void block_at(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t stream, uint32_t o[4])
{
    const uint32_t ctr[4] = {c0, c1, c2, stream};
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    philox4x32_10(ctr, key, o);
}

static double normal_at(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t stream)
{
    uint32_t o[4];
    block_at(seed, c0, c1, c2, stream, o);
    const double u1 = 1.0 - unit53(o[0], o[1]);
    const double u2 = unit53(o[2], o[3]);
    const double rad = std::sqrt(-2.0 * std::log(u1));
    const double ang = 6.283185307179586 * u2;
    return rad * std::cos(ang);
}

static double uniform_at(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t stream)
{
    uint32_t o[4];
    block_at(seed, c0, c1, c2, stream, o);
    return unit53(o[0], o[1]);
}

// ------------------------------------------------------------------ number formats
// Round-to-nearest-even from FP64, in one step, to the MFMA input types:
// bfloat16 (8 significant bits, FP32 exponent range) and OCP FP8 E4M3
// (4 significant bits, bias 7, subnormal quantum 2^-9, largest finite 448).
static uint16_t to_bf16_bits(double v)
{
    if (v == 0.0) return std::signbit(v) ? 0x8000u : 0u;
    int e;
    std::frexp(v, &e);                              // |v| in [2^(e-1), 2^e)
    const double q = std::ldexp(1.0, e - 8);        // quantum for 8 significant bits
    const double r = std::nearbyint(v / q) * q;     // default rounding mode: nearest-even
    const float f = (float)r;                       // exact: r has <= 8 significant bits
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
}

static uint8_t to_e4m3_bits(double v)
{
    const uint8_t sgn = std::signbit(v) ? 0x80 : 0x00;
    double a = std::fabs(v);
    if (a == 0.0) return sgn;
    int e;
    std::frexp(a, &e);
    int ue = e - 1;                                 // a in [2^ue, 2^(ue+1))
    if (ue < -6) ue = -6;                           // subnormal range shares the 2^-9 quantum
    const double q = std::ldexp(1.0, ue - 3);
    double r = std::nearbyint(a / q) * q;
    if (r > 448.0) r = 448.0;                       // saturate
    if (r == 0.0) return sgn;
    std::frexp(r, &e);
    int be = e - 1 + 7;                             // biased exponent
    uint8_t bits;
    if (be <= 0) {                                  // subnormal: r = m * 2^-9
        bits = (uint8_t)std::lround(r / std::ldexp(1.0, -9));
    } else {
        const double mant = r / std::ldexp(1.0, e - 1) - 1.0;   // in [0, 1)
        bits = (uint8_t)((be << 3) | (int)std::lround(mant * 8.0));
    }
    return sgn | bits;
}

// ------------------------------------------------------------------ profiling
// Optional per-kernel timing with HIP events recorded on the plan's stream
// around each launch; folded into totals whenever the host synchronises.
enum KernelId { KI_STATS, KI_RSAMPLE, KI_PROJ, KI_HIST, KI_SCAN, KI_SCATTER, KI_PROBE, KI_FPTABLE, KI_ENUM,
                KI_VERIFY, KI_FILTER, KI_POOL, KI_ALLPAIRS, KI_SWEEP, KI_COUNT };
static const char* const kKernelNames[KI_COUNT] = {
    "stats", "rsample", "proj", "sort_hist", "sort_scan", "sort_scatter", "probe", "fptable", "enum",
    "verify", "pool_filter", "pool", "allpairs", "sweep"};

struct KTotal {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0, flops = 0.0;
};

struct Profiler {
    bool on = false;
    bool enum_only = false;   // time only the pair enumeration
    struct Pending {
        int id;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<hipEvent_t> spare;
    std::vector<Pending> pending;
    KTotal tot[KI_COUNT];
};

// ------------------------------------------------------------------ plan
// Device blocks kept for reuse by the plans of one batch worker: a freed
// block goes back here and is handed to the next request it fits (at most
// twice the size asked for), so consecutive series stop paying for hipMalloc
// and hipFree. Blocks are released when the worker ends. A plan is charged a
// block's whole capacity, and the idle blocks count against its mem_limit
// too: they are returned to the runtime before an allocation that would put
// the plan's blocks plus the idle ones over the limit.
struct BlockCache {
    std::vector<std::pair<size_t, void*>> idle;    // (capacity, block)
    std::vector<std::pair<void*, size_t>> owned;   // every block, with its capacity
    size_t idle_bytes = 0;
    bool exact = false;                            // reuse only blocks of the requested size
    void* take(size_t bytes, size_t room, size_t* cap_out)
    {
        int best = -1;
        for (int q = 0; q < (int)idle.size(); ++q) {
            const size_t c = idle[q].first;
            const bool fits = exact ? c == bytes : (c >= bytes && c <= 2 * bytes + (1u << 20));
            if (fits && c <= room && (best < 0 || c < idle[best].first)) best = q;
        }
        if (best < 0) return nullptr;
        void* b = idle[best].second;
        *cap_out = idle[best].first;
        idle_bytes -= idle[best].first;
        idle.erase(idle.begin() + best);
        return b;
    }
    size_t capacity(void* b) const
    {
        for (auto& o : owned)
            if (o.first == b) return o.second;
        return 0;
    }
    void give(void* b)
    {
        for (auto& o : owned)
            if (o.first == b) {
                idle.push_back({o.second, b});
                idle_bytes += o.second;
                return;
            }
        (void)hipFree(b);   // not ours
    }
    void drop(void* b)   // return a block in use to the runtime
    {
        for (size_t q = 0; q < owned.size(); ++q)
            if (owned[q].first == b) {
                owned.erase(owned.begin() + q);
                break;
            }
        (void)hipFree(b);
    }
    void trim()   // return idle blocks to the runtime
    {
        for (auto& b : idle) {
            for (size_t q = 0; q < owned.size(); ++q)
                if (owned[q].first == b.second) {
                    owned.erase(owned.begin() + q);
                    break;
                }
            (void)hipFree(b.second);
        }
        idle.clear();
        idle_bytes = 0;
    }
    ~BlockCache()
    {
        for (auto& o : owned) (void)hipFree(o.first);
    }
};

struct momenti_plan {
    BlockCache* cache = nullptr;   // the batch worker's blocks, or own_cache
    BlockCache own_cache;          // a plan of its own: blocks its next search reuses
    bool recycle = false;          // own_cache: a search is releasing and re-taking its buffers
    // momenti_search_noalloc: traversal buffers are carved, in order, from the
    // device's scratch area (bytes = the part used, mem_limit = its size)
    bool arena = false;
    unsigned char* arena_base = nullptr;
    // several dimensionalities at once: records per candidate (one per d) and
    // the pool state in use (NULL: the one in the status block)
    int vsets = 1;
    PoolState* ps_cur = nullptr;
    int64_t n = 0, ns = 0;
    int D = 0, w = 0, dtype = 1;
    uint64_t mem_limit = 0;
    momenti_opts o{};
    int K = 8, L = 200, m = 15, NL = 14, NR = 15, NF = 29, Cpad = 128, wpad = 0;
    double r = 0.0;
    bool hashed = false, have_stats = false;
    hipStream_t st = nullptr;
    int dev = 0;

    void* series = nullptr;
    bool own_series = false;
    double* mu = nullptr;
    double* isig = nullptr;
    void* R = nullptr;
    void* U = nullptr;
    uint32_t* H = nullptr;
    double t_hash_ms = 0.0;

    // traversal buffers
    SortBufs sb{};
    int sb_nseg = 0, sb_reps = 0;
    uint32_t* fps = nullptr;    // fingerprint rows of a batch: [rep][window][fp_words(D)]
    uint32_t* fq = nullptr;     // second-stage rows of a batch: [rep][window][fq_words(D)]
    unsigned long long* coll_part = nullptr;   // per-work-group collision counts
    int64_t coll_parts = 0;
    Cand* cand = nullptr;       // candidates of one launch batch
    VRec* vrec = nullptr;       // their verified records
    uint32_t cap = 0;
    VRec* store = nullptr;      // verified records of the current round group
    uint32_t* keep = nullptr;   // 2 * store_cap: kept indices, then step order
    uint32_t store_cap = 0;
    VRec* pools = nullptr;
    int P = 0;
    VRec* top = nullptr;
    int top_k = 0;
    unsigned char* status = nullptr;   // Counters | PoolState
    ReplayCtl* rctl = nullptr;
    Snap* snaps = nullptr;             // one per step of a round group
    VRec* snap_tops = nullptr;         // k per step
    int snap_steps = 0, snap_k = 0;
    unsigned char* host_status = nullptr;
    Snap* host_snaps = nullptr;
    // pinned host blocks the plan keeps for its next search (pinning memory
    // is slow): freed by momenti_destroy
    struct HostBlock {
        void* ptr;
        size_t cap;
        bool used;
    };
    std::vector<HostBlock> host_blocks;

    uint64_t bytes = 0, peak = 0;
    Profiler prof;

    // trace
    int64_t* tr_cand = nullptr;
    int64_t tr_cap = 0;
    int64_t* tr_count = nullptr;
    int32_t* tr_top_size = nullptr;
    int64_t* tr_top_pairs = nullptr;
    int64_t tr_steps_cap = 0;
    int32_t tr_k = 0;
};

// Device block of at least `bytes` for the plan, within its mem_limit: the
// plan is charged the block's capacity, and its blocks plus the cache's idle
// ones stay within the limit.
static void note_peak(momenti_plan* p)
{
    p->peak = std::max<uint64_t>(p->peak, p->bytes + (p->cache ? p->cache->idle_bytes : 0));
}

static int dalloc(momenti_plan* p, void** ptr, size_t bytes)
{
    *ptr = nullptr;
    if (bytes == 0) bytes = 16;
    if (p->arena) {
        // the next 256-byte aligned piece of the scratch area; nothing is
        // given back before the call ends
        const size_t need = (bytes + 255) / 256 * 256;
        if (p->bytes + need > p->mem_limit)
            return fail(MOMENTI_E_NOMEM, "scratch area exhausted: %llu + %zu > %llu bytes (momenti_search "
                        "allocates what this input needs)", (unsigned long long)p->bytes, need,
                        (unsigned long long)p->mem_limit);
        *ptr = p->arena_base + p->bytes;
        p->bytes += need;
        p->peak = std::max<uint64_t>(p->peak, p->bytes);
        return MOMENTI_OK;
    }
    if (p->bytes + bytes > p->mem_limit)
        return fail(MOMENTI_E_NOMEM, "device budget exceeded: %llu + %zu > %llu bytes",
                    (unsigned long long)p->bytes, bytes, (unsigned long long)p->mem_limit);
    size_t capb = 0;
    if (p->cache && (*ptr = p->cache->take(bytes, p->mem_limit - p->bytes, &capb)) != nullptr) {
        p->bytes += capb;
        note_peak(p);
        return MOMENTI_OK;
    }
    // a fresh block: the idle ones go back to the runtime first if, with
    // them, the plan would hold more than its limit
    if (p->cache && p->bytes + p->cache->idle_bytes + bytes > p->mem_limit) p->cache->trim();
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess && p->cache) {
        (void)hipGetLastError();
        p->cache->trim();   // idle blocks may be what is missing
        e = hipMalloc(ptr, bytes);
    }
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(MOMENTI_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    if (p->cache) p->cache->owned.push_back({*ptr, bytes});
    p->bytes += bytes;
    note_peak(p);
    return MOMENTI_OK;
}

template <typename T>
static int dalloc_t(momenti_plan* p, T** ptr, size_t bytes)
{
    void* v = nullptr;
    int rc = dalloc(p, &v, bytes);
    *ptr = (T*)v;
    return rc;
}

// Host staging buffers: pinned, except under momenti_search_noalloc (plain
// memory: no allocating HIP call there). Pinned blocks stay with the plan
// after a search and serve the next one when large enough.
static bool host_alloc(momenti_plan* p, void** ptr, size_t bytes)
{
    if (p->arena) {
        *ptr = std::malloc(bytes);
        return *ptr != nullptr;
    }
    for (auto& b : p->host_blocks)
        if (!b.used && b.cap >= bytes) {
            b.used = true;
            *ptr = b.ptr;
            return true;
        }
    const size_t cap = (bytes + 4095) / 4096 * 4096;
    if (hipHostMalloc(ptr, cap, 0) != hipSuccess) return false;
    p->host_blocks.push_back({*ptr, cap, true});
    return true;
}

static void host_free(momenti_plan* p, void* ptr)
{
    if (!ptr) return;
    if (p->arena) {
        std::free(ptr);
        return;
    }
    for (auto& b : p->host_blocks)
        if (b.ptr == ptr) {
            b.used = false;
            return;
        }
    (void)hipHostFree(ptr);
}

static void dfree(momenti_plan* p, void* ptr, size_t bytes)
{
    if (!ptr || p->arena) return;   // scratch pieces are not given back one by one
    const size_t capb = p->cache->capacity(ptr);
    if (capb) bytes = capb;
    if (p->cache != &p->own_cache || p->recycle)
        p->cache->give(ptr);   // the plan's stream keeps later uses in order
    else
        p->cache->drop(ptr);
    if (bytes == 0) bytes = 16;
    p->bytes -= std::min<uint64_t>(p->bytes, bytes);
}

// Host <-> device copy ordered on the plan's stream (which may be a
// non-blocking stream of a batch worker), complete on return.
static hipError_t copy_sync(momenti_plan* p, void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, p->st);
    if (e == hipSuccess) e = hipStreamSynchronize(p->st);
    return e;
}

static hipEvent_t prof_event(momenti_plan* p)
{
    if (!p->prof.spare.empty()) {
        hipEvent_t e = p->prof.spare.back();
        p->prof.spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Launch through `fn`, bracketed by events when profiling. Returns the index
// of the pending record (or -1), so that work sizes known only later can be
// filled in with prof_set.
template <class F>
static hipError_t timed(momenti_plan* p, int id, double bytes, double flops, F&& fn, int* slot = nullptr)
{
    if (slot) *slot = -1;
    if (!p->prof.on || (p->prof.enum_only && id != KI_ENUM)) return fn();
    hipEvent_t a = prof_event(p), b = prof_event(p);
    (void)hipEventRecord(a, p->st);
    hipError_t e = fn();
    (void)hipEventRecord(b, p->st);
    if (slot) *slot = (int)p->prof.pending.size();
    p->prof.pending.push_back({id, a, b, bytes, flops});
    return e;
}

static void prof_set(momenti_plan* p, int slot, double bytes, double flops)
{
    if (slot < 0 || slot >= (int)p->prof.pending.size()) return;
    p->prof.pending[slot].bytes = bytes;
    p->prof.pending[slot].flops = flops;
}

// Fold completed launches into the totals (call after a stream synchronisation).
static void prof_flush(momenti_plan* p)
{
    for (auto& q : p->prof.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
            KTotal& t = p->prof.tot[q.id];
            t.launches += 1;
            t.ms += ms;
            t.bytes += q.bytes;
            t.flops += q.flops;
        }
        p->prof.spare.push_back(q.a);
        p->prof.spare.push_back(q.b);
    }
    p->prof.pending.clear();
}

static int64_t ceil_sqrt_i(int64_t v)
{
    int64_t m = (int64_t)std::sqrt((double)v);
    while (m * m < v) ++m;
    while (m > 1 && (m - 1) * (m - 1) >= v) --m;
    return m;
}

static void tensor_shape(int L, int* m, int* nl, int* nr)
{
    *m = (int)ceil_sqrt_i(L);
    *nl = (L + *m - 1) / *m;
    *nr = std::min(L, *m);
}

// Memory cap: the largest L' <= L_max whose index fits next to the series,
// the statistics and the fixed traversal reserve (index size O(K L D n)).
static int cap_repetitions(int64_t n, int D, int w, int L_max, int elem, uint64_t limit)
{
    const int64_t ns = n - w + 1;
    const int64_t fixed = n * D * elem + 16 * ns * D + 32 * ns * D + ((int64_t)64 << 20);
    for (int L = L_max; L >= 1; --L) {
        int m, nl, nr;
        tensor_shape(L, &m, &nl, &nr);
        const int64_t idx = 4 * ns * (int64_t)D * (nl + nr);
        if ((uint64_t)(fixed + idx) <= limit) return L;
    }
    return 0;
}

static size_t series_bytes(const momenti_plan* p) { return (size_t)p->n * p->D * (p->dtype == MOMENTI_F64 ? 8 : 4); }
static size_t proj_elem(int proj)
{
    return proj == MOMENTI_PROJ_F64 ? 8 : proj == MOMENTI_PROJ_F32 ? 4 : proj == MOMENTI_PROJ_BF16 ? 2 : 1;
}
static size_t offs_elem(int proj) { return proj == MOMENTI_PROJ_F64 ? 8 : 4; }

static void release_search(momenti_plan* p)
{
    for (int q = 0; q < 2; ++q) {
        dfree(p, p->sb.keys[q], (size_t)p->sb_nseg * p->ns * 8);
        dfree(p, p->sb.idx[q], (size_t)p->sb_nseg * p->ns * 4);
        p->sb.keys[q] = nullptr;
        p->sb.idx[q] = nullptr;
    }
    dfree(p, p->sb.hist, (size_t)p->sb_nseg * 256 * p->sb.tiles * 4);
    p->sb.hist = nullptr;
    dfree(p, p->sb.units, (size_t)p->sb.ucap * sizeof(RunRec));
    p->sb.units = nullptr;
    p->sb.ucap = 0;
    dfree(p, p->fps, (size_t)p->sb_reps * fp_words(p->D) * p->ns * 4);
    dfree(p, p->fq, (size_t)p->sb_reps * fq_words(p->D) * p->ns * 4);
    p->fps = nullptr;
    p->fq = nullptr;
    p->sb_nseg = 0;
    p->sb_reps = 0;
    dfree(p, p->cand, (size_t)p->cap * sizeof(Cand));
    dfree(p, p->vrec, (size_t)p->cap * sizeof(VRec));
    p->cand = nullptr; p->vrec = nullptr; p->cap = 0;
    dfree(p, p->coll_part, (size_t)p->coll_parts * 24);
    p->coll_part = nullptr; p->coll_parts = 0;
    dfree(p, p->store, (size_t)p->store_cap * sizeof(VRec));
    dfree(p, p->keep, (size_t)p->store_cap * 8);
    p->store = nullptr; p->keep = nullptr; p->store_cap = 0;
    dfree(p, p->pools, (size_t)2 * p->P * sizeof(VRec));
    p->pools = nullptr; p->P = 0;
    dfree(p, p->top, (size_t)p->top_k * sizeof(VRec));
    p->top = nullptr; p->top_k = 0;
    dfree(p, p->status, 4096);
    p->status = nullptr;
    dfree(p, p->rctl, sizeof(ReplayCtl));
    p->rctl = nullptr;
    dfree(p, p->snaps, (size_t)p->snap_steps * sizeof(Snap));
    dfree(p, p->snap_tops, (size_t)p->snap_steps * p->snap_k * sizeof(VRec));
    p->snaps = nullptr; p->snap_tops = nullptr; p->snap_steps = 0; p->snap_k = 0;
    host_free(p, p->host_status);
    p->host_status = nullptr;
    host_free(p, p->host_snaps);
    p->host_snaps = nullptr;
}

// ------------------------------------------------------------------ ABI
extern "C" {

void momenti_default_opts(momenti_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->seed = 0x5EED;
    o->K = 8;
    o->L = 200;
    o->r = 0.0;
    o->r_scale = 1.0;
    o->max_pairs = 0.0;
    o->merge_pairs = 8.0;
    o->proj = MOMENTI_PROJ_F32;
    o->stop_rule = MOMENTI_STOP_TENSOR;
}

const char* momenti_last_error(void) { return g_err.c_str(); }

void momenti_destroy(momenti_plan* p)
{
    if (!p) return;
    if (p->st) (void)hipStreamSynchronize(p->st); else (void)hipDeviceSynchronize();
    prof_flush(p);
    for (hipEvent_t e : p->prof.spare) (void)hipEventDestroy(e);
    p->prof.spare.clear();
    release_search(p);
    for (auto& b : p->host_blocks) (void)hipHostFree(b.ptr);
    p->host_blocks.clear();
    if (p->own_series) dfree(p, p->series, series_bytes(p));
    dfree(p, p->mu, (size_t)p->D * p->ns * 8);
    dfree(p, p->isig, (size_t)p->D * p->ns * 8);
    dfree(p, p->R, (size_t)p->D * p->wpad * p->Cpad * proj_elem(p->o.proj));
    dfree(p, p->U, (size_t)p->D * p->Cpad * offs_elem(p->o.proj));
    dfree(p, p->H, (size_t)p->D * p->NF * p->ns * 4);
    delete p;
}

static int prepare_impl(momenti_plan** out, int64_t n, int32_t D, int32_t w, int32_t dtype,
                        uint64_t mem_limit, const momenti_opts* opts, BlockCache* cache);

int momenti_prepare(momenti_plan** out, int64_t n, int32_t D, int32_t w, int32_t dtype,
                    uint64_t mem_limit, const momenti_opts* opts)
{
    return prepare_impl(out, n, D, w, dtype, mem_limit, opts, nullptr);
}

static int prepare_impl(momenti_plan** out, int64_t n, int32_t D, int32_t w, int32_t dtype,
                        uint64_t mem_limit, const momenti_opts* opts, BlockCache* cache)
{
    g_err.clear();
    if (!out) return fail(MOMENTI_E_ARG, "out is NULL");
    *out = nullptr;
    momenti_opts o;
    if (opts) o = *opts; else momenti_default_opts(&o);
    if (D < 1 || D > kMaxD) return fail(MOMENTI_E_ARG, "D=%d outside [1, %d]", D, kMaxD);
    if (w < 4 || w > kMaxW) return fail(MOMENTI_E_ARG, "w=%d outside [4, %d]", w, kMaxW);
    if (n < (int64_t)w + 1) return fail(MOMENTI_E_ARG, "n=%lld shorter than w+1", (long long)n);
    if (n - w + 1 > ((int64_t)1 << 31)) return fail(MOMENTI_E_ARG, "too many windows");
    if (dtype != MOMENTI_F64 && dtype != MOMENTI_F32) return fail(MOMENTI_E_ARG, "bad dtype %d", dtype);
    if (o.K < 2 || o.K > 8 || (o.K & 1)) return fail(MOMENTI_E_ARG, "K=%d must be even in [2, 8]", o.K);
    if (o.L < 1 || o.L > kMaxL) return fail(MOMENTI_E_ARG, "L=%d outside [1, %d]", o.L, kMaxL);
    if (o.proj < MOMENTI_PROJ_F64 || o.proj > MOMENTI_PROJ_FP8)
        return fail(MOMENTI_E_ARG, "projection precision %d not available", o.proj);
    if (o.stop_rule < MOMENTI_STOP_TENSOR || o.stop_rule > MOMENTI_STOP_RIGOROUS)
        return fail(MOMENTI_E_ARG, "bad stop rule %d", o.stop_rule);
    if (o.delta_mode != MOMENTI_DELTA_PER_MOTIF && o.delta_mode != MOMENTI_DELTA_JOINT)
        return fail(MOMENTI_E_ARG, "bad delta mode %d", o.delta_mode);
    if (!std::isfinite(o.max_ms)) return fail(MOMENTI_E_ARG, "max_ms must be finite");
    if (!std::isfinite(o.r_scale) || !std::isfinite(o.max_pairs) || !std::isfinite(o.r) ||
        !std::isfinite(o.merge_pairs))
        return fail(MOMENTI_E_ARG, "r, r_scale, merge_pairs and max_pairs must be finite");
    if (o.pool_size < 0 || o.batch_reps < 0) return fail(MOMENTI_E_ARG, "negative pool/batch size");

    const int elem = dtype == MOMENTI_F64 ? 8 : 4;
    const int L = cap_repetitions(n, D, w, o.L, elem, mem_limit);
    if (L < 1) return fail(MOMENTI_E_NOMEM, "mem_limit %llu below the one-repetition index",
                           (unsigned long long)mem_limit);

    momenti_plan* p = new (std::nothrow) momenti_plan();
    if (!p) return fail(MOMENTI_E_NOMEM, "host allocation failed");
    p->cache = cache ? cache : &p->own_cache;
    p->own_cache.exact = true;
    p->n = n; p->ns = n - w + 1; p->D = D; p->w = w; p->dtype = dtype; p->mem_limit = mem_limit;
    p->o = o; p->K = o.K; p->L = L;
    tensor_shape(L, &p->m, &p->NL, &p->NR);
    p->NF = p->NL + p->NR;
    const int C = 4 * p->NF;
    p->Cpad = ((C + 31) / 32) * 32;
    p->wpad = ((w + 63) / 64) * 64;
    if (o.proj == MOMENTI_PROJ_BF16 || o.proj == MOMENTI_PROJ_FP8) {
        // the projection's work-group holds four shifted copies of its series
        // tile and two chunks of projection rows in LDS
        const int proj = o.proj == MOMENTI_PROJ_BF16 ? 2 : 3;
        if (lowp_lds_bytes(proj, p->Cpad, p->wpad) > kMaxLdsBytes) {
            int wmax = p->wpad;
            while (wmax > 64 && lowp_lds_bytes(proj, p->Cpad, wmax) > kMaxLdsBytes) wmax -= 64;
            const int C0 = p->Cpad;
            delete p;
            return fail(MOMENTI_E_ARG, "w=%d too long for the %s projection with %d hash columns (at most %d)", w,
                        proj == 2 ? "BF16" : "FP8", C0, wmax);
        }
    }
    p->st = (hipStream_t)o.stream;
    p->prof.on = o.profile != 0;
    p->prof.enum_only = o.profile == 2;
    if (hipGetDevice(&p->dev) != hipSuccess) {
        delete p;
        return fail(MOMENTI_E_DEVICE, "no HIP device");
    }

    // random projections of Eq. drp: R[f][t][c] ~ N(0,1), U[f][c] ~ U[0,1)
    const size_t pe = proj_elem(o.proj);
    std::vector<double> R((size_t)D * p->wpad * p->Cpad, 0.0), U((size_t)D * p->Cpad, 0.0);
    for (int f = 0; f < D; ++f) {
        for (int t = 0; t < w; ++t)
            for (int c = 0; c < C; ++c)
                R[((size_t)f * p->wpad + t) * p->Cpad + c] =
                    normal_at(o.seed, (uint32_t)t, (uint32_t)c, (uint32_t)f, kStreamProj);
        for (int c = 0; c < C; ++c)
            U[(size_t)f * p->Cpad + c] = uniform_at(o.seed, (uint32_t)c, (uint32_t)f, 0u, kStreamOffset);
    }
    int rc;
    if ((rc = dalloc(p, &p->R, R.size() * pe)) || (rc = dalloc(p, &p->U, U.size() * offs_elem(o.proj))) ||
        (rc = dalloc_t(p, &p->mu, (size_t)D * p->ns * 8)) ||
        (rc = dalloc_t(p, &p->isig, (size_t)D * p->ns * 8)) ||
        (rc = dalloc_t(p, &p->H, (size_t)D * p->NF * p->ns * 4))) {
        momenti_destroy(p);
        return rc;
    }
    hipError_t e;
    if (o.proj == MOMENTI_PROJ_F64) {
        e = copy_sync(p, p->R, R.data(), R.size() * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = copy_sync(p, p->U, U.data(), U.size() * 8, hipMemcpyHostToDevice);
    } else if (o.proj == MOMENTI_PROJ_F32) {
        std::vector<float> Rf(R.begin(), R.end()), Uf(U.begin(), U.end());
        e = copy_sync(p, p->R, Rf.data(), Rf.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = copy_sync(p, p->U, Uf.data(), Uf.size() * 4, hipMemcpyHostToDevice);
    } else {
        // low precision: column-major [f][c][t] so that a lane loads consecutive t
        std::vector<float> Uf(U.begin(), U.end());
        const size_t cnt = (size_t)D * p->Cpad * p->wpad;
        if (o.proj == MOMENTI_PROJ_BF16) {
            std::vector<uint16_t> Rq(cnt, 0);
            for (int f = 0; f < D; ++f)
                for (int t = 0; t < p->wpad; ++t)
                    for (int c = 0; c < p->Cpad; ++c)
                        Rq[((size_t)f * p->Cpad + c) * p->wpad + t] =
                            to_bf16_bits(R[((size_t)f * p->wpad + t) * p->Cpad + c]);
            e = copy_sync(p, p->R, Rq.data(), cnt * 2, hipMemcpyHostToDevice);
        } else {
            std::vector<uint8_t> Rq(cnt, 0);
            for (int f = 0; f < D; ++f)
                for (int t = 0; t < p->wpad; ++t)
                    for (int c = 0; c < p->Cpad; ++c)
                        Rq[((size_t)f * p->Cpad + c) * p->wpad + t] =
                            to_e4m3_bits(R[((size_t)f * p->wpad + t) * p->Cpad + c]);
            e = copy_sync(p, p->R, Rq.data(), cnt, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = copy_sync(p, p->U, Uf.data(), Uf.size() * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        momenti_destroy(p);
        return fail(MOMENTI_E_DEVICE, "upload of projections failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return MOMENTI_OK;
}

int momenti_hash(momenti_plan* p, const void* series)
{
    g_err.clear();
    if (!p) return fail(MOMENTI_E_ARG, "plan is NULL");
    if (!series) return fail(MOMENTI_E_ARG, "series is NULL");
    const size_t sbytes = series_bytes(p);
    if (p->o.series_on_device) {
        if (p->own_series) {
            dfree(p, p->series, sbytes);
            p->own_series = false;
        }
        p->series = const_cast<void*>(series);
    } else {
        if (!p->own_series) {
            p->series = nullptr;
            int rc = dalloc(p, &p->series, sbytes);
            if (rc) return rc;
            p->own_series = true;
        }
        HIP_OK(hipMemcpyAsync(p->series, series, sbytes, hipMemcpyHostToDevice, p->st));
    }
    // a new series replaces the index: until it is built the plan has none
    p->hashed = false;
    p->have_stats = false;
    {
        // every value must be finite (the definitions of section 3.1 are over
        // real values); the statistics buffer's first word holds the answer
        // before the statistics overwrite it
        unsigned long long first = ~0ull;
        unsigned long long* d_first = reinterpret_cast<unsigned long long*>(p->mu);
        HIP_OK(hipMemcpyAsync(d_first, &first, sizeof first, hipMemcpyHostToDevice, p->st));
        HIP_OK(launch_first_nonfinite(p->series, p->dtype, p->n * p->D, d_first, p->st));
        HIP_OK(hipMemcpyAsync(&first, d_first, sizeof first, hipMemcpyDeviceToHost, p->st));
        HIP_OK(hipStreamSynchronize(p->st));
        if (first != ~0ull)
            return fail(MOMENTI_E_ARG, "series[%lld][%lld] is not finite (NaN or infinity)",
                        (long long)(first / (unsigned long long)p->n), (long long)(first % (unsigned long long)p->n));
    }
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, p->st));
    const double elem = p->dtype == MOMENTI_F64 ? 8.0 : 4.0;
    HIP_OK(timed(p, KI_STATS, (double)p->n * p->D * elem + 16.0 * p->ns * p->D, 0.0, [&] {
        return launch_stats(p->series, p->dtype, p->n, p->ns, p->D, p->w, p->mu, p->isig, p->st);
    }));

    // r (section 6.1): projections of sampled z-normalised windows on 8
    // Gaussian vectors, split into 256 equal buckets.
    double r = p->o.r;
    if (!(r > 0.0)) {
        const int nvec = 8;
        const int S = (int)std::min<int64_t>(p->ns, 4096);
        std::vector<int64_t> win((size_t)p->D * S);
        for (int f = 0; f < p->D; ++f)
            for (int q = 0; q < S; ++q) {
                const double u = uniform_at(p->o.seed, (uint32_t)q, (uint32_t)f, 0u, kStreamRWin);
                int64_t a = (int64_t)std::floor(u * (double)p->ns);
                win[(size_t)f * S + q] = std::min<int64_t>(a, p->ns - 1);
            }
        std::vector<double> vec((size_t)nvec * p->w);
        for (int v = 0; v < nvec; ++v)
            for (int t = 0; t < p->w; ++t)
                vec[(size_t)v * p->w + t] = normal_at(p->o.seed, (uint32_t)t, (uint32_t)v, 0u, kStreamRVec);
        int64_t* d_win = nullptr;
        double *d_vec = nullptr, *d_dots = nullptr;
        const size_t nd = (size_t)p->D * S * nvec;
        int rc;
        if ((rc = dalloc_t(p, &d_win, win.size() * 8)) || (rc = dalloc_t(p, &d_vec, vec.size() * 8)) ||
            (rc = dalloc_t(p, &d_dots, nd * 8))) {
            dfree(p, d_win, win.size() * 8);
            dfree(p, d_vec, vec.size() * 8);
            return rc;
        }
        std::vector<double> dots(nd);
        hipError_t e = hipMemcpyAsync(d_win, win.data(), win.size() * 8, hipMemcpyHostToDevice, p->st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_vec, vec.data(), vec.size() * 8, hipMemcpyHostToDevice, p->st);
        if (e == hipSuccess)
            e = timed(p, KI_RSAMPLE, (double)p->D * S * p->w * elem, 2.0 * p->D * S * p->w * (nvec + 2), [&] {
                return launch_rsample(p->series, p->dtype, p->n, p->D, p->w, d_win, S, d_vec, nvec, d_dots, p->st);
            });
        if (e == hipSuccess) e = hipMemcpyAsync(dots.data(), d_dots, nd * 8, hipMemcpyDeviceToHost, p->st);
        if (e == hipSuccess) e = hipStreamSynchronize(p->st);
        dfree(p, d_win, win.size() * 8);
        dfree(p, d_vec, vec.size() * 8);
        dfree(p, d_dots, nd * 8);
        if (e != hipSuccess) return fail(MOMENTI_E_DEVICE, "r estimate failed: %s", hipGetErrorString(e));
        double lo = INFINITY, hi = -INFINITY;
        for (double v : dots) {
            lo = std::min(lo, v);
            hi = std::max(hi, v);
        }
        r = (hi - lo) / 256.0;
        if (!(r > 0.0) || !std::isfinite(r)) r = 1.0;
        if (p->o.r_scale > 0.0) r *= p->o.r_scale;
    }
    p->r = r;
    {
        // useful work: K/2 positions of every half-function, 2 w flops each
        const double cols = (double)(p->K / 2) * p->NF;
        const double flops = 2.0 * p->w * cols * (double)p->ns * p->D;
        const double bytes = (double)p->n * p->D * elem + 16.0 * p->ns * p->D + 4.0 * p->NF * p->ns * p->D;
        HIP_OK(timed(p, KI_PROJ, bytes, flops, [&] {
            return launch_proj(p->o.proj, p->series, p->dtype, p->n, p->ns, p->D, p->w, p->mu, p->isig,
                               p->R, p->U, p->Cpad, p->wpad, p->NF, p->K, 1.0 / r, p->H, p->st);
        }));
    }
    HIP_OK(hipEventRecord(e1, p->st));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    prof_flush(p);
    p->t_hash_ms = ms;
    p->hashed = true;
    p->have_stats = true;
    return MOMENTI_OK;
}

int momenti_get_params(const momenti_plan* p, double* r, int32_t* L_used, int32_t* n_left, int32_t* n_right)
{
    if (!p) return fail(MOMENTI_E_ARG, "plan is NULL");
    if (r) *r = p->r;
    if (L_used) *L_used = p->L;
    if (n_left) *n_left = p->NL;
    if (n_right) *n_right = p->NR;
    return MOMENTI_OK;
}

int momenti_get_stats(momenti_plan* p, double* mu, double* inv_sigma, size_t count)
{
    if (!p) return fail(MOMENTI_E_ARG, "plan is NULL");
    if (!p->have_stats) return fail(MOMENTI_E_STATE, "no statistics yet");
    if (count != (size_t)p->D * p->ns) return fail(MOMENTI_E_ARG, "count must be D * n_s");
    HIP_OK(hipStreamSynchronize(p->st));
    if (mu) HIP_OK(copy_sync(p, mu, p->mu, count * 8, hipMemcpyDeviceToHost));
    if (inv_sigma) HIP_OK(copy_sync(p, inv_sigma, p->isig, count * 8, hipMemcpyDeviceToHost));
    return MOMENTI_OK;
}

int momenti_get_hashes(momenti_plan* p, uint32_t* dst, size_t count)
{
    if (!p || !dst) return fail(MOMENTI_E_ARG, "NULL argument");
    if (!p->hashed) return fail(MOMENTI_E_STATE, "no index yet");
    if (count != (size_t)p->D * p->NF * p->ns) return fail(MOMENTI_E_ARG, "count must be D * NF * n_s");
    HIP_OK(hipStreamSynchronize(p->st));
    HIP_OK(copy_sync(p, dst, p->H, count * 4, hipMemcpyDeviceToHost));
    return MOMENTI_OK;
}

int momenti_get_hash_words(momenti_plan* p, int32_t f, int64_t a0, int64_t count, uint32_t* dst)
{
    if (!p || !dst) return fail(MOMENTI_E_ARG, "NULL argument");
    if (!p->hashed) return fail(MOMENTI_E_STATE, "no index yet");
    if (f < 0 || f >= p->D || a0 < 0 || count < 0 || a0 + count > p->ns)
        return fail(MOMENTI_E_ARG, "dimension %d, windows [%lld, %lld) outside the index", f, (long long)a0,
                    (long long)(a0 + count));
    if (count == 0) return MOMENTI_OK;
    HIP_OK(hipStreamSynchronize(p->st));
    // rows of the dimension's half-functions, count words each
    HIP_OK(hipMemcpy2DAsync(dst, (size_t)count * 4, p->H + ((int64_t)f * p->NF) * p->ns + a0, (size_t)p->ns * 4,
                            (size_t)count * 4, (size_t)p->NF, hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    return MOMENTI_OK;
}

int momenti_set_hashes(momenti_plan* p, const uint32_t* src, size_t count)
{
    if (!p || !src) return fail(MOMENTI_E_ARG, "NULL argument");
    if (!p->have_stats) return fail(MOMENTI_E_STATE, "momenti_hash must run once first");
    if (count != (size_t)p->D * p->NF * p->ns) return fail(MOMENTI_E_ARG, "count must be D * NF * n_s");
    HIP_OK(hipStreamSynchronize(p->st));
    HIP_OK(copy_sync(p, p->H, src, count * 4, hipMemcpyHostToDevice));
    p->hashed = true;
    return MOMENTI_OK;
}

int momenti_get_profile(momenti_plan* p, momenti_kprof* out, int32_t cap, int32_t* n, int32_t clear)
{
    if (!p || !n) return fail(MOMENTI_E_ARG, "NULL argument");
    HIP_OK(p->st ? hipStreamSynchronize(p->st) : hipDeviceSynchronize());
    prof_flush(p);
    *n = KI_COUNT;
    for (int q = 0; q < KI_COUNT && q < cap && out; ++q) {
        std::memset(&out[q], 0, sizeof out[q]);
        std::snprintf(out[q].name, sizeof out[q].name, "%s", kKernelNames[q]);
        out[q].launches = p->prof.tot[q].launches;
        out[q].ms = p->prof.tot[q].ms;
        out[q].bytes = p->prof.tot[q].bytes;
        out[q].flops = p->prof.tot[q].flops;
    }
    if (clear)
        for (auto& t : p->prof.tot) t = KTotal();
    return MOMENTI_OK;
}

int momenti_set_profile(momenti_plan* p, int32_t mode)
{
    if (!p) return fail(MOMENTI_E_ARG, "plan is NULL");
    if (mode < 0 || mode > 2) return fail(MOMENTI_E_ARG, "profile mode %d outside [0, 2]", mode);
    p->prof.on = mode != 0;
    p->prof.enum_only = mode == 2;
    return MOMENTI_OK;
}

int momenti_set_trace(momenti_plan* p, int64_t* cand, int64_t cand_cap, int64_t* cand_count,
                      int32_t* top_size, int64_t* top_pairs, int64_t steps_cap, int32_t k_cap)
{
    if (!p) return fail(MOMENTI_E_ARG, "plan is NULL");
    p->tr_cand = cand;
    p->tr_cap = cand_cap;
    p->tr_count = cand_count;
    p->tr_top_size = top_size;
    p->tr_top_pairs = top_pairs;
    p->tr_steps_cap = steps_cap;
    p->tr_k = k_cap;
    return MOMENTI_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ stopping rule
// Eq. eucl-collision-probability, P(R) = erf(t / sqrt 2) - 2 / (sqrt(2 pi) t) (1 - e^{-t^2/2}),
// t = r / R (1 - 2 Phi(-t) = erf(t / sqrt 2)), with P(0) = 1.
static double collision_probability(double R, double r)
{
    if (!(R > 0.0)) return 1.0;
    const double t = r / R;
    return std::erf(t / std::sqrt(2.0)) + 2.0 / (std::sqrt(2.0 * M_PI) * t) * std::expm1(-0.5 * t * t);
}

// log of (1 - p^c)^e, with x^0 = 1 (also for x = 0). Under the TENSOR rule a
// half that contributes no symbol (c = 0, round 1) gives no collision chance
// of its own and the factor 1; printed literally it is (1 - p^0)^e = 0.
static double log_term(double logp, int c, int64_t e, bool empty_half_is_one = false)
{
    if (e == 0) return 0.0;
    if (c == 0 && empty_half_is_one) return 0.0;
    const double pc = std::exp((double)c * logp);   // p^c (p^0 = 1)
    if (pc >= 1.0) return -INFINITY;
    return (double)e * std::log1p(-pc);
}

// RIGOROUS rule: the failure probability of the tensored index with every
// half-function collapsed to a geometric collision depth (P(depth >= s) =
// p^s, each symbol colliding independently with probability p). Repetition
// j pairs left function j div m with right function j mod m; at prefix length
// i' it collides when the left depth reaches ceil(i'/2) and the right depth
// floor(i'/2). Failure after J repetitions of round i: none of repetitions
// 0 .. J-1 collides at i and (below round K) none of J .. L-1 at i + 1. Given
// which right functions reach depth floor(i/2) (and floor((i+1)/2)), the left
// functions decide independently, row by row; the right functions are
// summarised per column range between the row boundaries.
static double rigorous_fail(double p, int i, int J, int K, int L, int m)
{
    const int nl = (L + m - 1) / m, tail = L - (nl - 1) * m;   // rows; length of the last row
    const bool next = i < K;
    const double reach_b = std::pow(p, i / 2), reach_b1 = next ? std::pow(p, (i + 1) / 2) : 0.0;
    const double below_a = 1.0 - std::pow(p, (i + 1) / 2), below_a1 = 1.0 - std::pow(p, (i + 2) / 2);
    const int rows_i = J / m, cols_i = J % m;   // rows wholly at prefix i; prefix-i columns of the next row
    auto row_len = [&](int l) { return l == nl - 1 ? tail : m; };
    int edge[5] = {0, cols_i, tail, m, rows_i < nl ? row_len(rows_i) : 0};
    std::sort(edge, edge + 5);
    int lo[4], len[4], ns = 0;
    for (int u = 0; u + 1 < 5; ++u)
        if (edge[u + 1] > edge[u]) { lo[ns] = edge[u]; len[ns] = edge[u + 1] - edge[u]; ++ns; }
    double total = 0.0;
    int state[4] = {0, 0, 0, 0};   // per range: 0 none reaches b; 1 some reach b, none b'; 2 some reach b'
    for (;;) {
        double pr = 1.0;
        for (int u = 0; u < ns && pr > 0.0; ++u) {
            const double none_b = std::pow(1.0 - reach_b, len[u]), none_b1 = std::pow(1.0 - reach_b1, len[u]);
            pr *= state[u] == 0 ? none_b : state[u] == 1 ? none_b1 - none_b : 1.0 - none_b1;
        }
        if (pr > 0.0) {
            for (int l = 0; l < nl; ++l) {
                const int n = row_len(l);
                const int xi = l < rows_i ? n : (l == rows_i ? std::min(cols_i, n) : 0);   // [0, xi) at prefix i
                bool hit_i = false, hit_i1 = false;
                for (int u = 0; u < ns; ++u) {
                    if (lo[u] < xi && state[u] >= 1) hit_i = true;
                    if (next && lo[u] >= xi && lo[u] < n && state[u] == 2) hit_i1 = true;
                }
                pr *= hit_i ? below_a : hit_i1 ? below_a1 : 1.0;
            }
            total += pr;
        }
        int u = 0;
        while (u < ns && ++state[u] == 3) state[u++] = 0;
        if (u == ns) break;
    }
    return total;
}

// The stopping rule's bound on having never seen, in >= d dimensions, a pair
// at distance dist_max after J repetitions of round i (natural log; -inf when
// 0). TENSOR: Lemma 6.1; LEMMA52: Lemma 5.2; RIGOROUS: rigorous_fail.
static double log_fail(double dist_max, double r, int d, int i, int J, int K, int L, int m, int rule)
{
    const double P = collision_probability(dist_max, r);
    if (!(P > 0.0)) return 0.0;
    const double logp = (double)d * std::log(P);   // p = P^d
    if (rule == MOMENTI_STOP_RIGOROUS) {
        const double v = rigorous_fail(std::exp(logp), i, J, K, L, m);
        return v > 0.0 ? std::log(v) : -INFINITY;
    }
    double lf;
    if (rule == MOMENTI_STOP_LEMMA52) {
        lf = log_term(logp, i, J);
        if (i < K) lf += log_term(logp, i + 1, L - J);
    } else {
        const bool e1 = rule == MOMENTI_STOP_TENSOR;
        lf = log_term(logp, (i + 1) / 2, J / m, e1) + log_term(logp, i / 2, J % m, e1);
        if (i < K) {
            const int J2 = L - J;
            lf += log_term(logp, (i + 2) / 2, J2 / m, e1) + log_term(logp, (i + 1) / 2, J2 % m, e1);
        }
    }
    return lf;
}

// Algorithm 2: stop when the bound on never having seen a pair at the k-th
// motif's dist_max is at most delta.
static bool stop_holds(double dist_max, double r, int d, int i, int J, int K, int L, int m, int rule,
                       double delta)
{
    return log_fail(dist_max, r, d, i, J, K, L, m, rule) <= std::log(delta);
}

// ------------------------------------------------------------------ search
static Counters* st_counters(momenti_plan* p) { return (Counters*)p->status; }
static PoolState* st_pool(momenti_plan* p) { return p->ps_cur ? p->ps_cur : (PoolState*)(p->status + 64); }

// double-buffered keys and indices and digit histograms of reps * Ds
// segments, and the two fingerprint rows of reps repetitions
static size_t sort_bytes(int64_t reps, int64_t Ds, int64_t D, int64_t ns, int64_t tiles)
{
    return (size_t)(reps * Ds) * ns * (8 + 8 + 4 + 4) + (size_t)(reps * Ds) * 256 * tiles * 4 +
           (size_t)reps * ns * 4 * (fp_words((int)D) + fq_words((int)D)) +
           (size_t)units_bound(reps * Ds, ns) * sizeof(RunRec);
}
static size_t cand_bytes(uint32_t cap, int vsets = 1) { return (size_t)cap * (sizeof(Cand) + vsets * sizeof(VRec)); }
static size_t store_bytes(uint32_t cap) { return (size_t)cap * (sizeof(VRec) + 8); }

static int alloc_sort(momenti_plan* p, int reps, int Ds)
{
    const int64_t tiles = (p->ns + kSortTile - 1) / kSortTile;
    const int nseg = reps * Ds;
    int rc;
    p->sb.tiles = tiles;
    p->sb_nseg = nseg;
    p->sb_reps = reps;
    for (int q = 0; q < 2; ++q) {
        if ((rc = dalloc(p, &p->sb.keys[q], (size_t)nseg * p->ns * 8))) return rc;
        if ((rc = dalloc_t(p, &p->sb.idx[q], (size_t)nseg * p->ns * 4))) return rc;
    }
    if ((rc = dalloc_t(p, &p->sb.hist, (size_t)nseg * 256 * tiles * 4))) return rc;
    const int64_t ucap = units_bound(nseg, p->ns);
    if (ucap > 0xFFFFFFFFll) return fail(MOMENTI_E_UNSUPPORTED, "too many segment elements per batch");
    if ((rc = dalloc_t(p, &p->sb.units, (size_t)ucap * sizeof(RunRec)))) return rc;
    p->sb.ucap = (uint32_t)ucap;
    if ((rc = dalloc_t(p, &p->fps, (size_t)reps * fp_words(p->D) * p->ns * 4))) return rc;
    if ((rc = dalloc_t(p, &p->fq, (size_t)reps * fq_words(p->D) * p->ns * 4))) return rc;
    return MOMENTI_OK;
}

static int alloc_cand(momenti_plan* p, uint32_t cap)
{
    dfree(p, p->cand, (size_t)p->cap * sizeof(Cand));
    dfree(p, p->vrec, (size_t)p->cap * p->vsets * sizeof(VRec));
    p->cand = nullptr; p->vrec = nullptr; p->cap = 0;
    int rc;
    if ((rc = dalloc_t(p, &p->cand, (size_t)cap * sizeof(Cand)))) return rc;
    if ((rc = dalloc_t(p, &p->vrec, (size_t)cap * p->vsets * sizeof(VRec)))) return rc;
    p->cap = cap;
    return MOMENTI_OK;
}

// Grow the group store to hold at least `need` records, keeping `used` of them.
static int grow_store(momenti_plan* p, uint32_t need, uint32_t used)
{
    if (need <= p->store_cap) return MOMENTI_OK;
    uint32_t cap = std::max<uint32_t>(p->store_cap, 1u << 16);
    while (cap < need) cap = cap >= (1u << 31) ? need : cap * 2;
    VRec* ns = nullptr;
    uint32_t* nk = nullptr;
    int rc;
    if ((rc = dalloc_t(p, &ns, (size_t)cap * sizeof(VRec)))) return rc;
    if ((rc = dalloc_t(p, &nk, (size_t)cap * 8))) {
        dfree(p, ns, (size_t)cap * sizeof(VRec));
        return rc;
    }
    if (used) HIP_OK(hipMemcpyAsync(ns, p->store, (size_t)used * sizeof(VRec), hipMemcpyDeviceToDevice, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    dfree(p, p->store, (size_t)p->store_cap * sizeof(VRec));
    dfree(p, p->keep, (size_t)p->store_cap * 8);
    p->store = ns;
    p->keep = nk;
    p->store_cap = cap;
    return MOMENTI_OK;
}

static int alloc_pool(momenti_plan* p, int P, int k, int steps)
{
    dfree(p, p->pools, (size_t)2 * p->P * sizeof(VRec));
    dfree(p, p->top, (size_t)p->top_k * sizeof(VRec));
    dfree(p, p->snaps, (size_t)p->snap_steps * sizeof(Snap));
    dfree(p, p->snap_tops, (size_t)p->snap_steps * p->snap_k * sizeof(VRec));
    p->pools = nullptr; p->top = nullptr; p->snaps = nullptr; p->snap_tops = nullptr;
    host_free(p, p->host_snaps);
    p->host_snaps = nullptr;
    int rc;
    if ((rc = dalloc_t(p, &p->pools, (size_t)2 * P * sizeof(VRec)))) return rc;
    p->P = P;
    if ((rc = dalloc_t(p, &p->top, (size_t)k * sizeof(VRec)))) return rc;
    p->top_k = k;
    if ((rc = dalloc_t(p, &p->snaps, (size_t)steps * sizeof(Snap)))) return rc;
    if ((rc = dalloc_t(p, &p->snap_tops, (size_t)steps * k * sizeof(VRec)))) return rc;
    p->snap_steps = steps;
    p->snap_k = k;
    if (!host_alloc(p, (void**)&p->host_snaps, (size_t)steps * sizeof(Snap)))
        return fail(MOMENTI_E_NOMEM, "host staging allocation failed");
    return MOMENTI_OK;
}

// A pool of P pairs for a restart. When the budget is taken by the candidate
// buffer and the store, they are halved to make room (a repetition whose
// candidates then overflow them is enumerated in parts). Called only when
// nothing is stored (at a restart or before the exact answer), so the store's
// contents may go.
static int grow_pool(momenti_plan* p, int P, int k, int steps)
{
    int rc;
    while ((rc = alloc_pool(p, P, k, steps)) == MOMENTI_E_NOMEM && p->cap > (1u << 14)) {
        const uint32_t half = p->cap / 2;
        if ((rc = alloc_cand(p, half))) return rc;
        dfree(p, p->store, (size_t)p->store_cap * sizeof(VRec));
        dfree(p, p->keep, (size_t)p->store_cap * 8);
        p->store = nullptr;
        p->keep = nullptr;
        p->store_cap = 0;
        if ((rc = grow_store(p, half, 0))) return rc;
    }
    return rc;
}

// Replay `count` verified records at `rec` (tagged with round and repetition)
// through the pool for steps [s0, s0 + nsteps); snapshots land in p->snaps.
static int replay(momenti_plan* p, const VRec* rec, uint32_t count, uint32_t* keep, int k, int s0,
                  int nsteps, int wmin = 0)
{
    HIP_OK(launch_zero(p->rctl, offsetof(ReplayCtl, step_count) + (size_t)nsteps * 4, p->st));
    struct {
        uint32_t n_keep;
        int32_t K, L, s0, nsteps, dropped, wmin;
    } hdr = {0u, p->K, p->L, s0, nsteps, 0, wmin};
    HIP_OK(hipMemcpyAsync(p->rctl, &hdr, sizeof hdr, hipMemcpyHostToDevice, p->st));
    HIP_OK(timed(p, KI_POOL, 0.0, 0.0, [&] {
        return launch_replay(rec, count, keep, keep + std::max<uint32_t>(count, 1u), p->rctl, st_pool(p),
                             p->pools, p->P, p->top, k, p->w, p->snaps, p->snap_tops, p->st);
    }));
    HIP_OK(hipMemcpyAsync(p->host_snaps, p->snaps, (size_t)nsteps * sizeof(Snap), hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    prof_flush(p);
    return MOMENTI_OK;
}

static void to_motifs(const std::vector<VRec>& v, int count, momenti_motif* out)
{
    for (int s = 0; s < count; ++s) {
        out[s].a = v[s].a;
        out[s].b = v[s].b;
        out[s].dist_d = v[s].dist_d;
        out[s].dist_max = v[s].dist_max;
        out[s].dims[0] = v[s].dims[0];
        out[s].dims[1] = v[s].dims[1];
        out[s].fail_prob = 0.0;   // exact unless the search sets its bound
    }
}

static int exact_fallback(momenti_plan* p, int d, int k, momenti_motif* out, int32_t* n_out,
                          momenti_report* rep);

// Rounds processed from one sort. A segment sorted by its length-i prefix
// is sorted by every shorter prefix too, so one sort serves a group of
// rounds [i_hi .. i_lo] when it is by the lowest round's prefix. The first
// group reaches down to the lowest round whose colliding pairs are
// estimated to cost less to enumerate than a sort pass (about 8 pairs per
// segment element), at most 7 rounds; below it, where collisions multiply,
// every round has a sort of its own. pairs_est[i] estimates the colliding
// pairs of round i over all segments and repetitions.
static std::vector<std::pair<int, int>> round_groups(int K, const double* pairs_est, double budget)
{
    int lo = K;
    while (lo > 1 && K - lo + 2 <= 7 && pairs_est[lo - 1] <= budget) --lo;
    std::vector<std::pair<int, int>> g;
    g.push_back({K, lo});
    for (int i = lo - 1; i >= 1; --i) g.push_back({i, i});
    return g;
}

extern "C" int momenti_search(momenti_plan* p, int32_t d, int32_t k, double delta, momenti_motif* out,
                              int32_t* n_out, momenti_report* rep)
{
    g_err.clear();
    if (!p || !out || !n_out) return fail(MOMENTI_E_ARG, "NULL argument");
    if (!p->hashed) return fail(MOMENTI_E_STATE, "momenti_hash has not been called");
    if (d < 1 || d > p->D) return fail(MOMENTI_E_ARG, "d=%d outside [1, D=%d]", d, p->D);
    if (k < 1 || k > 4096) return fail(MOMENTI_E_ARG, "k=%d outside [1, 4096]", k);
    if (!(delta > 0.0 && delta < 1.0)) return fail(MOMENTI_E_ARG, "delta=%g outside (0, 1)", delta);
    // Lemma 5.4: all k motifs at once with probability >= 1 - delta
    const double delta_rule = p->o.delta_mode == MOMENTI_DELTA_JOINT ? delta / k : delta;
    *n_out = 0;
    const auto t0 = std::chrono::steady_clock::now();
    momenti_report R{};
    R.K = p->K;
    R.L_used = p->L;
    R.r = p->r;
    R.t_hash_ms = p->t_hash_ms;

    // a plan of its own keeps the blocks of its previous search for this one
    // (same sizes when the arguments repeat) until its allocations are done
    struct Recycle {
        momenti_plan* p;
        ~Recycle() { p->recycle = false; }
    } recycling{p};
    if (!p->arena) {
        p->recycle = true;
        release_search(p);
    }
    const int max_steps = std::min(p->K, 7) * p->L;   // steps of the largest round group
    int P = p->o.pool_size ? p->o.pool_size : std::max(4096, 128 * k);
    P = std::max(P, k);
    int rc;
    if ((rc = dalloc_t(p, &p->status, 4096))) return rc;
    if ((rc = dalloc_t(p, &p->rctl, sizeof(ReplayCtl)))) return rc;
    if (!host_alloc(p, (void**)&p->host_status, 4096))
        return fail(MOMENTI_E_NOMEM, "host staging allocation failed");
    if ((rc = alloc_pool(p, P, k, max_steps))) return rc;
    const int64_t tiles = (p->ns + kSortTile - 1) / kSortTile;
    // A pair colliding in >= d dimensions has its lowest colliding dimension
    // below D - d + 1, and only that dimension's segment reports it: the
    // last d - 1 dimensions need no segments.
    const int Ds = std::max(1, p->D - d + 1);
    const uint64_t left0 = p->mem_limit - p->bytes;
    uint32_t cap = 1u << 20;
    while (cap > (1u << 14) && cand_bytes(cap, p->vsets) + store_bytes(cap) + sort_bytes(1, Ds, p->D, p->ns, tiles) > left0)
        cap >>= 1;
    if ((rc = alloc_cand(p, cap))) return rc;
    if ((rc = grow_store(p, cap, 0))) return rc;
    int Bmax = p->o.batch_reps ? p->o.batch_reps : 16;
    Bmax = std::max(1, std::min({Bmax, p->L, 64}));
    int B = Bmax;
    while (B > 1 && sort_bytes(B, Ds, p->D, p->ns, tiles) > p->mem_limit - p->bytes) B >>= 1;
    if ((rc = alloc_sort(p, B, Ds))) return rc;
    {
        StepGeom gmax{};
        gmax.ns = p->ns;
        gmax.nseg = B * Ds;
        p->coll_parts = enum_partials(gmax);
        if ((rc = dalloc_t(p, &p->coll_part, (size_t)p->coll_parts * 24))) return rc;
    }
    R.batch_reps = B;
    // a plan of its own frees the blocks of its previous search that this one
    // did not take back, so that it holds what it uses (a batch worker keeps
    // them for its next series)
    if (p->cache == &p->own_cache && !p->arena) {
        p->own_cache.trim();
        p->recycle = false;
    }

    // Probe: repetition 0 of the first (up to 8) segment dimensions, sorted by
    // the full K-symbol prefix, gives the colliding pairs of every round;
    // scaled to all segments and repetitions they choose the round groups.
    double pairs_est[9] = {0};
    {
        const int Dp = std::min(Ds, 8);
        StepGeom g;
        g.ns = p->ns; g.D = p->D; g.NF = p->NF; g.NL = p->NL; g.m = p->m;
        g.j0 = 0; g.Ds = Ds; g.nseg = Dp; g.i = p->K; g.K = p->K; g.i_lo = p->K; g.hashed = 0;
        g.dhi = d; g.part = 0; g.nparts = 1; g.fq = 0;
        int buf = 0;
        const double elems = (double)Dp * p->ns, kb = p->K <= 4 ? 4.0 : 8.0;
        for (int pass = 0; pass < p->K; ++pass) {
            const double kin = pass == 0 ? 8.0 : kb;
            HIP_OK(timed(p, KI_HIST, elems * kin, 0.0, [&] { return launch_hist(g, p->H, p->sb, pass, buf, p->st); }));
            HIP_OK(timed(p, KI_SCAN, 8.0 * g.nseg * 256.0 * p->sb.tiles, 0.0, [&] { return launch_scan(g, p->sb, p->st); }));
            HIP_OK(timed(p, KI_SCATTER, elems * (kin + (pass == 0 ? 0.0 : 4.0) + kb + 4.0), 0.0,
                         [&] { return launch_scatter(g, p->H, p->sb, pass, buf, p->st); }));
            buf ^= 1;
        }
        unsigned long long* dcnt = (unsigned long long*)(p->status + 2048);
        HIP_OK(timed(p, KI_PROBE, elems * kb, 0.0, [&] { return launch_probe(g, p->sb, buf, dcnt, p->st); }));
        HIP_OK(hipMemcpyAsync(p->host_status + 2048, dcnt, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, p->st));
        HIP_OK(hipStreamSynchronize(p->st));
        prof_flush(p);
        const unsigned long long* hc = (const unsigned long long*)(p->host_status + 2048);
        for (int i = 1; i <= p->K; ++i) pairs_est[i] = (double)hc[i - 1] * ((double)Ds / Dp) * p->L;
    }
    const double per_elem = p->o.merge_pairs > 0.0 ? p->o.merge_pairs : 8.0;
    const auto groups = round_groups(p->K, pairs_est, per_elem * (double)p->ns * Ds * p->L);
    R.first_group_lo = groups[0].second;
    static const int verbose = [] {
        const char* v = std::getenv("MOMENTI_VERBOSE");
        return v ? std::atoi(v) : 0;
    }();
    if (verbose) {
        std::fprintf(stderr, "[momenti] probe: estimated pairs per round");
        for (int i = p->K; i >= 1; --i) std::fprintf(stderr, " %d:%.3g", i, pairs_est[i]);
        std::fprintf(stderr, "\n");
    }

    // The failure bound of each returned motif at step (i, J) of the traversal
    // (1 before any step), and the k-th's in the report.
    auto annotate = [&](int count, int i, int J) {
        for (int q = 0; q < count; ++q)
            out[q].fail_prob = i > 0 ? std::exp(log_fail(out[q].dist_max, p->r, d, i, J, p->K, p->L, p->m,
                                                         p->o.stop_rule)) : 1.0;
        R.fail_bound = count >= k ? out[k - 1].fail_prob : 1.0;
    };
    int last_i = 0, last_J = 0;   // the last step whose TOP is known
    const bool tracing = p->tr_cand || p->tr_top_size;
    if (p->tr_count) *p->tr_count = 0;
    if (p->tr_top_size)
        for (int64_t s = 0; s < p->tr_steps_cap; ++s) p->tr_top_size[s] = -1;
    std::vector<Cand> hcand;
    std::vector<VRec> hsnap;
    const double elem_x = p->dtype == MOMENTI_F64 ? 8.0 : 4.0;
    unsigned long long n_screened = 0;
    uint32_t max_run = 0;

    // Steps [s0, s0 + nsteps) have just been replayed: record the trace, then
    // test the stopping rule after each step in order. Returns 1 when it
    // held (out and rep filled), 2 when the pool must grow and the search
    // restart, 3 when a step or time budget ended the search (out and rep
    // filled with TOP at that step), 0 to go on, or an error code.
    auto check_steps = [&](int s0, int nsteps) -> int {
        if (tracing && p->tr_top_size) {
            hsnap.resize((size_t)nsteps * k);
            HIP_OK(copy_sync(p, hsnap.data(), p->snap_tops, hsnap.size() * sizeof(VRec), hipMemcpyDeviceToHost));
            for (int st = 0; st < nsteps; ++st) {
                const int64_t sg = s0 + st;
                if (sg >= p->tr_steps_cap) continue;
                p->tr_top_size[sg] = p->host_snaps[st].top_n;
                for (int q = 0; q < p->host_snaps[st].top_n && q < p->tr_k; ++q) {
                    p->tr_top_pairs[(sg * p->tr_k + q) * 2 + 0] = hsnap[(size_t)st * k + q].a;
                    p->tr_top_pairs[(sg * p->tr_k + q) * 2 + 1] = hsnap[(size_t)st * k + q].b;
                }
            }
        }
        for (int st = 0; st < nsteps; ++st) {
            const Snap& sn = p->host_snaps[st];
            const int sg = s0 + st;
            const int i = p->K - sg / p->L;
            const int J = sg % p->L + 1;
            ++R.n_steps;
            if (sn.top_n < k && sn.truncated) {
                // the pool dropped pairs that TOP may still need: redo with a larger pool
                ++R.pool_overflow;
                P *= 2;
                int e;
                if ((e = grow_pool(p, P, k, max_steps))) return e;
                return 2;
            }
            last_i = i;
            last_J = J;
            if (sn.top_n == k &&
                stop_holds(sn.dist_max, p->r, d, i, J, p->K, p->L, p->m, p->o.stop_rule, delta_rule)) {
                std::vector<VRec> tv(k);
                HIP_OK(copy_sync(p, tv.data(), p->snap_tops + (size_t)st * k, (size_t)k * sizeof(VRec),
                                 hipMemcpyDeviceToHost));
                to_motifs(tv, k, out);
                *n_out = k;
                annotate(k, i, J);
                R.i_stop = i;
                R.j_stop = J;
                if (verbose)
                    std::fprintf(stderr, "[momenti] stop (%d, %d): collisions %lld, screened %llu, longest run %u\n",
                                 i, J, (long long)R.n_collisions, n_screened, max_run);
                R.peak_bytes = p->peak;
                R.t_search_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (rep) *rep = R;
                return 1;
            }
            // anytime budgets: TOP as it stands after this step, with its bounds
            const double elapsed = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if ((p->o.max_steps > 0 && R.n_steps >= p->o.max_steps) || (p->o.max_ms > 0.0 && elapsed >= p->o.max_ms)) {
                const int nt = std::min(sn.top_n, k);
                std::vector<VRec> tv(std::max(nt, 1));
                if (nt)
                    HIP_OK(copy_sync(p, tv.data(), p->snap_tops + (size_t)st * k, (size_t)nt * sizeof(VRec),
                                     hipMemcpyDeviceToHost));
                to_motifs(tv, nt, out);
                *n_out = nt;
                annotate(nt, i, J);
                R.budget_round = i;
                R.peak_bytes = p->peak;
                R.t_search_ms = elapsed;
                if (rep) *rep = R;
                return 3;
            }
        }
        return 0;
    };

    // Round groups still to traverse. A multi-round group keeps its verified
    // records until its replay; when they would exceed the memory budget the
    // group is split into single-round groups (each replayed batch by batch).
    std::vector<std::pair<int, int>> todo(groups.begin(), groups.end());
restart:
    HIP_OK(launch_pool_reset(st_pool(p), p->st));
    R.n_steps = 0;
    if (tracing && p->tr_count) *p->tr_count = 0;
    for (size_t gi = 0; gi < todo.size(); ++gi) {
        const int i_hi = todo[gi].first, i_lo = todo[gi].second;
        const int s0 = (p->K - i_hi) * p->L;
        const int nsteps = (i_hi - i_lo + 1) * p->L;
        if (p->o.max_pairs > 0.0 && pairs_est[i_lo] > p->o.max_pairs) {
            // over the work budget: answer with TOP as it stands (anytime)
            PoolState ps;
            HIP_OK(hipMemcpyAsync(p->host_status + 64, st_pool(p), sizeof ps, hipMemcpyDeviceToHost, p->st));
            HIP_OK(hipStreamSynchronize(p->st));
            std::memcpy(&ps, p->host_status + 64, sizeof ps);
            const int nt = std::min(ps.top_n, k);
            if (nt > 0) {
                std::vector<VRec> tv(nt);
                HIP_OK(copy_sync(p, tv.data(), p->top, (size_t)nt * sizeof(VRec), hipMemcpyDeviceToHost));
                to_motifs(tv, nt, out);
            }
            *n_out = nt;
            annotate(nt, last_i, last_J);
            if (verbose)
                std::fprintf(stderr, "[momenti] budget: rounds %d..%d estimated at %.3g pairs > %.3g; %d motifs so far\n",
                             i_hi, i_lo, pairs_est[i_lo], p->o.max_pairs, nt);
            R.budget_round = i_hi;
            R.peak_bytes = p->peak;
            R.t_search_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rep) *rep = R;
            return MOMENTI_OK_PARTIAL;
        }
        if (verbose) {
            std::fprintf(stderr, "[momenti] rounds %d..%d: %.1f ms, steps %lld, collisions %lld, screened %llu, longest run %u, candidates %lld |",
                         i_hi, i_lo,
                         std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(),
                         (long long)R.n_steps, (long long)R.n_collisions, n_screened, max_run, (long long)R.n_cand);
            for (int q = 0; q < KI_COUNT; ++q)
                if (p->prof.tot[q].launches) std::fprintf(stderr, " %s %.1f", kKernelNames[q], p->prof.tot[q].ms);
            std::fprintf(stderr, "\n");
        }
        uint32_t stored = 0;
        // a single-round group replays each batch as soon as it is verified,
        // so that it stops at the first repetition where the rule holds
        const bool incremental = i_hi == i_lo;
        bool split = false;
        for (int j0 = 0; j0 < p->L && !split;) {
            const int Bc = std::min(B, p->L - j0);
            StepGeom g;
            g.ns = p->ns; g.D = p->D; g.NF = p->NF; g.NL = p->NL; g.m = p->m;
            g.j0 = j0; g.Ds = Ds; g.nseg = Bc * Ds; g.i = i_hi; g.K = p->K; g.i_lo = i_lo;
            g.hashed = i_lo > 4;   // longer prefixes are grouped by a 24-bit hash (3 passes)
            g.dhi = d;
            g.part = 0; g.nparts = 1;
            g.fq = second_stage_pays(p->D, d);
            int buf = 0;
            const double elems = (double)g.nseg * p->ns;
            const double kb = sort_keys_32(g) ? 4.0 : 8.0;
            const int kt = std::min(i_hi + 1, p->K);
            const int nw = fp_words(p->D);
            const int nq = fq_words(p->D);
            // the fingerprint tables, with the histogram of the sort's pass 0
            HIP_OK(timed(p, KI_FPTABLE, (double)Bc * p->ns * (p->D * 8.0 + 4.0 * (nw + (g.fq ? nq : 0))), 0.0, [&] {
                return launch_fptable(p->H, g, Bc, p->fps, p->fq, p->sb, p->st);
            }));
            for (int pass = 0; pass < sort_passes(g); ++pass) {
                const double kin = pass == 0 ? 8.0 : kb;   // pass 0 reads two index words
                if (pass > 0)
                    HIP_OK(timed(p, KI_HIST, elems * kin, 0.0, [&] { return launch_hist(g, p->H, p->sb, pass, buf, p->st); }));
                HIP_OK(timed(p, KI_SCAN, 8.0 * g.nseg * 256.0 * p->sb.tiles, 0.0, [&] { return launch_scan(g, p->sb, p->st); }));
                HIP_OK(timed(p, KI_SCATTER, elems * (kin + (pass == 0 ? 0.0 : 4.0) + kb + 4.0), 0.0,
                             [&] { return launch_scatter(g, p->H, p->sb, pass, buf, p->st); }));
                buf ^= 1;
            }
            // Enumeration, verification and (single-round groups) replay, in
            // g.nparts parts when one repetition's candidates do not fit in
            // memory at once: merging a step's records into the pool part by
            // part leaves the same pool (the best P of their union) and TOP.
            bool redo = false;   // fewer repetitions per launch, or a larger buffer
            for (g.part = 0; g.part < g.nparts && !redo && !split; ++g.part) {
                HIP_OK(launch_zero(p->status, 64, p->st));
                int enum_slot = -1, verify_slot = -1;
                HIP_OK(timed(p, KI_ENUM, 0.0, 0.0, [&] {
                    return launch_enum(g, p->sb, buf, p->H, p->fps, p->fq, kt, d, p->w, p->cand, p->cap,
                                       st_counters(p), p->coll_part, p->st);
                }, &enum_slot));
                HIP_OK(timed(p, KI_VERIFY, 0.0, 0.0, [&] {
                    return launch_verify(p->cand, p->cap, st_counters(p), p->series, p->dtype, p->n, p->ns,
                                         p->D, p->w, d, p->mu, p->isig, p->vrec, p->st);
                }, &verify_slot));
                Counters cnt;
                HIP_OK(hipMemcpyAsync(p->host_status, p->status, sizeof(Counters), hipMemcpyDeviceToHost, p->st));
                HIP_OK(hipStreamSynchronize(p->st));
                std::memcpy(&cnt, p->host_status, sizeof cnt);
                {
                    // sizes known only now: the enumeration read every key once and
                    // every run member's index and fingerprint row once (pairs that
                    // pass the screen re-read 4 D index words: negligible), and
                    // screened each pair of a run with one XOR and one OR per row
                    // word, a popcount per 32 dimensions and a compare;
                    // verification read 2 D w samples per candidate
                    const uint32_t nc = std::min(cnt.n_cand, p->cap);
                    prof_set(p, enum_slot, elems * kb + (double)cnt.n_memb * (4.0 + 4.0 * nw),
                             (double)cnt.n_coll * (2.0 * nw + (p->D + 31) / 32 + 1.0));
                    prof_set(p, verify_slot, (double)nc * (2.0 * p->D * p->w * elem_x + 32.0 * p->D + sizeof(VRec)),
                             (double)nc * 6.0 * p->D * p->w);
                    prof_flush(p);
                }
                if (cnt.n_units > p->sb.ucap)   // cannot happen: ucap bounds the tile rows of a batch
                    return fail(MOMENTI_E_DEVICE, "%u tile rows queued, room for %u", cnt.n_units, p->sb.ucap);
                if (cnt.n_cand > p->cap) {
                    // more candidates than room: fewer repetitions per launch, then a
                    // larger buffer, then (a single-round group) parts of the step;
                    // a multi-round group is split into single rounds
                    if (Bc > 1) {
                        B = std::max(1, Bc / 2);
                        redo = true;
                        break;
                    }
                    uint32_t need = p->cap;
                    while (need < cnt.n_cand && need < (1u << 30)) need <<= 1;
                    // a single-round group replays each batch from the store, whose
                    // capacity must stay >= the candidate buffer's
                    const bool grow_st = incremental && need > p->store_cap;
                    const uint64_t extra = cand_bytes(need, p->vsets) - cand_bytes(p->cap, p->vsets) + (grow_st ? store_bytes(need) : 0);
                    if (need >= cnt.n_cand && extra <= p->mem_limit - p->bytes) {
                        const uint32_t old_cap = p->cap;
                        rc = alloc_cand(p, need);
                        if (rc == MOMENTI_OK && grow_st) rc = grow_store(p, need, 0);
                        if (rc == MOMENTI_OK) {
                            redo = true;
                            break;
                        }
                        if (rc != MOMENTI_E_NOMEM) return rc;
                        // could not allocate after all: back to a buffer the store covers
                        if ((rc = alloc_cand(p, std::min(old_cap, std::max(p->store_cap, 1u << 14))))) return rc;
                    }
                    if (!incremental) {
                        split = true;
                        break;
                    }
                    int np = g.nparts;
                    while ((uint64_t)np * p->cap < 2ull * cnt.n_cand * (uint64_t)g.nparts && np < (1 << 16)) np <<= 1;
                    if (np == g.nparts)
                        return fail(MOMENTI_E_NOMEM, "%u candidates in one step exceed mem_limit", cnt.n_cand);
                    if (verbose)
                        std::fprintf(stderr, "[momenti] step (%d, %d): %u candidates, enumerated in %d parts\n",
                                     i_hi, j0 + 1, cnt.n_cand, np);
                    g.nparts = np;
                    R.step_parts = std::max(R.step_parts, np);
                    g.part = -1;   // parts already merged into the pool merge again as no-ops
                    continue;
                }
                if (cnt.n_cand) {
                    if (!incremental && (rc = grow_store(p, stored + cnt.n_cand, stored))) {
                        if (rc != MOMENTI_E_NOMEM) return rc;
                        split = true;   // the group's records would exceed the budget
                        break;
                    }
                    HIP_OK(hipMemcpyAsync(p->store + stored, p->vrec, (size_t)cnt.n_cand * sizeof(VRec),
                                          hipMemcpyDeviceToDevice, p->st));
                    stored += cnt.n_cand;
                }
                if (g.part == 0) {
                    R.n_collisions += (int64_t)cnt.n_coll;
                    n_screened += cnt.n_screen;
                }
                max_run = std::max(max_run, cnt.max_run);
                R.max_run = (int32_t)max_run;
                R.n_cand += cnt.n_cand;
                R.n_verified += cnt.n_cand;
                if (tracing && p->tr_cand && cnt.n_cand) {
                    hcand.resize(cnt.n_cand);
                    HIP_OK(copy_sync(p, hcand.data(), p->cand, cnt.n_cand * sizeof(Cand), hipMemcpyDeviceToHost));
                    for (const Cand& c : hcand) {
                        const int64_t s = (int64_t)(p->K - tag_round(c.pad)) * p->L + c.j;
                        if (*p->tr_count < p->tr_cap) {
                            p->tr_cand[3 * *p->tr_count + 0] = s;
                            p->tr_cand[3 * *p->tr_count + 1] = c.a;
                            p->tr_cand[3 * *p->tr_count + 2] = c.b;
                        }
                        ++*p->tr_count;
                    }
                }
                if (incremental) {
                    if ((rc = replay(p, p->store, stored, p->keep, k, s0 + j0, Bc))) return rc;
                    stored = 0;   // the pool holds what the next steps need
                }
            }
            if (redo || split) continue;
            if (incremental) {
                // the snapshots of the last part's replay are those of the whole batch
                const int cs = check_steps(s0 + j0, Bc);
                if (cs < 0) return cs;
                if (cs == 1) return MOMENTI_OK;
                if (cs == 3) return MOMENTI_OK_PARTIAL;
                if (cs == 2) goto restart;
            }
            j0 += Bc;
        }
        if (split) {
            // traverse the group's rounds one by one (the pool is unchanged:
            // none of this group's records has been replayed yet)
            if (verbose)
                std::fprintf(stderr, "[momenti] rounds %d..%d split into single rounds (memory budget)\n", i_hi, i_lo);
            todo.erase(todo.begin() + (std::ptrdiff_t)gi);
            for (int i = i_lo; i <= i_hi; ++i) todo.insert(todo.begin() + (std::ptrdiff_t)gi, {i, i});
            ++R.group_splits;
            --gi;
            continue;
        }
        // multi-round group: replay its verified records in step order now
        if (!incremental) {
            if ((rc = replay(p, p->store, stored, p->keep, k, s0, nsteps))) return rc;
            const int cs = check_steps(s0, nsteps);
            if (cs < 0) return cs;
            if (cs == 1) return MOMENTI_OK;
            if (cs == 3) return MOMENTI_OK_PARTIAL;
            if (cs == 2) goto restart;
        }
    }
    rc = exact_fallback(p, d, k, out, n_out, &R);
    R.fallback = 1;
    R.fail_bound = 0.0;   // the exact answer
    R.peak_bytes = p->peak;
    R.t_search_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = R;
    return rc == MOMENTI_OK ? MOMENTI_OK_FALLBACK : rc;
}

// Algorithm 1, last line: no step stopped, so answer with the exact top-k
// over every non-trivial pair. Short series stream every pair through the
// verifier and the pool as one step; longer ones sweep the diagonals of the
// pair matrix (exact_sweep).
constexpr int64_t kAllPairsMax = 4096;

static int exact_sweep(momenti_plan* p, int d, int k, momenti_motif* out, int32_t* n_out, momenti_report* rep);

static int exact_fallback(momenti_plan* p, int d, int k, momenti_motif* out, int32_t* n_out,
                          momenti_report* rep)
{
    if (p->ns > kAllPairsMax) return exact_sweep(p, d, k, out, n_out, rep);
    const int64_t h = p->w / 2;
    const int64_t M = p->ns - h - 1;
    auto off = [M](int64_t a) { int64_t aa = std::min(a, std::max<int64_t>(M, 0)); return aa * M - aa * (aa - 1) / 2; };
    int rc;
    if (M > (int64_t)p->cap) {
        uint32_t need = p->cap;
        while ((int64_t)need < M) need <<= 1;
        if ((rc = alloc_cand(p, need))) return rc;
    }
    if ((rc = grow_store(p, p->cap, 0))) return rc;
    for (;;) {
        HIP_OK(launch_pool_reset(st_pool(p), p->st));
        int64_t row = 0;
        Snap last{};
        while (row < std::max<int64_t>(M, 0)) {
            int64_t hi = row + 1;
            while (hi < M && off(hi + 1) - off(row) <= (int64_t)p->cap) ++hi;
            const uint32_t cnt = (uint32_t)(off(hi) - off(row));
            HIP_OK(launch_zero(p->status, 64, p->st));
            HIP_OK(timed(p, KI_ALLPAIRS, 16.0 * cnt, 0.0, [&] {
                return launch_allpairs(p->ns, p->w, row, hi, off(row), p->cand, st_counters(p), p->st);
            }));
            HIP_OK(timed(p, KI_VERIFY, 0.0, 0.0, [&] {
                return launch_verify(p->cand, p->cap, st_counters(p), p->series, p->dtype, p->n, p->ns,
                                     p->D, p->w, d, p->mu, p->isig, p->vrec, p->st);
            }));
            // all-pairs records carry round 0, repetition 0: the single step K L
            if ((rc = replay(p, p->vrec, cnt, p->keep, k, p->K * p->L, 1))) return rc;
            last = p->host_snaps[0];
            rep->n_verified += cnt;
            row = hi;
        }
        if (M <= 0 || !(last.top_n < k && last.truncated)) {
            const int got = M <= 0 ? 0 : last.top_n;
            std::vector<VRec> tv(std::max(got, 1));
            if (got)
                HIP_OK(copy_sync(p, tv.data(), p->snap_tops, (size_t)got * sizeof(VRec), hipMemcpyDeviceToHost));
            to_motifs(tv, got, out);
            *n_out = got;
            return MOMENTI_OK;
        }
        ++rep->pool_overflow;
        if ((rc = grow_pool(p, p->P * 2, k, p->snap_steps))) return rc;
    }
}

// The exact answer by the diagonal sweep of k_exact.hip. The pool keeps the
// pairs the traversal verified; the sweep adds every pair whose d smallest
// per-dimension distances, as the sweep evaluates them, sum below the cut
// theta (each verified by k_verify). A pair left out has a sweep value >=
// theta, hence an exact dist_d >= theta - eps (eps bounds the sweep's
// rounding). Greedy over all pairs decides each pick from earlier pairs only,
// so when TOP holds k picks and the k-th is below theta - eps, TOP is the
// greedy choice over every pair; otherwise the cut widens and the sweep
// repeats. The cut starts at TOP's k-th distance (plus margin) and follows it
// down as TOP improves.
static int exact_sweep(momenti_plan* p, int d, int k, momenti_motif* out, int32_t* n_out, momenti_report* rep)
{
    int rc;
    if ((rc = grow_store(p, p->cap, 0))) return rc;   // room to replay a whole candidate buffer
    const int DL = p->D > 64 ? 2 : 1;
    int Dp = 1;
    while (Dp < std::min(p->D, 64)) Dp <<= 1;
    if (DL == 2) Dp = 64;
    const int G = 64 / Dp;
    const int Lc = std::max(2048, 8 * p->w);
    const int64_t first = p->w / 2 + 1;   // smallest diagonal offset with 2 s > w
    if (first >= p->ns) {
        *n_out = 0;
        return MOMENTI_OK;
    }
    const int64_t groups = (p->ns - first + G - 1) / G;
    const int64_t chunks = (p->ns - first + Lc - 1) / Lc;
    const int64_t items = groups * chunks;
    const double eps = (double)d * std::sqrt(1e-6 * (double)p->w);
    // no pair is farther apart: a z-normalised window has norm sqrt(w) (a flat
    // one is all zeros), so each dimension's distance is at most 2 sqrt(w)
    const double dmax = 2.0 * d * std::sqrt((double)p->w);
    const double elem_x = p->dtype == MOMENTI_F64 ? 8.0 : 4.0;

    auto read_top = [&](int* topn, double* kth) -> int {
        PoolState ps;
        HIP_OK(hipMemcpyAsync(p->host_status + 64, st_pool(p), sizeof ps, hipMemcpyDeviceToHost, p->st));
        HIP_OK(hipStreamSynchronize(p->st));
        std::memcpy(&ps, p->host_status + 64, sizeof ps);
        *topn = ps.top_n;
        *kth = INFINITY;
        if (ps.top_n >= k) {
            VRec v;
            HIP_OK(copy_sync(p, &v, p->top + (k - 1), sizeof v, hipMemcpyDeviceToHost));
            *kth = v.dist_d;
        }
        return MOMENTI_OK;
    };
    int topn = 0;
    double kth = INFINITY;
    if ((rc = read_top(&topn, &kth))) return rc;
    double theta = topn >= k ? kth + 2.0 * eps : INFINITY;
    std::vector<double> buf;
    for (int attempt = 0; attempt < 64; ++attempt) {
        double theta_min = INFINITY;
        bool restart = false;
        std::vector<std::pair<int64_t, int64_t>> work;   // item ranges still to sweep (taken from the back)
        const int64_t per = std::max<int64_t>(1, (items + 31) / 32);
        for (int64_t lo = ((items + per - 1) / per - 1) * per; lo >= 0; lo -= per)
            work.push_back({lo, std::min(items, lo + per)});
        while (!work.empty() && !restart) {
            const auto range = work.back();
            work.pop_back();
            int nparts = 1;
            for (int part = 0; part < nparts; ++part) {
                SweepArgs g;
                g.n = p->n; g.ns = p->ns; g.s_lo = first; g.item_lo = range.first; g.item_hi = range.second;
                g.chunks = chunks; g.D = p->D; g.Dp = Dp; g.G = G; g.DL = DL; g.w = p->w; g.d = d; g.Lc = Lc;
                g.part = part; g.nparts = nparts;
                g.theta = theta;
                g.th2 = std::isinf(theta) ? INFINITY : theta * theta;
                g.low2 = std::isinf(theta) ? INFINITY : (theta / d) * (theta / d);
                HIP_OK(launch_zero(p->status, 64, p->st));
                const double pairs = (double)(range.second - range.first) * G * Lc;
                HIP_OK(timed(p, KI_SWEEP, pairs * p->D * 4.0 * elem_x, pairs * p->D * 12.0, [&] {
                    return launch_sweep(p->series, p->dtype, p->mu, p->isig, g, p->cand, p->cap, st_counters(p), p->st);
                }));
                HIP_OK(timed(p, KI_VERIFY, 0.0, 0.0, [&] {
                    return launch_verify(p->cand, p->cap, st_counters(p), p->series, p->dtype, p->n, p->ns,
                                         p->D, p->w, d, p->mu, p->isig, p->vrec, p->st);
                }));
                Counters cnt;
                HIP_OK(hipMemcpyAsync(p->host_status, p->status, sizeof(Counters), hipMemcpyDeviceToHost, p->st));
                HIP_OK(hipStreamSynchronize(p->st));
                std::memcpy(&cnt, p->host_status, sizeof cnt);
                prof_flush(p);
                if (cnt.n_cand > p->cap) {
                    // too many pairs below the cut in this range: while there is no
                    // cut yet (TOP short of k picks), take the distance that about
                    // cap / 8 of the buffered pairs reach; else sweep halves of the
                    // range; a single item is split into parts of its pairs
                    if (std::isinf(theta)) {
                        // verify the candidates the buffer holds (the verifier skips
                        // an overflowed buffer), then read their distances
                        HIP_OK(launch_set_count(st_counters(p), p->cap, p->st));
                        HIP_OK(launch_verify(p->cand, p->cap, st_counters(p), p->series, p->dtype, p->n, p->ns,
                                             p->D, p->w, d, p->mu, p->isig, p->vrec, p->st));
                        buf.resize(p->cap);
                        std::vector<VRec> vr(p->cap);
                        HIP_OK(copy_sync(p, vr.data(), p->vrec, (size_t)p->cap * sizeof(VRec), hipMemcpyDeviceToHost));
                        for (uint32_t q = 0; q < p->cap; ++q) buf[q] = vr[q].dist_d;
                        std::nth_element(buf.begin(), buf.begin() + p->cap / 8, buf.end());
                        const double th = buf[p->cap / 8] + 2.0 * eps;
                        if (th < theta) {
                            theta = th;
                            nparts = 0;   // ends the part loop; the range is swept again
                            work.push_back(range);
                            break;
                        }
                    }
                    if (range.second - range.first > 1) {
                        const int64_t mid = range.first + (range.second - range.first) / 2;
                        work.push_back({mid, range.second});
                        work.push_back({range.first, mid});
                        nparts = 0;
                        break;
                    }
                    int np = nparts;
                    while ((uint64_t)np * p->cap < 2ull * cnt.n_cand * (uint64_t)nparts && np < (1 << 20)) np <<= 1;
                    if (np == nparts)
                        return fail(MOMENTI_E_NOMEM, "exact answer: %u pairs below the cut in one part", cnt.n_cand);
                    nparts = np;
                    part = -1;   // parts already merged into the pool merge again as no-ops
                    continue;
                }
                theta_min = std::min(theta_min, theta);
                rep->n_verified += cnt.n_cand;
                if (cnt.n_cand == 0) continue;
                if ((rc = replay(p, p->vrec, cnt.n_cand, p->keep, k, p->K * p->L, 1))) return rc;
                const Snap sn = p->host_snaps[0];
                if (sn.top_n < k && sn.truncated) {
                    // the pool dropped pairs TOP may need: larger pool, sweep again
                    ++rep->pool_overflow;
                    if ((rc = grow_pool(p, p->P * 2, k, p->snap_steps))) return rc;
                    HIP_OK(launch_pool_reset(st_pool(p), p->st));
                    restart = true;
                    break;
                }
                if ((rc = read_top(&topn, &kth))) return rc;
                if (topn >= k) theta = std::min(theta, kth + 2.0 * eps);
            }
        }
        if (restart) {   // the pool was emptied: the same cut, every range again
            topn = 0;
            kth = INFINITY;
            continue;
        }
        if ((rc = read_top(&topn, &kth))) return rc;
        // certified when the cut left no pair out (fewer than k picks exist
        // then), or TOP's k-th pick lies below every pair it left out
        if (std::isinf(theta_min) || theta_min - eps > dmax || (topn >= k && kth < theta_min - eps)) {
            const int got = std::min(topn, k);
            std::vector<VRec> tv(std::max(got, 1));
            if (got) HIP_OK(copy_sync(p, tv.data(), p->top, (size_t)got * sizeof(VRec), hipMemcpyDeviceToHost));
            to_motifs(tv, got, out);
            *n_out = got;
            return MOMENTI_OK;
        }
        // not certified: widen the cut past TOP's k-th pick, or double it, at
        // most to a cut that leaves no pair out
        theta = topn >= k ? kth + 4.0 * eps : std::min(2.0 * theta_min, dmax + 2.0 * eps);
    }
    return fail(MOMENTI_E_DEVICE, "exact answer: the sweep did not certify its result");
}

// ------------------------------------------------------------------ several dimensionalities
// Section 6.3: one traversal answers every dimensionality d in [d_lo, d_hi].
// Each d has its own pool of verified pairs; one verification of a candidate
// gives its dist_d for every d (the d smallest per-dimension distances are a
// prefix of the same ranking). Pool d takes the candidates that collided in
// >= d dimensions, so after every step it holds the pairs a search for d
// alone holds, and d stops at that search's step with its answer. The
// enumeration follows the smallest d not yet answered (d_cur): fewer
// dimensions then count for nothing. Rounds are traversed one at a time,
// each batch of repetitions replayed into every open pool as it is verified.
struct PoolSet {
    VRec *pools = nullptr, *top = nullptr, *snap_tops = nullptr;
    Snap *snaps = nullptr, *host_snaps = nullptr;
    int P = 0, top_k = 0, steps = 0, snap_k = 0;
    PoolState* ps = nullptr;
};

static void pool_in(momenti_plan* p, const PoolSet& q)
{
    p->pools = q.pools; p->P = q.P; p->top = q.top; p->top_k = q.top_k; p->snaps = q.snaps;
    p->snap_tops = q.snap_tops; p->snap_steps = q.steps; p->snap_k = q.snap_k; p->host_snaps = q.host_snaps;
    p->ps_cur = q.ps;
}

static void pool_out(momenti_plan* p, PoolSet& q)
{
    q.pools = p->pools; q.P = p->P; q.top = p->top; q.top_k = p->top_k; q.snaps = p->snaps;
    q.snap_tops = p->snap_tops; q.steps = p->snap_steps; q.snap_k = p->snap_k; q.host_snaps = p->host_snaps;
    p->pools = nullptr; p->top = nullptr; p->snaps = nullptr; p->snap_tops = nullptr; p->host_snaps = nullptr;
    p->P = p->top_k = p->snap_steps = p->snap_k = 0;
    p->ps_cur = nullptr;
}

extern "C" int momenti_search_multi(momenti_plan* p, int32_t d_lo, int32_t d_hi, int32_t k, double delta,
                                    momenti_motif* out, int32_t* n_out, int32_t* status, momenti_report* reps)
{
    g_err.clear();
    if (!p || !out || !n_out || !status) return fail(MOMENTI_E_ARG, "NULL argument");
    if (!p->hashed) return fail(MOMENTI_E_STATE, "momenti_hash has not been called");
    if (d_lo < 1 || d_hi > p->D || d_lo > d_hi)
        return fail(MOMENTI_E_ARG, "dimensionalities [%d, %d] outside [1, D=%d]", d_lo, d_hi, p->D);
    if (k < 1 || k > 4096) return fail(MOMENTI_E_ARG, "k=%d outside [1, 4096]", k);
    if (!(delta > 0.0 && delta < 1.0)) return fail(MOMENTI_E_ARG, "delta=%g outside (0, 1)", delta);
    if (p->arena) return fail(MOMENTI_E_STATE, "not available without allocations");
    const int nd = d_hi - d_lo + 1;
    if (nd == 1) {
        momenti_report R{};
        const int rc = momenti_search(p, d_lo, k, delta, out, n_out, &R);
        if (rc < 0) return rc;
        status[0] = rc;
        if (reps) reps[0] = R;
        return MOMENTI_OK;
    }
    const double delta_rule = p->o.delta_mode == MOMENTI_DELTA_JOINT ? delta / k : delta;
    const auto t0 = std::chrono::steady_clock::now();
    for (int q = 0; q < nd; ++q) {
        n_out[q] = 0;
        status[q] = -1;   // not answered yet
    }
    struct Recycle {
        momenti_plan* p;
        ~Recycle() { p->recycle = false; p->vsets = 1; p->ps_cur = nullptr; }
    } recycling{p};
    p->recycle = true;
    release_search(p);
    p->vsets = nd;
    std::vector<PoolSet> sets(nd);
    PoolState* ps_block = nullptr;
    // every allocation of this search, freed before returning (the pools are
    // not kept from one search to the next)
    auto release_sets = [&]() {
        for (auto& q : sets) {
            pool_in(p, q);
            dfree(p, p->pools, (size_t)2 * p->P * sizeof(VRec));
            dfree(p, p->top, (size_t)p->top_k * sizeof(VRec));
            dfree(p, p->snaps, (size_t)p->snap_steps * sizeof(Snap));
            dfree(p, p->snap_tops, (size_t)p->snap_steps * p->snap_k * sizeof(VRec));
            host_free(p, p->host_snaps);
            p->pools = p->top = p->snap_tops = nullptr; p->snaps = p->host_snaps = nullptr;
            p->P = p->top_k = p->snap_steps = p->snap_k = 0;
            q = PoolSet{};
        }
        p->ps_cur = nullptr;
        dfree(p, ps_block, (size_t)nd * sizeof(PoolState));
        ps_block = nullptr;
    };
    struct Guard {
        std::function<void()> f;
        ~Guard() { f(); }
    } guard{release_sets};
    int rc;
    int B = std::max(1, std::min({p->o.batch_reps ? p->o.batch_reps : 16, p->L, 64}));
    int P = p->o.pool_size ? p->o.pool_size : std::max(4096, 128 * k);
    P = std::max(P, k);
    if ((rc = dalloc_t(p, &p->status, 4096))) return rc;
    if ((rc = dalloc_t(p, &p->rctl, sizeof(ReplayCtl)))) return rc;
    if ((rc = dalloc_t(p, &ps_block, (size_t)nd * sizeof(PoolState)))) return rc;
    if (!host_alloc(p, (void**)&p->host_status, 4096)) return fail(MOMENTI_E_NOMEM, "host staging allocation failed");
    for (int q = 0; q < nd; ++q) {
        if ((rc = alloc_pool(p, P, k, B))) return rc;
        pool_out(p, sets[q]);
        sets[q].ps = ps_block + q;
    }
    const int64_t tiles = (p->ns + kSortTile - 1) / kSortTile;
    const int Ds_max = std::max(1, p->D - d_lo + 1);
    const uint64_t left0 = p->mem_limit - p->bytes;
    uint32_t cap = 1u << 20;
    while (cap > (1u << 14) && cand_bytes(cap, nd) + store_bytes(cap) + sort_bytes(1, Ds_max, p->D, p->ns, tiles) > left0)
        cap >>= 1;
    if ((rc = alloc_cand(p, cap))) return rc;
    if ((rc = grow_store(p, cap, 0))) return rc;   // its keep half orders each replay
    while (B > 1 && sort_bytes(B, Ds_max, p->D, p->ns, tiles) > p->mem_limit - p->bytes) B >>= 1;
    if ((rc = alloc_sort(p, B, Ds_max))) return rc;
    {
        StepGeom gmax{};
        gmax.ns = p->ns;
        gmax.nseg = B * Ds_max;
        p->coll_parts = enum_partials(gmax);
        if ((rc = dalloc_t(p, &p->coll_part, (size_t)p->coll_parts * 24))) return rc;
    }
    if (p->cache == &p->own_cache) {
        p->own_cache.trim();
        p->recycle = false;
    }
    std::vector<momenti_report> R(nd);
    for (auto& r : R) {
        r.K = p->K; r.L_used = p->L; r.r = p->r; r.t_hash_ms = p->t_hash_ms; r.batch_reps = B;
        r.first_group_lo = p->K;
    }
    int64_t n_steps = 0, n_coll = 0, n_cand = 0;
    auto elapsed = [&]() { return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); };
    // answer for dimensionality index q from pool q at (i, J): TOP of snapshot st
    auto answer = [&](int q, int st, int i, int J, int code) -> int {
        PoolSet& ps = sets[q];
        const Snap& sn = ps.host_snaps[st];
        const int nt = std::min(sn.top_n, k), dq = d_lo + q;
        std::vector<VRec> tv(std::max(nt, 1));
        if (nt)
            HIP_OK(copy_sync(p, tv.data(), ps.snap_tops + (size_t)st * k, (size_t)nt * sizeof(VRec), hipMemcpyDeviceToHost));
        momenti_motif* o = out + (size_t)q * k;
        to_motifs(tv, nt, o);
        for (int u = 0; u < nt; ++u)
            o[u].fail_prob = std::exp(log_fail(o[u].dist_max, p->r, dq, i, J, p->K, p->L, p->m, p->o.stop_rule));
        n_out[q] = nt;
        status[q] = code;
        R[q].fail_bound = nt >= k ? o[k - 1].fail_prob : 1.0;
        if (code == MOMENTI_OK) { R[q].i_stop = i; R[q].j_stop = J; }
        if (code == MOMENTI_OK_PARTIAL) R[q].budget_round = i;
        R[q].n_steps = n_steps; R[q].n_collisions = n_coll; R[q].n_cand = R[q].n_verified = n_cand;
        R[q].peak_bytes = p->peak;
        R[q].t_search_ms = elapsed();
        return MOMENTI_OK;
    };
    const double elem_x = p->dtype == MOMENTI_F64 ? 8.0 : 4.0;
restart:
    for (int q = 0; q < nd; ++q)
        if (status[q] < 0) HIP_OK(launch_pool_reset(sets[q].ps, p->st));
    n_steps = 0;
    for (int i = p->K; i >= 1; --i) {
        for (int j0 = 0; j0 < p->L;) {
            int cur = 0;
            while (cur < nd && status[cur] >= 0) ++cur;
            if (cur == nd) return MOMENTI_OK;   // every dimensionality answered
            const int dcur = d_lo + cur, nact = nd - cur;
            const int Bc = std::min(B, p->L - j0);
            const int Ds = std::max(1, p->D - dcur + 1);
            StepGeom g;
            g.ns = p->ns; g.D = p->D; g.NF = p->NF; g.NL = p->NL; g.m = p->m;
            g.j0 = j0; g.Ds = Ds; g.nseg = Bc * Ds; g.i = i; g.K = p->K; g.i_lo = i;
            g.hashed = i > 4; g.dhi = d_hi; g.part = 0; g.nparts = 1;
            g.fq = second_stage_pays(p->D, dcur);
            int buf = 0;
            const double elems = (double)g.nseg * p->ns;
            const double kb = sort_keys_32(g) ? 4.0 : 8.0;
            const int kt = std::min(i + 1, p->K);
            const int nw = fp_words(p->D), nq = fq_words(p->D);
            // the fingerprint tables, with the histogram of the sort's pass 0
            HIP_OK(timed(p, KI_FPTABLE, (double)Bc * p->ns * (p->D * 8.0 + 4.0 * (nw + (g.fq ? nq : 0))), 0.0, [&] {
                return launch_fptable(p->H, g, Bc, p->fps, p->fq, p->sb, p->st);
            }));
            for (int pass = 0; pass < sort_passes(g); ++pass) {
                const double kin = pass == 0 ? 8.0 : kb;
                if (pass > 0)
                    HIP_OK(timed(p, KI_HIST, elems * kin, 0.0, [&] { return launch_hist(g, p->H, p->sb, pass, buf, p->st); }));
                HIP_OK(timed(p, KI_SCAN, 8.0 * g.nseg * 256.0 * p->sb.tiles, 0.0, [&] { return launch_scan(g, p->sb, p->st); }));
                HIP_OK(timed(p, KI_SCATTER, elems * (kin + (pass == 0 ? 0.0 : 4.0) + kb + 4.0), 0.0,
                             [&] { return launch_scatter(g, p->H, p->sb, pass, buf, p->st); }));
                buf ^= 1;
            }
            bool redo = false;
            for (g.part = 0; g.part < g.nparts && !redo; ++g.part) {
                HIP_OK(launch_zero(p->status, 64, p->st));
                HIP_OK(timed(p, KI_ENUM, 0.0, 0.0, [&] {
                    return launch_enum(g, p->sb, buf, p->H, p->fps, p->fq, kt, dcur, p->w, p->cand, p->cap,
                                       st_counters(p), p->coll_part, p->st);
                }));
                HIP_OK(timed(p, KI_VERIFY, 0.0, 0.0, [&] {
                    return launch_verify(p->cand, p->cap, st_counters(p), p->series, p->dtype, p->n, p->ns, p->D,
                                         p->w, dcur, p->mu, p->isig, p->vrec, p->st, nact);
                }));
                (void)elem_x;
                Counters cnt;
                HIP_OK(hipMemcpyAsync(p->host_status, p->status, sizeof(Counters), hipMemcpyDeviceToHost, p->st));
                HIP_OK(hipStreamSynchronize(p->st));
                std::memcpy(&cnt, p->host_status, sizeof cnt);
                prof_flush(p);
                if (cnt.n_units > p->sb.ucap)
                    return fail(MOMENTI_E_DEVICE, "%u tile rows queued, room for %u", cnt.n_units, p->sb.ucap);
                if (cnt.n_cand > p->cap) {
                    if (Bc > 1) {   // fewer repetitions per launch
                        B = std::max(1, Bc / 2);
                        redo = true;
                        break;
                    }
                    int np = g.nparts;   // else this repetition in parts
                    while ((uint64_t)np * p->cap < 2ull * cnt.n_cand * (uint64_t)g.nparts && np < (1 << 16)) np <<= 1;
                    if (np == g.nparts) return fail(MOMENTI_E_NOMEM, "%u candidates in one step exceed mem_limit", cnt.n_cand);
                    g.nparts = np;
                    g.part = -1;
                    continue;
                }
                if (g.part == 0) n_coll += (int64_t)cnt.n_coll;
                n_cand += cnt.n_cand;
                // every open dimensionality takes the records of its d
                for (int q = cur; q < nd; ++q) {
                    if (status[q] >= 0) continue;
                    pool_in(p, sets[q]);
                    rc = replay(p, p->vrec + (size_t)(q - cur) * p->cap, cnt.n_cand, p->keep, k,
                                (p->K - i) * p->L + j0, Bc, d_lo + q);
                    pool_out(p, sets[q]);
                    sets[q].ps = ps_block + q;
                    if (rc) return rc;
                }
            }
            if (redo) continue;
            // the stopping rule of every open dimensionality, step by step
            bool grow = false;
            for (int st = 0; st < Bc && !grow; ++st) {
                const int J = j0 + st + 1;
                ++n_steps;
                for (int q = cur; q < nd; ++q) {
                    if (status[q] >= 0) continue;
                    const Snap& sn = sets[q].host_snaps[st];
                    if (sn.top_n < k && sn.truncated) {   // pool q dropped what TOP needs
                        ++R[q].pool_overflow;
                        pool_in(p, sets[q]);
                        rc = grow_pool(p, sets[q].P * 2, k, B);
                        pool_out(p, sets[q]);
                        sets[q].ps = ps_block + q;
                        if (rc) return rc;
                        grow = true;
                        break;
                    }
                    if (sn.top_n == k &&
                        stop_holds(sn.dist_max, p->r, d_lo + q, i, J, p->K, p->L, p->m, p->o.stop_rule, delta_rule))
                        if ((rc = answer(q, st, i, J, MOMENTI_OK))) return rc;
                }
                if (!grow && ((p->o.max_steps > 0 && n_steps >= p->o.max_steps) ||
                              (p->o.max_ms > 0.0 && elapsed() >= p->o.max_ms))) {
                    for (int q = cur; q < nd; ++q)
                        if (status[q] < 0 && (rc = answer(q, st, i, J, MOMENTI_OK_PARTIAL))) return rc;
                    if (reps) std::copy(R.begin(), R.end(), reps);
                    return MOMENTI_OK;
                }
            }
            if (grow) goto restart;   // answered dimensionalities keep their answers
            j0 += Bc;
        }
    }
    // no step stopped for these: the exact answers
    for (int q = 0; q < nd; ++q) {
        if (status[q] >= 0) continue;
        pool_in(p, sets[q]);
        momenti_report Rq = R[q];
        rc = exact_fallback(p, d_lo + q, k, out + (size_t)q * k, &n_out[q], &Rq);
        pool_out(p, sets[q]);
        sets[q].ps = ps_block + q;
        if (rc) return rc;
        R[q] = Rq;
        R[q].fallback = 1;
        R[q].fail_bound = 0.0;
        R[q].n_steps = n_steps;
        status[q] = MOMENTI_OK_FALLBACK;
        R[q].t_search_ms = elapsed();
    }
    if (reps) std::copy(R.begin(), R.end(), reps);
    return MOMENTI_OK;
}

// ------------------------------------------------------------------ search without allocations
// The scratch area of momenti_search_noalloc: one per device, held until the
// process ends. In host code `scratch` names a host-side stand-in; its device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is ever handed to kernels or copies.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch area on device `dev` (made current for the
// lookup, then restored).
static int scratch_on(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return fail(MOMENTI_E_DEVICE, "device %d outside [0, %d)", dev, kMaxDevices);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIP_OK(hipGetDevice(&cur));
        if (cur != dev) HIP_OK(hipSetDevice(dev));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) HIP_OK(hipSetDevice(cur));
        if (e != hipSuccess || !ptr)
            return fail(MOMENTI_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MOMENTI_OK;
}

// The traversal buffers of a plan, set aside while momenti_search_noalloc runs.
struct SearchBuffers {
    SortBufs sb;
    int sb_nseg, sb_reps;
    uint32_t *fps, *fq;
    unsigned long long* coll_part;
    int64_t coll_parts;
    Cand* cand;
    VRec* vrec;
    uint32_t cap;
    VRec* store;
    uint32_t* keep;
    uint32_t store_cap;
    VRec* pools;
    int P;
    VRec* top;
    int top_k;
    unsigned char* status;
    ReplayCtl* rctl;
    Snap* snaps;
    VRec* snap_tops;
    int snap_steps, snap_k;
    unsigned char* host_status;
    Snap* host_snaps;
};

static SearchBuffers set_aside(momenti_plan* p)
{
    SearchBuffers b{p->sb, p->sb_nseg, p->sb_reps, p->fps, p->fq, p->coll_part, p->coll_parts, p->cand, p->vrec,
                    p->cap, p->store, p->keep, p->store_cap, p->pools, p->P, p->top, p->top_k, p->status, p->rctl,
                    p->snaps, p->snap_tops, p->snap_steps, p->snap_k, p->host_status, p->host_snaps};
    p->sb = SortBufs{};
    p->sb_nseg = p->sb_reps = 0;
    p->fps = p->fq = nullptr;
    p->coll_part = nullptr; p->coll_parts = 0;
    p->cand = nullptr; p->vrec = nullptr; p->cap = 0;
    p->store = nullptr; p->keep = nullptr; p->store_cap = 0;
    p->pools = nullptr; p->P = 0; p->top = nullptr; p->top_k = 0;
    p->status = nullptr; p->rctl = nullptr;
    p->snaps = nullptr; p->snap_tops = nullptr; p->snap_steps = p->snap_k = 0;
    p->host_status = nullptr; p->host_snaps = nullptr;
    return b;
}

static void put_back(momenti_plan* p, const SearchBuffers& b)
{
    p->sb = b.sb; p->sb_nseg = b.sb_nseg; p->sb_reps = b.sb_reps; p->fps = b.fps; p->fq = b.fq;
    p->coll_part = b.coll_part; p->coll_parts = b.coll_parts; p->cand = b.cand; p->vrec = b.vrec; p->cap = b.cap;
    p->store = b.store; p->keep = b.keep; p->store_cap = b.store_cap; p->pools = b.pools; p->P = b.P;
    p->top = b.top; p->top_k = b.top_k; p->status = b.status; p->rctl = b.rctl; p->snaps = b.snaps;
    p->snap_tops = b.snap_tops; p->snap_steps = b.snap_steps; p->snap_k = b.snap_k;
    p->host_status = b.host_status; p->host_snaps = b.host_snaps;
}

extern "C" int momenti_search_noalloc(momenti_plan* p, int32_t d, int32_t k, double delta, momenti_motif* out,
                                      int32_t* n_out, momenti_report* rep)
{
    g_err.clear();
    if (!p || !out || !n_out) return fail(MOMENTI_E_ARG, "NULL argument");
    void* base = nullptr;
    int rc = scratch_on(p->dev, &base);
    if (rc) return rc;
    HIP_OK(p->st ? hipStreamSynchronize(p->st) : hipDeviceSynchronize());   // earlier work on the plan is done
    const SearchBuffers kept = set_aside(p);
    const uint64_t limit = p->mem_limit, held = p->bytes, peak = p->peak;
    const bool prof_on = p->prof.on;
    p->arena = true;
    p->arena_base = (unsigned char*)base;
    p->mem_limit = kScratchBytes;
    p->bytes = 0;
    p->peak = 0;
    p->prof.on = false;   // no events are created during this call
    rc = momenti_search(p, d, k, delta, out, n_out, rep);
    // the call's work on the scratch area ends before the next call may use it
    const hipError_t e = p->st ? hipStreamSynchronize(p->st) : hipDeviceSynchronize();
    host_free(p, p->host_status);
    host_free(p, p->host_snaps);
    put_back(p, kept);
    p->arena = false;
    p->arena_base = nullptr;
    p->mem_limit = limit;
    p->bytes = held;
    p->peak = peak;
    p->prof.on = prof_on;
    if (rc >= 0 && e != hipSuccess) return fail(MOMENTI_E_DEVICE, "search without allocations: %s", hipGetErrorString(e));
    return rc;
}

// ------------------------------------------------------------------ autotuning
// The repetitions traversed per launch (B) change only the cost of a search:
// the ordered replay makes TOP after every step, the stop step and the answer
// independent of B. The tuner runs the search once per candidate B on the
// plan's index (after one untimed search for the allocations), checks that
// every answer is the same, and keeps the fastest B in the plan's options.
extern "C" int momenti_tune(momenti_plan* p, int32_t d, int32_t k, double delta, const int32_t* cands,
                            int32_t ncand, int32_t* best_reps, double* best_ms)
{
    g_err.clear();
    if (!p || !cands || !best_reps) return fail(MOMENTI_E_ARG, "NULL argument");
    if (ncand < 1 || ncand > 16) return fail(MOMENTI_E_ARG, "ncand=%d outside [1, 16]", ncand);
    if (!p->hashed) return fail(MOMENTI_E_STATE, "momenti_hash has not been called");
    if (p->arena) return fail(MOMENTI_E_STATE, "not available without allocations");
    const int saved = p->o.batch_reps;
    std::vector<momenti_motif> ref((size_t)std::max(k, 1)), out((size_t)std::max(k, 1));
    momenti_report rref{}, r{};
    int nref = -1, rcref = 0, n = 0;
    double bt = std::numeric_limits<double>::infinity();
    int bB = 0;
    std::vector<int> tried;
    for (int q = -1; q < ncand; ++q) {
        const int B = q < 0 ? cands[0] : cands[q];
        if (B < 1 || B > 64) {
            p->o.batch_reps = saved;
            return fail(MOMENTI_E_ARG, "candidate batch size %d outside [1, 64]", B);
        }
        p->o.batch_reps = B;
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = momenti_search(p, d, k, delta, out.data(), &n, &r);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rc < 0) {
            p->o.batch_reps = saved;
            return rc;
        }
        if (q < 0) {   // the untimed first search: the reference answer
            ref = out;
            nref = n;
            rref = r;
            rcref = rc;
            continue;
        }
        bool same = rc == rcref && n == nref && r.i_stop == rref.i_stop && r.j_stop == rref.j_stop;
        for (int u = 0; same && u < n; ++u)
            same = out[u].a == ref[u].a && out[u].b == ref[u].b && out[u].dist_d == ref[u].dist_d &&
                   out[u].dist_max == ref[u].dist_max;
        if (!same) {
            p->o.batch_reps = saved;
            return fail(MOMENTI_E_DEVICE, "the answer with %d repetitions per launch differs from the one with %d",
                        B, cands[0]);
        }
        // B as the search used it (the memory budget may lower it)
        if (std::find(tried.begin(), tried.end(), r.batch_reps) != tried.end()) continue;
        tried.push_back(r.batch_reps);
        if (ms < bt) {
            bt = ms;
            bB = r.batch_reps;
        }
    }
    p->o.batch_reps = bB;
    *best_reps = bB;
    if (best_ms) *best_ms = bt;
    return MOMENTI_OK;
}

extern "C" int momenti_topk(const void* series, int32_t dtype, int64_t n, int32_t D, int32_t w,
                            int32_t d, int32_t k, double delta, uint64_t mem_limit,
                            const momenti_opts* opts, momenti_motif* out, int32_t* n_out,
                            momenti_report* rep)
{
    momenti_plan* p = nullptr;
    int rc = momenti_prepare(&p, n, D, w, dtype, mem_limit, opts);
    if (rc) return rc;
    rc = momenti_hash(p, series);
    if (rc == MOMENTI_OK) rc = momenti_search(p, d, k, delta, out, n_out, rep);
    momenti_destroy(p);
    return rc;
}

extern "C" int momenti_topk_batch(const momenti_job* jobs, int32_t count, uint64_t mem_limit,
                                  const momenti_opts* opts, int32_t workers, momenti_motif* out,
                                  int32_t* n_out, int32_t* status, momenti_report* reps)
{
    g_err.clear();
    if (count < 0) return fail(MOMENTI_E_ARG, "count=%d is negative", count);
    if (count == 0) return MOMENTI_OK;
    if (!jobs || !out || !n_out || !status) return fail(MOMENTI_E_ARG, "NULL argument");
    if (workers < 1 || workers > 16) return fail(MOMENTI_E_ARG, "workers=%d outside [1, 16]", workers);
    std::vector<int64_t> off((size_t)count + 1, 0);
    for (int q = 0; q < count; ++q) {
        if (jobs[q].k < 1 || jobs[q].k > 4096) return fail(MOMENTI_E_ARG, "job %d: k=%d outside [1, 4096]", q, jobs[q].k);
        off[q + 1] = off[q] + jobs[q].k;
    }
    momenti_opts base;
    if (opts) base = *opts; else momenti_default_opts(&base);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MOMENTI_E_DEVICE, "no HIP device");
    std::vector<std::string> errs((size_t)count);
    std::atomic<int> next{0};
    const int nw = std::min<int>(workers, count);
    auto worker = [&]() {
        (void)hipSetDevice(dev);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
        BlockCache cache;
        momenti_opts o = base;
        o.stream = st;
        for (int q; (q = next.fetch_add(1)) < count;) {
            const momenti_job& jb = jobs[q];
            momenti_report rr{};
            n_out[q] = 0;
            auto run = [&]() {
                momenti_plan* p = nullptr;
                int r = prepare_impl(&p, jb.n, jb.D, jb.w, jb.dtype, mem_limit, &o, &cache);
                if (r == MOMENTI_OK) {
                    r = momenti_hash(p, jb.series);
                    if (r == MOMENTI_OK) r = momenti_search(p, jb.d, jb.k, jb.delta, out + off[q], &n_out[q], &rr);
                    momenti_destroy(p);
                }
                return r;
            };
            int rc = run();
            if (rc == MOMENTI_E_NOMEM) {
                // blocks reused from earlier series can be larger than asked
                // for, and a series close to its limit then runs out: run it
                // again on exact, fresh blocks, as a series on its own would
                cache.trim();
                cache.exact = true;
                rr = momenti_report{};
                n_out[q] = 0;
                rc = run();
                cache.exact = false;
            }
            status[q] = rc;
            if (reps) reps[q] = rr;
            if (rc < 0) errs[q] = g_err;
        }
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    };
    std::vector<std::thread> pool;
    for (int q = 1; q < nw; ++q) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
    for (int q = 0; q < count; ++q)
        if (status[q] < 0) {
            g_err = "job " + std::to_string(q) + ": " + errs[q];
            return status[q];
        }
    return MOMENTI_OK;
}
