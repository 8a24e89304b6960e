/*
 * momenti.h -- C ABI of an MI355X (gfx950) implementation of the MOMENTI
 * top-k multidimensional motif search (Ceccarello, Monaco, Silvestri,
 * "MOMENTI: Scalable Motif Mining in Multidimensional Time Series", PVLDB 18(10), 2025).
 *
 * Problem (section 3.1, definition "top-k multidimensional motifs"): given a
 * D-dimensional series of length n, a window length w, a motif dimensionality
 * d and a count k, return the k pairs of windows (a, b) with the smallest
 * d-dimensional distance dist_d (definition "d-dimensional distance": the sum
 * of the d smallest per-dimension z-normalised Euclidean distances, Eq. zned),
 * no two of them overlapping.
 *
 * Method (Algorithm 1 with Algorithm 2 and sections 6.1-6.2): every window of
 * every dimension is hashed with K concatenated discretised random projections
 * (Eq. drp) in L tensored repetitions; rounds i = K..1 scan the pairs whose
 * hash prefixes of length i collide in at least d dimensions, verify them
 * under dist_d, and stop as soon as the probability of having missed a better
 * pair is at most delta (Lemma 6.1 / Eq. probnotcolliding).
 *
 * Conventions
 *   - Windows are 0-based: window a covers series[f][a .. a+w-1], a in [0, n-w].
 *   - The series is [D][n], row-major, each dimension contiguous, float64 or
 *     float32, in host or device memory (momenti_opts.series_on_device). The
 *     caller owns it; the library only reads it during momenti_hash (or copies
 *     it when it is on the host).
 *   - Every function returns a status code (MOMENTI_OK ... MOMENTI_E_*); no
 *     exception crosses the boundary. On error momenti_last_error() returns a
 *     thread-local message.
 *   - A plan is not thread-safe; distinct plans may be used from distinct threads.
 *   - All GPU work runs on opts.stream (a hipStream_t; NULL = the default stream).
 */
#ifndef MOMENTI_H
#define MOMENTI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define MOMENTI_OK 0             /* the search stopped under the stopping rule */
#define MOMENTI_OK_FALLBACK 1    /* no round stopped: the exact all-pairs answer was returned */
#define MOMENTI_OK_PARTIAL 2     /* opts.max_pairs ended the search before the stopping rule held:
                                    out holds TOP as it stood (an anytime answer, no guarantee) */
#define MOMENTI_E_ARG (-1)       /* invalid argument (see each function) */
#define MOMENTI_E_NOMEM (-2)     /* mem_limit too small for the smallest index, or a device allocation failed */
#define MOMENTI_E_DEVICE (-3)    /* a HIP runtime call failed */
#define MOMENTI_E_STATE (-4)     /* call out of order (e.g. search before hash) */
#define MOMENTI_E_UNSUPPORTED (-5) /* an input size beyond what the index layout can address */

/* Series element type. */
#define MOMENTI_F64 0
#define MOMENTI_F32 1

/* Arithmetic of the projection a . x of Eq. drp (the hash). Statistics and
 * the dist_d verification are always float64. FP64 and F32 are the plain
 * method; BF16 and FP8 (e4m3, the z-normalisation being the per-window
 * scaling) change the hash function itself and are reported against FP64. */
#define MOMENTI_PROJ_F64 0
#define MOMENTI_PROJ_F32 1
#define MOMENTI_PROJ_BF16 2
#define MOMENTI_PROJ_FP8 3

/* Stopping rule. TENSOR: Lemma 6.1 (the bound for the tensored index,
 * P_t(i', J') = (1 - p^ceil(i'))^(J' div m) (1 - p^floor(i'))^(J' mod m)),
 * where a half contributing no symbol to the prefix (floor(i') = 0 in round
 * 1) gives the factor 1. TENSOR_LITERAL: the same bound with that factor
 * taken literally, (1 - p^0)^x = 0, which stops round 1 as soon as |TOP| = k.
 * LEMMA52: Eq. probnotcolliding of Lemma 5.2 ((1 - p^i)^J (1 - p^(i+1))^(L-J)). */
#define MOMENTI_STOP_TENSOR 0
#define MOMENTI_STOP_LEMMA52 1
#define MOMENTI_STOP_TENSOR_LITERAL 2
/* RIGOROUS: a bound that follows from the tensored index itself. Repetitions
 * that share a half-function are not independent, so Lemma 6.1's product is
 * not obviously an upper bound. Each symbol of a half-function collides with
 * probability >= p = P(dist_max)^d (Eq. eucl-collision-probability over the d
 * dimensions), independently, so each half-function collides at least to a
 * geometric depth (P(depth >= s) = p^s); the probability that no visited
 * repetition (left j div m, right j mod m) reached the prefix length of its
 * round, with those depths, is computed exactly (a finite sum over which
 * right functions reach the two depths involved). */
#define MOMENTI_STOP_RIGOROUS 3

/* Meaning of delta (opts.delta_mode). PER_MOTIF: each returned motif is the
 * true one with probability >= 1 - delta (Lemma 5.3). JOINT: all k at once
 * (Lemma 5.4: the rule runs with delta / k). */
#define MOMENTI_DELTA_PER_MOTIF 0
#define MOMENTI_DELTA_JOINT 1

typedef struct momenti_plan momenti_plan;   /* opaque, owned by the library */

typedef struct {
    uint64_t seed;            /* seed of the random projections (Philox4x32-10 streams) */
    int32_t K;                /* maximum concatenations: even, 2..8 (default 8, section 7 defaults) */
    int32_t L;                /* maximum repetitions, 1..256 (default 200; 256 makes the
                                 128 hash columns the projection tile holds) */
    double r;                 /* quantisation width of Eq. drp; <= 0 estimates it (section 6.1) */
    double r_scale;           /* with r <= 0: use r_scale times the estimate (<= 0 means 1).
                                 Section 6.1 leaves r free (any r keeps the guarantee; section
                                 7.4 varies it): a larger r makes the stopping rule hold at
                                 longer prefixes for the same distances, at the price of more
                                 collisions per round */
    int32_t proj;             /* MOMENTI_PROJ_* (default F32) */
    int32_t stop_rule;        /* MOMENTI_STOP_* (default TENSOR) */
    int32_t series_on_device; /* 1: the series pointer passed to momenti_hash is device memory */
    int32_t pool_size;        /* verified pairs kept on the device; 0 = max(4096, 128 k) */
    int32_t batch_reps;       /* repetitions traversed per launch; 0 = chosen from mem_limit */
    int32_t profile;          /* 1: time every kernel launch with HIP events (momenti_get_profile);
                                 2: time only the pair enumeration (the dominant kernel, least
                                 overhead); 0: off */
    double merge_pairs;       /* rounds join the first round group (one sort) while their colliding
                                 pairs are estimated at most this many per segment element;
                                 <= 0 means 8 (about the cost of one sort pass) */
    double max_pairs;         /* work budget: a round group whose colliding pairs are estimated
                                 (from one probed repetition) above this is not traversed and
                                 the search returns MOMENTI_OK_PARTIAL; <= 0: no budget */
    void* stream;             /* hipStream_t, NULL = default stream */
    int32_t delta_mode;       /* MOMENTI_DELTA_PER_MOTIF (default) or MOMENTI_DELTA_JOINT */
    int32_t max_steps;        /* anytime budget: after this many (round, repetition) steps the
                                 search returns TOP as it stands (MOMENTI_OK_PARTIAL, each motif
                                 with its failure bound); <= 0: none */
    double max_ms;            /* the same budget in wall-clock milliseconds of the traversal,
                                 checked after every replayed batch of repetitions; <= 0: none */
} momenti_opts;

/* Per-kernel totals collected when opts.profile is set: launches, summed
 * device time, and the algorithmic bytes moved / flops done by those launches
 * (what the method must read and write, not cache traffic). */
typedef struct {
    char name[24];        /* kernel family (stats, proj, sort_scatter, enum, ...) */
    int64_t launches;
    double ms;            /* summed launch durations, HIP events on the plan's stream */
    double bytes;         /* algorithmic device-memory bytes (minimum traffic) */
    double flops;         /* algorithmic operations: floating-point for stats, proj and
                             verify; for enum the integer screen operations, 5 per
                             fingerprint word and one compare for every pair scanned */
} momenti_kprof;

typedef struct {
    int64_t a, b;             /* window starts, a < b, 2 (b - a) > w */
    double dist_d;            /* definition "d-dimensional distance" */
    double dist_max;          /* Eq. distdmax: largest distance among the chosen dimensions */
    uint64_t dims[2];         /* bit f set for each chosen dimension (D <= 128) */
    double fail_prob;         /* the stopping rule's bound, at the step where the search ended,
                                 on the probability that a pair at this motif's dist_max was
                                 never a candidate (Lemma 5.2 / 6.1 with p = P(dist_max)^d; the
                                 anytime error probability); 0 for an exact answer */
} momenti_motif;

typedef struct {
    double t_hash_ms;         /* device time of statistics + projection (+ r estimate) */
    double t_search_ms;       /* wall time of the traversal */
    int32_t i_stop, j_stop;   /* round (prefix length) and repetition (1-based) at which STOP held; 0 on fallback */
    int32_t L_used, K;        /* repetitions after the memory cap; concatenations */
    double r;                 /* quantisation width in use */
    int64_t n_steps;          /* (round, repetition) steps traversed */
    int64_t n_collisions;     /* pairs of windows with equal prefixes in the traversed segments
                                 (one dimension each; trivial matches included) */
    int64_t n_cand;           /* candidate pairs emitted (W >= d, first time at this repetition) */
    int64_t n_verified;       /* dist_d evaluations */
    uint64_t peak_bytes;      /* device bytes held by the plan at its peak */
    int32_t fallback;         /* 1 when the exact all-pairs answer was returned */
    int32_t pool_overflow;    /* times the verified-pair pool had to be enlarged */
    int32_t batch_reps;       /* repetitions per launch actually used */
    int32_t first_group_lo;   /* rounds K .. first_group_lo were traversed from one sort */
    int32_t budget_round;     /* MOMENTI_OK_PARTIAL: the highest round not traversed; else 0 */
    int32_t max_run;          /* most windows sharing a prefix in one segment, among the runs
                                 that crossed a 64-window boundary (enumerated in tiles) */
    int32_t group_splits;     /* round groups whose verified records would have exceeded
                                 mem_limit, traversed again one round at a time */
    int32_t step_parts;       /* most parts one repetition was enumerated in (its candidates did
                                 not fit in mem_limit at once); 0 when none was */
    double fail_bound;        /* the rule's bound for TOP's k-th motif at the last step traversed
                                 (<= delta, or delta / k, when the rule held; 1 when TOP held
                                 fewer than k motifs; 0 for an exact answer) */
} momenti_report;

/* Fill *o with the defaults (K = 8, L = 200, r estimated, F32 projection,
 * TENSOR rule, delta-independent; seed 0x5EED). */
void momenti_default_opts(momenti_opts* o);

/* Plan a search over series of length n (>= w + 1) with D (1..128) dimensions
 * and window w (4..8192; with a BF16 projection at most 7616 for 128 hash
 * columns, since its work-group keeps four shifted copies of its series tile
 * and two chunks of projection rows in one CU's 160 KiB of LDS: E_ARG names
 * the limit). mem_limit bounds the device bytes the plan may hold
 * (series copy, statistics, index, traversal buffers); the number of
 * repetitions is the largest L' <= opts.L whose index fits (index size
 * O(K L D n), Theorem "space"):
 *   fixed = n D s + 16 n_s D + 32 n_s D + 64 MiB   (s = 8 for float64, 4 for float32 series)
 *   index(L') = 4 n_s D (ceil(L'/m') + min(L', m')),  m' = ceil(sqrt(L'))
 * L_used = max{L' : fixed + index(L') <= mem_limit}, E_NOMEM when L' = 1 does
 * not fit. dtype (MOMENTI_F64 / MOMENTI_F32) is the element type of the
 * series later passed to momenti_hash. Draws the random projections on the
 * host (Philox4x32-10 streams of opts.seed). *out receives a new plan.
 * Errors: E_ARG (bad sizes or options), E_NOMEM, E_DEVICE. */
int momenti_prepare(momenti_plan** out, int64_t n, int32_t D, int32_t w, int32_t dtype,
                    uint64_t mem_limit, const momenti_opts* opts /* NULL = defaults */);

/* Index construction (Algorithm 1 first loop, section 6.1): rolling window
 * statistics, the r estimate (unless fixed by opts.r), and the tensored hash
 * index of every window of every dimension. series: [D][n] of the plan's
 * dtype, host or device memory per opts.series_on_device (device memory is
 * borrowed until momenti_destroy). May be called again with new data; until
 * such a call succeeds the plan has no index (searches return E_STATE).
 * Errors: E_ARG (null series, or a value that is NaN or infinite: the message
 * names the first, series[f][t]), E_NOMEM, E_DEVICE. */
int momenti_hash(momenti_plan* p, const void* series);

/* Index traversal (Algorithm 1 rounds i = K..1, repetitions j = 1..L, with
 * Algorithm 2): writes up to k motifs to out (caller-owned, capacity >= k) in
 * increasing (dist_d, a, b) order and their count to *n_out (< k only when
 * fewer non-overlapping non-trivial pairs exist). rep may be NULL.
 * d in [1, D], k in [1, 4096], delta in (0, 1). The traversal buffers stay
 * with the plan after the call; the next search reuses those of the sizes it
 * needs and frees the others (all within mem_limit).
 * Returns MOMENTI_OK, MOMENTI_OK_FALLBACK (exact answer, no step stopped),
 * MOMENTI_OK_PARTIAL (opts.max_pairs reached: TOP so far, possibly fewer than
 * k pairs), or E_ARG, E_STATE (momenti_hash not called), E_NOMEM, E_DEVICE,
 * E_UNSUPPORTED (more windows per batch of segments than 32-bit positions hold). The exact
 * answer of the fallback covers every window count: short series stream every pair through
 * the verifier, longer ones sweep the diagonals of the pair matrix. */
int momenti_search(momenti_plan* p, int32_t d, int32_t k, double delta, momenti_motif* out,
                   int32_t* n_out, momenti_report* rep);

/* momenti_search for callers that cannot allocate device memory (code under
 * stream capture, serving loops or harnesses that forbid hipMalloc): every
 * traversal buffer is carved from a scratch area of 256 MiB that the library
 * keeps on each device it runs on (a static device array, held until the
 * process ends); host staging uses plain memory. Arguments, results and
 * report are those of momenti_search on the same plan (report.peak_bytes is
 * the part of the scratch area used); the plan's own traversal buffers are
 * left as they are. The call makes no hipMalloc, hipFree or hipHostMalloc;
 * it synchronises the plan's stream before and after. Every call on one
 * device shares that device's area, which keeps the last call's contents:
 * calls that overlap on one device race, so run them one at a time per
 * device. Errors as momenti_search, plus E_NOMEM when the traversal of this
 * input does not fit in the scratch area (momenti_search then allocates what
 * it needs). */
int momenti_search_noalloc(momenti_plan* p, int32_t d, int32_t k, double delta, momenti_motif* out,
                           int32_t* n_out, momenti_report* rep);

/* Several dimensionalities in one traversal (section 6.3): the top-k motifs
 * of every d in [d_lo, d_hi] (1 <= d_lo <= d_hi <= D). Each d has its own
 * pool; one verification of a candidate gives its distance for every d, and
 * the index is enumerated for the smallest d not yet answered, so a d stops
 * at the same step, with the same answer, as momenti_search(p, d, ...) with
 * the same plan (single-round traversal; the pairs counted are the same).
 * out (caller-owned, (d_hi - d_lo + 1) * k motifs) receives d's motifs at
 * offset (d - d_lo) * k; n_out[d - d_lo] their count; status[d - d_lo] what
 * momenti_search would return for d (MOMENTI_OK, _OK_FALLBACK or
 * _OK_PARTIAL); reps (NULL or one report per d) the report of d. Options
 * as momenti_search (max_steps and max_ms end every open d at once;
 * max_pairs and tracing are not applied). Returns MOMENTI_OK or an error
 * (E_STATE also for a plan in scratch mode). */
int momenti_search_multi(momenti_plan* p, int32_t d_lo, int32_t d_hi, int32_t k, double delta,
                         momenti_motif* out, int32_t* n_out, int32_t* status, momenti_report* reps);

/* Autotuning of the repetitions traversed per launch (opts.batch_reps),
 * which changes the cost of a search but not its steps or answer (the
 * verified pairs are replayed in step order). Runs momenti_search(p, d, k,
 * delta) once untimed, then once per candidate cands[0 .. ncand) (1 .. 64,
 * ncand 1 .. 16), checks that every answer and stop step equals the first,
 * and keeps the fastest in the plan's options (later searches use it).
 * best_reps receives it (as the search used it: mem_limit may lower a
 * candidate), best_ms (nullable) its search time. Returns MOMENTI_OK, an
 * error of momenti_search, E_DEVICE if two answers differ, E_STATE for a plan
 * in scratch mode. */
int momenti_tune(momenti_plan* p, int32_t d, int32_t k, double delta, const int32_t* cands, int32_t ncand,
                 int32_t* best_reps, double* best_ms);

/* One call: prepare + hash + search + destroy. Arguments as above. */
int momenti_topk(const void* series, int32_t dtype, int64_t n, int32_t D, int32_t w, int32_t d,
                 int32_t k, double delta, uint64_t mem_limit, const momenti_opts* opts,
                 momenti_motif* out, int32_t* n_out, momenti_report* rep);

/* One independent series of a batch (momenti_topk_batch). series is [D][n],
 * f32 or f64 (dtype), on the host or the device as opts->series_on_device
 * says; it is borrowed for the duration of the call. */
typedef struct {
    const void* series;
    int64_t n;
    int32_t dtype;            /* MOMENTI_F64 or MOMENTI_F32 */
    int32_t D, w, d, k;
    double delta;
} momenti_job;

/* Many independent series (e.g. a fleet of sensors): job q is run exactly as
 * momenti_topk(jobs[q]..., mem_limit, opts) would run it, with identical
 * results; up to `workers` (1..16) jobs are in flight at once, each worker on
 * its own stream with device blocks reused from one series to the next.
 * mem_limit applies to each job (so up to workers x mem_limit are held);
 * opts->stream is ignored. Device series must be ready when this is called.
 * out receives job q's motifs at offset k_0 + ... + k_{q-1} (caller-owned,
 * room for the sum of the k); n_out[q], status[q] and (if reps is not NULL)
 * reps[q] receive what momenti_topk would return for it. Returns MOMENTI_OK
 * when no job failed, else the first failing job's status (every job is
 * still attempted; momenti_last_error names the job). */
int momenti_topk_batch(const momenti_job* jobs, int32_t count, uint64_t mem_limit,
                       const momenti_opts* opts, int32_t workers, momenti_motif* out,
                       int32_t* n_out, int32_t* status, momenti_report* reps);

/* Release every resource of the plan (NULL is ignored). */
void momenti_destroy(momenti_plan* p);

/* Message of the last error on this thread ("" when none). */
const char* momenti_last_error(void);

/* ---- inspection (used by tests and tools; all copies are synchronous) ---- */

/* Quantisation width, repetitions in use, left/right half-functions. */
int momenti_get_params(const momenti_plan* p, double* r, int32_t* L_used, int32_t* n_left,
                       int32_t* n_right);

/* Window statistics [D][n_s] (float64): mean and 1/sigma (0 for a flat window,
 * sigma <= 1e-8 |mean|). Host buffers of `count` = D * n_s elements. */
int momenti_get_stats(momenti_plan* p, double* mu, double* inv_sigma, size_t count);

/* The index: hash words [D][n_left + n_right][n_s] (uint32), one word per
 * half-function holding its K/2 one-byte symbols, position 0 most significant
 * (symbol = (floor((a.x + b)/r) + 128) mod 256, Eq. drp). Host buffer. */
int momenti_get_hashes(momenti_plan* p, uint32_t* dst, size_t count);

/* The index words of `count` consecutive windows a0 .. a0 + count - 1 of
 * dimension f: dst is [n_left + n_right][count] (uint32, host). For sampling
 * a large index without copying it whole. Errors: E_ARG (range outside the
 * index), E_STATE (no index yet). */
int momenti_get_hash_words(momenti_plan* p, int32_t f, int64_t a0, int64_t count, uint32_t* dst);

/* Replace the index by words computed elsewhere (same layout), e.g. to
 * traverse a reference index. Host buffer. Marks the plan hashed; the
 * statistics must already exist (momenti_hash called once). */
int momenti_set_hashes(momenti_plan* p, const uint32_t* src, size_t count);

/* Record the traversal of the next momenti_search in host buffers (NULL
 * disables): cand receives triples (step, a, b) of every emitted candidate,
 * step = (K - i) L + (J - 1); top_size[step] the size of TOP after the step
 * (-1 if not reached); top_pairs[step][k][2] its pairs. cand_count receives
 * the number of candidates (may exceed cand_cap: the trace is then cut). */
int momenti_set_trace(momenti_plan* p, int64_t* cand, int64_t cand_cap, int64_t* cand_count,
                      int32_t* top_size, int64_t* top_pairs, int64_t steps_cap, int32_t k_cap);

/* Copy up to cap per-kernel profile records (see momenti_kprof) accumulated
 * since the plan was prepared or the profile was last cleared; *n gets the
 * number of kernels. clear != 0 resets the totals afterwards. */
int momenti_get_profile(momenti_plan* p, momenti_kprof* out, int32_t cap, int32_t* n, int32_t clear);

/* Change the profiling mode of a prepared plan (values as opts.profile);
 * totals already collected are kept. */
int momenti_set_profile(momenti_plan* p, int32_t mode);

#ifdef __cplusplus
}
#endif

#endif /* MOMENTI_H */
