/*
 * CPU oracle for the MOMENTI motif search (Ceccarello, Monaco, Silvestri,
 * "MOMENTI: Scalable Motif Mining in Multidimensional Time Series",
 * PVLDB 18(10), 2025).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU library shares no
 * code, header or table with it, and it never receives a value computed on
 * the GPU.
 *
 * Everything here is plain double precision, written to be checked against
 * the paper by eye: no blocking, no fusion, no reordering. It is compiled
 * with -ffp-contract=off, so every expression is evaluated as written (no
 * fused multiply-add).
 *
 * Parts:
 *   O1  exact top-k motifs by the definitions of section 3.1 (brute force);
 *       o1fast.c gives the same answer for long inputs (a diagonal sweep
 *       used as a filter, every kept pair recomputed by these definitions);
 *   O2  the LSH search of Algorithm 1 with the stopping rule of Algorithm 2 /
 *       Lemma 6.1, the tensored index of section 6.1 and the r heuristic of
 *       section 6.1, step after step with an unbounded set of verified pairs.
 *
 * Indices are 0-based: window a covers x[a .. a+w-1], a in [0, n-w].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The library is built twice from this file: sequentially (the checker the
 * tests use) and with OpenMP (the CPU baseline the benchmark times, all host
 * cores). The parallel loops only split independent work (dimensions, the
 * distances of distinct pairs); every result is the same in both builds. */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                   */
/* The paper only says that a and b are drawn at random (Eq. drp); the      */
/* streams below are this implementation's reading.                          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t purpose,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0, 1) from two 32-bit words (hi first). */
static double uniform53(uint32_t hi, uint32_t lo)
{
    uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

/* Standard normal by Box-Muller (cosine branch) from one Philox block. */
double orc_gauss(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t purpose)
{
    uint32_t o[4];
    draw(seed, c0, c1, c2, purpose, o);
    double u1 = 1.0 - uniform53(o[0], o[1]);   /* (0, 1] */
    double u2 = uniform53(o[2], o[3]);         /* [0, 1) */
    double radius = sqrt(-2.0 * log(u1));
    double angle = 6.283185307179586 * u2;
    return radius * cos(angle);
}

double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t purpose)
{
    uint32_t o[4];
    draw(seed, c0, c1, c2, purpose, o);
    return uniform53(o[0], o[1]);
}

enum { STREAM_PROJ = 0, STREAM_OFFSET = 1, STREAM_RVEC = 2, STREAM_RWIN = 3 };

/* ------------------------------------------------------------------------ */
/* Section 3.1: subsequences, mean, standard deviation, z-normalisation.     */
/* ------------------------------------------------------------------------ */

/* A window whose standard deviation is negligible next to its mean is treated
 * as flat and its z-normalised form is all zeros (the paper does not say what
 * happens when sigma = 0). */
#define ORC_FLAT_REL 1e-8

/* Mean and population standard deviation of x[a .. a+w-1] (Eq. zned uses
 * mu and sigma of each subsequence). Two passes, sequential sums. */
void orc_window_stats(const double* x, int32_t w, double* mu_out, double* sigma_out, int32_t* flat_out)
{
    double s = 0.0;
    for (int32_t t = 0; t < w; ++t) s = s + x[t];
    double mu = s / (double)w;
    double m2 = 0.0;
    for (int32_t t = 0; t < w; ++t) {
        double dlt = x[t] - mu;
        m2 = m2 + dlt * dlt;
    }
    double sigma = sqrt(m2 / (double)w);
    *mu_out = mu;
    *sigma_out = sigma;
    *flat_out = (sigma <= ORC_FLAT_REL * fabs(mu)) ? 1 : 0;
}

/* Stats of every window of every dimension. x is [D][n]; outputs [D][n_s]. */
void orc_stats(const double* x, int64_t n, int32_t D, int32_t w,
               double* mu, double* sigma, int32_t* flat)
{
    int64_t ns = n - w + 1;
    for (int32_t f = 0; f < D; ++f)
        for (int64_t a = 0; a < ns; ++a)
            orc_window_stats(x + (int64_t)f * n + a, w, &mu[f * ns + a], &sigma[f * ns + a],
                             &flat[f * ns + a]);
}

/* The z-normalised window (x - mu) / sigma, or zeros for a flat window. */
static void znorm(const double* x, int32_t w, double* out)
{
    double mu, sigma;
    int32_t flat;
    orc_window_stats(x, w, &mu, &sigma, &flat);
    for (int32_t t = 0; t < w; ++t) out[t] = flat ? 0.0 : (x[t] - mu) / sigma;
}

/* Eq. zned: z-normalised Euclidean distance of two windows. */
double orc_dist(const double* xa, const double* xb, int32_t w)
{
    double* za = (double*)malloc(sizeof(double) * (size_t)w);
    double* zb = (double*)malloc(sizeof(double) * (size_t)w);
    znorm(xa, w, za);
    znorm(xb, w, zb);
    double s = 0.0;
    for (int32_t t = 0; t < w; ++t) {
        double dlt = za[t] - zb[t];
        s = s + dlt * dlt;
    }
    free(za);
    free(zb);
    return sqrt(s);
}

/* Definition "d-dimensional distance" and Eq. distdmax: the d dimensions with
 * the smallest per-dimension distances (ties to the lower dimension index),
 * their sum, and the largest of them. dims_mask gets bit f set for each
 * chosen dimension (D <= 128). */
void orc_distd(const double* x, int64_t n, int32_t D, int32_t w, int64_t a, int64_t b, int32_t d,
               double* dist_d, double* dist_max, uint64_t dims_mask[2], double* per_dim /* [D] or NULL */)
{
    double* df = (double*)malloc(sizeof(double) * (size_t)D);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
    for (int32_t f = 0; f < D; ++f) {
        df[f] = orc_dist(x + (int64_t)f * n + a, x + (int64_t)f * n + b, w);
        order[f] = f;
        if (per_dim) per_dim[f] = df[f];
    }
    /* insertion sort of dimension indices by (distance, index) */
    for (int32_t u = 1; u < D; ++u) {
        int32_t v = order[u];
        int32_t q = u - 1;
        while (q >= 0 && (df[order[q]] > df[v] || (df[order[q]] == df[v] && order[q] > v))) {
            order[q + 1] = order[q];
            --q;
        }
        order[q + 1] = v;
    }
    double s = 0.0;
    dims_mask[0] = 0;
    dims_mask[1] = 0;
    for (int32_t u = 0; u < d; ++u) {
        s = s + df[order[u]];
        dims_mask[order[u] >> 6] |= (uint64_t)1 << (order[u] & 63);
    }
    *dist_d = s;
    *dist_max = df[order[d - 1]];
    free(df);
    free(order);
}

/* ------------------------------------------------------------------------ */
/* Top-k motifs (definition "top-k multidimensional motifs").                */
/* A pair (a, b), a < b, is a trivial match when |a - b| <= w/2, i.e.         */
/* 2|a - b| <= w (exclusion zone epsilon = w/2). The k motifs are chosen      */
/* greedily in increasing (dist_d, a, b) order, skipping any pair with an    */
/* endpoint inside the exclusion zone of an endpoint of an already chosen    */
/* motif, so that no two motifs overlap.                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t a, b;
    double dist_d, dist_max;
    uint64_t dims[2];
} orc_motif;

static int motif_cmp(const void* p, const void* q)
{
    const orc_motif* x = (const orc_motif*)p;
    const orc_motif* y = (const orc_motif*)q;
    if (x->dist_d < y->dist_d) return -1;
    if (x->dist_d > y->dist_d) return 1;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

static int trivial(int64_t u, int64_t v, int32_t w)
{
    int64_t g = u > v ? u - v : v - u;
    return 2 * g <= (int64_t)w;
}

/* Greedy selection over pairs already sorted by (dist_d, a, b). */
static int32_t greedy(const orc_motif* sorted, int64_t count, int32_t k, int32_t w, orc_motif* out)
{
    int32_t got = 0;
    for (int64_t e = 0; e < count && got < k; ++e) {
        const orc_motif* c = &sorted[e];
        int ok = 1;
        for (int32_t s = 0; s < got && ok; ++s) {
            if (trivial(c->a, out[s].a, w) || trivial(c->a, out[s].b, w) ||
                trivial(c->b, out[s].a, w) || trivial(c->b, out[s].b, w))
                ok = 0;
        }
        if (ok) out[got++] = *c;
    }
    return got;
}

/* O1: exact top-k by enumerating every non-trivial pair. Returns the number
 * of motifs found (< k only when fewer non-overlapping pairs exist), or -1
 * on allocation failure. */
int32_t orc_topk_exact(const double* x, int64_t n, int32_t D, int32_t w, int32_t d, int32_t k,
                       orc_motif* out)
{
    int64_t ns = n - w + 1;
    int64_t cap = 0;
    for (int64_t a = 0; a < ns; ++a) {
        int64_t first = a + w / 2 + 1;     /* smallest b with 2(b - a) > w */
        if (first < ns) cap += ns - first;
    }
    orc_motif* all = (orc_motif*)malloc(sizeof(orc_motif) * (size_t)(cap > 0 ? cap : 1));
    if (!all) return -1;
    int64_t cnt = 0;
    for (int64_t a = 0; a < ns; ++a)
        for (int64_t b = a + 1; b < ns; ++b) {
            if (trivial(a, b, w)) continue;
            orc_motif* m = &all[cnt++];
            m->a = a;
            m->b = b;
            orc_distd(x, n, D, w, a, b, d, &m->dist_d, &m->dist_max, m->dims, NULL);
        }
    qsort(all, (size_t)cnt, sizeof(orc_motif), motif_cmp);
    int32_t got = greedy(all, cnt, k, w, out);
    free(all);
    return got;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2 / 6.1: the hash family, tensoring and the index parameters.   */
/* ------------------------------------------------------------------------ */

static int64_t ceil_sqrt(int64_t v)
{
    int64_t m = (int64_t)sqrt((double)v);
    while (m * m < v) ++m;
    while (m > 1 && (m - 1) * (m - 1) >= v) --m;
    return m;
}

/* Tensoring (section 6.1): m = ceil(sqrt(L)) half-functions per side would
 * give m^2 >= L repetitions; repetition j (0-based) uses left function
 * j div m and right function j mod m, so only ceil(L/m) left and min(L, m)
 * right functions are ever used. */
void orc_tensor_shape(int32_t L, int32_t* m, int32_t* n_left, int32_t* n_right)
{
    int32_t mm = (int32_t)ceil_sqrt(L);
    *m = mm;
    *n_left = (L + mm - 1) / mm;
    *n_right = L < mm ? L : mm;
}

/* Bytes of the tensored index for L repetitions: every window of every
 * dimension stores one 4-byte word per left and per right half-function. */
static int64_t index_bytes(int64_t ns, int32_t D, int32_t L)
{
    int32_t m, nl, nr;
    orc_tensor_shape(L, &m, &nl, &nr);
    return 4 * ns * (int64_t)D * (int64_t)(nl + nr);
}

/* Memory cap (index size O(K L D n), Theorem "space"): the largest number of
 * repetitions L' <= L_max whose index, together with the series, the window
 * statistics and a fixed traversal reserve, fits in mem_limit bytes.
 * reserve = 32 bytes per window per dimension + 64 MiB. Returns 0 when not
 * even L' = 1 fits. */
int32_t orc_L_used(int64_t n, int32_t D, int32_t w, int32_t L_max, int32_t series_elem_bytes,
                   uint64_t mem_limit)
{
    int64_t ns = n - w + 1;
    int64_t fixed = n * (int64_t)D * series_elem_bytes + 16 * ns * (int64_t)D
                  + 32 * ns * (int64_t)D + ((int64_t)64 << 20);
    for (int32_t L = L_max; L >= 1; --L)
        if ((uint64_t)(fixed + index_bytes(ns, D, L)) <= mem_limit) return L;
    return 0;
}

/* Random projection vectors and offsets of Eq. drp for every dimension and
 * every column c = 4*function + position: R is [D][w][C], U is [D][C] with
 * b = r * U uniform in [0, r). */
void orc_draw_projections(uint64_t seed, int32_t D, int32_t w, int32_t C, double* R, double* U)
{
    for (int32_t f = 0; f < D; ++f) {
        for (int32_t t = 0; t < w; ++t)
            for (int32_t c = 0; c < C; ++c)
                R[((int64_t)f * w + t) * C + c] =
                    orc_gauss(seed, (uint32_t)t, (uint32_t)c, (uint32_t)f, STREAM_PROJ);
        for (int32_t c = 0; c < C; ++c)
            U[(int64_t)f * C + c] = orc_uniform(seed, (uint32_t)c, (uint32_t)f, 0u, STREAM_OFFSET);
    }
}

/* Section 6.1 "Setting the quantization width r": project a random sample of
 * z-normalised windows on a few random Gaussian vectors and split the range
 * of the projections into 256 equal buckets; r is the bucket width.
 * Reading: 8 vectors, min(n_s, 4096) windows per dimension drawn with
 * replacement, all dimensions pooled, offsets b not included. */
double orc_estimate_r(const double* x, int64_t n, int32_t D, int32_t w, uint64_t seed)
{
    const int32_t n_vec = 8;
    int64_t ns = n - w + 1;
    int64_t n_win = ns < 4096 ? ns : 4096;
    double* vec = (double*)malloc(sizeof(double) * (size_t)n_vec * (size_t)w);
    double* z = (double*)malloc(sizeof(double) * (size_t)w);
    for (int32_t s = 0; s < n_vec; ++s)
        for (int32_t t = 0; t < w; ++t)
            vec[(int64_t)s * w + t] = orc_gauss(seed, (uint32_t)t, (uint32_t)s, 0u, STREAM_RVEC);
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t f = 0; f < D; ++f)
        for (int64_t q = 0; q < n_win; ++q) {
            double u = orc_uniform(seed, (uint32_t)q, (uint32_t)f, 0u, STREAM_RWIN);
            int64_t a = (int64_t)floor(u * (double)ns);
            if (a > ns - 1) a = ns - 1;
            znorm(x + (int64_t)f * n + a, w, z);
            for (int32_t s = 0; s < n_vec; ++s) {
                double dot = 0.0;
                for (int32_t t = 0; t < w; ++t) dot = dot + vec[(int64_t)s * w + t] * z[t];
                if (dot < lo) lo = dot;
                if (dot > hi) hi = dot;
            }
        }
    free(vec);
    free(z);
    double r = (hi - lo) / 256.0;
    if (!(r > 0.0) || !isfinite(r)) r = 1.0;
    return r;
}

/* Eq. drp on one window and one column: h = floor((a.x + b) / r) with
 * b = r * U. The integer is stored as one byte, (h + 128) mod 256 (the paper
 * sizes r so that a hash value fits in a byte). Also returns the pre-floor
 * value and sum_t |a_t x_t| (used to bound rounding in other precisions). */
int32_t orc_hash_value(const double* z, int32_t w, const double* R_col, int64_t R_stride,
                       double U, double r, double* pre_floor, double* abs_sum)
{
    double dot = 0.0, sabs = 0.0;
    for (int32_t t = 0; t < w; ++t) {
        double term = R_col[(int64_t)t * R_stride] * z[t];
        dot = dot + term;
        sabs = sabs + fabs(term);
    }
    double b = r * U;
    double u = (dot + b) / r;
    double h = floor(u);
    int64_t hv = (int64_t)h;
    int64_t byte = ((hv + 128) % 256 + 256) % 256;
    if (pre_floor) *pre_floor = u;
    if (abs_sum) *abs_sum = sabs;
    return (int32_t)byte;
}

/* ------------------------------------------------------------------------ */
/* Low-precision forms of the projection (no counterpart in the paper: the  */
/* inputs of a . x are rounded to a narrow format, the sum is exact).       */
/* ------------------------------------------------------------------------ */

enum { ORC_FMT_BF16 = 2, ORC_FMT_E4M3 = 3 };

/* Round to nearest, ties to even, to bfloat16 (8 significant bits) or to the
 * OCP FP8 E4M3 format (4 significant bits, exponent bias 7, subnormal quantum
 * 2^-9, largest finite value 448, saturating). */
double orc_round_fmt(double v, int32_t fmt)
{
    if (v == 0.0) return v;
    double a = fabs(v);
    int ex;
    frexp(a, &ex);                  /* a in [2^(ex-1), 2^ex) */
    int lead = ex - 1;
    int bits = fmt == ORC_FMT_BF16 ? 8 : 4;
    if (fmt == ORC_FMT_E4M3 && lead < -6) lead = -6;
    double q = ldexp(1.0, lead - (bits - 1));
    double r = nearbyint(a / q) * q;
    if (fmt == ORC_FMT_E4M3 && r > 448.0) r = 448.0;
    return v < 0 ? -r : r;
}

/* orc_round_fmt over an array (the form the tests call on many values). */
void orc_round_fmt_array(const double* v, int64_t count, int32_t fmt, double* out)
{
    for (int64_t q = 0; q < count; ++q) out[q] = orc_round_fmt(v[q], fmt);
}

/* Spacing of the format's values around v. */
static double fmt_gap(double v, int32_t fmt)
{
    double a = fabs(v);
    int ex;
    if (a == 0.0) return fmt == ORC_FMT_BF16 ? ldexp(1.0, -133) : ldexp(1.0, -9);
    frexp(a, &ex);
    int lead = ex - 1;
    int bits = fmt == ORC_FMT_BF16 ? 8 : 4;
    if (fmt == ORC_FMT_E4M3 && lead < -6) lead = -6;
    return ldexp(1.0, lead - (bits - 1));
}

/* Eq. drp with both a and the normal form rounded to the format (the normal
 * form first to float32): h = floor((Q(a) . Q(x) + b) / r). Subnormal values
 * of the format are kept (rounded on the format's smallest quantum), never
 * flushed. abs_sum gets sum |Q(a_t) Q(x_t)|; amb bounds the change from
 * inputs that another valid evaluation may round differently: sum
 * |Q(a_t)| * gap over samples whose float32 value lies within
 * 1e-5 (1 + |x_t|) of a rounding midpoint (a normal form evaluated in float32
 * may land on either side of it). */
int32_t orc_hash_value_lowp(const double* z, int32_t w, const double* R_col, int64_t R_stride,
                            double U, double r, int32_t fmt, double* pre_floor, double* abs_sum,
                            double* amb)
{
    double dot = 0.0, sabs = 0.0, ambs = 0.0;
    for (int32_t t = 0; t < w; ++t) {
        double rq = orc_round_fmt(R_col[(int64_t)t * R_stride], fmt);
        double zf = (double)(float)z[t];
        double zq = orc_round_fmt(zf, fmt);
        double term = rq * zq;
        dot = dot + term;
        sabs = sabs + fabs(term);
        double g = fmt_gap(zf, fmt);
        double to_mid = fabs(g / 2.0 - fabs(zf - zq));
        if (to_mid <= 1e-5 * (1.0 + fabs(zf))) ambs = ambs + fabs(rq) * g;
    }
    double b = r * U;
    double u = (dot + b) / r;
    int64_t hv = (int64_t)floor(u);
    if (pre_floor) *pre_floor = u;
    if (abs_sum) *abs_sum = sabs;
    if (amb) *amb = ambs;
    return (int32_t)(((hv + 128) % 256 + 256) % 256);
}

void orc_hash_dim_lowp(const double* xf, int64_t n, int32_t w, const double* Rf, const double* Uf,
                       int32_t C, double r, int32_t fmt, uint8_t* bytes, double* pre, double* sabs,
                       double* amb)
{
    int64_t ns = n - w + 1;
    double* z = (double*)malloc(sizeof(double) * (size_t)w);
    for (int64_t a = 0; a < ns; ++a) {
        znorm(xf + a, w, z);
        for (int32_t c = 0; c < C; ++c)
            bytes[a * C + c] = (uint8_t)orc_hash_value_lowp(z, w, Rf + c, C, Uf[c], r, fmt,
                                                            &pre[a * C + c], &sabs[a * C + c],
                                                            &amb[a * C + c]);
    }
    free(z);
}

/* Hash every window of one dimension f at the given columns. Outputs are
 * [n_s][C] (bytes, and optionally the pre-floor values and |.| sums). */
void orc_hash_dim(const double* xf, int64_t n, int32_t w, const double* Rf /* [w][C] */,
                  const double* Uf /* [C] */, int32_t C, double r,
                  uint8_t* bytes, double* pre, double* sabs)
{
    int64_t ns = n - w + 1;
    double* z = (double*)malloc(sizeof(double) * (size_t)w);
    for (int64_t a = 0; a < ns; ++a) {
        znorm(xf + a, w, z);
        for (int32_t c = 0; c < C; ++c) {
            double pv, sv;
            int32_t byte = orc_hash_value(z, w, Rf + c, C, Uf[c], r, &pv, &sv);
            bytes[a * C + c] = (uint8_t)byte;
            if (pre) pre[a * C + c] = pv;
            if (sabs) sabs[a * C + c] = sv;
        }
    }
    free(z);
}

/* Hash every window of every dimension: bytes [D][n_s][C], x [D][n],
 * R [D][w][C], U [D][C]. */
void orc_hash_all(const double* x, int64_t n, int32_t D, int32_t w, const double* R, const double* U,
                  int32_t C, double r, uint8_t* bytes)
{
    int64_t ns = n - w + 1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int32_t f = 0; f < D; ++f)
        orc_hash_dim(x + (int64_t)f * n, n, w, R + (int64_t)f * w * C, U + (int64_t)f * C, C, r,
                     bytes + (int64_t)f * ns * C, NULL, NULL);
}

/* Hash one window (f, a) at every column: the "one by one" form used to
 * check samples of large inputs. */
void orc_hash_one(const double* xf, int32_t w, int64_t a, const double* Rf, const double* Uf,
                  int32_t C, double r, uint8_t* bytes, double* pre, double* sabs)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)w);
    znorm(xf + a, w, z);
    for (int32_t c = 0; c < C; ++c)
        bytes[c] = (uint8_t)orc_hash_value(z, w, Rf + c, C, Uf[c], r, pre ? &pre[c] : NULL,
                                           sabs ? &sabs[c] : NULL);
    free(z);
}

/* Pack the K/2 bytes of each half-function into a 32-bit word, position 0
 * in the most significant byte: words[f][F][a]. bytes is [D][n_s][C],
 * column c = 4 F + p. */
void orc_pack(const uint8_t* bytes, int64_t ns, int32_t D, int32_t NF, int32_t K, uint32_t* words)
{
    int32_t C = 4 * NF;
    for (int32_t f = 0; f < D; ++f)
        for (int32_t F = 0; F < NF; ++F)
            for (int64_t a = 0; a < ns; ++a) {
                uint32_t v = 0;
                for (int32_t p = 0; p < K / 2; ++p)
                    v |= (uint32_t)bytes[((int64_t)f * ns + a) * C + 4 * F + p] << (24 - 8 * p);
                words[((int64_t)f * NF + F) * ns + a] = v;
            }
}

/* The composite hash of repetition j (section 6.1): the left half-function
 * j div m and the right half-function j mod m, their values interleaved
 * (l0 r0 l1 r1 ...). Returns the first i symbols as an integer, first
 * symbol most significant. */
uint64_t orc_prefix(const uint32_t* words, int64_t ns, int32_t NF, int32_t n_left, int32_t m,
                    int32_t f, int32_t j, int64_t a, int32_t i)
{
    int32_t l = j / m, rr = j % m;
    uint32_t left = words[((int64_t)f * NF + l) * ns + a];
    uint32_t right = words[((int64_t)f * NF + n_left + rr) * ns + a];
    uint64_t v = 0;
    for (int32_t q = 0; q < i; ++q) {
        uint32_t src = (q % 2 == 0) ? left : right;
        uint32_t sym = (src >> (24 - 8 * (q / 2))) & 255u;
        v = (v << 8) | sym;
    }
    return v;
}

/* ------------------------------------------------------------------------ */
/* Eq. eucl-collision-probability and the stopping rule.                     */
/* ------------------------------------------------------------------------ */

/* Probability that one hash of Eq. drp (width r) collides on two vectors at
 * distance R: 1 - 2 Phi(-r/R) - 2/(sqrt(2 pi) r/R) (1 - exp(-(r/R)^2 / 2)). */
double orc_collision_prob(double R, double r)
{
    if (R <= 0.0) return 1.0;
    double t = r / R;
    double Phi = 0.5 * erfc(t / sqrt(2.0));    /* Phi(-t) */
    return 1.0 - 2.0 * Phi - 2.0 / (sqrt(2.0 * M_PI) * t) * (1.0 - exp(-(t * t) / 2.0));
}

enum { ORC_STOP_TENSOR = 0, ORC_STOP_LEMMA52 = 1, ORC_STOP_TENSOR_LITERAL = 2, ORC_STOP_RIGOROUS = 3 };



/* Failure bound after J repetitions of round i.
 * rule TENSOR: Lemma 6.1 with P_t(i', J') = (1 - p^ceil(i'))^(J' div m) *
 *              (1 - p^floor(i'))^(J' mod m), m = ceil(sqrt(L)), where a half
 *              that contributes no symbol to the prefix (floor(i') = 0, i.e.
 *              round 1) gives the factor 1: it offers no collision chance of
 *              its own. Printed literally that factor is (1 - p^0)^x = 0,
 *              which would stop round 1 unconditionally (rule TENSOR_LITERAL).
 * rule LEMMA52: Eq. probnotcolliding, (1 - p^i)^J [ * (1 - p^(i+1))^(L - J) ].
 * x^0 is 1 (including 0^0). */
static double powi_(double base, int64_t e)
{
    return e == 0 ? 1.0 : pow(base, (double)e);
}

/* (1 - p^c)^e, one factor of P_t; c = 0 is the empty half (see above). */
static double tfactor(double p, int32_t c, int64_t e, int32_t rule)
{
    if (c == 0 && rule == ORC_STOP_TENSOR) return 1.0;
    return powi_(1.0 - powi_(p, c), e);
}

/* A bound on the failure probability under tensoring that follows from the
 * index's structure itself (rule RIGOROUS; the printed Lemma 6.1 multiplies
 * over repetitions that share half-functions, which are not independent).
 * Repetition j uses left function l = j div m and right function r = j mod m;
 * at prefix length i it collides on the pair (in the d dimensions of its
 * dist_max) when the left function's first ceil(i/2) symbols and the right
 * function's first floor(i/2) symbols all collide. Each symbol collides with
 * probability >= p = P(dist_max)^d, independently of every other symbol, so
 * the collision depth of each half-function is at least a geometric depth G
 * with P(G >= s) = p^s; failure only becomes likelier when depths shrink, so
 * the probability of failure with exactly these depths bounds it. Failure
 * after J repetitions of round i (below round K, after every repetition of
 * round i+1 too): no repetition j < J collides at prefix i and no repetition
 * j >= J at prefix i+1 (a collision at i+1 is one at i). Conditioned on
 * which right functions reach the two depths, the left functions are
 * independent, which gives the sum below over the states of a few column
 * ranges. */
static double seg_state_prob(int st, int64_t len, double qx, double qy)
{
    /* st 0: no right function of the range reaches depth b (prob of each: qx);
     * 1: some reach b, none b' (qy); 2: some reach b' (b' >= b) */
    double none_x = powi_(1.0 - qx, len), none_y = powi_(1.0 - qy, len);
    if (st == 0) return none_x;
    if (st == 1) return none_y - none_x;
    return 1.0 - none_y;
}

static double rigorous_bound(double p, int32_t i, int32_t J, int32_t K, int32_t L)
{
    int32_t m = (int32_t)ceil_sqrt(L);
    int32_t nl = (L + m - 1) / m;
    int32_t a = (i + 1) / 2, b = i / 2;            /* left / right symbols at prefix i */
    int32_t a2 = (i + 2) / 2, b2 = (i + 1) / 2;    /* at prefix i + 1 */
    int deeper = i < K;
    double qx = powi_(p, b), qy = deeper ? powi_(p, b2) : 0.0;
    double keep_a = 1.0 - powi_(p, a), keep_a2 = 1.0 - powi_(p, a2);
    /* column ranges cut at c = J mod m and at the lengths of the rows */
    int32_t lstar = J / m, c = J % m;
    int32_t len_last = L - (nl - 1) * m;
    int32_t cuts[6] = {0, c, m, len_last, 0, 0};
    int32_t ncut = 4;
    /* the partial row's length */
    int32_t len_star = lstar < nl ? (lstar == nl - 1 ? len_last : m) : 0;
    cuts[ncut++] = len_star;
    /* sort and dedupe */
    for (int32_t u = 1; u < ncut; ++u)
        for (int32_t v = u; v > 0 && cuts[v - 1] > cuts[v]; --v) {
            int32_t t = cuts[v]; cuts[v] = cuts[v - 1]; cuts[v - 1] = t;
        }
    int32_t seg_lo[5], seg_hi[5], nseg = 0;
    for (int32_t u = 0; u + 1 < ncut; ++u)
        if (cuts[u + 1] > cuts[u]) {
            seg_lo[nseg] = cuts[u];
            seg_hi[nseg] = cuts[u + 1];
            ++nseg;
        }
    int64_t nstates = 1;
    for (int32_t u = 0; u < nseg; ++u) nstates *= 3;
    double total = 0.0;
    for (int64_t code = 0; code < nstates; ++code) {
        int32_t st[5];
        int64_t cc = code;
        double pr = 1.0;
        for (int32_t u = 0; u < nseg; ++u) {
            st[u] = (int32_t)(cc % 3);
            cc /= 3;
            pr *= seg_state_prob(st[u], seg_hi[u] - seg_lo[u], qx, qy);
        }
        if (pr == 0.0) continue;
        /* for every row: does some right function of its prefix-i columns reach
         * depth b (fx), of its prefix-(i+1) columns depth b' (fy)? */
        double rows = 1.0;
        for (int32_t l = 0; l < nl; ++l) {
            int32_t len = l == nl - 1 ? len_last : m;
            int32_t xi_hi = l < lstar ? len : (l == lstar ? c : 0);   /* columns [0, xi_hi) at prefix i */
            int32_t yi_lo = xi_hi, yi_hi = deeper ? len : xi_hi;       /* columns [yi_lo, yi_hi) at i + 1 */
            int fx = 0, fy = 0;
            for (int32_t u = 0; u < nseg; ++u) {
                if (seg_lo[u] < xi_hi && st[u] >= 1) fx = 1;            /* ranges never straddle a cut */
                if (seg_lo[u] >= yi_lo && seg_lo[u] < yi_hi && st[u] == 2) fy = 1;
            }
            double ok = 1.0;
            if (fx) ok = keep_a;                 /* the left function must stay below depth a */
            else if (fy) ok = keep_a2;           /* ... below depth a' only */
            rows *= ok;
        }
        total += pr * rows;
    }
    return total;
}

double orc_fail_bound(double p, int32_t i, int32_t J, int32_t K, int32_t L, int32_t rule)
{
    if (rule == ORC_STOP_RIGOROUS) return rigorous_bound(p, i, J, K, L);
    if (rule == ORC_STOP_LEMMA52) {
        double v = powi_(1.0 - powi_(p, i), J);
        if (i < K) v = v * powi_(1.0 - powi_(p, i + 1), L - J);
        return v;
    }
    int32_t m = (int32_t)ceil_sqrt(L);
    /* P_t(i/2, J): ceil(i/2) = (i+1)/2, floor(i/2) = i/2 */
    double v = tfactor(p, (i + 1) / 2, J / m, rule) * tfactor(p, i / 2, J % m, rule);
    if (i < K) {
        /* P_t((i+1)/2, L-J): ceil((i+1)/2) = (i+2)/2, floor((i+1)/2) = (i+1)/2 */
        int32_t J2 = L - J;
        v = v * tfactor(p, (i + 2) / 2, J2 / m, rule) * tfactor(p, (i + 1) / 2, J2 % m, rule);
    }
    return v;
}

/* Algorithm 2: p = P(dist_max of the k-th motif)^d; stop when the bound on
 * having missed a better pair is at most delta. */
int32_t orc_stop(double dist_max, double r, int32_t d, int32_t i, int32_t J, int32_t K, int32_t L,
                 int32_t rule, double delta)
{
    double p = pow(orc_collision_prob(dist_max, r), (double)d);
    return orc_fail_bound(p, i, J, K, L, rule) <= delta;
}

/* ------------------------------------------------------------------------ */
/* O2: Algorithm 1 (with comparisons of section 6.2), sequential.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t a, b;
} pair_t;

static int pair_cmp(const void* p, const void* q)
{
    const pair_t* x = (const pair_t*)p;
    const pair_t* y = (const pair_t*)q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

/* growable list of the pairs one dimension contributes to a step */
typedef struct {
    pair_t* p;
    int64_t cnt, cap;
} pair_list;

static void free_dim_pairs(pair_list* pl, int32_t D)
{
    for (int32_t f = 0; f < D; ++f) free(pl[f].p);
    free(pl);
}

typedef struct {
    uint64_t key;
    int64_t a;
} keyed_t;

static int keyed_cmp(const void* p, const void* q)
{
    const keyed_t* x = (const keyed_t*)p;
    const keyed_t* y = (const keyed_t*)q;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    return 0;
}

/* open-addressing set of pairs (the set of distinct verified pairs) */
typedef struct {
    uint64_t* slot;   /* 0 = empty, else (a * ns + b) + 1 */
    int64_t cap;
    int64_t used;
} pairset;

static uint64_t mix64(uint64_t v)
{
    v ^= v >> 33;
    v *= 0xff51afd7ed558ccdULL;
    v ^= v >> 33;
    v *= 0xc4ceb9fe1a85ec53ULL;
    v ^= v >> 33;
    return v;
}

static int pairset_insert(pairset* s, uint64_t code)   /* returns 1 when newly inserted */
{
    if (2 * (s->used + 1) > s->cap) {
        int64_t ncap = s->cap ? 2 * s->cap : 1024;
        uint64_t* ns_ = (uint64_t*)calloc((size_t)ncap, sizeof(uint64_t));
        for (int64_t e = 0; e < s->cap; ++e)
            if (s->slot[e]) {
                int64_t h = (int64_t)(mix64(s->slot[e]) & (uint64_t)(ncap - 1));
                while (ns_[h]) h = (h + 1) & (ncap - 1);
                ns_[h] = s->slot[e];
            }
        free(s->slot);
        s->slot = ns_;
        s->cap = ncap;
    }
    uint64_t v = code + 1;
    int64_t h = (int64_t)(mix64(v) & (uint64_t)(s->cap - 1));
    while (s->slot[h]) {
        if (s->slot[h] == v) return 0;
        h = (h + 1) & (s->cap - 1);
    }
    s->slot[h] = v;
    s->used++;
    return 1;
}

typedef struct {
    /* inputs */
    int32_t K, L, rule;
    int32_t no_fallback;     /* 1: when no step stops, return 0 motifs instead of the exact answer */
    double r;
    /* optional trace of every step (step s = (K - i) * L + (J - 1)) */
    int64_t* cand;           /* triples (s, a, b): the pairs with W >= d at step s */
    int64_t cand_cap;
    int64_t cand_count;      /* may exceed cand_cap (then the trace is truncated) */
    int32_t* top_size;       /* [K*L]: |TOP| after step s, -1 if not reached */
    int64_t* top_pairs;      /* [K*L][k][2] */
    double* top_distmax;     /* [K*L]: dist_max of TOP[k-1] (or NaN) */
    /* outputs */
    int32_t i_stop, J_stop;  /* 0 when the exact fallback answered */
    int64_t n_verified;      /* distinct verified pairs */
    int64_t n_collisions;    /* one-dimensional non-trivial collisions seen */
} orc_lsh_ctl;

/* Algorithm 1, rounds i = K..1 and repetitions J = 1..L. For each step every
 * dimension contributes its non-trivial colliding pairs (equal prefixes of
 * length i, found through a sort of the prefixes as in the index of
 * section 4); W(a, b) counts the dimensions in which a pair collides; pairs
 * with W >= d join the set of verified pairs with their exact dist_d; TOP is
 * the greedy top-k of that set; the stopping rule is checked when |TOP| = k.
 * words is the packed index [D][NF][n_s] (orc_pack). Returns the number of
 * motifs written to out (the exact top-k when no step stops). */
int32_t orc_lsh_search(const double* x, int64_t n, int32_t D, int32_t w, int32_t d, int32_t k,
                       double delta, const uint32_t* words, orc_lsh_ctl* ctl, orc_motif* out)
{
    int64_t ns = n - w + 1;
    int32_t K = ctl->K, L = ctl->L;
    int32_t m, n_left, n_right;
    orc_tensor_shape(L, &m, &n_left, &n_right);
    int32_t NF = n_left + n_right;

    keyed_t* keyed = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)ns * (size_t)D);
    pair_list* dim_pairs = (pair_list*)calloc((size_t)D, sizeof(pair_list));
    int64_t pcap = 1 << 16, pcnt = 0;
    pair_t* pairs = (pair_t*)malloc(sizeof(pair_t) * (size_t)pcap);
    int64_t vcap = 1024, vcnt = 0;
    orc_motif* ver = (orc_motif*)malloc(sizeof(orc_motif) * (size_t)vcap);
    orc_motif* sorted = NULL;
    int64_t sorted_cap = 0;
    orc_motif* top = (orc_motif*)malloc(sizeof(orc_motif) * (size_t)(k > 0 ? k : 1));
    pairset seen = {0, 0, 0};
    int32_t got = 0;
    ctl->cand_count = 0;
    ctl->n_verified = 0;
    ctl->n_collisions = 0;
    ctl->i_stop = 0;
    ctl->J_stop = 0;
    if (ctl->top_size)
        for (int64_t s = 0; s < (int64_t)K * L; ++s) ctl->top_size[s] = -1;

    for (int32_t i = K; i >= 1; --i) {
        for (int32_t J = 1; J <= L; ++J) {
            int32_t j = J - 1;
            int64_t step = (int64_t)(K - i) * L + j;
            /* step 1: one-dimensional collisions of every dimension */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
            for (int32_t f = 0; f < D; ++f) {
                keyed_t* kf = keyed + (int64_t)f * ns;
                pair_list* pl = &dim_pairs[f];
                pl->cnt = 0;
                for (int64_t a = 0; a < ns; ++a) {
                    kf[a].key = orc_prefix(words, ns, NF, n_left, m, f, j, a, i);
                    kf[a].a = a;
                }
                qsort(kf, (size_t)ns, sizeof(keyed_t), keyed_cmp);
                int64_t s0 = 0;
                while (s0 < ns) {
                    int64_t e = s0 + 1;
                    while (e < ns && kf[e].key == kf[s0].key) ++e;
                    for (int64_t p = s0; p < e; ++p)
                        for (int64_t q = p + 1; q < e; ++q) {
                            int64_t a = kf[p].a, b = kf[q].a;   /* a < b (sorted by a within a run) */
                            if (trivial(a, b, w)) continue;
                            if (pl->cnt == pl->cap) {
                                pl->cap = pl->cap ? 2 * pl->cap : 1024;
                                pl->p = (pair_t*)realloc(pl->p, sizeof(pair_t) * (size_t)pl->cap);
                            }
                            pl->p[pl->cnt].a = a;
                            pl->p[pl->cnt].b = b;
                            ++pl->cnt;
                        }
                    s0 = e;
                }
            }
            pcnt = 0;
            for (int32_t f = 0; f < D; ++f) pcnt += dim_pairs[f].cnt;
            if (pcnt > pcap) {
                pcap = pcnt;
                pairs = (pair_t*)realloc(pairs, sizeof(pair_t) * (size_t)pcap);
            }
            pcnt = 0;
            for (int32_t f = 0; f < D; ++f) {
                if (dim_pairs[f].cnt == 0) continue;   /* no list yet (p may be NULL) */
                memcpy(pairs + pcnt, dim_pairs[f].p, sizeof(pair_t) * (size_t)dim_pairs[f].cnt);
                pcnt += dim_pairs[f].cnt;
            }
            ctl->n_collisions += pcnt;
            /* W(a, b): multiplicity of each pair over the dimensions */
            qsort(pairs, (size_t)pcnt, sizeof(pair_t), pair_cmp);
            int added = 0;
            const int64_t v_before = vcnt;
            int64_t s0 = 0;
            while (s0 < pcnt) {
                int64_t e = s0 + 1;
                while (e < pcnt && pairs[e].a == pairs[s0].a && pairs[e].b == pairs[s0].b) ++e;
                int64_t W = e - s0;
                if (W >= d) {
                    int64_t a = pairs[s0].a, b = pairs[s0].b;
                    if (ctl->cand) {
                        if (ctl->cand_count < ctl->cand_cap) {
                            ctl->cand[3 * ctl->cand_count + 0] = step;
                            ctl->cand[3 * ctl->cand_count + 1] = a;
                            ctl->cand[3 * ctl->cand_count + 2] = b;
                        }
                    }
                    ctl->cand_count++;
                    /* step 2: each new pair joins the verified set */
                    if (pairset_insert(&seen, (uint64_t)a * (uint64_t)ns + (uint64_t)b)) {
                        if (vcnt == vcap) {
                            vcap *= 2;
                            ver = (orc_motif*)realloc(ver, sizeof(orc_motif) * (size_t)vcap);
                        }
                        orc_motif* v = &ver[vcnt++];
                        v->a = a;
                        v->b = b;
                        added = 1;
                    }
                }
                s0 = e;
            }
            /* ... with its distance (definition "d-dimensional distance") */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
            for (int64_t q = v_before; q < vcnt; ++q)
                orc_distd(x, n, D, w, ver[q].a, ver[q].b, d, &ver[q].dist_d, &ver[q].dist_max, ver[q].dims, NULL);
            ctl->n_verified = vcnt;
            if (added) {
                if (sorted_cap < vcnt) {
                    sorted_cap = vcap;
                    sorted = (orc_motif*)realloc(sorted, sizeof(orc_motif) * (size_t)sorted_cap);
                }
                memcpy(sorted, ver, sizeof(orc_motif) * (size_t)vcnt);
                qsort(sorted, (size_t)vcnt, sizeof(orc_motif), motif_cmp);
                got = greedy(sorted, vcnt, k, w, top);
            }
            if (ctl->top_size) {
                ctl->top_size[step] = got;
                for (int32_t s = 0; s < got; ++s) {
                    ctl->top_pairs[(step * k + s) * 2 + 0] = top[s].a;
                    ctl->top_pairs[(step * k + s) * 2 + 1] = top[s].b;
                }
                ctl->top_distmax[step] = got == k ? top[k - 1].dist_max : NAN;
            }
            /* step 3: the stopping condition on the k-th motif */
            if (got == k && orc_stop(top[k - 1].dist_max, ctl->r, d, i, J, K, L, ctl->rule, delta)) {
                ctl->i_stop = i;
                ctl->J_stop = J;
                memcpy(out, top, sizeof(orc_motif) * (size_t)k);
                free(keyed); free(pairs); free(ver); free(sorted); free(top); free(seen.slot);
                free_dim_pairs(dim_pairs, D);
                return k;
            }
        }
    }
    free(keyed); free(pairs); free(ver); free(sorted); free(top); free(seen.slot);
    free_dim_pairs(dim_pairs, D);
    /* no step stopped: the exact answer over all pairs */
    if (ctl->no_fallback) return 0;
    return orc_topk_exact(x, n, D, w, d, k, out);
}

/* Size of the motif record, so that callers can check their layout. */
int32_t orc_motif_size(void) { return (int32_t)sizeof(orc_motif); }
int32_t orc_ctl_size(void) { return (int32_t)sizeof(orc_lsh_ctl); }
