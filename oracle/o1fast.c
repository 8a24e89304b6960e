/*
 * O1-fast: the exact top-k motifs of section 3.1 (the same answer as
 * orc_topk_exact) for inputs too long for the all-pairs brute force.
 *
 * TEST INFRASTRUCTURE ONLY (see momenti_oracle.c): it writes golden files and
 * checks large answers; it shares nothing with the GPU library.
 *
 * The definitions are not changed, only the order in which pairs are looked
 * at. Pairs (a, a + s) are visited diagonal by diagonal (s > w/2, so no
 * trivial match is ever formed). Along a diagonal the centred cross product
 *   C_f(a, b) = sum_t (x_f[a+t] - mu_f(a)) (x_f[b+t] - mu_f(b))
 * follows the recurrence
 *   C(a+1, b+1) = C(a, b) + df(a) dg(b) + df(b) dg(a),
 *   df(i) = (x[i+w] - x[i]) / 2,  dg(i) = (x[i+w] - mu(i+1)) + (x[i] - mu(i)),
 * which is exact algebra (expand mu(i+1) = mu(i) + (x[i+w] - x[i]) / w), and
 * is re-seeded by the direct sum every kReseed steps. With the population
 * standard deviation of every window, sum_t z_a[t]^2 = w for a window that is
 * not flat, so the squared z-normalised distance (Eq. zned) is
 *   dist_f^2 = w (s_a + s_b) - 2 C_f / (sigma_a sigma_b),
 * s = 1 for a window that is not flat and 0 for a flat one (whose normal form
 * is all zeros). That value is used only as a FILTER: the best `pool` pairs
 * by the approximate dist_d are kept, every one of them is recomputed with
 * orc_distd (the O1 definition, bit for bit), and the greedy non-overlapping
 * selection of O1 runs on them.
 *
 * Exactness: every pair left out has an approximate dist_d >= theta (the
 * pool's cut), so an exact dist_d >= theta - eps, eps bounding the filter's
 * error. The greedy choice over all pairs takes its first k picks in
 * increasing (dist_d, a, b) order and each decision depends only on earlier
 * pairs; if the k-th pick over the pool is below theta - eps, no pair left
 * out comes before it and the two greedy runs agree (the same argument as
 * for the bounded pool of verified pairs). Otherwise the sweep is repeated
 * with a pool four times larger.
 *
 * Threads (OpenMP, when the library is built with it) take groups of
 * diagonals; each keeps its own pool, and the pools are merged at the end.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t a, b;
    double dist_d, dist_max;
    uint64_t dims[2];
} orc_motif;

/* from momenti_oracle.c */
void orc_window_stats(const double* x, int32_t w, double* mu_out, double* sigma_out, int32_t* flat_out);
void orc_distd(const double* x, int64_t n, int32_t D, int32_t w, int64_t a, int64_t b, int32_t d,
               double* dist_d, double* dist_max, uint64_t dims_mask[2], double* per_dim);

enum { kDiag = 8, kReseed = 1024, kBlock = 256 };

typedef struct {
    double v;       /* approximate dist_d */
    int64_t a, b;
} approx_pair;

/* max-heap of approx_pair by v */
typedef struct {
    approx_pair* e;
    int64_t n, cap;
} heap_t;

static void heap_push(heap_t* h, approx_pair p)
{
    int64_t i = h->n++;
    h->e[i] = p;
    while (i > 0) {
        int64_t up = (i - 1) / 2;
        if (h->e[up].v >= h->e[i].v) break;
        approx_pair t = h->e[up]; h->e[up] = h->e[i]; h->e[i] = t;
        i = up;
    }
}

static void heap_replace_top(heap_t* h, approx_pair p)
{
    int64_t i = 0;
    h->e[0] = p;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && h->e[l].v > h->e[m].v) m = l;
        if (r < h->n && h->e[r].v > h->e[m].v) m = r;
        if (m == i) break;
        approx_pair t = h->e[m]; h->e[m] = h->e[i]; h->e[i] = t;
        i = m;
    }
}

static double heap_cut(const heap_t* h)   /* pairs at or above it are not kept */
{
    return h->n < h->cap ? INFINITY : h->e[0].v;
}

static int approx_cmp(const void* p, const void* q)
{
    const approx_pair* x = (const approx_pair*)p;
    const approx_pair* y = (const approx_pair*)q;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

static int motif_cmp2(const void* p, const void* q)
{
    const orc_motif* x = (const orc_motif*)p;
    const orc_motif* y = (const orc_motif*)q;
    if (x->dist_d < y->dist_d) return -1;
    if (x->dist_d > y->dist_d) return 1;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

static int overlaps(int64_t u, int64_t v, int32_t w)
{
    int64_t g = u > v ? u - v : v - u;
    return 2 * g <= (int64_t)w;
}

/* Sum of the d smallest square roots of d2[0..D-1] (d2 clamped at 0). */
static double smallest_sum(const double* d2, int32_t D, int32_t d)
{
    double best[128];
    int32_t nb = 0;
    for (int32_t f = 0; f < D; ++f) {
        double v = d2[f] > 0.0 ? d2[f] : 0.0;
        if (nb < d) {
            int32_t q = nb++;
            while (q > 0 && best[q - 1] > v) { best[q] = best[q - 1]; --q; }
            best[q] = v;
        } else if (v < best[d - 1]) {
            int32_t q = d - 1;
            while (q > 0 && best[q - 1] > v) { best[q] = best[q - 1]; --q; }
            best[q] = v;
        }
    }
    double s = 0.0;
    for (int32_t q = 0; q < d; ++q) s += sqrt(best[q]);
    return s;
}

typedef struct {
    int64_t n, ns;
    int32_t D, w, d;
    const double* x;
    double* mu;      /* [D][ns] */
    double* inv;     /* [D][ns]: 1 / sigma, 0 when flat */
    double* sflag;   /* [D][ns]: 1 when not flat, 0 when flat */
    double* df;      /* [D][ns] */
    double* dg;      /* [D][ns] */
} sweep_ctx;

static double direct_C(const sweep_ctx* c, int32_t f, int64_t a, int64_t b)
{
    const double* xf = c->x + (int64_t)f * c->n;
    const double ma = c->mu[(int64_t)f * c->ns + a], mb = c->mu[(int64_t)f * c->ns + b];
    double s = 0.0;
    for (int32_t t = 0; t < c->w; ++t) s += (xf[a + t] - ma) * (xf[b + t] - mb);
    return s;
}

/* One pass over every diagonal with per-thread pools of `pool` pairs.
 * Returns the merged candidates (sorted by approximate value, at most pool)
 * and the cut theta (+inf when nothing was left out). */
static approx_pair* sweep(const sweep_ctx* c, int64_t pool, int64_t* count, double* theta)
{
    const int64_t ns = c->ns, h = c->w / 2;
    const int32_t D = c->D, d = c->d;
    const double w = (double)c->w;
    const int64_t first = h + 1;                 /* smallest non-trivial offset */
    const int64_t ngroups = first < ns ? (ns - first + kDiag - 1) / kDiag : 0;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    heap_t* heaps = (heap_t*)calloc((size_t)nthreads, sizeof(heap_t));
    for (int t = 0; t < nthreads; ++t) {
        heaps[t].cap = pool;
        heaps[t].e = (approx_pair*)malloc(sizeof(approx_pair) * (size_t)pool);
    }
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        heap_t* hp = &heaps[tid];
        double* C = (double*)malloc(sizeof(double) * (size_t)D * kDiag);
        /* squared distances of a block of steps: [step][dimension][diagonal] */
        double* d2 = (double*)malloc(sizeof(double) * (size_t)kBlock * D * kDiag);
        double one[128];
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t gq = 0; gq < ngroups; ++gq) {
            const int64_t s0 = first + gq * kDiag;
            const int nd = (int)(ns - s0 < kDiag ? ns - s0 : kDiag);
            const int64_t len0 = ns - s0;        /* pairs on the longest diagonal */
            for (int64_t a0 = 0; a0 < len0; a0 += kBlock) {
                const int64_t a1 = a0 + kBlock < len0 ? a0 + kBlock : len0;
                /* one dimension at a time over the block (few memory streams);
                 * all kDiag lanes are computed (the arrays are padded past the
                 * last window), lanes past the end of a diagonal are ignored */
                for (int32_t f = 0; f < D; ++f) {
                    const int64_t o = (int64_t)f * ns;
                    double* Cf = C + f * kDiag;
                    for (int64_t a = a0; a < a1; ++a) {
                        if (a % kReseed == 0) {
                            for (int q = 0; q < kDiag; ++q)
                                Cf[q] = a + s0 + q < ns ? direct_C(c, f, a, a + s0 + q) : 0.0;
                        } else {
                            const double* dff = c->df + o + (a - 1 + s0);
                            const double* dgf = c->dg + o + (a - 1 + s0);
                            const double dfa = c->df[o + a - 1], dga = c->dg[o + a - 1];
                            for (int q = 0; q < kDiag; ++q) Cf[q] += dfa * dgf[q] + dff[q] * dga;
                        }
                        const double ia = c->inv[o + a], sa = c->sflag[o + a];
                        const double* ib = c->inv + o + a + s0;
                        const double* sb = c->sflag + o + a + s0;
                        double* out = d2 + ((a - a0) * D + f) * kDiag;
                        for (int q = 0; q < kDiag; ++q) out[q] = w * (sa + sb[q]) - 2.0 * Cf[q] * ia * ib[q];
                    }
                }
                for (int64_t a = a0; a < a1; ++a) {
                    int nq = nd;
                    while (nq > 0 && a + s0 + nq - 1 >= ns) --nq;
                    /* a sum of d distances below the cut needs all d of them
                     * below the cut and the smallest below cut / d */
                    const double cut = heap_cut(hp);
                    const double cut2 = cut * cut, low2 = (cut / d) * (cut / d);
                    int cnt[kDiag], low[kDiag];
                    for (int q = 0; q < kDiag; ++q) cnt[q] = low[q] = 0;
                    const double* blk = d2 + (a - a0) * D * kDiag;
                    for (int32_t f = 0; f < D; ++f)
                        for (int q = 0; q < kDiag; ++q) {
                            cnt[q] += blk[f * kDiag + q] < cut2;
                            low[q] += blk[f * kDiag + q] < low2;
                        }
                    for (int q = 0; q < nq; ++q) {
                        if (cnt[q] < d || low[q] < 1) continue;
                        for (int32_t f = 0; f < D; ++f) one[f] = blk[f * kDiag + q];
                        const double v = smallest_sum(one, D, d);
                        if (!(v < heap_cut(hp))) continue;
                        approx_pair p = {v, a, a + s0 + q};
                        if (hp->n < hp->cap) heap_push(hp, p); else heap_replace_top(hp, p);
                    }
                }
            }
        }
        free(C);
        free(d2);
    }
    /* merge: every pair left out by a thread is >= that thread's final cut */
    double th = INFINITY;
    int64_t total = 0;
    for (int t = 0; t < nthreads; ++t) {
        total += heaps[t].n;
        if (heaps[t].n == heaps[t].cap && heaps[t].e[0].v < th) th = heaps[t].e[0].v;
    }
    approx_pair* all = (approx_pair*)malloc(sizeof(approx_pair) * (size_t)(total > 0 ? total : 1));
    int64_t m = 0;
    for (int t = 0; t < nthreads; ++t) {
        memcpy(all + m, heaps[t].e, sizeof(approx_pair) * (size_t)heaps[t].n);
        m += heaps[t].n;
        free(heaps[t].e);
    }
    free(heaps);
    qsort(all, (size_t)m, sizeof(approx_pair), approx_cmp);
    if (m > pool) {
        if (all[pool].v < th) th = all[pool].v;
        m = pool;
    }
    *count = m;
    *theta = th;
    return all;
}

/* Exact top-k (the answer of orc_topk_exact) by the diagonal sweep. pool is
 * the initial number of pairs kept (per thread and after the merge); info,
 * if not NULL, receives {theta, eps, pool, passes, max |approx - exact| over
 * the kept pairs}. Returns the number of motifs, -1 on allocation failure,
 * -2 when no pool up to 2^26 pairs certifies the answer. */
int32_t orc_topk_exact_sweep(const double* x, int64_t n, int32_t D, int32_t w, int32_t d, int32_t k,
                             int64_t pool, orc_motif* out, double* info)
{
    const int64_t ns = n - w + 1;
    sweep_ctx c;
    c.n = n; c.ns = ns; c.D = D; c.w = w; c.d = d; c.x = x;
    /* kDiag zeros of padding after the last window of the last dimension */
    const size_t cells = (size_t)D * (size_t)ns + kDiag;
    c.mu = (double*)calloc(cells, sizeof(double));
    c.inv = (double*)calloc(cells, sizeof(double));
    c.sflag = (double*)calloc(cells, sizeof(double));
    c.df = (double*)calloc(cells, sizeof(double));
    c.dg = (double*)calloc(cells, sizeof(double));
    if (!c.mu || !c.inv || !c.sflag || !c.df || !c.dg) return -1;
    for (int32_t f = 0; f < D; ++f) {
        const double* xf = x + (int64_t)f * n;
        for (int64_t a = 0; a < ns; ++a) {
            double mu, sg;
            int32_t flat;
            orc_window_stats(xf + a, w, &mu, &sg, &flat);
            c.mu[(int64_t)f * ns + a] = mu;
            c.inv[(int64_t)f * ns + a] = flat ? 0.0 : 1.0 / sg;
            c.sflag[(int64_t)f * ns + a] = flat ? 0.0 : 1.0;
        }
        for (int64_t i = 0; i + 1 < ns; ++i) {
            const double* m = c.mu + (int64_t)f * ns;
            c.df[(int64_t)f * ns + i] = (xf[i + w] - xf[i]) / 2.0;
            c.dg[(int64_t)f * ns + i] = (xf[i + w] - m[i + 1]) + (xf[i] - m[i]);
        }
    }
    /* Filter error bound: the sweep's dist_f^2 differs from the definition's
     * by rounding only (re-seeded every kReseed steps); 1e-6 w bounds it with
     * a wide margin (the tests report the largest difference seen), and
     * |sqrt(u) - sqrt(v)| <= sqrt(|u - v|). */
    const double eps = (double)d * sqrt(1e-6 * (double)w);
    int32_t got = 0;
    int passes = 0, exact = 0;
    double maxerr = 0.0, theta = INFINITY;
    for (;;) {
        ++passes;
        int64_t cnt = 0;
        approx_pair* cand = sweep(&c, pool, &cnt, &theta);
        orc_motif* ex = (orc_motif*)malloc(sizeof(orc_motif) * (size_t)(cnt > 0 ? cnt : 1));
        maxerr = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(max : maxerr)
#endif
        for (int64_t e = 0; e < cnt; ++e) {
            ex[e].a = cand[e].a;
            ex[e].b = cand[e].b;
            orc_distd(x, n, D, w, cand[e].a, cand[e].b, d, &ex[e].dist_d, &ex[e].dist_max, ex[e].dims, NULL);
            const double err = fabs(ex[e].dist_d - cand[e].v);
            if (err > maxerr) maxerr = err;
        }
        free(cand);
        qsort(ex, (size_t)cnt, sizeof(orc_motif), motif_cmp2);
        got = 0;
        for (int64_t e = 0; e < cnt && got < k; ++e) {
            int ok = 1;
            for (int32_t s = 0; s < got && ok; ++s)
                if (overlaps(ex[e].a, out[s].a, w) || overlaps(ex[e].a, out[s].b, w) ||
                    overlaps(ex[e].b, out[s].a, w) || overlaps(ex[e].b, out[s].b, w))
                    ok = 0;
            if (ok) out[got++] = ex[e];
        }
        free(ex);
        exact = isinf(theta) || (got == k && out[k - 1].dist_d < theta - eps);
        if (exact || pool >= ((int64_t)1 << 26)) break;
        pool *= 4;
    }
    if (info) {
        info[0] = theta;
        info[1] = eps;
        info[2] = (double)pool;
        info[3] = (double)passes;
        info[4] = maxerr;
    }
    free(c.mu); free(c.inv); free(c.sflag); free(c.df); free(c.dg);
    return exact ? got : -2;   /* -2: no pool size up to 2^26 could certify the answer */
}
