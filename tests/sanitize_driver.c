/* Drives the C oracle end to end on a small seeded input so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer can check its memory
 * accesses and arithmetic: window statistics, projections and r, hashing and
 * packing, the LSH search under each stopping rule (with and without the
 * step trace and the exact fallback), and both exact top-k routines, whose
 * answers must agree. Test infrastructure only (built and run by
 * tests/test_oracle_sanitize.py); the oracle's own functions are declared
 * here as the oracle defines them. Prints "ok" when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t a, b;
    double dist_d, dist_max;
    uint64_t dims[2];
} orc_motif;

typedef struct {
    int32_t K, L, rule;
    int32_t no_fallback;
    double r;
    int64_t* cand;
    int64_t cand_cap;
    int64_t cand_count;
    int32_t* top_size;
    int64_t* top_pairs;
    double* top_distmax;
    int32_t i_stop, J_stop;
    int64_t n_verified;
    int64_t n_collisions;
} orc_lsh_ctl;

void orc_stats(const double* x, int64_t n, int32_t D, int32_t w, double* mu, double* sigma, int32_t* flat);
void orc_tensor_shape(int32_t L, int32_t* m, int32_t* n_left, int32_t* n_right);
void orc_draw_projections(uint64_t seed, int32_t D, int32_t w, int32_t C, double* R, double* U);
double orc_estimate_r(const double* x, int64_t n, int32_t D, int32_t w, uint64_t seed);
void orc_hash_all(const double* x, int64_t n, int32_t D, int32_t w, const double* R, const double* U,
                  int32_t C, double r, uint8_t* bytes);
void orc_pack(const uint8_t* bytes, int64_t ns, int32_t D, int32_t NF, int32_t K, uint32_t* words);
int32_t orc_lsh_search(const double* x, int64_t n, int32_t D, int32_t w, int32_t d, int32_t k,
                       double delta, const uint32_t* words, orc_lsh_ctl* ctl, orc_motif* out);
int32_t orc_topk_exact(const double* x, int64_t n, int32_t D, int32_t w, int32_t d, int32_t k,
                       orc_motif* out);
int32_t orc_topk_exact_sweep(const double* x, int64_t n, int32_t D, int32_t w, int32_t d, int32_t k,
                             int64_t pool, orc_motif* out, double* info);
int32_t orc_motif_size(void);
int32_t orc_ctl_size(void);

static int fails = 0;
#define CHECK(c, ...)                      \
    do {                                   \
        if (!(c)) {                        \
            fprintf(stderr, __VA_ARGS__);  \
            fprintf(stderr, "\n");         \
            ++fails;                       \
        }                                  \
    } while (0)

/* Seeded input: D random walks of n points (a 64-bit LCG and the sum of
 * twelve uniforms as a unit-variance step), one window copied with small
 * noise into two dimensions, and a flat stretch (constant windows, sigma 0). */
static uint64_t lcg = 0x9E3779B97F4A7C15ull;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}
static double step(void)
{
    double s = 0.0;
    for (int i = 0; i < 12; ++i) s += unif();
    return s - 6.0;
}

static void make_series(double* x, int64_t n, int32_t D, int32_t w)
{
    for (int32_t f = 0; f < D; ++f) {
        double v = 0.0;
        for (int64_t t = 0; t < n; ++t) x[f * n + t] = (v += step());
    }
    const int64_t p0 = n / 8, p1 = n / 2;
    for (int32_t f = 0; f < 2; ++f)
        for (int32_t t = 0; t < w; ++t) x[f * n + p1 + t] = x[f * n + p0 + t] + 0.05 * step();
    for (int64_t t = 3 * n / 4; t < 3 * n / 4 + w + 5 && t < n; ++t) x[(D - 1) * n + t] = 1.5;
}

static int same_answer(const orc_motif* a, int32_t na, const orc_motif* b, int32_t nb)
{
    if (na != nb) return 0;
    for (int32_t s = 0; s < na; ++s)
        if (a[s].a != b[s].a || a[s].b != b[s].b || fabs(a[s].dist_d - b[s].dist_d) > 1e-9 * (1.0 + a[s].dist_d))
            return 0;
    return 1;
}

int main(void)
{
    CHECK(orc_motif_size() == (int32_t)sizeof(orc_motif), "motif layout differs");
    CHECK(orc_ctl_size() == (int32_t)sizeof(orc_lsh_ctl), "control block layout differs");
    const int64_t n = 700;
    const int32_t D = 4, w = 24, d = 2, k = 3, K = 8, L = 12;
    const int64_t ns = n - w + 1;
    const uint64_t seed = 20250214ull;
    double* x = (double*)malloc(sizeof(double) * (size_t)(n * D));
    make_series(x, n, D, w);

    double* mu = (double*)malloc(sizeof(double) * (size_t)(ns * D));
    double* sg = (double*)malloc(sizeof(double) * (size_t)(ns * D));
    int32_t* flat = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ns * D));
    orc_stats(x, n, D, w, mu, sg, flat);
    int64_t nflat = 0;
    for (int64_t i = 0; i < ns * D; ++i) nflat += flat[i] != 0;
    CHECK(nflat > 0, "the flat stretch gave no flat window");

    int32_t m, nl, nr;
    orc_tensor_shape(L, &m, &nl, &nr);
    const int32_t NF = nl + nr, C = 4 * NF;
    double* R = (double*)malloc(sizeof(double) * (size_t)D * w * C);
    double* U = (double*)malloc(sizeof(double) * (size_t)D * C);
    orc_draw_projections(seed, D, w, C, R, U);
    const double r = orc_estimate_r(x, n, D, w, seed);
    CHECK(r > 0.0 && isfinite(r), "r = %g", r);
    uint8_t* bytes = (uint8_t*)malloc((size_t)D * ns * C);
    orc_hash_all(x, n, D, w, R, U, C, r, bytes);
    uint32_t* words = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)D * NF * ns);
    orc_pack(bytes, ns, D, NF, K, words);

    orc_motif exact[3], sweep[3], lsh[3];
    const int32_t ne = orc_topk_exact(x, n, D, w, d, k, exact);
    double info[5];
    const int32_t nsw = orc_topk_exact_sweep(x, n, D, w, d, k, 1 << 12, sweep, info);
    CHECK(ne == k, "exact top-k found %d motifs", ne);
    CHECK(same_answer(exact, ne, sweep, nsw), "the sweep's answer differs from the exact enumeration's");

    const int32_t steps = K * L;
    for (int32_t rule = 0; rule < 4; ++rule)
        for (int32_t traced = 0; traced < 2; ++traced) {
            orc_lsh_ctl ctl;
            memset(&ctl, 0, sizeof ctl);
            ctl.K = K;
            ctl.L = L;
            ctl.rule = rule;
            ctl.r = r;
            int64_t* cand = NULL;
            int32_t* tsz = NULL;
            int64_t* tp = NULL;
            double* tdm = NULL;
            if (traced) {
                ctl.cand_cap = 1 << 14;
                cand = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)ctl.cand_cap);
                tsz = (int32_t*)malloc(sizeof(int32_t) * (size_t)steps);
                tp = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)steps * k);
                tdm = (double*)malloc(sizeof(double) * (size_t)steps);
                ctl.cand = cand;
                ctl.top_size = tsz;
                ctl.top_pairs = tp;
                ctl.top_distmax = tdm;
            }
            const int32_t got = orc_lsh_search(x, n, D, w, d, k, 0.1, words, &ctl, lsh);
            CHECK(got >= 1 && got <= k, "rule %d: %d motifs", rule, got);
            if (ctl.i_stop == 0)   /* no step stopped: the exact answer */
                CHECK(same_answer(exact, ne, lsh, got), "rule %d: fallback differs from the exact answer", rule);
            for (int32_t s = 1; s < got; ++s)
                CHECK(lsh[s - 1].dist_d <= lsh[s].dist_d, "rule %d: answer out of order", rule);
            /* a delta that no step reaches (under the literal tensoring
             * reading a pair whose collision probability rounds to 1 can
             * still stop): the exact answer */
            orc_lsh_ctl c2 = ctl;
            c2.cand = NULL;
            c2.cand_cap = 0;
            c2.top_size = NULL;
            c2.top_pairs = NULL;
            c2.top_distmax = NULL;
            const int32_t g2 = orc_lsh_search(x, n, D, w, d, k, 1e-300, words, &c2, lsh);
            CHECK(rule == 2 || c2.i_stop == 0, "rule %d: stopped at delta 1e-300", rule);
            if (c2.i_stop == 0)
                CHECK(same_answer(exact, ne, lsh, g2), "rule %d: delta 1e-300 is not exact", rule);
            /* no fallback: nothing when no step stops */
            c2.no_fallback = 1;
            const int32_t g3 = orc_lsh_search(x, n, D, w, d, k, 1e-300, words, &c2, lsh);
            CHECK((g3 == 0) == (c2.i_stop == 0), "rule %d: %d motifs without fallback, stop %d", rule, g3,
                  c2.i_stop);
            free(cand);
            free(tsz);
            free(tp);
            free(tdm);
        }

    free(x);
    free(mu);
    free(sg);
    free(flat);
    free(R);
    free(U);
    free(bytes);
    free(words);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
