/* Drives the oracle's entry points on small seeded inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py):
 * the flat and bucketed searches (with eps and a core subset), per-target
 * numerators, top-k, class counts, PT2, the balance and the dense H.  Exits 0
 * when every call succeeds and the bucketed search agrees with the flat one. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t count;
    uint64_t *keys;
    double *num, *hdiag, *score, *num_abs, *hdiag_abs, *tol;
    int64_t npairs;
} oracle_result;
typedef struct {
    int64_t candidates, npairs;
    double pt2, pt2_abs, pt2_tol, max_drop_upper;
} oracle_bucket_stats;

int oracle_search(const double *, const double *, int, int, int, double, const uint64_t *, const double *, int64_t,
                  double, int64_t, double, int, oracle_result *);
int oracle_search_buckets(const double *, const double *, int, int, int, double, const uint64_t *, const double *,
                          int64_t, double, int64_t, double, int, int, int, int, int64_t, oracle_result *,
                          oracle_bucket_stats *);
void oracle_free(oracle_result *);
int64_t oracle_topk(const uint64_t *, const double *, int64_t, int64_t, int64_t *);
double oracle_energy(const double *, const double *, int, double, const uint64_t *, const double *, int64_t);
int64_t oracle_class_counts(int, int, int, const uint64_t *, const double *, int64_t, int64_t, int, uint64_t *,
                            int64_t *, int64_t);
int oracle_target_numerators(const double *, const double *, int, int, int, double, const uint64_t *, const double *,
                             int64_t, int64_t, const uint64_t *, int64_t, double *, double *, int *, int64_t *,
                             double *, double *);
int oracle_pt2(const double *, const double *, int, int, int, double, const uint64_t *, const double *, int64_t, double,
               int64_t, double, double *, double *, int64_t *);
int oracle_balance(const int64_t *, int64_t, int, int *, int64_t *);
int oracle_hmat_dense(const double *, const double *, int, double, const uint64_t *, int64_t, double *, double *);

static uint64_t rng = 88172645463325252ull;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * 0x1p-53;
}

static uint64_t random_string(int n, int k)
{
    uint64_t s = 0;
    while (__builtin_popcountll(s) < k) s |= 1ull << (int)(urand() * n);
    return s;
}

static int run_case(int n, int na, int nb, int nd, int64_t ncore, double eps)
{
    double *h = calloc((size_t)n * n, sizeof(double)), *eri = calloc((size_t)n * n * n * n, sizeof(double));
    for (int p = 0; p < n; ++p)
        for (int q = 0; q <= p; ++q) h[p * n + q] = h[q * n + p] = (p == q ? -1.0 + 0.2 * p : 0.1 * (urand() - 0.5));
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    /* symmetric by construction: a function of the unordered pairs */
                    int a = p < q ? p : q, b = p < q ? q : p, c = r < s ? r : s, d = r < s ? s : r;
                    int x = a * n + b, y = c * n + d, lo = x < y ? x : y, hi = x < y ? y : x;
                    eri[((p * n + q) * n + r) * n + s] = 0.05 * ((lo * 31 + hi * 17) % 13) / 13.0 + (p == q && r == s ? 0.5 : 0.0);
                }
    uint64_t *dets = malloc(sizeof(uint64_t) * 2 * (size_t)nd);
    double *c = malloc(sizeof(double) * (size_t)nd);
    int m = 0;
    while (m < nd) {
        uint64_t a = random_string(n, na), b = random_string(n, nb);
        int dup = 0;
        for (int j = 0; j < m; ++j) dup |= dets[2 * j] == a && dets[2 * j + 1] == b;
        if (dup) continue;
        dets[2 * m] = a;
        dets[2 * m + 1] = b;
        c[m] = (urand() - 0.5) / (1.0 + m);
        ++m;
    }
    const double E0 = oracle_energy(h, eri, n, 0.1, dets, c, nd);
    oracle_result flat, bk;
    oracle_bucket_stats st;
    int bad = 0;
    bad |= oracle_search(h, eri, n, na, nb, 0.1, dets, c, nd, E0, ncore, eps, 0, &flat) != 0;
    bad |= oracle_search_buckets(h, eri, n, na, nb, 0.1, dets, c, nd, E0, ncore, eps, 7, 0, 7, 3, 0, &bk, &st) != 0;
    bad |= flat.count != bk.count || st.candidates != flat.count;
    /* same multiset of (key, score) bits: compare sums of hashed records */
    uint64_t hf = 0, hb = 0;
    for (int64_t j = 0; j < flat.count; ++j) {
        uint64_t w;
        memcpy(&w, &flat.score[j], 8);
        hf += (flat.keys[2 * j] * 0x9E3779B97F4A7C15ull) ^ (flat.keys[2 * j + 1] + w);
        memcpy(&w, &bk.score[j], 8);
        hb += (bk.keys[2 * j] * 0x9E3779B97F4A7C15ull) ^ (bk.keys[2 * j + 1] + w);
    }
    bad |= hf != hb;
    int64_t k = flat.count < 50 ? flat.count : 50;
    int64_t *idx = malloc(sizeof(int64_t) * (size_t)(k + 1));
    bad |= oracle_topk(flat.keys, flat.score, flat.count, k, idx) != k;
    oracle_result top;
    bad |= oracle_search_buckets(h, eri, n, na, nb, 0.1, dets, c, nd, E0, ncore, eps, 4, 0, 4, 2, 5, &top, &st) != 0;
    double *num = malloc(sizeof(double) * (size_t)(k + 1)), *hd = malloc(sizeof(double) * (size_t)(k + 1));
    double *na_ = malloc(sizeof(double) * (size_t)(k + 1)), *ha_ = malloc(sizeof(double) * (size_t)(k + 1));
    int *inp = malloc(sizeof(int) * (size_t)(k + 1));
    int64_t *nc = malloc(sizeof(int64_t) * (size_t)(k + 1));
    uint64_t *tg = malloc(sizeof(uint64_t) * 2 * (size_t)(k + 1));
    for (int64_t j = 0; j < k; ++j) {
        tg[2 * j] = flat.keys[2 * idx[j]];
        tg[2 * j + 1] = flat.keys[2 * idx[j] + 1];
    }
    bad |= oracle_target_numerators(h, eri, n, na, nb, 0.1, dets, c, nd, ncore, tg, k, num, hd, inp, nc, na_, ha_) != 0;
    uint64_t masks[4096];
    int64_t counts[4096];
    bad |= oracle_class_counts(n, na, nb, dets, c, nd, ncore, 3, masks, counts, 4096) < 0;
    double e2, sabs;
    int64_t cnt;
    bad |= oracle_pt2(h, eri, n, na, nb, 0.1, dets, c, nd, E0, ncore, eps, &e2, &sabs, &cnt) != 0;
    int owner[4096];
    int64_t work[8];
    bad |= oracle_balance(counts, 100, 8, owner, work) != 0;
    double *H = malloc(sizeof(double) * (size_t)nd * nd), *Ha = malloc(sizeof(double) * (size_t)nd * nd);
    bad |= oracle_hmat_dense(h, eri, n, 0.1, dets, nd, H, Ha) != 0;
    oracle_free(&flat);
    oracle_free(&bk);
    oracle_free(&top);
    free(h); free(eri); free(dets); free(c); free(idx); free(num); free(hd); free(na_); free(ha_);
    free(inp); free(nc); free(tg); free(H); free(Ha);
    printf("case n=%d na=%d nb=%d nd=%d ncore=%lld eps=%g: %s\n", n, na, nb, nd, (long long)ncore, eps,
           bad ? "FAIL" : "ok");
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_case(6, 3, 3, 12, 0, 0.0);
    bad |= run_case(8, 4, 3, 30, 10, 0.0);
    bad |= run_case(9, 4, 4, 25, 0, 1e-3);
    bad |= run_case(34, 3, 2, 8, 0, 0.0);
    bad |= run_case(5, 0, 2, 6, 0, 0.0);
    return bad;
}
