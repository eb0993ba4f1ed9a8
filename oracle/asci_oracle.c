/*
 * ASCI determinant-search oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of what the ASCI
 * determinant search computes.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, calls or includes it, and it shares no code with that library.
 *
 * What it follows (paper: Williams-Young et al., "A Parallel, Distributed Memory
 * Implementation of the Adaptive Sampling Configuration Interaction Method"):
 *   - Eq. (1): a candidate a outside the wave function gets the partial scores
 *     H_ai C_i / (E0 - H_aa) from every core determinant i; the score is their
 *     sum.  (The paper writes the denominator as H_aa - E0; this library
 *     uses E0 - H_aa, so every score is the negative of the paper's S_a.  The
 *     selection uses |score| and is unaffected.)
 *   - Sec. II.A: only determinants singly or doubly connected to a core
 *     determinant can receive a non-zero score; candidates exclude every input
 *     determinant.
 *   - Alg. 2 (ASCI search): core set = the N_cdets input determinants of
 *     largest |C|; one pass over the cores generates (target, partial score)
 *     pairs; pairs are sorted on the target bitstring and summed per target;
 *     the N_tdets targets of largest |score| are kept.
 *   - Alg. 2's threshold: with eps > 0 a pair is kept only when its partial
 *     score exceeds eps in magnitude.
 *
 * Conventions (the paper fixes none; they are part of this library's ABI):
 *   - a determinant is (alpha, beta), two 64-bit strings, bit p = spatial
 *     orbital p;
 *   - spin orbitals are ordered alpha first then beta, each ascending, and a
 *     determinant is the product of creators in that order acting on vacuum,
 *     so a^+_q a_p acting on a determinant has sign (-1)^(number of occupied
 *     orbitals of that spin strictly between p and q);
 *   - h is n x n, eri is (pq|rs) in chemists' notation, n^4 row-major, real,
 *     with the 8-fold permutational symmetry;
 *   - sums are evaluated left to right in the order written below, with no
 *     fused multiply-add (build with -ffp-contract=off).
 *
 * Slater-Condon rules used by oracle_helem (textbook, written out here):
 *   diagonal: H_aa = ecore + sum_{p in alpha} h_pp + sum_{p in beta} h_pp
 *                   + sum_{p<q in alpha} (J_pq - K_pq) + sum_{p<q in beta} (J_pq - K_pq)
 *                   + sum_{p in alpha, q in beta} J_pq,
 *             with J_pq = (pp|qq), K_pq = (pq|qp); one running sum from ecore,
 *             the groups in the order written, each ascending in p, then q.
 *   single p -> q of spin s (i has p, a has q):
 *             H_ai = sign * ( h_qp + sum_{r in occ_s(i), r != p} [(qp|rr) - (qr|rp)]
 *                                  + sum_{r in occ_other(i)} (qp|rr) ), r ascending.
 *   same-spin double, holes p < r of i, particles q < s of a:
 *             H_ai = sign(p->q on i) * sign(r->s on i') * [(qp|sr) - (qr|sp)],
 *             i' = i with p replaced by q.
 *   opposite-spin double, alpha p -> q, beta r -> s:
 *             H_ai = sign_alpha(p->q) * sign_beta(r->s) * (qp|sr).
 *
 * Rounding.  The paper fixes no evaluation order, and E0 lies inside the
 * diagonal spectrum, so E0 - H_aa can cancel badly.  Besides each value the
 * oracle therefore reports the magnitude sums that bound the effect of any
 * other evaluation order: for N_a, num_abs = sum_i |C_i| * (sum of |terms| of
 * H_ai) over the integrals entering H_ai; for H_aa, hdiag_abs = |ecore| +
 * sum of |h_pp|, |J_pq|, |K_pq| over its terms.  A result computed in another
 * order is accepted when it lies within
 *     tol_a = max(1e-12 |A_a|, 64 u (num_abs + |N_a| (|E0| + hdiag_abs) / |d|) / |d|),
 *     d = E0 - H_aa, u = 2^-53,
 * i.e. max(1e-12, 64 u (kappa_num + kappa_den)) relative to |A_a| with the
 * condition numbers kappa_num = num_abs / |N_a| and
 * kappa_den = (|E0| + hdiag_abs) / |d| (oracle_score_tol).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

typedef struct {
    int n;
    const double *h;
    const double *eri;
    double ecore;
} ham_t;

static double H1(const ham_t *H, int p, int q) { return H->h[(size_t)p * H->n + q]; }

static double V(const ham_t *H, int p, int q, int r, int s)
{
    size_t n = (size_t)H->n;
    return H->eri[((p * n + q) * n + r) * n + s];
}

static int popc(uint64_t x) { return __builtin_popcountll(x); }

/* (-1)^(number of set bits of occ strictly between orbitals p and q) */
static int between_sign(uint64_t occ, int p, int q)
{
    int lo = p < q ? p : q, hi = p < q ? q : p;
    int cnt = 0;
    for (int t = lo + 1; t < hi; ++t)
        if ((occ >> t) & 1ull)
            ++cnt;
    return (cnt & 1) ? -1 : 1;
}

/* lowest set bit index; x must be non-zero */
static int first_bit(uint64_t x)
{
    for (int t = 0; t < 64; ++t)
        if ((x >> t) & 1ull)
            return t;
    return -1;
}

/* H_aa by the diagonal rule above: one running sum from ecore, the groups in
 * the order written; *abs_out (optional) receives |ecore| + the sum of
 * |h_pp|, |J_pq|, |K_pq| over the terms */
static double hdiag_eval(const ham_t *H, uint64_t alpha, uint64_t beta, double *abs_out)
{
    const int n = H->n;
    double e = H->ecore, s = fabs(H->ecore);
    for (int p = 0; p < n; ++p)
        if ((alpha >> p) & 1ull) { e = e + H1(H, p, p); s = s + fabs(H1(H, p, p)); }
    for (int p = 0; p < n; ++p)
        if ((beta >> p) & 1ull) { e = e + H1(H, p, p); s = s + fabs(H1(H, p, p)); }
    for (int spin = 0; spin < 2; ++spin) {
        const uint64_t x = spin == 0 ? alpha : beta;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q)
                if (((x >> p) & 1ull) && ((x >> q) & 1ull)) {
                    const double J = V(H, p, p, q, q), K = V(H, p, q, q, p);
                    e = e + (J - K);
                    s = s + (fabs(J) + fabs(K));
                }
    }
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            if (((alpha >> p) & 1ull) && ((beta >> q) & 1ull)) {
                e = e + V(H, p, p, q, q);
                s = s + fabs(V(H, p, p, q, q));
            }
    if (abs_out) *abs_out = s;
    return e;
}

double oracle_hdiag(const double *h, const double *eri, int n, double ecore,
                    uint64_t alpha, uint64_t beta)
{
    ham_t Hs = {n, h, eri, ecore};
    return hdiag_eval(&Hs, alpha, beta, NULL);
}

/* single excitation p -> q in the string `same` (spin s) of determinant i,
 * with `other` the string of the other spin of i; *abs_out gets the sum of
 * |terms| */
static double single_elem(const ham_t *H, uint64_t same, uint64_t other, int p, int q, double *abs_out)
{
    double v = H1(H, q, p), s = fabs(H1(H, q, p));
    for (int r = 0; r < H->n; ++r)
        if (r != p && ((same >> r) & 1ull)) {
            const double J = V(H, q, p, r, r), K = V(H, q, r, r, p);
            v = v + (J - K);
            s = s + (fabs(J) + fabs(K));
        }
    for (int r = 0; r < H->n; ++r)
        if ((other >> r) & 1ull) {
            v = v + V(H, q, p, r, r);
            s = s + fabs(V(H, q, p, r, r));
        }
    *abs_out = s;
    return between_sign(same, p, q) * v;
}

/* <a|H|i> and the sum of |terms| that form it; zero beyond double excitations */
static double helem_eval(const ham_t *H, uint64_t a_alpha, uint64_t a_beta, uint64_t i_alpha, uint64_t i_beta,
                         double *abs_out)
{
    uint64_t da = a_alpha ^ i_alpha, db = a_beta ^ i_beta;
    int ea = popc(da) / 2, eb = popc(db) / 2;
    double s = 0.0;
    double v;
    if (ea + eb == 0) {
        v = hdiag_eval(H, a_alpha, a_beta, &s);
    } else if (ea + eb > 2) {
        v = 0.0;
    } else if (ea == 1 && eb == 0) {
        int p = first_bit(i_alpha & ~a_alpha), q = first_bit(a_alpha & ~i_alpha);
        v = single_elem(H, i_alpha, i_beta, p, q, &s);
    } else if (ea == 0 && eb == 1) {
        int p = first_bit(i_beta & ~a_beta), q = first_bit(a_beta & ~i_beta);
        v = single_elem(H, i_beta, i_alpha, p, q, &s);
    } else if (ea == 1 && eb == 1) {
        int p = first_bit(i_alpha & ~a_alpha), q = first_bit(a_alpha & ~i_alpha);
        int r = first_bit(i_beta & ~a_beta), t = first_bit(a_beta & ~i_beta);
        int sg = between_sign(i_alpha, p, q) * between_sign(i_beta, r, t);
        v = sg * V(H, q, p, t, r);
        s = fabs(V(H, q, p, t, r));
    } else {
        /* same-spin double */
        uint64_t si = ea == 2 ? i_alpha : i_beta;
        uint64_t sa = ea == 2 ? a_alpha : a_beta;
        uint64_t holes = si & ~sa, parts = sa & ~si;
        int p = first_bit(holes), r = first_bit(holes & (holes - 1));
        int q = first_bit(parts), t = first_bit(parts & (parts - 1));
        int s1 = between_sign(si, p, q);
        uint64_t mid = (si & ~(1ull << p)) | (1ull << q);
        int s2 = between_sign(mid, r, t);
        v = s1 * s2 * (V(H, q, p, t, r) - V(H, q, r, t, p));
        s = fabs(V(H, q, p, t, r)) + fabs(V(H, q, r, t, p));
    }
    if (abs_out) *abs_out = s;
    return v;
}

double oracle_helem(const double *h, const double *eri, int n, double ecore,
                    uint64_t a_alpha, uint64_t a_beta, uint64_t i_alpha, uint64_t i_beta)
{
    ham_t Hs = {n, h, eri, ecore};
    return helem_eval(&Hs, a_alpha, a_beta, i_alpha, i_beta, NULL);
}

/* Absolute tolerance of a score computed in another evaluation order (see
 * "Rounding" above): max(1e-12 |A|, 64 u (num_abs + |N| (|E0| + hdiag_abs) / |d|) / |d|) */
double oracle_score_tol(double num, double num_abs, double hdiag, double hdiag_abs, double E0)
{
    const double u = 0x1p-53;
    const double d = fabs(E0 - hdiag);
    const double A = fabs(num / (E0 - hdiag));
    const double cond = 64.0 * u * (num_abs + fabs(num) * (fabs(E0) + hdiag_abs) / d) / d;
    const double rel = 1e-12 * A;
    return cond > rel ? cond : rel;
}

/* ---- enumeration of the singles and doubles of one determinant (Sec. II.A) ---- */

/* all strings reachable from `x` (width n) by moving exactly m = 1 or 2 electrons */
static int64_t string_moves(uint64_t x, int n, int m, uint64_t *out)
{
    int64_t cnt = 0;
    for (int p = 0; p < n; ++p) {
        if (!((x >> p) & 1ull))
            continue;
        for (int q = 0; q < n; ++q) {
            if ((x >> q) & 1ull)
                continue;
            uint64_t y = (x & ~(1ull << p)) | (1ull << q);
            if (m == 1) {
                out[cnt++] = y;
                continue;
            }
            for (int r = p + 1; r < n; ++r) {
                if (!((x >> r) & 1ull))
                    continue;
                for (int s = q + 1; s < n; ++s) {
                    if (((x >> s) & 1ull) || s == q)
                        continue;
                    out[cnt++] = (y & ~(1ull << r)) | (1ull << s);
                }
            }
        }
    }
    return cnt;
}

static int64_t choose2(int64_t k) { return k * (k - 1) / 2; }

/* number of singles + doubles of any determinant with these occupations */
int64_t oracle_sd_count(int n, int na, int nb)
{
    int64_t va = n - na, vb = n - nb;
    return (int64_t)na * va + (int64_t)nb * vb + choose2(na) * choose2(va) +
           choose2(nb) * choose2(vb) + (int64_t)na * va * nb * vb;
}

/* every determinant at excitation degree 1 or 2 from (alpha, beta); returns the count */
int64_t oracle_sd_targets(int n, uint64_t alpha, uint64_t beta, uint64_t *out /* 2*cap */)
{
    int na = popc(alpha), nb = popc(beta);
    int64_t ma1 = (int64_t)na * (n - na), mb1 = (int64_t)nb * (n - nb);
    int64_t ma2 = choose2(na) * choose2(n - na), mb2 = choose2(nb) * choose2(n - nb);
    int64_t cap = ma1 > mb1 ? ma1 : mb1;
    if (ma2 > cap) cap = ma2;
    if (mb2 > cap) cap = mb2;
    uint64_t *a1 = malloc(sizeof(uint64_t) * (size_t)(ma1 + 1));
    uint64_t *b1 = malloc(sizeof(uint64_t) * (size_t)(mb1 + 1));
    uint64_t *t2 = malloc(sizeof(uint64_t) * (size_t)(cap + 1));
    int64_t cnt = 0;
    string_moves(alpha, n, 1, a1);
    string_moves(beta, n, 1, b1);
    for (int64_t x = 0; x < ma1; ++x) { out[2 * cnt] = a1[x]; out[2 * cnt + 1] = beta; ++cnt; }
    for (int64_t y = 0; y < mb1; ++y) { out[2 * cnt] = alpha; out[2 * cnt + 1] = b1[y]; ++cnt; }
    int64_t k2 = string_moves(alpha, n, 2, t2);
    for (int64_t x = 0; x < k2; ++x) { out[2 * cnt] = t2[x]; out[2 * cnt + 1] = beta; ++cnt; }
    k2 = string_moves(beta, n, 2, t2);
    for (int64_t y = 0; y < k2; ++y) { out[2 * cnt] = alpha; out[2 * cnt + 1] = t2[y]; ++cnt; }
    for (int64_t x = 0; x < ma1; ++x)
        for (int64_t y = 0; y < mb1; ++y) { out[2 * cnt] = a1[x]; out[2 * cnt + 1] = b1[y]; ++cnt; }
    free(a1);
    free(b1);
    free(t2);
    return cnt;
}

/* ---- validation ---- */

static int validate(int n, int na, int nb, const uint64_t *dets, int64_t ndets)
{
    if (n < 1 || n > 64 || na < 0 || na > n || nb < 0 || nb > n || ndets < 0)
        return ORACLE_EINVAL;
    uint64_t full = n == 64 ? ~0ull : ((1ull << n) - 1);
    for (int64_t i = 0; i < ndets; ++i) {
        uint64_t a = dets[2 * i], b = dets[2 * i + 1];
        if ((a & ~full) || (b & ~full) || popc(a) != na || popc(b) != nb)
            return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/* ---- ASCI search (Alg. 2) ---- */

typedef struct {
    uint64_t a, b;
    int64_t core;
    double v;     /* H_ai C_i */
    double vabs;  /* |C_i| * (sum of |terms| of H_ai) */
} pair_rec;

static int cmp_pair(const void *x, const void *y)
{
    const pair_rec *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->core != q->core) return p->core < q->core ? -1 : 1;
    return 0;
}

typedef struct { uint64_t a, b; } key_t2;

static int cmp_key(const void *x, const void *y)
{
    const key_t2 *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return 0;
}

typedef struct { double absc; int64_t idx; } core_rank;

static int cmp_core(const void *x, const void *y)
{
    const core_rank *p = x, *q = y;
    if (p->absc != q->absc) return p->absc > q->absc ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

static int cmp_i64(const void *x, const void *y)
{
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return a < b ? -1 : (a > b);
}

/* Indices of the core determinants in ascending input order: the ncore inputs of
 * largest |C| (ties: lower index first), or all inputs when ncore <= 0 or ncore >= ndets. */
int64_t oracle_core_set(const double *coeffs, int64_t ndets, int64_t ncore, int64_t *out)
{
    if (ncore <= 0 || ncore >= ndets) {
        for (int64_t i = 0; i < ndets; ++i) out[i] = i;
        return ndets;
    }
    core_rank *r = malloc(sizeof(core_rank) * (size_t)ndets);
    for (int64_t i = 0; i < ndets; ++i) { r[i].absc = fabs(coeffs[i]); r[i].idx = i; }
    qsort(r, (size_t)ndets, sizeof(core_rank), cmp_core);
    for (int64_t i = 0; i < ncore; ++i) out[i] = r[i].idx;
    free(r);
    qsort(out, (size_t)ncore, sizeof(int64_t), cmp_i64);
    return ncore;
}

typedef struct {
    int64_t count;     /* number of candidates */
    uint64_t *keys;    /* 2*count: alpha, beta, ascending (alpha, beta) */
    double *num;       /* count: N_a = sum_i H_ai C_i, ascending core index */
    double *hdiag;     /* count: H_aa */
    double *score;     /* count: A_a = N_a / (E0 - H_aa) */
    double *num_abs;   /* count: sum_i |C_i| * (sum of |terms| of H_ai) */
    double *hdiag_abs; /* count: |ecore| + sum of |h_pp|, |J_pq|, |K_pq| of H_aa */
    double *tol;       /* count: oracle_score_tol of the candidate */
    int64_t npairs;    /* number of (core, target) pairs kept */
} oracle_result;

void oracle_free(oracle_result *r)
{
    if (!r) return;
    free(r->keys);
    free(r->num);
    free(r->hdiag);
    free(r->score);
    free(r->num_abs);
    free(r->hdiag_abs);
    free(r->tol);
    memset(r, 0, sizeof(*r));
}

static int result_alloc(oracle_result *res, int64_t nu)
{
    res->keys = malloc(sizeof(uint64_t) * 2 * (size_t)(nu + 1));
    res->num = malloc(sizeof(double) * (size_t)(nu + 1));
    res->hdiag = malloc(sizeof(double) * (size_t)(nu + 1));
    res->score = malloc(sizeof(double) * (size_t)(nu + 1));
    res->num_abs = malloc(sizeof(double) * (size_t)(nu + 1));
    res->hdiag_abs = malloc(sizeof(double) * (size_t)(nu + 1));
    res->tol = malloc(sizeof(double) * (size_t)(nu + 1));
    if (!res->keys || !res->num || !res->hdiag || !res->score || !res->num_abs || !res->hdiag_abs || !res->tol) {
        oracle_free(res);
        return ORACLE_ENOMEM;
    }
    return ORACLE_OK;
}

/* Sum every run of equal targets of `pairs` (sorted by target, then core
 * index) in that order, drop input determinants unless keep_psi, and score
 * the rest (Eq. (1)); writes the candidates at res[*u ...].  With res == NULL
 * only counts them. */
static void accumulate_runs(const ham_t *H, const pair_rec *pairs, int64_t np, const key_t2 *psi, int64_t ndets,
                            double E0, int keep_psi, oracle_result *res, int64_t *u)
{
    for (int64_t j = 0; j < np;) {
        int64_t e = j;
        double s = 0.0, sa = 0.0;
        while (e < np && pairs[e].a == pairs[j].a && pairs[e].b == pairs[j].b) {
            s = s + pairs[e].v;
            sa = sa + pairs[e].vabs;
            ++e;
        }
        key_t2 k = {pairs[j].a, pairs[j].b};
        int in_psi = bsearch(&k, psi, (size_t)ndets, sizeof(key_t2), cmp_key) != NULL;
        if (keep_psi || !in_psi) {
            if (res) {
                double ha = 0.0;
                double hd = hdiag_eval(H, k.a, k.b, &ha);
                res->keys[2 * *u] = k.a;
                res->keys[2 * *u + 1] = k.b;
                res->num[*u] = s;
                res->hdiag[*u] = hd;
                res->score[*u] = s / (E0 - hd);
                res->num_abs[*u] = sa;
                res->hdiag_abs[*u] = ha;
                res->tol[*u] = oracle_score_tol(s, sa, hd, ha, E0);
            }
            ++*u;
        }
        j = e;
    }
}

/* psi as a sorted key list, for exclusion and duplicate detection; NULL on
 * duplicates */
static key_t2 *psi_keys(const uint64_t *dets, int64_t ndets)
{
    key_t2 *psi = malloc(sizeof(key_t2) * (size_t)(ndets + 1));
    for (int64_t i = 0; i < ndets; ++i) { psi[i].a = dets[2 * i]; psi[i].b = dets[2 * i + 1]; }
    qsort(psi, (size_t)ndets, sizeof(key_t2), cmp_key);
    for (int64_t i = 1; i < ndets; ++i)
        if (cmp_key(&psi[i - 1], &psi[i]) == 0) { free(psi); return NULL; }
    return psi;
}

/* the pair (core i -> target t): value H_ti C_i and its magnitude sum; with
 * eps > 0, 0 when the partial score |H_ti C_i / (E0 - H_tt)| is not > eps */
static int make_pair(const ham_t *H, uint64_t ta, uint64_t tb, uint64_t ia, uint64_t ib, int64_t i, double ci,
                     double E0, double eps, pair_rec *out)
{
    double ab = 0.0;
    double v = helem_eval(H, ta, tb, ia, ib, &ab) * ci;
    if (eps > 0.0) {
        double d = E0 - hdiag_eval(H, ta, tb, NULL);
        if (!(fabs(v / d) > eps))
            return 0;
    }
    out->a = ta; out->b = tb; out->core = i; out->v = v; out->vabs = ab * fabs(ci);
    return 1;
}

/*
 * The search.  keep_psi != 0 keeps targets that are input determinants (their
 * N_a is then (H C)_a minus the diagonal term, used to pin E0); 0 is the
 * search proper.
 */
int oracle_search(const double *h, const double *eri, int n, int na, int nb, double ecore,
                  const uint64_t *dets, const double *coeffs, int64_t ndets, double E0,
                  int64_t ncore, double eps, int keep_psi, oracle_result *res)
{
    memset(res, 0, sizeof(*res));
    if (validate(n, na, nb, dets, ndets) != ORACLE_OK)
        return ORACLE_EINVAL;
    ham_t Hs = {n, h, eri, ecore};
    const ham_t *H = &Hs;

    key_t2 *psi = psi_keys(dets, ndets);
    if (!psi) return ORACLE_EINVAL;

    int64_t *core = malloc(sizeof(int64_t) * (size_t)(ndets + 1));
    int64_t nq = oracle_core_set(coeffs, ndets, ncore, core);

    int64_t per = oracle_sd_count(n, na, nb);
    int64_t cap = per * nq;
    pair_rec *pairs = malloc(sizeof(pair_rec) * (size_t)(cap + 1));
    uint64_t *tg = malloc(sizeof(uint64_t) * 2 * (size_t)(per + 1));
    if (!pairs || !tg) { free(psi); free(core); free(pairs); free(tg); return ORACLE_ENOMEM; }

    /* one pass over the cores in ascending index: generate every single and
     * double, evaluate the pair value H_ai C_i (and screen it when eps > 0) */
    int64_t np = 0;
    for (int64_t c = 0; c < nq; ++c) {
        int64_t i = core[c];
        uint64_t ia = dets[2 * i], ib = dets[2 * i + 1];
        int64_t nt = oracle_sd_targets(n, ia, ib, tg);
        for (int64_t t = 0; t < nt; ++t)
            np += make_pair(H, tg[2 * t], tg[2 * t + 1], ia, ib, i, coeffs[i], E0, eps, &pairs[np]);
    }
    free(tg);

    /* sort on the target bitstring (core index breaks ties), then accumulate */
    qsort(pairs, (size_t)np, sizeof(pair_rec), cmp_pair);
    int64_t nu = 0;
    accumulate_runs(H, pairs, np, psi, ndets, E0, keep_psi, NULL, &nu);
    int rc = result_alloc(res, nu);
    int64_t u = 0;
    if (rc == ORACLE_OK) accumulate_runs(H, pairs, np, psi, ndets, E0, keep_psi, res, &u);
    res->count = u;
    res->npairs = np;
    free(pairs);
    free(psi);
    free(core);
    return rc;
}

/* ---- selection of the k largest |score| (Alg. 2, last step; duplicate-aware
 *      selection semantics of Sec. II.B): order is |score| descending, compared as
 *      the IEEE-754 bit pattern of |score| (numeric order for non-NaN values),
 *      ties broken by the (alpha, beta) key ascending ---- */

typedef struct {
    uint64_t ord, a, b;
    int64_t idx;
} sel_rec;

static int cmp_sel(const void *x, const void *y)
{
    const sel_rec *p = x, *q = y;
    if (p->ord != q->ord) return p->ord > q->ord ? -1 : 1;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return 0;
}

static uint64_t abs_bits(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof(u));
    return u & 0x7fffffffffffffffull;
}

int64_t oracle_topk(const uint64_t *keys, const double *score, int64_t count, int64_t k,
                    int64_t *out_idx)
{
    if (k < 0)
        return ORACLE_EINVAL;
    sel_rec *r = malloc(sizeof(sel_rec) * (size_t)(count + 1));
    for (int64_t i = 0; i < count; ++i) {
        r[i].ord = abs_bits(score[i]);
        r[i].a = keys[2 * i];
        r[i].b = keys[2 * i + 1];
        r[i].idx = i;
    }
    qsort(r, (size_t)count, sizeof(sel_rec), cmp_sel);
    int64_t m = k < count ? k : count;
    for (int64_t i = 0; i < m; ++i) out_idx[i] = r[i].idx;
    free(r);
    return m;
}

/* ---- the search by target buckets (memory-bounded, threaded) ----
 * The same result as oracle_search, computed bucket by bucket: the targets are
 * partitioned by a hash of their alpha string into nbuckets buckets (a
 * partition of the candidates, so every target, its pairs and its sum stay in
 * one bucket).  A bucket's pairs come from a scan over every core in
 * ascending index that enumerates the core's singles and doubles alpha string
 * first and keeps the targets whose alpha string lies in the bucket; the
 * pairs are then sorted on (target, core), summed and scored by the same
 * routines as oracle_search, so every N_a, H_aa and A_a carries the same bits.
 *
 * The alpha-string hash is an XOR of one random 64-bit word per occupied
 * orbital, bucket = high 32 bits mod nbuckets: moving electrons p -> q changes
 * it by R_p ^ R_q, so the buckets of all singles and doubles of a core are
 * found with a few XORs each.
 *
 * Buckets [b0, b1) are processed, up to nthreads at once.  Candidates are
 * returned bucket by bucket, in ascending key order inside a bucket; with
 * keep_top > 0 a bucket keeps only its keep_top first candidates by (|A| desc,
 * key asc), in that order, and st->max_drop_upper receives the largest
 * |A_a| + tol_a over the candidates dropped (0 when none).  st also receives
 * the candidate and pair counts of the processed buckets and the PT2 sum of
 * their candidates (Neumaier's sum per bucket in key order, the bucket sums
 * then added the same way in bucket order; exact to about 4u sum |terms|),
 * with sum |N_a A_a| and sum (|N_a| tol_a + |A_a| tol(N_a)), tol(N_a) =
 * max(1e-12 |N_a|, 64 u num_abs): how far the terms of another evaluation
 * order may lie from these. */
typedef struct {
    int64_t candidates;
    int64_t npairs;
    double pt2;
    double pt2_abs;
    double pt2_tol;
    double max_drop_upper;
} oracle_bucket_stats;

static uint64_t orb_word(int p)
{
    /* splitmix64 of the orbital index: fixed random words */
    uint64_t z = 0x9E3779B97F4A7C15ull * (uint64_t)(p + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t string_hash(uint64_t x)
{
    uint64_t hsh = 0;
    for (int p = 0; p < 64; ++p)
        if ((x >> p) & 1ull) hsh ^= orb_word(p);
    return hsh;
}

static int bucket_of(uint64_t hsh, int nbuckets) { return (int)((hsh >> 32) % (uint64_t)nbuckets); }

typedef struct {
    double e, c;  /* Neumaier running sum and compensation */
} nsum;

static void nsum_add(nsum *s, double t)
{
    const double y = s->e + t;
    if (fabs(s->e) >= fabs(t))
        s->c = s->c + ((s->e - y) + t);
    else
        s->c = s->c + ((t - y) + s->e);
    s->e = y;
}

/* Every pair of bucket b, or (out == NULL) just their number. */
static int64_t bucket_pairs(const ham_t *H, int na, int nb, const uint64_t *dets, const double *coeffs,
                            const int64_t *core, int64_t nq, int b, int nbuckets, const uint64_t *R, double E0,
                            double eps, pair_rec *out)
{
    const int n = H->n;
    int64_t np = 0;
    uint64_t *b1 = malloc(sizeof(uint64_t) * (size_t)(nb * (n - nb) + 1));
    uint64_t *b2 = malloc(sizeof(uint64_t) * (size_t)(choose2(nb) * choose2(n - nb) + 1));
    const int64_t nb1 = (int64_t)nb * (n - nb), nb2 = choose2(nb) * choose2(n - nb);
    int occ[64], vir[64];
    for (int64_t c = 0; c < nq; ++c) {
        const int64_t i = core[c];
        const uint64_t ia = dets[2 * i], ib = dets[2 * i + 1];
        const double ci = coeffs[i];
        int no = 0, nv = 0;
        for (int p = 0; p < n; ++p) {
            if ((ia >> p) & 1ull) occ[no++] = p;
            else vir[nv++] = p;
        }
        const uint64_t ha = string_hash(ia);
        int have_beta = 0;
        /* alpha unchanged: beta singles and doubles */
        if (bucket_of(ha, nbuckets) == b) {
            if (!out) {
                np += nb1 + nb2;
            } else {
                string_moves(ib, n, 1, b1);
                string_moves(ib, n, 2, b2);
                have_beta = 1;
                for (int64_t y = 0; y < nb1; ++y) np += make_pair(H, ia, b1[y], ia, ib, i, ci, E0, eps, &out[np]);
                for (int64_t y = 0; y < nb2; ++y) np += make_pair(H, ia, b2[y], ia, ib, i, ci, E0, eps, &out[np]);
            }
        }
        /* one alpha electron moves: the alpha single alone, or with a beta single */
        for (int x = 0; x < no; ++x)
            for (int y = 0; y < nv; ++y) {
                if (bucket_of(ha ^ R[occ[x]] ^ R[vir[y]], nbuckets) != b) continue;
                if (!out) { np += 1 + nb1; continue; }
                if (!have_beta) {
                    string_moves(ib, n, 1, b1);
                    string_moves(ib, n, 2, b2);
                    have_beta = 1;
                }
                const uint64_t a2 = (ia & ~(1ull << occ[x])) | (1ull << vir[y]);
                np += make_pair(H, a2, ib, ia, ib, i, ci, E0, eps, &out[np]);
                for (int64_t t = 0; t < nb1; ++t) np += make_pair(H, a2, b1[t], ia, ib, i, ci, E0, eps, &out[np]);
            }
        /* two alpha electrons move: holes x1 < x2, particles y1 < y2 */
        for (int x1 = 0; x1 < no; ++x1)
            for (int x2 = x1 + 1; x2 < no; ++x2) {
                const uint64_t hh = ha ^ R[occ[x1]] ^ R[occ[x2]];
                for (int y1 = 0; y1 < nv; ++y1)
                    for (int y2 = y1 + 1; y2 < nv; ++y2) {
                        if (bucket_of(hh ^ R[vir[y1]] ^ R[vir[y2]], nbuckets) != b) continue;
                        if (!out) { ++np; continue; }
                        const uint64_t a2 = (ia & ~((1ull << occ[x1]) | (1ull << occ[x2]))) |
                                            (1ull << vir[y1]) | (1ull << vir[y2]);
                        np += make_pair(H, a2, ib, ia, ib, i, ci, E0, eps, &out[np]);
                    }
            }
    }
    free(b1);
    free(b2);
    return np;
}

typedef struct {
    oracle_result r;
    int64_t candidates, npairs;
    nsum pt2;
    double pt2_abs, pt2_tol, max_drop_upper;
    int rc;
} bucket_out;

static void run_bucket(const ham_t *H, int na, int nb, const uint64_t *dets, const double *coeffs,
                       const int64_t *core, int64_t nq, const key_t2 *psi, int64_t ndets, int b, int nbuckets,
                       const uint64_t *R, double E0, double eps, int64_t keep_top, bucket_out *o)
{
    memset(o, 0, sizeof(*o));
    const int64_t cap = bucket_pairs(H, na, nb, dets, coeffs, core, nq, b, nbuckets, R, E0, 0.0, NULL);
    pair_rec *pairs = malloc(sizeof(pair_rec) * (size_t)(cap + 1));
    if (!pairs) { o->rc = ORACLE_ENOMEM; return; }
    const int64_t np = bucket_pairs(H, na, nb, dets, coeffs, core, nq, b, nbuckets, R, E0, eps, pairs);
    qsort(pairs, (size_t)np, sizeof(pair_rec), cmp_pair);
    int64_t nu = 0;
    accumulate_runs(H, pairs, np, psi, ndets, E0, 0, NULL, &nu);
    oracle_result all;
    memset(&all, 0, sizeof(all));
    o->rc = result_alloc(&all, nu);
    if (o->rc != ORACLE_OK) { free(pairs); return; }
    int64_t u = 0;
    accumulate_runs(H, pairs, np, psi, ndets, E0, 0, &all, &u);
    free(pairs);
    all.count = u;
    all.npairs = np;
    o->candidates = u;
    o->npairs = np;
    const double uu = 0x1p-53;
    for (int64_t j = 0; j < u; ++j) {
        const double t = all.num[j] * all.score[j];
        nsum_add(&o->pt2, t);
        o->pt2_abs = o->pt2_abs + fabs(t);
        double tn = 64.0 * uu * all.num_abs[j];
        if (tn < 1e-12 * fabs(all.num[j])) tn = 1e-12 * fabs(all.num[j]);
        o->pt2_tol = o->pt2_tol + (fabs(all.num[j]) * all.tol[j] + fabs(all.score[j]) * tn);
    }
    if (keep_top <= 0 || u <= keep_top) {
        o->r = all;
        return;
    }
    int64_t *idx = malloc(sizeof(int64_t) * (size_t)(keep_top + 1));
    sel_rec *sr = malloc(sizeof(sel_rec) * (size_t)u);
    for (int64_t j = 0; j < u; ++j) {
        sr[j].ord = abs_bits(all.score[j]);
        sr[j].a = all.keys[2 * j];
        sr[j].b = all.keys[2 * j + 1];
        sr[j].idx = j;
    }
    qsort(sr, (size_t)u, sizeof(sel_rec), cmp_sel);
    for (int64_t j = 0; j < keep_top; ++j) idx[j] = sr[j].idx;
    for (int64_t j = keep_top; j < u; ++j) {
        const int64_t x = sr[j].idx;
        const double up = fabs(all.score[x]) + all.tol[x];
        if (up > o->max_drop_upper) o->max_drop_upper = up;
    }
    free(sr);
    o->rc = result_alloc(&o->r, keep_top);
    if (o->rc == ORACLE_OK) {
        for (int64_t j = 0; j < keep_top; ++j) {
            const int64_t x = idx[j];
            o->r.keys[2 * j] = all.keys[2 * x];
            o->r.keys[2 * j + 1] = all.keys[2 * x + 1];
            o->r.num[j] = all.num[x];
            o->r.hdiag[j] = all.hdiag[x];
            o->r.score[j] = all.score[x];
            o->r.num_abs[j] = all.num_abs[x];
            o->r.hdiag_abs[j] = all.hdiag_abs[x];
            o->r.tol[j] = all.tol[x];
        }
        o->r.count = keep_top;
    }
    free(idx);
    oracle_free(&all);
}

int oracle_search_buckets(const double *h, const double *eri, int n, int na, int nb, double ecore,
                          const uint64_t *dets, const double *coeffs, int64_t ndets, double E0, int64_t ncore,
                          double eps, int nbuckets, int b0, int b1, int nthreads, int64_t keep_top,
                          oracle_result *res, oracle_bucket_stats *st)
{
    memset(res, 0, sizeof(*res));
    memset(st, 0, sizeof(*st));
    if (validate(n, na, nb, dets, ndets) != ORACLE_OK || nbuckets < 1 || b0 < 0 || b1 > nbuckets || b0 > b1 ||
        nthreads < 1)
        return ORACLE_EINVAL;
    ham_t Hs = {n, h, eri, ecore};
    key_t2 *psi = psi_keys(dets, ndets);
    if (!psi) return ORACLE_EINVAL;
    int64_t *core = malloc(sizeof(int64_t) * (size_t)(ndets + 1));
    const int64_t nq = oracle_core_set(coeffs, ndets, ncore, core);
    uint64_t R[64];
    for (int p = 0; p < 64; ++p) R[p] = orb_word(p);
    const int m = b1 - b0;
    bucket_out *outs = calloc((size_t)(m + 1), sizeof(bucket_out));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int j = 0; j < m; ++j)
        run_bucket(&Hs, na, nb, dets, coeffs, core, nq, psi, ndets, b0 + j, nbuckets, R, E0, eps, keep_top, &outs[j]);
    int rc = ORACLE_OK;
    int64_t total = 0;
    nsum pt2 = {0.0, 0.0};
    for (int j = 0; j < m; ++j) {
        if (outs[j].rc != ORACLE_OK) rc = outs[j].rc;
        total += outs[j].r.count;
        st->candidates += outs[j].candidates;
        st->npairs += outs[j].npairs;
        nsum_add(&pt2, outs[j].pt2.e + outs[j].pt2.c);
        st->pt2_abs = st->pt2_abs + outs[j].pt2_abs;
        st->pt2_tol = st->pt2_tol + outs[j].pt2_tol;
        if (outs[j].max_drop_upper > st->max_drop_upper) st->max_drop_upper = outs[j].max_drop_upper;
    }
    st->pt2 = pt2.e + pt2.c;
    if (rc == ORACLE_OK) rc = result_alloc(res, total);
    if (rc == ORACLE_OK) {
        int64_t u = 0;
        for (int j = 0; j < m; ++j) {
            const oracle_result *r = &outs[j].r;
            const size_t c = (size_t)r->count;
            if (!c) continue;
            memcpy(res->keys + 2 * u, r->keys, 2 * c * sizeof(uint64_t));
            memcpy(res->num + u, r->num, c * sizeof(double));
            memcpy(res->hdiag + u, r->hdiag, c * sizeof(double));
            memcpy(res->score + u, r->score, c * sizeof(double));
            memcpy(res->num_abs + u, r->num_abs, c * sizeof(double));
            memcpy(res->hdiag_abs + u, r->hdiag_abs, c * sizeof(double));
            memcpy(res->tol + u, r->tol, c * sizeof(double));
            u += (int64_t)c;
        }
        res->count = u;
        res->npairs = st->npairs;
    }
    for (int j = 0; j < m; ++j) oracle_free(&outs[j].r);
    free(outs);
    free(core);
    free(psi);
    return rc;
}

/* ---- variational energy <C|H|C> by the plain double loop (Eq. (1), E_k) ---- */

double oracle_energy(const double *h, const double *eri, int n, double ecore,
                     const uint64_t *dets, const double *coeffs, int64_t ndets)
{
    double e = 0.0;
    for (int64_t i = 0; i < ndets; ++i)
        for (int64_t j = 0; j < ndets; ++j) {
            uint64_t da = dets[2 * i] ^ dets[2 * j], db = dets[2 * i + 1] ^ dets[2 * j + 1];
            if (popc(da) + popc(db) > 4)
                continue;
            e = e + coeffs[i] * oracle_helem(h, eri, n, ecore, dets[2 * i], dets[2 * i + 1],
                                             dets[2 * j], dets[2 * j + 1]) * coeffs[j];
        }
    return e;
}

/* ---- pair counts per constraint class (Sec. II.B: triplets and the
 * higher-order constraints that split heavy classes) ----
 * A target's class at level L is the set of the L highest occupied orbitals of
 * its alpha string (all of them when it has fewer than L).  For each core (in
 * the core set) every single and double is generated and counted against its
 * class: brute force, nothing is counted in closed form.  Classes are reported
 * by their mask; out_masks/out_counts receive the first `cap` non-empty classes
 * in ascending mask order.  Returns the number of non-empty classes. */

typedef struct { uint64_t mask; int64_t count; } cls_rec;

static int cmp_cls(const void *x, const void *y)
{
    const cls_rec *p = x, *q = y;
    return p->mask < q->mask ? -1 : (p->mask > q->mask);
}

/* the constraint of an alpha string: its `level` highest occupied orbitals
 * (all of them when it has fewer) */
static uint64_t top_bits(uint64_t a, int level)
{
    uint64_t m = 0;
    for (int t = 63, got = 0; t >= 0 && got < level; --t)
        if ((a >> t) & 1ull) { m |= 1ull << t; ++got; }
    return m;
}

int64_t oracle_class_counts(int n, int na, int nb, const uint64_t *dets, const double *coeffs,
                            int64_t ndets, int64_t ncore, int level, uint64_t *out_masks,
                            int64_t *out_counts, int64_t cap)
{
    if (validate(n, na, nb, dets, ndets) != ORACLE_OK || level < 1)
        return ORACLE_EINVAL;
    int64_t *core = malloc(sizeof(int64_t) * (size_t)(ndets + 1));
    int64_t nq = oracle_core_set(coeffs, ndets, ncore, core);
    int64_t per = oracle_sd_count(n, na, nb);
    uint64_t *tg = malloc(sizeof(uint64_t) * 2 * (size_t)(per + 1));
    cls_rec *all = malloc(sizeof(cls_rec) * (size_t)(per * nq + 1));
    int64_t m = 0;
    for (int64_t c = 0; c < nq; ++c) {
        int64_t i = core[c];
        int64_t nt = oracle_sd_targets(n, dets[2 * i], dets[2 * i + 1], tg);
        for (int64_t t = 0; t < nt; ++t) { all[m].mask = top_bits(tg[2 * t], level); all[m].count = 1; ++m; }
    }
    qsort(all, (size_t)m, sizeof(cls_rec), cmp_cls);
    int64_t nc = 0;
    for (int64_t j = 0; j < m;) {
        int64_t e = j;
        while (e < m && all[e].mask == all[j].mask) ++e;
        if (nc < cap) { out_masks[nc] = all[j].mask; out_counts[nc] = e - j; }
        ++nc;
        j = e;
    }
    free(all);
    free(tg);
    free(core);
    return nc;
}

/* ---- numerators of given targets, one at a time (for sampled checks) ----
 * N_a = sum over core determinants i (ascending input index) that differ from
 * a by a single or double excitation of H_ai C_i; also reports whether a is an
 * input determinant, the number of such cores, and (when the pointers are not
 * NULL) the magnitude sums num_abs and hdiag_abs of the tolerance.  A plain
 * scan over the cores: no enumeration of excitations and no sort. */
int oracle_target_numerators(const double *h, const double *eri, int n, int na, int nb, double ecore,
                             const uint64_t *dets, const double *coeffs, int64_t ndets, int64_t ncore,
                             const uint64_t *targets, int64_t ntargets, double *out_num,
                             double *out_hdiag, int *out_in_psi, int64_t *out_nconn, double *out_num_abs,
                             double *out_hdiag_abs)
{
    if (validate(n, na, nb, dets, ndets) != ORACLE_OK)
        return ORACLE_EINVAL;
    ham_t Hs = {n, h, eri, ecore};
    int64_t *core = malloc(sizeof(int64_t) * (size_t)(ndets + 1));
    int64_t nq = oracle_core_set(coeffs, ndets, ncore, core);
    for (int64_t t = 0; t < ntargets; ++t) {
        uint64_t ta = targets[2 * t], tb = targets[2 * t + 1];
        double s = 0.0, sa = 0.0;
        int64_t nc = 0;
        for (int64_t c = 0; c < nq; ++c) {
            int64_t i = core[c];
            int d = popc(ta ^ dets[2 * i]) + popc(tb ^ dets[2 * i + 1]);
            if (d == 0 || d > 4)
                continue;
            double ab = 0.0;
            s = s + helem_eval(&Hs, ta, tb, dets[2 * i], dets[2 * i + 1], &ab) * coeffs[i];
            sa = sa + ab * fabs(coeffs[i]);
            ++nc;
        }
        int in_psi = 0;
        for (int64_t i = 0; i < ndets; ++i)
            if (dets[2 * i] == ta && dets[2 * i + 1] == tb) { in_psi = 1; break; }
        double ha = 0.0;
        out_num[t] = s;
        out_hdiag[t] = hdiag_eval(&Hs, ta, tb, &ha);
        out_in_psi[t] = in_psi;
        out_nconn[t] = nc;
        if (out_num_abs) out_num_abs[t] = sa;
        if (out_hdiag_abs) out_hdiag_abs[t] = ha;
    }
    free(core);
    return ORACLE_OK;
}

/* ---- second-order (Epstein-Nesbet) energy of the candidates (Sec. II.A:
 * the PT2 correction is closely related to the scores of Eq. (1)) ----
 * E_PT2 = sum over candidates a (ascending key) of N_a^2 / (E0 - H_aa)
 *       = sum_a N_a * A_a, with N_a and A_a exactly as in oracle_search.
 * The terms are added with Neumaier's compensated summation, so the result
 * is the exact sum of the terms to within about 2u|E_PT2| (plus m u^2 S);
 * out_abs = S = sum_a |N_a * A_a| sizes the error of any other summation
 * order (Higham, Accuracy and Stability of Numerical Algorithms, ch. 4). */
int oracle_pt2(const double *h, const double *eri, int n, int na, int nb, double ecore,
               const uint64_t *dets, const double *coeffs, int64_t ndets, double E0, int64_t ncore,
               double eps, double *out_e, double *out_abs, int64_t *out_count)
{
    oracle_result r;
    int rc = oracle_search(h, eri, n, na, nb, ecore, dets, coeffs, ndets, E0, ncore, eps, 0, &r);
    if (rc != ORACLE_OK)
        return rc;
    double e = 0.0, comp = 0.0, sabs = 0.0;
    for (int64_t u = 0; u < r.count; ++u) {
        const double t = r.num[u] * r.score[u];
        const double y = e + t;
        if (fabs(e) >= fabs(t))
            comp = comp + ((e - y) + t);
        else
            comp = comp + ((t - y) + e);
        e = y;
        sabs = sabs + fabs(t);
    }
    *out_e = e + comp;
    *out_abs = sabs;
    *out_count = r.count;
    oracle_free(&r);
    return ORACLE_OK;
}

/* ---- static load balance over processing elements (Alg. 3) ----
 * The classes are visited in the order given.  A class that yields pairs
 * (h > 0) is assigned to the element with the smallest accumulated work,
 * the first such element when several tie, and that element's work grows by h.
 * (The printed algorithm never adds h to W; the reading taken here adds it,
 * otherwise every class would land on element 0.)  Classes without pairs are
 * not assigned (owner -1).  A plain linear arg-min scan over the elements. */
int oracle_balance(const int64_t *counts, int64_t nclasses, int npe, int *owner, int64_t *work)
{
    if (npe < 1 || nclasses < 0)
        return ORACLE_EINVAL;
    for (int p = 0; p < npe; ++p)
        work[p] = 0;
    for (int64_t c = 0; c < nclasses; ++c) {
        const int64_t h = counts[c];
        if (h < 0)
            return ORACLE_EINVAL;
        if (h == 0) {
            owner[c] = -1;
            continue;
        }
        int q = 0;
        for (int p = 1; p < npe; ++p)
            if (work[p] < work[q])
                q = p;
        owner[c] = q;
        work[q] += h;
    }
    return ORACLE_OK;
}

/* ---- Hamiltonian over a determinant set by the double loop (Sec. II.C) ----
 * out (nd x nd, row-major) gets <D_i|H|D_j> for every pair that differs by at
 * most a double excitation and 0 elsewhere; H_ii includes ecore.  out_abs
 * (optional, same shape) gets the sum of |terms| of each element. */
int oracle_hmat_dense(const double *h, const double *eri, int n, double ecore, const uint64_t *dets, int64_t nd,
                      double *out, double *out_abs)
{
    ham_t Hs = {n, h, eri, ecore};
    for (int64_t i = 0; i < nd; ++i)
        for (int64_t j = 0; j < nd; ++j) {
            uint64_t da = dets[2 * i] ^ dets[2 * j], db = dets[2 * i + 1] ^ dets[2 * j + 1];
            double ab = 0.0;
            out[i * nd + j] = (popc(da) + popc(db) > 4)
                                  ? 0.0
                                  : helem_eval(&Hs, dets[2 * i], dets[2 * i + 1], dets[2 * j], dets[2 * j + 1], &ab);
            if (out_abs) out_abs[i * nd + j] = ab;
        }
    return ORACLE_OK;
}
