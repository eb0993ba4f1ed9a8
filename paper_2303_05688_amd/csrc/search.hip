// The ASCI determinant search on gfx950 (Alg. 2 with the constraint-class
// partition of Sec. II.B).
//
// Pipeline, per batch of consecutive triplet classes:
//   count   : exact pair count of every (class, core) in closed form
//   scan    : record offsets, (class, core, excitation) order
//   generate: one wavefront per (class, core); each lane unranks its record
//             index into an excitation, evaluates H_ai and writes
//             (key, H_ai * C_i) at its offset
//   sort    : stable LSD radix sort on the key (equal keys keep ascending core
//             order, the summation order)
//   reduce  : one thread per run of equal keys sums in record order, drops
//             input determinants, forms H_aa and A_a = N_a / (E0 - H_aa)
//   append  : surviving candidates join a pool kept in ascending key order
// then radix selection of the k largest |A_a| (ties: smaller key) and a final
// stable sort of the k winners on |A_a|.
#include "hamiltonian.h"

#include <algorithm>
#include <cstring>
#include <functional>

namespace asci {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- class items
// Counts of one (class T, core alpha string a) item.  A target is in class T
// when its alpha string has exactly T's bits at or above T's lowest bit o.
// With hi = bits >= o and lo = bits < o: the electrons R = (a & hi) \ T must
// leave, the orbitals A = T \ (a & hi) must fill, and m = 0, 1, 2 alpha
// electrons move in total (m >= |R|, |A|); the remaining m - |R| holes and
// m - |A| particles come from the low part.  The beta string then does a single
// or double (m = 0), nothing or a single (m = 1), or nothing (m = 2).
struct ClassItem {
    uint64_t R, A, lo_occ, lo_vir;
    int nr, nA, no, nv;
    uint32_t cnt[3];
    uint32_t total;
};

struct BetaFactors {
    uint32_t f[3];  // beta completions per alpha move count m
    uint32_t nb, vb, pairs_vb;
};

__device__ __forceinline__ ClassItem class_item(uint64_t a, uint64_t T, uint64_t full, const BetaFactors &bf)
{
    ClassItem it;
    uint64_t lowmask = T ? ((1ull << lowbit(T)) - 1ull) : 0ull;
    uint64_t hi = full & ~lowmask;
    it.R = (a & hi) & ~T;
    it.A = T & ~(a & hi);
    it.lo_occ = a & lowmask;
    it.lo_vir = ~a & lowmask;
    it.nr = popc64(it.R);
    it.nA = popc64(it.A);
    it.no = popc64(it.lo_occ);
    it.nv = popc64(it.lo_vir);
    it.total = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        uint32_t c = 0;
        if (it.nr <= m && it.nA <= m)
            c = (uint32_t)(choose_small(it.no, m - it.nr) * choose_small(it.nv, m - it.nA)) * bf.f[m];
        it.cnt[m] = c;
        it.total += c;
    }
    return it;
}

// totals per class (no matrix), or the (class, core) count matrix of classes
// [c0, c0 + gridDim.y) when `counts` is non-null
__global__ __launch_bounds__(kBlock) void k_count(const uint64_t *__restrict__ core_a, uint32_t nq,
                                                  const uint64_t *__restrict__ cls, uint32_t c0,
                                                  uint64_t full, BetaFactors bf,
                                                  uint32_t *__restrict__ counts,
                                                  unsigned long long *__restrict__ cls_total)
{
    __shared__ unsigned long long s_sum[kBlock / 64];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t c = c0 + blockIdx.y;
    uint32_t cnt = 0;
    if (i < nq) {
        cnt = class_item(core_a[i], cls[c], full, bf).total;
        if (counts) counts[(size_t)blockIdx.y * nq + i] = cnt;
    }
    if (cls_total) {
        unsigned long long v = cnt;
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
        if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < kBlock / 64; ++w) t += s_sum[w];
            if (t) atomicAdd(&cls_total[c], t);
        }
    }
}

template <int W>
__device__ __forceinline__ void put_key(uint64_t *klo, uint64_t *khi, size_t j, uint64_t a, uint64_t b, int n)
{
    if (W == 1) {
        klo[j] = (a << n) | b;
    } else {
        klo[j] = b;
        khi[j] = a;
    }
}

// one wavefront per (class, core) entry of the batch
template <int W>
__global__ __launch_bounds__(kBlock) void k_generate(
    const uint64_t *__restrict__ core_a, const uint64_t *__restrict__ core_b,
    const double *__restrict__ core_c, uint32_t nq, const uint64_t *__restrict__ cls, uint32_t c0,
    uint32_t nentries, const uint32_t *__restrict__ counts, const uint32_t *__restrict__ offsets,
    const double *__restrict__ h, const double *__restrict__ eri, int n, uint64_t full, BetaFactors bf,
    uint64_t *__restrict__ klo, uint64_t *__restrict__ khi, double *__restrict__ vals, size_t cap,
    unsigned long long *__restrict__ key_or_and)
{
    const uint32_t e = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (e >= nentries) return;
    const uint32_t cnt = counts[e];
    if (cnt == 0) return;
    const uint32_t i = e % nq;
    const uint32_t c = c0 + e / nq;
    const uint64_t a = core_a[i], b = core_b[i];
    const double ci = core_c[i];
    const ClassItem it = class_item(a, cls[c], full, bf);
    const uint32_t off = offsets[e];
    const uint64_t bvir = ~b & full;
    const uint32_t nbvb = bf.nb * bf.vb;

    uint64_t kor0 = 0, kand0 = ~0ull, kor1 = 0, kand1 = ~0ull;
    for (uint32_t j0 = lane; j0 < cnt; j0 += 64) {
        uint32_t j = j0;
        int m;
        if (j < it.cnt[0]) {
            m = 0;
        } else {
            j -= it.cnt[0];
            if (j < it.cnt[1]) {
                m = 1;
            } else {
                j -= it.cnt[1];
                m = 2;
            }
        }
        const uint32_t fm = m == 0 ? bf.f[0] : (m == 1 ? bf.f[1] : bf.f[2]);
        const uint32_t ac = j / fm, bc = j - ac * fm;
        const int kh = m - it.nr, kp = m - it.nA;
        const uint32_t npart = (uint32_t)choose_small(it.nv, kp);
        const uint32_t hidx = ac / npart, pidx = ac - hidx * npart;
        const uint64_t holes = it.R | pick_bits(it.lo_occ, kh, hidx);
        const uint64_t parts = it.A | pick_bits(it.lo_vir, kp, pidx);
        const uint64_t a2 = (a & ~holes) | parts;
        uint64_t b2 = b;
        double hv;
        if (m == 0) {
            if (bc < nbvb) {
                const uint32_t hh = bc / bf.vb, pp = bc - hh * bf.vb;
                const int r = select_bit(b, (int)hh), s = select_bit(bvir, (int)pp);
                b2 = (b & ~(1ull << r)) | (1ull << s);
                hv = single_value(h, eri, n, b, a, r, s);
            } else {
                const uint32_t x = bc - nbvb;
                const uint32_t hh = x / bf.pairs_vb, pp = x - hh * bf.pairs_vb;
                const uint64_t hb = pick_bits(b, 2, hh), pb = pick_bits(bvir, 2, pp);
                b2 = (b & ~hb) | pb;
                hv = double_same_value(eri, n, b, hb, pb);
            }
        } else if (m == 1) {
            const int p = lowbit(holes), q = lowbit(parts);
            if (bc == 0) {
                hv = single_value(h, eri, n, a, b, p, q);
            } else {
                const uint32_t x = bc - 1;
                const uint32_t hh = x / bf.vb, pp = x - hh * bf.vb;
                const int r = select_bit(b, (int)hh), s = select_bit(bvir, (int)pp);
                b2 = (b & ~(1ull << r)) | (1ull << s);
                hv = double_opp_value(eri, n, a, b, p, q, r, s);
            }
        } else {
            hv = double_same_value(eri, n, a, holes, parts);
        }
        const size_t dst = (size_t)off + j0;
        if (dst < cap) {
            put_key<W>(klo, khi, dst, a2, b2, n);
            vals[dst] = hv * ci;
        }
        if (W == 1) {
            const uint64_t k = (a2 << n) | b2;
            kor0 |= k;
            kand0 &= k;
        } else {
            kor0 |= b2;
            kand0 &= b2;
            kor1 |= a2;
            kand1 &= a2;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        kor0 |= __shfl_xor(kor0, d, 64);
        kand0 &= __shfl_xor(kand0, d, 64);
        kor1 |= __shfl_xor(kor1, d, 64);
        kand1 &= __shfl_xor(kand1, d, 64);
    }
    if (lane == 0) {
        atomicOr(&key_or_and[0], (unsigned long long)kor0);
        atomicAnd(&key_or_and[1], (unsigned long long)kand0);
        if (W == 2) {
            atomicOr(&key_or_and[2], (unsigned long long)kor1);
            atomicAnd(&key_or_and[3], (unsigned long long)kand1);
        }
    }
}

__global__ void k_init_or_and(unsigned long long *p)
{
    if (threadIdx.x < 4) p[threadIdx.x] = (threadIdx.x & 1) ? ~0ull : 0ull;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_head_flags(const uint64_t *__restrict__ klo,
                                                       const uint64_t *__restrict__ khi, size_t n,
                                                       uint32_t *__restrict__ flag)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    bool head = j == 0 || klo[j] != klo[j - 1];
    if (W == 2 && j > 0) head = head || khi[j] != khi[j - 1];
    flag[j] = head ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_head_scatter(const uint32_t *__restrict__ flag,
                                                         const uint32_t *__restrict__ pos, size_t n,
                                                         uint32_t *__restrict__ heads,
                                                         const uint32_t *__restrict__ d_count)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n && flag[j] && pos[j] < n) heads[pos[j]] = (uint32_t)j;
    if (j == 0) heads[min((size_t)*d_count, n)] = (uint32_t)n;
}

// binary search of (a, b) in the sorted input keys
template <int W>
__device__ __forceinline__ bool in_psi(const uint64_t *__restrict__ plo, const uint64_t *__restrict__ phi,
                                       uint32_t npsi, uint64_t lo, uint64_t hi)
{
    uint32_t L = 0, R = npsi;
    while (L < R) {
        const uint32_t mid = (L + R) >> 1;
        const uint64_t ml = plo[mid];
        bool less;
        if (W == 1) {
            less = ml < lo;
        } else {
            const uint64_t mh = phi[mid];
            less = mh < hi || (mh == hi && ml < lo);
        }
        if (less) L = mid + 1;
        else R = mid;
    }
    if (L >= npsi) return false;
    return plo[L] == lo && (W == 1 || phi[L] == hi);
}

// one thread per run of equal keys (grid-stride); J/K/h-diagonal in LDS
template <int W>
__global__ __launch_bounds__(kBlock) void k_reduce_score(
    const uint64_t *__restrict__ klo, const uint64_t *__restrict__ khi, const double *__restrict__ vals,
    const uint32_t *__restrict__ heads, const uint32_t *__restrict__ d_nuniq, uint32_t nrec,
    const uint64_t *__restrict__ plo, const uint64_t *__restrict__ phi, uint32_t npsi,
    const double *__restrict__ jk, const double *__restrict__ h, int n, double ecore, double E0,
    uint64_t *__restrict__ clo, uint64_t *__restrict__ chi, double *__restrict__ cnum,
    double *__restrict__ cscore, uint32_t *__restrict__ keep)
{
    extern __shared__ double s_tab[];
    double *J = s_tab, *K = s_tab + n * n, *hd = s_tab + 2 * n * n;
    for (int t = threadIdx.x; t < 2 * n * n; t += kBlock) s_tab[t] = jk[t];
    for (int t = threadIdx.x; t < n; t += kBlock) hd[t] = h[(size_t)t * n + t];
    __syncthreads();
    const uint32_t nu = *d_nuniq;
    const uint64_t nmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    for (uint32_t u = blockIdx.x * kBlock + threadIdx.x; u < nu; u += gridDim.x * kBlock) {
        const uint32_t j0 = heads[u], j1 = min(heads[u + 1], nrec);
        double s = 0.0;
        for (uint32_t j = j0; j < j1; ++j) s = s + vals[j];
        const uint64_t lo = klo[j0];
        const uint64_t hi = (W == 2) ? khi[j0] : 0ull;
        const uint64_t a = (W == 1) ? (lo >> n) : hi;
        const uint64_t b = (W == 1) ? (lo & nmask) : lo;
        const bool ex = in_psi<W>(plo, phi, npsi, lo, hi);
        const double hdv = diag_value(J, K, hd, n, ecore, a, b);
        clo[u] = lo;
        if (W == 2) chi[u] = hi;
        cnum[u] = s;
        cscore[u] = s / (E0 - hdv);
        keep[u] = ex ? 0u : 1u;
    }
}

// append kept candidates to the pool (stable)
template <int W>
__global__ __launch_bounds__(kBlock) void k_append(const uint64_t *__restrict__ clo,
                                                   const uint64_t *__restrict__ chi,
                                                   const double *__restrict__ cnum,
                                                   const double *__restrict__ cscore,
                                                   const uint32_t *__restrict__ keep,
                                                   const uint32_t *__restrict__ pos,
                                                   const uint32_t *__restrict__ d_n, uint64_t *__restrict__ plo,
                                                   uint64_t *__restrict__ phi, double *__restrict__ pnum,
                                                   double *__restrict__ pscore, size_t base, size_t cap)
{
    const uint32_t n = *d_n;
    for (uint32_t u = blockIdx.x * kBlock + threadIdx.x; u < n; u += gridDim.x * kBlock) {
        if (!keep[u]) continue;
        const size_t d = base + pos[u];
        if (d >= cap) continue;
        plo[d] = clo[u];
        if (W == 2) phi[d] = chi[u];
        if (pnum) pnum[d] = cnum[u];
        pscore[d] = cscore[u];
    }
}

// ---------------------------------------------------------------- selection helpers
__global__ __launch_bounds__(kBlock) void k_flag_equal(const double *__restrict__ score, size_t n,
                                                       const SelectState *__restrict__ st,
                                                       uint32_t *__restrict__ flag)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n) flag[j] = abs_order(score[j]) == st->prefix ? 1u : 0u;
}

// keep[j] = ord > t, or ord == t among the first krem such entries
__global__ __launch_bounds__(kBlock) void k_flag_keep(const double *__restrict__ score, size_t n,
                                                      const SelectState *__restrict__ st,
                                                      const uint32_t *__restrict__ eq_rank,
                                                      uint32_t *__restrict__ flag)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint64_t o = abs_order(score[j]), t = st->prefix;
    flag[j] = (o > t || (o == t && eq_rank[j] < st->krem)) ? 1u : 0u;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_compact(const uint64_t *__restrict__ ilo,
                                                    const uint64_t *__restrict__ ihi,
                                                    const double *__restrict__ inum,
                                                    const double *__restrict__ iscore, size_t n,
                                                    const uint32_t *__restrict__ flag,
                                                    const uint32_t *__restrict__ pos, uint64_t *__restrict__ olo,
                                                    uint64_t *__restrict__ ohi, double *__restrict__ onum,
                                                    double *__restrict__ oscore)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n || !flag[j]) return;
    const uint32_t d = pos[j];
    if (d >= n) return;
    olo[d] = ilo[j];
    if (W == 2) ohi[d] = ihi[j];
    if (onum) onum[d] = inum[j];
    oscore[d] = iscore[j];
}

// sort key for the final order: ~|score| bits so that ascending = descending |score|
__global__ __launch_bounds__(kBlock) void k_final_keys(const double *__restrict__ score, size_t n,
                                                       uint64_t *__restrict__ key, uint32_t *__restrict__ idx)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    key[j] = ~abs_order(score[j]);
    idx[j] = (uint32_t)j;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_final_gather(const uint32_t *__restrict__ idx, size_t n,
                                                         const uint64_t *__restrict__ slo,
                                                         const uint64_t *__restrict__ shi,
                                                         const double *__restrict__ sscore, int norb,
                                                         uint64_t *__restrict__ out_dets,
                                                         double *__restrict__ out_scores)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = idx[j];
    const uint64_t lo = slo[i];
    const uint64_t nmask = (norb == 64) ? ~0ull : ((1ull << norb) - 1ull);
    out_dets[2 * j] = (W == 1) ? (lo >> norb) : shi[i];
    out_dets[2 * j + 1] = (W == 1) ? (lo & nmask) : lo;
    out_scores[j] = sscore[i];
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_unpack(const uint64_t *__restrict__ klo,
                                                   const uint64_t *__restrict__ khi, size_t n, int norb,
                                                   uint64_t *__restrict__ out_dets)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint64_t lo = klo[j];
    const uint64_t nmask = (norb == 64) ? ~0ull : ((1ull << norb) - 1ull);
    out_dets[2 * j] = (W == 1) ? (lo >> norb) : khi[j];
    out_dets[2 * j + 1] = (W == 1) ? (lo & nmask) : lo;
}

// ---------------------------------------------------------------- input preparation
// validation flags: bit 0 = wrong electron count or orbital out of range
__global__ __launch_bounds__(kBlock) void k_validate(const uint64_t *__restrict__ dets, size_t nd,
                                                     uint64_t full, int na, int nb,
                                                     unsigned int *__restrict__ err)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd) return;
    const uint64_t a = dets[2 * j], b = dets[2 * j + 1];
    if ((a & ~full) || (b & ~full) || popc64(a) != na || popc64(b) != nb) atomicOr(err, 1u);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_pack_keys(const uint64_t *__restrict__ dets, size_t nd, int n,
                                                      uint64_t *__restrict__ klo, uint64_t *__restrict__ khi,
                                                      uint32_t *__restrict__ idx)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd) return;
    put_key<W>(klo, khi, j, dets[2 * j], dets[2 * j + 1], n);
    idx[j] = (uint32_t)j;
}

// bit 1 of err: two equal input determinants (keys sorted)
template <int W>
__global__ __launch_bounds__(kBlock) void k_check_dups(const uint64_t *__restrict__ klo,
                                                       const uint64_t *__restrict__ khi, size_t n,
                                                       unsigned int *__restrict__ err)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j == 0 || j >= n) return;
    if (klo[j] == klo[j - 1] && (W == 1 || khi[j] == khi[j - 1])) atomicOr(err, 2u);
}

// core-selection sort key: ~|C| bits, so ascending order is |C| descending
__global__ __launch_bounds__(kBlock) void k_core_keys(const double *__restrict__ c, size_t nd,
                                                      uint64_t *__restrict__ key, uint32_t *__restrict__ idx)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd) return;
    key[j] = ~abs_order(c[j]);
    idx[j] = (uint32_t)j;
}

__global__ __launch_bounds__(kBlock) void k_index_keys(const uint32_t *__restrict__ idx, size_t n,
                                                       uint64_t *__restrict__ key)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n) key[j] = idx[j];
}

__global__ __launch_bounds__(kBlock) void k_gather_core(const uint64_t *__restrict__ dets,
                                                        const double *__restrict__ c,
                                                        const uint64_t *__restrict__ sel, size_t nq,
                                                        uint64_t *__restrict__ qa, uint64_t *__restrict__ qb,
                                                        double *__restrict__ qc)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nq) return;
    const size_t i = sel ? (size_t)sel[j] : j;
    qa[j] = dets[2 * i];
    qb[j] = dets[2 * i + 1];
    qc[j] = c[i];
}

__global__ __launch_bounds__(kBlock) void k_jk(const double *__restrict__ eri, int n, double *__restrict__ jk)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    jk[t] = eri4(eri, n, p, p, q, q);
    jk[n * n + t] = eri4(eri, n, p, q, q, p);
}

inline unsigned grid_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

inline uint64_t choose_u64(uint64_t x, int k)
{
    if (k < 0 || (uint64_t)k > x) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (x - k + i) / i;
    return r;
}

// the constraint classes in ascending mask order: the sets of the three
// highest occupied alpha orbitals that a string with na electrons can have
// (all na orbitals when na < 3)
std::vector<uint64_t> make_classes(int n, int na)
{
    std::vector<uint64_t> out;
    const int L = na < 3 ? na : 3;
    if (L == 0) {
        out.push_back(0ull);
        return out;
    }
    std::vector<int> c(L);
    // all L-subsets o_1 > ... > o_L with o_L >= na - L
    std::function<void(int, int, uint64_t)> rec;
    for (int i = 0; i < L; ++i) c[i] = 0;
    rec = [&](int depth, int below, uint64_t mask) {
        if (depth == L) {
            out.push_back(mask);
            return;
        }
        // choose the next (lower) orbital strictly below `below`
        const int minimum = (depth == L - 1) ? (na - L) : (L - 1 - depth);
        for (int o = below - 1; o >= minimum; --o) rec(depth + 1, o, mask | (1ull << o));
    };
    rec(0, n, 0ull);
    std::sort(out.begin(), out.end());
    return out;
}

}  // namespace

// ---------------------------------------------------------------- host driver
static BetaFactors beta_factors(int n, int nb)
{
    BetaFactors bf;
    const uint32_t vb = (uint32_t)(n - nb);
    const uint32_t pnb = (uint32_t)nb * (nb - 1) / 2, pvb = vb * (vb - 1) / 2;
    bf.f[0] = (uint32_t)nb * vb + pnb * pvb;
    bf.f[1] = 1u + (uint32_t)nb * vb;
    bf.f[2] = 1u;
    bf.nb = (uint32_t)nb;
    bf.vb = vb;
    bf.pairs_vb = pvb;
    return bf;
}

// inputs shared by the search entry points: validated, keyed and core-selected
template <int W>
struct Prepared {
    size_t nd = 0, nq = 0;
    const uint64_t *plo = nullptr, *phi = nullptr;  // sorted keys of every input determinant
    uint64_t *q_a = nullptr, *q_b = nullptr;         // core set, ascending input index
    double *q_c = nullptr;
    uint64_t *d_cls = nullptr;
    double *d_jk = nullptr;
    std::vector<uint64_t> cls, totals;
};

static std::vector<Digit> full_key_digits(int n, int W)
{
    std::vector<Digit> d;
    if (W == 1) {
        for (int sh = 0; sh < 2 * n; sh += 8) d.push_back({0, sh});
    } else {
        for (int sh = 0; sh < n; sh += 8) d.push_back({0, sh});
        for (int sh = 0; sh < n; sh += 8) d.push_back({1, sh});
    }
    return d;
}

// Validate the determinants, sort their keys, pick the core set and count the
// pairs of every constraint class.  All buffers live in ctx->setup.
template <int W>
static void prepare(asci_ctx *ctx, const double *d_eri, int n, int na, int nb, const uint64_t *dets,
                    const double *coeffs, int64_t ndets, int64_t ncore, bool need_psi, Prepared<W> &pp,
                    hipStream_t s)
{
    const size_t nd = (size_t)ndets;
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const BetaFactors bf = beta_factors(n, nb);
    pp.nd = nd;
    pp.nq = (ncore > 0 && (size_t)ncore < nd) ? (size_t)ncore : nd;
    const size_t nq = pp.nq;
    pp.cls = make_classes(n, na);
    const uint32_t ncls = (uint32_t)pp.cls.size();
    require(ncls <= 65535, ASCI_EINVAL, "too many constraint classes");

    Arena &ar = ctx->setup;
    const size_t hist_bytes = ((nd + kScanTile - 1) / kScanTile) * 256 * 4 * 2 + (1 << 16);
    ar.reset();
    ar.reserve(nd * (8 * 2 * W + 4 * 2) + nd * (8 * 2 + 4 * 2) + nq * 8 * 4 + (size_t)ncls * 16 +
               (size_t)2 * n * n * 8 + 2 * hist_bytes + 64 * 256);
    ar.reset();
    unsigned int *d_err = ar.take<unsigned int>(16);
    pp.d_cls = ar.take<uint64_t>(ncls);
    unsigned long long *d_tot = ar.take<unsigned long long>(ncls);
    pp.d_jk = ar.take<double>((size_t)2 * n * n);
    uint64_t *psi_lo[2] = {ar.take<uint64_t>(nd), ar.take<uint64_t>(nd)};
    uint64_t *psi_hi[2] = {W == 2 ? ar.take<uint64_t>(nd) : nullptr, W == 2 ? ar.take<uint64_t>(nd) : nullptr};
    uint32_t *psi_idx[2] = {ar.take<uint32_t>(nd), ar.take<uint32_t>(nd)};
    pp.q_a = ar.take<uint64_t>(nq);
    pp.q_b = ar.take<uint64_t>(nq);
    pp.q_c = ar.take<double>(nq);

    ASCI_HIP(hipMemsetAsync(d_err, 0, 16 * sizeof(unsigned int), s));
    ASCI_HIP(hipMemsetAsync(d_tot, 0, ncls * sizeof(unsigned long long), s));
    ASCI_HIP(hipMemcpyAsync(pp.d_cls, pp.cls.data(), ncls * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    k_validate<<<grid_for(nd), kBlock, 0, s>>>(dets, nd, full, na, nb, d_err);
    ASCI_LAUNCH_CHECK();
    if (d_eri) {
        k_jk<<<grid_for((size_t)n * n), kBlock, 0, s>>>(d_eri, n, pp.d_jk);
        ASCI_LAUNCH_CHECK();
    }
    if (need_psi) {
        k_pack_keys<W><<<grid_for(nd), kBlock, 0, s>>>(dets, nd, n, psi_lo[0], psi_hi[0], psi_idx[0]);
        ASCI_LAUNCH_CHECK();
        const int pc = radix_sort<uint32_t>(psi_lo, psi_hi, psi_idx, nd, W, full_key_digits(n, W), ar, s);
        pp.plo = psi_lo[pc];
        pp.phi = psi_hi[pc];
        k_check_dups<W><<<grid_for(nd), kBlock, 0, s>>>(psi_lo[pc], psi_hi[pc], nd, d_err);
        ASCI_LAUNCH_CHECK();
    }
    // core set: the nq inputs of largest |C| (ties: lower index), ascending index
    if (nq < nd) {
        uint64_t *ck[2] = {ar.take<uint64_t>(nd), ar.take<uint64_t>(nd)};
        uint32_t *ci[2] = {ar.take<uint32_t>(nd), ar.take<uint32_t>(nd)};
        uint64_t *nohi[2] = {nullptr, nullptr};
        k_core_keys<<<grid_for(nd), kBlock, 0, s>>>(coeffs, nd, ck[0], ci[0]);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> cd;
        for (int sh = 0; sh < 64; sh += 8) cd.push_back({0, sh});
        const int r1 = radix_sort<uint32_t>(ck, nohi, ci, nd, 1, cd, ar, s);
        // first nq indices as keys, sorted ascending (payload unused)
        uint64_t *ik[2] = {ck[r1 ^ 1], ar.take<uint64_t>(nq)};
        uint32_t *ii[2] = {ci[r1 ^ 1], ar.take<uint32_t>(nq)};
        k_index_keys<<<grid_for(nq), kBlock, 0, s>>>(ci[r1], nq, ik[0]);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> id;
        for (int sh = 0; sh < 32; sh += 8) id.push_back({0, sh});
        const int r2 = radix_sort<uint32_t>(ik, nohi, ii, nq, 1, id, ar, s);
        k_gather_core<<<grid_for(nq), kBlock, 0, s>>>(dets, coeffs, ik[r2], nq, pp.q_a, pp.q_b, pp.q_c);
    } else {
        k_gather_core<<<grid_for(nq), kBlock, 0, s>>>(dets, coeffs, nullptr, nq, pp.q_a, pp.q_b, pp.q_c);
    }
    ASCI_LAUNCH_CHECK();
    // step 4, totals per class
    {
        dim3 g((unsigned)((nq + kBlock - 1) / kBlock), ncls);
        k_count<<<g, kBlock, 0, s>>>(pp.q_a, (uint32_t)nq, pp.d_cls, 0, full, bf, nullptr, d_tot);
        ASCI_LAUNCH_CHECK();
    }
    HostStage &hs = ctx->stage;
    hs.reserve(256 + ncls * sizeof(uint64_t));
    unsigned int *h_err = (unsigned int *)hs.ptr;
    uint64_t *h_tot = (uint64_t *)((char *)hs.ptr + 256);
    ASCI_HIP(hipMemcpyAsync(h_err, d_err, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipMemcpyAsync(h_tot, d_tot, ncls * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    if (h_err[0] & 1u) throw Error{ASCI_EINVAL, "input determinant with wrong electron count or orbital >= norb"};
    if (h_err[0] & 2u) throw Error{ASCI_EINVAL, "duplicate input determinants"};
    pp.totals.assign(h_tot, h_tot + ncls);
}

template <int W>
static void run_search(asci_ctx *ctx, const SearchArgs &in, SearchOut &out, hipStream_t s)
{
    const int n = in.n;
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const BetaFactors bf = beta_factors(n, in.nb);
    const bool topk = out.k > 0;
    require(!(in.opt.eps > 0.0), ASCI_EINVAL, "eps > 0 is not supported by this build");

    Profiler *prof = &ctx->prof;
    Prepared<W> pp;
    prepare<W>(ctx, in.eri, n, in.na, in.nb, in.dets, in.coeffs, in.ndets, in.opt.ncore, true, pp, s);
    const size_t nd = pp.nd, nq = pp.nq;
    const uint32_t ncls = (uint32_t)pp.cls.size();

    // ---- batch plan: consecutive classes up to the pair-buffer capacity
    const size_t rec_bytes = 2 * (8 * W + 8);  // ping-pong keys + values
    uint64_t cap;
    if (in.opt.pair_buffer_bytes > 0) {
        cap = (uint64_t)in.opt.pair_buffer_bytes / rec_bytes;
    } else {
        size_t fr = 0, tt = 0;
        ASCI_HIP(hipMemGetInfo(&fr, &tt));
        fr += ctx->main.capacity();
        cap = std::min<uint64_t>((uint64_t)1 << 30, (uint64_t)(fr / 2) / (rec_bytes + 3 * 4 + 8 * W + 20));
    }
    cap = std::max<uint64_t>(cap, 1);
    std::vector<std::pair<uint32_t, uint32_t>> batches;
    uint64_t max_batch = 0, max_entries = 0, total = 0;
    for (uint32_t c = 0; c < ncls;) {
        uint64_t sum = 0;
        uint32_t c1 = c;
        while (c1 < ncls && (c1 == c || sum + pp.totals[c1] <= cap)) sum += pp.totals[c1++];
        require(sum < (1ull << 31), ASCI_ENOMEM, "one constraint class exceeds 2^31 pairs");
        batches.push_back({c, c1});
        max_batch = std::max(max_batch, sum);
        max_entries = std::max<uint64_t>(max_entries, (uint64_t)(c1 - c) * nq);
        total += sum;
        c = c1;
    }
    require(max_entries < (1ull << 31), ASCI_ENOMEM, "batch (class x core) matrix too large");

    // ---- main workspace
    const size_t Pb = std::max<uint64_t>(max_batch, 1);
    const size_t E = std::max<uint64_t>(max_entries, 1);
    size_t pool_cap;
    if (topk) pool_cap = (size_t)std::min<uint64_t>(total + 1, std::max<uint64_t>(4 * (uint64_t)out.k, Pb) + (uint64_t)out.k);
    else pool_cap = total + 1;
    require(pool_cap < (1ull << 32), ASCI_ENOMEM, "candidate pool too large");
    const size_t nbp = (Pb + kScanTile - 1) / kScanTile;
    const size_t scan_tmp = ((std::max<size_t>(Pb, std::max<size_t>(E, nbp * 256)) + kScanTile - 1) / kScanTile) * 4 + 4096;
    const size_t kk_max = topk ? (size_t)std::min<uint64_t>((uint64_t)out.k, pool_cap) : 0;
    Arena &ar = ctx->main;
    ar.reset();
    ar.reserve(E * 8 + Pb * rec_bytes + 3 * (Pb + 1) * 4 + nbp * 256 * 4 + scan_tmp +
               Pb * (8 * W + 16) + pool_cap * ((8 * W + 8) * 2 + (topk ? 0 : 8) + 12) +
               kk_max * 24 + 64 * 256 + (1 << 16));
    ar.reset();
    uint32_t *counts = ar.take<uint32_t>(E);
    uint32_t *offs = ar.take<uint32_t>(E);
    uint64_t *k_lo[2] = {ar.take<uint64_t>(Pb), ar.take<uint64_t>(Pb)};
    uint64_t *k_hi[2] = {W == 2 ? ar.take<uint64_t>(Pb) : nullptr, W == 2 ? ar.take<uint64_t>(Pb) : nullptr};
    double *v[2] = {ar.take<double>(Pb), ar.take<double>(Pb)};
    uint32_t *flag = ar.take<uint32_t>(Pb + 1);
    uint32_t *pos = ar.take<uint32_t>(Pb + 1);
    uint32_t *heads = ar.take<uint32_t>(Pb + 1);
    uint64_t *c_lo = ar.take<uint64_t>(Pb);
    uint64_t *c_hi = W == 2 ? ar.take<uint64_t>(Pb) : nullptr;
    double *c_num = ar.take<double>(Pb);
    double *c_score = ar.take<double>(Pb);
    uint64_t *p_lo[2] = {ar.take<uint64_t>(pool_cap), ar.take<uint64_t>(pool_cap)};
    uint64_t *p_hi[2] = {W == 2 ? ar.take<uint64_t>(pool_cap) : nullptr, W == 2 ? ar.take<uint64_t>(pool_cap) : nullptr};
    double *p_num = topk ? nullptr : ar.take<double>(pool_cap);
    double *p_score[2] = {ar.take<double>(pool_cap), ar.take<double>(pool_cap)};
    uint32_t *pflag = ar.take<uint32_t>(pool_cap);
    uint32_t *ppos = ar.take<uint32_t>(pool_cap);
    uint32_t *prank = ar.take<uint32_t>(pool_cap);
    SelectState *d_sel = ar.take<SelectState>(1);
    uint32_t *d_cnt = ar.take<uint32_t>(16);
    unsigned long long *d_misc = ar.take<unsigned long long>(16);
    const size_t loop_mark = ar.used();

    HostStage &hs = ctx->stage;
    hs.reserve(256);
    unsigned long long *h_misc = (unsigned long long *)hs.ptr;
    const size_t jk_lds = ((size_t)2 * n * n + n) * sizeof(double);
    int pcur = 0;
    size_t pool_n = 0;

    // keep the pool's keepk entries of largest |score|, in ascending key order
    auto prune = [&](size_t keepk) {
        radix_select_abs(p_score[pcur], pool_n, keepk, d_sel, s, prof);
        k_flag_equal<<<grid_for(pool_n), kBlock, 0, s>>>(p_score[pcur], pool_n, d_sel, pflag);
        ASCI_LAUNCH_CHECK();
        scan_u32(pflag, prank, pool_n, nullptr, ar, s);
        k_flag_keep<<<grid_for(pool_n), kBlock, 0, s>>>(p_score[pcur], pool_n, d_sel, prank, pflag);
        ASCI_LAUNCH_CHECK();
        scan_u32(pflag, ppos, pool_n, nullptr, ar, s);
        const int o = pcur ^ 1;
        k_compact<W><<<grid_for(pool_n), kBlock, 0, s>>>(p_lo[pcur], p_hi[pcur], nullptr, p_score[pcur], pool_n,
                                                         pflag, ppos, p_lo[o], p_hi[o], nullptr, p_score[o]);
        ASCI_LAUNCH_CHECK();
        pcur = o;
        pool_n = keepk;
        ar.reset();
        (void)ar.take<char>(loop_mark);
    };

    for (const auto &bt : batches) {
        const uint32_t c0 = bt.first, nc = bt.second - bt.first;
        uint64_t btotal = 0;
        for (uint32_t c = bt.first; c < bt.second; ++c) btotal += pp.totals[c];
        if (btotal == 0) continue;
        const size_t ent = (size_t)nc * nq;
        const size_t P = (size_t)btotal;
        ar.reset();
        (void)ar.take<char>(loop_mark);
        // step 4: count matrix of the batch and record offsets
        {
            ProfScope ps(prof, "count", 8.0 * nq + 4.0 * ent, s);
            dim3 g((unsigned)((nq + kBlock - 1) / kBlock), nc);
            k_count<<<g, kBlock, 0, s>>>(pp.q_a, (uint32_t)nq, pp.d_cls, c0, full, bf, counts, nullptr);
            ASCI_LAUNCH_CHECK();
        }
        scan_u32(counts, offs, ent, nullptr, ar, s, prof);
        // step 5: generate
        k_init_or_and<<<1, 64, 0, s>>>(d_misc);
        ASCI_LAUNCH_CHECK();
        const unsigned gblocks = (unsigned)((ent + (kBlock / 64) - 1) / (kBlock / 64));
        {
        ProfScope ps(prof, "generate", (8.0 * W + 8.0) * P, s);
        k_generate<W><<<gblocks, kBlock, 0, s>>>(pp.q_a, pp.q_b, pp.q_c, (uint32_t)nq, pp.d_cls, c0, (uint32_t)ent,
                                                 counts, offs, in.h, in.eri, n, full, bf, k_lo[0], k_hi[0], v[0], Pb,
                                                 d_misc);
        ASCI_LAUNCH_CHECK();
        }
        ASCI_HIP(hipMemcpyAsync(h_misc, d_misc, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        // step 6: sort on the digits that vary inside the batch
        std::vector<Digit> dig;
        if (W == 1) {
            const uint64_t var = h_misc[0] ^ h_misc[1];
            for (int sh = 0; sh < 2 * n; sh += 8)
                if ((var >> sh) & 0xFFull) dig.push_back({0, sh});
        } else {
            const uint64_t var0 = h_misc[0] ^ h_misc[1], var1 = h_misc[2] ^ h_misc[3];
            for (int sh = 0; sh < n; sh += 8)
                if ((var0 >> sh) & 0xFFull) dig.push_back({0, sh});
            for (int sh = 0; sh < n; sh += 8)
                if ((var1 >> sh) & 0xFFull) dig.push_back({1, sh});
        }
        const int r = radix_sort<double>(k_lo, k_hi, v, P, W, dig, ar, s, prof);
        // steps 7-9: runs of equal keys, sum, exclusion, H_aa, score
        {
            ProfScope ps(prof, "head_flags", (8.0 * W + 4.0) * P, s);
            k_head_flags<W><<<grid_for(P), kBlock, 0, s>>>(k_lo[r], k_hi[r], P, flag);
            ASCI_LAUNCH_CHECK();
        }
        scan_u32(flag, pos, P, d_cnt, ar, s, prof);
        ASCI_HIP(hipMemcpyAsync(h_misc, d_cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        const uint32_t U = *(uint32_t *)h_misc;
        {
            ProfScope ps(prof, "head_scatter", 8.0 * P + 4.0 * U, s);
            k_head_scatter<<<grid_for(P), kBlock, 0, s>>>(flag, pos, P, heads, d_cnt);
            ASCI_LAUNCH_CHECK();
        }
        {
            ProfScope ps(prof, "reduce_score", 8.0 * P + (8.0 * W + 8.0) * U + (8.0 * W + 20.0) * U, s);
            const unsigned rg = (unsigned)std::max<size_t>(1, std::min<size_t>(grid_for(U), 4096));
            k_reduce_score<W><<<rg, kBlock, jk_lds, s>>>(k_lo[r], k_hi[r], v[r], heads, d_cnt, (uint32_t)P, pp.plo,
                                                         pp.phi,
                                                         (uint32_t)nd, pp.d_jk, in.h, n, in.opt.ecore, in.E0, c_lo,
                                                         c_hi, c_num, c_score, flag);
            ASCI_LAUNCH_CHECK();
        }
        scan_u32(flag, pos, U, d_cnt + 1, ar, s, prof);
        ASCI_HIP(hipMemcpyAsync(h_misc, d_cnt + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        const uint32_t V = *(uint32_t *)h_misc;
        if (topk && pool_n + V > pool_cap) prune((size_t)std::min<uint64_t>(pool_n, (uint64_t)out.k));
        require(pool_n + V <= pool_cap, ASCI_ENOMEM, "candidate pool overflow");
        {
            ProfScope ps(prof, "append", (8.0 * W + 24.0) * U + (8.0 * W + 8.0) * V, s);
            k_append<W><<<1024, kBlock, 0, s>>>(c_lo, c_hi, c_num, c_score, flag, pos, d_cnt, p_lo[pcur],
                                                p_hi[pcur], p_num, p_score[pcur], pool_n, pool_cap);
            ASCI_LAUNCH_CHECK();
        }
        pool_n += V;
    }

    ar.reset();
    (void)ar.take<char>(loop_mark);
    if (!topk) {
        out.count = (int64_t)pool_n;
        if (pool_n > (size_t)out.capacity) return;  // the caller reports ENOMEM
        if (pool_n) {
            k_unpack<W><<<grid_for(pool_n), kBlock, 0, s>>>(p_lo[pcur], p_hi[pcur], pool_n, n, out.out_dets);
            ASCI_LAUNCH_CHECK();
            ASCI_HIP(hipMemcpyAsync(out.out_num, p_num, pool_n * sizeof(double), hipMemcpyDeviceToDevice, s));
            ASCI_HIP(hipMemcpyAsync(out.out_scores, p_score[pcur], pool_n * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        ASCI_HIP(hipStreamSynchronize(s));
        return;
    }
    // step 10: the k largest |A| (ties: smaller key), then |A| descending
    const size_t kk = (size_t)std::min<uint64_t>((uint64_t)out.k, pool_n);
    out.count = (int64_t)kk;
    if (kk == 0) {
        ASCI_HIP(hipStreamSynchronize(s));
        return;
    }
    if (kk < pool_n) prune(kk);
    {
        uint64_t *fk[2] = {ar.take<uint64_t>(kk), ar.take<uint64_t>(kk)};
        uint32_t *fi[2] = {ar.take<uint32_t>(kk), ar.take<uint32_t>(kk)};
        uint64_t *nohi[2] = {nullptr, nullptr};
        k_final_keys<<<grid_for(kk), kBlock, 0, s>>>(p_score[pcur], kk, fk[0], fi[0]);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> fd;
        for (int sh = 0; sh < 64; sh += 8) fd.push_back({0, sh});
        const int rr = radix_sort<uint32_t>(fk, nohi, fi, kk, 1, fd, ar, s, prof);
        k_final_gather<W><<<grid_for(kk), kBlock, 0, s>>>(fi[rr], kk, p_lo[pcur], p_hi[pcur], p_score[pcur], n,
                                                          out.out_dets, out.out_scores);
        ASCI_LAUNCH_CHECK();
    }
    ASCI_HIP(hipStreamSynchronize(s));
}

void search_device(asci_ctx *ctx, const SearchArgs &in, SearchOut &out, hipStream_t s)
{
    if (in.n <= 32) run_search<1>(ctx, in, out, s);
    else run_search<2>(ctx, in, out, s);
    if (ctx->prof.on) ctx->prof.collect();
}

// ---------------------------------------------------------------- class counts (step 4 exposed)
void validate_dets(asci_ctx *ctx, const uint64_t *dets, int64_t ndets, int n, int na, int nb, hipStream_t s)
{
    const size_t nd = (size_t)ndets;
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    Arena &ar = ctx->setup;
    ar.reset();
    ar.reserve(4096);
    ar.reset();
    unsigned int *d_err = ar.take<unsigned int>(16);
    ASCI_HIP(hipMemsetAsync(d_err, 0, 16 * sizeof(unsigned int), s));
    k_validate<<<grid_for(nd), kBlock, 0, s>>>(dets, nd, full, na, nb, d_err);
    ASCI_LAUNCH_CHECK();
    HostStage &hs = ctx->stage;
    hs.reserve(256);
    ASCI_HIP(hipMemcpyAsync(hs.ptr, d_err, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    if (*(unsigned int *)hs.ptr) throw Error{ASCI_EINVAL, "input determinant with wrong electron count or orbital >= norb"};
}

void class_counts_device(asci_ctx *ctx, int n, int na, int nb, const uint64_t *dets, const double *coeffs,
                         int64_t ndets, int64_t ncore, std::vector<uint64_t> &masks,
                         std::vector<uint64_t> &counts, hipStream_t s)
{
    masks.clear();
    counts.clear();
    auto collect = [&](const std::vector<uint64_t> &cls, const std::vector<uint64_t> &tot) {
        for (size_t c = 0; c < cls.size(); ++c)
            if (tot[c]) {
                masks.push_back(cls[c]);
                counts.push_back(tot[c]);
            }
    };
    if (n <= 32) {
        Prepared<1> pp;
        prepare<1>(ctx, nullptr, n, na, nb, dets, coeffs, ndets, ncore, false, pp, s);
        collect(pp.cls, pp.totals);
    } else {
        Prepared<2> pp;
        prepare<2>(ctx, nullptr, n, na, nb, dets, coeffs, ndets, ncore, false, pp, s);
        collect(pp.cls, pp.totals);
    }
}

}  // namespace asci
