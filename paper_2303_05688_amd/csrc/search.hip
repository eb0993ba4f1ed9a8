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
constexpr uint32_t kMaxBatchClasses = 2048;
constexpr size_t kMaxClasses = (size_t)1 << 20;  // classes of one search, all levels

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

// C(x, k) for k <= 6 and x < 64 (exact: every partial product is a binomial).
// Unrolled, so that every division is by a constant (a multiply and a shift).
__device__ __forceinline__ uint32_t choose_le6(uint32_t x, int k)
{
    if ((int)x < k) return 0u;
    uint32_t r = 1u;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        if (i < k) r = r * (x - (uint32_t)i) / (uint32_t)(i + 1);
    return r;
}

// The class of an alpha string.  Root classes are the sets of its top Lr
// occupied orbitals, ranked among all admissible Lr-subsets in ascending mask
// order (combinatorial number system on x = orbital - (n_alpha - Lr)).  A root
// class that was split (a heavy class, refined by one more highest occupied
// orbital per level) is followed through `tree`: an entry with the top bit set
// is the base of its children, indexed by the next orbital's rank
// o - (n_alpha - level); any other entry is the final class number.  Class
// numbers follow ascending mask order, i.e. key order.
struct ClassMap {
    int Lr;                // root level (0: a single class)
    int na;
    const uint32_t *tree;  // null when no class is split
};

__device__ __forceinline__ uint32_t class_of(uint64_t a, const ClassMap &m)
{
    if (m.Lr == 0) return 0u;
    const int L0 = m.na - m.Lr;
    uint32_t idx = 0u;
    for (int j = 0; j < m.Lr; ++j) {
        const int o = 63 - __clzll((long long)a);
        a &= ~(1ull << o);
        idx += choose_le6((uint32_t)(o - L0), m.Lr - j);
    }
    if (!m.tree) return idx;
    uint32_t e = m.tree[idx];
    int level = m.Lr;
    while (e & 0x80000000u) {
        const int o = 63 - __clzll((long long)a);
        a &= ~(1ull << o);
        ++level;
        e = m.tree[(e & 0x7FFFFFFFu) + (uint32_t)(o - (m.na - level))];
    }
    return e;
}

struct GenArgs {
    const uint64_t *core_a, *core_b;
    const double *core_c;
    uint32_t nq;
    uint32_t c0, nc;          // batch classes [c0, c0 + nc)
    int nbits;                // bits of nc - 1
    const uint32_t *offsets;  // [nc][nq] start of every (class, core) item
    const double *h;
    const double *eri8;  // the integrals in 8-fold packed form (checked symmetric)
    int n, na, nb;
    ClassMap cmap;
    uint64_t full;
    uint32_t nas, nbs, f0, f1, pva2, npa2, pvb2, npb2;  // table sizes and block sizes
    uint64_t *klo, *khi;
    double *vals;
    size_t cap;
    int force_fault;  // raise kFaultForced once (tests of the error path)
};

// a spin string with the two orbitals of a single's table entry (p | q << 8) flipped
__device__ __forceinline__ uint64_t flip2(uint64_t s, uint32_t x)
{
    return s ^ (1ull << (x & 0xFFu)) ^ (1ull << ((x >> 8) & 0xFFu));
}

template <int W>
__device__ __forceinline__ void emit(const GenArgs &g, size_t dst, uint64_t a2, uint64_t b2, double v)
{
    if (dst < g.cap) {
        put_key<W>(g.klo, g.khi, dst, a2, b2, g.n);
        g.vals[dst] = v;
    } else {
        raise_fault(kFaultSlot);
    }
}

// One wavefront per core determinant: emits every single and double of the
// core whose target lies in the batch's classes, at the slots of the
// (class, core) items.  Per-core tables in LDS: occupied / virtual orbital
// lists, all alpha singles (target string, H value, class, slot) and all beta
// singles (target string, orbitals, sign).  Records are emitted by type in
// flattened lane-parallel loops:
//   f0 block (alpha unchanged): beta singles, then beta-beta doubles;
//   one block per alpha single p->q: the single itself, then the alpha-beta
//     doubles with every beta single;
//   alpha-alpha doubles, one record each.
// Inside an item the record order is arbitrary (each target appears once per
// core); items are laid out (class, core), so equal keys of different cores
// stay in ascending core order through the stable sort.
template <int W>
__global__ __launch_bounds__(64) void k_generate(GenArgs g)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // workgroups go to the 8 XCDs in turn: give each XCD a contiguous range of
    // cores, so that neighbouring cores (which share lines of the offset
    // matrix) meet in the same L2
    const uint32_t per = (g.nq + 7u) / 8u;
    const uint32_t i = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    if (g.force_fault && blockIdx.x == 0 && threadIdx.x == 0) raise_fault(kFaultForced);
    if (i >= g.nq) return;
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int n = g.n;
    const uint32_t va = (uint32_t)(n - g.na), vb = (uint32_t)(n - g.nb);
    // Every orbital below comes from the lists built here out of the core's
    // bits below n (the input strings are validated), so the integrals are
    // read without a range test (EriListed, EriPacked::pairs).
    const EriPacked E{g.eri8, n};
    const EriListed L{E};

    // (a single's target string is the core's string with the two orbital
    // bits of its table entry flipped: flip2)
    double *asV = (double *)smem;                     // nas
    uint32_t *asP = (uint32_t *)(asV + g.nas);        // nas: slot, or ~0 outside the batch
    uint32_t *asX = asP + g.nas;                      // nas: p | q << 8 | (sign < 0) << 16 | tri(p, q) << 20
    uint32_t *asL = asX + g.nas;                      // nas: compacted in-batch alpha singles
    uint32_t *bsX = asL + g.nas;                      // nbs: r | s << 8 | (sign < 0) << 16 | tri(r, s) << 20
    uint32_t *cur = bsX + g.nbs;                      // nc cursors
    uint8_t *occA = (uint8_t *)(cur + g.nc), *virA = occA + 64, *occB = occA + 128, *virB = occA + 192;
    // orbital pairs in the order unrank_pair enumerates them: lo | hi << 8
    uint16_t *pOA = (uint16_t *)(occA + 256), *pVA = pOA + g.npa2, *pOB = pVA + g.pva2, *pVB = pOB + g.npb2;
    uint16_t *hpL = pVB + g.pvb2;  // npa2: alpha hole pairs whose doubles reach the batch
    // npa2: their particle-pair ranges (first | end << 16)
    uint32_t *hpR = reinterpret_cast<uint32_t *>((reinterpret_cast<uintptr_t>(hpL + g.npa2) + 3u) & ~(uintptr_t)3u);
    __shared__ uint32_t s_nsel;

    const uint64_t a = g.core_a[i], b = g.core_b[i];
    const double ci = g.core_c[i];
    {
        const bool inr = lane < n;
        const bool oa = inr && ((a >> lane) & 1ull), ob = inr && ((b >> lane) & 1ull);
        const uint64_t boa = __ballot(oa), bva = __ballot(inr && !oa);
        const uint64_t bob = __ballot(ob), bvb = __ballot(inr && !ob);
        if (oa) occA[__popcll(boa & lt)] = (uint8_t)lane;
        else if (inr) virA[__popcll(bva & lt)] = (uint8_t)lane;
        if (ob) occB[__popcll(bob & lt)] = (uint8_t)lane;
        else if (inr) virB[__popcll(bvb & lt)] = (uint8_t)lane;
        // cursors start at the (class, core) item starts: one strided read per
        // class here instead of one per record below
        for (uint32_t t = lane; t < g.nc; t += 64) cur[t] = g.offsets[(size_t)t * g.nq + i];
    }
    __syncthreads();
    // alpha singles: target, class, H value (the O(n) sums, lane-parallel)
    for (uint32_t u = lane; u < g.nas; u += 64) {
        const int p = occA[u / va], q = virA[u % va];
        const uint64_t a2 = (a & ~(1ull << p)) | (1ull << q);
        const uint32_t c = class_of(a2, g.cmap);
        const bool in = c >= g.c0 && c < g.c0 + g.nc;
        // the element (an O(n) sum) only for singles whose class is in the batch
        asV[u] = in ? single_value_e(g.h, L, n, a, b, p, q) : 0.0;
        asX[u] = (uint32_t)p | ((uint32_t)q << 8) | (between_sign(a, p, q) < 0 ? (1u << 16) : 0u) |
                 (tri((uint32_t)p, (uint32_t)q) << 20);
        asP[u] = in ? c - g.c0 : ~0u;
    }
    // occupied and virtual orbital pairs of both spins (hole and particle pairs
    // of the doubles)
    {
        auto fill = [&](uint16_t *tab, uint32_t cnt, const uint8_t *orb) {
            for (uint32_t t = lane; t < cnt; t += 64) {
                int i1, j1;
                unrank_pair(t, i1, j1);
                tab[t] = (uint16_t)(orb[i1] | ((uint32_t)orb[j1] << 8));
            }
        };
        fill(pOA, g.npa2, occA);
        fill(pVA, g.pva2, virA);
        fill(pOB, g.npb2, occB);
        fill(pVB, g.pvb2, virB);
    }
    // beta singles: target, orbitals, sign
    for (uint32_t t = lane; t < g.nbs; t += 64) {
        const int r = occB[t / vb], s = virB[t % vb];
        bsX[t] = (uint32_t)r | ((uint32_t)s << 8) | (between_sign(b, r, s) < 0 ? (1u << 16) : 0u) |
                 (tri((uint32_t)r, (uint32_t)s) << 20);
    }
    const uint32_t cs = class_of(a, g.cmap);
    const bool self_in = cs >= g.c0 && cs < g.c0 + g.nc;
    if (lane == 0 && self_in) cur[cs - g.c0] += g.f0;
    __syncthreads();

    // f0 block: the alpha string is unchanged
    if (self_in && g.f0) {
        const size_t base = g.offsets[(size_t)(cs - g.c0) * g.nq + i];
        const uint32_t ns1 = min(g.nbs, g.f0);
        for (uint32_t t = lane; t < ns1; t += 64) {
            const uint32_t x = bsX[t];
            const double hv = single_value_e(g.h, L, n, b, a, (int)(x & 0xFFu), (int)((x >> 8) & 0xFFu));
            emit<W>(g, base + t, a, flip2(b, x), hv * ci);
        }
        // beta-beta doubles y = hole pair * pvb2 + particle pair, the pair
        // indices advanced by the 64 records a lane strides over
        const uint32_t nd2 = g.f0 - ns1;
        if (nd2) {
            const uint32_t q64 = 64u / g.pvb2, r64 = 64u % g.pvb2;
            uint32_t hp = (uint32_t)lane / g.pvb2, pp = (uint32_t)lane % g.pvb2;
            for (uint32_t y = lane; y < nd2; y += 64) {
                const uint32_t po = pOB[hp], pv = pVB[pp];
                const uint64_t hb = (1ull << (po & 0xFFu)) | (1ull << (po >> 8));
                const uint64_t pb = (1ull << (pv & 0xFFu)) | (1ull << (pv >> 8));
                const uint64_t b2 = (b & ~hb) | pb;
                emit<W>(g, base + ns1 + y, a, b2,
                        double_same_times(E, b, (int)(po & 0xFFu), (int)(po >> 8), (int)(pv & 0xFFu), (int)(pv >> 8), ci));
                pp += r64;
                hp += q64;
                if (pp >= g.pvb2) {
                    pp -= g.pvb2;
                    ++hp;
                }
            }
        }
    }
    // slots of the alpha-single blocks: rank among equal classes, in u order
    if (lane == 0) s_nsel = 0u;
    __syncthreads();
    for (uint32_t u0 = 0; u0 < g.nas; u0 += 64) {
        const uint32_t u = u0 + lane;
        const uint32_t lc = u < g.nas ? asP[u] : ~0u;
        const bool act = lc != ~0u;
        const uint32_t key = act ? lc : 0u;
        const uint64_t peers = wave_match(key, act, g.nbits);
        const uint32_t before = cur[key];
        const uint64_t sel = __ballot(act);
        const uint32_t nsel0 = s_nsel;
        if (act) {
            asP[u] = before + (uint32_t)__popcll(peers & lt) * g.f1;
            asL[nsel0 + __popcll(sel & lt)] = u;
            if ((peers & lt) == 0ull) cur[key] = before + (uint32_t)__popcll(peers) * g.f1;
        }
        if (lane == 0) s_nsel = nsel0 + (uint32_t)__popcll(sel);
        __syncthreads();
    }
    // alpha-single blocks: the single at the block's first slot, then its
    // alpha-beta doubles with every beta single, flattened over (selected
    // single, beta single).  The double's integral (qp|sr) is read at the pair
    // indices kept in the tables; its sign is applied to the product with c_i.
    for (uint32_t k = lane; k < s_nsel; k += 64) {
        const uint32_t u = asL[k];
        emit<W>(g, (size_t)asP[u], flip2(a, asX[u]), b, asV[u] * ci);
    }
    if (g.nbs) {
        const uint32_t nbs = g.nbs, total = s_nsel * nbs;
        const uint32_t q64 = 64u / nbs, r64 = 64u % nbs;
        uint32_t k = (uint32_t)lane / nbs, j = (uint32_t)lane % nbs;  // t = k * nbs + j
        for (uint32_t t = lane; t < total; t += 64, j += r64, k += q64) {
            if (j >= nbs) {
                j -= nbs;
                ++k;
            }
            const uint32_t u = asL[k];
            const uint32_t x = bsX[j], xa = asX[u];
            const double v = E.pairs(xa >> 20, x >> 20) * ci;
            emit<W>(g, (size_t)asP[u] + 1u + j, flip2(a, xa), flip2(b, x), (((xa ^ x) >> 16) & 1u) ? -v : v);
        }
    }
    // alpha-alpha doubles, one record each.  The class index grows with the
    // alpha string, and for one hole pair the target grows with the particle
    // pair's index (pairs are listed by their higher, then their lower
    // orbital), so the doubles of a hole pair whose class lies in the batch
    // are one range of particle pairs: bounded by the classes of its lowest
    // and highest targets when those fall inside the batch, else found by a
    // binary search.
    if (g.npa2 && g.pva2) {
        const uint32_t cend = g.c0 + g.nc;
        const uint64_t vlo = (1ull << virA[0]) | (1ull << virA[1]);
        const uint64_t vhi = (1ull << virA[va - 1]) | (1ull << virA[va - 2]);
        // first particle pair whose target's class is at least cb (pva2: none)
        auto first_at = [&](uint64_t rest, uint32_t cb) {
            uint32_t l = 0u, r = g.pva2;
            while (l < r) {
                const uint32_t m = (l + r) >> 1;
                const uint32_t pv = pVA[m];
                const uint64_t a2 = rest | (1ull << (pv & 0xFFu)) | (1ull << (pv >> 8));
                if (class_of(a2, g.cmap) >= cb) r = m;
                else l = m + 1u;
            }
            return l;
        };
        uint32_t nact = 0;
        for (uint32_t h0 = 0; h0 < g.npa2; h0 += 64) {
            const uint32_t hp = h0 + (uint32_t)lane;
            uint32_t lo = 0u, hi = 0u;
            if (hp < g.npa2) {
                const uint32_t po = pOA[hp];
                const uint64_t rest = a & ~((1ull << (po & 0xFFu)) | (1ull << (po >> 8)));
                const uint32_t clo = class_of(rest | vlo, g.cmap), chi = class_of(rest | vhi, g.cmap);
                if (chi >= g.c0 && clo < cend) {
                    lo = clo >= g.c0 ? 0u : first_at(rest, g.c0);
                    hi = chi < cend ? g.pva2 : first_at(rest, cend);
                }
            }
            const bool act = hi > lo;
            const uint64_t m = __ballot(act);
            if (act) {
                const uint32_t slot = nact + (uint32_t)__popcll(m & lt);
                hpL[slot] = (uint16_t)hp;
                hpR[slot] = lo | (hi << 16);
            }
            nact += (uint32_t)__popcll(m);
        }
        __syncthreads();
        // The doubles are enumerated particle-pair major: for one particle
        // pair, the targets of most hole pairs share their highest orbitals
        // and hence their class, so the records of one (class, core) item are
        // written in a few contiguous bursts instead of one at a time (stores
        // of single records to many items leave partial cache lines).  Items
        // run over the rectangle [x0, x1) x listed hole pairs, hole pair
        // minor; an item outside its hole pair's range is skipped.
        uint32_t x0 = g.pva2, x1 = 0u;
        for (uint32_t kk = lane; kk < nact; kk += 64) {
            x0 = min(x0, hpR[kk] & 0xFFFFu);
            x1 = max(x1, hpR[kk] >> 16);
        }
        for (int d = 32; d >= 1; d >>= 1) {
            x0 = min(x0, (uint32_t)__shfl_xor((int)x0, d, 64));
            x1 = max(x1, (uint32_t)__shfl_xor((int)x1, d, 64));
        }
        const uint32_t total = (nact && x1 > x0) ? (x1 - x0) * nact : 0u;
        const uint32_t q64 = nact ? 64u / nact : 0u, r64 = nact ? 64u % nact : 0u;
        // t = (x - x0) * nact + k, advanced by the 64 items a lane strides over
        uint32_t k = nact ? (uint32_t)lane % nact : 0u, x = x0 + (nact ? (uint32_t)lane / nact : 0u);
        for (uint32_t t0 = 0; t0 < total; t0 += 64) {
            bool act = false;
            uint64_t a2 = a;
            uint32_t c = g.c0, po = 0u, pv = 0u;
            if (t0 + (uint32_t)lane < total) {
                const uint32_t rg = hpR[k];
                if (x >= (rg & 0xFFFFu) && x < (rg >> 16)) {
                    act = true;
                    po = pOA[hpL[k]];
                    pv = pVA[x];
                    a2 = (a & ~((1ull << (po & 0xFFu)) | (1ull << (po >> 8)))) | (1ull << (pv & 0xFFu)) |
                         (1ull << (pv >> 8));
                    c = class_of(a2, g.cmap);
                    // in the batch by construction; a class outside it is a logic error
                    if (c < g.c0 || c >= cend) {
                        raise_fault(kFaultSlot);
                        c = g.c0;
                    }
                }
            }
            k += r64;
            x += q64;
            if (k >= nact) {
                k -= nact;
                ++x;
            }
            if (__ballot(act) == 0ull) continue;  // no item of this round in a range
            const uint32_t key = c - g.c0;
            const uint64_t peers = wave_match(key, act, g.nbits);
            const uint32_t before = cur[key];
            if (act) {
                const size_t dst = (size_t)before + (uint32_t)__popcll(peers & lt);
                if ((peers & lt) == 0ull) cur[key] = before + (uint32_t)__popcll(peers);
                emit<W>(g, dst, a2, b,
                        double_same_times(E, a, (int)(po & 0xFFu), (int)(po >> 8), (int)(pv & 0xFFu), (int)(pv >> 8), ci));
            }
        }
    }
}

// ---- stable compaction of the pool to its keepk largest |score| entries:
// keep ord > t, plus the first krem entries with ord == t in pool order.
// Tiles of kKeepTile entries: per-tile counts, one pass over the tiles for
// their bases, then an in-order scatter (no per-entry flag or rank arrays).
constexpr int kKeepItems = 16;
constexpr int kKeepTile = kBlock * kKeepItems;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        base += i < w ? s_w[i] : 0u;
        tot += s_w[i];
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

__device__ __forceinline__ size_t dcount(size_t n, const uint32_t *dn) { return dn ? min(n, (size_t)*dn) : n; }

__global__ __launch_bounds__(kBlock) void k_keep_count(const double *__restrict__ score, size_t n,
                                                       const SelectState *__restrict__ st, uint32_t *__restrict__ tgt,
                                                       uint32_t *__restrict__ teq, const uint32_t *dn)
{
    n = dcount(n, dn);
    __shared__ uint32_t s_w[kBlock / 64];
    const uint64_t t = st->prefix;
    const size_t base = (size_t)blockIdx.x * kKeepTile;
    uint32_t gt = 0, eq = 0;
#pragma unroll
    for (int i = 0; i < kKeepItems; ++i) {
        const size_t j = base + (size_t)i * kBlock + threadIdx.x;
        if (j < n) {
            const uint64_t o = abs_order(score[j]);
            gt += o > t ? 1u : 0u;
            eq += o == t ? 1u : 0u;
        }
    }
    uint32_t tg, te;
    (void)block_excl_scan(gt, s_w, tg);
    (void)block_excl_scan(eq, s_w, te);
    if (threadIdx.x == 0) {
        tgt[blockIdx.x] = tg;
        teq[blockIdx.x] = te;
    }
}

// one block walks the tiles: equal-entry bases and output bases
__global__ __launch_bounds__(1024) void k_keep_bases(const uint32_t *__restrict__ tgt, const uint32_t *__restrict__ teq,
                                                     uint32_t nt, const SelectState *__restrict__ st,
                                                     uint32_t *__restrict__ eqbase, uint32_t *__restrict__ keptbase)
{
    __shared__ uint32_t s_w[16];
    const uint64_t krem = st->krem;
    uint32_t eq_run = 0, kept_run = 0;
    for (uint32_t c0 = 0; c0 < nt; c0 += 1024) {
        const uint32_t i = c0 + threadIdx.x;
        const uint32_t e = i < nt ? teq[i] : 0u, g = i < nt ? tgt[i] : 0u;
        uint32_t etot, ktot;
        const uint32_t eb = eq_run + block_excl_scan(e, s_w, etot);
        const uint64_t left = krem > eb ? krem - eb : 0ull;
        const uint32_t kept = g + (uint32_t)(left < e ? left : e);
        const uint32_t kb = kept_run + block_excl_scan(kept, s_w, ktot);
        if (i < nt) {
            eqbase[i] = eb;
            keptbase[i] = kb;
        }
        eq_run += etot;
        kept_run += ktot;
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_keep_scatter(const uint64_t *__restrict__ ilo,
                                                         const uint64_t *__restrict__ ihi,
                                                         const double *__restrict__ iscore, size_t n,
                                                         const SelectState *__restrict__ st,
                                                         const uint32_t *__restrict__ eqbase,
                                                         const uint32_t *__restrict__ keptbase,
                                                         uint64_t *__restrict__ olo, uint64_t *__restrict__ ohi,
                                                         double *__restrict__ oscore, size_t cap, const uint32_t *dn)
{
    constexpr int NW = kBlock / 64;
    n = dcount(n, dn);
    __shared__ uint32_t s_w[NW];
    const uint64_t t = st->prefix, krem = st->krem;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    // wave-contiguous chunks, lane-strided inside (coalesced loads); the pool
    // order inside the tile is (wave, item, lane), and ranks follow it
    const size_t wbase = (size_t)blockIdx.x * kKeepTile + (size_t)wv * 64 * kKeepItems;
    uint64_t o[kKeepItems];
    uint64_t eqm[kKeepItems];
    uint32_t weq = 0;
#pragma unroll
    for (int i = 0; i < kKeepItems; ++i) {
        const size_t j = wbase + (size_t)i * 64 + lane;
        o[i] = j < n ? abs_order(iscore[j]) : 0ull;
        eqm[i] = __ballot(j < n && o[i] == t);
        weq += (uint32_t)__popcll(eqm[i]);
    }
    uint32_t tot;
    uint32_t erank = eqbase[blockIdx.x] + block_excl_scan(lane == 0 ? weq : 0u, s_w, tot);
    erank = (uint32_t)__shfl((int)erank, 0, 64);
    uint64_t keptm[kKeepItems];
    uint32_t wkept = 0;
#pragma unroll
    for (int i = 0; i < kKeepItems; ++i) {
        const size_t j = wbase + (size_t)i * 64 + lane;
        bool k = false;
        if (j < n) {
            if (o[i] > t) k = true;
            else if (o[i] == t) k = erank + (uint32_t)__popcll(eqm[i] & lt) < krem;
        }
        erank += (uint32_t)__popcll(eqm[i]);
        keptm[i] = __ballot(k);
        wkept += (uint32_t)__popcll(keptm[i]);
    }
    uint32_t at = keptbase[blockIdx.x] + block_excl_scan(lane == 0 ? wkept : 0u, s_w, tot);
    at = (uint32_t)__shfl((int)at, 0, 64);
#pragma unroll
    for (int i = 0; i < kKeepItems; ++i) {
        if ((keptm[i] >> lane) & 1ull) {
            const size_t j = wbase + (size_t)i * 64 + lane;
            const uint32_t d = at + (uint32_t)__popcll(keptm[i] & lt);
            if (d < cap) {
                olo[d] = ilo[j];
                if (W == 2) ohi[d] = ihi[j];
                oscore[d] = iscore[j];
            } else {
                raise_fault(kFaultSlot);
            }
        }
        at += (uint32_t)__popcll(keptm[i]);
    }
}

// sort key for the final order: ~|score| bits so that ascending = descending |score|
__global__ __launch_bounds__(kBlock) void k_final_keys(const double *__restrict__ score, size_t n,
                                                       uint64_t *__restrict__ key, uint32_t *__restrict__ idx,
                                                       const uint32_t *dn)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= dcount(n, dn)) return;
    key[j] = ~abs_order(score[j]);
    idx[j] = (uint32_t)j;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_final_gather(const uint32_t *__restrict__ idx, size_t n,
                                                         const uint64_t *__restrict__ slo,
                                                         const uint64_t *__restrict__ shi,
                                                         const double *__restrict__ sscore, int norb,
                                                         uint64_t *__restrict__ out_dets,
                                                         double *__restrict__ out_scores, const uint32_t *dn,
                                                         const uint32_t *stat)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= dcount(n, dn) || (stat && *stat)) return;  // a failed call writes no output
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

// insert every input key into the hash set (keys as (lo, hi) words)
template <int W>
__global__ __launch_bounds__(kBlock) void k_psi_insert(const uint64_t *__restrict__ dets, size_t nd, int n,
                                                       uint64_t *__restrict__ tlo, uint64_t *__restrict__ thi,
                                                       uint32_t *__restrict__ state, uint32_t mask,
                                                       unsigned long long *__restrict__ filter, uint32_t fmask)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd) return;
    const uint64_t a = dets[2 * j], b = dets[2 * j + 1];
    const uint64_t lo = W == 1 ? ((a << n) | b) : b, hi = W == 1 ? 0ull : a;
    const uint64_t fh = psi_filter_hash(lo, hi);
    atomicOr(&filter[psi_filter_word(fh, fmask)], (unsigned long long)psi_filter_bits(fh));
    uint32_t s = psi_hash(lo, hi, mask);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        if (atomicCAS(&state[s], 0u, 1u) == 0u) {
            tlo[s] = lo;
            thi[s] = hi;
            return;
        }
        s = (s + 1u) & mask;
    }
}

// bit 1 of err: an input determinant stored twice in the hash set (every insert
// has finished: this runs as a kernel of its own)
template <int W>
__global__ __launch_bounds__(kBlock) void k_psi_dups(const uint64_t *__restrict__ dets, size_t nd, int n, PsiSet t,
                                                     unsigned int *__restrict__ err)
{
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd) return;
    const uint64_t a = dets[2 * j], b = dets[2 * j + 1];
    const uint64_t lo = W == 1 ? ((a << n) | b) : b, hi = W == 1 ? 0ull : a;
    uint32_t sl = psi_hash(lo, hi, t.mask), seen = 0;
    for (uint32_t probe = 0; probe <= t.mask && t.state[sl]; ++probe) {
        if (t.lo[sl] == lo && t.hi[sl] == hi) ++seen;
        sl = (sl + 1u) & t.mask;
    }
    if (seen > 1) atomicOr(err, 2u);
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

// J_pq = (pp|qq), X_pq = (pp|qq) - (pq|qp), then h_pp: the tables of the diagonal H_aa
__global__ __launch_bounds__(kBlock) void k_jk(const double *__restrict__ eri, const double *__restrict__ h, int n,
                                               double *__restrict__ jk)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    jk[t] = eri4(eri, n, p, p, q, q);
    jk[n * n + t] = eri4(eri, n, p, p, q, q) - eri4(eri, n, p, q, q, p);
    if (q == 0) jk[2 * n * n + p] = h[(size_t)p * n + p];
}

// The 8-fold packed copy of the integrals (the form the generator reads: a
// few hundred KB that stay in L2, where the full tensor does not), written by
// the canonical entry of each set of equal ones (p >= q, r >= s, pq >= rs).
__global__ __launch_bounds__(kBlock) void k_eri_pack(const double *__restrict__ eri, int n,
                                                     double *__restrict__ packed)
{
    const uint32_t un = (uint32_t)n;
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= un * un * un * un) return;
    const uint32_t s_ = t % un, r = (t / un) % un, q = (t / (un * un)) % un, p = t / (un * un * un);
    if (p < q || r < s_) return;
    const uint32_t pq = tri(p, q), rs = tri(r, s_);
    if (pq >= rs) packed[tri(pq, rs)] = eri[t];
}

// every entry equals its packed representative bit for bit, else the
// integrals are not 8-fold symmetric: err |= 4
__global__ __launch_bounds__(kBlock) void k_eri_check(const double *__restrict__ eri, int n,
                                                      const double *__restrict__ packed, unsigned int *err)
{
    const uint32_t un = (uint32_t)n;
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= un * un * un * un) return;
    const uint32_t s_ = t % un, r = (t / un) % un, q = (t / (un * un)) % un, p = t / (un * un * un);
    const double v = packed[tri(tri(p, q), tri(r, s_))];
    if (__double_as_longlong(v) != __double_as_longlong(eri[t])) atomicOr(err, 4u);
}

inline unsigned grid_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

inline uint64_t choose_u64(uint64_t x, int k)
{
    if (k < 0 || (uint64_t)k > x) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (x - k + i) / i;
    return r;
}

// the constraint classes of level L in ascending mask order: the sets of the L
// highest occupied alpha orbitals that a string with na electrons can have
// (all na orbitals when na < L)
std::vector<uint64_t> make_classes(int n, int na, int L)
{
    require(L >= 0 && L <= 64 && na >= 0 && na <= n, ASCI_EINVAL, "constraint level out of range");
    std::vector<uint64_t> out;
    L = std::min(L, na);
    if (L == 0) {
        out.push_back(0ull);
        return out;
    }
    // all L-subsets o_1 > ... > o_L with o_L >= na - L
    std::function<void(int, int, uint64_t)> rec = [&](int depth, int below, uint64_t mask) {
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

// E(s) of every string of ne electrons in n orbitals, by rank: the string is
// unranked in the combinatorial number system (highest bit first: the largest
// p with C(p, j) <= remaining rank, for j = ne, ..., 1) and evaluated by the
// same routine as the direct path, so a looked-up value equals a computed one
__global__ __launch_bounds__(kBlock) void k_spin_table(const double *__restrict__ jk, int n, int ne,
                                                      const uint32_t *__restrict__ binom, uint32_t count,
                                                      double *__restrict__ out)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= count) return;
    uint32_t rem = r;
    uint64_t str = 0;
    int p = n - 1;
    for (int j = ne; j >= 1; --j) {
        const uint32_t *row = binom + (size_t)j * (n + 1);
        while (p > 0 && row[p] > rem) --p;  // C(p, j) = 0 <= rem once p < j
        str |= 1ull << p;
        rem -= row[p];
        --p;
    }
    out[r] = spin_energy(jk + n * n, jk + 2 * n * n, n, str);
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

// ---- spin-string energy tables (E(alpha), E(beta) looked up by rank)
static uint64_t binom_sat(int n, int k)
{
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    unsigned __int128 c = 1;
    for (int i = 1; i <= k; ++i) {
        c = c * (unsigned)(n - k + i) / (unsigned)i;
        if (c > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    }
    return (uint64_t)c;
}

SpinTablePlan spin_table_plan(int n, int na, int nb, uint64_t pairs, bool enabled)
{
    SpinTablePlan pl;
    const int ne[2] = {na, nb};
    for (int i = 0; i < 2; ++i) {
        const uint64_t c = binom_sat(n, ne[i]);
        // a table pays when it is small next to the search that reads it
        pl.count[i] = (enabled && c <= kSpinTableMax && (c <= (1u << 16) || 4 * c <= pairs)) ? c : 0;
    }
    pl.share = na == nb;
    if (pl.share) pl.count[1] = pl.count[0];
    if (pl.count[0] == 0 && pl.count[1] == 0) return pl;
    pl.kmax = std::max(pl.count[0] ? na : 0, pl.count[1] ? nb : 0);
    const size_t tab = (size_t)(pl.count[0] + (pl.share ? 0 : pl.count[1])) * 8;
    pl.bytes = tab + (size_t)(pl.kmax + 4) * (n + 1) * 4 + 1024;
    return pl;
}

// Build the tables of `pl` for the integrals' J / J-K / h_pp table `jk`.
static SpinTables build_spin_tables(asci_ctx *ctx, const SpinTablePlan &pl, const double *jk, int n, int na, int nb,
                                    hipStream_t s)
{
    SpinTables st;
    if (pl.bytes == 0) return st;
    Arena &ar = ctx->tables;
    ar.reset();
    ar.reserve(pl.bytes);
    ar.reset();
    // rows 0..kmax, and three zero rows that the rank's unconditional loads may
    // touch past the last electron
    std::vector<uint32_t> hb((size_t)(pl.kmax + 4) * (n + 1), 0u);
    for (int k = 0; k <= pl.kmax; ++k)
        for (int p = 0; p <= n; ++p)
            hb[(size_t)k * (n + 1) + p] = (uint32_t)std::min<uint64_t>(binom_sat(p, k), UINT32_MAX);
    uint32_t *d_binom = ar.take<uint32_t>(hb.size());
    HostStage &hs = ctx->stage;
    hs.reserve(hb.size() * 4);
    std::memcpy(hs.ptr, hb.data(), hb.size() * 4);
    ASCI_HIP(hipMemcpyAsync(d_binom, hs.ptr, hb.size() * 4, hipMemcpyHostToDevice, s));
    st.binom = d_binom;
    st.kmax = pl.kmax;
    const int ne[2] = {na, nb};
    for (int i = 0; i < 2; ++i) {
        if (pl.count[i] == 0) continue;
        if (i == 1 && pl.share) {
            st.e[1] = st.e[0];
            continue;
        }
        double *t = ar.take<double>(pl.count[i]);
        k_spin_table<<<(unsigned)((pl.count[i] + kBlock - 1) / kBlock), kBlock, 0, s>>>(jk, n, ne[i], d_binom,
                                                                                    (uint32_t)pl.count[i], t);
        ASCI_LAUNCH_CHECK();
        st.e[i] = t;
    }
    // the staged binomials are read by the copy above
    ASCI_HIP(hipStreamSynchronize(s));
    return st;
}

// bytes of the setup arena of a search: inputs keyed, the psi hash set and
// filter, core set, class masks / totals / split tree, integral tables
static size_t setup_bytes(size_t nd, size_t nq, int n, int W)
{
    const size_t hist_bytes = ((nd + kScanTile - 1) / kScanTile) * 256 * 4 * 2 + (1 << 16);
    return nd * (8 * 2 * W + 4 * 2) + nd * (8 * 2 + 4 * 2) + nq * 8 * 4 + kMaxClasses * 20 + (size_t)2 * n * n * 8 +
           2 * hist_bytes + 64 * 256 + (nd * 8 + 1024) * 20 + nd * 8 + eri_packed_count(n) * 8 + 256 + (1 << 14);
}

// bytes of the main arena: count matrix and offsets (E entries), the pair
// buffers of one class batch (Pb records), the candidate pool, the selection
static size_t main_bytes(size_t E, size_t Pb, size_t pool_cap, uint32_t max_nc, size_t kk_max, bool topk, int W,
                         int finish_cap)
{
    const size_t rec_bytes = 2 * (8 * W + 8);
    const size_t scan_tmp = ((std::max<size_t>(Pb, E) + kScanTile - 1) / kScanTile) * 4 + 4096;
    return E * 8 + Pb * rec_bytes + scan_tmp + Pb * (8 * W + (topk ? 8 : 16)) +
           bucket_workspace_bytes(Pb, max_nc, W, finish_cap) + pool_cap * ((8 * W + 8) * 2 + (topk ? 0 : 8) + 1) +
           kk_max * 24 + 64 * 256 + (1 << 16);
}

// inputs shared by the search entry points: validated, keyed and core-selected
template <int W>
struct Prepared {
    size_t nd = 0, nq = 0;
    uint64_t *q_a = nullptr, *q_b = nullptr;         // core set, ascending input index
    double *q_c = nullptr;
    uint64_t *d_cls = nullptr;
    double *d_jk = nullptr;
    double *d_eri8 = nullptr;  // the integrals, 8-fold packed (when given)
    std::vector<uint64_t> cls, totals;  // final classes (ascending mask) and their pair counts
    int Lr = 0;                         // level of the root classes
    uint32_t *d_tree = nullptr;         // split tree (null when no class is split)
    PsiSet psi;
    ClassMap cmap(int na) const { return ClassMap{Lr, na, d_tree}; }
};

// pair totals of a list of classes (step 4 without the matrix), on the host
static void count_classes(const uint64_t *q_a, uint32_t nq, const std::vector<uint64_t> &masks, uint64_t *d_cls,
                          unsigned long long *d_tot, uint64_t full, const BetaFactors &bf, HostStage &hs,
                          std::vector<uint64_t> &tot, hipStream_t s)
{
    const size_t m = masks.size();
    tot.assign(m, 0);
    if (m == 0) return;
    ASCI_HIP(hipMemcpyAsync(d_cls, masks.data(), m * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    ASCI_HIP(hipMemsetAsync(d_tot, 0, m * sizeof(unsigned long long), s));
    for (size_t c0 = 0; c0 < m; c0 += 65535) {
        const unsigned ny = (unsigned)std::min<size_t>(65535, m - c0);
        dim3 g((unsigned)((nq + kBlock - 1) / kBlock), ny);
        k_count<<<g, kBlock, 0, s>>>(q_a, nq, d_cls, (uint32_t)c0, full, bf, nullptr, d_tot);
        ASCI_LAUNCH_CHECK();
    }
    hs.reserve(m * sizeof(uint64_t));
    ASCI_HIP(hipMemcpyAsync(hs.ptr, d_tot, m * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    std::memcpy(tot.data(), hs.ptr, m * sizeof(uint64_t));
}

// Classes of the search (Sec. II.B, Alg. 3).  Uniform (split_pairs == 0): every
// class at level L.  Adaptive (split_pairs > 0): the classes start at level
// min(L, 3) and a class with more than split_pairs pairs is replaced by the
// classes of the next level (one more highest occupied orbital) up to level L.
// Either way a class with more than `fit` pairs (the pair buffer) is split
// further, up to level 6, so that it fits.  The split classes partition the
// targets exactly like the classes they replace.
static void plan_classes(int n, int na, int L, int64_t split_pairs, uint64_t fit, const uint64_t *q_a,
                         uint32_t nq, uint64_t *d_cls, unsigned long long *d_tot, uint64_t full,
                         const BetaFactors &bf, HostStage &hs, std::vector<uint64_t> &cls,
                         std::vector<uint64_t> &totals, std::vector<uint32_t> &tree, int &Lr, hipStream_t s)
{
    Lr = std::min(split_pairs > 0 ? std::min(L, 3) : L, na);
    require(choose_u64((uint64_t)(n - na + Lr), Lr) <= kMaxClasses, ASCI_EINVAL,
            "too many constraint classes at this level");
    std::vector<uint64_t> roots = make_classes(n, na, Lr);
    std::vector<uint64_t> rt;
    count_classes(q_a, nq, roots, d_cls, d_tot, full, bf, hs, rt, s);
    struct Node {
        uint64_t mask, total;
        int level;
        int64_t child0;
        uint32_t nchild;
    };
    std::vector<Node> nodes;
    for (size_t r = 0; r < roots.size(); ++r) nodes.push_back({roots[r], rt[r], Lr, -1, 0});
    std::vector<size_t> frontier(roots.size());
    for (size_t r = 0; r < roots.size(); ++r) frontier[r] = r;
    bool split_any = false;
    while (!frontier.empty()) {
        std::vector<uint64_t> kids;
        for (size_t v : frontier) {
            Node &nd = nodes[v];
            const int lim = nd.total > fit ? 6 : (split_pairs > 0 ? L : 0);
            const bool heavy = nd.total > fit || (split_pairs > 0 && nd.total > (uint64_t)split_pairs);
            if (!heavy || nd.level >= lim || nd.level >= na || nd.mask == 0) continue;
            const int o_lo = na - nd.level - 1, o_hi = __builtin_ctzll(nd.mask);
            if (o_hi <= o_lo) continue;
            nd.child0 = (int64_t)(nodes.size() + kids.size());
            nd.nchild = (uint32_t)(o_hi - o_lo);
            for (int o = o_lo; o < o_hi; ++o) kids.push_back(nd.mask | (1ull << o));
        }
        if (kids.empty()) break;
        split_any = true;
        require(nodes.size() + kids.size() <= kMaxClasses, ASCI_ENOMEM, "too many split constraint classes");
        std::vector<uint64_t> kt;
        count_classes(q_a, nq, kids, d_cls, d_tot, full, bf, hs, kt, s);
        std::vector<size_t> next;
        const size_t base = nodes.size();
        for (size_t c = 0; c < kids.size(); ++c) {
            // the level of a child is its parent's plus one; kids are grouped by parent
            next.push_back(base + c);
            nodes.push_back({kids[c], kt[c], 0, -1, 0});
        }
        for (size_t v : frontier)
            if (nodes[v].child0 >= 0)
                for (uint32_t c = 0; c < nodes[v].nchild; ++c) nodes[(size_t)nodes[v].child0 + c].level = nodes[v].level + 1;
        frontier.swap(next);
    }
    cls.clear();
    totals.clear();
    tree.clear();
    if (!split_any) {
        cls = roots;
        totals = rt;
        return;
    }
    // leaves in depth-first order, children ascending: ascending masks
    tree.resize(roots.size());
    std::function<void(size_t, size_t)> place = [&](size_t v, size_t slot) {
        const Node nd = nodes[v];
        if (nd.child0 < 0) {
            tree[slot] = (uint32_t)cls.size();
            cls.push_back(nd.mask);
            totals.push_back(nd.total);
            return;
        }
        const size_t base = tree.size();
        tree.resize(base + nd.nchild);
        tree[slot] = 0x80000000u | (uint32_t)base;
        for (uint32_t c = 0; c < nd.nchild; ++c) place((size_t)nd.child0 + c, base + c);
    };
    for (size_t r = 0; r < roots.size(); ++r) place(r, r);
}

// Validate the determinants, sort their keys, pick the core set and count the
// pairs of every constraint class.  All buffers live in ctx->setup.
template <int W>
static void prepare(asci_ctx *ctx, const double *d_h, const double *d_eri, int n, int na, int nb, const uint64_t *dets,
                    const double *coeffs, int64_t ndets, const asci_options &opt, uint64_t fit, bool need_psi,
                    Prepared<W> &pp, hipStream_t s)
{
    const size_t nd = (size_t)ndets;
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const BetaFactors bf = beta_factors(n, nb);
    const int64_t ncore = opt.ncore;
    pp.nd = nd;
    pp.nq = (ncore > 0 && (size_t)ncore < nd) ? (size_t)ncore : nd;
    const size_t nq = pp.nq;

    Arena &ar = ctx->setup;
    ar.reset();
    ar.reserve(setup_bytes(nd, nq, n, W));
    ar.reset();
    unsigned int *d_err = ar.take<unsigned int>(16);
    pp.d_cls = ar.take<uint64_t>(kMaxClasses);
    unsigned long long *d_tot = ar.take<unsigned long long>(kMaxClasses);
    uint32_t *d_tree = ar.take<uint32_t>(kMaxClasses);
    pp.d_jk = ar.take<double>((size_t)2 * n * n + n);
    pp.d_eri8 = ar.take<double>(eri_packed_count(n));
    pp.q_a = ar.take<uint64_t>(nq);
    pp.q_b = ar.take<uint64_t>(nq);
    pp.q_c = ar.take<double>(nq);
    uint32_t tsize = 1024;
    while (tsize < 4 * nd) tsize <<= 1;
    uint64_t *t_lo = ar.take<uint64_t>(tsize), *t_hi = ar.take<uint64_t>(tsize);
    uint32_t *t_state = ar.take<uint32_t>(tsize);
    // exclusion filter: 32 bits per input determinant (a power of two, at least 2^16)
    size_t fbits = (size_t)1 << 16;
    while (fbits < 32 * nd && fbits < ((size_t)1 << 34)) fbits <<= 1;
    unsigned long long *t_filter = ar.take<unsigned long long>(fbits / 64);
    pp.psi.lo = t_lo;
    pp.psi.hi = t_hi;
    pp.psi.state = t_state;
    pp.psi.mask = tsize - 1;
    pp.psi.filter = t_filter;
    pp.psi.fmask = (uint32_t)(fbits / 64 - 1);

    ASCI_HIP(hipMemsetAsync(d_err, 0, 16 * sizeof(unsigned int), s));
    k_validate<<<grid_for(nd), kBlock, 0, s>>>(dets, nd, full, na, nb, d_err);
    ASCI_LAUNCH_CHECK();
    if (d_eri && d_h) {
        k_jk<<<grid_for((size_t)n * n), kBlock, 0, s>>>(d_eri, d_h, n, pp.d_jk);
        ASCI_LAUNCH_CHECK();
        const size_t n4 = (size_t)n * n * n * n;
        k_eri_pack<<<grid_for(n4), kBlock, 0, s>>>(d_eri, n, pp.d_eri8);
        ASCI_LAUNCH_CHECK();
        k_eri_check<<<grid_for(n4), kBlock, 0, s>>>(d_eri, n, pp.d_eri8, d_err);
        ASCI_LAUNCH_CHECK();
    }
    if (need_psi) {
        ASCI_HIP(hipMemsetAsync(t_state, 0, (size_t)tsize * sizeof(uint32_t), s));
        ASCI_HIP(hipMemsetAsync(t_filter, 0, (size_t)fbits / 8, s));
        k_psi_insert<W><<<grid_for(nd), kBlock, 0, s>>>(dets, nd, n, t_lo, t_hi, t_state, tsize - 1, t_filter,
                                                        pp.psi.fmask);
        ASCI_LAUNCH_CHECK();
        k_psi_dups<W><<<grid_for(nd), kBlock, 0, s>>>(dets, nd, n, pp.psi, d_err);
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
    HostStage &hs = ctx->stage;
    hs.reserve(256);
    unsigned int *h_err = (unsigned int *)hs.ptr;
    ASCI_HIP(hipMemcpyAsync(h_err, d_err, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    if (h_err[0] & 1u) throw Error{ASCI_EINVAL, "input determinant with wrong electron count or orbital >= norb"};
    if (h_err[0] & 2u) throw Error{ASCI_EINVAL, "duplicate input determinants"};
    if (h_err[0] & 4u) throw Error{ASCI_EINVAL, "two-electron integrals are not 8-fold symmetric"};
    // step 4, totals per class (and the split of heavy classes)
    std::vector<uint32_t> tree;
    plan_classes(n, na, opt.constraint_level, opt.split_pairs, fit, pp.q_a, (uint32_t)nq, pp.d_cls, d_tot, full, bf,
                 hs, pp.cls, pp.totals, tree, pp.Lr, s);
    ASCI_HIP(hipMemcpyAsync(pp.d_cls, pp.cls.data(), pp.cls.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    if (!tree.empty()) {
        ASCI_HIP(hipMemcpyAsync(d_tree, tree.data(), tree.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        pp.d_tree = d_tree;
    }
    // the host vectors are read by the copies above: finish them before returning
    ASCI_HIP(hipStreamSynchronize(s));
}

template <int W>
static void run_search(asci_ctx *ctx, const SearchArgs &in, SearchOut &out, hipStream_t s)
{
    // a batch pool on this context is idle between batch calls: its workers'
    // workspaces give way to this search (they grow again in the next batch)
    if (ctx->batch_pool && ctx->batch_pool_trim) ctx->batch_pool_trim(ctx->batch_pool);
    const int n = in.n;
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const BetaFactors bf = beta_factors(n, in.nb);
    const bool topk = out.k > 0;

    Profiler *prof = &ctx->prof;
    // ---- pair-buffer capacity (records of one class batch)
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

    Prepared<W> pp;
    prepare<W>(ctx, in.h, in.eri, n, in.na, in.nb, in.dets, in.coeffs, in.ndets, in.opt, cap, true, pp, s);
    const size_t nq = pp.nq;
    const uint32_t ncls = (uint32_t)pp.cls.size();
    uint64_t all_pairs = 0;
    for (uint64_t t : pp.totals) all_pairs += t;
    const SpinTables st = build_spin_tables(ctx, spin_table_plan(n, in.na, in.nb, all_pairs, ctx->spin_tables != 0),
                                            pp.d_jk, n, in.na, in.nb, s);

    // ---- batch plan: consecutive classes up to the pair-buffer capacity
    std::vector<std::pair<uint32_t, uint32_t>> batches;
    uint64_t max_batch = 0, max_entries = 0, total = 0;
    for (uint32_t c = 0; c < ncls;) {
        uint64_t sum = 0;
        uint32_t c1 = c;
        // at most kMaxBatchClasses classes: the generator keeps one LDS cursor per class
        while (c1 < ncls && c1 - c < kMaxBatchClasses && (c1 == c || sum + pp.totals[c1] <= cap))
            sum += pp.totals[c1++];
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
    if (out.pt2) pool_cap = 1;
    else if (topk) pool_cap = (size_t)std::min<uint64_t>(total + 1, std::max<uint64_t>(4 * (uint64_t)out.k, Pb) + (uint64_t)out.k);
    else pool_cap = total + 1;
    require(pool_cap < (1ull << 32), ASCI_ENOMEM, "candidate pool too large");
    const size_t kk_max = topk ? (size_t)std::min<uint64_t>((uint64_t)out.k, pool_cap) : 0;
    uint32_t max_nc = 1;
    for (const auto &bt : batches) max_nc = std::max<uint32_t>(max_nc, bt.second - bt.first);
    Arena &ar = ctx->main;
    ar.reset();
    const int fcap = effective_finish_cap(ctx, n, in.na, search_pairs(in));
    ar.reserve(main_bytes(E, Pb, pool_cap, max_nc, kk_max, topk, W, fcap));
    ar.reset();
    uint32_t *counts = ar.take<uint32_t>(E);
    uint32_t *offs = ar.take<uint32_t>(E);
    uint64_t *k_lo[2] = {ar.take<uint64_t>(Pb), ar.take<uint64_t>(Pb)};
    uint64_t *k_hi[2] = {W == 2 ? ar.take<uint64_t>(Pb) : nullptr, W == 2 ? ar.take<uint64_t>(Pb) : nullptr};
    double *v[2] = {ar.take<double>(Pb), ar.take<double>(Pb)};
    uint64_t *c_lo = ar.take<uint64_t>(Pb);
    uint64_t *c_hi = W == 2 ? ar.take<uint64_t>(Pb) : nullptr;
    double *c_num = topk ? nullptr : ar.take<double>(Pb);  // N_a is needed only without a top k
    double *c_score = ar.take<double>(Pb);
    uint64_t *p_lo[2] = {ar.take<uint64_t>(pool_cap), ar.take<uint64_t>(pool_cap)};
    uint64_t *p_hi[2] = {W == 2 ? ar.take<uint64_t>(pool_cap) : nullptr, W == 2 ? ar.take<uint64_t>(pool_cap) : nullptr};
    double *p_num = topk ? nullptr : ar.take<double>(pool_cap);
    double *p_score[2] = {ar.take<double>(pool_cap), ar.take<double>(pool_cap)};
    SelectState *d_sel = ar.take<SelectState>(1);
    uint32_t *d_cnt = ar.take<uint32_t>(16);
    const size_t loop_mark = ar.used();

    HostStage &hs = ctx->stage;
    hs.reserve(256);
    fault_clear(s);
    bucket_fault_clear(s);
    // the end of every path: both fault words read with the last sync
    unsigned int *h_fault = (unsigned int *)((char *)hs.ptr + 224);
    auto finish = [&]() {
        fault_fetch(h_fault, s);
        bucket_fault_fetch(h_fault + 1, s);
        ASCI_HIP(hipStreamSynchronize(s));
        fault_check(h_fault[0] | h_fault[1], "the search");
    };
    int pcur = 0;
    size_t pool_n = 0;
    ctx->last_batches = (int64_t)batches.size();
    ctx->last_finals = ctx->last_levels = ctx->last_candidates = 0;

    // keep the pool's keepk entries of largest |score|, in ascending key order
    auto prune = [&](size_t keepk) {
        const size_t entry_mark = ar.used();
        const SelectWork sw{p_score[pcur ^ 1], d_cnt + 8, (unsigned int *)((char *)hs.ptr + 192)};
        radix_select_abs(p_score[pcur], pool_n, keepk, d_sel, s, prof, &sw);
        const uint32_t ntile = (uint32_t)((pool_n + kKeepTile - 1) / kKeepTile);
        uint32_t *tgt = ar.take<uint32_t>(ntile), *teq = ar.take<uint32_t>(ntile);
        uint32_t *eqb = ar.take<uint32_t>(ntile), *kb = ar.take<uint32_t>(ntile);
        const int o = pcur ^ 1;
        {
            ProfScope ps(prof, "keep", 2.0 * 8.0 * pool_n + (8.0 * W + 8.0) * 2.0 * keepk, s);
            k_keep_count<<<ntile, kBlock, 0, s>>>(p_score[pcur], pool_n, d_sel, tgt, teq, nullptr);
            ASCI_LAUNCH_CHECK();
            k_keep_bases<<<1, 1024, 0, s>>>(tgt, teq, ntile, d_sel, eqb, kb);
            ASCI_LAUNCH_CHECK();
            k_keep_scatter<W><<<ntile, kBlock, 0, s>>>(p_lo[pcur], p_hi[pcur], p_score[pcur], pool_n, d_sel, eqb, kb,
                                                       p_lo[o], p_hi[o], p_score[o], keepk, nullptr);
            ASCI_LAUNCH_CHECK();
        }
        pcur = o;
        pool_n = keepk;
        ar.reset();
        (void)ar.take<char>(entry_mark);
    };

    // after a class batch the pool is cut to the k best; the k-th |A| then
    // bounds the final one from below, and later batches (larger keys, so they
    // lose every tie) drop candidates under it in the finish kernel
    const uint64_t *d_thr = nullptr;
    for (size_t bi = 0; bi < batches.size(); ++bi) {
        const auto &bt = batches[bi];
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
        scan_u32(counts, offs, ent, d_cnt + 2, ar, s, prof);
        // step 5: generate
        ASCI_LAUNCH_CHECK();
        {
            ProfScope ps(prof, "generate", (8.0 * W + 8.0) * P, s);
            GenArgs ga;
            ga.core_a = pp.q_a;
            ga.core_b = pp.q_b;
            ga.core_c = pp.q_c;
            ga.nq = (uint32_t)nq;
            ga.c0 = c0;
            ga.nc = nc;
            ga.nbits = 1;
            while ((1u << ga.nbits) < nc) ++ga.nbits;
            ga.offsets = offs;
            ga.h = in.h;
            ga.eri8 = pp.d_eri8;
            ga.n = n;
            ga.na = in.na;
            ga.nb = in.nb;
            ga.cmap = pp.cmap(in.na);
            ga.full = full;
            const uint32_t va = (uint32_t)(n - in.na), vb = (uint32_t)(n - in.nb);
            ga.nas = (uint32_t)in.na * va;
            ga.nbs = (uint32_t)in.nb * vb;
            ga.f0 = bf.f[0];
            ga.f1 = bf.f[1];
            ga.pva2 = va * (va - (va ? 1u : 0u)) / 2u;
            ga.npa2 = (uint32_t)in.na * (uint32_t)(in.na - (in.na ? 1 : 0)) / 2u;
            ga.pvb2 = bf.pairs_vb;
            ga.npb2 = (uint32_t)in.nb * (uint32_t)(in.nb - (in.nb ? 1 : 0)) / 2u;
            ga.klo = k_lo[0];
            ga.khi = k_hi[0];
            ga.vals = v[0];
            ga.cap = Pb;
            ga.force_fault = ctx->fault_test;
            const size_t lds = (size_t)ga.nas * (8 + 4 + 4 + 4) + (size_t)ga.nbs * 4 + (size_t)nc * 4 + 256 +
                               2 * ((size_t)2 * ga.npa2 + ga.pva2 + ga.npb2 + ga.pvb2) + 4 * (size_t)ga.npa2 + 68;
            k_generate<W><<<(unsigned)(8 * ((nq + 7) / 8)), 64, lds, s>>>(ga);
            ASCI_LAUNCH_CHECK();
        }
        // steps 6-9: bucket sort-and-accumulate, exclusion, diagonal, score
        BucketArgs ba;
        ba.P = P;
        ba.c0 = c0;
        ba.nc = nc;
        ba.nq = (uint32_t)nq;
        ba.n = n;
        ba.cls = pp.d_cls;
        ba.offsets = offs;
        ba.total = d_cnt + 2;
        ba.klo[0] = k_lo[0];
        ba.klo[1] = k_lo[1];
        ba.khi[0] = k_hi[0];
        ba.khi[1] = k_hi[1];
        ba.val[0] = v[0];
        ba.val[1] = v[1];
        ba.psi = pp.psi;
        ba.jk = pp.d_jk;
        ba.h = in.h;
        ba.st = st;
        ba.thr = topk ? d_thr : nullptr;
        ba.ecore = in.opt.ecore;
        ba.E0 = in.E0;
        ba.eps = in.opt.eps;
        ba.finish_cap = fcap;
        ba.clo = c_lo;
        ba.chi = c_hi;
        ba.cnum = c_num;
        ba.cscore = c_score;
        // when the batch cannot overflow the pool, its collect is queued
        // before the host waits for the candidate count
        const bool early = !out.pt2 && pool_n + P <= pool_cap;
        ba.defer_v = early;
        ba.pool_lo = p_lo[pcur];
        ba.pool_hi = p_hi[pcur];
        ba.pool_num = p_num;
        ba.pool_score = p_score[pcur];
        ba.pool_base = pool_n;
        ba.pool_cap = pool_cap;
        bucket_accumulate<W>(ba, ar, s, prof, hs);
        if (out.pt2) {
            out.pt2_energy = out.pt2_energy + bucket_pt2(ba, ar, s, hs);
            out.count += ba.V;
            continue;
        }
        int collect_tok = -1;
        if (early) {
            collect_tok = bucket_collect<W>(ba, s, prof);
            bucket_read_v(ba, s);
            if (prof) prof->set_bytes(collect_tok, (8.0 * W + 8.0) * 2.0 * ba.V);
        }
        const uint32_t V = ba.V;
        ctx->last_finals += ba.nfinal;
        ctx->last_levels = std::max<int64_t>(ctx->last_levels, ba.levels);
        ctx->last_candidates += V;
        if (!early) {
            if (topk && pool_n + V > pool_cap) prune((size_t)std::min<uint64_t>(pool_n, (uint64_t)out.k));
            if (pool_n + V > pool_cap)
                throw Error{ASCI_ENOMEM, "candidate pool overflow: pool " + std::to_string(pool_n) + " + batch " +
                                             std::to_string(V) + " > capacity " + std::to_string(pool_cap) +
                                             " (batch pairs " + std::to_string(P) + ", finals " +
                                             std::to_string(ba.nfinal) + ", max batch " + std::to_string(Pb) + ")"};
            ba.pool_lo = p_lo[pcur];
            ba.pool_hi = p_hi[pcur];
            ba.pool_num = p_num;
            ba.pool_score = p_score[pcur];
            ba.pool_base = pool_n;
            ba.pool_cap = pool_cap;
            bucket_collect<W>(ba, s, prof);
        }
        pool_n += V;
        if (topk && bi + 1 < batches.size() && pool_n > (uint64_t)out.k) {
            prune((size_t)out.k);
            d_thr = &d_sel->prefix;
        }
    }

    ar.reset();
    (void)ar.take<char>(loop_mark);
    if (out.pt2) {
        finish();
        return;
    }
    if (!topk) {
        out.count = (int64_t)pool_n;
        if (pool_n > (size_t)out.capacity) {  // the caller reports ENOMEM
            finish();
            return;
        }
        if (pool_n) {
            k_unpack<W><<<grid_for(pool_n), kBlock, 0, s>>>(p_lo[pcur], p_hi[pcur], pool_n, n, out.out_dets);
            ASCI_LAUNCH_CHECK();
            ASCI_HIP(hipMemcpyAsync(out.out_num, p_num, pool_n * sizeof(double), hipMemcpyDeviceToDevice, s));
            ASCI_HIP(hipMemcpyAsync(out.out_scores, p_score[pcur], pool_n * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        finish();
        return;
    }
    // step 10: the k largest |A| (ties: smaller key), then |A| descending
    const size_t kk = (size_t)std::min<uint64_t>((uint64_t)out.k, pool_n);
    out.count = (int64_t)kk;
    if (kk == 0) {
        finish();
        return;
    }
    if (kk < pool_n) prune(kk);
    {
        uint64_t *fk[2] = {ar.take<uint64_t>(kk), ar.take<uint64_t>(kk)};
        uint32_t *fi[2] = {ar.take<uint32_t>(kk), ar.take<uint32_t>(kk)};
        uint64_t *nohi[2] = {nullptr, nullptr};
        k_final_keys<<<grid_for(kk), kBlock, 0, s>>>(p_score[pcur], kk, fk[0], fi[0], nullptr);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> fd;
        for (int sh = 0; sh < 64; sh += 8) fd.push_back({0, sh});
        const int rr = radix_sort<uint32_t>(fk, nohi, fi, kk, 1, fd, ar, s, prof);
        k_final_gather<W><<<grid_for(kk), kBlock, 0, s>>>(fi[rr], kk, p_lo[pcur], p_hi[pcur], p_score[pcur], n,
                                                          out.out_dets, out.out_scores, nullptr, nullptr);
        ASCI_LAUNCH_CHECK();
    }
    finish();
}

// ---------------------------------------------------------------- the search with nothing read back
namespace {

// class c of level L in ascending mask order: the c-th L-subset (colex rank)
// of the orbitals na - L .. n - 1, unranked in the combinatorial number system
__global__ __launch_bounds__(kBlock) void k_class_masks(uint64_t *__restrict__ cls, uint32_t ncls, int n, int na,
                                                        int L)
{
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncls) return;
    uint64_t m = 0;
    uint32_t r = c;
    int x = n - na + L - 1;
    for (int j = L; j >= 1; --j) {
        while (x > 0 && choose_le6((uint32_t)x, j) > r) --x;
        m |= 1ull << (x + na - L);
        r -= choose_le6((uint32_t)x, j);
        --x;
    }
    cls[c] = m;
}

// C(p, k) for k < rows, p <= n, saturated at 2^32 - 1; rows past kmax are zero
__global__ __launch_bounds__(64) void k_binom_table(uint32_t *__restrict__ out, int n, int kmax, int rows)
{
    if (threadIdx.x != 0) return;
    // Pascal's rule row by row over p (64-bit, saturating)
    uint64_t prev[65], cur[65];
    for (int k = 0; k <= 64; ++k) prev[k] = k == 0 ? 1ull : 0ull;  // p = 0
    for (int p = 0; p <= n; ++p) {
        if (p > 0) {
            cur[0] = 1ull;
            for (int k = 1; k <= 64; ++k) {
                const uint64_t v = prev[k - 1] + prev[k];
                cur[k] = v > 0xFFFFFFFFull ? 0xFFFFFFFFull : v;
            }
            for (int k = 0; k <= 64; ++k) prev[k] = cur[k];
        }
        for (int k = 0; k < rows; ++k) out[(size_t)k * (n + 1) + p] = k <= kmax ? (uint32_t)prev[k] : 0u;
    }
}

// *dst = min(k, *n)
__global__ __launch_bounds__(64) void k_min_count(const uint32_t *__restrict__ n, uint64_t k, uint32_t *__restrict__ dst)
{
    if (threadIdx.x == 0) *dst = (uint32_t)min((uint64_t)*n, k);
}

// the validation flags of the setup arena folded into the status word
__global__ __launch_bounds__(64) void k_stat_or(const unsigned int *__restrict__ err, uint32_t *__restrict__ stat)
{
    if (threadIdx.x == 0 && *err)
        atomicOr(stat, (*err & (kStatInvalid | kStatDuplicate)) | ((*err & 4u) ? kStatIntegrals : 0u));
}

__global__ __launch_bounds__(64) void k_async_done(const uint32_t *__restrict__ stat, const uint32_t *__restrict__ kk,
                                                   asci_async_result *__restrict__ res)
{
    if (threadIdx.x != 0) return;
    const uint32_t f = *stat;
    res->flags = (int32_t)f;
    res->status = f == 0u ? ASCI_OK
                          : ((f & (kStatInvalid | kStatDuplicate | kStatIntegrals)) ? ASCI_EINVAL : ASCI_EDEVICE);
    res->count = f == 0u ? (int64_t)*kk : 0;
}

}  // namespace

template <int W>
static void run_search_async(asci_ctx *ctx, const SearchArgs &in, int64_t k, uint64_t *out_dets, double *out_scores,
                             asci_async_result *d_result, hipStream_t s, bool plan_only)
{
    const int n = in.n, na = in.na, nb = in.nb;
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const BetaFactors bf = beta_factors(n, nb);
    const size_t nd = (size_t)in.ndets;
    const size_t nq = (in.opt.ncore > 0 && (size_t)in.opt.ncore < nd) ? (size_t)in.opt.ncore : nd;
    const uint64_t P = search_pairs(in);
    // the requested level, or the highest lower one whose classes fit one batch
    // (the classes only partition the targets: the result is the same)
    int L = std::min(in.opt.constraint_level, na);
    while (L > 0 && choose_u64((uint64_t)(n - na + L), L) > kMaxBatchClasses) --L;
    const uint64_t ncls = std::max<uint64_t>(choose_u64((uint64_t)(n - na + L), L), 1);
    require(in.opt.split_pairs == 0, ASCI_EINVAL, "asynchronous search: split_pairs needs class totals on the host");
    require(P >= 1 && P < (1ull << 31), ASCI_EINVAL, "asynchronous search: pair count outside one class batch");
    const size_t rec_bytes = 2 * (8 * W + 8);
    if (in.opt.pair_buffer_bytes > 0)
        require(P <= (uint64_t)in.opt.pair_buffer_bytes / rec_bytes, ASCI_EINVAL,
                "asynchronous search: the pair buffer does not hold every pair");
    const size_t E = (size_t)ncls * nq;
    require(E < (1ull << 31), ASCI_ENOMEM, "batch (class x core) matrix too large");
    const size_t Pb = (size_t)P;
    const size_t pool_cap = Pb + 1;
    const uint64_t kh = std::min<uint64_t>((uint64_t)k, P);  // a bound on the selection's size

    // ---- workspaces (allocated only when larger than what ctx holds)
    Arena &su = ctx->setup;
    su.reset();
    su.reserve(setup_bytes(nd, nq, n, W));
    su.reset();
    Arena &ar = ctx->main;
    ar.reset();
    const SpinTablePlan pl = spin_table_plan(n, na, nb, P, ctx->spin_tables != 0);
    // the bound of the one-batch search, the tables, and the collect's sort of
    // final segments sized for their bound instead of their count
    const int fcap = effective_finish_cap(ctx, n, na, P);
    ar.reserve(main_bytes(E, Pb, pool_cap, (uint32_t)ncls, (size_t)kh, true, W, fcap) + pl.bytes + Pb / 4 +
               ((size_t)16 << 20));
    ar.reset();
    if (plan_only) return;  // workspaces sized, nothing queued

    // ---- inputs: validation (flags on the device), integral tables, psi set, core set, class masks
    unsigned int *d_err = su.take<unsigned int>(16);
    uint64_t *d_cls = su.take<uint64_t>(kMaxClasses);
    (void)su.take<unsigned long long>(kMaxClasses);
    (void)su.take<uint32_t>(kMaxClasses);
    double *d_jk = su.take<double>((size_t)2 * n * n + n);
    double *d_eri8 = su.take<double>(eri_packed_count(n));
    uint64_t *q_a = su.take<uint64_t>(nq), *q_b = su.take<uint64_t>(nq);
    double *q_c = su.take<double>(nq);
    uint32_t tsize = 1024;
    while (tsize < 4 * nd) tsize <<= 1;
    uint64_t *t_lo = su.take<uint64_t>(tsize), *t_hi = su.take<uint64_t>(tsize);
    uint32_t *t_state = su.take<uint32_t>(tsize);
    size_t fbits = (size_t)1 << 16;
    while (fbits < 32 * nd && fbits < ((size_t)1 << 34)) fbits <<= 1;
    unsigned long long *t_filter = su.take<unsigned long long>(fbits / 64);
    PsiSet psi;
    psi.lo = t_lo;
    psi.hi = t_hi;
    psi.state = t_state;
    psi.mask = tsize - 1;
    psi.filter = t_filter;
    psi.fmask = (uint32_t)(fbits / 64 - 1);
    uint32_t *d_stat = ar.take<uint32_t>(16);  // [0] status bits, [1] selection size
    fill_u32(d_stat, 16, 0u, s);
    fill_u32((uint32_t *)d_err, 16, 0u, s);
    k_fault_reset<<<1, 64, 0, s>>>();
    bucket_fault_reset_dev(s);
    k_validate<<<grid_for(nd), kBlock, 0, s>>>(in.dets, nd, full, na, nb, d_err);
    ASCI_LAUNCH_CHECK();
    k_jk<<<grid_for((size_t)n * n), kBlock, 0, s>>>(in.eri, in.h, n, d_jk);
    ASCI_LAUNCH_CHECK();
    {
        const size_t n4 = (size_t)n * n * n * n;
        k_eri_pack<<<grid_for(n4), kBlock, 0, s>>>(in.eri, n, d_eri8);
        ASCI_LAUNCH_CHECK();
        k_eri_check<<<grid_for(n4), kBlock, 0, s>>>(in.eri, n, d_eri8, d_err);
        ASCI_LAUNCH_CHECK();
    }
    fill_u32(t_state, tsize, 0u, s);
    fill_u32((uint32_t *)t_filter, fbits / 32, 0u, s);
    k_psi_insert<W><<<grid_for(nd), kBlock, 0, s>>>(in.dets, nd, n, t_lo, t_hi, t_state, tsize - 1, t_filter, psi.fmask);
    ASCI_LAUNCH_CHECK();
    k_psi_dups<W><<<grid_for(nd), kBlock, 0, s>>>(in.dets, nd, n, psi, d_err);
    ASCI_LAUNCH_CHECK();
    k_stat_or<<<1, 64, 0, s>>>(d_err, d_stat);
    ASCI_LAUNCH_CHECK();
    if (nq < nd) {
        uint64_t *ck[2] = {su.take<uint64_t>(nd), su.take<uint64_t>(nd)};
        uint32_t *ci[2] = {su.take<uint32_t>(nd), su.take<uint32_t>(nd)};
        uint64_t *nohi[2] = {nullptr, nullptr};
        k_core_keys<<<grid_for(nd), kBlock, 0, s>>>(in.coeffs, nd, ck[0], ci[0]);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> cd;
        for (int sh = 0; sh < 64; sh += 8) cd.push_back({0, sh});
        const int r1 = radix_sort<uint32_t>(ck, nohi, ci, nd, 1, cd, su, s);
        uint64_t *ik[2] = {ck[r1 ^ 1], su.take<uint64_t>(nq)};
        uint32_t *ii[2] = {ci[r1 ^ 1], su.take<uint32_t>(nq)};
        k_index_keys<<<grid_for(nq), kBlock, 0, s>>>(ci[r1], nq, ik[0]);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> id;
        for (int sh = 0; sh < 32; sh += 8) id.push_back({0, sh});
        const int r2 = radix_sort<uint32_t>(ik, nohi, ii, nq, 1, id, su, s);
        k_gather_core<<<grid_for(nq), kBlock, 0, s>>>(in.dets, in.coeffs, ik[r2], nq, q_a, q_b, q_c);
    } else {
        k_gather_core<<<grid_for(nq), kBlock, 0, s>>>(in.dets, in.coeffs, nullptr, nq, q_a, q_b, q_c);
    }
    ASCI_LAUNCH_CHECK();
    k_class_masks<<<grid_for(ncls), kBlock, 0, s>>>(d_cls, (uint32_t)ncls, n, na, L);
    ASCI_LAUNCH_CHECK();

    // ---- spin-string tables (binomials built on the device)
    SpinTables st;
    if (pl.bytes) {
        uint32_t *d_binom = ar.take<uint32_t>((size_t)(pl.kmax + 4) * (n + 1));
        k_binom_table<<<1, 64, 0, s>>>(d_binom, n, pl.kmax, pl.kmax + 4);
        ASCI_LAUNCH_CHECK();
        st.binom = d_binom;
        st.kmax = pl.kmax;
        const int ne[2] = {na, nb};
        for (int i = 0; i < 2; ++i) {
            if (pl.count[i] == 0) continue;
            if (i == 1 && pl.share) {
                st.e[1] = st.e[0];
                continue;
            }
            double *t = ar.take<double>(pl.count[i]);
            k_spin_table<<<(unsigned)((pl.count[i] + kBlock - 1) / kBlock), kBlock, 0, s>>>(d_jk, n, ne[i], d_binom,
                                                                                        (uint32_t)pl.count[i], t);
            ASCI_LAUNCH_CHECK();
            st.e[i] = t;
        }
    }

    // ---- count matrix, record offsets, generation (one batch: every class)
    uint32_t *counts = ar.take<uint32_t>(E);
    uint32_t *offs = ar.take<uint32_t>(E);
    uint64_t *k_lo[2] = {ar.take<uint64_t>(Pb), ar.take<uint64_t>(Pb)};
    uint64_t *k_hi[2] = {W == 2 ? ar.take<uint64_t>(Pb) : nullptr, W == 2 ? ar.take<uint64_t>(Pb) : nullptr};
    double *v[2] = {ar.take<double>(Pb), ar.take<double>(Pb)};
    uint64_t *c_lo = ar.take<uint64_t>(Pb);
    uint64_t *c_hi = W == 2 ? ar.take<uint64_t>(Pb) : nullptr;
    double *c_score = ar.take<double>(Pb);
    uint64_t *p_lo[2] = {ar.take<uint64_t>(pool_cap), ar.take<uint64_t>(pool_cap)};
    uint64_t *p_hi[2] = {W == 2 ? ar.take<uint64_t>(pool_cap) : nullptr, W == 2 ? ar.take<uint64_t>(pool_cap) : nullptr};
    double *p_score[2] = {ar.take<double>(pool_cap), ar.take<double>(pool_cap)};
    SelectState *d_sel = ar.take<SelectState>(1);
    uint32_t *d_cnt = ar.take<uint32_t>(16);
    const ClassMap cmap{L, na, nullptr};
    {
        dim3 g((unsigned)((nq + kBlock - 1) / kBlock), (unsigned)ncls);
        k_count<<<g, kBlock, 0, s>>>(q_a, (uint32_t)nq, d_cls, 0u, full, bf, counts, nullptr);
        ASCI_LAUNCH_CHECK();
    }
    scan_u32(counts, offs, E, d_cnt + 2, ar, s, nullptr);
    {
        GenArgs ga;
        ga.core_a = q_a;
        ga.core_b = q_b;
        ga.core_c = q_c;
        ga.nq = (uint32_t)nq;
        ga.c0 = 0;
        ga.nc = (uint32_t)ncls;
        ga.nbits = 1;
        while ((1u << ga.nbits) < ga.nc) ++ga.nbits;
        ga.offsets = offs;
        ga.h = in.h;
        ga.eri8 = d_eri8;
        ga.n = n;
        ga.na = na;
        ga.nb = nb;
        ga.cmap = cmap;
        ga.full = full;
        const uint32_t va = (uint32_t)(n - na), vb = (uint32_t)(n - nb);
        ga.nas = (uint32_t)na * va;
        ga.nbs = (uint32_t)nb * vb;
        ga.f0 = bf.f[0];
        ga.f1 = bf.f[1];
        ga.pva2 = va * (va - (va ? 1u : 0u)) / 2u;
        ga.npa2 = (uint32_t)na * (uint32_t)(na - (na ? 1 : 0)) / 2u;
        ga.pvb2 = bf.pairs_vb;
        ga.npb2 = (uint32_t)nb * (uint32_t)(nb - (nb ? 1 : 0)) / 2u;
        ga.klo = k_lo[0];
        ga.khi = k_hi[0];
        ga.vals = v[0];
        ga.cap = Pb;
        ga.force_fault = ctx->fault_test;
        const size_t lds = (size_t)ga.nas * (8 + 4 + 4 + 4) + (size_t)ga.nbs * 4 + (size_t)ga.nc * 4 + 256 +
                           2 * ((size_t)2 * ga.npa2 + ga.pva2 + ga.npb2 + ga.pvb2) + 4 * (size_t)ga.npa2 + 68;
        k_generate<W><<<(unsigned)(8 * ((nq + 7) / 8)), 64, lds, s>>>(ga);
        ASCI_LAUNCH_CHECK();
    }

    // ---- sort and accumulate, exclusion, diagonal and score (device-driven)
    BucketArgs ba;
    ba.P = Pb;
    ba.c0 = 0;
    ba.nc = (uint32_t)ncls;
    ba.nq = (uint32_t)nq;
    ba.n = n;
    ba.cls = d_cls;
    ba.offsets = offs;
    ba.total = d_cnt + 2;
    ba.klo[0] = k_lo[0];
    ba.klo[1] = k_lo[1];
    ba.khi[0] = k_hi[0];
    ba.khi[1] = k_hi[1];
    ba.val[0] = v[0];
    ba.val[1] = v[1];
    ba.psi = psi;
    ba.jk = d_jk;
    ba.h = in.h;
    ba.st = st;
    ba.thr = nullptr;
    ba.ecore = in.opt.ecore;
    ba.E0 = in.E0;
    ba.eps = in.opt.eps;
    ba.finish_cap = fcap;
    ba.clo = c_lo;
    ba.chi = c_hi;
    ba.cnum = nullptr;
    ba.cscore = c_score;
    ba.pool_lo = p_lo[0];
    ba.pool_hi = p_hi[0];
    ba.pool_num = nullptr;
    ba.pool_score = p_score[0];
    ba.pool_base = 0;
    ba.pool_cap = pool_cap;
    bucket_accumulate_dev<W>(ba, ar, s, d_stat);
    bucket_collect_dev<W>(ba, s);
    const uint32_t *d_V = ba.dn_V;

    // ---- the k largest |A| (ties: smaller key), then |A| descending
    uint32_t *d_kk = d_stat + 1;
    k_min_count<<<1, 64, 0, s>>>(d_V, (uint64_t)k, d_kk);
    ASCI_LAUNCH_CHECK();
    radix_select_abs(p_score[0], Pb, kh, d_sel, s, nullptr, nullptr, d_V, d_kk);
    const uint32_t ntile = (uint32_t)((Pb + kKeepTile - 1) / kKeepTile);
    uint32_t *tgt = ar.take<uint32_t>(ntile), *teq = ar.take<uint32_t>(ntile);
    uint32_t *eqb = ar.take<uint32_t>(ntile), *kbs = ar.take<uint32_t>(ntile);
    k_keep_count<<<ntile, kBlock, 0, s>>>(p_score[0], Pb, d_sel, tgt, teq, d_V);
    ASCI_LAUNCH_CHECK();
    k_keep_bases<<<1, 1024, 0, s>>>(tgt, teq, ntile, d_sel, eqb, kbs);
    ASCI_LAUNCH_CHECK();
    k_keep_scatter<W><<<ntile, kBlock, 0, s>>>(p_lo[0], p_hi[0], p_score[0], Pb, d_sel, eqb, kbs, p_lo[1], p_hi[1],
                                               p_score[1], (size_t)kh, d_V);
    ASCI_LAUNCH_CHECK();
    {
        uint64_t *fk[2] = {ar.take<uint64_t>(kh), ar.take<uint64_t>(kh)};
        uint32_t *fi[2] = {ar.take<uint32_t>(kh), ar.take<uint32_t>(kh)};
        uint64_t *nohi[2] = {nullptr, nullptr};
        k_final_keys<<<grid_for(kh), kBlock, 0, s>>>(p_score[1], kh, fk[0], fi[0], d_kk);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> fd;
        for (int sh = 0; sh < 64; sh += 8) fd.push_back({0, sh});
        const int rr = radix_sort<uint32_t>(fk, nohi, fi, kh, 1, fd, ar, s, nullptr, d_kk);
        // every fault raised so far fails the call before any output is written
        k_fault_take<<<1, 64, 0, s>>>(d_stat, kStatFault);
        ASCI_LAUNCH_CHECK();
        bucket_fault_take_dev(d_stat, kStatFault, s);
        k_final_gather<W><<<grid_for(kh), kBlock, 0, s>>>(fi[rr], kh, p_lo[1], p_hi[1], p_score[1], n, out_dets,
                                                          out_scores, d_kk, d_stat);
        ASCI_LAUNCH_CHECK();
    }
    k_async_done<<<1, 64, 0, s>>>(d_stat, d_kk, d_result);
    ASCI_LAUNCH_CHECK();
}

void search_async(asci_ctx *ctx, const SearchArgs &in, int64_t k, uint64_t *out_dets, double *out_scores,
                  asci_async_result *d_result, hipStream_t s, bool plan_only)
{
    require(k >= 1, ASCI_EINVAL, "k must be >= 1");
    if (in.n <= 32) run_search_async<1>(ctx, in, k, out_dets, out_scores, d_result, s, plan_only);
    else run_search_async<2>(ctx, in, k, out_dets, out_scores, d_result, s, plan_only);
}

size_t search_async_bytes(const SearchArgs &in, int64_t k, int finish_cap, bool spin_tables)
{
    const int n = in.n, na = in.na, W = n <= 32 ? 1 : 2;
    const size_t nd = (size_t)in.ndets;
    const size_t nq = (in.opt.ncore > 0 && (size_t)in.opt.ncore < nd) ? (size_t)in.opt.ncore : nd;
    const uint64_t P = search_pairs(in);
    if (in.opt.split_pairs != 0 || P < 1 || P >= (1ull << 31) || k < 1) return 0;
    if (in.opt.pair_buffer_bytes > 0 && P > (uint64_t)in.opt.pair_buffer_bytes / (2 * (8 * W + 8))) return 0;
    int L = std::min(in.opt.constraint_level, na);
    while (L > 0 && choose_u64((uint64_t)(n - na + L), L) > kMaxBatchClasses) --L;
    const uint64_t ncls = std::max<uint64_t>(choose_u64((uint64_t)(n - na + L), L), 1);
    if ((size_t)ncls * nq >= (1ull << 31)) return 0;
    const uint64_t kh = std::min<uint64_t>((uint64_t)k, P);
    const SpinTablePlan pl = spin_table_plan(n, na, in.nb, P, spin_tables);
    return setup_bytes(nd, nq, n, W) + main_bytes((size_t)ncls * nq, (size_t)P, (size_t)P + 1, (uint32_t)ncls,
                                                  (size_t)kh, true, W, finish_cap) +
           pl.bytes + (size_t)P / 4 + ((size_t)16 << 20);
}

size_t search_scratch_bound(const SearchArgs &in, int64_t k, int finish_cap, size_t &setup_part)
{
    const int W = in.n <= 32 ? 1 : 2;
    const size_t nd = (size_t)in.ndets;
    const size_t nq = (in.opt.ncore > 0 && (size_t)in.opt.ncore < nd) ? (size_t)in.opt.ncore : nd;
    const BetaFactors bf = beta_factors(in.n, in.nb);
    const uint64_t va = (uint64_t)(in.n - in.na);
    const uint64_t per = (uint64_t)in.na * va + choose_u64((uint64_t)in.na, 2) * choose_u64(va, 2) +
                         (uint64_t)bf.f[0] + (uint64_t)in.na * va * (uint64_t)(bf.f[1] - 1u);
    const uint64_t P = std::max<uint64_t>(per * nq, 1);
    const int L = std::min(in.opt.constraint_level, in.na);
    const uint64_t ncls = std::max<uint64_t>(choose_u64((uint64_t)(in.n - in.na + L), L), 1);
    const size_t E = (size_t)std::min<uint64_t>(ncls, kMaxBatchClasses) * nq;
    const size_t pool_cap = k > 0 ? (size_t)std::min<uint64_t>(P + 1, std::max<uint64_t>(4 * (uint64_t)k, P) + (uint64_t)k)
                                  : (size_t)P + 1;
    const size_t kk = k > 0 ? (size_t)std::min<uint64_t>((uint64_t)k, pool_cap) : 0;
    setup_part = (setup_bytes(nd, nq, in.n, W) + 255) & ~size_t(255);
    return setup_part + main_bytes(E, (size_t)P, pool_cap, (uint32_t)std::min<uint64_t>(ncls, kMaxBatchClasses), kk,
                                   k > 0, W, finish_cap);
}

uint64_t search_pairs(const SearchArgs &in)
{
    const BetaFactors bf = beta_factors(in.n, in.nb);
    const uint64_t va = (uint64_t)(in.n - in.na);
    const size_t nd = (size_t)in.ndets;
    const size_t nq = (in.opt.ncore > 0 && (size_t)in.opt.ncore < nd) ? (size_t)in.opt.ncore : nd;
    return ((uint64_t)in.na * va + choose_u64((uint64_t)in.na, 2) * choose_u64(va, 2) + (uint64_t)bf.f[0] +
            (uint64_t)in.na * va * (uint64_t)(bf.f[1] - 1u)) * nq;
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
                         int64_t ndets, const asci_options &opt, std::vector<uint64_t> &masks,
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
    const uint64_t no_fit = ~0ull;
    if (n <= 32) {
        Prepared<1> pp;
        prepare<1>(ctx, nullptr, nullptr, n, na, nb, dets, coeffs, ndets, opt, no_fit, false, pp, s);
        collect(pp.cls, pp.totals);
    } else {
        Prepared<2> pp;
        prepare<2>(ctx, nullptr, nullptr, n, na, nb, dets, coeffs, ndets, opt, no_fit, false, pp, s);
        collect(pp.cls, pp.totals);
    }
}

}  // namespace asci
