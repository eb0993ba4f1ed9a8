// Slater-Condon matrix elements on 64-bit occupation strings (device side).
//
// Phase convention: spin orbitals alpha first then beta, ascending; a^+_q a_p
// on a determinant has sign (-1)^(occupied orbitals of that spin strictly
// between p and q).  Integrals: h[p*n+q], eri[((p*n+q)*n+r)*n+s] = (pq|rs).
// Sums run in ascending orbital order and the library is built without
// floating-point contraction, so every value is reproducible bit for bit.
#pragma once

#include "asci_internal.h"

namespace asci {

// Internal-consistency faults of this translation unit's kernels, one bit per
// kind.  Only a logic error sets them: a record whose slot lies past its
// buffer (the counts and offsets disagree with what a kernel writes), or an
// orbital index outside the string width.  The write is dropped (or the index
// clamped) so that no access leaves its buffer, the bit records it, and the
// host fails the call with ASCI_EDEVICE after reading the word (fault_fetch).
// The word is per device and per translation unit; calls running at once on
// one device may see each other's faults.
constexpr unsigned kFaultSlot = 1u;     // a write past the end of its buffer was dropped
constexpr unsigned kFaultOrbital = 2u;  // an orbital index >= norb was clamped
constexpr unsigned kFaultForced = 4u;   // raised on request (tests of the error path)
static __device__ unsigned int g_fault;

__device__ __forceinline__ void raise_fault(unsigned f) { atomicOr(&g_fault, f); }

// Orbital indices come from validated bit strings; an index out of range is a
// logic error, clamped so that it cannot turn into an out-of-bounds load.
__device__ __forceinline__ int orb(int p, int n)
{
    if ((unsigned)p >= (unsigned)n) {
        raise_fault(kFaultOrbital);
        return n - 1;
    }
    return p;
}

// Host side: clear the word (queued on s), and queue its copy to pinned host
// memory *dst (valid once s has been synchronised).
static inline void fault_clear(hipStream_t s)
{
    void *p = nullptr;
    ASCI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_fault)));
    ASCI_HIP(hipMemsetAsync(p, 0, sizeof(unsigned int), s));
}

static inline void fault_fetch(unsigned int *dst, hipStream_t s)
{
    void *p = nullptr;
    ASCI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_fault)));
    ASCI_HIP(hipMemcpyAsync(dst, p, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
}

// The same word handled on the device (no host readback): cleared by a kernel
// (a fill that a captured graph replays correctly), and folded into a status
// word at the end of a call.
namespace {
__global__ __launch_bounds__(64) void k_fault_reset()
{
    if (threadIdx.x == 0) atomicAnd(&g_fault, 0u);
}
__global__ __launch_bounds__(64) void k_fault_take(uint32_t *stat, uint32_t bit)
{
    if (threadIdx.x == 0 && atomicOr(&g_fault, 0u) != 0u) atomicOr(stat, bit);
}
}  // namespace

// after the stream has been synchronised: fail on any recorded fault
static inline void fault_check(unsigned int word, const char *where)
{
    if (word)
        throw Error{ASCI_EDEVICE, std::string("internal consistency fault in ") + where + ": " +
                                      ((word & kFaultSlot) ? "a record slot past its buffer; " : "") +
                                      ((word & kFaultOrbital) ? "an orbital index out of range; " : "") +
                                      ((word & kFaultForced) ? "forced by the fault_test parameter" : "")};
}

// n <= 64, so the flat index (below 64^4) fits 32-bit arithmetic
__device__ __forceinline__ double eri4(const double *__restrict__ eri, int n, int p, int q, int r, int s)
{
    const uint32_t un = (uint32_t)n;
    return eri[(((uint32_t)orb(p, n) * un + (uint32_t)orb(q, n)) * un + (uint32_t)orb(r, n)) * un +
               (uint32_t)orb(s, n)];
}

// The integrals behind an accessor E(p, q, r, s) = (pq|rs): the full n^4
// tensor, or its 8-fold packed form.  Packed: pair indices pq = tri(p, q) and
// rs = tri(r, s), then tri(pq, rs), with tri(a, b) = max(a,b)(max(a,b)+1)/2 +
// min(a,b); 8-fold symmetric integrals give the same value either way (the
// search checks that they are, bit for bit, before it reads the packed form).
__device__ __forceinline__ uint32_t tri(uint32_t a, uint32_t b)
{
    return a >= b ? a * (a + 1u) / 2u + b : b * (b + 1u) / 2u + a;
}

struct EriFull {
    const double *__restrict__ e;
    int n;
    __device__ __forceinline__ double operator()(int p, int q, int r, int s) const { return eri4(e, n, p, q, r, s); }
};

struct EriPacked {
    const double *__restrict__ e;
    int n;
    __device__ __forceinline__ double operator()(int p, int q, int r, int s) const
    {
        uint32_t up = (uint32_t)p, uq = (uint32_t)q, ur = (uint32_t)r, us = (uint32_t)s;
        // one range test for the four indices (orb's clamp and fault, taken together)
        if (max(max(up, uq), max(ur, us)) >= (uint32_t)n) {
            raise_fault(kFaultOrbital);
            const uint32_t m = (uint32_t)n - 1u;
            up = min(up, m);
            uq = min(uq, m);
            ur = min(ur, m);
            us = min(us, m);
        }
        return e[tri(tri(up, uq), tri(ur, us))];
    }
    // the entry at pair indices pq = tri(p, q), rs = tri(r, s), for callers
    // whose orbitals come from the lists a kernel builds out of a validated
    // string's bits (every index below n by construction, so no range test)
    __device__ __forceinline__ double pairs(uint32_t pq, uint32_t rs) const { return e[tri(pq, rs)]; }
    __device__ __forceinline__ double listed(int p, int q, int r, int s) const
    {
        return pairs(tri((uint32_t)p, (uint32_t)q), tri((uint32_t)r, (uint32_t)s));
    }
};

// the packed integrals read through `listed` (orbitals from validated lists)
struct EriListed {
    EriPacked e;
    __device__ __forceinline__ double operator()(int p, int q, int r, int s) const { return e.listed(p, q, r, s); }
};

// entries of the packed form of n orbitals
inline size_t eri_packed_count(int n)
{
    const size_t npp = (size_t)n * (n + 1) / 2;
    return npp * (npp + 1) / 2;
}

// <a|H|i> for a single p -> q in the spin string `same` of i; `other` is the
// other spin string of i:
//   sign * ( h_qp + sum_{r in same, r != p} [(qp|rr) - (qr|rp)] + sum_{r in other} (qp|rr) )
template <class E>
__device__ __forceinline__ double single_value_e(const double *__restrict__ h, const E &eri, int n, uint64_t same,
                                                 uint64_t other, int p, int q)
{
    double v = h[(size_t)orb(q, n) * n + orb(p, n)];
    for (uint64_t m = same & ~(1ull << p); m; m &= m - 1ull) {
        const int r = lowbit(m);
        v = v + (eri(q, p, r, r) - eri(q, r, r, p));
    }
    for (uint64_t m = other; m; m &= m - 1ull) {
        const int r = lowbit(m);
        v = v + eri(q, p, r, r);
    }
    return between_sign(same, p, q) * v;
}

__device__ __forceinline__ double single_value(const double *__restrict__ h, const double *__restrict__ eri, int n,
                                               uint64_t same, uint64_t other, int p, int q)
{
    return single_value_e(h, EriFull{eri, n}, n, same, other, p, q);
}

// same-spin double: holes p < r (in string si), particles q < s
//   sign(p->q on si) * sign(r->s on si') * [(qp|sr) - (qr|sp)]
template <class E>
__device__ __forceinline__ double double_same_value_e(const E &eri, int n, uint64_t si, uint64_t holes,
                                                      uint64_t parts)
{
    const int p = lowbit(holes), r = lowbit(holes & (holes - 1ull));
    const int q = lowbit(parts), s = lowbit(parts & (parts - 1ull));
    const int s1 = between_sign(si, p, q);
    const uint64_t mid = (si & ~(1ull << p)) | (1ull << q);
    const int s2 = between_sign(mid, r, s);
    return s1 * s2 * (eri(q, p, s, r) - eri(q, r, s, p));
}

__device__ __forceinline__ double double_same_value(const double *__restrict__ eri, int n, uint64_t si,
                                                    uint64_t holes, uint64_t parts)
{
    return double_same_value_e(EriFull{eri, n}, n, si, holes, parts);
}

// The same element times c, for holes p < r and particles q < s taken from
// validated orbital lists: the sign (+-1) is applied to [(qp|sr) - (qr|sp)] * c
// instead of before the product, which rounds to the same bits (negation is
// exact and rounding is symmetric in sign).
__device__ __forceinline__ double double_same_times(const EriPacked &eri, uint64_t si, int p, int r, int q, int s,
                                                    double c)
{
    const uint64_t mid = (si & ~(1ull << p)) | (1ull << q);
    const bool neg = between_sign(si, p, q) != between_sign(mid, r, s);
    const double v = (eri.listed(q, p, s, r) - eri.listed(q, r, s, p)) * c;
    return neg ? -v : v;
}

// opposite-spin double: alpha p -> q, beta r -> s: sign_a * sign_b * (qp|sr)
__device__ __forceinline__ double double_opp_value(const double *__restrict__ eri, int n, uint64_t ia,
                                                   uint64_t ib, int p, int q, int r, int s)
{
    const int sg = between_sign(ia, p, q) * between_sign(ib, r, s);
    return sg * eri4(eri, n, q, p, s, r);
}

// H_aa from the tables J[p*n+q] = (pp|qq), X[p*n+q] = (pp|qq) - (pq|qp) and
// hd[p] = h_pp, as ((ecore + E(alpha)) + E(beta)) + E(alpha, beta):
//   E(s)           = sum_{p in s} h_pp + sum_{p<q in s} X_pq (one running sum from 0)
//   E(alpha, beta) = sum_{q in beta} c_q(alpha),  c_q(alpha) = sum_{p in alpha} J_pq
// every sum ascending.  Grouping the opposite-spin term by beta orbital lets
// c_q(alpha) be computed once per alpha string and reused.  M is the string
// word type: a 32-bit word when every orbital fits in it.
__device__ __forceinline__ int tz(uint32_t m) { return __builtin_ctz(m); }
__device__ __forceinline__ int tz(uint64_t m) { return __builtin_ctzll(m); }

template <typename M>
__device__ __forceinline__ double spin_energy_m(const double *X, const double *hd, int n, M s)
{
    double e = 0.0;
    for (M m = s; m; m &= m - 1) e = e + hd[tz(m)];
    for (M m = s; m; m &= m - 1) {
        const double *row = X + tz(m) * n;
        for (M m2 = m & (m - 1); m2; m2 &= m2 - 1) e = e + row[tz(m2)];
    }
    return e;
}

// sum over the set bits p of m, ascending, of v(p): the adds run in that order
// from 0.0; the values are loaded four at a time (a spare slot loads v(0) and
// is not added), so their latencies overlap
template <typename M, typename F>
__device__ __forceinline__ double bit_sum(M m, F v)
{
    double s = 0.0;
    while (m) {
        double x[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ok[k] = m != 0;
            x[k] = v(ok[k] ? tz(m) : 0);
            m &= m - 1;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) s = ok[k] ? s + x[k] : s;
    }
    return s;
}

template <typename M>
__device__ __forceinline__ double cross_col_m(const double *J, int n, M a, int q)
{
    return bit_sum<M>(a, [&](int p) { return J[p * n + q]; });
}

template <typename M>
__device__ __forceinline__ double diag_value_m(const double *J, const double *X, const double *hd, int n,
                                               double ecore, M a, M b)
{
    double cross = 0.0;
    for (M m = b; m; m &= m - 1) cross = cross + cross_col_m<M>(J, n, a, tz(m));
    return ((ecore + spin_energy_m<M>(X, hd, n, a)) + spin_energy_m<M>(X, hd, n, b)) + cross;
}

__device__ __forceinline__ double diag_value(const double *J, const double *X, const double *hd, int n,
                                             double ecore, uint64_t a, uint64_t b)
{
    if (n <= 32) return diag_value_m<uint32_t>(J, X, hd, n, ecore, (uint32_t)a, (uint32_t)b);
    return diag_value_m<uint64_t>(J, X, hd, n, ecore, a, b);
}

__device__ __forceinline__ double spin_energy(const double *X, const double *hd, int n, uint64_t s)
{
    if (n <= 32) return spin_energy_m<uint32_t>(X, hd, n, (uint32_t)s);
    return spin_energy_m<uint64_t>(X, hd, n, s);
}

// E(alpha, beta) of the diagonal element: sum over q in beta of c_q(alpha)
__device__ __forceinline__ double cross_energy(const double *J, int n, uint64_t a, uint64_t b)
{
    if (n <= 32) {
        double cross = 0.0;
        for (uint32_t m = (uint32_t)b; m; m &= m - 1) cross = cross + cross_col_m<uint32_t>(J, n, (uint32_t)a, tz(m));
        return cross;
    }
    double cross = 0.0;
    for (uint64_t m = b; m; m &= m - 1) cross = cross + cross_col_m<uint64_t>(J, n, a, tz(m));
    return cross;
}

// combinatorial rank of a spin string: sum over its set bits p_1 < p_2 < ...
// of C(p_j, j), with binom[k * (n + 1) + p] = C(p, k)
// (four table loads in flight at a time; integer sums need no order)
template <typename M>
__device__ __forceinline__ uint32_t spin_rank_m(const uint32_t *binom, int n, M m)
{
    uint32_t r = 0;
    const uint32_t *row = binom + (n + 1);
    while (m) {
        // unconditional loads (a spare slot reads C(0, k) and adds nothing)
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool ok = m != 0;
            v[k] = row[k * (n + 1) + (ok ? tz(m) : 0)] & (ok ? ~0u : 0u);
            m &= m - 1;
        }
        r += (v[0] + v[1]) + (v[2] + v[3]);
        row += 4 * (n + 1);
    }
    return r;
}

__device__ __forceinline__ uint32_t spin_rank(const uint32_t *binom, int n, uint64_t s)
{
    if (n <= 32) return spin_rank_m<uint32_t>(binom, n, (uint32_t)s);
    return spin_rank_m<uint64_t>(binom, n, s);
}

__device__ __forceinline__ double cross_col(const double *J, int n, uint64_t a, int q)
{
    if (n <= 32) return cross_col_m<uint32_t>(J, n, (uint32_t)a, q);
    return cross_col_m<uint64_t>(J, n, a, q);
}

}  // namespace asci
