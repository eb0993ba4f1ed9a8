// Device primitives for the search: exclusive scan, stable LSD radix sort and
// radix selection.  Written for 64-wide wavefronts (gfx950): ranking inside a
// wave uses ballots, blocks are 256 threads (4 waves).
#include <type_traits>
#include "asci_internal.h"

namespace asci {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096
static_assert(kTile == kScanTile, "scan tile");

// a host bound on a count, tightened by the count on the device when given
__device__ __forceinline__ size_t dev_n(size_t n, const uint32_t *dn) { return dn ? min(n, (size_t)*dn) : n; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// exclusive scan across a block of NW waves; every thread must call it
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = wave_incl_scan(v);
    if (lane == 63) s_tmp[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint32_t t = s_tmp[i];
        base += (i < w) ? t : 0u;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return base + x - v;
}

// ---------------------------------------------------------------- scan
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ in, size_t n,
                                                          uint32_t *__restrict__ partial, const uint32_t *dn)
{
    __shared__ uint32_t s_tmp[kWaves];
    n = dev_n(n, dn);
    const size_t base = (size_t)blockIdx.x * kTile;
    uint32_t s = 0;
    if (base + kTile <= n && (reinterpret_cast<uintptr_t>(in) & 15u) == 0) {
        // a whole tile: 16-byte loads, coalesced across the block
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int i = 0; i < kTile / 4 / kThreads; ++i) {
            const uint4 q = p[i * kThreads + threadIdx.x];
            s += (q.x + q.y) + (q.z + q.w);
        }
    } else {
        for (int i = threadIdx.x; i < kTile; i += kThreads) {
            size_t j = base + i;
            if (j < n) s += in[j];
        }
    }
    uint32_t tot;
    block_excl_scan<kWaves>(s, s_tmp, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *__restrict__ partial, uint32_t np,
                                                        uint32_t *__restrict__ d_total)
{
    __shared__ uint32_t s_tmp[16];
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < np; c0 += 1024) {
        uint32_t j = c0 + threadIdx.x;
        uint32_t v = j < np ? partial[j] : 0u;
        uint32_t tot;
        uint32_t e = block_excl_scan<16>(v, s_tmp, tot);
        if (j < np) partial[j] = carry + e;
        carry += tot;
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

// short inputs (at most kScanSmall elements): one workgroup, one launch,
// chunks of 4096 scanned in turn with a running carry
constexpr size_t kScanSmall = 65536;
__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t *in, uint32_t *out, uint32_t n,
                                                     uint32_t *__restrict__ d_total, const uint32_t *dn)
{
    __shared__ uint32_t s_tmp[16];
    n = (uint32_t)dev_n(n, dn);
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += 4096) {
        const uint32_t j0 = c0 + threadIdx.x * 4u;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = j0 + i < n ? in[j0 + i] : 0u;
            sum += v[i];
        }
        uint32_t tot;
        uint32_t e = carry + block_excl_scan<16>(sum, s_tmp, tot);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (j0 + i < n) out[j0 + i] = e;
            e += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t *in, uint32_t *out, size_t n,
                                                        const uint32_t *__restrict__ partial, const uint32_t *dn)
{
    __shared__ uint32_t s_tmp[kWaves];
    n = dev_n(n, dn);
    const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kItems;
    // a whole tile with aligned ends moves each thread's 16 items as four
    // 16-byte words (the scan may run in place: every word is read before the
    // block's barrier and written after it)
    const bool full = (size_t)blockIdx.x * kTile + kTile <= n &&
                      ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
    uint32_t v[kItems];
    uint32_t s = 0;
    if (full) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int i = 0; i < kItems / 4; ++i) {
            const uint4 q = p[i];
            v[4 * i] = q.x;
            v[4 * i + 1] = q.y;
            v[4 * i + 2] = q.z;
            v[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            size_t j = base + i;
            v[i] = j < n ? in[j] : 0u;
        }
    }
#pragma unroll
    for (int i = 0; i < kItems; ++i) s += v[i];
    uint32_t tot;
    uint32_t e = block_excl_scan<kWaves>(s, s_tmp, tot) + partial[blockIdx.x];
    if (full) {
        uint4 *p = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int i = 0; i < kItems / 4; ++i) {
            uint4 q;
            q.x = e;
            e += v[4 * i];
            q.y = e;
            e += v[4 * i + 1];
            q.z = e;
            e += v[4 * i + 2];
            q.w = e;
            e += v[4 * i + 3];
            p[i] = q;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            size_t j = base + i;
            if (j < n) out[j] = e;
            e += v[i];
        }
    }
}

// ---------------------------------------------------------------- radix sort
template <int W>
__device__ __forceinline__ uint32_t digit_of(uint64_t lo, uint64_t hi, int word, int shift)
{
    uint64_t k = (W == 2 && word == 1) ? hi : lo;
    return (uint32_t)(k >> shift) & 0xFFu;
}

// IT records per thread: a tile of kThreads * IT records per workgroup (small
// sorts take small tiles, so that they still spread over the CUs)
template <int W, int IT>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ klo,
                                                      const uint64_t *__restrict__ khi, size_t n,
                                                      int word, int shift,
                                                      uint32_t *__restrict__ hist, uint32_t nblocks,
                                                      const uint32_t *dn)
{
    constexpr int TILE = kThreads * IT;
    n = dev_n(n, dn);
    __shared__ uint32_t h[kWaves][256];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int i = tid; i < kWaves * 256; i += kThreads) (&h[0][0])[i] = 0u;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * TILE;
    for (int i = tid; i < TILE; i += kThreads) {
        size_t j = base + i;
        if (j < n) {
            uint64_t lo = klo[j];
            uint64_t hi = (W == 2) ? khi[j] : 0ull;
            atomicAdd(&h[w][digit_of<W>(lo, hi, word, shift)], 1u);
        }
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) c += h[i][tid];
    hist[(size_t)tid * nblocks + blockIdx.x] = c;
}

// Stable scatter of one tile.  Tile order is (wave, slot, lane), which is the
// input index order, so equal digits keep their input order.
template <int W, typename V, int IT>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(
    const uint64_t *__restrict__ ilo, const uint64_t *__restrict__ ihi, const V *__restrict__ ival,
    uint64_t *__restrict__ olo, uint64_t *__restrict__ ohi, V *__restrict__ oval, size_t n, int word,
    int shift, const uint32_t *__restrict__ hist, uint32_t nblocks, const uint32_t *dn)
{
    constexpr int kTile = kThreads * IT, kItems = IT;
    n = dev_n(n, dn);
    __shared__ uint64_t s_lo[kTile];
    __shared__ uint64_t s_hi[W == 2 ? kTile : 1];
    __shared__ V s_val[kTile];
    __shared__ uint32_t s_wcnt[kWaves][256];
    __shared__ uint32_t s_dbase[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_tmp[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const size_t tile0 = (size_t)blockIdx.x * kTile;
    if (tile0 >= n) return;  // uniform: a tile past a device-side count
    for (int i = tid; i < kWaves * 256; i += kThreads) (&s_wcnt[0][0])[i] = 0u;
    __syncthreads();

    uint64_t rlo[kItems], rhi[kItems];
    V rv[kItems];
    uint32_t rrank[kItems];
    const uint64_t lt = (1ull << lane) - 1ull;
    const size_t wbase = tile0 + (size_t)w * 64 * kItems;
#pragma unroll
    for (int s = 0; s < kItems; ++s) {
        size_t j = wbase + (size_t)s * 64 + lane;
        bool valid = j < n;
        rlo[s] = valid ? ilo[j] : 0ull;
        rhi[s] = (W == 2 && valid) ? ihi[j] : 0ull;
        rv[s] = valid ? ival[j] : V(0);
        uint32_t d = digit_of<W>(rlo[s], rhi[s], word, shift);
        const uint64_t peers = wave_match(d, valid, 8);
        uint32_t before = s_wcnt[w][d];
        rrank[s] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0ull) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = tid;
        uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
        s_wcnt[0][d] = 0u;
        s_wcnt[1][d] = c0;
        s_wcnt[2][d] = c0 + c1;
        s_wcnt[3][d] = c0 + c1 + c2;
        uint32_t tot;
        s_dbase[d] = block_excl_scan<kWaves>(c0 + c1 + c2 + c3, s_tmp, tot);
        s_gbase[d] = hist[(size_t)d * nblocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kItems; ++s) {
        size_t j = wbase + (size_t)s * 64 + lane;
        if (j < n) {
            uint32_t d = digit_of<W>(rlo[s], rhi[s], word, shift);
            uint32_t pos = min(s_dbase[d] + s_wcnt[w][d] + rrank[s], (uint32_t)kTile - 1u);
            s_lo[pos] = rlo[s];
            if (W == 2) s_hi[pos] = rhi[s];
            s_val[pos] = rv[s];
        }
    }
    __syncthreads();
    const uint32_t tn = (uint32_t)((n - tile0) < (size_t)kTile ? (n - tile0) : (size_t)kTile);
    for (uint32_t i = tid; i < tn; i += kThreads) {
        uint64_t lo = s_lo[i];
        uint64_t hi = (W == 2) ? s_hi[i] : 0ull;
        uint32_t d = digit_of<W>(lo, hi, word, shift);
        size_t g = (size_t)s_gbase[d] + (i - s_dbase[d]);
        if (g < n) {
            olo[g] = lo;
            if (W == 2) ohi[g] = hi;
            oval[g] = s_val[i];
        }
    }
}

// ---------------------------------------------------------------- radix select
__global__ __launch_bounds__(kThreads) void k_sel_init(SelectState *st, uint64_t k, const uint32_t *dk)
{
    if (threadIdx.x == 0) {
        st->prefix = 0ull;
        st->mask = 0ull;
        st->krem = dk ? min(k, (uint64_t)*dk) : k;
    }
    st->hist[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(kThreads) void k_sel_hist(const double *__restrict__ score, size_t n,
                                                       int shift, SelectState *st, const uint32_t *dn)
{
    __shared__ uint32_t h[256];
    n = dev_n(n, dn);
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    // the workgroups stride over the tiles, so that few of them add their
    // counts to the global bins (the leading digits of |A| fall into very few
    // bins, and atomics on one address serialise)
    for (size_t base = (size_t)blockIdx.x * kTile; base < n; base += (size_t)gridDim.x * kTile) {
        for (int i = threadIdx.x; i < kTile; i += kThreads) {
            size_t j = base + i;
            if (j < n) {
                uint64_t o = abs_order(score[j]);
                if ((o & mask) == prefix) atomicAdd(&h[(o >> shift) & 0xFFu], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(&st->hist[threadIdx.x], c);
}

// the entries that still match the selected prefix, copied (in any order:
// only their count per digit matters) to a smaller array
__global__ __launch_bounds__(kThreads) void k_sel_compact(const double *__restrict__ score, size_t n,
                                                          const SelectState *__restrict__ st, double *__restrict__ out,
                                                          unsigned int *__restrict__ count)
{
    const uint64_t prefix = st->prefix, mask = st->mask;
    const size_t base = (size_t)blockIdx.x * kTile;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int i = threadIdx.x; i < kTile; i += kThreads) {
        const size_t j = base + i;
        const double v = j < n ? score[j] : 0.0;
        const bool keep = j < n && (abs_order(v) & mask) == prefix;
        const uint64_t b = __ballot(keep);
        unsigned int at = 0;
        if (lane == 0 && b) at = atomicAdd(count, (unsigned int)__popcll(b));
        at = __shfl(at, 0, 64);
        if (keep) out[at + __popcll(b & lt)] = v;
    }
}

// one wavefront: lane l holds digits 255 - 4l .. 252 - 4l, so a scan across
// the lanes counts the entries above every digit; the digit taken is the
// largest d >= 1 with (entries above d) + hist[d] >= krem, else 0
__global__ __launch_bounds__(64) void k_sel_pick(SelectState *st, int shift)
{
    const int lane = threadIdx.x;
    uint32_t c[4];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = st->hist[255 - 4 * lane - k];
        sum += c[k];
    }
    uint64_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t ylo = __shfl_up((uint32_t)incl, d, 64), yhi = __shfl_up((uint32_t)(incl >> 32), d, 64);
        if (lane >= d) incl += (uint64_t)ylo | ((uint64_t)yhi << 32);
    }
    const uint64_t need = st->krem;
    uint64_t cum = incl - sum, above = 0;
    int found = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int dg = 255 - 4 * lane - k;
        if (found < 0 && (dg == 0 || cum + c[k] >= need)) {
            found = dg;
            above = cum;
        }
        cum += c[k];
    }
    const uint64_t bal = __ballot(found >= 0);
    const int src = __ffsll((long long)bal) - 1;
    const int d = __shfl(found, src, 64);
    const uint32_t alo = __shfl((uint32_t)above, src, 64), ahi = __shfl((uint32_t)(above >> 32), src, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) st->hist[4 * lane + k] = 0u;
    if (lane == 0) {
        st->krem = need - ((uint64_t)alo | ((uint64_t)ahi << 32));
        st->prefix |= (uint64_t)d << shift;
        st->mask |= 0xFFull << shift;
    }
}

}  // namespace

__global__ __launch_bounds__(64) void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v)
{
    for (uint32_t i = blockIdx.x * 64 + threadIdx.x; i < n; i += gridDim.x * 64) p[i] = v;
}

void fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return;
    k_fill_u32<<<(unsigned)std::min<size_t>((n + 63) / 64, 4096), 64, 0, s>>>(p, (uint32_t)n, v);
    ASCI_LAUNCH_CHECK();
}

void scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, Arena &ar, hipStream_t s,
              Profiler *prof, const uint32_t *dn)
{
    if (n == 0) {
        if (d_total) {
            k_fill_u32<<<1, 64, 0, s>>>(d_total, 1, 0u);
            ASCI_LAUNCH_CHECK();
        }
        return;
    }
    ProfScope ps(prof, "scan", 8.0 * n, s);
    if (n <= kScanSmall) {
        k_scan_small<<<1, 1024, 0, s>>>(in, out, (uint32_t)n, d_total, dn);
        ASCI_LAUNCH_CHECK();
        return;
    }
    size_t nb = (n + kTile - 1) / kTile;
    require(nb <= (1u << 26), ASCI_EINVAL, "scan too long");
    size_t mark = ar.used();
    uint32_t *partial = ar.take<uint32_t>(nb);
    k_scan_reduce<<<(unsigned)nb, kThreads, 0, s>>>(in, n, partial, dn);
    ASCI_LAUNCH_CHECK();
    k_scan_partials<<<1, 1024, 0, s>>>(partial, (uint32_t)nb, d_total);
    ASCI_LAUNCH_CHECK();
    k_scan_down<<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, partial, dn);
    ASCI_LAUNCH_CHECK();
    (void)mark;
}

template <typename V>
int radix_sort(uint64_t *keys_lo[2], uint64_t *keys_hi[2], V *vals[2], size_t n, int words,
               const std::vector<Digit> &digits, Arena &ar, hipStream_t s, Profiler *prof, const uint32_t *dn)
{
    int cur = 0;
    if (n <= 1 || digits.empty()) return cur;
    require(n < (1ull << 32), ASCI_EINVAL, "radix sort: too many records");
    // the smallest tile that keeps the histogram short (its scan is one small launch)
    int it = 16;
    for (int c : {2, 4, 8})
        if ((n + (size_t)kThreads * c - 1) / ((size_t)kThreads * c) <= 64) {
            it = c;
            break;
        }
    const size_t tile = (size_t)kThreads * it;
    size_t nb = (n + tile - 1) / tile;
    uint32_t *hist = ar.take<uint32_t>(nb * 256);
    for (const Digit &d : digits) {
        const int nxt = cur ^ 1;
        const double kb = 8.0 * words, rb = kb + sizeof(V);
        {
        ProfScope ps(prof, "rs_hist", kb * n, s);
        auto hist_k = [&](auto itc) {
            constexpr int I = decltype(itc)::value;
            if (words == 2)
                k_rs_hist<2, I><<<(unsigned)nb, kThreads, 0, s>>>(keys_lo[cur], keys_hi[cur], n, d.word, d.shift,
                                                                  hist, (uint32_t)nb, dn);
            else
                k_rs_hist<1, I><<<(unsigned)nb, kThreads, 0, s>>>(keys_lo[cur], nullptr, n, 0, d.shift, hist,
                                                                  (uint32_t)nb, dn);
        };
        if (it == 2) hist_k(std::integral_constant<int, 2>{});
        else if (it == 4) hist_k(std::integral_constant<int, 4>{});
        else if (it == 8) hist_k(std::integral_constant<int, 8>{});
        else hist_k(std::integral_constant<int, 16>{});
        ASCI_LAUNCH_CHECK();
        }
        scan_u32(hist, hist, nb * 256, nullptr, ar, s, prof);  // every block writes its column
        ProfScope ps(prof, "rs_scatter", 2.0 * rb * n, s);
        auto scat_k = [&](auto itc) {
            constexpr int I = decltype(itc)::value;
            if (words == 2)
                k_rs_scatter<2, V, I><<<(unsigned)nb, kThreads, 0, s>>>(
                    keys_lo[cur], keys_hi[cur], vals[cur], keys_lo[nxt], keys_hi[nxt], vals[nxt], n, d.word,
                    d.shift, hist, (uint32_t)nb, dn);
            else
                k_rs_scatter<1, V, I><<<(unsigned)nb, kThreads, 0, s>>>(keys_lo[cur], nullptr, vals[cur],
                                                                        keys_lo[nxt], nullptr, vals[nxt], n, 0,
                                                                        d.shift, hist, (uint32_t)nb, dn);
        };
        if (it == 2) scat_k(std::integral_constant<int, 2>{});
        else if (it == 4) scat_k(std::integral_constant<int, 4>{});
        else if (it == 8) scat_k(std::integral_constant<int, 8>{});
        else scat_k(std::integral_constant<int, 16>{});
        ASCI_LAUNCH_CHECK();
        cur = nxt;
    }
    return cur;
}

template int radix_sort<double>(uint64_t *[2], uint64_t *[2], double *[2], size_t, int,
                                const std::vector<Digit> &, Arena &, hipStream_t, Profiler *, const uint32_t *);
template int radix_sort<uint32_t>(uint64_t *[2], uint64_t *[2], uint32_t *[2], size_t, int,
                                  const std::vector<Digit> &, Arena &, hipStream_t, Profiler *, const uint32_t *);

Profiler::~Profiler()
{
    for (auto &p : pending_) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : pool_) (void)hipEventDestroy(e);
}

hipEvent_t Profiler::get_event()
{
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e;
    ASCI_HIP(hipEventCreate(&e));
    return e;
}

int Profiler::begin(const char *name, double bytes, hipStream_t s)
{
    int idx = -1;
    for (size_t i = 0; i < entries.size(); ++i)
        if (entries[i].name == name) idx = (int)i;
    if (idx < 0) {
        entries.push_back(ProfEntry{name});
        idx = (int)entries.size() - 1;
    }
    Pending p{idx, get_event(), get_event(), bytes};
    ASCI_HIP(hipEventRecord(p.a, s));
    pending_.push_back(p);
    return (int)pending_.size() - 1;
}

void Profiler::end(int token, hipStream_t s) { ASCI_HIP(hipEventRecord(pending_[token].b, s)); }

void Profiler::set_bytes(int token, double bytes)
{
    if (token >= 0 && (size_t)token < pending_.size()) pending_[(size_t)token].bytes = bytes;
}

void Profiler::collect()
{
    for (auto &p : pending_) {
        float ms = 0.f;
        ASCI_HIP(hipEventSynchronize(p.b));
        ASCI_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        ProfEntry &e = entries[p.entry];
        e.ms += ms;
        e.launches += 1;
        e.bytes += p.bytes;
        pool_.push_back(p.a);
        pool_.push_back(p.b);
    }
    pending_.clear();
}

void Profiler::reset()
{
    collect();
    entries.clear();
}

void radix_select_abs(const double *score, size_t n, uint64_t k, SelectState *d_state, hipStream_t s,
                      Profiler *prof, const SelectWork *work, const uint32_t *dn, const uint32_t *dk)
{
    require(k >= 1 && k <= n, ASCI_EINVAL, "radix select: k out of range");
    if (dn) work = nullptr;  // the compaction reads its count back on the host
    size_t nb = (n + kTile - 1) / kTile;
    k_sel_init<<<1, kThreads, 0, s>>>(d_state, k, dk);
    ASCI_LAUNCH_CHECK();
    const double *x = score;
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (shift == 40 && work) {
            // after 16 bits only the entries of the selected prefix matter:
            // copy them out and run the remaining passes on the copy
            ASCI_HIP(hipMemsetAsync(work->d_count, 0, sizeof(unsigned int), s));
            {
                ProfScope ps(prof, "select_compact", 8.0 * n, s);
                k_sel_compact<<<(unsigned)nb, kThreads, 0, s>>>(x, n, d_state, work->tmp, work->d_count);
                ASCI_LAUNCH_CHECK();
            }
            ASCI_HIP(hipMemcpyAsync(work->h_count, work->d_count, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
            ASCI_HIP(hipStreamSynchronize(s));
            x = work->tmp;
            n = *work->h_count;
            nb = (n + kTile - 1) / kTile;
        }
        if (nb) {
            ProfScope ps(prof, "select_hist", 8.0 * n, s);
            k_sel_hist<<<(unsigned)std::min<size_t>(nb, 2048), kThreads, 0, s>>>(x, n, shift, d_state, dn);
            ASCI_LAUNCH_CHECK();
        }
        k_sel_pick<<<1, 64, 0, s>>>(d_state, shift);
        ASCI_LAUNCH_CHECK();
    }
}

}  // namespace asci
