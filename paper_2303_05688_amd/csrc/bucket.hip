// Sort-and-accumulate of one class batch by buckets (Alg. 2, the sort on
// the target bitstring and the sum per unique target), built for LDS:
//
//   segments: contiguous record ranges whose keys agree on every bit at or
//             above `top`; the classes of the batch are the first segments
//             (the generator lays records out class by class).
//   split   : a segment larger than the LDS capacity is split, stably, into
//             up to 256 key ranges bounded by splitters sampled from it
//             (sample sort: the ranges are balanced however skewed the keys
//             are, and they keep key order), with per-tile histograms laid out
//             segment by segment, one global exclusive scan and a ranked
//             scatter into the other buffer.  A segment the splitters cannot
//             divide (its keys lie in one range) is split at the next level
//             on the 8 key bits just below `top` instead, which always lowers
//             `top`.  Repeat level by level.
//   finish  : one workgroup per final segment sorts the segment's record
//             indices in LDS (stable LSD on a 32-bit window of each key that
//             holds the bits varying inside the segment), gathers the values
//             in sorted order, sums every run of equal keys in record order
//             (record order is ascending core index), drops input
//             determinants (and, after an earlier class batch, candidates
//             below the pool's k-th |A|), forms H_aa and A_a, and writes the
//             surviving candidates, compacted, at the segment's start in slot
//             arrays.
//   collect : final segments ordered by start (= key order), their candidate
//             counts scanned, and the candidates copied to the pool.
//
// Keys are handled as the 2n-bit value (alpha << n) | beta: one word for
// n <= 32, two words (hi = alpha, lo = beta) above.
#include "hamiltonian.h"

#include <algorithm>

namespace asci {

namespace {

constexpr int kTileT = 1024;          // threads of the scatter: two workgroups of 16 waves per CU
constexpr int kTileItems = 4;
constexpr int kHistT = 256;           // threads of the histogram pass
constexpr int kTileN = kTileT * kTileItems;  // 4096 records per tile

struct Seg {
    // meta: top (bits 0-7) | buf (bit 8) | single key (bit 9) | split on key bits (bit 10)
    uint32_t start, size, meta;
};

__host__ __device__ __forceinline__ uint32_t seg_top(const Seg &s) { return s.meta & 0xFFu; }
__host__ __device__ __forceinline__ uint32_t seg_buf(const Seg &s) { return (s.meta >> 8) & 1u; }
__host__ __device__ __forceinline__ bool seg_single(const Seg &s) { return (s.meta >> 9) & 1u; }
__host__ __device__ __forceinline__ bool seg_bits(const Seg &s) { return (s.meta >> 10) & 1u; }
__host__ __device__ __forceinline__ uint32_t make_meta(uint32_t top, uint32_t buf, bool single, bool bits = false)
{
    return top | (buf << 8) | (single ? 512u : 0u) | (bits ? 1024u : 0u);
}

constexpr int kMaxSplit = 256;       // ranges per split
constexpr int kSplitSample = 16;     // samples per range

// bits [sh, sh + w) of the 2n-bit key, w <= 8
template <int W>
__device__ __forceinline__ uint32_t vdigit(uint64_t lo, uint64_t hi, int n, int sh, int w)
{
    uint64_t x;
    if (W == 1) {
        x = lo >> sh;
    } else if (sh >= n) {
        x = hi >> (sh - n);
    } else {
        x = lo >> sh;
        if (sh + w > n) x |= hi << (n - sh);
    }
    return (uint32_t)x & ((1u << w) - 1u);
}

template <int W>
__device__ __forceinline__ bool key_less(uint64_t alo, uint64_t ahi, uint64_t blo, uint64_t bhi)
{
    return W == 1 ? alo < blo : (ahi < bhi || (ahi == bhi && alo < blo));
}

// a value every lane of the wavefront holds, moved to a scalar register
__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// exclusive scan over the block (NW waves); every thread must call it
template <int NW>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t x = wave_incl_scan(v);
    if (lane == 63) s_tmp[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t t = s_tmp[i];
        base += (i < w) ? t : 0u;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return base + x - v;
}

// The same scan with one barrier: consecutive calls alternate between the two
// halves of s_tmp (2 * NW entries), so a call's totals are never overwritten
// before every thread has passed the next call's barrier.  `parity` flips per
// call and must be uniform across the workgroup.
template <int NW>
__device__ __forceinline__ uint32_t block_scan1(uint32_t v, uint32_t *s_tmp, uint32_t &parity, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t *buf = s_tmp + parity * NW;
    parity ^= 1u;
    const uint32_t x = wave_incl_scan(v);
    if (lane == 63) buf[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t t = buf[i];
        base += (i < w) ? t : 0u;
        tot += t;
    }
    total = tot;
    return base + x - v;
}

// ---------------------------------------------------------------- split level
struct SplitArgs {
    const Seg *segs;          // large segments of this level
    uint32_t nseg;
    const uint32_t *tile_base;  // per segment: first tile (exclusive scan of tile counts)
    const uint32_t *tile_seg;   // per tile: its segment
    uint32_t ntiles;
    uint32_t *hist;             // [tiles * 256], segment-major, digit-major inside a segment
    uint64_t *klo[2], *khi[2];
    double *val[2];
    int n;
    uint32_t cap;
    const uint64_t *spl_lo, *spl_hi;  // splitters: kMaxSplit - 1 per segment
    unsigned long long *kvar;         // per segment: the key bits that vary in it (2 words each)
    uint8_t *dig;                     // per record: its digit, from the histogram pass
    const uint32_t *dn_seg = nullptr;    // device: segments of the level (nseg is then a bound)
    const uint32_t *dn_tiles = nullptr;  // device: tiles of the level (ntiles is then a bound)
};

__device__ __forceinline__ uint32_t dev_count(uint32_t n, const uint32_t *dn) { return dn ? min(n, *dn) : n; }

// ranges of a splitter split: about half the LDS capacity each, 2 to 256
__host__ __device__ __forceinline__ uint32_t split_ranges(uint32_t size, uint32_t cap)
{
    const uint64_t want = ((uint64_t)size * 2 + cap - 1) / cap;
    return (uint32_t)(want < 2 ? 2 : (want > (uint64_t)kMaxSplit ? (uint64_t)kMaxSplit : want));
}

// How one split level divides a segment: by splitters (nb ranges, the
// splitters of segment s staged in LDS by the caller) or by key bits.
struct SplitRule {
    bool bits;
    int sh, w;
    uint32_t nb;  // digits in use
};

__device__ __forceinline__ SplitRule split_rule(const Seg &sg, uint32_t cap)
{
    SplitRule r;
    r.bits = seg_bits(sg);
    if (r.bits) {
        // the fallback: the 8 bits below top (top is the highest varying bit + 1)
        const int top = (int)seg_top(sg);
        r.w = top < 8 ? top : 8;
        r.sh = top - r.w;
        r.nb = 1u << r.w;
    } else {
        r.sh = r.w = 0;
        r.nb = split_ranges(sg.size, cap);
    }
    return r;
}

// the digit of a key: its range (number of splitters <= key) or its key bits
template <int W>
__device__ __forceinline__ uint32_t split_key_digit(const SplitRule &r, const uint64_t *spl_lo,
                                                   const uint64_t *spl_hi, uint64_t lo, uint64_t hi, int n)
{
    if (r.bits) return vdigit<W>(lo, hi, n, r.sh, r.w);
    // count of splitters <= key by binary lifting over the 255 staged entries
    // (the unused ones hold the largest key): eight steps, no branches, so
    // the searches of several keys overlap
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t step = 128; step >= 1; step >>= 1) {
        const uint32_t m = pos + step - 1u;
        const bool le = W == 1 ? spl_lo[m] <= lo : (spl_hi[m] < hi || (spl_hi[m] == hi && spl_lo[m] <= lo));
        pos += le ? step : 0u;
    }
    return min(pos, r.nb - 1u);
}

// stage the splitters of segment s in LDS (every thread of the block calls it)
template <int W>
__device__ __forceinline__ void load_splitters(const SplitRule &r, const uint64_t *__restrict__ g_lo,
                                               const uint64_t *__restrict__ g_hi, uint32_t s, uint64_t *spl_lo,
                                               uint64_t *spl_hi)
{
    static_assert(kMaxSplit == 256, "binary lifting over 255 splitters");
    if (!r.bits)
        for (uint32_t j = threadIdx.x; j < kMaxSplit - 1; j += blockDim.x) {
            const bool used = j + 1u < r.nb;
            spl_lo[j] = used ? g_lo[(size_t)s * (kMaxSplit - 1) + j] : ~0ull;
            if (W == 2) spl_hi[j] = used ? g_hi[(size_t)s * (kMaxSplit - 1) + j] : ~0ull;
        }
    __syncthreads();
}

// Splitters of every large segment that splits by ranges: kSplitSample
// records per range, taken at even strides (the records are in generation
// order, not key order, so a strided pick is a fair sample), sorted in LDS by
// a bitonic network; the splitters are the sample's quantiles.
struct KeyBufs {
    const uint64_t *lo[2], *hi[2];
};

template <int W, int T>
__global__ __launch_bounds__(T) void k_seg_splitters(const Seg *__restrict__ segs, uint32_t cap, KeyBufs kb,
                                                       uint64_t *__restrict__ g_lo, uint64_t *__restrict__ g_hi,
                                                       uint32_t nseg, const uint32_t *dn_seg)
{
    constexpr int kMaxSample = kMaxSplit * kSplitSample;  // 4096
    __shared__ uint64_t x_lo[kMaxSample];
    __shared__ uint64_t x_hi[W == 2 ? kMaxSample : 1];
    const uint32_t ns = dev_count(nseg, dn_seg);
    for (uint32_t s = blockIdx.x; s < ns; s += gridDim.x) {
    const Seg sg = segs[s];
    if (seg_bits(sg)) continue;  // uniform per block
    const uint32_t nb = split_ranges(sg.size, cap);
    const uint32_t m = min(sg.size, nb * (uint32_t)kSplitSample);
    uint32_t p = 1;
    while (p < m) p <<= 1;
    const uint64_t *klo = kb.lo[seg_buf(sg)], *khi = kb.hi[seg_buf(sg)];
    __syncthreads();  // the previous segment's samples are read
    for (uint32_t i = threadIdx.x; i < p; i += T) {
        if (i < m) {
            const size_t j = (size_t)sg.start + (size_t)(((uint64_t)2 * i + 1) * sg.size / (2 * (uint64_t)m));
            x_lo[i] = klo[j];
            if (W == 2) x_hi[i] = khi[j];
        } else {
            x_lo[i] = ~0ull;
            if (W == 2) x_hi[i] = ~0ull;
        }
    }
    __syncthreads();
    for (uint32_t k = 2; k <= p; k <<= 1) {
        for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (uint32_t i = threadIdx.x; i < p; i += T) {
                const uint32_t o = i ^ jj;
                if (o > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t al = x_lo[i], bl = x_lo[o];
                    const uint64_t ah = W == 2 ? x_hi[i] : 0ull, bh = W == 2 ? x_hi[o] : 0ull;
                    const bool gt = key_less<W>(bl, bh, al, ah);
                    if (gt == up) {
                        x_lo[i] = bl;
                        x_lo[o] = al;
                        if (W == 2) {
                            x_hi[i] = bh;
                            x_hi[o] = ah;
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t j = threadIdx.x; j + 1u < nb; j += T) {
        const uint32_t q = (uint32_t)(((uint64_t)(j + 1) * m) / nb);
        g_lo[(size_t)s * (kMaxSplit - 1) + j] = x_lo[q];
        if (W == 2) g_hi[(size_t)s * (kMaxSplit - 1) + j] = x_hi[q];
    }
    }
}

// tiles per large segment; also clears the level's skip flags and the count of
// next-level segments (instead of separate fill launches)
__global__ __launch_bounds__(256) void k_seg_tiles(const Seg *__restrict__ segs, uint32_t nseg,
                                                   uint32_t *__restrict__ ntile, uint32_t *__restrict__ skip,
                                                   uint32_t *__restrict__ nnext, const uint32_t *dn_seg)
{
    const uint32_t ns = dev_count(nseg, dn_seg);
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s <= ns; s += gridDim.x * 256) {
        if (s < ns) ntile[s] = (segs[s].size + kTileN - 1) / kTileN;
        skip[s] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *nnext = 0u;
}

// the segment of every tile; also clears the varying-bit words of every segment
__global__ __launch_bounds__(256) void k_seg_expand(const Seg *__restrict__ segs, uint32_t nseg,
                                                    const uint32_t *__restrict__ tile_base,
                                                    uint32_t *__restrict__ tile_seg, unsigned long long *__restrict__ kvar,
                                                    const uint32_t *dn_seg)
{
    const uint32_t ns = dev_count(nseg, dn_seg);
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < ns; s += gridDim.x * 256) {
        kvar[2 * s] = 0ull;
        kvar[2 * s + 1] = 0ull;
        const uint32_t nt = (segs[s].size + kTileN - 1) / kTileN, tb = tile_base[s];
        for (uint32_t t = 0; t < nt; ++t) tile_seg[tb + t] = s;
    }
}

// Tiles of a level, XCD-contiguous: the tiles [x * per, (x + 1) * per) go to
// XCD x (workgroups are handed to the 8 XCDs in turn), taken by that XCD's
// workgroups in turn.  With a grid of 8 * per workgroups each takes one tile.
#define FOR_LEVEL_TILES(a, t)                                                          \
    const uint32_t nt_all_ = dev_count((a).ntiles, (a).dn_tiles);                     \
    const uint32_t per_ = (nt_all_ + 7u) / 8u, slots_ = max(gridDim.x >> 3, 1u);      \
    for (uint32_t i_ = blockIdx.x >> 3, t = (blockIdx.x & 7u) * per_ + i_;            \
         i_ < per_ && t < nt_all_; i_ += slots_, t = (blockIdx.x & 7u) * per_ + i_)

template <int W>
__global__ __launch_bounds__(kHistT) void k_split_hist(SplitArgs a)
{
    __shared__ uint32_t h[kHistT / 64][256];
    __shared__ uint64_t spl_lo[kMaxSplit - 1];
    __shared__ uint64_t spl_hi[W == 2 ? kMaxSplit - 1 : 1];
    FOR_LEVEL_TILES(a, t) {
    const uint32_t s = a.tile_seg[t];
    const Seg sg = a.segs[s];
    const uint32_t tb = a.tile_base[s], nt = (sg.size + kTileN - 1) / kTileN, tl = t - tb;
    const SplitRule rule = split_rule(sg, a.cap);
    const uint32_t buf = seg_buf(sg);
    __syncthreads();  // the previous tile's counts are written out
    for (int i = threadIdx.x; i < (kHistT / 64) * 256; i += kHistT) (&h[0][0])[i] = 0u;
    load_splitters<W>(rule, a.spl_lo, a.spl_hi, s, spl_lo, spl_hi);
    const uint32_t r0 = tl * kTileN, r1 = min(sg.size, r0 + kTileN);
    const int wv = threadIdx.x >> 6;
    // the bits in which some key differs from the segment's first key vary in
    // the segment (one OR per word instead of an OR and an AND)
    const uint64_t ref_lo = a.klo[buf][sg.start], ref_hi = W == 2 ? a.khi[buf][sg.start] : 0ull;
    uint64_t d0 = 0ull, d1 = 0ull;
    // four records per step, their searches interleaved
    for (uint32_t rb = r0 + threadIdx.x; rb < r1; rb += 4 * kHistT) {
        uint64_t lo[4], hi[4];
        uint32_t dg[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = rb + (uint32_t)k * kHistT;
            const size_t j = (size_t)sg.start + (r < r1 ? r : r0);
            lo[k] = a.klo[buf][j];
            hi[k] = W == 2 ? a.khi[buf][j] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) dg[k] = split_key_digit<W>(rule, spl_lo, spl_hi, lo[k], hi[k], a.n);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = rb + (uint32_t)k * kHistT;
            if (r < r1) {
                d0 |= lo[k] ^ ref_lo;
                d1 |= hi[k] ^ ref_hi;
                a.dig[(size_t)sg.start + r] = (uint8_t)dg[k];
                atomicAdd(&h[wv][dg[k]], 1u);
            }
        }
    }
    // which key bits vary inside the segment (for segments the split cannot divide)
    for (int dd = 32; dd >= 1; dd >>= 1) {
        d0 |= __shfl_xor(d0, dd, 64);
        if (W == 2) d1 |= __shfl_xor(d1, dd, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicOr(&a.kvar[2 * s], (unsigned long long)d0);
        if (W == 2) atomicOr(&a.kvar[2 * s + 1], (unsigned long long)d1);
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d < 256) {
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kHistT / 64; ++i) c += h[i][d];
        a.hist[(size_t)tb * 256 + (size_t)d * nt + tl] = c;
    }
    }
}

// children of every large segment (one block of 256 threads per segment).
// Digits larger than the LDS capacity become large segments of the next level
// (or single-key finals once no bits are left); runs of consecutive smaller
// digits are coalesced into final segments of at most `cap` records, so the
// finish never sees fragments.  A segment whose records all share the digit
// is not moved: skip[s] = 1 and its child keeps its buffer.
template <int W>
__global__ __launch_bounds__(256) void k_split_children(const Seg *__restrict__ segs, uint32_t nseg,
                                                        const uint32_t *__restrict__ tile_base,
                                                        const uint32_t *__restrict__ scan, uint32_t cap,
                                                        uint32_t *__restrict__ skip, Seg *__restrict__ finals,
                                                        uint32_t *__restrict__ nfinal, uint32_t finals_cap,
                                                        Seg *__restrict__ next, uint32_t *__restrict__ nnext,
                                                        uint32_t next_cap, uint32_t *__restrict__ overflow,
                                                        const unsigned long long *__restrict__ kvar, int n,
                                                        const uint32_t *dn_seg)
{
    __shared__ uint32_t s_cnt[256], s_off[256];
    __shared__ Seg s_fin[256], s_nxt[256];
    __shared__ uint32_t s_nf, s_nn, s_bf, s_bn;
    const uint32_t ns = dev_count(nseg, dn_seg);
    for (uint32_t s = blockIdx.x; s < ns; s += gridDim.x) {
    __syncthreads();  // the previous segment's children are copied out
    const Seg sg = segs[s];
    const uint32_t tb = tile_base[s], nt = (sg.size + kTileN - 1) / kTileN;
    const SplitRule rule = split_rule(sg, cap);
    const uint32_t d = threadIdx.x;
    const size_t b0 = (size_t)tb * 256;
    const uint32_t base = scan[b0];
    const uint32_t off = scan[b0 + (size_t)d * nt] - base;
    const uint32_t end = (d + 1 < 256u) ? scan[b0 + (size_t)(d + 1) * nt] - base : sg.size;
    s_cnt[d] = (d < rule.nb) ? end - off : 0u;
    s_off[d] = off;
    __syncthreads();
    // thread 0 lays out the children in LDS (no global atomics in the loop)
    if (d == 0) {
    uint32_t nf = 0, nn = 0;
    auto push_fin = [&](const Seg &c) { s_fin[nf++] = c; };
    auto push_nxt = [&](const Seg &c) { s_nxt[nn++] = c; };
    // the children of a range split keep the parent's top (their keys share at
    // least its prefix); those of a bit split share bits down to sh
    const uint32_t ptop = seg_top(sg), top = rule.bits ? (uint32_t)rule.sh : ptop;
    bool whole = false;
    for (uint32_t x = 0; x < rule.nb; ++x) {
        if (s_cnt[x] == sg.size) {  // one digit holds everything: relabel, do not move
            whole = true;
            skip[s] = 1u;
            Seg c{sg.start, sg.size, 0u};
            // highest key bit that varies inside the segment, + 1 (0: one key)
            const uint64_t v0 = kvar[2 * s], v1 = W == 2 ? kvar[2 * s + 1] : 0ull;
            const uint32_t vtop = W == 1 ? (v0 ? 64u - (uint32_t)__clzll((long long)v0) : 0u)
                                         : (v1 ? (uint32_t)n + 64u - (uint32_t)__clzll((long long)v1)
                                               : (v0 ? 64u - (uint32_t)__clzll((long long)v0) : 0u));
            if (vtop == 0) {
                // a single key: one final segment, summed in record order
                c.meta = make_meta(0u, seg_buf(sg), sg.size > cap);
                push_fin(c);
            } else if (!rule.bits) {
                // the splitters cannot divide it: split on its top varying bits next
                c.meta = make_meta(vtop, seg_buf(sg), false, true);
                push_nxt(c);
            } else if (sg.size <= cap || top == 0) {
                c.meta = make_meta(top, seg_buf(sg), sg.size > cap);
                push_fin(c);
            } else {
                c.meta = make_meta(top, seg_buf(sg), false);
                push_nxt(c);
            }
            break;
        }
    }
    const uint32_t buf = seg_buf(sg) ^ 1u;
    uint32_t g_start = 0, g_size = 0, g_digits = 0;
    auto flush = [&]() {
        if (g_size) {
            Seg c{sg.start + g_start, g_size, make_meta(g_digits == 1 ? top : ptop, buf, false)};
            push_fin(c);
        }
        g_size = 0;
        g_digits = 0;
    };
    for (uint32_t x = 0; x < (whole ? 0u : rule.nb); ++x) {
        const uint32_t c = s_cnt[x];
        if (c == 0) continue;
        if (c > cap) {
            flush();
            Seg L{sg.start + s_off[x], c, 0u};
            if (top == 0) {
                L.meta = make_meta(0u, buf, true);
                push_fin(L);
            } else {
                L.meta = make_meta(top, buf, false);
                push_nxt(L);
            }
            continue;
        }
        if (g_size + c > cap) flush();
        if (g_size == 0) g_start = s_off[x];
        g_size += c;
        ++g_digits;
    }
    flush();
    s_nf = nf;
    s_nn = nn;
    s_bf = nf ? atomicAdd(nfinal, nf) : 0u;
    s_bn = nn ? atomicAdd(nnext, nn) : 0u;
    }
    __syncthreads();
    // every thread copies its share of the children out
    const uint32_t nf = s_nf, nn = s_nn, bf = s_bf, bn = s_bn;
    for (uint32_t i = d; i < nf; i += 256) {
        if (bf + i < finals_cap) finals[bf + i] = s_fin[i];
        else atomicOr(overflow, 1u);
    }
    for (uint32_t i = d; i < nn; i += 256) {
        if (bn + i < next_cap) next[bn + i] = s_nxt[i];
        else atomicOr(overflow, 1u);
    }
    }
}

template <int W>
// eight waves per SIMD (64 VGPRs): the load, rank and write phases of four
// workgroups' worth of waves overlap on each CU
__global__ __launch_bounds__(kTileT) __attribute__((amdgpu_waves_per_eu(8))) void k_split_scatter(SplitArgs a, const uint32_t *__restrict__ scan,
                                                          const uint32_t *__restrict__ skip)
{
    constexpr int NW = kTileT / 64;
    __shared__ uint64_t s_lo[kTileN];
    __shared__ uint64_t s_hi[W == 2 ? kTileN : 1];
    __shared__ double s_val[kTileN];
    __shared__ uint16_t s_wcnt[NW][256];  // counts and prefixes below kTileN
    __shared__ uint32_t s_dbase[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_tmp[NW];
    __shared__ uint8_t s_dg[kTileN];

    FOR_LEVEL_TILES(a, t) {
    const uint32_t s = a.tile_seg[t];
    if (skip[s]) continue;  // uniform per block
    const Seg sg = a.segs[s];
    const uint32_t tb = a.tile_base[s], nt = (sg.size + kTileN - 1) / kTileN, tl = t - tb;
    const uint32_t ib = seg_buf(sg), ob = ib ^ 1u;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __syncthreads();  // the previous tile's records are written out
    for (int i = tid; i < NW * 256; i += kTileT) (&s_wcnt[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t r0 = tl * kTileN, rn = min(sg.size - r0, (uint32_t)kTileN);
    uint64_t rlo[kTileItems], rhi[kTileItems];
    double rv[kTileItems];
    uint32_t rrank[kTileItems], rd[kTileItems];
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < kTileItems; ++q) {
        const uint32_t li = (uint32_t)wv * 64 * kTileItems + (uint32_t)q * 64 + lane;
        const bool valid = li < rn;
        const size_t j = (size_t)sg.start + r0 + li;
        rlo[q] = valid ? a.klo[ib][j] : 0ull;
        rhi[q] = (W == 2 && valid) ? a.khi[ib][j] : 0ull;
        rv[q] = valid ? a.val[ib][j] : 0.0;
        const uint32_t d = valid ? (uint32_t)a.dig[j] : 0u;
        rd[q] = d;
        const uint64_t peers = wave_match(d, valid, 8);
        const uint32_t before = s_wcnt[wv][d];
        rrank[q] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0ull) s_wcnt[wv][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = tid;
        uint32_t run = 0;
        if (d < 256) {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const uint32_t c = s_wcnt[i][d];
                s_wcnt[i][d] = run;
                run += c;
            }
        }
        uint32_t tot;
        const uint32_t e = block_scan<NW>(d < 256 ? run : 0u, s_tmp, tot);
        if (d < 256) {
            s_dbase[d] = e;
            const size_t b0 = (size_t)tb * 256;
            s_gbase[d] = sg.start + (a.hist[b0 + (size_t)d * nt + tl] - a.hist[b0]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTileItems; ++q) {
        const uint32_t li = (uint32_t)wv * 64 * kTileItems + (uint32_t)q * 64 + lane;
        if (li < rn) {
            const uint32_t d = rd[q];
            const uint32_t p = min(s_dbase[d] + s_wcnt[wv][d] + rrank[q], (uint32_t)kTileN - 1u);
            s_lo[p] = rlo[q];
            if (W == 2) s_hi[p] = rhi[q];
            s_val[p] = rv[q];
            s_dg[p] = (uint8_t)d;
        }
    }
    __syncthreads();
    const uint32_t seg_end = sg.start + sg.size;
    for (uint32_t i = tid; i < rn; i += kTileT) {
        const uint64_t lo = s_lo[i];
        const uint64_t hi = W == 2 ? s_hi[i] : 0ull;
        const uint32_t d = s_dg[i];
        const uint32_t g = s_gbase[d] + (i - s_dbase[d]);
        if (g >= sg.start && g < seg_end) {
            a.klo[ob][g] = lo;
            if (W == 2) a.khi[ob][g] = hi;
            a.val[ob][g] = s_val[i];
        }
    }
    }
    (void)scan;
}

// ---------------------------------------------------------------- finish
struct FinishArgs {
    const Seg *finals;
    uint64_t *klo[2], *khi[2];
    double *val[2];
    int n;
    const double *jk, *h;       // J, J-K (n^2 each), h_pp (n); h (n^2)
    SpinTables st;              // E(alpha), E(beta) by string rank (optional)
    const uint64_t *thr;        // candidates with abs_order(A) below *thr cannot enter the top k (optional)
    double ecore, E0, eps;      // eps > 0: keep a pair only if |H_ai C_i / (E0 - H_aa)| > eps
    uint64_t *clo, *chi;        // slot arrays (batch positions)
    double *cnum, *cscore;
    uint32_t *cnt;              // per final segment: candidates written
    uint32_t nfinal;
    const uint32_t *dn_final;   // device: final segments (nfinal is then a bound; optional)
    PsiSet psi;                 // input determinants (exclusion)
    int tab_in_lds;             // staged in LDS: 1 J, J-K, h_pp; 2 J and the binomials; 3 the binomials; 0 none
};

// E(s) of one spin string (0 = alpha, 1 = beta): looked up when tabulated
__device__ __forceinline__ double spin_e(const SpinTables &st, int spin, const double *X, const double *hd, int n,
                                         uint64_t str)
{
    const double *t = st.e[spin];
    return t ? t[spin_rank(st.binom, n, str)] : spin_energy(X, hd, n, str);
}

// H_aa = ((ecore + E(alpha)) + E(beta)) + E(alpha, beta)
__device__ __forceinline__ double diag_tab(const SpinTables &st, const double *J, const double *X, const double *hd,
                                           int n, double ecore, uint64_t a, uint64_t b)
{
    return ((ecore + spin_e(st, 0, X, hd, n, a)) + spin_e(st, 1, X, hd, n, b)) + cross_energy(J, n, a, b);
}

// The key as one 2n-bit value (alpha << n) | beta.  Bits [o, o + 32) of it:
template <int W>
__device__ __forceinline__ uint32_t key_window(uint64_t lo, uint64_t hi, int n, int o)
{
    if (W == 1) return o < 64 ? (uint32_t)(lo >> o) : 0u;
    if (o >= n) return (uint32_t)(hi >> (o - n));
    uint64_t x = lo >> o;
    if (n - o < 32) x |= hi << (n - o);
    return (uint32_t)x;
}

// OR a 32-bit window c into bits [o, o + 32) of the key (bits past 2n are 0 in c)
template <int W>
__device__ __forceinline__ void key_put(uint32_t c, int o, int n, uint64_t &lo, uint64_t &hi)
{
    if (W == 1) {
        lo |= (uint64_t)c << o;
        return;
    }
    if (o >= n) {
        hi |= (uint64_t)c << (o - n);
        return;
    }
    const uint64_t nmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    lo |= ((uint64_t)c << o) & nmask;
    if (n - o < 32) hi |= (uint64_t)c >> (n - o);
}

// lowest varying key bit (-1: none) and one past the highest
template <int W>
__device__ __forceinline__ int key_low(uint64_t vlo, uint64_t vhi, int n)
{
    if (vlo) return __builtin_ctzll(vlo);
    if (W == 2 && vhi) return n + __builtin_ctzll(vhi);
    return -1;
}
template <int W>
__device__ __forceinline__ int key_top(uint64_t vlo, uint64_t vhi, int n)
{
    if (W == 2 && vhi) return n + 64 - __builtin_clzll(vhi);
    if (vlo) return 64 - __builtin_clzll(vlo);
    return 0;
}

// LDS of one workgroup.  The sort permutes 16-bit record indices, ranking
// them by a 32-bit window of each key that holds its varying bits (a key is
// rebuilt from its window and the segment's constant bits); the values are
// then gathered from the segment in sorted order.  After the sort ix[cur ^ 1] holds the run
// heads, `aidx` (over the digit counters) each run's alpha slot, and `acache`
// E(alpha) and c_q(alpha) of the segment's alpha strings when they fit: a
// segment whose keys need two or more windows reads its keys from memory
// after the sort, so the window array `ck` just before `acache` extends it.
template <int W, int CAP, int NT>
struct FinishLds {
    static constexpr int NW = NT / 64;
    static constexpr uint32_t kAcacheBytes = CAP;
    uint32_t ck[CAP];
    uint64_t acache[kAcacheBytes / 8];
    uint16_t ix[2][CAP + 8];
    double val[CAP];
    union {
        uint16_t wcnt[NW][256];
        uint8_t aidx[CAP];
    };
    uint32_t dbase[256];
    uint32_t tmp[2 * NW];
    uint32_t nruns, nalpha;
    uint64_t red[2][NW];  // per wave: OR of the key words' differences from the first key
};

// one final segment, processed by the whole workgroup
template <int W, int CAP, int NT>
__device__ __forceinline__ void finish_segment(const FinishArgs &f, const SpinTables &st, FinishLds<W, CAP, NT> &S,
                                               const double *J, const double *X, const double *hd, uint32_t sidx)
{
    using L = FinishLds<W, CAP, NT>;
    constexpr int NW = L::NW;
    constexpr int IT = CAP / NT;
    static_assert(CAP % NT == 0 && NW * 256 * 2 >= CAP, "aidx must fit over the digit counters");
    const int n = f.n;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;

    const Seg sg = f.finals[sidx];
    const uint32_t buf = seg_buf(sg);
    const uint64_t nmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    uint32_t parity = 0;  // half of S.tmp for the next block scan
    const uint64_t *gk = f.klo[buf] + sg.start;
    const uint64_t *gh = f.khi[buf] + sg.start;
    const double *gv = f.val[buf] + sg.start;

    if (seg_single(sg)) {
        // more records than fit in LDS, all with one key: sum in record order
        __syncthreads();
        if (tid == 0) {
            const uint64_t lo = gk[0], hi = W == 2 ? gh[0] : 0ull;
            const bool ex = psi_contains(f.psi, lo, hi);
            uint32_t c = 0;
            if (!ex) {
                const uint64_t a = W == 1 ? (lo >> n) : hi, b = W == 1 ? (lo & nmask) : lo;
                const double den = f.E0 - diag_tab(st, J, X, hd, n, f.ecore, a, b);
                double sum = 0.0;
                uint32_t kept = 0;
                for (uint32_t r = 0; r < sg.size; ++r) {
                    const double v = gv[r];
                    if (f.eps > 0.0 && !(fabs(v / den) > f.eps)) continue;
                    sum = sum + v;
                    ++kept;
                }
                if (kept && (!f.thr || abs_order(sum / den) >= *f.thr)) {
                    const size_t j0 = sg.start;
                    f.clo[j0] = lo;
                    if (W == 2) f.chi[j0] = hi;
                    if (f.cnum) f.cnum[j0] = sum;
                    f.cscore[j0] = sum / den;
                    c = 1;
                }
            }
            f.cnt[sidx] = c;
        }
        return;
    }

    const uint32_t size = sg.size;
    // identity order; the values in record order (permuted in LDS once the
    // sort is done, instead of gathered from memory in sorted order).  One-word
    // keys stay in registers for their windows; two-word keys are read again,
    // from cache.
    uint64_t rk[IT];
    // the bits that vary inside the segment: those in which some key differs
    // from the first (one OR reduction; the constant bits are the first key's)
    const uint64_t k0lo = size ? gk[0] : 0ull, k0hi = (W == 2 && size) ? gh[0] : 0ull;
    {
        uint64_t d0 = 0ull, d1 = 0ull;
        double rv[IT];
        // record r = wv * 64 * IT + k * 64 + lane: the layout of the radix
        // passes' items, so the first pass ranks straight from these registers
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const uint32_t r = (uint32_t)wv * 64 * IT + (uint32_t)k * 64 + (uint32_t)lane;
            rk[k] = r < size ? gk[r] : 0ull;
            rv[k] = r < size ? gv[r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const uint32_t r = (uint32_t)wv * 64 * IT + (uint32_t)k * 64 + (uint32_t)lane;
            if (r < size) {
                S.val[r] = rv[k];
                d0 |= rk[k] ^ k0lo;
                if (W == 2) d1 |= gh[r] ^ k0hi;
            }
        }
        for (int d = 32; d >= 1; d >>= 1) {
            d0 |= __shfl_xor(d0, d, 64);
            if (W == 2) d1 |= __shfl_xor(d1, d, 64);
        }
        if (lane == 0) {
            S.red[0][wv] = d0;
            S.red[1][wv] = d1;
        }
    }
    __syncthreads();
    uint64_t var_lo = 0ull, var_hi = 0ull;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        var_lo |= S.red[0][i];
        if (W == 2) var_hi |= S.red[1][i];
    }
    // the same for every lane: kept in scalar registers
    var_lo = uniform64(var_lo);
    var_hi = uniform64(var_hi);
    const uint64_t and_lo = k0lo & ~var_lo, and_hi = k0hi & ~var_hi;
    const int low = key_low<W>(var_lo, var_hi, n);
    const int span = low < 0 ? 0 : key_top<W>(var_lo, var_hi, n) - low;
    const int nwin = (span + 31) / 32;  // 32-bit windows holding the varying bits

    // stable LSD radix sort of the record indices, one window at a time.  The
    // first pass of one-word keys takes its items (the identity order) and
    // windows from registers and stores the windows for the later passes.
    int cur = 0;
    if (nwin == 0) {
        // one key: no pass runs, the order stays the identity
        for (uint32_t r = tid; r < size; r += NT) S.ix[0][r] = (uint16_t)r;
        __syncthreads();
    }
    for (int win = 0; win < nwin; ++win) {
        const int o = low + 32 * win;
        const uint32_t vwin = key_window<W>(var_lo, var_hi, n, o);
        // the first window comes from the low key words held in registers when
        // it lies inside them (always for one-word keys; for two-word keys when
        // it ends at or below bit n, i.e. inside the beta word)
        const bool regs = win == 0 && (W == 1 || low + 32 <= n);
        if (W == 1 && !regs) {
#pragma unroll
            for (int k = 0; k < IT; ++k) {
                const uint32_t r = (uint32_t)wv * 64 * IT + (uint32_t)k * 64 + (uint32_t)lane;
                if (r < size) S.ck[r] = key_window<W>(rk[k], 0ull, n, o);
            }
        } else if (W == 2 && !regs) {
            for (uint32_t r = tid; r < size; r += NT) S.ck[r] = key_window<W>(gk[r], gh[r], n, o);
            // a first pass of two-word keys not taken from registers reads the
            // identity order from LDS
            if (win == 0)
                for (uint32_t r = tid; r < size; r += NT) S.ix[0][r] = (uint16_t)r;
        }
        if (!regs) __syncthreads();
        for (int sh = 0; sh < 32; sh += 8) {
            const uint32_t dv = (vwin >> sh) & 0xFFu;
            if (dv == 0u) continue;  // no record differs in these bits
            const int w = 32 - __builtin_clz(dv);  // up to the highest varying bit
            const uint32_t dmask = (1u << w) - 1u;
            for (int i = lane; i < (1 << w); i += 64) S.wcnt[wv][i] = 0;
            static_assert(CAP <= 4096, "rank and record index take 12 bits each");
            uint32_t item[IT];  // rank | record << 12 | digit << 24
            // records and digits of all items first, so their loads overlap (the
            // loads are unconditional and in bounds; past the segment's end the
            // values are ignored)
            static_assert((CAP & (CAP - 1)) == 0, "CAP must be a power of two");
            uint32_t cw[IT];
            if (regs && sh == 0) {
                // window 0 always varies in its lowest bit, so this is the first pass
#pragma unroll
                for (int q = 0; q < IT; ++q) {
                    const uint32_t li = (uint32_t)wv * 64 * IT + (uint32_t)q * 64 + lane;
                    item[q] = li;
                    cw[q] = key_window<W>(rk[q], 0ull, n, o);
                    if (li < size) S.ck[li] = cw[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < IT; ++q) {
                    const uint32_t li = (uint32_t)wv * 64 * IT + (uint32_t)q * 64 + lane;
                    item[q] = (uint32_t)S.ix[cur][li] & (uint32_t)(CAP - 1);
                }
#pragma unroll
                for (int q = 0; q < IT; ++q) cw[q] = S.ck[item[q]];
            }
#pragma unroll
            for (int q = 0; q < IT; ++q) {
                const uint32_t li = (uint32_t)wv * 64 * IT + (uint32_t)q * 64 + lane;
                const uint32_t v = (item[q] << 12) | (((cw[q] >> sh) & dmask) << 24);
                item[q] = li < size ? v : 0u;
            }
#pragma unroll
            for (int q = 0; q < IT; ++q) {
                if ((uint32_t)wv * 64 * IT + (uint32_t)q * 64 >= size) break;  // whole wave past the end
                const uint32_t li = (uint32_t)wv * 64 * IT + (uint32_t)q * 64 + lane;
                const bool valid = li < size;
                const uint32_t d = item[q] >> 24;
                const uint64_t peers = wave_match(d, valid, w);
                const uint32_t before = S.wcnt[wv][d];
                item[q] |= before + (uint32_t)__popcll(peers & lt);
                if (valid && (peers & lt) == 0ull) S.wcnt[wv][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
            }
            __syncthreads();
            if (wv == 0) {
                // one wavefront scans the (digit, wave) counts: each lane takes up
                // to four consecutive digits, then one scan across the lanes
                const int nd = 1 << w, dpl = (nd + 63) >> 6;
                uint32_t dsum[4], lane_tot = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    dsum[k] = 0;
                    const int dg = lane * dpl + k;
                    if (k < dpl && dg < nd) {
                        uint32_t run = 0;
#pragma unroll
                        for (int i = 0; i < NW; ++i) {
                            const uint32_t c = S.wcnt[i][dg];
                            S.wcnt[i][dg] = (uint16_t)run;
                            run += c;
                        }
                        dsum[k] = run;
                        lane_tot += run;
                    }
                }
                uint32_t base = wave_incl_scan(lane_tot) - lane_tot;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int dg = lane * dpl + k;
                    if (k < dpl && dg < nd) {
                        S.dbase[dg] = base;
                        base += dsum[k];
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < IT; ++q) {
                const uint32_t li = (uint32_t)wv * 64 * IT + (uint32_t)q * 64 + lane;
                if (li < size) {
                    const uint32_t d = item[q] >> 24;
                    const uint32_t p = min(S.dbase[d] + (uint32_t)S.wcnt[wv][d] + (item[q] & 0xFFFu), (uint32_t)CAP - 1u);
                    S.ix[cur ^ 1][p] = (uint16_t)((item[q] >> 12) & 0xFFFu);
                }
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    // runs of equal keys and the alpha strings among them.  Each thread owns IT
    // consecutive sorted records; one scan of packed counts (runs low, alpha
    // heads high) places both.  With one window the window decides equality,
    // else the keys are read back from the segment.
    uint16_t *head = &S.ix[cur ^ 1][0];
    const uint16_t *perm = &S.ix[cur][0];
    // values in sorted order: each thread gathers the IT consecutive positions
    // it owns below from the record-order copy in LDS and stores them back in
    // sorted order after the scan of the run-head pass (whose barriers order
    // every read before any write)
    double gval[IT];
    {
        const uint32_t j0 = (uint32_t)tid * IT;
#pragma unroll
        for (int i = 0; i < IT; ++i) gval[i] = j0 + i < size ? S.val[perm[j0 + i]] : 0.0;
    }
    const int aw = n - low;  // window bits at or above this one are alpha bits (one-word keys: also two-word)
    const uint32_t cache_bytes = L::kAcacheBytes + (nwin >= 2 ? (uint32_t)sizeof(S.ck) : 0u);
    const uint32_t amax = min(255u, cache_bytes / (8u * (uint32_t)(n + 2)));
    static_assert(offsetof(L, acache) == sizeof(S.ck), "the window array must end where the cache starts");
    double *ealpha = reinterpret_cast<double *>(nwin >= 2 ? (void *)&S.ck[0] : (void *)&S.acache[0]);
    double *colsum = ealpha + amax;
    uint32_t nalpha, nruns;
    {
        const uint32_t j0 = (uint32_t)tid * IT;
        uint32_t flags = 0;  // bit i: run head, bit 16 + i: alpha head
        uint64_t prev_lo = 0ull, prev_hi = 0ull;
        uint32_t prev_c = 0;
        if (j0 > 0 && j0 < size) {
            const uint32_t r = perm[j0 - 1];
            if (nwin >= 2) {
                prev_lo = gk[r];
                prev_hi = W == 2 ? gh[r] : 0ull;
            } else {
                prev_c = nwin ? S.ck[r] : 0u;
            }
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t j = j0 + i;
            if (j >= size) continue;
            const uint32_t r = perm[j];
            bool rh, ah;
            if (nwin >= 2) {
                const uint64_t klo = gk[r], khi = W == 2 ? gh[r] : 0ull;
                rh = j == 0 || klo != prev_lo || khi != prev_hi;
                ah = j == 0 || (W == 1 ? (klo >> n) != (prev_lo >> n) : khi != prev_hi);
                prev_lo = klo;
                prev_hi = khi;
            } else {
                const uint32_t c = nwin ? S.ck[r] : 0u;
                const uint32_t x = c ^ prev_c;
                rh = j == 0 || x != 0u;
                ah = j == 0 || (aw < 32 && (x >> max(aw, 0)) != 0u);
                prev_c = c;
            }
            flags |= (rh ? 1u : 0u) << i;
            flags |= (ah ? 1u : 0u) << (16 + i);
        }
        const uint32_t cnt = (uint32_t)__popc(flags & 0xFFFFu) | ((uint32_t)__popc(flags >> 16) << 16);
        uint32_t tot;
        const uint32_t at = block_scan1<NW>(cnt, S.tmp, parity, tot);
        nruns = tot & 0xFFFFu;
        nalpha = tot >> 16;
        // counts are below 2^16 (size <= CAP <= 4096), so the packed scan is exact
        uint32_t rb = at & 0xFFFFu, ab = at >> 16;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            if ((flags >> (16 + i)) & 1u) ++ab;
            if ((flags >> i) & 1u) {
                head[rb] = (uint16_t)(j0 + i);
                S.aidx[rb] = (uint8_t)min(ab - 1u, 255u);
                ++rb;
            }
        }
        if (tid == 0) head[nruns] = (uint16_t)size;
        // the alpha strings, in order: E(alpha) by the thread that owns the
        // alpha head, the column sums c_q(alpha) by the lanes of its wavefront
        // (one alpha head of the wavefront at a time)
        if (nalpha <= amax) {
            uint32_t ai_next = at >> 16;
            uint32_t pend = (flags >> 16) & ((1u << IT) - 1u);
            for (uint64_t owners = __ballot(pend != 0u); owners; owners = __ballot(pend != 0u)) {
                const int src = __ffsll((long long)owners) - 1;
                uint32_t a_lo = 0u, a_hi = 0u, ai = 0u;
                if (lane == src) {
                    const int i = __ffs(pend) - 1;
                    const uint32_t r = perm[j0 + (uint32_t)i];
                    uint64_t klo = and_lo, khi = and_hi;
                    if (nwin >= 2) {
                        klo = gk[r];
                        khi = W == 2 ? gh[r] : 0ull;
                    } else if (nwin == 1) {
                        key_put<W>(S.ck[r], low, n, klo, khi);
                    }
                    const uint64_t alpha = W == 1 ? (klo >> n) : khi;
                    ai = ai_next++;
                    ealpha[ai] = spin_e(st, 0, X, hd, n, alpha);
                    a_lo = (uint32_t)alpha;
                    a_hi = (uint32_t)(alpha >> 32);
                    pend &= pend - 1u;
                }
                a_lo = __shfl(a_lo, src, 64);
                a_hi = __shfl(a_hi, src, 64);
                ai = __shfl(ai, src, 64);
                const uint64_t alpha = (uint64_t)a_lo | ((uint64_t)a_hi << 32);
                for (int q = lane; q < n; q += 64) colsum[(size_t)ai * n + q] = cross_col(J, n, alpha, q);
            }
        }
#pragma unroll
        for (int i = 0; i < IT; ++i)
            if (j0 + i < size) S.val[j0 + i] = gval[i];
        __syncthreads();
    }
    const bool cached = nalpha <= amax;
    // runs, NT at a time: key (read back from the segment), exclusion,
    // diagonal, sum in record order, score; one scan per round places the
    // surviving candidates, compacted, in run order
    // a lower bound of the final k-th |A| from earlier class batches, if any
    const uint64_t thr = f.thr ? *f.thr : 0ull;
    uint32_t written = 0;
    for (uint32_t base = 0; base < nruns; base += NT) {
        const uint32_t u = base + (uint32_t)tid;
        bool keep = false;
        uint64_t lo = 0ull, hi = 0ull;
        double sum = 0.0, score = 0.0;
        if (u < nruns) {
            const uint32_t j0 = head[u], j1 = head[u + 1];
            const uint32_t r0 = perm[j0];
            lo = and_lo;
            hi = and_hi;
            if (nwin >= 2) {
                lo = gk[r0];
                hi = W == 2 ? gh[r0] : 0ull;
            } else if (nwin == 1) {
                key_put<W>(S.ck[r0], low, n, lo, hi);
            }
            // the exclusion filter is read before H_aa and the sum are formed,
            // so its latency overlaps theirs; the table is probed only when the
            // filter bit is set
            const bool maybe = psi_maybe(f.psi, lo, hi);
            {
                const uint64_t a = W == 1 ? (lo >> n) : hi, b = W == 1 ? (lo & nmask) : lo;
                double haa;
                const uint32_t ai = S.aidx[u];
                // E(beta) first: a table entry read at random from HBM, whose
                // latency then overlaps the LDS work below (the sums keep their order)
                const double eb = cached ? spin_e(st, 1, X, hd, n, b) : 0.0;
                double cross = 0.0;
                if (cached) {
                    const double *cs = colsum + (size_t)ai * n;
                    cross = n <= 32 ? bit_sum<uint32_t>((uint32_t)b, [&](int q) { return cs[q]; })
                                    : bit_sum<uint64_t>(b, [&](int q) { return cs[q]; });
                }
                if (f.eps <= 0.0) {
                    // the run's values, in sorted (= record, ascending core)
                    // order, four in flight at a time, added in order
                    for (uint32_t j = j0; j < j1; j += 4) {
                        double v[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) v[k] = S.val[min(j + (uint32_t)k, j1 - 1u)];
#pragma unroll
                        for (int k = 0; k < 4; ++k) sum = j + (uint32_t)k < j1 ? sum + v[k] : sum;
                    }
                    keep = true;
                }
                if (cached) haa = ((f.ecore + ealpha[ai]) + eb) + cross;
                else haa = diag_tab(st, J, X, hd, n, f.ecore, a, b);
                const double den = f.E0 - haa;
                if (f.eps > 0.0) {
                    // Alg. 2's threshold, per pair
                    for (uint32_t j = j0; j < j1; ++j) {
                        const double v = S.val[j];
                        if (fabs(v / den) > f.eps) {
                            sum = sum + v;
                            keep = true;
                        }
                    }
                }
                score = sum / den;
                keep = keep && abs_order(score) >= thr;
            }
            // an input determinant is not a candidate
            if (maybe && keep) {
                uint32_t sl = psi_hash(lo, hi, f.psi.mask);
                bool found = false;
                for (uint32_t st = f.psi.state[sl]; st != 0u; st = f.psi.state[sl]) {
                    if (f.psi.lo[sl] == lo && f.psi.hi[sl] == hi) {
                        found = true;
                        break;
                    }
                    sl = (sl + 1u) & f.psi.mask;
                }
                keep = !found;
            }
        }
        uint32_t tot;
        const uint32_t at = block_scan1<NW>(keep ? 1u : 0u, S.tmp, parity, tot);
        if (keep) {
            const size_t d = (size_t)sg.start + written + at;
            f.clo[d] = lo;
            if (W == 2) f.chi[d] = hi;
            if (f.cnum) f.cnum[d] = sum;
            f.cscore[d] = score;
        }
        written += tot;
    }
    if (tid == 0) f.cnt[sidx] = written;
}

// persistent workgroups loop over the final segments (a grid of one
// workgroup per segment could exceed the 2^32 work-item limit of a dispatch)
template <int W, int CAP, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_finish(FinishArgs f)
{
    using L = FinishLds<W, CAP, NT>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    L &S = *reinterpret_cast<L *>(smem_raw);
    double *tab = reinterpret_cast<double *>(smem_raw + ((sizeof(L) + 15) & ~size_t(15)));
    const int n = f.n;
    const int tid = threadIdx.x;
    const double *J = f.jk, *X = f.jk + n * n, *hd = f.jk + 2 * n * n;
    SpinTables st = f.st;
    if (f.tab_in_lds == 1) {
        for (int t = tid; t < 2 * n * n; t += NT) tab[t] = f.jk[t];
        for (int t = tid; t < n; t += NT) tab[2 * n * n + t] = f.h[(size_t)t * n + t];
        J = tab;
        X = tab + n * n;
        hd = tab + 2 * n * n;
    } else if (f.tab_in_lds >= 2) {
        // with both spin tables only J and the binomials of the string ranks are read
        const int nj = f.tab_in_lds == 2 ? n * n : 0;
        for (int t = tid; t < nj; t += NT) tab[t] = f.jk[t];
        uint32_t *bt = reinterpret_cast<uint32_t *>(tab + nj);
        for (int t = tid; t < (st.kmax + 4) * (n + 1); t += NT) bt[t] = f.st.binom[t];
        if (nj) J = tab;
        st.binom = bt;
    }
    const uint32_t nf = dev_count(f.nfinal, f.dn_final);
    for (uint32_t sidx = blockIdx.x; sidx < nf; sidx += gridDim.x) {
        __syncthreads();
        finish_segment<W, CAP, NT>(f, st, S, J, X, hd, sidx);
    }
}

// ---------------------------------------------------------------- collect
__global__ __launch_bounds__(256) void k_final_keys_start(const Seg *__restrict__ finals, uint32_t nf,
                                                          uint64_t *__restrict__ key, uint32_t *__restrict__ idx,
                                                          const uint32_t *dn)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dev_count(nf, dn)) return;
    key[j] = finals[j].start;
    idx[j] = j;
}

__global__ __launch_bounds__(256) void k_gather_counts(const uint32_t *__restrict__ order,
                                                       const uint32_t *__restrict__ cnt, uint32_t nf,
                                                       uint32_t *__restrict__ out, const uint32_t *dn)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < dev_count(nf, dn)) out[j] = cnt[order[j]];
}

// one block per final segment (in key order): copy its candidates to the pool
template <int W>
__global__ __launch_bounds__(256) void k_collect(const Seg *__restrict__ finals, uint32_t nf,
                                                 const uint32_t *__restrict__ order,
                                                 const uint32_t *__restrict__ cnt_sorted,
                                                 const uint32_t *__restrict__ off, const uint64_t *__restrict__ clo,
                                                 const uint64_t *__restrict__ chi, const double *__restrict__ cnum,
                                                 const double *__restrict__ cscore, uint64_t *__restrict__ plo,
                                                 uint64_t *__restrict__ phi, double *__restrict__ pnum,
                                                 double *__restrict__ pscore, size_t base, size_t cap,
                                                 const uint32_t *dn)
{
    nf = dev_count(nf, dn);
    for (uint32_t j = blockIdx.x; j < nf; j += gridDim.x) {
        const Seg sg = finals[order[j]];
        const uint32_t c = cnt_sorted[j];
        const size_t dst0 = base + off[j];
        for (uint32_t t = threadIdx.x; t < c; t += 256) {
            const size_t s = (size_t)sg.start + t, d = dst0 + t;
            if (d >= cap) {
                raise_fault(kFaultSlot);
                break;
            }
            plo[d] = clo[s];
            if (W == 2) phi[d] = chi[s];
            if (pnum) pnum[d] = cnum[s];
            pscore[d] = cscore[s];
        }
    }
}

constexpr uint32_t kMaxClassSegs = 2048;  // classes of one batch

__global__ __launch_bounds__(256) void k_class_segs(const uint64_t *__restrict__ cls, uint32_t c0, uint32_t nc,
                                                    uint32_t nq, const uint32_t *__restrict__ offsets,
                                                    const uint32_t *__restrict__ total, int n, uint32_t cap,
                                                    Seg *__restrict__ large, uint32_t *__restrict__ nlarge,
                                                    Seg *__restrict__ finals, uint32_t *__restrict__ nfinal,
                                                    uint32_t nrec)
{
    // class bounds and masks staged in LDS in parallel; one thread then walks
    // the classes (the counters start at zero and this kernel is their only
    // writer).  Bounds are clamped to the record buffer (nrec records): counts
    // that overrun it (inputs that fail validation) cannot send a segment past it.
    __shared__ uint32_t s_start[kMaxClassSegs + 1];
    __shared__ uint64_t s_cls[kMaxClassSegs];
    for (uint32_t c = threadIdx.x; c < nc; c += 256) {
        s_start[c] = min(offsets[(size_t)c * nq], nrec);
        s_cls[c] = cls[c0 + c];
    }
    if (threadIdx.x == 0) s_start[nc] = min(*total, nrec);
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t nf = 0, nl = 0;
    // a class's keys share every bit at or above n + (lowest bit of its mask);
    // a run of classes shares the bits above the highest bit where its first
    // lower bound and last upper bound differ
    uint32_t g_start = 0, g_size = 0;
    uint64_t g_first = 0, g_last = 0;  // masks of the run's first and last class
    bool g_one = true;                 // the run holds one class
    auto top_of = [&](uint64_t Tf, uint64_t Tl, bool one) -> uint32_t {
        const int of = Tf ? __ffsll((unsigned long long)Tf) - 1 : 0;
        const int ol = Tl ? __ffsll((unsigned long long)Tl) - 1 : 0;
        if (one) return (uint32_t)(n + of);
        // alpha range [Tf, Tl | (2^ol - 1)]
        const uint64_t lo = Tf, hi = Tl | ((1ull << ol) - 1ull);
        const uint64_t diff = lo ^ hi;
        return (uint32_t)n + (diff ? (uint32_t)(64 - __clzll((long long)diff)) : 0u);
    };
    auto flush = [&]() {
        if (g_size) finals[nf++] = Seg{g_start, g_size, make_meta(top_of(g_first, g_last, g_one), 0u, false)};
        g_size = 0;
    };
    // eight classes' bounds and masks are read at a time, so the walk waits on
    // LDS once per eight classes
    uint32_t prev = s_start[0];
    for (uint32_t cb = 0; cb < nc; cb += 8) {
        uint32_t e8[8];
        uint64_t t8[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t c = min(cb + (uint32_t)k, nc - 1u);
            e8[k] = s_start[c + 1];
            t8[k] = s_cls[c];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (cb + (uint32_t)k >= nc) break;
            const uint32_t start = prev, end = e8[k];
            prev = end;
            if (end <= start) continue;
            const uint32_t size = end - start;
            if (size > cap) {
                flush();
                large[nl++] = Seg{start, size, make_meta(top_of(t8[k], t8[k], true), 0u, false)};
                continue;
            }
            if (g_size + size > cap) flush();
            if (g_size == 0) {
                g_start = start;
                g_first = t8[k];
                g_one = true;
            } else {
                g_one = false;
            }
            g_size += size;
            g_last = t8[k];
        }
    }
    flush();
    *nfinal = nf;
    *nlarge = nl;
}

}  // namespace

// ---------------------------------------------------------------- host side
size_t bucket_workspace_bytes(size_t P, size_t nc, int W, int finish_cap)
{
    const size_t cap = finish_cap >= 4096 ? 4096 : (finish_cap >= 2048 ? 2048 : 1024);
    const size_t finals = nc + P / 8 + 65536, level = P / cap + nc + 16;
    const size_t tiles = (P + kTileN - 1) / kTileN + level;
    return finals * sizeof(Seg) + 2 * level * sizeof(Seg) + level * 16 + tiles * (256 * 8 + 8) +
           level * ((kMaxSplit - 1) * 8 * W + 32) + P + 256 + finals * (8 * 2 + 4 * 4 + 8) + (finals + tiles * 256) / 1024 +
           (4 << 20);
}

// LDS per workgroup: the table of J, J-K and h_pp is staged when the whole
// still lets two workgroups share a CU (their barriers then overlap)
constexpr size_t kFinishLdsBudget = 80 * 1024;

template <int W, int CAP, int NT>
static int launch_finish(FinishArgs &fa, const BucketArgs &b, uint32_t nf, hipStream_t s, Profiler *prof)
{
    const size_t base_lds = (sizeof(FinishLds<W, CAP, NT>) + 15) & ~size_t(15);
    const size_t n = (size_t)b.n;
    size_t tab_lds = 0;
    fa.tab_in_lds = 0;
    if (b.st.e[0] && b.st.e[1]) {
        // E(alpha), E(beta) are looked up: stage J and the binomials, else the binomials
        const size_t bin = (size_t)(b.st.kmax + 4) * (n + 1) * 4;
        if (base_lds + n * n * 8 + bin <= kFinishLdsBudget) {
            fa.tab_in_lds = 2;
            tab_lds = n * n * 8 + bin;
        } else if (base_lds + bin <= kFinishLdsBudget) {
            fa.tab_in_lds = 3;
            tab_lds = bin;
        }
    } else if (base_lds + (2 * n * n + n) * 8 <= kFinishLdsBudget) {
        fa.tab_in_lds = 1;
        tab_lds = (2 * n * n + n) * 8;
    }
    const size_t lds = base_lds + ((tab_lds + 15) & ~size_t(15));
    const void *fn = (const void *)k_finish<W, CAP, NT>;
    ASCI_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int dev = 0, ncu = 0, per_cu = 0;
    ASCI_HIP(hipGetDevice(&dev));
    ASCI_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    ASCI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds));
    // one resident grid: every workgroup strides over the segments
    const uint32_t grid = std::min<uint32_t>(nf, (uint32_t)std::max(1, ncu * std::max(per_cu, 1)));
    // bytes: every record read once; the candidates it writes are added once
    // their number is known (finish_bytes)
    ProfScope ps(prof, "finish", (8.0 * W + 8.0) * (double)b.P, s);
    k_finish<W, CAP, NT><<<grid, NT, lds, s>>>(fa);
    ASCI_LAUNCH_CHECK();
    return ps.tok;
}

// algorithmic bytes of a finish launch: records read, candidates written
// (key and score, plus N_a when every candidate is kept)
static void finish_bytes(const BucketArgs &b, int W)
{
    if (b.prof && b.finish_tok >= 0)
        b.prof->set_bytes(b.finish_tok, (8.0 * W + 8.0) * (double)b.P +
                                            (8.0 * W + 8.0 + (b.cnum ? 8.0 : 0.0)) * (double)b.V);
}

template <int W>
void bucket_accumulate(BucketArgs &b, Arena &ar, hipStream_t s, Profiler *prof, HostStage &hs)
{
    // LDS capacity of a final segment: 4096, 2048 or 1024 records
    const int CAP = b.finish_cap >= 4096 ? 4096 : (b.finish_cap >= 2048 ? 2048 : 1024);
    const size_t P = b.P;
    const uint32_t finals_cap = (uint32_t)std::min<size_t>(b.nc + P / 8 + 65536, 0xFFFFFFF0u);
    const uint32_t level_cap = (uint32_t)(P / CAP + b.nc + 16);
    Seg *finals = ar.take<Seg>(finals_cap);
    Seg *lv[2] = {ar.take<Seg>(level_cap), ar.take<Seg>(level_cap)};
    uint32_t *ctr = ar.take<uint32_t>(8);  // 0: finals, 1/2: large segments per level parity, 3: overflow
    uint32_t *hcnt = (uint32_t *)hs.ptr;
    ASCI_HIP(hipMemsetAsync(ctr, 0, 8 * sizeof(uint32_t), s));
    require(b.nc <= kMaxClassSegs, ASCI_EINVAL, "too many classes in one batch");
    k_class_segs<<<1, 256, 0, s>>>(b.cls, b.c0, b.nc, b.nq, b.offsets, b.total, b.n, (uint32_t)CAP, lv[0], ctr + 1,
                                   finals, ctr, (uint32_t)std::min<size_t>(P, 0xFFFFFFFFu));
    ASCI_LAUNCH_CHECK();
    ASCI_HIP(hipMemcpyAsync(hcnt, ctr, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    uint32_t nlarge = hcnt[1];
    int lev = 0;
    uint8_t *dig = ar.take<uint8_t>(P + 1);
    const size_t mark = ar.used();
    while (nlarge > 0) {
        ar.reset();
        (void)ar.take<char>(mark);
        require(lev < 64, ASCI_EDEVICE, "bucket split did not converge");
        Seg *segs = lv[lev & 1], *next = lv[(lev & 1) ^ 1];
        uint32_t *nnext = ctr + 1 + ((lev & 1) ^ 1);
        uint32_t *ntile = ar.take<uint32_t>(nlarge + 1);
        uint32_t *tbase = ar.take<uint32_t>(nlarge + 1);
        uint32_t *skip = ar.take<uint32_t>(nlarge + 1);
        uint32_t *d_ntiles = ar.take<uint32_t>(4);
        k_seg_tiles<<<(nlarge + 256) / 256, 256, 0, s>>>(segs, nlarge, ntile, skip, nnext, nullptr);
        ASCI_LAUNCH_CHECK();
        scan_u32(ntile, tbase, nlarge, d_ntiles, ar, s, prof);
        ASCI_HIP(hipMemcpyAsync(hcnt + 4, d_ntiles, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        const uint32_t ntiles = hcnt[4];
        uint32_t *tseg = ar.take<uint32_t>(ntiles + 1);
        uint32_t *hist = ar.take<uint32_t>((size_t)ntiles * 256 + 1);
        uint32_t *hscan = ar.take<uint32_t>((size_t)ntiles * 256 + 1);
        uint64_t *spl_lo = ar.take<uint64_t>((size_t)nlarge * (kMaxSplit - 1));
        uint64_t *spl_hi = W == 2 ? ar.take<uint64_t>((size_t)nlarge * (kMaxSplit - 1)) : nullptr;
        unsigned long long *kvar = ar.take<unsigned long long>(2 * (size_t)nlarge);
        k_seg_expand<<<(nlarge + 255) / 256, 256, 0, s>>>(segs, nlarge, tbase, tseg, kvar, nullptr);
        ASCI_LAUNCH_CHECK();
        {
            ProfScope ps(prof, "split_sample", 0.0, s);
            const KeyBufs kb{{b.klo[0], b.klo[1]}, {b.khi[0], b.khi[1]}};
            // class-sized segments of the first level sort up to 4096 samples:
            // more threads per sort; later levels sort a few hundred
            if (lev == 0) k_seg_splitters<W, 1024><<<nlarge, 1024, 0, s>>>(segs, (uint32_t)CAP, kb, spl_lo, spl_hi, nlarge, nullptr);
            else k_seg_splitters<W, 256><<<nlarge, 256, 0, s>>>(segs, (uint32_t)CAP, kb, spl_lo, spl_hi, nlarge, nullptr);
            ASCI_LAUNCH_CHECK();
        }
        SplitArgs sa;
        sa.segs = segs;
        sa.nseg = nlarge;
        sa.tile_base = tbase;
        sa.tile_seg = tseg;
        sa.ntiles = ntiles;
        sa.hist = hist;
        sa.klo[0] = b.klo[0];
        sa.klo[1] = b.klo[1];
        sa.khi[0] = b.khi[0];
        sa.khi[1] = b.khi[1];
        sa.val[0] = b.val[0];
        sa.val[1] = b.val[1];
        sa.n = b.n;
        sa.cap = (uint32_t)CAP;
        sa.spl_lo = spl_lo;
        sa.spl_hi = spl_hi;
        sa.kvar = kvar;
        sa.dig = dig;
        {
            ProfScope ps(prof, "split_hist", (8.0 * W) * (double)ntiles * kTileN, s);
            k_split_hist<W><<<8 * ((ntiles + 7) / 8), kHistT, 0, s>>>(sa);
            ASCI_LAUNCH_CHECK();
        }
        scan_u32(hist, hscan, (size_t)ntiles * 256, nullptr, ar, s, prof);
        k_split_children<W><<<nlarge, 256, 0, s>>>(segs, nlarge, tbase, hscan, (uint32_t)CAP, skip, finals, ctr,
                                                   finals_cap, next, nnext, level_cap, ctr + 3, kvar, b.n, nullptr);
        ASCI_LAUNCH_CHECK();
        sa.hist = hscan;
        {
            ProfScope ps(prof, "split_scatter", 2.0 * (8.0 * W + 8.0) * (double)ntiles * kTileN, s);
            k_split_scatter<W><<<8 * ((ntiles + 7) / 8), kTileT, 0, s>>>(sa, hscan, skip);
            ASCI_LAUNCH_CHECK();
        }
        ASCI_HIP(hipMemcpyAsync(hcnt, ctr, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        require(hcnt[3] == 0, ASCI_EDEVICE, "bucket segment list overflow");
        nlarge = hcnt[1 + ((lev & 1) ^ 1)];
        ++lev;
    }
    ar.reset();
    (void)ar.take<char>(mark);
    const uint32_t nf = hcnt[0];
    b.nfinal = nf;
    b.levels = (uint32_t)lev;
    uint32_t *cnt = ar.take<uint32_t>(nf + 1);
    if (nf) {
        FinishArgs fa;
        fa.finals = finals;
        fa.klo[0] = b.klo[0];
        fa.klo[1] = b.klo[1];
        fa.khi[0] = b.khi[0];
        fa.khi[1] = b.khi[1];
        fa.val[0] = b.val[0];
        fa.val[1] = b.val[1];
        fa.n = b.n;
        fa.jk = b.jk;
        fa.h = b.h;
        fa.st = b.st;
        fa.thr = b.thr;
        fa.ecore = b.ecore;
        fa.E0 = b.E0;
        fa.eps = b.eps;
        fa.clo = b.clo;
        fa.chi = b.chi;
        fa.cnum = b.cnum;
        fa.cscore = b.cscore;
        fa.cnt = cnt;
        fa.nfinal = nf;
        fa.dn_final = nullptr;
        fa.psi = b.psi;
        // eight records per thread
        b.prof = prof;
        if (CAP == 4096) b.finish_tok = launch_finish<W, 4096, 512>(fa, b, nf, s, prof);
        else if (CAP == 2048) b.finish_tok = launch_finish<W, 2048, 256>(fa, b, nf, s, prof);
        else b.finish_tok = launch_finish<W, 1024, 128>(fa, b, nf, s, prof);
    }
    // candidates in key order: final segments by start, counts scanned
    uint64_t *sk[2] = {ar.take<uint64_t>(nf + 1), ar.take<uint64_t>(nf + 1)};
    uint32_t *si[2] = {ar.take<uint32_t>(nf + 1), ar.take<uint32_t>(nf + 1)};
    uint32_t *cs = ar.take<uint32_t>(nf + 1);
    uint32_t *co = ar.take<uint32_t>(nf + 1);
    uint32_t *d_v = ar.take<uint32_t>(4);
    uint64_t *nohi[2] = {nullptr, nullptr};
    int r = 0;
    if (nf) {
        k_final_keys_start<<<(nf + 255) / 256, 256, 0, s>>>(finals, nf, sk[0], si[0], nullptr);
        ASCI_LAUNCH_CHECK();
        std::vector<Digit> dg;
        for (int sh = 0; sh < 32; sh += 8) dg.push_back({0, sh});
        r = radix_sort<uint32_t>(sk, nohi, si, nf, 1, dg, ar, s, nullptr);
        k_gather_counts<<<(nf + 255) / 256, 256, 0, s>>>(si[r], cnt, nf, cs, nullptr);
        ASCI_LAUNCH_CHECK();
    }
    scan_u32(cs, co, nf, d_v, ar, s, nullptr);
    ASCI_HIP(hipMemcpyAsync(hcnt + 6, d_v, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    b.h_v = hcnt + 6;
    if (b.defer_v) {
        b.V = ~0u;  // unknown until bucket_read_v
    } else {
        ASCI_HIP(hipStreamSynchronize(s));
        b.V = hcnt[6];
        finish_bytes(b, W);
    }
    b.order = si[r];
    b.cnt_sorted = cs;
    b.off = co;
    b.finals = finals;
}

template <int W>
int bucket_collect(BucketArgs &b, hipStream_t s, Profiler *prof)
{
    if (b.nfinal == 0 || b.V == 0) return -1;
    // with the count still in flight the bytes are set once it is known
    ProfScope ps(prof, "collect", b.defer_v ? 0.0 : (8.0 * W + 8.0) * 2.0 * b.V, s);
    k_collect<W><<<std::min<uint32_t>(b.nfinal, 65536u), 256, 0, s>>>((const Seg *)b.finals, b.nfinal, b.order, b.cnt_sorted, b.off, b.clo, b.chi, b.cnum,
                                         b.cscore, b.pool_lo, b.pool_hi, b.pool_num, b.pool_score, b.pool_base,
                                         b.pool_cap, nullptr);
    ASCI_LAUNCH_CHECK();
    return ps.tok;
}

void bucket_read_v(BucketArgs &b, hipStream_t s)
{
    if (!b.defer_v) return;
    ASCI_HIP(hipStreamSynchronize(s));
    b.V = *b.h_v;
    b.defer_v = false;
    finish_bytes(b, b.n <= 32 ? 1 : 2);
}

// sum of N_a * A_a over the batch's candidates: per final segment in key
// order (sequential inside a segment), then a fixed-order tree over segments
__global__ __launch_bounds__(256) void k_pt2_segments(const Seg *__restrict__ finals, uint32_t nf,
                                                      const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ cnt_sorted,
                                                      const double *__restrict__ cnum,
                                                      const double *__restrict__ cscore, double *__restrict__ part)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nf) return;
    const Seg sg = finals[order[j]];
    double e = 0.0;
    for (uint32_t t = 0; t < cnt_sorted[j]; ++t) e = e + cnum[sg.start + t] * cscore[sg.start + t];
    part[j] = e;
}

__global__ __launch_bounds__(1024) void k_sum_fixed(const double *__restrict__ x, uint32_t n, double *__restrict__ out)
{
    __shared__ double sh[1024];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += 1024) acc = acc + x[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (threadIdx.x < (unsigned)w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

double bucket_pt2(BucketArgs &b, Arena &ar, hipStream_t s, HostStage &hs)
{
    if (b.nfinal == 0) return 0.0;
    double *part = ar.take<double>(b.nfinal);
    double *tot = ar.take<double>(1);
    k_pt2_segments<<<(b.nfinal + 255) / 256, 256, 0, s>>>((const Seg *)b.finals, b.nfinal, b.order, b.cnt_sorted,
                                                          b.cnum, b.cscore, part);
    ASCI_LAUNCH_CHECK();
    k_sum_fixed<<<1, 1024, 0, s>>>(part, b.nfinal, tot);
    ASCI_LAUNCH_CHECK();
    double *h = (double *)((char *)hs.ptr + 128);
    ASCI_HIP(hipMemcpyAsync(h, tot, sizeof(double), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    return *h;
}

// ---------------------------------------------------------------- device-driven variant
constexpr int kDevLevels = 8;  // split levels run when no count is read back

__global__ __launch_bounds__(64) void k_times256(const uint32_t *__restrict__ n, uint32_t *__restrict__ out)
{
    if (threadIdx.x == 0) *out = *n * 256u;
}

// after the last level: segments still too large for the finish, or a list
// that overflowed its capacity, fail the call
__global__ __launch_bounds__(64) void k_levels_done(const uint32_t *__restrict__ ctr, int last_parity,
                                                    uint32_t *__restrict__ stat)
{
    if (threadIdx.x != 0) return;
    if (ctr[1 + last_parity] != 0u || ctr[3] != 0u) atomicOr(stat, kStatSplit);
}

template <int W>
void bucket_accumulate_dev(BucketArgs &b, Arena &ar, hipStream_t s, uint32_t *d_stat)
{
    const int CAP = b.finish_cap >= 4096 ? 4096 : (b.finish_cap >= 2048 ? 2048 : 1024);
    const size_t P = b.P;
    const uint32_t finals_cap = (uint32_t)std::min<size_t>(b.nc + P / 8 + 65536, 0xFFFFFFF0u);
    const uint32_t level_cap = (uint32_t)(P / CAP + b.nc + 16);
    const uint32_t max_tiles = (uint32_t)((P + kTileN - 1) / kTileN + level_cap);
    Seg *finals = ar.take<Seg>(finals_cap);
    Seg *lv[2] = {ar.take<Seg>(level_cap), ar.take<Seg>(level_cap)};
    uint32_t *ctr = ar.take<uint32_t>(8);  // 0: finals, 1/2: large segments per level parity, 3: overflow
    require(b.nc <= kMaxClassSegs, ASCI_EINVAL, "too many classes in one batch");
    fill_u32(ctr, 8, 0u, s);
    k_class_segs<<<1, 256, 0, s>>>(b.cls, b.c0, b.nc, b.nq, b.offsets, b.total, b.n, (uint32_t)CAP, lv[0], ctr + 1,
                                   finals, ctr, (uint32_t)std::min<size_t>(P, 0xFFFFFFFFu));
    ASCI_LAUNCH_CHECK();
    uint8_t *dig = ar.take<uint8_t>(P + 1);
    uint32_t *ntile = ar.take<uint32_t>((size_t)level_cap + 1);
    uint32_t *tbase = ar.take<uint32_t>((size_t)level_cap + 1);
    uint32_t *skip = ar.take<uint32_t>((size_t)level_cap + 1);
    uint32_t *d_ntiles = ar.take<uint32_t>(4);
    uint32_t *tseg = ar.take<uint32_t>((size_t)max_tiles + 1);
    uint32_t *hist = ar.take<uint32_t>((size_t)max_tiles * 256 + 1);
    uint32_t *hscan = ar.take<uint32_t>((size_t)max_tiles * 256 + 1);
    uint64_t *spl_lo = ar.take<uint64_t>((size_t)level_cap * (kMaxSplit - 1));
    uint64_t *spl_hi = W == 2 ? ar.take<uint64_t>((size_t)level_cap * (kMaxSplit - 1)) : nullptr;
    unsigned long long *kvar = ar.take<unsigned long long>(2 * (size_t)level_cap);
    // launch shapes: per-segment kernels stride over the level's segments, tile
    // kernels over its tiles (eight XCD groups of workgroups)
    const unsigned g_seg = std::min<uint32_t>(level_cap, 2048u);
    const unsigned g_seg256 = std::min<uint32_t>((level_cap + 256) / 256, 1024u);
    const unsigned g_tiles = 8u * std::min<uint32_t>((max_tiles + 7) / 8, 256u);
    const size_t mark = ar.used();
    const KeyBufs kb{{b.klo[0], b.klo[1]}, {b.khi[0], b.khi[1]}};
    for (int lev = 0; lev < kDevLevels; ++lev) {
        ar.reset();
        (void)ar.take<char>(mark);
        Seg *segs = lv[lev & 1], *next = lv[(lev & 1) ^ 1];
        const uint32_t *dn_seg = ctr + 1 + (lev & 1);
        uint32_t *nnext = ctr + 1 + ((lev & 1) ^ 1);
        k_seg_tiles<<<g_seg256, 256, 0, s>>>(segs, level_cap, ntile, skip, nnext, dn_seg);
        ASCI_LAUNCH_CHECK();
        scan_u32(ntile, tbase, level_cap, d_ntiles, ar, s, nullptr, dn_seg);
        k_seg_expand<<<g_seg256, 256, 0, s>>>(segs, level_cap, tbase, tseg, kvar, dn_seg);
        ASCI_LAUNCH_CHECK();
        if (lev == 0) k_seg_splitters<W, 1024><<<g_seg, 1024, 0, s>>>(segs, (uint32_t)CAP, kb, spl_lo, spl_hi, level_cap, dn_seg);
        else k_seg_splitters<W, 256><<<g_seg, 256, 0, s>>>(segs, (uint32_t)CAP, kb, spl_lo, spl_hi, level_cap, dn_seg);
        ASCI_LAUNCH_CHECK();
        SplitArgs sa;
        sa.segs = segs;
        sa.nseg = level_cap;
        sa.tile_base = tbase;
        sa.tile_seg = tseg;
        sa.ntiles = max_tiles;
        sa.hist = hist;
        sa.klo[0] = b.klo[0];
        sa.klo[1] = b.klo[1];
        sa.khi[0] = b.khi[0];
        sa.khi[1] = b.khi[1];
        sa.val[0] = b.val[0];
        sa.val[1] = b.val[1];
        sa.n = b.n;
        sa.cap = (uint32_t)CAP;
        sa.spl_lo = spl_lo;
        sa.spl_hi = spl_hi;
        sa.kvar = kvar;
        sa.dig = dig;
        sa.dn_seg = dn_seg;
        sa.dn_tiles = d_ntiles;
        k_split_hist<W><<<g_tiles, kHistT, 0, s>>>(sa);
        ASCI_LAUNCH_CHECK();
        k_times256<<<1, 64, 0, s>>>(d_ntiles, d_ntiles + 1);
        ASCI_LAUNCH_CHECK();
        scan_u32(hist, hscan, (size_t)max_tiles * 256, nullptr, ar, s, nullptr, d_ntiles + 1);
        k_split_children<W><<<g_seg, 256, 0, s>>>(segs, level_cap, tbase, hscan, (uint32_t)CAP, skip, finals, ctr,
                                                  finals_cap, next, nnext, level_cap, ctr + 3, kvar, b.n, dn_seg);
        ASCI_LAUNCH_CHECK();
        sa.hist = hscan;
        k_split_scatter<W><<<g_tiles, kTileT, 0, s>>>(sa, hscan, skip);
        ASCI_LAUNCH_CHECK();
    }
    k_levels_done<<<1, 64, 0, s>>>(ctr, kDevLevels & 1, d_stat);
    ASCI_LAUNCH_CHECK();
    ar.reset();
    (void)ar.take<char>(mark);
    uint32_t *cnt = ar.take<uint32_t>((size_t)finals_cap + 1);
    FinishArgs fa;
    fa.finals = finals;
    fa.klo[0] = b.klo[0];
    fa.klo[1] = b.klo[1];
    fa.khi[0] = b.khi[0];
    fa.khi[1] = b.khi[1];
    fa.val[0] = b.val[0];
    fa.val[1] = b.val[1];
    fa.n = b.n;
    fa.jk = b.jk;
    fa.h = b.h;
    fa.st = b.st;
    fa.thr = nullptr;
    fa.ecore = b.ecore;
    fa.E0 = b.E0;
    fa.eps = b.eps;
    fa.clo = b.clo;
    fa.chi = b.chi;
    fa.cnum = b.cnum;
    fa.cscore = b.cscore;
    fa.cnt = cnt;
    fa.nfinal = finals_cap;
    fa.dn_final = ctr;
    fa.psi = b.psi;
    if (CAP == 4096) (void)launch_finish<W, 4096, 512>(fa, b, finals_cap, s, nullptr);
    else if (CAP == 2048) (void)launch_finish<W, 2048, 256>(fa, b, finals_cap, s, nullptr);
    else (void)launch_finish<W, 1024, 128>(fa, b, finals_cap, s, nullptr);
    // candidates in key order: final segments by start, counts scanned
    uint64_t *sk[2] = {ar.take<uint64_t>((size_t)finals_cap + 1), ar.take<uint64_t>((size_t)finals_cap + 1)};
    uint32_t *si[2] = {ar.take<uint32_t>((size_t)finals_cap + 1), ar.take<uint32_t>((size_t)finals_cap + 1)};
    uint32_t *cs = ar.take<uint32_t>((size_t)finals_cap + 1);
    uint32_t *co = ar.take<uint32_t>((size_t)finals_cap + 1);
    uint32_t *d_v = ar.take<uint32_t>(4);
    uint64_t *nohi[2] = {nullptr, nullptr};
    const unsigned gf = std::min<uint32_t>((finals_cap + 255) / 256, 65535u);
    k_final_keys_start<<<(finals_cap + 255) / 256, 256, 0, s>>>(finals, finals_cap, sk[0], si[0], ctr);
    ASCI_LAUNCH_CHECK();
    std::vector<Digit> dg;
    for (int sh = 0; sh < 32; sh += 8) dg.push_back({0, sh});
    const int r = radix_sort<uint32_t>(sk, nohi, si, finals_cap, 1, dg, ar, s, nullptr, ctr);
    k_gather_counts<<<(finals_cap + 255) / 256, 256, 0, s>>>(si[r], cnt, finals_cap, cs, ctr);
    ASCI_LAUNCH_CHECK();
    scan_u32(cs, co, finals_cap, d_v, ar, s, nullptr, ctr);
    (void)gf;
    b.nfinal = finals_cap;  // a bound: the count is *dn_final
    b.dn_final = ctr;
    b.dn_V = d_v;
    b.V = (uint32_t)std::min<size_t>(P, 0xFFFFFFFFu);  // a bound: the count is *dn_V
    b.order = si[r];
    b.cnt_sorted = cs;
    b.off = co;
    b.finals = finals;
}

// the collect of the device-driven variant: counts read on the device
template <int W>
void bucket_collect_dev(BucketArgs &b, hipStream_t s)
{
    k_collect<W><<<std::min<uint32_t>(b.nfinal, 65536u), 256, 0, s>>>(
        (const Seg *)b.finals, b.nfinal, b.order, b.cnt_sorted, b.off, b.clo, b.chi, b.cnum, b.cscore, b.pool_lo,
        b.pool_hi, b.pool_num, b.pool_score, b.pool_base, b.pool_cap, b.dn_final);
    ASCI_LAUNCH_CHECK();
}

template void bucket_accumulate_dev<1>(BucketArgs &, Arena &, hipStream_t, uint32_t *);
template void bucket_accumulate_dev<2>(BucketArgs &, Arena &, hipStream_t, uint32_t *);
template void bucket_collect_dev<1>(BucketArgs &, hipStream_t);
template void bucket_collect_dev<2>(BucketArgs &, hipStream_t);

void bucket_fault_clear(hipStream_t s) { fault_clear(s); }
void bucket_fault_reset_dev(hipStream_t s)
{
    k_fault_reset<<<1, 64, 0, s>>>();
    ASCI_LAUNCH_CHECK();
}
void bucket_fault_take_dev(uint32_t *stat, uint32_t bit, hipStream_t s)
{
    k_fault_take<<<1, 64, 0, s>>>(stat, bit);
    ASCI_LAUNCH_CHECK();
}
void bucket_fault_fetch(unsigned int *dst, hipStream_t s) { fault_fetch(dst, s); }

template void bucket_accumulate<1>(BucketArgs &, Arena &, hipStream_t, Profiler *, HostStage &);
template void bucket_accumulate<2>(BucketArgs &, Arena &, hipStream_t, Profiler *, HostStage &);
template int bucket_collect<1>(BucketArgs &, hipStream_t, Profiler *);
template int bucket_collect<2>(BucketArgs &, hipStream_t, Profiler *);

}  // namespace asci
