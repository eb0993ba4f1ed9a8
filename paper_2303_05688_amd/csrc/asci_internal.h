// Internal declarations of the ASCI search library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/asci.h"

namespace asci {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string what;
};

#define ASCI_HIP(call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            throw ::asci::Error{e_ == hipErrorOutOfMemory ? ASCI_ENOMEM : ASCI_EDEVICE, \
                                std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define ASCI_LAUNCH_CHECK() ASCI_HIP(hipGetLastError())

inline void require(bool ok, int code, const char *what)
{
    if (!ok)
        throw Error{code, what};
}

// ---------------------------------------------------------------- workspace
// A bump allocator over one device allocation that grows on demand.  Every
// search carves its buffers from it; nothing is freed until the context dies.
// An attached arena carves from memory it does not own (a fixed region) and
// never allocates: a reserve beyond the region fails with ASCI_ENOMEM.
class Arena {
  public:
    ~Arena() { release(); }
    void reserve(size_t bytes);  // ensure capacity; invalidates earlier carves
    void attach(void *base, size_t bytes)
    {
        release();
        base_ = (char *)base;
        cap_ = bytes;
        used_ = 0;
        fixed_ = true;
    }
    void reset() { used_ = 0; }
    template <typename T> T *take(size_t count)
    {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        require(used_ + bytes <= cap_, ASCI_ENOMEM, "workspace exhausted (internal sizing error)");
        T *p = reinterpret_cast<T *>(base_ + used_);
        used_ += bytes;
        return p;
    }
    size_t used() const { return used_; }
    size_t capacity() const { return cap_; }
    void release();

  private:
    char *base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    bool fixed_ = false;
};

// Pinned host staging for small device->host reads.  An attached stage uses
// host memory it does not own and never allocates.
struct HostStage {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;
    void reserve(size_t b);
    void attach(void *p, size_t b)
    {
        ptr = p;
        bytes = b;
        fixed = true;
    }
    ~HostStage();
};

// Per-kernel timing with HIP events on the launching stream (opt-in).  Each
// timed launch also carries its algorithmic byte count, so achieved bandwidth
// can be derived from the events alone.
struct ProfEntry {
    std::string name;
    double ms = 0.0;
    int64_t launches = 0;
    double bytes = 0.0;
};

class Profiler {
  public:
    ~Profiler();
    bool on = false;
    std::string only;  // non-empty: time only launches of this name
    std::vector<ProfEntry> entries;
    int begin(const char *name, double bytes, hipStream_t s);  // -1 when off
    void end(int token, hipStream_t s);
    void set_bytes(int token, double bytes);  // bytes of a launch only known later
    void collect();  // after the stream has been synchronised
    void reset();

  private:
    struct Pending {
        int entry;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Pending> pending_;
    std::vector<hipEvent_t> pool_;
    hipEvent_t get_event();
};

// RAII helper: times the launches issued in its scope
struct ProfScope {
    Profiler *p;
    int tok;
    hipStream_t s;
    ProfScope(Profiler *p_, const char *name, double bytes, hipStream_t s_) : p(p_), tok(-1), s(s_)
    {
        if (p && p->on && (p->only.empty() || p->only == name)) tok = p->begin(name, bytes, s);
    }
    ~ProfScope()
    {
        if (p && tok >= 0) p->end(tok, s);
    }
};

}  // namespace asci

struct asci_ctx {
    int device = 0;
    int finish_cap = 4096;  // tunable: records per LDS bucket (see asci_ctx_set_param)
    int batch_slots = 4;    // tunable: concurrent searches of a batch
    int spin_tables = 1;    // tunable: 1 = spin-string energy tables when they pay, 0 = never
    int fault_test = 0;     // 1: the next search raises a forced fault (tests of the error path)
    int batch_graph = 0;    // 1: batch requests within the asynchronous search's scope run as one graph
    int64_t batch_solo_pairs = (int64_t)1 << 26;  // batch requests with this many pairs run alone (0: none)
    int use_tuned = 1;      // 1: a search takes the tuned finish_cap of its shape when one is recorded
    // diagnostics of the last search
    int64_t last_batches = 0, last_finals = 0, last_levels = 0, last_candidates = 0;
    asci::Profiler prof;
    asci::Arena setup;  // inputs, psi hash set, core set, class totals
    asci::Arena main;   // per-batch pair buffers, candidate pool, selection
    asci::Arena tables; // spin-string energy tables of the current integrals
    asci::HostStage stage;
    // worker pool of asci_search_batch, kept between calls so that its
    // workspaces stay allocated (rebuilt when batch_slots or finish_cap change)
    void *batch_pool = nullptr;
    void (*batch_pool_free)(void *) = nullptr;
    void (*batch_pool_trim)(void *) = nullptr;  // free the idle workers' workspaces
    int batch_pool_slots = 0, batch_pool_cap = 0;
    void *graph_batch = nullptr;  // asci::GraphBatch of asci_search_batch (graph part)
    void (*graph_batch_free)(void *) = nullptr;
    asci_ctx() = default;
    asci_ctx(const asci_ctx &) = delete;
    asci_ctx &operator=(const asci_ctx &) = delete;
    ~asci_ctx()
    {
        if (batch_pool && batch_pool_free) batch_pool_free(batch_pool);
        if (graph_batch && graph_batch_free) graph_batch_free(graph_batch);
    }
};

namespace asci {

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int lowbit(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }

// Lanes of the wavefront whose (active, key) equal this lane's, key < 2^nbits:
// one ballot per key bit.  The bit is taken sign-extended (0 or all ones), so
// folding a ballot into the mask is a single three-input logic op per half.
__device__ __forceinline__ uint64_t wave_match(uint32_t key, bool active, int nbits)
{
    const uint64_t act = __builtin_amdgcn_ballot_w64(active);
    uint32_t plo = (uint32_t)act, phi = (uint32_t)(act >> 32);
#pragma nounroll
    for (int b = 0; b < nbits; ++b) {
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)key, b, 1);
        const uint64_t bb = __builtin_amdgcn_ballot_w64(m != 0u);
        plo &= ~((uint32_t)bb ^ m);
        phi &= ~((uint32_t)(bb >> 32) ^ m);
    }
    return ((uint64_t)phi << 32) | plo;
}

// index of the k-th (0-based) set bit of x; requires k < popc64(x)
__device__ __forceinline__ int select_bit(uint64_t x, int k)
{
    int pos = 0;
    int c = __popc((uint32_t)x);
    if (k >= c) { k -= c; x >>= 32; pos += 32; }
    c = __popc((uint32_t)x & 0xFFFFu);
    if (k >= c) { k -= c; x >>= 16; pos += 16; }
    c = __popc((uint32_t)x & 0xFFu);
    if (k >= c) { k -= c; x >>= 8; pos += 8; }
    c = __popc((uint32_t)x & 0xFu);
    if (k >= c) { k -= c; x >>= 4; pos += 4; }
    c = __popc((uint32_t)x & 0x3u);
    if (k >= c) { k -= c; x >>= 2; pos += 2; }
    if (k >= (int)(x & 1u)) pos += 1;
    return pos;
}

// (-1)^(set bits of occ strictly between orbitals p and q), p != q
__device__ __forceinline__ int between_sign(uint64_t occ, int p, int q)
{
    int lo = p < q ? p : q, hi = p < q ? q : p;
    uint64_t m = ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
    return (popc64(occ & m) & 1) ? -1 : 1;
}

// pairs (i < j) enumerated j-major: x = j(j-1)/2 + i
__device__ __forceinline__ void unrank_pair(uint32_t x, int &i, int &j)
{
    int jj = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)x)) * 0.5f);
    while ((uint32_t)(jj * (jj - 1) / 2) > x) --jj;
    while ((uint32_t)((jj + 1) * jj / 2) <= x) ++jj;
    j = jj;
    i = (int)(x - (uint32_t)(jj * (jj - 1) / 2));
}

__device__ __forceinline__ uint64_t choose_small(uint64_t x, int k)
{
    return k == 0 ? 1ull : (k == 1 ? x : (x * (x - 1ull)) / 2ull);
}

// k (0, 1 or 2) set bits of `mask`, chosen by index idx in [0, C(popc(mask), k))
__device__ __forceinline__ uint64_t pick_bits(uint64_t mask, int k, uint32_t idx)
{
    if (k == 0) return 0ull;
    if (k == 1) return 1ull << select_bit(mask, (int)idx);
    int i, j;
    unrank_pair(idx, i, j);
    return (1ull << select_bit(mask, i)) | (1ull << select_bit(mask, j));
}

// IEEE-754 bit pattern of |x|: orders non-negative doubles as integers
__device__ __forceinline__ uint64_t abs_order(double x)
{
    return (uint64_t)__double_as_longlong(x) & 0x7fffffffffffffffull;
}

// ---------------------------------------------------------------- key layout
// Keys: for norb <= 32 a single word (alpha << norb) | beta ("packed"); above,
// two words (hi = alpha, lo = beta).  Both orders equal (alpha, beta) order.
struct KeySpec {
    int norb;
    int words;  // 1 or 2
};

// ---------------------------------------------------------------- primitives (prims.hip)
constexpr int kScanTile = 4096;

// Device-side counts: a primitive given `dn` (device) treats min(n, *dn) as
// its length, with n the host bound its launch is sized for; nothing past the
// count is read or written.

// exclusive scan of n uint32 values (n < 2^28); *d_total (device) gets the sum
void scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, Arena &ar,
              hipStream_t s, Profiler *prof = nullptr, const uint32_t *dn = nullptr);

// p[0 .. n) = v by a kernel (a fill that a captured graph replays correctly)
__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v);
void fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);

// stable LSD radix sort by selected 8-bit digits of a 1- or 2-word key, with a
// payload.  keys_lo/keys_hi/vals are ping-pong pairs; `digits` lists (word,
// shift) from least significant.  Returns the index (0/1) of the buffer that
// holds the result.
struct Digit {
    int word;   // 0 = lo word, 1 = hi word
    int shift;  // bit offset of the 8-bit digit
};
template <typename V>
int radix_sort(uint64_t *keys_lo[2], uint64_t *keys_hi[2], V *vals[2], size_t n, int words,
               const std::vector<Digit> &digits, Arena &ar, hipStream_t s, Profiler *prof = nullptr,
               const uint32_t *dn = nullptr);

// radix selection on the IEEE bit pattern of |score[j]|, j < n: finds t, the
// k-th largest value (1 <= k <= n), and how many entries equal to t must be
// taken (device struct).  The caller then keeps ord > t, plus the first
// `take_equal` entries with ord == t.
struct SelectState {
    uint64_t prefix;
    uint64_t mask;
    uint64_t krem;  // after the passes: number of entries equal to t to take
    uint32_t hist[256];
};
// optional workspace: after two digit passes the entries that still match the
// selected prefix are copied to tmp (capacity n) and the remaining passes run
// on the copy; d_count (device) and h_count (pinned host) hold its length
struct SelectWork {
    double *tmp;
    unsigned int *d_count;
    unsigned int *h_count;
};
// With dn (and dk: k = min(k, *dk), device) the compaction is skipped.
void radix_select_abs(const double *score, size_t n, uint64_t k, SelectState *d_state,
                      hipStream_t s, Profiler *prof = nullptr, const SelectWork *work = nullptr,
                      const uint32_t *dn = nullptr, const uint32_t *dk = nullptr);

// ---------------------------------------------------------------- input-determinant set
// Open-addressing hash set of the input keys (linear probing; a slot is taken
// when state != 0), fronted by a one-hash bit filter of about 8 bits per key
// (a clear bit proves a key absent; a set bit sends the lookup to the table):
// most lookups of non-members cost one read of a small, cache-resident array.
struct PsiSet {
    const uint64_t *lo = nullptr, *hi = nullptr;
    const uint32_t *state = nullptr;
    uint32_t mask = 0;                  // table size - 1 (a power of two minus one)
    const unsigned long long *filter = nullptr;  // filter words (null: no filter)
    uint32_t fmask = 0;                          // filter words - 1 (a power of two minus one)
};

__device__ __forceinline__ uint32_t psi_hash(uint64_t lo, uint64_t hi, uint32_t mask)
{
    const uint64_t h = lo * 0x9E3779B97F4A7C15ull ^ (hi + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
    return (uint32_t)(h >> 32) & mask;
}

// Blocked Bloom filter in front of the table: a key sets (and is tested
// against) four bits of one 64-bit word, both drawn from a hash independent of
// psi_hash's slot.  At 32 filter bits per key about one absent key in a
// thousand reaches the table.
__device__ __forceinline__ uint64_t psi_filter_hash(uint64_t lo, uint64_t hi)
{
    uint64_t h = (lo ^ 0xA0761D6478BD642Full) * 0xE7037ED1A0B428DBull + hi * 0x8EBC6AF09C88C6E3ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    return h ^ (h >> 32);
}
__device__ __forceinline__ uint32_t psi_filter_word(uint64_t h, uint32_t fmask) { return (uint32_t)(h >> 32) & fmask; }
__device__ __forceinline__ uint64_t psi_filter_bits(uint64_t h)
{
    return (1ull << (h & 63u)) | (1ull << ((h >> 6) & 63u)) | (1ull << ((h >> 12) & 63u)) |
           (1ull << ((h >> 18) & 63u));
}

// false: the key is certainly not in the set
__device__ __forceinline__ bool psi_maybe(const PsiSet &t, uint64_t lo, uint64_t hi)
{
    if (!t.filter) return true;
    const uint64_t h = psi_filter_hash(lo, hi), m = psi_filter_bits(h);
    return (t.filter[psi_filter_word(h, t.fmask)] & m) == m;
}

__device__ __forceinline__ bool psi_contains(const PsiSet &t, uint64_t lo, uint64_t hi)
{
    if (!psi_maybe(t, lo, hi)) return false;
    uint32_t s = psi_hash(lo, hi, t.mask);
    while (t.state[s]) {
        if (t.lo[s] == lo && t.hi[s] == hi) return true;
        s = (s + 1u) & t.mask;
    }
    return false;
}

// Energies E(s) of every spin string with a given electron count, indexed by
// the combinatorial rank of the string (sum over its set bits p_1 < p_2 < ...
// of C(p_j, j)); binom[k * (n + 1) + p] = C(p, k).  e[0] covers the alpha
// strings, e[1] the beta strings (null: no table, evaluate directly).
struct SpinTables {
    const double *e[2] = {nullptr, nullptr};
    const uint32_t *binom = nullptr;  // (kmax + 4) rows of n + 1: C(p, k) for k <= kmax, then zeros
    int kmax = 0;
};

// Which tables a search builds: count[i] strings (0 = none) for alpha (0) and
// beta (1); share when both spins have the same electron count.
constexpr uint64_t kSpinTableMax = (uint64_t)1 << 27;
struct SpinTablePlan {
    uint64_t count[2] = {0, 0};
    bool share = false;
    int kmax = 0;
    size_t bytes = 0;
};
SpinTablePlan spin_table_plan(int n, int na, int nb, uint64_t pairs, bool enabled);

// ---------------------------------------------------------------- buckets (bucket.hip)
struct BucketArgs {
    size_t P;                       // records of the batch
    uint32_t c0, nc, nq;            // classes [c0, c0 + nc), core count
    int n;
    const uint64_t *cls;            // class masks (all classes)
    const uint32_t *offsets;        // [nc][nq] item starts
    const uint32_t *total;          // device: records of the batch
    uint64_t *klo[2], *khi[2];      // record buffers (ping-pong)
    double *val[2];
    PsiSet psi;                     // the same keys as a hash set
    const double *jk, *h;
    SpinTables st;                  // tabulated E(alpha), E(beta) (optional)
    const uint64_t *thr = nullptr;  // device: drop candidates whose |A| order bits are below (optional)
    double ecore, E0, eps;
    int finish_cap = 4096;          // LDS capacity of a final segment (tunable)
    uint64_t *clo, *chi;            // candidate slots (P)
    double *cnum, *cscore;
    // results of bucket_accumulate.  With defer_v the candidate count V is
    // left in flight to *h_v (pinned): bucket_read_v waits for it, so that
    // work the count does not gate (the collect) can be queued first.
    bool defer_v = false;
    const uint32_t *h_v = nullptr;
    uint32_t nfinal = 0, V = 0, levels = 0;
    Profiler *prof = nullptr;       // the finish launch's profiler token, for its byte count
    int finish_tok = -1;
    // the device-driven variant: nfinal and V are then bounds, the counts are on the device
    const uint32_t *dn_final = nullptr, *dn_V = nullptr;
    const uint32_t *order = nullptr, *cnt_sorted = nullptr, *off = nullptr;
    const void *finals = nullptr;
    // destination of bucket_collect
    uint64_t *pool_lo = nullptr, *pool_hi = nullptr;
    double *pool_num = nullptr, *pool_score = nullptr;
    size_t pool_base = 0, pool_cap = 0;
};
size_t bucket_workspace_bytes(size_t P, size_t nc, int W, int finish_cap);
template <int W>
void bucket_accumulate(BucketArgs &b, Arena &ar, hipStream_t s, Profiler *prof, HostStage &hs);
template <int W>
int bucket_collect(BucketArgs &b, hipStream_t s, Profiler *prof);  // profiler token (-1: untimed)
void bucket_read_v(BucketArgs &b, hipStream_t s);
// sum over the batch's candidates of N_a * A_a (deterministic order)
double bucket_pt2(BucketArgs &b, Arena &ar, hipStream_t s, HostStage &hs);
// The same sort-and-accumulate with no count read back (asynchronous search):
// launches sized for host bounds, a fixed number of split levels, counts in
// b.dn_final and b.dn_V.  A failure sets bits of *d_stat (kStat*).
template <int W>
void bucket_accumulate_dev(BucketArgs &b, Arena &ar, hipStream_t s, uint32_t *d_stat);
template <int W>
void bucket_collect_dev(BucketArgs &b, hipStream_t s);
// status bits of a search that reads nothing back
constexpr uint32_t kStatInvalid = 1u;    // wrong electron count or orbital >= norb
constexpr uint32_t kStatDuplicate = 2u;  // an input determinant given twice
constexpr uint32_t kStatSplit = 4u;      // the bucket split did not finish in its levels / lists overflowed
constexpr uint32_t kStatPool = 8u;       // candidate pool overflow
constexpr uint32_t kStatFault = 16u;     // a kernel consistency fault (see hamiltonian.h)
constexpr uint32_t kStatIntegrals = 32u; // two-electron integrals not 8-fold symmetric

// the fault word of the bucket kernels (see hamiltonian.h): clear / queue a copy to pinned *dst
void bucket_fault_clear(hipStream_t s);
void bucket_fault_reset_dev(hipStream_t s);                          // by a kernel
void bucket_fault_take_dev(uint32_t *stat, uint32_t bit, hipStream_t s);  // stat |= bit if set
void bucket_fault_fetch(unsigned int *dst, hipStream_t s);

// ---------------------------------------------------------------- search (search.hip)
struct SearchArgs {
    const double *h, *eri;  // device
    int n, na, nb;
    const uint64_t *dets;   // device, ndets x 2
    const double *coeffs;   // device
    int64_t ndets;
    double E0;
    asci_options opt;
};

struct SearchOut {
    int64_t k = 0;                 // > 0: top-k mode; 0: every candidate
    uint64_t *out_dets = nullptr;  // device
    double *out_scores = nullptr;  // device
    int64_t capacity = 0;          // every-candidate mode: output length
    double *out_num = nullptr;     // every-candidate mode: N_a (device)
    bool pt2 = false;              // second-order energy mode: no candidates are kept
    double pt2_energy = 0.0;
    int64_t count = 0;             // result count
};

void search_device(asci_ctx *ctx, const SearchArgs &in, SearchOut &out, hipStream_t s);
// closed-form number of (core, target) pairs of a search
uint64_t search_pairs(const SearchArgs &in);
// the finish capacity a search of this shape uses on ctx (tune.hip)
int effective_finish_cap(const asci_ctx *ctx, int norb, int na, uint64_t pairs);
// The top-k search with nothing read back (asci_search_async): one class batch,
// every count on the device; d_result (device) receives count and status.
// plan_only: check the request and size ctx's workspaces, queue nothing.
void search_async(asci_ctx *ctx, const SearchArgs &in, int64_t k, uint64_t *out_dets, double *out_scores,
                  asci_async_result *d_result, hipStream_t s, bool plan_only = false);
// device bytes of search_async's workspaces for this request; 0 when the
// request is outside its scope (one class batch)
size_t search_async_bytes(const SearchArgs &in, int64_t k, int finish_cap, bool spin_tables);
// Upper bound of the device bytes a search of one class batch takes from its
// setup and main arenas (top-k mode when k > 0), with the pair buffer set to
// hold every pair; setup_part receives the setup arena's share (first).
size_t search_scratch_bound(const SearchArgs &in, int64_t k, int finish_cap, size_t &setup_part);
void class_counts_device(asci_ctx *ctx, int n, int na, int nb, const uint64_t *dets, const double *coeffs,
                         int64_t ndets, const asci_options &opt, std::vector<uint64_t> &masks,
                         std::vector<uint64_t> &counts, hipStream_t s);
// closed-form pair count and workspace estimate of a request (server.hip)
int64_t request_pairs(const asci_request &r);
int64_t request_footprint(const asci_request &r, uint64_t cap_records, int finish_cap = 4096);

// argument checks shared by every entry point (ASCI_EINVAL on failure): sizes,
// and options resolved against the defaults (NULL = defaults)
void check_common(int norb, int nalpha, int nbeta, int64_t ndets);
// records e as the calling thread's last error (asci_last_error); returns its code
int report_error(const Error &e);
asci_options resolve(const asci_options *opt);

// throws ASCI_EINVAL unless every determinant has na/nb electrons inside norb orbitals
void validate_dets(asci_ctx *ctx, const uint64_t *dets, int64_t ndets, int n, int na, int nb, hipStream_t s);

// ---------------------------------------------------------------- batches as one graph (graph.hip)
// Contexts and streams of the graph slots, the captured graph and the device
// result records of its requests; replayed while the requests stay the same.
struct GraphBatch {
    int device = 0;
    std::vector<std::unique_ptr<asci_ctx>> ctxs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipStream_t main = nullptr;   // capture and launch stream
    hipEvent_t order = nullptr;   // orders it with the caller's stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
    asci_async_result *d_res = nullptr;
    size_t nres = 0;
    GraphBatch() = default;
    GraphBatch(const GraphBatch &) = delete;
    GraphBatch &operator=(const GraphBatch &) = delete;
    ~GraphBatch();
    void release_graph();
};
// workspace bytes of a request in a graph slot, 0 when outside the asynchronous search's scope
size_t graph_request_bytes(const asci_request &r, int finish_cap, bool spin_tables);
// queue requests reqs[idx[j]] as one graph on `stream` (captured, or replayed
// when the same requests were captured last); result j goes to record j
void graph_batch_launch(GraphBatch &gb, int device, const asci_request *reqs, const std::vector<int> &idx, int slots,
                        int finish_cap, int spin_tables, hipStream_t stream);
// after the stream has finished: the result records of the last launch
void graph_batch_results(GraphBatch &gb, size_t count, std::vector<asci_async_result> &out);

// ---------------------------------------------------------------- variational step (eigen.hip)
// H over a determinant set in CSR: rows in set order, columns ascending, both
// triangles and the diagonal; device memory owned by the object.
struct HMat {
    int device = 0;
    int64_t nrows = 0, nnz = 0;
    int64_t *rowptr = nullptr;
    int32_t *cols = nullptr;
    double *vals = nullptr;
    double *diag = nullptr;
    HMat() = default;
    HMat(const HMat &) = delete;
    HMat &operator=(const HMat &) = delete;
    ~HMat();
    void release();
};
void hmat_build(asci_ctx *ctx, const double *h, const double *eri, int n, int na, int nb, const uint64_t *dets,
                int64_t ndets, double ecore, HMat &H, hipStream_t s);
void hmat_matvec(const HMat &H, const double *x, double *y, hipStream_t s, Profiler *prof = nullptr);

struct DavidsonOpts {
    int max_subspace = 24;
    int max_iter = 200;
    double tol = 1e-8;  // residual norm of the Ritz pair
};
struct DavidsonOut {
    double energy, resid;
    int iters;
    bool converged;
};
DavidsonOut davidson(asci_ctx *ctx, const HMat &H, const double *guess, const DavidsonOpts &o, double *vec,
                     hipStream_t s);

// ---------------------------------------------------------------- the ASCI loop (loop.hip)
struct LoopArgs {
    const double *h, *eri;  // device
    int n, na, nb;
    asci_loop_options opt;
    DavidsonOpts dav;
};
using LoopIter = asci_loop_iter;
void loop_step(asci_ctx *ctx, const LoopArgs &a, const uint64_t *dets, const double *coeffs, int64_t nd, double Ek,
               uint64_t *out_dets, double *out_coeffs, int64_t &out_nd, LoopIter &info, hipStream_t s);
void loop_run(asci_ctx *ctx, const LoopArgs &a, const uint64_t *dets0, const double *c0, int64_t n0,
              uint64_t *out_dets, double *out_coeffs, int64_t &out_nd, double &energy, double &pt2,
              std::vector<LoopIter> &iters, hipStream_t s);
double energy_device(asci_ctx *ctx, const double *h, const double *eri, int n, const uint64_t *dets,
                     const double *coeffs, int64_t ndets, double ecore, hipStream_t s);

}  // namespace asci
