// The ASCI loop (Alg. 1) on one GPU: search, selection of the next
// determinant set, Hamiltonian over it, Davidson, repeated until the energy
// settles; optionally a final PT2 step.
//
// Selection of psi_{k+1} (Alg. 1 "sort and select"): the search returns new
// determinants ranked by |A_a| (the first-order estimate of their
// coefficients); psi_k keeps its determinants ranked by |C_i|.  The next set is
// the N_tdets entries of largest score over both lists, ties by key ascending,
// stored in that order.  The Davidson guess is C_k on the kept determinants and
// zero on the new ones.
#include "asci_internal.h"

#include <chrono>
#include <cmath>
#include <cstring>

namespace asci {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// union entries: key words, ~|score| bits (ascending = score descending), index
template <int W>
__global__ __launch_bounds__(kBlock) void k_union_keys(const uint64_t *__restrict__ dets, const double *__restrict__ c,
                                                       uint32_t nd, const uint64_t *__restrict__ cand,
                                                       const double *__restrict__ cscore, uint32_t nc, int n,
                                                       uint64_t *__restrict__ klo, uint64_t *__restrict__ khi,
                                                       uint64_t *__restrict__ ord, uint32_t *__restrict__ idx)
{
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= nd + nc) return;
    const bool old = j < nd;
    const uint64_t a = old ? dets[2 * (size_t)j] : cand[2 * (size_t)(j - nd)];
    const uint64_t b = old ? dets[2 * (size_t)j + 1] : cand[2 * (size_t)(j - nd) + 1];
    const double v = old ? c[j] : cscore[j - nd];
    if (W == 1) {
        klo[j] = (a << n) | b;
    } else {
        klo[j] = b;
        khi[j] = a;
    }
    ord[j] = ~abs_order(v);
    idx[j] = j;
}

__global__ __launch_bounds__(kBlock) void k_gather_ord(const uint32_t *__restrict__ idx,
                                                       const uint64_t *__restrict__ ord_by_index, uint32_t m,
                                                       uint64_t *__restrict__ out)
{
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j < m) out[j] = ord_by_index[idx[j]];
}

// the first `take` entries of the sorted union: determinants and the guess
__global__ __launch_bounds__(kBlock) void k_take(const uint32_t *__restrict__ idx, uint32_t take,
                                                 const uint64_t *__restrict__ dets, const double *__restrict__ c,
                                                 uint32_t nd, const uint64_t *__restrict__ cand,
                                                 uint64_t *__restrict__ out_dets, double *__restrict__ guess,
                                                 unsigned int *__restrict__ kept)
{
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= take) return;
    const uint32_t u = idx[j];
    const bool old = u < nd;
    out_dets[2 * (size_t)j] = old ? dets[2 * (size_t)u] : cand[2 * (size_t)(u - nd)];
    out_dets[2 * (size_t)j + 1] = old ? dets[2 * (size_t)u + 1] : cand[2 * (size_t)(u - nd) + 1];
    guess[j] = old ? c[u] : 0.0;
    if (old) atomicAdd(kept, 1u);
}

std::vector<Digit> key_digits(int n, int W)
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

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// device buffer owned by the loop (freed on scope exit)
template <typename T>
struct DevBuf {
    T *p = nullptr;
    int dev = 0;
    DevBuf(size_t n, int device) : dev(device)
    {
        ASCI_HIP(hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T)));
    }
    ~DevBuf()
    {
        (void)hipSetDevice(dev);
        (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

// merge psi_k (by |C|) with the candidates (by |A|): returns the new size and
// whether any old determinant was kept
template <int W>
int64_t select_next(asci_ctx *ctx, int n, const uint64_t *dets, const double *c, int64_t nd, const uint64_t *cand,
                    const double *cscore, int64_t nc, int64_t ntdets, uint64_t *out_dets, double *guess, bool &kept,
                    hipStream_t s)
{
    const size_t U = (size_t)(nd + nc);
    const size_t take = (size_t)std::min<int64_t>((int64_t)U, ntdets);
    Arena &ar = ctx->main;
    ar.reset();
    const size_t nb = (U + kScanTile - 1) / kScanTile;
    ar.reserve(U * (8 * 2 * W + 8 * 3 + 4 * 2) + 4 * (nb * 256 * 4 + (1 << 16)) + 64 * 256);
    ar.reset();
    uint64_t *klo[2] = {ar.take<uint64_t>(U), ar.take<uint64_t>(U)};
    uint64_t *khi[2] = {W == 2 ? ar.take<uint64_t>(U) : nullptr, W == 2 ? ar.take<uint64_t>(U) : nullptr};
    uint64_t *ord_by_index = ar.take<uint64_t>(U);
    uint64_t *ord[2] = {ar.take<uint64_t>(U), ar.take<uint64_t>(U)};
    uint32_t *idx[2] = {ar.take<uint32_t>(U), ar.take<uint32_t>(U)};
    unsigned int *d_kept = ar.take<unsigned int>(4);
    k_union_keys<W><<<grid_for(U), kBlock, 0, s>>>(dets, c, (uint32_t)nd, cand, cscore, (uint32_t)nc, n, klo[0],
                                                   khi[0], ord_by_index, idx[0]);
    ASCI_LAUNCH_CHECK();
    // stable: key ascending, then ~|score| ascending (score descending, ties by key)
    const int r1 = radix_sort<uint32_t>(klo, khi, idx, U, W, key_digits(n, W), ar, s);
    k_gather_ord<<<grid_for(U), kBlock, 0, s>>>(idx[r1], ord_by_index, (uint32_t)U, ord[0]);
    ASCI_LAUNCH_CHECK();
    uint32_t *idx2[2] = {idx[r1], idx[r1 ^ 1]};
    uint64_t *nohi[2] = {nullptr, nullptr};
    std::vector<Digit> od;
    for (int sh = 0; sh < 64; sh += 8) od.push_back({0, sh});
    const int r2 = radix_sort<uint32_t>(ord, nohi, idx2, U, 1, od, ar, s);
    ASCI_HIP(hipMemsetAsync(d_kept, 0, sizeof(unsigned int), s));
    k_take<<<grid_for(take), kBlock, 0, s>>>(idx2[r2], (uint32_t)take, dets, c, (uint32_t)nd, cand, out_dets, guess,
                                             d_kept);
    ASCI_LAUNCH_CHECK();
    HostStage &hs = ctx->stage;
    hs.reserve(64);
    ASCI_HIP(hipMemcpyAsync(hs.ptr, d_kept, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    kept = *(unsigned int *)hs.ptr > 0;
    return (int64_t)take;
}

}  // namespace

void loop_step(asci_ctx *ctx, const LoopArgs &a, const uint64_t *dets, const double *coeffs, int64_t nd, double Ek,
               uint64_t *out_dets, double *out_coeffs, int64_t &out_nd, LoopIter &info, hipStream_t s)
{
    const int64_t ntdets = a.opt.ntdets;
    // 1. search: the N_tdets best new determinants
    auto t0 = std::chrono::steady_clock::now();
    DevBuf<uint64_t> cand((size_t)2 * ntdets, ctx->device);
    DevBuf<double> cscore((size_t)ntdets, ctx->device);
    SearchArgs in;
    in.h = a.h;
    in.eri = a.eri;
    in.n = a.n;
    in.na = a.na;
    in.nb = a.nb;
    in.dets = dets;
    in.coeffs = coeffs;
    in.ndets = nd;
    in.E0 = Ek;
    in.opt = a.opt.search;
    in.opt.ncore = a.opt.ncore;
    SearchOut so;
    so.k = ntdets;
    so.out_dets = cand.p;
    so.out_scores = cscore.p;
    search_device(ctx, in, so, s);
    const int64_t nc = so.count;
    info.search_ms = ms_since(t0);
    info.candidates = ctx->last_candidates;

    // 2. selection of psi_{k+1}
    t0 = std::chrono::steady_clock::now();
    DevBuf<double> guess((size_t)ntdets, ctx->device);
    bool kept = false;
    if (a.n <= 32)
        out_nd = select_next<1>(ctx, a.n, dets, coeffs, nd, cand.p, cscore.p, nc, ntdets, out_dets, guess.p, kept, s);
    else
        out_nd = select_next<2>(ctx, a.n, dets, coeffs, nd, cand.p, cscore.p, nc, ntdets, out_dets, guess.p, kept, s);
    info.select_ms = ms_since(t0);
    info.ndets = out_nd;

    // 3. H over psi_{k+1} (double loop), 4. Davidson
    t0 = std::chrono::steady_clock::now();
    HMat H;
    hmat_build(ctx, a.h, a.eri, a.n, a.na, a.nb, out_dets, out_nd, a.opt.search.ecore, H, s);
    info.hbuild_ms = ms_since(t0);
    info.nnz = H.nnz;
    t0 = std::chrono::steady_clock::now();
    const DavidsonOut d = davidson(ctx, H, kept ? guess.p : nullptr, a.dav, out_coeffs, s);
    info.davidson_ms = ms_since(t0);
    info.energy = d.energy;
    info.davidson_resid = d.resid;
    info.davidson_iters = d.iters;
}

void loop_run(asci_ctx *ctx, const LoopArgs &a, const uint64_t *dets0, const double *c0, int64_t n0,
              uint64_t *out_dets, double *out_coeffs, int64_t &out_nd, double &energy, double &pt2,
              std::vector<LoopIter> &iters, hipStream_t s)
{
    const int64_t cap = std::max<int64_t>(a.opt.ntdets, n0);
    DevBuf<uint64_t> d0((size_t)2 * cap, ctx->device), d1((size_t)2 * cap, ctx->device);
    DevBuf<double> cA((size_t)cap, ctx->device), cB((size_t)cap, ctx->device);
    ASCI_HIP(hipMemcpyAsync(d0.p, dets0, (size_t)2 * n0 * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    ASCI_HIP(hipMemcpyAsync(cA.p, c0, (size_t)n0 * sizeof(double), hipMemcpyDeviceToDevice, s));
    uint64_t *cur_d = d0.p, *nxt_d = d1.p;
    double *cur_c = cA.p, *nxt_c = cB.p;
    int64_t nd = n0;
    double E = energy_device(ctx, a.h, a.eri, a.n, cur_d, cur_c, nd, a.opt.search.ecore, s);
    iters.clear();
    for (int it = 0; it < a.opt.max_iter; ++it) {
        LoopIter info{};
        int64_t nn = 0;
        loop_step(ctx, a, cur_d, cur_c, nd, E, nxt_d, nxt_c, nn, info, s);
        iters.push_back(info);
        const double dE = std::fabs(info.energy - E);
        std::swap(cur_d, nxt_d);
        std::swap(cur_c, nxt_c);
        nd = nn;
        E = info.energy;
        if (dE < a.opt.e_tol) break;
    }
    energy = E;
    pt2 = 0.0;
    if (a.opt.pt2) {
        SearchArgs in;
        in.h = a.h;
        in.eri = a.eri;
        in.n = a.n;
        in.na = a.na;
        in.nb = a.nb;
        in.dets = cur_d;
        in.coeffs = cur_c;
        in.ndets = nd;
        in.E0 = E;
        in.opt = a.opt.search;
        in.opt.ncore = 0;
        in.opt.eps = 0.0;
        SearchOut so;
        so.pt2 = true;
        search_device(ctx, in, so, s);
        pt2 = so.pt2_energy;
    }
    ASCI_HIP(hipMemcpyAsync(out_dets, cur_d, (size_t)2 * nd * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    ASCI_HIP(hipMemcpyAsync(out_coeffs, cur_c, (size_t)nd * sizeof(double), hipMemcpyDeviceToDevice, s));
    ASCI_HIP(hipStreamSynchronize(s));
    out_nd = nd;
}

}  // namespace asci
