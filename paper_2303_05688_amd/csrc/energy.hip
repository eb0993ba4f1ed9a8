// Variational energy E = sum_ij C_i H_ij C_j over a determinant set: the E_k
// of Eq. (1), by the double loop over determinant pairs that the paper uses to
// build H (Sec. II.C).  One thread per row i; the determinants of column tiles
// are staged in LDS; pairs beyond double excitations are skipped by popcount.
#include "hamiltonian.h"

namespace asci {

namespace {

constexpr int kBlock = 256;

// <a|H|i> for two arbitrary determinants (zero beyond doubles)
__device__ double pair_value(const double *__restrict__ h, const double *__restrict__ eri,
                             const double *__restrict__ jk, int n, double ecore, uint64_t aa, uint64_t ab,
                             uint64_t ia, uint64_t ib)
{
    const uint64_t da = aa ^ ia, db = ab ^ ib;
    const int ea = popc64(da) >> 1, eb = popc64(db) >> 1;
    if (ea + eb == 0) return diag_value(jk, jk + n * n, jk + 2 * n * n, n, ecore, aa, ab);
    if (ea + eb > 2) return 0.0;
    if (ea == 1 && eb == 0) return single_value(h, eri, n, ia, ib, lowbit(ia & ~aa), lowbit(aa & ~ia));
    if (ea == 0 && eb == 1) return single_value(h, eri, n, ib, ia, lowbit(ib & ~ab), lowbit(ab & ~ib));
    if (ea == 1 && eb == 1)
        return double_opp_value(eri, n, ia, ib, lowbit(ia & ~aa), lowbit(aa & ~ia), lowbit(ib & ~ab),
                                lowbit(ab & ~ib));
    if (ea == 2) return double_same_value(eri, n, ia, ia & ~aa, aa & ~ia);
    return double_same_value(eri, n, ib, ib & ~ab, ab & ~ib);
}

__global__ __launch_bounds__(kBlock) void k_energy_rows(const uint64_t *__restrict__ dets,
                                                        const double *__restrict__ c, uint32_t nd,
                                                        const double *__restrict__ h,
                                                        const double *__restrict__ eri,
                                                        const double *__restrict__ jk, int n, double ecore,
                                                        double *__restrict__ row)
{
    __shared__ uint64_t s_a[kBlock], s_b[kBlock];
    __shared__ double s_c[kBlock];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool act = i < nd;
    const uint64_t ia = act ? dets[2 * (size_t)i] : 0ull, ib = act ? dets[2 * (size_t)i + 1] : 0ull;
    const double ci = act ? c[i] : 0.0;
    double acc = 0.0;
    for (uint32_t t0 = 0; t0 < nd; t0 += kBlock) {
        __syncthreads();
        const uint32_t j = t0 + threadIdx.x;
        if (j < nd) {
            s_a[threadIdx.x] = dets[2 * (size_t)j];
            s_b[threadIdx.x] = dets[2 * (size_t)j + 1];
            s_c[threadIdx.x] = c[j];
        }
        __syncthreads();
        const uint32_t tn = (nd - t0) < (uint32_t)kBlock ? (nd - t0) : (uint32_t)kBlock;
        if (!act) continue;
        for (uint32_t t = 0; t < tn; ++t) {
            const uint64_t ja = s_a[t], jb = s_b[t];
            if (popc64(ia ^ ja) + popc64(ib ^ jb) > 4) continue;
            acc = acc + ci * pair_value(h, eri, jk, n, ecore, ia, ib, ja, jb) * s_c[t];
        }
    }
    if (act) row[i] = acc;
}

// deterministic sum of the row totals: one block, fixed order
__global__ __launch_bounds__(1024) void k_sum(const double *__restrict__ x, uint32_t n, double *__restrict__ out)
{
    __shared__ double s[1024];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += 1024) acc = acc + x[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (threadIdx.x < (unsigned)w) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// J_pq = (pp|qq), X_pq = (pp|qq) - (pq|qp), h_pp: the tables of H_aa
__global__ __launch_bounds__(kBlock) void k_jk_table(const double *__restrict__ eri, const double *__restrict__ h,
                                                     int n, double *__restrict__ jk)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    jk[t] = eri4(eri, n, p, p, q, q);
    jk[n * n + t] = eri4(eri, n, p, p, q, q) - eri4(eri, n, p, q, q, p);
    if (q == 0) jk[2 * n * n + p] = h[(size_t)p * n + p];
}

}  // namespace

double energy_device(asci_ctx *ctx, const double *h, const double *eri, int n, const uint64_t *dets,
                     const double *coeffs, int64_t ndets, double ecore, hipStream_t s)
{
    require(ndets >= 1 && ndets < (1ll << 31), ASCI_EINVAL, "ndets out of range");
    const uint32_t nd = (uint32_t)ndets;
    Arena &ar = ctx->main;
    ar.reset();
    ar.reserve((size_t)nd * 8 + ((size_t)2 * n * n + n) * 8 + 4096);
    ar.reset();
    double *row = ar.take<double>(nd);
    double *jk = ar.take<double>((size_t)2 * n * n + n);
    double *out = ar.take<double>(1);
    fault_clear(s);
    k_jk_table<<<(unsigned)((n * n + kBlock - 1) / kBlock), kBlock, 0, s>>>(eri, h, n, jk);
    ASCI_LAUNCH_CHECK();
    k_energy_rows<<<(nd + kBlock - 1) / kBlock, kBlock, 0, s>>>(dets, coeffs, nd, h, eri, jk, n, ecore, row);
    ASCI_LAUNCH_CHECK();
    k_sum<<<1, 1024, 0, s>>>(row, nd, out);
    ASCI_LAUNCH_CHECK();
    HostStage &hs = ctx->stage;
    hs.reserve(256);
    ASCI_HIP(hipMemcpyAsync(hs.ptr, out, sizeof(double), hipMemcpyDeviceToHost, s));
    fault_fetch((unsigned int *)((char *)hs.ptr + 64), s);
    ASCI_HIP(hipStreamSynchronize(s));
    fault_check(*(unsigned int *)((char *)hs.ptr + 64), "the energy double loop");
    return *(double *)hs.ptr;
}

}  // namespace asci
