// The variational step of the ASCI loop on one GPU (Sec. II.C): the
// Hamiltonian over a determinant set by the double loop over determinant
// pairs, stored as CSR, its product with a vector, and the Davidson method
// (Alg. 5) with the shifted-Jacobi (diagonal) preconditioner.
//
// H: rows in the order of the determinant set, columns ascending, both
// triangles and the diagonal stored.  Matrix elements use the same
// Slater-Condon routines (and the same operation order) as the search.
#include "asci_internal.h"
#include "hamiltonian.h"

#include <cmath>
#include <cstring>

namespace asci {

namespace {

constexpr int kHBlock = 256;      // 4 wavefronts
constexpr int kHRows = 4;         // rows per wavefront
constexpr int kHTile = 2048;      // column determinants staged in LDS per tile
constexpr int kChunk = 4096;      // rows per chunk of the row-pointer scan

// J_pq = (pp|qq), X_pq = (pp|qq) - (pq|qp), h_pp: the tables of H_aa
__global__ __launch_bounds__(kHBlock) void k_hm_table(const double *__restrict__ eri, const double *__restrict__ h,
                                                      int n, double *__restrict__ jk)
{
    const int t = blockIdx.x * kHBlock + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    jk[t] = eri4(eri, n, p, p, q, q);
    jk[n * n + t] = eri4(eri, n, p, p, q, q) - eri4(eri, n, p, q, q, p);
    if (q == 0) jk[2 * n * n + p] = h[(size_t)p * n + p];
}

// <a|H|i> for determinants a = (aa, ab) and i = (ia, ib) that differ by at
// most a double excitation: the excitation is read from i to a
__device__ __forceinline__ double helem_value(const double *__restrict__ h, const double *__restrict__ eri,
                                              const double *jk, int n, double ecore, uint64_t aa, uint64_t ab,
                                              uint64_t ia, uint64_t ib)
{
    const int ea = popc64(aa ^ ia) >> 1, eb = popc64(ab ^ ib) >> 1;
    if (ea + eb == 0) return diag_value(jk, jk + n * n, jk + 2 * n * n, n, ecore, aa, ab);
    if (ea == 1 && eb == 0) return single_value(h, eri, n, ia, ib, lowbit(ia & ~aa), lowbit(aa & ~ia));
    if (ea == 0 && eb == 1) return single_value(h, eri, n, ib, ia, lowbit(ib & ~ab), lowbit(ab & ~ib));
    if (ea == 1 && eb == 1)
        return double_opp_value(eri, n, ia, ib, lowbit(ia & ~aa), lowbit(aa & ~ia), lowbit(ib & ~ab),
                                lowbit(ab & ~ib));
    if (ea == 2) return double_same_value(eri, n, ia, ia & ~aa, aa & ~ia);
    return double_same_value(eri, n, ib, ib & ~ab, ab & ~ib);
}

struct HBuildArgs {
    const uint64_t *dets;
    uint32_t nd;
    int n;
    double ecore;
    const double *h, *eri, *jk;
    uint32_t *rowcnt;        // count pass: nonzeros per row
    const int64_t *rowptr;   // fill pass
    int32_t *cols;
    double *vals, *diag;
};

// The double loop: every wavefront owns kHRows rows and tests them against all
// determinants, staged tile by tile in LDS; a pair is coupled when the two
// strings differ in at most four spin orbitals.  The count pass stores the
// number of couplings per row; the fill pass writes them in ascending column
// order (ballot + prefix count inside each 64-column chunk).
template <bool FILL>
__global__ __launch_bounds__(kHBlock) void k_hbuild(HBuildArgs g)
{
    __shared__ uint64_t ta[kHTile], tb[kHTile];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint32_t row0 = (blockIdx.x * (kHBlock / 64) + wv) * kHRows;
    uint64_t ra[kHRows], rb[kHRows];
    int64_t run[kHRows];
#pragma unroll
    for (int t = 0; t < kHRows; ++t) {
        const bool ok = row0 + t < g.nd;
        ra[t] = ok ? g.dets[2 * (size_t)(row0 + t)] : 0ull;
        rb[t] = ok ? g.dets[2 * (size_t)(row0 + t) + 1] : 0ull;
        run[t] = (FILL && ok) ? g.rowptr[row0 + t] : 0;
    }
    for (uint32_t j0 = 0; j0 < g.nd; j0 += kHTile) {
        const uint32_t tn = min((uint32_t)kHTile, g.nd - j0);
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < tn; k += kHBlock) {
            ta[k] = g.dets[2 * (size_t)(j0 + k)];
            tb[k] = g.dets[2 * (size_t)(j0 + k) + 1];
        }
        __syncthreads();
        for (uint32_t c = 0; c < tn; c += 64) {
            const uint32_t jl = c + lane;
            const bool in = jl < tn;
            const uint64_t ca = in ? ta[jl] : 0ull, cb = in ? tb[jl] : 0ull;
#pragma unroll
            for (int t = 0; t < kHRows; ++t) {
                if (row0 + t >= g.nd) break;  // the same for the whole wavefront
                const bool hit = in && (popc64(ra[t] ^ ca) + popc64(rb[t] ^ cb)) <= 4;
                const uint64_t m = __ballot(hit);
                if (FILL && hit) {
                    const int64_t pos = run[t] + (int64_t)__popcll(m & lt);
                    const double v = helem_value(g.h, g.eri, g.jk, g.n, g.ecore, ra[t], rb[t], ca, cb);
                    g.cols[pos] = (int32_t)(j0 + jl);
                    g.vals[pos] = v;
                    if (j0 + jl == row0 + t) g.diag[row0 + t] = v;
                }
                run[t] += (int64_t)__popcll(m);
            }
        }
    }
    if (!FILL && lane == 0) {
#pragma unroll
        for (int t = 0; t < kHRows; ++t)
            if (row0 + t < g.nd) g.rowcnt[row0 + t] = (uint32_t)run[t];
    }
}

// 64-bit exclusive scan of the row counts, chunk by chunk
__global__ __launch_bounds__(256) void k_chunk_sums(const uint32_t *__restrict__ cnt, uint32_t n,
                                                    unsigned long long *__restrict__ sums)
{
    __shared__ unsigned long long s[256];
    const uint32_t base = blockIdx.x * kChunk;
    unsigned long long acc = 0;
    for (uint32_t i = threadIdx.x; i < kChunk && base + i < n; i += 256) acc += cnt[base + i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_chunk_scan(const uint32_t *__restrict__ cnt, uint32_t n,
                                                    const unsigned long long *__restrict__ base,
                                                    int64_t *__restrict__ rowptr)
{
    constexpr int per = kChunk / 256;
    __shared__ unsigned long long s[256];
    const uint32_t c0 = blockIdx.x * kChunk + threadIdx.x * per;
    uint32_t v[per];
    unsigned long long tot = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = (c0 + k < n) ? cnt[c0 + k] : 0u;
        tot += v[k];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    // Hillis-Steele inclusive scan of the thread totals
    for (int d = 1; d < 256; d <<= 1) {
        const unsigned long long add = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0ull;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = base[blockIdx.x] + s[threadIdx.x] - tot;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (c0 + k < n) rowptr[c0 + k] = (int64_t)run;
        run += v[k];
    }
}

// ---------------------------------------------------------------- vectors
// y = H x, one wavefront per row (lane-strided, then a fixed shuffle tree)
__global__ __launch_bounds__(256) void k_spmv(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ cols,
                                              const double *__restrict__ vals, const double *__restrict__ x,
                                              double *__restrict__ y, uint32_t nrows)
{
    const uint32_t row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    double acc = 0.0;
    for (int64_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += 64) acc = acc + vals[k] * x[cols[k]];
    for (int d = 32; d >= 1; d >>= 1) acc = acc + __shfl_xor(acc, d, 64);
    if (lane == 0) y[row] = acc;
}

constexpr int kDotBlocks = 512;
constexpr int kMaxSub = 48;  // largest Davidson subspace

// partial[j][b] = sum over block b's share of i of V[j][i] * x[i], j < m
__global__ __launch_bounds__(256) void k_multidot(const double *__restrict__ V, size_t ld, int m,
                                                  const double *__restrict__ x, size_t n,
                                                  double *__restrict__ partial)
{
    __shared__ double s[256];
    for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
            acc = acc + V[(size_t)j * ld + i] * x[i];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if ((int)threadIdx.x < w) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)j * gridDim.x + blockIdx.x] = s[0];
        __syncthreads();
    }
}

__global__ void k_rowsum(const double *__restrict__ partial, int m, int nb, double *__restrict__ out)
{
    const int j = threadIdx.x;
    if (j >= m) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc = acc + partial[(size_t)j * nb + b];
    out[j] = acc;
}

// y = sum_j c[j] V[j] (j ascending)
__global__ __launch_bounds__(256) void k_combine(const double *__restrict__ V, size_t ld, int m,
                                                 const double *__restrict__ c, size_t n, double *__restrict__ y)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc = acc + c[j] * V[(size_t)j * ld + i];
    y[i] = acc;
}

// r = W c - theta u, with u = V c (both written)
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ V, const double *__restrict__ W,
                                                  size_t ld, int m, const double *__restrict__ c, double theta,
                                                  size_t n, double *__restrict__ u, double *__restrict__ wc,
                                                  double *__restrict__ r)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double a = 0.0, b = 0.0;
    for (int j = 0; j < m; ++j) {
        a = a + c[j] * V[(size_t)j * ld + i];
        b = b + c[j] * W[(size_t)j * ld + i];
    }
    u[i] = a;
    wc[i] = b;
    r[i] = b - theta * a;
}

// shifted Jacobi: t = r / (D - theta), the denominator kept away from zero
__global__ __launch_bounds__(256) void k_precond(const double *__restrict__ r, const double *__restrict__ diag,
                                                 double theta, size_t n, double *__restrict__ t)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double d = diag[i] - theta;
    if (fabs(d) < 1e-8) d = d < 0.0 ? -1e-8 : 1e-8;
    t[i] = r[i] / d;
}

// t = t - sum_j h[j] V[j]
__global__ __launch_bounds__(256) void k_orth(const double *__restrict__ V, size_t ld, int m,
                                              const double *__restrict__ hcoef, size_t n, double *__restrict__ t)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double acc = t[i];
    for (int j = 0; j < m; ++j) acc = acc - hcoef[j] * V[(size_t)j * ld + i];
    t[i] = acc;
}

__global__ __launch_bounds__(256) void k_scale_copy(const double *__restrict__ x, double a, size_t n,
                                                    double *__restrict__ y)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

// lowest eigenpair of a small symmetric matrix (row-major, m x m) by cyclic
// Jacobi rotations (Golub and Van Loan, Sec. 8.5)
void small_lowest(const std::vector<double> &A_in, int m, double &theta, std::vector<double> &vec)
{
    std::vector<double> A = A_in, Q((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < m; ++p)
            for (int q = 0; q < m; ++q) {
                tot += A[(size_t)p * m + q] * A[(size_t)p * m + q];
                if (p != q) off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < m; ++k) {
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double qkp = Q[(size_t)k * m + p], qkq = Q[(size_t)k * m + q];
                    Q[(size_t)k * m + p] = c * qkp - s * qkq;
                    Q[(size_t)k * m + q] = s * qkp + c * qkq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < m; ++i)
        if (A[(size_t)i * m + i] < A[(size_t)best * m + best]) best = i;
    theta = A[(size_t)best * m + best];
    vec.assign((size_t)m, 0.0);
    for (int k = 0; k < m; ++k) vec[(size_t)k] = Q[(size_t)k * m + best];
}

}  // namespace

// ---------------------------------------------------------------- HMat
HMat::~HMat() { release(); }

void HMat::release()
{
    if (rowptr || cols || vals || diag) {
        (void)hipSetDevice(device);
        (void)hipFree(rowptr);
        (void)hipFree(cols);
        (void)hipFree(vals);
        (void)hipFree(diag);
    }
    rowptr = nullptr;
    cols = nullptr;
    vals = nullptr;
    diag = nullptr;
    nrows = nnz = 0;
}

void hmat_build(asci_ctx *ctx, const double *h, const double *eri, int n, int na, int nb, const uint64_t *dets,
                int64_t ndets, double ecore, HMat &H, hipStream_t s)
{
    require(ndets >= 1 && ndets < ((int64_t)1 << 31), ASCI_EINVAL, "ndets must be in [1, 2^31)");
    validate_dets(ctx, dets, ndets, n, na, nb, s);
    H.release();
    H.device = ctx->device;
    const uint32_t nd = (uint32_t)ndets;
    const uint32_t nchunks = (nd + kChunk - 1) / kChunk;
    Arena &ar = ctx->main;
    ar.reset();
    ar.reserve((size_t)(2 * n * n + n) * 8 + (size_t)nd * 4 + (size_t)nchunks * 8 + 4096);
    ar.reset();
    double *jk = ar.take<double>((size_t)2 * n * n + n);
    uint32_t *cnt = ar.take<uint32_t>(nd);
    unsigned long long *csum = ar.take<unsigned long long>(nchunks);
    ASCI_HIP(hipMalloc((void **)&H.rowptr, ((size_t)nd + 1) * sizeof(int64_t)));
    ASCI_HIP(hipMalloc((void **)&H.diag, (size_t)nd * sizeof(double)));
    fault_clear(s);
    k_hm_table<<<(unsigned)((n * n + kHBlock - 1) / kHBlock), kHBlock, 0, s>>>(eri, h, n, jk);
    ASCI_LAUNCH_CHECK();

    HBuildArgs g;
    g.dets = dets;
    g.nd = nd;
    g.n = n;
    g.ecore = ecore;
    g.h = h;
    g.eri = eri;
    g.jk = jk;
    g.rowcnt = cnt;
    g.rowptr = H.rowptr;
    g.cols = nullptr;
    g.vals = nullptr;
    g.diag = H.diag;
    const unsigned grid = (unsigned)((nd + (kHBlock / 64) * kHRows - 1) / ((kHBlock / 64) * kHRows));
    Profiler *prof = &ctx->prof;
    {
        ProfScope ps(prof, "hbuild_count", 0.0, s);
        k_hbuild<false><<<grid, kHBlock, 0, s>>>(g);
        ASCI_LAUNCH_CHECK();
    }
    k_chunk_sums<<<nchunks, 256, 0, s>>>(cnt, nd, csum);
    ASCI_LAUNCH_CHECK();
    // chunk bases on the host (one value per 4096 rows)
    std::vector<unsigned long long> hb(nchunks);
    ASCI_HIP(hipMemcpyAsync(hb.data(), csum, nchunks * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    ASCI_HIP(hipStreamSynchronize(s));
    unsigned long long tot = 0;
    for (uint32_t c = 0; c < nchunks; ++c) {
        const unsigned long long v = hb[c];
        hb[c] = tot;
        tot += v;
    }
    ASCI_HIP(hipMemcpyAsync(csum, hb.data(), nchunks * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
    k_chunk_scan<<<nchunks, 256, 0, s>>>(cnt, nd, csum, H.rowptr);
    ASCI_LAUNCH_CHECK();
    const int64_t nnz = (int64_t)tot;
    ASCI_HIP(hipMemcpyAsync(H.rowptr + nd, &nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
    ASCI_HIP(hipMalloc((void **)&H.cols, (size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
    ASCI_HIP(hipMalloc((void **)&H.vals, (size_t)std::max<int64_t>(nnz, 1) * sizeof(double)));
    g.cols = H.cols;
    g.vals = H.vals;
    {
        ProfScope ps(prof, "hbuild_fill", 12.0 * (double)nnz, s);
        k_hbuild<true><<<grid, kHBlock, 0, s>>>(g);
        ASCI_LAUNCH_CHECK();
    }
    HostStage &hst = ctx->stage;
    hst.reserve(256);
    fault_fetch((unsigned int *)((char *)hst.ptr + 64), s);
    ASCI_HIP(hipStreamSynchronize(s));
    fault_check(*(unsigned int *)((char *)hst.ptr + 64), "the Hamiltonian build");
    H.nrows = ndets;
    H.nnz = nnz;
}

void hmat_matvec(const HMat &H, const double *x, double *y, hipStream_t s, Profiler *prof)
{
    ProfScope ps(prof, "spmv", 12.0 * (double)H.nnz + 16.0 * (double)H.nrows, s);
    k_spmv<<<(unsigned)((H.nrows + 3) / 4), 256, 0, s>>>(H.rowptr, H.cols, H.vals, x, y, (uint32_t)H.nrows);
    ASCI_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Davidson (Alg. 5)
// The subspace V (orthonormal columns) and W = H V grow one vector per
// iteration; the projected matrix V^T W is solved on the host; the residual
// of the lowest Ritz pair is preconditioned by (D - theta)^-1, orthogonalised
// twice against V and appended.  A full subspace restarts from the Ritz vector.
DavidsonOut davidson(asci_ctx *ctx, const HMat &H, const double *guess, const DavidsonOpts &o, double *vec,
                     hipStream_t s)
{
    const size_t N = (size_t)H.nrows;
    const int mmax = std::max(2, std::min(o.max_subspace, kMaxSub));
    Arena &ar = ctx->main;
    ar.reset();
    ar.reserve((size_t)2 * mmax * N * 8 + 6 * N * 8 + (size_t)kDotBlocks * kMaxSub * 8 + 4 * kMaxSub * 8 +
               64 * 256);
    ar.reset();
    double *V = ar.take<double>((size_t)mmax * N);
    double *W = ar.take<double>((size_t)mmax * N);
    double *u = ar.take<double>(N), *wc = ar.take<double>(N), *r = ar.take<double>(N), *t = ar.take<double>(N);
    double *partial = ar.take<double>((size_t)kDotBlocks * kMaxSub);
    double *dsmall = ar.take<double>(4 * kMaxSub);
    Profiler *prof = &ctx->prof;
    const unsigned nb = (unsigned)std::min<size_t>(kDotBlocks, std::max<size_t>(1, (N + 255) / 256));
    // pinned staging: [0, kMaxSub) results coming back, [kMaxSub, 2 kMaxSub)
    // coefficients going out; every upload is followed by a synchronising
    // download before the next upload reuses the buffer
    HostStage &hst = ctx->stage;
    hst.reserve(2 * kMaxSub * sizeof(double));
    double *h_down = (double *)hst.ptr, *h_up = h_down + kMaxSub;

    // dots of the first m columns of M with x, on the host
    auto dots = [&](const double *M, int m, const double *x) {
        k_multidot<<<nb, 256, 0, s>>>(M, N, m, x, N, partial);
        ASCI_LAUNCH_CHECK();
        k_rowsum<<<1, 64, 0, s>>>(partial, m, (int)nb, dsmall);
        ASCI_LAUNCH_CHECK();
        ASCI_HIP(hipMemcpyAsync(h_down, dsmall, m * sizeof(double), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        return std::vector<double>(h_down, h_down + m);
    };
    auto upload = [&](const std::vector<double> &c) {
        std::memcpy(h_up, c.data(), c.size() * sizeof(double));
        ASCI_HIP(hipMemcpyAsync(dsmall + kMaxSub, h_up, c.size() * sizeof(double), hipMemcpyHostToDevice, s));
        return dsmall + kMaxSub;
    };
    // orthogonalise t against V[0..m) twice and normalise it into V[m]; false
    // when nothing independent is left
    auto append = [&](int m, double ref) -> bool {
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<double> hcoef = dots(V, m, t);
            k_orth<<<blocks_for(N), 256, 0, s>>>(V, N, m, upload(hcoef), N, t);
            ASCI_LAUNCH_CHECK();
        }
        const double nrm = std::sqrt(dots(t, 1, t)[0]);
        if (!(nrm > 1e-12 * std::max(ref, 1e-300))) return false;
        k_scale_copy<<<blocks_for(N), 256, 0, s>>>(t, 1.0 / nrm, N, V + (size_t)m * N);
        ASCI_LAUNCH_CHECK();
        hmat_matvec(H, V + (size_t)m * N, W + (size_t)m * N, s, prof);
        return true;
    };

    // start vector: the guess, else the unit vector of the lowest diagonal element
    if (guess) {
        ASCI_HIP(hipMemcpyAsync(t, guess, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        std::vector<double> d(N);
        ASCI_HIP(hipMemcpyAsync(d.data(), H.diag, N * sizeof(double), hipMemcpyDeviceToHost, s));
        ASCI_HIP(hipStreamSynchronize(s));
        size_t best = 0;
        for (size_t i = 1; i < N; ++i)
            if (d[i] < d[best]) best = i;
        std::vector<double> e(N, 0.0);
        e[best] = 1.0;
        ASCI_HIP(hipMemcpyAsync(t, e.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
        ASCI_HIP(hipStreamSynchronize(s));
    }
    const double n0 = std::sqrt(dots(t, 1, t)[0]);
    require(n0 > 0.0, ASCI_EINVAL, "Davidson guess vector is zero");
    k_scale_copy<<<blocks_for(N), 256, 0, s>>>(t, 1.0 / n0, N, V);
    ASCI_LAUNCH_CHECK();
    hmat_matvec(H, V, W, s, prof);
    int m = 1;
    std::vector<double> A((size_t)mmax * mmax, 0.0);
    A[0] = dots(W, 1, V)[0];

    DavidsonOut out{0.0, 0.0, 0, false};
    std::vector<double> c;
    double theta = 0.0;
    for (int it = 1; it <= o.max_iter; ++it) {
        std::vector<double> Am((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Am[(size_t)i * m + j] = A[(size_t)i * mmax + j];
        small_lowest(Am, m, theta, c);
        k_residual<<<blocks_for(N), 256, 0, s>>>(V, W, N, m, upload(c), theta, N, u, wc, r);
        ASCI_LAUNCH_CHECK();
        const double rn = std::sqrt(dots(r, 1, r)[0]);
        out.energy = theta;
        out.resid = rn;
        out.iters = it;
        if (rn <= o.tol) {
            out.converged = true;
            break;
        }
        k_precond<<<blocks_for(N), 256, 0, s>>>(r, H.diag, theta, N, t);
        ASCI_LAUNCH_CHECK();
        if (m == mmax) {
            // restart from the Ritz vector (u, W u) alone
            ASCI_HIP(hipMemcpyAsync(V, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            ASCI_HIP(hipMemcpyAsync(W, wc, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            std::fill(A.begin(), A.end(), 0.0);
            A[0] = theta;
            m = 1;
        }
        const double tn = std::sqrt(dots(t, 1, t)[0]);
        if (!append(m, tn)) break;
        // new row and column of the projected matrix: V^T (H v_m)
        const std::vector<double> col = dots(V, m + 1, W + (size_t)m * N);
        for (int i = 0; i <= m; ++i) {
            A[(size_t)i * mmax + m] = col[(size_t)i];
            A[(size_t)m * mmax + i] = col[(size_t)i];
        }
        ++m;
    }
    // the Ritz vector of the last projected solve
    ASCI_HIP(hipMemcpyAsync(vec, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    ASCI_HIP(hipStreamSynchronize(s));
    return out;
}

}  // namespace asci
