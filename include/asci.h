/*
 * asci.h -- C ABI of the MI355X (gfx950) ASCI determinant search.
 *
 * The search is the determinant-selection step of adaptive sampling
 * configuration interaction (Williams-Young et al., "A Parallel, Distributed
 * Memory Implementation of the Adaptive Sampling Configuration Interaction
 * Method", Sec. II.A-II.B, Alg. 2): for every core determinant D_i with
 * coefficient C_i, enumerate its single and double excitations D_a, evaluate
 * the Slater-Condon element H_ai, and give every candidate D_a outside the
 * wave function the score (Eq. (1), denominator read as E0 - H_aa)
 *
 *     A_a = N_a / (E0 - H_aa),   N_a = sum_i H_ai C_i  (ascending input index i),
 *
 * then return the k candidates of largest |A_a|.
 *
 * Conventions shared by every entry point:
 *   - norb in [1, 64]; nalpha, nbeta in [0, norb].
 *   - A determinant is two uint64 words {alpha, beta}; bit p is spatial
 *     orbital p.  Arrays of determinants are ndets x 2, row-major.
 *   - Spin orbitals are ordered alpha first, then beta, each ascending; a
 *     determinant is the product of creators in that order acting on the
 *     vacuum.  This fixes the sign of every H_ai, hence of every score.
 *   - h is norb x norb, eri is (pq|rs) in chemists' notation, norb^4,
 *     row-major, real, with the 8-fold permutational symmetry (h symmetric).
 *     The search entry points check the symmetry bit for bit (their
 *     generator reads a packed copy of the distinct entries) and fail with
 *     ASCI_EINVAL otherwise (asynchronous search: status ASCI_EINVAL).
 *   - The candidate key order is (alpha, beta) compared as unsigned integers.
 *   - Output order is |A| descending (compared as the IEEE-754 bit pattern of
 *     |A|, i.e. numerically for non-NaN values), ties by key ascending.
 *   - Candidates exclude every input determinant, not only the core set.
 *   - All arithmetic is IEEE binary64 without fused multiply-add; H_aa and the
 *     single-excitation sums are evaluated in ascending orbital order, so the
 *     result is deterministic run to run.
 *
 * Ownership: the caller owns every input and output buffer.  The library
 * owns its device workspace (held by an asci_ctx and reused across calls).
 * Errors: every entry point returns ASCI_OK (0) or a negative code; a failed
 * call leaves its outputs unwritten (output counts excepted where stated).
 */
#ifndef ASCI_H
#define ASCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASCI_OK 0
#define ASCI_EINVAL (-1)  /* invalid argument or input determinants          */
#define ASCI_ENOMEM (-2)  /* device memory, or a capacity given by the caller */
#define ASCI_EDEVICE (-3) /* a HIP call failed                                */

typedef struct asci_options {
    int64_t ncore;             /* core set size N_cdets (Alg. 2): the ncore inputs of
                                  largest |C| (ties: lower index); 0 = all inputs    */
    double eps;                /* pair threshold eps_search (Alg. 2): keep a pair
                                  only if |H_ai C_i / (E0 - H_aa)| > eps; 0 = exact  */
    int32_t constraint_level;  /* L in [1, 6]: constraint classes by the top-L
                                  occupied alpha orbitals (Sec. II.B; 3 = triplets) */
    double ecore;              /* constant added to every H_aa (E0 must include it) */
    int64_t pair_buffer_bytes; /* cap on the pair buffer of one class batch;
                                  0 = automatic                                    */
    int64_t split_pairs;       /* 0: every class at level L.  > 0: classes start at
                                  level min(L, 3) and a class with more pairs than
                                  this is split into the classes of the next level,
                                  up to L (Sec. II.B: only heavy classes are split).
                                  Either way a class larger than the pair buffer is
                                  split further, up to level 6.  The classes only
                                  partition the work: results do not depend on
                                  L or split_pairs.                                 */
} asci_options;

typedef struct asci_ctx asci_ctx;

/* Library version, (major << 16) | minor. */
int asci_version(void);

/* Static description of an error code; never NULL. */
const char *asci_strerror(int code);

/* Description of the last failure on the calling thread ("" if none). */
const char *asci_last_error(void);

/* Fill *opt with the defaults (ncore 0, eps 0, constraint_level 3, ecore 0,
 * pair_buffer_bytes 0, split_pairs 0). */
void asci_options_default(asci_options *opt);

/* Create a context bound to HIP device `device`; it owns a workspace that grows
 * on demand and is reused by later calls.  A context must not be used by two
 * host threads at once. */
int asci_ctx_create(int device, asci_ctx **out);
int asci_ctx_destroy(asci_ctx *ctx);

/*
 * Tuning parameters of a context (they change speed, never results):
 *   "finish_cap": records per LDS bucket in the sort-and-accumulate finish,
 *                 1024, 2048 or 4096 (default 4096, any key width).  A
 *                 workgroup of cap / 8 threads takes a bucket; smaller
 *                 buckets let more workgroups share a CU but need more split
 *                 passes.
 *   "batch_slots": concurrent searches of asci_search_batch, 1..8 (default 4).
 *   "spin_tables": 1 (default) tabulates E(s) of every alpha and beta string
 *                 (at most 2^27 strings per spin, and only when the search
 *                 has at least four pairs per string) so the diagonal element
 *                 looks them up by string rank; 0 evaluates them directly.
 *                 Both give the same bits (same summation order).
 *   "release_workspace" (value 1): free the context's device workspaces and
 *                 the batch workers (they are allocated again on demand).
 *   "use_tuned": 1 (default) lets a search use the per-shape finish_cap that
 *                 asci_tune_shapes recorded for its shape; 0 always uses
 *                 the context's "finish_cap".
 *   "batch_solo_pairs": requests of asci_search_batch with at least this
 *                 many (core, target) pairs run one at a time on ctx itself
 *                 (default 2^26: searches of that size fill the GPU alone,
 *                 and two of them at once run slower than one after the
 *                 other); 0 sends every request to the workers.
 *   "batch_graph": 1 runs the requests of asci_search_batch that fit
 *                 asci_search_async's scope as one captured graph; 0
 *                 (default) sends them to the worker streams.
 *   "fault_test": 1 makes every later search on ctx raise a forced fault in
 *                 its generator, so that the call fails with ASCI_EDEVICE
 *                 (a test of the error path: the kernels' internal-consistency
 *                 faults, such as a record slot past its buffer, are reported
 *                 the same way); 0 (default) turns it off.
 * Read-only diagnostics of the last search on ctx (asci_ctx_get_param):
 *   "last_batches" (class batches), "last_finals" (LDS buckets),
 *   "last_levels" (deepest bucket split), "last_candidates" (candidates).
 * Unknown names or values: ASCI_EINVAL.
 */
int asci_ctx_set_param(asci_ctx *ctx, const char *name, int64_t value);
int asci_ctx_get_param(asci_ctx *ctx, const char *name, int64_t *value);

/*
 * Per-kernel timing (measurement support, not part of the method).  With
 * profiling on, every timed kernel launch of later calls on ctx is bracketed by
 * HIP events on the call's stream; entries accumulate per kernel name: total
 * milliseconds, number of launches, and the algorithmic bytes those launches
 * must move (inputs read once plus outputs written once).  Enabling (or
 * disabling) clears the entries.  asci_ctx_profile_entry returns ASCI_EINVAL
 * once index is past the last entry; name receives at most name_cap - 1 chars.
 */
int asci_ctx_set_profiling(asci_ctx *ctx, int enable);
/*
 * Restrict profiling to the launches of one kernel name (null or "" = every
 * timed kernel), so that the events bracket only that kernel; set before
 * asci_ctx_set_profiling.
 */
int asci_ctx_profile_only(asci_ctx *ctx, const char *kernel);
int asci_ctx_profile_entry(asci_ctx *ctx, int index, char *name, int name_cap, double *total_ms,
                           int64_t *launches, double *bytes);

/*
 * ASCI search, host buffers (Alg. 2; Eq. (1)).
 *   h[norb*norb], eri[norb^4]: integrals (host).
 *   dets[ndets*2], coeffs[ndets]: the wave function psi_k (host); ndets >= 1;
 *     determinants must be distinct, inside norb, with the given electron counts.
 *   E0: the energy in the score denominator (normally <psi|H|psi>, including ecore).
 *   k >= 1: number of candidates to return (N_tdets).
 *   opt: NULL for the defaults.
 *   out_dets[k*2], out_scores[k] (host): the selected candidates and A_a.
 *   *out_count = min(k, number of candidates).
 * Uses an internal context on the current device.  Synchronous.
 */
int asci_search(const double *h, const double *eri, int norb, int nalpha, int nbeta,
                const uint64_t *dets, const double *coeffs, int64_t ndets, double E0,
                int64_t k, const asci_options *opt, uint64_t *out_dets, double *out_scores,
                int64_t *out_count);

/*
 * ASCI search, device buffers.  Same meaning as asci_search; every array
 * pointer is device memory of ctx's device; work is queued on `stream` (a
 * hipStream_t, NULL = default stream).  The call waits on the stream at a few
 * planning points and returns after the outputs are written.
 */
int asci_search_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb,
                       int nalpha, int nbeta, const uint64_t *d_dets, const double *d_coeffs,
                       int64_t ndets, double E0, int64_t k, const asci_options *opt,
                       uint64_t *d_out_dets, double *d_out_scores, int64_t *out_count,
                       void *stream);

/*
 * The search of asci_search_device for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, meaning and result (the same kernels);
 * no device or pinned host memory is allocated: every device buffer of the
 * call comes from a fixed scratch region of 256 MiB that the library holds
 * on each device it runs on from load time until the process ends, and host
 * readbacks go through a fixed host buffer (the host-side planning still uses
 * the C++ heap).  The pair buffer holds every pair of the search (one class
 * batch) and the spin-string tables are not built (the diagonal element is
 * evaluated directly, the same bits).  A search whose workspace bound
 * exceeds the region (roughly beyond 2.5e6 pairs) is rejected with
 * ASCI_ENOMEM before any device work.  Calls on one device share the region:
 * the library runs them one at a time (each returns after its outputs are
 * written), and a call starts from no state of the previous one.
 */
int asci_search_device_noalloc(const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                               const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double E0,
                               int64_t k, const asci_options *opt, uint64_t *d_out_dets, double *d_out_scores,
                               int64_t *out_count, void *stream);

/*
 * Every candidate of the search (no selection), device buffers: keys in
 * ascending (alpha, beta) order, their numerators N_a and scores A_a.
 * capacity: length of the output arrays.  *out_count receives the number of
 * candidates; when it exceeds capacity the call returns ASCI_ENOMEM and writes
 * nothing else (call again with a larger capacity).
 */
int asci_candidates_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb,
                           int nalpha, int nbeta, const uint64_t *d_dets,
                           const double *d_coeffs, int64_t ndets, double E0,
                           const asci_options *opt, int64_t capacity, uint64_t *d_out_dets,
                           double *d_out_num, double *d_out_scores, int64_t *out_count,
                           void *stream);

/*
 * Second-order (Epstein-Nesbet) energy of the candidates, on the search's own
 * pipeline (Sec. II.A: the PT2 correction is closely related to the scores of
 * Eq. (1); ASCI's final step in Alg. 1):
 *     E_PT2 = sum over candidates a of N_a^2 / (E0 - H_aa) = sum_a N_a * A_a,
 * with N_a, A_a, the core set and eps exactly as in asci_search.  Summation:
 * per bucket of candidates in key order, then a fixed-order tree, so the
 * result is reproducible run to run.  *out_count receives the number of
 * candidates.  d_*: device.
 */
int asci_pt2_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha,
                    int nbeta, const uint64_t *d_dets, const double *d_coeffs, int64_t ndets,
                    double E0, const asci_options *opt, double *out_energy, int64_t *out_count,
                    void *stream);

/*
 * Pair counts per constraint class (Sec. II.B; the work estimate of the
 * load-balancing algorithm, Alg. 3): a target belongs to the class named by the
 * mask of the L = opt->constraint_level highest occupied orbitals of its alpha
 * string (all of them when nalpha < L); with opt->split_pairs > 0 the classes
 * start at level min(L, 3) and only those with more pairs are split, level by
 * level, up to L.  For the core set chosen by opt->ncore, returns the non-empty
 * classes in ascending mask order: h_masks[j], h_counts[j] (host arrays of
 * length capacity; the level of a class is the popcount of its mask).
 * *out_nclasses receives the number of non-empty classes; beyond capacity the
 * call returns ASCI_ENOMEM.  d_dets, d_coeffs: device.
 */
int asci_class_counts_device(asci_ctx *ctx, int norb, int nalpha, int nbeta,
                             const uint64_t *d_dets, const double *d_coeffs, int64_t ndets,
                             const asci_options *opt, int64_t capacity, uint64_t *h_masks,
                             int64_t *h_counts, int64_t *out_nclasses, void *stream);

/*
 * Static load balance of Alg. 3 (host only, no device work): the classes are
 * taken in the given order, and a class with h = counts[c] > 0 pairs goes to
 * the processing element with the smallest load so far (lowest index on ties),
 * whose load then grows by h (the load array is updated after every
 * assignment).  owner[c] receives the element of class c (-1 when h == 0),
 * load[p] the pairs of element p.  counts, owner (nclasses) and load (npe) are
 * caller-owned host arrays.  Errors: ASCI_EINVAL for null pointers,
 * nclasses < 0, npe < 1 or a negative count.
 */
int asci_balance_classes(const int64_t *counts, int64_t nclasses, int32_t npe, int32_t *owner, int64_t *load);

/*
 * Variational energy E = <C|H|C> = sum_ij C_i H_ij C_j over the given
 * determinants (E_k of Eq. (1)), by a double loop over determinant pairs on
 * the device.  C is used as given (not normalised).  d_*: device.
 */
int asci_energy_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb,
                       int nalpha, int nbeta, const uint64_t *d_dets, const double *d_coeffs,
                       int64_t ndets, double ecore, double *out_energy, void *stream);

/* ------------------------------------------------------------------------
 * The variational step and the ASCI loop (Alg. 1, Sec. II.C).
 * ------------------------------------------------------------------------ */

/* Hamiltonian over a determinant set, built by the double loop over
 * determinant pairs (Sec. II.C) and stored as CSR on the device: row i is
 * determinant i of the set, columns ascending, both triangles and the
 * diagonal stored; H_ij = <D_i|H|D_j> by the Slater-Condon rules with the
 * phase convention of the search, H_ii including ecore.  The object owns its
 * device memory until asci_hmat_destroy. */
typedef struct asci_hmat asci_hmat;

/* d_h, d_eri, d_dets: device.  Errors: ASCI_EINVAL (bad sizes, invalid
 * determinants), ASCI_ENOMEM, ASCI_EDEVICE.  The set should hold distinct
 * determinants (a repeated one gives repeated rows). */
int asci_hmat_build_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha,
                           int nbeta, const uint64_t *d_dets, int64_t ndets, double ecore, asci_hmat **out,
                           void *stream);
int asci_hmat_info(const asci_hmat *H, int64_t *nrows, int64_t *nnz);
/* Copy the CSR arrays into caller-owned device buffers (nrows + 1, nnz, nnz). */
int asci_hmat_export(const asci_hmat *H, int64_t *d_rowptr, int32_t *d_cols, double *d_vals, void *stream);
/* d_y = H d_x (device vectors of length nrows). */
int asci_hmat_matvec_device(const asci_hmat *H, const double *d_x, double *d_y, void *stream);
void asci_hmat_destroy(asci_hmat *H);

/* Lowest eigenpair of H by the Davidson method of Alg. 5 with the
 * shifted-Jacobi preconditioner (D - theta)^-1 (D = diag H).  d_guess: device
 * start vector (NULL = the unit vector of the lowest diagonal element).  A full
 * subspace (max_subspace in [2, 48]) restarts from the current Ritz vector.
 * Stops when |H u - theta u| <= tol or after max_iter iterations.  Writes the
 * Ritz value, the unit Ritz vector d_vec (device, nrows), the residual norm
 * and the iterations used. */
int asci_davidson_device(asci_ctx *ctx, const asci_hmat *H, const double *d_guess, int32_t max_subspace,
                         int32_t max_iter, double tol, double *out_energy, double *d_vec, double *out_resid,
                         int32_t *out_iters, void *stream);

typedef struct asci_loop_options {
    int64_t ncore;              /* N_cdets: core determinants of every search (0 = all of psi_k) */
    int64_t ntdets;             /* N_tdets: size of the next determinant set               */
    int32_t max_iter;           /* outer iterations of Alg. 1                              */
    double e_tol;               /* stop when |E_{k+1} - E_k| < e_tol                       */
    int32_t davidson_subspace;  /* largest Davidson subspace, in [2, 48]                   */
    int32_t davidson_max_iter;  /* Davidson iterations per solve                           */
    double davidson_tol;        /* residual norm of a converged Ritz pair                  */
    int32_t pt2;                /* 1: final PT2 step on the last set (exact, eps = 0)      */
    asci_options search;        /* eps, constraint classes, ecore, pair buffer; its ncore is
                                   replaced by the field above                             */
} asci_loop_options;

/* One outer iteration: sizes, energy and the host wall time of each phase. */
typedef struct asci_loop_iter {
    int64_t ndets;       /* size of psi_{k+1}                */
    int64_t candidates;  /* candidates of the search         */
    int64_t nnz;         /* nonzeros of H over psi_{k+1}     */
    double energy;       /* E_{k+1}, lowest Ritz value       */
    double davidson_resid;
    int32_t davidson_iters;
    double search_ms, select_ms, hbuild_ms, davidson_ms;
} asci_loop_iter;

/* Defaults: ncore 0, ntdets 1000, max_iter 10, e_tol 1e-6, Davidson subspace
 * 24, 200 iterations, tol 1e-8, pt2 0, search options as asci_options_default. */
void asci_loop_options_default(asci_loop_options *opt);

/* One iteration of Alg. 1 from psi_k = (d_dets, d_coeffs) with energy Ek:
 * search (top N_tdets new determinants by |A|), selection of psi_{k+1} = the
 * N_tdets entries of largest score among psi_k (score |C_i|) and the new ones
 * (score |A_a|), ties by key ascending, stored in that order; H over psi_{k+1}
 * and Davidson (guess: C_k on the kept determinants, zero elsewhere).  Outputs
 * (device, capacity ntdets): the set, its coefficients; *out_ndets and *info
 * (host).  C_k should be normalised. */
int asci_loop_step_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                          const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double Ek,
                          const asci_loop_options *opt, uint64_t *d_out_dets, double *d_out_coeffs,
                          int64_t *out_ndets, asci_loop_iter *info, void *stream);

/* Alg. 1 from a starting set (e.g. the Hartree-Fock determinant with C = 1):
 * E_0 = <C|H|C>, then iterations until |E_{k+1} - E_k| < e_tol or max_iter,
 * then the optional PT2 step.  Outputs: the final set and coefficients (device,
 * capacity max(ntdets, n0)), *out_ndets, *out_energy, *out_pt2 (0 without the
 * PT2 step), per-iteration records iters[0 .. *out_iters) (host, capacity
 * max_iter). */
int asci_run_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                    const uint64_t *d_dets0, const double *d_coeffs0, int64_t ndets0, const asci_loop_options *opt,
                    uint64_t *d_out_dets, double *d_out_coeffs, int64_t *out_ndets, double *out_energy,
                    double *out_pt2, asci_loop_iter *iters, int32_t *out_iters, void *stream);

/* ------------------------------------------------------------------------
 * Batched and served searches.
 *
 * A request names device buffers that stay resident (integrals, determinant
 * sets) and device outputs of capacity k; its result equals the result of
 * asci_search_device on the same inputs, bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct asci_request {
    const double *h, *eri;     /* device */
    int norb, nalpha, nbeta;
    const uint64_t *dets;      /* device, ndets x 2 */
    const double *coeffs;      /* device */
    int64_t ndets;
    double E0;
    int64_t k;
    asci_options opt;
    uint64_t *out_dets;        /* device, k x 2 */
    double *out_scores;        /* device, k */
} asci_request;

typedef struct asci_result {
    int status;                /* ASCI_OK or an error code */
    int64_t count;             /* candidates written */
    double latency_ms;         /* submission to completion */
    double run_ms;             /* admission to completion */
    int64_t contributions;     /* pairs the search generated */
} asci_result;

/*
 * The search of asci_search_device, queued with nothing read back (Alg. 2;
 * the per-class counts are formed on the fly on the device, Sec. II.B): the
 * class plan, the pair counts, the bucket split levels, the candidate count
 * and the selection run from counts kept in device memory, so the call
 * returns once the work is queued on `stream` and never waits on the device.
 * req names device buffers (req->out_dets, req->out_scores: capacity k);
 * d_result is device memory that receives, when the queued work completes,
 * the number of candidates written (min(k, candidates)) and the status
 * (ASCI_OK, ASCI_EINVAL for invalid or repeated input determinants found on
 * the device, ASCI_EDEVICE for an internal failure); on a failure no output is
 * written and count is 0.  Synchronise the stream (or wait on an event
 * recorded after the call) before reading it.  Results equal
 * asci_search_device's bit for bit.
 * Scope: the search must fit one class batch: every pair in the pair buffer
 * (fewer than 2^31 pairs), split_pairs = 0; when the requested constraint
 * level has more than 2048 classes the highest lower level with at most 2048
 * is used (the classes only partition the work).  Otherwise the call returns
 * ASCI_EINVAL at once and queues nothing.
 * ctx's workspace is in use until the queued work completes: calls that may
 * overlap need contexts of their own (one per stream).  A call that needs more
 * workspace than ctx holds allocates it first (hipMalloc, which may wait for
 * the device); later calls of the same or smaller size allocate nothing.
 * The call itself returns ASCI_OK once queued, or ASCI_EINVAL / ASCI_ENOMEM
 * for argument and workspace failures (nothing queued).
 */
typedef struct asci_async_result {
    int64_t count;   /* candidates written */
    int32_t status;  /* ASCI_OK or an error code */
    int32_t flags;   /* device-side failure bits (0 when status is ASCI_OK) */
} asci_async_result;

int asci_search_async(asci_ctx *ctx, const asci_request *req, asci_async_result *d_result, void *stream);

/* Device bytes asci_search_async's workspace takes for req on ctx (*out_bytes;
 * 0 when req is outside its scope).  Host only; ASCI_EINVAL for bad sizes. */
int asci_request_async_bytes(asci_ctx *ctx, const asci_request *req, int64_t *out_bytes);

/* Device bytes the library budgets for one request (workspace estimate). */
int64_t asci_request_footprint(const asci_request *req);

/*
 * Run nreq searches as one batch on ctx's device.  Requests of at least
 * "batch_solo_pairs" pairs fill the GPU on their own: they run one at a
 * time on ctx (largest first, with its whole workspace) after the others,
 * which run at the same time as follows.  With context parameter
 * "batch_graph" = 1, requests inside the scope of asci_search_async whose
 * workspace fits a share of the free HBM run as one captured HIP graph: placed on "batch_slots" streams (largest first, to
 * the least loaded; each stream with a context of its own) that fork from
 * and join back to one launch stream; the graph is replayed by later calls
 * with the same requests (same buffers, sizes and options) and captured
 * again otherwise.  The other requests are ordered by estimated cost
 * (largest first) and run at the same time on worker streams, each with its
 * own workspace ("batch_graph" = 0, the default, sends every request to the
 * workers).  The workers and the graph's contexts stay with ctx between
 * calls (until "release_workspace", a change of "batch_slots" or
 * "finish_cap", or asci_ctx_destroy); the context's own workspaces are
 * freed when a batch without requests for ctx itself starts, and a search
 * on ctx frees the idle workers' workspaces.  Work already queued on `stream` completes first; the
 * call returns when every result is written.  res[i] is request i's result;
 * the return value is ASCI_OK when every request succeeded, else the first
 * error code.
 */
int asci_search_batch(asci_ctx *ctx, const asci_request *reqs, int nreq, asci_result *res, void *stream);

/*
 * Tune for requests like the given sample: every distinct shape of the
 * sample gets its finish capacity by asci_tune_shapes (synchronous searches
 * on ctx).  *best_finish_cap receives the capacity recorded for the sample's
 * largest request, *best_slots ctx's "batch_slots" (left unchanged).
 * Results never depend on either.
 */
int asci_autotune(asci_ctx *ctx, const asci_request *sample, int nsample, int64_t *best_slots,
                  int64_t *best_finish_cap);

/*
 * Per-shape tuning (speed only, never results): asci_tune_shapes times each
 * distinct shape of the given requests (device architecture, norb, nalpha,
 * floor(log2 pairs)) with the finish capacity ("finish_cap") 4096, 2048 and
 * 1024 (one untimed and two timed searches each, on ctx, synchronous) and
 * records the fastest in a process-wide table; searches on contexts with
 * "use_tuned" = 1 (the default) then use the recorded capacity of their shape.
 * *out_tuned receives the number of shapes timed.  The table can be saved to
 * a text file and loaded in a later process (one "arch norb nalpha bucket
 * finish_cap" line per shape; ASCI_EINVAL for a malformed line), looked up
 * (*finish_cap = 0 when the shape has no entry), recorded directly, and
 * cleared.  asci_tune_arch writes the architecture name the table keys
 * device's entries by ("gfx950", or "unknown" without a device) into
 * buf[cap] (ASCI_EINVAL when it does not fit).
 */
int asci_tune_shapes(asci_ctx *ctx, const asci_request *reqs, int nreq, int *out_tuned);
int asci_tune_record(const char *arch, int norb, int nalpha, int bucket, int finish_cap);
int asci_tune_lookup(int device, int norb, int nalpha, int64_t pairs, int *finish_cap);
int asci_tune_arch(int device, char *buf, int cap);
int asci_tune_clear(void);
int asci_tune_save(const char *path);
int asci_tune_load(const char *path, int *out_entries);

/*
 * A request loop with continuous batching on one device.  Requests wait in
 * arrival order; a free worker slot takes the oldest request whose bytes,
 * added to those budgeted for the running requests and the workspace the
 * workers keep, stay within hbm_budget, so a small request passes a large one
 * that does not fit yet; once the oldest request has waited longer than the
 * age bound ("age_ms", default 250 ms) nothing passes it.  Requests that
 * arrive while others run are admitted as slots and memory free up, and
 * their kernels overlap on the device.  A request is checked at submission
 * like asci_search_device's arguments (ASCI_EINVAL, nothing queued); one whose
 * footprint alone exceeds hbm_budget is rejected with ASCI_ENOMEM.  Request
 * buffers must stay valid until the request completes.  Each result is handed
 * over once, by poll or wait, and then forgotten (a later poll or wait of the
 * ticket returns ASCI_EINVAL).
 */
typedef struct asci_server asci_server;

typedef struct asci_server_stats {
    int64_t submitted, completed, failed, rejected;
    int64_t max_running;        /* most requests running at once */
    int64_t peak_bytes;         /* most bytes budgeted at once (<= hbm_budget) */
    double p50_ms, p99_ms, mean_ms;  /* latency: submission to completion */
    double wall_s;              /* first submission to last completion */
    int64_t contributions;      /* pairs generated by completed requests */
    int64_t bypassed;           /* requests started before an older one that did not fit */
    int64_t held_results;       /* finished results not yet handed over by poll / wait */
} asci_server_stats;

int asci_server_create(int device, int64_t hbm_budget, int slots, asci_server **out);
/* Scheduler test double: no GPU is touched; a request "runs" for
 * footprint * ns_per_byte nanoseconds and keeps its footprint resident. */
int asci_server_create_fake(int64_t hbm_budget, int slots, double ns_per_byte, asci_server **out);
int asci_server_submit(asci_server *srv, const asci_request *req, uint64_t *ticket);
/* Scheduler parameters: "age_ms" (>= 0), the wait after which the oldest
 * request can no longer be passed.  Unknown names or values: ASCI_EINVAL. */
int asci_server_set_param(asci_server *srv, const char *name, double value);
/* Bytes this server budgets for a request: the server caps each request's
 * pair buffer at hbm_budget / (slots * 160) records, so large requests run in
 * more class batches instead of being refused. */
int64_t asci_server_footprint(asci_server *srv, const asci_request *req);
/* ASCI_OK and *res when the request has completed (the result is then
 * forgotten), ASCI_EAGAIN (1) while it has not; ASCI_EINVAL for an unknown
 * ticket or one whose result was already handed over. */
int asci_server_poll(asci_server *srv, uint64_t ticket, asci_result *res);
int asci_server_wait(asci_server *srv, uint64_t ticket, asci_result *res);
int asci_server_get_stats(asci_server *srv, asci_server_stats *st);
/* Waits for running requests, then frees the server. */
int asci_server_destroy(asci_server *srv);

#define ASCI_EAGAIN 1

#ifdef __cplusplus
}
#endif

#endif /* ASCI_H */
