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
    int32_t constraint_level;  /* constraint classes by the top-L occupied alpha
                                  orbitals (Sec. II.B); only 3 (triplets) for now   */
    double ecore;              /* constant added to every H_aa (E0 must include it) */
    int64_t pair_buffer_bytes; /* cap on the pair buffer of one class batch;
                                  0 = automatic                                    */
} asci_options;

typedef struct asci_ctx asci_ctx;

/* Library version, (major << 16) | minor. */
int asci_version(void);

/* Static description of an error code; never NULL. */
const char *asci_strerror(int code);

/* Description of the last failure on the calling thread ("" if none). */
const char *asci_last_error(void);

/* Fill *opt with the defaults (ncore 0, eps 0, constraint_level 3, ecore 0,
 * pair_buffer_bytes 0). */
void asci_options_default(asci_options *opt);

/* Create a context bound to HIP device `device`; it owns a workspace that grows
 * on demand and is reused by later calls.  A context must not be used by two
 * host threads at once. */
int asci_ctx_create(int device, asci_ctx **out);
int asci_ctx_destroy(asci_ctx *ctx);

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
 * Pair counts per triplet constraint class (Sec. II.B; the work estimate of
 * the load-balancing algorithm, Alg. 3): a target belongs to the class named
 * by the mask of the three highest occupied orbitals of its alpha string (all
 * of them when nalpha < 3).  For the core set chosen by opt->ncore, returns
 * the non-empty classes in ascending mask order: h_masks[j], h_counts[j]
 * (host arrays of length capacity).  *out_nclasses receives the number of
 * non-empty classes; beyond capacity the call returns ASCI_ENOMEM.
 * d_dets, d_coeffs: device.
 */
int asci_class_counts_device(asci_ctx *ctx, int norb, int nalpha, int nbeta,
                             const uint64_t *d_dets, const double *d_coeffs, int64_t ndets,
                             const asci_options *opt, int64_t capacity, uint64_t *h_masks,
                             int64_t *h_counts, int64_t *out_nclasses, void *stream);

/*
 * Variational energy E = <C|H|C> = sum_ij C_i H_ij C_j over the given
 * determinants (E_k of Eq. (1)), by a double loop over determinant pairs on
 * the device.  C is used as given (not normalised).  d_*: device.
 */
int asci_energy_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb,
                       int nalpha, int nbeta, const uint64_t *d_dets, const double *d_coeffs,
                       int64_t ndets, double ecore, double *out_energy, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ASCI_H */
