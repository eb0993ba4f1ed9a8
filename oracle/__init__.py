"""CPU oracle for the ASCI determinant search -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library (the HIP path) never
imports, links or calls it.

The arithmetic lives in ``asci_oracle.c`` (plain C, compiled with gcc
``-O2 -ffp-contract=off -fopenmp``); this module compiles it and wraps it with
ctypes.  Which passage of the paper each function follows is stated in the C
file.  Every function here is pinned by tests against brute force, closed
forms, invariants or another oracle function that is itself pinned; none is
"parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asci_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the shared-library path."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Result(C.Structure):
    _fields_ = [("count", C.c_int64), ("keys", C.POINTER(C.c_uint64)),
                ("num", C.POINTER(C.c_double)), ("hdiag", C.POINTER(C.c_double)),
                ("score", C.POINTER(C.c_double)), ("num_abs", C.POINTER(C.c_double)),
                ("hdiag_abs", C.POINTER(C.c_double)), ("tol", C.POINTER(C.c_double)),
                ("npairs", C.c_int64)]


class _BucketStats(C.Structure):
    _fields_ = [("candidates", C.c_int64), ("npairs", C.c_int64), ("pt2", C.c_double),
                ("pt2_abs", C.c_double), ("pt2_tol", C.c_double), ("max_drop_upper", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp, up, ip = C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.POINTER(C.c_int64)
        L.oracle_hdiag.restype = C.c_double
        L.oracle_hdiag.argtypes = [dp, dp, C.c_int, C.c_double, C.c_uint64, C.c_uint64]
        L.oracle_helem.restype = C.c_double
        L.oracle_helem.argtypes = [dp, dp, C.c_int, C.c_double, C.c_uint64, C.c_uint64,
                                   C.c_uint64, C.c_uint64]
        L.oracle_sd_count.restype = C.c_int64
        L.oracle_sd_count.argtypes = [C.c_int, C.c_int, C.c_int]
        L.oracle_sd_targets.restype = C.c_int64
        L.oracle_sd_targets.argtypes = [C.c_int, C.c_uint64, C.c_uint64, up]
        L.oracle_core_set.restype = C.c_int64
        L.oracle_core_set.argtypes = [dp, C.c_int64, C.c_int64, ip]
        L.oracle_search.restype = C.c_int
        L.oracle_search.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, up, dp,
                                    C.c_int64, C.c_double, C.c_int64, C.c_double, C.c_int,
                                    C.POINTER(_Result)]
        L.oracle_free.restype = None
        L.oracle_free.argtypes = [C.POINTER(_Result)]
        L.oracle_topk.restype = C.c_int64
        L.oracle_topk.argtypes = [up, dp, C.c_int64, C.c_int64, ip]
        L.oracle_energy.restype = C.c_double
        L.oracle_energy.argtypes = [dp, dp, C.c_int, C.c_double, up, dp, C.c_int64]
        L.oracle_class_counts.restype = C.c_int64
        L.oracle_class_counts.argtypes = [C.c_int, C.c_int, C.c_int, up, dp, C.c_int64,
                                          C.c_int64, C.c_int, up, ip, C.c_int64]
        L.oracle_pt2.restype = C.c_int
        L.oracle_pt2.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, up, dp, C.c_int64, C.c_double,
                                 C.c_int64, C.c_double, dp, dp, ip]
        L.oracle_target_numerators.restype = C.c_int
        L.oracle_target_numerators.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, up, dp,
                                               C.c_int64, C.c_int64, up, C.c_int64, dp, dp,
                                               C.POINTER(C.c_int), ip, dp, dp]
        L.oracle_score_tol.restype = C.c_double
        L.oracle_score_tol.argtypes = [C.c_double] * 5
        L.oracle_search_buckets.restype = C.c_int
        L.oracle_search_buckets.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, up, dp,
                                            C.c_int64, C.c_double, C.c_int64, C.c_double, C.c_int, C.c_int,
                                            C.c_int, C.c_int, C.c_int64, C.POINTER(_Result),
                                            C.POINTER(_BucketStats)]
        L.oracle_hmat_dense.restype = C.c_int
        L.oracle_hmat_dense.argtypes = [dp, dp, C.c_int, C.c_double, up, C.c_int64, dp, dp]
        L.oracle_balance.restype = C.c_int
        L.oracle_balance.argtypes = [ip, C.c_int64, C.c_int, C.POINTER(C.c_int), ip]
        _lib = L
    return _lib


def _d(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return x, x.ctypes.data_as(C.POINTER(C.c_double))


def _u(x):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    return x, x.ctypes.data_as(C.POINTER(C.c_uint64))


def _ham(h, eri):
    h, hp = _d(h)
    eri, ep = _d(eri)
    n = h.shape[0]
    if h.shape != (n, n) or eri.size != n ** 4:
        raise ValueError("integral shapes")
    return (h, eri), hp, ep, n


def hdiag(h, eri, alpha, beta, ecore=0.0):
    keep, hp, ep, n = _ham(h, eri)
    return lib().oracle_hdiag(hp, ep, n, ecore, int(alpha), int(beta))


def helem(h, eri, a, i, ecore=0.0):
    """<a|H|i> for determinants a = (alpha, beta), i = (alpha, beta)."""
    keep, hp, ep, n = _ham(h, eri)
    return lib().oracle_helem(hp, ep, n, ecore, int(a[0]), int(a[1]), int(i[0]), int(i[1]))


def sd_count(n, na, nb):
    return lib().oracle_sd_count(n, na, nb)


def sd_targets(n, alpha, beta):
    na, nb = bin(int(alpha)).count("1"), bin(int(beta)).count("1")
    cap = sd_count(n, na, nb)
    out = np.zeros(2 * cap + 2, dtype=np.uint64)
    cnt = lib().oracle_sd_targets(n, int(alpha), int(beta), out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return out[: 2 * cnt].reshape(cnt, 2)


def core_set(coeffs, ncore):
    c, cp = _d(coeffs)
    out = np.zeros(len(c) + 1, dtype=np.int64)
    m = lib().oracle_core_set(cp, len(c), int(ncore), out.ctypes.data_as(C.POINTER(C.c_int64)))
    return out[:m]


def energy(h, eri, dets, coeffs, ecore=0.0):
    """<C|H|C> by the plain double loop."""
    keep, hp, ep, n = _ham(h, eri)
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    return lib().oracle_energy(hp, ep, n, ecore, dp, cp, len(c))


_FIELDS = ("num", "hdiag", "score", "num_abs", "hdiag_abs", "tol")


def _take(r):
    """Copy an oracle_result into numpy arrays (the C side is freed by the caller)."""
    u = r.count
    out = {"keys": np.ctypeslib.as_array(r.keys, shape=(2 * u,)).reshape(u, 2).copy() if u
           else np.zeros((0, 2), np.uint64), "npairs": r.npairs}
    for f in _FIELDS:
        out[f] = np.ctypeslib.as_array(getattr(r, f), shape=(u,)).copy() if u else np.zeros(0)
    return out


def score_tol(num, num_abs, hdiag, hdiag_abs, E0):
    """Absolute tolerance of a score evaluated in another order (C: oracle_score_tol)."""
    return lib().oracle_score_tol(float(num), float(num_abs), float(hdiag), float(hdiag_abs), float(E0))


def search_all(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore=0, eps=0.0, ecore=0.0,
               keep_psi=False):
    """Every candidate of the search: dict of keys (U x 2 uint64, ascending),
    num (N_a), hdiag (H_aa), score (A_a), the magnitude sums num_abs and
    hdiag_abs, tol (absolute score tolerance of another evaluation order), npairs."""
    keep, hp, ep, n = _ham(h, eri)
    if n != norb:
        raise ValueError("norb does not match the integrals")
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    r = _Result()
    rc = lib().oracle_search(hp, ep, n, nalpha, nbeta, ecore, dp, cp, len(c), float(E0),
                             int(ncore), float(eps), int(bool(keep_psi)), C.byref(r))
    if rc != 0:
        raise ValueError("oracle_search failed with code %d" % rc)
    try:
        out = _take(r)
    finally:
        lib().oracle_free(C.byref(r))
    return out


def search_buckets(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore=0, eps=0.0, ecore=0.0, nbuckets=64,
                   buckets=None, threads=None, keep_top=0):
    """The search computed by target buckets (C: oracle_search_buckets): the
    candidates of buckets [b0, b1) (default all), bucket by bucket, ascending key
    inside a bucket, or each bucket's keep_top best by (|A| desc, key asc).
    Returns (dict as search_all, stats dict)."""
    keep, hp, ep, n = _ham(h, eri)
    if n != norb:
        raise ValueError("norb does not match the integrals")
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    b0, b1 = (0, nbuckets) if buckets is None else buckets
    if threads is None:
        threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    r = _Result()
    st = _BucketStats()
    rc = lib().oracle_search_buckets(hp, ep, n, nalpha, nbeta, ecore, dp, cp, len(c), float(E0), int(ncore),
                                     float(eps), int(nbuckets), int(b0), int(b1), int(threads), int(keep_top),
                                     C.byref(r), C.byref(st))
    try:
        if rc != 0:
            raise ValueError("oracle_search_buckets failed with code %d" % rc)
        out = _take(r)
    finally:
        lib().oracle_free(C.byref(r))
    stats = {f: getattr(st, f) for f, _ in _BucketStats._fields_}
    stats["threads"] = threads
    return out, stats


def topk_index(keys, score, k):
    keys, kp = _u(keys)
    s, sp = _d(score)
    out = np.zeros(max(int(k), 0) + 1, dtype=np.int64)
    m = lib().oracle_topk(kp, sp, len(s), int(k), out.ctypes.data_as(C.POINTER(C.c_int64)))
    if m < 0:
        raise ValueError("k < 0")
    return out[:m]


def search(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, k, ncore=0, eps=0.0, ecore=0.0):
    """The search result: (dets[m,2] uint64, scores[m]) ordered by |score|
    descending, ties by key ascending; m = min(k, number of candidates)."""
    allc = search_all(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore, eps, ecore)
    idx = topk_index(allc["keys"], allc["score"], k)
    return allc["keys"][idx], allc["score"][idx]


def class_counts(norb, nalpha, nbeta, dets, coeffs, ncore=0, level=3):
    """Non-empty constraint classes of the given level (3 = triplets):
    (masks ascending, pair counts)."""
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    cap = 1
    for _ in range(2):
        masks = np.zeros(cap, dtype=np.uint64)
        counts = np.zeros(cap, dtype=np.int64)
        m = lib().oracle_class_counts(norb, nalpha, nbeta, dp, cp, len(c), int(ncore), int(level),
                                      masks.ctypes.data_as(C.POINTER(C.c_uint64)),
                                      counts.ctypes.data_as(C.POINTER(C.c_int64)), cap)
        if m < 0:
            raise ValueError("invalid determinants")
        if m <= cap:
            return masks[:m], counts[:m]
        cap = m
    raise RuntimeError("class count changed between calls")


def target_numerators(h, eri, norb, nalpha, nbeta, dets, coeffs, targets, ncore=0, ecore=0.0, with_abs=False):
    """For each target determinant: (N_a, H_aa, is an input determinant, number of
    connected core determinants), evaluated one target at a time; with_abs adds
    the magnitude sums (num_abs, hdiag_abs) of the tolerance."""
    keep, hp, ep, n = _ham(h, eri)
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    t, tp = _u(np.asarray(targets, dtype=np.uint64).reshape(-1, 2))
    m = t.shape[0]
    num = np.zeros(m)
    hd = np.zeros(m)
    inp = np.zeros(m, dtype=np.int32)
    nconn = np.zeros(m, dtype=np.int64)
    na_, ha_ = np.zeros(m), np.zeros(m)
    rc = lib().oracle_target_numerators(hp, ep, n, nalpha, nbeta, ecore, dp, cp, len(c), int(ncore), tp, m,
                                        num.ctypes.data_as(C.POINTER(C.c_double)),
                                        hd.ctypes.data_as(C.POINTER(C.c_double)),
                                        inp.ctypes.data_as(C.POINTER(C.c_int)),
                                        nconn.ctypes.data_as(C.POINTER(C.c_int64)),
                                        na_.ctypes.data_as(C.POINTER(C.c_double)),
                                        ha_.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ValueError("invalid determinants")
    if with_abs:
        return num, hd, inp.astype(bool), nconn, na_, ha_
    return num, hd, inp.astype(bool), nconn


def pt2(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore=0, eps=0.0, ecore=0.0, with_abs=False):
    """E_PT2 = sum over candidates of N_a^2 / (E0 - H_aa), summed with
    compensation; returns (energy, candidates), or (energy, candidates, S)
    with S = sum of |terms| when with_abs is set."""
    keep, hp, ep, n = _ham(h, eri)
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    e = C.c_double()
    sabs = C.c_double()
    cnt = C.c_int64()
    rc = lib().oracle_pt2(hp, ep, n, nalpha, nbeta, ecore, dp, cp, len(c), float(E0), int(ncore), float(eps),
                          C.byref(e), C.byref(sabs), C.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_pt2 failed with code %d" % rc)
    if with_abs:
        return e.value, cnt.value, sabs.value
    return e.value, cnt.value


def balance(counts, npe):
    """Alg. 3: (owner[m] (-1 for empty classes), work[npe])."""
    c = np.ascontiguousarray(counts, dtype=np.int64)
    owner = np.zeros(len(c), dtype=np.int32)
    work = np.zeros(int(npe), dtype=np.int64)
    rc = lib().oracle_balance(c.ctypes.data_as(C.POINTER(C.c_int64)), len(c), int(npe),
                              owner.ctypes.data_as(C.POINTER(C.c_int)), work.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc != 0:
        raise ValueError("oracle_balance failed with code %d" % rc)
    return owner, work


# ---------------------------------------------------------------- the ASCI loop (Alg. 1)

def hamiltonian(h, eri, dets, ecore=0.0, with_abs=False):
    """Dense H over a determinant set by the plain double loop (Sec. II.C):
    <D_i|H|D_j> where the two differ by at most a double excitation, else 0;
    with_abs also returns the sum of |terms| of every element."""
    keep, hp, ep, n = _ham(h, eri)
    d, dp = _u(dets)
    nd = len(d)
    out = np.zeros((nd, nd))
    ab = np.zeros((nd, nd)) if with_abs else None
    lib().oracle_hmat_dense(hp, ep, n, float(ecore), dp, nd, out.ctypes.data_as(C.POINTER(C.c_double)),
                            ab.ctypes.data_as(C.POINTER(C.c_double)) if with_abs else None)
    return (out, ab) if with_abs else out


def lowest(H):
    """Lowest eigenpair of a dense symmetric matrix (LAPACK through numpy)."""
    w, v = np.linalg.eigh(H)
    return float(w[0]), v[:, 0]


def select_next(dets, coeffs, cand, cand_scores, ntdets):
    """Alg. 1's selection: the ntdets entries of largest score over psi_k
    (score |C_i|) and the new determinants (score |A_a|), ties by (alpha, beta)
    ascending, in that order.  Returns (dets, guess coefficients) where the
    guess is C_i on kept determinants and 0 on new ones."""
    dets = np.asarray(dets, dtype=np.uint64).reshape(-1, 2)
    cand = np.asarray(cand, dtype=np.uint64).reshape(-1, 2)
    allk = np.concatenate([dets, cand])
    score = np.concatenate([np.abs(np.asarray(coeffs, float)), np.abs(np.asarray(cand_scores, float))])
    guess = np.concatenate([np.asarray(coeffs, float), np.zeros(len(cand))])
    # compare |score| by its IEEE bits, as the selection of the search does
    ordkey = score.view(np.uint64)
    order = np.lexsort((allk[:, 1], allk[:, 0], ~ordkey))[:ntdets]
    return allk[order], guess[order]


def asci_loop(h, eri, norb, nalpha, nbeta, dets0, coeffs0, ntdets, ncore=0, max_iter=10, e_tol=1e-6, eps=0.0,
              ecore=0.0):
    """Alg. 1 with the oracle search, the double-loop H and a dense
    eigensolver: returns the list of (dets, coeffs, energy) per iteration,
    starting with the input set and E_0 = <C|H|C>."""
    dets = np.asarray(dets0, dtype=np.uint64).reshape(-1, 2)
    C = np.asarray(coeffs0, dtype=float)
    E = energy(h, eri, dets, C, ecore)
    hist = [(dets, C, E)]
    for _ in range(max_iter):
        cand, sc = search(h, eri, norb, nalpha, nbeta, dets, C, E, ntdets, ncore=ncore, eps=eps, ecore=ecore)
        nd, guess = select_next(dets, C, cand, sc, ntdets)
        Enew, Cnew = lowest(hamiltonian(h, eri, nd, ecore))
        hist.append((nd, Cnew, Enew))
        done = abs(Enew - E) < e_tol
        dets, C, E = nd, Cnew, Enew
        if done:
            break
    return hist


# ---------------------------------------------------------------- selection under the score tolerance

def topk_bands(keys, score, tol, k, outside_upper=0.0):
    """Which candidates any evaluation order within the tolerance must select.

    Every score A_a is known to lie in [|A_a| - tol_a, |A_a| + tol_a] (L_a, U_a)
    for a result computed in another order.  A candidate is surely among the k
    selected when fewer than k others can reach its lower bound
    (#{b != a: U_b >= L_a} < k) and it beats every candidate not listed
    (L_a > outside_upper, the largest U of those); it is surely out when k
    others are above it for certain (#{b: L_b > U_a} >= k).  The rest are
    ambiguous: the selection may take either.  Returns (sure_in, ambiguous)
    masks and whether every candidate not listed is surely out."""
    a = np.abs(np.asarray(score, dtype=np.float64))
    tol = np.asarray(tol, dtype=np.float64)
    L, U = a - tol, a + tol
    Us, Ls = np.sort(U), np.sort(L)
    reach = len(U) - np.searchsorted(Us, L, side="left") - 1  # others with U_b >= L_a
    sure_in = (reach < k) & (L > outside_upper)
    above = len(L) - np.searchsorted(Ls, U, side="right")      # others with L_b > U_a
    sure_out = above >= k
    if (sure_in & sure_out).any():
        raise AssertionError("inconsistent tolerance bands")
    outside_ok = outside_upper <= 0.0 or (len(L) - np.searchsorted(Ls, outside_upper, side="right")) >= k
    return sure_in, ~sure_in & ~sure_out, bool(outside_ok)


def key_codes(keys):
    """(alpha, beta) keys as one sortable structured array (order = key order)."""
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64).reshape(-1, 2))
    return keys.view([("a", np.uint64), ("b", np.uint64)]).ravel()
