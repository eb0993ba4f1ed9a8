"""CPU oracle for the ASCI determinant search -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library (the HIP path) never
imports, links or calls it.

The arithmetic lives in ``asci_oracle.c`` (plain C, compiled with gcc
``-O2 -ffp-contract=off``); this module compiles it and wraps it with ctypes.
Which passage of the paper each function follows is stated in the C file.
Every function here is pinned by tests against brute force, closed forms or
invariants; none is "parity unpinned".
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
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Result(C.Structure):
    _fields_ = [("count", C.c_int64), ("keys", C.POINTER(C.c_uint64)),
                ("num", C.POINTER(C.c_double)), ("hdiag", C.POINTER(C.c_double)),
                ("score", C.POINTER(C.c_double)), ("npairs", C.c_int64)]


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
                                               C.POINTER(C.c_int), ip]
        L.oracle_hmat_dense.restype = C.c_int
        L.oracle_hmat_dense.argtypes = [dp, dp, C.c_int, C.c_double, up, C.c_int64, dp]
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


def search_all(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore=0, eps=0.0, ecore=0.0,
               keep_psi=False):
    """Every candidate of the search: dict of keys (U x 2 uint64, ascending),
    num (N_a), hdiag (H_aa), score (A_a), npairs."""
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
        u = r.count
        out = {
            "keys": np.ctypeslib.as_array(r.keys, shape=(2 * u,)).reshape(u, 2).copy() if u else np.zeros((0, 2), np.uint64),
            "num": np.ctypeslib.as_array(r.num, shape=(u,)).copy() if u else np.zeros(0),
            "hdiag": np.ctypeslib.as_array(r.hdiag, shape=(u,)).copy() if u else np.zeros(0),
            "score": np.ctypeslib.as_array(r.score, shape=(u,)).copy() if u else np.zeros(0),
            "npairs": r.npairs,
        }
    finally:
        lib().oracle_free(C.byref(r))
    return out


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


def target_numerators(h, eri, norb, nalpha, nbeta, dets, coeffs, targets, ncore=0, ecore=0.0):
    """For each target determinant: (N_a, H_aa, is an input determinant, number of
    connected core determinants), evaluated one target at a time."""
    keep, hp, ep, n = _ham(h, eri)
    d, dp = _u(dets)
    c, cp = _d(coeffs)
    t, tp = _u(np.asarray(targets, dtype=np.uint64).reshape(-1, 2))
    m = t.shape[0]
    num = np.zeros(m)
    hd = np.zeros(m)
    inp = np.zeros(m, dtype=np.int32)
    nconn = np.zeros(m, dtype=np.int64)
    rc = lib().oracle_target_numerators(hp, ep, n, nalpha, nbeta, ecore, dp, cp, len(c), int(ncore), tp, m,
                                        num.ctypes.data_as(C.POINTER(C.c_double)),
                                        hd.ctypes.data_as(C.POINTER(C.c_double)),
                                        inp.ctypes.data_as(C.POINTER(C.c_int)),
                                        nconn.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc != 0:
        raise ValueError("invalid determinants")
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

def hamiltonian(h, eri, dets, ecore=0.0):
    """Dense H over a determinant set by the plain double loop (Sec. II.C):
    <D_i|H|D_j> where the two differ by at most a double excitation, else 0."""
    keep, hp, ep, n = _ham(h, eri)
    d, dp = _u(dets)
    nd = len(d)
    out = np.zeros((nd, nd))
    lib().oracle_hmat_dense(hp, ep, n, float(ecore), dp, nd, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


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
