"""Pins for the oracle's per-target numerators, its bucketed mode, and the score
tolerance that lets another evaluation order be compared with it.

- oracle_target_numerators (a plain scan over the cores for one target) equals
  the search's accumulation for every candidate and every input determinant of
  the (8e,12o) workload, with the connection count from popcounts;
- the bucketed, threaded search gives the flat search's result bit for bit;
- the tolerance covers a different grouping of the H_aa sum: the diagonal
  element regrouped by spin string (same-spin energies first, the
  opposite-spin Coulomb sum by beta orbital) lands inside it on every
  candidate, while the two orders differ in the last bits on many of them;
- the top-k bands: a candidate that is surely selected is in the oracle's
  top-k; a hand-built near tie is reported as ambiguous.
"""
import numpy as np
import pytest

import asci_synth as syn


def popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


def _cfg1():
    c = syn.workload("8e12o")
    return c


def test_target_numerators_equal_search_accumulation(oracle_lib):
    c = _cfg1()
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    allc = oracle_lib.search_all(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, keep_psi=True)
    targets = np.concatenate([allc["keys"], c["dets"]])
    num, hd, inp, nconn, nabs, habs = oracle_lib.target_numerators(c["h"], c["eri"], n, na, nb, c["dets"],
                                                                   c["coeffs"], targets, with_abs=True)
    m = len(allc["keys"])
    # every candidate (input determinants included): the same bits
    assert np.array_equal(num[:m], allc["num"])
    assert np.array_equal(hd[:m], allc["hdiag"])
    assert np.array_equal(nabs[:m], allc["num_abs"])
    assert np.array_equal(habs[:m], allc["hdiag_abs"])
    # connection counts from popcounts: cores at excitation degree 1 or 2
    dA = popcount(targets[:, 0][:, None] ^ c["dets"][:, 0][None, :])
    dB = popcount(targets[:, 1][:, None] ^ c["dets"][:, 1][None, :])
    deg = (dA + dB) // 2
    assert np.array_equal(nconn, ((deg >= 1) & (deg <= 2)).sum(axis=1))
    # the input-determinant flag
    psi = set(map(tuple, c["dets"].tolist()))
    assert np.array_equal(inp, np.array([tuple(t) in psi for t in targets.tolist()]))
    # an input determinant connected to no core has N_a = 0 and is absent from the candidates
    far = (nconn[m:] == 0)
    assert (num[m:][far] == 0.0).all()
    keyset = set(map(tuple, allc["keys"].tolist()))
    for t, f in zip(c["dets"].tolist(), far):
        assert (tuple(t) in keyset) == (not f)
    # with a core subset, only the chosen cores contribute
    num5, _, _, nconn5 = oracle_lib.target_numerators(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"],
                                                      targets[:500], ncore=5)
    core = oracle_lib.core_set(c["coeffs"], 5)
    assert np.array_equal(nconn5, ((deg[:500][:, core] >= 1) & (deg[:500][:, core] <= 2)).sum(axis=1))


BUCKET_CASES = [(6, 3, 3, 20, 0, 0.0), (9, 4, 2, 40, 0, 0.0), (8, 4, 3, 40, 11, 0.0), (12, 6, 6, 60, 0, 1e-3),
                (34, 3, 2, 12, 0, 0.0), (7, 0, 3, 6, 0, 0.0), (1, 1, 0, 1, 0, 0.0)]


@pytest.mark.parametrize("n,na,nb,nd,ncore,eps", BUCKET_CASES)
def test_bucketed_search_equals_flat(oracle_lib, n, na, nb, nd, ncore, eps):
    c = syn.make_case(n, na, nb, nd, 700 + n + nd, sampler="uniform", tau=max(nd / 5.0, 1.0))
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    want = oracle_lib.search_all(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, ncore=ncore, eps=eps)
    for nbk in (1, 5, 64):
        got, st = oracle_lib.search_buckets(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, ncore=ncore,
                                            eps=eps, nbuckets=nbk, threads=3)
        o = np.argsort(oracle_lib.key_codes(got["keys"]), kind="stable")
        assert st["candidates"] == len(want["keys"]) and st["npairs"] == want["npairs"]
        for f in ("keys", "num", "hdiag", "score", "num_abs", "hdiag_abs", "tol"):
            assert np.array_equal(got[f][o], want[f]), f


def test_bucketed_search_cfg1_keep_top_and_pt2(oracle_lib):
    c = _cfg1()
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    want = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0)
    full, st = oracle_lib.search_buckets(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0, nbuckets=16)
    o = np.argsort(oracle_lib.key_codes(full["keys"]), kind="stable")
    assert np.array_equal(full["keys"][o], want["keys"]) and np.array_equal(full["score"][o], want["score"])
    e, cnt, sabs = oracle_lib.pt2(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0, with_abs=True)
    assert st["candidates"] == cnt
    assert abs(st["pt2"] - e) <= 8 * 2.0 ** -53 * sabs
    assert st["pt2_abs"] == pytest.approx(sabs, rel=1e-12)
    # keep_top: each bucket's best; the union holds the global top-k
    k = 500
    top, st2 = oracle_lib.search_buckets(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0, nbuckets=16,
                                         keep_top=k)
    widx = oracle_lib.topk_index(want["keys"], want["score"], k)
    tidx = oracle_lib.topk_index(top["keys"], top["score"], k)
    assert np.array_equal(top["keys"][tidx], want["keys"][widx])
    # the largest |A| + tol among dropped candidates is below the k-th kept value
    assert 0.0 < st2["max_drop_upper"] <= abs(want["score"][widx[-1]]) + want["tol"][widx[-1]]


def _grouped_hdiag(h, eri, n, alpha, beta):
    """H_aa regrouped: ((E(alpha) + E(beta)) + sum_{q in beta} sum_{p in alpha} J_pq,
    E(s) = sum_p h_pp + sum_{p<q} (J_pq - K_pq); each candidate summed term by term."""
    e4 = eri.reshape(n, n, n, n)
    bit = lambda s, p: ((s >> np.uint64(p)) & np.uint64(1)).astype(bool)  # noqa: E731

    def spin(s):
        e = np.zeros(len(s))
        for p in range(n):
            e = np.where(bit(s, p), e + h[p, p], e)
        for p in range(n):
            for q in range(p + 1, n):
                e = np.where(bit(s, p) & bit(s, q), e + (e4[p, p, q, q] - e4[p, q, q, p]), e)
        return e

    cross = np.zeros(len(alpha))
    for q in range(n):
        cq = np.zeros(len(alpha))
        for p in range(n):
            cq = np.where(bit(alpha, p), cq + e4[p, p, q, q], cq)
        cross = np.where(bit(beta, q), cross + cq, cross)
    return (spin(alpha) + spin(beta)) + cross


@pytest.mark.parametrize("case", ["8e12o", (14, 6, 6, 300)])
def test_tolerance_covers_a_regrouped_diagonal(oracle_lib, case):
    if case == "8e12o":
        c = _cfg1()
    else:
        n, na, nb, nd = case
        c = syn.make_case(n, na, nb, nd, 91, sampler="level", tau=nd / 10.0)
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    r = oracle_lib.search_all(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0)
    hg = _grouped_hdiag(c["h"], c["eri"], n, r["keys"][:, 0], r["keys"][:, 1])
    ag = r["num"] / (E0 - hg)
    assert (hg != r["hdiag"]).mean() > 0.1          # the two orders round differently
    assert (np.abs(hg - r["hdiag"]) <= 1e-12 * np.maximum(1.0, np.abs(r["hdiag"]))).all()
    assert (np.abs(ag - r["score"]) <= r["tol"]).all()
    # the relaxed band exists (E0 inside the diagonal spectrum) and a 1e-12
    # relative bar alone would not cover the regrouping everywhere it applies
    rel = r["tol"] / np.abs(r["score"])
    assert (rel > 1.000001e-12).any()
    # tolerance formula: max(1e-12 |A|, 64 u (num_abs + |N| (|E0| + hdiag_abs) / |d|) / |d|)
    j = np.argmax(rel)
    d = abs(E0 - r["hdiag"][j])
    u = 2.0 ** -53
    want = max(1e-12 * abs(r["score"][j]),
               64 * u * (r["num_abs"][j] + abs(r["num"][j]) * (abs(E0) + r["hdiag_abs"][j]) / d) / d)
    assert r["tol"][j] == pytest.approx(want, rel=1e-14)


def test_magnitude_sums_bound_the_values(oracle_lib):
    """|N_a| <= num_abs and |H_aa| <= hdiag_abs; for a one-body diagonal
    Hamiltonian hdiag_abs is the sum of |h_pp| over occupied orbitals."""
    c = _cfg1()
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    r = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0)
    assert (np.abs(r["num"]) <= r["num_abs"] * (1 + 1e-15)).all()
    assert (np.abs(r["hdiag"]) <= r["hdiag_abs"] * (1 + 1e-15)).all()
    n = 6
    d = np.linspace(-1.0, 1.0, n)
    h, eri = np.diag(d), np.zeros((n,) * 4)
    dets = np.array([[0b111, 0b11], [0b1011, 0b101]], dtype=np.uint64)
    _, hd, _, _, _, habs = oracle_lib.target_numerators(h, eri, n, 3, 2, dets, np.array([0.8, 0.6]), dets,
                                                        ecore=-0.5, with_abs=True)
    assert habs[0] == pytest.approx(0.5 + np.abs(d[[0, 1, 2]]).sum() + np.abs(d[[0, 1]]).sum())
    assert hd[0] == pytest.approx(-0.5 + d[[0, 1, 2]].sum() + d[[0, 1]].sum())


def test_topk_bands_near_tie_and_sure_set(oracle_lib):
    keys = np.array([[1, 0], [2, 0], [3, 0], [4, 0], [5, 0]], np.uint64)
    sc = np.array([5.0, -4.0, 3.0, 3.0 + 1e-9, 1.0])
    tol = np.array([1e-12, 1e-12, 1e-8, 1e-8, 1e-12])
    sure, amb, ok = oracle_lib.topk_bands(keys, sc, tol, 3)
    assert sure.tolist() == [True, True, False, False, False]
    assert amb.tolist() == [False, False, True, True, False] and ok
    # a dropped candidate that could reach the k-th value is reported
    assert not oracle_lib.topk_bands(keys, sc, tol, 3, outside_upper=3.5)[2]
    c = _cfg1()
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    r = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0)
    for k in (1, 100, 2000, 10 ** 6):
        sure, amb, _ = oracle_lib.topk_bands(r["keys"], r["score"], r["tol"], k)
        idx = oracle_lib.topk_index(r["keys"], r["score"], k)
        chosen = np.zeros(len(sure), bool)
        chosen[idx] = True
        assert not (sure & ~chosen).any() and not (chosen & ~sure & ~amb).any()
