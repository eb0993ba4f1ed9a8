"""Pins for the CPU oracle against what the mathematics fixes independently of it.

- Slater-Condon elements vs a brute-force second-quantised H (generic operator
  strings, no case analysis) on every determinant pair of tiny spaces;
- hermiticity and alpha/beta spin-flip symmetry at 12 orbitals;
- a Hamiltonian with only a diagonal one-body part has no couplings;
- the single/double target set vs a Hilbert-space scan with popcounts;
- N_a vs a dense matrix-vector product H[:, Q] C_Q (numpy);
- E_0: dense <C|H|C> = oracle double loop = sum C_i^2 H_ii + sum_{a in psi} C_a N_a;
- closed-form number of pairs;
- top-k vs numpy lexsort, tie handling, k beyond the candidate count;
- per-class pair counts vs a Python classification of every generated target;
- eps screening vs a filter over dense quantities.
"""
import numpy as np
import pytest

import asci_synth as syn
import sq_bruteforce as bf

TINY = [(4, 2, 2), (5, 2, 1), (5, 3, 2), (4, 1, 0), (4, 0, 2), (6, 3, 3), (5, 1, 1), (4, 4, 3)]


def popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


def strings(n, k):
    from itertools import combinations
    return np.array(sorted(sum(1 << p for p in c) for c in combinations(range(n), k)),
                    dtype=np.uint64)


@pytest.mark.parametrize("n,na,nb", TINY)
def test_helem_matches_second_quantised_h(oracle_lib, n, na, nb):
    rng = np.random.default_rng(100 + 7 * n + na + 3 * nb)
    h, eri = syn.integrals(n, rng)
    dets, H = bf.dense_h(h, eri, n, na, nb, ecore=0.25)
    O = np.array([[oracle_lib.helem(h, eri, a, i, 0.25) for i in dets] for a in dets])
    assert np.abs(H - O).max() < 1e-12
    D = np.array([oracle_lib.hdiag(h, eri, a, b, 0.25) for a, b in dets])
    assert np.abs(np.diag(H) - D).max() < 1e-12


def test_hermitian_and_spin_flip_at_12_orbitals(oracle_lib):
    rng = np.random.default_rng(5)
    n, na = 12, 5
    h, eri = syn.integrals(n, rng)
    dets = syn.uniform_dets(n, na, na, 60, rng)
    checked = 0
    for a in dets:
        for t in oracle_lib.sd_targets(n, a[0], a[1])[::37]:
            t = (int(t[0]), int(t[1]))
            x = oracle_lib.helem(h, eri, t, a)
            assert abs(x - oracle_lib.helem(h, eri, a, t)) <= 1e-13 * (1 + abs(x))
            flip = oracle_lib.helem(h, eri, (t[1], t[0]), (a[1], a[0]))
            assert abs(x - flip) <= 1e-13 * (1 + abs(x))
            checked += 1
    assert checked > 1000


def test_diagonal_one_body_hamiltonian_has_no_couplings(oracle_lib):
    n, na, nb = 8, 3, 2
    d = np.linspace(-1.0, 1.0, n)
    h, eri = np.diag(d), np.zeros((n,) * 4)
    a = (0b10110, 0b1001)
    for t in oracle_lib.sd_targets(n, *a):
        assert oracle_lib.helem(h, eri, (int(t[0]), int(t[1])), a) == 0.0
    assert oracle_lib.hdiag(h, eri, *a) == pytest.approx(d[[1, 2, 4]].sum() + d[[0, 3]].sum())


@pytest.mark.parametrize("n,na,nb", [(5, 2, 2), (6, 3, 1), (6, 0, 3), (7, 3, 3)])
def test_sd_targets_match_hilbert_scan(oracle_lib, n, na, nb):
    A, B = strings(n, na), strings(n, nb)
    rng = np.random.default_rng(n * 10 + na)
    for _ in range(5):
        a = int(A[rng.integers(len(A))])
        b = int(B[rng.integers(len(B))])
        deg = (popcount(A ^ np.uint64(a))[:, None] + popcount(B ^ np.uint64(b))[None, :]) // 2
        ia, ib = np.nonzero((deg >= 1) & (deg <= 2))
        scan = set(zip(A[ia].tolist(), B[ib].tolist()))
        got = oracle_lib.sd_targets(n, a, b)
        assert len(got) == len(scan) == oracle_lib.sd_count(n, na, nb)
        assert set(map(tuple, got.tolist())) == scan


def test_sd_count_closed_form(oracle_lib):
    from math import comb
    for n, na, nb in [(12, 4, 4), (20, 8, 8), (30, 12, 12), (40, 14, 14), (9, 0, 4), (7, 7, 3)]:
        va, vb = n - na, n - nb
        want = na * va + nb * vb + comb(na, 2) * comb(va, 2) + comb(nb, 2) * comb(vb, 2) + na * va * nb * vb
        assert oracle_lib.sd_count(n, na, nb) == want
    assert oracle_lib.sd_count(12, 4, 4) == 1424
    assert oracle_lib.sd_count(20, 8, 8) == 13104
    assert oracle_lib.sd_count(30, 12, 12) == 67284


def _tiny_case(n, na, nb, ndets, seed):
    rng = np.random.default_rng(seed)
    h, eri = syn.integrals(n, rng)
    first = syn.aufbau(n, na, nb)
    dets = [first] + syn.uniform_dets(n, na, nb, ndets - 1, rng, exclude=(first,))
    C = syn.coefficients(ndets, 3.0, rng)
    return h, eri, np.array(dets, dtype=np.uint64), C


@pytest.mark.parametrize("n,na,nb,ndets,ncore", [(5, 2, 2, 6, 0), (6, 3, 3, 12, 0), (6, 3, 3, 12, 5),
                                                 (6, 2, 1, 4, 0), (5, 3, 2, 9, 2), (6, 3, 3, 1, 0)])
def test_numerators_and_scores_equal_dense_algebra(oracle_lib, n, na, nb, ndets, ncore):
    h, eri, dets, C = _tiny_case(n, na, nb, ndets, seed=n * 100 + ndets + ncore)
    space, H = bf.dense_h(h, eri, n, na, nb)
    index = {d: i for i, d in enumerate(space)}
    psi_idx = [index[(int(a), int(b))] for a, b in dets]
    E0 = float(C @ H[np.ix_(psi_idx, psi_idx)] @ C)
    assert E0 == pytest.approx(oracle_lib.energy(h, eri, dets, C), rel=1e-12, abs=1e-12)

    if ncore and ncore < ndets:
        order = sorted(range(ndets), key=lambda i: (-abs(C[i]), i))[:ncore]
        Q = sorted(order)
    else:
        Q = list(range(ndets))
    assert list(oracle_lib.core_set(C, ncore)) == Q

    N_dense = H[:, [psi_idx[i] for i in Q]] @ C[Q]
    # candidates: connected to a core by a single or double, not in psi
    A = np.array([a for a, _ in space], dtype=np.uint64)
    B = np.array([b for _, b in space], dtype=np.uint64)
    conn = np.zeros(len(space), bool)
    for i in Q:
        deg = (popcount(A ^ dets[i, 0]) + popcount(B ^ dets[i, 1])) // 2
        conn |= (deg >= 1) & (deg <= 2)
    conn[psi_idx] = False
    want = [space[j] for j in np.nonzero(conn)[0]]

    r = oracle_lib.search_all(h, eri, n, na, nb, dets, C, E0, ncore=ncore)
    got = [tuple(x) for x in r["keys"].tolist()]
    assert got == sorted(want)
    for (a, b), num, hd, sc in zip(got, r["num"], r["hdiag"], r["score"]):
        j = index[(a, b)]
        assert num == pytest.approx(N_dense[j], abs=1e-12)
        assert hd == pytest.approx(H[j, j], abs=1e-12)
        assert sc == pytest.approx(N_dense[j] / (E0 - H[j, j]), rel=1e-10, abs=1e-12)
    assert r["npairs"] == len(Q) * oracle_lib.sd_count(n, na, nb)


def test_energy_triangle_cfg1(oracle_lib):
    """<C|H|C> by the double loop equals sum C_i^2 H_ii + sum_{a in psi} C_a N_a,
    where N_a are the search's numerators for the input determinants."""
    c = syn.workload("8e12o")
    h, eri, dets, C = c["h"], c["eri"], c["dets"], c["coeffs"]
    E0 = oracle_lib.energy(h, eri, dets, C)
    r = oracle_lib.search_all(h, eri, 12, 4, 4, dets, C, E0, keep_psi=True)
    pos = {tuple(k): j for j, k in enumerate(r["keys"].tolist())}
    tri = sum(C[i] ** 2 * oracle_lib.hdiag(h, eri, int(a), int(b)) for i, (a, b) in enumerate(dets))
    for i, (a, b) in enumerate(dets.tolist()):
        j = pos.get((a, b))
        if j is not None:
            tri += C[i] * r["num"][j]
    assert tri == pytest.approx(E0, rel=1e-12)


def test_energy_triangle_dense_tiny(oracle_lib):
    h, eri, dets, C = _tiny_case(6, 3, 3, 15, seed=11)
    space, H = bf.dense_h(h, eri, 6, 3, 3)
    index = {d: i for i, d in enumerate(space)}
    v = np.zeros(len(space))
    for (a, b), c in zip(dets.tolist(), C):
        v[index[(a, b)]] = c
    assert oracle_lib.energy(h, eri, dets, C) == pytest.approx(v @ H @ v, rel=1e-12)


def test_candidate_set_cfg1_equals_hilbert_scan(oracle_lib):
    c = syn.workload("8e12o")
    dets, C = c["dets"], c["coeffs"]
    A, B = strings(12, 4), strings(12, 4)
    pa = popcount(A[None, :] ^ dets[:, :1])  # ndets x |A|
    pb = popcount(B[None, :] ^ dets[:, 1:2])
    conn = np.zeros((len(A), len(B)), bool)
    for i in range(len(dets)):
        deg = (pa[i][:, None] + pb[i][None, :]) // 2
        conn |= (deg >= 1) & (deg <= 2)
    ia = np.searchsorted(A, dets[:, 0])
    ib = np.searchsorted(B, dets[:, 1])
    conn[ia, ib] = False
    want = np.stack(np.nonzero(conn), 1)
    r = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, dets, C, 0.0)
    got = np.stack([np.searchsorted(A, r["keys"][:, 0]), np.searchsorted(B, r["keys"][:, 1])], 1)
    assert len(got) == len(want)
    assert (got == want).all()
    assert r["npairs"] == 201 * 1424


def test_topk_equals_library_sort(oracle_lib):
    rng = np.random.default_rng(3)
    m = 5000
    keys = np.unique(rng.integers(0, 2**40, size=(m, 2), dtype=np.uint64), axis=0)
    m = len(keys)
    score = rng.normal(size=m)
    score[rng.integers(0, m, 400)] = 0.5      # ties on the value
    score[rng.integers(0, m, 300)] = -0.5     # ties on |value| with the other sign
    score[rng.integers(0, m, 50)] = 0.0
    score[7] = np.inf
    ordkey = np.abs(score).view(np.uint64)
    for k in (1, 17, 1000, 4000, m, m + 10):
        want = np.lexsort((keys[:, 1], keys[:, 0], ~ordkey))[:k]
        got = oracle_lib.topk_index(keys, score, k)
        assert (got == want).all()
    assert len(oracle_lib.topk_index(keys, score, 0)) == 0


def test_class_counts_match_classification(oracle_lib):
    n, na, nb = 9, 4, 3
    rng = np.random.default_rng(21)
    dets = [syn.aufbau(n, na, nb)] + syn.uniform_dets(n, na, nb, 30, rng, exclude=(syn.aufbau(n, na, nb),))
    dets = np.array(dets, dtype=np.uint64)
    C = syn.coefficients(len(dets), 5.0, rng)

    def top3(a):
        bits = [p for p in range(63, -1, -1) if (a >> p) & 1][:3]
        return sum(1 << p for p in bits)

    from collections import Counter
    want = Counter()
    for a, b in dets.tolist():
        for t in oracle_lib.sd_targets(n, a, b).tolist():
            want[top3(t[0])] += 1
    masks, counts = oracle_lib.class_counts(n, na, nb, dets, C)
    assert list(masks) == sorted(want)
    assert [want[m] for m in masks.tolist()] == list(counts)
    assert counts.sum() == len(dets) * oracle_lib.sd_count(n, na, nb)


def test_eps_screening_matches_dense_filter(oracle_lib):
    n, na, nb = 6, 3, 3
    h, eri, dets, C = _tiny_case(n, na, nb, 10, seed=9)
    space, H = bf.dense_h(h, eri, n, na, nb)
    index = {d: i for i, d in enumerate(space)}
    E0 = oracle_lib.energy(h, eri, dets, C)
    eps = 2e-3
    psi = {(int(a), int(b)) for a, b in dets}
    num = {}
    for i, (a, b) in enumerate(dets.tolist()):
        j = index[(a, b)]
        for t in oracle_lib.sd_targets(n, a, b).tolist():
            t = tuple(t)
            ti = index[t]
            v = H[ti, j] * C[i]
            if abs(v / (E0 - H[ti, ti])) > eps:
                num[t] = num.get(t, 0.0) + v
    want = sorted(t for t in num if t not in psi)
    r = oracle_lib.search_all(h, eri, n, na, nb, dets, C, E0, eps=eps)
    assert [tuple(k) for k in r["keys"].tolist()] == want
    assert np.allclose(r["num"], [num[t] for t in want], atol=1e-12)
    # the screen removes something here, and no pair survives a huge threshold
    assert len(want) < len(oracle_lib.search_all(h, eri, n, na, nb, dets, C, E0)["keys"])
    assert oracle_lib.search_all(h, eri, n, na, nb, dets, C, E0, eps=1e9)["keys"].shape[0] == 0


def test_invalid_inputs_rejected(oracle_lib):
    h, eri, dets, C = _tiny_case(5, 2, 2, 4, seed=1)
    bad = dets.copy()
    bad[1, 0] = 0b111  # three alpha electrons
    with pytest.raises(ValueError):
        oracle_lib.search_all(h, eri, 5, 2, 2, bad, C, 0.0)
    dup = dets.copy()
    dup[2] = dup[1]
    with pytest.raises(ValueError):
        oracle_lib.search_all(h, eri, 5, 2, 2, dup, C, 0.0)
    out_of_range = dets.copy()
    out_of_range[1, 1] = (1 << 5) | 1
    with pytest.raises(ValueError):
        oracle_lib.search_all(h, eri, 5, 2, 2, out_of_range, C, 0.0)
