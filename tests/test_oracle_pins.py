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


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5, 6])
def test_class_counts_match_classification(oracle_lib, level):
    """Every pair lands in the class of its target's top-`level` alpha orbitals;
    the classes are disjoint and cover all pairs (Sec. II.B)."""
    n, na, nb = 9, 4, 3
    rng = np.random.default_rng(21)
    dets = [syn.aufbau(n, na, nb)] + syn.uniform_dets(n, na, nb, 30, rng, exclude=(syn.aufbau(n, na, nb),))
    dets = np.array(dets, dtype=np.uint64)
    C = syn.coefficients(len(dets), 5.0, rng)

    def top(a):
        bits = [p for p in range(63, -1, -1) if (a >> p) & 1][:level]
        return sum(1 << p for p in bits)

    from collections import Counter
    want = Counter()
    for a, b in dets.tolist():
        for t in oracle_lib.sd_targets(n, a, b).tolist():
            want[top(t[0])] += 1
    masks, counts = oracle_lib.class_counts(n, na, nb, dets, C, level=level)
    assert list(masks) == sorted(want)
    assert [want[m] for m in masks.tolist()] == list(counts)
    assert counts.sum() == len(dets) * oracle_lib.sd_count(n, na, nb)


def test_higher_level_classes_refine_lower_ones(oracle_lib):
    """A level-(L+1) class lies inside the level-L class of its top L orbitals,
    so its counts add up to the parent's (the split of a heavy class)."""
    c = syn.workload("8e12o")
    prev = None
    for level in range(1, 7):
        masks, counts = oracle_lib.class_counts(12, 4, 4, c["dets"], c["coeffs"], level=level)
        assert (np.diff(masks.astype(np.float64)) > 0).all()
        if prev is not None:
            pm, pc = prev
            parent = {}
            for m, k in zip(masks.tolist(), counts.tolist()):
                bits = [p for p in range(63, -1, -1) if (m >> p) & 1][:level - 1]
                key = sum(1 << p for p in bits)
                parent[key] = parent.get(key, 0) + k
            assert parent == dict(zip(pm.tolist(), pc.tolist()))
        prev = (masks, counts)
    # level >= n_alpha: one class per alpha string, the strings targets reach
    from math import comb

    assert len(prev[0]) <= comb(12, 4)


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


@pytest.mark.parametrize("n,na,nb,ndets", [(5, 2, 2, 6), (6, 3, 3, 15), (6, 2, 3, 10)])
def test_pt2_equals_dense_epstein_nesbet(oracle_lib, n, na, nb, ndets):
    """E_PT2 = sum_{a not in psi} (H C)_a^2 / (E0 - H_aa), from the dense H."""
    h, eri, dets, C = _tiny_case(n, na, nb, ndets, seed=70 + n + ndets)
    space, H = bf.dense_h(h, eri, n, na, nb)
    index = {d: i for i, d in enumerate(space)}
    psi = [index[(int(a), int(b))] for a, b in dets]
    v = np.zeros(len(space))
    v[psi] = C
    E0 = float(v @ H @ v)
    sigma = H @ v
    mask = np.ones(len(space), bool)
    mask[psi] = False
    conn = np.abs(H[:, psi]).sum(axis=1) > 0
    sel = mask & conn
    want = float(np.sum(sigma[sel] ** 2 / (E0 - np.diag(H)[sel])))
    got, cnt = oracle_lib.pt2(h, eri, n, na, nb, dets, C, E0)
    assert got == pytest.approx(want, rel=1e-11, abs=1e-13)
    assert cnt == len(oracle_lib.search_all(h, eri, n, na, nb, dets, C, E0)["keys"])


def test_pt2_compensated_sum_is_the_exact_sum(oracle_lib):
    """The oracle's compensated PT2 sum equals the correctly rounded sum of its
    terms (math.fsum) to within 2u|E|, and S is the sum of their magnitudes."""
    import math

    c = syn.workload("8e12o")
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    r = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0)
    terms = r["num"] * r["score"]
    e, cnt, sabs = oracle_lib.pt2(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0, with_abs=True)
    exact = math.fsum(terms.tolist())
    assert cnt == len(terms)
    assert abs(e - exact) <= 2.3e-16 * abs(exact)
    assert sabs == pytest.approx(math.fsum(np.abs(terms).tolist()), rel=1e-12)


@pytest.mark.parametrize("npe", [1, 3, 8, 64])
def test_balance_invariants(oracle_lib, npe):
    """Alg. 3 (greedy list scheduling): work is conserved, the first npe
    non-empty classes land on distinct elements, and the largest load obeys
    Graham's bound max <= total/npe + max class (a missing load update, an
    arg-max or a dropped class breaks one of these)."""
    rng = np.random.default_rng(npe)
    counts = rng.integers(0, 1000, 300) * (rng.random(300) < 0.8)
    counts[5] = 50_000  # one heavy class
    owner, work = oracle_lib.balance(counts, npe)
    nz = counts > 0
    assert (owner[~nz] == -1).all() and (owner[nz] >= 0).all() and (owner < npe).all()
    assert work.sum() == counts.sum()
    assert (np.bincount(owner[nz], weights=counts[nz], minlength=npe) == work).all()
    first = owner[nz][:npe]
    assert len(set(first.tolist())) == len(first)
    assert work.max() <= counts.sum() / npe + counts.max()
    # the heavy class is indivisible: with many elements it sets the maximum
    if npe >= 64:
        assert work.max() == 50_000
