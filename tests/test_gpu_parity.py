"""GPU parity: the HIP search (through the C ABI) against the CPU oracle.

Bar: candidate sets and selected keys bit-exact (a selection may differ only
among candidates the oracle's tolerance bands mark ambiguous); N_a within
max(1e-12 |N_a|, 64 u num_abs) and A_a within the oracle's per-candidate
tolerance max(1e-12 |A_a|, 64 u |A_a| (kappa_num + kappa_den)).  The oracle
adds the diagonal element in the textbook order, the kernels group it by spin
string, so the two differ in the last bits on most candidates; the tests do
not rely on a shared rounding order.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import asci_synth as syn
from gpu_util import (assert_candidates, assert_head, assert_selection_order, assert_topk, assert_topk_golden,
                      host, locate, num_tol, to_dev)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def asci():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05688_amd as pkg

    return pkg


def _case(n, na, nb, ndets, seed, sampler="uniform"):
    return syn.make_case(n, na, nb, ndets, seed, sampler=sampler, tau=max(ndets / 5.0, 1.0))


def _golden(name):
    with open(os.path.join(GOLDEN, "search_%s.json" % name)) as f:
        return json.load(f)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _all_parity(asci, oracle_lib, c, E0, ncore=0, pair_buffer_bytes=0, eps=0.0, constraint_level=3, split_pairs=0):
    d = to_dev(c)
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    print("case n=%d na=%d nb=%d ndets=%d seed=%s ncore=%d buf=%d eps=%g level=%d split=%d" % (
        n, na, nb, len(c["coeffs"]), c["seed"], ncore, pair_buffer_bytes, eps, constraint_level, split_pairs),
        flush=True)
    keys, num, score = asci.candidates(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0, ncore=ncore,
                                       pair_buffer_bytes=pair_buffer_bytes, eps=eps,
                                       constraint_level=constraint_level, split_pairs=split_pairs)
    want = oracle_lib.search_all(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, ncore=ncore, eps=eps)
    exact, relaxed = assert_candidates(host(keys), host(num), host(score), want)
    print("  %d candidates, %d scores bit-identical, %d in the relaxed band" % (len(want["keys"]), exact, relaxed))
    return want


TINY = [
    (4, 2, 2, 5, 0), (5, 2, 1, 7, 0), (6, 3, 3, 20, 0), (6, 3, 3, 20, 6), (7, 1, 2, 10, 0),
    (7, 0, 3, 6, 0), (6, 6, 2, 4, 0), (8, 4, 3, 40, 0), (9, 5, 4, 60, 17), (10, 3, 3, 90, 0),
    (12, 6, 6, 150, 0), (1, 1, 0, 1, 0), (3, 1, 1, 9, 0),
]


@pytest.mark.parametrize("n,na,nb,ndets,ncore", TINY)
def test_candidates_tiny(asci, oracle_lib, n, na, nb, ndets, ncore):
    c = _case(n, na, nb, ndets, seed=1000 + n * 31 + ndets)
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    _all_parity(asci, oracle_lib, c, E0, ncore=ncore)


@pytest.mark.parametrize("n,na,nb,ndets", [(33, 3, 2, 12), (40, 4, 4, 8), (36, 2, 3, 20), (50, 2, 2, 6),
                                             (64, 2, 2, 5), (32, 3, 3, 10)])
def test_candidates_two_word_keys(asci, oracle_lib, n, na, nb, ndets):
    c = _case(n, na, nb, ndets, seed=77 + n)
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    _all_parity(asci, oracle_lib, c, E0)


@pytest.mark.parametrize("n,na,nb,ndets,buf", [(20, 12, 6, 40, 1 << 18), (34, 12, 4, 12, 1 << 19)])
def test_many_hole_pairs_in_small_batches(asci, oracle_lib, n, na, nb, ndets, buf):
    """More alpha hole pairs than a wavefront has lanes (66), the alpha-alpha
    doubles of each core spread over many class batches: the in-batch
    particle-pair ranges and their enumeration order, one- and two-word keys."""
    c = _case(n, na, nb, ndets, seed=4100 + n)
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    _all_parity(asci, oracle_lib, c, E0, pair_buffer_bytes=buf)
    d = to_dev(c)
    k1, s1 = asci.search(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0, 500, pair_buffer_bytes=buf)
    k2, s2 = asci.search(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0, 500)
    assert (host(k1) == host(k2)).all() and (host(s1) == host(s2)).all()


def test_candidates_8e12o(asci, oracle_lib):
    c = syn.workload("8e12o")
    g = _golden("8e12o")
    E0 = float.fromhex(g["E0"])
    want = _all_parity(asci, oracle_lib, c, E0)
    assert len(want["keys"]) == g["ncandidates"]


@pytest.mark.parametrize("eps", [1e-10, 1e-4, 3e-3])
def test_pair_threshold_eps(asci, oracle_lib, eps):
    """Alg. 2's threshold: a pair joins the sum only if its partial score
    exceeds eps in magnitude (1e-10 is the value the paper's runs used)."""
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    want = _all_parity(asci, oracle_lib, c, E0, eps=eps)
    if eps >= 1e-4:
        assert len(want["keys"]) < _golden("8e12o")["ncandidates"]
    d = to_dev(c)
    gk, gs = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, 700, eps=eps)
    assert_topk(host(gk), host(gs), want, 700)


def test_pair_threshold_eps_tiny(asci, oracle_lib):
    for (n, na, nb, nd) in [(6, 3, 3, 12), (8, 4, 2, 30)]:
        c = _case(n, na, nb, nd, seed=300 + n)
        E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
        _all_parity(asci, oracle_lib, c, E0, eps=1e-3)


@pytest.mark.parametrize("buf", [1 << 16, 3 << 18, 1 << 21])
def test_small_pair_buffer_gives_same_result(asci, oracle_lib, buf):
    """A forced small pair buffer splits the classes into many batches."""
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    _all_parity(asci, oracle_lib, c, E0, pair_buffer_bytes=buf)
    d = to_dev(c)
    k1, s1 = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, 2000, pair_buffer_bytes=buf)
    k2, s2 = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, 2000)
    assert (host(k1) == host(k2)).all() and (host(s1) == host(s2)).all()


@pytest.mark.parametrize("k", [1, 7, 2000, 50_000, 10**7])
def test_topk_8e12o(asci, oracle_lib, k):
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    d = to_dev(c)
    gk, gs = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, k)
    want = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0)
    assert_topk(host(gk), host(gs), want, k)


def test_topk_8e12o_matches_golden_bands(asci):
    c = syn.workload("8e12o")
    g = _golden("8e12o")
    d = to_dev(c)
    gk, gs = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], float.fromhex(g["E0"]), c["k"])
    assert_topk_golden(host(gk), host(gs), g)


@pytest.mark.parametrize("ncore", [1, 50, 200])
def test_topk_core_subset(asci, oracle_lib, ncore):
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    d = to_dev(c)
    gk, gs = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, 500, ncore=ncore)
    want = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0, ncore=ncore)
    assert_topk(host(gk), host(gs), want, 500)


def test_host_entry_point_matches_device(asci, oracle_lib):
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    hk, hs = asci.search_host(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0, 1000)
    want = oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0)
    assert_topk(hk, hs, want, 1000)


def test_class_counts(asci, oracle_lib):
    for c in (syn.workload("8e12o"), _case(9, 4, 2, 40, 5), _case(7, 2, 3, 15, 6), _case(6, 0, 2, 5, 7),
              _case(34, 3, 3, 10, 8)):
        d = to_dev(c)
        gm, gc = asci.class_counts(c["norb"], c["nalpha"], c["nbeta"], d["dets"], d["coeffs"])
        wm, wc = oracle_lib.class_counts(c["norb"], c["nalpha"], c["nbeta"], c["dets"], c["coeffs"])
        assert (gm == wm).all() and (gc == wc).all()
        gm, gc = asci.class_counts(c["norb"], c["nalpha"], c["nbeta"], d["dets"], d["coeffs"], ncore=3)
        wm, wc = oracle_lib.class_counts(c["norb"], c["nalpha"], c["nbeta"], c["dets"], c["coeffs"], ncore=3)
        assert (gm == wm).all() and (gc == wc).all()


def test_class_counts_sum_to_closed_form_16e20o(asci, oracle_lib):
    c = syn.workload("16e20o")
    d = to_dev(c)
    gm, gc = asci.class_counts(20, 8, 8, d["dets"], d["coeffs"])
    assert len(gm) == 455  # C(20 - 8 + 3, 3) triplet classes, all non-empty here
    assert int(gc.sum()) == _golden("16e20o")["pairs_closed_form"] == 10_000 * oracle_lib.sd_count(20, 8, 8)


@pytest.mark.parametrize("name", ["8e12o", "16e20o"])
def test_energy(asci, oracle_lib, name):
    c = syn.workload(name)
    d = to_dev(c)
    e = asci.energy(d["h"], d["eri"], c["norb"], c["nalpha"], c["nbeta"], d["dets"], d["coeffs"])
    # the GPU groups the diagonal differently: E0 agrees to a few ulps of sum |C_i C_j H_ij| (~|E0| here)
    assert e == pytest.approx(float.fromhex(_golden(name)["E0"]), rel=1e-12)


def test_deterministic_and_permutation_invariant(asci, oracle_lib):
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    d = to_dev(c)
    k1, s1 = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, 2000)
    k2, s2 = asci.search(d["h"], d["eri"], 12, 4, 4, d["dets"], d["coeffs"], E0, 2000)
    assert (host(k1) == host(k2)).all() and (host(s1) == host(s2)).all()
    perm = np.random.default_rng(0).permutation(len(c["coeffs"]))
    cp = dict(c, dets=c["dets"][perm], coeffs=c["coeffs"][perm])
    dp = to_dev(cp)
    k3, s3 = asci.search(dp["h"], dp["eri"], 12, 4, 4, dp["dets"], dp["coeffs"], E0, 2000)
    want = oracle_lib.search_all(cp["h"], cp["eri"], 12, 4, 4, cp["dets"], cp["coeffs"], E0)
    assert_topk(host(k3), host(s3), want, 2000)
    # a permutation of the inputs changes the core order (hence the summation
    # order of N_a) but not the selection outside near ties
    assert_topk(host(k1), host(s1), oracle_lib.search_all(c["h"], c["eri"], 12, 4, 4, c["dets"], c["coeffs"], E0),
                2000)


def test_invalid_inputs(asci):
    import torch

    c = _case(6, 3, 3, 10, 3)
    d = to_dev(c)
    bad = d["dets"].clone().view(torch.int64)
    bad[2, 0] = 0b1111  # four alpha electrons
    with pytest.raises(asci.AsciError) as e:
        asci.search(d["h"], d["eri"], 6, 3, 3, bad.view(torch.uint64), d["coeffs"], 0.0, 10)
    assert e.value.code == asci.ASCI_EINVAL
    dup = d["dets"].clone().view(torch.int64)
    dup[3] = dup[1]
    with pytest.raises(asci.AsciError):
        asci.search(d["h"], d["eri"], 6, 3, 3, dup.view(torch.uint64), d["coeffs"], 0.0, 10)
    high = d["dets"].clone().view(torch.int64)
    high[1, 1] = (1 << 6) | 0b11
    with pytest.raises(asci.AsciError):
        asci.search(d["h"], d["eri"], 6, 3, 3, high.view(torch.uint64), d["coeffs"], 0.0, 10)
    with pytest.raises(asci.AsciError):
        asci.search(d["h"], d["eri"], 6, 3, 3, d["dets"], d["coeffs"], 0.0, 0)
    with pytest.raises(asci.AsciError):
        asci.search(d["h"], d["eri"], 65, 3, 3, d["dets"], d["coeffs"], 0.0, 10)
    with pytest.raises(asci.AsciError):
        asci.search(d["h"], d["eri"], 6, 3, 3, d["dets"], d["coeffs"], 0.0, 10, eps=-1.0)
    # integrals without the 8-fold symmetry: one entry changed alone, then the
    # same change made to all eight equal entries (accepted again)
    asym = d["eri"].clone()
    asym.view(-1)[((0 * 6 + 2) * 6 + 1) * 6 + 4] += 1e-3
    with pytest.raises(asci.AsciError) as e:
        asci.search(d["h"], asym, 6, 3, 3, d["dets"], d["coeffs"], 0.0, 10)
    assert e.value.code == asci.ASCI_EINVAL and "symmetric" in str(e.value)
    sym = d["eri"].clone().view(6, 6, 6, 6)
    for p, q, r, t in {(0, 2, 1, 4), (2, 0, 1, 4), (0, 2, 4, 1), (2, 0, 4, 1),
                       (1, 4, 0, 2), (4, 1, 0, 2), (1, 4, 2, 0), (4, 1, 2, 0)}:
        sym[p, q, r, t] += 1e-3
    k_, s_ = asci.search(d["h"], sym.reshape(-1), 6, 3, 3, d["dets"], d["coeffs"], 0.0, 10)
    assert len(k_) == 10


def _sampled_checks(oracle_lib, c, E0, gk, gs, ncheck=1500, seed=0):
    """Check returned candidates one at a time against the oracle: connected to
    the core set, not an input determinant, A_a = N_a / (E0 - H_aa) within the
    candidate's tolerance.  Returns how many of the checked scores are bit-identical."""
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    rng = np.random.default_rng(seed)
    m = len(gk)
    idx = np.unique(np.concatenate([np.arange(min(m, ncheck // 3)),
                                    rng.integers(0, m, ncheck - ncheck // 3), [m - 1]]))
    num, hd, inp, nconn, nabs, habs = oracle_lib.target_numerators(c["h"], c["eri"], n, na, nb, c["dets"],
                                                                   c["coeffs"], gk[idx], with_abs=True)
    assert not inp.any()
    assert (nconn >= 1).all()
    want = num / (E0 - hd)
    tol = np.array([oracle_lib.score_tol(x, xa, y, ya, E0) for x, xa, y, ya in zip(num, nabs, hd, habs)])
    assert (np.abs(gs[idx] - want) <= tol).all()
    return int((gs[idx] == want).sum())


def _oracle_full(oracle_lib, c, E0, **kw):
    """Every candidate from the oracle's bucketed mode, ascending key order."""
    r, st = oracle_lib.search_buckets(c["h"], c["eri"], c["norb"], c["nalpha"], c["nbeta"], c["dets"], c["coeffs"],
                                      E0, nbuckets=64, **kw)
    o = np.lexsort((r["keys"][:, 1], r["keys"][:, 0]))
    return {f: (v[o] if isinstance(v, np.ndarray) else v) for f, v in r.items()}, st


def test_full_size_16e20o(asci, oracle_lib):
    """The (16e,20o) workload at full size, element by element: every one of
    the 3.7e7 candidates against the oracle (run here, threaded over target
    buckets), the candidate keys against the stored hash, and the top 10^5
    against the stored bands."""
    c = syn.workload("16e20o")
    g = _golden("16e20o")
    E0 = float.fromhex(g["E0"])
    d = to_dev(c)
    keys, num, score = asci.candidates(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], E0)
    hk, hn, hs = host(keys), host(num), host(score)
    del keys, num, score
    assert len(hk) == g["ncandidates"]
    assert _sha(hk) == g["cand_keys_sha256"]
    want, st = _oracle_full(oracle_lib, c, E0)
    assert st["npairs"] == g["npairs"]
    exact, relaxed = assert_candidates(hk, hn, hs, want)
    print("16e20o: %d candidates, %d scores bit-identical, %d in the relaxed band" % (len(hk), exact, relaxed))
    del hk, hn, hs
    gk, gs = asci.search(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], E0, c["k"])
    gk, gs = host(gk), host(gs)
    assert_topk_golden(gk, gs, g)
    assert_topk(gk, gs, want, c["k"])


SPIN_TABLE_CASES = [(12, 6, 6, 150, 41), (9, 5, 2, 60, 42), (34, 3, 2, 12, 43), (14, 7, 1, 80, 44), (6, 0, 3, 6, 45)]


def test_spin_tables_change_no_bit(asci, oracle_lib):
    """E(alpha) and E(beta) looked up from the rank-indexed tables or evaluated
    directly give the same bits (one summation order); both match the oracle."""
    ctx = asci.Context.get(0)
    try:
        for n, na, nb, nd, seed in SPIN_TABLE_CASES:
            c = _case(n, na, nb, nd, seed=seed, sampler="level")
            E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
            d = to_dev(c)
            got = []
            for flag in (1, 0):
                ctx.set_param("spin_tables", flag)
                _all_parity(asci, oracle_lib, c, E0)
                got.append([host(t) for t in asci.candidates(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"],
                                                             E0)])
            for a, b in zip(*got):
                assert a.shape == b.shape and a.tobytes() == b.tobytes()
        # the full-size workload: direct evaluation gives the tables' bits
        c = syn.workload("16e20o")
        g = _golden("16e20o")
        d = to_dev(c)
        got = []
        for flag in (1, 0):
            ctx.set_param("spin_tables", flag)
            keys, num, score = asci.candidates(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"],
                                               float.fromhex(g["E0"]))
            assert _sha(host(keys)) == g["cand_keys_sha256"]
            got.append((_sha(host(num)), _sha(host(score))))
            del keys, num, score
        assert got[0] == got[1]
    finally:
        ctx.set_param("spin_tables", 1)


LEVEL_CASES = [(12, 4, 4, 150, 31), (16, 6, 6, 300, 32), (34, 3, 2, 12, 33), (9, 2, 3, 30, 34), (14, 7, 1, 80, 35)]


@pytest.mark.parametrize("level,split", [(1, 0), (2, 0), (4, 0), (5, 0), (6, 0), (6, 300), (5, 5000), (4, 1)])
def test_constraint_levels_same_candidates(asci, oracle_lib, level, split):
    """The classes only partition the targets (Sec. II.B): any level, uniform or
    with only the heavy classes split, gives the oracle's candidates exactly."""
    for n, na, nb, nd, seed in LEVEL_CASES:
        c = _case(n, na, nb, nd, seed=seed, sampler="level")
        E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
        _all_parity(asci, oracle_lib, c, E0, constraint_level=level, split_pairs=split)


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5, 6])
def test_class_counts_by_level(asci, oracle_lib, level):
    """Pair counts of the level-L classes (closed form on the GPU) equal the
    oracle's enumeration."""
    for n, na, nb, nd, seed in LEVEL_CASES[:3]:
        c = _case(n, na, nb, nd, seed=seed, sampler="level")
        d = to_dev(c)
        gm, gc = asci.class_counts(n, na, nb, d["dets"], d["coeffs"], constraint_level=level)
        wm, wc = oracle_lib.class_counts(n, na, nb, c["dets"], c["coeffs"], level=level)
        assert (gm == wm).all() and (gc == wc).all()


def test_heavy_classes_split_adaptively(asci, oracle_lib):
    """split_pairs > 0: classes start as triplets and only the heavy ones are
    refined, up to the maximum level; every final class has the oracle's count
    at its own level, and a class left unsplit below the maximum is light."""
    n, na, nb, nd, seed = LEVEL_CASES[1]
    c = _case(n, na, nb, nd, seed=seed, sampler="level")
    d = to_dev(c)
    split = 4000
    gm, gc = asci.class_counts(n, na, nb, d["dets"], d["coeffs"], constraint_level=6, split_pairs=split)
    assert gc.sum() == nd * oracle_lib.sd_count(n, na, nb)
    assert (np.diff(gm.astype(np.float64)) > 0).all()
    want = {lv: dict(zip(*[a.tolist() for a in oracle_lib.class_counts(n, na, nb, c["dets"], c["coeffs"],
                                                                      level=lv)])) for lv in range(3, 7)}
    levels = set()
    for m, k in zip(gm.tolist(), gc.tolist()):
        lv = bin(m).count("1")
        levels.add(lv)
        assert want[lv][m] == k
        if lv < 6:
            assert k <= split
    assert levels == {3, 4, 5, 6}
    # refining never makes the partition coarser (the paper's Fig. 3 trend); the
    # heaviest class here is a single alpha string, which no constraint divides
    st3 = asci.class_skew(asci.class_counts(n, na, nb, d["dets"], d["coeffs"])[1], npes=(64,))
    sta = asci.class_skew(gc, npes=(64,))
    assert sta["classes"] > st3["classes"]
    assert sta["largest_share"] <= st3["largest_share"]
    assert sta["imbalance"][64] <= st3["imbalance"][64]


def test_class_larger_than_pair_buffer_is_split(asci, oracle_lib):
    """A triplet class bigger than the whole pair buffer is split further
    automatically; the candidates do not change."""
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    m, k = oracle_lib.class_counts(12, 4, 4, c["dets"], c["coeffs"])
    big = int(k.max())
    _all_parity(asci, oracle_lib, c, E0, pair_buffer_bytes=32 * (big // 3))


@pytest.mark.parametrize("level,split", [(6, 0), (6, 1 << 18)])
def test_full_size_16e20o_levels(asci, level, split):
    """The (16e,20o) workload with hextuplet classes (18,564 of them, about ten
    class batches) and with only the heavy triplets split: the oracle's
    candidate keys, and numerators and scores bit-identical to the triplet
    search (the classes only partition the work)."""
    c = syn.workload("16e20o")
    g = _golden("16e20o")
    d = to_dev(c)
    E0 = float.fromhex(g["E0"])
    ref = [_sha(host(t)) for t in asci.candidates(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], E0)]
    keys, num, score = asci.candidates(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], E0,
                                       constraint_level=level, split_pairs=split)
    assert _sha(host(keys)) == g["cand_keys_sha256"] == ref[0]
    assert _sha(host(num)) == ref[1]
    assert _sha(host(score)) == ref[2]


def test_full_size_16e20o_multi_batch(asci, oracle_lib):
    """The bench workload split into about five class batches (a forced pair
    buffer of 1 GiB): the top-k must not change."""
    c = syn.workload("16e20o")
    g = _golden("16e20o")
    d = to_dev(c)
    gk, gs = asci.search(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], float.fromhex(g["E0"]), c["k"],
                         pair_buffer_bytes=1 << 30)
    gk, gs = host(gk), host(gs)
    assert_topk_golden(gk, gs, g)
    k1, s1 = asci.search(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], float.fromhex(g["E0"]), c["k"])
    assert (host(k1) == gk).all() and (host(s1) == gs).all()


def test_full_size_24e30o(asci, oracle_lib):
    """The Cr2-shaped (24e,30o) workload: 6.7e9 pairs in class batches.  The top
    10^6 against the oracle's stored bands (every surely selected key, nothing
    surely out, the k-th |A| inside its bounds, the head), returned entries
    checked one at a time against the oracle, and the number of candidates and
    the PT2 sum over all of them against the stored totals."""
    c = syn.workload("24e30o")
    g = _golden("24e30o")
    E0 = float.fromhex(g["E0"])
    d = to_dev(c)
    gk, gs = asci.search(d["h"], d["eri"], 30, 12, 12, d["dets"], d["coeffs"], E0, c["k"])
    gk, gs = host(gk), host(gs)
    assert len(gk) == c["k"]
    assert_topk_golden(gk, gs, g)
    same = _sampled_checks(oracle_lib, c, E0, gk, gs, ncheck=900, seed=3)
    print("24e30o: %d of ~900 sampled scores bit-identical" % same)
    e, cnt = asci.pt2(d["h"], d["eri"], 30, 12, 12, d["dets"], d["coeffs"], E0)
    assert cnt == g["ncandidates"]
    want = float.fromhex(g["pt2"])
    assert abs(e - want) <= pt2_tol(want, float.fromhex(g["pt2_abs_terms"]), float.fromhex(g["pt2_term_tol"]))


def test_two_word_keys_batch_sized(asci, oracle_lib):
    """Keys of two words at a batch-like size: (16e,36o), 150 determinants,
    1.1e7 pairs, every candidate compared with the oracle, then the top 10^4."""
    c = _case(36, 8, 8, 150, seed=3608, sampler="level")
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    assert len(c["coeffs"]) * oracle_lib.sd_count(36, 8, 8) >= 10 ** 7
    d = to_dev(c)
    keys, num, score = asci.candidates(d["h"], d["eri"], 36, 8, 8, d["dets"], d["coeffs"], E0)
    want, st = _oracle_full(oracle_lib, c, E0)
    exact, relaxed = assert_candidates(host(keys), host(num), host(score), want)
    print("36 orbitals: %d candidates, %d bit-identical, %d relaxed" % (len(want["keys"]), exact, relaxed))
    gk, gs = asci.search(d["h"], d["eri"], 36, 8, 8, d["dets"], d["coeffs"], E0, 10_000)
    assert_topk(host(gk), host(gs), want, 10_000)


def test_one_target_from_more_cores_than_fit_in_lds(asci, oracle_lib):
    """psi = every single and double of one determinant t (7875 of them at
    (10e,20o)): t collects 7875 contributions, more than one LDS bucket holds,
    and psi is dense in the key ranges around t."""
    n, na, nb = 20, 5, 5
    rng = np.random.default_rng(8)
    h, eri = syn.integrals(n, rng)
    t = (0b1011000100001 << 2, 0b110000011001)
    t = (int(t[0]) & ((1 << n) - 1), int(t[1]))
    assert bin(t[0]).count("1") == na and bin(t[1]).count("1") == nb
    dets = oracle_lib.sd_targets(n, t[0], t[1])
    assert len(dets) == 7875
    C = syn.coefficients(len(dets), 2000.0, rng)
    c = {"norb": n, "nalpha": na, "nbeta": nb, "h": h, "eri": eri, "dets": dets, "coeffs": C, "seed": 8}
    E0 = oracle_lib.energy(h, eri, dets[:500], C[:500])
    d = to_dev(c)
    keys, num, score = asci.candidates(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0)
    hk, hn, hs = host(keys), host(num), host(score)
    at = np.nonzero((hk[:, 0] == t[0]) & (hk[:, 1] == t[1]))[0]
    assert len(at) == 1
    wn, wh, inp, nconn, wna, wha = oracle_lib.target_numerators(h, eri, n, na, nb, dets, C,
                                                                np.array([t], dtype=np.uint64), with_abs=True)
    assert nconn[0] == 7875 and not inp[0]
    assert abs(hn[at][0] - wn[0]) <= num_tol(wn, wna)[0]
    assert abs(hs[at][0] - wn[0] / (E0 - wh[0])) <= oracle_lib.score_tol(wn[0], wna[0], wh[0], wha[0], E0)
    # sampled candidates, and no input determinant among them
    rng2 = np.random.default_rng(1)
    idx = rng2.integers(0, len(hk), 400)
    wn2, wh2, inp2, nconn2, wna2, _ = oracle_lib.target_numerators(h, eri, n, na, nb, dets, C, hk[idx],
                                                                   with_abs=True)
    assert not inp2.any() and (nconn2 >= 1).all()
    assert (np.abs(hn[idx] - wn2) <= num_tol(wn2, wna2)).all()
    gk, gs = asci.search(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0, 1000)
    assert_selection_order(host(gk), host(gs))


def _pt2_case(asci, oracle_lib, c, E0, **kw):
    d = to_dev(c)
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    e, cnt = asci.pt2(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0, **kw)
    okw = {k: v for k, v in kw.items() if k != "pair_buffer_bytes"}
    _, st = oracle_lib.search_buckets(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, nbuckets=8, **okw)
    assert cnt == st["candidates"]
    tol = pt2_tol(st["pt2"], st["pt2_abs"], st["pt2_tol"])
    assert abs(e - st["pt2"]) <= tol
    return e, tol


def pt2_tol(exact, sabs, term_tol):
    """The GPU adds the terms N_a * A_a in segments of at most 4096 candidates,
    then adds the segment sums (a few per thread, then a 1024-wide tree, then the
    batches), so its summation error is at most about (4096 + 2048) u S with S
    the sum of |terms| (Higham, ch. 4); the oracle's compensated sums are exact
    to 4u S; and each term may differ from the oracle's by its own tolerance
    (term_tol: sum of |N_a| tol_a + |A_a| tol(N_a))."""
    u = 2.0 ** -53
    return 6144 * u * sabs + 4 * u * sabs + term_tol


def test_pt2_energy(asci, oracle_lib):
    """E_PT2 = sum_a N_a^2 / (E0 - H_aa): the candidates are exact, every term
    within its tolerance, only the order of the additions differs."""
    c = syn.workload("8e12o")
    E0 = float.fromhex(_golden("8e12o")["E0"])
    e1, tol = _pt2_case(asci, oracle_lib, c, E0)
    e2, _ = _pt2_case(asci, oracle_lib, c, E0, pair_buffer_bytes=1 << 18)
    assert abs(e1 - e2) <= 2 * tol
    _pt2_case(asci, oracle_lib, c, E0, eps=1e-4)
    _pt2_case(asci, oracle_lib, c, E0, ncore=40)
    for (n, na, nb, nd) in [(6, 3, 3, 12), (9, 4, 2, 30), (34, 3, 2, 10)]:
        cc = _case(n, na, nb, nd, seed=900 + n)
        E0 = oracle_lib.energy(cc["h"], cc["eri"], cc["dets"], cc["coeffs"])
        _pt2_case(asci, oracle_lib, cc, E0)


def test_pt2_energy_16e20o(asci):
    c = syn.workload("16e20o")
    g = _golden("16e20o")
    d = to_dev(c)
    e, cnt = asci.pt2(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], float.fromhex(g["E0"]))
    assert cnt == g["ncandidates"]
    want = float.fromhex(g["pt2"])
    assert abs(e - want) <= pt2_tol(want, float.fromhex(g["pt2_abs_terms"]), float.fromhex(g["pt2_term_tol"]))


def test_profiler_entries_and_kernel_filter(asci, oracle_lib):
    """Per-kernel timing: every timed kernel gets an entry with launches and
    algorithmic bytes; restricted to one name, only that kernel is timed; the
    results do not change either way."""
    import torch

    c = _case(12, 6, 6, 150, seed=41, sampler="level")
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    d = to_dev(c)
    ctx = asci.Context.get(0)
    base = [host(t) for t in asci.search(d["h"], d["eri"], 12, 6, 6, d["dets"], d["coeffs"], E0, 100, ctx=ctx)]
    try:
        ctx.set_profiling(True)
        got = [host(t) for t in asci.search(d["h"], d["eri"], 12, 6, 6, d["dets"], d["coeffs"], E0, 100, ctx=ctx)]
        torch.cuda.synchronize()
        prof = ctx.profile()
        assert {"generate", "finish", "collect"} <= set(prof)
        assert all(v[1] >= 1 and v[0] >= 0.0 for v in prof.values())
        assert prof["finish"][2] > 0.0
        ctx.set_profiling(True, only="finish")
        got2 = [host(t) for t in asci.search(d["h"], d["eri"], 12, 6, 6, d["dets"], d["coeffs"], E0, 100, ctx=ctx)]
        torch.cuda.synchronize()
        assert set(ctx.profile()) == {"finish"}
    finally:
        ctx.set_profiling(False)
    for a, b, e in zip(base, got, got2):
        assert a.tobytes() == b.tobytes() == e.tobytes()


def test_forced_fault_fails_the_call_and_clears(asci, oracle_lib):
    """The kernels' internal-consistency fault word (a dropped write past a
    buffer, a clamped orbital index) fails the call with ASCI_EDEVICE; forced
    from the host, the search raises it, writes no result, and the next
    search on the context is correct again."""
    c = _case(8, 4, 3, 40, seed=5)
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    d = to_dev(c)
    ctx = asci.Context.get(0)
    try:
        ctx.set_param("fault_test", 1)
        with pytest.raises(asci.AsciError) as e:
            asci.search(d["h"], d["eri"], 8, 4, 3, d["dets"], d["coeffs"], E0, 100, ctx=ctx)
        assert e.value.code == asci.ASCI_EDEVICE
    finally:
        ctx.set_param("fault_test", 0)
    gk, gs = asci.search(d["h"], d["eri"], 8, 4, 3, d["dets"], d["coeffs"], E0, 100, ctx=ctx)
    want = oracle_lib.search_all(c["h"], c["eri"], 8, 4, 3, c["dets"], c["coeffs"], E0)
    assert_topk(host(gk), host(gs), want, 100)


def test_invalid_requests_rejected_by_batch_and_server(asci, oracle_lib):
    """A request with an invalid option (a negative constraint level) is
    refused before any GPU work: by the server at submission, by the batch
    per request while the valid requests of the batch still complete."""
    c = _case(10, 4, 4, 50, seed=6)
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    d = to_dev(c)
    good = asci.SearchRequest(d["h"], d["eri"], 10, 4, 4, d["dets"], d["coeffs"], E0, 50)
    bad = asci.SearchRequest(d["h"], d["eri"], 10, 4, 4, d["dets"], d["coeffs"], E0, 50, constraint_level=-1)
    srv = asci.Server(device=0, slots=1)
    try:
        with pytest.raises(asci.AsciError) as e:
            srv.submit(bad)
        assert e.value.code == asci.ASCI_EINVAL
        assert srv.wait(srv.submit(good)).status == 0
    finally:
        srv.close()
    with pytest.raises(asci.AsciError):
        asci.search_batch([good, bad])
