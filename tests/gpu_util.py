"""Helpers for GPU tests: move seeded inputs to the device, compare with the oracle.

The bar (Eq. (1) with the oracle's evaluation order as the reference):
candidate keys and selected keys are bit-exact; N_a lies within
max(1e-12 |N_a|, 64 u num_abs) and A_a within the oracle's tol_a of the
oracle's value, whatever order the GPU adds the terms in; a selection takes
every candidate the oracle's bands mark surely in and nothing outside the
ambiguous ones.
"""
import numpy as np

U = 2.0 ** -53


def to_dev(case):
    import torch

    dev = torch.device("cuda", 0)
    return {
        "h": torch.from_numpy(np.ascontiguousarray(case["h"])).to(dev),
        "eri": torch.from_numpy(np.ascontiguousarray(case["eri"])).to(dev),
        "dets": torch.from_numpy(np.ascontiguousarray(case["dets"]).view(np.int64)).to(dev).view(torch.uint64),
        "coeffs": torch.from_numpy(np.ascontiguousarray(case["coeffs"])).to(dev),
    }


def host(t):
    import torch

    if t.dtype == torch.uint64:
        return t.view(torch.int64).cpu().numpy().view(np.uint64)
    return t.cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.maximum(np.abs(b), 1e-300)
    return np.where(a == b, 0.0, np.abs(a - b) / den)


def num_tol(num, num_abs):
    return np.maximum(1e-12 * np.abs(num), 64 * U * np.asarray(num_abs))


def abs_bits(x):
    return np.ascontiguousarray(np.abs(np.asarray(x, dtype=np.float64))).view(np.uint64)


def assert_selection_order(keys, scores):
    """(|A| desc compared as IEEE bits, key asc): the order every selection is emitted in."""
    if len(keys) == 0:
        return
    order = np.lexsort((keys[:, 1], keys[:, 0], ~abs_bits(scores)))
    assert (order == np.arange(len(keys))).all(), "selection not in (|A| desc, key asc) order"


def locate(want_keys, keys):
    """Positions of keys in the oracle's ascending key list (every key must be there)."""
    import oracle

    codes = oracle.key_codes(want_keys)
    q = oracle.key_codes(keys)
    pos = np.searchsorted(codes, q)
    ok = pos < len(codes)
    ok[ok] = codes[pos[ok]] == q[ok]
    assert ok.all(), "%d returned keys are not oracle candidates" % (~ok).sum()
    return pos


def assert_candidates(keys, num, score, want):
    """Every-candidate output against the oracle's search_all: keys bit-exact,
    N_a and A_a within their tolerances.  Returns (bit-exact scores, relaxed band)."""
    assert keys.shape == want["keys"].shape, (keys.shape, want["keys"].shape)
    assert (keys == want["keys"]).all()
    if num is not None:
        assert (np.abs(num - want["num"]) <= num_tol(want["num"], want["num_abs"])).all()
    bad = ~(np.abs(score - want["score"]) <= want["tol"])
    assert not bad.any(), "%d scores outside the tolerance, e.g. %s" % (
        bad.sum(), list(zip(score[bad][:3], want["score"][bad][:3], want["tol"][bad][:3])))
    relaxed = int((want["tol"] > 1.000001e-12 * np.abs(want["score"])).sum())
    return int((score == want["score"]).sum()), relaxed


def assert_topk(keys, scores, want, k):
    """A top-k selection against the oracle's candidates (search_all with tol)."""
    import oracle

    m = min(k, len(want["keys"]))
    assert keys.shape == (m, 2), (keys.shape, m)
    if m == 0:
        return
    assert_selection_order(keys, scores)
    assert len(np.unique(oracle.key_codes(keys))) == m
    pos = locate(want["keys"], keys)
    diff = np.abs(scores - want["score"][pos])
    assert (diff <= want["tol"][pos]).all(), "selected scores outside the tolerance"
    sure, amb, _ = oracle.topk_bands(want["keys"], want["score"], want["tol"], k)
    chosen = np.zeros(len(sure), bool)
    chosen[pos] = True
    assert not (sure & ~chosen).any(), "%d surely selected candidates missing" % (sure & ~chosen).sum()
    assert not (chosen & ~sure & ~amb).any(), "selected a candidate that is surely out"


def assert_topk_golden(keys, scores, g):
    """A top-k selection against the stored bands of a golden record."""
    import hashlib

    import oracle

    assert len(keys) == g["topk_count"]
    assert_selection_order(keys, scores)
    amb = oracle.key_codes(np.array([[a, b] for a, b, _, _ in g["ambiguous"]], dtype=np.uint64).reshape(-1, 2))
    codes = oracle.key_codes(keys)
    sure = np.sort(codes[~np.isin(codes, amb)])
    assert len(sure) == g["sure_count"]
    assert hashlib.sha256(np.ascontiguousarray(sure).tobytes()).hexdigest() == g["sure_keys_sha256"]
    kth = abs(float(scores[-1]))
    assert float.fromhex(g["kth_lo"]) <= kth <= float.fromhex(g["kth_hi"])
    assert_head(keys, scores, g["topk_head"])


def assert_head(keys, scores, head_rec):
    """The first entries of a selection against the oracle's (key, A, tol)
    records: the same key at each position with the score within tol, except
    where two entries are within tolerance of each other (a near tie that
    another evaluation order may swap)."""
    head = [(int(a), int(b)) for a, b, _, _ in head_rec]
    hs = [float.fromhex(s) for _, _, s, _ in head_rec]
    ht = [float.fromhex(t) for _, _, _, t in head_rec]
    at = {kk: i for i, kk in enumerate(head)}
    for i in range(min(len(head), len(keys))):
        kk, sc = (int(keys[i, 0]), int(keys[i, 1])), float(scores[i])
        if kk == head[i]:
            assert abs(sc - hs[i]) <= ht[i], (i, sc, hs[i], ht[i])
            continue
        j = at.get(kk)
        if j is None:  # swapped with the entry after the recorded head
            assert i >= len(head) - 2 and abs(abs(sc) - abs(hs[i])) <= 2 * ht[i], (i, kk, head[i])
            continue
        assert abs(sc - hs[j]) <= ht[j], (i, sc, hs[j])
        assert abs(abs(hs[i]) - abs(hs[j])) <= ht[i] + ht[j], ("order differs outside a near tie", i, j)
