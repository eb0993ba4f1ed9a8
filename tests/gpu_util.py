"""Helpers for GPU tests: move seeded inputs to the device, compare with the oracle."""
import numpy as np


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


def assert_topk_parity(got_keys, got_scores, want_keys, want_scores, tol=1e-12):
    """Top-k parity: bit-exact keys and order, scores within tol relative.
    Positions whose |score| lies within tol of the k-th value are tie-band
    positions: there the key set may differ only among tie-band members."""
    assert got_keys.shape == want_keys.shape, (got_keys.shape, want_keys.shape)
    if len(want_keys) == 0:
        return
    r = rel_err(got_scores, want_scores)
    kth = abs(want_scores[-1])
    band = np.abs(np.abs(want_scores) - kth) <= tol * max(kth, 1e-300)
    same = (got_keys == want_keys).all(axis=1)
    assert (same | band).all(), "top-k keys differ outside the tie band"
    assert r[same].max(initial=0.0) <= tol, r.max()
