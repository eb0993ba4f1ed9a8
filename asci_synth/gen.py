"""Seeded synthetic workloads shaped like the paper's Cr2 (24e,30o) search.

The paper's integrals (a Molpro Cr2/def-SVP calculation) are not available, so
every workload here is synthetic.  The recipe (fixed draw order, one
``numpy.random.default_rng(seed)`` per workload):

integrals(n)
    d = sort(U(-2, 2)^n) gives h_pp ("uniform"), or, for the Cr2-shaped
    variant, n/3 orbitals in each of three blocks centred at -2, 0, +2 with
    U(-0.1, 0.1) jitter, clipped to [-3, 3] and sorted.
    For p < q (row-major): h_pq = h_qp = N(0, 0.3) * exp(-|p-q|/4).
    For canonical index quadruples p >= q, r >= s, pq >= rs (pair index
    pq = p(p+1)/2 + q, visited in ascending pq then rs):
    (pq|rs) = 0.1 * exp(-(|p-q| + |r-s|)/3) * N(0, 1), plus 0.5 when p == q
    and r == s; all 8 index permutations receive the same value.

determinants
    The aufbau determinant (lowest n_alpha / n_beta orbitals) is index 0.
    "uniform": further determinants are uniform draws from the Hilbert space
    (alpha and beta occupations chosen independently), duplicates rejected.
    "level": an excitation level L >= 1 relative to aufbau is drawn with
    P(L) ~ exp(-L); the split L = L_a + L_b is drawn with weight equal to the
    number of determinants with that split, then holes and particles uniformly;
    duplicates are rejected and the accepted determinants are ordered by L.

coefficients
    C_i = N(0, 1) * exp(-i / tau), normalised to unit 2-norm.

Bit p of a 64-bit word is spatial orbital p; a determinant is (alpha, beta).
"""
from __future__ import annotations

from math import comb

import numpy as np

__all__ = [
    "integrals",
    "aufbau",
    "uniform_dets",
    "level_dets",
    "coefficients",
    "hilbert_dim",
    "make_case",
    "workload",
    "WORKLOADS",
    "batch_specs",
    "small_batch_specs",
]


def _mask(orbs) -> int:
    m = 0
    for p in orbs:
        m |= 1 << int(p)
    return m


def hilbert_dim(n: int, na: int, nb: int) -> int:
    return comb(n, na) * comb(n, nb)


def integrals(n: int, rng: np.random.Generator, orbital_energies: str = "uniform"):
    """Return (h, eri): h is n x n, eri is n^4 row-major (pq|rs), both float64."""
    if orbital_energies == "uniform":
        d = np.sort(rng.uniform(-2.0, 2.0, n))
    elif orbital_energies == "cr2":
        centres = np.array([-2.0, 0.0, 2.0])
        sizes = [n // 3 + (1 if b < n % 3 else 0) for b in range(3)]
        base = np.concatenate([np.full(s, c) for s, c in zip(sizes, centres)])
        d = np.sort(np.clip(base + rng.uniform(-0.1, 0.1, n), -3.0, 3.0))
    else:
        raise ValueError(orbital_energies)
    h = np.diag(d).astype(np.float64)
    iu = np.triu_indices(n, 1)
    off = rng.normal(0.0, 0.3, len(iu[0])) * np.exp(-np.abs(iu[0] - iu[1]) / 4.0)
    h[iu] = off
    h[(iu[1], iu[0])] = off

    # canonical pairs pq (p >= q) in ascending pair index
    pairs = [(p, q) for p in range(n) for q in range(p + 1)]
    npair = len(pairs)
    pa = np.array(pairs, dtype=np.int64)
    I, J = np.tril_indices(npair)  # I >= J, visited row-major: pq = I ascending, rs = J
    p, q = pa[I, 0], pa[I, 1]
    r, s = pa[J, 0], pa[J, 1]
    vals = 0.1 * np.exp(-(np.abs(p - q) + np.abs(r - s)) / 3.0) * rng.normal(0.0, 1.0, len(I))
    vals = vals + np.where((p == q) & (r == s), 0.5, 0.0)
    eri = np.zeros((n, n, n, n), dtype=np.float64)
    for (a, b, c, d_) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                          (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
        eri[a, b, c, d_] = vals
    return h, eri


def aufbau(n: int, na: int, nb: int):
    return ((1 << na) - 1, (1 << nb) - 1)


def uniform_dets(n, na, nb, count, rng, exclude=()):
    seen = set(exclude)
    out = []
    while len(out) < count:
        a = _mask(rng.choice(n, size=na, replace=False))
        b = _mask(rng.choice(n, size=nb, replace=False))
        if (a, b) in seen:
            continue
        seen.add((a, b))
        out.append((a, b))
    return out


def level_dets(n, na, nb, count, rng, exclude=()):
    """Draw `count` distinct determinants by excitation level from aufbau.

    Draws are made in blocks: per block, the levels, then the alpha/beta splits,
    then uniform random subsets (holes of alpha, particles of alpha, holes of
    beta, particles of beta) as the lowest-ranked entries of uniform keys.
    Duplicates (and the aufbau determinant) are rejected in draw order."""
    va, vb = n - na, n - nb
    lmax = min(na, va) + min(nb, vb)
    if lmax < 1:
        raise ValueError("Hilbert space has a single determinant")
    levels = np.arange(1, lmax + 1)
    pl = np.exp(-levels.astype(np.float64))
    pl /= pl.sum()
    split_la, split_cdf = {}, {}
    for L in levels:
        las = np.array([la for la in range(0, L + 1)
                        if la <= min(na, va) and L - la <= min(nb, vb)], dtype=np.int64)
        w = np.array([comb(na, la) * comb(va, la) * comb(nb, L - la) * comb(vb, L - la)
                      for la in las], dtype=np.float64)
        split_la[L] = las
        split_cdf[L] = np.cumsum(w / w.sum())
    fa, fb = aufbau(n, na, nb)
    seen = set(exclude)
    seen.add((fa, fb))
    if count > hilbert_dim(n, na, nb) - len(seen):
        raise ValueError("not enough determinants in the Hilbert space")
    bit = np.uint64(1) << np.arange(n, dtype=np.uint64)

    def subset_bits(nrow, width, size, offset):
        if width == 0:
            return np.zeros(nrow, dtype=np.uint64)
        rank = np.argsort(np.argsort(rng.random((nrow, width)), axis=1), axis=1)
        take = rank < size[:, None]
        return (take.astype(np.uint64) * bit[offset:offset + width]).sum(axis=1, dtype=np.uint64)

    drawn = []
    while len(drawn) < count:
        B = max(1024, 2 * (count - len(drawn)))
        Ls = rng.choice(levels, size=B, p=pl)
        u = rng.random(B)
        la = np.zeros(B, dtype=np.int64)
        for L in np.unique(Ls):
            sel = Ls == L
            j = np.minimum(np.searchsorted(split_cdf[L], u[sel], side="right"),
                           len(split_la[L]) - 1)
            la[sel] = split_la[L][j]
        lb = Ls - la
        ha = subset_bits(B, na, la, 0)
        pa = subset_bits(B, va, la, na)
        hb = subset_bits(B, nb, lb, 0)
        pb = subset_bits(B, vb, lb, nb)
        A = (np.uint64(fa) & ~ha) | pa
        Bb = (np.uint64(fb) & ~hb) | pb
        for i in range(B):
            key = (int(A[i]), int(Bb[i]))
            if key in seen:
                continue
            seen.add(key)
            drawn.append((int(Ls[i]), len(drawn), key[0], key[1]))
            if len(drawn) == count:
                break
    drawn.sort()
    return [(a, b) for _, _, a, b in drawn]


def coefficients(count, tau, rng):
    c = rng.normal(0.0, 1.0, count) * np.exp(-np.arange(count) / float(tau))
    return c / np.linalg.norm(c)


def make_case(n, na, nb, ndets, seed, sampler="uniform", tau=None, k=None,
              orbital_energies="uniform"):
    """One search input: integrals, determinants (aufbau first) and coefficients."""
    rng = np.random.default_rng(seed)
    h, eri = integrals(n, rng, orbital_energies)
    first = aufbau(n, na, nb)
    rest = ndets - 1
    if sampler == "uniform":
        dets = [first] + uniform_dets(n, na, nb, rest, rng, exclude=(first,))
    elif sampler == "level":
        dets = [first] + level_dets(n, na, nb, rest, rng, exclude=(first,))
    else:
        raise ValueError(sampler)
    if tau is None:
        tau = max(ndets / 10.0, 1.0)
    C = coefficients(ndets, tau, rng)
    return {
        "norb": n, "nalpha": na, "nbeta": nb,
        "h": h, "eri": eri,
        "dets": np.array(dets, dtype=np.uint64).reshape(ndets, 2),
        "coeffs": C,
        "k": int(k) if k is not None else 10 * ndets,
        "seed": seed,
    }


# The three single-search workloads: (8e,12o) uniform cores, (16e,20o) and the
# Cr2-shaped (24e,30o) with level-sampled cores.
WORKLOADS = {
    "8e12o": dict(n=12, na=4, nb=4, ndets=201, seed=1, sampler="uniform", tau=20.0, k=2000),
    "16e20o": dict(n=20, na=8, nb=8, ndets=10_000, seed=2, sampler="level", tau=1000.0, k=100_000),
    "24e30o": dict(n=30, na=12, nb=12, ndets=100_000, seed=3, sampler="level", tau=10_000.0,
                   k=1_000_000, orbital_energies="cr2"),
}


def workload(name: str):
    w = dict(WORKLOADS[name])
    case = make_case(w.pop("n"), w.pop("na"), w.pop("nb"), w.pop("ndets"), w.pop("seed"), **w)
    case["name"] = name
    return case


def batch_specs(count=64, seed=64):
    """Sizes for a batch of uneven searches: norb ~ U{16..40}, even electron count
    ~ U{8..28} with n_alpha = n_beta <= norb - 2, core count round(10^U(3,5))
    clamped to a quarter of the Hilbert space, k = 10 x core count."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(rng.integers(16, 41))
        ne = int(rng.integers(4, 15)) * 2
        na = min(ne // 2, n - 2)
        ncore = int(round(10 ** rng.uniform(3, 5)))
        ncore = max(1, min(ncore, hilbert_dim(n, na, na) // 4))
        specs.append(dict(n=n, na=na, nb=na, ndets=ncore, seed=1000 + i, sampler="level",
                          tau=max(ncore / 10.0, 1.0), k=10 * ncore))
    return specs


def small_batch_specs(count=256, seed=65):
    """Sizes for a batch of small searches (the regime where one search does
    not fill the GPU): norb ~ U{10..20}, even electron count ~ U{4..12} with
    n_alpha = n_beta <= norb - 2, core count round(10^U(2,3)) clamped to a
    quarter of the Hilbert space, k = 10 x core count."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(rng.integers(10, 21))
        ne = int(rng.integers(2, 7)) * 2
        na = min(ne // 2, n - 2)
        ncore = int(round(10 ** rng.uniform(2, 3)))
        ncore = max(1, min(ncore, hilbert_dim(n, na, na) // 4))
        specs.append(dict(n=n, na=na, nb=na, ndets=ncore, seed=5000 + i, sampler="level",
                          tau=max(ncore / 10.0, 1.0), k=10 * ncore))
    return specs
