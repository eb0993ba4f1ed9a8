"""Brute-force second-quantised Hamiltonian on tiny spaces (a pin for the oracle).

Independent of the oracle and of the HIP path: it applies the operator strings
of H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q (spin summed)
one operator at a time to occupation bitmasks over 2n spin orbitals, alpha
orbitals first.  The sign of a_x or a+_x on a determinant is
(-1)^(number of occupied spin orbitals below x), which fixes the same phase
convention the library documents (creators in ascending spin-orbital order).
No Slater-Condon case analysis is used.
"""
from __future__ import annotations

from collections import defaultdict
from itertools import combinations

import numpy as np


def _sign_below(det, x):
    return -1 if bin(det & ((1 << x) - 1)).count("1") & 1 else 1


def _annih(det, x):
    if not (det >> x) & 1:
        return None, 0
    return det & ~(1 << x), _sign_below(det, x)


def _create(det, x):
    if (det >> x) & 1:
        return None, 0
    return det | (1 << x), _sign_below(det, x)


def to_so(n, alpha, beta):
    return int(alpha) | (int(beta) << n)


def from_so(n, d):
    m = (1 << n) - 1
    return d & m, (d >> n) & m


def apply_h(h, eri, n, det_so):
    """H|det> as {det_so': coefficient}."""
    out = defaultdict(float)
    spins = (0, 1)
    for sg in spins:
        for q in range(n):
            d1, s1 = _annih(det_so, sg * n + q)
            if d1 is None:
                continue
            for p in range(n):
                d2, s2 = _create(d1, sg * n + p)
                if d2 is None:
                    continue
                out[d2] += h[p, q] * s1 * s2
    for sg in spins:
        for tau in spins:
            for q in range(n):
                d1, s1 = _annih(det_so, sg * n + q)
                if d1 is None:
                    continue
                for s in range(n):
                    d2, s2 = _annih(d1, tau * n + s)
                    if d2 is None:
                        continue
                    for r in range(n):
                        d3, s3 = _create(d2, tau * n + r)
                        if d3 is None:
                            continue
                        for p in range(n):
                            d4, s4 = _create(d3, sg * n + p)
                            if d4 is None:
                                continue
                            out[d4] += 0.5 * eri[p, q, r, s] * s1 * s2 * s3 * s4
    return out


def space(n, na, nb):
    """All determinants (alpha, beta) of the space, alpha-major ascending."""
    A = [sum(1 << p for p in c) for c in combinations(range(n), na)]
    B = [sum(1 << p for p in c) for c in combinations(range(n), nb)]
    A.sort()
    B.sort()
    return [(a, b) for a in A for b in B]


def dense_h(h, eri, n, na, nb, ecore=0.0):
    dets = space(n, na, nb)
    index = {to_so(n, a, b): i for i, (a, b) in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)))
    for j, (a, b) in enumerate(dets):
        for d, v in apply_h(h, eri, n, to_so(n, a, b)).items():
            H[index[d], j] += v
    H += ecore * np.eye(len(dets))
    return dets, H
