"""Pins of the oracle's ASCI loop (Alg. 1, Sec. II.C): the double-loop
Hamiltonian against the brute-force second-quantised H, the selection rule on
a hand-made case, and the whole loop against full CI on tiny spaces."""
import numpy as np
import pytest

import asci_synth as syn
import sq_bruteforce as bf


def _ints(n, seed):
    return syn.integrals(n, np.random.default_rng(seed))


@pytest.mark.parametrize("n,na,nb", [(5, 2, 2), (6, 3, 2), (4, 1, 3)])
def test_double_loop_h_equals_second_quantised_h(oracle_lib, n, na, nb):
    h, eri = _ints(n, 40 + n)
    space, H = bf.dense_h(h, eri, n, na, nb, ecore=0.7)
    dets = np.array(space, dtype=np.uint64)
    got = oracle_lib.hamiltonian(h, eri, dets, ecore=0.7)
    assert np.abs(got - H).max() <= 1e-12 * max(1.0, np.abs(H).max())
    # a subset in another order: rows and columns follow the set's order
    rng = np.random.default_rng(n)
    sub = rng.permutation(len(space))[: len(space) // 2]
    got = oracle_lib.hamiltonian(h, eri, dets[sub], ecore=0.7)
    assert np.abs(got - H[np.ix_(sub, sub)]).max() <= 1e-12 * max(1.0, np.abs(H).max())


def test_selection_rule(oracle_lib):
    dets = np.array([[3, 3], [5, 3], [6, 3]], dtype=np.uint64)
    C = np.array([0.9, -0.3, 0.05])
    cand = np.array([[9, 3], [3, 5], [10, 3], [12, 3]], dtype=np.uint64)
    A = np.array([-0.3, 0.4, 0.01, 0.3])
    got, guess = oracle_lib.select_next(dets, C, cand, A, 4)
    # 0.9 (old), 0.4 (new), then three entries tie at 0.3: keys (5,3) < (9,3) < (12,3)
    assert got.tolist() == [[3, 3], [3, 5], [5, 3], [9, 3]]
    assert guess.tolist() == [0.9, 0.0, -0.3, 0.0]
    got, _ = oracle_lib.select_next(dets, C, cand, A, 100)
    assert len(got) == 7


@pytest.mark.parametrize("n,na,nb", [(6, 2, 2), (6, 3, 3), (7, 2, 3)])
def test_loop_reaches_full_ci(oracle_lib, n, na, nb):
    """With N_tdets at least the Hilbert dimension the loop fills the space and
    its energy is the FCI ground state; every iterate lies above it."""
    h, eri = _ints(n, 60 + n)
    space, H = bf.dense_h(h, eri, n, na, nb)
    efci = float(np.linalg.eigvalsh(H)[0])
    hf = np.array([syn.aufbau(n, na, nb)], dtype=np.uint64)
    hist = oracle_lib.asci_loop(h, eri, n, na, nb, hf, np.ones(1), ntdets=len(space), max_iter=8, e_tol=1e-12)
    for dets, C, E in hist:
        assert E >= efci - 1e-10
    assert len(hist[-1][0]) == len(space)
    assert abs(hist[-1][2] - efci) <= 1e-10 * max(1.0, abs(efci))


def test_truncated_loop_is_variational(oracle_lib):
    n, na, nb = 7, 3, 3
    h, eri = _ints(n, 77)
    space, H = bf.dense_h(h, eri, n, na, nb)
    efci = float(np.linalg.eigvalsh(H)[0])
    hf = np.array([syn.aufbau(n, na, nb)], dtype=np.uint64)
    hist = oracle_lib.asci_loop(h, eri, n, na, nb, hf, np.ones(1), ntdets=60, max_iter=6, e_tol=0.0)
    for dets, C, E in hist[1:]:
        assert len(dets) == 60 and len(np.unique(dets, axis=0)) == 60
        assert E >= efci - 1e-10
        # E is the lowest eigenvalue of H over its own set
        assert abs(E - np.linalg.eigvalsh(oracle_lib.hamiltonian(h, eri, dets))[0]) <= 1e-10
    assert hist[-1][2] < hist[0][2]
