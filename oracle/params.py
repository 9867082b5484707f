"""Reference of the minimal parameter basis (f = T e) of a simplified diagram.

TEST INFRASTRUCTURE ONLY (imported by ``tests/`` and the CPU-baseline leg of
``bench.py``).

Section on the repetition-code example, equation detector_sampling and the
sentence after it: the parameters that survive reduction are linear
combinations of the error bits e; a minimal set f is chosen by Gaussian
elimination over F2 of the matrix of these dependencies, keeping a linearly
independent basis.  Here the dependency vectors are the parameter rows of the
spiders still present and the selector rows u, v of the recorded terms.  With
R the reduced row echelon form of the stacked vectors and r its rank:

  T      = the first r rows of R  (f = T e, one row per basis parameter);
  coeff  = for each vector d, the bits d[pivot_i], i < r, so that d = coeff . T
           (R has the identity in its pivot columns).
"""
from __future__ import annotations

import numpy as np

from . import gf2_rref, words_for


def dependency_vectors(g) -> np.ndarray:
    """Parameter rows of the present spiders, then each term's u and v rows."""
    alive = g.alive_list()
    _, tu, tv = g.terms()
    rows = [g.params[v] for v in alive] + list(tu) + list(tv)
    if not rows:
        return np.zeros((0, max(g.pw, 1)), np.uint64)
    return np.ascontiguousarray(np.array(rows, dtype=np.uint64).reshape(len(rows), -1))


def fbasis(D: np.ndarray, n_cols: int):
    """(T (r x words), coeff (rows(D) x ceil(r/64) words), pivots (r,), r)."""
    D = np.ascontiguousarray(D, dtype=np.uint64)
    m = D.shape[0]
    if m == 0:
        return np.zeros((0, D.shape[1]), np.uint64), np.zeros((0, 1), np.uint64), np.zeros(0, np.int32), 0
    R, piv, rank, _ = gf2_rref(D, n_cols)
    T = R[:rank].copy()
    cw = max(1, words_for(rank))
    coeff = np.zeros((m, cw), np.uint64)
    for i in range(m):
        for j in range(rank):
            c = int(piv[j])
            if (int(D[i, c // 64]) >> (c % 64)) & 1:
                coeff[i, j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return T, coeff, piv[:rank].copy(), rank
