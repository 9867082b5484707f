"""Pins of the oracle's graph operations, GF(2) elimination and Pauli table.

* local complementation as a graph operation is an involution and keeps every
  cut-rank; the pivot's toggle equals tau_u tau_v tau_u away from u and v;
* reduced row echelon form is unique: brute-force row spaces on tiny inputs,
  planted instances A = P R0, the hand-worked fixture, T A = R;
* Pauli commutation equals the matrix commutator of the textbook Pauli
  matrices built from the paper's (x, z) encoding.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from workloads.generators import pack_rows, unpack_rows

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_bits(rng, n, dens):
    b = np.triu((rng.random((n, n)) < dens).astype(np.uint8), 1)
    return b + b.T


def gf2_rank_bruteforce(rows):
    """Rank as log2 of the size of the span (enumeration; tiny inputs only)."""
    rows = [int(r) for r in rows]
    span = {0}
    for r in rows:
        span |= {s ^ r for s in span}
    return int(np.log2(len(span))), span


def bits_to_ints(B):
    return [int("".join(str(int(x)) for x in row[::-1]), 2) if len(row) else 0 for row in B]


def cut_rank(bits, X):
    Y = [v for v in range(bits.shape[0]) if v not in X]
    sub = bits[np.ix_(sorted(X), Y)]
    r, _ = gf2_rank_bruteforce(bits_to_ints(sub))
    return r


@pytest.mark.parametrize("seed", range(30))
def test_tau_involution_and_cut_rank(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 10))
    bits = rand_bits(rng, n, [0.3, 0.5, 0.8][seed % 3])
    g = oracle.Graph(n, pack_rows(bits), np.zeros(n))
    u = int(rng.integers(0, n))
    h = g.copy()
    assert h.local_comp(u, graph_only=True) == oracle.OK
    nb = [x for x in range(n) if bits[u, x]]
    # tau_u complements exactly the pairs inside N(u)
    diff = h.bits() ^ bits
    for x in range(n):
        for y in range(n):
            assert diff[x, y] == (1 if (x != y and x in nb and y in nb) else 0)
    for _ in range(10):
        X = set(int(v) for v in rng.choice(n, int(rng.integers(1, n)), replace=False))
        assert cut_rank(bits, X) == cut_rank(h.bits(), X)
    assert h.local_comp(u, graph_only=True) == oracle.OK
    assert np.array_equal(h.bits(), bits)


@pytest.mark.parametrize("seed", range(40))
def test_pivot_toggle_is_tau_u_tau_v_tau_u(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 11))
    bits = rand_bits(rng, n, [0.3, 0.5, 0.8][seed % 3])
    u, v = (int(x) for x in rng.choice(n, 2, replace=False))
    bits[u, v] = bits[v, u] = 1
    g = oracle.Graph(n, pack_rows(bits), np.zeros(n))
    p = g.copy()
    assert p.pivot(u, v, graph_only=True) == oracle.OK
    t = g.copy()
    for w in (u, v, u):
        assert t.local_comp(w, graph_only=True) == oracle.OK
    rest = [x for x in range(n) if x not in (u, v)]
    assert np.array_equal(p.bits()[np.ix_(rest, rest)], t.bits()[np.ix_(rest, rest)])
    # and cut-ranks survive the pivot toggle too
    for _ in range(5):
        X = set(int(x) for x in rng.choice(n, int(rng.integers(1, n)), replace=False))
        assert cut_rank(t.bits(), X) == cut_rank(bits, X)


def is_rref(R, rank, piv):
    m, n = R.shape
    for i in range(m):
        nz = np.nonzero(R[i])[0]
        if i >= rank:
            if len(nz):
                return False
            continue
        if len(nz) == 0 or nz[0] != piv[i]:
            return False
        if i > 0 and piv[i] <= piv[i - 1]:
            return False
        col = R[:, piv[i]]
        if col.sum() != 1:
            return False
    return True


@pytest.mark.parametrize("seed", range(60))
def test_rref_bruteforce_tiny(seed):
    rng = np.random.default_rng(500 + seed)
    m = int(rng.integers(1, 8))
    n = int(rng.integers(1, 9))
    B = (rng.random((m, n)) < [0.2, 0.5, 0.8][seed % 3]).astype(np.uint8)
    R, piv, rank, ops = oracle.gf2_rref(pack_rows(B), n)
    Rb = unpack_rows(R, n)
    assert is_rref(Rb, rank, piv)
    ra, span_a = gf2_rank_bruteforce(bits_to_ints(B))
    rr, span_r = gf2_rank_bruteforce(bits_to_ints(Rb))
    assert ra == rr == rank
    assert span_a == span_r
    assert all(p == -1 for p in piv[rank:])


def planted(rng, m, n, rank):
    """R0: a random m x n RREF of the given rank; P: random invertible."""
    piv = np.sort(rng.choice(n, rank, replace=False))
    R0 = np.zeros((m, n), np.uint8)
    for i, c in enumerate(piv):
        R0[i, c] = 1
        free = [x for x in range(c + 1, n) if x not in set(piv)]
        R0[i, free] = rng.integers(0, 2, len(free))
    A = R0.copy()
    for _ in range(4 * m * max(1, m)):
        a, b = rng.choice(m, 2, replace=False) if m > 1 else (0, 0)
        if a == b:
            continue
        if rng.random() < 0.2:
            A[[a, b]] = A[[b, a]]
        else:
            A[a] ^= A[b]
    return A, R0, piv


@pytest.mark.parametrize("m,n,rank", [(5, 9, 3), (16, 40, 16), (40, 100, 25), (64, 64, 64),
                                      (70, 130, 66), (128, 300, 100), (200, 180, 180)])
def test_rref_planted(m, n, rank):
    rng = np.random.default_rng(m * 1000 + n)
    A, R0, piv0 = planted(rng, m, n, rank)
    R, piv, r, _ = oracle.gf2_rref(pack_rows(A), n)
    assert r == rank
    assert np.array_equal(unpack_rows(R, n), R0)
    assert list(piv[:rank]) == list(piv0)


def test_rref_transform():
    rng = np.random.default_rng(11)
    for m, n in [(7, 12), (30, 20), (65, 130)]:
        B = (rng.random((m, n)) < 0.5).astype(np.uint8)
        R, piv, rank, ops, T = oracle.gf2_rref(pack_rows(B), n, want_T=True)
        Tb = unpack_rows(T, m).astype(np.int64)
        assert np.array_equal((Tb @ B.astype(np.int64)) % 2, unpack_rows(R, n))
        # T invertible: full rank
        assert gf2_rank_bruteforce(bits_to_ints(Tb))[0] == m if m <= 20 else True


def read_gold_gf2(name):
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLD, name))]
    lines = [l for l in lines if l]
    ia, ir = lines.index("A"), lines.index("R")
    A = [list(map(int, l)) for l in lines[ia + 1:ir]]
    rest = lines[ir + 1:]
    R = [list(map(int, l)) for l in rest if set(l) <= {"0", "1"}]
    meta = {l.split()[0]: [int(x) for x in l.split()[1:]] for l in rest if not set(l) <= {"0", "1"}}
    return np.array(A, np.uint8), np.array(R, np.uint8), meta


def test_rref_worked_example():
    A, Rexp, meta = read_gold_gf2("gf2_worked_3x4.txt")
    R, piv, rank, ops = oracle.gf2_rref(pack_rows(A), A.shape[1])
    assert np.array_equal(unpack_rows(R, A.shape[1]), Rexp)
    assert list(piv) == meta["pivots"]
    assert rank == meta["rank"][0]
    assert ops == meta["rowops"][0]


# ------------------------------------------------------------------ Pauli --
I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], complex)
PZ = np.array([[1, 0], [0, -1]], complex)
PY = np.array([[0, -1j], [1j, 0]], complex)


def pauli_matrix(xbits, zbits):
    M = np.ones((1, 1), complex)
    for x, z in zip(xbits, zbits):
        P = {(0, 0): I2, (1, 0): PX, (1, 1): PY, (0, 1): PZ}[(int(x), int(z))]
        M = np.kron(M, P)
    return M


def test_pauli_single_qubit_table():
    lines = [l.split("#")[0].split() for l in open(os.path.join(GOLD, "pauli_1q.txt"))]
    rows = [l for l in lines if l and l[0] in "IXYZ"]
    enc = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}
    names = [r[0] for r in rows]
    X = np.array([[enc[p][0]] for p in names], np.uint64)
    Z = np.array([[enc[p][1]] for p in names], np.uint64)
    C = oracle.pauli_commute(X, Z)
    for i, r in enumerate(rows):
        for j in range(4):
            assert ((int(C[i, 0]) >> j) & 1) == int(r[1 + j])


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5])
def test_pauli_bruteforce_matrices(nq):
    rng = np.random.default_rng(nq)
    n = 24
    xb = rng.integers(0, 2, (n, nq)).astype(np.uint8)
    zb = rng.integers(0, 2, (n, nq)).astype(np.uint8)
    C = oracle.pauli_commute(pack_rows(xb), pack_rows(zb))
    Cb = unpack_rows(C, n)
    mats = [pauli_matrix(xb[i], zb[i]) for i in range(n)]
    for i in range(n):
        for j in range(n):
            comm = np.allclose(mats[i] @ mats[j], mats[j] @ mats[i])
            assert Cb[i, j] == (0 if comm else 1)


def test_pauli_symmetry_bilinearity():
    rng = np.random.default_rng(5)
    n, nq = 200, 130
    xb = rng.integers(0, 2, (n, nq)).astype(np.uint8)
    zb = rng.integers(0, 2, (n, nq)).astype(np.uint8)
    X, Z = pack_rows(xb), pack_rows(zb)
    Cb = unpack_rows(oracle.pauli_commute(X, Z), n)
    assert np.array_equal(Cb, Cb.T)
    assert not Cb.diagonal().any()
    # C(P, Q R) = C(P, Q) xor C(P, R): product of strings XORs their bit vectors
    X2 = np.vstack([X, X[:50] ^ X[50:100]])
    Z2 = np.vstack([Z, Z[:50] ^ Z[50:100]])
    C2 = unpack_rows(oracle.pauli_commute(X2, Z2), n + 50)
    assert np.array_equal(C2[:n, n:], Cb[:, :50] ^ Cb[:, 50:100])
