"""Pins of the oracle's output-frontier build and of the round checks.

The frontier matrix is this library's reading of the extraction step (the
paper gives only the GF(2) elimination): row j = the spider carrying output j,
column c = spider c, bit set for a Hadamard edge to a present spider that
carries no output.  Here it is rebuilt from the dense 0/1 adjacency by that
definition alone and compared with ``oracle.Graph.frontier``:

* a hand-worked 8-spider fixture (``golden/frontier_worked_8.txt``) with an
  output-output edge, a removed spider whose edge bit is still set, and outputs
  out of id order;
* random diagrams of at most 10 qubits, from their source state and from
  states part-way through simplification, also with spiders marked removed
  without clearing their edges (so only the alive mask can drop them).

A frontier build that kept output columns, kept removed spiders or took rows
in id order instead of output order fails these tests.

``policy.round_is_valid`` is pinned on constructed rounds: a pivot round that
leaves out an edge compatible with every taken edge is rejected.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import policy
from workloads import batch_diagram, single_diagram
from workloads.generators import pack_rows, unpack_rows

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def frontier_by_definition(bits, alive, outputs):
    """q x n 0/1 matrix straight from the definition (dense numpy)."""
    n = bits.shape[0]
    is_out = np.zeros(n, bool)
    is_out[list(outputs)] = True
    M = np.zeros((len(outputs), n), np.uint8)
    for j, o in enumerate(outputs):
        for c in range(n):
            M[j, c] = bits[o, c] and alive[c] and not is_out[c]
    return M


def span(rows):
    s = {0}
    for r in rows:
        v = int("".join(str(int(x)) for x in r[::-1]), 2) if len(r) else 0
        s |= {t ^ v for t in s}
    return s


def is_rref(R, piv, rank):
    """Every pivot is the leading 1 of its row, the only 1 in its column,
    pivots strictly increase, rows past the rank are zero."""
    for i in range(R.shape[0]):
        nz = np.nonzero(R[i])[0]
        if i >= rank:
            if len(nz) or piv[i] != -1:
                return False
            continue
        if not len(nz) or nz[0] != piv[i] or R[:, piv[i]].sum() != 1:
            return False
        if i and piv[i] <= piv[i - 1]:
            return False
    return True


def read_gold():
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLD, "frontier_worked_8.txt"))]
    lines = [l for l in lines if l]
    kv = {}
    mats = {"M": [], "R": []}
    cur = None
    for l in lines:
        if l in mats:
            cur = l
        elif set(l) <= {"0", "1"} and cur:
            mats[cur].append([int(c) for c in l])
        else:
            key, *vals = l.split()
            kv[key] = vals
            cur = None
    return kv, np.array(mats["M"], np.uint8), np.array(mats["R"], np.uint8)


def test_frontier_worked_example():
    kv, Mexp, Rexp = read_gold()
    n = int(kv["n"][0])
    bits = np.zeros((n, n), np.uint8)
    for e in kv["edges"]:
        a, b = map(int, e.split("-"))
        bits[a, b] = bits[b, a] = 1
    ins = [int(x) for x in kv["inputs"]]
    outs = [int(x) for x in kv["outputs"]]
    alive = np.zeros(n, bool)
    alive[[int(x) for x in kv["alive"]]] = True
    # the definition reproduces the hand-built matrix
    assert np.array_equal(frontier_by_definition(bits, alive, outs), Mexp)
    g = oracle.Graph(n, pack_rows(bits), np.zeros(n, np.int8), ins, outs)
    for v in range(n):
        if not alive[v]:   # removed without clearing its edges
            g.alive[v // 64] &= ~(np.uint64(1) << np.uint64(v % 64))
    R, piv, rank, ops = g.frontier()
    assert np.array_equal(unpack_rows(R, n), Rexp)
    assert list(piv) == [int(x) for x in kv["pivots"]] and rank == int(kv["rank"][0])
    assert ops == int(kv["rowops"][0])


def _check_state(g):
    bits = g.bits()
    alive = np.array([g.is_alive(v) for v in range(g.n)])
    outs = [int(o) for o in g.outputs]
    Md = frontier_by_definition(bits, alive, outs)
    R, piv, rank, ops = g.frontier()
    Rb = unpack_rows(R, g.n)
    # same row space as the definition's matrix, in RREF: equal to its unique RREF
    assert is_rref(Rb, piv, rank)
    if len(outs) <= 12:
        assert span(Rb) == span(Md)
    # the elimination of the definition's matrix gives the same result and row-op count
    R2, piv2, rank2, ops2 = oracle.gf2_rref(pack_rows(Md), g.n)
    assert np.array_equal(R2, R) and list(piv2) == list(piv) and rank2 == rank and ops2 == ops


@pytest.mark.parametrize("seed", range(24))
def test_frontier_matches_definition(seed):
    rng = np.random.default_rng(900 + seed)
    d = batch_diagram(77, seed, q_lo=2, q_hi=10) if seed % 2 else single_diagram(1 + seed)
    g = oracle.Graph.from_diagram(d)
    _check_state(g)
    # part-way through simplification (removed spiders have zero rows)
    for r in (1, 3):
        h = oracle.Graph.from_diagram(d)
        assert h.simplify(max_rounds=r) == oracle.OK
        _check_state(h)
    # removed spiders whose edges stay set: only the alive mask may drop them
    h = oracle.Graph.from_diagram(d)
    for v in rng.choice(d.n, max(1, d.n // 5), replace=False):
        h.alive[int(v) // 64] &= ~(np.uint64(1) << np.uint64(int(v) % 64))
    _check_state(h)
    # outputs in reverse id order: rows follow output order
    d2 = single_diagram(40 + seed)
    h = oracle.Graph(d2.n, d2.adj, d2.phase, d2.inputs, d2.outputs[::-1].copy())
    _check_state(h)


def _graph(n, edges, k, bnd=()):
    bits = np.zeros((n, n), np.uint8)
    for a, b in edges:
        bits[a, b] = bits[b, a] = 1
    return oracle.Graph(n, pack_rows(bits), np.array(k, np.int8), list(bnd), [])


def test_pivot_round_maximality():
    # two disjoint, non-adjacent edges of interior Pauli spiders: 0-1 and 3-4,
    # joined through the non-Pauli spider 2
    g = _graph(5, [(0, 1), (1, 2), (2, 3), (3, 4)], [0, 4, 1, 0, 4])
    h = g.copy()
    assert h.simplify(max_rounds=1) == oracle.OK
    taken = [(int(u), int(v)) for _, rule, u, v in h.trace]
    assert taken == [(0, 1), (3, 4)]
    assert policy.round_is_valid(g, taken, pivot=True)
    assert not policy.round_is_valid(g, taken[:1], pivot=True)
    assert not policy.round_is_valid(g, taken[1:], pivot=True)
    # an edge adjacent to a taken one may be left out
    g2 = _graph(4, [(0, 1), (1, 2), (2, 3)], [0, 0, 0, 0])
    assert policy.round_is_valid(g2, [(0, 1)], pivot=True)
    assert not policy.round_is_valid(g2, [(0, 1), (2, 3)], pivot=True)
    # LC rounds: leaving out a non-adjacent candidate is rejected
    g3 = _graph(3, [(0, 1)], [2, 6, 2])
    assert policy.round_is_valid(g3, [(0, -1), (2, -1)], pivot=False)
    assert not policy.round_is_valid(g3, [(0, -1)], pivot=False)
