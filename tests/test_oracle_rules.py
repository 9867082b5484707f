"""Pins of the oracle's rewrite rules against exact tensor evaluation.

The tensor evaluator sums the spider and Hadamard-edge tensors directly
(appendix "ZX-Calculus": spider and Hadamard definitions), so it is an
independent definition of what a diagram means.  Each rewrite must leave the
linear map unchanged *including* the scalar it emits (local complementation
rule and pivoting rule of the appendix; scalar readings for general
neighbourhoods as documented in the oracle).
"""
import cmath
import math

import numpy as np
import pytest

import oracle
from oracle.tensor import evaluate_graph, to_complex
from workloads.generators import pack_rows


def random_graph(rng, n, q, dens, hwire=False):
    bits = (rng.random((n, n)) < dens).astype(np.uint8)
    bits = np.triu(bits, 1)
    bits = bits + bits.T
    adj = pack_rows(bits)
    k = rng.integers(0, 8, n).astype(np.int8)
    spiders = rng.permutation(n)
    ins = spiders[:q].astype(np.int32)
    outs = spiders[q:2 * q].astype(np.int32)
    bh = (rng.random(2 * q) < 0.3).astype(np.uint8) if hwire else np.zeros(2 * q, np.uint8)
    return oracle.Graph(n, adj, k, ins, outs, bh)


def interior(g):
    return [v for v in g.alive_list() if not g.has_boundary(v)]


@pytest.mark.parametrize("seed", range(60))
def test_lc_preserves_map_exactly(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 11))
    q = int(rng.integers(0, min(2, (n - 1) // 2) + 1))
    g = random_graph(rng, n, q, [0.3, 0.5, 0.8][seed % 3], hwire=seed % 4 == 0)
    cands = interior(g)
    u = int(rng.choice(cands))
    g.k[u] = 2 if seed % 2 == 0 else 6
    before = evaluate_graph(g)
    h = g.copy()
    assert h.local_comp(u) == oracle.OK
    after = evaluate_graph(h)
    assert before.equals(after)
    assert not h.is_alive(u)


@pytest.mark.parametrize("seed", range(60))
def test_pivot_preserves_map_exactly(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(3, 11))
    q = int(rng.integers(0, min(2, (n - 2) // 2) + 1))
    g = random_graph(rng, n, q, [0.3, 0.5, 0.8][seed % 3], hwire=seed % 5 == 0)
    ins = interior(g)
    if len(ins) < 2:
        pytest.skip("need two interior spiders")
    u, v = (int(x) for x in rng.choice(ins, 2, replace=False))
    if not g.edge(u, v):
        g.adj[u, v // 64] ^= np.uint64(1) << np.uint64(v % 64)
        g.adj[v, u // 64] ^= np.uint64(1) << np.uint64(u % 64)
    g.k[u] = int(rng.choice([0, 4]))
    g.k[v] = int(rng.choice([0, 4]))
    before = evaluate_graph(g)
    h = g.copy()
    assert h.pivot(u, v) == oracle.OK
    after = evaluate_graph(h)
    assert before.equals(after)
    assert not h.is_alive(u) and not h.is_alive(v)


def test_lc_drops_the_toggled_off_correction_would_fail():
    """A neighbourhood with existing edges needs the -2 per removed edge term:
    brute force on a triangle-plus-centre shows the printed scalar alone is off."""
    # centre 0 joined to 1,2,3; edge 1-2 present.
    bits = np.zeros((4, 4), np.uint8)
    for a, b in [(0, 1), (0, 2), (0, 3), (1, 2)]:
        bits[a, b] = bits[b, a] = 1
    g = oracle.Graph(4, pack_rows(bits), [2, 0, 0, 0])
    before = evaluate_graph(g)
    h = g.copy()
    assert h.local_comp(0) == oracle.OK
    after = evaluate_graph(h)
    assert before.equals(after)
    # (n-1)(n-2)/2 = 1 for n = 3, one edge toggled off -> net power -1
    assert h.scalar.pow_sqrt2 == 1 - 2
    wrong = oracle.tensor.Amp(after.M, after.pow + 2, after.phase)
    assert not before.equals(wrong)


def test_isolated_half_pi_spider_closed_form():
    """A lone Z spider of phase pi/2 is the number 1 + e^{i pi/2} = 1 + i; the
    LC rule removes it and must emit exactly sqrt(2) e^{i pi/4} = 1 + i.
    With phase 3pi/2 the value is 1 - i = sqrt(2) e^{-i pi/4}."""
    for k, expect in [(2, 1 + 1j), (6, 1 - 1j)]:
        g = oracle.Graph(1, np.zeros((1, 1), np.uint64), [k])
        val = complex(to_complex(evaluate_graph(g))[0, 0])
        assert abs(val - expect) < 1e-12
        assert g.local_comp(0) == oracle.OK
        assert g.alive_list() == []
        emitted = (math.sqrt(2) ** g.scalar.pow_sqrt2) * cmath.exp(1j * math.pi * g.scalar.phase8 / 4)
        assert abs(emitted - expect) < 1e-12


def test_isolated_edge_pivot_closed_form():
    """Two Pauli spiders a*pi, b*pi joined by one Hadamard edge evaluate to
    sum_{x,y} (-1)^{ax + by + xy} / sqrt(2) = sqrt(2) (-1)^{ab}."""
    bits = np.array([[0, 1], [1, 0]], np.uint8)
    for a in (0, 1):
        for b in (0, 1):
            g = oracle.Graph(2, pack_rows(bits), [4 * a, 4 * b])
            val = complex(to_complex(evaluate_graph(g))[0, 0])
            assert abs(val - math.sqrt(2) * (-1) ** (a * b)) < 1e-12
            assert g.pivot(0, 1) == oracle.OK
            emitted = (math.sqrt(2) ** g.scalar.pow_sqrt2) * cmath.exp(1j * math.pi * g.scalar.phase8 / 4)
            assert abs(emitted - val) < 1e-12


@pytest.mark.parametrize("nleaf", [1, 2, 3, 5, 8])
def test_star_lc_gives_complete_graph(nleaf):
    n = nleaf + 1
    bits = np.zeros((n, n), np.uint8)
    bits[0, 1:] = bits[1:, 0] = 1
    g = oracle.Graph(n, pack_rows(bits), [2] + [1] * nleaf)
    assert g.local_comp(0) == oracle.OK
    b = g.bits()
    for x in range(1, n):
        for y in range(1, n):
            assert b[x, y] == (1 if x != y else 0)
    assert list(g.k[1:]) == [7] * nleaf  # pi/4 - pi/2 = -pi/4
    assert g.scalar.pow_sqrt2 == (nleaf - 1) * (nleaf - 2) // 2


def test_rule_preconditions_rejected():
    bits = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], np.uint8)
    g = oracle.Graph(3, pack_rows(bits), [1, 2, 0], inputs=[0], outputs=[2])
    assert g.local_comp(0) == oracle.ENOMATCH     # phase pi/4
    assert g.local_comp(2) == oracle.ENOMATCH     # boundary spider
    assert g.pivot(0, 2) == oracle.ENOMATCH       # not adjacent
    assert g.pivot(1, 2) == oracle.ENOMATCH       # phase pi/2, boundary
    assert g.local_comp(7) == oracle.EINVAL


@pytest.mark.parametrize("seed", range(40))
def test_simplify_preserves_map_exactly(seed):
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(4, 17))
    q = int(rng.integers(1, 3))
    g = random_graph(rng, n, q, [0.2, 0.35, 0.5][seed % 3], hwire=seed % 6 == 0)
    # bias phases toward Clifford so that rewrites happen
    cl = rng.random(n) < 0.8
    g.k[cl] = (rng.integers(0, 4, cl.sum()) * 2).astype(np.int8)
    if n - 2 * q > 16:
        pytest.skip("too many free spiders")
    before = evaluate_graph(g)
    h = g.copy()
    k0 = h.k.copy()
    assert h.simplify() == oracle.OK
    after = evaluate_graph(h)
    assert before.equals(after)
    # fixed point: no interior pi/2 spider, no adjacent interior Pauli pair
    alive = h.alive_list()
    for v in alive:
        if not h.has_boundary(v):
            assert h.k[v] not in (2, 6)
    for u in alive:
        for v in alive:
            if u < v and h.edge(u, v) and not h.has_boundary(u) and not h.has_boundary(v):
                assert not (h.k[u] in (0, 4) and h.k[v] in (0, 4))
    # invariants: boundary and odd-phase spiders survive; survivors keep k mod 2
    for v in range(n):
        if g.has_boundary(v) or k0[v] % 2 == 1:
            assert h.is_alive(v)
    for v in alive:
        assert h.k[v] % 2 == k0[v] % 2
    removed = sum(1 if r[1] == 0 else 2 for r in h.trace)
    assert removed == n - len(alive)


def test_all_clifford_interior_reduces_to_scalar():
    """With every spider Clifford and no boundary the rules remove everything
    that is interior (appendix: the Clifford case reduces to a scalar)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        n = int(rng.integers(2, 12))
        g = random_graph(rng, n, 0, 0.4)
        g.k[:] = (rng.integers(0, 4, n) * 2).astype(np.int8)
        before = evaluate_graph(g)
        assert g.simplify() == oracle.OK
        after = evaluate_graph(g)
        assert before.equals(after)
        # remaining spiders (if any) are isolated Pauli spiders: a Pauli spider
        # with no neighbour is not matched by either rule
        for v in g.alive_list():
            assert g.k[v] in (0, 4)
            assert all(not g.edge(v, w) for w in g.alive_list())
