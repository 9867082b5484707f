"""Reference of the learned proposal's candidate handling and of the checks
on schedules other than the canonical one.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).

The paper names the two rules and their fixed point (appendix "Rewrite
rules", equations local_comp and pivoting; appendix "Stabilizer
decompositions", first paragraph) but no order of application.  Any order
reaches a fixed point by sound rewrites, so a schedule that is not the
canonical one is checked by replaying its trace with the rule
implementations of the C oracle, which verify each precondition.

The learned schedule keeps the canonical phases (local complementations
until none is left, then pivots) and reorders each round's candidates by
the network's scores:
* an LC round lists its candidate spiders (ascending) and takes them in
  priority order, each unless adjacent to one taken before;
* a pivot round lists the candidate edges u < v between Pauli spiders in
  lexicographic order, at most list_cap(n) of them, takes them in priority
  order, each unless an end is taken or adjacent to a taken end, and then
  completes the round with the canonical lexicographic pass over what is
  left (so the round is maximal even when the list was cut short).

Everything here is written with plain Python loops over an oracle ``Graph``.
"""
from __future__ import annotations

import numpy as np

from . import OK, Graph


def lc_candidates(g: Graph):
    """Interior present spiders with phase pi/2 or 3pi/2, ascending."""
    return [u for u in range(g.n) if g.is_alive(u) and not g.has_boundary(u) and g.k[u] % 4 == 2]


def pauli_candidates(g: Graph):
    return [u for u in range(g.n) if g.is_alive(u) and not g.has_boundary(u) and g.k[u] % 4 == 0]


def list_cap(n: int) -> int:
    """Length of a round's candidate list: the least power of two >= max(64, n)."""
    c = 64
    while c < n:
        c *= 2
    return c


def pivot_edges(g: Graph):
    """Edges (u, v), u < v, between Pauli candidates, lexicographic, at most
    list_cap(n) of them."""
    P = pauli_candidates(g)
    edges = []
    for i, u in enumerate(P):
        for v in P[i + 1:]:
            if g.edge(u, v):
                edges.append((u, v))
    return edges[: list_cap(g.n)]


def candidate_list(g: Graph):
    """The candidates of the next round as the learned schedule lists them:
    (u, -1) for the LC candidates, ascending, while there are any; then the
    pivot edges (u, v)."""
    lc = lc_candidates(g)
    if lc:
        return [(u, -1) for u in lc]
    return pivot_edges(g)


def neighbours(g: Graph, x):
    return [y for y in range(g.n) if g.edge(x, y)]


def endpoint_features(g: Graph, x, N):
    """Seven numbers (fp32 quotients): degree/N, phase class one-hot
    {k = 0 mod 4, k = 2 mod 4, k odd}, boundary-attached neighbours/N,
    spiders at distance exactly two/N, neighbours with k = 0 mod 4 / N."""
    nb = neighbours(g, x)
    two = set()
    for y in nb:
        for z in neighbours(g, y):
            if z != x and not g.edge(x, z):
                two.add(z)
    bnd = sum(1 for y in nb if g.has_boundary(y))
    pauli = sum(1 for y in nb if g.k[y] % 4 == 0)
    k = int(g.k[x])
    f32 = np.float32
    Nf = f32(N)
    return [f32(len(nb)) / Nf, f32(k % 4 == 0), f32(k % 4 == 2), f32(k % 2 == 1),
            f32(bnd) / Nf, f32(len(two)) / Nf, f32(pauli) / Nf]


def _entry(e):
    return (int(e), -1) if np.ndim(e) == 0 else (int(e[0]), int(e[1]))


def features(g: Graph, entry) -> np.ndarray:
    """The 16 features of a candidate as bf16 bit patterns (uint16): the seven
    endpoint features of u, those of v (zeros for an LC candidate), the rule
    bit (1 for a pivot), constant 1.  entry: u, (u, -1) or (u, v)."""
    from .mlp import bf16_round
    u, v = _entry(entry)
    N = max(1, len(g.alive_list()))
    f = endpoint_features(g, u, N)
    f += endpoint_features(g, v, N) if v >= 0 else [np.float32(0)] * 7
    f += [np.float32(1.0 if v >= 0 else 0.0), np.float32(1.0)]
    r = bf16_round(np.array(f, dtype=np.float32))
    return (r.view(np.uint32) >> 16).astype(np.uint16)


def gate2q(g: Graph) -> int:
    """Hadamard edges left plus the row additions of the output frontier."""
    if len(g.outputs):
        _, _, _, ops = g.frontier()
    else:
        ops = 0
    return g.n_edges() + ops


def rollout(state: Graph, entry):
    """Apply the candidate (LC at u, or the pivot on (u, v)), then the
    canonical schedule to the fixed point: (cost, fill-in added)."""
    g = state.copy()
    f0 = g.scalar.fill_in
    u, v = _entry(entry)
    rc = g.local_comp(u) if v < 0 else g.pivot(u, v)
    assert rc == OK, "candidate precondition failed"
    rc = g.simplify()
    assert rc == OK
    return gate2q(g), g.scalar.fill_in - f0


def lc_round_in_order(g: Graph, order):
    """An LC round that visits the candidates in the given order: each is
    taken unless adjacent to one taken before it."""
    taken = []
    for u in order:
        if not any(g.edge(u, t) for t in taken):
            taken.append(u)
    return taken


def pivot_round_in_order(g: Graph, order):
    """A pivot round that visits the listed edges in the given order, then
    completes it canonically: for each Pauli candidate u (ascending) whose
    end is free, the smallest free Pauli neighbour v > u.  An end is free
    when it is neither taken nor adjacent to a taken end.  Returns the pairs
    in the order taken."""
    blocked = set()
    pairs = []

    def take(u, v):
        pairs.append((u, v))
        blocked.update((u, v))
        blocked.update(y for y in range(g.n) if g.edge(u, y) or g.edge(v, y))

    for u, v in order:
        if u not in blocked and v not in blocked:
            take(u, v)
    P = pauli_candidates(g)
    for u in P:
        if u in blocked:
            continue
        for v in P:
            if v > u and v not in blocked and g.edge(u, v):
                take(u, v)
                break
    return pairs


def replay(g: Graph, trace) -> Graph:
    """Re-apply a trace (round, rule, u, v) in order with precondition checks;
    returns the final state.  Raises AssertionError on an invalid step or if
    a candidate remains at the end."""
    g = g.copy()
    for rnd, rule, u, v in np.asarray(trace).reshape(-1, 4):
        rc = g.local_comp(int(u)) if rule == 0 else g.pivot(int(u), int(v))
        assert rc == OK, "step (%d, %d, %d, %d) not applicable" % (rnd, rule, u, v)
    assert not lc_candidates(g), "LC candidate left"
    P = pauli_candidates(g)
    for i, u in enumerate(P):
        for w in P[i + 1:]:
            assert not g.edge(u, w), "pivot candidate left"
    return g


def round_is_valid(before: Graph, entries, pivot: bool) -> bool:
    """One round of a schedule: LC spiders pairwise non-adjacent and maximal
    among the candidates; pivot pairs disjoint, mutually non-adjacent, and
    maximal among the candidate edges."""
    if not pivot:
        sel = [u for u, _ in entries]
        for i, a in enumerate(sel):
            for b in sel[i + 1:]:
                if before.edge(a, b):
                    return False
        s = set(sel)
        for c in lc_candidates(before):
            if c not in s and not any(before.edge(c, x) for x in sel):
                return False
        return True
    ends = []
    for u, v in entries:
        for w in ends:
            if w in (u, v) or before.edge(u, w) or before.edge(v, w):
                return False
        ends += [u, v]
    # maximal: every candidate edge left out shares an end with, or is
    # adjacent to, an end already taken
    P = pauli_candidates(before)
    taken = set((min(u, v), max(u, v)) for u, v in entries)
    for i, u in enumerate(P):
        for v in P[i + 1:]:
            if not before.edge(u, v) or (u, v) in taken:
                continue
            if not any(w in (u, v) or before.edge(u, w) or before.edge(v, w) for w in ends):
                return False
    return True
