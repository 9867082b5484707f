"""Reference of flow checks and circuit extraction on graph-like diagrams.

TEST INFRASTRUCTURE ONLY (imported by ``tests/`` and the CPU-baseline leg of
``bench.py``).

The paper simplifies diagrams and eliminates binary matrices over F2 but does
not spell out extraction or flow checking; both are the standard published
procedures, restated here from their definitions on the dense 0/1 adjacency,
with every elimination done by the pinned ``oracle.gf2_rref``:

* generalised flow (Mhalla and Perdrix, ICALP 2008): with outputs O and
  inputs I, vertices are processed in layers.  A vertex u not yet processed
  joins the next layer when some set K of processed non-input vertices has
  Odd(K) restricted to the unprocessed vertices equal to {u}.  The sets
  reachable as Odd(K) restricted to the unprocessed vertices are the row
  space of the correctors' adjacency rows restricted to those columns, and
  e_u lies in a row space exactly when the reduced row echelon form holds
  the row e_u.  A gflow exists when every vertex gets a layer.
* extraction (Backens, Miller-Bakewell, de Felice, Lobski, van de Wetering,
  "There and back again", Quantum 2021): from the outputs inwards, take the
  phases of the frontier spiders as Z rotations and their mutual edges as CZ
  gates, reduce the biadjacency between the frontier and its other
  neighbours by Gauss-Jordan elimination (every row addition is a CNOT and
  is applied to the graph), and move the frontier through each row left
  with a single 1 (a Hadamard gate); at the end the frontier is the input
  spiders, a permutation of the inputs.  Every input is first unfused into
  two phase-free spiders joined by Hadamard edges (an identity), so that the
  input spiders carry nothing but their wire.
"""
from __future__ import annotations

import numpy as np

from . import gf2_rref
from .tensor import evaluate  # noqa: F401  (tests compare with it)


def _pack(rows01: np.ndarray) -> np.ndarray:
    r, c = rows01.shape
    w = max(1, (c + 63) // 64)
    out = np.zeros((r, w), np.uint64)
    for i in range(r):
        for j in np.nonzero(rows01[i])[0]:
            out[i, j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return out


def _unpack(words: np.ndarray, c: int) -> np.ndarray:
    out = np.zeros((words.shape[0], c), np.uint8)
    for i in range(words.shape[0]):
        for j in range(c):
            out[i, j] = (int(words[i, j // 64]) >> (j % 64)) & 1
    return out


def gflow_layers(g):
    """(exists, layer): layer[v] = 0 for outputs, k >= 1 for the k-th layer
    found, -1 for spiders that get none (and for removed spiders)."""
    A = g.bits()
    V = g.alive_list()
    I = set(int(v) for v in g.inputs)
    layer = np.full(g.n, -1, np.int32)
    processed = set()
    correctors = []
    for v in g.outputs:
        v = int(v)
        layer[v] = 0
        processed.add(v)
        if v not in I:
            correctors.append(v)
    k = 1
    while True:
        U = [v for v in V if v not in processed]
        if not U or not correctors:
            break
        MT = A[np.ix_(correctors, U)]
        R, piv, rank, _ = gf2_rref(_pack(MT), len(U))
        Rb = _unpack(R[:rank], len(U))
        newly = [U[j] for j in range(len(U)) if any(Rb[i].sum() == 1 and Rb[i, j] for i in range(rank))]
        if not newly:
            break
        for u in newly:
            layer[u] = k
            processed.add(u)
            if u not in I:
                correctors.append(u)
        k += 1
    return len(processed) == len(V), layer


class ExtractError(Exception):
    pass


def extract_circuit(g):
    """Circuit of a diagram with gflow.  Returns (gates, perm, in_h):
    gates in extraction order (closest to the outputs first):
      ("H", q), ("RZ", q, k) (diag(1, omega^k)), ("CZ", a, b), ("CNOT", c, t);
    perm[q] = input wire that output qubit q starts from; in_h[i] = 1 for a
    Hadamard input wire.  The map is  U = G_1 G_2 ... G_m P_in  up to a
    scalar.  Raises ExtractError when no frontier row can be advanced."""
    n0 = g.n
    n_in = len(g.inputs)
    # Unfuse every input: input i -- a_i -H- b_i -H- v_i.  The phase-free
    # spider b_i between two Hadamard edges is a plain wire, and a_i then
    # fuses back into v_i, so the map is unchanged; the input spiders a_i
    # have the single neighbour b_i and are reached only at the very end.
    n = n0 + 2 * n_in
    A = np.zeros((n, n), np.uint8)
    A[:n0, :n0] = g.bits()
    k = np.zeros(n, np.int64)
    k[:n0] = g.k.astype(np.int64) % 8
    alive = set(g.alive_list())
    inputs = []
    for i, v in enumerate(g.inputs):
        a, b = n0 + 2 * i, n0 + 2 * i + 1
        A[a, b] = A[b, a] = A[b, int(v)] = A[int(v), b] = 1
        alive |= {a, b}
        inputs.append(a)
    in_of = {v: i for i, v in enumerate(inputs)}
    frontier = [int(v) for v in g.outputs]
    Q = len(frontier)
    gates = []
    for q in range(Q):
        if g.bnd_is_h[n_in + q]:
            gates.append(("H", q))
    while True:
        for q, v in enumerate(frontier):
            if k[v]:
                gates.append(("RZ", q, int(k[v])))
                k[v] = 0
        for a in range(Q):
            for b in range(a + 1, Q):
                if A[frontier[a], frontier[b]]:
                    gates.append(("CZ", a, b))
                    A[frontier[a], frontier[b]] = A[frontier[b], frontier[a]] = 0
        fset = set(frontier)
        N = sorted(set(int(w) for v in frontier for w in np.nonzero(A[v])[0]) - fset)
        if not N:
            break
        # Gauss-Jordan on the biadjacency between the frontier spiders that
        # are not input spiders (those qubits are finished) and N, with the
        # lowest-index pivot row; every row addition row_t += row_s is a
        # CNOT and is applied to the graph
        act = [q for q in range(Q) if frontier[q] not in in_of]
        B = A[np.ix_([frontier[q] for q in act], N)].copy()
        cur = 0
        for c in range(len(N)):
            if cur == len(act):
                break
            rows = [r for r in range(cur, len(act)) if B[r, c]]
            if not rows:
                continue
            r = rows[0]
            if r != cur:  # a swap is three row additions
                for t, s in ((cur, r), (r, cur), (cur, r)):
                    B[t] ^= B[s]
                    _row_add(A, gates, frontier, N, act[t], act[s])
            for t in range(len(act)):
                if t != cur and B[t, c]:
                    B[t] ^= B[cur]
                    _row_add(A, gates, frontier, N, act[t], act[cur])
            cur += 1
        progress = False
        for q in act:
            v = frontier[q]
            nb = [w for w in N if A[v, w]]
            if len(nb) == 1:
                w = nb[0]
                gates.append(("H", q))
                A[v, w] = A[w, v] = 0
                alive.discard(v)
                frontier[q] = w
                progress = True
        if not progress:
            raise ExtractError("no frontier row with a single neighbour")
    if alive != set(frontier):
        raise ExtractError("spiders left outside the frontier")
    perm = []
    for v in frontier:
        if v not in in_of:
            raise ExtractError("frontier spider %d carries no input" % v)
        perm.append(in_of[v])
    in_h = [int(x) for x in g.bnd_is_h[:n_in]]
    return gates, perm, in_h


def _row_add(A, gates, frontier, N, t, s):
    """row_t += row_s: the frontier spider of qubit t takes the symmetric
    difference of its neighbours in N with those of qubit s's spider."""
    vt, vs = frontier[t], frontier[s]
    for w in N:
        if A[vs, w]:
            A[vt, w] ^= 1
            A[w, vt] ^= 1
    gates.append(("CNOT", t, s))  # control t, target s


def gate_counts(gates):
    out = {"H": 0, "RZ": 0, "CZ": 0, "CNOT": 0}
    for gt in gates:
        out[gt[0]] += 1
    out["two_qubit"] = out["CZ"] + out["CNOT"]
    return out


# ---------------------------------------------------------------- unitary --
# Small circuits only (tests): complex matrices, qubit q = bit q of the index.

_H = np.array([[1, 1], [1, -1]], complex) / np.sqrt(2)


def _op1(nq, q, M):
    out = np.ones((1, 1), complex)
    for j in reversed(range(nq)):
        out = np.kron(out, M if j == q else np.eye(2))
    return out


def circuit_unitary(nq, gates, perm, in_h):
    """U = G_1 ... G_m P_in (output index bits = qubits)."""
    dim = 1 << nq
    P = np.zeros((dim, dim), complex)
    for x in range(dim):
        y = 0
        for q in range(nq):
            y |= ((x >> perm[q]) & 1) << q
        P[y, x] = 1
    for i, h in enumerate(in_h):
        if h:
            P = P @ _op1(nq, i, _H)
    U = np.eye(dim, dtype=complex)
    for gt in gates:
        if gt[0] == "H":
            G = _op1(nq, gt[1], _H)
        elif gt[0] == "RZ":
            G = _op1(nq, gt[1], np.diag([1, np.exp(1j * np.pi * gt[2] / 4)]))
        elif gt[0] == "CZ":
            d = np.ones(dim, complex)
            for x in range(dim):
                if (x >> gt[1]) & 1 and (x >> gt[2]) & 1:
                    d[x] = -1
            G = np.diag(d)
        else:
            c, t = gt[1], gt[2]
            G = np.zeros((dim, dim), complex)
            for x in range(dim):
                y = x ^ (((x >> c) & 1) << t)
                G[y, x] = 1
        U = U @ G
    return U @ P
