"""Pins of the oracle's flow check and circuit extraction.

* gflow: the layered check (Mhalla-Perdrix) against a brute-force search of
  the definition on tiny open graphs: a correction set g(u) of non-inputs for
  every non-output u, with u in Odd(g(u)), and an order in which every
  member of g(u) and of Odd(g(u)) - {u} comes after u (acyclicity of those
  relations);
* extraction: the extracted circuit's unitary equals, up to a scalar, the
  unitary of the generating circuit (a product of exp(-i k pi/8 P) computed
  with numpy) and the diagram's exact tensor (for the smallest cases), before
  and after simplification;
* diagrams without a gflow are refused by extraction.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle.extract import ExtractError, circuit_unitary, extract_circuit, gate_counts, gflow_layers
from oracle.tensor import evaluate_graph, to_complex
from workloads.circuits import circuit_diagram, pauli_exp_circuit
from workloads.generators import pack_rows

PX = np.array([[0, 1], [1, 0]], complex)
PY = np.array([[0, -1j], [1j, 0]])
PZ = np.diag([1, -1]).astype(complex)


def pauli_circuit_unitary(nq, gates):
    U = np.eye(2 ** nq, dtype=complex)
    for qs, letters, k in gates:
        mats = [np.eye(2, dtype=complex)] * nq
        for q, l in zip(qs, letters):
            mats[q] = {"X": PX, "Y": PY, "Z": PZ}[l]
        P = np.ones((1, 1), complex)
        for q in reversed(range(nq)):
            P = np.kron(P, mats[q])
        th = k * np.pi / 8
        U = (np.cos(th) * np.eye(2 ** nq) - 1j * np.sin(th) * P) @ U
    return U


def equal_up_to_scalar(U, V):
    i = np.unravel_index(np.argmax(abs(V)), V.shape)
    if abs(V[i]) < 1e-12:
        return np.allclose(U, 0)
    c = U[i] / V[i]
    return abs(c) > 1e-12 and np.allclose(U, c * V, atol=1e-8 * max(1.0, abs(c)))


def gflow_bruteforce(A, V, I, O):
    nonout = [u for u in V if u not in O]
    cand = [v for v in V if v not in I]
    options = []
    for u in nonout:
        opts = []
        for r in range(len(cand) + 1):
            for K in itertools.combinations(cand, r):
                odd = [w for w in V if sum(A[w, x] for x in K) % 2]
                if u not in odd:
                    continue
                after = set(K) | (set(odd) - {u})
                if u in after:
                    continue
                opts.append(after)
        if not opts:
            return False
        options.append(opts)
    for choice in itertools.product(*options):
        succ = {u: s for u, s in zip(nonout, choice)}
        # acyclic "u before s" relation
        state = {}

        def cyc(x):
            if state.get(x) == 1:
                return True
            if state.get(x) == 2:
                return False
            state[x] = 1
            for y in succ.get(x, ()):
                if cyc(y):
                    return True
            state[x] = 2
            return False
        if not any(cyc(u) for u in nonout):
            return True
    return False


@pytest.mark.parametrize("seed", range(40))
def test_gflow_matches_bruteforce(seed):
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(2, 6))
    bits = np.triu((rng.random((n, n)) < [0.3, 0.5, 0.7][seed % 3]).astype(np.uint8), 1)
    bits = bits + bits.T
    perm = rng.permutation(n)
    n_out = int(rng.integers(1, n + 1))
    n_in = int(rng.integers(0, n - n_out + 1))
    outs, ins = perm[:n_out], perm[n_out:n_out + n_in]
    g = oracle.Graph(n, pack_rows(bits), np.zeros(n, np.int8), ins, outs)
    exists, layer = gflow_layers(g)
    assert exists == gflow_bruteforce(bits, list(range(n)), set(map(int, ins)), set(map(int, outs)))
    if exists:
        assert (layer >= 0).all() and all(layer[int(o)] == 0 for o in outs)


@pytest.mark.parametrize("seed", range(30))
def test_extraction_reproduces_the_circuit(seed):
    nq = [2, 3, 4, 5, 6][seed % 5]
    depth = 1 + seed % 9
    gates = pauli_exp_circuit(seed, 7, nq, depth)
    d = circuit_diagram(nq, gates)
    U0 = pauli_circuit_unitary(nq, gates)
    for simplify in (False, True):
        g = oracle.Graph.from_diagram(d)
        if simplify:
            assert g.simplify() == oracle.OK
        assert gflow_layers(g)[0]
        ex, perm, in_h = extract_circuit(g)
        assert equal_up_to_scalar(circuit_unitary(nq, ex, perm, in_h), U0), (seed, simplify)
        c = gate_counts(ex)
        assert c["two_qubit"] == c["CZ"] + c["CNOT"]


@pytest.mark.parametrize("seed", range(8))
def test_extraction_equals_tensor(seed):
    """Independent of the generator's circuit: the diagram's exact tensor."""
    nq = 2 + seed % 2
    d = circuit_diagram(nq, pauli_exp_circuit(seed, 8, nq, 1 + seed % 3))
    g = oracle.Graph.from_diagram(d)
    assert g.simplify() == oracle.OK
    T = to_complex(evaluate_graph(g))
    ex, perm, in_h = extract_circuit(g)
    assert equal_up_to_scalar(circuit_unitary(nq, ex, perm, in_h), T.reshape(2 ** nq, 2 ** nq))


def test_no_gflow_is_refused():
    from workloads import batch_diagram
    refused = 0
    for i in range(20):
        g = oracle.Graph.from_diagram(batch_diagram(88, i, q_lo=2, q_hi=4))
        exists, _ = gflow_layers(g)
        if not exists:
            with pytest.raises(ExtractError):
                extract_circuit(g)
            refused += 1
    assert refused > 0
