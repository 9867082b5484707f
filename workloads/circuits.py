"""Circuit-derived graph-like diagrams: random circuits of exponentiated
Pauli strings (the comparison workload of the paper's benchmark section:
20 qubits, Pauli strings of weight 2-4, depth 1-21), written out as
graph-like ZX diagrams.

Input generation only: this module turns a gate list into a diagram by the
textbook translation (Z rotations are Z spiders, Hadamards are Hadamard
edges, a CZ is a Hadamard edge, a Pauli exponential is a CNOT ladder around
a Z rotation between basis changes); it holds none of the rewriting,
elimination or extraction arithmetic.

Graph-like form is kept while the diagram is built: each qubit has a current
spider and a flag for a pending Hadamard on its wire.  A Z rotation on a wire
without a pending Hadamard adds to the current spider's phase (spider
fusion); otherwise it opens a new spider joined by a Hadamard edge.  Edges
are toggled, so parallel Hadamard edges cancel (up to a scalar, which the
tests ignore by comparing maps up to a scalar).
"""
from __future__ import annotations

import numpy as np

from .generators import Diagram, pack_rows
from .splitmix import draw, randint, stream_seed

P_CIRCUIT = 11


def pauli_exp_circuit(seed: int, item: int, n_qubits: int, depth: int, w_lo: int = 2, w_hi: int = 4):
    """``depth`` gates exp(-i k pi/8 P): P a Pauli string of weight
    U{w_lo..w_hi} on distinct qubits, each letter uniform over X, Y, Z;
    k uniform in 0..7.  Returns [(qubits, letters, k)]."""
    s = stream_seed(seed, item, P_CIRCUIT)
    h = draw(s, np.arange(depth * 16, dtype=np.uint64)).reshape(depth, 16)
    gates = []
    for g in range(depth):
        w = int(randint(h[g, 0], w_lo, min(w_hi, n_qubits)))
        qs = []
        t = 1
        while len(qs) < w:
            q = int(randint(h[g, t], 0, n_qubits - 1))
            t += 1
            if q not in qs:
                qs.append(q)
            if t >= 11:  # fall back to the lowest unused qubits
                for q in range(n_qubits):
                    if len(qs) < w and q not in qs:
                        qs.append(q)
        letters = ["XYZ"[(int(h[g, 11 + i]) >> 8) % 3] for i in range(w)]
        k = int(h[g, 15] & np.uint64(7))
        gates.append((qs, letters, k))
    return gates


class _Builder:
    def __init__(self, n_qubits):
        self.n_q = n_qubits
        self.phase = []
        self.edges = set()
        self.cur = []
        self.hpend = [0] * n_qubits
        self.inputs = []
        for q in range(n_qubits):
            v = self.spider(0)
            self.cur.append(v)
            self.inputs.append(v)

    def spider(self, k):
        self.phase.append(k % 8)
        return len(self.phase) - 1

    def toggle(self, a, b):
        e = (min(a, b), max(a, b))
        if e in self.edges:
            self.edges.remove(e)
        else:
            self.edges.add(e)

    def plain(self, q):
        """Make the wire of q end in a spider with no pending Hadamard."""
        if self.hpend[q]:
            w = self.spider(0)
            self.toggle(self.cur[q], w)
            self.cur[q] = w
            self.hpend[q] = 0

    def rz(self, q, k):
        self.plain(q)
        self.phase[self.cur[q]] = (self.phase[self.cur[q]] + k) % 8

    def had(self, q):
        self.hpend[q] ^= 1

    def cz(self, a, b):
        self.plain(a)
        self.plain(b)
        self.toggle(self.cur[a], self.cur[b])

    def cnot(self, c, t):
        self.had(t)
        self.cz(c, t)
        self.had(t)

    def finish(self):
        outs, bh_out = [], []
        for q in range(self.n_q):
            v = self.cur[q]
            if v in self.inputs or v in outs:
                # a spider may carry one boundary wire only: insert H H
                w = self.spider(0)
                self.toggle(v, w)
                self.cur[q] = w
                self.hpend[q] ^= 1
            outs.append(self.cur[q])
            bh_out.append(self.hpend[q])
        n = len(self.phase)
        bits = np.zeros((n, n), np.uint8)
        for a, b in self.edges:
            bits[a, b] = bits[b, a] = 1
        return Diagram(n=n, adj=pack_rows(bits), phase=np.array(self.phase, np.int8),
                       inputs=np.array(self.inputs, np.int32), outputs=np.array(outs, np.int32),
                       bnd_is_h=np.array([0] * self.n_q + bh_out, np.uint8))


def circuit_diagram(n_qubits: int, gates) -> Diagram:
    """Graph-like diagram of the gate list.  exp(-i k pi/8 P): X letters
    conjugated by H, Y letters by S^dag H before and H S after; the Z string
    as a CNOT ladder onto its last qubit, a Z rotation by k pi/4 there, and
    the ladder undone (so the diagram is built from H, Z rotations and CZ
    only, as a circuit is, and has a gflow).  A CNOT is H on the target
    around a CZ."""
    b = _Builder(n_qubits)
    for qs, letters, k in gates:
        for q, l in zip(qs, letters):
            if l == "Y":
                b.rz(q, 6)
            if l in "XY":
                b.had(q)
        last = qs[-1]
        for q in qs[:-1]:
            b.cnot(q, last)
        b.rz(last, k)
        for q in reversed(qs[:-1]):
            b.cnot(q, last)
        for q, l in zip(qs, letters):
            if l in "XY":
                b.had(q)
            if l == "Y":
                b.rz(q, 2)
    return b.finish()


def circuit_params(seed: int, item: int, q_lo: int = 4, q_hi: int = 20, d_lo: int = 1, d_hi: int = 21):
    """(qubits, depth) of item: uniform integers."""
    s = stream_seed(seed, item, P_CIRCUIT)
    h = draw(s, np.array([1 << 20, (1 << 20) + 1], dtype=np.uint64))
    return int(randint(h[0], q_lo, q_hi)), int(randint(h[1], d_lo, d_hi))


def circuit_workload(seed: int, item: int, **kw) -> Diagram:
    q, d = circuit_params(seed, item, **kw)
    return circuit_diagram(q, pauli_exp_circuit(seed, item, q, d))
