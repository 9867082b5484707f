"""Seeded synthetic workloads: graph-like ZX diagrams, GF(2) matrices, Pauli strings.

Every value is a SplitMix64 draw (see ``splitmix``) from a stream identified by
(workload seed, item id, purpose), so any diagram or matrix row can be rebuilt
on its own.  The shapes follow the workloads of the build:

* one diagram: 8 qubits, 64 spiders, Erdos-Renyi Hadamard edges p = 0.1,
  phases k*pi/4 with k uniform in 0..7, 8 inputs / 8 outputs;
* batched diagrams: qubits q ~ U{4..64}, spiders N = q * U{4..16},
  edge density p ~ U[0.05, 0.3];
* dense GF(2) matrix: Bernoulli(1/2) bits;
* Pauli strings: X and Z bit vectors, each bit Bernoulli(1/2), which makes
  every qubit uniform over I/X/Y/Z under the (x, z) encoding.

Layout conventions shared by both sides of every test:

* adjacency: N x W uint64, W = ceil(N/64), bit c of row r is word c//64,
  bit c%64; symmetric, zero diagonal;
* boundary: input i attached to spider i, output j to spider N - q + j, both by
  plain (non-Hadamard) wires; boundary vertices are not rows of the matrix.

This module contains no ZX-rule or elimination arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .splitmix import bernoulli_threshold, draw, randint, stream_seed, unit

# stream purposes
P_PARAMS = 0
P_EDGES = 1
P_PHASES = 2
P_MATRIX = 3
P_PAULI = 4
P_ARRIVAL = 5
P_WEIGHTS = 6
P_SERVE = 7
P_PARITY = 8
P_DEM = 9
P_PROWS = 10


@dataclass
class Diagram:
    """A graph-like ZX diagram in bit-packed form (host arrays)."""

    n: int  # spiders
    adj: np.ndarray  # (n, W) uint64
    phase: np.ndarray  # (n,) int8, units of pi/4, 0..7
    inputs: np.ndarray  # (q_in,) int32 spider ids
    outputs: np.ndarray  # (q_out,) int32 spider ids
    bnd_is_h: np.ndarray  # (q_in + q_out,) uint8, 1 = Hadamard boundary wire

    @property
    def words(self) -> int:
        return (self.n + 63) // 64

    @property
    def qubits(self) -> int:
        return int(len(self.outputs))


def words_for(n: int) -> int:
    return (n + 63) // 64


def pack_rows(bits: np.ndarray) -> np.ndarray:
    """(r, c) bool -> (r, ceil(c/64)) uint64, bit c%64 of word c//64."""
    r, c = bits.shape
    w = words_for(c)
    padded = np.zeros((r, w * 64), dtype=np.uint8)
    padded[:, :c] = bits
    by = np.packbits(padded, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8").reshape(r, w).astype(np.uint64)


def unpack_rows(words: np.ndarray, c: int) -> np.ndarray:
    """(r, W) uint64 -> (r, c) uint8 bits."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    by = words.view(np.uint8).reshape(words.shape[0], -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :c]


def er_adjacency(seed: int, item: int, n: int, p: float) -> np.ndarray:
    """Symmetric ER adjacency, pair (i<j) -> draw index j(j-1)/2 + i."""
    s = stream_seed(seed, item, P_EDGES)
    thr = bernoulli_threshold(p)
    bits = np.zeros((n, n), dtype=np.uint8)
    # generate row by row blocks of j to bound memory
    j0 = 1
    while j0 < n:
        j1 = min(n, j0 + max(1, (1 << 22) // max(1, j0)))
        js = np.arange(j0, j1, dtype=np.int64)
        counts = js  # pairs (i, j) for i < j
        base = js * (js - 1) // 2
        tot = int(counts.sum())
        jj = np.repeat(js, counts)
        ii = np.arange(tot, dtype=np.int64) - np.repeat(np.cumsum(counts) - counts, counts)
        t = np.repeat(base, counts) + ii
        e = (draw(s, t.astype(np.uint64)) >> np.uint64(11)) < thr
        bits[ii[e], jj[e]] = 1
        bits[jj[e], ii[e]] = 1
        j0 = j1
    return pack_rows(bits)


def phases(seed: int, item: int, n: int) -> np.ndarray:
    s = stream_seed(seed, item, P_PHASES)
    return (draw(s, np.arange(n, dtype=np.uint64)) & np.uint64(7)).astype(np.int8)


def make_diagram(seed: int, item: int, q: int, n: int, p: float) -> Diagram:
    if n < 2 * q:
        raise ValueError("need at least 2q spiders")
    adj = er_adjacency(seed, item, n, p)
    ph = phases(seed, item, n)
    inputs = np.arange(q, dtype=np.int32)
    outputs = (n - q + np.arange(q)).astype(np.int32)
    return Diagram(n=n, adj=adj, phase=ph, inputs=inputs, outputs=outputs,
                   bnd_is_h=np.zeros(2 * q, dtype=np.uint8))


# --- workload recipes ------------------------------------------------------

def single_diagram(seed: int) -> Diagram:
    """8 qubits, 64 spiders, ER p = 0.1 (one-diagram workload, seeds 1..1000)."""
    return make_diagram(seed, 0, 8, 64, 0.1)


def batch_params(seed: int, item: int, q_lo=4, q_hi=64, m_lo=4, m_hi=16,
                 p_lo=0.05, p_hi=0.3):
    """(q, N, p) of diagram ``item`` of a batched workload."""
    s = stream_seed(seed, item, P_PARAMS)
    h = draw(s, np.arange(3, dtype=np.uint64))
    q = int(randint(h[0], q_lo, q_hi))
    mult = int(randint(h[1], m_lo, m_hi))
    p = p_lo + (p_hi - p_lo) * float(unit(h[2]))
    return q, q * mult, p


def batch_diagram(seed: int, item: int, **kw) -> Diagram:
    q, n, p = batch_params(seed, item, **kw)
    return make_diagram(seed, item, q, n, p)


def bernoulli_matrix(seed: int, m: int, n_cols: int, ld: int | None = None) -> np.ndarray:
    """m x ld uint64 words of Bernoulli(1/2) bits; bits >= n_cols are zero."""
    w = words_for(n_cols)
    ld = w if ld is None else ld
    s = stream_seed(seed, 0, P_MATRIX)
    t = (np.arange(m, dtype=np.uint64)[:, None] * np.uint64(w)
         + np.arange(w, dtype=np.uint64)[None, :])
    a = np.zeros((m, ld), dtype=np.uint64)
    a[:, :w] = draw(s, t)
    tail = n_cols - 64 * (w - 1)
    if tail < 64:
        a[:, w - 1] &= np.uint64((1 << tail) - 1)
    return a


def bernoulli_rows(seed: int, rows: np.ndarray, n_cols: int) -> np.ndarray:
    """Selected rows of ``bernoulli_matrix`` without building the whole matrix."""
    w = words_for(n_cols)
    s = stream_seed(seed, 0, P_MATRIX)
    t = (np.asarray(rows, dtype=np.uint64)[:, None] * np.uint64(w)
         + np.arange(w, dtype=np.uint64)[None, :])
    a = draw(s, t)
    tail = n_cols - 64 * (w - 1)
    if tail < 64:
        a[:, w - 1] &= np.uint64((1 << tail) - 1)
    return a


def pauli_strings(seed: int, n_paulis: int, n_qubits: int, rows=None):
    """X, Z words ((n, ceil(q/64)) uint64 each); x word = draw(2t), z = draw(2t+1),
    t = i * W + w.  ``rows`` selects a subset of Pauli indices."""
    w = words_for(n_qubits)
    s = stream_seed(seed, 0, P_PAULI)
    idx = np.arange(n_paulis, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    t = idx[:, None] * np.uint64(w) + np.arange(w, dtype=np.uint64)[None, :]
    x = draw(s, np.uint64(2) * t)
    z = draw(s, np.uint64(2) * t + np.uint64(1))
    tail = n_qubits - 64 * (w - 1)
    if tail < 64:
        msk = np.uint64((1 << tail) - 1)
        x[:, w - 1] &= msk
        z[:, w - 1] &= msk
    return x, z


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential gaps, inverse CDF."""
    s = stream_seed(seed, 0, P_ARRIVAL)
    u = unit(draw(s, np.arange(count, dtype=np.uint64)))
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


def network_init(seed: int, n_in: int = 16, n_hid: int = 256) -> np.ndarray:
    """fp32 parameter vector W1[n_in][n_hid] | b1 | w2 | b2: weights uniform
    in +-sqrt(6 / (fan_in + fan_out)), biases zero."""
    s = stream_seed(seed, 0, P_WEIGHTS)
    n1, n2 = n_in * n_hid, n_hid
    u = unit(draw(s, np.arange(n1 + n2, dtype=np.uint64))) * 2.0 - 1.0
    p = np.zeros(n1 + 2 * n_hid + 1, np.float32)
    p[:n1] = u[:n1] * np.sqrt(6.0 / (n_in + n_hid))
    p[n1 + n_hid:n1 + 2 * n_hid] = u[n1:] * np.sqrt(6.0 / (n_hid + 1))
    return p


def serve_params(seed: int, item: int, q_lo: int = 8, q_hi: int = 512, m_lo: int = 4, m_hi: int = 16,
                 p_lo: float = 0.05, p_hi: float = 0.3):
    """(q, N, p) of request ``item`` of a serving stream: q = round(exp(U[ln
    q_lo, ln q_hi])), N = q * U{m_lo..m_hi}, p ~ U[p_lo, p_hi]."""
    s = stream_seed(seed, item, P_SERVE)
    h = draw(s, np.arange(3, dtype=np.uint64))
    q = int(round(float(np.exp(np.log(q_lo) + (np.log(q_hi) - np.log(q_lo)) * float(unit(h[0]))))))
    mult = int(randint(h[1], m_lo, m_hi))
    p = p_lo + (p_hi - p_lo) * float(unit(h[2]))
    return q, q * mult, p


def serve_diagram(seed: int, item: int, **kw) -> Diagram:
    q, n, p = serve_params(seed, item, **kw)
    return make_diagram(seed, item, q, n, p)


@dataclass
class ParityProblem:
    """Inputs of the batched phase-pair evaluation: term selectors U, V
    (n_terms x n_params bits), parameter settings F (n_settings x n_params
    bits, one row per setting) and the terms' phase codes (multiples of pi/4)."""

    n_params: int
    U: np.ndarray
    V: np.ndarray
    F: np.ndarray
    k_alpha: np.ndarray
    k_beta: np.ndarray


def _bits(seed: int, purpose_item: int, rows: int, cols: int, p: float) -> np.ndarray:
    """rows x ceil(cols/64) words of Bernoulli(p) bits (bit = draw < p 2^53)."""
    s = stream_seed(seed, purpose_item, P_PARITY)
    w = words_for(cols)
    out = np.zeros((rows, w), np.uint64)
    thr = bernoulli_threshold(p)
    step = max(1, (1 << 22) // max(1, cols))
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        t = (np.arange(r0, r1, dtype=np.uint64)[:, None] * np.uint64(cols)
             + np.arange(cols, dtype=np.uint64)[None, :])
        b = ((draw(s, t) >> np.uint64(11)) < thr).astype(np.uint8)
        out[r0:r1] = pack_rows(b)
    return out


def parity_problem(seed: int, n_terms: int, n_settings: int, n_params: int,
                   p_select: float = 1.0 / 16, p_setting: float = 0.5,
                   any_phase: bool = False) -> ParityProblem:
    """Selectors Bernoulli(p_select) (a parity touches n_params * p_select
    parameters on average), settings Bernoulli(p_setting).  Terms are of the
    two kinds the rewrite rules produce, half each: half-pi terms
    (k_alpha in {0, 4}, k_beta = 2, no second parity: V row zero) and pi-pair
    terms (k_alpha, k_beta in {0, 4}); with any_phase, phase codes uniform in
    0..7 instead."""
    U = _bits(seed, 0, n_terms, n_params, p_select)
    V = _bits(seed, 1, n_terms, n_params, p_select)
    F = _bits(seed, 2, n_settings, n_params, p_setting)
    s = stream_seed(seed, 3, P_PARITY)
    h = draw(s, np.arange(3 * n_terms, dtype=np.uint64))
    if any_phase:
        ka = (h[:n_terms] & np.uint64(7)).astype(np.int8)
        kb = (h[n_terms:2 * n_terms] & np.uint64(7)).astype(np.int8)
    else:
        half = (h[2 * n_terms:] & np.uint64(1)).astype(bool)
        ka = (4 * (h[:n_terms] & np.uint64(1))).astype(np.int8)
        kb = np.where(half, 2, 4 * (h[n_terms:2 * n_terms] & np.uint64(1))).astype(np.int8)
        V[half] = 0
    return ParityProblem(n_params, U, V, F, ka, kb)


@dataclass
class DetectorModel:
    """Binary matrix T of the sampling step (f = T e): column j lists the f
    bits (detectors, then the observable) flipped by error mechanism j,
    CSC arrays; prob[j] is the mechanism's firing probability."""

    n_f: int
    n_det: int
    col_ptr: np.ndarray  # int32 [n_err + 1]
    col_idx: np.ndarray  # int32 [nnz]
    prob: np.ndarray     # float64 [n_err]

    @property
    def n_err(self) -> int:
        return len(self.prob)


def surface_dem(seed: int, d: int, rounds: int, p: float = 1e-3) -> DetectorModel:
    """Detector error model shaped like a distance-d rotated surface code
    memory experiment with ``rounds`` rounds: checks on an a x b grid,
    a = (d+1)/2, b = d-1 (a b = (d^2-1)/2 checks), detectors for rounds
    0..rounds (the last from the final data readout), one observable.
    Mechanisms per round r, in this order: horizontal neighbour pairs,
    vertical neighbour pairs, single checks on the two boundary columns
    (those on column 0 also flip the observable), then, for r < rounds,
    time-like pairs (check c in rounds r and r + 1) and diagonal pairs
    ((x, y, r), (x + 1, y + 1, r + 1)).  prob = p * U[0.5, 1.5] each."""
    a, b = (d + 1) // 2, d - 1
    K = a * b
    n_det = K * (rounds + 1)
    obs = n_det
    det = lambda x, y, r: r * K + x * b + y
    cols = []
    for r in range(rounds + 1):
        for x in range(a):
            for y in range(b - 1):
                cols.append([det(x, y, r), det(x, y + 1, r)])
        for x in range(a - 1):
            for y in range(b):
                cols.append([det(x, y, r), det(x + 1, y, r)])
        for x in range(a):
            cols.append([det(x, 0, r), obs])
            cols.append([det(x, b - 1, r)])
        if r < rounds:
            for c in range(K):
                cols.append([r * K + c, (r + 1) * K + c])
            for x in range(a - 1):
                for y in range(b - 1):
                    cols.append([det(x, y, r), det(x + 1, y + 1, r + 1)])
    col_ptr = np.zeros(len(cols) + 1, np.int32)
    col_ptr[1:] = np.cumsum([len(c) for c in cols])
    col_idx = np.array([i for c in cols for i in c], np.int32)
    s = stream_seed(seed, d * 1000 + rounds, P_DEM)
    u = unit(draw(s, np.arange(len(cols), dtype=np.uint64)))
    prob = p * (0.5 + u)
    return DetectorModel(n_det + 1, n_det, col_ptr, col_idx, prob.astype(np.float64))


def param_rows(seed: int, item: int, n: int, n_params: int, frac: float = 0.3, per: int = 2) -> np.ndarray:
    """Parameter rows of a diagram's spiders (n x ceil(n_params/64) words):
    each spider carries parameters with probability ``frac``, then ``per``
    parameter indices uniform in [0, n_params) (XORed, so a repeat cancels),
    as a Pauli noise location flips the phase of the spiders it touches."""
    pw = words_for(n_params)
    out = np.zeros((n, pw), np.uint64)
    if n_params == 0:
        return out
    s = stream_seed(seed, item, P_PROWS)
    h = draw(s, np.arange(n * (per + 1), dtype=np.uint64)).reshape(n, per + 1)
    thr = bernoulli_threshold(frac)
    for v in range(n):
        if (h[v, 0] >> np.uint64(11)) >= thr:
            continue
        for t in range(per):
            b = int((h[v, 1 + t] >> np.uint64(11)) % np.uint64(n_params))
            out[v, b // 64] ^= np.uint64(1) << np.uint64(b % 64)
    return out
