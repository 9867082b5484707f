"""CPU oracle for the bit-packed GF(2) ZX path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``; the product library never uses it.

``zx_oracle.c`` holds the rewrite rules, the simplification schedule, GF(2)
Gauss-Jordan elimination, frontier extraction and Pauli commutation as plain
single-threaded C.  ``tensor.py`` evaluates small diagrams exactly.
This module is a ctypes wrapper over numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMATCH = 0, -1, -2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Scalar(C.Structure):
    _fields_ = [("pow_sqrt2", C.c_int64), ("phase8", C.c_int32), ("pad", C.c_int32),
                ("fill_in", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("pw", C.c_int), ("rows", C.c_void_p), ("term_k", C.c_void_p), ("term_u", C.c_void_p),
                ("term_v", C.c_void_p), ("cap", C.c_int32), ("n_terms", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        PP = C.POINTER(Params)
        _lib.or_local_comp.argtypes = [C.c_int, C.c_int, P, P, P, P, C.c_int, C.c_int, C.POINTER(Scalar), PP]
        _lib.or_pivot.argtypes = [C.c_int, C.c_int, P, P, P, P, C.c_int, C.c_int, C.c_int, C.POINTER(Scalar),
                                  PP]
        _lib.or_simplify.argtypes = [C.c_int, C.c_int, P, P, P, P, C.POINTER(Scalar), P, C.c_int,
                                     C.POINTER(C.c_int), C.POINTER(C.c_int)]
        _lib.or_simplify_rounds.argtypes = [C.c_int, C.c_int, P, P, P, P, C.POINTER(Scalar), P, C.c_int,
                                            C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int, PP]
        _lib.or_gf2_rref.argtypes = [C.c_int, C.c_int, i64, P, P, C.POINTER(i32), C.POINTER(i64), P, i64]
        _lib.or_frontier.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, P, P, C.POINTER(i32), C.POINTER(i64)]
        _lib.or_pauli_commute.argtypes = [i64, C.c_int, P, P, i64, i64, i64, P, i64]
        _lib.or_pauli_commute.restype = None
        _lib.or_gf2_matmul.argtypes = [i64, i64, C.c_int, P, i64, P, i64, P, i64]
        _lib.or_gf2_matmul.restype = None
        _lib.or_gf2_rref_omp.argtypes = [C.c_int, C.c_int, i64, P, P, C.POINTER(i32)]
        _lib.or_detector_sample.argtypes = [C.c_int, C.c_int, P, P, P, C.c_uint64, i64, i64, P, i64]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def words_for(n: int) -> int:
    return (n + 63) // 64


class Graph:
    """Mutable graph-like diagram state held by the oracle (host numpy arrays)."""

    def __init__(self, n, adj, phase, inputs=(), outputs=(), bnd_is_h=None, params=None):
        """params: optional n x pw uint64 parameter rows (spider v's phase is
        k_v pi/4 + (params[v] . f) pi); terms recorded by rewrites are kept
        in term_k (m x 2: k_alpha, k_beta), term_u, term_v (m x pw)."""
        self.n = int(n)
        self.W = words_for(self.n)
        self.adj = np.ascontiguousarray(np.array(adj, dtype=np.uint64).reshape(self.n, self.W))
        self.k = np.ascontiguousarray(np.array(phase, dtype=np.int8) % 8).astype(np.int8)
        self.inputs = np.asarray(inputs, dtype=np.int32)
        self.outputs = np.asarray(outputs, dtype=np.int32)
        nb = len(self.inputs) + len(self.outputs)
        self.bnd_is_h = np.zeros(nb, np.uint8) if bnd_is_h is None else np.asarray(bnd_is_h, np.uint8)
        self.alive = np.zeros(self.W, dtype=np.uint64)
        for v in range(self.n):
            self.alive[v // 64] |= np.uint64(1) << np.uint64(v % 64)
        self.bnd = np.zeros(self.W, dtype=np.uint64)
        for v in list(self.inputs) + list(self.outputs):
            self.bnd[v // 64] |= np.uint64(1) << np.uint64(int(v) % 64)
        self.scalar = Scalar(0, 0, 0, 0)
        self.trace = np.zeros((0, 4), np.int32)
        self.rounds = 0
        if params is None:
            self.pw = 0
            self.params = np.zeros((self.n, 0), np.uint64)
        else:
            self.params = np.ascontiguousarray(np.array(params, dtype=np.uint64).reshape(self.n, -1))
            self.pw = self.params.shape[1]
        cap = self.n + 1
        self.term_k = np.zeros((cap, 2), np.int32)
        self.term_u = np.zeros((cap, max(self.pw, 1)), np.uint64)
        self.term_v = np.zeros((cap, max(self.pw, 1)), np.uint64)
        self.n_terms = 0

    def _par(self):
        if self.pw == 0:
            return None
        self._pstruct = Params(self.pw, self.params.ctypes.data, self.term_k.ctypes.data, self.term_u.ctypes.data,
                               self.term_v.ctypes.data, self.term_k.shape[0], self.n_terms)
        return C.byref(self._pstruct)

    def _par_done(self):
        if self.pw:
            self.n_terms = self._pstruct.n_terms

    def terms(self):
        """(k (m x 2), u (m x pw), v (m x pw)) of the terms recorded so far."""
        m = self.n_terms
        return self.term_k[:m].copy(), self.term_u[:m, : self.pw].copy(), self.term_v[:m, : self.pw].copy()

    @classmethod
    def from_diagram(cls, d):
        return cls(d.n, d.adj, d.phase, d.inputs, d.outputs, d.bnd_is_h)

    def copy(self):
        g = Graph.__new__(Graph)
        g.n, g.W = self.n, self.W
        g.adj, g.k = self.adj.copy(), self.k.copy()
        g.inputs, g.outputs, g.bnd_is_h = self.inputs.copy(), self.outputs.copy(), self.bnd_is_h.copy()
        g.alive, g.bnd = self.alive.copy(), self.bnd.copy()
        g.scalar = Scalar(self.scalar.pow_sqrt2, self.scalar.phase8, 0, self.scalar.fill_in)
        g.trace, g.rounds = self.trace.copy(), self.rounds
        g.pw, g.params = self.pw, self.params.copy()
        g.term_k, g.term_u, g.term_v = self.term_k.copy(), self.term_u.copy(), self.term_v.copy()
        g.n_terms = self.n_terms
        return g

    # -- queries --------------------------------------------------------
    def edge(self, x, y) -> bool:
        return bool((int(self.adj[x, y // 64]) >> (y % 64)) & 1)

    def is_alive(self, v) -> bool:
        return bool((int(self.alive[v // 64]) >> (v % 64)) & 1)

    def has_boundary(self, v) -> bool:
        return bool((int(self.bnd[v // 64]) >> (v % 64)) & 1)

    def bits(self) -> np.ndarray:
        by = self.adj.view(np.uint8).reshape(self.n, -1)
        return np.unpackbits(by, axis=1, bitorder="little")[:, : self.n]

    def alive_list(self):
        return [v for v in range(self.n) if self.is_alive(v)]

    def n_edges(self) -> int:
        return int(self.bits().sum()) // 2

    # -- rules ------------------------------------------------------------
    def local_comp(self, u, graph_only=False) -> int:
        par = self._par()
        rc = lib().or_local_comp(self.n, self.W, _p(self.adj), _p(self.k), _p(self.alive),
                                 _p(self.bnd), int(u), int(graph_only), C.byref(self.scalar), par)
        self._par_done()
        return rc

    def pivot(self, u, v, graph_only=False) -> int:
        par = self._par()
        rc = lib().or_pivot(self.n, self.W, _p(self.adj), _p(self.k), _p(self.alive),
                            _p(self.bnd), int(u), int(v), int(graph_only), C.byref(self.scalar), par)
        self._par_done()
        return rc

    def simplify(self, max_rounds: int = 0) -> int:
        """Canonical greedy schedule to the fixed point, or for max_rounds
        (> 0) rounds; the trace and round count of this call replace the
        previous ones."""
        cap = 2 * self.n + 2
        tr = np.zeros((cap, 4), np.int32)
        nt, nr = C.c_int(0), C.c_int(0)
        par = self._par()
        rc = lib().or_simplify_rounds(self.n, self.W, _p(self.adj), _p(self.k), _p(self.alive), _p(self.bnd),
                                      C.byref(self.scalar), _p(tr), cap, C.byref(nt), C.byref(nr),
                                      int(max_rounds), par)
        self._par_done()
        self.trace = tr[: nt.value].copy()
        self.rounds = nr.value
        return rc

    def frontier(self):
        """(M (q x W), pivots (q,), rank, rowops) of the output frontier."""
        q = len(self.outputs)
        M = np.zeros((q, self.W), np.uint64)
        piv = np.zeros(max(q, 1), np.int32)
        rank, ops = C.c_int32(0), C.c_int64(0)
        rc = lib().or_frontier(self.n, self.W, _p(self.adj), _p(self.alive),
                               _p(np.ascontiguousarray(self.outputs)), q, _p(M), _p(piv),
                               C.byref(rank), C.byref(ops))
        if rc != OK:
            raise ValueError("frontier failed %d" % rc)
        return M, piv[:q].copy(), rank.value, ops.value


def gf2_rref(A: np.ndarray, n_cols: int | None = None, want_T: bool = False):
    """Reduced row echelon form (copy).  Returns (R, pivots, rank, rowops[, T])."""
    A = np.array(A, dtype=np.uint64, copy=True, order="C")
    m, ld = A.shape
    n_cols = 64 * ld if n_cols is None else n_cols
    piv = np.zeros(max(m, 1), np.int32)
    rank, ops = C.c_int32(0), C.c_int64(0)
    ldt = words_for(m)
    T = np.zeros((m, max(ldt, 1)), np.uint64) if want_T else None
    rc = lib().or_gf2_rref(m, n_cols, ld, _p(A), _p(piv), C.byref(rank), C.byref(ops),
                           _p(T) if want_T else None, max(ldt, 1))
    if rc != OK:
        raise ValueError("rref failed %d" % rc)
    if want_T:
        return A, piv[:m].copy(), rank.value, ops.value, T
    return A, piv[:m].copy(), rank.value, ops.value


def pauli_commute(X: np.ndarray, Z: np.ndarray, rows=None, n_paulis: int | None = None,
                  Xall=None, Zall=None):
    """Commutation bits.  Default: full table of X/Z.  With ``rows`` = (i0, i1):
    rows i0..i1-1 of the table against all n strings."""
    X = np.ascontiguousarray(X, dtype=np.uint64)
    Z = np.ascontiguousarray(Z, dtype=np.uint64)
    n, w = X.shape
    i0, i1 = (0, n) if rows is None else rows
    ldc = words_for(n)
    out = np.zeros((i1 - i0, ldc), np.uint64)
    lib().or_pauli_commute(n, w, _p(X), _p(Z), w, i0, i1, _p(out), ldc)
    return out


def gf2_matmul(U: np.ndarray, F: np.ndarray, k_bits: int):
    """C[k][l] = parity of the first k_bits bits of U[k] & F[l] (m x ceil(n/64) words)."""
    U = np.ascontiguousarray(U, dtype=np.uint64)
    F = np.ascontiguousarray(F, dtype=np.uint64)
    m, n = U.shape[0], F.shape[0]
    ldc = max(1, words_for(n))
    out = np.zeros((m, ldc), np.uint64)
    lib().or_gf2_matmul(m, n, int(k_bits), _p(U), U.shape[1], _p(F), F.shape[1], _p(out), ldc)
    return out


def detector_sample(col_ptr, col_idx, prob, n_f: int, seed: int, shot0: int, n_shots: int):
    """Shots shot0 .. shot0 + n_shots - 1 of f = T e (rows of ceil(n_f/64) words)."""
    col_ptr = np.ascontiguousarray(col_ptr, np.int32)
    col_idx = np.ascontiguousarray(col_idx, np.int32)
    prob = np.ascontiguousarray(prob, np.float64)
    ldf = max(1, words_for(n_f))
    out = np.zeros((n_shots, ldf), np.uint64)
    rc = lib().or_detector_sample(len(prob), n_f, _p(col_ptr), _p(col_idx), _p(prob), int(seed) & (2**64 - 1),
                                  int(shot0), int(n_shots), _p(out), ldf)
    if rc != OK:
        raise ValueError("detector_sample failed %d" % rc)
    return out


def gf2_rref_threads(A: np.ndarray, n_cols: int):
    """The elimination with row additions spread over OpenMP threads (timing
    only).  Returns (R, pivots, rank)."""
    A = np.array(A, dtype=np.uint64, copy=True, order="C")
    m, ld = A.shape
    piv = np.zeros(max(m, 1), np.int32)
    rank = C.c_int32(0)
    rc = lib().or_gf2_rref_omp(m, n_cols, ld, _p(A), _p(piv), C.byref(rank))
    if rc != OK:
        raise ValueError("rref failed %d" % rc)
    return A, piv[:m].copy(), rank.value
