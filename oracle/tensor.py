"""Exact tensor evaluation of small graph-like ZX diagrams.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Semantics (appendix "ZX-Calculus", tensor definition of the Z spider and the
Hadamard edge): a Z spider with phase alpha is |0..0><0..0| + e^{i alpha}
|1..1><1..1|, i.e. all of its wires carry the same bit x_v and it contributes
e^{i alpha x_v}; a Hadamard edge between u and v contributes
H[x_u, x_v] = (-1)^{x_u x_v} / sqrt(2).  Contracting the diagram therefore
gives, for boundary bits b,

    M[b_out, b_in] = sum over x of  prod_v omega^{k_v x_v}
                     * prod_{uv in E} (-1)^{x_u x_v} / sqrt(2)
                     * prod_{Hadamard boundary wires (v, b)} (-1)^{x_v b} / sqrt(2)

with omega = e^{i pi/4} and phases alpha_v = k_v pi/4; a spider on a plain
boundary wire has x_v equal to that wire's bit.  Every term is a power of
omega, so M is computed exactly as an element of Z[omega] (coefficients of
1, omega, omega^2, omega^3, using omega^4 = -1) times a power of sqrt(2).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- Z[omega] --

def zw_from_hist(hist):
    """Histogram over omega^0..omega^7 -> Z[omega] coefficients (..., 4)."""
    hist = np.asarray(hist, dtype=object)
    return hist[..., 0:4] - hist[..., 4:8]


def zw_mul(a, b):
    """Product in Z[omega] (negacyclic convolution, omega^4 = -1); object ints."""
    a = np.asarray(a, dtype=object)
    b = np.asarray(b, dtype=object)
    out = np.zeros(np.broadcast_shapes(a.shape, b.shape), dtype=object)
    for i in range(4):
        for j in range(4):
            t = a[..., i] * b[..., j]
            if i + j < 4:
                out[..., i + j] += t
            else:
                out[..., i + j - 4] -= t
    return out


def zw_omega_pow(a, m):
    """a * omega^m."""
    a = np.asarray(a, dtype=object)
    m %= 8
    out = a.copy()
    for _ in range(m):
        out = np.concatenate([-out[..., 3:4], out[..., 0:3]], axis=-1)
    return out


SQRT2 = np.array([0, 1, 0, -1], dtype=object)  # omega - omega^3 = sqrt(2)


def zw_sqrt2_pow(a, d):
    """a * sqrt(2)^d for d >= 0."""
    assert d >= 0
    a = np.asarray(a, dtype=object) * (2 ** (d // 2))
    if d % 2:
        a = zw_mul(a, SQRT2)
    return a


class Amp:
    """Exact linear map  omega^phase * sqrt(2)^pow * M,  M in Z[omega]^(2^out x 2^in)."""

    def __init__(self, M, pow_sqrt2, phase8):
        self.M = np.asarray(M, dtype=object)
        self.pow = int(pow_sqrt2)
        self.phase = int(phase8) % 8

    def normalized(self, pow_floor):
        """M * omega^phase * sqrt(2)^(pow - pow_floor), pow_floor <= pow."""
        return zw_sqrt2_pow(zw_omega_pow(self.M, self.phase), self.pow - pow_floor)

    def equals(self, other) -> bool:
        if self.M.shape != other.M.shape:
            return False
        lo = min(self.pow, other.pow)
        return bool(np.all(self.normalized(lo) == other.normalized(lo)))

    def equals_up_to_scalar(self, other) -> bool:
        if self.M.shape != other.M.shape:
            return False
        a = self.M.reshape(-1, 4)
        b = other.M.reshape(-1, 4)
        za = np.all(a == 0, axis=1)
        zb = np.all(b == 0, axis=1)
        if not np.array_equal(za, zb):
            return False
        if za.all():
            return True
        i0 = int(np.argmin(za))
        # a[x] * b[i0] == b[x] * a[i0] for all x
        return bool(np.all(zw_mul(a, b[i0]) == zw_mul(b, a[i0])))

    def is_zero(self) -> bool:
        return bool(np.all(self.M == 0))


def omega_power_value(m: int) -> complex:
    return complex(np.exp(1j * np.pi * m / 4))


def to_complex(amp: Amp) -> np.ndarray:
    """Floating-point view (for diagnostics only)."""
    w = np.exp(1j * np.pi / 4)
    M = amp.M.astype(np.float64)
    vals = M[..., 0] + M[..., 1] * w + M[..., 2] * w ** 2 + M[..., 3] * w ** 3
    return vals * (w ** amp.phase) * (np.sqrt(2.0) ** amp.pow)


# ----------------------------------------------------------- evaluation --

def evaluate(n, edges_bits, phase, alive, inputs, outputs, bnd_is_h, pow_sqrt2=0, phase8=0,
             max_free=24) -> Amp:
    """Exact linear map of a graph-like diagram.

    edges_bits: (n, n) 0/1 symmetric matrix; phase: k per spider (pi/4 units);
    alive: iterable of present spiders; inputs/outputs: spider ids of the
    boundary wires in order; bnd_is_h: per wire (inputs then outputs), 1 for a
    Hadamard wire.  Output index = sum_j b_out[j] 2^j, input index likewise.
    """
    alive = sorted(int(v) for v in alive)
    aset = set(alive)
    wires = [(int(v), int(h), "in", j) for j, (v, h) in enumerate(zip(inputs, bnd_is_h[: len(inputs)]))]
    wires += [(int(v), int(h), "out", j) for j, (v, h) in enumerate(zip(outputs, bnd_is_h[len(inputs):]))]
    for v, _, _, _ in wires:
        if v not in aset:
            raise ValueError("boundary wire on a removed spider")
    plain = {}
    for v, h, side, j in wires:
        if not h:
            plain.setdefault(v, []).append((side, j))
    free = [v for v in alive if v not in plain]
    fixed = [v for v in alive if v in plain]
    F = len(free)
    if F > max_free:
        raise ValueError("too many free spiders for brute force")
    fidx = {v: i for i, v in enumerate(free)}
    E = np.asarray(edges_bits, dtype=np.int64)
    edges = [(u, v) for u in alive for v in alive if u < v and E[u, v]]
    n_h_wires = sum(1 for _, h, _, _ in wires if h)

    t = np.arange(1 << F, dtype=np.int64)
    xbit = [(t >> i) & 1 for i in range(F)]
    base = np.zeros(1 << F, dtype=np.int64)
    for v in free:
        base += int(phase[v]) * xbit[fidx[v]]
    for u, v in edges:
        if u in fidx and v in fidx:
            base += 4 * (xbit[fidx[u]] & xbit[fidx[v]])

    n_in, n_out = len(inputs), len(outputs)
    M = np.zeros((1 << n_out, 1 << n_in, 4), dtype=object)
    for bo in range(1 << n_out):
        for bi in range(1 << n_in):
            bits = {"in": [(bi >> j) & 1 for j in range(n_in)], "out": [(bo >> j) & 1 for j in range(n_out)]}
            xfix = {}
            ok = True
            for v in fixed:
                vals = {bits[s][j] for s, j in plain[v]}
                if len(vals) > 1:
                    ok = False
                    break
                xfix[v] = vals.pop()
            if not ok:
                continue
            const = 0
            lin = np.zeros(F, dtype=np.int64)  # coefficient (mod 8) of x_free
            for v in fixed:
                const += int(phase[v]) * xfix[v]
            for u, v in edges:
                if u in xfix and v in xfix:
                    const += 4 * xfix[u] * xfix[v]
                elif u in xfix and v in fidx:
                    lin[fidx[v]] += 4 * xfix[u]
                elif v in xfix and u in fidx:
                    lin[fidx[u]] += 4 * xfix[v]
            for v, h, side, j in wires:
                if h:
                    b = bits[side][j]
                    if v in xfix:
                        const += 4 * xfix[v] * b
                    else:
                        lin[fidx[v]] += 4 * b
            e = base + const
            for i in range(F):
                if lin[i] % 8:
                    e = e + (lin[i] % 8) * xbit[i]
            hist = np.bincount(e % 8, minlength=8)
            M[bo, bi] = zw_from_hist(hist)
    return Amp(M, pow_sqrt2 - len(edges) - n_h_wires, phase8)


def evaluate_graph(g) -> Amp:
    """Exact map of an ``oracle.Graph`` including its tracked scalar."""
    return evaluate(g.n, g.bits(), g.k, g.alive_list(), g.inputs, g.outputs, g.bnd_is_h,
                    g.scalar.pow_sqrt2, g.scalar.phase8)
