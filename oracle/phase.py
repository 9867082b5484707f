"""Reference of the phase-pair evaluation of parameterized Clifford diagrams.

TEST INFRASTRUCTURE ONLY (imported by ``tests/`` and the CPU-baseline leg of
``bench.py``); the product library never uses it.

Appendix "Parameterized evaluation of Clifford ZX diagrams": after reduction
the diagram's amplitude is c * prod_k h(alpha_k, beta_k; a_k, b_k) with
  h(alpha, beta; a, b) = 1 + e^{i(alpha + a pi)} + e^{i(beta + b pi)}
                           - e^{i(alpha + beta + a pi + b pi)}   (eq. phase_pair)
and a_k, b_k parities of the parameters (eq. parities; ``oracle.gf2_matmul``).
Phases here are multiples of pi/4 (integer codes k, phase k pi/4), as every
phase of this library; c = omega^phase8 * sqrt(2)^pow_sqrt2, omega = e^{i pi/4}.

Results are (mantissa, exponent) pairs, value = mantissa * 2^exponent, with
the mantissa's larger component in [0.5, 1) (or exactly zero), so that long
products neither overflow nor underflow.  Arithmetic is complex fp64.

``exact_*`` evaluate the same products exactly in Z[omega] with Python
integers (small cases only): they pin the floating-point reference.
"""
from __future__ import annotations

import math

import numpy as np


_R = math.sqrt(0.5)
# e^{i k pi/4} for k = 0..7, with the exact values 0 and +-1 where they occur
_OMEGA = [complex(1, 0), complex(_R, _R), complex(0, 1), complex(-_R, _R),
          complex(-1, 0), complex(-_R, -_R), complex(0, -1), complex(_R, -_R)]


def omega_pow(k: int) -> complex:
    """e^{i k pi / 4} in fp64 (cos and sin of multiples of pi/4)."""
    return _OMEGA[int(k) % 8]


def h_value(ka: int, kb: int, a: int, b: int) -> complex:
    """Equation phase_pair with alpha = ka pi/4, beta = kb pi/4."""
    x = omega_pow(ka + 4 * a)
    y = omega_pow(kb + 4 * b)
    return 1 + x + y - omega_pow(ka + kb + 4 * a + 4 * b)


def normalise(z: complex, e: int):
    """(mantissa, exponent) with max(|re|, |im|) in [0.5, 1), or (0, 0)."""
    m = max(abs(z.real), abs(z.imag))
    if m == 0.0:
        return 0j, 0
    _, ex = math.frexp(m)
    return complex(math.ldexp(z.real, -ex), math.ldexp(z.imag, -ex)), e + ex


def bit(row: np.ndarray, j: int) -> int:
    return int((int(row[j // 64]) >> (j % 64)) & 1)


def phase_pair_product(A: np.ndarray, B: np.ndarray, ka, kb, n_shots: int, phase8: int = 0,
                       pow_sqrt2: int = 0):
    """Per shot l: c * prod_k h(ka_k, kb_k; A[k][l], B[k][l]).

    A, B: m x ceil(n_shots/64) words (bit l of row k = a_kl, b_kl).
    Returns (complex128 mantissas, int64 exponents), one per shot."""
    m = len(ka)
    table = [[h_value(int(ka[k]), int(kb[k]), a, b) for b in (0, 1) for a in (0, 1)] for k in range(m)]
    c = omega_pow(phase8)
    c0, e0 = normalise(c * (math.sqrt(2.0) if pow_sqrt2 % 2 else 1.0), pow_sqrt2 // 2)
    mant = np.zeros(n_shots, np.complex128)
    expo = np.zeros(n_shots, np.int64)
    for l in range(n_shots):
        z, e = c0, e0
        for k in range(m):
            z, e = normalise(z * table[k][bit(A[k], l) + 2 * bit(B[k], l)], e)
        mant[l], expo[l] = z, e
    return mant, expo


# ---------------------------------------------------------------- exact --
# Elements of Z[omega] as 4-tuples (c0, c1, c2, c3): c0 + c1 w + c2 w^2 + c3 w^3,
# with w^4 = -1.

def zw_pow(k: int):
    k %= 8
    v = [0, 0, 0, 0]
    v[k % 4] = 1 if k < 4 else -1
    return tuple(v)


def zw_add(p, q):
    return tuple(a + b for a, b in zip(p, q))


def zw_neg(p):
    return tuple(-a for a in p)


def zw_mul(p, q):
    r = [0, 0, 0, 0]
    for i in range(4):
        for j in range(4):
            t = p[i] * q[j]
            if i + j < 4:
                r[i + j] += t
            else:
                r[i + j - 4] -= t
    return tuple(r)


def zw_complex(p) -> complex:
    return sum(c * omega_pow(i) for i, c in enumerate(p))


def exact_h(ka, kb, a, b):
    x, y = zw_pow(ka + 4 * a), zw_pow(kb + 4 * b)
    return zw_add(zw_add(zw_add((1, 0, 0, 0), x), y), zw_neg(zw_pow(ka + kb + 4 * a + 4 * b)))


def exact_product(ka, kb, avals, bvals):
    """prod_k h exactly in Z[omega] for given bits a_k, b_k."""
    z = (1, 0, 0, 0)
    for k in range(len(ka)):
        z = zw_mul(z, exact_h(int(ka[k]), int(kb[k]), int(avals[k]), int(bvals[k])))
    return z
