"""Pins of the oracle's batched parities and phase-pair products.

* ``oracle.gf2_matmul`` equals the integer matrix product of the unpacked
  bits reduced mod 2 (numpy), ignores bits at or beyond k_bits, and is
  bilinear;
* ``oracle.phase.h_value`` reproduces the special cases the paper's term
  table lists as phase-pair forms: the pi-pair (-1)^{ab} (alpha = beta = 0)
  and the half-pi factors e^{+-i a pi/2} (beta = pi/2), and vanishes at
  (alpha, beta) = (pi/2, -pi/2);
* ``oracle.phase.phase_pair_product`` (fp64) equals the exact product in
  Z[omega] (Python integers) to within the rounding of fp64 products.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import phase as ph
from workloads.generators import pack_rows, unpack_rows


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 70, 64), (65, 130, 200), (17, 5, 1000)])
def test_gf2_matmul_is_integer_product_mod_2(m, n, k):
    rng = np.random.default_rng(m * 1000 + n + k)
    U = (rng.random((m, k)) < 0.5).astype(np.uint8)
    F = (rng.random((n, k)) < 0.5).astype(np.uint8)
    Up, Fp = pack_rows(U), pack_rows(F)
    # garbage beyond k_bits must not matter
    if k % 64:
        Up[:, -1] |= np.uint64(~((1 << (k % 64)) - 1) & (2 ** 64 - 1))
        Fp[:, -1] |= np.uint64(~((1 << (k % 64)) - 1) & (2 ** 64 - 1))
    C = oracle.gf2_matmul(Up, Fp, k)
    ref = (U.astype(np.int64) @ F.astype(np.int64).T) % 2
    assert np.array_equal(unpack_rows(C, n), ref.astype(np.uint8))


def test_gf2_matmul_bilinear():
    rng = np.random.default_rng(5)
    k = 300
    U = pack_rows((rng.random((9, k)) < 0.5).astype(np.uint8))
    F1 = pack_rows((rng.random((40, k)) < 0.5).astype(np.uint8))
    F2 = pack_rows((rng.random((40, k)) < 0.5).astype(np.uint8))
    assert np.array_equal(oracle.gf2_matmul(U, F1 ^ F2, k),
                          oracle.gf2_matmul(U, F1, k) ^ oracle.gf2_matmul(U, F2, k))


def test_h_special_cases():
    # pi-pair: h(0, 0; a, b) = 2 (-1)^{ab}
    for a in (0, 1):
        for b in (0, 1):
            assert abs(ph.h_value(0, 0, a, b) - 2 * (-1) ** (a * b)) < 1e-12
    # half-pi: beta = pi/2, b = 0: alpha = 0 gives 2 e^{i a pi/2}, alpha = pi gives 2i e^{-i a pi/2}
    for a in (0, 1):
        assert abs(ph.h_value(0, 2, a, 0) - 2 * 1j ** a) < 1e-12
        assert abs(ph.h_value(4, 2, a, 0) - 2j * (-1j) ** a) < 1e-12
    # a zero factor
    assert ph.h_value(2, 6, 0, 0) == 0 or abs(ph.h_value(2, 6, 0, 0)) < 1e-15
    assert ph.exact_h(2, 6, 0, 0) == (0, 0, 0, 0)
    # exact and fp64 agree on every phase pair
    for ka in range(8):
        for kb in range(8):
            for a in (0, 1):
                for b in (0, 1):
                    assert abs(ph.zw_complex(ph.exact_h(ka, kb, a, b)) - ph.h_value(ka, kb, a, b)) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_phase_pair_product_matches_exact(seed):
    rng = np.random.default_rng(40 + seed)
    m, n = int(rng.integers(1, 40)), int(rng.integers(1, 100))
    ka, kb = rng.integers(0, 8, m), rng.integers(0, 8, m)
    if seed == 0:
        ka[:], kb[:] = 2, 6   # zero factors where a = b = 0
    A = (rng.random((m, n)) < 0.5).astype(np.uint8)
    B = (rng.random((m, n)) < 0.5).astype(np.uint8)
    phase8, pw = int(rng.integers(0, 8)), int(rng.integers(-7, 8))
    mant, expo = ph.phase_pair_product(pack_rows(A), pack_rows(B), ka, kb, n, phase8, pw)
    for l in range(n):
        z = ph.exact_product(ka, kb, A[:, l], B[:, l])
        zc = ph.zw_complex(ph.zw_mul(z, ph.zw_pow(phase8))) * math.sqrt(2.0) ** pw
        got = mant[l] * 2.0 ** float(expo[l])
        assert abs(got - zc) <= 1e-12 * max(1.0, abs(zc)) * (m + 4)
        am = max(abs(mant[l].real), abs(mant[l].imag))
        assert am == 0 or 0.5 <= am < 1
