"""Batched parities on the matrix cores (zx_gf2_matmul) and the phase-pair
product (zx_phase_pair_product) against the oracle.

Parities are bits: compared exactly.  The phase-pair product is fp32 complex
against the oracle's fp64; the tolerance is derived from the arithmetic:
each factor h has four terms of magnitude <= 1 summed with three fp32
roundings (<= 12u per component) plus the fp32 rounding of sqrt(1/2) in the
table (< 1.1u), i.e. an absolute error < 18.6u, which is a relative error
< 17.2u since every non-zero h has |h| >= 1.0824; each complex product adds
< 3u; the constant sqrt(2) and table value add < 2u.  Relative tolerance
(21 m + 4) u, u = 2^-24, m terms.  Zero factors (h = 0 exactly) are exact
zeros on both sides.
"""
import numpy as np
import pytest

import oracle
from oracle import phase as oph
from workloads import parity_problem
from workloads.generators import pack_rows

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 70, 64), (257, 300, 200), (513, 1000, 130),
                                   (40, 600, 2000), (300, 257, 63),
                                   # beyond 2048 bits: the chunked 256 x 256 kernel, ragged rows and K
                                   (300, 700, 3000), (1100, 530, 2100), (5, 2049, 4100)])
def test_gf2_matmul_matches_oracle(zx, m, n, k):
    import torch
    print("gf2_matmul case", m, n, k, flush=True)
    rng = np.random.default_rng(m + 7 * n + 13 * k)
    U = pack_rows((rng.random((m, k)) < 0.5).astype(np.uint8))
    F = pack_rows((rng.random((n, k)) < 0.3).astype(np.uint8))
    Ug, Fg = U.copy(), F.copy()
    if k % 64:  # junk beyond k_bits must be ignored
        junk = np.uint64(~((1 << (k % 64)) - 1) & (2 ** 64 - 1))
        Ug[:, -1] |= junk
        Fg[:, -1] |= junk
    C = zx.gf2_matmul(zx.to_device_words(Ug), zx.to_device_words(Fg), k)
    torch.cuda.synchronize()
    assert np.array_equal(zx.to_host_words(C), oracle.gf2_matmul(U, F, k))


def test_gf2_matmul_full_size_sampled(zx):
    """The benchmark contraction (4096 terms x 65536 settings x 1024
    parameters): sampled term rows against the oracle, all settings."""
    import torch
    P = parity_problem(61, 4096, 65536, 1024)
    C = zx.gf2_matmul(zx.to_device_words(P.U), zx.to_device_words(P.F), P.n_params)
    torch.cuda.synchronize()
    Ch = zx.to_host_words(C)
    for r in (0, 255, 256, 4095):
        assert np.array_equal(Ch[r:r + 1], oracle.gf2_matmul(P.U[r:r + 1], P.F, P.n_params)), r


def _compare(mg, eg, mo, eo, m):
    tol = (21 * m + 4) * U32
    zg = mg[:, 0].astype(np.float64) + 1j * mg[:, 1].astype(np.float64)
    for l in range(len(mo)):
        if mo[l] == 0:
            assert zg[l] == 0, l
            continue
        d = abs(zg[l] * 2.0 ** float(int(eg[l]) - int(eo[l])) - mo[l])
        assert d <= tol * abs(mo[l]), (l, d, tol)


@pytest.mark.parametrize("seed,m,n", [(0, 0, 5), (1, 1, 64), (2, 37, 300), (3, 300, 200), (4, 1000, 65)])
def test_phase_pair_product_matches_oracle(zx, seed, m, n):
    import torch
    print("phase_pair case", seed, m, n, flush=True)
    rng = np.random.default_rng(500 + seed)
    ka = rng.integers(0, 8, m).astype(np.int8)
    kb = rng.integers(0, 8, m).astype(np.int8)
    if seed == 2:
        ka[::3], kb[::3] = 2, 6   # zero factors where a = b = 0
    A = pack_rows((rng.random((m, n)) < 0.5).astype(np.uint8)) if m else np.zeros((0, 1), np.uint64)
    B = pack_rows((rng.random((m, n)) < 0.5).astype(np.uint8)) if m else np.zeros((0, 1), np.uint64)
    phase8, pw = int(rng.integers(0, 8)), int(rng.integers(-9, 10))
    mo, eo = oph.phase_pair_product(A, B, ka, kb, n, phase8, pw)
    dev = "cuda"
    tA = zx.to_device_words(A) if m else None
    tB = zx.to_device_words(B) if m else None
    mg, eg = zx.phase_pair_product(tA, tB, torch.from_numpy(ka).to(dev), torch.from_numpy(kb).to(dev), n,
                                   phase8, pw)
    torch.cuda.synchronize()
    _compare(mg.cpu().numpy(), eg.cpu().numpy(), mo, eo, m)
