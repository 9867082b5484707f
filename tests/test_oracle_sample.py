"""Pins of the oracle's detector sampler (f = T e with geometric gaps).

Closed forms fix the distribution the sampler must produce: for independent
mechanisms j firing with probability p_j, the parity of any set S of f bits
is 1 with probability (1 - prod_j (1 - 2 p_j)^{[|col_j & S| odd]}) / 2.  The
tests check single bits and random sets against it within 5 standard
deviations, a single mechanism's firing rate, and the deterministic cases
(all probabilities 0, all 1, a mix of 0 and 1).  A gap drawn off by one, a
thinning threshold taken against the wrong maximum, or a column applied to
the wrong shot changes these rates.
"""
import numpy as np
import pytest

import oracle
from workloads import surface_dem
from workloads.generators import unpack_rows


def parity_prob(M, S):
    prod = 1.0
    Sset = set(S)
    for j in range(M.n_err):
        c = M.col_idx[M.col_ptr[j]:M.col_ptr[j + 1]]
        if sum(1 for i in c if i in Sset) % 2:
            prod *= 1.0 - 2.0 * M.prob[j]
    return (1.0 - prod) / 2.0


def check_rate(bits, p, n):
    emp = bits.mean()
    sd = np.sqrt(max(p * (1 - p), 1e-12) / n)
    assert abs(emp - p) <= 5 * sd + 1e-12, (emp, p, sd)


@pytest.mark.parametrize("d,rounds,p", [(3, 2, 0.02), (5, 3, 0.05)])
def test_marginals_and_parities(d, rounds, p):
    M = surface_dem(3, d, rounds, p)
    n = 60000
    F = oracle.detector_sample(M.col_ptr, M.col_idx, M.prob, M.n_f, 123, 0, n)
    B = unpack_rows(F, M.n_f)
    for i in range(M.n_f):
        check_rate(B[:, i], parity_prob(M, [i]), n)
    rng = np.random.default_rng(d)
    for _ in range(20):
        S = rng.choice(M.n_f, int(rng.integers(2, 6)), replace=False)
        check_rate(B[:, S].sum(axis=1) % 2, parity_prob(M, S), n)


def test_single_mechanism_rate():
    for p in (0.3, 0.01):
        n = 200000
        F = oracle.detector_sample([0, 1], [0], [p], 1, 9, 0, n)
        check_rate(unpack_rows(F, 1)[:, 0], p, n)


def test_deterministic_cases():
    M = surface_dem(4, 5, 2, 0.01)
    zero = oracle.detector_sample(M.col_ptr, M.col_idx, np.zeros(M.n_err), M.n_f, 1, 0, 50)
    assert not zero.any()
    allx = np.zeros(M.n_f, np.uint8)
    for j in range(M.n_err):
        allx[M.col_idx[M.col_ptr[j]:M.col_ptr[j + 1]]] ^= 1
    ones = oracle.detector_sample(M.col_ptr, M.col_idx, np.ones(M.n_err), M.n_f, 1, 0, 50)
    assert (unpack_rows(ones, M.n_f) == allx[None, :]).all()
    mix = (np.arange(M.n_err) % 3 == 0).astype(np.float64)
    want = np.zeros(M.n_f, np.uint8)
    for j in range(0, M.n_err, 3):
        want[M.col_idx[M.col_ptr[j]:M.col_ptr[j + 1]]] ^= 1
    got = oracle.detector_sample(M.col_ptr, M.col_idx, mix, M.n_f, 5, 0, 50)
    assert (unpack_rows(got, M.n_f) == want[None, :]).all()


def test_shots_are_independent_of_batching():
    """Shot s depends only on (seed, s): a range equals the same rows of a
    larger range."""
    M = surface_dem(2, 5, 2, 0.03)
    A = oracle.detector_sample(M.col_ptr, M.col_idx, M.prob, M.n_f, 77, 0, 500)
    B = oracle.detector_sample(M.col_ptr, M.col_idx, M.prob, M.n_f, 77, 200, 100)
    assert np.array_equal(A[200:300], B)
