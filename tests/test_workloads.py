"""The seeded input generators: reference values, determinism and statistics."""
import numpy as np

from workloads import (batch_diagram, batch_params, bernoulli_matrix, bernoulli_rows, draw,
                       pauli_strings, single_diagram, unpack_rows)


def test_splitmix64_published_values():
    # SplitMix64 seeded with 0: the first two outputs of the published generator
    assert int(draw(np.uint64(0), 0)) == 0xE220A8397B1DCDAF
    assert int(draw(np.uint64(0), 1)) == 0x6E789E6AA1B965F4


def test_single_diagram_shape_and_density():
    d = single_diagram(1)
    assert d.n == 64 and d.adj.shape == (64, 1)
    b = unpack_rows(d.adj, 64)
    assert np.array_equal(b, b.T) and not b.diagonal().any()
    assert list(d.inputs) == list(range(8)) and list(d.outputs) == list(range(56, 64))
    dens = np.mean([unpack_rows(single_diagram(s).adj, 64).sum() / (64 * 63) for s in range(1, 60)])
    assert abs(dens - 0.1) < 0.01
    assert np.array_equal(single_diagram(7).adj, single_diagram(7).adj)
    assert not np.array_equal(single_diagram(7).adj, single_diagram(8).adj)


def test_batch_params_ranges():
    qs, ns, ps = zip(*[batch_params(3, i) for i in range(400)])
    assert min(qs) >= 4 and max(qs) <= 64
    assert all(n % q == 0 and 4 <= n // q <= 16 for q, n in zip(qs, ns))
    assert min(ps) >= 0.05 and max(ps) <= 0.3
    d = batch_diagram(3, 5)
    assert d.adj.shape == (d.n, (d.n + 63) // 64)


def test_bernoulli_matrix_rows_agree():
    A = bernoulli_matrix(21, 64, 200)
    assert A.shape == (64, 4)
    assert int(A[:, 3].max()) < (1 << 8)  # bits >= 200 cleared
    assert np.array_equal(bernoulli_rows(21, np.array([3, 17, 63]), 200), A[[3, 17, 63]])
    frac = unpack_rows(A, 200).mean()
    assert abs(frac - 0.5) < 0.02


def test_pauli_strings_uniform():
    X, Z = pauli_strings(22, 4096, 64)
    x = unpack_rows(X, 64)
    z = unpack_rows(Z, 64)
    code = x * 2 + z
    counts = np.bincount(code.ravel(), minlength=4) / code.size
    assert np.all(np.abs(counts - 0.25) < 0.01)
    Xs, Zs = pauli_strings(22, 4096, 64, rows=np.array([5, 9]))
    assert np.array_equal(Xs, X[[5, 9]]) and np.array_equal(Zs, Z[[5, 9]])
