"""GPU symplectic commutation table (zx_pauli_commute) vs the CPU oracle."""
import numpy as np
import pytest

import oracle
from workloads import pauli_strings

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,q", [(1, 1), (2, 3), (63, 64), (64, 65), (65, 100), (200, 130),
                                 (300, 1024), (1000, 17), (129, 2000)])
def test_full_table(zx, n, q):
    import torch
    print("pauli case", n, q, flush=True)
    X, Z = pauli_strings(100 + n, n, q)
    Cg = zx.pauli_commute(zx.to_device_words(X), zx.to_device_words(Z), q)
    torch.cuda.synchronize()
    Co = oracle.pauli_commute(X, Z)
    assert np.array_equal(zx.to_host_words(Cg), Co)


def test_full_size_sampled_rows(zx):
    """65536 strings on 1024 qubits (seed 22): rows from several tiles,
    including the first, the last and rows straddling tile borders."""
    import torch
    n, q = 65536, 1024
    X, Z = pauli_strings(22, n, q)
    Cg = zx.pauli_commute(zx.to_device_words(X), zx.to_device_words(Z), q)
    torch.cuda.synchronize()
    rows = [0, 1, 63, 64, 65, 4095, 30000, 32767, 32768, 65471, 65472, 65535]
    Ch = Cg.cpu()
    for r in rows:
        Co = oracle.pauli_commute(X, Z, rows=(r, r + 1))
        assert np.array_equal(Ch[r].numpy().view(np.uint64), Co[0]), r
    # symmetry and zero diagonal on a sampled block
    blk = Ch[:256, :4].numpy().view(np.uint64)
    bits = np.unpackbits(blk.view(np.uint8), axis=1, bitorder="little")[:, :256]
    assert np.array_equal(bits, bits.T)
    assert not bits.diagonal().any()
