"""GPU symplectic commutation table (zx_pauli_commute) vs the CPU oracle."""
import numpy as np
import pytest

import oracle
from workloads import pauli_strings

pytestmark = pytest.mark.gpu


VARIANTS = ["valu", "mfma"]


def _flags(zx, variant):
    return zx.ZX_PAULI_FORCE_VALU if variant == "valu" else zx.ZX_PAULI_FORCE_MFMA


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n,q", [(1, 1), (2, 3), (63, 64), (64, 65), (65, 100), (200, 130),
                                 (300, 1024), (1000, 17), (129, 2000), (257, 64), (600, 300)])
def test_full_table(zx, n, q, variant):
    import torch
    print("pauli case", n, q, variant, flush=True)
    X, Z = pauli_strings(100 + n, n, q)
    Cg = zx.pauli_commute(zx.to_device_words(X), zx.to_device_words(Z), q, flags=_flags(zx, variant))
    torch.cuda.synchronize()
    Co = oracle.pauli_commute(X, Z)
    assert np.array_equal(zx.to_host_words(Cg), Co)


@pytest.mark.parametrize("variant", VARIANTS)
def test_bits_beyond_qubits_ignored(zx, variant):
    """Set bits at or beyond n_qubits in the last word change nothing."""
    import torch
    n, q = 700, 100
    X, Z = pauli_strings(7, n, q)
    Xg, Zg = X.copy(), Z.copy()
    junk = np.uint64(~((1 << (q % 64)) - 1) & (2 ** 64 - 1))
    Xg[:, -1] |= junk
    Zg[:, -1] |= junk
    Cg = zx.pauli_commute(zx.to_device_words(Xg), zx.to_device_words(Zg), q, flags=_flags(zx, variant))
    torch.cuda.synchronize()
    assert np.array_equal(zx.to_host_words(Cg), oracle.pauli_commute(X, Z))


def test_variants_equal_at_full_size(zx):
    """65536 strings on 1024 qubits (seed 22): the matrix-core table equals
    the vector-unit table bit for bit (both are compared with the oracle on
    sampled rows below)."""
    import torch
    n, q = 65536, 1024
    X, Z = pauli_strings(22, n, q)
    dX, dZ = zx.to_device_words(X), zx.to_device_words(Z)
    C1 = zx.pauli_commute(dX, dZ, q, flags=zx.ZX_PAULI_FORCE_VALU)
    C2 = zx.pauli_commute(dX, dZ, q, flags=zx.ZX_PAULI_FORCE_MFMA)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_sampled_rows(zx, variant):
    """65536 strings on 1024 qubits (seed 22): rows from several tiles,
    including the first, the last and rows straddling tile borders."""
    import torch
    n, q = 65536, 1024
    X, Z = pauli_strings(22, n, q)
    Cg = zx.pauli_commute(zx.to_device_words(X), zx.to_device_words(Z), q, flags=_flags(zx, variant))
    torch.cuda.synchronize()
    rows = [0, 1, 63, 64, 65, 255, 256, 4095, 30000, 32767, 32768, 65471, 65472, 65535]
    Ch = Cg.cpu()
    for r in rows:
        Co = oracle.pauli_commute(X, Z, rows=(r, r + 1))
        assert np.array_equal(Ch[r].numpy().view(np.uint64), Co[0]), r
    # symmetry and zero diagonal on a sampled block
    blk = Ch[:256, :4].numpy().view(np.uint64)
    bits = np.unpackbits(blk.view(np.uint8), axis=1, bitorder="little")[:, :256]
    assert np.array_equal(bits, bits.T)
    assert not bits.diagonal().any()
