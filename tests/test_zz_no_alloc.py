"""The allocation-free GF(2) elimination (static device scratch) against the
workspace entry point: two calls in a row through the C ABI, the second on a
smaller matrix, each compared bit for bit (R, rank, pivots, and T where
asked) with zx_gf2_eliminate on the same input."""
import numpy as np
import pytest
import torch

from workloads import bernoulli_matrix, bernoulli_rows  # noqa: F401

pytestmark = pytest.mark.gpu


def _both(zx, A, n_cols, want_T):
    m = A.shape[0]
    dA = zx.to_device_words(A)
    mw = (m + 63) // 64
    T1 = T2 = None
    if want_T:
        eye = np.zeros((m, mw), np.uint64)
        for i in range(m):
            eye[i, i // 64] = np.uint64(1) << np.uint64(i % 64)
        T1, T2 = zx.to_device_words(eye), zx.to_device_words(eye)
    R1, rank1, piv1, ws = zx.gf2_eliminate(dA, n_cols=n_cols, T=T1)
    R2 = torch.full_like(dA, -1)
    rank2 = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    piv2 = torch.full((m,), 77, dtype=torch.int32, device="cuda")
    zx.gf2_eliminate_noalloc(dA, R2, rank2, piv2, n_cols=n_cols, T=T2)
    torch.cuda.synchronize()
    assert zx.gf2_status(ws) == 0
    assert int(rank2.item()) == int(rank1.item()) >= 0
    assert np.array_equal(zx.to_host_words(R2), zx.to_host_words(R1))
    assert np.array_equal(piv2.cpu().numpy(), piv1.cpu().numpy())
    if want_T:
        assert np.array_equal(zx.to_host_words(T2), zx.to_host_words(T1))
    return int(rank1.item())


def test_noalloc_matches_workspace_entry_point(zx):
    print("noalloc: 2048 x 8192 with T, then 300 x 1000 low rank", flush=True)
    A = bernoulli_matrix(91, 2048, 8192)
    assert _both(zx, A, 8192, want_T=True) == 2048
    # smaller and rank-deficient: rows repeat, so the scratch's earlier
    # contents (longer ring, more snapshot rows) must not leak into this call
    B = bernoulli_matrix(92, 150, 1000)
    B = np.concatenate([B, B], axis=0)
    assert _both(zx, B, 1000, want_T=False) == 150


def test_noalloc_rejects_beyond_scratch(zx):
    A = torch.zeros((16385, 1), dtype=torch.int64, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    piv = torch.zeros(16385, dtype=torch.int32, device="cuda")
    with pytest.raises(zx.ZxError) as e:
        zx.gf2_eliminate_noalloc(A, A, rank, piv, n_cols=64)
    assert e.value.code == zx.ZX_ECAPACITY
