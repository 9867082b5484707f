"""GPU GF(2) RREF (zx_gf2_eliminate) vs the CPU oracle, bit-exact.

RREF is unique, so R, the rank and the pivot columns must match the oracle
exactly on every input; zero rows fill the bottom.
"""
import numpy as np
import pytest

import oracle
from workloads import bernoulli_matrix
from workloads.generators import pack_rows

pytestmark = pytest.mark.gpu


def run_gpu(zx, A, n_cols, inplace=False):
    import torch
    dA = zx.to_device_words(A)
    if inplace:
        R, rank, piv, ws = zx.gf2_eliminate(dA, R=dA, n_cols=n_cols)
    else:
        R, rank, piv, ws = zx.gf2_eliminate(dA, n_cols=n_cols)
    torch.cuda.synchronize()
    assert zx.gf2_status(ws) == 0
    return zx.to_host_words(R), int(rank.item()), piv.cpu().numpy()


def check(zx, A, n_cols, inplace=False):
    print("gf2 case", A.shape, n_cols, flush=True)
    R, rank, piv = run_gpu(zx, A, n_cols, inplace)
    Ro, pivo, ranko, _ = oracle.gf2_rref(A, n_cols)
    assert rank == ranko
    assert np.array_equal(piv, pivo)
    nw = (n_cols + 63) // 64
    assert np.array_equal(R[:, :nw], Ro[:, :nw])


@pytest.mark.parametrize("m,n", [(1, 1), (1, 64), (3, 5), (5, 9), (64, 64), (63, 130), (100, 300),
                                 (130, 64), (129, 129), (200, 1000), (64, 4096), (700, 2000),
                                 (1000, 700), (257, 4100), (2048, 2048)])
def test_random(zx, m, n):
    A = bernoulli_matrix(1000 + m, m, n)
    check(zx, A, n)


@pytest.mark.parametrize("dens", [0.02, 0.1, 0.9])
def test_sparse_dense(zx, dens):
    rng = np.random.default_rng(int(dens * 100))
    B = (rng.random((300, 700)) < dens).astype(np.uint8)
    check(zx, pack_rows(B), 700)


def test_zero_and_identity(zx):
    check(zx, np.zeros((50, 3), np.uint64), 150)
    eye = pack_rows(np.eye(130, dtype=np.uint8))
    check(zx, eye, 130)
    # duplicated rows: rank half the rows
    rng = np.random.default_rng(3)
    B = rng.integers(0, 2, (200, 500)).astype(np.uint8)
    check(zx, pack_rows(np.vstack([B, B])), 500)


def test_low_rank_multi_pass(zx):
    """Rank-deficient strips force residual passes (fewer than 64 pivots among
    128 candidates while more non-zero rows remain)."""
    rng = np.random.default_rng(17)
    for r in (3, 40, 63, 100):
        L = rng.integers(0, 2, (1000, r)).astype(np.uint8)
        Rm = rng.integers(0, 2, (r, 900)).astype(np.uint8)
        B = (L.astype(np.int64) @ Rm.astype(np.int64) % 2).astype(np.uint8)
        check(zx, pack_rows(B), 900)


def test_inplace_and_ld(zx):
    A = bernoulli_matrix(5, 300, 640)
    check(zx, A, 640, inplace=True)
    # leading dimension larger than the row: padding words untouched
    import torch
    Ap = np.zeros((300, 13), np.uint64)
    Ap[:, :10] = A
    Ap[:, 10:] = np.uint64(0xDEADBEEF)
    dA = zx.to_device_words(Ap)
    R, rank, piv, ws = zx.gf2_eliminate(dA, n_cols=640)
    torch.cuda.synchronize()
    Rh = zx.to_host_words(R)
    Ro, pivo, ranko, _ = oracle.gf2_rref(A, 640)
    assert np.array_equal(Rh[:, :10], Ro)
    assert int(rank.item()) == ranko


def test_full_size_4096x16384(zx):
    """The benchmark matrix (Bernoulli(1/2), seed 21): whole-matrix bit-exact."""
    A = bernoulli_matrix(21, 4096, 16384)
    check(zx, A, 16384)


def test_repeat_reuses_workspace(zx):
    import torch
    A = bernoulli_matrix(7, 512, 4096)
    dA = zx.to_device_words(A)
    R, rank, piv, ws = zx.gf2_eliminate(dA, n_cols=4096)
    first = zx.to_host_words(R).copy()
    for _ in range(3):
        zx.gf2_eliminate(dA, R=R, n_cols=4096, rank=rank, pivots=piv, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(zx.to_host_words(R), first)


def test_workspace_reuse_different_inputs(zx):
    """One workspace through eliminations of different matrices: the pass
    records an earlier launch left in the workspace never stand in for this
    launch's (each result equals the oracle's)."""
    import torch
    from workloads.generators import unpack_rows
    m, n = 512, 4096
    ws = None
    rng = np.random.default_rng(5)
    cases = [bernoulli_matrix(s, m, n) for s in (7, 8, 9)]
    # rank-deficient: 200 independent rows repeated, so strips take residual passes
    base = unpack_rows(bernoulli_matrix(10, 200, n), n)
    cases.append(pack_rows(base[rng.integers(0, 200, m)]))
    for A in cases:
        dA = zx.to_device_words(A)
        R, rank, piv, ws = zx.gf2_eliminate(dA, n_cols=n, ws=ws)
        torch.cuda.synchronize()
        assert zx.gf2_status(ws) == 0
        Ro, pivo, ranko, _ = oracle.gf2_rref(A, n)
        assert int(rank.item()) == ranko
        assert np.array_equal(piv.cpu().numpy(), pivo)
        assert np.array_equal(zx.to_host_words(R), Ro)


def test_capacity_error(zx):
    import torch
    dA = torch.zeros((16385, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(zx.ZxError) as e:
        zx.gf2_eliminate(dA, n_cols=64)
    assert e.value.code == zx.ZX_ECAPACITY


# ---------------------------------------------------------------- transform --

def gf2_matmul(Tw, Aw, m, n_cols):
    """T A over F2 (packed rows in, packed rows out), by unpacked integer products."""
    from workloads.generators import unpack_rows
    Tb = unpack_rows(Tw, m).astype(np.int64)
    Ab = unpack_rows(Aw, n_cols).astype(np.int64)
    return pack_rows(((Tb @ Ab) & 1).astype(np.uint8))


def run_gpu_t(zx, A, n_cols, ldt_extra=0):
    import torch
    m = A.shape[0]
    mw = (m + 63) // 64
    dA = zx.to_device_words(A)
    dT = torch.full((m, mw + ldt_extra), -1, dtype=torch.int64, device="cuda")
    R, rank, piv, ws = zx.gf2_eliminate(dA, n_cols=n_cols, T=dT)
    torch.cuda.synchronize()
    assert zx.gf2_status(ws) == 0
    T = zx.to_host_words(dT)
    if ldt_extra:
        assert np.all(T[:, mw:] == np.uint64(0xFFFFFFFFFFFFFFFF))  # padding words untouched
    return zx.to_host_words(R), int(rank.item()), piv.cpu().numpy(), T[:, :mw]


@pytest.mark.parametrize("m,n", [(1, 64), (64, 64), (100, 300), (130, 700), (700, 2000), (1000, 700)])
def test_transform_random(zx, m, n):
    """R and pivots as without T; T A = R; T equals the oracle's transform when
    A has full row rank (the transform is unique then), and is invertible."""
    A = bernoulli_matrix(2000 + m, m, n)
    print("gf2 transform", m, n, flush=True)
    R, rank, piv, T = run_gpu_t(zx, A, n, ldt_extra=1 if m == 100 else 0)
    Ro, pivo, ranko, _, To = oracle.gf2_rref(A, n, want_T=True)
    nw = (n + 63) // 64
    assert rank == ranko and np.array_equal(piv, pivo)
    assert np.array_equal(R[:, :nw], Ro[:, :nw])
    assert np.array_equal(gf2_matmul(T, A, m, n)[:, :nw], Ro[:, :nw])
    if ranko == m:
        assert np.array_equal(T, To)
    assert oracle.gf2_rref(T, m)[2] == m


def test_transform_rank_deficient(zx):
    """Low rank: T A = R, T invertible, and the rows of T beyond the rank lie in
    the left null space (the transform is not unique here)."""
    rng = np.random.default_rng(23)
    for r, m, n in ((5, 300, 500), (70, 400, 900), (200, 1000, 1500)):
        L = rng.integers(0, 2, (m, r)).astype(np.uint8)
        Rm = rng.integers(0, 2, (r, n)).astype(np.uint8)
        A = pack_rows((L.astype(np.int64) @ Rm.astype(np.int64) % 2).astype(np.uint8))
        print("gf2 transform low rank", r, m, n, flush=True)
        R, rank, piv, T = run_gpu_t(zx, A, n)
        Ro, pivo, ranko, _ = oracle.gf2_rref(A, n)
        nw = (n + 63) // 64
        assert rank == ranko and np.array_equal(R[:, :nw], Ro[:, :nw])
        TA = gf2_matmul(T, A, m, n)[:, :nw]
        assert np.array_equal(TA, Ro[:, :nw])
        assert not TA[rank:].any()
        assert oracle.gf2_rref(T, m)[2] == m


def test_transform_full_size(zx):
    """The benchmark matrix with its transform: unique (full row rank), so T
    equals the oracle's bit for bit."""
    A = bernoulli_matrix(21, 4096, 16384)
    R, rank, piv, T = run_gpu_t(zx, A, 16384)
    Ro, pivo, ranko, _, To = oracle.gf2_rref(A, 16384, want_T=True)
    assert rank == ranko == 4096
    assert np.array_equal(R, Ro) and np.array_equal(piv, pivo)
    assert np.array_equal(T, To)
