"""Detector sampling on the GPU (zx_detector_sample) against the oracle:
bit-exact shots for the same model, seed and shot range."""
import numpy as np
import pytest

import oracle
from workloads import surface_dem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,rounds,p,shot0,n", [(7, 7, 1e-3, 0, 100000), (15, 15, 1e-3, 12345, 20000),
                                                (5, 3, 0.05, 7, 3001), (3, 1, 0.3, 0, 257)])
def test_shots_match_oracle(zx, d, rounds, p, shot0, n):
    import torch
    print("sample case", d, rounds, p, shot0, n, flush=True)
    M = surface_dem(11, d, rounds, p)
    S = zx.DetectorSampler(M.col_ptr, M.col_idx, M.prob, M.n_f)
    out = S.sample(2024, shot0, n)
    torch.cuda.synchronize()
    assert S.status() == 0
    ref = oracle.detector_sample(M.col_ptr, M.col_idx, M.prob, M.n_f, 2024, shot0, n)
    got = zx.to_host_words(out)
    assert np.array_equal(got, ref), int((got != ref).any(axis=1).sum())


def test_wide_rows_and_deterministic_cases(zx):
    import torch
    M = surface_dem(12, 5, 2, 0.01)
    fw = (M.n_f + 63) // 64
    # ld_out beyond the row: the extra words are not written
    out = torch.full((300, fw + 3), -1, dtype=torch.int64, device="cuda")
    for prob in (np.zeros(M.n_err), np.ones(M.n_err), (np.arange(M.n_err) % 4 == 1) * 1.0, M.prob,
                 np.full(M.n_err, 1e-18)):
        S = zx.DetectorSampler(M.col_ptr, M.col_idx, prob, M.n_f)
        S.sample(5, 0, 300, out=out)
        torch.cuda.synchronize()
        assert S.status() == 0
        got = zx.to_host_words(out)
        assert np.array_equal(got[:, :fw], oracle.detector_sample(M.col_ptr, M.col_idx, prob, M.n_f, 5, 0, 300))
        assert (got[:, fw:] == np.uint64(2 ** 64 - 1)).all()


def test_invalid_model_sets_status(zx):
    import torch
    M = surface_dem(13, 3, 1, 0.01)
    bad_p = M.prob.copy()
    bad_p[3] = 1.5
    S = zx.DetectorSampler(M.col_ptr, M.col_idx, bad_p, M.n_f)
    out = S.sample(1, 0, 100)
    torch.cuda.synchronize()
    assert S.status() == zx.ZX_EINVAL
    assert not zx.to_host_words(out).any()
    bad_idx = M.col_idx.copy()
    bad_idx[0] = M.n_f  # beyond the f bits
    S = zx.DetectorSampler(M.col_ptr, bad_idx, M.prob, M.n_f)
    out = S.sample(1, 0, 100)
    torch.cuda.synchronize()
    assert S.status() == zx.ZX_EINVAL
    assert not zx.to_host_words(out).any()
