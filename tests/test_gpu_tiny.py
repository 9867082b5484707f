"""Diagrams of at most 64 spiders without parameters run their whole greedy
simplification and output frontier in one wavefront's registers.  Against
the oracle: round-limited runs and their resumption, runs without the
frontier, a batch of mixed small sizes (the one-wavefront variant a batch
of such diagrams takes) and the same diagrams through a wider variant.  The
one-wavefront variant refuses the learned policy."""
import numpy as np
import pytest

import oracle
from workloads import batch_diagram, single_diagram

pytestmark = pytest.mark.gpu


def compare_state(zg, og, ctx):
    adj, ph, al, info = zg.read()
    assert info.status == 0, ctx
    assert np.array_equal(al, og.alive), ctx
    assert np.array_equal(adj, og.adj), ctx
    assert np.array_equal(ph, og.k), ctx
    assert info.pow_sqrt2 == og.scalar.pow_sqrt2, ctx
    assert info.phase8 == og.scalar.phase8 % 8, ctx
    assert info.fill_in == og.scalar.fill_in, ctx
    assert info.rounds == og.rounds, ctx
    np.testing.assert_array_equal(zg.trace(), og.trace)
    return info


def compare_frontier(zg, og, ctx):
    M, piv, rank, ops = og.frontier()
    rows, gpiv = zg.frontier()
    info = zg.info()
    assert info.rank == rank and info.rowops == ops, ctx
    assert np.array_equal(rows, M), ctx
    assert np.array_equal(gpiv, piv), ctx


def small_diagrams():
    # q in 2..4 qubits, N = q x 4..16 spiders: 8 to 64
    ds = [batch_diagram(17, i, q_lo=2, q_hi=4) for i in range(120)]
    ds = [d for d in ds if d.n <= 64]
    assert len(ds) >= 60 and min(d.n for d in ds) <= 16
    return ds


@pytest.mark.parametrize("seed", [1, 2, 3, 7, 11])
def test_round_limited_and_resumed(zx, seed):
    d = single_diagram(seed)
    assert d.n <= 64
    full = oracle.Graph.from_diagram(d)
    full.simplify()
    for r in [1, 2, 3]:
        og = oracle.Graph.from_diagram(d)
        og.simplify(max_rounds=r)
        zg = zx.Graph.from_diagram(d)
        print("tiny round-limited", seed, r, flush=True)
        zx.simplify([zg], extract=False, max_rounds=r)
        info = compare_state(zg, og, (seed, r))
        assert info.rank == -1 and info.rowops == 0
        zx.simplify([zg], extract=True, resume=True)
        compare_state(zg, full, (seed, r, "resumed"))
        compare_frontier(zg, full, (seed, r, "resumed"))


def test_small_batch_and_wider_variant(zx):
    ds = small_diagrams()
    print("tiny batch sizes", sorted(d.n for d in ds)[:8], "...", flush=True)
    names = zx.simplify_variants()
    one_wave = names.index("bs64-lds32k")
    wide = names.index("bs512-lds152k")
    for tune in (-1, one_wave, wide):
        gs = [zx.Graph.from_diagram(d) for d in ds]
        zx.simplify(gs, extract=True, tune_id=tune)
        for i, (g, d) in enumerate(zip(gs, ds)):
            og = oracle.Graph.from_diagram(d)
            assert og.simplify() == oracle.OK
            compare_state(g, og, (tune, i, d.n))
            compare_frontier(g, og, (tune, i, d.n))


def test_one_wave_variant_refuses_learned(zx):
    import torch
    from oracle import mlp as omlp
    p = (np.random.default_rng(5).standard_normal(omlp.NPARAM) * 0.3).astype(np.float32)
    m = zx.MLP(torch.from_numpy(p).cuda())
    g = zx.Graph.from_diagram(single_diagram(4))
    one_wave = zx.simplify_variants().index("bs64-lds32k")
    with pytest.raises(zx.ZxError):
        zx.simplify([g], extract=True, tune_id=one_wave, policy=zx.ZX_POLICY_LEARNED, mlp=m)
