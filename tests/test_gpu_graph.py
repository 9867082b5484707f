"""GPU rewriting (zx_local_comp, zx_pivot, zx_simplify + frontier) vs the
CPU oracle: adjacency, phases, alive set, scalar, fill-in, trace and the
reduced output frontier must all match bit for bit."""
import numpy as np
import pytest

import oracle
from workloads import batch_diagram, single_diagram
from workloads.generators import pack_rows

pytestmark = pytest.mark.gpu


def compare_state(zg, og, ctx=""):
    adj, ph, al, info = zg.read()
    assert info.status == 0, ctx
    assert np.array_equal(al, og.alive), ctx
    assert np.array_equal(adj, og.adj), ctx
    assert np.array_equal(ph, og.k), ctx
    assert info.pow_sqrt2 == og.scalar.pow_sqrt2, ctx
    assert info.phase8 == og.scalar.phase8 % 8, ctx
    assert info.fill_in == og.scalar.fill_in, ctx
    assert info.n_edges == og.n_edges(), ctx
    assert info.n_alive == len(og.alive_list()), ctx
    return info


def random_graph(rng, n, q, dens):
    b = np.triu((rng.random((n, n)) < dens).astype(np.uint8), 1)
    b = b + b.T
    k = rng.integers(0, 8, n).astype(np.int8)
    perm = rng.permutation(n)
    return pack_rows(b), k, perm[:q].astype(np.int32), perm[q:2 * q].astype(np.int32)


@pytest.mark.parametrize("seed", range(24))
def test_single_rewrites(zx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.choice([5, 17, 64, 65, 130, 300]))
    q = int(rng.integers(0, 4))
    adj, k, ins, outs = random_graph(rng, n, q, [0.1, 0.3, 0.6][seed % 3])
    interior = [v for v in range(n) if v not in set(ins) | set(outs)]
    og = oracle.Graph(n, adj, k, ins, outs)
    zg = zx.Graph.create(adj, k, ins, outs)
    print("single case", seed, n, q, flush=True)
    for step in range(6):
        alive = [v for v in interior if og.is_alive(v)]
        if len(alive) < 2:
            break
        kind = step % 3
        if kind == 0:  # LC with a pi/2 phase forced through a fresh graph state
            u = int(rng.choice(alive))
            if og.k[u] not in (2, 6):
                continue
            assert og.local_comp(u) == oracle.OK
            zg.local_comp(u)
        elif kind == 1:
            u, v = (int(x) for x in rng.choice(alive, 2, replace=False))
            if not og.edge(u, v) or og.k[u] not in (0, 4) or og.k[v] not in (0, 4):
                continue
            assert og.pivot(u, v) == oracle.OK
            zg.pivot(u, v)
        else:
            u = int(rng.choice(alive))
            assert og.local_comp(u, graph_only=True) == oracle.OK
            zg.local_comp(u, graph_only=True)
        compare_state(zg, og, "seed %d step %d" % (seed, step))


@pytest.mark.parametrize("seed", range(12))
def test_graph_only_pivot(zx, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.choice([6, 40, 70, 200]))
    adj, k, ins, outs = random_graph(rng, n, 0, 0.4)
    og = oracle.Graph(n, adj, k)
    # the pair is drawn among the edges, so every seed runs a pivot
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if og.edge(a, b)]
    assert pairs
    u, v = pairs[int(rng.integers(len(pairs)))]
    zg = zx.Graph.create(adj, k, ins, outs)
    assert og.pivot(u, v, graph_only=True) == oracle.OK
    zg.pivot(u, v, graph_only=True)
    compare_state(zg, og)


def test_precondition_failure_sets_status(zx):
    b = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], np.uint8)
    zg = zx.Graph.create(pack_rows(b), np.array([1, 2, 0], np.int8), np.array([0], np.int32),
                         np.array([2], np.int32))
    before = zg.read()
    zg.local_comp(0)  # phase pi/4: no match
    assert zg.status() == zx.ZX_ENOMATCH
    after = zg.read()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    zg2 = zx.Graph.create(pack_rows(b), np.array([1, 2, 0], np.int8), np.array([0], np.int32),
                          np.array([2], np.int32))
    zg2.pivot(0, 2)  # not adjacent
    assert zg2.status() == zx.ZX_ENOMATCH


def check_simplified(zg, d, extract=True, ctx=""):
    og = oracle.Graph.from_diagram(d)
    assert og.simplify() == oracle.OK
    info = compare_state(zg, og, ctx)
    tr = zg.trace()
    assert np.array_equal(tr, og.trace), ctx
    assert info.rounds == og.rounds, ctx
    if extract:
        M, piv, rank, ops = og.frontier()
        rows, gpiv = zg.frontier()
        assert info.rank == rank, ctx
        assert info.rowops == ops, ctx
        assert np.array_equal(rows, M), ctx
        assert np.array_equal(gpiv, piv), ctx
    return og


def test_single_diagram_workload(zx):
    """8 qubits, 64 spiders, ER p = 0.1: all seeds 1..1000 in one batch."""
    ds = [single_diagram(s) for s in range(1, 1001)]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    zx.simplify(gs, extract=True)
    for s, (g, d) in enumerate(zip(gs, ds), start=1):
        check_simplified(g, d, ctx="seed %d" % s)


def batch_sample():
    idx = list(range(0, 48)) + [100, 500, 1000, 2000, 3000, 4095]
    return idx, [batch_diagram(3, i) for i in idx]


def test_batched_workload_sample(zx):
    """Diagrams of the batched workload (q in 4..64, N = q * 4..16)."""
    idx, ds = batch_sample()
    gs = [zx.Graph.from_diagram(d) for d in ds]
    print("batched sample sizes", [d.n for d in ds], flush=True)
    zx.simplify(gs, extract=True)
    for i, g, d in zip(idx, gs, ds):
        check_simplified(g, d, ctx="item %d n %d" % (i, d.n))


def test_batched_equals_one_launch_per_diagram(zx):
    import torch
    ds = [batch_diagram(3, i) for i in range(64)]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    zx.simplify(gs, extract=True)
    batched = [g.read() for g in gs]
    btr = [g.trace() for g in gs]
    for g in gs:
        zx.simplify([g], extract=True)
        torch.cuda.synchronize()
    for g, b, t in zip(gs, batched, btr):
        a = g.read()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert a[3].pow_sqrt2 == b[3].pow_sqrt2 and a[3].rowops == b[3].rowops
        assert np.array_equal(g.trace(), t)


def test_every_variant_identical(zx):
    ds = [batch_diagram(3, i) for i in range(40)] + [single_diagram(5)]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    ref = None
    for v in range(len(zx.simplify_variants())):
        try:
            zx.simplify(gs, extract=True, tune_id=v)
        except zx.ZxError as e:
            assert e.code == zx.ZX_ECAPACITY
            continue
        out = [(g.read()[0], g.read()[1], g.frontier()[0]) for g in gs]
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
    assert ref is not None


def test_autotune_and_graph_capture(zx):
    """The prepared batch launch replays from a HIP graph; every replay equals
    the eager result (several replays, with eager work in between)."""
    import torch
    ds = [batch_diagram(3, i) for i in range(100, 164)]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    b = zx.Batch(gs)
    best, ms = b.autotune(extract=True, reps=2)
    assert 0 <= best < len(zx.simplify_variants()) and ms > 0
    b.run(extract=True)
    torch.cuda.synchronize()
    eager = [(g.read()[0].copy(), g.frontier()[0].copy()) for g in gs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.run(extract=True, stream=s)  # warm-up on the capture stream
        s.synchronize()
        graph.capture_begin()
        b.run(extract=True, stream=s)
        graph.capture_end()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for g in gs:
            g.reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for g, e in zip(gs, eager):
            assert np.array_equal(g.read()[0], e[0]), rep
            assert np.array_equal(g.frontier()[0], e[1]), rep
    assert b.status() == 0
