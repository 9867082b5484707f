"""Degenerate diagrams through every simplification path (batched greedy,
learned priority, serving) against the oracle: a single spider, no edges,
no outputs, every spider on a boundary wire, complete graphs with 64 and 65
spiders (one word and a ragged second word), stars."""
import numpy as np
import pytest
import torch

import oracle
from workloads.generators import Diagram, pack_rows

pytestmark = pytest.mark.gpu


def diagram(bits, phase, ins, outs):
    n = len(phase)
    return Diagram(n=n, adj=pack_rows(np.asarray(bits, np.uint8)), phase=np.asarray(phase, np.int8),
                   inputs=np.asarray(ins, np.int32), outputs=np.asarray(outs, np.int32),
                   bnd_is_h=np.zeros(len(ins) + len(outs), np.uint8))


def cases():
    out = []
    out.append(("single", diagram(np.zeros((1, 1)), [2], [], [])))
    out.append(("single-boundary", diagram(np.zeros((1, 1)), [2], [], [0])))
    z = np.zeros((100, 100))
    out.append(("no-edges", diagram(z, np.arange(100) % 8, [0, 1], [98, 99])))
    for n in (64, 65):
        k = np.ones((n, n)) - np.eye(n)
        out.append(("clique-pauli-%d" % n, diagram(k, [0] * n, [0], [n - 1])))
        out.append(("clique-lc-%d" % n, diagram(k, [2] * n, [0], [n - 1])))
    s = np.zeros((70, 70))
    s[0, 1:] = s[1:, 0] = 1
    out.append(("star-lc", diagram(s, [2] + [4] * 69, [1], [69])))
    out.append(("star-no-outputs", diagram(s, [6] + [0] * 69, [], [])))
    b = np.ones((8, 8)) - np.eye(8)
    out.append(("all-boundary", diagram(b, [2] * 8, [0, 1, 2, 3], [4, 5, 6, 7])))
    rng = np.random.default_rng(3)
    r = np.triu(rng.random((130, 130)) < 0.5, 1)
    out.append(("dense-130-no-outputs", diagram(r + r.T, rng.integers(0, 8, 130), [0, 1, 2], [])))
    return out


def expect(d):
    g = oracle.Graph.from_diagram(d)
    assert g.simplify() == oracle.OK
    rank, ops = -1, 0
    if len(d.outputs):
        _, _, rank, ops = g.frontier()
    return g, rank, ops


def test_edge_cases_batched(zx):
    cs = cases()
    gs = [zx.Graph.from_diagram(d) for _, d in cs]
    print("edge cases", [name for name, _ in cs], flush=True)
    zx.simplify(gs, extract=True)
    for (name, d), zg in zip(cs, gs):
        og, rank, ops = expect(d)
        adj, ph, al, info = zg.read()
        assert info.status == 0, name
        assert np.array_equal(adj, og.adj) and np.array_equal(ph, og.k) and np.array_equal(al, og.alive), name
        assert info.pow_sqrt2 == og.scalar.pow_sqrt2 and info.phase8 == og.scalar.phase8 % 8, name
        assert info.fill_in == og.scalar.fill_in, name
        np.testing.assert_array_equal(zg.trace(), og.trace, err_msg=name)
        if len(d.outputs):
            assert info.rank == rank and info.rowops == ops, name


def test_edge_cases_learned(zx):
    from oracle import policy as opol
    rng = np.random.default_rng(4)
    m = zx.MLP(torch.from_numpy((rng.standard_normal(zx.MLP_NPARAM) * 0.3).astype(np.float32)))
    cs = cases()
    gs = [zx.Graph.from_diagram(d) for _, d in cs]
    zx.simplify(gs, extract=True, policy=zx.ZX_POLICY_LEARNED, mlp=m)
    for (name, d), zg in zip(cs, gs):
        fin = opol.replay(oracle.Graph.from_diagram(d), zg.trace())
        adj, ph, al, info = zg.read()
        assert info.status == 0, name
        assert np.array_equal(adj, fin.adj) and np.array_equal(ph, fin.k), name
        assert info.pow_sqrt2 == fin.scalar.pow_sqrt2 and info.phase8 == fin.scalar.phase8 % 8, name


def test_edge_cases_served(zx):
    import time
    cs = cases()
    sv = zx.Server(64 << 20, max_batch=16)
    for i, (_, d) in enumerate(cs):
        assert sv.submit(d, tag=i) is not None
    res, t0 = [], time.time()
    while len(res) < len(cs):
        res += sv.poll()
        assert time.time() - t0 < 60
    for r in res:
        name, d = cs[r.tag]
        og, rank, ops = expect(d)
        assert r.status == 0 and r.n_edges == og.n_edges() and r.pow_sqrt2 == og.scalar.pow_sqrt2, name
        assert r.rank == rank and r.rowops == ops, name
    sv.close()
