"""Diagrams of several thousand spiders (the serving stream's large
requests, 2000 to 8000 spiders) simplified on the GPU, in zx_simplify and
in the serving loop, against the oracle's results stored in
tests/golden/large_diagrams.json (written by make_large_diagrams.py from the
oracle alone; the N = 8000 oracle run takes about three minutes)."""
import hashlib
import json
import os
import time

import numpy as np
import pytest

from workloads import serve_diagram

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_diagrams.json")


def entries():
    with open(GOLDEN) as f:
        return json.load(f)["entries"]


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_golden_covers_the_large_sizes():
    ns = sorted(e["n"] for e in entries())
    assert ns[0] <= 2100 and ns[-1] >= 7900 and len(ns) >= 5


def test_simplify_large_against_oracle(zx):
    es = entries()
    ds = [serve_diagram(e["seed"], e["item"]) for e in es]
    for d, e in zip(ds, es):
        assert d.n == e["n"]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    print("large simplify", [d.n for d in ds], flush=True)
    t0 = time.time()
    zx.simplify(gs, extract=True)
    for g, e in zip(gs, es):
        adj, ph, al, info = g.read()
        ctx = (e["item"], e["n"])
        assert info.status == 0, ctx
        assert info.n_edges == e["n_edges"] and info.n_alive == e["n_alive"], ctx
        assert info.pow_sqrt2 == e["pow_sqrt2"] and info.phase8 == e["phase8"], ctx
        assert info.fill_in == e["fill_in"] and info.rounds == e["rounds"], ctx
        assert info.n_trace == e["n_trace"], ctx
        assert info.rank == e["rank"] and info.rowops == e["rowops"], ctx
        assert digest(adj.astype("<u8")) == e["sha_adj"], ctx
        assert digest(ph.astype("i1")) == e["sha_phase"], ctx
        assert digest(al.astype("<u8")) == e["sha_alive"], ctx
        assert digest(g.trace().astype("<i4")) == e["sha_trace"], ctx
        rows, piv = g.frontier()
        assert digest(rows.astype("<u8")) == e["sha_front"], ctx
        assert digest(piv.astype("<i4")) == e["sha_fpiv"], ctx
    print("large simplify %.2f s" % (time.time() - t0), flush=True)


def test_serve_large_against_oracle(zx):
    es = entries()
    ds = [serve_diagram(e["seed"], e["item"]) for e in es]
    sv = zx.Server(512 << 20, max_batch=16)
    print("serve large", [d.n for d in ds], flush=True)
    for i, d in enumerate(ds):
        assert sv.submit(d, tag=i) is not None
    res = []
    t0 = time.time()
    while len(res) < len(ds):
        res += sv.poll()
        assert time.time() - t0 < 100, "server did not finish"
    for r in res:
        e = es[r.tag]
        ctx = (e["item"], e["n"])
        assert r.status == 0, ctx
        assert r.n_edges == e["n_edges"] and r.n_alive == e["n_alive"], ctx
        assert r.pow_sqrt2 == e["pow_sqrt2"] and r.phase8 == e["phase8"], ctx
        assert r.fill_in == e["fill_in"] and r.rounds == e["rounds"] and r.n_trace == e["n_trace"], ctx
        assert r.rank == e["rank"] and r.rowops == e["rowops"], ctx
    sv.close()


def test_mixed_batch_large_and_small(zx):
    """One batch with large diagrams (run by the team kernel) and small ones
    (run by the regular kernel after it): every result as the oracle's."""
    import oracle
    from workloads import batch_diagram
    es = [e for e in entries() if e["n"] < 3500]
    big = [serve_diagram(e["seed"], e["item"]) for e in es]
    small = [batch_diagram(3, i) for i in range(24)]
    ds = small[:12] + big + small[12:]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    print("mixed batch", [d.n for d in ds], flush=True)
    zx.simplify(gs, extract=True)
    for g, e in zip(gs[12:12 + len(big)], es):
        adj, ph, al, info = g.read()
        assert info.status == 0 and info.rounds == e["rounds"] and info.rowops == e["rowops"], e["n"]
        assert digest(adj.astype("<u8")) == e["sha_adj"] and digest(g.trace().astype("<i4")) == e["sha_trace"]
    for g, d in zip(gs[:12] + gs[12 + len(big):], small):
        og = oracle.Graph.from_diagram(d)
        og.simplify()
        adj, ph, al, info = g.read()
        assert info.status == 0
        assert np.array_equal(adj, og.adj) and np.array_equal(ph, og.k) and np.array_equal(al, og.alive)
        np.testing.assert_array_equal(g.trace(), og.trace)
