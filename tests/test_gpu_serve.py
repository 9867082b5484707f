"""Serving loop on the GPU: every result equals the oracle's simplification
of the same request; admission refuses (ZX_EBUSY) when the pool is full and
accepts again once results are harvested; oversize requests are rejected."""
import time

import numpy as np
import pytest

import oracle
from workloads import serve_diagram
from workloads.generators import Diagram

pytestmark = pytest.mark.gpu


def drain(sv, want, timeout=120):
    out = []
    t0 = time.time()
    while len(out) < want:
        out += sv.poll()
        assert time.time() - t0 < timeout, "server did not finish"
    return out


def check(r, d):
    og = oracle.Graph.from_diagram(d)
    assert og.simplify() == oracle.OK
    rank, ops = -1, 0
    if len(og.outputs):
        _, _, rank, ops = og.frontier()
    ctx = (r.tag, d.n)
    assert r.status == 0, ctx
    assert r.n_edges == og.n_edges(), ctx
    assert r.n_alive == len(og.alive_list()), ctx
    assert r.pow_sqrt2 == og.scalar.pow_sqrt2, ctx
    assert r.phase8 == og.scalar.phase8 % 8, ctx
    assert r.fill_in == og.scalar.fill_in, ctx
    assert r.rounds == og.rounds and r.n_trace == len(og.trace), ctx
    assert r.rank == rank and r.rowops == ops, ctx
    assert r.t_submit <= r.t_launch <= r.t_done, ctx


def test_serve_matches_oracle(zx):
    ds = [serve_diagram(5, i, q_hi=64) for i in range(120)]
    # a few above 1024 spiders: they are batched apart from the rest
    big = [d for d in (serve_diagram(5, 500 + i, q_lo=100, q_hi=128) for i in range(12)) if d.n > 1024][:3]
    assert big
    ds = ds[:60] + big + ds[60:]
    sv = zx.Server(256 << 20, max_batch=48)
    res = []
    print("serve", len(ds), "requests", flush=True)
    for i, d in enumerate(ds):
        assert sv.submit(d, tag=i) is not None
        if i % 10 == 9:
            res += sv.poll()
    res += drain(sv, len(ds) - len(res))
    assert sorted(r.tag for r in res) == list(range(len(ds)))
    assert len({r.ticket for r in res}) == len(ds)
    for r in res:
        check(r, ds[r.tag])
    st = sv.stats()
    assert st.completed == len(ds) and st.submitted == len(ds) and st.refused == 0
    assert st.batches >= 1 and st.pool_used == 0 and st.pending == 0
    sv.close()


def test_serve_idle_exit_and_relaunch(zx):
    """The resident kernel leaves after a quiet spell; a later request starts
    it again and is answered."""
    ds = [serve_diagram(5, 2000 + i, q_hi=32) for i in range(2)]
    sv = zx.Server(64 << 20, max_batch=16)
    assert sv.submit(ds[0], tag=0) is not None
    r0 = drain(sv, 1)
    t0 = time.time()
    while sv.stats().running and time.time() - t0 < 10:
        time.sleep(0.05)
        sv.poll()
    assert sv.stats().running == 0  # idle exit
    assert sv.submit(ds[1], tag=1) is not None
    r1 = drain(sv, 1)
    check(r0[0], ds[0])
    check(r1[0], ds[1])
    assert sv.stats().batches >= 2
    sv.close()


def test_serve_admission(zx):
    ds = [serve_diagram(5, 1000 + i, q_hi=48) for i in range(40)]
    biggest = max(zx.Graph.bytes_for(d.n, len(d.inputs), len(d.outputs)) for d in ds)
    head = 256  # the server's control word
    sv = zx.Server(head + 3 * ((biggest + 255) // 256 * 256), max_batch=4)
    todo = list(range(len(ds)))
    res, refused = [], 0
    t0 = time.time()
    while todo or len(res) < len(ds):
        while todo:
            if sv.submit(ds[todo[0]], tag=todo[0]) is None:
                refused += 1
                break
            todo.pop(0)
        res += sv.poll()
        assert time.time() - t0 < 120
    assert refused > 0
    st = sv.stats()
    assert st.refused == refused and st.completed == len(ds) and st.pool_used == 0
    assert st.pool_peak <= st.pool_bytes
    for r in res[:10]:
        check(r, ds[r.tag])
    sv.close()


def test_serve_rejects_oversize(zx):
    n = 9000  # beyond the kernels' 8192-spider limit
    W = (n + 63) // 64
    d = Diagram(n=n, adj=np.zeros((n, W), np.uint64), phase=np.zeros(n, np.int8),
                inputs=np.array([0], np.int32), outputs=np.array([1], np.int32), bnd_is_h=None)
    sv = zx.Server(64 << 20, max_batch=4)
    with pytest.raises(zx.ZxError) as e:
        sv.submit(d)
    assert e.value.code == zx.ZX_ECAPACITY
    sv.close()
