"""Parameterized Pauli spiders on the GPU against the oracle: simplification
with parameter rows (LDS and arena modes, single rewrites), the recorded
phase-pair terms, and the minimal parameter basis (zx_gf2_basis), all bit
for bit."""
import numpy as np
import pytest

import oracle
from oracle.params import dependency_vectors, fbasis
from workloads import batch_diagram, param_rows, serve_diagram, single_diagram

pytestmark = pytest.mark.gpu


def _pair(zx, d, n_params, seed):
    prm = param_rows(seed, 0, d.n, n_params)
    g = zx.Graph.create(d.adj, d.phase, d.inputs, d.outputs, d.bnd_is_h, n_params=n_params, params=prm)
    og = oracle.Graph(d.n, d.adj, d.phase, d.inputs, d.outputs, d.bnd_is_h, params=prm)
    return g, og


def _same(g, og):
    adj, ph, al, info = g.read()
    assert np.array_equal(adj, og.adj) and np.array_equal(ph, og.k) and np.array_equal(al, og.alive)
    assert info.pow_sqrt2 == og.scalar.pow_sqrt2 and info.phase8 == og.scalar.phase8 % 8
    rows, kab, u, v = g.params()
    tk, tu, tv = og.terms()
    assert np.array_equal(rows, og.params)
    assert np.array_equal(kab, tk) and np.array_equal(u, tu) and np.array_equal(v, tv), (len(kab), len(tk))


@pytest.mark.parametrize("case", ["one64_p1", "one64_p64", "batch_p130", "batch_p4096", "big_p70"])
def test_simplify_with_parameters(zx, case):
    import torch
    print("params case", case, flush=True)
    gens = {"one64_p1": (lambda i: single_diagram(300 + i), 1),
            "one64_p64": (lambda i: single_diagram(400 + i), 64),
            "batch_p130": (lambda i: batch_diagram(71, i), 130),
            "batch_p4096": (lambda i: batch_diagram(72, i, q_lo=4, q_hi=16), 4096),
            "big_p70": (lambda i: serve_diagram(73, i, q_lo=100, q_hi=150), 70)}
    gen, P = gens[case]
    n_items = 2 if case == "big_p70" else 12
    pairs = [_pair(zx, gen(i), P, 1000 + i) for i in range(n_items)]
    zx.simplify([g for g, _ in pairs], extract=True)
    torch.cuda.synchronize()
    for i, (g, og) in enumerate(pairs):
        assert og.simplify() == oracle.OK
        assert g.status() == 0, i
        _same(g, og)
        assert np.array_equal(g.trace(), og.trace), i
        # reset + rerun reproduces the same parameter state
    g, og = pairs[0]
    g.reset()
    zx.simplify([g], extract=False)
    torch.cuda.synchronize()
    _same(g, og)


def test_single_rewrites_with_parameters(zx):
    import torch
    rng = np.random.default_rng(5)
    d = batch_diagram(74, 3, q_lo=4, q_hi=8)
    g, og = _pair(zx, d, 100, 77)
    done = 0
    for _ in range(60):
        cands = [v for v in range(d.n) if og.is_alive(v) and not og.has_boundary(v)]
        lc = [v for v in cands if og.k[v] % 4 == 2]
        pv = [(a, b) for a in cands for b in cands if a < b and og.k[a] % 4 == 0 and og.k[b] % 4 == 0
              and og.edge(a, b)]
        if lc and (rng.random() < 0.5 or not pv):
            u = int(rng.choice(lc))
            assert og.local_comp(u) == oracle.OK
            g.local_comp(u)
        elif pv:
            a, b = pv[int(rng.integers(0, len(pv)))]
            assert og.pivot(a, b) == oracle.OK
            g.pivot(a, b)
        else:
            break
        done += 1
    torch.cuda.synchronize()
    assert done > 3 and g.status() == 0
    _same(g, og)


@pytest.mark.parametrize("seed,P", [(1, 64), (2, 300), (3, 4096)])
def test_fbasis_matches_oracle(zx, seed, P):
    import torch
    d = batch_diagram(75, seed, q_lo=30, q_hi=60)
    g, og = _pair(zx, d, P, 500 + seed)
    assert og.simplify() == oracle.OK
    D = dependency_vectors(og)
    if D.shape[0] == 0:
        pytest.skip("no dependency vectors")
    T, coeff, piv, r = fbasis(D, P)
    R, rank, pv, cf = zx.gf2_basis(zx.to_device_words(D), P)
    torch.cuda.synchronize()
    assert int(rank.item()) == r
    assert np.array_equal(zx.to_host_words(R)[:r], T)
    assert np.array_equal(pv.cpu().numpy()[:r], piv)
    got = zx.to_host_words(cf)
    cw = coeff.shape[1]
    assert got.shape[1] >= cw
    assert np.array_equal(got[:, :cw], coeff) and not got[:, cw:].any()
