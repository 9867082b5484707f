"""Pins of the learned-proposal oracle (oracle/mlp.py, oracle/policy.py)
against independent computations: torch's bf16 conversion, torch float64
layers, autograd, cross-entropy and Adam, finite differences, matrix powers
for the two-hop sets, and the exact tensor evaluator."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp, policy
from oracle.tensor import evaluate_graph
from workloads import single_diagram

rng = np.random.default_rng(7)


def rand_param(scale=0.3):
    return (rng.standard_normal(mlp.NPARAM) * scale).astype(np.float32)


def test_bf16_round_matches_torch():
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 5000),
                        # exact ties: lower 16 bits 0x8000, both parities of bit 16
                        (np.arange(1000, dtype=np.uint32) << 16 | 0x8000).view(np.float32) + 0,
                        np.array([0.0, -0.0, 1.0, -1.0], np.float32)])
    x = x[np.isfinite(x)].astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x).view(np.uint32), ref.view(np.uint32))


def test_forward_matches_torch_layers():
    p = rand_param()
    X = rng.standard_normal((300, mlp.IN)).astype(np.float32)
    s, _ = mlp.forward(p, X)
    W1, b1, w2, b2 = mlp.unpack(p)
    lin1 = torch.nn.Linear(mlp.IN, mlp.HID).double()
    lin2 = torch.nn.Linear(mlp.HID, 1).double()
    with torch.no_grad():
        lin1.weight.copy_(torch.from_numpy(mlp.bf16_round(W1).T.astype(np.float64)))
        lin1.bias.copy_(torch.from_numpy(b1.astype(np.float64)))
        lin2.weight.copy_(torch.from_numpy(mlp.bf16_round(w2).astype(np.float64))[None])
        lin2.bias.fill_(float(b2))
        xt = torch.from_numpy(mlp.bf16_round(X).astype(np.float64))
        ref = lin2(torch.relu(lin1(xt)))[:, 0].numpy()
    np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-12)


def test_backward_matches_autograd_and_finite_differences():
    p = mlp.bf16_round(rand_param())  # bf16-exact weights: rounding is the identity
    X = mlp.bf16_round(rng.standard_normal((64, mlp.IN)).astype(np.float32))
    d = rng.standard_normal(64)
    g = mlp.backward(p, X, d)
    # autograd on the same function
    pt = torch.tensor(p.astype(np.float64), requires_grad=True)
    W1 = pt[: mlp.P_B1].reshape(mlp.IN, mlp.HID)
    b1, w2, b2 = pt[mlp.P_B1:mlp.P_W2], pt[mlp.P_W2:mlp.P_B2], pt[mlp.P_B2]
    s = torch.relu(torch.from_numpy(X.astype(np.float64)) @ W1 + b1) @ w2 + b2
    (s * torch.from_numpy(d)).sum().backward()
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-10)
    # central differences on a sample of parameters (rounding switched off)
    base = p.astype(np.float64)
    for i in rng.choice(mlp.NPARAM, 40, replace=False):
        h = 1e-6
        pp, pm = base.copy(), base.copy()
        pp[i] += h
        pm[i] -= h
        fp = (mlp.forward(pp.astype(np.float32), X, round_weights=False)[0] * d).sum()
        fm = (mlp.forward(pm.astype(np.float32), X, round_weights=False)[0] * d).sum()
        # float32 parameter storage limits the step; compare loosely
        num = (fp - fm) / (np.float32(pp[i]) - np.float32(pm[i]))
        assert abs(num - g[i]) <= 1e-3 * max(1.0, abs(g[i])), (i, num, g[i])


def test_loss_matches_torch_cross_entropy():
    score = rng.standard_normal(40)
    cost = rng.integers(0, 3, 40)  # ties at the least cost are common
    cost[[3, 17, 18]] = -1  # absent rows
    seg = np.array([0, 7, 7, 20, 33, 40])
    loss, ds = mlp.loss_and_dscore(score, cost, seg)
    for i in range(len(seg) - 1):
        rows = [r for r in range(seg[i], seg[i + 1]) if cost[r] >= 0]
        if not rows:
            assert loss[i] == 0
            continue
        best = min(cost[r] for r in rows)
        prob = torch.tensor([1.0 if cost[r] == best else 0.0 for r in rows], dtype=torch.float64)
        prob /= prob.sum()  # even over the least-cost rows
        st = torch.tensor(score[rows], requires_grad=True)
        ref = torch.nn.functional.cross_entropy(st[None], prob[None])
        ref.backward()
        assert abs(loss[i] - ref.item()) < 1e-12
        np.testing.assert_allclose(ds[rows] * (len(seg) - 1), st.grad.numpy(), atol=1e-12)
    assert np.all(ds[[3, 17, 18]] == 0)
    ties = [sum(1 for r in range(seg[i], seg[i + 1]) if cost[r] >= 0 and cost[r] == min(
        [cost[q] for q in range(seg[i], seg[i + 1]) if cost[q] >= 0] or [-9])) for i in range(len(seg) - 1)]
    assert max(ties) >= 2  # the even target over tied rows is exercised


def test_adam_matches_torch():
    p0 = rand_param().astype(np.float64)
    pt = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in range(1, 4):
        g = rng.standard_normal(p0.size)
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = mlp.adam(p, g, m, v, step, 1e-2)
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-12)


def small_graph(n, p_edge, seed):
    r = np.random.default_rng(seed)
    A = np.triu(r.random((n, n)) < p_edge, 1)
    A = A | A.T
    W = (n + 63) // 64
    adj = np.zeros((n, W), np.uint64)
    for i in range(n):
        for j in range(n):
            if A[i, j]:
                adj[i, j // 64] |= np.uint64(1) << np.uint64(j % 64)
    ph = r.integers(0, 8, n).astype(np.int8)
    return oracle.Graph(n, adj, ph, inputs=[0, 1], outputs=[n - 2, n - 1]), A


@pytest.mark.parametrize("seed", range(6))
def test_features_against_matrix_powers(seed):
    g, A = small_graph(30 + seed, 0.15 + 0.05 * seed, seed)
    Ai = A.astype(np.int64)
    two = ((Ai @ Ai) > 0) & ~A & ~np.eye(len(A), dtype=bool)
    N = g.n
    for x in range(g.n):
        f = policy.endpoint_features(g, x, N)
        assert f[0] == np.float32(A[x].sum()) / np.float32(N)
        assert f[5] == np.float32(two[x].sum()) / np.float32(N)
        assert f[4] == np.float32(sum(A[x, b] for b in (0, 1, g.n - 2, g.n - 1))) / np.float32(N)
        assert f[6] == np.float32(sum(1 for y in range(g.n) if A[x, y] and g.k[y] % 4 == 0)) / np.float32(N)
        assert f[1] + f[2] == (1 - g.k[x] % 2) and f[3] == (g.k[x] % 2)


def test_candidate_list_is_the_lc_candidates():
    g, _ = small_graph(40, 0.2, 11)
    ent = policy.candidate_list(g)
    expect = [u for u in range(g.n) if g.k[u] % 4 == 2 and u not in (0, 1, g.n - 2, g.n - 1)]
    assert [u for u, _ in ent] == expect and all(v == -1 for _, v in ent)
    f = policy.features(g, expect[0])
    assert f.dtype == np.uint16 and f.shape == (16,)
    assert np.all(f[7:15] == 0) and f[15] == 0x3F80  # bf16(1.0)
    np.testing.assert_array_equal(policy.features(g, ent[0]), f)


def test_pivot_candidate_list_is_lexicographic_and_capped():
    n = 20  # 16 interior Pauli spiders, complete among themselves: 120 edges > cap 64
    adj = np.zeros((n, 1), np.uint64)
    for i in range(2, 18):
        for j in range(2, 18):
            if i != j:
                adj[i, 0] |= np.uint64(1) << np.uint64(j)
    ph = np.zeros(n, np.int8)
    g = oracle.Graph(n, adj, ph, inputs=[0, 1], outputs=[18, 19])
    ent = policy.candidate_list(g)
    assert len(ent) == 64 == policy.list_cap(n)
    allp = [(u, v) for u in range(2, 18) for v in range(u + 1, 18)]
    assert ent == allp[:64]
    # features of an edge: both endpoints' seven, rule bit 1, constant 1
    f = policy.features(g, ent[5])
    N = n
    from oracle.mlp import bf16_round
    e = policy.endpoint_features(g, ent[5][0], N) + policy.endpoint_features(g, ent[5][1], N)
    expect = (bf16_round(np.array(e + [1.0, 1.0], np.float32)).view(np.uint32) >> 16).astype(np.uint16)
    np.testing.assert_array_equal(f, expect)
    assert f[14] == 0x3F80 and f[15] == 0x3F80
    # the list continues from an LC phase only once it is over
    ph2 = ph.copy()
    ph2[7] = 2
    g2 = oracle.Graph(n, adj, ph2, inputs=[0, 1], outputs=[18, 19])
    assert policy.candidate_list(g2) == [(7, -1)]


def pivot_phase_states(seeds):
    """(state, next round's pairs) at the pivot rounds of the C oracle's
    canonical schedule."""
    out = []
    for seed in seeds:
        d = single_diagram(seed)
        full = oracle.Graph.from_diagram(d)
        full.simplify()
        tr = full.trace
        for r in range(full.rounds):
            sel = tr[tr[:, 0] == r]
            if sel[0, 1] != 1:
                continue
            g = oracle.Graph.from_diagram(d)
            if r:
                g.simplify(max_rounds=r)
            out.append((g, [(int(u), int(v)) for _, _, u, v in sel]))
    return out


def test_canonical_pivot_round_is_the_completion_alone():
    """With nothing listed first, the learned pivot round is the canonical one
    (the C oracle's trace), pair for pair and in order."""
    states = pivot_phase_states(range(1, 9))
    assert len(states) >= 5
    for g, pairs in states:
        assert not policy.lc_candidates(g)
        assert policy.pivot_round_in_order(g, []) == pairs


@pytest.mark.parametrize("seed", range(4))
def test_pivot_rounds_in_any_order_are_valid_and_maximal(seed):
    """Any visiting order of the listed edges, including a list cut short,
    gives a round the independent validity check accepts (pairs disjoint,
    mutually non-adjacent, maximal); the visiting order decides which pairs
    come first."""
    r = np.random.default_rng(seed)
    states = pivot_phase_states(range(1 + 8 * seed, 9 + 8 * seed))
    checked = 0
    for g, _ in states:
        ent = policy.candidate_list(g)
        assert ent and all(v >= 0 for _, v in ent)
        for trial in range(3):
            order = [ent[i] for i in r.permutation(len(ent))]
            if trial == 2:
                order = order[: max(1, len(order) // 3)]
            pairs = policy.pivot_round_in_order(g, order)
            assert policy.round_is_valid(g, pairs, True)
            assert pairs[0] == order[0]
            h = g.copy()
            for u, v in pairs:
                assert h.pivot(u, v) == oracle.OK
            checked += 1
    assert checked >= 6


def test_lc_round_in_order_is_valid():
    for seed in range(1, 6):
        g = oracle.Graph.from_diagram(single_diagram(seed))
        lc = policy.lc_candidates(g)
        if not lc:
            continue
        order = list(reversed(lc))
        taken = policy.lc_round_in_order(g, order)
        assert taken[0] == order[0]
        assert policy.round_is_valid(g, [(u, -1) for u in taken], False)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_canonical_trace_replays_and_rounds_are_valid(seed):
    d = single_diagram(seed)
    g0 = oracle.Graph.from_diagram(d)
    g = g0.copy()
    assert g.simplify() == oracle.OK
    fin = policy.replay(g0, g.trace)
    np.testing.assert_array_equal(fin.adj, g.adj)
    np.testing.assert_array_equal(fin.k, g.k)
    assert fin.scalar.pow_sqrt2 == g.scalar.pow_sqrt2 and fin.scalar.phase8 == g.scalar.phase8
    cur = g0.copy()
    tr = g.trace
    for r in range(g.rounds):
        ent = [(int(u), int(v)) for _, rule, u, v in tr[tr[:, 0] == r]]
        piv = bool(tr[tr[:, 0] == r][0, 1])
        assert policy.round_is_valid(cur, ent, piv)
        for u, v in ent:
            assert (cur.pivot(u, v) if piv else cur.local_comp(u)) == oracle.OK
    # a corrupted trace is rejected
    bad = g.trace.copy()
    bad[0, 2] = next(v for v in range(g0.n) if g0.has_boundary(v))
    with pytest.raises(AssertionError):
        policy.replay(g0, bad)


def test_round_limited_schedule_composes():
    d = single_diagram(4)
    g = oracle.Graph.from_diagram(d)
    full = g.copy()
    full.simplify()
    part = g.copy()
    part.simplify(max_rounds=2)
    assert part.rounds == min(2, full.rounds)
    part.simplify()
    np.testing.assert_array_equal(part.adj, full.adj)
    np.testing.assert_array_equal(part.k, full.k)
    assert part.scalar.pow_sqrt2 == full.scalar.pow_sqrt2


def test_rollout_is_sound_on_a_tiny_diagram():
    # a small diagram whose tensor the exact evaluator can afford
    for seed in range(40):
        g, _ = small_graph(9, 0.45, 100 + seed)
        ent = policy.candidate_list(g)
        if ent:
            break
    amp0 = evaluate_graph(g)
    for u, _ in ent[:4]:
        h = g.copy()
        assert h.local_comp(u) == oracle.OK
        h.simplify()
        assert evaluate_graph(h).equals(amp0)
        cost, _ = policy.rollout(g, u)
        assert cost == policy.gate2q(h)


def test_pivot_rollout_is_sound_on_a_tiny_diagram():
    """A pivot candidate's rollout: the pivot, then the canonical schedule;
    the result has the diagram's exact tensor."""
    found = 0
    for seed in range(400):
        g, _ = small_graph(9, 0.45, 500 + seed)
        if policy.lc_candidates(g):
            continue
        ent = policy.candidate_list(g)
        if not ent:
            continue
        amp0 = evaluate_graph(g)
        for u, v in ent[:3]:
            h = g.copy()
            assert h.pivot(u, v) == oracle.OK
            h.simplify()
            assert evaluate_graph(h).equals(amp0)
            cost, fill = policy.rollout(g, (u, v))
            assert cost == policy.gate2q(h) and fill == h.scalar.fill_in - g.scalar.fill_in
            found += 1
        if found >= 4:
            break
    assert found >= 4
