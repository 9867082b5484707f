"""Learned proposal on the GPU vs the oracle: the network kernels (sync,
forward, loss, backward, Adam) against oracle/mlp.py, round-limited and
resumed simplification, rollouts (features, moves, costs) and learned
simplification checked by trace replay."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
from oracle import policy as opol
from workloads import batch_diagram, single_diagram

pytestmark = pytest.mark.gpu


def rand_param(rng, scale=0.3):
    return (rng.standard_normal(omlp.NPARAM) * scale).astype(np.float32)


def make_mlp(zx, p):
    return zx.MLP(torch.from_numpy(p).cuda())


def bf16_bits(x):
    return (omlp.bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def test_mlp_sync_bits(zx):
    rng = np.random.default_rng(0)
    p = rand_param(rng)
    m = make_mlp(zx, p)
    got = m.wbf16.cpu().numpy().view(np.uint16)
    W1, _, w2, _ = omlp.unpack(p)
    np.testing.assert_array_equal(got[: omlp.IN * omlp.HID].reshape(omlp.HID, omlp.IN), bf16_bits(W1).T)
    np.testing.assert_array_equal(got[omlp.IN * omlp.HID:], bf16_bits(w2))


@pytest.mark.parametrize("rows", [1, 31, 32, 33, 1000, 4097])
def test_mlp_forward(zx, rows):
    rng = np.random.default_rng(rows)
    p = rand_param(rng)
    m = make_mlp(zx, p)
    X = bf16_bits(rng.standard_normal((rows, omlp.IN)).astype(np.float32))
    print("forward rows", rows, flush=True)
    s = m.forward(torch.from_numpy(X.view(np.int16)).cuda()).cpu().numpy()
    ref, _ = omlp.forward(p, X)
    # fp32 sums of 16 and 256 terms
    np.testing.assert_allclose(s, ref, rtol=1e-5, atol=1e-5)


def test_mlp_loss(zx):
    rng = np.random.default_rng(1)
    seg = np.array([0, 5, 5, 40, 41, 140, 200], np.int32)
    R = int(seg[-1])
    score = rng.standard_normal(R).astype(np.float32) * 3
    cost = rng.integers(0, 6, R).astype(np.int64)
    cost[rng.choice(R, 20, replace=False)] = -1
    cost[40] = -1  # a segment with no present row
    ds, loss = zx.MLP.loss(torch.from_numpy(score).cuda(), torch.from_numpy(cost).cuda(),
                           torch.from_numpy(seg).cuda())
    rl, rds = omlp.loss_and_dscore(score.astype(np.float64), cost, seg)
    np.testing.assert_allclose(loss.cpu().numpy(), rl, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(ds.cpu().numpy(), rds, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("rows", [40, 5000, 70000])
def test_mlp_backward_gradcheck(zx, rows):
    rng = np.random.default_rng(rows)
    p = rand_param(rng)
    m = make_mlp(zx, p)
    X = bf16_bits(rng.standard_normal((rows, omlp.IN)).astype(np.float32))
    d = (rng.standard_normal(rows) / rows).astype(np.float32)
    xt = torch.from_numpy(X.view(np.int16)).cuda()
    dt = torch.from_numpy(d).cuda()
    print("backward rows", rows, flush=True)
    g1 = m.backward(xt, dt).clone().cpu().numpy()
    g2 = m.backward(xt, dt).clone().cpu().numpy()
    np.testing.assert_array_equal(g1, g2)  # fixed reduction order
    ref = omlp.backward(p, X, d.astype(np.float64))
    # bf16-rounded operands on both sides, fp32 sums here: relative error
    # 1e-3 of the gradient's scale
    scale = np.abs(ref).max()
    assert np.abs(g1 - ref).max() <= 1e-3 * scale, np.abs(g1 - ref).max() / scale
    assert np.linalg.norm(g1 - ref) <= 1e-4 * np.linalg.norm(ref)


def test_mlp_adam(zx):
    rng = np.random.default_rng(2)
    p = rand_param(rng)
    m = make_mlp(zx, p)
    rp, rm, rv = p.astype(np.float64), np.zeros(omlp.NPARAM), np.zeros(omlp.NPARAM)
    for step in range(1, 4):
        g = rng.standard_normal(omlp.NPARAM).astype(np.float32)
        m.adam(lr=1e-2, grad=torch.from_numpy(g).cuda())
        rp, rm, rv = omlp.adam(rp, g, rm, rv, step, 1e-2)
    np.testing.assert_allclose(m.param.cpu().numpy(), rp, rtol=1e-5, atol=1e-6)
    got = m.wbf16.cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got[omlp.IN * omlp.HID:],
                                  bf16_bits(m.param.cpu().numpy()[omlp.P_W2:omlp.P_B2]))


def compare_state(zg, og, ctx=""):
    adj, ph, al, info = zg.read()
    assert info.status == 0, ctx
    assert np.array_equal(al, og.alive), ctx
    assert np.array_equal(adj, og.adj), ctx
    assert np.array_equal(ph, og.k), ctx
    assert info.pow_sqrt2 == og.scalar.pow_sqrt2, ctx
    assert info.phase8 == og.scalar.phase8 % 8, ctx
    assert info.fill_in == og.scalar.fill_in, ctx
    return info


@pytest.mark.parametrize("item", range(6))
def test_round_limited_and_resume(zx, item):
    d = batch_diagram(41, item)
    full = oracle.Graph.from_diagram(d)
    full.simplify()
    for r in [1, 2, 5]:
        og = oracle.Graph.from_diagram(d)
        og.simplify(max_rounds=r)
        zg = zx.Graph.from_diagram(d)
        print("round-limited", item, d.n, r, flush=True)
        zx.simplify([zg], extract=False, max_rounds=r)
        info = compare_state(zg, og, (item, r))
        assert info.rounds == og.rounds
        np.testing.assert_array_equal(zg.trace(), og.trace)
        zx.simplify([zg], extract=True, resume=True)
        compare_state(zg, full, (item, r, "resumed"))
        np.testing.assert_array_equal(zg.trace(), full.trace)
        _, _, rank, ops = full.frontier()
        info = zg.info()
        assert info.rank == rank and info.rowops == ops


def pivot_phase_round(d):
    """Index of the first pivot round of the oracle's canonical schedule (None
    when it has none)."""
    full = oracle.Graph.from_diagram(d)
    full.simplify()
    tr = full.trace
    piv = tr[tr[:, 1] == 1]
    return int(piv[0, 0]) if len(piv) else None


def pauli_only(d):
    """The diagram with every interior phase of class pi/2 moved to the Pauli
    class (k + 2 mod 8): no LC candidate, so the first round is a pivot round."""
    import dataclasses
    bnd = set(int(v) for v in d.inputs) | set(int(v) for v in d.outputs)
    ph = d.phase.copy()
    for v in range(d.n):
        if v not in bnd and ph[v] % 4 == 2:
            ph[v] = (ph[v] + 2) % 8
    return dataclasses.replace(d, phase=ph)


@pytest.mark.parametrize("item", range(5))
def test_rollout_parity(zx, item):
    # item 2 (diagram 102, 44 spiders) is the one case here whose states have
    # fewer candidates than slots (4 and 0 against 6): the empty-slot path
    # that the structured per-item branch of the rollout kernel now covers.
    # The last state is the first pivot round's: its candidates are edges.
    d = batch_diagram(41, 100 + item)
    states_o, states_z = [], []
    rp = pivot_phase_round(d)
    for r in [0, 1, 3] + ([rp] if rp else []):
        og = oracle.Graph.from_diagram(d)
        og.simplify(max_rounds=r) if r else None
        if og.rounds < r:
            continue
        zg = zx.Graph.from_diagram(d)
        if r:
            zx.simplify([zg], extract=False, max_rounds=r)
        states_o.append(og)
        states_z.append(zg)
    K = 6
    print("rollout", item, d.n, len(states_z), rp, flush=True)
    cost, fill, move, feats = zx.rollout(states_z, K)
    cost, fill, move = cost.cpu().numpy(), fill.cpu().numpy(), move.cpu().numpy()
    feats = feats.cpu().numpy().view(np.uint16)
    kinds = set()
    for si, og in enumerate(states_o):
        ent = opol.candidate_list(og)
        C = len(ent)
        for k in range(K):
            i = si * K + k
            if k >= C:
                assert cost[i] == -1 and move[i, 0] == -1
                continue
            u, v = ent[k if C <= K else (k * C) // K]
            kinds.add(v >= 0)
            assert tuple(move[i]) == (1 if v >= 0 else 0, u, v), (si, k)
            np.testing.assert_array_equal(feats[i], opol.features(og, (u, v)), err_msg=str((si, k)))
            rc, rf = opol.rollout(og, (u, v))
            assert cost[i] == rc and fill[i] == rf, (si, k, cost[i], rc)
        # the states themselves were not modified
        compare_state(states_z[si], og, ("state", si))
    if rp:
        assert True in kinds


def learned_run(zx, diagrams, p, **kw):
    m = make_mlp(zx, p)
    gs = [zx.Graph.from_diagram(d) for d in diagrams]
    zx.simplify(gs, extract=True, policy=zx.ZX_POLICY_LEARNED, mlp=m, **kw)
    return gs


@pytest.mark.parametrize("seed", [0, 1])
def test_learned_simplify_replays(zx, seed):
    rng = np.random.default_rng(10 + seed)
    p = rand_param(rng, 0.5)
    diagrams = [batch_diagram(42, i) for i in range(24)] + [single_diagram(s) for s in range(4)]
    print("learned batch", seed, len(diagrams), flush=True)
    gs = learned_run(zx, diagrams, p)
    again = learned_run(zx, diagrams, p)
    for i, (d, zg) in enumerate(zip(diagrams, gs)):
        tr = zg.trace()
        np.testing.assert_array_equal(tr, again[i].trace())  # deterministic
        g0 = oracle.Graph.from_diagram(d)
        fin = opol.replay(g0, tr)
        compare_state(zg, fin, ("learned", i))
        cur = g0.copy()
        for r in range(zg.info().rounds):
            sel = tr[tr[:, 0] == r]
            piv = bool(sel[0, 1])
            assert opol.round_is_valid(cur, [(int(u), int(v)) for _, _, u, v in sel], piv), (i, r)
            for _, _, u, v in sel:
                assert (cur.pivot(int(u), int(v)) if piv else cur.local_comp(int(u))) == oracle.OK
        _, _, rank, ops = fin.frontier()
        info = zg.info()
        assert info.rank == rank and info.rowops == ops, i
    # one diagram alone gives the same trace as inside the batch
    solo = learned_run(zx, diagrams[3:4], p)[0]
    np.testing.assert_array_equal(solo.trace(), gs[3].trace())


def test_learned_first_round_follows_scores(zx):
    """The first LC round takes candidates in descending score order (oracle
    features and float64 scores), checked where no two scores are close."""
    rng = np.random.default_rng(5)
    p = rand_param(rng, 0.5)
    checked = 0
    for i in range(80):
        d = batch_diagram(42, 200 + i, q_hi=24)
        g0 = oracle.Graph.from_diagram(d)
        ent = opol.candidate_list(g0)
        if not ent:
            continue
        X = np.stack([opol.features(g0, u) for u, _ in ent])
        s, _ = omlp.forward(p, X)
        srt = np.sort(s)
        # fp32 sums on the GPU vs float64 here: about 1e-6 relative
        if len(s) > 1 and np.min(np.diff(srt)) < 1e-4 * max(1.0, np.abs(s).max()):
            continue
        order = sorted(range(len(ent)), key=lambda j: (-s[j], j))
        taken = []
        for j in order:
            u = ent[j][0]
            if not any(g0.edge(u, t) for t in taken):
                taken.append(u)
        zg = learned_run(zx, [d], p, max_rounds=1)[0]
        tr = zg.trace()
        assert sorted(int(u) for u in tr[:, 2]) == sorted(taken), i
        checked += 1
    assert checked >= 5


def test_learned_pivot_round_follows_scores(zx):
    """A pivot round takes the listed edges in descending score order (oracle
    features and float64 scores) unless an end is taken or adjacent to a
    taken end, then completes canonically: pair for pair, in order, where no
    two scores are close."""
    rng = np.random.default_rng(6)
    p = rand_param(rng, 0.5)
    checked = 0
    for i in range(120):
        d = pauli_only(batch_diagram(42, 400 + i, q_hi=24))
        g0 = oracle.Graph.from_diagram(d)
        ent = opol.candidate_list(g0)
        if len(ent) < 2:
            continue
        assert all(v >= 0 for _, v in ent)
        X = np.stack([opol.features(g0, e) for e in ent])
        s, _ = omlp.forward(p, X)
        srt = np.sort(s)
        if np.min(np.diff(srt)) < 1e-4 * max(1.0, np.abs(s).max()):
            continue
        order = sorted(range(len(ent)), key=lambda j: (-s[j], j))
        pairs = opol.pivot_round_in_order(g0, [ent[j] for j in order])
        zg = learned_run(zx, [d], p, max_rounds=1)[0]
        tr = zg.trace()
        assert (tr[:, 1] == 1).all() and (tr[:, 0] == 0).all(), i
        assert [(int(u), int(v)) for _, _, u, v in tr] == pairs, i
        checked += 1
    assert checked >= 5


def test_learned_pivot_runs_replay(zx):
    """Learned runs that are pivot rounds from the start, checked round by
    round (valid and maximal) and by replay."""
    rng = np.random.default_rng(8)
    p = rand_param(rng, 0.5)
    ds = [pauli_only(batch_diagram(42, 600 + i)) for i in range(16)]
    gs = learned_run(zx, ds, p)
    n_piv = 0
    for i, (d, zg) in enumerate(zip(ds, gs)):
        tr = zg.trace()
        g0 = oracle.Graph.from_diagram(d)
        fin = opol.replay(g0, tr)
        compare_state(zg, fin, ("pivot-learned", i))
        cur = g0.copy()
        for r in range(zg.info().rounds):
            sel = tr[tr[:, 0] == r]
            piv = bool(sel[0, 1])
            n_piv += piv
            assert opol.round_is_valid(cur, [(int(u), int(v)) for _, _, u, v in sel], piv), (i, r)
            for _, _, u, v in sel:
                assert (cur.pivot(int(u), int(v)) if piv else cur.local_comp(int(u))) == oracle.OK
    assert n_piv >= 16


@pytest.mark.parametrize("item", range(6))
def test_policy_features_match_oracle(zx, item):
    """zx_policy_features: the next round's candidates (LC spiders ascending,
    then pivot edges) and their features equal the oracle's, bit for bit, at
    the start, after some rounds, at the first pivot round and at the fixed
    point (none)."""
    d = batch_diagram(43, 300 + item, q_hi=24)
    full = oracle.Graph.from_diagram(d)
    full.simplify()
    rp = pivot_phase_round(d)
    for r in [0, 1, 2, full.rounds] + ([rp] if rp else []):
        og = oracle.Graph.from_diagram(d)
        if r:
            og.simplify(max_rounds=r)
        zg = zx.Graph.from_diagram(d)
        if r:
            zx.simplify([zg], extract=False, max_rounds=r)
        print("features", item, d.n, r, flush=True)
        cand, feats, C = zx.policy_features(zg)
        ent = opol.candidate_list(og)
        assert C == len(ent), (item, r)
        assert [tuple(int(x) for x in e) for e in cand.cpu().numpy()] == ent
        fb = feats.cpu().numpy().view(np.uint16)
        for i, e in enumerate(ent):
            np.testing.assert_array_equal(fb[i], opol.features(og, e), err_msg=str((item, r, e)))
    # a short output buffer gets the first rows and the full count
    zg = zx.Graph.from_diagram(d)
    cand, feats, C = zx.policy_features(zg, max_cand=2)
    assert C == len(opol.candidate_list(oracle.Graph.from_diagram(d))) and len(cand) == min(C, 2)


def replay_and_compare(zg, d, ctx):
    tr = zg.trace()
    g0 = oracle.Graph.from_diagram(d)
    fin = opol.replay(g0, tr)
    compare_state(zg, fin, ctx)
    _, _, rank, ops = fin.frontier()
    info = zg.info()
    assert info.rank == rank and info.rowops == ops, ctx


def test_learned_arena_mode_replays(zx):
    """Learned runs on diagrams of 1190 to 1952 spiders (adjacency in the arena,
    not in LDS), checked by replaying their traces on the oracle."""
    rng = np.random.default_rng(21)
    p = rand_param(rng, 0.5)
    items = [8, 13, 19]
    ds = [batch_diagram(42, i, q_lo=100, q_hi=128) for i in items]
    assert all(1100 <= d.n <= 2048 for d in ds)
    print("learned arena", [d.n for d in ds], flush=True)
    gs = learned_run(zx, ds, p)
    for i, (zg, d) in enumerate(zip(gs, ds)):
        assert zg.info().policy == zx.ZX_POLICY_LEARNED
        replay_and_compare(zg, d, ("arena", items[i], d.n))


def gate2q(info):
    return int(info.n_edges) + int(info.rowops)


def test_fallback_keeps_the_cheaper_schedule(zx):
    """ZX_FALLBACK: each arena ends with the learned result unless the greedy
    one has lower gate2q, bit for bit as the separate runs, and says which."""
    rng = np.random.default_rng(22)
    p = rand_param(rng, 0.5)
    ds = [batch_diagram(42, i, q_lo=32, q_hi=128) for i in range(40)]
    m = make_mlp(zx, p)
    G = [zx.Graph.from_diagram(d) for d in ds]
    L = [zx.Graph.from_diagram(d) for d in ds]
    F = [zx.Graph.from_diagram(d) for d in ds]
    print("fallback", [d.n for d in ds], flush=True)
    zx.simplify(G, extract=True)
    zx.simplify(L, extract=True, policy=zx.ZX_POLICY_LEARNED, mlp=m)
    zx.simplify(F, extract=True, policy=zx.ZX_POLICY_LEARNED, mlp=m, fallback=True)
    kinds = set()
    for i in range(len(ds)):
        gi, li = G[i].info(), L[i].info()
        exp, pol = (L[i], zx.ZX_POLICY_LEARNED) if gate2q(li) <= gate2q(gi) else (G[i], zx.ZX_POLICY_GREEDY)
        kinds.add(pol)
        fa, fp, fl, fi = F[i].read()
        ea, ep, el, ei = exp.read()
        assert fi.status == 0 and fi.policy == pol, i
        assert np.array_equal(fa, ea) and np.array_equal(fp, ep) and np.array_equal(fl, el), i
        for f in ("pow_sqrt2", "phase8", "n_edges", "n_alive", "fill_in", "rounds", "n_trace", "rank", "rowops"):
            assert getattr(fi, f) == getattr(ei, f), (i, f)
        np.testing.assert_array_equal(F[i].trace(), exp.trace())
        assert np.array_equal(F[i].frontier()[0], exp.frontier()[0])
    assert kinds == {zx.ZX_POLICY_LEARNED, zx.ZX_POLICY_GREEDY}, kinds
    # the kept learned results are exact rewrites (oracle replay)
    for i in range(6):
        if F[i].info().policy == zx.ZX_POLICY_LEARNED:
            replay_and_compare(F[i], ds[i], ("fallback", i))


def test_fallback_rejects_partial_schedules(zx):
    m = make_mlp(zx, rand_param(np.random.default_rng(3)))
    g = zx.Graph.from_diagram(batch_diagram(42, 0))
    with pytest.raises(zx.ZxError):
        zx.simplify([g], policy=zx.ZX_POLICY_LEARNED, mlp=m, fallback=True, max_rounds=2)


def test_serve_learned_with_fallback(zx):
    """The server with the learned policy and the greedy fallback answers each
    request with the stand-alone ZX_FALLBACK result of the same diagram."""
    import time
    from workloads import serve_diagram
    rng = np.random.default_rng(23)
    m = make_mlp(zx, rand_param(rng, 0.5))
    ds = [serve_diagram(5, 3000 + i, q_hi=128) for i in range(48)]
    ref = [zx.Graph.from_diagram(d) for d in ds]
    zx.simplify(ref, extract=True, policy=zx.ZX_POLICY_LEARNED, mlp=m, fallback=True)
    sv = zx.Server(512 << 20, policy=zx.ZX_POLICY_LEARNED, mlp=m, fallback=True)
    print("serve learned", [d.n for d in ds], flush=True)
    for i, d in enumerate(ds):
        assert sv.submit(d, tag=i) is not None
    res = []
    t0 = time.time()
    while len(res) < len(ds):
        res += sv.poll()
        assert time.time() - t0 < 100, "server did not finish"
    pols = set()
    for r in res:
        e = ref[r.tag].info()
        ctx = (r.tag, ds[r.tag].n)
        assert r.status == 0 and e.status == 0, ctx
        for f in ("n_edges", "n_alive", "pow_sqrt2", "phase8", "fill_in", "rounds", "n_trace", "rank", "rowops",
                  "policy"):
            assert getattr(r, f) == getattr(e, f), (ctx, f)
        assert r.t_submit <= r.t_launch <= r.t_done and r.t_device > 0, ctx
        pols.add(r.policy)
    assert zx.ZX_POLICY_LEARNED in pols
    sv.close()


def test_training_gains(zx):
    """What training buys: on held-out states of other diagrams the trained
    network's loss is below the untrained one's, and on held-out diagrams its
    schedule toggles fewer edges on (fill-in) than the greedy schedule, while
    the greedy fallback keeps gate2q at or below greedy's on every diagram
    (every result an exact rewrite sequence: the fallback test replays them)."""
    from paper_2604_01059_amd import learned
    mlp = learned.new_network()
    feats, costs = learned.make_dataset(6000, per_state=16)
    vf, vc = learned.make_dataset(2000, per_state=16, first_item=1 << 20)
    before = learned.state_metrics(mlp, vf, vc)
    ev0 = learned.evaluate(mlp, n=128)
    learned.train(mlp, feats, costs, epochs=4)
    after = learned.state_metrics(mlp, vf, vc)
    ev = learned.evaluate(mlp, n=128)
    print("held-out before", before, "after", after, flush=True)
    print("eval untrained", ev0, "trained", ev, flush=True)
    assert after["loss"] < before["loss"] - 0.01
    assert after["top1_least_cost"] > after["random_least_cost"]
    assert ev["fill_learned"] < ev["fill_greedy"]
    assert ev["fallback_equals_min"] and ev["gate2q_fallback"] <= ev["gate2q_greedy"]
