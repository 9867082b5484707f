"""Learned rewrite proposal: training data from greedy runs, training with the
library's network kernels, evaluation against the greedy schedule.

The paper applies its two rules (appendix "Rewrite rules") greedily to the
fixed point (appendix "Stabilizer decompositions") and says nothing on the
order; a different order reaches a different, equally valid fixed point with
a different cost.  This module learns an order.

* State: a diagram at the start of a round of a greedy run.
* Candidates: the local-complementation candidates of the round, or in a
  pivot round the candidate edges between Pauli spiders (``zx.rollout``
  lists them as the learned schedule does).
* Label of a candidate: its rollout cost -- apply it, finish greedily, and
  count the edges the run toggled on (fill-in, the default) or the Hadamard
  edges left plus frontier row additions (gate2q) (``zx.rollout``).  The
  features carry next to no information on the gate2q label (within-state
  rank correlations below 0.03), and some on the fill-in label (about
  0.18 for the degree).
* Loss: softmax cross-entropy of the scores of a state's candidates toward
  its cheapest candidate (``zx_mlp_loss``).
* Use: ``policy=ZX_POLICY_LEARNED`` takes each round's candidates in
  descending score order (a pivot round then completes canonically, so it
  stays maximal); with ``ZX_FALLBACK`` the library keeps, per
  diagram, the cheaper of the learned and the greedy result
  (``simplify_with_fallback``).

Every step runs in the HIP library; this module only moves tensors.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import zx

TRAIN_SEED = 41
EVAL_SEED = 42


def gate2q(info) -> int:
    """Hadamard edges left plus the row additions of the output frontier."""
    return int(info.n_edges) + int(info.rowops)


def new_network(seed: int = TRAIN_SEED) -> zx.MLP:
    from workloads import network_init
    return zx.MLP(torch.from_numpy(network_init(seed)))


def greedy_states(diagrams, max_states=None):
    """Snapshots of every round start of the greedy runs of ``diagrams``
    (states at their fixed point are dropped)."""
    graphs = [zx.Graph.from_diagram(d) for d in diagrams]
    states = []
    r = 0
    active = graphs
    while active:
        snaps = [g.snapshot() for g in active]
        zx.simplify(active, extract=False, max_rounds=r + 1, resume=True)
        nxt = []
        for g, s in zip(active, snaps):
            if g.info().rounds > r:
                states.append(s)
                nxt.append(g)
        active = nxt
        r += 1
        if max_states is not None and len(states) >= max_states:
            break
    return states[:max_states] if max_states is not None else states


def make_dataset(n_states: int, per_state: int = 16, seed: int = TRAIN_SEED, chunk: int = 128,
                 log=None, informative: bool = True, first_item: int = 0, label: str = "fill"):
    """(features, costs) for n_states states of greedy runs on the batched
    generator's diagrams (items first_item, first_item + 1, ...): features
    (n_states * per_state, 16) int16 bf16 bits, costs (n_states * per_state,)
    int64 (-1 = no candidate in that slot).  label: the rollout's fill-in
    ("fill", edges toggled on from the candidate to the fixed point) or its
    gate2q ("gate2q").  informative: keep only states whose candidates do not
    all cost the same (a state of equal costs gives every order the same
    target and teaches nothing)."""
    assert label in ("fill", "gate2q")
    from workloads import batch_diagram
    feats, costs = [], []
    have, item = 0, first_item
    t0 = time.time()
    while have < n_states:
        ds = [batch_diagram(seed, item + i) for i in range(chunk)]
        item += chunk
        states = greedy_states(ds, max_states=n_states - have)
        if not states:
            continue
        if log:
            log("dataset: %d round-start states from diagrams %d..%d, %.1f s"
                % (len(states), item - chunk, item - 1, time.time() - t0))
        cost, fill, _, f = zx.rollout(states, per_state)
        if label == "fill":
            cost = torch.where(cost >= 0, fill, cost)
        # a state whose slots are all empty teaches nothing: drop it
        cv = cost.view(-1, per_state)
        present = cv >= 0
        keep = present.any(dim=1)
        if informative:
            big = torch.iinfo(torch.int64).max
            lo = torch.where(present, cv, torch.full_like(cv, big)).min(dim=1).values
            hi = torch.where(present, cv, torch.full_like(cv, -1)).max(dim=1).values
            keep &= hi > lo
        rows = keep.repeat_interleave(per_state)
        take = int(keep.sum())
        if have + take > n_states:  # the last chunk fills the request exactly
            idx = torch.nonzero(keep).flatten()[n_states - have:]
            keep[idx] = False
            rows = keep.repeat_interleave(per_state)
            take = n_states - have
        feats.append(f[rows])
        costs.append(cost[rows])
        have += take
        del states
        if log:
            log("dataset: %d states, %d diagrams, %.1f s" % (have, item, time.time() - t0))
    return torch.cat(feats), torch.cat(costs)


def state_metrics(mlp: zx.MLP, feats, costs, per_state: int = 16, chunk_states: int = 4096):
    """Held-out quality of the network's ranking over states: mean loss, and
    how often its top-scored candidate is one of the least-cost ones, beside
    the same rate for the lowest-id candidate (the greedy schedule's first
    pick) and for a uniformly random pick."""
    S = costs.numel() // per_state
    dev = feats.device
    seg = torch.arange(0, chunk_states * per_state + 1, per_state, dtype=torch.int32, device=dev)
    tot_loss, hit, first, rand = 0.0, 0.0, 0.0, 0.0
    for b in range(0, S, chunk_states):
        ns = min(chunk_states, S - b)
        x = feats[b * per_state:(b + ns) * per_state].contiguous()
        c = costs[b * per_state:(b + ns) * per_state].contiguous()
        score = mlp.forward(x)
        _, loss = zx.MLP.loss(score, c, seg[:ns + 1].contiguous())
        tot_loss += float(loss.sum())
        cv, sv = c.view(ns, per_state), score.view(ns, per_state)
        present = cv >= 0
        big = torch.iinfo(torch.int64).max
        best = torch.where(present, cv, torch.full_like(cv, big)).min(dim=1, keepdim=True).values
        good = present & (cv == best)
        top = torch.where(present, sv, torch.full_like(sv, -float("inf"))).argmax(dim=1, keepdim=True)
        hit += float(good.gather(1, top).sum())
        first += float(good[:, :1].sum())  # slot 0 holds the lowest-id candidate
        rand += float((good.sum(dim=1).float() / present.sum(dim=1).clamp(min=1).float()).sum())
    return {"states": S, "loss": tot_loss / max(S, 1), "top1_least_cost": hit / max(S, 1),
            "first_candidate_least_cost": first / max(S, 1), "random_least_cost": rand / max(S, 1)}


def train(mlp: zx.MLP, feats, costs, per_state: int = 16, epochs: int = 4, batch_states: int = 128,
          lr: float = 1e-3, seed: int = TRAIN_SEED, log=None, val=None):
    """Adam on the per-state cross-entropy.  Returns the loss curve (mean
    loss of every 20th step) and, with val = (features, costs) of held-out
    states, the held-out loss after every epoch."""
    S = costs.numel() // per_state
    dev = feats.device
    seg = torch.arange(0, batch_states * per_state + 1, per_state, dtype=torch.int32, device=dev)
    ws = None
    gen = torch.Generator().manual_seed(seed)
    curve, val_curve = [], []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(S, generator=gen).to(dev)
        for b in range(0, S - batch_states + 1, batch_states):
            idx = perm[b:b + batch_states]
            rows = (idx[:, None] * per_state + torch.arange(per_state, device=dev)[None]).reshape(-1)
            x = feats[rows].contiguous()
            c = costs[rows].contiguous()
            score = mlp.forward(x)
            ds, loss = zx.MLP.loss(score, c, seg)
            if ws is None:
                ws = torch.empty(zx.load().zx_mlp_workspace_bytes(x.shape[0]), dtype=torch.uint8, device=dev)
            mlp.backward(x, ds, ws=ws)
            mlp.adam(lr=lr)
            step += 1
            if step % 20 == 0:
                curve.append((step, float(loss.mean())))
        if val is not None:
            val_curve.append((ep + 1, state_metrics(mlp, val[0], val[1], per_state)["loss"]))
        if log and curve:
            log("epoch %d: loss %.4f%s" % (ep, curve[-1][1],
                                           ", held-out %.4f" % val_curve[-1][1] if val_curve else ""))
    return (curve, val_curve) if val is not None else curve


def evaluate(mlp: zx.MLP, n: int = 1024, seed: int = EVAL_SEED, q_lo: int = 32, q_hi: int = 128,
             keep_graphs: bool = False):
    """Learned vs greedy on n held-out diagrams: gate2q, fill-in, wall time,
    and the library's greedy fallback (ZX_FALLBACK).  keep_graphs: also
    return the learned and fallback graphs (for replay checks)."""
    from workloads import batch_diagram
    ds = [batch_diagram(seed, i, q_lo=q_lo, q_hi=q_hi) for i in range(n)]
    greedy = [zx.Graph.from_diagram(d) for d in ds]
    learned = [zx.Graph.from_diagram(d) for d in ds]
    fallback = [zx.Graph.from_diagram(d) for d in ds]
    bg, bl, bf = zx.Batch(greedy), zx.Batch(learned), zx.Batch(fallback)
    times = {}
    for name, run in (("greedy", lambda: bg.run()),
                      ("learned", lambda: bl.run(policy=zx.ZX_POLICY_LEARNED, mlp=mlp)),
                      ("fallback", lambda: bf.run(policy=zx.ZX_POLICY_LEARNED, mlp=mlp, fallback=True))):
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1)
    for b, name in ((bg, "greedy"), (bl, "learned"), (bf, "fallback")):
        st = b.status()
        if st != zx.ZX_OK:
            raise zx.ZxError(st, "%s batch failed" % name)
    gi = [g.info() for g in greedy]
    li = [g.info() for g in learned]
    fi = [g.info() for g in fallback]
    cg = np.array([gate2q(i) for i in gi])
    cl = np.array([gate2q(i) for i in li])
    cf = np.array([gate2q(i) for i in fi])
    best = np.minimum(cg, cl)
    out = {
        "diagrams": n,
        "mean_spiders": float(np.mean([d.n for d in ds])),
        "gate2q_greedy": int(cg.sum()),
        "gate2q_learned": int(cl.sum()),
        "gate2q_fallback": int(cf.sum()),
        "fallback_equals_min": bool(np.array_equal(cf, best)),
        "fallback_kept_learned": int(sum(i.policy == zx.ZX_POLICY_LEARNED for i in fi)),
        "gain_learned": float(1 - cl.sum() / cg.sum()),
        "gain_fallback": float(1 - cf.sum() / cg.sum()),
        "learned_better": int((cl < cg).sum()),
        "learned_worse": int((cl > cg).sum()),
        "fill_greedy": int(sum(i.fill_in for i in gi)),
        "fill_learned": int(sum(i.fill_in for i in li)),
        "fill_fallback": int(sum(i.fill_in for i in fi)),
        "ms_greedy": times["greedy"],
        "ms_learned": times["learned"],
        "ms_fallback": times["fallback"],
    }
    if keep_graphs:
        return out, ds, learned, fallback
    return out


def simplify_with_fallback(graphs, mlp: zx.MLP):
    """Simplify each graph with the learned policy and the library's greedy
    fallback (ZX_FALLBACK): the arena keeps the learned result unless the
    greedy one has lower gate2q.  Returns, per graph, True where the learned
    result was kept."""
    zx.simplify(graphs, extract=True, policy=zx.ZX_POLICY_LEARNED, mlp=mlp, fallback=True)
    return [g.info().policy == zx.ZX_POLICY_LEARNED for g in graphs]


def save(mlp: zx.MLP, path: str):
    """Network and optimiser state as safetensors."""
    from safetensors.torch import save_file
    save_file({"param": mlp.param.cpu(), "wbf16": mlp.wbf16.cpu(), "adam_m": mlp.m.cpu(),
               "adam_v": mlp.v.cpu(), "step": torch.tensor([mlp.step], dtype=torch.int64)}, path)


def load(path: str) -> zx.MLP:
    from safetensors.torch import load_file
    t = load_file(path)
    m = zx.MLP(t["param"])
    m.m.copy_(t["adam_m"])
    m.v.copy_(t["adam_v"])
    m.step = int(t["step"][0])
    return m
