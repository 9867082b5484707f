"""Write large_diagrams.json: the oracle's simplification of serving-stream
diagrams with several thousand spiders, for GPU tests whose oracle run would
take minutes (N = 8000 takes about three minutes of plain C).

Calls only the oracle and the seeded generators.  Each entry holds the
request (stream seed, item), its size, the oracle's counts and SHA-256
digests of the final adjacency rows, phases, alive mask, trace and frontier
rows (numpy's native little-endian bytes).

    python tests/golden/make_large_diagrams.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import serve_diagram, serve_params  # noqa: E402

SEED = 5
TARGETS = [2048, 3000, 4096, 5000, 6500, 8000]


def digest(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()


def pick_items():
    items, seen = [], set()
    for t in TARGETS:
        for i in range(50000):
            _, n, _ = serve_params(SEED, i)
            if abs(n - t) <= 200 and i not in seen:
                items.append(i)
                seen.add(i)
                break
    return items


def main():
    out = []
    for i in pick_items():
        d = serve_diagram(SEED, i)
        t0 = time.time()
        g = oracle.Graph.from_diagram(d)
        assert g.simplify() == oracle.OK
        M, piv, rank, ops = g.frontier()
        dt = time.time() - t0
        out.append(dict(seed=SEED, item=i, n=int(d.n), q=int(len(d.outputs)),
                        n_edges=int(g.n_edges()), n_alive=len(g.alive_list()),
                        pow_sqrt2=int(g.scalar.pow_sqrt2), phase8=int(g.scalar.phase8 % 8),
                        fill_in=int(g.scalar.fill_in), rounds=int(g.rounds), n_trace=int(len(g.trace)),
                        rank=int(rank), rowops=int(ops),
                        sha_adj=digest(g.adj), sha_phase=digest(g.k), sha_alive=digest(g.alive),
                        sha_trace=digest(g.trace.astype("<i4")), sha_front=digest(M),
                        sha_fpiv=digest(piv.astype("<i4"))))
        print("item %d n %d: %.1f s" % (i, d.n, dt), flush=True)
    with open(os.path.join(HERE, "large_diagrams.json"), "w") as f:
        json.dump({"generator": "serve_diagram(seed, item)", "entries": out}, f, indent=1)


if __name__ == "__main__":
    main()
