"""Generalised flow on the GPU (zx_gflow) against the oracle's layers
(oracle.extract.gflow_layers): circuit-derived diagrams (exponentiated
Pauli strings; these have a flow) before and after simplification, and
random diagrams (most of which have none), layer by layer."""
import numpy as np
import pytest

import oracle
from oracle import extract as ox
from workloads import batch_diagram, single_diagram
from workloads.circuits import circuit_workload

pytestmark = pytest.mark.gpu


def check(zx, ds, simplify):
    gs = [zx.Graph.from_diagram(d) for d in ds]
    if simplify:
        zx.simplify(gs, extract=False)
    exists, layers = zx.gflow(gs)
    seen = set()
    for i, d in enumerate(ds):
        og = oracle.Graph.from_diagram(d)
        if simplify:
            og.simplify()
        ex, lay = ox.gflow_layers(og)
        assert exists[i] == int(ex), (i, d.n)
        np.testing.assert_array_equal(layers[i], lay, err_msg=str((i, d.n)))
        seen.add(bool(ex))
    return seen


@pytest.mark.parametrize("simplify", [False, True])
def test_circuit_diagrams(zx, simplify):
    ds = [circuit_workload(7, i) for i in range(60)]
    print("flow circuits", [d.n for d in ds[:10]], flush=True)
    assert check(zx, ds, simplify) == {True}


def test_random_diagrams(zx):
    ds = [single_diagram(s) for s in range(1, 41)] + [batch_diagram(3, i) for i in range(24)]
    print("flow random", [d.n for d in ds[-24:]], flush=True)
    check(zx, ds, True)
    check(zx, ds[:20], False)


def test_capacity(zx):
    from workloads import serve_diagram
    from workloads.generators import serve_params
    i = next(i for i in range(1000) if serve_params(5, i)[1] > 1024)
    g = zx.Graph.from_diagram(serve_diagram(5, i))
    with pytest.raises(zx.ZxError):
        zx.gflow([g])
