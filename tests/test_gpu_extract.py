"""Circuit extraction on the GPU (zx_extract) against the oracle's
(oracle.extract.extract_circuit): the gate list, gate by gate, and the input
permutation, on circuit-derived diagrams (which have a flow) before and after
simplification, on larger circuits (20 qubits, depth up to 60), and on
random diagrams, where the status (extracted or refused) must agree too."""
import numpy as np
import pytest

import oracle
from oracle import extract as ox
from workloads import batch_diagram, single_diagram
from workloads.circuits import circuit_workload

pytestmark = pytest.mark.gpu


def reference(d, simplify):
    og = oracle.Graph.from_diagram(d)
    if simplify:
        og.simplify()
    try:
        gates, perm, _ = ox.extract_circuit(og)
        return gates, list(perm)
    except ox.ExtractError:
        return None


def check(zx, ds, simplify):
    gs = [zx.Graph.from_diagram(d) for d in ds]
    if simplify:
        zx.simplify(gs, extract=False)
    res = zx.extract(gs)
    n_ok = 0
    for i, d in enumerate(ds):
        st, gates, perm = res[i]
        ref = reference(d, simplify)
        if ref is None:
            assert st == zx.ZX_ENOMATCH, (i, d.n, st)
            continue
        assert st == zx.ZX_OK, (i, d.n, st)
        assert gates == ref[0], (i, d.n, len(gates), len(ref[0]))
        assert list(perm) == ref[1], (i, d.n)
        n_ok += 1
    return n_ok


@pytest.mark.parametrize("simplify", [False, True])
def test_circuit_diagrams(zx, simplify):
    ds = [circuit_workload(7, i) for i in range(60)]
    print("extract circuits", [d.n for d in ds[:10]], flush=True)
    assert check(zx, ds, simplify) == len(ds)


def test_large_circuits(zx):
    # 20 qubits, up to 60 Pauli exponentials: several hundred spiders, many
    # 64-row blocks of frontier rows and columns
    ds = [circuit_workload(8, i, q_lo=20, q_hi=20, d_lo=30, d_hi=60) for i in range(12)]
    print("extract large circuits", [d.n for d in ds], flush=True)
    assert max(d.n + 2 * len(d.inputs) for d in ds) <= 1024
    assert check(zx, ds, True) == len(ds)
    assert check(zx, ds[:4], False) == 4


def test_wide_circuits(zx):
    # 70-130 qubits: frontiers of two or three 64-qubit blocks with a ragged
    # tail, n + 2 n_in up to about 800
    ds = [circuit_workload(9, i, q_lo=70, q_hi=130, d_lo=40, d_hi=100) for i in range(6)]
    print("extract wide circuits", [(d.n, len(d.inputs)) for d in ds], flush=True)
    assert max(d.n + 2 * len(d.inputs) for d in ds) <= 1024
    assert min(len(d.inputs) for d in ds) > 64
    assert check(zx, ds, True) == len(ds)
    assert check(zx, ds, False) == len(ds)


def test_random_diagrams(zx):
    # diagrams the kernel takes (n + 2 n_in <= 1024; the capacity test covers the rest)
    ds = [single_diagram(s) for s in range(1, 41)] + [batch_diagram(3, i) for i in range(40)]
    ds = [d for d in ds if d.n + 2 * len(d.inputs) <= 1024]
    assert len(ds) >= 60
    print("extract random", [d.n for d in ds[-24:]], flush=True)
    check(zx, ds, True)
    check(zx, ds[:20], False)


def test_short_gate_buffer(zx):
    """A buffer shorter than the circuit: status ZX_ECAPACITY with the full
    count, the first max_gates gates written; the binding's second call with
    the counted size gives the whole circuit."""
    d = circuit_workload(7, 3)
    g = zx.Graph.from_diagram(d)
    zx.simplify([g], extract=False)
    ref = reference(d, True)
    import torch
    cap = 16
    gates = torch.zeros(cap, dtype=torch.int32, device="cuda")
    n_gates = torch.zeros(1, dtype=torch.int32, device="cuda")
    perm = torch.zeros(g.n_out, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb = zx.load().zx_extract_workspace_bytes(1)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    zx._check(zx.load().zx_extract(zx._graph_array([g]), 1, cap, zx._ptr(gates), zx._ptr(n_gates),
                                   zx._ptr(perm), zx._ptr(status), zx._ptr(ws), nb, zx._stream(None)))
    torch.cuda.synchronize()
    assert int(status[0]) == zx.ZX_ECAPACITY
    assert int(n_gates[0]) == len(ref[0]) > cap
    assert zx.decode_gates(gates.cpu().numpy().view(np.uint32)) == ref[0][:cap]
    st, full, p = zx.extract([g], max_gates=cap)[0]
    assert st == zx.ZX_OK and full == ref[0] and list(p) == ref[1]


def test_capacity(zx):
    from workloads import serve_diagram
    from workloads.generators import serve_params
    i = next(i for i in range(1000) if serve_params(5, i)[1] > 1024)
    g = zx.Graph.from_diagram(serve_diagram(5, i))
    with pytest.raises(zx.ZxError):
        zx.extract([g])
