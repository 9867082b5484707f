"""Pins of the oracle's parameterized Pauli spiders (Pauli boxes).

A spider's phase is k pi/4 + (p . f) pi for a parameter row p over binary
parameters f.  For every assignment f the rewritten diagram must equal the
original one exactly, once the recorded terms are evaluated at f:

    D(f) = omega^phase8 sqrt(2)^pow * prod_t h(k_alpha pi/4, k_beta pi/4; u_t.f, v_t.f) * D'(f)

(the product of phase-pair factors of the paper's parameterized evaluation
appendix, equations parities, phase_pair and scalar_product).  Both sides are
evaluated exactly in Z[omega] by the tensor evaluator, which knows nothing of
parameters: each f gives an ordinary diagram with phases k + 4 (p . f).
A dropped parameter update (a neighbour not XORed, B given only one of
p_u, p_v) or a wrong term constant fails these tests.
"""
import numpy as np
import pytest

import oracle
from oracle import phase as ph
from oracle.tensor import Amp, evaluate, zw_mul
from workloads.generators import pack_rows


def parity(row, f):
    x = 0
    for w, word in enumerate(row):
        for b in range(64):
            if (int(word) >> b) & 1 and f[64 * w + b]:
                x ^= 1
    return x


def instantiate(g, f):
    """Ordinary phases of every spider at parameter assignment f."""
    return np.array([(int(g.k[v]) + 4 * parity(g.params[v], f)) % 8 for v in range(g.n)], np.int64)


def amp_at(g, f, with_terms):
    a = evaluate(g.n, g.bits(), instantiate(g, f), g.alive_list(), g.inputs, g.outputs, g.bnd_is_h,
                 g.scalar.pow_sqrt2, g.scalar.phase8)
    if not with_terms:
        return a
    tk, tu, tv = g.terms()
    z = (1, 0, 0, 0)
    for t in range(len(tk)):
        z = ph.zw_mul(z, ph.exact_h(int(tk[t, 0]), int(tk[t, 1]), parity(tu[t], f), parity(tv[t], f)))
    return Amp(zw_mul(a.M, np.array(z, dtype=object)), a.pow, a.phase)


def random_param_graph(rng, n, q, dens, P, clifford=0.8):
    bits = np.triu((rng.random((n, n)) < dens).astype(np.uint8), 1)
    bits = bits + bits.T
    # mostly Clifford phases so that many rewrites apply
    k = np.where(rng.random(n) < clifford, 2 * rng.integers(0, 4, n), rng.integers(0, 8, n)).astype(np.int8)
    spiders = rng.permutation(n)
    ins, outs = spiders[:q].astype(np.int32), spiders[q:2 * q].astype(np.int32)
    pw = (P + 63) // 64
    prm = np.zeros((n, pw), np.uint64)
    for v in range(n):
        if rng.random() < 0.6:
            for b in range(P):
                if rng.random() < 0.5:
                    prm[v, b // 64] |= np.uint64(1) << np.uint64(b % 64)
    return oracle.Graph(n, pack_rows(bits), k, ins, outs, None, params=prm)


def all_f(P):
    for m in range(1 << P):
        yield [(m >> b) & 1 for b in range(P)] + [0] * (64 - P)


@pytest.mark.parametrize("seed", range(40))
def test_single_rules_with_parameters(seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(3, 10))
    P = int(rng.integers(1, 4))
    g = random_param_graph(rng, n, 0, [0.3, 0.5, 0.8][seed % 3], P)
    h = g.copy()
    if seed % 2 == 0:
        u = int(rng.integers(0, n))
        h.k[u] = g.k[u] = 2 if seed % 4 == 0 else 6
        assert h.local_comp(u) == oracle.OK
    else:
        u, v = (int(x) for x in rng.choice(n, 2, replace=False))
        bits = g.bits()
        if not bits[u, v]:
            for gg in (g, h):
                gg.adj[u, v // 64] |= np.uint64(1) << np.uint64(v % 64)
                gg.adj[v, u // 64] |= np.uint64(1) << np.uint64(u % 64)
        h.k[u] = g.k[u] = 4 * int(rng.integers(0, 2))
        h.k[v] = g.k[v] = 4 * int(rng.integers(0, 2))
        assert h.pivot(u, v) == oracle.OK
    for f in all_f(P):
        assert amp_at(g, f, False).equals(amp_at(h, f, True)), f[:P]


@pytest.mark.parametrize("seed", range(30))
def test_simplify_with_parameters(seed):
    rng = np.random.default_rng(8000 + seed)
    n = int(rng.integers(4, 12))
    q = int(rng.integers(0, 3))
    P = int(rng.integers(1, 5))
    g = random_param_graph(rng, n, q, [0.25, 0.4, 0.6][seed % 3], P)
    h = g.copy()
    assert h.simplify() == oracle.OK
    for f in all_f(P):
        assert amp_at(g, f, False).equals(amp_at(h, f, True)), f[:P]


@pytest.mark.parametrize("seed", range(10))
def test_parameters_do_not_change_the_schedule(seed):
    """Rewrite choices depend on the constant phases only: with the
    parameters at f = 0 the run equals the unparameterized one, trace and
    graph alike, and the terms evaluate to the scalar it tracks."""
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(6, 40))
    g = random_param_graph(rng, n, 2, 0.3, 70)
    plain = oracle.Graph(g.n, g.adj, g.k, g.inputs, g.outputs, g.bnd_is_h)
    h = g.copy()
    assert h.simplify() == oracle.OK and plain.simplify() == oracle.OK
    assert np.array_equal(h.trace, plain.trace) and np.array_equal(h.adj, plain.adj)
    assert np.array_equal(h.k, plain.k)
    tk, tu, tv = h.terms()
    z = (1, 0, 0, 0)
    for t in range(len(tk)):
        z = ph.zw_mul(z, ph.exact_h(int(tk[t, 0]), int(tk[t, 1]), 0, 0))
    zc = ph.zw_complex(z) * ph.omega_pow(h.scalar.phase8) * 2 ** (h.scalar.pow_sqrt2 / 2)
    zp = ph.omega_pow(plain.scalar.phase8) * 2 ** (plain.scalar.pow_sqrt2 / 2)
    assert abs(zc - zp) <= 1e-9 * abs(zp)
    # every spider still present keeps its parameter row; removed ones are cleared
    for v in range(n):
        if not h.is_alive(v):
            assert not h.params[v].any()


@pytest.mark.parametrize("seed", range(12))
def test_fbasis_reconstructs_dependencies(seed):
    """T has full row rank r = rank of the dependency vectors, and every
    vector is its coefficient row times T (the basis of the sampling step,
    equation detector_sampling and the sentence after it)."""
    from oracle.params import dependency_vectors, fbasis
    from workloads.generators import unpack_rows
    rng = np.random.default_rng(9500 + seed)
    n = int(rng.integers(8, 60))
    P = [3, 40, 64, 130][seed % 4]
    g = random_param_graph(rng, n, 2, 0.3, P)
    assert g.simplify() == oracle.OK
    D = dependency_vectors(g)
    T, coeff, piv, r = fbasis(D, P)
    Db, Tb = unpack_rows(D, P).astype(np.int64), unpack_rows(T, P).astype(np.int64)
    Cb = unpack_rows(coeff, max(r, 1))[:, :r].astype(np.int64)
    assert np.array_equal((Cb @ Tb) % 2, Db)
    # rank by brute-force elimination on the integer matrix
    M = Db.copy() % 2
    rk = 0
    for c in range(P):
        rows = [i for i in range(rk, M.shape[0]) if M[i, c]]
        if not rows:
            continue
        M[[rk, rows[0]]] = M[[rows[0], rk]]
        for i in range(M.shape[0]):
            if i != rk and M[i, c]:
                M[i] ^= M[rk]
        rk += 1
    assert r == rk
