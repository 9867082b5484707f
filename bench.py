"""Benchmark of the bit-packed GF(2) ZX hot path on one MI355X.

Headline (the JSON line's value): GF(2) reduced row echelon form of a
4096 x 16384 Bernoulli(1/2) bit matrix (seed 21), in GB/s of algorithmic
traffic: one read and one write of the trailing matrix per 64-column strip
that holds pivots, sum_s 2 * 8 * m * (W - s) bytes (W = 256 words per row).
A step is one elimination with the input resident in HBM.

Extra legs reported on the same line (timed separately, outside the
headline's timed region):
  pauli    symplectic commutation table of 65536 Pauli strings on 1024 qubits
  batched  4096 diagrams (q in 4..64, N = q * 4..16, p in [0.05, 0.3]):
           one persistent launch replayed from a HIP graph vs one launch per
           diagram (same kernel, host-synchronised); bit-exact vs the oracle
  learned  training-set generation (rollouts), training and evaluation of
           the learned proposal vs the greedy schedule on 1024 diagrams
  serve    Poisson request stream into the continuous-batching server:
           p50 / p99 latency (arrival to result on the host), throughput
  cpu_baseline  the plain C oracle on the same matrix, on this host's cores
                (per leg: the oracle on that leg's workload)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per rref_kernel launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# (KiB, already scaled by the copy-kernel calibration), valid only for the
# gf2.hip source they were measured on (sha256 prefix); see profiles/.
RREF_TRAFFIC = {
    "33a1b390f0dd9346": {"fetch_kib": 25724.2, "write_kib": 11388.3},
    # the same kernels with the allocation-free entry point beside them
    "de70e2edf8bc1717": {"fetch_kib": 25725.0, "write_kib": 11388.3},
    # the strip reduction at raised wave priority
    "1692da521e87034f": {"fetch_kib": 25722.2, "write_kib": 11388.3},
}
METRIC = "GF(2) elim GB/s (% HBM peak); diagrams simplified/sec batched vs plain, bit-exact"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def gf2_source_hash() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_2604_01059_amd", "csrc", "gf2.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def rref_traffic_bytes():
    t = RREF_TRAFFIC.get(gf2_source_hash())
    if t is None:
        return None
    return int(1024 * (t["fetch_kib"] + t["write_kib"]))


def strip_timeline(zx, ws, m):
    """Median per-strip phases from the kernel's timestamps (us)."""
    P = zx.gf2_profile(ws, m).astype(np.int64)
    used = np.nonzero(P[:, 0])[0]
    if len(used) < 3:
        return None
    S = used[-1] + 1
    us = lambda x: float(np.median(x)) * 0.01
    s = np.arange(1, S - 1)
    return {"strips": int(S),
            "factor_us": us(P[s, 6] - P[s, 1]), "publish_us": us(P[s, 2] - P[s, 6]),
            "owner_apply_us": us(P[s, 3] - P[s, 2]),
            "handoff_us": us((P[s, 4] - P[s, 2])[P[s, 4] > 0]) if (P[s, 4] > 0).any() else None,
            "next_apply_us": us((P[s, 5] - P[s, 4])[P[s, 4] > 0]) if (P[s, 4] > 0).any() else None,
            "strip_period_us": us(np.diff(P[:S, 0])),
            "span_us": float(P[S - 1, 3] - P[0, 0]) * 0.01}


def rref_algorithmic_bytes(m: int, nw: int, last_strip: int) -> int:
    """sum over strips s = 0..last_strip of one read + one write of the
    trailing matrix (words s..nw-1 of all m rows)."""
    return sum(2 * 8 * m * (nw - s) for s in range(last_strip + 1))


def bench_rref(zx, args):
    import torch
    from workloads import bernoulli_matrix
    m, n = 4096, 16384
    nw = n // 64
    A = bernoulli_matrix(21, m, n)
    dA = zx.to_device_words(A)
    R = torch.empty_like(dA)
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    piv = torch.zeros(m, dtype=torch.int32, device="cuda")
    ws = torch.empty(zx.gf2_workspace_bytes(m, n), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        zx.gf2_eliminate(dA, R=R, n_cols=n, rank=rank, pivots=piv, ws=ws)
    torch.cuda.synchronize()
    assert zx.gf2_status(ws) == 0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        zx.gf2_eliminate(dA, R=R, n_cols=n, rank=rank, pivots=piv, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    assert zx.gf2_status(ws) == 0
    r = int(rank.item())
    pv = piv.cpu().numpy()
    last_strip = int(pv[r - 1]) // 64 if r > 0 else 0
    strips32 = int(pv[r - 1]) // 32 + 1 if r > 0 else 0  # the kernel's 32-column strips up to the last pivot
    nbytes = rref_algorithmic_bytes(m, nw, last_strip)
    Rh = zx.to_host_words(R)
    timeline = strip_timeline(zx, ws, m) if args.rref_strips else None
    return dict(A=A, R=Rh, rank=r, piv=pv, ms=ms, wall_ms=1e3 * wall / args.steps, bytes=nbytes,
                last_strip=last_strip, strips32=strips32, m=m, n=n, timeline=timeline)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the all-core baselines use: this process's CPU share (at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_rref(res, budget_s):
    """The oracle on the whole matrix: single-threaded, median of 3 runs; the
    same loops with row additions over all host threads, median of 3."""
    import oracle
    A = res["A"]
    one = []
    Ro = pivo = ranko = None
    for _ in range(3):
        t0 = time.perf_counter()
        Ro, pivo, ranko, ops = oracle.gf2_rref(A, res["n"])
        one.append(time.perf_counter() - t0)
    exact = bool(np.array_equal(Ro, res["R"]) and ranko == res["rank"] and np.array_equal(pivo, res["piv"]))
    th = host_threads()
    os.environ["OMP_NUM_THREADS"] = str(th)
    allc = []
    for _ in range(3):
        t0 = time.perf_counter()
        R2, p2, r2 = oracle.gf2_rref_threads(A, res["n"])
        allc.append(time.perf_counter() - t0)
    exact = exact and bool(np.array_equal(R2, res["R"]))
    s1, sa = float(np.median(one)), float(np.median(allc))
    return dict(value=round(res["bytes"] / s1 / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                sample="whole 4096x16384 matrix, median of 3 runs (%.2f s each), plain single-threaded C "
                       "Gauss-Jordan" % s1,
                seconds_per_run=round(s1, 3),
                all_cores={"value": round(res["bytes"] / sa / 1e9, 4), "unit": "GB/s", "cores": th,
                           "seconds_per_run": round(sa, 3),
                           "sample": "same matrix, row additions over %d OpenMP threads, median of 3" % th},
                cpu_model=cpu_model()), exact


def _time_launches(fn, steps):
    """Average ms of fn() over steps launches, HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


_PAULI = {}


def _oracle_pauli_block(args):
    """sha256 of rows i0..i1-1 of the oracle's table (worker process)."""
    import hashlib
    import oracle
    from workloads import pauli_strings
    i0, i1 = args
    if "XZ" not in _PAULI:
        _PAULI["XZ"] = pauli_strings(22, 65536, 1024)
    X, Z = _PAULI["XZ"]
    blk = oracle.pauli_commute(X, Z, rows=(i0, i1))
    return hashlib.sha256(np.ascontiguousarray(blk).tobytes()).hexdigest()


def bench_pauli(zx, steps, pool):
    import hashlib
    import torch
    from workloads import pauli_strings
    n, q = 65536, 1024
    X, Z = pauli_strings(22, n, q)
    dX, dZ = zx.to_device_words(X), zx.to_device_words(Z)
    C = torch.empty((n, n // 64), dtype=torch.int64, device="cuda")
    pairs = float(n) * n
    out = {"workload": "65536 Pauli strings x 1024 qubits (seed 22), 65536^2-bit table"}
    for name, flag in (("valu", zx.ZX_PAULI_FORCE_VALU), ("mfma", zx.ZX_PAULI_FORCE_MFMA)):
        ms = _time_launches(lambda: zx.pauli_commute(dX, dZ, q, C_out=C, flags=flag), steps)
        out[name] = {"ms": round(ms, 4), "pairs_per_s": pairs / (ms * 1e-3),
                     "out_GBps": round(n * n / 8 / (ms * 1e-3) / 1e9, 2)}
    # VALU work: 64x64 tiles on and above the diagonal, AND + XOR per qubit per term
    tiles = (n // 64) * (n // 64 + 1) / 2
    out["valu"]["bitop_Tops"] = round(tiles * 4096 * 2 * q * 2 / (out["valu"]["ms"] * 1e-3) / 1e12, 2)
    # matrix cores: 256x256 tiles on and above the diagonal, K = 2q, 2 flops per product
    t256 = (n // 256) * (n // 256 + 1) / 2
    mflops = t256 * 256 * 256 * 2 * q * 2
    out["mfma"]["TFLOPs"] = round(mflops / (out["mfma"]["ms"] * 1e-3) / 1e12, 1)
    out["mfma"]["frac_of_fp4_peak"] = round(mflops / (out["mfma"]["ms"] * 1e-3) / 10.1e15, 4)
    best = min(("valu", "mfma"), key=lambda k: out[k]["ms"])
    out["auto_picks"] = "mfma"
    out["faster"] = best
    out["ms"] = out["mfma"]["ms"]
    # the table of the variant AUTO runs, compared in full with the oracle
    zx.pauli_commute(dX, dZ, q, C_out=C)
    torch.cuda.synchronize()
    if pool is not None:
        blocks = [(i, min(n, i + 1024)) for i in range(0, n, 1024)]
        t0 = time.perf_counter()
        digests = list(pool.map(_oracle_pauli_block, blocks, chunksize=1))
        cpu_s = time.perf_counter() - t0
        Ch = C.cpu().numpy().view(np.uint64)
        same = sum(hashlib.sha256(np.ascontiguousarray(Ch[i0:i1]).tobytes()).hexdigest() == d
                   for (i0, i1), d in zip(blocks, digests))
        out["full_exact"] = "%d/%d row blocks" % (same, len(blocks))
        out["cpu_baseline"] = {"value": round(pairs / cpu_s, 1), "unit": "pairs/s", "cores": pool._processes,
                               "kind": "oracle", "sample": "the whole 65536^2 table, 64 blocks of 1024 rows "
                               "over %d worker processes (%.1f s)" % (pool._processes, cpu_s)}
    return out


def bench_parity(zx, steps):
    """Batched phase-pair evaluation: parities a = U F^T, b = V F^T on the
    matrix cores, then the phase-pair product per setting."""
    import torch
    import oracle
    from oracle import phase as oph
    from workloads import parity_problem
    m, L, P = 4096, 65536, 1024
    prob = parity_problem(61, m, L, P)
    dU, dV, dF = (zx.to_device_words(x) for x in (prob.U, prob.V, prob.F))
    ka = torch.from_numpy(prob.k_alpha).cuda()
    kb = torch.from_numpy(prob.k_beta).cuda()
    A = torch.empty((m, L // 64), dtype=torch.int64, device="cuda")
    B = torch.empty_like(A)
    mant = torch.empty((L, 2), dtype=torch.float32, device="cuda")
    expo = torch.empty(L, dtype=torch.int32, device="cuda")
    ms_mm = _time_launches(lambda: zx.gf2_matmul(dU, dF, P, C_out=A), steps)
    zx.gf2_matmul(dV, dF, P, C_out=B)
    ms_pp = _time_launches(lambda: zx.phase_pair_product(A, B, ka, kb, L, 3, -5, mant=mant, expo=expo), steps)
    torch.cuda.synchronize()
    flops = 2.0 * m * L * P
    Ah = zx.to_host_words(A)
    rows = (0, 1, 2047, 4095)
    rows_ok = all(np.array_equal(Ah[r:r + 1], oracle.gf2_matmul(prob.U[r:r + 1], prob.F, P)) for r in rows)
    # product on 64 settings, against the fp64 oracle (its tolerance: tests)
    S = 64
    Bh = zx.to_host_words(B)
    t0 = time.perf_counter()
    Ao = oracle.gf2_matmul(prob.U, prob.F[:S], P)
    Bo = oracle.gf2_matmul(prob.V, prob.F[:S], P)
    mo, eo = oph.phase_pair_product(Ao, Bo, prob.k_alpha, prob.k_beta, S, 3, -5)
    cpu_s = time.perf_counter() - t0
    mg, eg = mant.cpu().numpy()[:S], expo.cpu().numpy()[:S]
    zg = mg[:, 0].astype(np.float64) + 1j * mg[:, 1]
    errs = [abs(zg[l] * 2.0 ** float(int(eg[l]) - int(eo[l])) - mo[l]) / abs(mo[l]) for l in range(S) if mo[l] != 0]
    rel = max(errs) if errs else 0.0
    zeros_agree = all((mo[l] == 0) == (zg[l] == 0) for l in range(S))
    total = 2 * ms_mm + ms_pp
    return {"workload": "4096 terms x 65536 settings x 1024 parameters (seed 61): a = U F^T, b = V F^T, "
                        "then prod_k h(alpha_k, beta_k; a_k, b_k)",
            "ms_matmul": round(ms_mm, 4), "ms_product": round(ms_pp, 4), "ms_total": round(total, 4),
            "settings_per_s": round(L / (total * 1e-3), 1),
            "matmul_TFLOPs": round(flops / (ms_mm * 1e-3) / 1e12, 1),
            "matmul_frac_of_fp4_peak": round(flops / (ms_mm * 1e-3) / 10.1e15, 4),
            "parity_rows_exact": rows_ok, "a_b_bits_equal_oracle_on_64_settings":
                bool(np.array_equal(Ah[:, :1], Ao[:, :1]) and np.array_equal(Bh[:, :1], Bo[:, :1])),
            "product_max_rel_err_64_settings": float(rel), "product_zeros_agree": zeros_agree,
            "product_rel_tolerance": (21 * m + 4) * 2.0 ** -24,
            "cpu_baseline": {"value": round(S / cpu_s, 2), "unit": "settings/s", "cores": 1, "kind": "oracle",
                             "sample": "parities of all 4096 terms (two products) and the fp64 product for "
                                       "64 settings, %.1f s" % cpu_s}}


def bench_sample(zx, steps):
    """Detector sampling f = T e, surface-code-shaped model d = 7, 7 rounds."""
    import torch
    import oracle
    from workloads import surface_dem
    M = surface_dem(7, 7, 7, 1e-3)
    S = zx.DetectorSampler(M.col_ptr, M.col_idx, M.prob, M.n_f)
    shots = 1 << 24
    fw = (M.n_f + 63) // 64
    out = torch.empty((shots, fw), dtype=torch.int64, device="cuda")
    ms = _time_launches(lambda: S.sample(2024, 0, shots, out=out), steps)
    assert S.status() == 0
    n_chk = 100000
    got = zx.to_host_words(out[:n_chk])
    ref = oracle.detector_sample(M.col_ptr, M.col_idx, M.prob, M.n_f, 2024, 0, n_chk)
    tail0 = shots - 20000
    got_t = zx.to_host_words(out[tail0:])
    t0 = time.perf_counter()
    ref_t = oracle.detector_sample(M.col_ptr, M.col_idx, M.prob, M.n_f, 2024, tail0, 20000)
    cpu_s = time.perf_counter() - t0
    written = shots * fw * 8
    gbs = written / (ms * 1e-3) / 1e9
    return {"workload": "detector error model shaped like a d=7 surface-code memory experiment, 7 rounds "
                        "(%d detectors + 1 observable, %d mechanisms, p ~ 1e-3 U[0.5,1.5]); %d shots per "
                        "launch" % (M.n_det, M.n_err, shots),
            "ms": round(ms, 4), "shots_per_s": round(shots / (ms * 1e-3), 1),
            "out_GBps": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "exact_first_100k": bool(np.array_equal(got, ref)),
            "exact_last_20k": bool(np.array_equal(got_t, ref_t)),
            "cpu_baseline": {"value": round(20000 / cpu_s, 1), "unit": "shots/s", "cores": 1, "kind": "oracle",
                             "sample": "20000 shots (the last of the launch), %.2f s" % cpu_s}}


def _oracle_param_diag(args):
    import oracle
    from workloads import batch_diagram, param_rows
    i, P = args
    d = batch_diagram(3, i)
    g = oracle.Graph(d.n, d.adj, d.phase, d.inputs, d.outputs, d.bnd_is_h, params=param_rows(3, i, d.n, P))
    g.simplify()
    tk, tu, tv = g.terms()
    import hashlib
    hsh = hashlib.sha256()
    for a in (g.adj, g.k, g.params, tk, tu, tv):
        hsh.update(np.ascontiguousarray(a).tobytes())
    hsh.update(np.array([g.scalar.pow_sqrt2, g.scalar.phase8 % 8], np.int64).tobytes())
    return hsh.hexdigest()


def bench_params(zx, pool):
    """Batched simplification of the 4096 batched-workload diagrams with
    parameterized Pauli spiders (1024 parameters), against the same batch
    without parameters; bit-exact against the oracle."""
    import hashlib
    import torch
    from workloads import batch_diagram, param_rows
    P = 1024
    ds = list(pool.map(_gen_diag, range(4096), chunksize=32)) if pool is not None else \
        [_gen_diag(i) for i in range(4096)]
    prs = [param_rows(3, i, d.n, P) for i, d in enumerate(ds)]
    gs = [zx.Graph.create(d.adj, d.phase, d.inputs, d.outputs, d.bnd_is_h, n_params=P, params=pr)
          for d, pr in zip(ds, prs)]
    plain = [zx.Graph.from_diagram(d) for d in ds]
    res = {}
    for name, graphs in (("with_params", gs), ("without_params", plain)):
        b = zx.Batch(graphs)
        ms = _time_launches(lambda: b.run(extract=True), 3)
        assert b.status() == 0
        res[name + "_ms"] = round(ms, 3)
    out = {"workload": "4096 diagrams of the batched workload (seed 3), ~30% of spiders carrying 2 of "
                       "1024 parameters", **res,
           "diagrams_per_s": round(4096 / (res["with_params_ms"] * 1e-3), 1)}
    if pool is not None:
        t0 = time.perf_counter()
        digests = list(pool.map(_oracle_param_diag, [(i, P) for i in range(4096)], chunksize=16))
        cpu_s = time.perf_counter() - t0
        same = 0
        for g, dg in zip(gs, digests):
            adj, ph, al, info = g.read()
            rows, kab, u, v = g.params()
            hsh = hashlib.sha256()
            for a in (adj, ph, rows, kab, u, v):
                hsh.update(np.ascontiguousarray(a).tobytes())
            hsh.update(np.array([info.pow_sqrt2, info.phase8], np.int64).tobytes())
            same += hsh.hexdigest() == dg
        out["bit_exact_vs_oracle"] = "%d/4096" % same
        out["cpu_baseline"] = {"value": round(4096 / cpu_s, 1), "unit": "diagrams/s", "cores": pool._processes,
                               "kind": "oracle", "sample": "all 4096 diagrams, one per worker process"}
    return out


def _oracle_c1(seed):
    import oracle
    from workloads import single_diagram
    d = single_diagram(seed)
    t0 = time.perf_counter()
    g = oracle.Graph.from_diagram(d)
    g.simplify()
    M, piv, rank, ops = g.frontier()
    dt = time.perf_counter() - t0
    return dt, (g.adj.tobytes(), g.k.tobytes(), int(g.scalar.pow_sqrt2), int(g.scalar.phase8 % 8), M.tobytes(),
                int(rank), int(ops))


def bench_c1(zx):
    """One diagram (8 qubits, 64 spiders, p = 0.1), seeds 1..1000: latency of
    one launch per diagram, kernel only (HIP events around the launch, queued
    behind a spin so that host launch work is not counted) and end to end
    (host clock around launch and result read), against the oracle on one
    core."""
    import torch
    from workloads import single_diagram
    ds = [single_diagram(s) for s in range(1, 1001)]
    gs = [zx.Graph.from_diagram(d) for d in ds]
    bs = [zx.Batch([g]) for g in gs]
    for b in bs[:20]:
        b.run(extract=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    kern, e2e = [], []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # Kernel time: a spin on the stream holds it while the host queues the
    # launch, so that the events bracket device time alone (with an idle
    # stream, the first event would also count the host's launch work).
    cycles = 20000
    for _ in range(12):
        e0.record(stream)
        torch.cuda._sleep(cycles)
        e1.record(stream)
        torch.cuda.synchronize()
        if e0.elapsed_time(e1) >= 0.3:
            break
        cycles *= 2
    for g, b in zip(gs, bs):
        torch.cuda._sleep(cycles)
        e0.record(stream)
        b.run(extract=True)
        e1.record(stream)
        torch.cuda.synchronize()
        kern.append(e0.elapsed_time(e1) * 1e-3)
        # end to end: host clock around the launch and the result read
        t0 = time.perf_counter()
        b.run(extract=True)
        info = g.info()  # synchronises
        e2e.append(time.perf_counter() - t0)
        assert info.status == 0
    exact = 0
    cpu = []
    for s, g in zip(range(1, 1001), gs):
        dt, ref = _oracle_c1(s)
        cpu.append(dt)
        adj, ph, al, info = g.read()
        M, piv = g.frontier()
        got = (adj.tobytes(), ph.tobytes(), int(info.pow_sqrt2), int(info.phase8), M.tobytes(), int(info.rank),
               int(info.rowops))
        exact += got == ref
    us = lambda a, q: round(float(np.percentile(np.array(a), q)) * 1e6, 2)
    return {"workload": "one diagram per launch: 8 qubits, 64 spiders, ER p=0.1, seeds 1..1000; simplify + "
                        "8x64 frontier RREF",
            "kernel_us_p50": us(kern, 50), "kernel_us_p99": us(kern, 99),
            "end_to_end_us_p50": us(e2e, 50), "end_to_end_us_p99": us(e2e, 99),
            "bit_exact_vs_oracle": "%d/1000" % exact,
            "cpu_baseline": {"value": us(cpu, 50), "unit": "us per diagram (p50)", "p99": us(cpu, 99), "cores": 1,
                             "kind": "oracle", "sample": "the same 1000 diagrams, one at a time"}}


def _circ_diag(i):
    from workloads.circuits import circuit_workload
    return circuit_workload(12, i, q_lo=20, q_hi=20)


def _oracle_extract(d):
    """The oracle's flow check and circuit of one simplified circuit diagram
    (digest of the gate list and permutation)."""
    import hashlib
    import oracle
    from oracle import extract as ox
    g = oracle.Graph.from_diagram(d)
    g.simplify()
    ex, layers = ox.gflow_layers(g)
    gates, perm, _ = ox.extract_circuit(g)
    return bool(ex), hashlib.sha256(repr((gates, [int(p) for p in perm])).encode()).hexdigest(), len(gates)


def bench_extract(zx, pool, steps=5):
    """Flow check and circuit extraction of 4096 simplified circuit diagrams
    (20 qubits, 1-21 exponentiated Pauli strings of weight 2-4), each kernel
    timed over the whole batch with HIP events; every circuit compared with
    the oracle's."""
    import hashlib
    import torch
    t0 = time.perf_counter()
    ds = list(pool.map(_circ_diag, range(4096), chunksize=32))
    log("extract: generated 4096 circuit diagrams in %.1f s (mean N %.0f, max N %d)" %
        (time.perf_counter() - t0, np.mean([d.n for d in ds]), max(d.n for d in ds)))
    gs, big = make_graphs(zx, ds)
    b = zx.Batch(gs)
    simp_ms = _time_launches(lambda: b.run(extract=False), 1)
    b.run(extract=False)
    torch.cuda.synchronize()
    assert b.status() == 0
    lib = zx.load()
    n = len(gs)
    arr = zx._graph_array(gs)
    layers = torch.empty(sum(g.n for g in gs), dtype=torch.int32, device="cuda")
    exists = torch.empty(n, dtype=torch.int32, device="cuda")
    fws_b = lib.zx_gflow_workspace_bytes(n)
    fws = torch.empty(fws_b, dtype=torch.uint8, device="cuda")
    cap = max((g.n + 2 * g.n_in) * (g.n_out + 4) for g in gs)
    gates = torch.empty(n * cap, dtype=torch.int32, device="cuda")
    n_gates = torch.empty(n, dtype=torch.int32, device="cuda")
    perm = torch.empty(sum(g.n_out for g in gs), dtype=torch.int32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    ews_b = lib.zx_extract_workspace_bytes(n)
    ews = torch.empty(ews_b, dtype=torch.uint8, device="cuda")
    st = zx._stream(None)
    flow_ms = _time_launches(lambda: zx._check(lib.zx_gflow(arr, n, zx._ptr(layers), zx._ptr(exists),
                                                            zx._ptr(fws), fws_b, st)), steps)
    ext_ms = _time_launches(lambda: zx._check(lib.zx_extract(arr, n, cap, zx._ptr(gates), zx._ptr(n_gates),
                                                             zx._ptr(perm), zx._ptr(status), zx._ptr(ews),
                                                             ews_b, st)), steps)
    ex_h, st_h, ng_h = exists.cpu().numpy(), status.cpu().numpy(), n_gates.cpu().numpy()
    G = gates.cpu().numpy().view(np.uint32).reshape(n, cap)
    P = perm.cpu().numpy()
    out = {"workload": "4096 circuit diagrams: 20 qubits, U{1..21} exponentiated Pauli strings of weight "
                       "U{2..4} (seed 12), simplified; flow layers, then the circuit",
           "mean_spiders_simplified": round(float(np.mean([g.info().n_alive for g in gs])), 1),
           "simplify_ms": round(simp_ms, 3), "gflow_ms": round(flow_ms, 3), "extract_ms": round(ext_ms, 3),
           "circuits_per_s": round(n / ((flow_ms + ext_ms) * 1e-3), 1),
           "gates_total": int(ng_h.sum()), "all_have_flow": bool((ex_h == 1).all()),
           "all_extracted": bool((st_h == 0).all())}
    t0 = time.perf_counter()
    refs = list(pool.map(_oracle_extract, ds, chunksize=16))
    cpu_s = time.perf_counter() - t0
    same, off = 0, 0
    for i, g in enumerate(gs):
        ref_ex, ref_dg, _ = refs[i]
        pm = [int(x) for x in P[off:off + g.n_out]]
        off += g.n_out
        dg = hashlib.sha256(repr((zx.decode_gates(G[i, :int(ng_h[i])]), pm)).encode()).hexdigest()
        same += int(ex_h[i] == int(ref_ex) and st_h[i] == 0 and dg == ref_dg)
    out["bit_exact_vs_oracle"] = "%d/%d" % (same, n)
    out["cpu_baseline"] = {"value": round(n / cpu_s, 1), "unit": "circuits/s", "cores": pool._processes,
                           "kind": "oracle", "sample": "all 4096 diagrams (simplify, flow layers, extraction), "
                                                       "one per worker process"}
    return out


def bench_large(zx, reps=3):
    """Serving-stream diagrams of 2000 to 8000 spiders, one zx_simplify call each
    (large diagrams run on a team of workgroups), checked against the oracle's
    stored results (tests/golden/large_diagrams.json)."""
    import hashlib
    import torch
    from workloads import serve_diagram
    path = os.path.join(ROOT, "tests", "golden", "large_diagrams.json")
    es = sorted(json.load(open(path))["entries"], key=lambda e: e["n"])
    out = {"workload": "serving-stream diagrams (seed 5) of %d to %d spiders, one zx_simplify call each, "
                       "with the output frontier" % (es[0]["n"], es[-1]["n"]), "diagrams": []}
    exact = 0
    for e in es:
        d = serve_diagram(e["seed"], e["item"])
        g = zx.Graph.from_diagram(d)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            zx.simplify([g], extract=True)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        adj, ph, al, info = g.read()
        ok = (info.status == 0 and info.n_edges == e["n_edges"] and info.rounds == e["rounds"] and
              info.rowops == e["rowops"] and
              hashlib.sha256(np.ascontiguousarray(adj.astype("<u8")).tobytes()).hexdigest() == e["sha_adj"])
        exact += ok
        out["diagrams"].append({"n": d.n, "rounds": int(info.rounds), "ms": round(min(ts), 2)})
        log("large: n %d, %.2f ms" % (d.n, min(ts)))
    out["bit_exact_vs_oracle"] = "%d/%d" % (exact, len(es))
    return out


def _gen_diag(i):
    from workloads import batch_diagram
    return batch_diagram(3, i)


def _oracle_diag(d):
    import oracle
    g = oracle.Graph.from_diagram(d)
    g.simplify()
    M, piv, rank, ops = g.frontier()
    return (g.adj, g.k, g.alive, g.scalar.pow_sqrt2, g.scalar.phase8 % 8, g.trace, M, rank, ops)


def make_graphs(zx, ds):
    """All arenas carved from one device allocation."""
    import torch
    sizes = [zx.Graph.bytes_for(d.n, len(d.inputs), len(d.outputs)) for d in ds]
    offs = np.concatenate([[0], np.cumsum([(s + 255) // 256 * 256 for s in sizes])])
    big = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    gs = [zx.Graph.from_diagram(d, arena=big[int(offs[i]):int(offs[i]) + sizes[i]]) for i, d in enumerate(ds)]
    return gs, big


def bench_batched(zx, args, pool):
    import torch
    t0 = time.perf_counter()
    ds = list(pool.map(_gen_diag, range(4096), chunksize=32))
    log("batched: generated 4096 diagrams in %.1f s (mean N %.0f, max N %d)" %
        (time.perf_counter() - t0, np.mean([d.n for d in ds]), max(d.n for d in ds)))
    gs, big = make_graphs(zx, ds)
    b = zx.Batch(gs)
    best, best_ms = b.autotune(extract=True, reps=2)
    variant = zx.simplify_variants()[best]
    log("batched: autotuned variant %s (%.3f ms)" % (variant, best_ms))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.run(extract=True, stream=stream)
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        graph.capture_begin()
        b.run(extract=True, stream=stream)
        graph.capture_end()
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / reps
    assert b.status() == 0
    res_b = [(g.read(), g.trace(), g.frontier()) for g in gs]
    # plain GPU path: same kernel, one launch per diagram, host-synchronised
    singles = [zx.Batch([g]) for g in gs]
    for sb in singles[:16]:
        sb.run(extract=True, tune_id=best)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sb in singles:
        sb.run(extract=True, tune_id=best)
        torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    same = 0
    for g, rb in zip(gs, res_b):
        a = g.read()
        if (np.array_equal(a[0], rb[0][0]) and np.array_equal(a[1], rb[0][1]) and
                np.array_equal(g.frontier()[0], rb[2][0])):
            same += 1
    cb = cpu_baseline_batched(pool, ds, res_b)
    return dict(
        workload="4096 diagrams: q~U{4..64}, N=q*U{4..16}, p~U[0.05,0.3], seed 3; simplify + frontier RREF",
        variant=variant, batched_ms=round(batched_s * 1e3, 3), plain_ms=round(plain_s * 1e3, 2),
        batched_diagrams_per_s=round(4096 / batched_s, 1), plain_diagrams_per_s=round(4096 / plain_s, 1),
        speedup=round(plain_s / batched_s, 2), bit_exact_vs_oracle=cb.pop("bit_exact"),
        batched_equals_plain="%d/4096" % same, cpu_baseline=cb)


def cpu_baseline_batched(pool, ds, res_b):
    """The oracle (plain C, one diagram per worker process) on the same 4096
    diagrams: its throughput, and whether every GPU result equals it."""
    t0 = time.perf_counter()
    outs = list(pool.map(_oracle_diag, ds, chunksize=16))
    oracle_s = time.perf_counter() - t0
    exact = 0
    for (st, tr, fr), o in zip(res_b, outs):
        adj, ph, al, info = st
        ok = (np.array_equal(adj, o[0]) and np.array_equal(ph, o[1]) and np.array_equal(al, o[2])
              and info.pow_sqrt2 == o[3] and info.phase8 == o[4] and np.array_equal(tr, o[5])
              and np.array_equal(fr[0], o[6]) and info.rank == o[7] and info.rowops == o[8])
        exact += ok
    return {"value": round(len(ds) / oracle_s, 1), "unit": "diagrams/s", "cores": pool._processes,
            "kind": "oracle", "sample": "all %d diagrams, one per worker process" % len(ds),
            "bit_exact": "%d/%d" % (exact, len(ds))}


def _oracle_eval(d):
    import oracle
    g = oracle.Graph.from_diagram(d)
    g.simplify()
    ops = g.frontier()[3] if len(g.outputs) else 0
    return g.n_edges() + ops


def _oracle_replay(args):
    """Replay one learned trace on the oracle and compare the final state with
    the GPU's (digests of adjacency, phases, alive mask; scalar; frontier)."""
    import hashlib
    import oracle
    from oracle import policy as opol
    from workloads import batch_diagram
    item, trace, dig, scal = args
    d = batch_diagram(42, item, q_lo=32, q_hi=128)
    try:
        fin = opol.replay(oracle.Graph.from_diagram(d), trace)
    except AssertionError:
        return False
    h = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
    rank, ops = -1, 0
    if len(fin.outputs):
        _, _, rank, ops = fin.frontier()
    got = (h(fin.adj), h(fin.k), h(fin.alive), int(fin.scalar.pow_sqrt2), int(fin.scalar.phase8 % 8), int(rank),
           int(ops))
    return got == tuple(dig) + tuple(scal)


def bench_learned(zx, args, pool):
    """Learned proposal: dataset from greedy runs (rollout labels), training
    with the network kernels, held-out ranking quality, evaluation on
    held-out diagrams vs greedy and with the greedy fallback, every learned
    trace replayed on the oracle."""
    import hashlib
    import torch
    from paper_2604_01059_amd import learned
    t0 = time.perf_counter()
    mlp = learned.new_network()
    ev0 = learned.evaluate(mlp, n=1024)  # the untrained network, for comparison
    feats, costs = learned.make_dataset(args.learned_states, per_state=16, log=log, label=args.learned_label)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    rollouts = int((costs >= 0).sum())
    # held-out states: greedy runs of other diagrams of the same generator
    vf, vc = learned.make_dataset(args.learned_val_states, per_state=16, first_item=1 << 20,
                                  label=args.learned_label)
    untrained = learned.state_metrics(mlp, vf, vc)
    t0 = time.perf_counter()
    curve, val_curve = learned.train(mlp, feats, costs, per_state=16, epochs=args.learned_epochs, log=log,
                                     val=(vf, vc))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    trained = learned.state_metrics(mlp, vf, vc)
    ev, ds, lg, fg = learned.evaluate(mlp, n=1024, keep_graphs=True)
    args._trained_mlp = mlp
    out = dict(workload="train: %d greedy-run states of the batched generator (seed %d) whose candidates differ "
                        "in rollout %s, 16 rollouts each; held-out: %d states of other diagrams; eval: 1024 "
                        "diagrams q~U{32..128}, N=q*U{4..16}, seed %d"
                        % (args.learned_states, learned.TRAIN_SEED, args.learned_label, args.learned_val_states,
                           learned.EVAL_SEED),
               label=args.learned_label,
               dataset_s=round(data_s, 2), rollouts=rollouts, train_s=round(train_s, 2), epochs=args.learned_epochs,
               loss_first=curve[0][1] if curve else None, loss_last=curve[-1][1] if curve else None,
               loss_curve=curve[:: max(1, len(curve) // 12)], heldout_loss_per_epoch=val_curve,
               heldout_untrained=untrained, heldout_trained=trained,
               untrained_network={k: ev0[k] for k in ("gate2q_learned", "gate2q_fallback", "fill_learned",
                                                      "fill_fallback", "learned_better", "learned_worse")},
               **ev)
    if pool is not None:
        h = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
        jobs = []
        for i, g in enumerate(lg):
            adj, ph, al, info = g.read()
            jobs.append((i, g.trace(), (h(adj), h(ph), h(al)),
                         (int(info.pow_sqrt2), int(info.phase8), int(info.rank), int(info.rowops))))
        t0 = time.perf_counter()
        ok = list(pool.map(_oracle_replay, jobs, chunksize=8))
        out["learned_replay_exact"] = "%d/%d" % (sum(ok), len(ok))
        out["replay_s"] = round(time.perf_counter() - t0, 1)
        t0 = time.perf_counter()
        costs_cpu = list(pool.map(_oracle_eval, ds, chunksize=8))
        out["cpu_baseline"] = {"value": round(1024 / (time.perf_counter() - t0), 1), "unit": "diagrams/s",
                               "cores": pool._processes, "kind": "oracle",
                               "sample": "the 1024 evaluation diagrams, greedy schedule",
                               "gate2q": int(sum(costs_cpu)),
                               "equals_gpu_greedy": int(sum(costs_cpu)) == ev["gate2q_greedy"]}
    return out


def _gen_serve(i):
    from workloads import serve_diagram
    return serve_diagram(5, i)


def serve_diagrams(args, pool):
    n_unique = args.serve_unique
    t0 = time.perf_counter()
    ds = list(pool.map(_gen_serve, range(n_unique), chunksize=8)) if pool is not None else \
        [_gen_serve(i) for i in range(n_unique)]
    log("serve: generated %d request diagrams in %.1f s (median N %d, max N %d)" %
        (n_unique, time.perf_counter() - t0, int(np.median([d.n for d in ds])), max(d.n for d in ds)))
    return ds


def bench_serve(zx, args, ds, mlp=None, seconds=None):
    """Serving: Poisson arrivals into a continuous-batching server; with mlp,
    the learned policy with the greedy fallback, else greedy."""
    from workloads import poisson_arrivals
    n_unique = len(ds)
    rate, warm = args.serve_rate, args.serve_warmup
    dur = args.serve_seconds if seconds is None else seconds
    count = int(rate * (warm + dur) * 1.05) + 16
    arr = poisson_arrivals(5, rate, count)
    arr = arr[arr < warm + dur]
    if mlp is None:
        sv = zx.Server(args.serve_pool_gib << 30, max_batch=2048, trusted=True)
    else:
        sv = zx.Server(args.serve_pool_gib << 30, max_batch=2048, trusted=True, policy=zx.ZX_POLICY_LEARNED, mlp=mlp,
                       fallback=True)
    start = time.perf_counter() + 0.05
    backlog = []
    lat, refused, nxt, done = [], 0, 0, 0
    dev, queue, sizes = [], [], []
    claim_dev, end_dev, done_host, arr_host = [], [], [], []
    host_submit_s = host_poll_s = 0.0
    learned_kept = 0
    max_backlog = 0
    last_log = 0.0
    deadline = warm + dur + args.serve_drain
    while done < len(arr):
        now = time.perf_counter() - start
        if now - last_log >= 5.0:
            log("serve: t=%.1f s, %d arrived, %d submitted, %d done, %d waiting on the host"
                % (now, nxt, nxt - len(backlog), done, len(backlog)))
            last_log = now
        if now > deadline:
            log("serve: not drained %.0f s after the last arrival; stopping" % args.serve_drain)
            break
        while nxt < len(arr) and arr[nxt] <= now:
            backlog.append(nxt)
            nxt += 1
        ts = time.perf_counter()
        while backlog:
            i = backlog[0]
            if sv.submit(ds[i % n_unique], tag=i) is None:
                refused += 1
                break
            backlog.pop(0)
        tp = time.perf_counter()
        host_submit_s += tp - ts
        max_backlog = max(max_backlog, len(backlog))
        got = sv.poll()
        host_poll_s += time.perf_counter() - tp
        for r in got:
            done += 1
            if arr[r.tag] >= warm:
                lat.append(r.t_done - (start + arr[r.tag]))
                dev.append(r.t_device)
                queue.append(r.t_launch - (start + arr[r.tag]))
                sizes.append(ds[r.tag % n_unique].n)
                learned_kept += r.policy == zx.ZX_POLICY_LEARNED
                claim_dev.append(r.t_claim_dev)
                end_dev.append(r.t_end_dev)
                done_host.append(r.t_done)
                arr_host.append(start + arr[r.tag])
    wall = time.perf_counter() - start
    st = sv.stats()
    sv.close()
    drained = done == len(arr)
    # device clock on the host clock: the smallest (seen - written) gap is
    # taken as a poll lag of zero; then submit -> claim is the true queue,
    # claim -> written the device time, written -> seen the host's lag
    if end_dev:
        ce, ee, dh, ah = map(np.array, (claim_dev, end_dev, done_host, arr_host))
        off = float(np.min(dh - ee))
        true_queue = (ce + off) - ah
        lag = dh - (ee + off)
    else:
        true_queue = lag = np.array([])
    lat, dev, queue, sizes = np.array(lat), np.array(dev), np.array(queue), np.array(sizes)
    measured = int((arr >= warm).sum())
    ms = lambda a, q: round(float(np.percentile(a, q)) * 1e3, 3) if len(a) else None
    by_size = {}
    for lo, hi in ((0, 1000), (1000, 3000), (3000, 1 << 20)):
        sel = (sizes >= lo) & (sizes < hi)
        by_size["N%d-%d" % (lo, hi)] = {"share": round(float(sel.mean()), 4), "device_ms_p50": ms(dev[sel], 50),
                                        "device_ms_p99": ms(dev[sel], 99), "latency_ms_p50": ms(lat[sel], 50),
                                        "device_s_share": round(float(dev[sel].sum() / max(1e-12, dev.sum())), 4)}
    return dict(workload="Poisson %g req/s (seed 5), q=round(exp(U[ln 8, ln 512])), N=q*U{4..16}, "
                         "p~U[0.05,0.3]; %d unique diagrams cycled; %g s warm-up + %g s measured; %s"
                         % (rate, n_unique, warm, dur,
                            "learned policy with the greedy fallback" if mlp is not None else "greedy policy"),
                requests=len(arr), measured=measured, throughput_req_s=round(measured / max(1e-9, wall - warm), 1),
                p50_ms=ms(lat, 50), p99_ms=ms(lat, 99), max_ms=ms(lat, 100),
                device_ms_p50=ms(dev, 50), device_ms_p99=ms(dev, 99), queue_ms_p50=ms(queue, 50),
                queue_ms_p99=ms(queue, 99), busy_workgroups_mean=round(float(dev.sum()) / max(1e-9, wall - warm), 1),
                by_size=by_size, claim_queue_ms_p50=ms(true_queue, 50), claim_queue_ms_p99=ms(true_queue, 99),
                result_seen_lag_ms_p50=ms(lag, 50), result_seen_lag_ms_p99=ms(lag, 99),
                host_submit_s=round(host_submit_s, 2), host_poll_s=round(host_poll_s, 2),
                drained=drained, completed=done, learned_result_share=round(learned_kept / max(1, len(lat)), 4),
                refused=refused, max_backlog=max_backlog, batches=int(st.batches),
                pool_gib=args.serve_pool_gib, pool_peak_gib=round(st.pool_peak / 2 ** 30, 3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default="all", choices=["all", "rref", "pauli", "batched", "learned", "serve", "copy",
                                                      "parity", "sample", "params", "c1", "extract", "large"])
    ap.add_argument("--learned-states", type=int, default=200000)
    ap.add_argument("--learned-val-states", type=int, default=8000)
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--learned-label", default="fill", choices=["fill", "gate2q"])
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-learned-seconds", type=float, default=20.0)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-unique", type=int, default=2048)
    ap.add_argument("--serve-drain", type=float, default=60.0, help="seconds allowed after the last arrival")
    ap.add_argument("--serve-pool-gib", type=int, default=8)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time")
    ap.add_argument("--rref-strips", action="store_true",
                    help="record per-strip timestamps in the elimination kernel and report them")
    args = ap.parse_args()
    if args.rref_strips:
        os.environ["ZX_RREF_PROFILE"] = "1"
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (the GF(2) "
              "elimination would shard rows across GPUs with a per-strip pivot broadcast; "
              "see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    pool = None
    if args.only in ("all", "batched", "learned", "serve", "pauli", "params", "extract"):
        # worker processes (generation, oracle checks) are forked before any
        # GPU call, so they never inherit an initialised device
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(min(16, os.cpu_count() or 1))
    import torch
    from paper_2604_01059_amd import zx
    zx.load()
    torch.cuda.set_device(0)
    name, n_cu = zx.device_info()
    log("device %s, %d CUs" % (name, n_cu))

    if args.only == "copy":
        # calibration kernel for the HBM byte counters: 256 MiB read + 256 MiB write
        src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 1 << 28, "launches": max(1, args.steps)}))
        return

    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic"}
    if args.only in ("all", "rref"):
        res = bench_rref(zx, args)
        gbs = res["bytes"] / (res["ms"] * 1e-3) / 1e9
        out.update(value=round(gbs, 2), unit="GB/s", ms_per_step=round(res["ms"], 4))
        out["config"] = {"workload": "gf2_rref 4096x16384 Bernoulli(1/2) seed 21 (full RREF)",
                         "m": 4096, "n_cols": 16384, "rank": res["rank"],
                         "word_columns_with_pivots": res["last_strip"] + 1,
                         "strips_32_columns_to_last_pivot": res["strips32"],
                         "algorithmic_bytes_per_step": res["bytes"]}
        out["pct_hbm_peak"] = round(100 * gbs / HBM_PEAK_GBS, 2)
        traffic = rref_traffic_bytes()
        out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                           "traffic_note": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, "
                                           "copy-calibrated) for gf2.hip " + gf2_source_hash()
                                           + ("" if traffic else " (not measured for this source)"),
                           "kernel": "rref_kernel (+ rref_init)", "avg_launch_ms": round(res["ms"], 4),
                           "wall_ms_per_step": round(res["wall_ms"], 4),
                           # the limiter: the serial chain of strip reductions and hand-offs
                           "serial_chain": {"strips": res["strips32"],
                                            "us_per_strip": round(1e3 * res["ms"] / max(1, res["strips32"]), 2)}}
        log("rref: %.4f ms/step, %.1f GB/s algorithmic (%.1f%% of 8 TB/s), rank %d" %
            (res["ms"], gbs, 100 * gbs / HBM_PEAK_GBS, res["rank"]))
        if res["timeline"]:
            out["rref_strip_timeline"] = res["timeline"]
            log("rref strips: %s" % res["timeline"])
        cb, exact = cpu_baseline_rref(res, args.cpu_budget)
        cb["threads"] = 1
        out["cpu_baseline"] = cb
        out["bit_exact_rref_vs_oracle"] = exact
        log("cpu baseline: %s GB/s (%s)" % (cb["value"], cb["sample"]))
    if args.only in ("all", "pauli"):
        out["pauli"] = bench_pauli(zx, max(3, args.steps // 4), pool)
        log("pauli: %s" % out["pauli"])
    if args.only in ("all", "parity"):
        out["parity"] = bench_parity(zx, max(3, args.steps // 4))
        log("parity: %s" % out["parity"])
    if args.only in ("all", "sample"):
        out["sample"] = bench_sample(zx, max(3, args.steps // 4))
        log("sample: %s" % out["sample"])
    if args.only in ("all", "c1"):
        out["c1"] = bench_c1(zx)
        log("c1: %s" % out["c1"])
    if args.only in ("all", "batched"):
        out["batched"] = bench_batched(zx, args, pool)
        log("batched: %s" % out["batched"])
    if args.only in ("all", "params"):
        out["params"] = bench_params(zx, pool)
        log("params: %s" % out["params"])
    if args.only in ("all", "extract"):
        out["extract"] = bench_extract(zx, pool)
        log("extract: %s" % out["extract"])
    if args.only in ("all", "large"):
        out["large"] = bench_large(zx)
        log("large: %s" % out["large"])
    if args.only in ("all", "learned"):
        out["learned"] = bench_learned(zx, args, pool)
        log("learned: %s" % out["learned"])
    if args.only in ("all", "serve"):
        ds = serve_diagrams(args, pool)
        out["serve"] = bench_serve(zx, args, ds)
        log("serve: %s" % out["serve"])
        mlp = getattr(args, "_trained_mlp", None)
        if mlp is None:
            from paper_2604_01059_amd import learned
            mlp = learned.new_network()  # untrained when the learned leg did not run
        out["serve_learned"] = bench_serve(zx, args, ds, mlp=mlp, seconds=args.serve_learned_seconds)
        out["serve_learned"]["network"] = "trained" if hasattr(args, "_trained_mlp") else "untrained"
        log("serve (learned + fallback): %s" % out["serve_learned"])
    if pool is not None:
        pool.close()
        pool.join()
    if "value" not in out:
        out.update(value=None, unit="GB/s", ms_per_step=None, config={"workload": args.only})
    print(json.dumps(out))


if __name__ == "__main__":
    main()
