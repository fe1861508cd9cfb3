"""Benchmark: time to the k smallest Laplacian eigenpairs at relative
residual 1e-8 on one MI355X, FP32 + learned warm start against plain FP64
Jacobi-Davidson, plus the bandwidth of the Laplacian product.

Workload (one "step" = inference of the warm-start network plus one full
Jacobi-Davidson solve, lap_eigs in its block form with a 10-column block,
started from the network's block, with the plan already resident in HBM): the collaboration-like graph, Chung-Lu
exponent 2.3, n = 1.1M, mean degree 7, triadic closure p = 0.3, largest
connected component (1,032,939 vertices, 10,697,907 nonzeros of G for seed
1001); k = 10 smallest eigenpairs (the zero pair included), each certified
at ||Gu - theta u|| <= 1e-8 min(theta, 1) in FP64; mixed precision (FP32
products and PCG, FP64 outer iteration).  The network is trained first, on
the GPU, on eigenvectors that lap_eigs computes for graphs of the same
family with n <= 50k.  Beside it: the 2 x 2 table {mixed, FP64} x {random
start, network start} for block JD and for the single-vector Algorithm 2
(plain FP64 JD is the baseline), the FSAI preconditioner, the per-pair error against the FP64 oracle's
eigenvalues (tests/golden, written by an oracle-only script), the product's
bandwidth (FP32, FP64, 20-column block), a copy bandwidth, the other
workloads, and the CPU oracle on a bounded sample of the same solve.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-configs]
    python bench.py --sweep          # product bandwidth on graphs past the 256 MB MALL

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to k eigenpairs @ rel.res 1e-8 + SpMV GB/s; FP32+warm-start vs FP64 JD"
HBM_PEAK_GBS = 8000.0
SEED = 1001
K_PAIRS = 10
TOL = 1e-8
WORKLOAD = "cl1m_tc"
GOLDEN = os.path.join(ROOT, "tests", "golden", "cl1m_tc_k10.json")
PCG_Q = 10  # projector width of the roofline measurement: [zero vector, 8 locked, u] at the last pair
# training graphs of the warm-start network: the same family, n <= 50k
TRAIN_GRAPHS = [(10000, 101), (20000, 102), (30000, 103), (40000, 104), (50000, 105),
                (15000, 106), (25000, 107), (35000, 108), (45000, 109)]
TRAIN_STEPS = 450
NET = dict(layers=2, hidden=32, random_channels=4, out_cols=9, seed=7)
# the headline solver: block JD, a 10-column block (the network's 9 columns
# and one seeded random column start it), basis between 20 and 50 columns
HEADLINE = dict(block=10, m_min=20, m_max=50)


def spmv_bytes(n: int, nnz_a: int, elem: int = 4, b: int = 1) -> int:
    """Algorithmic bytes of one unweighted Laplacian product over b columns:
    row pointers, column indices, one compulsory read of X and one write of
    Y (n x b values each)."""
    return 4 * (n + 1) + 4 * nnz_a + 2 * elem * b * n


def pcg_iter_bytes(n: int, nnz_a: int, q: int, elem: int = 4) -> int:
    """Algorithmic bytes of one launch of the one-launch projected-PCG
    iteration (two-sided preconditioner (I-QQ')D^-1(I-QQ')): the product's
    row offsets and column indices, one read of the gathered vector, and
    every other n-vector once: the 3q columns of Q, G Q and G D^-1 Q, D^-1
    and eight iterate vectors read, nine vectors written (the product's
    result stays in registers, so spmv_bytes' write of y is not counted)."""
    return spmv_bytes(n, nnz_a, elem) - n * elem + (3 * q + 18) * n * elem


def kernel_sources_sha(files=("spmv.hip", "lapeig_dev.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1311_1695_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def random_read_rate(n, count, reps=5):
    """Random 4-byte reads per second that the device serves from a vector
    of about n FP32 values (bench_gather.hip: indices hashed in registers, no
    index stream, no locality), or None if the helper is not built."""
    import ctypes
    path = os.path.join(ROOT, "bench_gather.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.bench_random_reads.argtypes = [ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double)]
    rate = ctypes.c_double(0.0)
    rc = lib.bench_random_reads(n, count, reps, ctypes.byref(rate))
    return rate.value if rc == 0 else None


def random_row_rate(n, b, count, reps=5):
    """Random whole-row reads per second that the device serves from an
    n x b FP32 row-major array (bench_gather.hip: b / 2 lanes per row with
    8-byte loads, as the block product reads a neighbour; indices hashed in
    registers, no locality), or None if the helper is not built."""
    import ctypes
    path = os.path.join(ROOT, "bench_gather.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    if not hasattr(lib, "bench_random_rows"):
        return None
    lib.bench_random_rows.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.c_longlong, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_double)]
    rate = ctypes.c_double(0.0)
    rc = lib.bench_random_rows(n, b, count, reps, ctypes.byref(rate))
    return rate.value if rc == 0 else None


def time_spmv(lap, torch, plan, n, reps=200, dtype=None, b=1):
    """Average duration of the product kernel: `reps` back-to-back launches
    captured in a graph and replayed between two HIP events on the stream
    they run on, so host launch gaps are not counted."""
    dtype = dtype or torch.float32
    x = torch.randn((n, b) if b > 1 else (n,), dtype=dtype, device="cuda")
    y = torch.empty_like(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(5):
            lap.lap_spmv(plan, x, y, plan_order=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            lap.lap_spmv(plan, x, y, plan_order=True)
    g.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(3):
        e0.record(s)
        g.replay()
        e1.record(s)
        e1.synchronize()
        t = e0.elapsed_time(e1) / reps * 1e-3
        best = t if best is None else min(best, t)
    return best  # seconds per launch


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second) of a
    buffer far larger than the 256 MB MALL."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.copy_(a)
    e1.record(s)
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2 * nbytes / t


def time_pcg_iteration(lap, torch, np, plan, n, q=PCG_Q, reps=5):
    """Average time of one iteration launch of the projected PCG in FP32:
    lap_pcg with rtol = 1e-30 runs exactly itmax iteration launches, so the
    difference of a 40- and a 10-iteration call, timed with HIP events on
    the stream lap_pcg launches on, divided by 30, is one launch (its
    dispatch gap included).  Q = [1/sqrt(n), q-1 random orthonormal
    columns], theta = 0: the projected operator is positive definite, so no
    breakdown ends the iteration early."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, q))
    X[:, 0] = 1.0
    Q = np.linalg.qr(X)[0]
    r = rng.standard_normal(n)
    r -= Q @ (Q.T @ r)
    Qt = torch.tensor(Q.T.copy(), device="cuda")
    Rt = torch.tensor(r[None, :].copy(), device="cuda")
    Tt = torch.zeros_like(Rt)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run(its):
        best = None
        for _ in range(reps):
            e0.record(s)
            got = lap.lap_pcg(plan, 0.0, Qt, Rt, Tt, itmax=its, rtol=1e-30, dtype="f32", stream=s)
            e1.record(s)
            e1.synchronize()
            assert int(got[0]) == its, "the timing run stopped early"
            t = e0.elapsed_time(e1) * 1e-3
            best = t if best is None else min(best, t)
        return best

    run(40)
    return (run(40) - run(10)) / 30.0


def traffic_from_profile(sha: str):
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "spmm_b10_f32_cl1m_tc_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_sources_sha") != sha:
        return None
    return d.get("hbm_bytes_per_launch")


def host_info():
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(L, golden, budget_outer=15):
    """The CPU oracle (FP64 Algorithm 2 with IC(0), paper parameters, one
    thread) on a bounded sample of the same solve: the first `budget_outer`
    outer iterations (IC(0) set-up included), scaled to the full solve by
    the products the full oracle solve needs (tests/golden, measured by the
    oracle-only script at the same graph, seed and k)."""
    import oracle
    t0 = time.perf_counter()
    res = oracle.jd(L, K_PAIRS, TOL, precond=oracle.PREC_IC0, seed=1, kmax=budget_outer)
    dt = time.perf_counter() - t0
    full = (golden.get("oracle_at_tol") or golden["oracle"]) if golden else None
    full_mvp = full["mvp"] if full else None
    est = dt / res.mvp * full_mvp if (full_mvp and res.mvp) else None
    return dt, res, est, full_mvp


def host_evecs(r):
    """The eigenvectors of a result as an n x k host array (a result kept on
    the device holds them as a k x n tensor)."""
    E = r.evecs
    if hasattr(E, "cpu"):
        E = E.cpu().numpy().T
    return E


def certify(L, r):
    """Largest relative residual ||Gx - lx|| / min(l, 1) over the non-zero
    pairs, recomputed on the host in FP64."""
    import numpy as np
    G = L.to_scipy()
    E = host_evecs(r)
    res = np.linalg.norm(G @ E - E * r.evals, axis=0)
    pos = r.evals > 0
    return float(np.max(res[pos] / np.minimum(r.evals[pos], 1.0))) if pos.any() else 0.0


def pair_errors(evals, golden):
    """|theta_gpu - theta_oracle| / theta_oracle per pair (absolute for the
    zero pair)."""
    ref = golden["evals"]
    out = []
    for a, b in zip(evals, ref):
        out.append(float(abs(a - b) / b) if b > 0 else float(abs(a - b)))
    return out


def median_time(fn, reps, torch):
    times, last = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        last = fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    return statistics.median(times), times, last


def train_network(lap, torch, gg, np):
    """Train the warm-start network on the GPU on eigenvectors that lap_eigs
    computes for same-family graphs with n <= 50k (k = 10, tol 1e-6)."""
    t0 = time.perf_counter()
    train = [gg.collaboration(n, s) for n, s in TRAIN_GRAPHS]
    t_gen = time.perf_counter() - t0
    t1 = time.perf_counter()
    plans = [lap.Plan(L) for L in train]
    targets = [lap.lap_eigs(p, K_PAIRS, 1e-6, evecs_on_device=True).evecs[1:].contiguous() for p in plans]
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t1
    net = lap.Mpnn(**NET)
    losses = []
    t2 = time.perf_counter()
    for s in range(TRAIN_STEPS):
        g = s % len(plans)
        losses.append(net.train_step(plans[g], targets[g], lr=3e-3, feature_seed=1 + (s // len(plans)) % 4))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t2
    for p in plans:
        p.close()
    info = {"train_graphs_n": [L.n for L in train], "train_steps": TRAIN_STEPS, "params": net.num_params,
            **{k: v for k, v in NET.items() if k != "seed"},
            "targets_s": round(t_targets, 3), "train_s": round(t_train, 3), "graph_gen_s": round(t_gen, 2),
            "loss_first": round(float(np.mean(losses[:len(plans)])), 4),
            "loss_last": round(float(np.mean(losses[-len(plans):])), 4)}
    return net, info


def extra_configs(lap, torch, gg, np, reps=3):
    """The other workloads: plain FP64 JD on the preferential-attachment
    graph (n = 5000, k = 10), mixed vs FP64 on the Chung-Lu exponent-2.2
    graph (n = 30,000, k = 10), block JD (b = 20) on the Chung-Lu
    exponent-2.1 graph (n = 330,000, k = 20), and the batch of 256 uneven
    preferential-attachment graphs (5 pairs each, one launch); times with
    the eigenvectors left in device memory, and with their copy to the
    host beside them."""
    out = []
    runs = [
        ("pa5k", 10, [("fp64", dict(precision="fp64")), ("mixed", dict(precision="mixed"))]),
        ("cl30k", 10, [("mixed", dict(precision="mixed")), ("fp64", dict(precision="fp64"))]),
        ("cl330k", 20, [("mixed_block20", dict(precision="mixed", block=20, m_min=20, m_max=60)),
                        ("fp64_block20", dict(precision="fp64", block=20, m_min=20, m_max=60))]),
    ]
    for name, k, variants in runs:
        L = gg.workload(name, SEED)
        plan = lap.Plan(L)
        entry = {"workload": name, "n": L.n, "nnz": L.nnz, "k": k, "tol": TOL, "runs": {}}
        for label, kw in variants:
            # timed with the eigenvectors left in HBM (as the headline step),
            # the call that copies them to host memory beside it
            lap.lap_eigs(plan, k, TOL, seed=1, evecs_on_device=True, **kw)
            dt, _, r = median_time(lambda: lap.lap_eigs(plan, k, TOL, seed=1, evecs_on_device=True, **kw), reps,
                                   torch)
            dt_host, _, rh = median_time(lambda: lap.lap_eigs(plan, k, TOL, seed=1, **kw), reps, torch)
            assert np.array_equal(r.evecs.cpu().numpy().T, rh.evecs)
            entry["runs"][label] = {"s": round(dt, 5), "s_evecs_to_host": round(dt_host, 5), "mvp": r.mvp,
                                    "outer": r.outer, "inner": r.inner, "nconv": r.nconv,
                                    "max_rel_residual": certify(L, rh),
                                    "lambda2": float(r.evals[1]), "lambda_k": float(r.evals[-1])}
        plan.close()
        out.append(entry)
    out.append(methods_entry(lap, torch, gg, np, reps))
    out.append(batch_entry(lap, torch, gg, np))
    return out


def methods_entry(lap, torch, gg, np, reps=3):
    """The paper's comparison of the three eigensolvers (JD, IRLM with PCG
    inner solves, DACG), here on the Chung-Lu exponent-2.2 graph (n = 30,000),
    10 smallest pairs at 1e-6 (DACG's last digits to 1e-8 are dominated by
    rounding on this graph), all from the seeded start, Jacobi-preconditioned."""
    L = gg.workload("cl30k", SEED)
    plan = lap.Plan(L)
    tol = 1e-6
    entry = {"workload": "cl30k_methods", "n": L.n, "nnz": L.nnz, "k": 10, "tol": tol, "runs": {}}
    calls = (("jd_fp64", lambda: lap.lap_eigs(plan, 10, tol, precision="fp64", seed=1)),
             ("jd_mixed", lambda: lap.lap_eigs(plan, 10, tol, precision="mixed", seed=1)),
             ("irlm_fp64", lambda: lap.lap_eigs_irlm(plan, 10, tol, precision="fp64", seed=1)),
             ("dacg_fp64", lambda: lap.lap_eigs_dacg(plan, 10, tol, seed=1, kmax=40000, allow_noconv=True)))
    for label, fn in calls:
        fn()
        dt, _, r = median_time(fn, reps, torch)
        entry["runs"][label] = {"s": round(dt, 5), "mvp": int(r.mvp), "outer": int(r.outer), "inner": int(r.inner),
                                "nconv": int(r.nconv),
                                "max_rel_residual": certify(L, r) if r.nconv == 10 else None}
    plan.close()
    return entry


def batch_entry(lap, torch, gg, np):
    """The batch of 256 uneven preferential-attachment graphs (5 pairs each,
    one persistent launch) in both precisions: time to k with the vectors
    left in device memory (and with their copy to the host), products, the
    autotuned row-class threshold, and the aggregate product bandwidth:
    every graph's products times its algorithmic product bytes (offsets,
    indices, one read of x, one write of y, at the PCG's precision; the FP64
    outer products are counted at that precision too), over the time."""
    graphs = gg.pa_batch(256, SEED)
    b = lap.lap_batch_create(graphs)
    sum_nnz = sum(g.nnz for g in graphs)
    entry = {"workload": "pa_batch256", "graphs": len(graphs), "sum_n": sum(g.n for g in graphs),
             "sum_nnz": sum_nnz, "k": 5, "tol": TOL, "runs": {}}
    for label, prec, elem in (("mixed", "mixed", 4), ("fp64", "fp64", 8)):
        t0 = time.perf_counter()
        thr, pass_s = b.autotune(prec)
        t_tune = time.perf_counter() - t0
        # timed with the eigenvectors left in HBM (as the headline step); the
        # same solve with the copy of the vectors to host memory beside it
        lap.lap_batch_eigs(b, 5, TOL, precision=prec, evecs_on_device=True)
        dt, _, _ = median_time(lambda: lap.lap_batch_eigs(b, 5, TOL, precision=prec, evecs_on_device=True), 2,
                               torch)
        dt_host, _, res = median_time(lambda: lap.lap_batch_eigs(b, 5, TOL, precision=prec), 2, torch)
        worst = max(certify(L, r) for L, r in zip(graphs, res))
        prod_bytes = sum(int(r.mvp) * spmv_bytes(L.n, L.nnz - L.n, elem) for L, r in zip(graphs, res))
        entry["runs"][label] = {"s": round(dt, 4), "s_evecs_to_host": round(dt_host, 4),
                                "mvp_total": int(sum(r.mvp for r in res)),
                                "nconv_min": int(min(r.nconv for r in res)),
                                "max_rel_residual": worst, "long_threshold": thr,
                                "autotune_s": round(t_tune, 3), "product_pass_us": round(pass_s * 1e6, 1),
                                "aggregate_product_GB/s": round(prod_bytes / dt / 1e9, 1),
                                "aggregate_product_frac": round(prod_bytes / dt / 1e9 / HBM_PEAK_GBS, 4)}
    b.close()
    return entry


def spmv_entries(lap, torch, gg, np, L, plan):
    """Bandwidth of the Laplacian product on the headline graph: FP32 and
    FP64 on one vector, FP32 on a 20-column block, with the gather rate and
    the random-read rate of the device beside it."""
    n, nnz_a = L.n, L.nnz - L.n
    out = []
    for label, dt, b, elem in (("f32_b1", torch.float32, 1, 4), ("f64_b1", torch.float64, 1, 8),
                               ("f32_b20", torch.float32, 20, 4)):
        t = time_spmv(lap, torch, plan, n, reps=100 if b > 1 else 200, dtype=dt, b=b)
        ab = spmv_bytes(n, nnz_a, elem, b)
        out.append({"kernel": "k_spmv" if b == 1 else "k_spmm", "dtype": label.split("_")[0], "b": b,
                    "alg_bytes_per_launch": ab, "avg_launch_us": round(t * 1e6, 3),
                    "GB/s": round(ab / t / 1e9, 1), "frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4),
                    "gathers_per_s_1e9": round(nnz_a / t / 1e9, 1)})
    rr = random_read_rate(n, max(nnz_a, 1 << 24))
    return out, (None if rr is None else round(rr / 1e9, 1))


def relabel(gg, np, L, perm):
    """The same graph with vertex perm[k] renamed k."""
    A = L.to_scipy().tocoo()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    r, c, v = inv[A.row], inv[A.col], A.data
    up = r < c
    w = -v[up]
    return gg.laplacian_from_edges(L.n, r[up], c[up], None if np.all(w == 1.0) else w, name=L.name)


def order_experiment(lap, torch, gg, np, orders):
    """Products on the headline graph with the vertices of one degree in the
    plan's hub order, or in the caller's order for three labellings of the
    graph: the generator's, a random one, and reverse Cuthill-McKee (a
    breadth-first locality order)."""
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    L0 = gg.workload(WORKLOAD, SEED)
    for o in orders:
        if o in ("hub", "caller_gen"):
            L = L0
        elif o == "caller_random":
            L = relabel(gg, np, L0, np.random.default_rng(3).permutation(L0.n))
        elif o == "caller_rcm":
            L = relabel(gg, np, L0, reverse_cuthill_mckee(L0.to_scipy().tocsr(), symmetric_mode=True).astype(np.int64))
        else:
            raise SystemExit(f"unknown order {o}")
        plan = lap.Plan(L, order="hub" if o == "hub" else "caller")
        nnz_a = L.nnz - L.n
        t1 = time_spmv(lap, torch, plan, L.n, reps=100, dtype=torch.float32, b=1)
        t10 = time_spmv(lap, torch, plan, L.n, reps=100, dtype=torch.float32, b=10)
        t10d = time_spmv(lap, torch, plan, L.n, reps=50, dtype=torch.float64, b=10)
        print(json.dumps({"order": o, "workload": WORKLOAD, "row_gathers": nnz_a,
                          "spmv_f32_us": round(t1 * 1e6, 2), "spmm_b10_f32_us": round(t10 * 1e6, 2),
                          "spmm_b10_f64_us": round(t10d * 1e6, 2)}), flush=True)
        plan.close()


def sweep(lap, torch, gg, np):
    """The product on the collaboration-like generator at n = 1.1M, 4.4M and
    8.8M (the FP32 working set grows past the 256 MB MALL)."""
    rows = []
    for n in (1_100_000, 4_400_000, 8_800_000):
        t0 = time.perf_counter()
        L = gg.collaboration(n, SEED)
        tg = time.perf_counter() - t0
        plan = lap.Plan(L)
        nnz_a = L.nnz - L.n
        for label, dt, b, elem in (("f32", torch.float32, 1, 4), ("f64", torch.float64, 1, 8),
                                   ("f32", torch.float32, 20, 4)):
            t = time_spmv(lap, torch, plan, L.n, reps=50, dtype=dt, b=b)
            ab = spmv_bytes(L.n, nnz_a, elem, b)
            rows.append({"n_generated": n, "n": L.n, "nnz": L.nnz, "dtype": label, "b": b,
                         "alg_bytes_per_launch": ab, "avg_launch_us": round(t * 1e6, 2),
                         "GB/s": round(ab / t / 1e9, 1), "frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4),
                         "gen_s": round(tg, 1)})
            print(json.dumps(rows[-1]), flush=True)
        plan.close()
        del L
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads")
    ap.add_argument("--spmv-only", default=None, metavar="GRAPH",
                    help="only the product kernel loop on one workload (for profiling)")
    ap.add_argument("--pcg-q", type=int, default=PCG_Q,
                    help="projector width of the PCG-iteration timing of --roofline-only")
    ap.add_argument("--order-exp", nargs="*", default=None, metavar="ORDER",
                    help="product timings of the headline graph under vertex orders inside a degree: hub (the "
                         "plan's default), and the caller's order with the generator's, a random or a reverse "
                         "Cuthill-McKee labelling (caller_gen, caller_random, caller_rcm); all four if none named")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batch of 256 preferential-attachment graphs, both precisions")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the PCG iteration timing on the headline graph and a copy of known size "
                         "(for profiling)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the headline solves, no training (random start; for profiling)")
    ap.add_argument("--headline-only", action="store_true",
                    help="train the network, then three timed headline steps (network start; for profiling)")
    ap.add_argument("--block-only", action="store_true",
                    help="only block JD (b = 20, mixed) on the 330k-vertex graph (for profiling)")
    ap.add_argument("--sweep", action="store_true",
                    help="only the product bandwidth on generated graphs of 1.1M, 4.4M and 8.8M vertices")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1311_1695_amd as lap
    from paper_1311_1695_amd import graphgen as gg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lap.load_library()
    if args.sweep:
        rows = sweep(lap, torch, gg, np)
        print(json.dumps({"spmv_sweep": rows, "copy_GB/s": round(copy_bandwidth(torch) / 1e9, 1)}))
        return
    if args.block_only:
        Lb = gg.workload("cl330k", SEED)
        pb = lap.Plan(Lb)
        kw = dict(precision="mixed", block=20, m_min=20, m_max=60)
        lap.lap_eigs(pb, 20, TOL, seed=1, evecs_on_device=True, **kw)
        dt, _, rb = median_time(lambda: lap.lap_eigs(pb, 20, TOL, seed=1, evecs_on_device=True, **kw), 2, torch)
        print(json.dumps({"workload": "cl330k", "block": 20, "s": dt, "outer": rb.outer, "inner": rb.inner,
                          "mvp": rb.mvp, "nconv": rb.nconv}))
        return
    if args.batch_only:
        entry = batch_entry(lap, torch, gg, np)
        entry["copy_GB/s"] = round(copy_bandwidth(torch, 256 << 20, reps=20) / 1e9, 1)
        print(json.dumps(entry), flush=True)
        return
    if args.order_exp is not None:
        order_experiment(lap, torch, gg, np, args.order_exp or ["hub", "caller_gen", "caller_random", "caller_rcm"])
        return
    if args.spmv_only:
        Ls = gg.workload(args.spmv_only, SEED)
        ps = lap.Plan(Ls)
        t = time_spmv(lap, torch, ps, Ls.n, reps=500)
        cb = copy_bandwidth(torch, 256 << 20, reps=20)
        print(json.dumps({"workload": args.spmv_only, "spmv_s": t, "alg_bytes": spmv_bytes(Ls.n, Ls.nnz - Ls.n),
                          "copy_bytes_each_way": 256 << 20, "copy_GB/s": round(cb / 1e9, 1)}))
        return

    t0 = time.perf_counter()
    L = gg.workload(WORKLOAD, SEED)
    t_gen = time.perf_counter() - t0
    st = L.stats()
    nnz_a = L.nnz - L.n
    t0 = time.perf_counter()
    plan = lap.Plan(L)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    print(f"bench: {WORKLOAD} n={L.n} nnz={L.nnz} generated in {t_gen:.1f}s, plan {t_plan:.2f}s",
          file=sys.stderr, flush=True)

    # ---- the dominant kernel of the headline solve (block JD, b = 10): the
    # 10-column FP32 block product of its PCG, live timing for the roofline;
    # beside it one iteration of the single-vector pipelined PCG
    t_blk = time_spmv(lap, torch, plan, L.n, reps=100, dtype=torch.float32, b=HEADLINE["block"])
    alg_blk = spmv_bytes(L.n, nnz_a, 4, HEADLINE["block"])
    t_pcg = time_pcg_iteration(lap, torch, np, plan, L.n, q=args.pcg_q)
    alg_pcg = pcg_iter_bytes(L.n, nnz_a, args.pcg_q)
    if args.roofline_only:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        rows_rate = random_row_rate(L.n, HEADLINE["block"], max(nnz_a, 1 << 24))
        print(json.dumps({"workload": WORKLOAD, "block_product_s": t_blk, "block_alg_bytes": alg_blk,
                          "row_gathers": nnz_a, "random_row_rate": rows_rate,
                          "pcg_iter_s": t_pcg, "alg_bytes": alg_pcg, "copy_bytes_each_way": a.numel() * 4}))
        return
    if args.solve_only:
        # the headline solver's kernels (block JD, mixed precision) from the random start
        lap.lap_eigs(plan, K_PAIRS, TOL, precision="mixed", seed=1, evecs_on_device=True, **HEADLINE)
        dt, _, r = median_time(lambda: lap.lap_eigs(plan, K_PAIRS, TOL, precision="mixed", seed=1, evecs_on_device=True,
                                                    **HEADLINE), 2, torch)
        print(json.dumps({"solver": HEADLINE, "s": dt, "outer": r.outer, "mvp": r.mvp}), flush=True)
        return

    golden = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as fh:
            golden = json.load(fh)
        assert golden["n"] == L.n and golden["nnz"] == L.nnz, "golden file does not match the workload"

    net, net_info = train_network(lap, torch, gg, np)
    print(f"bench: network trained, loss {net_info['loss_first']} -> {net_info['loss_last']}",
          file=sys.stderr, flush=True)
    if args.headline_only:
        def one():
            V0 = net.infer(plan, feature_seed=1)
            return lap.lap_eigs(plan, K_PAIRS, TOL, precision="mixed", seed=1, init=V0, evecs_on_device=True,
                                **HEADLINE)
        one()
        dt, _, r = median_time(one, 3, torch)
        print(json.dumps({"solver": HEADLINE, "start": "network", "s": dt, "outer": r.outer, "mvp": r.mvp}),
              flush=True)
        return

    def step(precision="mixed"):
        V0 = net.infer(plan, feature_seed=1)
        # the eigenvectors stay in HBM: the timed step holds no host transfer
        return lap.lap_eigs(plan, K_PAIRS, TOL, precision=precision, seed=1, init=V0, evecs_on_device=True,
                            **HEADLINE)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        runs.append(step())
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    r = runs[-1]

    # inference alone
    t_inf, _, V0 = median_time(lambda: net.infer(plan, feature_seed=1), 5, torch)
    # the 2 x 2 table {mixed, FP64} x {random, network} for the headline
    # solver (block JD, b = 10) and for the paper's single-vector Algorithm 2,
    # same seeds; plus single-vector JD with the FSAI preconditioner
    table = {}
    cells = [("block10_mixed_network", dict(precision="mixed", init=V0, **HEADLINE)),
             ("block10_mixed_random", dict(precision="mixed", **HEADLINE)),
             ("block10_fp64_network", dict(precision="fp64", init=V0, **HEADLINE)),
             ("block10_fp64_random", dict(precision="fp64", **HEADLINE)),
             ("single_mixed_network", dict(precision="mixed", init=V0)),
             ("single_mixed_random", dict(precision="mixed")),
             ("single_fp64_network", dict(precision="fp64", init=V0)),
             ("single_fp64_random", dict(precision="fp64")),
             ("single_mixed_random_fsai", dict(precision="mixed", precond="fsai")),
             ("single_fp64_random_fsai", dict(precision="fp64", precond="fsai"))]
    for label, kw in cells:
        lap.lap_eigs(plan, K_PAIRS, TOL, seed=1, evecs_on_device=True, **kw)
        dt, times, rr = median_time(lambda: lap.lap_eigs(plan, K_PAIRS, TOL, seed=1, evecs_on_device=True, **kw),
                                    3, torch)
        table[label] = {"solve_s": round(dt, 5), "mvp": rr.mvp, "outer": rr.outer, "inner": rr.inner,
                        "nconv": rr.nconv, "warm_start_used": rr.warm_start_used,
                        "max_rel_residual": certify(L, rr)}
        if golden:
            table[label]["max_pair_err_vs_oracle"] = max(pair_errors(rr.evals, golden))
    t_fp64 = table["single_fp64_random"]["solve_s"]

    G = L.to_scipy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E = host_evecs(r)  # the PCIe leg a caller who wants the vectors on the host adds
    t_d2h = time.perf_counter() - t0
    resid = np.linalg.norm(G @ E - E * r.evals, axis=0)
    out = {
        "metric": METRIC,
        "value": round(t_step, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "collaboration_like_chung_lu_gamma2.3_n1.1M_deg7_triadic0.3_lcc", "name": WORKLOAD,
                   "n": L.n, "nnz": L.nnz, "d_max": st["d_max"], "leaf_frac": round(st["leaf_frac"], 4),
                   "k": K_PAIRS, "tol": TOL, "precision": "mixed", "start": "learned network block",
                   "solver": f"block JD, block {HEADLINE['block']}, m_min {HEADLINE['m_min']}, "
                             f"m_max {HEADLINE['m_max']}",
                   "step": "network inference + lap_eigs from its block", "seed": SEED},
        "solve": {"mvp": r.mvp, "outer": r.outer, "inner": r.inner, "nconv": r.nconv,
                  "max_rel_residual": float(np.max(resid[1:] / np.minimum(r.evals[1:], 1.0))),
                  "evals": [float(x) for x in r.evals],
                  "pair_err_vs_oracle": pair_errors(r.evals, golden) if golden else None,
                  "oracle_evals_tol": golden["oracle_tol"] if golden else None},
        "speedup_vs_plain_fp64_jd": round(t_fp64 / t_step, 3),
        "plain_fp64_jd": "single-vector Algorithm 2 in FP64 from the seeded random start (single_fp64_random)",
        "start_x_precision": table,
        "inference_s": round(t_inf, 5),
        "evecs_to_host_s": round(t_d2h, 5),
        "network": net_info,
        "plan_create_s": round(t_plan, 3),
    }
    sha = kernel_sources_sha()
    achieved = alg_blk / t_blk / 1e9
    out["roofline"] = {"kernel": f"k_spmm<float> + k_spmm_combine<float>: the {HEADLINE['block']}-column FP32 "
                                 f"block product of the block PCG ({WORKLOAD}), the largest share of the "
                                 f"headline solve's kernel time",
                       "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic_from_profile(sha),
                       "alg_bytes_per_launch": alg_blk, "avg_launch_us": round(t_blk * 1e6, 3),
                       "kernel_sources_sha": sha}
    rows_rate = random_row_rate(L.n, HEADLINE["block"], max(nnz_a, 1 << 24))
    out["roofline"]["gather_bound"] = {
        "what": "the product's neighbour-row gathers (nnz_A rows of b FP32 values per launch) against the rate "
                "at which the device serves random whole-row reads from an array of the same shape "
                "(bench_gather.hip, no index stream, no locality)",
        "row_gathers_per_launch": nnz_a, "achieved_rows_per_s_1e9": round(nnz_a / t_blk / 1e9, 2),
        "random_row_rate_1e9_per_s": None if rows_rate is None else round(rows_rate / 1e9, 2),
        "frac": None if rows_rate is None else round(nnz_a / t_blk / rows_rate, 4)}
    pcg_runs = []
    for qq in (6, PCG_Q):
        tq = t_pcg if qq == args.pcg_q else time_pcg_iteration(lap, torch, np, plan, L.n, q=qq)
        aq = pcg_iter_bytes(L.n, nnz_a, qq)
        pcg_runs.append({"q": qq, "achieved_GB/s": round(aq / tq / 1e9, 1), "frac": round(aq / tq / 1e9 / HBM_PEAK_GBS, 4),
                         "alg_bytes_per_launch": aq, "avg_launch_us": round(tq * 1e6, 3)})
    out["pcg_iteration"] = {"kernel": f"k_pp_iter<float> (one projected PCG iteration of single-vector JD, "
                                      f"{WORKLOAD})", "runs": pcg_runs}
    sp, rr_rate = spmv_entries(lap, torch, gg, np, L, plan)
    out["spmv"] = {"workload": WORKLOAD, "runs": sp, "random_read_rate_1e9_per_s": rr_rate,
                   "copy_GB/s": round(copy_bandwidth(torch) / 1e9, 1)}
    plan.close()
    net.close()
    if not args.no_configs:
        out["configs"] = extra_configs(lap, torch, gg, np)
    if not args.no_cpu:
        t_cpu, cres, est, full_mvp = cpu_baseline(L, golden)
        out["cpu_baseline"] = {"value": None if est is None else round(est, 2), "unit": "s", "cores": 1,
                               "kind": "oracle", **host_info(),
                               "sample": f"oracle (FP64 Algorithm 2, IC(0), paper parameters, one thread) on the "
                                         f"same graph, k={K_PAIRS}, tol={TOL}, seed 1: first {cres.outer} outer "
                                         f"iterations ({cres.mvp} products, IC(0) set-up included) in "
                                         f"{t_cpu:.2f}s, scaled by the {full_mvp} products of the full oracle "
                                         f"solve", "sample_s": round(t_cpu, 3), "sample_mvp": cres.mvp,
                               "speedup_gpu_vs_cpu": None if est is None else round(est / t_step, 1)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
