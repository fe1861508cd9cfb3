"""Benchmark: time to the k smallest Laplacian eigenpairs at relative
residual 1e-8 on one MI355X, plus the SpMV bandwidth of the product kernel.

Workload (one "step" = one full Jacobi-Davidson solve, lap_eigs, with the
plan already resident in HBM): Chung-Lu power-law graph, exponent 2.2,
n = 30,000, mean degree 4, largest connected component (24,137 vertices,
142,967 nonzeros for seed 1001); k = 10 smallest eigenpairs (the zero pair
included), certified at ||Gu - theta u|| <= 1e-8 min(theta, 1); mixed
precision (FP32 products and PCG, FP64 outer iteration).  The same solve in
plain FP64 is timed beside it, and the CPU oracle (the paper's FP64
Algorithm 2 with IC(0)) on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--sweep]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
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


def spmv_bytes(n: int, nnz_a: int, elem: int = 4) -> int:
    """Algorithmic bytes of one unweighted Laplacian product: row pointers,
    column indices, one compulsory read of x and one write of y."""
    return 4 * (n + 1) + 4 * nnz_a + 2 * elem * n


def pcg_iter_bytes(n: int, nnz_a: int, q: int, elem: int = 4) -> int:
    """Algorithmic bytes of one iteration launch of the projected PCG
    (k_pp_iter, unweighted): the CSR structure, one compulsory read of the
    gathered vector wh, nine n-vectors read (dinv, t, res, u, w, p, s, q, z)
    and nine written (t, res, u, w, wh, p, s, q, z), and the rows of Q, GQ
    and G D^-1 Q (3q values per row)."""
    return 4 * (n + 1) + 4 * nnz_a + elem * n * (1 + 9 + 9) + 3 * q * elem * n


def kernel_sources_sha(files=("pcg.hip", "lapeig_dev.h", "lapeig_internal.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1311_1695_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def random_read_rate(n, count, reps=5):
    """Random 4-byte reads per second that the device serves from a vector
    of about n FP32 values (bench_gather.hip, built by __graft_entry__.build:
    indices hashed in registers, no index stream, no locality), or None if
    the helper is not built."""
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


def time_spmv(lap, torch, plan, n, reps=200, dtype=None):
    """Average duration of the FP32 product kernel: `reps` back-to-back
    launches captured in a graph and replayed between two HIP events on the
    stream they run on, so host launch gaps are not counted."""
    dtype = dtype or torch.float32
    x = torch.randn(n, dtype=dtype, device="cuda")
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


PCG_Q = 10  # projector width of the roofline measurement: k = 10 pairs, as in the solve's last steps


def time_pcg_iteration(lap, torch, np, plan, n, q=PCG_Q, reps=5):
    """Average time of one iteration launch of the projected PCG in FP32:
    lap_pcg with rtol = 1e-30 runs exactly itmax iteration launches, so the
    difference of a 40- and a 10-iteration call, timed with HIP events on
    the stream lap_pcg launches on, divided by 30, is one launch (its
    dispatch gap included).  (Beyond about 50 iterations the FP32
    recurrences of this system lose positivity and stop early.)  Q = [1/sqrt(n), q-1 random orthonormal
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


def traffic_from_profile(sha: str, nbytes_alg: int):
    path = os.path.join(ROOT, "profiles", "pp_iter_f32_cl30k_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_sources_sha") != sha:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(L, k, tol, budget_s=12.0):
    import oracle
    times = []
    res = None
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        res = oracle.jd(L, k, tol, precond=oracle.PREC_IC0, seed=1)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end or len(times) >= 20:
            break
    return statistics.median(times), len(times), res


def certify(L, r, tol):
    """Largest relative residual ||Gx - lx|| / min(l, 1) over the non-zero pairs,
    recomputed on the host in FP64."""
    import numpy as np
    G = L.to_scipy()
    res = np.linalg.norm(G @ r.evecs - r.evecs * r.evals, axis=0)
    pos = r.evals > 0
    return float(np.max(res[pos] / np.minimum(r.evals[pos], 1.0))) if pos.any() else 0.0


def extra_configs(lap, torch, gg, np, reps=3):
    """The other workloads: plain FP64 JD on the preferential-attachment
    graph (n = 5000, k = 10) and block JD (b = 20) on the Chung-Lu
    exponent-2.1 graph (n = 330,000, k = 20), mixed and FP64."""
    out = []
    runs = [
        ("pa5k", 10, 1e-8, [("fp64", dict(precision="fp64")), ("mixed", dict(precision="mixed"))]),
        ("cl330k", 20, 1e-8, [("mixed_block20", dict(precision="mixed", block=20, m_min=20, m_max=60)),
                              ("fp64_block20", dict(precision="fp64", block=20, m_min=20, m_max=60)),
                              ("mixed_single", dict(precision="mixed", m_min=5, m_max=10))]),
    ]
    for name, k, tol, variants in runs:
        L = gg.workload(name, SEED)
        plan = lap.Plan(L)
        entry = {"workload": name, "n": L.n, "nnz": L.nnz, "k": k, "tol": tol, "runs": {}}
        for label, kw in variants:
            r = lap.lap_eigs(plan, k, tol, seed=1, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = lap.lap_eigs(plan, k, tol, seed=1, **kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            entry["runs"][label] = {"s": round(dt, 5), "mvp": r.mvp, "outer": r.outer, "inner": r.inner,
                                    "nconv": r.nconv, "max_rel_residual": certify(L, r, tol),
                                    "lambda2": float(r.evals[1]), "lambda_k": float(r.evals[-1])}
        plan.close()
        out.append(entry)
    # a batch of 256 uneven preferential-attachment graphs, 5 pairs each, one launch
    graphs = gg.pa_batch(256, SEED)
    b = lap.lap_batch_create(graphs)
    entry = {"workload": "pa_batch256", "graphs": len(graphs), "sum_n": sum(g.n for g in graphs),
             "sum_nnz": sum(g.nnz for g in graphs), "k": 5, "tol": 1e-8, "runs": {}}
    for label, prec in (("mixed", "mixed"), ("fp64", "fp64")):
        lap.lap_batch_eigs(b, 5, 1e-8, precision=prec)
        t0 = time.perf_counter()
        res = lap.lap_batch_eigs(b, 5, 1e-8, precision=prec)
        dt = time.perf_counter() - t0
        worst = max(certify(L, r, 1e-8) for L, r in zip(graphs[:16], res[:16]))
        entry["runs"][label] = {"s": round(dt, 4), "mvp_total": int(sum(r.mvp for r in res)),
                                "nconv_min": int(min(r.nconv for r in res)),
                                "max_rel_residual_first16": worst}
    b.close()
    out.append(entry)
    return out


def warm_start_config(lap, torch, gg, np, reps=2):
    """The collaboration-like graph (Chung-Lu exponent 2.3, n = 1.1M, mean
    degree 7, triadic closure 0.3, largest component), k = 10 at 1e-8: JD
    started from the learned network's block vs from the seeded random
    vector (mixed precision), and plain FP64 JD from the random vector.
    The network (2 layers, width 32, 4 random channels, 9 columns) is
    trained first, on the GPU, on six graphs of the same family with
    n <= 20k whose eigenvectors lap_eigs computes (tol 1e-6)."""
    t0 = time.perf_counter()
    train = [gg.collaboration(n, s) for n, s in [(8000, 101), (12000, 102), (16000, 103), (20000, 104),
                                                 (10000, 105), (14000, 106)]]
    plans = [lap.Plan(L) for L in train]
    targets = [lap.lap_eigs(p, 10, 1e-6, evecs_on_device=True).evecs[1:].contiguous() for p in plans]
    net = lap.Mpnn(layers=2, hidden=32, random_channels=4, out_cols=9, seed=7)
    losses = []
    for s in range(400):
        g = s % len(plans)
        losses.append(net.train_step(plans[g], targets[g], lr=3e-3, feature_seed=1 + (s // len(plans)) % 4))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for p in plans:
        p.close()
    L = gg.workload("cl1m_tc", SEED)
    plan = lap.Plan(L)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    V0 = net.infer(plan, feature_seed=1)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t1
    entry = {"workload": "cl1m_tc", "n": L.n, "nnz": L.nnz, "k": 10, "tol": 1e-8,
             "network": {"layers": 2, "hidden": 32, "random_channels": 4, "out_cols": 9,
                         "params": net.num_params, "train_steps": 400, "train_s": round(t_train, 3),
                         "loss_first": round(float(np.mean(losses[:6])), 4),
                         "loss_last": round(float(np.mean(losses[-6:])), 4),
                         "infer_ms": round(t_infer * 1e3, 3)},
             "runs": {}}
    variants = [("mixed_warm", dict(precision="mixed", init=V0)), ("mixed_random", dict(precision="mixed")),
                ("fp64_random", dict(precision="fp64"))]
    for label, kw in variants:
        best, r = None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = lap.lap_eigs(plan, 10, 1e-8, seed=1, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        entry["runs"][label] = {"s": round(best, 5), "mvp": r.mvp, "outer": r.outer, "inner": r.inner,
                                "nconv": r.nconv, "max_rel_residual": certify(L, r, 1e-8)}
    entry["runs"]["mixed_warm"]["s_with_inference"] = round(entry["runs"]["mixed_warm"]["s"] + t_infer, 5)
    plan.close()
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--spmv-graph", default="cl30k",
                    help="workload of the --spmv-only leg (cl30k, cl330k, cl1m_tc)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--spmv-only", action="store_true", help="only the product kernel loop (for profiling)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the PCG iteration timing and a copy of known size (for profiling)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the other workloads (pa5k FP64; cl330k block JD; batch)")
    ap.add_argument("--block-only", action="store_true",
                    help="only block JD (b = 20, mixed) on the 330k-vertex graph (for profiling)")
    ap.add_argument("--warmstart", action="store_true",
                    help="also time the learned warm start on the 1.1M-vertex collaboration graph")
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
    if args.block_only:
        Lb = gg.workload("cl330k", SEED)
        pb = lap.Plan(Lb)
        kw = dict(precision="mixed", block=20, m_min=20, m_max=60)
        lap.lap_eigs(pb, 20, TOL, seed=1, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            rb = lap.lap_eigs(pb, 20, TOL, seed=1, **kw)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "cl330k", "block": 20, "s": (time.perf_counter() - t0) / 2,
                          "outer": rb.outer, "inner": rb.inner, "mvp": rb.mvp, "nconv": rb.nconv}))
        return
    L = gg.workload("cl30k", SEED)
    st = L.stats()
    nnz_a = L.nnz - L.n
    plan = lap.Plan(L)

    # ---- the dominant kernel, one PCG iteration launch: live timing for the roofline
    t_pcg = time_pcg_iteration(lap, torch, np, plan, L.n)
    alg_pcg = pcg_iter_bytes(L.n, nnz_a, PCG_Q)
    if args.roofline_only:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"pcg_iter_s": t_pcg, "alg_bytes": alg_pcg, "copy_bytes_each_way": a.numel() * 4}))
        return
    # ---- the plain product kernel, for the SpMV bandwidth of the metric
    if args.spmv_only and args.spmv_graph != "cl30k":
        L = gg.workload(args.spmv_graph, SEED)
        nnz_a = L.nnz - L.n
        plan = lap.Plan(L)
    t_spmv = time_spmv(lap, torch, plan, L.n, reps=2000 if args.spmv_only else 500)
    alg = spmv_bytes(L.n, nnz_a, 4)
    if args.spmv_only:
        # a plain copy of known size, for calibrating HBM counters
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": args.spmv_graph, "spmv_s": t_spmv, "alg_bytes": alg,
                          "copy_bytes_each_way": a.numel() * 4}))
        return

    def solve(precision):
        return lap.lap_eigs(plan, K_PAIRS, TOL, precision=precision, seed=1)

    for _ in range(args.warmup):
        solve("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        runs.append(solve("mixed"))
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    r = runs[-1]

    # plain FP64 Jacobi-Davidson on the same GPU, same seed
    solve("fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f64 = []
    for _ in range(max(3, args.steps // 2)):
        f64.append(solve("fp64"))
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0) / len(f64)
    rf = f64[-1]

    G = L.to_scipy()
    resid = np.linalg.norm(G @ r.evecs - r.evecs * r.evals, axis=0)
    out = {
        "metric": METRIC,
        "value": round(t_mixed, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "chung_lu_gamma2.2_n30000_deg4_lcc", "n": L.n, "nnz": L.nnz,
                   "d_max": st["d_max"], "leaf_frac": round(st["leaf_frac"], 4), "k": K_PAIRS, "tol": TOL,
                   "precision": "mixed", "seed": SEED},
        "solve": {"mvp": r.mvp, "outer": r.outer, "inner": r.inner, "nconv": r.nconv,
                  "max_rel_residual": float(np.max(resid[1:] / np.minimum(r.evals[1:], 1.0))),
                  "evals": [float(x) for x in r.evals]},
        "fp64_jd": {"s": round(t_fp64, 6), "mvp": rf.mvp, "outer": rf.outer, "inner": rf.inner,
                    "speedup_mixed_vs_fp64": round(t_fp64 / t_mixed, 3)},
    }
    sha = kernel_sources_sha()
    achieved = alg_pcg / t_pcg / 1e9
    out["roofline"] = {"kernel": f"k_pp_iter<float> (one projected PCG iteration, q={PCG_Q})", "bound": "hbm",
                       "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic_from_profile(sha, alg_pcg),
                       "alg_bytes_per_launch": alg_pcg, "avg_launch_us": round(t_pcg * 1e6, 3),
                       "kernel_sources_sha": sha}
    a_spmv = alg / t_spmv / 1e9
    out["spmv"] = {"kernel": "k_spmv<float> (unweighted Laplacian product, b=1)", "GB/s": round(a_spmv, 2),
                   "frac": round(a_spmv / HBM_PEAK_GBS, 5), "alg_bytes_per_launch": alg,
                   "avg_launch_us": round(t_spmv * 1e6, 3)}
    # the same product on the large power-law graphs of the other workloads,
    # where it moves tens of megabytes per launch instead of under one
    large, pcg_large = [], []
    for name in ("cl330k", "cl1m_tc"):
        Lb = gg.workload(name, SEED)
        pb = lap.Plan(Lb)
        tb = time_spmv(lap, torch, pb, Lb.n, reps=200)
        nnz_a = Lb.nnz - Lb.n  # one neighbour gather per off-diagonal entry
        ab = spmv_bytes(Lb.n, nnz_a, 4)
        g_spmv = nnz_a / tb
        # at least 16M reads per launch, so that the launch itself does not count
        g_rand = random_read_rate(Lb.n, max(nnz_a, 1 << 24))
        large.append({"workload": name, "n": Lb.n, "nnz": Lb.nnz, "alg_bytes_per_launch": ab,
                      "avg_launch_us": round(tb * 1e6, 3), "GB/s": round(ab / tb / 1e9, 1),
                      "frac": round(ab / tb / 1e9 / HBM_PEAK_GBS, 4),
                      "gathers_per_s": round(g_spmv / 1e9, 1),
                      "random_read_rate_per_s": None if g_rand is None else round(g_rand / 1e9, 1),
                      "frac_of_random_read_rate": None if g_rand is None else round(g_spmv / g_rand, 3),
                      "gather_unit": "1e9 4-byte reads per second"})
        # the dominant kernel at the same sizes: one pipelined PCG iteration,
        # q = 10, FP32, timed as in the roofline leg
        try:
            tp = time_pcg_iteration(lap, torch, np, pb, Lb.n, q=PCG_Q)
            ap = pcg_iter_bytes(Lb.n, nnz_a, PCG_Q)
            pcg_large.append({"workload": name, "n": Lb.n, "q": PCG_Q, "alg_bytes_per_launch": ap,
                              "avg_launch_us": round(tp * 1e6, 3), "GB/s": round(ap / tp / 1e9, 1),
                              "frac": round(ap / tp / 1e9 / HBM_PEAK_GBS, 4)})
        except AssertionError:  # an FP32 breakdown ended a timing call early
            pcg_large.append({"workload": name, "n": Lb.n, "q": PCG_Q, "avg_launch_us": None})
        pb.close()
        del Lb
    out["spmv"]["large_graphs"] = large
    out["pcg_large_graphs"] = {"kernel": "k_pp_iter<float> (one projected PCG iteration)", "runs": pcg_large}
    if args.extra:
        out["configs"] = extra_configs(lap, torch, gg, np)
    if args.warmstart:
        out["warm_start"] = warm_start_config(lap, torch, gg, np)
    if not args.no_cpu:
        t_cpu, reps, cres = cpu_baseline(L, K_PAIRS, TOL)
        out["cpu_baseline"] = {"value": round(t_cpu, 4), "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": f"full solve of the same workload (k={K_PAIRS}, tol={TOL}), "
                                         f"median of {reps} runs; FP64 Algorithm 2 with IC(0), m_min 5, "
                                         f"m_max 10, ITMAX 20, delta_PCG 1e-2",
                               "mvp": cres.mvp, "outer": cres.outer,
                               "speedup_gpu_vs_cpu": round(t_cpu / t_mixed, 2)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
