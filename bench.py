#!/usr/bin/env python3
"""Benchmark of the HDF hot path on one MI355X.

One step = factor build (geometry, degree, radial Gram, compression, factor
evaluation) + K~V with 16 right-hand sides, inputs resident in HBM.  The
adjoint (dF/dl and dF/dX of w^T K~ v) is not part of the measured method;
--with-backward adds it to the step.
Prints one JSON line.  Default workload: N = 1e6 points in d = 5 (10-component
Gaussian mixture scaled to max-norm 1), Cauchy kernel l = 1, tol 1e-4,
binary32 MFMA path; the plain binary64 path on the same inputs is timed
beside it, and the FP64 CPU oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor-build Mpoints/s + K~V GFLOP/s at tol 1e-4, FP32-MFMA vs plain FP64 on GPU"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2202_03655_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.txt")

WORKLOAD_DESC = {
    "gmm5_cauchy_1e-4": "N=1e6 d=5 10-component Gaussian mixture (means N(0,4I), cov 0.25I) centred "
                        "and scaled to max-norm 1; Cauchy l=1; tol 1e-4; 16 RHS",
    "gmm5_cauchy_1e-3": "N=1e6 d=5 10-component Gaussian mixture scaled to max-norm 1; Cauchy l=1; "
                        "tol 1e-3; 16 RHS",
    "cube4_gauss": "N=2e5 uniform in [-1,1]^4; Gaussian l=0.7; tol 1e-5",
    "ball3_gauss": "N=2000 uniform in the unit ball, d=3; Gaussian l=1; tol 1e-6",
    "shell6_matern52_l8": "N=5e5 shell r in [0.9,1.1], d=6; Matern-5/2 l=8; tol 1e-7",
}


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def read_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries (or None).

    Lines: kernel workload source_sha fetch_kib write_kib fetch_factor
    write_factor, the counters per dispatch and the factors that map each
    counter onto the bytes of a plain device copy of known size.
    """
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src = kernel_source_hash()
    for line in open(TRAFFIC_FILE):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if len(f) >= 7 and f[0] == kernel and f[1] == workload:
            if f[2] != src:
                return None          # kernel changed since the counters were taken
            return (float(f[3]) * float(f[5]) + float(f[4]) * float(f[6])) * 1024.0
    return None


def run_gpu(wname, X, V, Wm, precision, steps, warmup, with_backward, rank_rule="bound", storage="factor",
            fused=True):
    import torch
    from paper_2202_03655_amd import hdf
    cfg = hdf_cfg(wname)
    dt = torch.float32 if precision == "mixed" else torch.float64
    prec = hdf.HDF_MIXED if precision == "mixed" else hdf.HDF_FP64
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    Vd = torch.tensor(V, dtype=dt, device="cuda")
    Wd = torch.tensor(Wm, dtype=dt, device="cuda")
    out = torch.empty_like(Vd)

    def step():
        t0 = time.perf_counter()
        f = hdf.Factor(Xd, cfg["kernel"], cfg["l"], cfg["tol"], precision=prec, rank_rule=rank_rule,
                       storage=storage, fused=fused)
        t1 = time.perf_counter()
        f.matvec(Vd, out=out)
        t2 = time.perf_counter()
        grads = f.backward(Wd[:, :1], Vd[:, :1]) if with_backward else None
        t3 = time.perf_counter()
        return f, t1 - t0, grads, t3 - t2

    for _ in range(warmup):
        f, _, _, _ = step()
        f.info()
        del f
    torch.cuda.synchronize()
    rec = dict(build_s=[], bw_s=[], k_build=[], k_mv_t=[], k_mv_n=[], k_mv_red=[], k_adj=[], h_prep=[],
               h_plan=[], h_gram=[], h_compress=[], h_finish=[])
    t_start = time.perf_counter()
    info = None
    for _ in range(steps):
        f, tb, _, tbw = step()
        info = f.info()                      # waits for the step's last kernel
        rec["build_s"].append(tb)
        rec["bw_s"].append(tbw)
        for key in ("prep", "plan", "gram", "compress", "finish"):
            rec["h_" + key].append(info[f"t_{key}_ms"])
        rec["k_build"].append(info["t_build_ms"])
        rec["k_mv_t"].append(info["t_mv_t_ms"])
        rec["k_mv_n"].append(info["t_mv_n_ms"])
        rec["k_mv_red"].append(info["t_mv_reduce_ms"])
        rec["k_adj"].append(info["t_adjoint_ms"])
        del f
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    # build to completion: the build call returns with the factor evaluation still running on the
    # device, so each build here is followed by a device synchronisation before the clock stops
    reps = max(3, steps)
    tb = []
    for _ in range(reps):
        t0 = time.perf_counter()
        f = hdf.Factor(Xd, cfg["kernel"], cfg["l"], cfg["tol"], precision=prec, rank_rule=rank_rule,
                       storage=storage, fused=fused)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        del f
    build_done_s = sorted(tb)[len(tb) // 2]
    # separate matvec timing on a resident factor (wall clock of the call)
    f = hdf.Factor(Xd, cfg["kernel"], cfg["l"], cfg["tol"], precision=prec, rank_rule=rank_rule, storage=storage,
                   fused=fused)
    for _ in range(2):
        f.matvec(Vd, out=out)
    torch.cuda.synchronize()
    reps = max(3, steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        f.matvec(Vd, out=out)
    torch.cuda.synchronize()
    mv_s = (time.perf_counter() - t0) / reps
    del f
    avg = {k: sum(v) / len(v) for k, v in rec.items()}
    return dict(ms_per_step=1e3 * t_total / steps, build_ms=1e3 * build_done_s,
                build_return_ms=1e3 * avg["build_s"], matvec_ms=1e3 * mv_s,
                backward_ms=1e3 * avg["bw_s"],
                build_phases_ms={k[2:]: round(avg[k], 3) for k in ("h_prep", "h_plan", "h_gram", "h_compress",
                                                                   "h_finish")},
                k_build_ms=avg["k_build"], k_mv_t_ms=avg["k_mv_t"], k_mv_n_ms=avg["k_mv_n"],
                k_mv_reduce_ms=avg["k_mv_red"], k_adjoint_ms=avg["k_adj"], info=info)


def run_cross(wname, X, nq, m, precision, steps, warmup):
    """General factor K(X*, X) on the workload's cloud X and nq query points
    drawn from the same family (shifted, seed 9): one step = hdf_build_cross +
    hdf_matvec (m RHS of the training side)."""
    import numpy as np
    import torch
    from paper_2202_03655_amd import hdf, workloads
    cfg = hdf_cfg(wname)
    rng = np.random.default_rng(9)
    Q = X[rng.choice(len(X), nq, replace=False)] * 0.95 + 0.01
    dt = torch.float32 if precision == "mixed" else torch.float64
    prec = hdf.HDF_MIXED if precision == "mixed" else hdf.HDF_FP64
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    Qd = torch.tensor(Q, dtype=dt, device="cuda")
    W = torch.tensor(workloads.rhs(len(X), m, 12), dtype=dt, device="cuda")
    out = torch.empty((nq, m), dtype=dt, device="cuda")

    def step():
        f = hdf.CrossFactor(Qd, Xd, cfg["kernel"], cfg["l"], cfg["tol"], precision=prec)
        f.matvec(W, out=out)
        return f

    for _ in range(warmup):
        step().info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = None
    for _ in range(steps):
        info = step().info()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return {"n_query": nq, "n_train": len(X), "rhs": m, "ms_per_step": round(ms, 3),
            "value": round((nq + len(X)) / (ms * 1e-3) / 1e6, 3), "unit": "Mpoints/s",
            "rank": info["rank"], "degree_p": info["degree_p"],
            "kernel_ms": {"build_both_sides": round(info["t_build_ms"], 4), "matvec_pass1": round(info["t_mv_t_ms"], 4),
                          "matvec_pass2": round(info["t_mv_n_ms"], 4)},
            "step": "hdf_build_cross + hdf_matvec"}


MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
MFMA_FILE = os.path.join(ROOT, "profiles", "pmc_mfma.txt")


def read_mfma_busy(kernel, workload):
    """MFMA pipe busy fraction (SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x SQ_BUSY_CU_CYCLES)) from the
    committed rocprofv3 --pmc summary, or None when the kernels changed since it was taken."""
    if not os.path.exists(MFMA_FILE):
        return None
    src = kernel_source_hash()
    for line in open(MFMA_FILE):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if len(f) >= 4 and f[0] == kernel and f[1] == workload:
            return float(f[3]) if f[2] == src else None
    return None


def run_mfma_line(wname, m, reps=5):
    """The two passes of K~V on a resident factor of workload wname with m right-hand sides (the MFMA-bound
    regime when 2 r m flops per point exceed the ridge times the factor bytes): kernel times from HIP events
    inside the library, algorithmic MFMA flops 2 N r m per pass against the peak of the factor's type."""
    import numpy as np
    import torch
    from paper_2202_03655_amd import hdf, workloads
    cfg = hdf_cfg(wname)
    X = workloads.points(wname).astype(np.float32)
    Xd = torch.tensor(X, device="cuda")
    V = torch.tensor(workloads.rhs(len(X), m, 7).astype(np.float32), device="cuda")
    out = torch.empty_like(V)
    f = hdf.Factor(Xd, cfg["kernel"], cfg["l"], cfg["tol"], precision=hdf.HDF_MIXED)
    for _ in range(2):
        f.matvec(V, out=out)
    t1, t2 = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        f.matvec(V, out=out)
        inf = f.info()
        t1.append(inf["t_mv_t_ms"])
        t2.append(inf["t_mv_n_ms"])
    torch.cuda.synchronize()
    wall = 1e3 * (time.perf_counter() - t0) / reps
    inf = f.info()
    n, r = len(X), inf["rank"]
    ftype = "f32" if inf["factor_precision"] == hdf.HDF_MIXED else "f64"
    flops = 2.0 * n * r * m
    peak = MFMA_PEAK_TFLOPS[ftype]
    p1, p2 = sorted(t1)[len(t1) // 2], sorted(t2)[len(t2) // 2]
    el = 4 if ftype == "f32" else 8
    intensity = flops / ((inf["n_harmonics"] + inf["n_radial"] + m) * el * n)
    return {"workload": wname, "rhs": m, "factor": ftype, "rank": r, "n_points": n,
            "flop_per_byte": round(intensity, 1), "ridge_flop_per_byte": round(peak * 1e12 / 8e12, 1),
            "matvec_ms": round(wall, 3),
            "pass1": {"ms": round(p1, 4), "tflops": round(flops / (p1 * 1e-3) / 1e12, 1), "peak": peak,
                      "frac": round(flops / (p1 * 1e-3) / 1e12 / peak, 4),
                      "pipe_busy_pmc": read_mfma_busy("k_mv_t", f"{wname}:m{m}")},
            "pass2": {"ms": round(p2, 4), "tflops": round(flops / (p2 * 1e-3) / 1e12, 1), "peak": peak,
                      "frac": round(flops / (p2 * 1e-3) / 1e12 / peak, 4),
                      "pipe_busy_pmc": read_mfma_busy("k_mv_n", f"{wname}:m{m}")}}


def hdf_cfg(wname):
    from paper_2202_03655_amd import workloads
    return workloads.CONFIGS[wname]


def cpu_baseline(wname, X, V, n_sample):
    """The FP64 oracle (as it stands) on the first n_sample points of the workload."""
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=cores)
    except Exception:                        # pragma: no cover
        ctx = None
    from oracle import hdf as ohdf
    cfg = hdf_cfg(wname)
    Xs = np.asarray(X[:n_sample], dtype=np.float64)
    Vs = np.asarray(V[:n_sample], dtype=np.float64)
    t0 = time.perf_counter()
    st = ohdf.build(Xs, cfg["kernel"], cfg["l"], cfg["tol"])
    t1 = time.perf_counter()
    ohdf.matvec_chunked(st, Vs, chunk=8192)
    t2 = time.perf_counter()
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    return dict(value=n_sample / (t2 - t0) / 1e6, unit="Mpoints/s", cores=cores, kind="oracle",
                sample=f"first {n_sample} points of the workload (same cloud, same kernel/l/tol), "
                       f"oracle build + K~V with {Vs.shape[1]} RHS; build {t1 - t0:.2f}s, "
                       f"matvec {t2 - t1:.2f}s, rank {st['r']}")


# fp64 VALU lane-instructions per (i, j) pair in the inner loop of the off-diagonal kernel
# k_kmv<8, Gaussian, masked> (its compiled gfx950 assembly, loop unrolled by 4: 140 fp64 + 36 other VALU
# instructions per 4 pairs); the VALU issue peak is 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
KMV_VALU_PER_PAIR = 44.0
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def run_krr(steps):
    """KRR consumer (Sec. 4.2) on the housing-shaped d = 8 workload: k-means, the system with HDF diagonal
    blocks and its preconditioner, PCG to rtol, predictions; everything resident on the device."""
    import numpy as np
    import torch
    from paper_2202_03655_amd import hdf, workloads as wl
    c = wl.KRR
    Xtr, ytr, Xte, yte = wl.housing_split(c["n"])
    Xd = torch.tensor(Xtr, device="cuda")
    yd = torch.tensor(ytr, device="cuda")
    Xq = torch.tensor(Xte, device="cuda")

    def fit_predict():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lab, _, its = hdf.kmeans(Xd, c["clusters"], max_iter=c["kmeans_iter"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sysm = hdf.KRR(Xd, lab, c["clusters"], c["kernel"], c["l"], c["tol"], c["lam"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        w, it, rr = sysm.solve(yd, c["max_iter"], c["rtol"])
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        pred = hdf.kernel_matvec(Xq, Xd, w, c["kernel"], c["l"])
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        return dict(kmeans=t1 - t0, create=t2 - t1, solve=t3 - t2, predict=t4 - t3, its=its, it=it, rr=rr,
                    sysm=sysm, w=w, pred=pred, lab=lab)

    fit_predict()
    runs = [fit_predict() for _ in range(max(1, steps))]
    med = {k: float(np.median([r[k] for r in runs])) * 1e3 for k in ("kmeans", "create", "solve", "predict")}
    last = runs[-1]
    sysm, inf = last["sysm"], last["sysm"].info()
    # off-diagonal kernel: HIP events around its launch inside hdf_krr_apply
    v = torch.randn(len(Xtr), dtype=torch.float64, device="cuda")
    od = []
    for _ in range(10):
        sysm.apply(v)
        od.append(sysm.info()["t_offdiag_ms"])
    od_ms = float(np.mean(od[2:]))
    n = len(Xtr)
    sizes = np.bincount(last["lab"].cpu().numpy(), minlength=c["clusters"])
    pairs = float(n) * n - float((sizes.astype(np.float64) ** 2).sum())
    evals = float(n) * n            # the kernel evaluates every pair and masks the own cluster
    achieved = evals / (od_ms * 1e-3)
    peak = VALU_PEAK_LANE_OPS / KMV_VALU_PER_PAIR
    mse = float(((last["pred"].cpu().numpy() - yte) ** 2).mean())
    fit = med["kmeans"] + med["create"] + med["solve"]
    # relative Frobenius error of every diagonal-block factor against the exact block (the quantity the
    # paper reports per cluster): K~_cc from the factor applied to identity columns, K_cc in binary64 by torch
    labels = last["lab"].cpu().numpy()
    ls = c["l"]
    block_err = []
    for cl in range(c["clusters"]):
        blk = sysm.block(cl)
        if blk is None:
            continue
        Xc = Xd[torch.tensor(np.flatnonzero(labels == cl), device="cuda")]
        nc = Xc.shape[0]
        r2 = torch.cdist(Xc, Xc) ** 2
        Kc = torch.exp(-r2 / (2.0 * ls * ls)) if c["kernel"] == "gaussian" else None
        Kt = torch.empty((nc, nc), dtype=torch.float64, device="cuda")
        for j0 in range(0, nc, 256):
            j1 = min(nc, j0 + 256)
            E = torch.zeros((nc, j1 - j0), dtype=torch.float64, device="cuda")
            E[torch.arange(j0, j1, device="cuda"), torch.arange(j1 - j0, device="cuda")] = 1.0
            Kt[:, j0:j1] = blk.matvec(E)
        if Kc is not None:
            block_err.append(float(torch.linalg.norm(Kt - Kc) / torch.linalg.norm(Kc)))
    return {
        "workload": f"housing8_krr: N={c['n']} d=8 housing-shaped cloud, {n} train / {len(Xte)} test, "
                    f"{c['clusters']} k-means clusters, {c['kernel']} l={c['l']}, block tol {c['tol']}, "
                    f"lambda {c['lam']}, PCG to rtol {c['rtol']} (max {c['max_iter']})",
        "fit_ms": round(fit, 2), "fit_predict_ms": round(fit + med["predict"], 2),
        "phases_ms": {k: round(v, 2) for k, v in med.items()},
        "create_ms": {"factors": round(inf["t_factor_ms"], 2), "precond": round(inf["t_precond_ms"], 2)},
        "kmeans_iterations": last["its"], "cg_iterations": last["it"], "relres": last["rr"],
        "ms_per_cg_iteration": round(med["solve"] / max(1, last["it"]), 4),
        "test_mse": mse, "label_var": float(np.var(yte)),
        "blocks": {"n": inf["n_blocks"], "max": inf["max_block"], "max_degree": inf["max_degree"],
                   "sum_rank": inf["sum_rank"], "factor_bytes": inf["factor_bytes"],
                   "precond_bytes": inf["precond_bytes"],
                   "rel_fro_error": {"max": max(block_err), "median": float(np.median(block_err)),
                                     "min": min(block_err), "tol": c["tol"]} if block_err else None},
        "offdiag_kernel": {"ms": round(od_ms, 4), "pair_evals": evals, "offdiag_pairs": pairs,
                           "roofline": {"kernel": "k_kmv", "bound": "alu", "achieved": round(achieved / 1e9, 1),
                                        "peak": round(peak / 1e9, 1), "unit": "Gpair/s",
                                        "frac": round(achieved / peak, 4),
                                        "valu_per_pair": KMV_VALU_PER_PAIR}},
        "_state": (Xtr, ytr, last["lab"].cpu().numpy()),
    }


def krr_cpu_baseline(Xtr, ytr, labels):
    """The oracle on the same system: block factors and preconditioner, then two CG iterations."""
    import numpy as np
    from oracle import krr
    from paper_2202_03655_amd import workloads as wl
    c = wl.KRR
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    S = krr.create(Xtr, labels, c["clusters"], c["kernel"], c["l"], c["tol"], c["lam"])
    t1 = time.perf_counter()
    krr.solve(S, ytr, 0.0, 2)
    t2 = time.perf_counter()
    return dict(value=round((t2 - t1) / 2 * 1e3, 1), unit="ms per CG iteration", cores=cores, kind="oracle",
                create_ms=round((t1 - t0) * 1e3, 1),
                sample="the full housing8_krr system (same labels): oracle block factors + Cholesky "
                       "preconditioner, then 2 PCG iterations")


def calibrate_copy(nbytes):
    """Plain device copy of known size, used to scale the PMC byte counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gmm5_cauchy_1e-4")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--rhs", type=int, default=16)
    ap.add_argument("--no-fp64", action="store_true", help="skip the binary64 comparison path")
    ap.add_argument("--no-sampled", action="store_true", help="skip the run with the sampled degree/rank rule")
    ap.add_argument("--with-backward", action="store_true",
                    help="add hdf_backward (dF/dl and dF/dX, one right-hand side) to the step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=400000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES")
    ap.add_argument("--no-krr", action="store_true", help="skip the KRR consumer (Sec. 4.2)")
    ap.add_argument("--no-matrix-free", action="store_true", help="skip the matrix-free factor run")
    ap.add_argument("--no-mfma-lines", action="store_true", help="skip the 64-RHS (MFMA-bound) product lines")
    ap.add_argument("--mfma-line", default="", metavar="WORKLOAD",
                    help="run only the 64-RHS product of WORKLOAD and print its JSON object (for profiling)")
    ap.add_argument("--krr-only", action="store_true",
                    help="run only the KRR consumer and print its JSON object (for profiling)")
    ap.add_argument("--cross", type=int, default=0, metavar="NQ",
                    help="also time the general factor K(X*, X) (X* = NQ query points) and its product")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sharding is a design, not code); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    from paper_2202_03655_amd import hdf, workloads
    hdf.lib()
    if args.mfma_line:
        print(json.dumps({"mfma_line": run_mfma_line(args.mfma_line, 64)}), flush=True)
        return
    if args.krr_only:
        kr = run_krr(max(1, args.steps))
        kr.pop("_state")
        print(json.dumps({"krr": kr}), flush=True)
        return
    cfg = workloads.CONFIGS[args.workload]
    X = workloads.points(args.workload)
    if args.precision == "mixed":
        X = X.astype(np.float32).astype(np.float64)     # the values the mixed path consumes
    N, d = X.shape
    m = args.rhs
    V = workloads.rhs(N, m, 7)
    Wm = workloads.rhs(N, m, 8)
    # hdf_backward (dF/dl and dF/dX) is not part of the default step: the
    # measured method is the build and the product
    with_backward = args.with_backward
    print(f"# workload {args.workload}: N={N} d={d} precision={args.precision}", file=sys.stderr, flush=True)
    res = run_gpu(args.workload, X, V, Wm, args.precision, args.steps, args.warmup, with_backward)
    info = res["info"]
    r, H, S = info["rank"], info["n_harmonics"], info["n_radial"]
    el = 4 if args.precision == "mixed" else 8
    # algorithmic work per launch
    build_bytes = N * (d * el + (H + S) * el)
    mv_flops = 4.0 * N * r * m
    mvt_bytes = N * (H + S + m) * el
    mvn_bytes = N * (H + S + m) * el
    kernels = {"k_build": (res["k_build_ms"], build_bytes), "k_mv_t": (res["k_mv_t_ms"], mvt_bytes),
               "k_mv_n": (res["k_mv_n_ms"], mvn_bytes)}
    # launches per step: pass 1 runs once in hdf_matvec and once in
    # hdf_backward (U^T [V | W] in one pass); the dominant kernel has the
    # largest device time per step
    per_step = {"k_build": res["k_build_ms"], "k_mv_t": res["k_mv_t_ms"] * (2 if with_backward else 1),
                "k_mv_n": res["k_mv_n_ms"]}
    dom = max(per_step, key=lambda k: per_step[k])
    t_ms, nbytes = kernels[dom]
    achieved = nbytes / (t_ms * 1e-3) / 1e9
    traffic = read_traffic(dom, args.workload)
    print(f"# step {res['ms_per_step']:.2f} ms (build {res['build_ms']:.2f} ms {res['build_phases_ms']}, "
          f"matvec {res['matvec_ms']:.3f} ms, backward {res['backward_ms']:.2f} ms); "
          f"kernels build {res['k_build_ms']:.3f} mv_t {res['k_mv_t_ms']:.3f} mv_n {res['k_mv_n_ms']:.3f} "
          f"adjoint {res['k_adjoint_ms']:.3f} ms; "
          f"p={info['degree_p']} r={r} H={H} S={S}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": round(N / (res["ms_per_step"] * 1e-3) / 1e6, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "desc": WORKLOAD_DESC.get(args.workload, ""),
                   "n_points": N, "dim": d, "kernel": cfg["kernel"], "lengthscale": cfg["l"],
                   "tol": cfg["tol"], "rhs": m, "precision": args.precision,
                   "step": "hdf_build + hdf_matvec(16 RHS)" + (" + hdf_backward" if with_backward else "")},
        "build_mpoints_s": round(N / (res["build_ms"] * 1e-3) / 1e6, 3),
        "build_ms": round(res["build_ms"], 3),
        "build_return_ms": round(res["build_return_ms"], 3),
        "matvec_gflops": round(mv_flops / (res["matvec_ms"] * 1e-3) / 1e9, 1),
        "kernel_ms": {"build": round(res["k_build_ms"], 4), "matvec_pass1": round(res["k_mv_t_ms"], 4),
                      "matvec_reduce": round(res["k_mv_reduce_ms"], 4), "matvec_pass2": round(res["k_mv_n_ms"], 4),
                      **({"adjoint": round(res["k_adjoint_ms"], 4)} if with_backward else {})},
        "factor": {"p": info["degree_p"], "rank": r, "harmonics": H, "radial": S,
                   "bytes": info["factor_bytes"]},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / (t_ms * 1e-3) / 1e9, 1),
                     "algorithmic_bytes": nbytes},
    }
    if args.precision == "mixed" and not args.no_fp64:
        r64 = run_gpu(args.workload, X, V, Wm, "fp64", max(2, args.steps // 2), 1, with_backward)
        out["fp64"] = {"ms_per_step": round(r64["ms_per_step"], 3),
                       "value": round(N / (r64["ms_per_step"] * 1e-3) / 1e6, 3),
                       "build_mpoints_s": round(N / (r64["build_ms"] * 1e-3) / 1e6, 3),
                       "matvec_gflops": round(4.0 * N * r64["info"]["rank"] * m / (r64["matvec_ms"] * 1e-3) / 1e9, 1),
                       "rank": r64["info"]["rank"]}
        out["speedup_vs_fp64"] = round(r64["ms_per_step"] / res["ms_per_step"], 3)
    if not args.no_sampled:
        # the tighter degree / rank rule (remark after Eq. bound) on the same inputs
        rs = run_gpu(args.workload, X, V, Wm, args.precision, args.steps, args.warmup, False, "sampled")
        si = rs["info"]
        out["sampled_rule"] = {"ms_per_step": round(rs["ms_per_step"], 3),
                               "value": round(N / (rs["ms_per_step"] * 1e-3) / 1e6, 3),
                               "build_ms": round(rs["build_ms"], 3), "matvec_ms": round(rs["matvec_ms"], 3),
                               "p": si["degree_p"], "p_bound": si["degree_bound"], "rank": si["rank"],
                               "tau": si["tau"], "tau_bound": si["tau_bound"],
                               "est_error": si["est_error"]}
    if not args.no_matrix_free:
        # the same step with nothing stored per point: the factor is re-evaluated in each pass, by the
        # fused kernels (16 points at a time in LDS) and, for comparison, chunk by chunk into a scratch
        out["matrix_free"] = {}
        for fused in (True, False):
            rm = run_gpu(args.workload, X, V, Wm, args.precision, args.steps, args.warmup, False, "bound", "none",
                         fused=fused)
            mi = rm["info"]
            fl = 2.0 * N * mi["rank"] * m
            ob = {"ms_per_step": round(rm["ms_per_step"], 3),
                  "value": round(N / (rm["ms_per_step"] * 1e-3) / 1e6, 3),
                  "build_ms": round(rm["build_ms"], 3), "matvec_ms": round(rm["matvec_ms"], 3),
                  "pass1_with_eval_ms": round(rm["k_mv_t_ms"], 4),
                  "pass2_with_eval_ms": round(rm["k_mv_n_ms"], 4),
                  "pass1_mfma_tflops": round(fl / (rm["k_mv_t_ms"] * 1e-3) / 1e12, 1),
                  "pass2_mfma_tflops": round(fl / (rm["k_mv_n_ms"] * 1e-3) / 1e12, 1),
                  "fused": mi["mf_fused"], "chunk_points": None if mi["mf_fused"] else mi["chunk_points"],
                  "scratch_bytes": mi["factor_bytes"], "stored_factor_bytes": info["factor_bytes"],
                  "stored_matvec_ms": round(res["matvec_ms"], 3), "rank": mi["rank"]}
            out["matrix_free"]["fused" if fused else "chunked"] = ob
            print(f"# matrix-free ({'fused' if fused else 'chunked'}): step {ob['ms_per_step']} ms, product "
                  f"{ob['matvec_ms']} ms (stored {ob['stored_matvec_ms']} ms), pass 1 {ob['pass1_with_eval_ms']} ms, "
                  f"pass 2 {ob['pass2_with_eval_ms']} ms", file=sys.stderr, flush=True)
    # MFMA: the passes' algorithmic flops (2 N r m each) against the FP32 MFMA peak, live; the MFMA pipe
    # busy fraction from the committed PMC summary (None once the kernels changed)
    fl = 2.0 * N * r * m
    ptype = "f32" if info["factor_precision"] == 1 else "f64"
    pk = MFMA_PEAK_TFLOPS[ptype]
    out["mfma"] = {
        "peak_tflops": pk,
        "pass1": {"tflops": round(fl / (res["k_mv_t_ms"] * 1e-3) / 1e12, 1),
                  "frac": round(fl / (res["k_mv_t_ms"] * 1e-3) / 1e12 / pk, 4),
                  "pipe_busy_pmc": read_mfma_busy("k_mv_t", args.workload)},
        "pass2": {"tflops": round(fl / (res["k_mv_n_ms"] * 1e-3) / 1e12, 1),
                  "frac": round(fl / (res["k_mv_n_ms"] * 1e-3) / 1e12 / pk, 4),
                  "pipe_busy_pmc": read_mfma_busy("k_mv_n", args.workload)},
        "gram": {"pipe_busy_pmc": read_mfma_busy("k_gram", args.workload)},
    }
    if not args.no_mfma_lines:
        # 64 right-hand sides: 2 r m flops per point above the ridge times the factor bytes (MFMA-bound)
        out["mfma_lines"] = [run_mfma_line(args.workload, 64)]
        if args.workload != "shell6_matern52_l8":
            out["mfma_lines"].append(run_mfma_line("shell6_matern52_l8", 64))
        for ln in out["mfma_lines"]:
            print(f"# m=64 {ln['workload']} ({ln['factor']} factor, {ln['flop_per_byte']} flop/B): pass 1 "
                  f"{ln['pass1']['ms']} ms {ln['pass1']['tflops']} TF ({ln['pass1']['frac']:.2%}), pass 2 "
                  f"{ln['pass2']['ms']} ms {ln['pass2']['tflops']} TF ({ln['pass2']['frac']:.2%})",
                  file=sys.stderr, flush=True)
    if args.cross:
        out["cross"] = run_cross(args.workload, X, args.cross, m, args.precision, args.steps, args.warmup)
    if not args.no_krr:
        kr = run_krr(max(1, args.steps // 2))
        state = kr.pop("_state")
        print(f"# krr fit {kr['fit_ms']} ms {kr['phases_ms']}, {kr['cg_iterations']} CG iterations "
              f"({kr['ms_per_cg_iteration']} ms each), off-diagonal kernel {kr['offdiag_kernel']['ms']} ms",
              file=sys.stderr, flush=True)
        if not args.no_cpu_baseline:
            kr["cpu_baseline"] = krr_cpu_baseline(*state)
        out["krr"] = kr
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, X, V, min(args.cpu_sample, N))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
