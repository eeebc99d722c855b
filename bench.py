#!/usr/bin/env python
"""Benchmark of the streaming chiral-SVD multigrid hot path on one MI355X.

Metric: seconds of the multigrid solve to a true relative residual of 1e-10 (mixed
FP32-inner / FP64-outer, compared with the plain FP64 path), dslash bandwidth and setup
seconds.  One step is one pass of the whole hot path on the workload: setup (Philox test
vectors, GMRES smoothing, chiral split, streaming SVD over all streams, P and R, Galerkin
coarse operator) followed by the MG-preconditioned solve of one Gaussian right-hand side.

Prints one JSON line.  `value` is the median mixed-precision solve time (s) over the timed
steps; `roofline` describes the dominant kernel measured live with HIP events over the timed
region; `cpu_baseline` is the CPU oracle timed on this host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="aniso16x32_fp32")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparator solve")
    ap.add_argument("--mass", type=float, default=None, help="override the workload's quark mass")
    return ap.parse_args()


def cpu_baseline(w, counts):
    """Time the oracle's unit operations on this workload and scale by the solve's op counts."""
    import numpy as np
    import fields
    from oracle import wilson, transfer, coarse, geometry as geo, krylov  # noqa: F401

    dims, block, k = w["dims"], w["block"], w["rank"]
    V = geo.volume(dims)
    cd = geo.coarse_dims(dims, block)
    d = geo.volume(cd)
    N = 6 * int(np.prod(block))
    rng = np.random.default_rng(0)
    U = fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])
    psi = fields.gaussian_spinor(dims, 1, w["seed"])[0]
    P, _ = np.linalg.qr(rng.standard_normal((d, 2, N, k)) + 1j * rng.standard_normal((d, 2, N, k)))
    Y = rng.standard_normal((d, 9, 2 * k, 2 * k)) + 1j * rng.standard_normal((d, 9, 2 * k, 2 * k))
    vc = rng.standard_normal((1, d, 2, k)) + 1j * rng.standard_normal((1, d, 2, k))

    def tm(f, n):
        t0 = time.perf_counter()
        for _ in range(n):
            f()
        return (time.perf_counter() - t0) / n

    t_D = tm(lambda: wilson.apply_wilson(U, psi, w["mass"], w["xi"], w["bc_t"], dims), 3)
    t_Dc = tm(lambda: coarse.coarse_apply(Y, vc, cd), 5)
    t_RP = tm(lambda: transfer.prolong(P, transfer.restrict(P, psi[None], dims, block), dims, block), 2)
    a, b = psi.ravel(), psi.ravel().copy()
    t_vec = tm(lambda: (np.vdot(a, b), b + 0.5 * a), 5)
    est = (counts["dslash"] * t_D + counts["coarse_apply"] * t_Dc + counts["restrict"] * t_RP
           + counts["vector_ops"] * t_vec)
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return {
        "value": est, "unit": "s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle unit operations timed on this workload ({dims}, k={k}): Wilson D apply "
                   f"{t_D:.3f}s, coarse apply {t_Dc:.4f}s, restrict+prolong {t_RP:.3f}s, fine vector op "
                   f"{t_vec:.4f}s; scaled by the GPU solve's operation counts {counts}; numpy stencil code "
                   f"is single-threaded ({ncpu} host cpus visible)"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU runs are not part "
              f"of this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import fields
    from fields import workloads
    import paper_2505_14399_amd as q

    if args.mass is not None:
        w = dict(workloads.WORKLOADS[args.workload], name=args.workload, mass=args.mass)
    else:
        w = workloads.get(args.workload)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(fields.gaussian_spinor(dims, 1, w["seed"], tag=w["tag"])).cuda()
    setup_kw = dict(block=w["block"], n_test=w["n_test"], batch=w["batch"], rank=w["rank"], n_setup_iter=16,
                    n_post_smooth=8, coarse_tol=0.03, coarse_max_iter=500, inner=w["inner"], seed=w["seed"])

    def step():
        t0 = time.perf_counter()
        mg = q.mg_setup_stream_chiral_svd(lat, U, **setup_kw)
        t1 = time.perf_counter()
        x, info = q.mg_solve(mg, b, tol=args.tol)
        t2 = time.perf_counter()
        mg.close()
        return t1 - t0, t2 - t1, info[0]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    q.timing_enable(True)
    setups, solves, infos = [], [], []
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    for _ in range(args.steps):
        ts, tv, info = step()
        setups.append(ts)
        solves.append(tv)
        infos.append(info)
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    fams = {f: q.timing_query(f) for f in ("dslash", "isvd", "coarse_apply", "prolong", "restrict",
                                           "coarse_build")}
    q.timing_enable(False)
    for i in infos:
        if i["true_rel_res"] > args.tol:
            raise SystemExit(f"solve did not reach {args.tol}: {i}")

    # operation counts of one mixed solve (for the CPU baseline), from an untimed solve
    mg = q.mg_setup_stream_chiral_svd(lat, U, **setup_kw)
    q.timing_enable(True)
    _, sinfo = q.mg_solve(mg, b, tol=args.tol)
    cnt = {f: q.timing_query(f)["launches"] for f in ("dslash", "coarse_apply", "restrict")}
    q.timing_enable(False)
    mg.close()
    cnt["vector_ops"] = 12 * (sinfo[0]["smoother_iters"] + sinfo[0]["outer_iters"])

    # FP64 comparator on the same lattice (own FP64 setup, untimed)
    fp64_solve = None
    if not args.no_fp64 and w["inner"] != "f64":
        kw64 = dict(setup_kw, inner="f64")
        mg64 = q.mg_setup_stream_chiral_svd(lat, U, **kw64)
        ts64 = []
        for _ in range(2):
            t0 = time.perf_counter()
            _, i64 = q.mg_solve(mg64, b, tol=args.tol)
            ts64.append(time.perf_counter() - t0)
        mg64.close()
        fp64_solve = {"s": float(np.median(ts64)), "outer_iters": i64[0]["outer_iters"],
                      "true_rel_res": i64[0]["true_rel_res"]}

    # dominant kernel by summed device time in the timed region
    dom = max(fams, key=lambda f: fams[f]["ms"])
    ds = fams["dslash"]
    ds_avg_ms = ds["ms"] / max(1, ds["launches"])
    ds_gbps = ds["bytes"] / max(1, ds["launches"]) / (ds_avg_ms * 1e-3) / 1e9
    fam = fams[dom]
    avg_ms = fam["ms"] / max(1, fam["launches"])
    if dom == "isvd":
        ach = fam["flops"] / max(1, fam["launches"]) / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64_TFLOPS, "traffic": None, "kernel": "isvd", "avg_launch_ms": avg_ms}
    else:
        ach = fam["bytes"] / max(1, fam["launches"]) / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBPS,
                "traffic": None, "kernel": dom, "avg_launch_ms": avg_ms}

    res = {
        "metric": "MG solve s to rel.res 1e-10 (mixed vs FP64); dslash HBM GB/s; setup s",
        "value": float(np.median(solves)),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": (T1 - T0) / args.steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner, f64 outer" if w["inner"] == "f32" else w["inner"],
        "data": "synthetic",
        "config": {"workload": w["name"], "lattice": list(dims), "xi": w["xi"], "eps": w["eps"],
                   "mass": w["mass"], "bc_t": w["bc_t"], "block": list(w["block"]), "n_test": w["n_test"],
                   "batch": w["batch"], "rank": w["rank"], "nrhs": 1, "tol": args.tol},
        "setup_s": float(np.median(setups)),
        "solve_fp64": fp64_solve,
        "solve_info": infos[-1],
        "dslash": {"launches": ds["launches"], "avg_launch_us": ds_avg_ms * 1e3, "GBps": ds_gbps,
                   "frac_hbm": ds_gbps / PEAK_HBM_GBPS},
        "kernel_ms_per_step": {f: fams[f]["ms"] / args.steps for f in fams},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, cnt)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
