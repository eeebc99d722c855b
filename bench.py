#!/usr/bin/env python
"""Benchmark of the streaming chiral-SVD multigrid hot path on one MI355X.

Metric: seconds of the multigrid solve to a true relative residual of 1e-10 (mixed
FP32-inner / FP64-outer, compared with the plain FP64 path), dslash bandwidth and setup
seconds.  One step is one pass of the whole hot path on the workload: setup (Philox test
vectors, GMRES smoothing, chiral split, streaming SVD over all streams, P and R, Galerkin
coarse operator, the half-lattice fields of the even-odd smoother) followed by the
MG-preconditioned solve of one Gaussian right-hand side, whose fine-level post-smoother works on
the even-odd Schur system with its GMRES(8) steps in s-step form (`--plain-smoother`: GMRES on D;
the line reports the other smoother's solve on the same hierarchy beside it), and whose coarse
solve runs GMRES(32) on the even-odd Schur complement of D_c where every coarse extent is even
and the hierarchy has two levels (`--full-coarse`: on D_c; the other coarse solve on the same
hierarchy is reported beside it).

Prints one JSON line.  `value` is the median mixed-precision solve time (s) over the timed
steps; `roofline` describes the dominant kernel measured live with HIP events over the timed
region; `cpu_baseline` is the CPU oracle timed on this host on a bounded sample; `dslash_hbm` is
the dslash's algorithmic bandwidth on a 32^3 x 64 lattice (fields larger than the 256 MB
last-level cache) at 1 and 12 right-hand sides; `clover` is the same pair for the Wilson-clover
operator (site term fused into the stencil) and the clover multigrid (setup and mixed-precision
solve) on the same 16^3 x 32 anisotropic lattice with unit clover coefficients and a mass
tuned for that operator; `evenodd` is the even-odd Schur operator's bandwidth on 32^3 x 64 and
its GMRES solve against GMRES on the full operator.  `--workload aniso16x32_clover` makes the clover workload the main line.

Counter runs: `bench.py --traffic-probe` runs three 256 MiB device copies (calibration) and one
step of the benchmark as timed; run it
under `rocprofv3 --pmc FETCH_SIZE` and, separately, `--pmc WRITE_SIZE`, then
`bench.py --traffic-from FETCH_DIR WRITE_DIR` writes profiles/traffic.json (bytes per launch,
scaled by the copy calibration, with the SHA-256 of the kernel source) and a text summary.
`roofline.traffic` is filled from that record while the kernel source is unchanged.
"""
import argparse
from types import SimpleNamespace
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
TIMING_SAMPLE = 4  # time about one launch in 4 of each kernel family in the timed region
COPY_BYTES = 256 << 20
# timing family -> (kernel symbol prefix in counter output, source file)
FAMILY_KERNEL = {
    "dslash/dir": ("k_dslash_dir", "dslash.hip"),
    "dslash/site": ("k_dslash<", "dslash.hip"),
    "dslash/twalk": ("k_dslash_t<", "dslash.hip"),
    "coarse_apply": ("k_coarse_apply", "transfer.hip"),
    "restrict": ("k_restrict", "transfer.hip"),
    "prolong": ("k_prolong", "transfer.hip"),
    "coarse_build": ("k_build_coarse", "transfer.hip"),
    "evenodd/hop": ("k_hop_eo", "dslash.hip"),
    "coarse_eo": ("k_coarse_eo_apply", "coarse_evenodd.hip"),
    "sstep/gram": ("k_sstep_gram", "evenodd.hip"),
    "blas/axpby": ("k_axpby<", "krylov.hip"),
    "blas/axpy_multi": ("k_axpy_multi", "krylov.hip"),
    "batch/dslash": ("k_dslash_padded", "dslash.hip"),
    "batch/coarse_build": ("k_b_galerkin", "batch.hip"),
}
FAMILIES = ("dslash/site", "dslash/twalk", "dslash/dir", "isvd", "coarse_apply", "prolong", "restrict",
            "coarse_build", "evenodd/hop", "coarse_eo")
CLOVER_FAMILIES = tuple(f.replace("dslash/", "clover/") for f in FAMILIES)
CLOVER_WORKLOAD = "aniso16x32_clover"


def progress(msg):
    """One line on stderr per finished phase (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


_ROCTX = []


def roctx(push=None):
    """roctx range around the timed region, so that a kernel trace (rocprofv3 --marker-trace) can
    be cut to it; a no-op without the profiler library."""
    import ctypes
    if not _ROCTX:
        try:
            lib = ctypes.CDLL("librocprofiler-sdk-roctx.so.1")
            lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            _ROCTX.append(lib)
        except OSError:
            _ROCTX.append(None)
    lib = _ROCTX[0]
    if lib is None:
        return
    if push:
        lib.roctxRangePushA(push.encode())
    else:
        lib.roctxRangePop()


def trace_summary(args):
    """Per-kernel and per-family device time inside the timed region (the roctx range
    "bench/timed") from a rocprofv3 --kernel-trace --marker-trace CSV output folder."""
    d = args.trace_summary
    ktr = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    mtr = glob.glob(os.path.join(d, "**", "*marker_api_trace.csv"), recursive=True)
    if not ktr or not mtr:
        raise SystemExit(f"need *kernel_trace.csv and *marker_api_trace.csv under {d}")
    t0, t1 = None, None
    for f in mtr:
        for r in csv.DictReader(open(f)):
            if any(v == "bench/timed" for v in r.values()):
                a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                t0 = a if t0 is None else min(t0, a)
                t1 = b if t1 is None else max(t1, b)
    if t0 is None:
        raise SystemExit("no bench/timed range in the marker trace")
    per = {}
    for f in ktr:
        for r in csv.DictReader(open(f)):
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            if a >= t0 and b <= t1:
                e = per.setdefault(r["Kernel_Name"], [0, 0])
                e[0] += 1
                e[1] += b - a
    short = lambda n: n.replace("qmg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
    total = sum(v[1] for v in per.values())
    steps = args.steps
    out = [f"timed region {(t1 - t0) * 1e-9:.3f} s ({steps} steps), kernel time {total * 1e-9:.3f} s, "
           f"{sum(v[0] for v in per.values())} dispatches", "",
           "| family | kernel instances | dispatches | ms per step | average launch us |", "|---|---:|---:|---:|---:|"]
    for fam, (prefix, _) in FAMILY_KERNEL.items():
        ks = [k for k in per if short(k).startswith(prefix)]
        if not ks:
            continue
        n = sum(per[k][0] for k in ks)
        t = sum(per[k][1] for k in ks)
        out.append(f"| {fam} | {len(ks)} | {n} | {t * 1e-6 / steps:.2f} | {t / n * 1e-3:.1f} |")
    out += ["", "| kernel | dispatches | ms per step | average us |", "|---|---:|---:|---:|"]
    for k, (n, t) in sorted(per.items(), key=lambda kv: -kv[1][1])[:30]:
        out.append(f"| `{short(k)[:100]}` | {n} | {t * 1e-6 / steps:.2f} | {t / n * 1e-3:.1f} |")
    print("\n".join(out))


DSLASH_VARIANTS = {1: (8, 10008, 16), 4: (208, 1208, 11208, 8, 10008),
                   8: (11204, 11208, 10204, 10208, 1204, 10008, 10004),
                   12: (308, 1308, 11308, 1208, 11208, 8, 10008)}


def dslash_variants(args):
    """The Wilson stencil's launch forms on 32^3 x 64 (FP32, random links) at 1, 4 and 12
    right-hand sides: per form the average launch (HIP events, 10 launches after 3 warm-up
    launches), its algorithmic bandwidth and its largest deviation from the first form.  With
    --launch-only every form is launched three times and nothing is timed (for counter runs:
    the dispatches come in the order of DSLASH_VARIANTS)."""
    import torch
    import paper_2505_14399_amd as q

    if args.launch_only:  # calibration copies for the counter runs
        a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    lat = q.Lattice(DSLASH_HBM_DIMS, -0.2, 1.0, -1)
    V = lat.volume
    g = torch.Generator(device="cuda").manual_seed(9)
    U = random_su3_device(V, 0.6, g)
    Un = q.pack_gauge(lat, U, "f32")
    del U
    try:
        for nrhs, forms in DSLASH_VARIANTS.items():
            x = q.pack_spinor(lat, torch.randn(nrhs, V, 4, 3, dtype=torch.complex128, device="cuda", generator=g), "f32")
            y = torch.empty_like(x)
            ref = None
            for v in forms:
                q.set_dslash_variant(v)
                q.wilson_apply(lat, Un, x, layout="native", out=y)
                torch.cuda.synchronize()
                if ref is None:
                    ref = y.clone()
                err = float((y - ref).abs().max() / ref.abs().max())
                row = {"nrhs": nrhs, "form": v, "max_dev": err}
                if args.launch_only:
                    for _ in range(2):
                        q.wilson_apply(lat, Un, x, layout="native", out=y)
                    torch.cuda.synchronize()
                else:
                    for _ in range(3):
                        q.wilson_apply(lat, Un, x, layout="native", out=y)
                    q.timing_enable(True)
                    for _ in range(10):
                        q.wilson_apply(lat, Un, x, layout="native", out=y)
                    t = q.timing_query("dslash")
                    q.timing_enable(False)
                    ms = t["ms"] / t["launches"]
                    row.update(us=round(ms * 1e3, 1), algorithmic_MB=round(t["bytes"] / t["launches"] / 1e6, 1),
                               GBps=round(t["bytes"] / t["launches"] / (ms * 1e-3) / 1e9))
                print(json.dumps(row), flush=True)
            del x, y, ref
    finally:
        q.set_dslash_variant(0)


def variants_from(args):
    """FETCH_SIZE / WRITE_SIZE of the --dslash-variants --launch-only run, per (rhs count, form):
    the stencil dispatches in launch order, three per form, scaled by the copy calibration and
    set against the algorithmic bytes (spinor in and out per site and rhs, four links per site)."""
    import numpy as np

    def rows(d, counter):
        out = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        out.sort()
        copy = [v for _, n, v in out if "copyBuffer" in n][:3]  # the calibration copies come first
        scale = COPY_BYTES / (float(np.median(copy)) * 1024.0)
        st = [v * 1024.0 * scale for _, n, v in out if "k_dslash" in n]
        return st, scale

    fe, fs = rows(args.variants_from[0], "FETCH_SIZE")
    wr, ws = rows(args.variants_from[1], "WRITE_SIZE")
    V = 1
    for L in DSLASH_HBM_DIMS:
        V *= L
    print(f"# copy calibration: fetch x{fs:.3f}, write x{ws:.3f}")
    print("| rhs | form | fetch MB | write MB | algorithmic read MB | fetch / algorithmic read |")
    print("|---:|---:|---:|---:|---:|---:|")
    i = 0
    for nrhs, forms in DSLASH_VARIANTS.items():
        for v in forms:
            f = float(np.mean(fe[i + 1:i + 3]))
            w = float(np.mean(wr[i + 1:i + 3]))
            i += 3
            alg = V * (12.0 * nrhs + 36.0) * 8.0
            print(f"| {nrhs} | {v} | {f / 1e6:.0f} | {w / 1e6:.0f} | {alg / 1e6:.0f} | {f / alg:.2f} |")


def source_sha(fname):
    path = os.path.join(ROOT, "paper_2505_14399_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched32x64")
    ap.add_argument("--no-small", action="store_true",
                    help="leave out the 64 small lattices of the batched workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the setup / mixed / FP64 solve lines of the other lattices (16^3x32, 24^3x64)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparator solve")
    ap.add_argument("--mass", type=float, default=None, help="override the workload's quark mass")
    ap.add_argument("--inner", default=None, choices=("f64", "f32", "bf16", "f16"),
                    help="override the workload's K-cycle storage precision (--critical-table, --compare-setups)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="copy calibration plus one benchmark step (for the FETCH_SIZE / WRITE_SIZE counter runs)")
    ap.add_argument("--no-clover", action="store_true", help="skip the clover operator and clover MG leg")
    ap.add_argument("--no-evenodd", action="store_true", help="skip the even-odd preconditioning leg")
    ap.add_argument("--full-coarse", action="store_true",
                    help="coarse solve of the K-cycle on D_c (default: on its even-odd Schur complement)")
    ap.add_argument("--plain-smoother", action="store_true",
                    help="GMRES post-smoothing on D instead of the even-odd smoother in the main solve")
    ap.add_argument("--no-dslash-hbm", action="store_true",
                    help="skip the dslash bandwidth measurement on the 32^3x64 lattice")
    ap.add_argument("--levels", action="store_true",
                    help="two- vs three- vs four-level solve on the workload (further levels: 2^4 blocks of "
                         "the level above, 48 test vectors in batches of 8, rank 24)")
    ap.add_argument("--critical-table", action="store_true",
                    help="Regular / CSVD / iCSVD (n_s = 4, 8, 12, 16) on a --n-levels hierarchy of the workload "
                         "(near-critical comparison: --workload critical16x32_clover)")
    ap.add_argument("--n-levels", type=int, default=4, help="levels of the --critical-table hierarchies (2..4)")
    ap.add_argument("--max-streams", type=int, default=16,
                    help="--critical-table: leave out the iCSVD rows with more streams than this")
    ap.add_argument("--compare-setups", action="store_true",
                    help="Regular / CSVD / streaming (iCSVD) setups on the workload: iterations per level, "
                         "setup and solve seconds, leading singular values (prints a table and JSON lines)")
    ap.add_argument("--dslash-variants", action="store_true",
                    help="time the stencil's launch forms on 32^3x64 (FP32) at 1, 4 and 12 right-hand sides")
    ap.add_argument("--launch-only", action="store_true",
                    help="with --dslash-variants: launch each form three times, time nothing (counter runs)")
    ap.add_argument("--variants-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="counter output of --dslash-variants --launch-only: traffic per launch form")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="per-kernel and per-family device time inside the timed region from rocprofv3 "
                         "--kernel-trace --marker-trace CSV output (--steps: the run's timed steps)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="read rocprofv3 FETCH_SIZE / WRITE_SIZE counter output and write profiles/traffic.json")
    return ap.parse_args()


def load_workload(args):
    from fields import workloads
    if args.mass is not None:
        w = dict(workloads.WORKLOADS[args.workload], name=args.workload, mass=args.mass)
    else:
        w = dict(workloads.get(args.workload))
    if getattr(args, "inner", None):
        w["inner"] = args.inner
    return w


def traffic_probe(args):
    """Launch sequence measured by the counter runs (nothing is timed here): three 256 MiB device
    copies (calibration), then one step of the benchmark exactly as timed (setup and solve of
    the main lattice, and of the small lattices where the workload has them)."""
    import torch

    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    P = prepare(args)
    _, _, info, _ = P.step()
    torch.cuda.synchronize()
    print(json.dumps({"probe": P.w["name"], "dims": list(P.dims), "prec": P.w["inner"],
                      "worst_rel_res": max(i["true_rel_res"] for i in info)}), flush=True)


# dslash bandwidth on a lattice whose fields do not fit the 256 MB MALL (the workload's own
# 16^3 x 32 fields do): 32^3 x 64, FP32 storage, the default launch form, 1 and 12 right-hand
# sides.  Algorithmic bytes per site: (24 nrhs + 36) complex numbers of 8 bytes (spinor in and
# out per rhs, four links).
DSLASH_HBM_DIMS = (32, 32, 32, 64)


def random_su3_device(V, eps, g):
    """[4, V, 3, 3] complex128 SU(3) links on the device: exp(i eps H), H traceless hermitian with
    Gaussian entries (bandwidth legs only; the workloads' fields come from fields.random_gauge)."""
    import torch
    H = torch.randn(4, V, 3, 3, dtype=torch.complex128, device="cuda", generator=g)
    H = (H + H.conj().transpose(-1, -2)) / 2
    tr = torch.diagonal(H, dim1=-2, dim2=-1).sum(-1) / 3
    H = H - tr[..., None, None] * torch.eye(3, dtype=H.dtype, device=H.device)
    return torch.linalg.matrix_exp(1j * eps * H)


def dslash_hbm(clover=False):
    """Algorithmic bandwidth of the default launch form on 32^3 x 64 (FP32 storage): per site and
    right-hand side the spinor in and out, per site the four links (and with the clover term the
    two packed 6 x 6 hermitian blocks, 36 complex numbers)."""
    import numpy as np
    import torch

    import paper_2505_14399_amd as q

    lat = q.Lattice(DSLASH_HBM_DIMS, -0.2, 1.0, -1)
    V = lat.volume
    g = torch.Generator(device="cuda").manual_seed(7)
    # random SU(3) links exp(i eps H), H traceless hermitian (eps 0.6 as the workloads; 0.3 for
    # the clover leg, a near-unit field, so that the clover term is of natural size)
    U = random_su3_device(V, 0.3 if clover else 0.6, g)
    A = q.clover_field(lat, U, 1.0, 1.0, "f32") if clover else None
    Un = q.pack_gauge(lat, U, "f32")
    del U
    # target_frac: the stencil's bandwidth goal, 0.70 of the HBM peak at 1 and at 12 rhs
    out = {"lattice": list(DSLASH_HBM_DIMS), "prec": "f32", "launch": "default form", "target_frac": 0.70,
           "per_rhs": {}}

    def apply(x, y):
        if clover:
            q.clover_apply(lat, Un, A, x, layout="native", out=y)
        else:
            q.wilson_apply(lat, Un, x, layout="native", out=y)

    for nrhs in (1, 12):
        x = q.pack_spinor(lat, torch.randn(nrhs, V, 4, 3, dtype=torch.complex128, device="cuda", generator=g), "f32")
        y = torch.empty_like(x)
        for _ in range(3):
            apply(x, y)
        n, reps = (20 if nrhs == 1 else 6), []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for i in range(n):  # alternate the buffers so no application reads its own output
                apply(x if i % 2 == 0 else y, y if i % 2 == 0 else x)
            e1.record()
            torch.cuda.synchronize()
            reps.append(e0.elapsed_time(e1) / n * 1e-3)
        t = float(np.median(reps))
        byt = V * (24.0 * nrhs + 36.0 + (36.0 if clover else 0.0)) * 8.0
        out["per_rhs"][str(nrhs)] = {"us": t * 1e6, "algorithmic_MB": byt / 1e6, "GBps": byt / t / 1e9,
                                     "frac_hbm": byt / t / 1e9 / PEAK_HBM_GBPS}
        del x, y
    del Un, A
    torch.cuda.empty_cache()
    return out


def clover_mg(args):
    """The clover workload's setup and mixed-precision solve (one untimed warm-up setup + solve,
    then three timed setups, each followed by one timed solve)."""
    import numpy as np
    import torch

    import fields
    import paper_2505_14399_amd as q

    w = workloads_get(CLOVER_WORKLOAD)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(fields.gaussian_spinor(dims, 1, w["seed"], tag=w["tag"])).cuda()
    kw = dict(block=w["block"], n_test=w["n_test"], batch=w["batch"], rank=w["rank"], n_setup_iter=16,
              n_post_smooth=8, coarse_tol=0.03, coarse_max_iter=500, inner=w["inner"], seed=w["seed"], c_sw=w["c_sw"])
    eo = not args.plain_smoother
    # the coarse solve stays on the full D_c here: on this workload the Schur-complement coarse
    # solve took 23 outer iterations (0.027 s) against 9 (0.013 s)
    mg = q.mg_setup_stream_chiral_svd(lat, U, **kw)
    mg.set_smoother(eo=eo, sstep=True)
    q.mg_solve(mg, b, tol=args.tol)
    mg.close()
    torch.cuda.synchronize()
    setups, solves, info = [], [], None
    for _ in range(3):
        t0 = time.perf_counter()
        mg = q.mg_setup_stream_chiral_svd(lat, U, **kw)
        mg.set_smoother(eo=eo, sstep=True)
        t1 = time.perf_counter()
        _, inf = q.mg_solve(mg, b, tol=args.tol)
        t2 = time.perf_counter()
        mg.close()
        setups.append(t1 - t0)
        solves.append(t2 - t1)
        info = inf[0]
    if info["true_rel_res"] > args.tol:
        raise SystemExit(f"clover solve did not reach {args.tol}: {info}")
    return {"workload": w["name"], "c_sw": list(w["c_sw"]), "mass": w["mass"],
            "smoother": "even-odd GMRES(8), s-step form" if eo else "GMRES(8)",
            "coarse_solve": "full D_c",
            "setup_s": float(np.median(setups)), "solve_s": float(np.median(solves)), "outer_iters": info["outer_iters"],
            "coarse_iters": info["coarse_iters"], "true_rel_res": info["true_rel_res"]}


def evenodd_leg(args):
    """Even-odd preconditioning: the Schur operator Dhat = A_ee - D_eo A_oo^-1 D_oe on 32^3 x 64
    (FP32 storage, one right-hand side, Wilson and clover), timed per hop launch with the
    library's dispatch events, and FP64 GMRES(32) on the Schur complement against GMRES(32) on the
    full operator on the benchmark lattice, each operator at a mass about 0.3 above the left edge
    of its spectrum (Wilson -0.4, edge -0.694; clover 0.05, edge -0.255): unpreconditioned GMRES
    does not finish near the critical mass."""
    import numpy as np
    import torch

    import fields
    import paper_2505_14399_amd as q

    out = {"schur_apply": {}, "solve": {}}
    lat = q.Lattice(DSLASH_HBM_DIMS, -0.2, 1.0, -1)
    V = lat.volume
    g = torch.Generator(device="cuda").manual_seed(9)
    H = torch.randn(4, V, 3, 3, dtype=torch.complex128, device="cuda", generator=g)
    U = torch.linalg.matrix_exp(0.3j * (H + H.conj().transpose(-1, -2)) / 2)
    del H
    Ueo = q.eo_pack_gauge(lat, U, "f32")
    x = torch.randn(1, V, 4, 3, dtype=torch.complex128, device="cuda", generator=g)
    xe, _ = q.eo_pack_spinor(lat, x, "f32")
    del x
    for name, c in (("wilson", None), ("clover", 1.0)):
        A, Ai = q.eo_site_term(lat, U, c, c, "f32") if c else (None, None)
        y = torch.empty_like(xe)
        for _ in range(3):
            q.schur_apply(lat, Ueo, xe, A, Ai, out=y)
        q.timing_enable(True)
        for _ in range(10):
            q.schur_apply(lat, Ueo, xe, A, Ai, out=y)
        t = q.timing_query("evenodd")
        q.timing_enable(False)
        ms = t["ms"] / max(1, t["launches"])
        gbps = t["bytes"] / max(1, t["launches"]) / (ms * 1e-3) / 1e9
        out["schur_apply"][name] = {"lattice": list(DSLASH_HBM_DIMS), "prec": "f32", "hop_launch_us": ms * 1e3,
                                    "apply_us": 2 * ms * 1e3, "GBps": gbps, "frac_hbm": gbps / PEAK_HBM_GBPS}
        del A, Ai, y
    del U, Ueo, xe
    torch.cuda.empty_cache()
    w = workloads_get(args.workload)
    dims = w["dims"]
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(fields.gaussian_spinor(dims, 1, w["seed"], tag=w["tag"])).cuda()
    for name, c, m in (("wilson", None, -0.4), ("clover", 1.0, 0.05)):
        lat = q.Lattice(dims, m, w["xi"], w["bc_t"])
        res = {}
        for form, eo in (("schur", True), ("full", False)):
            q.eo_solve(lat, U, b, c_sw=c, tol=args.tol, eo=eo, max_iter=6000, check=False)  # warm-up
            ts, info = [], None
            for _ in range(3):
                _, info = q.eo_solve(lat, U, b, c_sw=c, tol=args.tol, eo=eo, max_iter=6000, check=False)
                ts.append(info["seconds"])
            res[form] = {"s": float(np.median(ts)), "gmres_iters": info["outer_iters"],
                         "true_rel_res": info["true_rel_res"], "status": info["status"]}
        out["solve"][name] = dict(res, mass=m, lattice=list(dims))
    return out


def workloads_get(name):
    from fields import workloads
    return workloads.get(name)


# setup methods compared by --compare-setups: (name, n_test m, batch r); rank k from the workload.
# Regular = one batch of k test vectors (its span is that of the block-orthonormalised vectors of
# the regular setup); CSVD = one batch of m vectors truncated to k; iCSVD = m vectors streamed in
# m / r batches of r.  Test vector i is the same in every method (the counter of its random
# initial guess is its global index), so the methods differ only in how the basis is formed.
SETUP_METHODS = (("Regular", 24, 24), ("CSVD", 48, 48), ("iCSVD", 48, 24), ("iCSVD", 48, 16), ("iCSVD", 48, 12),
                 ("iCSVD", 48, 8), ("iCSVD", 48, 6), ("iCSVD", 48, 4), ("iCSVD", 96, 24), ("iCSVD", 96, 16),
                 ("iCSVD", 96, 8))


def compare_setups(args):
    """Setup methods on the workload's lattice: per method one untimed setup + solve (warm-up), then
    a timed setup and the median of three solves.  Levels: l = 0 the outer (fine) iterations, l = 1
    the coarse GMRES iterations summed over the solve; 'normalised' is l = 1 per l = 0 iteration."""
    import numpy as np
    import torch

    import fields
    import paper_2505_14399_amd as q

    w = load_workload(args)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(fields.gaussian_spinor(dims, 1, w["seed"], tag=w["tag"])).cuda()
    k = w["rank"]
    rows = []
    for name, m, r in SETUP_METHODS:
        kw = dict(block=w["block"], n_test=m, batch=r, rank=k, n_setup_iter=16, n_post_smooth=8, coarse_tol=0.03,
                  coarse_max_iter=500, inner=w["inner"], seed=w["seed"])
        mg = q.mg_setup_stream_chiral_svd(lat, U, **kw)
        q.mg_solve(mg, b, tol=args.tol)
        mg.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mg = q.mg_setup_stream_chiral_svd(lat, U, **kw)
        t_setup = time.perf_counter() - t0
        ts, info = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            _, info = q.mg_solve(mg, b, tol=args.tol)
            ts.append(time.perf_counter() - t0)
        _, sig = mg.prolongator()
        mg.close()
        i0 = info[0]
        if i0["true_rel_res"] > args.tol:
            raise SystemExit(f"{name} m={m} r={r}: solve did not reach {args.tol}: {i0}")
        row = {"method": name, "m": m, "r": r, "n_s": m // r, "k": k, "setup_s": t_setup,
               "solve_s": float(np.median(ts)), "iters_l0": i0["outer_iters"], "iters_l1": i0["coarse_iters"],
               "normalised_l1": i0["coarse_iters"] / max(1, i0["outer_iters"]),
               "sigma_agg0": [[float(v) for v in sig[0, a]] for a in (0, 1)]}
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(f"\n# setup methods on {w['name']} {dims}, k = {k}, n_setup = 16, inner {w['inner']}, tol {args.tol}")
    print("| method | m | r | n_s | iterations l=0 | iterations l=1 | l=1 per l=0 | setup s | solve s |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|")
    for x in rows:
        print(f"| {x['method']} | {x['m']} | {x['r']} | {x['n_s']} | {x['iters_l0']} | {x['iters_l1']} | "
              f"{x['normalised_l1']:.2f} | {x['setup_s']:.3f} | {x['solve_s']:.3f} |")
    print("\nLeading singular values of aggregate 0 (chirality 0), sigma_1 .. sigma_k:")
    for x in rows:
        sv = x["sigma_agg0"][0]
        print(f"{x['method']:8s} m={x['m']:3d} r={x['r']:2d}: " + " ".join(f"{v:.3g}" for v in sv))


# setup methods of the near-critical comparison: (name, test vectors per level, vectors per
# stream); Regular keeps k = 24 vectors, CSVD truncates one batch of 48 (the largest batch the
# streaming SVD takes), iCSVD streams n_s batches of 24 (n_s = 4, 8, 12, 16), the same at every
# level
# relative tolerances of the solves on levels 2 and 3 in the near-critical comparison (level 1:
# the hierarchy's coarse_tol, 0.03), the loosened criteria the comparison needs there
LEVEL_TOLS = {2: 0.06, 3: 0.6}
CRITICAL_METHODS = (("Regular", 24, 24), ("CSVD", 48, 48), ("iCSVD n_s=4", 96, 24), ("iCSVD n_s=8", 192, 24),
                    ("iCSVD n_s=12", 288, 24), ("iCSVD n_s=16", 384, 24))


def critical_table(args):
    """Setup methods on a four-level hierarchy (levels 2 and 3 on 2^4 blocks of the level above,
    rank 24 everywhere, each level built by the method under test): per method one untimed
    setup + solve, then a timed setup and the median of three solves; iterations per level
    (l = 0 outer flexible GMRES, l = 1..3 the Krylov iterations on the coarse levels, summed over
    the solve) and per iteration of the level above."""
    import numpy as np
    import torch

    import fields
    import paper_2505_14399_amd as q

    w = load_workload(args)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(fields.gaussian_spinor(dims, 1, w["seed"], tag=w["tag"])).cuda()
    k = w["rank"]
    rows = []

    def build(m, r):
        mg = q.mg_setup_stream_chiral_svd(lat, U, block=w["block"], n_test=m, batch=r, rank=k, n_setup_iter=16,
                                          n_post_smooth=8, coarse_tol=0.03, coarse_max_iter=500, inner=w["inner"],
                                          seed=w["seed"], c_sw=w.get("c_sw"))
        for lv in range(2, args.n_levels):
            ext = mg.levels[lv - 1]["dims"] if lv > 2 else tuple(e // bb for e, bb in zip(dims, w["block"]))
            blk = tuple(2 if e % 2 == 0 else 3 if e % 3 == 0 else 1 for e in ext)
            mg.add_level(block=blk, n_test=m, batch=r, rank=k, n_setup_iter=16)
            mg.set_level_tol(lv, LEVEL_TOLS[lv])
        return mg

    for name, m, r in CRITICAL_METHODS:
        if m // r > args.max_streams:
            continue
        progress(f"critical table: {name} (n_test {m}, batch {r})")
        mg = build(m, r)
        q.mg_solve(mg, b, tol=args.tol)
        mg.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mg = build(m, r)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        ts, info = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            _, info = q.mg_solve(mg, b, tol=args.tol)
            ts.append(time.perf_counter() - t0)
            progress(f"  solve {len(ts)}/3: {ts[-1]:.3f} s")
        dims_l = {lv: list(mg.levels[lv]["dims"]) for lv in mg.levels}
        mg.close()
        i0 = info[0]
        if i0["true_rel_res"] > args.tol:
            raise SystemExit(f"{name}: solve did not reach {args.tol}: {i0}")
        it = [i0["outer_iters"], i0["coarse_iters"], i0["coarse2_iters"], i0["coarse3_iters"]][:args.n_levels]
        row = {"method": name, "m": m, "r": r, "n_s": m // r, "k": k, "levels": args.n_levels, "level_dims": dims_l,
               "setup_s": t_setup, "solve_s": float(np.median(ts)), "iters": it,
               "per_level_above": [it[i] / max(1, it[i - 1]) for i in range(1, len(it))],
               "true_rel_res": i0["true_rel_res"]}
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(f"\n# {w['name']} {dims}, mass {w['mass']:.8f}, c_sw {w.get('c_sw')}, k = {k}, {args.n_levels} levels, "
          f"inner {w['inner']}, tol {args.tol}, level tolerances 0.03 (l = 1), "
          + ", ".join(f"{LEVEL_TOLS[lv]} (l = {lv})" for lv in range(2, args.n_levels)))
    print("| level | " + " | ".join(x["method"] for x in rows) + " |")
    print("|---|" + "---:|" * len(rows))
    for lv in range(args.n_levels):
        print(f"| l = {lv} | " + " | ".join(str(x["iters"][lv]) for x in rows) + " |")
    print("\nPer iteration of the level above:\n")
    print("| level | " + " | ".join(x["method"] for x in rows) + " |")
    print("|---|" + "---:|" * len(rows))
    for lv in range(1, args.n_levels):
        print(f"| l = {lv} | " + " | ".join(f"{x['per_level_above'][lv - 1]:.2f}" for x in rows) + " |")
    print("\n| | " + " | ".join(x["method"] for x in rows) + " |")
    print("|---|" + "---:|" * len(rows))
    print("| setup s | " + " | ".join(f"{x['setup_s']:.3f}" for x in rows) + " |")
    print("| solve s | " + " | ".join(f"{x['solve_s']:.3f}" for x in rows) + " |")


LEVEL2 = dict(block=(2, 2, 2, 2), n_test=48, batch=8, rank=24, n_setup_iter=16)
LEVEL3 = dict(block=None, n_test=48, batch=8, rank=24, n_setup_iter=16)  # block from the extents of level 2


def isvd_rate(fam):
    if not fam["launches"]:
        return None
    ms = fam["ms"] / fam["launches"]
    tf = fam["flops"] / fam["launches"] / (ms * 1e-3) / 1e12
    return {"timed_streams": fam["launches"], "avg_stream_ms": ms, "TFLOPs_fp64": tf, "frac_fp64": tf / PEAK_FP64_TFLOPS}


def compare_levels(args):
    """The workload's two-level hierarchy, then the same hierarchy with a third and with a third
    and fourth level: setup seconds of the extra levels, median of three solves, iterations per
    level (l = 0 outer, l = 1 on D_c, l = 2 and l = 3 on the further levels)."""
    import numpy as np
    import torch

    import fields
    import paper_2505_14399_amd as q

    w = load_workload(args)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(fields.gaussian_spinor(dims, 1, w["seed"], tag=w["tag"])).cuda()
    kw = dict(block=w["block"], n_test=w["n_test"], batch=w["batch"], rank=w["rank"], n_setup_iter=16,
              inner=w["inner"], seed=w["seed"])
    rows = []
    for levels in (2, 3, 3, 4):  # the first three-level pass is a warm-up of its kernels
        mg = q.mg_setup_stream_chiral_svd(lat, U, **kw)
        t_level = 0.0
        if levels >= 3:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mg.add_level(**LEVEL2)
            if levels == 4:  # block 2 along extents of level 2 that are even, 3 along multiples of 3, else 1
                ext = mg.levels[2]["dims"]
                blk = tuple(2 if e % 2 == 0 else 3 if e % 3 == 0 else 1 for e in ext)
                mg.add_level(**dict(LEVEL3, block=blk))
            torch.cuda.synchronize()
            t_level = time.perf_counter() - t0
        ts, info = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            _, info = q.mg_solve(mg, b, tol=args.tol)
            ts.append(time.perf_counter() - t0)
        dims_l = {lv: list(mg.levels[lv]["dims"]) for lv in mg.levels}
        mg.close()
        i0 = info[0]
        rows.append({"levels": levels, "workload": w["name"], "level_dims": dims_l, "level_setup_s": t_level,
                     "solve_s": float(np.median(ts)), "iters_l0": i0["outer_iters"], "iters_l1": i0["coarse_iters"],
                     "iters_l2": i0["coarse2_iters"], "iters_l3": i0["coarse3_iters"],
                     "smoother_l1": i0["smoother1_iters"], "smoother_l2": i0["smoother2_iters"],
                     "true_rel_res": i0["true_rel_res"]})
    rows = [rows[0], rows[2], rows[3]]
    for x in rows:
        print(json.dumps(x), flush=True)
    print(f"\n# {w['name']} {dims}, inner {w['inner']}, tol {args.tol}; level 2 {LEVEL2}; level 3 {LEVEL3}")
    print("| levels | iterations l=0 | l=1 | l=2 | l=3 | l=1 per l=0 | l=2 per l=1 | l=3 per l=2 | extra setup s | "
          "solve s |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
    for x in rows:
        lv = x["levels"]
        c = lambda a, b: f"{a / max(1, b):.2f}"
        print(f"| {lv} | {x['iters_l0']} | {x['iters_l1']} | {x['iters_l2'] if lv >= 3 else '-'} | "
              f"{x['iters_l3'] if lv >= 4 else '-'} | {c(x['iters_l1'], x['iters_l0'])} | "
              f"{c(x['iters_l2'], x['iters_l1']) if lv >= 3 else '-'} | {c(x['iters_l3'], x['iters_l2']) if lv >= 4 else '-'} | "
              f"{x['level_setup_s']:.3f} | {x['solve_s']:.3f} |")


def read_counter(d, counter):
    """{kernel name: [per-dispatch counter values]} from a rocprofv3 --pmc output folder."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic_from(args):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by the copy calibration; write the record."""
    import numpy as np
    w = load_workload(args)
    fetch = read_counter(args.traffic_from[0], "FETCH_SIZE")
    write = read_counter(args.traffic_from[1], "WRITE_SIZE")

    def pick(tab, prefix, merge=False):
        found, allv = None, []
        for name, vals in tab.items():
            short = name.replace("qmg::(anonymous namespace)::", "").split("void ")[-1]
            if short.startswith(prefix):
                if not merge:
                    return name, vals
                found = found or name
                allv += list(vals)
        return found, allv

    # the calibration copy: the runtime's device-to-device copy kernel at its largest dispatches
    # (the three 256 MiB copies; the runtime's other copies are a few KiB)
    def calib(tab):
        vals = [v for n, vs in tab.items() if "copyBuffer" in n for v in vs]
        if not vals:
            raise SystemExit("no device copy dispatches in the counter output")
        top = max(vals)
        return float(np.median([v for v in vals if v >= 0.99 * top])) * 1024.0

    copy_name = "__amd_rocclr_copyBuffer"
    f_copy, w_copy = calib(fetch), calib(write)
    f_scale, w_scale = COPY_BYTES / f_copy, COPY_BYTES / w_copy
    rec = json.load(open(TRAFFIC_JSON)) if os.path.exists(TRAFFIC_JSON) else {}
    lines = [f"# HBM-side traffic per launch, workload {w['name']} {w['dims']} inner {w['inner']}",
             f"# copy calibration ({copy_name}): FETCH_SIZE {f_copy / 1024:.0f} KiB and WRITE_SIZE "
             f"{w_copy / 1024:.0f} KiB for a {COPY_BYTES >> 20} MiB copy -> scale fetch x{f_scale:.3f}, "
             f"write x{w_scale:.3f}"]
    entry = rec.setdefault(w["name"], {})
    for fam in FAMILY_KERNEL:
        prefix, src = FAMILY_KERNEL[fam]
        name, fv = pick(fetch, prefix, True)
        _, wv = pick(write, prefix, True)
        if not fv or not wv:
            continue
        # every instance of the family's kernel in the step (forms, precisions, right-hand-side
        # counts) mixes as in the timed region: the mean over the step's dispatches is the
        # family's launch, as bench.py's timed averages are
        fb = float(np.mean(fv)) * 1024.0 * f_scale
        wb = float(np.mean(wv)) * 1024.0 * w_scale
        entry[fam] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                      "dispatches": [len(fv), len(wv)], "kernel": name, "source": src,
                      "source_sha256": source_sha(src)}
        lines.append(f"{fam:14s} {name[:70]}: fetch {fb / 1e6:.2f} MB + write {wb / 1e6:.2f} MB = "
                     f"{(fb + wb) / 1e6:.2f} MB per launch (mean of {len(fv)}/{len(wv)} dispatches)")
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    json.dump(rec, open(TRAFFIC_JSON, "w"), indent=1)
    print("\n".join(lines))


def recorded_traffic(wname, fam):
    """Bytes per launch from the committed counter record, None if absent or the source changed."""
    if fam not in FAMILY_KERNEL or not os.path.exists(TRAFFIC_JSON):
        return None
    e = json.load(open(TRAFFIC_JSON)).get(wname, {}).get(fam)
    if not e or e.get("source_sha256") != source_sha(FAMILY_KERNEL[fam][1]):
        return None
    return e["bytes_per_launch"]


def _host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(w, counts, U=None, small=None):
    """The CPU oracle on this host, on a bounded sample of the workload (its unit operations at
    the workload's shapes, each timed directly), composed into an estimate of the oracle's time
    for the GPU solve's own operation counts (the oracle is never run on the whole solve here)."""
    import numpy as np
    import fields
    from oracle import wilson, clover, transfer, coarse, icsvd, geometry as geo  # noqa: F401
    from threadpoolctl import threadpool_info

    dims, block, k, r = w["dims"], w["block"], w["rank"], w["batch"]
    V = geo.volume(dims)
    cd = geo.coarse_dims(dims, block)
    d = geo.volume(cd)
    nd = int(np.prod(block))
    N = 6 * nd
    rng = np.random.default_rng(0)
    if U is None:
        U = fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])
    psi = fields.gaussian_spinor(dims, 1, w["seed"])[0]
    m = 2 * k
    # the coarse operator's values do not change the oracle's work: one random block broadcast
    Y = np.broadcast_to(rng.standard_normal((1, 9, m, m)) + 1j * rng.standard_normal((1, 9, m, m)), (d, 9, m, m))
    vc = rng.standard_normal((1, d, 2, k)) + 1j * rng.standard_normal((1, d, 2, k))
    # restrict + prolong and the streaming SVD on a slice of the aggregates (both are independent
    # per aggregate), scaled to all of them
    ds = min(d, 512)
    Ps, _ = np.linalg.qr(rng.standard_normal((ds, 2, N, k)) + 1j * rng.standard_normal((ds, 2, N, k)))
    sdims = (block[0], block[1], block[2], block[3] * ds)  # ds aggregates stacked along t
    psis = fields.gaussian_spinor(sdims, 1, 3)[0]
    nprob = min(2 * d, 256)
    Phi = [rng.standard_normal((N, k)) + 1j * rng.standard_normal((N, k)) for _ in range(nprob)]
    Psi = [rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r)) for _ in range(nprob)]

    def tm(f, n):
        t0 = time.perf_counter()
        for _ in range(n):
            f()
        return (time.perf_counter() - t0) / n

    if w.get("c_sw"):  # the clover term is setup work, built once outside the timed calls
        T = clover.clover_term(U, dims, *w["c_sw"])
        apply_D = lambda: clover.apply_clover(U, T, psi, w["mass"], w["xi"], w["bc_t"], dims)  # noqa: E731
    else:
        apply_D = lambda: wilson.apply_wilson(U, psi, w["mass"], w["xi"], w["bc_t"], dims)  # noqa: E731
    t_D = tm(apply_D, 1 if V > 1 << 20 else 3)
    t_Dc = tm(lambda: coarse.coarse_apply(Y, vc, cd), 1 if d > 4096 else 3)
    t_RP = tm(lambda: transfer.prolong(Ps, transfer.restrict(Ps, psis[None], sdims, block), sdims, block), 1) * d / ds
    t_svd = tm(lambda: [icsvd.icsvd_update(Phi[i], Psi[i], k) for i in range(nprob)], 1) * (2 * d) / nprob
    a, b = psi.ravel(), psi.ravel().copy()
    t_vec = tm(lambda: (np.vdot(a, b), b + 0.5 * a), 3)
    est = (counts["dslash"] * t_D + counts["coarse_apply"] * t_Dc + counts["restrict"] * t_RP
           + counts["vector_ops"] * t_vec)
    small_txt = ""
    if small:  # the small lattices: the oracle's D apply per size times the fine applies of their solve
        from collections import Counter
        sizes = Counter(d[0] for d, _, _ in small["spec"])
        t_L = {}
        for L in sizes:
            dL = (L,) * 4
            UL = fields.random_gauge(dL, 0.3, 1)
            pL = fields.gaussian_spinor(dL, 1, 1)[0]
            t_L[L] = tm(lambda: wilson.apply_wilson(UL, pL, 0.05, 1.0, -1, dL), 2)
        applies = small["outer"] * (1 + 8) + small["refinements"] + 1
        est_small = applies * sum(n * t_L[L] for L, n in sizes.items())
        est += est_small
        small_txt = (f"; plus the {len(small['spec'])} small lattices: oracle D apply per size "
                     f"{ {L: round(t, 4) for L, t in t_L.items()} } s x {applies} fine applies each (their batched "
                     f"solve's outer iterations x 9 + refinements; coarse work not counted) = {est_small:.1f}s")
    blas = [f"{p.get('internal_api')}:{p.get('num_threads')}" for p in threadpool_info()]
    ncpu = _host_cores()
    ns = w["n_test"] // w["batch"]
    setup_est = ns * (w["batch"] * (16 + 1) * t_D + t_svd)
    return {
        "value": est, "unit": "s", "cores": ncpu, "kind": "oracle",
        "sample": (f"oracle unit operations on this workload's shapes ({dims}, k={k}), each timed directly: fine D "
                   f"apply {t_D:.3f}s{' (with the clover term)' if w.get('c_sw') else ''} (one rhs), coarse apply "
                   f"{t_Dc:.4f}s ({d} aggregates), restrict+prolong {t_RP:.3f}s (timed on {ds} aggregates, scaled), "
                   f"one streaming-SVD stream {t_svd:.3f}s (LAPACK per problem, timed on {nprob} of {2 * d} problems, "
                   f"scaled), fine vector op {t_vec:.4f}s; value = these times x the GPU solve's operation counts "
                   f"{counts} (coarse Schur launches counted as the fraction of a coarse apply they stream); oracle "
                   f"setup estimate {setup_est:.1f}s (smoothing applies + {ns} streams); BLAS/LAPACK pools "
                   f"{blas} over {ncpu} affinity cores, stencil and vector arithmetic single-threaded (NumPy)"
                   f"{small_txt}"),
    }


def family_table(families, steps):
    """Per family: timed launches, calls, average launch ms, device ms per step, algorithmic
    bytes and flops per launch."""
    import paper_2505_14399_amd as q
    out = {}
    for f in families:
        t = q.timing_query(f)
        if not t["launches"]:
            continue
        avg = t["ms"] / t["launches"]
        out[f] = {"launches_timed": t["launches"], "calls": t["calls"], "avg_launch_ms": avg,
                  "ms_per_step": avg * t["calls"] / steps, "bytes_per_launch": t["bytes"] / t["launches"],
                  "flops_per_launch": t["flops"] / t["launches"]}
    return out


def roofline_of(fam_name, f, wname):
    """Roofline object of one family: FP64 flops for the streaming-SVD kernels, else algorithmic
    bytes over HBM."""
    avg_s = f["avg_launch_ms"] * 1e-3
    if fam_name == "isvd/small" or (f["bytes_per_launch"] == 0 and f["flops_per_launch"] > 0):
        ach = f["flops_per_launch"] / avg_s / 1e12
        return {"bound": "alu", "achieved": ach,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "traffic": None,
                "kernel": fam_name, "avg_launch_ms": f["avg_launch_ms"],
                "algorithmic_flops_per_launch": f["flops_per_launch"]}
    ach = f["bytes_per_launch"] / avg_s / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBPS,
            "traffic": recorded_traffic(wname, fam_name), "kernel": fam_name, "avg_launch_ms": f["avg_launch_ms"],
            "algorithmic_bytes_per_launch": f["bytes_per_launch"]}


def make_solver(args, q, w=None):
    eo_smoother = not args.plain_smoother

    def coarse_eo(mg):
        """The Schur-complement coarse solve unless --full-coarse, the workload's own choice
        (coarse_solve = "full"), or where it does not apply (an odd coarse extent, further levels):
        returns whether it is on."""
        if args.full_coarse or (w is not None and w.get("coarse_solve") == "full"):
            return False
        try:
            mg.set_coarse_eo(True)
            return True
        except q.QmgError:
            return False
    return eo_smoother, coarse_eo


def measure_config(args, name, steps=2):
    """Setup and mixed-precision solve of another workload (one warm-up step, then `steps` timed
    steps) and the FP64 path on the same lattice: medians and iteration counts."""
    import numpy as np
    import torch
    import fields
    from fields import workloads
    import paper_2505_14399_amd as q

    w = workloads.get(name)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U = torch.from_numpy(fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])).cuda()
    b = torch.from_numpy(workloads.rhs(w)).cuda()
    eo_smoother, coarse_eo = make_solver(args, q, w)
    kw = dict(block=w["block"], n_test=w["n_test"], batch=w["batch"], rank=w["rank"], n_setup_iter=16,
              n_post_smooth=8, coarse_tol=0.03, coarse_max_iter=500, seed=w["seed"], c_sw=w.get("c_sw"))
    res = {"workload": name, "lattice": list(dims), "mass": w["mass"], "inner": w["inner"], "nrhs": int(b.shape[0])}
    for inner in (w["inner"], "f64"):
        setups, solves, info = [], [], None
        for it in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mg = q.mg_setup_stream_chiral_svd(lat, U, inner=inner, **kw)
            mg.set_smoother(eo=eo_smoother, sstep=True)
            coarse_eo(mg)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = q.mg_solve(mg, b, tol=args.tol)
            t2 = time.perf_counter()
            mg.close()
            if it:
                setups.append(t1 - t0)
                solves.append(t2 - t1)
        worst = max(i["true_rel_res"] for i in info)
        if worst > args.tol:
            raise SystemExit(f"{name} ({inner}) did not reach {args.tol}: {info}")
        key = "mixed" if inner != "f64" else "fp64"
        res[key] = {"setup_s": float(np.median(setups)), "solve_s": float(np.median(solves)),
                    "outer_iters": info[0]["outer_iters"], "coarse_iters": info[0]["coarse_iters"],
                    "true_rel_res": worst}
    del U
    torch.cuda.empty_cache()
    return res


def prepare(args):
    """The workload's fields and right-hand sides on the device, and one step of the benchmark:
    setup and mixed-precision solve of the main lattice, then (batched workload) the setups and
    solves of the 64 small lattices in shared launches."""
    import torch

    import fields
    from fields import workloads
    import paper_2505_14399_amd as q

    w = load_workload(args)
    dims = w["dims"]
    lat = q.Lattice(dims, w["mass"], w["xi"], w["bc_t"])
    U_host = fields.random_gauge(dims, w["eps"], w["seed"], w["tag"])
    U = torch.from_numpy(U_host).cuda()
    b = torch.from_numpy(workloads.rhs(w)).cuda()
    nrhs = int(b.shape[0])
    setup_kw = dict(block=w["block"], n_test=w["n_test"], batch=w["batch"], rank=w["rank"], n_setup_iter=16,
                    n_post_smooth=8, coarse_tol=0.03, coarse_max_iter=500, inner=w["inner"], seed=w["seed"],
                    c_sw=w.get("c_sw"))
    eo_smoother, coarse_eo = make_solver(args, q, w)
    # the 64 independent small lattices of the batched workload: one hierarchy object whose
    # setups and solves run in shared launches over all of them
    small = None
    if w.get("small_lattices") and not args.no_small:
        sw = workloads.SMALL_LATTICES
        spec = workloads.small_lattices()
        small = {"spec": spec, "lats": [q.Lattice(d, m, sw["xi"], sw["bc_t"]) for d, m, _ in spec],
                 "U_host": [fields.random_gauge(d, sw["eps"], sw["seed"], t) for d, _, t in spec],
                 "b": [torch.from_numpy(fields.gaussian_spinor(d, 1, sw["seed"], tag=500 + i)).cuda()
                       for i, (d, _, _) in enumerate(spec)],
                 "kw": dict(block=sw["block"], n_test=sw["n_test"], batch=sw["batch"], rank=sw["rank"],
                            n_setup_iter=16, seed=sw["seed"], inner=sw["inner"])}
        small["U"] = [torch.from_numpy(u).cuda() for u in small["U_host"]]

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mg = q.mg_setup_stream_chiral_svd(lat, U, **setup_kw)
        mg.set_smoother(eo=eo_smoother, sstep=True)  # builds the half-lattice fields: part of the setup
        coarse_eo(mg)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = q.mg_solve(mg, b, tol=args.tol)
        t2 = time.perf_counter()
        mg.close()
        part = {"setup_s": t1 - t0, "solve_s": t2 - t1}
        if small:
            t3 = time.perf_counter()
            bt = q.batch_setup(small["lats"], small["U"], **small["kw"])
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            _, sinf = q.batch_solve(bt, small["b"], tol=args.tol)
            t5 = time.perf_counter()
            bt.close()
            part.update(small_setup_s=t4 - t3, small_solve_s=t5 - t4,
                        small_info={"outer_iters": sinf[0][0]["outer_iters"], "refinements": sinf[0][0]["refinements"],
                                    "coarse_iters": sinf[0][0]["coarse_iters"],
                                    "true_rel_res": max(i[0]["true_rel_res"] for i in sinf)})
            info = info + [{"true_rel_res": part["small_info"]["true_rel_res"]}]
        return part["setup_s"] + part.get("small_setup_s", 0.0), part["solve_s"] + part.get("small_solve_s", 0.0), \
            info, part

    return SimpleNamespace(w=w, dims=dims, lat=lat, U_host=U_host, U=U, b=b, nrhs=nrhs, setup_kw=setup_kw,
                           eo_smoother=eo_smoother, coarse_eo=coarse_eo, small=small, step=step)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the solver path is not sharded "
              f"across GPUs", file=sys.stderr)
        sys.exit(2)
    if args.traffic_from:
        traffic_from(args)
        return
    if args.trace_summary:
        trace_summary(args)
        return
    if args.variants_from:
        variants_from(args)
        return
    if args.dslash_variants:
        dslash_variants(args)
        return
    if args.traffic_probe:
        traffic_probe(args)
        return
    if args.compare_setups:
        compare_setups(args)
        return
    if args.critical_table:
        critical_table(args)
        return
    if args.levels:
        compare_levels(args)
        return
    import numpy as np
    import torch

    import fields
    from fields import workloads
    import paper_2505_14399_amd as q

    P = prepare(args)
    w, dims, lat, U_host, U, b, nrhs = P.w, P.dims, P.lat, P.U_host, P.U, P.b, P.nrhs
    setup_kw, eo_smoother, coarse_eo, small, step = P.setup_kw, P.eo_smoother, P.coarse_eo, P.small, P.step
    for i in range(args.warmup):
        step()
        progress(f"warm-up step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    # about one launch in TIMING_SAMPLE of each kernel family is timed with events attached to the dispatch
    q.timing_enable(True, every=TIMING_SAMPLE)
    setups, solves, infos, parts = [], [], [], []
    torch.cuda.synchronize()
    roctx("bench/timed")
    T0 = time.perf_counter()
    for _ in range(args.steps):
        ts, tv, info, part = step()
        setups.append(ts)
        solves.append(tv)
        infos.append(info)
        parts.append(part)
        progress(f"timed step {len(parts)}/{args.steps} done: setup {ts:.3f} s, solve {tv:.3f} s")
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    roctx()
    fams = family_table(q.timing_families(), args.steps)
    q.timing_enable(False)
    for info in infos:
        for i in info:
            if i["true_rel_res"] > args.tol:
                raise SystemExit(f"solve did not reach {args.tol}: {i}")
    info = infos[-1][:nrhs]

    # operation counts of one mixed solve (for the CPU baseline), from an untimed solve
    mg = q.mg_setup_stream_chiral_svd(lat, U, **setup_kw)
    mg.set_smoother(eo=eo_smoother, sstep=True)
    ceo_on = coarse_eo(mg)
    q.timing_enable(True)
    _, sinfo = q.mg_solve(mg, b, tol=args.tol)
    op_name = "clover" if w.get("c_sw") else "dslash"
    cnt = {"dslash": q.timing_query(op_name)["calls"] * nrhs, "restrict": q.timing_query("restrict")["calls"],
           "coarse_apply": q.timing_query("coarse_apply")["calls"]}
    # an even-odd hop does the work of half a fine operator application per right-hand side, a
    # coarse Schur launch streams about (slots / 9) of half the coarse operator
    cnt["dslash"] += q.timing_query("evenodd")["calls"] * nrhs // 2
    ceo = q.timing_query("coarse_eo")
    cnt["coarse_apply"] += int(round(ceo["calls"] * 0.5 * 8.5 / 9))
    cnt["restrict"] *= nrhs
    cnt["coarse_apply"] *= nrhs
    cnt["vector_ops"] = 12 * sum(i["smoother_iters"] + i["outer_iters"] for i in sinfo)
    q.timing_enable(False)
    # the other smoother and the other coarse solve on the same hierarchy, for comparison
    mg.set_smoother(eo=not eo_smoother, sstep=True)
    q.mg_solve(mg, b, tol=args.tol)
    t0 = time.perf_counter()
    _, other = q.mg_solve(mg, b, tol=args.tol)
    other_solve = {"smoother": "plain" if eo_smoother else "even-odd", "s": time.perf_counter() - t0,
                   "outer_iters": [i["outer_iters"] for i in other], "coarse_iters": other[0]["coarse_iters"],
                   "true_rel_res": max(i["true_rel_res"] for i in other)}
    other_coarse = None
    mg.set_smoother(eo=eo_smoother, sstep=True)
    try:
        mg.set_coarse_eo(not ceo_on)
    except q.QmgError:
        pass
    else:
        q.mg_solve(mg, b, tol=args.tol)
        t0 = time.perf_counter()
        _, oc = q.mg_solve(mg, b, tol=args.tol)
        other_coarse = {"coarse_solve": "full D_c" if ceo_on else "even-odd Schur complement",
                        "s": time.perf_counter() - t0, "outer_iters": [i["outer_iters"] for i in oc],
                        "coarse_iters": oc[0]["coarse_iters"], "true_rel_res": max(i["true_rel_res"] for i in oc)}
    mg.close()

    # FP64 path on the same lattices (own FP64 setup, the same smoother and coarse solve; untimed)
    fp64_solve = None
    if not args.no_fp64 and w["inner"] != "f64" and small:
        bt = q.batch_setup(small["lats"], small["U"], **dict(small["kw"], inner="f64"))
        q.batch_solve(bt, small["b"], tol=args.tol)
        t0 = time.perf_counter()
        _, s64 = q.batch_solve(bt, small["b"], tol=args.tol)
        small_fp64 = {"s": time.perf_counter() - t0, "outer_iters": s64[0][0]["outer_iters"],
                      "true_rel_res": max(i[0]["true_rel_res"] for i in s64)}
        bt.close()
    if not args.no_fp64 and w["inner"] != "f64":
        mg64 = q.mg_setup_stream_chiral_svd(lat, U, **dict(setup_kw, inner="f64"))
        mg64.set_smoother(eo=eo_smoother, sstep=True)
        coarse_eo(mg64)
        q.mg_solve(mg64, b, tol=args.tol)  # warm-up of the FP64 kernels
        ts64 = []
        for _ in range(2):
            t0 = time.perf_counter()
            _, i64 = q.mg_solve(mg64, b, tol=args.tol)
            ts64.append(time.perf_counter() - t0)
        mg64.close()
        fp64_solve = {"s": float(np.median(ts64)), "outer_iters": [i["outer_iters"] for i in i64],
                      "coarse_iters": i64[0]["coarse_iters"], "true_rel_res": max(i["true_rel_res"] for i in i64)}
        if small:
            fp64_solve = {"s": fp64_solve["s"] + small_fp64["s"], "lattice32x64": fp64_solve,
                          "small_lattices": small_fp64}
    del U
    torch.cuda.empty_cache()

    # the dominant kernel family: the largest device time per step
    dom = max(fams, key=lambda f: fams[f]["ms_per_step"])
    roof = roofline_of(dom, fams[dom], w["name"])
    top = sorted(fams, key=lambda f: -fams[f]["ms_per_step"])[:12]
    op = [f for f in fams if f.startswith(op_name + "/")]
    op_ms = sum(fams[f]["avg_launch_ms"] * fams[f]["launches_timed"] for f in op)
    op_bytes = sum(fams[f]["bytes_per_launch"] * fams[f]["launches_timed"] for f in op)
    op_n = sum(fams[f]["launches_timed"] for f in op)
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
        "dtype": "f32 inner, f64 outer" if w["inner"] == "f32" else f"{w['inner']} inner, f64 outer",
        "data": "synthetic",
        "config": {"workload": w["name"], "lattice": list(dims), "xi": w["xi"], "eps": w["eps"],
                   "mass": w["mass"], "bc_t": w["bc_t"], "block": list(w["block"]), "n_test": w["n_test"],
                   "batch": w["batch"], "rank": w["rank"], "nrhs": nrhs,
                   "rhs": "12 spin-colour point sources" if w.get("rhs") == "point12" else "1 complex Gaussian",
                   "tol": args.tol,
                   "smoother": "even-odd GMRES(8), s-step form" if eo_smoother else "GMRES(8)",
                   "coarse_solve": "GMRES(32) on the even-odd Schur complement of D_c" if ceo_on
                   else "GMRES(32) on D_c",
                   **({"small_lattices": "64 lattices L^4, L in {8, 10, 12}, masses uniform in [0.01, 0.1], eps 0.3, "
                                         "2^4 blocks, 16 / 4 / 8, FP32 inner, one Gaussian rhs each, all in one "
                                         "batched hierarchy"} if small else {}),
                   **({"c_sw": list(w["c_sw"])} if w.get("c_sw") else {})},
        "setup_s": float(np.median(setups)),
        "parts": {"lattice32x64" if small else w["name"]: {
                      "setup_s": float(np.median([p["setup_s"] for p in parts])),
                      "solve_s": float(np.median([p["solve_s"] for p in parts]))},
                  **({"small_lattices": {
                      "lattices": len(small["spec"]), "sites": int(sum(d[0] ** 4 for d, _, _ in small["spec"])),
                      "extents": "L^4, L in {8, 10, 12}", "mass_range": [0.01, 0.1],
                      "setup_s": float(np.median([p["small_setup_s"] for p in parts])),
                      "solve_s": float(np.median([p["small_solve_s"] for p in parts])),
                      **parts[-1]["small_info"]}} if small else {})},
        "solve_fp64": fp64_solve,
        "solve_other_smoother": other_solve,
        "solve_other_coarse": other_coarse,
        "solve_info": {"outer_iters": [i["outer_iters"] for i in info], "coarse_iters": info[0]["coarse_iters"],
                       "refinements": info[0]["refinements"],
                       "true_rel_res": max(i["true_rel_res"] for i in info)},
        "timing_sample": TIMING_SAMPLE,
        "dslash": ({"timed_launches": op_n, "avg_launch_us": op_ms / op_n * 1e3,
                    "GBps": op_bytes / (op_ms * 1e-3) / 1e9, "frac_hbm": op_bytes / (op_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS}
                   if op_n else None),
        "kernel_ms_per_step": {f: round(fams[f]["ms_per_step"], 4) for f in top},
        "kernel_rates": {f: roofline_of(f, fams[f], w["name"])["frac"] for f in top},
        "roofline": roof,
    }
    if not args.no_configs:
        res["configs"] = {}
        for name in ("aniso16x32_fp32", "iso24x64_bf16"):
            if name != w["name"]:
                res["configs"][name] = measure_config(args, name)
                progress(f"config {name} done")
    if not args.no_dslash_hbm:
        res["dslash_hbm"] = dslash_hbm()
        progress("dslash bandwidth done")
    if not args.no_clover and not w.get("c_sw"):
        res["clover"] = {"mg": clover_mg(args)}
        if not args.no_dslash_hbm:
            res["clover"]["dslash_hbm"] = dslash_hbm(clover=True)
        progress("clover leg done")
    if not args.no_evenodd and not w.get("c_sw"):
        res["evenodd"] = evenodd_leg(args)
        progress("even-odd leg done")
    if not args.no_cpu_baseline:
        sm = None
        if small:
            sm = {"spec": small["spec"], "outer": parts[-1]["small_info"]["outer_iters"],
                  "refinements": parts[-1]["small_info"]["refinements"]}
        res["cpu_baseline"] = cpu_baseline(w, cnt, U_host, sm)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
