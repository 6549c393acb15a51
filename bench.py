"""Benchmark: unknowns/s to FP64 relative residual 1e-5, complex64 sweep vs complex128 sweep.

A step is one whole solve of the 100^3 layered workload with its 16 surface
shots as one block (workload "layered100", the largest configuration of the
benchmark set that fits one GPU): assembly, setup (factor and invert every
panel of the moving-PML sweep) and flexible GMRES(20) in FP64 until every
shot's true relative residual is below 1e-5, with the fronts and the sweep in
complex64.  The velocity and the right-hand sides are resident on the device
before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  value = N_int * nrhs * K / (wall seconds of K steps),
reported only when every shot of every timed step converged (status HSW_OK and
true relative residual below 1e-5); otherwise value is null and the exit code
is 1.  The complex128 path (the plain FP64 sweep) is timed the same way as the
comparator, and so is the variant whose Schur-update GEMMs take complex BF16
inputs ("bf16_gemm_variant").  The 50^3 single-source workload and the
48-problem uneven batch are timed as sub-records of the same line.  The CPU
oracle is timed on a bounded sample by a pool of worker processes (rank 0
only).
"""

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns/s to FP64 rel-res 1e-5: batched FP32-MFMA sweep vs plain FP64 sweep"
RTOL = 1e-5
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
PEAK_TFLOPS = {"fp32_mfma": 157.3, "fp64_mfma": 78.6}
KERNEL_CLASSES = ["fwd", "bwd", "scatter", "diag", "panel", "trailing", "schur", "assemble", "inverse",
                  "matvec"]
MM_FROM = 4  # solves with this many right-hand sides or more take the matrix-core passes (mm_min_rhs)


def kernel_info(kclass, nrhs):
    """(symbol in rocprof output, bound, source file) of a kernel class."""
    mm = nrhs >= MM_FROM
    return {"fwd": ("k_fwd_mm" if mm else "k_fwd", "hbm", "solve.hip"),
            "bwd": ("k_bwd_mm" if mm else "k_bwd", "hbm", "solve.hip"),
            "scatter": ("k_rhs_scatter", "hbm", "solve.hip"),
            "diag": ("k_ldlt_diag", "hbm", "factor.hip"),
            "panel": ("k_panel_trsm", "mfma", "factor.hip"),
            "trailing": ("k_update", "mfma", "factor.hip"),
            "schur": ("k_update", "mfma", "factor.hip"),
            "assemble": ("k_assemble", "hbm", "factor.hip"),
            "inverse": ("k_inverse", "mfma", "factor.hip"),
            "matvec": ("k_matvec", "hbm", "krylov.hip")}[kclass]


PROFILES = os.path.join(ROOT, "profiles")


def workload(name):
    """The workload's problems and right-hand-side blocks (lists; the uneven
    batch has one entry per problem)."""
    from paper_1204_0111_amd import workloads as wl
    nsub = wl.WORKLOADS[name].get("nprob", 1)
    Ps = [wl.make_problem(name, sub=k) for k in range(nsub)]
    return Ps, [wl.sources(P) for P in Ps]


MODEL_TEXT = {"constant": "constant velocity 1",
              "grf": "Gaussian-random-field velocity in [1,3]",
              "layered": "8 dipping layers, velocity 1.5-6.0 with 5% noise",
              "wedge_salt": "wedge layers 2.0/3.0/4.5 with a c=4.5 salt body and 3% noise",
              "barrier": "unit velocity with a c=1e10 barrier slab (Sec. 3)",
              "wedge_paper": "three-layer wedge 2/1.5/3 (Sec. 3)",
              "two_layer": "two layers 4/1 split at x2=0.5 (Sec. 3)",
              "waveguide": "Gaussian waveguide 1.25(1-0.4exp(-32r^2)) (Sec. 3)"}


def describe(Ps):
    from paper_1204_0111_amd import workloads as wl
    if len(Ps) > 1:
        P = Ps[0]
        sizes = [list(Q["n"]) for Q in Ps]
        return dict(workload="uneven batch of %d problems, interior sizes drawn from 30..70 per "
                             "axis, %s each, 10 points per wavelength, PML gamma=%d (amplitude %.1f), "
                             "panel depth %d, ND leaf %d, %d surface shots per problem, one batched "
                             "setup and solve, GMRES(20) to FP64 rel-res 1e-5"
                             % (len(Ps), MODEL_TEXT[wl.WORKLOADS[P["name"]]["model"]], P["gamma"],
                                P["C"], P["d"], P["leaf"], P["nrhs"]),
                    name=P["name"], problems=len(Ps), n=sizes, gamma=P["gamma"], panel_depth=P["d"],
                    leaf=P["leaf"], pml_amp=P["C"], alpha=P["alpha"], nrhs=P["nrhs"])
    P = Ps[0]
    model = MODEL_TEXT[wl.WORKLOADS[P["name"]]["model"]]
    if P["src"] == "paper":
        src = "the four forcings f0-f3 of Sec. 3"
    elif P["nrhs"] > 1:
        src = "%d Gaussian surface shots solved as one block" % P["nrhs"]
    else:
        src = "1 Gaussian point source"
    return dict(workload="%dx%dx%d interior, %s, 10 points per wavelength, PML gamma=%d "
                         "(amplitude %.1f), panel depth %d, ND leaf %d, %s, "
                         "GMRES(20) to FP64 rel-res 1e-5"
                         % (P["n"] + (model, P["gamma"], P["C"], P["d"], P["leaf"], src)),
                name=P["name"], n=list(P["n"]), gamma=P["gamma"], panel_depth=P["d"],
                leaf=P["leaf"], pml_amp=P["C"], alpha=P["alpha"], omega=P["omega"],
                nrhs=P["nrhs"])


def source_hash(fname):
    import hashlib
    path = os.path.join(ROOT, "paper_1204_0111_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def stored_traffic(sym, src, workload_key):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or None.

    The summary records FETCH_SIZE and WRITE_SIZE per dispatch of the kernel,
    the same counters read for a plain device copy of known size (the
    calibration factor) and the hash of the kernel's source file; a changed
    source makes the stored counters stale and the traffic is reported as None.
    """
    path = os.path.join(PROFILES, "%s_%s_pmc.txt" % (sym, workload_key))
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("result:"):
            rec = json.loads(line[len("result:"):])
    if not rec or rec.get("source_hash") != source_hash(src):
        return None
    return rec.get("hbm_bytes_per_launch")


def converged(info):
    return info["status"] == "HSW_OK" and max(info["relres"]) < RTOL


def run_path(Ps, bs, prec, steps, warmup, measure=False, rhs_group=0, options=None):
    """Time whole solves of every problem of Ps in one context.  rhs_group > 0
    solves the right-hand sides in groups of that many columns (bounds the
    GMRES workspace of very large problems).  Every timed step's status and
    residuals are kept: the rate counts only if all of them converged.
    options: context options set before the first step."""
    import torch
    from paper_1204_0111_amd.hsweep import Solver
    S = Solver(Ps, precision=prec)
    for key, val in (options or {}).items():
        S.set_option(key, val)
    c_dev = [torch.as_tensor(P["c"]).to("cuda") for P in Ps]
    b_dev = [torch.as_tensor(b).to("cuda") for b in bs]
    nr = max(b.shape[0] for b in bs)
    groups = [(0, nr)] if rhs_group <= 0 else [(g, g + rhs_group) for g in range(0, nr, rhs_group)]

    def step():
        S.assemble(c_dev)
        S.setup()
        acc = None
        for g0, g1 in groups:
            r = S.solve([b[g0:g1].contiguous() for b in b_dev], rtol=RTOL, restart=20)[1]
            if acc is None:
                acc = dict(r)
            else:
                acc["iters"] = acc["iters"] + r["iters"]
                acc["relres"] = acc["relres"] + r["relres"]
                acc["t_solve"] += r["t_solve"]
                if r["status"] != "HSW_OK":
                    acc["status"] = r["status"]
        return acc

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = infos[-1]
    ok = all(converged(i) for i in infos)
    work = sum(P["n"][0] * P["n"][1] * P["n"][2] * b.shape[0] for P, b in zip(Ps, bs))
    nprob = len(Ps)
    out = dict(precision=prec, converged=ok,
               status=sorted(set(i["status"] for i in infos)),
               value=work * steps / wall if ok else None, ms_per_step=1e3 * wall / steps,
               # the many-shot use: the setup is reused, only the solve counts
               solve_only_value=work / info["t_solve"] if ok else None,
               iters=info["iters"], relres=info["relres"],
               max_relres=max(max(i["relres"]) for i in infos),
               t_setup_ms=1e3 * info["t_setup"], t_solve_ms=1e3 * info["t_solve"],
               factor_bytes=sum(S.query(k, "factor_bytes") for k in range(nprob)),
               setup_flops=sum(S.query(k, "setup_flops") for k in range(nprob)),
               apply_flops=sum(S.query(k, "apply_flops") for k in range(nprob)),
               panels=sum(S.query(k, "m") for k in range(nprob)))
    if measure:
        # after the timed steps: one instrumented step per kernel class, each
        # launch of the class bracketed by HIP events on its own stream
        out["kernels"] = {}
        for k in KERNEL_CLASSES:
            S.kernel_timing(k, True)
            step()
            out["kernels"][k] = S.kernel_timing(k, False)
    S.close()
    return out


def roofline_entry(kernels, prec, workload_key, nrhs):
    """Roofline object of the dominant kernel class (largest summed launch time)."""
    dom = max(kernels, key=lambda k: kernels[k]["seconds"])
    t = kernels[dom]
    sym, bound, src = kernel_info(dom, nrhs)
    n = max(t["launches"], 1)
    avg = t["seconds"] / n
    traffic = stored_traffic(sym, src, workload_key)
    if bound == "hbm":
        achieved = t["bytes"] / n / avg / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    else:
        achieved = t["flops"] / n / avg / 1e12
        peak = PEAK_TFLOPS["fp32_mfma" if prec != "c128" else "fp64_mfma"]
        unit = "TFLOP/s"
    return dict(kernel=sym, kernel_class=dom, bound=bound, achieved=achieved, peak=peak, unit=unit,
                frac=achieved / peak, traffic=traffic, launches=t["launches"],
                avg_launch_us=1e6 * avg, algorithmic_bytes_per_launch=t["bytes"] / n,
                algorithmic_flops_per_launch=t["flops"] / n)


def kernel_table(kernels):
    """Per kernel class over one step: launches, summed time and the
    algorithmic rates against the class's roofline."""
    return {k: dict(launches=v["launches"], ms=1e3 * v["seconds"],
                    gbs=v["bytes"] / max(v["seconds"], 1e-30) / 1e9,
                    tflops=v["flops"] / max(v["seconds"], 1e-30) / 1e12)
            for k, v in kernels.items()}


# ---------------------------------------------------------------- CPU oracle
def _oracle_panel(args):
    """Worker: the oracle's work for one panel of the workload -- assemble
    its auxiliary problem H_i, factor it with SciPy's sparse LU (as
    oracle.sweep.Sweep does) and apply T_i to nrhs vectors once."""
    name, i, nrhs = args
    # one thread per worker (set before NumPy loads its BLAS): the pool's
    # workers are the parallelism, and threaded BLAS inside eight concurrent
    # sparse LUs oversubscribes the host
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy as np
    import scipy.sparse.linalg as spla

    from oracle import panels as pn
    from paper_1204_0111_amd import workloads as wl
    P = wl.make_problem(name)
    t0 = time.perf_counter()
    H, lo, hi, ga = pn.aux_operator(P["c"], P["h"], P["omega"], P["alpha"], P["gamma"], P["C"],
                                    P["d"], i)
    print("# oracle panel %d: factoring H_i of order %d" % (i, H.shape[0]), file=sys.stderr, flush=True)
    lu = spla.splu(H.tocsc())
    t1 = time.perf_counter()
    v = wl.random_complex((H.shape[0], nrhs), 7 + i)
    lu.solve(v)
    t2 = time.perf_counter()
    return i, t1 - t0, t2 - t1


def cpu_workers():
    """Worker processes of the oracle pool: the process's CPU share, at most 8
    (the sparse LU of a 100^3 panel fills about 5 GB; more concurrent ones
    contend for host memory bandwidth and each takes far longer)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(8, n))


def cpu_baseline(name, iters, max_workers=None):
    """The oracle on a bounded sample of the workload, timed by a pool of
    worker processes (spawned: no GPU state is inherited).

    Sample: P = min(workers, m) panels are factored at once, one per worker,
    each also applying its T_i to the workload's nrhs vectors; the main
    process times one oracle mat-vec of the block and one Arnoldi
    orthogonalisation step.  Extrapolation to the whole job: the pool
    factors all m panels in ceil(m / P) rounds of the measured wall time; a
    sweep is 2m - 1 panel solves in sequence (Alg. 1.5) at the mean measured
    time; GMRES(20) runs `iters` iterations, each a sweep, a mat-vec and the
    orthogonalisation against on average 10 basis vectors."""
    import numpy as np

    from oracle import helmholtz as hz
    from oracle import panels as pn
    from paper_1204_0111_amd import workloads as wl
    P = wl.make_problem(name)
    nrhs = P["nrhs"]
    m = len(pn.panel_bounds(P["n"][2], P["gamma"], P["d"]))
    workers = min(max_workers or cpu_workers(), m)
    jobs = [(name, i, nrhs) for i in range(workers)]
    ctx = mp.get_context("spawn")
    res = []
    with ctx.Pool(workers) as pool:
        for r in pool.imap_unordered(_oracle_panel, jobs):
            res.append(r)
            print("# oracle panel %d: factored in %.1f s, T_i of %d vectors in %.2f s"
                  % (r[0], r[1], nrhs, r[2]), file=sys.stderr, flush=True)
    # the round of concurrent factorisations lasts as long as its slowest
    # worker (the workers' own clocks leave out the processes' start-up)
    t_round = max(r[1] for r in res)
    t_solve_panel = sum(r[2] for r in res) / len(res)
    A = hz.helmholtz_operator(P["c"], P["h"], P["omega"], P["gamma"], P["C"], 0.0)
    X = wl.random_complex((A.shape[0], nrhs), 2)
    t0 = time.perf_counter()
    A @ X
    t_mv = time.perf_counter() - t0
    V = wl.random_complex((A.shape[0], 10), 3)
    w = X[:, 0].copy()
    t0 = time.perf_counter()
    for j in range(10):  # modified Gram-Schmidt against 10 basis vectors, one right-hand side
        w -= np.vdot(V[:, j], w) * V[:, j]
    t_orth = (time.perf_counter() - t0) * nrhs
    t_setup = t_round * math.ceil(m / workers)
    t_solve = iters * ((2 * m - 1) * t_solve_panel + t_mv + t_orth)
    nint = P["n"][0] * P["n"][1] * P["n"][2]
    # cores: the worker processes, one BLAS thread each
    return dict(value=nint * nrhs / (t_setup + t_solve), unit="unknowns/s", cores=workers,
                kind="oracle",
                sample="%d of the %d panels factored at once by %d worker processes (SciPy SuperLU, "
                       "as the oracle's sweep does), each applying its T_i to %d vectors, plus one "
                       "oracle mat-vec and one orthogonalisation step; extrapolated to %d panels "
                       "(%d rounds), %d panel solves per sweep and %d GMRES iterations "
                       "(setup %.1f s, solve %.1f s estimated)"
                       % (workers, m, workers, nrhs, m, math.ceil(m / workers), 2 * m - 1, iters,
                          t_setup, t_solve),
                measured_s=round(t_round + t_solve_panel + t_mv + t_orth, 2),
                host_cpus=os.cpu_count())


# ------------------------------------------------------------------ records
def measure_workload(name, steps, warmup, comparator=True, bf16=False, roofline=False, rhs_group=0,
                     log=None, device_test=False, options=None):
    Ps, bs = workload(name)
    nrhs = max(b.shape[0] for b in bs)
    rec = dict(config=describe(Ps))
    main_run = run_path(Ps, bs, "c64", steps, warmup, measure=roofline, rhs_group=rhs_group, options=options)
    kernels = main_run.pop("kernels", None)
    if log:
        log("c64 %s" % name, main_run)
    rec["c64"] = main_run
    if kernels:
        rec["roofline"] = roofline_entry(kernels, "c64", name, nrhs)
        rec["kernel_classes"] = kernel_table(kernels)
    if bf16:
        rec["bf16"] = run_path(Ps, bs, "c64_bf16", steps, warmup, rhs_group=rhs_group)
        if log:
            log("c64_bf16 %s" % name, rec["bf16"])
    if device_test:
        # GMRES with the convergence test on the device, one read per cycle,
        # the cycle's steps issued one by one or replayed from a capture
        rec["device_test"] = {}
        for graph in (0, 1):
            r = run_path(Ps, bs, "c64", steps, warmup, rhs_group=rhs_group,
                         options=dict(gmres_device_test=1, graph=graph))
            rec["device_test"]["captured" if graph else "issued"] = dict(
                (k, r[k]) for k in ("value", "ms_per_step", "t_solve_ms", "converged", "iters"))
            if log:
                log("c64 device test graph=%d %s" % (graph, name), r)
    if comparator:
        try:
            rec["c128"] = run_path(Ps, bs, "c128", steps, warmup, rhs_group=rhs_group)
        except RuntimeError as e:  # HSW_E_NOMEM: the complex128 factors do not fit one device
            rec["c128"] = dict(precision="c128", value=None, error=str(e))
        if log:
            log("c128 %s" % name, rec["c128"])
    return rec


def sub_record(rec):
    c64, c128 = rec["c64"], rec.get("c128")
    out = dict(config=rec["config"], value=c64["value"], ms_per_step=c64["ms_per_step"],
               converged=c64["converged"], status=c64["status"], iters=c64["iters"],
               max_relres=c64["max_relres"], t_setup_ms=c64["t_setup_ms"],
               t_solve_ms=c64["t_solve_ms"], solve_only_value=c64["solve_only_value"])
    if c128 is not None:
        out["comparator"] = c128
        out["speedup_vs_fp64"] = (c64["value"] / c128["value"]) if c64["value"] and c128.get("value") \
            else None
    if rec.get("roofline") is not None:
        out["roofline"] = rec["roofline"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered100",
                    help="a workload name of paper_1204_0111_amd.workloads.WORKLOADS")
    ap.add_argument("--sub", default="grf50,batch48",
                    help="comma-separated workloads timed as sub-records ('' for none)")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the variant with BF16 Schur-update GEMM inputs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="worker processes of the oracle pool (default: the CPU share, at most 8)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-device-test", action="store_true",
                    help="skip the GMRES variant with the convergence test on the device")
    ap.add_argument("--set", default="",
                    help="context options of the headline's complex64 run, as key=value,... "
                         "(e.g. mm_fwd_form=2; see hsw_set_option)")
    ap.add_argument("--rhs-group", type=int, default=0,
                    help="solve the right-hand sides in groups of this many columns")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sweeping preconditioner is built and timed on a "
              "single MI355X; runs on several GPUs are not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    def log(tag, rec):
        print("# %s: %s" % (tag, json.dumps(rec)), file=sys.stderr, flush=True)

    if args.calibrate_copy_mb:
        src = torch.empty(args.calibrate_copy_mb * (1 << 20) // 4, dtype=torch.float32,
                          device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    opts = dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in args.set.split(",") if kv)
    head = measure_workload(args.workload, args.steps, args.warmup, comparator=not args.no_comparator,
                            bf16=not args.no_bf16, roofline=not args.no_roofline,
                            rhs_group=args.rhs_group, log=log, device_test=not args.no_device_test,
                            options=opts)
    main_run, comp = head["c64"], head.get("c128")
    subs = {}
    for name in [s for s in args.sub.split(",") if s and s != args.workload]:
        rec = measure_workload(name, args.steps, args.warmup, comparator=not args.no_comparator,
                               roofline=not args.no_roofline, log=log)
        subs[name] = sub_record(rec)
    cpu = None
    if not args.no_cpu_baseline:
        its = max((comp or main_run)["iters"])
        cpu = cpu_baseline(args.workload, its, args.cpu_workers or None)
    ok = main_run["converged"] and (comp is None or comp.get("converged", False))
    if head.get("bf16") is not None:
        ok = ok and head["bf16"]["converged"]
    line = dict(metric=METRIC, value=main_run["value"] if ok else None, unit="unknowns/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=main_run["ms_per_step"],
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="c64",
                data="synthetic", config=head["config"],
                precision="complex64 fronts and sweep, FP64 GMRES and residual",
                status=main_run["status"], converged=main_run["converged"],
                iters=main_run["iters"], relres=main_run["relres"], max_relres=main_run["max_relres"],
                t_setup_ms=main_run["t_setup_ms"], t_solve_ms=main_run["t_solve_ms"],
                solve_only_value=main_run["solve_only_value"],
                factor_bytes=main_run["factor_bytes"],
                comparator=comp,
                bf16_gemm_variant=head.get("bf16"),
                gmres_device_test=head.get("device_test"),
                speedup_vs_fp64=(main_run["value"] / comp["value"])
                if ok and comp and comp.get("value") else None,
                roofline=head.get("roofline"),
                kernel_classes=head.get("kernel_classes"),
                sub_records=subs,
                cpu_baseline=cpu)
    print(json.dumps(line), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
