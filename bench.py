"""Benchmark: unknowns/s to FP64 relative residual 1e-5, complex64 sweep vs complex128 sweep.

A step is one whole solve of the 50^3 Gaussian-random-field workload
(workload "grf50"): assembly, setup (factor and invert every panel) and
flexible GMRES(20) in FP64 until the true relative residual is below 1e-5,
with the fronts and the sweep in complex64.  The velocity and the
right-hand side are resident on the device before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  value = N_int * nrhs * K / (wall seconds of K steps).
The complex128 path (the plain FP64 sweep) is timed the same way as the
comparator, and so is the variant whose Schur-update GEMMs take complex BF16
inputs (FP32 accumulation, "bf16_gemm_variant"); the CPU oracle is timed on a
bounded sample (rank 0 only).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns/s to FP64 rel-res 1e-5: batched FP32-MFMA sweep vs plain FP64 sweep"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
PEAK_TFLOPS = {"fp32_mfma": 157.3, "fp64_mfma": 78.6, "fp32_vector_nonpacked": 78.6}
KERNEL_CLASSES = ["fwd", "bwd", "diag", "panel", "trailing", "schur", "assemble", "inverse", "matvec"]
# kernel class -> (symbol in rocprof output, bound, source file holding it)
KERNEL_INFO = {"fwd": ("k_fwd", "hbm", "solve.hip"), "bwd": ("k_bwd", "hbm", "solve.hip"),
               "diag": ("k_ldlt_diag", "hbm", "factor.hip"),
               "panel": ("k_panel_trsm", "hbm", "factor.hip"),
               "trailing": ("k_update", "mfma", "factor.hip"),
               "schur": ("k_update", "mfma", "factor.hip"),
               "assemble": ("k_assemble", "hbm", "factor.hip"),
               "inverse": ("k_inverse", "mfma", "factor.hip"),
               "matvec": ("k_matvec", "hbm", "krylov.hip")}
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
    src = ("the four forcings f0-f3 of Sec. 3" if P["src"] == "paper"
           else "%d Gaussian point source(s)" % P["nrhs"])
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


def stored_traffic(kclass, workload_key):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or None.

    The summary records FETCH_SIZE and WRITE_SIZE per dispatch of the kernel,
    the same counters read for a plain device copy of known size (the
    calibration factor) and the hash of the kernel's source file; a changed
    source makes the stored counters stale and the traffic is reported as None.
    """
    sym, _, src = KERNEL_INFO[kclass]
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


def roofline(S, step, kclass, prec):
    """Time every launch of one kernel class over one full step with HIP events."""
    S.kernel_timing(kclass, True)
    step()
    t = S.kernel_timing(kclass, False)
    return t


def run_path(Ps, bs, prec, steps, warmup, measure=False, rhs_group=0):
    """Time whole solves of every problem of Ps in one context.  rhs_group > 0
    solves the right-hand sides in groups of that many columns (bounds the
    GMRES workspace of very large problems)."""
    import torch
    from paper_1204_0111_amd.hsweep import Solver
    S = Solver(Ps, precision=prec)
    c_dev = [torch.as_tensor(P["c"]).to("cuda") for P in Ps]
    b_dev = [torch.as_tensor(b).to("cuda") for b in bs]
    nr = max(b.shape[0] for b in bs)
    groups = [(0, nr)] if rhs_group <= 0 else [(g, g + rhs_group) for g in range(0, nr, rhs_group)]
    info = None

    def step():
        S.assemble(c_dev)
        S.setup()
        acc = None
        for g0, g1 in groups:
            r = S.solve([b[g0:g1].contiguous() for b in b_dev], rtol=1e-5, restart=20)[1]
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
        info = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = infos[-1]
    work = sum(P["n"][0] * P["n"][1] * P["n"][2] * b.shape[0] for P, b in zip(Ps, bs))
    nprob = len(Ps)
    out = dict(precision=prec, value=work * steps / wall, ms_per_step=1e3 * wall / steps,
               # the many-shot use: the setup is reused, only the solve counts
               solve_only_value=work / info["t_solve"],
               iters=info["iters"], relres=info["relres"], status=info["status"],
               t_setup_ms=1e3 * info["t_setup"], t_solve_ms=1e3 * info["t_solve"],
               factor_bytes=sum(S.query(k, "factor_bytes") for k in range(nprob)),
               setup_flops=sum(S.query(k, "setup_flops") for k in range(nprob)),
               apply_flops=sum(S.query(k, "apply_flops") for k in range(nprob)),
               panels=sum(S.query(k, "m") for k in range(nprob)))
    if measure:
        # after the timed steps: one instrumented step per kernel class
        out["kernels"] = {k: roofline(S, step, k, prec) for k in KERNEL_CLASSES}
    S.close()
    return out


def roofline_entry(kernels, prec, workload_key):
    """Roofline object of the dominant kernel class (largest summed launch time)."""
    dom = max(kernels, key=lambda k: kernels[k]["seconds"])
    t = kernels[dom]
    sym, bound, _ = KERNEL_INFO[dom]
    n = max(t["launches"], 1)
    avg = t["seconds"] / n
    traffic = stored_traffic(dom, workload_key)
    if bound == "hbm":
        achieved = t["bytes"] / n / avg / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    else:
        achieved = t["flops"] / n / avg / 1e12
        peak = PEAK_TFLOPS["fp32_mfma" if prec != "c128" else "fp64_mfma"]
        unit = "TFLOP/s"
    return dict(kernel=sym, bound=bound, achieved=achieved, peak=peak, unit=unit,
                frac=achieved / peak, traffic=traffic, launches=t["launches"],
                avg_launch_us=1e6 * avg, algorithmic_bytes_per_launch=t["bytes"] / n,
                algorithmic_flops_per_launch=t["flops"] / n)


def cpu_baseline(P, iters):
    """Oracle on a bounded sample: two panel factorisations, one panel solve, one mat-vec.

    Extrapolated to the whole job: setup = first panel + (m-1) x a middle
    panel; one sweep = (2m-1) panel solves; solve = iters x (sweep + mat-vec).
    """
    import numpy as np
    import scipy.sparse.linalg as spla

    from oracle import helmholtz as hz
    from oracle import panels as pn
    from paper_1204_0111_amd import workloads as wl
    c, h, om, al, g, C, d = P["c"], P["h"], P["omega"], P["alpha"], P["gamma"], P["C"], P["d"]
    m = len(pn.panel_bounds(P["n"][2], g, d))
    t0 = time.perf_counter()
    H0 = pn.aux_operator(c, h, om, al, g, C, d, 0)[0]
    lu0 = spla.splu(H0.tocsc())
    t_f0 = time.perf_counter() - t0
    t0 = time.perf_counter()
    H1, lo, hi, ga = pn.aux_operator(c, h, om, al, g, C, d, 1)
    lu1 = spla.splu(H1.tocsc())
    t_f1 = time.perf_counter() - t0
    v = wl.random_complex(H1.shape[0], 1)
    t0 = time.perf_counter()
    lu1.solve(v)
    t_s = time.perf_counter() - t0
    A = hz.helmholtz_operator(c, h, om, g, C, 0.0)
    x = wl.random_complex(A.shape[0], 2)
    t0 = time.perf_counter()
    A @ x
    t_mv = time.perf_counter() - t0
    t_setup = t_f0 + (m - 1) * t_f1
    t_solve = iters * ((2 * m - 1) * t_s + t_mv)
    nint = P["n"][0] * P["n"][1] * P["n"][2]
    del lu0
    return dict(value=nint * P["nrhs"] / (t_setup + t_solve), unit="unknowns/s", cores=1,
                kind="oracle", host_cpus=os.cpu_count(),
                sample="SciPy SuperLU factorisation of panels 0 and 1, one panel solve and one "
                       "mat-vec, extrapolated to %d panels and %d GMRES iterations "
                       "(setup %.1f s, solve %.1f s estimated)" % (m, iters, t_setup, t_solve),
                measured_s=round(t_f0 + t_f1 + t_s + t_mv, 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grf50",
                    help="a workload name of paper_1204_0111_amd.workloads.WORKLOADS")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the variant with BF16 Schur-update GEMM inputs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pml-amp", type=float, default=None,
                    help="override the PML amplitude C (exploration only)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--rhs-group", type=int, default=0,
                    help="solve the right-hand sides in groups of this many columns")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sweeping preconditioner is built and timed on a "
              "single MI355X; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    Ps, bs = workload(args.workload)
    if args.pml_amp is not None:
        for P in Ps:
            P["C"] = args.pml_amp
    P = Ps[0]
    if args.calibrate_copy_mb:
        src = torch.empty(args.calibrate_copy_mb * (1 << 20) // 4, dtype=torch.float32,
                          device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    main_run = run_path(Ps, bs, "c64", args.steps, args.warmup, measure=not args.no_roofline,
                        rhs_group=args.rhs_group)
    kernels = main_run.pop("kernels", None)
    print("# c64: %s" % json.dumps(main_run), file=sys.stderr, flush=True)
    if kernels:
        print("# kernels: %s" % json.dumps(kernels), file=sys.stderr, flush=True)
    bf16 = None
    if not args.no_bf16:
        # the variant with complex BF16 inputs to the Schur-update GEMMs (FP32 accumulation)
        bf16 = run_path(Ps, bs, "c64_bf16", args.steps, args.warmup, rhs_group=args.rhs_group)
        print("# c64_bf16: %s" % json.dumps(bf16), file=sys.stderr, flush=True)
    comp = None
    if not args.no_comparator:
        comp = run_path(Ps, bs, "c128", args.steps, args.warmup, rhs_group=args.rhs_group)
        print("# c128: %s" % json.dumps(comp), file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P, max(comp["iters"]) if comp else max(main_run["iters"]))
    line = dict(metric=METRIC, value=main_run["value"], unit="unknowns/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=main_run["ms_per_step"],
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="c64",
                data="synthetic", config=describe(Ps),
                precision="complex64 fronts and sweep, FP64 GMRES and residual",
                iters=main_run["iters"], relres=main_run["relres"],
                t_setup_ms=main_run["t_setup_ms"], t_solve_ms=main_run["t_solve_ms"],
                solve_only_value=main_run["solve_only_value"],
                comparator=comp,
                bf16_gemm_variant=bf16,
                speedup_vs_fp64=(main_run["value"] / comp["value"]) if comp else None,
                roofline=roofline_entry(kernels, "c64", args.workload) if kernels else None,
                kernel_times_ms={k: 1e3 * v["seconds"] for k, v in kernels.items()} if kernels
                else None,
                # per kernel class over one step: launches, summed time, and the
                # algorithmic rate against the class's roofline
                kernel_classes={k: dict(launches=v["launches"], ms=1e3 * v["seconds"],
                                        gbs=v["bytes"] / max(v["seconds"], 1e-30) / 1e9,
                                        tflops=v["flops"] / max(v["seconds"], 1e-30) / 1e12)
                                for k, v in kernels.items()} if kernels else None,
                cpu_baseline=cpu)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
