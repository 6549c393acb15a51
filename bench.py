"""Benchmark: unknowns/s to FP64 relative residual 1e-5, complex64 sweep vs complex128 sweep.

A step is one whole solve of the 50^3 workload (second benchmark
configuration): assembly, setup (factor and invert every panel) and
flexible GMRES(20) in FP64 until the true relative residual is below 1e-5,
with the fronts and the sweep in complex64.  The velocity and the
right-hand side are resident on the device before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  value = N_int * nrhs * K / (wall seconds of K steps).
The complex128 path (the plain FP64 sweep) is timed the same way as the
comparator; the CPU oracle is timed on a bounded sample (rank 0 only).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns/s to FP64 rel-res 1e-5: batched FP32-MFMA sweep vs plain FP64 sweep"
HBM_PEAK_GBS = 8000.0


def workload(cfg):
    from paper_1204_0111_amd import workloads as wl
    P = wl.make_problem(cfg)
    b = wl.gaussian_sources(P["n"], P["gamma"], P["h"], P["centers"])
    return P, b.reshape(b.shape[0], -1)


def describe(P):
    return dict(workload="%dx%dx%d interior, Gaussian-random-field velocity in [1,3], 10 points "
                         "per wavelength, PML gamma=%d (amplitude %.1f), panel depth %d, ND leaf %d, "
                         "%d Gaussian point source(s), GMRES(20) to FP64 rel-res 1e-5"
                         % (P["n"] + (P["gamma"], P["C"], P["d"], P["leaf"], P["nrhs"])),
                n=list(P["n"]), gamma=P["gamma"], panel_depth=P["d"], leaf=P["leaf"],
                pml_amp=P["C"], alpha=P["alpha"], omega=P["omega"], nrhs=P["nrhs"])


def run_path(P, b, prec, steps, warmup):
    import torch
    from paper_1204_0111_amd.hsweep import Solver
    S = Solver(P, precision=prec)
    c_dev = torch.as_tensor(P["c"]).to("cuda")
    b_dev = torch.as_tensor(b).to("cuda")
    info = None

    def step():
        S.assemble([c_dev])
        S.setup()
        return S.solve([b_dev], rtol=1e-5, restart=20)[1]

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
    nint = P["n"][0] * P["n"][1] * P["n"][2]
    out = dict(precision=prec, value=nint * P["nrhs"] * steps / wall, ms_per_step=1e3 * wall / steps,
               iters=info["iters"], relres=info["relres"], status=info["status"],
               t_setup_ms=1e3 * info["t_setup"], t_solve_ms=1e3 * info["t_solve"],
               factor_bytes=S.query(0, "factor_bytes"), setup_flops=S.query(0, "setup_flops"),
               apply_flops=S.query(0, "apply_flops"), panels=S.query(0, "m"))
    S.close()
    return out


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
    ap.add_argument("--cfg", type=int, default=2)
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sweeping preconditioner is built and timed on a "
              "single MI355X; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    P, b = workload(args.cfg)
    main_run = run_path(P, b, "c64", args.steps, args.warmup)
    print("# c64: %s" % json.dumps(main_run), file=sys.stderr, flush=True)
    comp = None
    if not args.no_comparator:
        comp = run_path(P, b, "c128", args.steps, args.warmup)
        print("# c128: %s" % json.dumps(comp), file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P, max(comp["iters"]) if comp else max(main_run["iters"]))
    line = dict(metric=METRIC, value=main_run["value"], unit="unknowns/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=main_run["ms_per_step"],
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="c64",
                data="synthetic", config=describe(P),
                precision="complex64 fronts and sweep, FP64 GMRES and residual",
                iters=main_run["iters"], relres=main_run["relres"],
                t_setup_ms=main_run["t_setup_ms"], t_solve_ms=main_run["t_solve_ms"],
                comparator=comp,
                speedup_vs_fp64=(main_run["value"] / comp["value"]) if comp else None,
                cpu_baseline=cpu)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
