"""PML studies of Sec. 3 on the GPU path: the amplitude search and the PML-size study.

The paper picks the PML amplitude C (the "C" of the cited PML profile) for
each problem by a small search, and reports that one more PML grid point
lowers the waveguide problem's iteration count sharply, so that the best PML
size grows slowly with the frequency.  Both studies are loops of ordinary
solves.  Here every candidate of a study is one problem of a single context:
the candidates share every setup launch (each launch covers the fronts of one
tree depth over all candidates), and their GMRES solves follow one another on
the same factors' context.

Usage (one JSON line per study on stdout):

    python -m paper_1204_0111_amd.studies amplitude --workload barrier50 \
        --values 2,4,8,15,30 [--precision c128]
    python -m paper_1204_0111_amd.studies gamma --workload waveguide50 --values 5,6,8
"""

import argparse
import json
import time

from . import workloads as wl

MAXIT = 400


def choose(results):
    """The candidate with the fewest iterations over all right-hand sides;
    ties go to the fewer total iterations, then to the smaller value.
    Candidates that did not converge are never chosen while one did."""
    ok = [r for r in results if r["converged"]] or list(results)
    return min(ok, key=lambda r: (r["iters"], sum(r["iters_per_rhs"]), r["value"]))["value"]


def run_candidates(Ps, bs, precision="c128", rtol=1e-5, restart=20, maxit=MAXIT):
    """Set up and solve every problem of Ps in one context; bs[k] is
    (nrhs, N_pad) complex128 on the host.  Returns one dict per problem."""
    import torch
    from .hsweep import Solver
    S = Solver(Ps, precision=precision)
    try:
        S.assemble([P["c"] for P in Ps])
        t0 = time.perf_counter()
        S.setup()
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        fbytes = [S.query(k, "factor_bytes") for k in range(len(Ps))]
        dev = [torch.as_tensor(b).to("cuda") for b in bs]
        _, info = S.solve(dev, rtol=rtol, restart=restart, maxit=maxit)
    finally:
        S.close()
    out, k = [], 0
    for b in bs:
        its = info["iters"][k:k + b.shape[0]]
        rr = info["relres"][k:k + b.shape[0]]
        k += b.shape[0]
        out.append(dict(iters=max(its), iters_per_rhs=its, relres=rr,
                        converged=all(r <= rtol for r in rr), factor_bytes=fbytes[len(out)]))
    return out, dict(t_setup=t_setup, t_solve=info["t_solve"])


def study(P, key, values, precision="c128", rtol=1e-5, restart=20, maxit=MAXIT):
    """Solve P's right-hand sides once per value of P[key] ("C" or "gamma")."""
    Ps, bs = [], []
    for v in values:
        Q = dict(P, **{key: type(P[key])(v)})
        Ps.append(Q)
        bs.append(wl.sources(Q))
    res, times = run_candidates(Ps, bs, precision, rtol, restart, maxit)
    for v, r in zip(values, res):
        r["value"] = v
    return dict(study=key, workload=P["name"], precision=precision, n=list(P["n"]),
                omega=P["omega"], gamma=P["gamma"], C=P["C"], d=P["d"], candidates=res,
                best=choose(res), **times)


def pml_amplitude_search(P, amplitudes, precision="c128", **kw):
    return study(P, "C", [float(a) for a in amplitudes], precision, **kw)


def pml_size_study(P, gammas, precision="c128", **kw):
    return study(P, "gamma", [int(g) for g in gammas], precision, **kw)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("kind", choices=["amplitude", "gamma"])
    ap.add_argument("--workload", default="barrier50")
    ap.add_argument("--values", required=True, help="comma-separated candidates")
    ap.add_argument("--precision", default="c128")
    ap.add_argument("--C", type=float, default=None, help="PML amplitude for the gamma study")
    ap.add_argument("--scale", type=int, default=None,
                    help="interior points per axis (a cube; still 10 points per wavelength)")
    a = ap.parse_args(argv)
    P = wl.make_problem(a.workload, scale_n=None if a.scale is None else (a.scale,) * 3)
    if a.C is not None:
        P["C"] = a.C
    vals = [float(v) for v in a.values.split(",")]
    fn = pml_amplitude_search if a.kind == "amplitude" else pml_size_study
    print(json.dumps(fn(P, vals, a.precision)), flush=True)


if __name__ == "__main__":
    main()
