"""Throughput benchmark of the IPCS P2-P1 step on one MI355X.

    python bench.py [--gpus 1] [--steps 100] [--warmup 3] [--workload c2]

Default workload (c2): unit square 512 x 512 squares (524,288 triangles,
N2 = 1,050,625 P2 nodes per component, N1 = 263,169 P1 nodes, 2,364,419 DOFs),
FP64, Taylor-Green manufactured solution with seed-drawn (k, nu) (seed 0),
dt = 1e-3, Krylov tolerance 1e-12. A step is one full IPCS step: Dirichlet
data, convection assembly, momentum RHS + BiCGStab, pressure RHS + PCG,
correction RHS + PCG. The run's mesh, matrices and fields are resident in HBM
before the timed region. Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def kernel_bytes(kernel, c, dim):
    """Algorithmic bytes per launch: each array read once, each output written
    once, 8-byte values and vectors, 4-byte indices (formulas in the design doc)."""
    n1, n2 = c.n1, c.n2
    nnz22, nnz11 = c.nnz[0], c.nnz[1]
    sl1, sl2 = 4 * (n1 // 64 + 2), 4 * (n2 // 64 + 2)     # SELL-64 slice pointers
    if kernel == "pcg_spmv_p":     # Kp values+cols once; u in, w = Kp u out
        return 12 * nnz11 + sl1 + 2 * 8 * n1
    if kernel == "pcg_update_p":   # x, r, p, s, w, dinv in; x, r, p, s, u out
        return 11 * 8 * n1
    if kernel == "bicg_spmv":      # A once for all components; phat, rhat in, v out each
        return 12 * nnz22 + sl2 + dim * 3 * 8 * n2
    if kernel == "pcg_spmv_m":     # M once for all components; u in, w out each
        return 12 * nnz22 + sl2 + dim * 2 * 8 * n2
    if kernel == "asm_conv":       # E out, U in, cell DOFs, vertex coordinates
        nloc = 6 if dim == 2 else 10
        return 8 * nnz22 + 8 * dim * n2 + 4 * nloc * c.nc + 8 * dim * c.nv
    raise KeyError(kernel)


def cpu_baseline(w, budget_steps=1):
    """The FP64 oracle on the host cores: one step of the same workload from
    the same initial state (setup not timed)."""
    from threadpoolctl import threadpool_info
    from oracle import fem, ipcs, mesh, problems
    dim, n = w["dim"], w["n"]
    S = fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)))
    pb = problems.TaylorGreen2D(w["k"], w["nu"]) if dim == 2 else problems.Beltrami3D(nu=w["nu"])
    o = ipcs.IPCS(S, pb, ipcs.Params(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                     tol_corr=w["tol"]))
    t0 = time.perf_counter()
    for _ in range(budget_steps):
        o.step()
    dt = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    from paper_2605_25403_amd.workloads import dofs
    return {"value": dofs(dim, n) * budget_steps / dt, "unit": "DOF-steps/s",
            "cores": int(threads), "kind": "oracle",
            "sample": f"{budget_steps} of {w['steps']} IPCS steps of the same workload from "
                      f"the interpolated initial state ({dt:.1f} s; setup not timed; "
                      f"scipy CSR products single-threaded, BLAS up to {threads} threads)",
            "seconds": dt, "iterations": o.iters[-1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-launches", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not "
              "supported (multi-GPU sharding is described in DESIGN.md, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_25403_amd import ipcs as I
    from paper_2605_25403_amd.workloads import dofs, resolve

    w = resolve(args.workload)
    steps = args.steps if args.steps is not None else w["steps"]
    dim, n = w["dim"], w["n"]
    mixed = w["precision"] == "mixed"
    m = I.Mesh.unit_square(n) if dim == 2 else I.Mesh.unit_cube(n)
    p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                              tol_corr=w["tol"],
                              precision=I.IPCS_MIXED if mixed else I.IPCS_FP64)
    stream = torch.cuda.Stream()
    r = I.Run(m, p, stream=stream)
    if dim == 2:
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
    else:
        r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
    ndof = dofs(dim, n)

    for _ in range(args.warmup):
        r.advance(1)
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        stats.append(r.advance(1)[0])
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0

    # per-kernel live timing (HIP events on the run's stream), outside the timed region
    c = m.counts
    it_p = float(np.median([s["it_p"] for s in stats]))
    it_m = float(np.median([max(s["it_mom"][:dim]) for s in stats]))
    it_c = float(np.median([max(s["it_corr"][:dim]) for s in stats]))
    launches = {"pcg_spmv_p": it_p, "pcg_update_p": it_p, "bicg_spmv": 2 * it_m,
                "pcg_spmv_m": it_c, "asm_conv": 1.0}
    ids = {"pcg_spmv_p": I.IPCS_KERNEL_PCG_SPMV_P, "pcg_update_p": I.IPCS_KERNEL_PCG_UPDATE_P,
           "bicg_spmv": I.IPCS_KERNEL_BICG_SPMV, "pcg_spmv_m": I.IPCS_KERNEL_PCG_SPMV_M,
           "asm_conv": I.IPCS_KERNEL_ASM_CONV}
    kern = {}
    for name, kid in ids.items():
        us = I.ipcs_profile_kernel(r.h, kid, args.profile_launches)
        b = kernel_bytes(name, c, dim)
        kern[name] = {"us_per_launch": us, "bytes": b, "GBps": b / (us * 1e-6) / 1e9,
                      "launches_per_step": launches[name],
                      "ms_per_step_est": us * launches[name] / 1000.0}
    dom = max(kern, key=lambda k: kern[k]["ms_per_step_est"])
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{dom}_{args.workload}.json")
    if os.path.exists(tfile):
        traffic = json.load(open(tfile)).get("bytes_per_launch")
    roof = {"bound": "hbm", "kernel": dom, "achieved": kern[dom]["GBps"], "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": kern[dom]["GBps"] / PEAK_HBM_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": kern[dom]["bytes"],
            "us_per_launch": kern[dom]["us_per_launch"]}

    ph = np.array([s["ms"] for s in stats])
    out = {
        "metric": "P2-P1 IPCS DOF-steps/s & HBM GB/s vs FP64 plain; p50/p99 step latency",
        "value": ndof * steps / total,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * total / steps,
        "p50_step_ms": 1000.0 * float(np.percentile(lat, 50)),
        "p99_step_ms": 1000.0 * float(np.percentile(lat, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {dim}D P2-P1 IPCS "
                               f"{'mixed' if mixed else 'FP64 plain'}, "
                               f"unit {'square' if dim == 2 else 'cube'} {n}^{dim} "
                               f"({c.nc} cells), {'TG' if dim == 2 else 'Beltrami'} "
                               f"manufactured solution, dt={w['dt']}, tol={w['tol']}",
                   "dofs": ndof, "N2": c.n2, "N1": c.n1, "nnz_p2p2": c.nnz[0],
                   "k": w.get("k"), "nu": w["nu"], "dt": w["dt"], "seed": w.get("seed")},
        "roofline": roof,
        "kernels": kern,
        "phase_ms_median": {"asm": float(np.median(ph[:, 0])), "momentum": float(np.median(ph[:, 1])),
                            "pressure": float(np.median(ph[:, 2])),
                            "correction": float(np.median(ph[:, 3]))},
        "iterations_median": {"momentum": it_m, "pressure": it_p, "correction": it_c},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
