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
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    """Progress of the benchmark's stages, on stderr (the JSON line is stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# kernel name -> (library kernel id, source file); ids are IPCS_KERNEL_* of include/ipcs.h
KERNELS = {
    "pcg_spmv_p": (0, "kernels_krylov.hip"),
    "pcg_update_p": (1, "kernels_krylov.hip"),
    "asm_conv": (2, "kernels_asm.hip"),
    "bicg_spmv": (3, "kernels_krylov.hip"),
    "pcg_spmv_m": (4, "kernels_krylov.hip"),
    "bicg_spmv_t": (5, "kernels_krylov.hip"),
    "bicg_update_s": (6, "kernels_krylov.hip"),
    "bicg_update_x": (7, "kernels_krylov.hip"),
    "pcg_update_m": (8, "kernels_krylov.hip"),
    "pcg_fused_p": (9, "kernels_fcg.hip"),
    "asm_sum": (10, "kernels_asm.hip"),
}


def kernel_bytes(kernel, c, dim, vsz=8, p3=False):
    """Algorithmic bytes per launch: each array read once, each output written
    once, vsz-byte matrix values, 8-byte vectors, 4-byte indices (2-byte local
    indices in the fused Poisson CG; its halo re-reads are not counted)."""
    n1, n2 = c.n1, c.n2
    if kernel == "pcg_fused_p":    # Kp values + local cols; dinv, x, p, r, s, w in; x, p, s, r, w out
        return (vsz + 2) * c.nnz[1] + 11 * 8 * n1
    nnz22, nnz11 = c.nnz[0], c.nnz[1]
    sl1, sl2 = 4 * (n1 // 64 + 2), 4 * (n2 // 64 + 2)     # SELL-64 slice pointers
    if kernel == "pcg_spmv_p":     # Kp values+cols once; u in, w = Kp u out
        return (vsz + 4) * nnz11 + sl1 + 2 * 8 * n1
    if kernel == "pcg_update_p":   # x, r, p, s, w, dinv in; x, r, p, s, u out
        return 11 * 8 * n1
    if kernel == "bicg_spmv":      # A once for all components; phat, rhat in, v out each
        return (vsz + 4) * nnz22 + sl2 + dim * 3 * 8 * n2
    if kernel == "bicg_spmv_t":    # A once; shat, s, rhat in, t out each
        return (vsz + 4) * nnz22 + sl2 + dim * 4 * 8 * n2
    if kernel == "bicg_update_s":  # dinv; r, v in, s, shat out each
        return 8 * n2 + dim * 4 * 8 * n2
    if kernel == "bicg_update_x":  # dinv; x, s, t, p, v in, x, r, p, phat out each
        return 8 * n2 + dim * 9 * 8 * n2
    if kernel == "pcg_spmv_m":     # M once for all components; u in, w out each
        return (vsz + 4) * nnz22 + sl2 + dim * 2 * 8 * n2
    if kernel == "pcg_update_m":   # dinv; x, r, p, s, w in, x, r, p, s, u out each
        return 8 * n2 + dim * 10 * 8 * n2
    nloc = 10 if (p3 or dim == 3) else 6
    if kernel == "asm_conv" and dim == 2:   # row-owner: E out; U, cell DOFs, vertices in
        return vsz * nnz22 + 8 * dim * n2 + 4 * nloc * c.nc + 8 * dim * c.nv
    if kernel == "asm_conv":       # 3D cell pass: local matrices out; U, DOFs, vertices in
        return vsz * nloc * nloc * c.nc + 8 * dim * n2 + 4 * nloc * c.nc + 8 * dim * c.nv
    if kernel == "asm_sum":        # local matrices in, E out, incidences and slots in
        return vsz * nloc * nloc * c.nc + vsz * nnz22 + 4 * nloc * c.nc + nloc * nloc * c.nc
    raise KeyError(kernel)


def unit_bytes(kernel, c, dim, vsz=8):
    """Algorithmic bytes per launch in the units of the method's byte model:
    each array read once, each output written once, vsz-byte matrix values,
    8-byte vectors, 4-byte CSR indices (column per entry, row pointer per row).
    SpMV of a pattern with N rows: (vsz + 4) nnz + 4 (N + 1) + 2 * 8 * N per
    vector; a vector pass: 8 * N. One launch of the one-kernel Poisson CG is
    one iteration: an SpMV of Kp and five P1 vector passes. The velocity
    SpMVs apply A (or M) to d vectors at once. None when the model has no unit
    for the kernel (then kernel_bytes is used)."""
    n1, n2, nnz22, nnz11 = c.n1, c.n2, c.nnz[0], c.nnz[1]
    spmv = lambda nnz, n, nvec: (vsz + 4) * nnz + 4 * (n + 1) + 2 * 8 * n * nvec
    if kernel == "pcg_fused_p":
        return spmv(nnz11, n1, 1) + 5 * 8 * n1
    if kernel in ("bicg_spmv", "bicg_spmv_t", "pcg_spmv_m"):
        return spmv(nnz22, n2, dim)
    if kernel == "pcg_spmv_p":
        return spmv(nnz11, n1, 1)
    if kernel == "asm_conv" and dim == 2:
        return kernel_bytes(kernel, c, dim, vsz)
    return None


def rocprof_avg_us(kernel, workload):
    """Average duration (us) of a kernel in the committed rocprofv3 kernel
    statistics of a workload (profiles/kernels_<workload>.txt), or None."""
    import re
    f = os.path.join(ROOT, "profiles", f"kernels_{workload}.txt")
    sym = {"pcg_fused_p": r"^void k_fcg_iter1<", "bicg_spmv": r"^void k_bicg_spmv<0,",
           "bicg_spmv_t": r"^void k_bicg_spmv<1,", "asm_conv": r"^void k_(asm_rows<2, OpConv|conv_cells)",
           "asm_sum": r"^void k_asm_local<"}.get(kernel)
    if sym is None or not os.path.exists(f):
        return None
    for line in open(f):
        if re.search(sym, line):
            parts = line.split()
            # name ... calls avg min max %
            return float(parts[-4])
    return None


def source_sha1(fname):
    with open(os.path.join(ROOT, "paper_2605_25403_amd", "csrc", fname), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, or None when there is none or the kernel's
    source has changed since the counters were taken."""
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(tfile):
        return None
    kv = {}
    for line in open(tfile):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha1") != source_sha1(KERNELS[kernel][1]):
        return None
    return float(kv["bytes_per_launch"])


def cpu_baseline(w, budget_steps=3):
    """The FP64 oracle on the host cores: the first budget_steps steps of the
    same workload from the same initial state (setup not timed), with the
    wall time of each phase per step, then one more step with every thread
    pool limited to one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import fem, ipcs, mesh, problems
    dim, n = w["dim"], w["n"]
    order = 3 if w.get("pair", 0) == 1 else 2
    S = fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)), order=order)
    pb = problems.TaylorGreen2D(w["k"], w["nu"]) if dim == 2 else problems.Beltrami3D(nu=w["nu"])
    o = ipcs.IPCS(S, pb, ipcs.Params(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                     tol_corr=w["tol"]))
    t0 = time.perf_counter()
    for _ in range(budget_steps):
        o.step()
    dt = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    phases = {k: [round(tt[k] * 1000.0, 1) for tt in o.times] for k in o.times[0]}
    # the next step again, with every thread pool limited to one thread
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        o.step()
        dt1 = time.perf_counter() - t1
    ndof = dim * S.Nu + S.Np
    # the steady solver's oracle (Newton with sparse direct solves) on the
    # Section 4.2 example at its largest printed size, 64 x 64 squares
    from oracle import steady
    Ss = fem.Space(*mesh.unit_square(64, 64))
    so = steady.SteadyNewton(Ss, problems.SteadyPaper2D(1.0), 1.0)
    t2 = time.perf_counter()
    so.run()
    dts = time.perf_counter() - t2
    steady_cpu = {"n": 64, "dofs": 2 * Ss.Nu + Ss.Np, "newton_steps": len(so.history),
                  "seconds": dts,
                  "dof_newton_steps_per_s": (2 * Ss.Nu + Ss.Np) * len(so.history) / dts}
    return {"value": ndof * budget_steps / dt, "unit": "DOF-steps/s", "steady_newton": steady_cpu,
            "cores": int(threads), "kind": "oracle",
            "sample": f"the first {budget_steps} of {w['steps']} IPCS steps of the same workload "
                      f"from the interpolated initial state ({dt:.1f} s; setup not timed; "
                      f"scipy CSR products single-threaded, BLAS up to {threads} threads); "
                      f"the following step with one thread: {dt1:.1f} s",
            "seconds": dt, "phase_ms_per_step": phases,
            "iterations": [[list(map(int, m)), int(pi), list(map(int, cc))]
                           for m, pi, cc in o.iters[:budget_steps]],
            "value_1thread": ndof / dt1}


def pmc_summary(fetch_dir, write_dir, kernel, workload, calib_mib, command):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; CSV output)
    of one bench command into HBM bytes per launch of one kernel, each counter
    scaled by what it reads for a plain device copy of calib_mib MiB in the
    same run. Writes profiles/traffic_<kernel>_<workload>.json and .txt."""
    import csv
    import glob
    import re

    def rows(d, counter):
        out = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out

    sym = {"pcg_update_p": r"k_cg_update<1>", "pcg_spmv_p": r"k_cg_spmv<1,",
           "pcg_fused_p": r"k_fcg_iter1?<",
           "bicg_update_x": r"k_bicg_5<", "bicg_spmv": r"k_bicg_spmv<0,",
           "asm_conv": r"OpConv<|k_conv_cells(_mfma)?<", "asm_sum": r"k_asm_local<"}[kernel]
    # the calibration copy is a device-to-device hipMemcpy (torch's copy_ of
    # contiguous tensors); fills (torch's elementwise FillFunctor) are not
    copy_re = re.compile(r"copyBuffer")
    res = {}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rr = rows(d, counter)
        k = [v for n, v in rr if re.search(sym, n.replace(" ", ""))]
        cp = [v for n, v in rr if copy_re.search(n) and not n.startswith("void ipcs")]
        if not k or not cp:
            raise SystemExit(f"pmc-summary: no {counter} rows for {kernel} or the copy kernel in {d}")
        kib = float(np.median(k))
        copy_kib = max(cp)                      # the large calibration copy
        factor = calib_mib * 1024.0 / copy_kib  # true KiB per counted KiB
        res[name] = {"counter": counter, "kib_per_dispatch_median": kib, "dispatches": len(k),
                     "copy_kib": copy_kib, "scale": factor,
                     "bytes_per_launch": kib * factor * 1024.0}
    fname = KERNELS[kernel][1]
    summary = {"kernel": kernel, "workload": workload, "command": command,
               "calibration": f"device copy of {calib_mib} MiB (reads and writes {calib_mib} MiB)",
               "fetch": res["fetch"], "write": res["write"],
               "bytes_per_launch": res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"],
               "source": f"paper_2605_25403_amd/csrc/{fname}", "source_sha1": source_sha1(fname)}
    base = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}")
    with open(base + ".txt", "w") as f:
        f.write(f"HBM traffic of {kernel} on workload {workload} (rocprofv3 PMC)\n")
        f.write(f"command: {command}\n")
        for nm in ("fetch", "write"):
            r_ = res[nm]
            f.write(f"{r_['counter']}: median {r_['kib_per_dispatch_median']:.1f} KiB/dispatch over "
                    f"{r_['dispatches']} dispatches; the copy of {calib_mib} MiB counts "
                    f"{r_['copy_kib']:.1f} KiB -> scale {r_['scale']:.3f} -> "
                    f"{r_['bytes_per_launch'] / 1e6:.2f} MB per launch\n")
        f.write(f"total HBM bytes per launch: {summary['bytes_per_launch'] / 1e6:.2f} MB\n")
        f.write(f"bytes_per_launch: {summary['bytes_per_launch']:.0f}\n")
        f.write(f"source: {summary['source']}\n")
        f.write(f"source_sha1: {summary['source_sha1']}\n")
    print(json.dumps(summary))


def counters_summary(run_dirs, kernel_regex, name, workload, command, clock_ghz=2.4):
    """Writes profiles/counters_<name>_<workload>.txt from rocprofv3 --pmc runs
    (CSV output; one directory per pass) of one bench command: the median per
    dispatch of each counter for the kernels whose name matches kernel_regex,
    and the VALU utilization they imply. A wave64 FP64 (or non-packed FP32)
    VALU instruction occupies a 16-lane SIMD for 4 cycles, so the VALU issue
    fraction is 4 SQ_INSTS_VALU / (SIMDs x kernel cycles), with 1024 SIMDs
    (256 CUs x 4) and the kernel's cycles from its dispatch timestamps at the
    engine clock; SQ_ACTIVE_INST_VALU (quad-cycles) gives the busy form of
    the same ratio. No GPU use."""
    import csv
    import glob
    import re
    rx = re.compile(kernel_regex)
    vals, durs = {}, []
    for d in run_dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if not rx.search(r["Kernel_Name"].replace(" ", "")):
                    continue
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                if "Start_Timestamp" in r and r.get("End_Timestamp"):
                    durs.append((float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9)
    if not vals:
        raise SystemExit(f"counters-summary: no rows for {kernel_regex} under {run_dirs}")
    med = {k: float(np.median(v)) for k, v in vals.items()}
    dur = float(np.median(durs)) if durs else None
    out = os.path.join(ROOT, "profiles", f"counters_{name}_{workload}.txt")
    with open(out, "w") as o:
        o.write(f"rocprofv3 counters of {name} ({kernel_regex}) on workload {workload}\n")
        o.write(f"command: {command}\n")
        for k in sorted(med):
            o.write(f"{k}: median {med[k]:.6g} per dispatch over {len(vals[k])} dispatches\n")
        if dur:
            o.write(f"dispatch duration (median, counter run): {dur * 1e6:.2f} us\n")
            cyc = dur * clock_ghz * 1e9
            if "SQ_INSTS_VALU" in med:
                o.write(f"VALU issue fraction 4*SQ_INSTS_VALU/(1024*cycles): "
                        f"{4 * med['SQ_INSTS_VALU'] / (1024 * cyc):.3f}\n")
            if "SQ_ACTIVE_INST_VALU" in med:
                o.write(f"VALU busy 4*SQ_ACTIVE_INST_VALU/(1024*cycles): "
                        f"{4 * med['SQ_ACTIVE_INST_VALU'] / (1024 * cyc):.3f}\n")
            if "SQ_VALU_MFMA_BUSY_CYCLES" in med:
                # summed over the SIMDs, as SQ_BUSY_CYCLES is summed over the SEs
                o.write(f"MFMA busy SQ_VALU_MFMA_BUSY_CYCLES/(1024*cycles): "
                        f"{med['SQ_VALU_MFMA_BUSY_CYCLES'] / (1024 * cyc):.3f}\n")
        if "GRBM_GUI_ACTIVE" in med and "SQ_ACTIVE_INST_VALU" in med:
            # GRBM_GUI_ACTIVE reads the busy cycles of the 8 XCDs summed
            o.write(f"VALU busy 4*SQ_ACTIVE_INST_VALU/(1024*GRBM_GUI_ACTIVE/8): "
                    f"{32 * med['SQ_ACTIVE_INST_VALU'] / (1024 * med['GRBM_GUI_ACTIVE']):.3f}\n")
    print(open(out).read())


def trace_summary(trace_dir, workload, command):
    """Writes profiles/kernels_<workload>.txt from the kernel statistics of a
    rocprofv3 --kernel-trace --stats -f csv run (no GPU use)."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit(f"trace-summary: no kernel_stats.csv under {trace_dir}")
    rows = sorted(csv.DictReader(open(f[0])), key=lambda r: -float(r["TotalDurationNs"]))
    out = os.path.join(ROOT, "profiles", f"kernels_{workload}.txt")
    with open(out, "w") as o:
        o.write(f"rocprofv3 kernel statistics, workload {workload}\n")
        o.write(f"command: {command}\n\n")
        o.write(f"{'kernel':70s} {'calls':>7s} {'avg us':>9s} {'min us':>8s} {'max us':>8s} {'%':>6s}\n")
        for r in rows[:30]:
            name = r["Name"].replace("ipcs::", "")
            name = name[:name.index("(")] if "(" in name else name
            o.write(f"{name[:70]:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
                    f"{float(r['MinNs']) / 1e3:8.2f} {float(r['MaxNs']) / 1e3:8.2f} "
                    f"{float(r['Percentage']):6.2f}\n")
    print(open(out).read())


def mixed_form(w, steps, torch, I):
    """The mixed-precision form against the FP64 form on the same problem and
    start: per-step relative L2 (nodal) difference of u and p, and throughput."""
    from paper_2605_25403_amd.workloads import dofs
    m = I.Mesh.unit_square(w["n"]) if w["dim"] == 2 else I.Mesh.unit_cube(w["n"])
    runs = {}
    for name, prec in (("fp64", I.IPCS_FP64), ("mixed", I.IPCS_MIXED)):
        p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                  tol_corr=w["tol"], tol_ir=1e-10, precision=prec)
        r = I.Run(m, p, stream=torch.cuda.Stream())
        if w["dim"] == 2:
            r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
        else:
            r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
        runs[name] = r
    err_u, err_p, lat = [], [], {"fp64": [], "mixed": []}
    it = {"fp64": [], "mixed": []}
    for _ in range(steps):
        for name, r in runs.items():
            t0 = time.perf_counter()
            st = r.advance(1)[0]
            lat[name].append(time.perf_counter() - t0)
            it[name].append(st["it_p"])
        U64, U32 = runs["fp64"].velocity(), runs["mixed"].velocity()
        P64, P32 = runs["fp64"].pressure(), runs["mixed"].pressure()
        err_u.append(float(np.linalg.norm(U32 - U64) / np.linalg.norm(U64)))
        err_p.append(float(np.linalg.norm(P32 - P64) / np.linalg.norm(P64)))
    nd = dofs(w["dim"], w["n"])
    out = {}
    for name in ("fp64", "mixed"):
        ms = 1000.0 * float(np.median(lat[name]))
        out[name] = {"value": nd / (ms / 1000.0), "p50_step_ms": ms,
                     "p99_step_ms": 1000.0 * float(np.percentile(lat[name], 99)),
                     "pressure_iterations_median": float(np.median(it[name]))}
    out["steps"] = steps
    out["rel_l2_diff_vs_fp64_u"] = err_u
    out["rel_l2_diff_vs_fp64_p"] = err_p
    out["speedup_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    return out


def start_form(w, steps, torch, I):
    """The pressure Poisson solve started from the previous step's increment
    against the zero start, on the same problem and start (FP64, and the
    mixed form with the previous start): throughput, Poisson iterations, and
    the per-step relative L2 difference of u and p from the zero start's
    fields (both meet the same stopping test, eq. (9), second line)."""
    from paper_2605_25403_amd.workloads import dofs
    m = I.Mesh.unit_square(w["n"]) if w["dim"] == 2 else I.Mesh.unit_cube(w["n"])
    variants = {"fp64_zero": (I.IPCS_FP64, I.IPCS_START_ZERO),
                "fp64_previous": (I.IPCS_FP64, I.IPCS_START_PREVIOUS),
                "mixed_previous": (I.IPCS_MIXED, I.IPCS_START_PREVIOUS)}
    runs = {}
    for name, (prec, start) in variants.items():
        p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                  tol_corr=w["tol"], tol_ir=1e-10, precision=prec,
                                  poisson_start=start)
        r = I.Run(m, p, stream=torch.cuda.Stream())
        if w["dim"] == 2:
            r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
        else:
            r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
        runs[name] = r
    lat = {k: [] for k in runs}
    it = {k: [] for k in runs}
    diff = {k: {"u": [], "p": []} for k in runs if k != "fp64_zero"}
    for _ in range(steps):
        for name, r in runs.items():
            t0 = time.perf_counter()
            st = r.advance(1)[0]
            lat[name].append(time.perf_counter() - t0)
            it[name].append(st["it_p"])
        U0, P0 = runs["fp64_zero"].velocity(), runs["fp64_zero"].pressure()
        for name, d in diff.items():
            d["u"].append(float(np.linalg.norm(runs[name].velocity() - U0) / np.linalg.norm(U0)))
            d["p"].append(float(np.linalg.norm(runs[name].pressure() - P0) / np.linalg.norm(P0)))
    nd = dofs(w["dim"], w["n"])
    out = {"steps": steps}
    for name in runs:
        # the first step starts from zero in every variant: medians over the rest
        ms = 1000.0 * float(np.median(lat[name][1:]))
        out[name] = {"value": nd / (ms / 1000.0), "p50_step_ms": ms,
                     "pressure_iterations_median": float(np.median(it[name][1:])),
                     "pressure_iterations": it[name]}
        if name in diff:
            out[name]["rel_l2_diff_vs_zero_start_u"] = diff[name]["u"]
            out[name]["rel_l2_diff_vs_zero_start_p"] = diff[name]["p"]
            out[name]["speedup_vs_zero_start"] = out[name]["value"] / out["fp64_zero"]["value"]
    return out


def momentum_start_form(w, steps, torch, I):
    """The momentum solve from U^n against the default extrapolated start
    2 U*^n - U*^(n-1), same problem and start (FP64): throughput, BiCGStab
    iterations per component, and the per-step relative L2 difference of the
    two runs' u and p (both meet the same stopping test, eq. (9), first
    line)."""
    from paper_2605_25403_amd.workloads import dofs
    m = I.Mesh.unit_square(w["n"]) if w["dim"] == 2 else I.Mesh.unit_cube(w["n"])
    runs = {}
    for name, ms in (("from_state", I.IPCS_MSTART_STATE),
                     ("extrapolated", I.IPCS_MSTART_EXTRAPOLATED)):
        p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                  tol_corr=w["tol"], momentum_start=ms)
        r = I.Run(m, p, stream=torch.cuda.Stream())
        if w["dim"] == 2:
            r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
        else:
            r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
        runs[name] = r
    lat = {k: [] for k in runs}
    it = {k: [] for k in runs}
    mom = {k: [] for k in runs}
    du, dp = [], []
    for _ in range(steps):
        for name, r in runs.items():
            t0 = time.perf_counter()
            st = r.advance(1)[0]
            lat[name].append(time.perf_counter() - t0)
            it[name].append(max(st["it_mom"][:w["dim"]]))
            mom[name].append(st["ms"][1])
        a, b = runs["from_state"], runs["extrapolated"]
        du.append(float(np.linalg.norm(b.velocity() - a.velocity()) / np.linalg.norm(a.velocity())))
        dp.append(float(np.linalg.norm(b.pressure() - a.pressure()) / np.linalg.norm(a.pressure())))
    nd = dofs(w["dim"], w["n"])
    out = {"steps": steps}
    for name in runs:
        # the first two steps start from U^n in both: medians over the rest
        ms = 1000.0 * float(np.median(lat[name][2:]))
        out[name] = {"value": nd / (ms / 1000.0), "p50_step_ms": ms,
                     "momentum_ms_median": float(np.median(mom[name][2:])),
                     "momentum_iterations": it[name]}
    out["rel_l2_diff_u"] = du
    out["rel_l2_diff_p"] = dp
    out["speedup"] = out["extrapolated"]["value"] / out["from_state"]["value"]
    return out


def scheme_forms(w, steps, torch, I):
    """IPCS with explicit convection (eq. (9) as printed), IPCS with
    semi-implicit convection, and the Chorin-Temam projection, on the same
    problem, start and precision (FP64): throughput, iterations, and each
    one's relative L2 (nodal) distance to the interpolated exact solution after
    `steps` steps."""
    from paper_2605_25403_amd.workloads import dofs
    m = I.Mesh.unit_square(w["n"]) if w["dim"] == 2 else I.Mesh.unit_cube(w["n"])

    def builtin(r):
        if w["dim"] == 2:
            r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
        else:
            r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())

    base = dict(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"], tol_corr=w["tol"])
    variants = {"ipcs_explicit": dict(),
                "ipcs_semi_implicit": dict(convection=I.IPCS_CONV_SEMI_IMPLICIT),
                "chorin": dict(scheme=I.IPCS_SCHEME_CHORIN)}
    runs = {}
    for name, kw in variants.items():
        r = I.Run(m, I.ipcs_params_default(**base, **kw), stream=torch.cuda.Stream())
        builtin(r)
        runs[name] = r
    lat = {k: [] for k in runs}
    it_m = {k: [] for k in runs}
    it_p = {k: [] for k in runs}
    for _ in range(steps):
        for name, r in runs.items():
            t0 = time.perf_counter()
            st = r.advance(1)[0]
            lat[name].append(time.perf_counter() - t0)
            it_m[name].append(max(st["it_mom"][:w["dim"]]))
            it_p[name].append(st["it_p"])
    exact = I.Run(m, I.ipcs_params_default(t0=runs["ipcs_explicit"].time(), **base))
    builtin(exact)
    Ue, Pe = exact.velocity(), exact.pressure()
    nd = dofs(w["dim"], w["n"])
    out = {"steps": steps}
    for name, r in runs.items():
        ms = 1000.0 * float(np.median(lat[name]))
        out[name] = {"value": nd / (ms / 1000.0), "p50_step_ms": ms,
                     "momentum_iterations_median": float(np.median(it_m[name])),
                     "pressure_iterations_median": float(np.median(it_p[name])),
                     "rel_l2_to_exact_u": float(np.linalg.norm(r.velocity() - Ue)
                                                / np.linalg.norm(Ue)),
                     "rel_l2_to_exact_p": float(np.linalg.norm(r.pressure() - Pe)
                                                / np.linalg.norm(Pe))}
    return out


def pair_forms(w, steps, torch, I, dim=2, n=None):
    """The P3-P2 pair against P2-P1 with the same pressure system size: P2-P1
    on n^d cells, P3-P2 on (n/2)^d (both pressure spaces have (n+1)^d nodes).
    2D: Taylor-Green with the workload's k, nu, dt and tolerance; 3D: Beltrami
    (a = pi/4, d = pi/2) with nu = 0.01, dt = 1e-3, tol 1e-12. FP64. Per pair:
    throughput, iterations, per-launch times of the convection assembly and
    the Poisson CG, and the nodal relative L2 distance to the interpolated
    exact solution after `steps` steps."""
    out = {"steps": steps}
    if dim == 2:
        n = n or w["n"]
        kind, prm = I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],)
        base = dict(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"], tol_corr=w["tol"])
        mk = lambda nn, pair: I.Mesh.unit_square(nn, pair=pair)
    else:
        kind, prm = I.IPCS_SOL_BELTRAMI_3D, ()
        base = dict(nu=0.01, dt=1e-3, tol_mom=1e-12, tol_p=1e-12, tol_corr=1e-12)
        mk = lambda nn, pair: I.Mesh.unit_cube(nn, pair=pair)
    out["n"] = n
    for name, pair, nn in (("p2p1", I.IPCS_PAIR_P2P1, n), ("p3p2", I.IPCS_PAIR_P3P2, n // 2)):
        m = mk(nn, pair)
        c = m.counts
        ndof = dim * c.n2 + c.n1
        r = I.Run(m, I.ipcs_params_default(**base), stream=torch.cuda.Stream())
        r.set_builtin(kind, prm)
        lat, it_p = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            st = r.advance(1)[0]
            lat.append(time.perf_counter() - t0)
            it_p.append(st["it_p"])
        ex = I.Run(m, I.ipcs_params_default(t0=r.time(), **base))
        ex.set_builtin(kind, prm)
        Ue, Pe = ex.velocity(), ex.pressure()
        eu = float(np.linalg.norm(r.velocity() - Ue) / np.linalg.norm(Ue))
        ep = float(np.linalg.norm(r.pressure() - Pe) / np.linalg.norm(Pe))
        del ex
        # per-launch kernel times over two more steps (after the errors)
        r.kernel_timing((1 << I.IPCS_NKERNEL) - 1)
        r.advance(2)
        torch.cuda.synchronize()
        kms, kcnt = r.kernel_times()
        r.kernel_timing(0)
        us = lambda k: 1000.0 * kms[k] / kcnt[k] if kcnt[k] else None
        ms = 1000.0 * float(np.median(lat))
        fus = us(I.IPCS_KERNEL_PCG_FUSED_P)
        fgb = kernel_bytes("pcg_fused_p", c, dim, 8) / (fus * 1e-6) / 1e9 if fus else None
        # the cell pass and the local sum where the convection takes two passes
        asm = (us(I.IPCS_KERNEL_ASM_CONV) or 0.0) + (us(I.IPCS_KERNEL_ASM_SUM) or 0.0)
        out[name] = {"n": nn, "dofs": int(ndof), "velocity_dofs_per_component": int(c.n2),
                     "pressure_dofs": int(c.n1), "value": ndof / (ms / 1000.0),
                     "p50_step_ms": ms, "pressure_iterations_median": float(np.median(it_p)),
                     "asm_conv_us": asm,
                     "pcg_fused_p_us": fus, "pcg_fused_p_GBps": fgb,
                     "pcg_fused_p_frac_of_hbm_peak": fgb / PEAK_HBM_GBS if fgb else None,
                     "rel_l2_to_exact_u": eu, "rel_l2_to_exact_p": ep}
        del r
        torch.cuda.empty_cache()
    return out


def seed_forms(w, steps, torch, I, seeds=(0, 1, 2)):
    """The 2D workload for each seed's (k, nu), FP64, same mesh: DOF-steps/s
    over `steps` steps after one warm-up step, and the median over seeds."""
    from paper_2605_25403_amd.workloads import tg_params
    m = I.Mesh.unit_square(w["n"])
    ndof = 2 * m.counts.n2 + m.counts.n1
    out = {"steps": steps}
    vals = []
    for seed in seeds:
        k, nu = tg_params(seed)
        p = I.ipcs_params_default(nu=nu, dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                  tol_corr=w["tol"])
        r = I.Run(m, p, stream=torch.cuda.Stream())
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (k,))
        r.advance(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = [r.advance(1)[0] for _ in range(steps)]
        torch.cuda.synchronize()
        v = ndof * steps / (time.perf_counter() - t0)
        vals.append(v)
        out[f"seed{seed}"] = {"k": k, "nu": nu, "value": v,
                              "momentum_iterations_median":
                                  float(np.median([max(s["it_mom"][:2]) for s in st])),
                              "pressure_iterations_median": float(np.median([s["it_p"] for s in st]))}
        del r
    out["median_value"] = float(np.median(vals))
    return out


def microbench(r, torch, I, c, dim, vsz, p3, reps=5):
    """Stand-alone launches of the velocity SpMV and the convection assembly on
    the run's own data: 20 back to back (warm: the data stays in the caches),
    and single launches after writing a 1 GiB buffer (cold: the Infinity Cache
    holds none of their data), median of reps."""
    names = ["bicg_spmv", "asm_conv"] + (["asm_sum"] if dim == 3 else [])
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    out = {}
    for name in names:
        kid = KERNELS[name][0]
        warm = I.ipcs_profile_kernel(r.h, kid, 20)
        cold = []
        for _ in range(reps):
            flush.fill_(1)
            torch.cuda.synchronize()
            cold.append(I.ipcs_profile_kernel(r.h, kid, 1))
        cold_us = float(np.median(cold))
        b = kernel_bytes(name, c, dim, vsz, p3)
        out[name] = {"bytes": b, "warm_us": warm, "cold_us": cold_us,
                     "warm_GBps": b / (warm * 1e-6) / 1e9, "cold_GBps": b / (cold_us * 1e-6) / 1e9}
    del flush
    return out


def copy_peak(torch, mib=1024, reps=5):
    """Device-to-device copy bandwidth (GB/s, bytes read + written), best of
    reps copies of mib MiB, timed with events on the current stream."""
    src = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = max(best, 2.0 * src.numel() * 8 / (a.elapsed_time(b) * 1e-3) / 1e9)
    del src, dst
    return best


def serving_form(torch, I, count=256, rate=20.0, max_slots=64, seq_sample=16,
                 lanes=((32,), (64,), (128,), (256,))):
    """C5: Poisson-arrival stream of 2D TG requests (n in {32,64,128,256},
    seed-drawn k and nu, 50 steps at dt = 1e-3), mixed form, continuous
    batching in one lane per mesh size (each with its own stream), the same
    lanes with 16 CUs reserved for each of the two small sizes, the same
    lanes serving the plain FP64 form, and the same stream in a single lane
    for comparison. Beside them, the first
    seq_sample requests run one after the other, each alone, in the mixed form
    (the served form's alone latency per mesh size) and in the plain FP64
    form at tolerance 1e-12 (the baseline): per-step latency p50/p99 and
    throughput, and each served result's relative difference from its FP64
    run (nodal L2 and per entry, largest over u and p)."""
    from paper_2605_25403_amd.serve import Server, requests_from
    from paper_2605_25403_amd.workloads import serving_requests
    reqs = requests_from(serving_requests(seed=0, count=count, rate=rate))
    sample = reqs[:seq_sample]
    srv = Server(max_slots=max_slots, lanes=lanes)
    report, res = srv.serve(reqs, keep_ids={q.id for q in sample})
    one, _ = Server(max_slots=max_slots).serve(reqs)
    keys = ("dof_steps_per_s", "p50_step_ms", "p99_step_ms", "step_ms_by_n",
            "queue_delay_p99_ms", "end_to_end_p99_ms", "rounds")
    report["one_lane"] = {k: one[k] for k in keys}
    # the same lanes with CUs reserved for the two small sizes (16 each) and
    # the large lanes on the other CUs
    rsv, _ = Server(max_slots=max_slots, lanes=lanes, lane_cus=(16, 16, None, None)).serve(reqs)
    report["reserved_cus"] = dict({k: rsv[k] for k in keys}, lane_cus=rsv["lane_cus"])
    # the same lanes serving the plain FP64 form (each result bitwise the run
    # alone in FP64, so at the baseline's accuracy)
    f64s, _ = Server(max_slots=max_slots, lanes=lanes, precision=I.IPCS_FP64).serve(reqs)
    report["fp64_served"] = {k: f64s[k] for k in keys}

    def alone(prec):
        base = Server(precision=prec)
        lat, by_n, fields = [], {}, {}
        dsteps, t_all = 0, 0.0
        for q in sample:
            r = base.start_run(q)
            torch.cuda.synchronize()
            for _ in range(q.steps):
                t0 = time.perf_counter()
                r.advance(1)
                dt = time.perf_counter() - t0
                lat.append(dt)
                by_n.setdefault(q.n, []).append(dt)
                t_all += dt
            dsteps += (2 * (2 * q.n + 1) ** 2 + (q.n + 1) ** 2) * q.steps
            fields[q.id] = (r.velocity(), r.pressure())
            del r
        out = {"requests": len(sample), "dof_steps_per_s": dsteps / t_all,
               "p50_step_ms": 1000 * float(np.percentile(lat, 50)),
               "p99_step_ms": 1000 * float(np.percentile(lat, 99)),
               "step_ms_by_n": {str(n): {"p50_step_ms": 1000 * float(np.percentile(v, 50)),
                                         "p99_step_ms": 1000 * float(np.percentile(v, 99))}
                                for n, v in sorted(by_n.items())}}
        return out, fields

    mixed_alone, _ = alone(I.IPCS_MIXED)
    fp64, f64 = alone(I.IPCS_FP64)

    def diff(a, b):
        return max(float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                   float(np.abs(a - b).max() / np.abs(b).max()))

    errs = [max(diff(res[q.id]["U"], f64[q.id][0]), diff(res[q.id]["P"], f64[q.id][1]))
            for q in sample]
    report["sequential_mixed_alone"] = mixed_alone
    report["sequential_fp64_plain"] = fp64
    report["served_vs_fp64_rel_diff"] = {"max": max(errs), "median": float(np.median(errs)),
                                         "requests": len(errs)}
    report["speedup_vs_sequential_fp64"] = report["dof_steps_per_s"] / fp64["dof_steps_per_s"]
    report["workload"] = (f"c5: {count} requests, Poisson arrivals at {rate}/s, 2D TG, "
                          "n in {32,64,128,256}, 50 steps at dt=1e-3, mixed form, "
                          f"max_slots {max_slots}, lanes {[list(l) for l in lanes]}")
    return report


def steady_form(torch, I, sizes=(64, 128)):
    """Steady Navier-Stokes by Newton's method (the Section 4.2 example,
    nu = 1, tol 1e-10) on n x n squares: n = 64 is the largest mesh of the
    paper's table "convergence_data" (33,282 velocity DOFs). Per size: DOFs,
    Newton steps, FGMRES and inner BiCGStab iterations, wall and device time
    of the solve, and DOF-Newton-steps/s."""
    out = {}
    for n in sizes:
        m = I.Mesh.unit_square(n)
        s = I.Steady(m, nu=1.0)
        s.set_builtin(I.IPCS_SOL_STEADY_PAPER_2D)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.solve()
        wall = time.perf_counter() - t0
        c = m.counts
        ndof = 2 * c.n2 + c.n1
        out[str(n)] = {"dofs": int(ndof), "newton_steps": st["newton_steps"],
                       "fgmres_iterations": st["lin_it"], "inner_iterations": st["inner_it"],
                       "wall_ms": 1000.0 * wall, "device_ms": st["ms"],
                       "ms_per_fgmres_iteration": 1000.0 * wall / max(1, st["lin_it"]),
                       "rel_change": st["rel_change"],
                       "dof_newton_steps_per_s": ndof * st["newton_steps"] / wall}
        del s
    return out


def c4_form(torch, I, steps=10, warmup=2):
    """The 3D workload (64^3 cubes x 6 Kuhn tetrahedra, Beltrami a = pi/4,
    d = pi/2, nu = 0.01, dt = 1e-3) in the mixed form and in the plain FP64
    form, from the same start, stepped in lockstep: DOF-steps/s of each over
    `steps` steps after `warmup`, phase medians, the mixed fields' relative
    difference from the FP64 ones per step, and per-launch times of the
    velocity SpMV and the one-kernel Poisson CG (two more steps with
    per-launch events) with their unit bytes and fraction of the HBM peak."""
    from paper_2605_25403_amd.workloads import resolve
    w = resolve("c4")
    m = I.Mesh.unit_cube(w["n"])
    c = m.counts
    ndof = 3 * c.n2 + c.n1
    runs = {}
    for name, prec in (("fp64", I.IPCS_FP64), ("mixed", I.IPCS_MIXED)):
        p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                                  tol_corr=w["tol"], tol_ir=1e-10, precision=prec)
        r = I.Run(m, p, stream=torch.cuda.Stream())
        r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
        runs[name] = r
    for _ in range(warmup):
        for r in runs.values():
            r.advance(1)
    lat = {k: [] for k in runs}
    ph = {k: [] for k in runs}
    it_p = {k: [] for k in runs}
    du, dp = [], []
    for step in range(steps):
        for name, r in runs.items():
            t0 = time.perf_counter()
            st = r.advance(1)[0]
            lat[name].append(time.perf_counter() - t0)
            ph[name].append(st["ms"])
            it_p[name].append(st["it_p"])
        if step in (0, steps // 2, steps - 1):
            U64, U32 = runs["fp64"].velocity(), runs["mixed"].velocity()
            P64, P32 = runs["fp64"].pressure(), runs["mixed"].pressure()
            du.append(float(np.linalg.norm(U32 - U64) / np.linalg.norm(U64)))
            dp.append(float(np.linalg.norm(P32 - P64) / np.linalg.norm(P64)))
    out = {"workload": "c4: 3D P2-P1 IPCS, unit cube 64^3 (1572864 tets), Beltrami, dt=1e-3, "
                       "tol=1e-12 (mixed: refinement of the Poisson solve to 1e-10)",
           "dofs": ndof, "steps": steps, "warmup": warmup,
           "rel_l2_diff_mixed_vs_fp64_u": du, "rel_l2_diff_mixed_vs_fp64_p": dp,
           "diff_steps": [0, steps // 2, steps - 1]}
    for name, r in runs.items():
        vb = 4 if name == "mixed" else 8
        tot = float(np.sum(lat[name]))
        a = np.array(ph[name])
        r.kernel_timing((1 << I.IPCS_NKERNEL) - 1)
        r.advance(2)
        torch.cuda.synchronize()
        kms, kcnt = r.kernel_times()
        r.kernel_timing(0)
        kern = {}
        for kname in ("bicg_spmv", "bicg_spmv_t", "pcg_fused_p", "asm_conv", "asm_sum"):
            kid = KERNELS[kname][0]
            if kcnt[kid] == 0:
                continue
            us = 1000.0 * kms[kid] / kcnt[kid]
            ub = unit_bytes(kname, c, 3, vb)
            b = ub if ub is not None else kernel_bytes(kname, c, 3, vb)
            kern[kname] = {"us_per_launch": us, "bytes": b, "GBps": b / (us * 1e-6) / 1e9,
                           "frac_of_hbm_peak": b / (us * 1e-6) / 1e9 / PEAK_HBM_GBS,
                           "launches_per_step": kcnt[kid] / 2.0}
        out[name] = {"value": ndof * steps / tot, "ms_per_step": 1000.0 * tot / steps,
                     "p50_step_ms": 1000.0 * float(np.percentile(lat[name], 50)),
                     "p99_step_ms": 1000.0 * float(np.percentile(lat[name], 99)),
                     "phase_ms_median": {k: float(np.median(a[:, i])) for i, k in
                                         enumerate(("asm", "momentum", "pressure", "correction"))},
                     "pressure_iterations_median": float(np.median(it_p[name])),
                     "kernels": kern}
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    del runs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--poisson-s", type=int, default=0,
                    help="CG iterations per launch of the one-kernel Poisson CG (0: default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=5,
                    help="steps after the timed region with per-launch kernel timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="end with a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarize two rocprofv3 --pmc runs and exit (no GPU use)")
    ap.add_argument("--pmc-kernel", default="pcg_update_p")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision and serving form reports")
    ap.add_argument("--form-steps", type=int, default=10)
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="summarize a rocprofv3 --kernel-trace --stats -f csv run and exit")
    ap.add_argument("--pmc-command", default="")
    ap.add_argument("--counters-summary", nargs="+", metavar="DIR",
                    help="summarize rocprofv3 --pmc runs of one kernel (see --counters-kernel) "
                         "and exit (no GPU use)")
    ap.add_argument("--counters-kernel", nargs=2, metavar=("NAME", "REGEX"))
    args = ap.parse_args()
    if args.counters_summary:
        counters_summary(args.counters_summary, args.counters_kernel[1], args.counters_kernel[0],
                         args.workload, args.pmc_command)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.workload, args.pmc_command)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_kernel, args.workload,
                    args.calibrate_copy or 256, args.pmc_command)
        return
    if args.gpus != 1:
        print(f"bench.py: the IPCS step runs on one GPU; --gpus {args.gpus} is not "
              "supported (the solver is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_25403_amd import ipcs as I
    from paper_2605_25403_amd.workloads import dofs, resolve

    w = resolve(args.workload)
    steps = args.steps if args.steps is not None else w["steps"]
    dim, n = w["dim"], w["n"]
    mixed = w["precision"] == "mixed"
    p3 = w.get("pair", 0) == I.IPCS_PAIR_P3P2
    m = I.Mesh.unit_square(n, pair=w.get("pair", 0)) if dim == 2 else I.Mesh.unit_cube(n)
    p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=w["tol"], tol_p=w["tol"],
                              tol_corr=w["tol"],
                              precision=I.IPCS_MIXED if mixed else I.IPCS_FP64,
                              poisson_s=args.poisson_s)
    stream = torch.cuda.Stream()
    r = I.Run(m, p, stream=stream)
    if dim == 2:
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
    else:
        r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
    ndof = dim * m.counts.n2 + m.counts.n1      # velocity components and pressure

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

    # per-kernel durations: every launch of every kernel bracketed by HIP events
    # on the run's stream, in the normal launch sequence of kernel_steps more steps
    c = m.counts
    it_p = float(np.median([s["it_p"] for s in stats]))
    it_m = float(np.median([max(s["it_mom"][:dim]) for s in stats]))
    it_c = float(np.median([max(s["it_corr"][:dim]) for s in stats]))
    # CG iterations per launch of the one-kernel Poisson CG (two for s-step
    # CG): the byte models count that many iterations per launch
    ipl = 2 if args.poisson_s == 2 else 1
    r.kernel_timing((1 << I.IPCS_NKERNEL) - 1 if args.kernel_steps > 0 else 0)
    kstats = [r.advance(1)[0] for _ in range(args.kernel_steps)]
    torch.cuda.synchronize()
    kms, kcnt = r.kernel_times()
    r.kernel_timing(0)
    ksteps = max(1, args.kernel_steps)
    kern = {}
    for name, (kid, _) in KERNELS.items():
        if kcnt[kid] == 0:
            continue
        us = 1000.0 * kms[kid] / kcnt[kid]
        b = kernel_bytes(name, c, dim, 4 if mixed else 8, p3)
        if name == "pcg_fused_p":
            b *= ipl
        kern[name] = {"us_per_launch": us, "bytes": b, "GBps": b / (us * 1e-6) / 1e9,
                      "launches_per_step": kcnt[kid] / ksteps,
                      "ms_per_step": kms[kid] / ksteps}
    roof = None
    if kern:
        dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
        vb = 4 if mixed else 8
        ub = unit_bytes(dom, c, dim, vb)
        if ub is not None and dom == "pcg_fused_p":
            ub *= ipl
        us = kern[dom]["us_per_launch"]
        b = ub if ub is not None else kern[dom]["bytes"]
        ach = b / (us * 1e-6) / 1e9
        rp = rocprof_avg_us(dom, args.workload)
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                "traffic": measured_traffic(dom, args.workload),
                "algorithmic_bytes_per_launch": b,
                "bytes_model": "unit" if ub is not None else "kernel",
                "kernel_bytes_per_launch": kern[dom]["bytes"],
                "us_per_launch": us,
                "rocprof_us_per_launch": rp,
                "frac_at_rocprof_us": (b / (rp * 1e-6) / 1e9 / PEAK_HBM_GBS) if rp else None}

    log(f"timed region done ({steps} steps), kernel timing done")
    micro = microbench(r, torch, I, c, dim, 4 if mixed else 8, p3)
    log("microbenchmarks done")
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
        "config": {"workload": f"{args.workload}: {dim}D {'P3-P2' if p3 else 'P2-P1'} IPCS "
                               f"{'mixed' if mixed else 'FP64 plain'}, "
                               f"unit {'square' if dim == 2 else 'cube'} {n}^{dim} "
                               f"({c.nc} cells), {'TG' if dim == 2 else 'Beltrami'} "
                               f"manufactured solution, dt={w['dt']}, tol={w['tol']}",
                   "dofs": ndof, "N2": c.n2, "N1": c.n1, "nnz_p2p2": c.nnz[0],
                   "k": w.get("k"), "nu": w["nu"], "dt": w["dt"], "seed": w.get("seed")},
        "roofline": roof,
        "kernels": kern,
        # iterations of the kernel-timed steps (the launches_per_step above
        # count launches of the same steps: their excess over these is the
        # polling overrun)
        "kernel_steps_iterations_mean": None if not kstats else {
            "momentum": float(np.mean([max(k["it_mom"][:dim]) for k in kstats])),
            "pressure": float(np.mean([k["it_p"] for k in kstats])),
            "correction": float(np.mean([max(k["it_corr"][:dim]) for k in kstats]))},
        "phase_ms_median": {"asm": float(np.median(ph[:, 0])), "momentum": float(np.median(ph[:, 1])),
                            "pressure": float(np.median(ph[:, 2])),
                            "correction": float(np.median(ph[:, 3]))},
        "phase_ms_p90": {"asm": float(np.percentile(ph[:, 0], 90)),
                         "momentum": float(np.percentile(ph[:, 1], 90)),
                         "pressure": float(np.percentile(ph[:, 2], 90)),
                         "correction": float(np.percentile(ph[:, 3], 90))},
        "iterations_median": {"momentum": it_m, "pressure": it_p, "correction": it_c},
        "microbench": micro,
    }
    if not args.no_forms and not mixed and not p3:
        out["forms"] = {}
        for name, fn in (("mixed", lambda: mixed_form(w, args.form_steps, torch, I)),
                         ("poisson_start", lambda: start_form(w, args.form_steps, torch, I)),
                         ("momentum_start",
                          lambda: momentum_start_form(w, args.form_steps, torch, I)),
                         ("schemes", lambda: scheme_forms(w, args.form_steps, torch, I)),
                         ("serving", lambda: serving_form(torch, I)),
                         ("c4", lambda: c4_form(torch, I)),
                         ("steady", lambda: steady_form(torch, I)),
                         ("pairs", lambda: pair_forms(w, args.form_steps, torch, I)),
                         ("pairs_3d", lambda: pair_forms(w, args.form_steps, torch, I, 3, 32)),
                         ("seeds", lambda: seed_forms(w, 20, torch, I))):
            if name in ("pairs", "pairs_3d", "seeds") and w["dim"] != 2:
                continue
            out["forms"][name] = fn()
            torch.cuda.empty_cache()
            log(f"form {name} done")
    if roof is not None:
        # the measured device copy rate beside the published peak
        roof["copy_GBps"] = copy_peak(torch)
        roof["frac_of_copy"] = roof["achieved"] / roof["copy_GBps"]
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        log("cpu baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
