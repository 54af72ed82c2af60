#!/usr/bin/env python3
"""Benchmark of the batched Galerkin assembly hot path on one MI355X.

Workload: 3D Poisson with P1 tetrahedra on the unit cube, 64^3 grid, 6 Kuhn
tets per cube (1,572,864 elements, 274,625 vertices), interior vertices
jittered by U(-0.15h, 0.15h), a = exp(N(0,1)) and f = U(-1,1) per element
(seed 0, synthetic).  One step = the whole hot path on resident inputs:
FP64 assembly of K and F (one fused Map+Reduce kernel), Dirichlet elimination
on all faces, and Jacobi-PCG to a relative residual of 1e-8.  The CSR
pattern and routing are built once, before the timed region (timed apart).

Before each step's assembly a 1 GiB read-modify-write of a scratch buffer
evicts the 256 MB Infinity Cache, so the assembly reads its inputs from HBM
(the "cold" protocol); warm numbers are reported beside it.

Prints ONE JSON line.  `value` is assembled elements/s of the FP64 assembly
kernel (mean duration over the timed steps, measured with HIP events on its
stream); `ms_per_step` is the wall time of one whole step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one FP64 CG iteration on the 64^3 Poisson system (274,625 rows, 4,018,753 nonzeros):
# the SpMV's values and column indices once (48.2 MB), row pointers, and about ten FP64 vector passes
PCG_ITER_BYTES_64 = 75.7e6
METRIC = "assembled elements/s + HBM GB/s (FP64 vs FP32); p50/p99 assemble+solve latency"


def source_hash() -> str:
    """Hash of the device code and of the pattern builder (which fixes blocks and routing); a stored
    counter measurement is used only while it matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2602_05052_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")) or f == "tg_pattern.cpp":
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def stats_us(t):
    """mean / median / p90 of a sample of durations in seconds, in microseconds."""
    import numpy as np
    return {"mean": float(np.mean(t)) * 1e6, "p50": float(np.median(t)) * 1e6,
            "p90": float(np.percentile(t, 90)) * 1e6, "samples": int(len(t))}


def kernel_key(name: str) -> str:
    """'void tg::(anonymous namespace)::p1_assemble_kernel<3, double, 0, true, false>(...)' ->
    'p1_assemble_kernel<3,double,0,true,false>'."""
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("tg::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += (ch == "<") - (ch == ">")
        if ch == "(" and depth == 0:
            name = name[:i]
            break
    return name.replace(" ", "")


def traffic_from_pmc(fetch_csv: str, write_csv: str, out_json: str, workload: str,
                     copy_kernel: str = "CUDAFunctorOnSelf_add"):
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) of one
    workload, each scaled so that the 1 GiB read-modify-write `add_` of the cold protocol reads 1 GiB and
    writes 1 GiB; stored under "<workload>:<kernel>" (a kernel's traffic depends on the mesh it ran on)."""
    import csv
    from collections import defaultdict

    def load(path, counter):
        per = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return per

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    cal_f = [v for k, vs in fetch.items() if copy_kernel in k for v in vs]
    cal_w = [v for k, vs in write.items() if copy_kernel in k for v in vs]
    if cal_f and cal_w:
        fs, ws = gib_kib / (sum(cal_f) / len(cal_f)), gib_kib / (sum(cal_w) / len(cal_w))
        rec = {"_calibration": {"kernel": copy_kernel, "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                                "fetch_kib": sum(cal_f) / len(cal_f), "write_kib": sum(cal_w) / len(cal_w),
                                "fetch_scale": fs, "write_scale": ws}}
    else:  # a workload without the 1 GiB copy: the stored calibration (same counters, same GPU model)
        with open(out_json) as fh:
            cal = json.load(fh)["_calibration"]
        fs, ws = cal["fetch_scale"], cal["write_scale"]
        rec = {}
    for name in fetch:
        if copy_kernel in name or name not in write or "tg::" not in name:
            continue
        f = sum(fetch[name]) / len(fetch[name])
        w = sum(write[name]) / len(write[name])
        rec[f"{workload}:{kernel_key(name)}"] = {"source_hash": source_hash(), "fetch_kib_raw": f, "write_kib_raw": w,
                                 "fetch_scale": fs, "write_scale": ws,
                                 "bytes_per_launch": int(round((f * fs + w * ws) * 1024)),
                                 "dispatches": len(fetch[name])}
    try:  # merge into the stored measurements (other workloads' kernels stay; this workload's are replaced)
        with open(out_json) as fh:
            old = json.load(fh)
    except (OSError, ValueError):
        old = {}
    old = {k: v for k, v in old.items() if not k.startswith(workload + ":")}
    old.update(rec)
    with open(out_json, "w") as fh:
        json.dump(old, fh, indent=1, sort_keys=True)
    return rec


def stored_traffic(kernel: str, workload: str = "poisson3d"):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(f"{workload}:{kernel}")
    if not ent or ent.get("source_hash") != source_hash():
        return None
    return ent.get("bytes_per_launch")


def normwise_err(v, ref, row_ptr):
    """||v - ref||_inf / ||ref||_inf for CSR values (max absolute row sum) or vectors (row_ptr None)."""
    import numpy as np
    v = np.asarray(v, dtype=np.float64)
    if row_ptr is None:
        return float(np.abs(v - ref).max() / max(np.abs(ref).max(), 1e-300))
    row = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    return float(np.bincount(row, np.abs(v - ref)).max() / max(np.bincount(row, np.abs(ref)).max(), 1e-300))


def cpu_threads() -> int:
    """The host threads the multi-core CPU baseline uses (OMP_NUM_THREADS, else the CPUs this process may use)."""
    try:
        return max(1, int(os.environ["OMP_NUM_THREADS"]))
    except (KeyError, ValueError):
        return len(os.sched_getaffinity(0))


def p1_bytes(nv, dim, E, nnz, ndof, s, n_coef):
    """Algorithmic bytes of one P1 assembly call: inputs and outputs (b_min) plus the routing (b_alg)."""
    k = dim + 1
    b_min = nv * dim * 8 + E * k * 4 + E * n_coef * s + nnz * s + ndof * s
    routing = E * k * k * 4 + (nnz + 1) * 4 + E * k * 4 + (nv + 1) * 4
    return b_min, b_min + routing


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=64, help="grid cells per axis (64 = the benchmark mesh)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle timing sample")
    ap.add_argument("--samples", type=int, default=100,
                    help="latency samples and side-measurement repeats (fewer for profiler runs)")
    ap.add_argument("--workload", choices=["poisson3d", "elasticity", "heat", "batched", "serve", "c1"],
                    default="poisson3d",
                    help="poisson3d: the benchmark line; elasticity: P2 32^3 assembly-only timing; heat: "
                         "differentiable 2D heat rollout 256^2 (forward + adjoint gradient); batched: B "
                         "coefficient sets on the 64^3 pattern in one launch; serve: a stream of assemble+solve "
                         "requests through the continuous-batching server; c1: the 2D P1 64^2 assembly latency")
    ap.add_argument("--batch", type=int, default=8, help="coefficient sets for --workload batched")
    ap.add_argument("--requests", type=int, default=64, help="requests for --workload serve")
    ap.add_argument("--slots", type=int, default=16, help="slots per group for --workload serve")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="request arrivals per second for --workload serve (0: 0.5x and 0.8x of saturation)")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="server HBM budget for --workload serve")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="merge into profiles/traffic.json the traffic of two rocprofv3 --pmc runs of this script "
                         "(of --workload) and exit")
    args = ap.parse_args()
    if args.traffic_from:
        rec = traffic_from_pmc(*args.traffic_from, os.path.join(ROOT, "profiles", "traffic.json"), args.workload)
        for k, v in sorted(rec.items()):
            if not k.startswith("_"):
                print(f"| `{k}` | {v['dispatches']} | {v['fetch_kib_raw']:.1f} | {v['write_kib_raw']:.1f} | "
                      f"{v['bytes_per_launch'] / 1e6:.1f} MB |")
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            print(json.dumps(json.load(fh)["_calibration"]))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the path would shard by row blocks across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    import paper_2602_05052_amd as tg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.workload == "elasticity":
        return run_elasticity(args, dev)
    if args.workload == "heat":
        return run_heat(args, dev)
    if args.workload == "batched":
        return run_batched(args, dev)
    if args.workload == "serve":
        return run_serve(args, dev)
    if args.workload == "c1":
        s = torch.cuda.Stream(device=dev)
        print(json.dumps(measure_c1(dev, s, torch.zeros(1 << 28, dtype=torch.float32, device=dev),
                                    cpu=not args.no_cpu_baseline, reps=args.samples)))
        return

    # ---------------------------------------------------------------- inputs (resident in HBM)
    d = meshgen.poisson_inputs(3, args.n, seed=0)
    E, nv = d["conn"].shape[0], d["coords"].shape[0]
    t0 = time.perf_counter()
    pat = tg.Pattern(d["conn"], nv)
    pattern_s = time.perf_counter() - t0
    coords = torch.from_numpy(d["coords"]).to(dev)
    a64 = torch.from_numpy(d["a"]).to(dev)
    f64 = torch.from_numpy(d["f"]).to(dev)
    a32, f32 = a64.float(), f64.float()
    vals = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
    rhs = torch.empty(pat.n_dofs, dtype=torch.float64, device=dev)
    vals32 = torch.empty(pat.nnz, dtype=torch.float32, device=dev)
    rhs32 = torch.empty(pat.n_dofs, dtype=torch.float32, device=dev)
    x = torch.empty(pat.n_dofs, dtype=torch.float64, device=dev)
    flush = torch.zeros(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
    s = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()

    def assemble64():
        tg.assemble(pat, tg.LAPLACE, coords, a64, f64, values=vals, rhs=rhs, stream=s)

    def assemble32():
        tg.assemble(pat, tg.LAPLACE, coords, a32, f32, values=vals32, rhs=rhs32, stream=s)

    # ---------------------------------------------------------------- timed steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    iters, relres = [], []
    print(f"# bench: E={E} nnz={pat.nnz} dofs={pat.n_dofs}; warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
          flush=True)
    with torch.cuda.stream(s):
        for w in range(args.warmup):
            flush.add_(1.0)
            assemble64()
            tg.apply_dirichlet(pat, vals, rhs, stream=s)
            tg.pcg(pat, vals, rhs, rtol=args.rtol, x=x, stream=s, check_every=25)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        for k in range(args.steps):
            flush.add_(1.0)
            ev[k][0].record(s)
            assemble64()
            ev[k][1].record(s)
            tg.apply_dirichlet(pat, vals, rhs, stream=s)
            _, it, rr = tg.pcg(pat, vals, rhs, rtol=args.rtol, x=x, stream=s, check_every=25)
            ev[k][2].record(s)
            iters.append(it)
            relres.append(rr)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
    print(f"# timed steps done: {wall:.3f} s", file=sys.stderr, flush=True)
    t_asm = np.array([e[0].elapsed_time(e[1]) for e in ev]) * 1e-3  # s
    t_step = np.array([e[0].elapsed_time(e[2]) for e in ev]) * 1e-3
    t_solve = t_step - t_asm

    # ---------------------------------------------------------------- side legs (outside the timed region)
    def time_kernel(fn, reps, cold):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        with torch.cuda.stream(s):
            fn()
            for e0, e1 in evs:
                if cold:
                    flush.add_(1.0)
                e0.record(s)
                fn()
                e1.record(s)
        torch.cuda.synchronize()
        return np.array([e0.elapsed_time(e1) for e0, e1 in evs]) * 1e-3

    t64_warm = time_kernel(assemble64, max(2, args.samples // 2), cold=False)
    t32_cold = time_kernel(assemble32, max(2, args.samples // 2), cold=True)
    t32_warm = time_kernel(assemble32, max(2, args.samples // 2), cold=False)
    # attainable HBM bandwidth: the 1 GiB read-modify-write of the flush (2 GiB moved per launch)
    t_copy = time_kernel(lambda: flush.add_(1.0), 10, cold=False)
    attainable_gbs = 2.0 * flush.numel() * 4 / float(np.median(t_copy)) / 1e9
    # assemble + Dirichlet + solve latency over at least 100 repeats (after the timed steps; p99 needs the
    # samples), the cold flush before each as in the timed steps
    n_lat = max(args.samples, args.steps)
    lat_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n_lat)]
    with torch.cuda.stream(s):
        for e0, e1 in lat_ev:
            flush.add_(1.0)
            e0.record(s)
            assemble64()
            tg.apply_dirichlet(pat, vals, rhs, stream=s)
            tg.pcg(pat, vals, rhs, rtol=args.rtol, x=x, stream=s, check_every=25)
            e1.record(s)
    torch.cuda.synchronize()
    t_lat = np.array([a.elapsed_time(b) for a, b in lat_ev]) * 1e-3
    c1 = measure_c1(dev, s, flush, cpu=not args.no_cpu_baseline, reps=args.samples)
    # the CG iteration kernel (the step's dominant kernel): its time per launch from two fixed-length solves
    # (50 and 250 iterations, unreachable rtol, the same chunks of launches as the timed solves), differenced
    # so that the setup kernels cancel; HIP events on the solver's stream
    it_lo, it_hi = 50, 250
    t_it = {it_lo: [], it_hi: []}
    with torch.cuda.stream(s):
        for rep in range(4 if args.samples >= 20 else 2):
            for n_it in (it_lo, it_hi):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                tg.pcg(pat, vals, rhs, rtol=1e-30, max_iter=n_it, x=x, stream=s, check_every=25,
                       raise_on_noconv=False)
                e1.record(s)
                torch.cuda.synchronize()
                if rep:
                    t_it[n_it].append(e0.elapsed_time(e1) * 1e-3)
    t_iter = (float(np.median(t_it[it_hi])) - float(np.median(t_it[it_lo]))) / (it_hi - it_lo)
    # the FP32 system: Dirichlet + Jacobi-PCG to 1e-6 (true residual), beside the FP64 one
    t32 = []
    with torch.cuda.stream(s):
        x32 = torch.empty(pat.n_dofs, dtype=torch.float32, device=dev)
        for rep in range(3):
            assemble32()
            tg.apply_dirichlet(pat, vals32, rhs32, stream=s)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            _, it32, rr32, st32 = tg.pcg(pat, vals32, rhs32, rtol=1e-6, x=x32, stream=s, check_every=25,
                                         raise_on_noconv=False, return_status=True)
            e1.record(s)
            torch.cuda.synchronize()
            t32.append(e0.elapsed_time(e1) * 1e-3)
    solve32 = {"rtol": 1e-6, "pcg_iterations": int(it32), "relres": float(rr32), "status": tg._STATUS_NAMES[st32],
               "solve_ms_p50": float(np.median(t32)) * 1e3, "us_per_iteration": float(np.median(t32)) / it32 * 1e6}
    # bitwise repeatability of the FP64 assembly (two fresh assemblies; the loops above leave Dirichlet-
    # eliminated values behind)
    assemble64()
    torch.cuda.synchronize()
    ref_vals, ref_rhs = vals.clone(), rhs.clone()
    assemble64()
    torch.cuda.synchronize()
    bitwise = bool(torch.equal(ref_vals, vals) and torch.equal(ref_rhs, rhs))

    bmin64, balg64 = p1_bytes(nv, 3, E, pat.nnz, pat.n_dofs, 8, 2)
    bmin32, balg32 = p1_bytes(nv, 3, E, pat.nnz, pat.n_dofs, 4, 2)
    mean_asm = float(t_asm.mean())
    gbs = balg64 / mean_asm / 1e9
    routing = "true" if pat.compact_routing() is not None else "false"  # the kernel instance the pattern selects
    traffic = stored_traffic(f"p1_assemble_kernel<3,double,0,true,false,{routing}>")
    # the CG iteration instance the pattern selects (16-bit column offsets or 32-bit columns)
    pcg_kernel = f"pcg_iter_kernel<double,false,true,{'short' if pat.sell_index_bytes == 2 else 'int'}>"

    out = {
        "metric": METRIC,
        "value": E / mean_asm,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Poisson P1 tets, unit cube {args.n}^3 x 6 Kuhn tets, jitter 0.15h, a=exp(N(0,1)), "
                        f"f=U(-1,1), seed 0; FP64 assembly + Dirichlet on all faces + Jacobi-PCG to {args.rtol:g}",
            "elements": E, "vertices": nv, "nnz": pat.nnz, "dofs": pat.n_dofs,
            "constrained_dofs": pat.n_constrained, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "kernel": pcg_kernel + " (one CG iteration; the step's dominant "
                                                   "kernel: iterations x time per launch is most of ms_per_step)",
            "achieved": PCG_ITER_BYTES_64 / t_iter / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": PCG_ITER_BYTES_64 / t_iter / 1e9 / HBM_PEAK_GBS,
            "traffic": stored_traffic(pcg_kernel),
            "traffic_gbs": (stored_traffic(pcg_kernel) / t_iter / 1e9) if stored_traffic(pcg_kernel) else None,
            "algorithmic_bytes_per_launch": PCG_ITER_BYTES_64, "us_per_launch": t_iter * 1e6,
            "launches_per_step": int(np.median(iters)),
            "attainable_gbs": attainable_gbs,
        },
        "roofline_assembly": {
            "bound": "hbm", "kernel": "p1_assemble_kernel<3,double,laplace> (the assembly: value = its elements/s)",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_gbs": (traffic / mean_asm / 1e9) if traffic else None,
            "algorithmic_bytes_per_launch": balg64, "bytes_per_element": balg64 / E,
            "b_min_bytes_per_launch": bmin64,
            "attainable_gbs": attainable_gbs, "frac_of_attainable": gbs / attainable_gbs,
        },
        "assembly": {
            "fp64_cold_us": stats_us(t_asm),
            "fp64_warm_us": stats_us(t64_warm),
            "fp32_cold_us": stats_us(t32_cold),
            "fp32_warm_us": stats_us(t32_warm),
            "fp64_elements_per_s": E / mean_asm,
            "fp32_elements_per_s": E / float(t32_cold.mean()),
            "fp64_gbs_b_alg": gbs, "fp32_gbs_b_alg": balg32 / float(t32_cold.mean()) / 1e9,
            "fp64_gbs_b_min": bmin64 / mean_asm / 1e9, "fp32_gbs_b_min": bmin32 / float(t32_cold.mean()) / 1e9,
            "bitwise_repeatable": bitwise,
            "pattern_build_s": pattern_s,
        },
        "solve": {
            "pcg_iterations": int(np.median(iters)), "relres_max": float(max(relres)),
            "solve_ms_p50": float(np.median(t_solve)) * 1e3,
            "us_per_iteration": float(np.median(t_solve) / max(1, np.median(iters))) * 1e6,
            "fp32": solve32,
        },
        "latency_ms": {"assemble_solve_p50": float(np.percentile(t_lat, 50)) * 1e3,
                       "assemble_solve_p99": float(np.percentile(t_lat, 99)) * 1e3,
                       "samples": int(len(t_lat)),
                       "timed_steps_p50": float(np.percentile(t_step, 50)) * 1e3},
        "c1_2d_64": c1,
    }

    # ---------------------------------------------------------------- CPU baseline (the oracle, as it stands)
    if not args.no_cpu_baseline:
        import oracle

        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        rp, ci = oracle.csr_pattern(nv, d["conn"])
        inc_ptr, inc = oracle.p1_incidence(nv, d["conn"])
        threads = cpu_threads()
        budget = args.cpu_seconds / 2

        def timed(fn):
            calls, t_cpu, res = 0, 0.0, None
            while t_cpu < budget or calls < 2:
                c0 = time.perf_counter()
                res = fn()
                t_cpu += time.perf_counter() - c0
                calls += 1
            return calls, t_cpu, res

        calls1, t1, (ovals, orhs) = timed(lambda: oracle.assemble_p1_values(d["coords"], d["conn"], d["a"], d["f"],
                                                                            rp, ci))
        callsp, tp, (pvals, prhs) = timed(lambda: oracle.assemble_p1_values_parallel(
            d["coords"], d["conn"], d["a"], d["f"], rp, ci, inc_ptr, inc, threads))
        out["cpu_baseline"] = {
            "value": callsp * E / tp, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"{callsp} full value+load assemblies of the same {E}-element mesh by the FP64 C oracle on "
                      f"{threads} threads (OpenMP element Map, then per-row sums in ascending element order: "
                      f"bitwise the serial result), {tp:.1f} s; CSR pattern and incidence prebuilt, not timed",
            "serial_value": calls1 * E / t1, "serial_cores": 1,
            "serial_sample": f"{calls1} assemblies by the serial element loop, {t1:.1f} s",
            "parallel_bitwise_equal_serial": bool(np.array_equal(pvals, ovals) and np.array_equal(prhs, orhs)),
            "cpu": _cpu_model(),
        }
        # error of the GPU results against the oracle (normwise, max abs row sum)
        tg.assemble(pat, tg.LAPLACE, coords, a64, f64, values=vals, rhs=rhs)
        assemble32()
        torch.cuda.synchronize()
        row = np.repeat(np.arange(pat.n_dofs), np.diff(rp))
        den = np.bincount(row, np.abs(ovals)).max()
        for name, v in (("fp64", vals), ("fp32", vals32)):
            diff = np.abs(v.double().cpu().numpy() - ovals)
            out["assembly"][f"{name}_err_vs_oracle"] = float(np.bincount(row, diff).max() / den)

    print(json.dumps(out))


def measure_c1(dev, s, flush, cpu=True, reps=100):
    """The 2D P1 Poisson config on 64^2 x 2 triangles (8,192 elements), FP64: assembly latency (cold and
    warm, HIP events on the stream), launch-bound; error against the oracle."""
    import numpy as np
    import torch

    import meshgen
    import paper_2602_05052_amd as tg

    d = meshgen.poisson_inputs(2, 64, seed=0)
    E, nv = d["conn"].shape[0], d["coords"].shape[0]
    pat = tg.Pattern(d["conn"], nv)
    coords = torch.from_numpy(d["coords"]).to(dev)
    a, f = torch.from_numpy(d["a"]).to(dev), torch.from_numpy(d["f"]).to(dev)
    vals = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
    rhs = torch.empty(pat.n_dofs, dtype=torch.float64, device=dev)
    res = {}
    for cold in (True, False):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        with torch.cuda.stream(s):
            for _ in range(5):
                tg.assemble(pat, tg.LAPLACE, coords, a, f, values=vals, rhs=rhs, stream=s)
            if not cold:  # a few ms of GPU spin first, so the host queues every launch before the GPU reaches it
                torch.cuda._sleep(20_000_000)
            for e0, e1 in evs:
                if cold:
                    flush.add_(1.0)
                e0.record(s)
                tg.assemble(pat, tg.LAPLACE, coords, a, f, values=vals, rhs=rhs, stream=s)
                e1.record(s)
        torch.cuda.synchronize()
        res["cold_us" if cold else "warm_us"] = stats_us(np.array([x.elapsed_time(y) for x, y in evs]) * 1e-3)
    bmin, balg = p1_bytes(nv, 2, E, pat.nnz, pat.n_dofs, 8, 2)
    out = {"workload": "2D Poisson P1, 64^2 x 2 triangles (8192 elements, 4225 vertices), jitter 0.2h, "
                       "a=exp(N(0,1)), f=U(-1,1), seed 0, FP64 assembly", "elements": E, "nnz": pat.nnz,
           "b_alg_bytes": balg, "elements_per_s_warm": E / (res["warm_us"]["p50"] * 1e-6), **res}
    if cpu:
        import oracle
        A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
        rp, ci = pat.csr()
        assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_idx)
        out["err_vs_oracle"] = {"values": normwise_err(vals.cpu().numpy(), A.vals, A.row_ptr),
                                "rhs": normwise_err(rhs.cpu().numpy(), A.rhs, None)}
    return out


def p2_bytes(nv, E, nnz, ndof, n_nodes, s):
    """Algorithmic bytes of one P2 elasticity call (routing counted on 3x3 node-pair blocks)."""
    b_min = nv * 3 * 8 + E * 4 * 4 + E * 5 * s + nnz * s + ndof * s
    nnz_b = nnz // 9
    routing = E * 100 * 4 + (nnz_b + 1) * 4 + E * 10 * 4 + (n_nodes + 1) * 4
    return b_min, b_min + routing


def run_elasticity(args, dev):
    """P2 elasticity, 32^3 x 6 tets: FP64 and FP32 assembly (cold and warm), assembly only."""
    import numpy as np
    import torch

    import meshgen
    import paper_2602_05052_amd as tg

    n = 32 if args.n == 64 else args.n
    d = meshgen.elasticity_inputs(n, seed=0)
    E, nv = d["conn"].shape[0], d["coords"].shape[0]
    t0 = time.perf_counter()
    pat = tg.Pattern(d["conn"], nv, order=2, ncomp=3)
    pattern_s = time.perf_counter() - t0
    coords = torch.from_numpy(d["coords"]).to(dev)
    flush = torch.zeros(1 << 28, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream(device=dev)
    res = {}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        coef = torch.from_numpy(np.stack([d["lam"], d["mu"]])).to(dt).to(dev)
        load = torch.from_numpy(d["b"]).to(dt).to(dev)
        vals = torch.empty(pat.nnz, dtype=dt, device=dev)
        rhs = torch.empty(pat.n_dofs, dtype=dt, device=dev)
        for cold in (True, False):
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            with torch.cuda.stream(s):
                for _ in range(args.warmup):
                    tg.assemble(pat, tg.ELASTICITY, coords, coef, load, values=vals, rhs=rhs, stream=s)
                for e0, e1 in evs:
                    if cold:
                        flush.add_(1.0)
                    e0.record(s)
                    tg.assemble(pat, tg.ELASTICITY, coords, coef, load, values=vals, rhs=rhs, stream=s)
                    e1.record(s)
            torch.cuda.synchronize()
            t = np.array([a.elapsed_time(b) for a, b in evs]) * 1e-3
            bmin, balg = p2_bytes(nv, E, pat.nnz, pat.n_dofs, pat.n_nodes, 8 if dt == torch.float64 else 4)
            res[f"{name}_{'cold' if cold else 'warm'}"] = {
                "us": float(t.mean()) * 1e6, "elements_per_s": E / float(t.mean()),
                "gbs_b_alg": balg / float(t.mean()) / 1e9, "gbs_b_min": bmin / float(t.mean()) / 1e9,
                "frac_b_alg": balg / float(t.mean()) / 1e9 / HBM_PEAK_GBS, "b_alg_bytes": balg,
                "traffic": stored_traffic(f"p2_elasticity_kernel<{'double' if dt == torch.float64 else 'float'}>",
                                          "elasticity")}
        torch.cuda.synchronize()
        res[f"{name}_result"] = (vals.double().cpu().numpy(), rhs.double().cpu().numpy())
    out = {"workload": f"3D linear elasticity P2 tets, {n}^3 x 6 Kuhn, lambda,mu~U(0.5,2), b~N(0,1)^3, seed 0",
           "elements": E, "nnz": pat.nnz, "dofs": pat.n_dofs, "pattern_build_s": pattern_s}
    if not args.no_cpu_baseline:  # the error of both results against the FP64 oracle, and the oracle's time
        import oracle
        print("# elasticity: oracle ...", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        A = oracle.assemble_p2_elasticity(d["coords"], d["conn"], d["lam"], d["mu"], d["b"])
        t_or = time.perf_counter() - c0
        rp, ci = pat.csr()
        out["pattern_equal_oracle"] = bool(np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_idx))
        for name in ("fp64", "fp32"):
            v, r = res[f"{name}_result"]
            res[f"{name}_err_vs_oracle"] = {"values": normwise_err(v, A.vals, A.row_ptr),
                                            "rhs": normwise_err(r, A.rhs, None)}
        out["cpu_baseline"] = {"value": E / t_or, "unit": "elements/s", "cores": 1, "kind": "oracle",
                               "sample": f"one serial FP64 P2 assembly of the {E}-element mesh with its pattern, "
                                         f"{t_or:.1f} s"}
    for name in ("fp64", "fp32"):
        res.pop(f"{name}_result")
    out.update(res)
    print(json.dumps(out))


def adjoint_bytes(nv, dim, E, ndof, nbatch, s):
    """Algorithmic bytes of one tg_adjoint_p1 call with w = the states shifted by one (heat):
    element kernel (conn, coords, coef, nbatch lam + nbatch+1 state vectors, dlogc, scratch write)
    plus the vertex Reduce (inc_ptr, inc, scratch read, dcoords)."""
    k = dim + 1
    elem = E * k * 4 + nv * dim * 8 + E * s + (2 * nbatch + 1) * ndof * s + E * 8 + E * k * dim * 8
    red = (nv + 1) * 4 + E * k * 4 + E * k * dim * 8 + nv * dim * 8
    return elem + red


def run_heat(args, dev):
    """Differentiable heat: 2D P1 256^2 (131,072 triangles), 20 implicit-Euler steps, dt = 1e-3;
    one step of the benchmark = forward rollout + dL/du^N + adjoint gradient (log a, x, u0)."""
    import numpy as np
    import torch

    import meshgen
    import paper_2602_05052_amd as tg

    n = 256 if args.n == 64 else args.n
    dt_, nsteps, rtol = 1e-3, 20, 1e-10
    d = meshgen.heat_inputs(n, seed=0)
    E, nv = d["conn"].shape[0], d["coords"].shape[0]
    pat = tg.Pattern(d["conn"], nv)
    coords = torch.from_numpy(d["coords"]).to(dev)
    log_a = torch.from_numpy(d["log_a"]).to(dev)
    log_t = torch.from_numpy(meshgen.heat_inputs(n, seed=1)["log_a"]).to(dev)
    u0_np = np.sin(np.pi * d["coords"][:, 0]) * np.sin(np.pi * d["coords"][:, 1])
    s = torch.cuda.Stream(device=dev)
    res = {}
    print(f"# bench heat: E={E} nv={nv} steps {args.steps}", file=sys.stderr, flush=True)
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        r = rtol if dt == torch.float64 else 1e-6
        u0 = torch.from_numpy(u0_np).to(dt).to(dev)
        with torch.cuda.stream(s):
            target = tg.heat_rollout(pat, coords, log_t, u0, dt_, nsteps, rtol=r, stream=s)[0][-1].clone()
            t_f, t_b, it_f, it_b = [], [], [], []
            for k in range(args.warmup + args.steps):
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                e0.record(s)
                states, itf, _ = tg.heat_rollout(pat, coords, log_a, u0, dt_, nsteps, rtol=r, stream=s)
                e1.record(s)
                g = 2.0 * (states[-1] - target)
                dla, dx, du0, itb, _ = tg.heat_adjoint(pat, coords, log_a, states, g, dt_, rtol=r, stream=s)
                e2.record(s)
                torch.cuda.synchronize()
                if k >= args.warmup:
                    t_f.append(e0.elapsed_time(e1) * 1e-3)
                    t_b.append(e1.elapsed_time(e2) * 1e-3)
                    it_f.append(itf)
                    it_b.append(itb)
            # the batched adjoint kernel alone (element kernel + vertex Reduce), same shapes as in the backward
            lam = states[1:].clone()
            coef = (dt_ * torch.exp(log_a)).to(dt)
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
            dlc = torch.empty(E, dtype=torch.float64, device=dev)
            dxc = torch.empty(nv, 2, dtype=torch.float64, device=dev)
            tg.adjoint_p1(pat, tg.MASS_LAPLACE, coords, coef, lam, states[1:], states[:-1], -1.0, dlc, dxc, stream=s)
            for a0, a1 in evs:
                a0.record(s)
                tg.adjoint_p1(pat, tg.MASS_LAPLACE, coords, coef, lam, states[1:], states[:-1], -1.0, dlc, dxc,
                              stream=s)
                a1.record(s)
            torch.cuda.synchronize()
        t_adj = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3
        badj = adjoint_bytes(nv, 2, E, pat.n_dofs, nsteps, 8 if dt == torch.float64 else 4)
        tf, tb = float(np.mean(t_f)), float(np.mean(t_b))
        res[name] = {"forward_ms": tf * 1e3, "backward_ms": tb * 1e3, "grad_evals_per_s": 1.0 / (tf + tb),
                     "forward_pcg_iters": int(np.median(it_f)), "backward_pcg_iters": int(np.median(it_b)),
                     "pcg_us_per_iter": (tf + tb) / max(1, np.median(it_f) + np.median(it_b)) * 1e6,
                     "adjoint_kernel_us": t_adj * 1e6, "adjoint_gbs": badj / t_adj / 1e9,
                     "adjoint_bytes": badj, "pcg_rtol": r}
        res[name]["_grads"] = (dla, dx, du0, g)
    ta = stored_traffic("p1_adjoint_element_kernel<2,double,3>", "heat")
    tr = stored_traffic("vertex_reduce_kernel<2>", "heat")
    adjoint_traffic = ta + tr if ta is not None and tr is not None else None
    out = {"metric": "differentiable heat: gradient evaluations/s (forward rollout + adjoint)",
           "value": res["fp64"]["grad_evals_per_s"], "unit": "grad/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": (res["fp64"]["forward_ms"] + res["fp64"]["backward_ms"]),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"2D heat P1 triangles {n}^2 x 2, jitter 0.2h, log a~N(0,1) (seed 0), target "
                                  f"from log a seed 1, u0 = sin(pi x) sin(pi y), {nsteps} implicit-Euler steps dt "
                                  f"{dt_:g}, Dirichlet u = 0 on the boundary, loss ||u^N - target||^2",
                      "elements": E, "vertices": nv, "nnz": pat.nnz, "parallelism": "single GPU"},
           "roofline": {"bound": "hbm", "kernel": "p1_adjoint_element_kernel<2,double,mass_laplace> + "
                                                  "vertex_reduce_kernel<2> (nbatch 20)",
                        "achieved": res["fp64"]["adjoint_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": res["fp64"]["adjoint_gbs"] / HBM_PEAK_GBS, "traffic": adjoint_traffic,
                        "algorithmic_bytes_per_launch": res["fp64"]["adjoint_bytes"],
                        "note": "the step time is dominated by the 40 PCG solves, not by this kernel"}}
    if not args.no_cpu_baseline:
        import oracle

        print("# cpu baseline (oracle heat rollout + adjoint) ...", file=sys.stderr, flush=True)
        bnd = meshgen.boundary_vertices(d["coords"])
        c0 = time.perf_counter()
        U = oracle.heat_rollout(d["coords"], d["conn"], d["log_a"], u0_np, dt_, nsteps, bnd)
        Ut = oracle.heat_rollout(d["coords"], d["conn"], meshgen.heat_inputs(n, seed=1)["log_a"], u0_np, dt_,
                                 nsteps, bnd)
        c1 = time.perf_counter()
        ref = oracle.heat_adjoint(d["coords"], d["conn"], d["log_a"], U, dt_, 2 * (U[-1] - Ut[-1]), bnd)
        c2 = time.perf_counter()
        t_cpu = (c1 - c0) / 2 + (c2 - c1)
        out["cpu_baseline"] = {"value": 1.0 / t_cpu, "unit": "grad/s", "cores": 1, "kind": "oracle",
                               "sample": f"one forward rollout + adjoint of the same problem by the oracle (scipy "
                                         f"sparse LU factorised once per call, FP64 C element adjoint), {t_cpu:.2f} s",
                               "cpu": _cpu_model()}
        for name in ("fp64", "fp32"):
            dla, dx, du0, _ = res[name]["_grads"]
            errs = [float(np.max(np.abs(x.double().cpu().numpy() - r)) / np.max(np.abs(r)))
                    for x, r in zip((dla, dx, du0), ref)]
            res[name]["grad_err_vs_oracle"] = {"log_a": errs[0], "coords": errs[1], "u0": errs[2]}
    for name in ("fp64", "fp32"):
        res[name].pop("_grads")
    out["heat"] = res
    print(json.dumps(out))


def run_batched(args, dev):
    """B coefficient sets on the 64^3 Poisson pattern in one launch (values + rhs per member) against
    B single launches; bytes counted with the geometry and the routing read once per launch."""
    import numpy as np
    import torch

    import meshgen
    import paper_2602_05052_amd as tg

    B = args.batch
    d = meshgen.poisson_inputs(3, args.n, seed=0)
    E, nv = d["conn"].shape[0], d["coords"].shape[0]
    pat = tg.Pattern(d["conn"], nv)
    coords = torch.from_numpy(d["coords"]).to(dev)
    rng = np.random.default_rng(5)
    flush = torch.zeros(1 << 28, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream(device=dev)
    res = {}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        sz = 8 if dt == torch.float64 else 4
        coef = torch.from_numpy(np.exp(rng.standard_normal((B, E)))).to(dt).to(dev)
        load = torch.from_numpy(rng.uniform(-1, 1, (B, E))).to(dt).to(dev)
        vals = torch.empty(B, pat.nnz, dtype=dt, device=dev)
        rhs = torch.empty(B, pat.n_dofs, dtype=dt, device=dev)

        def batched():
            tg.assemble_batched(pat, tg.LAPLACE, coords, coef, load, values=vals, rhs=rhs, stream=s)

        def solo():
            for b in range(B):
                tg.assemble(pat, tg.LAPLACE, coords, coef[b], load[b], values=vals[b], rhs=rhs[b], stream=s)

        times = {}
        for label, fn in (("batched", batched), ("solo_loop", solo)):
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            with torch.cuda.stream(s):
                for _ in range(args.warmup):
                    fn()
                for e0, e1 in evs:
                    flush.add_(1.0)
                    e0.record(s)
                    fn()
                    e1.record(s)
            torch.cuda.synchronize()
            times[label] = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3
        bmin, balg = p1_bytes(nv, 3, E, pat.nnz, pat.n_dofs, sz, 2)
        per_member = E * 2 * sz + pat.nnz * sz + pat.n_dofs * sz
        b_batch = balg + (B - 1) * per_member  # geometry + routing once, B sets of coefficients/outputs
        # members 0 and B-1 of the batched launch against the oracle; every member bitwise equals its solo launch
        batched()
        torch.cuda.synchronize()
        vb, rb = vals.clone(), rhs.clone()
        solo()
        torch.cuda.synchronize()
        same = bool(torch.equal(vb, vals) and torch.equal(rb, rhs))
        errs = {}
        if not args.no_cpu_baseline:
            import oracle
            rp, ci = oracle.csr_pattern(nv, d["conn"])
            for b in (0, B - 1):
                ov, orr = oracle.assemble_p1_values(d["coords"], d["conn"], coef[b].double().cpu().numpy(),
                                                    load[b].double().cpu().numpy(), rp, ci)
                errs[f"member_{b}"] = {"values": normwise_err(vb[b].double().cpu().numpy(), ov, rp),
                                       "rhs": normwise_err(rb[b].double().cpu().numpy(), orr, None)}
        res[name] = {"members_bitwise_equal_solo": same, "err_vs_oracle": errs,
                     "batched_us": times["batched"] * 1e6, "solo_loop_us": times["solo_loop"] * 1e6,
                     "speedup": times["solo_loop"] / times["batched"],
                     "member_elements_per_s": B * E / times["batched"],
                     "gbs_routing_once": b_batch / times["batched"] / 1e9, "bytes_per_launch": b_batch,
                     "frac": b_batch / times["batched"] / 1e9 / HBM_PEAK_GBS}
    out = {"workload": f"3D Poisson P1 64^3 x 6 Kuhn, {B} coefficient sets (a=exp(N(0,1)), f=U(-1,1)) on one "
                       f"pattern, cold (1 GiB flush before each launch)",
           "batch": B, "elements": E, "nnz": pat.nnz, **res}
    print(json.dumps(out))


def run_serve(args, dev):
    """Served assemble+solve stream: each request is a Poisson problem on its own jittered 2D P1 (1k-500k
    triangles) or 3D P1 (6k-1.5M tets) mesh whose element count is log-uniform (grid n = round(sqrt(E/2)) or
    round(cbrt(E/6)), so sizes are continuous), with lognormal a and f = U(-1,1), FP32 assembly + Dirichlet +
    Jacobi-PCG to 1e-6.  Requests reach the server by connectivity (tg_server_submit_mesh): it builds, caches
    (keyed by (dim, n)) and evicts CSR patterns within its HBM budget (--budget-gib), so topologies it has
    not seen cost a pattern build.  The same requests served one at a time (patterns cached in a dictionary
    by the same key, built on a miss) are the baseline.  Legs: a warm-up draw, then all requests at once
    (saturation throughput), then Poisson arrivals at 0.5x and 0.8x of the served saturation rate (or at
    --rate); each leg draws its own sizes, so both caches see hits and misses."""
    import numpy as np
    import torch

    import meshgen
    import oracle
    import paper_2602_05052_amd as tg

    R = args.requests
    rtol = 1e-6
    s = torch.cuda.Stream(device=dev)
    OK = (tg.TG_OK, tg.TG_E_ACCURACY)  # ACCURACY: rtol below the FP32 attainable true residual

    def draw(seed):
        rng = np.random.default_rng(seed)
        out = []
        for i in range(R):
            dim = 2 if rng.random() < 0.5 else 3
            lo, hi = (1000, 500000) if dim == 2 else (6000, 1.5e6)
            E = np.exp(rng.uniform(np.log(lo), np.log(hi)))
            n = int(np.clip(round(np.sqrt(E / 2)), 22, 500)) if dim == 2 else int(np.clip(round(np.cbrt(E / 6)), 10, 63))
            m = meshgen.poisson_inputs(dim, n, seed=seed * 1000 + i)
            out.append({"dim": dim, "n": n, "key": dim * 1000 + n, "conn": np.ascontiguousarray(m["conn"], dtype=np.int32),
                        "nv": len(m["coords"]), "coords": torch.from_numpy(m["coords"]).to(dev),
                        "a": torch.from_numpy(m["a"]).float().to(dev), "f": torch.from_numpy(m["f"]).float().to(dev),
                        "x": torch.empty(len(m["coords"]), dtype=torch.float32, device=dev), "m": m})
        return out, rng.exponential(1.0, R)

    seq_cache, seq_build = {}, [0, 0.0]

    def sequential(reqs, arrive):
        lat, its, st_count = [], 0, {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            for i, r in enumerate(reqs):
                while time.perf_counter() - t0 < arrive[i]:
                    pass
                pat = seq_cache.get(r["key"])
                if pat is None:
                    tb = time.perf_counter()
                    pat = seq_cache[r["key"]] = tg.Pattern(r["conn"], r["nv"])
                    seq_build[0] += 1
                    seq_build[1] += time.perf_counter() - tb
                vals, rhs = tg.assemble(pat, tg.LAPLACE, r["coords"], r["a"], r["f"], stream=s)
                tg.apply_dirichlet(pat, vals, rhs, stream=s)
                _, it, rr, st = tg.pcg(pat, vals, rhs, rtol=rtol, x=r["x"], check_every=10, stream=s,
                                       raise_on_noconv=False, return_status=True)
                if st not in OK:
                    raise RuntimeError(f"sequential request {i} ended with {st}")
                st_count[st] = st_count.get(st, 0) + 1
                r["seq_relres"] = rr
                its += it
                lat.append(time.perf_counter() - t0 - arrive[i])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, np.array(lat), its, st_count

    srv = tg.Server(hbm_budget=int(args.budget_gib * (1 << 30)), max_slots=args.slots, check_every=10, stream=s)

    def served(reqs, arrive):
        torch.cuda.synchronize()
        i0 = srv.info()
        t0 = time.perf_counter()
        nxt, lat, arr, st_count, rel = 0, [], {}, {}, []
        while len(lat) < R:
            now = time.perf_counter() - t0
            while nxt < R and arrive[nxt] <= now:
                r = reqs[nxt]
                rid = srv.submit_mesh(r["conn"], r["nv"], tg.LAPLACE, r["coords"], r["a"], r["f"],
                                      topology_key=r["key"], x=r["x"], rtol=rtol)
                arr[rid] = arrive[nxt]
                nxt += 1
            if srv.pending():
                srv.step()
            for res in srv.poll():
                if res["status"] not in OK:
                    raise RuntimeError(f"request {res['request_id']} ended with status {res['status']}")
                st_count[res["status"]] = st_count.get(res["status"], 0) + 1
                rel.append(res["relres"])
                lat.append(time.perf_counter() - t0 - arr[res["request_id"]])
        torch.cuda.synchronize()
        i1 = srv.info()
        cache = {"pattern_builds": i1["n_pattern_builds"] - i0["n_pattern_builds"],
                 "pattern_evictions": i1["n_pattern_evictions"] - i0["n_pattern_evictions"],
                 "pattern_build_s": i1["pattern_build_s"] - i0["pattern_build_s"], "hbm_used_gib": i1["hbm_used"] / 2**30}
        return time.perf_counter() - t0, np.array(lat), st_count, float(max(rel)), cache

    def pct(v):
        return {"p50": float(np.percentile(v, 50)) * 1e3, "p90": float(np.percentile(v, 90)) * 1e3,
                "p99": float(np.percentile(v, 99)) * 1e3}

    def leg(seed, rate):
        reqs, gaps = draw(seed)
        arrive = np.zeros(R) if rate is None else np.cumsum(gaps / rate)
        b0 = list(seq_build)
        ts, ls, its, sst = sequential(reqs, arrive)
        ref = [r["x"].clone() for r in reqs]
        tv, lv, vst, relmax, cache = served(reqs, arrive)
        same = all(torch.equal(a, r["x"]) for a, r in zip(ref, reqs))
        out = {"rate_per_s": rate, "served_requests_per_s": R / tv, "sequential_requests_per_s": R / ts,
               "served_latency_ms": pct(lv), "sequential_latency_ms": pct(ls), "served_status": sst_name(vst),
               "sequential_status": sst_name(sst), "served_relres_max": relmax, "server_cache": cache,
               "sequential_pattern_builds": seq_build[0] - b0[0], "sequential_pattern_build_s": seq_build[1] - b0[1],
               "bitwise_equal_to_sequential": bool(same), "pcg_iterations_total": int(its),
               "elements_total": int(sum(len(r["conn"]) for r in reqs)),
               "distinct_topologies": len({r["key"] for r in reqs})}
        return out, reqs, tv

    def sst_name(d):
        return {tg._STATUS_NAMES[k]: v for k, v in sorted(d.items())}

    print(f"# serve: {R} requests per leg, continuous sizes, budget {args.budget_gib} GiB", file=sys.stderr, flush=True)
    leg(1, None)  # warm-up: code paths, slots, first patterns
    sat_leg, sat_reqs, t_sat = leg(2, None)
    # error of the served FP32 solutions against the FP64 oracle (condensed direct solve), sampled: the
    # smallest 2D and 3D requests of the saturation leg
    errs = []
    for dim in (2, 3):
        r = min((q for q in sat_reqs if q["dim"] == dim), key=lambda q: q["n"], default=None)
        if r is None:
            continue
        m = r["m"]
        A = oracle.assemble_p1(m["coords"], m["conn"], m["a"], m["f"])
        bnd = meshgen.boundary_vertices(m["coords"])
        ref = oracle.condensed_solve(A, bnd)
        errs.append({"dim": dim, "n": r["n"], "relerr_vs_oracle": oracle.relerr(r["x"].double().cpu().numpy(), ref),
                     "relres_lin_vs_oracle": oracle.relres_lin(A, r["x"].double().cpu().numpy(), bnd)})
    sat = R / t_sat
    rates = [args.rate] if args.rate > 0 else [0.5 * sat, 0.8 * sat]
    legs = [leg(3 + k, rate)[0] for k, rate in enumerate(rates)]
    out = {"metric": "served assemble+solve requests/s and p50/p99 latency", "unit": "requests/s",
           "value": sat_leg["served_requests_per_s"],
           "workload": f"served stream: {R} requests per leg, jittered 2D P1 1k-500k triangles and 3D P1 6k-1.5M "
                       f"tets (log-uniform element counts, continuous grid sizes), lognormal a, f=U(-1,1), FP32 "
                       f"assembly + Dirichlet + Jacobi-PCG to {rtol:g}; submitted by connectivity, patterns cached "
                       f"by (dim, n) within the HBM budget; all at once, then Poisson arrivals",
           "requests": R, "slots_per_group": args.slots, "hbm_budget_gib": args.budget_gib,
           "saturation": sat_leg, "poisson_arrivals": legs, "sampled_error_vs_fp64_oracle": errs}
    print(json.dumps(out))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs visible)"
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
