"""Benchmark: one energy of the N = 25600 coupled-channel R-matrix solve per step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu]

Workload "large": nc = 256 channels x nr = 100 Lagrange-Legendre points
(N = 25600), a = 30 fm, seeded Woods-Saxon optical-potential family, 10
energies in [5, 30] MeV; step s solves energy s mod 10.  A step is the whole
hot path on device-resident inputs: assemble C(E) -> LU -> solve for the 256
surface right-hand sides (+ FP64 refinement) -> R-matrix -> collision matrix.

Headline: FP32-LU + FP64 iterative refinement.  The plain FP64 LU is timed
the same way and reported beside it.  TF/s counts the LU's (8/3) N^3 real
flops per solve (the paper's count, Sec. 3.3).  The roofline entry is the
dominant kernel, the trailing-update complex GEMM, measured with HIP events
around its launches inside the timed region; its achieved rate counts the
real matrix-core flops of the product it performs (6MNK for the FP32 3M
product, 8MNK for the FP64 4M one).  cpu_baseline times the CPU
oracle (plain Gaussian elimination) on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N=25600 complex solve s & TF/s, FP32-LU+IR vs FP64 LU; served solves/s, p99"
PEAK_FP32_MFMA = 157.3  # TF/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6   # TF/s, MI355X dense FP64 matrix
PEAK_FP16_MFMA = 2500.0  # TF/s, MI355X dense FP16 matrix
# HBM bytes per launch of the FP32 GEMM on this command, over the launches
# the roofline timers see (each step's factorization and first solve), from
# FETCH_SIZE and WRITE_SIZE counter runs scaled by a 1 GiB copy
# (profiles/gemm_direct_kernel_fp32_large_N25600_traffic.md); valid only for
# the GEMM source it was measured on.
GEMM_TRAFFIC = {"bytes_per_launch": 3.3425e+08,
                "gemm_source_sha256": "eb8322e4a8d94eff31b1c7563e7a8fc9c34ed4338b59a1b362586c2fa9ee4a44"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="large")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-update variant")
    ap.add_argument("--scan-slots", type=int, default=3,
                    help="solvers in flight in the FP32+IR energy-scan block (0: skip the block)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-refine", type=int, default=30)
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-closed", action="store_true", help="skip the closed-channel matching block")
    ap.add_argument("--no-nonlocal", action="store_true", help="skip the non-local potential block")
    ap.add_argument("--no-woodbury", action="store_true", help="skip the Woodbury-kinetic (Type 3) block")
    ap.add_argument("--block-steps", type=int, default=3,
                    help="timed energies of the non-local and Woodbury-kinetic blocks")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-systems", type=int, default=512)
    ap.add_argument("--served-requests", type=int, default=24)
    ap.add_argument("--served-rate", type=float, default=4.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--served-rate-sustained", type=float, default=2.0,
                    help="a second, lower arrival rate for the same requests (0: skip)")
    ap.add_argument("--only", choices=("batched", "served", "nonlocal", "woodbury"), default=None,
                    help="run only this block (for profiling) and print it as the JSON line")
    ap.add_argument("--counter-summary", metavar="CSV", default=None,
                    help="read a rocprofv3 --pmc counter CSV or --kernel-trace CSV (no GPU) and print "
                         "per-kernel counter (or duration) sums, then exit")
    ap.add_argument("--kernel", default="", help="with --counter-summary: only kernels whose name contains this")
    ap.add_argument("--window", nargs=2, metavar=("FIRST", "LAST"), default=None,
                    help="with --counter-summary: only dispatches from each dispatch of a kernel named FIRST "
                         "up to the next one named LAST")
    ap.add_argument("--trace-overlap", metavar="CSV", default=None,
                    help="read a rocprofv3 kernel-trace CSV (no GPU) and print how long factorization "
                         "kernels of different hardware queues ran at the same time, then exit")
    ap.add_argument("--served-slots", type=int, default=4)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (a plain copy of known size, "
                         "to scale hardware traffic counters) and exit")
    return ap.parse_args()


def timed_steps(solver, energies, steps, warmup, H, torch, gemm_stage, **run):
    """Warmup, then exactly `steps` steps bracketed by synchronizations.

    Inside the timed region only the launches of the dominant kernel (the
    trailing-update GEMM, stage `gemm_stage`) are bracketed with HIP events;
    the per-stage breakdown comes from one further step, outside the timed
    region, with every stage timed."""
    ne = len(energies)
    for s in range(warmup):
        solver.run(float(energies[s % ne]), **run)
    torch.cuda.synchronize()
    H.hp_trace_enable(True, stages=[gemm_stage])
    infos = []
    t0 = time.perf_counter()
    for s in range(steps):
        r = solver.run(float(energies[s % ne]), **run)
        infos.append((r.iterations, r.backward_error, r.fallback))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gemm = H.hp_trace_read()[gemm_stage]
    H.hp_trace_enable(True)
    solver.run(float(energies[steps % ne]), **run)
    torch.cuda.synchronize()
    stages = H.hp_trace_read()
    H.hp_trace_enable(False)
    return (t1 - t0) / steps, infos, gemm, stages


def gemm_traffic():
    """Measured HBM bytes per GEMM launch, or None if the GEMM source changed since."""
    import hashlib
    path = os.path.join(ROOT, "paper_2512_11590_amd", "csrc", "gemm.hip")
    with open(path, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return GEMM_TRAFFIC["bytes_per_launch"] if sha == GEMM_TRAFFIC["gemm_source_sha256"] else None


def batched(args, H, torch):
    """The uneven batch: nc ~ U{5..80}, nr ~ U{40..50}, one energy per system,
    one workgroup per system in size buckets (autotuned on each bucket's 8
    largest systems), FP32 + IR and FP64.  Rate: (8/3) sum N^3 / time of
    build + factor + solve (+ refinement) + R for the whole batch."""
    import numpy as np
    from paper_2512_11590_amd import batch as B
    from workload import batch_systems
    sps = batch_systems(args.batched_systems)
    res = {"systems": len(sps), "N_range": [min(s.nc * s.nr for s in sps), max(s.nc * s.nr for s in sps)]}
    for name, prec in (("fp32_ir", H.HP_C64), ("fp64", H.HP_C128)):
        print(f"[bench] batched {name}: {len(sps)} systems", file=sys.stderr, flush=True)
        bt = B.Batch(sps, [s.energies[0] for s in sps], prec)
        tuned = bt.tune(sample=16, panels=(8, 16, 32), groups_per_cu=(2,))
        bt.run()  # warm (captures the refinement graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = bt.run()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st, it = bt.status()
        res[name] = {"ms": t * 1e3, "tflops": bt.flops / t / 1e12, "systems_per_s": len(sps) / t,
                     "buckets": tuned, "refinement_steps": steps,
                     "converged": int(np.sum(st == 1)), "mean_corrections": float(it.mean())}
        del bt
        torch.cuda.empty_cache()
    return res


def closed_channels(sp, H, P, torch):
    """The matching step with closed channels at full size: the same system
    with the thresholds of every eighth channel raised above the energy
    (32 of 256 closed), one FP32+IR solve there, then hp_smatrix timed on its
    R against the all-open matching of the original system's R."""
    import copy
    import numpy as np
    E = 16.25
    spc = copy.deepcopy(sp)
    e = np.asarray(sp.eps, dtype=np.float64)
    spc.eps = np.where(np.arange(sp.nc) % 8 != 7, e, 22.0 + e)
    res = {"energy": E, "closed": int(np.sum(spc.eps > E)), "open": int(np.sum(spc.eps < E))}
    for name, params in (("all_open", sp), ("closed", spc)):
        d = P.DeviceSystem(params)
        s = P.Solver(d, H.HP_C64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.run(E)
        torch.cuda.synchronize()
        t_step = time.perf_counter() - t0
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            nopen = H.hp_smatrix(d.sys, E, s.R, s.S, s.swork)
        torch.cuda.synchronize()
        res[name] = {"step_ms": t_step * 1e3, "smatrix_ms": (time.perf_counter() - t0) / reps * 1e3,
                     "nopen": nopen, "refinement_steps": r.iterations}
        del s, d
        torch.cuda.empty_cache()
    return res


def nonlocal_block(sp, H, P, torch, steps=3):
    """The headline system with a non-local kernel added (Sec. 2: full
    coupling blocks): a Perey-Buck-form optical kernel coupled across the
    channels like the local couplings, passed as dense n x n values
    (10.5 GB at N = 25600), built on the device as kron(B, K).  FP32 LU +
    FP64 refinement steps timed as in the main line (one warmup), then one
    FP64-LU solve of the same system for the S difference."""
    import numpy as np
    from workload import perey_buck_factors
    n = sp.nc * sp.nr
    r = H.hp_mesh(sp.nr, float(sp.a))[0]
    B, K = perey_buck_factors(sp, r)
    W = torch.kron(torch.from_numpy(B.astype(np.complex128)).to("cuda"), torch.from_numpy(K).to("cuda"))
    d = P.DeviceSystem(sp, vnl=W)
    E = float(sp.energies[steps % len(sp.energies)])
    res = {"N": n, "kernel": "Perey-Buck form x0.4, width 0.85 fm, channel coupling I + beta",
           "kernel_bytes": int(W.numel() * W.element_size()), "energy_of_checks": E}
    print("[bench] non-local block: fp32+ir", file=sys.stderr, flush=True)
    s = P.Solver(d, H.HP_C64)
    t, infos, _, stages = timed_steps(s, sp.energies, steps, 1, H, torch, "gemm_c64")
    S32 = s.S.cpu().numpy()
    res["fp32_ir"] = {"ms_per_step": t * 1e3, "refinement_steps": [i[0] for i in infos],
                      "backward_error": [i[1] for i in infos], "fp64_fallbacks": sum(bool(i[2]) for i in infos),
                      "stages_ms_one_step": {k: round(v["ms"], 3) for k, v in stages.items() if v["launches"]}}
    del s
    torch.cuda.empty_cache()
    print("[bench] non-local block: fp64 check", file=sys.stderr, flush=True)
    s = P.Solver(d, H.HP_C128)
    s.run(E)
    S64 = s.S.cpu().numpy()
    res["S_relerr_fp32ir_vs_fp64"] = float(np.max(np.abs(S32 - S64)) / np.max(np.abs(S64)))
    del s, d, W
    torch.cuda.empty_cache()
    return res


def woodbury_block(sp, H, P, torch, steps=3):
    """The Woodbury-kinetic form (the paper's Type 3, Sec. 3.3) on the headline
    system: FP32 factors of S(E) = I + K_diag^-1 V, FP64 refinement on
    C(E)'s residual, timed like the main line (one warmup, `steps` energies);
    then the same energy through the direct form for the S difference and
    the refinement steps side by side."""
    import numpy as np
    d = P.DeviceSystem(sp)
    res = {}
    for name, schur in (("schur", True), ("direct", False)):
        print(f"[bench] woodbury block: {name}", file=sys.stderr, flush=True)
        s = P.Solver(d, H.HP_C64, schur=schur)
        t, infos, _, stages = timed_steps(s, sp.energies, steps, 1, H, torch, "gemm_c64")
        res[name] = {"ms_per_step": t * 1e3, "refinement_steps": [i[0] for i in infos],
                     "fp64_fallbacks": sum(bool(i[2]) for i in infos),
                     "stages_ms_one_step": {k: round(v["ms"], 3) for k, v in stages.items() if v["launches"]}}
        res[name + "_S"] = s.S.cpu().numpy()
        del s
        torch.cuda.empty_cache()
    a, b = res.pop("schur_S"), res.pop("direct_S")
    res["energy_of_check"] = float(sp.energies[steps % len(sp.energies)])
    res["S_relerr_schur_vs_direct"] = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return res


def served_stream(args, H, torch, rate=None):
    """The served stream: Poisson arrivals, N log-uniform in [500, 16000],
    1-8 energies each, continuous batching over a few slots; FP32 + IR, then
    FP64 on the same arrivals.  Reports solves/s, p50/p99 latency and the
    largest S difference between the two precisions per request."""
    import numpy as np
    from paper_2512_11590_amd import serve
    from workload import served_requests
    rate = args.served_rate if rate is None else rate
    reqs = served_requests(args.served_requests, rate)
    res = {"requests": len(reqs), "rate_hz": rate, "slots": args.served_slots,
           "N_range": [min(sp.nc * sp.nr for _, sp in reqs), max(sp.nc * sp.nr for _, sp in reqs)],
           "energies": int(sum(len(sp.energies) for _, sp in reqs))}
    runs = {}
    for name, prec in (("fp32_ir", H.HP_C64), ("fp64", H.HP_C128)):
        print(f"[bench] served stream {name}: {len(reqs)} requests at {rate}/s", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        done = []

        def progress(req, name=name, t0=t0):
            done.append(req.rid)
            print(f"[bench]   {name}: request {req.rid} (N={req.n}, {len(req.energies)} energies) done, "
                  f"{len(done)}/{len(reqs)} at {time.perf_counter() - t0:.1f} s"
                  + (f" error {req.error}" if req.error else ""), file=sys.stderr, flush=True)

        runs[name] = serve.Server(slots=args.served_slots, prec=prec).run(reqs, progress=progress)
        torch.cuda.empty_cache()
        res[name] = serve.summary(runs[name])
    diffs = [float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
             for ra, rb in zip(runs["fp32_ir"], runs["fp64"]) if ra.error is None and rb.error is None
             for a, b in zip(ra.S, rb.S)]
    res["S_relerr_fp32ir_vs_fp64_max"] = max(diffs) if diffs else None
    return res


def counter_summary(path: str, kernel: str = "", window=None) -> dict:
    """Per-kernel sums of rocprofv3 --pmc counters (one row per dispatch and
    counter; from a --kernel-trace CSV, the dispatch durations as the counter
    DurationNs), over the dispatches whose name contains `kernel`; with window =
    (FIRST, LAST), only dispatches from a FIRST dispatch up to the next LAST
    one (by dispatch id), e.g. one LU step's factorization and first solve."""
    import csv
    from collections import defaultdict
    disp = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            e = disp.setdefault(d, {"name": r["Kernel_Name"], "counters": {}})
            if "Counter_Name" in r:
                c, v = r["Counter_Name"], float(r["Counter_Value"])
            else:  # a --kernel-trace CSV: the dispatch's duration
                c, v = "DurationNs", float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            e["counters"][c] = e["counters"].get(c, 0.0) + v
    keep = set(disp)
    if window:
        keep, inside = set(), False
        for d in sorted(disp):
            nm = disp[d]["name"]
            if window[0] in nm:
                inside = True
            if inside:
                keep.add(d)
            if inside and window[1] in nm:
                inside = False
    out = defaultdict(lambda: {"dispatches": 0, "counters": defaultdict(float)})
    for d in sorted(keep):
        nm = disp[d]["name"]
        if kernel and kernel not in nm:
            continue
        key = nm.split("(")[0] if "(anonymous" not in nm else nm.replace("(anonymous namespace)::", "").split("(")[0]
        out[key]["dispatches"] += 1
        for c, v in disp[d]["counters"].items():
            out[key]["counters"][c] += v
    return {k: {"dispatches": v["dispatches"], "counters": dict(v["counters"])} for k, v in out.items()}


def trace_overlap(path: str) -> dict:
    """Factorization kernels in a rocprofv3 kernel trace (single-system panel
    grids and panel finishes; batched panel, interchange/block-row and
    trailing-update steps): total time with at least one of them running,
    time with kernels of two or more hardware queues running at once, and
    time with a batched and a single-system factorization running at once."""
    import csv
    from collections import Counter
    single = ("panel_kernel", "panel_finish_kernel")
    batched_k = ("batch_panel_kernel", "batch_trail_kernel", "batch_lu_kernel", "batch_swap_brow_kernel",
                 "batch_brow_kernel")
    edges = []
    kinds = Counter()
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1]
            base = name.split("<")[0]
            kind = "single" if base in single else "batched" if base in batched_k else None
            if kind is None:
                continue
            q = r["Queue_Id"]
            kinds[(kind, q)] += 1
            edges.append((int(r["Start_Timestamp"]), 1, q, kind))
            edges.append((int(r["End_Timestamp"]), -1, q, kind))
    edges.sort()
    live = Counter()
    t_any = t_multi = t_mixed = 0
    last = edges[0][0] if edges else 0
    for t, d, q, kind in edges:
        on = [k for k, v in live.items() if v > 0]
        dt = t - last
        if on:
            t_any += dt
        if len({k[0] for k in on}) >= 2:
            t_multi += dt
        if {"single", "batched"} <= {k[1] for k in on}:
            t_mixed += dt
        live[(q, kind)] += d
        last = t
    return {"factorization_kernels": {f"{k} queue {q}": v for (k, q), v in sorted(kinds.items())},
            "ms_any_running": t_any / 1e6, "ms_two_or_more_queues": t_multi / 1e6,
            "ms_batched_and_single_system": t_mixed / 1e6}


def cpu_baseline(n_full: int):
    """Oracle (plain GE + R + S) on a reduced system of the same family, N^3-scaled."""
    import numpy as np  # noqa: F401
    from oracle import ge, pipeline as opipe, system as osys
    from workload import make_system
    ge.build(force=False)
    nc_s = 48
    sp = make_system("large", nc=nc_s)
    md = osys.MeshData(sp.nr, sp.a)
    E = float(sp.energies[0])
    t0 = time.perf_counter()
    opipe.solve_energy(sp, E, md)
    t = time.perf_counter() - t0
    n_s = sp.n
    tflops = (8.0 / 3.0) * n_s ** 3 / t / 1e12
    t_full = (8.0 / 3.0) * n_full ** 3 / (tflops * 1e12)
    return {"value": tflops, "unit": "TF/s", "cores": ge.threads(), "kind": "oracle",
            "sample": (f"one full oracle solve (GE with partial pivoting + R + S) of the same potential family "
                       f"at nc={nc_s}, nr={sp.nr} (N={n_s}), E={E} MeV: {t:.2f} s; "
                       f"N={n_full} time extrapolated as (8/3)N^3 / rate = {t_full:.0f} s")}


def main():
    args = parse()
    if args.trace_overlap:
        print(json.dumps(trace_overlap(args.trace_overlap)), flush=True)
        return
    if args.counter_summary:
        print(json.dumps(counter_summary(args.counter_summary, args.kernel, args.window)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2512_11590_amd import hprmat as H
    from paper_2512_11590_amd import pipeline as P
    from workload import make_system

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(1)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes}))
        return
    if args.only:
        if args.only == "nonlocal":
            blk = nonlocal_block(make_system(args.config), H, P, torch, steps=args.block_steps)
        elif args.only == "woodbury":
            blk = woodbury_block(make_system(args.config), H, P, torch, steps=args.block_steps)
        else:
            blk = batched(args, H, torch) if args.only == "batched" else served_stream(args, H, torch)
        print(json.dumps({"only": args.only, args.only: blk}), flush=True)
        return
    sp = make_system(args.config)
    n = sp.n
    flops = (8.0 / 3.0) * n ** 3
    d = P.DeviceSystem(sp)
    torch.cuda.synchronize()

    out = {"metric": METRIC, "unit": "TF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64 LU + f64 refinement", "data": "synthetic",
           "config": {"workload": f"{args.config}: nc={sp.nc}, nr={sp.nr} (N={n}), a={sp.a} fm, "
                                  f"Woods-Saxon optical family seed {sp.label}, energies 5..30 MeV",
                      "global_batch": 1, "nrhs": sp.nc}}

    s32 = P.Solver(d, H.HP_C64)
    print(f"[bench] fp32-LU+IR N={n}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    t32, info32, g, st32 = timed_steps(s32, sp.energies, args.steps, args.warmup, H, torch, "gemm_c64",
                                       max_refine=args.max_refine, tol=args.tol)
    out["value"] = flops / t32 / 1e12
    out["ms_per_step"] = t32 * 1e3
    out["refinement"] = [{"steps": it, "backward_error": c, "fp64_fallback": fb} for it, c, fb in info32]
    out["stages_ms_one_step"] = {k: round(v["ms"], 3) for k, v in st32.items() if v["launches"]}
    ach = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    out["roofline"] = {"bound": "mfma", "kernel": "FP32 complex 3M GEMM (gemm_direct_kernel, with "
                                                  "gemm_sub_kernel<float> for ragged shapes; achieved counts the "
                                                  "6MNK real flops per launch)",
                       "achieved": ach, "peak": PEAK_FP32_MFMA, "unit": "TF/s", "frac": ach / PEAK_FP32_MFMA,
                       "traffic": gemm_traffic(), "launches_per_step": g["launches"] / args.steps,
                       "avg_launch_us": g["ms"] * 1e3 / max(1, g["launches"])}
    # S of the breakdown step that timed_steps runs after the timed ones
    S32 = s32.S.cpu().numpy().copy()
    last_e = float(sp.energies[args.steps % len(sp.energies)])
    del s32
    torch.cuda.empty_cache()

    if args.scan_slots > 0:
        # the same FP32+IR solves as an energy scan with several solvers in
        # flight: one energy's solves, refinement, R and S run beside the
        # next one's assembly and factorization (factorizations serialized)
        import numpy as np
        scan = P.EnergyScan(d, H.HP_C64, slots=args.scan_slots)
        ne = len(sp.energies)
        es = [float(sp.energies[s % ne]) for s in range(max(args.steps + 1, 3 * args.scan_slots))]
        print(f"[bench] fp32-LU+IR energy scan, {args.scan_slots} solvers in flight, {len(es)} energies",
              file=sys.stderr, flush=True)
        scan.run(es[:args.scan_slots], max_refine=args.max_refine, tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = scan.run(es, max_refine=args.max_refine, tol=args.tol)
        torch.cuda.synchronize()
        tsc = (time.perf_counter() - t0) / len(es)
        k_last = args.steps % ne
        same = [float(np.max(np.abs(r.S.numpy() - S32)) / np.max(np.abs(S32)))
                for i, r in enumerate(res) if i % ne == k_last]
        out["fp32_ir_scan"] = {"solvers_in_flight": args.scan_slots, "energies": len(es),
                               "ms_per_energy": tsc * 1e3, "tflops": flops / tsc / 1e12,
                               "refinement_steps": [r.iterations for r in res],
                               "fp64_fallbacks": int(sum(r.fallback for r in res)),
                               "S_relerr_vs_single_solver_at_E": [last_e, max(same) if same else None]}
        del scan
        torch.cuda.empty_cache()

    if not args.no_fp16:
        # the FP16 variant: FP32 factors whose trailing updates run on the
        # FP16 matrix cores (split operands under row/column scaling), the
        # same FP64 refinement; same energies, same step count
        s16 = P.Solver(d, H.HP_C64H)
        print(f"[bench] fp16x3-update LU+IR N={n}", file=sys.stderr, flush=True)
        t16, info16, g16, st16 = timed_steps(s16, sp.energies, args.steps, args.warmup, H, torch, "gemm_f16x3",
                                             max_refine=args.max_refine, tol=args.tol)
        ach16 = g16["flops"] / (g16["ms"] * 1e-3) / 1e12 if g16["ms"] > 0 else 0.0
        import numpy as np
        S16 = s16.S.cpu().numpy()
        out["fp16x3_lu_ir"] = {
            "ms_per_step": t16 * 1e3, "tflops": flops / t16 / 1e12,
            "refinement_steps": [it for it, _, _ in info16],
            "fp64_fallbacks": int(sum(1 for _, _, fb in info16 if fb)),
            "S_relerr_vs_fp32ir_at_E": [last_e, float(np.max(np.abs(S16 - S32)) / np.max(np.abs(S32)))],
            "stages_ms_one_step": {k: round(v["ms"], 3) for k, v in st16.items() if v["launches"]},
            "roofline_update": {"bound": "mfma", "kernel": "split-FP16 complex GEMM (gemm_h3_kernel; achieved "
                                                            "counts the 24MNK FP16 matrix-core flops per launch)",
                                "achieved": ach16, "peak": PEAK_FP16_MFMA, "unit": "TF/s",
                                "frac": ach16 / PEAK_FP16_MFMA,
                                "launches_per_step": g16["launches"] / args.steps,
                                "avg_launch_us": g16["ms"] * 1e3 / max(1, g16["launches"])}}
        del s16
        torch.cuda.empty_cache()

    if not args.no_fp64:
        s64 = P.Solver(d, H.HP_C128)
        print(f"[bench] fp64-LU N={n}", file=sys.stderr, flush=True)
        t64, _, g64, st64 = timed_steps(s64, sp.energies, args.steps, args.warmup, H, torch, "gemm_c128")
        ach64 = g64["flops"] / (g64["ms"] * 1e-3) / 1e12 if g64["ms"] > 0 else 0.0
        S64 = s64.S.cpu().numpy()
        import numpy as np
        err = float(np.max(np.abs(S32 - S64)) / np.max(np.abs(S64)))
        out["fp64_lu"] = {"ms_per_step": t64 * 1e3, "tflops": flops / t64 / 1e12,
                          "gemm_achieved_tflops": ach64, "gemm_frac_of_fp64_peak": ach64 / PEAK_FP64_MFMA,
                          "stages_ms_one_step": {k: round(v["ms"], 3) for k, v in st64.items()
                                                 if v["launches"]},
                          "S_relerr_fp32ir_vs_fp64_at_E": [last_e, err]}
        del s64
        torch.cuda.empty_cache()
    if not args.no_closed:
        out["closed_channels"] = closed_channels(sp, H, P, torch)
    if not args.no_nonlocal:
        out["nonlocal"] = nonlocal_block(sp, H, P, torch, steps=args.block_steps)
    if not args.no_woodbury:
        out["woodbury_kinetic"] = woodbury_block(sp, H, P, torch, steps=args.block_steps)
    if not args.no_batched:
        out["batched"] = batched(args, H, torch)
    if not args.no_served:
        out["served"] = served_stream(args, H, torch)
        if args.served_rate_sustained > 0:
            out["served_sustained"] = served_stream(args, H, torch, rate=args.served_rate_sustained)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
