#!/usr/bin/env python3
"""Benchmark of the NOLSM hot path on one MI355X.

One step = the whole path for every molecule of the workload at one chemical
potential: gather T_k(H0), T_k(S) -> FP64 set-up -> batched sign iteration ->
panel refinement and density columns -> scatter into D -> Tr(DH), Tr(DS).
Inputs are resident in HBM before the timed region starts.

The reported value follows the paper's accounting (Sec. V-B, "FLOPs in the NOLSM
method" and "Node-Performance"): FLOPs are 2 n^3 per n x n x n product of the
matrix iterations (two products per Newton-Schulz step), O(n^2) work is not
counted, and the time is the wall time of the whole step.  The roofline entry is
for the dominant kernel (the sign-iteration GEMM) on the MFMA flops it executes.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--batch B]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sign-iteration TFLOP/s & submatrices/s at <=1e-5 Ha/atom, mixed vs plain FP32"
FP16_PEAK = 2516.6            # TFLOP/s, MI355X dense FP16 MFMA
FP32_PEAK = 157.3             # TFLOP/s, MI355X FP32


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def paper_flops(stats, products_per_iter=2):
    """2 n^3 per product, two products per Newton-Schulz iteration (Eq. 6; every
    schedule timed here is Newton-Schulz; a third-order phase takes three)."""
    n3 = stats["n"].astype(np.float64) ** 3
    return float((2.0 * products_per_iter * n3 * (stats["iters_lo"] + stats["iters_fb"])).sum())


def timed_steps(runner, sched, steps, L, torch, predictor=None):
    for p in runner.plans:
        L.nolsm_plan_get_timings(p, reset=True)
        L.nolsm_plan_set_timing(p, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        runner.run(sched=sched, predictor=predictor)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    tot = {}
    for p in runner.plans:
        t = L.nolsm_plan_get_timings(p, reset=True).as_dict()
        for k, v in t.items():
            tot[k] = tot.get(k, 0) + v
        L.nolsm_plan_set_timing(p, False)
    return wall, tot


def oracle_sample(inst, runner, O, sample, flops_per_sub):
    """The oracle on `sample` evenly spaced molecules (one submatrix each), timed on
    the host cores; the same results give the GPU path's error on that sample."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    ks = np.linspace(0, inst.nmol - 1, sample).astype(int)
    t0 = time.perf_counter()
    refs = [O.submatrix_result(inst, int(k)) for k in ks]
    dt = time.perf_counter() - t0
    subs_per_s = len(ks) / dt
    cpu = {"value": round(subs_per_s * flops_per_sub / 1e12, 6), "unit": "TFLOP/s",
           "cores": int(cores), "kind": "oracle",
           "submatrices_per_s": round(subs_per_s, 4),
           "sample": f"{len(ks)} evenly spaced submatrices of the same workload "
                     f"({dt:.1f} s); TFLOP/s = the paper-convention sign-iteration FLOPs "
                     f"the GPU schedule counts for those submatrices / oracle time"}
    # error of the GPU result on the same submatrices: block column k of D read back
    # into T_k layout, and the per-column Tr(DH) contributions
    D = runner.D.cpu().numpy()
    st = runner.stats_host()
    pos = {int(k): i for i, k in enumerate(runner.mols)}
    dmax, demax = 0.0, 0.0
    for k, ref in zip(ks, refs):
        got = np.zeros_like(ref["D_cols"])
        for a, I in enumerate(ref["members"]):
            t = int(inst.colptr[k]) + a
            dI = int(inst.blk_dim[I])
            m = int(inst.blk_dim[k])
            blk = D[inst.valoff[t]:inst.valoff[t] + dI * m].reshape(m, dI).T
            got[ref["offs"][a]:ref["offs"][a + 1], :] = blk
        dmax = max(dmax, float(np.abs(got - ref["D_cols"]).max()))
        de = abs(float(st["tr_dh"][pos[int(k)]]) - ref["tr_dh"]) / int(inst.atoms[k])
        demax = max(demax, de)
    err = {"max_abs_dD": dmax, "max_dE_per_atom": demax, "sampled_submatrices": int(len(ks))}
    return cpu, err


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "ns_gemm_rect_fp16_c2_traffic.json")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("ns_gemm.h", "ns_gemm_rect.h"):
        with open(os.path.join(ROOT, "paper_2205_12182_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_summary(fetch_db, write_db, workload, schedule, calib_mib, command):
    """Write the sign GEMM's HBM bytes per launch from two rocprofv3 --pmc databases
    (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by what the same
    counter reads for the plain copy of calib_mib MiB that --calibrate-copy runs."""
    import sqlite3

    def per_kernel(db, counter):
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, kernel_name, value from counters_collection "
                           "where counter_name = ?", (counter,)).fetchall()
        con.close()
        acc = {}
        for did, name, v in rows:
            key = ("square" if "ns_gemm_rect_kernel" in name and "Li0E" in name else
                   "update" if "ns_gemm_rect_kernel" in name and "Li1E" in name else
                   "copy" if "elementwise" in name and "MulFunctor" in name else None)
            if key is None:
                continue
            acc.setdefault(key, {}).setdefault(did, 0.0)
            acc[key][did] += v                   # summed over the counter's instances
        return {k: sorted(d.values()) for k, d in acc.items()}

    f, w = per_kernel(fetch_db, "FETCH_SIZE"), per_kernel(write_db, "WRITE_SIZE")
    nbytes = calib_mib * (1 << 20)
    f_copy, w_copy = f["copy"][len(f["copy"]) // 2], w["copy"][len(w["copy"]) // 2]
    fs, ws = nbytes / (f_copy * 1024.0), nbytes / (w_copy * 1024.0)
    rec = {"kernel": "ns_gemm_rect_kernel<_Float16> (SQUARE and UPDATE), 256x128 tiles",
           "kernel_sources_sha256": kernel_sources_sha256(), "workload": workload,
           "schedule": schedule, "command": command,
           "calibration": {"copy_bytes_read": nbytes, "fetch_kib_read": f_copy,
                           "fetch_scale": round(fs, 3), "copy_bytes_written": nbytes,
                           "write_kib_read": w_copy, "write_scale": round(ws, 3)},
           "dispatches_per_product": len(f["square"])}
    tot = 0.0
    for k in ("square", "update"):
        fb = float(np.mean(f[k])) * 1024.0 * round(fs, 3)
        wb = float(np.mean(w[k])) * 1024.0 * round(ws, 3)
        rec[k] = {"fetch_bytes": fb, "write_bytes": wb}
        tot += fb + wb
    rec["per_launch_bytes"] = tot / 2.0
    with open(TRAFFIC_PATH, "w") as fh:
        json.dump(rec, fh, indent=1)
    log(f"wrote {TRAFFIC_PATH}: {rec['per_launch_bytes'] / 1e9:.2f} GB per launch "
        f"(fetch x{fs:.3f}, write x{ws:.3f})")


def measured_traffic(workload, schedule):
    """HBM bytes per GEMM launch from the committed counter summary, if it was taken
    for this kernel source, workload and schedule (otherwise None)."""
    if not os.path.exists(TRAFFIC_PATH):
        return None
    with open(TRAFFIC_PATH) as fh:
        rec = json.load(fh)
    if (kernel_sources_sha256() != rec["kernel_sources_sha256"] or rec["workload"] != workload
            or rec["schedule"] != schedule):
        return None
    return float(rec["per_launch_bytes"])


def copy_calibration(torch, mib):
    """A plain elementwise copy of known size (read mib MiB, write mib MiB), run three
    times so that hardware byte counters can be scaled against it."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x elementwise copy of {mib} MiB")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=0, help="fixed FP16 iterations (0: to tolerance)")
    ap.add_argument("--prec", default="fp16")
    ap.add_argument("--schedule", choices=("learned", "default"), default=None,
                    help="learned: scaled iteration from the trained network's lower bound "
                         "(the default when trained weights exist); default: unscaled")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of plain FP32 (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=40,
                    help="submatrices the oracle solves on the host (0: skip)")
    ap.add_argument("--graph-steps", type=int, default=2,
                    help="timed replays of the step captured as a HIP graph (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, three elementwise copies of MIB MiB (counter scaling)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the GEMM traffic profile from two rocprofv3 --pmc databases "
                         "(runs nothing on the GPU); with --calibrate-copy, --workload, "
                         "--schedule and --traffic-command")
    ap.add_argument("--traffic-command", default="", help="command recorded in the profile")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1], args.workload,
                        args.schedule or "learned", args.calibrate_copy or 1024,
                        args.traffic_command)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (with more GPUs each would take its own share of "
              "the independent submatrices); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2205_12182_amd import _lib as L
    from paper_2205_12182_amd import learn
    from paper_2205_12182_amd.runner import (Runner, default_mixed_schedule, learned_schedule,
                                             plain_fp32_schedule)
    from workloads import get_config
    if not torch.cuda.is_available():
        print("no GPU: the benchmark needs an MI355X", file=sys.stderr)
        sys.exit(1)
    L.lib()

    t = time.perf_counter()
    inst = get_config(args.workload)
    dims = inst.submatrix_dims()
    log(f"workload {args.workload}: {inst.nmol} molecules, n_k {dims.min()}-{dims.max()}, "
        f"built in {time.perf_counter() - t:.1f} s")
    runner = Runner(inst, batch=args.batch)
    log(f"{len(runner.plans)} batches, workspace {runner.workspace.numel() / 2**30:.1f} GiB")

    weights = os.path.join(os.path.dirname(learn.__file__), "data", "schedule_mlp.npz")
    if args.schedule is None:
        args.schedule = "learned" if (os.path.exists(weights) and not args.iters) else "default"
    predictor = None
    if args.schedule == "learned":
        predictor = learn.ScheduleMLP.load(weights)
        mixed = learned_schedule(prec=args.prec)
    else:
        mixed = default_mixed_schedule(fixed_iters=args.iters or None, prec=args.prec)
    for w in range(args.warmup):
        runner.run(sched=mixed, predictor=predictor)
        torch.cuda.synchronize()
        log(f"warmup {w} done")
    wall, tm = timed_steps(runner, mixed, args.steps, L, torch, predictor)
    log(f"mixed: {wall * 1e3:.1f} ms/step  phases {json.dumps({k: round(v, 1) for k, v in tm.items()})}")
    st = runner.stats_host()
    e_mixed, n_mixed = runner.energy_host()
    flops = paper_flops(st)
    K = len(st)
    gemm_ms = tm["ms_gemm"] / args.steps
    sign_ms = tm["ms_sign"] / args.steps
    exec_flop_step = tm["gemm_flop"] / args.steps

    graph = None
    if args.graph_steps > 0:
        g = runner.capture(sched=mixed, predictor=predictor)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            g.replay()
        torch.cuda.synchronize()
        graph = {"ms_per_step": round((time.perf_counter() - t0) / args.graph_steps * 1e3, 2),
                 "steps": args.graph_steps,
                 "energy_matches_eager": runner.energy_host()[0] == e_mixed}
        log(f"graph replay: {json.dumps(graph)}")
        del g

    cpu, err = None, None
    if args.cpu_sample > 0:
        from oracle import nolsm_oracle as O
        cpu, err = oracle_sample(inst, runner, O, args.cpu_sample, flops / K)
        log(f"cpu baseline: {json.dumps(cpu)}")
        log(f"error vs oracle: {json.dumps(err)}")
    other = None
    if args.schedule == "learned" and args.plain_steps > 0:
        dflt = default_mixed_schedule(prec=args.prec)
        runner.run(sched=dflt)
        wall_d, tm_d = timed_steps(runner, dflt, 1, L, torch)
        st_d = runner.stats_host()
        other = {"ms_per_step": round(wall_d * 1e3, 2),
                 "tflops": round(paper_flops(st_d) / wall_d / 1e12, 3),
                 "sign_ms": round(tm_d["ms_sign"], 2),
                 "iters_mean": round(float(st_d["iters_lo"].mean()), 2),
                 "fallbacks": int(st_d["fell_back"].sum()),
                 "energy_per_atom_diff_vs_learned": abs(runner.energy_host()[0] - e_mixed) / inst.natoms}
        log(f"default schedule: {json.dumps(other)}")
    plain = None
    if args.plain_steps > 0:
        pl = plain_fp32_schedule()
        wall_p, tm_p = timed_steps(runner, pl, args.plain_steps, L, torch)
        st_p = runner.stats_host()
        e_plain, _ = runner.energy_host()
        fl_p = paper_flops(st_p)
        plain = {"ms_per_step": round(wall_p * 1e3, 2),
                 "tflops": round(fl_p / wall_p / 1e12, 3),
                 "sign_phase_tflops": round(fl_p / (tm_p["ms_sign"] / args.plain_steps * 1e-3) / 1e12, 3),
                 "submatrices_per_s": round(K / wall_p, 2),
                 "iters_mean": round(float(st_p["iters_lo"].mean()), 2),
                 "gemm_roofline_frac_fp32": round(tm_p["gemm_flop"] / (tm_p["ms_gemm"] * 1e-3) / 1e12 / FP32_PEAK, 4)
                 if tm_p["ms_gemm"] > 0 else None,
                 "energy_per_atom_diff_vs_mixed": abs(e_plain - e_mixed) / inst.natoms}
        log(f"plain fp32: {json.dumps(plain)}")

    if args.calibrate_copy > 0:
        copy_calibration(torch, args.calibrate_copy)

    # executed MFMA flops of the active tiles (device counter) over the time of every
    # GEMM launch in the timed region (HIP events around each launch)
    achieved = exec_flop_step / (gemm_ms * 1e-3) / 1e12
    n_gemm = tm["n_gemm"] / args.steps
    out = {
        "metric": METRIC,
        "value": round(flops / wall / 1e12, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {inst.nmol} water-like molecules, "
                               f"{int(inst.blk_dim[0])} functions each, r_c {inst.r_cut} A, "
                               f"submatrices n {dims.min()}-{dims.max()}",
                   "batch": args.batch,
                   "schedule": (f"{args.prec} Newton-Schulz " +
                                (f"x{args.iters}" if args.iters else "to ||X^2-I||_F<=0.1 +1") +
                                (", learned lower bound -> scaled iteration (cap 16)"
                                 if args.schedule == "learned" else ", unscaled") +
                                ", Gershgorin scale, FP32 fallback and panel step, FP64 "
                                "Cholesky/L^-1/D columns/traces, set-up and panel products on "
                                "FP16 MFMAs with split (hi + 2^-11 lo) FP32-class operands"),
                   "iters_mean": round(float(st["iters_lo"].mean()), 2),
                   "fallbacks": int(st["fell_back"].sum()),
                   "parallelism": "none (1 GPU)"},
        "submatrices_per_s": round(K / wall, 2),
        "sign_phase_tflops": round(flops / (sign_ms * 1e-3) / 1e12, 3),
        "phase_ms": {k[3:]: round(v / args.steps, 2) for k, v in tm.items() if k.startswith("ms_")},
        "energy": e_mixed, "electrons": n_mixed,
        "error_vs_oracle": err,
        "graph_replay": graph,
        "default_schedule": other,
        "plain_fp32": plain,
        "speedup_vs_plain_fp32": round(plain["ms_per_step"] / (wall * 1e3), 3) if plain else None,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP16_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP16_PEAK, 4),
                     "traffic": measured_traffic(args.workload, args.schedule),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE x2.00 + WRITE_SIZE x1.00, "
                                     "copy-calibrated; profiles/ns_gemm_rect_fp16_c2_traffic.json)",
                     "kernel": "ns_gemm_rect_kernel (symmetric upper-tile FP16 product, 256x128 tiles)",
                     "launches_per_step": n_gemm,
                     "avg_launch_ms": round(gemm_ms / max(n_gemm, 1), 4),
                     "executed_flop_per_step": exec_flop_step,
                     "note": "achieved = executed MFMA flops of active tiles / summed launch time"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
