#!/usr/bin/env python3
"""Benchmark of the NOLSM hot path on one MI355X.

One step = the whole path for every molecule of the workload at one chemical
potential: gather T_k(H0), T_k(S) -> FP64 set-up -> batched sign iteration ->
panel refinement and density columns -> scatter into D -> Tr(DH), Tr(DS).
Inputs are resident in HBM before the timed region starts.

A chemical-potential iteration (Sec. V-A/V-B: the runs iterate mu until the system
is charge neutral, and the paper times each such iteration) reuses the gather and
set-up of every batch (each batch keeps M_k and L^-1 in a buffer of its own), so
it costs the sign iteration, density columns, scatter and traces only; the line
also reports that time, measured over trial values of mu inside the gap.

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


def method_flops(stats, products_per_iter=2):
    """The algorithmic work of the low-precision sign GEMMs: n^3 per product (every
    product is symmetric, so its upper triangle, n^2/2 outputs of 2n flops each,
    determines it), products_per_iter products per iteration of the phases."""
    n3 = stats["n"].astype(np.float64) ** 3
    return float((products_per_iter * n3 * stats["iters_lo"]).sum())


def paper_flops(stats, products_per_iter=2):
    """2 n^3 per product, two products per Newton-Schulz iteration (Eq. 6; every
    schedule timed here is Newton-Schulz; a third-order phase takes three)."""
    n3 = stats["n"].astype(np.float64) ** 3
    return float((2.0 * products_per_iter * n3 * (stats["iters_lo"] + stats["iters_fb"])).sum())


def timed_steps(runner, sched, steps, L, torch, predictor=None, mu=None):
    for p in runner.plans:
        L.nolsm_plan_get_timings(p, reset=True)
        L.nolsm_plan_set_timing(p, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        runner.run(mu=mu, sched=sched, predictor=predictor)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    tot = {}
    for p in runner.plans:
        t = L.nolsm_plan_get_timings(p, reset=True).as_dict()
        for k, v in t.items():
            tot[k] = tot.get(k, 0) + v
        L.nolsm_plan_set_timing(p, False)
    return wall, tot


def oracle_sample(inst, runner, O, sample, flops_per_sub, mu=None):
    """The oracle on `sample` evenly spaced molecules (one submatrix each), timed on
    the host cores; the same results give the GPU path's error on that sample."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    ks = np.linspace(0, inst.nmol - 1, sample).astype(int)
    t0 = time.perf_counter()
    refs = [O.submatrix_result(inst, int(k), mu=mu) for k in ks]
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
    dmax, demax, wrong = 0.0, 0.0, 0
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
        # wrong-sign guard: the eigenvalues the iteration sent to -1 against the
        # oracle's count of eigenvalues below mu
        wrong += int(st["n_neg"][pos[int(k)]] != ref["n_occ"])
    err = {"max_abs_dD": dmax, "max_dE_per_atom": demax, "sampled_submatrices": int(len(ks)),
           "wrong_sign_counts": wrong}
    return cpu, err


def combination_table(inst, L, torch, args, log_fn, mu=None):
    """Sec. IV-B, Table II on this GPU: the workload without combination and with the
    groups of Eq. 9 and Eq. 10 (p(n) = the autotuner's measured rates), each run
    through the whole path with the default mixed schedule: submatrix count, smallest,
    largest and mean dimension, FLOPs of one multiplication of every submatrix
    (2 n^3), the estimated throughput and speedup from p(n), and the measured
    sign-phase and step times and throughputs."""
    from paper_2205_12182_amd.autotune import rate_table
    from paper_2205_12182_amd.runner import Runner, default_mixed_schedule
    table = rate_table()
    tn = np.array([a for a, _ in table])
    tr = np.array([b for _, b in table])
    hp = L.HostPattern(inst)
    mols = np.arange(inst.nmol, dtype=np.int32)
    sched = default_mixed_schedule()
    rows = {}
    for crit in ("none", "eq9", "eq10"):
        groups = ([[int(k)] for k in mols] if crit == "none" else
                  L.nolsm_combine(hp, mols, 9 if crit == "eq9" else 10,
                                  table if crit == "eq10" else None, args.combine_max_n))
        r = Runner(inst, groups=groups, batch=args.combine_batch)
        ns = np.array([L.nolsm_plan_query(p, i).n for p, b in zip(r.plans, r.batches)
                       for i in range(len(b))], dtype=np.float64)
        r.run(mu=mu, sched=sched)
        torch.cuda.synchronize()
        wall, tm = timed_steps(r, sched, args.combine_steps, L, torch, mu=mu)
        st = r.stats_host()
        e, ne = r.energy_host()
        flops_mult = float((2.0 * ns ** 3).sum())
        est_time = float((2.0 * ns ** 3 / np.interp(ns, tn, tr)).sum())
        sign_s = tm["ms_sign"] / args.combine_steps * 1e-3
        rows[crit] = {"submatrices": int(ns.size), "n_min": int(ns.min()), "n_max": int(ns.max()),
                      "n_mean": round(float(ns.mean()), 1),
                      "pflop_one_multiplication": round(flops_mult / 1e15, 4),
                      "estimated_tflops": round(flops_mult / est_time, 1),
                      "estimated_time_rel": est_time,
                      "ms_per_step": round(wall * 1e3, 2), "sign_ms": round(sign_s * 1e3, 2),
                      "sign_tflops": round(paper_flops(st) / sign_s / 1e12, 1),
                      "step_tflops": round(paper_flops(st) / wall / 1e12, 1),
                      "iters_mean": round(float(st["iters_lo"].mean()), 2),
                      "fallbacks": int(st["fell_back"].sum()),
                      "failed": int((st["status"] != 0).sum()),
                      "energy": e, "electrons": ne}
        log_fn(f"combination {crit}: {json.dumps(rows[crit])}")
        del r
        torch.cuda.empty_cache()
    base = rows["none"]
    for crit in ("eq9", "eq10"):
        rows[crit]["estimated_speedup"] = round(base["estimated_time_rel"] /
                                                rows[crit]["estimated_time_rel"], 3)
        rows[crit]["measured_speedup_sign"] = round(base["sign_ms"] / rows[crit]["sign_ms"], 3)
        rows[crit]["measured_speedup_step"] = round(base["ms_per_step"] / rows[crit]["ms_per_step"], 3)
    for v in rows.values():
        v.pop("estimated_time_rel")
    return {"schedule": "default mixed (fp16 to ||X^2-I||_F<=0.1 +1, unscaled)", "mu": mu,
            "rate_table_n_tflops": [[round(a, 1), round(b, 1)] for a, b in table],
            "max_n": args.combine_max_n, "rows": rows}


def golden_energies(inst, workload, mu):
    """Per-molecule oracle energies of the whole workload at mu (tests/golden), if they
    were written for this exact instance; else None."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_energies import golden_name, instance_digest
    path = os.path.join(ROOT, "tests", "golden",
                        golden_name(workload, None if mu == inst.mu else mu))
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        rec = {k: z[k] for k in z.files}
    if str(rec["instance_sha256"]) != instance_digest(inst):
        log(f"{path} was written for another instance: not used")
        return None
    return rec


def system_errors(inst, runner, st, e_gpu, gold):
    """|E - E_oracle| / N_atoms over the whole system, and the largest single molecule's
    |dE_k| / atoms_k, against the oracle's energies of every molecule."""
    mols = runner.mols
    de_k = np.abs(st["tr_dh"] - gold["tr_dh"][mols]) / inst.atoms[mols]
    return {"system_dE_per_atom": abs(e_gpu - math.fsum(gold["tr_dh"].tolist())) / inst.natoms,
            "max_single_molecule_dE_per_atom": float(de_k.max()),
            "electrons_oracle": math.fsum(gold["tr_ds"].tolist()),
            "molecules": int(len(mols))}


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


def _short_name(name):
    """Readable kernel name of a rocprofv3 record (mangled or demangled)."""
    import re
    for pat, nice in (("ns_gemm_rect_kernelIDF16_Li0E", "ns_gemm_rect_kernel<_Float16, SQUARE>"),
                      ("ns_gemm_rect_kernelIDF16_Li1E", "ns_gemm_rect_kernel<_Float16, UPDATE>")):
        if pat in name:
            return nice
    name = re.sub(r"^void ", "", name)
    return name.split("(")[0]


def trace_summary(trace_csv, fetch_csv=None, write_csv=None, calib_mib=1024, top=24):
    """Markdown summary of a rocprofv3 kernel trace (csv): per-kernel totals, the
    sign GEMM's duration by iteration (launch index within each batch), and, given
    FETCH_SIZE / WRITE_SIZE collections (csv, KiB per dispatch, scaled by the same
    counters on a plain copy of calib_mib MiB), the bytes and rates of the gather
    and scatter kernels."""
    import csv
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    per = {}
    seq = []
    for r in rows:
        k = _short_name(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        per.setdefault(k, []).append(d)
        if k.startswith("ns_gemm_rect_kernel"):
            seq.append((k.endswith("SQUARE>"), d))
    tot = sum(sum(v) for v in per.values())
    out = ["| Kernel | Calls | Total ms | Avg us | % |", "|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append(f"| {k} | {len(v)} | {sum(v):.1f} | {1e3 * sum(v) / len(v):.1f} | "
                   f"{100 * sum(v) / tot:.1f} |")
    sq = [d for is_sq, d in seq if is_sq]
    up = [d for is_sq, d in seq if not is_sq]
    per_batch = None
    for cand in range(30, 0, -1):           # launches per batch: the longest period that fits
        if len(sq) % cand == 0 and len(up) == len(sq) and min(sq[cand - 1::cand]) < 0.2:
            per_batch = cand
            break
    if per_batch:
        S = np.array(sq).reshape(-1, per_batch)
        U = np.array(up).reshape(-1, per_batch)
        out += ["", f"Sign GEMM launches by iteration (mean over {S.shape[0]} batches):", "",
                "| Iteration | SQUARE ms | UPDATE ms |", "|---|---|---|"]
        for t in range(per_batch):
            out.append(f"| {t} | {S[:, t].mean():.3f} | {U[:, t].mean():.3f} |")
    if fetch_csv and write_csv:
        def counters(path):
            acc = {}
            for r in csv.DictReader(open(path)):
                acc.setdefault(_short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
            return acc
        f, w = counters(fetch_csv), counters(write_csv)
        nbytes = calib_mib * (1 << 20)
        cp = [k for k in f if "MulFunctor" in k]          # the copy of --calibrate-copy
        fcopy = max(max(f[k]) for k in cp)
        wcopy = max(max(w[k]) for k in cp)
        fs, ws = nbytes / (fcopy * 1024.0), nbytes / (wcopy * 1024.0)
        out += ["", f"HBM bytes per dispatch (FETCH_SIZE x{fs:.2f}, WRITE_SIZE x{ws:.2f}: the "
                    f"scales that make the counters read the {calib_mib} MiB of a plain copy):", "",
                "| Kernel | Read GB | Written GB | Avg ms (trace) | GB/s | Fraction of 8 TB/s |",
                "|---|---|---|---|---|---|"]
        for k in sorted(f):
            if "elementwise" in k:
                continue
            rb = np.mean(f[k]) * 1024.0 * fs
            wb = np.mean(w.get(k, [0.0])) * 1024.0 * ws
            ms = np.mean(per.get(k, [np.nan]))
            rate = (rb + wb) / (ms * 1e-3) / 1e9
            out.append(f"| {k} | {rb / 1e9:.2f} | {wb / 1e9:.2f} | {ms:.3f} | {rate:.0f} | "
                       f"{rate / 8000.0:.2f} |")
    print("\n".join(out))


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


def workload_text(name, inst, dims):
    if name == "c5":
        kind = (f"{inst.nmol} water-like molecules, {int(inst.blk_dim[0])} functions each "
                f"(streamed in batches)")
    elif name.startswith("c3"):
        kind = (f"{int((inst.blk_dim == 23).sum())} water-like molecules (23 functions) around a "
                f"slab of {int((inst.blk_dim == 30).sum())} five-site units (30 functions)")
    else:
        kind = f"{inst.nmol} water-like molecules, {int(inst.blk_dim[0])} functions each"
    return f"{name}: {kind}, r_c {inst.r_cut} A, submatrices n {dims.min()}-{dims.max()}"


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
    ap.add_argument("--extra", type=int, default=1,
                    help="low-precision iterations after the tolerance is reached")
    ap.add_argument("--panel-steps", type=int, default=1,
                    help="FP32 Newton-Schulz steps on the own-column panel")
    ap.add_argument("--factor-tiles", choices=("fp32", "fp64"), default="fp32",
                    help="precision of the tile products of the set-up's Cholesky factorisation "
                         "and inverse (FP64 storage either way)")
    ap.add_argument("--overlap", action="store_true",
                    help="gather and set up batch i + 1 on a second stream while batch i "
                         "iterates (two shared workspaces; measured no faster on c2)")
    ap.add_argument("--mu-trials", type=int, default=3,
                    help="chemical-potential iterations timed after the first (0: skip)")
    ap.add_argument("--mu-trial-step", type=float, default=-0.03,
                    help="offset between the timed chemical-potential trials")
    ap.add_argument("--mu-search", default="", metavar="LO:HI",
                    help="first search the charge-neutral mu in [LO, HI] (Tr(DS) = N_e within "
                         "half an electron) and run every step there")
    ap.add_argument("--combination", type=int, default=1,
                    help="1: also run the workload without and with submatrix combination "
                         "(Eq. 9, Eq. 10) and report the Table II analogue; 0: skip")
    ap.add_argument("--combine-max-n", type=int, default=6000)
    ap.add_argument("--combine-batch", type=int, default=512)
    ap.add_argument("--combine-steps", type=int, default=2)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, three elementwise copies of MIB MiB (counter scaling)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the GEMM traffic profile from two rocprofv3 --pmc databases "
                         "(runs nothing on the GPU); with --calibrate-copy, --workload, "
                         "--schedule and --traffic-command")
    ap.add_argument("--traffic-command", default="", help="command recorded in the profile")
    ap.add_argument("--trace-summary", nargs="+", metavar="CSV",
                    help="print a markdown summary of a rocprofv3 kernel trace (csv), and with "
                         "two more csv files (FETCH_SIZE, WRITE_SIZE collections) the bytes and "
                         "rates of the kernels they cover (runs nothing on the GPU)")
    args = ap.parse_args()
    if args.trace_summary:
        t = args.trace_summary
        trace_summary(t[0], *(t[1:3] if len(t) >= 3 else (None, None)),
                      calib_mib=args.calibrate_copy or 1024)
        return
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
    runner = Runner(inst, batch=args.batch, persist="auto", overlap=args.overlap,
                    factor_tiles=L.FACTOR_FP64 if args.factor_tiles == "fp64" else
                    L.FACTOR_FP32_TILES)
    overlap_used = runner.overlap
    log(f"{len(runner.plans)} batches, {len(runner.workspaces)} workspaces of "
        f"{runner.workspace.numel() / 2**30:.1f} GiB, set-up buffers "
        + (f"{sum(b.numel() for b in runner.persist_bufs) / 2**30:.1f} GiB" if runner.persist
           else "none (they do not fit: a new mu gathers and sets up again)"))

    weights = os.path.join(os.path.dirname(learn.__file__), "data", "schedule_mlp.npz")
    if args.schedule is None:
        args.schedule = "learned" if (os.path.exists(weights) and not args.iters) else "default"
    predictor = None
    if args.schedule == "learned":
        predictor = learn.ScheduleMLP.load(weights)
        mixed = learned_schedule(prec=args.prec, extra=args.extra, panel_steps=args.panel_steps)
    else:
        mixed = default_mixed_schedule(fixed_iters=args.iters or None, prec=args.prec,
                                       extra=args.extra, panel_steps=args.panel_steps)
    step_mu = inst.mu
    search = None
    if args.mu_search:
        lo, hi = (float(v) for v in args.mu_search.split(":"))
        t_prev = [time.perf_counter()]
        trials = []

        def on_trial(t, mu, ne, e):
            now = time.perf_counter()
            trials.append({"mu": mu, "electrons": ne, "energy": e,
                           "ms": round((now - t_prev[0]) * 1e3, 1)})
            log(f"mu trial {t}: {json.dumps(trials[-1])}")
            t_prev[0] = now
        torch.cuda.synchronize()
        t_prev[0] = time.perf_counter()
        m, _ = runner.mu_search(inst.n_elec, lo, hi, tol=0.5, max_iter=40, sched=mixed,
                                predictor=predictor, on_trial=on_trial)
        step_mu = m.mu
        search = {"bracket": [lo, hi], "n_elec": inst.n_elec, "converged": m.done == 1,
                  "mu": m.mu, "trials": trials}
    for w in range(args.warmup):
        runner.run(mu=step_mu, sched=mixed, predictor=predictor)
        torch.cuda.synchronize()
        log(f"warmup {w} done")
    wall, tm = timed_steps(runner, mixed, args.steps, L, torch, predictor, mu=step_mu)
    log(f"mixed: {wall * 1e3:.1f} ms/step  phases {json.dumps({k: round(v, 1) for k, v in tm.items()})}")
    st = runner.stats_host()
    e_mixed, n_mixed = runner.energy_host()
    failed = int((st["status"] != 0).sum())
    check = runner.check()
    if failed or check != L.OK:
        log(f"{failed} submatrices failed: {runner.last_check_message}")
    flops = paper_flops(st)
    alg_flop_step = method_flops(st)
    K = len(st)
    gemm_ms = tm["ms_gemm"] / args.steps
    sign_ms = tm["ms_sign"] / args.steps
    exec_flop_step = tm["gemm_flop"] / args.steps

    graph = None
    if args.graph_steps > 0:
        g = runner.capture(mu=step_mu, sched=mixed, predictor=predictor)
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

    mu_iter = None
    if args.mu_trials > 0:
        # trial chemical potentials inside the gap at mu = 0, as the last iterations of
        # a charge-neutrality search visit them; the first trial gathers and sets up, the
        # others reuse the set-up where every batch keeps it
        mus = [step_mu + args.mu_trial_step * (t + 1) for t in range(args.mu_trials + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runner.run(mu=mus[0], sched=mixed, predictor=predictor)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        ne = [runner.energy_host()[1]]
        t0 = time.perf_counter()
        for mu in mus[1:]:
            runner.run(mu=mu, sched=mixed, predictor=predictor, regather=False)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.mu_trials
        ne.append(runner.energy_host()[1])
        mu_iter = {"ms": round(per * 1e3, 2), "first_ms": round(first * 1e3, 2),
                   "setup_kept": runner.keeps_setup,
                   "mus": [round(m, 4) for m in mus], "electrons_first_last": ne,
                   "n_elec": inst.n_elec, "failed": int((runner.stats_host()["status"] != 0).sum()),
                   "submatrices_per_s": round(K / per, 2),
                   "tflops": round(paper_flops(runner.stats_host()) / per / 1e12, 3)}
        log(f"mu iterations: {json.dumps(mu_iter)}")
        runner.run(mu=step_mu, sched=mixed, predictor=predictor)    # back to the step's mu
        torch.cuda.synchronize()

    cpu, err = None, None
    if args.cpu_sample > 0:
        from oracle import nolsm_oracle as O
        cpu, err = oracle_sample(inst, runner, O, args.cpu_sample, flops / K, mu=step_mu)
        gold = golden_energies(inst, args.workload, step_mu)
        if gold is not None:
            err.update(system_errors(inst, runner, st, e_mixed, gold))
        log(f"cpu baseline: {json.dumps(cpu)}")
        log(f"error vs oracle: {json.dumps(err)}")
    other = None
    if args.schedule == "learned" and args.plain_steps > 0:
        dflt = default_mixed_schedule(prec=args.prec)
        runner.run(mu=step_mu, sched=dflt)
        wall_d, tm_d = timed_steps(runner, dflt, 1, L, torch, mu=step_mu)
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
        wall_p, tm_p = timed_steps(runner, pl, args.plain_steps, L, torch, mu=step_mu)
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
                 "energy_per_atom_diff_vs_mixed": abs(e_plain - e_mixed) / inst.natoms,
                 "max_single_molecule_diff_vs_mixed": float(
                     (np.abs(st_p["tr_dh"] - st["tr_dh"]) / inst.atoms[runner.mols]).max())}
        log(f"plain fp32: {json.dumps(plain)}")

    if args.calibrate_copy > 0:
        copy_calibration(torch, args.calibrate_copy)

    combo = None
    if args.combination:
        del runner
        torch.cuda.empty_cache()
        combo = combination_table(inst, L, torch, args, log, mu=step_mu)

    # the method's work of the sign GEMMs (n^3 per symmetric product of each active
    # submatrix) over the time of every GEMM launch in the timed region (HIP events
    # around each launch); the executed MFMA flops of the active tiles (device counter:
    # whole tiles across the diagonal, padding to 64) are reported beside it
    achieved = alg_flop_step / (gemm_ms * 1e-3) / 1e12
    executed = exec_flop_step / (gemm_ms * 1e-3) / 1e12
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
        "config": {"workload": workload_text(args.workload, inst, dims),
                   "batch": args.batch,
                   "schedule": (f"{args.prec} Newton-Schulz " +
                                (f"x{args.iters}" if args.iters else f"to ||X^2-I||_F<=0.1 +{args.extra}") +
                                (", learned lower bound -> scaled iteration (cap 16)"
                                 if args.schedule == "learned" else ", unscaled") +
                                f", Gershgorin scale, FP32 fallback, {args.panel_steps} FP32 panel step(s), FP64 "
                                "Cholesky/L^-1 storage (tile products on " +
                                ("FP64" if args.factor_tiles == "fp64" else "FP32") +
                                " MFMAs), FP64 D columns/traces, set-up and panel products on "
                                "FP16 MFMAs with split (hi + 2^-11 lo) FP32-class operands"),
                   "iters_mean": round(float(st["iters_lo"].mean()), 2),
                   "fallbacks": int(st["fell_back"].sum()),
                   "failed": failed,
                   "parallelism": "none (1 GPU)",
                   "overlap": overlap_used},
        "submatrices_per_s": round(K / wall, 2),
        "sign_phase_tflops": round(flops / (sign_ms * 1e-3) / 1e12, 3),
        "phase_ms": {k[3:]: round(v / args.steps, 2) for k, v in tm.items() if k.startswith("ms_")},
        "energy": e_mixed, "electrons": n_mixed, "n_elec": inst.n_elec, "mu": step_mu,
        "mu_search": search,
        "mu_iteration": mu_iter,
        "error_vs_oracle": err,
        "graph_replay": graph,
        "default_schedule": other,
        "plain_fp32": plain,
        "speedup_vs_plain_fp32": round(plain["ms_per_step"] / (wall * 1e3), 3) if plain else None,
        "submatrix_combination": combo,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP16_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP16_PEAK, 4),
                     "traffic": measured_traffic(args.workload, args.schedule),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE x2.00 + WRITE_SIZE x1.00, "
                                     "copy-calibrated; profiles/ns_gemm_rect_fp16_c2_traffic.json)",
                     "kernel": "ns_gemm_rect_kernel (symmetric upper-tile FP16 product, 256x128 tiles)",
                     "launches_per_step": n_gemm,
                     "avg_launch_ms": round(gemm_ms / max(n_gemm, 1), 4),
                     "method_flop_per_step": alg_flop_step,
                     "executed_achieved": round(executed, 2),
                     "executed_frac": round(executed / FP16_PEAK, 4),
                     "executed_flop_per_step": exec_flop_step,
                     "note": "achieved = the method's work (n^3 per symmetric product of each "
                             "active submatrix) / summed launch time; executed_* counts the MFMA "
                             "work the tiles ran (device counter)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if failed or check != L.OK:
        sys.exit(3)


if __name__ == "__main__":
    main()
