"""Train and evaluate the learned schedule on slab-in-water geometries.

    python -m paper_2205_12182_amd.train_schedule --train 0:100 --eval 100:120 \
        --per-seed 32 --eval-per-seed 64 --out paper_2205_12182_amd/data/schedule_mlp.npz

Every seed is one geometry of the uneven-batch workload (3,000 water-like
molecules around a slab of 600 five-site units, r_c = 8 A) with a fixed diagonal
shift of S (the per-seed Lanczos estimate of lambda_min is too slow to repeat for
120 geometries; the shift keeps lambda_min(S) >= 0.1 for lambda_min(S0) >= -1.3,
and a submatrix whose S_k is not positive definite is reported and left out).

Further training geometries (--water-seeds): 2,048-molecule water boxes built like the
4,096-molecule benchmark box, with a per-seed diagonal shift in [0.75, 1.5].

Training data: for `per-seed` seeded molecules of each training geometry, the
descriptors (nolsm_features) and the plain FP32 iteration count turned into a
lower-bound label (learn.collect), at mu = 0 and at `mus-per-seed` further chemical
potentials drawn per geometry from --mu-range (a chemical-potential search visits
such values, and the descriptors of M - mu I change with mu).  The network is trained on the GPU with the
library's forward / backward / Adam kernels.  Evaluation: on `eval-per-seed`
molecules of each held-out geometry, plain FP32, the default mixed schedule and
the learned mixed schedule are run on the same submatrices, and iterations, time,
throughput and the density / energy differences against plain FP32 are reported.

All GPU work runs in worker processes (one geometry per task); this process only
dispatches tasks and writes the results.
"""
from __future__ import annotations

import argparse
import ast
import concurrent.futures as cf
import hashlib
import json
import multiprocessing
import os
import sys
import time

import numpy as np

SHIFT = 1.4
WORKLOAD = "c3"
# Additional training geometries: water boxes built like the 4,096-molecule benchmark
# box (13+5+5 functions, r_c = 8 A) but with 2,048 molecules and a per-seed diagonal
# shift drawn from [WATER_SHIFT_LO, WATER_SHIFT_HI], so that the network also sees
# the pure-water environment and a range of overlap conditioning.
WATER_NMOL = 2048
WATER_SHIFT_LO, WATER_SHIFT_HI = 0.75, 1.5


def water_shift(seed: int) -> float:
    u = np.random.default_rng([0x5A1F, seed]).random()
    return round(WATER_SHIFT_LO + (WATER_SHIFT_HI - WATER_SHIFT_LO) * u, 3)


def build(kind: str, seed: int):
    from workloads import get_config
    from workloads.water import water_box
    if kind == "water":
        return water_box(WATER_NMOL, (13, 5, 5), 8.0, seed=seed, shift=water_shift(seed),
                         name=f"water{WATER_NMOL}")
    if kind == "c2":
        return get_config("c2")
    return get_config(WORKLOAD, seed=seed, shift=SHIFT)


def _range(s: str):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


# ----------------------------------------------------------------- worker tasks

def sample_mus(seed: int, count: int, lo: float, hi: float, salt: int = 0x3A5C) -> list:
    """mu = 0 and `count` chemical potentials drawn uniformly from [lo, hi] per seed."""
    rng = np.random.default_rng([salt, seed])
    return [0.0] + [round(float(x), 4) for x in rng.uniform(lo, hi, count)]


def _collect_task(seed, per_seed, tol, extra, kind="slab", mus=(0.0,)):
    from . import learn
    t0 = time.perf_counter()
    inst = build(kind, seed)
    t1 = time.perf_counter()
    mols = learn.pick_molecules(inst.nmol, per_seed, seed)
    feat, lab, iters, ok, mu = learn.collect(inst, mols, tol=tol, extra=extra, mus=mus)
    dims = inst.submatrix_dims()[mols]
    return {"seed": seed, "kind": kind, "mols": mols, "n": dims, "feat": feat, "label": lab,
            "iters": iters, "ok": ok, "mu": mu, "t_build": t1 - t0,
            "t_gpu": time.perf_counter() - t1}


def _train_task(x, t, steps, lr, seed):
    from . import learn
    m = learn.ScheduleMLP(nout=1, seed=seed)
    t0 = time.perf_counter()
    hist = m.fit(x, t, steps=steps, lr=lr)
    dt = time.perf_counter() - t0
    import torch
    pred = m.predict(torch.from_numpy(np.asarray(x, np.float32)).cuda()).cpu().numpy()[:, 0]
    return {"params": m.params.cpu().numpy(), "loss": hist, "t_train": dt, "pred": pred}


def _eval_task(seed, per_seed, params, lower_factor, kind="slab", mu=0.0):
    from . import learn
    inst = build(kind, seed)
    mols = learn.pick_molecules(inst.nmol, per_seed, seed, salt=0xE7A1)
    model = learn.ScheduleMLP(nout=1, params=params)
    res = learn.compare_schedules(inst, mols, model, lower_factor=lower_factor, mu=mu)
    res["seed"] = seed
    res["kind"] = kind
    res["mu"] = mu
    res["n_mean"] = float(inst.submatrix_dims()[mols].mean())
    return res


# ----------------------------------------------------------------- driver

def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train", default="0:100", help="training seeds a:b")
    ap.add_argument("--eval", default="100:120", help="evaluation seeds a:b")
    ap.add_argument("--water-seeds", default="1:41",
                    help="additional training water boxes a:b (empty: none)")
    ap.add_argument("--c2-check", type=int, default=64,
                    help="also evaluate on this many molecules of the 4,096-molecule box (0: skip)")
    ap.add_argument("--per-seed", type=int, default=32)
    ap.add_argument("--eval-per-seed", type=int, default=64)
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lower-factor", type=float, default=0.5)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--extra", type=int, default=2)
    ap.add_argument("--mus-per-seed", type=int, default=2,
                    help="chemical potentials per training geometry besides mu = 0")
    ap.add_argument("--mu-range", default="-0.45:0.02",
                    help="interval lo:hi the extra chemical potentials are drawn from")
    ap.add_argument("--out", required=True, help="weights (.npz); the report goes next to it")
    ap.add_argument("--eval-only", action="store_true",
                    help="skip collection and training: evaluate the weights in --out")
    args = ap.parse_args(argv)

    def say(msg):
        print(f"[train_schedule] {msg}", flush=True)

    ctx = multiprocessing.get_context("spawn")
    t_all = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=args.workers, mp_context=ctx) as pool:
        if args.eval_only:
            with np.load(args.out, allow_pickle=False) as z:
                p = z["params"]
                assert hashlib.sha256(p.tobytes()).hexdigest() == str(z["sha256"])
            tr = {"params": p, "loss": [float("nan"), float("nan")]}
            futs = []
        else:
            mlo, mhi = (float(v) for v in args.mu_range.split(":"))
            futs = [pool.submit(_collect_task, s, args.per_seed, args.tol, args.extra, "slab",
                                sample_mus(s, args.mus_per_seed, mlo, mhi))
                    for s in _range(args.train)]
            if args.water_seeds:
                futs += [pool.submit(_collect_task, s, args.per_seed, args.tol, args.extra, "water",
                                     sample_mus(s + 1000, args.mus_per_seed, mlo, mhi))
                         for s in _range(args.water_seeds)]
        data = []
        for f in cf.as_completed(futs):
            r = f.result()
            data.append(r)
            say(f"collected {r['kind']} seed {r['seed']}: {int(r['ok'].sum())}/{len(r['ok'])} usable, "
                f"plain iters {r['iters'].min()}-{r['iters'].max()}, build {r['t_build']:.1f} s, "
                f"gpu {r['t_gpu']:.1f} s  ({len(data)}/{len(futs)})")
        if not args.eval_only:
            data.sort(key=lambda r: (r["kind"], r["seed"]))
            x = np.concatenate([r["feat"][r["ok"]] for r in data])
            t = np.concatenate([r["label"][r["ok"]] for r in data])
            say(f"training on {len(x)} submatrices, label log10 l in [{t.min():.2f}, {t.max():.2f}]")
            tr = pool.submit(_train_task, x, t, args.steps, args.lr, 0).result()
            resid = tr["pred"] - t
            say(f"trained in {tr['t_train']:.1f} s: loss {tr['loss'][0]:.4f} -> "
                f"{tr['loss'][-1]:.4f}, train rms {np.sqrt(np.mean(resid ** 2)):.3f} (log10)")
        mlo, mhi = (float(v) for v in args.mu_range.split(":"))
        # every held-out geometry at mu = 0 and at one drawn chemical potential
        efuts = [pool.submit(_eval_task, s, args.eval_per_seed, tr["params"], args.lower_factor,
                             "slab", mu)
                 for s in _range(args.eval)
                 for mu in sample_mus(s + 5000, 1, mlo, mhi)]
        c2fut = (pool.submit(_eval_task, 0, args.c2_check, tr["params"], args.lower_factor, "c2")
                 if args.c2_check > 0 else None)
        evals = []
        for f in cf.as_completed(efuts):
            r = f.result()
            evals.append(r)
            say(f"evaluated seed {r['seed']} mu {r['mu']}: "
                f"iters plain {r['plain_fp32']['iters_lo_mean']:.2f} "
                f"default {r['mixed_default']['iters_lo_mean']:.2f} "
                f"learned {r['mixed_learned']['iters_lo_mean']:.2f}  ({len(evals)}/{len(efuts)})")
        c2res = c2fut.result() if c2fut is not None else None
        if c2res is not None:
            say(f"4,096-molecule box: iters plain {c2res['plain_fp32']['iters_lo_mean']:.2f} "
                f"default {c2res['mixed_default']['iters_lo_mean']:.2f} "
                f"learned {c2res['mixed_learned']['iters_lo_mean']:.2f}")
    evals.sort(key=lambda r: (r["seed"], r["mu"]))

    def summarise(sel):
        def agg(name, key, fn=np.mean):
            v = [e[name][key] for e in sel if e[name].get(key) is not None]
            return float(fn(v)) if v else None

        summary = {}
        for name in ("plain_fp32", "mixed_default", "mixed_learned"):
            s = {"iters_lo_mean": agg(name, "iters_lo_mean"),
                 "iters_fb_mean": agg(name, "iters_fb_mean"),
                 "fallbacks": int(sum(e[name]["fallbacks"] for e in sel)),
                 "failed": int(sum(e[name]["failed"] for e in sel)),
                 "ms_sign_total": agg(name, "ms_sign", np.sum),
                 "ms_gemm_total": agg(name, "ms_gemm", np.sum),
                 "sign_tflops_mean": agg(name, "sign_tflops")}
            if name != "plain_fp32":
                s["max_abs_dD_vs_plain"] = agg(name, "max_abs_dD_vs_plain", np.max)
                s["max_dE_per_atom_vs_plain"] = agg(name, "dE_per_atom_vs_plain", np.max)
                s["max_sub_dE_per_atom_vs_plain"] = agg(name, "max_sub_dE_per_atom_vs_plain",
                                                        np.max)
            summary[name] = s
        d, l_ = summary["mixed_default"], summary["mixed_learned"]
        summary["learned_vs_default"] = {
            "iteration_ratio": l_["iters_lo_mean"] / d["iters_lo_mean"],
            "sign_time_ratio": l_["ms_sign_total"] / d["ms_sign_total"]}
        return summary

    summary = summarise(evals)
    summary["at_mu_0"] = summarise([e for e in evals if e["mu"] == 0.0])
    summary["away_from_mu_0"] = summarise([e for e in evals if e["mu"] != 0.0])

    if args.eval_only:
        with np.load(args.out, allow_pickle=False) as z:
            meta = dict(ast.literal_eval(str(z["meta"])))
        meta.update(eval_seeds=args.eval, eval_per_seed=args.eval_per_seed,
                    lower_factor=args.lower_factor)
        digest = hashlib.sha256(np.asarray(tr["params"], np.float32).tobytes()).hexdigest()
    else:
        meta = {"workload": WORKLOAD, "shift": SHIFT, "train_seeds": args.train,
                "eval_seeds": args.eval, "per_seed": args.per_seed, "samples": int(len(x)),
                "steps": args.steps, "lr": args.lr, "tol": args.tol, "extra": args.extra,
                "lower_factor": args.lower_factor, "eval_per_seed": args.eval_per_seed,
                "mus_per_seed": args.mus_per_seed, "mu_range": args.mu_range,
                "water_seeds": args.water_seeds, "water_nmol": WATER_NMOL,
                "water_shift_range": [WATER_SHIFT_LO, WATER_SHIFT_HI],
                "loss_first_last": [float(tr["loss"][0]), float(tr["loss"][-1])],
                "train_rms_log10": float(np.sqrt(np.mean(resid ** 2)))}
        p = np.asarray(tr["params"], np.float32)
        digest = hashlib.sha256(p.tobytes()).hexdigest()
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        np.savez(args.out, params=p, nout=np.int32(1), sha256=np.array(digest),
                 meta=np.array(repr(meta)))
    report = {"meta": meta, "sha256": digest, "summary": summary, "per_seed": evals,
              "box_4096": c2res, "wall_s": time.perf_counter() - t_all}
    rpath = os.path.splitext(args.out)[0] + "_report.json"
    with open(rpath, "w") as fh:
        json.dump(report, fh, indent=1, default=lambda o: o.tolist() if hasattr(o, "tolist") else str(o))
    say(f"wrote {args.out} (sha256 {digest[:12]}) and {rpath}")
    say(json.dumps(summary))
    return 0


if __name__ == "__main__":
    sys.exit(main())
