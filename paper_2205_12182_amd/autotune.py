"""Tile-shape autotuner for the sign-iteration GEMM.

    python -m paper_2205_12182_amd.autotune --out paper_2205_12182_amd/data/tile_policy.json

GEMM throughput depends on the submatrix size (paper, Sec. IV-B and Table II).  For a
sweep of sizes (water boxes of 1,024 molecules with 13+5+5 functions and a range of
cutoff radii), the FP16 products of a fixed number of Newton-Schulz iterations are
timed with every submatrix on 128 x 128 tiles and with every submatrix on 256 x 128
tiles (HIP events around each launch; executed MFMA flops from the device counter).
The policy is the smallest padded dimension from which the 256 x 128 kernel takes less
time per launch at every measured size above it; the table of rates (this GPU's p(n)) is stored with
it.  Runner applies the stored policy to every plan it creates, provided it was
measured on the same GPU architecture (the file records the gfx target, the HIP and
PyTorch versions and a digest of the GEMM kernel sources it was measured with).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

RADII = (4.5, 5.0, 5.5, 6.0, 6.5, 7.0, 7.5, 8.0, 9.0, 10.0)
POLICY_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "tile_policy.json")
GEMM_SOURCES = ("ns_gemm.h", "ns_gemm_rect.h", "sign.hip")
NMOL, SHIFT, ITERS = 1024, 1.5, 4
NEVER = 1 << 20


def measure(r_cut: float, batch: int, say) -> dict:
    import torch
    from . import _lib as L
    from .runner import Runner
    from workloads.water import water_box
    inst = water_box(NMOL, (13, 5, 5), r_cut, seed=7, shift=SHIFT, name="tune")
    dims = inst.submatrix_dims()
    npad = int((dims.max() + 63) // 64 * 64)
    # keep the workspace (28 bytes per padded element and submatrix) near 60 GB
    batch = max(64, min(batch, int(60e9 // (28 * npad * npad))))
    mols = np.arange(min(batch, inst.nmol), dtype=np.int32)
    sched = L.schedule([("fp16", ITERS, 0.0, 0)], fallback_iters=0, panel_steps=0)
    rec = {"r_cut": r_cut, "submatrices": int(mols.size), "n_mean": float(dims[mols].mean()),
           "npad_mean": float(((dims[mols] + 63) // 64 * 64).mean())}
    for name, big in (("tile128", NEVER), ("tile256x128", 0)):
        r = Runner(inst, mols=mols, big_tile_min_npad=big)
        p = r.plans[0]
        r.run(sched=sched, energy=False)
        torch.cuda.synchronize()
        L.nolsm_plan_get_timings(p, reset=True)
        L.nolsm_plan_set_timing(p, True)
        for _ in range(2):
            r.run(sched=sched, energy=False)
        torch.cuda.synchronize()
        t = L.nolsm_plan_get_timings(p, reset=True).as_dict()
        L.nolsm_plan_set_timing(p, False)
        rec[name] = {"tflops_executed": t["gemm_flop"] / (t["ms_gemm"] * 1e-3) / 1e12,
                     "ms_per_launch": t["ms_gemm"] / max(t["n_gemm"], 1)}
        del r
    say(f"r_c {r_cut}: n {rec['n_mean']:.0f}  128x128 {rec['tile128']['tflops_executed']:.0f} TF/s"
        f"  256x128 {rec['tile256x128']['tflops_executed']:.0f} TF/s")
    return rec


def gemm_sources_digest() -> str:
    """sha256 over the sign-GEMM kernel sources (first 16 hex digits)."""
    import hashlib
    h = hashlib.sha256()
    for name in GEMM_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", name),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def target_key() -> dict:
    """What a policy is measured on: gfx target, HIP and PyTorch versions, kernels."""
    import torch
    return {"gfx_arch": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
            "hip_version": str(torch.version.hip), "torch_version": torch.__version__,
            "kernel_sha256": gemm_sources_digest()}


def policy_applies(policy: dict, gfx_arch: str) -> tuple:
    """(usable, note): a policy applies on the architecture it was measured on; one
    without a recorded target is taken as it is.  A changed kernel digest is noted
    (the crossover may have moved) but does not void the policy."""
    key = policy.get("target")
    if not key:
        return True, ""
    if key.get("gfx_arch") != gfx_arch:
        return False, f"measured on {key.get('gfx_arch')}, this GPU is {gfx_arch}"
    if key.get("kernel_sha256") != gemm_sources_digest():
        return True, "the GEMM kernel sources changed since the measurement"
    return True, ""


def rate_table(policy: dict | None = None) -> list:
    """p(n) of Sec. IV-B from the stored measurements: for each measured size, the
    sign-GEMM throughput in the paper's accounting (2 n^3 per product and submatrix)
    with the tile shape the policy picks there, [(n_mean, TFLOP/s), ...] ascending.
    Eq. 10 combines submatrices on the predicted time n^3 / p(n)."""
    if policy is None:
        with open(POLICY_PATH) as fh:
            policy = json.load(fh)
    out = []
    for m in sorted(policy["measurements"], key=lambda r: r["n_mean"]):
        key = "tile256x128" if m["npad_mean"] >= policy["big_tile_min_npad"] else "tile128"
        t = m[key]["ms_per_launch"] * 1e-3
        out.append((float(m["n_mean"]), 2.0 * m["submatrices"] * m["n_mean"] ** 3 / t / 1e12))
    return out


def choose(recs) -> int:
    """Smallest mean padded size from which the large tiles take less time per launch
    at every larger size.  Both kernels form the same products; their executed-flop
    rates are not comparable, since the large tiles skip the blocks of diagonal tiles
    that lie wholly below the diagonal and the 128 x 128 tiles do not."""
    recs = sorted(recs, key=lambda r: r["npad_mean"])
    big_min = NEVER
    for r in reversed(recs):
        if r["tile256x128"]["ms_per_launch"] < r["tile128"]["ms_per_launch"]:
            big_min = int(r["npad_mean"] // 64 * 64)
        else:
            break
    return big_min


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--batch", type=int, default=512, help="submatrices per measurement")
    args = ap.parse_args(argv)

    def say(msg):
        print(f"[autotune] {msg}", flush=True)

    t0 = time.perf_counter()
    recs = [measure(rc, args.batch, say) for rc in RADII]
    big_min = choose(recs)
    out = {"big_tile_min_npad": big_min, "iterations": ITERS, "batch": args.batch,
           "target": target_key(), "measurements": recs, "wall_s": time.perf_counter() - t0}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    say(f"big_tile_min_npad = {big_min}; wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
