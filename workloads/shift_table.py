"""Compute the diagonal shift delta of S for named workloads.

    python -m workloads.shift_table c1 c2 ...
    python -m workloads.shift_table --device cuda c2 c5

Builds each workload with delta = 0, estimates lambda_min(S0) and prints the table
entries for workloads/configs.py.  delta = max(0, 0.1 - lambda_min) rounded up to
1e-3.  On the host: dense eigvalsh up to 3,000 functions, ARPACK Lanczos above.
With --device: Lanczos with full reorthogonalisation, the matrix-vector products
on that PyTorch device (the 65,536-molecule box, whose host-side products are too
slow for ARPACK); the residual bound of the smallest Ritz value is printed with it.
"""
import sys
import time

from .configs import get_config
from .water import lambda_min, lambda_min_lanczos, shift_for


def main(names, seeds=(0,), device=None):
    for name in names:
        for seed in seeds:
            t = time.time()
            print(f"[shift_table] building {name} seed {seed}", file=sys.stderr, flush=True)
            inst = get_config(name, seed=seed, shift=0.0)
            built = time.time() - t
            blk = (inst.blk_dim, inst.blk_off, inst.colptr, inst.rowblk, inst.valoff)
            how = ""
            if device is None:
                lm = lambda_min(blk, inst.S_val, inst.nfunc)
            else:
                lm, res, steps = lambda_min_lanczos(
                    blk, inst.S_val, inst.nfunc, device,
                    log=lambda m: print(f"[shift_table] {name}: {m}", file=sys.stderr, flush=True))
                how = f" (Lanczos on {device}: {steps} steps, residual {res:.1e})"
            print(f"    ({name!r}, {seed}): {shift_for(lm)!r},   # lambda_min(S0) = {lm:.6f}"
                  f"{how}  [built {built:.0f} s, total {time.time() - t:.0f} s]", flush=True)
            del inst


if __name__ == "__main__":
    args = sys.argv[1:]
    seeds = (0,)
    device = None
    if "--seeds" in args:
        i = args.index("--seeds")
        a, b = args[i + 1].split(":")
        seeds = tuple(range(int(a), int(b)))
        args = args[:i] + args[i + 2:]
    if "--device" in args:
        i = args.index("--device")
        device = args[i + 1]
        args = args[:i] + args[i + 2:]
    main(args, seeds, device)
