"""Compute the diagonal shift delta of S for named workloads.

    python -m workloads.shift_table c1 c2 ...

Builds each workload with delta = 0, estimates lambda_min(S0) (dense eigvalsh up
to 3,000 functions, ARPACK Lanczos above), and prints the table entries for
workloads/configs.py.  delta = max(0, 0.1 - lambda_min) rounded up to 1e-3.
"""
import sys
import time

from .configs import get_config
from .water import lambda_min, shift_for


def main(names, seeds=(0,)):
    for name in names:
        for seed in seeds:
            t = time.time()
            inst = get_config(name, seed=seed, shift=0.0)
            blk = (inst.blk_dim, inst.blk_off, inst.colptr, inst.rowblk, inst.valoff)
            lm = lambda_min(blk, inst.S_val, inst.nfunc)
            print(f"    ({name!r}, {seed}): {shift_for(lm)!r},   # lambda_min(S0) = {lm:.6f}"
                  f"  [{time.time() - t:.0f} s]", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    seeds = (0,)
    if "--seeds" in args:
        i = args.index("--seeds")
        a, b = args[i + 1].split(":")
        seeds = tuple(range(int(a), int(b)))
        args = args[:i] + args[i + 2:]
    main(args, seeds)
