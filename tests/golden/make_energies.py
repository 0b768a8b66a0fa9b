"""Per-molecule energies of the FP64 oracle for a whole named workload.

    python -m tests.golden.make_energies c2 [--workers 6] [--mu MU]

For every molecule k, the oracle's contribution of block column k to Tr(D H0) and
Tr(D S) (Eq. 4 and the electron count, Eq. 8 per submatrix) at the workload's mu
(or --mu; the file name then carries it),
the submatrix dimension and the gap min |lambda - mu|.  Only `oracle/` computes
anything here; the inputs come from the seeded generators in `workloads/`.  The
file records a SHA-256 of the generated H0 and S values, so a test can tell whether
the generator still produces the same instance.
"""
import argparse
import hashlib
import os
import sys
import time

# one BLAS thread per worker process (set before numpy loads its BLAS)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_inst = None


def instance_digest(inst) -> str:
    h = hashlib.sha256()
    for a in (inst.blk_dim, inst.colptr, inst.rowblk, inst.valoff, inst.H_val, inst.S_val):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


_mu = None


def golden_name(workload, mu=None):
    return f"{workload}_energies.npz" if mu is None else f"{workload}_mu{mu:+.4f}_energies.npz"


def _work(ks):
    from oracle import nolsm_oracle as O
    out = []
    for k in ks:
        r = O.submatrix_result(_inst, int(k), mu=_mu)
        out.append((int(k), r["tr_dh"], r["tr_ds"], r["n"], r["gap"]))
    return out


def main():
    global _inst, _mu
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--mu", type=float, default=None)
    args = ap.parse_args()
    _mu = args.mu
    import multiprocessing as mp
    from workloads import get_config
    t0 = time.time()
    _inst = get_config(args.workload)
    chunks = np.array_split(np.arange(_inst.nmol), 8 * args.workers)
    res = []
    with mp.get_context("fork").Pool(args.workers) as pool:
        for part in pool.imap_unordered(_work, chunks):
            res.extend(part)
            print(f"{len(res)}/{_inst.nmol} molecules, {time.time() - t0:.0f} s", flush=True)
    res.sort()
    k, eh, es, n, gap = (np.array(x) for x in zip(*res))
    assert np.array_equal(k, np.arange(_inst.nmol))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        golden_name(args.workload, args.mu))
    mu = _inst.mu if args.mu is None else args.mu
    cmd = f"python -m tests.golden.make_energies {args.workload}" + (
        "" if args.mu is None else f" --mu {args.mu}")
    np.savez(path, workload=args.workload, seed=0, shift=_inst.shift, mu=mu,
             instance_sha256=instance_digest(_inst), tr_dh=eh, tr_ds=es, n=n, gap=gap,
             atoms=_inst.atoms, command=cmd)
    print(f"wrote {path}: E = {eh.sum():.10f}, N = {es.sum():.6f} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
