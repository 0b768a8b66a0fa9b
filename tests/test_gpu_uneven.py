"""The uneven batch (slab of five-site units in water, submatrices of 1,300-2,800)
through the learned schedule, captured as one HIP graph (needs an MI355X).

A sample of molecules spanning both species is planned as one batch: both GEMM tile
shapes run in the same step.  Graph replays must reproduce the eager result bit for
bit, and sampled submatrices must match the FP64 oracle to the accuracy target.
"""
import os

import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import learn
from paper_2205_12182_amd.runner import Runner, learned_schedule
from workloads import get_config

pytestmark = pytest.mark.gpu

D_TOL, E_TOL = 1e-3, 1e-5
WEIGHTS = os.path.join(os.path.dirname(learn.__file__), "data", "schedule_mlp.npz")


def test_uneven_batch_graph_and_parity(gpu_ok):
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    inst = get_config("c3")
    mols = np.concatenate([np.arange(0, 3000, 60), np.arange(3000, 3600, 12)]).astype(np.int32)
    dims = inst.submatrix_dims()[mols]
    print(f"[case] c3 sample: {mols.size} molecules, n {dims.min()}-{dims.max()}", flush=True)
    model = learn.ScheduleMLP.load(WEIGHTS)
    r = Runner(inst, mols=mols)
    sched = learned_schedule()
    r.run(sched=sched, predictor=model)
    torch.cuda.synchronize()
    D_ref, e_ref, st = r.D.clone(), r.energy_host(), r.stats_host()
    assert (st["status"] == 0).all()
    g = r.capture(sched=sched, predictor=model)
    for rep in range(2):
        r.D.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.D, D_ref), rep
        assert r.energy_host() == e_ref, rep
    D = D_ref.cpu().numpy()
    pos = {int(k): i for i, k in enumerate(mols)}
    picks = [int(mols[0]), int(mols[25]), int(mols[-10]), int(mols[-1])]
    dmax, de, atoms = 0.0, 0.0, 0
    for k in picks:
        ref = O.submatrix_result(inst, k)
        got = np.zeros_like(ref["D_cols"])
        for a, I in enumerate(ref["members"]):
            t = int(inst.colptr[k]) + a
            dI, m = int(inst.blk_dim[I]), int(inst.blk_dim[k])
            got[ref["offs"][a]:ref["offs"][a + 1], :] = \
                D[inst.valoff[t]:inst.valoff[t] + dI * m].reshape(m, dI).T
        dmax = max(dmax, float(np.abs(got - ref["D_cols"]).max()))
        de += float(st["tr_dh"][pos[k]]) - ref["tr_dh"]
        atoms += int(inst.atoms[k])
    print(f"[case] c3 vs oracle: dD {dmax:.2e} dE/atom {abs(de) / atoms:.2e}", flush=True)
    assert dmax <= D_TOL and abs(de) / atoms <= E_TOL
