"""Uneven batches through the learned schedule, captured as one HIP graph (needs an
MI355X).

* The slab of five-site units in water (c3, submatrices of 1,311-2,801): a sample of
  molecules spanning both species as one batch.  Every submatrix is above the tuned
  tile threshold (npad 448), so one tile shape runs.
* Five water boxes with cutoffs of 3.2-7 A side by side (t_sweep, submatrices of
  69-989): the batch straddles the tuned threshold, so every product launches the
  128 x 128 tiles of the small submatrices and the 256 x 128 tiles of the large ones
  in the same step.

Graph replays must reproduce the eager result bit for bit, and the result must
match the FP64 oracle to the accuracy target: every written density element within
1e-3 (sampled molecules), and the energy of everything computed -- the whole batch
-- within 1e-5 Ha/atom (the oracle's energies of every c3 molecule are stored in
tests/golden).  A single molecule's energy carries first-order FP16 rounding that
the batch's sum does not; its |dE_k| / atoms_k is printed and bounded at 1e-4.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import learn
from paper_2205_12182_amd.runner import Runner, learned_schedule, tuned_tile_policy
from tests.helpers import golden_energies
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
    dmax, _, _ = per_molecule_errors(inst, D, st, picks, pos)
    # the energy of the whole batch (every molecule computed) against the oracle's
    # energies of the same molecules, and every single molecule
    gold = golden_energies("c3", inst)
    de_batch = abs(e_ref[0] - math.fsum(gold["tr_dh"][mols].tolist())) / inst.atoms[mols].sum()
    de_each = np.abs(st["tr_dh"] - gold["tr_dh"][mols]) / inst.atoms[mols]
    print(f"[case] c3 vs oracle: dD {dmax:.2e} batch dE/atom {de_batch:.2e} "
          f"largest single molecule {de_each.max():.2e}", flush=True)
    assert dmax <= D_TOL and de_batch <= E_TOL and de_each.max() <= SINGLE_E_TOL


# A single molecule's energy carries less cancellation of FP16 rounding than a sum
# over many; on the slab geometries it reaches a few 1e-5 Ha/atom (about 5e-5 was
# the largest seen over 1,280 held-out submatrices against plain FP32).
SINGLE_E_TOL = 1e-4


def per_molecule_errors(inst, D, st, picks, pos):
    """max |D - D_oracle| over the written columns of `picks`, sum |dE_k| / sum atoms_k,
    and max |dE_k| / atoms_k, with dE_k the molecule's Tr(D H) column contribution."""
    dmax, de_abs, atoms, de_max = 0.0, 0.0, 0, 0.0
    for k in picks:
        ref = O.submatrix_result(inst, k)
        got = np.zeros_like(ref["D_cols"])
        for a, I in enumerate(ref["members"]):
            t = int(inst.colptr[k]) + a
            dI, m = int(inst.blk_dim[I]), int(inst.blk_dim[k])
            got[ref["offs"][a]:ref["offs"][a + 1], :] = \
                D[inst.valoff[t]:inst.valoff[t] + dI * m].reshape(m, dI).T
        dmax = max(dmax, float(np.abs(got - ref["D_cols"]).max()))
        assert st["n_neg"][pos[k]] == ref["n_occ"], k      # no wrong-sign convergence
        dk = abs(float(st["tr_dh"][pos[k]]) - ref["tr_dh"])
        de_abs += dk
        atoms += int(inst.atoms[k])
        de_max = max(de_max, dk / int(inst.atoms[k]))
    return dmax, de_abs / atoms, de_max


def test_batch_straddling_tile_threshold(gpu_ok):
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    inst = get_config("t_sweep")
    dims = inst.submatrix_dims()
    npad = (dims + 63) // 64 * 64
    thr = tuned_tile_policy()
    small, large = int((npad < thr).sum()), int((npad >= thr).sum())
    print(f"[case] t_sweep: {inst.nmol} molecules, n {dims.min()}-{dims.max()}, "
          f"{small} below and {large} at or above npad {thr}", flush=True)
    assert small > 0 and large > 0
    model = learn.ScheduleMLP.load(WEIGHTS)
    r = Runner(inst)
    sched = learned_schedule()
    r.run(sched=sched, predictor=model)
    torch.cuda.synchronize()
    D_ref, e_ref, st = r.D.clone(), r.energy_host(), r.stats_host()
    assert (st["status"] == 0).all() and r.check() == 0
    g = r.capture(sched=sched, predictor=model)
    for rep in range(3):
        r.D.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.D, D_ref), rep
        assert r.energy_host() == e_ref, rep
    Do, _ = O.density_matrix(inst)
    eo, neo = O.traces(inst, Do, inst.H_val, inst.S_val)
    dmax = float(np.abs(D_ref.cpu().numpy() - Do).max())
    de = abs(e_ref[0] - eo) / inst.natoms
    picks = list(range(0, inst.nmol, 16))
    _, de_sum, de_max = per_molecule_errors(inst, D_ref.cpu().numpy(), st, picks,
                                            {k: k for k in picks})
    print(f"[case] t_sweep vs oracle: dD {dmax:.2e} dE/atom {de:.2e} sampled sum|dE|/atoms "
          f"{de_sum:.2e} max single {de_max:.2e} iterations {st['iters_lo'].mean():.2f} "
          f"restarts {int(st['fell_back'].sum())}", flush=True)
    assert dmax <= D_TOL and de <= E_TOL and de_sum <= E_TOL and de_max <= SINGLE_E_TOL


def test_c3_full_size_at_charge_neutral_mu(gpu_ok):
    """All 3,600 molecules of the uneven workload (n 1,265-2,988) in the benchmark's
    configuration (batches of 1,024 with their set-ups kept, learned schedule): the
    chemical-potential search finds a charge-neutral mu (at mu = 0 the slab holds 14
    electrons too many), and the whole system's energy there matches the oracle's
    energies of every molecule at that mu (stored, tests/golden)."""
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    torch.cuda.empty_cache()
    inst = get_config("c3")
    model = learn.ScheduleMLP.load(WEIGHTS)
    r = Runner(inst, batch=1024, persist=True)
    print(f"[case] c3 full size, mu search in [-0.6, 0.1], {len(r.plans)} batches", flush=True)
    m, hist = r.mu_search(inst.n_elec, -0.6, 0.1, tol=0.5, sched=learned_schedule(),
                          predictor=model)
    assert m.done == 1 and r.check() == 0, r.last_check_message
    e, ne = r.energy_host()
    gold = golden_energies("c3", inst, mu=m.mu)
    st = r.stats_host()
    de_sys = abs(e - math.fsum(gold["tr_dh"].tolist())) / inst.natoms
    de_each = np.abs(st["tr_dh"] - gold["tr_dh"]) / inst.atoms
    print(f"[case] c3 mu {m.mu} after {m.iters} trials: N {ne:.4f} (oracle "
          f"{math.fsum(gold['tr_ds'].tolist()):.4f}), system dE/atom {de_sys:.2e}, largest "
          f"molecule {de_each.max():.2e}", flush=True)
    assert abs(ne - inst.n_elec) <= 0.5
    assert de_sys <= E_TOL and de_each.max() <= SINGLE_E_TOL
    picks = [0, 1500, 2999, 3000, 3599]
    D = r.D.cpu().numpy()
    dmax = 0.0
    for k in picks:
        ref = O.submatrix_result(inst, k, mu=m.mu)
        assert st["n_neg"][k] == ref["n_occ"], k
        got = np.zeros_like(ref["D_cols"])
        for a, I in enumerate(ref["members"]):
            t = int(inst.colptr[k]) + a
            dI, mm = int(inst.blk_dim[I]), int(inst.blk_dim[k])
            got[ref["offs"][a]:ref["offs"][a + 1], :] = \
                D[inst.valoff[t]:inst.valoff[t] + dI * mm].reshape(mm, dI).T
        dmax = max(dmax, float(np.abs(got - ref["D_cols"]).max()))
    print(f"[case] c3 sampled dD {dmax:.2e}", flush=True)
    assert dmax <= D_TOL
    del r
    torch.cuda.empty_cache()
