"""The learned schedule end to end (needs an MI355X).

Training data come from plain FP32 runs of the method on small slab-in-water
geometries; the network is trained with the library's forward / backward / Adam
kernels; on a held-out geometry the learned schedule must need clearly fewer
low-precision iterations than the default schedule while every density element
stays within 1e-3 and the energy within 1e-5 Ha/atom of the FP64 oracle.  The
committed weights (trained on the uneven-batch workload) are checked the same way
on one of their held-out geometries.
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

SHIFT = 1.4
D_TOL, E_TOL = 1e-3, 1e-5
WEIGHTS = os.path.join(os.path.dirname(learn.__file__), "data", "schedule_mlp.npz")


def print_case(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def trained():
    xs, ts = [], []
    for seed in range(4):
        inst = get_config("t_slab", seed=seed, shift=SHIFT)
        mols = learn.pick_molecules(inst.nmol, 160, seed)
        print_case(f"collect t_slab seed {seed}")
        f, lab, iters, ok, _ = learn.collect(inst, mols)
        assert ok.all()
        xs.append(f)
        ts.append(lab)
    x, t = np.concatenate(xs), np.concatenate(ts)
    m = learn.ScheduleMLP(seed=0)
    print_case("train")
    hist = m.fit(x, t, steps=1500)
    return m, x, t, hist


def oracle_errors(inst, r, mols, picks):
    """Largest |dD| over the written columns of `picks`, and the summed |dE_k| of those
    molecules over their atoms (the whole-system measure restricted to the sample,
    without cancellation between molecules)."""
    D = r.D.cpu().numpy()
    st = r.stats_host()
    pos = {int(k): i for i, k in enumerate(mols)}
    dmax, de, atoms = 0.0, 0.0, 0
    for k in picks:
        ref = O.submatrix_result(inst, int(k))
        got = np.zeros_like(ref["D_cols"])
        for a, I in enumerate(ref["members"]):
            t = int(inst.colptr[k]) + a
            dI, m = int(inst.blk_dim[I]), int(inst.blk_dim[k])
            got[ref["offs"][a]:ref["offs"][a + 1], :] = \
                D[inst.valoff[t]:inst.valoff[t] + dI * m].reshape(m, dI).T
        dmax = max(dmax, float(np.abs(got - ref["D_cols"]).max()))
        de += abs(float(st["tr_dh"][pos[int(k)]]) - ref["tr_dh"])
        atoms += int(inst.atoms[k])
    return dmax, abs(de) / atoms


def test_training_fits_labels(gpu_ok, trained):
    m, x, t, hist = trained
    assert hist[-1] < 0.3 * hist[0]
    pred = m.predict(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()[:, 0]
    # better than predicting the mean label by a wide margin (log10 units)
    assert np.sqrt(np.mean((pred - t) ** 2)) < 0.5 * np.std(t)


def test_learned_schedule_gain_and_parity(gpu_ok, trained):
    m = trained[0]
    inst = get_config("t_slab", seed=10, shift=SHIFT)
    mols = learn.pick_molecules(inst.nmol, 64, 10, salt=0xE7A1)
    print_case("compare schedules t_slab seed 10")
    res = learn.compare_schedules(inst, mols, m)
    d, l_ = res["mixed_default"], res["mixed_learned"]
    print_case(f"iters default {d['iters_lo_mean']:.2f} learned {l_['iters_lo_mean']:.2f}")
    assert l_["failed"] == 0 and l_["fallbacks"] == 0
    assert l_["iters_lo_mean"] <= 0.75 * d["iters_lo_mean"]
    assert l_["max_abs_dD_vs_plain"] <= D_TOL and l_["dE_per_atom_vs_plain"] <= E_TOL
    r = Runner(inst, mols=mols)
    r.run(sched=learned_schedule(), predictor=m, energy=False)
    picks = mols[[0, len(mols) // 2, len(mols) - 1]]
    dmax, demax = oracle_errors(inst, r, mols, picks)
    print_case(f"learned vs oracle: dD {dmax:.2e} dE/atom {demax:.2e}")
    assert dmax <= D_TOL and demax <= E_TOL


def test_committed_weights(gpu_ok):
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    m = learn.ScheduleMLP.load(WEIGHTS)          # checks the content hash
    inst = get_config("c3", seed=100, shift=SHIFT)
    mols = learn.pick_molecules(inst.nmol, 16, 100, salt=0x7E57)
    print_case("committed weights on c3 seed 100")
    res = learn.compare_schedules(inst, mols, m)
    d, l_ = res["mixed_default"], res["mixed_learned"]
    print_case(f"iters default {d['iters_lo_mean']:.2f} learned {l_['iters_lo_mean']:.2f}")
    assert l_["failed"] == 0
    assert l_["iters_lo_mean"] <= 0.75 * d["iters_lo_mean"]
    assert l_["max_abs_dD_vs_plain"] <= D_TOL and l_["dE_per_atom_vs_plain"] <= E_TOL
    r = Runner(inst, mols=mols)
    r.run(sched=learned_schedule(), predictor=m, energy=False)
    dmax, demax = oracle_errors(inst, r, mols, mols)
    print_case(f"learned vs oracle: dD {dmax:.2e} dE/atom {demax:.2e}")
    assert dmax <= D_TOL and demax <= E_TOL


def test_committed_weights_away_from_mu_zero(gpu_ok):
    """Trials of a chemical-potential search (mu inside the gap, away from 0): the
    network's lower bound still saves iterations and sends no submatrix to the FP32
    restart, on molecules of the 4,096-molecule benchmark box."""
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights committed")
    m = learn.ScheduleMLP.load(WEIGHTS)
    inst = get_config("c2")
    mols = np.arange(0, inst.nmol, 64, dtype=np.int32)
    for mu in (-0.1, -0.25):
        res = learn.compare_schedules(inst, mols, m, mu=mu)
        d, l_ = res["mixed_default"], res["mixed_learned"]
        print_case(f"c2 mu {mu}: iters default {d['iters_lo_mean']:.2f} learned "
                   f"{l_['iters_lo_mean']:.2f} restarts {l_['fallbacks']}")
        assert l_["failed"] == 0 and l_["fallbacks"] == 0
        assert l_["iters_lo_mean"] <= 0.8 * d["iters_lo_mean"]
        assert l_["max_abs_dD_vs_plain"] <= D_TOL and l_["dE_per_atom_vs_plain"] <= E_TOL
