"""The path at chemical potentials other than 0, the set-up shared between mu
values, and the chemical-potential search (needs an MI355X).

Eq. 5 and Eq. 8 take mu as an input, and the runs of the paper iterate mu until
the system is charge neutral (Sec. V-A).  Inside the gap at mu = 0 the mixed FP16
schedule is held to the accuracy target; inside the bands, where occupations
change and some submatrix has an eigenvalue within 1e-3 of mu, the FP16 rounding
is amplified by 1/gap and only the plain FP32 schedule is compared with the
oracle.  The oracle's smallest per-submatrix gap |lambda - mu| is printed and
checked for every case, so that each case is what it claims to be.
"""
import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import _lib as L
from paper_2205_12182_amd import learn
from paper_2205_12182_amd.runner import (Runner, default_mixed_schedule, learned_schedule,
                                         plain_fp32_schedule)
from workloads import get_config

pytestmark = pytest.mark.gpu

D_TOL, E_TOL = 1e-3, 1e-5
_spec = {}


def spectra(name):
    if name not in _spec:
        inst = get_config(name)
        _spec[name] = (inst, O.submatrix_spectra(inst))
    return _spec[name]


def reference(name, mu):
    inst, sp = spectra(name)
    D = O.density_matrix_at(inst, sp, mu)
    e, ne = O.traces(inst, D, inst.H_val, inst.S_val)
    gap = min(float(np.abs(s["lam"] - mu).min()) for s in sp)
    return inst, D, e, ne, gap


def compare(r, inst, D_ref, e_ref, ne_ref, label):
    D = r.D.cpu().numpy()
    e, ne = r.energy_host()
    dmax = float(np.abs(D - D_ref).max())
    de = abs(e - e_ref) / inst.natoms
    print(f"[case] {label}: dD {dmax:.2e} dE/atom {de:.2e} Tr(DS) {ne:.5f} (oracle {ne_ref:.5f})",
          flush=True)
    return dmax, de, abs(ne - ne_ref)


@pytest.mark.parametrize("name,mus", [("c1", (-0.6, -0.3, 0.15)), ("t_23", (-0.4, -0.1))])
def test_mixed_fp16_inside_gap_shared_setup(gpu_ok, name, mus):
    """One gather and set-up, then the mixed schedule at several mu inside the gap:
    X_0 = (M - mu I)/b and the Gershgorin bound of M - mu I change with mu."""
    r = Runner(get_config(name))
    for t, mu in enumerate(mus):
        inst, D_ref, e_ref, ne_ref, gap = reference(name, mu)
        assert gap > 0.05, (mu, gap)
        r.run(mu=mu, sched=default_mixed_schedule(), regather=(t == 0))
        assert r.check() == L.OK, r.last_check_message
        dmax, de, dn = compare(r, inst, D_ref, e_ref, ne_ref, f"{name} mixed mu {mu} gap {gap:.2e}")
        assert dmax <= D_TOL and de <= E_TOL and dn <= 1e-3


@pytest.mark.parametrize("name,mus", [("c1", (-1.2, -1.15, 0.95)), ("t_23", (0.05,))])
def test_plain_fp32_inside_bands(gpu_ok, name, mus):
    """mu inside the occupied or empty bands: occupations differ from mu = 0 (the
    electron count moves by up to 72), and the plain FP32 iteration meets the target."""
    r = Runner(get_config(name))
    for t, mu in enumerate(mus):
        inst, D_ref, e_ref, ne_ref, gap = reference(name, mu)
        assert gap > 1e-4 and abs(ne_ref - inst.n_elec) > 0.5, (mu, gap, ne_ref)
        r.run(mu=mu, sched=plain_fp32_schedule(), regather=(t == 0))
        assert r.check() == L.OK, r.last_check_message
        dmax, de, dn = compare(r, inst, D_ref, e_ref, ne_ref, f"{name} fp32 mu {mu} gap {gap:.2e}")
        assert dmax <= D_TOL and de <= E_TOL and dn <= 1e-3


def test_setup_reuse_is_exact(gpu_ok):
    """A run at mu2 after a run at mu1 without a new gather and set-up equals a fresh
    run at mu2 bit for bit: one plan, and several persist plans on one workspace."""
    inst = get_config("t_23")
    mu1, mu2 = -0.45, -0.2
    fresh = Runner(inst)
    fresh.run(mu=mu2, sched=default_mixed_schedule())
    one = Runner(inst)
    one.run(mu=mu1, sched=default_mixed_schedule())
    one.run(mu=mu2, sched=default_mixed_schedule(), regather=False)
    split = Runner(inst, batch=48, persist=True)          # three batches
    assert len(split.plans) == 3 and split.keeps_setup
    split.run(mu=mu1, sched=default_mixed_schedule())
    split.run(mu=mu2, sched=default_mixed_schedule(), regather=False)
    torch.cuda.synchronize()
    assert torch.equal(one.D, fresh.D) and torch.equal(one.out2, fresh.out2)
    assert torch.equal(split.D, fresh.D) and torch.equal(split.out2, fresh.out2)
    assert split.check() == L.OK


def test_gershgorin_bound_recomputed_for_another_mu(gpu_ok):
    """Descriptors (which leave their Gershgorin bounds in the plan) at mu1, then the
    sign iteration at mu2: the bounds of M - mu2 I are used, not mu1's."""
    inst = get_config("c1")
    mu1, mu2 = 0.0, -0.7
    r = Runner(inst)
    p = r.plans[0]
    L.nolsm_build_submatrices(p, r.dpat, r.H, r.S)
    feat = torch.empty(inst.nmol, L.NFEAT, device="cuda")
    L.nolsm_features(p, mu1, feat)
    L.nolsm_sign_batched(p, mu2, default_mixed_schedule(), r.stats[0])
    L.nolsm_scatter_density(p, r.dpat, r.D, r.H, r.S, r.stats[0])
    L.nolsm_energy(r.dpat, r.D, r.H, r.S, r.col_traces, r.out2)
    fresh = Runner(inst)
    fresh.run(mu=mu2, sched=default_mixed_schedule())
    torch.cuda.synchronize()
    assert torch.equal(r.D, fresh.D)
    st, st2 = r.stats_host(), fresh.stats_host()
    assert np.array_equal(st["scale"], st2["scale"])


def test_learned_schedule_away_from_zero(gpu_ok):
    """The learned schedule's descriptors and scaled iteration at mu != 0."""
    import os
    w = os.path.join(os.path.dirname(learn.__file__), "data", "schedule_mlp.npz")
    if not os.path.exists(w):
        pytest.skip("no trained weights committed")
    model = learn.ScheduleMLP.load(w)
    for name, mu in (("t_23", -0.35), ("c1", -0.5)):
        inst, D_ref, e_ref, ne_ref, gap = reference(name, mu)
        assert gap > 0.05
        r = Runner(inst)
        r.run(mu=mu, sched=learned_schedule(), predictor=model)
        assert r.check() == L.OK, r.last_check_message
        dmax, de, dn = compare(r, inst, D_ref, e_ref, ne_ref, f"{name} learned mu {mu}")
        assert dmax <= D_TOL and de <= E_TOL and dn <= 1e-3


@pytest.mark.parametrize("name,bracket,persist", [("c1", (-2.9, 1.1), False),
                                                  ("t_23", (-2.6, 1.0), True)])
def test_mu_search_against_oracle(gpu_ok, name, bracket, persist):
    """The bisection on Tr(D S) = N_e on the GPU takes the oracle's trials (every
    trial's electron count is at least 1 electron from a decision threshold, so the
    same decisions are expected) and ends at the same mu with the oracle's D and E
    there.  Trials after the first reuse the gather and set-up."""
    inst, sp = spectra(name)
    ref = O.mu_search(inst, inst.n_elec, *bracket, tol=0.5)
    print(f"[case] {name} oracle mu trials {[(round(m, 5), round(n, 3)) for m, n in ref['hist']]}",
          flush=True)
    assert ref["converged"] and len(ref["hist"]) >= 2
    for _, n in ref["hist"][:-1]:
        assert abs(abs(n - inst.n_elec) - 0.5) > 1.0
    r = Runner(inst, batch=(48 if persist else None), persist=persist)
    m, hist = r.mu_search(inst.n_elec, *bracket, tol=0.5, sched=default_mixed_schedule())
    print(f"[case] {name} gpu mu trials {[(round(a, 5), round(b, 3)) for a, b, _ in hist]}",
          flush=True)
    assert m.done == 1 and [h[0] for h in hist] == [h[0] for h in ref["hist"]]
    assert m.mu == ref["mu"]
    assert r.check() == L.OK, r.last_check_message
    _, D_ref, e_ref, ne_ref, gap = reference(name, m.mu)
    assert gap > 0.05
    dmax, de, dn = compare(r, inst, D_ref, e_ref, ne_ref, f"{name} mu search result {m.mu}")
    assert dmax <= D_TOL and de <= E_TOL and dn <= 1e-3


@pytest.mark.parametrize("name,mu,plain", [("c1", 0.0, False), ("c1", -1.2, True),
                                           ("t_23", -0.4, False), ("t_23", 0.05, True)])
def test_sign_counts_match_inertia(gpu_ok, name, mu, plain):
    """Wrong-sign guard: the count of eigenvalues the iteration sent to -1,
    round((n - Tr X) / 2), equals for every submatrix the number of generalized
    eigenvalues of (H_k, S_k) below mu (the oracle's; by Sylvester's law the
    inertia of H_k - mu S_k), inside the gap and inside the bands."""
    inst, sp = spectra(name)
    r = Runner(inst)
    r.run(mu=mu, sched=plain_fp32_schedule() if plain else default_mixed_schedule())
    assert r.check() == L.OK, r.last_check_message
    st = r.stats_host()
    want = np.array([int(np.sum(s["lam"] < mu)) for s in sp])
    frac = np.abs(0.5 * (st["n"] - st["tr_x"]) - st["n_neg"])
    print(f"[case] {name} mu {mu}: counts {st['n_neg'][:4]}..., largest distance of "
          f"(n - Tr X)/2 from an integer {frac.max():.3f}", flush=True)
    assert np.array_equal(st["n_neg"], want)
    assert frac.max() < 0.25
