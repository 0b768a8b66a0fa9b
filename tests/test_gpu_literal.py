"""The literal form of Eq. 8 on the GPU against the FP64 oracle (needs an MI355X).

Plans made with form = NOLSM_FORM_LITERAL iterate on A_k = S_k^-1 H_k - mu I itself
(non-symmetric; S^-1 H formed in FP64, stored in FP32) with general products and
write T_k(D) = 1/2 (I - sign(A_k)) S_k^-1.  The density is the same as that of the
symmetric congruent form in exact arithmetic, so the tolerances are those of the
symmetric form in plain FP32: within 1e-4 (density) and 1e-6 Ha/atom (energy); an
FP16 bulk meets the energy target (1e-5 Ha/atom) but not always the density target
(see LIT_FP16_D_TOL).  The oracle's own
literal evaluation (an explicit FP64 S^-1) is pinned against its eigen form on the
CPU (tests/test_oracle_pins.py).
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import _lib as L
from paper_2205_12182_amd.runner import Runner, default_mixed_schedule, plain_fp32_schedule
from workloads import get_config

pytestmark = pytest.mark.gpu

D_TOL, E_TOL = 1e-3, 1e-5
_cache = {}


def oracle(name, mu=None):
    key = (name, mu)
    if key not in _cache:
        inst = get_config(name)
        D, _ = O.density_matrix(inst, mu)
        e, ne = O.traces(inst, D, inst.H_val, inst.S_val)
        _cache[key] = (inst, D, e, ne)
    return _cache[key]


def print_case(*a):
    print("[case]", *a, flush=True)


def errors(inst, r, D_ref, e_ref):
    e, ne = r.energy_host()
    return float(np.abs(r.D.cpu().numpy() - D_ref).max()), abs(e - e_ref) / inst.natoms, ne


@pytest.mark.parametrize("name", ["c1", "t_23"])
def test_literal_plain_fp32(gpu_ok, name):
    inst, D_ref, e_ref, ne_ref = oracle(name)
    print_case("literal plain fp32", name)
    r = Runner(inst, form=L.FORM_LITERAL)
    r.run(sched=plain_fp32_schedule())
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, ne = errors(inst, r, D_ref, e_ref)
    st = r.stats_host()
    print_case(name, "literal plain dD", dmax, "dE/atom", de, "iters", int(st["iters_lo"].max()))
    assert dmax < 1e-4 and de < 1e-6 and abs(ne - ne_ref) < 1e-3
    assert np.all(st["status"] == 0) and np.all(st["iters_lo"] > 5)


# The FP16 bulk rounds X_0 = (A_k - mu I) / b to FP16, and the iteration converges to
# the sign of the rounded matrix; no later FP32 step undoes that (a second panel step
# leaves the error unchanged: 2.05e-3 on t_23 either way).  A_k = L^-T (M_k - mu I) L^T
# is not normal: a rounding E of A_k is a perturbation L^T E L^-T of the congruent
# symmetric matrix, up to kappa(L) = kappa(S_k)^(1/2) (about 3 for these overlaps)
# times larger relative to its spectrum, so the literal form's FP16 density errors
# are a few times those of the symmetric form (5e-4 on t_23) and can exceed the 1e-3
# target; the energies stay far inside theirs.  Bounded here at 5e-3.
LIT_FP16_D_TOL = 5e-3


@pytest.mark.parametrize("name", ["c1", "t_tiles", "t_23"])
def test_literal_mixed_fp16(gpu_ok, name):
    """FP16 bulk, FP32 restarts where needed and the FP32 panel step (the default
    mixed schedule of the symmetric form)."""
    inst, D_ref, e_ref, ne_ref = oracle(name)
    print_case("literal mixed fp16", name)
    r = Runner(inst, form=L.FORM_LITERAL)
    r.run(sched=default_mixed_schedule())
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, ne = errors(inst, r, D_ref, e_ref)
    st = r.stats_host()
    print_case(name, "literal mixed dD", dmax, "dE/atom", de, "restarts",
               int(st["fell_back"].sum()))
    assert dmax < LIT_FP16_D_TOL and de < E_TOL


def test_literal_at_other_mu_and_eigenvalue_counts(gpu_ok):
    """A chemical potential inside the valence band (occupations change) and the
    count of eigenvalues sent to -1, against the oracle's count below mu."""
    mu = -0.9
    inst, D_ref, e_ref, ne_ref = oracle("t_23", mu)
    print_case("literal plain fp32 t_23 mu", mu)
    r = Runner(inst, form=L.FORM_LITERAL)
    r.run(mu=mu, sched=plain_fp32_schedule())
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, ne = errors(inst, r, D_ref, e_ref)
    print_case("mu", mu, "literal dD", dmax, "dE/atom", de, "Tr(DS)", ne, "oracle", ne_ref)
    assert dmax < 1e-4 and de < 1e-6 and abs(ne - ne_ref) < 1e-3
    st = r.stats_host()
    for i in [0, inst.nmol // 2, inst.nmol - 1]:
        ref = O.submatrix_result(inst, i, mu=mu)
        assert st["n_neg"][i] == ref["n_occ"], (i, st["n_neg"][i], ref["n_occ"])


def test_literal_matches_symmetric_form(gpu_ok):
    inst = get_config("t_23")
    print_case("literal vs symmetric, plain fp32, t_23")
    rl = Runner(inst, form=L.FORM_LITERAL)
    rl.run(sched=plain_fp32_schedule())
    rs = Runner(inst)
    rs.run(sched=plain_fp32_schedule())
    d = float(np.abs(rl.D.cpu().numpy() - rs.D.cpu().numpy()).max())
    e = abs(rl.energy_host()[0] - rs.energy_host()[0]) / inst.natoms
    print_case("max |D_literal - D_symmetric|", d, "dE/atom", e)
    assert d < 1e-4 and e < 1e-6


def test_literal_setup_and_transposed_iterate(gpu_ok):
    """A0 = S^-1 H (FP32, where the symmetric form keeps M) against FP64 solves of the
    oracle's submatrices, within the FP32 rounding of A0 and the FP32-class rounding
    of the factorisation's tile products; after the iteration buffer 1 holds the
    exact transpose of buffer 0 (the final X and X^T)."""
    inst = get_config("t_23")
    print_case("literal set-up t_23")
    r = Runner(inst, form=L.FORM_LITERAL)
    r.run(sched=plain_fp32_schedule(), energy=False)
    torch.cuda.synchronize()
    for i in [0, inst.nmol // 2, inst.nmol - 1]:
        info = r.sub_info(0, i)
        npad, n = info.npad, info.n
        A0 = r.ws_view(info.off_h, npad * npad, torch.float32).reshape(npad, npad).T.cpu().numpy()
        Hk, _ = O.gather(inst, inst.H_val, info.mol)
        Sk, _ = O.gather(inst, inst.S_val, info.mol)
        ref = np.linalg.solve(Sk, Hk)
        err = float(np.abs(A0[:n, :n].astype(np.float64) - ref).max())
        print_case(f"sub {i}: max |A0 - S^-1 H| {err:.2e} (max |S^-1 H| {np.abs(ref).max():.2f})")
        assert err <= 1e-5 * np.abs(ref).max()
        assert not A0[n:, :].any() and not A0[:, n:].any()
        X = r.ws_view(info.off_lo, npad * npad, torch.float32).reshape(npad, npad).T.cpu().numpy()
        Xt = r.ws_view(info.off_lo + 4 * npad * npad, npad * npad,
                       torch.float32).reshape(npad, npad).T.cpu().numpy()
        assert np.array_equal(Xt, X.T)
        assert np.abs(X[:n, :n] - X[:n, :n].T).max() > 1e-3      # the iterate is not symmetric


def test_literal_schedule_limits(gpu_ok):
    """Two precisions or an order-3 phase are rejected for literal plans."""
    inst = get_config("c1")
    r = Runner(inst, form=L.FORM_LITERAL)
    L.nolsm_build_submatrices(r.plans[0], r.dpat, r.H, r.S)
    two = L.schedule([("fp16", 10, 0.0, 0, 2), ("fp32", 5, 0.0, 0, 2)], fallback_iters=0,
                     panel_steps=0)
    o3 = plain_fp32_schedule(order=3)
    for sched, word in ((two, "one precision"), (o3, "order 3")):
        rc = L.lib().nolsm_sign_batched(r.plans[0], ctypes.c_double(0.0), ctypes.byref(sched),
                                        None, None)
        assert rc == L.EINVAL and word in L.nolsm_last_error()
