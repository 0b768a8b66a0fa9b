"""Combined submatrices (Sec. IV-B, Eq. 9 and Eq. 10) on the GPU against the FP64
oracle evaluated on the same groups (needs an MI355X).

The groups come from the library's combination heuristic, which the CPU tests hold
to the oracle's greedy scan bit for bit.  Each group shares one submatrix (the union
of its molecules' rows) and every molecule of the group writes its block column
from it, so the density differs from the one-molecule-per-submatrix density by the
larger submatrices' better approximation, and the oracle is evaluated on the same
groups.  Tolerances are the accuracy target (density elements within 1e-3, energy
within 1e-5 Ha/atom; plain FP32 tighter).
"""
import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import _lib as L
from paper_2205_12182_amd.runner import Runner, default_mixed_schedule, plain_fp32_schedule
from workloads import get_config

pytestmark = pytest.mark.gpu

D_TOL, E_TOL = 1e-3, 1e-5
RATE_TABLE = [(341.0, 150.0), (603.0, 420.0), (1243.0, 900.0), (2404.0, 1500.0), (3190.0, 1700.0)]


def check(r, inst, groups, label, dtol, etol):
    D_ref, recs = O.density_matrix_groups(inst, groups)
    e_ref, ne_ref = O.traces(inst, D_ref, inst.H_val, inst.S_val)
    D = r.D.cpu().numpy()
    e, ne = r.energy_host()
    st = r.stats_host()
    dmax = float(np.abs(D - D_ref).max())
    de = abs(e - e_ref) / inst.natoms
    # per-submatrix traces: the sum of the group's column contributions
    tr = np.array([sum(t[0] for t in rec["traces"]) for rec in recs])
    dtr = float(np.abs(st["tr_dh"] - tr).max())
    print(f"[case] {label}: {len(groups)} submatrices (n {min(x['n'] for x in recs)}-"
          f"{max(x['n'] for x in recs)}), dD {dmax:.2e} dE/atom {de:.2e} "
          f"Tr(DS) {ne:.5f} (oracle {ne_ref:.5f}) per-submatrix Tr(DH) {dtr:.2e}", flush=True)
    assert (st["status"] == 0).all() and r.check() == L.OK
    assert dmax <= dtol and de <= etol and abs(ne - ne_ref) <= 1e-3 and dtr <= 1e3 * etol


@pytest.mark.parametrize("criterion,max_n", [(9, 0), (10, 1200)])
def test_combined_submatrices_mixed(gpu_ok, criterion, max_n):
    inst = get_config("t_sweep")
    hp = L.HostPattern(inst)
    groups = L.nolsm_combine(hp, np.arange(inst.nmol, dtype=np.int32), criterion,
                             RATE_TABLE if criterion == 10 else None, max_n)
    assert len(groups) < inst.nmol and max(len(g) for g in groups) > 1
    r = Runner(inst, groups=groups)
    r.run(sched=default_mixed_schedule())
    check(r, inst, groups, f"t_sweep eq{criterion} mixed", D_TOL, E_TOL)


def test_combined_submatrices_plain_fp32_batched_persist(gpu_ok):
    """Plain FP32, three batches of groups with their set-ups kept (persist)."""
    inst = get_config("t_23")
    hp = L.HostPattern(inst)
    groups = L.nolsm_combine(hp, np.arange(inst.nmol, dtype=np.int32), 10, RATE_TABLE, 2400)
    assert max(len(g) for g in groups) > 1
    r = Runner(inst, groups=groups, batch=max(1, len(groups) // 3 + 1), persist=True)
    r.run(sched=plain_fp32_schedule())
    check(r, inst, groups, "t_23 eq10 fp32", 1e-4, 1e-6)


def test_singleton_groups_equal_molecule_plan(gpu_ok):
    """One molecule per group is the plain per-molecule plan, bit for bit (the
    general scatter reproduces the per-molecule one)."""
    inst = get_config("c1")
    a = Runner(inst)
    b = Runner(inst, groups=[[k] for k in range(inst.nmol)])
    a.run(sched=default_mixed_schedule())
    b.run(sched=default_mixed_schedule())
    torch.cuda.synchronize()
    assert torch.equal(a.D, b.D) and torch.equal(a.out2, b.out2)
    assert np.array_equal(a.stats_host()["tr_dh"], b.stats_host()["tr_dh"])


def test_combined_graph_replay(gpu_ok):
    inst = get_config("t_sweep")
    hp = L.HostPattern(inst)
    groups = L.nolsm_combine(hp, np.arange(inst.nmol, dtype=np.int32), 9)
    r = Runner(inst, groups=groups)
    sched = default_mixed_schedule()
    r.run(sched=sched)
    torch.cuda.synchronize()
    D0, E0 = r.D.clone(), r.out2.clone()
    g = r.capture(sched=sched)
    for rep in range(3):
        r.D.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.D, D0) and torch.equal(r.out2, E0), rep
