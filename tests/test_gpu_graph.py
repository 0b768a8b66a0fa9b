"""A whole step captured as a HIP graph and replayed (needs an MI355X).

Three batches share one workspace inside the capture.  Each replay, with eager
work on the same buffers between replays, must reproduce the eager results bit
for bit (the path is deterministic), and the eager path must still work after.
"""
import numpy as np
import pytest
import torch

from paper_2205_12182_amd import _lib as L
from paper_2205_12182_amd.runner import Runner, default_mixed_schedule
from workloads import get_config

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager(gpu_ok):
    inst = get_config("t_tiles")
    print("[case] graph t_tiles, 3 batches", flush=True)
    r = Runner(inst, batch=inst.nmol // 3 + 1)
    assert len(r.plans) == 3
    sched = default_mixed_schedule()
    r.run(sched=sched)
    torch.cuda.synchronize()
    D_ref, e_ref, st_ref = r.D.clone(), r.energy_host(), r.stats_host()
    g = r.capture(sched=sched)
    for rep in range(3):
        r.D.zero_()
        r.out2.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.D, D_ref), rep
        assert r.energy_host() == e_ref, rep
        assert np.array_equal(r.stats_host(), st_ref), rep
    r.D.zero_()
    r.run(sched=sched)
    torch.cuda.synchronize()
    assert torch.equal(r.D, D_ref)


def test_overlapped_setup_matches_serial(gpu_ok):
    """Gather and set-up of batch i + 1 on a second stream while batch i iterates
    (two shared workspaces, persist set-up buffers): the same result as the serial
    order, bit for bit, with the learned schedule, also when repeated."""
    import os
    from paper_2205_12182_amd import learn
    from paper_2205_12182_amd.runner import learned_schedule
    w = os.path.join(os.path.dirname(learn.__file__), "data", "schedule_mlp.npz")
    model = learn.ScheduleMLP.load(w) if os.path.exists(w) else None
    sched = learned_schedule() if model is not None else default_mixed_schedule()
    inst = get_config("t_slab")
    a = Runner(inst, batch=40)
    a.run(sched=sched, predictor=model)
    b = Runner(inst, batch=40, persist=True, overlap=True)
    assert b.overlap and len(b.plans) >= 4 and len(b.workspaces) == 2
    for rep in range(2):
        b.D.zero_()
        b.run(sched=sched, predictor=model)
        torch.cuda.synchronize()
        assert torch.equal(a.D, b.D) and torch.equal(a.out2, b.out2), rep
        assert np.array_equal(a.stats_host(), b.stats_host()), rep
    assert b.check() == L.OK
