"""A whole step captured as a HIP graph and replayed (needs an MI355X).

Three batches share one workspace inside the capture.  Each replay, with eager
work on the same buffers between replays, must reproduce the eager results bit
for bit (the path is deterministic), and the eager path must still work after.
"""
import numpy as np
import pytest
import torch

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
