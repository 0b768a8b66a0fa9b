"""nolsm_energy_noalloc (the entry point for callers that cannot allocate) against
nolsm_energy: the same result bit for bit, on two calls in a row with the second
on a smaller instance, and within FP64 summation error of the oracle's traces."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import _lib as L
from workloads import get_config

pytestmark = pytest.mark.gpu


def _inputs(name, seed):
    inst = get_config(name)
    dpat = L.DevicePattern(inst, "cuda")
    H = torch.from_numpy(inst.H_val).cuda()
    S = torch.from_numpy(inst.S_val).cuda()
    D = torch.from_numpy(np.random.default_rng(seed).standard_normal(inst.nval)).cuda()
    return inst, dpat, H, S, D


def test_noalloc_energy_matches_energy(gpu_ok):
    for name, seed in (("t_tiles", 1), ("c1", 2)):          # second call: fewer molecules
        print(f"no-alloc energy: {name}", flush=True)
        inst, dpat, H, S, D = _inputs(name, seed)
        out_ref = torch.zeros(2, dtype=torch.float64, device="cuda")
        col = torch.zeros(2 * inst.nmol, dtype=torch.float64, device="cuda")
        L.nolsm_energy(dpat, D, H, S, col, out_ref)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        L.nolsm_energy_noalloc(dpat, D, H, S, out)
        torch.cuda.synchronize()
        assert torch.equal(out, out_ref), (out, out_ref)
        Dh = D.cpu().numpy()
        want = O.traces(inst, Dh, inst.H_val, inst.S_val)
        got = out.cpu().numpy()
        assert abs(got[0] - want[0]) <= 1e-12 * np.abs(Dh * inst.H_val).sum()
        assert abs(got[1] - want[1]) <= 1e-12 * np.abs(Dh * inst.S_val).sum()


def test_noalloc_energy_rejects_too_many_molecules(gpu_ok):
    inst, dpat, H, S, D = _inputs("c1", 0)
    big = L.Pattern.from_buffer_copy(dpat.struct)
    big.nmol = L.ENERGY_NOALLOC_MAXMOL + 1
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    code = L.lib().nolsm_energy_noalloc(ctypes.byref(big), big.nmol, D.data_ptr(), H.data_ptr(),
                                        S.data_ptr(), out.data_ptr(), L._stream())
    assert code == L.EINVAL
    assert "exceeds the limit" in L.nolsm_last_error()
