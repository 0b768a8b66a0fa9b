"""The C ABI without a GPU: the library loads, exports what include/nolsm.h
declares, and the host-side planning validates its arguments."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2205_12182_amd import _lib as L
from workloads import get_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nolsm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nolsm_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_struct_sizes_match_header():
    assert ctypes.sizeof(L.SubInfo) == 64
    assert ctypes.sizeof(L.Phase) == 20
    assert L.Schedule.phase.offset == 4 and L.Schedule.scale.offset == 96
    assert L.STATS_DTYPE.itemsize == 48
    assert ctypes.sizeof(L.Pattern) == 8 * 8


def test_plan_layout_c1():
    inst = get_config("c1")
    hp = L.HostPattern(inst)
    mols = np.arange(inst.nmol, dtype=np.int32)
    plan = L.nolsm_plan_create(hp, mols)
    try:
        nb = L.nolsm_plan_workspace_bytes(plan)
        dims = inst.submatrix_dims()
        # per submatrix: two FP64 n^2, three 4-byte n^2, plus small panels
        npad = (dims + 63) // 64 * 64
        assert nb >= int((8 * 2 + 12) * (npad.astype(np.int64) ** 2).sum())
        # the query API needs a bound plan only for device pointers; sizes are host-side
    finally:
        L.nolsm_plan_destroy(plan)


def test_bind_checks_buffers_before_any_device_work():
    """Null, short or misaligned buffers are refused before anything is enqueued
    (the fake addresses below are never dereferenced)."""
    inst = get_config("c1")
    hp = L.HostPattern(inst)
    plan = L.nolsm_plan_create(hp, np.arange(inst.nmol, dtype=np.int32))
    try:
        tb, wb = L.nolsm_plan_table_bytes(plan), L.nolsm_plan_workspace_bytes(plan)
        assert tb > 0 and wb > tb
        fake_t, fake_w = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
        bind = L.lib().nolsm_plan_bind
        assert bind(plan, None, tb, fake_w, wb, None) == L.EINVAL
        assert bind(plan, fake_t, tb - 1, fake_w, wb, None) == L.EWORKSPACE
        assert "table buffer" in L.nolsm_last_error()
        assert bind(plan, fake_t, tb, fake_w, wb - 1, None) == L.EWORKSPACE
        assert bind(plan, ctypes.c_void_p((1 << 20) + 64), tb, fake_w, wb, None) == L.EWORKSPACE
        assert "aligned" in L.nolsm_last_error()
    finally:
        L.nolsm_plan_destroy(plan)


def test_plan_options_tile_policy():
    """The tile policy changes the tile lists (so the table size); reserved fields must be zero."""
    inst = get_config("t_23")
    hp = L.HostPattern(inst)
    mols = np.arange(inst.nmol, dtype=np.int32)
    sizes = []
    for big in (None, 0, 1 << 20):
        plan = L.nolsm_plan_create(hp, mols, big)
        sizes.append(L.nolsm_plan_table_bytes(plan))
        L.nolsm_plan_destroy(plan)
    # t_23 submatrices have npad < 768: the default and the "never" policy agree,
    # "always large" produces different tile lists
    assert sizes[0] == sizes[2] and sizes[1] != sizes[0]
    opt = L.PlanOptions()
    opt.big_tile_min_npad = 0
    opt.reserved[3] = 1
    out = ctypes.c_void_p()
    rc = L.lib().nolsm_plan_create_ex(ctypes.byref(hp.struct), mols.ctypes.data, int(mols.size),
                                      ctypes.byref(opt), ctypes.byref(out))
    assert rc == L.EINVAL and "reserved" in L.nolsm_last_error()
    opt.reserved[3] = 0
    opt.setup_products = 2
    rc = L.lib().nolsm_plan_create_ex(ctypes.byref(hp.struct), mols.ctypes.data, int(mols.size),
                                      ctypes.byref(opt), ctypes.byref(out))
    assert rc == L.EINVAL and "setup_products" in L.nolsm_last_error()
    for sp in (L.SETUP_SPLIT_FP16, L.SETUP_FP32):
        plan = L.nolsm_plan_create(hp, mols, setup_products=sp)
        L.nolsm_plan_destroy(plan)


def test_plan_rejects_bad_molecule():
    inst = get_config("c1")
    hp = L.HostPattern(inst)
    with pytest.raises(L.NolsmError) as e:
        L.nolsm_plan_create(hp, np.array([0, 99], dtype=np.int32))
    assert e.value.code == L.EINVAL
    assert "out of range" in L.nolsm_last_error()


def test_plan_rejects_missing_diagonal():
    from tests.helpers import instance_from_dense
    inst = instance_from_dense(np.eye(2), np.eye(2), [1, 1], np.ones((2, 2)))
    # drop the diagonal block of column 0
    keep = np.ones(inst.nnzb, dtype=bool)
    keep[0] = False
    inst.rowblk = inst.rowblk[keep]
    inst.valoff = inst.valoff[keep]
    inst.colptr = np.array([0, 1, 3], dtype=np.int64)
    hp = L.HostPattern(inst)
    with pytest.raises(L.NolsmError) as e:
        L.nolsm_plan_create(hp, np.array([0], dtype=np.int32))
    assert e.value.code == L.EINVAL


def test_sign_rejects_unbound_plan():
    inst = get_config("c1")
    plan = L.nolsm_plan_create(L.HostPattern(inst), np.array([0], dtype=np.int32))
    try:
        code = L.lib().nolsm_sign_batched(plan, 0.0, None, None, None)
        assert code == L.EINVAL
        assert "not bound" in L.nolsm_last_error()
    finally:
        L.nolsm_plan_destroy(plan)


@pytest.mark.parametrize("case", ["order", "order3_scaled", "prec", "nphase"])
def test_sign_rejects_bad_schedule(case):
    """Schedules are checked before anything is enqueued (the plan is not bound and
    the lower-bound address is never dereferenced)."""
    inst = get_config("c1")
    plan = L.nolsm_plan_create(L.HostPattern(inst), np.array([0], dtype=np.int32))
    try:
        sch = L.schedule([("fp16", 10, 0.1, 1, 2)])
        if case == "order":
            sch.phase[0].order = 4
        elif case == "order3_scaled":
            sch.phase[0].order = 3
            sch.lower = 0x1000
        elif case == "prec":
            sch.phase[0].prec = 7
        else:
            sch.nphase = 5
        code = L.lib().nolsm_sign_batched(plan, 0.0, ctypes.byref(sch), None, None)
        assert code == L.EINVAL
        msg = L.nolsm_last_error()
        assert "not bound" not in msg, msg
        if case == "order3_scaled":
            assert "unscaled" in msg
        # a valid order-3 schedule passes the checks and stops at the unbound plan
        ok = L.schedule([("fp16", 10, 0.1, 1, 3)])
        assert L.lib().nolsm_sign_batched(plan, 0.0, ctypes.byref(ok), None, None) == L.EINVAL
        assert "not bound" in L.nolsm_last_error()
    finally:
        L.nolsm_plan_destroy(plan)
