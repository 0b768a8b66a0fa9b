"""ctypes binding of libnolsm.so (argument marshalling only).

Every entry point of include/nolsm.h has a function of the same name here.  Device
memory and streams come from PyTorch (tensors' data_ptr() and the current HIP
stream); all arithmetic happens in the library's kernels.  If the shared library
is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnolsm.so")

# status codes (nolsm_status)
OK, EINVAL, ENOTSPD, ENOCONV, EHIP, EWORKSPACE, ENOMEM = range(7)
PREC_FP32, PREC_FP16, PREC_BF16 = 0, 1, 2
PREC_NAMES = {"fp32": PREC_FP32, "fp16": PREC_FP16, "bf16": PREC_BF16}


class NolsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nolsm error {code}: {msg}")
        self.code = code


class Pattern(ctypes.Structure):
    _fields_ = [("nmol", ctypes.c_int32), ("nnzb", ctypes.c_int64), ("nval", ctypes.c_int64),
                ("blk_dim", ctypes.c_void_p), ("blk_off", ctypes.c_void_p),
                ("colptr", ctypes.c_void_p), ("rowblk", ctypes.c_void_p),
                ("valoff", ctypes.c_void_p)]


class Phase(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("iters", ctypes.c_int32), ("tol", ctypes.c_float),
                ("extra", ctypes.c_int32), ("order", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("nphase", ctypes.c_int32), ("phase", Phase * 4),
                ("fallback_tol", ctypes.c_float), ("fallback_iters", ctypes.c_int32),
                ("panel_steps", ctypes.c_int32), ("scale", ctypes.c_void_p),
                ("lower", ctypes.c_void_p), ("lower_log10", ctypes.c_void_p),
                ("lower_factor", ctypes.c_float)]


class SubInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("npad", ctypes.c_int32), ("mol", ctypes.c_int32),
                ("m", ctypes.c_int32), ("own_lo", ctypes.c_int32), ("nmem", ctypes.c_int32),
                ("ngrp", ctypes.c_int32), ("own_mem", ctypes.c_int32), ("off_h", ctypes.c_int64),
                ("off_s", ctypes.c_int64), ("off_lo", ctypes.c_int64),
                ("off_dcol", ctypes.c_int64)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("big_tile_min_npad", ctypes.c_int32), ("setup_products", ctypes.c_int32),
                ("persist", ctypes.c_int32), ("factor_tiles", ctypes.c_int32),
                ("form", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


SETUP_SPLIT_FP16, SETUP_FP32 = 0, 1
FACTOR_FP32_TILES, FACTOR_FP64 = 0, 1
FORM_SYM, FORM_LITERAL = 0, 1


class Timings(ctypes.Structure):
    _fields_ = [("ms_gather", ctypes.c_double), ("ms_setup", ctypes.c_double),
                ("ms_sign", ctypes.c_double), ("ms_gemm", ctypes.c_double),
                ("ms_panel", ctypes.c_double), ("ms_scatter", ctypes.c_double),
                ("n_gemm", ctypes.c_int64), ("gemm_flop", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CombineOptions(ctypes.Structure):
    _fields_ = [("criterion", ctypes.c_int32), ("max_n", ctypes.c_int32),
                ("npoints", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("rate_n", ctypes.c_void_p), ("rate", ctypes.c_void_p)]


class MuSearch(ctypes.Structure):
    _fields_ = [("n_target", ctypes.c_double), ("tol", ctypes.c_double),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("mu", ctypes.c_double),
                ("last_n", ctypes.c_double), ("iters", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("done", ctypes.c_int32), ("pad", ctypes.c_int32)]


# nolsm_stats as a numpy record (56 bytes)
STATS_DTYPE = np.dtype([("n", "<i4"), ("status", "<i4"), ("iters_lo", "<i4"),
                        ("iters_fb", "<i4"), ("resid", "<f4"), ("fell_back", "<i4"),
                        ("scale", "<f8"), ("tr_dh", "<f8"), ("tr_ds", "<f8"),
                        ("tr_x", "<f4"), ("n_neg", "<i4")])
assert STATS_DTYPE.itemsize == 56

_lib = None


def lib():
    """Load libnolsm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2205_12182_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_size_t)
    P = ctypes.POINTER
    sigs = {
        "nolsm_plan_create": (i32, [P(Pattern), vp, i32, P(vp)]),
        "nolsm_plan_create_ex": (i32, [P(Pattern), vp, i32, P(PlanOptions), P(vp)]),
        "nolsm_plan_create_groups": (i32, [P(Pattern), vp, vp, i32, P(PlanOptions), P(vp)]),
        "nolsm_combine": (i32, [P(Pattern), vp, i32, P(CombineOptions), vp, vp, P(i32)]),
        "nolsm_plan_destroy": (None, [vp]),
        "nolsm_plan_workspace_bytes": (sz, [vp]),
        "nolsm_plan_table_bytes": (sz, [vp]),
        "nolsm_plan_bind": (i32, [vp, vp, sz, vp, sz, vp]),
        "nolsm_plan_bind_persist": (i32, [vp, vp, sz, vp, sz, vp, sz, vp]),
        "nolsm_plan_persist_bytes": (sz, [vp]),
        "nolsm_mu_search_init": (i32, [P(MuSearch), dbl, dbl, dbl, dbl, i32]),
        "nolsm_mu_search_update": (i32, [P(MuSearch), dbl]),
        "nolsm_plan_query": (i32, [vp, i32, P(SubInfo)]),
        "nolsm_build_submatrices": (i32, [vp, P(Pattern), vp, vp, vp]),
        "nolsm_sign_batched": (i32, [vp, dbl, P(Schedule), vp, vp]),
        "nolsm_scatter_density": (i32, [vp, P(Pattern), vp, vp, vp, vp, vp]),
        "nolsm_energy": (i32, [P(Pattern), i32, vp, vp, vp, vp, vp, vp]),
        "nolsm_energy_noalloc": (i32, [P(Pattern), i32, vp, vp, vp, vp, vp]),
        "nolsm_check": (i32, [vp, vp]),
        "nolsm_plan_set_timing": (i32, [vp, i32]),
        "nolsm_setup_batched": (i32, [vp, vp]),
        "nolsm_features": (i32, [vp, dbl, vp, vp]),
        "nolsm_mlp_param_count": (i64, [i32]),
        "nolsm_mlp_scratch_floats": (i64, [i64, i32]),
        "nolsm_mlp_forward": (i32, [vp, i32, vp, i64, vp, vp, vp]),
        "nolsm_mlp_backward": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp]),
        "nolsm_mlp_mse": (i32, [vp, vp, i64, i32, vp, vp, vp, vp]),
        "nolsm_mlp_adam": (i32, [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, i32, vp]),
        "nolsm_plan_get_timings": (i32, [vp, P(Timings), i32]),
        "nolsm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ("nolsm_plan_create", "nolsm_plan_create_ex", "nolsm_plan_create_groups",
            "nolsm_combine", "nolsm_plan_destroy", "nolsm_plan_workspace_bytes",
            "nolsm_plan_table_bytes", "nolsm_plan_bind", "nolsm_plan_bind_persist",
            "nolsm_plan_persist_bytes", "nolsm_mu_search_init", "nolsm_mu_search_update",
            "nolsm_plan_query", "nolsm_build_submatrices",
            "nolsm_sign_batched", "nolsm_scatter_density", "nolsm_energy", "nolsm_energy_noalloc", "nolsm_check",
            "nolsm_last_error", "nolsm_plan_set_timing", "nolsm_plan_get_timings",
            "nolsm_setup_batched", "nolsm_features", "nolsm_mlp_param_count",
            "nolsm_mlp_scratch_floats", "nolsm_mlp_forward", "nolsm_mlp_backward",
            "nolsm_mlp_mse", "nolsm_mlp_adam")
NFEAT = 16
MLP_HIDDEN = 64


def _ok(code):
    if code != OK:
        raise NolsmError(code, lib().nolsm_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------- patterns

class HostPattern:
    """nolsm_pattern over host (numpy) copies of an instance's pattern arrays."""

    def __init__(self, inst):
        self.arrays = [np.ascontiguousarray(inst.blk_dim, dtype=np.int32),
                       np.ascontiguousarray(inst.blk_off, dtype=np.int64),
                       np.ascontiguousarray(inst.colptr, dtype=np.int64),
                       np.ascontiguousarray(inst.rowblk, dtype=np.int32),
                       np.ascontiguousarray(inst.valoff, dtype=np.int64)]
        a = self.arrays
        self.struct = Pattern(inst.nmol, inst.nnzb, inst.nval, *[x.ctypes.data for x in a])


class DevicePattern:
    """nolsm_pattern over device (torch) copies of an instance's pattern arrays."""

    def __init__(self, inst, device="cuda"):
        import torch
        self.tensors = [torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(device)
                        for x, dt in ((inst.blk_dim, np.int32), (inst.blk_off, np.int64),
                                      (inst.colptr, np.int64), (inst.rowblk, np.int32),
                                      (inst.valoff, np.int64))]
        self.nmol = inst.nmol
        self.struct = Pattern(inst.nmol, inst.nnzb, inst.nval,
                              *[t.data_ptr() for t in self.tensors])


def schedule(phases, fallback_tol=0.05, fallback_iters=0, panel_steps=1, scale=None,
             lower=None, lower_log10=None, lower_factor=1.0):
    """nolsm_schedule from [(prec, iters, tol, extra[, order]), ...].

    order 2 (the default) is the Newton-Schulz step, order 3 the third-order
    polynomial step.  scale, lower: device FP64 tensors [K]; lower_log10: device
    FP32 tensor [K].
    """
    s = Schedule()
    s.nphase = len(phases)
    for i, ph in enumerate(phases):
        prec, iters, tol, extra = ph[:4]
        order = ph[4] if len(ph) > 4 else 2
        p = PREC_NAMES[prec] if isinstance(prec, str) else prec
        s.phase[i] = Phase(p, iters, tol, extra, order)
    s.fallback_tol = fallback_tol
    s.fallback_iters = fallback_iters
    s.panel_steps = panel_steps
    s.scale = None if scale is None else scale.data_ptr()
    s.lower = None if lower is None else lower.data_ptr()
    s.lower_log10 = None if lower_log10 is None else lower_log10.data_ptr()
    s.lower_factor = lower_factor
    s._keep = (scale, lower, lower_log10)
    return s


# ----------------------------------------------------------------------------- entry points

def nolsm_plan_create(host_pattern: HostPattern, mols, big_tile_min_npad=None,
                      setup_products=None, persist=False, factor_tiles=None,
                      form=None) -> ctypes.c_void_p:
    """Plan for `mols`; big_tile_min_npad (optional) sets the tile policy,
    setup_products (optional) how M_k is formed (SETUP_SPLIT_FP16 or SETUP_FP32),
    persist keeps the set-up results in a buffer of the plan's own, and factor_tiles
    (optional) the precision of the factorisation's tile products (FACTOR_FP32_TILES
    or FACTOR_FP64), form (optional) FORM_SYM or FORM_LITERAL."""
    mols = np.ascontiguousarray(mols, dtype=np.int32)
    out = ctypes.c_void_p()
    if (big_tile_min_npad is None and setup_products is None and not persist
            and factor_tiles is None and form is None):
        _ok(lib().nolsm_plan_create(ctypes.byref(host_pattern.struct), mols.ctypes.data,
                                    int(mols.size), ctypes.byref(out)))
    else:
        opt = _options(big_tile_min_npad, setup_products, persist, factor_tiles, form)
        _ok(lib().nolsm_plan_create_ex(ctypes.byref(host_pattern.struct), mols.ctypes.data,
                                       int(mols.size), ctypes.byref(opt), ctypes.byref(out)))
    return out


def _options(big_tile_min_npad, setup_products, persist, factor_tiles=None, form=None):
    opt = PlanOptions()
    opt.big_tile_min_npad = -1 if big_tile_min_npad is None else int(big_tile_min_npad)
    opt.setup_products = SETUP_SPLIT_FP16 if setup_products is None else int(setup_products)
    opt.persist = 1 if persist else 0
    opt.factor_tiles = FACTOR_FP32_TILES if factor_tiles is None else int(factor_tiles)
    opt.form = FORM_SYM if form is None else int(form)
    return opt


def nolsm_plan_create_groups(host_pattern: HostPattern, groups, big_tile_min_npad=None,
                             setup_products=None, persist=False,
                             factor_tiles=None, form=None) -> ctypes.c_void_p:
    """Plan one submatrix per group of molecules (lists of molecule indices)."""
    ptr = np.zeros(len(groups) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(g) for g in groups])
    flat = np.ascontiguousarray(np.concatenate([np.asarray(g, np.int32) for g in groups])
                                if groups else np.zeros(0, np.int32), dtype=np.int32)
    out = ctypes.c_void_p()
    opt = _options(big_tile_min_npad, setup_products, persist, factor_tiles, form)
    _ok(lib().nolsm_plan_create_groups(ctypes.byref(host_pattern.struct), ptr.ctypes.data,
                                       flat.ctypes.data, int(len(groups)), ctypes.byref(opt),
                                       ctypes.byref(out)))
    return out


def nolsm_combine(host_pattern: HostPattern, mols, criterion=9, table=None, max_n=0):
    """Groups of molecules from the combination heuristic (Eq. 9, or Eq. 10 with the
    rate table [(n, rate), ...]); a list of ascending molecule lists."""
    mols = np.ascontiguousarray(mols, dtype=np.int32)
    K = int(mols.size)
    ptr = np.zeros(K + 1, dtype=np.int32)
    flat = np.zeros(max(K, 1), dtype=np.int32)
    ng = ctypes.c_int32()
    opt = CombineOptions()
    opt.criterion = int(criterion)
    opt.max_n = int(max_n or 0)
    keep = None
    if table is not None:
        tn = np.ascontiguousarray([float(a) for a, _ in table], dtype=np.float64)
        tr = np.ascontiguousarray([float(b) for _, b in table], dtype=np.float64)
        keep = (tn, tr)
        opt.npoints = int(tn.size)
        opt.rate_n = tn.ctypes.data
        opt.rate = tr.ctypes.data
    _ok(lib().nolsm_combine(ctypes.byref(host_pattern.struct), mols.ctypes.data, K,
                            ctypes.byref(opt), ptr.ctypes.data, flat.ctypes.data,
                            ctypes.byref(ng)))
    del keep
    return [flat[ptr[g]:ptr[g + 1]].tolist() for g in range(ng.value)]


def nolsm_plan_destroy(plan):
    lib().nolsm_plan_destroy(plan)


def nolsm_plan_workspace_bytes(plan) -> int:
    return int(lib().nolsm_plan_workspace_bytes(plan))


def nolsm_plan_table_bytes(plan) -> int:
    return int(lib().nolsm_plan_table_bytes(plan))


def nolsm_plan_bind(plan, tables, workspace, stream=None):
    _ok(lib().nolsm_plan_bind(plan, _ptr(tables), tables.numel() * tables.element_size(),
                              _ptr(workspace), workspace.numel() * workspace.element_size(),
                              _stream(stream)))


def nolsm_plan_persist_bytes(plan) -> int:
    return int(lib().nolsm_plan_persist_bytes(plan))


def nolsm_plan_bind_persist(plan, tables, workspace, persist, stream=None):
    _ok(lib().nolsm_plan_bind_persist(plan, _ptr(tables), tables.numel() * tables.element_size(),
                                      _ptr(workspace),
                                      workspace.numel() * workspace.element_size(),
                                      _ptr(persist), persist.numel() * persist.element_size(),
                                      _stream(stream)))


def nolsm_mu_search_init(n_target, mu_lo, mu_hi, tol=0.5, max_iter=40) -> MuSearch:
    m = MuSearch()
    _ok(lib().nolsm_mu_search_init(ctypes.byref(m), float(n_target), float(mu_lo), float(mu_hi),
                                   float(tol), int(max_iter)))
    return m


def nolsm_mu_search_update(m: MuSearch, n_at_mu):
    _ok(lib().nolsm_mu_search_update(ctypes.byref(m), float(n_at_mu)))


def nolsm_plan_query(plan, i) -> SubInfo:
    info = SubInfo()
    _ok(lib().nolsm_plan_query(plan, int(i), ctypes.byref(info)))
    return info


def nolsm_build_submatrices(plan, dev_pattern: DevicePattern, H_val, S_val, stream=None):
    _ok(lib().nolsm_build_submatrices(plan, ctypes.byref(dev_pattern.struct), _ptr(H_val),
                                      _ptr(S_val), _stream(stream)))


def nolsm_sign_batched(plan, mu, sched=None, stats=None, stream=None):
    _ok(lib().nolsm_sign_batched(plan, float(mu), None if sched is None else ctypes.byref(sched),
                                 _ptr(stats), _stream(stream)))


def nolsm_scatter_density(plan, dev_pattern: DevicePattern, D_val, H_val, S_val, stats=None,
                          stream=None):
    _ok(lib().nolsm_scatter_density(plan, ctypes.byref(dev_pattern.struct), _ptr(D_val),
                                    _ptr(H_val), _ptr(S_val), _ptr(stats), _stream(stream)))


def nolsm_energy(dev_pattern: DevicePattern, D_val, H_val, S_val, col_traces, out2, stream=None):
    _ok(lib().nolsm_energy(ctypes.byref(dev_pattern.struct), dev_pattern.nmol, _ptr(D_val),
                           _ptr(H_val), _ptr(S_val), _ptr(col_traces), _ptr(out2),
                           _stream(stream)))


def nolsm_energy_noalloc(dev_pattern: DevicePattern, D_val, H_val, S_val, out2, stream=None):
    _ok(lib().nolsm_energy_noalloc(ctypes.byref(dev_pattern.struct), dev_pattern.nmol, _ptr(D_val),
                                   _ptr(H_val), _ptr(S_val), _ptr(out2), _stream(stream)))


ENERGY_NOALLOC_MAXMOL = 131072


def nolsm_check(plan, stream=None) -> int:
    code = lib().nolsm_check(plan, _stream(stream))
    return int(code)


def nolsm_setup_batched(plan, stream=None):
    _ok(lib().nolsm_setup_batched(plan, _stream(stream)))


def nolsm_features(plan, mu, feat, stream=None):
    _ok(lib().nolsm_features(plan, float(mu), _ptr(feat), _stream(stream)))


def nolsm_mlp_param_count(nout) -> int:
    return int(lib().nolsm_mlp_param_count(int(nout)))


def nolsm_mlp_scratch_floats(B, nout) -> int:
    return int(lib().nolsm_mlp_scratch_floats(int(B), int(nout)))


def nolsm_mlp_forward(params, nout, x, y, act=None, stream=None):
    _ok(lib().nolsm_mlp_forward(_ptr(params), int(nout), _ptr(x), int(x.shape[0]), _ptr(y),
                                _ptr(act), _stream(stream)))


def nolsm_mlp_backward(params, nout, x, act, dy, grad, scratch, stream=None):
    _ok(lib().nolsm_mlp_backward(_ptr(params), int(nout), _ptr(x), _ptr(act), _ptr(dy),
                                 int(x.shape[0]), _ptr(grad), _ptr(scratch), _stream(stream)))


def nolsm_mlp_mse(y, t, dy, loss, scratch, stream=None):
    _ok(lib().nolsm_mlp_mse(_ptr(y), _ptr(t), int(y.shape[0]), int(y.shape[1]), _ptr(dy),
                            _ptr(loss), _ptr(scratch), _stream(stream)))


def nolsm_mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, step, stream=None):
    _ok(lib().nolsm_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(params.numel()),
                             float(lr), float(beta1), float(beta2), float(eps), int(step),
                             _stream(stream)))


def nolsm_plan_set_timing(plan, enable=True):
    _ok(lib().nolsm_plan_set_timing(plan, 1 if enable else 0))


def nolsm_plan_get_timings(plan, reset=True) -> Timings:
    t = Timings()
    _ok(lib().nolsm_plan_get_timings(plan, ctypes.byref(t), 1 if reset else 0))
    return t


def nolsm_last_error() -> str:
    return lib().nolsm_last_error().decode()
