"""Parity of the HIP path with the FP64 oracle (needs an MI355X).

Tolerances follow the accuracy target of the method: every stored density element
within 1e-3 of the oracle, and |E - E_oracle| / N_atoms within 1e-5 Ha.  The
plain FP32 form is held to tighter bounds that follow from FP32 arithmetic.
Intermediate buffers (gathered submatrices, L^-1, M) are read back from the
workspace and checked against exact index arithmetic or FP64 identities.
"""
import math

import numpy as np
import pytest
import torch

from oracle import nolsm_oracle as O
from paper_2205_12182_amd import _lib as L
from paper_2205_12182_amd.runner import Runner, default_mixed_schedule, plain_fp32_schedule
from workloads import get_config

pytestmark = pytest.mark.gpu

D_TOL = 1e-3          # max |D - D_oracle| over stored elements
E_TOL = 1e-5          # |E - E_oracle| / N_atoms (Ha)

_cache = {}


def oracle(name):
    if name not in _cache:
        inst = get_config(name)
        D, st = O.density_matrix(inst)
        e, ne = O.traces(inst, D, inst.H_val, inst.S_val)
        _cache[name] = (inst, D, e, ne, st)
    return _cache[name]


def col_major(t, npad):
    return t.reshape(npad, npad).T.cpu().numpy()


def errors(inst, r, D_ref, e_ref):
    D = r.D.cpu().numpy()
    e, ne = r.energy_host()
    return float(np.abs(D - D_ref).max()), abs(e - e_ref) / inst.natoms, e, ne


def print_case(*a):
    print("[case]", *a, flush=True)


def split_rows(r, info):
    """The split FP16 rows of H (hi parts, lo parts) the gather writes for the split
    set-up products: iteration buffer 1, the hi part then the lo part, each k-blocked
    (element k of row j at ((k // 32) npad + j) 32 + k % 32)."""
    npad = info.npad
    v = r.ws_view(info.off_lo + 4 * npad * npad, 2 * npad * npad, torch.float16).cpu().numpy()

    def rows(x):
        return x.reshape(npad // 32, npad, 32).transpose(1, 0, 2).reshape(npad, npad)
    return rows(v[:npad * npad]), rows(v[npad * npad:])


@pytest.mark.parametrize("setup", [L.SETUP_SPLIT_FP16, L.SETUP_FP32])
def test_gather_bit_exact(gpu_ok, setup):
    """S_k in FP64 (its lower triangle, the part the factorisation reads) and H_k in
    FP64 (FP32 set-up option) equal the oracle's gather bit for bit; with split set-up products, H_k arrives as hi = fp16(H), lo = fp16(2^11
    (H - hi)), each rounded once from FP64, also bit for bit."""
    inst = get_config("t_slab")
    print_case("gather t_slab", setup)
    r = Runner(inst, setup_products=setup)
    L.nolsm_build_submatrices(r.plans[0], r.dpat, r.H, r.S)
    torch.cuda.synchronize()
    for i in [0, 1, inst.nmol // 2, inst.nmol - 1]:
        info = r.sub_info(0, i)
        npad, n = info.npad, info.n
        Sk = col_major(r.ws_view(info.off_s, npad * npad, torch.float64), npad)
        Href, offs = O.gather(inst, inst.H_val, info.mol)
        Sref, _ = O.gather(inst, inst.S_val, info.mol)
        assert n == Href.shape[0]
        if setup == L.SETUP_FP32:
            Hk = col_major(r.ws_view(info.off_h, npad * npad, torch.float64), npad)
            assert np.array_equal(Hk[:n, :n], Href)
            assert not Hk[n:, :].any() and not Hk[:, n:].any()
        else:
            hi, lo = split_rows(r, info)
            ref_hi = Href.astype(np.float16)
            ref_lo = ((Href - ref_hi.astype(np.float64)) * 2048.0).astype(np.float16)
            assert np.array_equal(hi[:n, :n].view(np.uint16), ref_hi.view(np.uint16))
            assert np.array_equal(lo[:n, :n].view(np.uint16), ref_lo.view(np.uint16))
            assert not hi[n:, :].any() and not hi[:, n:].any()
            assert not lo[n:, :].any() and not lo[:, n:].any()
        assert np.array_equal(np.tril(Sk[:n, :n]), np.tril(Sref))      # lower triangle only
        assert np.array_equal(Sk[n:, n:], np.eye(npad - n)) and not Sk[n:, :n].any()
        assert info.own_lo == int(O.own_columns(inst, info.mol, offs)[0])


@pytest.mark.parametrize("setup", [L.SETUP_SPLIT_FP16, L.SETUP_FP32])
@pytest.mark.parametrize("factor", [L.FACTOR_FP32_TILES, L.FACTOR_FP64])
def test_setup_identities(gpu_ok, setup, factor):
    """L^-1 S L^-T = I (to FP64 rounding with the FP64 factorisation; with its tile
    products on FP32 MFMAs every operand of those products is rounded to FP32 and
    the sums run in FP32, which leaves a few 1e-7 at these sizes: bounded at 1e-5,
    well inside the density target's 1e-3); M = L^-1 H L^-T exactly symmetric and within the
    rounding bound of its two products C = A B.  FP32 operands: each operand
    rounded to FP32 (u = 2^-24), FP32 accumulation over at most n terms, so
    |dC| <= (n + 2) u |A| |B| per product.  Split FP16 operands: an operand is
    represented within 2^-22 |x| + 2^-36 (the absolute term covers values in the
    FP16 subnormal range), each term keeps three of its four partial products, so
    |dC| <= (n + 14) u |A| |B| + 2^-36 (|A| J + J |B|) per product (J: all ones),
    and the first product's error is carried through L^-1 by the second."""
    inst = get_config("t_23")
    print_case("setup t_23", setup, factor)
    r = Runner(inst, setup_products=setup, factor_tiles=factor)
    r.run(sched=plain_fp32_schedule(), energy=False)
    torch.cuda.synchronize()
    for i in [0, inst.nmol // 3, inst.nmol - 1]:
        info = r.sub_info(0, i)
        npad, n = info.npad, info.n
        Li = col_major(r.ws_view(info.off_s, npad * npad, torch.float64), npad)[:n, :n]
        M = col_major(r.ws_view(info.off_h, npad * npad, torch.float32), npad).astype(np.float64)
        Hk, _ = O.gather(inst, inst.H_val, info.mol)
        Sk, _ = O.gather(inst, inst.S_val, info.mol)
        assert np.array_equal(Li, np.tril(Li))
        ident = np.abs(Li @ Sk @ Li.T - np.eye(n)).max()
        print_case(f"sub {i}: |L^-1 S L^-T - I| {ident:.2e}")
        assert ident < (1e-11 if factor == L.FACTOR_FP64 else 1e-5)
        assert np.array_equal(M, M.T)
        u, t = 2.0 ** -24, 2.0 ** -36
        aL, aH = np.abs(Li), np.abs(Hk)
        if setup == L.SETUP_FP32:
            bound = 2 * (n + 2) * u * (aL @ aH @ aL.T)
        else:
            J = np.ones((n, n))
            aU = aH @ aL.T
            e1 = (n + 14) * u * aU + t * (aH @ J + J @ aL.T)
            bound = (n + 14) * u * (aL @ aU) + t * (aL @ J + J @ aU) + aL @ e1
        err = np.abs(M[:n, :n] - Li @ Hk @ Li.T)
        pos = bound > 0
        assert not err[~pos].any()              # exact where every term is zero
        ratio = err[pos] / bound[pos]
        print_case(f"sub {i}: max error / bound {ratio.max():.3f}")
        assert ratio.max() <= 1.0
        assert not M[n:, :].any()


@pytest.mark.parametrize("name", ["c1", "t_tiles", "t_23"])
def test_parity_plain_fp32(gpu_ok, name):
    inst, D_ref, e_ref, ne_ref, _ = oracle(name)
    print_case("plain fp32", name)
    r = Runner(inst)
    r.run(sched=plain_fp32_schedule())
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
    print_case(name, "plain dD", dmax, "dE/atom", de)
    assert dmax < 1e-4 and de < 1e-6
    assert abs(ne - ne_ref) < 1e-3
    st = r.stats_host()
    assert np.all(st["status"] == 0) and np.all(st["iters_lo"] > 5)


@pytest.mark.parametrize("name", ["c1", "t_tiles", "t_23", "t_slab"])
def test_parity_mixed_fp16(gpu_ok, name):
    inst, D_ref, e_ref, ne_ref, _ = oracle(name)
    print_case("mixed fp16", name)
    r = Runner(inst)
    r.run(sched=default_mixed_schedule())
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
    st = r.stats_host()
    print_case(name, "mixed dD", dmax, "dE/atom", de, "fallbacks", int(st["fell_back"].sum()),
               "resid max", float(st["resid"].max()))
    assert dmax < D_TOL and de < E_TOL


@pytest.mark.parametrize("name", ["c1", "t_tiles"])
def test_parity_third_order(gpu_ok, name):
    """The third-order polynomial step, in plain FP32 and as the FP16 bulk, meets the
    same bounds as Newton-Schulz and converges in fewer steps (cubic rate)."""
    inst, D_ref, e_ref, ne_ref, _ = oracle(name)
    r = Runner(inst)
    print_case("plain fp32 order 2", name)
    r.run(sched=plain_fp32_schedule())
    assert r.check() == L.OK, L.nolsm_last_error()
    it2 = r.stats_host()["iters_lo"].copy()
    print_case("plain fp32 order 3", name)
    r.run(sched=plain_fp32_schedule(order=3))
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
    st = r.stats_host()
    it3 = st["iters_lo"]
    print_case(name, "order-3 plain dD", dmax, "dE/atom", de, "iters", int(it3.max()), "vs",
               int(it2.max()))
    assert dmax < 1e-4 and de < 1e-6
    assert abs(ne - ne_ref) < 1e-3
    assert np.all(st["status"] == 0) and np.all(it3 < it2)
    print_case("mixed fp16 order 3", name)
    r.run(sched=default_mixed_schedule(order=3))
    assert r.check() == L.OK, L.nolsm_last_error()
    dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
    st = r.stats_host()
    print_case(name, "order-3 mixed dD", dmax, "dE/atom", de, "fallbacks",
               int(st["fell_back"].sum()))
    assert dmax < D_TOL and de < E_TOL


@pytest.mark.parametrize("name", ["c1", "t_tiles"])
def test_parity_bf16_and_phase_change(gpu_ok, name):
    """The BF16 bulk, alone and as a first phase converted to an FP16 phase.

    BF16 keeps 8 significand bits against FP16's 11, so its unit roundoff is 8 times
    larger; rounding errors of the iterates stay in the sign (its derivative weighs
    them by at least 1), so the BF16 bound is 8 times the FP16 accuracy target.  The
    two-phase schedule runs the conversion of the iterate between precisions."""
    inst, D_ref, e_ref, ne_ref, _ = oracle(name)
    r = Runner(inst)
    for label, sched in (
            ("bf16 bulk", default_mixed_schedule(prec="bf16")),
            ("bf16 -> fp16", L.schedule([("bf16", 3, 0.0, 0), ("fp16", 30, 0.1, 1)],
                                        fallback_tol=0.1, fallback_iters=60, panel_steps=1))):
        print_case(label, name)
        r.run(sched=sched)
        assert r.check() == L.OK, L.nolsm_last_error()
        dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
        st = r.stats_host()
        print_case(name, label, "dD", dmax, "dE/atom", de, "iters", int(st["iters_lo"].max()),
                   "fallbacks", int(st["fell_back"].sum()))
        assert np.all(st["status"] == 0)
        assert dmax < 8 * D_TOL and de < 8 * E_TOL


def test_per_column_traces_match_oracle(gpu_ok):
    inst, D_ref, e_ref, ne_ref, _ = oracle("c1")
    r = Runner(inst)
    r.run(sched=plain_fp32_schedule())
    st = r.stats_host()
    for i, k in enumerate(r.mols):
        eh, es = O.column_traces(inst, D_ref, inst.H_val, inst.S_val, int(k))
        assert abs(st["tr_dh"][i] - eh) < 1e-5
        assert abs(st["tr_ds"][i] - es) < 1e-5
    e, ne = r.energy_host()
    assert abs(math.fsum(st["tr_dh"].tolist()) - e) < 1e-9


def test_energy_kernel_against_cpu_sum(gpu_ok):
    inst = get_config("t_tiles")
    r = Runner(inst)
    D = torch.from_numpy(np.random.default_rng(0).standard_normal(inst.nval)).cuda()
    L.nolsm_energy(r.dpat, D, r.H, r.S, r.col_traces, r.out2)
    torch.cuda.synchronize()
    got = r.out2.cpu().numpy()
    Dh = D.cpu().numpy()
    want = O.traces(inst, Dh, inst.H_val, inst.S_val)
    assert abs(got[0] - want[0]) <= 1e-12 * np.abs(Dh * inst.H_val).sum()
    assert abs(got[1] - want[1]) <= 1e-12 * np.abs(Dh * inst.S_val).sum()


def test_deterministic_and_batch_invariant(gpu_ok):
    inst = get_config("t_tiles")
    r1 = Runner(inst)
    r1.run(sched=default_mixed_schedule())
    D1 = r1.D.clone()
    E1 = r1.out2.clone()
    r1.run(sched=default_mixed_schedule())
    assert torch.equal(D1, r1.D) and torch.equal(E1, r1.out2)
    r2 = Runner(inst, batch=100)
    r2.run(sched=default_mixed_schedule())
    assert torch.equal(D1, r2.D) and torch.equal(E1, r2.out2)


def test_not_spd_is_reported(gpu_ok):
    inst = get_config("c1")
    S = inst.S_val.copy()
    # make S_00 negative: every submatrix containing molecule 0 is indefinite
    S[inst.valoff[inst.colptr[0]]] = -1.0
    inst.S_val = S
    r = Runner(inst)
    r.run(sched=plain_fp32_schedule())
    code = r.check()
    assert code == L.ENOTSPD
    st = r.stats_host()
    bad = st["status"] == L.ENOTSPD
    assert bad[0] and bad.sum() < inst.nmol


def test_fallback_recovers(gpu_ok):
    """Too few low-precision iterations: the residual check sends every
    submatrix to the FP32 continuation, which converges to the oracle."""
    inst, D_ref, e_ref, _, _ = oracle("c1")
    r = Runner(inst)
    r.run(sched=default_mixed_schedule(fixed_iters=3, fallback_iters=80))
    assert r.check() == L.OK, L.nolsm_last_error()
    st = r.stats_host()
    assert np.all(st["fell_back"] == 1) and np.all(st["iters_fb"] > 5)
    dmax, de, _, _ = errors(inst, r, D_ref, e_ref)
    assert dmax < 1e-4 and de < 1e-6


def test_nonconvergence_is_reported(gpu_ok):
    inst = get_config("c1")
    r = Runner(inst)
    r.run(sched=L.schedule([("fp32", 3, 1e-4, 2)], fallback_iters=0, panel_steps=0))
    assert r.check() == L.ENOCONV


def test_tile_shapes_agree(gpu_ok):
    """The 256 x 128 tiles (16 x 16 x 32 MFMAs) and the 128 x 128 tiles (32 x 32 x 16
    MFMAs) sum each element's products in different orders, so the FP16 iterates
    differ by rounding only: under either tile policy the whole path matches the
    oracle, and the two results agree with each other to the same tolerance."""
    inst, D_ref, e_ref, ne_ref, _ = oracle("t_23")
    print_case("tile policies t_23")
    out = []
    for big in (0, 1 << 20):
        r = Runner(inst, big_tile_min_npad=big)
        r.run(sched=default_mixed_schedule())
        assert r.check() == L.OK, L.nolsm_last_error()
        dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
        print_case("policy", big, "dD", dmax, "dE/atom", de)
        assert dmax < D_TOL and de < E_TOL
        out.append((r.D.clone(), e))
    assert float((out[0][0] - out[1][0]).abs().max()) < D_TOL
    assert abs(out[0][1] - out[1][1]) / inst.natoms < E_TOL


@pytest.mark.parametrize("nmol,r_cut,seed", [(27, 2.0, 3), (64, 3.6, 5)])
def test_single_tile_submatrices(gpu_ok, nmol, r_cut, seed):
    """Submatrices smaller than one 64-wide block (n = 6: each molecule alone; n = 30-42):
    every tile is a ragged edge tile, the factorisation and inverse are one diagonal
    block, and the FP32 and mixed schedules still match the oracle."""
    from workloads.water import water_box
    inst = water_box(nmol, (4, 1, 1), r_cut, seed=seed, name="tiny")
    dims = inst.submatrix_dims()
    print_case(f"tiny water box: {nmol} molecules, n {dims.min()}-{dims.max()}")
    D_ref, _ = O.density_matrix(inst)
    e_ref, _ = O.traces(inst, D_ref, inst.H_val, inst.S_val)
    for sched, dtol, etol in ((plain_fp32_schedule(), 1e-4, 1e-6),
                              (default_mixed_schedule(), D_TOL, E_TOL)):
        r = Runner(inst)
        r.run(sched=sched)
        assert r.check() == L.OK, L.nolsm_last_error()
        dmax, de, e, ne = errors(inst, r, D_ref, e_ref)
        print_case("dD", dmax, "dE/atom", de)
        assert dmax < dtol and de < etol


def test_empty_plan(gpu_ok):
    """A plan of no molecules binds and runs every entry point as a no-op."""
    inst = get_config("c1")
    hp = L.HostPattern(inst)
    dp = L.DevicePattern(inst, "cuda")
    plan = L.nolsm_plan_create(hp, np.zeros(0, dtype=np.int32))
    try:
        tab = torch.empty(max(L.nolsm_plan_table_bytes(plan), 256), dtype=torch.uint8,
                          device="cuda")
        ws = torch.empty(max(L.nolsm_plan_workspace_bytes(plan), 256), dtype=torch.uint8,
                         device="cuda")
        H = torch.from_numpy(inst.H_val).cuda()
        S = torch.from_numpy(inst.S_val).cuda()
        D = torch.full_like(H, 7.0)
        L.nolsm_plan_bind(plan, tab, ws)
        L.nolsm_build_submatrices(plan, dp, H, S)
        L.nolsm_sign_batched(plan, inst.mu, default_mixed_schedule())
        L.nolsm_scatter_density(plan, dp, D, H, S)
        torch.cuda.synchronize()
        assert L.nolsm_check(plan) == L.OK
        assert bool((D == 7.0).all())                  # nothing written
    finally:
        L.nolsm_plan_destroy(plan)


@pytest.mark.parametrize("which", ["H", "S"])
def test_nan_input_is_reported(gpu_ok, which):
    """A NaN planted in one stored element (a diagonal block of molecule 3): every
    submatrix that contains molecule 3 is reported (ENOCONV when the NaN is in H0:
    the residual test and the FP32 restart both fail; ENOTSPD when it is in S: the
    Cholesky pivot is not positive), in every batch (Runner.check folds them all),
    and every other submatrix gives exactly the result of the clean input."""
    inst = get_config("c1")
    clean = Runner(inst, batch=12)
    clean.run(sched=default_mixed_schedule())
    vals = (inst.H_val if which == "H" else inst.S_val).copy()
    t = int(inst.colptr[3]) + int(np.searchsorted(inst.members(3), 3))
    vals[int(inst.valoff[t]) + 1] = np.nan           # element (1, 0) of block (3, 3)
    bad_inst = get_config("c1")
    if which == "H":
        bad_inst.H_val = vals
    else:
        bad_inst.S_val = vals
    r = Runner(bad_inst, batch=12)                    # three batches
    r.run(sched=default_mixed_schedule())
    code = r.check()
    want = L.ENOCONV if which == "H" else L.ENOTSPD
    print_case(f"nan in {which}: check {code}, {r.last_check_message}")
    assert code == want
    st, st0 = r.stats_host(), clean.stats_host()
    hit = np.array([3 in inst.members(k) for k in range(inst.nmol)])
    assert np.array_equal(st["status"] == want, hit)
    assert (st["status"][~hit] == 0).all()
    # clean submatrices are unaffected: their written block columns match bit for bit
    D, D0 = r.D.cpu().numpy(), clean.D.cpu().numpy()
    for k in np.nonzero(~hit)[0]:
        lo, hi = int(inst.valoff[inst.colptr[k]]), int(inst.valoff[inst.colptr[k + 1] - 1])
        hi += int(inst.blk_dim[inst.rowblk[inst.colptr[k + 1] - 1]]) * int(inst.blk_dim[k])
        assert np.array_equal(D[lo:hi], D0[lo:hi]), k
    assert np.array_equal(st["tr_dh"][~hit], st0["tr_dh"][~hit])
