"""Why the sign iteration keeps its early steps out of FP8 (a CPU experiment).

The target asks for FP8 (OCP e4m3) with per-matrix scaling for the early sign
iterations.  This test emulates that arithmetic in NumPy on submatrices of a
benchmark-like water box and measures the density error against the FP64
oracle: the products take e4m3 operands (3 mantissa bits, exponent bias 7,
largest finite 448, round to nearest even, each matrix scaled so that its largest
entry maps to a power of two at or below 448) with exact accumulation, the later
steps FP16 operands, and the result gets the FP32 panel step of the GPU path.

It pins the decision recorded in the design notes: one e4m3 step already moves
the density by more than the 1e-3 target, while FP16 throughout stays well inside
it.  The reason is structural: Newton-Schulz converges to the sign of its current
iterate, so rounding of the early iterates (whose eigenvalues near the gap are
small) stays in the result, amplified by 1/|x|.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import nolsm_oracle as O
from workloads import get_config


def round_e4m3(x):
    """Round to the nearest OCP e4m3 value (ties to even), saturating at 448."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)                      # subnormals share the step 2^-9
    step = 2.0 ** (e - 3)
    q = np.round(a / step) * step
    q = np.minimum(q, 448.0)
    return np.sign(x) * q


def round_fp16(x):
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def q8(X):
    m = np.abs(X).max()
    s = 2.0 ** np.floor(np.log2(448.0 / m))
    return round_e4m3(X * s) / s


def q8_mx(X, axis):
    """e4m3 with one power-of-two scale per block of 32 consecutive entries along the
    contraction axis (the block scaling of the MX formats)."""
    Xt = np.moveaxis(np.asarray(X, np.float64), axis, -1)
    n = Xt.shape[-1]
    out = np.empty_like(Xt)
    for b in range(0, n, 32):
        blk = Xt[..., b:b + 32]
        m = np.abs(blk).max(axis=-1, keepdims=True)
        s = 2.0 ** np.floor(np.log2(448.0 / np.where(m > 0, m, 1.0)))
        out[..., b:b + 32] = round_e4m3(blk * s) / s
    return np.moveaxis(out, -1, axis)


def emulated_density(Hk, Sk, cols, n_fp8, mu=0.0, tol=0.1, mx=False):
    """Symmetric form: M = L^-1 H L^-T (FP64), X0 = (M - mu) / b; n_fp8 steps with
    e4m3 operands (one scale per matrix, or per 32-entry block along the
    contraction with mx), then FP16 operands to ||X^2 - I||_F <= tol plus one step,
    then one FP64 Newton-Schulz step on the own-column panel; D[:, cols]."""
    L = np.linalg.cholesky(Sk)
    Li = scipy.linalg.solve_triangular(L, np.eye(L.shape[0]), lower=True)
    M = Li @ Hk @ Li.T - mu * np.eye(L.shape[0])
    X = M / np.abs(M).sum(axis=1).max()
    eye = np.eye(X.shape[0])
    extra = None
    for it in range(80):
        if it < n_fp8 and mx:
            Y = q8_mx(X, 1) @ q8_mx(X, 0)
            Z = 1.5 * eye - 0.5 * Y
            X = round_fp16(q8_mx(X, 1) @ q8_mx(Z, 0))
            continue
        q = q8 if it < n_fp8 else round_fp16
        Xq = q(X)
        Y = Xq @ Xq
        if it >= n_fp8:
            r = np.linalg.norm(Y - eye)
            if extra == 0:
                break
            if extra is None and r <= tol:
                extra = 1
            elif extra is not None:
                extra -= 1
        X = q(Xq @ q(1.5 * eye - 0.5 * Y))
    V = Li[:, cols]
    W = 0.5 * X @ (3.0 * V - X @ (X @ V))
    return 0.5 * Li.T @ (V - W)


@pytest.mark.slow
def test_fp8_early_step_misses_the_density_target():
    inst = get_config("t_23")
    errs = {"fp16": [], "e4m3": [], "e4m3_mx": []}
    for k in (3, 77):
        Hk, offs = O.gather(inst, inst.H_val, k)
        Sk, _ = O.gather(inst, inst.S_val, k)
        cols = O.own_columns(inst, k, offs)
        ref, _ = O.density(Hk, Sk, inst.mu)
        for key, n8, mx in (("fp16", 0, False), ("e4m3", 1, False), ("e4m3_mx", 1, True)):
            D = emulated_density(Hk, Sk, cols, n8, mx=mx)
            errs[key].append(float(np.abs(D - ref[:, cols]).max()))
    print(f"[case] t_23 max |dD|: {errs}")
    assert max(errs["fp16"]) < 1e-3              # FP16 meets the target
    for key in ("e4m3", "e4m3_mx"):              # one e4m3 step, either scaling, does not
        assert min(errs[key]) > 1e-3
        assert min(errs[key]) > 5 * max(errs["fp16"])


def test_e4m3_rounding():
    """Spot values of the e4m3 grid: 1 + 2^-3 steps near 1, 2^-9 subnormal steps,
    ties to even, saturation."""
    assert round_e4m3(1.0625) == 1.0                       # tie between 1 and 1.125 -> even
    assert round_e4m3(1.1) == 1.125
    assert round_e4m3(0.3) == 0.3125                       # step 2^-5 in [0.25, 0.5)
    assert round_e4m3(2.0 ** -9 * 1.4) == 2.0 ** -9        # subnormal step
    assert round_e4m3(500.0) == 448.0 and round_e4m3(-500.0) == -448.0
    assert round_e4m3(240.0) == 240.0 and round_e4m3(250.0) == 256.0
