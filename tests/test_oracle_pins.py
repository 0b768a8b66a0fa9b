"""Pins for the FP64 oracle: closed forms, invariants and brute force.

Each check below rests on something other than the oracle itself: a closed form
worked out by hand, a textbook identity of the matrix sign function, a different
library route (signm, LDL^T inertia, eigenvalues only), or plain dense index
arithmetic.  The planted-mistake tests at the end confirm that plausible slips in
the oracle (a flipped occupation, a transposed operand, a wrong index) make at
least one of these checks fail.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import nolsm_oracle as O
from tests.helpers import dense, instance_from_dense, permuted
from workloads import get_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers

def inertia_below(H, S, mu):
    """Number of generalized eigenvalues below mu from an LDL^T of H - mu S.

    Sylvester's law of inertia: H - mu S is congruent to the block-diagonal
    factor D of its LDL^T, whose negative eigenvalues count eigenvalues < mu.
    """
    _, d, _ = scipy.linalg.ldl(H - mu * S)
    return int(np.sum(np.linalg.eigvalsh(d) < 0))


def dense_density_by_columns(inst, D_val_unused=None):
    """Brute-force assembly of D from the oracle's per-molecule results using
    global index arithmetic on dense matrices (no block storage involved)."""
    H = dense(inst, inst.H_val)
    S = dense(inst, inst.S_val)
    n = inst.nfunc
    D = np.zeros((n, n))
    for k in range(inst.nmol):
        mem = inst.rowblk[inst.colptr[k]:inst.colptr[k + 1]]
        fidx = np.concatenate([np.arange(inst.blk_off[J], inst.blk_off[J + 1]) for J in mem])
        Hk = H[np.ix_(fidx, fidx)]
        Sk = S[np.ix_(fidx, fidx)]
        Dk, _ = O.density(Hk, Sk, inst.mu)
        own = np.nonzero((fidx >= inst.blk_off[k]) & (fidx < inst.blk_off[k + 1]))[0]
        D[np.ix_(fidx, fidx[own])] = Dk[:, own]
    return D, H, S


# ------------------------------------------------------------------ pin checks
# Each raises AssertionError on failure; the planted-mistake tests reuse them.

def check_scalar_closed_form():
    for h, s, mu in [(-0.7, 1.3, 0.0), (0.4, 0.8, 0.0), (0.4, 0.8, 1.0), (-2.0, 0.5, -3.0)]:
        inst = instance_from_dense(np.array([[h]]), np.array([[s]]), [1], [[True]], mu=mu)
        D, _ = O.density_matrix(inst)
        want = (1.0 / s) if h / s < mu else 0.0          # 1/2 (1 - sign(h/s - mu)) / s
        assert abs(D[0] - want) < 1e-14, (h, s, mu, D[0], want)


def check_diagonal_orthogonal():
    h = np.array([-1.5, 0.3, -0.2, 2.0, -0.01, 0.7])
    inst = instance_from_dense(np.diag(h), np.eye(6), [2, 2, 2], np.ones((3, 3)), mu=0.0)
    D, _ = O.density_matrix(inst)
    want = np.diag((h < 0).astype(float))
    assert np.allclose(dense(inst, D), want, atol=1e-14, rtol=0)


def check_golden_2x2():
    g = json.load(open(os.path.join(GOLDEN, "gen2x2.json")))
    H, S = np.array(g["H"]), np.array(g["S"])
    inst = instance_from_dense(H, S, [1, 1], np.ones((2, 2)), mu=g["mu"])
    D, _ = O.density_matrix(inst)
    Dd = dense(inst, D)
    assert np.allclose(Dd, np.array(g["D"]), atol=1e-14, rtol=0)
    e, ne = O.traces(inst, D, inst.H_val, inst.S_val)
    assert abs(e - g["tr_DH"]) < 1e-14 and abs(ne - g["tr_DS"]) < 1e-14


def check_general_2x2_closed_form(seed):
    rng = np.random.default_rng(seed)
    a, c, d = rng.uniform(-2, 2, 3)
    s = rng.uniform(-0.6, 0.6)
    H = np.array([[a, c], [c, d]])
    S = np.array([[1.0, s], [s, 1.0]])
    # det(H - l S) = (1 - s^2) l^2 - (a + d - 2 c s) l + (a d - c^2)
    A2, A1, A0 = 1 - s * s, -(a + d - 2 * c * s), a * d - c * c
    disc = math.sqrt(A1 * A1 - 4 * A2 * A0)
    lm, lp = (-A1 - disc) / (2 * A2), (-A1 + disc) / (2 * A2)
    mu = 0.5 * (lm + lp)
    v = np.array([c - lm * s, -(a - lm)])
    if np.linalg.norm(v) < 1e-8:
        v = np.array([d - lm, -(c - lm * s)])
    v = v / math.sqrt(v @ S @ v)
    want = np.outer(v, v)
    inst = instance_from_dense(H, S, [1, 1], np.ones((2, 2)), mu=mu)
    D, _ = O.density_matrix(inst)
    assert np.allclose(dense(inst, D), want, atol=1e-12, rtol=0)


def check_tiny_bruteforce(seed):
    """Eigen route == literal Eq. 8 via signm == Newton-Schulz (Eq. 6-7) route."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 9))
    B = rng.standard_normal((n, n))
    S = B @ B.T / n + 0.5 * np.eye(n)
    H = rng.standard_normal((n, n))
    H = 0.5 * (H + H.T)
    lam = scipy.linalg.eigvalsh(H, S)
    mu = 0.5 * (lam[n // 2 - 1] + lam[n // 2]) if n > 1 else lam[0] + 1
    D_eig, _ = O.density(H, S, mu)
    D_lit = O.density_literal(H, S, mu)
    Sinv = np.linalg.inv(S)
    X, it, hist = O.newton_schulz_sign(Sinv @ H - mu * np.eye(n), tol=1e-13, maxit=200)
    D_ns = 0.5 * (np.eye(n) - X) @ Sinv
    assert np.allclose(D_eig, D_lit, atol=1e-9, rtol=0)
    assert np.allclose(D_eig, D_ns, atol=1e-8, rtol=0)


def check_sign_invariants(seed, order=2):
    rng = np.random.default_rng(seed)
    n = 24
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    X, it, hist = O.newton_schulz_sign(A, order=order)
    eye = np.eye(n)
    assert np.abs(X @ X - eye).max() < 1e-10                         # sign(A)^2 = I
    assert np.abs(A @ X - X @ A).max() < 1e-9                        # commutes with A
    lam = np.linalg.eigvalsh(A)
    assert abs(np.trace(X) - (np.sum(lam > 0) - np.sum(lam < 0))) < 1e-9
    X3, _, _ = O.newton_schulz_sign(3.7 * A, order=order)
    assert np.abs(X3 - X).max() < 1e-9                               # sign(cA) = sign(A)
    assert hist[-1] <= 1e-12 and it < 100


def check_whole_system():
    """Each submatrix is the whole system: the assembled D is the exact D."""
    inst = get_config("c1_whole")
    D_val, _ = O.density_matrix(inst)
    D = dense(inst, D_val)
    H = dense(inst, inst.H_val)
    S = dense(inst, inst.S_val)
    assert np.abs(D @ S @ D - D).max() < 1e-12                       # idempotency
    n_occ = inertia_below(H, S, inst.mu)
    e, ne = O.traces(inst, D_val, inst.H_val, inst.S_val)
    assert n_occ == 96 and abs(ne - n_occ) < 1e-10                   # Tr(DS) = N_occ
    lam = scipy.linalg.eigh(H, S, eigvals_only=True)
    assert abs(e - math.fsum(lam[lam < inst.mu].tolist())) < 1e-10   # Tr(DH) = sum occupied
    D_lit = O.density_literal(H, S, inst.mu)
    assert np.abs(D - D_lit).max() < 1e-9                            # literal Eq. 5


def check_submatrices(name="c1"):
    inst = get_config(name)
    for k in range(0, inst.nmol, max(1, inst.nmol // 8)):
        Hk, offs = O.gather(inst, inst.H_val, k)
        Sk, _ = O.gather(inst, inst.S_val, k)
        Dk, lam = O.density(Hk, Sk, inst.mu)
        assert np.abs(Dk @ Sk @ Dk - Dk).max() < 1e-11
        assert abs(np.trace(Dk @ Sk) - inertia_below(Hk, Sk, inst.mu)) < 1e-9


def check_gather(name="t_small"):
    inst = get_config(name)
    H = dense(inst, inst.H_val)
    for k in [0, 1, inst.nmol // 2, inst.nmol - 1]:
        mem = inst.rowblk[inst.colptr[k]:inst.colptr[k + 1]]
        fidx = np.concatenate([np.arange(inst.blk_off[J], inst.blk_off[J + 1]) for J in mem])
        Hk, offs = O.gather(inst, inst.H_val, k)
        # blocks (I, J) with both in mem but not stored are zero in T_k
        want = H[np.ix_(fidx, fidx)]
        assert np.array_equal(Hk, want)
        cols = O.own_columns(inst, k, offs)
        assert np.array_equal(fidx[cols], np.arange(inst.blk_off[k], inst.blk_off[k + 1]))


def check_scatter_and_traces(name="c1"):
    inst = get_config(name)
    D_val, _ = O.density_matrix(inst)
    Dref, H, S = dense_density_by_columns(inst)
    assert np.array_equal(dense(inst, D_val), Dref)
    e, ne = O.traces(inst, D_val, inst.H_val, inst.S_val)
    assert abs(e - np.trace(Dref @ H)) < 1e-10
    assert abs(ne - np.trace(Dref @ S)) < 1e-10


def check_chain_truncation(t=0.45):
    """Three molecules with one function each, block (0, 2) absent.

    Columns 0 and 2 come from 2x2 submatrices, column 1 from the full 3x3; both
    have closed forms (see the comments).
    """
    H = np.array([[-1.0, t, 0.0], [t, 1.0, t], [0.0, t, -1.0]])
    present = np.array([[1, 1, 0], [1, 1, 1], [0, 1, 1]], dtype=bool)
    inst = instance_from_dense(H, np.eye(3), [1, 1, 1], present, mu=0.0)
    D_val, _ = O.density_matrix(inst)
    D = dense(inst, D_val)
    s = math.sqrt(1 + t * t)          # 2x2 [[-1, t], [t, 1]]: eigenvalues -+s
    r = math.sqrt(1 + 2 * t * t)      # 3x3: antisymmetric -1, symmetric block -+r
    want = np.array([[(1 + s) / (2 * s), -t / (2 * r), 0.0],
                     [-t / (2 * s), (r - 1) / (2 * r), -t / (2 * s)],
                     [0.0, -t / (2 * r), (1 + s) / (2 * s)]])
    assert np.allclose(D, want, atol=1e-14, rtol=0), (D, want)
    e, _ = O.traces(inst, D_val, inst.H_val, inst.S_val)
    assert abs(e - float(np.sum(want * H))) < 1e-14


def check_mu_in_gap():
    inst = get_config("c1")
    D0, st = O.density_matrix(inst)
    gap = min(s["gap"] for s in st)
    for dmu in (-0.5 * gap, 0.5 * gap):
        D1, _ = O.density_matrix(inst, mu=inst.mu + dmu)
        assert np.abs(D1 - D0).max() < 1e-10


def check_permutation(name="t_small"):
    inst = get_config(name)
    perm = np.random.default_rng(11).permutation(inst.nmol)
    pinst, fidx = permuted(inst, perm)
    D_val, _ = O.density_matrix(inst)
    P_val, _ = O.density_matrix(pinst)
    e0, n0 = O.traces(inst, D_val, inst.H_val, inst.S_val)
    e1, n1 = O.traces(pinst, P_val, pinst.H_val, pinst.S_val)
    assert abs(e0 - e1) < 1e-9 and abs(n0 - n1) < 1e-9
    assert np.abs(dense(inst, D_val)[np.ix_(fidx, fidx)] - dense(pinst, P_val)).max() < 1e-10


# ------------------------------------------------------------------ tests

def test_scalar_closed_form():
    check_scalar_closed_form()


def test_diagonal_orthogonal():
    check_diagonal_orthogonal()


def test_golden_2x2():
    check_golden_2x2()


@pytest.mark.parametrize("seed", range(20))
def test_general_2x2_closed_form(seed):
    check_general_2x2_closed_form(seed)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_bruteforce(seed):
    check_tiny_bruteforce(seed)


@pytest.mark.parametrize("seed", range(3))
def test_sign_invariants(seed):
    check_sign_invariants(seed)


def test_whole_system():
    check_whole_system()


def test_submatrices_idempotent_and_inertia():
    check_submatrices("c1")
    check_submatrices("t_23")


def test_gather_against_dense():
    check_gather("t_small")
    check_gather("t_slab")


def test_scatter_and_traces_against_dense():
    check_scatter_and_traces("c1")


def test_chain_truncation():
    check_chain_truncation()


def test_mu_inside_gap():
    check_mu_in_gap()


def test_permutation_invariance():
    check_permutation()


def test_gaps_open_at_mu():
    """mu = 0 sits in a gap of every submatrix (no occupation 1/2 cases)."""
    for name in ("c1", "t_small", "t_23"):
        inst = get_config(name)
        _, st = O.density_matrix(inst, mols=range(0, inst.nmol, 4))
        assert min(s["gap"] for s in st) > 1e-3


# ------------------------------------------------------------------ planted mistakes

def _fails(check, *args):
    try:
        check(*args)
    except (AssertionError, np.linalg.LinAlgError, ValueError, IndexError):
        return True
    return False


def test_planted_flipped_occupation(monkeypatch):
    monkeypatch.setattr(O, "theta", lambda x: np.where(x < 0, 1.0, np.where(x > 0, 0.0, 0.5)))
    assert _fails(check_whole_system) and _fails(check_golden_2x2)


def test_planted_transposed_eigvecs(monkeypatch):
    def bad(Hk, Sk, mu):
        lam, C = scipy.linalg.eigh(Hk, Sk)
        return (C.T * O.theta(mu - lam)[None, :]) @ C, lam
    monkeypatch.setattr(O, "density", bad)
    assert _fails(check_general_2x2_closed_form, 3) and _fails(check_whole_system)


def test_planted_missing_overlap_metric(monkeypatch):
    def bad(Hk, Sk, mu):          # ordinary eigenproblem: drops S
        lam, C = np.linalg.eigh(Hk)
        return (C * O.theta(mu - lam)[None, :]) @ C.T, lam
    monkeypatch.setattr(O, "density", bad)
    assert _fails(check_golden_2x2) and _fails(check_whole_system)


def test_planted_transposed_block_gather(monkeypatch):
    def bad_block(pattern, val, t):
        I = int(pattern.rowblk[t])
        J = int(np.searchsorted(pattern.colptr, t, side="right") - 1)
        dI, dJ = int(pattern.blk_dim[I]), int(pattern.blk_dim[J])
        s = int(pattern.valoff[t])
        return val[s:s + dI * dJ].reshape(dI, dJ)          # row-major read of a col-major block
    monkeypatch.setattr(O, "_block", bad_block)
    assert _fails(check_gather, "t_small")


def test_planted_wrong_own_columns(monkeypatch):
    def bad(pattern, k, offs):
        return np.arange(offs[0], offs[1])                  # first member, not molecule k
    monkeypatch.setattr(O, "own_columns", bad)
    assert _fails(check_scatter_and_traces, "c1") or _fails(check_gather, "t_small")


def test_planted_ns_missing_half(monkeypatch):
    orig = O.newton_schulz_sign

    def bad(A, scale=None, tol=1e-12, maxit=100, order=2):
        n = A.shape[0]
        b = np.abs(A).sum(axis=1).max() if scale is None else scale
        X = A / b
        for it in range(maxit):
            X = X @ (3.0 * np.eye(n) - X @ X)               # the 1/2 is dropped
            if not np.all(np.isfinite(X)):
                break
        r = np.linalg.norm(X @ X - np.eye(n)) / math.sqrt(n)
        return X, maxit, [r]
    monkeypatch.setattr(O, "newton_schulz_sign", bad)
    assert _fails(check_sign_invariants, 0)
    monkeypatch.setattr(O, "newton_schulz_sign", orig)


def test_planted_trace_wrong_matrix(monkeypatch):
    def bad(pattern, D_val, H_val, S_val, k):
        eh, es = [], []
        for t in range(int(pattern.colptr[k]), int(pattern.colptr[k + 1])):
            I = int(pattern.rowblk[t])
            sz = int(pattern.blk_dim[I]) * int(pattern.blk_dim[k])
            s = int(pattern.valoff[t])
            eh.append(math.fsum((D_val[s:s + sz] * S_val[s:s + sz]).tolist()))   # H <-> S swapped
            es.append(math.fsum((D_val[s:s + sz] * H_val[s:s + sz]).tolist()))
        return math.fsum(eh), math.fsum(es)
    monkeypatch.setattr(O, "column_traces", bad)
    assert _fails(check_whole_system) and _fails(check_chain_truncation)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_third_order_sign_invariants(seed):
    """The order-3 polynomial iteration reaches the same sign (X^2 = I, commutes with
    A, integer trace, scale invariance)."""
    check_sign_invariants(seed, order=3)


def test_third_order_polynomial_and_rate():
    """The order-3 step on scalars is p(x) = x (15 - 10 x^2 + 3 x^4) / 8: p(1) = 1,
    p'(1) = p''(1) = 0 (so 1 - p(1 - e) = O(e^3)), p(-x) = -p(x); on a matrix it
    needs fewer steps than Newton-Schulz and agrees with the eigen-decomposition."""
    x = np.array([0.3, 0.9, 1.0, -0.7])
    A = np.diag(x)
    X, _, _ = O.newton_schulz_sign(A, scale=1.0, maxit=1, tol=0.0, order=3)
    p = x * (15 - 10 * x ** 2 + 3 * x ** 4) / 8
    assert np.allclose(np.diag(X), p, rtol=0, atol=1e-15)
    for e in (1e-2, 1e-3):
        y = 1 - e
        assert abs(1 - y * (15 - 10 * y ** 2 + 3 * y ** 4) / 8) < 20 * e ** 3
    rng = np.random.default_rng(7)
    n = 40
    B = rng.standard_normal((n, n))
    A = 0.5 * (B + B.T)
    lam, V = np.linalg.eigh(A)
    ref = V @ np.diag(np.sign(lam)) @ V.T
    X2, it2, _ = O.newton_schulz_sign(A, tol=1e-12, maxit=300)
    X3, it3, _ = O.newton_schulz_sign(A, tol=1e-12, maxit=300, order=3)
    assert np.abs(X3 - ref).max() < 1e-8 and np.abs(X2 - ref).max() < 1e-8
    assert it3 < it2


def test_planted_third_order_coefficient(monkeypatch):
    orig = O.newton_schulz_sign

    def bad(A, scale=None, tol=1e-12, maxit=100, order=2):
        n = A.shape[0]
        b = np.abs(A).sum(axis=1).max() if scale is None else scale
        X = A / b
        for it in range(maxit):
            X2 = X @ X
            X = 0.125 * X @ (15.0 * np.eye(n) - 10.0 * X2 + 2.0 * X2 @ X2)   # 3 -> 2
            if not np.all(np.isfinite(X)):
                break
        r = np.linalg.norm(X @ X - np.eye(n)) / math.sqrt(n)
        return X, maxit, [r]
    monkeypatch.setattr(O, "newton_schulz_sign", bad)
    assert _fails(check_sign_invariants, 0, 3)
    monkeypatch.setattr(O, "newton_schulz_sign", orig)


# ------------------------------------------------------------------ per-submatrix driver

def read_block_column(inst, D_val, k, offs):
    """Block column k of a scattered D, laid out as T_k(D)[:, own columns]."""
    mem = inst.members(k)
    m = int(inst.blk_dim[k])
    out = np.zeros((int(offs[-1]), m))
    for a, I in enumerate(mem):
        t = int(inst.colptr[k]) + a
        dI = int(inst.blk_dim[I])
        s = int(inst.valoff[t])
        out[offs[a]:offs[a + 1], :] = D_val[s:s + dI * m].reshape(m, dI).T
    return out


@pytest.mark.parametrize("name,mu", [("c1", None), ("c1", -0.3), ("t_23", None)])
def test_submatrix_result_matches_scattered_density(name, mu):
    """submatrix_result (the per-molecule record the GPU tests and the benchmark
    compare against) holds exactly block column k of density_matrix's D, which the
    whole-system, closed-form and inertia pins fix; its traces are the column sums."""
    inst = get_config(name)
    ks = list(range(0, inst.nmol, max(1, inst.nmol // 6)))
    D_val, _ = O.density_matrix(inst, mu=mu, mols=ks)
    for k in ks:
        r = O.submatrix_result(inst, k, mu=mu)
        assert np.array_equal(r["members"], inst.members(k))
        assert r["D_cols"].shape == (r["n"], int(inst.blk_dim[k]))
        assert np.array_equal(read_block_column(inst, D_val, k, r["offs"]), r["D_cols"])
        eh, es = O.column_traces(inst, D_val, inst.H_val, inst.S_val, k)
        assert abs(r["tr_dh"] - eh) <= 1e-12 * max(1.0, abs(eh))
        assert abs(r["tr_ds"] - es) <= 1e-12 * max(1.0, abs(es))


# ------------------------------------------------------------------ chemical potential search

LEVELS = np.array([-1.5, -0.2, -0.01, 0.3, 0.7, 2.0])


def check_mu_bisection_hand():
    """Diagonal system, S = I: Tr(D(mu) S) = #{h_i < mu}.  Target 3, tolerance 0.5,
    bracket [-4, 3]; the trials worked out by hand:
      -0.5 (count 1: lo), 1.25 (5: hi), 0.375 (4: hi), -0.0625 (2: lo), 0.15625 (3: done)."""
    inst = instance_from_dense(np.diag(LEVELS), np.eye(6), [2, 2, 2], np.ones((3, 3)))
    r = O.mu_search(inst, 3, -4.0, 3.0, tol=0.5)
    assert r["converged"]
    assert [m for m, _ in r["hist"]] == [-0.5, 1.25, 0.375, -0.0625, 0.15625]
    assert [round(n, 12) for _, n in r["hist"]] == [1.0, 5.0, 4.0, 2.0, 3.0]
    assert abs(r["tr_dh"] - LEVELS[:3].sum()) < 1e-14


def check_mu_search_whole_system():
    """c1 with every submatrix the whole system: the count is the number of
    generalized eigenvalues below mu (SciPy eigenvalues of the dense pair), and the
    search ends between the 96th and 97th eigenvalue, with D S D = D there."""
    inst = get_config("c1_whole")
    H, S = dense(inst, inst.H_val), dense(inst, inst.S_val)
    lam = scipy.linalg.eigvalsh(H, S)
    spectra = O.submatrix_spectra(inst, mols=[0])
    for mu in (-1.2, -0.9, -0.5, 0.0, 0.4, 0.8):
        # one submatrix is the whole system: its columns for molecule 0 only, so
        # evaluate the full D from the whole-system decomposition directly
        C, lk = spectra[0]["C"], spectra[0]["lam"]
        Dfull = (C * O.theta(mu - lk)[None, :]) @ C.T
        assert abs(np.trace(Dfull @ S) - np.sum(lam < mu)) < 1e-9
    r = O.mu_search(inst, inst.n_elec, -1.0, 3.0)
    assert len(r["hist"]) >= 2
    assert r["converged"]
    assert lam[inst.n_elec - 1] < r["mu"] < lam[inst.n_elec]
    assert abs(r["tr_ds"] - inst.n_elec) < 1e-9
    assert abs(r["tr_dh"] - lam[:inst.n_elec].sum()) < 1e-9
    D = dense(inst, r["D_val"])
    assert np.abs(D @ S @ D - D).max() < 1e-10
    # every trial's count is the number of eigenvalues below it
    for mu, n in r["hist"]:
        assert abs(n - np.sum(lam < mu)) < 1e-9


def test_mu_bisection_hand_sequence():
    check_mu_bisection_hand()


def test_mu_search_whole_system():
    check_mu_search_whole_system()


def test_density_at_reuses_spectra():
    """The cached-spectrum route equals the fresh per-mu route bit for bit."""
    inst = get_config("c1")
    ks = [0, 5, 17, 31]
    spectra = O.submatrix_spectra(inst, mols=ks)
    for mu in (-0.9, -0.3, 0.0, 0.3):
        D1 = O.density_matrix_at(inst, spectra, mu)
        D2, _ = O.density_matrix(inst, mu=mu, mols=ks)
        assert np.array_equal(D1, D2)


def test_planted_bisection_swapped(monkeypatch):
    def bad(count, n_target, mu_lo, mu_hi, tol=0.5, max_iter=40):
        lo, hi, hist = mu_lo, mu_hi, []
        for _ in range(max_iter):
            mu = 0.5 * (lo + hi)
            n = count(mu)
            hist.append((mu, n))
            if n < n_target - tol:
                hi = mu                      # wrong side
            elif n > n_target + tol:
                lo = mu
            else:
                return mu, hist, True
        return mu, hist, False
    monkeypatch.setattr(O, "mu_bisection", bad)
    assert _fails(check_mu_bisection_hand) and _fails(check_mu_search_whole_system)


def test_planted_occupation_ignores_mu(monkeypatch):
    def bad(inst, spectra, mu):
        return O.density_matrix(inst, mu=0.0, mols=[s["k"] for s in spectra])[0]
    monkeypatch.setattr(O, "density_matrix_at", bad)
    assert _fails(check_mu_bisection_hand)


# ------------------------------------------------------------------ submatrix combination

def chain_instance(dims):
    """Molecules 0..len(dims)-1 in a chain: block (I, J) stored for |I - J| <= 1."""
    nm = len(dims)
    nf = int(sum(dims))
    present = np.abs(np.subtract.outer(np.arange(nm), np.arange(nm))) <= 1
    rng = np.random.default_rng(5)
    B = rng.standard_normal((nf, nf))
    return instance_from_dense(0.5 * (B + B.T), np.eye(nf), dims, present)


def check_combination_hand():
    """Chain 0-1-2-3 of one-function molecules: submatrix sizes 2, 3, 3, 2.
    Eq. 9 gains: (0,1) 8 + 27 - 27 = 8, (1,2) 27 + 27 - 64 = -10, (2,3) 8; (0,2) and
    (1,3) overlap too, but their union is all four rows: 8 + 27 - 64 < 0.  The best
    is a tie at 8 between (0,1) and (2,3); (0,1) comes first, leaving {0,1} (rows
    0-2, n 3); then (2,3) gains 8; then {0,1} with {2,3} would need n 4:
    27 + 27 - 64 < 0.  Result [[0, 1], [2, 3]].
    Eq. 10 with rates (1, 1) .. (4, 100) (time per flop 1 / rate): c(2) = 8/34,
    c(3) = 27/67, c(4) = 64/100; (0,1) and (2,3) gain c(2), {0,1} with {2,3} gains
    2 c(3) - c(4) > 0, so everything ends in one group."""
    inst = chain_instance([1, 1, 1, 1])
    assert [len(inst.members(k)) for k in range(4)] == [2, 3, 3, 2]
    assert O.combine_groups(inst, range(4), 9) == [[0, 1], [2, 3]]
    table = [(1, 1.0), (4, 100.0)]
    assert abs(O.rate_at(3, table) - 67.0) < 1e-12
    assert O.combine_groups(inst, range(4), 10, table) == [[0, 1, 2, 3]]
    # a size limit of 3 stops Eq. 10 at the first two combinations
    assert O.combine_groups(inst, range(4), 10, table, max_n=3) == [[0, 1], [2, 3]]


def check_combination_local_optimum(name, criterion, table=None):
    """No pair of final groups whose submatrices overlap satisfies the criterion (the
    gains recomputed from the group rows by brute force), every molecule is in
    exactly one group, and the groups' D equals the plain per-molecule D when every
    group is a single molecule."""
    inst = get_config(name)
    groups = O.combine_groups(inst, range(inst.nmol), criterion, table)
    flat = sorted(k for g in groups for k in g)
    assert flat == list(range(inst.nmol))
    rows = [set(O.submatrix_rows(inst, g).tolist()) for g in groups]

    def n_of(r):
        return int(sum(int(inst.blk_dim[j]) for j in r))
    for i in range(len(groups)):
        for j in range(i + 1, len(groups)):
            if rows[i] & rows[j]:
                gain = (O.combination_cost(n_of(rows[i]), criterion, table)
                        + O.combination_cost(n_of(rows[j]), criterion, table)
                        - O.combination_cost(n_of(rows[i] | rows[j]), criterion, table))
                assert not gain > 0, (i, j, gain)
    return inst, groups


def test_combination_hand_example():
    check_combination_hand()


def test_combination_local_optimum_and_constant_rate():
    inst, g9 = check_combination_local_optimum("t_sweep", 9)
    assert len(g9) < inst.nmol          # the small-cutoff boxes combine
    # a constant rate makes Eq. 10 the cubic criterion of Eq. 9
    _, g10 = check_combination_local_optimum("t_sweep", 10, [(1, 5.0), (10000, 5.0)])
    assert g10 == g9


def test_groups_density_special_cases():
    """Singleton groups give density_matrix's D bit for bit; one group holding every
    molecule makes each submatrix the whole system, whose exact D (eigenvalues of the
    dense pair) fills every stored block."""
    inst = get_config("c1")
    D1, _ = O.density_matrix(inst)
    D2, recs = O.density_matrix_groups(inst, [[k] for k in range(inst.nmol)])
    assert np.array_equal(D1, D2)
    Dw, recs = O.density_matrix_groups(inst, [list(range(inst.nmol))])
    H, S = dense(inst, inst.H_val), dense(inst, inst.S_val)
    lam, C = scipy.linalg.eigh(H, S)
    Dex = (C[:, lam < 0]) @ C[:, lam < 0].T
    mask = dense(inst, np.ones_like(inst.H_val)) != 0
    assert np.abs(dense(inst, Dw)[mask] - Dex[mask]).max() < 1e-10
    assert recs[0]["n"] == inst.nfunc


def test_planted_combination_ignores_overlap(monkeypatch):
    """Counting n_i + n_j instead of the union never satisfies Eq. 9."""
    monkeypatch.setattr(O, "combined_dimension", lambda ni, nj, nij: ni + nj)
    assert _fails(check_combination_hand)


def test_planted_combination_criterion_reversed(monkeypatch):
    real = O.combination_cost
    monkeypatch.setattr(O, "combination_cost", lambda n, c, t=None: -real(n, c, t))
    assert _fails(check_combination_hand)
