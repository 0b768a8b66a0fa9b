"""FP64 CPU oracle for the non-orthogonal local submatrix method (NOLSM).

TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this module; only the
tests, the smoke check and the benchmark's CPU-baseline leg do.  It shares no
code with the GPU path: inputs come from the seeded generators in `workloads`,
and every step below is a plain, slow restatement of the paper.

What the method computes (paper, Sec. II "Overview of the Problem"):

  * Eq. 5: at zero electronic temperature the density matrix is
        D = 1/2 (I - sign(S^-1 H0 - mu I)) S^-1.
  * Submatrix method, steps 1-3 (Sec. II, Fig. 1): for a column (here: the
    column block of one molecule, the "one submatrix for several columns"
    variant), keep the rows that are non-zero in that column, evaluate the
    matrix function on the dense submatrix, and write the columns that belong
    to the molecule back into a result with the pattern of the input.
  * Eq. 8: the non-orthogonal variant combines the patterns of H0 and S, builds
    T_i(H0) and T_i(S), and evaluates
        T_i(D) = 1/2 (I - sign(T_i(S)^-1 T_i(H0) - mu I)) T_i(S)^-1.
  * Eq. 4: E_elec = Tr(D H0).

Because sign() of a diagonalisable matrix with real spectrum is defined through
its eigen-decomposition, the oracle evaluates Eq. 8 exactly via the generalized
symmetric eigenproblem H_k C = S_k C Lambda, C^T S_k C = I:
    S_k^-1 H_k - mu I = C (Lambda - mu) C^-1,  C^-1 = C^T S_k,  S_k^-1 = C C^T,
    T_k(D) = 1/2 C (I - sgn(Lambda - mu)) C^T S_k C C^T = C theta(mu - Lambda) C^T,
with theta(x) = 1 for x > 0, 0 for x < 0 and 1/2 at x = 0 (sign(0) = 0).

Eq. 6-7 (Newton-Schulz) is provided as `newton_schulz_sign` for the tests (which
pin it and compare it with the eigen route); the oracle's density never depends
on it, and nothing else uses it.
`order=3` gives the third-order member of the same polynomial family (Sec. II's
higher-order schemes); both are pinned by the sign identities, the eigen-
decomposition, the scalar map and (order 3) its cubic rate.

The chemical potential (Sec. V-A: the runs iterate mu until the system is
charge neutral) is found by `mu_search`: bisection of the electron count
Tr(D(mu) S) against the target, with every submatrix's eigen-decomposition
computed once and reused for every trial mu, since only the occupations
theta(mu - Lambda) depend on mu.

Readings of points the paper leaves open are listed in the design notes: the
molecule-column grouping, mu = 0, no spin factor (Tr(DS) counts occupied
orbitals), sign(0) = 0, and the scaling X0 = A / b with b >= rho(A) that puts the
spectrum inside the Newton-Schulz basin.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


# ----------------------------------------------------------------- step 1: submatrix

def members(pattern, k: int) -> np.ndarray:
    """Molecules whose block in column block k is stored (ascending, includes k).

    Submatrix method step 1: the rows kept for column block k are those with
    non-zero elements in that column block; H and S share one pattern here, so
    this is already the combined pattern of Eq. 8.
    """
    return np.asarray(pattern.rowblk[pattern.colptr[k]:pattern.colptr[k + 1]])


def _find_block(pattern, I: int, J: int) -> int:
    """Index of stored block (I, J) or -1 (binary search of column J's rows)."""
    lo, hi = int(pattern.colptr[J]), int(pattern.colptr[J + 1])
    rows = pattern.rowblk[lo:hi]
    p = int(np.searchsorted(rows, I))
    if p < rows.shape[0] and int(rows[p]) == I:
        return lo + p
    return -1


def _block(pattern, val: np.ndarray, t: int) -> np.ndarray:
    """Stored block t as a dense dI x dJ array (column-major storage)."""
    I = int(pattern.rowblk[t])
    J = int(np.searchsorted(pattern.colptr, t, side="right") - 1)
    dI, dJ = int(pattern.blk_dim[I]), int(pattern.blk_dim[J])
    start = int(pattern.valoff[t])
    return val[start:start + dI * dJ].reshape(dJ, dI).T


def gather(pattern, val: np.ndarray, k: int):
    """T_k(A): dense principal submatrix of A on the functions of members(k).

    Returns (A_k, offsets) with offsets[a] the first row of member a in A_k.
    Blocks absent from the pattern are zero.
    """
    mem = members(pattern, k)
    dims = [int(pattern.blk_dim[J]) for J in mem]
    offs = np.zeros(len(mem) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(dims)
    n = int(offs[-1])
    A = np.zeros((n, n))
    for b, J in enumerate(mem):
        for a, I in enumerate(mem):
            t = _find_block(pattern, int(I), int(J))
            if t < 0:
                continue
            A[offs[a]:offs[a + 1], offs[b]:offs[b + 1]] = _block(pattern, val, t)
    return A, offs


def own_columns(pattern, k: int, offs: np.ndarray) -> np.ndarray:
    """Local column indices of molecule k's own functions inside T_k."""
    mem = members(pattern, k)
    a = int(np.nonzero(mem == k)[0][0])
    return np.arange(offs[a], offs[a + 1])


# ----------------------------------------------------------------- step 2: matrix function

def theta(x: np.ndarray) -> np.ndarray:
    """Occupation 1/2 (1 - sgn(x_in)) written for x = mu - lambda."""
    return np.where(x > 0, 1.0, np.where(x < 0, 0.0, 0.5))


def density(Hk: np.ndarray, Sk: np.ndarray, mu: float):
    """Eq. 8 evaluated exactly: T_k(D) = C theta(mu - Lambda) C^T.

    Returns (D_k, eigenvalues).
    """
    lam, C = scipy.linalg.eigh(Hk, Sk)
    occ = theta(mu - lam)
    Dk = (C * occ[None, :]) @ C.T
    return Dk, lam


def density_literal(Hk: np.ndarray, Sk: np.ndarray, mu: float) -> np.ndarray:
    """Eq. 8 typed as printed, with an explicit inverse and scipy's signm.

    For small cross-checks only (signm works on the non-symmetric S^-1 H).
    """
    n = Hk.shape[0]
    Sinv = np.linalg.inv(Sk)
    sgn = scipy.linalg.signm(Sinv @ Hk - mu * np.eye(n))
    return 0.5 * (np.eye(n) - np.real(sgn)) @ Sinv


def newton_schulz_sign(A: np.ndarray, scale: float | None = None, tol: float = 1e-12,
                       maxit: int = 100, order: int = 2):
    """Eq. 6-7: X0 = A / b, X_{k+1} = 1/2 X_k (3 I - X_k^2), sign(A) = lim X_k.

    order = 3 takes the next member of the same family of matrix-polynomial sign
    iterations (the higher-order schemes Sec. II mentions): the odd polynomial of
    degree 5 with p(1) = 1 and p'(1) = p''(1) = 0,
        X_{k+1} = 1/8 X_k (15 I - 10 X_k^2 + 3 X_k^4),
    which converges cubically from the same basin.

    b defaults to the infinity norm (a Gershgorin bound on the spectral radius,
    valid for the real spectra of S^-1 H - mu I), which keeps every eigenvalue of
    X0 inside the convergence basin in modulus.  Stops when
    ||X^2 - I||_F / sqrt(n) <= tol.  Returns (X, iterations, residual history).
    """
    if order not in (2, 3):
        raise ValueError("order must be 2 or 3")
    n = A.shape[0]
    b = np.abs(A).sum(axis=1).max() if scale is None else scale
    X = A / b
    eye = np.eye(n)
    hist = []
    for it in range(maxit + 1):
        X2 = X @ X
        r = np.linalg.norm(X2 - eye) / math.sqrt(n)
        hist.append(r)
        if r <= tol or it == maxit:
            return X, it, hist
        if order == 2:
            X = 0.5 * X @ (3.0 * eye - X2)
        else:
            X = 0.125 * X @ (15.0 * eye - 10.0 * X2 + 3.0 * X2 @ X2)
    return X, maxit, hist


# ----------------------------------------------------------------- step 3: write back

def scatter(pattern, D_val: np.ndarray, k: int, Dk: np.ndarray, offs: np.ndarray) -> None:
    """Write the columns of molecule k from T_k(D) into block column k of D.

    Submatrix method step 3: for every stored block (I, k), rows of member I in
    T_k(D), columns of molecule k.  Nothing outside the pattern is written.
    """
    mem = members(pattern, k)
    cols = own_columns(pattern, k, offs)
    dk = int(pattern.blk_dim[k])
    for a, I in enumerate(mem):
        t = _find_block(pattern, int(I), k)
        dI = int(pattern.blk_dim[I])
        start = int(pattern.valoff[t])
        # column-major block (I, k): element (r, c) at start + r + c * dI
        D_val[start:start + dI * dk] = Dk[offs[a]:offs[a + 1], cols].T.reshape(-1)


# ----------------------------------------------------------------- Eq. 4 and the electron count

def column_traces(pattern, D_val, H_val, S_val, k: int):
    """Contributions of block column k to Tr(D H) and Tr(D S).

    Tr(D H) = sum_ij D_ij H_ji = sum_ij D_ij H_ij because H is symmetric; the
    sum over block column k collects the terms with j in molecule k.
    """
    eh, es = [], []
    for t in range(int(pattern.colptr[k]), int(pattern.colptr[k + 1])):
        I = int(pattern.rowblk[t])
        sz = int(pattern.blk_dim[I]) * int(pattern.blk_dim[k])
        s = int(pattern.valoff[t])
        eh.append(math.fsum((D_val[s:s + sz] * H_val[s:s + sz]).tolist()))
        es.append(math.fsum((D_val[s:s + sz] * S_val[s:s + sz]).tolist()))
    return math.fsum(eh), math.fsum(es)


def traces(pattern, D_val, H_val, S_val):
    """(Tr(D H), Tr(D S)) summed exactly-rounded over block columns (Eq. 4)."""
    parts = [column_traces(pattern, D_val, H_val, S_val, k) for k in range(pattern.nmol)]
    return math.fsum(p[0] for p in parts), math.fsum(p[1] for p in parts)


# ----------------------------------------------------------------- drivers

def submatrix_result(inst, k: int, mu: float | None = None) -> dict:
    """Everything the oracle knows about molecule k's submatrix.

    D_cols is T_k(D)[:, own columns] (n_k x m_k), i.e. exactly the values the
    write-back step stores into block column k.
    """
    mu = inst.mu if mu is None else mu
    Hk, offs = gather(inst, inst.H_val, k)
    Sk, _ = gather(inst, inst.S_val, k)
    Dk, lam = density(Hk, Sk, mu)
    cols = own_columns(inst, k, offs)
    Dc = Dk[:, cols]
    e_h = math.fsum((Dc * Hk[:, cols]).ravel().tolist())
    e_s = math.fsum((Dc * Sk[:, cols]).ravel().tolist())
    return {"k": k, "n": Hk.shape[0], "members": members(inst, k), "offs": offs,
            "cols": cols, "D_cols": Dc, "tr_dh": e_h, "tr_ds": e_s,
            "gap": float(np.min(np.abs(lam - mu))), "rho": float(np.max(np.abs(lam - mu))),
            "n_occ": int(np.sum(lam < mu)), "eigvals": lam}


def density_matrix(inst, mu: float | None = None, mols=None):
    """Scattered D (values aligned with H_val / S_val) and per-molecule stats.

    mols: molecules to evaluate (default all).  Block columns of molecules not
    evaluated stay zero.
    """
    mu = inst.mu if mu is None else mu
    D_val = np.zeros_like(inst.H_val)
    stats = []
    for k in (range(inst.nmol) if mols is None else mols):
        Hk, offs = gather(inst, inst.H_val, k)
        Sk, _ = gather(inst, inst.S_val, k)
        Dk, lam = density(Hk, Sk, mu)
        scatter(inst, D_val, int(k), Dk, offs)
        stats.append({"k": int(k), "n": Hk.shape[0],
                      "gap": float(np.min(np.abs(lam - mu))),
                      "rho": float(np.max(np.abs(lam - mu)))})
    return D_val, stats


def energy_per_atom_error(inst, e_a: float, e_b: float) -> float:
    """|E_a - E_b| / N_atoms (sites count as atoms)."""
    return abs(e_a - e_b) / inst.natoms


# ----------------------------------------------------------------- chemical potential

def submatrix_spectra(inst, mols=None) -> list:
    """Generalized eigen-decomposition H_k C = S_k C Lambda of every submatrix.

    Eq. 8 depends on mu only through the occupations theta(mu - Lambda), so one
    decomposition per submatrix serves every trial chemical potential.
    """
    out = []
    for k in (range(inst.nmol) if mols is None else mols):
        Hk, offs = gather(inst, inst.H_val, int(k))
        Sk, _ = gather(inst, inst.S_val, int(k))
        lam, C = scipy.linalg.eigh(Hk, Sk)
        out.append({"k": int(k), "offs": offs, "lam": lam, "C": C})
    return out


def density_matrix_at(inst, spectra: list, mu: float) -> np.ndarray:
    """Scattered D at chemical potential mu from precomputed submatrix spectra."""
    D_val = np.zeros_like(inst.H_val)
    for sp in spectra:
        Dk = (sp["C"] * theta(mu - sp["lam"])[None, :]) @ sp["C"].T
        scatter(inst, D_val, sp["k"], Dk, sp["offs"])
    return D_val


def mu_bisection(count, n_target: float, mu_lo: float, mu_hi: float, tol: float = 0.5,
                 max_iter: int = 40):
    """Bisection of the chemical potential on the electron count.

    count(mu) returns Tr(D(mu) S).  The bracket keeps count(lo) below
    n_target - tol and count(hi) above n_target + tol (the caller's bracket is
    taken as such); every trial is the midpoint, and the search ends at the
    first trial whose count lies within tol of the target, or after max_iter
    trials.  Returns (mu, [(mu_t, count_t), ...], converged).
    """
    lo, hi = float(mu_lo), float(mu_hi)
    hist = []
    mu = 0.5 * (lo + hi)
    for _ in range(max_iter):
        mu = 0.5 * (lo + hi)
        n = float(count(mu))
        hist.append((mu, n))
        if n < n_target - tol:
            lo = mu
        elif n > n_target + tol:
            hi = mu
        else:
            return mu, hist, True
    return mu, hist, False


def mu_search(inst, n_target: float, mu_lo: float, mu_hi: float, tol: float = 0.5,
              max_iter: int = 40) -> dict:
    """Charge-neutral chemical potential of the whole instance (Sec. V-A).

    Returns the final mu, the trial history, the scattered D at that mu and its
    traces (Tr(D H0), Tr(D S)).
    """
    spectra = submatrix_spectra(inst)

    def count(mu):
        D = density_matrix_at(inst, spectra, mu)
        return traces(inst, D, inst.H_val, inst.S_val)[1]

    mu, hist, ok = mu_bisection(count, n_target, mu_lo, mu_hi, tol, max_iter)
    D = density_matrix_at(inst, spectra, mu)
    e, ne = traces(inst, D, inst.H_val, inst.S_val)
    return {"mu": mu, "hist": hist, "converged": ok, "D_val": D, "tr_dh": e, "tr_ds": ne}


# ----------------------------------------------------------------- submatrix combination

def submatrix_rows(pattern, group) -> np.ndarray:
    """Molecules of the submatrix shared by the columns of `group` (Sec. IV-B: the
    submatrix of a set of combined columns keeps every row that is non-zero in any
    of them): the union of the block columns' stored rows, ascending."""
    rows = np.unique(np.concatenate([members(pattern, int(k)) for k in group]))
    return rows.astype(np.int64)


def rate_at(n: int, table) -> float:
    """Measured GEMM throughput at dimension n: linear interpolation of the table
    [(n_i, rate_i)] (ascending n_i), constant beyond its ends."""
    ns = [float(a) for a, _ in table]
    rs = [float(b) for _, b in table]
    x = float(n)
    if x <= ns[0]:
        return rs[0]
    if x >= ns[-1]:
        return rs[-1]
    i = 0
    while ns[i + 1] < x:
        i += 1
    t = (x - ns[i]) / (ns[i + 1] - ns[i])
    d = (rs[i + 1] - rs[i]) * t
    return rs[i] + d


def combined_dimension(n_i: int, n_j: int, n_ij: int) -> int:
    """Dimension of the submatrix of two combined column sets (Eq. 9):
    n_i + n_j - n_(i and j), with n_(i and j) the rows the two share."""
    return n_i + n_j - n_ij


def combination_cost(n: int, criterion: int, table=None):
    """Eq. 9: n^3 (the flop count of the dense products, exact integer).
    Eq. 10: p(n) n^3 with p(n) the time per flop, 1 / rate_at(n) (reading: the
    predicted run time of the submatrix's products)."""
    n3 = int(n) ** 3
    if criterion == 9:
        return n3
    return float(n3) / rate_at(n, table)


def combine_groups(pattern, mols, criterion: int = 9, table=None, max_n: int | None = None):
    """Greedy submatrix combination (Sec. IV-B, Eq. 9 or Eq. 10).

    Start from one group per molecule.  Two groups are candidates when their
    submatrices overlap (share at least one row molecule).  Combining them gives the
    submatrix on the union of their rows, of dimension n_i + n_j - n_(i and j); the
    gain is cost(n_i) + cost(n_j) - cost(n_i + n_j - n_(i and j)), positive exactly
    when the criterion of Eq. 9 (or Eq. 10) holds.  Repeatedly combine the candidate
    pair with the largest gain (ties: the pair whose smallest molecules, smaller
    first, come first in lexicographic order), skipping pairs whose combined
    dimension would exceed max_n, until no candidate pair has a positive gain.

    Returns the groups as ascending molecule lists, ordered by their first molecule.
    """
    dims = np.asarray(pattern.blk_dim, dtype=np.int64)
    group = {int(k): [int(k)] for k in mols}             # keyed by smallest molecule
    rows = {k: set(int(j) for j in members(pattern, k)) for k in group}

    def dim(rset):
        return int(sum(int(dims[j]) for j in rset))

    def gain(a, b):
        nu = combined_dimension(dim(rows[a]), dim(rows[b]), dim(rows[a] & rows[b]))
        if max_n is not None and nu > max_n:
            return None
        return (combination_cost(dim(rows[a]), criterion, table)
                + combination_cost(dim(rows[b]), criterion, table)
                - combination_cost(nu, criterion, table))

    while True:
        best = None
        keys = sorted(group)
        for i, a in enumerate(keys):
            for b in keys[i + 1:]:
                if not rows[a] & rows[b]:
                    continue
                g = gain(a, b)
                if g is None or not g > 0:
                    continue
                if best is None or g > best[0]:
                    best = (g, a, b)
        if best is None:
            break
        _, a, b = best
        group[a] = sorted(group[a] + group.pop(b))
        rows[a] = rows[a] | rows.pop(b)
    return [group[a] for a in sorted(group)]


def density_matrix_groups(inst, groups, mu: float | None = None):
    """Scattered D when each group of molecules shares one submatrix (Sec. IV-B):
    Eq. 8 on the submatrix over the union of the group's rows, and every molecule of
    the group writes its own block column from it (step 3 of the submatrix method).
    Returns D and per-group records (molecules, n, per-molecule Tr(D H0) and Tr(D S)
    column contributions)."""
    mu = inst.mu if mu is None else mu
    D_val = np.zeros_like(inst.H_val)
    recs = []
    for grp in groups:
        rows = submatrix_rows(inst, grp)
        idx = np.concatenate([np.arange(inst.blk_off[j], inst.blk_off[j + 1]) for j in rows])
        pos = {int(j): a for a, j in enumerate(rows)}
        loc = np.zeros(len(rows) + 1, dtype=np.int64)
        loc[1:] = np.cumsum([int(inst.blk_dim[j]) for j in rows])
        Hk = np.zeros((idx.size, idx.size))
        Sk = np.zeros((idx.size, idx.size))
        for b, J in enumerate(rows):
            for t in range(int(inst.colptr[J]), int(inst.colptr[J + 1])):
                I = int(inst.rowblk[t])
                if I not in pos:
                    continue
                a = pos[I]
                Hk[loc[a]:loc[a + 1], loc[b]:loc[b + 1]] = _block(inst, inst.H_val, t)
                Sk[loc[a]:loc[a + 1], loc[b]:loc[b + 1]] = _block(inst, inst.S_val, t)
        Dk, lam = density(Hk, Sk, mu)
        per = []
        for k in grp:
            cols = np.arange(loc[pos[k]], loc[pos[k] + 1])
            dk = int(inst.blk_dim[k])
            for t in range(int(inst.colptr[k]), int(inst.colptr[k + 1])):
                I = int(inst.rowblk[t])
                a = pos[I]
                s = int(inst.valoff[t])
                D_val[s:s + int(inst.blk_dim[I]) * dk] = Dk[loc[a]:loc[a + 1], cols].T.reshape(-1)
            per.append(column_traces(inst, D_val, inst.H_val, inst.S_val, k))
        recs.append({"mols": list(grp), "n": int(idx.size), "traces": per,
                     "gap": float(np.min(np.abs(lam - mu)))})
    return D_val, recs
