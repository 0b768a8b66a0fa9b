"""Synthetic molecular systems with a block-sparse Hamiltonian and overlap matrix.

The paper's benchmark (a solvated spike protein under GFN-xTB) is not available,
so these seeded generators stand in for it with the same structure: molecules
carry a few basis functions on each of their sites, the overlap decays with
distance and is cut off at r_c, and a molecule's submatrix spans every molecule
whose centre lies within r_c.  Nothing here evaluates the density matrix; it only
produces the two input matrices and their sparsity pattern.

Storage (shared by every consumer): a symmetric molecule-block-sparse matrix in
compressed sparse column form over block columns.

  blk_dim[I]            basis functions of molecule I
  blk_off[I]            first global basis function of molecule I (length nmol+1)
  colptr[J]..colptr[J+1]  stored blocks of block column J
  rowblk[t]             block row I of stored block t (ascending inside a column)
  valoff[t]             offset of block t in the value array; the block is
                        dense, column major, blk_dim[I] x blk_dim[J]

H and S share the pattern and the value offsets, so H_val[valoff[t] + r + c*dI]
is H_{blk_off[I]+r, blk_off[J]+c}.  Both triangles are stored.

Construction (the instance recipe):
  * water-like molecules: a heavy site and two light sites at 0.96 A with a
    104.5 degree angle, Haar-random orientation, centres on a jittered cubic grid
    at the number density of liquid water (0.03343 per A^3);
  * protein-like units: five sites in a zig-zag chain (1.5 A bonds), six
    functions per site, the middle site is the centre;
  * S0_ij = exp(-r_ij^2 / (2 * 1.2^2)) * c_ij for i != j, with r_ij the
    minimum-image distance between the sites of the two functions and
    c_ij ~ U(-0.3, 0.3) drawn per unordered pair from a counter-based generator;
    S0_ij = 0 if r_ij >= r_c or the molecule pair is not in the pattern;
    S0_ii = 1;
  * block (I, J) is stored iff the minimum-image centre distance d_IJ < r_c;
  * S = S0 + delta * I with delta = max(0, 0.1 - lambda_min(S0)), so that
    lambda_min(S) >= 0.1 and, by Cauchy interlacing, every principal submatrix
    is positive definite with smallest eigenvalue >= 0.1;
  * H_ii = -1.0 for the first floor(n_f/2) functions of each molecule and +0.5
    for the rest; H_ij = -0.4 * S0_ij off the diagonal.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os
import sys

import numpy as np

from .rng import MAX_INDEX, pair_uniform

WATER_DENSITY = 0.03343          # molecules per A^3 at 1 g/cm^3
SIGMA = 1.2                      # Gaussian width of the overlap decay (A)
C_AMPL = 0.3                     # c_ij ~ U(-C_AMPL, C_AMPL)
H_OFFDIAG = -0.4                 # H_ij = H_OFFDIAG * S0_ij
ONSITE_LO, ONSITE_HI = -1.0, 0.5
LAMBDA_FLOOR = 0.1               # target lower bound on lambda_min(S)


@dataclasses.dataclass
class Instance:
    """A block-sparse (H, S) pair plus the geometry it was built from."""
    name: str
    nmol: int
    blk_dim: np.ndarray          # int32 [nmol]
    blk_off: np.ndarray          # int64 [nmol+1]
    colptr: np.ndarray           # int64 [nmol+1]
    rowblk: np.ndarray           # int32 [nnzb]
    valoff: np.ndarray           # int64 [nnzb]
    H_val: np.ndarray            # float64 [nval]
    S_val: np.ndarray            # float64 [nval]
    mu: float
    atoms: np.ndarray            # int32 [nmol] atoms (sites) per molecule
    box: float                   # cubic box edge (A)
    r_cut: float
    shift: float                 # delta added to the diagonal of S
    centres: np.ndarray          # float64 [nmol, 3]
    meta: dict

    @property
    def nnzb(self) -> int:
        return int(self.rowblk.shape[0])

    @property
    def nval(self) -> int:
        return int(self.H_val.shape[0])

    @property
    def nfunc(self) -> int:
        return int(self.blk_off[-1])

    @property
    def natoms(self) -> int:
        return int(self.atoms.sum())

    @property
    def n_elec(self) -> int:
        """Electrons of the neutral system: one per function with the lower onsite
        energy, i.e. floor(n_f / 2) per molecule (no spin factor)."""
        return int((self.blk_dim // 2).sum())

    def members(self, k: int) -> np.ndarray:
        """Molecules present in block column k (ascending; includes k)."""
        return self.rowblk[self.colptr[k]:self.colptr[k + 1]]

    def submatrix_dims(self) -> np.ndarray:
        """n_k for every molecule's submatrix."""
        out = np.empty(self.nmol, dtype=np.int64)
        for k in range(self.nmol):
            out[k] = int(self.blk_dim[self.members(k)].sum())
        return out


# ----------------------------------------------------------------------------- geometry

def _haar_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-random rotation matrices from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_frame() -> np.ndarray:
    """Heavy site at the origin, two light sites at 0.96 A, 104.5 degrees apart."""
    half = math.radians(104.5) / 2
    b = 0.96
    return np.array([[0.0, 0.0, 0.0],
                     [b * math.sin(half), 0.0, b * math.cos(half)],
                     [-b * math.sin(half), 0.0, b * math.cos(half)]])


def _unit_frame() -> np.ndarray:
    """Five-site zig-zag chain (1.5 A bonds, 110 degree angles), centre site first."""
    b = 1.5
    half = math.radians(110.0) / 2
    dx, dz = b * math.sin(half), b * math.cos(half)
    chain = np.array([[-2 * dx, 0.0, 0.0], [-dx, 0.0, dz], [0.0, 0.0, 0.0],
                      [dx, 0.0, dz], [2 * dx, 0.0, 0.0]])
    chain -= chain[2]
    return chain[[2, 0, 1, 3, 4]]


def _grid_centres(rng, n: int, lo: np.ndarray, edge: np.ndarray, jitter: float = 0.1):
    """First n points of a seeded permutation of an m^3 grid filling the box
    [lo, lo+edge), each jittered uniformly by +-jitter of the grid spacing."""
    m = int(math.ceil(round(n ** (1.0 / 3.0), 9)))
    while m ** 3 < n:
        m += 1
    idx = rng.permutation(m ** 3)[:n]
    ix, iy, iz = idx // (m * m), (idx // m) % m, idx % m
    spacing = edge / m
    grid = np.stack([ix, iy, iz], axis=1).astype(np.float64) + 0.5
    pos = lo + grid * spacing
    pos += (rng.random((n, 3)) * 2.0 - 1.0) * jitter * spacing
    return pos


# ----------------------------------------------------------------------------- pattern

def _min_image(d: np.ndarray, box: float) -> np.ndarray:
    return d - box * np.round(d / box)


def _neighbour_pairs(centres: np.ndarray, box: float, r_cut: float):
    """All ordered pairs (I, J), I != J, with minimum-image centre distance < r_cut."""
    n = centres.shape[0]
    if not math.isfinite(r_cut):
        I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        mask = I != J
        return I[mask], J[mask]
    if n > 16384 and r_cut < box / 2:
        from scipy.spatial import cKDTree
        wrapped = np.mod(centres, box)
        tree = cKDTree(wrapped, boxsize=box)
        pairs = tree.query_pairs(r_cut, output_type="ndarray")
        # re-check with the generator's own distance so the pattern is exact
        d = _min_image(centres[pairs[:, 0]] - centres[pairs[:, 1]], box)
        keep = np.einsum("ij,ij->i", d, d) < r_cut * r_cut
        pairs = pairs[keep]
        return (np.concatenate([pairs[:, 0], pairs[:, 1]]),
                np.concatenate([pairs[:, 1], pairs[:, 0]]))
    Is, Js = [], []
    chunk = max(1, (1 << 22) // n)
    for a in range(0, n, chunk):
        d = _min_image(centres[a:a + chunk, None, :] - centres[None, :, :], box)
        r2 = np.einsum("ijk,ijk->ij", d, d)
        ii, jj = np.nonzero(r2 < r_cut * r_cut)
        ii = ii + a
        keep = ii != jj
        Is.append(ii[keep])
        Js.append(jj[keep])
    return np.concatenate(Is), np.concatenate(Js)


def _csc_pattern(nmol: int, I: np.ndarray, J: np.ndarray):
    """Block CSC with the diagonal block always present, rows ascending."""
    rows = np.concatenate([I, np.arange(nmol)])
    cols = np.concatenate([J, np.arange(nmol)])
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    colptr = np.zeros(nmol + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, rows.astype(np.int32), cols.astype(np.int32)


# ----------------------------------------------------------------------------- values

def _fill_values(inst_dims, blk_off, rowblk, colblk, valoff, sites, fn_site, onsite,
                 box, r_cut, seed, H_val, S_val):
    """Evaluate S0 and H for every stored block, grouped by block shape."""
    rc2 = r_cut * r_cut if math.isfinite(r_cut) else np.inf
    two_s2 = 2.0 * SIGMA * SIGMA
    shapes = np.stack([inst_dims[rowblk], inst_dims[colblk]], axis=1)
    jobs = []
    for dI, dJ in np.unique(shapes, axis=0):
        sel = np.nonzero((shapes[:, 0] == dI) & (shapes[:, 1] == dJ))[0]
        step = max(1, (1 << 21) // int(dI * dJ))
        jobs += [(int(dI), int(dJ), sel[a:a + step]) for a in range(0, sel.size, step)]

    def work(job):
        dI, dJ, t = job
        fr = np.arange(dI)
        fc = np.arange(dJ)
        if True:
            Ib, Jb = rowblk[t], colblk[t]
            sI = fn_site[Ib][:, :dI]                      # [nt, dI] site of each row fn
            sJ = fn_site[Jb][:, :dJ]
            pI = np.take_along_axis(sites[Ib], sI[:, :, None], axis=1)   # [nt, dI, 3]
            pJ = np.take_along_axis(sites[Jb], sJ[:, :, None], axis=1)   # [nt, dJ, 3]
            d = _min_image(pI[:, :, None, :] - pJ[:, None, :, :], box)   # [nt, dI, dJ, 3]
            r2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
            gi = blk_off[Ib][:, None] + fr[None, :]                       # [nt, dI]
            gj = blk_off[Jb][:, None] + fc[None, :]
            GI = np.broadcast_to(gi[:, :, None], r2.shape)
            GJ = np.broadcast_to(gj[:, None, :], r2.shape)
            c = (2.0 * pair_uniform(seed, GI, GJ) - 1.0) * C_AMPL
            s0 = np.exp(-r2 / two_s2) * c
            s0 = np.where(r2 < rc2, s0, 0.0)
            diag = GI == GJ
            s0 = np.where(diag, 1.0, s0)
            h = np.where(diag, onsite[GI], H_OFFDIAG * s0)
            # column-major blocks: element (r, c) at r + c*dI
            sz = int(dI * dJ)
            dst = (valoff[t][:, None] + np.arange(sz)[None, :]).ravel()
            S_val[dst] = np.transpose(s0, (0, 2, 1)).reshape(-1)
            H_val[dst] = np.transpose(h, (0, 2, 1)).reshape(-1)

    # chunks write disjoint slices; NumPy releases the GIL inside the array work
    workers = min(16, os.cpu_count() or 1)
    # large instances (the 65,536-molecule box takes minutes) report their progress
    report = H_val.size > (1 << 30)
    if workers > 1 and len(jobs) > 1:
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            for i, _ in enumerate(ex.map(work, jobs)):
                if report and (i + 1) % max(1, len(jobs) // 10) == 0:
                    print(f"[workloads] values: {i + 1}/{len(jobs)} chunks", file=sys.stderr,
                          flush=True)
    else:
        for j in jobs:
            work(j)


def block_matvec(inst_like, val: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A x for a symmetric block-sparse matrix (used for the diagonal shift)."""
    blk_dim, blk_off, colptr, rowblk, valoff = inst_like
    nmol = blk_dim.shape[0]
    y = np.zeros_like(x)
    colblk = np.repeat(np.arange(nmol), np.diff(colptr))
    shapes = np.stack([blk_dim[rowblk], blk_dim[colblk]], axis=1)
    for dI, dJ in np.unique(shapes, axis=0):
        sel = np.nonzero((shapes[:, 0] == dI) & (shapes[:, 1] == dJ))[0]
        idx = valoff[sel][:, None] + np.arange(dI * dJ)[None, :]
        B = val[idx].reshape(-1, dJ, dI)            # B[t, c, r] = A_{I r, J c}
        xr = x[blk_off[rowblk[sel]][:, None] + np.arange(dI)[None, :]]   # [nt, dI]
        contrib = np.einsum("tcr,tr->tc", B, xr)   # (A^T x)_J = (A x)_J by symmetry
        dst = blk_off[colblk[sel]][:, None] + np.arange(dJ)[None, :]
        np.add.at(y, dst.ravel(), contrib.ravel())
    return y


def to_dense(blk, val: np.ndarray) -> np.ndarray:
    """Dense copy of a block-sparse matrix (small instances only)."""
    blk_dim, blk_off, colptr, rowblk, valoff = blk
    n = int(blk_off[-1])
    A = np.zeros((n, n))
    for J in range(blk_dim.shape[0]):
        dJ = int(blk_dim[J])
        for t in range(int(colptr[J]), int(colptr[J + 1])):
            I = int(rowblk[t])
            dI = int(blk_dim[I])
            blk_vals = val[valoff[t]:valoff[t] + dI * dJ].reshape(dJ, dI).T
            A[blk_off[I]:blk_off[I] + dI, blk_off[J]:blk_off[J] + dJ] = blk_vals
    return A


def lambda_min(blk, S_val: np.ndarray, nfunc: int) -> float:
    """Smallest eigenvalue of a symmetric block-sparse matrix (dense for small)."""
    if nfunc <= 3000:
        return float(np.linalg.eigvalsh(to_dense(blk, S_val))[0])
    from scipy.sparse.linalg import LinearOperator, eigsh
    op = LinearOperator((nfunc, nfunc), matvec=lambda v: block_matvec(blk, S_val, v),
                        dtype=np.float64)
    w = eigsh(op, k=1, which="SA", tol=1e-6, v0=np.ones(nfunc), return_eigenvectors=False)
    return float(w[0])


def lambda_min_lanczos(blk, S_val: np.ndarray, nfunc: int, device: str = "cuda",
                       tol: float = 1e-8, max_steps: int = 800, check_every: int = 10,
                       log=None):
    """Smallest eigenvalue of a symmetric block-sparse matrix by Lanczos with full
    reorthogonalisation, the products evaluated with PyTorch on `device` (for
    instances whose host-side matrix-vector product is too slow, such as the
    65,536-molecule box).  Returns (theta, residual, steps): theta is the smallest
    Ritz value, an upper bound on lambda_min, and residual = |beta_j s_j| bounds the
    distance from theta to the nearest eigenvalue."""
    import torch
    from scipy.linalg import eigh_tridiagonal
    blk_dim, blk_off, colptr, rowblk, valoff = blk
    nmol = blk_dim.shape[0]
    dev = torch.device(device)
    colblk = np.repeat(np.arange(nmol), np.diff(colptr))
    shapes = np.stack([blk_dim[rowblk], blk_dim[colblk]], axis=1)
    S_dev = torch.from_numpy(S_val).to(dev)
    groups = []
    for dI, dJ in np.unique(shapes, axis=0):
        dI, dJ = int(dI), int(dJ)
        sel = np.nonzero((shapes[:, 0] == dI) & (shapes[:, 1] == dJ))[0]
        step = max(1, (1 << 25) // (dI * dJ))
        for a in range(0, sel.size, step):
            s = sel[a:a + step]
            groups.append((dI, dJ,
                           torch.from_numpy(valoff[s]).to(dev),
                           torch.from_numpy(blk_off[rowblk[s]]).to(dev),
                           torch.from_numpy(blk_off[colblk[s]]).to(dev)))

    def matvec(x):
        y = torch.zeros_like(x)
        for dI, dJ, vo, ro, co in groups:
            idx = vo[:, None] + torch.arange(dI * dJ, device=dev)[None, :]
            B = S_dev[idx].view(-1, dJ, dI)                       # B[t, c, r] = A_{I r, J c}
            xr = x[ro[:, None] + torch.arange(dI, device=dev)[None, :]]
            contrib = torch.bmm(B, xr.unsqueeze(-1)).squeeze(-1)  # (A^T x)_J = (A x)_J
            y.index_add_(0, (co[:, None] + torch.arange(dJ, device=dev)[None, :]).reshape(-1),
                         contrib.reshape(-1))
        return y

    Q = torch.empty((max_steps + 1, nfunc), dtype=torch.float64, device=dev)
    Q[0] = 1.0 / math.sqrt(nfunc)
    alpha, beta = [], []
    theta, resid = float("nan"), float("inf")
    for j in range(max_steps):
        w = matvec(Q[j])
        a = float(torch.dot(w, Q[j]))
        w -= a * Q[j]
        if j > 0:
            w -= beta[-1] * Q[j - 1]
        for _ in range(2):                                      # full reorthogonalisation
            w -= Q[:j + 1].T @ (Q[:j + 1] @ w)
        b = float(torch.linalg.vector_norm(w))
        alpha.append(a)
        beta.append(b)
        if (j + 1) % check_every == 0 or b == 0.0 or j + 1 == max_steps:
            ev, vec = eigh_tridiagonal(np.asarray(alpha), np.asarray(beta[:-1]),
                                       select="i", select_range=(0, 0))
            theta, resid = float(ev[0]), abs(b * float(vec[-1, 0]))
            if log is not None:
                log(f"Lanczos step {j + 1}: theta {theta:.9f}, residual {resid:.2e}")
            if resid <= tol * max(1.0, abs(theta)):
                return theta, resid, j + 1
        if b == 0.0:
            break
        Q[j + 1] = w / b
    return theta, resid, len(alpha)


def shift_for(lmin: float) -> float:
    """delta = max(0, 0.1 - lambda_min), rounded up to a 1e-3 grid."""
    need = LAMBDA_FLOOR - lmin + 1e-4
    return 0.0 if need <= 0 else math.ceil(need * 1000.0) / 1000.0


# ----------------------------------------------------------------------------- builder

def build_instance(name: str, species: list, box: float, r_cut: float, seed: int,
                   mu: float = 0.0, shift: float | None = None) -> Instance:
    """Assemble H and S for a list of molecules.

    species: list of (centres [m,3], frame [ns,3], fn_per_site tuple, atoms) groups.
    The geometry RNG stream is numpy's PCG64 seeded with `seed` (rotations drawn
    per group in order); the couplings use the counter generator with `seed`.
    """
    rng = np.random.default_rng([seed, 0x5eed])
    cents, site_list, fnsite_list, dims, atoms, onsites = [], [], [], [], [], []
    max_sites = max(fr.shape[0] for _, fr, _, _ in species)
    max_fn = max(sum(f) for _, _, f, _ in species)
    for centres, frame, fps, nat in species:
        m = centres.shape[0]
        R = _haar_rotations(rng, m)
        pos = centres[:, None, :] + np.einsum("mij,sj->msi", R, frame)
        padded = np.zeros((m, max_sites, 3))
        padded[:, :frame.shape[0]] = pos
        site_list.append(padded)
        fs = np.concatenate([np.full(c, s, dtype=np.int64) for s, c in enumerate(fps)])
        nf = fs.size
        fsp = np.zeros((m, max_fn), dtype=np.int64)
        fsp[:, :nf] = fs
        fnsite_list.append(fsp)
        dims.append(np.full(m, nf, dtype=np.int32))
        atoms.append(np.full(m, nat, dtype=np.int32))
        ons = np.where(np.arange(nf) < nf // 2, ONSITE_LO, ONSITE_HI)
        onsites.append(np.tile(ons, m))
        cents.append(centres)
    centres = np.concatenate(cents)
    sites = np.concatenate(site_list)
    fn_site = np.concatenate(fnsite_list)
    blk_dim = np.concatenate(dims)
    atoms = np.concatenate(atoms)
    onsite = np.concatenate(onsites)
    nmol = centres.shape[0]
    blk_off = np.zeros(nmol + 1, dtype=np.int64)
    blk_off[1:] = np.cumsum(blk_dim)
    if blk_off[-1] > MAX_INDEX:
        raise ValueError("instance too large for the coupling counter")

    I, J = _neighbour_pairs(centres, box, r_cut)
    colptr, rowblk, colblk = _csc_pattern(nmol, I, J)
    sizes = blk_dim[rowblk].astype(np.int64) * blk_dim[colblk].astype(np.int64)
    valoff = np.zeros(rowblk.size, dtype=np.int64)
    valoff[1:] = np.cumsum(sizes)[:-1]
    nval = int(sizes.sum())
    H_val = np.empty(nval)
    S_val = np.empty(nval)
    _fill_values(blk_dim, blk_off, rowblk, colblk, valoff, sites, fn_site, onsite,
                 box, r_cut, seed, H_val, S_val)

    blk = (blk_dim, blk_off, colptr, rowblk, valoff)
    lmin0 = None
    if shift is None:
        lmin0 = lambda_min(blk, S_val, int(blk_off[-1]))
        shift = shift_for(lmin0)
    if shift != 0.0:
        d = blk_dim[colblk]
        # diagonal blocks: element (r, r) sits at r*(d+1)
        diag_t = np.nonzero(rowblk == colblk)[0]
        for t in diag_t:
            dd = int(blk_dim[rowblk[t]])
            S_val[valoff[t] + np.arange(dd) * (dd + 1)] += shift
        del d
    return Instance(name=name, nmol=nmol, blk_dim=blk_dim, blk_off=blk_off, colptr=colptr,
                    rowblk=rowblk, valoff=valoff, H_val=H_val, S_val=S_val, mu=mu,
                    atoms=atoms, box=box, r_cut=r_cut, shift=float(shift), centres=centres,
                    meta={"seed": seed, "lambda_min_S0": lmin0})


def water_box(nmol: int, fn_split=(4, 1, 1), r_cut: float = 6.0, seed: int = 0,
              mu: float = 0.0, shift: float | None = None, name: str = "water") -> Instance:
    """nmol water-like molecules in a periodic cube at liquid-water density."""
    box = (nmol / WATER_DENSITY) ** (1.0 / 3.0)
    rng = np.random.default_rng([seed, 0xce17])
    centres = _grid_centres(rng, nmol, np.zeros(3), np.full(3, box))
    return build_instance(name, [(centres, _water_frame(), tuple(fn_split), 3)], box,
                          r_cut, seed, mu=mu, shift=shift)


def water_with_slab(n_water: int, n_units: int, unit_density_ratio: float = 1.35,
                    r_cut: float = 8.0, seed: int = 0, mu: float = 0.0,
                    shift: float | None = None, name: str = "water+slab") -> Instance:
    """Water box (13+5+5 functions) embedding a slab of five-site units
    (6 functions per site) at unit_density_ratio times water's number density.

    The box volume is the water volume plus the slab volume; the slab spans the
    full x-y cross-section and is centred in z.
    """
    v_w = n_water / WATER_DENSITY
    v_s = n_units / (WATER_DENSITY * unit_density_ratio)
    box = (v_w + v_s) ** (1.0 / 3.0)
    thick = v_s / (box * box)
    z0 = 0.5 * (box - thick)
    rng = np.random.default_rng([seed, 0xce17])
    # water fills the two regions outside the slab, split by volume
    below = int(round(n_water * z0 / (box - thick)))
    above = n_water - below
    w1 = _grid_centres(rng, below, np.zeros(3), np.array([box, box, z0]))
    w2 = _grid_centres(rng, above, np.array([0.0, 0.0, z0 + thick]),
                       np.array([box, box, box - z0 - thick]))
    u = _grid_centres(rng, n_units, np.array([0.0, 0.0, z0]), np.array([box, box, thick]))
    waters = np.concatenate([w1, w2])
    inst = build_instance(name, [(waters, _water_frame(), (13, 5, 5), 3),
                                 (u, _unit_frame(), (6, 6, 6, 6, 6), 5)],
                          box, r_cut, seed, mu=mu, shift=shift)
    inst.meta.update({"slab_z0": z0, "slab_thickness": thick})
    return inst


def direct_sum(parts: list, name: str = "sum") -> Instance:
    """Independent instances side by side as one block-diagonal instance (molecules
    renumbered in order; no block couples two parts).  Used to put submatrices of
    very different sizes into one batch."""
    nmol = sum(p.nmol for p in parts)
    blk_dim = np.concatenate([p.blk_dim for p in parts]).astype(np.int32)
    blk_off = np.zeros(nmol + 1, dtype=np.int64)
    blk_off[1:] = np.cumsum(blk_dim)
    colptr, rowblk, valoff, H, S = [np.zeros(1, dtype=np.int64)], [], [], [], []
    m0 = nnz0 = val0 = 0
    for p in parts:
        colptr.append(p.colptr[1:] + nnz0)
        rowblk.append(p.rowblk + m0)
        valoff.append(p.valoff + val0)
        H.append(p.H_val)
        S.append(p.S_val)
        m0 += p.nmol
        nnz0 += p.nnzb
        val0 += p.nval
    return Instance(name=name, nmol=nmol, blk_dim=blk_dim, blk_off=blk_off,
                    colptr=np.concatenate(colptr), rowblk=np.concatenate(rowblk).astype(np.int32),
                    valoff=np.concatenate(valoff), H_val=np.concatenate(H),
                    S_val=np.concatenate(S), mu=parts[0].mu,
                    atoms=np.concatenate([p.atoms for p in parts]).astype(np.int32),
                    box=max(p.box for p in parts), r_cut=max(p.r_cut for p in parts),
                    shift=max(p.shift for p in parts),
                    centres=np.concatenate([p.centres for p in parts]),
                    meta={"parts": [(p.name, p.nmol, p.r_cut, p.shift) for p in parts]})
