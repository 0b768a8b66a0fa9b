"""Small hand-made block-sparse instances for the oracle pins."""
import numpy as np

from workloads.water import Instance


def instance_from_dense(H, S, blk_dim, present, mu=0.0, atoms=None, name="hand"):
    """Block-sparse Instance from dense H, S and a molecule-pair mask.

    present[I, J] says whether block (I, J) is stored (the diagonal always is).
    Values of absent blocks are dropped.
    """
    blk_dim = np.asarray(blk_dim, dtype=np.int32)
    nmol = blk_dim.size
    blk_off = np.zeros(nmol + 1, dtype=np.int64)
    blk_off[1:] = np.cumsum(blk_dim)
    present = np.array(present, dtype=bool) | np.eye(nmol, dtype=bool)
    colptr = [0]
    rowblk, valoff, Hv, Sv = [], [], [], []
    off = 0
    for J in range(nmol):
        for I in range(nmol):
            if not present[I, J]:
                continue
            rowblk.append(I)
            valoff.append(off)
            hb = H[blk_off[I]:blk_off[I + 1], blk_off[J]:blk_off[J + 1]]
            sb = S[blk_off[I]:blk_off[I + 1], blk_off[J]:blk_off[J + 1]]
            Hv.append(hb.T.reshape(-1))     # column major
            Sv.append(sb.T.reshape(-1))
            off += hb.size
        colptr.append(len(rowblk))
    atoms = np.ones(nmol, dtype=np.int32) if atoms is None else np.asarray(atoms, np.int32)
    return Instance(name=name, nmol=nmol, blk_dim=blk_dim, blk_off=blk_off,
                    colptr=np.array(colptr, dtype=np.int64),
                    rowblk=np.array(rowblk, dtype=np.int32),
                    valoff=np.array(valoff, dtype=np.int64),
                    H_val=np.concatenate(Hv), S_val=np.concatenate(Sv), mu=mu, atoms=atoms,
                    box=0.0, r_cut=0.0, shift=0.0, centres=np.zeros((nmol, 3)), meta={})


def permuted(inst, perm):
    """The same system with molecules renumbered: new molecule p is old perm[p]."""
    from workloads import to_dense
    blk = (inst.blk_dim, inst.blk_off, inst.colptr, inst.rowblk, inst.valoff)
    H = to_dense(blk, inst.H_val)
    S = to_dense(blk, inst.S_val)
    present = np.zeros((inst.nmol, inst.nmol), dtype=bool)
    for J in range(inst.nmol):
        present[inst.rowblk[inst.colptr[J]:inst.colptr[J + 1]], J] = True
    fidx = np.concatenate([np.arange(inst.blk_off[p], inst.blk_off[p + 1]) for p in perm])
    return instance_from_dense(H[np.ix_(fidx, fidx)], S[np.ix_(fidx, fidx)],
                               inst.blk_dim[perm], present[np.ix_(perm, perm)], mu=inst.mu,
                               atoms=inst.atoms[perm]), fidx


def dense(inst, val):
    from workloads import to_dense
    return to_dense((inst.blk_dim, inst.blk_off, inst.colptr, inst.rowblk, inst.valoff), val)


def golden_energies(name, inst, mu=None):
    """The oracle's per-molecule Tr(D H0), Tr(D S) column contributions for the whole
    named workload at the instance's mu (or `mu`) (tests/golden/, written by
    tests/golden/make_energies.py), checked against the instance's digest."""
    import os
    from tests.golden.make_energies import golden_name, instance_digest
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        golden_name(name, None if mu is None or mu == inst.mu else mu))
    with np.load(path, allow_pickle=False) as z:
        rec = {k: z[k] for k in z.files}
    assert str(rec["instance_sha256"]) == instance_digest(inst), f"{path}: other instance"
    return rec


def sampled_errors(inst, D, st, picks, index, mu=None):
    """Max |D - D_oracle| over the written columns of molecules `picks` and the
    largest single-molecule |Tr(D_k H) difference| / atoms_k (no cancellation
    between molecules); st[index[k]] is molecule k's record."""
    from oracle import nolsm_oracle as O
    dmax, de = 0.0, 0.0
    for k in picks:
        ref = O.submatrix_result(inst, k, mu=mu)
        got = np.zeros_like(ref["D_cols"])
        for a, I in enumerate(ref["members"]):
            t = int(inst.colptr[k]) + a
            dI, m = int(inst.blk_dim[I]), int(inst.blk_dim[k])
            got[ref["offs"][a]:ref["offs"][a + 1], :] = \
                D[inst.valoff[t]:inst.valoff[t] + dI * m].reshape(m, dI).T
        dmax = max(dmax, float(np.abs(got - ref["D_cols"]).max()))
        de = max(de, abs(float(st["tr_dh"][index[k]]) - ref["tr_dh"]) / int(inst.atoms[k]))
        # no eigenvalue converged to the wrong sign
        assert st["n_neg"][index[k]] == ref["n_occ"], (k, st["n_neg"][index[k]], ref["n_occ"])
    return dmax, de
