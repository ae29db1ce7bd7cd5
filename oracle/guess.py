"""Initial guess of section 3.3 (oracle side; test infrastructure only).

For every fragment (molecule), the generalized eigenproblem H0 c = lambda S c restricted to the
fragment's own AOs, solved by LAPACK (scipy.linalg.eigh, the routine family the paper uses as
its reference); eigenvalues ascending; each vector's first entry within a relative 1e-10 of its
largest |c| made positive.  C0 columns: the occupied MOs of group 0, 1, .. (fragments ascending within a group,
lambda ascending within a fragment), then the virtual MOs in the same order.  Independent of the
HIP library.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh

# entries within this relative distance of the largest |c| count as tied for the sign rule
# (symmetric molecules have exactly equal entries, which rounding would otherwise decide)
TIE = 1e-10


def fragment_blocks(system, atom_frag):
    """Dense S and H0 of each fragment from the atom-block pattern."""
    aoo = system.ao_offset()
    n_frag = int(atom_frag.max()) + 1
    first = np.searchsorted(atom_frag, np.arange(n_frag))
    last = np.searchsorted(atom_frag, np.arange(n_frag), side="right")
    out = []
    for f in range(n_frag):
        a0, a1 = first[f], last[f]
        lo, hi = aoo[a0], aoo[a1]
        S = np.zeros((hi - lo, hi - lo))
        H = np.zeros((hi - lo, hi - lo))
        for a in range(a0, a1):
            for k in range(system.blk_rowptr[a], system.blk_rowptr[a + 1]):
                b = system.blk_col[k]
                if b < a0 or b >= a1:
                    continue
                na, nb = system.atom_nao[a], system.atom_nao[b]
                sl = slice(system.blk_off[k], system.blk_off[k] + na * nb)
                S[aoo[a] - lo:aoo[a] - lo + na, aoo[b] - lo:aoo[b] - lo + nb] = system.S_val[sl].reshape(na, nb)
                H[aoo[a] - lo:aoo[a] - lo + na, aoo[b] - lo:aoo[b] - lo + nb] = system.H0_val[sl].reshape(na, nb)
        out.append((int(lo), S, H))
    return out


def fragment_guess(system, atom_frag, frag_nocc, frag_group, drop: float = 0.0):
    """(c0_colptr, c0_row, c0_val, mo_group, n_occ, eigenvalues per fragment)."""
    atom_frag = np.asarray(atom_frag)
    blocks = fragment_blocks(system, atom_frag)
    vecs, lams = [], []
    for lo, S, H in blocks:
        w, V = eigh(H, S)
        for j in range(V.shape[1]):
            a = np.abs(V[:, j])
            k = int(np.nonzero(a >= a.max() * (1.0 - TIE))[0][0])
            if V[k, j] < 0:
                V[:, j] = -V[:, j]
        vecs.append(V)
        lams.append(w)
    n_groups = int(np.max(frag_group)) + 1
    order = [[f for f in range(len(blocks)) if frag_group[f] == g] for g in range(n_groups)]
    cols, groups = [], []
    for occ in (True, False):
        for g in range(n_groups):
            for f in order[g]:
                n = vecs[f].shape[0]
                js = range(0, frag_nocc[f]) if occ else range(frag_nocc[f], n)
                for j in js:
                    cols.append((blocks[f][0], vecs[f][:, j]))
                    groups.append(g)
    cp = np.zeros(len(cols) + 1, dtype=np.int64)
    rr, vv = [], []
    for c, (lo, v) in enumerate(cols):
        keep = np.abs(v) >= drop
        rr.append(np.arange(lo, lo + len(v), dtype=np.int32)[keep])
        vv.append(v[keep])
        cp[c + 1] = cp[c] + int(keep.sum())
    return cp, np.concatenate(rr), np.concatenate(vv), np.array(groups, dtype=np.int32), int(sum(frag_nocc)), lams
