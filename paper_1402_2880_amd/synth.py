"""Seeded synthetic tight-binding systems shaped like the paper's liquid-water boxes.

This module only builds the *inputs* of the sparse SCF problem (paper, section 2
and section 3.7): atomic positions, the AO overlap S and the reference
Kohn-Sham matrix H0 on the atom-neighbour pattern, Hubbard parameters U and
reference populations q0, together with the two set-up products that the
method's hot path takes as given:

* the MO groups, from the constrained k-means of section 3.2 (run on molecule
  centres so that groups never split a molecule);
* the initial guess C0 of section 3.3: one non-self-consistent solve per
  molecule, occupied MOs of every group followed by virtual MOs of every group.

It holds none of the SCF arithmetic (orthonormalization, C^T X C products,
Jacobi rotations, charges, energies).  Both the FP64 oracle and the HIP library
receive exactly these arrays.

Model (the paper uses DFTB Slater-Koster tables that are not available; this
is a synthetic stand-in with the same structure):

* water: O carries s, px, py, pz (4 AOs), H carries s (1 AO); O-H 0.96 A,
  H-O-H 104.5 deg, uniformly random orientation;
* molecules placed by random sequential addition in an open cube: O-O >= 2.8 A,
  and every intermolecular O-H or H-H contact >= 1.8 A (the orientation is
  redrawn until it fits);
* two-centre integrals V(r) = 0.3 exp(-r/0.9) Ha and sigma(r) = 0.2 exp(-r/0.9)
  (r in Angstrom, hard cut at 6 A) with Slater-Koster direction-cosine factors;
* onsite energies O s -0.88, O p -0.45, H s +0.30 Ha; U_O = 0.30, U_H = 0.25 Ha;
  q0 = 6 (O), 1 (H).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
from scipy.linalg import eigh

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903

# element codes
EL_O, EL_H, EL_C = 0, 1, 2
NAO = {EL_O: 4, EL_H: 1, EL_C: 4}
# With typical DFTB onsite energies (O p -0.33, H s -0.24) and Hubbard values (0.50, 0.42)
# the weak two-centre hopping of this model (0.10 Ha at the O-H bond) leaves a
# self-consistent HOMO-LUMO gap of ~0.01 Ha in the 128-molecule box and the plain SCC
# iteration diverges.  O p -0.45, U 0.30 / 0.25 and H s +0.30 give a self-consistent gap
# of ~0.36 Ha; with H s +0.10 (gap ~0.2 Ha) the unmixed SCC iteration still converges for
# 1024 molecules but turns unstable at 4096 (charge sloshing grows with the box).
# V0, r0 and the geometry rules are untouched.
ONSITE = {EL_O: (-0.88, -0.45), EL_H: (0.30, None), EL_C: (-0.50, -0.20)}
HUBBARD_U = {EL_O: 0.30, EL_H: 0.25, EL_C: 0.30}
Q0 = {EL_O: 6.0, EL_H: 1.0, EL_C: 4.0}

SK_V0 = 0.3       # Ha
SK_SIGMA0 = 0.2   # dimensionless
SK_R0 = 0.9       # Angstrom
# pairs with a carbon atom: the curve above gives 0.05-0.09 Ha hoppings at C-C and C-H bond
# lengths and metallic chains (H0 gap ~4e-4 Ha); covalent chains need stronger, longer-ranged
# two-centre elements (gap ~0.6 Ha for octanes with these)
SK_C_V0, SK_C_SIGMA0, SK_C_R0 = 1.5, 0.3, 1.2
SK_CUTOFF = 6.0   # Angstrom

OH_BOND = 0.96              # Angstrom
HOH_ANGLE = 104.5           # degrees
MIN_OO = 2.8                # Angstrom
N_LINK = 16                 # molecules per MO group


@dataclasses.dataclass
class System:
    """Inputs of one sparse SCF problem.  Arrays are numpy, C-contiguous.

    Atom-block CSR pattern: block (a, b) for b in blk_col[blk_rowptr[a]:blk_rowptr[a+1]]
    holds the nao_a x nao_b row-major sub-matrix starting at blk_off[k] in S_val / H0_val.
    The self block (a, a) is always present.  Columns are sorted within each row.

    C0 is given column-wise (CSC): column j has rows c0_row[c0_colptr[j]:c0_colptr[j+1]].
    The first n_occ columns are the doubly occupied MOs.
    """

    name: str
    seed: int
    box_angstrom: float
    n_atoms: int
    atom_el: np.ndarray        # int32 [n_atoms]
    atom_nao: np.ndarray       # int32 [n_atoms]
    xyz_bohr: np.ndarray       # float64 [n_atoms, 3]
    hubbard_u: np.ndarray      # float64 [n_atoms]
    q0: np.ndarray             # float64 [n_atoms]
    atom_mol: np.ndarray       # int32 [n_atoms]
    atom_group: np.ndarray     # int32 [n_atoms]
    n_groups: int
    blk_rowptr: np.ndarray     # int64 [n_atoms + 1]
    blk_col: np.ndarray        # int32 [nnzb]
    blk_off: np.ndarray        # int64 [nnzb]
    S_val: np.ndarray          # float64
    H0_val: np.ndarray         # float64
    n_occ: int
    mo_group: np.ndarray       # int32 [n_mo]
    c0_colptr: np.ndarray      # int64 [n_mo + 1]
    c0_row: np.ndarray         # int32 [nnz]
    c0_val: np.ndarray         # float64 [nnz]
    info: Dict[str, float] = dataclasses.field(default_factory=dict)

    @property
    def n_ao(self) -> int:
        return int(self.atom_nao.sum())

    @property
    def n_mo(self) -> int:
        return int(self.c0_colptr.shape[0] - 1)

    @property
    def n_el(self) -> float:
        return float(self.q0.sum())

    def ao_offset(self) -> np.ndarray:
        off = np.zeros(self.n_atoms + 1, dtype=np.int64)
        np.cumsum(self.atom_nao, out=off[1:])
        return off

    def dense(self, which: str) -> np.ndarray:
        """Dense AO matrix ('S' or 'H0'); for small systems and tests only."""
        vals = self.S_val if which == "S" else self.H0_val
        n = self.n_ao
        out = np.zeros((n, n))
        aoo = self.ao_offset()
        for a in range(self.n_atoms):
            for k in range(self.blk_rowptr[a], self.blk_rowptr[a + 1]):
                b = self.blk_col[k]
                na, nb = self.atom_nao[a], self.atom_nao[b]
                blk = vals[self.blk_off[k]:self.blk_off[k] + na * nb].reshape(na, nb)
                out[aoo[a]:aoo[a] + na, aoo[b]:aoo[b] + nb] = blk
        return out

    def dense_c0(self) -> np.ndarray:
        out = np.zeros((self.n_ao, self.n_mo))
        for j in range(self.n_mo):
            sl = slice(self.c0_colptr[j], self.c0_colptr[j + 1])
            out[self.c0_row[sl], j] = self.c0_val[sl]
        return out


# --------------------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------------------

def _rsa_positions(rng: np.random.Generator, n: int, box: float, dmin: float,
                   max_attempts: int = 200_000_000) -> np.ndarray:
    """Random sequential addition of n points in [0, box)^3 with pairwise distance >= dmin."""
    cell = dmin / math.sqrt(3.0)          # at most one point per cell
    nc = max(1, int(math.floor(box / cell)))
    cell = box / nc
    reach = int(math.ceil(dmin / cell))
    grid = -np.ones((nc, nc, nc), dtype=np.int64)
    pts = np.empty((n, 3))
    count = 0
    attempts = 0
    d2min = dmin * dmin
    batch = 4096
    while count < n:
        cand = rng.random((batch, 3)) * box
        attempts += batch
        if attempts > max_attempts:
            raise RuntimeError(f"random sequential addition stalled at {count}/{n} points "
                               f"(box {box} A, dmin {dmin} A)")
        ci = np.minimum((cand / cell).astype(np.int64), nc - 1)
        for t in range(batch):
            x, y, z = ci[t]
            ok = True
            for ix in range(max(0, x - reach), min(nc, x + reach + 1)):
                for iy in range(max(0, y - reach), min(nc, y + reach + 1)):
                    sub = grid[ix, iy, max(0, z - reach):min(nc, z + reach + 1)]
                    for idx in sub[sub >= 0]:
                        dv = pts[idx] - cand[t]
                        if dv @ dv < d2min:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pts[count] = cand[t]
                grid[x, y, z] = count
                count += 1
                if count == n:
                    break
    return pts


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly random rotation matrices from unit quaternions (Shoemake)."""
    u1, u2, u3 = rng.random((3, n))
    q = np.stack([np.sqrt(1 - u1) * np.sin(2 * np.pi * u2),
                  np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
                  np.sqrt(u1) * np.sin(2 * np.pi * u3),
                  np.sqrt(u1) * np.cos(2 * np.pi * u3)], axis=1)
    x, y, z, w = q.T
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


MIN_INTER = 1.8             # Angstrom, any intermolecular O-H or H-H contact
N_ORIENT = 64               # orientation draws per accepted O position


def _water_local() -> np.ndarray:
    half = math.radians(HOH_ANGLE) / 2.0
    return np.array([[OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)],
                     [-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]])


def water_geometry(rng: np.random.Generator, n_mol: int, box: float,
                   max_attempts: int = 50_000_000):
    """Random sequential addition of rigid water molecules (Angstrom).

    O positions are uniform in [0, box)^3 with O-O >= 2.8 A.  For an O position
    that passes, up to N_ORIENT uniformly random orientations are drawn and the
    first one whose O-H and H-H contacts with every placed molecule are all
    >= MIN_INTER is kept; otherwise the position is rejected.
    Returns (xyz [3 n_mol, 3] as O, H, H per molecule, element codes).
    """
    local = _water_local()
    reach_r = MIN_OO + 2 * OH_BOND          # farthest O-O distance at which atoms can clash
    cell = MIN_OO / math.sqrt(3.0)
    nc = max(1, int(math.floor(box / cell)))
    cell = box / nc
    reach = int(math.ceil(reach_r / cell))
    grid = -np.ones((nc, nc, nc), dtype=np.int64)
    xyz = np.empty((n_mol, 3, 3))
    count = 0
    attempts = 0

    while count < n_mol:
        cand = rng.random((1024, 3)) * box
        attempts += 1024
        if attempts > max_attempts:
            raise RuntimeError(f"random sequential addition stalled at {count}/{n_mol} molecules "
                               f"(box {box} A)")
        ci = np.minimum((cand / cell).astype(np.int64), nc - 1)
        for t in range(cand.shape[0]):
            x, y, z = ci[t]
            sub = grid[max(0, x - reach):x + reach + 1, max(0, y - reach):y + reach + 1,
                       max(0, z - reach):z + reach + 1]
            nb = sub[sub >= 0]
            o = cand[t]
            if nb.size:
                d_oo = ((xyz[nb, 0] - o) ** 2).sum(-1)
                if (d_oo < MIN_OO * MIN_OO).any():
                    continue
                near = nb[d_oo < reach_r * reach_r]
            else:
                near = nb
            R = _random_rotations(rng, N_ORIENT)
            hpos = o[None, None, :] + np.einsum("nij,kj->nki", R, local)      # [N, 2, 3]
            if near.size:
                other = xyz[near].reshape(-1, 3)                                # [M, 3]
                mine = np.concatenate([np.broadcast_to(o, (N_ORIENT, 1, 3)), hpos], axis=1)
                d2 = ((mine[:, :, None, :] - other[None, None, :, :]) ** 2).sum(-1)
                d2[:, 0, 0::3] = np.inf           # O-O pairs are governed by MIN_OO
                ok = (d2 >= MIN_INTER * MIN_INTER).all(axis=(1, 2))
                if not ok.any():
                    continue
                k = int(np.argmax(ok))
            else:
                k = 0
            xyz[count, 0] = o
            xyz[count, 1:] = hpos[k]
            grid[x, y, z] = count
            count += 1
            if count == n_mol:
                break
    el = np.tile(np.array([EL_O, EL_H, EL_H], dtype=np.int32), n_mol)
    return xyz.reshape(-1, 3), el


# --------------------------------------------------------------------------------------
# constrained k-means (paper section 3.2), on molecule centres
# --------------------------------------------------------------------------------------

def _morton_key(p: np.ndarray, lo: np.ndarray, span: float, bits: int = 10) -> np.ndarray:
    q = np.clip(((p - lo) / max(span, 1e-12) * (2 ** bits - 1)).astype(np.int64), 0, 2 ** bits - 1)
    key = np.zeros(p.shape[0], dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            key |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return key


def initial_means(rng: np.random.Generator, centres: np.ndarray, m: int) -> np.ndarray:
    """m starting means spread evenly over the points' bounding box: a random pick of m
    cells of the smallest k x k x k grid with k^3 >= m (cell centres, ascending cell order)."""
    lo = centres.min(axis=0)
    hi = centres.max(axis=0)
    k = int(math.ceil(m ** (1.0 / 3.0) - 1e-9))
    g = (np.arange(k) + 0.5) / k
    grid = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pick = np.sort(rng.permutation(grid.shape[0])[:m])
    return lo + grid[pick] * (hi - lo)


def constrained_kmeans(rng: np.random.Generator, centres: np.ndarray, n_link: int,
                       max_iter: int = 100, tol: float = 1e-4):
    """Assign points to m = ceil(n / n_link) means, no mean holding more than n_link points.

    Means start on an even grid; each iteration draws a fresh order of the means
    (and of the points: the paper's parallel attribution visits atoms in no fixed
    order), links each point to its nearest mean that still has room, then moves
    every mean to the centroid of its points.  Stops when the mean displacement
    falls below tol (Angstrom) or after max_iter iterations.
    """
    n = centres.shape[0]
    m = max(1, -(-n // n_link))
    means = initial_means(rng, centres, m)
    assign = np.zeros(n, dtype=np.int64)
    for _ in range(max_iter):
        mean_perm = rng.permutation(m)          # shuffled list of means
        point_order = rng.permutation(n)
        d2 = ((centres[:, None, :] - means[None, mean_perm, :]) ** 2).sum(-1)
        ranked = np.argsort(d2, axis=1, kind="stable")
        fill = np.zeros(m, dtype=np.int64)
        for p in point_order:
            for r in ranked[p]:
                c = mean_perm[r]
                if fill[c] < n_link:
                    assign[p] = c
                    fill[c] += 1
                    break
        new = np.array([centres[assign == c].mean(axis=0) if (assign == c).any() else means[c]
                        for c in range(m)])
        disp = np.sqrt(((new - means) ** 2).sum(-1)).mean()
        means = new
        if disp < tol:
            break
    return assign, means


# --------------------------------------------------------------------------------------
# Slater-Koster two-centre blocks
# --------------------------------------------------------------------------------------

def _sk_block(el_a: int, el_b: int, d: np.ndarray, r: np.ndarray, kind: str) -> np.ndarray:
    """Blocks for many pairs of (el_a, el_b) atoms.  d: unit vectors a->b [P, 3], r in A.

    Returns [P, nao_a, nao_b].  kind 'H' -> (ss, sp, pp_sigma, pp_pi) = (-V, +V, +V, -V/2);
    kind 'S' -> (+s, -s, -s, +s/2), with V = 0.3 exp(-r/0.9), s = 0.2 exp(-r/0.9) (pairs with a
    carbon: V = 1.5 exp(-r/1.2), s = 0.3 exp(-r/1.2)).
    """
    v0, s0, r0 = (SK_C_V0, SK_C_SIGMA0, SK_C_R0) if EL_C in (el_a, el_b) else (SK_V0, SK_SIGMA0, SK_R0)
    e = np.exp(-r / r0) * (r < SK_CUTOFF)
    if kind == "H":
        v = v0 * e
        ss, sp, pps, ppp = -v, v, v, -0.5 * v
    else:
        s = s0 * e
        ss, sp, pps, ppp = s, -s, -s, 0.5 * s
    na, nb = NAO[el_a], NAO[el_b]
    P = r.shape[0]
    out = np.zeros((P, na, nb))
    out[:, 0, 0] = ss
    if nb == 4:
        out[:, 0, 1:] = d * sp[:, None]
    if na == 4:
        out[:, 1:, 0] = -d * sp[:, None]
    if na == 4 and nb == 4:
        out[:, 1:, 1:] = (d[:, :, None] * d[:, None, :] * (pps - ppp)[:, None, None]
                          + np.eye(3)[None] * ppp[:, None, None])
    return out


def _atom_pairs(xyz_ang: np.ndarray, cutoff: float):
    from scipy.spatial import cKDTree
    tree = cKDTree(xyz_ang)
    pairs = tree.query_pairs(cutoff, output_type="ndarray")
    if pairs.size == 0:
        pairs = np.zeros((0, 2), dtype=np.int64)
    return pairs


def build_matrices(xyz_ang: np.ndarray, el: np.ndarray):
    """Atom-block CSR pattern and S / H0 values on it."""
    n = xyz_ang.shape[0]
    nao = np.array([NAO[int(e)] for e in el], dtype=np.int32)
    pairs = _atom_pairs(xyz_ang, SK_CUTOFF)
    both = np.concatenate([pairs, pairs[:, ::-1]], axis=0) if pairs.size else pairs
    selfp = np.stack([np.arange(n), np.arange(n)], axis=1)
    allp = np.concatenate([selfp, both], axis=0)
    order = np.lexsort((allp[:, 1], allp[:, 0]))
    allp = allp[order]
    rows, cols = allp[:, 0], allp[:, 1]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    sizes = nao[rows].astype(np.int64) * nao[cols].astype(np.int64)
    off = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    S = np.zeros(off[-1])
    H = np.zeros(off[-1])
    # self blocks
    is_self = rows == cols
    for k in np.nonzero(is_self)[0]:
        a = rows[k]
        na = nao[a]
        S[off[k]:off[k] + na * na] = np.eye(na).ravel()
        es, ep = ONSITE[int(el[a])]
        diag = [es] + ([ep] * 3 if na == 4 else [])
        H[off[k]:off[k] + na * na] = np.diag(diag).ravel()
    # two-centre blocks, vectorised per element pair
    off_idx = np.nonzero(~is_self)[0]
    dv = xyz_ang[cols[off_idx]] - xyz_ang[rows[off_idx]]
    r = np.sqrt((dv * dv).sum(1))
    d = dv / r[:, None]
    ea, eb = el[rows[off_idx]], el[cols[off_idx]]
    for A in (EL_O, EL_H, EL_C):
        for B in (EL_O, EL_H, EL_C):
            sel = np.nonzero((ea == A) & (eb == B))[0]
            if sel.size == 0:
                continue
            ks = off_idx[sel]
            sz = NAO[A] * NAO[B]
            idx = off[ks][:, None] + np.arange(sz)[None, :]
            S[idx] = _sk_block(A, B, d[sel], r[sel], "S").reshape(-1, sz)
            H[idx] = _sk_block(A, B, d[sel], r[sel], "H").reshape(-1, sz)
    return nao, rowptr, cols.astype(np.int32), off[:-1].copy(), S, H


# --------------------------------------------------------------------------------------
# per-molecule guess (paper section 3.3)
# --------------------------------------------------------------------------------------

def molecular_guess(Hm: np.ndarray, Sm: np.ndarray, n_occ_m: int):
    """Lowest-first solutions of Hm c = lambda Sm c; the largest |c| entry is made positive."""
    w, V = eigh(Hm, Sm)
    for j in range(V.shape[1]):
        k = int(np.argmax(np.abs(V[:, j])))
        if V[k, j] < 0:
            V[:, j] = -V[:, j]
    return w, V[:, :n_occ_m], V[:, n_occ_m:]


def cholesky_local(M: np.ndarray, rank: int, tol: float = 1e-12):
    """Pivoted Cholesky factor of a positive semi-definite matrix of the given rank: M = L L^T
    with L's columns in pivot order, and the pivot (row) of each column.  For the density of a
    gapped system its columns are local (Cholesky MOs)."""
    from scipy.linalg.lapack import dpstrf
    A = np.array(M, dtype=np.float64, order="F", copy=True)
    L, piv, r, info = dpstrf(A, lower=1, tol=tol)
    if info < 0:
        raise RuntimeError(f"dpstrf failed ({info})")
    L = np.tril(L)
    r = min(int(r), rank)
    piv = piv - 1                                   # LAPACK pivots are 1-based
    out = np.zeros((M.shape[0], r))
    out[piv, :] = L[:, :r]
    return out, piv[:r]


def assemble(name, seed, box, xyz_ang, el, atom_mol, mol_group, n_groups, c0_drop=1e-13, mol_nocc=None,
             unit_group=None, atom_unit=None, log=None):
    """System from explicit geometry (Angstrom), molecule ids and MO group per molecule.

    The guess of section 3.3 is solved per molecule (atom_mol: contiguous runs of atoms), its
    doubly occupied count in mol_nocc (default: half the reference electrons of its atoms).
    With unit_group and atom_unit (a long molecule split into units, each in an MO group), the
    molecule's own occupied and virtual spaces are spanned by local MOs instead: the columns of
    pivoted Cholesky factors of C_occ C_occ^T and C_virt C_virt^T (Cholesky MOs: the density of
    a gapped molecule decays with distance, and so do they, away from their pivot AO).  Each
    goes to the group of the unit of its pivot.  They are not orthonormal (the library's first
    orthonormalization makes them so).  log: optional callable for progress lines."""
    n_atoms = xyz_ang.shape[0]
    nao, rowptr, col, off, S, H = build_matrices(xyz_ang, el)
    aoo = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(nao, out=aoo[1:])
    n_mol = int(atom_mol.max()) + 1
    # molecule -> atoms (contiguous by construction)
    mol_first = np.searchsorted(atom_mol, np.arange(n_mol))
    mol_last = np.searchsorted(atom_mol, np.arange(n_mol), side="right")
    q0 = np.array([Q0[int(e)] for e in el])
    occ_cols: List[List] = [[] for _ in range(n_groups)]
    virt_cols: List[List] = [[] for _ in range(n_groups)]
    for m in range(n_mol):
        a0, a1 = mol_first[m], mol_last[m]
        lo, hi = aoo[a0], aoo[a1]
        nm = hi - lo
        Hm = np.zeros((nm, nm))
        Sm = np.zeros((nm, nm))
        for a in range(a0, a1):
            for k in range(rowptr[a], rowptr[a + 1]):
                b = col[k]
                if b < a0 or b >= a1:
                    continue
                na, nb = nao[a], nao[b]
                blkS = S[off[k]:off[k] + na * nb].reshape(na, nb)
                blkH = H[off[k]:off[k] + na * nb].reshape(na, nb)
                Sm[aoo[a] - lo:aoo[a] - lo + na, aoo[b] - lo:aoo[b] - lo + nb] = blkS
                Hm[aoo[a] - lo:aoo[a] - lo + na, aoo[b] - lo:aoo[b] - lo + nb] = blkH
        n_el_m = q0[a0:a1].sum()
        n_occ_m = int(round(n_el_m)) // 2 if mol_nocc is None else int(mol_nocc[m])
        _, Vo, Vv = molecular_guess(Hm, Sm, n_occ_m)
        rows = np.arange(lo, hi, dtype=np.int32)
        if unit_group is None:
            g = mol_group[m]
            for j in range(Vo.shape[1]):
                occ_cols[g].append((rows, Vo[:, j]))
            for j in range(Vv.shape[1]):
                virt_cols[g].append((rows, Vv[:, j]))
        else:
            # local MOs: Cholesky factors of the molecule's occupied and virtual projectors, in
            # the order of their pivots along the molecule
            ao_unit = np.repeat(atom_unit[a0:a1], nao[a0:a1])
            for V, dest in ((Vo, occ_cols), (Vv, virt_cols)):
                L, piv = cholesky_local(V @ V.T, V.shape[1])
                if L.shape[1] != V.shape[1]:
                    raise RuntimeError("local guess: the Cholesky factor lost rank")
                L = L / np.sqrt(np.einsum("ij,ij->j", L, Sm @ L))            # S-normalized
                L = L * np.sign(L[np.argmax(np.abs(L), axis=0), np.arange(L.shape[1])])
                for j in np.argsort(piv, kind="stable"):      # along the molecule
                    dest[unit_group[ao_unit[piv[j]]]].append((rows, L[:, j]))
        if log is not None and (m + 1) % 100 == 0:
            log(f"[synth] {name}: guess of {m + 1} of {n_mol} molecules")
    cols, groups = [], []
    for g in range(n_groups):
        cols += occ_cols[g]
        groups += [g] * len(occ_cols[g])
    n_occ = len(cols)
    for g in range(n_groups):
        cols += virt_cols[g]
        groups += [g] * len(virt_cols[g])
    colptr = np.zeros(len(cols) + 1, dtype=np.int64)
    rr, vv = [], []
    for j, (rows, v) in enumerate(cols):
        keep = np.abs(v) >= c0_drop
        rr.append(rows[keep])
        vv.append(v[keep])
        colptr[j + 1] = colptr[j] + int(keep.sum())
    atom_group = (mol_group[atom_mol] if unit_group is None else unit_group[atom_unit]).astype(np.int32)
    sysm = System(
        name=name, seed=seed, box_angstrom=box, n_atoms=n_atoms,
        atom_el=el.astype(np.int32), atom_nao=nao.astype(np.int32),
        xyz_bohr=np.ascontiguousarray(xyz_ang * BOHR_PER_ANGSTROM),
        hubbard_u=np.array([HUBBARD_U[int(e)] for e in el]), q0=q0,
        atom_mol=atom_mol.astype(np.int32), atom_group=atom_group, n_groups=n_groups,
        blk_rowptr=rowptr, blk_col=col, blk_off=off, S_val=S, H0_val=H,
        n_occ=n_occ, mo_group=np.array(groups, dtype=np.int32),
        c0_colptr=colptr, c0_row=np.concatenate(rr).astype(np.int32),
        c0_val=np.concatenate(vv))
    return sysm


def water_box(n_mol: int, box: float, seed: int, n_link: int = N_LINK, name: str = "") -> System:
    """A seeded open water-like box: n_mol molecules in a cube of side `box` Angstrom.

    Atoms are ordered group by group (constrained k-means on O positions), molecules
    inside a group along a Morton curve, each molecule as O, H, H.
    """
    rng = np.random.default_rng(seed)
    xyz, el = water_geometry(rng, n_mol, box)
    opos = xyz[0::3]
    assign, means = constrained_kmeans(rng, opos, n_link)
    n_groups = int(assign.max()) + 1
    lo = opos.min(axis=0)
    span = float((opos.max(axis=0) - lo).max())
    gkey = _morton_key(means, lo, span)
    gorder = np.argsort(gkey, kind="stable")
    grank = np.empty(n_groups, dtype=np.int64)
    grank[gorder] = np.arange(n_groups)
    mkey = _morton_key(opos, lo, span)
    mol_order = np.lexsort((mkey, grank[assign]))
    mol_group = grank[assign][mol_order]
    atom_idx = (3 * mol_order[:, None] + np.arange(3)[None, :]).ravel()
    xyz = xyz[atom_idx]
    el = el[atom_idx]
    atom_mol = np.repeat(np.arange(n_mol), 3)
    sysm = assemble(name or f"water{n_mol}", seed, box, xyz, el, atom_mol, mol_group, n_groups)
    d = np.sqrt(((opos[:, None, :] - opos[None, :, :]) ** 2).sum(-1)) if n_mol <= 2048 else None
    if d is not None and n_mol > 1:
        np.fill_diagonal(d, np.inf)
        sysm.info["min_OO_angstrom"] = float(d.min())
    return sysm


CONFIGS = {
    # small case: 128 molecules, 16 A cube
    "water128": dict(n_mol=128, box=16.0),
    # headline case: 4096 molecules (12,288 atoms, 24,576 AOs), 50 A cube
    "water4096": dict(n_mol=4096, box=50.0),
    # differentiation case: 512 molecules, 25 A cube
    "water512": dict(n_mol=512, box=25.0),
    # alkane-like chains at about the headline size: 400 octanes (10,400 atoms, 20,000 AOs),
    # 60 A cube (about half the liquid density), groups of two chains
    "octane400": dict(n_chains=400, n_c=8, box=60.0),
    # the large alkane form: 400 chains of C83H168 (100,400 atoms, 200,000 AOs), 160 A cube
    # (half the octane400 density: the coils are long), local guess from each chain's own
    # solution, MO groups of 10 carbons along a chain.  Without the charge term: the plain SCC iteration (no mixing)
    # grows a charge oscillation on these long chains; the library options are in RUN_OPTIONS
    "alkane400x83": dict(n_chains=400, n_c=83, box=160.0, seg=10),
}


# library options a workload needs besides its system (scc: the DFTB charge term; slot_margin_bohr:
# storage only for the row blocks within that distance beyond the reach of each MO group's
# initial MOs; on a 60-chain box of the same chains the MOs grew at most 46 bohr past it)
RUN_OPTIONS = {"alkane400x83": dict(scc=False, slot_margin_bohr=90.0)}


def make_config(name: str, seed: int = 1, log=None) -> System:
    """A named workload; log: optional callable for progress lines of long generations."""
    c = CONFIGS[name]
    if "seg" in c:
        return alkane_segments_box(c["n_chains"], c["n_c"], c["box"], seed, seg=c["seg"], name=name, log=log)
    if "n_chains" in c:
        return alkane_box(c["n_chains"], c["n_c"], c["box"], seed, name=name)
    return water_box(c["n_mol"], c["box"], seed, name=name)


_CACHE: Dict = {}


def cached(name: str, seed: int = 1) -> System:
    key = (name, seed)
    if key not in _CACHE:
        _CACHE[key] = make_config(name, seed)
    return _CACHE[key]


def water_molecules(o_pos_angstrom: np.ndarray, seed: int, mol_group=None, name: str = "waters") -> System:
    """Waters at given O positions with seeded random orientations (no packing rules)."""
    rng = np.random.default_rng(seed)
    o = np.asarray(o_pos_angstrom, dtype=np.float64)
    n = o.shape[0]
    R = _random_rotations(rng, n)
    h = o[:, None, :] + np.einsum("nij,kj->nki", R, _water_local())
    xyz = np.concatenate([o[:, None, :], h], axis=1).reshape(-1, 3)
    el = np.tile(np.array([EL_O, EL_H, EL_H], dtype=np.int32), n)
    mg = np.zeros(n, dtype=np.int64) if mol_group is None else np.asarray(mol_group, dtype=np.int64)
    return assemble(name, seed, float(np.ptp(o)) if n > 1 else 0.0, xyz, el, np.repeat(np.arange(n), 3),
                    mg, int(mg.max()) + 1)


# --------------------------------------------------------------------------------------
# alkane-like chains: non-water molecules (carbon s+p, hydrogen s) and groups of chains
# --------------------------------------------------------------------------------------

CC_BOND, CH_BOND = 1.54, 1.09          # Angstrom
CCC_ANGLE = np.deg2rad(112.0)
TETRA = np.deg2rad(109.47)


def _place(a, b, c, bond, angle, torsion):
    """Atom d with |cd| = bond, angle(b, c, d) = angle, dihedral(a, b, c, d) = torsion."""
    bc = c - b
    bc /= np.linalg.norm(bc)
    n = np.cross(b - a, bc)
    n /= np.linalg.norm(n)
    m = np.cross(n, bc)
    d2 = np.array([-bond * np.cos(angle), bond * np.sin(angle) * np.cos(torsion), bond * np.sin(angle) * np.sin(torsion)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * n


def alkane_chain(rng: np.random.Generator, n_c: int):
    """One C_nH_(2n+2) chain in local coordinates, atoms ordered C, its H's, next C, ...:
    a carbon backbone with C-C 1.54 A and C-C-C 112 degrees, torsions trans (180) or gauche
    (+-65) drawn with probabilities 0.7 / 0.15 / 0.15 plus +-10 degrees of seeded noise, and
    tetrahedral hydrogens at 1.09 A (three on each end carbon, two on the others)."""
    c = [np.zeros(3), np.array([CC_BOND, 0.0, 0.0])]
    if n_c >= 3:
        c.append(c[1] + CC_BOND * np.array([-np.cos(CCC_ANGLE), np.sin(CCC_ANGLE), 0.0]))
    for i in range(3, n_c):
        u = rng.random()
        tor = np.pi if u < 0.7 else (np.deg2rad(65.0) if u < 0.85 else -np.deg2rad(65.0))
        tor += np.deg2rad(10.0) * (2.0 * rng.random() - 1.0)
        c.append(_place(c[i - 3], c[i - 2], c[i - 1], CC_BOND, CCC_ANGLE, tor))
    c = c[:n_c]
    xyz, el = [], []
    for i in range(n_c):
        xyz.append(c[i])
        el.append(EL_C)
        if n_c == 1:
            nb = []
        else:
            nb = [c[j] for j in (i - 1, i + 1) if 0 <= j < n_c]
        if len(nb) == 2:                       # CH2: the two H in the plane bisecting C-C-C
            u = (c[i] - nb[0]) / np.linalg.norm(c[i] - nb[0]) + (c[i] - nb[1]) / np.linalg.norm(c[i] - nb[1])
            u /= np.linalg.norm(u)
            v = np.cross(nb[0] - c[i], nb[1] - c[i])
            v /= np.linalg.norm(v)
            for sgn in (1.0, -1.0):
                xyz.append(c[i] + CH_BOND * (np.cos(TETRA / 2) * u + sgn * np.sin(TETRA / 2) * v))
                el.append(EL_H)
        else:                                  # CH3 end: three H around the C-C axis
            other = nb[0]
            if n_c > 2:
                ref = c[2] if i == 0 else c[i - 2]
            else:
                ref = other + np.array([0.0, 1.0, 0.0])
            for k in range(3):
                xyz.append(_place(ref, other, c[i], CH_BOND, TETRA, np.pi + k * 2.0 * np.pi / 3.0))
                el.append(EL_H)
    return np.array(xyz), np.array(el, dtype=np.int32)


def alkane_box(n_chains: int, n_c: int, box: float, seed: int, n_link: int = 2, name: str = "") -> System:
    """A seeded open box of n_chains C_nH_(2n+2) chains (each its own molecule and guess fragment),
    placed with uniformly random centres and orientations and no two atoms of different chains
    closer than 2.2 A; MO groups of n_link chains from the constrained k-means on chain centres."""
    rng = np.random.default_rng(seed)
    xyz_all, el_all, centres = [], [], []
    for _ in range(n_chains):
        local, el = alkane_chain(rng, n_c)
        local = local - local.mean(axis=0)
        for attempt in range(2000):
            R = _random_rotations(rng, 1)[0]
            pos = rng.uniform(0.0, box, 3)
            cand = local @ R.T + pos
            if all(np.min(((cand[:, None, :] - x[None, :, :]) ** 2).sum(-1)) >= 2.2 ** 2 for x in xyz_all):
                break
        else:
            raise RuntimeError(f"alkane_box: no room for chain {len(xyz_all)} (seed {seed})")
        xyz_all.append(cand)
        el_all.append(el)
        centres.append(pos)
    centres = np.array(centres)
    assign, means = constrained_kmeans(rng, centres, n_link)
    used = np.unique(assign)
    ren = np.full(assign.max() + 1, -1)
    ren[used] = np.arange(used.size)
    order = np.lexsort((np.arange(n_chains), ren[assign]))
    per = len(el_all[0])
    xyz = np.concatenate([xyz_all[i] for i in order])
    el = np.concatenate([el_all[i] for i in order])
    atom_mol = np.repeat(np.arange(n_chains), per)
    return assemble(name or f"alkane{n_chains}x{n_c}", seed, box, xyz, el, atom_mol, ren[assign[order]], used.size)


def alkane_segments_box(n_chains: int, n_c: int, box: float, seed: int, seg: int = 10, name: str = "",
                        log=None) -> System:
    """A seeded open box of long C_nH_(2n+2) chains with local MOs from the start.

    Chains: seeded conformations (alkane_chain) with random centres in [0, box)^3 and random
    orientations, no two atoms of different chains closer than 2.2 A; chains follow a Morton
    order of their centres.  A chain is one molecule of the guess of section 3.3, but its
    solution spreads over the whole chain, so it is made local before it enters C (see
    assemble): the units are a carbon and its hydrogens, and each local MO goes to the group of
    its pivot's unit.  The SCF starts from the chain's own solution, in a local basis.  MO groups
    (section 3.2) are runs of `seg` consecutive units along a chain, spatially compact as the
    constrained k-means would make them."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    placed, recent, chains, centres = [], [], [], []
    tree = None
    for ci in range(n_chains):
        local, el = alkane_chain(rng, n_c)
        local = local - local.mean(axis=0)
        for attempt in range(20000):
            R = _random_rotations(rng, 1)[0]
            pos = rng.uniform(0.0, box, 3)
            cand = local @ R.T + pos
            ok = True
            if tree is not None:
                d, _ = tree.query(cand, k=1, distance_upper_bound=2.2)
                ok = not np.isfinite(d).any()
            if ok:
                for x in recent:
                    if np.min(((cand[:, None, :] - x[None, :, :]) ** 2).sum(-1)) < 2.2 ** 2:
                        ok = False
                        break
            if ok:
                break
        else:
            raise RuntimeError(f"alkane_segments_box: no room for chain {ci} (seed {seed})")
        chains.append((cand, el))
        centres.append(pos)
        recent.append(cand)
        if len(recent) >= 16:
            placed.extend(recent)
            recent = []
            tree = cKDTree(np.concatenate(placed))
        if log is not None and (ci + 1) % 100 == 0:
            log(f"[synth] {name}: placed {ci + 1} of {n_chains} chains")
    centres = np.array(centres)
    lo = centres.min(axis=0)
    span = float((centres.max(axis=0) - lo).max())
    order = np.argsort(_morton_key(centres, lo, span), kind="stable")
    xyz, els, atom_mol, atom_unit, unit_group = [], [], [], [], []
    n_unit = n_grp = 0
    for m, c in enumerate(order):
        cx, cel = chains[c]
        cpos = np.flatnonzero(cel == EL_C)
        for u, a0 in enumerate(cpos):
            a1 = cpos[u + 1] if u + 1 < len(cpos) else len(cel)
            atom_unit += [n_unit] * (a1 - a0)
            unit_group.append(n_grp + u // seg)
            n_unit += 1
        xyz.append(cx)
        els.append(cel)
        atom_mol += [m] * len(cel)
        n_grp += -(-len(cpos) // seg)
    # coefficients below 1e-5 (the rotation threshold eps of section 3.5) are left out: the guess
    # only starts the iteration, and the slowly decaying tails of the Cholesky MOs along a chain
    # would otherwise reach tens of Angstrom from their group
    return assemble(name or f"alkanes{n_chains}x{n_c}", seed, box, np.concatenate(xyz), np.concatenate(els),
                    np.array(atom_mol), np.zeros(n_chains, dtype=np.int64), n_grp, c0_drop=1e-5,
                    unit_group=np.array(unit_group), atom_unit=np.array(atom_unit), log=log)
