"""The seeded input generator: determinism, geometry rules, matrix properties."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1402_2880_amd import synth


def test_deterministic_per_seed():
    a = synth.water_box(24, 10.0, 7)
    b = synth.water_box(24, 10.0, 7)
    c = synth.water_box(24, 10.0, 8)
    assert np.array_equal(a.xyz_bohr, b.xyz_bohr)
    assert np.array_equal(a.S_val, b.S_val) and np.array_equal(a.c0_val, b.c0_val)
    assert not np.array_equal(a.xyz_bohr, c.xyz_bohr)


def test_geometry_rules(water128):
    s = water128
    x = s.xyz_bohr / synth.BOHR_PER_ANGSTROM
    o = x[0::3]
    assert o.min() >= 0.0 and o.max() < 16.0
    d = np.sqrt(((o[:, None] - o[None]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    assert d.min() >= synth.MIN_OO - 1e-12
    for m in range(s.n_atoms // 3):
        oh = np.linalg.norm(x[3 * m + 1:3 * m + 3] - x[3 * m], axis=1)
        assert np.allclose(oh, synth.OH_BOND, atol=1e-12)
        v1, v2 = x[3 * m + 1] - x[3 * m], x[3 * m + 2] - x[3 * m]
        ang = np.degrees(np.arccos(v1 @ v2 / (np.linalg.norm(v1) * np.linalg.norm(v2))))
        assert abs(ang - synth.HOH_ANGLE) < 1e-9
    pairs = cKDTree(x).query_pairs(2.5, output_type="ndarray")
    inter = pairs[s.atom_mol[pairs[:, 0]] != s.atom_mol[pairs[:, 1]]]
    dd = np.linalg.norm(x[inter[:, 0]] - x[inter[:, 1]], axis=1)
    assert dd.min() >= synth.MIN_INTER - 1e-12


def test_matrices(water128):
    s = water128
    S, H0 = s.dense("S"), s.dense("H0")
    assert np.array_equal(S, S.T) and np.array_equal(H0, H0.T)
    assert np.linalg.eigvalsh(S).min() > 0.5
    # pattern: sorted columns, self block first-class, 6 A cutoff
    for a in range(s.n_atoms):
        cols = s.blk_col[s.blk_rowptr[a]:s.blk_rowptr[a + 1]]
        assert np.all(np.diff(cols) > 0) and a in cols
    x = s.xyz_bohr / synth.BOHR_PER_ANGSTROM
    nb = cKDTree(x).query_pairs(synth.SK_CUTOFF, output_type="ndarray")
    assert len(s.blk_col) == s.n_atoms + 2 * len(nb)
    # one closed form: O s - H s overlap of the bonded pair = 0.2 exp(-0.96/0.9)
    aoo = s.ao_offset()
    assert abs(S[aoo[0], aoo[1]] - 0.2 * np.exp(-0.96 / 0.9)) < 1e-15
    assert abs(H0[aoo[0], aoo[1]] + 0.3 * np.exp(-0.96 / 0.9)) < 1e-15


def test_groups_and_guess(water128):
    s = water128
    assert s.n_groups == 128 // synth.N_LINK
    assert np.all(np.bincount(s.atom_group) == 3 * synth.N_LINK)
    assert np.all(np.diff(s.atom_group) >= 0)          # atoms ordered group by group
    assert s.n_occ == 4 * 128 and s.n_mo == 6 * 128
    assert np.all(np.diff(s.mo_group[:s.n_occ]) >= 0) and np.all(np.diff(s.mo_group[s.n_occ:]) >= 0)
    S = s.dense("S")
    C0 = s.dense_c0()
    O = C0.T @ S @ C0
    # MOs of one molecule are S-orthonormal; every MO lives on one molecule
    mol_of_ao = np.repeat(s.atom_mol, s.atom_nao)
    for j in range(s.n_mo):
        rows = s.c0_row[s.c0_colptr[j]:s.c0_colptr[j + 1]]
        assert len(set(mol_of_ao[rows])) == 1
    same = mol_of_ao[np.argmax(np.abs(C0), axis=0)]
    mask = same[:, None] == same[None, :]
    assert np.abs(O[mask] - np.eye(s.n_mo)[mask]).max() < 1e-12
