"""Pins of the oracle's atom neighbour map (section 3.2).

* random points: the same pairs as scipy's k-d tree (pairs within the radius) plus the self
  pairs (no pair sits on the boundary for such inputs);
* the water boxes: the atom-block pattern the input generator builds its S and H on;
* the unit cubic lattice: closed-form counts (1 + 6 + 12 neighbours of an interior site for a
  cut-off between sqrt(2) and sqrt(3); only the site itself for a cut-off of exactly 1, the
  test being strict);
* symmetry of the map and ascending columns.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle.neighbours import atom_neighbours
from paper_1402_2880_amd import synth


def kdtree_map(x, r):
    n = x.shape[0]
    pairs = cKDTree(x).query_pairs(r, output_type="ndarray")
    allp = np.concatenate([np.stack([np.arange(n), np.arange(n)], 1), pairs, pairs[:, ::-1]])
    allp = allp[np.lexsort((allp[:, 1], allp[:, 0]))]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, allp[:, 0] + 1, 1)
    return np.cumsum(rowptr), allp[:, 1]


@pytest.mark.parametrize("seed,n,box,r", [(0, 300, 10.0, 2.5), (1, 1000, 20.0, 3.0), (2, 5, 1.0, 10.0)])
def test_matches_kdtree(seed, n, box, r):
    x = np.random.default_rng(seed).uniform(0, box, (n, 3))
    rp, col = atom_neighbours(x, r)
    krp, kcol = kdtree_map(x, r)
    assert np.array_equal(rp, krp) and np.array_equal(col, kcol)


def test_matches_generator_pattern():
    for n_mol, box, seed in [(64, 13.0, 3), (128, 16.0, 1)]:
        s = synth.water_box(n_mol, box, seed)
        rp, col = atom_neighbours(s.xyz_bohr, synth.SK_CUTOFF * synth.BOHR_PER_ANGSTROM)
        assert np.array_equal(rp, s.blk_rowptr) and np.array_equal(col, s.blk_col)


def test_unit_lattice_counts():
    ax = np.arange(5, dtype=float)
    x = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    centre = 2 * 25 + 2 * 5 + 2
    rp, col = atom_neighbours(x, 1.5)
    assert rp[centre + 1] - rp[centre] == 19
    corner = 0
    assert rp[corner + 1] - rp[corner] == 1 + 3 + 3
    rp1, col1 = atom_neighbours(x, 1.0)
    assert np.array_equal(np.diff(rp1), np.ones(125)) and np.array_equal(col1, np.arange(125))


def test_symmetric_and_sorted():
    x = np.random.default_rng(4).uniform(0, 8, (400, 3))
    rp, col = atom_neighbours(x, 2.0)
    rows = np.repeat(np.arange(400), np.diff(rp))
    pairs = set(zip(rows.tolist(), col.tolist()))
    assert all((b, a) in pairs for a, b in pairs)
    assert all(np.all(np.diff(col[rp[a]:rp[a + 1]]) > 0) for a in range(400))
