"""The alkane chain generator (input side of the large alkane form): formula, bond lengths,
tetrahedral hydrogens, sp3 coordination, packing of a box and seeding."""
import numpy as np
import pytest

from paper_1402_2880_amd import synth


@pytest.mark.parametrize("n_c", [2, 3, 8, 20])
def test_chain_geometry(n_c):
    x, el = synth.alkane_chain(np.random.default_rng(n_c), n_c)
    C, H = x[el == synth.EL_C], x[el == synth.EL_H]
    assert len(C) == n_c and len(H) == 2 * n_c + 2                       # C_n H_(2n+2)
    d = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    dcc = np.sqrt(((C[1:] - C[:-1]) ** 2).sum(-1))
    assert np.allclose(dcc, synth.CC_BOND, atol=1e-12)
    dch = np.sqrt(((H[:, None] - C[None]) ** 2).sum(-1))
    assert np.allclose(dch.min(axis=1), synth.CH_BOND, atol=1e-12)     # every H on one carbon
    assert ((dch < 1.2).sum(axis=1) == 1).all()
    ci = np.flatnonzero(el == synth.EL_C)
    assert ((d[ci] < 1.6).sum(axis=1) == 4).all()                        # sp3: four bonded neighbours
    hh = np.sqrt(((H[:, None] - H[None]) ** 2).sum(-1))[np.triu_indices(len(H), 1)]
    assert hh.min() > 1.7                                                 # tetrahedral H-C-H: 1.78 A
    # bond angles at every carbon close to tetrahedral (109.5) or the backbone's 112
    for i in ci:
        nb = np.flatnonzero(d[i] < 1.6)
        for a in range(len(nb)):
            for b in range(a + 1, len(nb)):
                u, v = x[nb[a]] - x[i], x[nb[b]] - x[i]
                ang = np.degrees(np.arccos(u @ v / np.linalg.norm(u) / np.linalg.norm(v)))
                assert 100.0 < ang < 120.0, ang


def test_box_packing_and_seed():
    s1 = synth.alkane_box(12, 6, 18.0, 3)
    s2 = synth.alkane_box(12, 6, 18.0, 3)
    assert np.array_equal(s1.xyz_bohr, s2.xyz_bohr) and np.array_equal(s1.mo_group, s2.mo_group)
    x = s1.xyz_bohr / synth.BOHR_PER_ANGSTROM
    mol = s1.atom_mol
    d = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
    other = mol[:, None] != mol[None, :]
    assert d[other].min() >= 2.2 - 1e-9
    assert s1.n_occ == 12 * (4 * 6 + 2 * 6 + 2) // 2                  # 19 doubly occupied MOs per C6H14
    assert np.bincount(s1.mo_group).max() <= 2 * (4 * 6 + 2 * 6 + 2)   # at most two chains per group


def test_alkane_box_dense_limit_and_config_eps():
    """Octane chains (carbon s+p, hydrogen s, groups of two chains): the oracle reaches the dense
    SCC-DFTB energy in the dense limit, and stays within 1e-5 Ha of it at eps = 1e-5."""
    from oracle.oracle import Oracle
    from tests.dense_ref import dense_scf
    s = synth.alkane_box(4, 8, 12.0, 2)
    ref = dense_scf(s)
    assert ref["converged"] and ref["gap"] > 0.3
    for kw, tol in [(dict(eps=1e-12, e_conv=1e-13, r_nbr_bohr=1e6, max_sweeps_step=50), 1e-9), ({}, 1e-5)]:
        o = Oracle(s, **kw)
        for _ in range(80):
            if o.step()["converged"]:
                break
        assert abs(o.energy() - ref["energy"]) < tol, (kw, o.energy() - ref["energy"])
