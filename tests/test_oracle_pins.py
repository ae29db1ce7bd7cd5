"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: the references are dense
generalized diagonalization (tests/dense_ref.py), closed forms, invariants that
follow from the definitions, brute force, and the paper's accuracy claim.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, jacobi_angle
from paper_1402_2880_amd import synth
from tests.dense_ref import dense_scf, gamma_matrix

TIGHT = dict(eps=1e-11, e_conv=1e-12, max_sweeps_step=50)


def run_to_convergence(o, max_steps=200):
    info = None
    for _ in range(max_steps):
        info = o.step()
        if info["converged"]:
            return info
    raise AssertionError("oracle SCF did not converge")


def pattern_values(system, P):
    """Values of a dense AO matrix on the atom-block pattern (same layout as S_val)."""
    aoo = system.ao_offset()
    out = np.zeros_like(system.S_val)
    for a in range(system.n_atoms):
        for k in range(system.blk_rowptr[a], system.blk_rowptr[a + 1]):
            b = system.blk_col[k]
            na, nb = system.atom_nao[a], system.atom_nao[b]
            out[system.blk_off[k]:system.blk_off[k] + na * nb] = \
                P[aoo[a]:aoo[a] + na, aoo[b]:aoo[b] + nb].ravel()
    return out


# ---------------------------------------------------------------------------------------
# P3: closed forms of the 2x2 rotation (section 3.5)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("fii,faa,fia", [(-0.5, 0.1, 0.03), (-0.5, 0.1, -0.03), (0.2, -0.4, 0.07),
                                         (0.1, 0.1, 0.02), (0.1, 0.1, -0.02), (-0.3, 0.2, 1e-9)])
def test_jacobi_rotation_annihilates(fii, faa, fia):
    c, s = jacobi_angle(fii, faa, fia)
    F = np.array([[fii, fia], [fia, faa]])
    R = np.array([[c, -s], [s, c]])          # columns: new i = c i + s a, new a = -s i + c a
    Fp = R.T @ F @ R
    assert abs(c * c + s * s - 1.0) < 1e-15
    assert abs(Fp[0, 1]) < 1e-15 * max(1.0, abs(fii), abs(faa))
    t = s / c
    assert abs(t) <= 1.0 + 1e-15                       # the smaller root
    assert abs(Fp[0, 0] - (fii + t * fia)) < 1e-14
    assert abs(Fp[1, 1] - (faa - t * fia)) < 1e-14
    if fii == faa:                                       # sgn(0) = +1: 45 degrees, t = 1
        assert abs(t - 1.0) < 1e-15


def test_printed_second_rotation_line_is_not_a_rotation():
    """The printed C'_j = -s C_j + c C_i does not annihilate F_ij; the corrected one does."""
    fii, faa, fia = -0.5, 0.1, 0.03
    c, s = jacobi_angle(fii, faa, fia)
    F = np.array([[fii, fia], [fia, faa]])
    printed = np.array([[c, c], [s, -s]])
    Fp = printed.T @ F @ printed
    assert abs(Fp[0, 1]) > 1e-3


# ---------------------------------------------------------------------------------------
# P1: the dense limit (section 4.1: epsilon -> 0 recovers the exact result)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("n_mol,box,n_link", [(1, 5.0, 16), (2, 6.0, 1), (4, 7.0, 2), (8, 8.0, 2)])
def test_dense_limit_small(n_mol, box, n_link):
    s = synth.water_box(n_mol, box, 3, n_link=n_link)
    ref = dense_scf(s, tol=1e-13)
    assert ref["converged"]
    o = Oracle(s, r_nbr_bohr=1e6, **TIGHT)
    run_to_convergence(o)
    assert abs(o.energy() - ref["energy"]) < 1e-9
    assert np.abs(o.charges() - ref["charges"]).max() < 1e-7
    assert np.abs(o.density() - pattern_values(s, ref["density"])).max() < 1e-7


@pytest.mark.slow
def test_dense_limit_water128(water128):
    s = water128
    ref = dense_scf(s, tol=1e-12)
    assert ref["converged"] and ref["gap"] > 0.1
    o = Oracle(s, r_nbr_bohr=1e6, **TIGHT)
    run_to_convergence(o)
    assert abs(o.energy() - ref["energy"]) < 1e-9
    assert np.abs(o.charges() - ref["charges"]).max() < 1e-7


# ---------------------------------------------------------------------------------------
# P2: textbook special cases
# ---------------------------------------------------------------------------------------

def test_non_scc_equals_twice_lowest_eigenvalues():
    from scipy.linalg import eigh
    s = synth.water_box(12, 9.0, 5, n_link=3)
    w = eigh(s.dense("H0"), s.dense("S"), eigvals_only=True)
    o = Oracle(s, scc=False, r_nbr_bohr=1e6, **TIGHT)
    run_to_convergence(o)
    assert abs(o.energy() - 2.0 * w[:s.n_occ].sum()) < 1e-9


def test_isolated_molecules_need_no_rotation():
    from scipy.linalg import eigh
    o_pos = np.array([[0.0, 0.0, 0.0], [25.0, 0.0, 0.0], [0.0, 25.0, 0.0], [25.0, 25.0, 25.0]])
    s = synth.water_molecules(o_pos, seed=2, mol_group=[0, 1, 2, 3])
    o = Oracle(s, scc=False, eps=1e-10, e_conv=1e-12)
    info = o.step()
    assert info["n_rotations"] == 0 and info["n_candidates"] == 0
    ref = 0.0
    S, H0 = s.dense("S"), s.dense("H0")
    for m in range(4):
        sl = slice(6 * m, 6 * m + 6)
        ref += 2.0 * eigh(H0[sl, sl], S[sl, sl], eigvals_only=True)[:4].sum()
    assert abs(o.energy() - ref) < 1e-12
    assert not o.group_nbr()[0, 1]                    # 25 A > 20 bohr


# ---------------------------------------------------------------------------------------
# Neighbour map and rotation schedule against brute force (sections 3.2, 3.5)
# ---------------------------------------------------------------------------------------

def test_group_neighbours_and_rounds(water128):
    s = water128
    o = Oracle(s)
    x = s.xyz_bohr
    d = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
    G = s.n_groups
    ref = np.zeros((G, G), dtype=bool)
    for g in range(G):
        for h in range(G):
            ref[g, h] = (d[np.ix_(s.atom_group == g, s.atom_group == h)] < 20.0).any()
    assert np.array_equal(o.group_nbr().astype(bool), ref)
    g_, h_, r_ = o.schedule()
    assert sorted(zip(g_.tolist(), h_.tolist())) == [(a, b) for a in range(G) for b in range(G) if ref[a, b]]
    for r in np.unique(r_):
        sel = r_ == r
        assert len(set(g_[sel])) == sel.sum() and len(set(h_[sel])) == sel.sum()


def test_schedule_conflict_free_on_sparse_neighbourhood():
    s = synth.water_box(96, 20.0, 4, n_link=4)
    o = Oracle(s)
    g_, h_, r_ = o.schedule()
    nbr = o.group_nbr()
    assert not nbr.all()                              # some groups are not neighbours
    assert np.all(nbr[g_, h_])
    for r in np.unique(r_):
        sel = r_ == r
        assert len(set(g_[sel])) == sel.sum() and len(set(h_[sel])) == sel.sum()
    # greedy colouring in (g, h) order: each block takes the smallest free round
    used_o, used_v = {}, {}
    for g, h, r in zip(g_, h_, r_):
        k = 0
        while k in used_o.get(g, set()) or k in used_v.get(h, set()):
            k += 1
        assert k == r
        used_o.setdefault(g, set()).add(r)
        used_v.setdefault(h, set()).add(r)


# ---------------------------------------------------------------------------------------
# P4: invariants after set-up and after every step, checked densely from the oracle's C
# ---------------------------------------------------------------------------------------

def test_invariants_along_scf(water128):
    s = water128
    eps = 1e-5
    o = Oracle(s, eps=eps)
    S, H0 = s.dense("S"), s.dense("H0")
    g = gamma_matrix(s)
    nbr = o.group_nbr().astype(bool)
    mask = nbr[np.ix_(s.mo_group, s.mo_group)]
    aoo = s.ao_offset()
    for step in range(4):
        C = o.mo_dense()
        O = C.T @ S @ C
        assert np.abs((O - np.eye(s.n_mo))[mask]).max() < eps / 100
        nz = np.abs(C[C != 0.0])
        assert nz.min() >= 0.999 * 1e-3 * eps          # orthonormalization cut-off
        Cocc = C[:, :s.n_occ]
        P = 2.0 * Cocc @ Cocc.T
        q = np.add.reduceat((P * S).sum(1), aoo[:-1])
        assert np.abs(o.charges() - q).max() < 1e-11
        assert abs(o.charges().sum() - s.n_el) < 1e-9
        dq = q - s.q0
        E = (P * H0).sum() + 0.5 * dq @ g @ dq
        assert abs(o.energy() - E) < 1e-9
        assert np.abs(o.density() - pattern_values(s, P)).max() < 1e-12
        o.step()


def test_thread_count_does_not_change_results():
    s = synth.water_box(32, 10.0, 6, n_link=8)
    e = []
    for nt in (1, 3):
        o = Oracle(s, n_threads=nt)
        e.append([o.step()["energy"] for _ in range(3)])
    assert e[0] == e[1]


# ---------------------------------------------------------------------------------------
# P5: the paper's accuracy claim (abstract item iii; section 4.1, table 1)
# ---------------------------------------------------------------------------------------

@pytest.mark.slow
def test_cutoff_error_below_scf_criterion(water128):
    s = water128
    ref = dense_scf(s, tol=1e-12)
    e_conv = 1e-6
    o = Oracle(s, eps=e_conv / 10, e_conv=1e-10)
    run_to_convergence(o)
    assert abs(o.energy() - ref["energy"]) < e_conv
