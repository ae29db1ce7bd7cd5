"""Pins of the oracle's initial guess (section 3.3): each fragment's columns solve
H0 c = lambda S c on its AOs (residual), are S-orthonormal, ordered by lambda, carry the sign
convention, and the assembled C0 has the documented column order (it is the input C0 of the
synthetic systems, which the input generator builds by the same definition)."""
import numpy as np

from oracle.guess import fragment_blocks, fragment_guess
from paper_1402_2880_amd import synth


def frag_inputs(s):
    n_mol = int(s.atom_mol.max()) + 1
    first = np.searchsorted(s.atom_mol, np.arange(n_mol))
    last = np.searchsorted(s.atom_mol, np.arange(n_mol), side="right")
    nocc = np.array([int(round(s.q0[a:b].sum())) // 2 for a, b in zip(first, last)], dtype=np.int32)
    return s.atom_mol.astype(np.int32), nocc, s.atom_group[first].astype(np.int32)


def test_guess_solves_each_fragment():
    s = synth.water_box(27, 10.0, 3, n_link=3)
    af, fn, fg = frag_inputs(s)
    cp, row, val, mg, n_occ, lams = fragment_guess(s, af, fn, fg)
    blocks = fragment_blocks(s, af)
    col_of = {}
    for j in range(len(cp) - 1):
        col_of.setdefault(int(row[cp[j]]), []).append(j)
    for f, (lo, S, H) in enumerate(blocks):
        cols = sorted(col_of[lo])
        C = np.zeros((S.shape[0], len(cols)))
        for t, j in enumerate(cols):
            C[row[cp[j]:cp[j + 1]] - lo, t] = val[cp[j]:cp[j + 1]]
        lam = np.concatenate([lams[f][:fn[f]], lams[f][fn[f]:]])
        assert np.abs(C.T @ S @ C - np.eye(len(cols))).max() < 1e-12
        assert np.abs(H @ C - S @ C * lam[None, :]).max() < 1e-12
        assert np.all(np.diff(lams[f]) > 0)
        for t in range(C.shape[1]):
            a = np.abs(C[:, t])
            k = int(np.nonzero(a >= a.max() * (1 - 1e-10))[0][0])
            assert C[k, t] > 0


def test_guess_column_order_matches_the_input_c0():
    s = synth.make_config("water128", 1)
    af, fn, fg = frag_inputs(s)
    cp, row, val, mg, n_occ, _ = fragment_guess(s, af, fn, fg, drop=1e-13)
    assert n_occ == s.n_occ
    assert np.array_equal(mg, s.mo_group)
    assert np.array_equal(cp, s.c0_colptr) and np.array_equal(row, s.c0_row)
    # the input generator takes the strict argmax for the sign: equal up to each column's sign
    for j in range(len(cp) - 1):
        a, b = val[cp[j]:cp[j + 1]], s.c0_val[cp[j]:cp[j + 1]]
        assert min(np.abs(a - b).max(), np.abs(a + b).max()) < 1e-14
