"""Pins of the oracle's energy gradient (differentiation form).

The gradient formulas (dE/dH0 = P, dE/dS = -W + 1/2 P (Q_a + Q_b)) rest on the energy being
stationary at self-consistency.  They are pinned against:
  * central finite differences of the converged energy, recomputed from scratch for
    perturbed inputs (nothing of the gradient code is used), along random symmetric
    directions on the pattern and along an onsite (diagonal) direction;
  * the dense identity W = 1/2 P H P with H = H0 + 1/2 S (Q_a + Q_b), computed with numpy
    from the density and charges alone.
"""
import dataclasses

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1402_2880_amd import synth
from tests.dense_ref import gamma_matrix
from tests.test_oracle_pins import pattern_values

# dense limit: every group pair is a neighbour pair, thresholds far below the FD noise
TIGHT = dict(eps=1e-12, e_conv=1e-13, r_nbr_bohr=1e6, max_sweeps_step=50)


def converged(system, **kw):
    """Oracle run until converged, then until the occupied-virtual coupling is negligible."""
    o = Oracle(system, **{**TIGHT, **kw})
    for _ in range(400):
        info = o.step()
        if info["converged"] and info["max_abs_fov"] < 1e-10:
            return o
    raise AssertionError("oracle SCF did not converge")


def sym_direction(system, rng, diag_atoms=None):
    """A symmetric AO-matrix direction on the atom-block pattern (S_val layout)."""
    n = system.n_ao
    if diag_atoms is None:
        D = rng.standard_normal((n, n))
        D = 0.5 * (D + D.T)
    else:
        D = np.zeros((n, n))
        aoo = system.ao_offset()
        for a in diag_atoms:
            D[aoo[a]:aoo[a + 1], aoo[a]:aoo[a + 1]] = np.eye(aoo[a + 1] - aoo[a])
    return pattern_values(system, D)


def fd(system, field, d, h):
    vals = getattr(system, field)
    ep = converged(dataclasses.replace(system, **{field: vals + h * d})).energy()
    em = converged(dataclasses.replace(system, **{field: vals - h * d})).energy()
    return (ep - em) / (2 * h)


@pytest.fixture(scope="module")
def small():
    return synth.water_box(4, 6.0, 3, n_link=2)


@pytest.fixture(scope="module")
def small_state(small):
    o = converged(small)
    return o, o.gradient()


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_h0_matches_finite_differences(small, small_state, seed):
    o, (gx, gs) = small_state
    d = sym_direction(small, np.random.default_rng(seed))
    num = fd(small, "H0_val", d, 1e-5)      # FD error ~ 1e2 h^2 for these directions
    ana = float(gx @ d)
    assert abs(num - ana) < 5e-8 * max(1.0, abs(ana)), (num, ana)


@pytest.mark.parametrize("seed", [2, 3])
def test_gradient_s_matches_finite_differences(small, small_state, seed):
    o, (gx, gs) = small_state
    d = sym_direction(small, np.random.default_rng(seed))
    num = fd(small, "S_val", d, 3e-6)
    ana = float(gs @ d)
    assert abs(num - ana) < 5e-8 * max(1.0, abs(ana)), (num, ana)


def test_gradient_onsite_matches_finite_differences(small, small_state):
    """dE/d(onsite energy of one atom's AOs) = sum of P over those diagonal entries."""
    o, (gx, gs) = small_state
    d = sym_direction(small, None, diag_atoms=[0])
    num = fd(small, "H0_val", d, 1e-5)
    assert abs(num - float(gx @ d)) < 5e-8


def test_gradient_non_scc_matches_finite_differences(small):
    o = converged(small, scc=False)
    gx, gs = o.gradient()
    d = sym_direction(small, np.random.default_rng(7))
    vals = small.S_val
    h = 3e-6
    ep = converged(dataclasses.replace(small, S_val=vals + h * d), scc=False).energy()
    em = converged(dataclasses.replace(small, S_val=vals - h * d), scc=False).energy()
    assert abs((ep - em) / (2 * h) - float(gs @ d)) < 5e-8 * max(1.0, abs(float(gs @ d)))


def test_w_is_half_php(small, small_state):
    """Sparse W (pair blocks of C^T H C, then C F C^T) equals 1/2 P H P formed densely."""
    o, (gx, gs) = small_state
    S, H0 = small.dense("S"), small.dense("H0")
    P = np.zeros_like(S)
    aoo = small.ao_offset()
    pv = o.density()
    for a in range(small.n_atoms):
        for k in range(small.blk_rowptr[a], small.blk_rowptr[a + 1]):
            b = small.blk_col[k]
            na, nb = small.atom_nao[a], small.atom_nao[b]
            P[aoo[a]:aoo[a] + na, aoo[b]:aoo[b] + nb] = \
                pv[small.blk_off[k]:small.blk_off[k] + na * nb].reshape(na, nb)
    dq = o.charges() - small.q0
    Q = gamma_matrix(small) @ dq
    Qao = Q[np.repeat(np.arange(small.n_atoms), small.atom_nao)]
    Qs = Qao[:, None] + Qao[None, :]
    H = H0 + 0.5 * S * Qs
    W = 0.5 * P @ H @ P
    ref_s = pattern_values(small, -W + 0.5 * P * Qs)
    assert np.abs(gx - pv).max() == 0.0
    assert np.abs(gs - ref_s).max() < 1e-10


def test_gradient_with_complete_fock(small):
    """With a complete Fock matrix F, E = tr(P F): dE/dF = P and dE/dS = -1/2 P F P."""
    o = Oracle(small, **TIGHT)
    F = small.H0_val * 1.01
    o.set_fock(F, 1)
    for _ in range(200):
        info = o.step()
        if info["converged"] and info["max_abs_fov"] < 1e-10:
            break
    gx, gs = o.gradient()
    S = small.dense("S")
    Fd = small.dense("H0") * 1.01
    pv = o.density()
    P = np.zeros_like(S)
    aoo = small.ao_offset()
    for a in range(small.n_atoms):
        for k in range(small.blk_rowptr[a], small.blk_rowptr[a + 1]):
            b = small.blk_col[k]
            na, nb = small.atom_nao[a], small.atom_nao[b]
            P[aoo[a]:aoo[a] + na, aoo[b]:aoo[b] + nb] = \
                pv[small.blk_off[k]:small.blk_off[k] + na * nb].reshape(na, nb)
    assert np.abs(gx - pv).max() == 0.0
    assert np.abs(gs - pattern_values(small, -0.5 * P @ Fd @ P)).max() < 1e-10
