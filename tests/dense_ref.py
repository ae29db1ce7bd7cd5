"""Dense references that pin the oracle (test infrastructure).

These do not follow the sparse algorithm at all: they solve the same
SCC-DFTB problem by full generalized diagonalization (LAPACK sygvd through
scipy, the routine family the paper compares against in its accuracy table),
so an error anywhere in the sparse oracle shows up as a disagreement.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh


def gamma_matrix(system) -> np.ndarray:
    """gamma_ab = 1/sqrt(r^2 + u^2), u = (1/U_a + 1/U_b)/2 (bohr, Ha); gamma_aa = U_a."""
    x = system.xyz_bohr
    U = system.hubbard_u
    r2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    u = 0.5 * (1.0 / U[:, None] + 1.0 / U[None, :])
    g = 1.0 / np.sqrt(r2 + u * u)
    np.fill_diagonal(g, U)
    return g


def _scc_map(system, S, H0, g, ao_atom, aoo, dq, scc=True):
    Q = g @ dq if scc else np.zeros_like(dq)
    Qao = Q[ao_atom]
    H = H0 + 0.5 * S * (Qao[:, None] + Qao[None, :])
    w, V = eigh(H, S)
    C = V[:, :system.n_occ]
    P = 2.0 * C @ C.T
    q = np.add.reduceat((P * S).sum(1), aoo[:-1])
    dqn = q - system.q0
    E = float((P * H0).sum() + (0.5 * dqn @ g @ dqn if scc else 0.0))
    return dqn, E, w, P


def dense_scf(system, scc: bool = True, tol: float = 1e-12, maxit: int = 200, ndiis: int = 8,
              mix: float = 0.3):
    """Aufbau SCC-DFTB SCF by dense diagonalization with DIIS on the charges.

    Returns dict(energy, charges, gap, density (dense AO), iterations, converged).
    """
    S = system.dense("S")
    H0 = system.dense("H0")
    g = gamma_matrix(system)
    aoo = system.ao_offset()
    ao_atom = np.repeat(np.arange(system.n_atoms), system.atom_nao)
    dq = np.zeros(system.n_atoms)
    hx, hr = [], []
    converged = False
    for it in range(maxit):
        dqn, E, w, P = _scc_map(system, S, H0, g, ao_atom, aoo, dq, scc)
        r = dqn - dq
        if not scc or np.abs(r).max() < tol:
            converged = True
            break
        hx.append(dq.copy())
        hr.append(r.copy())
        hx, hr = hx[-ndiis:], hr[-ndiis:]
        m = len(hr)
        R = np.array(hr)
        B = np.zeros((m + 1, m + 1))
        B[:m, :m] = R @ R.T
        B[m, :m] = B[:m, m] = -1.0
        rhs = np.zeros(m + 1)
        rhs[m] = -1.0
        try:
            c = np.linalg.solve(B, rhs)[:m]
        except np.linalg.LinAlgError:
            c = np.full(m, 1.0 / m)
        dq = sum(ci * (x + mix * ri) for ci, x, ri in zip(c, hx, hr))
    return dict(energy=E, charges=dqn + system.q0, gap=float(w[system.n_occ] - w[system.n_occ - 1]),
                density=P, iterations=it, converged=converged, eigenvalues=w)
