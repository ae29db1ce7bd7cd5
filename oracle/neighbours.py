"""Atom neighbour map of section 3.2 (oracle side; test infrastructure only).

Two atoms are neighbours unless every S and H element between their AOs is zero.  With
two-centre elements that vanish beyond a radial cut-off this is the pair distance test
(dx*dx + dy*dy) + dz*dz < cutoff*cutoff, each operation a rounded IEEE double, d = r_a - r_b;
every atom is its own neighbour.  The map is written as CSR rows in atom order with ascending
columns.  Plain brute force over all pairs, row by row; independent of the HIP library.
"""
from __future__ import annotations

import numpy as np


def atom_neighbours(xyz, cutoff: float):
    """(rowptr int64[n + 1], col int64[nnz]) of the pairs closer than cutoff, self included."""
    x = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    c2 = cutoff * cutoff
    rowptr = np.zeros(x.shape[0] + 1, dtype=np.int64)
    cols = []
    for a in range(x.shape[0]):
        dx = x[a, 0] - x[:, 0]
        dy = x[a, 1] - x[:, 1]
        dz = x[a, 2] - x[:, 2]
        nb = np.flatnonzero((dx * dx + dy * dy) + dz * dz < c2)
        cols.append(nb)
        rowptr[a + 1] = rowptr[a] + nb.size
    return rowptr, (np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64))
