"""Atom neighbour map of section 3.2 on the GPU against the oracle's (oracle/neighbours.py):
identical CSR (integer-exact) on the water boxes (also equal to the pattern S and H are given
on), on unordered random points (every tile near every other), on a lattice whose pair
distances sit exactly on the cut-off, on ragged sizes, and the capacity and error paths."""
import numpy as np
import pytest

from oracle.neighbours import atom_neighbours as oracle_map
from paper_1402_2880_amd import synth

pytestmark = pytest.mark.gpu

CUT = synth.SK_CUTOFF * synth.BOHR_PER_ANGSTROM


def check(x, cutoff, label):
    from paper_1402_2880_amd.sscf import atom_neighbours
    print(f"[neighbours] {label}: n={len(x)} cutoff={cutoff}", flush=True)
    rp, col = atom_neighbours(x, cutoff)
    orp, ocol = oracle_map(x, cutoff)
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)
    return rp, col


@pytest.mark.parametrize("config", ["water128", "water512", "water4096"])
def test_water_boxes(config):
    s = synth.cached(config, 1) if config == "water4096" else synth.make_config(config, 1)
    rp, col = check(s.xyz_bohr, CUT, config)
    assert np.array_equal(rp, s.blk_rowptr) and np.array_equal(col, s.blk_col)


def test_unordered_points_and_ragged_sizes():
    rng = np.random.default_rng(31)
    check(rng.uniform(0, 30, (3000, 3)), 4.0, "random 3000")
    for n in (1, 2, 63, 64, 65, 130):
        check(rng.uniform(0, 5, (n, 3)), 2.0, f"random {n}")
    check(rng.uniform(0, 5, (200, 3)), 1e3, "all pairs")


def test_lattice_on_the_cutoff():
    ax = np.arange(6, dtype=float)
    x = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    rp, _ = check(x, 1.0, "lattice, cut-off 1")
    assert np.array_equal(np.diff(rp), np.ones(216))
    check(x, 2.0 ** 0.5, "lattice, cut-off sqrt(2)")
    check(x, 1.5, "lattice, cut-off 1.5")


def test_capacity_and_errors():
    import ctypes as ct
    from paper_1402_2880_amd import sscf
    x = np.ascontiguousarray(np.random.default_rng(32).uniform(0, 4, (50, 3)))
    orp, ocol = oracle_map(x, 1.5)
    nnz = ct.c_int64(0)
    rp = np.zeros(51, dtype=np.int64)
    col = np.zeros(10, dtype=np.int32)
    rc = sscf.lib().sscf_atom_neighbours(50, x.ctypes.data, 1.5, None, rp.ctypes.data, col.ctypes.data, 10,
                                         ct.byref(nnz))
    assert rc == sscf.STATUS_CAPACITY and nnz.value == ocol.size and not rp.any()
    with pytest.raises(sscf.SSCFError) as e:
        sscf.atom_neighbours(np.where(x > 3.9, np.nan, x), 1.0)
    assert e.value.status == -1
    with pytest.raises(sscf.SSCFError) as e:
        sscf.atom_neighbours(x, 0.0)
    assert e.value.status == -1
