"""The allocation-free atom neighbour map (sscf_atom_neighbours_noalloc) through the C ABI.

Its map must equal the allocating call's (sscf_atom_neighbours, section 3.2) entry for entry,
on two calls in a row, the second on a smaller input: the fixed scratch keeps the first call's
contents, so a stale count or error flag would show.  Also its refusals.
"""
import ctypes as ct

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def call(xyz, cutoff, rowptr, col, cap):
    import torch
    from paper_1402_2880_amd.sscf import lib
    nnz = ct.c_int64(-1)
    rc = lib().sscf_atom_neighbours_noalloc(xyz.shape[0], xyz.data_ptr(), cutoff, torch.cuda.current_stream().cuda_stream,
                                            rowptr.data_ptr(), None if col is None else col.data_ptr(), cap,
                                            ct.byref(nnz))
    return rc, nnz.value


def noalloc_map(xyz_host, cutoff):
    import torch
    n = xyz_host.shape[0]
    x = torch.tensor(np.ascontiguousarray(xyz_host), dtype=torch.float64, device="cuda")
    rp = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
    rc, nnz = call(x, cutoff, rp, None, 0)                 # size first: col NULL
    assert rc == -6 and nnz > 0
    col = torch.full((nnz,), -7, dtype=torch.int32, device="cuda")
    rc, nnz2 = call(x, cutoff, rp, col, nnz)
    assert rc == 0 and nnz2 == nnz
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col.cpu().numpy()


def test_noalloc_equals_allocating_call_on_two_calls():
    from paper_1402_2880_amd import synth
    from paper_1402_2880_amd.sscf import atom_neighbours
    cut = synth.SK_CUTOFF * synth.BOHR_PER_ANGSTROM
    for s in (synth.make_config("water512", 1), synth.water_box(40, 10.0, 3)):   # 1,536 then 120 atoms
        rp_a, col_a = atom_neighbours(s.xyz_bohr, cut)
        rp_b, col_b = noalloc_map(s.xyz_bohr, cut)
        print(f"[noalloc] {s.n_atoms} atoms: {rp_b[-1]} entries", flush=True)
        assert np.array_equal(rp_a, rp_b)
        assert np.array_equal(col_a, col_b)


def test_noalloc_ragged_and_lattice():
    """A lattice with distances exactly on the cut-off (strict test) and a ragged last tile."""
    from paper_1402_2880_amd.sscf import atom_neighbours
    g = np.arange(5, dtype=np.float64)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)[:123]
    for cut in (1.0, 1.5):
        rp_a, col_a = atom_neighbours(pts, cut)
        rp_b, col_b = noalloc_map(pts, cut)
        assert np.array_equal(rp_a, rp_b) and np.array_equal(col_a, col_b)


def test_noalloc_refusals_leave_later_calls_correct():
    import torch
    from paper_1402_2880_amd.sscf import atom_neighbours, lib
    cut = 3.0
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, 20, size=(300, 3))
    # too many atoms for the fixed scratch: refused before any device work
    big = torch.zeros((262145, 3), dtype=torch.float64, device="cuda")
    rp_big = torch.zeros(262146, dtype=torch.int64, device="cuda")
    rc, _ = call(big, cut, rp_big, None, 0)
    assert rc == -6
    # host pointers are refused
    nnz = ct.c_int64(0)
    hx = np.ascontiguousarray(pts)
    hrp = np.zeros(301, dtype=np.int64)
    rc = lib().sscf_atom_neighbours_noalloc(300, hx.ctypes.data, cut, None, hrp.ctypes.data, None, 0, ct.byref(nnz))
    assert rc == -1
    # a non-finite coordinate sets the error flag; the next call starts from a clear flag
    bad = pts.copy()
    bad[17, 1] = np.nan
    x = torch.tensor(bad, device="cuda")
    rp = torch.zeros(301, dtype=torch.int64, device="cuda")
    rc, _ = call(x, cut, rp, None, 0)
    assert rc == -1
    rp_a, col_a = atom_neighbours(pts, cut)
    rp_b, col_b = noalloc_map(pts, cut)
    assert np.array_equal(rp_a, rp_b) and np.array_equal(col_a, col_b)
