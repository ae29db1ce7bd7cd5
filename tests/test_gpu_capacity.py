"""Tile capacity of C (slot_margin_bohr): storage only for the row blocks near each group.

Group g keeps the row blocks within reach_g + margin of it (reach_g: how far its initial MOs
reach); the products Y = X C keep the row blocks that S links to those.  Where the MOs stay
inside, every result is the dense-capacity one bit for bit (the same kernels run on the same
values; only the addresses differ), with fewer tiles stored.  Tiles just outside that a
combination reaches are computed and checked to stay zero.  An MO that does reach beyond is
refused with SSCF_E_CAPACITY instead of dropping values.
"""
import numpy as np
import pytest

from paper_1402_2880_amd import synth

pytestmark = pytest.mark.gpu


def gpu(system, **kw):
    from paper_1402_2880_amd.sscf import SparseSCF
    return SparseSCF(system, **kw)


@pytest.fixture(scope="module")
def water4096():
    return synth.make_config("water4096", 1)


@pytest.mark.parametrize("precision", [0, 1])
def test_slots_bit_identical_to_dense_capacity(water4096, precision):
    """12,288 atoms in a 50 A box; the MOs reach about 24 bohr past their group's molecules,
    so a margin of 30 bohr holds them while storing about a third of the tiles."""
    s = water4096
    dense = gpu(s, precision=precision)
    pool = gpu(s, precision=precision, slot_margin_bohr=30.0)
    md, mp = dense.memory_info(), pool.memory_info()
    print(f"[capacity] water4096: C {mp['tile_slots']} and Y {mp['tile_slots_y']} of {mp['tiles']} tiles stored, "
          f"device bytes {mp['device_bytes'] / 1e9:.3f} GB against {md['device_bytes'] / 1e9:.3f} GB", flush=True)
    assert md["tile_slots"] == md["tile_slots_y"] == md["tiles"]
    assert mp["tile_slots"] < 0.5 * mp["tiles"] and mp["tile_slots"] < mp["tile_slots_y"] < mp["tiles"]
    assert pool.init_info()["energy"] == dense.init_info()["energy"]
    for k in range(10):
        a, b = dense.step(), pool.step()
        assert a["energy"] == b["energy"] and a["n_rotations"] == b["n_rotations"], k
        assert a["n_ortho_sweeps"] == b["n_ortho_sweeps"] and a["nnz_tiles"] == b["nnz_tiles"], k
    assert np.array_equal(dense.charges(), pool.charges())
    assert np.array_equal(dense.density(), pool.density())
    ga, gb = dense.energy_gradient(), pool.energy_gradient()
    assert np.array_equal(ga[0], gb[0]) and np.array_equal(ga[1], gb[1])
    ca, cb = dense.mo_csc(), pool.mo_csc()
    assert all(np.array_equal(x, y) for x, y in zip(ca, cb))
    dense.close()
    pool.close()


def test_margin_too_small_is_refused():
    from paper_1402_2880_amd.sscf import SSCFError
    s = synth.water_box(64, 13.0, 16, n_link=8)
    with pytest.raises(SSCFError) as e:
        gpu(s, slot_margin_bohr=3.0)         # the first orthonormalization spreads the MOs further
    assert e.value.status == -6 and "group" in str(e.value) and "bohr" in str(e.value)
    print(f"[capacity] refused: {e.value}", flush=True)
    g = gpu(s, slot_margin_bohr=100.0)       # the box is smaller than that: same as dense
    m = g.memory_info()
    assert m["tile_slots"] == m["tile_slots_y"] == m["tiles"]
    d = gpu(s)
    for _ in range(3):
        assert g.step()["energy"] == d.step()["energy"]
