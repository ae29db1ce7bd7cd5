"""The library's algorithmic work counters (SSCF_FLAG_COUNT_WORK) against the oracle's.

Both sides count the same definitions (include/sscf.h, sscf_get_kernel_stats; oracle.h,
orc_work) on their own state, pass by pass: nonzeros of C, D_sel, S C and H C, support
intersections of the C^T X C pairs, selected pairs, rows reached by the rotations.  The
oracle's counts are pinned on the CPU against dense recounts (tests/test_selection_pins.py).
The two states agree to rounding, so the counts agree exactly unless a value sits within
rounding of a truncation threshold; the bar leaves room for a few such values.
"""
import json
import os

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1402_2880_amd import synth

pytestmark = pytest.mark.gpu

CLASSES = {"spmm_tiles": "product", "pair_overlap": "overlap", "pair_fock": "fock_blocks",
           "ortho_update": "combine", "rotations": "rotate"}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "{}_seed{}.json")


def gpu(system, **kw):
    from paper_1402_2880_amd.sscf import SparseSCF
    return SparseSCF(system, count_work=True, profile=True, **kw)


def check_counts(ks, work, rel, label):
    for gk, ok in CLASSES.items():
        for q in ("flops", "bytes"):
            a, b = ks[gk]["alg_" + q], work[ok][q]
            assert abs(a - b) <= rel * max(b, 1.0), (label, gk, q, a, b)


def compare_work(system, n_steps, rel=0.0, label="", **kw):
    o = Oracle(system, **kw)
    o.set_count(True)
    g = gpu(system, **kw)
    for k in range(n_steps):
        g.reset_kernel_stats()
        gs, os_ = g.step(), o.step()
        ks = g.kernel_stats()
        print(f"[work] {label} step {k + 1}: " + " ".join(
            f"{c} {ks[c]['alg_flops']:.4e}/{ks[c]['alg_bytes']:.4e}" for c in CLASSES), flush=True)
        assert gs["n_rotations"] == os_["n_rotations"] and gs["n_ortho_sweeps"] == os_["n_ortho_sweeps"]
        assert gs["post_ortho"] == os_["post_ortho"]
        check_counts(ks, o.work()["classes"], rel, f"{label} step {k + 1}")
        assert abs(gs["nnz_c"] - os_["nnz_c"]) <= rel * os_["nnz_c"]
    g.close()


def test_work_counts_binding_cap():
    """48 molecules, a rotation cap of N_occ / 4 that binds every step."""
    compare_work(synth.water_box(48, 12.0, 8, n_link=8), 4, label="cap", rot_cap_factor=0.25)


def test_work_counts_water128(water128):
    """The 128-molecule box through convergence (occupied-only step III included)."""
    compare_work(water128, 12, label="water128")


def test_work_counts_panel_128():
    compare_work(synth.water_box(60, 12.5, 7, n_link=20), 4, label="panel 128")


def test_counts_off_by_default(water128):
    from paper_1402_2880_amd.sscf import SparseSCF
    g = SparseSCF(water128, profile=True)
    si = g.step()
    assert si["nnz_c"] == -1
    ks = g.kernel_stats()
    assert all(v["alg_flops"] == -1.0 for v in ks.values())
    assert ks["spmm_tiles"]["mfma_flops"] > 0
    g.close()


@pytest.mark.parametrize("config,seed", [("water4096", 1), ("water4096", 2), ("octane400", 1)])
def test_work_counts_stored(config, seed):
    """The 12,288-atom water box and the 10,400-atom octane box: every stored step's counts
    (oracle, tests/golden/make_golden.py)."""
    path = GOLDEN.format(config, seed)
    if not os.path.exists(path):
        pytest.skip("no stored values")
    rec = json.load(open(path))
    steps = [st for st in rec["steps"] if "work" in st]
    if not steps:
        pytest.skip("stored values hold no work counts")
    s = synth.make_config(config, seed)
    print(f"[work] {config} seed {seed}: {len(steps)} stored steps", flush=True)
    g = gpu(s, eps=rec["eps"], e_conv=rec["e_conv"], **rec.get("options", {}))
    for k, st in enumerate(steps):
        g.reset_kernel_stats()
        gs = g.step()
        ks = g.kernel_stats()
        print(f"[work] {config} step {k + 1}: combination {ks['ortho_update']['alg_flops']:.4e} flops "
              f"(oracle {st['work']['classes']['combine']['flops']:.4e}), nnz C {gs['nnz_c']} "
              f"(oracle {st['nnz_c']})", flush=True)
        check_counts(ks, st["work"]["classes"], 1e-5, f"{config} step {k + 1}")
        assert abs(gs["nnz_c"] - st["nnz_c"]) <= 1e-5 * st["nnz_c"]
    g.close()
