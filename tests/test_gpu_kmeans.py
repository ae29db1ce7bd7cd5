"""Constrained k-means of section 3.2 on the GPU against the oracle's (oracle/kmeans.py).

Parity is exact: the same attribution of every point, the same means bit for bit, the same
number of iterations and the same last displacement.  The water boxes do not settle below the
threshold and run all 100 iterations, so one rounding difference anywhere would show.
Cases: the three water boxes' molecule centres, an integer lattice full of exact ties,
proposals to one mean spanning several LDS chunks, empty means, one point,
one point per mean, and the error paths.  Last, an SCF on MO groups made by the GPU k-means
agrees with the oracle's SCF on the same system.
"""
import numpy as np
import pytest

from oracle import kmeans as km
from oracle.oracle import Oracle
from paper_1402_2880_amd import synth

pytestmark = pytest.mark.gpu


def water_inputs(n_mol, box, seed=1, n_link=synth.N_LINK):
    rng = np.random.default_rng(seed)
    xyz, el = synth.water_geometry(rng, n_mol, box)
    opos = xyz[0::3]
    m = -(-n_mol // n_link)
    return xyz, el, opos, synth.initial_means(rng, opos, m)


def check(points, means0, n_link, label, **kw):
    from paper_1402_2880_amd.sscf import constrained_kmeans
    print(f"[kmeans] {label}: n={len(points)} m={len(means0)} n_link={n_link} {kw}", flush=True)
    g, means, info = constrained_kmeans(points, means0, n_link, **kw)
    og, omeans, oit, odisp = km.constrained_kmeans(points, means0, n_link, **kw)
    assert np.array_equal(g, og), np.flatnonzero(g != og)[:10]
    assert np.array_equal(means, omeans), np.abs(means - omeans).max()
    assert info["iterations"] == oit
    assert info["displacement"] == odisp
    return g, means, info


@pytest.mark.parametrize("name,n_mol,box", [("water128", 128, 16.0), ("water512", 512, 25.0),
                                            ("water4096", 4096, 50.0)])
def test_water_boxes_match_oracle(name, n_mol, box):
    _, _, opos, means0 = water_inputs(n_mol, box)
    g, _, info = check(opos, means0, synth.N_LINK, name)
    assert np.bincount(g).max() <= synth.N_LINK
    print(f"[kmeans] {name}: {info}", flush=True)


def test_lattice_ties():
    ax = np.arange(6, dtype=float)
    points = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)   # 216 points
    means0 = np.stack(np.meshgrid([1.0, 2.5, 4.0], [1.0, 4.0], [0.5, 2.5, 4.5], indexing="ij"), -1).reshape(-1, 3)
    check(points, means0, 12, "lattice", max_iter=30, tol=0.0)
    check(points, means0, 216, "lattice, unconstrained", max_iter=10)


def test_chunked_proposals():
    """Few means with a large n_link: a mean receives proposals from several chunks of
    KM_SLOTS - n_link points and merges them."""
    rng = np.random.default_rng(21)
    points = rng.uniform(0, 30, (5000, 3))
    check(points, rng.uniform(0, 30, (5, 3)), 1000, "5 means x 1000", max_iter=4)
    check(points, rng.uniform(0, 30, (6, 3)), 1024, "6 means x 1024", max_iter=3)


def test_small_and_degenerate():
    rng = np.random.default_rng(22)
    check(np.array([[1.0, 2.0, 3.0]]), np.array([[0.0, 0.0, 0.0]]), 1, "one point")
    p5 = rng.uniform(0, 3, (5, 3))
    check(p5, rng.uniform(0, 3, (5, 3)), 1, "one point per mean")
    # a mean far away never gets a point and stays where it is
    far = np.vstack([rng.uniform(0, 3, (3, 3)), [[1e3, 1e3, 1e3]]])
    g, means, _ = check(rng.uniform(0, 3, (20, 3)), far, 10, "empty mean")
    assert not (g == 3).any() and np.array_equal(means[3], far[3])
    check(rng.uniform(0, 3, (77, 3)), rng.uniform(0, 3, (26, 3)), 3, "ragged 77 / 3", max_iter=1)
    check(rng.uniform(0, 3, (100, 3)), rng.uniform(0, 3, (3, 3)), 100, "room everywhere", max_iter=100, tol=1e-12)


def test_errors():
    from paper_1402_2880_amd.sscf import SSCFError, constrained_kmeans
    rng = np.random.default_rng(23)
    p = rng.uniform(0, 1, (10, 3))
    bad = [(p, p[:3], 3, {}),                           # 3 x 3 < 10
           (p, p[:1], 1025, {}),                        # n_link above 1024
           (np.zeros((5000, 3)), np.zeros((4097, 3)), 2, {}),   # more than 4096 means
           (p, p[:5], 2, dict(max_iter=0)),
           (p, p[:5], 2, dict(tol=-1.0)),
           (np.where(np.arange(30).reshape(10, 3) == 4, np.nan, p), p[:5], 2, {})]
    for pts, m0, nl, kw in bad:
        with pytest.raises(SSCFError) as e:
            constrained_kmeans(pts, m0, nl, **kw)
        assert e.value.status == -1


def test_scf_on_gpu_groups():
    """Molecules ordered by the GPU attribution (the concatenation of the means' lists),
    MO groups = means: GPU and oracle SCF agree, and the converged energy is the one of the
    same box grouped by the input generator (the grouping does not change the energy)."""
    from paper_1402_2880_amd.sscf import SparseSCF, constrained_kmeans
    n_mol, box = 128, 16.0
    xyz, el, opos, means0 = water_inputs(n_mol, box)
    g, _, _ = constrained_kmeans(opos, means0, synth.N_LINK)
    order = np.lexsort((np.arange(n_mol), g))
    used = np.unique(g)
    ren = np.full(len(means0), -1)
    ren[used] = np.arange(used.size)
    atom_idx = (3 * order[:, None] + np.arange(3)[None, :]).ravel()
    s = synth.assemble("water128 gpu groups", 1, box, xyz[atom_idx], el[atom_idx], np.repeat(np.arange(n_mol), 3),
                       ren[g[order]], used.size)
    o, gp = Oracle(s), SparseSCF(s)
    for _ in range(30):
        a, b = o.step(), gp.step()
        assert abs(a["energy"] - b["energy"]) < 1e-8
        if a["converged"] and b["converged"]:
            break
    assert a["converged"] and b["converged"]
    ref = Oracle(synth.make_config("water128", 1))
    for _ in range(30):
        if ref.step()["converged"]:
            break
    assert abs(ref.energy() - gp.energy()) < 1e-6
