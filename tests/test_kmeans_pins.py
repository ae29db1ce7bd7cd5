"""Pins of the oracle's constrained k-means (section 3.2).

* brute force on tiny inputs: every capacity-respecting attribution is enumerated, the stable
  ones kept (distances from scipy's cdist, not the oracle's); the oracle's attribution is
  stable and gives every point its best mean over all stable attributions;
* exact ties on an integer lattice, decided by the index rules, against the same brute force;
* with room for every point at every mean the attribution is the plain nearest-mean one
  (scipy.cluster.vq.vq) and the iteration is Lloyd's k-means;
* the attribution does not depend on the order of the points;
* the stop rule and the displacement, against numpy's own norm;
* invariants (capacity, every point placed, stability) on water boxes.
"""
import itertools

import numpy as np
import pytest
from scipy.cluster.vq import vq
from scipy.spatial.distance import cdist

from oracle import kmeans as km
from paper_1402_2880_amd import synth


def is_stable(points, means, group, n_link, d2=None):
    """No point ranks another mean higher that has room or holds a point it outranks."""
    d2 = cdist(points, means, "sqeuclidean") if d2 is None else d2
    n, m = d2.shape
    members = [np.flatnonzero(group == c) for c in range(m)]
    if any(len(x) > n_link for x in members) or (group < 0).any():
        return False
    for p in range(n):
        mine = (d2[p, group[p]], group[p])
        for c in range(m):
            if (d2[p, c], c) >= mine:
                continue
            if len(members[c]) < n_link:
                return False
            worst = max((d2[q, c], q) for q in members[c])
            if (d2[p, c], p) < worst:
                return False
    return True


def brute_force_best(points, means, n_link):
    """For every point, the best mean (by (d2, index)) it gets in any stable attribution,
    and the number of stable attributions."""
    d2 = cdist(points, means, "sqeuclidean")
    n, m = d2.shape
    best = np.full(n, -1)
    count = 0
    for g in itertools.product(range(m), repeat=n):
        g = np.array(g)
        if np.bincount(g, minlength=m).max() > n_link or not is_stable(points, means, g, n_link, d2):
            continue
        count += 1
        for p in range(n):
            if best[p] < 0 or (d2[p, g[p]], g[p]) < (d2[p, best[p]], best[p]):
                best[p] = g[p]
    return best, count


@pytest.mark.parametrize("seed,n,m,n_link", [(0, 5, 2, 3), (1, 6, 3, 2), (2, 6, 2, 3), (3, 7, 3, 3),
                                             (4, 6, 3, 2), (5, 7, 2, 4), (6, 5, 5, 1)])
def test_attribution_is_points_best_stable_matching(seed, n, m, n_link):
    rng = np.random.default_rng(seed)
    points = rng.standard_normal((n, 3))
    means = 0.5 * rng.standard_normal((m, 3))
    g = km.attribution(points, means, n_link)
    best, count = brute_force_best(points, means, n_link)
    assert count >= 1
    assert is_stable(points, means, g, n_link)
    assert np.array_equal(g, best)


def test_attribution_ties_follow_index_rules():
    """Integer lattice: many exactly equal distances, decided by lower mean index (points'
    side) and lower point index (means' side)."""
    points = np.array([[0, 0, 0], [2, 0, 0], [1, 0, 0], [1, 1, 0], [1, -1, 0], [0, 2, 0]], dtype=float)
    means = np.array([[0, 1, 0], [2, 1, 0], [1, 0, 1]], dtype=float)
    g = km.attribution(points, means, 2)
    best, count = brute_force_best(points, means, 2)
    assert count >= 1
    assert np.array_equal(g, best)
    # exact distances on both sides, so the oracle's own d2 must agree bit for bit
    assert np.array_equal(km.squared_distances(points, means), cdist(points, means, "sqeuclidean"))


def test_unconstrained_is_nearest_mean_and_lloyd():
    rng = np.random.default_rng(11)
    points = rng.uniform(0, 10, (200, 3))
    means0 = rng.uniform(2, 8, (6, 3))
    g = km.attribution(points, means0, 200)
    assert np.array_equal(g, vq(points, means0)[0])
    group, means, it, disp = km.constrained_kmeans(points, means0, 200, max_iter=5, tol=0.0)
    ref = means0.copy()
    for _ in range(5):
        code = vq(points, ref)[0]
        ref = np.array([points[code == c].mean(axis=0) if (code == c).any() else ref[c] for c in range(6)])
    assert it == 5
    assert np.array_equal(group, code)
    assert np.abs(means - ref).max() < 1e-12


def test_attribution_independent_of_point_order():
    rng = np.random.default_rng(12)
    points = rng.uniform(0, 6, (90, 3))
    means = synth.initial_means(rng, points, 10)
    g = km.attribution(points, means, 9)
    perm = rng.permutation(90)
    gp = km.attribution(points[perm], means, 9)
    assert np.array_equal(gp, g[perm])


def test_capacity_binds_and_stop_rule():
    rng = np.random.default_rng(13)
    points = rng.uniform(0, 5, (64, 3))
    means0 = synth.initial_means(rng, points, 8)
    group, means, it, disp = km.constrained_kmeans(points, means0, 8, max_iter=1, tol=0.0)
    assert it == 1 and np.bincount(group, minlength=8).max() == 8
    g1 = km.attribution(points, means0, 8)
    assert np.array_equal(group, g1)
    ref_disp = np.linalg.norm(means - means0, axis=1).mean()
    assert abs(disp - ref_disp) <= 1e-15 * max(1.0, ref_disp)
    # a threshold above the first displacement stops after one iteration
    assert km.constrained_kmeans(points, means0, 8, max_iter=50, tol=disp * 1.01)[2] == 1
    g3, m3, it3, d3 = km.constrained_kmeans(points, means0, 8, max_iter=3, tol=0.0)
    assert it3 == 3
    with pytest.raises(ValueError):
        km.attribution(points, means0[:7], 8)


@pytest.mark.parametrize("n_mol,box,n_link", [(128, 16.0, 16), (300, 20.0, 7)])
def test_water_box_invariants(n_mol, box, n_link):
    rng = np.random.default_rng(5)
    xyz, _ = synth.water_geometry(rng, n_mol, box)
    opos = xyz[0::3]
    m = -(-n_mol // n_link)
    means0 = synth.initial_means(rng, opos, m)
    group, means, it, disp = km.constrained_kmeans(opos, means0, n_link)
    assert (group >= 0).all() and np.bincount(group, minlength=m).max() <= n_link
    assert it <= 100 and (disp < 1e-4 or it == 100)
    # the returned attribution is the stable one for the means it was made with
    prev = km.constrained_kmeans(opos, means0, n_link, max_iter=it - 1)[1] if it > 1 else means0
    assert np.array_equal(km.attribution(opos, prev, n_link), group)
    assert is_stable(opos, prev, group, n_link)
