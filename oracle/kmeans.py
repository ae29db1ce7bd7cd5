"""Constrained k-means of section 3.2 (oracle side; test infrastructure only).

Every point (an atom, or a molecule centre) is linked to one of m means, no mean holding more
than n_link points; each mean then moves to the centroid of its points, and the two steps
repeat until the average displacement of the means falls below a threshold or an iteration
cap is reached.

Reading of the linking step.  The section links each point to its closest mean and, when that
mean is full, to the next closest one with room; it notes that the result then depends on the
order in which points are visited.  The attribution taken here is the order-free one with the
same rule: the stable matching in which points rank means by squared distance (ties: lower
mean index) and a full mean prefers its closest points (ties: lower point index).  No point
could move to a mean it ranks higher that has room, or that holds a point ranking below it.
It is computed by the textbook one-proposal-at-a-time deferred acceptance (Gale and Shapley,
1962; many-to-one form): a free point proposes to the best mean that has not turned it down;
the mean keeps it if it has room, otherwise keeps the better of the newcomer and its worst
point and turns the other one away.  The stable matching this reaches is the same for every
order of proposals (the points' best stable matching), which the tests check by brute force.

Arithmetic: squared distances are (dx*dx + dy*dy) + dz*dz, every operation a rounded IEEE
double; centroids are the coordinate sums in point order divided by the count (an empty mean
stays where it is); the displacement is the sum over means, in mean order, of the Euclidean
length of new - old, divided by m.  Independent of the HIP library.
"""
from __future__ import annotations

import math

import numpy as np


def squared_distances(points: np.ndarray, means: np.ndarray) -> np.ndarray:
    """d2[p, c] = (dx*dx + dy*dy) + dz*dz with d = point p - mean c."""
    dx = points[:, None, 0] - means[None, :, 0]
    dy = points[:, None, 1] - means[None, :, 1]
    dz = points[:, None, 2] - means[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def attribution(points: np.ndarray, means: np.ndarray, n_link: int) -> np.ndarray:
    """Mean of every point in the stable capacity-n_link attribution (see the module text)."""
    n, m = points.shape[0], means.shape[0]
    if m * n_link < n:
        raise ValueError("the means cannot hold all points")
    d2 = squared_distances(points, means)
    pref = np.argsort(d2, axis=1, kind="stable")       # ties keep the lower mean index first
    nxt = np.zeros(n, dtype=np.int64)                  # next mean to try, as a rank
    held: list[list[tuple[float, int]]] = [[] for _ in range(m)]
    group = np.full(n, -1, dtype=np.int64)
    free = list(range(n - 1, -1, -1))                  # proposals start with point 0
    while free:
        p = free.pop()
        c = int(pref[p, nxt[p]])
        key = (float(d2[p, c]), p)
        if len(held[c]) < n_link:
            held[c].append(key)
            group[p] = c
            continue
        worst = max(held[c])
        if key < worst:
            held[c].remove(worst)
            held[c].append(key)
            group[p] = c
            q = worst[1]
            group[q] = -1
            nxt[q] += 1
            free.append(q)
        else:
            nxt[p] += 1
            free.append(p)
    return group


def centroids(points: np.ndarray, group: np.ndarray, means: np.ndarray) -> np.ndarray:
    """Each mean moved to the centroid of its points (sums in point order)."""
    m = means.shape[0]
    sums = [[0.0, 0.0, 0.0] for _ in range(m)]
    count = [0] * m
    for p in range(points.shape[0]):
        c = int(group[p])
        for k in range(3):
            sums[c][k] += float(points[p, k])
        count[c] += 1
    out = np.array(means, dtype=np.float64, copy=True)
    for c in range(m):
        if count[c]:
            out[c] = [sums[c][k] / count[c] for k in range(3)]
    return out


def average_displacement(old: np.ndarray, new: np.ndarray) -> float:
    """Sum over the means, in mean order, of |new - old|, divided by m."""
    total = 0.0
    for c in range(old.shape[0]):
        dx, dy, dz = (float(new[c, k] - old[c, k]) for k in range(3))
        total += math.sqrt((dx * dx + dy * dy) + dz * dz)
    return total / old.shape[0]


def constrained_kmeans(points, means0, n_link: int, max_iter: int = 100, tol: float = 1e-4):
    """Iterate attribution and move.  Returns (group of each point in the last attribution,
    means after the last move, iterations done, last average displacement)."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    means = np.asarray(means0, dtype=np.float64).reshape(-1, 3).copy()
    group = None
    disp = 0.0
    it = 0
    while it < max_iter:
        group = attribution(points, means, n_link)
        new = centroids(points, group, means)
        disp = average_displacement(means, new)
        means = new
        it += 1
        if disp < tol:
            break
    return group, means, it, disp
