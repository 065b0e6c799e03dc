"""The oracle's bucket-grid neighbour sets equal brute-force O(N^2) search.

The paper restricts the particle sums to particles inside the kernel support
(Section 3.1, footnote to eq. suminterp); the predicate is |s_i - s_j|^2 < R^2.
Adversarial placements put points on cell edges and at exactly R apart.
"""
import numpy as np
import pytest

from oracle import sph as O


def _as_set(pi, pj):
    return set(zip(pi.tolist(), pj.tolist()))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cells_equal_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-0.1, 0.1, (500, 2))
    R = 0.0125
    lo, hi = (-0.11, -0.11), (0.11, 0.11)
    a = O.pairs(pts, R, use_cells=False, domain_min=lo, domain_max=hi)
    b = O.pairs(pts, R, use_cells=True, domain_min=lo, domain_max=hi)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[0].size > 500


def test_cells_equal_brute_force_adversarial():
    R = 0.01
    cell = R * (1 + 1e-6)
    lo = np.array([-0.05, -0.05])
    pts = []
    # points exactly on cell edges, and pairs at exactly R and just inside R
    for k in range(-4, 5):
        e = lo[0] + (k + 5) * cell
        pts += [[e, 0.0], [e, e], [e - 1e-15, 0.013]]
    pts += [[0.0, 0.0], [R, 0.0], [0.0, R * (1 - 1e-12)], [-R * np.sqrt(0.5), -R * np.sqrt(0.5)]]
    pts = np.array(pts)
    a = O.pairs(pts, R, use_cells=False, domain_min=lo, domain_max=(0.05, 0.05))
    b = O.pairs(pts, R, use_cells=True, domain_min=lo, domain_max=(0.05, 0.05))
    assert _as_set(*a) == _as_set(*b)
    sa = _as_set(*a)
    # strict inequality: the pair exactly R apart is not a neighbour
    i0 = len(pts) - 4
    assert (i0, i0 + 1) not in sa and (i0, i0 + 2) in sa


def test_pairs_are_symmetric():
    rng = np.random.default_rng(7)
    pts = rng.uniform(0, 0.05, (200, 2))
    pi, pj = O.pairs(pts, 0.006)
    s = _as_set(pi, pj)
    assert all((j, i) in s for i, j in s)


def test_f32_predicate_agrees_with_f64_away_from_the_cutoff():
    rng = np.random.default_rng(11)
    n = 300
    pts = rng.uniform(-0.05, 0.05, (n, 2)).astype(np.float32)
    R = np.float32(0.008)
    a = _as_set(*O.pairs_f32(pts, R))
    b = _as_set(*O.pairs(pts.astype(np.float64), float(R), use_cells=False))
    d = np.sqrt(((pts[:, None, :].astype(np.float64) - pts[None, :, :]) ** 2).sum(-1))
    near_cut = np.abs(d - float(R)) < 1e-6 * float(R)
    diff = a ^ b
    assert all(near_cut[i, j] for i, j in diff)
