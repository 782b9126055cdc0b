"""Pins of the oracle's neighbor search (paper II, Sec. 2 and 2.1: a strict,
fixed-radius, non-mutual sphere of radius 2.3 lambda_i about each particle).

* a hand-derived tiny example (tests/golden/neighbors_tiny.json) with the
  strict-inequality tie, the periodic wrap, a non-periodic axis and a
  non-mutual pair;
* an independent library routine (scipy's periodic k-d tree) on random sets;
* the closed-form expected count 1 + (N-1) (4/3) pi r^3 / V for uniform
  random points (one particle per lambda^3 gives 50.97, Sec. 2);
* symmetry of membership when all radii are equal.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "neighbors_tiny.json")


def _tiny():
    g = json.load(open(GOLD))
    r0 = 2.3 * 0.5
    sub = {"r0": r0, "r0-": float(np.nextafter(r0, 0.0))}
    x = [sub[v] if isinstance(v, str) else v for v in g["x"]]
    pos = np.array([x, g["y"], g["z"]], dtype=np.float64)
    return g, pos, np.array(g["lambda"])


def _rows(off, idx):
    return [list(idx[off[i]:off[i + 1]]) for i in range(len(off) - 1)]


def test_golden_tiny_rows():
    g, pos, lam = _tiny()
    off, idx = oracle.neighbors(pos, lam, L=g["L"], periodic=g["periodic"])
    assert _rows(off, idx) == g["rows"]


def test_row_subset_matches_full():
    c = synth.random_cloud(700, seed=11)
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    rows = np.array([5, 0, 699, 123, 5])
    off2, idx2 = oracle.neighbors(c["pos"], c["lam"], rows=rows)
    full = _rows(off, idx)
    assert _rows(off2, idx2) == [full[r] for r in rows]


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0), (1, 0, 1)])
def test_matches_scipy_kdtree(periodic):
    from scipy.spatial import cKDTree
    c = synth.random_cloud(3000, seed=12, box=(1.0, 0.8, 1.2), lam_range=(0.05, 0.1),
                           periodic=periodic)
    pos, lam = c["pos"], c["lam"]
    L = np.array(c["L"])
    off, idx = oracle.neighbors(pos, lam, L=L, periodic=periodic)
    # scipy: per-axis periodicity is given by boxsize; open axes get a box far larger
    # than the data so no image ever comes in range.
    boxsize = np.where(np.array(periodic) == 1, L, 1e6)
    tree = cKDTree(pos.T, boxsize=boxsize)
    for i in range(0, pos.shape[1], 7):
        got = list(idx[off[i]:off[i + 1]])
        ref = sorted(tree.query_ball_point(pos[:, i], 2.3 * lam[i]))
        assert got == ref, i


def test_mean_count_closed_form():
    # uniform random points in a periodic box: every other point falls inside a
    # sphere of volume v with probability v / V, so E[n_i] = 1 + (N - 1) v / V.
    n = 40000
    lam = (1.0 / n) ** (1.0 / 3.0)  # one particle per lambda^3
    rng = np.random.default_rng(13)
    pos = rng.uniform(0.0, 1.0, size=(3, n))
    off, idx = oracle.neighbors(pos, np.full(n, lam))
    counts = np.diff(off)
    v = 4.0 / 3.0 * math.pi * (2.3 * lam) ** 3
    expect = 1.0 + (n - 1) * v
    assert abs(n * v - 50.97) < 0.01  # (4/3) pi 2.3^3 particles per sphere volume
    # standard error of the mean is below sqrt(expect / n) * 2 (pair correlations)
    se = 2.0 * math.sqrt(expect / n)
    assert abs(counts.mean() - expect) < 4 * se, (counts.mean(), expect)


def test_jittered_lattice_count_near_expectation():
    c = synth.cubic_set()
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    counts = np.diff(off)
    # self plus ~50.97 others; the jittered lattice is not Poisson, so only a loose band
    assert 36 <= counts.min() and counts.max() <= 68
    assert abs(counts.mean() - 51.97) < 1.5


def test_symmetric_when_radii_equal():
    c = synth.random_cloud(1500, seed=14, lam_range=(0.09, 0.09))
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    pairs = set()
    for i in range(len(off) - 1):
        for j in idx[off[i]:off[i + 1]]:
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)


def test_not_mutual_with_unequal_radii():
    c = synth.random_cloud(1500, seed=15, lam_range=(0.04, 0.12))
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    pos, lam = c["pos"], c["lam"]
    one_way = 0
    for i in range(0, 1500, 3):
        for j in idx[off[i]:off[i + 1]]:
            if i not in idx[off[j]:off[j + 1]]:
                one_way += 1
                assert lam[j] < lam[i]  # only the smaller sphere can miss the pair
    assert one_way > 0


def test_self_always_included():
    c = synth.random_cloud(500, seed=16, lam_range=(0.001, 0.002))
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    for i in range(500):
        assert i in idx[off[i]:off[i + 1]]
