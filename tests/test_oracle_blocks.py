"""Pins of the oracle's individual power-of-two time steps (Sec. 2 and 2.1).

* With one level for every particle the block scheme is the global Heun
  step: the results equal orc_evolve bit for bit (same operations in the
  same order), on an ideal and a stabilised set.
* On a set whose resolution varies (lambda between 0.9 and 1.6 spacings)
  the particles spread over several levels, the levels obey the neighbor
  limiter, the scheme evaluates fewer particles than global steps of the
  smallest size, and it tracks the global solution to second order: halving
  the Courant number cuts the difference from a fine global reference about
  fourfold.
"""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth


graded_set = synth.graded_lattice


@pytest.mark.parametrize("stab", [None, (0.3, 0.3, 0.3)])
def test_one_level_is_the_global_step(stab):
    c = synth.cp_alfven(8)
    dt = 0.8 * oracle.courant_dt(c["q"], c["lam"], 0.3, stab=stab)
    p1, q1, s1, lev, stats = oracle.evolve_blocks(c["pos"], c["lam"], c["q"], dt, 3, cfl=0.3,
                                                  stab=stab)
    p0, q0, s0 = oracle.evolve(c["pos"], c["lam"], c["q"], dt, 3, stab=stab)
    assert np.all(lev == 0)
    assert np.array_equal(p1, p0) and np.array_equal(q1, q0) and np.array_equal(s1, s0)
    n = c["lam"].shape[0]
    assert stats[0] == 3 and stats[1] == 2 * 3 * n  # two evaluations per step


def _levels(c, dt_max, cfl=0.3):
    """Courant levels and the limiter's fixed point at the initial state."""
    gam = 5.0 / 3.0
    q = c["q"]
    cf = np.sqrt((gam * (gam - 1) * q[7] + (q[4:7] ** 2).sum(0)) / q[0])
    dtc = cfl * (c["lam"] / cf)
    k = np.zeros(len(dtc), int)
    for i, d in enumerate(dtc):
        while k[i] < 20 and not (dt_max / 2 ** k[i] <= d):
            k[i] += 1
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    while True:
        kn = k.copy()
        for i in range(len(k)):
            kn[i] = max(kn[i], max(k[j] for j in idx[off[i]:off[i + 1]]) - 1)
        if np.array_equal(kn, k):
            return k
        k = kn


def test_graded_set_uses_several_levels_under_the_limiter():
    c = graded_set(wave=False)
    gam = 5.0 / 3.0
    cf = np.sqrt((gam * (gam - 1) * c["q"][7] + (c["q"][4:7] ** 2).sum(0)) / c["q"][0])
    dt_max = np.median(0.3 * c["lam"] / cf)   # about half the particles on level 0
    k0 = _levels(c, dt_max)
    assert np.bincount(k0).min() > 0.2 * len(k0)
    p, q, st, lev, stats = oracle.evolve_blocks(c["pos"], c["lam"], c["q"], dt_max, 2)
    assert np.all(st == 0) and len(np.unique(lev)) >= 2
    # the final levels obey the limiter against the final neighbor lists,
    # up to the one step the neighbors took since
    off, idx = oracle.neighbors(p, c["lam"])
    gap = max(int(lev[idx[off[i]:off[i + 1]]].max() - lev[i]) for i in range(len(lev)))
    assert gap <= 2
    n = len(lev)
    fine_evals = 2 * n * 2 * 2 ** int(lev.max())
    assert stats[1] < 0.9 * fine_evals


def test_graded_sound_wave_converges_to_the_global_solution():
    c = graded_set(side=8)
    # sound speed 1: particle i's Courant step is cfl lambda_i; a dt_max of
    # four median steps puts the median particle on a level boundary
    dt_max = 4 * np.median(0.3 * c["lam"])
    T = 2 * dt_max
    nf = int(np.ceil(T / (0.3 * c["lam"].min() / 16)))
    pr, qr, _ = oracle.evolve(c["pos"], c["lam"], c["q"], T / nf, nf)   # fine global reference
    diffs = []
    for cfl in (0.3, 0.15):   # the levels follow the Courant limit, so shrink cfl
        p, q, st, lev, stats = oracle.evolve_blocks(c["pos"], c["lam"], c["q"], dt_max, 2,
                                                    cfl=cfl)
        assert np.all(st == 0) and np.bincount(lev)[lev.min():].min() > 0.1 * len(lev)
        diffs.append(np.abs(q - qr).max() / 1e-3)
    ratio = diffs[0] / diffs[1]
    print("block-step difference from the fine global solution", diffs, "ratio", ratio)
    assert ratio > 3.0
