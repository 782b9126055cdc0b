"""Pins of the oracle's reverse-mode gradient of a scalar of the MHD time
derivatives with respect to field values and positions (neighbor sets held
fixed).

* complex-step directional derivatives of the oracle's forward map (h = 1e-30,
  exact to roundoff, an independent forward-mode computation) along random
  directions and along single coordinates;
* central finite differences with h = 1e-6 on the real forward map, with the
  neighbor sets rebuilt at every perturbed state;
* the sampled gradient (any n) equals the full gradient.
"""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth


def _set(side=8, seed=41):
    rng = np.random.default_rng(seed)
    pos = synth.jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side) * rng.uniform(0.95, 1.05, size=n)
    q = np.zeros((8, n))
    q[0] = 1.0 + 0.2 * rng.uniform(-1, 1, n)
    q[1:7] = 0.3 * rng.uniform(-1, 1, (6, n))
    q[7] = 1.5 + 0.2 * rng.uniform(-1, 1, n)
    gbar = rng.normal(size=(8, n))
    xbar = rng.normal(size=(3, n))
    return pos, lam, q, gbar, xbar


def test_complex_step_directions():
    pos, lam, q, gbar, xbar = _set()
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, st = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, xbar)
    assert np.all(st == 0)
    rng = np.random.default_rng(42)
    for trial in range(4):
        dpos = rng.normal(size=pos.shape) if trial != 1 else None
        dq = rng.normal(size=q.shape) if trial != 2 else None
        _, rdir, _ = oracle.mhd_rhs_cstep(pos, lam, off, idx, q, dpos=dpos, dq=dq)
        # d/dt of sum gbar.rhs + xbar.dxdt with dxdt = V
        lhs = np.sum(gbar * rdir) + (np.sum(xbar * dq[1:4]) if dq is not None else 0.0)
        rhs = (np.sum(qb * dq) if dq is not None else 0.0) + \
              (np.sum(pb * dpos) if dpos is not None else 0.0)
        assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (trial, lhs, rhs)


def test_complex_step_coordinates():
    pos, lam, q, gbar, _ = _set(seed=43)
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, st = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar)
    n = pos.shape[1]
    rng = np.random.default_rng(44)
    for _ in range(12):
        j = int(rng.integers(n))
        if rng.uniform() < 0.5:
            a = int(rng.integers(3))
            dpos = np.zeros_like(pos)
            dpos[a, j] = 1.0
            _, rdir, _ = oracle.mhd_rhs_cstep(pos, lam, off, idx, q, dpos=dpos)
            ref, got = np.sum(gbar * rdir), pb[a, j]
        else:
            f = int(rng.integers(8))
            dq = np.zeros_like(q)
            dq[f, j] = 1.0
            _, rdir, _ = oracle.mhd_rhs_cstep(pos, lam, off, idx, q, dq=dq)
            ref, got = np.sum(gbar * rdir), qb[f, j]
        assert abs(got - ref) <= 1e-11 * max(abs(ref), 1e-3), (got, ref)


def test_central_differences():
    pos, lam, q, gbar, _ = _set(seed=45)
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar)
    n = pos.shape[1]
    h = 1e-6

    def loss(p2, q2):
        o2, i2 = oracle.neighbors(p2, lam)
        r, _, _ = oracle.mhd_rhs(p2, lam, o2, i2, q2)
        return r

    rng = np.random.default_rng(46)
    for _ in range(8):
        j = int(rng.integers(n))
        a = int(rng.integers(3))
        pp, pm = pos.copy(), pos.copy()
        pp[a, j] += h
        pm[a, j] -= h
        fd = np.sum(gbar * (loss(pp, q) - loss(pm, q))) / (2 * h)
        assert abs(fd - pb[a, j]) <= 1e-6 * max(abs(pb[a, j]), 1.0), (fd, pb[a, j])
        f = int(rng.integers(8))
        qp, qm = q.copy(), q.copy()
        qp[f, j] += h
        qm[f, j] -= h
        fd = np.sum(gbar * (loss(pos, qp) - loss(pos, qm))) / (2 * h)
        assert abs(fd - qb[f, j]) <= 1e-6 * max(abs(qb[f, j]), 1.0), (fd, qb[f, j])


def test_sampled_equals_full():
    pos, lam, q, gbar, xbar = _set(seed=47)
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, xbar)
    samples = np.array([0, 17, 255, 511, 300])
    qs, ps = oracle.adjoint_sampled(pos, lam, q, gbar, samples, dxdt_bar=xbar)
    assert np.allclose(qs, qb[:, samples], rtol=1e-12, atol=1e-12)
    assert np.allclose(ps, pb[:, samples], rtol=1e-12, atol=1e-12)


def test_failed_particles_pass_no_gradient():
    pos, lam, q, gbar, _ = _set(seed=48)
    lam = lam.copy()
    lam[5] = 0.02  # a tiny sphere: too few neighbors, NaN outputs
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, st = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar)
    assert st[5] == 1 and np.all(np.isfinite(qb)) and np.all(np.isfinite(pb))
    g2 = gbar.copy()
    g2[:, 5] = 0.0
    qb2, pb2, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, g2)
    assert np.array_equal(qb, qb2) and np.array_equal(pb, pb2)


def _restrict(off, idx, rows):
    """The CSR lists of the given rows only, in that order."""
    counts = np.array([off[r + 1] - off[r] for r in rows], np.int64)
    roff = np.concatenate([[0], np.cumsum(counts)])
    ridx = np.concatenate([idx[off[r]:off[r + 1]] for r in rows]).astype(np.int32)
    return roff, ridx


def test_rows_all_equals_full():
    # every owner row listed in order: the same sums in the same order as the
    # full reverse mode, so the results are equal bit for bit
    pos, lam, q, gbar, xbar = _set(seed=49)
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, xbar)
    rows = np.arange(lam.shape[0])
    qr, pr = oracle.adjoint_rows(pos, lam, off, idx, q, gbar, rows, dxdt_bar=xbar)
    assert np.array_equal(qr, qb) and np.array_equal(pr, pb)


@pytest.mark.parametrize("stab", [None, (0.5, 0.5, 0.5)])
def test_rows_partition_sums_to_full(stab):
    # the reverse mode is a sum over owners: two disjoint row sets, listed in
    # shuffled order with their own restricted lists, add up to the full
    # gradient (an owner paired with another owner's list, or a neighbor entry
    # indexed through the wrong row, breaks this)
    pos, lam, q, gbar, xbar = _set(seed=50)
    n = lam.shape[0]
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, xbar, stab=stab)
    perm = np.random.default_rng(51).permutation(n)
    parts = (perm[: n // 3], perm[n // 3:])
    qs, ps = np.zeros_like(qb), np.zeros_like(pb)
    for rows in parts:
        roff, ridx = _restrict(off, idx, rows)
        qr, pr = oracle.adjoint_rows(pos, lam, roff, ridx, q, gbar, rows, dxdt_bar=xbar,
                                     stab=stab)
        qs += qr
        ps += pr
    assert np.abs(qs - qb).max() <= 1e-12 * np.abs(qb).max()
    assert np.abs(ps - pb).max() <= 1e-12 * np.abs(pb).max()
    # one part alone is not the whole gradient
    roff, ridx = _restrict(off, idx, parts[0])
    q0, _ = oracle.adjoint_rows(pos, lam, roff, ridx, q, gbar, parts[0], dxdt_bar=xbar,
                                stab=stab)
    assert np.abs(q0 - qb).max() > 1e-3 * np.abs(qb).max()
