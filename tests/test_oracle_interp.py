"""Pins of the oracle's interpolating fit and div-B diagnostic.

* Interpolating fit (the paper's tests use interpolating fits, per its
  acknowledgements): the 19 monomials without the constant, so the local
  polynomial passes through the particle's own value.  Cubic fields are still
  reproduced exactly; an independent weighted least-squares solve (numpy
  lstsq) without the constant column agrees on non-polynomial data; the
  reverse mode agrees with complex-step derivatives.
* lambda (div B) / |B| (Sec. 3.3): zero to roundoff for a divergence-free
  cubic field (the curl of a quartic potential), the closed form for a linear
  field; the binned mean against numpy's bincount.
"""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from test_oracle_mls import _analytic


def test_interpolating_fit_reproduces_cubics():
    c = synth.cubic_set(pin=True)
    off, idx = oracle.neighbors(c["pos"], c["lam"], periodic=c["periodic"])
    d1, d2, st = oracle.mls_derivs(c["pos"], c["lam"], off, idx, c["q"], periodic=c["periodic"],
                                   fit=1)
    ok = st == 0
    rf = 2.3 * c["lam"]
    inner = ok & np.all((c["pos"] > rf) & (c["pos"] < 1 - rf), axis=0)
    g1, g2 = _analytic(c["pos"], c["coef"], c["exponents"])
    for a, b in ((d1, g1), (d2, g2)):
        assert np.abs(a[:, :, inner] - b[:, :, inner]).max() < 1e-12 * np.abs(b).max()


def _lstsq19(pos, lam, i, nb, f):
    d = pos[:, nb] - pos[:, [i]]
    d = np.where(d > 0.5, d - 1.0, np.where(d < -0.5, d + 1.0, d))
    xi = d / lam[i]
    w = (1 - (d * d).sum(0) / (2.3 * lam[i]) ** 2) ** 3
    ex = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1),
          (0, 0, 2), (3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0),
          (0, 2, 1), (0, 1, 2), (0, 0, 3)]
    P = np.stack([xi[0] ** e[0] * xi[1] ** e[1] * xi[2] ** e[2] for e in ex], axis=1)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(sw[:, None] * P, sw * (f[nb] - f[i]), rcond=None)
    return coef[0:3] / lam[i], np.array([2 * coef[3], coef[4], coef[5], 2 * coef[6], coef[7],
                                         2 * coef[8]]) / lam[i] ** 2


def test_interpolating_fit_matches_independent_lstsq():
    c = synth.random_cloud(2500, seed=81, lam_range=(0.07, 0.1))
    pos, lam, q = c["pos"], c["lam"], c["q"]
    rng = np.random.default_rng(82)
    q = q + 0.01 * rng.normal(size=q.shape)    # noise: the two fits must differ
    off, idx = oracle.neighbors(pos, lam)
    d1, d2, st = oracle.mls_derivs(pos, lam, off, idx, q, fit=1)
    f1, _, _ = oracle.mls_derivs(pos, lam, off, idx, q, fit=0)
    assert np.abs(d1 - f1).max() > 1e-3 * np.abs(f1).max()
    for i in range(0, 2500, 113):
        assert st[i] == 0
        nb = idx[off[i]:off[i + 1]]
        for f in (0, 3, 6):
            g1, g2 = _lstsq19(pos, lam, i, nb, q[f])
            assert np.allclose(d1[f, :, i], g1, rtol=1e-9, atol=1e-9)
            assert np.allclose(d2[f, :, i], g2, rtol=1e-8, atol=1e-7)


def test_interpolating_fit_reverse_mode_complex_step():
    rng = np.random.default_rng(83)
    pos = synth.jittered_lattice(8, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1.0 / 8) * rng.uniform(0.95, 1.05, n)
    q = np.zeros((8, n))
    q[0] = 1.0 + 0.2 * rng.uniform(-1, 1, n)
    q[1:7] = 0.3 * rng.uniform(-1, 1, (6, n))
    q[7] = 1.5 + 0.2 * rng.uniform(-1, 1, n)
    gbar = rng.normal(size=(8, n))
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, st = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, fit=1)
    assert np.all(st == 0)
    for trial in range(3):
        dpos = rng.normal(size=pos.shape) if trial != 1 else None
        dq = rng.normal(size=q.shape) if trial != 2 else None
        _, rdir, _ = oracle.mhd_rhs_cstep(pos, lam, off, idx, q, dpos=dpos, dq=dq, fit=1)
        lhs = np.sum(gbar * rdir)
        rhs = (np.sum(qb * dq) if dq is not None else 0.0) + \
              (np.sum(pb * dpos) if dpos is not None else 0.0)
        assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0), (trial, lhs, rhs)


def _quartic_curl(pos, rng):
    """B = curl A for A with random quartic components: a divergence-free cubic
    field, returned with nothing else (its divergence is zero identically)."""
    d = pos - 0.5
    ex = [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c == 4]
    co = rng.uniform(-1, 1, size=(3, len(ex)))

    def dmono(e, axis):
        if e[axis] == 0:
            return np.zeros(pos.shape[1])
        e2 = list(e)
        e2[axis] -= 1
        return e[axis] * d[0] ** e2[0] * d[1] ** e2[1] * d[2] ** e2[2]

    def dA(comp, axis):
        return sum(co[comp, k] * dmono(e, axis) for k, e in enumerate(ex))

    return np.stack([dA(2, 1) - dA(1, 2), dA(0, 2) - dA(2, 0), dA(1, 0) - dA(0, 1)])


def test_divb_zero_for_solenoidal_cubic_field():
    c = synth.cubic_set(pin=True)
    rng = np.random.default_rng(84)
    q = np.ones((8, c["pos"].shape[1]))
    q[4:7] = np.array([2.0, -1.0, 1.5])[:, None] + 0.3 * _quartic_curl(c["pos"], rng)
    off, idx = oracle.neighbors(c["pos"], c["lam"], periodic=c["periodic"])
    for fit in (0, 1):
        out, st = oracle.divb_norm(c["pos"], c["lam"], off, idx, q, periodic=c["periodic"],
                                   fit=fit)
        rf = 2.3 * c["lam"]
        inner = (st == 0) & np.all((c["pos"] > rf) & (c["pos"] < 1 - rf), axis=0)
        d1, _, _ = oracle.mls_derivs(c["pos"], c["lam"], off, idx, q[4:7], periodic=c["periodic"])
        scale = c["lam"].max() * np.nanmax(np.abs(d1)) / np.sqrt((q[4:7] ** 2).sum(0)).min()
        assert inner.sum() > 1000 and np.abs(out[inner]).max() < 1e-12 * scale


def test_divb_linear_field_closed_form():
    c = synth.random_cloud(1500, seed=85, lam_range=(0.08, 0.1))
    pos = c["pos"]
    a = np.array([0.7, -0.2, 0.4])
    q = np.ones((8, pos.shape[1]))
    q[4:7] = np.array([1.0, 2.0, -0.5])[:, None] + a[:, None] * (pos - 0.5)
    # periodic box with a linear field is discontinuous at the seams: open box
    off, idx = oracle.neighbors(pos, c["lam"], periodic=(0, 0, 0))
    out, st = oracle.divb_norm(pos, c["lam"], off, idx, q, periodic=(0, 0, 0))
    ok = st == 0
    want = c["lam"] * a.sum() / np.sqrt((q[4:7] ** 2).sum(0))
    assert ok.mean() > 0.8
    assert np.allclose(out[ok], want[ok], rtol=1e-8, atol=0)
    assert np.all(np.isnan(out[~ok]))


def test_bin_mean_against_bincount():
    rng = np.random.default_rng(86)
    x = rng.uniform(-0.1, 1.1, 5000)
    v = rng.normal(size=5000)
    v[::37] = np.nan
    mean, cnt = oracle.bin_mean(x, v, 0.0, 0.125, 8)
    b = np.floor(x / 0.125).astype(int)
    keep = (b >= 0) & (b < 8) & np.isfinite(v)
    s = np.bincount(b[keep], weights=v[keep], minlength=8)
    k = np.bincount(b[keep], minlength=8)
    assert np.array_equal(cnt, k)
    assert np.allclose(mean, s / k, rtol=1e-12)
    e, ce = oracle.bin_mean(x, v, 5.0, 1.0, 3)   # all outside: empty bins are NaN
    assert np.all(ce == 0) and np.all(np.isnan(e))
