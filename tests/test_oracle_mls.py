"""Pins of the oracle's moving-least-squares derivatives (paper II, Sec. 2: a
local third-order polynomial fit over the sphere of radius 2.3 lambda_i).

* cubic polynomial fields are reproduced exactly, so their first and second
  derivatives come back to roundoff, for any positive weight;
* constant and linear special cases;
* an independent weighted least-squares solve (numpy lstsq) on non-polynomial
  data, with the weight reading w = (1 - q)^3 written out again here;
* the status paths: too few neighbors (1) and a singular (coplanar) sample (2).
"""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth


def _analytic(pos, coef, expo, center=0.5):
    d = pos - center
    n = pos.shape[1]
    nf = coef.shape[0]
    g1 = np.zeros((nf, 3, n))
    g2 = np.zeros((nf, 6, n))
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]

    def mono(e):
        if min(e) < 0:
            return np.zeros(n)
        return d[0] ** e[0] * d[1] ** e[1] * d[2] ** e[2]

    for k, e in enumerate(expo):
        e = list(e)
        for a in range(3):
            if e[a]:
                e2 = list(e)
                e2[a] -= 1
                g1[:, a] += coef[:, k:k + 1] * e[a] * mono(e2)[None]
        for s, (a, b) in enumerate(pairs):
            e2 = list(e)
            fa = e2[a]
            e2[a] -= 1
            fb = e2[b]
            e2[b] -= 1
            if fa > 0 and fb > 0:
                g2[:, s] += coef[:, k:k + 1] * fa * fb * mono(e2)[None]
    return g1, g2


@pytest.mark.parametrize("weight", [0, 1])
def test_cubic_fields_exact(weight):
    c = synth.cubic_set(pin=True)
    off, idx = oracle.neighbors(c["pos"], c["lam"], periodic=c["periodic"])
    d1, d2, st = oracle.mls_derivs(c["pos"], c["lam"], off, idx, c["q"],
                                   periodic=c["periodic"], weight=weight)
    ok = st == 0
    assert ok.sum() > 3900
    g1, g2 = _analytic(c["pos"], c["coef"], c["exponents"])
    # interior particles (whole sphere inside the open box) are well conditioned:
    # roundoff level; truncated spheres at the faces amplify roundoff more.
    rf = 2.3 * c["lam"]
    inner = ok & np.all((c["pos"] > rf) & (c["pos"] < 1 - rf), axis=0)
    for sel, tol in ((inner, 1e-12), (ok, 1e-7)):
        e1 = np.abs(d1[:, :, sel] - g1[:, :, sel]).max() / np.abs(g1[:, :, sel]).max()
        e2 = np.abs(d2[:, :, sel] - g2[:, :, sel]).max() / np.abs(g2[:, :, sel]).max()
        assert e1 < tol and e2 < tol, (e1, e2, tol)
    assert np.all(np.isnan(d1[:, :, ~ok]))


def test_constant_and_linear_fields():
    c = synth.cubic_set(pin=True)
    pos = c["pos"]
    off, idx = oracle.neighbors(pos, c["lam"], periodic=c["periodic"])
    a = np.array([0.3, -1.7, 2.2])
    fields = np.stack([np.full(pos.shape[1], 4.25), 1.5 + a @ pos])
    d1, d2, st = oracle.mls_derivs(pos, c["lam"], off, idx, fields, periodic=c["periodic"])
    ok = st == 0
    assert np.abs(d1[0][:, ok]).max() == 0.0 and np.abs(d2[0][:, ok]).max() == 0.0
    rf = 2.3 * c["lam"]
    inner = ok & np.all((pos > rf) & (pos < 1 - rf), axis=0)
    assert np.abs(d1[1][:, inner] - a[:, None]).max() < 1e-12
    assert np.abs(d1[1][:, ok] - a[:, None]).max() < 1e-9
    assert np.abs(d2[1][:, inner]).max() < 1e-10
    assert np.abs(d2[1][:, ok]).max() < 1e-7


def _weighted_lstsq(pos, lam, i, nb, f, L, periodic):
    d = pos[:, nb] - pos[:, [i]]
    for a in range(3):
        if periodic[a]:
            d[a] = np.where(d[a] > 0.5 * L[a], d[a] - L[a], np.where(d[a] < -0.5 * L[a], d[a] + L[a], d[a]))
    xi = d / lam[i]
    qq = (d * d).sum(0) / (2.3 * lam[i]) ** 2
    w = (1 - qq) ** 3
    ex = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0),
          (0, 1, 1), (0, 0, 2), (3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2),
          (0, 3, 0), (0, 2, 1), (0, 1, 2), (0, 0, 3)]
    P = np.stack([xi[0] ** e[0] * xi[1] ** e[1] * xi[2] ** e[2] for e in ex], axis=1)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(sw[:, None] * P, sw * (f[nb] - f[i]), rcond=None)
    return coef[1:4] / lam[i], np.array([2 * coef[4], coef[5], coef[6], 2 * coef[7], coef[8],
                                         2 * coef[9]]) / lam[i] ** 2


def test_matches_independent_weighted_lstsq():
    c = synth.random_cloud(2500, seed=21, lam_range=(0.07, 0.1))
    pos, lam, q = c["pos"], c["lam"], c["q"]
    off, idx = oracle.neighbors(pos, lam)
    d1, d2, st = oracle.mls_derivs(pos, lam, off, idx, q)
    for i in range(0, 2500, 97):
        assert st[i] == 0
        nb = idx[off[i]:off[i + 1]]
        for f in (1, 5, 7):
            g1, g2 = _weighted_lstsq(pos, lam, i, nb, q[f], c["L"], c["periodic"])
            assert np.allclose(d1[f, :, i], g1, rtol=1e-9, atol=1e-11)
            assert np.allclose(d2[f, :, i], g2, rtol=1e-8, atol=1e-9)


def test_status_too_few_neighbors():
    c = synth.random_cloud(300, seed=22, lam_range=(0.02, 0.03))  # ~1 neighbor each
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    d1, d2, st = oracle.mls_derivs(c["pos"], c["lam"], off, idx, c["q"])
    small = np.diff(off) < 20
    assert small.all() and np.all(st == 1)
    assert np.all(np.isnan(d1)) and np.all(np.isnan(d2))


def test_status_singular_coplanar():
    # every particle in the plane z = 0.5: the z-monomials vanish on the sample
    rng = np.random.default_rng(23)
    n = 1500
    pos = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), np.full(n, 0.5)])
    lam = np.full(n, 0.04)
    off, idx = oracle.neighbors(pos, lam)
    assert np.diff(off).min() >= 20
    d1, d2, st = oracle.mls_derivs(pos, lam, off, idx, np.ones((1, n)))
    assert np.all(st == 2)
    assert np.all(np.isnan(d1))
