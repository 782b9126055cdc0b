"""Pins of the oracle's non-ideal stabilisers (Sec. 2: a bulk viscosity in a
grid-scale and an adaptive coefficient field, and a diffusive div-B term in
the induction equation; App. A: the viscous term and its damping rate).

* cubic polynomial fields in an open box: the MLS second derivatives are
  exact, so the added terms equal their closed forms built from the
  polynomials' analytic derivatives (grad div V, grad div B, (div V)^2);
* App. A: the viscous acceleration of a sound wave is -zeta k^2 V (the sign
  that damps), converging with resolution; evolved over half a period, the
  wave decays at the rate zeta k^2 / 2 and oscillates at
  sqrt(c^2 k^2 - zeta^2 k^4 / 4);
* the reverse mode with stabilisers against complex-step derivatives;
* zero coefficients reproduce ideal MHD bit for bit; the Courant step.
"""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth

STAB = (0.4, 0.9, 0.3)


def _poly_derivs(coef, expo, pos, center=(0.5, 0.5, 0.5)):
    """Values, gradients (nf,3,n) and Hessians (nf,3,3,n) of the cubic fields."""
    d = pos - np.asarray(center)[:, None]
    nf = coef.shape[0]
    n = pos.shape[1]
    grad = np.zeros((nf, 3, n))
    hess = np.zeros((nf, 3, 3, n))

    def mono(e):
        if min(e) < 0:
            return np.zeros(n)
        return d[0] ** e[0] * d[1] ** e[1] * d[2] ** e[2]

    for k, e in enumerate(expo):
        for a in range(3):
            ea = list(e)
            ea[a] -= 1
            grad[:, a] += coef[:, k:k + 1] * (e[a] * mono(ea))[None]
            for b in range(3):
                eb = list(ea)
                eb[b] -= 1
                fac = e[a] * (e[b] - (1 if a == b else 0))
                hess[:, a, b] += coef[:, k:k + 1] * (fac * mono(eb))[None]
    return grad, hess


def test_polynomial_fields_match_closed_form():
    rng = np.random.default_rng(61)
    side = 10
    pos = synth.jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side)
    L, per = (1.0, 1.0, 1.0), (0, 0, 0)
    poly, coef, expo = synth.cubic_poly_fields(pos, 6, rng)
    gpoly, hpoly = _poly_derivs(coef, expo, pos)
    gamma = 5.0 / 3.0
    q = np.zeros((8, n))
    q[0] = 1.0 + 0.3 * (pos[0] - 0.5)          # linear: grad rho exact
    q[1:4] = 0.2 * poly[0:3]
    q[4:7] = np.array([0.4, -0.3, 0.8])[:, None] + 0.2 * poly[3:6]
    q[7] = 1.2
    off, idx = oracle.neighbors(pos, lam, L=L, periodic=per)
    r0, _, st0 = oracle.mhd_rhs(pos, lam, off, idx, q, L=L, periodic=per, gamma=gamma)
    r1, _, st1 = oracle.mhd_rhs(pos, lam, off, idx, q, L=L, periodic=per, gamma=gamma, stab=STAB)
    assert np.array_equal(st0, st1)
    ok = st1 == 0           # box corners see too few neighbors
    assert ok.sum() > 0.9 * n
    # closed form of the added terms from the polynomials' own derivatives
    hv = 0.2 * hpoly[0:3]
    hb = 0.2 * hpoly[3:6]
    gdV = np.einsum("babn->an", hv)   # d_a div V = sum_b d_a d_b V_b
    gdB = np.einsum("babn->an", hb)
    divV = 0.2 * (gpoly[0, 0] + gpoly[1, 1] + gpoly[2, 2])
    rho, sig, B = q[0], q[7], q[4:7]
    cf = np.sqrt((gamma * (gamma - 1) * sig + (B * B).sum(0)) / rho)
    s2 = (lam * 0.3 / rho) ** 2
    zeta = lam * cf * (STAB[0] + STAB[1] * np.minimum(1.0, s2))
    eta = STAB[2] * lam * cf
    want = np.zeros((8, n))
    want[1:4] = zeta * gdV
    want[4:7] = eta * gdB
    want[7] = rho * zeta * divV ** 2
    got = (r1 - r0)[:, ok]
    want = want[:, ok]
    for f in range(8):
        scale = max(np.abs(want[f]).max(), 1e-3 * np.abs(want).max())
        assert np.abs(got[f] - want[f]).max() <= 1e-8 * scale, f
    # the terms are not trivially small, and grad div differs from the Laplacian
    lapV = np.einsum("abbn->an", hv)
    assert np.abs(gdV - lapV).max() > 0.1 * np.abs(gdV).max()
    assert np.abs(want[1:4]).max() > 1e-2 and np.abs(want[7]).max() > 1e-4


def _sound(side):
    c = synth.linear_wave("sound", side)
    k = 2 * np.pi
    return c, k


def test_sound_wave_viscous_acceleration_converges():
    """App. A: grad(zeta div V) = -zeta k^2 V for the longitudinal wave, with
    zeta = visc_grid lambda c (c = 1; the wave's density gradient is O(eps), so
    the adaptive part is negligible)."""
    errs = []
    for side in (8, 16):
        c, k = _sound(side)
        off, idx = oracle.neighbors(c["pos"], c["lam"])
        r0, _, _ = oracle.mhd_rhs(c["pos"], c["lam"], off, idx, c["q"])
        r1, _, _ = oracle.mhd_rhs(c["pos"], c["lam"], off, idx, c["q"], stab=(0.5, 0.5, 0.0))
        zeta = 0.5 * c["lam"][0]
        want = -zeta * k * k * (c["q"][1] - c["q0"][1])
        got = r1[1] - r0[1]
        errs.append(np.abs(got - want).max() / np.abs(want).max())
        # rho and B are untouched (no div-B diffusion here); the transverse
        # components are the fit's truncation error of d_x d_y V_x
        assert np.array_equal(r1[0], r0[0]) and np.array_equal(r1[4:7], r0[4:7])
        assert np.abs(r1[2:4] - r0[2:4]).max() <= 0.1 * np.abs(want).max()
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 0.05 and order > 1.5, (errs, order)


def _vx_fit(pos, vx, eps, k):
    a = (vx * np.cos(k * pos[0])).sum() / (np.cos(k * pos[0]) ** 2).sum() / eps
    b = (vx * np.sin(k * pos[0])).sum() / (np.sin(k * pos[0]) ** 2).sum() / eps
    return np.hypot(a, b), np.arctan2(b, a)


def test_sound_wave_decays_at_appendix_a_rate():
    side, cg, t_end = 16, 0.5, 0.5
    c, k = _sound(side)
    zeta = cg * c["lam"][0]
    rate = zeta * k * k / 2
    omega_r = np.sqrt(k * k - zeta ** 2 * k ** 4 / 4)
    stab = (cg, 0.0, 0.0)
    dt = oracle.courant_dt(c["q"], c["lam"], 0.2, stab=stab)
    nsteps = int(np.ceil(t_end / dt))
    res = {}
    for s in (None, stab):
        pos, q, st = oracle.evolve(c["pos"], c["lam"], c["q"], t_end / nsteps, nsteps, stab=s)
        assert np.all(st == 0)
        res[s] = _vx_fit(pos, q[1], c["eps"] * c["R"][1], k)
    amp0, ph0 = res[None]
    amp1, ph1 = res[stab]
    measured = -np.log(amp1 / amp0) / t_end
    # V_x = eps e^{-rate t} cos(k x - omega_r t): the phase is omega_r t
    assert abs(measured / rate - 1) < 0.05, (measured, rate)
    assert abs(amp0 - 1) < 0.02
    assert abs(np.angle(np.exp(1j * (ph1 - omega_r * t_end)))) < 0.02 * omega_r * t_end


def _rand_set(side=8, seed=62):
    rng = np.random.default_rng(seed)
    pos = synth.jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side) * rng.uniform(0.95, 1.05, size=n)
    q = np.zeros((8, n))
    q[0] = 1.0 + 0.2 * rng.uniform(-1, 1, n)
    q[1:7] = 0.3 * rng.uniform(-1, 1, (6, n))
    q[7] = 1.5 + 0.2 * rng.uniform(-1, 1, n)
    return rng, pos, lam, q


def test_reverse_mode_with_stabilisers_complex_step():
    rng, pos, lam, q = _rand_set()
    n = pos.shape[1]
    gbar = rng.normal(size=(8, n))
    off, idx = oracle.neighbors(pos, lam)
    qb, pb, st = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, stab=STAB)
    assert np.all(st == 0)
    # the adaptive coefficient is unsaturated at some particles, saturated at none
    d1, _, _ = oracle.mhd_rhs(pos, lam, off, idx, q, stab=STAB)
    for trial in range(3):
        dpos = rng.normal(size=pos.shape) if trial != 1 else None
        dq = rng.normal(size=q.shape) if trial != 2 else None
        _, rdir, _ = oracle.mhd_rhs_cstep(pos, lam, off, idx, q, dpos=dpos, dq=dq, stab=STAB)
        lhs = np.sum(gbar * rdir)
        rhs = (np.sum(qb * dq) if dq is not None else 0.0) + \
              (np.sum(pb * dpos) if dpos is not None else 0.0)
        assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0), (trial, lhs, rhs)
    # and the stabilisers change the gradient
    qb0, pb0, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar)
    assert np.abs(qb - qb0).max() > 1e-2 * np.abs(qb0).max()


def test_adaptive_coefficient_saturates():
    """A density jump of order one across a smoothing length saturates the
    adaptive coefficient: doubling visc_adapt there doubles its share, and the
    reverse mode passes no gradient through the saturated sensor."""
    rng, pos, lam, q = _rand_set(seed=63)
    q[0] = np.where(pos[0] < 0.5, 1.0, 4.0) + 0.05 * rng.uniform(-1, 1, pos.shape[1])
    off, idx = oracle.neighbors(pos, lam)
    r_a, _, _ = oracle.mhd_rhs(pos, lam, off, idx, q, stab=(0.0, 0.5, 0.0))
    r_b, _, _ = oracle.mhd_rhs(pos, lam, off, idx, q, stab=(0.0, 1.0, 0.0))
    r_0, _, _ = oracle.mhd_rhs(pos, lam, off, idx, q)
    assert np.allclose(r_b - r_0, 2 * (r_a - r_0), rtol=1e-9, atol=1e-12)
    gbar = rng.normal(size=(8, pos.shape[1]))
    qb, pb, _ = oracle.mhd_rhs_adjoint(pos, lam, off, idx, q, gbar, stab=(0.2, 1.0, 0.1))
    dq = rng.normal(size=q.shape)
    _, rdir, _ = oracle.mhd_rhs_cstep(pos, lam, off, idx, q, dq=dq, stab=(0.2, 1.0, 0.1))
    lhs, rhs = np.sum(gbar * rdir), np.sum(qb * dq)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0)


def test_zero_coefficients_are_ideal_mhd():
    rng, pos, lam, q = _rand_set(seed=64)
    off, idx = oracle.neighbors(pos, lam)
    a = oracle.mhd_rhs(pos, lam, off, idx, q)
    b = oracle.mhd_rhs(pos, lam, off, idx, q, stab=(0.0, 0.0, 0.0))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_courant_step_with_stabilisers():
    rng, pos, lam, q = _rand_set(seed=65)
    q[1:4] = 0.0
    dt0 = oracle.courant_dt(q, lam, 0.3)
    dt1 = oracle.courant_dt(q, lam, 0.3, stab=STAB)
    assert dt1 == pytest.approx(dt0 / (1 + 2 * sum(STAB)), rel=1e-14)
