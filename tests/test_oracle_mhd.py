"""Pins of the oracle's ideal-MHD time derivatives (paper II, Sec. 2; the
evolution equations of App. A with zero bulk viscosity).

* App. A linear eigenmodes: for delta q = eps R cos(k.x) the exact time
  derivative at t = 0 is eps omega R sin(k.x) (fast magnetosonic wave of the
  rhs benchmark set, plus the sound and shear Alfven waves of Sec. 3.1);
  the MLS answer converges to it as lambda shrinks;
* the circularly polarized Alfven wave of Sec. 3.2 is an exact nonlinear
  solution with closed-form time derivatives;
* Galilean invariance (Sec. 4.2: only Galilean-invariant quantities enter),
  axis permutation and periodic translation.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth


def _run(c, q=None, pos=None):
    pos = c["pos"] if pos is None else pos
    q = c["q"] if q is None else q
    off, idx = oracle.neighbors(pos, c["lam"], L=c["L"], periodic=c["periodic"])
    return oracle.mhd_rhs(pos, c["lam"], off, idx, q, L=c["L"], periodic=c["periodic"],
                          gamma=c["gamma"])


def test_fast_mode_satisfies_appendix_a_relations():
    # Fourier form of the linearized equations of App. A (zero viscosity):
    #   omega rho = rho0 k.V ;  omega P = gamma P0 k.V ;
    #   omega B = (k.V) B0 - (k.B0) V ;  omega rho0 V = k P - (k x B) x B0
    omega, R = synth.fast_mode(P0=1.0)
    k = np.array([2 * math.pi, 0, 0])
    B0 = np.array(synth.B0_WAVE)
    rho, V, B, sig = R[0], R[1:4], R[4:7], R[7]
    P = (synth.GAMMA - 1) * sig
    assert abs(omega * rho - k @ V) < 1e-12
    assert abs(omega * P - synth.GAMMA * (k @ V)) < 1e-12
    assert np.allclose(omega * B, (k @ V) * B0 - (k @ B0) * V, atol=1e-12)
    assert np.allclose(omega * V, k * P - np.cross(np.cross(k, B), B0), atol=1e-12)
    # fast speed exceeds both the sound and the Alfven speed
    assert omega / (2 * math.pi) > max(math.sqrt(synth.GAMMA), math.sqrt(B0 @ B0))


def _wave_error(side, B0, P0=1.0, eps=1e-6, seed=31):
    rng = np.random.default_rng(seed)
    pos = synth.jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    sigma0 = P0 / (synth.GAMMA - 1)
    omega, R = synth.fast_mode(B0=B0, P0=P0)
    q = synth.wave_background(n, 1.0, sigma0, B0=B0)
    q += eps * R[:, None] * np.cos(2 * math.pi * pos[0])[None]
    c = dict(pos=pos, lam=np.full(n, 1.0 / side), q=q, L=(1, 1, 1), periodic=(1, 1, 1),
             gamma=synth.GAMMA)
    rhs, dxdt, st = _run(c)
    assert np.all(st == 0)
    exact = eps * omega * R[:, None] * np.sin(2 * math.pi * pos[0])[None]
    return np.abs(rhs - exact).max() / (eps * omega * np.abs(R).max())


@pytest.mark.parametrize("B0,label", [((1.0, math.sqrt(2.0), 0.5), "fast"),
                                      ((0.0, 0.0, math.sqrt(3.0)), "magnetosonic"),
                                      ((0.0, 0.0, 0.0), "sound")])
def test_linear_wave_rhs_converges(B0, label):
    e16 = _wave_error(16, B0)
    e32 = _wave_error(32, B0)
    assert e16 < 2e-2 and e32 < 3e-3, (e16, e32)
    assert e16 / e32 > 4.0, (e16, e32)  # better than second order


def test_shear_alfven_wave_rhs():
    # B0 = x_hat, k = 2 pi x_hat: dV_y/dt = B0 dB_y/dx, dB_y/dt = B0 dV_y/dx
    side, eps = 16, 1e-6
    rng = np.random.default_rng(32)
    pos = synth.jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    q = synth.wave_background(n, 1.0, 1.0 / synth.GAMMA / (synth.GAMMA - 1), B0=(1, 0, 0))
    x = pos[0]
    q[2] += eps * np.cos(2 * math.pi * x)
    q[5] += -eps * np.cos(2 * math.pi * x)
    c = dict(pos=pos, lam=np.full(n, 1.0 / side), q=q, L=(1, 1, 1), periodic=(1, 1, 1),
             gamma=synth.GAMMA)
    rhs, _, st = _run(c)
    w = 2 * math.pi
    ex_vy = eps * w * np.sin(w * x)    # = B0 d(By)/dx
    ex_by = -eps * w * np.sin(w * x)   # = B0 d(Vy)/dx
    assert np.abs(rhs[2] - ex_vy).max() < 2e-2 * eps * w
    assert np.abs(rhs[5] - ex_by).max() < 2e-2 * eps * w
    for f in (0, 1, 3, 4, 6, 7):
        assert np.abs(rhs[f]).max() < 1e-2 * eps * w


def _cp_error(side):
    c = synth.cp_alfven(side)
    rhs, dxdt, st = _run(c)
    assert np.all(st == 0)
    x = c["pos"][0]
    a = 0.2 * math.pi
    exact = np.zeros_like(rhs)
    exact[2] = exact[5] = a * np.cos(2 * math.pi * x)
    exact[3] = exact[6] = -a * np.sin(2 * math.pi * x)
    assert np.array_equal(dxdt, c["q"][1:4])
    return np.abs(rhs - exact).max() / a


def test_cp_alfven_exact_rhs():
    e16 = _cp_error(16)
    e32 = _cp_error(32)
    assert e16 < 1e-2 and e32 < 2e-3, (e16, e32)
    assert e16 / e32 > 4.0


def test_galilean_invariance():
    c = synth.cubic_set()
    q = c["q"].copy()
    q[0] = 1.0 + 0.2 * np.abs(q[0])  # positive density
    q[7] = 1.0 + 0.2 * np.abs(q[7])
    r0, _, st = _run(c, q=q)
    q2 = q.copy()
    q2[1:4] += np.array([3.0, -1.25, 0.5])[:, None]
    r1, dx1, st1 = _run(c, q=q2)
    ok = st == 0
    assert np.array_equal(st, st1)
    scale = np.abs(r0[:, ok]).max()
    assert np.abs(r1[:, ok] - r0[:, ok]).max() < 1e-11 * scale


def test_axis_permutation():
    c = synth.random_cloud(2000, seed=33, lam_range=(0.08, 0.1))
    perm = [1, 2, 0]  # new axis a is old axis perm[a]
    rhs, dxdt, st = _run(c)
    pos2 = c["pos"][perm]
    q2 = c["q"].copy()
    q2[1:4] = c["q"][1:4][perm]
    q2[4:7] = c["q"][4:7][perm]
    rhs2, dxdt2, st2 = _run(c, q=q2, pos=pos2)
    assert np.array_equal(st, st2)
    ref = rhs.copy()
    ref[1:4] = rhs[1:4][perm]
    ref[4:7] = rhs[4:7][perm]
    assert np.abs(rhs2 - ref).max() < 1e-10 * np.abs(rhs).max()


def test_periodic_translation():
    c = synth.random_cloud(2000, seed=34, lam_range=(0.08, 0.1))
    rhs, _, st = _run(c)
    shift = np.array([0.375, 0.625, 0.125])[:, None]  # exact binary fractions
    pos2 = np.mod(c["pos"] + shift, 1.0)
    rhs2, _, st2 = _run(c, pos=pos2)
    assert np.array_equal(st, st2)
    assert np.abs(rhs2 - rhs).max() < 1e-10 * np.abs(rhs).max()
