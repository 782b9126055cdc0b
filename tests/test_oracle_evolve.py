"""Oracle multi-step evolution (Sec. 2 predictor-corrector, read as Heun),
pinned to what the paper fixes: the exact nonlinear circularly polarized
Alfven wave of Sec. 3.2 (converging with resolution), exact translation of a
uniform state past frozen particles, the frozen particles themselves, and
agreement of repeated single steps with the multi-step loop."""
import numpy as np

import oracle
from paper_1110_0836_amd import synth


def cp_exact(x, t):
    """The Sec. 3.2 wave (V_perp = B_perp, B_x = 1) travels towards -x at V_A = 1."""
    ph = 2 * np.pi * (x + t)
    return np.stack([0.1 * np.sin(ph), 0.1 * np.cos(ph)])


def cp_error(side, t_end, cfl=0.3):
    c = synth.cp_alfven(side)
    dt0 = oracle.courant_dt(c["q"], c["lam"], cfl)
    nsteps = int(np.ceil(t_end / dt0))
    pos, q, st = oracle.evolve(c["pos"], c["lam"], c["q"], t_end / nsteps, nsteps)
    assert np.all(st == 0)
    ex = cp_exact(pos[0], t_end)
    num = np.abs(q[2:4] - ex).sum() + np.abs(q[5:7] - ex).sum()
    return num / (2 * np.abs(ex).sum())


def test_cp_alfven_converges_to_the_exact_wave():
    e8, e12 = cp_error(8, 0.1), cp_error(12, 0.1)
    order = np.log(e8 / e12) / np.log(12 / 8)
    print("CP Alfven relative L1 error", e8, e12, "order", order)
    assert e12 < e8 and order > 1.5 and e12 < 1e-2


def test_uniform_flow_past_frozen_particles():
    rng = np.random.default_rng(3)
    pos = synth.jittered_lattice(8, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1 / 8)
    q = np.zeros((8, n))
    q[0], q[1], q[2], q[4], q[7] = 1.0, 0.3, -0.2, 0.5, 1.5
    frozen = (pos[0] < 0.25).astype(np.int32)
    p2, q2, st = oracle.evolve(pos, lam, q, 0.01, 3, frozen=frozen)
    fz = frozen == 1
    assert np.array_equal(p2[:, fz], pos[:, fz]) and np.array_equal(q2[:, fz], q[:, fz])
    moved = np.mod(pos[:, ~fz] + 0.03 * q[1:4, ~fz], 1.0)
    assert np.abs(p2[:, ~fz] - moved).max() < 1e-14
    assert np.abs(q2[:, ~fz] - q[:, ~fz]).max() < 1e-12
    assert np.all(st[fz] == 0)


def test_multi_step_equals_repeated_single_steps():
    c = synth.cp_alfven(6)
    p1, q1, s1 = oracle.evolve(c["pos"], c["lam"], c["q"], 0.02, 3)
    p2, q2 = c["pos"], c["q"]
    for _ in range(3):
        p2, q2, _ = oracle.pc_step(p2, c["lam"], q2, 0.02)
    assert np.array_equal(p1, p2) and np.array_equal(q1, q2)


def test_courant_dt_formula():
    c = synth.cp_alfven(6)
    q, lam = c["q"], c["lam"]
    gam = 5.0 / 3.0
    cf = np.sqrt((gam * (gam - 1) * q[7] + (q[4:7] ** 2).sum(0)) / q[0])
    ref = 0.4 * np.min(lam / cf)
    assert abs(oracle.courant_dt(q, lam, 0.4) - ref) <= 1e-15 * ref
    frozen = np.ones(lam.shape[0], np.int32)
    frozen[5] = 0
    ref5 = 0.4 * lam[5] / cf[5]
    assert abs(oracle.courant_dt(q, lam, 0.4, frozen=frozen) - ref5) <= 1e-15 * ref5
    # Sec. 2: the step does not depend on the bulk velocity
    q2 = q.copy()
    q2[1:4] += np.array([3.0, -2.0, 5.0])[:, None]
    assert oracle.courant_dt(q2, lam, 0.4) == oracle.courant_dt(q, lam, 0.4)


def test_linear_wave_eigenvectors_are_consistent():
    """The generated waves satisfy the linear momentum equation
    omega rho0 V = k (P + B0.B) - (k.B0) B with the stated speeds."""
    for kind, speed in (("sound", 1.0), ("alfven", 1.0), ("fast", 2.0)):
        c = synth.linear_wave(kind, 4)
        R, om = c["R"], c["omega"]
        assert abs(om - 2 * np.pi * speed) < 1e-12
        k = np.array([2 * np.pi, 0, 0])
        B0 = c["q0"][4:7]
        P = (5 / 3 - 1) * R[7]
        lhs = om * c["q0"][0] * R[1:4]
        rhs = k * (P + B0 @ R[4:7]) - (k @ B0) * R[4:7]
        assert np.abs(lhs - rhs).max() < 1e-12
