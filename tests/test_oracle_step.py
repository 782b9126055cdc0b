"""Pins of the oracle's second-order predictor-corrector step (paper II,
Sec. 2; read as Heun's trapezoidal scheme with neighbor sets rebuilt at the
predicted state).

* a uniform state is translated exactly: x -> x + V dt (wrapped), fields
  unchanged;
* self-convergence of order two in dt on the circularly polarized Alfven
  wave (Sec. 3.2).
"""
import numpy as np

import oracle
from paper_1110_0836_amd import synth


def test_uniform_state_translates():
    c = synth.cubic_set()
    n = c["pos"].shape[1]
    q = synth.wave_background(n, 1.0, 1.5)
    V = np.array([0.3, -0.2, 0.45])
    q[1:4] = V[:, None]
    dt = 0.37
    pos2, q2, st = oracle.pc_step(c["pos"], c["lam"], q, dt)
    assert np.all(st == 0)
    expect = np.mod(c["pos"] + V[:, None] * dt, 1.0)
    d = np.abs(pos2 - expect)
    d = np.minimum(d, 1.0 - d)  # compare on the circle
    assert d.max() < 1e-15
    assert np.abs(q2 - q).max() < 1e-13
    assert np.all((pos2 >= 0) & (pos2 < 1))


def _run(c, T, nsteps):
    pos, q = c["pos"], c["q"]
    for _ in range(nsteps):
        pos, q, st = oracle.pc_step(pos, c["lam"], q, T / nsteps, gamma=c["gamma"])
        assert np.all(st == 0)
    return pos, q


def test_second_order_in_dt():
    c = synth.cp_alfven(12)
    T = 0.08
    _, qref = _run(c, T, 32)
    errs = []
    for ns in (2, 4, 8):
        _, qs = _run(c, T, ns)
        errs.append(np.abs(qs - qref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs
