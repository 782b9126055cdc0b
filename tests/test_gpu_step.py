"""GPU predictor-corrector step against the oracle's step (Heun with the
neighbor lists rebuilt at the predicted state)."""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import dev, setup_of, rhs_err

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")


def gpu_steps(c, dt, nsteps):
    s = setup_of(c)
    pos, q, lam = dev(c["pos"]), dev(c["q"]), dev(c["lam"])
    for _ in range(nsteps):
        st, off, idx = P.pc_step(pos, q, lam, dt, s)
    return pos.cpu().numpy(), q.cpu().numpy(), st.cpu().numpy(), off, idx


def oracle_steps(c, dt, nsteps):
    pos, q = c["pos"], c["q"]
    for _ in range(nsteps):
        pos, q, st = oracle.pc_step(pos, c["lam"], q, dt, L=c["L"], periodic=c["periodic"],
                                    gamma=c["gamma"])
    return pos, q, st


@pytest.mark.parametrize("name", ["cp_alfven", "fast_wave"])
def test_steps_match_oracle(name):
    c = synth.cp_alfven(12) if name == "cp_alfven" else synth.fast_wave_set(side=16)
    dt = 0.01
    gp, gq, gs, _, _ = gpu_steps(c, dt, 3)
    op, oq, os_ = oracle_steps(c, dt, 3)
    assert np.array_equal(gs, os_)
    d = np.abs(gp - op)
    d = np.minimum(d, 1.0 - d)
    assert d.max() < 1e-14
    # field changes relative to the size of the change over the steps
    e = rhs_err(gq - c["q"], oq - c["q"])
    print("field change rel err", e)
    assert max(e.values()) < 1e-10


def test_uniform_flow_translates_exactly():
    c = synth.cubic_set()
    n = c["pos"].shape[1]
    q = synth.wave_background(n, 1.0, 1.5)
    q[1:4] = np.array([0.3, -0.2, 0.45])[:, None]
    c = dict(c, q=q)
    gp, gq, gs, off, idx = gpu_steps(c, 0.37, 1)
    expect = np.mod(c["pos"] + q[1:4] * 0.37, 1.0)
    d = np.abs(gp - expect)
    d = np.minimum(d, 1.0 - d)
    assert d.max() < 1e-15 and np.abs(gq - q).max() < 1e-13
    # the returned lists belong to the predicted state, which here is the final one
    ooff, oidx = oracle.neighbors(gp, c["lam"])
    assert np.array_equal(off.cpu().numpy(), ooff) and np.array_equal(idx.cpu().numpy(), oidx)


def test_particle_leaving_open_box_is_an_error():
    c = synth.random_cloud(3000, seed=61, lam_range=(0.07, 0.1), periodic=(0, 1, 1))
    q = c["q"].copy()
    q[0] = 1.0
    q[1] = 0.5  # everything drifts towards x = 1
    s = setup_of(c)
    pos, lam = dev(c["pos"]), dev(c["lam"])
    with pytest.raises(P.PhurbasError) as e:
        P.pc_step(pos, dev(q), lam, 0.5, s, capacity=3000 * 3000)
    assert e.value.code == P.PHB_EINVAL
