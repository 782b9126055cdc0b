"""Every schedule knob gives the oracle's results (FP64 within 1e-12, mixed
within 1e-5): each knob is moved away from its default in turn, on a ragged
cloud whose rows run from one entry to about eighty, so that blocks of the
pair-parallel reverse kernel touch both few rows (owner records staged in
LDS) and many short rows (records read from global memory).  Rows shorter
than 40 entries run through every kernel but are not compared (see the
fixture)."""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import dev, setup_of, rel_err

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")

VARIANTS = [("lanes_moments", 1), ("lanes_moments", 2), ("lanes_apply", 1), ("lanes_apply", 2),
            ("lanes_adj_y", 1), ("lanes_adj_y", 4), ("lanes_gather", 1), ("lanes_gather", 2),
            ("adj_pairs_mode", 0), ("record_order", 1), ("cells_per_rf", 1),
            ("cells_per_rf", 3)]


@pytest.fixture(scope="module")
def cloud():
    # a jittered 14^3 lattice whose resolution lengths vary from 0.45 to 1.6
    # spacings: rows of ~4 to ~200 entries, every fit well posed
    rng = np.random.default_rng(31)
    side = 14
    pos = synth.jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    lam = rng.uniform(0.45, 1.6, n) / side
    q = synth.random_cloud(n, seed=33)["q"]
    q[0] = 1.0 + 0.1 * np.abs(q[0])
    c = dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=5 / 3)
    gbar = rng.normal(size=(8, n))
    off, idx = oracle.neighbors(c["pos"], c["lam"])
    # rows of fewer than 40 entries give nearly square, ill-conditioned fits
    # (the normal equations then differ from the oracle's QR by kappa^2 eps,
    # whatever the schedule): they pass through the kernels, but seed no
    # gradient and are left out of the comparison
    well = np.diff(off) >= 40
    gbar[:, ~well] = 0.0
    orhs, _, ost = oracle.mhd_rhs(c["pos"], c["lam"], off, idx, c["q"])
    oq, op, _ = oracle.mhd_rhs_adjoint(c["pos"], c["lam"], off, idx, c["q"], gbar)
    counts = np.diff(off)
    assert counts.min() <= 6 and counts.max() >= 150 and (ost == 0).sum() > 1000
    return c, gbar, well, (off, idx), (orhs, ost), (oq, op)


def run_pass(c, gbar, s):
    pos, lam, q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
    off, idx = P.neighbors(pos, lam, s)
    rhs, _, st, tape = P.mhd_rhs(pos, lam, off, idx, q, s, tape=True)
    qb, pb = P.mhd_rhs_adjoint(pos, lam, off, idx, P.transpose(off, idx), q, dev(gbar), setup=s,
                               tape=tape)
    return (off.cpu().numpy(), idx.cpu().numpy(), rhs.cpu().numpy(), st.cpu().numpy(),
            qb.cpu().numpy(), pb.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("key,value", VARIANTS)
def test_variant_matches_oracle(cloud, key, value, precision):
    c, gbar, well, (ooff, oidx), (orhs, ost), (oq, op) = cloud
    s = setup_of(c, precision=P.PHB_FP64 if precision == "fp64" else P.PHB_MIXED)
    old = P.phb_tune_get(key)
    P.phb_tune_set(key, value)
    try:
        off, idx, rhs, st, qb, pb = run_pass(c, gbar, s)
    finally:
        P.phb_tune_set(key, old)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
    assert np.array_equal(st, ost)
    ok = (st == 0) & well
    er = max(rel_err(rhs[grp][:, ok], orhs[grp][:, ok])
             for grp in ([0], [1, 2, 3], [4, 5, 6], [7]))
    eq = max(rel_err(qb[f], oq[f]) for f in range(8))
    ep = rel_err(pb, op)
    print(f"{key}={value} {precision}: rhs {er:.2e} q_bar {eq:.2e} pos_bar {ep:.2e}")
    assert er < tol and eq < tol and ep < tol
