"""Every schedule knob gives the oracle's results (FP64 within 1e-12 plus the
condition-scaled share of each fit: 64 sqrt(kappa) eps for the time
derivatives, plus kappa eps / 32 for reverse-mode entries; mixed within 1e-5,
or the FP64 bound where that is larger):
each knob is moved away from its default in turn, on a graded cloud whose
rows run from a few entries to about two hundred, so that blocks of the
pair-parallel reverse kernel touch both few rows (owner records staged in
LDS) and many short rows (records read from global memory).  The nearly
square fits of the short rows reach kappa ~ 1e13 and are compared too."""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import (dev, setup_of, rel_err, fit_kappa, kappa_spread, kappa_tol, kappa_tol_adj,
                     particle_err, rhs_particle_err)

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")

VARIANTS = [("lanes_moments", 1), ("lanes_moments", 2), ("lanes_apply", 1), ("lanes_apply", 2),
            ("lanes_adj_y", 1), ("lanes_adj_y", 4), ("lanes_gather", 1), ("lanes_gather", 2),
            ("adj_pairs_mode", 0), ("adj_pairs_mode", 1), ("adj_pairs_mode", 2), ("record_order", 1), ("cells_per_rf", 1),
            ("cells_per_rf", 3), ("fit_fields", 2), ("moments_mfma", 1)]


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
    orhs, _, ost = oracle.mhd_rhs(c["pos"], c["lam"], off, idx, c["q"])
    od1, _, _ = oracle.mls_derivs(c["pos"], c["lam"], off, idx, c["q"], second=False)
    oq, op, _ = oracle.mhd_rhs_adjoint(c["pos"], c["lam"], off, idx, c["q"], gbar)
    counts = np.diff(off)
    assert counts.min() <= 6 and counts.max() >= 150 and (ost == 0).sum() > 1000
    kappa = fit_kappa(c["pos"], c["lam"], off, idx)
    assert kappa[ost == 0].max() > 1e12  # the ill-conditioned fits are there
    return c, gbar, kappa, (off, idx), (orhs, ost, od1), (oq, op)


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
    c, gbar, kappa, (ooff, oidx), (orhs, ost, od1), (oq, op) = cloud
    s = setup_of(c, precision=P.PHB_FP64 if precision == "fp64" else P.PHB_MIXED)
    old = P.phb_tune_get(key)
    P.phb_tune_set(key, value)
    try:
        off, idx, rhs, st, qb, pb = run_pass(c, gbar, s)
    finally:
        P.phb_tune_set(key, old)
    assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
    assert np.array_equal(st, ost)
    ok = st == 0
    # each particle within the bound of its own fit; each gradient entry
    # within that of the worst fit it receives a contribution from
    bound = kappa_tol_adj(kappa_spread(kappa, ooff, oidx))
    if precision == "fp64":
        wr = (rhs_particle_err(rhs[:, ok], orhs[:, ok], c["q"][:, ok], od1[:, :, ok])
              / kappa_tol(kappa[ok])).max()
    else:
        er = max(rel_err(rhs[grp][:, ok], orhs[grp][:, ok])
                 for grp in ([0], [1, 2, 3], [4, 5, 6], [7]))
        wr = er / 1e-5
        bound = np.maximum(bound, 1e-5)
    wq = max((particle_err(qb[f], oq[f]) / bound).max() for f in range(8))
    wp = (particle_err(pb, op) / bound).max()
    print(f"{key}={value} {precision}: error over the bound, worst particle: "
          f"rhs {wr:.2e} q_bar {wq:.2e} pos_bar {wp:.2e}")
    assert wr <= 1.0 and wq <= 1.0 and wp <= 1.0
