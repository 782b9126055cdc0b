"""GPU moving-least-squares derivatives and ideal-MHD time derivatives
against the oracle (FP64 form): element by element within 1e-12 relative
(per field and derivative order; per physical quantity for the time
derivatives) at sizes the oracle finishes quickly, and on sampled particles
at the benchmark sizes.

Open boxes: particles whose sphere is cut by a face are fitted from a
lopsided sample, with condition numbers up to ~1e10.  The oracle's QR is
itself exact only to about kappa(P) eps = sqrt(kappa) eps there, so each
particle is held to 1e-12 plus 64 sqrt(kappa) eps (kappa of its equilibrated
moment matrix), and, for the exact cubic fields of the pin variant, the GPU's
error against the analytic derivatives to within a small factor of the
oracle's own."""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import (dev, setup_of, rel_err, rhs_err, interior, fit_kappa, kappa_tol,
                     particle_err, rhs_particle_err)
from test_oracle_mls import _analytic

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")

TOL64 = 1e-12


def derivs_both(c, fields=None):
    fields = c["q"] if fields is None else fields
    s = setup_of(c)
    pos, lam = dev(c["pos"]), dev(c["lam"])
    off, idx = P.neighbors(pos, lam, s)
    d1, d2, st = P.mls_derivs(pos, lam, off, idx, dev(fields), s)
    ooff, oidx = oracle.neighbors(c["pos"], c["lam"], L=c["L"], periodic=c["periodic"])
    o1, o2, ost = oracle.mls_derivs(c["pos"], c["lam"], ooff, oidx, fields, L=c["L"],
                                    periodic=c["periodic"])
    return (d1.cpu().numpy(), d2.cpu().numpy(), st.cpu().numpy()), (o1, o2, ost)


@pytest.mark.parametrize("pin", [False, True])
def test_cubic_set_derivatives(pin):
    c = synth.cubic_set(pin=pin)
    (g1, g2, gs), (o1, o2, os_) = derivs_both(c)
    assert np.array_equal(gs, os_)
    ok = gs == 0
    inner = ok & interior(c["pos"], c["lam"], c["L"], c["periodic"])
    e1 = rel_err(g1[:, :, inner], o1[:, :, inner], axis=(1, 2))
    e2 = rel_err(g2[:, :, inner], o2[:, :, inner], axis=(1, 2))
    print("whole spheres: first-order max rel err per field", e1, "second-order", e2)
    assert e1.max() < TOL64 and e2.max() < TOL64
    if pin:
        # every particle, face particles included, within the condition-scaled
        # bound of the oracle ...
        off, idx = oracle.neighbors(c["pos"], c["lam"], L=c["L"], periodic=c["periodic"])
        tol = kappa_tol(fit_kappa(c["pos"], c["lam"], off, idx, L=c["L"],
                                  periodic=c["periodic"])[ok])
        for g, o in ((g1, o1), (g2, o2)):
            worst = max((particle_err(g[f], o[f], ok) / tol).max() for f in range(8))
            print("error over the condition-scaled bound, worst particle", worst)
            assert worst <= 1.0
        # ... and as close to the exact cubic as the oracle (Sec. 2's third-order
        # fit reproduces cubics): per field and derivative order, the GPU's
        # largest error against the analytic derivatives within a small factor
        # of the oracle's own
        x1, x2 = _analytic(c["pos"], c["coef"], c["exponents"])
        for g, o, x in ((g1, o1, x1), (g2, o2, x2)):
            for f in range(8):
                eg = particle_err(g[f], x[f], ok).max()
                eo = particle_err(o[f], x[f], ok).max()
                print(f"field {f}: exact-cubic error, GPU max {eg:.2e}, oracle max {eo:.2e}")
                assert eg <= 2.0 * eo + 1e-13
    assert np.all(np.isnan(g1[:, :, ~ok])) and np.all(np.isnan(g2[:, :, ~ok]))


def test_many_fields_ragged_set():
    c = synth.random_cloud(3001, seed=5, lam_range=(0.06, 0.1))
    rng = np.random.default_rng(6)
    fields = np.concatenate([c["q"], rng.normal(size=(3, 3001))])  # 11 fields: two chunks
    (g1, g2, gs), (o1, o2, os_) = derivs_both(c, fields)
    assert np.array_equal(gs, os_)
    ok = gs == 0
    assert rel_err(g1[:, :, ok], o1[:, :, ok], axis=(1, 2)).max() < TOL64
    assert rel_err(g2[:, :, ok], o2[:, :, ok], axis=(1, 2)).max() < TOL64


def test_status_paths():
    # isolated particles (status 1) and a coplanar set (status 2)
    rng = np.random.default_rng(8)
    n = 1500
    pos = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), np.full(n, 0.5)])
    lam = np.full(n, 0.04)
    lam[:10] = 0.004
    c = dict(pos=pos, lam=lam, q=np.ones((8, n)), L=(1, 1, 1), periodic=(1, 1, 1))
    (g1, g2, gs), (o1, o2, os_) = derivs_both(c)
    off, _ = oracle.neighbors(pos, lam)
    few = np.diff(off) < 20
    assert few[:10].all()
    assert np.array_equal(gs, np.where(few, 1, 2))
    assert np.array_equal(gs, os_)
    assert np.all(np.isnan(g1))


def rhs_both(c, rows=None, **kw):
    """GPU and oracle time derivatives (optionally on sampled rows), plus the
    GPU's saved gradients and the oracle's first derivatives of all fields."""
    s = setup_of(c, **kw)
    pos, lam = dev(c["pos"]), dev(c["lam"])
    off, idx = P.neighbors(pos, lam, s)
    rhs, dxdt, st, tape = P.mhd_rhs(pos, lam, off, idx, dev(c["q"]), s, tape=True)
    n = c["lam"].shape[0]
    ooff, oidx = oracle.neighbors(c["pos"], c["lam"], L=c["L"], periodic=c["periodic"], rows=rows)
    orhs, odx, ost = oracle.mhd_rhs(c["pos"], c["lam"], ooff, oidx, c["q"], L=c["L"],
                                    periodic=c["periodic"], gamma=c["gamma"], rows=rows,
                                    weight=kw.get("weight", 0))
    od1, _, _ = oracle.mls_derivs(c["pos"], c["lam"], ooff, oidx, c["q"], L=c["L"],
                                  periodic=c["periodic"], rows=rows, second=False,
                                  weight=kw.get("weight", 0))
    grads = P.tape_rows(tape, n)[:21].reshape(7, 3, n).cpu().numpy()
    g = (rhs.cpu().numpy(), dxdt.cpu().numpy(), st.cpu().numpy(), grads)
    qs = c["q"]
    if rows is not None:
        g = (g[0][:, rows], g[1][:, rows], g[2][rows], g[3][:, :, rows])
        qs = c["q"][:, rows]
    return g, (orhs, odx, ost, od1), qs


def check_rhs(g, o, qs, tol, sel=None, gamma=5.0 / 3.0, kappa=None):
    """tol: the bound of every selected particle; kappa (all particles): each
    particle's bound is instead kappa_tol(kappa), 1e-12 + 64 sqrt(kappa) eps."""
    (r, x, s, gd), (orr, ox, os_, od1) = g, o
    assert np.array_equal(s, os_)
    ok = s == 0 if sel is None else (s == 0) & sel
    if kappa is not None:
        bound = kappa_tol(kappa[ok])
        # the derivative operator itself, per field (V, B, sigma), and the
        # time derivatives per quantity, particle by particle
        wd = max((particle_err(gd[f], od1[1 + f], ok) / bound).max() for f in range(7))
        wr = (rhs_particle_err(r[:, ok], orr[:, ok], qs[:, ok], od1[:, :, ok], gamma)
              / bound).max()
        print("error over the condition-scaled bound, worst particle: gradients", wd, "rhs", wr)
        assert wd <= 1.0 and wr <= 1.0
        assert np.array_equal(x, ox)
        return None
    # the derivative operator itself, per field (V, B, sigma)
    ed = rel_err(gd[:, :, ok], od1[1:, :, ok], axis=(1, 2))
    print("gradient max rel err per field", ed)
    assert ed.max() < tol
    e = rhs_err(r[:, ok], orr[:, ok], qs[:, ok], od1[:, :, ok], gamma)
    print("rhs max rel err per quantity (relative to its terms)", e)
    assert max(e.values()) < tol
    assert np.array_equal(x, ox)
    return e


@pytest.mark.parametrize("side", [16, 24])
def test_rhs_fast_wave_small(side):
    check_rhs(*rhs_both(synth.fast_wave_set(side=side)), TOL64)


def test_rhs_cp_alfven():
    check_rhs(*rhs_both(synth.cp_alfven(16)), TOL64)


def test_rhs_random_open_box():
    c = synth.random_cloud(2500, seed=12, lam_range=(0.07, 0.1), periodic=(0, 1, 0))
    c["q"][0] = 1.0 + 0.1 * np.abs(c["q"][0])
    g, o, qs = rhs_both(c)
    check_rhs(g, o, qs, TOL64, interior(c["pos"], c["lam"], c["L"], c["periodic"]))
    off, idx = oracle.neighbors(c["pos"], c["lam"], L=c["L"], periodic=c["periodic"])
    check_rhs(g, o, qs, None, kappa=fit_kappa(c["pos"], c["lam"], off, idx, L=c["L"],
                                              periodic=c["periodic"]))


def test_rhs_unit_weight():
    c = synth.fast_wave_set(side=16)
    g, o, qs = rhs_both(c, weight=P.PHB_W_UNIT)
    orhs, _, _ = oracle.mhd_rhs(c["pos"], c["lam"], *oracle.neighbors(c["pos"], c["lam"]),
                                c["q"], weight=1)
    assert np.array_equal(o[0], orhs)  # rhs_both passed the weight to the oracle
    check_rhs(g, o, qs, TOL64)


def test_rhs_fast_wave_full_size_sampled():
    c = synth.fast_wave_set()
    rows = np.random.default_rng(3).choice(c["lam"].shape[0], 2000, replace=False)
    check_rhs(*rhs_both(c, rows=rows), TOL64)


def test_rhs_shear_layer_full_size_sampled():
    c = synth.shear_layer()
    rows = np.random.default_rng(4).choice(c["lam"].shape[0], 300, replace=False)
    check_rhs(*rhs_both(c, rows=rows), TOL64)


def test_tape_holds_gradients():
    c = synth.fast_wave_set(side=16)
    s = setup_of(c)
    pos, lam = dev(c["pos"]), dev(c["lam"])
    off, idx = P.neighbors(pos, lam, s)
    rhs, dxdt, st, tape = P.mhd_rhs(pos, lam, off, idx, dev(c["q"]), s, tape=True)
    d1, _, _ = P.mls_derivs(pos, lam, off, idx, dev(c["q"][1:]), s, second=False)
    n = lam.shape[0]
    assert np.allclose(P.tape_rows(tape, n)[:21].reshape(7, 3, n).cpu().numpy(), d1.cpu().numpy(), rtol=1e-13,
                       atol=1e-20)
