"""Degenerate and boundary inputs on the GPU, checked against the oracle:
one particle, too few particles, coincident particles (a rank-one moment
matrix), an unjittered lattice whose spacings fall exactly on the cut-off
radius, the 19/20-neighbor status boundary, and rejected inputs (n = 0)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import dev, setup_of, csr_rows

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")
torch = pytest.importorskip("torch")


def both(c, precision=None):
    s = setup_of(c, **({} if precision is None else {"precision": precision}))
    pos, lam, q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
    off, idx = P.neighbors(pos, lam, s)
    rhs, dxdt, st = P.mhd_rhs(pos, lam, off, idx, q, s)
    ooff, oidx = oracle.neighbors(c["pos"], c["lam"], L=c["L"], periodic=c["periodic"])
    orhs, odx, ost = oracle.mhd_rhs(c["pos"], c["lam"], ooff, oidx, c["q"], L=c["L"],
                                    periodic=c["periodic"])
    return ((off.cpu().numpy(), idx.cpu().numpy(), rhs.cpu().numpy(), dxdt.cpu().numpy(),
             st.cpu().numpy()), (ooff, oidx, orhs, odx, ost))


def state(pos, lam, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), seed=0):
    n = pos.shape[1]
    rng = np.random.default_rng(seed)
    q = np.zeros((8, n))
    q[0] = 1.0 + 0.1 * rng.uniform(size=n)
    q[1:7] = 0.1 * rng.normal(size=(6, n))
    q[7] = 1.5
    return dict(pos=pos, lam=np.asarray(lam, dtype=np.float64), q=q, L=L, periodic=periodic,
                gamma=5 / 3)


@pytest.mark.parametrize("precision", [0, 1])
def test_single_particle(precision):
    c = state(np.array([[0.3], [0.6], [0.9]]), [0.05])
    (off, idx, rhs, dxdt, st), (ooff, oidx, orhs, odx, ost) = both(c, precision)
    assert off.tolist() == [0, 1] and idx.tolist() == [0]
    assert st.tolist() == [1] == ost.tolist()
    assert np.all(np.isnan(rhs)) and np.array_equal(dxdt, odx)
    # reverse mode: only the dxdt seed reaches q
    pos, lam, q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
    s = setup_of(c, precision=precision)
    o, i = P.neighbors(pos, lam, s)
    xbar = np.array([[1.0], [2.0], [3.0]])
    qb, pb = P.mhd_rhs_adjoint(pos, lam, o, i, P.transpose(o, i), q, dev(np.ones((8, 1))),
                               dev(xbar), setup=s)
    assert np.array_equal(qb.cpu().numpy()[1:4, 0], xbar[:, 0])
    assert np.all(qb.cpu().numpy()[[0, 4, 5, 6, 7], 0] == 0) and np.all(pb.cpu().numpy() == 0)


def test_too_few_particles_everywhere():
    rng = np.random.default_rng(2)
    c = state(rng.uniform(0, 1, (3, 12)), np.full(12, 0.1))
    (off, idx, rhs, dxdt, st), (ooff, oidx, orhs, odx, ost) = both(c)
    assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
    assert np.all(st == 1) and np.array_equal(st, ost) and np.all(np.isnan(rhs))


@pytest.mark.parametrize("precision", [0, 1])
def test_coincident_particles_are_singular(precision):
    # 30 particles on one point and a sparse background: the stacked ones see
    # each other only (xi = 0 for every neighbor), a rank-one moment matrix
    rng = np.random.default_rng(3)
    pos = np.concatenate([np.full((3, 30), 0.5), rng.uniform(0, 1, (3, 40))], axis=1)
    c = state(pos, np.full(70, 0.02))
    (off, idx, rhs, dxdt, st), (ooff, oidx, orhs, odx, ost) = both(c, precision)
    assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
    assert np.all(np.diff(off)[:30] == 30)
    assert np.all(st[:30] == 2) and np.array_equal(st, ost)
    assert np.all(np.isnan(rhs[:, :30]))


def test_lattice_spacings_on_the_cut_off():
    # unjittered 8^3 lattice, spacing 1/8, and lambda chosen so that r_f is the
    # second-shell distance up to rounding: which pairs are in is decided by
    # the last bit of the FP64 expression, on both sides alike
    g = (np.arange(8) + 0.5) / 8
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    for r in (0.25, np.sqrt(2) * 0.125, np.sqrt(3) * 0.125):
        c = state(pos, np.full(512, r / 2.3), seed=4)
        (off, idx, rhs, dxdt, st), (ooff, oidx, orhs, odx, ost) = both(c)
        assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
        assert np.array_equal(st, ost)


def test_status_boundary_at_twenty_neighbors():
    # particle 0 at the centre with exactly 19 others inside its sphere, then 20
    rng = np.random.default_rng(5)
    for k, want in ((18, 1), (19, 0)):
        d = rng.normal(size=(3, k))
        d /= np.linalg.norm(d, axis=0)
        d *= rng.uniform(0.2, 0.9, k) * 0.1
        pos = np.concatenate([np.full((3, 1), 0.5), 0.5 + d], axis=1)
        lam = np.concatenate([[0.1 / 2.3], np.full(k, 0.001)])
        c = state(pos, lam, seed=6)
        (off, idx, rhs, dxdt, st), (ooff, oidx, orhs, odx, ost) = both(c)
        assert off[1] == k + 1 and np.array_equal(st, ost)
        assert st[0] == (1 if k + 1 < 20 else ost[0]) and (want == 1) == (st[0] == 1)


def test_zero_particles_are_rejected():
    ctx = P.context()
    s = P.Setup().params()
    nnz = ctypes.c_int64(0)
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    rc = P.lib().phb_neighbors_build(ctx, ctypes.byref(s), 0, P._ptr(buf), P._ptr(buf),
                                     P._ptr(buf), P._ptr(buf), 0, ctypes.byref(nnz))
    assert rc == P.PHB_EINVAL
    rc = P.lib().phb_mhd_rhs(ctx, ctypes.byref(s), 0, P._ptr(buf), P._ptr(buf), P._ptr(buf),
                             P._ptr(buf), P._ptr(buf), P._ptr(buf), P._ptr(buf), P._ptr(buf),
                             None)
    assert rc == P.PHB_EINVAL


def test_transpose_rejects_nnz_beyond_int32_positions():
    # the transposed positions are int32: a list of more than 2^31 - 1 entries
    # is refused on the host, before any kernel reads the (small) buffers
    off = torch.zeros(5, dtype=torch.int64, device="cuda")
    idx = torch.zeros(4, dtype=torch.int32, device="cuda")
    t_off = torch.empty_like(off)
    t_src = torch.empty_like(idx)
    t_pos = torch.empty_like(idx)
    ctx = P.context()
    lib = P.lib()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = lib.phb_neighbors_transpose(ctx, 4, 1 << 31, p(off), p(idx), p(t_off), p(t_src),
                                     p(t_pos))
    assert rc == P.PHB_EINVAL
    assert b"int32" in lib.phb_last_error(ctx)
    # at the limit's edge the same call is accepted (an empty list here)
    assert lib.phb_neighbors_transpose(ctx, 4, 0, p(off), p(idx), p(t_off), p(t_src),
                                       p(t_pos)) == P.PHB_OK
    torch.cuda.synchronize()
