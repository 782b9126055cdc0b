"""The neighbor build, its transpose, the forward evaluation and the reverse
mode captured in one HIP graph (Sec. 2.1: the neighbor retrieval is part of
every derivative evaluation), through the calls that keep every size on the
device: phb_neighbors_build_async (total and status words on the device,
lists bounded by the idx capacity), the transpose (the capacity as its entry
bound) and phb_mhd_rhs_adjoint_async (the same bound).

The set is a random cloud with lambda over a 2.5x range, so that its lists
are not mutual and the transpose's one-way part is exercised.  The graph is
replayed three times with eager work and synchronizations between the
replays, the particles moved before the last: every replay is checked
against the oracle's lists bit for bit and its derivatives (FP64 per
particle to the condition-scaled bound of the other parity tests; mixed to
1e-5), and against the eager calls on the same inputs, which run the same
kernels and agree bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import (dev, setup_of, fit_kappa, kappa_tol, kappa_tol_adj, kappa_spread,
                     particle_err, rhs_particle_err, rel_err)

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")
torch = pytest.importorskip("torch")


class Pass:
    """Device buffers of one build + transpose + forward + reverse pass."""

    def __init__(self, c, setup, cap, gbar):
        n = c["lam"].shape[0]
        f64 = dict(dtype=torch.float64, device="cuda")
        i32 = dict(dtype=torch.int32, device="cuda")
        self.n, self.cap, self.s = n, cap, setup
        self.pos, self.lam, self.q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
        self.gbar = dev(gbar)
        self.off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        self.idx = torch.zeros(cap, **i32)
        self.nnz = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.flag = torch.full((1,), -1, **i32)
        self.t_off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        self.t_src = torch.zeros(cap, **i32)
        self.t_pos = torch.zeros(cap, **i32)
        self.rhs = torch.zeros((8, n), **f64)
        self.dxdt = torch.zeros((3, n), **f64)
        self.st = torch.zeros(n, **i32)
        self.tape = torch.zeros(P.phb_tape_bytes(n) // 8, **f64)
        self.qb = torch.zeros((8, n), **f64)
        self.pb = torch.zeros((3, n), **f64)

    def run(self):
        P.phb_neighbors_build_async(self.s, self.pos, self.lam, self.off, self.idx, self.cap,
                                    self.nnz, self.flag)
        ctx = P.context()
        rc = P.lib().phb_neighbors_transpose(ctx, self.n, self.cap, P._ptr(self.off),
                                             P._ptr(self.idx), P._ptr(self.t_off),
                                             P._ptr(self.t_src), P._ptr(self.t_pos))
        P._check(ctx, rc)
        P.phb_mhd_rhs(self.s, self.pos, self.lam, self.off, self.idx, self.q, self.rhs,
                      self.dxdt, self.st, self.tape)
        P.phb_mhd_rhs_adjoint_async(self.s, self.pos, self.lam, self.off, self.idx, self.t_off,
                                    self.t_src, self.t_pos, self.q, self.gbar, None, self.qb,
                                    self.pb, self.tape, self.cap)

    def clear(self):
        for t in (self.off, self.idx, self.t_off, self.t_src, self.t_pos, self.rhs, self.dxdt,
                  self.st, self.qb, self.pb, self.nnz):
            t.zero_()
        self.flag.fill_(-1)

    def outputs(self):
        torch.cuda.synchronize()
        nnz = int(self.nnz.item())
        return dict(flag=int(self.flag.item()), nnz=nnz, off=self.off.cpu().numpy(),
                    idx=self.idx[:nnz].cpu().numpy(), t_off=self.t_off.cpu().numpy(),
                    t_src=self.t_src[:nnz].cpu().numpy(), t_pos=self.t_pos[:nnz].cpu().numpy(),
                    rhs=self.rhs.cpu().numpy(), st=self.st.cpu().numpy(),
                    qb=self.qb.cpu().numpy(), pb=self.pb.cpu().numpy())


def check_transpose(off, idx, t_off, t_src, t_pos):
    n = len(off) - 1
    rows_i = np.repeat(np.arange(n), np.diff(off))
    order = np.lexsort((rows_i, idx))  # by j then i
    assert np.array_equal(t_src, rows_i[order].astype(np.int32))
    assert np.array_equal(t_off, np.concatenate([[0], np.cumsum(np.bincount(idx, minlength=n))]))
    assert np.array_equal(t_src[t_pos], rows_i)
    j_of_t = np.repeat(np.arange(n), np.diff(t_off))
    assert np.array_equal(j_of_t[t_pos], idx)


def check_against_oracle(c, out, precision):
    off, idx = oracle.neighbors(c["pos"], c["lam"], c["L"], c["periodic"])
    assert out["flag"] == 0
    assert out["nnz"] == off[-1]
    assert np.array_equal(out["off"], off) and np.array_equal(out["idx"], idx)
    check_transpose(out["off"], out["idx"], out["t_off"], out["t_src"], out["t_pos"])
    orhs, _, ost = oracle.mhd_rhs(c["pos"], c["lam"], off, idx, c["q"], c["L"], c["periodic"])
    oq, op, _ = oracle.mhd_rhs_adjoint(c["pos"], c["lam"], off, idx, c["q"], c["gbar"], None,
                                       c["L"], c["periodic"])
    assert np.array_equal(out["st"], ost)
    ok = ost == 0
    if precision == P.PHB_MIXED:
        er = max(rel_err(out["rhs"][g][:, ok], orhs[g][:, ok]) for g in ([0], [1, 2, 3],
                                                                        [4, 5, 6], [7]))
        kap = fit_kappa(c["pos"], c["lam"], off, idx, c["L"], c["periodic"])
        bound = np.maximum(kappa_tol_adj(kappa_spread(kap, off, idx)), 1e-5)
        wq = max((particle_err(out["qb"][f], oq[f]) / bound).max() for f in range(8))
        wp = (particle_err(out["pb"], op) / bound).max()
        print(f"mixed: rhs {er:.2e}, reverse mode over its bound q_bar {wq:.2e} "
              f"pos_bar {wp:.2e}")
        assert er < 1e-5 and wq <= 1.0 and wp <= 1.0
    else:
        kap = fit_kappa(c["pos"], c["lam"], off, idx, c["L"], c["periodic"])
        od1, _, _ = oracle.mls_derivs(c["pos"], c["lam"], off, idx, c["q"], c["L"],
                                      c["periodic"], second=False)
        e = rhs_particle_err(out["rhs"][:, ok], orhs[:, ok], c["q"][:, ok], od1[:, :, ok])
        wr = (e / kappa_tol(kap[ok])).max()
        bound = kappa_tol_adj(kappa_spread(kap, off, idx))
        wq = max((particle_err(out["qb"][f], oq[f]) / bound).max() for f in range(8))
        wp = (particle_err(out["pb"], op) / bound).max()
        print(f"FP64 over the condition-scaled bounds: rhs {wr:.3f} q_bar {wq:.3f} "
              f"pos_bar {wp:.3f}")
        assert wr <= 1.0 and wq <= 1.0 and wp <= 1.0


def same(a, b):
    # failed fits (status != 0) return NaN in both
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k]), equal_nan=True), k


@pytest.mark.parametrize("precision", [P.PHB_FP64, P.PHB_MIXED])
def test_build_transpose_forward_reverse_in_one_graph(precision):
    c = synth.random_cloud(3000, seed=41, lam_range=(0.04, 0.1))
    rng = np.random.default_rng(42)
    c["gbar"] = rng.normal(size=(8, c["lam"].shape[0]))
    s = setup_of(c, precision=precision)
    nnz0 = int(oracle.neighbors(c["pos"], c["lam"], c["L"], c["periodic"])[0][-1])
    cap = int(1.2 * nnz0)
    ps = Pass(c, s, cap, c["gbar"])
    P.phb_reserve(ps.n, cap)
    # eager: loads the kernels and is the reference of the first replays
    ps.run()
    eager = ps.outputs()
    check_against_oracle(c, eager, precision)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        ps.run()
    torch.cuda.synchronize()
    for rep in range(2):
        ps.clear()
        torch.cuda.synchronize()
        g.replay()
        got = ps.outputs()
        print(f"replay {rep}: nnz {got['nnz']} flag {got['flag']}")
        same(got, eager)
    # the particles move (wrapped into the box); the graph rebuilds the lists
    moved = dict(c)
    moved["pos"] = np.mod(c["pos"] + rng.uniform(-0.01, 0.01, size=c["pos"].shape), 1.0)
    moved["pos"] = np.minimum(moved["pos"], np.nextafter(1.0, 0.0))
    ps.pos.copy_(dev(moved["pos"]))
    ps.clear()
    torch.cuda.synchronize()
    g.replay()
    got = ps.outputs()
    check_against_oracle(moved, got, precision)
    ps.run()  # eager on the moved set
    same(ps.outputs(), got)


def test_async_build_status_words():
    c = synth.random_cloud(2000, seed=43, lam_range=(0.04, 0.1))
    s = setup_of(c)
    n = c["lam"].shape[0]
    off_o, idx_o = oracle.neighbors(c["pos"], c["lam"], c["L"], c["periodic"])
    nnz = int(off_o[-1])
    pos, lam = dev(c["pos"]), dev(c["lam"])
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    nz = torch.zeros(1, dtype=torch.int64, device="cuda")
    flag = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    # too small: offsets and the total written, the status says so
    idx = torch.full((nnz - 1,), -5, dtype=torch.int32, device="cuda")
    P.phb_neighbors_build_async(s, pos, lam, off, idx, nnz - 1, nz, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == P.PHB_NB_OVERFLOW and int(nz.item()) == nnz
    assert np.array_equal(off.cpu().numpy(), off_o)
    assert (idx.cpu().numpy() == -5).all()  # idx untouched
    # exact capacity
    idx = torch.zeros(nnz, dtype=torch.int32, device="cuda")
    P.phb_neighbors_build_async(s, pos, lam, off, idx, nnz, nz, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0 and np.array_equal(idx.cpu().numpy(), idx_o)
    # invalid positions and too large a radius: status bits, zero offsets
    bad = c["pos"].copy()
    bad[2, 7] = np.nan
    P.phb_neighbors_build_async(s, dev(bad), lam, off, idx, nnz, nz, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == P.PHB_NB_INVALID and int(nz.item()) == 0
    assert not off.cpu().numpy().any()
    P.phb_neighbors_build_async(s, pos, dev(np.full(n, 0.25)), off, idx, nnz, nz, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == P.PHB_NB_RADIUS


def test_long_rows_and_long_transposed_rows():
    # 40 % of the particles with r_f = 0.41: their rows hold about 870 entries
    # (past the in-register sort, into the row-sort path), and every particle
    # lies in about 350 of their spheres (past the transpose's in-register sort)
    c = synth.random_cloud(3000, seed=44, lam_range=(0.03, 0.05))
    rng = np.random.default_rng(45)
    big = rng.random(3000) < 0.4
    c["lam"] = np.where(big, 0.41 / 2.3, c["lam"])
    s = setup_of(c)
    off_o, idx_o = oracle.neighbors(c["pos"], c["lam"], c["L"], c["periodic"])
    lens = np.diff(off_o)
    assert lens.max() > 256
    off, idx = P.neighbors(dev(c["pos"]), dev(c["lam"]), s)
    assert np.array_equal(off.cpu().numpy(), off_o) and np.array_equal(idx.cpu().numpy(), idx_o)
    t_off, t_src, t_pos = P.transpose(off, idx)
    t_off = t_off.cpu().numpy()
    assert np.diff(t_off).max() > 256
    check_transpose(off_o, idx_o, t_off, t_src.cpu().numpy(), t_pos.cpu().numpy())
