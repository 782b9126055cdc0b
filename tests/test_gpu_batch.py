"""Many independent particle sets in one concatenation, replayed from one
captured HIP graph, and the schedule autotuner.

- Batched neighbor lists equal each set's brute-force lists, shifted to
  global indices (bit-exact).
- One batched forward and reverse pass matches the oracle set by set (FP64
  within 1e-12, mixed within 1e-5) and equals the per-set library calls.
- Graph replays, with eager work and new input values between them, match an
  eager pass every time.
- The autotuner picks valid values, does not change results beyond
  rounding, and reads its cache back."""
import os

import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import dev, rhs_err, rel_err

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")
torch = pytest.importorskip("torch")


def concat(sets):
    pos = np.concatenate([s["pos"] for s in sets], axis=1)
    lam = np.concatenate([s["lam"] for s in sets])
    q = np.concatenate([s["q"] for s in sets], axis=1)
    return pos, lam, q


def small_sets(seed=11, n_sets=4):
    return synth.batched_cubes(seed=seed, n_sets=n_sets, smin=8, smax=12)["sets"]


class Pass:
    """Device buffers of one batched forward + reverse pass."""

    def __init__(self, batch, pos, lam, q, gbar, xbar=None, lists=None):
        n = lam.shape[0]
        self.pos, self.lam, self.q = dev(pos), dev(lam), dev(q)
        if lists is None:  # (re)building the lists drops the batch's graph
            self.off, self.idx = batch.neighbors(self.pos, self.lam)
            self.trans = P.transpose(self.off, self.idx)
        else:
            self.off, self.idx, self.trans = lists
        f64 = dict(dtype=torch.float64, device="cuda")
        self.rhs = torch.empty((8, n), **f64)
        self.dxdt = torch.empty((3, n), **f64)
        self.st = torch.empty(n, dtype=torch.int32, device="cuda")
        self.tape = torch.empty(P.phb_tape_bytes(n) // 8, **f64)
        self.gbar = dev(gbar)
        self.xbar = None if xbar is None else dev(xbar)
        self.qb = torch.empty((8, n), **f64)
        self.pb = torch.empty((3, n), **f64)

    def args(self):
        return (self.pos, self.lam, self.off, self.idx, self.q, self.rhs, self.dxdt, self.st)

    def kw(self):
        return dict(tape=self.tape, trans=self.trans, rhs_bar=self.gbar, dxdt_bar=self.xbar,
                    q_bar=self.qb, pos_bar=self.pb)

    def outputs(self):
        return [t.cpu().numpy() for t in (self.rhs, self.dxdt, self.st, self.qb, self.pb)]


def test_batched_neighbors_equal_each_sets_brute_force():
    sets = small_sets()
    pos, lam, q = concat(sets)
    b = P.Batch([s["lam"].shape[0] for s in sets])
    off, idx = b.neighbors(dev(pos), dev(lam))
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    start = 0
    for s in sets:
        ns = s["lam"].shape[0]
        ooff, oidx = oracle.neighbors(s["pos"], s["lam"])
        rows = off[start:start + ns + 1]
        assert np.array_equal(rows - rows[0], ooff)
        assert np.array_equal(idx[rows[0]:rows[-1]], oidx + start)
        start += ns
    assert off[-1] == idx.shape[0] == b.nnz
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_pass_matches_oracle_per_set(precision):
    sets = small_sets(seed=12)
    pos, lam, q = concat(sets)
    n = lam.shape[0]
    rng = np.random.default_rng(13)
    gbar = rng.normal(size=(8, n))
    setup = P.Setup(precision=P.PHB_FP64 if precision == "fp64" else P.PHB_MIXED)
    tol = 1e-12 if precision == "fp64" else 1e-5
    b = P.Batch([s["lam"].shape[0] for s in sets], setup)
    ps = Pass(b, pos, lam, q, gbar)
    b.run(*ps.args(), **ps.kw())
    rhs, dxdt, st, qb, pb = ps.outputs()
    start = 0
    for s in sets:
        ns = s["lam"].shape[0]
        sl = slice(start, start + ns)
        ooff, oidx = oracle.neighbors(s["pos"], s["lam"])
        orhs, odx, ost = oracle.mhd_rhs(s["pos"], s["lam"], ooff, oidx, s["q"])
        od1, _, _ = oracle.mls_derivs(s["pos"], s["lam"], ooff, oidx, s["q"], second=False)
        assert np.array_equal(st[sl], ost) and np.all(ost == 0)
        e = rhs_err(rhs[:, sl], orhs, s["q"], od1)
        print(precision, "set", ns, "rhs err", e)
        assert max(e.values()) < tol
        assert np.array_equal(dxdt[:, sl], odx)
        oq, op, _ = oracle.mhd_rhs_adjoint(s["pos"], s["lam"], ooff, oidx, s["q"], gbar[:, sl])
        eq = max(rel_err(qb[f, sl], oq[f]) for f in range(8))
        ep = rel_err(pb[:, sl], op)
        print(precision, "set", ns, "q_bar err", eq, "pos_bar err", ep)
        assert eq < tol and ep < tol
        start += ns
    b.close()


def test_batched_pass_equals_per_set_calls():
    sets = small_sets(seed=14, n_sets=3)
    pos, lam, q = concat(sets)
    n = lam.shape[0]
    gbar = np.random.default_rng(15).normal(size=(8, n))
    b = P.Batch([s["lam"].shape[0] for s in sets])
    ps = Pass(b, pos, lam, q, gbar)
    b.run(*ps.args(), **ps.kw())
    rhs, _, _, qb, pb = ps.outputs()
    start = 0
    for s in sets:
        ns = s["lam"].shape[0]
        sl = slice(start, start + ns)
        spos, slam, sq = dev(s["pos"]), dev(s["lam"]), dev(s["q"])
        off, idx = P.neighbors(spos, slam)
        r, _, _, tp = P.mhd_rhs(spos, slam, off, idx, sq, tape=True)
        q1, p1 = P.mhd_rhs_adjoint(spos, slam, off, idx, P.transpose(off, idx), sq,
                                   dev(gbar[:, sl]), tape=tp)
        # the same kernels on the same rows: equal up to the last bit
        assert np.array_equal(rhs[:, sl], r.cpu().numpy())
        assert np.array_equal(qb[:, sl], q1.cpu().numpy())
        assert np.array_equal(pb[:, sl], p1.cpu().numpy())
        start += ns
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(precision):
    sets = small_sets(seed=16, n_sets=5)
    pos, lam, q = concat(sets)
    n = lam.shape[0]
    rng = np.random.default_rng(17)
    setup = P.Setup(precision=P.PHB_FP64 if precision == "fp64" else P.PHB_MIXED)
    b = P.Batch([s["lam"].shape[0] for s in sets], setup)
    g = Pass(b, pos, lam, q, rng.normal(size=(8, n)), rng.normal(size=(3, n)))
    b.capture(*g.args(), **g.kw())
    # eager reference: same lists, its own outputs
    e = Pass(b, pos, lam, q, np.zeros((8, n)), lists=(g.off, g.idx, g.trans))
    for k in range(3):
        # new inputs in the bound buffers, written by eager torch work
        g.q.mul_(1.0 + 0.01 * (k + 1))
        g.q[0].add_(0.05)
        g.gbar.copy_(torch.from_numpy(rng.normal(size=(8, n))).cuda())
        torch.cuda.synchronize()
        b.launch()
        e.q.copy_(g.q)
        e.gbar.copy_(g.gbar)
        e.xbar = g.xbar
        b.run(*e.args(), **e.kw())
        torch.cuda.synchronize()
        for a, r in zip(g.outputs(), e.outputs()):
            assert np.array_equal(a, r), f"replay {k}"
    b.close()


def test_capture_before_neighbors_is_refused():
    sets = small_sets(seed=18, n_sets=2)
    pos, lam, q = concat(sets)
    n = lam.shape[0]
    b = P.Batch([s["lam"].shape[0] for s in sets])
    f64 = dict(dtype=torch.float64, device="cuda")
    dummy_off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    dummy_idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(P.PhurbasError) as ei:
        b.capture(dev(pos), dev(lam), dummy_off, dummy_idx, dev(q), torch.empty((8, n), **f64),
                  torch.empty((3, n), **f64), torch.empty(n, dtype=torch.int32, device="cuda"))
    assert ei.value.code == P.PHB_ESTATE
    with pytest.raises(P.PhurbasError) as ei:
        b.launch()
    assert ei.value.code == P.PHB_ESTATE
    b.close()


def test_tuner_choices_cache_and_results(tmp_path):
    c = synth.fast_wave_set(side=20)
    s = P.Setup()
    pos, lam, q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
    off, idx = P.neighbors(pos, lam, s)
    tr = P.transpose(off, idx)
    gbar = dev(np.random.default_rng(19).normal(size=(8, lam.shape[0])))
    before = P.mhd_rhs_adjoint(pos, lam, off, idx, tr, q, gbar, setup=s)
    saved = {k: P.phb_tune_get(k) for k in P.TUNE_KEYS}
    cache = os.path.join(tmp_path, "tune.txt")
    try:
        got = P.phb_tune(s, pos, lam, off, idx, *tr, q, reps=2, cache=cache)
        assert got["lanes_moments"] in (1, 2, 4) and got["lanes_gather"] in (1, 2, 4)
        assert got["adj_pairs_mode"] in (0, 1, 2, 3) and got["record_order"] in (0, 1)
        text = open(cache).read()
        assert text.startswith("# phurbas-tune n=%d" % lam.shape[0])
        after = P.mhd_rhs_adjoint(pos, lam, off, idx, tr, q, gbar, setup=s)
        for a, b in zip(after, before):
            assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-12
        # the cache supplies the same values without timing
        for k in ("lanes_moments", "lanes_gather", "adj_pairs_mode"):
            P.phb_tune_set(k, 1 if k != "adj_pairs_mode" else 0)
        again = P.phb_tune(s, pos, lam, off, idx, *tr, q, reps=2, cache=cache)
        assert again == got
    finally:
        for k, v in saved.items():
            P.phb_tune_set(k, v)


def test_full_batched_sets_graph_sampled():
    """32 sets, sides 16..64 (about 2.8M particles): mixed forward and reverse
    pass in one graph, replayed twice, checked on sampled particles of every
    set against the oracle."""
    cfg = synth.batched_cubes()
    sets = cfg["sets"]
    pos, lam, q = concat(sets)
    n = lam.shape[0]
    rng = np.random.default_rng(20)
    gbar = rng.uniform(0, 1, size=(8, n))
    setup = P.Setup(precision=P.PHB_MIXED)
    b = P.Batch([s["lam"].shape[0] for s in sets], setup)
    g = Pass(b, pos, lam, q, gbar)
    b.capture(*g.args(), **g.kw())
    for _ in range(2):
        b.launch()
    torch.cuda.synchronize()
    rhs, dxdt, st, qb, pb = g.outputs()
    start = 0
    worst = {"rhs": 0.0, "q_bar": 0.0, "pos_bar": 0.0}
    for k, s in enumerate(sets):
        ns = s["lam"].shape[0]
        rows = np.sort(rng.choice(ns, 20, replace=False))
        ooff, oidx = oracle.neighbors(s["pos"], s["lam"], rows=rows)
        orhs, _, ost = oracle.mhd_rhs(s["pos"], s["lam"], ooff, oidx, s["q"], rows=rows)
        od1, _, _ = oracle.mls_derivs(s["pos"], s["lam"], ooff, oidx, s["q"], rows=rows,
                                      second=False)
        assert np.array_equal(st[start + rows], ost)
        e = rhs_err(rhs[:, start + rows], orhs, s["q"][:, rows], od1)
        worst["rhs"] = max(worst["rhs"], max(e.values()))
        if k % 8 == 0:  # the reverse mode's oracle is a whole-set pass: a few sets
            ocols = rows[:4]
            oq, op = oracle.adjoint_sampled(s["pos"], s["lam"], s["q"], gbar[:, start:start + ns],
                                            ocols)
            qscale = np.abs(qb[:, start:start + ns]).max(axis=1)
            worst["q_bar"] = max(worst["q_bar"],
                                 float((np.abs(qb[:, start + ocols] - oq).max(axis=1)
                                        / qscale).max()))
            worst["pos_bar"] = max(worst["pos_bar"],
                                   float(np.abs(pb[:, start + ocols] - op).max()
                                         / np.abs(pb[:, start:start + ns]).max()))
        start += ns
    print("batched sets, mixed: worst sampled errors", worst)
    assert max(worst.values()) < 1e-5
    b.close()
