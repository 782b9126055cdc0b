"""The allocation-free variant phb_mhd_rhs_noalloc (static device scratch,
for callers that cannot allocate) against phb_mhd_rhs, through the C-ABI:
two calls in a row on fresh contexts, the second on a smaller set and in the
other precision, each compared with the allocating entry point on the same
inputs (FP64 within 1e-12 per quantity, as every FP64 parity test; the same
kernels run, so the results are in fact identical); free device memory is
unchanged across an allocation-free call (once the process has launched the
kernels: the HIP runtime loads device code at a module's first launch), and
a set too large for the scratch is refused before any work."""
import ctypes

import numpy as np
import pytest

from paper_1110_0836_amd import synth
from _common import dev, rhs_err

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")
torch = pytest.importorskip("torch")


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Ctx:
    """A context of its own (its workspace starts empty), on torch's stream."""

    def __init__(self):
        self.c = ctypes.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        assert P.lib().phb_create(ctypes.byref(self.c), torch.cuda.current_device(),
                                  ctypes.c_void_p(stream)) == P.PHB_OK

    def close(self):
        P.lib().phb_destroy(self.c)


def call(entry, ctx, c, setup, lists, tape=False):
    pos, lam, q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
    off, idx = lists
    n = c["lam"].shape[0]
    rhs = torch.full((8, n), np.nan, dtype=torch.float64, device="cuda")
    dxdt = torch.full((3, n), np.nan, dtype=torch.float64, device="cuda")
    st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    tp = (torch.zeros(P.phb_tape_bytes(n) // 8, dtype=torch.float64, device="cuda")
          if tape else None)
    p = setup.params()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rc = getattr(P.lib(), entry)(ctx.c, ctypes.byref(p), n, ptr(pos), ptr(lam), ptr(off),
                                 ptr(idx), ptr(q), ptr(rhs), ptr(dxdt), ptr(st), ptr(tp))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert rc == P.PHB_OK, P.lib().phb_last_error(ctx.c)
    out = (rhs.cpu().numpy(), dxdt.cpu().numpy(), st.cpu().numpy(),
           None if tp is None else tp.cpu().numpy())
    return out, free0 - free1


def compare(a, b, q):
    assert np.array_equal(a[2], b[2])
    ok = a[2] == 0
    e = rhs_err(a[0][:, ok], b[0][:, ok])
    print("allocation-free against allocating, max rel err per quantity", e,
          "identical:", np.array_equal(a[0][:, ok], b[0][:, ok]))
    assert max(e.values()) <= 1e-12
    assert np.array_equal(a[1], b[1])
    assert np.all(np.isnan(a[0][:, ~ok]))
    if a[3] is not None:
        assert np.array_equal(a[3], b[3])


def lists_of(c, setup):
    return P.neighbors(dev(c["pos"]), dev(c["lam"]), setup)


def test_two_calls_match_the_allocating_entry_point():
    # The HIP runtime loads a module's device code at its first kernel launch
    # in the process (its own allocation, not the library's): one small
    # warm-up call of each precision runs the kernels once first.
    for kw in ({}, {"precision": P.PHB_MIXED}):
        c = synth.cp_alfven(6)
        s = P.Setup(L=c["L"], periodic=c["periodic"], gamma=c["gamma"], **kw)
        warm = Ctx()
        try:
            _, grew = call("phb_mhd_rhs_noalloc", warm, c, s, lists_of(c, s), True)
            print("warm-up call (first kernel launches of the process):", grew, "bytes")
        finally:
            warm.close()
    # first call: 8,000 particles, FP64, with a tape; second: 1,728, mixed
    runs = [(synth.fast_wave_set(side=20), {}, True),
            (synth.cp_alfven(12), {"precision": P.PHB_MIXED}, False)]
    for c, kw, tape in runs:
        s = P.Setup(L=c["L"], periodic=c["periodic"], gamma=c["gamma"], **kw)
        lists = lists_of(c, s)
        fresh = Ctx()
        try:
            na, grew = call("phb_mhd_rhs_noalloc", fresh, c, s, lists, tape)
            print(f"n = {c['lam'].shape[0]}: free device memory change across the "
                  f"allocation-free call {grew} bytes")
            assert grew == 0
            ref, grew_ref = call("phb_mhd_rhs", fresh, c, s, lists, tape)
            print("the allocating call on the same fresh context took", grew_ref, "bytes")
        finally:
            fresh.close()
        compare(na, ref, c["q"])


def test_too_large_a_set_is_refused():
    c = synth.fast_wave_set(side=40)  # 64,000 particles: more than the scratch holds
    s = P.Setup(L=c["L"], periodic=c["periodic"], gamma=c["gamma"])
    fresh = Ctx()
    try:
        n = c["lam"].shape[0]
        pos, lam, q = dev(c["pos"]), dev(c["lam"]), dev(c["q"])
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        idx = torch.zeros(1, dtype=torch.int32, device="cuda")
        rhs = torch.zeros((8, n), dtype=torch.float64, device="cuda")
        dxdt = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        rc = P.lib().phb_mhd_rhs_noalloc(fresh.c, ctypes.byref(s.params()), n, ptr(pos),
                                         ptr(lam), ptr(off), ptr(idx), ptr(q), ptr(rhs),
                                         ptr(dxdt), ptr(st), None)
        assert rc == P.PHB_ECAPACITY
        assert b"scratch" in P.lib().phb_last_error(fresh.c)
        torch.cuda.synchronize()
        assert float(rhs.abs().max()) == 0.0  # nothing ran
    finally:
        fresh.close()
