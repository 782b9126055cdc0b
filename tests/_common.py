"""Shared test helpers: moving seeded numpy inputs to the GPU and the
relative max-error metric used for every FP parity check:
    e = max_i |g_i - o_i| / max_i |o_i|   over particles with status 0,
taken per field and derivative order."""
import numpy as np


def dev(a, dtype=None):
    """Copy a numpy array to the GPU (dtype: a numpy or torch dtype)."""
    import torch
    if dtype is not None and not isinstance(dtype, torch.dtype):
        a = np.asarray(a, dtype=dtype)
        dtype = None
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def setup_of(c, **kw):
    import paper_1110_0836_amd as P
    return P.Setup(L=tuple(c["L"]), periodic=tuple(c["periodic"]), gamma=c.get("gamma", 5 / 3),
                   **kw)


def rel_err(g, o, axis=None):
    g = np.asarray(g)
    o = np.asarray(o)
    den = np.abs(o).max(axis=axis)
    num = np.abs(g - o).max(axis=axis)
    return num / np.maximum(den, 1e-300)


GROUPS = {"rho": [0], "V": [1, 2, 3], "B": [4, 5, 6], "sigma": [7]}


def rhs_err(g, o, q=None, d1=None, gamma=5.0 / 3.0):
    """Max relative error of (8, m) time derivatives per physical quantity.
    Components of a vector share one denominator (a component that vanishes
    identically, such as dBx/dt of a plane wave along x, is judged against
    the size of its vector).  Given the fields q (8, m) and their first
    derivatives d1 (8, 3, m), the denominator is at least the size of the
    terms each quantity is summed from, e.g. |rho| max|grad V| for drho/dt:
    a time derivative that cancels to far below its terms (div V of a
    shear flow) cannot be held to 1e-12 of its own size by any evaluation."""
    g = np.asarray(g)
    o = np.asarray(o)
    floor = {k: 0.0 for k in GROUPS}
    if q is not None and d1 is not None:
        q = np.asarray(q)
        d1 = np.asarray(d1)
        gv = np.abs(d1[1:4]).max()
        gb = np.abs(d1[4:7]).max()
        gs = np.abs(d1[7]).max()
        bmax = np.abs(q[4:7]).max()
        rmin = np.abs(q[0]).min()
        floor = {"rho": np.abs(q[0]).max() * gv,
                 "V": ((gamma - 1) * gs + bmax * gb) / rmin,
                 "B": bmax * gv,
                 "sigma": gamma * np.abs(q[7]).max() * gv}
    return {k: float(np.abs(g[v] - o[v]).max() / max(np.abs(o[v]).max(), floor[k], 1e-300))
            for k, v in GROUPS.items()}


def interior(pos, lam, L, periodic, rf_ratio=2.3):
    """Particles whose whole sphere lies inside the box on every open axis."""
    pos = np.asarray(pos)
    r = rf_ratio * np.asarray(lam)
    ok = np.ones(pos.shape[1], bool)
    for a in range(3):
        if not periodic[a]:
            ok &= (pos[a] > r) & (pos[a] < L[a] - r)
    return ok


def csr_rows(off, idx):
    off = np.asarray(off)
    idx = np.asarray(idx)
    return [idx[off[i]:off[i + 1]] for i in range(len(off) - 1)]
