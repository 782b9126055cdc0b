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
    den = rhs_dens(o, q, d1, gamma)
    return {k: float(np.abs(g[v] - o[v]).max() / den[k]) for k, v in GROUPS.items()}


def rhs_particle_err(g, o, q=None, d1=None, gamma=5.0 / 3.0):
    """Per-particle form of rhs_err: for each particle the largest error over
    the physical quantities, each over the same denominator as rhs_err."""
    g = np.asarray(g)
    o = np.asarray(o)
    den = rhs_dens(o, q, d1, gamma)
    return np.max([np.abs(g[v] - o[v]).max(axis=0) / den[k] for k, v in GROUPS.items()], axis=0)


def rhs_dens(o, q=None, d1=None, gamma=5.0 / 3.0):
    """The per-quantity denominators of rhs_err."""
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
    return {k: max(np.abs(o[v]).max(), floor[k], 1e-300) for k, v in GROUPS.items()}


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


def fit_kappa(pos, lam, off, idx, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), rf_ratio=2.3, fit=0):
    """2-norm condition number of each particle's equilibrated moment matrix
    (unit diagonal; the matrix of the weighted 20-monomial fit, or of the 19
    non-constant monomials for the interpolating fit), from the given lists;
    inf below 20 entries.  A tolerance helper: the fit's accuracy in FP64 is
    about kappa(P) eps = sqrt(kappa) eps by QR and kappa eps by the normal
    equations."""
    pos = np.asarray(pos)
    lam = np.asarray(lam)
    off = np.asarray(off)
    idx = np.asarray(idx)
    n = lam.shape[0]
    out = np.full(n, np.inf)
    for i in range(n):
        nb = idx[off[i]:off[i + 1]]
        if len(nb) < 20:
            continue
        d = pos[:, nb] - pos[:, i:i + 1]
        for a in range(3):
            if periodic[a]:
                d[a] = np.where(d[a] > 0.5 * L[a], d[a] - L[a], d[a])
                d[a] = np.where(d[a] < -0.5 * L[a], d[a] + L[a], d[a])
        r2 = (rf_ratio * lam[i]) ** 2
        w = (1.0 - (d * d).sum(0) / r2) ** 3
        x, y, z = d / lam[i]
        P = np.stack([np.ones_like(x), x, y, z, x * x, x * y, x * z, y * y, y * z, z * z,
                      x ** 3, x * x * y, x * x * z, x * y * y, x * y * z, x * z * z, y ** 3,
                      y * y * z, y * z * z, z ** 3], axis=1)
        if fit == 1:
            P = P[:, 1:]
        A = (P * w[:, None]).T @ P
        s = 1.0 / np.sqrt(np.diag(A))
        out[i] = np.linalg.cond(A * s[:, None] * s[None, :])
    return out


EPS64 = float(np.finfo(np.float64).eps)
# Constant of the condition-scaled bound: the oracle's QR loses up to about
# 10 kappa(P) eps on the open-box and graded sets (measured against the exact
# cubic and against refined fits), and 64 leaves room for the GPU's own share.
KAPPA_C = 64.0


def kappa_tol(kappa, base=1e-12, c=KAPPA_C):
    """Per-particle bound of the FP64 parity tests: base (1e-12 of the largest
    value, the metric's own bar) plus c kappa(P) eps = c sqrt(kappa) eps, the
    accuracy of a backward-stable fit of that condition -- the oracle's QR is
    exact only to that, so no evaluation can agree with it more closely."""
    k = np.where(np.isfinite(kappa), kappa, 0.0)
    return base + c * np.sqrt(k) * EPS64


def kappa_tol_adj(kappa, base=1e-12, c=KAPPA_C):
    """Bound of a reverse-mode entry, kappa of the worst fit it receives a
    contribution from: kappa_tol plus kappa eps / 32.  The reverse mode applies
    rows of the inverse to monomial vectors of every neighbor (the oracle's
    Bbar^T p, the GPU's G p), and for a fit of condition kappa those products
    cancel to kappa eps whatever the factorization: the oracle's own reverse
    mode is that far from the complex-step derivative of its forward map at the
    worst-conditioned fits (measured up to 0.004 kappa eps; the GPU's own
    difference from the oracle, up to 0.013 kappa eps)."""
    k = np.where(np.isfinite(kappa), kappa, 0.0)
    return kappa_tol(kappa, base, c) + k * EPS64 / 32.0


def kappa_spread(kappa, off, idx):
    """For each particle, the largest kappa among the owners whose lists hold
    it (itself included): the fits its reverse-mode entries come from."""
    k = np.where(np.isfinite(kappa), kappa, 0.0)
    off = np.asarray(off)
    idx = np.asarray(idx)
    owner = np.repeat(np.arange(len(off) - 1), np.diff(off))
    out = k.copy()
    np.maximum.at(out, idx, k[owner])
    return out


def particle_err(g, o, sel=None):
    """Per-particle error of (..., n) arrays against the oracle: max over the
    leading axes of |g - o| / max |o| (the denominator over all components and
    the selected particles, as in rel_err)."""
    g = np.asarray(g)
    o = np.asarray(o)
    if sel is not None:
        g = g[..., sel]
        o = o[..., sel]
    den = max(np.abs(o).max(), 1e-300)
    return (np.abs(g - o) / den).reshape(-1, g.shape[-1]).max(axis=0)
