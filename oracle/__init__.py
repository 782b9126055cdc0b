"""CPU FP64 oracle for the Phurbas MLS / ideal-MHD hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg may call it; the product path never does.
It shares no code with the GPU library.  The arithmetic lives in
``phurbas_oracle.cpp`` (plain C++17 + OpenMP); this module only marshals
numpy arrays through ctypes.

Array layouts are structure-of-arrays, FP64, particle index last:
``pos`` (3, n), ``lam`` (n,), ``q`` (8, n) with fields
(rho, Vx, Vy, Vz, Bx, By, Bz, sigma).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phurbas_oracle.cpp")
_LIB = os.path.join(_HERE, "liborc.so")

RF_RATIO = 2.3


def build(force: bool = False) -> str:
    """Compile the oracle shared library in place (g++, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        D = ctypes.c_double
        L.orc_neighbors.restype = I64
        L.orc_neighbors.argtypes = [I64, P, P, P, P, D, I64, P, P, P, I64, I]
        L.orc_mls_derivs.restype = I
        L.orc_mls_derivs.argtypes = [I64, P, P, P, P, D, I, I, I64, P, P, P, I, P, P, P, P, I]
        L.orc_mhd_rhs.restype = I
        L.orc_mhd_rhs.argtypes = [I64, P, P, P, P, D, D, I, I, I64, P, P, P, P, P, P, P, I, P]
        L.orc_mhd_rhs_cstep.restype = I
        L.orc_mhd_rhs_cstep.argtypes = [I64, P, P, P, P, D, D, I, I, P, P, P, P, P, D, P, P, P, I,
                                       P]
        L.orc_mhd_rhs_adjoint.restype = I
        L.orc_mhd_rhs_adjoint.argtypes = [I64, P, P, P, P, D, D, I, I, P, P, P, P, P, P, P, P, I,
                                         P]
        L.orc_adjoint_sampled.restype = I
        L.orc_adjoint_sampled.argtypes = [I64, P, P, P, P, D, D, I, I, P, P, P, I64, P, P, P, I,
                                         P]
        L.orc_adjoint_rows.restype = I
        L.orc_adjoint_rows.argtypes = [I64, P, P, P, P, D, D, I, I, I64, P, P, P, P, P, P, P,
                                       P, I, P]
        L.orc_pc_step.restype = I
        L.orc_pc_step.argtypes = [I64, P, P, P, P, P, D, D, I, I, D, P, I, P]
        L.orc_evolve.restype = I
        L.orc_evolve.argtypes = [I64, P, P, P, P, P, D, D, I, I, D, I, P, P, I, P]
        L.orc_divb_norm.restype = I
        L.orc_divb_norm.argtypes = [I64, P, P, P, P, D, I, I, I64, P, P, P, P, P, P, I]
        L.orc_evolve_blocks.restype = I
        L.orc_evolve_blocks.argtypes = [I64, P, P, P, P, P, D, D, I, I, D, I, D, I, P, P, P, P,
                                        I, P]
        L.orc_courant_dt.restype = D
        L.orc_courant_dt.argtypes = [I64, P, P, D, P, D, P]
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _box(L, periodic):
    return _c(L, np.float64), _c(periodic, np.int32)


def _stab(stab):
    """None (ideal MHD) or the stabiliser coefficients (visc_grid, visc_adapt,
    divb_diff) as a float64 array."""
    if stab is None:
        return None
    a = _c(stab, np.float64)
    if a.shape != (3,):
        raise ValueError("stab must hold (visc_grid, visc_adapt, divb_diff)")
    return a


def neighbors(pos, lam, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), rows=None, threads=0,
              rf_ratio=RF_RATIO):
    """Brute-force neighbor CSR (offsets int64, idx int32) for ``rows`` (default all)."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    rows_a = None if rows is None else _c(rows, np.int64)
    nrows = n if rows_a is None else rows_a.shape[0]
    off = np.zeros(nrows + 1, np.int64)
    nnz = lib().orc_neighbors(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, nrows, _p(rows_a),
                              _p(off), None, 0, threads)
    if nnz < 0:
        raise ValueError("orc_neighbors: invalid arguments")
    idx = np.zeros(max(nnz, 1), np.int32)
    lib().orc_neighbors(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, nrows, _p(rows_a),
                        _p(off), _p(idx), nnz, threads)
    return off, idx[:nnz]


def mls_derivs(pos, lam, off, idx, fields, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), rows=None,
               second=True, weight=0, fit=0, threads=0, rf_ratio=RF_RATIO):
    """First (nf,3,nrows) and second (nf,6,nrows) derivatives and status (nrows,)."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    fields = _c(fields, np.float64)
    n = lam.shape[0]
    nf = fields.shape[0]
    Lb, pb = _box(L, periodic)
    rows_a = None if rows is None else _c(rows, np.int64)
    nrows = n if rows_a is None else rows_a.shape[0]
    off = _c(off, np.int64)
    idx = _c(idx, np.int32)
    d1 = np.zeros((nf, 3, nrows))
    d2 = np.zeros((nf, 6, nrows)) if second else None
    st = np.zeros(nrows, np.int32)
    rc = lib().orc_mls_derivs(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, weight, fit, nrows,
                              _p(rows_a), _p(off), _p(idx), nf, _p(fields), _p(d1), _p(d2),
                              _p(st), threads)
    if rc != 0:
        raise ValueError("orc_mls_derivs: invalid arguments")
    return d1, d2, st


def mhd_rhs(pos, lam, off, idx, q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=5.0 / 3.0,
            rows=None, weight=0, fit=0, threads=0, rf_ratio=RF_RATIO, stab=None):
    """MHD time derivatives: rhs (8,nrows), dxdt (3,nrows), status (nrows,).
    stab: None (ideal) or (visc_grid, visc_adapt, divb_diff)."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    q = _c(q, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    rows_a = None if rows is None else _c(rows, np.int64)
    nrows = n if rows_a is None else rows_a.shape[0]
    off = _c(off, np.int64)
    idx = _c(idx, np.int32)
    rhs = np.zeros((8, nrows))
    dxdt = np.zeros((3, nrows))
    st = np.zeros(nrows, np.int32)
    rc = lib().orc_mhd_rhs(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight, fit,
                           nrows, _p(rows_a), _p(off), _p(idx), _p(q), _p(rhs), _p(dxdt), _p(st),
                           threads, _p(_stab(stab)))
    if rc != 0:
        raise ValueError("orc_mhd_rhs: invalid arguments")
    return rhs, dxdt, st


def mhd_rhs_cstep(pos, lam, off, idx, q, dpos=None, dq=None, h=1e-30, L=(1.0, 1.0, 1.0),
                  periodic=(1, 1, 1), gamma=5.0 / 3.0, weight=0, fit=0, threads=0,
                  rf_ratio=RF_RATIO, stab=None):
    """Complex-step directional derivative of the RHS along (dpos, dq): (rhs, d rhs, status)."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    q = _c(q, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    dpos = None if dpos is None else _c(dpos, np.float64)
    dq = None if dq is None else _c(dq, np.float64)
    rre = np.zeros((8, n))
    rdir = np.zeros((8, n))
    st = np.zeros(n, np.int32)
    rc = lib().orc_mhd_rhs_cstep(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight,
                                 fit, _p(_c(off, np.int64)), _p(_c(idx, np.int32)), _p(q),
                                 _p(dpos), _p(dq), h, _p(rre), _p(rdir), _p(st), threads,
                                 _p(_stab(stab)))
    if rc != 0:
        raise ValueError("orc_mhd_rhs_cstep: invalid arguments")
    return rre, rdir, st


def mhd_rhs_adjoint(pos, lam, off, idx, q, rhs_bar, dxdt_bar=None, L=(1.0, 1.0, 1.0),
                    periodic=(1, 1, 1), gamma=5.0 / 3.0, weight=0, fit=0, threads=0,
                    rf_ratio=RF_RATIO, stab=None):
    """Reverse-mode gradient (q_bar (8,n), pos_bar (3,n), status) of rhs_bar.rhs + dxdt_bar.dxdt."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    q = _c(q, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    rb = _c(rhs_bar, np.float64)
    xb = None if dxdt_bar is None else _c(dxdt_bar, np.float64)
    qbar = np.zeros((8, n))
    pbar = np.zeros((3, n))
    st = np.zeros(n, np.int32)
    rc = lib().orc_mhd_rhs_adjoint(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight,
                                   fit, _p(_c(off, np.int64)), _p(_c(idx, np.int32)), _p(q),
                                   _p(rb), _p(xb), _p(qbar), _p(pbar), _p(st), threads,
                                   _p(_stab(stab)))
    if rc != 0:
        raise ValueError("orc_mhd_rhs_adjoint: invalid arguments")
    return qbar, pbar, st


def adjoint_rows(pos, lam, off, idx, q, rhs_bar, rows, dxdt_bar=None, L=(1.0, 1.0, 1.0),
                 periodic=(1, 1, 1), gamma=5.0 / 3.0, weight=0, fit=0, threads=0,
                 rf_ratio=RF_RATIO, stab=None):
    """Contributions of the owner ``rows`` (CSR restricted to them) to (q_bar, pos_bar)."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    q = _c(q, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    r = _c(rows, np.int64)
    qbar = np.zeros((8, n))
    pbar = np.zeros((3, n))
    xb = None if dxdt_bar is None else _c(dxdt_bar, np.float64)
    rc = lib().orc_adjoint_rows(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight, fit,
                                r.shape[0], _p(r), _p(_c(off, np.int64)), _p(_c(idx, np.int32)),
                                _p(q), _p(_c(rhs_bar, np.float64)), _p(xb), _p(qbar), _p(pbar),
                                threads, _p(_stab(stab)))
    if rc != 0:
        raise ValueError("orc_adjoint_rows: invalid arguments")
    return qbar, pbar


def adjoint_sampled(pos, lam, q, rhs_bar, samples, dxdt_bar=None, L=(1.0, 1.0, 1.0),
                    periodic=(1, 1, 1), gamma=5.0 / 3.0, weight=0, fit=0, threads=0,
                    rf_ratio=RF_RATIO, stab=None):
    """Gradient columns (8,ns) and (3,ns) for the sampled particle indices, at any n."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    q = _c(q, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    s = _c(samples, np.int64)
    ns = s.shape[0]
    qs = np.zeros((8, ns))
    ps = np.zeros((3, ns))
    xb = None if dxdt_bar is None else _c(dxdt_bar, np.float64)
    rc = lib().orc_adjoint_sampled(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight,
                                   fit, _p(q), _p(_c(rhs_bar, np.float64)), _p(xb), ns, _p(s),
                                   _p(qs), _p(ps), threads, _p(_stab(stab)))
    if rc != 0:
        raise ValueError("orc_adjoint_sampled: invalid arguments")
    return qs, ps


def pc_step(pos, lam, q, dt, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=5.0 / 3.0, weight=0,
            fit=0, threads=0, rf_ratio=RF_RATIO, stab=None):
    """One predictor-corrector step; returns new (pos, q, status)."""
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    lam = _c(lam, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    st = np.zeros(n, np.int32)
    rc = lib().orc_pc_step(n, _p(pos), _p(q), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight,
                           fit, dt, _p(st), threads, _p(_stab(stab)))
    if rc == -1:
        raise ValueError("orc_pc_step: invalid arguments")
    if rc == -2:
        raise ValueError("orc_pc_step: a particle left the box on a non-periodic axis")
    return pos, q, st


def evolve(pos, lam, q, dt, nsteps, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=5.0 / 3.0,
           frozen=None, weight=0, fit=0, threads=0, rf_ratio=RF_RATIO, stab=None):
    """nsteps predictor-corrector steps (frozen: optional mask of particles held
    fixed); returns new (pos, q, status)."""
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    lam = _c(lam, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    fz = None if frozen is None else _c(frozen, np.int32)
    st = np.zeros(n, np.int32)
    rc = lib().orc_evolve(n, _p(pos), _p(q), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma, weight,
                          fit, dt, int(nsteps), _p(fz), _p(st), threads, _p(_stab(stab)))
    if rc == -1:
        raise ValueError("orc_evolve: invalid arguments")
    if rc == -2:
        raise ValueError("orc_evolve: a particle left the box on a non-periodic axis")
    return pos, q, st


def courant_dt(q, lam, cfl=0.3, gamma=5.0 / 3.0, frozen=None, stab=None):
    """cfl * min lambda / (c_fast (1 + 2 sum(stab))) over non-frozen particles."""
    q = _c(q, np.float64)
    lam = _c(lam, np.float64)
    fz = None if frozen is None else _c(frozen, np.int32)
    dt = lib().orc_courant_dt(lam.shape[0], _p(q), _p(lam), gamma, _p(fz), cfl,
                              _p(_stab(stab)))
    if dt < 0:
        raise ValueError("orc_courant_dt: no particle to time-step")
    return dt


def divb_norm(pos, lam, off, idx, q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), rows=None,
              weight=0, fit=0, threads=0, rf_ratio=RF_RATIO):
    """lambda (div B) / |B| per particle (Sec. 3.3) and the fit status."""
    pos = _c(pos, np.float64)
    lam = _c(lam, np.float64)
    q = _c(q, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    rows_a = None if rows is None else _c(rows, np.int64)
    nrows = n if rows_a is None else rows_a.shape[0]
    out = np.zeros(nrows)
    st = np.zeros(nrows, np.int32)
    rc = lib().orc_divb_norm(n, _p(pos), _p(lam), _p(Lb), _p(pb), rf_ratio, weight, fit, nrows,
                             _p(rows_a), _p(_c(off, np.int64)), _p(_c(idx, np.int32)), _p(q),
                             _p(out), _p(st), threads)
    if rc != 0:
        raise ValueError("orc_divb_norm: invalid arguments")
    return out, st


def bin_mean(coord, values, x0, width, nbins):
    """Mean of the finite values per bin [x0 + b width, x0 + (b+1) width) of
    coord (Sec. 3.3 bins the div-B diagnostic in bins one lambda wide), by
    plain loops: (mean (nbins,), NaN for empty bins; count (nbins,))."""
    total = [0.0] * nbins
    count = [0] * nbins
    for x, v in zip(np.asarray(coord, dtype=np.float64).tolist(),
                    np.asarray(values, dtype=np.float64).tolist()):
        if v != v:
            continue
        b = int(np.floor((x - x0) / width))
        if 0 <= b < nbins:
            total[b] += v
            count[b] += 1
    mean = np.array([t / c if c else np.nan for t, c in zip(total, count)])
    return mean, np.array(count, dtype=np.int64)


def evolve_blocks(pos, lam, q, dt_max, nblocks, cfl=0.3, kmax=20, L=(1.0, 1.0, 1.0),
                  periodic=(1, 1, 1), gamma=5.0 / 3.0, frozen=None, weight=0, fit=0, threads=0,
                  rf_ratio=RF_RATIO, stab=None):
    """nblocks periods of dt_max with individual power-of-two steps; returns
    (pos, q, status, levels (n,), stats (step-end times, particle evaluations))."""
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    lam = _c(lam, np.float64)
    n = lam.shape[0]
    Lb, pb = _box(L, periodic)
    fz = None if frozen is None else _c(frozen, np.int32)
    st = np.zeros(n, np.int32)
    lev = np.zeros(n, np.int32)
    stats = np.zeros(2, np.int64)
    rc = lib().orc_evolve_blocks(n, _p(pos), _p(q), _p(lam), _p(Lb), _p(pb), rf_ratio, gamma,
                                 weight, fit, float(dt_max), int(nblocks), float(cfl), int(kmax),
                                 _p(fz), _p(st), _p(lev), _p(stats), threads, _p(_stab(stab)))
    if rc == -1:
        raise ValueError("orc_evolve_blocks: invalid arguments")
    if rc == -2:
        raise ValueError("orc_evolve_blocks: a particle left the box on a non-periodic axis")
    return pos, q, st, lev, stats
