"""Python binding of libphurbas, the MI355X implementation of the Phurbas
moving-least-squares / ideal-MHD hot path (McNally, Maron & Mac Low, paper II).

Argument marshalling only: every step runs in the library's HIP kernels.
Tensors must be contiguous CUDA (ROCm) tensors; FP64 for real data, int64
offsets and int32 indices.  Work is enqueued on torch's current stream.

The functions named ``phb_*`` mirror the C entry points of include/phurbas.h
one to one; the lower-case helpers allocate outputs with torch and call them.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphurbas.so")

PHB_OK = 0
PHB_EINVAL = -1
PHB_ENOMEM = -2
PHB_ECAPACITY = -3
PHB_EHIP = -4
PHB_ESTATE = -5
PHB_ENOTIMPL = -6
PHB_FP64 = 0
PHB_MIXED = 1
PHB_W_POLY3 = 0
PHB_W_UNIT = 1
PHB_FIT_FULL20 = 0
PHB_FIT_INTERP19 = 1
PHB_NB_OVERFLOW = 1
PHB_NB_INVALID = 2
PHB_NB_RADIUS = 4

EXPORTS = [
    "phb_create", "phb_destroy", "phb_set_stream", "phb_reserve", "phb_strerror",
    "phb_last_error", "phb_neighbors_build", "phb_neighbors_transpose", "phb_spatial_order",
    "phb_permute", "phb_mls_derivs", "phb_mhd_rhs", "phb_tape_bytes", "phb_mhd_rhs_adjoint",
    "phb_pc_step", "phb_profile", "phb_profile_read", "phb_tune_set", "phb_tune_get",
    "phb_evolve", "phb_courant_dt", "phb_tune", "phb_batch_create", "phb_batch_destroy", "phb_batch_neighbors", "phb_batch_run",
    "phb_batch_capture", "phb_batch_launch", "phb_divb_norm", "phb_bin_mean",
    "phb_neighbors_build_rows", "phb_mhd_rhs_rows", "phb_evolve_blocks", "phb_mhd_rhs_noalloc",
    "phb_neighbors_build_async", "phb_mhd_rhs_adjoint_async",
]


class PhurbasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libphurbas error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("periodic", ctypes.c_int32 * 3),
                ("gamma", ctypes.c_double), ("rf_ratio", ctypes.c_double),
                ("precision", ctypes.c_int32), ("weight", ctypes.c_int32),
                ("fit", ctypes.c_int32), ("visc_grid", ctypes.c_double),
                ("visc_adapt", ctypes.c_double), ("divb_diff", ctypes.c_double)]


class BatchIO(ctypes.Structure):
    """phb_batch_io: the buffers of one batched pass."""
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "pos", "lambda_", "offsets", "idx", "t_offsets", "t_src", "t_pos", "q", "rhs", "dxdt",
        "status", "tape", "rhs_bar", "dxdt_bar", "q_bar", "pos_bar")]


@dataclass
class Setup:
    """Box, physics and numerics options of one particle set."""
    L: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (1, 1, 1)
    gamma: float = 5.0 / 3.0
    rf_ratio: float = 2.3
    precision: int = PHB_FP64
    weight: int = PHB_W_POLY3
    fit: int = PHB_FIT_FULL20
    # non-ideal stabilisers (all zero: ideal MHD); see phb_params
    visc_grid: float = 0.0
    visc_adapt: float = 0.0
    divb_diff: float = 0.0

    @property
    def stab(self):
        """(visc_grid, visc_adapt, divb_diff), or None when all are zero."""
        t = (float(self.visc_grid), float(self.visc_adapt), float(self.divb_diff))
        return t if any(t) else None

    def params(self) -> Params:
        p = Params()
        for a in range(3):
            p.L[a] = float(self.L[a])
            p.periodic[a] = int(self.periodic[a])
        p.gamma = float(self.gamma)
        p.rf_ratio = float(self.rf_ratio)
        p.precision = int(self.precision)
        p.weight = int(self.weight)
        p.fit = int(self.fit)
        p.visc_grid = float(self.visc_grid)
        p.visc_adapt = float(self.visc_adapt)
        p.divb_diff = float(self.divb_diff)
        return p


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        I = ctypes.c_int
        D = ctypes.c_double
        PP = ctypes.POINTER(Params)
        sig = {
            "phb_create": (I, [ctypes.POINTER(P), I, P]),
            "phb_destroy": (I, [P]),
            "phb_set_stream": (I, [P, P]),
            "phb_reserve": (I, [P, I64, I64]),
            "phb_strerror": (ctypes.c_char_p, [I]),
            "phb_last_error": (ctypes.c_char_p, [P]),
            "phb_neighbors_build": (I, [P, PP, I64, P, P, P, P, I64, ctypes.POINTER(I64)]),
            "phb_neighbors_build_async": (I, [P, PP, I64, P, P, P, P, I64, P, P]),
            "phb_neighbors_transpose": (I, [P, I64, I64, P, P, P, P, P]),
            "phb_spatial_order": (I, [P, PP, I64, P, P, P]),
            "phb_permute": (I, [P, I64, P, I32, P, P]),
            "phb_mls_derivs": (I, [P, PP, I64, P, P, P, P, I32, P, I32, P, P, P]),
            "phb_mhd_rhs": (I, [P, PP, I64, P, P, P, P, P, P, P, P, P]),
            "phb_mhd_rhs_noalloc": (I, [P, PP, I64, P, P, P, P, P, P, P, P, P]),
            "phb_tape_bytes": (I64, [I64]),
            "phb_mhd_rhs_adjoint": (I, [P, PP, I64, P, P, P, P, P, P, P, P, P, P, P, P, P]),
            "phb_mhd_rhs_adjoint_async": (I, [P, PP, I64, P, P, P, P, P, P, P, P, P, P, P, P, P,
                                              I64]),
            "phb_pc_step": (I, [P, PP, I64, D, P, P, P, P, P, I64, ctypes.POINTER(I64), P]),
            "phb_profile": (I, [P, I]),
            "phb_tune_set": (I, [P, ctypes.c_char_p, I]),
            "phb_tune_get": (I, [P, ctypes.c_char_p, ctypes.POINTER(I)]),
            "phb_profile_read": (I, [P, I32, P, P, P, ctypes.POINTER(I32)]),
            "phb_evolve": (I, [P, PP, I64, D, I32, P, P, P, P, P, P, I64, ctypes.POINTER(I64),
                               P]),
            "phb_courant_dt": (I, [P, PP, I64, P, P, P, D, ctypes.POINTER(D)]),
            "phb_tune": (I, [P, PP, I64, P, P, P, P, P, P, P, I64, P, I32, ctypes.c_char_p]),
            "phb_batch_create": (I, [P, PP, I32, ctypes.POINTER(I64), ctypes.POINTER(P)]),
            "phb_batch_destroy": (I, [P]),
            "phb_batch_neighbors": (I, [P, P, P, P, P, P, I64, ctypes.POINTER(I64)]),
            "phb_batch_run": (I, [P, P, ctypes.POINTER(BatchIO)]),
            "phb_batch_capture": (I, [P, P, ctypes.POINTER(BatchIO)]),
            "phb_batch_launch": (I, [P, P]),
            "phb_divb_norm": (I, [P, PP, I64, P, P, P, P, P, P, P]),
            "phb_neighbors_build_rows": (I, [P, PP, I64, P, P, I64, P, P, P, I64,
                                             ctypes.POINTER(I64)]),
            "phb_mhd_rhs_rows": (I, [P, PP, I64, P, P, I64, P, P, P, P, P, P, P]),
            "phb_evolve_blocks": (I, [P, PP, I64, D, I32, D, I32, P, P, P, P, P, P, I64, P, P,
                                      P]),
            "phb_bin_mean": (I, [P, I64, P, P, D, D, I32, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


_ctx = {}


def context(device=None):
    """The library context of a device, bound to torch's current stream."""
    if not torch.cuda.is_available():
        raise RuntimeError("libphurbas needs a ROCm GPU; none is visible")
    dev = torch.cuda.current_device() if device is None else int(device)
    c = _ctx.get(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    if c is None:
        c = ctypes.c_void_p()
        _check(None, lib().phb_create(ctypes.byref(c), dev, ctypes.c_void_p(stream)))
        _ctx[dev] = c
    else:
        _check(c, lib().phb_set_stream(c, ctypes.c_void_p(stream)))
    return c


def _check(ctx, rc):
    if rc != PHB_OK:
        msg = lib().phb_last_error(ctx).decode() if ctx is not None else \
            lib().phb_strerror(rc).decode()
        raise PhurbasError(rc, msg)
    return rc


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t):
    if t.dtype != torch.float64:
        raise TypeError("expected float64")
    return _ptr(t)


# ---- C entry points (same names) ---------------------------------------------

def phb_neighbors_build(setup, pos, lam, offsets, idx, capacity):
    ctx = context(pos.device.index)
    nnz = ctypes.c_int64(0)
    p = setup.params()
    rc = lib().phb_neighbors_build(ctx, ctypes.byref(p), lam.shape[0], _f64(pos), _f64(lam),
                                   _ptr(offsets), _ptr(idx), capacity, ctypes.byref(nnz))
    if rc not in (PHB_OK, PHB_ECAPACITY):
        _check(ctx, rc)
    return rc, nnz.value


def phb_neighbors_build_async(setup, pos, lam, offsets, idx, capacity, nnz_dev, flag_dev):
    """The build without host synchronization: nnz_dev (int64[1]) and flag_dev
    (int32[1]) are device tensors that receive the total and the status bits
    (PHB_NB_*)."""
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_neighbors_build_async(ctx, ctypes.byref(p), lam.shape[0], _f64(pos),
                                                _f64(lam), _ptr(offsets), _ptr(idx), capacity,
                                                _ptr(nnz_dev), _ptr(flag_dev)))


def phb_neighbors_transpose(offsets, idx, t_offsets, t_src, t_pos):
    ctx = context(offsets.device.index)
    n = offsets.shape[0] - 1
    _check(ctx, lib().phb_neighbors_transpose(ctx, n, idx.shape[0], _ptr(offsets), _ptr(idx),
                                              _ptr(t_offsets), _ptr(t_src), _ptr(t_pos)))


def phb_spatial_order(setup, pos, lam, perm):
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_spatial_order(ctx, ctypes.byref(p), lam.shape[0], _f64(pos), _f64(lam),
                                        _ptr(perm)))


def phb_permute(perm, src, dst):
    ctx = context(src.device.index)
    n = perm.shape[0]
    ncomp = src.numel() // n
    _check(ctx, lib().phb_permute(ctx, n, _ptr(perm), ncomp, _f64(src), _f64(dst)))


def phb_mls_derivs(setup, pos, lam, offsets, idx, fields, max_order, d1, d2, status):
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_mls_derivs(ctx, ctypes.byref(p), lam.shape[0], _f64(pos), _f64(lam),
                                     _ptr(offsets), _ptr(idx), fields.shape[0], _f64(fields),
                                     max_order, _f64(d1), _ptr(d2), _ptr(status)))


def phb_mhd_rhs(setup, pos, lam, offsets, idx, q, rhs, dxdt, status, tape=None):
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_mhd_rhs(ctx, ctypes.byref(p), lam.shape[0], _f64(pos), _f64(lam),
                                  _ptr(offsets), _ptr(idx), _f64(q), _f64(rhs), _f64(dxdt),
                                  _ptr(status), _ptr(tape)))


def phb_mhd_rhs_noalloc(setup, pos, lam, offsets, idx, q, rhs, dxdt, status, tape=None):
    """phb_mhd_rhs without any allocation: the library's static scratch holds
    the intermediates (for callers that cannot allocate; size limit in
    include/phurbas.h)."""
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_mhd_rhs_noalloc(ctx, ctypes.byref(p), lam.shape[0], _f64(pos),
                                          _f64(lam), _ptr(offsets), _ptr(idx), _f64(q),
                                          _f64(rhs), _f64(dxdt), _ptr(status), _ptr(tape)))


def phb_tape_bytes(n):
    return lib().phb_tape_bytes(n)


TAPE_ROWS = 31  # per-particle rows at the start of a tape
TAPE_AOS = 340  # doubles per particle in the tape's block that follows them


def tape_rows(tape, n):
    """The tape's (TAPE_ROWS, n) rows as a view: phb_tape_bytes(n) is
    8 (TAPE_ROWS ld + TAPE_AOS n) for rows padded to ld entries."""
    ld = (phb_tape_bytes(n) // 8 - TAPE_AOS * n) // TAPE_ROWS
    return tape[:TAPE_ROWS * ld].view(TAPE_ROWS, ld)[:, :n]


def phb_mhd_rhs_adjoint(setup, pos, lam, offsets, idx, t_offsets, t_src, t_pos, q, rhs_bar,
                        dxdt_bar, q_bar, pos_bar, tape=None):
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_mhd_rhs_adjoint(ctx, ctypes.byref(p), lam.shape[0], _f64(pos),
                                          _f64(lam), _ptr(offsets), _ptr(idx), _ptr(t_offsets),
                                          _ptr(t_src), _ptr(t_pos), _f64(q), _f64(rhs_bar),
                                          _ptr(dxdt_bar), _f64(q_bar), _f64(pos_bar),
                                          _ptr(tape)))


def phb_mhd_rhs_adjoint_async(setup, pos, lam, offsets, idx, t_offsets, t_src, t_pos, q,
                              rhs_bar, dxdt_bar, q_bar, pos_bar, tape, nnz_bound):
    """phb_mhd_rhs_adjoint without the read-back of offsets[n]: nnz_bound sizes
    the pair records (capturable in a HIP graph)."""
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_mhd_rhs_adjoint_async(ctx, ctypes.byref(p), lam.shape[0], _f64(pos),
                                                _f64(lam), _ptr(offsets), _ptr(idx),
                                                _ptr(t_offsets), _ptr(t_src), _ptr(t_pos),
                                                _f64(q), _f64(rhs_bar), _ptr(dxdt_bar),
                                                _f64(q_bar), _f64(pos_bar), _ptr(tape),
                                                int(nnz_bound)))


def phb_reserve(n_max, nnz_max, device=None):
    ctx = context(device)
    _check(ctx, lib().phb_reserve(ctx, int(n_max), int(nnz_max)))


def phb_pc_step(setup, dt, pos, q, lam, offsets, idx, capacity, status):
    ctx = context(pos.device.index)
    p = setup.params()
    nnz = ctypes.c_int64(0)
    rc = lib().phb_pc_step(ctx, ctypes.byref(p), lam.shape[0], float(dt), _f64(pos), _f64(q),
                           _f64(lam), _ptr(offsets), _ptr(idx), capacity, ctypes.byref(nnz),
                           _ptr(status))
    if rc not in (PHB_OK, PHB_ECAPACITY):
        _check(ctx, rc)
    return rc, nnz.value


def phb_evolve(setup, dt, nsteps, pos, q, lam, frozen, offsets, idx, capacity, status):
    ctx = context(pos.device.index)
    p = setup.params()
    nnz = ctypes.c_int64(0)
    rc = lib().phb_evolve(ctx, ctypes.byref(p), lam.shape[0], float(dt), int(nsteps), _f64(pos),
                          _f64(q), _f64(lam), _ptr(frozen), _ptr(offsets), _ptr(idx), capacity,
                          ctypes.byref(nnz), _ptr(status))
    if rc not in (PHB_OK, PHB_ECAPACITY):
        _check(ctx, rc)
    return rc, nnz.value


def phb_courant_dt(setup, q, lam, frozen, cfl):
    ctx = context(q.device.index)
    p = setup.params()
    dt = ctypes.c_double(0.0)
    _check(ctx, lib().phb_courant_dt(ctx, ctypes.byref(p), lam.shape[0], _f64(q), _f64(lam),
                                     _ptr(frozen), float(cfl), ctypes.byref(dt)))
    return dt.value


TUNE_KEYS = ("cells_per_rf", "lanes_moments", "lanes_apply", "lanes_adj_y", "lanes_gather",
             "adj_pairs_mode", "record_order", "mixed_cond_x10", "mixed_refine", "fp64_cut_x10",
             "fit_fields", "moments_mfma")


def phb_tune_set(key, value, device=None):
    ctx = context(device)
    _check(ctx, lib().phb_tune_set(ctx, key.encode(), int(value)))


def phb_tune_get(key, device=None):
    ctx = context(device)
    v = ctypes.c_int(0)
    _check(ctx, lib().phb_tune_get(ctx, key.encode(), ctypes.byref(v)))
    return v.value


def phb_tune(setup, pos, lam, offsets, idx, t_offsets, t_src, t_pos, q, reps=3, cache=None):
    """Autotune the schedule knobs on this set; returns {key: chosen value}."""
    ctx = context(pos.device.index)
    p = setup.params()
    _check(ctx, lib().phb_tune(ctx, ctypes.byref(p), lam.shape[0], _f64(pos), _f64(lam),
                               _ptr(offsets), _ptr(idx), _ptr(t_offsets), _ptr(t_src),
                               _ptr(t_pos), idx.shape[0], _f64(q), int(reps),
                               None if cache is None else os.fsencode(cache)))
    return {k: phb_tune_get(k, pos.device.index) for k in TUNE_KEYS}


def phb_profile(enable, device=None):
    ctx = context(device)
    _check(ctx, lib().phb_profile(ctx, 1 if enable else 0))


def phb_profile_read(device=None, max_entries=64):
    """{kernel name: (total ms, launches)} since profiling was enabled."""
    ctx = context(device)
    names = ctypes.create_string_buffer(64 * max_entries)
    ms = (ctypes.c_double * max_entries)()
    cnt = (ctypes.c_int32 * max_entries)()
    n = ctypes.c_int32(0)
    _check(ctx, lib().phb_profile_read(ctx, max_entries, names, ms, cnt, ctypes.byref(n)))
    out = {}
    for k in range(min(n.value, max_entries)):
        name = names.raw[64 * k:64 * (k + 1)].split(b"\0", 1)[0].decode()
        out[name] = (ms[k], cnt[k])
    return out


# ---- helpers that allocate outputs -------------------------------------------

def neighbors(pos, lam, setup=None, capacity=None):
    """CSR neighbor lists (offsets int64[n+1], idx int32[nnz])."""
    setup = setup or Setup()
    n = lam.shape[0]
    offsets = torch.empty(n + 1, dtype=torch.int64, device=pos.device)
    cap = capacity if capacity is not None else 64 * n
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pos.device)
    rc, nnz = phb_neighbors_build(setup, pos, lam, offsets, idx, cap)
    if rc == PHB_ECAPACITY:
        idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=pos.device)
        rc, nnz = phb_neighbors_build(setup, pos, lam, offsets, idx, nnz)
        _check(context(pos.device.index), rc)
    return offsets, idx[:nnz]


def neighbors_rows(pos, lam, rows, setup=None, capacity=None):
    """CSR lists of the particles rows (int32) among all: (offsets int64[m+1], idx)."""
    setup = setup or Setup()
    m = rows.shape[0]
    ctx = context(pos.device.index)
    p = setup.params()
    offsets = torch.empty(m + 1, dtype=torch.int64, device=pos.device)
    cap = capacity if capacity is not None else 64 * max(m, 1)
    for _ in range(2):
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pos.device)
        nnz = ctypes.c_int64(0)
        rc = lib().phb_neighbors_build_rows(ctx, ctypes.byref(p), lam.shape[0], _f64(pos),
                                            _f64(lam), m, _ptr(rows), _ptr(offsets), _ptr(idx),
                                            cap, ctypes.byref(nnz))
        if rc != PHB_ECAPACITY:
            break
        cap = nnz.value
    _check(ctx, rc)
    return offsets, idx[:nnz.value]


def mhd_rhs_rows(pos, lam, rows, offsets, idx, q, setup=None):
    """Time derivatives of the particles rows only: rhs (8,m), dxdt (3,m), status (m,)."""
    m = rows.shape[0]
    rhs = torch.empty((8, m), dtype=torch.float64, device=q.device)
    dxdt = torch.empty((3, m), dtype=torch.float64, device=q.device)
    st = torch.empty(m, dtype=torch.int32, device=q.device)
    ctx = context(q.device.index)
    p = (setup or Setup()).params()
    _check(ctx, lib().phb_mhd_rhs_rows(ctx, ctypes.byref(p), lam.shape[0], _f64(pos), _f64(lam),
                                       m, _ptr(rows), _ptr(offsets), _ptr(idx), _f64(q),
                                       _ptr(rhs), _ptr(dxdt), _ptr(st)))
    return rhs, dxdt, st


def transpose(offsets, idx):
    n = offsets.shape[0] - 1
    t_off = torch.empty(n + 1, dtype=torch.int64, device=offsets.device)
    t_src = torch.empty(max(idx.shape[0], 1), dtype=torch.int32, device=offsets.device)
    t_pos = torch.empty(max(idx.shape[0], 1), dtype=torch.int32, device=offsets.device)
    phb_neighbors_transpose(offsets, idx, t_off, t_src, t_pos)
    return t_off, t_src[:idx.shape[0]], t_pos[:idx.shape[0]]


def spatial_order(pos, lam, setup=None):
    perm = torch.empty(lam.shape[0], dtype=torch.int32, device=pos.device)
    phb_spatial_order(setup or Setup(), pos, lam, perm)
    return perm


def permute(perm, src):
    dst = torch.empty_like(src)
    phb_permute(perm, src.contiguous(), dst)
    return dst


def mls_derivs(pos, lam, offsets, idx, fields, setup=None, second=True):
    """Physical first (nf,3,n) and second (nf,6,n) derivatives and status (n,)."""
    n = lam.shape[0]
    nf = fields.shape[0]
    d1 = torch.empty((nf, 3, n), dtype=torch.float64, device=pos.device)
    d2 = torch.empty((nf, 6, n), dtype=torch.float64, device=pos.device) if second else None
    st = torch.empty(n, dtype=torch.int32, device=pos.device)
    phb_mls_derivs(setup or Setup(), pos, lam, offsets, idx, fields, 2 if second else 1, d1, d2, st)
    return d1, d2, st


def mhd_rhs(pos, lam, offsets, idx, q, setup=None, tape=False):
    """Ideal-MHD time derivatives rhs (8,n), dxdt (3,n), status (n,) [, tape]."""
    n = lam.shape[0]
    rhs = torch.empty((8, n), dtype=torch.float64, device=pos.device)
    dxdt = torch.empty((3, n), dtype=torch.float64, device=pos.device)
    st = torch.empty(n, dtype=torch.int32, device=pos.device)
    tp = torch.empty(phb_tape_bytes(n) // 8, dtype=torch.float64, device=pos.device) if tape else None
    phb_mhd_rhs(setup or Setup(), pos, lam, offsets, idx, q, rhs, dxdt, st, tp)
    return (rhs, dxdt, st, tp) if tape else (rhs, dxdt, st)


def mhd_rhs_adjoint(pos, lam, offsets, idx, trans, q, rhs_bar, dxdt_bar=None, setup=None,
                    tape=None):
    """Gradients (q_bar (8,n), pos_bar (3,n)) of sum rhs_bar.rhs + dxdt_bar.dxdt."""
    t_off, t_src, t_pos = trans
    q_bar = torch.empty_like(q)
    pos_bar = torch.empty_like(pos)
    phb_mhd_rhs_adjoint(setup or Setup(), pos, lam, offsets, idx, t_off, t_src, t_pos, q,
                        rhs_bar.contiguous(), None if dxdt_bar is None else dxdt_bar.contiguous(),
                        q_bar, pos_bar, tape)
    return q_bar, pos_bar


def pc_step(pos, q, lam, dt, setup=None, capacity=None):
    """One predictor-corrector step in place; returns (status, offsets, idx) of the
    predicted state."""
    setup = setup or Setup()
    n = lam.shape[0]
    offsets = torch.empty(n + 1, dtype=torch.int64, device=pos.device)
    cap = capacity if capacity is not None else 64 * n
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pos.device)
    st = torch.empty(n, dtype=torch.int32, device=pos.device)
    rc, nnz = phb_pc_step(setup, dt, pos, q, lam, offsets, idx, cap, st)
    if rc == PHB_ECAPACITY:
        raise PhurbasError(rc, f"neighbor capacity {cap} < {nnz}; pass capacity=")
    return st, offsets, idx[:nnz]


def evolve(pos, q, lam, dt, nsteps, setup=None, frozen=None, capacity=None):
    """nsteps predictor-corrector steps in place; returns the status (n,)
    (largest over all stages).  frozen: optional int32 (n,) mask of particles
    held fixed."""
    setup = setup or Setup()
    n = lam.shape[0]
    offsets = torch.empty(n + 1, dtype=torch.int64, device=pos.device)
    cap = capacity if capacity is not None else 64 * n
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pos.device)
    st = torch.empty(n, dtype=torch.int32, device=pos.device)
    rc, nnz = phb_evolve(setup, dt, nsteps, pos, q, lam, frozen, offsets, idx, cap, st)
    if rc == PHB_ECAPACITY:
        raise PhurbasError(rc, f"neighbor capacity {cap} < {nnz}; pass capacity=")
    return st


def evolve_blocks(pos, q, lam, dt_max, nblocks, cfl=0.3, kmax=20, setup=None, frozen=None,
                  capacity=None):
    """nblocks periods of dt_max with individual power-of-two steps, in place on
    pos and q; returns (status (n,), levels (n,), (step-end times, particle
    evaluations))."""
    setup = setup or Setup()
    n = lam.shape[0]
    ctx = context(pos.device.index)
    p = setup.params()
    offsets = torch.empty(n + 1, dtype=torch.int64, device=pos.device)
    cap = capacity if capacity is not None else 128 * n
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pos.device)
    st = torch.empty(n, dtype=torch.int32, device=pos.device)
    lev = torch.empty(n, dtype=torch.int32, device=pos.device)
    stats = (ctypes.c_int64 * 2)()
    _check(ctx, lib().phb_evolve_blocks(ctx, ctypes.byref(p), n, float(dt_max), int(nblocks),
                                        float(cfl), int(kmax), _f64(pos), _f64(q), _f64(lam),
                                        _ptr(frozen), _ptr(offsets), _ptr(idx), cap, _ptr(st),
                                        _ptr(lev), stats))
    return st, lev, (int(stats[0]), int(stats[1]))


def courant_dt(q, lam, cfl=0.3, setup=None, frozen=None):
    """Courant step cfl * min lambda / c_fast over non-frozen particles: the fast
    signal speed alone, so a uniform velocity shift leaves the step unchanged."""
    return phb_courant_dt(setup or Setup(), q, lam, frozen, cfl)


def divb_norm(pos, lam, offsets, idx, q, setup=None):
    """lambda (div B) / |B| per particle (Sec. 3.3) and the fit status."""
    n = lam.shape[0]
    out = torch.empty(n, dtype=torch.float64, device=q.device)
    st = torch.empty(n, dtype=torch.int32, device=q.device)
    ctx = context(q.device.index)
    p = (setup or Setup()).params()
    _check(ctx, lib().phb_divb_norm(ctx, ctypes.byref(p), n, _f64(pos), _f64(lam),
                                    _ptr(offsets), _ptr(idx), _f64(q), _ptr(out), _ptr(st)))
    return out, st


def bin_mean(coord, values, x0, width, nbins):
    """Mean of the finite values in bins of width `width` from x0 along coord:
    (mean (nbins,) with NaN for empty bins, count (nbins,) int64)."""
    mean = torch.empty(nbins, dtype=torch.float64, device=values.device)
    count = torch.empty(nbins, dtype=torch.int64, device=values.device)
    ctx = context(values.device.index)
    _check(ctx, lib().phb_bin_mean(ctx, values.shape[0], _f64(coord), _f64(values), float(x0),
                                   float(width), int(nbins), _ptr(mean), _ptr(count)))
    return mean, count


class MHDRHS(torch.autograd.Function):
    """rhs, dxdt = MHDRHS.apply(q, pos, lam, offsets, idx, trans, setup).

    Differentiable in q (8,n) and pos (3,n) with the neighbor lists held fixed;
    the backward pass runs the library's reverse-mode kernels."""

    @staticmethod
    def forward(ctx, q, pos, lam, offsets, idx, trans, setup):
        q = q.detach().contiguous()
        pos = pos.detach().contiguous()
        rhs, dxdt, st, tp = mhd_rhs(pos, lam, offsets, idx, q, setup=setup, tape=True)
        ctx.save_for_backward(q, pos, lam, offsets, idx, *trans, tp)
        ctx.setup = setup
        ctx.mark_non_differentiable(st)
        return rhs, dxdt, st

    @staticmethod
    def backward(ctx, g_rhs, g_dxdt, g_st):
        q, pos, lam, offsets, idx, t_off, t_src, t_pos, tp = ctx.saved_tensors
        if g_rhs is None:
            g_rhs = torch.zeros((8, lam.shape[0]), dtype=torch.float64, device=q.device)
        q_bar, pos_bar = mhd_rhs_adjoint(pos, lam, offsets, idx, (t_off, t_src, t_pos), q,
                                         g_rhs, g_dxdt, setup=ctx.setup, tape=tp)
        return q_bar, pos_bar, None, None, None, None, None


class Batch:
    """Independent particle sets evaluated as one concatenation and replayed
    from one captured HIP graph (phb_batch_*).

    sizes: particle count of each set; the sets are stored one after the
    other in every SoA array.  All sets share `setup`."""

    def __init__(self, sizes, setup=None, device=None):
        self.setup = setup or Setup()
        self.sizes = [int(v) for v in sizes]
        off = [0]
        for v in self.sizes:
            off.append(off[-1] + v)
        self.set_offsets = off
        self.n = off[-1]
        self._dev = torch.cuda.current_device() if device is None else int(device)
        ctx = context(self._dev)
        arr = (ctypes.c_int64 * len(off))(*off)
        self._p = self.setup.params()
        self._h = ctypes.c_void_p()
        _check(ctx, lib().phb_batch_create(ctx, ctypes.byref(self._p), len(self.sizes), arr,
                                           ctypes.byref(self._h)))
        self._bound = None
        self.nnz = None

    def close(self):
        if self._h:
            torch.cuda.synchronize(self._dev)
            lib().phb_batch_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def neighbors(self, pos, lam, capacity=None):
        """Global CSR lists of all sets: (offsets int64[n+1], idx int32[nnz])."""
        ctx = context(self._dev)
        offsets = torch.empty(self.n + 1, dtype=torch.int64, device=pos.device)
        cap = capacity if capacity is not None else 64 * self.n
        for _ in range(2):
            idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pos.device)
            nnz = ctypes.c_int64(0)
            rc = lib().phb_batch_neighbors(ctx, self._h, _f64(pos), _f64(lam), _ptr(offsets),
                                           _ptr(idx), cap, ctypes.byref(nnz))
            if rc != PHB_ECAPACITY:
                break
            cap = nnz.value
        _check(ctx, rc)
        self.nnz = nnz.value
        return offsets, idx[:nnz.value]

    def _io(self, pos, lam, offsets, idx, q, rhs, dxdt, status, tape=None, trans=None,
            rhs_bar=None, dxdt_bar=None, q_bar=None, pos_bar=None):
        t_off, t_src, t_pos = trans if trans is not None else (None, None, None)
        tensors = dict(pos=pos, lambda_=lam, offsets=offsets, idx=idx, t_offsets=t_off,
                       t_src=t_src, t_pos=t_pos, q=q, rhs=rhs, dxdt=dxdt, status=status,
                       tape=tape, rhs_bar=rhs_bar, dxdt_bar=dxdt_bar, q_bar=q_bar,
                       pos_bar=pos_bar)
        io = BatchIO(**{k: (None if v is None else _ptr(v).value) for k, v in tensors.items()})
        return io, tensors

    def run(self, *args, **kw):
        """One eager pass (arguments as for capture)."""
        io, _ = self._io(*args, **kw)
        _check(context(self._dev), lib().phb_batch_run(context(self._dev), self._h,
                                                       ctypes.byref(io)))

    def capture(self, *args, **kw):
        """Capture one pass over these tensors (pos, lam, offsets, idx, q, rhs,
        dxdt, status, tape=, trans=, rhs_bar=, dxdt_bar=, q_bar=, pos_bar=); the
        batch keeps references so that they stay alive while it may replay."""
        io, tensors = self._io(*args, **kw)
        ctx = context(self._dev)
        _check(ctx, lib().phb_batch_capture(ctx, self._h, ctypes.byref(io)))
        self._bound = tensors

    def launch(self):
        """Replay the captured pass on torch's current stream order."""
        ctx = context(self._dev)
        _check(ctx, lib().phb_batch_launch(ctx, self._h))
