"""Seeded synthetic particle sets for the Phurbas hot path.

This module only draws inputs: positions, resolution lengths and field
values.  It holds none of the method's arithmetic (no neighbor search, fit,
or time derivative) and imports neither the GPU binding nor the oracle, so
both sides can be fed the very same arrays.

Layouts: ``pos`` (3, n) float64 in [0, L), ``lam`` (n,), ``q`` (8, n) with
fields (rho, Vx, Vy, Vz, Bx, By, Bz, sigma).  Every draw uses
``numpy.random.default_rng(seed)`` in the order written below.

The sets stand in for the paper's test problems (Sec. 3): relaxed glassy
particle distributions are replaced by jittered lattices, the linear-wave
tests by an exact fast-magnetosonic eigenmode (App. A), and the
Kelvin-Helmholtz shear layer by a tanh profile sampled at a density that
follows the local resolution length.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 5.0 / 3.0
B0_WAVE = (1.0, math.sqrt(2.0), 0.5)


def jittered_lattice(side: int, jitter: float = 0.3, rng=None, box: float = 1.0):
    """side^3 points at cell centres ((i + 1/2) h), each moved by U(-jitter h, jitter h)
    per axis and wrapped into [0, box).  Index order: x fastest, then y, then z."""
    h = box / side
    g = (np.arange(side) + 0.5) * h
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    if jitter > 0:
        pos = pos + rng.uniform(-jitter * h, jitter * h, size=pos.shape)
    pos = np.mod(pos, box)
    pos[pos >= box] -= box  # np.mod can return box for tiny negatives
    return pos


def tiled_lattice(base: int, tiles: int, jitter: float = 0.3, seed: int = 11,
                  box: float = 1.0):
    """A jittered base^3 lattice of the unit cube, scaled by 1/tiles and tiled
    tiles^3 times to fill the box: (base tiles)^3 points whose neighborhoods
    repeat the base set's at every resolution (Sec. 3.1 refines its relaxed
    set this way, so that convergence studies see the same local particle
    arrangements).  Index order: tiles in x fastest, then y, then z."""
    rng = np.random.default_rng(seed)
    b = jittered_lattice(base, jitter, rng)
    parts = []
    for tz in range(tiles):
        for ty in range(tiles):
            for tx in range(tiles):
                parts.append((b + np.array([[tx], [ty], [tz]], dtype=np.float64)) / tiles)
    pos = np.concatenate(parts, axis=1) * box
    pos[pos >= box] -= box
    return pos


# Exponent table of the cubic polynomial fields (all |alpha| <= 3), used only
# to draw test inputs with a known polynomial form.
CUBIC_EXPONENTS = [(a, b, c) for a in range(4) for b in range(4) for c in range(4)
                   if a + b + c <= 3]


def cubic_poly_fields(pos, nf, rng, center=(0.5, 0.5, 0.5)):
    """nf fields, each sum_alpha a_alpha (x - c)^alpha with a_alpha ~ U(-1, 1).
    Returns (fields (nf, n), coefficient array (nf, 20), exponent list)."""
    coef = rng.uniform(-1.0, 1.0, size=(nf, len(CUBIC_EXPONENTS)))
    d = pos - np.asarray(center, dtype=np.float64)[:, None]
    out = np.zeros((nf, pos.shape[1]))
    for k, (a, b, c) in enumerate(CUBIC_EXPONENTS):
        mono = d[0] ** a * d[1] ** b * d[2] ** c
        out += coef[:, k:k + 1] * mono[None, :]
    return out, coef, CUBIC_EXPONENTS


def nonzero_mode(rng):
    """A wave vector m in {-2..2}^3 without the zero vector."""
    while True:
        m = rng.integers(-2, 3, size=3)
        if np.any(m != 0):
            return m


def cubic_set(seed: int = 1, pin: bool = False):
    """4,096 particles on a jittered 16^3 lattice, lambda = 1/16, periodic unit cube.
    Fields: random cubic polynomials in (x - 1/2) plus 1e-3 sin(2 pi m.x + phi).
    ``pin=True``: no sine and an open (non-periodic) box, so that the fields are
    exact cubics."""
    rng = np.random.default_rng(seed)
    side = 16
    pos = jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side)
    fields, coef, expo = cubic_poly_fields(pos, 8, rng)
    amp = 0.0 if pin else 1e-3
    for f in range(8):
        m = nonzero_mode(rng)
        phi = rng.uniform(0.0, 2 * np.pi)
        fields[f] += amp * np.sin(2 * np.pi * (m @ pos) + phi)
    periodic = (0, 0, 0) if pin else (1, 1, 1)
    return dict(pos=pos, lam=lam, q=fields, L=(1.0, 1.0, 1.0), periodic=periodic,
                gamma=GAMMA, coef=coef, exponents=expo, name="lattice16_cubic")


def fast_mode(B0=B0_WAVE, rho0=1.0, P0=1.0, gamma=GAMMA, k=(2 * np.pi, 0.0, 0.0)):
    """Fast magnetosonic eigenmode of the linearized ideal-MHD system with zero
    bulk viscosity (App. A).  Velocity eigenvector from
        omega^2 V = [(k.VA)^2 I + (Vs^2 + VA^2) k k^T - (k.VA)(VA k^T + k VA^T)] V,
    largest eigenvalue; density, pressure and field from the linearized mass,
    energy and induction relations.  Returns (omega, R) with R the 8-vector
    (rho, V, B, sigma) of unit 2-norm, sigma = P / (gamma - 1)."""
    k = np.asarray(k, dtype=np.float64)
    B0 = np.asarray(B0, dtype=np.float64)
    VA = B0 / math.sqrt(rho0)
    Vs2 = gamma * P0 / rho0
    kVA = k @ VA
    M = (kVA ** 2) * np.eye(3) + (Vs2 + VA @ VA) * np.outer(k, k) \
        - kVA * (np.outer(VA, k) + np.outer(k, VA))
    evals, evecs = np.linalg.eigh(M)
    omega = math.sqrt(evals[-1])
    V = evecs[:, -1]
    if V @ k < 0:
        V = -V
    kV = k @ V
    rho = rho0 * kV / omega
    P = gamma * P0 * kV / omega
    B = (kV * B0 - (k @ B0) * V) / omega
    sigma = P / (gamma - 1.0)
    R = np.concatenate([[rho], V, B, [sigma]])
    nrm = np.linalg.norm(R)
    return omega, R / nrm


def wave_background(n, rho0=1.0, sigma0=1.5, B0=B0_WAVE):
    q = np.zeros((8, n))
    q[0] = rho0
    q[4:7] = np.asarray(B0)[:, None]
    q[7] = sigma0
    return q


def fast_wave_set(seed: int = 2, side: int = 64, eps: float = 1e-6):
    """side^3 jittered lattice (lambda = 1/side) in a periodic unit cube carrying a
    fast-magnetosonic plane wave of amplitude eps along x on the background
    rho = 1, sigma = 1/(gamma - 1), V = 0, B = (1, sqrt 2, 0.5)."""
    rng = np.random.default_rng(seed)
    pos = jittered_lattice(side, 0.3, rng)
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side)
    sigma0 = 1.0 / (GAMMA - 1.0)
    P0 = (GAMMA - 1.0) * sigma0
    omega, R = fast_mode(P0=P0)
    q = wave_background(n, 1.0, sigma0)
    q += eps * R[:, None] * np.cos(2 * np.pi * pos[0])[None, :]
    return dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=GAMMA,
                omega=omega, R=R, eps=eps, k=(2 * np.pi, 0.0, 0.0),
                name=f"fastwave_lattice{side}")


def weighted_wave_set(seed: int = 4, side: int = 64):
    """The wave set of fast_wave_set plus loss weights w_i ~ U(0, 1)."""
    c = fast_wave_set(seed=2, side=side)
    rng = np.random.default_rng(seed)
    c["w"] = rng.uniform(0.0, 1.0, size=c["lam"].shape[0])
    c["name"] = f"fastwave_adjoint_lattice{side}"
    return c


def _shear_profile(y):
    """+-1 tanh profile of two layers at y = 1/4 and 3/4 (width 0.05)."""
    return np.where(y < 0.5, np.tanh((y - 0.25) / 0.05), -np.tanh((y - 0.75) / 0.05))


def shear_g(y):
    """Resolution shape g(y) = 1 - 0.75 max(sech^2((y - 1/4)/0.02), sech^2((y - 3/4)/0.02))."""
    s1 = 1.0 / np.cosh((y - 0.25) / 0.02) ** 2
    s2 = 1.0 / np.cosh((y - 0.75) / 0.02) ** 2
    return 1.0 - 0.75 * np.maximum(s1, s2)


def shear_layer(seed: int = 3, n: int = 1 << 20):
    """Adaptive shear-layer set: x, z ~ U(0,1); y drawn from the density
    proportional to g(y)^-3 (exactly n draws); lambda = s g(y) with s fixed by
    one particle per lambda^3 on average.  Fields: tanh shear V_x = 0.5 T(y),
    small V_y = 0.01 sin(4 pi x) exp(-4 pi |y - y_layer|), rho = 1.05 + 0.05 T(y),
    sigma = 2.5/(gamma - 1), B = (0.1, 0, 0).  Periodic unit cube."""
    rng = np.random.default_rng(seed)
    grid = np.linspace(0.0, 1.0, 200001)
    dens = shear_g(grid) ** -3
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    integral = cdf[-1]
    cdf /= integral
    x = rng.uniform(0.0, 1.0, size=n)
    u = rng.uniform(0.0, 1.0, size=n)
    z = rng.uniform(0.0, 1.0, size=n)
    y = np.interp(u, cdf, grid)
    y = np.clip(y, 0.0, np.nextafter(1.0, 0.0))
    pos = np.stack([x, y, z])
    s = (integral / n) ** (1.0 / 3.0)
    lam = s * shear_g(y)
    T = _shear_profile(y)
    ylayer = np.where(y < 0.5, 0.25, 0.75)
    q = np.zeros((8, n))
    q[0] = 1.05 + 0.05 * T
    q[1] = 0.5 * T
    q[2] = 0.01 * np.sin(4 * np.pi * x) * np.exp(-4 * np.pi * np.abs(y - ylayer))
    q[4] = 0.1
    q[7] = 2.5 / (GAMMA - 1.0)
    return dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=GAMMA,
                name=f"shear_layer_adaptive_{n}")


def linear_wave(kind: str, side: int, eps: float = 1e-6, seed: int = 6, jitter: float = 0.3,
                base: int = 0):
    """Linear-wave set of Sec. 3.1: a jittered side^3 lattice in the periodic unit
    cube, rho = 1, P = 1/gamma (sound speed 1), gamma = 5/3, carrying
    eps R cos(2 pi x - omega t) at t = 0 with R of unit 2-norm:
      "sound":  B = 0,             V along x, omega = 2 pi;
      "alfven": B = (1, 0, 0),     V along y, omega = 2 pi (shear Alfven wave);
      "fast":   B = (0, 0, sqrt 3), V along x, omega = 4 pi (magnetoacoustic, k
                perpendicular to B).
    The other components follow from the linearized equations (App. A with no
    viscosity): rho = rho0 k.V/omega, P = gamma P0 k.V/omega,
    B = (B0 k.V - (k.B0) V)/omega, sigma = P/(gamma - 1).  Returns the set with
    omega, R, eps and the background q0.  base > 0: the particles are a jittered
    base^3 cube tiled side / base times per axis (tiled_lattice)."""
    rng = np.random.default_rng(seed)
    pos = (tiled_lattice(base, side // base, jitter, seed) if base else
           jittered_lattice(side, jitter, rng))
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side)
    rho0, P0 = 1.0, 1.0 / GAMMA
    k = np.array([2 * np.pi, 0.0, 0.0])
    if kind == "sound":
        B0, V, speed = np.zeros(3), np.array([1.0, 0.0, 0.0]), 1.0
    elif kind == "alfven":
        B0, V, speed = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), 1.0
    elif kind == "fast":
        B0, V, speed = np.array([0.0, 0.0, math.sqrt(3.0)]), np.array([1.0, 0.0, 0.0]), 2.0
    else:
        raise ValueError(kind)
    omega = speed * 2 * np.pi
    kv = k @ V
    R = np.concatenate([[rho0 * kv / omega], V, (B0 * kv - (k @ B0) * V) / omega,
                        [GAMMA * P0 * kv / omega / (GAMMA - 1.0)]])
    R /= np.linalg.norm(R)
    q0 = np.zeros(8)
    q0[0] = rho0
    q0[4:7] = B0
    q0[7] = P0 / (GAMMA - 1.0)
    q = q0[:, None] + eps * R[:, None] * np.cos(2 * np.pi * pos[0])[None, :]
    return dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=GAMMA,
                omega=omega, R=R, eps=eps, q0=q0, name=f"{kind}_wave_lattice{side}")


def batched_cubes(seed: int = 5, n_sets: int = 32, smin: int = 16, smax: int = 64):
    """n_sets independent periodic unit cubes, side n_s ~ U{smin..smax}, jittered
    lattice with lambda = 1/n_s.  Each field a0 + sum_{m=1..3} a_m sin(2 pi k_m.x + phi_m)
    with k_m in {-2..2}^3 \\ 0, a_m ~ U(-0.05, 0.05); a0 = 1 (rho), 1.5 (sigma), else 0."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(smin, smax + 1, size=n_sets)
    sets = []
    for s in sides:
        pos = jittered_lattice(int(s), 0.3, rng)
        n = pos.shape[1]
        lam = np.full(n, 1.0 / s)
        q = np.zeros((8, n))
        for f in range(8):
            a0 = 1.0 if f == 0 else (1.5 if f == 7 else 0.0)
            q[f] = a0
            for _ in range(3):
                km = nonzero_mode(rng)
                am = rng.uniform(-0.05, 0.05)
                ph = rng.uniform(0.0, 2 * np.pi)
                q[f] += am * np.sin(2 * np.pi * (km @ pos) + ph)
        sets.append(dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
                         gamma=GAMMA))
    return dict(sets=sets, sides=sides, name=f"batched_{n_sets}_sets")


def cp_alfven(side: int = 16, seed: int = 7, jitter: float = 0.3, gamma: float = GAMMA,
              base: int = 0):
    """Circularly polarized Alfven wave initial state (Sec. 3.2): rho = 1, Vx = 0,
    Bx = 1, Vy = By = 0.1 sin 2 pi x, Vz = Bz = 0.1 cos 2 pi x, P = 0.1.  base > 0:
    particles tiled from a base^3 cube (tiled_lattice)."""
    rng = np.random.default_rng(seed)
    pos = (tiled_lattice(base, side // base, jitter, seed) if base else
           jittered_lattice(side, jitter, rng))
    n = pos.shape[1]
    lam = np.full(n, 1.0 / side)
    x = pos[0]
    q = np.zeros((8, n))
    q[0] = 1.0
    q[2] = 0.1 * np.sin(2 * np.pi * x)
    q[3] = 0.1 * np.cos(2 * np.pi * x)
    q[4] = 1.0
    q[5] = 0.1 * np.sin(2 * np.pi * x)
    q[6] = 0.1 * np.cos(2 * np.pi * x)
    q[7] = 0.1 / (gamma - 1.0)
    return dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=gamma,
                name=f"cp_alfven_lattice{side}")


def random_cloud(n: int, seed: int, box=(1.0, 1.0, 1.0), lam_range=(0.08, 0.12),
                 periodic=(1, 1, 1)):
    """n uniform random points in the box with per-particle lambda ~ U(lam_range)
    and smooth random fields; a generic irregular set for ragged-size tests."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pos = rng.uniform(0.0, 1.0, size=(3, n)) * box[:, None]
    pos = np.minimum(pos, np.nextafter(box, 0.0)[:, None])
    lam = rng.uniform(lam_range[0], lam_range[1], size=n)
    q = np.zeros((8, n))
    for f in range(8):
        a0 = 1.0 if f == 0 else (1.5 if f == 7 else 0.0)
        q[f] = a0
        for _ in range(3):
            km = nonzero_mode(rng)
            am = rng.uniform(-0.05, 0.05)
            ph = rng.uniform(0.0, 2 * np.pi)
            q[f] += am * np.sin(2 * np.pi * ((km / box) @ pos) + ph)
    return dict(pos=pos, lam=lam, q=q, L=tuple(box), periodic=tuple(periodic), gamma=GAMMA,
                name=f"cloud_{n}")


def graded_lattice(side: int = 10, seed: int = 101, wave: bool = True):
    """A jittered side^3 lattice in the periodic unit cube whose resolution
    varies smoothly, lambda = h (1.25 + 0.35 sin 2 pi x) with h = 1/side (0.9 to
    1.6 spacings), so that individual time steps spread over levels.  It
    carries a small sound wave (the set of linear_wave("sound"), eps = 1e-3)
    or smooth random-phase fields."""
    h = 1.0 / side
    if wave:
        c = linear_wave("sound", side, eps=1e-3, seed=seed)
        pos, q = c["pos"], c["q"]
    else:
        rng = np.random.default_rng(seed)
        pos = jittered_lattice(side, 0.3, rng)
        n = pos.shape[1]
        q = np.zeros((8, n))
        q[0] = 1.0 + 0.1 * np.sin(2 * np.pi * (pos[1] + 0.2))
        q[1:4] = 0.05 * np.cos(2 * np.pi * pos[[2, 0, 1]])
        q[4:7] = np.array([0.5, -0.2, 0.3])[:, None] + 0.05 * np.sin(2 * np.pi * pos)
        q[7] = 1.5 + 0.1 * np.cos(2 * np.pi * pos[2])
    lam = h * (1.25 + 0.35 * np.sin(2 * np.pi * pos[0]))
    return dict(pos=pos, lam=lam, q=q, L=(1.0, 1.0, 1.0), periodic=(1, 1, 1), gamma=GAMMA,
                name=f"graded_lattice{side}")
