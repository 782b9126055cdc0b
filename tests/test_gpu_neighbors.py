"""GPU neighbor lists against the oracle's brute-force search: bit-exact CSR
(offsets and ascending rows), at small sizes in full and at the benchmark
sizes on sampled rows; the transpose; the argument and data checks."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1110_0836_amd import synth
from _common import dev, setup_of, csr_rows

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1110_0836_amd")


def gpu_csr(c, **kw):
    off, idx = P.neighbors(dev(c["pos"]), dev(c["lam"]), setup_of(c), **kw)
    return off.cpu().numpy(), idx.cpu().numpy()


def assert_same(c, rows=None):
    goff, gidx = gpu_csr(c)
    ooff, oidx = oracle.neighbors(c["pos"], c["lam"], L=c["L"], periodic=c["periodic"], rows=rows)
    if rows is None:
        assert np.array_equal(goff, ooff)
        assert np.array_equal(gidx, oidx)
    else:
        g = csr_rows(goff, gidx)
        o = csr_rows(ooff, oidx)
        for k, r in enumerate(rows):
            assert np.array_equal(g[r], o[k]), r


def test_golden_tiny():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "neighbors_tiny.json")))
    r0 = 2.3 * 0.5
    sub = {"r0": r0, "r0-": float(np.nextafter(r0, 0.0))}
    x = [sub[v] if isinstance(v, str) else v for v in g["x"]]
    c = dict(pos=np.array([x, g["y"], g["z"]]), lam=np.array(g["lambda"]), L=g["L"],
             periodic=g["periodic"])
    goff, gidx = gpu_csr(c)
    assert [list(r) for r in csr_rows(goff, gidx)] == g["rows"]


def test_cubic_set_lattice():
    assert_same(synth.cubic_set())
    assert_same(synth.cubic_set(pin=True))


@pytest.mark.parametrize("n", [1, 2, 7, 333, 2049, 5003])
@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0), (1, 0, 1)])
def test_ragged_random_sets(n, periodic):
    c = synth.random_cloud(n, seed=100 + n, box=(1.0, 0.7, 1.3), lam_range=(0.03, 0.12),
                           periodic=periodic)
    assert_same(c)


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 1, 0), (1, 0, 1)])
def test_wide_spheres_in_few_cells(periodic):
    """Radii close to half the box: few cells per axis, and periodic ranges that
    wrap past either end or cover a whole axis (where the search visits every
    cell row of that axis, since a row index no longer names one image)."""
    c = synth.random_cloud(900, seed=31, box=(1.0, 0.8, 1.1), lam_range=(0.1, 0.17),
                           periodic=periodic)
    assert_same(c)


def test_long_rows_use_the_fallback_sort():
    # ~1500 neighbors per particle: rows longer than the LDS sort buffer
    c = synth.random_cloud(3000, seed=7, lam_range=(0.2, 0.21))
    goff, _ = gpu_csr(c)
    assert np.diff(goff).max() > 1024
    assert_same(c)


def test_shear_layer_reduced():
    c = synth.shear_layer(n=1 << 15)
    assert_same(c)


def test_fast_wave_full_size_sampled():
    c = synth.fast_wave_set()
    rows = np.random.default_rng(1).choice(c["lam"].shape[0], 1500, replace=False)
    assert_same(c, rows=rows)


def test_shear_layer_full_size_sampled():
    c = synth.shear_layer()
    rows = np.random.default_rng(2).choice(c["lam"].shape[0], 300, replace=False)
    assert_same(c, rows=rows)


def test_transpose():
    c = synth.random_cloud(4000, seed=9, lam_range=(0.04, 0.1))
    off, idx = P.neighbors(dev(c["pos"]), dev(c["lam"]), setup_of(c))
    t_off, t_src, t_pos = P.transpose(off, idx)
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    t_off, t_src, t_pos = t_off.cpu().numpy(), t_src.cpu().numpy(), t_pos.cpu().numpy()
    n = len(off) - 1
    rows_i = np.repeat(np.arange(n), np.diff(off))
    order = np.lexsort((rows_i, idx))  # by j then i
    assert np.array_equal(t_src, rows_i[order].astype(np.int32))
    assert np.array_equal(t_off, np.concatenate([[0], np.cumsum(np.bincount(idx, minlength=n))]))
    # t_pos[s] points at the entry of slot s in the transposed rows
    assert np.array_equal(t_src[t_pos], rows_i)
    j_of_t = np.repeat(np.arange(n), np.diff(t_off))
    assert np.array_equal(j_of_t[t_pos], idx)


def test_capacity_and_input_errors():
    import torch
    c = synth.cubic_set()
    pos, lam = dev(c["pos"]), dev(c["lam"])
    s = setup_of(c)
    off = torch.empty(lam.shape[0] + 1, dtype=torch.int64, device="cuda")
    idx = torch.empty(100, dtype=torch.int32, device="cuda")
    rc, nnz = P.phb_neighbors_build(s, pos, lam, off, idx, 100)
    assert rc == P.PHB_ECAPACITY and nnz == oracle.neighbors(c["pos"], c["lam"])[0][-1]
    bad = c["pos"].copy()
    bad[1, 17] = 1.0  # == L: outside [0, L)
    with pytest.raises(P.PhurbasError) as e:
        P.neighbors(dev(bad), lam, s)
    assert e.value.code == P.PHB_EINVAL
    badl = c["lam"].copy()
    badl[3] = -1.0
    with pytest.raises(P.PhurbasError):
        P.neighbors(pos, dev(badl), s)
    with pytest.raises(P.PhurbasError):  # r_f = 2.3 * 0.25 > L/2 on a periodic axis
        P.neighbors(pos, dev(np.full_like(c["lam"], 0.25)), s)
    nanp = c["pos"].copy()
    nanp[0, 5] = np.nan
    with pytest.raises(P.PhurbasError):
        P.neighbors(dev(nanp), lam, s)


def test_spatial_order_is_a_permutation_and_local():
    c = synth.shear_layer(n=1 << 16)
    perm = P.spatial_order(dev(c["pos"]), dev(c["lam"]), setup_of(c)).cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(len(perm)))
    p = c["pos"][:, perm]
    step = np.abs(np.diff(p, axis=1)).sum(0)
    assert np.median(step) < 0.05  # consecutive particles are close
    # same call, same answer
    perm2 = P.spatial_order(dev(c["pos"]), dev(c["lam"]), setup_of(c)).cpu().numpy()
    assert np.array_equal(perm, perm2)
    src = dev(c["q"])
    got = P.permute(dev(perm.astype(np.int32)), src).cpu().numpy()
    assert np.array_equal(got, c["q"][:, perm])


@pytest.mark.parametrize("L", [(1.0, 1.0, 1.0), (1.0, 0.8, 1.1)])
def test_spatial_order_walks_a_lattice_by_face_steps(L):
    """On a 16^3 lattice of cell centres (shuffled) the order is a Hilbert
    walk: it starts at the corner cell and every step moves to a lattice
    neighbour sharing a face (a Morton order jumps)."""
    side = 16
    g = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij")).reshape(3, -1)
    shuffle = np.random.default_rng(11).permutation(g.shape[1])
    g = g[:, shuffle]
    Ls = np.array(L)[:, None]
    pos = (g + 0.5) / side * Ls
    lam = np.full(g.shape[1], 1.0 / side)
    s = P.Setup(L=L, periodic=(1, 1, 1))
    perm = P.spatial_order(dev(pos), dev(lam), s).cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(g.shape[1]))
    walk = g[:, perm]
    assert np.array_equal(walk[:, 0], [0, 0, 0])
    step = np.abs(np.diff(walk, axis=1))
    assert np.all(step.sum(0) == 1)
