"""Seeded input generators: quadrature sets against the published LQ_n table
and their moment invariants; workload shapes."""
import math
import os

import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "level_symmetric_lq.txt")


def _table():
    rows = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        left, right = line.split("|")
        toks = left.split()
        N = int(toks[0])
        levels = [float(t) for t in toks[1:]]
        cls = {}
        for item in right.split():
            k, v = item.split(":")
            cls[tuple(int(x) for x in k.split(","))] = float(v)
        rows[N] = (levels, cls)
    return rows


@pytest.mark.parametrize("N", [4, 8, 12])
def test_level_symmetric_matches_table(N):
    levels, cls = _table()[N]
    om, w = W.level_symmetric_2d(N)
    got = sorted(set(np.round(np.abs(om[:, 0]), 7)))
    assert np.allclose(got, levels, atol=1.5e-7)
    wo = w[:len(w) // 4] / math.pi
    lev = np.array(levels)
    for k in range(len(wo)):
        idx = tuple(sorted(int(np.argmin(np.abs(lev - abs(om[k, a])))) + 1 for a in range(3)))
        assert abs(wo[k] - cls[idx]) < 1.5e-7


@pytest.mark.parametrize("N", [4, 8, 12])
def test_quadrature_invariants(N):
    om, w = W.level_symmetric_2d(N)
    assert len(w) == N * (N + 2) // 2
    assert abs(w.sum() - 4 * math.pi) < 1e-12 * 4 * math.pi
    assert np.abs((w[:, None] * om).sum(0)[:2]).max() < 1e-14
    assert abs((w * om[:, 0] ** 2).sum() - 4 * math.pi / 3) < 1e-13
    assert abs((w * om[:, 1] ** 2).sum() - 4 * math.pi / 3) < 1e-13
    assert abs((w * om[:, 0] * om[:, 1]).sum()) < 1e-14
    assert np.abs(np.linalg.norm(om, axis=1) - 1).max() < 1e-12
    assert (np.abs(om[:, :2]) > 0).all()


def test_gauss_legendre_slab():
    om, w = W.gauss_legendre_slab(8)
    assert abs(w.sum() - 4 * math.pi) < 1e-12
    assert abs((w * om[:, 0]).sum()) < 1e-14
    assert abs((w * om[:, 0] ** 2).sum() - 4 * math.pi / 3) < 1e-13


def test_workload_shapes():
    p = W.multigroup_2d()
    assert p.units_per_sweep == 256 * 256 * 40 * 16
    assert p.n_regions == 256 and p.sigma0.min() >= 1 and p.sigma0.max() <= 100
    q = W.gray_2d()
    assert q.units_per_sweep == 128 * 128 * 40
    assert q.sigma0.min() >= 0.1 and q.sigma0.max() <= 1000
    b = W.batch_2d()
    assert len(b) == 32
    assert all(64 <= x.nx <= 384 and x.G in (4, 8, 16, 32) and x.n_angles in (12, 40, 84) for x in b)
    a = W.adjoint_2d()
    assert a.n_regions == 64 and 0.5 <= a.cv.min() and a.cv.max() <= 2.0


def test_marshak_units_and_first_steps(oracle_mod):
    """The Marshak wave's constants (a from 7.5657e-15 erg cm^-3 K^-4 and
    11604.518 K/eV), its opacity at 1 eV and 1 keV through the library's
    power-law model, and 40 oracle steps with the fixup and the floor: the
    temperature stays below 1 keV and near or above 1 eV, and the 500 eV
    front only moves right."""
    p = W.marshak_1d(32, 8e-3)
    assert abs(p.a - 137.2) < 0.01 and p.n_steps == 312
    o = oracle_mod.Oracle(p)
    assert abs(o.opacity(np.full(p.n_nodes, 1.0))[0, 0] - 1e12) < 1e-3
    assert abs(o.opacity(np.full(p.n_nodes, 1000.0))[0, 0] - 1e3) < 1e-12
    st = o.initial_state()
    opts = oracle_mod.default_opts(eps_outer=1e-8, eps_inner=1e-10, cg_rtol=1e-12, elim_rtol=1e-12, max_outer=200,
                                   max_inner=60, max_cg=2000, fixup=1, T_floor=1e-8)
    last = 0
    for k in range(40):
        r, st, _ = o.step(st, opts)
        assert r == 0
        T = st["T"]
        assert T.max() <= 1000.0 and T.min() >= 0.999      # the cold end radiates through the vacuum face
        front = int(np.argmax(T < 500.0))
        assert front >= last
        last = front
    assert last > 4


def _refined_gold():
    vals = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "refined_block_mesh.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals


def test_chebyshev_block_mesh_matches_printed_lengths():
    """The refined mesh of the multigroup test (30 cells per 1 cm block at the
    Chebyshev points of the second kind) has the smallest and largest mesh
    lengths the paper prints, to their 4 digits, and 9x the elements of the
    10-per-block uniform mesh; cells are mirror-symmetric inside a block and
    block boundaries are mesh lines."""
    g = _refined_gold()
    n = int(g["per_block"])
    e = W.chebyshev_block_edges(3, n)
    h = np.diff(e)
    assert len(h) == 3 * n and np.all(h > 0)
    assert abs(h.min() - g["h_min_cm"]) < 0.5e-6
    assert abs(h.max() - g["h_max_cm"]) < 0.5e-5
    assert (n / g["coarse_per_block"]) ** 2 * g["coarse_elements"] == g["fine_elements"]
    for b in range(3):
        hb = h[b * n:(b + 1) * n]
        assert np.allclose(hb, hb[::-1], rtol=0, atol=1e-15)
        assert e[b * n] == b and abs(hb.sum() - 1.0) < 1e-14
    p = W.multigroup_2d_clustered(blocks=2, per_block=6, G=3, sn=4)
    assert p.nx == p.ny == 12 and p.x_edges[-1] == 2.0 and len(np.unique(p.region_of_cell)) == 4
    assert np.array_equal(p.region_of_cell.reshape(12, 12)[:6, :6], np.zeros((6, 6), p.region_of_cell.dtype))
