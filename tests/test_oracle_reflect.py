"""Pins of the oracle's reflective sides (specular reflection, the symmetry
planes of Sec. 6) against results that need no reflection:

* infinite medium: a 2D multigroup box with every side reflective and a
  uniform start (material hotter than the radiation) stays uniform and
  follows the spatially uniform backward-Euler recursion of Sec. 2, written
  here per group with the Planck fractions integrated by scipy and the
  temperature found by brentq;
* symmetry plane, 2D: a problem symmetric about y = 1/2 solved on the full
  domain equals, on the lower half, the same problem on the half domain
  with a reflective y+ side;
* symmetry plane, 1D: a slab heated from both ends with mirror-symmetric
  materials equals, on its left half, the half slab with a reflective right
  side.

The reflected inflow is refreshed from the newest intensity after every
sweep, so each step's fixed point is the reflective one; the comparisons are
made at tight outer tolerances.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

from paper_2504_21784_amd import workloads as W

TIGHT = dict(eps_outer=1e-11, eps_inner=1e-12, cg_rtol=1e-13, elim_rtol=1e-15, max_outer=200, max_inner=60,
             max_cg=3000)


def infinite_medium_2d(G_sigma=(0.5, 3.0, 20.0, 100.0)):
    p = W.multigroup_2d(n=6, G=len(G_sigma), sn=4, region=6, seed=1)
    p.model = W.MODEL_CONST
    p.sigma0 = np.array([G_sigma])
    p.cv = np.array([0.7])
    p.region_of_cell = np.zeros(p.n_cells, np.int32)
    p.bc_kind = [W.BC_REFLECT] * 4
    p.T0 = 0.3
    p.dt = 0.05
    return p


def planck_fractions(nu_edges, T):
    """b_g(T): (15/pi^4) int x^3/(e^x - 1) dx over the group, the first group
    from 0 and the last to infinity."""
    f = lambda x: x ** 3 * math.exp(-x) / -math.expm1(-x) if x > 0 else 0.0
    xs = [0.0] + list(np.asarray(nu_edges[1:-1]) / T) + [np.inf]
    return np.array([quad(f, xs[g], xs[g + 1], epsabs=0, epsrel=1e-13, limit=200)[0]
                     for g in range(len(xs) - 1)]) * 15 / math.pi ** 4


def uniform_recursion(p, T_mat0, n_steps):
    """Uniform isotropic intensity I_g and temperature T of backward Euler:
    (sigma_g + 1/(c dt)) I_g = sigma_g a c T^4 b_g(T)/(4 pi) + I_g*/(c dt),
    c_v (T - T*)/dt = sum_g sigma_g (4 pi I_g - a c T^4 b_g(T))."""
    a, c, dt, cv, sg = p.a, p.c, p.dt, p.cv[0], p.sigma0[0]
    I = a * c * p.T0 ** 4 * planck_fractions(p.nu_edges, p.T0) / (4 * math.pi)
    T = T_mat0
    out = []
    for _ in range(n_steps):
        def Ig(Tn, I=I):
            return (sg * a * c * Tn ** 4 * planck_fractions(p.nu_edges, Tn) / (4 * math.pi) + I / (c * dt)) / \
                (sg + 1 / (c * dt))

        f = lambda Tn, T=T: cv * (Tn - T) / dt - np.sum(sg * (4 * math.pi * Ig(Tn) - a * c * Tn ** 4 *
                                                              planck_fractions(p.nu_edges, Tn)))
        T = brentq(f, 1e-6, 10.0, xtol=1e-15, rtol=1e-15)
        I = Ig(T)
        out.append((T, I))
    return out


def test_reflective_infinite_medium_2d(oracle_mod):
    p = infinite_medium_2d()
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    st["T"] = 2.0 * st["T"]
    for k, (T_ref, I_ref) in enumerate(uniform_recursion(p, 2.0 * p.T0, 3)):
        r, st, _ = o.step(st, oracle_mod.default_opts(**TIGHT))
        assert r == 0
        assert np.ptp(st["T"]) <= 1e-10 * T_ref                   # uniform
        assert abs(st["T"].mean() - T_ref) <= 1e-11 * T_ref, k
        assert np.abs(st["psi"] - I_ref[None, :, None]).max() <= 1e-9 * I_ref.max(), k


def symmetric_2d(ny, half):
    """12 x 12 cells on [0,1]^2 (or the lower 12 x 6 half), per-cell gray
    opacities mirror-symmetric about y = 1/2, a Planck source on x-, vacuum
    elsewhere; the half problem has a reflective y+ side instead."""
    p = W.gray_2d(n=12, sn=4, block=2, seed=2)
    p.ny = ny
    p.y_edges = np.linspace(0.0, ny / 12.0, ny + 1)
    rng = np.random.default_rng(5)
    lower = 10.0 ** rng.uniform(-1, 2, (6, 12))
    rows = np.vstack([lower, lower[::-1]])[:ny]
    p.region_of_cell = np.arange(p.nx * ny, dtype=np.int32)
    p.sigma0 = rows.reshape(-1, 1).copy()
    p.cv = np.ones(p.nx * ny)
    p.bc_kind = [W.BC_PLANCK, W.BC_VACUUM, W.BC_VACUUM, W.BC_REFLECT if half else W.BC_VACUUM]
    p.dt = 0.05
    return p


def test_reflective_symmetry_plane_2d(oracle_mod):
    pf, ph = symmetric_2d(12, False), symmetric_2d(6, True)
    of, oh = oracle_mod.Oracle(pf), oracle_mod.Oracle(ph)
    sf, sh = of.initial_state(), oh.initial_state()
    for k in range(2):
        r1, sf, _ = of.step(sf, oracle_mod.default_opts(**TIGHT))
        r2, sh, _ = oh.step(sh, oracle_mod.default_opts(**TIGHT))
        assert r1 == 0 and r2 == 0
        Tf = sf["T"].reshape(12, 12, 4)[:6].reshape(-1)
        assert np.abs(Tf - sh["T"]).max() <= 1e-11 * Tf.max(), k
        psif = sf["psi"].reshape(pf.n_angles, 1, 12, 12, 4)[:, :, :6].reshape(pf.n_angles, 1, -1)
        assert np.abs(psif - sh["psi"]).max() <= 1e-10 * psif.max(), k


def symmetric_1d(n, half):
    p = W.slab_1d(n_cells=n, n_angles=8)
    rng = np.random.default_rng(7)
    m = n if half else n // 2
    left = 10.0 ** rng.uniform(-1, 2, m)
    sig = left if half else np.r_[left, left[::-1]]
    p.x_edges = np.linspace(0.0, 0.5 if half else 1.0, n + 1)
    p.region_of_cell = np.arange(n, dtype=np.int32)
    p.sigma0 = sig.reshape(-1, 1).copy()
    p.cv = np.ones(n)
    p.bc_kind = [W.BC_PLANCK, W.BC_REFLECT if half else W.BC_PLANCK]
    p.T_bdr = [1.0, 0.0 if half else 1.0]
    p.dt = 0.02
    return p


def test_reflective_symmetry_plane_1d(oracle_mod):
    pf, ph = symmetric_1d(40, False), symmetric_1d(20, True)
    of, oh = oracle_mod.Oracle(pf), oracle_mod.Oracle(ph)
    sf, sh = of.initial_state(), oh.initial_state()
    for k in range(4):
        r1, sf, _ = of.step(sf, oracle_mod.default_opts(**TIGHT))
        r2, sh, _ = oh.step(sh, oracle_mod.default_opts(**TIGHT))
        assert r1 == 0 and r2 == 0
        assert np.abs(sf["T"][:40] - sh["T"]).max() <= 1e-11 * sf["T"].max(), k


def test_reflective_inflow_mirrors_the_boundary_intensity(oracle_mod):
    """On a random intensity, every entering direction of a reflective side
    gets the mirrored direction's value at the same boundary node; the other
    sides keep their boundary-description values."""
    p = W.gray_2d(n=5, sn=4, block=5, seed=2)
    p.ny = 3
    p.y_edges = np.linspace(0.0, 0.6, 4)
    p.region_of_cell = np.zeros(15, np.int32)
    p.bc_kind = [W.BC_PLANCK, W.BC_VACUUM, W.BC_VACUUM, W.BC_REFLECT]
    o = oracle_mod.Oracle(p)
    psi = np.random.default_rng(3).uniform(size=(p.n_angles, 1, p.n_nodes))
    inf = o.inflow(psi)
    base = o.inflow()
    nx, ny = p.nx, p.ny
    for d in range(p.n_angles):
        mu, eta = p.omega[d, 0], p.omega[d, 1]
        if eta < 0:        # enters through y+
            e = [k for k in range(p.n_angles) if abs(p.omega[k, 0] - mu) < 1e-14 and abs(p.omega[k, 1] + eta) < 1e-14]
            assert len(e) == 1
            for i in range(nx):
                for lx in range(2):
                    b = 4 * ny + 2 * nx + 2 * i + lx
                    node = 4 * (i + nx * (ny - 1)) + lx + 2
                    assert inf[d, 0, b] == psi[e[0], 0, node]
        mask = np.ones(inf.shape[2], bool)
        mask[4 * ny + 2 * nx:] = eta >= 0
        assert np.array_equal(inf[d, 0, mask], base[d, 0, mask])


def test_reflective_box_conserves_energy(oracle_mod):
    """Every side reflective, blocky random opacities, a hot spot in the
    material: nothing enters or leaves, so the total energy
    sum_n w_n (E_n + c_v T_n) of each step equals that of the step before
    (the time-edge E being the high-order energy density of the previous
    intensity), to the iteration tolerances."""
    p = W.multigroup_2d(n=10, G=3, sn=4, region=5, seed=8)
    p.ny = 8
    p.y_edges = np.linspace(0.0, 0.8, 9)
    p.region_of_cell = p.region_of_cell[:80].copy()
    p.bc_kind = [W.BC_REFLECT] * 4
    p.T0 = 0.1
    p.dt = 0.02
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    hot = (np.arange(p.n_nodes) // 4) % 10 < 3
    st["T"] = np.where(hot, 0.5, st["T"])
    wv = 0.1 * 0.1 / 4
    cvn = p.cv[p.region_of_cell][np.arange(p.n_nodes) // 4]
    for k in range(3):
        Estar = np.einsum("d,dgn->n", p.w, st["psi"]) / p.c
        r, new, _ = o.step(st, oracle_mod.default_opts(**TIGHT))
        assert r == 0
        before = wv * (Estar + cvn * st["T"]).sum()
        after = wv * (new["E"] + cvn * new["T"]).sum()
        assert abs(after - before) <= 1e-10 * before, k
        assert np.ptp(new["T"]) > 1e-3                # not trivially uniform
        st = new
