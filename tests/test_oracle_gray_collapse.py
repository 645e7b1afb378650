"""Pins of the oracle's gray first-moment opacity and its Planck boundary inflow.

* sigma_F is the Rosseland-collapsed opacity of Sec. 2 (Eq. sigmaF): the group
  opacities averaged with the normalised Rosseland spectrum r_g(T) at the
  node's temperature; sigma_P averages them with the normalised Planck
  spectrum b_g(T).  Both are checked against r_g and b_g integrated here with
  scipy (not the oracle's Gauss-Kronrod panels), and the group-constant case
  must return that constant.
* A Planck side of temperature T_bdr emits B_g(T_bdr)/(4 pi) = a c T_bdr^4
  b_g(T_bdr)/(4 pi) into every entering direction (Sec. 2, inflow condition
  of the transport equation; Sec. 3, its DG form).  Checked value by value,
  and through an equilibrium: a uniform medium at T_eq whose four sides are
  Planck sides at T_eq stays at equilibrium, step after step.

Each pin is shown to catch a planted mistake: the oracle source is copied,
one line changed (b_g weights in sigma_F, the wrong group's opacity, a
missing 1/(4 pi), the boundary temperature's power), compiled on the CPU and
run through the same check, which must then fail.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2504_21784_amd import workloads as W


def _fractions(nu_edges, T, density):
    """Group integrals of a normalised spectral density at temperature T; the
    first group starts at 0 and the last ends at infinity (the reading that
    makes the fractions sum to one)."""
    xs = [0.0] + list(np.asarray(nu_edges[1:-1]) / T) + [np.inf]
    return np.array([quad(density, xs[g], xs[g + 1], epsabs=0, epsrel=1e-13, limit=400)[0]
                     for g in range(len(xs) - 1)])


def planck_fractions(nu_edges, T):
    f = lambda x: 15 / math.pi ** 4 * x ** 3 * math.exp(-x) / -math.expm1(-x) if 0 < x < 700 else 0.0
    return _fractions(nu_edges, T, f)


def rosseland_fractions(nu_edges, T):
    f = lambda x: (15 / (4 * math.pi ** 4) * x ** 4 * math.exp(-x) / math.expm1(-x) ** 2
                   if 0 < x < 700 else 0.0)
    return _fractions(nu_edges, T, f)


def three_group_box(n=3, sig_g=(0.7, 25.0, 900.0)):
    """n x n cells, 3 groups on bounds (0.05, 0.4, 2.5, 12) (the end bounds
    are extended to 0 and infinity), constant group opacities, S4."""
    p = W.multigroup_2d(n=n, G=3, sn=4, region=n, seed=1)
    p.nu_edges = np.array([0.05, 0.4, 2.5, 12.0])
    p.model = W.MODEL_CONST
    p.sigma0 = np.array([sig_g])
    p.region_of_cell = np.zeros(p.n_cells, np.int32)
    p.cv = np.array([1.0])
    return p


def _closure_opacities(o, p, T_nodes, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    nn = p.n_nodes
    sig = o.opacity(T_nodes)
    psi = rng.uniform(0.5, 1.0, (p.n_angles, p.G, nn))
    cl = o.closures(0, p.dt, sig, T_nodes, np.zeros(nn), np.zeros((nn, p.dim)), psi,
                    np.zeros((p.n_angles, p.G, o.nb)))
    return sig, cl


def _node_temperatures(p, seed=3):
    # spans the group bounds: the hottest nodes put most of the spectrum in
    # the last group, the coldest in the first
    rng = np.random.Generator(np.random.PCG64(seed))
    return 10 ** rng.uniform(math.log10(0.03), math.log10(3.0), p.n_nodes)


def _check_sigma_F(o, p):
    T = _node_temperatures(p)
    sig, cl = _closure_opacities(o, p, T)
    sg = sig[0]                                      # one region: the same in every cell
    for n in range(p.n_nodes):
        r = rosseland_fractions(p.nu_edges, T[n])
        b = planck_fractions(p.nu_edges, T[n])
        assert abs(cl["sigF"][n] - np.dot(r, sg) / r.sum()) <= 1e-12 * np.dot(r, sg) / r.sum(), n
        assert abs(cl["sigP"][n] - np.dot(b, sg) / b.sum()) <= 1e-12 * np.dot(b, sg) / b.sum(), n


def test_sigma_F_group_constant_opacity(oracle_mod):
    p = three_group_box(sig_g=(13.0, 13.0, 13.0))
    o = oracle_mod.Oracle(p)
    _, cl = _closure_opacities(o, p, _node_temperatures(p))
    np.testing.assert_allclose(cl["sigF"], 13.0, rtol=1e-14, atol=0)
    np.testing.assert_allclose(cl["sigP"], 13.0, rtol=1e-14, atol=0)


def test_sigma_F_is_the_rosseland_weighted_mean(oracle_mod):
    p = three_group_box()
    o = oracle_mod.Oracle(p)
    _check_sigma_F(o, p)
    # the two weightings really differ on these nodes (else the pin could not
    # tell them apart)
    T = _node_temperatures(p)
    sg = np.array(p.sigma0[0])
    gaps = [abs(np.dot(rosseland_fractions(p.nu_edges, t), sg) - np.dot(planck_fractions(p.nu_edges, t), sg))
            / np.dot(planck_fractions(p.nu_edges, t), sg) for t in T[:8]]
    assert max(gaps) > 1e-2


def test_rosseland_fractions_sum_and_derivative():
    # r_g is the normalised temperature derivative of the Planck group
    # emission: d(T^4 b_g)/dT = 4 T^3 r_g (Sec. 2), so the independent
    # integrals used above are themselves consistent
    nu = [0.05, 0.4, 2.5, 12.0]
    for T in (0.05, 0.3, 1.7):
        r = rosseland_fractions(nu, T)
        assert abs(r.sum() - 1.0) < 1e-13
        h = 1e-5 * T
        d = ((T + h) ** 4 * planck_fractions(nu, T + h) - (T - h) ** 4 * planck_fractions(nu, T - h)) / (2 * h)
        np.testing.assert_allclose(d, 4 * T ** 3 * r, rtol=1e-7, atol=1e-12)


def planck_side_problem(T_bdr=(0.8, 0.3, 1.4, 0.55)):
    """4 x 3 cells, the 3-group box, every side a Planck side at its own temperature."""
    p = three_group_box(n=4)
    p.ny = 3
    p.y_edges = np.linspace(0.0, 0.75, 4)
    p.region_of_cell = np.zeros(p.n_cells, np.int32)
    p.bc_kind = [W.BC_PLANCK] * 4
    p.T_bdr = list(T_bdr)
    return p


def _check_planck_inflow(o, p):
    inf = o.inflow()
    NB = o.nb
    nx, ny = p.nx, p.ny
    # side ranges of the boundary-node index (x-, x+, y-, y+)
    ranges = [(0, 2 * ny), (2 * ny, 4 * ny), (4 * ny, 4 * ny + 2 * nx), (4 * ny + 2 * nx, NB)]
    for s, (lo, hi) in enumerate(ranges):
        T = p.T_bdr[s]
        want = p.a * p.c * T ** 4 * planck_fractions(p.nu_edges, T) / (4 * math.pi)
        got = inf[:, :, lo:hi]
        np.testing.assert_allclose(got, np.broadcast_to(want[None, :, None], got.shape), rtol=1e-12, atol=0)


def test_planck_side_inflow_value(oracle_mod):
    p = planck_side_problem()
    _check_planck_inflow(oracle_mod.Oracle(p), p)


def _equilibrium_problem():
    p = W.multigroup_2d(n=4, G=3, sn=4, region=2, seed=11)     # power-law opacities, 4 regions
    p.nu_edges = np.array([0.05, 0.4, 2.5, 12.0])
    p.T0 = 0.45
    p.bc_kind = [W.BC_PLANCK] * 4
    p.T_bdr = [0.45] * 4
    p.dt = 0.02
    return p


def _check_equilibrium(o, p, oracle_mod, n_steps=3):
    st = o.initial_state()
    opts = oracle_mod.default_opts(eps_outer=1e-13, eps_inner=1e-14, cg_rtol=1e-14, elim_rtol=1e-15,
                                   max_outer=50, max_inner=50, max_cg=500)
    E_eq = p.a * p.T0 ** 4
    for _ in range(n_steps):
        _, st, _ = o.step(st, opts)
        np.testing.assert_allclose(st["T"], p.T0, rtol=1e-12, atol=0)
        np.testing.assert_allclose(st["E"], E_eq, rtol=1e-11, atol=0)


def test_planck_sides_keep_equilibrium(oracle_mod):
    p = _equilibrium_problem()
    _check_equilibrium(oracle_mod.Oracle(p), p, oracle_mod)


# -- planted mistakes: each must make its pin fail ---------------------------

SIGF_LINE = "sr += rg[k]; srs += rg[k] * s;"
PLANTED = {
    "sigma_F with Planck weights": [(SIGF_LINE, "sr += bg[k]; srs += bg[k] * s;")],
    "sigma_F with the next group's opacity": [
        (SIGF_LINE, "sr += rg[k]; srs += rg[k] * sig[(size_t)cc * G + (k + 1) % G];")],
    "Planck inflow without 1/(4 pi)": [("val[s * G + k] = B * b[k] / (4.0 * M_PI);", "val[s * G + k] = B * b[k];")],
    "Planck inflow with T_bdr^3": [("double B = g->a * g->c * pow(bc->T_bdr[s], 4);",
                                    "double B = g->a * g->c * pow(bc->T_bdr[s], 3);")],
}


@pytest.mark.parametrize("name", list(PLANTED))
def test_planted_mistakes_fail_the_pins(oracle_mod, tmp_path, name):
    L = oracle_mod.build_variant(os.path.join(str(tmp_path), "liboracle_planted.so"), PLANTED[name])
    if name.startswith("sigma_F"):
        p = three_group_box()
        with pytest.raises(AssertionError):
            _check_sigma_F(oracle_mod.Oracle(p, L=L), p)
    else:
        p = planck_side_problem()
        with pytest.raises(AssertionError):
            _check_planck_inflow(oracle_mod.Oracle(p, L=L), p)
        p = _equilibrium_problem()
        with pytest.raises(AssertionError):
            _check_equilibrium(oracle_mod.Oracle(p, L=L), p, oracle_mod, n_steps=1)
