"""GPU parity of the transport sweep and its fused moments against the FP64
oracle on identical seeded inputs (element by element), through the C ABI.

FP64: <= 1e-10 relative (to the field's max); FP32: <= 1e-5 relative.  The
pointwise relative error (relative to each value, floored at 1e-12 of the
field's max) is asserted too: for the scalar flux (positive) 1e-13 in FP64
and 1e-6 in FP32; for the angular flux, which these random inputs drive
through sign changes (values near a sign change keep only absolute accuracy,
about the rounding of the terms that cancel), 1e-9 in FP64 and 5e-2 in FP32.
Shapes span several 16-row bands with ragged tails, several (angle, group)
chunks, and the degenerate cases (one cell, one row, one band exactly).
"""
import math

import numpy as np
import pytest
from parity import rel_pointwise

from paper_2504_21784_amd import workloads as W

pytestmark = pytest.mark.gpu


def _prob2d(nx, ny, sn=4, G=2, seed=0, nonuniform=False):
    p = W.gray_2d(n=4, sn=sn)
    p.nx, p.ny = nx, ny
    rng = np.random.default_rng(seed)
    if nonuniform:
        xe = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, nx)])
        ye = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, ny)])
        p.x_edges, p.y_edges = xe / xe[-1], ye / ye[-1]
    else:
        p.x_edges, p.y_edges = np.linspace(0, 1, nx + 1), np.linspace(0, 1, ny + 1)
    p.region_of_cell = np.zeros(nx * ny, np.int32)
    p.G = G
    p.nu_edges = np.logspace(-2, 1, G + 1)
    p.sigma0 = np.ones((1, G))
    p.cv = np.ones(1)
    return p


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SHAPES = [(37, 35, 4, 3), (16, 16, 8, 1), (20, 33, 4, 5), (1, 1, 4, 2), (9, 1, 8, 2), (1, 20, 4, 1), (64, 48, 8, 2)]


@pytest.mark.parametrize("nx,ny,sn,G", SHAPES)
def test_sweep2d_fp64_matches_oracle(smrt_mod, oracle_mod, nx, ny, sn, G):
    p = _prob2d(nx, ny, sn, G, seed=nx * 131 + ny, nonuniform=True)
    print(f"shape nx={nx} ny={ny} S{sn} G={G}", flush=True)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=nx + 7 * ny)
    sig = sigt * 0.6
    o = oracle_mod.Oracle(p)
    ref = o.sweep(sigt, q, pp, 0.8, inf)
    ref_mom = o.moments(sig, ref)
    ctx = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP64)
    psi, mom = ctx.sweep(sigt, sig, q, pp, 0.8, inf)
    pw = rel_pointwise(psi, ref)
    print(f"  psi: max-normalised {_rel(psi, ref):.3e}, pointwise {pw:.3e}", flush=True)
    assert _rel(psi, ref) < 1e-10
    assert pw < PW64
    phi = sum(mom[6 * k] for k in range(4))
    phi_ref = sum(ref_mom[6 * k] for k in range(4))
    assert rel_pointwise(phi, phi_ref) < PW64_PHI
    for m in range(27):
        assert _rel(mom[m], ref_mom[m]) < 1e-10, m
    ctx.close()


# pointwise relative error bounds (floor 1e-12 of the max): angular flux, scalar flux
PW64, PW32 = 1e-9, 5e-2
PW64_PHI, PW32_PHI = 1e-13, 1e-6

# (waves per band, bands per workgroup, groups per lane); (0, 0, 0) = automatic
FP32_LAUNCHES = [(0, 0, 0), (1, 1, 1), (1, 2, 1), (1, 4, 1), (2, 2, 1), (4, 4, 1), (1, 16, 1), (2, 8, 1), (1, 4, 2),
                 (2, 1, 2), (1, 8, 4), (4, 2, 4)]


@pytest.mark.parametrize("nx,ny,sn,G", [(37, 35, 4, 3), (20, 33, 8, 4), (64, 48, 8, 2)])
@pytest.mark.parametrize("launch", FP32_LAUNCHES)
def test_sweep2d_fp32_matches_oracle(smrt_mod, oracle_mod, nx, ny, sn, G, launch):
    p = _prob2d(nx, ny, sn, G, seed=3)
    print(f"shape nx={nx} ny={ny} S{sn} G={G} launch={launch}", flush=True)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=5)
    sig = sigt * 0.5
    o = oracle_mod.Oracle(p)
    ref = o.sweep(sigt, q, pp, 1.0, inf)
    ref_mom = o.moments(sig, ref)
    ctx = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP32)
    ctx.set_launch(*launch)
    psi, mom = ctx.sweep(sigt, sig, q, pp, 1.0, inf)
    pw = rel_pointwise(psi, ref)
    print(f"  psi: max-normalised {_rel(psi, ref):.3e}, pointwise {pw:.3e}", flush=True)
    assert _rel(psi, ref) < 1e-5
    assert pw < PW32
    phi = sum(mom[6 * k] for k in range(4))
    phi_ref = sum(ref_mom[6 * k] for k in range(4))
    assert np.linalg.norm(phi - phi_ref) / np.linalg.norm(phi_ref) < 1e-5
    assert rel_pointwise(phi, phi_ref) < PW32_PHI
    for m in range(27):
        assert _rel(mom[m], ref_mom[m]) < 1e-5, m
    ctx.close()


def test_sweep2d_inactive_slots_large(smrt_mod, oracle_mod):
    """Regression: chunks with inactive (angle, group) slots (4 waves x 2 pairs
    = 32 group slots for 4 groups) at a size where a negative slot index would
    leave the inflow buffer, on band groups of 2 (the last one partial)."""
    p = _prob2d(96, 80, 8, 4, seed=8)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=21)
    ref = oracle_mod.Oracle(p).sweep(sigt, q, pp, 0.5, inf)
    ctx = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP32)
    ctx.set_launch(4, 2, 2)
    psi, _ = ctx.sweep(sigt, 0.5 * sigt, q, pp, 0.5, inf)
    assert _rel(psi, ref) < 1e-5
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_sweep2d_without_time_edge_source(smrt_mod, oracle_mod, prec, tol):
    """No psi_prev (the raw-sweep form the adjoint uses): the time-edge term
    drops out, including on lanes with no (angle, group) pair (G = 3)."""
    p = _prob2d(27, 21, 4, 3, seed=12)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=13)
    sig = 0.7 * sigt
    o = oracle_mod.Oracle(p)
    ref = o.sweep(sigt, q, np.zeros_like(pp), 0.9, inf)
    ref_mom = o.moments(sig, ref)
    ctx = smrt_mod.Context(p, precision=prec)
    psi, mom = ctx.sweep(sigt, sig, q, None, 0.9, inf)
    assert _rel(psi, ref) < tol
    for m in range(27):
        assert _rel(mom[m], ref_mom[m]) < tol, m
    ctx.close()


def test_sweep2d_launch_shapes_agree_fp64(smrt_mod, oracle_mod):
    p = _prob2d(45, 40, 8, 3, seed=1)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=9)
    ref = oracle_mod.Oracle(p).sweep(sigt, q, pp, 0.3, inf)
    ctx = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP64)
    for nw, nb, k in ((1, 1, 1), (2, 1, 1), (4, 1, 1), (1, 2, 1), (1, 4, 1), (1, 8, 1), (1, 16, 1), (2, 8, 1),
                      (4, 4, 1), (1, 2, 2), (2, 4, 2), (1, 8, 2)):
        print(f"waves per band {nw}, bands per workgroup {nb}, groups per lane {k}", flush=True)
        ctx.set_launch(nw, nb, k)
        psi, _ = ctx.sweep(sigt, sigt * 0.5, q, pp, 0.3, inf)
        assert _rel(psi, ref) < 1e-10
    ctx.close()


def test_sweep2d_manufactured_bilinear_exact(smrt_mod):
    """Lumped bilinear DG reproduces a bilinear intensity exactly (no oracle)."""
    p = _prob2d(23, 19, 8, 1, seed=4, nonuniform=True)
    a, b, c, d = 1.0, 0.3, -0.2, 0.5
    X = np.zeros(p.n_nodes)
    Y = np.zeros(p.n_nodes)
    for j in range(p.ny):
        for i in range(p.nx):
            for l in range(4):
                X[4 * (i + p.nx * j) + l] = p.x_edges[i + (l & 1)]
                Y[4 * (i + p.nx * j) + l] = p.y_edges[j + (l >> 1)]
    I = a + b * X + c * Y + d * X * Y
    sigt = np.full((p.n_cells, 1), 2.5)
    q = (2.5 * I)[:, None]
    ang = np.array([[p.omega[k, 0] * (b + d * Y) + p.omega[k, 1] * (c + d * X)] for k in range(p.n_angles)])
    nb = W.boundary_node_count(p)
    bx, by = np.zeros(nb), np.zeros(nb)
    for j in range(p.ny):
        for ly in range(2):
            bx[2 * j + ly], by[2 * j + ly] = 0.0, p.y_edges[j + ly]
            bx[2 * p.ny + 2 * j + ly], by[2 * p.ny + 2 * j + ly] = 1.0, p.y_edges[j + ly]
    for i in range(p.nx):
        for lx in range(2):
            bx[4 * p.ny + 2 * i + lx], by[4 * p.ny + 2 * i + lx] = p.x_edges[i + lx], 0.0
            bx[4 * p.ny + 2 * p.nx + 2 * i + lx], by[4 * p.ny + 2 * p.nx + 2 * i + lx] = p.x_edges[i + lx], 1.0
    inflow = np.broadcast_to(a + b * bx + c * by + d * bx * by, (p.n_angles, 1, nb)).copy()
    ctx = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP64)
    psi, _ = ctx.sweep(sigt, sigt, q, ang, 1.0, inflow)
    assert _rel(psi[:, 0, :], np.broadcast_to(I, psi[:, 0, :].shape)) < 1e-13
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6)])
def test_sweep1d_matches_oracle(smrt_mod, oracle_mod, prec, tol):
    p = W.slab_1d(n_cells=53, n_angles=8)
    p.G = 3
    p.nu_edges = np.array([0.01, 0.1, 1.0, 10.0])
    p.sigma0 = np.ones((1, 3))
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=17)
    o = oracle_mod.Oracle(p)
    ref = o.sweep(sigt, q, pp, 0.4, inf)
    ref_mom = o.moments(sigt * 0.3, ref)
    ctx = smrt_mod.Context(p, precision=prec)
    psi, mom = ctx.sweep(sigt, sigt * 0.3, q, pp, 0.4, inf)
    assert _rel(psi, ref) < tol
    for m in range(8):
        assert _rel(mom[m], ref_mom[m]) < tol
    ctx.close()


def test_sweep_rejects_bad_input(smrt_mod):
    p = _prob2d(8, 8, 4, 1)
    ctx = smrt_mod.Context(p)
    sigt = np.ones((p.n_cells, 1))
    sigt[3] = -1.0
    with pytest.raises(smrt_mod.SmrtError):
        ctx.sweep(sigt, sigt, np.zeros((p.n_nodes, 1)), None, 0.0)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_dev_matches_host_sweep(smrt_mod, prec):
    """The device-array entry point runs the same kernels on torch tensors:
    bitwise equal to the host-array sweep; bad opacities are caught on the
    device, bad tensors by the binding."""
    import torch
    p = _prob2d(29, 23, 4, 3, seed=17)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=18)
    sig = 0.6 * sigt
    ctx = smrt_mod.Context(p, precision=prec)
    psi_h, mom_h = ctx.sweep(sigt, sig, q, pp, 0.4, inf)
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
         dict(sigt=sigt, sig=sig, q=q, pp=pp, inf=inf).items()}
    mom_d = torch.zeros((27, p.n_nodes), dtype=torch.float64, device=dev)
    psi_d, _ = ctx.sweep_dev(t["sigt"], t["sig"], t["q"], t["pp"], 0.4, t["inf"], moments_out=mom_d)
    assert np.array_equal(psi_d.cpu().numpy(), psi_h)
    assert np.array_equal(mom_d.cpu().numpy(), mom_h)
    bad = t["sigt"].clone()
    bad[3, 1] = -1.0
    with pytest.raises(smrt_mod.SmrtError):
        ctx.sweep_dev(bad, t["sig"], t["q"], t["pp"], 0.4, t["inf"])
    with pytest.raises(ValueError):
        ctx.sweep_dev(t["sigt"].float(), t["sig"], t["q"], t["pp"], 0.4, t["inf"])
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_sweep2d_s12_max_groups(smrt_mod, oracle_mod, prec, tol):
    """The top of the supported ranges: level-symmetric S12 (84 angles, 21 per
    quadrant: three direction blocks) and 64 groups (the maximum: 16 group
    blocks), ragged mesh, against the oracle element by element."""
    p = _prob2d(21, 18, 12, 64, seed=31, nonuniform=True)
    assert p.n_angles == 84 and p.G == 64
    print(f"S12 G64 21x18 precision {prec}", flush=True)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=32)
    sig = 0.4 * sigt
    o = oracle_mod.Oracle(p)
    ref = o.sweep(sigt, q, pp, 0.6, inf)
    ref_mom = o.moments(sig, ref)
    ctx = smrt_mod.Context(p, precision=prec)
    psi, mom = ctx.sweep(sigt, sig, q, pp, 0.6, inf)
    assert _rel(psi, ref) < tol
    for m in range(27):
        assert _rel(mom[m], ref_mom[m]) < tol, m
    ctx.close()
