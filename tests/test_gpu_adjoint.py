"""GPU adjoint sweep (transpose of the lumped upwind DG operator) against the
FP64 oracle's explicitly transposed sweep, and the GPU dot-product identity
<w.s, L^{-1}(w.q)> = <L^{-T}(w.s), w.q>, through the C ABI."""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W

from test_gpu_sweep import _prob2d

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _wnodes(p):
    if p.dim == 1:
        return np.repeat(np.diff(p.x_edges) / 2, 2)
    hx, hy = np.diff(p.x_edges), np.diff(p.y_edges)
    return np.repeat((hy[:, None] * hx[None, :] / 4).ravel(), 4)


def _inputs(p, seed):
    rng = np.random.default_rng(seed)
    sigt = 10 ** rng.uniform(np.log10(0.5), np.log10(200.0), (p.n_cells, p.G))
    src = rng.uniform(-1, 1, (p.n_angles, p.G, p.n_nodes))
    emis = rng.uniform(0, 1, (p.n_nodes, p.G))
    I = rng.uniform(0, 1, (p.n_angles, p.G, p.n_nodes))
    return sigt, src, emis, I


@pytest.mark.parametrize("nx,ny,sn,G", [(37, 35, 4, 3), (16, 16, 8, 1), (20, 33, 8, 2), (1, 1, 4, 2)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_adjoint_sweep_matches_oracle_2d(smrt_mod, oracle_mod, nx, ny, sn, G, prec, tol):
    p = _prob2d(nx, ny, sn, G, seed=nx + ny, nonuniform=True)
    print(f"adjoint nx={nx} ny={ny} S{sn} G={G} prec={prec}", flush=True)
    sigt, src, emis, I = _inputs(p, 13)
    ref, ref_d = oracle_mod.Oracle(p).adjoint_sweep(sigt, src, emis, I)
    ctx = smrt_mod.Context(p, precision=prec)
    lam, dsig = ctx.adjoint_sweep(sigt, src, emis, I, want_dsig=True)
    assert _rel(lam, ref) < tol
    assert _rel(dsig, ref_d) < tol
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6)])
def test_adjoint_sweep_matches_oracle_1d(smrt_mod, oracle_mod, prec, tol):
    p = W.slab_1d(n_cells=41, n_angles=8)
    p.G = 3
    p.nu_edges = np.array([0.01, 0.1, 1.0, 10.0])
    p.sigma0 = np.ones((1, 3))
    sigt, src, emis, I = _inputs(p, 21)
    ref, ref_d = oracle_mod.Oracle(p).adjoint_sweep(sigt, src, emis, I)
    ctx = smrt_mod.Context(p, precision=prec)
    lam, dsig = ctx.adjoint_sweep(sigt, src, emis, I, want_dsig=True)
    assert _rel(lam, ref) < tol
    assert _rel(dsig, ref_d) < tol
    ctx.close()


def test_adjoint_dot_product_on_gpu(smrt_mod):
    p = _prob2d(45, 29, 8, 2, seed=2, nonuniform=True)
    sigt, s, _, _ = _inputs(p, 3)
    rng = np.random.default_rng(4)
    q = rng.uniform(-1, 1, s.shape)
    nb = W.boundary_node_count(p)
    ctx = smrt_mod.Context(p, precision=0)
    I, _ = ctx.sweep(sigt, sigt, np.zeros((p.n_nodes, p.G)), q, 1.0, np.zeros((p.n_angles, p.G, nb)))
    lam = ctx.adjoint_sweep(sigt, s)
    w = _wnodes(p)
    lhs, rhs = np.sum(w * s * I), np.sum(lam * w * q)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(w * s * I))
    ctx.close()
