"""The allocation-free sweep entry point (smrt_sweep_dev_static) against the
allocating one it mirrors (smrt_sweep_dev), through the C ABI on device
tensors.  Both run the same kernels in the same launch shape, so the results
must agree bit for bit (which is within every parity tolerance).  Two calls in
a row share the library's static work array: the second, on a smaller
problem, must not see what the first left there."""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W

pytestmark = pytest.mark.gpu


def _prob2d(nx, ny, sn, G, seed):
    p = W.gray_2d(n=4, sn=sn)
    p.nx, p.ny = nx, ny
    rng = np.random.default_rng(seed)
    xe = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, nx)])
    ye = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, ny)])
    p.x_edges, p.y_edges = xe / xe[-1], ye / ye[-1]
    p.region_of_cell = np.zeros(nx * ny, np.int32)
    p.G = G
    p.nu_edges = np.logspace(-2, 1, G + 1)
    p.sigma0 = np.ones((1, G))
    p.cv = np.ones(1)
    return p


def _device_inputs(p, seed):
    import torch
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=seed)
    dev = torch.device("cuda:0")
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
            for k, v in dict(sigt=sigt, sig=0.6 * sigt, q=q, pp=pp, inf=inf).items()}


def _both(ctx, t, nmom, with_moments=True, with_prev=True, with_inflow=True):
    import torch
    dev = t["sigt"].device
    out = []
    for static in (False, True):
        mom = torch.full((nmom, t["q"].shape[0]), -7.0, dtype=torch.float64, device=dev) if with_moments else None
        psi, _ = ctx.sweep_dev(t["sigt"], t["sig"], t["q"], t["pp"] if with_prev else None, 0.4,
                               t["inf"] if with_inflow else None, moments_out=mom, static_scratch=static)
        out.append((psi.cpu().numpy(), None if mom is None else mom.cpu().numpy()))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_static_sweep_matches_allocating_sweep_two_calls(smrt_mod, prec):
    # first call: 5 bands in groups of 2 (trace words between workgroups)
    big = _prob2d(45, 70, 4, 3, seed=31)
    print(f"precision {prec}: call 1, 45x70 S4 G3, 2 bands per workgroup", flush=True)
    c1 = smrt_mod.Context(big, precision=prec)
    c1.set_launch(1, 2, 1)
    (pa, ma), (ps, ms) = _both(c1, _device_inputs(big, 32), 27)
    assert np.array_equal(ps, pa) and np.array_equal(ms, ma)
    c1.close()
    # second call: a smaller problem, in the array the first call left behind
    small = _prob2d(20, 18, 4, 2, seed=33)
    print(f"precision {prec}: call 2, 20x18 S4 G2", flush=True)
    c2 = smrt_mod.Context(small, precision=prec)
    t = _device_inputs(small, 34)
    (pa, ma), (ps, ms) = _both(c2, t, 27)
    assert np.array_equal(ps, pa) and np.array_equal(ms, ma)
    # optional arrays absent: no moments, no time-edge source, inflow from the boundary description
    (pa, _), (ps, _) = _both(c2, t, 27, with_moments=False, with_prev=False, with_inflow=False)
    assert np.array_equal(ps, pa)
    c2.close()


def test_static_sweep_1d(smrt_mod):
    p = W.slab_1d(n_cells=53, n_angles=8)
    print("1D static sweep", flush=True)
    c = smrt_mod.Context(p, precision=1)
    t = _device_inputs(p, 41)
    (pa, ma), (ps, ms) = _both(c, t, 8)
    assert np.array_equal(ps, pa) and np.array_equal(ms, ma)
    c.close()


def test_static_sweep_rejects_oversize_and_bad_opacity(smrt_mod):
    import torch
    # 128x128, S8, 16 groups: the internal intensities alone exceed the 64 MiB array
    p = W.multigroup_2d(n=128, G=16)
    print("oversize problem", flush=True)
    c = smrt_mod.Context(p, precision=1)
    dev = torch.device("cuda:0")
    sigt = torch.ones((p.n_cells, p.G), dtype=torch.float64, device=dev)
    q = torch.zeros((p.n_nodes, p.G), dtype=torch.float64, device=dev)
    with pytest.raises(smrt_mod.SmrtError, match="static scratch"):
        c.sweep_dev(sigt, sigt, q, None, 0.0, static_scratch=True)
    c.close()
    small = _prob2d(9, 12, 4, 1, seed=5)
    c = smrt_mod.Context(small, precision=0)
    t = _device_inputs(small, 6)
    bad = t["sigt"].clone()
    bad[3, 0] = -1.0
    with pytest.raises(smrt_mod.SmrtError):
        c.sweep_dev(bad, t["sig"], t["q"], t["pp"], 0.4, t["inf"], static_scratch=True)
    # the array is usable again after a rejected call
    (pa, ma), (ps, ms) = _both(c, t, 27)
    assert np.array_equal(ps, pa) and np.array_equal(ms, ma)
    c.close()
