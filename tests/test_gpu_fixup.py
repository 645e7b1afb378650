"""GPU parity of the zero-and-scale negative-flux fixup and the temperature
floor (Sec. 6) against the FP64 oracle, through the C ABI.

* Sweeps with the fixup (FP64 to 1e-10 of the field's maximum, FP32 to
  1e-5; the FP32 kernel takes the fixup decision in FP32, and a value that
  rounds to the other side of zero moves its cell by about one FP32
  rounding) on optically thin and thick cells with a beam entering through
  part of one side, over several tiles, a ragged tail, every launch shape
  family and the 1D kernel; the returned intensity is never negative and
  the fused moments follow the fixed intensity.
* The benchmark's full size and launch (256x256, S8, 16 groups, 5 waves, 1
  group per lane) with the fixup on: sampled groups against the oracle.
* A batch with the fixup matches its problems swept alone; a batch whose
  problems disagree on the fixup is rejected.
* Time steps of a thick gray problem where the fixup changes the answer
  (and, with the time step 10x longer, where the unfixed step has no
  positive temperature), and the temperature floor in the low-order solve
  and in a full step.
* The adjoint refuses the fixup and the floor.
"""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W
from test_oracle_fixup import _mesh2d, beam_inputs_2d

pytestmark = pytest.mark.gpu

TIGHT = dict(eps_outer=1e-11, eps_inner=1e-12, cg_rtol=1e-13, elim_rtol=1e-15, max_outer=200, max_inner=60,
             max_cg=3000)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _inputs(p, seed):
    sigt, q, _, inf = beam_inputs_2d(p, seed)
    rng = np.random.default_rng(seed + 100)
    pp = rng.uniform(0, 1e-3, (p.n_angles, p.G, p.n_nodes))
    return sigt + 0.3, q, pp, inf


SHAPES = [(37, 35, 4, 3), (64, 48, 8, 2), (20, 33, 4, 5), (1, 1, 4, 2), (9, 1, 8, 2)]


@pytest.mark.parametrize("nx,ny,sn,G", SHAPES)
@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_sweep2d_fixup_matches_oracle(smrt_mod, oracle_mod, nx, ny, sn, G, prec, tol):
    print(f"fixup sweep nx={nx} ny={ny} S{sn} G={G} precision {prec}", flush=True)
    p = _mesh2d(nx, ny, sn, G, seed=nx + ny)
    sigt, q, pp, inf = _inputs(p, nx * ny)
    sig = 0.6 * sigt
    o = oracle_mod.Oracle(p)
    ref = o.sweep(sigt, q, pp, 0.3, inf, fixup=True)
    if nx * ny > 100:
        assert (o.sweep(sigt, q, pp, 0.3, inf) < 0).any()      # the case exercises the fixup
    ref_mom = o.moments(sig, ref)
    ctx = smrt_mod.Context(p, precision=prec, fixup=1)
    psi, mom = ctx.sweep(sigt, sig, q, pp, 0.3, inf)
    ctx.close()
    assert psi.min() >= 0.0
    assert _rel(psi, ref) < tol
    for m in range(27):
        assert _rel(mom[m], ref_mom[m]) < tol, m


@pytest.mark.parametrize("launch", [(1, 1, 1), (2, 1, 1), (4, 2, 2), (4, 1, 1), (1, 4, 4), (1, 16, 1), (2, 2, 2)])
def test_sweep2d_fixup_launch_shapes(smrt_mod, oracle_mod, launch):
    p = _mesh2d(45, 40, 8, 3, seed=4)
    sigt, q, pp, inf = _inputs(p, 4)
    ref = oracle_mod.Oracle(p).sweep(sigt, q, pp, 0.3, inf, fixup=True)
    prec = 1 if launch[2] >= 2 else 0
    print(f"fixup launch {launch} precision {prec}", flush=True)
    ctx = smrt_mod.Context(p, precision=prec, fixup=1)
    ctx.set_launch(*launch)
    psi, _ = ctx.sweep(sigt, 0.5 * sigt, q, pp, 0.3, inf)
    ctx.close()
    assert psi.min() >= 0.0
    assert _rel(psi, ref) < (1e-5 if prec else 1e-10)


def test_fixup_switch_at_run_time(smrt_mod, oracle_mod):
    """smrt_set_options turns the fixup on and off on a live context."""
    p = _mesh2d(30, 26, 4, 2, seed=6)
    sigt, q, pp, inf = _inputs(p, 6)
    o = oracle_mod.Oracle(p)
    ctx = smrt_mod.Context(p, precision=0)
    for fix in (0, 1, 0):
        ctx.set_options(fixup=fix)
        psi, _ = ctx.sweep(sigt, 0.5 * sigt, q, pp, 0.3, inf)
        assert _rel(psi, o.sweep(sigt, q, pp, 0.3, inf, fixup=bool(fix))) < 1e-10, fix
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6)])
def test_sweep1d_fixup_matches_oracle(smrt_mod, oracle_mod, prec, tol):
    p = W.slab_1d(n_cells=53, n_angles=8)
    rng = np.random.default_rng(9)
    h = rng.uniform(0.5, 1.5, p.nx)
    p.x_edges = np.r_[0.0, np.cumsum(h)] / h.sum()
    p.G = 3
    p.nu_edges = np.array([0.01, 0.1, 1.0, 10.0])
    p.sigma0 = np.ones((1, 3))
    sigt = 10.0 ** rng.uniform(-1, 3, (p.n_cells, p.G))
    q = rng.uniform(0, 1, (p.n_nodes, p.G)) ** 4
    inf = np.zeros((p.n_angles, p.G, 2))
    inf[:, :, 0] = 1.0
    o = oracle_mod.Oracle(p)
    assert (o.sweep(sigt, q, None, 0.0, inf) < 0).any()
    ref = o.sweep(sigt, q, None, 0.0, inf, fixup=True)
    ctx = smrt_mod.Context(p, precision=prec, fixup=1)
    psi, _ = ctx.sweep(sigt, 0.3 * sigt, q, None, 0.0, inf)
    ctx.close()
    assert psi.min() >= 0.0
    assert _rel(psi, ref) < tol


@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (0, 1e-10)])
def test_fixup_full_size_sampled_groups(smrt_mod, oracle_mod, prec, tol):
    import copy
    p = W.multigroup_2d()
    print(f"full size 256x256 S8 G16 with fixup, precision {prec}, launch (5 waves, 1 group per lane)", flush=True)
    sigt, q, pp, inf = W.random_sweep_inputs(p, seed=77)
    rng = np.random.default_rng(77)
    sigt = 10.0 ** rng.uniform(-1, 3, sigt.shape)
    inf[:] = 0.0
    inf[:, :, 2 * 64:2 * 128] = 1.0               # a beam through a quarter of the x- side
    sig = 0.8 * sigt
    ctx = smrt_mod.Context(p, precision=prec, fixup=1)
    psi, mom = ctx.sweep(sigt, sig, q, pp, 0.5, inf)
    ctx.close()
    assert psi.min() >= 0.0
    S = [0, 15]
    sub = copy.copy(p)
    sub.G = len(S)
    sub.nu_edges = np.logspace(-3.0, 1.0, sub.G + 1)
    o = oracle_mod.Oracle(sub)
    args = (np.ascontiguousarray(sigt[:, S]), np.ascontiguousarray(q[:, S]), np.ascontiguousarray(pp[:, S, :]), 0.5,
            np.ascontiguousarray(inf[:, S, :]))
    ref = o.sweep(*args, fixup=True)
    assert (o.sweep(*args) < 0).any()
    for i, g in enumerate(S):
        assert _rel(psi[:, g, :], ref[:, i, :]) < tol, g
    # the fused scalar flux follows the fixed intensity
    phi = sum(mom[6 * k] for k in range(4))
    want = np.einsum("d,dgn->n", p.w, psi)
    assert _rel(phi, want) < (1e-5 if prec else 1e-12)


def _batch_problems():
    ps = W.batch_2d(n_problems=3, seed=11, sizes=[16, 24, 40])
    for p in ps:
        p.T0 = 0.001                      # a cold start: steep inflow, negative unfixed intensities
        p.dt = 0.1
    return ps


def test_batch_fixup_matches_single_problem_launches(smrt_mod):
    ps = _batch_problems()
    single, batched = [], []
    for p in ps:
        for lst in (single, batched):
            c = smrt_mod.Context(p, precision=0, fixup=1)
            c.set_state(p.initial_T_nodes())
            lst.append(c)
    b = smrt_mod.Batch(batched)
    info = b.info()
    for c in single:
        c.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
        c.sweep_resident(ps[0].dt, n_times=1)
    b.sweep_resident(ps[0].dt, n_times=1)
    for c1, c2 in zip(single, batched):
        assert _rel(c2.get_moments(), c1.get_moments()) < 1e-12
    b.close()
    for c in single + batched:
        c.close()


def test_batch_rejects_mixed_fixup(smrt_mod):
    ps = _batch_problems()[:2]
    cs = []
    for p, fix in zip(ps, (0, 1)):
        c = smrt_mod.Context(p, precision=0, fixup=fix)
        c.set_state(p.initial_T_nodes())
        cs.append(c)
    b = smrt_mod.Batch(cs)
    with pytest.raises(smrt_mod.SmrtError) as e:
        b.sweep_resident(ps[0].dt, n_times=1)
    assert e.value.status == smrt_mod.SMRT_E_INVALID_ARG
    b.close()
    for c in cs:
        c.close()


def _gray_thick(dt, block=1):
    p = W.gray_2d(n=16, sn=4, block=block, seed=2)
    p.dt = dt
    return p


def _steps(smrt_mod, oracle_mod, p, n_steps, opts):
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    ctx = smrt_mod.Context(p, precision=0, **opts)
    ctx.set_state(st["T"])
    out = []
    for k in range(n_steps):
        print(f"step {k} opts {sorted(opts)}", flush=True)
        r, st, ost = o.step(st, oracle_mod.default_opts(**opts))
        assert r == 0
        gst = ctx.step()
        out.append((st, ost, ctx.get_state(), gst))
    ctx.close()
    return out


def test_step_with_fixup_matches_oracle(smrt_mod, oracle_mod):
    p = _gray_thick(0.1)
    o = oracle_mod.Oracle(p)
    st0 = o.initial_state()
    _, plain, _ = o.step(st0, oracle_mod.default_opts(**TIGHT))
    _, fixed, _ = o.step(st0, oracle_mod.default_opts(fixup=1, **TIGHT))
    assert plain["psi"].min() < 0.0 and _rel(fixed["T"], plain["T"]) > 1e-3    # the fixup changes the step
    for ref, ost, got, gst in _steps(smrt_mod, oracle_mod, p, 2, dict(TIGHT, fixup=1)):
        assert got["psi"].min() >= 0.0
        assert _rel(got["T"], ref["T"]) < 1e-10
        assert _rel(got["E"], ref["E"]) < 1e-10
        assert _rel(got["psi"], ref["psi"]) < 1e-10
        assert abs(gst["outer"] - ost["outer"]) <= 1


def test_lo_solve_temperature_floor(smrt_mod, oracle_mod):
    """Half the nodes get an energy source so negative that their balance has
    no positive root: the floored solve succeeds and matches the oracle."""
    p = W.gray_2d(n=8, sn=4, block=4, seed=2)
    nn = p.n_nodes
    T = p.initial_T_nodes()
    qE = np.full(nn, -1.0e6)
    qE[: nn // 2] = 0.0
    cl = dict(sigE=np.ones(nn), sigF=np.ones(nn), sigP=np.ones(nn), qE=qE, qF=np.zeros((nn, p.dim)))
    floor = 1e-8
    r, E_ref, F_ref, T_ref, _ = oracle_mod.Oracle(p).lo_solve(oracle_mod.default_opts(T_floor=floor, **TIGHT), p.dt,
                                                              T, cl, p.a * T ** 4, T)
    assert r == 0 and (T_ref == floor).any()
    ctx = smrt_mod.Context(p, precision=0, T_floor=floor, **TIGHT)
    rows = np.vstack([cl["sigE"], cl["sigF"], cl["sigP"], cl["qE"], cl["qF"].T])
    E, F, Tg, _ = ctx.lo_solve(rows, T, p.dt, p.a * T ** 4, T)
    ctx.close()
    assert Tg.min() >= floor
    assert np.array_equal(Tg == floor, T_ref == floor)
    assert _rel(Tg, T_ref) < 1e-10
    assert _rel(E, E_ref) < 1e-10


def test_step_temperature_floor_matches_oracle(smrt_mod, oracle_mod):
    """A time step 10x longer: without the floor (and without the fixup) the
    energy balance loses its positive root; with the floor the step
    converges, on the GPU as in the oracle."""
    p = _gray_thick(1.0, block=2)
    o = oracle_mod.Oracle(p)
    r, _, _ = o.step(o.initial_state(), oracle_mod.default_opts(**TIGHT))
    assert r == 5
    for ref, ost, got, gst in _steps(smrt_mod, oracle_mod, p, 1, dict(TIGHT, T_floor=1e-8)):
        assert got["T"].min() >= 1e-8
        assert _rel(got["T"], ref["T"]) < 1e-8
        assert _rel(got["E"], ref["E"]) < 1e-8
        assert abs(gst["outer"] - ost["outer"]) <= 3


def test_adjoint_rejects_fixup_and_floor(smrt_mod):
    p = W.adjoint_2d(n=16, G=2)
    for kw in (dict(fixup=1), dict(T_floor=1e-8)):
        ctx = smrt_mod.Context(p, precision=0, **kw)
        ctx.set_state(p.initial_T_nodes())
        with pytest.raises(smrt_mod.SmrtError) as e:
            ctx.adjoint(1, p.dt)
        assert e.value.status == smrt_mod.SMRT_E_INVALID_ARG
        ctx.close()
