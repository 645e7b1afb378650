"""GPU tests of the batched persistent sweep (many uneven problems in one
launch), its HIP-graph replay, the lock-stepped batched time step and the
launch-shape autotuners, through the C ABI.

Each batched result is compared with the same problem run on its own
context (the single-problem launch) and, for one problem, with the FP64
oracle on identical inputs.
"""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _problems():
    # uneven sizes, group counts and quadratures from the batch recipe
    ps = W.batch_2d(n_problems=4, seed=11, sizes=[16, 24, 40])
    return ps


def _contexts(smrt_mod, problems, prec):
    cs = []
    for p in problems:
        c = smrt_mod.Context(p, precision=prec)
        c.set_state(p.initial_T_nodes())
        cs.append(c)
    return cs


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)])
def test_batched_pass_matches_single_problem_launches(smrt_mod, prec, tol):
    ps = _problems()
    print("batch:", [p.name for p in ps], flush=True)
    single = _contexts(smrt_mod, ps, prec)
    batched = _contexts(smrt_mod, ps, prec)
    b = smrt_mod.Batch(batched)
    info = b.info()
    for c in single:
        c.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
        c.sweep_resident(n_times=1)
    b.sweep_resident(ps[0].dt, n_times=1)
    for c1, c2 in zip(single, batched):
        m1, m2 = c1.get_moments(), c2.get_moments()
        assert _rel(m2, m1) < tol
    b.close()
    for c in single + batched:
        c.close()


def test_batched_pass_fp64_matches_oracle(smrt_mod, oracle_mod):
    ps = _problems()
    cs = _contexts(smrt_mod, ps, 0)
    b = smrt_mod.Batch(cs)
    b.sweep_resident(ps[0].dt, n_times=1)
    p = ps[0]
    o = oracle_mod.Oracle(p)
    T = p.initial_T_nodes()
    sig = o.opacity(T)
    icdt = 1.0 / (p.c * p.dt)
    st = o.initial_state()
    B = p.a * p.c * T ** 4 / (4 * np.pi)
    frac = np.array([o.spectra(t)[0] for t in T])
    q = sig[np.arange(p.n_nodes) // 4, :] * B[:, None] * frac
    ref = o.sweep(sig + icdt, q, st["psi"], icdt, o.inflow())
    ref_m = o.moments(sig, ref)
    m = cs[0].get_moments()
    for k in range(27):
        assert _rel(m[k], ref_m[k]) < 1e-10, k
    b.close()
    for c in cs:
        c.close()


def test_batched_graph_replay_matches_eager(smrt_mod):
    ps = _problems()
    cs = _contexts(smrt_mod, ps, 1)
    b = smrt_mod.Batch(cs)
    b.sweep_resident(ps[0].dt, n_times=1, capture_graph=False)
    eager = [c.get_moments() for c in cs]
    for rep in range(3):
        # replays with eager work and synchronisation in between
        b.sweep_resident(ps[0].dt, n_times=2, capture_graph=True)
        for c, e in zip(cs, eager):
            assert np.array_equal(c.get_moments(), e), rep
        b.sweep_resident(ps[0].dt, n_times=1, capture_graph=False)
    b.close()
    for c in cs:
        c.close()


def test_batched_steps_match_single_problem_steps(smrt_mod):
    ps = _problems()[:3]
    single = _contexts(smrt_mod, ps, 0)
    batched = _contexts(smrt_mod, ps, 0)
    b = smrt_mod.Batch(batched)
    info = b.info()
    for c in single:
        c.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
    for step in range(2):
        print("step", step, flush=True)
        s1 = [c.step(p.dt) for c, p in zip(single, ps)]
        s2 = b.step([p.dt for p in ps])
        for a, c in zip(s1, s2):
            assert a["outer"] == c["outer"] and a["cg_total"] == c["cg_total"]
    for c1, c2 in zip(single, batched):
        g1, g2 = c1.get_state(), c2.get_state()
        for k in ("T", "E", "F", "psi"):
            assert _rel(g2[k], g1[k]) < 1e-12, k
    b.close()
    for c in single + batched:
        c.close()


def test_batch_autotune_keeps_results(smrt_mod):
    ps = _problems()
    cs = _contexts(smrt_mod, ps, 1)
    b = smrt_mod.Batch(cs)
    b.sweep_resident(ps[0].dt, n_times=1)
    before = [c.get_moments() for c in cs]
    nw, nb, k, ms = b.autotune(ps[0].dt)
    print("batch autotune:", nw, nb, k, ms, flush=True)
    assert nw in (1, 2, 4) and nb in (1, 2, 4, 8, 16) and nw * nb <= 16 and k in (1, 2, 4) and ms > 0
    assert b.info()["waves_per_band"] == nw and b.info()["bands_per_group"] == nb
    b.sweep_resident(ps[0].dt, n_times=1)
    for c, m in zip(cs, before):
        assert _rel(c.get_moments(), m) < 1e-6
    b.close()
    for c in cs:
        c.close()


def test_single_autotune(smrt_mod):
    p = W.multigroup_2d(n=48, G=8)
    c = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP32)
    c.set_state(p.initial_T_nodes())
    c.sweep_resident(n_times=1)
    before = c.get_moments()
    nw, nb, k, ms = c.autotune()
    print("autotune:", nw, nb, k, ms, flush=True)
    i = c.info()
    assert i["waves_per_band"] == nw and i["bands_per_group"] == nb and i["pairs_per_lane"] == k
    c.sweep_resident(n_times=1)
    assert _rel(c.get_moments(), before) < 1e-6
    c.close()


def test_autotune_cache_reuses_shape(smrt_mod, tmp_path):
    """A tuned shape is stored on disk under the device and sweep shape and
    applied without timing on the next call (single context and batch)."""
    from paper_2504_21784_amd.tune_cache import TuneCache
    cache = TuneCache(str(tmp_path / "shapes.json"))
    print("device:", smrt_mod.device_name(), flush=True)
    p = W.multigroup_2d(n=48, G=8)
    c = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP32)
    c.set_state(p.initial_T_nodes())
    first = c.autotune(cache=cache)
    assert not c.last_tune_cached
    c2 = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP32)
    c2.set_state(p.initial_T_nodes())
    again = c2.autotune(cache=cache)
    assert c2.last_tune_cached and again[:3] == first[:3]
    i = c2.info()
    assert (i["waves_per_band"], i["bands_per_group"], i["pairs_per_lane"]) == first[:3]
    c.sweep_resident(n_times=1)
    c2.sweep_resident(n_times=1)
    assert np.array_equal(c.get_moments(), c2.get_moments())
    c.close()
    c2.close()
    ps = _problems()
    b = smrt_mod.Batch(_contexts(smrt_mod, ps, 1))
    bf = b.autotune(ps[0].dt, cache=cache)
    assert not b.last_tune_cached
    b2 = smrt_mod.Batch(_contexts(smrt_mod, ps, 1))
    bs = b2.autotune(ps[0].dt, cache=cache)
    assert b2.last_tune_cached and bs[:3] == bf[:3]
    for bb in (b, b2):
        for x in bb.contexts:
            x.close()
        bb.close()


def test_batch_rejects_mixed_precision(smrt_mod):
    ps = _problems()[:2]
    a = smrt_mod.Context(ps[0], precision=0)
    c = smrt_mod.Context(ps[1], precision=1)
    a.set_state(ps[0].initial_T_nodes())
    c.set_state(ps[1].initial_T_nodes())
    with pytest.raises(smrt_mod.SmrtError):
        smrt_mod.Batch([a, c])
    a.close()
    c.close()


def test_full_batch_matches_single_problem_launches(smrt_mod):
    """The benchmark's batch at full size (32 problems, n in {64..384}, G in
    {4..32}, S4/S8/S12, FP32) in one launch with the launch shape the
    benchmark reports (4 waves x 2 groups per lane): the largest, the
    smallest and one middle problem match the same problem launched alone
    with the same shape (which the full-size sweep test checks against the
    oracle).  The shape (2 waves per band, 4 bands per workgroup, 2 groups
    per lane) puts several band groups on the larger problems, so the
    workgroup-to-workgroup trace hand-off is exercised too."""
    ps = W.batch_2d()
    print("full batch:", len(ps), "problems", flush=True)
    cs = _contexts(smrt_mod, ps, 1)
    b = smrt_mod.Batch(cs)
    b.set_launch(2, 4, 2)
    b.sweep_resident(ps[0].dt, n_times=1)
    sizes = [p.nx * p.ny * p.n_angles * p.G for p in ps]
    picks = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), len(ps) // 2})
    for i in picks:
        print("problem", ps[i].name, flush=True)
        single = smrt_mod.Context(ps[i], precision=1)
        single.set_state(ps[i].initial_T_nodes())
        single.set_launch(2, 4, 2)
        single.sweep_resident(ps[i].dt, n_times=1)
        assert _rel(cs[i].get_moments(), single.get_moments()) < 1e-6, ps[i].name
        single.close()
    b.close()
    for c in cs:
        c.close()
