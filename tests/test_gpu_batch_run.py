"""GPU tests of the multi-step batched run with device-side convergence
control (smrt_batch_run), through the C ABI.

Every problem of a batched run must equal, bit for bit, the same problem
stepped alone with smrt_step (same launch shape, FP64): the outer decision
is the same test taken on the device, and the batched LO launch runs the
single-problem LO's block decomposition through the same device bodies.
The captured block of outer iterations must replay to the eager result, and
the smallest problems of the full 32-problem batch are checked against the
FP64 oracle's steps.
"""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W
from parity import rel_pointwise

pytestmark = pytest.mark.gpu

TIGHT = dict(eps_outer=1e-11, eps_inner=1e-12, cg_rtol=1e-13, elim_rtol=1e-15, max_outer=200, max_inner=60,
             max_cg=3000)
STAT_KEYS = ("outer", "inner_total", "cg_total", "elim_max", "hit_max")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _contexts(smrt_mod, problems, prec, **opts):
    cs = []
    for p in problems:
        c = smrt_mod.Context(p, precision=prec, **opts)
        c.set_state(p.initial_T_nodes())
        cs.append(c)
    return cs


def _close(*groups):
    for g in groups:
        for c in g:
            c.close()


def _assert_same_state(c1, c2, what):
    g1, g2 = c1.get_state(), c2.get_state()
    for k in ("T", "E", "F", "psi"):
        if not np.array_equal(g1[k], g2[k]):
            raise AssertionError(f"{what}: {k} differs, max rel {_rel(g2[k], g1[k]):.3e}")


@pytest.mark.parametrize("scheme", [0, 1])
def test_batch_run_fp64_equals_single_steps(smrt_mod, scheme):
    ps = W.batch_2d(n_problems=4, seed=11, sizes=[16, 24, 40])[:3]
    print("batch:", [p.name for p in ps], flush=True)
    single = _contexts(smrt_mod, ps, 0, scheme=scheme)
    batched = _contexts(smrt_mod, ps, 0, scheme=scheme)
    b = smrt_mod.Batch(batched)
    info = b.info()
    for c in single:
        c.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
    n_steps = 3
    ref = [[c.step(p.dt) for c, p in zip(single, ps)] for _ in range(n_steps)]
    got = b.run(n_steps, [p.dt for p in ps])
    for s in range(n_steps):
        for i in range(len(ps)):
            for k in STAT_KEYS:
                assert got[s][i][k] == ref[s][i][k], (s, i, k, got[s][i][k], ref[s][i][k])
    for i, (c1, c2) in enumerate(zip(single, batched)):
        _assert_same_state(c1, c2, f"problem {i}")
    b.close()
    _close(single, batched)


def test_batch_run_fp32_equals_single_steps(smrt_mod):
    ps = W.batch_2d(n_problems=4, seed=12, sizes=[16, 32])
    single = _contexts(smrt_mod, ps, 1)
    batched = _contexts(smrt_mod, ps, 1)
    b = smrt_mod.Batch(batched)
    info = b.info()
    for c in single:
        c.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
    ref = [[c.step(p.dt) for c, p in zip(single, ps)] for _ in range(2)]
    got = b.run(2, [p.dt for p in ps])
    for s in range(2):
        for i in range(len(ps)):
            assert got[s][i]["outer"] == ref[s][i]["outer"], (s, i)
            assert got[s][i]["cg_total"] == ref[s][i]["cg_total"], (s, i)
    for i, (c1, c2) in enumerate(zip(single, batched)):
        _assert_same_state(c1, c2, f"problem {i}")
    b.close()
    _close(single, batched)


def test_batch_run_graph_equals_eager(smrt_mod):
    ps = W.batch_2d(n_problems=4, seed=11, sizes=[16, 24, 40])
    eager = _contexts(smrt_mod, ps, 1)
    graph = _contexts(smrt_mod, ps, 1)
    be, bg = smrt_mod.Batch(eager), smrt_mod.Batch(graph)
    dts = [p.dt for p in ps]
    for rep in range(3):
        # captured replays, with eager work and waits between the calls
        se = be.run(2, dts, capture_graph=False)
        sg = bg.run(2, dts, capture_graph=True)
        for s in range(2):
            for i in range(len(ps)):
                assert se[s][i]["outer"] == sg[s][i]["outer"], (rep, s, i)
        for i, (c1, c2) in enumerate(zip(eager, graph)):
            _assert_same_state(c1, c2, f"rep {rep} problem {i}")
        be.sweep_resident(ps[0].dt, n_times=1)
    be.close()
    bg.close()
    _close(eager, graph)


def test_batch_run_per_step_dt_and_fixed_outer(smrt_mod):
    ps = W.batch_2d(n_problems=3, seed=13, sizes=[16, 24])
    single = _contexts(smrt_mod, ps, 0, fixed_outer=3)
    batched = _contexts(smrt_mod, ps, 0, fixed_outer=3)
    b = smrt_mod.Batch(batched)
    info = b.info()
    for c in single:
        c.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
    dt = np.array([[1e-3, 2e-3, 5e-4], [3e-3, 1e-3, 1e-3]])
    ref = [[c.step(dt[s, i]) for i, c in enumerate(single)] for s in range(2)]
    got = b.run(2, dt, capture_graph=True)
    for s in range(2):
        for i in range(3):
            assert got[s][i]["outer"] == 3 == ref[s][i]["outer"]
            assert got[s][i]["cg_total"] == ref[s][i]["cg_total"]
    for i, (c1, c2) in enumerate(zip(single, batched)):
        _assert_same_state(c1, c2, f"problem {i}")
    b.close()
    _close(single, batched)


def test_batch_run_rejects_unsupported(smrt_mod):
    ps = W.batch_2d(n_problems=2, seed=11, sizes=[16])
    cs = _contexts(smrt_mod, ps, 0)
    b = smrt_mod.Batch(cs)
    with pytest.raises(smrt_mod.SmrtError) as e:
        b.run(0, [p.dt for p in ps])
    assert e.value.status == smrt_mod.SMRT_E_INVALID_ARG
    with pytest.raises(smrt_mod.SmrtError) as e:
        b.run(1, [-1.0, 1e-3])
    assert e.value.status == smrt_mod.SMRT_E_INVALID_ARG
    cs[1].set_options(lo_precond=1)
    with pytest.raises(smrt_mod.SmrtError) as e:
        b.run(1, [p.dt for p in ps])
    assert e.value.status == smrt_mod.SMRT_E_INVALID_ARG
    cs[1].set_options(lo_precond=0, scheme=2)
    with pytest.raises(smrt_mod.SmrtError) as e:
        b.run(1, [p.dt for p in ps])
    assert e.value.status == smrt_mod.SMRT_E_INVALID_ARG
    b.close()
    _close(cs)


def test_batch_run_strict_reports_capped_iterations(smrt_mod):
    ps = W.batch_2d(n_problems=2, seed=11, sizes=[16])
    cs = _contexts(smrt_mod, ps, 0, max_cg=1, strict=1)
    b = smrt_mod.Batch(cs)
    with pytest.raises(smrt_mod.SmrtError) as e:
        b.run(2, [p.dt for p in ps])
    assert e.value.status == smrt_mod.SMRT_E_NOT_CONVERGED
    b.close()
    _close(cs)


def test_full_batch_run_fp64_smallest_against_oracle(smrt_mod, oracle_mod):
    """The full 32-problem batch (seed 5), one FP64 step with tight
    tolerances: its two smallest problems against the FP64 oracle's step
    (1e-10 max-normalised; pointwise 1e-10 for T and E, 1e-9 for the
    intensity) and its largest against the same problem stepped alone (bit
    for bit)."""
    ps = W.batch_2d()
    units = [p.nx * p.ny * p.n_angles * p.G for p in ps]
    order = np.argsort(units)
    small, big = [int(i) for i in order[:2]], int(order[-1])
    print("smallest:", [ps[i].name for i in small], "largest:", ps[big].name, flush=True)
    cs = _contexts(smrt_mod, ps, 0, **TIGHT)
    b = smrt_mod.Batch(cs)
    info = b.info()
    st = b.run(1, [p.dt for p in ps], capture_graph=True)
    print("batched step done; outer counts", [s["outer"] for s in st[0]], flush=True)
    for i in small:
        p = ps[i]
        o = oracle_mod.Oracle(p)
        r, ref, ost = o.step(o.initial_state(), oracle_mod.default_opts(**TIGHT))
        assert r == 0
        got = cs[i].get_state()
        print(f"{p.name}: outer {st[0][i]['outer']} (oracle {ost['outer']}), T {_rel(got['T'], ref['T']):.2e}",
              flush=True)
        for k in ("T", "E", "psi"):
            assert _rel(got[k], ref[k]) < 1e-10, (p.name, k)
            # the intensity pointwise to 1e-9, as at the full benchmark size: its
            # smallest elements above the floor carry the tiny Planck fractions
            # of the highest groups, which the GPU's series and the oracle's
            # quadrature round differently
            assert rel_pointwise(got[k], ref[k]) < (1e-9 if k == "psi" else 1e-10), (p.name, k)
        assert abs(st[0][i]["outer"] - ost["outer"]) <= 1
    alone = _contexts(smrt_mod, [ps[big]], 0, **TIGHT)[0]
    alone.set_launch(info["waves_per_band"], info["bands_per_group"], info["pairs_per_lane"])
    sa = alone.step(ps[big].dt)
    assert sa["outer"] == st[0][big]["outer"] and sa["cg_total"] == st[0][big]["cg_total"]
    _assert_same_state(alone, cs[big], ps[big].name)
    alone.close()
    b.close()
    _close(cs)


def test_batch_run_captured_as_first_call_of_a_process():
    """A fresh process whose first GPU work is a captured batched run (so the
    sweep's one-time launch attributes are set during capture) gets the same
    bits as an eager run in another fresh process."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys, hashlib, numpy as np\n"
        f"sys.path.insert(0, {root!r})\n"
        "from paper_2504_21784_amd import smrt, workloads as W\n"
        "ps = W.batch_2d(n_problems=3, seed=11, sizes=[16, 24])\n"
        "cs = []\n"
        "for p in ps:\n"
        "    c = smrt.Context(p, precision=smrt.SMRT_FP32)\n"
        "    c.set_state(p.initial_T_nodes())\n"
        "    cs.append(c)\n"
        "b = smrt.Batch(cs)\n"
        "b.run(2, [p.dt for p in ps], capture_graph=bool(int(sys.argv[1])))\n"
        "h = hashlib.sha256()\n"
        "for c in cs:\n"
        "    s = c.get_state()\n"
        "    for k in ('T', 'E', 'psi'):\n"
        "        h.update(np.ascontiguousarray(s[k]).tobytes())\n"
        "print(h.hexdigest())\n")
    out = []
    for cap in ("1", "0"):
        r = subprocess.run([sys.executable, "-c", code, cap], capture_output=True, text=True, timeout=180)
        assert r.returncode == 0, r.stderr[-2000:]
        out.append(r.stdout.strip().splitlines()[-1])
        print("capture", cap, out[-1][:16], flush=True)
    assert out[0] == out[1]
