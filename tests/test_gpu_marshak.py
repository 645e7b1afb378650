"""The Marshak wave of Sec. 6 on the GPU against the FP64 oracle (through
the C ABI): the 1D gray slab in physical units (eV, cm, s), sigma = 1e12/T^3
per cm, c_v = 3e12 erg/(cm^3 eV), a 1 keV source, S6 Gauss-Legendre, on
32 cells with dt = 8e-3 ns to the final 2.5 ns (312 steps), consistent SM
with the zero-and-scale fixup and the temperature floor (as the paper runs
its problems).  Without them the step fails on both sides with the same
status (no positive temperature root ahead of the front).

Tolerance.  With cold cells of optical depth ~1e9 next to the 1 keV face,
the first steps' low-order Newton does not reach the relative inner
tolerance in either implementation (both stop at the 60-iteration cap in the
first outer iteration, with the same CG counts), and with the fixup's
switching the outer iteration has rounding-level limit cycles (the oracle
itself hits the outer cap on two steps at tolerances between 1e-8 and
1e-10).  The two FP64 implementations, which differ in summation order,
then differ by up to ~2e-7 in T at the heated face within the first step's
outer iterations and by 2e-8 after it, and by ~1e-9 for the rest of the run
(measured), so the comparison is made at 1e-6 relative, well below the
errors against the refined reference that the paper reports for this
problem.
"""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W
from test_oracle_reflect import TIGHT

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_marshak_without_fixup_fails_like_the_oracle(smrt_mod, oracle_mod):
    p = W.marshak_1d(32, 8e-3)
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    ctx = smrt_mod.Context(p, precision=0, **TIGHT)
    ctx.set_state(st["T"])
    for k in range(6):
        r, st, _ = o.step(st, oracle_mod.default_opts(**TIGHT))
        if r != 0:
            break
        ctx.step()
    assert r == 5
    with pytest.raises(smrt_mod.SmrtError) as e:
        ctx.step()
    assert e.value.status == smrt_mod.SMRT_E_NONPHYSICAL
    ctx.close()


def test_marshak_wave_to_final_time(smrt_mod, oracle_mod):
    p = W.marshak_1d(32, 8e-3)
    opts = dict(TIGHT, fixup=1, T_floor=1e-8)
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    ctx = smrt_mod.Context(p, precision=0, **opts)
    ctx.set_state(st["T"])
    worst = 0.0
    for k in range(p.n_steps):
        r, st, ost = o.step(st, oracle_mod.default_opts(**opts))
        assert r == 0
        gst = ctx.step()
        if k % 50 == 0 or k == p.n_steps - 1:
            got = ctx.get_state()
            err = _rel(got["T"], st["T"])
            worst = max(worst, err)
            print(f"step {k}: outer {gst['outer']} vs {ost['outer']}, T rel diff {err:.2e}", flush=True)
            assert err < 1e-6, k
            assert got["psi"].min() >= 0.0
    T = ctx.get_state()["T"]
    ctx.close()
    # the wave: hot behind the front, cold ahead; nothing above the source temperature, and the
    # cold end only cools slightly (it radiates through the vacuum face)
    assert T.max() <= 1000.0 and T.min() >= 0.999
    front = np.argmax(T < 500.0) / (2 * p.nx) * 0.05
    assert 0.02 < front < 0.045
