"""One time step of the full-size multigroup workload (256x256, S8, 16
groups) on the GPU in the form the benchmark times (FP32 sweep, FP64
low-order solve), against the FP64 oracle's step stored by
tests/golden/make_c3_step.py (both sides iterated to tight tolerances, so the
difference is the FP32 sweep's rounding).  Errors at the 4096 stored nodes:
scalar flux and E within 1e-5, T within 1e-6 (sampled relative L2 and
pointwise, the latter floored at 1e-12 of the field's max), total energy
within 1e-6."""
import os

import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_step1_oracle.npz")


def c3_errors(smrt_mod, precision):
    """The GPU step against the stored oracle step: dict of errors."""
    g = np.load(GOLDEN, allow_pickle=False)
    opts = {str(k): float(v) for k, v in zip(g["opt_names"], g["opts"])}
    for k in ("max_outer", "max_inner", "max_cg"):
        opts[k] = int(opts[k])
    p = W.multigroup_2d()
    ctx = smrt_mod.Context(p, precision=precision, **opts)
    ctx.set_state(p.initial_T_nodes())
    st = ctx.step()
    s = ctx.get_state()
    ctx.close()
    phi = np.einsum("d,dgn->n", p.w, s["psi"])
    hx, hy = np.diff(p.x_edges), np.diff(p.y_edges)
    V = np.repeat((hx[None, :] * hy[:, None]).ravel() / 4.0, 4)
    cv = np.repeat(np.asarray(p.cv)[np.asarray(p.region_of_cell)], 4)
    idx = g["nodes"]
    out = {"outer": int(st["outer"]), "oracle_outer": int(g["outer"])}
    for name, field in (("phi", phi), ("T", s["T"]), ("E", s["E"])):
        ref, got = g[name], field[idx]
        out[name + "_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        floor = 1e-12 * float(g[name + "_max"])
        out[name + "_pointwise"] = float((np.abs(got - ref) / np.maximum(np.abs(ref), floor)).max())
        out[name + "_norm_rel"] = float(abs(np.linalg.norm(field) - g[name + "_norm"]) / g[name + "_norm"])
    energy = float(np.sum(V * (s["E"] + cv * s["T"])))
    out["energy_rel"] = abs(energy - float(g["energy"])) / abs(float(g["energy"]))
    return out


@pytest.mark.parametrize("precision", [1, 0])
def test_c3_step_against_oracle(smrt_mod, precision):
    print(f"256x256 S8 G16 step, precision {precision}", flush=True)
    e = c3_errors(smrt_mod, precision)
    print("  ", {k: (f"{v:.3e}" if isinstance(v, float) else v) for k, v in e.items()}, flush=True)
    if precision == 1:
        tol = {"phi": 1e-5, "T": 1e-6, "E": 1e-5}
        etol = 1e-6
    else:
        tol = {"phi": 1e-10, "T": 1e-10, "E": 1e-10}
        etol = 1e-10
    for name, t in tol.items():
        assert e[name + "_rel_l2"] < t, name
        assert e[name + "_pointwise"] < t, name
        assert e[name + "_norm_rel"] < t, name
    assert e["energy_rel"] < etol
    assert abs(e["outer"] - e["oracle_outer"]) <= 1
