"""GPU tests of the aggregation multigrid preconditioner of the LO conjugate
gradients (Sec. 5 preconditions them with algebraic multigrid), through the
C ABI.  The preconditioner changes the iteration, not the solution:

* the LO solve with the V-cycle equals the FP64 oracle's solve (Jacobi-PCG
  to 1e-13) to 1e-10, in 2D and 1D, on a diffusion-dominated linearisation
  (long time step), where it needs several times fewer CG iterations than
  Jacobi;
* full time steps with it equal the oracle's steps;
* the captured-graph replay gives the same bits as direct launches;
* at the benchmark size the multigrid and Jacobi steps agree.
"""
import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W
from test_oracle_reflect import TIGHT

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _lo_case(oracle_mod, p):
    """Closures of one sweep from a perturbed equilibrium state."""
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    T = st["T"] * (1.0 + 0.3 * np.random.default_rng(1).uniform(size=p.n_nodes))
    sig = o.opacity(T)
    sigt = sig + 1.0 / (p.c * p.dt)
    q = np.zeros((p.n_nodes, p.G))
    npc = p.nodes_per_cell
    for n in range(p.n_nodes):
        b, _ = o.spectra(T[n])
        q[n] = sig[n // npc] * p.a * p.c * T[n] ** 4 * b / (4 * np.pi)
    psi = o.sweep(sigt, q, st["psi"], 1.0 / (p.c * p.dt), o.inflow())
    Estar = np.einsum("d,dgn->n", p.w, st["psi"]) / p.c
    Fstar = np.einsum("d,da,dgn->na", p.w, p.omega[:, :p.dim], st["psi"])
    cl = o.closures(0, p.dt, sig, T, Estar, Fstar, psi, o.inflow())
    return o, T, cl, Estar


def _diffusive_2d():
    # gray, sigma per 4x4-cell block log-uniform in [0.1, 1000], a long step: in the thin
    # blocks the diffusion term outweighs the diagonal by orders of magnitude (Jacobi-PCG
    # needs ~275 iterations per Newton step on 48x48 cells)
    p = W.gray_2d(n=48, sn=4, block=4, seed=2)
    p.T0 = 0.3
    p.dt = 1.0
    return p


@pytest.mark.parametrize("dim", [2, 1])
def test_lo_solve_multigrid_matches_oracle(smrt_mod, oracle_mod, dim):
    p = _diffusive_2d() if dim == 2 else W.slab_1d(n_cells=300, n_angles=8, sigma=0.05)
    if dim == 1:
        p.dt = 10.0
        p.T0 = 0.3
    o, T, cl, E0 = _lo_case(oracle_mod, p)
    r, E_ref, F_ref, T_ref, ost = o.lo_solve(oracle_mod.default_opts(**TIGHT), p.dt, T, cl, E0, T)
    assert r == 0
    rows = np.vstack([cl["sigE"], cl["sigF"], cl["sigP"], cl["qE"], cl["qF"].T])
    res = {}
    for pc in (0, 1):
        ctx = smrt_mod.Context(p, precision=0, lo_precond=pc, **TIGHT)
        E, F, Tg, gst = ctx.lo_solve(rows, T, p.dt, E0, T)
        ctx.close()
        print(f"dim {dim} precond {pc}: cg {gst['cg_total']} newton {gst['inner_total']} "
              f"(oracle cg {ost['cg_total']} newton {ost['inner_total']})", flush=True)
        assert _rel(Tg, T_ref) < 1e-10
        assert _rel(E, E_ref) < 1e-10
        assert _rel(F, F_ref) < 1e-9
        res[pc] = gst
    assert res[1]["cg_total"] * 3 <= res[0]["cg_total"]


@pytest.mark.parametrize("scheme", [0, 1])
def test_steps_with_multigrid_match_oracle(smrt_mod, oracle_mod, scheme):
    p = _diffusive_2d()
    p.dt = 0.1
    o = oracle_mod.Oracle(p)
    st = o.initial_state()
    ctx = smrt_mod.Context(p, precision=0, scheme=scheme, lo_precond=1, **TIGHT)
    ctx.set_state(st["T"])
    for k in range(2):
        print(f"multigrid step {k} scheme {scheme}", flush=True)
        r, st, ost = o.step(st, oracle_mod.default_opts(scheme=scheme, **TIGHT))
        assert r == 0
        gst = ctx.step()
        got = ctx.get_state()
        assert _rel(got["T"], st["T"]) < 1e-10
        assert _rel(got["E"], st["E"]) < 1e-10
        assert abs(gst["outer"] - ost["outer"]) <= 1
    ctx.close()


def test_multigrid_graph_replay_matches_direct_launches(smrt_mod):
    p = _diffusive_2d()
    out = []
    for graphs in (1, 0):
        ctx = smrt_mod.Context(p, precision=0, lo_precond=1, lo_graphs=graphs)
        ctx.set_state(p.initial_T_nodes())
        st = ctx.step()
        out.append((ctx.get_state(with_psi=False)["T"], st["cg_total"]))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_full_size_step_multigrid_agrees_with_jacobi(smrt_mod):
    """The benchmark workload (256x256, S8, 16 groups) with a long time step:
    both preconditioners converge the same SM step (paper tolerances)."""
    p = W.multigroup_2d()
    p.dt = 0.05
    res = {}
    for pc in (0, 1):
        ctx = smrt_mod.Context(p, precision=smrt_mod.SMRT_FP32, lo_precond=pc, cg_rtol=1e-12, max_cg=2000,
                               eps_inner=1e-8, eps_outer=1e-6)
        ctx.set_state(p.initial_T_nodes())
        st = ctx.step()
        print(f"full size dt 0.05 precond {pc}: {st}", flush=True)
        res[pc] = (ctx.get_state(with_psi=False)["T"], st)
        ctx.close()
    assert _rel(res[1][0], res[0][0]) < 1e-6
    assert res[1][1]["cg_total"] < res[0][1]["cg_total"]
