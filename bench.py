#!/usr/bin/env python3
"""Throughput benchmark of the SM-TRT high-order path on one MI355X.

Workload: 2D 256x256 bilinear DG, level-symmetric S8 (40 angles), 16 groups
log-spaced on [1e-3, 10], power-law opacities with per-region coefficients
(synthetic, seeded), Planck emission at T0 = 0.01, left inflow at T = 1,
dt = 1e-3 -- the multigroup throughput configuration.

One bench step = one resident high-order pass: opacity table, emission and
gray-collapse tables, the FP32 sweep over all 640 (angle, group) pairs with
fused moments, the moment finalisation and the SM closure post-pass, with
every input already in HBM, on fixed inputs from a mid-run state (two FP64
time steps from the initial state).  value = swept cell*angle*group units
per second of that pass, the K timed passes queued back to back in one
library call (ms_per_step_host_wait_each_step: the same passes with a host
wait after each).  The JSON line also carries the sweep kernel's
HBM roofline (algorithmic bytes: read I* + write I; measured bytes from the
committed counters; the measured device-to-device copy rate as a practical
ceiling), the FP64 sweep for the FP32-vs-FP64 ratio and errors (one sweep
and one full step from the same state), the sweep with the negative-flux
fixup switched on (its cost), full time steps, the LO preconditioners
(Jacobi, multigrid) on a diffusion-dominated step, the sweep on
unstructured quadrilateral meshes, the batched and
adjoint workloads, and the FP64 CPU oracle timed on a bounded sample of the
same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LO_GRAPHS = 1   # --lo-graphs: 1 replays the LO conjugate-gradient blocks as HIP graphs (the library default)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep2d_fp32_256x256_S8_G16_hbm_bytes.md")
SWEEP_SOURCES = [os.path.join(ROOT, "paper_2504_21784_amd", "csrc", f)
                 for f in ("sweep2d.inc", "sweep2d_f32.hip", "smrt_internal.h")]


def measured_traffic(info):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the sweep source or the launch shape differs from the
    one those counters were taken on."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        h = hashlib.sha256(b"".join(open(f, "rb").read() for f in SWEEP_SOURCES)).hexdigest()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines()
                if l.startswith(("traffic_bytes_per_launch:", "source_sha256:", "launch:")))
    if vals.get("source_sha256", "").strip() != h:
        return None
    shape = (f"waves_per_band={info['waves_per_band']} bands_per_group={info['bands_per_group']} "
             f"pairs_per_lane={info['pairs_per_lane']}")
    if vals.get("launch", "").strip() != shape:
        return None
    return float(vals["traffic_bytes_per_launch"])


def sweep_kernel_name(info):
    """The FP32 sweep kernel instance a launch shape runs (its template
    arguments: pairs per lane, prefetch depth, waves per band, bands per
    workgroup, fixup, and whether a publisher and a receiver wave carry the
    outflow between stacked band groups), as the profiler names it."""
    k, nw, nb = info["pairs_per_lane"], info["waves_per_band"], info["bands_per_group"]
    n_bands = -(-info["ny"] // info["band_rows"])
    xw = n_bands > nb
    waves = nw * nb + (2 if xw else 0)
    if waves >= 16:
        prefetch = 3 if k == 1 else 1
    else:
        prefetch = {1: 4, 2: 3, 4: 1}[k]
    return f"sweep2d_kernel<float, {k}, {prefetch}, {nw}, {nb}, false, {str(xw).lower()}>"


def planck_group_fractions(nu_edges, T):
    """Fractions b_g(T) of a c T^4 in the groups [nu_g, nu_g+1) (the first from
    0, the last to infinity) for an array of temperatures, from the standard
    series for the Planck integral: below x = nu/T < 1 its Taylor series
    (Bernoulli coefficients), above it the exponential series.  Input preparation of the CPU baseline
    only (the oracle's own spectra integrate numerically)."""
    import numpy as np

    def below(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.empty_like(x)
        small = x < 1.0
        xs = x[small]
        # sum_n B_n x^(n+3) / (n! (n+3)) through x^17
        out[small] = (xs ** 3 / 3 - xs ** 4 / 8 + xs ** 5 / 60 - xs ** 7 / 5040 + xs ** 9 / 272160
                      - xs ** 11 / 13305600 + xs ** 13 / 622702080 - 691 * xs ** 15 / 19615115520000
                      + 7 * xs ** 17 / 8892185702400) * 15 / np.pi ** 4
        xl = x[~small]
        above = np.zeros_like(xl)
        for k in range(1, 60):
            above += np.exp(-k * xl) * (xl ** 3 / k + 3 * xl ** 2 / k ** 2 + 6 * xl / k ** 3 + 6 / k ** 4)
        out[~small] = 1.0 - above * 15 / np.pi ** 4
        return out

    nu = np.asarray(nu_edges, dtype=np.float64)
    G = len(nu) - 1
    Fb = np.stack([below(nu[g] / T) if g > 0 else np.zeros_like(T) for g in range(G)] + [np.ones_like(T)], axis=1)
    return np.diff(Fb, axis=1)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, mid, reps=5):
    """The FP64 oracle's sweep + moments on the inputs of the timed GPU sweep
    (the mid-run state: opacities from its T, emission source sigma a c T^4
    b_g(T) / 4 pi, its intensity as the time-edge source, the boundary
    inflow), median of `reps` sweeps: all 16 groups on every host thread the
    oracle's OpenMP sweep uses, and group 1 alone on one thread."""
    import copy
    import numpy as np
    import oracle

    T, psi = mid["T"], mid["psi"]
    full = oracle.Oracle(p)
    sig = full.opacity(T)
    sigt = sig + 1.0 / (p.c * p.dt)
    b = planck_group_fractions(p.nu_edges, T)
    q = sig[np.arange(p.n_nodes) // 4] * (p.a * p.c * T ** 4 / (4 * np.pi))[:, None] * b
    inflow = full.inflow()
    icdt = 1.0 / (p.c * p.dt)

    def run(G, threads):
        n_thr = oracle.set_threads(threads)
        sub = copy.copy(p)
        sub.G = G
        sub.nu_edges = p.nu_edges[:G + 1]
        o = oracle.Oracle(sub) if G != p.G else full
        args = [np.ascontiguousarray(a) for a in (sigt[:, :G], q[:, :G], psi[:, :G, :], inflow[:, :G, :])]
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = o.sweep(args[0], args[1], args[2], icdt, args[3])
            o.moments(np.ascontiguousarray(sig[:, :G]), out)
            ts.append(time.perf_counter() - t0)
        units = p.n_cells * p.n_angles * G
        return units / float(np.median(ts)), n_thr, float(np.median(ts)), units

    v_all, n_all, t_all, u_all = run(p.G, 0)
    v_one, _, t_one, u_one = run(1, 1)
    oracle.set_threads(0)
    return {"value": v_all, "unit": "units/s", "cores": n_all, "kind": "oracle",
            "sample": f"mid-run 256x256 S8 G16 inputs: FP64 sweep + moments of all {u_all / 1e6:.1f} M units on "
                      f"{n_all} threads (OpenMP over (angle, group) pairs), median of {reps}: {t_all:.2f} s",
            "one_thread": {"value": v_one, "unit": "units/s", "cores": 1,
                           "sample": f"group 1 only ({u_one / 1e6:.2f} M units), 1 thread, median of {reps}: "
                                     f"{t_one:.2f} s"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def c3_oracle_errors():
    """One step of the 256x256 S8 G16 workload from its initial state, FP32
    sweep + FP64 low order and all-FP64, both iterated to the tight
    tolerances of the stored FP64 oracle step (tests/golden/c3_step1_oracle.npz,
    written by tests/golden/make_c3_step.py): relative L2 and pointwise
    (floor 1e-12 of the max) errors of phi, T and E at its 4096 stored
    nodes, and the relative error of the total energy."""
    import numpy as np
    from paper_2504_21784_amd import smrt, workloads as W

    path = os.path.join(ROOT, "tests", "golden", "c3_step1_oracle.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    opts = {str(k): float(v) for k, v in zip(g["opt_names"], g["opts"])}
    for k in ("max_outer", "max_inner", "max_cg"):
        opts[k] = int(opts[k])
    p = W.multigroup_2d()
    hx, hy = np.diff(p.x_edges), np.diff(p.y_edges)
    V = np.repeat((hx[None, :] * hy[:, None]).ravel() / 4.0, 4)
    cv = np.repeat(np.asarray(p.cv)[np.asarray(p.region_of_cell)], 4)
    res = {"workload": "one step of multigroup_2d (256x256 S8 G16) from its initial state, outer 1e-11, "
                       "inner 1e-12, CG 1e-13; errors at 4096 sampled nodes against the stored FP64 oracle step",
           "oracle_outer": int(g["outer"])}
    for name, prec in (("fp32_sweep", smrt.SMRT_FP32), ("fp64", smrt.SMRT_FP64)):
        ctx = smrt.Context(p, precision=prec, lo_graphs=LO_GRAPHS, **opts)
        ctx.set_state(p.initial_T_nodes())
        st = ctx.step()
        s = ctx.get_state()
        ctx.close()
        phi = np.einsum("d,dgn->n", p.w, s["psi"])
        e = {"outer": int(st["outer"])}
        for f, field in (("phi", phi), ("T", s["T"]), ("E", s["E"])):
            ref, got = g[f], field[g["nodes"]]
            e[f + "_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            e[f + "_pointwise"] = float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-12 * float(g[f + "_max"]))).max())
        energy = float(np.sum(V * (s["E"] + cv * s["T"])))
        e["energy_rel"] = abs(energy - float(g["energy"])) / abs(float(g["energy"]))
        res[name] = e
    return res


def batched(args):
    """The uneven batch: 32 problems (seed 5: n in {64..384}, G in {4..32},
    S4/S8/S12), FP32, every sweep task in one launch with the autotuned launch
    shape; the resident pass of all problems is replayed as a HIP graph."""
    import time as _t
    from paper_2504_21784_amd import smrt, workloads as W

    t0 = _t.perf_counter()
    ps = W.batch_2d()
    ctxs = []
    for q in ps:
        c = smrt.Context(q, precision=smrt.SMRT_FP32, lo_graphs=LO_GRAPHS)
        c.set_state(q.initial_T_nodes())
        ctxs.append(c)
    b = smrt.Batch(ctxs)
    setup_s = _t.perf_counter() - t0
    dt = ps[0].dt
    nw, nb, k, tune_ms = b.autotune(dt)
    info = b.info()
    b.sweep_resident(dt, n_times=1, capture_graph=False)
    ms, ks = b.sweep_resident(dt, n_times=max(3, args.steps // 4), capture_graph=True)
    units = info["units_per_sweep"]
    alg = 32.0 * units
    res = {"workload": "32 independent 2D problems (seed 5): n in {64,...,384}, G in {4,8,16,32}, "
                       "level-symmetric S4/S8/S12, power-law region opacities (seed 5000+i), dt=1e-3, FP32",
           "units_per_sweep": units, "n_tasks": info["n_tasks"],
           "launch": {"waves_per_band": nw, "bands_per_group": nb, "pairs_per_lane": k}, "autotuned_sweep_ms": tune_ms,
           "sweep_ms": ks, "sweep_units_per_s": units / (ks * 1e-3),
           "sweep_hbm_frac": alg / (ks * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "graph_pass_ms": ms, "graph_pass_units_per_s": units / (ms * 1e-3), "setup_s": setup_s}
    # five backward-Euler steps of every problem (FP32 sweep, FP64 LO), from
    # the initial states: the host-driven lock-stepped step, then the run with
    # device-side convergence control replayed from one captured HIP graph
    n_steps = 5
    pu = [q.nx * q.ny * q.n_angles * q.G for q in ps]

    def swept(stats):
        return sum(st[i]["outer"] * pu[i] for st in stats for i in range(len(ps)))

    for c, q in zip(ctxs, ps):
        c.set_state(q.initial_T_nodes())
    t0 = _t.perf_counter()
    host = [b.step(dt) for _ in range(n_steps)]
    t_host = _t.perf_counter() - t0
    for c, q in zip(ctxs, ps):
        c.set_state(q.initial_T_nodes())
    t0 = _t.perf_counter()
    dev = b.run(n_steps, dt, capture_graph=True)
    t_dev = _t.perf_counter() - t0
    res["five_steps"] = {
        "workload": "5 steps of every problem from its initial state, dt=1e-3, consistent SM, eps 1e-3, FP32 sweep + "
                    "FP64 LO (Jacobi CG)",
        "device_control": {"wall_s": t_dev, "ms_per_step": t_dev / n_steps * 1e3,
                           "swept_units_per_s": swept(dev) / t_dev,
                           "outer_per_step": [max(st[i]["outer"] for i in range(len(ps))) for st in dev],
                           "outer_total": sum(st[i]["outer"] for st in dev for i in range(len(ps))),
                           "cg_total": sum(st[i]["cg_total"] for st in dev for i in range(len(ps)))},
        "host_lockstep": {"wall_s": t_host, "ms_per_step": t_host / n_steps * 1e3,
                          "swept_units_per_s": swept(host) / t_host,
                          "outer_total": sum(st[i]["outer"] for st in host for i in range(len(ps)))},
        "speedup": t_host / t_dev}
    b.close()
    for c in ctxs:
        c.close()
    return res


def time_steps(p, T0, n=3):
    """Full backward-Euler steps (Algorithm 1: consistent SM, FP32 sweep, FP64
    LO, the paper's tolerances 1e-3) on the benchmark workload: wall time per
    step and the iteration counts."""
    import time as _t
    import numpy as np
    from paper_2504_21784_amd import smrt

    ctx = smrt.Context(p, precision=smrt.SMRT_FP32, lo_graphs=LO_GRAPHS)
    ctx.set_state(T0)
    ctx.step(p.dt)   # warm-up step
    t0 = _t.perf_counter()
    stats = [ctx.step(p.dt) for _ in range(n)]
    wall = (_t.perf_counter() - t0) / n
    ctx.close()
    return {"workload": "same 256x256 S8 G16 workload, consistent SM, FP32 sweep + FP64 LO, eps 1e-3",
            "ms_per_step": 1e3 * wall,
            "outer_per_step": float(np.mean([s["outer"] for s in stats])),
            "inner_per_step": float(np.mean([s["inner_total"] for s in stats])),
            "cg_per_step": float(np.mean([s["cg_total"] for s in stats])),
            "sweep_ms_per_step": float(np.mean([s["t_sweep_ms"] for s in stats]))}


def lo_multigrid():
    """The LO preconditioners on a diffusion-dominated step: gray 256x256,
    level-symmetric S8, per-8x8-block opacity log-uniform [0.1, 1000] (seed 2),
    T0 = 0.3, dt = 1 (cells thin enough that the diffusion term outweighs the
    diagonal), consistent SM with the fixup and the floor, FP32 sweep, CG to
    1e-12.  One warm-up step (it includes the one-time multigrid set-up), then
    the second step timed, with Jacobi and with the multigrid V-cycle."""
    import time as _t
    from paper_2504_21784_amd import smrt, workloads as W

    p = W.gray_2d(n=256, sn=8, block=8, seed=2)
    p.dt = 1.0
    p.T0 = 0.3
    out = {"workload": "gray 256x256, S8, sigma per 8x8 block log-uniform [0.1, 1000] (seed 2), T0 = 0.3, dt = 1, "
                       "fixup + floor, FP32 sweep, CG rtol 1e-12, outer/inner 1e-6/1e-8; second step timed"}
    for pc, name in ((0, "jacobi"), (1, "multigrid")):
        ctx = smrt.Context(p, precision=smrt.SMRT_FP32, lo_precond=pc, lo_graphs=LO_GRAPHS, cg_rtol=1e-12, max_cg=4000,
                           eps_inner=1e-8, eps_outer=1e-6, fixup=1, T_floor=1e-6)
        ctx.set_state(p.initial_T_nodes())
        ctx.step()
        t0 = _t.perf_counter()
        st = ctx.step()
        wall = _t.perf_counter() - t0
        ctx.close()
        out[name] = {"ms_per_step": 1e3 * wall, "lo_ms": st["t_lo_ms"], "outer": st["outer"],
                     "newton": st["inner_total"], "cg": st["cg_total"],
                     "us_per_cg_iteration": 1e3 * st["t_lo_ms"] / max(st["cg_total"], 1)}
    out["step_speedup"] = out["jacobi"]["ms_per_step"] / out["multigrid"]["ms_per_step"]
    return out


def qmesh_sweep():
    """The sweep on unstructured quadrilateral meshes (dependency levels per
    direction), S8, 16 groups, FP32, sigma_t log-uniform [0.1, 100], no
    time-edge source: the 256x256 mesh given as quadrilaterals (the
    rectilinear kernel's workload) and an unstructured mesh of 64,896 cells
    (104x104 squares, jittered, each cut into two triangles and each triangle
    into three quadrilaterals; seed 2).  Second sweep timed, then the gray
    moments of its intensity (a separate kernel on this path)."""
    import numpy as np
    from paper_2504_21784_amd import smrt, workloads as W

    out = {}
    om, w = W.level_symmetric_2d(8)
    G = 16
    for name, (xy, cells) in (("rectilinear_256x256_as_quads", W.quad_mesh_jittered(256, 256, jitter=0.0)),
                              ("unstructured_64896_cells", W.quad_mesh_split_triangles(104, seed=2))):
        m = smrt.QuadMeshSweep(xy, cells, om, w, G, precision=smrt.SMRT_FP32)
        rng = np.random.default_rng(1)
        nc = len(cells)
        sigt = 10.0 ** rng.uniform(-1, 2, (nc, G))
        q = rng.uniform(0, 1, (4 * nc, G))
        m.sweep(sigt, q, None, 0.0)
        _, ms = m.sweep(sigt, q, None, 0.0)
        _, ms_mom = m.moments(0.5 * sigt)
        units = nc * len(w) * G
        out[name] = {"cells": nc, "levels": m.n_levels, "sweep_ms": ms, "units_per_s": units / (ms * 1e-3),
                     "moments_ms": ms_mom}
        m.close()
    out["unaccelerated_step"] = qmesh_step()
    return out


def qmesh_step():
    """The unaccelerated time step on the 64,896-cell unstructured mesh (S8,
    16 groups, FP32): 4 regions (cell index mod 4) with tabulated opacities
    log-uniform in [0.1, 100] per (region, group) (seed 3), c_v = 1, group
    bounds logspace(-2, 1.5), T0 = 0.5 with its equilibrium intensity,
    vacuum sides, dt = 1e-3.  Each step runs a fixed 5 outer iterations
    (emission, sweep, gray moments, energy balance, outer test), so the time
    per outer iteration is the path's cost; the second step is timed."""
    import numpy as np
    from paper_2504_21784_amd import smrt, workloads as W

    xy, cells = W.quad_mesh_split_triangles(104, seed=2)
    om, w = W.level_symmetric_2d(8)
    G, nc, n_outer = 16, len(cells), 5
    rng = np.random.default_rng(3)
    s0 = 10.0 ** rng.uniform(-1, 2, (4, G))
    m = smrt.QuadMeshSweep(xy, cells, om, w, G, precision=smrt.SMRT_FP32)
    m.set_materials((np.arange(nc) % 4).astype(np.int32), s0, np.ones(4), np.logspace(-2, 1.5, G + 1), model=0)
    m.set_state(np.full(4 * nc, 0.5))
    m.step(1e-3, fixed_outer=n_outer)
    st = m.step(1e-3, fixed_outer=n_outer)
    m.close()
    ms = st["t_total_ms"]
    return {"cells": nc, "outer": st["outer"], "ms_per_step": ms, "ms_per_outer": ms / max(st["outer"], 1),
            "sweep_units_per_s": st["outer"] * nc * len(w) * G / (ms * 1e-3)}


def adjoint():
    """Adjoint workload: 128x128, S8, 8 groups, 64 regions (seed 4), 10 steps of
    dt = 1e-3, FP64: time of the gradient of the time-integrated x+ outflow
    with respect to the 128 region parameters (forward with checkpoints +
    reverse), and its agreement with central finite differences (h = 1e-4)
    on the two largest components of each kind."""
    import time as _t
    import numpy as np
    from paper_2504_21784_amd import smrt, workloads as W

    p = W.adjoint_2d()
    tight = dict(eps_outer=1e-10, eps_inner=1e-11, cg_rtol=1e-13, elim_rtol=1e-15, max_outer=200, max_inner=60,
                 max_cg=500, max_elim=100)
    ctx = smrt.Context(p, precision=smrt.SMRT_FP64, lo_graphs=LO_GRAPHS, **tight)
    T0 = p.initial_T_nodes()
    ctx.set_state(T0)
    t0 = _t.perf_counter()
    J, gs, gc, its = ctx.adjoint(p.n_steps)
    t_adj = _t.perf_counter() - t0

    def J_at(s0, cv):
        ctx.set_materials(s0, cv)
        ctx.set_state(T0)
        return ctx.adjoint(p.n_steps)[0]

    h = 1e-4
    errs = []
    for g, which in ((gs, 0), (gc, 1)):
        for r in np.argsort(-np.abs(g))[:2]:
            e = np.zeros(p.n_regions)
            e[r] = h
            args_p = (p.sigma0 * np.exp(e), p.cv) if which == 0 else (p.sigma0, p.cv * np.exp(e))
            args_m = (p.sigma0 * np.exp(-e), p.cv) if which == 0 else (p.sigma0, p.cv * np.exp(-e))
            fd = (J_at(*args_p) - J_at(*args_m)) / (2 * h)
            errs.append(abs(g[r] - fd) / max(abs(fd), 1e-300))
    ctx.close()
    return {"workload": "128x128 bilinear DG, S8, 8 groups, 64 regions of sigma0 and c_v (seed 4), 10 steps "
                        "dt=1e-3, FP64; J = time-integrated x+ outflow",
            "J": J, "n_parameters": 2 * p.n_regions, "adjoint_iterations": its, "gradient_s": t_adj,
            "fd_max_rel_err_top4": max(errs), "fd_h": h}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--waves", type=int, default=0, help="sweep waves per band (0 = automatic)")
    ap.add_argument("--bands", type=int, default=0, help="sweep bands per workgroup (0 = automatic)")
    ap.add_argument("--pairs", type=int, default=0, help="(angle,group) pairs per lane (0 = automatic)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 32-problem batched-sweep measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-gradient measurement")
    ap.add_argument("--no-step", action="store_true", help="skip the full time-step measurement")
    ap.add_argument("--no-multigrid", action="store_true", help="skip the LO preconditioner comparison")
    ap.add_argument("--no-qmesh", action="store_true", help="skip the unstructured-mesh sweep")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the full-size step against the stored oracle step")
    ap.add_argument("--lo-graphs", type=int, default=1, choices=(0, 1),
                    help="0: launch the LO conjugate-gradient kernels directly instead of replaying graphs")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (reference point for HBM byte counters)")
    args = ap.parse_args()
    global LO_GRAPHS
    LO_GRAPHS = args.lo_graphs
    if args.gpus != 1:
        print("bench.py measures one MI355X: the library runs on a single GPU (sharding the sweep "
              "over several GPUs is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_21784_amd import smrt, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    p = W.multigroup_2d()
    T0 = p.initial_T_nodes()

    def make(prec, T=T0, psi=None):
        ctx = smrt.Context(p, precision=prec, stream=stream, lo_graphs=LO_GRAPHS)
        if args.waves or args.bands or args.pairs:
            ctx.set_launch(args.waves, args.bands, args.pairs if prec == smrt.SMRT_FP32 else min(args.pairs, 2))
        ctx.set_state(T, psi)
        return ctx

    # a mid-run state (two FP64 steps from the initial state): the fixed inputs
    # of the timed passes and of the FP32-vs-FP64 comparisons
    c = make(smrt.SMRT_FP64)
    for _ in range(2):
        c.step()
    mid = c.get_state()
    c.close()

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = make(smrt.SMRT_FP32, mid["T"], mid["psi"])
    info = ctx.info()
    units = info["units_per_sweep"]
    for _ in range(args.warmup):
        ctx.sweep_resident(n_times=1)
    torch.cuda.synchronize()
    # the K passes are queued back to back in one call (one host wait at the
    # end), as a run that keeps its iteration control on the device issues them
    t0 = time.perf_counter()
    _, k_ms = ctx.sweep_resident(n_times=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    # the same passes with a host wait after each one (one call per pass)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.sweep_resident(n_times=1)
    torch.cuda.synchronize()
    ms_per_step_host_wait = 1e3 * (time.perf_counter() - t0) / args.steps
    mom32 = ctx.get_moments()
    ctx.step()                                  # one full FP32 step from the mid-run state
    step32 = (ctx.get_moments(), ctx.get_state(with_psi=False)["T"])
    alg_bytes = info["algorithmic_bytes_per_sweep"]
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    sweep_kernel = sweep_kernel_name(info)
    ctx.close()

    # the same sweep with the zero-and-scale negative-flux fixup compiled in
    # (same inputs, same launch): the cost of the fixup
    cf = make(smrt.SMRT_FP32, mid["T"], mid["psi"])
    cf.set_options(fixup=1)
    cf.sweep_resident(n_times=1)
    _, k_fix = cf.sweep_resident(n_times=max(3, args.steps // 4))
    cf.close()

    # FP64 sweep on the same inputs: throughput ratio and FP32 error
    c64 = make(smrt.SMRT_FP64, mid["T"], mid["psi"])
    c64.sweep_resident(n_times=1)
    _, k64 = c64.sweep_resident(n_times=max(3, args.steps // 4))
    mom64 = c64.get_moments()
    c64.step()
    step64 = (c64.get_moments(), c64.get_state(with_psi=False)["T"])
    c64.close()
    if args.no_cpu_baseline:
        del mid   # the CPU baseline sweeps the same mid-run inputs

    def rel_l2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def phi(m):
        return sum(m[6 * q] for q in range(4))

    phi_err = rel_l2(phi(mom32), phi(mom64))
    step_err = {"phi_rel_l2": rel_l2(phi(step32[0]), phi(step64[0])), "T_rel_l2": rel_l2(step32[1], step64[1])}

    # measured device-to-device copy rate (read + write bytes), the practical
    # ceiling for mixed traffic, timed with events on torch's stream
    nc = (1 << 30) // 4
    a = torch.ones(nc, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rates = []
    for _ in range(5):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        rates.append(2.0 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    copy_gbs = float(np.median(rates))
    del a, b
    traffic = measured_traffic(info)

    out = {
        "metric": "swept cell*angle*group unknowns/s (FP32 sweep with fused moments and closures, 1 GPU)",
        "value": units / (ms_per_step * 1e-3),
        "unit": "units/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "multigroup_2d: 256x256 bilinear DG, level-symmetric S8 (40 angles), 16 groups, "
                               "power-law region opacities (seed 3), dt=1e-3; step = opacity + sources + FP32 sweep "
                               "with fused moments + moment finalisation + SM closures",
                   "units_per_sweep": units, "launch": {k: info[k] for k in ("band_rows", "waves_per_band", "bands_per_group",
                                                                             "pairs_per_lane", "pairs_per_chunk",
                                                                             "n_chunks", "n_workgroups")}},
        "ms_per_step_host_wait_each_step": ms_per_step_host_wait,
        "sweep_kernel_ms": k_ms,
        "sweep_units_per_s": units / (k_ms * 1e-3),
        "fp64_sweep_kernel_ms": k64,
        "fp64_sweep_units_per_s": units / (k64 * 1e-3),
        # the FP64 sweep moves twice the bytes per unit (64 B: read I*, write I)
        "fp64_sweep_hbm_frac": 2 * alg_bytes / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "fp32_vs_fp64_sweep_speedup": k64 / k_ms,
        "fixup_sweep_kernel_ms": k_fix,
        "fixup_sweep_cost": k_fix / k_ms - 1.0,
        "fp32_phi_rel_l2_vs_fp64": phi_err,
        "fp32_step_vs_fp64_step": step_err,
        "inputs": "mid-run state: two FP64 steps from the initial state",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": sweep_kernel,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "device_copy_GBs": copy_gbs, "frac_of_device_copy": achieved / copy_gbs,
                     "traffic_GBs": (traffic / (k_ms * 1e-3) / 1e9) if traffic else None},
    }
    if not args.no_step:
        out["time_step"] = time_steps(p, T0)
    if not args.no_oracle_error:
        out["error_vs_oracle_c3_step"] = c3_oracle_errors()
    if not args.no_batch:
        out["batched"] = batched(args)
    if not args.no_adjoint:
        out["adjoint"] = adjoint()
    if not args.no_multigrid:
        out["lo_multigrid"] = lo_multigrid()
    if not args.no_qmesh:
        out["qmesh_sweep"] = qmesh_sweep()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, mid)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
