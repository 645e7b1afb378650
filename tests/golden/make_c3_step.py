"""Writes c3_step1_oracle.npz: one backward-Euler SM step of the FP64 oracle
on the 256x256, S8, 16-group multigroup workload (power-law region
opacities, seed 3; T0 = 0.01, left inflow at T = 1, dt = 1e-3) from its
initial equilibrium state, iterated to tight tolerances (outer 1e-11, inner
1e-12, CG 1e-13, elimination 1e-15) so that the result is the discrete
step's fixed point, not an iteration-count artefact.

Stored: the scalar flux phi = sum_d w_d sum_g I, T and E at 4096 nodes drawn
with seed 77, the same fields' global L2 norms, sums and maxima, the total
energy sum_n V_n (E_n + c_v T_n) (V_n = cell area / 4), the oracle's
iteration statistics, the options, and the SHA-256 of the oracle source.
It calls only oracle/ (the GPU library is not involved).  Run from the
repository root: python tests/golden/make_c3_step.py
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from paper_2504_21784_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_step1_oracle.npz")
OPTS = dict(eps_outer=1e-11, eps_inner=1e-12, cg_rtol=1e-13, elim_rtol=1e-15, max_outer=200, max_inner=60,
            max_cg=3000)
N_SAMPLE, SAMPLE_SEED = 4096, 77


def node_volumes(p):
    hx, hy = np.diff(p.x_edges), np.diff(p.y_edges)
    area = (hx[None, :] * hy[:, None]).ravel()          # cell c = i + nx j
    return np.repeat(area / 4.0, 4)


def cv_nodes(p):
    return np.repeat(np.asarray(p.cv)[np.asarray(p.region_of_cell)], 4)


def main():
    p = W.multigroup_2d()
    assert (p.nx, p.ny, p.n_angles, p.G) == (256, 256, 40, 16)
    src_hash = hashlib.sha256(open(os.path.join(ROOT, "oracle", "oracle.c"), "rb").read()).hexdigest()
    o = oracle.Oracle(p)
    st = o.initial_state()
    t0 = time.time()
    r, s, stats = o.step(st, oracle.default_opts(**OPTS))
    assert r == 0, r
    phi = np.einsum("d,dgn->n", p.w, s["psi"])
    V, cv = node_volumes(p), cv_nodes(p)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(p.n_nodes, N_SAMPLE, replace=False))
    np.savez_compressed(
        OUT, nodes=idx, phi=phi[idx], T=s["T"][idx], E=s["E"][idx],
        phi_norm=np.linalg.norm(phi), T_norm=np.linalg.norm(s["T"]), E_norm=np.linalg.norm(s["E"]),
        phi_max=np.abs(phi).max(), T_max=np.abs(s["T"]).max(), E_max=np.abs(s["E"]).max(),
        phi_sum=phi.sum(), T_sum=s["T"].sum(), E_sum=s["E"].sum(),
        energy=np.sum(V * (s["E"] + cv * s["T"])),
        outer=stats["outer"], inner_total=stats["inner_total"], cg_total=stats["cg_total"],
        opts=np.array([OPTS[k] for k in sorted(OPTS)], dtype=np.float64), opt_names=np.array(sorted(OPTS)),
        oracle_sha256=np.array(src_hash), workload=np.array("multigroup_2d(): 256x256 S8 G16 seed 3, dt 1e-3"))
    print(f"wrote {OUT}: {stats['outer']} outer iterations, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
