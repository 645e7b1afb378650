"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module produces *data only*: angular quadratures, rectilinear meshes,
group bounds, per-region material tables, boundary descriptions and the
initial state of each workload.  It contains none of the transport, moment,
closure or low-order arithmetic of the method, so that the CPU oracle and
the GPU library can both be fed identical arrays without sharing any of
their numerics.

Every random array comes from numpy's PCG64 with an explicit seed.
"log-uniform [lo, hi]" means 10**U(log10 lo, log10 hi).  Units are
normalised (a = c = 1) and frequency and temperature share one unit,
as in the paper's convention that h*nu -> nu and k*T -> T (Sec. 2).

Workloads (the paper's own geometries and opacity data are not
available, so these are synthetic stand-ins with the shapes of its
benchmarks: block-structured materials, 1-33 groups, 8-84 angles):
  * ``slab_1d``      -- 1D slab, 64 cells, Gauss-Legendre S8, gray
                        (Marshak-like: cold slab heated from the left).
  * ``gray_2d``      -- 2D 128x128, level-symmetric S8, gray, block
                        opacities log-uniform on [0.1, 1000].
  * ``multigroup_2d``-- 2D 256x256, S8, 16 groups, power-law opacities
                        with per-region coefficients (lattice-like).
  * ``adjoint_2d``   -- 2D 128x128, S8, 8 groups, 64 regions with
                        per-region opacity and heat-capacity parameters.
  * ``batch_2d``     -- 32 independent 2D problems of uneven size.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FOUR_PI = 4.0 * math.pi

# ----------------------------------------------------------------------------
# Angular quadratures (input data)
# ----------------------------------------------------------------------------


def gauss_legendre_slab(n: int):
    """1D slab S_N: Gauss-Legendre cosines, weights scaled by 2*pi.

    Returns (omega[n,3], w[n]) with sum(w) = 4*pi.  Only omega[:,0] (mu) is
    used in slab geometry.
    """
    mu, wgl = np.polynomial.legendre.leggauss(n)
    omega = np.zeros((n, 3))
    omega[:, 0] = mu
    return omega, wgl * 2.0 * math.pi


# Level-symmetric first cosines (standard LQ_n values).  With the level
# rule below, the m = 1 moment condition holds by symmetry for any mu1, and
# the remaining even-moment conditions determine one weight per permutation
# class (S4: 1, S8: 3, S12: 5 classes).
_LS_MU1 = {4: 0.3500212, 6: 0.2666355, 8: 0.2182179, 12: 0.1672126}


def _ls_octant(N: int):
    """Octant points (mu, eta, xi) and weights (summing to 1) of the LQ_N set."""
    mu1 = _LS_MU1[N]
    half = N // 2
    levels = np.sqrt(np.array([mu1 ** 2 + i * 2.0 * (1.0 - 3.0 * mu1 ** 2) / (N - 2)
                               for i in range(half)]))
    pts = [(i, j, half + 2 - i - j) for i in range(1, half + 1) for j in range(1, half + 1)
           if 1 <= half + 2 - i - j <= half]
    classes = sorted({tuple(sorted(p)) for p in pts})
    cls_of = [classes.index(tuple(sorted(p))) for p in pts]
    A = np.zeros((half, len(classes)))
    for p, c in zip(pts, cls_of):
        for m in range(half):
            A[m, c] += levels[p[0] - 1] ** (2 * m)
    b = np.array([1.0 / (2 * m + 1) for m in range(half)])
    w = np.linalg.lstsq(A, b, rcond=None)[0]
    wp = np.array([w[c] for c in cls_of])
    mus = np.array([[levels[p[0] - 1], levels[p[1] - 1], levels[p[2] - 1]] for p in pts])
    return mus, wp / wp.sum()


def level_symmetric_2d(N: int):
    """2D level-symmetric S_N set (ξ > 0 half of the sphere).

    Returns (omega[n,3], w[n]); n = N(N+2)/2 (12, 40, 84 for S4, S8, S12),
    sum(w) = 4*pi.  Directions are ordered by quadrant
    (mu>0,eta>0), (mu<0,eta>0), (mu<0,eta<0), (mu>0,eta<0).
    """
    mus, wo = _ls_octant(N)
    om, ww = [], []
    for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        for (m, e, x), wt in zip(mus, wo):
            om.append((sx * m, sy * e, x))
            ww.append(wt * math.pi)
    return np.array(om), np.array(ww)


# ----------------------------------------------------------------------------
# Problem description
# ----------------------------------------------------------------------------

BC_VACUUM, BC_PLANCK, BC_EXPLICIT, BC_REFLECT = 0, 1, 2, 3
MODEL_CONST, MODEL_POWERLAW = 0, 1


@dataclasses.dataclass
class Problem:
    name: str
    dim: int
    nx: int
    ny: int
    x_edges: np.ndarray
    y_edges: Optional[np.ndarray]
    omega: np.ndarray          # [n_angles, 3]
    w: np.ndarray              # [n_angles], sums to 4*pi
    G: int
    nu_edges: np.ndarray       # [G+1] stated group bounds
    a: float
    c: float
    region_of_cell: np.ndarray  # int32 [n_cells]
    model: int
    sigma0: np.ndarray         # [n_regions][G] (const) or [n_regions] (power law)
    clip_lo: float
    clip_hi: float
    cv: np.ndarray             # [n_regions]
    bc_kind: List[int]         # per side: 1D (x-, x+); 2D (x-, x+, y-, y+)
    T_bdr: List[float]
    inflow_g: List[Optional[np.ndarray]]
    T0: float
    dt: float
    n_steps: int
    seed: Optional[int] = None

    @property
    def n_cells(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def nodes_per_cell(self) -> int:
        return 2 ** self.dim

    @property
    def n_nodes(self) -> int:
        return self.n_cells * self.nodes_per_cell

    @property
    def n_angles(self) -> int:
        return self.omega.shape[0]

    @property
    def units_per_sweep(self) -> int:
        return self.n_cells * self.n_angles * self.G

    @property
    def n_regions(self) -> int:
        return int(self.cv.shape[0])

    def initial_T_nodes(self) -> np.ndarray:
        return np.full(self.n_nodes, self.T0)


def _log_uniform(rng, lo, hi, size):
    return 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size)


def _block_regions(nx, ny, bs):
    i = np.arange(nx)[None, :] // bs
    j = np.arange(ny)[:, None] // bs
    nbx = (nx + bs - 1) // bs
    return (i + nbx * j).reshape(-1).astype(np.int32), nbx * ((ny + bs - 1) // bs)


def slab_1d(n_cells: int = 64, n_angles: int = 8, sigma: float = 10.0, n_steps: int = 10) -> Problem:
    """1D gray slab on [0,1]: sigma=10, c_v=1, T0=0.01, left inflow at T=1, right vacuum."""
    om, w = gauss_legendre_slab(n_angles)
    return Problem(
        name=f"slab_1d_{n_cells}", dim=1, nx=n_cells, ny=1,
        x_edges=np.linspace(0.0, 1.0, n_cells + 1), y_edges=None,
        omega=om, w=w, G=1, nu_edges=np.array([1e-3, 10.0]), a=1.0, c=1.0,
        region_of_cell=np.zeros(n_cells, np.int32), model=MODEL_CONST,
        sigma0=np.array([[sigma]]), clip_lo=0.0, clip_hi=1e300, cv=np.array([1.0]),
        bc_kind=[BC_PLANCK, BC_VACUUM], T_bdr=[1.0, 0.0], inflow_g=[None, None],
        T0=0.01, dt=0.01, n_steps=n_steps)


# Physical constants of the Marshak wave (T in eV, lengths in cm, time in s):
# the radiation constant 7.5657e-15 erg cm^-3 K^-4 with 1 eV = 11604.518 K.
RAD_CONST_EV = 7.5657e-15 * 11604.518 ** 4      # 137.20 erg cm^-3 eV^-4
LIGHT_SPEED_CM_S = 2.99792458e10


def marshak_1d(n_cells: int = 128, dt_ns: float = 8e-3, t_end_ns: float = 2.5) -> Problem:
    """Marshak wave (Sec. 6): gray slab [0, 0.05] cm, sigma(T) = 1e12/T^3 per cm
    (T in eV), c_v = 3e12 erg/(cm^3 eV), initial equilibrium at 1 eV, a 1 keV
    Planck source on the left, Gauss-Legendre S6.  The paper leaves the right
    boundary and c unstated: vacuum and c = 2.99792458e10 cm/s.  The power law
    is the library's model 1 with one group whose bounds have geometric mean
    1, so sigma = sigma0/T^3 with sigma0 = 1e12 (no clipping)."""
    om, w = gauss_legendre_slab(6)
    dt = dt_ns * 1e-9
    return Problem(
        name=f"marshak_1d_{n_cells}", dim=1, nx=n_cells, ny=1,
        x_edges=np.linspace(0.0, 0.05, n_cells + 1), y_edges=None,
        omega=om, w=w, G=1, nu_edges=np.array([0.5, 2.0]), a=RAD_CONST_EV, c=LIGHT_SPEED_CM_S,
        region_of_cell=np.zeros(n_cells, np.int32), model=MODEL_POWERLAW,
        sigma0=np.array([1e12]), clip_lo=0.0, clip_hi=1e300, cv=np.array([3e12]),
        bc_kind=[BC_PLANCK, BC_VACUUM], T_bdr=[1000.0, 0.0], inflow_g=[None, None],
        T0=1.0, dt=dt, n_steps=int(round(t_end_ns / dt_ns)))


def gray_2d(n: int = 128, sn: int = 8, block: int = 8, seed: int = 2, n_steps: int = 20) -> Problem:
    """2D gray [0,1]^2 with per-block opacity log-uniform on [0.1, 1000]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    om, w = level_symmetric_2d(sn)
    reg, nreg = _block_regions(n, n, block)
    sig = _log_uniform(rng, 0.1, 1000.0, nreg).reshape(nreg, 1)
    return Problem(
        name=f"gray_2d_{n}", dim=2, nx=n, ny=n,
        x_edges=np.linspace(0.0, 1.0, n + 1), y_edges=np.linspace(0.0, 1.0, n + 1),
        omega=om, w=w, G=1, nu_edges=np.array([1e-3, 10.0]), a=1.0, c=1.0,
        region_of_cell=reg, model=MODEL_CONST, sigma0=sig, clip_lo=0.0, clip_hi=1e300,
        cv=np.ones(nreg), bc_kind=[BC_PLANCK, BC_VACUUM, BC_VACUUM, BC_VACUUM],
        T_bdr=[1.0, 0.0, 0.0, 0.0], inflow_g=[None] * 4, T0=0.01, dt=1e-3,
        n_steps=n_steps, seed=seed)


def multigroup_2d(n: int = 256, G: int = 16, sn: int = 8, region: int = 16, seed: int = 3,
                  n_steps: int = 10, cv_range=None, domain: float = 1.0) -> Problem:
    """2D multigroup lattice-like problem.

    Groups log-spaced on [1e-3, 10]; sigma_g(T) = sigma0_r / (nubar_g^3 T^3)
    clipped to [1e-2, 1e5], sigma0_r per region log-uniform on [1, 100];
    c_v = 1 unless ``cv_range`` gives a per-region log-uniform range.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    om, w = level_symmetric_2d(sn)
    reg, nreg = _block_regions(n, n, region)
    s0 = _log_uniform(rng, 1.0, 100.0, nreg)
    cv = _log_uniform(rng, cv_range[0], cv_range[1], nreg) if cv_range else np.ones(nreg)
    return Problem(
        name=f"multigroup_2d_{n}_g{G}_s{sn}", dim=2, nx=n, ny=n,
        x_edges=np.linspace(0.0, domain, n + 1), y_edges=np.linspace(0.0, domain, n + 1),
        omega=om, w=w, G=G, nu_edges=np.logspace(-3.0, 1.0, G + 1), a=1.0, c=1.0,
        region_of_cell=reg, model=MODEL_POWERLAW, sigma0=s0, clip_lo=1e-2, clip_hi=1e5,
        cv=cv, bc_kind=[BC_PLANCK, BC_VACUUM, BC_VACUUM, BC_VACUUM],
        T_bdr=[1.0, 0.0, 0.0, 0.0], inflow_g=[None] * 4, T0=0.01, dt=1e-3,
        n_steps=n_steps, seed=seed)


def chebyshev_block_edges(n_blocks: int, per_block: int, block: float = 1.0) -> np.ndarray:
    """Cell edges along one axis of ``n_blocks`` blocks of width ``block``,
    each cut into ``per_block`` cells at the Chebyshev points of the second
    kind (x_k = (1 - cos(pi k / n)) / 2 inside a block), so that cells cluster
    at every block boundary: the refined meshes of the multigroup test of
    Sec. 6 (30 cells per 1 cm block there)."""
    k = np.arange(per_block + 1)
    local = 0.5 * (1.0 - np.cos(np.pi * k / per_block))
    local[0], local[-1] = 0.0, 1.0
    edges = [0.0]
    for b in range(n_blocks):
        edges.extend(((b + local[1:]) * block).tolist())
    return np.array(edges)


def multigroup_2d_clustered(blocks: int = 2, per_block: int = 30, G: int = 16, sn: int = 8, seed: int = 3,
                            n_steps: int = 10) -> Problem:
    """The multigroup problem on a Chebyshev-clustered rectilinear mesh:
    ``blocks`` x ``blocks`` unit blocks of ``per_block``^2 cells each
    (``chebyshev_block_edges``), one opacity region per block, otherwise as
    ``multigroup_2d`` (left side incident at T = 1, others vacuum)."""
    n = blocks * per_block
    p = multigroup_2d(n=n, G=G, sn=sn, region=per_block, seed=seed, n_steps=n_steps, domain=float(blocks))
    p.x_edges = chebyshev_block_edges(blocks, per_block)
    p.y_edges = chebyshev_block_edges(blocks, per_block)
    p.name = f"multigroup_2d_clustered_{blocks}x{per_block}_g{G}_s{sn}"
    return p


def adjoint_2d(n: int = 128, G: int = 8, seed: int = 4, n_steps: int = 10) -> Problem:
    """Adjoint workload: 128^2, S8, 8 groups, 8x8 regions of 16x16 cells with
    per-region sigma0 (log-uniform [1,100]) and c_v (log-uniform [0.5, 2])."""
    p = multigroup_2d(n=n, G=G, sn=8, region=n // 8, seed=seed, n_steps=n_steps, cv_range=(0.5, 2.0))
    p.name = f"adjoint_2d_{n}_g{G}"
    return p


def batch_2d(n_problems: int = 32, seed: int = 5, n_steps: int = 5, sizes=None) -> List[Problem]:
    """Uneven batch: mesh n in {64, 96, ..., 384}, G in {4,8,16,32}, S4/S8/S12.

    The (n, G, S_N) draws come from ``seed``; problem i's opacities come from
    seed 5000+i.  ``sizes`` optionally restricts the mesh sizes (used to make
    small parity batches with the same recipe).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.array(sizes if sizes is not None else list(range(64, 385, 32)))
    out = []
    for i in range(n_problems):
        n = int(rng.choice(ns))
        G = int(rng.choice([4, 8, 16, 32]))
        sn = int(rng.choice([4, 8, 12]))
        p = multigroup_2d(n=n, G=G, sn=sn, region=16, seed=5000 + i, n_steps=n_steps)
        p.name = f"batch{i}_{n}_g{G}_s{sn}"
        out.append(p)
    return out


def workload(name: str, **kw) -> Problem:
    return {"slab_1d": slab_1d, "gray_2d": gray_2d, "multigroup_2d": multigroup_2d,
            "adjoint_2d": adjoint_2d}[name](**kw)


# ----------------------------------------------------------------------------
# Seeded raw arrays for the sweep-only tests
# ----------------------------------------------------------------------------


def random_sweep_inputs(p: Problem, seed: int, dtype=np.float64):
    """Random positive sigma_t[cell][G], q_iso[node][G], psi_prev[d][g][node],
    and general inflow[d][g][boundary node] for raw sweep tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nd, G = p.n_angles, p.G
    sig_t = _log_uniform(rng, 0.5, 200.0, (p.n_cells, G))
    q_iso = rng.uniform(0.0, 1.0, (p.n_nodes, G))
    psi_prev = rng.uniform(0.0, 1.0, (nd, G, p.n_nodes))
    nb = boundary_node_count(p)
    inflow = rng.uniform(0.0, 1.0, (nd, G, nb))
    return (sig_t.astype(dtype), q_iso.astype(dtype), psi_prev.astype(dtype), inflow.astype(dtype))


def boundary_node_count(p: Problem) -> int:
    """Boundary face-node count: 2 in 1D; 4*(nx+ny) in 2D, laid out as
    x- side (2*ny), x+ side (2*ny), y- side (2*nx), y+ side (2*nx); along a
    side, cell index then local face node in increasing coordinate."""
    return 2 if p.dim == 1 else 4 * (p.nx + p.ny)


# ----------------------------------------------------------------------------
# Unstructured quadrilateral meshes (vertices xy[v][2], cells [c][4]
# counter-clockwise), seeded
# ----------------------------------------------------------------------------

def quad_mesh_jittered(nx: int, ny: int, jitter: float = 0.25, seed: int = 0, x_edges=None, y_edges=None):
    """Logically structured quadrilaterals: the vertices of a rectilinear grid
    (uniform on [0,1]^2 unless edges are given), interior ones moved by up to
    jitter x the local spacing in each coordinate (jitter < 0.3 keeps every
    cell convex).  Returns (xy, cells)."""
    xs = np.linspace(0.0, 1.0, nx + 1) if x_edges is None else np.asarray(x_edges, float)
    ys = np.linspace(0.0, 1.0, ny + 1) if y_edges is None else np.asarray(y_edges, float)
    X, Y = np.meshgrid(xs, ys)
    if jitter > 0 and nx > 1 and ny > 1:
        rng = np.random.Generator(np.random.PCG64(seed))
        hx = np.minimum(np.diff(xs)[:-1], np.diff(xs)[1:])[None, :]
        hy = np.minimum(np.diff(ys)[:-1], np.diff(ys)[1:])[:, None]
        X[1:-1, 1:-1] += jitter * hx * rng.uniform(-1, 1, (ny - 1, nx - 1))
        Y[1:-1, 1:-1] += jitter * hy * rng.uniform(-1, 1, (ny - 1, nx - 1))
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    v = lambda i, j: j * (nx + 1) + i
    cells = np.array([[v(i, j), v(i + 1, j), v(i + 1, j + 1), v(i, j + 1)] for j in range(ny) for i in range(nx)],
                     dtype=np.int32)
    return xy, cells


def quad_mesh_split_triangles(n: int, jitter: float = 0.2, seed: int = 0):
    """An unstructured quadrilateral mesh of [0,1]^2: an n x n grid of squares
    (interior vertices jittered), each cut into two triangles along a
    diagonal chosen at random, each triangle cut into three quadrilaterals by
    its centroid and edge midpoints (vertices of valence 3 at the centroids,
    up to 8 at the grid vertices).  Returns (xy, cells)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gx, gy = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1))
    if jitter > 0 and n > 1:
        gx[1:-1, 1:-1] += jitter / n * rng.uniform(-1, 1, (n - 1, n - 1))
        gy[1:-1, 1:-1] += jitter / n * rng.uniform(-1, 1, (n - 1, n - 1))
    pts = [tuple(p) for p in np.stack([gx.ravel(), gy.ravel()], axis=1)]
    mid = {}

    def midpoint(a, b):
        k = (min(a, b), max(a, b))
        if k not in mid:
            pts.append(((pts[a][0] + pts[b][0]) / 2, (pts[a][1] + pts[b][1]) / 2))
            mid[k] = len(pts) - 1
        return mid[k]

    cells = []
    g = lambda i, j: j * (n + 1) + i
    for j in range(n):
        for i in range(n):
            a, b, c, d = g(i, j), g(i + 1, j), g(i + 1, j + 1), g(i, j + 1)
            tris = [(a, b, c), (a, c, d)] if rng.uniform() < 0.5 else [(a, b, d), (b, c, d)]
            for (p, q, r) in tris:                                   # counter-clockwise
                pts.append(tuple(np.mean([pts[p], pts[q], pts[r]], axis=0)))
                ctr = len(pts) - 1
                mpq, mqr, mrp = midpoint(p, q), midpoint(q, r), midpoint(r, p)
                cells += [[p, mpq, ctr, mrp], [q, mqr, ctr, mpq], [r, mrp, ctr, mqr]]
    return np.array(pts, dtype=np.float64), np.array(cells, dtype=np.int32)


def quad_sweep_inputs(n_cells: int, n_angles: int, G: int, n_bnodes: int, seed: int = 0):
    """Seeded sweep inputs on a quadrilateral mesh: sig_t[c][G] log-uniform
    [0.5, 200], q_iso[node][G], psi_prev[d][g][node] and inflow[d][g][b]
    uniform [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sigt = _log_uniform(rng, 0.5, 200.0, (n_cells, G))
    q = rng.uniform(0, 1, (4 * n_cells, G))
    pp = rng.uniform(0, 1, (n_angles, G, 4 * n_cells))
    inf = rng.uniform(0, 1, (n_angles, G, n_bnodes))
    return sigt, q, pp, inf
