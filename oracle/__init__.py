"""ctypes wrapper around the plain FP64 C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s CPU-baseline leg may import this package.  It shares no code
with the GPU library; both receive the same seeded input arrays from
``paper_2504_21784_amd.workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2; OpenMP only spreads the
    sweep's independent (direction, group) pairs over threads)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC,
                               "-lm"])
    return _LIB


_lib = None


def build_variant(path: str, edits) -> C.CDLL:
    """Compile a copy of ``oracle.c`` with textual ``edits`` [(old, new)]
    applied (each must match exactly once) into ``path`` and load it.  Used
    only by the pins, to plant a known mistake and check that a pin fails."""
    src = open(_SRC).read()
    for old, new in edits:
        if src.count(old) != 1:
            raise ValueError(f"edit does not match exactly once: {old!r}")
        src = src.replace(old, new)
    csrc = path + ".c"
    with open(csrc, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-w", "-fopenmp", "-fPIC", "-shared", "-o", path, csrc, "-lm"])
    L = C.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's sweep (0: the OpenMP default); returns the
    count its next sweep uses.  Results do not depend on it."""
    return lib().orc_set_threads(int(n))


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Geom(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("xe", _dp), ("ye", _dp),
                ("nang", C.c_int), ("om", _dp), ("w", _dp), ("G", C.c_int), ("nu", _dp),
                ("a", C.c_double), ("c", C.c_double)]


class Mat(C.Structure):
    _fields_ = [("region", _ip), ("model", C.c_int), ("sigma0", _dp), ("clip_lo", C.c_double),
                ("clip_hi", C.c_double), ("cv", _dp)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int * 4), ("T_bdr", C.c_double * 4), ("inflow_g", _dp * 4)]


class Opts(C.Structure):
    _fields_ = [("eps_outer", C.c_double), ("eps_inner", C.c_double), ("cg_rtol", C.c_double),
                ("elim_rtol", C.c_double), ("max_outer", C.c_int), ("max_inner", C.c_int),
                ("max_cg", C.c_int), ("max_elim", C.c_int), ("scheme", C.c_int), ("lo_time_edge", C.c_int),
                ("fixup", C.c_int), ("T_floor", C.c_double)]


class QGeom(C.Structure):
    _fields_ = [("nv", C.c_int), ("nc", C.c_int), ("xy", _dp), ("cv", _ip), ("nang", C.c_int), ("om", _dp),
                ("w", _dp), ("G", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("outer", C.c_int), ("inner_total", C.c_int), ("cg_total", C.c_int),
                ("elim_max", C.c_int), ("hit_max", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _declare(L):
    gp, mp, bp, op, sp = C.POINTER(Geom), C.POINTER(Mat), C.POINTER(BC), C.POINTER(Opts), C.POINTER(Stats)
    L.orc_spectra.argtypes = [C.c_int, _dp, C.c_double, _dp, _dp]
    L.orc_opacity.argtypes = [gp, mp, _dp, _dp]
    L.orc_sweep.argtypes = [gp, _dp, _dp, _dp, C.c_double, _dp, C.c_int, _dp]
    L.orc_sweep.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    L.orc_adjoint_sweep.argtypes = [gp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_adjoint_sweep.restype = C.c_int
    L.orc_adjoint_gradient.argtypes = [gp, mp, bp, C.POINTER(Opts), C.c_double, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp,
                                       C.c_int, C.POINTER(C.c_int)]
    L.orc_adjoint_gradient.restype = C.c_int
    L.orc_objective.argtypes = [gp, mp, bp, C.POINTER(Opts), C.c_double, C.c_int, C.c_int, _dp, _dp, _dp]
    L.orc_objective.restype = C.c_int
    L.orc_moments.argtypes = [gp, _dp, _dp, _dp]
    L.orc_n_moments.argtypes = [C.c_int]
    L.orc_inflow_from_bc.argtypes = [gp, bp, _dp]
    L.orc_reflect_inflow.argtypes = [gp, bp, _dp, _dp]
    L.orc_reflect_inflow.restype = C.c_int
    L.orc_closures.argtypes = [gp, bp, C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_energy_solve.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, _dp]
    L.orc_energy_solve.restype = C.c_int
    L.orc_lo_solve.argtypes = [gp, mp, op, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, sp]
    L.orc_lo_solve.restype = C.c_int
    L.orc_schur_dense.argtypes = [gp, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_lo_dense.argtypes = [gp, _dp, _dp, _dp]
    L.orc_step.argtypes = [gp, mp, bp, op, C.c_double, _dp, _dp, _dp, _dp, sp]
    L.orc_step.restype = C.c_int
    L.orc_equilibrium_psi.argtypes = [gp, _dp, _dp]
    L.orc_qmesh_nbnodes.argtypes = [C.POINTER(QGeom)]
    L.orc_qmesh_nbnodes.restype = C.c_int
    L.orc_qsweep.argtypes = [C.POINTER(QGeom), _dp, _dp, _dp, C.c_double, _dp, _dp]
    L.orc_qsweep.restype = C.c_int
    L.orc_qstep_unacc.argtypes = [C.POINTER(QGeom), _dp, C.c_double, C.c_double, mp, _dp, op, C.c_double, _dp, _dp,
                                  _dp, sp]
    L.orc_qstep_unacc.restype = C.c_int


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw) -> dict:
    """Tolerances and caps of the paper's numerical results section:
    outer/inner 1e-3, CG 1e-10, elimination 1e-10; caps 100/30/50/40."""
    o = dict(eps_outer=1e-3, eps_inner=1e-3, cg_rtol=1e-10, elim_rtol=1e-10, max_outer=100,
             max_inner=30, max_cg=50, max_elim=40, scheme=0, lo_time_edge=0, fixup=0, T_floor=0.0)
    o.update(kw)
    return o


class Oracle:
    """Holds ctypes descriptors (and keeps the numpy arrays alive) for one Problem."""

    def __init__(self, p, L=None):
        """``L``: an already loaded oracle library (default: the built one);
        the pins load deliberately broken copies this way to show that they
        catch the mistake."""
        self.p = p
        self.L = L if L is not None else lib()
        self._keep = []
        k = self._keep.append
        xe = _f64(p.x_edges); k(xe)
        ye = _f64(p.y_edges) if p.y_edges is not None else None
        if ye is not None:
            k(ye)
        om = _f64(p.omega); k(om)
        w = _f64(p.w); k(w)
        nu = _f64(p.nu_edges); k(nu)
        self.geom = Geom(p.dim, p.nx, p.ny if p.dim == 2 else 1, _p(xe), _p(ye), p.n_angles, _p(om), _p(w),
                         p.G, _p(nu), p.a, p.c)
        reg = np.ascontiguousarray(p.region_of_cell, dtype=np.int32); k(reg)
        s0 = _f64(p.sigma0); k(s0)
        cv = _f64(p.cv); k(cv)
        self.mat = Mat(reg.ctypes.data_as(_ip), p.model, _p(s0), p.clip_lo, p.clip_hi, _p(cv))
        bc = BC()
        for s in range(2 * p.dim):
            bc.kind[s] = p.bc_kind[s]
            bc.T_bdr[s] = p.T_bdr[s]
            if p.inflow_g[s] is not None:
                arr = _f64(p.inflow_g[s]); k(arr)
                bc.inflow_g[s] = _p(arr)
        self.bc = bc
        self.nb = 2 if p.dim == 1 else 4 * (p.nx + p.ny)

    # -- pieces -------------------------------------------------------------
    def spectra(self, T):
        b = np.zeros(self.p.G)
        r = np.zeros(self.p.G)
        self.L.orc_spectra(self.p.G, self.geom.nu, float(T), _p(b), _p(r))
        return b, r

    def opacity(self, T_nodes):
        sig = np.zeros((self.p.n_cells, self.p.G))
        T = _f64(T_nodes)
        self.L.orc_opacity(C.byref(self.geom), C.byref(self.mat), _p(T), _p(sig))
        return sig

    def inflow(self, psi=None):
        """Boundary inflow [d][g][NB] from the boundary description; with psi
        the reflective sides carry the mirrored intensities of psi."""
        a = np.zeros((self.p.n_angles, self.p.G, self.nb))
        self.L.orc_inflow_from_bc(C.byref(self.geom), C.byref(self.bc), _p(a))
        if psi is not None:
            r = self.L.orc_reflect_inflow(C.byref(self.geom), C.byref(self.bc), _p(_f64(psi)), _p(a))
            assert r == 0, "a reflective side needs the mirrored direction of every direction"
        return a

    def sweep(self, sig_t, q_iso, psi_prev, inv_c_dt, inflow, fixup=False):
        """Lumped DG sweep of every (d, g); fixup=True applies the
        zero-and-scale negative-flux fixup in every cell."""
        p = self.p
        out = np.zeros((p.n_angles, p.G, p.n_nodes))
        st, q = _f64(sig_t), _f64(q_iso)
        pp = _f64(psi_prev) if psi_prev is not None else None
        inf = _f64(inflow) if inflow is not None else None
        r = self.L.orc_sweep(C.byref(self.geom), _p(st), _p(q), _p(pp), float(inv_c_dt), _p(inf), int(bool(fixup)),
                             _p(out))
        assert r == 0
        return out

    def adjoint_sweep(self, sig_t, src, emis=None, psi_fwd=None):
        """lambda = L^{-T} (w . src) per (d, g) (zero inflow); with emis and
        psi_fwd also dsig[cell][G]."""
        p = self.p
        lam = np.zeros((p.n_angles, p.G, p.n_nodes))
        want = emis is not None and psi_fwd is not None
        dsig = np.zeros((p.n_cells, p.G)) if want else None
        r = self.L.orc_adjoint_sweep(C.byref(self.geom), _p(_f64(sig_t)), _p(_f64(src)),
                                     _p(_f64(emis)) if want else None, _p(_f64(psi_fwd)) if want else None,
                                     _p(lam), _p(dsig))
        assert r == 0
        return (lam, dsig) if want else lam

    def objective(self, opts, n_steps, objective=0, dt=None):
        """J over n_steps from the initial state: objective 0 the time-integrated
        right-boundary outflow, 1 the material energy sum_n w_n c_v T_n at the end."""
        st = self.initial_state()
        J = C.c_double(0.0)
        o = Opts(**opts)
        r = self.L.orc_objective(C.byref(self.geom), C.byref(self.mat), C.byref(self.bc), C.byref(o),
                                 float(dt if dt is not None else self.p.dt), int(n_steps), int(objective),
                                 _p(st["psi"]), _p(st["T"]), C.byref(J))
        assert r == 0, r
        return J.value

    def leakage(self, opts, n_steps, dt=None):
        """Time-integrated right-boundary outflow over n_steps from the initial state."""
        return self.objective(opts, n_steps, 0, dt)

    def adjoint_gradient(self, opts, n_steps, dt=None, objective=0):
        """(J, dJ/dlog sigma0 [n_regions], dJ/dlog c_v [n_regions], adjoint iterations)."""
        st = self.initial_state()
        nr = self.p.n_regions
        J = C.c_double(0.0)
        gs, gc = np.zeros(nr), np.zeros(nr)
        it = C.c_int(0)
        o = Opts(**opts)
        r = self.L.orc_adjoint_gradient(C.byref(self.geom), C.byref(self.mat), C.byref(self.bc), C.byref(o),
                                        float(dt if dt is not None else self.p.dt), int(n_steps), int(objective),
                                        _p(st["psi"]), _p(st["T"]), C.byref(J), _p(gs), _p(gc), nr, C.byref(it))
        assert r == 0, r
        return J.value, gs, gc, it.value

    def moments(self, sig, psi):
        nm = self.L.orc_n_moments(self.p.dim)
        out = np.zeros((nm, self.p.n_nodes))
        self.L.orc_moments(C.byref(self.geom), _p(_f64(sig)), _p(_f64(psi)), _p(out))
        return out

    def closures(self, scheme, dt, sig, T_l, Estar, Fstar, psi, inflow):
        p, nn = self.p, self.p.n_nodes
        sigE, sigF, sigP, qE = (np.zeros(nn) for _ in range(4))
        qF = np.zeros((nn, p.dim))
        args = [_f64(sig), _f64(T_l), _f64(Estar), _f64(Fstar), _f64(psi), _f64(inflow)]
        self.L.orc_closures(C.byref(self.geom), C.byref(self.bc), scheme, float(dt), *[_p(a) for a in args],
                            _p(sigE), _p(sigF), _p(sigP), _p(qE), _p(qF))
        return dict(sigE=sigE, sigF=sigF, sigP=sigP, qE=qE, qF=qF)

    def energy_solve(self, cv_dt, k4, rhs, T0, rtol=1e-10, maxit=40):
        T = C.c_double(0.0)
        it = self.L.orc_energy_solve(cv_dt, k4, rhs, T0, rtol, maxit, C.byref(T))
        return it, T.value

    def lo_solve(self, opts, dt, Tstar, cl, E, T):
        p = self.p
        E = _f64(E).copy()
        T = _f64(T).copy()
        F = np.zeros((p.n_nodes, p.dim))
        st = Stats()
        o = Opts(**opts)
        r = self.L.orc_lo_solve(C.byref(self.geom), C.byref(self.mat), C.byref(o), float(dt), _p(_f64(Tstar)),
                                _p(_f64(cl["sigE"])), _p(_f64(cl["sigF"])), _p(_f64(cl["sigP"])),
                                _p(_f64(cl["qE"])), _p(_f64(cl["qF"])), _p(E), _p(F), _p(T), C.byref(st))
        return r, E, F, T, st.as_dict()

    def schur_dense(self, dt, sigE, sigF, sigP, cvn, T0):
        nn = self.p.n_nodes
        S = np.zeros((nn, nn))
        self.L.orc_schur_dense(C.byref(self.geom), float(dt), *[_p(_f64(a)) for a in (sigE, sigF, sigP, cvn, T0)], _p(S))
        return S

    def lo_dense(self):
        nn, dim = self.p.n_nodes, self.p.dim
        D = np.zeros((nn, nn * dim))
        P = np.zeros((nn, nn))
        wv = np.zeros(nn)
        self.L.orc_lo_dense(C.byref(self.geom), _p(D), _p(P), _p(wv))
        return D, P, wv

    def equilibrium_psi(self, T_nodes):
        p = self.p
        out = np.zeros((p.n_angles, p.G, p.n_nodes))
        self.L.orc_equilibrium_psi(C.byref(self.geom), _p(_f64(T_nodes)), _p(out))
        return out

    # -- state --------------------------------------------------------------
    def initial_state(self):
        p = self.p
        T = p.initial_T_nodes()
        psi = self.equilibrium_psi(T)
        E = np.full(p.n_nodes, p.a * p.T0 ** 4)
        F = np.zeros((p.n_nodes, p.dim))
        return dict(psi=psi, T=T, E=E, F=F)

    def step(self, state, opts, dt=None):
        """One backward-Euler step; returns (status, new_state, stats)."""
        p = self.p
        s = {k: _f64(v).copy() for k, v in state.items()}
        st = Stats()
        o = Opts(**opts)
        r = self.L.orc_step(C.byref(self.geom), C.byref(self.mat), C.byref(self.bc), C.byref(o),
                            float(dt if dt is not None else p.dt), _p(s["psi"]), _p(s["T"]), _p(s["E"]),
                            _p(s["F"]), C.byref(st))
        return r, s, st.as_dict()


class QuadMesh:
    """The lumped bilinear DG sweep on an unstructured quadrilateral mesh
    (vertices xy[v][2], cells[c][4] counter-clockwise) with the quadrature
    omega[d][3], w[d] and G groups."""

    def __init__(self, xy, cells, omega, w, G):
        self.L = lib()
        self.xy = _f64(xy).reshape(-1, 2)
        self.cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 4)
        self.om = _f64(omega).reshape(-1, 3)
        self.w = _f64(w)
        self.G = int(G)
        self.geom = QGeom(len(self.xy), len(self.cells), _p(self.xy), self.cells.ctypes.data_as(_ip),
                          len(self.w), _p(self.om), _p(self.w), self.G)
        self.nb = self.L.orc_qmesh_nbnodes(C.byref(self.geom))
        assert self.nb >= 0, "non-manifold mesh"

    def sweep(self, sig_t, q_iso, psi_prev, inv_c_dt, inflow, fill=0.0):
        """fill: the value the output buffer holds before the sweep (the
        result must not depend on it)."""
        nn = 4 * len(self.cells)
        out = np.full((len(self.w), self.G, nn), float(fill))
        pp = _f64(psi_prev) if psi_prev is not None else None
        inf = _f64(inflow) if inflow is not None else None
        r = self.L.orc_qsweep(C.byref(self.geom), _p(_f64(sig_t)), _p(_f64(q_iso)), _p(pp), float(inv_c_dt),
                              _p(inf), _p(out))
        assert r == 0, f"orc_qsweep returned {r}"
        return out

    def step_unaccelerated(self, T, psi, region, sigma0, cv, nu, a, c, dt, inflow=None, model=1, clip_lo=1e-2,
                           clip_hi=1e5, **opts):
        """One backward-Euler step of the unaccelerated scheme (Algorithm 1
        without the low-order solve) with a fixed boundary inflow[d][g][NB]:
        returns (status, T, E, psi, stats).  region[cell], sigma0 and cv per
        region, nu the G + 1 group bounds; options as default_opts."""
        o = Opts(**{k: v for k, v in default_opts(**opts).items() if k in dict(Opts._fields_)})
        reg = np.ascontiguousarray(region, dtype=np.int32)
        s0, cvr, nuv = _f64(sigma0), _f64(cv), _f64(nu)
        mat = Mat(reg.ctypes.data_as(_ip), int(model), _p(s0), float(clip_lo), float(clip_hi), _p(cvr))
        Tn, ps = _f64(T).copy(), _f64(psi).copy()
        E = np.zeros_like(Tn)
        st = Stats()
        inf = _f64(inflow) if inflow is not None else None
        r = self.L.orc_qstep_unacc(C.byref(self.geom), _p(nuv), float(a), float(c), C.byref(mat), _p(inf),
                                   C.byref(o), float(dt), _p(ps), _p(Tn), _p(E), C.byref(st))
        return r, Tn, E, ps, {f: getattr(st, f) for f, _ in Stats._fields_}

    def moments(self, sig, psi):
        """Gray angular moments per node of an intensity psi[d][g][node]: the
        moment sums of Sec. 2 over directions and groups, split by the
        quadrant of the direction as on the rectilinear mesh (for quadrant q,
        row 6q + m sums w_d f_m I with f = 1, mu, eta, mu^2, mu eta, eta^2;
        q = 0 for mu, eta > 0, 1 for mu < 0 < eta, 2 for both < 0, 3 for the
        rest), and rows 24-26 sum sig_g w_d (1, mu, eta) I with sig[cell][g].
        Written out one direction at a time."""
        nn = 4 * len(self.cells)
        psi = _f64(psi).reshape(len(self.w), self.G, nn)
        sg = np.repeat(_f64(sig).reshape(-1, self.G), 4, axis=0).T      # [g][node]
        mom = np.zeros((27, nn))
        for d in range(len(self.w)):
            mu, eta, w = self.om[d, 0], self.om[d, 1], self.w[d]
            q = 0 if (mu > 0 and eta > 0) else 1 if (mu < 0 and eta > 0) else 2 if (mu < 0 and eta < 0) else 3
            tot = psi[d].sum(axis=0)
            for m, f in enumerate((1.0, mu, eta, mu * mu, mu * eta, eta * eta)):
                mom[6 * q + m] += w * f * tot
            absorbed = (sg * psi[d]).sum(axis=0)
            for m, f in enumerate((1.0, mu, eta)):
                mom[24 + m] += w * f * absorbed
        return mom
