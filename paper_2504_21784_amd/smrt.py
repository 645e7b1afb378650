"""Thin ctypes binding of the gfx950 SM-TRT library (``libsmrt.so``).

Argument marshalling only: every step of the transport sweep, moments,
closures, low-order solve and time step runs in the HIP library.  The
binding raises if the compiled library is missing -- there is no CPU
fallback.  Names follow the C ABI in ``include/smrt.h``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from .tune_cache import TuneCache, problem_key

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmrt.so")

SMRT_FP64, SMRT_FP32 = 0, 1
SMRT_SM_CONSISTENT, SMRT_SM_INDEPENDENT, SMRT_UNACCELERATED = 0, 1, 2
STATUS = {0: "SMRT_OK", 1: "SMRT_E_INVALID_ARG", 2: "SMRT_E_OUT_OF_MEMORY", 3: "SMRT_E_DEVICE",
          4: "SMRT_E_NOT_CONVERGED", 5: "SMRT_E_NONPHYSICAL", 6: "SMRT_E_STATE"}
(SMRT_OK, SMRT_E_INVALID_ARG, SMRT_E_OUT_OF_MEMORY, SMRT_E_DEVICE, SMRT_E_NOT_CONVERGED, SMRT_E_NONPHYSICAL,
 SMRT_E_STATE) = range(7)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("x_edges", _dp), ("y_edges", _dp)]


class QuadDesc(C.Structure):
    _fields_ = [("n_angles", C.c_int), ("omega", _dp), ("w", _dp)]


class GroupsDesc(C.Structure):
    _fields_ = [("G", C.c_int), ("nu_edges", _dp), ("a", C.c_double), ("c", C.c_double)]


class MaterialDesc(C.Structure):
    _fields_ = [("n_regions", C.c_int), ("region_of_cell", C.POINTER(C.c_int32)), ("model", C.c_int),
                ("sigma0", _dp), ("clip_lo", C.c_double), ("clip_hi", C.c_double), ("cv", _dp)]


class BoundaryDesc(C.Structure):
    _fields_ = [("kind", C.c_int * 4), ("T_bdr", C.c_double * 4), ("inflow_g", _dp * 4)]


class Options(C.Structure):
    _fields_ = [("eps_outer", C.c_double), ("eps_inner", C.c_double), ("cg_rtol", C.c_double),
                ("elim_rtol", C.c_double), ("max_outer", C.c_int), ("max_inner", C.c_int), ("max_cg", C.c_int),
                ("max_elim", C.c_int), ("precision", C.c_int), ("scheme", C.c_int), ("strict", C.c_int),
                ("fixed_outer", C.c_int), ("lo_time_edge", C.c_int), ("lo_graphs", C.c_int),
                ("fixup", C.c_int), ("T_floor", C.c_double), ("lo_precond", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("outer", C.c_int), ("inner_total", C.c_int), ("cg_total", C.c_int), ("elim_max", C.c_int),
                ("hit_max", C.c_int), ("t_sweep_ms", C.c_double),
                ("t_lo_ms", C.c_double), ("t_total_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("n_angles", C.c_int), ("G", C.c_int),
                ("n_nodes", C.c_int), ("n_cells", C.c_int), ("units_per_sweep", C.c_int64),
                ("algorithmic_bytes_per_sweep", C.c_int64), ("band_rows", C.c_int), ("waves_per_band", C.c_int),
                ("pairs_per_lane", C.c_int), ("pairs_per_chunk", C.c_int), ("n_chunks", C.c_int),
                ("n_workgroups", C.c_int), ("bands_per_group", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def device_name() -> str:
    """The current HIP device as "<name> <arch> <n> CUs" (the tuning cache key)."""
    L = load()
    buf = C.create_string_buffer(256)
    n = C.c_int(0)
    st = L.smrt_device_name(buf, 256, C.byref(n))
    if st != 0:
        raise SmrtError(st, L.smrt_last_error(None).decode())
    return f"{buf.value.decode()} {n.value} CUs"


def _cache(cache):
    return TuneCache() if cache is True else cache

# exported names and ctypes signatures (argtypes, restype)
_SIGS = {
    "smrt_default_options": ([C.POINTER(Options)], None),
    "smrt_create": ([C.POINTER(MeshDesc), C.POINTER(QuadDesc), C.POINTER(GroupsDesc), C.POINTER(MaterialDesc),
                     C.POINTER(BoundaryDesc), C.POINTER(Options), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "smrt_destroy": ([C.c_void_p], None),
    "smrt_last_error": ([C.c_void_p], C.c_char_p),
    "smrt_set_options": ([C.c_void_p, C.POINTER(Options)], C.c_int),
    "smrt_set_boundary": ([C.c_void_p, C.POINTER(BoundaryDesc)], C.c_int),
    "smrt_set_state": ([C.c_void_p, _dp, _dp], C.c_int),
    "smrt_get_state": ([C.c_void_p, _dp, _dp, _dp, _dp], C.c_int),
    "smrt_sweep": ([C.c_void_p, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp], C.c_int),
    "smrt_sweep_dev": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                        C.c_void_p, C.c_void_p], C.c_int),
    "smrt_sweep_dev_static": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                               C.c_void_p, C.c_void_p], C.c_int),
    "smrt_compute_closures": ([C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.c_double, _dp], C.c_int),
    "smrt_lo_solve": ([C.c_void_p, _dp, _dp, C.c_double, _dp, _dp, _dp, C.POINTER(StepStats)], C.c_int),
    "smrt_step": ([C.c_void_p, C.c_double, C.POINTER(StepStats)], C.c_int),
    "smrt_sweep_resident": ([C.c_void_p, C.c_double, C.c_int, _dp, _dp], C.c_int),
    "smrt_get_info": ([C.c_void_p, C.POINTER(Info)], C.c_int),
    "smrt_get_moments": ([C.c_void_p, _dp], C.c_int),
    "smrt_set_launch": ([C.c_void_p, C.c_int, C.c_int, C.c_int], C.c_int),
    "smrt_autotune": ([C.c_void_p, C.c_double, _ip, _ip, _ip, _ip, _dp], C.c_int),
    "smrt_device_name": ([C.c_char_p, C.c_int, _ip], C.c_int),
    "smrt_set_occupancy": ([C.c_void_p, C.c_int], C.c_int),
    "smrt_batch_set_occupancy": ([C.c_void_p, C.c_int], C.c_int),
    "smrt_adjoint_sweep": ([C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp], C.c_int),
    "smrt_set_materials": ([C.c_void_p, _dp, _dp], C.c_int),
    "smrt_adjoint": ([C.c_void_p, C.c_int, C.c_int, C.c_double, _dp, _dp, _dp, _ip], C.c_int),
    "smrt_batch_create": ([C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)], C.c_int),
    "smrt_batch_destroy": ([C.c_void_p], None),
    "smrt_batch_last_error": ([C.c_void_p], C.c_char_p),
    "smrt_batch_set_launch": ([C.c_void_p, C.c_int, C.c_int, C.c_int], C.c_int),
    "smrt_batch_info": ([C.c_void_p, C.POINTER(C.c_int64), _ip, _ip, _ip, _ip], C.c_int),
    "smrt_batch_autotune": ([C.c_void_p, C.c_double, _ip, _ip, _ip, _ip, _dp], C.c_int),
    "smrt_batch_sweep_resident": ([C.c_void_p, C.c_double, C.c_int, C.c_int, _dp, _dp], C.c_int),
    "smrt_batch_step": ([C.c_void_p, _dp, C.POINTER(StepStats)], C.c_int),
    "smrt_batch_run": ([C.c_void_p, C.c_int, _dp, C.POINTER(StepStats), C.c_int], C.c_int),
    "smrt_qmesh_create": ([C.c_int, _dp, C.c_int, C.POINTER(C.c_int32), C.POINTER(QuadDesc), C.c_int, C.c_int,
                           C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "smrt_qmesh_destroy": ([C.c_void_p], None),
    "smrt_qmesh_last_error": ([C.c_void_p], C.c_char_p),
    "smrt_qmesh_info": ([C.c_void_p, _ip, _ip], C.c_int),
    "smrt_qmesh_sweep": ([C.c_void_p, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp], C.c_int),
    "smrt_qmesh_moments": ([C.c_void_p, _dp, _dp, _dp], C.c_int),
    "smrt_qmesh_set_materials": ([C.c_void_p, C.POINTER(C.c_int32), C.c_int, C.c_int, _dp, C.c_double, C.c_double,
                                  _dp, _dp, C.c_double, C.c_double], C.c_int),
    "smrt_qmesh_set_state": ([C.c_void_p, _dp, _dp], C.c_int),
    "smrt_qmesh_step": ([C.c_void_p, C.c_double, _dp, C.POINTER(Options), C.POINTER(StepStats)], C.c_int),
    "smrt_qmesh_get_state": ([C.c_void_p, _dp, _dp, _dp], C.c_int),
}


def load():
    """Load libsmrt.so (no fallback: raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2504_21784_amd.build.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


class SmrtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_options(**kw) -> Options:
    o = Options()
    load().smrt_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """One problem on the GPU.  ``problem`` is a workloads.Problem."""

    def __init__(self, problem, precision=SMRT_FP64, scheme=SMRT_SM_CONSISTENT, stream=None, **opts):
        L = load()
        self.L = L
        self.p = p = problem
        keep = self._keep = []

        def arr(a, dt=np.float64):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a

        xe = arr(p.x_edges)
        ye = arr(p.y_edges) if p.y_edges is not None else None
        self.mesh = MeshDesc(p.dim, p.nx, p.ny if p.dim == 2 else 1, _p(xe), _p(ye))
        om, w = arr(p.omega), arr(p.w)
        self.quad = QuadDesc(p.n_angles, _p(om), _p(w))
        nu = arr(p.nu_edges)
        self.groups = GroupsDesc(p.G, _p(nu), p.a, p.c)
        reg = arr(p.region_of_cell, np.int32)
        s0, cv = arr(p.sigma0), arr(p.cv)
        self.mat = MaterialDesc(p.n_regions, reg.ctypes.data_as(C.POINTER(C.c_int32)), p.model, _p(s0), p.clip_lo,
                                p.clip_hi, _p(cv))
        self.bc = self._bc(p)
        self.opts = default_options(precision=precision, scheme=scheme, **opts)
        h = C.c_void_p()
        st = L.smrt_create(C.byref(self.mesh), C.byref(self.quad), C.byref(self.groups), C.byref(self.mat),
                           C.byref(self.bc), C.byref(self.opts), stream, C.byref(h))
        if st != 0:
            raise SmrtError(st, L.smrt_last_error(None).decode())
        self.h = h

    def _bc(self, p):
        bc = BoundaryDesc()
        for s in range(2 * p.dim):
            bc.kind[s] = p.bc_kind[s]
            bc.T_bdr[s] = p.T_bdr[s]
            if p.inflow_g[s] is not None:
                a = _f64(p.inflow_g[s])
                self._keep.append(a)
                bc.inflow_g[s] = _p(a)
        return bc

    def _check(self, st):
        if st != 0:
            raise SmrtError(st, self.L.smrt_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.smrt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI wrappers ------------------------------------------------------
    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.opts, k, v)
        self._check(self.L.smrt_set_options(self.h, C.byref(self.opts)))

    def set_boundary(self, problem=None):
        self.bc = self._bc(problem or self.p)
        self._check(self.L.smrt_set_boundary(self.h, C.byref(self.bc)))

    def set_occupancy(self, workgroups_per_cu=0):
        self._check(self.L.smrt_set_occupancy(self.h, int(workgroups_per_cu)))

    def set_launch(self, waves_per_band=0, bands_per_group=0, pairs_per_lane=0):
        """Sweep launch shape (0 = automatic per field)."""
        self._check(self.L.smrt_set_launch(self.h, int(waves_per_band), int(bands_per_group), int(pairs_per_lane)))

    def info(self) -> dict:
        i = Info()
        self._check(self.L.smrt_get_info(self.h, C.byref(i)))
        return i.as_dict()

    def set_state(self, T, psi=None):
        T = _f64(T)
        ps = _f64(psi) if psi is not None else None
        self._check(self.L.smrt_set_state(self.h, _p(T), _p(ps)))

    def get_state(self, with_psi=True):
        p = self.p
        T, E = np.zeros(p.n_nodes), np.zeros(p.n_nodes)
        F = np.zeros((p.n_nodes, p.dim))
        psi = np.zeros((p.n_angles, p.G, p.n_nodes)) if with_psi else None
        self._check(self.L.smrt_get_state(self.h, _p(T), _p(E), _p(F), _p(psi)))
        return dict(T=T, E=E, F=F, psi=psi)

    def sweep(self, sig_t, sig, q_iso, psi_prev, inv_c_dt, inflow=None):
        p = self.p
        psi = np.zeros((p.n_angles, p.G, p.n_nodes))
        mom = np.zeros((27 if p.dim == 2 else 8, p.n_nodes))
        args = [_f64(sig_t), _f64(sig), _f64(q_iso)]
        pp = _f64(psi_prev) if psi_prev is not None else None
        inf = _f64(inflow) if inflow is not None else None
        self._check(self.L.smrt_sweep(self.h, *[_p(a) for a in args], _p(pp), float(inv_c_dt), _p(inf), _p(psi),
                                      _p(mom)))
        return psi, mom

    def sweep_dev(self, sig_t, sig, q_iso, psi_prev, inv_c_dt, inflow=None, psi_out=None, moments_out=None,
                  static_scratch=False):
        """smrt_sweep on device tensors (float64, contiguous, on the context's GPU), no host round trip.
        Returns (psi_out, moments_out or None); psi_out is allocated if not given.  static_scratch=True
        calls the allocation-free entry point (work arrays in the library's static device array)."""
        import torch
        p = self.p
        want = {"sig_t": (p.n_cells, p.G), "sig": (p.n_cells, p.G), "q_iso": (p.n_nodes, p.G),
                "psi_prev": (p.n_angles, p.G, p.n_nodes), "inflow": (p.n_angles, p.G, 2 if p.dim == 1 else 4 * (p.nx + p.ny)),
                "psi_out": (p.n_angles, p.G, p.n_nodes), "moments_out": (27 if p.dim == 2 else 8, p.n_nodes)}
        if psi_out is None:
            psi_out = torch.empty(want["psi_out"], dtype=torch.float64, device=sig_t.device)
        args = dict(sig_t=sig_t, sig=sig, q_iso=q_iso, psi_prev=psi_prev, inflow=inflow, psi_out=psi_out,
                    moments_out=moments_out)
        for name, t in args.items():
            if t is None:
                continue
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == want[name]):
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {want[name]}")
        ptr = {k: (v.data_ptr() if v is not None else None) for k, v in args.items()}
        torch.cuda.current_stream(sig_t.device).synchronize()   # inputs ready before the context stream reads them
        fn = self.L.smrt_sweep_dev_static if static_scratch else self.L.smrt_sweep_dev
        self._check(fn(self.h, ptr["sig_t"], ptr["sig"], ptr["q_iso"], ptr["psi_prev"], float(inv_c_dt), ptr["inflow"],
                       ptr["psi_out"], ptr["moments_out"]))
        return psi_out, moments_out

    def adjoint_sweep(self, sig_t, src, emis=None, psi_fwd=None, want_dsig=False):
        """lambda = L^{-T}(w . src) per (d, g); with want_dsig also the opacity
        sensitivity dsig[cell][G] (needs emis[node][G] and psi_fwd)."""
        p = self.p
        lam = np.zeros((p.n_angles, p.G, p.n_nodes))
        dsig = np.zeros((p.n_cells, p.G)) if want_dsig else None
        st, s = _f64(sig_t), _f64(src)
        e = _f64(emis) if emis is not None else None
        f = _f64(psi_fwd) if psi_fwd is not None else None
        self._check(self.L.smrt_adjoint_sweep(self.h, _p(st), _p(s), _p(e), _p(f), _p(lam), _p(dsig)))
        return (lam, dsig) if want_dsig else lam

    def set_materials(self, sigma0=None, cv=None):
        s0 = _f64(sigma0) if sigma0 is not None else None
        c = _f64(cv) if cv is not None else None
        self._check(self.L.smrt_set_materials(self.h, _p(s0), _p(c)))

    def adjoint(self, n_steps, dt=None, objective=0):
        """Runs n_steps from the current state; returns (J, dJ/dlog sigma0, dJ/dlog c_v, adjoint iterations).
        objective 0: time-integrated x+ outflow; 1: material energy at the last step."""
        nr = self.p.n_regions
        J = C.c_double(0.0)
        gs, gc = np.zeros(nr), np.zeros(nr)
        it = C.c_int(0)
        self._check(self.L.smrt_adjoint(self.h, int(objective), int(n_steps), float(dt if dt is not None else self.p.dt),
                                        C.byref(J), _p(gs), _p(gc), C.byref(it)))
        return J.value, gs, gc, it.value

    def compute_closures(self, moments, T_l, Estar, Fstar, sig, dt):
        p = self.p
        out = np.zeros((4 + p.dim, p.n_nodes))
        args = [_f64(moments), _f64(T_l), _f64(Estar), _f64(Fstar), _f64(sig)]
        self._check(self.L.smrt_compute_closures(self.h, *[_p(a) for a in args], float(dt), _p(out)))
        return out

    def lo_solve(self, closures, Tstar, dt, E, T):
        p = self.p
        E, T = _f64(E).copy(), _f64(T).copy()
        F = np.zeros((p.n_nodes, p.dim))
        st = StepStats()
        self._check(self.L.smrt_lo_solve(self.h, _p(_f64(closures)), _p(_f64(Tstar)), float(dt), _p(E), _p(F), _p(T),
                                         C.byref(st)))
        return E, F, T, st.as_dict()

    def get_moments(self):
        m = np.zeros((27 if self.p.dim == 2 else 8, self.p.n_nodes))
        self._check(self.L.smrt_get_moments(self.h, _p(m)))
        return m

    def step(self, dt=None) -> dict:
        st = StepStats()
        self._check(self.L.smrt_step(self.h, float(dt if dt is not None else self.p.dt), C.byref(st)))
        return st.as_dict()

    def sweep_resident(self, dt=None, n_times=1):
        """Returns (ms per high-order pass, ms of the sweep kernel alone)."""
        ms, ks = C.c_double(0.0), C.c_double(0.0)
        self._check(self.L.smrt_sweep_resident(self.h, float(dt if dt is not None else self.p.dt), int(n_times),
                                               C.byref(ms), C.byref(ks)))
        return ms.value, ks.value

    def autotune(self, dt=None, cache=None):
        """Pick the fastest sweep launch shape; returns (waves per band, bands per
        workgroup, groups per lane, ms).  cache: a tune_cache.TuneCache (or
        True for the default file): a shape stored for the same device and
        sweep shape is applied without timing (self.last_tune_cached says
        which happened), and a new one is stored."""
        key = None
        self.last_tune_cached = False
        if cache:
            cache = _cache(cache)
            p = self.p
            key = problem_key("single", device_name(), self.opts.precision,
                              [(p.nx, p.ny if p.dim == 2 else 1, p.G, p.n_angles)], self.opts.fixup)
            e = cache.get(key)
            if e is not None:
                self.set_launch(e["waves_per_band"], e["bands_per_group"], e["pairs_per_lane"])
                self.set_occupancy(e["workgroups_per_cu"])
                self.last_tune_cached = True
                return e["waves_per_band"], e["bands_per_group"], e["pairs_per_lane"], e["ms"]
        nw, nb, k, occ, ms = C.c_int(0), C.c_int(0), C.c_int(0), C.c_int(0), C.c_double(0.0)
        self._check(self.L.smrt_autotune(self.h, float(dt if dt is not None else self.p.dt), C.byref(nw), C.byref(nb),
                                         C.byref(k), C.byref(occ), C.byref(ms)))
        if key is not None:
            cache.put(key, {"waves_per_band": nw.value, "bands_per_group": nb.value, "pairs_per_lane": k.value,
                            "workgroups_per_cu": occ.value, "ms": ms.value})
        return nw.value, nb.value, k.value, ms.value


class Batch:
    """Many 2D contexts swept together (one launch per sweep).  The contexts
    stay owned by the caller and must outlive the batch."""

    def __init__(self, contexts):
        self.L = load()
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h for c in self.contexts])
        h = C.c_void_p()
        st = self.L.smrt_batch_create(len(self.contexts), arr, C.byref(h))
        if st != 0:
            raise SmrtError(st, self.L.smrt_batch_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != 0:
            raise SmrtError(st, self.L.smrt_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.smrt_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        u, t, nw, nb, k = C.c_int64(0), C.c_int(0), C.c_int(0), C.c_int(0), C.c_int(0)
        self._check(self.L.smrt_batch_info(self.h, C.byref(u), C.byref(t), C.byref(nw), C.byref(nb), C.byref(k)))
        return {"units_per_sweep": u.value, "n_tasks": t.value, "waves_per_band": nw.value, "bands_per_group": nb.value,
                "pairs_per_lane": k.value}

    def set_launch(self, waves_per_band, bands_per_group, pairs_per_lane=1):
        self._check(self.L.smrt_batch_set_launch(self.h, int(waves_per_band), int(bands_per_group), int(pairs_per_lane)))

    def set_occupancy(self, workgroups_per_cu=0):
        self._check(self.L.smrt_batch_set_occupancy(self.h, int(workgroups_per_cu)))

    def autotune(self, dt, cache=None):
        """Fastest batched launch shape (as Context.autotune, cache likewise)."""
        key = None
        self.last_tune_cached = False
        if cache:
            cache = _cache(cache)
            c0 = self.contexts[0]
            key = problem_key("batch", device_name(), c0.opts.precision,
                              [(c.p.nx, c.p.ny, c.p.G, c.p.n_angles) for c in self.contexts], c0.opts.fixup)
            e = cache.get(key)
            if e is not None:
                self.set_launch(e["waves_per_band"], e["bands_per_group"], e["pairs_per_lane"])
                self.set_occupancy(e["workgroups_per_cu"])
                self.last_tune_cached = True
                return e["waves_per_band"], e["bands_per_group"], e["pairs_per_lane"], e["ms"]
        nw, nb, k, occ, ms = C.c_int(0), C.c_int(0), C.c_int(0), C.c_int(0), C.c_double(0.0)
        self._check(self.L.smrt_batch_autotune(self.h, float(dt), C.byref(nw), C.byref(nb), C.byref(k), C.byref(occ),
                                               C.byref(ms)))
        if key is not None:
            cache.put(key, {"waves_per_band": nw.value, "bands_per_group": nb.value, "pairs_per_lane": k.value,
                            "workgroups_per_cu": occ.value, "ms": ms.value})
        return nw.value, nb.value, k.value, ms.value

    def sweep_resident(self, dt, n_times=1, capture_graph=False):
        """Returns (ms per batched high-order pass, ms of one batched sweep launch)."""
        ms, ks = C.c_double(0.0), C.c_double(0.0)
        self._check(self.L.smrt_batch_sweep_resident(self.h, float(dt), int(n_times), int(bool(capture_graph)),
                                                     C.byref(ms), C.byref(ks)))
        return ms.value, ks.value

    def step(self, dt):
        """One time step of every problem; dt scalar or per problem. Returns per-problem stats."""
        n = len(self.contexts)
        d = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)))
        st = (StepStats * n)()
        self._check(self.L.smrt_batch_step(self.h, _p(d), st))
        return [s.as_dict() for s in st]

    def run(self, n_steps, dt, capture_graph=False):
        """n_steps time steps of every problem with device-side convergence
        control; dt scalar, per problem [n] or per step and problem [n_steps][n].
        Returns the stats as a list of n_steps lists of per-problem dicts."""
        n, ns = len(self.contexts), int(n_steps)
        d = np.asarray(dt, dtype=np.float64)
        if d.ndim == 1:
            d = d[None, :]
        d = _f64(np.broadcast_to(d, (ns, n)).ravel())
        st = (StepStats * (ns * n))()
        self._check(self.L.smrt_batch_run(self.h, ns, _p(d), st, int(bool(capture_graph))))
        return [[st[s * n + i].as_dict() for i in range(n)] for s in range(ns)]


class QuadMeshSweep:
    """The sweep on an unstructured quadrilateral mesh (vertices xy[v][2],
    cells[c][4] counter-clockwise) with the quadrature omega[d][3], w[d] and
    G groups, on the GPU."""

    def __init__(self, xy, cells, omega, w, G, precision=SMRT_FP64, stream=None):
        self.L = load()
        self._xy = _f64(np.asarray(xy).reshape(-1, 2))
        self._cells = np.ascontiguousarray(np.asarray(cells).reshape(-1, 4), dtype=np.int32)
        self._om, self._w = _f64(np.asarray(omega).reshape(-1, 3)), _f64(w)
        self.G = int(G)
        self.quad = QuadDesc(len(self._w), _p(self._om), _p(self._w))
        h = C.c_void_p()
        st = self.L.smrt_qmesh_create(len(self._xy), _p(self._xy), len(self._cells),
                                      self._cells.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(self.quad), self.G,
                                      int(precision), stream, C.byref(h))
        if st != 0:
            raise SmrtError(st, self.L.smrt_qmesh_last_error(None).decode())
        self.h = h
        nb, nl = C.c_int(0), C.c_int(0)
        self.L.smrt_qmesh_info(self.h, C.byref(nb), C.byref(nl))
        self.nb, self.n_levels = nb.value, nl.value

    def sweep(self, sig_t, q_iso, psi_prev, inv_c_dt, inflow=None):
        """Returns (psi [d][g][node], milliseconds of the sweep launches)."""
        out = np.zeros((len(self._w), self.G, 4 * len(self._cells)))
        ms = C.c_double(0.0)
        pp = _f64(psi_prev) if psi_prev is not None else None
        inf = _f64(inflow) if inflow is not None else None
        st = self.L.smrt_qmesh_sweep(self.h, _p(_f64(sig_t)), _p(_f64(q_iso)), _p(pp), float(inv_c_dt), _p(inf),
                                     _p(out), C.byref(ms))
        if st != 0:
            raise SmrtError(st, self.L.smrt_qmesh_last_error(self.h).decode())
        return out, ms.value

    def moments(self, sig):
        """Gray moments of the last sweep's intensity, [27][node] in the
        rectilinear path's layout (quadrant-split 1, mu, eta, mu^2, mu eta,
        eta^2 sums, then the sig-weighted 1, mu, eta sums), with sig[cell][g];
        returns (moments, milliseconds of the kernel)."""
        out = np.zeros((27, 4 * len(self._cells)))
        ms = C.c_double(0.0)
        st = self.L.smrt_qmesh_moments(self.h, _p(_f64(sig)), _p(out), C.byref(ms))
        if st != 0:
            raise SmrtError(st, self.L.smrt_qmesh_last_error(self.h).decode())
        return out, ms.value

    def _qcheck(self, st):
        if st != 0:
            raise SmrtError(st, self.L.smrt_qmesh_last_error(self.h).decode())

    def set_materials(self, region, sigma0, cv, nu_edges, a=1.0, c=1.0, model=1, clip_lo=1e-2, clip_hi=1e5):
        """Materials of the time step: region[cell], sigma0 (per region, or
        [region][G] for model 0), c_v per region, the G + 1 group bounds."""
        self._reg = np.ascontiguousarray(region, dtype=np.int32)
        self._s0, self._cv, self._nu = _f64(sigma0).ravel(), _f64(cv), _f64(nu_edges)
        self._qcheck(self.L.smrt_qmesh_set_materials(self.h, self._reg.ctypes.data_as(C.POINTER(C.c_int32)),
                                                     len(self._cv), int(model), _p(self._s0), float(clip_lo),
                                                     float(clip_hi), _p(self._cv), _p(self._nu), float(a), float(c)))

    def set_state(self, T, psi=None):
        """Nodal temperature T[4 n_cells] and intensity psi[d][g][node]
        (None: the isotropic equilibrium at T)."""
        self._qcheck(self.L.smrt_qmesh_set_state(self.h, _p(_f64(T)), _p(_f64(psi) if psi is not None else None)))

    def step(self, dt, inflow=None, **opts):
        """One unaccelerated backward-Euler step with the fixed boundary
        inflow[d][g][NB] (None: vacuum); options as for Context (scheme is
        the unaccelerated one).  Returns the step's stats."""
        kw = dict(scheme=SMRT_UNACCELERATED)
        kw.update(opts)
        o = default_options(**kw)
        st = StepStats()
        inf = _f64(inflow) if inflow is not None else None
        self._qcheck(self.L.smrt_qmesh_step(self.h, float(dt), _p(inf), C.byref(o), C.byref(st)))
        return st.as_dict()

    def get_state(self):
        nn = 4 * len(self._cells)
        T, E = np.zeros(nn), np.zeros(nn)
        psi = np.zeros((len(self._w), self.G, nn))
        self._qcheck(self.L.smrt_qmesh_get_state(self.h, _p(T), _p(E), _p(psi)))
        return {"T": T, "E": E, "psi": psi}

    def close(self):
        if getattr(self, "h", None):
            self.L.smrt_qmesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
