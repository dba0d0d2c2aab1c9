"""FP64 CPU oracle of the two-phase shallow-flow step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.

``OracleSim`` wraps ``m2p_oracle.c`` (plain C, FP64, compiled with
``-O2 -ffp-contract=off``) over ctypes.  Problems come from
``paper_2104_06784_amd.inputs`` (data only).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "m2p_oracle.c")
_LIB = os.path.join(_HERE, "libm2p_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("delta_b_deg", C.c_double), ("c_d", C.c_double), ("inv_n_r", C.c_double),
                ("theta_b", C.c_double), ("rho_s", C.c_double), ("rho_f", C.c_double),
                ("cfl", C.c_double), ("L", C.c_double), ("H", C.c_double), ("chi", C.c_double),
                ("g", C.c_double), ("m_dry", C.c_double), ("a_min", C.c_double),
                ("bc", C.c_int32 * 4), ("flags", C.c_int32), ("delta_int_deg", C.c_double),
                ("v_eps", C.c_double)]


class _InflowState(C.Structure):
    _fields_ = [("side", C.c_int32), ("i0", C.c_int32), ("ncells", C.c_int32), ("nt", C.c_int32),
                ("t", C.POINTER(C.c_double)), ("h", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double))]


class _Inflow(C.Structure):
    _fields_ = [("side", C.c_int32), ("i0", C.c_int32), ("ncells", C.c_int32), ("nt", C.c_int32),
                ("t", C.POINTER(C.c_double)), ("Q", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        lib.ora_create.restype = P
        lib.ora_create.argtypes = [C.POINTER(_Params), dp, dp]
        lib.ora_destroy.argtypes = [P]
        lib.ora_set_state_si.restype = C.c_int
        lib.ora_set_state_si.argtypes = [P, C.c_int, dp, dp, dp, dp, dp, dp]
        lib.ora_set_state_raw.argtypes = [P, dp]
        lib.ora_get_state_raw.argtypes = [P, dp]
        lib.ora_set_time.argtypes = [P, C.c_double]
        lib.ora_set_inflow.restype = C.c_int
        lib.ora_set_inflow.argtypes = [P, C.POINTER(_Inflow), C.c_int]
        lib.ora_set_inflow_states.restype = C.c_int
        lib.ora_set_inflow_states.argtypes = [P, C.POINTER(_InflowState), C.c_int]
        lib.ora_step.restype = C.c_double
        lib.ora_step.argtypes = [P, C.c_double]
        lib.ora_run.restype = C.c_int64
        lib.ora_run.argtypes = [P, C.c_int64, C.c_double, dp]
        lib.ora_peek_dt.restype = C.c_double
        lib.ora_peek_dt.argtypes = [P, C.c_double]
        lib.ora_diag.argtypes = [P, dp]
        lib.ora_get_fields.argtypes = [P, dp, dp, dp, dp, dp, dp]
        lib.ora_probe.argtypes = [P, C.c_int, C.c_int, dp]
        lib.ora_stage_probe.argtypes = [P, C.c_double, dp]
        lib.ora_cbrt_nearest.restype = C.c_double
        lib.ora_cbrt_nearest.argtypes = [C.c_double]
        lib.ora_scales.argtypes = [P, dp]
        lib.ora_set_dt_schedule.argtypes = [P, dp, C.c_int64]
        lib.ora_set_threads.restype = C.c_int
        lib.ora_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def cbrt_nearest(x: float) -> float:
    """The oracle's cube root of the critical depth (test probe)."""
    return _load().ora_cbrt_nearest(float(x))


def set_threads(n: int) -> int:
    return _load().ora_set_threads(n)


class OracleSim:
    """One scenario on the CPU oracle.  State arrays are float64 [6, ny, nx] in
    the order (m^s, p^s_X, p^s_Y, m^f, p^f_X, p^f_Y), dimensionless."""

    def __init__(self, prob, params=None):
        lib = _load()
        p = prob.params if params is None else params
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        cp = _Params(prob.nx, prob.ny, prob.dx, prob.dy, p.delta_b_deg, p.c_d, p.inv_n_r, p.theta_b,
                     p.rho_s, p.rho_f, p.cfl, p.L, p.H, p.chi, p.g, p.m_dry, p.a_min,
                     (C.c_int32 * 4)(*p.bc), p.flags, p.delta_int_deg, p.v_eps)
        dem = np.ascontiguousarray(prob.dem, dtype=np.float64)
        mu = None if prob.tan_mu is None else np.ascontiguousarray(prob.tan_mu, dtype=np.float64)
        self._h = lib.ora_create(C.byref(cp), _ptr(dem), _ptr(mu))
        if not self._h:
            raise ValueError("oracle rejected the grid")
        self._keep = []
        self.set_state_si(prob.h_vert, prob.phi_s, vertical=True, vel=prob.vel)
        if prob.inflows:
            self.set_inflow(prob.inflows)
        if prob.inflow_states:
            self.set_inflow_states(prob.inflow_states)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().ora_destroy(h)
            self._h = None

    def set_state_si(self, h, phi_s, vertical=True, vel=None):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (h, phi_s)]
        v = [None] * 4 if vel is None else [np.ascontiguousarray(x, dtype=np.float64) for x in vel]
        rc = _load().ora_set_state_si(self._h, 1 if vertical else 0, _ptr(a[0]), _ptr(a[1]),
                                      *[_ptr(x) for x in v])
        if rc != 0:
            raise ValueError("invalid state")

    def set_inflow(self, inflows):
        arr = (_Inflow * len(inflows))()
        for k, s in enumerate(inflows):
            t = np.ascontiguousarray(s.t, dtype=np.float64)
            Q = np.ascontiguousarray(s.Q, dtype=np.float64)
            ph = np.ascontiguousarray(s.phi_s, dtype=np.float64)
            self._keep += [t, Q, ph]
            arr[k] = _Inflow(s.side, s.i0, s.ncells, len(t), _ptr(t), _ptr(Q), _ptr(ph))
        if _load().ora_set_inflow(self._h, arr, len(inflows)) != 0:
            raise ValueError("invalid inflow")

    def set_inflow_states(self, segs):
        arr = (_InflowState * max(len(segs), 1))()
        for k, s in enumerate(segs):
            a = [np.ascontiguousarray(x, dtype=np.float64) for x in (s.t, s.h, s.phi_s, s.v)]
            self._keep += a
            arr[k] = _InflowState(s.side, s.i0, s.ncells, len(a[0]), *[_ptr(x) for x in a])
        if _load().ora_set_inflow_states(self._h, arr, len(segs)) != 0:
            raise ValueError("invalid inflow state segment")

    def state(self) -> np.ndarray:
        U = np.empty((6, self.ny, self.nx), dtype=np.float64)
        _load().ora_get_state_raw(self._h, _ptr(U))
        return U

    def set_state_raw(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (6, self.ny, self.nx)
        _load().ora_set_state_raw(self._h, _ptr(U))

    def set_time(self, t):
        _load().ora_set_time(self._h, float(t))

    def step(self, t_end=float("inf")) -> float:
        return _load().ora_step(self._h, t_end)

    def run(self, nsteps, t_end=float("inf")):
        dts = np.zeros(int(nsteps), dtype=np.float64)
        n = _load().ora_run(self._h, int(nsteps), t_end, _ptr(dts))
        return dts[:n]

    def set_dt_schedule(self, dts):
        d = np.ascontiguousarray(dts, dtype=np.float64)
        self._keep.append(d)
        _load().ora_set_dt_schedule(self._h, _ptr(d), len(d))

    def peek_dt(self, t_end=float("inf")) -> float:
        return _load().ora_peek_dt(self._h, t_end)

    def diag(self) -> dict:
        d = np.zeros(10)
        _load().ora_diag(self._h, _ptr(d))
        keys = ["t", "steps", "mass_s", "mass_f", "in_s", "in_f", "out_s", "out_f", "clamps", "dt_last"]
        return dict(zip(keys, d.tolist()))

    def fields(self) -> dict:
        out = {k: np.empty((self.ny, self.nx)) for k in ("h", "phi_s", "vxs", "vys", "vxf", "vyf")}
        _load().ora_get_fields(self._h, *[_ptr(out[k]) for k in ("h", "phi_s", "vxs", "vys", "vxf", "vyf")])
        return out

    def probe(self, i, j) -> np.ndarray:
        out = np.zeros(34)
        _load().ora_probe(self._h, int(i), int(j), _ptr(out))
        return out

    def stage_probe(self, dt) -> np.ndarray:
        """One forward-Euler stage E(U) of the current state with step dt (s),
        raw layout [6, ny, nx]; the simulation itself does not advance."""
        E = np.empty((6, self.ny, self.nx), dtype=np.float64)
        _load().ora_stage_probe(self._h, float(dt), _ptr(E))
        return E

    def scales(self) -> dict:
        out = np.zeros(7)
        _load().ora_scales(self._h, _ptr(out))
        return dict(zip(["eps", "alpha", "T", "V", "dxi", "deta", "md"], out.tolist()))
