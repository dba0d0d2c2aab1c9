"""Python wrapper of one scenario context (argument marshalling over the C ABI).

``Sim`` owns an ``m2p_ctx``.  PyTorch, when given, supplies only device memory
(``buffers=``: two tensors that become the state buffers through
``m2p_bind_buffers``) and the HIP stream; the step itself runs in ``libm2p.so``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi as A


def make_params(p) -> A.Params:
    return A.Params(p.delta_b_deg, p.c_d, p.inv_n_r, p.theta_b, p.rho_s, p.rho_f, p.delta_int_deg, p.cfl,
                    p.L, p.H, p.chi, p.g, p.m_dry, p.a_min, (C.c_int32 * 4)(*p.bc), p.flags, p.v_eps)


class Sim:
    """One scenario on the GPU.

    ``prob`` is an ``inputs.Problem``; ``precision`` "f64" or "f32" (default:
    the problem's).  ``stream`` is an optional ``torch.cuda.Stream``.
    ``buffers`` is an optional pair of contiguous CUDA tensors, each at least
    ``Sim.buffer_bytes`` long and 256-byte aligned, that hold the two state
    buffers instead of context-owned memory (they must outlive the Sim; the
    current state U^n is in the first after every step, [6][ny][pitch] in the
    context precision).
    """

    FIELDS = ("h", "phi_s", "vxs", "vys", "vxf", "vyf")

    def __init__(self, prob, precision=None, stream=None, params=None, variant=A.M2P_VARIANT_AUTO,
                 tile_rows=0, set_state=True, buffers=None):
        L = A.lib()
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        prec = precision or prob.precision
        self.prec = A.M2P_FP64 if prec == "f64" else A.M2P_FP32
        self._grid = A.Grid(prob.nx, prob.ny, prob.dx, prob.dy)
        self._params = make_params(prob.params if params is None else params)
        dem = np.ascontiguousarray(prob.dem, dtype=np.float64)
        mu = None if prob.tan_mu is None else np.ascontiguousarray(prob.tan_mu, dtype=np.float64)
        sp = None if stream is None else C.c_void_p(stream.cuda_stream)
        h = C.c_void_p()
        A.check(L.m2p_create(C.byref(h), C.byref(self._grid), C.byref(self._params), self.prec,
                             A.dptr(dem), A.dptr(mu), sp), "m2p_create")
        self._h = h
        self._keep = []
        if variant != A.M2P_VARIANT_AUTO or tile_rows:
            self.set_variant(variant, tile_rows)
        if buffers is not None:
            self.bind_buffers(*buffers)
        if set_state:
            self.set_state(prob.h_vert, prob.phi_s, vertical=True, vel=prob.vel)
            if prob.inflows:
                self.set_inflow(prob.inflows)
            if prob.inflow_states:
                self.set_inflow_states(prob.inflow_states)

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            A.lib().m2p_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # -- set-up
    @staticmethod
    def buffer_bytes(nx, ny, precision="f64") -> int:
        """Bytes of one state buffer (6 fields of ny rows of nx rounded up to 64)."""
        out = C.c_size_t()
        g = A.Grid(int(nx), int(ny), 1.0, 1.0)
        prec = A.M2P_FP64 if precision == "f64" else A.M2P_FP32
        A.check(A.lib().m2p_buffer_bytes(C.byref(g), prec, C.byref(out)), "m2p_buffer_bytes")
        return out.value

    def bind_buffers(self, a, b):
        """Make two caller-owned device tensors the state buffers (m2p_bind_buffers)."""
        need = self.buffer_bytes(self.nx, self.ny, "f64" if self.prec == A.M2P_FP64 else "f32")
        for t in (a, b):
            if not (t.is_cuda and t.is_contiguous()):
                raise ValueError("state buffers must be contiguous device tensors")
            if t.numel() * t.element_size() < need:
                raise ValueError(f"state buffer of {t.numel() * t.element_size()} bytes, {need} needed")
        A.check(A.lib().m2p_bind_buffers(self._h, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), need),
                "m2p_bind_buffers")
        self._keep += [a, b]

    def set_variant(self, variant, tile_rows=0):
        A.check(A.lib().m2p_set_variant(self._h, variant, tile_rows), "m2p_set_variant")

    def set_state(self, h, phi_s, vertical=True, vel=None):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (h, phi_s)]
        v = [None] * 4 if vel is None else [np.ascontiguousarray(x, dtype=np.float64) for x in vel]
        kind = A.M2P_DEPTH_VERTICAL if vertical else A.M2P_DEPTH_NORMAL
        A.check(A.lib().m2p_set_state(self._h, kind, A.dptr(a[0]), A.dptr(a[1]), *[A.dptr(x) for x in v]),
                "m2p_set_state")

    def set_state_raw(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (6, self.ny, self.nx)
        A.check(A.lib().m2p_set_state_raw(self._h, A.dptr(U)), "m2p_set_state_raw")

    def set_time(self, t):
        A.check(A.lib().m2p_set_time(self._h, float(t)), "m2p_set_time")

    def set_inflow(self, inflows):
        arr = (A.Inflow * max(1, len(inflows)))()
        for k, s in enumerate(inflows):
            t = np.ascontiguousarray(s.t, dtype=np.float64)
            Q = np.ascontiguousarray(s.Q, dtype=np.float64)
            ph = np.ascontiguousarray(s.phi_s, dtype=np.float64)
            self._keep += [t, Q, ph]
            arr[k] = A.Inflow(s.side, s.i0, s.ncells, len(t), A.dptr(t), A.dptr(Q), A.dptr(ph))
        A.check(A.lib().m2p_set_inflow(self._h, arr, len(inflows)), "m2p_set_inflow")

    def set_inflow_states(self, segs):
        """Mode-II segments given as hydrographs of the inflowing state
        (``inputs.InflowState``: h in m, phi_s, inward speed v in m/s)."""
        arr = (A.InflowState * max(1, len(segs)))()
        for k, s in enumerate(segs):
            a = [np.ascontiguousarray(x, dtype=np.float64) for x in (s.t, s.h, s.phi_s, s.v)]
            self._keep += a
            arr[k] = A.InflowState(s.side, s.i0, s.ncells, len(a[0]), *[A.dptr(x) for x in a])
        A.check(A.lib().m2p_set_inflow_states(self._h, arr, len(segs)), "m2p_set_inflow_states")

    def autotune(self, trial_steps: int = 10):
        """Time a few tile heights on this context (state restored after each
        trial) and keep the fastest; returns (rows, ms per step)."""
        r = C.c_int32()
        ms = C.c_double()
        A.check(A.lib().m2p_autotune(self._h, int(trial_steps), C.byref(r), C.byref(ms)), "m2p_autotune")
        return r.value, ms.value

    # -- stepping
    def step(self) -> float:
        dt = C.c_double()
        A.check(A.lib().m2p_step(self._h, C.byref(dt)), "m2p_step")
        return dt.value

    def run(self, nsteps: int):
        A.check(A.lib().m2p_run(self._h, int(nsteps)), "m2p_run")

    def run_to(self, t_end: float, max_steps: int = 10 ** 9) -> int:
        n = C.c_int64()
        A.check(A.lib().m2p_run_to(self._h, float(t_end), int(max_steps), C.byref(n)), "m2p_run_to")
        return n.value

    def set_graph(self, chunk: int):
        """Steps per replayed HIP graph (0: kernel-by-kernel launches)."""
        A.check(A.lib().m2p_set_graph(self._h, int(chunk)), "m2p_set_graph")

    def run_outputs(self, times, max_steps: int = 10 ** 9):
        """Run through the output times (s); returns ([n, 6, ny, nx] fields
        h, phi_s, vxs, vys, vxf, vyf at each time, steps taken).  Snapshots
        are copied to the host while the next interval runs."""
        t = np.ascontiguousarray(times, dtype=np.float64)
        out = np.empty((len(t), 6, self.ny, self.nx), dtype=np.float64)
        n = C.c_int64()
        A.check(A.lib().m2p_run_outputs(self._h, A.dptr(t), len(t), int(max_steps), A.dptr(out), C.byref(n)),
                "m2p_run_outputs")
        return out, n.value

    def synchronize(self):
        A.check(A.lib().m2p_synchronize(self._h), "m2p_synchronize")

    # -- results
    def state(self) -> np.ndarray:
        U = np.empty((6, self.ny, self.nx), dtype=np.float64)
        A.check(A.lib().m2p_get_state_raw(self._h, A.dptr(U)), "m2p_get_state_raw")
        return U

    def fields(self) -> dict:
        out = {k: np.empty((self.ny, self.nx), dtype=np.float64) for k in self.FIELDS}
        A.check(A.lib().m2p_get_fields(self._h, *[A.dptr(out[k]) for k in self.FIELDS]), "m2p_get_fields")
        return out

    def diag(self) -> dict:
        d = A.Diag()
        A.check(A.lib().m2p_get_diag(self._h, C.byref(d)), "m2p_get_diag")
        return {k: getattr(d, k) for k, _ in A.Diag._fields_ if k != "pad"}

    def set_profiling(self, on: bool):
        A.check(A.lib().m2p_set_profiling(self._h, 1 if on else 0), "m2p_set_profiling")

    def kernel_times(self):
        """(ms of stage 1, stage 2, finalize summed over the timed steps, steps)."""
        ms = (C.c_double * 3)()
        n = C.c_int64()
        A.check(A.lib().m2p_kernel_times(self._h, ms, C.byref(n)), "m2p_kernel_times")
        return list(ms), n.value

    # -- gradients
    def set_friction_field(self, tan_mu):
        m = np.ascontiguousarray(tan_mu, dtype=np.float64)
        A.check(A.lib().m2p_set_friction_field(self._h, A.dptr(m)), "m2p_set_friction_field")

    def set_dt_schedule(self, dts):
        d = np.ascontiguousarray(dts, dtype=np.float64)
        A.check(A.lib().m2p_set_dt_schedule(self._h, A.dptr(d) if len(d) else None, len(d)),
                "m2p_set_dt_schedule")

    def loss(self, target_h) -> float:
        t = np.ascontiguousarray(target_h, dtype=np.float64)
        out = C.c_double()
        A.check(A.lib().m2p_loss(self._h, A.dptr(t), C.byref(out)), "m2p_loss")
        return out.value

    def stage_jvp(self, dU, dmu=None, stage=0):
        dU = np.ascontiguousarray(dU, dtype=np.float64)
        dm = None if dmu is None else np.ascontiguousarray(dmu, dtype=np.float64)
        E = np.empty_like(dU)
        dE = np.empty_like(dU)
        A.check(A.lib().m2p_stage_jvp(self._h, stage, A.dptr(dU), A.dptr(dm), A.dptr(E), A.dptr(dE)),
                "m2p_stage_jvp")
        return E, dE

    def stage_vjp(self, lam, stage=0):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        li = np.empty_like(lam)
        gmu = np.empty((self.ny, self.nx), dtype=np.float64)
        A.check(A.lib().m2p_stage_vjp(self._h, stage, A.dptr(lam), A.dptr(li), A.dptr(gmu)), "m2p_stage_vjp")
        return li, gmu

    def adjoint_run(self, nsteps, ckpt_every, target_h, vol_scale=1.0):
        """Loss, dL/dmu (per cell) and dL/d(volume scale) of an nsteps run."""
        t = np.ascontiguousarray(target_h, dtype=np.float64)
        loss, gv = C.c_double(), C.c_double()
        gmu = np.empty((self.ny, self.nx), dtype=np.float64)
        A.check(A.lib().m2p_adjoint_run(self._h, int(nsteps), int(ckpt_every), A.dptr(t), float(vol_scale),
                                        C.byref(loss), A.dptr(gmu), C.byref(gv)), "m2p_adjoint_run")
        return loss.value, gmu, gv.value

    def device_ptr(self):
        p, pitch = C.c_void_p(), C.c_int64()
        A.check(A.lib().m2p_state_device_ptr(self._h, C.byref(p), C.byref(pitch)), "m2p_state_device_ptr")
        return p.value, pitch.value


class Batch:
    """Ensemble of independent scenarios advanced together (``m2p_batch_*``).

    ``probs`` is a list of ``inputs.Problem`` (Mode-I); all share one precision.
    """

    def __init__(self, probs, precision="f32", stream=None, set_state=True):
        L = A.lib()
        self.probs = list(probs)
        n = len(self.probs)
        self.prec = A.M2P_FP64 if precision == "f64" else A.M2P_FP32
        grids = (A.Grid * n)(*[A.Grid(p.nx, p.ny, p.dx, p.dy) for p in self.probs])
        params = (A.Params * n)(*[make_params(p.params) for p in self.probs])
        self._dems = [np.ascontiguousarray(p.dem, dtype=np.float64) for p in self.probs]
        self._mus = [None if p.tan_mu is None else np.ascontiguousarray(p.tan_mu, dtype=np.float64)
                     for p in self.probs]
        dem_ptrs = (A._dp * n)(*[A.dptr(d) for d in self._dems])
        mu_ptrs = None
        if any(m is not None for m in self._mus):
            mu_ptrs = (A._dp * n)(*[A.dptr(m) if m is not None else A._dp() for m in self._mus])
        sp = None if stream is None else C.c_void_p(stream.cuda_stream)
        h = C.c_void_p()
        A.check(L.m2p_batch_create(C.byref(h), n, grids, params, dem_ptrs, mu_ptrs, self.prec, sp),
                "m2p_batch_create")
        self._h = h
        if set_state:
            for i, p in enumerate(self.probs):
                self.set_state(i, p.h_vert, p.phi_s, vertical=True, vel=p.vel)

    def close(self):
        if getattr(self, "_h", None):
            A.lib().m2p_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_state(self, i, h, phi_s, vertical=True, vel=None):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (h, phi_s)]
        v = [None] * 4 if vel is None else [np.ascontiguousarray(x, dtype=np.float64) for x in vel]
        kind = A.M2P_DEPTH_VERTICAL if vertical else A.M2P_DEPTH_NORMAL
        A.check(A.lib().m2p_batch_set_state(self._h, i, kind, A.dptr(a[0]), A.dptr(a[1]),
                                            *[A.dptr(x) for x in v]), "m2p_batch_set_state")

    def run(self, nsteps):
        A.check(A.lib().m2p_batch_run(self._h, int(nsteps)), "m2p_batch_run")

    def synchronize(self):
        A.check(A.lib().m2p_batch_synchronize(self._h), "m2p_batch_synchronize")

    def state(self, i):
        p = self.probs[i]
        U = np.empty((6, p.ny, p.nx), dtype=np.float64)
        A.check(A.lib().m2p_batch_get_state_raw(self._h, i, A.dptr(U)), "m2p_batch_get_state_raw")
        return U

    def fields(self, i):
        p = self.probs[i]
        out = {k: np.empty((p.ny, p.nx), dtype=np.float64) for k in Sim.FIELDS}
        A.check(A.lib().m2p_batch_get_fields(self._h, i, *[A.dptr(out[k]) for k in Sim.FIELDS]),
                "m2p_batch_get_fields")
        return out

    def diag(self, i):
        d = A.Diag()
        A.check(A.lib().m2p_batch_get_diag(self._h, i, C.byref(d)), "m2p_batch_get_diag")
        return {k: getattr(d, k) for k, _ in A.Diag._fields_ if k != "pad"}

    def set_tile(self, rows, blocks=0):
        A.check(A.lib().m2p_batch_set_tile(self._h, int(rows), int(blocks)), "m2p_batch_set_tile")

    def set_graph(self, chunk):
        A.check(A.lib().m2p_batch_set_graph(self._h, int(chunk)), "m2p_batch_set_graph")

    def autotune(self, trial_steps=5):
        r, b, ms = C.c_int32(), C.c_int32(), C.c_double()
        A.check(A.lib().m2p_batch_autotune(self._h, int(trial_steps), C.byref(r), C.byref(b), C.byref(ms)),
                "m2p_batch_autotune")
        return r.value, b.value, ms.value

    def info(self):
        n, c, r, b, w = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        A.check(A.lib().m2p_batch_info(self._h, C.byref(n), C.byref(c), C.byref(r), C.byref(b), C.byref(w)),
                "m2p_batch_info")
        return {"nscen": n.value, "cells": c.value, "rows": r.value, "blocks": b.value, "work": w.value}
