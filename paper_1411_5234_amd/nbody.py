"""Python front end of the HIP hot path: device state, context and block-step driver.

torch provides device memory and streams; every computation is a call into
libnbody.so through the C ABI (`_lib`).  Names follow include/nbody.h.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import (FIELDS32, FIELDS64, H6_FIELDS32, H6_FIELDS64, NbBatchItem, NbError,
                   NbHermite6, NbSystem, PRECISIONS)


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


class System:
    """One system of n bodies held in HBM as structure-of-arrays FP64 rows.

    buf64 rows follow FIELDS64 (x, y, z, vx, ..., dt, xp, ..., vzp); buf32 rows follow
    FIELDS32 (FP32 copies of the predicted velocities and the masses, used by the
    mixed-precision force).  Two allocations per system keep the footprint at
    21 * 8 + 4 * 4 = 184 bytes per body.
    """

    BYTES_PER_BODY = 8 * len(FIELDS64) + 4 * len(FIELDS32)

    def __init__(self, n: int, device: torch.device | str = "cuda", fp32_copies: bool = True,
                 buf64: torch.Tensor | None = None, buf32: torch.Tensor | None = None):
        self.n = int(n)
        self.device = torch.device(device)
        self.buf64 = buf64 if buf64 is not None else torch.zeros(
            (len(FIELDS64), max(self.n, 1)), dtype=torch.float64, device=self.device)
        if fp32_copies:
            self.buf32 = buf32 if buf32 is not None else torch.zeros(
                (len(FIELDS32), max(self.n, 1)), dtype=torch.float32, device=self.device)
        else:
            self.buf32 = None
        self._struct = NbSystem()
        self._struct.n = self.n
        for k, f in enumerate(FIELDS64):
            setattr(self._struct, f, self.buf64[k].data_ptr())
        for k, f in enumerate(FIELDS32):
            setattr(self._struct, f, self.buf32[k].data_ptr() if self.buf32 is not None else None)

    def row(self, name: str) -> torch.Tensor:
        if name in FIELDS64:
            return self.buf64[FIELDS64.index(name)][: self.n]
        return self.buf32[FIELDS32.index(name)][: self.n]

    @property
    def ref(self):
        return C.byref(self._struct)

    @classmethod
    def from_arrays(cls, x, v, m, device="cuda", fp32_copies=True) -> "System":
        x = np.asarray(x, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        m = np.asarray(m, dtype=np.float64)
        s = cls(m.shape[0], device, fp32_copies)
        # staged in pinned host memory (pageable copies go through a slow bounce
        # path); torch's pinned-block cache keeps the block until the copy is done
        pinned = s.buf64.is_cuda
        host = torch.empty((len(FIELDS64), max(s.n, 1)), dtype=torch.float64, pin_memory=pinned)
        h = host.numpy()
        h[:] = 0.0
        if s.n:
            h[0:3, : s.n] = x.T
            h[3:6, : s.n] = v.T
            h[12, : s.n] = m
            # the predicted set starts equal to the state (t = 0, nothing to extrapolate)
            h[15:18, : s.n] = h[0:3, : s.n]
            h[18:21, : s.n] = h[3:6, : s.n]
        s.buf64.copy_(host, non_blocking=pinned)
        if s.buf32 is not None:
            s.buf32[0:3].copy_(s.buf64[18:21].float())
            s.buf32[3].copy_(s.buf64[12].float())
        return s

    def state_numpy(self) -> dict:
        """Copy the FP64 state back as numpy: x, v, a, j (n, 3); m, t, dt (n,)."""
        if self.buf64.is_cuda:
            pin = torch.empty((self.buf64.shape[0], self.n), dtype=torch.float64, pin_memory=True)
            pin.copy_(self.buf64[:, : self.n])          # synchronous: pin is filled on return
            h = pin.numpy()
        else:
            h = self.buf64[:, : self.n].numpy()
        return {"x": h[0:3].T.copy(), "v": h[3:6].T.copy(), "a": h[6:9].T.copy(),
                "j": h[9:12].T.copy(), "m": h[12].copy(), "t": h[13].copy(), "dt": h[14].copy(),
                "xp": h[15:18].T.copy(), "vp": h[18:21].T.copy()}


class Hermite6:
    """The extra device arrays of the 6th-order scheme for one System: snap and
    crackle at the bodies' own times and the predicted acceleration (FP64 rows in
    H6_FIELDS64 order), plus FP32 copies of the predicted acceleration for the
    mixed and double-single forces.  All start at zero."""

    BYTES_PER_BODY = 8 * len(H6_FIELDS64) + 4 * len(H6_FIELDS32)

    def __init__(self, sys: System, fp32_copies: bool = True):
        self.n = sys.n
        n = max(sys.n, 1)
        self.buf64 = torch.zeros((len(H6_FIELDS64), n), dtype=torch.float64, device=sys.device)
        self.buf32 = (torch.zeros((len(H6_FIELDS32), n), dtype=torch.float32, device=sys.device)
                      if fp32_copies else None)
        self._struct = NbHermite6()
        for k, f in enumerate(H6_FIELDS64):
            setattr(self._struct, f, self.buf64[k].data_ptr())
        for k, f in enumerate(H6_FIELDS32):
            setattr(self._struct, f, self.buf32[k].data_ptr() if self.buf32 is not None else None)

    @property
    def ref(self):
        return C.byref(self._struct)

    def state_numpy(self) -> dict:
        """Snap s, crackle c and predicted acceleration ap as numpy (n, 3)."""
        if self.buf64.is_cuda:
            pin = torch.empty((self.buf64.shape[0], self.n), dtype=torch.float64, pin_memory=True)
            pin.copy_(self.buf64[:, : self.n])          # synchronous: pin is filled on return
            h = pin.numpy()
        else:
            h = self.buf64[:, : self.n].numpy()
        return {"s": h[0:3].T.copy(), "c": h[3:6].T.copy(), "ap": h[6:9].T.copy()}


class Context:
    """An nb_ctx bound to one device and one torch (HIP) stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.L = _lib.load()
        self.device = int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.L.nb_ctx_create(C.byref(h), self.device, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise NbError(rc, "nb_ctx_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.nb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            msg = self.L.nb_last_error(self.h)
            raise NbError(rc, msg.decode() if msg else "")

    # ---- entry points (names of include/nbody.h) --------------------------------
    def sync(self):
        self._check(self.L.nb_sync(self.h))

    def select_active(self, sys: System, i_idx: torch.Tensor):
        tn, m = C.c_double(), C.c_int32()
        self._check(self.L.nb_select_active(self.h, sys.ref, C.byref(tn), _ptr(i_idx), C.byref(m)))
        return tn.value, m.value

    def predict(self, sys: System, t_next: float):
        self._check(self.L.nb_predict(self.h, sys.ref, float(t_next)))

    def force_active(self, sys: System, i_idx: torch.Tensor | None, m: int, j0: int, j1: int,
                     eps: float, precision: str, acc: torch.Tensor, jerk: torch.Tensor,
                     plan: tuple | None = None):
        prec = PRECISIONS[precision]
        if acc.numel() < 3 * m or jerk.numel() < 3 * m:
            raise ValueError("acc/jerk need 3*m elements")
        if plan is None:
            rc = self.L.nb_force_active(self.h, sys.ref, _ptr(i_idx), int(m), int(j0), int(j1),
                                        float(eps), prec, _ptr(acc), _ptr(jerk))
        else:
            il, s, b = plan
            rc = self.L.nb_force_active_plan(self.h, sys.ref, _ptr(i_idx), int(m), int(j0),
                                             int(j1), float(eps), prec, int(il), int(s), int(b),
                                             _ptr(acc), _ptr(jerk))
        self._check(rc)

    def force_active_noalloc(self, sys: System, i_idx: torch.Tensor | None, m: int, j0: int,
                             j1: int, eps: float, precision: str, acc: torch.Tensor,
                             jerk: torch.Tensor):
        """nb_force_active_noalloc: the same forces with the library's static scratch."""
        if acc.numel() < 3 * m or jerk.numel() < 3 * m:
            raise ValueError("acc/jerk need 3*m elements")
        self._check(self.L.nb_force_active_noalloc(self.h, sys.ref, _ptr(i_idx), int(m), int(j0),
                                                   int(j1), float(eps), PRECISIONS[precision],
                                                   _ptr(acc), _ptr(jerk)))

    def init_steps(self, sys: System, acc, jerk, eta_s, dt_max, dt_min):
        self._check(self.L.nb_init_steps(self.h, sys.ref, _ptr(acc), _ptr(jerk), float(eta_s),
                                         float(dt_max), float(dt_min)))

    def correct(self, sys: System, i_idx, m, acc, jerk, t_next, eta, dt_max, dt_min):
        self._check(self.L.nb_correct(self.h, sys.ref, _ptr(i_idx), int(m), _ptr(acc), _ptr(jerk),
                                      float(t_next), float(eta), float(dt_max), float(dt_min)))

    # ---- 6th order ------------------------------------------------------------------
    def predict6(self, sys: System, h6: Hermite6, t_next: float):
        self._check(self.L.nb_predict6(self.h, sys.ref, h6.ref, float(t_next)))

    def force6_active(self, sys: System, h6: Hermite6, i_idx: torch.Tensor | None, m: int,
                      j0: int, j1: int, eps: float, precision: str, acc: torch.Tensor,
                      jerk: torch.Tensor, snap: torch.Tensor, plan: tuple | None = None):
        prec = PRECISIONS[precision]
        if min(acc.numel(), jerk.numel(), snap.numel()) < 3 * m:
            raise ValueError("acc/jerk/snap need 3*m elements")
        if plan is None:
            rc = self.L.nb_force6_active(self.h, sys.ref, h6.ref, _ptr(i_idx), int(m), int(j0),
                                         int(j1), float(eps), prec, _ptr(acc), _ptr(jerk),
                                         _ptr(snap))
        else:
            il, s, b = plan
            rc = self.L.nb_force6_active_plan(self.h, sys.ref, h6.ref, _ptr(i_idx), int(m),
                                              int(j0), int(j1), float(eps), prec, int(il), int(s),
                                              int(b), _ptr(acc), _ptr(jerk), _ptr(snap))
        self._check(rc)

    def init_steps6(self, sys: System, h6: Hermite6, acc, jerk, snap, eta_s, dt_max, dt_min):
        self._check(self.L.nb_init_steps6(self.h, sys.ref, h6.ref, _ptr(acc), _ptr(jerk),
                                          _ptr(snap), float(eta_s), float(dt_max), float(dt_min)))

    def correct6(self, sys: System, h6: Hermite6, i_idx, m, acc, jerk, snap, t_next, eta,
                 dt_max, dt_min):
        self._check(self.L.nb_correct6(self.h, sys.ref, h6.ref, _ptr(i_idx), int(m), _ptr(acc),
                                       _ptr(jerk), _ptr(snap), float(t_next), float(eta),
                                       float(dt_max), float(dt_min)))

    def energy(self, sys: System, eps: float):
        k, p = C.c_double(), C.c_double()
        self._check(self.L.nb_energy(self.h, sys.ref, float(eps), C.byref(k), C.byref(p)))
        return k.value, p.value, k.value + p.value


@dataclass
class Params:
    eps: float
    precision: str = "mixed"
    eta: float = 0.02
    eta_s: float = 0.01
    dt_max: float = 2.0 ** -3
    dt_min: float = 2.0 ** -40


class Integrator:
    """Hermite-4 block-step driver (Sec. 2 items 1-2): select, predict, force, correct."""

    NATIVE_STEP = True          # run() may step through nb_step_batch

    def __init__(self, ctx: Context, sys: System, p: Params):
        self.ctx, self.sys, self.p = ctx, sys, p
        n = max(sys.n, 1)
        dev = sys.device
        self.i_idx = torch.zeros(n, dtype=torch.int32, device=dev)
        self.acc = torch.zeros((3, n), dtype=torch.float64, device=dev)
        self.jerk = torch.zeros((3, n), dtype=torch.float64, device=dev)
        self.steps = 0
        self.interactions = 0
        self.t = 0.0

    def _force(self, i_idx, m):
        n = self.sys.n
        acc = self.acc.view(-1)[: 3 * m]
        jerk = self.jerk.view(-1)[: 3 * m]
        self.ctx.force_active(self.sys, i_idx, m, 0, n, self.p.eps, self.p.precision, acc, jerk)
        return acc, jerk

    def startup(self):
        """t = 0: all bodies active; acc/jerk from the initial state; startup steps."""
        n = self.sys.n
        acc, jerk = self._force(None, n)
        self.ctx.init_steps(self.sys, acc, jerk, self.p.eta_s, self.p.dt_max, self.p.dt_min)
        self.interactions += n * n
        self.t = 0.0

    def step(self):
        """One block step; returns (t_next, m)."""
        t_next, m = self.ctx.select_active(self.sys, self.i_idx)
        self._advance(t_next, m)
        return t_next, m

    def _advance(self, t_next, m):
        self.ctx.predict(self.sys, t_next)
        acc, jerk = self._force(self.i_idx, m)
        self.ctx.correct(self.sys, self.i_idx, m, acc, jerk, t_next, self.p.eta, self.p.dt_max,
                         self.p.dt_min)
        self.steps += 1
        self.interactions += m * self.sys.n
        self.t = t_next

    def run(self, t_end: float, log: list | None = None, progress=None):
        """Advance block steps until every body reaches t_end (a multiple of dt_max).

        With log (a list that receives (t_next, active indices) per block) every
        step goes through the separate calls.  Otherwise each step is one native
        call (nb_step_batch on this one system, nb_step6 for the 6th order:
        selection, predictor, force and corrector with the same kernels and
        results).  progress, if given, is called as progress(t, steps) after
        each step."""
        if log is not None or not self.NATIVE_STEP:
            while True:
                t_next, m = self.ctx.select_active(self.sys, self.i_idx)
                if t_next > t_end:
                    break
                if log is not None:
                    log.append((t_next, self.i_idx[:m].cpu().numpy().astype(np.int64)))
                self._advance(t_next, m)
                if progress is not None:
                    progress(self.t, self.steps)
            self.ctx.sync()
            return self.steps, self.interactions
        self._run_native(t_end, progress)
        self.ctx.sync()
        return self.steps, self.interactions

    def _run_native(self, t_end, progress):
        item = NbBatchItem()
        item.sys = self.sys._struct
        item.i_idx = self.i_idx.data_ptr()
        item.acc = self.acc.data_ptr()
        item.jerk = self.jerk.data_ptr()
        item.status = None
        item.eps = float(self.p.eps)
        item.t_end = float(t_end)
        item.startup = 0
        p, n = self.p, self.sys.n
        args = (self.ctx.h, C.byref(item), 1, PRECISIONS[p.precision], float(p.eta),
                float(p.eta_s), float(p.dt_max), float(p.dt_min))
        step = self.ctx.L.nb_step_batch
        while True:
            self.ctx._check(step(*args))
            if item.error:
                raise NbError(item.error, "block step at t = %.17g" % item.t_next)
            if item.done:
                break
            self.steps += 1
            self.interactions += item.m * n
            self.t = item.t_next
            if progress is not None:
                progress(self.t, self.steps)


@dataclass
class Params6(Params):
    """Step parameters of the 6th-order scheme.  Its criterion gives dt = eta/omega
    on a circular orbit where Aarseth's 4th-order one gives sqrt(eta)/omega, so
    eta = 0.14 takes the steps of the 4th-order eta = 0.02 there."""

    eta: float = 0.14


class Integrator6(Integrator):
    """Hermite-6 block-step driver: select, predict to the crackle, force with
    snap, 6th-order correct."""

    NATIVE_STEP = True          # run() may step through nb_step6

    def __init__(self, ctx: Context, sys: System, p: Params6, h6: Hermite6 | None = None):
        super().__init__(ctx, sys, p)
        self.h6 = h6 if h6 is not None else Hermite6(sys, fp32_copies=sys.buf32 is not None)
        self.snap = torch.zeros((3, max(sys.n, 1)), dtype=torch.float64, device=sys.device)

    def _force6(self, i_idx, m):
        n = self.sys.n
        acc = self.acc.view(-1)[: 3 * m]
        jerk = self.jerk.view(-1)[: 3 * m]
        snap = self.snap.view(-1)[: 3 * m]
        self.ctx.force6_active(self.sys, self.h6, i_idx, m, 0, n, self.p.eps, self.p.precision,
                               acc, jerk, snap)
        return acc, jerk, snap

    def startup(self):
        """t = 0, every body active.  A first pass gives the accelerations the
        snap needs (stored as the state by the 4th-order startup, which also sets
        t = 0); the prediction to t = 0 copies them into the predicted
        acceleration; the second pass gives acceleration, jerk and snap."""
        n = self.sys.n
        p = self.p
        acc, jerk = self._force(None, n)
        self.ctx.init_steps(self.sys, acc, jerk, p.eta_s, p.dt_max, p.dt_min)
        self.ctx.predict6(self.sys, self.h6, 0.0)
        acc, jerk, snap = self._force6(None, n)
        self.ctx.init_steps6(self.sys, self.h6, acc, jerk, snap, p.eta_s, p.dt_max, p.dt_min)
        self.interactions += 2 * n * n
        self.t = 0.0

    def _run_native(self, t_end, progress):
        p, n = self.p, self.sys.n
        tn, m, done = C.c_double(), C.c_int32(), C.c_int32()
        args = (self.ctx.h, self.sys.ref, self.h6.ref, self.i_idx.data_ptr(),
                self.acc.data_ptr(), self.jerk.data_ptr(), self.snap.data_ptr(), float(p.eps),
                PRECISIONS[p.precision], float(p.eta), float(p.dt_max), float(p.dt_min),
                float(t_end), C.byref(tn), C.byref(m), C.byref(done))
        step = self.ctx.L.nb_step6
        while True:
            self.ctx._check(step(*args))
            if done.value:
                break
            self.steps += 1
            self.interactions += m.value * n
            self.t = tn.value
            if progress is not None:
                progress(self.t, self.steps)

    def _advance(self, t_next, m):
        p = self.p
        self.ctx.predict6(self.sys, self.h6, t_next)
        acc, jerk, snap = self._force6(self.i_idx, m)
        self.ctx.correct6(self.sys, self.h6, self.i_idx, m, acc, jerk, snap, t_next, p.eta,
                          p.dt_max, p.dt_min)
        self.steps += 1
        self.interactions += m * self.sys.n
        self.t = t_next
