"""Continuous-batching server for ensembles of N-body simulations.

Each request is an initial condition to integrate to t_end with the Hermite
block-step scheme (4th order, or 6th with order=6).  The server keeps every
admitted system's state resident in HBM and advances ALL resident systems
together: one iteration is one block step of every resident system, done by one
native call (nb_step_batch or nb_step6_batch: selection, then one ragged batched
launch per phase for predict, force and correct).  Requests that arrive while
others run are admitted between iterations as slots and device memory free up; a
finished or failed system is retired at once and its memory is released.  A
failing system (non-finite values, a step below dt_min) is reported alone; the
others go on.

Every system is computed with the same kernels, launch plan and arithmetic
whether it runs alone or in a mix (the single-system calls are batches of one),
so its result is bitwise the same in both cases.  The launch plan depends on the
system's own sizes and on the server's lane target (the `lanes` argument), never
on the other systems.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import NbBatchItem, NbError, NbHermite6, NbTidalItem, PRECISIONS
from .groups import PairSet, PairTable
from .nbody import Context, Hermite6, System


@dataclass
class Result:
    rid: int
    n: int
    arrival: float               # seconds after the stream start
    admitted: float
    finished: float
    steps: int = 0
    interactions: int = 0
    energy0: float = float("nan")
    energy1: float = float("nan")
    error: str | None = None
    final: dict | None = None    # final state (when keep_state is set)
    # grouped systems: energy0/1 are the scheme's conserved quantity (reduced system
    # plus the pairs' two-body and tidal energies); these are the full N-body
    # energies of the reconstructed members
    direct0: float = float("nan")
    direct1: float = float("nan")
    pairs: int = 0               # pairs carried as centre-of-mass bodies at admission
    splits: int = 0              # pairs returned to the N-body system during the run
    split_energy: float = 0.0    # change of the conserved quantity at those returns

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def energy_error(self) -> float:
        """Relative error of the conserved quantity (grouped systems: the scheme's,
        with the known change at each pair's return to the N-body system removed)."""
        return abs(self.energy1 - self.split_energy - self.energy0) / abs(self.energy0)


class _Slot:
    """One resident system: device state, work buffers and its batch item."""

    def __init__(self, req, device, precision, now, order=4, L=None, groups=False, pairs=None,
                 snap=None, table=None, ctx=None):
        snap = req.snapshot() if snap is None else snap
        self.req = req
        self.snap = snap
        self.ps = None                     # PairSet of a grouped system
        self.device = device
        if pairs is None and groups:
            pairs = snap.meta.get("pairs")
        if pairs is not None and len(pairs):
            self.ps = PairSet(L, snap.x, snap.v, snap.m, pairs, table, ctx)
            self.n = self.ps.n - self.ps.np
            self.sys = System.from_arrays(self.ps.xr, self.ps.vr, self.ps.mr, device=device,
                                          fp32_copies=(precision != "fp64"))
            self.cm_idx = torch.arange(self.ps.cm0, self.n, dtype=torch.int32, device=device)
        else:
            self.n = snap.n
            self.sys = System.from_arrays(snap.x, snap.v, snap.m, device=device,
                                          fp32_copies=(precision != "fp64"))
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.item = NbBatchItem()
        self._work_buffers()
        self.item.status = self.status.data_ptr()
        self.item.eps = float(req.eps)
        self.item.t_end = float(req.t_end)
        self.item.startup = 1
        if order == 6:
            self.h6 = Hermite6(self.sys, fp32_copies=(precision != "fp64"))
            self.snap6 = torch.zeros(3 * max(self.n, 1), dtype=torch.float64, device=device)
        self.result = Result(req.rid, snap.n, req.arrival, now, float("nan"))
        if self.ps is not None:
            self.result.pairs = self.ps.np

    def _work_buffers(self):
        """Active list and force outputs sized for the system, pointed to by the item."""
        n1 = max(self.n, 1)
        self.i_idx = torch.zeros(n1, dtype=torch.int32, device=self.device)
        self.acc = torch.zeros(3 * n1, dtype=torch.float64, device=self.device)
        self.jerk = torch.zeros(3 * n1, dtype=torch.float64, device=self.device)
        self.item.sys = self.sys._struct
        self.item.i_idx = self.i_idx.data_ptr()
        self.item.acc = self.acc.data_ptr()
        self.item.jerk = self.jerk.data_ptr()


def footprint_bytes(n: int, precision: str = "mixed", order: int = 4) -> int:
    """Device bytes one resident system of n bodies holds (state + work buffers;
    at 6th order also snap, crackle, predicted acceleration and the snap output)."""
    per_body = 8 * 21 + (16 if precision != "fp64" else 0) + 4 + 48
    if order == 6:
        per_body += Hermite6.BYTES_PER_BODY + 24
    return per_body * max(n, 1) + 4 + 1024


class Admission:
    """Admission policy and slot/memory accounting of the server (no device work).

    Requests wait in FIFO order; the head is admitted while a slot is free and its
    footprint fits the budget next to the resident systems.  A request that could
    never fit is refused at submit.  Admission is in arrival order: a large request
    at the head is not overtaken by smaller ones behind it.
    """

    def __init__(self, budget: int, max_slots: int, footprint):
        if max_slots < 1:
            raise ValueError("max_slots must be >= 1")
        self.budget = int(budget)
        self.max_slots = int(max_slots)
        self.footprint = footprint
        self.queue: deque = deque()
        self.resident: dict = {}          # key -> bytes
        self.used = 0

    def submit(self, req):
        if self.footprint(req) > self.budget:
            raise ValueError("request of n=%d does not fit the memory budget" % req.n)
        self.queue.append(req)

    def admit_next(self):
        """Pop and return the next admissible request (or None); reserve its bytes."""
        if not self.queue or len(self.resident) >= self.max_slots:
            return None
        need = self.footprint(self.queue[0])
        if self.used + need > self.budget:
            return None
        req = self.queue.popleft()
        self.resident[id(req)] = need
        self.used += need
        return req

    def release(self, req):
        self.used -= self.resident.pop(id(req))


class Server:
    """Advance many systems together with ragged batched launches.

    precision: "mixed", "ds" or "fp64"; order: 4 or 6 (Hermite order; eta defaults to
    0.02 or 0.14); memory_budget: device bytes for resident systems (default 90% of
    free memory); max_slots: most systems resident at once; lanes: the force plan's
    lane target for every served system (0: the default, with which one system alone
    fills the GPU; a batch fills it together, so a smaller target trades the
    splitting of each system's work for longer lanes).  A system's results depend
    on its own sizes and this setting only, never on the other systems.
    """

    def __init__(self, ctx: Context | None = None, precision: str = "mixed",
                 memory_budget: int | None = None, max_slots: int = 256,
                 eta: float | None = None, eta_s: float = 0.01, dt_max: float = 2.0 ** -3,
                 dt_min: float = 2.0 ** -40, keep_state: bool = False, energy: bool = True,
                 order: int = 4, lanes: int = 0, groups: bool = False, per_period: int = 32,
                 max_sub: int = 1 << 20, group_gamma: float = 1e-3, split_gamma: float = 1e-2):
        if precision not in PRECISIONS:
            raise ValueError(precision)
        if order not in (4, 6):
            raise ValueError("order must be 4 or 6")
        if groups and order != 4:
            raise ValueError("grouped pairs are served at 4th order")
        # groups: requests whose initial condition lists bound pairs carry each pair
        # as one body at its centre of mass; its relative orbit advances on the
        # context's CPU thread (tidal kicks and exact two-body drifts) while the
        # GPU runs the block steps of every resident system
        # -- a pair is carried as one body only while its perturbation gamma (tidal
        # acceleration across its orbit over its own, nb_pairs_perturbation) is
        # small: below group_gamma at admission (wider or more perturbed pairs
        # stay two bodies), and it returns to the N-body system as two bodies when
        # gamma exceeds split_gamma at one of its steps (an approaching perturber)
        self.groups = bool(groups)
        self.per_period, self.max_sub = int(per_period), int(max_sub)
        self.group_gamma, self.split_gamma = float(group_gamma), float(split_gamma)
        self.ptab = PairTable(_lib.load()) if self.groups else None
        self._tid_stale = True
        self._tid_items = None
        self._tid_dev = None
        self._tid_host = None
        self._tid_slots = []
        self._returned = set()
        self.order = order
        _lib.force_plan(1, 1, "mixed", lanes)     # raises on a target out of range
        self.lanes = int(lanes)
        if eta is None:
            eta = 0.14 if order == 6 else 0.02
        self.ctx = ctx if ctx is not None else Context(0)
        self.L = _lib.load()
        self.precision = precision
        self.prec_code = PRECISIONS[precision]
        self.device = torch.device("cuda", self.ctx.device)
        if memory_budget is None:
            free, _ = torch.cuda.mem_get_info(self.ctx.device)
            memory_budget = int(0.9 * free)
        self.adm = Admission(memory_budget, max_slots,
                             lambda r: footprint_bytes(r.n, self.precision, self.order))
        self.eta, self.eta_s, self.dt_max, self.dt_min = eta, eta_s, dt_max, dt_min
        self.keep_state = keep_state
        self.energy = energy
        self.slots: list[_Slot] = []
        self.results: list[Result] = []
        self.iterations = 0
        self.t0 = None
        # the resident systems' batch items, one contiguous array handed to every
        # nb_step_batch call and updated in place by it; rebuilt only when the set
        # of resident systems changes.  _view reads its host fields with numpy.
        self._arr = None
        self._view = None
        self._n = None
        self._steps = None
        self._inter = None

    # ---- admission -----------------------------------------------------------
    @property
    def budget(self):
        return self.adm.budget

    @property
    def used(self):
        return self.adm.used

    @property
    def queue(self):
        return self.adm.queue

    def submit(self, req):
        if req.t_end / self.dt_max != math.floor(req.t_end / self.dt_max):
            raise ValueError("t_end must be a multiple of dt_max")
        self.adm.submit(req)

    def _now(self):
        return time.perf_counter() - self.t0

    def _admit(self):
        while True:
            req = self.adm.admit_next()
            if req is None:
                return
            slot = _Slot(req, self.device, self.precision, self._now(), self.order, self.L,
                         self.groups, table=self.ptab, ctx=self.ctx)
            if slot.ps is not None:
                self._pairs_startup(slot)
                gamma = slot.ps.perturbation()
                if np.any(gamma >= self.group_gamma):
                    slot.ps.release()
                    slot = _Slot(req, self.device, self.precision, slot.result.admitted,
                                 self.order, self.L, True, slot.ps.pairs[gamma < self.group_gamma],
                                 slot.snap, self.ptab, self.ctx)
                    if slot.ps is not None:
                        self._pairs_startup(slot)
            slot.item.lanes = self.lanes
            if self.energy:
                slot.result.energy0 = self.ctx.energy(slot.sys, req.eps)[2]
                if slot.ps is not None:
                    slot.result.energy0 += slot.ps.energy()
                    slot.result.direct0 = self._direct_energy(slot, slot.snap.x, slot.snap.v)
            self._sync_items()
            self.slots.append(slot)
            self._arr = None
            self._tid_stale = True

    # ---- grouped pairs -----------------------------------------------------------
    def _pairs_startup(self, slot):
        """The tidal tensor at every pair's centre of mass at t = 0 (the predicted set
        of a new system is its initial state)."""
        ps = slot.ps
        T = torch.zeros(9 * ps.np, dtype=torch.float64, device=self.device)
        self._check(self.L.nb_tidal_active(self.ctx.h, slot.sys.ref, slot.cm_idx.data_ptr(), ps.np,
                                           0, slot.n, float(slot.req.eps), T.data_ptr()))
        self.ctx.sync()
        ps.T[: ps.np] = T.cpu().numpy().reshape(9, ps.np).T
        ps.tpair[:] = 0.0

    def _direct_energy(self, slot, x, v):
        """Full N-body energy of the members (a temporary system on the device)."""
        full = System.from_arrays(x, v, slot.snap.m, device=self.device, fp32_copies=False)
        return self.ctx.energy(full, slot.req.eps)[2]

    def _grouped(self):
        return [sl for sl in self.slots if sl.ps is not None]

    def _queue_pairs(self, stepped):
        """Queue the advance of every grouped system's pairs that were in its last
        block, all systems in one pass and one queued call: their tensors and times
        reached the pinned host buffers before the selection's host sync of this
        iteration.  A pair whose perturbation has grown past split_gamma returns to
        the N-body system instead (only in a system that took a block step in this
        iteration, `stepped`: slot -> its block time).  Returns {slot: message} of
        systems whose pair return failed."""
        tab = self.ptab
        live = set(id(ps) for ps in tab.sets)
        sets = [(sl, sl.ps) for sl in self._tid_slots
                if sl.ps is not None and id(sl.ps) in live and sl.ps.np and sl in self.slots]
        if self._tid_host is None or not sets:
            return {}
        k = np.array([ps.np for _, ps in sets], dtype=np.int64)
        tot = int(k.sum())
        local = np.arange(tot) - np.repeat(np.cumsum(k) - k, k)
        rows = np.repeat([ps.base for _, ps in sets], k) + local        # table rows
        tid = np.repeat([ps.tid_base for _, ps in sets], k)             # their tidal offsets
        owner = np.repeat(np.arange(len(sets)), k)
        pt = tab.prev_t[rows]
        tcm = self._tcm_host.numpy()[tid + local]
        due = np.flatnonzero((tcm == pt) & (tab.tpair[rows] < pt))
        if not due.size:
            return {}
        r, o, t_b = rows[due], owner[due], pt[due]
        # tensor component c of pair `local` of a system at 9 tid_base + c np + local
        gi = (9 * tid[due] + local[due])[:, None] + np.arange(9)[None, :] * k[o][:, None]
        Tn = self._tid_host.numpy()[gi]
        out = np.zeros(due.size, dtype=bool)
        if self.split_gamma > 0:
            may = np.array([sl in stepped for sl, _ in sets])[o]
            if np.any(may):
                out[may] = tab.perturbation(r[may], Tn[may]) > self.split_gamma
        adv = ~out
        if np.any(adv):
            ra = r[adv]
            H = t_b[adv] - tab.tpair[ra]
            T0 = tab.T[ra].copy()
            tab.T[ra] = Tn[adv]
            tab.tpair[ra] = t_b[adv]
            tab.advance(self.ctx, ra, H, T0, Tn[adv], self.per_period, self.max_sub)
        failed = {}
        for q in np.unique(o[out]):
            sl, ps = sets[q]
            sel = out & (o == q)
            try:
                self._split(sl, r[sel] - ps.base, Tn[sel], float(t_b[sel][0]), stepped[sl])
            except (NbError, ValueError) as e:
                failed[sl] = "pair return failed: %s" % e
        return failed

    def _split(self, sl, ks, Tk, t_prev, t_now):
        """Return pairs ks of a grouped system to the N-body system as two bodies at
        the system's current block time t_now.  Their orbits advance to their last
        block t_prev (tensor Tk there), then to t_now with the tensor at t_now; each pair's
        centre of mass at t_now (its corrected state if it was in this block, else
        its prediction) is replaced by the two members; their accelerations and
        jerks come from the predicted set at t_now and their steps from the startup
        rule, capped by the centre of mass's step and by the largest power of two
        dividing t_now.  The rest of the system keeps its state."""
        ps, ctx = sl.ps, self.ctx
        eps = float(sl.req.eps)
        ps.drain(ctx)
        ps.advance(ctx, ks, t_prev, Tk, self.per_period, self.max_sub, queue=False)
        cm_rows = ps.cm0 + ks
        T = torch.zeros(9 * ks.size, dtype=torch.float64, device=self.device)
        rows_dev = torch.as_tensor(cm_rows.astype(np.int32), device=self.device)
        self._check(self.L.nb_tidal_active(ctx.h, sl.sys.ref, rows_dev.data_ptr(), ks.size, 0,
                                           sl.n, eps, T.data_ptr()))
        ctx.sync()
        Tnow = T.cpu().numpy().reshape(9, ks.size).T.copy()
        later = ps.tpair[ks] < t_now
        if np.any(later):
            ps.advance(ctx, ks[later], t_now, Tnow[later], self.per_period, self.max_sub,
                       queue=False)
        st = sl.sys.state_numpy()
        self._sync_items()
        sl.result.split_energy += ps.split_energy(ks, eps)
        sl.result.splits += ks.size
        # the centres of mass at t_now, the members from them and the pairs' orbits
        at_now = st["t"][cm_rows] == t_now
        xc = np.where(at_now[:, None], st["x"][cm_rows], st["xp"][cm_rows])
        vc = np.where(at_now[:, None], st["v"][cm_rows], st["vp"][cm_rows])
        members = ps.pairs[ks].ravel()
        xm, vm = ps.members_of(ks, xc, vc)
        cap_cm = float(st["dt"][cm_rows].min())
        new_ps = ps.without(ks, ctx)
        # the new reduced system: bodies in no pair in index order, then the
        # remaining pairs' centres of mass (the layout nb_pairs_reduce makes)
        old_row = {int(i): r for r, i in enumerate(ps.singles)}
        mem_row = {int(i): q for q, i in enumerate(members)}
        keep_pairs = np.setdiff1d(np.arange(ps.np), ks)
        n_new = new_ps.cm0 + new_ps.np
        src = np.empty(n_new, dtype=np.int64)          # old row, or -1 - member slot
        for r, i in enumerate(new_ps.singles):
            src[r] = old_row[int(i)] if int(i) in old_row else -1 - mem_row[int(i)]
        src[new_ps.cm0:] = ps.cm0 + keep_pairs
        old = src >= 0
        x, v = np.empty((n_new, 3)), np.empty((n_new, 3))
        a, j = np.zeros((n_new, 3)), np.zeros((n_new, 3))
        m, t, dt = np.empty(n_new), np.empty(n_new), np.empty(n_new)
        for f, arr in (("x", x), ("v", v), ("a", a), ("j", j), ("m", m), ("t", t), ("dt", dt)):
            arr[old] = st[f][src[old]]
        mq = -1 - src[~old]
        x[~old], v[~old] = xm[mq], vm[mq]
        m[~old] = ps.m[members[mq]]
        t[~old], dt[~old] = t_now, cap_cm
        sysn = System.from_arrays(x, v, m, device=self.device,
                                  fp32_copies=(self.precision != "fp64"))
        rows = sysn.buf64[:, :n_new]
        rows[6:9] = torch.from_numpy(np.ascontiguousarray(a.T)).to(self.device)
        rows[9:12] = torch.from_numpy(np.ascontiguousarray(j.T)).to(self.device)
        rows[13] = torch.from_numpy(t).to(self.device)
        rows[14] = torch.from_numpy(dt).to(self.device)
        # the members' acceleration, jerk and step at t_now
        new_rows = np.flatnonzero(~old).astype(np.int32)
        idx = torch.as_tensor(new_rows, device=self.device)
        k = new_rows.size
        acc = torch.zeros(3 * k, dtype=torch.float64, device=self.device)
        jerk = torch.zeros(3 * k, dtype=torch.float64, device=self.device)
        ctx.predict(sysn, t_now)
        ctx.force_active(sysn, idx, k, 0, n_new, eps, self.precision, acc, jerk)
        tick = math.ldexp(1.0, -40)
        steps = int(round(t_now / tick))
        cap = min(cap_cm, (steps & -steps) * tick) if steps else cap_cm
        self._check(self.L.nb_init_steps_active(ctx.h, sysn.ref, idx.data_ptr(), k,
                                                acc.data_ptr(), jerk.data_ptr(), float(t_now),
                                                self.eta_s, cap, self.dt_min))
        ctx.sync()
        sl.sys, sl.n, sl.ps = sysn, n_new, new_ps
        self._returned.add(sl)
        sl._work_buffers()
        sl.cm_idx = torch.arange(new_ps.cm0, n_new, dtype=torch.int32, device=self.device)
        self._arr = None
        self._tid_stale = True

    def _tidal_layout(self):
        """Device and pinned host buffers for the tidal outputs of every resident
        grouped system, rebuilt when the resident set changes: the tensors (9 per
        pair) and the centres of mass' times (1 per pair) at each system's table
        rows at this moment (its `tid_base`, kept when the table compacts later)."""
        gs = [sl for sl in self._grouped() if sl.ps.np]
        cap = max(self.ptab.cap, 1)
        for sl in gs:
            sl.ps.tid_base = sl.ps.base
        self._tid_slots = gs
        if self._tid_dev is None or self._tcm_dev.numel() < cap:
            # sized to the table's capacity, which grows geometrically: a rebuild of
            # the layout (admission, retirement, a pair's return) reuses them
            self._tid_dev = torch.zeros(9 * cap, dtype=torch.float64, device=self.device)
            self._tcm_dev = torch.zeros(cap, dtype=torch.float64, device=self.device)
            self._tid_host = torch.zeros(9 * cap, dtype=torch.float64).pin_memory()
            self._tcm_host = torch.zeros(cap, dtype=torch.float64).pin_memory()
        # rows of a moved or new system must not show an earlier owner's block time
        with torch.cuda.stream(self.ctx.stream):
            self._tcm_dev.fill_(float("nan"))
        items = (NbTidalItem * max(len(gs), 1))()
        tb, cb = self._tid_dev.data_ptr(), self._tcm_dev.data_ptr()
        for q, sl in enumerate(gs):
            it = items[q]
            it.sys = sl.sys._struct
            it.i_idx = sl.i_idx.data_ptr()        # the block's active list, set per step
            it.m = 0
            it.eps = float(sl.req.eps)
            it.tensor = tb + 8 * 9 * sl.ps.tid_base
            it.t_out = cb + 8 * sl.ps.tid_base
            it.status = sl.status.data_ptr()
            it.row0 = sl.ps.cm0                   # only centre-of-mass bodies write
            it.nrows = sl.ps.np
        self._tid_items = items
        self._tid_ext = max([sl.ps.tid_base + sl.ps.np for sl in gs], default=0)
        self._tid_stale = False

    def _tidal(self, ran_slots):
        """Tidal tensors at the centres of mass that were in this iteration's block of
        each grouped system that ran one (`ran_slots`: slot -> active-block size),
        from the predicted set of that step, copied to the pinned host buffer."""
        if self._tid_stale:
            self._tidal_layout()
        if not self._tid_slots:
            return
        items = self._tid_items
        for q, sl in enumerate(self._tid_slots):
            if sl in self._returned:
                # pairs returned this iteration: the system's bodies were renumbered
                # after its block, so every pair's tensor is taken (the times tell
                # the pairs of the block from the others)
                items[q].i_idx = sl.cm_idx.data_ptr()
                items[q].m = sl.ps.np if sl in ran_slots else 0
            else:
                items[q].i_idx = sl.i_idx.data_ptr()
                items[q].m = ran_slots.get(sl, 0)
        self._check(self.L.nb_tidal_active_batch(self.ctx.h, items, len(self._tid_slots)))
        e = self._tid_ext
        with torch.cuda.stream(self.ctx.stream):
            self._tid_host[: 9 * e].copy_(self._tid_dev[: 9 * e], non_blocking=True)
            self._tcm_host[:e].copy_(self._tcm_dev[:e], non_blocking=True)

    def _retire(self, slot: _Slot, error: str | None):
        self._sync_items()
        r = slot.result
        if slot.ps is not None:
            try:
                slot.ps.drain(self.ctx)        # its pairs' queued advances, before reading them
            except NbError as e:
                error = error or "NB_EUNBOUND: %s" % e
        r.error = error
        if error is None:
            if self.energy:
                r.energy1 = self.ctx.energy(slot.sys, slot.req.eps)[2]
            if slot.ps is not None:
                st = slot.sys.state_numpy()
                x, v = slot.ps.members(st["x"], st["v"])
                if self.energy:
                    r.energy1 += slot.ps.energy()
                    r.direct1 = self._direct_energy(slot, x, v)
                if self.keep_state:
                    r.final = dict(st, members_x=x, members_v=v,
                                   pair_r=slot.ps.r[: slot.ps.np].copy(),
                                   pair_w=slot.ps.w[: slot.ps.np].copy())
            elif self.keep_state:
                r.final = slot.sys.state_numpy()
        if slot.ps is not None:
            slot.ps.release()
        r.finished = self._now()
        self.results.append(r)
        self.adm.release(slot.req)
        self.slots.remove(slot)
        self._arr = None
        self._tid_stale = True

    # ---- one iteration: one block step of every resident system ---------------
    def _check(self, rc):
        if rc != 0:
            raise NbError(rc, self.L.nb_last_error(self.ctx.h).decode())

    _FIELDS = ("t_next", "m", "startup", "error", "done")
    _DTYPE = np.dtype({"names": list(_FIELDS), "formats": ["<f8", "<i4", "<i4", "<i4", "<i4"],
                       "offsets": [getattr(NbBatchItem, f).offset for f in _FIELDS],
                       "itemsize": C.sizeof(NbBatchItem)})

    def _sync_items(self):
        """Copy the item array's state (updated by the native calls) and the step
        counters back into the slots, before the resident set changes."""
        if self._arr is None:
            return
        for k, sl in enumerate(self.slots):
            sl.item = NbBatchItem.from_buffer_copy(self._arr[k])
            sl.result.steps = int(self._steps[k])
            sl.result.interactions = int(self._inter[k])

    def _build_items(self):
        k = len(self.slots)
        self._arr = (NbBatchItem * k)(*[sl.item for sl in self.slots])
        if self.order == 6:
            self._h6 = (NbHermite6 * k)(*[sl.h6._struct for sl in self.slots])
            self._snaps = (C.c_void_p * k)(*[sl.snap6.data_ptr() for sl in self.slots])
        raw = (C.c_char * C.sizeof(self._arr)).from_address(C.addressof(self._arr))
        self._view = np.frombuffer(raw, dtype=self._DTYPE)
        self._n = np.array([sl.n for sl in self.slots], dtype=np.int64)
        self._steps = np.array([sl.result.steps for sl in self.slots], dtype=np.int64)
        self._inter = np.array([sl.result.interactions for sl in self.slots], dtype=np.int64)

    def step(self):
        """One iteration: every resident system advances one block step in one
        native call (select, then predict, force and correct for every system not
        yet past its t_end, one launch per phase); finished or failed systems are
        retired.  The items live in one array across iterations and the per-system
        bookkeeping is vectorised, so the host work per iteration does not grow with
        the number of resident systems."""
        if not self.slots:
            return
        if self._arr is None:
            self._build_items()
        v = self._view
        startup = v["startup"] != 0          # before the call, which clears it
        if self.order == 6:
            self._check(self.L.nb_step6_batch(self.ctx.h, self._arr, self._h6, self._snaps,
                                              len(self.slots), self.prec_code, self.eta,
                                              self.eta_s, self.dt_max, self.dt_min))
        else:
            self._check(self.L.nb_step_batch(self.ctx.h, self._arr, len(self.slots),
                                             self.prec_code, self.eta, self.eta_s, self.dt_max,
                                             self.dt_min))
        # copies: a pair's return to the N-body system below rebuilds the item array
        err, done, t_next = v["error"].copy(), v["done"].copy(), v["t_next"].copy()
        at_step = list(self.slots)
        self._returned = set()
        m_blk = v["m"].astype(np.int64)
        ran = (err == 0) & (done == 0)
        n = self._n
        passes = 2 if self.order == 6 else 1        # force passes of a startup step
        inc = np.where(startup, passes * n * n, m_blk * n)
        self._inter[ran] += inc[ran]
        self._steps[ran & ~startup] += 1
        self.iterations += 1
        if self.groups:
            # the previous block's pairs go to the CPU thread (or return to the
            # N-body system); this block's systems get their tidal tensors after
            # the retirements below
            stepped = {}
            for k in np.flatnonzero(ran & ~startup):
                if self.slots[k].ps is not None:
                    stepped[self.slots[k]] = float(t_next[k])
            failed = self._queue_pairs(stepped) or {}
            for sl, tb in stepped.items():
                if sl.ps is not None and sl.ps.np:
                    self.ptab.prev_t[sl.ps.base: sl.ps.base + sl.ps.np] = tb
        else:
            failed = {}
        leave = np.flatnonzero((err != 0) | (done != 0))
        gone = [(self.slots[k], _lib.STATUS.get(int(err[k]), str(int(err[k])))
                 if err[k] != 0 else None) for k in leave]
        gone += [(sl, msg) for sl, msg in failed.items() if sl not in dict(gone)]
        for sl, e in gone:
            self._retire(sl, e)
        if self.groups:
            for sl, _ in gone:
                stepped.pop(sl, None)
            self._tidal({sl: int(m_blk[k]) for k, sl in enumerate(at_step) if sl in stepped})

    # ---- driving a request stream ------------------------------------------------
    def run(self, requests, realtime: bool = True, on_iteration=None):
        """Serve `requests` (with .arrival in seconds) until every one is finished.

        realtime: requests become visible at their arrival times on the wall clock;
        otherwise all are visible at once (a closed batch).  Returns the results.
        """
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = time.perf_counter()
        while pending or self.queue or self.slots:
            now = self._now()
            while pending and (not realtime or pending[0].arrival <= now):
                self.submit(pending.popleft())
            self._admit()
            if not self.slots:
                if pending and realtime:
                    time.sleep(max(0.0, min(pending[0].arrival - self._now(), 0.01)))
                    continue
                if self.queue:
                    raise RuntimeError("a queued request can never be admitted")
                continue
            self.step()
            if on_iteration is not None:
                on_iteration(self)
        self.ctx.sync()
        return self.results


def summarize(results, wall: float) -> dict:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.array([float("nan")])
    inter = sum(r.interactions for r in ok)
    out = {"requests": len(results), "completed": len(ok), "failed": len(results) - len(ok),
           "wall_s": wall, "solves_per_s": len(ok) / wall if wall > 0 else float("nan"),
           "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
           "interactions": int(inter), "interactions_per_s": inter / wall if wall > 0 else float("nan")}
    with_e = [r for r in ok if not math.isnan(r.energy1)]
    if with_e:
        errs = [r.energy_error for r in with_e]
        worst = with_e[int(np.argmax(errs))]
        out["energy_error_median"] = float(np.median(errs))
        out["energy_error_max"] = float(np.max(errs))
        out["energy_error_worst_request"] = {"rid": worst.rid, "n": worst.n}
    return out
