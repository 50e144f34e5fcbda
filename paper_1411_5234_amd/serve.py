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
from ._lib import FIELDS32, FIELDS64, NbBatchItem, NbError, NbHermite6, NbTidalItem, PRECISIONS
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
    captures: int = 0            # pairs formed from two single bodies during the run
    capture_energy: float = 0.0  # change of the conserved quantity at those captures

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def energy_error(self) -> float:
        """Relative error of the conserved quantity (grouped systems: the scheme's,
        with the known change at each pair's return to the N-body system and at each
        capture removed)."""
        return (abs(self.energy1 - self.split_energy - self.capture_energy - self.energy0)
                / abs(self.energy0))


class _Slot:
    """One resident system: device state, work buffers and its batch item."""

    def __init__(self, req, device, precision, now, order=4, L=None, groups=False, pairs=None,
                 snap=None, table=None, ctx=None, capture=False):
        snap = req.snapshot() if snap is None else snap
        self.req = req
        self.snap = snap
        self.ps = None                     # PairSet of a grouped system
        self.device = device
        if pairs is None and groups:
            pairs = snap.meta.get("pairs")
        if groups and capture and (pairs is None or not len(pairs)):
            pairs = np.zeros((0, 2), dtype=np.int64)     # pairs may still form during the run
        if pairs is not None and (len(pairs) or capture):
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
        self.pipe = None                   # the server pipe it is stepped on
        self.capture_pass = 0              # capture passes run on this system
        self.refused = {}                  # candidate pair -> pass at which it was refused

    def _work_buffers(self):
        """Active list and force outputs sized for the system, pointed to by the item."""
        n1 = max(self.n, 1)
        # written by the selection and the force before they are read
        self.i_idx = torch.empty(n1, dtype=torch.int32, device=self.device)
        self.acc = torch.empty(3 * n1, dtype=torch.float64, device=self.device)
        self.jerk = torch.empty(3 * n1, dtype=torch.float64, device=self.device)
        self.item.sys = self.sys._struct
        self.item.i_idx = self.i_idx.data_ptr()
        self.item.acc = self.acc.data_ptr()
        self.item.jerk = self.jerk.data_ptr()


class _Pipe:
    """A context (stream and scratch) and the resident systems stepped on it, with
    their batch items: one contiguous array handed to every nb_step_batch call and
    updated in place by it, rebuilt only when the set of resident systems changes
    (`view` reads its host fields with numpy)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.slots = []
        self.arr = None
        self.view = None
        self.n = None
        self.steps = None
        self.inter = None
        self.h6 = None
        self.snaps = None


def footprint_bytes(n: int, precision: str = "mixed", order: int = 4) -> int:
    """Device bytes one resident system of n bodies holds (state + work buffers;
    at 6th order also snap, crackle, predicted acceleration and the snap output)."""
    per_body = 8 * 21 + (16 if precision != "fp64" else 0) + 4 + 48
    if order == 6:
        per_body += Hermite6.BYTES_PER_BODY + 24
    return per_body * max(n, 1) + 4 + 1024


def return_layout(old_singles, new_singles, members, old_cm0, keep_pairs):
    """Rows of a reduced system after pairs return to the N-body system: for each row
    of the new system (its bodies in no pair, in index order, then the kept pairs'
    centres of mass), the row of the old system it continues (>= 0), or -1 - q for
    the q-th returning member (`members`, original indices).  old_singles and
    new_singles are the sorted original indices of the bodies in no pair."""
    ns = np.asarray(new_singles, dtype=np.int64)
    os_ = np.asarray(old_singles, dtype=np.int64)
    members = np.asarray(members, dtype=np.int64)
    keep_pairs = np.asarray(keep_pairs, dtype=np.int64)
    src = np.empty(ns.size + keep_pairs.size, dtype=np.int64)
    at = np.minimum(np.searchsorted(os_, ns), max(os_.size - 1, 0))
    is_old = (os_[at] == ns) if os_.size else np.zeros(ns.size, dtype=bool)
    src[: ns.size][is_old] = at[is_old]
    order = np.argsort(members)
    src[: ns.size][~is_old] = -1 - order[np.searchsorted(members[order], ns[~is_old])]
    src[ns.size:] = old_cm0 + keep_pairs
    return src


def capture_layout(old_cm0, old_np, p, q):
    """Rows of a reduced system after the single bodies at rows p[k] and q[k] (rows
    below old_cm0, all distinct) become the k-th new pair: for each row of the new
    system (its bodies in no pair, in index order, then the old pairs' centres of
    mass, then the new pairs'; the layout nb_pairs_reduce makes), the row of the old
    system it continues (>= 0), or -1 - k for the k-th new pair's centre of mass."""
    p = np.asarray(p, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    kt = p.size
    keep = np.ones(old_cm0, dtype=bool)
    keep[p] = False
    keep[q] = False
    old_rows = np.flatnonzero(keep)
    if q.size != kt or old_rows.size != old_cm0 - 2 * kt:
        raise ValueError("capture candidates are not distinct single bodies")
    ns = old_rows.size
    src = np.empty(ns + old_np + kt, dtype=np.int64)
    src[:ns] = old_rows
    src[ns: ns + old_np] = old_cm0 + np.arange(old_np)
    src[ns + old_np:] = -1 - np.arange(kt)
    return src


def mutual_nearest(rows, nn, n):
    """Pairs (p, q), p < q, of listed bodies that are each other's nearest neighbour:
    rows[k] lists a body, nn[k] its nearest neighbour (-1: not searched)."""
    rows = np.asarray(rows, dtype=np.int64)
    nn = np.asarray(nn, dtype=np.int64)
    ok = nn >= 0
    nbr = np.full(n, -1, dtype=np.int64)
    nbr[rows[ok]] = nn[ok]
    mutual = ok & (nbr[np.maximum(nn, 0)] == rows) & (rows < nn)
    return rows[mutual], nn[mutual]


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
                 max_sub: int = 1 << 20, group_gamma: float = 1e-3, split_gamma: float = 1e-2,
                 capture_every: int = 0, capture_dt: float | None = None, pipes: int = 1):
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
        # -- capture_every > 0: every that many iterations, two single bodies of a
        # grouped system that were in its block together, are each other's nearest
        # neighbours (nb_nearest_active_batch; only bodies whose step is at most
        # capture_dt, default dt_max / 256, are searched), form a bound pair and have
        # gamma below min(group_gamma, split_gamma / 10) in the field of the rest
        # (nb_tidal_points) become a pair carried as one body (the tight systems
        # that form during the run)
        self.groups = bool(groups)
        self.capture_every = int(capture_every) if self.groups else 0
        self.capture_dt = float(capture_dt) if capture_dt is not None else dt_max / 256.0
        # a captured pair starts at least ten times below the return threshold, so
        # that it does not return at its next step
        self.capture_gamma = min(float(group_gamma), 0.1 * float(split_gamma))
        self.per_period, self.max_sub = int(per_period), int(max_sub)
        self.group_gamma, self.split_gamma = float(group_gamma), float(split_gamma)
        self.ptab = PairTable(_lib.load()) if self.groups else None
        self._tid_stale = True
        self._tid_items = None
        self._tid_dev = None
        self._tid_host = None
        self._tid_slots = []
        self._q_sets = []
        self._q_rows = None
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
        # pipes: the resident systems are split between this many contexts, each
        # with its own stream and scratch; an iteration steps them one after the
        # other, so that one pipe's kernels run while the host waits for the other's
        # selection and builds its launches.  Grouped serving uses one pipe.
        if pipes not in (1, 2) or (pipes == 2 and self.groups):
            raise ValueError("pipes must be 1 or 2 (1 with groups)")
        self._pipes = [_Pipe(self.ctx)]
        if pipes == 2:
            self._pipes.append(_Pipe(Context(self.ctx.device,
                                             stream=torch.cuda.Stream(self.ctx.device))))

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
                         self.groups, table=self.ptab, ctx=self.ctx,
                         capture=self.capture_every > 0)
            if slot.ps is not None and slot.ps.np:
                self._pairs_startup(slot)
                gamma = slot.ps.perturbation()
                if np.any(gamma >= self.group_gamma):
                    slot.ps.release()
                    slot = _Slot(req, self.device, self.precision, slot.result.admitted,
                                 self.order, self.L, True, slot.ps.pairs[gamma < self.group_gamma],
                                 slot.snap, self.ptab, self.ctx, capture=self.capture_every > 0)
                    if slot.ps is not None and slot.ps.np:
                        self._pairs_startup(slot)
            slot.item.lanes = self.lanes
            # the pipe with the least resident work (the system's state was written
            # on torch's current stream: the pipe's stream waits for it)
            slot.pipe = min(self._pipes, key=lambda p: sum(sl.n * sl.n for sl in p.slots))
            slot.pipe.ctx.stream.wait_stream(torch.cuda.current_stream(self.device))
            if self.energy:
                slot.result.energy0 = slot.pipe.ctx.energy(slot.sys, req.eps)[2]
                if slot.ps is not None:
                    slot.result.energy0 += slot.ps.energy()
                    slot.result.direct0 = self._direct_energy(slot, slot.snap.x, slot.snap.v)
            self._sync_items()
            self.slots.append(slot)
            slot.pipe.slots.append(slot)
            self._invalidate()
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
        if self._tid_host is None or not self._q_sets:
            return {}
        # the sets of the last tidal layout, whose tensors and times are in the host
        # buffers (only admissions happen between that layout and this call, and
        # they add sets); the table rows from the sets' current bases, which a
        # compaction may have moved since
        sets, k, local = self._q_sets, self._q_k, self._q_local
        tid, owner = self._q_tid, self._q_owner                          # tidal offsets
        if any(sl.ps is not ps for sl, ps in sets):
            raise RuntimeError("pair sets changed without a new tidal layout")
        bases = tuple(ps.base for _, ps in sets)
        if self._q_rows is None or self._q_rows[0] != bases:
            self._q_rows = (bases, np.repeat(np.array(bases, dtype=np.int64), k) + local)
        rows = self._q_rows[1]                                           # table rows
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
                # pairs by their place in the set: an earlier return in this loop may
                # have compacted the table and moved this set's rows
                self._split(sl, local[due][sel], Tn[sel], float(t_b[sel][0]), stepped[sl])
            except (NbError, ValueError) as e:
                failed[sl] = "pair return failed: %s" % e
        return failed

    def _rows(self, sl, rows):
        """The FP64 state rows (FIELDS64 order, one column per body) of bodies `rows`
        of a slot's system, gathered on the device and copied to the host."""
        idx = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=self.device)
        with torch.cuda.stream(self.ctx.stream):
            return sl.sys.buf64[:, idx].cpu().numpy()

    def _rebuild(self, sl, src, new64):
        """A new System for a slot after pairs returned or formed: body r takes every
        row (state and predicted set, FP64 and FP32) of body src[r] of the slot's
        system when src[r] >= 0, gathered on the device, and otherwise the FP64 rows
        new64[:, -1 - src[r]] (FIELDS64 order, its predicted set equal to its state),
        with FP32 copies rounded from them."""
        n_new = src.size
        fp32 = self.precision != "fp64"
        # every column is written below
        sysn = System(n_new, self.device, fp32_copies=fp32,
                      buf64=torch.empty((len(FIELDS64), max(n_new, 1)), dtype=torch.float64,
                                        device=self.device),
                      buf32=torch.empty((len(FIELDS32), max(n_new, 1)), dtype=torch.float32,
                                        device=self.device) if fp32 else None)
        old = src >= 0
        with torch.cuda.stream(self.ctx.stream):
            if np.any(old):
                dst = torch.as_tensor(np.flatnonzero(old), device=self.device)
                so = torch.as_tensor(src[old], device=self.device)
                sysn.buf64[:, dst] = sl.sys.buf64[:, so]
                if sysn.buf32 is not None:
                    sysn.buf32[:, dst] = sl.sys.buf32[:, so]
            if not np.all(old):
                dn = torch.as_tensor(np.flatnonzero(~old), device=self.device)
                vals = torch.as_tensor(np.ascontiguousarray(new64[:, -1 - src[~old]]),
                                       device=self.device)
                sysn.buf64[:, dn] = vals
                if sysn.buf32 is not None:
                    sysn.buf32[0:3, dn] = vals[18:21].float()
                    sysn.buf32[3, dn] = vals[12].float()
        return sysn

    @staticmethod
    def _new_rows(x, v, a, j, m, t, dt):
        """FP64 rows (FIELDS64 order) of new bodies whose predicted set is their state."""
        k = len(m)
        out = np.empty((21, k))
        out[0:3], out[3:6], out[6:9], out[9:12] = x.T, v.T, a.T, j.T
        out[12], out[13], out[14] = m, t, dt
        out[15:18], out[18:21] = x.T, v.T
        return out

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
        T = torch.empty(9 * ks.size, dtype=torch.float64, device=self.device)
        rows_dev = torch.as_tensor(cm_rows.astype(np.int32), device=self.device)
        self._check(self.L.nb_tidal_active(ctx.h, sl.sys.ref, rows_dev.data_ptr(), ks.size, 0,
                                           sl.n, eps, T.data_ptr()))
        ctx.sync()
        Tnow = T.cpu().numpy().reshape(9, ks.size).T.copy()
        later = ps.tpair[ks] < t_now
        if np.any(later):
            ps.advance(ctx, ks[later], t_now, Tnow[later], self.per_period, self.max_sub,
                       queue=False)
        cm = self._rows(sl, cm_rows)                     # the centres of mass' rows
        self._sync_items()
        sl.result.split_energy += ps.split_energy(ks, eps)
        sl.result.splits += ks.size
        # the centres of mass at t_now, the members from them and the pairs' orbits
        at_now = cm[13] == t_now
        xc = np.where(at_now[:, None], cm[0:3].T, cm[15:18].T)
        vc = np.where(at_now[:, None], cm[3:6].T, cm[18:21].T)
        members = ps.pairs[ks].ravel()
        xm, vm = ps.members_of(ks, xc, vc)
        cap_cm = float(cm[14].min())
        new_ps = ps.without(ks, ctx)
        # the new reduced system: bodies in no pair in index order, then the
        # remaining pairs' centres of mass (the layout nb_pairs_reduce makes)
        keep_pairs = np.setdiff1d(np.arange(ps.np), ks)
        src = return_layout(ps.singles, new_ps.singles, members, ps.cm0, keep_pairs)
        n_new = src.size
        km = members.size
        new64 = self._new_rows(xm, vm, np.zeros((km, 3)), np.zeros((km, 3)), ps.m[members],
                               np.full(km, t_now), np.full(km, cap_cm))
        sysn = self._rebuild(sl, src, new64)
        old = src >= 0
        # the members' acceleration, jerk and step at t_now
        new_rows = np.flatnonzero(~old).astype(np.int32)
        idx = torch.as_tensor(new_rows, device=self.device)
        k = new_rows.size
        acc = torch.empty(3 * k, dtype=torch.float64, device=self.device)
        jerk = torch.empty(3 * k, dtype=torch.float64, device=self.device)
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
        self._invalidate()
        self._tid_stale = True

    # a candidate pair refused at a capture pass of its system is not examined again
    # for this many passes of that system (its perturbation changes slowly)
    CAPTURE_RETRY = 16

    def _capture(self, blocks, stepped):
        """Pairs that formed in this iteration's blocks (`blocks`: slot -> active-block
        size; `stepped`: slot -> block time).  The GPU finds the nearest neighbour of
        every single body of the block whose step is at most capture_dt; two bodies
        that are each other's nearest neighbour, bound to each other and perturbed by
        the rest below capture_gamma become a pair carried as one body.  Returns
        {slot: message} of systems whose capture failed."""
        from ._lib import NbNearestItem
        cand = [(sl, m) for sl, m in blocks.items()
                if sl.ps is not None and m > 0 and sl not in self._returned and sl.n >= 2]
        if not cand:
            return {}
        tot = sum(m for _, m in cand)
        nn = torch.empty(tot, dtype=torch.int32, device=self.device)
        r2 = torch.empty(tot, dtype=torch.float64, device=self.device)
        rows = torch.empty(tot, dtype=torch.int32, device=self.device)
        items = (NbNearestItem * len(cand))()
        off = 0
        with torch.cuda.stream(self.ctx.stream):
            for q, (sl, m) in enumerate(cand):
                it = items[q]
                it.sys = sl.sys._struct
                it.i_idx = sl.i_idx.data_ptr()
                it.m = m
                it.row_end = sl.ps.cm0
                it.dt_cap = self.capture_dt
                it.nn = nn.data_ptr() + 4 * off
                it.r2 = r2.data_ptr() + 8 * off
                it.status = sl.status.data_ptr()
                rows[off: off + m].copy_(sl.i_idx[:m])
                off += m
            self._check(self.L.nb_nearest_active_batch(self.ctx.h, items, len(cand)))
            nn_h = nn.cpu().numpy().astype(np.int64)
            rows_h = rows.cpu().numpy().astype(np.int64)
        failed = {}
        off = 0
        for sl, m in cand:
            r_, n_ = rows_h[off: off + m], nn_h[off: off + m]
            off += m
            sl.capture_pass += 1
            ok = n_ >= 0
            if not np.any(ok):
                continue
            p, q = mutual_nearest(r_, n_, sl.n)
            if p.size == 0:
                continue
            # candidates refused in the last CAPTURE_RETRY passes wait
            refused = sl.refused
            if len(refused) > 4096:          # forget refusals that have expired
                sl.refused = refused = {key: at for key, at in refused.items()
                                        if sl.capture_pass - at < self.CAPTURE_RETRY}
            keys = list(zip(sl.ps.singles[p].tolist(), sl.ps.singles[q].tolist()))
            fresh = np.array([sl.capture_pass - refused.get(key, -self.CAPTURE_RETRY)
                              >= self.CAPTURE_RETRY for key in keys])
            if not np.any(fresh):
                continue
            try:
                self._merge(sl, p[fresh], q[fresh], stepped[sl])
            except (NbError, ValueError) as e:
                failed[sl] = "pair capture failed: %s" % e
        return failed

    def _merge(self, sl, p, q, t_b):
        """Carry the bound, weakly perturbed ones of the candidate pairs (rows p[k],
        q[k] of the reduced system, both single bodies corrected at the block time
        t_b) as one body each from now on.  The new centre of mass takes the
        members' mass-weighted position, velocity, acceleration and jerk at t_b (the
        pair's internal forces cancel in these sums) and the smaller of their
        steps; the pair's relative orbit starts at t_b with the tidal tensor of the
        rest of the system at the centre of mass.  The rest keeps its state.
        Candidates that are refused are remembered for CAPTURE_RETRY passes."""
        ps, ctx = sl.ps, self.ctx
        eps = float(sl.req.eps)
        both = np.stack([p, q], axis=1).ravel()
        st = self._rows(sl, both)                     # the candidates' rows only
        t2 = st[13].reshape(-1, 2)
        sync = (t2[:, 0] == t_b) & (t2[:, 1] == t_b)
        _ptr = lambda z: z.ctypes.data_as(C.c_void_p)

        def refuse(mask):
            for key in zip(ps.singles[p[mask]].tolist(), ps.singles[q[mask]].tolist()):
                sl.refused[key] = sl.capture_pass

        def reduce(x, v, sel):
            cols = np.stack([2 * sel, 2 * sel + 1], axis=1).ravel()
            k = sel.size
            xr, vr = np.empty((k, 3)), np.empty((k, 3))
            mr, M = np.empty(k), np.empty(k)
            r, w = np.empty((k, 3)), np.empty((k, 3))
            local = np.arange(2 * k, dtype=np.int64).reshape(k, 2)
            args = [np.ascontiguousarray(z) for z in (x[:, cols].T, v[:, cols].T, st[12][cols])]
            rc = self.L.nb_pairs_reduce(2 * k, *[_ptr(z) for z in args], k, _ptr(local),
                                        *[_ptr(z) for z in (xr, vr, mr, M, r, w)])
            if rc != 0:
                raise ValueError("bad candidate pairs")
            return xr, vr, M, r, w

        sel = np.flatnonzero(sync)
        if sel.size == 0:
            return
        xc, vc, M, r, w = reduce(st[0:3], st[3:6], sel)
        k = sel.size
        a, g = np.empty(k), np.empty(k)
        self._check(self.L.nb_pairs_perturbation(k, _ptr(M), _ptr(r), _ptr(w), None, _ptr(a),
                                                 _ptr(g)))
        bound = np.isfinite(a) & (a > 0.0)
        refuse(np.isin(np.arange(p.size), sel[~bound]))
        if not np.any(bound):
            return
        sel, xc, vc, M, r, w, a = (z[bound] for z in (sel, xc, vc, M, r, w, a))
        kb = sel.size
        pts = torch.as_tensor(np.ascontiguousarray(xc.T).ravel(), device=self.device)
        exc = torch.as_tensor(np.ascontiguousarray(np.stack([p[sel], q[sel]])).ravel()
                              .astype(np.int32), device=self.device)
        T = torch.empty(9 * kb, dtype=torch.float64, device=self.device)
        self._check(self.L.nb_tidal_points(ctx.h, sl.sys.ref, kb, pts.data_ptr(), exc.data_ptr(),
                                           eps, T.data_ptr()))
        ctx.sync()
        Tk = np.ascontiguousarray(T.cpu().numpy().reshape(9, kb).T)
        ab, gb = np.ascontiguousarray(a), np.empty(kb)
        Mb = np.ascontiguousarray(M)
        self._check(self.L.nb_pairs_perturbation(kb, _ptr(Mb), None, None, _ptr(Tk), _ptr(ab),
                                                 _ptr(gb)))
        take = gb < self.capture_gamma
        refuse(np.isin(np.arange(p.size), sel[~take]))
        if not np.any(take):
            return
        sel, xc, vc, M, r, w, Tk, ab = (z[take] for z in (sel, xc, vc, M, r, w, Tk, ab))
        kt = sel.size
        # the centres of mass' acceleration and jerk: mass-weighted sums, as the
        # positions and velocities (the same reduction applied to a and j)
        ac, jc, _, _, _ = reduce(st[6:9], st[9:12], sel)
        dts = st[14].reshape(-1, 2)[sel].min(axis=1)
        ps.drain(ctx)
        self._sync_items()
        new_pairs = np.stack([ps.singles[p[sel]], ps.singles[q[sel]]], axis=1)
        out = C.c_double()
        rk = np.ascontiguousarray(r)
        npairs = np.ascontiguousarray(new_pairs)
        self._check(self.L.nb_pairs_split_energy(kt, _ptr(ps.m), _ptr(npairs), _ptr(rk), eps,
                                                 C.byref(out)))
        new_ps = ps.with_pairs(new_pairs, M, r, w, Tk, ab, t_b, ctx)
        # the new reduced system: bodies in no pair in index order, then the old
        # pairs' centres of mass, then the new ones (the layout nb_pairs_reduce makes)
        n_new = new_ps.cm0 + new_ps.np
        src = capture_layout(ps.cm0, ps.np, p[sel], q[sel])   # old row, or -1 - new pair
        if src.size != n_new:
            raise ValueError("capture layout does not match the new pair set")
        new64 = self._new_rows(xc, vc, ac, jc, M, np.full(kt, t_b), dts)
        sysn = self._rebuild(sl, src, new64)
        ctx.sync()
        sl.result.capture_energy -= out.value
        sl.result.captures += kt
        sl.sys, sl.n, sl.ps = sysn, n_new, new_ps
        self._returned.add(sl)
        sl._work_buffers()
        sl.cm_idx = torch.arange(new_ps.cm0, n_new, dtype=torch.int32, device=self.device)
        self._invalidate()
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
        # per layout: the numpy view of the items' i_idx and m, each slot's two lists
        # (its block's active list, its centres of mass), and the pair-queue arrays
        raw = (C.c_char * C.sizeof(items)).from_address(C.addressof(items))
        self._tid_view = np.frombuffer(raw, dtype=self._TID_DTYPE)
        self._tid_index = {id(sl): q for q, sl in enumerate(gs)}
        self._tid_iidx = np.array([sl.i_idx.data_ptr() for sl in gs], dtype=np.uint64)
        self._tid_cmidx = np.array([sl.cm_idx.data_ptr() for sl in gs], dtype=np.uint64)
        self._tid_np = np.array([sl.ps.np for sl in gs], dtype=np.int32)
        k = self._tid_np.astype(np.int64)
        self._q_sets = [(sl, sl.ps) for sl in gs]
        self._q_k = k
        self._q_local = np.arange(int(k.sum())) - np.repeat(np.cumsum(k) - k, k)
        self._q_tid = np.repeat(np.array([sl.ps.tid_base for sl in gs], dtype=np.int64), k)
        self._q_owner = np.repeat(np.arange(len(gs)), k)
        self._q_rows = None                      # (set bases, table rows), cached
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
        ptr = self._tid_iidx.copy()
        m = np.zeros(len(self._tid_slots), dtype=np.int32)
        for sl, mb in ran_slots.items():
            q = self._tid_index.get(id(sl))
            if q is not None:
                m[q] = mb
        for sl in self._returned:
            # pairs returned or formed this iteration: the system's bodies were
            # renumbered after its block, so every pair's tensor is taken (the times
            # tell the pairs of the block from the others)
            q = self._tid_index.get(id(sl))
            if q is not None:
                ptr[q] = self._tid_cmidx[q]
                m[q] = self._tid_np[q] if sl in ran_slots else 0
        self._tid_view["i_idx"] = ptr
        self._tid_view["m"] = m
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
            slot.pipe.ctx.sync()
            if self.energy:
                r.energy1 = slot.pipe.ctx.energy(slot.sys, slot.req.eps)[2]
            if slot.ps is not None:
                st = slot.sys.state_numpy()
                x, v = slot.ps.members(st["x"], st["v"])
                if self.energy:
                    r.energy1 += slot.ps.energy()
                    r.direct1 = self._direct_energy(slot, x, v)
                if self.keep_state:
                    r.final = dict(st, members_x=x, members_v=v,
                                   pair_r=slot.ps.r[: slot.ps.np].copy(),
                                   pair_w=slot.ps.w[: slot.ps.np].copy(),
                                   pairs=slot.ps.pairs.copy())
            elif self.keep_state:
                r.final = slot.sys.state_numpy()
        if slot.ps is not None:
            slot.ps.release()
        r.finished = self._now()
        self.results.append(r)
        self.adm.release(slot.req)
        self.slots.remove(slot)
        slot.pipe.slots.remove(slot)
        self._invalidate()
        self._tid_stale = True

    # ---- one iteration: one block step of every resident system ---------------
    def _check(self, rc, ctx=None):
        if rc != 0:
            raise NbError(rc, self.L.nb_last_error((ctx or self.ctx).h).decode())

    _TID_DTYPE = np.dtype({"names": ["i_idx", "m"], "formats": ["<u8", "<i4"],
                           "offsets": [NbTidalItem.i_idx.offset, NbTidalItem.m.offset],
                           "itemsize": C.sizeof(NbTidalItem)})
    _FIELDS = ("t_next", "m", "startup", "error", "done")
    _DTYPE = np.dtype({"names": list(_FIELDS), "formats": ["<f8", "<i4", "<i4", "<i4", "<i4"],
                       "offsets": [getattr(NbBatchItem, f).offset for f in _FIELDS],
                       "itemsize": C.sizeof(NbBatchItem)})

    def _invalidate(self):
        """The resident set changed: every pipe rebuilds its item array before its
        next step (after _sync_items has copied the arrays back)."""
        for p in self._pipes:
            p.arr = None

    def _sync_items(self):
        """Copy the item arrays' state (updated by the native calls) and the step
        counters back into the slots, before the resident set changes."""
        for p in self._pipes:
            if p.arr is None:
                continue
            for k, sl in enumerate(p.slots):
                sl.item = NbBatchItem.from_buffer_copy(p.arr[k])
                sl.result.steps = int(p.steps[k])
                sl.result.interactions = int(p.inter[k])

    def _build_items(self, p):
        k = len(p.slots)
        p.arr = (NbBatchItem * k)(*[sl.item for sl in p.slots])
        if self.order == 6:
            p.h6 = (NbHermite6 * k)(*[sl.h6._struct for sl in p.slots])
            p.snaps = (C.c_void_p * k)(*[sl.snap6.data_ptr() for sl in p.slots])
        raw = (C.c_char * C.sizeof(p.arr)).from_address(C.addressof(p.arr))
        p.view = np.frombuffer(raw, dtype=self._DTYPE)
        p.n = np.array([sl.n for sl in p.slots], dtype=np.int64)
        p.steps = np.array([sl.result.steps for sl in p.slots], dtype=np.int64)
        p.inter = np.array([sl.result.interactions for sl in p.slots], dtype=np.int64)

    def step(self):
        """One iteration: every resident system advances one block step, one native
        call per pipe (select, then predict, force and correct for every system of
        the pipe not yet past its t_end, one launch per phase); finished or failed
        systems are retired.  The items live in one array per pipe across iterations
        and the per-system bookkeeping is vectorised, so the host work per iteration
        does not grow with the number of resident systems."""
        if not self.slots:
            return
        for p in self._pipes:
            if p.slots:
                self._step_pipe(p)
        self.iterations += 1

    def _step_pipe(self, p):
        if p.arr is None:
            self._build_items(p)
        v = p.view
        k_items = len(p.slots)
        startup = v["startup"] != 0          # before the call, which clears it
        if self.order == 6:
            self._check(self.L.nb_step6_batch(p.ctx.h, p.arr, p.h6, p.snaps, k_items,
                                              self.prec_code, self.eta, self.eta_s, self.dt_max,
                                              self.dt_min), p.ctx)
        else:
            self._check(self.L.nb_step_batch(p.ctx.h, p.arr, k_items, self.prec_code, self.eta,
                                             self.eta_s, self.dt_max, self.dt_min), p.ctx)
        # copies: a pair's return to the N-body system below rebuilds the item array
        err, done, t_next = v["error"].copy(), v["done"].copy(), v["t_next"].copy()
        at_step = list(p.slots)
        self._returned = set()
        m_blk = v["m"].astype(np.int64)
        ran = (err == 0) & (done == 0)
        n = p.n
        passes = 2 if self.order == 6 else 1        # force passes of a startup step
        inc = np.where(startup, passes * n * n, m_blk * n)
        p.inter[ran] += inc[ran]
        p.steps[ran & ~startup] += 1
        steps = p.steps.copy()
        if self.groups:
            # the previous block's pairs go to the CPU thread (or return to the
            # N-body system); this block's systems get their tidal tensors after
            # the retirements below
            stepped = {}
            for k in np.flatnonzero(ran & ~startup):
                if at_step[k].ps is not None:
                    stepped[at_step[k]] = float(t_next[k])
            failed = self._queue_pairs(stepped) or {}
            if self.capture_every:
                # on every capture_every-th block step of each system (its own count,
                # so that a system's run does not depend on what else is resident)
                blocks = {sl: int(m_blk[k]) for k, sl in enumerate(at_step)
                          if sl in stepped and sl not in failed
                          and steps[k] % self.capture_every == 0}
                failed.update(self._capture(blocks, stepped))
            for sl, tb in stepped.items():
                if sl.ps is not None and sl.ps.np:
                    self.ptab.prev_t[sl.ps.base: sl.ps.base + sl.ps.np] = tb
        else:
            failed = {}
        leave = np.flatnonzero((err != 0) | (done != 0))
        gone = [(at_step[k], _lib.STATUS.get(int(err[k]), str(int(err[k])))
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
        for p in self._pipes:
            p.ctx.sync()
        return self.results


def summarize(results, wall: float) -> dict:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.array([float("nan")])
    inter = sum(r.interactions for r in ok)
    out = {"requests": len(results), "completed": len(ok), "failed": len(results) - len(ok),
           "wall_s": wall, "solves_per_s": len(ok) / wall if wall > 0 else float("nan"),
           "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
           "interactions": int(inter), "interactions_per_s": inter / wall if wall > 0 else float("nan")}
    if any(r.pairs or r.splits or r.captures for r in ok):
        out["pairs_at_admission"] = int(sum(r.pairs for r in ok))
        out["pair_returns"] = int(sum(r.splits for r in ok))
        out["pair_captures"] = int(sum(r.captures for r in ok))
    with_e = [r for r in ok if not math.isnan(r.energy1)]
    if with_e:
        errs = [r.energy_error for r in with_e]
        worst = with_e[int(np.argmax(errs))]
        out["energy_error_median"] = float(np.median(errs))
        out["energy_error_max"] = float(np.max(errs))
        out["energy_error_worst_request"] = {"rid": worst.rid, "n": worst.n}
    return out
