"""Tight pairs carried as centre-of-mass bodies, their relative orbits advanced on
CPU threads while the GPU runs the block steps (the HiGPUs-R scheme of Sec. 3 of
the paper, with bound pairs as the groups).

The reduced system (single bodies first, then one body per pair at the pair's
centre of mass) is integrated by the 4th-order block-step path on the GPU.  Each
block step also computes, on the GPU, the tidal tensor of the rest of the system
at every pair's centre of mass (`nb_tidal_active`, from the same predicted set as
the force).  A pair whose centre of mass was in a block advances its relative
orbit to that block time on the host (`nb_groups_advance_async`: exact two-body
drifts and tidal kicks, OpenMP over pairs).  The GPU never reads a pair's
relative orbit, so the host only queues that work: right after the selection's
host sync of the next block it queues the previous block's pairs on the
context's CPU thread and goes on enqueueing GPU work.  The queue runs in order
and may fall any number of blocks behind; the host waits for it only at the end
of a run (or when reading the pairs).  Tensors and times come back through pinned
buffers copied at the end of each block, so the pipeline adds no host sync of
its own.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import _lib
from .nbody import Context, Integrator, Params, System


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class PairTable:
    """Host arrays of the bound pairs of one or many systems, one contiguous segment
    per system: total mass M, relative coordinate r = x2 - x1 and velocity
    w = v2 - v1 (advanced in place by the library's CPU threads), the tidal tensor T
    (row-major 3x3) at the pair's own time tpair, its starting semimajor axis a0 and
    a status word.  Queued advances name rows of these arrays, so the arrays move
    (growth, compaction) only after the queue is drained.  A server keeps one table
    for all its resident systems and handles their pairs in one pass per iteration;
    `prev_t` (the block time of a system's last step, NaN when none) and
    `owner` (the PairSet of each row) serve that pass."""

    MAX_QUEUED = 4096

    def __init__(self, L, capacity: int = 256):
        self.L = L
        self.cap = 0
        self.used = 0
        self.sets = []                 # live PairSets, in the order of their segments
        self._pending = []
        self._grow(max(int(capacity), 1))

    FIELDS = (("M", (), np.float64), ("r", (3,), np.float64), ("w", (3,), np.float64),
              ("T", (9,), np.float64), ("tpair", (), np.float64), ("a0", (), np.float64),
              ("status", (), np.int32), ("prev_t", (), np.float64))

    def _grow(self, cap):
        for name, shape, dt in self.FIELDS:
            new = np.zeros((cap,) + shape, dtype=dt)
            if self.cap:
                new[: self.used] = getattr(self, name)[: self.used]
            setattr(self, name, new)
        self.prev_t[self.used:] = np.nan
        self.cap = cap

    def reserve(self, k, ctx=None):
        """Room for k more rows at the end (compacting and growing the arrays when
        needed; the caller has drained the queue when ctx is None)."""
        if self.used + k <= self.cap:
            return
        self.drain(ctx)
        live = sum(ps.np for ps in self.sets)
        pos = 0
        for ps in self.sets:                                   # compact, in segment order
            if ps.base != pos:
                for name, _, _ in self.FIELDS:
                    arr = getattr(self, name)
                    arr[pos: pos + ps.np] = arr[ps.base: ps.base + ps.np].copy()
            ps.base = pos
            pos += ps.np
        self.used = live
        self.prev_t[self.used:] = np.nan
        if self.used + k > self.cap:
            self._grow(max(2 * self.cap, self.used + k))

    def drain(self, ctx):
        """Wait until every queued advance has run.  Returns the seconds waited."""
        if not self._pending:
            return 0.0
        t0 = time.perf_counter()
        ctx.L.nb_groups_wait(ctx.h)
        self._pending.clear()
        return time.perf_counter() - t0

    def advance(self, ctx, rows, H, T0, T1, per_period, max_sub, queue=True):
        """Advance table rows `rows` over H with the tensor linear from T0 to T1;
        queued on the context's CPU thread, or run here (queue=False; returns the
        seconds spent)."""
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        H, T0, T1 = (np.ascontiguousarray(a, dtype=np.float64) for a in (H, T0, T1))
        args = (int(rows.size), _p(rows), _p(self.M), _p(self.r), _p(self.w), _p(H), _p(T0),
                _p(T1), int(per_period), int(max_sub), _p(self.status))
        if rows.size == 0:
            return 0.0
        if queue:
            if len(self._pending) >= self.MAX_QUEUED:
                self.drain(ctx)
            self._pending.append((rows, H, T0, T1))
            ctx._check(ctx.L.nb_groups_advance_async(ctx.h, *args))
            return 0.0
        t0 = time.perf_counter()
        rc = ctx.L.nb_groups_advance(*args)
        dt = time.perf_counter() - t0
        if rc != 0:
            bad = rows[self.status[rows] != 0]
            raise _lib.NbError(rc, "%d pairs are no longer bound" % bad.size)
        return dt

    def perturbation(self, rows, T):
        """gamma = |T| (2a0)^3 / M of table rows `rows` with tensors T (their rows)."""
        rows = np.asarray(rows)
        M = np.ascontiguousarray(self.M[rows])
        a = np.ascontiguousarray(self.a0[rows])
        Tk = np.ascontiguousarray(T, dtype=np.float64)
        g = np.empty(rows.size)
        if self.L.nb_pairs_perturbation(rows.size, _p(M), None, None, _p(Tk), _p(a), _p(g)) != 0:
            raise ValueError("bad pair arrays")
        return g


class PairSet:
    """The bound pairs of one system: a segment of a PairTable (a table of its own
    unless one is given) plus the system's masses and pair list.  The arithmetic
    (reduction to centre-of-mass bodies, members, pair energy, perturbation, pair
    advance) is the library's (nb_pairs_*, nb_groups_advance*)."""

    def __init__(self, L, x, v, m, pairs, table: PairTable | None = None, ctx=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        self.m = np.ascontiguousarray(m, dtype=np.float64)
        self.pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
        self.L = L
        self.n = self.m.shape[0]
        self.np = self.pairs.shape[0]
        nr = self.n - self.np
        self.xr, self.vr = np.empty((nr, 3)), np.empty((nr, 3))
        self.mr = np.empty(nr)
        M = np.zeros(max(self.np, 1))
        r, w = np.zeros((max(self.np, 1), 3)), np.zeros((max(self.np, 1), 3))
        rc = L.nb_pairs_reduce(self.n, _p(x), _p(v), _p(self.m), self.np, _p(self.pairs),
                               _p(self.xr), _p(self.vr), _p(self.mr), _p(M), _p(r), _p(w))
        if rc != 0:
            raise ValueError("pairs must be distinct indices in [0, n)")
        self.cm0 = nr - self.np                  # first centre-of-mass body of the reduced system
        # original indices of the bodies in no pair (the first cm0 reduced bodies)
        self.singles = np.setdiff1d(np.arange(self.n, dtype=np.int64), self.pairs.ravel())
        self.table = table if table is not None else PairTable(L, self.np)
        self._attach(ctx)
        self.M[:] = M[: self.np]
        self.r[:] = r[: self.np]
        self.w[:] = w[: self.np]
        self.advanced = 0
        if self.np:
            a, g = np.empty(self.np), np.empty(self.np)
            rc = L.nb_pairs_perturbation(self.np, _p(np.ascontiguousarray(self.M)),
                                         _p(np.ascontiguousarray(self.r)),
                                         _p(np.ascontiguousarray(self.w)), None, _p(a), _p(g))
            if rc != 0:
                raise ValueError("bad pair arrays")
            self.a0[:] = a

    def _attach(self, ctx):
        t = self.table
        t.reserve(self.np, ctx)
        self.base = t.used
        t.used += self.np
        t.sets.append(self)
        for name, _, _ in PairTable.FIELDS:
            getattr(t, name)[self.base: self.base + self.np] = 0
        t.prev_t[self.base: self.base + self.np] = np.nan

    def release(self):
        """Give the segment back to the table (after its queued advances have run)."""
        if self in self.table.sets:
            self.table.sets.remove(self)
            self.table.prev_t[self.base: self.base + self.np] = np.nan

    # the segment's rows of the table arrays (views)
    def _seg(self, name):
        return getattr(self.table, name)[self.base: self.base + self.np]

    M = property(lambda self: self._seg("M"))
    r = property(lambda self: self._seg("r"))
    w = property(lambda self: self._seg("w"))
    T = property(lambda self: self._seg("T"))
    tpair = property(lambda self: self._seg("tpair"))
    a0 = property(lambda self: self._seg("a0"))
    status = property(lambda self: self._seg("status"))

    def perturbation(self, T=None, idx=None):
        """gamma = |T| (2a)^3 / M of pairs idx (all by default) with tensors T (their
        rows; default: the stored ones), a the starting semimajor axes."""
        idx = np.arange(self.np) if idx is None else np.asarray(idx)
        return self.table.perturbation(self.base + idx, self.T[idx] if T is None else T)

    def due(self, tcm, t_block):
        """Pairs whose centre of mass was in the block at t_block (tcm: the
        centre-of-mass bodies' times after that block) and are not yet there."""
        idx = np.nonzero(tcm[: self.np] == t_block)[0]
        return idx[self.tpair[idx] < t_block]

    def advance(self, ctx, idx, t_block, Tn, per_period, max_sub, queue=True):
        """Advance pairs idx from their own times to t_block, the tidal tensor linear
        from T (at tpair) to Tn (at t_block); queued on the context's CPU thread
        (queue=True) or run here.  Returns the seconds spent here."""
        idx = np.asarray(idx)
        if idx.size == 0:
            return 0.0
        H = t_block - self.tpair[idx]
        T0 = self.T[idx].copy()
        Tn = np.asarray(Tn, dtype=np.float64)
        self.T[idx] = Tn
        self.tpair[idx] = t_block
        self.advanced += idx.size
        try:
            return self.table.advance(ctx, self.base + idx, H, T0, Tn, per_period, max_sub,
                                      queue)
        except _lib.NbError as e:
            raise _lib.NbError(e.code, "pairs %s are no longer bound"
                               % self.pairs[idx[self.status[idx] != 0]].tolist()) from None

    def drain(self, ctx):
        """Wait until every queued advance has run (r, w current); raises if a pair
        of this set became unbound."""
        dt = self.table.drain(ctx)
        if np.any(self.status != 0):
            self.fail(-7)
        return dt

    def fail(self, rc):
        bad = np.nonzero(self.status != 0)[0]
        raise _lib.NbError(rc, "pairs %s are no longer bound" % self.pairs[bad].tolist())

    def without(self, drop, ctx=None):
        """A PairSet of the same bodies without pairs `drop` (their members become
        single bodies), in the same table; the other pairs keep their orbits,
        tensors and times.  This set's segment is released."""
        keep = np.setdiff1d(np.arange(self.np), np.asarray(drop, dtype=np.int64))
        saved = {name: getattr(self, name)[keep].copy()
                 for name in ("M", "r", "w", "T", "tpair", "a0", "status")}
        self.release()
        out = PairSet.__new__(PairSet)
        out.L, out.m, out.n = self.L, self.m, self.n
        out.pairs = np.ascontiguousarray(self.pairs[keep])
        out.np = keep.size
        out.cm0 = self.n - 2 * out.np
        out.singles = np.setdiff1d(np.arange(self.n, dtype=np.int64), out.pairs.ravel())
        out.table = self.table
        out._attach(ctx)
        for name, val in saved.items():
            getattr(out, name)[:] = val
        out.advanced = self.advanced
        return out

    def with_pairs(self, new_pairs, M, r, w, T, a0, tpair, ctx=None):
        """A PairSet of the same bodies with the pairs `new_pairs` (index pairs of
        bodies in no pair) added after the existing ones, in the same table; their
        orbits (M, r, w), tensors T and starting semimajor axes a0 are given, at time
        tpair.  The existing pairs keep their orbits, tensors and times.  This set's
        segment is released (its queued advances must have run)."""
        new_pairs = np.asarray(new_pairs, dtype=np.int64).reshape(-1, 2)
        k = new_pairs.shape[0]
        pairs = np.ascontiguousarray(np.concatenate([self.pairs, new_pairs]))
        if (np.unique(pairs).size != pairs.size or new_pairs.min(initial=0) < 0
                or new_pairs.max(initial=0) >= self.n):
            raise ValueError("new pairs must be distinct bodies in no pair")
        saved = {name: getattr(self, name)[:].copy()
                 for name in ("M", "r", "w", "T", "tpair", "a0", "status")}
        self.release()
        out = PairSet.__new__(PairSet)
        out.L, out.m, out.n = self.L, self.m, self.n
        out.pairs = pairs
        out.np = out.pairs.shape[0]
        out.cm0 = self.n - 2 * out.np
        out.singles = np.setdiff1d(np.arange(self.n, dtype=np.int64), out.pairs.ravel())
        out.table = self.table
        out._attach(ctx)
        for name, val in saved.items():
            getattr(out, name)[: self.np] = val
        new = slice(self.np, out.np)
        out.M[new] = M
        out.r[new] = r
        out.w[new] = w
        out.T[new] = np.asarray(T).reshape(k, 9)
        out.a0[new] = a0
        out.tpair[new] = tpair
        out.status[new] = 0
        out.advanced = self.advanced
        return out

    def split_energy(self, idx, eps):
        """Change of the conserved quantity when pairs idx rejoin the N-body system
        as two bodies (their mutual potential becomes the softened one)."""
        out = C.c_double()
        pairs = np.ascontiguousarray(self.pairs[idx])
        r = np.ascontiguousarray(self.r[idx])
        rc = self.L.nb_pairs_split_energy(len(idx), _p(self.m), _p(pairs), _p(r), float(eps),
                                          C.byref(out))
        if rc != 0:
            raise ValueError("degenerate pair")
        return out.value

    def members(self, xr, vr):
        """(x, v) of all n original bodies from the reduced state and r, w."""
        x, v = np.empty((self.n, 3)), np.empty((self.n, 3))
        xr = np.ascontiguousarray(xr, dtype=np.float64)
        vr = np.ascontiguousarray(vr, dtype=np.float64)
        r, w = np.ascontiguousarray(self.r), np.ascontiguousarray(self.w)
        rc = self.L.nb_pairs_members(self.n, _p(xr), _p(vr), _p(self.m), self.np, _p(self.pairs),
                                     _p(r), _p(w), _p(x), _p(v))
        if rc != 0:
            raise ValueError("bad reduced state")
        return x, v

    def members_of(self, idx, xc, vc):
        """Positions and velocities of the members of pairs idx (rows in the order of
        pairs[idx].ravel()) from their centres of mass xc, vc and their r, w."""
        idx = np.asarray(idx)
        k = idx.size
        m = np.ascontiguousarray(self.m[self.pairs[idx].ravel()])
        local = np.arange(2 * k, dtype=np.int64).reshape(k, 2)
        xc, vc = np.ascontiguousarray(xc, dtype=np.float64), np.ascontiguousarray(vc, dtype=np.float64)
        r, w = np.ascontiguousarray(self.r[idx]), np.ascontiguousarray(self.w[idx])
        x, v = np.empty((2 * k, 3)), np.empty((2 * k, 3))
        if self.L.nb_pairs_members(2 * k, _p(xc), _p(vc), _p(m), k, _p(local), _p(r), _p(w),
                                   _p(x), _p(v)) != 0:
            raise ValueError("bad pair state")
        return x, v

    def energy(self):
        """The pairs' two-body and tidal energy (the pair part of the conserved
        quantity)."""
        out = C.c_double()
        r, w = np.ascontiguousarray(self.r), np.ascontiguousarray(self.w)
        T = np.ascontiguousarray(self.T)
        rc = self.L.nb_pairs_energy(self.np, _p(self.m), _p(self.pairs), _p(r), _p(w), _p(T),
                                    C.byref(out))
        if rc != 0:
            raise ValueError("degenerate pair")
        return out.value


class GroupedIntegrator:
    """Block-step integration of x, v, m (numpy, n bodies) with the given bound pairs
    (index pairs into x) carried as centre-of-mass bodies.

    per_period / max_sub: substeps of a relative orbit per orbital period and their
    cap per block step; overlap=False runs the pair advance on the calling thread
    (for timing the overlap)."""

    def __init__(self, ctx: Context, x, v, m, pairs, p: Params, per_period: int = 32,
                 max_sub: int = 1 << 20, overlap: bool = True, device="cuda"):
        self.ctx, self.p = ctx, p
        self.ps = PairSet(ctx.L, x, v, m, pairs)
        self.n, self.np, self.cm0 = self.ps.n, self.ps.np, self.ps.cm0
        self.pairs = self.ps.pairs
        self.per_period, self.max_sub, self.overlap = int(per_period), int(max_sub), overlap
        self.sys = System.from_arrays(self.ps.xr, self.ps.vr, self.ps.mr, device=device,
                                      fp32_copies=(p.precision != "fp64"))
        self.it = Integrator(ctx, self.sys, p)
        k = max(self.np, 1)
        self.cm_idx = torch.arange(self.cm0, self.cm0 + k, dtype=torch.int32, device=device)
        self.T_dev = torch.zeros(9 * k, dtype=torch.float64, device=device)
        self.T_host = torch.zeros(9 * k, dtype=torch.float64).pin_memory()
        self.tcm_host = torch.zeros(k, dtype=torch.float64).pin_memory()
        # the block's tensors: the active list, centre-of-mass bodies writing their rows
        self._tid_item = _lib.NbTidalItem()
        self._tid_item.sys = self.sys._struct
        self._tid_item.i_idx = self.it.i_idx.data_ptr()
        self._tid_item.eps = float(p.eps)
        self._tid_item.tensor = self.T_dev.data_ptr()
        self._tid_item.row0 = self.cm0
        self._tid_item.nrows = self.np
        self._prev_t = None                       # block time of the last GPU step
        self.cpu_seconds = 0.0                    # pair advance run on this thread
        self.wait_seconds = 0.0                   # time blocked waiting for the queue

    @property
    def M(self):
        return self.ps.M[: self.np]

    @property
    def r(self):
        return self.ps.r[: self.np]

    @property
    def w(self):
        return self.ps.w[: self.np]

    @property
    def cpu_pairs_advanced(self):
        return self.ps.advanced

    def __del__(self):
        # the CPU thread writes into this object's arrays: never free them under it
        try:
            if self.ps.table._pending:
                self.ctx.L.nb_groups_wait(self.ctx.h)
        except Exception:
            pass

    # ---- GPU side --------------------------------------------------------------------
    def _tidal_to_host(self, m=None):
        """Tidal tensors at the current predicted set -- of the pairs whose centre of
        mass is in the active block of m bodies (every pair when m is None) -- and
        the pairs' centre-of-mass times, copied back asynchronously."""
        if self.np == 0:
            return
        if m is None:
            self.ctx._check(self.ctx.L.nb_tidal_active(
                self.ctx.h, self.sys.ref, self.cm_idx.data_ptr(), self.np, 0, self.sys.n,
                float(self.p.eps), self.T_dev.data_ptr()))
        elif m:
            it = self._tid_item
            it.m = int(m)
            self.ctx._check(self.ctx.L.nb_tidal_active_batch(self.ctx.h, C.byref(it), 1))
        self.T_host.copy_(self.T_dev, non_blocking=True)
        self.tcm_host[: self.np].copy_(self.sys.row("t")[self.cm0:], non_blocking=True)

    def _host_tensor(self):
        # T_dev rows are (3a+b)*np + k
        return self.T_host.numpy()[: 9 * self.np].reshape(9, self.np).T

    def startup(self):
        self.it.startup()
        self._tidal_to_host()
        self.ctx.sync()
        self.ps.T[: self.np] = self._host_tensor()
        self.ps.tpair[:] = 0.0

    # ---- CPU side --------------------------------------------------------------------
    def _drain(self):
        """Wait until every queued pair advance has run (r, w current)."""
        self.wait_seconds += self.ps.drain(self.ctx)

    def _launch(self):
        """Queue the advance of the pairs whose centre of mass was in the previous
        block (their tensors and times are on the host after the selection's sync)."""
        if self._prev_t is None or self.np == 0:
            return
        idx = self.ps.due(self.tcm_host.numpy(), self._prev_t)
        if idx.size:
            self.cpu_seconds += self.ps.advance(self.ctx, idx, self._prev_t,
                                                self._host_tensor()[idx], self.per_period,
                                                self.max_sub, queue=self.overlap)

    # ---- block steps -----------------------------------------------------------------
    def step(self):
        """One block step; returns (t_next, m)."""
        t_next, m = self.ctx.select_active(self.sys, self.it.i_idx)
        self._launch()
        self.it._advance(t_next, m)
        self._tidal_to_host(m)
        self._prev_t = t_next
        return t_next, m

    def run(self, t_end: float, log: list | None = None):
        """Block steps until every body reaches t_end (a multiple of dt_max); the
        last block's pairs are advanced before returning."""
        while True:
            t_next, m = self.ctx.select_active(self.sys, self.it.i_idx)
            if t_next > t_end:
                break
            if log is not None:
                log.append((t_next, self.it.i_idx[:m].cpu().numpy().astype(np.int64)))
            self._launch()
            self.it._advance(t_next, m)
            self._tidal_to_host(m)
            self._prev_t = t_next
        self.ctx.sync()
        self._launch()
        self._drain()
        return self.it.steps, self.it.interactions

    # ---- results ---------------------------------------------------------------------
    def members(self):
        """(x, v) of all n original bodies; valid when every body and pair is at the
        same time (after run)."""
        self._drain()
        st = self.sys.state_numpy()
        return self.ps.members(st["x"], st["v"])

    def energy(self):
        """Reduced system's energy (softened) + each pair's two-body energy and tidal
        energy -mu r.T.r / 2 (the quantity the scheme conserves)."""
        self._drain()
        return self.ctx.energy(self.sys, self.p.eps)[2] + self.ps.energy()
