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


class GroupedIntegrator:
    """Block-step integration of x, v, m (numpy, n bodies) with the given bound pairs
    (index pairs into x) carried as centre-of-mass bodies.

    per_period / max_sub: substeps of a relative orbit per orbital period and their
    cap per block step; overlap=False runs the pair advance on the calling thread
    (for timing the overlap)."""

    def __init__(self, ctx: Context, x, v, m, pairs, p: Params, per_period: int = 32,
                 max_sub: int = 1 << 20, overlap: bool = True, device="cuda"):
        x = np.asarray(x, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        m = np.asarray(m, dtype=np.float64)
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        n = m.shape[0]
        if pairs.size and (pairs.min() < 0 or pairs.max() >= n or
                           np.unique(pairs.ravel()).size != pairs.size):
            raise ValueError("pairs must be distinct indices in [0, n)")
        self.ctx, self.p, self.n = ctx, p, n
        self.per_period, self.max_sub, self.overlap = int(per_period), int(max_sub), overlap
        self.m = m
        self.pairs = pairs
        in_pair = np.zeros(n, dtype=bool)
        in_pair[pairs.ravel()] = True
        self.singles = np.nonzero(~in_pair)[0]
        i, j = pairs[:, 0], pairs[:, 1]
        self.M = np.ascontiguousarray(m[i] + m[j])
        xc = (m[i, None] * x[i] + m[j, None] * x[j]) / self.M[:, None]
        vc = (m[i, None] * v[i] + m[j, None] * v[j]) / self.M[:, None]
        self.r = np.ascontiguousarray(x[j] - x[i])
        self.w = np.ascontiguousarray(v[j] - v[i])
        self.np = pairs.shape[0]
        self.cm0 = self.singles.size
        xr = np.concatenate([x[self.singles], xc])
        vr = np.concatenate([v[self.singles], vc])
        mr = np.concatenate([m[self.singles], self.M])
        self.sys = System.from_arrays(xr, vr, mr, device=device,
                                      fp32_copies=(p.precision != "fp64"))
        self.it = Integrator(ctx, self.sys, p)
        k = max(self.np, 1)
        self.cm_idx = torch.arange(self.cm0, self.cm0 + k, dtype=torch.int32, device=device)
        self.T_dev = torch.zeros(9 * k, dtype=torch.float64, device=device)
        self.T_host = torch.zeros(9 * k, dtype=torch.float64).pin_memory()
        self.tcm_host = torch.zeros(k, dtype=torch.float64).pin_memory()
        self.T = np.zeros((k, 9))                 # tensor at each pair's own time
        self.tpair = np.zeros(k)
        self.status = np.zeros(k, dtype=np.int32)
        self._pending = []                        # buffers of the queued advances
        self._prev_t = None                       # block time of the last GPU step
        self.cpu_pairs_advanced = 0
        self.cpu_seconds = 0.0                    # pair advance run on this thread
        self.wait_seconds = 0.0                   # time blocked waiting for the queue

    def __del__(self):
        # the CPU thread writes into this object's arrays: never free them under it
        try:
            if self._pending:
                self.ctx.L.nb_groups_wait(self.ctx.h)
        except Exception:
            pass

    # ---- GPU side --------------------------------------------------------------------
    def _tidal_to_host(self):
        """Tidal tensors of every pair at the current predicted set, and the pairs'
        centre-of-mass times, copied back asynchronously."""
        if self.np == 0:
            return
        self.ctx._check(self.ctx.L.nb_tidal_active(
            self.ctx.h, self.sys.ref, self.cm_idx.data_ptr(), self.np, 0, self.sys.n,
            float(self.p.eps), self.T_dev.data_ptr()))
        self.T_host.copy_(self.T_dev, non_blocking=True)
        self.tcm_host[: self.np].copy_(self.sys.row("t")[self.cm0:], non_blocking=True)

    def _host_tensor(self):
        # T_dev rows are (3a+b)*np + k
        return self.T_host.numpy()[: 9 * self.np].reshape(9, self.np).T

    def startup(self):
        self.it.startup()
        self._tidal_to_host()
        self.ctx.sync()
        self.T[: self.np] = self._host_tensor()
        self.tpair[:] = 0.0

    # ---- CPU side --------------------------------------------------------------------
    MAX_QUEUED = 4096

    def _fail(self, rc):
        bad = np.nonzero(self.status[: self.np] != 0)[0]
        raise _lib.NbError(rc, "pairs %s are no longer bound" % self.pairs[bad].tolist())

    def _drain(self):
        """Wait until every queued pair advance has run (self.r, self.w current)."""
        if not self._pending:
            return
        t0 = time.perf_counter()
        rc = self.ctx.L.nb_groups_wait(self.ctx.h)
        self.wait_seconds += time.perf_counter() - t0
        self._pending.clear()
        if rc != 0:
            self._fail(rc)

    def _launch(self):
        """Queue the advance of the pairs whose centre of mass was in the previous
        block (their tensors and times are on the host after the selection's sync)."""
        if self._prev_t is None or self.np == 0:
            return
        tcm = self.tcm_host.numpy()[: self.np]
        idx = np.nonzero(tcm == self._prev_t)[0]
        idx = idx[self.tpair[idx] < self._prev_t]
        if idx.size == 0:
            return
        Tn = self._host_tensor()[idx]
        rows = np.ascontiguousarray(idx, dtype=np.int32)
        H = np.ascontiguousarray(self._prev_t - self.tpair[idx])
        T0 = np.ascontiguousarray(self.T[idx])
        T1 = np.ascontiguousarray(Tn)
        self.T[idx] = Tn
        self.tpair[idx] = self._prev_t
        self.cpu_pairs_advanced += idx.size
        args = (int(idx.size), _p(rows), _p(self.M), _p(self.r), _p(self.w), _p(H), _p(T0),
                _p(T1), self.per_period, self.max_sub, _p(self.status))
        if self.overlap:
            if len(self._pending) >= self.MAX_QUEUED:
                self._drain()
            self._pending.append((rows, H, T0, T1))
            self.ctx._check(self.ctx.L.nb_groups_advance_async(self.ctx.h, *args))
        else:
            t0 = time.perf_counter()
            rc = self.ctx.L.nb_groups_advance(*args)
            self.cpu_seconds += time.perf_counter() - t0
            if rc != 0:
                self._fail(rc)

    # ---- block steps -----------------------------------------------------------------
    def step(self):
        """One block step; returns (t_next, m)."""
        t_next, m = self.ctx.select_active(self.sys, self.it.i_idx)
        self._launch()
        self.it._advance(t_next, m)
        self._tidal_to_host()
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
            self._tidal_to_host()
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
        x, v = np.empty((self.n, 3)), np.empty((self.n, 3))
        ns = self.cm0
        x[self.singles], v[self.singles] = st["x"][:ns], st["v"][:ns]
        i, j = self.pairs[:, 0], self.pairs[:, 1]
        fi = (self.m[j] / self.M)[:, None]
        fj = (self.m[i] / self.M)[:, None]
        x[i] = st["x"][ns:] - fi * self.r
        x[j] = st["x"][ns:] + fj * self.r
        v[i] = st["v"][ns:] - fi * self.w
        v[j] = st["v"][ns:] + fj * self.w
        return x, v

    def energy(self):
        """Reduced system's energy (softened) + each pair's two-body energy and tidal
        energy -mu r.T.r / 2 (the quantity the scheme conserves)."""
        self._drain()
        er = self.ctx.energy(self.sys, self.p.eps)[2]
        if self.np == 0:
            return er
        i, j = self.pairs[:, 0], self.pairs[:, 1]
        mu = self.m[i] * self.m[j] / self.M
        T = self.T[: self.np].reshape(-1, 3, 3)
        tid = np.einsum("ka,kab,kb->k", self.r, T, self.r)
        rr = np.linalg.norm(self.r, axis=1)
        return er + float((mu * (0.5 * (self.w ** 2).sum(1) - self.M / rr - 0.5 * tid)).sum())
