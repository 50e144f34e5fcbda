"""Plain FP64 CPU oracle for the direct N-body hot path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may use this package.  The GPU product path never imports it.

The arithmetic lives in ``nbody_oracle.c`` (plain C, FP64, no contraction, no
fast-math); this module loads it with ctypes and adds the block-step driver loop
(select -> predict all -> force on the active block -> correct), written in the
order of the paper's Sec. 2 items 1-2.  Arrays of vectors are numpy (n, 3) float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_lib = None
# Plain FP64: no contraction into FMA, no fast-math, so reductions keep their
# written order; -O3 without -march, so the library built here runs on any x86-64
# host it is copied to.
CFLAGS = ["-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so and return its path."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.orc_num_threads.restype = C.c_int
        L.orc_force.restype = C.c_int
        L.orc_force.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int64, _ip, C.c_int64, C.c_int64,
                                C.c_double, _dp, _dp]
        L.orc_force_scale.restype = C.c_int
        L.orc_force_scale.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int64, _ip, C.c_int64,
                                      C.c_int64, C.c_double, _dp, _dp]
        L.orc_energy.restype = None
        L.orc_energy.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_predict.restype = None
        L.orc_predict.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_select.restype = C.c_int64
        L.orc_select.argtypes = [C.c_int64, _dp, _dp, C.POINTER(C.c_double), _ip]
        L.orc_init_dt.restype = C.c_int
        L.orc_init_dt.argtypes = [C.c_int64, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_correct.restype = C.c_int
        L.orc_correct.argtypes = [C.c_int64, C.c_int64, _ip, C.c_double, _dp, _dp, _dp, _dp,
                                  _dp, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                  C.c_double, C.c_void_p]
        L.orc_force6.restype = C.c_int
        L.orc_force6.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_int64, _ip, C.c_int64,
                                 C.c_int64, C.c_double, _dp, _dp, _dp]
        L.orc_force6_scale.restype = C.c_int
        L.orc_force6_scale.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_int64, _ip, C.c_int64,
                                       C.c_int64, C.c_double, _dp]
        L.orc_init_dt6.restype = C.c_int
        L.orc_init_dt6.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                   _dp]
        L.orc_tidal.restype = C.c_int
        L.orc_tidal.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _ip, C.c_int64, C.c_int64,
                                C.c_double, _dp]
        L.orc_velocity_scale.restype = C.c_int
        L.orc_velocity_scale.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int64, _ip, C.c_int64,
                                         C.c_int64, C.c_double, _dp]
        L.orc_tidal_points.restype = C.c_int
        L.orc_tidal_points.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _dp, _ip, C.c_double,
                                       _dp]
        L.orc_nearest.restype = C.c_int
        L.orc_nearest.argtypes = [C.c_int64, _dp, C.c_int64, _ip, C.c_int64, C.c_void_p,
                                  C.c_double, _ip, _dp]
        L.orc_kepler_drift.restype = C.c_int
        L.orc_kepler_drift.argtypes = [C.c_double, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_group_advance.restype = C.c_int
        L.orc_group_advance.argtypes = [C.c_double, _dp, _dp, C.c_double, C.c_int64, _dp, _dp]
        L.orc_predict6.restype = None
        L.orc_predict6.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_double,
                                   _dp, _dp, _dp]
        L.orc_correct6.restype = C.c_int
        L.orc_correct6.argtypes = [C.c_int64, C.c_int64, _ip, C.c_double, _dp, _dp, _dp,
                                   _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_double,
                                   C.c_double, C.c_double, C.c_void_p]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleError(RuntimeError):
    pass


_CODES = {-1: "index or range out of bounds", -4: "time step below dt_min",
          -5: "non-finite acceleration, jerk or step"}


def _check(rc):
    if rc != 0:
        raise OracleError(_CODES.get(rc, "error %d" % rc))


def force(x, v, m, eps, ilist=None, j0=0, j1=None):
    """Acceleration and jerk of bodies `ilist` from j in [j0, j1): Eq. 1-2 and d/dt."""
    x, v, m = _c(x), _c(v), _c(m)
    n = m.shape[0]
    if ilist is None:
        ilist = np.arange(n, dtype=np.int64)
    ilist = _c(ilist, np.int64)
    j1 = n if j1 is None else int(j1)
    acc = np.zeros((ilist.size, 3))
    jerk = np.zeros((ilist.size, 3))
    _check(lib().orc_force(n, x, v, m, ilist.size, ilist, int(j0), j1, float(eps), acc, jerk))
    return acc, jerk


def force_scale(x, v, m, eps, ilist=None, j0=0, j1=None):
    """Per body: sum_j |a_ij| and sum_j |jerk_ij| (magnitude scale of the pair sums)."""
    x, v, m = _c(x), _c(v), _c(m)
    n = m.shape[0]
    if ilist is None:
        ilist = np.arange(n, dtype=np.int64)
    ilist = _c(ilist, np.int64)
    j1 = n if j1 is None else int(j1)
    sa = np.zeros(ilist.size)
    sj = np.zeros(ilist.size)
    _check(lib().orc_force_scale(n, x, v, m, ilist.size, ilist, int(j0), j1, float(eps), sa, sj))
    return sa, sj


def velocity_scale(x, v, m, eps, ilist=None, j0=0, j1=None):
    """Per body: sum_j m_j (|v_i| + |v_j|) / (|r_ij|^2 + eps^2)^(3/2)."""
    x, v, m = _c(x), _c(v), _c(m)
    n = m.shape[0]
    ilist = np.arange(n, dtype=np.int64) if ilist is None else _c(ilist, np.int64)
    j1 = n if j1 is None else int(j1)
    sv = np.zeros(ilist.size)
    _check(lib().orc_velocity_scale(n, x, v, m, ilist.size, ilist, int(j0), j1, float(eps), sv))
    return sv


def energy(x, v, m, eps):
    """(kinetic, potential, total) with the softened pair potential, self term excluded."""
    x, v, m = _c(x), _c(v), _c(m)
    k, p = C.c_double(), C.c_double()
    lib().orc_energy(m.shape[0], x, v, m, float(eps), C.byref(k), C.byref(p))
    return k.value, p.value, k.value + p.value


def predict(x, v, a, jk, t, t_next):
    x, v, a, jk, t = _c(x), _c(v), _c(a), _c(jk), _c(t)
    xp = np.empty_like(x)
    vp = np.empty_like(v)
    lib().orc_predict(t.shape[0], x, v, a, jk, t, float(t_next), xp, vp)
    return xp, vp


def select(t, dt):
    t, dt = _c(t), _c(dt)
    idx = np.empty(t.shape[0], dtype=np.int64)
    tn = C.c_double()
    mcount = lib().orc_select(t.shape[0], t, dt, C.byref(tn), idx)
    return tn.value, idx[:mcount].copy()


def init_dt(a, jk, eta_s, dt_max, dt_min):
    a, jk = _c(a), _c(jk)
    dt = np.empty(a.shape[0])
    _check(lib().orc_init_dt(a.shape[0], a, jk, float(eta_s), float(dt_max), float(dt_min), dt))
    return dt


@dataclass
class State:
    """Per-body Hermite state: x, v, a, j (n, 3); m, t, dt (n,).  All FP64."""

    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    a: np.ndarray = None
    j: np.ndarray = None
    t: np.ndarray = None
    dt: np.ndarray = None

    @property
    def n(self):
        return int(self.m.shape[0])

    def copy(self):
        return State(*(None if f is None else f.copy() for f in
                       (self.x, self.v, self.m, self.a, self.j, self.t, self.dt)))


def correct(st: State, ilist, t_next, xp, vp, acc, jerk, eta, dt_max, dt_min, want_dta=False):
    """Hermite-4 correction of the active bodies plus the new power-of-two step (in place)."""
    ilist = _c(ilist, np.int64)
    acc, jerk = _c(acc), _c(jerk)
    dta = np.empty(ilist.size) if want_dta else None
    ptr = dta.ctypes.data_as(C.c_void_p) if want_dta else None
    rc = lib().orc_correct(st.n, ilist.size, ilist, float(t_next), _c(xp), _c(vp), acc, jerk,
                           st.x, st.v, st.a, st.j, st.t, st.dt, float(eta), float(dt_max),
                           float(dt_min), ptr)
    _check(rc)
    return dta


@dataclass
class Params:
    eps: float
    eta: float = 0.02
    eta_s: float = 0.01
    dt_max: float = 2.0 ** -3
    dt_min: float = 2.0 ** -40


def startup(x, v, m, p: Params) -> State:
    """t = 0: every body active; compute a, j and the startup steps."""
    st = State(_c(x).copy(), _c(v).copy(), _c(m).copy())
    n = st.n
    st.a, st.j = force(st.x, st.v, st.m, p.eps)
    st.t = np.zeros(n)
    st.dt = init_dt(st.a, st.j, p.eta_s, p.dt_max, p.dt_min)
    return st


@dataclass
class StepRecord:
    t_next: float
    ilist: np.ndarray
    xp: np.ndarray = None
    vp: np.ndarray = None
    acc: np.ndarray = None
    jerk: np.ndarray = None


def block_step(st: State, p: Params, keep=False) -> StepRecord:
    """One block step: select the active block, predict all, force, correct."""
    t_next, ilist = select(st.t, st.dt)
    xp, vp = predict(st.x, st.v, st.a, st.j, st.t, t_next)
    acc, jerk = force(xp, vp, st.m, p.eps, ilist)
    rec = StepRecord(t_next, ilist)
    if keep:
        rec.xp, rec.vp, rec.acc, rec.jerk = xp, vp, acc, jerk
    correct(st, ilist, t_next, xp, vp, acc, jerk, p.eta, p.dt_max, p.dt_min)
    return rec


def integrate(x, v, m, t_end, p: Params, log=None):
    """Block-step Hermite-4 integration from t = 0 to t_end (a multiple of dt_max).

    Returns (state, n_steps, interactions) where interactions = sum of m * N.
    If `log` is a list, each step's (t_next, active indices) is appended.
    """
    st = startup(x, v, m, p)
    n = st.n
    steps, inter = 0, n * n
    while True:
        tmin = float(np.min(st.t + st.dt))
        if tmin > t_end:
            break
        rec = block_step(st, p)
        steps += 1
        inter += rec.ilist.size * n
        if log is not None:
            log.append((rec.t_next, rec.ilist))
        if np.all(st.t == t_end):
            break
    return st, steps, inter


# ---------------------------------------------------------------------------
# 6th-order Hermite (the order of the paper's HiGPUs code, Sec. 2 item 1)
# ---------------------------------------------------------------------------

def force6(x, v, a, m, eps, ilist=None, j0=0, j1=None):
    """Acceleration, jerk and snap of bodies `ilist` from j in [j0, j1).

    `a` holds the (predicted) accelerations of all bodies: the snap of a pair
    needs the relative acceleration of the two bodies.
    """
    x, v, a, m = _c(x), _c(v), _c(a), _c(m)
    n = m.shape[0]
    if ilist is None:
        ilist = np.arange(n, dtype=np.int64)
    ilist = _c(ilist, np.int64)
    j1 = n if j1 is None else int(j1)
    acc = np.zeros((ilist.size, 3))
    jerk = np.zeros((ilist.size, 3))
    snap = np.zeros((ilist.size, 3))
    _check(lib().orc_force6(n, x, v, a, m, ilist.size, ilist, int(j0), j1, float(eps),
                            acc, jerk, snap))
    return acc, jerk, snap


def force6_scale(x, v, a, m, eps, ilist=None, j0=0, j1=None):
    """Per body: sum_j |snap_ij| (magnitude scale of the snap sum)."""
    x, v, a, m = _c(x), _c(v), _c(a), _c(m)
    n = m.shape[0]
    if ilist is None:
        ilist = np.arange(n, dtype=np.int64)
    ilist = _c(ilist, np.int64)
    j1 = n if j1 is None else int(j1)
    ss = np.zeros(ilist.size)
    _check(lib().orc_force6_scale(n, x, v, a, m, ilist.size, ilist, int(j0), j1, float(eps), ss))
    return ss


def init_dt6(a, jk, sn, eta_s, dt_max, dt_min):
    """Startup steps of the 6th-order scheme from acceleration, jerk and snap."""
    a, jk, sn = _c(a), _c(jk), _c(sn)
    dt = np.empty(a.shape[0])
    _check(lib().orc_init_dt6(a.shape[0], a, jk, sn, float(eta_s), float(dt_max), float(dt_min),
                              dt))
    return dt


def predict6(x, v, a, jk, sn, cr, t, t_next):
    """Taylor prediction of position (to crackle), velocity and acceleration."""
    x, v, a, jk, sn, cr, t = (_c(q) for q in (x, v, a, jk, sn, cr, t))
    xp, vp, ap = np.empty_like(x), np.empty_like(v), np.empty_like(a)
    lib().orc_predict6(t.shape[0], x, v, a, jk, sn, cr, t, float(t_next), xp, vp, ap)
    return xp, vp, ap


@dataclass
class State6(State):
    """Hermite-6 state: the Hermite-4 fields plus snap s and crackle c (n, 3)."""

    s: np.ndarray = None
    c: np.ndarray = None

    def copy(self):
        return State6(*(None if f is None else f.copy() for f in
                        (self.x, self.v, self.m, self.a, self.j, self.t, self.dt,
                         self.s, self.c)))


def correct6(st: State6, ilist, t_next, acc, jerk, snap, eta, dt_max, dt_min, want_dta=False):
    """Hermite-6 correction of the active bodies plus the new power-of-two step (in place)."""
    ilist = _c(ilist, np.int64)
    acc, jerk, snap = _c(acc), _c(jerk), _c(snap)
    dta = np.empty(ilist.size) if want_dta else None
    ptr = dta.ctypes.data_as(C.c_void_p) if want_dta else None
    rc = lib().orc_correct6(st.n, ilist.size, ilist, float(t_next), acc, jerk, snap,
                            st.x, st.v, st.a, st.j, st.s, st.c, st.t, st.dt, float(eta),
                            float(dt_max), float(dt_min), ptr)
    _check(rc)
    return dta


@dataclass
class Params6(Params):
    """Step parameters of the 6th-order scheme.

    The generalized criterion gives dt = eta / omega on a circular orbit, where
    Aarseth's 4th-order one gives sqrt(eta) / omega; eta = 0.14 matches the
    4th-order eta = 0.02 there.
    """

    eta: float = 0.14


def startup6(x, v, m, p: Params6) -> State6:
    """t = 0: every body active.  A first pass gives the accelerations that the
    snap needs; the second gives acceleration, jerk and snap.  The crackle
    starts at zero; the first correction replaces it.  Startup steps from
    acceleration, jerk and snap (init_dt6)."""
    x, v, m = _c(x).copy(), _c(v).copy(), _c(m).copy()
    a0, _ = force(x, v, m, p.eps)
    a, jk, sn = force6(x, v, a0, m, p.eps)
    n = m.shape[0]
    st = State6(x, v, m, a, jk, np.zeros(n), None, sn, np.zeros((n, 3)))
    st.dt = init_dt6(st.a, st.j, st.s, p.eta_s, p.dt_max, p.dt_min)
    return st


@dataclass
class StepRecord6(StepRecord):
    ap: np.ndarray = None
    snap: np.ndarray = None


def block_step6(st: State6, p: Params6, keep=False) -> StepRecord6:
    """One Hermite-6 block step: select, predict all, force + snap, correct."""
    t_next, ilist = select(st.t, st.dt)
    xp, vp, ap = predict6(st.x, st.v, st.a, st.j, st.s, st.c, st.t, t_next)
    acc, jerk, snap = force6(xp, vp, ap, st.m, p.eps, ilist)
    rec = StepRecord6(t_next, ilist)
    if keep:
        rec.xp, rec.vp, rec.ap, rec.acc, rec.jerk, rec.snap = xp, vp, ap, acc, jerk, snap
    correct6(st, ilist, t_next, acc, jerk, snap, p.eta, p.dt_max, p.dt_min)
    return rec


def integrate6(x, v, m, t_end, p: Params6, log=None):
    """Block-step Hermite-6 integration from t = 0 to t_end (a multiple of dt_max).

    Returns (state, n_steps, interactions); the startup counts two passes.
    """
    st = startup6(x, v, m, p)
    n = st.n
    steps, inter = 0, 2 * n * n
    while True:
        if float(np.min(st.t + st.dt)) > t_end:
            break
        rec = block_step6(st, p)
        steps += 1
        inter += rec.ilist.size * n
        if log is not None:
            log.append((rec.t_next, rec.ilist))
        if np.all(st.t == t_end):
            break
    return st, steps, inter


# ---------------------------------------------------------------------------
# Tight groups (the HiGPUs-R scheme of Sec. 3): bound pairs carried as one body at
# their centre of mass, relative orbit advanced by Kepler drifts and tidal kicks
# ---------------------------------------------------------------------------

def tidal(x, m, eps, ilist=None, j0=0, j1=None):
    """Tidal tensor d a / d x (n_i, 3, 3) of the softened field of j in [j0, j1) at the
    listed bodies (self term excluded)."""
    x, m = _c(x), _c(m)
    n = m.shape[0]
    if ilist is None:
        ilist = np.arange(n, dtype=np.int64)
    ilist = _c(ilist, np.int64)
    j1 = n if j1 is None else int(j1)
    T = np.zeros(9 * ilist.size)
    _check(lib().orc_tidal(n, x, m, ilist.size, ilist, int(j0), j1, float(eps), T))
    return T.reshape(-1, 3, 3)


def tidal_points(x, m, eps, points, excl=None):
    """Tidal tensor (k, 3, 3) of the softened field at the points (k, 3), leaving out
    the bodies excl[k] (k, 2; -1: none) for point k."""
    x, m, points = _c(x), _c(m), _c(np.reshape(points, (-1, 3)))
    k = points.shape[0]
    excl = np.full((k, 2), -1, dtype=np.int64) if excl is None else _c(excl, np.int64)
    T = np.zeros(9 * k)
    _check(lib().orc_tidal_points(m.shape[0], x, m, k, points, excl.reshape(-1), float(eps), T))
    return T.reshape(-1, 3, 3)


def nearest(x, ilist=None, row_end=None, dt=None, dt_cap=float("inf")):
    """Nearest other body of each listed body (lowest index on equal distances) and
    its squared distance; -1 / inf for bodies not searched (index >= row_end, or
    dt > dt_cap)."""
    x = _c(x)
    n = x.shape[0]
    ilist = np.arange(n, dtype=np.int64) if ilist is None else _c(ilist, np.int64)
    row_end = n if row_end is None else int(row_end)
    dtp = None if dt is None else _c(dt)
    nn = np.empty(ilist.size, dtype=np.int64)
    r2 = np.empty(ilist.size)
    _check(lib().orc_nearest(n, x, ilist.size, ilist, row_end,
                             None if dtp is None else dtp.ctypes.data_as(C.c_void_p),
                             float(dt_cap), nn, r2))
    return nn, r2


def kepler_drift(M, r, v, dt):
    """Exact two-body motion of the relative coordinate (bound pairs only)."""
    r1, v1 = np.empty(3), np.empty(3)
    _check(lib().orc_kepler_drift(float(M), _c(r), _c(v), float(dt), r1, v1))
    return r1, v1


def group_advance(M, r, v, H, nsub, T0, T1):
    """Relative orbit over H: nsub kick-drift-kick substeps, T linear from T0 to T1."""
    r, v = _c(r).copy(), _c(v).copy()
    _check(lib().orc_group_advance(float(M), r, v, float(H), int(nsub), _c(T0).reshape(9),
                                   _c(T1).reshape(9)))
    return r, v


def orbit_period(M, r, v):
    inv_a = 2.0 / np.linalg.norm(r) - np.dot(v, v) / M
    if inv_a <= 0.0:
        raise OracleError("pair is not bound")
    return 2.0 * np.pi * np.sqrt(inv_a ** -3 / M)


def substeps(M, r, v, H, per_period=32, cap=1 << 20):
    """Substeps for a relative orbit over H: per_period per orbital period."""
    return int(min(cap, max(1, np.ceil(per_period * H / orbit_period(M, r, v)))))


@dataclass
class Grouped:
    """A block-step state with pairs carried as centre-of-mass bodies.

    st: the 4th-order state of the reduced system (singles first, then one body per
    pair); pairs: (i, j) original indices; rel: relative (r, v) of each pair at
    tpair; T: tidal tensor at each pair's centre of mass at tpair."""

    st: State
    singles: np.ndarray
    pairs: np.ndarray
    M: np.ndarray
    r: np.ndarray
    w: np.ndarray
    T: np.ndarray
    tpair: np.ndarray


def group_startup(x, v, m, pairs, p: Params) -> Grouped:
    x, v, m = _c(x), _c(v), _c(m)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    n = m.shape[0]
    in_pair = np.zeros(n, dtype=bool)
    in_pair[pairs.ravel()] = True
    singles = np.nonzero(~in_pair)[0]
    i, j = pairs[:, 0], pairs[:, 1]
    M = m[i] + m[j]
    xc = (m[i, None] * x[i] + m[j, None] * x[j]) / M[:, None]
    vc = (m[i, None] * v[i] + m[j, None] * v[j]) / M[:, None]
    xr = np.concatenate([x[singles], xc])
    vr = np.concatenate([v[singles], vc])
    mr = np.concatenate([m[singles], M])
    st = startup(xr, vr, mr, p)
    cm = singles.size + np.arange(pairs.shape[0])
    T = tidal(st.x, st.m, p.eps, cm)
    return Grouped(st, singles, pairs, M, x[j] - x[i], v[j] - v[i], T, np.zeros(pairs.shape[0]))


def group_block_step(g: Grouped, p: Params, per_period=32):
    """One block step of the reduced system; every pair whose centre of mass was
    in the active block then advances its relative orbit to the block time, with
    the tidal tensor interpolated between its value at the pair's previous time
    and its value at the block time (from the same predicted j-set as the force)."""
    rec = block_step(g.st, p, keep=True)
    ncm = g.singles.size
    act = rec.ilist[rec.ilist >= ncm]
    if act.size:
        Tn = tidal(rec.xp, g.st.m, p.eps, act)
        for q, b in enumerate(act - ncm):
            H = rec.t_next - g.tpair[b]
            ns = substeps(g.M[b], g.r[b], g.w[b], H, per_period)
            g.r[b], g.w[b] = group_advance(g.M[b], g.r[b], g.w[b], H, ns, g.T[b], Tn[q])
            g.T[b] = Tn[q]
            g.tpair[b] = rec.t_next
    return rec


def group_energy(g: Grouped, m, eps):
    """Energy of the grouped system: the reduced system's (pairs as point masses,
    softened), plus each pair's two-body energy (unsoftened, as its orbit is
    advanced) and its tidal energy -mu r.T.r / 2 in the field of the rest."""
    m = _c(m)
    er = energy(g.st.x, g.st.v, g.st.m, eps)[2]
    i, j = g.pairs[:, 0], g.pairs[:, 1]
    mu = m[i] * m[j] / g.M
    rr = np.linalg.norm(g.r, axis=1)
    tid = np.einsum("ka,kab,kb->k", g.r, g.T, g.r)
    return er + float((mu * (0.5 * (g.w ** 2).sum(1) - g.M / rr - 0.5 * tid)).sum())


def group_integrate(x, v, m, pairs, t_end, p: Params, per_period=32, log=None):
    """Block-step integration with the pairs grouped; returns (x, v) of all bodies
    at t_end, the number of block steps and the grouped state."""
    m = _c(m)
    g = group_startup(x, v, m, pairs, p)
    steps = 0
    while float(np.min(g.st.t + g.st.dt)) <= t_end:
        rec = group_block_step(g, p, per_period)
        steps += 1
        if log is not None:
            log.append((rec.t_next, rec.ilist))
        if np.all(g.st.t == t_end):
            break
    n = m.shape[0]
    xo, vo = np.empty((n, 3)), np.empty((n, 3))
    ns = g.singles.size
    xo[g.singles], vo[g.singles] = g.st.x[:ns], g.st.v[:ns]
    i, j = g.pairs[:, 0], g.pairs[:, 1]
    fi = (m[j] / g.M)[:, None]
    fj = (m[i] / g.M)[:, None]
    xo[i] = g.st.x[ns:] - fi * g.r
    xo[j] = g.st.x[ns:] + fj * g.r
    vo[i] = g.st.v[ns:] - fi * g.w
    vo[j] = g.st.v[ns:] + fj * g.w
    return xo, vo, steps, g
