"""Seeded synthetic inputs for the direct N-body path.

This module is shared by the GPU path, the oracle tests and the benchmark.  It only
draws initial conditions and request streams; it holds none of the method's
arithmetic (no force, potential, prediction, correction or time-step rule).

Units are Henon (N-body) units: G = 1, total mass M = 1, and the Plummer sphere is
scaled so that its expected total energy is E = -1/4 (the paper's Eq. 1 with G = 1).

Every generator takes an integer seed and draws from numpy's PCG64 so that the same
seed gives the same bytes on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Snapshot",
    "plummer",
    "salpeter_masses",
    "kroupa_masses",
    "with_binaries",
    "Request",
    "request_stream",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass
class Snapshot:
    """Positions, velocities (shape (n, 3), float64) and masses (n,) at t = 0."""

    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _plummer_speed_fraction(rng: np.random.Generator, n: int) -> np.ndarray:
    """q = v / v_esc drawn from g(q) ~ q^2 (1 - q^2)^(7/2) by rejection (bound 0.1)."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        want = n - filled
        k = int(want * 1.2) + 64  # acceptance is about 0.49 per draw pair; loop tops up
        q = rng.uniform(0.0, 1.0, k)
        y = rng.uniform(0.0, 0.1, k)
        ok = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(want, ok.size)
        out[filled:filled + take] = ok[:take]
        filled += take
    return out


def plummer(n: int, seed: int, masses: np.ndarray | None = None,
            x_max: float = 0.999) -> Snapshot:
    """Plummer sphere by the Aarseth-Henon-Wielen (1974) recipe, Henon units.

    Radii come from the cumulative mass fraction X ~ U(0, x_max] (the cut keeps the
    radius finite), speeds from the isotropic distribution function by rejection.
    Positions are scaled by 3*pi/16 and velocities by sqrt(16/(3*pi)) so that the
    expected energy is -1/4.  The mass-weighted centre of mass and its velocity are
    removed.  No exact virial rescale is applied (that would need the potential,
    which belongs to the method, not to the input recipe).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    if masses is None:
        m = np.full(n, 1.0 / n)
    else:
        m = np.asarray(masses, dtype=np.float64).copy()
        if m.shape != (n,):
            raise ValueError("masses must have shape (n,)")
    xfrac = x_max * (1.0 - rng.uniform(0.0, 1.0, n))  # in (0, x_max]
    r = 1.0 / np.sqrt(xfrac ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    q = _plummer_speed_fraction(rng, n)
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = speed[:, None] * _isotropic(rng, n)
    pos *= 3.0 * math.pi / 16.0
    vel *= math.sqrt(16.0 / (3.0 * math.pi))
    mt = m.sum()
    pos -= (m[:, None] * pos).sum(axis=0) / mt
    vel -= (m[:, None] * vel).sum(axis=0) / mt
    return Snapshot(pos, vel, m, {"kind": "plummer", "seed": int(seed), "n": n})


def _power_law(rng: np.random.Generator, k: int, alpha: float, lo: float, hi: float) -> np.ndarray:
    """Inverse-CDF draw from dN/dm ~ m^-alpha on [lo, hi] (alpha != 1)."""
    a1 = 1.0 - alpha
    u = rng.uniform(0.0, 1.0, k)
    return (lo ** a1 + u * (hi ** a1 - lo ** a1)) ** (1.0 / a1)


def salpeter_masses(n: int, seed: int, alpha: float = 2.35, lo: float = 1.0,
                    hi: float = 100.0) -> np.ndarray:
    """Salpeter power law dN/dm ~ m^-2.35 on [lo, hi] (range 1:100), normalised to sum 1."""
    m = _power_law(_rng(seed), n, alpha, lo, hi)
    return m / m.sum()


def _kroupa_raw(rng: np.random.Generator, n: int, lo: float = 0.08, brk: float = 0.5,
                hi: float = 100.0, a_low: float = 1.3, a_high: float = 2.3) -> np.ndarray:
    # Continuous two-segment power law: xi(m) = c1 m^-a_low below brk,
    # c2 m^-a_high above, with c2 = c1 brk^(a_high - a_low).
    def seg_int(alpha, a, b):
        e = 1.0 - alpha
        return (b ** e - a ** e) / e
    w1 = seg_int(a_low, lo, brk)
    w2 = brk ** (a_high - a_low) * seg_int(a_high, brk, hi)
    p1 = w1 / (w1 + w2)
    pick = rng.uniform(0.0, 1.0, n) < p1
    out = np.empty(n)
    k1 = int(pick.sum())
    out[pick] = _power_law(rng, k1, a_low, lo, brk)
    out[~pick] = _power_law(rng, n - k1, a_high, brk, hi)
    return out


def kroupa_masses(n: int, seed: int) -> np.ndarray:
    """Kroupa (2001) two-segment IMF on [0.08, 100] (slopes 1.3 / 2.3, break at 0.5), sum 1."""
    m = _kroupa_raw(_rng(seed), n)
    return m / m.sum()


def _kepler_E(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly from the mean anomaly by Newton iteration on E - e sin E = M."""
    E = np.where(e < 0.8, M, np.full_like(M, math.pi))
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E = E - f / (1.0 - e * np.cos(E))
    return E


def with_binaries(n: int, seed: int, frac_members: float = 0.10, a_lo: float = 1e-4,
                  a_hi: float = 1e-2, imf: str = "kroupa") -> Snapshot:
    """Plummer cluster of n bodies in which a fraction of bodies are binary members.

    floor(frac_members * n / 2) pairs are made.  Each pair's centre of mass is one
    particle of the Plummer sample (so the sample has n - n_pairs particles); the pair
    gets a semimajor axis log-uniform in [a_lo, a_hi], a thermal eccentricity
    e = sqrt(U), an isotropic orientation and a uniform mean anomaly.  Component
    masses are drawn from the IMF and the total is normalised to 1.
    """
    rng = _rng(seed)
    n_pairs = int(math.floor(frac_members * n / 2.0))
    n_cm = n - n_pairs
    if imf == "kroupa":
        raw = _kroupa_raw(rng, n)
    elif imf == "equal":
        raw = np.ones(n)
    else:
        raise ValueError(imf)
    raw = raw / raw.sum()
    m1 = raw[:n_pairs]
    m2 = raw[n_pairs:2 * n_pairs]
    singles = raw[2 * n_pairs:]
    cm_mass = np.concatenate([m1 + m2, singles])
    cm = plummer(n_cm, int(rng.integers(0, 2**62)), masses=cm_mass)
    a = np.exp(rng.uniform(math.log(a_lo), math.log(a_hi), n_pairs))
    e = np.sqrt(rng.uniform(0.0, 1.0, n_pairs))
    M = rng.uniform(0.0, 2.0 * math.pi, n_pairs)
    E = _kepler_E(M, e)
    mt = m1 + m2
    # relative orbit in the orbital plane (G = 1)
    cosE, sinE = np.cos(E), np.sin(E)
    sq = np.sqrt(1.0 - e * e)
    rx = a * (cosE - e)
    ry = a * sq * sinE
    rdot = np.sqrt(mt / a) / (1.0 - e * cosE)
    vx = -rdot * sinE
    vy = rdot * sq * cosE
    # random orientation: orthonormal frame from an isotropic normal vector
    nz = _isotropic(rng, n_pairs)
    tmp = np.where(np.abs(nz[:, 0:1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    ex = np.cross(nz, tmp)
    ex /= np.linalg.norm(ex, axis=1)[:, None]
    ey = np.cross(nz, ex)
    rel_x = rx[:, None] * ex + ry[:, None] * ey
    rel_v = vx[:, None] * ex + vy[:, None] * ey
    x = np.empty((n, 3))
    v = np.empty((n, 3))
    m = np.empty(n)
    f1 = (m2 / mt)[:, None]
    f2 = (m1 / mt)[:, None]
    x[0:2 * n_pairs:2] = cm.x[:n_pairs] + f1 * rel_x
    x[1:2 * n_pairs:2] = cm.x[:n_pairs] - f2 * rel_x
    v[0:2 * n_pairs:2] = cm.v[:n_pairs] + f1 * rel_v
    v[1:2 * n_pairs:2] = cm.v[:n_pairs] - f2 * rel_v
    m[0:2 * n_pairs:2] = m1
    m[1:2 * n_pairs:2] = m2
    x[2 * n_pairs:] = cm.x[n_pairs:]
    v[2 * n_pairs:] = cm.v[n_pairs:]
    m[2 * n_pairs:] = singles
    meta = {"kind": "plummer+binaries", "seed": int(seed), "n": n, "n_pairs": n_pairs,
            "a": a, "e": e,
            # the members of pair k are bodies 2k and 2k + 1
            "pairs": np.arange(2 * n_pairs, dtype=np.int64).reshape(-1, 2)}
    return Snapshot(x, v, m, meta)


@dataclass
class Request:
    """One ensemble-serving request: an initial condition to integrate to t_end."""

    rid: int
    arrival: float          # seconds after the start of the stream
    n: int
    seed: int
    eps: float
    t_end: float
    kind: str = "plummer"   # "plummer" (equal mass) or "kroupa_binaries"

    def snapshot(self) -> Snapshot:
        if self.kind == "plummer":
            return plummer(self.n, self.seed)
        if self.kind == "kroupa_binaries":
            return with_binaries(self.n, self.seed)
        raise ValueError(self.kind)


def request_stream(count: int, seed: int, n_lo: int, n_hi: int, rate: float,
                   eps: float, t_end: float, kind: str = "plummer",
                   ic_seed_base: int = 0) -> list[Request]:
    """Poisson stream: exponential gaps at `rate` per second, N log-uniform in [n_lo, n_hi].

    Sizes and arrival gaps come from independent streams of the seed, so the same seed
    gives the same requests at every rate (rate <= 0: all arrive at t = 0)."""
    size_rng, gap_rng = (np.random.Generator(np.random.PCG64(s))
                         for s in np.random.SeedSequence(int(seed)).spawn(2))
    ns = np.rint(np.exp(size_rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    gaps = gap_rng.exponential(1.0 / rate, count) if rate > 0 else np.zeros(count)
    arr = np.cumsum(gaps) - (gaps[0] if count else 0.0)
    ns = np.clip(ns, n_lo, n_hi)
    return [Request(k, float(arr[k]), int(ns[k]), ic_seed_base + k, eps, t_end, kind)
            for k in range(count)]
