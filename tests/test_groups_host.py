"""Host (CPU) parts of the tight-pair treatment in libnbody.so, against the oracle
and the Kepler closed form.  No GPU is used: these are the library's CPU-thread
routines (the HiGPUs-R scheme of Sec. 3 runs them beside the GPU kernels)."""
import ctypes as C
import math

import numpy as np
import pytest

from test_oracle_hermite import kepler_state


@pytest.fixture(scope="module")
def L():
    from paper_1411_5234_amd import _lib
    return _lib.load()


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _drift(L, M, r0, v0, dt):
    r0, v0 = np.ascontiguousarray(r0, float), np.ascontiguousarray(v0, float)
    r1, v1 = np.empty(3), np.empty(3)
    rc = L.nb_kepler_drift(float(M), _p(r0), _p(v0), float(dt), _p(r1), _p(v1))
    return rc, r1, v1


@pytest.mark.parametrize("e", [0.0, 0.4, 0.95, 0.9999])
@pytest.mark.parametrize("t", [1e-3, 0.8, -3.1, 57.0])
def test_library_drift_matches_oracle_and_closed_form(L, orc, e, t):
    x0, v0 = kepler_state(0.35, 0.65, 0.7, e, 0.0, M0=1.1)
    r0, w0 = x0[1] - x0[0], v0[1] - v0[0]
    rc, r1, w1 = _drift(L, 1.0, r0, w0, t)
    assert rc == 0
    ro, wo = orc.kepler_drift(1.0, r0, w0, t)
    vs = np.abs(wo).max() + 1.0
    assert np.abs(r1 - ro).max() <= 1e-11 * (1 + abs(t))
    assert np.abs(w1 - wo).max() <= 1e-11 * (1 + abs(t)) * vs
    if e < 0.99:
        xe, ve = kepler_state(0.35, 0.65, 0.7, e, t, M0=1.1)
        assert np.abs(r1 - (xe[1] - xe[0])).max() <= 1e-11 * (1 + abs(t))


def test_library_drift_refuses_unbound_and_bad_input(L):
    rc, _, _ = _drift(L, 1.0, [1.0, 0, 0], [0, 1.5, 0], 0.1)
    assert rc == -7
    rc, _, _ = _drift(L, 0.0, [1.0, 0, 0], [0, 0.5, 0], 0.1)
    assert rc == -7
    rc, _, _ = _drift(L, 1.0, [1.0, 0, 0], [0, 0.5, 0], float("nan"))
    assert rc == -1


def test_library_group_advance_matches_oracle(L, orc):
    rng = np.random.default_rng(11)
    n = 40
    M = rng.uniform(0.5, 2.0, n)
    r = np.empty((n, 3))
    v = np.empty((n, 3))
    for k in range(n):
        x0, v0 = kepler_state(0.5 * M[k], 0.5 * M[k], rng.uniform(0.2, 1.0), rng.uniform(0, 0.97),
                              0.0, M0=rng.uniform(0, 6.28))
        r[k], v[k] = x0[1] - x0[0], v0[1] - v0[0]
    A = rng.normal(size=(n, 3, 3)) * 0.01
    T0 = A + np.transpose(A, (0, 2, 1))
    B = rng.normal(size=(n, 3, 3)) * 0.01
    T1 = T0 + B + np.transpose(B, (0, 2, 1))
    H = rng.uniform(0.0, 5.0, n)
    H[0] = 0.0
    rl, vl = r.copy(), v.copy()
    status = np.full(n, 99, dtype=np.int32)
    rc = L.nb_groups_advance(n, None, _p(M), _p(rl), _p(vl), _p(H), _p(np.ascontiguousarray(T0)),
                             _p(np.ascontiguousarray(T1)), 32, 1 << 20, _p(status))
    assert rc == 0 and np.all(status == 0)
    for k in range(n):
        Mk, rk, vk = M[k], r[k], v[k]
        ns = orc.substeps(Mk, rk, vk, H[k], 32) if H[k] > 0 else 1
        ro, vo = orc.group_advance(Mk, rk, vk, H[k], ns, T0[k], T1[k])
        assert np.abs(rl[k] - ro).max() <= 1e-10, k
        assert np.abs(vl[k] - vo).max() <= 1e-10 * (1 + np.abs(vo).max()), k
    np.testing.assert_array_equal(rl[0], r[0])


def test_library_group_advance_reports_unbound_pairs(L):
    M = np.array([1.0, 1.0])
    r = np.array([[1.0, 0, 0], [1.0, 0, 0]])
    v = np.array([[0, 0.5, 0], [0, 2.0, 0]])     # the second is unbound
    H = np.array([0.3, 0.3])
    Z = np.zeros((2, 9))
    status = np.zeros(2, dtype=np.int32)
    rc = L.nb_groups_advance(2, None, _p(M), _p(r), _p(v), _p(H), _p(Z), _p(Z), 32, 1 << 20, _p(status))
    assert rc == -7 and list(status) == [0, -7]
    assert L.nb_groups_advance(2, None, _p(M), _p(r), _p(v), _p(H), _p(Z), _p(Z), 0, 1 << 20,
                               None) == -1


def _pairs(seed, n):
    rng = np.random.default_rng(seed)
    M = rng.uniform(0.5, 2.0, n)
    r, v = np.empty((n, 3)), np.empty((n, 3))
    for k in range(n):
        x0, v0 = kepler_state(0.5 * M[k], 0.5 * M[k], rng.uniform(0.2, 1.0), rng.uniform(0, 0.9),
                              0.0, M0=rng.uniform(0, 6.28))
        r[k], v[k] = x0[1] - x0[0], v0[1] - v0[0]
    A = rng.normal(size=(n, 9)) * 0.01
    return M, r, v, A


def test_library_group_advance_by_rows_equals_gathered_call(L):
    """Rows named by idx advance exactly as the same pairs passed contiguously;
    rows not named are left alone."""
    n = 12
    M, r, v, T = _pairs(5, n)
    idx = np.array([7, 2, 11, 0], dtype=np.int32)
    H = np.array([0.3, 1.1, 0.0, 2.5])
    T0 = np.ascontiguousarray(T[:4])
    T1 = np.ascontiguousarray(T[4:8])
    rr, vv = r.copy(), v.copy()
    status = np.full(n, 99, dtype=np.int32)
    assert L.nb_groups_advance(4, _p(idx), _p(M), _p(rr), _p(vv), _p(H), _p(T0), _p(T1), 32,
                               1 << 20, _p(status)) == 0
    Mg, rg, vg = M[idx].copy(), r[idx].copy(), v[idx].copy()
    assert L.nb_groups_advance(4, None, _p(Mg), _p(rg), _p(vg), _p(H), _p(T0), _p(T1), 32,
                               1 << 20, None) == 0
    np.testing.assert_array_equal(rr[idx], rg)
    np.testing.assert_array_equal(vv[idx], vg)
    rest = np.setdiff1d(np.arange(n), idx)
    np.testing.assert_array_equal(rr[rest], r[rest])
    np.testing.assert_array_equal(vv[rest], v[rest])
    assert list(status[idx]) == [0] * 4 and np.all(status[rest] == 99)


@pytest.mark.parametrize("idx", [[1, 1], [0, -1]])
def test_library_group_advance_refuses_repeated_or_negative_rows(L, idx):
    M, r, v, T = _pairs(6, 3)
    idx = np.array(idx, dtype=np.int32)
    H = np.array([0.1, 0.1])
    T0 = np.ascontiguousarray(T[:2])
    rr = r.copy()
    assert L.nb_groups_advance(2, _p(idx), _p(M), _p(rr), _p(v.copy()), _p(H), _p(T0), _p(T0),
                               32, 1 << 20, None) == -1
    np.testing.assert_array_equal(rr, r)


def _reduce(L, x, v, m, pairs):
    n, k = m.size, len(pairs)
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    xr, vr, mr = np.empty((n - k, 3)), np.empty((n - k, 3)), np.empty(n - k)
    M, r, w = np.empty(max(k, 1)), np.empty((max(k, 1), 3)), np.empty((max(k, 1), 3))
    rc = L.nb_pairs_reduce(n, _p(x), _p(v), _p(m), k, _p(pairs), _p(xr), _p(vr), _p(mr), _p(M),
                           _p(r), _p(w))
    return rc, xr, vr, mr, M[:k], r[:k], w[:k]


def test_pairs_reduce_members_energy_match_oracle(L, orc):
    """The library's reduction to centre-of-mass bodies equals the oracle's grouped
    startup state, the members it reconstructs are the inputs (to rounding), and the
    pairs' energy is the oracle's grouped energy less the reduced system's."""
    from paper_1411_5234_amd import inputs
    s = inputs.with_binaries(600, 7)
    pairs = s.meta["pairs"]
    x, v, m = (np.ascontiguousarray(a) for a in (s.x, s.v, s.m))
    rc, xr, vr, mr, M, r, w = _reduce(L, x, v, m, pairs)
    assert rc == 0
    eps = 1e-5
    g = orc.group_startup(x, v, m, pairs, orc.Params(eps=eps))
    np.testing.assert_array_equal(mr, g.st.m)
    np.testing.assert_array_equal(M, g.M)
    np.testing.assert_array_equal(r, g.r)
    np.testing.assert_array_equal(w, g.w)
    np.testing.assert_allclose(xr, g.st.x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(vr, g.st.v, rtol=0, atol=1e-15)
    xo, vo = np.empty_like(x), np.empty_like(v)
    rc = L.nb_pairs_members(m.size, _p(xr), _p(vr), _p(m), len(pairs), _p(np.ascontiguousarray(pairs)),
                            _p(r), _p(w), _p(xo), _p(vo))
    assert rc == 0
    np.testing.assert_allclose(xo, x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(vo, v, rtol=0, atol=1e-13)
    out = C.c_double()
    T = np.ascontiguousarray(g.T.reshape(-1, 9))
    rc = L.nb_pairs_energy(len(pairs), _p(m), _p(np.ascontiguousarray(pairs)), _p(r), _p(w), _p(T),
                           C.byref(out))
    assert rc == 0
    want = orc.group_energy(g, m, eps) - orc.energy(g.st.x, g.st.v, g.st.m, eps)[2]
    assert abs(out.value - want) <= 1e-12 * abs(want)


def test_pairs_reduce_rejects_bad_pairs(L):
    x = np.zeros((4, 3)); v = np.zeros((4, 3)); m = np.ones(4)
    assert _reduce(L, x, v, m, [(0, 1), (1, 2)])[0] == -1     # index twice
    assert _reduce(L, x, v, m, [(0, 4)])[0] == -1             # out of range
    assert _reduce(L, x, v, m, [(0, 1), (2, 3)])[0] == 0


def test_pair_perturbation_and_split_energy(L):
    """Semimajor axis of a circular and an eccentric orbit (vis-viva), the
    perturbation |T| (2a)^3 / M of an isotropic tensor, unbound pairs, the
    input-a form, and the change of the pair potential at a return."""
    M = np.array([2.0, 2.0, 2.0])
    a_c, rp, e = 0.3, 0.1, 0.5
    r = np.array([[a_c, 0, 0], [rp, 0, 0], [0.1, 0, 0]])
    w = np.array([[0, math.sqrt(M[0] / a_c), 0],
                  [0, math.sqrt(M[1] * (1 + e) / rp), 0],     # pericentre of a = rp / (1 - e)
                  [0, 10.0, 0]])                               # unbound
    T = np.zeros((3, 9))
    T[:, [0, 4, 8]] = 0.7
    a, g = np.empty(3), np.empty(3)
    assert L.nb_pairs_perturbation(3, _p(M), _p(r), _p(w), _p(T), _p(a), _p(g)) == 0
    np.testing.assert_allclose(a[:2], [a_c, rp / (1 - e)], rtol=1e-13)
    np.testing.assert_allclose(g[:2], 0.7 * math.sqrt(3) * (2 * a[:2]) ** 3 / 2.0, rtol=1e-13)
    assert math.isinf(a[2]) and math.isinf(g[2])
    a2, g2 = a[:2].copy(), np.empty(2)
    assert L.nb_pairs_perturbation(2, _p(M), None, None, None, _p(a2), _p(g2)) == 0
    assert np.all(g2 == 0.0)
    m = np.array([0.3, 0.5, 0.2, 0.1])
    pairs = np.array([[0, 1], [2, 3]], dtype=np.int64)
    rr = np.array([[1e-3, 0, 0], [0, 2e-4, 0]])
    out = C.c_double()
    assert L.nb_pairs_split_energy(2, _p(m), _p(pairs), _p(rr), 1e-5, C.byref(out)) == 0
    want = sum(m[i] * m[j] * (1 / np.linalg.norm(q) - 1 / math.hypot(np.linalg.norm(q), 1e-5))
               for (i, j), q in zip(pairs, rr))
    assert abs(out.value - want) <= 1e-14 * abs(want)


def test_pair_table_segments_compaction_and_removal(L):
    """Several systems' pairs in one table: each set reads and writes only its own
    segment, a released segment is reclaimed when the table compacts (rows keep
    their values), and a set without some pairs keeps the others' state."""
    from paper_1411_5234_amd import inputs
    from paper_1411_5234_amd.groups import PairSet, PairTable
    tab = PairTable(L, capacity=4)
    snaps = [inputs.with_binaries(n, seed) for n, seed in ((200, 1), (300, 2), (260, 3))]
    sets = [PairSet(L, s.x, s.v, s.m, s.meta["pairs"], tab) for s in snaps]
    assert [ps.np for ps in sets] == [10, 15, 13] and tab.cap >= 38
    for q, ps in enumerate(sets):
        ps.T[:] = q + 1.0
        ps.tpair[:] = 0.25 * q
    r1 = sets[1].r.copy()
    sets[0].release()
    extra = PairSet(L, snaps[0].x, snaps[0].v, snaps[0].m, snaps[0].meta["pairs"], tab)
    tab.reserve(tab.cap - tab.used + 1)          # forces a compaction (and growth)
    assert sets[1].base == 0 and np.array_equal(sets[1].r, r1)
    assert np.all(sets[1].T == 2.0) and np.all(sets[2].T == 3.0) and np.all(sets[2].tpair == 0.5)
    assert extra.base == sets[1].np + sets[2].np
    # advancing rows of the table equals advancing the set's own rows
    ps = sets[2]
    alone = PairSet(L, snaps[2].x, snaps[2].v, snaps[2].m, snaps[2].meta["pairs"])
    T1 = np.full((ps.np, 9), 0.1)
    for s_ in (ps, alone):
        s_.T[:] = 0.0
        s_.tpair[:] = 0.0
    ctx = type("Ctx", (), {"L": L})()
    ps.advance(ctx, np.arange(ps.np), 1e-3, T1, 32, 1 << 20, queue=False)
    alone.advance(ctx, np.arange(alone.np), 1e-3, T1, 32, 1 << 20, queue=False)
    assert np.array_equal(ps.r, alone.r) and np.array_equal(ps.w, alone.w)
    # dropping pairs keeps the others' orbits, tensors and times
    keep_r = ps.r[[0, 2, 3]].copy()
    out = ps.without([1] + list(range(4, ps.np)))
    assert out.np == 3 and np.array_equal(out.r, keep_r) and np.all(out.tpair == 1e-3)
    assert out.cm0 == out.n - 2 * out.np and ps not in tab.sets and out in tab.sets


def test_members_of_some_pairs_match_the_full_reconstruction(L):
    from paper_1411_5234_amd import inputs
    from paper_1411_5234_amd.groups import PairSet
    s = inputs.with_binaries(400, 11)
    ps = PairSet(L, s.x, s.v, s.m, s.meta["pairs"])
    x, v = ps.members(ps.xr, ps.vr)
    np.testing.assert_allclose(x, s.x, rtol=0, atol=1e-15)
    ks = np.array([3, 0, 7])
    xm, vm = ps.members_of(ks, ps.xr[ps.cm0 + ks], ps.vr[ps.cm0 + ks])
    rows = ps.pairs[ks].ravel()
    assert np.array_equal(xm, x[rows]) and np.array_equal(vm, v[rows])


def test_pairs_added_during_a_run_keep_the_layout_and_the_old_pairs(L):
    """PairSet.with_pairs: the old pairs keep their rows' orbits, tensors and times;
    the new ones follow them; the reduced layout (bodies in no pair in index order,
    then the centres of mass in pair order) is the one a fresh PairSet of all the
    pairs makes from the same state."""
    from paper_1411_5234_amd import inputs
    from paper_1411_5234_amd.groups import PairSet, PairTable
    s = inputs.with_binaries(300, 12)
    pairs = s.meta["pairs"]
    tab = PairTable(L, 4)
    old = PairSet(L, s.x, s.v, s.m, pairs[:5], tab)
    old.T[:] = np.arange(45.0).reshape(5, 9)
    old.tpair[:] = 0.25
    other = PairSet(L, s.x, s.v, s.m, pairs[9:11], tab)       # another system in the table
    other.T[:] = 7.0
    full = PairSet(L, s.x, s.v, s.m, pairs[:8])
    new = old.with_pairs(pairs[5:8], full.M[5:8], full.r[5:8], full.w[5:8],
                         np.ones((3, 9)), full.a0[5:8], 0.5)
    assert new.np == 8 and new.cm0 == full.cm0
    assert np.array_equal(new.pairs, full.pairs) and np.array_equal(new.singles, full.singles)
    for f in ("M", "r", "w", "a0"):
        assert np.array_equal(getattr(new, f), getattr(full, f)), f
    assert np.array_equal(new.T[:5], np.arange(45.0).reshape(5, 9))
    assert np.all(new.T[5:] == 1.0) and np.all(new.tpair[:5] == 0.25) and np.all(new.tpair[5:] == 0.5)
    assert np.all(other.T == 7.0)                               # untouched by the move
    assert old not in tab.sets and new in tab.sets
    with pytest.raises(ValueError):
        new.with_pairs([[pairs[0][0], pairs[9][0]]], [1.0], np.ones((1, 3)), np.ones((1, 3)),
                       np.zeros((1, 9)), [1.0], 0.5)
    assert new in tab.sets                                      # a refused call changes nothing
    empty = PairSet(L, s.x, s.v, s.m, np.zeros((0, 2), dtype=np.int64))
    assert empty.np == 0 and empty.cm0 == 300 and np.array_equal(empty.xr, s.x)
