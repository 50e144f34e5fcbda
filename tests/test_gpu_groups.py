"""GPU parity of the tight-pair treatment (the HiGPUs-R scheme of Sec. 3, with
bound pairs as the groups): nb_tidal_active against the oracle's tidal tensor, and
the grouped block-step integration (GPU block steps + CPU-thread pair advance,
overlapped) against the oracle's grouped integration."""
import numpy as np
import pytest
import torch

from gpu_helpers import device_system
from paper_1411_5234_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


def _gpu_tidal(ctx, sys, ilist, eps, j0=0, j1=None):
    n = sys.n
    m = len(ilist)
    idx = torch.as_tensor(np.asarray(ilist, dtype=np.int32), device="cuda")
    T = torch.full((9 * max(m, 1),), np.nan, dtype=torch.float64, device="cuda")
    ctx._check(ctx.L.nb_tidal_active(ctx.h, sys.ref, idx.data_ptr(), m, j0, n if j1 is None else j1,
                                     float(eps), T.data_ptr()))
    ctx.sync()
    return T[: 9 * m].view(9, m).T.cpu().numpy().reshape(m, 3, 3)


@pytest.mark.parametrize("eps", [1e-3, 0.0])
def test_tidal_matches_oracle(ctx, orc, eps):
    s = inputs.plummer(3000, 81, masses=inputs.salpeter_masses(3000, 82))
    sys = device_system(s.x, s.v, s.m)
    il = np.sort(np.random.default_rng(83).choice(3000, 77, replace=False))
    for j0, j1 in [(0, 3000), (13, 2911), (0, 1), (2999, 3000)]:
        g = _gpu_tidal(ctx, sys, il, eps, j0, j1)
        o = orc.tidal(s.x, s.m, eps, il, j0, j1)
        scale = np.abs(o).max(axis=(1, 2)) + 1e-300
        err = np.abs(g - o).max(axis=(1, 2)) / scale
        print("tidal eps=%g [%d,%d): max rel %.3e" % (eps, j0, j1, err.max()), flush=True)
        assert err.max() <= 1e-12


def test_tidal_at_points_matches_oracle(ctx, orc):
    """The field of the rest of the system at arbitrary points, two bodies left out
    per point (the centre of mass of a pair about to be formed)."""
    s = inputs.plummer(2500, 91, masses=inputs.salpeter_masses(2500, 92))
    sys = device_system(s.x, s.v, s.m)
    rng = np.random.default_rng(93)
    k = 37
    a = rng.choice(2500, k, replace=False)
    b = rng.choice(2500, k, replace=False)
    pts = 0.5 * (s.x[a] + s.x[b])
    pts[0] = s.x[a[0]]                       # a point on a body that is left out
    excl = np.stack([a, b], axis=1)
    excl[1] = -1                             # nothing left out
    excl[2, 1] = -1
    P = torch.as_tensor(np.ascontiguousarray(pts.T).ravel(), device="cuda")
    E = torch.as_tensor(np.ascontiguousarray(excl.T).ravel().astype(np.int32), device="cuda")
    for eps in (1e-3, 0.0):
        if eps == 0.0:
            pts_e, excl_e = pts[1:], excl[1:]
            P = torch.as_tensor(np.ascontiguousarray(pts_e.T).ravel(), device="cuda")
            E = torch.as_tensor(np.ascontiguousarray(excl_e.T).ravel().astype(np.int32),
                                device="cuda")
        else:
            pts_e, excl_e = pts, excl
        kk = len(pts_e)
        T = torch.full((9 * kk,), np.nan, dtype=torch.float64, device="cuda")
        ctx._check(ctx.L.nb_tidal_points(ctx.h, sys.ref, kk, P.data_ptr(), E.data_ptr(), eps,
                                         T.data_ptr()))
        ctx.sync()
        g = T.view(9, kk).T.cpu().numpy().reshape(kk, 3, 3)
        o = orc.tidal_points(s.x, s.m, eps, pts_e, excl_e)
        err = np.abs(g - o).max(axis=(1, 2)) / np.abs(o).max(axis=(1, 2))
        print("tidal at points eps=%g: max rel %.3e" % (eps, err.max()), flush=True)
        assert err.max() <= 1e-12


def _gpu_nearest(ctx, systems):
    """nb_nearest_active_batch over several (sys, rows, row_end, dt_cap) items."""
    from paper_1411_5234_amd._lib import NbNearestItem
    items = (NbNearestItem * len(systems))()
    keep = []
    for q, (sys, rows, row_end, cap) in enumerate(systems):
        m = len(rows)
        idx = torch.as_tensor(np.asarray(rows, dtype=np.int32), device="cuda")
        nn = torch.full((max(m, 1),), -7, dtype=torch.int32, device="cuda")
        r2 = torch.full((max(m, 1),), np.nan, dtype=torch.float64, device="cuda")
        keep.append((idx, nn, r2, m))
        it = items[q]
        it.sys = sys._struct
        it.i_idx = idx.data_ptr()
        it.m = m
        it.row_end = row_end
        it.dt_cap = cap
        it.nn = nn.data_ptr()
        it.r2 = r2.data_ptr()
        it.status = None
    ctx._check(ctx.L.nb_nearest_active_batch(ctx.h, items, len(systems)))
    ctx.sync()
    return [(nn[:m].cpu().numpy().astype(np.int64), r2[:m].cpu().numpy()) for _, nn, r2, m in keep]


def test_nearest_matches_oracle_exactly(ctx, orc):
    """Nearest-neighbour indices and squared distances, bit for bit: ragged systems
    in one launch (one body; a few tiles with a ragged tail; C5-sized), coincident
    bodies and equal distances planted, rows filtered by index and by step."""
    rng = np.random.default_rng(101)
    cases = []
    for n, seed in ((1, 1), (2, 2), (700, 3), (5003, 4), (65536, 5)):
        s = inputs.plummer(n, 100 + seed)
        x = s.x.copy()
        if n >= 700:
            x[5] = x[17]                                     # coincident
            x[30] = [0.5, 0.25, 0.125]                       # exactly equal distances
            x[40] = [0.5, 0.25 + 2.0 ** -10, 0.125]          # from 30 (exact differences)
            x[50] = [0.5, 0.25 - 2.0 ** -10, 0.125]
        sys = device_system(x, s.v, s.m)
        dt = rng.choice([2.0 ** -14, 2.0 ** -8, 2.0 ** -3], n)
        sys.buf64[14, :n] = torch.as_tensor(dt, device="cuda")
        m = min(n, 512)
        rows = np.sort(rng.choice(n, m, replace=False)) if n > m else np.arange(n)
        if n >= 700:
            rows = np.unique(np.concatenate([rows, [5, 17, 30, 40, 50]]))
        row_end = n if seed % 2 else max(n - 100, 0)
        cap = np.inf if seed % 2 else 2.0 ** -8
        cases.append((sys, rows, row_end, cap, x, dt))
    got = _gpu_nearest(ctx, [(c[0], c[1], c[2], c[3]) for c in cases])
    for (sys, rows, row_end, cap, x, dt), (nn, r2) in zip(cases, got):
        onn, or2 = orc.nearest(x, rows, row_end, dt, cap)
        print("nearest n=%d rows=%d searched=%d" % (len(x), len(rows), int((onn >= 0).sum())),
              flush=True)
        assert np.array_equal(nn, onn)
        assert np.array_equal(r2, or2)
    # the planted cases (n = 700: every row searched)
    rows, (nn, r2) = cases[2][1], got[2]
    at = {int(r): q for q, r in enumerate(rows)}
    assert nn[at[5]] == 17 and nn[at[17]] == 5 and r2[at[5]] == 0.0
    assert nn[at[30]] == 40                                  # the lower of two equal distances


def _cluster(a_hi=1e-3):
    s = inputs.with_binaries(160, 10, frac_members=0.2, a_lo=1e-4, a_hi=a_hi, imf="equal")
    return s, [(2 * k, 2 * k + 1) for k in range(16)]


def _elements(M, r, w):
    """Kepler energy, angular momentum and Laplace-Runge-Lenz vector per pair."""
    rn = np.linalg.norm(r, axis=1)
    E = 0.5 * (w ** 2).sum(1) - M / rn
    h = np.cross(r, w)
    lrl = np.cross(w, h) / M[:, None] - r / rn[:, None]
    return E, h, lrl


def test_grouped_integration_matches_oracle(ctx, orc):
    """FP64 path.  The reduced system (single bodies and centres of mass) must follow
    the oracle's to rounding and take the same block steps.  The pairs' relative
    orbits are advanced by two independent FP64 implementations over up to ~2e3
    orbits and ~1e5 substeps: rounding differences of ~1e-15 per substep shift
    the orbital phase quadratically in the number of substeps (Kepler shear), so
    the phase is compared loosely and the orbital elements, which the shear
    leaves alone, tightly."""
    from paper_1411_5234_amd.groups import GroupedIntegrator
    from paper_1411_5234_amd.nbody import Params
    s, pairs = _cluster()
    eps = 1e-5
    gi = GroupedIntegrator(ctx, s.x, s.v, s.m, pairs, Params(eps=eps, precision="fp64"))
    gi.startup()
    e0 = gi.energy()
    glog = []
    steps, _ = gi.run(0.125, log=glog)
    x, v = gi.members()
    olog = []
    xo, vo, osteps, g = orc.group_integrate(s.x, s.v, s.m, pairs, 0.125, orc.Params(eps=eps),
                                            log=olog)
    print("GPU %d block steps, oracle %d; pairs advanced on the CPU: %d" % (
        steps, osteps, gi.cpu_pairs_advanced), flush=True)
    assert steps == osteps
    for (tg, ig), (to, io) in zip(glog, olog):
        assert tg == to and np.array_equal(ig, io)
    st = gi.sys.state_numpy()
    assert np.abs(st["x"] - g.st.x).max() <= 1e-12
    assert np.abs(st["v"] - g.st.v).max() <= 1e-12 * (1 + np.abs(g.st.v).max())
    Eg, hg, lg = _elements(gi.M, gi.r, gi.w)
    Eo, ho, lo = _elements(g.M, g.r, g.w)
    dE = np.abs(Eg - Eo) / np.abs(Eo)
    dh = np.abs(hg - ho).max(1) / np.linalg.norm(ho, axis=1)
    dl = np.abs(lg - lo).max(1)
    dr = np.abs(gi.r - g.r).max(1) / np.linalg.norm(g.r, axis=1)
    print("pairs: max rel energy %.2e, angular momentum %.2e, |dLRL| %.2e, phase (|dr|/r) %.2e"
          % (dE.max(), dh.max(), dl.max(), dr.max()), flush=True)
    assert dE.max() <= 1e-8 and dh.max() <= 1e-8 and dl.max() <= 1e-8
    assert dr.max() <= 1e-4
    assert np.abs(x - xo).max() <= 1e-4 * np.linalg.norm(g.r, axis=1).max()
    e1 = gi.energy()
    assert abs(e1 - e0) / abs(e0) < 1e-6
    assert abs(e1 - orc.group_energy(g, s.m, eps)) <= 1e-8 * abs(e1)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_overlap_does_not_change_the_result(ctx, precision):
    from paper_1411_5234_amd.groups import GroupedIntegrator
    from paper_1411_5234_amd.nbody import Params
    s, pairs = _cluster(3e-4)
    out = []
    for overlap in (True, False):
        gi = GroupedIntegrator(ctx, s.x, s.v, s.m, pairs, Params(eps=1e-5, precision=precision),
                               overlap=overlap)
        gi.startup()
        e0 = gi.energy()
        gi.run(0.0625)
        out.append(gi.members())
        e1 = gi.energy()
        print("%s overlap=%s: scheme |dE/E| = %.3e" % (precision, overlap, abs(e1 - e0) / abs(e0)),
              flush=True)
        assert abs(e1 - e0) / abs(e0) < 1e-5
    assert out[0][0].tobytes() == out[1][0].tobytes()
    assert out[0][1].tobytes() == out[1][1].tobytes()


def test_unbound_pair_is_reported(ctx):
    from paper_1411_5234_amd import _lib
    from paper_1411_5234_amd.groups import GroupedIntegrator
    from paper_1411_5234_amd.nbody import Params
    s = inputs.plummer(64, 84)
    x, v = s.x.copy(), s.v.copy()
    v[1] = v[0] + np.array([10.0, 0.0, 0.0])      # bodies 0 and 1: far from bound
    gi = GroupedIntegrator(ctx, x, v, s.m, [(0, 1)], Params(eps=1e-3, precision="fp64"))
    gi.startup()
    with pytest.raises(_lib.NbError) as e:
        gi.run(0.125)
    assert e.value.name == "NB_EUNBOUND"


def test_queued_advances_run_in_call_order(ctx):
    """Queued calls that name the same rows run one after another, in call order:
    the result equals the same calls made on the calling thread, bitwise; a failure
    is reported by the next wait only."""
    import ctypes as C

    def p(a):
        return a.ctypes.data_as(C.c_void_p)

    rng = np.random.default_rng(31)
    n = 6
    M = rng.uniform(0.5, 2.0, n)
    r = rng.normal(size=(n, 3))
    rn = np.linalg.norm(r, axis=1)
    w = np.cross(r, rng.normal(size=(n, 3)))
    w *= (0.8 * np.sqrt(M / rn) / np.linalg.norm(w, axis=1))[:, None]
    calls = []
    for q in range(40):
        k = int(rng.integers(1, n + 1))
        rows = np.ascontiguousarray(rng.choice(n, k, replace=False), dtype=np.int32)
        H = rng.uniform(0.0, 0.7, k)
        T0 = rng.normal(size=(k, 9)) * 1e-3
        T1 = rng.normal(size=(k, 9)) * 1e-3
        calls.append((rows, H, T0, T1))
    res = []
    for queued in (True, False):
        rr, ww = r.copy(), w.copy()
        st = np.full(n, 99, dtype=np.int32)
        for rows, H, T0, T1 in calls:
            args = (rows.size, p(rows), p(M), p(rr), p(ww), p(H), p(T0), p(T1), 32, 1 << 20, p(st))
            if queued:
                assert ctx.L.nb_groups_advance_async(ctx.h, *args) == 0
            else:
                assert ctx.L.nb_groups_advance(*args) == 0
        if queued:
            assert ctx.L.nb_groups_wait(ctx.h) == 0
        assert np.all(st == 0)
        res.append((rr, ww))
    assert res[0][0].tobytes() == res[1][0].tobytes()
    assert res[0][1].tobytes() == res[1][1].tobytes()

    # an unbound row fails its call; the queue goes on and the next wait reports it
    wb = w.copy()
    wb[2] *= 5.0
    rr = r.copy()
    st = np.zeros(n, dtype=np.int32)
    rows = np.arange(n, dtype=np.int32)
    H = np.full(n, 0.1)
    Z = np.zeros((n, 9))
    for _ in range(3):
        assert ctx.L.nb_groups_advance_async(ctx.h, n, p(rows), p(M), p(rr), p(wb), p(H), p(Z),
                                             p(Z), 32, 1 << 20, p(st)) == 0
    assert ctx.L.nb_groups_wait(ctx.h) == -7
    assert list(st) == [0, 0, -7, 0, 0, 0]
    assert ctx.L.nb_groups_wait(ctx.h) == 0


def test_capture_calls_refuse_bad_arguments(ctx, orc):
    """nb_tidal_points and nb_nearest_active_batch check their arguments before
    anything is enqueued; an active index outside the system is reported in the
    item's status word and its row is not searched."""
    from paper_1411_5234_amd._lib import NbError, NbNearestItem
    s = inputs.plummer(300, 5)
    sys = device_system(s.x, s.v, s.m)
    P = torch.zeros(3, dtype=torch.float64, device="cuda")
    T = torch.zeros(9, dtype=torch.float64, device="cuda")
    for k, pts, eps in ((1, P.data_ptr(), -1.0), (-1, P.data_ptr(), 1e-3), (1, None, 1e-3)):
        with pytest.raises(NbError) as e:
            ctx._check(ctx.L.nb_tidal_points(ctx.h, sys.ref, k, pts, None, eps, T.data_ptr()))
        assert e.value.name == "NB_EINVAL"
    ctx._check(ctx.L.nb_tidal_points(ctx.h, sys.ref, 0, None, None, 1e-3, None))   # no-op

    idx = torch.as_tensor(np.array([3, 300, 7], dtype=np.int32), device="cuda")
    nn = torch.full((3,), -7, dtype=torch.int32, device="cuda")
    r2 = torch.zeros(3, dtype=torch.float64, device="cuda")
    word = torch.zeros(1, dtype=torch.int32, device="cuda")

    def item(m=3, cap=np.inf, nnp=None):
        it = (NbNearestItem * 1)()
        it[0].sys = sys._struct
        it[0].i_idx = idx.data_ptr()
        it[0].m = m
        it[0].row_end = 300
        it[0].dt_cap = cap
        it[0].nn = nn.data_ptr() if nnp is None else nnp
        it[0].r2 = r2.data_ptr()
        it[0].status = word.data_ptr()
        return it

    for bad in (item(m=301), item(cap=float("nan")), item(nnp=0)):
        with pytest.raises(NbError) as e:
            ctx._check(ctx.L.nb_nearest_active_batch(ctx.h, bad, 1))
        assert e.value.name == "NB_EINVAL"
    ctx._check(ctx.L.nb_nearest_active_batch(ctx.h, item(m=0), 1))           # skipped
    ctx._check(ctx.L.nb_nearest_active_batch(ctx.h, item(), 1))
    ctx.sync()
    got = nn.cpu().numpy()
    assert got[1] == -1 and got[0] >= 0 and got[2] >= 0
    assert word.item() != 0                     # the bad index was reported
    onn, _ = orc.nearest(s.x, [3, 7])
    assert [got[0], got[2]] == onn.tolist()
