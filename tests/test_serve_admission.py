"""Admission policy and slot/memory accounting of the server, on the CPU.

A test-only stub stands in for the device: each admitted request needs a fixed
number of iterations.  The policy must keep the slot and memory limits at every
iteration, admit in arrival order as soon as capacity frees up (continuous
batching), and refuse requests that could never fit.  Also the server's host-side
bookkeeping of grouped pairs: the row layout after pairs return, and the mutual
nearest neighbours from which new pairs are taken.
"""
from dataclasses import dataclass

import numpy as np
import pytest

from paper_1411_5234_amd.serve import Admission, footprint_bytes


@dataclass
class Req:
    rid: int
    n: int
    work: int          # iterations the stub needs for this request


def fp(r):
    return 100 * r.n


def run_stub(adm, reqs, arrivals):
    """Drive the policy: at iteration t the requests with arrival <= t are
    submitted; every resident request does one unit of work per iteration."""
    pending = sorted(zip(arrivals, reqs), key=lambda x: x[0])
    left = {}
    done, log = [], []
    t = 0
    while pending or adm.queue or left:
        while pending and pending[0][0] <= t:
            adm.submit(pending.pop(0)[1])
        while True:
            r = adm.admit_next()
            if r is None:
                break
            left[r.rid] = (r, r.work)
        log.append((t, len(left), adm.used, [q.rid for q in adm.queue]))
        assert len(left) <= adm.max_slots and adm.used <= adm.budget
        for rid in list(left):
            r, w = left[rid]
            if w == 1:
                del left[rid]
                adm.release(r)
                done.append((rid, t))
            else:
                left[rid] = (r, w - 1)
        t += 1
        assert t < 10000
    return done, log


def test_slots_limit_and_fifo_order():
    adm = Admission(budget=10 ** 9, max_slots=3, footprint=fp)
    reqs = [Req(k, 10, work=5) for k in range(7)]
    done, log = run_stub(adm, reqs, [0] * 7)
    assert sorted(r for r, _ in done) == list(range(7))
    assert max(k for _, k, _, _ in log) == 3
    # continuous batching: the fourth request starts the iteration after a slot frees
    assert [t for r, t in done] == [4, 4, 4, 9, 9, 9, 14]


def test_memory_budget_and_head_of_line():
    # budget fits one big (n=50) or five small (n=10) requests
    adm = Admission(budget=5000, max_slots=100, footprint=fp)
    reqs = [Req(0, 10, 3), Req(1, 50, 3), Req(2, 10, 1), Req(3, 10, 1)]
    done, log = run_stub(adm, reqs, [0, 0, 0, 0])
    assert all(u <= 5000 for _, _, u, _ in log)
    order = [r for r, _ in done]
    # the big request at the head of the queue is not overtaken by the small ones
    assert order.index(1) < order.index(2) and order.index(1) < order.index(3)
    assert adm.used == 0 and not adm.resident


def test_arrivals_while_running_are_admitted():
    adm = Admission(budget=10 ** 9, max_slots=2, footprint=fp)
    reqs = [Req(0, 10, 10), Req(1, 10, 2), Req(2, 10, 2), Req(3, 10, 2)]
    done, log = run_stub(adm, reqs, [0, 0, 3, 3])
    finished = dict(done)
    assert finished[1] == 1          # request 1 shares the device with request 0
    assert finished[2] == 4 and finished[3] == 6   # 2 starts at t=3 beside 0; 3 waits for a slot
    assert finished[0] == 9


def test_refuses_what_never_fits():
    adm = Admission(budget=1000, max_slots=4, footprint=fp)
    with pytest.raises(ValueError):
        adm.submit(Req(0, 11, 1))
    adm.submit(Req(1, 10, 1))
    assert adm.admit_next().rid == 1
    with pytest.raises(ValueError):
        Admission(budget=1000, max_slots=0, footprint=fp)


def test_footprint_covers_the_device_arrays():
    from paper_1411_5234_amd._lib import FIELDS32, FIELDS64
    n = 1000
    # state rows + FP32 copies + i_idx + acc/jerk (3n doubles each)
    need = 8 * len(FIELDS64) * n + 4 * len(FIELDS32) * n + 4 * n + 2 * 8 * 3 * n
    assert footprint_bytes(n, "mixed") >= need


def test_summary_names_the_request_with_the_largest_energy_error():
    from paper_1411_5234_amd.serve import Result, summarize

    def res(rid, n, e0, e1, t, err=None):
        return Result(rid=rid, n=n, arrival=0.0, admitted=0.0, finished=t, energy0=e0,
                      energy1=e1, error=err)

    rs = [res(0, 300, -0.25, -0.25000001, 1.0), res(1, 900, -0.25, -0.2501, 2.0),
          res(2, 500, -0.25, -0.3, 3.0, err="failed"), res(3, 700, -0.25, -0.25001, 4.0)]
    s = summarize(rs, wall=4.0)
    assert s["completed"] == 3 and s["failed"] == 1
    assert s["energy_error_worst_request"] == {"rid": 1, "n": 900}
    assert s["energy_error_max"] == pytest.approx(0.0001 / 0.25)
    assert s["solves_per_s"] == pytest.approx(0.75)


def test_return_layout_matches_a_plain_mapping():
    """The rows of a reduced system after pairs return: every body in no pair keeps
    its old row or is a returning member, the kept pairs' centres of mass follow;
    against a plain dictionary mapping on random pair sets."""
    from paper_1411_5234_amd.serve import return_layout
    rng = np.random.default_rng(7)
    for n, npairs, kret in ((40, 10, 3), (12, 6, 6), (30, 1, 1), (9, 0, 0), (50, 20, 0)):
        perm = rng.permutation(n)
        pairs = perm[: 2 * npairs].reshape(-1, 2)
        ks = np.sort(rng.choice(npairs, kret, replace=False)) if npairs else np.zeros(0, int)
        old_singles = np.setdiff1d(np.arange(n), pairs.ravel())
        keep = np.setdiff1d(np.arange(npairs), ks)
        new_singles = np.setdiff1d(np.arange(n), pairs[keep].ravel())
        members = pairs[ks].ravel()
        src = return_layout(old_singles, new_singles, members, old_singles.size, keep)
        old_row = {int(i): r for r, i in enumerate(old_singles)}
        mem_row = {int(i): q for q, i in enumerate(members)}
        want = [old_row[int(i)] if int(i) in old_row else -1 - mem_row[int(i)]
                for i in new_singles] + [old_singles.size + int(k) for k in keep]
        assert src.tolist() == want, (n, npairs, kret)


def test_capture_layout_matches_a_plain_mapping():
    """The rows of a reduced system after single bodies pair up: the other singles
    keep their old rows in order, the old centres of mass follow, then the new
    ones; against a plain dictionary mapping on random systems, and refused when
    the candidates are not distinct single bodies."""
    from paper_1411_5234_amd.serve import capture_layout
    rng = np.random.default_rng(11)
    for n, npairs, knew in ((40, 10, 3), (12, 0, 6), (30, 1, 1), (9, 2, 0), (50, 20, 5)):
        perm = rng.permutation(n)
        pairs = perm[: 2 * npairs].reshape(-1, 2)
        singles = np.setdiff1d(np.arange(n), pairs.ravel())
        cm0 = singles.size
        rows = rng.choice(cm0, 2 * knew, replace=False)
        p, q = rows[:knew], rows[knew:]
        src = capture_layout(cm0, npairs, p, q)
        new_pairs = np.stack([singles[p], singles[q]], axis=1)
        new_singles = np.setdiff1d(singles, new_pairs.ravel())
        old_row = {int(i): r for r, i in enumerate(singles)}
        want = ([old_row[int(i)] for i in new_singles] + [cm0 + k for k in range(npairs)]
                + [-1 - k for k in range(knew)])
        assert src.tolist() == want, (n, npairs, knew)
    with pytest.raises(ValueError):
        capture_layout(10, 0, np.array([1, 2]), np.array([2, 3]))   # body 2 twice


def test_mutual_nearest_neighbours():
    from paper_1411_5234_amd.serve import mutual_nearest
    rows = np.array([3, 5, 7, 9, 11, 2])
    nn = np.array([5, 3, 9, 4, -1, 7])      # 3<->5 mutual; 7->9 but 9->4; 11 unsearched
    p, q = mutual_nearest(rows, nn, 12)
    assert p.tolist() == [3] and q.tolist() == [5]
    # a body whose neighbour is not listed (not in the block) pairs with nobody
    p, q = mutual_nearest(np.array([1]), np.array([0]), 2)
    assert p.size == 0
    rng = np.random.default_rng(8)
    for _ in range(20):
        n = 40
        rows = np.sort(rng.choice(n, 25, replace=False))
        nn = np.where(rng.random(25) < 0.8, rng.choice(n, 25), -1)
        nn[nn == rows] = -1
        p, q = mutual_nearest(rows, nn, n)
        d = dict(zip(rows.tolist(), nn.tolist()))
        want = sorted((i, j) for i, j in d.items() if j >= 0 and d.get(j) == i and i < j)
        assert sorted(zip(p.tolist(), q.tolist())) == want
