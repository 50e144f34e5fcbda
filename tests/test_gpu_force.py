"""GPU parity of nb_force_active (acc + jerk) against the FP64 oracle.

Gates (maximum over bodies): FP64 path, relative error of acceleration and jerk
<= 1e-12; mixed and double-single (DS) paths, error <= 1e-6 of the magnitude scales
sum_j |a_ij| and sum_j |jerk_ij| for every body, and plain relative error <= 1e-6
for every body whose cancellation factor is below the bound of gpu_helpers.
Cases: the N = 1024 Plummer sphere with every body active, the N = 65536 Salpeter
cluster with active blocks of 64 .. 4096 (plus sampled bodies of larger blocks),
ragged sizes and j-ranges, every launch plan shape, bitwise repeatability, empty
blocks, error paths, and the N = 2^20 Plummer sphere with every body active (the
benchmarked launch) on random bodies and on the bodies of largest cancellation.
"""
import json
import os

import numpy as np
import pytest
import torch

from gpu_helpers import TOL, check, device_system, gpu_force, report
from paper_1411_5234_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2():
    n = 65536
    s = inputs.plummer(n, 2, masses=inputs.salpeter_masses(n, 2))
    return s


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_plummer_1024_all_active(ctx, orc, precision):
    s = inputs.plummer(1024, 1)
    sys = device_system(s.x, s.v, s.m)
    ga, gj = gpu_force(ctx, sys, 1e-3, precision)
    check(orc, precision, ga, gj, s.x, s.v, s.m, 1e-3, tag="N=1024")


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("m", [64, 256, 1000, 4096])
def test_salpeter_65536_active_blocks(ctx, orc, c2, precision, m):
    perm = np.random.default_rng(20).permutation(c2.n)[:m]
    il = np.sort(perm)
    sys = device_system(c2.x, c2.v, c2.m)
    ga, gj = gpu_force(ctx, sys, 1e-4, precision, il)
    check(orc, precision, ga, gj, c2.x, c2.v, c2.m, 1e-4, il, tag="N=65536 m=%d" % m)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("m", [16384, 65536])
def test_salpeter_65536_large_blocks_sampled(ctx, orc, c2, precision, m):
    il = np.sort(np.random.default_rng(21).permutation(c2.n)[:m])
    sys = device_system(c2.x, c2.v, c2.m)
    ga, gj = gpu_force(ctx, sys, 1e-4, precision, il)
    pick = np.random.default_rng(22).choice(m, 512, replace=False)
    check(orc, precision, ga[pick], gj[pick], c2.x, c2.v, c2.m, 1e-4, il[pick],
          tag="N=65536 m=%d (512 sampled)" % m)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_ragged_sizes_and_j_ranges(ctx, orc, precision):
    s = inputs.plummer(1000, 8, masses=inputs.salpeter_masses(1000, 9))
    sys = device_system(s.x, s.v, s.m)
    il = np.sort(np.random.default_rng(5).choice(1000, 77, replace=False))
    for j0, j1 in [(0, 1000), (13, 911), (0, 1), (999, 1000), (511, 513)]:
        ga, gj = gpu_force(ctx, sys, 1e-2, precision, il, j0, j1)
        oa, oj = check(orc, precision, ga, gj, s.x, s.v, s.m, 1e-2, il, j0, j1,
                       tag="ragged [%d,%d)" % (j0, j1))
        nz = np.linalg.norm(oa, axis=1) > 0
        # bodies whose only j is themselves get exactly zero
        assert np.all(ga[~nz] == 0.0) and np.all(gj[~nz] == 0.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_every_plan_shape_matches(ctx, orc, precision):
    s = inputs.plummer(3000, 12)
    sys = device_system(s.x, s.v, s.m)
    il = np.arange(0, 3000, 3)
    oa, oj = orc.force(s.x, s.v, s.m, 1e-3, il)
    sa, sj = orc.force_scale(s.x, s.v, s.m, 1e-3, il)
    for i_per_lane in (1, 2, 4):
        for lanes in (1, 4, 16, 64):
            for chunks in (1, 3, 8):
                ga, gj = gpu_force(ctx, sys, 1e-3, precision, il, plan=(i_per_lane, lanes, chunks))
                ea, ej = report("plan %d/%d/%d %s" % (i_per_lane, lanes, chunks, precision),
                                ga, gj, oa, oj)
                assert ea.max() <= TOL[precision]
                if precision == "fp64":
                    assert ej.max() <= TOL[precision]
                else:
                    assert (np.linalg.norm(gj - oj, axis=1) / sj).max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_many_j_chunks(ctx, orc, c2, precision):
    """Small active blocks split over up to 128 j-chunks: the partial sums are
    reduced with several lanes per output value (in a fixed order) and must match
    the oracle and repeat bitwise."""
    il = np.sort(np.random.default_rng(23).permutation(c2.n)[:37])
    sys = device_system(c2.x, c2.v, c2.m)
    oa, oj = orc.force(c2.x, c2.v, c2.m, 1e-4, il)
    sa, sj = orc.force_scale(c2.x, c2.v, c2.m, 1e-4, il)
    for plan in [(1, 64, 16), (1, 64, 32), (1, 16, 64), (1, 64, 128), (2, 4, 100)]:
        ga, gj = gpu_force(ctx, sys, 1e-4, precision, il, plan=plan)
        ea, ej = report("chunks %s %s" % (plan, precision), ga, gj, oa, oj)
        assert ea.max() <= TOL[precision]
        if precision == "fp64":
            assert ej.max() <= TOL[precision]
        else:
            assert (np.linalg.norm(gj - oj, axis=1) / sj).max() <= TOL[precision]
    a1, j1 = gpu_force(ctx, sys, 1e-4, precision, il, plan=(1, 64, 128))
    a2, j2 = gpu_force(ctx, sys, 1e-4, precision, il, plan=(1, 64, 128))
    assert a1.tobytes() == a2.tobytes() and j1.tobytes() == j2.tobytes()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_result_does_not_depend_on_active_order(ctx, c2, precision):
    """The same active bodies listed in another order get the same bits: a body's
    sum runs over the same j in the same order whichever lane or workgroup
    holds it."""
    il = np.sort(np.random.default_rng(24).permutation(c2.n)[:1000])
    perm = np.random.default_rng(25).permutation(il.size)
    sys = device_system(c2.x, c2.v, c2.m)
    a1, j1 = gpu_force(ctx, sys, 1e-4, precision, il)
    a2, j2 = gpu_force(ctx, sys, 1e-4, precision, il[perm])
    assert a1[perm].tobytes() == a2.tobytes() and j1[perm].tobytes() == j2.tobytes()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_bitwise_repeatable(ctx, precision):
    s = inputs.plummer(5000, 13)
    sys = device_system(s.x, s.v, s.m)
    il = np.arange(0, 5000, 7)
    a1, j1 = gpu_force(ctx, sys, 1e-3, precision, il)
    a2, j2 = gpu_force(ctx, sys, 1e-3, precision, il)
    assert a1.tobytes() == a2.tobytes() and j1.tobytes() == j2.tobytes()


def test_empty_block_and_empty_range(ctx):
    s = inputs.plummer(100, 3)
    sys = device_system(s.x, s.v, s.m)
    ga, gj = gpu_force(ctx, sys, 1e-3, "mixed", [])
    assert ga.shape == (0, 3)
    ga, gj = gpu_force(ctx, sys, 1e-3, "fp64", [1, 2, 3], 40, 40)
    assert np.all(ga == 0.0) and np.all(gj == 0.0)


def test_argument_errors(ctx):
    from paper_1411_5234_amd._lib import NbError
    s = inputs.plummer(100, 3)
    sys = device_system(s.x, s.v, s.m)
    with pytest.raises(NbError) as e:
        gpu_force(ctx, sys, 0.0, "mixed")
    assert e.value.name == "NB_EINVAL"
    with pytest.raises(NbError):
        gpu_force(ctx, sys, 1e-3, "mixed", [0, 1], 0, 101)
    with pytest.raises(NbError):
        gpu_force(ctx, sys, 1e-3, "mixed", [0], plan=(3, 1, 1))
    no32 = device_system(s.x, s.v, s.m, fp32=False)
    with pytest.raises(NbError):
        gpu_force(ctx, no32, 1e-3, "mixed", [0])
    # an out-of-range active index is clamped in the kernel and reported at sync
    with pytest.raises(NbError) as e:
        gpu_force(ctx, sys, 1e-3, "fp64", [0, 100])
    assert e.value.name == "NB_EINDEX"
    ctx.sync()   # the word was cleared by the failing sync


def top_kappa_2pow20():
    """The 64 bodies of largest sum|a_ij|/|a_i| and the 64 of largest
    sum|jerk_ij|/|jerk_i| of the N = 2^20 Plummer sphere (seed 3, eps = 1e-4), from a
    full oracle scan (tests/golden/make_kappa_plummer_2pow20.py)."""
    with open(os.path.join(GOLDEN, "kappa_plummer_2pow20_seed3.json")) as f:
        rec = json.load(f)
    return (np.asarray(rec["top_kappa_acc"]["index"], dtype=np.int64),
            np.asarray(rec["top_kappa_jerk"]["index"], dtype=np.int64))


@pytest.mark.parametrize("precision", ["mixed", "ds", "fp64"])
def test_plummer_2pow20_all_active_sampled(ctx, orc, precision):
    """The benchmarked launch (m = N = 2^20) on 256 random bodies and, chosen on
    purpose, the 128 bodies whose acceleration or jerk cancels most (largest
    kappa): there the FP32 pair sum is furthest from the plain relative error."""
    n = 1 << 20
    s = inputs.plummer(n, 3)
    sys = device_system(s.x, s.v, s.m)
    ga, gj = gpu_force(ctx, sys, 1e-4, precision)
    pick = np.sort(np.random.default_rng(30).choice(n, 256, replace=False))
    check(orc, precision, ga[pick], gj[pick], s.x, s.v, s.m, 1e-4, pick,
          tag="N=2^20 all active (256 sampled)")
    top_a, top_j = top_kappa_2pow20()
    for name, top in (("acceleration", top_a), ("jerk", top_j)):
        check(orc, precision, ga[top], gj[top], s.x, s.v, s.m, 1e-4, top,
              tag="N=2^20 all active (64 largest kappa of the %s)" % name)
    # momentum balance over every body (a property at any size)
    ma = (s.m[:, None] * ga).sum(0)
    assert np.all(np.abs(ma) <= 1e-6 * (s.m[:, None] * np.abs(ga)).sum(0))


@pytest.mark.parametrize("precision", ["mixed", "ds", "fp64"])
def test_c5_binaries_65536(ctx, orc, precision):
    """The precision-stress workload: a Kroupa cluster of 65536 bodies with 10% of
    them in binaries (separations 1e-4 .. 1e-2 at positions of order 1), eps = 1e-5.
    All bodies active, and a block made of binary members only (the small block of
    tiny steps such a cluster keeps running), each checked on every member of 64
    binaries and on 128 random bodies."""
    n = 1 << 16
    s = inputs.with_binaries(n, 5001)
    pairs = np.asarray(s.meta["pairs"])
    rng = np.random.default_rng(32)
    members = np.sort(pairs[rng.choice(len(pairs), 64, replace=False)].ravel())
    pick = np.unique(np.concatenate([members, rng.choice(n, 128, replace=False)]))
    sys = device_system(s.x, s.v, s.m)
    ga, gj = gpu_force(ctx, sys, 1e-5, precision)
    check(orc, precision, ga[pick], gj[pick], s.x, s.v, s.m, 1e-5, pick,
          tag="C5 N=65536 all active (binary members and random bodies)")
    block = np.sort(pairs[rng.choice(len(pairs), 200, replace=False)].ravel())
    ga, gj = gpu_force(ctx, sys, 1e-5, precision, block)
    check(orc, precision, ga, gj, s.x, s.v, s.m, 1e-5, block,
          tag="C5 N=65536 block of %d binary members" % block.size)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_single_body_and_coincident_bodies(ctx, precision):
    """A lone body feels exactly zero.  Bodies at one point (eps > 0) exert exactly
    zero acceleration on each other (r = 0 zeroes every pair term), while the jerk
    keeps its softened closed form: the time derivative of m r / (r^2 + eps^2)^(3/2)
    at r = 0 is m (v_j - v_i) / eps^3."""
    eps = 1e-3
    x = np.array([[0.3, -0.2, 0.1]])
    v = np.array([[1.0, 2.0, 3.0]])
    sys = device_system(x, v, np.array([1.0]))
    ga, gj = gpu_force(ctx, sys, eps, precision)
    assert np.all(ga == 0.0) and np.all(gj == 0.0)
    x3 = np.repeat(x, 3, axis=0)
    v3 = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0], [-1.0, 0.5, 2.0]])
    m3 = np.array([1.0, 2.0, 0.5])
    sys = device_system(x3, v3, m3)
    ga, gj = gpu_force(ctx, sys, eps, precision)
    assert np.all(ga == 0.0)
    want = np.array([(m3[:, None] * (v3 - v3[i])).sum(0) for i in range(3)]) / eps ** 3
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert np.abs(gj - want).max() <= tol * np.abs(want).max()
    assert np.all(gj[0] == gj[1])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_n_2pow23_small_active_block(ctx, orc, precision):
    """N = 2^23 (8 times the benchmarked system): a block of 200 active bodies
    against every body, split over the plan's largest chunk count, against the
    oracle."""
    n = 1 << 23
    s = inputs.plummer(n, 9)
    sys = device_system(s.x, s.v, s.m)
    il = np.sort(np.random.default_rng(31).choice(n, 200, replace=False))
    ga, gj = gpu_force(ctx, sys, 1e-4, precision, il)
    check(orc, precision, ga, gj, s.x, s.v, s.m, 1e-4, il, tag="N=2^23 m=200")
    del sys
    torch.cuda.empty_cache()
