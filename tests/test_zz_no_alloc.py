"""nb_force_active_noalloc (the allocation-free force entry point) against
nb_force_active, through the C ABI.

The two share the launch plan and the kernels; the allocation-free call keeps its
launch table and j-chunk partial sums in the library's static device area instead
of the context's scratch, so the outputs must be bitwise equal.  Two calls in a row
(the second with a smaller input, so the area still holds the first call's larger
contents), in every precision, with several j-chunks and with one, plus a call too
large for the area, which must be refused before anything runs.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import device_system
from paper_1411_5234_amd import _lib, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


def both(ctx, sys, eps, precision, ilist, j0=0, j1=None):
    n = sys.n
    j1 = n if j1 is None else j1
    m = n if ilist is None else len(ilist)
    idx = None if ilist is None else torch.as_tensor(np.asarray(ilist, dtype=np.int32),
                                                     device="cuda")
    out = [torch.full((3 * max(m, 1),), np.nan, dtype=torch.float64, device="cuda")
           for _ in range(4)]
    ctx.force_active(sys, idx, m, j0, j1, eps, precision, out[0], out[1])
    ctx.force_active_noalloc(sys, idx, m, j0, j1, eps, precision, out[2], out[3])
    ctx.sync()
    return [o[: 3 * m].cpu().numpy() for o in out]


@pytest.mark.parametrize("precision", ["mixed", "fp64", "ds"])
def test_noalloc_equals_force_active_two_calls(ctx, precision):
    big = inputs.plummer(20000, 41, masses=inputs.salpeter_masses(20000, 42))
    small = inputs.plummer(5000, 43)
    cases = [
        # (state, eps, active list, j-range): the second call is smaller
        (big, 1e-4, np.sort(np.random.default_rng(44).choice(20000, 3000, replace=False)),
         (0, 20000)),
        (small, 1e-3, np.sort(np.random.default_rng(45).choice(5000, 100, replace=False)),
         (17, 4901)),
    ]
    for s, eps, il, (j0, j1) in cases:
        _, _, b = _lib.force_plan(j1 - j0, len(il), precision)
        print("N=%d m=%d j=[%d,%d) %s: %d j-chunks" % (len(s.m), len(il), j0, j1, precision, b),
              flush=True)
        # both calls split j, so both keep partial sums in the area
        assert b > 1
        sys = device_system(s.x, s.v, s.m)
        a, j, a2, j2 = both(ctx, sys, eps, precision, il, j0, j1)
        assert np.all(np.isfinite(a)) and np.all(np.isfinite(j))
        assert np.array_equal(a, a2) and np.array_equal(j, j2)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_single_chunk_and_empty(ctx, precision):
    s = inputs.plummer(1500, 46)
    sys = device_system(s.x, s.v, s.m)
    # every body active: one j-chunk, so no partial sums
    assert _lib.force_plan(1500, 1500, precision)[2] == 1
    a, j, a2, j2 = both(ctx, sys, 1e-3, precision, None)
    assert np.array_equal(a, a2) and np.array_equal(j, j2)
    # an empty j-range gives zero forces, as nb_force_active does
    a, j, a2, j2 = both(ctx, sys, 1e-3, precision, [5, 9], 100, 100)
    assert np.array_equal(a, a2) and np.array_equal(j, j2) and np.all(a == 0.0)


def test_noalloc_refuses_what_does_not_fit(ctx):
    """Every body of N = 2^17 active: the plan's partial sums (6 doubles per body
    and chunk) exceed the static area, so the call fails before enqueueing and a
    later call still works."""
    from paper_1411_5234_amd._lib import NbError
    n = 1 << 17
    _, _, b = _lib.force_plan(n, n, "mixed")
    assert 6 * n * b * 8 > (64 << 20)
    s = inputs.plummer(n, 47)
    sys = device_system(s.x, s.v, s.m)
    acc = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    jerk = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    with pytest.raises(NbError) as e:
        ctx.force_active_noalloc(sys, None, n, 0, n, 1e-4, "mixed", acc, jerk)
    assert e.value.name == "NB_ESCRATCH"
    ctx.sync()
    il = np.arange(0, n, 97)
    a, j, a2, j2 = both(ctx, sys, 1e-4, "mixed", il)
    assert np.array_equal(a, a2) and np.array_equal(j, j2)
