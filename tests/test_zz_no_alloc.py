"""GPU: lb_moments_static, the allocation-free variant of lb_moments (its reduction scratch is
a fixed device array of the library), against lb_moments on the same state: bitwise equal
planes and totals, on two calls in a row, the second on a smaller replica (so that a call
reading stale partial sums of the first would show), and the documented error return."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1009_0254_amd import workloads as W  # noqa: E402


def say(*a):
    print("[gpu-no-alloc]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("precision", [2, 0])
def test_moments_static_matches_moments(precision):
    from paper_1009_0254_amd import lbfluct as L
    cfgs = [W.single_phase(300, 190, kT=1e-5, seed=31, replica=0),
            W.single_phase(40, 24, kT=1e-5, seed=32, replica=1),
            W.slab(64, 96, kT=1e-6, seed=33, replica=2)]
    lat = L.Lattice(cfgs, precision=precision)
    lat.step(21)
    for rep in (0, 1, 2, 1):      # large, then smaller, then larger again, then small
        ms, ts = lat.lb_moments_static(rep, True)
        mm, tm = lat.lb_moments(rep, True)
        say("precision", precision, "replica", rep, "totals", ts)
        assert torch.equal(ms, mm)
        assert np.array_equal(ts, tm)
        _, t2 = lat.lb_moments_static(rep, False)
        assert np.array_equal(t2, tm)
    # replica indices outside the handle, through the C ABI itself
    assert L.lib().lb_moments_static(lat._h, 3, None, None) == L.LB_EINVAL
    assert L.lib().lb_moments_static(lat._h, -1, None, None) == L.LB_EINVAL
    assert L.lib().lb_moments_static(None, 0, None, None) == L.LB_EINVAL
    lat.close()
