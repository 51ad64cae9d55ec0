"""Stream order: every entry point enqueues on the stream it is given and on nothing else, so work
written just before on that stream is seen without a host synchronisation, and two streams running
different reconstructions at once give the same bits as each alone (Section 2's operators and
Section 3.2's algorithms, as a caller with several streams drives them)."""
import numpy as np
import pytest
import torch

from _helpers import say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan, tv_steps

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def case():
    w = inputs.Workload("streams", (48, 44, 40), (1.0, 1.0, 1.0), (64, 48), (1.6, 1.6), 45, 10, 61)
    return w, inputs.voxelize(w)


def test_operators_follow_the_given_stream(case):
    w, vol = case
    plan = Plan(w.geometry_dict(), w.angles)
    x = torch.from_numpy(vol).to(DEV)
    ref_p = plan.forward(x)
    ref_v = plan.backproject(ref_p, "adjoint")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()   # default priority
    for rep in range(3):
        say(f"[streams] side stream, rep {rep}")
        with torch.cuda.stream(s):
            # produced on the side stream just before: the operators must order after it
            xs = torch.empty_like(x)
            xs.copy_(x, non_blocking=True)
            xs.mul_(2.0).mul_(0.5)
            p = plan.forward(xs, stream=s)
            v = plan.backproject(p, "adjoint", stream=s)
            v2 = plan.backproject(p, "fdk", stream=s)
        # the default stream has not waited; only the side stream's own order is relied on
        s.synchronize()
        assert torch.equal(p, ref_p) and torch.equal(v, ref_v)
        assert torch.isfinite(v2).all()


def test_two_streams_at_once_equal_each_alone(case):
    w, vol = case
    plan_a = Plan(w.geometry_dict(), w.angles)
    plan_b = Plan(w.geometry_dict(), w.angles[::2].copy())
    x = torch.from_numpy(vol).to(DEV)
    ba = plan_a.forward(x)
    bb = plan_b.forward(x)
    torch.cuda.synchronize()

    def run(plan, b, stream):
        xr, res = plan.cgls(b, 6, stream=stream)
        tv_steps(plan.geometry, xr, 3, 0.01, stream=stream)
        return xr, res

    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    say("[streams] each alone")
    with torch.cuda.stream(sa):
        xa0, ra0 = run(plan_a, ba, sa)
    sa.synchronize()
    with torch.cuda.stream(sb):
        xb0, rb0 = run(plan_b, bb, sb)
    sb.synchronize()
    say("[streams] both at once")
    with torch.cuda.stream(sa):
        xa1, ra1 = run(plan_a, ba, sa)
    with torch.cuda.stream(sb):
        xb1, rb1 = run(plan_b, bb, sb)
    sa.synchronize()
    sb.synchronize()
    assert torch.equal(xa0, xa1) and torch.equal(ra0, ra1)
    assert torch.equal(xb0, xb1) and torch.equal(rb0, rb1)
