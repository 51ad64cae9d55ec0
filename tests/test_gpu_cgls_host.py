"""Out-of-core CGLS (every vector in host memory, operators streamed under a device cap) on the tiny
workload, split into several slabs in both directions: against the FP64 oracle's CGLS, against the
device-resident CGLS, and on its edge cases (zero data, no iterations, a warm start)."""
import numpy as np
import pytest
import torch

from _helpers import rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan
from test_gpu_ooc import _cap_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tiny(orc):
    w = inputs.workload("tiny")
    ells = inputs.ellipsoids(w)
    b = inputs.analytic_projections(w, ells).astype(np.float32)
    plan = Plan(w.geometry_dict(), w.angles)
    cap = _cap_for(plan, 16, 0)
    return w, plan, b, orc.Geometry.from_dict(w.geometry_dict()), cap


def test_cgls_host_split(tiny):
    w, plan, b, og, cap = tiny
    f = plan.ooc_plan(0, "siddon", cap_bytes=cap)
    a = plan.ooc_plan(2, "siddon", cap_bytes=cap)
    say(f"[cgls host] forward split {f}, backprojection split {a}")
    assert f["n_slabs"] == 4 and a["n_slabs"] >= 2


def test_cgls_host_matches_oracle_and_resident(tiny, orc):
    w, plan, b, og, cap = tiny
    A = lambda x: orc.siddon_fwd(og, w.angles, x)
    At = lambda y: orc.siddon_adj(og, w.angles, y)
    xr, rr = orc.cgls(A, At, b.astype(np.float64), 5)
    say("[cgls host] tiny, 5 iterations out of core")
    x, res, st = plan.cgls_host(torch.from_numpy(b), 5, cap_bytes=cap)
    say(f"   stats {st}")
    assert st["n_slabs"] == 4 and st["bytes_h2d"] > 0
    x = x.numpy()
    e = rel_l2(x, xr)
    say(f"   x rel L2 vs oracle {e:.3e}; resid {res} vs {rr}")
    assert e <= 1e-4
    np.testing.assert_allclose(res, rr, rtol=1e-4)
    assert np.all(np.diff(res) <= 1e-6 * res[0])
    # the resident iteration: same recurrence, FP32 operators that differ only in the order the
    # forward adds slab partial sums, and FP64 dots summed in another order
    xd, rd = plan.cgls(torch.from_numpy(b).to(DEV), 5)
    ed = rel_l2(x, xd.cpu().numpy())
    say(f"   x rel L2 vs resident {ed:.3e}")
    assert ed <= 1e-5
    np.testing.assert_allclose(res, rd.cpu().numpy(), rtol=1e-5)


def test_cgls_host_edge_cases(tiny):
    w, plan, b, og, cap = tiny
    # zero data: the first step has A p = 0, the iteration stops, x stays 0
    x, res, _ = plan.cgls_host(torch.zeros(plan.proj_shape), 3, cap_bytes=cap)
    assert float(x.abs().max()) == 0.0 and np.all(res == 0.0) and res.size == 4
    # no iterations from a non-zero start: x unchanged, one norm ||b - A x0||
    bt = torch.from_numpy(b)
    x0 = torch.full(plan.vol_shape, 0.25)
    x, res, _ = plan.cgls_host(bt, 0, x=x0.clone(), cap_bytes=cap)
    assert torch.equal(x, x0) and res.size == 1
    r0 = bt.to(DEV).double() - plan.forward(x0.to(DEV)).double()
    assert abs(res[0] - float(r0.norm())) <= 1e-6 * float(r0.norm())
    # warm start: the same iterates as the resident CGLS from the same start
    x, res, _ = plan.cgls_host(bt, 3, x=x0.clone(), cap_bytes=cap)
    xd, rd = plan.cgls(bt.to(DEV), 3, x=x0.to(DEV))
    assert rel_l2(x.numpy(), xd.cpu().numpy()) <= 1e-5
    np.testing.assert_allclose(res, rd.cpu().numpy(), rtol=1e-5)


def test_cgls_host_rejects_bad_arguments(tiny):
    w, plan, b, og, cap = tiny
    with pytest.raises(ValueError):
        plan.cgls_host(torch.from_numpy(b).to(DEV), 1, cap_bytes=cap)
    with pytest.raises(ValueError):
        plan.cgls_host(torch.from_numpy(b).double(), 1, cap_bytes=cap)
    with pytest.raises(ValueError):
        plan.cgls_host(torch.from_numpy(b), 1, workspace=torch.empty(16, dtype=torch.uint8), cap_bytes=cap)
    with pytest.raises(RuntimeError):
        plan.cgls_host(torch.from_numpy(b), 1, cap_bytes=1 << 20)  # below one slice plus buffers
