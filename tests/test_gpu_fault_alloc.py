"""Allocation failures: with CT_FAULT_ALLOC=n the library's n-th device or pinned allocation fails as
out-of-memory.  For every entry point that allocates, and every allocation it makes, the call either
returns CT_ERR_OOM or (where the library has a fallback that needs no scratch) the right result;
afterwards the same call without injection gives the reference bits again and the device has not
lost memory.  The GPU itself never fails: the failure is decided on the host before the call."""
import numpy as np
import pytest
import torch

from _helpers import rel_l2, say
from paper_1905_03748_amd import _abi as A
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan, rof, rof_host, tv_steps_host

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def case():
    w = inputs.Workload("fault", (40, 36, 30), (1.0, 1.0, 1.0), (48, 40), (1.6, 1.6), 24, 10, 71)
    vol = inputs.voxelize(w)
    return w, vol


def _calls(w, vol):
    geo = w.geometry_dict()
    x = torch.from_numpy(vol).to(DEV)
    xh = torch.from_numpy(vol.copy())

    def fresh_plan():
        return Plan(geo, w.angles)

    def fwd(kind):
        def f():
            return fresh_plan().forward(x, kind)
        return f

    def bp(kind):
        def f():
            plan = fresh_plan()
            return plan.backproject(plan.forward(x), kind)
        return f

    def cgls():
        plan = fresh_plan()
        return plan.cgls(plan.forward(x), 3)[0]

    def sart():
        plan = fresh_plan()
        return plan.sart(plan.forward(x), 1, block=6)

    def fdk():
        plan = fresh_plan()
        return plan.fdk(plan.forward(x))

    def fwd_host():
        plan = fresh_plan()
        out = torch.zeros(plan.proj_shape)
        plan.forward_host(xh, out, "siddon", cap_bytes=(64 << 20) + 6 * 40 * 36 * 4 * 10)
        return out

    def bp_host(kind):
        def f():
            plan = fresh_plan()
            y = plan.forward(x).cpu()
            out = torch.zeros(plan.vol_shape)
            plan.backproject_host(y, out, kind, cap_bytes=(64 << 20) + 8 * 40 * 36 * 4 * 10)
            return out
        return f

    def rof_dev():
        xr = x.clone()
        rof(geo, xr, 4, 0.05)
        return xr

    def rof_h():
        xr = xh.clone()
        rof_host(geo, xr, 4, 0.05, halo_depth=2, cap_bytes=(64 << 20) + 40 * 36 * 4 * 40)
        return xr

    def tv_h():
        xr = xh.clone()
        tv_steps_host(geo, xr, 2, 0.01, cap_bytes=(64 << 20) + 40 * 36 * 4 * 12)
        return xr

    return {"forward_siddon": fwd("siddon"), "forward_interp": fwd("interp"), "bp_fdk": bp("fdk"),
            "bp_adjoint": bp("adjoint"), "cgls": cgls, "sart": sart, "fdk": fdk, "forward_host": fwd_host,
            "bp_host_fdk": bp_host("fdk"), "bp_host_adjoint": bp_host("adjoint"), "rof": rof_dev,
            "rof_host": rof_h, "tv_host": tv_h}


@pytest.mark.parametrize("name", ["forward_siddon", "forward_interp", "bp_fdk", "bp_adjoint", "cgls", "sart", "fdk",
                                  "forward_host", "bp_host_fdk", "bp_host_adjoint", "rof", "rof_host", "tv_host"])
def test_every_allocation_failure_is_clean(case, name, monkeypatch):
    w, vol = case
    call = _calls(w, vol)[name]
    monkeypatch.delenv("CT_FAULT_ALLOC", raising=False)
    ref = call()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failed = 0
    for n in range(1, 25):
        monkeypatch.setenv("CT_FAULT_ALLOC", f"{n}:{name}")
        say(f"[fault alloc] {name}: allocation {n} fails")
        try:
            out = call()
            torch.cuda.synchronize()
        except A.CtError as e:
            assert e.status == A.CT_ERR_OOM, (n, e)
            failed += 1
            continue
        # no failure reported: either the call makes fewer than n allocations (then the same bits),
        # or a fallback kernel that needs no scratch ran (the per-ray projector, the gather adjoint:
        # the same operator in FP32 with another summation order)
        if not torch.equal(out, ref):
            e = rel_l2(out.cpu().numpy(), ref.cpu().numpy())
            say(f"   fallback at allocation {n}: rel L2 {e:.2e} against the reference")
            assert e <= 2e-6, (name, n, e)
    monkeypatch.delenv("CT_FAULT_ALLOC")
    again = call()
    torch.cuda.synchronize()
    assert torch.equal(again, ref)
    torch.cuda.empty_cache()
    # the device lost no memory to the failed calls (the library frees what it took; 16 MiB of
    # allocator rounding allowed)
    assert torch.cuda.mem_get_info()[0] >= free0 - (16 << 20), (free0, torch.cuda.mem_get_info()[0])
    say(f"   {failed} failing allocation points")
