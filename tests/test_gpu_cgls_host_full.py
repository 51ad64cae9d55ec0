"""Three out-of-core CGLS iterations on an image larger than the device cap: 2048^3 FP32 (32 GiB) and
2048 projections of 2048^2 (32 GiB), the splitting workload's field of view at 2048 samples, under a
32 GiB device cap.  Every vector (x, b, r, q, s, p: 192 GiB) is in pageable host memory.

The splitting workload's own size (3072^3, 3072 angles) needs five such vectors of 108 GiB, more
host memory than the machine has; this is the largest cube whose CGLS vectors fit.  Correctness at
small sizes is covered by test_gpu_cgls_host.py; here the run checks that the residual decreases and
that the FP64 residual recurrence agrees with the residual recomputed from the result.

It needs about 200 GiB of host memory and several minutes, so it runs only when CT_FULL_OOC=1."""
import os
import time

import numpy as np
import pytest
import torch

from _helpers import say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("CT_FULL_OOC") != "1",
                                 reason="set CT_FULL_OOC=1 (needs ~200 GiB of host memory, minutes)")]
DEV = "cuda:0"
CAP = 32 << 30
N = 2048


def test_cgls_out_of_core_2048():
    base = inputs.workload("ooc")
    w = inputs.scaled_workload(base, (N, N, N), (N, N), N, name="ooc_2048")
    plan = Plan(w.geometry_dict(), w.angles)
    x = torch.empty(plan.vol_shape, dtype=torch.float32)
    b = torch.empty(plan.proj_shape, dtype=torch.float32)
    say("[cgls ooc 2048] phantom slab by slab")
    ells = inputs.ellipsoids(w)
    for z0 in range(0, N, 256):
        h = min(256, N - z0)
        ws = inputs.Workload("slab", (N, N, h), w.dvox, w.ndet, w.ddet, 1, 0, 0,
                             off_origin=(0.0, 0.0, (z0 + h / 2.0 - N / 2.0) * w.dvox[2]))
        x[z0:z0 + h].copy_(inputs.voxelize_torch(ws, ells, device=DEV))
        torch.cuda.synchronize()
    say("[cgls ooc 2048] data b = A x_true under the cap")
    st = plan.forward_host(x, b, "siddon", cap_bytes=CAP)
    say(f"[cgls ooc 2048] b: {st}")
    x.zero_()
    work = torch.empty(plan.cgls_host_workspace_bytes(), dtype=torch.uint8)
    say("[cgls ooc 2048] 3 CGLS iterations under the cap")
    t = time.perf_counter()
    x, res, st = plan.cgls_host(b, 3, x=x, cap_bytes=CAP, workspace=work)
    wall = time.perf_counter() - t
    say(f"[cgls ooc 2048] wall {wall:.1f} s, resid {res}, stats {st}")
    assert st["n_slabs"] > 1
    assert np.all(np.diff(res) < 0)
    # recompute ||b - A x|| with the workspace as the projection buffer
    ax = work[:b.numel() * 4].view(torch.float32).view(plan.proj_shape)
    say("[cgls ooc 2048] explicit residual")
    plan.forward_host(x, ax, "siddon", cap_bytes=CAP)
    rr = 0.0
    for a0 in range(0, N, 64):
        d = b[a0:a0 + 64].double() - ax[a0:a0 + 64].double()
        rr += float((d * d).sum())
    rr = rr ** 0.5
    say(f"[cgls ooc 2048] explicit residual {rr:.6e} vs recurrence {res[-1]:.6e}")
    assert abs(rr - res[-1]) <= 1e-3 * res[-1]
