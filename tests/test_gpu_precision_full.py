"""16-bit storage at the full size of the precision workload (1024^3 of 0.25 mm, 720 angles, 1024^2
detector of 0.4 mm): Siddon A x and FDK A^T y with inputs and outputs stored in FP32, FP16 and BF16
and FP32 arithmetic, each compared on seeded samples with the FP64 oracle applied to the FP32
inputs.  The 16-bit error is the rounding of the stored values: each input value and each output
value carries a relative error of at most the format's unit roundoff u (2^-11, 2^-8), and a
non-negative weighted sum of inputs inherits at most u, so |error| <= 1.5 u (relative) per sample
plus the FP32 arithmetic (below 1e-6)."""
import numpy as np
import pytest
import torch

from _helpers import TOL_BP, TOL_PROJ, rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BOUND = {torch.float32: None, torch.float16: 1.5 * 2.0 ** -11, torch.bfloat16: 1.5 * 2.0 ** -8}


@pytest.fixture(scope="module")
def case():
    w = inputs.workload("precision")
    plan = Plan(w.geometry_dict(), w.angles)
    say("[precision full] phantom 1024^3 on the GPU")
    x = inputs.voxelize_torch(w, device=DEV)
    rng = np.random.default_rng(404)
    y = torch.from_numpy(rng.uniform(0.0, 50.0, plan.proj_shape).astype(np.float32)).to(DEV)
    return w, plan, x, y


@pytest.mark.parametrize("dt", [torch.float32, torch.float16, torch.bfloat16])
def test_precision_workload_sampled(case, orc, dt):
    w, plan, x, y = case
    og = orc.Geometry.from_dict(w.geometry_dict())
    xd, yd = x.to(dt), y.to(dt)
    say(f"[precision full] {dt}: forward")
    p = plan.forward(xd, "siddon").float().cpu().numpy().reshape(-1)
    rays = inputs.sample_indices(p.size, 600, 41)
    x_host = x.cpu().numpy()
    e_fwd = rel_l2(p[rays].astype(np.float64), orc.siddon_rays(og, w.angles, rays, x_host.reshape(-1)))
    del p
    say(f"[precision full] {dt}: FDK backprojection")
    v = plan.backproject(yd, "fdk").float().cpu().numpy().reshape(-1)
    vox = inputs.sample_indices(v.size, 150, 42)
    y_host = y.cpu().numpy()
    e_bp = rel_l2(v[vox].astype(np.float64), orc.bp_voxels(og, w.angles, y_host.reshape(-1), vox, orc.W_FDK))
    say(f"[precision full] {dt}: rel L2 forward {e_fwd:.3e}, backprojection {e_bp:.3e}")
    b = BOUND[dt]
    assert e_fwd <= (TOL_PROJ if b is None else b)
    assert e_bp <= (TOL_BP if b is None else b)
