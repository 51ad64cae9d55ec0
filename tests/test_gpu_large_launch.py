"""A resident forward projection whose single launch would exceed the dispatch's 32-bit
work-item count: 2200 projections of 2048^2 (36.9 GB of FP32 projections) from a small volume.
The column walk needs about 4.6e9 lanes, so the launcher splits the angles over several launches.
Rays sampled over the whole range, the last angles included, are checked against the oracle for
both projectors."""
import numpy as np
import pytest
import torch

from _helpers import TOL_PROJ, rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_forward_split_over_launches(orc):
    w = inputs.Workload("wide_launch", (24, 24, 24), (1.0, 1.0, 1.0), (2048, 2048), (0.02, 0.02), 2200, 4, 61)
    vol = inputs.voxelize(w)
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    x = torch.from_numpy(vol).to(DEV)
    n = 2200 * 2048 * 2048
    rays = np.concatenate([inputs.sample_indices(n, 1500, 71),
                           n - 10 * 2048 * 2048 + inputs.sample_indices(10 * 2048 * 2048, 500, 72)])
    idx = torch.from_numpy(rays).to(DEV)
    out = torch.empty(plan.proj_shape, dtype=torch.float32, device=DEV)
    for projector, fn in (("siddon", orc.siddon_rays), ("interp", orc.interp_rays)):
        say(f"[large launch] {projector}: 2200 x 2048^2 projections")
        out.fill_(-1.0)
        plan.forward(x, projector, out=out)
        got = out.view(-1)[idx].cpu().numpy()
        ref = fn(og, w.angles, rays, vol.astype(np.float64))
        e = rel_l2(got, ref)
        say(f"   rel L2 on {len(rays)} rays {e:.3e}; {int((ref > 0).sum())} rays meet the volume")
        assert (ref > 0).sum() > 300
        assert e <= TOL_PROJ
