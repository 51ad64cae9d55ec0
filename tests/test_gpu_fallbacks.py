"""Geometries outside what the column and LDS kernels cover, so the host picks the per-ray and
gather kernels: a wide cone (rays steeper than the column walk allows), detector rows much finer
than the voxels (more rows per voxel than the column adjoint visits), and pixels so small that a
tile's detector window does not fit the LDS staging buffer.  Every operator is compared with the
oracle; on the wide cone CGLS and SART run their non-column paths too."""
import numpy as np
import pytest
import torch

from _helpers import TOL_BP, TOL_PROJ, rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    # half-height of the detector above 0.7 DSD: the column walk's one-crossing condition fails
    "wide_cone": inputs.Workload("wide_cone", (24, 24, 24), (2.0, 2.0, 2.0), (48, 48), (5.0, 5.0), 12, 8, 61,
                                 DSO=100.0, DSD=150.0),
    # 4 mm slices over 0.5 mm rows: about 12 rows can meet one voxel
    "fine_rows": inputs.Workload("fine_rows", (20, 20, 16), (1.0, 1.0, 4.0), (40, 64), (1.5, 0.5), 12, 8, 62,
                                 DSO=500.0, DSD=700.0),
    # 0.3 mm pixels under 2 mm voxels: a 16 x 16 tile spans hundreds of detector columns
    "tiny_pixels": inputs.Workload("tiny_pixels", (16, 16, 16), (2.0, 2.0, 2.0), (160, 160), (0.3, 0.3), 10, 8, 63,
                                   DSO=500.0, DSD=700.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fallback_operators(orc, name):
    w = CASES[name]
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    vol = inputs.voxelize(w)
    y = inputs.random_array(plan.proj_shape, 64, kind="uniform")
    x = torch.from_numpy(vol).to(DEV)
    yt = torch.from_numpy(y).to(DEV)
    for proj, fn in (("siddon", orc.siddon_fwd), ("interp", orc.interp_fwd)):
        e = rel_l2(plan.forward(x, proj).cpu().numpy(), fn(og, w.angles, vol.astype(np.float64)))
        say(f"[fallback {name}] {proj} rel L2 {e:.3e}")
        assert e <= TOL_PROJ
    y64 = y.astype(np.float64)
    for kind, ref in (("fdk", orc.bp(og, w.angles, y64, orc.W_FDK)), ("pm", orc.bp(og, w.angles, y64, orc.W_PM)),
                      ("adjoint", orc.siddon_adj(og, w.angles, y64))):
        e = rel_l2(plan.backproject(yt, kind).cpu().numpy(), ref)
        say(f"[fallback {name}] {kind} rel L2 {e:.3e}")
        assert e <= TOL_BP


def test_fallback_algorithms(orc):
    w = CASES["wide_cone"]
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    b = orc.siddon_fwd(og, w.angles, inputs.voxelize(w).astype(np.float64))
    x, res = plan.cgls(torch.from_numpy(b.astype(np.float32)).to(DEV), 3)
    xr, rr = orc.cgls(lambda v: orc.siddon_fwd(og, w.angles, v), lambda q: orc.siddon_adj(og, w.angles, q), b, 3)
    e = rel_l2(x.cpu().numpy(), xr)
    say(f"[fallback wide_cone] CGLS-3 rel L2 {e:.3e}")
    assert e <= 1e-4
    xs = plan.sart(torch.from_numpy(b.astype(np.float32)).to(DEV), 1).cpu().numpy()
    e = rel_l2(xs, orc.sart(og, w.angles, b, 1))
    say(f"[fallback wide_cone] SART-1 rel L2 {e:.3e}")
    assert e <= 1e-4
    # ordered subsets of 5 angles (the last one shorter) through the same fallback kernels
    xo = plan.sart(torch.from_numpy(b.astype(np.float32)).to(DEV), 2, block=5).cpu().numpy()
    e = rel_l2(xo, orc.os_sart(og, w.angles, b, 2, 5))
    say(f"[fallback wide_cone] OS-SART(5)-2 rel L2 {e:.3e}")
    assert e <= 1e-4
