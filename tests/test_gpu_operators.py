"""GPU parity of the projection operators against the CPU FP64 oracle, through the C ABI.

Bars (relative L2 over the compared outputs): projections 1e-5, backprojections 1e-4, for FP32
storage.  Small cases are compared element by element in full; the 512^3 / 360-angle workload in
the launch configuration the benchmark times is compared on seeded samples of rays and voxels that
the oracle evaluates one by one.
"""
import numpy as np
import pytest
import torch

from _helpers import TOL_BP, TOL_PROJ, rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(name):
    if name == "tiny":
        return inputs.workload("tiny")
    if name == "tiny_offsets":
        return inputs.workload("tiny", off_origin=(1.3, -0.7, 2.1), off_detector=(2.3, -1.7))
    if name == "ragged":
        # odd sizes that fill neither the 64x4 pixel tiles nor the 16x16x8 voxel tiles
        w = inputs.Workload("ragged", (37, 29, 23), (1.1, 0.9, 1.3), (45, 33), (1.7, 1.9), 23, 10, 9,
                            off_detector=(0.37, -0.21))
        w.angles = np.sort(np.random.default_rng(9).uniform(0, 2 * np.pi, 23))
        return w
    if name == "anisotropic":
        return inputs.Workload("aniso", (40, 24, 56), (0.8, 1.4, 0.6), (70, 52), (1.2, 0.9), 31, 10, 11,
                               off_origin=(-2.0, 1.5, -3.0), off_detector=(-1.1, 0.6), accuracy=0.37)
    raise KeyError(name)


CASES = ["tiny", "tiny_offsets", "ragged", "anisotropic"]


@pytest.fixture(scope="module")
def data(orc):
    out = {}
    for name in CASES:
        w = _case(name)
        vol = inputs.voxelize(w)
        y = inputs.random_array((len(w.angles), w.ndet[1], w.ndet[0]), 100 + w.seed, kind="uniform")
        geo = w.geometry_dict()
        out[name] = (w, geo, vol, y, orc.Geometry.from_dict(geo))
    return out


@pytest.mark.parametrize("name", CASES)
def test_forward_parity(data, orc, name):
    w, geo, vol, y, og = data[name]
    plan = Plan(geo, w.angles)
    x = torch.from_numpy(vol).to(DEV)
    for proj, ref_fn in (("siddon", orc.siddon_fwd), ("interp", orc.interp_fwd)):
        say(f"[forward parity] case={name} projector={proj}")
        p = plan.forward(x, proj).cpu().numpy()
        ref = ref_fn(og, w.angles, vol.astype(np.float64))
        e = rel_l2(p, ref)
        say(f"   rel L2 = {e:.3e}")
        assert e <= TOL_PROJ, (name, proj, e)


@pytest.mark.parametrize("name", CASES)
def test_backprojection_parity(data, orc, name):
    w, geo, vol, y, og = data[name]
    plan = Plan(geo, w.angles)
    yt = torch.from_numpy(y).to(DEV)
    y64 = y.astype(np.float64)
    refs = {"fdk": lambda: orc.bp(og, w.angles, y64, orc.W_FDK),
            "pm": lambda: orc.bp(og, w.angles, y64, orc.W_PM),
            "adjoint": lambda: orc.siddon_adj(og, w.angles, y64)}
    for kind, fn in refs.items():
        say(f"[backprojection parity] case={name} kind={kind}")
        v = plan.backproject(yt, kind).cpu().numpy()
        e = rel_l2(v, fn())
        say(f"   rel L2 = {e:.3e}")
        assert e <= TOL_BP, (name, kind, e)


@pytest.mark.parametrize("nz", [200, 300, 511, 700])
def test_adjoint_column_heights(orc, nz):
    """Tall, thin volumes whose column heights make the exact adjoint cover 4, 6, 8 and 6 voxels per
    lane (with idle lanes in the last z group for 300, 511 and 700), against the oracle."""
    w = inputs.Workload(f"tall{nz}", (12, 10, nz), (1.0, 1.1, 1.0), (24, nz + 24), (1.6, 1.55), 7, 0, 3,
                        off_origin=(0.4, -0.3, 0.7))
    w.angles = np.sort(np.random.default_rng(nz).uniform(0, 2 * np.pi, 7))
    plan = Plan(w.geometry_dict(), w.angles)
    og = orc.Geometry.from_dict(w.geometry_dict())
    y = inputs.random_array(plan.proj_shape, 500 + nz, kind="uniform")
    say(f"[adjoint column heights] nz={nz}")
    v = plan.backproject(torch.from_numpy(y).to(DEV), "adjoint").cpu().numpy()
    e = rel_l2(v, orc.siddon_adj(og, w.angles, y.astype(np.float64)))
    say(f"   rel L2 = {e:.3e}")
    assert e <= TOL_BP, (nz, e)


@pytest.mark.parametrize("name", CASES)
def test_gpu_adjoint_dot_product(data, name):
    """<A x, y> = <x, A^T y> for the GPU pair, in FP64 over the FP32 outputs.  Non-negative x and y
    keep the sums free of cancellation, so the relative gap measures the operators' mismatch."""
    w, geo, vol, y, og = data[name]
    plan = Plan(geo, w.angles)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.uniform(0, 1, plan.vol_shape).astype(np.float32)).to(DEV)
    yy = torch.from_numpy(rng.uniform(0, 1, plan.proj_shape).astype(np.float32)).to(DEV)
    say(f"[dot product] case={name}")
    ax = plan.forward(x, "siddon").double()
    aty = plan.backproject(yy, "adjoint").double()
    lhs = float((ax * yy.double()).sum())
    rhs = float((x.double() * aty).sum())
    say(f"   relative gap {abs(lhs - rhs) / abs(lhs):.3e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)


def test_angle_ranges_and_accumulate(data):
    w, geo, vol, y, og = data["tiny"]
    plan = Plan(geo, w.angles)
    x = torch.from_numpy(vol).to(DEV)
    say("[ranges] tiny")
    full = plan.forward(x, "siddon")
    part = plan.forward(x, "siddon", angle_begin=5, angle_end=17)
    assert torch.equal(part, full[5:17])
    acc = part.clone()
    plan.forward(x, "siddon", out=acc, accumulate=True, angle_begin=5, angle_end=17)
    torch.testing.assert_close(acc, 2 * part, rtol=1e-6, atol=0)
    yt = torch.from_numpy(y).to(DEV)
    for kind in ("fdk", "adjoint"):
        v_full = plan.backproject(yt, kind)
        v = plan.backproject(yt[:20].contiguous(), kind, angle_end=20)
        plan.backproject(yt[20:].contiguous(), kind, out=v, accumulate=True, angle_begin=20)
        torch.testing.assert_close(v, v_full, rtol=1e-5, atol=1e-5 * float(v_full.abs().max()))


def test_deterministic_repeat(data):
    w, geo, vol, y, og = data["ragged"]
    plan = Plan(geo, w.angles)
    x = torch.from_numpy(vol).to(DEV)
    yt = torch.from_numpy(y).to(DEV)
    say("[determinism] ragged")
    for proj in ("siddon", "interp"):
        assert torch.equal(plan.forward(x, proj), plan.forward(x, proj))
    for kind in ("fdk", "pm", "adjoint"):
        assert torch.equal(plan.backproject(yt, kind), plan.backproject(yt, kind))


def test_degenerate_sizes(orc):
    # one voxel, one pixel, one angle; and a detector whose rays all miss the volume
    for geo in (dict(DSO=500.0, DSD=800.0, nVoxel=(1, 1, 1), dVoxel=(3.0, 3.0, 3.0), offOrigin=(0.2, -0.1, 0.3),
                     nDetector=(1, 1), dDetector=(2.0, 2.0), offDetector=(0.1, 0.2), accuracy=0.5),
                dict(DSO=500.0, DSD=800.0, nVoxel=(4, 3, 2), dVoxel=(1.0, 1.0, 1.0), offOrigin=(0.0, 0.0, 0.0),
                     nDetector=(5, 3), dDetector=(1.0, 1.0), offDetector=(200.0, 0.0), accuracy=0.5)):
        ang = np.array([0.4])
        plan = Plan(geo, ang)
        og = orc.Geometry.from_dict(geo)
        vol = np.random.default_rng(1).uniform(0.5, 1, plan.vol_shape).astype(np.float32)
        say(f"[degenerate] {geo['nVoxel']} {geo['nDetector']}")
        p = plan.forward(torch.from_numpy(vol).to(DEV), "siddon").cpu().numpy()
        ref = orc.siddon_fwd(og, ang, vol.astype(np.float64))
        np.testing.assert_allclose(p, ref, rtol=1e-5, atol=1e-6)
        y = np.ones(plan.proj_shape, np.float32)
        for kind, fn in (("fdk", lambda: orc.bp(og, ang, y.astype(np.float64), orc.W_FDK)),
                         ("adjoint", lambda: orc.siddon_adj(og, ang, y.astype(np.float64)))):
            v = plan.backproject(torch.from_numpy(y).to(DEV), kind).cpu().numpy()
            np.testing.assert_allclose(v, fn(), rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("dt,bound", [(torch.float16, 2.0 ** -11), (torch.bfloat16, 2.0 ** -8)])
def test_16bit_storage(data, orc, dt, bound):
    """16-bit storage, FP32 arithmetic.  The oracle runs in FP64 on the rounded inputs, so the
    kernel error stays at the FP32 bar; a 16-bit output adds at most its rounding (bound)."""
    w, geo, vol, y, og = data["tiny"]
    plan = Plan(geo, w.angles)
    xh = torch.from_numpy(vol).to(DEV).to(dt)
    vol_r = xh.float().cpu().numpy().astype(np.float64)
    ref = orc.siddon_fwd(og, w.angles, vol_r)
    say(f"[16-bit] {dt}")
    p32 = plan.forward(xh, "siddon", out_dtype=torch.float32).cpu().numpy()
    assert rel_l2(p32, ref) <= TOL_PROJ
    p16 = plan.forward(xh, "siddon").float().cpu().numpy()
    assert rel_l2(p16, ref) <= TOL_PROJ + bound
    yh = torch.from_numpy(y).to(DEV).to(dt)
    y_r = yh.float().cpu().numpy().astype(np.float64)
    v = plan.backproject(yh, "fdk", out_dtype=torch.float32).cpu().numpy()
    assert rel_l2(v, orc.bp(og, w.angles, y_r, orc.W_FDK)) <= TOL_BP
    v = plan.backproject(yh, "adjoint", out_dtype=torch.float32).cpu().numpy()
    assert rel_l2(v, orc.siddon_adj(og, w.angles, y_r)) <= TOL_BP
    v16 = plan.backproject(yh, "fdk").float().cpu().numpy()
    assert rel_l2(v16, orc.bp(og, w.angles, y_r, orc.W_FDK)) <= TOL_BP + bound


# ------------------------------------------------------------------------------------------
# the 512^3 / 360-angle / 512^2 workload, sampled


@pytest.fixture(scope="module")
def medium():
    w = inputs.workload("medium")
    vol = inputs.voxelize(w)
    y = inputs.random_array((360, 512, 512), 202, kind="uniform")
    return w, vol, y


def test_medium_forward_sampled(medium, orc):
    w, vol, y = medium
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    x = torch.from_numpy(vol).to(DEV)
    v64 = vol.astype(np.float64)
    idx = inputs.sample_indices(360 * 512 * 512, 4000, 31)
    for proj, fn in (("siddon", orc.siddon_rays), ("interp", orc.interp_rays)):
        say(f"[medium forward sampled] projector={proj}")
        p = plan.forward(x, proj).cpu().numpy().ravel()[idx]
        n = 4000 if proj == "siddon" else 1500
        ref = fn(og, w.angles, idx[:n], v64)
        e = rel_l2(p[:n], ref)
        say(f"   rel L2 = {e:.3e}")
        assert e <= TOL_PROJ


def test_medium_backprojection_sampled(medium, orc):
    w, vol, y = medium
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    yt = torch.from_numpy(y).to(DEV)
    y64 = y.astype(np.float64)
    idx = inputs.sample_indices(512 ** 3, 600, 32)
    for kind, n, fn in (("fdk", 600, lambda i: orc.bp_voxels(og, w.angles, y64, i, orc.W_FDK)),
                        ("pm", 600, lambda i: orc.bp_voxels(og, w.angles, y64, i, orc.W_PM)),
                        ("adjoint", 300, lambda i: orc.siddon_adj_voxels(og, w.angles, y64, i))):
        say(f"[medium backprojection sampled] kind={kind}")
        v = plan.backproject(yt, kind).cpu().numpy().ravel()[idx[:n]]
        e = rel_l2(v, fn(idx[:n]))
        say(f"   rel L2 = {e:.3e}")
        assert e <= TOL_BP
