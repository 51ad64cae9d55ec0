"""FDK reconstruction on the GPU (ct_fdk_filter, ct_fdk) against the FP64 oracle: the weighted and
filtered projections (1e-5 relative L2, the projection bar) and the reconstruction (1e-4, the
backprojection bar), on the tiny workload, a ragged geometry with detector offsets, 16-bit inputs,
the oracle's sphere pin case and sampled outputs at the 512^3, 360-angle size."""
import numpy as np
import pytest
import torch

from _helpers import TOL_BP, TOL_PROJ, rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(w, proj, orc):
    geo = w.geometry_dict()
    return Plan(geo, w.angles), orc.Geometry.from_dict(geo), torch.from_numpy(proj).to(DEV)


@pytest.fixture(scope="module")
def tiny(orc):
    w = inputs.workload("tiny")
    p = inputs.analytic_projections(w, inputs.ellipsoids(w)).astype(np.float32)
    return (w, p) + _case(w, p, orc)


def test_fdk_filter_parity_tiny(tiny, orc):
    w, p, plan, og, pt = tiny
    say("[fdk] filter, tiny, all angles and the angle range [5, 17)")
    q = plan.fdk_filter(pt).cpu().numpy()
    ref = orc.fdk_filter(og, w.angles, p.astype(np.float64))
    e = rel_l2(q, ref)
    say(f"   rel L2 {e:.3e}")
    assert e <= TOL_PROJ
    # a sub-range: the same rows, still scaled by the plan's full angle count
    qs = plan.fdk_filter(pt[5:17].contiguous(), angle_begin=5, angle_end=17).cpu().numpy()
    assert rel_l2(qs, ref[5:17]) <= TOL_PROJ


def test_fdk_parity_tiny(tiny, orc):
    w, p, plan, og, pt = tiny
    say("[fdk] reconstruction, tiny, with and without a caller workspace")
    v = plan.fdk(pt).cpu().numpy()
    ref = orc.fdk(og, w.angles, p.astype(np.float64))
    e = rel_l2(v, ref)
    say(f"   rel L2 {e:.3e}")
    assert e <= TOL_BP
    ws = torch.empty(plan.fdk_workspace_bytes(), dtype=torch.uint8, device=DEV)
    v2 = plan.fdk(pt, workspace=ws).cpu().numpy()
    np.testing.assert_array_equal(v, v2)


def test_fdk_ragged_with_offsets(orc):
    """Odd, non-square sizes (a detector row of 77 pixels: two partial waves), offsets of the
    origin and the detector, 13 angles not dividing anything."""
    w = inputs.Workload("fdk_ragged", (37, 29, 23), (1.3, 1.1, 0.9), (77, 19), (1.7, 1.9), 13, 6, 41,
                        off_origin=(1.5, -2.0, 0.7), off_detector=(2.3, -1.4))
    p = inputs.random_array((13, 19, 77), 43, kind="uniform")
    plan, og, pt = _case(w, p, orc)
    say("[fdk] ragged geometry: filter and reconstruction")
    q = plan.fdk_filter(pt).cpu().numpy()
    assert rel_l2(q, orc.fdk_filter(og, w.angles, p.astype(np.float64))) <= TOL_PROJ
    v = plan.fdk(pt).cpu().numpy()
    e = rel_l2(v, orc.fdk(og, w.angles, p.astype(np.float64)))
    say(f"   reconstruction rel L2 {e:.3e}")
    assert e <= TOL_BP


@pytest.mark.parametrize("dt", [torch.float16, torch.bfloat16])
def test_fdk_16bit_projections(tiny, orc, dt):
    """16-bit projections: the oracle runs on the same rounded values, so only the kernels' FP32
    arithmetic separates the two; the volume is written in FP32 and in the 16-bit type."""
    w, p, plan, og, _ = tiny
    say(f"[fdk] 16-bit projections {dt}")
    p16 = torch.from_numpy(p).to(dt)
    ref = orc.fdk(og, w.angles, p16.float().numpy().astype(np.float64))
    v = plan.fdk(p16.to(DEV)).cpu().numpy()
    assert rel_l2(v, ref) <= TOL_BP
    v16 = plan.fdk(p16.to(DEV), out_dtype=dt).float().cpu().numpy()
    unit = 2.0 ** -11 if dt == torch.float16 else 2.0 ** -8
    assert rel_l2(v16, ref) <= unit


def test_fdk_reconstructs_a_centred_sphere(orc):
    """The oracle's sphere pin, on the GPU: the reconstruction of a unit sphere from its exact line
    integrals is 1 within 0.5 % inside, in the middle slices."""
    w = inputs.Workload("fdk_pin", (64, 64, 64), (1.0, 1.0, 1.0), (128, 128), (1.0, 1.0), 64, 0, 0,
                        DSO=60.0, DSD=90.0)
    ells = [inputs.Ellipsoid(np.zeros(3), np.array([28.0] * 3), 1.0, np.eye(3))]
    p = inputs.analytic_projections(w, ells).astype(np.float32)
    plan, og, pt = _case(w, p, orc)
    say("[fdk] centred sphere")
    v = plan.fdk(pt).cpu().numpy()
    c = inputs.voxel_centres_1d(64, 1.0, 0.0)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    m = (np.sqrt(xx ** 2 + yy ** 2 + zz ** 2) < 22.0) & (np.abs(zz) <= 1.0)
    err = np.max(np.abs(v[m] - 1.0))
    say(f"   max interior error {err:.2e}")
    assert err <= 5e-3
    assert rel_l2(v, orc.fdk(og, w.angles, p.astype(np.float64))) <= TOL_BP


@pytest.mark.parametrize("nu", [700, 2049, 3072, 4096])
def test_fdk_filter_wide_rows(orc, nu):
    """Rows of up to 4096 pixels (the filter's limit; 3072 is the splitting workload's detector):
    one row per block of up to 512 threads instead of several rows per block."""
    w = inputs.Workload("fdk_wide", (16, 16, 8), (1.0, 1.0, 1.0), (nu, 5), (0.1, 1.0), 6, 0, 0,
                        off_detector=(0.37, 0.0))
    p = inputs.random_array((6, 5, nu), 60 + nu, kind="uniform")
    plan, og, pt = _case(w, p, orc)
    say(f"[fdk] filter, rows of {nu} pixels")
    q = plan.fdk_filter(pt).cpu().numpy()
    e = rel_l2(q, orc.fdk_filter(og, w.angles, p.astype(np.float64)))
    say(f"   rel L2 {e:.3e}")
    assert e <= TOL_PROJ


@pytest.mark.parametrize("nu", [1, 2, 3, 9])
def test_fdk_degenerate_rows(orc, nu):
    """Rows of 1 to 9 pixels: no odd offset at all (1), a single tap pair, and a row shorter than
    one thread's 8 outputs; the reconstruction too."""
    w = inputs.Workload("fdk_short", (6, 5, 4), (1.0, 1.0, 1.0), (nu, 2), (1.3, 1.1), 3, 0, 0)
    p = inputs.random_array((3, 2, nu), 90 + nu, kind="uniform")
    plan, og, pt = _case(w, p, orc)
    say(f"[fdk] rows of {nu} pixels")
    assert rel_l2(plan.fdk_filter(pt).cpu().numpy(), orc.fdk_filter(og, w.angles, p.astype(np.float64))) <= TOL_PROJ
    assert rel_l2(plan.fdk(pt).cpu().numpy(), orc.fdk(og, w.angles, p.astype(np.float64))) <= TOL_BP


def test_fdk_medium_sampled(orc):
    """512^3, 360 angles, 512^2 detector (the benchmark's size, in the launch the benchmark times):
    filtered rows at 2000 sampled pixels, and the reconstruction at 400 sampled voxels against the
    oracle's FDK-weighted backprojection of the oracle's own filtered projections."""
    w = inputs.workload("medium")
    y = inputs.random_array((360, 512, 512), 202, kind="uniform")
    plan, og, yt = _case(w, y, orc)
    say("[fdk] medium: oracle filter (FP64) of all 360 x 512 rows")
    qref = orc.fdk_filter(og, w.angles, y)
    say("[fdk] medium: GPU filter and reconstruction")
    q = plan.fdk_filter(yt).cpu().numpy()
    pix = inputs.sample_indices(q.size, 2000, 51)
    e = rel_l2(q.ravel()[pix], qref.ravel()[pix])
    say(f"   filter rel L2 (sampled) {e:.3e}")
    assert e <= TOL_PROJ
    v = plan.fdk(yt).cpu().numpy().ravel()
    vox = inputs.sample_indices(512 ** 3, 400, 52)
    ref = orc.bp_voxels(og, w.angles, qref, vox, orc.W_FDK)
    e = rel_l2(v[vox], ref)
    say(f"   reconstruction rel L2 (sampled) {e:.3e}")
    assert e <= TOL_BP


def test_fdk_splitting_geometry_sampled(orc):
    """The splitting workload's geometry (3072^3 of 256/3072 mm, 3072^2 detector of 0.8*512/3072 mm)
    at 4 of its angles, resident (a 108 GiB FP32 volume in device memory), on the exact line
    integrals of 6 of its phantom's ellipsoids: the filtered rows, and the reconstruction at 400
    sampled voxels against the oracle's FDK-weighted backprojection of its own filtered rows.
    (Ramp-filtered noise at the same geometry: test_backprojectors_3072_detector_ramp_noise.)"""
    base = inputs.workload("ooc")
    w = inputs.Workload("ooc_4", base.nvox, base.dvox, base.ndet, base.ddet, 4, 6, base.seed,
                        angles=np.asarray(base.angles)[[0, 768, 1536, 2304]])
    say("[fdk] 3072^3 geometry, 4 angles: exact line integrals of 6 ellipsoids")
    y = inputs.analytic_projections(w, inputs.ellipsoids(w))
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    say("[fdk] 3072^3 geometry: oracle filter")
    qref = orc.fdk_filter(og, w.angles, y)
    say("[fdk] 3072^3 geometry: GPU reconstruction")
    yt = torch.from_numpy(y).to(DEV)
    q = plan.fdk_filter(yt).cpu().numpy()
    e = rel_l2(q, qref)
    say(f"   filter rel L2 {e:.3e}")
    assert e <= TOL_PROJ
    vol = plan.fdk(yt)
    vox = inputs.sample_indices(3072 ** 3, 400, 405)
    got = vol.view(-1)[torch.from_numpy(vox).to(DEV)].cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    ref = orc.bp_voxels(og, w.angles, qref, vox, orc.W_FDK)
    e = rel_l2(got, ref)
    say(f"   reconstruction rel L2 (sampled) {e:.3e}")
    assert e <= TOL_BP


def test_backprojectors_3072_detector_ramp_noise(orc):
    """The splitting workload's geometry (3072^3 voxels of 256/3072 mm, 3072^2 detector) at 4 of its
    angles on ramp-filtered uniform noise: data that changes by its full size from pixel to pixel,
    which is what the FDK reconstruction feeds the backprojector.  Every detector coordinate is
    above 2048 pixels from the edge somewhere, where an FP32 coordinate is resolved to only 2.4e-4
    pixel; the kernels form each voxel's coordinate as a small offset from a tile reference
    projected in FP64.  FDK-weighted, pseudo-matched and exact-adjoint backprojections of the same
    FP32 rows, each at 600 sampled voxels against the oracle (1e-4), then the whole FDK
    reconstruction of the noise."""
    base = inputs.workload("ooc")
    w = inputs.Workload("ooc_4", base.nvox, base.dvox, base.ndet, base.ddet, 4, 6, base.seed,
                        angles=np.asarray(base.angles)[[0, 769, 1536, 2305]])
    geo = w.geometry_dict()
    plan = Plan(geo, w.angles)
    og = orc.Geometry.from_dict(geo)
    noise = inputs.random_array(plan.proj_shape, 406, kind="uniform")
    say("[bp3072] oracle ramp filter of 4 x 3072^2 uniform noise")
    y64 = orc.fdk_filter(og, w.angles, noise.astype(np.float64))
    y = y64.astype(np.float32)
    yt = torch.from_numpy(y).to(DEV)
    vox = inputs.sample_indices(3072 ** 3, 600, 407)
    vt = torch.from_numpy(vox).to(DEV)
    vol = torch.empty(plan.vol_shape, dtype=torch.float32, device=DEV)
    refs = {"fdk": lambda: orc.bp_voxels(og, w.angles, y, vox, orc.W_FDK),
            "pm": lambda: orc.bp_voxels(og, w.angles, y, vox, orc.W_PM),
            "adjoint": lambda: orc.siddon_adj_voxels(og, w.angles, y, vox)}
    errs = {}
    for kind, ref_fn in refs.items():
        say(f"[bp3072] {kind} backprojection, 3072^3 x 4 angles, resident")
        plan.backproject(yt, kind, out=vol)
        got = vol.view(-1)[vt].cpu().numpy()
        errs[kind] = rel_l2(got, ref_fn())
        say(f"   {kind} rel L2 (600 sampled voxels) {errs[kind]:.3e}")
    say("[bp3072] FDK reconstruction of the noise")
    plan.fdk(torch.from_numpy(noise).to(DEV), out=vol)
    got = vol.view(-1)[vt].cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    errs["fdk_recon"] = rel_l2(got, orc.bp_voxels(og, w.angles, y64, vox, orc.W_FDK))
    say(f"   reconstruction rel L2 (sampled) {errs['fdk_recon']:.3e}")
    for kind, e in errs.items():
        assert e <= TOL_BP, (kind, e)


def test_fdk_rejects_bad_arguments(tiny):
    from paper_1905_03748_amd import _abi as A
    w, p, plan, og, pt = tiny
    q = torch.empty(plan.proj_shape, dtype=torch.float32, device=DEV)
    for a0, a1 in ((4, 4), (-1, 3), (0, plan.n_angles + 1)):
        with pytest.raises(A.CtError) as ei:
            A.ct_fdk_filter(plan.handle, pt.data_ptr(), A.CT_F32, q.data_ptr(), a0, a1, 0)
        assert ei.value.status == A.CT_ERR_ARG
    with pytest.raises(A.CtError) as ei:
        A.ct_fdk(plan.handle, 0, A.CT_F32, q.data_ptr(), A.CT_F32, 0, 0)
    assert ei.value.status == A.CT_ERR_ARG
    with pytest.raises(A.CtError) as ei:
        A.ct_fdk(plan.handle, pt.data_ptr(), 7, q.data_ptr(), A.CT_F32, 0, 0)
    assert ei.value.status == A.CT_ERR_DTYPE
    # rows longer than the filter's LDS row: rejected before any launch
    g = dict(w.geometry_dict(), nDetector=(4100, 2), dDetector=(0.01, 1.0))
    wide = Plan(g, w.angles[:2])
    with pytest.raises(A.CtError) as ei:
        A.ct_fdk_filter(wide.handle, q.data_ptr(), A.CT_F32, q.data_ptr(), 0, 2, 0)
    assert ei.value.status == A.CT_ERR_ARG
    with pytest.raises(ValueError):
        plan.fdk(pt, workspace=torch.empty(16, dtype=torch.uint8, device=DEV))
    with pytest.raises(TypeError):
        plan.fdk_filter(pt, out=torch.empty(plan.proj_shape, dtype=torch.float16, device=DEV))
