"""Host-side checks of the C ABI that need no GPU: the library loads and exports every function
declared in include/ct.h; geometry validation; the out-of-core slab/chunk planner (Algorithms 1
and 2: equal axial slabs as tall as the memory cap allows, projection chunk buffers)."""
import os
import re

import numpy as np
import pytest

from paper_1905_03748_amd import _abi as A
from paper_1905_03748_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return A.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18, names
    for n in names:
        assert hasattr(lib, n), n
        assert n in A.SIGNATURES, f"binding lacks {n}"
    assert A.ct_version().startswith("ct-mi355x")


def _geo(**kw):
    d = inputs.workload("tiny").geometry_dict()
    d.update(kw)
    return A.make_geometry(d)


def test_plan_create_and_info(lib):
    w = inputs.workload("tiny")
    p = A.ct_plan_create(_geo(), w.angles)
    g, n = A.ct_plan_info(p)
    assert n == 64 and g.nVoxel[:] == [64, 64, 64] and g.accuracy == 0.5
    A.ct_plan_destroy(p)
    p = A.ct_plan_create(_geo(accuracy=0.0), w.angles)   # 0 selects the default spacing
    assert A.ct_plan_info(p)[0].accuracy == 0.5
    A.ct_plan_destroy(p)


@pytest.mark.parametrize("kw,status", [
    (dict(DSD=900.0), A.CT_ERR_GEOMETRY),                      # DSD <= DSO
    (dict(DSO=-1.0), A.CT_ERR_GEOMETRY),
    (dict(nVoxel=(64, 0, 64)), A.CT_ERR_GEOMETRY),
    (dict(dVoxel=(1.0, -1.0, 1.0)), A.CT_ERR_GEOMETRY),
    (dict(dDetector=(0.0, 1.6)), A.CT_ERR_GEOMETRY),
    (dict(dVoxel=(40.0, 40.0, 1.0)), A.CT_ERR_GEOMETRY),      # volume reaches past the source orbit
    (dict(offOrigin=(990.0, 0.0, 0.0)), A.CT_ERR_GEOMETRY),
    (dict(accuracy=1.5), A.CT_ERR_GEOMETRY),
])
def test_plan_validation(lib, kw, status):
    with pytest.raises(A.CtError) as e:
        A.ct_plan_create(_geo(**kw), [0.0, 1.0])
    assert e.value.status == status
    assert A.ct_last_error()


def test_plan_rejects_bad_angles(lib):
    with pytest.raises(A.CtError) as e:
        A.ct_plan_create(_geo(), [0.0, float("nan")])
    assert e.value.status == A.CT_ERR_GEOMETRY
    with pytest.raises(A.CtError) as e:
        A.ct_plan_create(_geo(), [])
    assert e.value.status == A.CT_ERR_ARG


def test_calls_validate_before_device_work(lib):
    w = inputs.workload("tiny")
    p = A.ct_plan_create(_geo(), w.angles)
    try:
        for call in (lambda: A.ct_forward(p, A.CT_SIDDON, 0, A.CT_F32, 0, A.CT_F32, 0, 0, 64),
                     lambda: A.ct_forward(p, 7, 16, A.CT_F32, 16, A.CT_F32, 0, 0, 64),
                     lambda: A.ct_forward(p, A.CT_SIDDON, 16, A.CT_F32, 16, A.CT_F32, 0, 5, 5),
                     lambda: A.ct_forward(p, A.CT_SIDDON, 16, A.CT_F32, 16, A.CT_F32, 0, 0, 65),
                     lambda: A.ct_backproject(p, 9, 16, A.CT_F32, 16, A.CT_F32, 0, 0, 64),
                     lambda: A.ct_sart(p, 16, A.CT_F32, 16, A.CT_F32, 1, 1.0, 0),
                     lambda: A.ct_sart(p, 16, A.CT_F32, 16, A.CT_F32, 1, 1.0, 65),
                     lambda: A.ct_sart_workspace_bytes(p, 0),
                     lambda: A.ct_cgls(p, 16, A.CT_F32, 16, A.CT_F32, -1)):
            with pytest.raises(A.CtError) as e:
                call()
            assert e.value.status == A.CT_ERR_ARG
        with pytest.raises(A.CtError) as e:
            A.ct_forward(p, A.CT_SIDDON, 16, 9, 16, A.CT_F32, 0, 0, 64)
        assert e.value.status == A.CT_ERR_DTYPE
        # FP64 is a conversion and inner-product type only: the operators and algorithms refuse it
        # before any device work
        g = _geo()
        for call in (lambda: A.ct_forward(p, A.CT_SIDDON, 16, A.CT_F64, 16, A.CT_F32, 0, 0, 64),
                     lambda: A.ct_backproject(p, A.CT_BP_FDK, 16, A.CT_F32, 16, A.CT_F64, 0, 0, 64),
                     lambda: A.ct_sart(p, 16, A.CT_F64, 16, A.CT_F32, 1, 1.0, 1),
                     lambda: A.ct_sart(p, 16, A.CT_F32, 16, 5, 1, 1.0, 1),
                     lambda: A.ct_cgls(p, 16, A.CT_F32, 16, A.CT_F64, 1),
                     lambda: A.ct_tv_steps(g, 16, A.CT_F64, 1, 0.01),
                     lambda: A.ct_tv_workspace_bytes(g, A.CT_F64),
                     lambda: A.ct_convert(16, 4, 16, A.CT_F32, 1),
                     lambda: A.ct_dot(16, 16, 4, 1, 16)):
            with pytest.raises(A.CtError) as e:
                call()
            assert e.value.status == A.CT_ERR_DTYPE
    finally:
        A.ct_plan_destroy(p)


def test_tv_workspace_grows_for_16bit_storage(lib):
    g = _geo()
    f32 = A.ct_tv_workspace_bytes(g, A.CT_F32)
    # one more FP32 volume (64^3, 256-byte aligned) holds the FP32 copy of a 16-bit image
    for dt in (A.CT_F16, A.CT_BF16):
        assert A.ct_tv_workspace_bytes(g, dt) == f32 + 64 ** 3 * 4


def test_ooc_stats_layout_matches_header(lib):
    src = open(os.path.join(ROOT, "include", "ct.h")).read()
    body = src[src.index("typedef struct {\n    int32_t n_slabs"):src.index("} ct_ooc_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(int32_t|double)\s+([a-z_0-9]+)\s*;", body)
    assert [n for _, n in fields] == [n for n, _ in A.ct_ooc_stats._fields_]
    assert "t_pin_s" in dict(A.ct_ooc_stats._fields_)


def test_ooc_planner_out_of_core_config(lib):
    # 3072^3 FP32 volume (108 GiB), 3072 projections of 3072^2, 32 GiB device cap
    w = inputs.workload("ooc")
    p = A.ct_plan_create(A.make_geometry(w.geometry_dict()), w.angles)
    try:
        fw = A.ct_ooc_plan(p, 0, A.CT_SIDDON, A.CT_F32, A.CT_F32, 32 << 30)
        slice_b = 3072 * 3072 * 4
        assert fw.n_slabs == 4 and fw.slab_slices == 768, fw.as_dict()
        assert fw.slab_slices * slice_b + 3 * fw.chunk_angles * slice_b <= 32 << 30
        bp = A.ct_ooc_plan(p, 1, A.CT_SIDDON, A.CT_F32, A.CT_F32, 32 << 30)
        assert bp.n_slabs == 4 and bp.slab_slices * slice_b + 2 * bp.chunk_angles * slice_b <= 32 << 30
        # the exact adjoint adds its transposed copy (3072 x 3074 float pairs per angle) and keeps
        # the fewest slabs, taking the largest chunk that allows them
        adj = A.ct_ooc_plan(p, 2, A.CT_SIDDON, A.CT_F32, A.CT_F32, 32 << 30)
        per = 3072 * 3074 * 8
        assert adj.n_slabs == 4 and adj.chunk_angles == 32, adj.as_dict()
        assert adj.slab_slices * slice_b + adj.chunk_angles * (2 * slice_b + per) <= 32 << 30
        # FP16 storage halves the slabs
        h = A.ct_ooc_plan(p, 0, A.CT_SIDDON, A.CT_F16, A.CT_F16, 32 << 30)
        assert h.n_slabs == 2 and h.slab_slices == 1536
        # a cap below one slice plus the buffers fails cleanly
        with pytest.raises(A.CtError) as e:
            A.ct_ooc_plan(p, 0, A.CT_SIDDON, A.CT_F32, A.CT_F32, 100 << 20)
        assert e.value.status == A.CT_ERR_CAP
    finally:
        A.ct_plan_destroy(p)


def test_ooc_planner_equal_slabs_and_halo(lib):
    w = inputs.workload("tiny")
    p = A.ct_plan_create(_geo(), w.angles)
    reserve = 64 << 20
    try:
        slice_b = 64 * 64 * 4
        pangle = 64 * 64 * 4
        for nslices in (1, 5, 13, 40, 64, 100):
            cap = reserve + 3 * 64 * pangle + nslices * slice_b
            for kind, halo in ((A.CT_SIDDON, 0), (A.CT_INTERP, 1)):
                for direction, nbuf in ((0, 3), (1, 2), (2, 2), (3, 2)):
                    s = A.ct_ooc_plan(p, direction, kind, A.CT_F32, A.CT_F32, cap)
                    h = halo if direction == 0 else 0
                    adj = s.chunk_angles * 64 * 66 * 4 if direction == 2 else 0
                    filt = s.chunk_angles * 64 * 64 * 4 if direction == 3 else 0   # FDK's filtered chunk
                    assert s.n_slabs * s.slab_slices >= 64
                    assert s.slab_slices == -(-64 // s.n_slabs)            # equal slabs
                    assert (s.n_slabs - 1) * s.slab_slices < 64
                    assert (reserve + (s.slab_slices + 2 * h) * slice_b + nbuf * s.chunk_angles * pangle + adj + filt
                            <= cap)
                    assert s.n_chunks == -(-64 // s.chunk_angles)
                # the filtered chunk costs room: never fewer slabs than the plain FDK backprojection
                assert (A.ct_ooc_plan(p, 3, kind, A.CT_F32, A.CT_F32, cap).n_slabs
                        >= A.ct_ooc_plan(p, 1, kind, A.CT_F32, A.CT_F32, cap).n_slabs)
            for bad in (-1, 4):
                with pytest.raises(A.CtError) as e:
                    A.ct_ooc_plan(p, bad, A.CT_SIDDON, A.CT_F32, A.CT_F32, cap)
                assert e.value.status == A.CT_ERR_ARG
            # with room for the whole volume and full chunks: one slab
            if nslices >= 64:
                assert A.ct_ooc_plan(p, 0, A.CT_SIDDON, A.CT_F32, A.CT_F32, cap).n_slabs == 1
    finally:
        A.ct_plan_destroy(p)


def test_host_operators_reject_wrong_shapes_before_the_library(lib):
    """The out-of-core wrappers pass raw host pointers: a tensor of the wrong shape, device, layout
    or dtype is refused with ValueError (also under python -O) before anything reaches the library."""
    import torch
    from paper_1905_03748_amd.operators import Plan
    w = inputs.workload("tiny")
    plan = Plan(w.geometry_dict(), w.angles)
    vol = torch.zeros(plan.vol_shape)
    proj = torch.zeros(plan.proj_shape)
    short_proj = torch.zeros((plan.n_angles - 1,) + plan.proj_shape[1:])
    short_vol = torch.zeros((plan.vol_shape[0] - 1,) + plan.vol_shape[1:])
    bad = [
        lambda: plan.forward_host(vol, short_proj),
        lambda: plan.forward_host(short_vol, proj),
        lambda: plan.forward_host(vol, proj.view(-1)),                  # right size, wrong shape
        lambda: plan.forward_host(vol, torch.zeros(plan.proj_shape[::-1]).transpose(0, 2)),   # not contiguous
        lambda: plan.forward_host(vol.double(), proj),
        lambda: plan.backproject_host(short_proj, vol),
        lambda: plan.backproject_host(proj, short_vol),
        lambda: plan.backproject_host(proj, vol.to(torch.int32)),
        lambda: plan.fdk_host(proj, short_vol),
        lambda: plan.fdk_host(short_proj, vol),
    ]
    for k, call in enumerate(bad):
        with pytest.raises(ValueError):
            call()
    plan.close()


def test_plan_of_views_validation(lib):
    """ct_plan_create_views (per-view geometry, Section 2.1) checks every view on the host."""
    w = inputs.workload("tiny")
    views = inputs.carm_views(w.DSO, w.DSD, w.angles[:8], 3)
    p = A.ct_plan_create_views(_geo(), views.tolist())
    g, n = A.ct_plan_info(p)
    assert n == 8 and g.DSD > g.DSO > 0
    A.ct_plan_destroy(p)
    helical = inputs.helical_views(w.DSO, w.DSD, w.angles, 20.0)
    A.ct_plan_destroy(A.ct_plan_create_views(_geo(), helical.tolist()))

    def bad(mutate):
        v = views.copy()
        mutate(v)
        with pytest.raises(A.CtError) as e:
            A.ct_plan_create_views(_geo(), v.tolist())
        assert e.value.status == A.CT_ERR_GEOMETRY, A.ct_last_error()

    bad(lambda v: v.__setitem__((2, 6), v[2, 6] * 1.01))          # e_u not a unit vector
    bad(lambda v: v.__setitem__((1, slice(9, 12)), (v[1, 9:12] + 0.01 * v[1, 6:9]) / np.linalg.norm(v[1, 9:12] + 0.01 * v[1, 6:9])))  # not orthogonal
    bad(lambda v: v.__setitem__((0, slice(6, 9)), -v[0, 6:9]))    # normal turned away from the source
    bad(lambda v: v.__setitem__((3, slice(0, 3)), 0.0))           # source inside the volume box
    bad(lambda v: v.__setitem__((5, 4), float("nan")))
    with pytest.raises(A.CtError) as e:
        A.ct_plan_create_views(_geo(), [])
    assert e.value.status == A.CT_ERR_ARG
    with pytest.raises(ValueError):
        A.ct_plan_create_views(_geo(), [[0.0] * 11])


def test_plan_of_views_refuses_the_circular_only_calls(lib):
    """The FDK reconstruction and the out-of-core calls need a circular orbit; a plan of views is
    refused with CT_ERR_ARG before any device work (dummy pointers are never touched)."""
    w = inputs.workload("tiny")
    p = A.ct_plan_create_views(_geo(), inputs.carm_views(w.DSO, w.DSD, w.angles[:4], 5).tolist())
    try:
        for call in (lambda: A.ct_fdk_filter(p, 16, A.CT_F32, 16, 0, 4),
                     lambda: A.ct_fdk(p, 16, A.CT_F32, 16, A.CT_F32),
                     lambda: A.ct_fdk_host(p, 16, A.CT_F32, 16, A.CT_F32, 1 << 30),
                     lambda: A.ct_forward_host(p, A.CT_SIDDON, 16, A.CT_F32, 16, A.CT_F32, 1 << 30),
                     lambda: A.ct_backproject_host(p, A.CT_BP_FDK, 16, A.CT_F32, 16, A.CT_F32, 1 << 30),
                     lambda: A.ct_ooc_plan(p, 0, A.CT_SIDDON, A.CT_F32, A.CT_F32, 1 << 30)):
            with pytest.raises(A.CtError) as e:
                call()
            assert e.value.status == A.CT_ERR_ARG and "circular" in A.ct_last_error(), A.ct_last_error()
    finally:
        A.ct_plan_destroy(p)
