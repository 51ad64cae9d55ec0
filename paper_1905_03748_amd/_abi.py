"""ctypes binding of ``libct.so`` (declared in ``include/ct.h``): argument marshalling only.

Every function keeps the C name and argument order; pointers are passed as Python ints (device or
host addresses) and streams as ints (``hipStream_t``; 0 = default stream).  A non-zero status
raises ``CtError`` with the library's message.  If the library is not built, loading raises: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libct.so")

CT_OK, CT_ERR_ARG, CT_ERR_GEOMETRY, CT_ERR_DTYPE, CT_ERR_OOM, CT_ERR_CAP, CT_ERR_HIP, CT_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
CT_F32, CT_F16, CT_BF16, CT_F64 = 0, 1, 2, 3
CT_SIDDON, CT_INTERP = 0, 1
CT_BP_FDK, CT_BP_PSEUDO_MATCHED, CT_BP_ADJOINT = 0, 1, 2

STATUS_NAMES = {0: "CT_OK", -1: "CT_ERR_ARG", -2: "CT_ERR_GEOMETRY", -3: "CT_ERR_DTYPE", -4: "CT_ERR_OOM",
                -5: "CT_ERR_CAP", -6: "CT_ERR_HIP", -7: "CT_ERR_STATE"}


class CtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ct_geometry(C.Structure):
    _fields_ = [("DSO", C.c_double), ("DSD", C.c_double),
                ("nVoxel", C.c_int64 * 3), ("dVoxel", C.c_double * 3), ("offOrigin", C.c_double * 3),
                ("nDetector", C.c_int64 * 2), ("dDetector", C.c_double * 2), ("offDetector", C.c_double * 2),
                ("accuracy", C.c_double)]


class ct_ooc_stats(C.Structure):
    _fields_ = [("n_slabs", C.c_int32), ("slab_slices", C.c_int32), ("chunk_angles", C.c_int32),
                ("n_chunks", C.c_int32), ("bytes_h2d", C.c_double), ("bytes_d2h", C.c_double),
                ("t_total_s", C.c_double), ("t_compute_s", C.c_double), ("t_stage_s", C.c_double),
                ("t_other_mem_s", C.c_double), ("t_pin_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_I64 = C.c_int64
_U64 = C.c_uint64
_I32 = C.c_int32
_INT = C.c_int
_D = C.c_double
_ST = C.c_int

SIGNATURES = {
    "ct_plan_create": [C.POINTER(ct_geometry), C.POINTER(C.c_double), _I64, C.POINTER(_P)],
    "ct_plan_create_views": [C.POINTER(ct_geometry), C.POINTER(C.c_double), _I64, C.POINTER(_P)],
    "ct_plan_destroy": [_P],
    "ct_plan_info": [_P, C.POINTER(ct_geometry), C.POINTER(_I64)],
    "ct_forward": [_P, _INT, _P, _INT, _P, _INT, _INT, _I64, _I64, _P],
    "ct_backproject": [_P, _INT, _P, _INT, _P, _INT, _INT, _I64, _I64, _P],
    "ct_backproject_noalloc": [_P, _INT, _P, _INT, _P, _INT, _INT, _I64, _I64, _P],
    "ct_ooc_plan": [_P, _INT, _INT, _INT, _INT, _U64, C.POINTER(ct_ooc_stats)],
    "ct_forward_host": [_P, _INT, _P, _INT, _P, _INT, _U64, C.POINTER(ct_ooc_stats)],
    "ct_backproject_host": [_P, _INT, _P, _INT, _P, _INT, _U64, C.POINTER(ct_ooc_stats)],
    "ct_cgls_workspace_bytes": [_P, _INT, _INT, C.POINTER(_U64)],
    "ct_cgls": [_P, _P, _INT, _P, _INT, _I32, _P, _P, _P],
    "ct_cgls_host_workspace_bytes": [_P, C.POINTER(_U64)],
    "ct_cgls_host": [_P, _P, _P, _I32, _P, _P, _U64, C.POINTER(ct_ooc_stats)],
    "ct_sart_workspace_bytes": [_P, _I32, C.POINTER(_U64)],
    "ct_sart": [_P, _P, _INT, _P, _INT, _I32, _D, _I32, _P, _P],
    "ct_fdk_filter": [_P, _P, _INT, _P, _I64, _I64, _P],
    "ct_fdk_workspace_bytes": [_P, C.POINTER(_U64)],
    "ct_fdk_host": [_P, _P, _INT, _P, _INT, _U64, C.POINTER(ct_ooc_stats)],
    "ct_fdk": [_P, _P, _INT, _P, _INT, _P, _P],
    "ct_tv_workspace_bytes": [C.POINTER(ct_geometry), _INT, C.POINTER(_U64)],
    "ct_tv_steps": [C.POINTER(ct_geometry), _P, _INT, _I32, _D, _D, _P, _P],
    "ct_tv_steps_host": [C.POINTER(ct_geometry), _P, _I32, _D, _D, _I32, _U64, C.POINTER(ct_ooc_stats)],
    "ct_rof_workspace_bytes": [C.POINTER(ct_geometry), C.POINTER(_U64)],
    "ct_rof": [C.POINTER(ct_geometry), _P, _I32, _D, _D, _P, _P],
    "ct_rof_host_workspace_bytes": [C.POINTER(ct_geometry), C.POINTER(_U64)],
    "ct_rof_host": [C.POINTER(ct_geometry), _P, _I32, _D, _D, _I32, _P, _U64, C.POINTER(ct_ooc_stats)],
    "ct_dot": [_P, _P, _INT, _I64, _P, _P],
    "ct_convert": [_P, _INT, _P, _INT, _I64, _P],
    "ct_last_error": [],
    "ct_version": [],
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (or python -m "
                               "paper_1905_03748_amd.build); there is no non-HIP fallback")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_char_p if name in ("ct_last_error", "ct_version") else (None if name == "ct_plan_destroy" else _ST)
        _lib = L
    return _lib


def _check(st):
    if st != CT_OK:
        raise CtError(st, lib().ct_last_error().decode())
    return st


def make_geometry(d: dict) -> ct_geometry:
    g = ct_geometry()
    g.DSO, g.DSD = float(d["DSO"]), float(d["DSD"])
    g.nVoxel[:] = [int(v) for v in d["nVoxel"]]
    g.dVoxel[:] = [float(v) for v in d["dVoxel"]]
    g.offOrigin[:] = [float(v) for v in d.get("offOrigin", (0, 0, 0))]
    g.nDetector[:] = [int(v) for v in d["nDetector"]]
    g.dDetector[:] = [float(v) for v in d["dDetector"]]
    g.offDetector[:] = [float(v) for v in d.get("offDetector", (0, 0))]
    g.accuracy = float(d.get("accuracy", 0.5))
    return g


# --- same names as the C ABI ------------------------------------------------------------------

def ct_plan_create(geometry: ct_geometry, angles) -> int:
    arr = (C.c_double * len(angles))(*[float(a) for a in angles])
    out = _P()
    _check(lib().ct_plan_create(C.byref(geometry), arr, len(angles), C.byref(out)))
    return out.value


def ct_plan_create_views(geometry: ct_geometry, views) -> int:
    """views: n x 12 (source, detector centre, unit e_u, unit e_v per projection; mm)."""
    flat = [float(v) for row in views for v in row]
    if any(len(row) != 12 for row in views):
        raise ValueError("each view has 12 entries: source, detector centre, e_u, e_v")
    arr = (C.c_double * len(flat))(*flat)
    out = _P()
    _check(lib().ct_plan_create_views(C.byref(geometry), arr, len(views), C.byref(out)))
    return out.value


def ct_plan_destroy(plan: int) -> None:
    lib().ct_plan_destroy(plan)


def ct_plan_info(plan: int):
    g = ct_geometry()
    n = _I64()
    _check(lib().ct_plan_info(plan, C.byref(g), C.byref(n)))
    return g, n.value


def ct_forward(plan, projector, d_vol, vol_dtype, d_proj, proj_dtype, accumulate, angle_begin, angle_end, stream=0):
    return _check(lib().ct_forward(plan, projector, d_vol, vol_dtype, d_proj, proj_dtype, int(accumulate),
                                   angle_begin, angle_end, stream or None))


def ct_backproject(plan, backprojector, d_proj, proj_dtype, d_vol, vol_dtype, accumulate, angle_begin, angle_end,
                   stream=0):
    return _check(lib().ct_backproject(plan, backprojector, d_proj, proj_dtype, d_vol, vol_dtype, int(accumulate),
                                       angle_begin, angle_end, stream or None))


def ct_backproject_noalloc(plan, backprojector, d_proj, proj_dtype, d_vol, vol_dtype, accumulate, angle_begin,
                           angle_end, stream=0):
    return _check(lib().ct_backproject_noalloc(plan, backprojector, d_proj, proj_dtype, d_vol, vol_dtype,
                                               int(accumulate), angle_begin, angle_end, stream or None))


def ct_ooc_plan(plan, direction, projector, vol_dtype, proj_dtype, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_ooc_plan(plan, direction, projector, vol_dtype, proj_dtype, int(device_cap_bytes), C.byref(s)))
    return s


def ct_forward_host(plan, projector, h_vol, vol_dtype, h_proj, proj_dtype, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_forward_host(plan, projector, h_vol, vol_dtype, h_proj, proj_dtype, int(device_cap_bytes),
                                 C.byref(s)))
    return s


def ct_backproject_host(plan, backprojector, h_proj, proj_dtype, h_vol, vol_dtype, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_backproject_host(plan, backprojector, h_proj, proj_dtype, h_vol, vol_dtype,
                                     int(device_cap_bytes), C.byref(s)))
    return s


def ct_cgls_workspace_bytes(plan, vol_dtype, proj_dtype) -> int:
    b = _U64()
    _check(lib().ct_cgls_workspace_bytes(plan, vol_dtype, proj_dtype, C.byref(b)))
    return b.value


def ct_cgls(plan, d_b, proj_dtype, d_x, vol_dtype, niter, d_resid=0, d_workspace=0, stream=0):
    return _check(lib().ct_cgls(plan, d_b, proj_dtype, d_x, vol_dtype, niter, d_resid or None, d_workspace or None,
                                stream or None))


def ct_cgls_host_workspace_bytes(plan) -> int:
    b = _U64()
    _check(lib().ct_cgls_host_workspace_bytes(plan, C.byref(b)))
    return b.value


def ct_cgls_host(plan, h_b, h_x, niter, h_resid, h_workspace, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_cgls_host(plan, h_b, h_x, niter, h_resid or None, h_workspace, int(device_cap_bytes),
                              C.byref(s)))
    return s


def ct_sart_workspace_bytes(plan, block=1) -> int:
    b = _U64()
    _check(lib().ct_sart_workspace_bytes(plan, block, C.byref(b)))
    return b.value


def ct_sart(plan, d_b, proj_dtype, d_x, vol_dtype, niter, lam=1.0, block=1, d_workspace=0, stream=0):
    return _check(lib().ct_sart(plan, d_b, proj_dtype, d_x, vol_dtype, niter, float(lam), block, d_workspace or None,
                                stream or None))


def ct_fdk_filter(plan, d_proj, proj_dtype, d_q, angle_begin, angle_end, stream=0):
    return _check(lib().ct_fdk_filter(plan, d_proj, proj_dtype, d_q, angle_begin, angle_end, stream or None))


def ct_fdk_workspace_bytes(plan) -> int:
    b = _U64()
    _check(lib().ct_fdk_workspace_bytes(plan, C.byref(b)))
    return b.value


def ct_fdk_host(plan, h_proj, proj_dtype, h_vol, vol_dtype, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_fdk_host(plan, h_proj, proj_dtype, h_vol, vol_dtype, int(device_cap_bytes), C.byref(s)))
    return s


def ct_fdk(plan, d_proj, proj_dtype, d_vol, vol_dtype, d_workspace=0, stream=0):
    return _check(lib().ct_fdk(plan, d_proj, proj_dtype, d_vol, vol_dtype, d_workspace or None, stream or None))


def ct_tv_workspace_bytes(geometry: ct_geometry, dtype=CT_F32) -> int:
    b = _U64()
    _check(lib().ct_tv_workspace_bytes(C.byref(geometry), dtype, C.byref(b)))
    return b.value


def ct_tv_steps(geometry: ct_geometry, d_x, dtype, nsteps, lam, eps=1e-8, d_workspace=0, stream=0):
    return _check(lib().ct_tv_steps(C.byref(geometry), d_x, dtype, nsteps, float(lam), float(eps), d_workspace or None,
                                    stream or None))


def ct_tv_steps_host(geometry: ct_geometry, h_x, nsteps, lam, eps, halo_depth, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_tv_steps_host(C.byref(geometry), h_x, nsteps, float(lam), float(eps), int(halo_depth),
                                  int(device_cap_bytes), C.byref(s)))
    return s


def ct_rof_workspace_bytes(geometry: ct_geometry) -> int:
    b = _U64()
    _check(lib().ct_rof_workspace_bytes(C.byref(geometry), C.byref(b)))
    return b.value


def ct_rof(geometry: ct_geometry, d_x, niter, lam, tau, d_workspace=0, stream=0):
    return _check(lib().ct_rof(C.byref(geometry), d_x, niter, float(lam), float(tau), d_workspace or None,
                               stream or None))


def ct_rof_host_workspace_bytes(geometry: ct_geometry) -> int:
    b = _U64()
    _check(lib().ct_rof_host_workspace_bytes(C.byref(geometry), C.byref(b)))
    return b.value


def ct_rof_host(geometry: ct_geometry, h_x, niter, lam, tau, halo_depth, h_workspace, device_cap_bytes) -> ct_ooc_stats:
    s = ct_ooc_stats()
    _check(lib().ct_rof_host(C.byref(geometry), h_x, niter, float(lam), float(tau), int(halo_depth), h_workspace,
                             int(device_cap_bytes), C.byref(s)))
    return s


def ct_dot(d_a, d_b, dtype, n, d_out, stream=0):
    return _check(lib().ct_dot(d_a, d_b, dtype, n, d_out, stream or None))


def ct_convert(d_src, src_dtype, d_dst, dst_dtype, n, stream=0):
    return _check(lib().ct_convert(d_src, src_dtype, d_dst, dst_dtype, n, stream or None))


def ct_last_error() -> str:
    return lib().ct_last_error().decode()


def ct_version() -> str:
    return lib().ct_version().decode()
