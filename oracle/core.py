"""ctypes wrapper of the oracle's C operators (test infrastructure only).

Arrays are numpy float64, C-contiguous, volumes [z][y][x] and projections [angle][v][u].
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

W_FDK = 0
W_PM = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Geom(C.Structure):
    _fields_ = [("DSO", C.c_double), ("DSD", C.c_double),
                ("nvox", C.c_int64 * 3), ("dvox", C.c_double * 3), ("offorig", C.c_double * 3),
                ("ndet", C.c_int64 * 2), ("ddet", C.c_double * 2), ("offdet", C.c_double * 2),
                ("accuracy", C.c_double)]


@dataclass
class Geometry:
    """Circular cone-beam geometry in mm (the oracle's own copy of the conventions)."""
    DSO: float
    DSD: float
    nVoxel: tuple
    dVoxel: tuple
    offOrigin: tuple = (0.0, 0.0, 0.0)
    nDetector: tuple = (1, 1)
    dDetector: tuple = (1.0, 1.0)
    offDetector: tuple = (0.0, 0.0)
    accuracy: float = 0.5

    @classmethod
    def from_dict(cls, d: dict) -> "Geometry":
        return cls(d["DSO"], d["DSD"], tuple(d["nVoxel"]), tuple(d["dVoxel"]), tuple(d["offOrigin"]),
                   tuple(d["nDetector"]), tuple(d["dDetector"]), tuple(d["offDetector"]),
                   d.get("accuracy", 0.5))

    def c(self) -> _Geom:
        g = _Geom()
        g.DSO, g.DSD = self.DSO, self.DSD
        g.nvox[:] = [int(v) for v in self.nVoxel]
        g.dvox[:] = [float(v) for v in self.dVoxel]
        g.offorig[:] = [float(v) for v in self.offOrigin]
        g.ndet[:] = [int(v) for v in self.nDetector]
        g.ddet[:] = [float(v) for v in self.dDetector]
        g.offdet[:] = [float(v) for v in self.offDetector]
        g.accuracy = self.accuracy
        return g

    @property
    def vol_shape(self):
        nx, ny, nz = self.nVoxel
        return (nz, ny, nx)

    def proj_shape(self, n_angles):
        nu, nv = self.nDetector
        return (n_angles, nv, nu)


def load():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = C.CDLL(path)
        P = C.POINTER
        d, i64 = C.c_double, C.c_int64
        pd, pi = P(d), P(i64)
        g = P(_Geom)
        sig = {
            "orc_set_threads": (None, [C.c_int]),
            "orc_get_threads": (C.c_int, []),
            "orc_ray_endpoints": (None, [g, pd, d, d, pd, pd]),
            "orc_circular_views": (None, [g, pd, i64, pd]),
            "orc_siddon_ray": (d, [g, pd, pd, pd, pi]),
            "orc_interp_ray": (d, [g, pd, pd, pd, pi]),
            "orc_siddon_fwd": (None, [g, pd, i64, pd, pd, pi]),
            "orc_siddon_rays": (None, [g, pd, pi, i64, pd, pd]),
            "orc_siddon_segments": (None, [g, pd, pi, i64, pi]),
            "orc_siddon_adj": (None, [g, pd, i64, pd, pd]),
            "orc_siddon_adj_voxels": (None, [g, pd, i64, pd, pi, i64, pd]),
            "orc_interp_fwd": (None, [g, pd, i64, pd, pd, pi]),
            "orc_interp_rays": (None, [g, pd, pi, i64, pd, pd]),
            "orc_bp": (None, [g, pd, i64, pd, C.c_int, pd]),
            "orc_bp_voxels": (None, [g, pd, i64, pd, C.c_int, pi, i64, pd]),
            "orc_siddon_rays_f32": (None, [g, pd, pi, i64, C.POINTER(C.c_float), pd]),
            "orc_bp_voxels_f32": (None, [g, pd, i64, C.POINTER(C.c_float), C.c_int, pi, i64, pd]),
            "orc_siddon_adj_voxels_f32": (None, [g, pd, i64, C.POINTER(C.c_float), pi, i64, pd]),
            "orc_bp_transpose": (None, [g, pd, i64, pd, C.c_int, pd]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def circular_views(geo: Geometry, angles):
    """The per-view table (source, detector centre, e_u, e_v; n x 12) of a circular orbit."""
    angles = _f64(np.atleast_1d(angles))
    out = np.zeros((len(angles), 12))
    load().orc_circular_views(C.byref(geo.c()), _pd(angles), len(angles), _pd(out))
    return out


def _views(geo: Geometry, angles):
    """Views of the projections: a 1-D array of angles (circular orbit) or an n x 12 table of
    per-view source, detector centre and unit detector axes e_u, e_v (mm), as given."""
    a = np.asarray(angles, dtype=np.float64)
    if a.ndim == 2 and a.shape[1] == 12:
        return np.ascontiguousarray(a)
    if a.ndim != 1:
        raise ValueError("angles must be a 1-D array of angles or an n x 12 table of views")
    return circular_views(geo, a)


def set_threads(n: int):
    load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(load().orc_get_threads())


def ray_endpoints(geo: Geometry, theta, a: float, b: float):
    """Source and pixel centre of pixel (a, b) in one view (an angle, or a 12-vector view)."""
    v = np.asarray(theta, dtype=np.float64)
    view = _views(geo, v.reshape(1, 12) if v.size == 12 else v.reshape(1))[0].copy()
    S = np.zeros(3)
    P = np.zeros(3)
    load().orc_ray_endpoints(C.byref(geo.c()), _pd(view), float(a), float(b), _pd(S), _pd(P))
    return S, P


def siddon_ray(geo: Geometry, S, P, vol):
    vol = _f64(vol)
    S, P = _f64(S), _f64(P)
    ns = C.c_int64(0)
    v = load().orc_siddon_ray(C.byref(geo.c()), _pd(S), _pd(P), _pd(vol), C.byref(ns))
    return v, ns.value


def interp_ray(geo: Geometry, S, P, vol):
    vol = _f64(vol)
    S, P = _f64(S), _f64(P)
    ns = C.c_int64(0)
    v = load().orc_interp_ray(C.byref(geo.c()), _pd(S), _pd(P), _pd(vol), C.byref(ns))
    return v, ns.value


def siddon_fwd(geo: Geometry, angles, vol, return_counts=False):
    views = _views(geo, angles)
    vol = _f64(vol)
    out = np.zeros(geo.proj_shape(len(views)))
    cnt = np.zeros(len(views), dtype=np.int64)
    load().orc_siddon_fwd(C.byref(geo.c()), _pd(views), len(views), _pd(vol), _pd(out), _pi(cnt))
    return (out, cnt) if return_counts else out


def siddon_rays(geo: Geometry, angles, ray_idx, vol):
    """Selected rays.  A C-contiguous FP32 volume is read in place (widened per element), so
    volumes too large to copy to FP64 can be sampled."""
    views = _views(geo, angles)
    idx = np.ascontiguousarray(ray_idx, dtype=np.int64)
    out = np.zeros(len(idx))
    if vol.dtype == np.float32 and vol.flags["C_CONTIGUOUS"]:
        load().orc_siddon_rays_f32(C.byref(geo.c()), _pd(views), _pi(idx), len(idx),
                                   vol.ctypes.data_as(C.POINTER(C.c_float)), _pd(out))
        return out
    vol = _f64(vol)
    load().orc_siddon_rays(C.byref(geo.c()), _pd(views), _pi(idx), len(idx), _pd(vol), _pd(out))
    return out


def siddon_segments(geo: Geometry, angles, ray_idx):
    """Number of Siddon pieces of selected rays (flat indices as siddon_rays)."""
    views = _views(geo, angles)
    idx = np.ascontiguousarray(ray_idx, dtype=np.int64)
    out = np.zeros(len(idx), dtype=np.int64)
    load().orc_siddon_segments(C.byref(geo.c()), _pd(views), _pi(idx), len(idx), _pi(out))
    return out


def siddon_adj(geo: Geometry, angles, proj):
    views, proj = _views(geo, angles), _f64(proj)
    out = np.zeros(geo.vol_shape)
    load().orc_siddon_adj(C.byref(geo.c()), _pd(views), len(views), _pd(proj), _pd(out))
    return out


def siddon_adj_voxels(geo: Geometry, angles, proj, vox_idx):
    """Selected voxels.  A C-contiguous FP32 projection array is read in place."""
    views = _views(geo, angles)
    idx = np.ascontiguousarray(vox_idx, dtype=np.int64)
    out = np.zeros(len(idx))
    if proj.dtype == np.float32 and proj.flags["C_CONTIGUOUS"]:
        load().orc_siddon_adj_voxels_f32(C.byref(geo.c()), _pd(views), len(views),
                                         proj.ctypes.data_as(C.POINTER(C.c_float)), _pi(idx), len(idx),
                                         _pd(out))
        return out
    proj = _f64(proj)
    load().orc_siddon_adj_voxels(C.byref(geo.c()), _pd(views), len(views), _pd(proj), _pi(idx),
                                 len(idx), _pd(out))
    return out


def interp_fwd(geo: Geometry, angles, vol, return_counts=False):
    views, vol = _views(geo, angles), _f64(vol)
    out = np.zeros(geo.proj_shape(len(views)))
    cnt = np.zeros(len(views), dtype=np.int64)
    load().orc_interp_fwd(C.byref(geo.c()), _pd(views), len(views), _pd(vol), _pd(out), _pi(cnt))
    return (out, cnt) if return_counts else out


def interp_rays(geo: Geometry, angles, ray_idx, vol):
    views, vol = _views(geo, angles), _f64(vol)
    idx = np.ascontiguousarray(ray_idx, dtype=np.int64)
    out = np.zeros(len(idx))
    load().orc_interp_rays(C.byref(geo.c()), _pd(views), _pi(idx), len(idx), _pd(vol), _pd(out))
    return out


def bp(geo: Geometry, angles, proj, kind=W_FDK):
    views, proj = _views(geo, angles), _f64(proj)
    out = np.zeros(geo.vol_shape)
    load().orc_bp(C.byref(geo.c()), _pd(views), len(views), _pd(proj), int(kind), _pd(out))
    return out


def bp_voxels(geo: Geometry, angles, proj, vox_idx, kind=W_FDK):
    """Selected voxels.  A C-contiguous FP32 projection array is read in place."""
    views = _views(geo, angles)
    idx = np.ascontiguousarray(vox_idx, dtype=np.int64)
    out = np.zeros(len(idx))
    if proj.dtype == np.float32 and proj.flags["C_CONTIGUOUS"]:
        load().orc_bp_voxels_f32(C.byref(geo.c()), _pd(views), len(views),
                                 proj.ctypes.data_as(C.POINTER(C.c_float)), int(kind), _pi(idx), len(idx),
                                 _pd(out))
        return out
    proj = _f64(proj)
    load().orc_bp_voxels(C.byref(geo.c()), _pd(views), len(views), _pd(proj), int(kind), _pi(idx),
                         len(idx), _pd(out))
    return out


def bp_transpose(geo: Geometry, angles, vol, kind=W_FDK):
    views, vol = _views(geo, angles), _f64(vol)
    out = np.zeros(geo.proj_shape(len(views)))
    load().orc_bp_transpose(C.byref(geo.c()), _pd(views), len(views), _pd(vol), int(kind), _pd(out))
    return out
