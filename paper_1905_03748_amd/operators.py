"""Torch-facing wrappers over the C ABI: tensors in, tensors out, launched on torch's current
stream.  Only marshalling happens here (pointers, dtypes, shapes, stream handles); every step of
the computation runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A

_TORCH_DT = {torch.float32: A.CT_F32, torch.float16: A.CT_F16, torch.bfloat16: A.CT_BF16}
_PROJ = {"siddon": A.CT_SIDDON, "interp": A.CT_INTERP}
_BP = {"fdk": A.CT_BP_FDK, "pm": A.CT_BP_PSEUDO_MATCHED, "pseudo_matched": A.CT_BP_PSEUDO_MATCHED,
       "adjoint": A.CT_BP_ADJOINT, "matched": A.CT_BP_ADJOINT}


def ct_dtype(t: torch.dtype) -> int:
    try:
        return _TORCH_DT[t]
    except KeyError:
        raise TypeError(f"unsupported storage dtype {t}") from None


def _ct_dtype_any(t: torch.dtype) -> int:
    """ct_dtype, or CT_F64 for float64 (ct_dot and ct_convert only)."""
    return A.CT_F64 if t == torch.float64 else ct_dtype(t)


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev(t: torch.Tensor, shape, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape) and t.numel() != int(np.prod(shape)):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _host(t: torch.Tensor, shape, name):
    """Pointer of a host tensor that must hold exactly `shape` elements of a storage dtype: the
    library reads and writes through the raw pointer, so a short buffer would be overrun."""
    if t.device.type != "cpu":
        raise ValueError(f"{name} must be a host tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype not in _TORCH_DT:
        raise ValueError(f"{name} has unsupported dtype {t.dtype}")
    return t.data_ptr()


def _check_workspace(ws: torch.Tensor, need: int):
    if not ws.is_cuda or not ws.is_contiguous() or ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace must be a contiguous device tensor of at least {need} bytes")


class Plan:
    """A validated geometry and angle set (``ct_plan``).

    geometry: dict with DSO, DSD, nVoxel (Nx,Ny,Nz), dVoxel, offOrigin, nDetector (Nu,Nv),
    dDetector, offDetector, accuracy.  Volumes are [Nz, Ny, Nx]; projections [n_angles, Nv, Nu].
    angles: the angles of a circular orbit, or an n x 12 array of views (per projection the
    source, detector centre and unit detector axes e_u, e_v, mm; ``ct_plan_create_views``), for
    C-arm and helical scans.
    """

    def __init__(self, geometry: dict, angles):
        self.geometry = dict(geometry)
        self.cgeom = A.make_geometry(geometry)
        self.angles = np.ascontiguousarray(angles, dtype=np.float64)
        if self.angles.ndim == 2:
            if self.angles.shape[1] != 12:
                raise ValueError("views must be an n x 12 array")
            self.views = True
            self.handle = A.ct_plan_create_views(self.cgeom, self.angles.tolist())
        elif self.angles.ndim == 1:
            self.views = False
            self.handle = A.ct_plan_create(self.cgeom, self.angles)
        else:
            raise ValueError("angles must be 1-D (circular orbit) or n x 12 (views)")
        nx, ny, nz = (int(v) for v in geometry["nVoxel"])
        nu, nv = (int(v) for v in geometry["nDetector"])
        self.vol_shape = (nz, ny, nx)
        self.n_angles = len(self.angles)
        self.proj_shape = (self.n_angles, nv, nu)

    def close(self):
        if getattr(self, "handle", None):
            A.ct_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- resident operators ---------------------------------------------------------------------
    def forward(self, vol: torch.Tensor, projector="siddon", out: torch.Tensor | None = None, out_dtype=None,
                accumulate=False, angle_begin=0, angle_end=None, stream=None) -> torch.Tensor:
        angle_end = self.n_angles if angle_end is None else angle_end
        shape = (angle_end - angle_begin,) + self.proj_shape[1:]
        if out is None:
            out = torch.empty(shape, dtype=out_dtype or vol.dtype, device=vol.device)
        A.ct_forward(self.handle, _PROJ[projector], _dev(vol, self.vol_shape, "vol"), ct_dtype(vol.dtype),
                     _dev(out, shape, "proj"), ct_dtype(out.dtype), accumulate, angle_begin, angle_end,
                     _stream(stream))
        return out

    def backproject(self, proj: torch.Tensor, kind="fdk", out: torch.Tensor | None = None, out_dtype=None,
                    accumulate=False, angle_begin=0, angle_end=None, stream=None) -> torch.Tensor:
        angle_end = self.n_angles if angle_end is None else angle_end
        shape = (angle_end - angle_begin,) + self.proj_shape[1:]
        if out is None:
            out = torch.empty(self.vol_shape, dtype=out_dtype or proj.dtype, device=proj.device)
        A.ct_backproject(self.handle, _BP[kind], _dev(proj, shape, "proj"), ct_dtype(proj.dtype),
                         _dev(out, self.vol_shape, "vol"), ct_dtype(out.dtype), accumulate, angle_begin, angle_end,
                         _stream(stream))
        return out

    # -- out-of-core operators (host tensors) ---------------------------------------------------
    def forward_host(self, vol: torch.Tensor, out: torch.Tensor, projector="siddon", cap_bytes=32 << 30) -> dict:
        pv, po = _host(vol, self.vol_shape, "vol"), _host(out, self.proj_shape, "out")
        s = A.ct_forward_host(self.handle, _PROJ[projector], pv, ct_dtype(vol.dtype), po, ct_dtype(out.dtype),
                              cap_bytes)
        return s.as_dict()

    def backproject_host(self, proj: torch.Tensor, out: torch.Tensor, kind="fdk", cap_bytes=32 << 30) -> dict:
        pp, po = _host(proj, self.proj_shape, "proj"), _host(out, self.vol_shape, "out")
        s = A.ct_backproject_host(self.handle, _BP[kind], pp, ct_dtype(proj.dtype), po, ct_dtype(out.dtype),
                                  cap_bytes)
        return s.as_dict()

    def fdk_host(self, proj: torch.Tensor, out: torch.Tensor, cap_bytes=32 << 30) -> dict:
        """Out-of-core FDK reconstruction of host projections into the host volume `out`."""
        pp, po = _host(proj, self.proj_shape, "proj"), _host(out, self.vol_shape, "out")
        s = A.ct_fdk_host(self.handle, pp, ct_dtype(proj.dtype), po, ct_dtype(out.dtype), cap_bytes)
        return s.as_dict()

    def ooc_plan(self, direction=0, projector="siddon", vol_dtype=torch.float32, proj_dtype=torch.float32,
                 cap_bytes=32 << 30) -> dict:
        return A.ct_ooc_plan(self.handle, direction, _PROJ[projector], ct_dtype(vol_dtype), ct_dtype(proj_dtype),
                             cap_bytes).as_dict()

    # -- algorithms -----------------------------------------------------------------------------
    def cgls_workspace_bytes(self, vol_dtype=torch.float32, proj_dtype=torch.float32) -> int:
        return A.ct_cgls_workspace_bytes(self.handle, ct_dtype(vol_dtype), ct_dtype(proj_dtype))

    def cgls(self, b: torch.Tensor, niter: int, x: torch.Tensor | None = None, vol_dtype=None,
             resid: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None):
        """Runs CGLS in place on x (zeros if None); returns (x, resid) with resid a device FP64
        tensor of niter+1 residual norms."""
        if x is None:
            x = torch.zeros(self.vol_shape, dtype=vol_dtype or b.dtype, device=b.device)
        if workspace is not None:
            _check_workspace(workspace, self.cgls_workspace_bytes(x.dtype, b.dtype))
        if resid is None:
            resid = torch.empty(niter + 1, dtype=torch.float64, device=b.device)
        A.ct_cgls(self.handle, _dev(b, self.proj_shape, "b"), ct_dtype(b.dtype), _dev(x, self.vol_shape, "x"),
                  ct_dtype(x.dtype), niter, resid.data_ptr(), workspace.data_ptr() if workspace is not None else 0,
                  _stream(stream))
        return x, resid

    def cgls_host_workspace_bytes(self) -> int:
        return A.ct_cgls_host_workspace_bytes(self.handle)

    def cgls_host(self, b: torch.Tensor, niter: int, x: torch.Tensor | None = None, cap_bytes=32 << 30,
                  workspace: torch.Tensor | None = None):
        """Out-of-core CGLS on FP32 host tensors, in place on x (zeros if None); returns
        (x, resid, stats) with resid a NumPy array of niter+1 residual norms."""
        for t, name in ((b, "b"),) + (((x, "x"),) if x is not None else ()):
            if t.device.type != "cpu" or not t.is_contiguous() or t.dtype != torch.float32:
                raise ValueError(f"{name} must be a contiguous FP32 host tensor")
        if tuple(b.shape) != self.proj_shape:
            raise ValueError(f"b has shape {tuple(b.shape)}, expected {self.proj_shape}")
        if x is None:
            x = torch.zeros(self.vol_shape, dtype=torch.float32)
        elif tuple(x.shape) != self.vol_shape:
            raise ValueError(f"x has shape {tuple(x.shape)}, expected {self.vol_shape}")
        need = self.cgls_host_workspace_bytes()
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8)
        if workspace.device.type != "cpu" or workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace must be host memory of at least {need} bytes")
        resid = np.zeros(niter + 1, dtype=np.float64)
        st = A.ct_cgls_host(self.handle, b.data_ptr(), x.data_ptr(), niter, resid.ctypes.data, workspace.data_ptr(),
                            cap_bytes)
        return x, resid, st.as_dict()

    def sart_workspace_bytes(self, block=1) -> int:
        return A.ct_sart_workspace_bytes(self.handle, block)

    def sart(self, b: torch.Tensor, niter: int, x: torch.Tensor | None = None, lam=1.0, block=1, workspace=None,
             stream=None):
        """OS-SART in place on x (zeros if None): subsets of `block` consecutive angles, one update
        each (block = 1 is SART).  b and x may be stored in FP32, FP16 or BF16."""
        if x is None:
            x = torch.zeros(self.vol_shape, dtype=torch.float32, device=b.device)
        if workspace is not None:
            _check_workspace(workspace, self.sart_workspace_bytes(block))
        A.ct_sart(self.handle, _dev(b, self.proj_shape, "b"), ct_dtype(b.dtype), _dev(x, self.vol_shape, "x"),
                  ct_dtype(x.dtype), niter, lam, block, workspace.data_ptr() if workspace is not None else 0,
                  _stream(stream))
        return x

    def fdk_filter(self, proj: torch.Tensor, out: torch.Tensor | None = None, angle_begin=0, angle_end=None,
                   stream=None) -> torch.Tensor:
        """Cosine-weighted, ramp-filtered FP32 projections of the angles [angle_begin, angle_end)."""
        angle_end = self.n_angles if angle_end is None else angle_end
        shape = (angle_end - angle_begin,) + self.proj_shape[1:]
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=proj.device)
        if out.dtype != torch.float32:
            raise TypeError("filtered projections are FP32")
        A.ct_fdk_filter(self.handle, _dev(proj, shape, "proj"), ct_dtype(proj.dtype), _dev(out, shape, "q"),
                        angle_begin, angle_end, _stream(stream))
        return out

    def fdk_workspace_bytes(self) -> int:
        return A.ct_fdk_workspace_bytes(self.handle)

    def fdk(self, proj: torch.Tensor, out: torch.Tensor | None = None, out_dtype=None, workspace=None,
            stream=None) -> torch.Tensor:
        """FDK reconstruction of a full circular scan (filter, then FDK-weighted backprojection)."""
        if out is None:
            out = torch.empty(self.vol_shape, dtype=out_dtype or torch.float32, device=proj.device)
        if workspace is not None:
            _check_workspace(workspace, self.fdk_workspace_bytes())
        A.ct_fdk(self.handle, _dev(proj, self.proj_shape, "proj"), ct_dtype(proj.dtype),
                 _dev(out, self.vol_shape, "vol"), ct_dtype(out.dtype),
                 workspace.data_ptr() if workspace is not None else 0, _stream(stream))
        return out


def tv_steps(geometry: dict, x: torch.Tensor, nsteps: int, lam: float, eps: float = 1e-8, workspace=None,
             stream=None) -> torch.Tensor:
    """TV steepest descent in place on the device volume x (FP32, FP16 or BF16 storage)."""
    g = A.make_geometry(geometry)
    nx, ny, nz = (int(v) for v in geometry["nVoxel"])
    dt = ct_dtype(x.dtype)
    if workspace is not None:
        _check_workspace(workspace, tv_workspace_bytes(geometry, x.dtype))
    A.ct_tv_steps(g, _dev(x, (nz, ny, nx), "x"), dt, nsteps, lam, eps,
                  workspace.data_ptr() if workspace is not None else 0, _stream(stream))
    return x


def tv_steps_host(geometry: dict, x: torch.Tensor, nsteps: int, lam: float, eps: float = 1e-8,
                  cap_bytes=32 << 30, halo_depth=0) -> dict:
    """TV steepest descent in place on the FP32 host volume x, under a device memory cap:
    exact (halo_depth 0) or split with halos halo_depth deep and per-slab norm estimates."""
    nx, ny, nz = (int(v) for v in geometry["nVoxel"])
    if x.device.type != "cpu" or not x.is_contiguous() or x.dtype != torch.float32 or tuple(x.shape) != (nz, ny, nx):
        raise ValueError(f"x must be a contiguous FP32 host tensor of shape {(nz, ny, nx)}")
    return A.ct_tv_steps_host(A.make_geometry(geometry), x.data_ptr(), nsteps, lam, eps, halo_depth,
                              cap_bytes).as_dict()


def rof(geometry: dict, x: torch.Tensor, niter: int, lam: float, tau: float = 1.0 / 12.0, workspace=None,
        stream=None) -> torch.Tensor:
    """ROF denoising in place on the FP32 device volume x (Chambolle's projection, niter iterations)."""
    nx, ny, nz = (int(v) for v in geometry["nVoxel"])
    if x.dtype != torch.float32:
        raise TypeError("rof works on FP32 volumes")
    if workspace is not None:
        _check_workspace(workspace, rof_workspace_bytes(geometry))
    A.ct_rof(A.make_geometry(geometry), _dev(x, (nz, ny, nx), "x"), niter, lam, tau,
             workspace.data_ptr() if workspace is not None else 0, _stream(stream))
    return x


def rof_host(geometry: dict, x: torch.Tensor, niter: int, lam: float, tau: float = 1.0 / 12.0, halo_depth: int = 8,
             cap_bytes=32 << 30, workspace: torch.Tensor | None = None) -> dict:
    """ROF denoising in place on the FP32 host volume x under a device memory cap (slabs with halos
    halo_depth deep, the dual field in a host workspace of three volumes, allocated if None)."""
    nx, ny, nz = (int(v) for v in geometry["nVoxel"])
    if x.device.type != "cpu" or not x.is_contiguous() or x.dtype != torch.float32 or tuple(x.shape) != (nz, ny, nx):
        raise ValueError(f"x must be a contiguous FP32 host tensor of shape {(nz, ny, nx)}")
    g = A.make_geometry(geometry)
    need = A.ct_rof_host_workspace_bytes(g)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8)
    if workspace.device.type != "cpu" or not workspace.is_contiguous() or workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace must be a contiguous host tensor of at least {need} bytes")
    return A.ct_rof_host(g, x.data_ptr(), niter, lam, tau, halo_depth, workspace.data_ptr(), cap_bytes).as_dict()


def rof_workspace_bytes(geometry: dict) -> int:
    return A.ct_rof_workspace_bytes(A.make_geometry(geometry))


def tv_workspace_bytes(geometry: dict, dtype=torch.float32) -> int:
    return A.ct_tv_workspace_bytes(A.make_geometry(geometry), ct_dtype(dtype))


def dot(a: torch.Tensor, b: torch.Tensor, stream=None) -> torch.Tensor:
    if a.numel() != b.numel() or a.dtype != b.dtype:
        raise ValueError("dot needs two tensors of the same size and dtype")
    _dev(a, a.shape, "a")
    _dev(b, b.shape, "b")
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    A.ct_dot(a.data_ptr(), b.data_ptr(), _ct_dtype_any(a.dtype), a.numel(), out.data_ptr(), _stream(stream))
    return out


def convert(src: torch.Tensor, dtype: torch.dtype, stream=None) -> torch.Tensor:
    out = torch.empty(src.shape, dtype=dtype, device=src.device)
    _dev(src, src.shape, "src")
    A.ct_convert(src.data_ptr(), _ct_dtype_any(src.dtype), out.data_ptr(), _ct_dtype_any(dtype), src.numel(),
                 _stream(stream))
    return out
