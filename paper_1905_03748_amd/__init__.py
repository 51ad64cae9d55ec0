"""MI355X-native cone-beam CT operators (Biguri et al., TIGRE multi-GPU splitting paper):
Siddon and interpolated forward projection, FDK / pseudo-matched / exact-adjoint backprojection,
out-of-core slab/chunk streaming, CGLS, SART and TV on the device, behind the C ABI in
``include/ct.h`` (``libct.so``, HIP for gfx950).

Submodules: ``_abi`` (ctypes binding, C names), ``operators`` (torch tensors in/out),
``autograd`` (differentiable projector), ``serve`` (continuous-batching reconstruction server),
``inputs`` (seeded synthetic phantoms; no projector arithmetic), ``build`` (hipcc build).
"""
from . import _abi
from ._abi import (CT_BP_ADJOINT, CT_BP_FDK, CT_BP_PSEUDO_MATCHED, CT_BF16, CT_F16, CT_F32, CT_INTERP,
                   CT_SIDDON, CtError, ct_backproject, ct_backproject_host, ct_cgls, ct_cgls_workspace_bytes,
                   ct_convert, ct_dot, ct_forward, ct_forward_host, ct_last_error, ct_ooc_plan, ct_plan_create,
                   ct_plan_destroy, ct_plan_info, ct_sart, ct_sart_workspace_bytes, ct_tv_steps,
                   ct_tv_workspace_bytes, ct_version, make_geometry)


def __getattr__(name):
    # torch-dependent pieces load on first use
    if name in ("Plan", "tv_steps", "tv_workspace_bytes", "dot", "convert"):
        from . import operators
        return getattr(operators, name)
    if name in ("project", "SiddonProjection"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
