"""Out-of-core operators at the full size of the splitting workload: a 3072^3 FP32 volume and 3072
projections of 3072^2 (108 GiB each, in pageable host memory, which the streamer stages through its
own pinned ring) under a 32 GiB device cap.  One Siddon A x, one FDK A^T y and one exact-adjoint A^T y
(Algorithms 1 and 2), each checked on seeded samples of its output against the oracle, which reads
the FP32 host arrays in place.

It needs about 220 GiB of host memory and several minutes, so it runs only when CT_FULL_OOC=1."""
import os

import numpy as np
import pytest
import torch

from _helpers import TOL_BP, TOL_PROJ, rel_l2, say
from paper_1905_03748_amd import inputs
from paper_1905_03748_amd.operators import Plan

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("CT_FULL_OOC") != "1",
                                 reason="set CT_FULL_OOC=1 (needs ~220 GiB of host memory, minutes)")]
DEV = "cuda:0"
CAP = 32 << 30


def test_full_size_out_of_core(orc):
    w = inputs.workload("ooc")
    plan = Plan(w.geometry_dict(), w.angles)
    og = orc.Geometry.from_dict(w.geometry_dict())
    vol = np.empty(plan.vol_shape, dtype=np.float32)
    proj = np.empty(plan.proj_shape, dtype=np.float32)
    say("[ooc full] phantom slab by slab")
    try:
        ells = inputs.ellipsoids(w)
        nz = w.nvox[2]
        for z0 in range(0, nz, 256):
            h = min(256, nz - z0)
            ws = inputs.Workload("slab", (w.nvox[0], w.nvox[1], h), w.dvox, w.ndet, w.ddet, 1, 0, 0,
                                 off_origin=(0.0, 0.0, (z0 + h / 2.0 - nz / 2.0) * w.dvox[2]))
            torch.from_numpy(vol[z0:z0 + h]).copy_(inputs.voxelize_torch(ws, ells, device=DEV))
            torch.cuda.synchronize()
        vt, pt = torch.from_numpy(vol), torch.from_numpy(proj)

        say("[ooc full] Siddon forward under the cap")
        st = plan.forward_host(vt, pt, "siddon", cap_bytes=CAP)
        say(f"[ooc full] forward: {st}")
        assert st["n_slabs"] > 1
        rays = inputs.sample_indices(proj.size, 48, 301)
        ref = orc.siddon_rays(og, w.angles, rays, vol.reshape(-1))
        e = rel_l2(proj.reshape(-1)[rays].astype(np.float64), ref)
        say(f"[ooc full] forward vs oracle on 48 rays: rel L2 {e:.3e}")
        assert e <= TOL_PROJ

        say("[ooc full] FDK backprojection under the cap")
        st = plan.backproject_host(pt, vt, "fdk", cap_bytes=CAP)
        say(f"[ooc full] backprojection: {st}")
        assert st["n_slabs"] > 1
        vox = inputs.sample_indices(vol.size, 48, 302)
        ref = orc.bp_voxels(og, w.angles, proj.reshape(-1), vox, orc.W_FDK)
        e = rel_l2(vol.reshape(-1)[vox].astype(np.float64), ref)
        say(f"[ooc full] backprojection vs oracle on 48 voxels: rel L2 {e:.3e}")
        assert e <= TOL_BP

        say("[ooc full] exact-adjoint backprojection under the cap")
        st = plan.backproject_host(pt, vt, "adjoint", cap_bytes=CAP)
        say(f"[ooc full] exact adjoint: {st}")
        assert st["n_slabs"] > 1
        vox = inputs.sample_indices(vol.size, 32, 303)
        ref = orc.siddon_adj_voxels(og, w.angles, proj, vox)
        e = rel_l2(vol.reshape(-1)[vox].astype(np.float64), ref)
        say(f"[ooc full] exact adjoint vs oracle on 32 voxels: rel L2 {e:.3e}")
        assert e <= TOL_BP
    finally:
        del vol, proj
