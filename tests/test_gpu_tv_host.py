"""TV steepest descent out of core (ct_tv_steps_host): the image in host memory, slabs of axial
slices with one halo slice on either side under a device cap.  Against the FP64 oracle and the
resident ct_tv_steps, for slab heights from the whole volume down to one slice."""
import numpy as np
import pytest
import torch

from _helpers import rel_l2, say
from paper_1905_03748_amd.operators import tv_steps, tv_steps_host

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FIXED = (64 << 20) + 8192 + 256   # reserve, dot partials, scalars


def _geo(nx, ny, nz):
    return dict(DSO=1000.0, DSD=1500.0, nVoxel=(nx, ny, nz), dVoxel=(1.0, 1.0, 1.0), offOrigin=(0, 0, 0),
                nDetector=(8, 8), dDetector=(1.0, 1.0), offDetector=(0, 0), accuracy=0.5)


def _cap(nx, ny, h):
    # the slab with two halo slices, its gradient and one saved slice: 2 h + 3 slices
    return FIXED + (2 * h + 3) * nx * ny * 4


@pytest.mark.parametrize("h", [29, 10, 5, 1])
def test_tv_host_matches_oracle_and_resident(orc, h):
    nz, ny, nx = 29, 17, 31
    rng = np.random.default_rng(81)
    x0 = (rng.uniform(0, 1, (nz, ny, nx)) > 0.7).astype(np.float32) * 0.8 + \
        0.05 * rng.standard_normal((nz, ny, nx)).astype(np.float32)
    geo = _geo(nx, ny, nz)
    say(f"[tv host] slab height {h}")
    x = torch.from_numpy(x0.copy())
    st = tv_steps_host(geo, x, 5, 0.01, cap_bytes=_cap(nx, ny, h))
    nsp = -(-nz // h)
    assert st["n_slabs"] == nsp and st["slab_slices"] == -(-nz // nsp), st
    e = rel_l2(x.numpy(), orc.tv_steps(x0.astype(np.float64), 5, 0.01))
    say(f"   rel L2 vs oracle {e:.3e}")
    assert e <= 1e-5
    xd = torch.from_numpy(x0).to(DEV)
    tv_steps(geo, xd, 5, 0.01)
    xd = xd.cpu()
    if nsp == 1:
        assert torch.equal(x, xd)   # the same kernels and the same FP64 sums
    else:
        assert rel_l2(x.numpy(), xd.numpy()) <= 1e-6


def test_tv_host_edge_cases():
    nz, ny, nx = 6, 5, 7
    geo = _geo(nx, ny, nz)
    x = torch.full((nz, ny, nx), 0.3)
    tv_steps_host(geo, x, 3, 0.01, cap_bytes=_cap(nx, ny, 2))
    assert float((x - 0.3).abs().max()) == 0.0   # a constant image has no gradient
    x = torch.rand((nz, ny, nx), generator=torch.Generator().manual_seed(5))
    x0 = x.clone()
    tv_steps_host(geo, x, 0, 0.01, cap_bytes=_cap(nx, ny, 2))
    assert torch.equal(x, x0)
    from paper_1905_03748_amd._abi import CT_ERR_CAP, CtError
    with pytest.raises(CtError) as e:
        tv_steps_host(geo, x, 1, 0.01, cap_bytes=FIXED + 4 * nx * ny * 4)
    assert e.value.status == CT_ERR_CAP
    with pytest.raises(ValueError):
        tv_steps_host(geo, x.double(), 1, 0.01)


@pytest.mark.parametrize("h,d", [(29, 3), (10, 3), (5, 2), (1, 4), (3, 10)])
def test_tv_host_halo_split_matches_oracle(orc, h, d):
    """The splitting of Section 2.3 (halos d deep, d steps per exchange, per-slab norm estimates):
    against the oracle's form of the same scheme with the slab height the planner chose."""
    nz, ny, nx = 29, 17, 31
    rng = np.random.default_rng(82)
    x0 = (rng.uniform(0, 1, (nz, ny, nx)) > 0.7).astype(np.float32) * 0.8 + \
        0.05 * rng.standard_normal((nz, ny, nx)).astype(np.float32)
    say(f"[tv host halo] slab height {h}, depth {d}")
    x = torch.from_numpy(x0.copy())
    # the slab and its gradient with d halo slices each side, and d saved slices
    st = tv_steps_host(_geo(nx, ny, nz), x, 7, 0.01, cap_bytes=FIXED + (2 * h + 5 * d) * nx * ny * 4, halo_depth=d)
    assert st["n_slabs"] == -(-nz // h), st
    ref = orc.tv_steps_split(x0.astype(np.float64), 7, 0.01, st["slab_slices"], d, norm="split")
    e = rel_l2(x.numpy(), ref)
    say(f"   rel L2 vs oracle {e:.3e}")
    assert e <= 1e-5


@pytest.mark.parametrize("d", [0, 1, 3])
def test_tv_host_single_slice(orc, d):
    """A one-slice image: no halo on either side, in the exact form and the split form."""
    ny, nx = 19, 23
    x0 = np.random.default_rng(83).uniform(0, 1, (1, ny, nx)).astype(np.float32)
    x = torch.from_numpy(x0.copy())
    st = tv_steps_host(_geo(nx, ny, 1), x, 4, 0.01, cap_bytes=FIXED + (2 + 5 * max(d, 1)) * nx * ny * 4, halo_depth=d)
    assert st["n_slabs"] == 1
    assert rel_l2(x.numpy(), orc.tv_steps(x0.astype(np.float64), 4, 0.01)) <= 1e-5
