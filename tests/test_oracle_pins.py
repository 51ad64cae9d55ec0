"""Pins of the CPU FP64 oracle against things other than itself: hand-derived closed forms,
analytic chords, brute-force ray marching, library interpolation, dense linear algebra and
invariants.  CPU only.

Section references are to the paper (Biguri et al., TIGRE multi-GPU): Section 2 Eq. (1) defines A
as ray/element intersection lengths; Section 2.1 the ray-driven projectors (Siddon; interpolated);
Section 2.2 the voxel-driven backprojectors (FDK and pseudo-matched weights); Section 2.3 TV
steepest descent; Section 3.2 CGLS and OS-SART.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1905_03748_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _geo(orc, **kw):
    d = dict(DSO=1000.0, DSD=1500.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), offOrigin=(0.0, 0.0, 0.0),
             nDetector=(8, 8), dDetector=(1.6, 1.6), offDetector=(0.0, 0.0), accuracy=0.5)
    d.update(kw)
    return orc.Geometry.from_dict(d)


def _box_chord_faces(S, P, lo, hi):
    """Length of segment S->P inside the box [lo,hi], by intersecting the line with the six face
    rectangles (a different construction from slab clipping)."""
    S = np.asarray(S, float)
    P = np.asarray(P, float)
    D = P - S
    pts = []
    for ax in range(3):
        if D[ax] == 0:
            continue
        for plane in (lo[ax], hi[ax]):
            t = (plane - S[ax]) / D[ax]
            if not (0.0 <= t <= 1.0):
                continue
            X = S + t * D
            o = [a for a in range(3) if a != ax]
            if all(lo[a] - 1e-12 <= X[a] <= hi[a] + 1e-12 for a in o):
                pts.append(X)
    inside = [np.all((S >= lo) & (S <= hi)), np.all((P >= lo) & (P <= hi))]
    if inside[0]:
        pts.append(S)
    if inside[1]:
        pts.append(P)
    if len(pts) < 2:
        return 0.0
    best = 0.0
    for i in range(len(pts)):
        for j in range(i + 1, len(pts)):
            best = max(best, float(np.linalg.norm(pts[i] - pts[j])))
    return best


# --------------------------------------------------------------------------------------------
# hand-derived closed forms (tests/golden)

def test_golden_closed_forms(orc):
    gold = json.load(open(GOLD))
    geo = orc.Geometry.from_dict(gold["geometry"])
    nx, ny, nz = geo.nVoxel
    vol = np.broadcast_to(np.arange(nx, dtype=float) + 1.0, (nz, ny, nx)).copy()
    for case in gold["cases"]:
        if case["op"] == "siddon":
            S, P = orc.ray_endpoints(geo, case["theta"], *case["pixel"])
            got, _ = orc.siddon_ray(geo, S, P, vol)
        else:
            na = case["n_angles"]
            angles = inputs.uniform_angles(na)
            proj = np.zeros((na, 5, 5))
            if case["projection"].startswith("constant"):
                proj[:] = float(case["projection"].split()[1])
            else:
                proj[0, 2, 4] = 1.0
            kind = orc.W_FDK if case["op"] == "bp_fdk" else orc.W_PM
            i, j, k = case["voxel"]
            got = orc.bp_voxels(geo, angles, proj, [(k * ny + j) * nx + i], kind)[0]
        assert abs(got - case["expected"]) <= case["rtol"] * abs(case["expected"]), case["name"]


# --------------------------------------------------------------------------------------------
# C1 Siddon: P1 box chord, P2 single voxel, P3 ellipsoid convergence, P4 brute force,
# P5 adjoint identity, P6 symmetries

def test_P1_ones_volume_gives_box_chord(orc):
    rng = np.random.default_rng(11)
    for trial in range(4):
        geo = _geo(orc, nVoxel=tuple(rng.integers(5, 13, 3)), dVoxel=tuple(rng.uniform(0.7, 1.6, 3)),
                   offOrigin=tuple(rng.uniform(-2, 2, 3)), nDetector=(9, 7), dDetector=(2.3, 2.9),
                   offDetector=tuple(rng.uniform(-3, 3, 2)))
        vol = np.ones(geo.vol_shape)
        lo = [o - n * d / 2 for n, d, o in zip(geo.nVoxel, geo.dVoxel, geo.offOrigin)]
        hi = [o + n * d / 2 for n, d, o in zip(geo.nVoxel, geo.dVoxel, geo.offOrigin)]
        for th in rng.uniform(0, 2 * np.pi, 3):
            for a in range(9):
                for b in range(7):
                    S, P = orc.ray_endpoints(geo, th, a, b)
                    got, _ = orc.siddon_ray(geo, S, P, vol)
                    ref = _box_chord_faces(S, P, lo, hi)
                    assert abs(got - ref) <= 1e-12 * max(ref, 1.0)


def test_P2_single_voxel_gives_its_chord(orc):
    rng = np.random.default_rng(12)
    geo = _geo(orc, nVoxel=(6, 7, 5), dVoxel=(1.1, 0.9, 1.3), offOrigin=(0.3, -0.2, 0.4),
               nDetector=(24, 20), dDetector=(0.6, 0.7))
    nx, ny, nz = geo.nVoxel
    hits = 0
    for _ in range(6):
        i, j, k = rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)
        vol = np.zeros(geo.vol_shape)
        vol[k, j, i] = 1.0
        c = [geo.offOrigin[a] + ((i, j, k)[a] - (geo.nVoxel[a] - 1) / 2) * geo.dVoxel[a] for a in range(3)]
        lo = [c[a] - geo.dVoxel[a] / 2 for a in range(3)]
        hi = [c[a] + geo.dVoxel[a] / 2 for a in range(3)]
        th = rng.uniform(0, 2 * np.pi)
        for a in range(24):
            for b in range(20):
                S, P = orc.ray_endpoints(geo, th, a, b)
                got, _ = orc.siddon_ray(geo, S, P, vol)
                ref = _box_chord_faces(S, P, lo, hi)
                hits += ref > 0
                assert abs(got - ref) <= 1e-11
    assert hits > 20


def _ellipsoid_workload(n):
    return inputs.Workload("ell", (n, n, n), (64.0 / n,) * 3, (48, 48), (2.0, 2.0), 4, 1, 0)


@pytest.mark.slow
def test_P3_voxelised_ellipsoid_converges_to_analytic_chord(orc):
    ell = inputs.Ellipsoid(np.array([2.0, -3.0, 1.5]), np.array([20.0, 14.0, 10.0]), 0.7,
                           inputs._quat_to_rot(np.array([0.9, 0.2, -0.3, 0.25]) /
                                               np.linalg.norm([0.9, 0.2, -0.3, 0.25])))
    errs = []
    errs_ss = []
    for n in (32, 64, 128):
        w = _ellipsoid_workload(n)
        geo = orc.Geometry.from_dict(w.geometry_dict())
        vol = inputs.voxelize(w, [ell], dtype=np.float64)
        p = orc.siddon_fwd(geo, w.angles, vol)
        aa, bb = np.meshgrid(np.arange(48), np.arange(48))
        ref = np.stack([inputs.ellipsoid_line_integrals(*inputs.ray_endpoints(w, th, aa, bb), [ell])
                        for th in w.angles])
        errs.append(np.linalg.norm(p - ref) / np.linalg.norm(ref))
        if n == 64:
            vol4 = inputs.voxelize(w, [ell], dtype=np.float64, supersample=4)
            p4 = orc.siddon_fwd(geo, w.angles, vol4)
            errs_ss.append(np.linalg.norm(p4 - ref) / np.linalg.norm(ref))
    # O(h): roughly halves per halving of the voxel size
    assert errs[0] / errs[1] > 1.4 and errs[1] / errs[2] > 1.4, errs
    assert errs[2] < 0.04, errs
    assert errs_ss[0] < errs[1], (errs_ss, errs)


def test_P4_brute_force_ray_marching(orc):
    rng = np.random.default_rng(14)
    for n in (8, 13, 16):
        geo = _geo(orc, nVoxel=(n, n - 1, n + 2), dVoxel=(1.2, 0.8, 1.0), offOrigin=(0.5, -0.4, 0.2),
                   nDetector=(30, 30), dDetector=(0.9, 0.9))
        vol = rng.uniform(0, 1, geo.vol_shape)
        lo = np.array([o - k * d / 2 for k, d, o in zip(geo.nVoxel, geo.dVoxel, geo.offOrigin)])
        M = 1_000_000
        for _ in range(3):
            th = rng.uniform(0, 2 * np.pi)
            a, b = rng.integers(11, 19, 2)
            S, P = orc.ray_endpoints(geo, th, a, b)
            got, nseg = orc.siddon_ray(geo, S, P, vol)
            t = (np.arange(M) + 0.5) / M
            X = S[None, :] + t[:, None] * (P - S)[None, :]
            idx = np.floor((X - lo) / np.array(geo.dVoxel)).astype(np.int64)
            ok = np.all((idx >= 0) & (idx < np.array(geo.nVoxel)), axis=1)
            L = np.linalg.norm(P - S)
            ref = L / M * vol[idx[ok, 2], idx[ok, 1], idx[ok, 0]].sum()
            bound = (nseg + 2) * (L / M) * vol.max()
            assert nseg > 0
            assert abs(got - ref) <= bound


def test_P5_adjoint_dot_product_identity(orc):
    rng = np.random.default_rng(15)
    for n in (8, 17, 32):
        geo = _geo(orc, nVoxel=(n, n + 1, n - 1), dVoxel=tuple(rng.uniform(0.8, 1.3, 3)),
                   offOrigin=tuple(rng.uniform(-1, 1, 3)), nDetector=(n + 3, n - 2), dDetector=(1.5, 1.7),
                   offDetector=tuple(rng.uniform(-2, 2, 2)))
        angles = rng.uniform(0, 2 * np.pi, 7)
        x = rng.standard_normal(geo.vol_shape)
        y = rng.standard_normal(geo.proj_shape(7))
        lhs = float(np.sum(orc.siddon_fwd(geo, angles, x) * y))
        rhs = float(np.sum(x * orc.siddon_adj(geo, angles, y)))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        # the selected-voxel transpose agrees with the full scatter
        idx = inputs.sample_indices(x.size, 25, 3)
        full = orc.siddon_adj(geo, angles, y).ravel()[idx]
        part = orc.siddon_adj_voxels(geo, angles, y, idx)
        np.testing.assert_allclose(part, full, rtol=1e-11, atol=1e-11)


def test_P6_symmetries(orc):
    rng = np.random.default_rng(16)
    geo = _geo(orc, nVoxel=(12, 12, 10), nDetector=(20, 16), dDetector=(1.4, 1.3))
    v = rng.uniform(0, 1, geo.vol_shape)
    vz = v + v[::-1]                      # mirror-symmetric in z
    angles = rng.uniform(0, 2 * np.pi, 3)
    p = orc.siddon_fwd(geo, angles, vz)
    np.testing.assert_allclose(p, p[:, ::-1, :], rtol=1e-12, atol=1e-12 * np.abs(p).max())
    v4 = sum(np.rot90(v, k, axes=(1, 2)) for k in range(4))   # invariant under 90 deg about z
    th = np.array([0.3, 0.3 + np.pi / 2, 0.3 + np.pi, 0.3 + 1.5 * np.pi])
    p4 = orc.siddon_fwd(geo, th, v4)
    for k in range(1, 4):
        np.testing.assert_allclose(p4[k], p4[0], rtol=1e-11, atol=1e-11 * np.abs(p4).max())


# --------------------------------------------------------------------------------------------
# C2 interpolated projector: I1 convergence to the exact integral of the interpolant,
# I2 constant phantom along an axis, I3 close to Siddon (reported)

def _exact_interp_integral(geo, vol, S, P):
    """Exact line integral of the zero-padded trilinear interpolant: split the segment at every
    plane through voxel centres (the dual grid, where the interpolant is a cubic in t) and apply
    2-point Gauss-Legendre on each piece; the interpolant is evaluated with scipy."""
    from scipy.interpolate import RegularGridInterpolator
    n = np.array(geo.nVoxel)
    d = np.array(geo.dVoxel)
    o = np.array(geo.offOrigin)
    axes = [o[a] + (np.arange(-1, n[a] + 1) - (n[a] - 1) / 2) * d[a] for a in range(3)]
    pad = np.zeros(tuple(n[::-1] + 2))
    pad[1:-1, 1:-1, 1:-1] = vol
    f = RegularGridInterpolator((axes[2], axes[1], axes[0]), pad, method="linear", bounds_error=False,
                                fill_value=0.0)
    S = np.asarray(S, float)
    P = np.asarray(P, float)
    D = P - S
    ts = [0.0, 1.0]
    for a in range(3):
        if D[a] != 0:
            tt = (axes[a] - S[a]) / D[a]
            ts += list(tt[(tt > 0) & (tt < 1)])
    ts = np.unique(ts)
    g = 0.5 / math.sqrt(3.0)
    L = np.linalg.norm(D)
    tot = 0.0
    for t0, t1 in zip(ts[:-1], ts[1:]):
        tm, h = 0.5 * (t0 + t1), t1 - t0
        for s in (-g, g):
            X = S + (tm + s * h) * D
            tot += 0.5 * h * L * f(X[::-1][None, :])[0]
    return tot


def test_I1_lattice_converges_quadratically(orc):
    n = 10
    x = np.linspace(-1, 1, n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    vol = np.exp(-2.5 * (X ** 2 + 1.3 * Y ** 2 + 0.7 * Z ** 2))     # smooth phantom
    rng = np.random.default_rng(21)
    rays = [(rng.uniform(0, 2 * np.pi), *rng.uniform(4, 12, 2)) for _ in range(24)]
    rms = []
    for acc in (0.5, 0.25, 0.125):
        geo = _geo(orc, nVoxel=(n, n, n), nDetector=(16, 16), dDetector=(1.2, 1.2), accuracy=acc)
        e2, r2 = 0.0, 0.0
        for th, a, b in rays:
            S, P = orc.ray_endpoints(geo, th, a, b)
            got, _ = orc.interp_ray(geo, S, P, vol)
            ref = _exact_interp_integral(geo, vol, S, P)
            e2 += (got - ref) ** 2
            r2 += ref ** 2
        rms.append(math.sqrt(e2 / r2))
    # midpoint lattice on a piecewise-cubic interpolant: O(Delta^2) once averaged over rays
    assert rms[0] / rms[1] > 2.5 and rms[1] / rms[2] > 2.5, rms
    assert rms[0] < 1e-3, rms


def test_I2_constant_phantom_axis_parallel(orc):
    for acc in (0.5, 0.3, 0.125):
        geo = _geo(orc, nVoxel=(9, 6, 7), dVoxel=(1.1, 0.9, 1.2), offOrigin=(0.2, 0.1, -0.3), accuracy=acc)
        c = 0.7
        vol = np.full(geo.vol_shape, c)
        y0, z0 = 0.1 + 0.37, -0.3 + 0.21     # strictly between the first and last voxel centres
        S = np.array([-1000.0, y0, z0])
        P = np.array([600.0, y0, z0])
        got, ns = orc.interp_ray(geo, S, P, vol)
        ref = c * geo.nVoxel[0] * geo.dVoxel[0]
        assert abs(_exact_interp_integral(geo, vol, S, P) - ref) < 1e-12
        delta = acc * min(geo.dVoxel)
        kink_bound = 4 * (c / geo.dVoxel[0]) * delta ** 2 / 8
        assert abs(got - ref) <= kink_bound + 1e-12, (got, ref, kink_bound)


def test_I3_interpolated_close_to_siddon_reported(orc):
    w = inputs.workload("tiny")
    geo = orc.Geometry.from_dict(w.geometry_dict())
    vol = inputs.voxelize(w, dtype=np.float64)
    ang = w.angles[::8]
    ps = orc.siddon_fwd(geo, ang, vol)
    pi = orc.interp_fwd(geo, ang, vol)
    rel = np.linalg.norm(ps - pi) / np.linalg.norm(ps)
    print(f"interpolated vs Siddon relative L2 on tiny: {rel:.3e}")
    assert rel < 0.1


# --------------------------------------------------------------------------------------------
# C3/C4 voxel backprojectors: B1 constant projection, B2 impulse (golden), B3 transpose identity,
# M1 pseudo-matched weight against the Siddon column sums

def test_B1_constant_projection(orc):
    # odd grid: voxel (c,c,c) is the isocentre
    geo = _geo(orc, nVoxel=(9, 9, 9), dVoxel=(2.0, 2.0, 2.0), nDetector=(64, 64), dDetector=(1.6, 1.6))
    na = 64
    angles = inputs.uniform_angles(na)
    c = 1.7
    proj = np.full((na, 64, 64), c)
    vol = orc.bp(geo, angles, proj, orc.W_FDK)
    assert abs(vol[4, 4, 4] - c * na) <= 1e-12 * c * na
    # voxel at radius r in the mid-plane: sum of (DSO/(DSO - r cos t))^2 over uniform angles equals
    # (to machine precision for 64 angles) N * DSO^3 / (DSO^2 - r^2)^(3/2)
    for i in (0, 2, 7):
        r = abs((i - 4) * 2.0)
        ref = c * na * geo.DSO ** 3 / (geo.DSO ** 2 - r ** 2) ** 1.5
        assert abs(vol[4, 4, i] - ref) <= 1e-12 * ref


def test_B3_backprojector_is_transpose_of_splat(orc):
    rng = np.random.default_rng(33)
    geo = _geo(orc, nVoxel=(9, 10, 7), dVoxel=(1.1, 0.9, 1.4), offOrigin=(0.3, -0.6, 0.5), nDetector=(13, 11),
               dDetector=(1.3, 1.7), offDetector=(0.8, -1.1))
    angles = rng.uniform(0, 2 * np.pi, 6)
    x = rng.standard_normal(geo.vol_shape)
    y = rng.standard_normal(geo.proj_shape(6))
    for kind in (orc.W_FDK, orc.W_PM):
        lhs = float(np.sum(orc.bp_transpose(geo, angles, x, kind) * y))
        rhs = float(np.sum(x * orc.bp(geo, angles, y, kind)))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        idx = inputs.sample_indices(x.size, 30, 4)
        np.testing.assert_allclose(orc.bp_voxels(geo, angles, y, idx, kind), orc.bp(geo, angles, y, kind).ravel()[idx],
                                   rtol=1e-13, atol=1e-13)


def test_M1_pseudo_matched_weight_matches_siddon_column_sums(orc):
    # matched sampling: pixel size at the isocentre equals the voxel size (magnification 1.5)
    geo = _geo(orc, nVoxel=(32, 32, 32), dVoxel=(1.0, 1.0, 1.0), nDetector=(64, 64), dDetector=(1.5, 1.5))
    ratios = []
    for th in (0.0, 0.37, 1.1):
        ones_p = np.ones((1, 64, 64))
        col = orc.siddon_adj(geo, [th], ones_p)
        pm = orc.bp(geo, [th], ones_p, orc.W_PM)
        inner = (slice(8, 24),) * 3
        ratios.append(float(np.mean(col[inner] / pm[inner])))
    assert all(abs(r - 1.0) < 0.02 for r in ratios), ratios


def test_M2_pseudo_matched_gap_reported(orc):
    rng = np.random.default_rng(34)
    geo = _geo(orc, nVoxel=(16, 16, 16), nDetector=(24, 24), dDetector=(1.5, 1.5))
    angles = inputs.uniform_angles(16)
    x = rng.uniform(0, 1, geo.vol_shape)
    y = rng.uniform(0, 1, geo.proj_shape(16))
    ax = float(np.sum(orc.siddon_fwd(geo, angles, x) * y))
    for kind, name in ((orc.W_PM, "pseudo-matched"), (orc.W_FDK, "FDK")):
        gap = abs(ax - float(np.sum(x * orc.bp(geo, angles, y, kind)))) / abs(ax)
        print(f"{name} dot-product gap: {gap:.3e}")
    gap_pm = abs(ax - float(np.sum(x * orc.bp(geo, angles, y, orc.W_PM)))) / abs(ax)
    assert gap_pm < 0.05


# --------------------------------------------------------------------------------------------
# C6 CGLS against dense linear algebra

def _dense(orc, geo, angles):
    nvox = int(np.prod(geo.nVoxel))
    cols = []
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        cols.append(orc.siddon_fwd(geo, angles, e.reshape(geo.vol_shape)).ravel())
    return np.stack(cols, 1)


def test_Ca_cgls_equals_dense_cg_on_normal_equations(orc):
    geo = _geo(orc, nVoxel=(8, 8, 8), nDetector=(8, 8), dDetector=(1.6, 1.6))
    angles = inputs.uniform_angles(8)
    A = _dense(orc, geo, angles)
    rng = np.random.default_rng(41)
    b = A @ rng.uniform(0, 1, A.shape[1]) + 0.01 * rng.standard_normal(A.shape[0])
    Afn = lambda x: orc.siddon_fwd(geo, angles, x)
    Atfn = lambda y: orc.siddon_adj(geo, angles, y)
    # textbook CG on A^T A x = A^T b from x = 0
    M = A.T @ A
    rhs = A.T @ b
    x = np.zeros(A.shape[1])
    r = rhs.copy()
    p = r.copy()
    cg_iter = []
    for _ in range(6):
        Mp = M @ p
        al = (r @ r) / (p @ Mp)
        x = x + al * p
        rn = r - al * Mp
        p = rn + (rn @ rn) / (r @ r) * p
        r = rn
        cg_iter.append(x.copy())
    for k in (1, 3, 6):
        xk, res = orc.cgls(Afn, Atfn, b.reshape(geo.proj_shape(8)), k)
        ref = cg_iter[k - 1]
        assert np.linalg.norm(xk.ravel() - ref) <= 1e-9 * np.linalg.norm(ref)
        # the residual recurrence equals the explicit residual
        assert abs(res[-1] - np.linalg.norm(A @ xk.ravel() - b)) <= 1e-8 * res[0]
    # long run approaches the least-squares residual
    xk, res = orc.cgls(Afn, Atfn, b.reshape(geo.proj_shape(8)), 150)
    xls = np.linalg.lstsq(A, b, rcond=None)[0]
    r_ls = np.linalg.norm(A @ xls - b)
    assert np.linalg.norm(A @ xk.ravel() - b) <= r_ls * (1 + 1e-3) + 1e-9


def test_Cb_cgls_krylov_optimality_and_monotone(orc):
    geo = _geo(orc, nVoxel=(8, 8, 8), nDetector=(8, 8), dDetector=(1.6, 1.6))
    angles = inputs.uniform_angles(8)
    A = _dense(orc, geo, angles)
    rng = np.random.default_rng(42)
    b = rng.uniform(0, 5, A.shape[0])
    Afn = lambda x: orc.siddon_fwd(geo, angles, x)
    Atfn = lambda y: orc.siddon_adj(geo, angles, y)
    M = A.T @ A
    v = A.T @ b
    K = []
    for k in range(1, 6):
        K.append(v / np.linalg.norm(v))
        Q, _ = np.linalg.qr(np.stack(K, 1))
        c = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
        xopt = Q @ c
        xk, res = orc.cgls(Afn, Atfn, b.reshape(geo.proj_shape(8)), k)
        assert np.linalg.norm(xk.ravel() - xopt) <= 1e-8 * np.linalg.norm(xopt)
        assert np.all(np.diff(res) <= 1e-12 * res[0])
        v = M @ K[-1]


# --------------------------------------------------------------------------------------------
# C7 SART against explicit per-angle matrices

def test_sart_matches_dense_per_angle_update(orc):
    geo = _geo(orc, nVoxel=(8, 8, 8), nDetector=(10, 10), dDetector=(1.6, 1.6))
    angles = inputs.uniform_angles(6)
    nvox = 512
    rng = np.random.default_rng(51)
    xt = rng.uniform(0, 1, geo.vol_shape)
    b = orc.siddon_fwd(geo, angles, xt)
    # dense per-angle A_t (rays x voxels) and B_t (voxels x rays)
    A_t, B_t = [], []
    for t in range(6):
        cols = []
        for j in range(nvox):
            e = np.zeros(nvox)
            e[j] = 1
            cols.append(orc.siddon_fwd(geo, angles[t:t + 1], e.reshape(geo.vol_shape)).ravel())
        A_t.append(np.stack(cols, 1))
        rows = []
        for p in range(100):
            e = np.zeros(100)
            e[p] = 1
            rows.append(orc.bp(geo, angles[t:t + 1], e.reshape(1, 10, 10), orc.W_FDK).ravel())
        B_t.append(np.stack(rows, 1))
    x = np.zeros(nvox)
    for t in range(6):
        c = A_t[t] @ np.ones(nvox)
        W = np.where(c > 1e-2 * 1.0, 1 / np.where(c > 0, c, 1), 0)
        V = B_t[t] @ np.ones(100)
        num = B_t[t] @ (W * (b[t].ravel() - A_t[t] @ x))
        x = x + np.where(V > 1e-6, num / np.where(V > 0, V, 1), 0)
    got = orc.sart(geo, angles, b, 1)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-12, atol=1e-12)
    # residual decreases on consistent data
    r = [np.linalg.norm(orc.siddon_fwd(geo, angles, orc.sart(geo, angles, b, k)) - b) for k in (0, 1, 2, 3)]
    assert r[1] < r[0] and r[2] < r[1] and r[3] < r[2], r


def test_os_sart_matches_dense_subset_update(orc):
    """OS-SART against explicit subset matrices: subsets of 4 angles (the last one of 2), one subset
    of all 6 angles (a SIRT step), and block = 1 equal to SART."""
    geo = _geo(orc, nVoxel=(8, 8, 8), nDetector=(10, 10), dDetector=(1.6, 1.6))
    angles = inputs.uniform_angles(6)
    nvox = 512
    rng = np.random.default_rng(52)
    xt = rng.uniform(0, 1, geo.vol_shape)
    b = orc.siddon_fwd(geo, angles, xt)
    A_t, B_t = [], []
    for t in range(6):
        cols = []
        for j in range(nvox):
            e = np.zeros(nvox)
            e[j] = 1
            cols.append(orc.siddon_fwd(geo, angles[t:t + 1], e.reshape(geo.vol_shape)).ravel())
        A_t.append(np.stack(cols, 1))
        rows = []
        for p in range(100):
            e = np.zeros(100)
            e[p] = 1
            rows.append(orc.bp(geo, angles[t:t + 1], e.reshape(1, 10, 10), orc.W_FDK).ravel())
        B_t.append(np.stack(rows, 1))
    for block in (4, 6):
        x = np.zeros(nvox)
        for it in range(2):
            for s0 in range(0, 6, block):
                S = range(s0, min(6, s0 + block))
                A_S = np.concatenate([A_t[t] for t in S], 0)
                B_S = np.concatenate([B_t[t] for t in S], 1)
                bS = np.concatenate([b[t].ravel() for t in S])
                c = A_S @ np.ones(nvox)
                W = np.where(c > 1e-2 * 1.0, 1 / np.where(c > 0, c, 1), 0)
                V = B_S @ np.ones(len(bS))
                num = B_S @ (W * (bS - A_S @ x))
                x = x + 0.8 * np.where(V > 1e-6, num / np.where(V > 0, V, 1), 0)
        got = orc.os_sart(geo, angles, b, 2, block, lam=0.8)
        np.testing.assert_allclose(got.ravel(), x, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(orc.os_sart(geo, angles, b, 2, 1), orc.sart(geo, angles, b, 2))


# --------------------------------------------------------------------------------------------
# C8 TV: T1 finite differences, T2 constant, T3 1-D step edge, T4 descent

def test_T1_tv_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(61)
    x = rng.uniform(0, 1, (8, 8, 8))
    eps = 1e-8
    g = orc.tv_grad(x, eps)
    h = 1e-6
    for idx in [(0, 0, 0), (3, 4, 5), (7, 7, 7), (2, 7, 0), (5, 1, 6)]:
        xp = x.copy()
        xm = x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (orc.tv_value(xp, eps) - orc.tv_value(xm, eps)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx])) + 1e-8


def test_T2_constant_image_is_fixed(orc):
    x = np.full((6, 7, 8), 0.3)
    assert np.all(orc.tv_grad(x) == 0.0)
    np.testing.assert_array_equal(orc.tv_steps(x, 5, 0.01), x)


def test_T3_step_edge_closed_form(orc):
    # x = 0 for i < 4, 1 for i >= 4 along the fastest axis; the only nonzero difference is
    # D_x x at i = 3 (value 1, norm sqrt(1 + eps)); so g = +1/n at i = 3 ... wait: g_j picks
    # -D/n at j and +D/n at j+1: g(i=3) = -1/n, g(i=4) = +1/n, everything else 0.
    eps = 1e-8
    x = np.zeros((3, 4, 8))
    x[:, :, 4:] = 1.0
    g = orc.tv_grad(x, eps)
    n = math.sqrt(1 + eps)
    ref = np.zeros_like(x)
    ref[:, :, 3] = -1 / n
    ref[:, :, 4] = 1 / n
    np.testing.assert_allclose(g, ref, rtol=1e-14, atol=1e-14)


def test_T4_tv_decreases(orc):
    w = inputs.workload("tiny")
    vol = inputs.voxelize(w, dtype=np.float64)[16:48, 16:48, 16:48]
    vol = vol + 0.05 * np.random.default_rng(7).standard_normal(vol.shape)
    tv0 = orc.tv_value(vol)
    x = orc.tv_steps(vol, 5, 0.001)
    assert orc.tv_value(x) < tv0


def test_fp32_input_samplers_equal_fp64_on_widened_data(orc):
    """The per-ray and per-voxel samplers that read FP32 arrays in place (for inputs too large to
    copy) perform the FP64 arithmetic of the pinned FP64 samplers on the exactly widened values."""
    geo = _geo(orc, nVoxel=(11, 9, 7), dVoxel=(1.1, 0.9, 1.3), offOrigin=(0.3, -0.2, 0.4),
               nDetector=(13, 10), dDetector=(1.5, 1.7), offDetector=(0.4, -0.3))
    rng = np.random.default_rng(31)
    angles = inputs.uniform_angles(12)
    vol = rng.uniform(0, 1, geo.vol_shape).astype(np.float32)
    proj = rng.uniform(0, 1, geo.proj_shape(len(angles))).astype(np.float32)
    rays = rng.choice(proj.size, 40, replace=False)
    vox = rng.choice(vol.size, 40, replace=False)
    np.testing.assert_array_equal(orc.siddon_rays(geo, angles, rays, vol),
                                  orc.siddon_rays(geo, angles, rays, vol.astype(np.float64)))
    for kind in (orc.W_FDK, orc.W_PM):
        np.testing.assert_array_equal(orc.bp_voxels(geo, angles, proj, vox, kind),
                                      orc.bp_voxels(geo, angles, proj.astype(np.float64), vox, kind))
    np.testing.assert_array_equal(orc.siddon_adj_voxels(geo, angles, proj, vox),
                                  orc.siddon_adj_voxels(geo, angles, proj.astype(np.float64), vox))


# --- the sampled entry points (used by every large-size parity test and the CPU baseline)

def _pixel_ray_by_convention(geo, th, a, b):
    """Source and pixel centre of ray (th, a, b), written out from the stated conventions: source
    DSO (cos, sin, 0), detector centre -(DSD - DSO)(cos, sin, 0), e_u = (-sin, cos, 0), e_v = z."""
    c, s = math.cos(th), math.sin(th)
    u = (a - (geo.nDetector[0] - 1) / 2) * geo.dDetector[0] + geo.offDetector[0]
    v = (b - (geo.nDetector[1] - 1) / 2) * geo.dDetector[1] + geo.offDetector[1]
    S = np.array([geo.DSO * c, geo.DSO * s, 0.0])
    C = -(geo.DSD - geo.DSO) * np.array([c, s, 0.0])
    return S, C + u * np.array([-s, c, 0.0]) + v * np.array([0.0, 0.0, 1.0])


def _ragged_case(orc, seed):
    geo = _geo(orc, nVoxel=(11, 9, 7), dVoxel=(1.1, 0.9, 1.3), offOrigin=(0.3, -0.2, 0.4),
               nDetector=(13, 10), dDetector=(1.5, 1.7), offDetector=(0.4, -0.3))
    rng = np.random.default_rng(seed)
    angles = rng.uniform(0, 2 * np.pi, 5)
    vol = rng.uniform(0, 1, geo.vol_shape)
    return geo, angles, vol, rng


def test_sampled_rays_equal_the_whole_array_projectors(orc):
    """siddon_rays / interp_rays decode a flat index as (t Nv + b) Nu + a.  On a ragged geometry
    with volume and detector offsets and a 13 x 10 detector they must return, bit for bit, the
    whole-array projectors' values at those indices, for every index in a shuffled order; a decode
    with a and b (or the angle) swapped reads another pixel, and the data tell them apart."""
    geo, angles, vol, rng = _ragged_case(orc, 41)
    idx = rng.permutation(len(angles) * 10 * 13)
    for whole, sampled in ((orc.siddon_fwd, orc.siddon_rays), (orc.interp_fwd, orc.interp_rays)):
        full = whole(geo, angles, vol)
        assert full.shape == (5, 10, 13)
        np.testing.assert_array_equal(sampled(geo, angles, idx, vol), full.ravel()[idx])
        # the decodes a plausible mistake would make give other values on these data
        t, rem = np.divmod(idx, 10 * 13)
        b, a = np.divmod(rem, 13)
        ok = (a < 10) & (b < 13) & (a != b)
        swapped = full[t[ok], a[ok], b[ok]]
        assert np.mean(swapped != full.ravel()[idx[ok]]) > 0.8
    # the FP32 reader of the Siddon sampler, on FP32-representable data
    v32 = vol.astype(np.float32)
    np.testing.assert_array_equal(orc.siddon_rays(geo, angles, idx, v32),
                                  orc.siddon_fwd(geo, angles, v32.astype(np.float64)).ravel()[idx])


def test_whole_array_projectors_follow_the_pixel_convention(orc):
    """Every pixel of siddon_fwd and interp_fwd equals the single-ray projectors (themselves pinned
    by P1-P4 and I1-I2) on the ray whose endpoints are written out here from the conventions, so
    the pixel loops' angle, row and column decode and their pixel positions are pinned."""
    geo, angles, vol, _ = _ragged_case(orc, 42)
    fs = orc.siddon_fwd(geo, angles, vol)
    fi = orc.interp_fwd(geo, angles, vol)
    for t, th in enumerate(angles):
        for b in range(10):
            for a in range(13):
                S, P = _pixel_ray_by_convention(geo, th, a, b)
                rs, _ = orc.siddon_ray(geo, S, P, vol)
                ri, _ = orc.interp_ray(geo, S, P, vol)
                assert abs(fs[t, b, a] - rs) <= 1e-12 * max(abs(rs), 1.0), (t, b, a)
                assert abs(fi[t, b, a] - ri) <= 1e-12 * max(abs(ri), 1.0), (t, b, a)


def test_sampled_voxels_equal_the_whole_array_backprojectors(orc):
    """bp_voxels and siddon_adj_voxels decode a flat voxel index as (k Ny + j) Nx + i and must agree
    with the whole-volume backprojectors at every voxel (bitwise for the voxel-driven ones, which
    run the same per-voxel sum; to rounding for the exact transpose, whose whole-volume form adds
    the scattered pieces in another order)."""
    geo, angles, _, rng = _ragged_case(orc, 43)
    proj = rng.uniform(-1, 1, geo.proj_shape(len(angles)))
    idx = rng.permutation(11 * 9 * 7)
    for kind in (orc.W_FDK, orc.W_PM):
        np.testing.assert_array_equal(orc.bp_voxels(geo, angles, proj, idx, kind),
                                      orc.bp(geo, angles, proj, kind).ravel()[idx])
    full = orc.siddon_adj(geo, angles, proj).ravel()
    np.testing.assert_allclose(orc.siddon_adj_voxels(geo, angles, proj, idx), full[idx],
                               rtol=1e-12, atol=1e-12 * np.abs(full).max())


def test_siddon_segment_count_is_the_piece_count(orc):
    """siddon_segments counts a ray's pieces: an axis-aligned ray through the middle of an n-voxel
    row crosses n - 1 inner planes, so it has n pieces; the count matches siddon_ray's own."""
    geo, angles, vol, rng = _ragged_case(orc, 44)
    idx = rng.choice(5 * 10 * 13, 60, replace=False)
    got = orc.siddon_segments(geo, angles, idx)
    for q, r in enumerate(idx):
        t, rem = divmod(int(r), 130)
        b, a = divmod(rem, 13)
        S, P = _pixel_ray_by_convention(geo, angles[t], a, b)
        _, ns = orc.siddon_ray(geo, S, P, vol)
        assert got[q] == ns
    # theta = 0 and the central pixel of an odd detector: the ray runs along x through y = z = 0,
    # which lies inside one voxel row of a grid with odd Ny and Nz and no offset
    g2 = _geo(orc, nVoxel=(6, 5, 3), nDetector=(3, 3))
    assert orc.siddon_segments(g2, np.array([0.0]), np.array([4]))[0] == 6


# --- FDK reconstruction (Feldkamp, Davis & Kress 1984, the algorithm behind Section 2.2's FDK weight)

def test_F1_ramp_filter_response_to_a_cosine(orc):
    """The discrete ramp filter's response is |omega| / (2 pi) at every frequency below Nyquist:
    1/4 - (2/pi^2) sum_{odd m} cos(m w)/m^2 = |w|/(2 pi), from the Fourier series
    sum_{odd m} cos(m w)/m^2 = (pi/8)(pi - 2|w|).  With DSD so large that the cosine weight is 1 to
    1e-8, `fdk_filter` of the row cos(w a + phi) must be (dtheta/2)(1/ds)(|w|/2pi) cos(w a + phi)
    away from the row ends, where the truncated tail of the taps is below 1/(pi^2 * 127).  A shifted,
    mis-scaled or mis-signed tap set, or a wrong ds, fails this."""
    nu, nv, na = 512, 3, 8
    DSD, DSO, du = 1e7, 6e6, 0.7
    geo = orc.Geometry(DSO, DSD, (4, 4, 4), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), (nu, nv), (du, 1.0),
                       (0.0, 0.0), 0.5)
    angles = inputs.uniform_angles(na)
    a = np.arange(nu)
    ds = du * DSO / DSD
    for wfreq, phi in ((0.3 * np.pi, 0.4), (0.75 * np.pi, -1.1), (0.05 * np.pi, 2.0)):
        row = np.cos(wfreq * a + phi)
        proj = np.broadcast_to(row, (na, nv, nu)).copy()
        q = orc.fdk_filter(geo, angles, proj)
        want = (2 * np.pi / na / 2) / ds * (wfreq / (2 * np.pi)) * row
        amp = (2 * np.pi / na / 2) / ds
        inner = slice(nu // 4, 3 * nu // 4)
        np.testing.assert_allclose(q[:, :, inner] / amp, np.broadcast_to(want[inner] / amp, q[:, :, inner].shape),
                                   atol=1.5e-3)


def _fdk_pin_case(nv, n_angles=64):
    # a short source distance so that the fan reaches 28 degrees and the weights matter
    return inputs.Workload("fdk_pin", (64, 64, 64), (1.0, 1.0, 1.0), (128, nv), (1.0, 1.0), n_angles, 0, 0,
                           DSO=60.0, DSD=90.0)


def test_F2_fdk_reconstructs_a_centred_sphere(orc):
    """In the mid-plane FDK is fan-beam filtered backprojection, exact for band-limited data: the
    reconstruction of a unit-density sphere of radius 28 mm from its exact line integrals is 1
    inside (here within 0.5 % at every voxel at least 6 mm from the surface in the two middle
    slices; measured 0.17 %).  Without the cosine weight the error is 5.6 %; without the 1/2, or
    with ds left at the detector pitch, it is 100 % and 33 %."""
    w = _fdk_pin_case(128)
    ells = [inputs.Ellipsoid(np.zeros(3), np.array([28.0] * 3), 1.0, np.eye(3))]
    geo = orc.Geometry.from_dict(w.geometry_dict())
    p = inputs.analytic_projections(w, ells, dtype=np.float64)
    rec = orc.fdk(geo, w.angles, p)
    c = inputs.voxel_centres_1d(64, 1.0, 0.0)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    m = (np.sqrt(xx ** 2 + yy ** 2 + zz ** 2) < 22.0) & (np.abs(zz) <= 1.0)
    assert m.sum() > 2000
    assert np.max(np.abs(rec[m] - 1.0)) <= 5e-3


def test_F3_fdk_exact_for_an_axially_invariant_object(orc):
    """FDK is exact for objects that do not vary along the rotation axis: a ray at elevation kappa
    crosses such an object along 1/cos(kappa) times the in-plane chord, which the cosine weight's v
    term cancels, so every detector row carries the mid-plane data and every slice is reconstructed
    as the mid-plane.  A cylinder of radius 24 mm (an ellipsoid with a 1e7 mm axis, its line
    integrals not clipped to the grid) comes back as 1 inside, within 0.3 % at every voxel at least
    6 mm from its surface in every slice (measured 0.08 %).  Without the v term of the cosine
    weight the error is 17 %.  The detector is tall enough that every voxel projects onto it."""
    w = _fdk_pin_case(160)
    ells = [inputs.Ellipsoid(np.zeros(3), np.array([24.0, 24.0, 1e7]), 1.0, np.eye(3))]
    geo = orc.Geometry.from_dict(w.geometry_dict())
    p = inputs.analytic_projections(w, ells, clip_to_grid=False, dtype=np.float64)
    rec = orc.fdk(geo, w.angles, p)
    c = inputs.voxel_centres_1d(64, 1.0, 0.0)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    m = np.sqrt(xx ** 2 + yy ** 2) < 18.0
    assert m.sum() > 60000
    assert np.max(np.abs(rec[m] - 1.0)) <= 3e-3


def test_T5_split_tv_reproduces_whole_image_steps(orc):
    """Section 2.3's splitting with halos `depth` deep: with the exact image norm substituted for the
    per-slab estimate, every slab height and depth gives the whole-image steps (the halo keeps each
    slab's own slices exact for `depth` steps); with one slab the per-slab norm is the image norm.
    A halo too shallow for its round, or a stale copy of a neighbour, fails this."""
    rng = np.random.default_rng(4)
    x0 = (rng.uniform(0, 1, (29, 17, 13)) > 0.7) * 0.8 + 0.05 * rng.standard_normal((29, 17, 13))
    ref = orc.tv_steps(x0, 7, 0.01)
    for slab, depth in ((10, 3), (5, 2), (1, 4), (7, 7), (4, 1), (3, 10)):
        got = orc.tv_steps_split(x0, 7, 0.01, slab, depth, norm="global")
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(orc.tv_steps_split(x0, 7, 0.01, 29, 3), ref, rtol=0, atol=1e-13)
    # the per-slab norm is an approximation: close to, not equal to, the whole-image steps
    e = np.linalg.norm(orc.tv_steps_split(x0, 7, 0.01, 5, 2) - ref) / np.linalg.norm(ref)
    assert 1e-6 < e < 1e-2


# --- ROF model by Chambolle's projection (the second TV minimiser of Section 2.3)

def test_R1_divergence_is_minus_the_adjoint_of_the_gradient(orc):
    """<grad u, p> = -<u, div p> for any u and p, the identity Chambolle's iteration rests on; a
    wrong boundary row of either operator breaks it."""
    rng = np.random.default_rng(1)
    for shape in ((5, 6, 7), (1, 4, 9), (2, 1, 1)):
        u = rng.standard_normal(shape)
        p = rng.standard_normal((3,) + shape)
        lhs = np.sum(orc.grad3(u) * p)
        assert abs(lhs + np.sum(u * orc.div3(p))) <= 1e-12 * (np.abs(u).sum() * np.abs(p).sum())


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_R2_rof_of_a_step_has_the_closed_form(orc, axis):
    """A step of height h between two runs of n samples: the ROF solution keeps the step and moves
    each level by lam / n towards the other (minimise n a^2 + n (b - h)^2 over 2 lam + |b - a|),
    when h > 2 lam / n.  Along each axis in turn."""
    n, h, lam = 8, 1.0, 2.0
    shape = [1, 1, 1]
    shape[axis] = 2 * n
    idx = np.arange(2 * n).reshape(shape)
    f = np.where(idx >= n, h, 0.0)
    u = orc.rof_chambolle(f, lam, 5000)
    want = np.where(idx < n, lam / n, h - lam / n)
    np.testing.assert_allclose(u, want, rtol=0, atol=1e-8)


def test_R3_rof_keeps_the_mean_and_constant_images(orc):
    rng = np.random.default_rng(2)
    x0 = rng.uniform(0, 1, (9, 8, 7))
    assert abs(orc.rof_chambolle(x0, 0.1, 50).mean() - x0.mean()) <= 1e-14
    np.testing.assert_array_equal(orc.rof_chambolle(np.full((4, 5, 6), 0.3), 0.1, 20), np.full((4, 5, 6), 0.3))


def test_R4_split_rof_equals_the_whole_image_iteration(orc):
    """Chambolle's step is local (p at a slice depends on p one slice either side) and needs no
    image-wide sum, so slabs whose halos cover the iterations of a round reproduce the whole-image
    iteration; the upper halo needs one slice more, and without it the slabs' own slices go wrong."""
    rng = np.random.default_rng(3)
    f = ((rng.uniform(0, 1, (23, 9, 11)) > 0.6) * 1.0 + 0.1 * rng.standard_normal((23, 9, 11)))
    ref = orc.rof_chambolle(f, 0.2, 13)
    for slab, depth in ((23, 13), (7, 4), (5, 1), (1, 3), (4, 13), (6, 5)):
        np.testing.assert_allclose(orc.rof_chambolle_split(f, 0.2, 13, slab, depth), ref, rtol=0, atol=1e-14)
    for slab, depth in ((7, 4), (5, 1)):
        bad = orc.rof_chambolle_split(f, 0.2, 13, slab, depth, upper_extra=0)
        assert np.abs(bad - ref).max() > 1e-7


def test_stored_siddon_piece_count_reproduces():
    """The stored gather-model unit of the Siddon projector (pieces per voxel-projection at the
    512^3 / 360 / 512^2 workload) is reproduced by the oracle on an independent seeded sample of
    rays, within four standard errors of the two estimates."""
    sys_path = os.path.join(os.path.dirname(__file__), "golden")
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_siddon_segments",
                                                  os.path.join(sys_path, "make_siddon_segments.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    stored = json.load(open(os.path.join(sys_path, "siddon_segments.json")))
    fresh = mod.count(20000, seed=stored["seed"] + 1)
    err = math.hypot(stored["stderr_pieces_per_voxel_proj"], fresh["stderr_pieces_per_voxel_proj"])
    assert abs(fresh["pieces_per_voxel_proj"] - stored["pieces_per_voxel_proj"]) <= 4 * err
    assert 1.0 < stored["pieces_per_voxel_proj"] < 1.3
