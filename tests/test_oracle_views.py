"""Pins of the oracle's per-view geometry (Section 2.1: the projectors serve circular, C-arm and
helical scans; Section 3.2 runs OS-SART on them).  A view is a source S, a detector centre C and
the detector's unit axes e_u, e_v; the oracle's circular orbit is one such table, so every pin of
the circular operators already runs through the general code.  The pins here reach what a circular
orbit cannot: tilted detectors, sources off the mid-plane, views that differ by a translation along
the axis.  CPU only.
"""
import numpy as np
import pytest

from paper_1905_03748_amd import inputs
from test_oracle_pins import _box_chord_faces, _geo


def _carm(n=5, seed=3, tilt=20.0, jitter=4.0, orbit_tilt=10.0):
    return inputs.carm_views(1000.0, 1500.0, inputs.uniform_angles(n) + 0.3, seed, tilt, jitter, orbit_tilt)


def _pixel(geo, view, a, b):
    """Source and centre of pixel (a, b) of a view, written out from the pixel convention."""
    S, C, eu, ev = view[0:3], view[3:6], view[6:9], view[9:12]
    u = (a - (geo.nDetector[0] - 1) / 2.0) * geo.dDetector[0] + geo.offDetector[0]
    v = (b - (geo.nDetector[1] - 1) / 2.0) * geo.dDetector[1] + geo.offDetector[1]
    return S, C + u * eu + v * ev


def _detector_coords(geo, view, X):
    """(a*, b*) of the point X: the ray from S through X meets the detector plane at C + u e_u + v e_v;
    (m, u, v) from the 3 x 3 linear system S + m (X - S) = C + u e_u + v e_v."""
    S, C, eu, ev = view[0:3], view[3:6], view[6:9], view[9:12]
    m, u, v = np.linalg.solve(np.stack([X - S, -eu, -ev], 1), C - S)
    a = (u - geo.offDetector[0]) / geo.dDetector[0] + (geo.nDetector[0] - 1) / 2.0
    b = (v - geo.offDetector[1]) / geo.dDetector[1] + (geo.nDetector[1] - 1) / 2.0
    return a, b


def test_V1_views_table_equals_the_angle_form(orc):
    geo = _geo(orc, nVoxel=(9, 8, 7), offOrigin=(0.4, -0.3, 0.2), nDetector=(11, 9), offDetector=(0.3, -0.5))
    angles = inputs.uniform_angles(5) + 0.1
    views = orc.circular_views(geo, angles)
    rng = np.random.default_rng(71)
    x = rng.uniform(0, 1, geo.vol_shape)
    y = rng.uniform(-1, 1, geo.proj_shape(5))
    np.testing.assert_array_equal(orc.siddon_fwd(geo, views, x), orc.siddon_fwd(geo, angles, x))
    np.testing.assert_array_equal(orc.bp(geo, views, y, orc.W_PM), orc.bp(geo, angles, y, orc.W_PM))
    with pytest.raises(ValueError):
        orc.siddon_fwd(geo, views[:, :11], x)


def test_V2_ones_volume_gives_box_chords_under_tilted_and_raised_views(orc):
    """Siddon of a ones volume is the length of the ray inside the grid box, found here by face
    intersection from pixel rays written out from the convention: the ray geometry of tilted
    detectors, jittered sources and helical heights, with an off-centre box and detector, is pinned
    (swapping e_u and e_v, a sign of an axis or the pixel offsets moves rays and changes chords)."""
    geo = _geo(orc, nVoxel=(10, 7, 6), dVoxel=(1.2, 0.9, 1.4), offOrigin=(1.1, -0.7, 0.9), nDetector=(9, 8),
               dDetector=(1.9, 1.5), offDetector=(0.8, -0.6))
    lo = np.array(geo.offOrigin) - np.array(geo.nVoxel) * np.array(geo.dVoxel) / 2
    hi = np.array(geo.offOrigin) + np.array(geo.nVoxel) * np.array(geo.dVoxel) / 2
    ones = np.ones(geo.vol_shape)
    for views in (_carm(), inputs.helical_views(1000.0, 1500.0, inputs.uniform_angles(5) + 0.2, 7.0, -3.0)):
        p = orc.siddon_fwd(geo, views, ones)
        hit = 0
        for t in range(len(views)):
            for b in range(8):
                for a in range(9):
                    S, P = _pixel(geo, views[t], a, b)
                    ref = _box_chord_faces(S, P, lo, hi)
                    hit += ref > 0
                    assert abs(p[t, b, a] - ref) <= 1e-10 * max(ref, 1.0), (t, b, a, p[t, b, a], ref)
        assert hit > 0.5 * p.size  # most rays meet the box, so the pin has teeth


def test_V3_transposes_and_samplers_under_views(orc):
    """<A x, y> = <x, A^T y> for the Siddon pair and for the voxel-driven backprojectors with their
    splat transposes, on C-arm views; the sampled entry points equal the whole-array ones."""
    geo = _geo(orc, nVoxel=(9, 8, 7), offOrigin=(0.4, -0.3, 0.2), nDetector=(11, 9), offDetector=(0.3, -0.5))
    views = _carm(4, seed=5)
    rng = np.random.default_rng(72)
    x = rng.uniform(-1, 1, geo.vol_shape)
    y = rng.uniform(-1, 1, geo.proj_shape(4))
    lhs = float(np.sum(orc.siddon_fwd(geo, views, x) * y))
    rhs = float(np.sum(x * orc.siddon_adj(geo, views, y)))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(x).sum() * 10)
    for kind in (orc.W_FDK, orc.W_PM):
        lhs = float(np.sum(orc.bp(geo, views, y, kind) * x))
        rhs = float(np.sum(orc.bp_transpose(geo, views, x, kind) * y))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12
    ridx = rng.permutation(4 * 9 * 11)[:150]
    full = orc.siddon_fwd(geo, views, x).ravel()
    np.testing.assert_array_equal(orc.siddon_rays(geo, views, ridx, x), full[ridx])
    np.testing.assert_array_equal(orc.interp_rays(geo, views, ridx, x), orc.interp_fwd(geo, views, x).ravel()[ridx])
    vidx = rng.permutation(9 * 8 * 7)[:120]
    np.testing.assert_array_equal(orc.bp_voxels(geo, views, y, vidx, orc.W_FDK), orc.bp(geo, views, y).ravel()[vidx])
    adj = orc.siddon_adj(geo, views, y).ravel()
    np.testing.assert_allclose(orc.siddon_adj_voxels(geo, views, y, vidx), adj[vidx], rtol=1e-12,
                               atol=1e-12 * np.abs(adj).max())


def test_V4_backprojection_reads_where_the_ray_meets_the_tilted_detector(orc):
    """Bilinear interpolation reproduces a linear function of the pixel indices, so backprojecting
    y(a, b) = alpha a + beta b + gamma gives, at a voxel whose four taps lie on the detector,
    w (alpha a* + beta b* + gamma) with w the weight (the backprojection of ones there).  With (a*, b*)
    from a linear solve for the ray-plane intersection, this pins the oracle's map from voxel to
    detector coordinates on tilted, shifted detectors."""
    geo = _geo(orc, nVoxel=(7, 6, 5), dVoxel=(2.0, 2.0, 2.0), offOrigin=(1.0, -2.0, 1.5), nDetector=(40, 36),
               dDetector=(1.1, 1.3), offDetector=(0.7, -0.4))
    views = _carm(3, seed=8, tilt=25.0)
    al, be, ga = 0.37, -0.81, 2.5
    nu, nv = geo.nDetector
    lin = al * np.arange(nu)[None, :] + be * np.arange(nv)[:, None] + ga
    checked = 0
    for t in range(3):
        v1 = views[t:t + 1]
        for kind in (orc.W_FDK, orc.W_PM):
            got = orc.bp(geo, v1, lin[None], kind)
            w = orc.bp(geo, v1, np.ones((1, nv, nu)), kind)
            for k in range(5):
                for j in range(6):
                    for i in range(7):
                        X = np.array(geo.offOrigin) + (np.array([i, j, k]) - (np.array(geo.nVoxel) - 1) / 2) * 2.0
                        a, b = _detector_coords(geo, views[t], X)
                        if not (0 <= a < nu - 1 and 0 <= b < nv - 1):
                            continue
                        checked += 1
                        ref = w[k, j, i] * (al * a + be * b + ga)
                        assert abs(got[k, j, i] - ref) <= 1e-11 * abs(ref) + 1e-12, (t, kind, i, j, k)
    assert checked > 300


def test_V5_helical_views_are_the_circular_ones_shifted_along_the_axis(orc):
    """Raising the source and the detector by an integer number of slices k dz is the same as
    lowering the volume by k slices (Section 2.1's helical scans): every operator commutes with the
    shift (volumes padded with zeros so nothing leaves the grid).  Catches a weight that uses |S|
    (which grows with the height) where the depth along the normal belongs, and any use of the
    source height as if it were zero."""
    geo = _geo(orc, nVoxel=(8, 7, 12), dVoxel=(1.0, 1.1, 0.9), offOrigin=(0.2, -0.3, 0.1), nDetector=(12, 14),
               dDetector=(1.6, 1.4))
    angles = inputs.uniform_angles(5) + 0.4
    dz, k = geo.dVoxel[2], 3
    circ = orc.circular_views(geo, angles)
    hel = circ.copy()
    hel[:, 2] += k * dz
    hel[:, 5] += k * dz
    rng = np.random.default_rng(73)
    x = np.zeros(geo.vol_shape)
    x[k:12 - k] = rng.uniform(0, 1, (12 - 2 * k, 7, 8))
    xs = np.zeros_like(x)
    xs[k:] = x[:12 - k]               # the volume raised by k slices
    for fwd in (orc.siddon_fwd, orc.interp_fwd):
        np.testing.assert_allclose(fwd(geo, hel, xs), fwd(geo, circ, x), rtol=1e-11, atol=1e-11)
    y = rng.uniform(0, 1, geo.proj_shape(5))
    for kind in (orc.W_FDK, orc.W_PM):
        bh = orc.bp(geo, hel, y, kind)
        bc = orc.bp(geo, circ, y, kind)
        np.testing.assert_allclose(bh[k:], bc[:12 - k], rtol=1e-11, atol=1e-11)
    ah = orc.siddon_adj(geo, hel, y)
    ac = orc.siddon_adj(geo, circ, y)
    np.testing.assert_allclose(ah[k:], ac[:12 - k], rtol=1e-11, atol=1e-11 * np.abs(ac).max())


def test_V6_operators_commute_with_a_quarter_turn_of_the_scanner(orc):
    """Turning every view by 90 degrees about z (S, C, e_u, e_v) and the volume with it leaves the
    projections unchanged and turns the backprojections: on tilted, jittered C-arm views this
    checks every component of the vector arithmetic (a mixed-up x/y component, or a normal taken
    with the wrong orientation, breaks it)."""
    n = 8
    geo = _geo(orc, nVoxel=(n, n, 6), dVoxel=(1.3, 1.3, 1.0), offOrigin=(0.0, 0.0, 0.7), nDetector=(12, 10),
               offDetector=(0.5, -0.2))
    views = _carm(4, seed=11, tilt=18.0)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    turned = np.concatenate([views[:, 3 * q:3 * q + 3] @ R.T for q in range(4)], 1)
    rng = np.random.default_rng(74)
    x = rng.uniform(0, 1, geo.vol_shape)
    xr = x.transpose(0, 2, 1)[:, :, ::-1]   # xr[k, j', i'] = x at the turned-back position
    for fwd in (orc.siddon_fwd, orc.interp_fwd):
        np.testing.assert_allclose(fwd(geo, turned, xr), fwd(geo, views, x), rtol=1e-11, atol=1e-11)
    y = rng.uniform(0, 1, geo.proj_shape(4))
    for kind in (orc.W_FDK, orc.W_PM):
        np.testing.assert_allclose(orc.bp(geo, turned, y, kind),
                                   orc.bp(geo, views, y, kind).transpose(0, 2, 1)[:, :, ::-1], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(orc.siddon_adj(geo, turned, y),
                               orc.siddon_adj(geo, views, y).transpose(0, 2, 1)[:, :, ::-1], rtol=1e-11, atol=1e-11)


def test_V7_pseudo_matched_weight_matches_siddon_column_sums_on_tilted_detectors(orc):
    """The pseudo-matched weight is the Siddon projector's ray density at the voxel (its column sum
    of one view) for any detector pose: with the detector tilted, a pixel's ray tube narrows by
    cos^3 of the ray's angle to the normal, which |SX| DSD_v^2 / L^3 accounts for.  A weight that
    took depths along the central ray instead of the normal, or the source-to-centre distance for
    DSD_v, is off by several per cent at these tilts."""
    geo = _geo(orc, nVoxel=(32, 32, 32), dVoxel=(1.0, 1.0, 1.0), nDetector=(72, 72), dDetector=(1.5, 1.5))
    views = inputs.carm_views(1000.0, 1500.0, np.array([0.2, 1.3, 2.9]), 12, 25.0, 6.0, 15.0)
    ratios = []
    for t in range(3):
        ones_p = np.ones((1, 72, 72))
        col = orc.siddon_adj(geo, views[t:t + 1], ones_p)
        pm = orc.bp(geo, views[t:t + 1], ones_p, orc.W_PM)
        inner = (slice(8, 24),) * 3
        ratios.append(float(np.mean(col[inner] / pm[inner])))
    assert all(abs(r - 1.0) < 0.02 for r in ratios), ratios


def test_V8_os_sart_with_views_matches_dense_subset_update(orc):
    """OS-SART on C-arm views against explicit subset matrices (subsets of 2 of 5 views)."""
    geo = _geo(orc, nVoxel=(6, 6, 6), nDetector=(9, 8), dDetector=(1.6, 1.6))
    views = _carm(5, seed=13)
    nvox, npix = 216, 72
    rng = np.random.default_rng(75)
    b = orc.siddon_fwd(geo, views, rng.uniform(0, 1, geo.vol_shape))
    A_t, B_t = [], []
    for t in range(5):
        A_t.append(np.stack([orc.siddon_fwd(geo, views[t:t + 1], e.reshape(geo.vol_shape)).ravel()
                             for e in np.eye(nvox)], 1))
        B_t.append(np.stack([orc.bp(geo, views[t:t + 1], e.reshape(1, 8, 9), orc.W_FDK).ravel()
                             for e in np.eye(npix)], 1))
    x = np.zeros(nvox)
    for s0 in range(0, 5, 2):
        S = range(s0, min(5, s0 + 2))
        A_S = np.concatenate([A_t[t] for t in S], 0)
        B_S = np.concatenate([B_t[t] for t in S], 1)
        bS = np.concatenate([b[t].ravel() for t in S])
        c = A_S @ np.ones(nvox)
        W = np.where(c > 1e-2, 1 / np.where(c > 0, c, 1), 0)
        V = B_S @ np.ones(len(bS))
        x = x + np.where(V > 1e-6, (B_S @ (W * (bS - A_S @ x))) / np.where(V > 0, V, 1), 0)
    np.testing.assert_allclose(orc.os_sart(geo, views, b, 1, 2).ravel(), x, rtol=1e-12, atol=1e-12)
    with pytest.raises(ValueError):
        orc.fdk(geo, views, b)


def test_V9_weights_depend_on_the_detector_plane_not_on_its_centre(orc):
    """Both weights measure depths along the detector's normal (the view's principal axis), so
    sliding the detector within its own plane (C -> C + du_s e_u + dv_s e_v) leaves them unchanged
    and moves every voxel's detector coordinates by exactly (-du_s / du, -dv_s / dv).  A weight that
    measured depth along the source-to-centre ray would change with the slide."""
    geo = _geo(orc, nVoxel=(7, 6, 5), dVoxel=(2.0, 2.0, 2.0), nDetector=(48, 44), dDetector=(1.1, 1.3))
    views = _carm(3, seed=14, tilt=25.0)
    slid = views.copy()
    sh_u, sh_v = 6.3, -4.1
    slid[:, 3:6] += sh_u * views[:, 6:9] + sh_v * views[:, 9:12]
    nu, nv = geo.nDetector
    al, be, ga = 0.21, 0.57, -1.3
    lin = al * np.arange(nu)[None, :] + be * np.arange(nv)[:, None] + ga
    for t in range(3):
        for kind in (orc.W_FDK, orc.W_PM):
            w0 = orc.bp(geo, views[t:t + 1], np.ones((1, nv, nu)), kind)
            w1 = orc.bp(geo, slid[t:t + 1], np.ones((1, nv, nu)), kind)
            l0 = orc.bp(geo, views[t:t + 1], lin[None], kind)
            l1 = orc.bp(geo, slid[t:t + 1], lin[None], kind)
            # where the four taps are on the detector in both positions, the weight is the same and
            # the linear data read lower by the slide in pixels
            for k in range(5):
                for j in range(6):
                    for i in range(7):
                        X = np.array(geo.offOrigin) + (np.array([i, j, k]) - (np.array(geo.nVoxel) - 1) / 2) * 2.0
                        a0, b0 = _detector_coords(geo, views[t], X)
                        a1, b1 = _detector_coords(geo, slid[t], X)
                        if not (1 <= min(a0, a1) and max(a0, a1) < nu - 2 and 1 <= min(b0, b1) and max(b0, b1) < nv - 2):
                            continue
                        assert abs(w1[k, j, i] - w0[k, j, i]) <= 1e-12 * w0[k, j, i]
                        ref = l0[k, j, i] - w0[k, j, i] * (al * sh_u / geo.dDetector[0] + be * sh_v / geo.dDetector[1])
                        assert abs(l1[k, j, i] - ref) <= 1e-11 * abs(l0[k, j, i]) + 1e-11
