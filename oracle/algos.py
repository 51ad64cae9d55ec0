"""Oracle versions of the iterative algorithms that call the projection operators (test
infrastructure only), in FP64 numpy.  Each follows the published method step by step.

Operators are passed in as callables so the same code runs on the matrix-free oracle operators
and on dense matrices built from them (used by the pins).
"""
from __future__ import annotations

import numpy as np

from . import core


def _dot(a, b):
    return float(np.dot(np.ravel(a), np.ravel(b)))


def cgls(A, At, b, niter, x0=None):
    """Conjugate gradient least squares (Bjorck), the algorithm used for the coffee-bean scan
    (Section 3.2): minimises ||A x - b|| over Krylov spaces of A^T A.

    Returns (x, resid) where resid[k] = sqrt(rho_k) from the recurrence rho_{k+1} = rho_k - alpha
    gamma_k (which uses <r_k, A p_k> = gamma_k); resid has niter+1 entries and repeats its last
    value if the iteration stops early (A p = 0).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(At(b)) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x)
    s = At(r)
    p = s.copy()
    gamma = _dot(s, s)
    rho = _dot(r, r)
    resid = [np.sqrt(max(rho, 0.0))]
    for _ in range(niter):
        q = A(p)
        delta = _dot(q, q)
        if delta == 0.0:
            break
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        rho = rho - alpha * gamma
        resid.append(np.sqrt(max(rho, 0.0)))
        s = At(r)
        gamma_new = _dot(s, s)
        beta = gamma_new / gamma
        gamma = gamma_new
        p = s + beta * p
    while len(resid) < niter + 1:
        resid.append(resid[-1])
    return x, np.array(resid)


# SART thresholds (the paper gives no SART parameters; these are our readings):
#   a ray's weight 1/(A_t 1)_p is used only when its chord through the grid exceeds 1e-2 of the
#   smallest voxel size (shorter chords graze a corner and are dropped);
#   a voxel is updated only where the backprojected ones (B_t 1)_j exceed 1e-6.
SART_RAY_FRACTION = 1e-2
SART_VOXEL_MIN = 1e-6


def sart(geo: core.Geometry, angles, b, niter, lam=1.0, x0=None):
    """SART (Andersen & Kak 1984; the OS-SART family of Section 3.2 with one angle per block).

    For each sweep, for each projection t in natural order (`angles`: angles of a circular orbit
    or an n x 12 table of views, as the operators take):
        W_p = 1/(A_t 1)_p,  V_j = (B_t 1)_j,  x += lam * B_t(W * (b_t - A_t x)) / V
    with A the Siddon projector and B the FDK-weighted voxel backprojector.
    """
    angles = np.asarray(angles, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(geo.vol_shape) if x0 is None else np.array(x0, dtype=np.float64)
    ones_vol = np.ones(geo.vol_shape)
    dmin = min(geo.dVoxel)
    ones_proj = np.ones((1,) + b.shape[1:])
    for _ in range(niter):
        for t in range(len(angles)):
            th = angles[t:t + 1]
            chord = core.siddon_fwd(geo, th, ones_vol)[0]
            W = np.where(chord > SART_RAY_FRACTION * dmin, 1.0 / np.where(chord > 0, chord, 1.0), 0.0)
            r = W * (b[t] - core.siddon_fwd(geo, th, x)[0])
            num = core.bp(geo, th, r[None], core.W_FDK)
            V = core.bp(geo, th, ones_proj, core.W_FDK)
            upd = np.where(V > SART_VOXEL_MIN, num / np.where(V > 0, V, 1.0), 0.0)
            x = x + lam * upd
    return x


def os_sart(geo: core.Geometry, angles, b, niter, block, lam=1.0, x0=None):
    """OS-SART, the ordered-subset form of SART that Section 3.2 runs: the angles, in natural order,
    are cut into consecutive subsets of `block` angles (the last one may be shorter), and each
    subset S makes one update

        W_p = 1/(A_S 1)_p,  V_j = (B_S 1)_j,  x += lam * B_S(W * (b_S - A_S x)) / V

    with the thresholds of `sart`.  block = 1 is SART; block = number of angles is one SIRT step
    per sweep.
    """
    angles = np.asarray(angles, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(geo.vol_shape) if x0 is None else np.array(x0, dtype=np.float64)
    ones_vol = np.ones(geo.vol_shape)
    dmin = min(geo.dVoxel)
    for _ in range(niter):
        for s0 in range(0, len(angles), block):
            th = angles[s0:s0 + block]
            chord = core.siddon_fwd(geo, th, ones_vol)
            W = np.where(chord > SART_RAY_FRACTION * dmin, 1.0 / np.where(chord > 0, chord, 1.0), 0.0)
            r = W * (b[s0:s0 + block] - core.siddon_fwd(geo, th, x))
            num = core.bp(geo, th, r, core.W_FDK)
            V = core.bp(geo, th, np.ones_like(r), core.W_FDK)
            upd = np.where(V > SART_VOXEL_MIN, num / np.where(V > 0, V, 1.0), 0.0)
            x = x + lam * upd
    return x


def tv_grad(x, eps=1e-8):
    """Gradient of TV_eps(x) = sum_j sqrt(|D x_j|^2 + eps) with forward differences on a unit grid
    and zero difference at the last index of each axis (Neumann boundary)."""
    x = np.asarray(x, dtype=np.float64)
    d = [np.zeros_like(x) for _ in range(3)]
    # axes: 2 = x (fastest), 1 = y, 0 = z
    d[0][:, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    d[1][:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    d[2][:-1, :, :] = x[1:, :, :] - x[:-1, :, :]
    n = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + eps)
    g = -(d[0] + d[1] + d[2]) / n
    g[:, :, 1:] += (d[0] / n)[:, :, :-1]
    g[:, 1:, :] += (d[1] / n)[:, :-1, :]
    g[1:, :, :] += (d[2] / n)[:-1, :, :]
    return g


def tv_value(x, eps=1e-8):
    x = np.asarray(x, dtype=np.float64)
    dx = np.zeros_like(x)
    dy = np.zeros_like(x)
    dz = np.zeros_like(x)
    dx[:, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    dy[:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    dz[:-1, :, :] = x[1:, :, :] - x[:-1, :, :]
    return float(np.sum(np.sqrt(dx * dx + dy * dy + dz * dz + eps)))


def tv_steps(x, nsteps, lam, eps=1e-8):
    """Steepest descent on TV (Section 2.3, gradient-descent form): the step length is
    alpha = lam * ||x_in||_2, fixed for the block, and every step moves by alpha along -g/||g||_2
    (the norm of the update is needed at every iteration)."""
    x = np.array(x, dtype=np.float64)
    alpha = lam * float(np.linalg.norm(x.ravel()))
    for _ in range(nsteps):
        g = tv_grad(x, eps)
        ng = float(np.linalg.norm(g.ravel()))
        if ng > 0.0:
            x = x - alpha * g / ng
    return x


def ramp_taps(nu):
    """Band-limited ramp filter (Ram-Lak) sampled at integer offsets m = -(nu-1) .. nu-1, in units
    of 1/ds^2 for detector spacing ds: the inverse discrete-time Fourier transform of |f| cut off at
    the Nyquist frequency (Kak & Slaney, Ch. 3), which is 1/4 at m = 0, 0 at even m and
    -1/(pi m)^2 at odd m.  Returned as an array indexed by m + nu - 1."""
    m = np.arange(-(nu - 1), nu)
    h = np.zeros(2 * nu - 1)
    h[m == 0] = 0.25
    odd = (m % 2) != 0
    h[odd] = -1.0 / (np.pi * m[odd]) ** 2
    return h


def fdk_filter(geo: core.Geometry, angles, proj):
    """Weighting and filtering of the FDK reconstruction (Feldkamp, Davis & Kress 1984; the FDK
    algorithm that Section 2.2's FDK-weighted backprojector serves) for a full circular scan.

    Steps, for every projection and detector row:
      1. cosine weight: each pixel times DSD / |P - S|, with |P - S| = sqrt(DSD^2 + u^2 + v^2) for
         the pixel's detector coordinates (u, v) measured from the central ray;
      2. ramp filter along the row: q[a] = ds * sum_a' h((a - a') ds) p_w[a'] with h the band-limited
         ramp of `ramp_taps` and ds = du * DSO / DSD the pixel spacing scaled to the rotation axis
         (the linear convolution over the whole row, no periodic wrap);
      3. scale by dtheta / 2 with dtheta = 2 pi / N_angles (the 1/2 because every line is measured
         twice over a full turn).
    The reconstruction is then the FDK-weighted backprojection of q, see `fdk`.
    """
    angles = np.asarray(angles, dtype=np.float64)
    if angles.ndim != 1:
        raise ValueError("the FDK reconstruction is defined for a circular orbit: give angles, not views")
    proj = np.asarray(proj, dtype=np.float64)
    nu, nv = geo.nDetector
    du, dv = geo.dDetector
    u = (np.arange(nu) - (nu - 1) / 2.0) * du + geo.offDetector[0]
    v = (np.arange(nv) - (nv - 1) / 2.0) * dv + geo.offDetector[1]
    w = geo.DSD / np.sqrt(geo.DSD ** 2 + u[None, :] ** 2 + v[:, None] ** 2)
    ds = du * geo.DSO / geo.DSD
    h = ramp_taps(nu)
    a = np.arange(nu)
    H = h[a[None, :] - a[:, None] + nu - 1]          # H[a', a] = h(a - a')
    pw = (proj * w[None]).reshape(-1, nu)
    q = (pw @ H) / ds
    dtheta = 2.0 * np.pi / len(angles)
    return (q * (dtheta / 2.0)).reshape(proj.shape)


def fdk(geo: core.Geometry, angles, proj):
    """FDK reconstruction: the FDK-weighted voxel backprojection (weight (DSO/L)^2, Section 2.2) of
    the weighted, filtered projections of `fdk_filter`."""
    return core.bp(geo, angles, fdk_filter(geo, angles, proj), core.W_FDK)


def tv_steps_split(x, nsteps, lam, slab, depth, eps=1e-8, norm="split"):
    """TV steepest descent run split into slabs of `slab` axial slices, each carrying `depth` halo
    slices of its neighbours on either side (Section 2.3's splitting of the TV minimisation).

    Rounds of up to `depth` steps: at the start of a round every slab copies its slices and halo
    from the image as it stands, then takes the round's steps on its own copy.  The gradient at a
    slice needs its neighbours, so a halo slice stops being exact one step after its outer
    neighbour: after `depth` steps the slab's own slices are still exact.  At the end of the round
    each slab's own slices are written back.  alpha = lam ||x_in|| is computed once from the whole
    image.  The norm of each step's gradient is not exchanged between slabs: norm="split"
    approximates ||g||^2 by the slab's own sum scaled by (image slices / slab slices), the uniform
    distribution reading of Section 2.3; norm="global" takes the exact ||g|| of the image (a check
    of the splitting, not a method of the paper).  Axis 0 of x is the slice axis."""
    x = np.array(x, dtype=np.float64)
    nz = x.shape[0]
    alpha = lam * np.sqrt(np.sum(x * x))
    done = 0
    while done < nsteps:
        k = min(depth, nsteps - done)
        start = x.copy()
        if norm == "global":
            # exact steps on the whole image give the global norms the slabs would need
            ref = start.copy()
            gnorm = []
            for _ in range(k):
                g = tv_grad(ref, eps)
                ng = np.sqrt(np.sum(g * g))
                gnorm.append(ng)
                if ng > 0:
                    ref = ref - alpha * g / ng
        for o0 in range(0, nz, slab):
            o1 = min(nz, o0 + slab)
            m0, m1 = max(0, o0 - depth), min(nz, o1 + depth)
            loc = start[m0:m1].copy()
            for i in range(k):
                g = tv_grad(loc, eps)
                if norm == "global":
                    ng = gnorm[i]
                else:
                    own = g[o0 - m0:o1 - m0]
                    ng = np.sqrt(np.sum(own * own) * nz / (o1 - o0))
                if ng > 0:
                    loc = loc - alpha * g / ng
            x[o0:o1] = loc[o0 - m0:o1 - m0]
        done += k
    return x


def rof_chambolle_split(f, lam, niter, slab, depth, tau=1.0 / 12.0, upper_extra=1):
    """Chambolle's ROF iteration (rof_chambolle) run split into slabs of `slab` axial slices that
    carry halo slices of their neighbours (Section 2.3's splitting of the TV minimisers for images
    larger than the device): `depth` below and `depth + upper_extra` above.  Rounds of up to `depth`
    iterations: every slab copies f and p over its slices and halo from the state at the round's
    start, iterates on its copy with the array's ends treated as the image's ends, and writes back
    its own slices of p.  The new p at a slice reads p one slice either side, so a wrong end value
    spoils one more slice per iteration, and at the upper end two in the first (the forward
    difference there reads the slice above the copy): with upper_extra = 1 the slab's own slices
    equal the whole-image iteration after `depth` iterations, and no quantity summed over the image
    is needed.  Then u = f - lam div p from the final p.  Axis 0 of f is the slice axis."""
    f = np.asarray(f, dtype=np.float64)
    nz = f.shape[0]
    p = np.zeros((3,) + f.shape)
    done = 0
    while done < niter:
        k = min(depth, niter - done)
        start = p.copy()
        for o0 in range(0, nz, slab):
            o1 = min(nz, o0 + slab)
            m0, m1 = max(0, o0 - depth), min(nz, o1 + depth + upper_extra)
            loc, fl = start[:, m0:m1].copy(), f[m0:m1]
            for _ in range(k):
                g = grad3(div3(loc) - fl / lam)
                loc = (loc + tau * g) / (1.0 + tau * np.sqrt(np.sum(g * g, axis=0)))
            p[:, o0:o1] = loc[:, o0 - m0:o1 - m0]
        done += k
    return f - lam * div3(p)


def grad3(u):
    """Forward differences on a unit grid along each axis, zero at the last index (the gradient of
    the TV and ROF models); returns an array of shape (3,) + u.shape, axis order of u."""
    u = np.asarray(u, dtype=np.float64)
    g = np.zeros((3,) + u.shape)
    for a in range(3):
        d = np.diff(u, axis=a)
        sl = [slice(None)] * 3
        sl[a] = slice(0, u.shape[a] - 1)
        g[a][tuple(sl)] = d
    return g


def div3(p):
    """Discrete divergence, minus the adjoint of `grad3`: along each axis p_i - p_{i-1} inside,
    p_0 at the first index and -p_{n-2} at the last (Chambolle 2004, Section 2)."""
    p = np.asarray(p, dtype=np.float64)
    out = np.zeros(p.shape[1:])
    for a in range(3):
        q = np.moveaxis(p[a], a, 0)
        n = q.shape[0]
        d = np.zeros_like(q)
        if n == 1:
            d[0] = 0.0
        else:
            d[0] = q[0]
            d[1:n - 1] = q[1:n - 1] - q[0:n - 2]
            d[n - 1] = -q[n - 2]
        out += np.moveaxis(d, 0, a)
    return out


def rof_chambolle(f, lam, niter, tau=1.0 / 12.0):
    """The ROF model min_u ||u - f||^2 / (2 lam) + sum_j |(grad u)_j| (Rudin, Osher & Fatemi 1992,
    the second TV minimiser of Section 2.3), solved by Chambolle's dual projection iteration
    (Chambolle 2004): from p = 0,
        w = div p - f / lam,   p <- (p + tau grad w) / (1 + tau |grad w|),
    and u = f - lam div p.  tau <= 1/12 converges in 3D (||div||^2 <= 12)."""
    f = np.asarray(f, dtype=np.float64)
    p = np.zeros((3,) + f.shape)
    for _ in range(niter):
        g = grad3(div3(p) - f / lam)
        p = (p + tau * g) / (1.0 + tau * np.sqrt(np.sum(g * g, axis=0)))
    return f - lam * div3(p)
