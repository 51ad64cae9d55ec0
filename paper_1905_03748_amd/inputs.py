"""Seeded synthetic inputs for the cone-beam operators: geometries, ellipsoid phantoms, noise.

This module is the only code shared by the GPU path's tests/benchmark and the CPU oracle.  It holds
none of the projector arithmetic: it only draws random numbers, places ellipsoids on a voxel grid by a
point-inside test, integrates ellipsoids analytically along straight lines (a stand-in for a
measured scan), and applies a photon-counting noise model.

The paper's scans (a coffee bean and an Ichthyosaur fossil, Section 3.2) are not available; seeded
random ellipsoid phantoms of the same kind of structure (piecewise-constant, overlapping blobs) stand
in for them.

Recipe (fixed draw order per ellipsoid, numpy ``default_rng(seed)``):
  centre      c = U(-0.4, 0.4)^3 * FOV          (inner 80 % of the field of view, about the volume centre)
  semi-axes   a = U(5, 25)^3 mm
  density     rho = U(0.1, 1)
  rotation    q = N(0,1)^4 / |q|  ->  R(q)      (uniform on SO(3))
Densities add where ellipsoids overlap.  A voxel receives rho when its centre is inside.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Geometry shared by every workload: circular orbit about z, source 1000 mm from the axis,
# detector plane 1500 mm from the source (Section 3 uses scanner distances of this kind).
DSO_MM = 1000.0
DSD_MM = 1500.0


@dataclass
class Workload:
    """Sizes of one synthetic problem (all lengths in mm, angles in radians)."""
    name: str
    nvox: tuple          # (Nx, Ny, Nz)
    dvox: tuple          # voxel size (dx, dy, dz)
    ndet: tuple          # (Nu, Nv)
    ddet: tuple          # pixel size (du, dv)
    n_angles: int
    n_ellipsoids: int
    seed: int
    noise_photons: float = 0.0   # 0 = noiseless
    DSO: float = DSO_MM
    DSD: float = DSD_MM
    off_origin: tuple = (0.0, 0.0, 0.0)
    off_detector: tuple = (0.0, 0.0)
    accuracy: float = 0.5
    angles: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        if self.angles is None:
            self.angles = uniform_angles(self.n_angles)

    @property
    def voxel_proj(self) -> float:
        """Units of work per operator call: Nx*Ny*Nz*N_angles."""
        nx, ny, nz = self.nvox
        return float(nx) * ny * nz * len(self.angles)

    def geometry_dict(self) -> dict:
        return dict(DSO=self.DSO, DSD=self.DSD, nVoxel=tuple(self.nvox), dVoxel=tuple(self.dvox),
                    offOrigin=tuple(self.off_origin), nDetector=tuple(self.ndet),
                    dDetector=tuple(self.ddet), offDetector=tuple(self.off_detector),
                    accuracy=self.accuracy)


def uniform_angles(n: int) -> np.ndarray:
    """n angles uniform over a full turn, endpoint excluded: theta_k = 2*pi*k/n."""
    return 2.0 * np.pi * np.arange(n, dtype=np.float64) / n


def _rot(axis: np.ndarray, ang: float) -> np.ndarray:
    """Rotation matrix about a unit axis (Rodrigues)."""
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + np.sin(ang) * K + (1.0 - np.cos(ang)) * (K @ K)


def helical_views(DSO: float, DSD: float, angles, pitch: float, z0: float = 0.0) -> np.ndarray:
    """Per-view table (n x 12: source, detector centre, unit e_u, unit e_v, mm) of a helical scan:
    the circular orbit's views with source and detector centre raised by z0 + pitch * theta / (2 pi)
    (pitch in mm per turn)."""
    th = np.asarray(angles, dtype=np.float64)
    c, s = np.cos(th), np.sin(th)
    z = z0 + pitch * th / (2.0 * np.pi)
    k = -(DSD - DSO)
    zero, one = np.zeros_like(th), np.ones_like(th)
    return np.stack([DSO * c, DSO * s, z, k * c, k * s, z, -s, c, zero, zero, zero, one], -1)


def carm_views(DSO: float, DSD: float, angles, seed: int, tilt_deg: float = 15.0, jitter_mm: float = 5.0,
               orbit_tilt_deg: float = 0.0) -> np.ndarray:
    """Per-view table (n x 12) of a C-arm-like scan: the circular orbit, tilted about the x axis by
    orbit_tilt_deg, with each view's source and detector centre displaced by seeded offsets of up to
    jitter_mm per axis and its detector turned about its centre by seeded rotations of up to
    tilt_deg about e_u, e_v and the normal, in that order (e_u, e_v stay orthonormal)."""
    th = np.asarray(angles, dtype=np.float64)
    rng = np.random.default_rng(seed)
    R0 = _rot(np.array([1.0, 0.0, 0.0]), np.deg2rad(orbit_tilt_deg))
    out = np.zeros((len(th), 12))
    for t, a in enumerate(th):
        c, s = np.cos(a), np.sin(a)
        S = R0 @ np.array([DSO * c, DSO * s, 0.0])
        C = R0 @ np.array([-(DSD - DSO) * c, -(DSD - DSO) * s, 0.0])
        eu = R0 @ np.array([-s, c, 0.0])
        ev = R0 @ np.array([0.0, 0.0, 1.0])
        S = S + rng.uniform(-jitter_mm, jitter_mm, 3)
        C = C + rng.uniform(-jitter_mm, jitter_mm, 3)
        ang = np.deg2rad(rng.uniform(-tilt_deg, tilt_deg, 3))
        for axis, phi in ((eu, ang[0]), (ev, ang[1]), (np.cross(eu, ev), ang[2])):
            R = _rot(axis, phi)
            eu, ev = R @ eu, R @ ev
        out[t] = np.concatenate([S, C, eu, ev])
    return out


def workload(name: str, **over) -> Workload:
    """The named synthetic problems.

    tiny        64^3 of 1 mm, 64 angles, 64^2 detector of 1.6 mm, 10 ellipsoids, seed 1
    medium      512^3 of 0.5 mm, 360 angles, 512^2 detector of 0.8 mm, 40 ellipsoids, seed 2,
                Poisson noise at 1e5 photons per ray
    ooc         3072^3 of 256/3072 mm, 3072 angles, 3072^2 detector of 0.8*512/3072 mm, 200 ellipsoids
    precision   1024^3 of 0.25 mm, 720 angles, 1024^2 detector of 0.4 mm, 40 ellipsoids, seed 4
    autograd    128^3 of 2 mm, 90 angles, 128^2 detector of 3.2 mm, seed 5
    serve_N     N^3 of 256/N mm, N^2 detector of 409.6/N mm (angle count given by the caller)
    """
    if name == "tiny":
        w = Workload("tiny", (64, 64, 64), (1.0, 1.0, 1.0), (64, 64), (1.6, 1.6), 64, 10, 1)
    elif name == "medium":
        w = Workload("medium", (512, 512, 512), (0.5, 0.5, 0.5), (512, 512), (0.8, 0.8), 360, 40, 2,
                     noise_photons=1e5)
    elif name == "ooc":
        d = 256.0 / 3072
        p = 0.8 * 512 / 3072
        w = Workload("ooc", (3072, 3072, 3072), (d, d, d), (3072, 3072), (p, p), 3072, 200, 3)
    elif name == "precision":
        w = Workload("precision", (1024, 1024, 1024), (0.25, 0.25, 0.25), (1024, 1024), (0.4, 0.4),
                     720, 40, 4)
    elif name == "autograd":
        w = Workload("autograd", (128, 128, 128), (2.0, 2.0, 2.0), (128, 128), (3.2, 3.2), 90, 40, 5)
    elif name.startswith("serve_"):
        n = int(name.split("_")[1])
        n_angles = over.pop("n_angles", 90)
        seed = over.pop("seed", 1000)
        w = Workload(name, (n, n, n), (256.0 / n,) * 3, (n, n), (409.6 / n,) * 2, n_angles, 40, seed)
    else:
        raise KeyError(name)
    for k, v in over.items():
        setattr(w, k, v)
    if "n_angles" in over and "angles" not in over:
        w.angles = uniform_angles(w.n_angles)
    return w


def scaled_workload(base: Workload, nvox, ndet, n_angles, name=None, **over) -> Workload:
    """Same field of view and detector extent as ``base`` at another sampling (for small cases)."""
    fov = [n * d for n, d in zip(base.nvox, base.dvox)]
    det = [n * d for n, d in zip(base.ndet, base.ddet)]
    w = Workload(name or base.name + "_scaled", tuple(nvox), tuple(f / n for f, n in zip(fov, nvox)),
                 tuple(ndet), tuple(e / n for e, n in zip(det, ndet)), n_angles, base.n_ellipsoids,
                 base.seed, base.noise_photons, base.DSO, base.DSD, base.off_origin, base.off_detector,
                 base.accuracy)
    for k, v in over.items():
        setattr(w, k, v)
    return w


@dataclass
class Ellipsoid:
    centre: np.ndarray      # (3,) mm, absolute coordinates
    semi: np.ndarray        # (3,) mm
    rho: float
    R: np.ndarray           # (3,3) rotation: body axes are the columns


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoids(w: Workload, n: int | None = None, seed: int | None = None) -> list[Ellipsoid]:
    """Draw the phantom's ellipsoids in the fixed order documented at the top of this module."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    fov = np.array([nv * dv for nv, dv in zip(w.nvox, w.dvox)])
    out = []
    for _ in range(w.n_ellipsoids if n is None else n):
        c = rng.uniform(-0.4, 0.4, 3) * fov + np.asarray(w.off_origin)
        a = rng.uniform(5.0, 25.0, 3)
        rho = float(rng.uniform(0.1, 1.0))
        q = rng.normal(0.0, 1.0, 4)
        q /= np.linalg.norm(q)
        out.append(Ellipsoid(c, a, rho, _quat_to_rot(q)))
    return out


def voxel_centres_1d(n: int, d: float, off: float) -> np.ndarray:
    return off + (np.arange(n) - (n - 1) / 2.0) * d


def voxelize(w: Workload, ells: list[Ellipsoid] | None = None, dtype=np.float32, supersample: int = 1):
    """Phantom volume laid out [z][y][x] (x fastest).  A voxel (or sub-sample) gets rho if inside."""
    if ells is None:
        ells = ellipsoids(w)
    nx, ny, nz = w.nvox
    dx, dy, dz = w.dvox
    ox, oy, oz = w.off_origin
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    ss = supersample
    sub = (np.arange(ss) - (ss - 1) / 2.0) / ss
    for e in ells:
        r = float(np.max(e.semi))
        lo = [int(max(0, math.floor((e.centre[i] - r - o) / d + (n - 1) / 2.0)))
              for i, (n, d, o) in enumerate(zip((nx, ny, nz), (dx, dy, dz), (ox, oy, oz)))]
        hi = [int(min(n - 1, math.ceil((e.centre[i] + r - o) / d + (n - 1) / 2.0)))
              for i, (n, d, o) in enumerate(zip((nx, ny, nz), (dx, dy, dz), (ox, oy, oz)))]
        if any(h < l for l, h in zip(lo, hi)):
            continue
        xs = voxel_centres_1d(nx, dx, ox)[lo[0]:hi[0] + 1]
        ys = voxel_centres_1d(ny, dy, oy)[lo[1]:hi[1] + 1]
        zs = voxel_centres_1d(nz, dz, oz)[lo[2]:hi[2] + 1]
        Rt = e.R.T / e.semi[:, None]
        acc = np.zeros((len(zs), len(ys), len(xs)))
        for sz in sub:
            for sy in sub:
                for sx in sub:
                    Z, Y, X = np.meshgrid(zs + sz * dz - e.centre[2], ys + sy * dy - e.centre[1],
                                          xs + sx * dx - e.centre[0], indexing="ij")
                    q0 = Rt[0, 0] * X + Rt[0, 1] * Y + Rt[0, 2] * Z
                    q1 = Rt[1, 0] * X + Rt[1, 1] * Y + Rt[1, 2] * Z
                    q2 = Rt[2, 0] * X + Rt[2, 1] * Y + Rt[2, 2] * Z
                    acc += (q0 * q0 + q1 * q1 + q2 * q2 <= 1.0)
        vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += e.rho * acc / ss ** 3
    return vol.astype(dtype)


def ray_endpoints(w: Workload, theta: np.ndarray, a: np.ndarray, b: np.ndarray):
    """Source and pixel-centre positions (mm) for pixel (a, b) at angle theta (arrays broadcast).

    Source S = DSO (cos, sin, 0); detector centre C = -(DSD - DSO)(cos, sin, 0);
    e_u = (-sin, cos, 0), e_v = (0, 0, 1); pixel centre at C + u_a e_u + v_b e_v.
    """
    th = np.asarray(theta, dtype=np.float64)
    c, s = np.cos(th), np.sin(th)
    nu, nv = w.ndet
    du, dv = w.ddet
    u = (np.asarray(a) - (nu - 1) / 2.0) * du + w.off_detector[0]
    v = (np.asarray(b) - (nv - 1) / 2.0) * dv + w.off_detector[1]
    S = np.stack(np.broadcast_arrays(w.DSO * c, w.DSO * s, 0.0 * c), -1)
    k = -(w.DSD - w.DSO)
    P = np.stack(np.broadcast_arrays(k * c - u * s, k * s + u * c, v + 0.0 * c), -1)
    return S, P


def ellipsoid_line_integrals(S: np.ndarray, P: np.ndarray, ells: list[Ellipsoid],
                             box: tuple | None = None) -> np.ndarray:
    """Sum over ellipsoids of rho * (length of segment S->P inside the ellipsoid [and the box]).

    ``box`` = (lo[3], hi[3]) restricts each chord to that axis-aligned box (the voxel grid's extent),
    which is what a voxelised phantom clipped to the grid integrates to in the limit of fine voxels.
    """
    S = np.asarray(S, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    D = P - S
    L = np.linalg.norm(D, axis=-1)
    t_lo = np.zeros(L.shape)
    t_hi = np.ones(L.shape)
    if box is not None:
        lo, hi = box
        for ax in range(3):
            d = D[..., ax]
            with np.errstate(divide="ignore", invalid="ignore"):
                ta = (lo[ax] - S[..., ax]) / d
                tb = (hi[ax] - S[..., ax]) / d
            par = np.abs(d) < 1e-12 * L
            inside = (S[..., ax] >= lo[ax]) & (S[..., ax] <= hi[ax])
            t0 = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(ta, tb))
            t1 = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(ta, tb))
            t_lo = np.maximum(t_lo, t0)
            t_hi = np.minimum(t_hi, t1)
    out = np.zeros(L.shape)
    for e in ells:
        M = e.R.T / e.semi[:, None]
        p0 = (S - e.centre) @ M.T
        dd = D @ M.T
        A = np.sum(dd * dd, -1)
        B = 2.0 * np.sum(p0 * dd, -1)
        C = np.sum(p0 * p0, -1) - 1.0
        disc = B * B - 4 * A * C
        ok = disc > 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t1 = (-B - sq) / (2 * A)
        t2 = (-B + sq) / (2 * A)
        a_ = np.maximum(t1, t_lo)
        b_ = np.minimum(t2, t_hi)
        out += e.rho * L * np.where(ok, np.maximum(b_ - a_, 0.0), 0.0)
    return out


def analytic_projections(w: Workload, ells: list[Ellipsoid] | None = None, clip_to_grid=True,
                         angle_slice=slice(None), dtype=np.float32) -> np.ndarray:
    """Exact line integrals of the continuous phantom for every pixel: array [theta][v][u]."""
    if ells is None:
        ells = ellipsoids(w)
    nu, nv = w.ndet
    box = None
    if clip_to_grid:
        lo = [o - n * d / 2.0 for n, d, o in zip(w.nvox, w.dvox, w.off_origin)]
        hi = [o + n * d / 2.0 for n, d, o in zip(w.nvox, w.dvox, w.off_origin)]
        box = (lo, hi)
    angles = np.asarray(w.angles)[angle_slice]
    out = np.zeros((len(angles), nv, nu), dtype=dtype)
    bb, aa = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    for i, th in enumerate(angles):
        S, P = ray_endpoints(w, th, aa, bb)
        out[i] = ellipsoid_line_integrals(S, P, ells, box)
    return out


def add_poisson_noise(proj: np.ndarray, photons: float, seed: int) -> np.ndarray:
    """Photon-counting noise: densities are read as attenuation in 1/cm and lengths in mm, so the
    line integral in optical depth is p/10; counts n ~ Poisson(I0 exp(-p/10)), n >= 1, and the noisy
    line integral is -10 ln(n / I0)."""
    rng = np.random.default_rng(seed)
    p = np.asarray(proj, dtype=np.float64) / 10.0
    n = rng.poisson(photons * np.exp(-p)).astype(np.float64)
    n = np.maximum(n, 1.0)
    return (-10.0 * np.log(n / photons)).astype(proj.dtype)


def random_array(shape, seed: int, dtype=np.float32, kind="normal") -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(shape).astype(dtype)
    return rng.uniform(0.0, 1.0, shape).astype(dtype)


def sample_indices(n_total: int, n: int, seed: int) -> np.ndarray:
    """Seeded distinct flat indices, sorted."""
    rng = np.random.default_rng(seed)
    n = min(n, n_total)
    return np.sort(rng.choice(n_total, size=n, replace=False)).astype(np.int64)


def voxelize_torch(w: Workload, ells: list[Ellipsoid] | None = None, device="cpu"):
    """Same recipe as ``voxelize`` (centre-inside test, densities add), evaluated with torch on
    ``device`` one ellipsoid bounding box at a time; FP32 result [z][y][x]."""
    import torch
    if ells is None:
        ells = ellipsoids(w)
    nx, ny, nz = w.nvox
    dx, dy, dz = w.dvox
    ox, oy, oz = w.off_origin
    vol = torch.zeros((nz, ny, nx), dtype=torch.float32, device=device)
    cx = torch.tensor(voxel_centres_1d(nx, dx, ox), dtype=torch.float64, device=device)
    cy = torch.tensor(voxel_centres_1d(ny, dy, oy), dtype=torch.float64, device=device)
    cz = torch.tensor(voxel_centres_1d(nz, dz, oz), dtype=torch.float64, device=device)
    for e in ells:
        r = float(np.max(e.semi))
        lo, hi = [], []
        for i, (n, d, o) in enumerate(zip((nx, ny, nz), (dx, dy, dz), (ox, oy, oz))):
            lo.append(int(max(0, math.floor((e.centre[i] - r - o) / d + (n - 1) / 2.0))))
            hi.append(int(min(n - 1, math.ceil((e.centre[i] + r - o) / d + (n - 1) / 2.0))))
        if any(h < l for l, h in zip(lo, hi)):
            continue
        Rt = torch.tensor(e.R.T / e.semi[:, None], dtype=torch.float64, device=device)
        Z = (cz[lo[2]:hi[2] + 1] - e.centre[2])[:, None, None]
        Y = (cy[lo[1]:hi[1] + 1] - e.centre[1])[None, :, None]
        X = (cx[lo[0]:hi[0] + 1] - e.centre[0])[None, None, :]
        q0 = Rt[0, 0] * X + Rt[0, 1] * Y + Rt[0, 2] * Z
        q1 = Rt[1, 0] * X + Rt[1, 1] * Y + Rt[1, 2] * Z
        q2 = Rt[2, 0] * X + Rt[2, 1] * Y + Rt[2, 2] * Z
        inside = (q0 * q0 + q1 * q1 + q2 * q2 <= 1.0).to(torch.float32)
        vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += float(e.rho) * inside
    return vol
