// Ray-driven forward projectors (Section 2.1): one thread per detector pixel.
//
// Rays are set up in FP64 in voxel-index space (the source is ~DSO/d voxels from the grid, so an
// FP32 set-up would misplace rays by ~1e-4 voxel), clipped to the grid (or to a z-slab of it for
// the out-of-core schedule), and then traversed in FP32 relative to the entry voxel, where all
// quantities are O(grid size) and plane crossings are formed as t0 + n * dt by one FMA each.
//
// Launch shape: 256-thread blocks covering 64 pixels along u (one wave = 64 adjacent pixels of
// one detector row, whose rays are nearly parallel and walk neighbouring voxels in lock-step) by
// 4 rows.  Blocks are linearised as (u-tile fastest, then angle, then v-band) so the blocks in
// flight at any moment share a band of detector rows across many angles, i.e. an axial slab of
// the volume, which keeps the working set inside the 256 MB last-level cache.
#include <cfloat>
#include <cmath>

#include "dev_common.hpp"

namespace ct {

namespace {

constexpr int FWD_TU = 64;  // pixels per block along u
constexpr int FWD_TV = 4;   // rows per block

struct FwdArgs {
    const AngleGeo *tab;
    int64_t a0;
    int32_t nang;
    int32_t nx, ny, nz;
    double dx, dy, dz;
    int32_t nu, nv;
    double du, dv, cu, cv, offu, offv;
    int32_t own_lo, own_hi;  // owned slices [own_lo, own_hi)
    int32_t mem_lo, mem_n;   // slices held in memory, starting at the volume pointer
    int32_t first, last;     // interpolated projector: extend ownership to -inf / +inf
    int32_t accumulate;
    double delta;            // interpolated projector sample spacing (mm)
    int32_t ublocks;
};

struct RaySetup {
    double D[3];   // direction, index units per unit t (t in [0,1] from source to pixel)
    double L;      // mm per unit t (= |pixel - source|)
    double t0, t1; // clip interval
    bool par[3];
};

// Direction of the ray through pixel (a, b) and its clip against the box [lo, hi] (index space).
__device__ __forceinline__ bool ray_clip(const AngleGeo &G, const FwdArgs &A, int a, int b, const double lo[3],
                                         const double hi[3], RaySetup &R) {
    const double ua = (a - A.cu) * A.du + A.offu;
    const double vb = (b - A.cv) * A.dv + A.offv;
    R.D[0] = G.Dc[0] + ua * G.eu[0];
    R.D[1] = G.Dc[1] + ua * G.eu[1];
    R.D[2] = vb / A.dz;
    const double m0 = R.D[0] * A.dx, m1 = R.D[1] * A.dy, m2 = R.D[2] * A.dz;
    R.L = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
    const double mm[3] = {m0, m1, m2};
    double t0 = 0.0, t1 = 1.0;
    bool hit = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        R.par[ax] = fabs(mm[ax]) < 1e-12 * R.L;
        if (R.par[ax]) {
            if (G.S[ax] < lo[ax] || G.S[ax] > hi[ax]) hit = false;
        } else {
            const double ta = (lo[ax] - G.S[ax]) / R.D[ax];
            const double tb = (hi[ax] - G.S[ax]) / R.D[ax];
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        }
    }
    R.t0 = t0;
    R.t1 = t1;
    return hit && t0 < t1;
}

__device__ __forceinline__ void pixel_of(const FwdArgs &A, int &ai, int &a, int &b) {
    const int bid = blockIdx.x;
    const int ub = bid % A.ublocks;
    const int rest = bid / A.ublocks;
    ai = rest % A.nang;
    const int vb = rest / A.nang;
    a = ub * FWD_TU + (threadIdx.x & (FWD_TU - 1));
    b = vb * FWD_TV + (threadIdx.x / FWD_TU);
}

// ------------------------------------------------------------------------------------------
// Siddon: exact length of the ray inside each voxel it crosses (incremental traversal in the
// manner of Jacobs et al. 1998: step to whichever voxel plane comes next).

template <typename TV>
__device__ __forceinline__ float siddon_ray(const TV *__restrict__ vol, const FwdArgs &A, const AngleGeo &G,
                                            int a, int b) {
    const double lo[3] = {-0.5, -0.5, A.own_lo - 0.5};
    const double hi[3] = {A.nx - 0.5, A.ny - 0.5, A.own_hi - 0.5};
    RaySetup R;
    if (!ray_clip(G, A, a, b, lo, hi, R)) return 0.0f;

    const int ilo[3] = {0, 0, A.own_lo};
    const int ihi[3] = {A.nx - 1, A.ny - 1, A.own_hi - 1};
    int idx[3], step[3];
    float tn0[3], dtn[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double E = G.S[ax] + R.t0 * R.D[ax];
        int i = (int)floor(E + 0.5);
        i = i < ilo[ax] ? ilo[ax] : (i > ihi[ax] ? ihi[ax] : i);
        idx[ax] = i;
        if (R.par[ax]) {
            step[ax] = 0;
            tn0[ax] = FLT_MAX;
            dtn[ax] = 0.0f;
        } else {
            const double f = E - i;  // entry offset from the voxel centre, about [-0.5, 0.5]
            const int s = R.D[ax] > 0 ? 1 : -1;
            const double inv = 1.0 / fabs(R.D[ax]);
            step[ax] = s;
            tn0[ax] = (float)((0.5 - s * f) * inv);
            dtn[ax] = (float)inv;
        }
    }
    const float T = (float)(R.t1 - R.t0);
    const int64_t sy = A.nx, sz = (int64_t)A.nx * A.ny;
    int64_t lin = (int64_t)(idx[2] - A.mem_lo) * sz + (int64_t)idx[1] * sy + idx[0];
    const int64_t st0 = step[0], st1 = step[1] * sy, st2 = step[2] * sz;
    int ix = idx[0], iy = idx[1], iz = idx[2];
    const unsigned nzown = (unsigned)(A.own_hi - A.own_lo);
    float tx = tn0[0], ty = tn0[1], tz = tn0[2];
    int n0 = 0, n1 = 0, n2 = 0;
    float tc = 0.0f, acc = 0.0f;
    const int maxit = A.nx + A.ny + (A.own_hi - A.own_lo) + 4;
    for (int it = 0; it < maxit; ++it) {
        const float tn = fminf(fminf(tx, ty), fminf(tz, T));
        acc = fmaf(tn - tc, ldf(vol, lin), acc);
        if (tn >= T) break;
        tc = tn;
        if (tx <= ty && tx <= tz) {
            ix += step[0];
            if ((unsigned)ix >= (unsigned)A.nx) break;
            lin += st0;
            ++n0;
            tx = fmaf((float)n0, dtn[0], tn0[0]);
        } else if (ty <= tz) {
            iy += step[1];
            if ((unsigned)iy >= (unsigned)A.ny) break;
            lin += st1;
            ++n1;
            ty = fmaf((float)n1, dtn[1], tn0[1]);
        } else {
            iz += step[2];
            if ((unsigned)(iz - A.own_lo) >= nzown) break;
            lin += st2;
            ++n2;
            tz = fmaf((float)n2, dtn[2], tn0[2]);
        }
    }
    return (float)(acc * R.L);
}

template <typename TV, typename TP>
__global__ __launch_bounds__(256) void k_siddon(const TV *__restrict__ vol, TP *__restrict__ proj, FwdArgs A) {
    int ai, a, b;
    pixel_of(A, ai, a, b);
    if (a >= A.nu || b >= A.nv) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    const float v = siddon_ray(vol, A, G, a, b);
    const int64_t o = ((int64_t)ai * A.nv + b) * A.nu + a;
    const float prev = A.accumulate ? to_f(proj[o]) : 0.0f;
    proj[o] = from_f<TP>(prev + v);
}

// ------------------------------------------------------------------------------------------
// Interpolated projector: samples at s_k = (k + 1/2) delta mm from the source, every k whose
// sample lies in the grid box grown by half a voxel (outside it the zero-padded trilinear
// interpolant vanishes); p = delta * sum of the interpolant at the samples.

template <typename TV>
__device__ __forceinline__ float vox(const TV *__restrict__ vol, const FwdArgs &A, int x, int y, int z) {
    const bool ok = (unsigned)x < (unsigned)A.nx && (unsigned)y < (unsigned)A.ny &&
                    (unsigned)(z - A.mem_lo) < (unsigned)A.mem_n;
    const int xc = ok ? x : 0, yc = ok ? y : 0, zc = ok ? z - A.mem_lo : 0;
    const float v = ldf(vol, ((int64_t)zc * A.ny + yc) * A.nx + xc);
    return ok ? v : 0.0f;
}

template <typename TV>
__device__ __forceinline__ float interp_ray(const TV *__restrict__ vol, const FwdArgs &A, const AngleGeo &G,
                                            int a, int b) {
    const double lo[3] = {-1.0, -1.0, -1.0};
    const double hi[3] = {(double)A.nx, (double)A.ny, (double)A.nz};
    RaySetup R;
    if (!ray_clip(G, A, a, b, lo, hi, R)) return 0.0f;
    const double s_in = R.t0 * R.L, s_out = R.t1 * R.L;
    const double k0 = ceil(s_in / A.delta - 0.5);
    const double k1 = floor(s_out / A.delta - 0.5);
    if (k1 < k0) return 0.0f;
    const double tk0 = (k0 + 0.5) * A.delta / R.L;
    const double dt = A.delta / R.L;
    double B[3], stp[3];
    int ib[3];
    float fb[3], fs[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        B[ax] = G.S[ax] + tk0 * R.D[ax];
        stp[ax] = dt * R.D[ax];
        ib[ax] = (int)floor(B[ax]);
        fb[ax] = (float)(B[ax] - ib[ax]);
        fs[ax] = (float)stp[ax];
    }
    int jlo = 0, jhi = (int)(k1 - k0);
    float zlo = -FLT_MAX, zhi = FLT_MAX;
    const bool slab = !(A.first && A.last);
    if (slab) {
        zlo = A.first ? -FLT_MAX : (float)(A.own_lo - 0.5 - ib[2]);
        zhi = A.last ? FLT_MAX : (float)(A.own_hi - 0.5 - ib[2]);
        // samples whose z (relative to ib[2]) lies in [zlo, zhi), with a margin; the exact test
        // below is the same FP32 expression in every slab, so each sample has one owner
        if (!R.par[2] && fabs(stp[2]) > 0.0) {
            const double za = A.first ? -1e30 : (A.own_lo - 0.5 - B[2]) / stp[2];
            const double zb = A.last ? 1e30 : (A.own_hi - 0.5 - B[2]) / stp[2];
            const double j0 = floor(fmin(za, zb)) - 2, j1 = ceil(fmax(za, zb)) + 2;
            jlo = (int)fmax((double)jlo, j0);
            jhi = (int)fmin((double)jhi, j1);
        }
    }
    float acc = 0.0f;
    for (int j = jlo; j <= jhi; ++j) {
        const float px = fmaf((float)j, fs[0], fb[0]);
        const float py = fmaf((float)j, fs[1], fb[1]);
        const float pz = fmaf((float)j, fs[2], fb[2]);
        if (slab && !(pz >= zlo && pz < zhi)) continue;
        const float flx = floorf(px), fly = floorf(py), flz = floorf(pz);
        const float rx = px - flx, ry = py - fly, rz = pz - flz;
        const int x0 = ib[0] + (int)flx, y0 = ib[1] + (int)fly, z0 = ib[2] + (int)flz;
        const float c00 = fmaf(rx, vox(vol, A, x0 + 1, y0, z0) - vox(vol, A, x0, y0, z0), vox(vol, A, x0, y0, z0));
        const float c10 = fmaf(rx, vox(vol, A, x0 + 1, y0 + 1, z0) - vox(vol, A, x0, y0 + 1, z0),
                               vox(vol, A, x0, y0 + 1, z0));
        const float c01 = fmaf(rx, vox(vol, A, x0 + 1, y0, z0 + 1) - vox(vol, A, x0, y0, z0 + 1),
                               vox(vol, A, x0, y0, z0 + 1));
        const float c11 = fmaf(rx, vox(vol, A, x0 + 1, y0 + 1, z0 + 1) - vox(vol, A, x0, y0 + 1, z0 + 1),
                               vox(vol, A, x0, y0 + 1, z0 + 1));
        const float c0 = fmaf(ry, c10 - c00, c00);
        const float c1 = fmaf(ry, c11 - c01, c01);
        acc += fmaf(rz, c1 - c0, c0);
    }
    return (float)(acc * A.delta);
}

template <typename TV, typename TP>
__global__ __launch_bounds__(256) void k_interp(const TV *__restrict__ vol, TP *__restrict__ proj, FwdArgs A) {
    int ai, a, b;
    pixel_of(A, ai, a, b);
    if (a >= A.nu || b >= A.nv) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    const float v = interp_ray(vol, A, G, a, b);
    const int64_t o = ((int64_t)ai * A.nv + b) * A.nu + a;
    const float prev = A.accumulate ? to_f(proj[o]) : 0.0f;
    proj[o] = from_f<TP>(prev + v);
}

// Chord of each ray through the whole grid box (= A 1 of the Siddon projector), FP64 set-up.
__global__ __launch_bounds__(256) void k_ray_chord(float *__restrict__ chord, FwdArgs A) {
    int ai, a, b;
    pixel_of(A, ai, a, b);
    if (a >= A.nu || b >= A.nv) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    const double lo[3] = {-0.5, -0.5, -0.5};
    const double hi[3] = {A.nx - 0.5, A.ny - 0.5, A.nz - 0.5};
    RaySetup R;
    const float c = ray_clip(G, A, a, b, lo, hi, R) ? (float)((R.t1 - R.t0) * R.L) : 0.0f;
    chord[((int64_t)ai * A.nv + b) * A.nu + a] = c;
}

FwdArgs make_args(ct_plan *p, const AngleGeo *tab, int64_t a0, int64_t a1, const Slab &slab, int accumulate) {
    const ct_geometry &g = p->g;
    FwdArgs A;
    A.tab = tab;
    A.a0 = a0;
    A.nang = (int32_t)(a1 - a0);
    A.nx = (int32_t)g.nVoxel[0];
    A.ny = (int32_t)g.nVoxel[1];
    A.nz = (int32_t)g.nVoxel[2];
    A.dx = g.dVoxel[0];
    A.dy = g.dVoxel[1];
    A.dz = g.dVoxel[2];
    A.nu = (int32_t)g.nDetector[0];
    A.nv = (int32_t)g.nDetector[1];
    A.du = g.dDetector[0];
    A.dv = g.dDetector[1];
    A.cu = (A.nu - 1) / 2.0;
    A.cv = (A.nv - 1) / 2.0;
    A.offu = g.offDetector[0];
    A.offv = g.offDetector[1];
    A.own_lo = (int32_t)slab.own_lo;
    A.own_hi = (int32_t)slab.own_hi;
    A.mem_lo = (int32_t)slab.mem_lo;
    A.mem_n = (int32_t)slab.mem_n;
    A.first = slab.first;
    A.last = slab.last;
    A.accumulate = accumulate;
    A.delta = g.accuracy * fmin(g.dVoxel[0], fmin(g.dVoxel[1], g.dVoxel[2]));
    A.ublocks = (A.nu + FWD_TU - 1) / FWD_TU;
    return A;
}

unsigned fwd_grid(const FwdArgs &A) {
    const int64_t vb = (A.nv + FWD_TV - 1) / FWD_TV;
    return (unsigned)((int64_t)A.ublocks * A.nang * vb);
}

}  // namespace

ct_status launch_forward(ct_plan *p, ct_projector kind, const void *vol, ct_dtype vt, void *proj, ct_dtype pt,
                         int accumulate, int64_t a0, int64_t a1, const Slab &slab, hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    if (slab.own_hi <= slab.own_lo) return CT_OK;
    // launch in pieces of at most 2^30 blocks' worth of angles
    const int64_t vb = (p->g.nDetector[1] + FWD_TV - 1) / FWD_TV;
    const int64_t ub = (p->g.nDetector[0] + FWD_TU - 1) / FWD_TU;
    const int64_t max_ang = std::max<int64_t>(1, (int64_t(1) << 30) / (vb * ub));
    const size_t proj_angle = (size_t)p->g.nDetector[0] * p->g.nDetector[1] * dtype_size(pt);
    for (int64_t c0 = a0; c0 < a1; c0 += max_ang) {
        const int64_t c1 = std::min(a1, c0 + max_ang);
        FwdArgs A = make_args(p, tab, c0, c1, slab, accumulate);
        char *pp = (char *)proj + (size_t)(c0 - a0) * proj_angle;
        const dim3 grid(fwd_grid(A)), block(256);
        if (kind == CT_SIDDON) {
            CT_DISPATCH2(vt, TV, pt, TP,
                         hipLaunchKernelGGL((k_siddon<TV, TP>), grid, block, 0, st, (const TV *)vol, (TP *)pp, A));
        } else {
            CT_DISPATCH2(vt, TV, pt, TP,
                         hipLaunchKernelGGL((k_interp<TV, TP>), grid, block, 0, st, (const TV *)vol, (TP *)pp, A));
        }
        CT_HIP(hipGetLastError());
    }
    return CT_OK;
}

ct_status launch_ray_chord(ct_plan *p, float *chord, int64_t a0, int64_t a1, hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    FwdArgs A = make_args(p, tab, a0, a1, full_slab(p->g), 0);
    hipLaunchKernelGGL(k_ray_chord, dim3(fwd_grid(A)), dim3(256), 0, st, chord, A);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

}  // namespace ct
