// Voxel-driven backprojectors (Section 2.2): one thread per (x, y) voxel column and a run of BP_NZ
// consecutive z voxels, looping over the angles of the launch with the BP_NZ sums in registers.
//
// In a circular orbit every voxel of a column has the same depth L, magnification and detector
// column coordinate a*, so the per-angle set-up (one reciprocal, the FDK weight, the u bilinear
// weights) is done once per column and only the row coordinate b* steps along z.  Lanes of a wave
// hold an 16 x 4 patch of columns whose projections fall on a few neighbouring detector pixels of
// the same rows, so the four bilinear taps of a wave touch one or two cache lines.
//
// The exact adjoint of the Siddon projector gathers, for each voxel, every ray that crosses its
// box: the rays of detector column a all lie in one vertical plane, so their (x, y) traces are the
// same line and the parameter interval [t0, t1] inside the voxel column's square is shared by all
// rows b and all voxels of the column; only the z overlap depends on the row and the voxel.
#include <cfloat>
#include <cmath>

#include "dev_common.hpp"

namespace ct {

namespace {

constexpr int BP_TX = 16, BP_TY = 16;
constexpr int BP_NZ = 8;

struct BpArgs {
    const AngleGeo *tab;
    int64_t a0;
    int32_t nang;
    int32_t nx, ny, nz;
    float dx, dy, dz;
    float x0, y0, z0;       // centre of voxel (0, 0, 0), mm
    int32_t nu, nv;
    float inv_du, inv_dv;
    float au0, bv0;         // a* = u * inv_du + au0, b* = v * inv_dv + bv0
    float DSO, DSD;
    float pm_const;         // dx dy dz / (du dv) * DSD^2
    int32_t own_lo, own_hi; // voxels written: k in [own_lo, own_hi)
    int32_t mem_lo;         // slice at the volume pointer
    int32_t accumulate;
    // exact adjoint (FP64 set-up)
    double ddx, ddy, ddz, dx0, dy0, dz0;
    double dDSO, dDSD, du, dv, cu, cv, offu, offv;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int W, typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_voxel(const TP *__restrict__ proj, TV *__restrict__ vol, BpArgs A) {
    const int i = blockIdx.x * BP_TX + (threadIdx.x % BP_TX);
    const int j = blockIdx.y * BP_TY + (threadIdx.x / BP_TX);
    const int kb = A.own_lo + blockIdx.z * BP_NZ;
    if (i >= A.nx || j >= A.ny) return;
    const float x = fmaf((float)i, A.dx, A.x0);
    const float y = fmaf((float)j, A.dy, A.y0);
    const float zb = fmaf((float)kb, A.dz, A.z0);
    float acc[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) acc[k] = 0.0f;
    const int64_t psz = (int64_t)A.nu * A.nv;
    for (int t = 0; t < A.nang; ++t) {
        const AngleGeo &G = A.tab[A.a0 + t];
        const float c = (float)G.c, s = (float)G.s;
        const float Ld = A.DSO - (x * c + y * s);
        const float iL = 1.0f / Ld;
        const float m = A.DSD * iL;
        const float as = fmaf(m * (y * c - x * s), A.inv_du, A.au0);
        const float af = floorf(as);
        const float fa = as - af;
        const int ia = (int)af;
        const float wa0 = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa : 0.0f;
        const float wa1 = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa : 0.0f;
        if (wa0 == 0.0f && wa1 == 0.0f) continue;
        const int ia0 = clampi(ia, 0, A.nu - 1), ia1 = clampi(ia + 1, 0, A.nu - 1);
        const float bs0 = fmaf(m * zb, A.inv_dv, A.bv0);
        const float bst = m * A.dz * A.inv_dv;
        float w = 0.0f, rxy2 = 0.0f, wpm = 0.0f;
        if (W == CT_BP_FDK) {
            const float q = A.DSO * iL;
            w = q * q;
        } else {
            const float sx = x - A.DSO * c, sy = y - A.DSO * s;
            rxy2 = sx * sx + sy * sy;
            wpm = A.pm_const * iL * iL * iL;
        }
        const TP *P = proj + (int64_t)t * psz;
#pragma unroll
        for (int k = 0; k < BP_NZ; ++k) {
            const float bs = fmaf((float)k, bst, bs0);
            const float bf = floorf(bs);
            const float fb = bs - bf;
            const int ib = (int)bf;
            const float wb0 = ((unsigned)ib < (unsigned)A.nv) ? 1.0f - fb : 0.0f;
            const float wb1 = ((unsigned)(ib + 1) < (unsigned)A.nv) ? fb : 0.0f;
            const int r0 = clampi(ib, 0, A.nv - 1) * A.nu, r1 = clampi(ib + 1, 0, A.nv - 1) * A.nu;
            const float v0 = fmaf(wa1, ldf(P, r0 + ia1), wa0 * ldf(P, r0 + ia0));
            const float v1 = fmaf(wa1, ldf(P, r1 + ia1), wa0 * ldf(P, r1 + ia0));
            const float v = fmaf(wb1, v1, wb0 * v0);
            float wk = w;
            if (W != CT_BP_FDK) {
                const float z = fmaf((float)k, A.dz, zb);
                wk = wpm * sqrtf(fmaf(z, z, rxy2));
            }
            acc[k] = fmaf(wk, v, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        const float prev = A.accumulate ? to_f(vol[o]) : 0.0f;
        vol[o] = from_f<TV>(prev + acc[k]);
    }
}

// Exact transpose of the Siddon projector, gathered per voxel.
template <typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_adjoint(const TP *__restrict__ proj, TV *__restrict__ vol, BpArgs A) {
    const int i = blockIdx.x * BP_TX + (threadIdx.x % BP_TX);
    const int j = blockIdx.y * BP_TY + (threadIdx.x / BP_TX);
    const int kb = A.own_lo + blockIdx.z * BP_NZ;
    if (i >= A.nx || j >= A.ny) return;
    // column square (mm, FP64)
    const double xc = A.dx0 + i * A.ddx, yc = A.dy0 + j * A.ddy;
    const double xl = xc - 0.5 * A.ddx, xh = xc + 0.5 * A.ddx;
    const double yl = yc - 0.5 * A.ddy, yh = yc + 0.5 * A.ddy;
    const float zl0 = (float)(A.dz0 + (kb - 0.5) * A.ddz);  // lower face of voxel kb
    const float dz = A.dz;
    float acc[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) acc[k] = 0.0f;
    const int64_t psz = (int64_t)A.nu * A.nv;
    const float bscale = A.inv_dv;
    for (int t = 0; t < A.nang; ++t) {
        const AngleGeo &G = A.tab[A.a0 + t];
        const double c = G.c, s = G.s;
        const double Sx = A.dDSO * c, Sy = A.dDSO * s;
        // detector column range: central projection of the square's corners onto the u axis
        double umin = 1e300, umax = -1e300;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double X = (q & 1) ? xh : xl, Y = (q & 2) ? yh : yl;
            const double Ld = A.dDSO - (X * c + Y * s);
            const double u = A.dDSD * (Y * c - X * s) / Ld;
            umin = fmin(umin, u);
            umax = fmax(umax, u);
        }
        // clamp in floating point before converting, so the casts stay in range
        const int alo = (int)fmax(ceil((umin - A.offu) / A.du + A.cu - 1e-6), 0.0);
        const int ahi = (int)fmin(floor((umax - A.offu) / A.du + A.cu + 1e-6), (double)(A.nu - 1));
        const TP *P = proj + (int64_t)t * psz;
        for (int a = alo; a <= ahi; ++a) {
            const double ua = (a - A.cu) * A.du + A.offu;
            // ray (x, y) trace: S + t (P - S), P - S = -DSD (c, s) + ua (-s, c)
            const double Dx = -A.dDSD * c - ua * s, Dy = -A.dDSD * s + ua * c;
            const double Lxy = sqrt(Dx * Dx + Dy * Dy);
            double t0 = -1e300, t1 = 1e300;
            if (fabs(Dx) < 1e-12 * Lxy) {
                if (Sx < xl || Sx > xh) continue;
            } else {
                const double ta = (xl - Sx) / Dx, tb = (xh - Sx) / Dx;
                t0 = fmax(t0, fmin(ta, tb));
                t1 = fmin(t1, fmax(ta, tb));
            }
            if (fabs(Dy) < 1e-12 * Lxy) {
                if (Sy < yl || Sy > yh) continue;
            } else {
                const double ta = (yl - Sy) / Dy, tb = (yh - Sy) / Dy;
                t0 = fmax(t0, fmin(ta, tb));
                t1 = fmin(t1, fmax(ta, tb));
            }
            t0 = fmax(t0, 0.0);
            t1 = fmin(t1, 1.0);
            if (!(t0 < t1)) continue;
            // z along the ray: z(t) = t v_b (source in the z = 0 plane); local parameter tau = t - t0
            const float T = (float)(t1 - t0);
            const float ft0 = (float)t0;
            const float it0 = (float)(1.0 / t0), it1 = (float)(1.0 / t1);
            const float lxy2 = (float)(Lxy * Lxy);
#pragma unroll
            for (int k = 0; k < BP_NZ; ++k) {
                const float zl = fmaf((float)k, dz, zl0), zh = zl + dz;
                // rows whose ray can meet z in [zl, zh] for t in [t0, t1]: v in [vmin, vmax]
                const float vmin = fminf(zl * it0, zl * it1), vmax = fmaxf(zh * it0, zh * it1);
                const int blo = (int)fmaxf(ceilf(fmaf(vmin - (float)A.offv, bscale, (float)A.cv) - 1e-4f), 0.0f);
                const int bhi = (int)fminf(floorf(fmaf(vmax - (float)A.offv, bscale, (float)A.cv) + 1e-4f),
                                           (float)(A.nv - 1));
                float sum = 0.0f;
                for (int b = blo; b <= bhi; ++b) {
                    const float vb = (float)((b - A.cv) * A.dv + A.offv);
                    const float Z0 = ft0 * vb;  // z where the ray enters the column
                    float ta, tb;
                    if (fabsf(vb) > 0.0f) {
                        const float iv = 1.0f / vb;
                        const float q0 = (zl - Z0) * iv, q1 = (zh - Z0) * iv;
                        ta = fmaxf(0.0f, fminf(q0, q1));
                        tb = fminf(T, fmaxf(q0, q1));
                    } else {
                        ta = 0.0f;
                        tb = (zl <= 0.0f && 0.0f <= zh) ? T : 0.0f;
                    }
                    const float len = fmaxf(tb - ta, 0.0f) * sqrtf(fmaf(vb, vb, lxy2));
                    sum = fmaf(len, ldf(P, (int64_t)b * A.nu + a), sum);
                }
                acc[k] += sum;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        const float prev = A.accumulate ? to_f(vol[o]) : 0.0f;
        vol[o] = from_f<TV>(prev + acc[k]);
    }
}

// SART update for one angle t with FDK weights:
//   x_j += lambda * (w_j * bilinear(r)) / (w_j * bilinear(1))   where w_j * bilinear(1) > 1e-6
__global__ __launch_bounds__(256) void k_sart_update(const float *__restrict__ r, float *__restrict__ vol, BpArgs A,
                                                     float lambda) {
    const int i = blockIdx.x * BP_TX + (threadIdx.x % BP_TX);
    const int j = blockIdx.y * BP_TY + (threadIdx.x / BP_TX);
    const int kb = blockIdx.z * BP_NZ;
    if (i >= A.nx || j >= A.ny) return;
    const float x = fmaf((float)i, A.dx, A.x0);
    const float y = fmaf((float)j, A.dy, A.y0);
    const AngleGeo &G = A.tab[A.a0];
    const float c = (float)G.c, s = (float)G.s;
    const float Ld = A.DSO - (x * c + y * s);
    const float iL = 1.0f / Ld;
    const float m = A.DSD * iL;
    const float as = fmaf(m * (y * c - x * s), A.inv_du, A.au0);
    const float af = floorf(as);
    const float fa = as - af;
    const int ia = (int)af;
    const float wa0 = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa : 0.0f;
    const float wa1 = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa : 0.0f;
    if (wa0 == 0.0f && wa1 == 0.0f) return;
    const int ia0 = clampi(ia, 0, A.nu - 1), ia1 = clampi(ia + 1, 0, A.nu - 1);
    const float q = A.DSO * iL;
    const float w = q * q;
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        if (kk >= A.nz) break;
        const float z = fmaf((float)kk, A.dz, A.z0);
        const float bs = fmaf(m * z, A.inv_dv, A.bv0);
        const float bf = floorf(bs);
        const float fb = bs - bf;
        const int ib = (int)bf;
        const float wb0 = ((unsigned)ib < (unsigned)A.nv) ? 1.0f - fb : 0.0f;
        const float wb1 = ((unsigned)(ib + 1) < (unsigned)A.nv) ? fb : 0.0f;
        const int r0 = clampi(ib, 0, A.nv - 1) * A.nu, r1 = clampi(ib + 1, 0, A.nv - 1) * A.nu;
        const float v0 = fmaf(wa1, r[r0 + ia1], wa0 * r[r0 + ia0]);
        const float v1 = fmaf(wa1, r[r1 + ia1], wa0 * r[r1 + ia0]);
        const float num = w * fmaf(wb1, v1, wb0 * v0);
        const float V = w * ((wa0 + wa1) * (wb0 + wb1));
        if (V > 1e-6f) {
            const int64_t o = ((int64_t)kk * A.ny + j) * A.nx + i;
            vol[o] = fmaf(lambda, num / V, vol[o]);
        }
    }
}

BpArgs make_bp_args(ct_plan *p, const AngleGeo *tab, int64_t a0, int64_t a1, const Slab &slab, int accumulate) {
    const ct_geometry &g = p->g;
    BpArgs A;
    A.tab = tab;
    A.a0 = a0;
    A.nang = (int32_t)(a1 - a0);
    A.nx = (int32_t)g.nVoxel[0];
    A.ny = (int32_t)g.nVoxel[1];
    A.nz = (int32_t)g.nVoxel[2];
    A.dx = (float)g.dVoxel[0];
    A.dy = (float)g.dVoxel[1];
    A.dz = (float)g.dVoxel[2];
    A.ddx = g.dVoxel[0];
    A.ddy = g.dVoxel[1];
    A.ddz = g.dVoxel[2];
    A.dx0 = g.offOrigin[0] - (g.nVoxel[0] - 1) / 2.0 * g.dVoxel[0];
    A.dy0 = g.offOrigin[1] - (g.nVoxel[1] - 1) / 2.0 * g.dVoxel[1];
    A.dz0 = g.offOrigin[2] - (g.nVoxel[2] - 1) / 2.0 * g.dVoxel[2];
    A.x0 = (float)A.dx0;
    A.y0 = (float)A.dy0;
    A.z0 = (float)A.dz0;
    A.nu = (int32_t)g.nDetector[0];
    A.nv = (int32_t)g.nDetector[1];
    A.du = g.dDetector[0];
    A.dv = g.dDetector[1];
    A.cu = (g.nDetector[0] - 1) / 2.0;
    A.cv = (g.nDetector[1] - 1) / 2.0;
    A.offu = g.offDetector[0];
    A.offv = g.offDetector[1];
    A.inv_du = (float)(1.0 / g.dDetector[0]);
    A.inv_dv = (float)(1.0 / g.dDetector[1]);
    A.au0 = (float)(A.cu - g.offDetector[0] / g.dDetector[0]);
    A.bv0 = (float)(A.cv - g.offDetector[1] / g.dDetector[1]);
    A.DSO = (float)g.DSO;
    A.DSD = (float)g.DSD;
    A.dDSO = g.DSO;
    A.dDSD = g.DSD;
    A.pm_const = (float)(g.dVoxel[0] * g.dVoxel[1] * g.dVoxel[2] / (g.dDetector[0] * g.dDetector[1]) * g.DSD * g.DSD);
    A.own_lo = (int32_t)slab.own_lo;
    A.own_hi = (int32_t)slab.own_hi;
    A.mem_lo = (int32_t)slab.mem_lo;
    A.accumulate = accumulate;
    return A;
}

}  // namespace

ct_status launch_backproject(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                             ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab, hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    const int64_t nzown = slab.own_hi - slab.own_lo;
    if (nzown <= 0) return CT_OK;
    BpArgs A = make_bp_args(p, tab, a0, a1, slab, accumulate);
    const dim3 grid((A.nx + BP_TX - 1) / BP_TX, (A.ny + BP_TY - 1) / BP_TY, (unsigned)((nzown + BP_NZ - 1) / BP_NZ));
    const dim3 block(256);
    if (kind == CT_BP_FDK) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_voxel<CT_BP_FDK, TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    } else if (kind == CT_BP_PSEUDO_MATCHED) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_voxel<CT_BP_PSEUDO_MATCHED, TP, TV>), grid, block, 0, st, (const TP *)proj,
                                        (TV *)vol, A));
    } else {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_adjoint<TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_sart_update(ct_plan *p, const float *r, float *vol, int64_t angle, float lambda, hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    BpArgs A = make_bp_args(p, tab, angle, angle + 1, full_slab(p->g), 1);
    const dim3 grid((A.nx + BP_TX - 1) / BP_TX, (A.ny + BP_TY - 1) / BP_TY, (unsigned)((A.nz + BP_NZ - 1) / BP_NZ));
    hipLaunchKernelGGL(k_sart_update, grid, dim3(256), 0, st, r, vol, A, lambda);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

}  // namespace ct
