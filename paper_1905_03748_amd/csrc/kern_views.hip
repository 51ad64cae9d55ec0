// Backprojectors and the SART update for plans of views (Section 2.2's operators over any scan of
// Section 2.1: circular, C-arm, helical).  A view is a source, a detector centre and unit detector
// axes; the plan stores each view's projective map M (rows a* L, b* L and L, affine in the voxel
// index, L the depth from the source along the detector normal).
//
// One thread per (x, y) voxel column of a 16 x 16 tile and a run of VB_NZ slices, looping over the
// views of the launch with the run's sums in registers, as the circular kernels do.  Nothing is
// constant along a column here (a tilted detector changes the depth with z), so every voxel forms
// its own depth and detector coordinates, from FP32 offsets to a tile reference projected in FP64:
//   with A_r, B_r, W_r = M (x_r, 1) at the tile's reference point x_r and d = x - x_r (index units),
//   a* - a*_r = (M_a - a*_r M_w) . d / (W_r + M_w . d), and likewise b*,
// where the FP32 coefficients are formed in FP64, so every FP32 quantity is a few pixels or a tile
// in size, whatever the detector's.
//
// The exact adjoint (transpose of the Siddon projector) gathers per voxel every pixel whose ray can
// cross the voxel: the pixels whose centres fall in the box bounding the voxel's image, from the
// centre's detector coordinates and the local Jacobian.  The ray of pixel (a, b) passes through
// the voxel's depth plane (parallel to the detector) at x + (L / DSD_v) ((a - a*) du e_u +
// (b - b*) dv e_v), a point a voxel or less from the centre formed from small quantities, and its
// chord through the voxel box is the slab intersection about that point.  The chord equals the sum
// of the Siddon pieces the ray leaves in the voxel; a ray that lies in a face goes to the voxel
// above the face (a half-open slab), as in the projector.
#include <cfloat>
#include <cmath>

#include "dev_common.hpp"

namespace ct {

namespace {

constexpr int VB_TX = 16, VB_TY = 16;
#ifndef CT_VB_NZ
#define CT_VB_NZ 8
#endif
constexpr int VB_NZ = CT_VB_NZ;  // voxels per thread
constexpr int VB_G = 64;         // views per group of tile references

enum { VM_FDK = 0, VM_PM = 1, VM_SART = 2, VM_ADJ = 3 };

struct VArgs {
    const AngleGeo *tab;
    int64_t a0;
    int32_t nang;
    int32_t nx, ny, nz;
    float dx, dy, dz;        // voxel size, mm
    int32_t nu, nv;
    float du, dv, cu, cv, offu, offv;
    int32_t own_lo, own_hi;  // voxels written: k in [own_lo, own_hi)
    int32_t mem_lo;          // slice at the volume pointer
    int32_t accumulate;
    float lambda;            // SART relaxation
};

// FP32 factors of one (tile, view) pair
struct VRef {
    float ga[3], gb[3], mw[3];
    float wr;          // depth of the reference point, mm
    float Aloc, Bloc;  // its detector coordinates minus the integer origin
    float sx, sy, sz;  // reference point minus source, mm
    float w0;          // DSO_v (FDK, SART), the pseudo-matched constant (PM) or 1 / DSD_v (adjoint)
};

// per view: what the exact adjoint's pixel rays need (mm)
struct VPix {
    float cs[3];  // detector centre - source
    float eu[3], ev[3];
    float pad;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Reference point of a tile: the centre of its columns in the grid and of its run of slices
// clipped to the grid (independent of the slab, so slab splits do the same arithmetic).
__device__ __forceinline__ double tile_mid(int first, int len, int n) { return 0.5 * (double)(first + min(first + len, n) - 1); }

template <int MODE>
__device__ __forceinline__ void view_ref(const VArgs &A, const AngleGeo &G, double ir, double jr, double kr, VRef &R,
                                         float &ia0, float &ib0) {
    const double Ar = fma(G.M[0], ir, fma(G.M[1], jr, fma(G.M[2], kr, G.M[3])));
    const double Br = fma(G.M[4], ir, fma(G.M[5], jr, fma(G.M[6], kr, G.M[7])));
    const double Wr = fma(G.M[8], ir, fma(G.M[9], jr, fma(G.M[10], kr, G.M[11])));
    const double ar = Ar / Wr, br = Br / Wr;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        R.ga[q] = (float)fma(-ar, G.M[8 + q], G.M[q]);
        R.gb[q] = (float)fma(-br, G.M[8 + q], G.M[4 + q]);
        R.mw[q] = (float)G.M[8 + q];
    }
    R.wr = (float)Wr;
    // integer origins (clamped far outside the detector, where every tap is zero anyway)
    const double fa = fmin(fmax(floor(ar), -16777216.0), 16777216.0);
    const double fb = fmin(fmax(floor(br), -16777216.0), 16777216.0);
    R.Aloc = (float)(ar - fa);
    R.Bloc = (float)(br - fb);
    ia0 = (float)fa;
    ib0 = (float)fb;
    R.sx = (float)((ir - G.S[0]) * (double)A.dx);
    R.sy = (float)((jr - G.S[1]) * (double)A.dy);
    R.sz = (float)((kr - G.S[2]) * (double)A.dz);
    R.w0 = (float)(MODE == VM_PM ? G.pmc : MODE == VM_ADJ ? 1.0 / G.DSDv : G.DSOv);
}

// Runs of VB_NZ slices start at absolute multiples of VB_NZ.
__device__ __forceinline__ int run_base(const VArgs &A) { return (A.own_lo / VB_NZ + (int)blockIdx.z) * VB_NZ; }

// FDK, pseudo-matched or SART: bilinear taps at each voxel's own detector coordinates.
template <int MODE, typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_views(const TP *__restrict__ proj, TV *__restrict__ vol, VArgs A) {
    __shared__ VRef ref[VB_G];
    __shared__ float iref[VB_G][2];
    const int i0 = blockIdx.x * VB_TX, j0 = blockIdx.y * VB_TY;
    const int i = i0 + (threadIdx.x % VB_TX);
    const int j = j0 + (threadIdx.x / VB_TX);
    const int kb = run_base(A);
    const bool live = i < A.nx && j < A.ny;
    const double ir = tile_mid(i0, VB_TX, A.nx), jr = tile_mid(j0, VB_TY, A.ny), kr = tile_mid(kb, VB_NZ, A.nz);
    const float di = (float)((double)i - ir), dj = (float)((double)j - jr);
    float dk[VB_NZ];
#pragma unroll
    for (int k = 0; k < VB_NZ; ++k) dk[k] = (float)((double)(kb + k) - kr);
    float acc[VB_NZ], den[VB_NZ];
#pragma unroll
    for (int k = 0; k < VB_NZ; ++k) {
        const int kk = kb + k;
        acc[k] = (MODE != VM_SART && live && A.accumulate && kk >= A.own_lo && kk < A.own_hi)
                     ? to_f(vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i])
                     : 0.0f;
        den[k] = 0.0f;
    }
    const int64_t psz = (int64_t)A.nu * A.nv;
    constexpr int ES = (int)sizeof(TP);
    const int rowb = A.nu * ES;
    const float amax = (float)A.nu + 1.0f, bmax = (float)A.nv + 1.0f;
    for (int t0 = 0; t0 < A.nang; t0 += VB_G) {
        const int nk = min(VB_G, A.nang - t0);
        __syncthreads();  // the previous group's references have been read
        if ((int)threadIdx.x < nk) {
            VRef R;
            float fa, fb;
            view_ref<MODE>(A, A.tab[A.a0 + t0 + threadIdx.x], ir, jr, kr, R, fa, fb);
            ref[threadIdx.x] = R;
            iref[threadIdx.x][0] = fa;
            iref[threadIdx.x][1] = fb;
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nk; ++q) {
            const VRef R = ref[q];
            const float oa = iref[q][0], ob = iref[q][1];
            const float wxy = fmaf(R.mw[0], di, fmaf(R.mw[1], dj, R.wr));
            const float axy = fmaf(R.ga[0], di, R.ga[1] * dj), bxy = fmaf(R.gb[0], di, R.gb[1] * dj);
            const float sx = fmaf(di, A.dx, R.sx), sy = fmaf(dj, A.dy, R.sy);
            const __amdgpu_buffer_rsrc_t Rs = proj_rsrc(proj + (int64_t)(t0 + q) * psz, psz * ES);
            float p[VB_NZ][4], fa_[VB_NZ], fb_[VB_NZ], wa0[VB_NZ], wa1[VB_NZ], wt[VB_NZ];
#pragma unroll
            for (int k = 0; k < VB_NZ; ++k) {
                const float w = fmaf(R.mw[2], dk[k], wxy);
                const float iw = __builtin_amdgcn_rcpf(w);
                const float as = fmaf(fmaf(R.ga[2], dk[k], axy), iw, R.Aloc);
                const float bs = fmaf(fmaf(R.gb[2], dk[k], bxy), iw, R.Bloc);
                const float af = floorf(as), bf = floorf(bs);
                fa_[k] = as - af;
                fb_[k] = bs - bf;
                const int ia = (int)__builtin_amdgcn_fmed3f(oa + af, -2.0f, amax);
                wa0[k] = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa_[k] : 0.0f;
                wa1[k] = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa_[k] : 0.0f;
                const int ca0 = clampi(ia, 0, A.nu - 1) * ES;
                const int dca = (clampi(ia + 1, 0, A.nu - 1) - clampi(ia, 0, A.nu - 1)) * ES;
                // rows outside the detector read 0 (negative offsets wrap past the buffer's end)
                const int o00 = (int)__builtin_amdgcn_fmed3f(ob + bf, -2.0f, bmax) * rowb + ca0;
                p[k][0] = bload(Rs, o00, (TP *)nullptr);
                p[k][1] = bload(Rs, o00 + dca, (TP *)nullptr);
                p[k][2] = bload(Rs, o00 + rowb, (TP *)nullptr);
                p[k][3] = bload(Rs, o00 + rowb + dca, (TP *)nullptr);
                if (MODE == VM_PM) {
                    const float sz = fmaf(dk[k], A.dz, R.sz);
                    wt[k] = R.w0 * sqrtf(fmaf(sx, sx, fmaf(sy, sy, sz * sz))) * iw * iw * iw;
                } else {
                    const float qq = R.w0 * iw;
                    wt[k] = qq * qq;
                }
                if (MODE == VM_SART) {
                    // the bilinear weight of the taps on the detector (B 1 of the update)
                    const int ib = (int)__builtin_amdgcn_fmed3f(ob + bf, -2.0f, bmax);
                    const float wb0 = ((unsigned)ib < (unsigned)A.nv) ? 1.0f - fb_[k] : 0.0f;
                    const float wb1 = ((unsigned)(ib + 1) < (unsigned)A.nv) ? fb_[k] : 0.0f;
                    den[k] = fmaf(wt[k], (wa0[k] + wa1[k]) * (wb0 + wb1), den[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < VB_NZ; ++k) {
                const float v0 = fmaf(wa1[k], p[k][1], wa0[k] * p[k][0]);
                const float v1 = fmaf(wa1[k], p[k][3], wa0[k] * p[k][2]);
                const float v = fmaf(fb_[k], v1 - v0, v0);
                acc[k] = fmaf(wt[k], v, acc[k]);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < VB_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.own_lo) continue;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        if (MODE == VM_SART) {
            if (den[k] > 1e-6f) vol[o] = from_f<TV>(fmaf(A.lambda, acc[k] / den[k], to_f(vol[o])));
        } else {
            vol[o] = from_f<TV>(acc[k]);
        }
    }
}

// Exact adjoint of the Siddon projector for plans of views (see the header).
template <typename TP, typename TV>
__global__ __launch_bounds__(256) void k_adj_views(const TP *__restrict__ proj, TV *__restrict__ vol, VArgs A) {
    __shared__ VRef ref[VB_G];
    __shared__ float iref[VB_G][2];
    __shared__ VPix pixg[VB_G];
    const int i0 = blockIdx.x * VB_TX, j0 = blockIdx.y * VB_TY;
    const int i = i0 + (threadIdx.x % VB_TX);
    const int j = j0 + (threadIdx.x / VB_TX);
    const int kb = run_base(A);
    const bool live = i < A.nx && j < A.ny;
    const double ir = tile_mid(i0, VB_TX, A.nx), jr = tile_mid(j0, VB_TY, A.ny), kr = tile_mid(kb, VB_NZ, A.nz);
    const float di = (float)((double)i - ir), dj = (float)((double)j - jr);
    const float hx = 0.5f * A.dx, hy = 0.5f * A.dy, hz = 0.5f * A.dz;
    float acc[VB_NZ];
#pragma unroll
    for (int k = 0; k < VB_NZ; ++k) {
        const int kk = kb + k;
        acc[k] = (live && A.accumulate && kk >= A.own_lo && kk < A.own_hi)
                     ? to_f(vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i])
                     : 0.0f;
    }
    const int64_t psz = (int64_t)A.nu * A.nv;
    constexpr int ES = (int)sizeof(TP);
    for (int t0 = 0; t0 < A.nang; t0 += VB_G) {
        const int nk = min(VB_G, A.nang - t0);
        __syncthreads();
        if ((int)threadIdx.x < nk) {
            const AngleGeo &G = A.tab[A.a0 + t0 + threadIdx.x];
            VRef R;
            float fa, fb;
            view_ref<VM_ADJ>(A, G, ir, jr, kr, R, fa, fb);
            ref[threadIdx.x] = R;
            iref[threadIdx.x][0] = fa;
            iref[threadIdx.x][1] = fb;
            VPix P;
            P.cs[0] = (float)(G.Dc[0] * (double)A.dx);
            P.cs[1] = (float)(G.Dc[1] * (double)A.dy);
            P.cs[2] = (float)(G.Dc[2] * (double)A.dz);
            P.eu[0] = (float)(G.eu[0] * (double)A.dx);
            P.eu[1] = (float)(G.eu[1] * (double)A.dy);
            P.eu[2] = (float)(G.eu[2] * (double)A.dz);
            P.ev[0] = (float)(G.ev[0] * (double)A.dx);
            P.ev[1] = (float)(G.ev[1] * (double)A.dy);
            P.ev[2] = (float)(G.ev[2] * (double)A.dz);
            P.pad = 0.0f;
            pixg[threadIdx.x] = P;
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nk; ++q) {
            const VRef R = ref[q];
            const VPix P = pixg[q];
            const float oa = iref[q][0], ob = iref[q][1];
            const float wxy = fmaf(R.mw[0], di, fmaf(R.mw[1], dj, R.wr));
            const float axy = fmaf(R.ga[0], di, R.ga[1] * dj), bxy = fmaf(R.gb[0], di, R.gb[1] * dj);
            const __amdgpu_buffer_rsrc_t Rs = proj_rsrc(proj + (int64_t)(t0 + q) * psz, psz * ES);
            for (int k = 0; k < VB_NZ; ++k) {
                const float dkk = (float)((double)(kb + k) - kr);
                const float w = fmaf(R.mw[2], dkk, wxy);
                const float iw = __builtin_amdgcn_rcpf(w);
                const float al = fmaf(R.ga[2], dkk, axy) * iw, be = fmaf(R.gb[2], dkk, bxy) * iw;
                // half-extent of the voxel's image from the local Jacobian (index units), with a
                // margin for the perspective's curvature over one voxel
                const float ha = 0.5f * (fabsf(fmaf(-al, R.mw[0], R.ga[0])) + fabsf(fmaf(-al, R.mw[1], R.ga[1])) +
                                         fabsf(fmaf(-al, R.mw[2], R.ga[2]))) * iw;
                const float hb = 0.5f * (fabsf(fmaf(-be, R.mw[0], R.gb[0])) + fabsf(fmaf(-be, R.mw[1], R.gb[1])) +
                                         fabsf(fmaf(-be, R.mw[2], R.gb[2]))) * iw;
                const float as = al + R.Aloc, bs = be + R.Bloc;  // relative to the integer origin
                const float ma = fmaf(ha, 0.02f, 1e-3f), mb = fmaf(hb, 0.02f, 1e-3f);
                // pixel ranges clamped to the detector (in float first, so no conversion overflows)
                const float fnu = (float)A.nu, fnv = (float)A.nv;
                const int alo = (int)fmaxf(oa + ceilf(as - ha - ma), 0.0f);
                const int ahi = (int)fminf(oa + floorf(as + ha + ma), fnu - 1.0f);
                const int blo = (int)fmaxf(ob + ceilf(bs - hb - mb), 0.0f);
                const int bhi = (int)fminf(ob + floorf(bs + hb + mb), fnv - 1.0f);
                // the ray of pixel (a, b) crosses the voxel's depth plane at x + (a - a*) qa + (b - b*) qb
                const float sc = w * R.w0;
                const float qa0 = sc * A.du * P.eu[0], qa1 = sc * A.du * P.eu[1], qa2 = sc * A.du * P.eu[2];
                const float qb0 = sc * A.dv * P.ev[0], qb1 = sc * A.dv * P.ev[1], qb2 = sc * A.dv * P.ev[2];
                float s = 0.0f;
                for (int b = blo; b <= bhi; ++b) {
                    const float db = ((float)b - ob) - bs;
                    const float vb = fmaf((float)b - A.cv, A.dv, A.offv);
                    const float eb0 = fmaf(vb, P.ev[0], P.cs[0]), eb1 = fmaf(vb, P.ev[1], P.cs[1]),
                                eb2 = fmaf(vb, P.ev[2], P.cs[2]);
                    const float pb0 = db * qb0, pb1 = db * qb1, pb2 = db * qb2;
                    for (int a = alo; a <= ahi; ++a) {
                        const float da = ((float)a - oa) - as;
                        const float ua = fmaf((float)a - A.cu, A.du, A.offu);
                        const float D0 = fmaf(ua, P.eu[0], eb0), D1 = fmaf(ua, P.eu[1], eb1), D2 = fmaf(ua, P.eu[2], eb2);
                        const float Q0 = fmaf(da, qa0, pb0), Q1 = fmaf(da, qa1, pb1), Q2 = fmaf(da, qa2, pb2);
                        float tlo = -FLT_MAX, thi = FLT_MAX;
                        bool in = true;
                        const float Dq[3] = {D0, D1, D2}, Qq[3] = {Q0, Q1, Q2}, Hq[3] = {hx, hy, hz};
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (Dq[c] == 0.0f) {
                                // parallel to the planes of this axis: inside the half-open slab
                                in = in && (-Hq[c] <= Qq[c]) && (Qq[c] < Hq[c]);
                            } else {
                                const float inv = __builtin_amdgcn_rcpf(Dq[c]);
                                const float t1 = (-Hq[c] - Qq[c]) * inv, t2 = (Hq[c] - Qq[c]) * inv;
                                tlo = fmaxf(tlo, fminf(t1, t2));
                                thi = fminf(thi, fmaxf(t1, t2));
                            }
                        }
                        const float len = (in && thi > tlo) ? (thi - tlo) * sqrtf(fmaf(D0, D0, fmaf(D1, D1, D2 * D2))) : 0.0f;
                        if (len > 0.0f) s = fmaf(bload(Rs, (b * A.nu + a) * ES, (TP *)nullptr), len, s);
                    }
                }
                acc[k] += s;
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < VB_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.own_lo) continue;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        vol[o] = from_f<TV>(acc[k]);
    }
}

VArgs make_vargs(const ct_plan *p, const AngleGeo *tab, int64_t a0, int64_t a1, const Slab &slab, int accumulate) {
    const ct_geometry &g = p->g;
    VArgs A;
    A.tab = tab;
    A.a0 = a0;
    A.nang = (int32_t)(a1 - a0);
    A.nx = (int32_t)g.nVoxel[0];
    A.ny = (int32_t)g.nVoxel[1];
    A.nz = (int32_t)g.nVoxel[2];
    A.dx = (float)g.dVoxel[0];
    A.dy = (float)g.dVoxel[1];
    A.dz = (float)g.dVoxel[2];
    A.nu = (int32_t)g.nDetector[0];
    A.nv = (int32_t)g.nDetector[1];
    A.du = (float)g.dDetector[0];
    A.dv = (float)g.dDetector[1];
    A.cu = (float)((g.nDetector[0] - 1) / 2.0);
    A.cv = (float)((g.nDetector[1] - 1) / 2.0);
    A.offu = (float)g.offDetector[0];
    A.offv = (float)g.offDetector[1];
    A.own_lo = (int32_t)slab.own_lo;
    A.own_hi = (int32_t)slab.own_hi;
    A.mem_lo = (int32_t)slab.mem_lo;
    A.accumulate = accumulate;
    A.lambda = 0.0f;
    return A;
}

dim3 vgrid(const VArgs &A, const Slab &slab) {
    const unsigned runs = (unsigned)((slab.own_hi - 1) / VB_NZ - slab.own_lo / VB_NZ + 1);
    return dim3((unsigned)((A.nx + VB_TX - 1) / VB_TX), (unsigned)((A.ny + VB_TY - 1) / VB_TY), runs);
}

}  // namespace

ct_status launch_backproject_views(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                                   ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab,
                                   const AngleGeo *tab, hipStream_t st) {
    if (slab.own_hi <= slab.own_lo) return CT_OK;
    if (slab.zcol) return fail(CT_ERR_STATE, "a plan of views backprojects into [z][y][x] volumes only");
    const VArgs A = make_vargs(p, tab, a0, a1, slab, accumulate);
    const dim3 grid = vgrid(A, slab), block(256);
    if (kind == CT_BP_FDK) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_views<VM_FDK, TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    } else if (kind == CT_BP_PSEUDO_MATCHED) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_views<VM_PM, TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    } else {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_adj_views<TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_sart_update_views(ct_plan *p, const float *r, float *vol, int64_t a0, int64_t a1, float lambda,
                                   const AngleGeo *tab, hipStream_t st) {
    const Slab full = full_slab(p->g);
    VArgs A = make_vargs(p, tab, a0, a1, full, 1);
    A.lambda = lambda;
    hipLaunchKernelGGL((k_bp_views<VM_SART, float, float>), vgrid(A, full), dim3(256), 0, st, r, vol, A);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

}  // namespace ct
