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
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "dev_common.hpp"

namespace ct {

namespace {

constexpr int BP_TX = 16, BP_TY = 16;
#ifndef CT_BP_NZ
#define CT_BP_NZ 8
#endif
#ifndef CT_ADJ_NZ
#define CT_ADJ_NZ 16
#endif
#ifndef CT_ADJ_XCD_W
#define CT_ADJ_XCD_W 4
#endif
constexpr int BP_NZ = CT_BP_NZ;  // voxels per thread (FDK / pseudo-matched)

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
    int32_t zcol_n;         // exact adjoint: 0 = [z][y][x] volume; else column-major [y][x][zcol_n]
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
    float zk[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) zk[k] = fmaf((float)(kb + k), A.dz, A.z0);
    // with accumulate the sums start from the stored values, so a sequence of launches over
    // consecutive angle ranges performs exactly the additions of one launch over all of them
    float acc[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        acc[k] = (A.accumulate && kk < A.own_hi) ? to_f(vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i]) : 0.0f;
    }
    const int64_t psz = (int64_t)A.nu * A.nv;
    constexpr int ES = (int)sizeof(TP);
    const int rowb = A.nu * ES;
    for (int t = 0; t < A.nang; ++t) {
        const AngleGeo &G = A.tab[A.a0 + t];
        const float c = (float)G.c, s = (float)G.s;
        const float Ld = A.DSO - (x * c + y * s);
        const float iL = __builtin_amdgcn_rcpf(Ld);
        const float m = A.DSD * iL;
        const float as = fmaf(m * (y * c - x * s), A.inv_du, A.au0);
        const float af = floorf(as);
        const float fa = as - af;
        const int ia = (int)af;
        const float wa0 = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa : 0.0f;
        const float wa1 = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa : 0.0f;
        if (wa0 == 0.0f && wa1 == 0.0f) continue;
        const int ca0 = clampi(ia, 0, A.nu - 1) * ES;
        const int dca = (clampi(ia + 1, 0, A.nu - 1) - clampi(ia, 0, A.nu - 1)) * ES;
        const float mv = m * A.inv_dv;
        float w = 0.0f, rxy2 = 0.0f, wpm = 0.0f;
        if (W == CT_BP_FDK) {
            const float q = A.DSO * iL;
            w = q * q;
        } else {
            const float sx = x - A.DSO * c, sy = y - A.DSO * s;
            rxy2 = sx * sx + sy * sy;
            wpm = A.pm_const * iL * iL * iL;
        }
        const __amdgpu_buffer_rsrc_t R = proj_rsrc(proj + (int64_t)t * psz, psz * ES);
        // all taps of the column are issued before any is used, so they are in flight together
        float p[BP_NZ][4], fb[BP_NZ];
#pragma unroll
        for (int k = 0; k < BP_NZ; ++k) {
            // each voxel's row coordinate comes from its own absolute height, so a voxel's value
            // does not depend on how the volume is cut into launches or slabs
            const float bs = fmaf(zk[k], mv, A.bv0);
            const float bf = floorf(bs);
            fb[k] = bs - bf;
            const int o00 = (int)bf * rowb + ca0;  // rows outside the detector read 0
            p[k][0] = bload(R, o00, (TP *)nullptr);
            p[k][1] = bload(R, o00 + dca, (TP *)nullptr);
            p[k][2] = bload(R, o00 + rowb, (TP *)nullptr);
            p[k][3] = bload(R, o00 + rowb + dca, (TP *)nullptr);
        }
#pragma unroll
        for (int k = 0; k < BP_NZ; ++k) {
            const float v0 = fmaf(wa1, p[k][1], wa0 * p[k][0]);
            const float v1 = fmaf(wa1, p[k][3], wa0 * p[k][2]);
            const float v = fmaf(fb[k], v1 - v0, v0);
            float wk = w;
            if (W != CT_BP_FDK) wk = wpm * sqrtf(fmaf(zk[k], zk[k], rxy2));
            acc[k] = fmaf(wk, v, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        vol[o] = from_f<TV>(acc[k]);
    }
}

// ------------------------------------------------------------------------------------------
// The same backprojection with the projection taps staged in LDS.  For each group of up to
// BPL_K angles the block projects the eight corners of its 16 x 16 x BP_NZ voxel tile: a
// perspective map sends the box into the convex hull of its corners' images, so the detector
// window [floor(min a*) - 1, ...] x [floor(min b*) - 1, ...] of WW x HW pixels (sized on the host
// from an analytic bound) holds every tap of every voxel of the tile.  The windows are copied
// into LDS row by row (lanes on consecutive pixels, zeros outside the detector), and the voxels
// read their bilinear taps there.  The per-voxel arithmetic is that of k_bp_voxel.
#ifndef CT_BPL_NZ
#define CT_BPL_NZ 16
#endif
constexpr int BPL_NZ = CT_BPL_NZ;  // voxels per thread
#ifndef CT_BPL_K
#define CT_BPL_K 8
#endif
#ifndef CT_BPL_FLOATS
#define CT_BPL_FLOATS 4096
#endif
#ifndef CT_BPL_PITCH
#define CT_BPL_PITCH 37
#endif
constexpr int BPL_K = CT_BPL_K;            // angles per staging round (at most)
constexpr int BPL_FLOATS = CT_BPL_FLOATS;  // staged floats per block
constexpr int BPL_PN = CT_BPL_PITCH;       // row pitch of narrow windows (the common case)

// PITCH: LDS row pitch (floats) of a window, a compile-time constant so that both rows of a
// bilinear tap pair are one base address with immediate offsets.
template <int W, int PITCH, typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_lds(const TP *__restrict__ proj, TV *__restrict__ vol, BpArgs A, int WW,
                                                int HW, int K) {
    __shared__ float win[BPL_FLOATS];
    __shared__ int org[BPL_K][2];
    const int i0 = blockIdx.x * BP_TX, j0 = blockIdx.y * BP_TY;
    const int i = i0 + (threadIdx.x % BP_TX);
    const int j = j0 + (threadIdx.x / BP_TX);
    const int kb = A.own_lo + blockIdx.z * BPL_NZ;
    const bool live = i < A.nx && j < A.ny;
    const float x = fmaf((float)i, A.dx, A.x0);
    const float y = fmaf((float)j, A.dy, A.y0);
    float zk[BPL_NZ];
#pragma unroll
    for (int k = 0; k < BPL_NZ; ++k) zk[k] = fmaf((float)(kb + k), A.dz, A.z0);
    float acc[BPL_NZ];
#pragma unroll
    for (int k = 0; k < BPL_NZ; ++k) {
        const int kk = kb + k;
        acc[k] = (live && A.accumulate && kk < A.own_hi) ? to_f(vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i])
                                                          : 0.0f;
    }
    const int64_t psz = (int64_t)A.nu * A.nv;
    const int wsz = PITCH * HW;
    const float lamax = (float)(WW - 2), lbmax = (float)(HW - 2);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    for (int t0 = 0; t0 < A.nang; t0 += K) {
        const int nk = min(K, A.nang - t0);
        __syncthreads();  // the previous round's taps have been read
        // lanes 8q' .. 8q'+7 of wave 0: the tile's corners under angle t0 + q0 + q'
        for (int q0 = 0; wave == 0 && q0 < nk; q0 += 8) {
            const int q = q0 + (lane >> 3), cn = lane & 7;
            float as = 0.0f, bs = 0.0f;
            if (q < nk) {
                const AngleGeo &G = A.tab[A.a0 + t0 + q];
                const float c = (float)G.c, s = (float)G.s;
                const float xc = fmaf((float)(i0 + ((cn & 1) ? BP_TX - 1 : 0)), A.dx, A.x0);
                const float yc = fmaf((float)(j0 + ((cn & 2) ? BP_TY - 1 : 0)), A.dy, A.y0);
                const float zc = fmaf((float)(kb + ((cn & 4) ? BPL_NZ - 1 : 0)), A.dz, A.z0);
                const float iL = __builtin_amdgcn_rcpf(A.DSO - (xc * c + yc * s));
                const float m = A.DSD * iL;
                as = fmaf(m * (yc * c - xc * s), A.inv_du, A.au0);
                bs = fmaf(zc, m * A.inv_dv, A.bv0);
            }
            float amin = as, bmin = bs;
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                amin = fminf(amin, __shfl_xor(amin, off, 64));
                bmin = fminf(bmin, __shfl_xor(bmin, off, 64));
            }
            if (cn == 0 && q < nk) {
                org[q][0] = (int)floorf(amin) - 1;
                org[q][1] = (int)floorf(bmin) - 1;
            }
        }
        __syncthreads();
        // stage: wave w copies rows w, w + 4, ... of every window; lane = window column
        for (int q = 0; q < nk; ++q) {
            const int u = org[q][0] + lane;
            const bool uok = lane < WW && (unsigned)u < (unsigned)A.nu;
            const TP *pq = proj + (int64_t)(t0 + q) * psz + u;
            float *wq = win + q * wsz + lane;
            for (int r = wave; r < HW; r += 4) {
                const int v = org[q][1] + r;
                float val = 0.0f;
                if (uok && (unsigned)v < (unsigned)A.nv) val = to_f(pq[(int64_t)v * A.nu]);
                if (lane < WW) wq[r * PITCH] = val;
            }
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nk; ++q) {
            const AngleGeo &G = A.tab[A.a0 + t0 + q];
            const float c = (float)G.c, s = (float)G.s;
            const float Ld = A.DSO - (x * c + y * s);
            const float iL = __builtin_amdgcn_rcpf(Ld);
            const float m = A.DSD * iL;
            const float as = fmaf(m * (y * c - x * s), A.inv_du, A.au0);
            const float af = floorf(as);
            const float fa = as - af;
            const float wa0 = 1.0f - fa, wa1 = fa;  // taps off the detector are zeros in the window
            // window-local column and row (exact integers in FP32), clamped into the window
            const float la = __builtin_amdgcn_fmed3f(af - (float)org[q][0], 0.0f, lamax);
            const float ob = (float)org[q][1];
            const float mv = m * A.inv_dv;
            float w = 0.0f, rxy2 = 0.0f, wpm = 0.0f;
            if (W == CT_BP_FDK) {
                const float qq = A.DSO * iL;
                w = qq * qq;
            } else {
                const float sx = x - A.DSO * c, sy = y - A.DSO * s;
                rxy2 = sx * sx + sy * sy;
                wpm = A.pm_const * iL * iL * iL;
            }
            // LDS byte offset of the window column (exact in FP32), rebased so that the absolute row
            // index can be used directly; the clamp keeps rows 0 .. HW - 2 of the window
            const float cb = fmaf(la, 4.0f, (float)(q * wsz * 4));
            const float cbr = fmaf(-ob, (float)(4 * PITCH), cb), cbmax = fmaf(lbmax, (float)(4 * PITCH), cb);
#pragma unroll
            for (int k = 0; k < BPL_NZ; ++k) {
                // the row coordinate comes from the voxel's absolute height (independent of the
                // tile and slab the voxel is processed in)
                const float bs = fmaf(zk[k], mv, A.bv0);
                const float bf = floorf(bs);
                const float fb = bs - bf;
                const float off = __builtin_amdgcn_fmed3f(fmaf(bf, (float)(4 * PITCH), cbr), cb, cbmax);
                const float *t = (const float *)((const char *)win + (int)off);
                const float v0 = fmaf(wa1, t[1], wa0 * t[0]);
                const float v1 = fmaf(wa1, t[PITCH + 1], wa0 * t[PITCH]);
                const float v = fmaf(fb, v1 - v0, v0);
                float wk = w;
                if (W != CT_BP_FDK) wk = wpm * sqrtf(fmaf(zk[k], zk[k], rxy2));
                acc[k] = fmaf(wk, v, acc[k]);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < BPL_NZ; ++k) {
        const int kk = kb + k;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        vol[o] = from_f<TV>(acc[k]);
    }
}

// Exact transpose of the Siddon projector, gathered per voxel.
//
// For one angle and one detector column a, every ray lies in the vertical plane through the source
// and that column, so all rows share the (x, y) trace and its parameter interval [t0, t0 + T] inside
// the voxel column's square.  The trace is clipped in a frame centred on the column: only the
// signed distance of the column centre from the trace (a 2-D cross product of ~1e3 mm vectors,
// which cancels) is formed in FP64; the clip itself works on O(1 mm) local quantities in FP32.
// Along row b the height is z(t) = t v_b (the source is in the z = 0 plane), so inside the column
// the row covers [t0 v_b, (t0 + T) v_b]: a short segment, sorted in z by b.  Each candidate row is
// visited once per column; its exact chord goes to the voxel of the thread's z run that holds it, or
// is split in proportion to height when it crosses a voxel face.  Voxel ranges are computed from
// absolute indices, so a voxel's sum does not depend on how the volume is cut into launches or
// slabs.  The per-voxel sums live in LDS (one slot per thread per voxel, conflict-free) and are
// added in a fixed order (angle, a, b): deterministic.
constexpr int ADJ_NZ = CT_ADJ_NZ;  // voxels per thread (exact adjoint)

template <typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_adjoint(const TP *__restrict__ proj, TV *__restrict__ vol, BpArgs A) {
    __shared__ float accs[ADJ_NZ * 256];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * BP_TX + (tid % BP_TX);
    const int j = blockIdx.y * BP_TY + (tid / BP_TX);
    const int kb = A.own_lo + blockIdx.z * ADJ_NZ;
    const bool live = i < A.nx && j < A.ny;
#pragma unroll
    for (int k = 0; k < ADJ_NZ; ++k) {
        const int kk = kb + k;
        accs[k * 256 + tid] = (live && A.accumulate && kk < A.own_hi)
                                  ? to_f(vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i])
                                  : 0.0f;
    }
    if (!live) return;  // no barrier follows: each thread owns its LDS slots
    const double xc = A.dx0 + i * A.ddx, yc = A.dy0 + j * A.ddy;  // column centre (mm)
    const float hx = 0.5f * A.dx, hy = 0.5f * A.dy;
    const float fxc = (float)xc, fyc = (float)yc;
    const float zface0 = (float)(A.dz0 - 0.5 * A.ddz);  // lower face of voxel 0
    const float dz = A.dz, idz = 1.0f / A.dz;
    const int nzr = min(ADJ_NZ, A.own_hi - kb);
    const float zl0 = fmaf((float)kb, dz, zface0), zr_hi = fmaf((float)(kb + nzr), dz, zface0);
    const float v0 = (float)(A.offv - A.cv * A.dv), dv = (float)A.dv, idv = 1.0f / dv;
    const float aum = (float)(A.cu - A.offu / A.du), iau = (float)(1.0 / A.du);
    const int64_t psz = (int64_t)A.nu * A.nv;
    constexpr int ES = (int)sizeof(TP);
    const int rowb = A.nu * ES;
    for (int t = 0; t < A.nang; ++t) {
        const AngleGeo &G = A.tab[A.a0 + t];
        const double c = G.c, s = G.s;
        const double Wx = xc - A.dDSO * c, Wy = yc - A.dDSO * s;  // source -> column centre
        const float fc = (float)c, fs = (float)s;
        // detector columns whose rays can meet the square: central projection of its corners
        // (FP32 with a margin: the range only has to contain every hit column)
        float umin = FLT_MAX, umax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float X = fxc + ((q & 1) ? hx : -hx), Y = fyc + ((q & 2) ? hy : -hy);
            const float u = A.DSD * (Y * fc - X * fs) * __builtin_amdgcn_rcpf(A.DSO - (X * fc + Y * fs));
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
        const int alo = (int)fmaxf(ceilf(fmaf(umin, iau, aum) - 1e-3f), 0.0f);
        const int ahi = (int)fminf(floorf(fmaf(umax, iau, aum) + 1e-3f), (float)(A.nu - 1));
        const __amdgpu_buffer_rsrc_t R = proj_rsrc(proj + (int64_t)t * psz, psz * ES);
        for (int a = alo; a <= ahi; ++a) {
            const double ua = (a - A.cu) * A.du + A.offu;
            // (x, y) direction of the rays of column a: P - S = -DSD (c, s) + ua (-s, c)
            const double Dx = -A.dDSD * c - ua * s, Dy = -A.dDSD * s + ua * c;
            const float cross = (float)(Wx * Dy - Wy * Dx);   // = |D| * signed distance
            const float dotp = (float)(Wx * Dx + Wy * Dy);    // = |D|^2 * t of the closest point
            const float fDx = (float)Dx, fDy = (float)Dy;
            const float L2 = fmaf(fDx, fDx, fDy * fDy);
            const float iL = __builtin_amdgcn_rsqf(L2);
            const float ux = fDx * iL, uy = fDy * iL;
            const float dperp = cross * iL;
            // closest point of the trace to the column centre, relative to the centre
            const float fx = -dperp * uy, fy = dperp * ux;
            // slab clip of fx + s ux in [-hx, hx], fy + s uy in [-hy, hy]  (s in mm)
            float s0 = -FLT_MAX, s1 = FLT_MAX;
            if (fabsf(ux) > 1e-7f) {
                const float r = __builtin_amdgcn_rcpf(ux);
                const float qa = (-hx - fx) * r, qb = (hx - fx) * r;
                s0 = fmaxf(s0, fminf(qa, qb));
                s1 = fminf(s1, fmaxf(qa, qb));
            } else if (fabsf(fx) > hx) {
                continue;
            }
            if (fabsf(uy) > 1e-7f) {
                const float r = __builtin_amdgcn_rcpf(uy);
                const float qa = (-hy - fy) * r, qb = (hy - fy) * r;
                s0 = fmaxf(s0, fminf(qa, qb));
                s1 = fminf(s1, fmaxf(qa, qb));
            } else if (fabsf(fy) > hy) {
                continue;
            }
            if (!(s0 < s1)) continue;
            const float T = (s1 - s0) * iL;                       // t-length inside the column
            const float t0 = fmaf(s0, iL, dotp * (iL * iL));      // t where the trace enters
            const float t1 = t0 + T;
            // rows whose height range inside the column meets the thread's z run [zl0, zr_hi]
            const float it0 = __builtin_amdgcn_rcpf(t0), it1 = __builtin_amdgcn_rcpf(t1);
            const float vmin = fminf(zl0 * it0, zl0 * it1), vmax = fmaxf(zr_hi * it0, zr_hi * it1);
            const int blo = (int)fmaxf(ceilf((vmin - v0) * idv - 1e-3f), 0.0f);
            const int bhi = (int)fminf(floorf((vmax - v0) * idv + 1e-3f), (float)(A.nv - 1));
            int off = blo * rowb + a * ES;
            for (int b = blo; b <= bhi; ++b, off += rowb) {
                const float y = bload(R, off, (TP *)nullptr);
                const float vb = fmaf((float)b, dv, v0);
                const float za = t0 * vb;            // height where the row enters the column
                const float ext = T * vb;            // signed height change across the column
                const float lo = fminf(za, za + ext), hi = fmaxf(za, za + ext);
                const float full = T * sqrtf(fmaf(vb, vb, L2));   // chord inside the column
                const int klo = (int)floorf((lo - zface0) * idz) - kb;
                const int khi = (int)floorf((hi - zface0) * idz) - kb;
                if (klo == khi) {
                    // the row stays inside one voxel
                    if ((unsigned)klo < (unsigned)nzr) accs[klo * 256 + tid] = fmaf(full, y, accs[klo * 256 + tid]);
                } else {
                    const float iext = __builtin_amdgcn_rcpf(hi - lo);
                    const int ke = min(khi, nzr - 1);
                    for (int k = max(klo, 0); k <= ke; ++k) {
                        const float zl = fmaf((float)(kb + k), dz, zface0);
                        const float ov = fmaxf(fminf(hi, zl + dz) - fmaxf(lo, zl), 0.0f);
                        accs[k * 256 + tid] = fmaf(full * (ov * iext), y, accs[k * 256 + tid]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < ADJ_NZ; ++k) {
        const int kk = kb + k;
        if (kk >= A.own_hi) break;
        const int64_t o = ((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i;
        vol[o] = from_f<TV>(accs[k * 256 + tid]);
    }
}

// ------------------------------------------------------------------------------------------
// Exact adjoint with lanes on the voxels of one column (resident launches).
//
// A wave takes one voxel column and 64 * R of its voxels (lane = voxel; a lane's R voxels are 64
// apart), so the candidate detector columns of every angle and the column's parameter interval
// [t0, t1] on each of them are the same in all lanes: the FP64 clip is computed once per wave.
// Along the ray of row b the height is z = t v_b, so voxel [zl, zh) is met for t in
// [zl / v_b, zh / v_b] (ordered) clipped to [t0, t1]; the rows that can meet it have v_b in
// [min(zl / t0, zl / t1), max(zh / t0, zh / t1)], at most NR consecutive rows (NR from a host
// bound).  The projections are read from a copy [angle][u][1 + v] of pairs (y |P - S|, 1 / v_b)
// with a zero row below and above each column, so the rows of consecutive voxels are consecutive
// addresses and every row costs one 8-byte load, two products and four compares.

// proj [angle][v][u] -> yq [angle][u][v + 1] (nv + 2 rows, zero first and last), 32 x 32 tiles
template <typename TP>
__global__ __launch_bounds__(256) void k_adj_prep(const TP *__restrict__ proj, float2 *__restrict__ yq, BpArgs A) {
    __shared__ float tile[32][33];
    const int u0 = blockIdx.x * 32, r0 = blockIdx.y * 32, t = blockIdx.z;  // r = b + 1
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int nvp = A.nv + 2;
    const TP *pt = proj + (int64_t)t * A.nu * A.nv;
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int u = u0 + tx, b = r0 + ty + k - 1;
        float y = 0.0f;
        if (u < A.nu && b >= 0 && b < A.nv) y = to_f(pt[(int64_t)b * A.nu + u]);
        tile[ty + k][tx] = y;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int r = r0 + tx, u = u0 + ty + k;
        if (u < A.nu && r < nvp) {
            const int b = r - 1;
            float2 q = make_float2(0.0f, 0.0f);
            if (b >= 0 && b < A.nv) {
                const double ua = (u - A.cu) * A.du + A.offu, vb = (b - A.cv) * A.dv + A.offv;
                // |P - S| (mm per unit t) is the same for every angle in a circular orbit
                q.x = (float)(tile[tx][ty + k] * sqrt(A.dDSD * A.dDSD + ua * ua + vb * vb));
                q.y = vb != 0.0 ? (float)(1.0 / vb) : 1e30f;
            }
            yq[((int64_t)t * A.nu + u) * nvp + r] = q;
        }
    }
}

// ZC: the volume is a column-major slab of A.zcol_n slots per column (else [z][y][x] slices).
// ORD: no voxel of the launch has its lower face below the source plane z = 0 and its upper face
// above it.  A voxel above the plane is only met by rows climbing from the source (v_b > 0), for
// which zl / v_b < zh / v_b, and a voxel below only by falling rows, for which the order flips; the
// kernel then orders each voxel's faces once (za, zb) instead of ordering the two parameters of
// every row.  Rows of the other sign get an empty interval either way, so both forms give the same
// bits.
// at most 4 waves per SIMD: the compiler then keeps the row loads of all R voxels of a candidate
// column in flight together instead of two at a time (more registers, fewer exposed latencies)
#ifndef CT_ADJ_WAVES
#define CT_ADJ_WAVES 1, 4
#endif
#define CT_ADJ_OCC __attribute__((amdgpu_waves_per_eu(CT_ADJ_WAVES)))
template <typename TV, int R, int NR, bool ZC, bool ORD>
__global__ __launch_bounds__(256) CT_ADJ_OCC void k_adj_col(const float2 *__restrict__ yq, TV *__restrict__ vol, BpArgs A,
                                                 int zgroups, int xblocks) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    int bid = blockIdx.x;
#if CT_ADJ_XCD_W > 1
    // workgroups are dealt to the 8 XCDs in turn: give each XCD CT_ADJ_XCD_W consecutive blocks
    // (neighbouring columns, which read the same detector columns) out of every 8 * CT_ADJ_XCD_W
    {
        constexpr int W = CT_ADJ_XCD_W, C = 8 * W;
        const int full = (int)(gridDim.x / C) * C;
        if (bid < full) bid = (bid / C) * C + (bid % 8) * W + (bid % C) / 8;
    }
#endif
    const int zg = bid % zgroups;
    bid /= zgroups;
    const int i = (bid % xblocks) * 4 + wave;
    const int j = bid / xblocks;
    if (i >= A.nx) return;  // whole wave; no barriers follow
    const float zface0 = (float)(A.dz0 - 0.5 * A.ddz);  // lower face of voxel 0
    const float dz = A.dz;
    // voxel k of this column: a slice of a [z][y][x] volume, or a slot of a column-major slab
    // (lanes then read and write consecutive addresses)
    auto vidx = [&](int k) -> int64_t {
        return ZC ? ((int64_t)j * A.nx + i) * A.zcol_n + (k - A.mem_lo)
                  : ((int64_t)(k - A.mem_lo) * A.ny + j) * A.nx + i;
    };
    // za, zb: the voxel's faces in the order its rows reach them (lower face first unless ORD and
    // the voxel lies below the source plane)
    float acc[R], za[R], zb[R];
    bool kin[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = A.own_lo + zg * 64 * R + 64 * r + lane;
        kin[r] = k < A.own_hi;
        const float zl = fmaf((float)k, dz, zface0), zh = fmaf((float)(k + 1), dz, zface0);
        const bool flip = ORD && zh <= 0.0f;
        za[r] = flip ? zh : zl;
        zb[r] = flip ? zl : zh;
        const int64_t o = vidx(k);
        acc[r] = (kin[r] && A.accumulate) ? to_f(vol[o]) : 0.0f;
    }
    const double xc = A.dx0 + i * A.ddx, yc = A.dy0 + j * A.ddy;  // column centre (mm)
    const float hx = 0.5f * A.dx, hy = 0.5f * A.dy;
    const float fxc = (float)xc, fyc = (float)yc;
    const float v0 = (float)(A.offv - A.cv * A.dv), idv = 1.0f / (float)A.dv;
    const float nv0 = -v0 * idv;
    const float bmax = (float)(A.nv + 1 - NR);
    const float aum = (float)(A.cu - A.offu / A.du), iau = (float)(1.0 / A.du);
    const int nvp = A.nv + 2;
    for (int t = 0; t < A.nang; ++t) {
        const AngleGeo &G = A.tab[A.a0 + t];
        const double c = G.c, s = G.s;
        const double Wx = xc - A.dDSO * c, Wy = yc - A.dDSO * s;  // source -> column centre
        const float fc = (float)c, fs = (float)s;
        float umin = FLT_MAX, umax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float X = fxc + ((q & 1) ? hx : -hx), Y = fyc + ((q & 2) ? hy : -hy);
            const float u = A.DSD * (Y * fc - X * fs) * __builtin_amdgcn_rcpf(A.DSO - (X * fc + Y * fs));
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
        const int alo = (int)fmaxf(ceilf(fmaf(umin, iau, aum) - 1e-3f), 0.0f);
        const int ahi = (int)fminf(floorf(fmaf(umax, iau, aum) + 1e-3f), (float)(A.nu - 1));
        for (int a = alo; a <= ahi; ++a) {
            const double ua = (a - A.cu) * A.du + A.offu;
            const double Dx = -A.dDSD * c - ua * s, Dy = -A.dDSD * s + ua * c;
            const float cross = (float)(Wx * Dy - Wy * Dx);
            const float dotp = (float)(Wx * Dx + Wy * Dy);
            const float fDx = (float)Dx, fDy = (float)Dy;
            const float L2 = fmaf(fDx, fDx, fDy * fDy);
            const float iL = __builtin_amdgcn_rsqf(L2);
            const float ux = fDx * iL, uy = fDy * iL;
            const float dperp = cross * iL;
            const float fx = -dperp * uy, fy = dperp * ux;
            float s0 = -FLT_MAX, s1 = FLT_MAX;
            if (fabsf(ux) > 1e-7f) {
                const float rr = __builtin_amdgcn_rcpf(ux);
                const float qa = (-hx - fx) * rr, qb = (hx - fx) * rr;
                s0 = fmaxf(s0, fminf(qa, qb));
                s1 = fminf(s1, fmaxf(qa, qb));
            } else if (fabsf(fx) > hx) {
                continue;
            }
            if (fabsf(uy) > 1e-7f) {
                const float rr = __builtin_amdgcn_rcpf(uy);
                const float qa = (-hy - fy) * rr, qb = (hy - fy) * rr;
                s0 = fmaxf(s0, fminf(qa, qb));
                s1 = fminf(s1, fmaxf(qa, qb));
            } else if (fabsf(fy) > hy) {
                continue;
            }
            if (!(s0 < s1)) continue;
            const float T = (s1 - s0) * iL;
            const float t0 = fmaf(s0, iL, dotp * (iL * iL));
            const float it0 = __builtin_amdgcn_rcpf(t0), it1 = __builtin_amdgcn_rcpf(t0 + T);
            const float2 *col = yq + ((int64_t)t * A.nu + a) * nvp;  // row b at col[b + 1]
            // the rows of all R voxels are loaded first, so their loads are in flight together
            float2 wv[R][NR];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // first row that can meet the voxel, kept inside [-1, nv + 1 - NR]: the lowest
                // v = z / t over the lower face and t in [t0, t1] (with ORD, za * it1 for voxels
                // above the plane and zb * it0 for voxels below)
                const float vlo = ORD ? fminf(za[r] * it1, zb[r] * it0) : fminf(za[r] * it0, za[r] * it1);
                const float bl = __builtin_amdgcn_fmed3f(ceilf(fmaf(vlo, idv, nv0)), -1.0f, bmax);
                // uniform column base plus an unsigned 32-bit byte offset of row bl
                const float2 *cb = (const float2 *)((const char *)col + (uint32_t)((int)bl + 1) * 8u);
#pragma unroll
                for (int q = 0; q < NR; ++q) wv[r][q] = cb[q];
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const float2 w = wv[r][q];
                    // parameters relative to t0 (one rounding each), clipped to [0, T]: a row that
                    // stays inside the voxel gets exactly T
                    const float tA = fmaf(za[r], w.y, -t0), tB = fmaf(zb[r], w.y, -t0);
                    float len;
                    if (ORD) {
                        // tA <= tB for the rows that can meet the voxel; rows of the other sign have
                        // both parameters below 0, which clamp to the same value
                        len = __builtin_amdgcn_fmed3f(tB, 0.0f, T) - __builtin_amdgcn_fmed3f(tA, 0.0f, T);
                    } else {
                        const float lo = fmaxf(fminf(tA, tB), 0.0f), hi = fminf(fmaxf(tA, tB), T);
                        len = fmaxf(hi - lo, 0.0f);
                    }
                    acc[r] = fmaf(len, w.x, acc[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!kin[r]) continue;
        const int k = A.own_lo + zg * 64 * R + 64 * r + lane;
        const int64_t o = vidx(k);
        vol[o] = from_f<TV>(acc[r]);
    }
}

// SART update for one angle t with FDK weights:
//   x_j += lambda * (w_j * bilinear(r)) / (w_j * bilinear(1))   where w_j * bilinear(1) > 1e-6
__global__ __launch_bounds__(256) void k_sart_update(const float *__restrict__ r, float *__restrict__ vol,
                                                     BpArgs A, float lambda) {
    const int i = blockIdx.x * BP_TX + (threadIdx.x % BP_TX);
    const int j = blockIdx.y * BP_TY + (threadIdx.x / BP_TX);
    const int kb = blockIdx.z * BP_NZ;
    if (i >= A.nx || j >= A.ny) return;
    const float x = fmaf((float)i, A.dx, A.x0);
    const float y = fmaf((float)j, A.dy, A.y0);
    const int64_t pix = (int64_t)A.nu * A.nv;
    // sums over the subset's angles, in angle order
    float num[BP_NZ], V[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) num[k] = V[k] = 0.0f;
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
        const float q = A.DSO * iL;
        const float w = q * q;
        const float *rt = r + t * pix;
#pragma unroll
        for (int k = 0; k < BP_NZ; ++k) {
            const int kk = min(kb + k, A.nz - 1);
            const float z = fmaf((float)kk, A.dz, A.z0);
            const float bs = fmaf(m * z, A.inv_dv, A.bv0);
            const float bf = floorf(bs);
            const float fb = bs - bf;
            const int ib = (int)bf;
            const float wb0 = ((unsigned)ib < (unsigned)A.nv) ? 1.0f - fb : 0.0f;
            const float wb1 = ((unsigned)(ib + 1) < (unsigned)A.nv) ? fb : 0.0f;
            const int r0 = clampi(ib, 0, A.nv - 1) * A.nu, r1 = clampi(ib + 1, 0, A.nv - 1) * A.nu;
            const float v0 = fmaf(wa1, rt[r0 + ia1], wa0 * rt[r0 + ia0]);
            const float v1 = fmaf(wa1, rt[r1 + ia1], wa0 * rt[r1 + ia0]);
            num[k] += w * fmaf(wb1, v1, wb0 * v0);
            V[k] += w * ((wa0 + wa1) * (wb0 + wb1));
        }
    }
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.nz && V[k] > 1e-6f) {
            const int64_t o = ((int64_t)kk * A.ny + j) * A.nx + i;
            vol[o] = fmaf(lambda, num[k] / V[k], vol[o]);
        }
    }
}

// The same update on the column-major copy ([y][x][slot], slot k + 1 = voxel k) with the residual
// transposed to [u][v].
#ifndef CT_SART_R
#define CT_SART_R 8
#endif
constexpr int SART_R = CT_SART_R;  // voxels per lane of the column update

// One wave per voxel column and group of 64 SART_R heights (lane = height, SART_R heights 64 apart):
// the column's detector coordinate, FDK weight and column taps are set up once, and the lanes read
// the transposed residual rT[u][v] at consecutive rows and update consecutive slots of the
// column-major copy.
__global__ __launch_bounds__(256) void k_sart_update_col(const float *__restrict__ rT, float *__restrict__ vz,
                                                         BpArgs A, float lambda, int zwaves) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
    const int64_t col = gw / zwaves;
    if (col >= (int64_t)A.nx * A.ny) return;
    const int kk0 = (int)(gw % zwaves) * 64 * SART_R + (threadIdx.x & 63);
    const int i = (int)(col % A.nx), j = (int)(col / A.nx);
    const float x = fmaf((float)i, A.dx, A.x0);
    const float y = fmaf((float)j, A.dy, A.y0);
    const int64_t pix = (int64_t)A.nu * A.nv;
    float *vc = vz + col * (A.nz + 2) + 1;
    // the voxels' values are read first, so their loads overlap the first angle's taps
    float xo[SART_R];
#pragma unroll
    for (int r = 0; r < SART_R; ++r) xo[r] = vc[min(kk0 + 64 * r, A.nz - 1)];
    // sums over the subset's angles, in angle order
    float num[SART_R], V[SART_R];
#pragma unroll
    for (int r = 0; r < SART_R; ++r) num[r] = V[r] = 0.0f;
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
        const float *rt = rT + t * pix;
        const float *r0 = rt + (int64_t)clampi(ia, 0, A.nu - 1) * A.nv;
        const float *r1 = rt + (int64_t)clampi(ia + 1, 0, A.nu - 1) * A.nv;
        const float q = A.DSO * iL;
        const float w = q * q;
        const float wva = w * (wa0 + wa1);
        const float mv = m * A.inv_dv;
        // all taps of the wave's SART_R heights first (heights clamped into the column), then the sums
        float wb0[SART_R], wb1[SART_R], t00[SART_R], t01[SART_R], t10[SART_R], t11[SART_R];
#pragma unroll
        for (int r = 0; r < SART_R; ++r) {
            const int kk = min(kk0 + 64 * r, A.nz - 1);
            const float z = fmaf((float)kk, A.dz, A.z0);
            const float bs = fmaf(z, mv, A.bv0);
            const float bf = floorf(bs);
            const float fb = bs - bf;
            const int ib = (int)bf;
            wb0[r] = ((unsigned)ib < (unsigned)A.nv) ? 1.0f - fb : 0.0f;
            wb1[r] = ((unsigned)(ib + 1) < (unsigned)A.nv) ? fb : 0.0f;
            const int b0 = clampi(ib, 0, A.nv - 1), b1 = clampi(ib + 1, 0, A.nv - 1);
            t00[r] = r0[b0];
            t10[r] = r1[b0];
            t01[r] = r0[b1];
            t11[r] = r1[b1];
        }
#pragma unroll
        for (int r = 0; r < SART_R; ++r) {
            const float v0 = fmaf(wa1, t10[r], wa0 * t00[r]);
            const float v1 = fmaf(wa1, t11[r], wa0 * t01[r]);
            num[r] += w * fmaf(wb1[r], v1, wb0[r] * v0);
            V[r] += wva * (wb0[r] + wb1[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < SART_R; ++r) {
        const int kk = kk0 + 64 * r;
        // num / V through the hardware reciprocal (within 1 ulp)
        if (kk < A.nz && V[r] > 1e-6f) vc[kk] = fmaf(lambda, num[r] * __builtin_amdgcn_rcpf(V[r]), xo[r]);
    }
}

// Detector window (columns WW, rows HW) that holds the taps of one 16 x 16 x BP_NZ tile under any
// angle, or false when it does not fit the staging buffer.  For two points of the tile the
// detector coordinate u = m t (t transverse to the ray, m = DSD / depth) differs by at most
// m_max |dt| + |t|_max |dm| with |dt| <= D (the tile's xy diagonal) and
// |dm| <= DSD D / (DSO - R)^2, R bounding the distance of any voxel from the axis; likewise
// for v = m z with the tile's z extent.  Margins: one pixel each side plus the second tap.
bool bp_window(const ct_geometry &g, int &WW, int &HW) {
    double R = 0.0, Zmax = 0.0;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy) {
            const double xe = g.offOrigin[0] + (cx ? 0.5 : -0.5) * g.nVoxel[0] * g.dVoxel[0];
            const double ye = g.offOrigin[1] + (cy ? 0.5 : -0.5) * g.nVoxel[1] * g.dVoxel[1];
            R = std::max(R, std::sqrt(xe * xe + ye * ye));
        }
    for (int cz = 0; cz < 2; ++cz)
        Zmax = std::max(Zmax, std::fabs(g.offOrigin[2] + (cz ? 0.5 : -0.5) * g.nVoxel[2] * g.dVoxel[2]));
    const double D = std::sqrt(std::pow((BP_TX - 1) * g.dVoxel[0], 2) + std::pow((BP_TY - 1) * g.dVoxel[1], 2));
    // corners of edge tiles may lie up to one tile outside the grid
    R += D;
    Zmax += BPL_NZ * g.dVoxel[2];
    if (!(g.DSO - R > 0.0)) return false;
    const double mmax = g.DSD / (g.DSO - R);
    const double dm = g.DSD * D / ((g.DSO - R) * (g.DSO - R));
    const double eu = (mmax * D + R * dm) / g.dDetector[0];
    const double ev = (mmax * (BPL_NZ - 1) * g.dVoxel[2] + Zmax * dm) / g.dDetector[1];
    if (!(eu < 60.0 && ev < 1000.0)) return false;
    WW = (int)std::ceil(eu) + 4;
    HW = (int)std::ceil(ev) + 4;
    return WW <= 64 && (WW <= BPL_PN ? BPL_PN : 64) * HW <= BPL_FLOATS;
}

// Rows of one detector column that can meet one voxel, at most: the heights z of the voxel and
// the ray parameters t in the voxel column give v = z / t over an interval of width at most
// (dz / t_min + |z|_max (1/t0 - 1/t1)) / dv, with t_min = (DSO - R) / DSD and
// t1 - t0 <= sqrt(2) max(dx, dy) / DSD, R bounding the distance of any voxel from the axis.  An
// interval of width W holds at most floor(W) + 1 integers.
int adj_rows(const ct_geometry &g) {
    double R = 0.0, Zmax = 0.0;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy) {
            const double xe = g.offOrigin[0] + (cx ? 0.5 : -0.5) * g.nVoxel[0] * g.dVoxel[0];
            const double ye = g.offOrigin[1] + (cy ? 0.5 : -0.5) * g.nVoxel[1] * g.dVoxel[1];
            R = std::max(R, std::sqrt(xe * xe + ye * ye));
        }
    for (int cz = 0; cz < 2; ++cz)
        Zmax = std::max(Zmax, std::fabs(g.offOrigin[2] + (cz ? 0.5 : -0.5) * g.nVoxel[2] * g.dVoxel[2]));
    if (!(g.DSO - R > 0.0)) return 1 << 20;
    const double tmin = (g.DSO - R) / g.DSD;
    const double dt = std::sqrt(2.0) * std::max(g.dVoxel[0], g.dVoxel[1]) / g.DSD;
    const double W = (g.dVoxel[2] / tmin + Zmax * dt / (tmin * tmin)) / g.dDetector[1];
    return (int)std::floor(W * 1.001 + 1e-3) + 1;
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
    A.zcol_n = slab.zcol ? (int32_t)slab.mem_n : 0;
    A.accumulate = accumulate;
    return A;
}

}  // namespace

bool adj_col_ok(const ct_plan *p) {
#ifdef CT_NO_ADJ_COL
    return false;
#else
    return std::min<int>(adj_rows(p->g), (int)p->g.nDetector[1] + 2) <= 4;
#endif
}

size_t adj_chunk_bytes_per_angle(const ct_geometry &g) {
    return (size_t)g.nDetector[0] * (size_t)(g.nDetector[1] + 2) * sizeof(float2);
}

ct_status launch_backproject(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                             ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab, hipStream_t st,
                             void *adj_scratch, size_t adj_bytes) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    const int64_t nzown = slab.own_hi - slab.own_lo;
    if (nzown <= 0) return CT_OK;
    if (slab.zcol && (kind != CT_BP_ADJOINT || !adj_col_ok(p)))
        return fail(CT_ERR_STATE, "a column-major slab needs the exact adjoint's column kernel");
    BpArgs A = make_bp_args(p, tab, a0, a1, slab, accumulate);
    const int nzrun = kind == CT_BP_ADJOINT ? ADJ_NZ : BP_NZ;
    const dim3 grid((A.nx + BP_TX - 1) / BP_TX, (A.ny + BP_TY - 1) / BP_TY, (unsigned)((nzown + nzrun - 1) / nzrun));
    const dim3 block(256);
    int WW = 0, HW = 0;
#ifndef CT_NO_BP_LDS
    if (kind != CT_BP_ADJOINT && bp_window(p->g, WW, HW)) {
        const bool narrow = WW <= BPL_PN;
        const int K = std::min(BPL_K, BPL_FLOATS / ((narrow ? BPL_PN : 64) * HW));
        const dim3 lgrid(grid.x, grid.y, (unsigned)((nzown + BPL_NZ - 1) / BPL_NZ));
#define CT_BPL(KIND, PITCH)                                                                                      \
    CT_DISPATCH2(pt, TP, vt, TV,                                                                                 \
                 hipLaunchKernelGGL((k_bp_lds<KIND, PITCH, TP, TV>), lgrid, block, 0, st, (const TP *)proj,        \
                                    (TV *)vol, A, WW, HW, K))
        if (kind == CT_BP_FDK) {
            if (narrow) {
                CT_BPL(CT_BP_FDK, BPL_PN);
            } else {
                CT_BPL(CT_BP_FDK, 64);
            }
        } else {
            if (narrow) {
                CT_BPL(CT_BP_PSEUDO_MATCHED, BPL_PN);
            } else {
                CT_BPL(CT_BP_PSEUDO_MATCHED, 64);
            }
        }
#undef CT_BPL
        CT_HIP(hipGetLastError());
        return CT_OK;
    }
#endif
    if (kind == CT_BP_FDK) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_voxel<CT_BP_FDK, TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    } else if (kind == CT_BP_PSEUDO_MATCHED) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_voxel<CT_BP_PSEUDO_MATCHED, TP, TV>), grid, block, 0, st, (const TP *)proj,
                                        (TV *)vol, A));
    } else {
#ifndef CT_NO_ADJ_COL
        // voxel lanes over a transposed, pre-scaled copy of the projections, made in angle
        // sub-chunks that fit the scratch (the caller's, else stream-ordered scratch of the whole
        // range when the launch may allocate); accumulators pass between sub-chunks in FP32
        const int nr = std::min<int>(adj_rows(p->g), (int)p->g.nDetector[1] + 2);
        const size_t per_angle = adj_chunk_bytes_per_angle(p->g);
        void *yq = adj_scratch, *own = nullptr;
        size_t qcap = adj_scratch ? adj_bytes : 0;
        if (nr <= 4 && !yq && slab.scratch_ok) {
            if (hipMallocAsync(&own, (size_t)(a1 - a0) * per_angle, st) == hipSuccess) {
                yq = own;
                qcap = (size_t)(a1 - a0) * per_angle;
            } else {
                (void)hipGetLastError();
            }
        }
        if (nr <= 4 && yq && qcap >= per_angle) {
            const int64_t kq = std::min<int64_t>(a1 - a0, (int64_t)(qcap / per_angle));
            // voxels per lane R: a wave covers 64 R voxels of its column and sets up each (angle,
            // detector column) once for them, which costs about 2/R of the per-voxel work; pick the
            // R that minimises (voxels covered, idle lanes included) x (1 + 2/R)
            int R = 8;
            double best = DBL_MAX;
            for (int r : {8, 6, 4, 2, 1}) {
                const int64_t covered = (nzown + 64 * r - 1) / (64 * r) * (64 * r);
                const double cost = (double)covered * (1.0 + 2.0 / r);
                if (cost < best) {  // ties keep the larger R
                    best = cost;
                    R = r;
                }
            }
#ifdef CT_ADJ_R
            R = CT_ADJ_R;
#endif
            // no voxel of the launch straddles the source plane (the kernel's own FP32 faces)
            bool ord = true;
            {
                const float dzf = A.dz, zf0 = (float)(A.dz0 - 0.5 * A.ddz);
                for (int64_t k = slab.own_lo; k < slab.own_hi && ord; ++k)
                    ord = !(std::fma((float)k, dzf, zf0) < 0.0f && std::fma((float)(k + 1), dzf, zf0) > 0.0f);
            }
            const int zgroups = (int)((nzown + 64 * R - 1) / (64 * R));
            const int xblocks = (A.nx + 3) / 4;
            const dim3 ag((unsigned)((int64_t)zgroups * xblocks * A.ny));
            const size_t pangle = (size_t)A.nu * A.nv * dtype_size(pt);
            for (int64_t c0 = a0; c0 < a1; c0 += kq) {
                const int64_t c1 = std::min(a1, c0 + kq);
                const BpArgs Ac = make_bp_args(p, tab, c0, c1, slab, c0 == a0 ? accumulate : 1);
                const void *pc = (const char *)proj + (size_t)(c0 - a0) * pangle;
                const dim3 pg((unsigned)((A.nu + 31) / 32), (unsigned)((A.nv + 2 + 31) / 32), (unsigned)(c1 - c0));
                CT_DISPATCH1(pt, TP,
                             hipLaunchKernelGGL((k_adj_prep<TP>), pg, dim3(256), 0, st, (const TP *)pc, (float2 *)yq, Ac));
                CT_HIP(hipGetLastError());
#define CT_ADJ_L(RR, NN, Z, O)                                                                                  \
    hipLaunchKernelGGL((k_adj_col<TV, RR, NN, Z, O>), ag, block, 0, st, (const float2 *)yq, (TV *)vol, Ac, zgroups, \
                       xblocks)
#define CT_ADJ(RR, NN)                                  \
    CT_DISPATCH1(vt, TV, if (slab.zcol) {               \
        if (ord) CT_ADJ_L(RR, NN, true, true);          \
        else CT_ADJ_L(RR, NN, true, false);             \
    } else {                                            \
        if (ord) CT_ADJ_L(RR, NN, false, true);         \
        else CT_ADJ_L(RR, NN, false, false);            \
    })
#define CT_ADJ_R(NN)        \
    switch (R) {            \
        case 1:             \
            CT_ADJ(1, NN);  \
            break;          \
        case 2:             \
            CT_ADJ(2, NN);  \
            break;          \
        case 4:             \
            CT_ADJ(4, NN);  \
            break;          \
        case 6:             \
            CT_ADJ(6, NN);  \
            break;          \
        default:            \
            CT_ADJ(8, NN);  \
            break;          \
    }
                if (nr <= 2) {
                    CT_ADJ_R(2);
                } else if (nr == 3) {
                    CT_ADJ_R(3);
                } else {
                    CT_ADJ_R(4);
                }
#undef CT_ADJ_R
#undef CT_ADJ
#undef CT_ADJ_L
                CT_HIP(hipGetLastError());
            }
            if (own) CT_HIP(hipFreeAsync(own, st));
            return CT_OK;
        }
        if (own) CT_HIP(hipFreeAsync(own, st));
        if (slab.zcol) return fail(CT_ERR_STATE, "a column-major slab needs the exact adjoint's scratch");
#endif
        if (slab.zcol) return fail(CT_ERR_STATE, "a column-major slab needs the exact adjoint's column kernel");
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_adjoint<TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_sart_update(ct_plan *p, const float *r, float *vol, int64_t a0, int64_t a1, float lambda,
                             hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    BpArgs A = make_bp_args(p, tab, a0, a1, full_slab(p->g), 1);
    const dim3 grid((A.nx + BP_TX - 1) / BP_TX, (A.ny + BP_TY - 1) / BP_TY, (unsigned)((A.nz + BP_NZ - 1) / BP_NZ));
    hipLaunchKernelGGL(k_sart_update, grid, dim3(256), 0, st, r, vol, A, lambda);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_sart_update_col(ct_plan *p, const float *rT, float *vz, int64_t a0, int64_t a1, float lambda,
                                 hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    BpArgs A = make_bp_args(p, tab, a0, a1, full_slab(p->g), 1);
    const int zwaves = (A.nz + 64 * SART_R - 1) / (64 * SART_R);
    const int64_t waves = (int64_t)A.nx * A.ny * zwaves;
    hipLaunchKernelGGL(k_sart_update_col, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, rT, vz, A, lambda,
                       zwaves);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

}  // namespace ct
