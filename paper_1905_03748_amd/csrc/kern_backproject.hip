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
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

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
    double dau0, dbv0;      // au0, bv0 in FP64
    double idu, idv;        // 1 / du, 1 / dv in FP64
    int32_t vw;             // a plan of vertical views: the exact adjoint takes each view's S, C - S, e_u
    int32_t zrow;           // the detector row at the source's height (v_b = 0, rays parallel to the
                            // slices), or -1
};

// 1 / d in FP64 without a division: the FP32 reciprocal (about 1 ulp) refined by one Newton step,
// which squares its relative error (to ~1e-14) for the positive, moderate d used here.
__device__ __forceinline__ double rcp_f64(double d) {
    const double r = (double)__builtin_amdgcn_rcpf((float)d);
    return r * fma(-d, r, 2.0);
}

// LDS written by some lanes of a wave and read by others: the wave's LDS accesses complete in
// order, so this only keeps the compiler from moving accesses across it
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Detector coordinates of the voxels of a tile, relative to a reference point of the tile.
//
// At a detector of more than 2048 pixels an FP32 coordinate a* ~ 3000 is only resolved to
// 2.4e-4 pixel, and the FP32 chain that forms it from mm-sized quantities (products of ~1e3 mm
// depths, a reciprocal) loses a few ulps more; on ramp-filtered data that shows as 2e-4 relative
// error of the backprojection.  Instead the tile's reference point (x_r, y_r, z_r) is projected
// once per angle in FP64 and each voxel adds a small FP32 offset:
//   with N = y c - x s and D = DSO - (x c + y s) (transverse position and depth of the voxel),
//   a* - a*_r = DSD / du * (N / D - N_r / D_r) = Ka (dN D_r - N_r dD) / D,  Ka = DSD / (du D_r)
//   b* - b*_r = DSD / dv * (z / D - z_r / D_r) = (z - z_r) m / dv + Kb dD / D,
//                                                    Kb = -DSD z_r / (dv D_r),  m = DSD / D
// where dN, dD, z - z_r are the voxel's offsets from the reference (a tile width or less), so every
// FP32 quantity is a few pixels in size.  Aloc, Bloc: the reference's coordinates minus an integer
// origin (the staging window's corner, or the floor of the reference coordinate).
struct TileRef {
    float c, s;      // cos, sin of the angle
    float Dr, Nr;    // depth and transverse position of the reference point, mm
    float Ka, Kb;
    float Aloc, Bloc;
};

// FP64 projection of the reference point (xr, yr, zr) (mm) under the angle (c, s); returns a*_r, b*_r
// and fills the FP32 factors (Aloc / Bloc are left to the caller).
__device__ __forceinline__ void tile_ref(const BpArgs &A, double c, double s, double xr, double yr, double zr,
                                         TileRef &R, double &ar, double &br) {
    const double N = yr * c - xr * s, D = A.dDSO - (xr * c + yr * s);
    const double iD = rcp_f64(D);
    const double ka = A.dDSD * iD * A.idu, kb = A.dDSD * iD * A.idv;
    ar = fma(ka, N, A.dau0);
    br = fma(kb, zr, A.dbv0);
    R.c = (float)c;
    R.s = (float)s;
    R.Dr = (float)D;
    R.Nr = (float)N;
    R.Ka = (float)ka;
    R.Kb = (float)(-kb * zr);
}

// Per-voxel part: the voxel's offset (lx, ly) (mm) from the reference gives the local column
// coordinate as, the row coordinate at the reference height bq (add zl * mv for a height zl above
// it) and 1 / D.
__device__ __forceinline__ void tile_local(const TileRef &R, float lx, float ly, float DSD, float inv_dv, float &as,
                                           float &bq, float &mv, float &iL) {
    const float dN = fmaf(ly, R.c, -lx * R.s);
    const float dD = -fmaf(lx, R.c, ly * R.s);
    iL = __builtin_amdgcn_rcpf(R.Dr + dD);
    const float T = fmaf(dN, R.Dr, -R.Nr * dD);
    as = fmaf(R.Ka * T, iL, R.Aloc);
    bq = fmaf(R.Kb * dD, iL, R.Bloc);
    mv = DSD * iL * inv_dv;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Reference point of a tile: the centre of its columns that lie in the grid and of its run of
// slices clipped to the grid.  It depends only on the tile and the run, not on the slab or launch,
// so a voxel's arithmetic is the same however the volume is cut; and it lies inside the volume box,
// so its depth is positive.
__device__ __forceinline__ float tile_mid(int first, int len, int n) { return 0.5f * (float)(first + min(first + len, n) - 1); }

// Runs of nrun slices start at absolute multiples of nrun (the first run of a slab may begin below
// own_lo; those voxels are neither read nor written).
__device__ __forceinline__ int run_base(const BpArgs &A, int nrun) { return (A.own_lo / nrun + (int)blockIdx.z) * nrun; }

template <int W, typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_voxel(const TP *__restrict__ proj, TV *__restrict__ vol, BpArgs A) {
    __shared__ TileRef ref[64];
    __shared__ float iref[64][2];
    const int i0 = blockIdx.x * BP_TX, j0 = blockIdx.y * BP_TY;
    const int i = i0 + (threadIdx.x % BP_TX);
    const int j = j0 + (threadIdx.x / BP_TX);
    const int kb = run_base(A, BP_NZ);
    const bool live = i < A.nx && j < A.ny;
    const float ir = tile_mid(i0, BP_TX, A.nx), jr = tile_mid(j0, BP_TY, A.ny), kr = tile_mid(kb, BP_NZ, A.nz);
    const float lx = ((float)i - ir) * A.dx, ly = ((float)j - jr) * A.dy;
    const float x = fmaf((float)i, A.dx, A.x0);
    const float y = fmaf((float)j, A.dy, A.y0);
    float zk[BP_NZ], zl[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        zk[k] = fmaf((float)(kb + k), A.dz, A.z0);
        zl[k] = ((float)(kb + k) - kr) * A.dz;
    }
    // with accumulate the sums start from the stored values, so a sequence of launches over
    // consecutive angle ranges performs exactly the additions of one launch over all of them
    float acc[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        acc[k] = (live && A.accumulate && kk >= A.own_lo && kk < A.own_hi)
                     ? to_f(vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i])
                     : 0.0f;
    }
    const int64_t psz = (int64_t)A.nu * A.nv;
    constexpr int ES = (int)sizeof(TP);
    const int rowb = A.nu * ES;
    const float amax = (float)A.nu + 1.0f, bmax = (float)A.nv + 1.0f;
    for (int t0 = 0; t0 < A.nang; t0 += 64) {
        const int nk = min(64, A.nang - t0);
        __syncthreads();  // the previous chunk's references have been read
        if ((int)threadIdx.x < nk) {
            const AngleGeo &G = A.tab[A.a0 + t0 + threadIdx.x];
            TileRef R;
            double ar, br;
            tile_ref(A, G.c, G.s, A.dx0 + (double)ir * A.ddx, A.dy0 + (double)jr * A.ddy, A.dz0 + (double)kr * A.ddz, R,
                     ar, br);
            // integer origins (clamped far outside the detector, where every tap is zero anyway)
            const double fa = fmin(fmax(floor(ar), -16777216.0), 16777216.0);
            const double fbr = fmin(fmax(floor(br), -16777216.0), 16777216.0);
            R.Aloc = (float)(ar - fa);
            R.Bloc = (float)(br - fbr);
            ref[threadIdx.x] = R;
            iref[threadIdx.x][0] = (float)fa;
            iref[threadIdx.x][1] = (float)fbr;
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nk; ++q) {
            const TileRef R = ref[q];
            float as, bq, mv, iL;
            tile_local(R, lx, ly, A.DSD, A.inv_dv, as, bq, mv, iL);
            const float af = floorf(as);
            const float fa = as - af;
            const int ia = (int)__builtin_amdgcn_fmed3f(iref[q][0] + af, -2.0f, amax);
            const float wa0 = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa : 0.0f;
            const float wa1 = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa : 0.0f;
            if (wa0 == 0.0f && wa1 == 0.0f) continue;
            const int ca0 = clampi(ia, 0, A.nu - 1) * ES;
            const int dca = (clampi(ia + 1, 0, A.nu - 1) - clampi(ia, 0, A.nu - 1)) * ES;
            const float ob = iref[q][1];
            float w = 0.0f, rxy2 = 0.0f, wpm = 0.0f;
            if (W == CT_BP_FDK) {
                const float qq = A.DSO * iL;
                w = qq * qq;
            } else {
                const float sx = x - A.DSO * R.c, sy = y - A.DSO * R.s;
                rxy2 = sx * sx + sy * sy;
                wpm = A.pm_const * iL * iL * iL;
            }
            const __amdgpu_buffer_rsrc_t Rs = proj_rsrc(proj + (int64_t)(t0 + q) * psz, psz * ES);
            // all taps of the column are issued before any is used, so they are in flight together
            float p[BP_NZ][4], fb[BP_NZ];
#pragma unroll
            for (int k = 0; k < BP_NZ; ++k) {
                const float bs = fmaf(zl[k], mv, bq);
                const float bf = floorf(bs);
                fb[k] = bs - bf;
                // rows outside the detector read 0 (negative offsets wrap past the buffer's end)
                const int o00 = (int)__builtin_amdgcn_fmed3f(ob + bf, -2.0f, bmax) * rowb + ca0;
                p[k][0] = bload(Rs, o00, (TP *)nullptr);
                p[k][1] = bload(Rs, o00 + dca, (TP *)nullptr);
                p[k][2] = bload(Rs, o00 + rowb, (TP *)nullptr);
                p[k][3] = bload(Rs, o00 + rowb + dca, (TP *)nullptr);
            }
#pragma unroll
            for (int k = 0; k < BP_NZ; ++k) {
                const float v0 = fmaf(wa1, p[k][1], wa0 * p[k][0]);
                const float v1 = fmaf(wa1, p[k][3], wa0 * p[k][2]);
                const float v = fmaf(fb[k], v1 - v0, v0);
                float wk = w;
                if (W != CT_BP_FDK) wk = wpm * __builtin_amdgcn_sqrtf(fmaf(zk[k], zk[k], rxy2));
                acc[k] = fmaf(wk, v, acc[k]);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.own_lo) continue;
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
constexpr int BPL_G = 64;  // angles per group of tile references
static_assert(BPL_NZ * 256 <= BPL_FLOATS, "the staging window parks the accumulators");

// 8 (FDK) or 7 (pseudo-matched) waves per SIMD: the taps are LDS reads one after another, so
// their latency is hidden by the other waves rather than by reads kept in flight in one wave
// (which the compiler would otherwise schedule, at 4 waves per SIMD: 22.1 against 28.6 ms for
// the FDK backprojection at 512^3 / 360 angles)
#ifndef CT_BPL_WAVES
#define CT_BPL_WAVES 8
#endif
#ifndef CT_BPL_WAVES_PM
#define CT_BPL_WAVES_PM 7
#endif
template <int W, int PITCH, typename TP, typename TV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W == CT_BP_FDK ? CT_BPL_WAVES : CT_BPL_WAVES_PM))) void k_bp_lds(const TP *__restrict__ proj, TV *__restrict__ vol, BpArgs A, int WW,
                                                int HW, int K) {
    __shared__ float win[BPL_FLOATS];
    __shared__ TileRef ref[BPL_G];
    __shared__ int org[BPL_G][2];
    const int i0 = blockIdx.x * BP_TX, j0 = blockIdx.y * BP_TY;
    const int i = i0 + (threadIdx.x % BP_TX);
    const int j = j0 + (threadIdx.x / BP_TX);
    const int kb = run_base(A, BPL_NZ);
    const bool live = i < A.nx && j < A.ny;
    const float ir = tile_mid(i0, BP_TX, A.nx), jr = tile_mid(j0, BP_TY, A.ny), kr = tile_mid(kb, BPL_NZ, A.nz);
    const float lx = ((float)i - ir) * A.dx, ly = ((float)j - jr) * A.dy;
    // heights of the run's first voxel relative to the reference (row coordinates) and absolute
    // (the pseudo-matched weight); voxel k of the run adds k dz
    const float zl0 = ((float)kb - kr) * A.dz, zk0 = fmaf((float)kb, A.dz, A.z0);
    const int64_t psz = (int64_t)A.nu * A.nv;
    const int wsz = PITCH * HW;
    const float lamax = (float)(WW - 2), lbmax = (float)(HW - 2);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(tid >> 6));
    const int lane = tid & 63;
    float acc[BPL_NZ];
    for (int g0 = 0; g0 < A.nang; g0 += BPL_G) {
        const int ng = min(BPL_G, A.nang - g0);
        if (g0 > 0) {
            // park the sums in the window while the group's references are formed, so the FP64
            // set-up does not hold registers next to them
            __syncthreads();  // the last round's taps have been read
#pragma unroll
            for (int k = 0; k < BPL_NZ; ++k) win[k * 256 + tid] = acc[k];
        }
        // threads 8q' .. 8q'+7: the tile's corners under angle g0 + q0 + q' (FP32; the window has a
        // pixel of margin), then thread 8q' projects the reference point in FP64
        for (int q0 = 0; q0 < ng; q0 += 32) {
            const int q = q0 + (tid >> 3), cn = tid & 7;
            float as = 0.0f, bs = 0.0f;
            if (q < ng) {
                const AngleGeo &G = A.tab[A.a0 + g0 + q];
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
            if (cn == 0 && q < ng) {
                const int oa = (int)floorf(amin) - 1, ob = (int)floorf(bmin) - 1;
                org[q][0] = oa;
                org[q][1] = ob;
                const AngleGeo &G = A.tab[A.a0 + g0 + q];
                TileRef R;
                double ar, br;
                tile_ref(A, G.c, G.s, A.dx0 + (double)ir * A.ddx, A.dy0 + (double)jr * A.ddy, A.dz0 + (double)kr * A.ddz,
                         R, ar, br);
                R.Aloc = (float)(ar - oa);
                R.Bloc = (float)(br - ob);
                ref[q] = R;
            }
        }
        __syncthreads();
        if (g0 == 0) {
            // one base address, slices a uniform stride apart (the stride is hidden from the
            // compiler so the 16 addresses are not kept live until the stores at the end)
            int64_t sl = (int64_t)A.nx * A.ny;
            asm volatile("" : "+s"(sl));
            const TV *vb = vol + ((int64_t)(kb - A.mem_lo) * A.ny + j) * A.nx + i;
#pragma unroll
            for (int k = 0; k < BPL_NZ; ++k) {
                const int kk = kb + k;
                acc[k] = (live && A.accumulate && kk >= A.own_lo && kk < A.own_hi) ? to_f(vb[k * sl]) : 0.0f;
            }
        } else {
#pragma unroll
            for (int k = 0; k < BPL_NZ; ++k) acc[k] = win[k * 256 + tid];
        }
        for (int t0 = 0; t0 < ng; t0 += K) {
            const int nk = min(K, ng - t0);
            __syncthreads();  // the window is free (parked sums read back, or the last round's taps read)
            // stage: wave w copies rows w, w + 4, ... of every window; lane = window column
            for (int q = 0; q < nk; ++q) {
                const int u = org[t0 + q][0] + lane;
                const bool uok = lane < WW && (unsigned)u < (unsigned)A.nu;
                const TP *pq = proj + (int64_t)(g0 + t0 + q) * psz + u;
                float *wq = win + q * wsz + lane;
                const int ob = org[t0 + q][1];
                for (int r = wave; r < HW; r += 4) {
                    const int v = ob + r;
                    float val = 0.0f;
                    if (uok && (unsigned)v < (unsigned)A.nv) val = to_f(pq[(int64_t)v * A.nu]);
                    if (lane < WW) wq[r * PITCH] = val;
                }
            }
            __syncthreads();
            if (!live) continue;
            for (int q = 0; q < nk; ++q) {
                const TileRef R = ref[t0 + q];
                // window-local column coordinate, row coordinate at the reference height
                float as, bq, mv, iL;
                tile_local(R, lx, ly, A.DSD, A.inv_dv, as, bq, mv, iL);
                const float af = floorf(as);
                const float fa = as - af;
                const float wa0 = 1.0f - fa, wa1 = fa;  // taps off the detector are zeros in the window
                // window column clamped into the window (an exact integer in FP32)
                const float la = __builtin_amdgcn_fmed3f(af, 0.0f, lamax);
                float w = 0.0f, rxy2 = 0.0f, wpm = 0.0f;
                if (W == CT_BP_FDK) {
                    const float qq = A.DSO * iL;
                    w = qq * qq;
                } else {
                    const float sx = fmaf(-A.DSO, R.c, fmaf((float)i, A.dx, A.x0));
                    const float sy = fmaf(-A.DSO, R.s, fmaf((float)j, A.dy, A.y0));
                    rxy2 = sx * sx + sy * sy;
                    wpm = A.pm_const * iL * iL * iL;
                }
                // LDS byte offset of the window column (exact in FP32); the clamp keeps rows 0 .. HW - 2
                const float cb = fmaf(la, 4.0f, (float)(q * wsz * 4));
                const float cbmax = fmaf(lbmax, (float)(4 * PITCH), cb);
                // row coordinate of voxel k of the run: b0 + k db, with db a few pixels at most
                const float b0 = fmaf(zl0, mv, bq), db = A.dz * mv;
                // with the run climbing less than one row per voxel, a voxel's lower tap row is the
                // previous voxel's lower or upper row: only its upper row is read (the same taps)
                if (db < 0.999f) {
                    float l0 = 0.0f, l1 = 0.0f, u0 = 0.0f, u1 = 0.0f, offp = 0.0f;
#pragma unroll
                    for (int k = 0; k < BPL_NZ; ++k) {
                        const float bs = fmaf((float)k, db, b0);
                        const float bf = floorf(bs);
                        const float fb = bs - bf;
                        const float off = __builtin_amdgcn_fmed3f(fmaf(bf, (float)(4 * PITCH), cb), cb, cbmax);
                        const float *t = (const float *)((const char *)win + (int)off);
                        if (k == 0) {
                            l0 = t[0];
                            l1 = t[1];
                        } else {
                            const bool up = off != offp;  // one row up (4 PITCH bytes) or the same row
                            l0 = up ? u0 : l0;
                            l1 = up ? u1 : l1;
                        }
                        u0 = t[PITCH];
                        u1 = t[PITCH + 1];
                        offp = off;
                        const float v0 = fmaf(wa1, l1, wa0 * l0);
                        const float v1 = fmaf(wa1, u1, wa0 * u0);
                        const float v = fmaf(fb, v1 - v0, v0);
                        float wk = w;
                        if (W != CT_BP_FDK) {
                            const float zk = fmaf((float)k, A.dz, zk0);
                            wk = wpm * __builtin_amdgcn_sqrtf(fmaf(zk, zk, rxy2));
                        }
                        acc[k] = fmaf(wk, v, acc[k]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < BPL_NZ; ++k) {
                        const float bs = fmaf((float)k, db, b0);
                        const float bf = floorf(bs);
                        const float fb = bs - bf;
                        const float off = __builtin_amdgcn_fmed3f(fmaf(bf, (float)(4 * PITCH), cb), cb, cbmax);
                        const float *t = (const float *)((const char *)win + (int)off);
                        const float v0 = fmaf(wa1, t[1], wa0 * t[0]);
                        const float v1 = fmaf(wa1, t[PITCH + 1], wa0 * t[PITCH]);
                        const float v = fmaf(fb, v1 - v0, v0);
                        float wk = w;
                        if (W != CT_BP_FDK) {
                            const float zk = fmaf((float)k, A.dz, zk0);
                            wk = wpm * __builtin_amdgcn_sqrtf(fmaf(zk, zk, rxy2));
                        }
                        acc[k] = fmaf(wk, v, acc[k]);
                    }
                }
            }
        }
    }
    if (!live || A.nang <= 0) return;
    int64_t sl = (int64_t)A.nx * A.ny;
    asm volatile("" : "+s"(sl));
    TV *vs = vol + ((int64_t)(kb - A.mem_lo) * A.ny + j) * A.nx + i;
#pragma unroll
    for (int k = 0; k < BPL_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.own_lo) continue;
        if (kk >= A.own_hi) break;
        vs[k * sl] = from_f<TV>(acc[k]);
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
    const int kb = run_base(A, ADJ_NZ);  // heights are taken relative to the run's lowest face
    const bool live = i < A.nx && j < A.ny;
#pragma unroll
    for (int k = 0; k < ADJ_NZ; ++k) {
        const int kk = kb + k;
        accs[k * 256 + tid] = (live && A.accumulate && kk >= A.own_lo && kk < A.own_hi)
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
    const double v0d = A.offv - A.cv * A.dv;       // height of row 0 at the detector
    const double zl0d = A.dz0 + (kb - 0.5) * A.ddz;  // lower face of the run's first voxel
    const float v0 = (float)v0d, dv = (float)A.dv, idv = 1.0f / dv;
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
            const double dotd = Wx * Dx + Wy * Dy;            // = |D|^2 * t of the closest point
            const float fDx = (float)Dx, fDy = (float)Dy;
            const float L2 = fmaf(fDx, fDx, fDy * fDy);
            const float iL = __builtin_amdgcn_rsqf(L2);
            const float ux = fDx * iL, uy = fDy * iL;
            const float dperp = cross * iL;
            // closest point of the trace to the column centre, relative to the centre
            const float fx = -dperp * uy, fy = dperp * ux;
            // slab clip of fx + s ux in [-hx, hx], fy + s uy in [-hy, hy]  (s in mm)
            float s0 = -FLT_MAX, s1 = FLT_MAX;
            // a trace the projector takes as parallel to an axis (|D_c| < 1e-12 |D|, in FP64; here with
            // the horizontal |D|) runs at the source's coordinate: the column must hold it in its
            // half-open slab
            const double lpar = 1e-24 * (Dx * Dx + Dy * Dy);
            if (Dx * Dx >= lpar) {
                const float r = __builtin_amdgcn_rcpf(ux);
                const float qa = (-hx - fx) * r, qb = (hx - fx) * r;
                s0 = fmaxf(s0, fminf(qa, qb));
                s1 = fminf(s1, fmaxf(qa, qb));
            } else if ((int)floor(G.S[0] + 0.5) != i) {
                continue;
            }
            if (Dy * Dy >= lpar) {
                const float r = __builtin_amdgcn_rcpf(uy);
                const float qa = (-hy - fy) * r, qb = (hy - fy) * r;
                s0 = fmaxf(s0, fminf(qa, qb));
                s1 = fminf(s1, fmaxf(qa, qb));
            } else if ((int)floor(G.S[1] + 0.5) != j) {
                continue;
            }
            if (!(s0 < s1)) continue;
            const float T = (s1 - s0) * iL;                       // t-length inside the column
            // t where the trace enters, in FP64 (one Newton step on the FP32 reciprocal of |D|^2)
            const double L2d = Dx * Dx + Dy * Dy;
            const double rl = (double)__builtin_amdgcn_rcpf((float)L2d);
            const double t0d = fma(dotd, rl * fma(-L2d, rl, 2.0), (double)(s0 * iL));
            const float t0 = (float)t0d;
            const float t1 = t0 + T;
            // rows whose height range inside the column meets the thread's z run [zl0, zr_hi]
            const float it0 = __builtin_amdgcn_rcpf(t0), it1 = __builtin_amdgcn_rcpf(t1);
            const float vmin = fminf(zl0 * it0, zl0 * it1), vmax = fmaxf(zr_hi * it0, zr_hi * it1);
            const int blo = (int)fmaxf(ceilf((vmin - v0) * idv - 1e-3f), 0.0f);
            const int bhi = (int)fminf(floorf((vmax - v0) * idv + 1e-3f), (float)(A.nv - 1));
            int off = blo * rowb + a * ES;
            for (int b = blo; b <= bhi; ++b, off += rowb) {
                const float y = bload(R, off, (TP *)nullptr);
                const double vbd = fma((double)b, A.dv, v0d);
                const float vb = (float)vbd;
                // height where the row enters the column, relative to the run's lowest face (a
                // difference of heights of up to the volume's half height, formed in FP64)
                const float za = (float)fma(t0d, vbd, -zl0d);
                const float ext = T * vb;            // signed height change across the column
                const float lo = fminf(za, za + ext), hi = fmaxf(za, za + ext);
                const float full = T * sqrtf(fmaf(vb, vb, L2));   // chord inside the column
                const int klo = (int)floorf(lo * idz);
                const int khi = (int)floorf(hi * idz);
                if (klo == khi) {
                    // the row stays inside one voxel
                    if ((unsigned)klo < (unsigned)nzr) accs[klo * 256 + tid] = fmaf(full, y, accs[klo * 256 + tid]);
                } else {
                    const float iext = __builtin_amdgcn_rcpf(hi - lo);
                    const int ke = min(khi, nzr - 1);
                    for (int k = max(klo, 0); k <= ke; ++k) {
                        const float zl = (float)k * dz;
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
        if (kk < A.own_lo) continue;
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
// bound).  The projections are read from a copy [angle][u][1 + v] of y |P - S| with a zero row
// below and above each column, so the rows of consecutive voxels are consecutive addresses: a
// voxel's NR candidate rows are one load of 4 NR bytes.  The parameter step dz / v_b across one
// voxel height depends on the row alone (a circular orbit), so each block keeps the steps of all
// rows in LDS.  Every row then costs two products and four compares.

// Parameter step dz / v_b of row r = b + 1 of the padded copy (0 for the zero rows).
__device__ __forceinline__ float adj_row_step(const BpArgs &A, int r) {
    const int b = r - 1;
    if (b < 0 || b >= A.nv || b == A.zrow) return 0.0f;  // the row at the source's height: see k_adj_col
    const double vb = (b - A.cv) * A.dv + A.offv;
    return vb != 0.0 ? (float)(A.ddz / vb) : 1e30f;
}

// proj [angle][v][u] -> yq [angle][u][v + 1] (nv + 2 rows, zero first and last), 32 x 32 tiles
template <typename TP>
__global__ __launch_bounds__(256) void k_adj_prep(const TP *__restrict__ proj, float *__restrict__ yq, BpArgs A) {
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
            float q = 0.0f;
            if (b >= 0 && b < A.nv) {
                const double ua = (u - A.cu) * A.du + A.offu, vb = (b - A.cv) * A.dv + A.offv;
                if (A.vw) {
                    // |P - S| of a vertical view: its horizontal part C - S + u e_u, and v_b
                    const AngleGeo &G = A.tab[A.a0 + t];
                    const double px = fma(ua, G.eu[0], G.Dc[0]) * A.ddx, py = fma(ua, G.eu[1], G.Dc[1]) * A.ddy;
                    q = (float)(tile[tx][ty + k] * sqrt(px * px + py * py + vb * vb));
                } else {
                    // |P - S| (mm per unit t) is the same for every angle in a circular orbit
                    q = (float)(tile[tx][ty + k] * sqrt(A.dDSD * A.dDSD + ua * ua + vb * vb));
                }
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
// exactly 4 waves per SIMD: the compiler then keeps the row loads of all R voxels of a candidate
// column in flight together instead of two at a time (more registers, fewer exposed latencies)
#ifndef CT_ADJ_WAVES
#define CT_ADJ_WAVES 4, 4
#endif
#define CT_ADJ_OCC __attribute__((amdgpu_waves_per_eu(CT_ADJ_WAVES)))
// VW: a plan of vertical views (detector columns vertical, the detector centre at the source's
// height; circular and helical scans): each view's source, C - S and e_u replace the circular
// orbit's, heights are taken from the view's source plane, and the faces' order is set per view
// (VW implies !ORD and !ZC).
template <typename TV, int R, int NR, bool ZC, bool ORD, bool VW = false>
__global__ __launch_bounds__(256) CT_ADJ_OCC void k_adj_col(const float *__restrict__ yq, TV *__restrict__ vol, BpArgs A,
                                                 int zgroups, int xblocks) {
    static_assert(!VW || (!ORD && !ZC), "vertical views take the general face order and [z][y][x] volumes");
    extern __shared__ float rstep[];  // nv + 2 parameter steps, one per row of the padded copy
    __shared__ float4 chdr[4][64][3];  // per wave: the set-up of up to 64 (angle, column) pairs
    __shared__ int cslot[4][3][64];    // per wave and angle of a batch: first column, pairs before, through
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    for (int r = threadIdx.x; r < A.nv + 2; r += 256) rstep[r] = adj_row_step(A, r);
    __syncthreads();
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
    // the voxel lies below the source plane), for choosing the candidate rows.
    // kA, sg: index of the face that rows of the voxel's side of the source plane reach first (the
    // upper face for a voxel below the plane), an exact integer, and the direction of the other
    // face.  They are the same with and without ORD, so both forms give the same bits.
    float acc[R], za[R], zb[R], kA[R], sg[R];
    bool kin[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = A.own_lo + zg * 64 * R + 64 * r + lane;
        kin[r] = k < A.own_hi;
        const float zl = fmaf((float)k, dz, zface0), zh = fmaf((float)(k + 1), dz, zface0);
        if (VW) {
            // the faces in the world frame; each view takes them relative to its source
            za[r] = zl;
            zb[r] = zh;
            kA[r] = (float)k;
            sg[r] = 1.0f;
            acc[r] = (kin[r] && A.accumulate) ? to_f(vol[vidx(k)]) : 0.0f;
            continue;
        }
        const bool below = zh <= 0.0f;
        const bool flip = ORD && below;
        za[r] = flip ? zh : zl;
        zb[r] = flip ? zl : zh;
        kA[r] = (float)(below ? k + 1 : k);
        sg[r] = below ? -1.0f : 1.0f;
        const int64_t o = vidx(k);
        acc[r] = (kin[r] && A.accumulate) ? to_f(vol[o]) : 0.0f;
    }
    const double xc = A.dx0 + i * A.ddx, yc = A.dy0 + j * A.ddy;  // column centre (mm)
    const float hx = 0.5f * A.dx, hy = 0.5f * A.dy;
    const float fxc = (float)xc, fyc = (float)yc;
    const double v0d = A.offv - A.cv * A.dv;  // height of row 0 at the detector
    // heights in voxel units above the lower face of voxel 0: row b enters the square at height
    // H0 + b S with H0 = (t0 v0 - zface0) / dz and S = t0 dv / dz
    const double v0dz = v0d / A.ddz, zf0dz = (A.dz0 - 0.5 * A.ddz) / A.ddz, dvdz = A.dv / A.ddz;
    const float v0 = (float)v0d, idv = 1.0f / (float)A.dv;
    const float nv0 = -v0 * idv;
    const float bmax = (float)(A.nv + 1 - NR);
    const float aum = (float)(A.cu - A.offu / A.du), iau = (float)(1.0 / A.du);
    const int nvp = A.nv + 2;
    // The set-up of a candidate detector column (its trace through the column's square in FP64, the
    // entry parameter, the heights below) is the same for every lane of the wave, which holds one
    // voxel column.  So the lanes share it out: each lane takes one angle of a batch of 64 and finds
    // that angle's candidate columns, a prefix sum over the wave lays the (angle, column) pairs out
    // in angle order, each lane forms the set-up of one pair into LDS, and the voxel loop reads the
    // pairs back in that order (the same sums in the same order as one pair after another).
    const int kw0 = A.own_lo + zg * 64 * R;  // first voxel of the wave's lanes
    float4(*hdr)[3] = chdr[wave];
    int(*slot)[64] = cslot[wave];
    int tprev = -1;
    for (int tb = 0; tb < A.nang; tb += 64) {
        int alo = 0, cnt = 0;
        if (tb + lane < A.nang) {
            const AngleGeo &G = A.tab[A.a0 + tb + lane];
            float umin = FLT_MAX, umax = -FLT_MAX;
            if (VW) {
                // detector coordinate u of the ray through each corner of the column's square: with
                // X - S = Xr and C - S + u e_u parallel to it, u = (Xr x (C - S)) / (e_u x Xr)
                const double Wx = xc - G.Smm[0], Wy = yc - G.Smm[1];
                const float dcx = (float)(G.Dc[0] * A.ddx), dcy = (float)(G.Dc[1] * A.ddy);
                const float eux = (float)(G.eu[0] * A.ddx), euy = (float)(G.eu[1] * A.ddy);
                const float fwx = (float)Wx, fwy = (float)Wy;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float X = fwx + ((q & 1) ? hx : -hx), Y = fwy + ((q & 2) ? hy : -hy);
                    const float u = (X * dcy - Y * dcx) * __builtin_amdgcn_rcpf(eux * Y - euy * X);
                    umin = fminf(umin, u);
                    umax = fmaxf(umax, u);
                }
            } else {
                const float fc = (float)G.c, fs = (float)G.s;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float X = fxc + ((q & 1) ? hx : -hx), Y = fyc + ((q & 2) ? hy : -hy);
                    const float u = A.DSD * (Y * fc - X * fs) * __builtin_amdgcn_rcpf(A.DSO - (X * fc + Y * fs));
                    umin = fminf(umin, u);
                    umax = fmaxf(umax, u);
                }
            }
            // (a wider margin for views: their corner coordinates are formed from source-relative
            // vectors of about a metre; a column too many is clipped away below)
            const float um = VW ? 1e-2f : 1e-3f;
            alo = (int)fmaxf(ceilf(fmaf(umin, iau, aum) - um), 0.0f);
            const int ahi = (int)fminf(floorf(fmaf(umax, iau, aum) + um), (float)(A.nu - 1));
            cnt = max(ahi - alo + 1, 0);
        }
        int incl = cnt;  // inclusive prefix sum of the counts over the lanes
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d, 64);
            if (lane >= d) incl += v;
        }
        const int total = __builtin_amdgcn_readlane(incl, 63);
        slot[0][lane] = alo;
        slot[1][lane] = incl - cnt;
        slot[2][lane] = incl;
        wave_lds_sync();
        for (int e0 = 0; e0 < total; e0 += 64) {
            const int e = e0 + lane;
            if (e < total) {
                // the angle of pair e: the first lane whose inclusive sum exceeds e (at most lane 63)
                int sl = 0;
#pragma unroll
                for (int st = 32; st > 0; st >>= 1)
                    if (slot[2][sl + st - 1] <= e) sl += st;
                const int t = tb + sl, a = slot[0][sl] + (e - slot[1][sl]);
                hdr[lane][2] = make_float4(__int_as_float(-1), 0.0f, 0.0f, 0.0f);
                const AngleGeo &G = A.tab[A.a0 + t];
                double Wx, Wy;         // source -> column centre
                double zf0v = zf0dz;   // lower face of voxel 0 above the source plane, voxel units
                float szf = 0.0f;      // VW: the source's height
                double Dx, Dy;
                const double ua = (a - A.cu) * A.du + A.offu;
                if (VW) {
                    Wx = xc - G.Smm[0];
                    Wy = yc - G.Smm[1];
                    zf0v = zf0dz - G.Smm[2] / A.ddz;
                    szf = (float)G.Smm[2];
                    Dx = fma(ua, G.eu[0], G.Dc[0]) * A.ddx;
                    Dy = fma(ua, G.eu[1], G.Dc[1]) * A.ddy;
                } else {
                    Wx = xc - A.dDSO * G.c;
                    Wy = yc - A.dDSO * G.s;
                    // (the per-angle product rounded first, as one FMA adds the column's term)
                    Dx = fma(-ua, G.s, -A.dDSD * G.c);
                    Dy = fma(ua, G.c, -A.dDSD * G.s);
                }
                const float cross = (float)(Wx * Dy - Wy * Dx);
                const double dotd = Wx * Dx + Wy * Dy;
                const float fDx = (float)Dx, fDy = (float)Dy;
                const float L2 = fmaf(fDx, fDx, fDy * fDy);
                const float iL = __builtin_amdgcn_rsqf(L2);
                const float ux = fDx * iL, uy = fDy * iL;
                const float dperp = cross * iL;
                const float fx = -dperp * uy, fy = dperp * ux;
                float s0 = -FLT_MAX, s1 = FLT_MAX;
                // a trace the projector takes as parallel to an axis (|D_c| < 1e-12 |D|, in FP64; here
                // with the horizontal |D|) runs at the source's coordinate: the column must hold it in
                // its half-open slab
                const double lpar = 1e-24 * (Dx * Dx + Dy * Dy);
                bool hit = true;
                if (Dx * Dx >= lpar) {
                    const float rr = __builtin_amdgcn_rcpf(ux);
                    const float qa = (-hx - fx) * rr, qb = (hx - fx) * rr;
                    s0 = fmaxf(s0, fminf(qa, qb));
                    s1 = fminf(s1, fmaxf(qa, qb));
                } else {
                    hit = (int)floor(G.S[0] + 0.5) == i;
                }
                if (Dy * Dy >= lpar) {
                    const float rr = __builtin_amdgcn_rcpf(uy);
                    const float qa = (-hy - fy) * rr, qb = (hy - fy) * rr;
                    s0 = fmaxf(s0, fminf(qa, qb));
                    s1 = fminf(s1, fmaxf(qa, qb));
                } else {
                    hit = hit && (int)floor(G.S[1] + 0.5) == j;
                }
                if (hit && s0 < s1) {
                    const float T = (s1 - s0) * iL;
                    // t where the trace enters the square, in FP64: the foot point's parameter
                    // W.D / |D|^2 (one Newton step on the FP32 reciprocal) plus the small FP32 clip
                    // offset
                    const double L2d = Dx * Dx + Dy * Dy;
                    const double rl = (double)__builtin_amdgcn_rcpf((float)L2d);
                    const double t0d = fma(dotd, rl * fma(-L2d, rl, 2.0), (double)(s0 * iL));
                    const float t0 = (float)t0d;
                    // H0 = H0h + H0l with H0h on a grid of 2^-7 (adding and removing 1.5 * 2^16 rounds
                    // to it for |H0| < 2^15), S = Sh + Sr with Sh holding 10 significant bits: then
                    // for face index kA (an integer) and row b (|b| < 2^14) kA - H0h and b Sh are
                    // exact FP32 values and so is their difference, which is a few voxels for the
                    // candidate rows; only the small terms b Sr + H0l are rounded
                    const double H0d = fma(t0d, v0dz, -zf0v), Sd = t0d * dvdz;
                    const float H0h = ((float)H0d + 98304.0f) - 98304.0f;
                    const float H0l = (float)(H0d - (double)H0h);
                    const float Sf = (float)Sd;
                    const float Sh = __uint_as_float(__float_as_uint(Sf) & 0xFFFFC000u);
                    const float Sr = (float)(Sd - (double)Sh);
                    const float it0 = __builtin_amdgcn_rcpf(t0), it1 = __builtin_amdgcn_rcpf(t0 + T);
                    // the voxel (relative to kw0) whose half-open slab holds the source's height
                    const int ks = (int)floor(-zf0v) - kw0;
                    hdr[lane][0] = make_float4(T, H0h, H0l, Sf);
                    hdr[lane][1] = make_float4(Sh, Sr, it0, it1);
                    hdr[lane][2] = make_float4(__int_as_float(t), __int_as_float(a), szf, __int_as_float(ks));
                }
            }
            wave_lds_sync();
            const int ne = min(64, total - e0);
            for (int p = 0; p < ne; ++p) {
                const float4 h2 = hdr[p][2];
                const int t = __builtin_amdgcn_readfirstlane(__float_as_int(h2.x));
                if (t < 0) continue;  // the trace misses the column's square
                const float4 h0 = hdr[p][0], h1 = hdr[p][1];
                const int a = __builtin_amdgcn_readfirstlane(__float_as_int(h2.y));
                const float T = h0.x, H0h = h0.y, H0l = h0.z, Sf = h0.w;
                const float Sh = h1.x, Sr = h1.y, it0 = h1.z, it1 = h1.w;
                const float szf = h2.z;
                if (VW && t != tprev) {
                    tprev = t;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        // a voxel below the source plane is met by falling rows first at its upper face
                        const bool below = zb[r] - szf <= 0.0f;
                        kA[r] = below ? (float)(kw0 + 64 * r + lane + 1) : (float)(kw0 + 64 * r + lane);
                        sg[r] = below ? -1.0f : 1.0f;
                    }
                }
                const float *col = yq + ((int64_t)t * A.nu + a) * nvp;  // row b at col[b + 1]
                if (A.zrow >= 0) {
                    // the row at the source's height stays in one slice, the one whose half-open slab
                    // holds that height; its step is 0 in the table, so the loop below adds nothing
                    const int ks = __float_as_int(h2.w);
                    if (ks >= 0 && ks < 64 * R && (ks & 63) == lane) {
                        const float yz = col[A.zrow + 1];
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if ((ks >> 6) == r) acc[r] = fmaf(T, yz, acc[r]);
                    }
                }
                float wv[R][NR];
                float bl[R], E[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // first row that can meet the voxel, kept inside [-1, nv + 1 - NR]: the lowest
                    // v = z / t over the lower face and t in [t0, t1] (with ORD, za * it1 for voxels
                    // above the plane and zb * it0 for voxels below)
                    const float zlo = VW ? za[r] - szf : za[r];
                    const float vlo = ORD ? fminf(za[r] * it1, zb[r] * it0) : fminf(zlo * it0, zlo * it1);
                    bl[r] = __builtin_amdgcn_fmed3f(ceilf(fmaf(vlo, idv, nv0)), -1.0f, bmax);
                    // the height of face A above row bl where the row enters the square, in voxel
                    // units (kA - H0 - bl S: a difference of heights of up to the volume's height,
                    // formed exactly up to the small terms)
                    const float d = (kA[r] - H0h) - bl[r] * Sh;
                    E[r] = d - fmaf(bl[r], Sr, H0l);
                }
                // the rows of all R voxels are loaded before any is used, so they are in flight together
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // uniform column base plus an unsigned 32-bit byte offset of row bl
                    const float *cb = (const float *)((const char *)col + (uint32_t)((int)bl[r] + 1) * 4u);
#pragma unroll
                    for (int q = 0; q < NR; ++q) wv[r][q] = cb[q];
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float *sb = rstep + ((int)bl[r] + 1);
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const float2 w = make_float2(wv[r][q], sb[q]);
                        // parameters relative to t0 of the row's crossings of faces A and B (its
                        // height below face A in voxels times dz / v_b, and one step dz / v_b more),
                        // clipped to [0, T]: a row that stays inside the voxel gets exactly T
                        const float Eq = q == 0 ? E[r] : fmaf(-(float)q, Sf, E[r]);
                        const float tA = Eq * w.y, tB = fmaf(sg[r], w.y, tA);
                        float len;
                        if (ORD) {
                            // tA <= tB for the rows that can meet the voxel; rows of the other sign have
                            // both parameters below 0, which clamp to the same value
                            len = __builtin_amdgcn_fmed3f(tB, 0.0f, T) - __builtin_amdgcn_fmed3f(tA, 0.0f, T);
                        } else {
                            // either order: clamping to [0, T] is monotonic, so the clamped pair's distance
                            // is the overlap of [min, max] with [0, T] (0 when they miss), bit for bit the
                            // max(min(max, T) - max(min, 0), 0) it replaces; the |.| folds into the FMA
                            len = fabsf(__builtin_amdgcn_fmed3f(tB, 0.0f, T) - __builtin_amdgcn_fmed3f(tA, 0.0f, T));
                        }
                        acc[r] = fmaf(len, w.x, acc[r]);
                    }
                }
            }
            wave_lds_sync();
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
    __shared__ TileRef ref[64];
    __shared__ float iref[64][2];
    const int i0 = blockIdx.x * BP_TX, j0 = blockIdx.y * BP_TY;
    const int i = i0 + (threadIdx.x % BP_TX);
    const int j = j0 + (threadIdx.x / BP_TX);
    const int kb = blockIdx.z * BP_NZ;
    const bool live = i < A.nx && j < A.ny;
    // detector coordinates relative to the tile's reference point (see TileRef)
    const float ir = tile_mid(i0, BP_TX, A.nx), jr = tile_mid(j0, BP_TY, A.ny), kr = tile_mid(kb, BP_NZ, A.nz);
    const float lx = ((float)i - ir) * A.dx, ly = ((float)j - jr) * A.dy;
    const int64_t pix = (int64_t)A.nu * A.nv;
    const float amax = (float)A.nu + 1.0f, bmax = (float)A.nv + 1.0f;
    // sums over the subset's angles, in angle order
    float num[BP_NZ], V[BP_NZ];
#pragma unroll
    for (int k = 0; k < BP_NZ; ++k) num[k] = V[k] = 0.0f;
    for (int t0 = 0; t0 < A.nang; t0 += 64) {
        const int nk = min(64, A.nang - t0);
        __syncthreads();
        if ((int)threadIdx.x < nk) {
            const AngleGeo &G = A.tab[A.a0 + t0 + threadIdx.x];
            TileRef R;
            double ar, br;
            tile_ref(A, G.c, G.s, A.dx0 + (double)ir * A.ddx, A.dy0 + (double)jr * A.ddy, A.dz0 + (double)kr * A.ddz, R,
                     ar, br);
            const double fa = fmin(fmax(floor(ar), -16777216.0), 16777216.0);
            const double fbr = fmin(fmax(floor(br), -16777216.0), 16777216.0);
            R.Aloc = (float)(ar - fa);
            R.Bloc = (float)(br - fbr);
            ref[threadIdx.x] = R;
            iref[threadIdx.x][0] = (float)fa;
            iref[threadIdx.x][1] = (float)fbr;
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nk; ++q) {
            const TileRef R = ref[q];
            float as, bq, mv, iL;
            tile_local(R, lx, ly, A.DSD, A.inv_dv, as, bq, mv, iL);
            const float af = floorf(as);
            const float fa = as - af;
            const int ia = (int)__builtin_amdgcn_fmed3f(iref[q][0] + af, -2.0f, amax);
            const float wa0 = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa : 0.0f;
            const float wa1 = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa : 0.0f;
            if (wa0 == 0.0f && wa1 == 0.0f) continue;
            const int ia0 = clampi(ia, 0, A.nu - 1), ia1 = clampi(ia + 1, 0, A.nu - 1);
            const float qq = A.DSO * iL;
            const float w = qq * qq;
            const float *rt = r + (t0 + q) * pix;
            const float ob = iref[q][1];
#pragma unroll
            for (int k = 0; k < BP_NZ; ++k) {
                // heights past the top of the volume are clamped to the last slice (and not written)
                const float zlk = ((float)min(kb + k, A.nz - 1) - kr) * A.dz;
                const float bs = fmaf(zlk, mv, bq);
                const float bf = floorf(bs);
                const float fb = bs - bf;
                const int ib = (int)__builtin_amdgcn_fmed3f(ob + bf, -2.0f, bmax);
                const float wb0 = ((unsigned)ib < (unsigned)A.nv) ? 1.0f - fb : 0.0f;
                const float wb1 = ((unsigned)(ib + 1) < (unsigned)A.nv) ? fb : 0.0f;
                const int r0 = clampi(ib, 0, A.nv - 1) * A.nu, r1 = clampi(ib + 1, 0, A.nv - 1) * A.nu;
                const float v0 = fmaf(wa1, rt[r0 + ia1], wa0 * rt[r0 + ia0]);
                const float v1 = fmaf(wa1, rt[r1 + ia1], wa0 * rt[r1 + ia0]);
                num[k] += w * fmaf(wb1, v1, wb0 * v0);
                V[k] += w * ((wa0 + wa1) * (wb0 + wb1));
            }
        }
    }
    if (!live) return;
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
    // per wave and angle: the column's detector coordinate a* (origin and fraction), FDK weight and
    // row step per mm; per height group r, the row coordinate of the group's reference height
    // (origin and fraction).  All from FP64, so the FP32 per-height parts are a few pixels in size.
    struct ColRef {
        float fa, w, mv, ia;
    };
    __shared__ ColRef hdr[4][64];
    __shared__ float2 bref[4][64][SART_R];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
    const int64_t ncol = (int64_t)A.nx * A.ny;
    const bool live = gw / zwaves < ncol;
    const int64_t col = live ? gw / zwaves : ncol - 1;  // a wave past the last column writes nothing
    const int zbase = (int)(gw % zwaves) * 64 * SART_R;
    const int kk0 = zbase + lane;
    const int i = (int)(col % A.nx), j = (int)(col / A.nx);
    const int64_t pix = (int64_t)A.nu * A.nv;
    float *vc = vz + col * (A.nz + 2) + 1;
    // the voxels' values are read first, so their loads overlap the first angle's taps
    float xo[SART_R], kref[SART_R], zl[SART_R];
#pragma unroll
    for (int r = 0; r < SART_R; ++r) {
        const int kk = min(kk0 + 64 * r, A.nz - 1);
        xo[r] = vc[kk];
        kref[r] = tile_mid(min(zbase + 64 * r, A.nz - 1), 64, A.nz);
        zl[r] = ((float)kk - kref[r]) * A.dz;
    }
    const double xc = A.dx0 + i * A.ddx, yc = A.dy0 + j * A.ddy;
    const float amax = (float)A.nu + 1.0f, bmax = (float)A.nv + 1.0f;
    // sums over the subset's angles, in angle order
    float num[SART_R], V[SART_R];
#pragma unroll
    for (int r = 0; r < SART_R; ++r) num[r] = V[r] = 0.0f;
    for (int t0 = 0; t0 < A.nang; t0 += 64) {
        const int nk = min(64, A.nang - t0);
        __syncthreads();
        // lane = (angle, height group) pair, so a launch of one angle (SART) costs one pass
        for (int p0 = 0; p0 < nk * SART_R; p0 += 64) {
            const int q = (p0 + lane) / SART_R, r = (p0 + lane) % SART_R;
            if (q < nk) {
                const AngleGeo &G = A.tab[A.a0 + t0 + q];
                const double D = A.dDSO - (xc * G.c + yc * G.s), iD = rcp_f64(D);
                const double kv = A.dDSD * iD * A.idv;
                if (r == 0) {
                    const double ar = fma(A.dDSD * iD * A.idu, yc * G.c - xc * G.s, A.dau0);
                    const double fa = fmin(fmax(floor(ar), -16777216.0), 16777216.0);
                    const double w = A.dDSO * iD;
                    hdr[wave][q] = ColRef{(float)(ar - fa), (float)(w * w), (float)kv, (float)fa};
                }
                const float kr = tile_mid(min(zbase + 64 * r, A.nz - 1), 64, A.nz);
                const double br = fma(kv, A.dz0 + (double)kr * A.ddz, A.dbv0);
                const double fb = fmin(fmax(floor(br), -16777216.0), 16777216.0);
                bref[wave][q][r] = make_float2((float)fb, (float)(br - fb));
            }
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nk; ++q) {
            const ColRef H = hdr[wave][q];
            const int ia = (int)__builtin_amdgcn_fmed3f(H.ia, -2.0f, amax);
            const float fa = H.fa;
            const float wa0 = ((unsigned)ia < (unsigned)A.nu) ? 1.0f - fa : 0.0f;
            const float wa1 = ((unsigned)(ia + 1) < (unsigned)A.nu) ? fa : 0.0f;
            if (wa0 == 0.0f && wa1 == 0.0f) continue;
            const float *rt = rT + (t0 + q) * pix;
            const float *r0 = rt + (int64_t)clampi(ia, 0, A.nu - 1) * A.nv;
            const float *r1 = rt + (int64_t)clampi(ia + 1, 0, A.nu - 1) * A.nv;
            const float w = H.w;
            const float wva = w * (wa0 + wa1);
            // all taps of the wave's SART_R heights first (heights clamped into the column), then the sums
            float wb0[SART_R], wb1[SART_R], t00[SART_R], t01[SART_R], t10[SART_R], t11[SART_R];
#pragma unroll
            for (int r = 0; r < SART_R; ++r) {
                const float2 B = bref[wave][q][r];
                const float bs = fmaf(zl[r], H.mv, B.y);
                const float bf = floorf(bs);
                const float fb = bs - bf;
                const int ib = (int)__builtin_amdgcn_fmed3f(B.x + bf, -2.0f, bmax);
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
    }
    if (!live) return;
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

// The same bound for a plan of vertical views, taken over the views: with L_min the least depth
// (along the detector normal, which is horizontal) of the grid's corners from the view's source,
// t_min = L_min / DSD_v, the voxel column's t extent at most sqrt(2) max(dx, dy) / DSD_v, and |z|
// measured from the source's height.
int adj_rows_views(const ct_plan *p) {
    const ct_geometry &g = p->g;
    int rows = 0;
    for (const AngleGeo &t : p->tab) {
        const double eu[2] = {t.eu[0] * g.dVoxel[0], t.eu[1] * g.dVoxel[1]};
        const double n[2] = {eu[1], -eu[0]};  // e_u x e_z
        double Lmin = HUGE_VAL, Zmax = 0.0;
        for (int cx = 0; cx < 2; ++cx)
            for (int cy = 0; cy < 2; ++cy) {
                const double xe = g.offOrigin[0] + (cx ? 0.5 : -0.5) * g.nVoxel[0] * g.dVoxel[0];
                const double ye = g.offOrigin[1] + (cy ? 0.5 : -0.5) * g.nVoxel[1] * g.dVoxel[1];
                Lmin = std::min(Lmin, n[0] * (t.Smm[0] - xe) + n[1] * (t.Smm[1] - ye));
            }
        for (int cz = 0; cz < 2; ++cz)
            Zmax = std::max(Zmax, std::fabs(g.offOrigin[2] + (cz ? 0.5 : -0.5) * g.nVoxel[2] * g.dVoxel[2] - t.Smm[2]));
        if (!(Lmin > 0.0)) return 1 << 20;
        const double tmin = Lmin / t.DSDv;
        const double dt = std::sqrt(2.0) * std::max(g.dVoxel[0], g.dVoxel[1]) / t.DSDv;
        const double W = (g.dVoxel[2] / tmin + Zmax * dt / (tmin * tmin)) / g.dDetector[1];
        rows = std::max(rows, (int)std::floor(W * 1.001 + 1e-3) + 1);
    }
    return rows;
}

// The least source-detector distance over a plan's views.
double min_dsd(const ct_plan *p) {
    double m = HUGE_VAL;
    for (const AngleGeo &t : p->tab) m = std::min(m, t.DSDv);
    return m;
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
    A.dau0 = A.cu - g.offDetector[0] / g.dDetector[0];
    A.dbv0 = A.cv - g.offDetector[1] / g.dDetector[1];
    A.au0 = (float)A.dau0;
    A.bv0 = (float)A.dbv0;
    A.idu = 1.0 / g.dDetector[0];
    A.idv = 1.0 / g.dDetector[1];
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
    A.vw = p->views ? 1 : 0;
    // the row at the source's height, as the projector decides it (|v_b| < 1e-12 |P - S|)
    A.zrow = -1;
    {
        const double b0 = A.cv - A.offv / A.dv;
        const double bi = std::nearbyint(b0);
        if (bi >= 0.0 && bi < (double)A.nv) {
            const double vb = (bi - A.cv) * A.dv + A.offv;
            if (std::fabs(vb) < 1e-12 * (p->views ? min_dsd(p) : g.DSD)) A.zrow = (int32_t)bi;
        }
    }
    return A;
}

}  // namespace

// CT_VIEWS_ADJ_DIRECT=1 or 2 sends the exact adjoint of vertical views to a per-view kernel (tests
// compare them).
bool direct_views_adjoint() {
    const char *e = std::getenv("CT_VIEWS_ADJ_DIRECT");
    return e && (e[0] == '1' || e[0] == '2');
}

// rows of the padded copy whose parameter steps fit the column kernel's LDS table (48 KiB, beside
// the 15 KiB of candidate set-ups: 63 KiB per workgroup)
constexpr int64_t ADJ_MAX_ROWS = 12288;

bool adj_col_ok(const ct_plan *p) {
#ifdef CT_NO_ADJ_COL
    return false;
#else
    if (p->views || p->g.nDetector[1] + 2 > ADJ_MAX_ROWS) return false;
    return std::min<int>(adj_rows(p->g), (int)p->g.nDetector[1] + 2) <= 4;
#endif
}

size_t adj_chunk_bytes_per_angle(const ct_geometry &g) {
    return (size_t)g.nDetector[0] * (size_t)(g.nDetector[1] + 2) * sizeof(float);
}

ct_status launch_backproject(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                             ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab, hipStream_t st,
                             void *adj_scratch, size_t adj_bytes) {
    const AngleGeo *tab = nullptr;
    ct_status s = slab.no_alloc ? plan_device_table_existing(p, st, &tab) : plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    const int64_t nzown = slab.own_hi - slab.own_lo;
    if (nzown <= 0) return CT_OK;
    // plans of views: the per-view kernels, except the exact adjoint of vertical views (circular and
    // helical scans), which the column kernel serves
    const bool vw_col = p->views && kind == CT_BP_ADJOINT && p->vertical && !slab.zcol && !direct_views_adjoint();
    if (p->views && !vw_col) return launch_backproject_views(p, kind, proj, pt, vol, vt, accumulate, a0, a1, slab, tab, st);
    if (slab.zcol && (kind != CT_BP_ADJOINT || !adj_col_ok(p)))
        return fail(CT_ERR_STATE, "a column-major slab needs the exact adjoint's column kernel");
    BpArgs A = make_bp_args(p, tab, a0, a1, slab, accumulate);
    // voxel-driven kernels: runs of slices aligned to absolute multiples of the run length
    auto runs = [&](int n) { return (unsigned)((slab.own_hi - 1) / n - slab.own_lo / n + 1); };
    const dim3 grid((A.nx + BP_TX - 1) / BP_TX, (A.ny + BP_TY - 1) / BP_TY,
                    kind == CT_BP_ADJOINT ? runs(ADJ_NZ) : runs(BP_NZ));
    const dim3 block(256);
    int WW = 0, HW = 0;
#ifndef CT_NO_BP_LDS
    if (kind != CT_BP_ADJOINT && bp_window(p->g, WW, HW)) {
        const bool narrow = WW <= BPL_PN;
        const int K = std::min(BPL_K, BPL_FLOATS / ((narrow ? BPL_PN : 64) * HW));
        const dim3 lgrid(grid.x, grid.y, runs(BPL_NZ));
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
        const int nr = p->g.nDetector[1] + 2 > ADJ_MAX_ROWS
                           ? 5
                           : std::min<int>(p->views ? adj_rows_views(p) : adj_rows(p->g), (int)p->g.nDetector[1] + 2);
        const size_t per_angle = adj_chunk_bytes_per_angle(p->g);
        void *yq = adj_scratch, *own = nullptr;
        size_t qcap = adj_scratch ? adj_bytes : 0;
        if (nr <= 4 && !yq && slab.scratch_ok) {
            if (CT_MALLOC_ASYNC(&own, (size_t)(a1 - a0) * per_angle, st) == hipSuccess) {
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
            // no voxel of the launch straddles the source plane (the kernel's own FP32 faces); views
            // take the general order
            bool ord = !p->views;
            if (ord) {
                const float dzf = A.dz, zf0 = (float)(A.dz0 - 0.5 * A.ddz);
                for (int64_t k = slab.own_lo; k < slab.own_hi && ord; ++k)
                    ord = !(std::fma((float)k, dzf, zf0) < 0.0f && std::fma((float)(k + 1), dzf, zf0) > 0.0f);
            }
            const int zgroups = (int)((nzown + 64 * R - 1) / (64 * R));
            const int xblocks = (A.nx + 3) / 4;
            const dim3 ag((unsigned)((int64_t)zgroups * xblocks * A.ny));
            const size_t pangle = (size_t)A.nu * A.nv * dtype_size(pt);
            const size_t rsbytes = (size_t)(A.nv + 2) * sizeof(float);  // the rows' parameter steps (LDS)
            for (int64_t c0 = a0; c0 < a1; c0 += kq) {
                const int64_t c1 = std::min(a1, c0 + kq);
                const BpArgs Ac = make_bp_args(p, tab, c0, c1, slab, c0 == a0 ? accumulate : 1);
                const void *pc = (const char *)proj + (size_t)(c0 - a0) * pangle;
                const dim3 pg((unsigned)((A.nu + 31) / 32), (unsigned)((A.nv + 2 + 31) / 32), (unsigned)(c1 - c0));
                CT_DISPATCH1(pt, TP,
                             hipLaunchKernelGGL((k_adj_prep<TP>), pg, dim3(256), 0, st, (const TP *)pc, (float *)yq, Ac));
                CT_HIP(hipGetLastError());
#define CT_ADJ_L(RR, NN, Z, O)                                                                                  \
    hipLaunchKernelGGL((k_adj_col<TV, RR, NN, Z, O>), ag, block, rsbytes, st, (const float *)yq, (TV *)vol, Ac, \
                       zgroups, xblocks)
#define CT_ADJ(RR, NN)                                                                                        \
    CT_DISPATCH1(vt, TV, if (p->views) {                                                                      \
        hipLaunchKernelGGL((k_adj_col<TV, RR, NN, false, false, true>), ag, block, rsbytes, st, (const float *)yq, \
                           (TV *)vol, Ac, zgroups, xblocks);                                                  \
    } else if (slab.zcol) {                                                                                   \
        if (ord) CT_ADJ_L(RR, NN, true, true);                                                                \
        else CT_ADJ_L(RR, NN, true, false);                                                                   \
    } else {                                                                                                  \
        if (ord) CT_ADJ_L(RR, NN, false, true);                                                               \
        else CT_ADJ_L(RR, NN, false, false);                                                                  \
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
        if (p->views) return launch_backproject_views(p, kind, proj, pt, vol, vt, accumulate, a0, a1, slab, tab, st);
        if (slab.zcol) return fail(CT_ERR_STATE, "a column-major slab needs the exact adjoint's column kernel");
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_adjoint<TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

// ------------------------------------------------------------------------------------------
// Backprojection that allocates nothing: the exact adjoint's transposed projection copy goes to a
// static device array (one per device, held until the process ends), filled in angle sub-chunks
// that fit it, with the voxel sums passed between sub-chunks through the volume (FP32 volumes:
// bitwise the same as one chunk).  The FDK and pseudo-matched kernels need no scratch.  Every
// call on a device shares that device's array, so calls that overlap on one device race; the
// array needs no clearing (each sub-chunk writes all of the copy it reads).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;  // one angle of a 3072^2 detector: 75.5 MB
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device id -> that device's address of `scratch`

// The device address of `scratch` on the current device (the array's name in host code is only a
// host-side handle), looked up once per device.
ct_status scratch_address(void **out) {
    int dev = 0;
    CT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        CT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(CT_ERR_HIP, "no device address for the backprojection scratch");
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return CT_OK;
}
}  // namespace

ct_status backproject_noalloc(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                              ct_dtype vt, int accumulate, int64_t a0, int64_t a1, hipStream_t st) {
    if (kind == CT_BP_ADJOINT && adj_col_ok(p) && adj_chunk_bytes_per_angle(p->g) > NOALLOC_SCRATCH_BYTES)
        return fail(CT_ERR_ARG, "ct_backproject_noalloc: one angle's transposed copy of the detector (" +
                                    std::to_string(adj_chunk_bytes_per_angle(p->g)) + " bytes) exceeds the " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch");
    void *scr = nullptr;
    ct_status s = scratch_address(&scr);
    if (s != CT_OK) return s;
    Slab sl = full_slab(p->g);
    sl.scratch_ok = false;
    sl.no_alloc = true;
    return launch_backproject(p, kind, proj, pt, vol, vt, accumulate, a0, a1, sl, st, scr, NOALLOC_SCRATCH_BYTES);
}

ct_status launch_sart_update(ct_plan *p, const float *r, float *vol, int64_t a0, int64_t a1, float lambda,
                             hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    if (p->views) return launch_sart_update_views(p, r, vol, a0, a1, lambda, tab, st);
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
