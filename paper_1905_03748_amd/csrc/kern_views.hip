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
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <mutex>

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

// The projector's FP64 constants that fix a pixel's ray: detector spacing, centre and offset, voxel
// size (rays parallel to a grid plane are decided from them).
struct RayConst {
    double du, dv, cu, cv, offu, offv, dx, dy, dz;
};

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
    RayConst K;              // the projector's FP64 constants (rays parallel to a grid plane)
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
    int ks[3];    // voxel indices whose half-open slabs hold the source's coordinates
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// FP64 direction (mm per unit t) of the ray of pixel (a, b) of view G, as the projector forms it.
__device__ __forceinline__ void ray_dir(const RayConst &K, const AngleGeo *G, int a, int b, double m[3]) {
    const double ua = (a - K.cu) * K.du + K.offu;
    const double vb = (b - K.cv) * K.dv + K.offv;
    m[0] = fma(vb, G->ev[0], G->Dc[0] + ua * G->eu[0]) * K.dx;
    m[1] = fma(vb, G->ev[1], G->Dc[1] + ua * G->eu[1]) * K.dy;
    m[2] = fma(vb, G->ev[2], fma(ua, G->eu[2], G->Dc[2])) * K.dz;
}

// FP32 direction D (mm) with a component within rounding of zero: |D_c| <= 1e-5 |D|.
__device__ __forceinline__ bool near_parallel(float D0, float D1, float D2) {
    const float lim = 1e-10f * fmaf(D0, D0, fmaf(D1, D1, D2 * D2));
    return D0 * D0 <= lim || D1 * D1 <= lim || D2 * D2 <= lim;
}

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

// Runs of NZ slices start at absolute multiples of NZ.
template <int NZ = VB_NZ>
__device__ __forceinline__ int run_base(const VArgs &A) { return (A.own_lo / NZ + (int)blockIdx.z) * NZ; }

// FDK, pseudo-matched or SART: bilinear taps at each voxel's own detector coordinates.
template <int MODE, typename TP, typename TV>
__global__ __launch_bounds__(256) void k_bp_views(const TP *__restrict__ proj, TV *__restrict__ vol, VArgs A) {
    __shared__ VRef ref[VB_G];
    __shared__ float iref[VB_G][2];
    const int i0 = blockIdx.x * VB_TX, j0 = blockIdx.y * VB_TY;
    const int i = i0 + (threadIdx.x % VB_TX);
    const int j = j0 + (threadIdx.x / VB_TX);
    const int kb = run_base<>(A);
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
                    wt[k] = R.w0 * __builtin_amdgcn_sqrtf(fmaf(sx, sx, fmaf(sy, sy, sz * sz))) * iw * iw * iw;
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

// FDK and pseudo-matched backprojection with the taps staged in LDS.  For each view the block
// projects the eight corners of its 16 x 16 x VL_NZ tile (clipped to the grid) through the local
// form of the projective map: a perspective map with positive depth over the box sends it into the
// convex hull of its corners' images, so the window [floor(min a*) - 1, ...] x [floor(min b*) - 1,
// ...] holds every bilinear tap of every voxel of the tile.  Its width is at most WW columns and its
// height at most HW rows under any tile and view (vl_window, on the host); each view's own height
// comes from its corners, and as many views as fit (up to VL_K) are staged together, windows one
// after another at a row pitch of PITCH floats (lanes on consecutive pixels, zeros off the
// detector).  Taps are clamped into their view's window, so no access leaves it.  The voxels read
// their taps there with the per-voxel arithmetic of k_bp_views; the view's constant factor of the
// weight (DSO_v^2, or the pseudo-matched constant) is applied to the staged pixels.
#ifndef CT_VL_NZ
#define CT_VL_NZ 16
#endif
constexpr int VL_NZ = CT_VL_NZ;  // voxels per thread
#ifndef CT_VL_FLOATS
#define CT_VL_FLOATS 4096
#endif
constexpr int VL_FLOATS = CT_VL_FLOATS;  // staged floats per block
constexpr int VL_G = 32;                 // views per group of tile references (8 corner lanes each)
constexpr int VL_PN = 41, VL_PW = 65;    // row pitches of narrow and wide windows
#ifndef CT_VL_K
#define CT_VL_K 8
#endif
constexpr int VL_K = CT_VL_K;            // views per staging round, at most
static_assert(VL_NZ * 256 <= VL_FLOATS, "the staging window parks the sums");
#ifndef CT_VL_WAVES
#define CT_VL_WAVES 6
#endif

// VERT: every view vertical (e_v = +z, e_u horizontal, the detector centre at the source's height),
// where the depth and a* are constant along a voxel column.
template <int MODE, int PITCH, bool VERT, typename TP, typename TV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CT_VL_WAVES))) void k_bp_views_lds(
    const TP *__restrict__ proj, TV *__restrict__ vol, VArgs A, int WW, int HW) {
    __shared__ float win[VL_FLOATS];
    __shared__ VRef ref[VL_G];
    __shared__ int org[VL_G][2];
    __shared__ int hgt[VL_G];
    const int i0 = blockIdx.x * VB_TX, j0 = blockIdx.y * VB_TY;
    const int tid = threadIdx.x;
    const int i = i0 + (tid % VB_TX);
    const int j = j0 + (tid / VB_TX);
    const int kb = run_base<VL_NZ>(A);
    const bool live = i < A.nx && j < A.ny;
    const double ir = tile_mid(i0, VB_TX, A.nx), jr = tile_mid(j0, VB_TY, A.ny), kr = tile_mid(kb, VL_NZ, A.nz);
    const float di = (float)((double)i - ir), dj = (float)((double)j - jr), dk0 = (float)((double)kb - kr);
    const int64_t psz = (int64_t)A.nu * A.nv;
    constexpr int ROWS = VL_FLOATS / PITCH;  // rows of the staging buffer
    const float lamax = (float)(WW - 2);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    // this thread's tile corner (offsets from the reference point, clipped to the grid)
    const int cn = tid & 7;
    const float cx = (float)((double)((cn & 1) ? min(i0 + VB_TX, A.nx) - 1 : i0) - ir);
    const float cy = (float)((double)((cn & 2) ? min(j0 + VB_TY, A.ny) - 1 : j0) - jr);
    const float cz = (float)((double)((cn & 4) ? min(kb + VL_NZ, A.nz) - 1 : kb) - kr);
    float acc[VL_NZ];
    for (int g0 = 0; g0 < A.nang; g0 += VL_G) {
        const int ng = min(VL_G, A.nang - g0);
        if (g0 > 0) {
            // park the sums in the window while the group's references are formed in FP64
            __syncthreads();  // the last round's taps have been read
#pragma unroll
            for (int k = 0; k < VL_NZ; ++k) win[k * 256 + tid] = acc[k];
        }
        if (tid < ng) {
            VRef R;
            float fa, fb;
            view_ref<MODE>(A, A.tab[A.a0 + g0 + tid], ir, jr, kr, R, fa, fb);
            ref[tid] = R;
            org[tid][0] = (int)fa;
            org[tid][1] = (int)fb;
        }
        __syncthreads();
        {
            // lanes 8q .. 8q + 7: the tile's corners under view q of the group (FP32, relative to
            // the view's integer origin), reduced to the window's origin and height
            const int q = tid >> 3;
            float as = 0.0f, bs = 0.0f;
            if (q < ng) {
                const VRef &R = ref[q];
                const float w = fmaf(R.mw[0], cx, fmaf(R.mw[1], cy, fmaf(R.mw[2], cz, R.wr)));
                const float iw = __builtin_amdgcn_rcpf(w);
                // far off the detector every tap reads zero; the clamp keeps the integers small
                as = __builtin_amdgcn_fmed3f(fmaf(fmaf(R.ga[0], cx, fmaf(R.ga[1], cy, R.ga[2] * cz)), iw, R.Aloc),
                                             -16777216.0f, 16777216.0f);
                bs = __builtin_amdgcn_fmed3f(fmaf(fmaf(R.gb[0], cx, fmaf(R.gb[1], cy, R.gb[2] * cz)), iw, R.Bloc),
                                             -16777216.0f, 16777216.0f);
            }
            float amin = as, bmin = bs, bmax = bs;
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                amin = fminf(amin, __shfl_xor(amin, off, 64));
                bmin = fminf(bmin, __shfl_xor(bmin, off, 64));
                bmax = fmaxf(bmax, __shfl_xor(bmax, off, 64));
            }
            __syncthreads();  // every corner has read its reference
            if (cn == 0 && q < ng) {
                const int wa = (int)floorf(amin) - 1, wb = (int)floorf(bmin) - 1;
                ref[q].Aloc -= (float)wa;
                ref[q].Bloc -= (float)wb;
                org[q][0] += wa;
                org[q][1] += wb;
                // rows wb .. floor(bmax) + 2: the taps' rows with a row of margin each side
                hgt[q] = min((int)floorf(bmax) - wb + 3, HW);
            }
        }
        __syncthreads();
        if (g0 == 0) {
            // one base address, slices a uniform stride apart (the stride is hidden from the
            // compiler so the addresses of all slices are not kept live from the start)
            int64_t sl = (int64_t)A.nx * A.ny;
            asm volatile("" : "+s"(sl));
            const TV *vb = vol + ((int64_t)(kb - A.mem_lo) * A.ny + j) * A.nx + i;
#pragma unroll
            for (int k = 0; k < VL_NZ; ++k) {
                const int kk = kb + k;
                acc[k] = (live && A.accumulate && kk >= A.own_lo && kk < A.own_hi) ? to_f(vb[k * sl]) : 0.0f;
            }
        } else {
#pragma unroll
            for (int k = 0; k < VL_NZ; ++k) acc[k] = win[k * 256 + tid];
        }
        for (int t0 = 0; t0 < ng;) {
            // the views t0 .. t1 - 1 whose windows fit the buffer together (at least one: HW <= ROWS)
            int t1 = t0, rows = 0;
            while (t1 < ng && t1 - t0 < VL_K && rows + hgt[t1] <= ROWS) rows += hgt[t1++];
            __syncthreads();  // the buffer is free (parked sums read back, or the last round's taps read)
            // stage: wave w copies rows w, w + 4, ... of every window; lane = window column
            int rb = 0;
            for (int q = t0; q < t1; ++q) {
                const int h = hgt[q];
                const int u = org[q][0] + lane;
                const bool uok = lane < WW && (unsigned)u < (unsigned)A.nu;
                const TP *pq = proj + (int64_t)(g0 + q) * psz + u;
                float *wq = win + rb * PITCH + lane;
                const int ob = org[q][1];
                const float w0 = ref[q].w0;
                const float sc = MODE == VM_PM ? w0 : w0 * w0;
                for (int r = wave; r < h; r += 4) {
                    const int v = ob + r;
                    float val = 0.0f;
                    if (uok && (unsigned)v < (unsigned)A.nv) val = to_f(pq[(int64_t)v * A.nu]) * sc;
                    if (lane < WW) wq[r * PITCH] = val;
                }
                rb += h;
            }
            __syncthreads();
            if (live) {
                rb = 0;
                for (int q = t0; q < t1; ++q) {
                    const VRef R = ref[q];
                    const int h = hgt[q];
                    const float lbmax = (float)(h - 2);
                    const float qb = (float)(rb * PITCH * 4);
                    rb += h;
                    const float wxy = fmaf(R.mw[0], di, fmaf(R.mw[1], dj, R.wr));
                    const float axy = fmaf(R.ga[0], di, R.ga[1] * dj), bxy = fmaf(R.gb[0], di, R.gb[1] * dj);
                    const float sx = fmaf(di, A.dx, R.sx), sy = fmaf(dj, A.dy, R.sy);
                    const float sxy2 = fmaf(sx, sx, sy * sy);
                    if constexpr (VERT) {
                        // vertical views: the depth and a* do not change along the column, so the
                        // column's tap column, fraction and FDK weight are formed once; b* is affine in k
                        const float iw = __builtin_amdgcn_rcpf(wxy);
                        const float as = fmaf(axy, iw, R.Aloc);
                        const float af = floorf(as);
                        const float fa = as - af;
                        const float cb = fmaf(__builtin_amdgcn_fmed3f(af, 0.0f, lamax), 4.0f, qb);
                        const float b0 = fmaf(bxy, iw, R.Bloc), db = R.gb[2] * iw;
                        const float iw2 = iw * iw, iw3 = iw2 * iw;
#pragma unroll
                        for (int k = 0; k < VL_NZ; ++k) {
                            const float dk = dk0 + (float)k;
                            const float bs = fmaf(dk, db, b0);
                            const float bf = floorf(bs);
                            const float fb = bs - bf;
                            const float lb = __builtin_amdgcn_fmed3f(bf, 0.0f, lbmax);
                            const float *t = (const float *)((const char *)win + (int)fmaf(lb, (float)(4 * PITCH), cb));
                            const float v0 = fmaf(fa, t[1] - t[0], t[0]);
                            const float v1 = fmaf(fa, t[PITCH + 1] - t[PITCH], t[PITCH]);
                            const float v = fmaf(fb, v1 - v0, v0);
                            float wt;
                            if (MODE == VM_PM) {
                                const float sz = fmaf(dk, A.dz, R.sz);
                                wt = __builtin_amdgcn_sqrtf(fmaf(sz, sz, sxy2)) * iw3;
                            } else {
                                wt = iw2;
                            }
                            acc[k] = fmaf(wt, v, acc[k]);
                        }
                        continue;
                    }
#pragma unroll
                    for (int k = 0; k < VL_NZ; ++k) {
                        const float dk = dk0 + (float)k;
                        const float w = fmaf(R.mw[2], dk, wxy);
                        const float iw = __builtin_amdgcn_rcpf(w);
                        const float as = fmaf(fmaf(R.ga[2], dk, axy), iw, R.Aloc);
                        const float bs = fmaf(fmaf(R.gb[2], dk, bxy), iw, R.Bloc);
                        const float af = floorf(as), bf = floorf(bs);
                        const float fa = as - af, fb = bs - bf;
                        // LDS byte offset of the tap pair, clamped into the window (exact in FP32)
                        const float la = __builtin_amdgcn_fmed3f(af, 0.0f, lamax);
                        const float lb = __builtin_amdgcn_fmed3f(bf, 0.0f, lbmax);
                        const float *t =
                            (const float *)((const char *)win + (int)fmaf(lb, (float)(4 * PITCH), fmaf(la, 4.0f, qb)));
                        const float v0 = fmaf(fa, t[1] - t[0], t[0]);
                        const float v1 = fmaf(fa, t[PITCH + 1] - t[PITCH], t[PITCH]);
                        const float v = fmaf(fb, v1 - v0, v0);
                        float wt;
                        if (MODE == VM_PM) {
                            const float sz = fmaf(dk, A.dz, R.sz);
                            wt = __builtin_amdgcn_sqrtf(fmaf(sz, sz, sxy2)) * iw * iw * iw;
                        } else {
                            wt = iw * iw;
                        }
                        acc[k] = fmaf(wt, v, acc[k]);
                    }
                }
            }
            t0 = t1;
        }
    }
    if (!live || A.nang <= 0) return;
    int64_t sl = (int64_t)A.nx * A.ny;
    asm volatile("" : "+s"(sl));
    TV *vs = vol + ((int64_t)(kb - A.mem_lo) * A.ny + j) * A.nx + i;
#pragma unroll
    for (int k = 0; k < VL_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.own_lo) continue;
        if (kk >= A.own_hi) break;
        vs[k * sl] = from_f<TV>(acc[k]);
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
    const int kb = run_base<>(A);
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
            P.ks[0] = (int)fmin(fmax(floor(G.S[0] + 0.5), -2.0), 1e9);
            P.ks[1] = (int)fmin(fmax(floor(G.S[1] + 0.5), -2.0), 1e9);
            P.ks[2] = (int)fmin(fmax(floor(G.S[2] + 0.5), -2.0), 1e9);
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
                        const int vq[3] = {i, j, kb + k};
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (Dq[c] == 0.0f) {
                                // the ray runs in the plane of the source's coordinate: the voxel must
                                // hold it in its half-open slab [k - 1/2, k + 1/2), as in the projector
                                in = in && vq[c] == P.ks[c];
                            } else {
                                const float inv = __builtin_amdgcn_rcpf(Dq[c]);
                                const float t1 = (-Hq[c] - Qq[c]) * inv, t2 = (Hq[c] - Qq[c]) * inv;
                                tlo = fmaxf(tlo, fminf(t1, t2));
                                thi = fminf(thi, fmaxf(t1, t2));
                            }
                        }
                        const float len = (in && thi > tlo) ? (thi - tlo) * __builtin_amdgcn_sqrtf(fmaf(D0, D0, fmaf(D1, D1, D2 * D2))) : 0.0f;
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

// The exact adjoint with each tile's rays staged in LDS.  The arithmetic per (voxel, pixel) is that
// of k_adj_views, but what depends on the pixel alone is formed once per block and view: for every
// pixel of the window holding the image of the tile's voxel boxes (corners projected as in
// k_bp_views_lds, heights per view, windows packed at a row pitch of PITCH records), the
// reciprocals of the ray direction's components and the pixel's value times |P - S|.  A candidate
// pixel then costs one 16-byte LDS read and the slab test without reciprocals or a square root.  A
// ray within FP32 rounding of a grid plane has its record formed from the FP64 direction, which
// decides, as the projector does, whether it runs parallel to the plane; such an axis is NaN in the
// record, and a view whose window holds one reads its records with the half-open slab rule for it.
constexpr int VA_REC = 2048;  // pixel records (16 B) per block
constexpr int VA_G = 32;      // views per group of tile references
#ifndef CT_VA_K
#define CT_VA_K 8
#endif
constexpr int VA_K = CT_VA_K;  // views per staging round, at most
constexpr int VA_PN = 41, VA_PW = 65;

template <typename TP, typename TV, int PITCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_adj_views_lds(const TP *__restrict__ proj, TV *__restrict__ vol, VArgs A, int WW,
                                                      int HW) {
    __shared__ float4 rec[VA_REC];
    __shared__ VRef ref[VA_G];
    __shared__ float iref[VA_G][2];
    __shared__ VPix pixg[VA_G];
    __shared__ int org[VA_G][2];
    __shared__ int hgt[VA_G];
    __shared__ int zfl[VA_G];
    const int i0 = blockIdx.x * VB_TX, j0 = blockIdx.y * VB_TY;
    const int tid = threadIdx.x;
    const int i = i0 + (tid % VB_TX);
    const int j = j0 + (tid / VB_TX);
    const int kb = run_base<>(A);
    const bool live = i < A.nx && j < A.ny;
    const double ir = tile_mid(i0, VB_TX, A.nx), jr = tile_mid(j0, VB_TY, A.ny), kr = tile_mid(kb, VB_NZ, A.nz);
    const float di = (float)((double)i - ir), dj = (float)((double)j - jr);
    const float hx = 0.5f * A.dx, hy = 0.5f * A.dy, hz = 0.5f * A.dz;
    constexpr int ROWS = VA_REC / PITCH;
    // this thread's corner of the tile's voxel boxes (offsets from the reference point, clipped to the grid)
    const int cn = tid & 7;
    const float cx = (float)(((cn & 1) ? (double)min(i0 + VB_TX, A.nx) - 0.5 : (double)i0 - 0.5) - ir);
    const float cy = (float)(((cn & 2) ? (double)min(j0 + VB_TY, A.ny) - 0.5 : (double)j0 - 0.5) - jr);
    const float cz = (float)(((cn & 4) ? (double)min(kb + VB_NZ, A.nz) - 0.5 : (double)kb - 0.5) - kr);
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
    for (int g0 = 0; g0 < A.nang; g0 += VA_G) {
        const int ng = min(VA_G, A.nang - g0);
        __syncthreads();  // the last group's references and records have been read
        if (tid < ng) {
            const AngleGeo &G = A.tab[A.a0 + g0 + tid];
            VRef R;
            float fa, fb;
            view_ref<VM_ADJ>(A, G, ir, jr, kr, R, fa, fb);
            ref[tid] = R;
            iref[tid][0] = fa;
            iref[tid][1] = fb;
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
            P.ks[0] = (int)fmin(fmax(floor(G.S[0] + 0.5), -2.0), 1e9);
            P.ks[1] = (int)fmin(fmax(floor(G.S[1] + 0.5), -2.0), 1e9);
            P.ks[2] = (int)fmin(fmax(floor(G.S[2] + 0.5), -2.0), 1e9);
            pixg[tid] = P;
            zfl[tid] = 0;
        }
        __syncthreads();
        {
            // lanes 8q .. 8q + 7: the corners of the tile's voxel boxes under view q (FP32, relative to
            // the view's integer origin), reduced to the window's origin and height
            const int q = tid >> 3;
            float as = 0.0f, bs = 0.0f;
            if (q < ng) {
                const VRef &R = ref[q];
                const float w = fmaf(R.mw[0], cx, fmaf(R.mw[1], cy, fmaf(R.mw[2], cz, R.wr)));
                const float iw = __builtin_amdgcn_rcpf(w);
                as = __builtin_amdgcn_fmed3f(fmaf(fmaf(R.ga[0], cx, fmaf(R.ga[1], cy, R.ga[2] * cz)), iw, R.Aloc),
                                             -16777216.0f, 16777216.0f);
                bs = __builtin_amdgcn_fmed3f(fmaf(fmaf(R.gb[0], cx, fmaf(R.gb[1], cy, R.gb[2] * cz)), iw, R.Bloc),
                                             -16777216.0f, 16777216.0f);
            }
            float amin = as, bmin = bs, bmax = bs;
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                amin = fminf(amin, __shfl_xor(amin, off, 64));
                bmin = fminf(bmin, __shfl_xor(bmin, off, 64));
                bmax = fmaxf(bmax, __shfl_xor(bmax, off, 64));
            }
            if (cn == 0 && q < ng) {
                // pixels whose centres can fall in the image: columns from ceil(min a*), rows from
                // ceil(min b*) to floor(max b*), with a pixel of margin each side
                const int wa = (int)floorf(amin) - 1, wb = (int)floorf(bmin) - 1;
                org[q][0] = (int)iref[q][0] + wa;
                org[q][1] = (int)iref[q][1] + wb;
                hgt[q] = min((int)floorf(bmax) - wb + 2, HW);
            }
        }
        __syncthreads();
        for (int t0 = 0; t0 < ng;) {
            // the views t0 .. t1 - 1 whose windows fit the buffer together (at least one: HW <= ROWS)
            int t1 = t0, rows = 0;
            while (t1 < ng && t1 - t0 < VA_K && rows + hgt[t1] <= ROWS) rows += hgt[t1++];
            __syncthreads();  // the last round's records have been read
            // records of the round's windows, one thread per pixel
            for (int pix = tid; pix < rows * PITCH; pix += 256) {
                int r = pix / PITCH, q = t0;
                const int c = pix - r * PITCH;
                while (r >= hgt[q]) r -= hgt[q++];
                const int a = org[q][0] + c, b = org[q][1] + r;
                float4 R4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (c < WW && (unsigned)a < (unsigned)A.nu && (unsigned)b < (unsigned)A.nv) {
                    const VPix &P = pixg[q];
                    const float y = to_f(proj[(int64_t)(g0 + q) * psz + (int64_t)b * A.nu + a]);
                    // the ray direction as k_adj_views forms it
                    const float vb = fmaf((float)b - A.cv, A.dv, A.offv);
                    const float ua = fmaf((float)a - A.cu, A.du, A.offu);
                    const float D0 = fmaf(ua, P.eu[0], fmaf(vb, P.ev[0], P.cs[0]));
                    const float D1 = fmaf(ua, P.eu[1], fmaf(vb, P.ev[1], P.cs[1]));
                    const float D2 = fmaf(ua, P.eu[2], fmaf(vb, P.ev[2], P.cs[2]));
                    R4 = make_float4(__builtin_amdgcn_rcpf(D0), __builtin_amdgcn_rcpf(D1), __builtin_amdgcn_rcpf(D2),
                                     y * __builtin_amdgcn_sqrtf(fmaf(D0, D0, fmaf(D1, D1, D2 * D2))));
                    if (near_parallel(D0, D1, D2)) {
                        // within FP32 rounding of a grid plane: the FP64 direction decides, as the
                        // projector decides, which axes the ray runs parallel to (NaN in the record, and
                        // the view takes the form that reads it); the others take FP64 reciprocals
                        double m[3];
                        ray_dir(A.K, A.tab + A.a0 + g0 + q, a, b, m);
                        const double L = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
                        float rr[3];
                        bool par = false;
#pragma unroll
                        for (int c2 = 0; c2 < 3; ++c2) {
                            const bool pc = fabs(m[c2]) < 1e-12 * L;
                            par = par || pc;
                            rr[c2] = pc ? __builtin_nanf("") : (float)(1.0 / m[c2]);
                        }
                        R4 = make_float4(rr[0], rr[1], rr[2], (float)(y * L));
                        if (par) atomicOr(&zfl[q], 1);
                    }
                }
                rec[pix] = R4;
            }
            __syncthreads();
            if (live) {
                int rb = 0;
                for (int q = t0; q < t1; ++q) {
                    const VRef R = ref[q];
                    const VPix P = pixg[q];
                    const float oa = iref[q][0], ob = iref[q][1];
                    const int wa0 = org[q][0], wb0 = org[q][1], h = hgt[q];
                    const bool slow = zfl[q] != 0;
                    const int rbase = rb * PITCH - wa0;  // record of pixel (a, b): rbase + (b - wb0) PITCH + a
                    rb += h;
                    const float wxy = fmaf(R.mw[0], di, fmaf(R.mw[1], dj, R.wr));
                    const float axy = fmaf(R.ga[0], di, R.ga[1] * dj), bxy = fmaf(R.gb[0], di, R.gb[1] * dj);
#pragma unroll
                    for (int k = 0; k < VB_NZ; ++k) {
                        const float dkk = (float)((double)(kb + k) - kr);
                        const float w = fmaf(R.mw[2], dkk, wxy);
                        const float iw = __builtin_amdgcn_rcpf(w);
                        const float al = fmaf(R.ga[2], dkk, axy) * iw, be = fmaf(R.gb[2], dkk, bxy) * iw;
                        const float ha = 0.5f * (fabsf(fmaf(-al, R.mw[0], R.ga[0])) + fabsf(fmaf(-al, R.mw[1], R.ga[1])) +
                                                 fabsf(fmaf(-al, R.mw[2], R.ga[2]))) * iw;
                        const float hb = 0.5f * (fabsf(fmaf(-be, R.mw[0], R.gb[0])) + fabsf(fmaf(-be, R.mw[1], R.gb[1])) +
                                                 fabsf(fmaf(-be, R.mw[2], R.gb[2]))) * iw;
                        const float as = al + R.Aloc, bs = be + R.Bloc;
                        const float ma = fmaf(ha, 0.02f, 1e-3f), mb = fmaf(hb, 0.02f, 1e-3f);
                        const float fnu = (float)A.nu, fnv = (float)A.nv;
                        // candidate pixels, clamped to the detector and to the view's window
                        const int alo = max((int)fmaxf(oa + ceilf(as - ha - ma), 0.0f), wa0);
                        const int ahi = min((int)fminf(oa + floorf(as + ha + ma), fnu - 1.0f), wa0 + WW - 1);
                        const int blo = max((int)fmaxf(ob + ceilf(bs - hb - mb), 0.0f), wb0);
                        const int bhi = min((int)fminf(ob + floorf(bs + hb + mb), fnv - 1.0f), wb0 + h - 1);
                        const float sc = w * R.w0;
                        const float qa0 = sc * A.du * P.eu[0], qa1 = sc * A.du * P.eu[1], qa2 = sc * A.du * P.eu[2];
                        const float qb0 = sc * A.dv * P.ev[0], qb1 = sc * A.dv * P.ev[1], qb2 = sc * A.dv * P.ev[2];
                        float s = 0.0f;
                        if (!slow) {
                            for (int b = blo; b <= bhi; ++b) {
                                const float db = ((float)b - ob) - bs;
                                const float pb0 = db * qb0, pb1 = db * qb1, pb2 = db * qb2;
                                const float4 *rrow = rec + (rbase + (b - wb0) * PITCH);
                                for (int a = alo; a <= ahi; ++a) {
                                    const float da = ((float)a - oa) - as;
                                    const float Q0 = fmaf(da, qa0, pb0), Q1 = fmaf(da, qa1, pb1), Q2 = fmaf(da, qa2, pb2);
                                    const float4 ry = rrow[a];
                                    // slab of each axis: t in -Q / D -+ h / |D|
                                    const float m0 = -Q0 * ry.x, m1 = -Q1 * ry.y, m2 = -Q2 * ry.z;
                                    const float e0 = hx * fabsf(ry.x), e1 = hy * fabsf(ry.y), e2 = hz * fabsf(ry.z);
                                    const float tlo = fmaxf(fmaxf(m0 - e0, m1 - e1), m2 - e2);
                                    const float thi = fminf(fminf(m0 + e0, m1 + e1), m2 + e2);
                                    s = fmaf(fmaxf(thi - tlo, 0.0f), ry.w, s);
                                }
                            }
                        } else {
                            // records of rays parallel to a grid plane carry NaN for that axis: the voxel
                            // must then hold the source's coordinate in its half-open slab
                            for (int b = blo; b <= bhi; ++b) {
                                const float db = ((float)b - ob) - bs;
                                const float pb0 = db * qb0, pb1 = db * qb1, pb2 = db * qb2;
                                const float4 *rrow = rec + (rbase + (b - wb0) * PITCH);
                                for (int a = alo; a <= ahi; ++a) {
                                    const float da = ((float)a - oa) - as;
                                    const float Q0 = fmaf(da, qa0, pb0), Q1 = fmaf(da, qa1, pb1), Q2 = fmaf(da, qa2, pb2);
                                    const float4 ry = rrow[a];
                                    const float rq[3] = {ry.x, ry.y, ry.z}, Qq[3] = {Q0, Q1, Q2}, Hq[3] = {hx, hy, hz};
                                    const int vq[3] = {i, j, kb + k};
                                    float tlo = -FLT_MAX, thi = FLT_MAX;
                                    bool in = true;
#pragma unroll
                                    for (int c = 0; c < 3; ++c) {
                                        if (rq[c] != rq[c]) {
                                            in = in && vq[c] == P.ks[c];
                                        } else {
                                            const float m = -Qq[c] * rq[c], e = Hq[c] * fabsf(rq[c]);
                                            tlo = fmaxf(tlo, m - e);
                                            thi = fminf(thi, m + e);
                                        }
                                    }
                                    if (in) s = fmaf(fmaxf(thi - tlo, 0.0f), ry.w, s);
                                }
                            }
                        }
                        acc[k] += s;
                    }
                }
            }
            t0 = t1;
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < VB_NZ; ++k) {
        const int kk = kb + k;
        if (kk < A.own_lo) continue;
        if (kk >= A.own_hi) break;
        vol[((int64_t)(kk - A.mem_lo) * A.ny + j) * A.nx + i] = from_f<TV>(acc[k]);
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
    A.K = RayConst{g.dDetector[0], g.dDetector[1], (g.nDetector[0] - 1) / 2.0, (g.nDetector[1] - 1) / 2.0,
                   g.offDetector[0], g.offDetector[1], g.dVoxel[0], g.dVoxel[1], g.dVoxel[2]};
    return A;
}

// CT_VIEWS_BP_DIRECT=1 sends the FDK and pseudo-matched backprojections of plans of views to the
// kernel without LDS staging (tests compare the two).
bool direct_views_bp() {
    const char *e = std::getenv("CT_VIEWS_BP_DIRECT");
    return e && e[0] == '1';
}

dim3 vgrid(const VArgs &A, const Slab &slab, int nz = VB_NZ) {
    const unsigned runs = (unsigned)((slab.own_hi - 1) / nz - slab.own_lo / nz + 1);
    return dim3((unsigned)((A.nx + VB_TX - 1) / VB_TX), (unsigned)((A.ny + VB_TY - 1) / VB_TY), runs);
}

// Detector window (columns WW, rows HW) holding the image of any 16 x 16 x TZ tile of voxel centres
// (box = false: the backprojectors' bilinear taps) or of voxel boxes (box = true: the pixels whose
// rays can cross the tile), clipped to the grid, under any view of the plan; the staging buffer's
// limits (rows, pitch) are checked by the caller.
// With L = n.(S - X) the depth, p = e_u.(X - S) and a* = const + DSD_v p / (L du), two points of a
// tile differ in a* by at most DSD_v (E_p / L_min + |p|_max E_L / L_min^2) / du, where E_p and E_L
// bound the change of p and L over the tile's extent (the sums of |e_u| and |n| times the extent
// along each axis), and L_min and |p|_max are taken over the corners of a box holding the tile (both
// are affine in X).  The grid is cut into VL_NS^3 boxes, each grown by a tile's extent so that every
// tile lies in one, and the largest bound is kept; likewise for b* with e_v.  Margins: one pixel
// each side plus the second tap.  0 x 0 when a view's depth is not positive or the window is
// implausibly large.
constexpr int VL_NS = 4;
void window_bound(const ct_plan *p, int64_t tz, bool box, int &WW, int &HW) {
    const ct_geometry &g = p->g;
    double x0[3], x1[3], ext[3];
    const int64_t tn[3] = {VB_TX, VB_TY, tz};
    const double grow = box ? 0.5 : 0.0;  // voxel boxes reach half a voxel past the centres
    for (int a = 0; a < 3; ++a) {
        x0[a] = g.offOrigin[a] - ((g.nVoxel[a] - 1) / 2.0 + grow) * g.dVoxel[a];
        x1[a] = g.offOrigin[a] + ((g.nVoxel[a] - 1) / 2.0 + grow) * g.dVoxel[a];
        ext[a] = ((double)(std::min(tn[a], g.nVoxel[a]) - 1) + 2.0 * grow) * g.dVoxel[a];
    }
    double eu_max = 0.0, ev_max = 0.0;
    bool ok = true;
    for (const AngleGeo &t : p->tab) {
        double eu[3], ev[3];
        for (int a = 0; a < 3; ++a) {
            eu[a] = t.eu[a] * g.dVoxel[a];
            ev[a] = t.ev[a] * g.dVoxel[a];
        }
        const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        double Ep = 0.0, Eq = 0.0, EL = 0.0;
        for (int a = 0; a < 3; ++a) {
            Ep += std::fabs(eu[a]) * ext[a];
            Eq += std::fabs(ev[a]) * ext[a];
            EL += std::fabs(n[a]) * ext[a];
        }
        for (int b = 0; b < VL_NS * VL_NS * VL_NS; ++b) {
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                const int s = a == 0 ? b % VL_NS : a == 1 ? (b / VL_NS) % VL_NS : b / (VL_NS * VL_NS);
                lo[a] = std::max(x0[a] + (x1[a] - x0[a]) * s / VL_NS - ext[a], x0[a]);
                hi[a] = std::min(x0[a] + (x1[a] - x0[a]) * (s + 1) / VL_NS + ext[a], x1[a]);
            }
            double Lmin = HUGE_VAL, Pu = 0.0, Pv = 0.0;
            for (int c = 0; c < 8; ++c) {
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = (((c >> a) & 1) ? hi[a] : lo[a]) - t.Smm[a];
                Lmin = std::min(Lmin, -(n[0] * d[0] + n[1] * d[1] + n[2] * d[2]));
                Pu = std::max(Pu, std::fabs(eu[0] * d[0] + eu[1] * d[1] + eu[2] * d[2]));
                Pv = std::max(Pv, std::fabs(ev[0] * d[0] + ev[1] * d[1] + ev[2] * d[2]));
            }
            ok = ok && Lmin > 0.0;
            if (!ok) break;
            eu_max = std::max(eu_max, t.DSDv * (Ep / Lmin + Pu * EL / (Lmin * Lmin)) / g.dDetector[0]);
            ev_max = std::max(ev_max, t.DSDv * (Eq / Lmin + Pv * EL / (Lmin * Lmin)) / g.dDetector[1]);
        }
        if (!ok || !(eu_max < 62.0 && ev_max < 1000.0)) {
            ok = false;
            break;
        }
    }
    WW = HW = 0;
    if (ok) {
        WW = (int)std::ceil(eu_max) + 4;
        HW = (int)std::ceil(ev_max) + 4;
    }
}

// The exact adjoint's window (16 x 16 x VB_NZ tiles of voxel boxes), once per plan; 0 x 0 when it
// does not fit the records (VA_REC, at a pitch of at most VA_PW).
void va_window(ct_plan *p, int &WW, int &HW) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->va_ww < 0) {
        window_bound(p, VB_NZ, true, WW, HW);
        if (WW > VA_PW || HW > VA_REC / (WW <= VA_PN ? VA_PN : VA_PW)) WW = HW = 0;
        p->va_ww = WW;
        p->va_hw = HW;
    }
    WW = p->va_ww;
    HW = p->va_hw;
}

// CT_VIEWS_ADJ_DIRECT=1 sends the exact adjoint of plans of views to k_adj_views (no staging), =2 to
// the staged per-view kernel even for vertical views (tests compare them).
int views_adjoint_mode() {
    const char *e = std::getenv("CT_VIEWS_ADJ_DIRECT");
    return e && (e[0] == '1' || e[0] == '2') ? e[0] - '0' : 0;
}

// The backprojectors' window (16 x 16 x VL_NZ tiles of voxel centres), once per plan; 0 x 0 when it
// does not fit the staging buffer (one lane per window column, VL_FLOATS floats).
void vl_window(ct_plan *p, int &WW, int &HW) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->vl_ww < 0) {
        window_bound(p, VL_NZ, false, WW, HW);
        if (WW > 64 || HW > VL_FLOATS / (WW <= VL_PN ? VL_PN : VL_PW)) WW = HW = 0;
        p->vl_ww = WW;
        p->vl_hw = HW;
    }
    WW = p->vl_ww;
    HW = p->vl_hw;
}
}  // namespace

ct_status launch_backproject_views(ct_plan *p, ct_backprojector kind, const void *proj, ct_dtype pt, void *vol,
                                   ct_dtype vt, int accumulate, int64_t a0, int64_t a1, const Slab &slab,
                                   const AngleGeo *tab, hipStream_t st) {
    if (slab.own_hi <= slab.own_lo) return CT_OK;
    if (slab.zcol) return fail(CT_ERR_STATE, "a plan of views backprojects into [z][y][x] volumes only");
    const VArgs A = make_vargs(p, tab, a0, a1, slab, accumulate);
    const dim3 grid = vgrid(A, slab), block(256);
    int WW = 0, HW = 0;
    if (kind != CT_BP_ADJOINT) vl_window(p, WW, HW);
    if (WW > 0 && !direct_views_bp()) {
        const bool narrow = WW <= VL_PN;
        const dim3 lgrid = vgrid(A, slab, VL_NZ);
#define CT_VL2(MODE, PITCH, VERT)                                                                               \
    CT_DISPATCH2(pt, TP, vt, TV,                                                                                \
                 hipLaunchKernelGGL((k_bp_views_lds<MODE, PITCH, VERT, TP, TV>), lgrid, block, 0, st,           \
                                    (const TP *)proj, (TV *)vol, A, WW, HW))
#define CT_VL(MODE, PITCH)              \
    if (p->vertical) {                  \
        CT_VL2(MODE, PITCH, true);      \
    } else {                            \
        CT_VL2(MODE, PITCH, false);     \
    }
        if (kind == CT_BP_FDK) {
            if (narrow) {
                CT_VL(VM_FDK, VL_PN);
            } else {
                CT_VL(VM_FDK, VL_PW);
            }
        } else {
            if (narrow) {
                CT_VL(VM_PM, VL_PN);
            } else {
                CT_VL(VM_PM, VL_PW);
            }
        }
#undef CT_VL
#undef CT_VL2
        CT_HIP(hipGetLastError());
        return CT_OK;
    }
    if (kind == CT_BP_FDK) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_views<VM_FDK, TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    } else if (kind == CT_BP_PSEUDO_MATCHED) {
        CT_DISPATCH2(pt, TP, vt, TV,
                     hipLaunchKernelGGL((k_bp_views<VM_PM, TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
    } else {
        int AW = 0, AH = 0;
        va_window(p, AW, AH);
        if (AW > 0 && views_adjoint_mode() != 1) {
            if (AW <= VA_PN) {
                CT_DISPATCH2(pt, TP, vt, TV,
                             hipLaunchKernelGGL((k_adj_views_lds<TP, TV, VA_PN>), grid, block, 0, st, (const TP *)proj,
                                                (TV *)vol, A, AW, AH));
            } else {
                CT_DISPATCH2(pt, TP, vt, TV,
                             hipLaunchKernelGGL((k_adj_views_lds<TP, TV, VA_PW>), grid, block, 0, st, (const TP *)proj,
                                                (TV *)vol, A, AW, AH));
            }
        } else {
            CT_DISPATCH2(pt, TP, vt, TV,
                         hipLaunchKernelGGL((k_adj_views<TP, TV>), grid, block, 0, st, (const TP *)proj, (TV *)vol, A));
        }
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
