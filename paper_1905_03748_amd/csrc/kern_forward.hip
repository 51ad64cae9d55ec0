// Ray-driven forward projectors (Section 2.1): one thread per detector pixel.
//
// Rays are set up in FP64 in voxel-index space (the source is ~DSO/d voxels from the grid, so an
// FP32 set-up would misplace rays by ~1e-4 voxel), clipped to the grid (or to a z-slab of it for
// the out-of-core schedule), and then traversed in FP32 relative to the entry voxel, where all
// quantities are O(grid size) and plane crossings are formed as t0 + n * dt by one FMA each.
//
// Launch shape: 256-thread blocks covering 64 pixels along u (one wave = 64 adjacent pixels of
// one detector row, whose rays are nearly parallel and walk neighbouring voxels) by 4 rows.  Blocks are linearised as (u-tile fastest, then angle, then v-band) so the blocks in
// flight at any moment share a band of detector rows across many angles, i.e. an axial slab of
// the volume, which keeps the working set inside the 256 MB last-level cache.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "dev_common.hpp"

namespace ct {

namespace {

#ifndef CT_FWD_TV
#define CT_FWD_TV 4
#endif
constexpr int FWD_TU = 64;         // pixels per block along u (one wave)
constexpr int FWD_TV = CT_FWD_TV;  // rows per block (waves per block)

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
    int32_t cblocks, rgroups;  // column Siddon: column groups per angle, row groups per column
    int32_t gen;               // a plan of views: rays take e_v (and e_u, C - S) in all three axes
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
    if (A.gen) {
        // pixel centre C + ua e_u + vb e_v for any detector pose
        R.D[0] = fma(vb, G.ev[0], R.D[0]);
        R.D[1] = fma(vb, G.ev[1], R.D[1]);
        R.D[2] = fma(vb, G.ev[2], fma(ua, G.eu[2], G.Dc[2]));
    }
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

#ifndef CT_FWD_XCD_W
#define CT_FWD_XCD_W 32
#endif
__device__ __forceinline__ void pixel_of(const FwdArgs &A, int &ai, int &a, int &b) {
    int bid = blockIdx.x;
#if CT_FWD_XCD_W > 1
    {
        // workgroups are dealt to the 8 XCDs in turn: give each XCD CT_FWD_XCD_W consecutive blocks
        // (neighbouring pixels and angles, whose rays cross the same voxels) out of every 8 * CT_FWD_XCD_W
        constexpr int W = CT_FWD_XCD_W, C = 8 * W;
        const int full = (int)(gridDim.x / C) * C;
        if (bid < full) bid = (bid / C) * C + (bid % 8) * W + (bid % C) / 8;
    }
#endif
    const int ub = bid % A.ublocks;
    const int rest = bid / A.ublocks;
    ai = rest % A.nang;
    const int vb = rest / A.nang;
    a = ub * FWD_TU + (threadIdx.x & (FWD_TU - 1));
    b = vb * FWD_TV + (threadIdx.x / FWD_TU);
}

// Memory view of the volume: offset = (z - mem_lo) * sz + y * sy + x * sx.  Blocks whose rays run
// mostly along x read a transposed copy (y fastest), so that the 64 lanes of a wave, which hold 64
// adjacent pixels of a detector row (neighbouring rays displaced along e_u), read neighbouring
// addresses; blocks whose rays run mostly along y read the natural layout.
// Volumes below 4 GiB are read with buffer loads and 32-bit byte offsets (no 64-bit address
// arithmetic per gather); larger ones with 64-bit element offsets.
template <typename TV, bool BUF>
struct View;

template <typename TV>
struct View<TV, true> {
    using Off = int;
    static constexpr bool guarded = false;
    __amdgpu_buffer_rsrc_t r;
    int sx, sy, sz;  // bytes
    __device__ __forceinline__ float operator()(int off) const { return bload(r, off, (TV *)nullptr); }
};

template <typename TV>
struct View<TV, false> {
    using Off = int64_t;
    static constexpr bool guarded = true;
    const TV *p;
    int64_t sx, sy, sz;  // elements
    __device__ __forceinline__ float operator()(int64_t off) const { return ldf(p, off); }
};

template <typename TV, bool BUF>
__device__ __forceinline__ View<TV, BUF> pick_view(const TV *vol, const TV *volT, const FwdArgs &A, const AngleGeo &G) {
    View<TV, BUF> v;
    const bool along_x = volT != nullptr && fabs(G.Dc[0]) > fabs(G.Dc[1]);
    const TV *base = along_x ? volT : vol;
    using Off = typename View<TV, BUF>::Off;
    const Off unit = BUF ? (Off)sizeof(TV) : (Off)1;
    v.sx = along_x ? (Off)A.ny * unit : unit;
    v.sy = along_x ? unit : (Off)A.nx * unit;
    v.sz = (Off)A.nx * (Off)A.ny * unit;
    if constexpr (BUF) {
        v.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<TV *>(base), (short)0,
                                                (int)((int64_t)A.nx * A.ny * A.mem_n * (int64_t)sizeof(TV)), BUF_WORD3);
    } else {
        v.p = base;
    }
    return v;
}

// ------------------------------------------------------------------------------------------
// Siddon: exact length of the ray inside each voxel it crosses (incremental traversal in the
// manner of Jacobs et al. 1998: step to whichever voxel plane comes next).
//
// The step is branch-free: every axis whose next crossing equals the current minimum steps (a ray
// through an edge or corner steps several axes at once, which is Siddon's zero-length piece).
// The traversal stops at Te, the smaller of the clip exit and, per axis, the FP32 time of the
// crossing that would leave the owned grid -- computed by the same expression the loop uses -- so
// voxel indices never leave the grid and need no per-step checks.  Pieces are produced BATCH at a
// time and their gathers issued together, so several loads per lane are in flight.

#ifndef CT_SID_BATCH
#define CT_SID_BATCH 8
#endif
#ifndef CT_INT_BATCH
#define CT_INT_BATCH 8
#endif
constexpr int SID_BATCH = CT_SID_BATCH;  // Siddon pieces per trip
constexpr int INT_BATCH = CT_INT_BATCH;  // interpolation samples per trip

template <typename VIEW>
__device__ __forceinline__ float siddon_ray(const VIEW V, const FwdArgs &A, const AngleGeo &G, int a, int b) {
    using IDX = typename VIEW::Off;
    const double lo[3] = {-0.5, -0.5, A.own_lo - 0.5};
    const double hi[3] = {A.nx - 0.5, A.ny - 0.5, A.own_hi - 0.5};
    RaySetup R;
    if (!ray_clip(G, A, a, b, lo, hi, R)) return 0.0f;

    const int ilo[3] = {0, 0, A.own_lo};
    const int ihi[3] = {A.nx - 1, A.ny - 1, A.own_hi - 1};
    int idx[3];
    float tn0[3], dtn[3], st[3];
    float Te = (float)(R.t1 - R.t0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double E = G.S[ax] + R.t0 * R.D[ax];
        int i = (int)floor(E + 0.5);
        i = i < ilo[ax] ? ilo[ax] : (i > ihi[ax] ? ihi[ax] : i);
        idx[ax] = i;
        if (R.par[ax]) {
            st[ax] = 0.0f;
            tn0[ax] = FLT_MAX;
            dtn[ax] = 0.0f;
        } else {
            const double f = E - i;  // entry offset from the voxel centre, about [-0.5, 0.5]
            const int s = R.D[ax] > 0 ? 1 : -1;
            const double inv = 1.0 / fabs(R.D[ax]);
            st[ax] = (float)s;
            tn0[ax] = (float)((0.5 - s * f) * inv);
            dtn[ax] = (float)inv;
            const int nexit = s > 0 ? ihi[ax] - i : i - ilo[ax];
            Te = fminf(Te, fmaf((float)nexit, dtn[ax], tn0[ax]));
        }
    }
    const IDX s0 = (IDX)(int)st[0] * V.sx, s1 = (IDX)(int)st[1] * V.sy, s2 = (IDX)(int)st[2] * V.sz;
    IDX lin = (IDX)(idx[2] - A.mem_lo) * V.sz + (IDX)idx[1] * V.sy + (IDX)idx[0] * V.sx;
    float tx = tn0[0], ty = tn0[1], tz = tn0[2];
    float n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
    float tc = 0.0f, acc = 0.0f;
    const int maxtrips = (A.nx + A.ny + (A.own_hi - A.own_lo) + 3) / SID_BATCH + 2;
    for (int trip = 0; trip < maxtrips; ++trip) {
        float len[SID_BATCH];
        IDX off[SID_BATCH];
#pragma unroll
        for (int u = 0; u < SID_BATCH; ++u) {
            const float tn = fminf(fminf(fminf(tx, ty), tz), Te);
            len[u] = tn - tc;
            off[u] = lin;
            // Before Te every step stays inside the grid.  At Te the 64-bit path must not step
            // (an index past the grid would be read); the buffer path may, since reads past the
            // resource return 0 and every later piece has zero length.
            const bool act = VIEW::guarded ? tn < Te : true;
            const bool cx = act && tx == tn, cy = act && ty == tn, cz = act && tz == tn;
            lin += (cx ? s0 : (IDX)0) + (cy ? s1 : (IDX)0) + (cz ? s2 : (IDX)0);
            n0 += cx ? 1.0f : 0.0f;
            n1 += cy ? 1.0f : 0.0f;
            n2 += cz ? 1.0f : 0.0f;
            tx = fmaf(n0, dtn[0], tn0[0]);
            ty = fmaf(n1, dtn[1], tn0[1]);
            tz = fmaf(n2, dtn[2], tn0[2]);
            tc = tn;
        }
        float v[SID_BATCH];
#pragma unroll
        for (int u = 0; u < SID_BATCH; ++u) v[u] = V(off[u]);
#pragma unroll
        for (int u = 0; u < SID_BATCH; ++u) acc = fmaf(len[u], v[u], acc);
        if (!(tc < Te)) break;
    }
    return (float)(acc * R.L);
}

template <typename TV, typename TP, bool BUF>
__global__ __launch_bounds__(FWD_TU * FWD_TV) void k_siddon(const TV *__restrict__ vol, const TV *__restrict__ volT,
                                                TP *__restrict__ proj, FwdArgs A) {
    int ai, a, b;
    pixel_of(A, ai, a, b);
    if (a >= A.nu || b >= A.nv) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    const float v = siddon_ray(pick_view<TV, BUF>(vol, volT, A, G), A, G, a, b);
    const int64_t o = ((int64_t)ai * A.nv + b) * A.nu + a;
    const float prev = A.accumulate ? to_f(proj[o]) : 0.0f;
    proj[o] = from_f<TP>(prev + v);
}

// ------------------------------------------------------------------------------------------
// Column Siddon (resident volumes).
//
// A detector column and the source span a vertical plane, so every row of that column follows the
// same xy line S + t D_xy and crosses the x and y planes at the same t.  A wave takes one column
// and 64 * ROWS of its rows (lane = row): it walks the shared xy path with wave-uniform state and
// every lane splits each xy piece at its own z crossing.  While |Dz| < max(|Dx|, |Dy|) (index
// units) an xy piece climbs less than one slice, so it holds at most one z crossing and meets two
// consecutive voxels of one column.  The volume is read from a column-major copy ([y][x][z] with a
// zero slot below and above each column), where those two voxels are one 8-byte load (4-byte for
// 16-bit storage) and the lanes, holding consecutive rows, read consecutive addresses.  Rows
// outside the grid in z clamp to the zero slots, so no per-row clipping is needed.
//
// Per row the z coordinate is kept relative to the slot of its entry point (z = Zr + t Dz with
// Zr in [0, 1)), so the crossing time (lo + 1 - Zr) / Dz is one FMA without cancellation.

#ifndef CT_ZC_COLS
#define CT_ZC_COLS 4
#endif
#ifndef CT_ZC_ORDER
#define CT_ZC_ORDER 3
#endif
#ifndef CT_ZC_AK
#define CT_ZC_AK 32
#endif
#ifndef CT_ZC_XCD_W
#define CT_ZC_XCD_W 4
#endif
constexpr int ZC_COLS = CT_ZC_COLS;  // columns (waves) per block

template <typename TV>
struct ZPair;
template <>
struct ZPair<float> {
    static __device__ __forceinline__ void ld(const float *col, uint32_t k, float &a, float &b) {
        float2 v;
        __builtin_memcpy(&v, col + k, sizeof(v));
        a = v.x;
        b = v.y;
    }
};
template <>
struct ZPair<f16s> {
    static __device__ __forceinline__ void ld(const f16s *col, uint32_t k, float &a, float &b) {
        uint32_t w;
        __builtin_memcpy(&w, col + k, sizeof(w));
        a = (float)__builtin_bit_cast(f16s, (uint16_t)(w & 0xffffu));
        b = (float)__builtin_bit_cast(f16s, (uint16_t)(w >> 16));
    }
};
template <>
struct ZPair<bf16s> {
    static __device__ __forceinline__ void ld(const bf16s *col, uint32_t k, float &a, float &b) {
        uint32_t w;
        __builtin_memcpy(&w, col + k, sizeof(w));
        a = __uint_as_float(w << 16);
        b = __uint_as_float(w & 0xffff0000u);
    }
};

// Four taps of an x-paired copy: (x, z), (x + 1, z), (x, z + 1), (x + 1, z + 1) in one load
// (16 bytes for FP32, 8 for the 16-bit types; 4- or 8-byte aligned, which global loads allow).
template <typename TV>
struct XQuad;
template <>
struct XQuad<float> {
    static __device__ __forceinline__ void ld(const float *p, float &a, float &b, float &c, float &d) {
        float4 v;
        __builtin_memcpy(&v, p, sizeof(v));
        a = v.x;
        b = v.y;
        c = v.z;
        d = v.w;
    }
};
template <>
struct XQuad<f16s> {
    static __device__ __forceinline__ void ld(const f16s *p, float &a, float &b, float &c, float &d) {
        uint2 w;
        __builtin_memcpy(&w, p, sizeof(w));
        a = (float)__builtin_bit_cast(f16s, (uint16_t)(w.x & 0xffffu));
        b = (float)__builtin_bit_cast(f16s, (uint16_t)(w.x >> 16));
        c = (float)__builtin_bit_cast(f16s, (uint16_t)(w.y & 0xffffu));
        d = (float)__builtin_bit_cast(f16s, (uint16_t)(w.y >> 16));
    }
};
template <>
struct XQuad<bf16s> {
    static __device__ __forceinline__ void ld(const bf16s *p, float &a, float &b, float &c, float &d) {
        uint2 w;
        __builtin_memcpy(&w, p, sizeof(w));
        a = __uint_as_float(w.x << 16);
        b = __uint_as_float(w.x & 0xffff0000u);
        c = __uint_as_float(w.y << 16);
        d = __uint_as_float(w.y & 0xffff0000u);
    }
};

#ifndef CT_ZC_BATCH
#define CT_ZC_BATCH 8
#endif
constexpr int ZC_B = CT_ZC_BATCH;  // xy pieces per trip

// Per-row state of the column walk.
template <int ROWS>
struct ZRows {
    float Zr[ROWS];    // z at the xy entry, relative to slot k0 (in [0, 1))
    float Dz[ROWS];    // dz/dt (index units)
    float inv[ROWS];   // 1 / Dz (0 for rows parallel to the xy plane)
    float c1[ROWS];    // (1 - Zr) / Dz, or +-FLT_MAX for parallel rows
    float lmin[ROWS];  // pair slots are clamped to [lmin, lmax] (relative to k0)
    float lmax[ROWS];
    uint32_t kb[ROWS]; // byte offset of slot k0 in a column
    bool up[ROWS];     // Dz >= 0
};

// ORI: +1 all rows of the wave rise, -1 all fall, 0 mixed.  The xy walk (tx, ty, lin, ...) is the
// same in every lane.
template <int ORI, int ROWS, typename TV>
__device__ __forceinline__ void zc_walk(const TV *__restrict__ vz, int64_t lin, const int64_t sX, const int64_t sY,
                                        const float tx0, const float ty0, const float dtx, const float dty,
                                        const float Te, const ZRows<ROWS> &Z, float (&acc)[ROWS], const int maxtrips) {
    float fz[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) fz[r] = floorf(Z.Zr[r]);
    float tx = tx0, ty = ty0, nxc = 0.0f, nyc = 0.0f, tp = 0.0f;
    for (int trip = 0; trip < maxtrips; ++trip) {
        float ta[ZC_B], tb[ZC_B];
        int64_t ln[ZC_B];
#pragma unroll
        for (int u = 0; u < ZC_B; ++u) {
            const float tn = fminf(fminf(tx, ty), Te);
            ta[u] = tp;
            tb[u] = tn;
            ln[u] = lin;
            // at Te the walk stops: the column index never leaves the grid
            const bool act = tn < Te;
            const bool cx = act && tx == tn, cy = act && ty == tn;
            lin += (cx ? sX : (int64_t)0) + (cy ? sY : (int64_t)0);
            nxc += cx ? 1.0f : 0.0f;
            nyc += cy ? 1.0f : 0.0f;
            tx = fmaf(nxc, dtx, tx0);
            ty = fmaf(nyc, dty, ty0);
            tp = tn;
        }
        float w1[ZC_B][ROWS], w2[ZC_B][ROWS], va[ZC_B][ROWS], vb[ZC_B][ROWS];
#pragma unroll
        for (int u = 0; u < ZC_B; ++u) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const float fb = floorf(fmaf(tb[u], Z.Dz[r], Z.Zr[r]));
                float lo = ORI > 0 ? fz[r] : (ORI < 0 ? fb : fminf(fz[r], fb));
                lo = __builtin_amdgcn_fmed3f(lo, Z.lmin[r], Z.lmax[r]);
                fz[r] = fb;
                // the piece [ta, tb] meets slot lo on one side of tc and slot lo+1 on the other
                const float m = __builtin_amdgcn_fmed3f(fmaf(lo, Z.inv[r], Z.c1[r]), ta[u], tb[u]);
                w1[u][r] = m - ta[u];
                w2[u][r] = tb[u] - m;
                const uint32_t k = (uint32_t)((int)lo * (int)sizeof(TV)) + Z.kb[r];
                ZPair<TV>::ld((const TV *)((const char *)(vz + ln[u]) + k), 0u, va[u][r], vb[u][r]);
            }
        }
#pragma unroll
        for (int u = 0; u < ZC_B; ++u) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                // rising rows meet lo first, falling rows lo+1 first
                float first, second;
                if constexpr (ORI > 0) {
                    first = va[u][r];
                    second = vb[u][r];
                } else if constexpr (ORI < 0) {
                    first = vb[u][r];
                    second = va[u][r];
                } else {
                    first = Z.up[r] ? va[u][r] : vb[u][r];
                    second = Z.up[r] ? vb[u][r] : va[u][r];
                }
                acc[r] = fmaf(w1[u][r], first, acc[r]);
                acc[r] = fmaf(w2[u][r], second, acc[r]);
            }
        }
        if (!(tp < Te)) break;
    }
}


template <typename TV, typename TP, int ROWS>
__global__ __launch_bounds__(64 * ZC_COLS) void k_siddon_col(const TV *__restrict__ vz, TP *__restrict__ proj,
                                                             FwdArgs A) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    int bid = blockIdx.x;
#if CT_ZC_XCD_W > 1
    // workgroups are dealt to the 8 XCDs in turn: give each XCD CT_ZC_XCD_W consecutive column
    // groups out of every 8 * CT_ZC_XCD_W, so rays that share voxels share an L2
    {
        constexpr int W = CT_ZC_XCD_W, C = 8 * W;
        const int full = (int)(gridDim.x / C) * C;
        if (bid < full) bid = (bid / C) * C + (bid % 8) * W + (bid % C) / 8;
    }
#endif
    int cb, ai, rg;
#if CT_ZC_ORDER == 1
    ai = bid % A.nang;
    cb = (bid / A.nang) % A.cblocks;
    rg = bid / A.nang / A.cblocks;
#elif CT_ZC_ORDER == 2
    cb = bid % A.cblocks;
    rg = (bid / A.cblocks) % A.rgroups;
    ai = bid / A.cblocks / A.rgroups;
#elif CT_ZC_ORDER == 3
    {
        // groups of CT_ZC_AK consecutive angles: angle within the group fastest, then column block
        constexpr int AK = CT_ZC_AK;
        const int per = A.nang * A.cblocks, idx = bid % per, full = A.nang / AK;
        rg = bid / per;
        if (idx < full * AK * A.cblocks) {
            const int r = idx % (AK * A.cblocks);
            cb = r / AK;
            ai = (idx / (AK * A.cblocks)) * AK + r % AK;
        } else {
            const int rem = A.nang - full * AK, i2 = idx - full * AK * A.cblocks;
            cb = i2 / rem;
            ai = full * AK + i2 % rem;
        }
    }
#else
    cb = bid % A.cblocks;
    ai = (bid / A.cblocks) % A.nang;
    rg = bid / A.cblocks / A.nang;
#endif
    const int a = cb * ZC_COLS + wave;
    if (a >= A.nu) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    // the copy holds slices [mem_lo, mem_lo + mem_n) of the volume (all of it when resident)
    const int nzc = A.mem_n;
    const int64_t nzp = (int64_t)nzc + 2;

    // shared xy line of the column, clipped to the grid's xy box (FP64)
    const double ua = (a - A.cu) * A.du + A.offu;
    const double D[2] = {G.Dc[0] + ua * G.eu[0], G.Dc[1] + ua * G.eu[1]};
    const double mx = D[0] * A.dx, my = D[1] * A.dy;
    const double Lxy2 = mx * mx + my * my;
    const double Lref = sqrt(Lxy2);
    const double lo2[2] = {-0.5, -0.5}, hi2[2] = {A.nx - 0.5, A.ny - 0.5};
    bool par[2];
    double t0 = 0.0, t1 = 1.0;
    bool hit = true;
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        par[ax] = fabs(ax == 0 ? mx : my) < 1e-12 * Lref;
        if (par[ax]) {
            if (G.S[ax] < lo2[ax] || G.S[ax] > hi2[ax]) hit = false;
        } else {
            const double ta = (lo2[ax] - G.S[ax]) / D[ax];
            const double tb = (hi2[ax] - G.S[ax]) / D[ax];
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        }
    }
    hit = hit && t0 < t1;

    float acc[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = 0.0f;
    const int brow = rg * (64 * ROWS) + lane;
    double L[ROWS];
    ZRows<ROWS> Z;
    bool all_up = true, all_down = true;
    // the wave walks only where one of its rows is inside the owned slices: [t0, t1] shrinks to
    // the hull of the rows' own intervals (outside them every row reads zero slots anyway)
    {
        const double zlo = A.own_lo - 0.5, zhi = A.own_hi - 0.5;
        double win0 = 1e300, win1 = -1e300;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int b = min(brow + 64 * r, A.nv - 1);
            const double Dz = ((b - A.cv) * A.dv + A.offv) / A.dz;
            if (fabs(Dz * A.dz) < 1e-12 * Lref) {
                if (G.S[2] >= zlo && G.S[2] <= zhi) {
                    win0 = fmin(win0, t0);
                    win1 = fmax(win1, t1);
                }
            } else {
                const double ta = (zlo - G.S[2]) / Dz, tb = (zhi - G.S[2]) / Dz;
                win0 = fmin(win0, fmin(ta, tb));
                win1 = fmax(win1, fmax(ta, tb));
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            win0 = fmin(win0, __shfl_xor(win0, off, 64));
            win1 = fmax(win1, __shfl_xor(win1, off, 64));
        }
        t0 = fmax(t0, win0 - 1e-9);
        t1 = fmin(t1, win1 + 1e-9);
        hit = hit && t0 < t1;
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        // lanes past the last row repeat its geometry (their results are not stored)
        const int b = min(brow + 64 * r, A.nv - 1);
        const double vbm = (b - A.cv) * A.dv + A.offv;
        const double Dz = vbm / A.dz;
        const double mz = Dz * A.dz;
        L[r] = sqrt(Lxy2 + mz * mz);
        // slot coordinate: voxel mem_lo + k spans [k + 1, k + 2)
        const double ze = G.S[2] - A.mem_lo + t0 * Dz + 1.5;
        const double k0 = floor(ze);
        const double zr = ze - k0;
        const bool parz = fabs(mz) < 1e-12 * L[r];
        Z.Zr[r] = (float)zr;
        Z.Dz[r] = parz ? 0.0f : (float)Dz;
        Z.up[r] = parz || Dz > 0.0;
        // |k0| < 2^22 (checked on the host), so these are exact in FP32; the slot k0 + lo is in
        // [0, nz], and the byte offset is formed modulo 2^32
        const float lmin = (float)(-k0), lmax = (float)((double)nzc - k0);
        Z.lmin[r] = lmin;
        Z.lmax[r] = lmax;
        Z.kb[r] = (uint32_t)((int64_t)k0 * (int64_t)sizeof(TV));
        if (parz) {
            // constant z: the crossing of the plane above the clamped slot is in the future
            // (+inf) unless the clamp moved the slot below the row
            const float lo = fminf(fmaxf(floorf((float)zr), lmin), lmax);
            Z.inv[r] = 0.0f;
            Z.c1[r] = (lo + 1.0f > (float)zr) ? FLT_MAX : -FLT_MAX;
        } else {
            Z.inv[r] = (float)(1.0 / Dz);
            Z.c1[r] = (float)((1.0 - zr) / Dz);
        }
        all_up = all_up && Z.up[r];
        all_down = all_down && !Z.up[r];
    }

    if (hit) {
        int idx[2];
        float tn0[2], dtn[2];
        int sg[2];
        float Te = (float)(t1 - t0);
        const int ihi[2] = {A.nx - 1, A.ny - 1};
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const double E = G.S[ax] + t0 * D[ax];
            int i = (int)floor(E + 0.5);
            i = i < 0 ? 0 : (i > ihi[ax] ? ihi[ax] : i);
            idx[ax] = i;
            if (par[ax]) {
                sg[ax] = 0;
                tn0[ax] = FLT_MAX;
                dtn[ax] = 0.0f;
            } else {
                const double f = E - i;
                const int s = D[ax] > 0 ? 1 : -1;
                const double inv = 1.0 / fabs(D[ax]);
                sg[ax] = s;
                tn0[ax] = (float)((0.5 - s * f) * inv);
                dtn[ax] = (float)inv;
                const int nexit = s > 0 ? ihi[ax] - i : i;
                Te = fminf(Te, fmaf((float)nexit, dtn[ax], tn0[ax]));
            }
        }
        const int64_t sX = (int64_t)sg[0] * nzp, sY = (int64_t)sg[1] * A.nx * nzp;
        const int64_t lin = ((int64_t)idx[1] * A.nx + idx[0]) * nzp;
        const int maxtrips = (A.nx + A.ny + 2) / ZC_B + 2;
        all_up = __all(all_up);
        all_down = __all(all_down);
        if (all_up)
            zc_walk<1>(vz, lin, sX, sY, tn0[0], tn0[1], dtn[0], dtn[1], Te, Z, acc, maxtrips);
        else if (all_down)
            zc_walk<-1>(vz, lin, sX, sY, tn0[0], tn0[1], dtn[0], dtn[1], Te, Z, acc, maxtrips);
        else
            zc_walk<0>(vz, lin, sX, sY, tn0[0], tn0[1], dtn[0], dtn[1], Te, Z, acc, maxtrips);
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int b = brow + 64 * r;
        if (b >= A.nv) continue;
        const int64_t o = ((int64_t)ai * A.nv + b) * A.nu + a;
        const float prev = A.accumulate ? to_f(proj[o]) : 0.0f;
        proj[o] = from_f<TP>(prev + (float)(acc[r] * L[r]));
    }
}

// [z][y][x] -> column-major slots: slices [0, nz) of src go to slots slot0 + z of columns of nzp
// slots ([y][x][slot]); pads: bit 0 zeroes slot 0, bit 1 zeroes slot nzp - 1.  32 x 32 (z, x) tiles.
// Values pass through FP32 (exact for the storage types), so the copy may also change the type.
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_zcols(const TS *__restrict__ src, TD *__restrict__ dst, int nx, int ny, int nz,
                                               int64_t nzp, int slot0, int pads) {
    __shared__ float tile[32][33];
    const int x0 = blockIdx.x * 32, z0 = blockIdx.y * 32, y = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int x = x0 + tx, z = z0 + ty + r;
        if (x < nx && z < nz) tile[ty + r][tx] = to_f(src[((int64_t)z * ny + y) * nx + x]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int z = z0 + tx, x = x0 + ty + r;
        if (x < nx && z < nz) dst[((int64_t)y * nx + x) * nzp + slot0 + z] = from_f<TD>(tile[tx][ty + r]);
    }
    if (threadIdx.x < 32) {
        const int x = x0 + threadIdx.x;
        if (x < nx) {
            const int64_t c = ((int64_t)y * nx + x) * nzp;
            if ((pads & 1) && blockIdx.y == 0) dst[c] = from_f<TD>(0.0f);
            if ((pads & 2) && blockIdx.y == gridDim.y - 1) dst[c + nzp - 1] = from_f<TD>(0.0f);
        }
    }
}

// column-major slots -> [z][y][x]: slots slot0 .. slot0 + nz - 1 of columns of nzp slots go to
// slices 0 .. nz - 1 of dst
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_zcols_inv(const TS *__restrict__ src, TD *__restrict__ dst, int nx, int ny, int nz,
                                                   int64_t nzp, int slot0) {
    __shared__ float tile[32][33];
    const int x0 = blockIdx.x * 32, z0 = blockIdx.y * 32, y = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int z = z0 + tx, x = x0 + ty + r;
        if (x < nx && z < nz) tile[ty + r][tx] = to_f(src[((int64_t)y * nx + x) * nzp + slot0 + z]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int x = x0 + tx, z = z0 + ty + r;
        if (x < nx && z < nz) dst[((int64_t)z * ny + y) * nx + x] = from_f<TD>(tile[tx][ty + r]);
    }
}

// ------------------------------------------------------------------------------------------
// Interpolated projector over a zero-padded column-major copy (resident volumes).
//
// The copy holds voxel (x, y, z) at ((y + 1) PX + x + 1) PZ + z + 1 with PX = nx + 3, PY = ny + 3,
// PZ = nz + 3 and zeros elsewhere, so every tap of a sample inside the grid box grown by one voxel
// is in range and the zero padding of the interpolant needs no tests.  A wave takes one detector
// column and 64 * ROWS of its rows (lane = row): the rows share the xy line, and at the same
// sample index their sample points stay within about a voxel of each other in xy, so the four
// (x, y) tap columns of a sample are mostly common to the wave and each holds the two z taps of
// every lane in one 8-byte load at consecutive addresses.

template <typename TV>
__global__ __launch_bounds__(256) void k_pcols(const TV *__restrict__ src, TV *__restrict__ dst, int nx, int ny, int nz) {
    // one thread per padded (slot, column): tiles of 32 slots x 32 padded x for one padded y
    __shared__ TV tile[32][33];
    const int PX = nx + 3, PZ = nz + 3;
    const int xp0 = blockIdx.x * 32, zp0 = blockIdx.y * 32, yp = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int y = yp - 1;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int x = xp0 + tx - 1, z = zp0 + ty + r - 1;
        TV v = from_f<TV>(0.0f);
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) v = src[((int64_t)z * ny + y) * nx + x];
        tile[ty + r][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int zp = zp0 + tx, xp = xp0 + ty + r;
        if (xp < PX && zp < PZ) dst[((int64_t)yp * PX + xp) * PZ + zp] = tile[tx][ty + r];
    }
}

// The same zero-padded copy with x neighbours paired: element 2 (((yp PX + xp) PZ + zp)) + e holds
// the padded voxel (xp + e - 1, yp - 1, zp - 1), so one load brings the two z taps of two x
// neighbours (twice the memory of k_pcols' copy, half the loads per sample).
template <typename TV>
__global__ __launch_bounds__(256) void k_pcols2(const TV *__restrict__ src, TV *__restrict__ dst, int nx, int ny,
                                                int nz) {
    __shared__ TV tile[32][34];
    const int PX = nx + 3, PZ = nz + 3;
    const int xp0 = blockIdx.x * 32, zp0 = blockIdx.y * 32, yp = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int y = yp - 1;
    // tile[z][x] for padded x in [xp0, xp0 + 33) and padded z in [zp0, zp0 + 32)
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int z = zp0 + ty + r - 1;
        for (int c = tx; c < 33; c += 32) {
            const int x = xp0 + c - 1;
            TV v = from_f<TV>(0.0f);
            if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) v = src[((int64_t)z * ny + y) * nx + x];
            tile[ty + r][c] = v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int zp = zp0 + tx, xp = xp0 + ty + r;
        if (xp < PX && zp < PZ) {
            const int64_t o = (((int64_t)yp * PX + xp) * PZ + zp) * 2;
            dst[o] = tile[tx][ty + r];
            dst[o + 1] = tile[tx][ty + r + 1];
        }
    }
}

// Samples per trip (IC_B): a lane issues the loads of IC_B samples before using them.  One sample
// per trip suits detector columns whose rows share a vertical plane (circular and helical scans: a
// wave's lanes change cells together, 101 ms at 512^3 / 360 against 104 with two and 135 with four);
// four suit tilted columns, whose rows drift apart (168 ms for a C-arm scan against 183 with one).
#ifndef CT_IC_BATCH_V
#define CT_IC_BATCH_V 1
#endif
#ifndef CT_IC_BATCH_T
#define CT_IC_BATCH_T 4
#endif

template <typename TV, typename TP, int ROWS, bool XP, int IC_B>
__global__ __launch_bounds__(64 * ZC_COLS) void k_interp_col(const TV *__restrict__ vp, TP *__restrict__ proj,
                                                             FwdArgs A) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    int bid = blockIdx.x;
#if CT_ZC_XCD_W > 1
    {
        constexpr int W = CT_ZC_XCD_W, C = 8 * W;
        const int full = (int)(gridDim.x / C) * C;
        if (bid < full) bid = (bid / C) * C + (bid % 8) * W + (bid % C) / 8;
    }
#endif
    const int cb = bid % A.cblocks;
    const int rest = bid / A.cblocks;
    const int ai = rest % A.nang;
    const int rg = rest / A.nang;
    const int a = cb * ZC_COLS + wave;
    if (a >= A.nu) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    const int64_t PX = A.nx + 3, PZ = A.nz + 3;
    const double lo[3] = {-1.0, -1.0, -1.0};
    const double hi[3] = {(double)A.nx, (double)A.ny, (double)A.nz};
    // per row: samples k0 .. k0 + n - 1, sample j at fb + j fs relative to voxel ib
    int ib[ROWS][3], nsm[ROWS];
    float fb[ROWS][3], fs[ROWS][3];
    int nmax = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int b = min(rg * (64 * ROWS) + 64 * r + lane, A.nv - 1);
        RaySetup R;
        nsm[r] = 0;
        ib[r][0] = ib[r][1] = ib[r][2] = 0;
        fb[r][0] = fb[r][1] = fb[r][2] = 0.0f;
        fs[r][0] = fs[r][1] = fs[r][2] = 0.0f;
        if (ray_clip(G, A, a, b, lo, hi, R)) {
            const double s_in = R.t0 * R.L, s_out = R.t1 * R.L;
            const double k0 = ceil(s_in / A.delta - 0.5);
            const double k1 = floor(s_out / A.delta - 0.5);
            if (k1 >= k0) {
                const double tk0 = (k0 + 0.5) * A.delta / R.L;
                const double dt = A.delta / R.L;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const double B = G.S[ax] + tk0 * R.D[ax];
                    ib[r][ax] = (int)floor(B);
                    fb[r][ax] = (float)(B - ib[r][ax]);
                    fs[r][ax] = (float)(dt * R.D[ax]);
                }
                nsm[r] = (int)(k1 - k0) + 1;
            }
        }
        nmax = max(nmax, nsm[r]);
    }
    // lanes stop together: the wave runs to its longest row, shorter rows add zero
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) nmax = max(nmax, __shfl_xor(nmax, off, 64));
    float acc[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = 0.0f;
    const int64_t cy = PX * PZ;
    const float xhi = (float)A.nx, yhi = (float)A.ny, zhi = (float)A.nz;
#ifndef CT_IC_NO_REUSE
    constexpr bool REUSE = XP;
#else
    constexpr bool REUSE = false;
#endif
    // the previous sample's cell and taps: samples half a voxel apart share a cell about half the
    // time, and a lane that stays in its cell loads nothing
    int64_t cprev[ROWS];
    float vprev[ROWS][8];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        cprev[r] = -1;
#pragma unroll
        for (int i = 0; i < 8; ++i) vprev[r][i] = 0.0f;
    }
    for (int j0 = 0; j0 < nmax; j0 += IC_B) {
        float w[IC_B][ROWS][3], v[IC_B][ROWS][8];
        int64_t cu[IC_B][ROWS];
#pragma unroll
        for (int u = 0; u < IC_B; ++u) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                // rows with fewer samples repeat their last one (and add nothing)
                const int j = max(0, min(j0 + u, nsm[r] - 1));
                const float px = fmaf((float)j, fs[r][0], fb[r][0]);
                const float py = fmaf((float)j, fs[r][1], fb[r][1]);
                const float pz = fmaf((float)j, fs[r][2], fb[r][2]);
                const float flx = floorf(px), fly = floorf(py), flz = floorf(pz);
                w[u][r][0] = px - flx;
                w[u][r][1] = py - fly;
                w[u][r][2] = pz - flz;
                // tap (x0, y0, z0) with each index kept in [-1, n] (samples lie in the box grown by
                // one voxel up to rounding), so all eight taps are inside the padded copy
                const int x0 = (int)__builtin_amdgcn_fmed3f(flx + (float)ib[r][0], -1.0f, xhi);
                const int y0 = (int)__builtin_amdgcn_fmed3f(fly + (float)ib[r][1], -1.0f, yhi);
                const int z0 = (int)__builtin_amdgcn_fmed3f(flz + (float)ib[r][2], -1.0f, zhi);
                const int64_t c = nsm[r] > 0 ? ((int64_t)(y0 + 1) * PX + (x0 + 1)) * PZ + (z0 + 1) : 0;
                cu[u][r] = c;
                if constexpr (REUSE) {
                    const int64_t cp = u == 0 ? cprev[r] : cu[u - 1][r];
                    if (c != cp) {
                        const TV *q = vp + 2 * c;
                        XQuad<TV>::ld(q, v[u][r][0], v[u][r][2], v[u][r][1], v[u][r][3]);
                        XQuad<TV>::ld(q + 2 * cy, v[u][r][4], v[u][r][6], v[u][r][5], v[u][r][7]);
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) v[u][r][i] = u == 0 ? vprev[r][i] : v[u - 1][r][i];
                    }
                } else if constexpr (XP) {
                    // (x0, z0), (x0 + 1, z0), (x0, z0 + 1), (x0 + 1, z0 + 1) of rows y0 and y0 + 1
                    const TV *q = vp + 2 * c;
                    XQuad<TV>::ld(q, v[u][r][0], v[u][r][2], v[u][r][1], v[u][r][3]);
                    XQuad<TV>::ld(q + 2 * cy, v[u][r][4], v[u][r][6], v[u][r][5], v[u][r][7]);
                } else {
                    const TV *q = vp + c;
                    ZPair<TV>::ld(q, 0u, v[u][r][0], v[u][r][1]);
                    ZPair<TV>::ld(q + PZ, 0u, v[u][r][2], v[u][r][3]);
                    ZPair<TV>::ld(q + cy, 0u, v[u][r][4], v[u][r][5]);
                    ZPair<TV>::ld(q + cy + PZ, 0u, v[u][r][6], v[u][r][7]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < IC_B; ++u) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const float *q = v[u][r];
                const float rx = w[u][r][0], ry = w[u][r][1], rz = w[u][r][2];
                // z lerps of the columns (x0, y0), (x0 + 1, y0), (x0, y0 + 1), (x0 + 1, y0 + 1)
                const float c00 = fmaf(rz, q[1] - q[0], q[0]), c10 = fmaf(rz, q[3] - q[2], q[2]);
                const float c01 = fmaf(rz, q[5] - q[4], q[4]), c11 = fmaf(rz, q[7] - q[6], q[6]);
                const float c0 = fmaf(rx, c10 - c00, c00), c1 = fmaf(rx, c11 - c01, c01);
                const float val = fmaf(ry, c1 - c0, c0);
                acc[r] += (j0 + u < nsm[r]) ? val : 0.0f;
            }
        }
        if constexpr (REUSE) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                cprev[r] = cu[IC_B - 1][r];
#pragma unroll
                for (int i = 0; i < 8; ++i) vprev[r][i] = v[IC_B - 1][r][i];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int b = rg * (64 * ROWS) + 64 * r + lane;
        if (b >= A.nv) continue;
        const int64_t o = ((int64_t)ai * A.nv + b) * A.nu + a;
        const float prev = A.accumulate ? to_f(proj[o]) : 0.0f;
        proj[o] = from_f<TP>(prev + (float)(acc[r] * A.delta));
    }
}

// ------------------------------------------------------------------------------------------
// Interpolated projector: samples at s_k = (k + 1/2) delta mm from the source, every k whose
// sample lies in the grid box grown by half a voxel (outside it the zero-padded trilinear
// interpolant vanishes); p = delta * sum of the interpolant at the samples.  All rays of a wave
// reach sample j at the same distance from the source, so the lanes stay in step through the
// volume and the eight taps of a wave fall on a few cache lines.

template <typename VIEW>
__device__ __forceinline__ float interp_ray(const VIEW V, const FwdArgs &A, const AngleGeo &G, int a, int b) {
    using IDX = typename VIEW::Off;
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
            // sample index where z meets each owned boundary; an open end (first or last slab)
            // lies at -inf / +inf in z, which is -inf or +inf in j depending on the z direction
            const double up = stp[2] > 0.0 ? 1.0 : -1.0;
            const double ja = A.first ? -up * 1e30 : (A.own_lo - 0.5 - B[2]) / stp[2];
            const double jb = A.last ? up * 1e30 : (A.own_hi - 0.5 - B[2]) / stp[2];
            const double j0 = floor(fmin(ja, jb)) - 2, j1 = ceil(fmax(ja, jb)) + 2;
            jlo = (int)fmax((double)jlo, j0);
            jhi = (int)fmin((double)jhi, j1);
        }
    }
    const int zm_hi = A.mem_n - 1;
    float acc = 0.0f;
    // INT_BATCH samples per trip: all their taps are issued before any is used
    for (int j0 = jlo; j0 <= jhi; j0 += INT_BATCH) {
        float wgt[INT_BATCH][6];
        IDX off[INT_BATCH][8];
#pragma unroll
        for (int u = 0; u < INT_BATCH; ++u) {
            const int j = min(j0 + u, jhi);
            const float px = fmaf((float)j, fs[0], fb[0]);
            const float py = fmaf((float)j, fs[1], fb[1]);
            const float pz = fmaf((float)j, fs[2], fb[2]);
            const bool own = (j0 + u <= jhi) && (!slab || (pz >= zlo && pz < zhi));
            const float flx = floorf(px), fly = floorf(py), flz = floorf(pz);
            const float rx = px - flx, ry = py - fly, rz = pz - flz;
            const int x0 = ib[0] + (int)flx, y0 = ib[1] + (int)fly, z0 = ib[2] + (int)flz - A.mem_lo;
            // zero padding: taps outside the grid (or outside the slices in memory) weigh 0
            const bool vx0 = (unsigned)x0 < (unsigned)A.nx, vx1 = (unsigned)(x0 + 1) < (unsigned)A.nx;
            const bool vy0 = (unsigned)y0 < (unsigned)A.ny, vy1 = (unsigned)(y0 + 1) < (unsigned)A.ny;
            const bool vz0 = (unsigned)z0 < (unsigned)A.mem_n, vz1 = (unsigned)(z0 + 1) < (unsigned)A.mem_n;
            const IDX ox0 = (IDX)(vx0 ? x0 : 0) * V.sx, ox1 = (IDX)(vx1 ? x0 + 1 : A.nx - 1) * V.sx;
            const IDX oy0 = (IDX)(vy0 ? y0 : 0) * V.sy, oy1 = (IDX)(vy1 ? y0 + 1 : A.ny - 1) * V.sy;
            const IDX oz0 = (IDX)(vz0 ? z0 : 0) * V.sz, oz1 = (IDX)(vz1 ? z0 + 1 : zm_hi) * V.sz;
            wgt[u][0] = vx0 ? 1.0f - rx : 0.0f;
            wgt[u][1] = vx1 ? rx : 0.0f;
            wgt[u][2] = vy0 ? 1.0f - ry : 0.0f;
            wgt[u][3] = vy1 ? ry : 0.0f;
            wgt[u][4] = (own && vz0) ? 1.0f - rz : 0.0f;
            wgt[u][5] = (own && vz1) ? rz : 0.0f;
            const IDX r00 = oz0 + oy0, r01 = oz0 + oy1, r10 = oz1 + oy0, r11 = oz1 + oy1;
            off[u][0] = r00 + ox0;
            off[u][1] = r00 + ox1;
            off[u][2] = r01 + ox0;
            off[u][3] = r01 + ox1;
            off[u][4] = r10 + ox0;
            off[u][5] = r10 + ox1;
            off[u][6] = r11 + ox0;
            off[u][7] = r11 + ox1;
        }
        float v[INT_BATCH][8];
#pragma unroll
        for (int u = 0; u < INT_BATCH; ++u)
#pragma unroll
            for (int q = 0; q < 8; ++q) v[u][q] = V(off[u][q]);
#pragma unroll
        for (int u = 0; u < INT_BATCH; ++u) {
            const float *w = wgt[u];
            const float c00 = fmaf(w[1], v[u][1], w[0] * v[u][0]), c01 = fmaf(w[1], v[u][3], w[0] * v[u][2]);
            const float c10 = fmaf(w[1], v[u][5], w[0] * v[u][4]), c11 = fmaf(w[1], v[u][7], w[0] * v[u][6]);
            const float c0 = fmaf(w[3], c01, w[2] * c00), c1 = fmaf(w[3], c11, w[2] * c10);
            acc += fmaf(w[5], c1, w[4] * c0);
        }
    }
    return (float)(acc * A.delta);
}

template <typename TV, typename TP, bool BUF>
__global__ __launch_bounds__(FWD_TU * FWD_TV) void k_interp(const TV *__restrict__ vol, const TV *__restrict__ volT,
                                                TP *__restrict__ proj, FwdArgs A) {
    int ai, a, b;
    pixel_of(A, ai, a, b);
    if (a >= A.nu || b >= A.nv) return;
    const AngleGeo &G = A.tab[A.a0 + ai];
    const float v = interp_ray(pick_view<TV, BUF>(vol, volT, A, G), A, G, a, b);
    const int64_t o = ((int64_t)ai * A.nv + b) * A.nu + a;
    const float prev = A.accumulate ? to_f(proj[o]) : 0.0f;
    proj[o] = from_f<TP>(prev + v);
}

// [z][y][x] -> [z][x][y], 32 x 32 tiles through LDS
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_xy(const T *__restrict__ src, T *__restrict__ dst, int nx, int ny) {
    __shared__ T tile[32][33];
    const int64_t zoff = (int64_t)blockIdx.z * nx * ny;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int x = x0 + tx, y = y0 + ty + r;
        if (x < nx && y < ny) tile[ty + r][tx] = src[zoff + (int64_t)y * nx + x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int y = y0 + tx, x = x0 + ty + r;
        if (x < nx && y < ny) dst[zoff + (int64_t)x * ny + y] = tile[tx][ty + r];
    }
}

// Chord of each ray through the whole grid box (= A 1 of the Siddon projector), FP64 set-up.
__global__ __launch_bounds__(FWD_TU * FWD_TV) void k_ray_chord(float *__restrict__ chord, FwdArgs A) {
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
    A.gen = p->views ? 1 : 0;
    return A;
}

// Angles per launch: a dispatch holds its grid size in work-items as a 32-bit count, so one launch
// stays below 2^31 work-items and longer angle ranges go in several launches.
int64_t angles_per_launch(int64_t blocks_per_angle, int64_t threads_per_block) {
    return std::max<int64_t>(1, (int64_t(1) << 31) / std::max<int64_t>(1, blocks_per_angle * threads_per_block));
}

unsigned fwd_grid(const FwdArgs &A) {
    const int64_t vb = (A.nv + FWD_TV - 1) / FWD_TV;
    return (unsigned)((int64_t)A.ublocks * A.nang * vb);
}

}  // namespace

ct_status launch_transpose_xy(const void *vol, ct_dtype vt, void *volT, int64_t nx, int64_t ny, int64_t nz,
                              hipStream_t st) {
    const dim3 tg((unsigned)((nx + 31) / 32), (unsigned)((ny + 31) / 32), (unsigned)nz);
    CT_DISPATCH1(vt, T,
                 hipLaunchKernelGGL((k_transpose_xy<T>), tg, dim3(256), 0, st, (const T *)vol, (T *)volT, (int)nx, (int)ny));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_zcols(const void *vol, ct_dtype vt, void *vz, int64_t nx, int64_t ny, int64_t nz, hipStream_t st) {
    return launch_zcols_piece(vol, vt, vz, nx, ny, nz, nz + 2, 1, 3, st);
}

ct_status launch_zcols_piece(const void *src, ct_dtype vt, void *vz, int64_t nx, int64_t ny, int64_t nz, int64_t nzp,
                             int64_t slot0, int pads, hipStream_t st) {
    const dim3 tg((unsigned)((nx + 31) / 32), (unsigned)((nz + 31) / 32), (unsigned)ny);
    CT_DISPATCH1(vt, T,
                 hipLaunchKernelGGL((k_zcols<T, T>), tg, dim3(256), 0, st, (const T *)src, (T *)vz, (int)nx, (int)ny,
                                    (int)nz, nzp, (int)slot0, pads));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_zcols_f32(const void *vol, ct_dtype vt, float *vz, int64_t nx, int64_t ny, int64_t nz, hipStream_t st) {
    const dim3 tg((unsigned)((nx + 31) / 32), (unsigned)((nz + 31) / 32), (unsigned)ny);
    CT_DISPATCH1(vt, T,
                 hipLaunchKernelGGL((k_zcols<T, float>), tg, dim3(256), 0, st, (const T *)vol, vz, (int)nx, (int)ny,
                                    (int)nz, nz + 2, 1, 3));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_zcols_inv_f32(const float *vz, void *vol, ct_dtype vt, int64_t nx, int64_t ny, int64_t nz,
                               hipStream_t st) {
    const dim3 tg((unsigned)((nx + 31) / 32), (unsigned)((nz + 31) / 32), (unsigned)ny);
    CT_DISPATCH1(vt, T,
                 hipLaunchKernelGGL((k_zcols_inv<float, T>), tg, dim3(256), 0, st, vz, (T *)vol, (int)nx, (int)ny,
                                    (int)nz, nz + 2, 1));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status launch_zcols_inv(const void *vz, ct_dtype vt, void *vol, int64_t nx, int64_t ny, int64_t nz, hipStream_t st) {
    return launch_zcols_inv_piece(vz, vt, vol, nx, ny, nz, nz + 2, 1, st);
}

ct_status launch_zcols_inv_piece(const void *vz, ct_dtype vt, void *dst, int64_t nx, int64_t ny, int64_t zn,
                                 int64_t nzp, int64_t slot0, hipStream_t st) {
    if (zn <= 0) return CT_OK;
    if (slot0 < 0 || slot0 + zn > nzp) return fail(CT_ERR_ARG, "column-major piece outside its columns");
    const dim3 tg((unsigned)((nx + 31) / 32), (unsigned)((zn + 31) / 32), (unsigned)ny);
    CT_DISPATCH1(vt, T,
                 hipLaunchKernelGGL((k_zcols_inv<T, T>), tg, dim3(256), 0, st, (const T *)vz, (T *)dst, (int)nx, (int)ny,
                                    (int)zn, nzp, (int)slot0));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

bool zcol_ok(const ct_plan *p, int64_t a0, int64_t a1) {
    // the column walk needs vertical detector columns whose rays start at the source's height
    if (p->views && !p->vertical) return false;
    // every xy piece must climb less than one slice: |Dz| < max(|Dx|, |Dy|) for every ray.
    // max(|Dx|, |Dy|) is convex and piecewise linear in the detector coordinate u, so its minimum
    // over the detector lies at an end or where Dx, Dy or Dx +- Dy vanish.
    const ct_geometry &g = p->g;
    const double nu = (double)g.nDetector[0], nv = (double)g.nDetector[1];
    const double u0 = (0 - (nu - 1) / 2.0) * g.dDetector[0] + g.offDetector[0];
    const double u1 = ((nu - 1) - (nu - 1) / 2.0) * g.dDetector[0] + g.offDetector[0];
    const double v0 = (0 - (nv - 1) / 2.0) * g.dDetector[1] + g.offDetector[1];
    const double v1 = ((nv - 1) - (nv - 1) / 2.0) * g.dDetector[1] + g.offDetector[1];
    const double dzmax = std::max(fabs(v0), fabs(v1)) / g.dVoxel[2];
    for (int64_t i = a0; i < a1; ++i) {
        const AngleGeo &G = p->tab[(size_t)i];
        const double ulo = std::min(u0, u1), uhi = std::max(u0, u1);
        double cand[6] = {ulo, uhi, 0, 0, 0, 0};
        int nc = 2;
        auto root = [&](double c0, double c1) {
            if (c1 != 0.0) {
                const double r = -c0 / c1;
                if (r > ulo && r < uhi) cand[nc++] = r;
            }
        };
        root(G.Dc[0], G.eu[0]);
        root(G.Dc[1], G.eu[1]);
        root(G.Dc[0] + G.Dc[1], G.eu[0] + G.eu[1]);
        root(G.Dc[0] - G.Dc[1], G.eu[0] - G.eu[1]);
        double fmin_ = 1e300;
        for (int k = 0; k < nc; ++k) {
            const double dx = G.Dc[0] + cand[k] * G.eu[0], dy = G.Dc[1] + cand[k] * G.eu[1];
            fmin_ = std::min(fmin_, std::max(fabs(dx), fabs(dy)));
        }
        if (!(dzmax < 0.999 * fmin_)) return false;
        // slot offsets of a row's entry point stay far inside FP32's exact integers
        if (fabs(G.S[2]) + (double)g.nVoxel[2] + dzmax + 2.0 > 4194304.0) return false;
    }
    return true;
}

ct_status launch_forward(ct_plan *p, ct_projector kind, const void *vol, ct_dtype vt, void *proj, ct_dtype pt,
                         int accumulate, int64_t a0, int64_t a1, const Slab &slab, hipStream_t st,
                         const void *vcopy) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    if (slab.own_hi <= slab.own_lo) return CT_OK;
    const ct_geometry &g = p->g;
    const int64_t nx = g.nVoxel[0], ny = g.nVoxel[1];
#ifndef CT_NO_ZCOL
    // Siddon on a resident volume: column walk over the column-major copy
    // a slab launch must bring its own copy (mem_n + 2 slots per column) and own all it holds
    const bool whole = slab.own_lo == 0 && slab.own_hi == g.nVoxel[2] && slab.mem_lo == 0 &&
                       slab.mem_n == g.nVoxel[2];
    const bool slab_ok = vcopy && slab.own_lo == slab.mem_lo && slab.own_hi == slab.mem_lo + slab.mem_n;
    if (kind == CT_SIDDON && (whole ? (vcopy || slab.scratch_ok) : slab_ok) && zcol_ok(p, a0, a1)) {
        const int64_t nz = g.nVoxel[2];
        void *vz = const_cast<void *>(vcopy);
        void *own_z = nullptr;
        if (!vz) {
            const size_t zbytes = (size_t)(nx * ny * (nz + 2)) * dtype_size(vt);
            if (CT_MALLOC_ASYNC(&own_z, zbytes, st) == hipSuccess) {
                ct_status zs = launch_zcols(vol, vt, own_z, nx, ny, nz, st);
                if (zs != CT_OK) return zs;
                vz = own_z;
            } else {
                (void)hipGetLastError();
            }
        }
        if (vz) {
            const int64_t nu = g.nDetector[0], nv = g.nDetector[1];
            const int64_t cblocks = (nu + ZC_COLS - 1) / ZC_COLS;
            // two rows per lane when the launch is large enough to fill the chip with them
#ifdef CT_ZC_ROWS
            const int rows = CT_ZC_ROWS;
#else
#ifndef CT_IC_ROWS
            const int rows = cblocks * (a1 - a0) * ((nv + 127) / 128) >= 4096 ? 2 : 1;
#else
            const int rows = CT_IC_ROWS;
#endif
#endif
            const int64_t rgroups = (nv + 64 * rows - 1) / (64 * rows);
            const int64_t max_ang = angles_per_launch(cblocks * rgroups, 64 * ZC_COLS);
            const size_t proj_angle = (size_t)nu * nv * dtype_size(pt);
            for (int64_t c0 = a0; c0 < a1; c0 += max_ang) {
                const int64_t c1 = std::min(a1, c0 + max_ang);
                FwdArgs A = make_args(p, tab, c0, c1, slab, accumulate);
                A.cblocks = (int32_t)cblocks;
                A.rgroups = (int32_t)rgroups;
                char *pp = (char *)proj + (size_t)(c0 - a0) * proj_angle;
                const dim3 grid((unsigned)(cblocks * (c1 - c0) * rgroups)), block(64 * ZC_COLS);
#ifdef CT_ZC_ROWS
                if (rows == 4) {
                    CT_DISPATCH2(vt, TV, pt, TP,
                                 hipLaunchKernelGGL((k_siddon_col<TV, TP, 4>), grid, block, 0, st, (const TV *)vz,
                                                    (TP *)pp, A));
                } else
#endif
                if (rows == 2) {
                    CT_DISPATCH2(vt, TV, pt, TP,
                                 hipLaunchKernelGGL((k_siddon_col<TV, TP, 2>), grid, block, 0, st, (const TV *)vz,
                                                    (TP *)pp, A));
                } else {
                    CT_DISPATCH2(vt, TV, pt, TP,
                                 hipLaunchKernelGGL((k_siddon_col<TV, TP, 1>), grid, block, 0, st, (const TV *)vz,
                                                    (TP *)pp, A));
                }
                CT_HIP(hipGetLastError());
            }
            if (own_z) CT_HIP(hipFreeAsync(own_z, st));
            return CT_OK;
        }
    }
    // interpolated projector on a resident volume: zero-padded column-major copy, x-paired when
    // its doubled size stays modest
    if (kind == CT_INTERP && whole && slab.scratch_ok) {
        const int64_t nz = g.nVoxel[2];
        const size_t pbytes = (size_t)((nx + 3) * (ny + 3) * (nz + 3)) * dtype_size(vt);
#ifndef CT_IC_XPAIR_MAX
#define CT_IC_XPAIR_MAX (size_t(16) << 30)
#endif
        const bool xp = 2 * pbytes <= CT_IC_XPAIR_MAX;
        void *vpad = nullptr;
        if (CT_MALLOC_ASYNC(&vpad, xp ? 2 * pbytes : pbytes, st) == hipSuccess) {
            const dim3 tg((unsigned)((nx + 3 + 31) / 32), (unsigned)((nz + 3 + 31) / 32), (unsigned)(ny + 3));
            if (xp) {
                CT_DISPATCH1(vt, T,
                             hipLaunchKernelGGL((k_pcols2<T>), tg, dim3(256), 0, st, (const T *)vol, (T *)vpad, (int)nx,
                                                (int)ny, (int)nz));
            } else {
                CT_DISPATCH1(vt, T,
                             hipLaunchKernelGGL((k_pcols<T>), tg, dim3(256), 0, st, (const T *)vol, (T *)vpad, (int)nx,
                                                (int)ny, (int)nz));
            }
            CT_HIP(hipGetLastError());
            const int64_t nu = g.nDetector[0], nv = g.nDetector[1];
            const int64_t cblocks = (nu + ZC_COLS - 1) / ZC_COLS;
            const int rows = cblocks * (a1 - a0) * ((nv + 127) / 128) >= 4096 ? 2 : 1;
            const int64_t rgroups = (nv + 64 * rows - 1) / (64 * rows);
            const int64_t max_ang = angles_per_launch(cblocks * rgroups, 64 * ZC_COLS);
            const size_t proj_angle = (size_t)nu * nv * dtype_size(pt);
            for (int64_t c0 = a0; c0 < a1; c0 += max_ang) {
                const int64_t c1 = std::min(a1, c0 + max_ang);
                FwdArgs A = make_args(p, tab, c0, c1, slab, accumulate);
                A.cblocks = (int32_t)cblocks;
                A.rgroups = (int32_t)rgroups;
                char *pp = (char *)proj + (size_t)(c0 - a0) * proj_angle;
                const dim3 grid((unsigned)(cblocks * (c1 - c0) * rgroups)), block(64 * ZC_COLS);
#define CT_ICOL2(R, X, B)                                                                                      \
    CT_DISPATCH2(vt, TV, pt, TP,                                                                               \
                 hipLaunchKernelGGL((k_interp_col<TV, TP, R, X, B>), grid, block, 0, st, (const TV *)vpad, (TP *)pp, \
                                    A))
#define CT_ICOL(R, X)                          \
    if (p->views && !p->vertical) {            \
        CT_ICOL2(R, X, CT_IC_BATCH_T);         \
    } else {                                   \
        CT_ICOL2(R, X, CT_IC_BATCH_V);         \
    }
                if (rows == 2) {
                    if (xp) {
                        CT_ICOL(2, true);
                    } else {
                        CT_ICOL(2, false);
                    }
                } else {
                    if (xp) {
                        CT_ICOL(1, true);
                    } else {
                        CT_ICOL(1, false);
                    }
                }
#undef CT_ICOL
#undef CT_ICOL2
                CT_HIP(hipGetLastError());
            }
            CT_HIP(hipFreeAsync(vpad, st));
            return CT_OK;
        }
        (void)hipGetLastError();
    }
#endif
    const void *volT_given = kind == CT_SIDDON ? nullptr : vcopy;
    const int64_t elems = nx * ny * slab.mem_n;
    const size_t vbytes = (size_t)elems * dtype_size(vt);
    // transposed copy for the blocks whose rays run along x (stream-ordered scratch; without it
    // every block reads the natural layout)
    void *volT = const_cast<void *>(volT_given);
    void *own_t = nullptr;
#ifdef CT_NO_TRANSPOSE
    const bool want_t = false;
#else
    const bool want_t = !volT && slab.scratch_ok && nx > 1 && ny > 1;
#endif
    if (want_t && CT_MALLOC_ASYNC(&own_t, vbytes, st) != hipSuccess) {
        (void)hipGetLastError();
        own_t = nullptr;
    }
    if (own_t) {
        ct_status ts = launch_transpose_xy(vol, vt, own_t, nx, ny, slab.mem_n, st);
        if (ts != CT_OK) return ts;
        volT = own_t;
    }
    // 32-bit signed byte offsets: volumes (or slabs) below 2 GiB
    const bool buf = (uint64_t)vbytes < (uint64_t(1) << 31);
    const int64_t vb = (g.nDetector[1] + FWD_TV - 1) / FWD_TV;
    const int64_t ub = (g.nDetector[0] + FWD_TU - 1) / FWD_TU;
    const int64_t max_ang = angles_per_launch(vb * ub, FWD_TU * FWD_TV);
    const size_t proj_angle = (size_t)g.nDetector[0] * g.nDetector[1] * dtype_size(pt);
    for (int64_t c0 = a0; c0 < a1; c0 += max_ang) {
        const int64_t c1 = std::min(a1, c0 + max_ang);
        FwdArgs A = make_args(p, tab, c0, c1, slab, accumulate);
        char *pp = (char *)proj + (size_t)(c0 - a0) * proj_angle;
        const dim3 grid(fwd_grid(A)), block(FWD_TU * FWD_TV);
#define CT_FWD_LAUNCH(KERN, IDX)                                                                             \
    CT_DISPATCH2(vt, TV, pt, TP,                                                                             \
                 hipLaunchKernelGGL((KERN<TV, TP, IDX>), grid, block, 0, st, (const TV *)vol, (const TV *)volT, \
                                    (TP *)pp, A))
        if (kind == CT_SIDDON) {
            if (buf) {
                CT_FWD_LAUNCH(k_siddon, true);
            } else {
                CT_FWD_LAUNCH(k_siddon, false);
            }
        } else {
            if (buf) {
                CT_FWD_LAUNCH(k_interp, true);
            } else {
                CT_FWD_LAUNCH(k_interp, false);
            }
        }
#undef CT_FWD_LAUNCH
        CT_HIP(hipGetLastError());
    }
    if (own_t) CT_HIP(hipFreeAsync(own_t, st));
    return CT_OK;
}

ct_status launch_ray_chord(ct_plan *p, float *chord, int64_t a0, int64_t a1, hipStream_t st) {
    const AngleGeo *tab = nullptr;
    ct_status s = plan_device_table(p, st, &tab);
    if (s != CT_OK) return s;
    const ct_geometry &g = p->g;
    const int64_t vb = (g.nDetector[1] + FWD_TV - 1) / FWD_TV;
    const int64_t ub = (g.nDetector[0] + FWD_TU - 1) / FWD_TU;
    const int64_t max_ang = angles_per_launch(vb * ub, FWD_TU * FWD_TV);
    const size_t pix = (size_t)g.nDetector[0] * g.nDetector[1];
    for (int64_t c0 = a0; c0 < a1; c0 += max_ang) {
        const int64_t c1 = std::min(a1, c0 + max_ang);
        FwdArgs A = make_args(p, tab, c0, c1, full_slab(g), 0);
        hipLaunchKernelGGL(k_ray_chord, dim3(fwd_grid(A)), dim3(FWD_TU * FWD_TV), 0, st, chord + (size_t)(c0 - a0) * pix,
                           A);
        CT_HIP(hipGetLastError());
    }
    return CT_OK;
}

}  // namespace ct
