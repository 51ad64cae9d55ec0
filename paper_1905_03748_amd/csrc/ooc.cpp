// Out-of-core operators (Algorithm 1: forward; Algorithm 2: backprojection) on one device under a
// memory cap.  The image is split into equal axial slabs, as tall as the cap allows after the
// projection buffers; projections move in chunks of K angles.
//
// Forward: per slab, the slab is copied in; for each angle chunk the projection kernel runs into
// one of three device buffers while, on two copy streams, the previous chunk's result goes out
// and the next chunk's partial sums (from earlier slabs) come in.  Partial sums are accumulated
// by the projection kernel itself (it adds into the buffer), so no separate accumulation pass is
// needed.  Backprojection: per slab, projection chunks stream in double-buffered while the
// previous chunk is backprojected into the resident slab, which is copied out at the end.
//
// Pageable caller memory is staged through pinned buffers by host threads while the device
// computes; pinned caller memory (hipHostMalloc) is copied directly.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr uint64_t RESERVE = 64ull << 20;      // angle table, allocator slack
constexpr int64_t ZSTAGE = 8;                   // slices per column-major upload piece
constexpr size_t STAGE_PIECE = 64ull << 20;    // slab staging piece

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); }

// CT_OOC_VERBOSE=1 reports each finished slab on stderr (long out-of-core runs)
bool verbose() {
    static const bool v = [] {
        const char *e = std::getenv("CT_OOC_VERBOSE");
        return e && e[0] && e[0] != '0';
    }();
    return v;
}

void par_memcpy(void *dst, const void *src, size_t n) {
    if (n < (16u << 20)) {
        std::memcpy(dst, src, n);
        return;
    }
    const int nt = 8;
    std::vector<std::thread> th;
    const size_t part = (n + nt - 1) / nt;
    for (int i = 0; i < nt; ++i) {
        const size_t o = i * part;
        if (o >= n) break;
        const size_t len = std::min(part, n - o);
        th.emplace_back([=] { std::memcpy((char *)dst + o, (const char *)src + o, len); });
    }
    for (auto &t : th) t.join();
}

bool is_pinned(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};
struct HostBuf {
    void *p = nullptr;
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
};
struct Streams {
    hipStream_t comp = nullptr, h2d = nullptr, d2h = nullptr;
    ~Streams() {
        if (comp) (void)hipStreamDestroy(comp);
        if (h2d) (void)hipStreamDestroy(h2d);
        if (d2h) (void)hipStreamDestroy(d2h);
    }
};
struct Events {
    std::vector<hipEvent_t> e;
    ~Events() {
        for (auto x : e) (void)hipEventDestroy(x);
    }
    ct_status make(int n) {
        e.resize(n, nullptr);
        for (int i = 0; i < n; ++i) CT_HIP(hipEventCreateWithFlags(&e[i], hipEventDisableTiming));
        return CT_OK;
    }
};

struct Layout {
    int64_t h;        // slab height
    int64_t nsp;      // number of slabs
    int64_t K;        // angles per chunk
    int64_t halo;     // extra slices each side (interpolated forward)
    bool col;         // Siddon forward: the slab is held column-major (2 zero slots per column)
                      // and uploaded through a device stage of ZSTAGE slices
    int nbufs = 1;    // backprojection: slab buffers (2: the finished slab goes out while the next
                      // one accumulates)
};

// Slab buffers for the backprojection: CT_OOC_SLAB_BUFFERS=2 holds two slabs (each half as tall)
// so that a finished slab is copied out while the next one accumulates, overlapping the copy with
// the kernels (double-slab buffering); the default 1 keeps the tallest slabs.
int slab_buffers() {
    const char *e = std::getenv("CT_OOC_SLAB_BUFFERS");
    return (e && e[0] == '2') ? 2 : 1;
}

// direction: 0 forward, 1 backprojection (FDK, pseudo-matched), 2 exact-adjoint backprojection
ct_status layout_for(const ct_plan *p, int direction, ct_projector proj, ct_dtype vt, ct_dtype pt, uint64_t cap,
                     Layout &L) {
    const ct_geometry &g = p->g;
    const int64_t na = (int64_t)p->angles.size();
    const uint64_t slice = (uint64_t)g.nVoxel[0] * g.nVoxel[1] * dtype_size(vt);
    const uint64_t pangle = (uint64_t)g.nDetector[0] * g.nDetector[1] * dtype_size(pt);
    const int nbuf = direction == 0 ? 3 : 2;
    L.halo = (direction == 0 && proj == CT_INTERP) ? 1 : 0;
    L.col = direction == 0 && proj == CT_SIDDON && zcol_ok(p, 0, na);
    // slices held besides the slab: the forward's column stage, the interpolated projector's halo,
    // or the exact adjoint's stage for turning its column-major slab back into slices
    const int64_t extra = L.col ? 2 + ZSTAGE : (direction == 2 && adj_col_ok(p) ? ZSTAGE : 2 * L.halo);
    const int want_bufs = direction == 0 ? 1 : slab_buffers();
    L.nbufs = 1;
    // chunk size: enough rays (forward) or angles (backprojection) per launch to fill the device.
    // The exact adjoint's lanes run down voxel columns, so its slab accumulators are read and
    // written with a stride of one slice once per launch: it takes more angles per launch, each
    // with its transposed projection copy.
    const uint64_t pix = (uint64_t)g.nDetector[0] * g.nDetector[1];
    int64_t K = direction == 0 ? (int64_t)std::max<uint64_t>(1, (8ull << 20) / std::max<uint64_t>(pix, 1))
                               : (direction == 2 ? 128 : 32);
    K = std::min<int64_t>(K, na);
    K = std::max<int64_t>(K, 1);
    // fewest slabs wins (the image is split as little as possible); among equal counts the larger
    // chunk, down to an eighth of the target chunk (or 1 angle when not even one slice fits)
    const int64_t kmin = std::max<int64_t>(1, K / 8);
    bool found = false;
    for (int64_t k = K; k >= 1; k = (k == 1 ? 0 : std::max<int64_t>(1, k / 2))) {
        // the FDK reconstruction (direction 3) also holds the filtered FP32 copy of a chunk
        const uint64_t bufs = nbuf * (uint64_t)k * pangle +
                              (direction == 2 ? (uint64_t)k * adj_chunk_bytes_per_angle(g) : 0) +
                              (direction == 3 ? (uint64_t)k * pix * sizeof(float) : 0);
        int64_t h = 0;
        if (cap > RESERVE + bufs) h = (int64_t)((cap - RESERVE - bufs) / slice) - extra;
        if (h >= 1) {
            h = std::min<int64_t>(h, g.nVoxel[2]);
            const int64_t nsp = (g.nVoxel[2] + h - 1) / h;
            if (!found || nsp < L.nsp) {
                L.nsp = nsp;
                L.h = (g.nVoxel[2] + nsp - 1) / nsp;  // equal slabs, as tall as possible
                L.K = k;
                found = true;
            }
        }
        if (found && k <= kmin) break;
    }
    if (!found) return fail(CT_ERR_CAP, "device memory cap is below one slice plus the projection buffers");
    if (want_bufs == 2 && L.nsp > 1) {
        // two slab buffers in the same budget, with the chunk size of the single-buffer plan (its
        // kernels' efficiency is unchanged; only the slabs get thinner)
        const int64_t k = L.K;
        const uint64_t bufs = nbuf * (uint64_t)k * pangle +
                              (direction == 2 ? (uint64_t)k * adj_chunk_bytes_per_angle(g) : 0) +
                              (direction == 3 ? (uint64_t)k * pix * sizeof(float) : 0);
        const int64_t h = ((int64_t)((cap - RESERVE - bufs) / slice) - 2 * extra) / 2;
        if (h >= 1) {
            const int64_t nsp = (g.nVoxel[2] + h - 1) / h;
            L.nsp = nsp;
            L.h = (g.nVoxel[2] + nsp - 1) / nsp;
            L.nbufs = 2;
        }
    }
    return CT_OK;
}

// Detector rows [b0, b1) whose rays can meet the heights [zlo, zhi] (mm) of the volume (Section
// 2.1's observation that a slab of the image projects to a band of the detector).  The source lies
// in the plane z = 0 and a ray of row height v is at height t v at parameter t (t = 1 at the
// detector); inside the volume's xy extent t lies in [(DSO - R) / DSD, (DSO + R) / DSD], R bounding
// the distance of the volume box (grown by `grow` mm) from the axis, so the ray's v lies between
// zlo / t and zhi / t over that range.  `margin` rows are added on either side.
void row_band(const ct_geometry &g, double zlo, double zhi, double grow, int64_t margin, int64_t &b0, int64_t &b1) {
    double R = 0.0;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy) {
            const double xe = g.offOrigin[0] + (cx ? 0.5 : -0.5) * g.nVoxel[0] * g.dVoxel[0];
            const double ye = g.offOrigin[1] + (cy ? 0.5 : -0.5) * g.nVoxel[1] * g.dVoxel[1];
            R = std::max(R, std::sqrt(xe * xe + ye * ye));
        }
    R += grow;
    const int64_t nv = g.nDetector[1];
    b0 = 0;
    b1 = nv;
    if (!(g.DSO - R > 0.0)) return;
    const double tmin = (g.DSO - R) / g.DSD, tmax = (g.DSO + R) / g.DSD;
    const double vmin = std::min(zlo / tmin, zlo / tmax), vmax = std::max(zhi / tmin, zhi / tmax);
    const double cv = (nv - 1) / 2.0;
    const double bmin = (vmin - g.offDetector[1]) / g.dDetector[1] + cv;
    const double bmax = (vmax - g.offDetector[1]) / g.dDetector[1] + cv;
    b0 = std::max<int64_t>(0, (int64_t)std::floor(bmin) - margin);
    b1 = std::min<int64_t>(nv, (int64_t)std::floor(bmax) + 2 + margin);
    if (b1 < b0) b1 = b0;
}

// Height (mm) of the lower face of slice k.
double face_z(const ct_geometry &g, int64_t k) {
    return g.offOrigin[2] + ((double)k - 0.5 - (g.nVoxel[2] - 1) / 2.0) * g.dVoxel[2];
}

// rows [b0, b1) of each of n projections (pitch `pangle` bytes, rows of `rowb` bytes), 2-D copy
ct_status copy_rows(void *dst, const void *src, size_t pangle, size_t rowb, int64_t b0, int64_t b1, int64_t n,
                    hipMemcpyKind kind, hipStream_t st) {
    if (b1 <= b0 || n <= 0) return CT_OK;
    CT_HIP(hipMemcpy2DAsync((char *)dst + b0 * rowb, pangle, (const char *)src + b0 * rowb, pangle, (b1 - b0) * rowb, n,
                            kind, st));
    return CT_OK;
}

// the same between host buffers (staging), in parallel for large bands
void host_rows(void *dst, const void *src, size_t pangle, size_t rowb, int64_t b0, int64_t b1, int64_t n) {
    if (b1 <= b0) return;
    for (int64_t a = 0; a < n; ++a)
        par_memcpy((char *)dst + a * pangle + b0 * rowb, (const char *)src + a * pangle + b0 * rowb, (b1 - b0) * rowb);
}

}  // namespace

ct_status ooc_plan(const ct_plan *p, int direction, ct_projector proj, ct_dtype vt, ct_dtype pt, uint64_t cap,
                   ct_ooc_stats *out) {
    Layout L;
    ct_status s = layout_for(p, direction, proj, vt, pt, cap, L);
    if (s != CT_OK) return s;
    std::memset(out, 0, sizeof(*out));
    out->n_slabs = (int32_t)L.nsp;
    out->slab_slices = (int32_t)L.h;
    out->chunk_angles = (int32_t)L.K;
    out->n_chunks = (int32_t)(((int64_t)p->angles.size() + L.K - 1) / L.K);
    return CT_OK;
}

ct_status ooc_forward(ct_plan *p, ct_projector kind, const void *h_vol, ct_dtype vt, void *h_proj, ct_dtype pt,
                      uint64_t cap, ct_ooc_stats *stats) {
    const auto t_start = clk::now();
    const ct_geometry &g = p->g;
    Layout L;
    ct_status s = layout_for(p, 0, kind, vt, pt, cap, L);
    if (s != CT_OK) return s;
    ct_ooc_stats st;
    std::memset(&st, 0, sizeof(st));
    st.n_slabs = (int32_t)L.nsp;
    st.slab_slices = (int32_t)L.h;
    st.chunk_angles = (int32_t)L.K;
    const int64_t na = (int64_t)p->angles.size(), nz = g.nVoxel[2];
    const int64_t nchunks = (na + L.K - 1) / L.K;
    st.n_chunks = (int32_t)nchunks;
    const size_t slice = (size_t)g.nVoxel[0] * g.nVoxel[1] * dtype_size(vt);
    const size_t pangle = (size_t)g.nDetector[0] * g.nDetector[1] * dtype_size(pt);
    const size_t chunk_bytes = (size_t)L.K * pangle;
    const bool vol_pinned = is_pinned(h_vol), proj_pinned = is_pinned(h_proj);

    auto t0 = clk::now();
    Streams S;
    CT_HIP(hipStreamCreateWithFlags(&S.comp, hipStreamNonBlocking));
    CT_HIP(hipStreamCreateWithFlags(&S.h2d, hipStreamNonBlocking));
    CT_HIP(hipStreamCreateWithFlags(&S.d2h, hipStreamNonBlocking));
    DevBuf slab, stage, dbuf[3];
    CT_HIP(CT_MALLOC(&slab.p, (L.h + (L.col ? 2 : 2 * L.halo)) * slice));
    if (L.col) CT_HIP(CT_MALLOC(&stage.p, ZSTAGE * slice));
    for (auto &b : dbuf) CT_HIP(CT_MALLOC(&b.p, chunk_bytes));
    HostBuf sin[3], sout[3], svol[2];
    const auto tp = clk::now();
    if (!proj_pinned)
        for (int j = 0; j < 3; ++j) {
            CT_HIP(CT_HOST_MALLOC(&sin[j].p, chunk_bytes));
            CT_HIP(CT_HOST_MALLOC(&sout[j].p, chunk_bytes));
        }
    if (!vol_pinned)
        for (auto &b : svol) CT_HIP(CT_HOST_MALLOC(&b.p, STAGE_PIECE));
    st.t_pin_s += secs(tp, clk::now());
    Events ev_h2d, ev_k, ev_d2h, ev_vol, tk0, tk1;
    if ((s = ev_h2d.make(3)) != CT_OK || (s = ev_k.make(3)) != CT_OK || (s = ev_d2h.make(3)) != CT_OK ||
        (s = ev_vol.make(2)) != CT_OK)
        return s;
    tk0.e.resize(nchunks, nullptr);
    tk1.e.resize(nchunks, nullptr);
    for (int64_t c = 0; c < nchunks; ++c) {
        CT_HIP(hipEventCreate(&tk0.e[c]));
        CT_HIP(hipEventCreate(&tk1.e[c]));
    }
    st.t_other_mem_s += secs(t0, clk::now());

    // pending output chunks (and the row band they carry) waiting for their staging buffer to be
    // drained into h_proj
    int64_t pending[3] = {-1, -1, -1}, pend_b0[3] = {0, 0, 0}, pend_b1[3] = {0, 0, 0};
    const size_t rowb = (size_t)g.nDetector[0] * dtype_size(pt);
    auto drain = [&](int j) -> ct_status {
        if (pending[j] < 0) return CT_OK;
        CT_HIP(hipEventSynchronize(ev_d2h.e[j]));
        const int64_t c = pending[j];
        const int64_t nang = std::min(L.K, na - c * L.K);
        if (!proj_pinned) {
            auto a = clk::now();
            host_rows((char *)h_proj + c * chunk_bytes, sout[j].p, pangle, rowb, pend_b0[j], pend_b1[j], nang);
            st.t_stage_s += secs(a, clk::now());
        }
        pending[j] = -1;
        return CT_OK;
    };
    // detector rows already written by earlier slabs: [0, covered)
    int64_t covered = 0;

    for (int64_t n = 0; n < L.nsp; ++n) {
        const int64_t own_lo = n * L.h, own_hi = std::min(nz, own_lo + L.h);
        if (own_lo >= own_hi) break;
        const int64_t mem_lo = std::max<int64_t>(0, own_lo - L.halo);
        const int64_t mem_hi = std::min<int64_t>(nz, own_hi + L.halo);
        // the previous slab's kernels must finish before its buffer is overwritten
        auto a = clk::now();
        CT_HIP(hipStreamSynchronize(S.comp));
        // host bytes [src, src + total) to device dst, through the pinned ring when pageable
        auto upload = [&](void *dst, const char *src, size_t total) -> ct_status {
            if (vol_pinned) {
                CT_HIP(hipMemcpyAsync(dst, src, total, hipMemcpyHostToDevice, S.h2d));
            } else {
                size_t off = 0;
                int q = 0;
                bool used[2] = {false, false};
                while (off < total) {
                    const size_t len = std::min(STAGE_PIECE, total - off);
                    if (used[q]) CT_HIP(hipEventSynchronize(ev_vol.e[q]));
                    auto b = clk::now();
                    par_memcpy(svol[q].p, src + off, len);
                    st.t_stage_s += secs(b, clk::now());
                    CT_HIP(hipMemcpyAsync((char *)dst + off, svol[q].p, len, hipMemcpyHostToDevice, S.h2d));
                    CT_HIP(hipEventRecord(ev_vol.e[q], S.h2d));
                    used[q] = true;
                    off += len;
                    q ^= 1;
                }
            }
            CT_HIP(hipStreamSynchronize(S.h2d));
            st.bytes_h2d += (double)total;
            return CT_OK;
        };
        if (L.col) {
            // column-major slab: pieces of ZSTAGE slices through the stage, transposed into place
            const int64_t nzp = (own_hi - own_lo) + 2;
            for (int64_t z0 = own_lo; z0 < own_hi; z0 += ZSTAGE) {
                const int64_t zn = std::min(ZSTAGE, own_hi - z0);
                if ((s = upload(stage.p, (const char *)h_vol + z0 * slice, zn * slice)) != CT_OK) return s;
                const int pads = (z0 == own_lo ? 1 : 0) | (z0 + zn == own_hi ? 2 : 0);
                if ((s = launch_zcols_piece(stage.p, vt, slab.p, g.nVoxel[0], g.nVoxel[1], zn, nzp, 1 + (z0 - own_lo),
                                            pads, S.comp)) != CT_OK)
                    return s;
                CT_HIP(hipStreamSynchronize(S.comp));  // the stage is reused by the next piece
            }
        } else {
            if ((s = upload(slab.p, (const char *)h_vol + mem_lo * slice, (mem_hi - mem_lo) * slice)) != CT_OK)
                return s;
        }
        st.t_other_mem_s += secs(a, clk::now());

        Slab sl;
        sl.own_lo = own_lo;
        sl.own_hi = own_hi;
        sl.mem_lo = mem_lo;
        sl.mem_n = mem_hi - mem_lo;
        sl.first = (n == 0);
        sl.last = (own_hi == nz);
        sl.scratch_ok = false;
        // the rows this slab can add to (the interpolated projector's samples reach one voxel past
        // the owned faces); the first slab's band starts at row 0 and the last one's ends at the
        // top, so every row is written at least once.  Rows outside the band get exactly zero from
        // this slab: they are neither sent in nor read back.
        int64_t b0, b1;
        {
            const bool interp = kind == CT_INTERP;
            const double dz = g.dVoxel[2], grow = interp ? std::max(g.dVoxel[0], g.dVoxel[1]) : 0.0;
            row_band(g, face_z(g, own_lo) - (interp ? dz : 0.0), face_z(g, own_hi) + (interp ? dz : 0.0), grow,
                     interp ? 2 : 1, b0, b1);
            if (n == 0) b0 = 0;
            if (own_hi == nz) b1 = g.nDetector[1];
        }
        // rows [b0, min(b1, covered)) carry partial sums of earlier slabs; [max(b0, covered), b1)
        // start at zero here
        const int64_t in_hi = std::min(b1, covered), new_lo = std::max(b0, covered);
        const bool acc = n > 0;
        for (int64_t c = 0; c < nchunks; ++c) {
            const int j = (int)(c % 3);
            const int64_t a0 = c * L.K, a1 = std::min(na, a0 + L.K);
            const int64_t nang = a1 - a0;
            if ((s = drain(j)) != CT_OK) return s;
            if (acc) {
                // partial sums of earlier slabs for this chunk come in (buffer free once its last D2H ended)
                CT_HIP(hipStreamWaitEvent(S.h2d, ev_d2h.e[j], 0));
                const void *from = (const char *)h_proj + a0 * pangle;
                if (!proj_pinned) {
                    CT_HIP(hipEventSynchronize(ev_h2d.e[j]));
                    auto b = clk::now();
                    host_rows(sin[j].p, from, pangle, rowb, b0, in_hi, nang);
                    st.t_stage_s += secs(b, clk::now());
                    from = sin[j].p;
                }
                if ((s = copy_rows(dbuf[j].p, from, pangle, rowb, b0, in_hi, nang, hipMemcpyHostToDevice, S.h2d)) !=
                    CT_OK)
                    return s;
                CT_HIP(hipEventRecord(ev_h2d.e[j], S.h2d));
                CT_HIP(hipStreamWaitEvent(S.comp, ev_h2d.e[j], 0));
                st.bytes_h2d += (double)(std::max<int64_t>(0, in_hi - b0) * rowb * nang);
                if (b1 > new_lo)
                    CT_HIP(hipMemset2DAsync((char *)dbuf[j].p + new_lo * rowb, pangle, 0, (b1 - new_lo) * rowb, nang,
                                            S.comp));
            } else {
                CT_HIP(hipStreamWaitEvent(S.comp, ev_d2h.e[j], 0));
            }
            CT_HIP(hipEventRecord(tk0.e[c], S.comp));
            if ((s = launch_forward(p, kind, slab.p, vt, dbuf[j].p, pt, acc ? 1 : 0, a0, a1, sl, S.comp,
                                    L.col ? slab.p : nullptr)) != CT_OK)
                return s;
            CT_HIP(hipEventRecord(tk1.e[c], S.comp));
            CT_HIP(hipEventRecord(ev_k.e[j], S.comp));
            CT_HIP(hipStreamWaitEvent(S.d2h, ev_k.e[j], 0));
            void *to = proj_pinned ? (char *)h_proj + a0 * pangle : sout[j].p;
            if ((s = copy_rows(to, dbuf[j].p, pangle, rowb, b0, b1, nang, hipMemcpyDeviceToHost, S.d2h)) != CT_OK)
                return s;
            CT_HIP(hipEventRecord(ev_d2h.e[j], S.d2h));
            st.bytes_d2h += (double)((b1 - b0) * rowb * nang);
            pending[j] = c;
            pend_b0[j] = b0;
            pend_b1[j] = b1;
        }
        covered = std::max(covered, b1);
        for (int j = 0; j < 3; ++j)
            if ((s = drain(j)) != CT_OK) return s;
        CT_HIP(hipStreamSynchronize(S.comp));
        for (int64_t c = 0; c < nchunks; ++c) {
            float ms = 0;
            CT_HIP(hipEventElapsedTime(&ms, tk0.e[c], tk1.e[c]));
            st.t_compute_s += ms * 1e-3;
        }
        if (verbose()) {
            std::fprintf(stderr, "[ct ooc forward] slab %lld/%lld (slices %lld-%lld) done at %.1f s\n", (long long)n + 1,
                         (long long)L.nsp, (long long)own_lo, (long long)own_hi - 1, secs(t_start, clk::now()));
            std::fflush(stderr);
        }
    }
    CT_HIP(hipStreamSynchronize(S.d2h));
    st.t_total_s = secs(t_start, clk::now());
    if (stats) *stats = st;
    return CT_OK;
}

ct_status ooc_backproject(ct_plan *p, ct_backprojector kind, const void *h_proj, ct_dtype pt, void *h_vol, ct_dtype vt,
                          uint64_t cap, ct_ooc_stats *stats, bool fdk_filtered) {
    const auto t_start = clk::now();
    const ct_geometry &g = p->g;
    Layout L;
    if (fdk_filtered) kind = CT_BP_FDK;
    ct_status s = layout_for(p, fdk_filtered ? 3 : (kind == CT_BP_ADJOINT ? 2 : 1), CT_SIDDON, vt, pt, cap, L);
    if (s != CT_OK) return s;
    ct_ooc_stats st;
    std::memset(&st, 0, sizeof(st));
    st.n_slabs = (int32_t)L.nsp;
    st.slab_slices = (int32_t)L.h;
    st.chunk_angles = (int32_t)L.K;
    const int64_t na = (int64_t)p->angles.size(), nz = g.nVoxel[2];
    const int64_t nchunks = (na + L.K - 1) / L.K;
    st.n_chunks = (int32_t)nchunks;
    const size_t slice = (size_t)g.nVoxel[0] * g.nVoxel[1] * dtype_size(vt);
    const size_t pangle = (size_t)g.nDetector[0] * g.nDetector[1] * dtype_size(pt);
    const size_t chunk_bytes = (size_t)L.K * pangle;
    const bool vol_pinned = is_pinned(h_vol), proj_pinned = is_pinned(h_proj);

    auto t0 = clk::now();
    Streams S;
    CT_HIP(hipStreamCreateWithFlags(&S.comp, hipStreamNonBlocking));
    CT_HIP(hipStreamCreateWithFlags(&S.h2d, hipStreamNonBlocking));
    CT_HIP(hipStreamCreateWithFlags(&S.d2h, hipStreamNonBlocking));
    // the exact adjoint accumulates into a column-major slab (its lanes run down the columns), which
    // goes out through a stage of ZSTAGE slices
    const bool zcol = kind == CT_BP_ADJOINT && adj_col_ok(p);
    const int NB = L.nbufs;
    DevBuf slab[2], dbuf[2], adj, stage[2], filt;
    for (int k = 0; k < NB; ++k) {
        CT_HIP(CT_MALLOC(&slab[k].p, L.h * slice));
        if (zcol) CT_HIP(CT_MALLOC(&stage[k].p, ZSTAGE * slice));
    }
    for (auto &b : dbuf) CT_HIP(CT_MALLOC(&b.p, chunk_bytes));
    const size_t adj_bytes = (size_t)L.K * adj_chunk_bytes_per_angle(g);  // one transposed copy per chunk
    if (kind == CT_BP_ADJOINT) CT_HIP(CT_MALLOC(&adj.p, adj_bytes));
    // FDK reconstruction: each chunk is weighted and filtered into an FP32 buffer, which the
    // backprojection reads (both on the compute stream, so the buffer is reused in order)
    if (fdk_filtered) CT_HIP(CT_MALLOC(&filt.p, (size_t)L.K * g.nDetector[0] * g.nDetector[1] * sizeof(float)));
    HostBuf sin[2], svol[2][2];
    const auto tp = clk::now();
    if (!proj_pinned)
        for (auto &b : sin) CT_HIP(CT_HOST_MALLOC(&b.p, chunk_bytes));
    if (!vol_pinned)
        for (int k = 0; k < NB; ++k)
            for (auto &b : svol[k]) CT_HIP(CT_HOST_MALLOC(&b.p, STAGE_PIECE));
    st.t_pin_s += secs(tp, clk::now());
    Events ev_h2d, ev_k, ev_vol[2], ev_slab, tk0, tk1;
    if ((s = ev_h2d.make(2)) != CT_OK || (s = ev_k.make(2)) != CT_OK || (s = ev_vol[0].make(2)) != CT_OK ||
        (s = ev_vol[1].make(2)) != CT_OK || (s = ev_slab.make(2)) != CT_OK)
        return s;
    // the way out for finished slabs (with two slab buffers, on a thread of its own)
    hipStream_t s_out[2] = {nullptr, nullptr};
    struct OutStreams {
        hipStream_t *s;
        ~OutStreams() {
            for (int k = 0; k < 2; ++k)
                if (s[k]) (void)hipStreamDestroy(s[k]);
        }
    } out_guard{s_out};
    for (int k = 0; k < NB; ++k) CT_HIP(hipStreamCreateWithFlags(&s_out[k], hipStreamNonBlocking));
    tk0.e.resize(nchunks, nullptr);
    tk1.e.resize(nchunks, nullptr);
    for (int64_t c = 0; c < nchunks; ++c) {
        CT_HIP(hipEventCreate(&tk0.e[c]));
        CT_HIP(hipEventCreate(&tk1.e[c]));
    }
    st.t_other_mem_s += secs(t0, clk::now());
    int dev = 0;
    CT_HIP(hipGetDevice(&dev));

    // Copy slab n (buffer k, slices [own_lo, own_hi)) to h_vol once its kernels have finished (event
    // ev_slab[k]): column-major slabs through the stage, pageable memory through the pinned ring.
    // Stages its own buffers and stream only, so it may run beside the next slab's chunk loop.
    struct OutResult {
        ct_status s = CT_OK;
        std::string err;
        double t_stage = 0.0;
    };
    auto slab_out = [&](int k, int64_t own_lo, int64_t own_hi, OutResult &r) {
        auto chk = [&](hipError_t e, const char *what) {
            if (e != hipSuccess && r.s == CT_OK) {
                r.s = e == hipErrorOutOfMemory ? CT_ERR_OOM : CT_ERR_HIP;
                r.err = std::string(what) + ": " + hipGetErrorString(e);
            }
            return e == hipSuccess;
        };
        if (!chk(hipSetDevice(dev), "hipSetDevice")) return;
        hipStream_t so = s_out[k];
        if (!chk(hipStreamWaitEvent(so, ev_slab.e[k], 0), "hipStreamWaitEvent")) return;
        char *dst = (char *)h_vol + own_lo * slice;
        auto download = [&](const char *src, char *hdst, size_t len_all) -> bool {
            if (vol_pinned) {
                return chk(hipMemcpyAsync(hdst, src, len_all, hipMemcpyDeviceToHost, so), "slab download") &&
                       chk(hipStreamSynchronize(so), "slab download");
            }
            // pipelined: piece q goes D2H while piece q-1 is copied out of staging by the host
            size_t off = 0, prev_off = 0, prev_len = 0;
            int q = 0, prev_q = -1;
            while (off < len_all || prev_q >= 0) {
                int cur = -1;
                size_t len = 0;
                if (off < len_all) {
                    len = std::min(STAGE_PIECE, len_all - off);
                    if (!chk(hipMemcpyAsync(svol[k][q].p, src + off, len, hipMemcpyDeviceToHost, so), "slab download") ||
                        !chk(hipEventRecord(ev_vol[k].e[q], so), "hipEventRecord"))
                        return false;
                    cur = q;
                }
                if (prev_q >= 0) {
                    if (!chk(hipEventSynchronize(ev_vol[k].e[prev_q]), "hipEventSynchronize")) return false;
                    auto b = clk::now();
                    par_memcpy(hdst + prev_off, svol[k][prev_q].p, prev_len);
                    r.t_stage += secs(b, clk::now());
                }
                prev_q = cur;
                prev_off = off;
                prev_len = len;
                off += len;
                q ^= 1;
            }
            return true;
        };
        if (zcol) {
            const int64_t nzown = own_hi - own_lo;
            for (int64_t z0 = 0; z0 < nzown; z0 += ZSTAGE) {
                const int64_t zn = std::min(ZSTAGE, nzown - z0);
                ct_status zs = launch_zcols_inv_piece(slab[k].p, vt, stage[k].p, g.nVoxel[0], g.nVoxel[1], zn, nzown, z0, so);
                if (zs != CT_OK) {
                    r.s = zs;
                    r.err = "slab transpose launch failed";
                    return;
                }
                if (!chk(hipStreamSynchronize(so), "slab transpose")) return;
                if (!download((const char *)stage[k].p, dst + z0 * slice, zn * slice)) return;
            }
        } else {
            download((const char *)slab[k].p, dst, (size_t)(own_hi - own_lo) * slice);
        }
    };
    std::thread out_thread[2];
    OutResult out_res[2];
    int64_t out_lo[2] = {0, 0}, out_hi[2] = {0, 0};
    // wait for the copy-out of buffer k (if any) and take over its result
    auto join_out = [&](int k) -> ct_status {
        if (!out_thread[k].joinable()) return CT_OK;
        auto a = clk::now();
        out_thread[k].join();
        st.t_other_mem_s += secs(a, clk::now());
        st.t_stage_s += out_res[k].t_stage;
        st.bytes_d2h += (double)(out_hi[k] - out_lo[k]) * slice;
        if (out_res[k].s != CT_OK) return fail(out_res[k].s, out_res[k].err);
        if (verbose()) {
            std::fprintf(stderr, "[ct ooc backprojection] slices %lld-%lld out at %.1f s\n", (long long)out_lo[k],
                         (long long)out_hi[k] - 1, secs(t_start, clk::now()));
            std::fflush(stderr);
        }
        return CT_OK;
    };
    struct JoinAll {
        std::thread *t;
        ~JoinAll() {
            for (int k = 0; k < 2; ++k)
                if (t[k].joinable()) t[k].join();
        }
    } join_guard{out_thread};

    for (int64_t n = 0; n < L.nsp; ++n) {
        const int64_t own_lo = n * L.h, own_hi = std::min(nz, own_lo + L.h);
        if (own_lo >= own_hi) break;
        const int kbuf = (int)(n % NB);
        // the buffer's previous slab must be out before it accumulates again
        if ((s = join_out(kbuf)) != CT_OK) return s;
        Slab sl;
        sl.own_lo = own_lo;
        sl.own_hi = own_hi;
        sl.mem_lo = own_lo;
        sl.mem_n = own_hi - own_lo;
        sl.first = sl.last = true;
        sl.scratch_ok = false;
        sl.zcol = zcol;
        // the detector rows the slab's voxels read (bilinear taps, or the rays that cross their
        // boxes, with two rows to spare for the candidate rows the exact adjoint visits); the rest of
        // each chunk buffer is zeroed once per slab and never sent
        int64_t b0, b1;
        row_band(g, face_z(g, own_lo), face_z(g, own_hi), 0.0, 2, b0, b1);
        const int64_t nv = g.nDetector[1];
        const size_t rowb = (size_t)g.nDetector[0] * dtype_size(pt);
        bool h2d_used[2] = {false, false};
        for (int64_t c = 0; c < nchunks; ++c) {
            const int j = (int)(c % 2);
            const int64_t a0 = c * L.K, a1 = std::min(na, a0 + L.K);
            const int64_t nang = a1 - a0;
            // device buffer j is free once the kernel two chunks back has read it
            CT_HIP(hipStreamWaitEvent(S.h2d, ev_k.e[j], 0));
            if (c < 2) {
                if (b0 > 0) CT_HIP(hipMemset2DAsync(dbuf[j].p, pangle, 0, b0 * rowb, L.K, S.h2d));
                if (b1 < nv) CT_HIP(hipMemset2DAsync((char *)dbuf[j].p + b1 * rowb, pangle, 0, (nv - b1) * rowb, L.K, S.h2d));
            }
            const void *from = (const char *)h_proj + a0 * pangle;
            if (!proj_pinned) {
                if (h2d_used[j]) CT_HIP(hipEventSynchronize(ev_h2d.e[j]));
                auto b = clk::now();
                host_rows(sin[j].p, from, pangle, rowb, b0, b1, nang);
                st.t_stage_s += secs(b, clk::now());
                from = sin[j].p;
            }
            if ((s = copy_rows(dbuf[j].p, from, pangle, rowb, b0, b1, nang, hipMemcpyHostToDevice, S.h2d)) != CT_OK)
                return s;
            CT_HIP(hipEventRecord(ev_h2d.e[j], S.h2d));
            h2d_used[j] = true;
            st.bytes_h2d += (double)((b1 - b0) * rowb * nang);
            CT_HIP(hipStreamWaitEvent(S.comp, ev_h2d.e[j], 0));
            CT_HIP(hipEventRecord(tk0.e[c], S.comp));
            const void *bp_in = dbuf[j].p;
            ct_dtype bp_t = pt;
            if (fdk_filtered) {
                if ((s = fdk_filter(p, dbuf[j].p, pt, (float *)filt.p, a0, a1, S.comp)) != CT_OK) return s;
                bp_in = filt.p;
                bp_t = CT_F32;
            }
            if ((s = launch_backproject(p, kind, bp_in, bp_t, slab[kbuf].p, vt, c > 0 ? 1 : 0, a0, a1, sl, S.comp,
                                        adj.p, adj.p ? adj_bytes : 0)) != CT_OK)
                return s;
            CT_HIP(hipEventRecord(tk1.e[c], S.comp));
            CT_HIP(hipEventRecord(ev_k.e[j], S.comp));
        }
        // slab out: after its last kernel; with two buffers on a thread of its own while the next
        // slab accumulates in the other buffer
        CT_HIP(hipEventRecord(ev_slab.e[kbuf], S.comp));
        out_lo[kbuf] = own_lo;
        out_hi[kbuf] = own_hi;
        out_res[kbuf] = OutResult();
        if (NB == 2) {
            out_thread[kbuf] = std::thread(slab_out, kbuf, own_lo, own_hi, std::ref(out_res[kbuf]));
        } else {
            auto a = clk::now();
            slab_out(kbuf, own_lo, own_hi, out_res[kbuf]);
            st.t_other_mem_s += secs(a, clk::now());
            st.t_stage_s += out_res[kbuf].t_stage;
            st.bytes_d2h += (double)(own_hi - own_lo) * slice;
            if (out_res[kbuf].s != CT_OK) return fail(out_res[kbuf].s, out_res[kbuf].err);
        }
        // the chunk kernels' times (their events are reused by the next slab)
        CT_HIP(hipEventSynchronize(tk1.e[nchunks - 1]));
        for (int64_t c = 0; c < nchunks; ++c) {
            float ms = 0;
            CT_HIP(hipEventElapsedTime(&ms, tk0.e[c], tk1.e[c]));
            st.t_compute_s += ms * 1e-3;
        }
        if (verbose()) {
            std::fprintf(stderr, "[ct ooc backprojection] slab %lld/%lld (slices %lld-%lld) done at %.1f s\n",
                         (long long)n + 1, (long long)L.nsp, (long long)own_lo, (long long)own_hi - 1,
                         secs(t_start, clk::now()));
            std::fflush(stderr);
        }
    }
    for (int k = 0; k < NB; ++k)
        if ((s = join_out(k)) != CT_OK) return s;
    st.t_total_s = secs(t_start, clk::now());
    if (stats) *stats = st;
    return CT_OK;
}

}  // namespace ct
