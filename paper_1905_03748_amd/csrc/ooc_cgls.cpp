// Out-of-core CGLS (Bjorck's iteration, as the paper's CGLS; Section 3.2 runs it on images larger
// than device memory).  Every vector lives in host memory: the operators are the out-of-core Siddon
// forward (Algorithm 1) and exact-adjoint backprojection (Algorithm 2) under the caller's device
// cap, and the vector updates and FP64 inner products run on the host's cores.
//
// The recurrence is the resident one: x += alpha p, r -= alpha q and p = s + beta p in FP32 with a
// fused multiply-add and the scalars rounded to FP32 once; gamma = <s,s>, delta = <q,q>,
// rho_{k+1} = rho_k - alpha gamma in FP64.  Inner products sum fixed blocks of elements in FP64
// and add the block sums in order, so results do not depend on the number of host threads.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <thread>
#include <vector>

#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr int64_t BLK = 1 << 20;  // elements per host block

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); }

int host_threads() {
    static const int n = [] {
        const unsigned h = std::thread::hardware_concurrency();
        return (int)std::max(1u, std::min(h ? h : 1u, 16u));
    }();
    return n;
}

// f(block, lo, hi) over the blocks of [0, n), spread over the host threads
template <typename F>
void par_blocks(int64_t n, F f) {
    const int64_t nb = (n + BLK - 1) / BLK;
    const int nt = (int)std::min<int64_t>(host_threads(), nb);
    if (nt <= 1) {
        for (int64_t b = 0; b < nb; ++b) f(b, b * BLK, std::min(n, (b + 1) * BLK));
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (int64_t b; (b = next.fetch_add(1)) < nb;) f(b, b * BLK, std::min(n, (b + 1) * BLK));
        });
    for (auto &x : th) x.join();
}

bool has_fma() {
    static const bool v = __builtin_cpu_supports("fma");
    return v;
}

// y[i] = fma(a, x[i], y[i])
__attribute__((target("fma"))) void axpy_hw(float *y, const float *x, float a, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) y[i] = __builtin_fmaf(a, x[i], y[i]);
}
void axpy_sw(float *y, const float *x, float a, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) y[i] = std::fma(a, x[i], y[i]);
}
// p[i] = fma(b, p[i], s[i])
__attribute__((target("fma"))) void xpby_hw(float *p, const float *s, float b, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) p[i] = __builtin_fmaf(b, p[i], s[i]);
}
void xpby_sw(float *p, const float *s, float b, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) p[i] = std::fma(b, p[i], s[i]);
}

void axpy(float *y, const float *x, float a, int64_t n) {
    if (a == 0.0f) return;
    const bool hw = has_fma();
    par_blocks(n, [&](int64_t, int64_t lo, int64_t hi) { hw ? axpy_hw(y, x, a, lo, hi) : axpy_sw(y, x, a, lo, hi); });
}

void xpby(float *p, const float *s, float b, int64_t n) {
    const bool hw = has_fma();
    par_blocks(n, [&](int64_t, int64_t lo, int64_t hi) { hw ? xpby_hw(p, s, b, lo, hi) : xpby_sw(p, s, b, lo, hi); });
}

// sum_i a[i] b[i] in FP64: four interleaved partial sums per block, block sums added in order
double dot(const float *a, const float *b, int64_t n) {
    const int64_t nb = (n + BLK - 1) / BLK;
    std::vector<double> part((size_t)nb, 0.0);
    par_blocks(n, [&](int64_t blk, int64_t lo, int64_t hi) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t i = lo;
        for (; i + 4 <= hi; i += 4) {
            s0 += (double)a[i] * b[i];
            s1 += (double)a[i + 1] * b[i + 1];
            s2 += (double)a[i + 2] * b[i + 2];
            s3 += (double)a[i + 3] * b[i + 3];
        }
        for (; i < hi; ++i) s0 += (double)a[i] * b[i];
        part[(size_t)blk] = (s0 + s1) + (s2 + s3);
    });
    double s = 0.0;
    for (double v : part) s += v;
    return s;
}

void copy(float *d, const float *s, int64_t n) {
    par_blocks(n, [&](int64_t, int64_t lo, int64_t hi) { std::memcpy(d + lo, s + lo, (size_t)(hi - lo) * 4); });
}

// d = b - d
void rsub(float *d, const float *b, int64_t n) {
    par_blocks(n, [&](int64_t, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) d[i] = b[i] - d[i];
    });
}

bool all_zero(const float *x, int64_t n) {
    std::atomic<bool> nz(false);
    par_blocks(n, [&](int64_t, int64_t lo, int64_t hi) {
        if (nz.load(std::memory_order_relaxed)) return;
        for (int64_t i = lo; i < hi; ++i)
            if (x[i] != 0.0f) {
                nz.store(true, std::memory_order_relaxed);
                return;
            }
    });
    return !nz.load();
}

void add_stats(ct_ooc_stats &t, const ct_ooc_stats &s) {
    t.bytes_h2d += s.bytes_h2d;
    t.bytes_d2h += s.bytes_d2h;
    t.t_compute_s += s.t_compute_s;
    t.t_stage_s += s.t_stage_s;
    t.t_other_mem_s += s.t_other_mem_s;
    t.t_pin_s += s.t_pin_s;
}

}  // namespace

size_t cgls_host_workspace(const ct_plan *p) {
    const ct_geometry &g = p->g;
    const size_t nv = (size_t)g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    const size_t np = (size_t)g.nDetector[0] * g.nDetector[1] * p->angles.size();
    return 2 * nv * 4 + 2 * np * 4;
}

ct_status cgls_host_run(ct_plan *p, const float *b, float *x, int32_t niter, double *resid, void *work, uint64_t cap,
                        ct_ooc_stats *stats) try {
    const auto t_start = clk::now();
    const ct_geometry &g = p->g;
    const int64_t nv = g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    const int64_t np = g.nDetector[0] * g.nDetector[1] * (int64_t)p->angles.size();
    float *r = (float *)work;
    float *q = r + np;
    float *sv = q + np;
    float *pv = sv + nv;
    ct_ooc_stats tot;
    std::memset(&tot, 0, sizeof(tot));
    bool planned = false;
    double t_host = 0.0;
    ct_status s;
    auto fwd = [&](const float *v, float *out) -> ct_status {
        ct_ooc_stats st;
        ct_status e = ooc_forward(p, CT_SIDDON, v, CT_F32, out, CT_F32, cap, &st);
        if (e != CT_OK) return e;
        if (!planned) {
            tot.n_slabs = st.n_slabs;
            tot.slab_slices = st.slab_slices;
            tot.chunk_angles = st.chunk_angles;
            tot.n_chunks = st.n_chunks;
            planned = true;
        }
        add_stats(tot, st);
        return CT_OK;
    };
    auto adj = [&](const float *y, float *out) -> ct_status {
        ct_ooc_stats st;
        ct_status e = ooc_backproject(p, CT_BP_ADJOINT, y, CT_F32, out, CT_F32, cap, &st);
        if (e != CT_OK) return e;
        add_stats(tot, st);
        return CT_OK;
    };
    auto host = [&](auto fn) {
        const auto a = clk::now();
        fn();
        t_host += secs(a, clk::now());
    };

    // r = b - A x (A 0 = 0 exactly, so a zero start skips the projection) ; s = A^T r ; p = s
    bool x0 = false;
    host([&] { x0 = all_zero(x, nv); });
    if (x0) {
        host([&] { copy(r, b, np); });
    } else {
        if ((s = fwd(x, r)) != CT_OK) return s;
        host([&] { rsub(r, b, np); });
    }
    if ((s = adj(r, sv)) != CT_OK) return s;
    double gamma = 0.0, rho = 0.0;
    host([&] {
        copy(pv, sv, nv);
        gamma = dot(sv, sv, nv);
        rho = dot(r, r, np);
    });
    if (resid) resid[0] = std::sqrt(std::max(rho, 0.0));
    bool stop = false;
    for (int32_t k = 0; k < niter; ++k) {
        if (!stop) {
            // q = A p ; delta = <q,q> ; alpha = gamma / delta
            if ((s = fwd(pv, q)) != CT_OK) return s;
            double delta = 0.0;
            host([&] { delta = dot(q, q, np); });
            if (delta == 0.0) {
                stop = true;
            } else {
                const double alpha = gamma / delta;
                rho -= alpha * gamma;
                // x += alpha p ; r -= alpha q
                host([&] {
                    axpy(x, pv, (float)alpha, nv);
                    axpy(r, q, -(float)alpha, np);
                });
                // s = A^T r ; beta = <s,s> / gamma ; p = s + beta p
                if ((s = adj(r, sv)) != CT_OK) return s;
                double gnew = 0.0;
                host([&] { gnew = dot(sv, sv, nv); });
                const double beta = gamma != 0.0 ? gnew / gamma : 0.0;
                gamma = gnew;
                host([&] { xpby(pv, sv, (float)beta, nv); });
            }
        }
        if (resid) resid[k + 1] = std::sqrt(std::max(rho, 0.0));
    }
    tot.t_other_mem_s += t_host;
    tot.t_total_s = secs(t_start, clk::now());
    if (stats) *stats = tot;
    return CT_OK;
} catch (const std::exception &e) {
    return fail(CT_ERR_STATE, std::string("ct_cgls_host: ") + e.what());
}

}  // namespace ct
