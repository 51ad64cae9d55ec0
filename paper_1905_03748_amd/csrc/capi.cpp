// C ABI entry points, geometry validation, per-angle tables and error reporting.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "ct_internal.hpp"

namespace ct {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ct_status fail(ct_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

ct_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return CT_ERR_OOM;
    return CT_ERR_HIP;
}

hipError_t fault_check() {
    const char *e = std::getenv("CT_FAULT_ALLOC");
    if (!e || !e[0]) return hipSuccess;
    static std::mutex mu;
    static std::string last;
    static long count = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (last != e) {
        last = e;
        count = 0;
    }
    return ++count == std::strtol(e, nullptr, 10) ? hipErrorOutOfMemory : hipSuccess;
}

size_t dtype_size(ct_dtype t) { return t == CT_F64 ? 8 : t == CT_F32 ? 4 : 2; }
bool dtype_ok(int t) { return t == CT_F32 || t == CT_F16 || t == CT_BF16; }
bool dtype_ok_any(int t) { return dtype_ok(t) || t == CT_F64; }

// the grid, detector and accuracy fields (all plans)
static ct_status validate_grid(const ct_geometry &g) {
    for (int a = 0; a < 3; ++a) {
        if (g.nVoxel[a] <= 0 || !(g.dVoxel[a] > 0) || !std::isfinite(g.dVoxel[a]) ||
            !std::isfinite(g.offOrigin[a]))
            return fail(CT_ERR_GEOMETRY, "geometry: voxel counts and sizes must be positive and finite");
    }
    for (int a = 0; a < 2; ++a) {
        if (g.nDetector[a] <= 0 || !(g.dDetector[a] > 0) || !std::isfinite(g.dDetector[a]) ||
            !std::isfinite(g.offDetector[a]))
            return fail(CT_ERR_GEOMETRY, "geometry: detector counts and sizes must be positive and finite");
    }
    if (g.nVoxel[0] > (1 << 24) || g.nVoxel[1] > (1 << 24) || g.nVoxel[2] > (1 << 24) ||
        g.nDetector[0] > (1 << 24) || g.nDetector[1] > (1 << 24))
        return fail(CT_ERR_GEOMETRY, "geometry: a dimension exceeds 2^24");
    if (!(g.accuracy >= 0.0 && g.accuracy <= 1.0))
        return fail(CT_ERR_GEOMETRY, "geometry: accuracy must be in (0, 1] (0 selects 0.5)");
    return CT_OK;
}

// a circular orbit: also the distances
static ct_status validate(const ct_geometry &g) {
    if (!(g.DSO > 0) || !(g.DSD > g.DSO) || !std::isfinite(g.DSD))
        return fail(CT_ERR_GEOMETRY, "geometry: need DSD > DSO > 0");
    ct_status st = validate_grid(g);
    if (st != CT_OK) return st;
    double r2 = 0;
    for (int sx = -1; sx <= 1; sx += 2)
        for (int sy = -1; sy <= 1; sy += 2) {
            double x = g.offOrigin[0] + sx * g.nVoxel[0] * g.dVoxel[0] / 2.0;
            double y = g.offOrigin[1] + sy * g.nVoxel[1] * g.dVoxel[1] / 2.0;
            r2 = std::fmax(r2, x * x + y * y);
        }
    if (!(r2 < g.DSO * g.DSO))
        return fail(CT_ERR_GEOMETRY, "geometry: the volume box must lie strictly inside the source orbit");
    return CT_OK;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// The general part of a view's table entry from its source Smm, detector centre Cmm and unit axes
// eu, ev (mm, world frame): e_v in index units, the projective map M, DSO_v and the pseudo-matched
// constant (see AngleGeo).
static void fill_general(const ct_geometry &g, const double *Smm, const double *Cmm, const double *eu,
                         const double *ev, AngleGeo &t) {
    const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
    double x0[3], SC[3];
    for (int a = 0; a < 3; ++a) {
        t.ev[a] = ev[a] / g.dVoxel[a];
        t.Smm[a] = Smm[a];
        x0[a] = g.offOrigin[a] - (g.nVoxel[a] - 1) / 2.0 * g.dVoxel[a];  // centre of voxel (0, 0, 0)
        SC[a] = Smm[a] - Cmm[a];
    }
    const double DSDv = dot3(SC, n);
    t.DSOv = dot3(Smm, n);
    t.DSDv = DSDv;
    t.pmc = g.dVoxel[0] * g.dVoxel[1] * g.dVoxel[2] / (g.dDetector[0] * g.dDetector[1]) * DSDv * DSDv;
    // L(X) = n.(S - X); u* L = ((S - C).e_u) L + DSD_v e_u.(X - S); a* L = u* L / du + (cu - offU / du) L
    const double cu = (g.nDetector[0] - 1) / 2.0, cv = (g.nDetector[1] - 1) / 2.0;
    double Lr[4], Ur[4], Vr[4];
    Lr[3] = dot3(n, Smm) - dot3(n, x0);
    for (int a = 0; a < 3; ++a) Lr[a] = -n[a] * g.dVoxel[a];
    const double seu = dot3(SC, eu), sev = dot3(SC, ev);
    for (int a = 0; a < 3; ++a) {
        Ur[a] = seu * Lr[a] + DSDv * eu[a] * g.dVoxel[a];
        Vr[a] = sev * Lr[a] + DSDv * ev[a] * g.dVoxel[a];
    }
    Ur[3] = seu * Lr[3] + DSDv * (dot3(eu, x0) - dot3(eu, Smm));
    Vr[3] = sev * Lr[3] + DSDv * (dot3(ev, x0) - dot3(ev, Smm));
    const double ka = cu - g.offDetector[0] / g.dDetector[0], kb = cv - g.offDetector[1] / g.dDetector[1];
    for (int a = 0; a < 4; ++a) {
        t.M[a] = Ur[a] / g.dDetector[0] + ka * Lr[a];
        t.M[4 + a] = Vr[a] / g.dDetector[1] + kb * Lr[a];
        t.M[8 + a] = Lr[a];
    }
}

static AngleGeo angle_geo(const ct_geometry &g, double th) {
    AngleGeo t;
    std::memset(&t, 0, sizeof(t));
    t.c = std::cos(th);
    t.s = std::sin(th);
    const double Smm[3] = {g.DSO * t.c, g.DSO * t.s, 0.0};
    for (int a = 0; a < 3; ++a)
        t.S[a] = (Smm[a] - g.offOrigin[a]) / g.dVoxel[a] + (g.nVoxel[a] - 1) / 2.0;
    // detector centre minus source = -DSD (cos, sin, 0)
    t.Dc[0] = -g.DSD * t.c / g.dVoxel[0];
    t.Dc[1] = -g.DSD * t.s / g.dVoxel[1];
    t.Dc[2] = 0.0;
    t.eu[0] = -t.s / g.dVoxel[0];
    t.eu[1] = t.c / g.dVoxel[1];
    t.eu[2] = 0.0;
    const double Cmm[3] = {-(g.DSD - g.DSO) * t.c, -(g.DSD - g.DSO) * t.s, 0.0};
    const double eu[3] = {-t.s, t.c, 0.0}, ev[3] = {0.0, 0.0, 1.0};
    fill_general(g, Smm, Cmm, eu, ev, t);
    return t;
}

// The table entry of a view (source S, detector centre C, unit axes e_u, e_v; mm).
static AngleGeo view_geo(const ct_geometry &g, const double *v) {
    AngleGeo t;
    std::memset(&t, 0, sizeof(t));
    for (int a = 0; a < 3; ++a) {
        t.S[a] = (v[a] - g.offOrigin[a]) / g.dVoxel[a] + (g.nVoxel[a] - 1) / 2.0;
        t.Dc[a] = (v[3 + a] - v[a]) / g.dVoxel[a];
        t.eu[a] = v[6 + a] / g.dVoxel[a];
    }
    fill_general(g, v, v + 3, v + 6, v + 9, t);
    return t;
}

// A view the kernels can serve: finite, orthonormal detector axes, the source in front of the
// detector plane (on the side its normal points to), and every corner of the volume box at a
// positive depth from the source.
static ct_status validate_view(const ct_geometry &g, const double *v, int64_t i) {
    const std::string who = "ct_plan_create_views: view " + std::to_string(i) + ": ";
    for (int a = 0; a < 12; ++a)
        if (!std::isfinite(v[a])) return fail(CT_ERR_GEOMETRY, who + "non-finite entry");
    const double *eu = v + 6, *ev = v + 9;
    if (std::fabs(dot3(eu, eu) - 1.0) > 1e-9 || std::fabs(dot3(ev, ev) - 1.0) > 1e-9 || std::fabs(dot3(eu, ev)) > 1e-9)
        return fail(CT_ERR_GEOMETRY, who + "e_u and e_v must be orthonormal (to 1e-9)");
    const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
    const double SC[3] = {v[0] - v[3], v[1] - v[4], v[2] - v[5]};
    if (!(dot3(SC, n) > 0.0)) return fail(CT_ERR_GEOMETRY, who + "the source must lie in front of the detector (along e_u x e_v)");
    for (int c = 0; c < 8; ++c) {
        double X[3];
        for (int a = 0; a < 3; ++a) X[a] = g.offOrigin[a] + (((c >> a) & 1) ? 0.5 : -0.5) * g.nVoxel[a] * g.dVoxel[a] - v[a];
        if (!(-dot3(X, n) > 1e-6 * std::sqrt(dot3(SC, SC))))
            return fail(CT_ERR_GEOMETRY, who + "the volume box must lie at positive depth from the source (in front of its plane)");
    }
    return CT_OK;
}

ct_status plan_device_table(ct_plan *p, hipStream_t st, const AngleGeo **out) {
    int dev = 0;
    CT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->dtab.find(dev);
    if (it == p->dtab.end()) {
        ct_plan::DevTab t{nullptr, nullptr};
        const size_t bytes = sizeof(AngleGeo) * p->tab.size();
        CT_HIP(CT_MALLOC_ASYNC((void **)&t.ptr, bytes, st));
        hipError_t e = hipMemcpyAsync(t.ptr, p->tab.data(), bytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&t.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(t.ready, st);
        if (e != hipSuccess) {
            (void)hipFreeAsync(t.ptr, st);
            if (t.ready) (void)hipEventDestroy(t.ready);
            return hip_fail(e, "angle table upload");
        }
        it = p->dtab.emplace(dev, t).first;
    } else {
        CT_HIP(hipStreamWaitEvent(st, it->second.ready, 0));
    }
    *out = it->second.ptr;
    return CT_OK;
}

ct_status plan_device_table_existing(ct_plan *p, hipStream_t st, const AngleGeo **out) {
    int dev = 0;
    CT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->dtab.find(dev);
    if (it == p->dtab.end())
        return fail(CT_ERR_STATE, "the plan's angle table is not on this device yet: one allocating call with the plan "
                                  "on this device (e.g. ct_backproject) uploads it");
    CT_HIP(hipStreamWaitEvent(st, it->second.ready, 0));
    *out = it->second.ptr;
    return CT_OK;
}

}  // namespace ct

using namespace ct;

extern "C" {

const char *ct_last_error(void) { return g_last_error.c_str(); }

const char *ct_version(void) { return "ct-mi355x 0.1 (gfx950)"; }

ct_status ct_plan_create(const ct_geometry *geometry, const double *angles, int64_t n_angles,
                         ct_plan **out) {
    if (!geometry || !angles || !out) return fail(CT_ERR_ARG, "ct_plan_create: null pointer");
    if (n_angles <= 0) return fail(CT_ERR_ARG, "ct_plan_create: n_angles must be positive");
    ct_geometry g = *geometry;
    if (g.accuracy == 0.0) g.accuracy = 0.5;
    ct_status st = validate(g);
    if (st != CT_OK) return st;
    for (int64_t i = 0; i < n_angles; ++i)
        if (!std::isfinite(angles[i])) return fail(CT_ERR_GEOMETRY, "ct_plan_create: non-finite angle");
    ct_plan *p = new (std::nothrow) ct_plan();
    if (!p) return fail(CT_ERR_OOM, "ct_plan_create: host allocation failed");
    p->g = g;
    p->angles.assign(angles, angles + n_angles);
    p->tab.resize(n_angles);
    for (int64_t i = 0; i < n_angles; ++i) p->tab[i] = angle_geo(g, angles[i]);
    *out = p;
    return CT_OK;
}

ct_status ct_plan_create_views(const ct_geometry *geometry, const double *views, int64_t n_views, ct_plan **out) {
    if (!geometry || !views || !out) return fail(CT_ERR_ARG, "ct_plan_create_views: null pointer");
    if (n_views <= 0) return fail(CT_ERR_ARG, "ct_plan_create_views: n_views must be positive");
    ct_geometry g = *geometry;
    if (g.accuracy == 0.0) g.accuracy = 0.5;
    ct_status st = validate_grid(g);
    if (st != CT_OK) return st;
    for (int64_t i = 0; i < n_views; ++i)
        if ((st = validate_view(g, views + 12 * i, i)) != CT_OK) return st;
    ct_plan *p = new (std::nothrow) ct_plan();
    if (!p) return fail(CT_ERR_OOM, "ct_plan_create_views: host allocation failed");
    p->views = true;
    p->angles.assign((size_t)n_views, 0.0);
    p->tab.resize(n_views);
    double dso = 0.0, dsd = 0.0;
    for (int64_t i = 0; i < n_views; ++i) {
        const double *v = views + 12 * i;
        p->vertical = p->vertical && v[8] == 0.0 && v[9] == 0.0 && v[10] == 0.0 && v[11] == 1.0 && v[5] == v[2];
        p->tab[i] = view_geo(g, views + 12 * i);
        dso = std::fmax(dso, p->tab[i].DSOv);
        dsd = std::fmax(dsd, p->tab[i].DSDv);
    }
    // informative only (ct_plan_info): the largest distances over the views
    g.DSO = dso;
    g.DSD = dsd;
    p->g = g;
    *out = p;
    return CT_OK;
}

void ct_plan_destroy(ct_plan *plan) {
    if (!plan) return;
    int cur = 0;
    bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto &kv : plan->dtab) {
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        // stream-ordered release: the caller has finished all work that uses the plan
        (void)hipFreeAsync(kv.second.ptr, nullptr);
        (void)hipEventDestroy(kv.second.ready);
    }
    if (have && !plan->dtab.empty()) (void)hipSetDevice(cur);
    delete plan;
}

ct_status ct_plan_info(const ct_plan *plan, ct_geometry *geometry, int64_t *n_angles) {
    if (!plan) return fail(CT_ERR_ARG, "ct_plan_info: null plan");
    if (geometry) *geometry = plan->g;
    if (n_angles) *n_angles = (int64_t)plan->angles.size();
    return CT_OK;
}

static ct_status check_range(const ct_plan *p, int64_t a0, int64_t a1, const char *who) {
    if (a0 < 0 || a1 > (int64_t)p->angles.size() || a0 >= a1)
        return fail(CT_ERR_ARG, std::string(who) + ": angle range must satisfy 0 <= begin < end <= n_angles");
    return CT_OK;
}

ct_status ct_forward(ct_plan *plan, ct_projector projector, const void *d_vol, ct_dtype vol_dtype,
                     void *d_proj, ct_dtype proj_dtype, int accumulate, int64_t angle_begin,
                     int64_t angle_end, void *stream) {
    if (!plan || !d_vol || !d_proj) return fail(CT_ERR_ARG, "ct_forward: null pointer");
    if (projector != CT_SIDDON && projector != CT_INTERP) return fail(CT_ERR_ARG, "ct_forward: unknown projector");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_forward: dtype must be CT_F32, CT_F16 or CT_BF16");
    ct_status st = check_range(plan, angle_begin, angle_end, "ct_forward");
    if (st != CT_OK) return st;
    return launch_forward(plan, projector, d_vol, vol_dtype, d_proj, proj_dtype, accumulate, angle_begin,
                          angle_end, full_slab(plan->g), (hipStream_t)stream);
}

ct_status ct_backproject(ct_plan *plan, ct_backprojector backprojector, const void *d_proj,
                         ct_dtype proj_dtype, void *d_vol, ct_dtype vol_dtype, int accumulate,
                         int64_t angle_begin, int64_t angle_end, void *stream) {
    if (!plan || !d_vol || !d_proj) return fail(CT_ERR_ARG, "ct_backproject: null pointer");
    if (backprojector != CT_BP_FDK && backprojector != CT_BP_PSEUDO_MATCHED && backprojector != CT_BP_ADJOINT)
        return fail(CT_ERR_ARG, "ct_backproject: unknown backprojector");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_backproject: dtype must be CT_F32, CT_F16 or CT_BF16");
    ct_status st = check_range(plan, angle_begin, angle_end, "ct_backproject");
    if (st != CT_OK) return st;
    return launch_backproject(plan, backprojector, d_proj, proj_dtype, d_vol, vol_dtype, accumulate,
                              angle_begin, angle_end, full_slab(plan->g), (hipStream_t)stream);
}

ct_status ct_backproject_noalloc(ct_plan *plan, ct_backprojector backprojector, const void *d_proj,
                                 ct_dtype proj_dtype, void *d_vol, ct_dtype vol_dtype, int accumulate,
                                 int64_t angle_begin, int64_t angle_end, void *stream) {
    if (!plan || !d_vol || !d_proj) return fail(CT_ERR_ARG, "ct_backproject_noalloc: null pointer");
    if (backprojector != CT_BP_FDK && backprojector != CT_BP_PSEUDO_MATCHED && backprojector != CT_BP_ADJOINT)
        return fail(CT_ERR_ARG, "ct_backproject_noalloc: unknown backprojector");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype))
        return fail(CT_ERR_DTYPE, "ct_backproject_noalloc: dtype must be CT_F32, CT_F16 or CT_BF16");
    ct_status st = check_range(plan, angle_begin, angle_end, "ct_backproject_noalloc");
    if (st != CT_OK) return st;
    return backproject_noalloc(plan, backprojector, d_proj, proj_dtype, d_vol, vol_dtype, accumulate, angle_begin,
                               angle_end, (hipStream_t)stream);
}

ct_status ct_ooc_plan(const ct_plan *plan, int direction, ct_projector projector, ct_dtype vol_dtype,
                      ct_dtype proj_dtype, uint64_t device_cap_bytes, ct_ooc_stats *out) {
    if (!plan || !out) return fail(CT_ERR_ARG, "ct_ooc_plan: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_ooc_plan: needs a circular orbit (not a plan of views)");
    if (direction < 0 || direction > 3) return fail(CT_ERR_ARG, "ct_ooc_plan: direction must be 0, 1, 2 or 3");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_ooc_plan: dtype must be CT_F32, CT_F16 or CT_BF16");
    return ooc_plan(plan, direction, projector, vol_dtype, proj_dtype, device_cap_bytes, out);
}

ct_status ct_forward_host(ct_plan *plan, ct_projector projector, const void *h_vol, ct_dtype vol_dtype,
                          void *h_proj, ct_dtype proj_dtype, uint64_t device_cap_bytes,
                          ct_ooc_stats *stats) {
    if (!plan || !h_vol || !h_proj) return fail(CT_ERR_ARG, "ct_forward_host: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_forward_host: needs a circular orbit (not a plan of views)");
    if (projector != CT_SIDDON && projector != CT_INTERP) return fail(CT_ERR_ARG, "ct_forward_host: unknown projector");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_forward_host: dtype must be CT_F32, CT_F16 or CT_BF16");
    return ooc_forward(plan, projector, h_vol, vol_dtype, h_proj, proj_dtype, device_cap_bytes, stats);
}

ct_status ct_backproject_host(ct_plan *plan, ct_backprojector backprojector, const void *h_proj,
                              ct_dtype proj_dtype, void *h_vol, ct_dtype vol_dtype,
                              uint64_t device_cap_bytes, ct_ooc_stats *stats) {
    if (!plan || !h_vol || !h_proj) return fail(CT_ERR_ARG, "ct_backproject_host: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_backproject_host: needs a circular orbit (not a plan of views)");
    if (backprojector != CT_BP_FDK && backprojector != CT_BP_PSEUDO_MATCHED && backprojector != CT_BP_ADJOINT)
        return fail(CT_ERR_ARG, "ct_backproject_host: unknown backprojector");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_backproject_host: dtype must be CT_F32, CT_F16 or CT_BF16");
    return ooc_backproject(plan, backprojector, h_proj, proj_dtype, h_vol, vol_dtype, device_cap_bytes, stats);
}

ct_status ct_cgls_workspace_bytes(const ct_plan *plan, ct_dtype vol_dtype, ct_dtype proj_dtype,
                                  uint64_t *bytes) {
    if (!plan || !bytes) return fail(CT_ERR_ARG, "ct_cgls_workspace_bytes: null pointer");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_cgls_workspace_bytes: dtype must be CT_F32, CT_F16 or CT_BF16");
    *bytes = cgls_workspace(plan, vol_dtype, proj_dtype);
    return CT_OK;
}

ct_status ct_cgls(ct_plan *plan, const void *d_b, ct_dtype proj_dtype, void *d_x, ct_dtype vol_dtype,
                  int32_t niter, double *d_resid, void *d_workspace, void *stream) {
    if (!plan || !d_b || !d_x) return fail(CT_ERR_ARG, "ct_cgls: null pointer");
    if (niter < 0) return fail(CT_ERR_ARG, "ct_cgls: niter must be >= 0");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_cgls: dtype must be CT_F32, CT_F16 or CT_BF16");
    return cgls_run(plan, d_b, proj_dtype, d_x, vol_dtype, niter, d_resid, d_workspace, (hipStream_t)stream);
}

ct_status ct_cgls_host_workspace_bytes(const ct_plan *plan, uint64_t *bytes) {
    if (!plan || !bytes) return fail(CT_ERR_ARG, "ct_cgls_host_workspace_bytes: null pointer");
    *bytes = cgls_host_workspace(plan);
    return CT_OK;
}

ct_status ct_cgls_host(ct_plan *plan, const float *h_b, float *h_x, int32_t niter, double *resid, void *h_workspace,
                       uint64_t device_cap_bytes, ct_ooc_stats *stats) {
    if (!plan || !h_b || !h_x || !h_workspace) return fail(CT_ERR_ARG, "ct_cgls_host: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_cgls_host: needs a circular orbit (not a plan of views)");
    if (niter < 0) return fail(CT_ERR_ARG, "ct_cgls_host: niter must be >= 0");
    return cgls_host_run(plan, h_b, h_x, niter, resid, h_workspace, device_cap_bytes, stats);
}

ct_status ct_sart_workspace_bytes(const ct_plan *plan, int32_t block, uint64_t *bytes) {
    if (!plan || !bytes) return fail(CT_ERR_ARG, "ct_sart_workspace_bytes: null pointer");
    if (block < 1 || block > (int64_t)plan->angles.size())
        return fail(CT_ERR_ARG, "ct_sart_workspace_bytes: block must be in [1, n_angles]");
    *bytes = sart_workspace(plan, block);
    return CT_OK;
}

ct_status ct_sart(ct_plan *plan, const void *d_b, ct_dtype proj_dtype, void *d_x, ct_dtype vol_dtype, int32_t niter,
                  double lambda, int32_t block, void *d_workspace, void *stream) {
    if (!plan || !d_b || !d_x) return fail(CT_ERR_ARG, "ct_sart: null pointer");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_sart: unsupported dtype");
    if (niter < 0) return fail(CT_ERR_ARG, "ct_sart: niter must be >= 0");
    if (block < 1 || block > (int64_t)plan->angles.size())
        return fail(CT_ERR_ARG, "ct_sart: block must be in [1, n_angles]");
    if (!std::isfinite(lambda)) return fail(CT_ERR_ARG, "ct_sart: lambda must be finite");
    return sart_run(plan, d_b, proj_dtype, d_x, vol_dtype, niter, lambda, block, d_workspace, (hipStream_t)stream);
}

ct_status ct_fdk_filter(ct_plan *plan, const void *d_proj, ct_dtype proj_dtype, float *d_q, int64_t angle_begin,
                        int64_t angle_end, void *stream) {
    if (!plan || !d_proj || !d_q) return fail(CT_ERR_ARG, "ct_fdk_filter: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_fdk_filter: needs a circular orbit (not a plan of views)");
    if (!dtype_ok(proj_dtype)) return fail(CT_ERR_DTYPE, "ct_fdk_filter: dtype must be CT_F32, CT_F16 or CT_BF16");
    ct_status st = check_range(plan, angle_begin, angle_end, "ct_fdk_filter");
    if (st != CT_OK) return st;
    return fdk_filter(plan, d_proj, proj_dtype, d_q, angle_begin, angle_end, (hipStream_t)stream);
}

ct_status ct_fdk_host(ct_plan *plan, const void *h_proj, ct_dtype proj_dtype, void *h_vol, ct_dtype vol_dtype,
                      uint64_t device_cap_bytes, ct_ooc_stats *stats) {
    if (!plan || !h_proj || !h_vol) return fail(CT_ERR_ARG, "ct_fdk_host: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_fdk_host: needs a circular orbit (not a plan of views)");
    if (!dtype_ok(proj_dtype) || !dtype_ok(vol_dtype)) return fail(CT_ERR_DTYPE, "ct_fdk_host: dtype must be CT_F32, CT_F16 or CT_BF16");
    if (plan->g.nDetector[0] > 4096)
        return fail(CT_ERR_ARG, "ct_fdk_host: detector rows longer than 4096 pixels are not supported");
    return ooc_backproject(plan, CT_BP_FDK, h_proj, proj_dtype, h_vol, vol_dtype, device_cap_bytes, stats, true);
}

ct_status ct_fdk_workspace_bytes(const ct_plan *plan, uint64_t *bytes) {
    if (!plan || !bytes) return fail(CT_ERR_ARG, "ct_fdk_workspace_bytes: null pointer");
    *bytes = fdk_workspace(plan);
    return CT_OK;
}

ct_status ct_fdk(ct_plan *plan, const void *d_proj, ct_dtype proj_dtype, void *d_vol, ct_dtype vol_dtype,
                 void *d_workspace, void *stream) {
    if (!plan || !d_proj || !d_vol) return fail(CT_ERR_ARG, "ct_fdk: null pointer");
    if (plan->views) return fail(CT_ERR_ARG, "ct_fdk: needs a circular orbit (not a plan of views)");
    if (!dtype_ok(proj_dtype) || !dtype_ok(vol_dtype)) return fail(CT_ERR_DTYPE, "ct_fdk: dtype must be CT_F32, CT_F16 or CT_BF16");
    return fdk_run(plan, d_proj, proj_dtype, d_vol, vol_dtype, d_workspace, (hipStream_t)stream);
}

ct_status ct_tv_workspace_bytes(const ct_geometry *geometry, ct_dtype dtype, uint64_t *bytes) {
    if (!geometry || !bytes) return fail(CT_ERR_ARG, "ct_tv_workspace_bytes: null pointer");
    if (!dtype_ok(dtype)) return fail(CT_ERR_DTYPE, "ct_tv_workspace_bytes: unsupported dtype");
    *bytes = tv_workspace(*geometry, dtype);
    return CT_OK;
}

ct_status ct_tv_steps(const ct_geometry *geometry, void *d_x, ct_dtype dtype, int32_t nsteps, double lambda, double eps,
                      void *d_workspace, void *stream) {
    if (!geometry || !d_x) return fail(CT_ERR_ARG, "ct_tv_steps: null pointer");
    if (!dtype_ok(dtype)) return fail(CT_ERR_DTYPE, "ct_tv_steps: unsupported dtype");
    if (nsteps < 0) return fail(CT_ERR_ARG, "ct_tv_steps: nsteps must be >= 0");
    if (!(eps > 0) || !std::isfinite(lambda)) return fail(CT_ERR_ARG, "ct_tv_steps: need eps > 0 and finite lambda");
    for (int a = 0; a < 3; ++a)
        if (geometry->nVoxel[a] <= 0) return fail(CT_ERR_GEOMETRY, "ct_tv_steps: voxel counts must be positive");
    return tv_run(*geometry, d_x, dtype, nsteps, lambda, eps, d_workspace, (hipStream_t)stream);
}

ct_status ct_tv_steps_host(const ct_geometry *geometry, float *h_x, int32_t nsteps, double lambda, double eps,
                           int32_t halo_depth, uint64_t device_cap_bytes, ct_ooc_stats *stats) {
    if (!geometry || !h_x) return fail(CT_ERR_ARG, "ct_tv_steps_host: null pointer");
    if (nsteps < 0) return fail(CT_ERR_ARG, "ct_tv_steps_host: nsteps must be >= 0");
    if (halo_depth < 0 || halo_depth > 4096) return fail(CT_ERR_ARG, "ct_tv_steps_host: halo_depth must be in [0, 4096]");
    if (!(eps > 0) || !std::isfinite(lambda)) return fail(CT_ERR_ARG, "ct_tv_steps_host: need eps > 0 and finite lambda");
    for (int a = 0; a < 3; ++a)
        if (geometry->nVoxel[a] <= 0) return fail(CT_ERR_GEOMETRY, "ct_tv_steps_host: voxel counts must be positive");
    return tv_host_run(*geometry, h_x, nsteps, lambda, eps, halo_depth, device_cap_bytes, stats);
}

ct_status ct_rof_workspace_bytes(const ct_geometry *geometry, uint64_t *bytes) {
    if (!geometry || !bytes) return fail(CT_ERR_ARG, "ct_rof_workspace_bytes: null pointer");
    *bytes = rof_workspace(*geometry);
    return CT_OK;
}

ct_status ct_rof(const ct_geometry *geometry, void *d_x, int32_t niter, double lambda, double tau, void *d_workspace,
                 void *stream) {
    if (!geometry || !d_x) return fail(CT_ERR_ARG, "ct_rof: null pointer");
    if (niter < 0) return fail(CT_ERR_ARG, "ct_rof: niter must be >= 0");
    if (!(lambda > 0) || !std::isfinite(lambda) || !(tau > 0) || !std::isfinite(tau))
        return fail(CT_ERR_ARG, "ct_rof: need finite lambda > 0 and tau > 0");
    for (int a = 0; a < 3; ++a)
        if (geometry->nVoxel[a] <= 0) return fail(CT_ERR_GEOMETRY, "ct_rof: voxel counts must be positive");
    if (geometry->nVoxel[2] > 65535) return fail(CT_ERR_ARG, "ct_rof: more than 65535 slices");
    return rof_run(*geometry, d_x, niter, lambda, tau, d_workspace, (hipStream_t)stream);
}

ct_status ct_rof_host_workspace_bytes(const ct_geometry *geometry, uint64_t *bytes) {
    if (!geometry || !bytes) return fail(CT_ERR_ARG, "ct_rof_host_workspace_bytes: null pointer");
    *bytes = rof_host_workspace(*geometry);
    return CT_OK;
}

ct_status ct_rof_host(const ct_geometry *geometry, float *h_x, int32_t niter, double lambda, double tau,
                      int32_t halo_depth, void *h_workspace, uint64_t device_cap_bytes, ct_ooc_stats *stats) {
    if (!geometry || !h_x || !h_workspace) return fail(CT_ERR_ARG, "ct_rof_host: null pointer");
    if (niter < 0) return fail(CT_ERR_ARG, "ct_rof_host: niter must be >= 0");
    if (!(lambda > 0) || !std::isfinite(lambda) || !(tau > 0) || !std::isfinite(tau))
        return fail(CT_ERR_ARG, "ct_rof_host: need finite lambda > 0 and tau > 0");
    if (halo_depth < 1 || halo_depth > 4096) return fail(CT_ERR_ARG, "ct_rof_host: halo_depth must be in [1, 4096]");
    for (int a = 0; a < 3; ++a)
        if (geometry->nVoxel[a] <= 0) return fail(CT_ERR_GEOMETRY, "ct_rof_host: voxel counts must be positive");
    return rof_host_run(*geometry, h_x, niter, lambda, tau, halo_depth, (float *)h_workspace, device_cap_bytes, stats);
}

ct_status ct_dot(const void *d_a, const void *d_b, ct_dtype dtype, int64_t n, double *d_out, void *stream) {
    if (!d_a || !d_b || !d_out) return fail(CT_ERR_ARG, "ct_dot: null pointer");
    if (n < 0) return fail(CT_ERR_ARG, "ct_dot: negative length");
    if (!dtype_ok_any(dtype)) return fail(CT_ERR_DTYPE, "ct_dot: unknown dtype");
    return dot_f64(d_a, d_b, dtype, n, d_out, nullptr, (hipStream_t)stream);
}

ct_status ct_convert(const void *d_src, ct_dtype src_dtype, void *d_dst, ct_dtype dst_dtype, int64_t n,
                     void *stream) {
    if (!d_src || !d_dst) return fail(CT_ERR_ARG, "ct_convert: null pointer");
    if (n < 0) return fail(CT_ERR_ARG, "ct_convert: negative length");
    if (!dtype_ok_any(src_dtype) || !dtype_ok_any(dst_dtype)) return fail(CT_ERR_DTYPE, "ct_convert: unknown dtype");
    return convert(d_src, src_dtype, d_dst, dst_dtype, n, (hipStream_t)stream);
}

}  // extern "C"
