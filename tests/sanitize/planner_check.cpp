// Host-side checks of the library's planner and validation under AddressSanitizer and
// UndefinedBehaviorSanitizer (built without device code; nothing here touches a GPU): geometry and
// per-view validation on valid and invalid inputs, plan info, and the out-of-core planner over every
// direction, storage type and a sweep of caps from below one slice to beyond the volume.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#include "ct.h"

static int failures = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static ct_geometry geo(int64_t nx, int64_t ny, int64_t nz, int64_t nu, int64_t nv) {
    ct_geometry g;
    std::memset(&g, 0, sizeof(g));
    g.DSO = 1000.0;
    g.DSD = 1500.0;
    g.nVoxel[0] = nx;
    g.nVoxel[1] = ny;
    g.nVoxel[2] = nz;
    const int64_t nmax = std::max(nx, std::max(ny, nz));
    for (int a = 0; a < 3; ++a) g.dVoxel[a] = 256.0 / (double)nmax;
    g.nDetector[0] = nu;
    g.nDetector[1] = nv;
    g.dDetector[0] = g.dDetector[1] = 409.6 / (double)std::max<int64_t>(nu, 1);
    g.accuracy = 0.5;
    return g;
}

static std::vector<double> angles(int n) {
    std::vector<double> a(n);
    for (int i = 0; i < n; ++i) a[i] = 2.0 * M_PI * i / n;
    return a;
}

// circular views of the same angles, with a tilt of the detector about e_u when tilt != 0
static std::vector<double> views(const ct_geometry &g, int n, double tilt, double rise) {
    std::vector<double> v(12 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const double t = 2.0 * M_PI * i / n, c = std::cos(t), s = std::sin(t);
        double *w = &v[12 * (size_t)i];
        const double eu[3] = {-s, c, 0.0};
        const double ev[3] = {std::sin(tilt) * c, std::sin(tilt) * s, std::cos(tilt)};
        const double S[3] = {g.DSO * c, g.DSO * s, rise * i}, C[3] = {-(g.DSD - g.DSO) * c, -(g.DSD - g.DSO) * s, rise * i};
        for (int a = 0; a < 3; ++a) {
            w[a] = S[a];
            w[3 + a] = C[a];
            w[6 + a] = eu[a];
            w[9 + a] = ev[a];
        }
    }
    return v;
}

int main() {
    const ct_dtype dts[3] = {CT_F32, CT_F16, CT_BF16};
    const int64_t sizes[][5] = {{1, 1, 1, 1, 1}, {7, 5, 3, 9, 4}, {64, 64, 64, 64, 64}, {256, 256, 300, 300, 200},
                                {3072, 3072, 3072, 3072, 3072}, {1, 4096, 17, 4096, 1}};
    for (const auto &sz : sizes) {
        ct_geometry g = geo(sz[0], sz[1], sz[2], sz[3], sz[4]);
        const int na = sz[0] > 1000 ? 3072 : 37;
        std::vector<double> a = angles(na);
        ct_plan *p = nullptr;
        CHECK(ct_plan_create(&g, a.data(), na, &p) == CT_OK && p);
        if (!p) continue;
        ct_geometry gi;
        int64_t n = 0;
        CHECK(ct_plan_info(p, &gi, &n) == CT_OK && n == na && gi.nVoxel[2] == sz[2]);
        const double vol = (double)sz[0] * sz[1] * sz[2] * 4.0;
        for (int dir = 0; dir < 4; ++dir)
            for (ct_projector pr : {CT_SIDDON, CT_INTERP})
                for (ct_dtype vt : dts)
                    for (ct_dtype pt : dts) {
                        for (double f = 1e-6; f < 4.0; f *= 1.7) {
                            const uint64_t cap = (uint64_t)(vol * f) + (64ull << 20);
                            ct_ooc_stats st;
                            const ct_status s = ct_ooc_plan(p, dir, pr, vt, pt, cap, &st);
                            if (s == CT_OK) {
                                CHECK(st.n_slabs >= 1 && st.slab_slices >= 1 && st.chunk_angles >= 1);
                                CHECK((int64_t)st.n_slabs * st.slab_slices >= sz[2]);
                                CHECK((int64_t)(st.n_slabs - 1) * st.slab_slices < sz[2]);
                                CHECK(st.n_chunks == (na + st.chunk_angles - 1) / st.chunk_angles);
                            } else {
                                CHECK(s == CT_ERR_CAP && std::strlen(ct_last_error()) > 0);
                            }
                        }
                    }
        ct_ooc_stats st;
        CHECK(ct_ooc_plan(p, 5, CT_SIDDON, CT_F32, CT_F32, 1ull << 30, &st) == CT_ERR_ARG);
        CHECK(ct_ooc_plan(p, 0, CT_SIDDON, CT_F64, CT_F32, 1ull << 30, &st) == CT_ERR_DTYPE);
        ct_plan_destroy(p);
        if (sz[0] > 1000) continue;
        // plans of views: valid tables, helical rises, tilted detectors, and invalid ones
        for (double tilt : {0.0, 0.2}) {
            std::vector<double> v = views(g, na, tilt, 0.7);
            CHECK(ct_plan_create_views(&g, v.data(), na, &p) == CT_OK);
            CHECK(ct_plan_info(p, &gi, &n) == CT_OK && n == na);
            CHECK(ct_ooc_plan(p, 0, CT_SIDDON, CT_F32, CT_F32, 1ull << 30, &st) == CT_ERR_ARG);
            ct_plan_destroy(p);
            v[12 + 7] *= 1.5;                              // e_u of view 1 no longer a unit vector
            CHECK(ct_plan_create_views(&g, v.data(), na, &p) == CT_ERR_GEOMETRY);
            v[12 + 7] /= 1.5;
            v[12 * 2 + 9] += 0.01;                         // e_v of view 2 no longer orthogonal to e_u
            CHECK(ct_plan_create_views(&g, v.data(), na, &p) == CT_ERR_GEOMETRY);
            v[12 * 2 + 9] -= 0.01;
            for (int a = 0; a < 3; ++a) std::swap(v[6 + a], v[9 + a]);  // normal turned away from the source
            CHECK(ct_plan_create_views(&g, v.data(), na, &p) == CT_ERR_GEOMETRY);
            for (int a = 0; a < 3; ++a) std::swap(v[6 + a], v[9 + a]);
            v[12 * (na - 1) + 4] = NAN;                    // a non-finite entry
            CHECK(ct_plan_create_views(&g, v.data(), na, &p) == CT_ERR_GEOMETRY);
        }
    }
    // invalid circular geometries and arguments
    ct_geometry g = geo(16, 16, 16, 16, 16);
    std::vector<double> a = angles(4);
    ct_plan *p = nullptr;
    g.DSD = 500.0;
    CHECK(ct_plan_create(&g, a.data(), 4, &p) == CT_ERR_GEOMETRY);
    g = geo(16, 16, 16, 16, 16);
    g.nVoxel[1] = 0;
    CHECK(ct_plan_create(&g, a.data(), 4, &p) == CT_ERR_GEOMETRY);
    g = geo(16, 16, 16, 16, 16);
    g.offOrigin[0] = 2000.0;
    CHECK(ct_plan_create(&g, a.data(), 4, &p) == CT_ERR_GEOMETRY);
    g = geo(16, 16, 16, 16, 16);
    g.nVoxel[2] = (1 << 24) + 1;
    CHECK(ct_plan_create(&g, a.data(), 4, &p) == CT_ERR_GEOMETRY);
    g = geo(16, 16, 16, 16, 16);
    CHECK(ct_plan_create(&g, a.data(), 0, &p) == CT_ERR_ARG);
    CHECK(ct_plan_create(nullptr, a.data(), 4, &p) == CT_ERR_ARG);
    CHECK(ct_plan_create_views(&g, nullptr, 4, &p) == CT_ERR_ARG);
    a[2] = INFINITY;
    CHECK(ct_plan_create(&g, a.data(), 4, &p) == CT_ERR_GEOMETRY);
    ct_plan_destroy(nullptr);
    std::printf("planner check: %d failures\n", failures);
    return failures ? 1 : 0;
}
