/*
 * CPU FP64 oracle for the cone-beam projection operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline leg may load this library.  It shares no code with the GPU path: no headers, no tables,
 * no helpers.  Everything here is deliberately plain: one ray or one voxel at a time, in double
 * precision, following the definitions step by step; OpenMP only splits independent rays/voxels.
 *
 * Conventions (the paper gives the scanner distances but no coordinate system, so these are our
 * readings, shared with the GPU path only through this written description):
 *   mm, radians; voxel (i,j,k) centre at offOrigin + ((i-(Nx-1)/2)dx, ...); volume layout
 *   vol[k][j][i], projection layout proj[view][b][a]; one ray per pixel centre.
 *   Every operator takes one view per projection: source S, detector centre C and the detector's
 *   unit axes e_u, e_v (orthonormal), 12 doubles.  Pixel (a,b) has its centre at
 *   C + u_a e_u + v_b e_v with u_a = (a-(Nu-1)/2) du + offU, v_b = (b-(Nv-1)/2) dv + offV.
 *   The circular orbit about z (orc_circular_views) is the view of angle t:
 *   S = DSO (cos t, sin t, 0), C = -(DSD-DSO)(cos t, sin t, 0), e_u = (-sin t, cos t, 0),
 *   e_v = (0,0,1).  Per-view tables also describe C-arm and helical scans (Section 2.1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double DSO, DSD;
    int64_t nvox[3];
    double dvox[3];
    double offorig[3];
    int64_t ndet[2];
    double ddet[2];
    double offdet[2];
    double accuracy;
} orc_geom;

enum { ORC_W_FDK = 0, ORC_W_PM = 1 };

/* ------------------------------------------------------------------------------------------ */
/* geometry                                                                                     */

typedef struct {
    double S[3], C[3], eu[3], ev[3];
} orc_view;

static const orc_view *view_at(const double *views, int64_t t) { return (const orc_view *)(views + 12 * t); }

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* The views of a circular orbit at the given angles (conventions above). */
void orc_circular_views(const orc_geom *g, const double *angles, int64_t na, double *views) {
    for (int64_t t = 0; t < na; ++t) {
        double c = cos(angles[t]), s = sin(angles[t]);
        double k = -(g->DSD - g->DSO);
        double *v = views + 12 * t;
        v[0] = g->DSO * c; v[1] = g->DSO * s; v[2] = 0.0;
        v[3] = k * c;      v[4] = k * s;      v[5] = 0.0;
        v[6] = -s;         v[7] = c;          v[8] = 0.0;
        v[9] = 0.0;        v[10] = 0.0;       v[11] = 1.0;
    }
}

static void source_pos(const orc_view *v, double S[3]) {
    for (int a = 0; a < 3; ++a) S[a] = v->S[a];
}

static void pixel_pos(const orc_geom *g, const orc_view *v, double a, double b, double P[3]) {
    double u = (a - (g->ndet[0] - 1) / 2.0) * g->ddet[0] + g->offdet[0];
    double w = (b - (g->ndet[1] - 1) / 2.0) * g->ddet[1] + g->offdet[1];
    for (int x = 0; x < 3; ++x) P[x] = v->C[x] + u * v->eu[x] + w * v->ev[x];
}

static void box_bounds(const orc_geom *g, double lo[3], double hi[3]) {
    for (int a = 0; a < 3; ++a) {
        lo[a] = g->offorig[a] - g->nvox[a] * g->dvox[a] / 2.0;
        hi[a] = g->offorig[a] + g->nvox[a] * g->dvox[a] / 2.0;
    }
}

void orc_ray_endpoints(const orc_geom *g, const double *view, double a, double b, double *S, double *P) {
    source_pos((const orc_view *)view, S);
    pixel_pos(g, (const orc_view *)view, a, b, P);
}

/* Slab clip of R(t) = S + t D, t in [0,1], against [lo,hi]; axes with |D_a| < 1e-12 L are
 * parallel.  Returns 0 when the ray misses the box. */
static int clip_unit(const double S[3], const double D[3], double L, const double lo[3],
                     const double hi[3], double *tin, double *tout) {
    double t0 = 0.0, t1 = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (fabs(D[a]) < 1e-12 * L) {
            if (S[a] < lo[a] || S[a] > hi[a]) return 0;
        } else {
            double ta = (lo[a] - S[a]) / D[a], tb = (hi[a] - S[a]) / D[a];
            if (ta > tb) { double x = ta; ta = tb; tb = x; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        }
    }
    *tin = t0;
    *tout = t1;
    return t0 < t1;
}

/* ------------------------------------------------------------------------------------------ */
/* Siddon's exact radiological path (Siddon 1985, cited in Section 2.1): the ray is cut at every
 * voxel-plane crossing inside the box; each piece lies in one voxel, found from its midpoint, and
 * contributes (piece length) x (voxel value).  `mode` 0 gathers from vol; 1 scatters y*len into
 * vol; 2 returns the length inside voxel `target` only. */

typedef struct {
    double *buf; /* 3 sorted crossing lists + merged list */
    int64_t cap;
} scratch_t;

static void scratch_init(scratch_t *s, const orc_geom *g) {
    s->cap = g->nvox[0] + g->nvox[1] + g->nvox[2] + 8;
    s->buf = (double *)malloc(sizeof(double) * 2 * s->cap);
}

static double siddon_core(const orc_geom *g, const double S[3], const double P[3], const double *vol,
                          const float *volf, double *scat, double y, int64_t target, int64_t *nseg,
                          scratch_t *sc) {
    double lo[3], hi[3], D[3];
    box_bounds(g, lo, hi);
    for (int a = 0; a < 3; ++a) D[a] = P[a] - S[a];
    double L = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    double tin, tout;
    if (!clip_unit(S, D, L, lo, hi, &tin, &tout)) {
        if (nseg) *nseg = 0;
        return 0.0;
    }
    /* crossing parameters per axis, each list ascending in t */
    double *lists = sc->buf;
    double *merged = sc->buf + sc->cap;
    int64_t start[3], cnt[3], off = 0;
    for (int a = 0; a < 3; ++a) {
        start[a] = off;
        cnt[a] = 0;
        if (fabs(D[a]) < 1e-12 * L) continue;
        int64_t n = g->nvox[a];
        for (int64_t m = 0; m <= n; ++m) {
            int64_t mm = D[a] > 0 ? m : n - m;
            double t = (lo[a] + mm * g->dvox[a] - S[a]) / D[a];
            if (t > tin && t < tout) lists[off + cnt[a]++] = t;
        }
        off += cnt[a];
    }
    /* three-way merge */
    int64_t p[3] = {0, 0, 0}, nm = 0;
    merged[nm++] = tin;
    for (;;) {
        int best = -1;
        double bt = 0.0;
        for (int a = 0; a < 3; ++a)
            if (p[a] < cnt[a]) {
                double t = lists[start[a] + p[a]];
                if (best < 0 || t < bt) { best = a; bt = t; }
            }
        if (best < 0) break;
        merged[nm++] = bt;
        p[best]++;
    }
    merged[nm++] = tout;

    double acc = 0.0;
    int64_t segs = 0;
    const int64_t nx = g->nvox[0], ny = g->nvox[1], nz = g->nvox[2];
    for (int64_t q = 0; q + 1 < nm; ++q) {
        double ta = merged[q], tb = merged[q + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        int64_t idx[3];
        for (int a = 0; a < 3; ++a) {
            double x = S[a] + tm * D[a];
            int64_t i = (int64_t)floor((x - lo[a]) / g->dvox[a]);
            if (i < 0) i = 0;
            if (i > g->nvox[a] - 1) i = g->nvox[a] - 1;
            idx[a] = i;
        }
        int64_t lin = (idx[2] * ny + idx[1]) * nx + idx[0];
        double len = L * (tb - ta);
        segs++;
        if (vol) acc += len * vol[lin];
        if (volf) acc += len * (double)volf[lin];
        if (scat) scat[lin] += y * len;
        if (target >= 0 && lin == target) acc += len;
    }
    (void)nz;
    if (nseg) *nseg = segs;
    return acc;
}

/* ------------------------------------------------------------------------------------------ */
/* Interpolated projector (Chou 2011, cited in Section 2.1): the volume is read through its
 * trilinear interpolant x~ (voxel centres as nodes, zero outside the grid, so x~ vanishes outside
 * the box grown by half a voxel); samples at s_k = (k + 1/2) Delta from the source along the unit
 * direction, every k with s_in <= s_k <= s_out inside the grown box; p = Delta * sum x~(samples),
 * Delta = accuracy * min voxel size. */

static double vol_at(const orc_geom *g, const double *vol, int64_t i, int64_t j, int64_t k) {
    if (i < 0 || j < 0 || k < 0 || i >= g->nvox[0] || j >= g->nvox[1] || k >= g->nvox[2]) return 0.0;
    return vol[(k * g->nvox[1] + j) * g->nvox[0] + i];
}

static double trilinear(const orc_geom *g, const double *vol, const double X[3]) {
    double f[3];
    int64_t i0[3];
    for (int a = 0; a < 3; ++a) {
        double c = (X[a] - g->offorig[a]) / g->dvox[a] + (g->nvox[a] - 1) / 2.0;
        double fl = floor(c);
        i0[a] = (int64_t)fl;
        f[a] = c - fl;
    }
    double s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                double w = (di ? f[0] : 1 - f[0]) * (dj ? f[1] : 1 - f[1]) * (dk ? f[2] : 1 - f[2]);
                s += w * vol_at(g, vol, i0[0] + di, i0[1] + dj, i0[2] + dk);
            }
    return s;
}

static double interp_ray(const orc_geom *g, const double S[3], const double P[3], const double *vol,
                         int64_t *nsamp) {
    double lo[3], hi[3], D[3];
    box_bounds(g, lo, hi);
    for (int a = 0; a < 3; ++a) {
        lo[a] -= g->dvox[a] / 2.0;
        hi[a] += g->dvox[a] / 2.0;
        D[a] = P[a] - S[a];
    }
    double L = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    double tin, tout;
    if (nsamp) *nsamp = 0;
    if (!clip_unit(S, D, L, lo, hi, &tin, &tout)) return 0.0;
    double dmin = g->dvox[0];
    if (g->dvox[1] < dmin) dmin = g->dvox[1];
    if (g->dvox[2] < dmin) dmin = g->dvox[2];
    double delta = g->accuracy * dmin;
    double sin_ = tin * L, sout = tout * L;
    int64_t k0 = (int64_t)ceil(sin_ / delta - 0.5);
    int64_t k1 = (int64_t)floor(sout / delta - 0.5);
    double acc = 0.0;
    for (int64_t k = k0; k <= k1; ++k) {
        double s = (k + 0.5) * delta;
        double X[3];
        for (int a = 0; a < 3; ++a) X[a] = S[a] + s * D[a] / L;
        acc += trilinear(g, vol, X);
    }
    if (nsamp && k1 >= k0) *nsamp = k1 - k0 + 1;
    return delta * acc;
}

/* ------------------------------------------------------------------------------------------ */
/* Voxel-driven backprojection (Section 2.2): each voxel centre is projected from the source onto
 * the detector, the projection is read there by bilinear interpolation (pixels outside the
 * detector count as zero) and weighted.  FDK weight (DSO/L)^2 with L the voxel depth along the
 * central ray; pseudo-matched weight (dx dy dz)/(du dv) * DSD^2 |SX| / L^3, the ray-tube density
 * that makes the sum approximate the transpose of the ray-driven projector. */

static double proj_at(const orc_geom *g, const double *pr, const float *prf, int64_t a, int64_t b) {
    if (a < 0 || b < 0 || a >= g->ndet[0] || b >= g->ndet[1]) return 0.0;
    return pr ? pr[b * g->ndet[0] + a] : (double)prf[b * g->ndet[0] + a];
}

static void voxel_centre(const orc_geom *g, int64_t i, int64_t j, int64_t k, double X[3]) {
    int64_t id[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) X[a] = g->offorig[a] + (id[a] - (g->nvox[a] - 1) / 2.0) * g->dvox[a];
}

/* Continuous detector indices (a*, b*) and the weight of voxel X in view v.  The detector normal
 * n = e_u x e_v points from the detector towards the source; L = (S - X).n is the voxel's depth
 * from the source, DSD_v = (S - C).n the source's distance to the detector plane, and the ray from
 * S through X meets that plane at S + (DSD_v / L)(X - S).  FDK weight (DSO_v / L)^2 with
 * DSO_v = S.n, the source's distance to the plane through the origin parallel to the detector
 * (the rotation axis's distance, DSO, in a circular orbit); pseudo-matched weight
 * (dx dy dz)/(du dv) DSD_v^2 |SX| / L^3. */
static void project_voxel(const orc_geom *g, const orc_view *v, const double X[3], int kind, double *as,
                          double *bs, double *w) {
    double n[3], SX[3], SC[3], P[3];
    cross3(v->eu, v->ev, n);
    for (int a = 0; a < 3; ++a) {
        SX[a] = X[a] - v->S[a];
        SC[a] = v->C[a] - v->S[a];
    }
    double Ld = -dot3(SX, n);
    double DSDv = -dot3(SC, n);
    double m = DSDv / Ld;
    for (int a = 0; a < 3; ++a) P[a] = v->S[a] + m * SX[a] - v->C[a];
    double us = dot3(P, v->eu), vs = dot3(P, v->ev);
    *as = (us - g->offdet[0]) / g->ddet[0] + (g->ndet[0] - 1) / 2.0;
    *bs = (vs - g->offdet[1]) / g->ddet[1] + (g->ndet[1] - 1) / 2.0;
    if (kind == ORC_W_FDK) {
        double DSOv = dot3(v->S, n);
        *w = (DSOv / Ld) * (DSOv / Ld);
    } else {
        double SXn = sqrt(dot3(SX, SX));
        *w = (g->dvox[0] * g->dvox[1] * g->dvox[2]) / (g->ddet[0] * g->ddet[1]) * DSDv * DSDv * SXn /
             (Ld * Ld * Ld);
    }
}

static double bp_voxel(const orc_geom *g, const double *views, int64_t na, const double *proj,
                       const float *projf, int kind, int64_t i, int64_t j, int64_t k) {
    double X[3];
    voxel_centre(g, i, j, k, X);
    const int64_t psz = g->ndet[0] * g->ndet[1];
    double acc = 0.0;
    for (int64_t t = 0; t < na; ++t) {
        double as, bs, w;
        project_voxel(g, view_at(views, t), X, kind, &as, &bs, &w);
        double a0 = floor(as), b0 = floor(bs);
        double fa = as - a0, fb = bs - b0;
        int64_t ia = (int64_t)a0, ib = (int64_t)b0;
        const double *pr = proj ? proj + t * psz : NULL;
        const float *prf = projf ? projf + t * psz : NULL;
        double v = (1 - fa) * (1 - fb) * proj_at(g, pr, prf, ia, ib) + fa * (1 - fb) * proj_at(g, pr, prf, ia + 1, ib) +
                   (1 - fa) * fb * proj_at(g, pr, prf, ia, ib + 1) + fa * fb * proj_at(g, pr, prf, ia + 1, ib + 1);
        acc += w * v;
    }
    return acc;
}

/* ------------------------------------------------------------------------------------------ */
/* exported entry points                                                                        */

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Chord sum of one ray S->P through vol (Siddon); nseg receives the number of pieces. */
double orc_siddon_ray(const orc_geom *g, const double *S, const double *P, const double *vol,
                      int64_t *nseg) {
    scratch_t sc;
    scratch_init(&sc, g);
    double r = siddon_core(g, S, P, vol, NULL, NULL, 0.0, -1, nseg, &sc);
    free(sc.buf);
    return r;
}

/* Interpolated line integral of one ray S->P. */
double orc_interp_ray(const orc_geom *g, const double *S, const double *P, const double *vol,
                      int64_t *nsamp) {
    return interp_ray(g, S, P, vol, nsamp);
}

/* proj[t][b][a] = Siddon(ray(view t, a, b)) for every pixel; optional per-view segment counts */
void orc_siddon_fwd(const orc_geom *g, const double *views, int64_t na, const double *vol,
                    double *proj, int64_t *seg_count_per_angle) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
    if (seg_count_per_angle) memset(seg_count_per_angle, 0, sizeof(int64_t) * na);
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, g);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < na * nv; ++r) {
            int64_t t = r / nv, b = r % nv;
            double S[3], P[3];
            int64_t rowsegs = 0;
            source_pos(view_at(views, t), S);
            for (int64_t a = 0; a < nu; ++a) {
                int64_t ns = 0;
                pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
                proj[(t * nv + b) * nu + a] = siddon_core(g, S, P, vol, NULL, NULL, 0.0, -1, &ns, &sc);
                rowsegs += ns;
            }
            if (seg_count_per_angle) {
#pragma omp atomic
                seg_count_per_angle[t] += rowsegs;
            }
        }
        free(sc.buf);
    }
}

/* Selected rays only: ray_idx[n] are flat indices (t*Nv + b)*Nu + a into the projection array. */
void orc_siddon_rays(const orc_geom *g, const double *views, const int64_t *ray_idx, int64_t n,
                     const double *vol, double *out) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, g);
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < n; ++q) {
            int64_t r = ray_idx[q];
            int64_t a = r % nu, b = (r / nu) % nv, t = r / (nu * nv);
            double S[3], P[3];
            source_pos(view_at(views, t), S);
            pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
            out[q] = siddon_core(g, S, P, vol, NULL, NULL, 0.0, -1, NULL, &sc);
        }
        free(sc.buf);
    }
}

/* Number of Siddon pieces (non-empty segments between consecutive plane crossings) of selected
 * rays, ray_idx as orc_siddon_rays: the count of voxel reads a ray costs. */
void orc_siddon_segments(const orc_geom *g, const double *views, const int64_t *ray_idx, int64_t n,
                         int64_t *out) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, g);
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < n; ++q) {
            int64_t r = ray_idx[q];
            int64_t a = r % nu, b = (r / nu) % nv, t = r / (nu * nv);
            double S[3], P[3];
            int64_t ns = 0;
            source_pos(view_at(views, t), S);
            pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
            siddon_core(g, S, P, NULL, NULL, NULL, 0.0, -1, &ns, &sc);
            out[q] = ns;
        }
        free(sc.buf);
    }
}

/* Exact transpose of orc_siddon_fwd: vol = sum over rays of y_ray * (piece lengths), scattered.
 * Threads scatter into private volumes that are summed at the end. */
void orc_siddon_adj(const orc_geom *g, const double *views, int64_t na, const double *proj,
                    double *vol) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
    const int64_t nvox = g->nvox[0] * g->nvox[1] * g->nvox[2];
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
    while (nthr > 1 && (double)nthr * nvox * 8.0 > 4e9) nthr--;
#endif
    double *priv = (double *)calloc((size_t)nthr * nvox, sizeof(double));
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = priv + (size_t)tid * nvox;
        scratch_t sc;
        scratch_init(&sc, g);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < na * nv; ++r) {
            int64_t t = r / nv, b = r % nv;
            double S[3], P[3];
            source_pos(view_at(views, t), S);
            for (int64_t a = 0; a < nu; ++a) {
                double y = proj[(t * nv + b) * nu + a];
                if (y == 0.0) continue;
                pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
                siddon_core(g, S, P, NULL, NULL, mine, y, -1, NULL, &sc);
            }
        }
        free(sc.buf);
    }
    for (int64_t v = 0; v < nvox; ++v) {
        double s = 0.0;
        for (int q = 0; q < nthr; ++q) s += priv[(size_t)q * nvox + v];
        vol[v] = s;
    }
    free(priv);
}

/* The transpose of the Siddon projector at selected voxels only: for each voxel and angle, every
 * pixel whose ray can meet the voxel (bounding box of the 8 projected corners, widened by one
 * pixel) is traversed and the length it spends in that voxel is weighted by the pixel value. */
static void adj_voxels(const orc_geom *g, const double *views, int64_t na, const double *proj,
                       const float *projf, const int64_t *vox_idx, int64_t n, double *out) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
    const int64_t nx = g->nvox[0], ny = g->nvox[1];
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, g);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; ++q) {
            int64_t lin = vox_idx[q];
            int64_t i = lin % nx, j = (lin / nx) % ny, k = lin / (nx * ny);
            double acc = 0.0;
            for (int64_t t = 0; t < na; ++t) {
                double amin = 1e300, amax = -1e300, bmin = 1e300, bmax = -1e300;
                for (int c = 0; c < 8; ++c) {
                    double X[3];
                    voxel_centre(g, i, j, k, X);
                    X[0] += ((c & 1) ? 0.5 : -0.5) * g->dvox[0];
                    X[1] += ((c & 2) ? 0.5 : -0.5) * g->dvox[1];
                    X[2] += ((c & 4) ? 0.5 : -0.5) * g->dvox[2];
                    double as, bs, w;
                    project_voxel(g, view_at(views, t), X, ORC_W_FDK, &as, &bs, &w);
                    if (as < amin) amin = as;
                    if (as > amax) amax = as;
                    if (bs < bmin) bmin = bs;
                    if (bs > bmax) bmax = bs;
                }
                int64_t a0 = (int64_t)floor(amin) - 1, a1 = (int64_t)ceil(amax) + 1;
                int64_t b0 = (int64_t)floor(bmin) - 1, b1 = (int64_t)ceil(bmax) + 1;
                if (a0 < 0) a0 = 0;
                if (b0 < 0) b0 = 0;
                if (a1 > nu - 1) a1 = nu - 1;
                if (b1 > nv - 1) b1 = nv - 1;
                double S[3], P[3];
                source_pos(view_at(views, t), S);
                for (int64_t b = b0; b <= b1; ++b)
                    for (int64_t a = a0; a <= a1; ++a) {
                        const int64_t o = (t * nv + b) * nu + a;
                        double y = projf ? (double)projf[o] : proj[o];
                        if (y == 0.0) continue;
                        pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
                        acc += y * siddon_core(g, S, P, NULL, NULL, NULL, 0.0, lin, NULL, &sc);
                    }
            }
            out[q] = acc;
        }
        free(sc.buf);
    }
}

void orc_siddon_adj_voxels(const orc_geom *g, const double *views, int64_t na, const double *proj,
                           const int64_t *vox_idx, int64_t n, double *out) {
    adj_voxels(g, views, na, proj, NULL, vox_idx, n, out);
}

/* The same with FP32 projections read in place (each value widened exactly to FP64). */
void orc_siddon_adj_voxels_f32(const orc_geom *g, const double *views, int64_t na, const float *proj,
                               const int64_t *vox_idx, int64_t n, double *out) {
    adj_voxels(g, views, na, NULL, proj, vox_idx, n, out);
}

void orc_interp_fwd(const orc_geom *g, const double *views, int64_t na, const double *vol,
                    double *proj, int64_t *samples_per_angle) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
    if (samples_per_angle) memset(samples_per_angle, 0, sizeof(int64_t) * na);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < na * nv; ++r) {
        int64_t t = r / nv, b = r % nv;
        double S[3], P[3];
        int64_t rows = 0;
        source_pos(view_at(views, t), S);
        for (int64_t a = 0; a < nu; ++a) {
            int64_t ns = 0;
            pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
            proj[(t * nv + b) * nu + a] = interp_ray(g, S, P, vol, &ns);
            rows += ns;
        }
        if (samples_per_angle) {
#pragma omp atomic
            samples_per_angle[t] += rows;
        }
    }
}

void orc_interp_rays(const orc_geom *g, const double *views, const int64_t *ray_idx, int64_t n,
                     const double *vol, double *out) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n; ++q) {
        int64_t r = ray_idx[q];
        int64_t a = r % nu, b = (r / nu) % nv, t = r / (nu * nv);
        double S[3], P[3];
        source_pos(view_at(views, t), S);
        pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
        out[q] = interp_ray(g, S, P, vol, NULL);
    }
}

/* vol[k][j][i] = sum over angles of w * bilinear(proj_t at the voxel's projection) */
void orc_bp(const orc_geom *g, const double *views, int64_t na, const double *proj, int kind,
            double *vol) {
    const int64_t nx = g->nvox[0], ny = g->nvox[1], nz = g->nvox[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nz * ny; ++r) {
        int64_t k = r / ny, j = r % ny;
        for (int64_t i = 0; i < nx; ++i) vol[(k * ny + j) * nx + i] = bp_voxel(g, views, na, proj, NULL, kind, i, j, k);
    }
}

void orc_bp_voxels(const orc_geom *g, const double *views, int64_t na, const double *proj, int kind,
                   const int64_t *vox_idx, int64_t n, double *out) {
    const int64_t nx = g->nvox[0], ny = g->nvox[1];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n; ++q) {
        int64_t lin = vox_idx[q];
        out[q] = bp_voxel(g, views, na, proj, NULL, kind, lin % nx, (lin / nx) % ny, lin / (nx * ny));
    }
}

/* The same samplers reading FP32 inputs (each element is widened to FP64 when read; the
 * arithmetic is that of the FP64 versions).  For inputs too large to hold twice. */
void orc_siddon_rays_f32(const orc_geom *g, const double *views, const int64_t *ray_idx, int64_t n,
                         const float *vol, double *out) {
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, g);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; ++q) {
            int64_t r = ray_idx[q];
            int64_t a = r % nu, b = (r / nu) % nv, t = r / (nu * nv);
            double S[3], P[3];
            source_pos(view_at(views, t), S);
            pixel_pos(g, view_at(views, t), (double)a, (double)b, P);
            out[q] = siddon_core(g, S, P, NULL, vol, NULL, 0.0, -1, NULL, &sc);
        }
        free(sc.buf);
    }
}

void orc_bp_voxels_f32(const orc_geom *g, const double *views, int64_t na, const float *proj, int kind,
                       const int64_t *vox_idx, int64_t n, double *out) {
    const int64_t nx = g->nvox[0], ny = g->nvox[1];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n; ++q) {
        int64_t lin = vox_idx[q];
        out[q] = bp_voxel(g, views, na, NULL, proj, kind, lin % nx, (lin / nx) % ny, lin / (nx * ny));
    }
}

/* Transpose of orc_bp (a voxel-driven bilinear "splat" projector with the same weight); used only
 * to check the indexing of the backprojector by the dot-product identity. */
void orc_bp_transpose(const orc_geom *g, const double *views, int64_t na, const double *vol, int kind,
                      double *proj) {
    const int64_t nx = g->nvox[0], ny = g->nvox[1], nz = g->nvox[2];
    const int64_t nu = g->ndet[0], nv = g->ndet[1];
    memset(proj, 0, sizeof(double) * na * nu * nv);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < na; ++t) {
        double *pr = proj + t * nu * nv;
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    double x = vol[(k * ny + j) * nx + i];
                    if (x == 0.0) continue;
                    double X[3], as, bs, w;
                    voxel_centre(g, i, j, k, X);
                    project_voxel(g, view_at(views, t), X, kind, &as, &bs, &w);
                    double a0 = floor(as), b0 = floor(bs), fa = as - a0, fb = bs - b0;
                    int64_t ia = (int64_t)a0, ib = (int64_t)b0;
                    for (int db = 0; db < 2; ++db)
                        for (int da = 0; da < 2; ++da) {
                            int64_t aa = ia + da, bb = ib + db;
                            if (aa < 0 || bb < 0 || aa >= nu || bb >= nv) continue;
                            pr[bb * nu + aa] += w * x * (da ? fa : 1 - fa) * (db ? fb : 1 - fb);
                        }
                }
    }
}
