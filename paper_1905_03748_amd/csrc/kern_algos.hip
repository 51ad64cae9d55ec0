// Device-resident iterative algorithms built on the operators: CGLS (FP64 inner products and
// residual recurrence, scalars kept in device memory so an iteration never waits on the host),
// OS-SART (SART with one angle per update when block = 1) and TV steepest descent.  Reductions use a fixed partition
// (DOT_BLOCKS contiguous ranges, fixed wave/block trees, fixed final sum), so results are bitwise
// repeatable regardless of what else shares the device.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dev_common.hpp"

namespace ct {

namespace {

constexpr int DOT_BLOCKS = 1024;
constexpr int DOT_THREADS = 256;
constexpr int EW_THREADS = 256;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

inline unsigned ew_grid(int64_t n) {
    int64_t g = (n + EW_THREADS - 1) / EW_THREADS;
    if (g > 65536 * 16) g = 65536 * 16;
    if (g < 1) g = 1;
    return (unsigned)g;
}

template <typename T>
__global__ __launch_bounds__(DOT_THREADS) void k_dot_partial(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                                             double *__restrict__ partials) {
    __shared__ double lds[DOT_THREADS / 64];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += to_d(a[i]) * to_d(b[i]);
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(DOT_THREADS) void k_sum_partials(const double *__restrict__ partials, int n,
                                                              double *__restrict__ out) {
    __shared__ double lds[DOT_THREADS / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) *out = s;
}

template <typename TS, typename TD>
__global__ void k_convert(const TS *__restrict__ s, TD *__restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = from_d<TD>(to_d(s[i]));
}

// r (FP32) = b - r, b in its storage type
template <typename T>
__global__ void k_rsub_from(const T *__restrict__ b, float *__restrict__ r, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = ldf(b, i) - r[i];
}

// y (storage type) += sign * scal[idx] * x (FP32)
template <typename T>
__global__ void k_axpy_mixed(T *__restrict__ y, const float *__restrict__ x, const double *__restrict__ scal, int idx,
                             float sign, int64_t n) {
    const float a = sign * (float)scal[idx];
    if (a == 0.0f) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = from_f<T>(fmaf(a, x[i], ldf(y, i)));
}

template <typename T>
__global__ void k_copy(const T *__restrict__ s, T *__restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

// y += sign * scal[idx] * x
template <typename T>
__global__ void k_axpy_s(T *__restrict__ y, const T *__restrict__ x, const double *__restrict__ scal, int idx,
                         float sign, int64_t n) {
    const float a = sign * (float)scal[idx];
    if (a == 0.0f) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = from_f<T>(fmaf(a, ldf(x, i), ldf(y, i)));
}

// p = s + scal[idx] * p
template <typename T>
__global__ void k_xpby_s(T *__restrict__ p, const T *__restrict__ s, const double *__restrict__ scal, int idx,
                         int64_t n) {
    const float bta = (float)scal[idx];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = from_f<T>(fmaf(bta, ldf(p, i), ldf(s, i)));
}

// CGLS scalar slots
enum { S_GAMMA = 0, S_DELTA = 1, S_ALPHA = 2, S_BETA = 3, S_RHO = 4, S_STOP = 5, S_TMP = 6, S_COUNT = 8 };

__global__ void k_cgls_start(double *scal, double *resid) {
    scal[S_STOP] = 0.0;
    scal[S_ALPHA] = 0.0;
    scal[S_BETA] = 0.0;
    if (resid) resid[0] = sqrt(fmax(scal[S_RHO], 0.0));
}

__global__ void k_cgls_alpha(double *scal, double *resid, int k) {
    const double delta = scal[S_DELTA];
    if (scal[S_STOP] != 0.0 || delta == 0.0) {
        scal[S_STOP] = 1.0;
        scal[S_ALPHA] = 0.0;
    } else {
        const double alpha = scal[S_GAMMA] / delta;
        scal[S_ALPHA] = alpha;
        scal[S_RHO] = scal[S_RHO] - alpha * scal[S_GAMMA];
    }
    if (resid) resid[k + 1] = sqrt(fmax(scal[S_RHO], 0.0));
}

__global__ void k_cgls_beta(double *scal) {
    const double gnew = scal[S_TMP];
    if (scal[S_STOP] != 0.0) {
        scal[S_BETA] = 0.0;
        return;
    }
    scal[S_BETA] = scal[S_GAMMA] != 0.0 ? gnew / scal[S_GAMMA] : 0.0;
    scal[S_GAMMA] = gnew;
}

// SART residual for one angle: r = (b - r) / chord where chord > thr, else 0 (b in its storage type)
template <typename TP>
__global__ void k_sart_resid(const TP *__restrict__ b, const float *__restrict__ chord, float *__restrict__ r,
                             float thr, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float c = chord[i];
        r[i] = c > thr ? (to_f(b[i]) - r[i]) / c : 0.0f;
    }
}

// The same residual written transposed, rT[u][v], through 32 x 32 LDS tiles; blockIdx.z is the
// angle within the subset (each array advances by one projection per angle)
template <typename TP>
__global__ __launch_bounds__(256) void k_sart_resid_t(const TP *__restrict__ b, const float *__restrict__ chord,
                                                      const float *__restrict__ r, float *__restrict__ rT, float thr,
                                                      int nu, int nv) {
    __shared__ float tile[32][33];
    const int u0 = blockIdx.x * 32, v0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t po = (int64_t)blockIdx.z * nu * nv;
    b += po;
    chord += po;
    r += po;
    rT += po;
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int u = u0 + tx, v = v0 + ty + k;
        if (u < nu && v < nv) {
            const int64_t i = (int64_t)v * nu + u;
            const float c = chord[i];
            tile[ty + k][tx] = c > thr ? (to_f(b[i]) - r[i]) / c : 0.0f;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int v = v0 + tx, u = u0 + ty + k;
        if (u < nu && v < nv) rT[(int64_t)u * nv + v] = tile[tx][ty + k];
    }
}

// TV_eps gradient with forward differences, unit spacing, zero difference at the last index.
// Slices kg0 .. kg0 + nk - 1 of the volume (nz slices in all); x holds slices from kx0 on (at least
// z - 1 .. z + 1 where they exist) and g from kg0 on.  A whole resident volume has kx0 = kg0 = 0.
// Each thread walks TV_ZR slices of one (i, j) column: a voxel's gradient reads seven positions of
// its own slice, three of the slice above and three of the one below, so the thread loads the
// seven positions of each slice once and carries them up the column (7 loads per voxel, not 13).
constexpr int TV_ZR = 8;
struct TvPlane {
    float c, e, n, w, wn, s, se;  // (i, j), (i + 1, j), (i, j + 1), (i - 1, j), (i - 1, j + 1), (i, j - 1), (i + 1, j - 1)
};
__global__ __launch_bounds__(256) void k_tv_grad(const float *__restrict__ x, float *__restrict__ g, int nx, int ny,
                                                 int nz, float eps, int64_t kx0, int64_t kg0, int64_t nk) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const bool hx = i < nx - 1, hy = j < ny - 1, lx = i > 0, ly = j > 0;
    auto plane = [&](int64_t k) {  // positions outside the volume's x-y extent read as 0 (unused)
        const int64_t o = (k - kx0) * sz + (int64_t)j * sy + i;
        TvPlane p;
        p.c = x[o];
        p.e = hx ? x[o + 1] : 0.0f;
        p.n = hy ? x[o + sy] : 0.0f;
        p.w = lx ? x[o - 1] : 0.0f;
        p.wn = (lx && hy) ? x[o - 1 + sy] : 0.0f;
        p.s = ly ? x[o - sy] : 0.0f;
        p.se = (ly && hx) ? x[o - sy + 1] : 0.0f;
        return p;
    };
    const int64_t r0 = (int64_t)blockIdx.z * TV_ZR, r1 = min(r0 + (int64_t)TV_ZR, nk);
    int64_t k = kg0 + r0;
    TvPlane pm = {}, pn = {};
    if (k > 0) pm = plane(k - 1);
    TvPlane pc = plane(k);
    for (int64_t r = r0; r < r1; ++r, ++k) {
        const bool hz = k < nz - 1;
        if (hz) pn = plane(k + 1);
        const float xc = pc.c;
        // differences at the voxel
        const float dxc = hx ? pc.e - xc : 0.0f;
        const float dyc = hy ? pc.n - xc : 0.0f;
        const float dzc = hz ? pn.c - xc : 0.0f;
        float gv = -(dxc + dyc + dzc) / sqrtf(dxc * dxc + dyc * dyc + dzc * dzc + eps);
        if (lx) {  // neighbour - e_x
            const float xm = pc.w;
            const float a = xc - xm;
            const float b = hy ? pc.wn - xm : 0.0f;
            const float c = hz ? pn.w - xm : 0.0f;
            gv += a / sqrtf(a * a + b * b + c * c + eps);
        }
        if (ly) {
            const float xm = pc.s;
            const float a = hx ? pc.se - xm : 0.0f;
            const float b = xc - xm;
            const float c = hz ? pn.s - xm : 0.0f;
            gv += b / sqrtf(a * a + b * b + c * c + eps);
        }
        if (k > 0) {
            const float xm = pm.c;
            const float a = hx ? pm.e - xm : 0.0f;
            const float b = hy ? pm.n - xm : 0.0f;
            const float c = xc - xm;
            gv += c / sqrtf(a * a + b * b + c * c + eps);
        }
        g[(k - kg0) * sz + (int64_t)j * sy + i] = gv;
        pm = pc;
        pc = pn;
    }
}

// gradient of slices kg0 .. kg0 + nk - 1 (see k_tv_grad)
static ct_status launch_tv_grad(const float *x, float *g, int nx, int ny, int nz, float eps, int64_t kx0, int64_t kg0,
                                int64_t nk, hipStream_t st) {
    if (nk <= 0) return CT_OK;
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4, (unsigned)((nk + TV_ZR - 1) / TV_ZR));
    hipLaunchKernelGGL(k_tv_grad, grid, dim3(256), 0, st, x, g, nx, ny, nz, eps, kx0, kg0, nk);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

// ROF model by Chambolle's projection.  The dual field p = (px, py, pz) holds one FP32 volume per
// axis.  Divergence, minus the adjoint of the forward-difference gradient: along each axis
// p_i - p_{i-1} inside, p_0 at the first index, -p_{n-2} at the last, 0 for an axis of one voxel.
__device__ __forceinline__ float rof_div(const float *__restrict__ px, const float *__restrict__ py,
                                         const float *__restrict__ pz, int i, int j, int k, int nx, int ny, int nz,
                                         int64_t o, int64_t sy, int64_t sz) {
    float d = 0.0f;
    if (nz > 1) d += k == 0 ? pz[o] : (k == nz - 1 ? -pz[o - sz] : pz[o] - pz[o - sz]);
    if (ny > 1) d += j == 0 ? py[o] : (j == ny - 1 ? -py[o - sy] : py[o] - py[o - sy]);
    if (nx > 1) d += i == 0 ? px[o] : (i == nx - 1 ? -px[o - 1] : px[o] - px[o - 1]);
    return d;
}

// w = div p - f / lam
__global__ __launch_bounds__(256) void k_rof_w(const float *__restrict__ f, const float *__restrict__ px,
                                               const float *__restrict__ py, const float *__restrict__ pz,
                                               float *__restrict__ w, int nx, int ny, int nz, float inv_lam) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t o = k * sz + (int64_t)j * sy + i;
    w[o] = rof_div(px, py, pz, i, j, k, nx, ny, nz, o, sy, sz) - f[o] * inv_lam;
}

// p <- (p + tau grad w) / (1 + tau |grad w|), forward differences, zero at the last index
__global__ __launch_bounds__(256) void k_rof_p(const float *__restrict__ w, float *__restrict__ px,
                                               float *__restrict__ py, float *__restrict__ pz, int nx, int ny, int nz,
                                               float tau) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t o = k * sz + (int64_t)j * sy + i;
    const float wc = w[o];
    const float gx = i < nx - 1 ? w[o + 1] - wc : 0.0f;
    const float gy = j < ny - 1 ? w[o + sy] - wc : 0.0f;
    const float gz = k < nz - 1 ? w[o + sz] - wc : 0.0f;
    const float den = 1.0f + tau * sqrtf(gx * gx + gy * gy + gz * gz);
    px[o] = (px[o] + tau * gx) / den;
    py[o] = (py[o] + tau * gy) / den;
    pz[o] = (pz[o] + tau * gz) / den;
}

// u = f - lam div p, in place over f (each voxel reads only its own f)
__global__ __launch_bounds__(256) void k_rof_u(float *__restrict__ x, const float *__restrict__ px,
                                               const float *__restrict__ py, const float *__restrict__ pz, int nx,
                                               int ny, int nz, float lam) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t o = k * sz + (int64_t)j * sy + i;
    x[o] = fmaf(-lam, rof_div(px, py, pz, i, j, k, nx, ny, nz, o, sy, sz), x[o]);
}

__global__ void k_fill_zero(float *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// TV scalars: [0] = ||x_in||^2, [1] = alpha, [2] = ||g||^2
__global__ void k_tv_alpha(double *scal, double lambda) { scal[1] = lambda * sqrt(scal[0]); }

__global__ void k_tv_update(float *__restrict__ x, const float *__restrict__ g, const double *__restrict__ scal,
                            int64_t n) {
    const double ng2 = scal[2];
    if (!(ng2 > 0.0)) return;
    const float a = (float)(scal[1] / sqrt(ng2));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = fmaf(-a, g[i], x[i]);
}

struct Workspace {
    char *base = nullptr;
    bool owned = false;
    hipStream_t st = nullptr;
    size_t off = 0;
    void *take(size_t bytes) {
        void *p = base + off;
        off += align256(bytes);
        return p;
    }
    ct_status acquire(void *user, size_t bytes, hipStream_t s) {
        st = s;
        if (user) {
            base = (char *)user;
            return CT_OK;
        }
        owned = true;
        CT_HIP(CT_MALLOC_ASYNC((void **)&base, bytes ? bytes : 256, s));
        return CT_OK;
    }
    ~Workspace() {
        if (owned && base) (void)hipFreeAsync(base, st);
    }
};

}  // namespace

size_t dot_partials_count() { return DOT_BLOCKS; }

ct_status dot_f64(const void *a, const void *b, ct_dtype t, int64_t n, double *out, double *partials, hipStream_t st) {
    Workspace ws;
    if (!partials) {
        ct_status s = ws.acquire(nullptr, DOT_BLOCKS * sizeof(double), st);
        if (s != CT_OK) return s;
        partials = (double *)ws.take(DOT_BLOCKS * sizeof(double));
    }
    CT_DISPATCH1_ANY(t, T,
                     hipLaunchKernelGGL((k_dot_partial<T>), dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, st, (const T *)a,
                                        (const T *)b, n, partials));
    CT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(DOT_THREADS), 0, st, partials, DOT_BLOCKS, out);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status convert(const void *src, ct_dtype s_t, void *dst, ct_dtype d_t, int64_t n, hipStream_t st) {
    if (n == 0) return CT_OK;
    CT_DISPATCH1_ANY(s_t, TS,
                     CT_DISPATCH1_ANY(d_t, TD,
                                      hipLaunchKernelGGL((k_convert<TS, TD>), dim3(ew_grid(n)), dim3(EW_THREADS), 0, st,
                                                         (const TS *)src, (TD *)dst, n)));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

// ---------------------------------------------------------------------------------------------
// CGLS

// The recurrence vectors r, q (projection-shaped) and s, p (volume-shaped) are FP32 whatever the
// storage of x and b: CGLS search directions are unnormalised (A p grows like the operator norm
// squared times the data), which overflows FP16's range on realistic problems.
// r, q (projections), s, p (volumes), partials and scalars, the Siddon column copy of the volume
// being projected, and the exact adjoint's transposed projection copy: no allocation per iteration
size_t cgls_workspace(const ct_plan *p, ct_dtype, ct_dtype) {
    const ct_geometry &g = p->g;
    const size_t nv = (size_t)g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    const size_t np = (size_t)g.nDetector[0] * g.nDetector[1] * p->angles.size();
    return 2 * align256(nv * 4) + 2 * align256(np * 4) + align256(DOT_BLOCKS * 8) + align256(S_COUNT * 8) +
           align256((size_t)zcol_elems(g) * 4) + align256(p->angles.size() * adj_chunk_bytes_per_angle(g));
}

ct_status cgls_run(ct_plan *p, const void *b, ct_dtype pt, void *x, ct_dtype vt, int32_t niter, double *resid,
                   void *work, hipStream_t st) {
    const ct_geometry &g = p->g;
    const int64_t nv = g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    const int64_t na = (int64_t)p->angles.size();
    const int64_t np = g.nDetector[0] * g.nDetector[1] * na;
    Workspace ws;
    ct_status s = ws.acquire(work, cgls_workspace(p, vt, pt), st);
    if (s != CT_OK) return s;
    float *r = (float *)ws.take(np * 4);
    float *q = (float *)ws.take(np * 4);
    float *sv = (float *)ws.take(nv * 4);
    float *pv = (float *)ws.take(nv * 4);
    double *parts = (double *)ws.take(DOT_BLOCKS * 8);
    double *scal = (double *)ws.take(S_COUNT * 8);
    void *vz = ws.take((size_t)zcol_elems(g) * 4);
    const size_t qbytes = (size_t)na * adj_chunk_bytes_per_angle(g);
    void *yq = ws.take(qbytes);
    const Slab full = full_slab(g);
    const bool col = zcol_ok(p, 0, na);
#define CK(e)                          \
    do {                               \
        ct_status s_ = (e);            \
        if (s_ != CT_OK) return s_;    \
    } while (0)
    // A v through the column copy in the workspace (refreshed from v first)
    auto fwd = [&](const void *v, ct_dtype t, float *out) -> ct_status {
        if (col) {
            ct_status s_ = launch_zcols(v, t, vz, g.nVoxel[0], g.nVoxel[1], g.nVoxel[2], st);
            if (s_ != CT_OK) return s_;
        }
        return launch_forward(p, CT_SIDDON, v, t, out, CT_F32, 0, 0, na, full, st, col ? vz : nullptr);
    };
    // r = b - A x ; s = A^T r ; p = s ; gamma = <s,s> ; rho = <r,r>
    CK(fwd(x, vt, r));
    CT_DISPATCH1(pt, T, hipLaunchKernelGGL((k_rsub_from<T>), dim3(ew_grid(np)), dim3(EW_THREADS), 0, st, (const T *)b, r, np));
    CT_HIP(hipGetLastError());
    CK(launch_backproject(p, CT_BP_ADJOINT, r, CT_F32, sv, CT_F32, 0, 0, na, full, st, yq, qbytes));
    hipLaunchKernelGGL((k_copy<float>), dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, (const float *)sv, pv, nv);
    CT_HIP(hipGetLastError());
    CK(dot_f64(sv, sv, CT_F32, nv, scal + S_GAMMA, parts, st));
    CK(dot_f64(r, r, CT_F32, np, scal + S_RHO, parts, st));
    hipLaunchKernelGGL(k_cgls_start, dim3(1), dim3(1), 0, st, scal, resid);
    CT_HIP(hipGetLastError());
    for (int32_t k = 0; k < niter; ++k) {
        // q = A p ; delta = <q,q> ; alpha = gamma / delta
        CK(fwd(pv, CT_F32, q));
        CK(dot_f64(q, q, CT_F32, np, scal + S_DELTA, parts, st));
        hipLaunchKernelGGL(k_cgls_alpha, dim3(1), dim3(1), 0, st, scal, resid, k);
        CT_HIP(hipGetLastError());
        // x += alpha p (x in its storage type) ; r -= alpha q
        CT_DISPATCH1(vt, T, hipLaunchKernelGGL((k_axpy_mixed<T>), dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, (T *)x,
                                               (const float *)pv, scal, (int)S_ALPHA, 1.0f, nv));
        hipLaunchKernelGGL((k_axpy_s<float>), dim3(ew_grid(np)), dim3(EW_THREADS), 0, st, r, (const float *)q, scal,
                           (int)S_ALPHA, -1.0f, np);
        CT_HIP(hipGetLastError());
        // s = A^T r ; gamma' = <s,s> ; beta = gamma'/gamma ; p = s + beta p
        CK(launch_backproject(p, CT_BP_ADJOINT, r, CT_F32, sv, CT_F32, 0, 0, na, full, st, yq, qbytes));
        CK(dot_f64(sv, sv, CT_F32, nv, scal + S_TMP, parts, st));
        hipLaunchKernelGGL(k_cgls_beta, dim3(1), dim3(1), 0, st, scal);
        CT_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_xpby_s<float>), dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, pv, (const float *)sv, scal,
                           (int)S_BETA, nv);
        CT_HIP(hipGetLastError());
    }
    return CT_OK;
}

// ---------------------------------------------------------------------------------------------
// SART

// chords of every ray, one subset's residuals (and their transposes), and a column-major copy of x
// that the sweep projects from and updates in place (x is restored from it at the end)
size_t sart_workspace(const ct_plan *p, int32_t block) {
    const ct_geometry &g = p->g;
    const size_t pix = (size_t)g.nDetector[0] * g.nDetector[1];
    const size_t nb = (size_t)std::max<int32_t>(block, 1);
    return align256(pix * p->angles.size() * 4) + 2 * align256(pix * nb * 4) + align256((size_t)zcol_elems(g) * 4);
}

// OS-SART: the angles in natural order, cut into consecutive subsets of `block` (the last one may be
// shorter); each subset projects, forms its weighted residuals and makes one update (block = 1 is
// SART)
ct_status sart_run(ct_plan *p, const void *b, ct_dtype pt, void *x, ct_dtype vt, int32_t niter, double lambda,
                   int32_t block, void *work, hipStream_t st) {
    const ct_geometry &g = p->g;
    const int64_t na = (int64_t)p->angles.size();
    const int64_t pix = g.nDetector[0] * g.nDetector[1];
    const int64_t nvox = g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    const size_t pe = dtype_size(pt);
    Workspace ws;
    ct_status s = ws.acquire(work, sart_workspace(p, block), st);
    if (s != CT_OK) return s;
    float *chord = (float *)ws.take(pix * na * 4);
    float *r = (float *)ws.take(pix * block * 4);
    float *rT = (float *)ws.take(pix * block * 4);
    float *xz = (float *)ws.take((size_t)zcol_elems(g) * 4);
    const float thr = (float)(1e-2 * std::fmin(g.dVoxel[0], std::fmin(g.dVoxel[1], g.dVoxel[2])));
    const int nu = (int)g.nDetector[0], nv = (int)g.nDetector[1];
    CK(launch_ray_chord(p, chord, 0, na, st));
    const Slab full = full_slab(g);
    // the sweep updates an FP32 image: the column-major copy, or (other geometries) x itself when
    // it is stored in FP32, else an FP32 copy of it; a 16-bit x is rounded once, at the end
    // the column-major sweep's update kernel is written for a circular orbit; plans of views update
    // x through the per-view kernel
    if (zcol_ok(p, 0, na) && !p->views) {
        CK(launch_zcols_f32(x, vt, xz, g.nVoxel[0], g.nVoxel[1], g.nVoxel[2], st));
        for (int32_t it = 0; it < niter; ++it) {
            for (int64_t t0 = 0; t0 < na; t0 += block) {
                const int64_t t1 = std::min<int64_t>(na, t0 + block);
                CK(launch_forward(p, CT_SIDDON, xz, CT_F32, r, CT_F32, 0, t0, t1, full, st, xz));
                const dim3 tg((unsigned)((nu + 31) / 32), (unsigned)((nv + 31) / 32), (unsigned)(t1 - t0));
                const void *bt = (const char *)b + t0 * pix * pe;
                CT_DISPATCH1(pt, TP,
                             hipLaunchKernelGGL((k_sart_resid_t<TP>), tg, dim3(256), 0, st, (const TP *)bt,
                                                chord + t0 * pix, (const float *)r, rT, thr, nu, nv));
                CT_HIP(hipGetLastError());
                CK(launch_sart_update_col(p, rT, xz, t0, t1, (float)lambda, st));
            }
        }
        CK(launch_zcols_inv_f32(xz, x, vt, g.nVoxel[0], g.nVoxel[1], g.nVoxel[2], st));
        return CT_OK;
    }
    float *xf = (float *)x;
    if (vt != CT_F32) {
        xf = xz;
        CK(convert(x, vt, xf, CT_F32, nvox, st));
    }
    for (int32_t it = 0; it < niter; ++it) {
        for (int64_t t0 = 0; t0 < na; t0 += block) {
            const int64_t t1 = std::min<int64_t>(na, t0 + block);
            CK(launch_forward(p, CT_SIDDON, xf, CT_F32, r, CT_F32, 0, t0, t1, full, st));
            const void *bt = (const char *)b + t0 * pix * pe;
            CT_DISPATCH1(pt, TP,
                         hipLaunchKernelGGL((k_sart_resid<TP>), dim3(ew_grid((t1 - t0) * pix)), dim3(EW_THREADS), 0, st,
                                            (const TP *)bt, chord + t0 * pix, r, thr, (t1 - t0) * pix));
            CT_HIP(hipGetLastError());
            CK(launch_sart_update(p, r, xf, t0, t1, (float)lambda, st));
        }
    }
    if (vt != CT_F32) CK(convert(xf, CT_F32, x, vt, nvox, st));
    return CT_OK;
}

// ---------------------------------------------------------------------------------------------
// TV steepest descent

size_t tv_workspace(const ct_geometry &g, ct_dtype vt) {
    const size_t nv = (size_t)g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    // a 16-bit image is stepped in an FP32 copy
    return align256(nv * 4) * (vt == CT_F32 ? 1 : 2) + align256(DOT_BLOCKS * 8) + align256(4 * 8);
}

ct_status tv_run(const ct_geometry &g, void *xs, ct_dtype vt, int32_t nsteps, double lambda, double eps, void *work,
                 hipStream_t st) {
    const int nx = (int)g.nVoxel[0], ny = (int)g.nVoxel[1], nz = (int)g.nVoxel[2];
    const int64_t nv = (int64_t)nx * ny * nz;
    Workspace ws;
    ct_status s = ws.acquire(work, tv_workspace(g, vt), st);
    if (s != CT_OK) return s;
    float *gbuf = (float *)ws.take(nv * 4);
    double *parts = (double *)ws.take(DOT_BLOCKS * 8);
    double *scal = (double *)ws.take(4 * 8);
    void *x = xs;
    if (vt != CT_F32) {
        x = ws.take(nv * 4);
        CK(convert(xs, vt, x, CT_F32, nv, st));
    }
    CK(dot_f64(x, x, CT_F32, nv, scal + 0, parts, st));
    hipLaunchKernelGGL(k_tv_alpha, dim3(1), dim3(1), 0, st, scal, lambda);
    CT_HIP(hipGetLastError());
    for (int32_t k = 0; k < nsteps; ++k) {
        CK(launch_tv_grad((const float *)x, gbuf, nx, ny, nz, (float)eps, 0, 0, nz, st));
        CK(dot_f64(gbuf, gbuf, CT_F32, nv, scal + 2, parts, st));
        hipLaunchKernelGGL(k_tv_update, dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, (float *)x, (const float *)gbuf, scal, nv);
        CT_HIP(hipGetLastError());
    }
    if (vt != CT_F32) CK(convert(x, CT_F32, xs, vt, nv, st));
    return CT_OK;
#undef CK
}


// ---------------------------------------------------------------------------------------------
// ROF model (Chambolle's projection): workspace px, py, pz, w

size_t rof_workspace(const ct_geometry &g) {
    const size_t nv = (size_t)g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2];
    return 4 * align256(nv * 4);
}

ct_status rof_run(const ct_geometry &g, void *x, int32_t niter, double lambda, double tau, void *work, hipStream_t st) {
    const int nx = (int)g.nVoxel[0], ny = (int)g.nVoxel[1], nz = (int)g.nVoxel[2];
    const int64_t nv = (int64_t)nx * ny * nz;
    Workspace ws;
    ct_status s = ws.acquire(work, rof_workspace(g), st);
    if (s != CT_OK) return s;
    float *px = (float *)ws.take(nv * 4), *py = (float *)ws.take(nv * 4), *pz = (float *)ws.take(nv * 4);
    float *w = (float *)ws.take(nv * 4);
    hipLaunchKernelGGL(k_fill_zero, dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, px, nv);
    hipLaunchKernelGGL(k_fill_zero, dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, py, nv);
    hipLaunchKernelGGL(k_fill_zero, dim3(ew_grid(nv)), dim3(EW_THREADS), 0, st, pz, nv);
    CT_HIP(hipGetLastError());
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz);
    for (int32_t it = 0; it < niter; ++it) {
        hipLaunchKernelGGL(k_rof_w, grid, dim3(256), 0, st, (const float *)x, px, py, pz, w, nx, ny, nz,
                           (float)(1.0 / lambda));
        hipLaunchKernelGGL(k_rof_p, grid, dim3(256), 0, st, (const float *)w, px, py, pz, nx, ny, nz, (float)tau);
        CT_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_rof_u, grid, dim3(256), 0, st, (float *)x, px, py, pz, nx, ny, nz, (float)lambda);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

// ---------------------------------------------------------------------------------------------
// TV steepest descent out of core: the image in host memory, slabs of axial slices under a device
// memory cap.  The gradient at slice z needs slices z - 1 .. z + 1, so each slab is uploaded with a
// halo slice on either side.  A step is two passes over the slabs: the first sums ||g||^2 (and,
// at the first step, ||x_in||^2) slab by slab in FP64, in slab order; the second recomputes each
// slab's gradient and applies x -= alpha g / ||g||.  In the second pass the slab below has already
// been updated, so its last slice is kept on the device as it was before that update and replaces
// the uploaded lower halo: every gradient of a step sees the image from before the step.

namespace {

constexpr uint64_t TV_RESERVE = 64ull << 20;

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

// CT_OOC_VERBOSE=1 reports each finished pass on stderr (long out-of-core runs)
bool tv_verbose() {
    static const bool v = [] {
        const char *e = std::getenv("CT_OOC_VERBOSE");
        return e && e[0] && e[0] != '0';
    }();
    return v;
}

struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() {
        if (s) (void)hipStreamDestroy(s);
    }
};

}  // namespace

__global__ void k_scale_entry(double *p, double f) { *p *= f; }

ct_status tv_host_run_halo(const ct_geometry &g, float *hx, int32_t nsteps, double lambda, double eps, int32_t depth,
                           uint64_t cap, ct_ooc_stats *stats);

ct_status tv_host_run(const ct_geometry &g, float *hx, int32_t nsteps, double lambda, double eps, int32_t depth,
                      uint64_t cap, ct_ooc_stats *stats) {
    if (depth > 0) return tv_host_run_halo(g, hx, nsteps, lambda, eps, depth, cap, stats);
    const auto t_start = std::chrono::steady_clock::now();
    const int nx = (int)g.nVoxel[0], ny = (int)g.nVoxel[1];
    const int64_t nz = g.nVoxel[2];
    const int64_t slice = (int64_t)nx * ny;
    const uint64_t sb = (uint64_t)slice * sizeof(float);
    const uint64_t fixed = TV_RESERVE + align256(DOT_BLOCKS * 8) + align256(4 * 8);
    // device: the slab with two halo slices, its gradient, one saved slice
    if (cap <= fixed || (cap - fixed) / sb < 5)
        return fail(CT_ERR_CAP, "device memory cap is below one slab slice plus halos and buffers");
    int64_t h = (int64_t)(((cap - fixed) / sb - 3) / 2);
    h = std::max<int64_t>(1, std::min<int64_t>(h, nz));
    const int64_t nsp = (nz + h - 1) / h;
    h = (nz + nsp - 1) / nsp;
    ct_ooc_stats st;
    std::memset(&st, 0, sizeof(st));
    st.n_slabs = (int32_t)nsp;
    st.slab_slices = (int32_t)h;
    OwnStream S;
    CT_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
    DevMem xb, gb, saved, parts, scal;
    CT_HIP(CT_MALLOC(&xb.p, (size_t)(h + 2) * sb));
    CT_HIP(CT_MALLOC(&gb.p, (size_t)h * sb));
    CT_HIP(CT_MALLOC(&saved.p, (size_t)sb));
    CT_HIP(CT_MALLOC(&parts.p, DOT_BLOCKS * 8));
    CT_HIP(CT_MALLOC(&scal.p, 4 * 8));
    float *xbuf = (float *)xb.p, *gbuf = (float *)gb.p;
    double *dscal = (double *)scal.p;
    const hipStream_t s = S.s;
    auto bounds = [&](int64_t n, int64_t &o0, int64_t &o1, int64_t &m0, int64_t &m1) {
        o0 = n * h;
        o1 = std::min(nz, o0 + h);
        m0 = std::max<int64_t>(0, o0 - 1);
        m1 = std::min(nz, o1 + 1);
    };
    auto grad = [&](int64_t m0, int64_t o0, int64_t o1) -> ct_status {
        return launch_tv_grad((const float *)xbuf, gbuf, nx, ny, (int)nz, (float)eps, m0, o0, o1 - o0, s);
    };
    auto dot_host = [&](const float *a, int64_t n, double &out) -> ct_status {
        ct_status e = dot_f64(a, a, CT_F32, n, dscal + 3, (double *)parts.p, s);
        if (e != CT_OK) return e;
        CT_HIP(hipMemcpyAsync(&out, dscal + 3, 8, hipMemcpyDeviceToHost, s));
        CT_HIP(hipStreamSynchronize(s));
        return CT_OK;
    };
    double alpha = 0.0;
    ct_status e = CT_OK;
    for (int32_t step = 0; step < nsteps; ++step) {
        double gg = 0.0, xx = 0.0;
        for (int64_t n = 0; n < nsp; ++n) {  // pass 1: norms
            int64_t o0, o1, m0, m1;
            bounds(n, o0, o1, m0, m1);
            CT_HIP(hipMemcpyAsync(xbuf, hx + m0 * slice, (size_t)(m1 - m0) * sb, hipMemcpyHostToDevice, s));
            st.bytes_h2d += (double)(m1 - m0) * sb;
            if ((e = grad(m0, o0, o1)) != CT_OK) return e;
            double d = 0.0;
            if ((e = dot_host(gbuf, (o1 - o0) * slice, d)) != CT_OK) return e;
            gg += d;
            if (step == 0) {
                if ((e = dot_host(xbuf + (o0 - m0) * slice, (o1 - o0) * slice, d)) != CT_OK) return e;
                xx += d;
            }
        }
        if (step == 0) alpha = lambda * std::sqrt(xx);
        if (tv_verbose()) {
            std::fprintf(stderr, "[ct ooc tv] step %d: norms done at %.1f s\n", step + 1,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
            std::fflush(stderr);
        }
        const double hs[4] = {xx, alpha, gg, 0.0};
        CT_HIP(hipMemcpyAsync(dscal, hs, sizeof(hs), hipMemcpyHostToDevice, s));
        for (int64_t n = 0; n < nsp; ++n) {  // pass 2: update
            int64_t o0, o1, m0, m1;
            bounds(n, o0, o1, m0, m1);
            CT_HIP(hipMemcpyAsync(xbuf, hx + m0 * slice, (size_t)(m1 - m0) * sb, hipMemcpyHostToDevice, s));
            st.bytes_h2d += (double)(m1 - m0) * sb;
            if (n > 0) CT_HIP(hipMemcpyAsync(xbuf, saved.p, (size_t)sb, hipMemcpyDeviceToDevice, s));
            if (n + 1 < nsp)
                CT_HIP(hipMemcpyAsync(saved.p, xbuf + (o1 - 1 - m0) * slice, (size_t)sb, hipMemcpyDeviceToDevice, s));
            if ((e = grad(m0, o0, o1)) != CT_OK) return e;
            const int64_t nown = (o1 - o0) * slice;
            hipLaunchKernelGGL(k_tv_update, dim3(ew_grid(nown)), dim3(EW_THREADS), 0, s, xbuf + (o0 - m0) * slice,
                               (const float *)gbuf, (const double *)dscal, nown);
            CT_HIP(hipGetLastError());
            CT_HIP(hipMemcpyAsync(hx + o0 * slice, xbuf + (o0 - m0) * slice, (size_t)nown * 4, hipMemcpyDeviceToHost,
                                  s));
            CT_HIP(hipStreamSynchronize(s));
            st.bytes_d2h += (double)nown * 4;
        }
        if (tv_verbose()) {
            std::fprintf(stderr, "[ct ooc tv] step %d: update done at %.1f s\n", step + 1,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
            std::fflush(stderr);
        }
    }
    CT_HIP(hipStreamSynchronize(s));
    st.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = st;
    return CT_OK;
}


// The splitting of Section 2.3: each slab carries `depth` halo slices of its neighbours on either
// side and takes up to `depth` steps on its own copy before the slabs exchange anything.  A halo
// slice stops being exact one step after its outer neighbour, so the gradient is computed on a
// region that shrinks by a slice per step at each inner boundary and always covers the slab's own
// slices.  Each step's ||g||^2 is the slab's own sum scaled by (image slices / slab slices), the
// uniform-distribution estimate, so no norm is exchanged; alpha = lambda ||x_in|| comes from one
// pass over the whole image first.  In a round every slab starts from the image as it stood at the
// round's start: the lower halo is a device copy of the slices below, taken before their update.
ct_status tv_host_run_halo(const ct_geometry &g, float *hx, int32_t nsteps, double lambda, double eps, int32_t depth,
                           uint64_t cap, ct_ooc_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    const int nx = (int)g.nVoxel[0], ny = (int)g.nVoxel[1];
    const int64_t nz = g.nVoxel[2];
    const int64_t d = depth;
    const int64_t slice = (int64_t)nx * ny;
    const uint64_t sb = (uint64_t)slice * sizeof(float);
    const uint64_t fixed = TV_RESERVE + align256(DOT_BLOCKS * 8) + align256(4 * 8);
    // device: the slab with its halos, the gradient of the same, `depth` saved slices
    if (cap <= fixed || (cap - fixed) / sb < (uint64_t)(5 * d + 2))
        return fail(CT_ERR_CAP, "device memory cap is below one slab slice plus halos and buffers");
    int64_t h = (int64_t)(((cap - fixed) / sb - 5 * d) / 2);
    h = std::max<int64_t>(1, std::min<int64_t>(h, nz));
    const int64_t nsp = (nz + h - 1) / h;
    h = (nz + nsp - 1) / nsp;
    ct_ooc_stats st;
    std::memset(&st, 0, sizeof(st));
    st.n_slabs = (int32_t)nsp;
    st.slab_slices = (int32_t)h;
    OwnStream S;
    CT_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
    DevMem xb, gb, saved, parts, scal;
    CT_HIP(CT_MALLOC(&xb.p, (size_t)(h + 2 * d) * sb));
    CT_HIP(CT_MALLOC(&gb.p, (size_t)(h + 2 * d) * sb));
    CT_HIP(CT_MALLOC(&saved.p, (size_t)d * sb));
    CT_HIP(CT_MALLOC(&parts.p, DOT_BLOCKS * 8));
    CT_HIP(CT_MALLOC(&scal.p, 4 * 8));
    float *xbuf = (float *)xb.p, *gbuf = (float *)gb.p, *sbuf = (float *)saved.p;
    double *dscal = (double *)scal.p;
    const hipStream_t s = S.s;
    ct_status e = CT_OK;
    // alpha from ||x_in||, summed slab by slab in FP64
    double xx = 0.0;
    for (int64_t n = 0; n < nsp; ++n) {
        const int64_t o0 = n * h, o1 = std::min(nz, o0 + h);
        CT_HIP(hipMemcpyAsync(xbuf, hx + o0 * slice, (size_t)(o1 - o0) * sb, hipMemcpyHostToDevice, s));
        st.bytes_h2d += (double)(o1 - o0) * sb;
        if ((e = dot_f64(xbuf, xbuf, CT_F32, (o1 - o0) * slice, dscal + 3, (double *)parts.p, s)) != CT_OK) return e;
        double v = 0.0;
        CT_HIP(hipMemcpyAsync(&v, dscal + 3, 8, hipMemcpyDeviceToHost, s));
        CT_HIP(hipStreamSynchronize(s));
        xx += v;
    }
    const double hs[4] = {xx, lambda * std::sqrt(xx), 0.0, 0.0};
    CT_HIP(hipMemcpyAsync(dscal, hs, sizeof(hs), hipMemcpyHostToDevice, s));
    CT_HIP(hipStreamSynchronize(s));
    for (int32_t done = 0; done < nsteps;) {
        const int64_t k = std::min<int64_t>(d, nsteps - done);
        for (int64_t n = 0; n < nsp; ++n) {
            const int64_t o0 = n * h, o1 = std::min(nz, o0 + h);
            const int64_t m0 = std::max<int64_t>(0, o0 - d), m1 = std::min(nz, o1 + d);
            CT_HIP(hipMemcpyAsync(xbuf + (o0 - m0) * slice, hx + o0 * slice, (size_t)(m1 - o0) * sb,
                                  hipMemcpyHostToDevice, s));
            st.bytes_h2d += (double)(m1 - o0) * sb;
            if (o0 > m0) CT_HIP(hipMemcpyAsync(xbuf, sbuf, (size_t)(o0 - m0) * sb, hipMemcpyDeviceToDevice, s));
            if (n + 1 < nsp) {  // the next slab's lower halo, as it stands at the round's start
                const int64_t n0 = std::max<int64_t>(0, o1 - d);
                CT_HIP(hipMemcpyAsync(sbuf, xbuf + (n0 - m0) * slice, (size_t)(o1 - n0) * sb, hipMemcpyDeviceToDevice,
                                      s));
            }
            const int64_t nown = (o1 - o0) * slice;
            for (int64_t i = 0; i < k; ++i) {
                const int64_t r0 = m0 == 0 ? 0 : m0 + i + 1, r1 = m1 == nz ? nz : m1 - i - 1;
                if ((e = launch_tv_grad((const float *)xbuf, gbuf, nx, ny, (int)nz, (float)eps, m0, r0, r1 - r0, s)) !=
                    CT_OK)
                    return e;
                if ((e = dot_f64(gbuf + (o0 - r0) * slice, gbuf + (o0 - r0) * slice, CT_F32, nown, dscal + 2,
                                 (double *)parts.p, s)) != CT_OK)
                    return e;
                hipLaunchKernelGGL(k_scale_entry, dim3(1), dim3(1), 0, s, dscal + 2, (double)nz / (double)(o1 - o0));
                CT_HIP(hipGetLastError());
                const int64_t nr = (r1 - r0) * slice;
                hipLaunchKernelGGL(k_tv_update, dim3(ew_grid(nr)), dim3(EW_THREADS), 0, s, xbuf + (r0 - m0) * slice,
                                   (const float *)gbuf, (const double *)dscal, nr);
                CT_HIP(hipGetLastError());
            }
            CT_HIP(hipMemcpyAsync(hx + o0 * slice, xbuf + (o0 - m0) * slice, (size_t)nown * 4, hipMemcpyDeviceToHost,
                                  s));
            CT_HIP(hipStreamSynchronize(s));
            st.bytes_d2h += (double)nown * 4;
        }
        done += (int32_t)k;
        if (tv_verbose()) {
            std::fprintf(stderr, "[ct ooc tv] %d of %d steps done at %.1f s\n", done, nsteps,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
            std::fflush(stderr);
        }
    }
    st.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = st;
    return CT_OK;
}

// The ROF iteration of rof_run on an image in host memory (Section 2.3: the minimiser holds five
// image copies, f, the dual field p and w, and its image splits stream through host memory).  The
// dual field lives in the caller's host workspace (three images).  Rounds of up to `depth`
// iterations: each slab uploads f and p over its slices with `depth` halo slices below and
// depth + 1 above, iterates on its copy with the copy's ends treated as the image's ends, and writes
// back its own slices of p.  A wrong end value spoils one more slice per iteration (two at the upper
// end in the first, where the forward difference reads the slice above), so the own slices equal
// the whole-image iteration bit for bit: the step needs no sum over the image.  In a round every
// slab starts from the state at the round's start: its lower halo is a device copy of the slices
// below, taken before their update.  A last pass forms u = f - lam div p slab by slab.
size_t rof_host_workspace(const ct_geometry &g) {
    return (size_t)3 * g.nVoxel[0] * g.nVoxel[1] * g.nVoxel[2] * sizeof(float);
}

ct_status rof_host_run(const ct_geometry &g, float *hx, int32_t niter, double lambda, double tau, int32_t depth,
                       float *hp, uint64_t cap, ct_ooc_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    const int nx = (int)g.nVoxel[0], ny = (int)g.nVoxel[1];
    const int64_t nz = g.nVoxel[2];
    const int64_t d = depth;
    const int64_t slice = (int64_t)nx * ny;
    const int64_t nvox = slice * nz;
    const uint64_t sb = (uint64_t)slice * sizeof(float);
    // device: f, px, py, pz and w over the slab with its halos, and the next slab's lower halo of p
    const uint64_t avail = cap > TV_RESERVE ? (cap - TV_RESERVE) / sb : 0;
    if (avail < (uint64_t)(5 * (2 * d + 2) + 3 * d))
        return fail(CT_ERR_CAP, "device memory cap is below one slab slice plus halos and buffers");
    int64_t h = (int64_t)((avail - 3 * d) / 5) - 2 * d - 1;
    h = std::max<int64_t>(1, std::min<int64_t>(h, nz));
    const int64_t nsp = (nz + h - 1) / h;
    h = (nz + nsp - 1) / nsp;
    const int64_t L = std::min<int64_t>(nz, h + 2 * d + 1);  // slices of the largest copy
    ct_ooc_stats st;
    std::memset(&st, 0, sizeof(st));
    st.n_slabs = (int32_t)nsp;
    st.slab_slices = (int32_t)h;
    OwnStream S;
    CT_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
    DevMem fm, pm[3], wm, sm;
    CT_HIP(CT_MALLOC(&fm.p, (size_t)L * sb));
    for (auto &b : pm) CT_HIP(CT_MALLOC(&b.p, (size_t)L * sb));
    CT_HIP(CT_MALLOC(&wm.p, (size_t)L * sb));
    CT_HIP(CT_MALLOC(&sm.p, (size_t)3 * d * sb));
    float *fb = (float *)fm.p, *wb = (float *)wm.p, *sv = (float *)sm.p;
    float *pb[3] = {(float *)pm[0].p, (float *)pm[1].p, (float *)pm[2].p};
    const hipStream_t s = S.s;
    auto up = [&](float *dst, const float *src, int64_t n_sl) -> ct_status {
        if (n_sl <= 0) return CT_OK;
        CT_HIP(hipMemcpyAsync(dst, src, (size_t)n_sl * sb, hipMemcpyHostToDevice, s));
        st.bytes_h2d += (double)n_sl * sb;
        return CT_OK;
    };
    auto down = [&](float *dst, const float *src, int64_t n_sl) -> ct_status {
        CT_HIP(hipMemcpyAsync(dst, src, (size_t)n_sl * sb, hipMemcpyDeviceToHost, s));
        st.bytes_d2h += (double)n_sl * sb;
        return CT_OK;
    };
    ct_status e = CT_OK;
    bool first = true;
    for (int32_t done = 0; done < niter;) {
        const int64_t k = std::min<int64_t>(d, niter - done);
        for (int64_t n = 0; n < nsp; ++n) {
            const int64_t o0 = n * h, o1 = std::min(nz, o0 + h);
            const int64_t m0 = std::max<int64_t>(0, o0 - d), m1 = std::min(nz, o1 + d + 1), len = m1 - m0;
            if ((e = up(fb, hx + m0 * slice, len)) != CT_OK) return e;
            for (int c = 0; c < 3; ++c) {
                if (first) {  // p = 0 at the start
                    hipLaunchKernelGGL(k_fill_zero, dim3(ew_grid(len * slice)), dim3(EW_THREADS), 0, s, pb[c], len * slice);
                    CT_HIP(hipGetLastError());
                } else {
                    if ((e = up(pb[c] + (o0 - m0) * slice, hp + c * nvox + o0 * slice, m1 - o0)) != CT_OK) return e;
                    if (o0 > m0)
                        CT_HIP(hipMemcpyAsync(pb[c], sv + c * d * slice, (size_t)(o0 - m0) * sb, hipMemcpyDeviceToDevice, s));
                }
                if (n + 1 < nsp) {  // the next slab's lower halo, as it stands at the round's start
                    const int64_t n0 = std::max<int64_t>(0, o1 - d);
                    CT_HIP(hipMemcpyAsync(sv + c * d * slice, pb[c] + (n0 - m0) * slice, (size_t)(o1 - n0) * sb,
                                          hipMemcpyDeviceToDevice, s));
                }
            }
            const dim3 grid((nx + 63) / 64, (ny + 3) / 4, (unsigned)len);
            for (int64_t i = 0; i < k; ++i) {
                hipLaunchKernelGGL(k_rof_w, grid, dim3(256), 0, s, (const float *)fb, pb[0], pb[1], pb[2], wb, nx, ny,
                                   (int)len, (float)(1.0 / lambda));
                hipLaunchKernelGGL(k_rof_p, grid, dim3(256), 0, s, (const float *)wb, pb[0], pb[1], pb[2], nx, ny,
                                   (int)len, (float)tau);
                CT_HIP(hipGetLastError());
            }
            for (int c = 0; c < 3; ++c)
                if ((e = down(hp + c * nvox + o0 * slice, pb[c] + (o0 - m0) * slice, o1 - o0)) != CT_OK) return e;
            CT_HIP(hipStreamSynchronize(s));
        }
        first = false;
        done += (int32_t)k;
        if (tv_verbose()) {
            std::fprintf(stderr, "[ct ooc rof] %d of %d iterations done at %.1f s\n", done, niter,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
            std::fflush(stderr);
        }
    }
    // u = f - lam div p: the divergence at a slice reads p there and one slice below, and is the
    // interior form only below the copy's top, so each slab takes one slice either side
    for (int64_t n = 0; n < nsp; ++n) {
        const int64_t o0 = n * h, o1 = std::min(nz, o0 + h);
        const int64_t m0 = std::max<int64_t>(0, o0 - 1), m1 = std::min(nz, o1 + 1), len = m1 - m0;
        if ((e = up(fb, hx + m0 * slice, len)) != CT_OK) return e;
        for (int c = 0; c < 3; ++c) {
            if (niter == 0) {
                hipLaunchKernelGGL(k_fill_zero, dim3(ew_grid(len * slice)), dim3(EW_THREADS), 0, s, pb[c], len * slice);
                CT_HIP(hipGetLastError());
            } else if ((e = up(pb[c], hp + c * nvox + m0 * slice, len)) != CT_OK) {
                return e;
            }
        }
        const dim3 grid((nx + 63) / 64, (ny + 3) / 4, (unsigned)len);
        hipLaunchKernelGGL(k_rof_u, grid, dim3(256), 0, s, fb, pb[0], pb[1], pb[2], nx, ny, (int)len, (float)lambda);
        CT_HIP(hipGetLastError());
        if ((e = down(hx + o0 * slice, fb + (o0 - m0) * slice, o1 - o0)) != CT_OK) return e;
        CT_HIP(hipStreamSynchronize(s));
    }
    st.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = st;
    return CT_OK;
}

}  // namespace ct
