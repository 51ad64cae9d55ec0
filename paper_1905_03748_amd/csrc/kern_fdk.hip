// FDK reconstruction (Feldkamp, Davis & Kress 1984; the algorithm the FDK-weighted voxel
// backprojector of Section 2.2 belongs to) for a full circular scan: cosine weighting and ramp
// filtering of every detector row, then the FDK-weighted backprojection of the filtered rows.
//
// Filter: the band-limited ramp (Ram-Lak) sampled at the pixel spacing scaled to the rotation
// axis, ds = du DSO / DSD.  Its taps are 1/4 at offset 0, 0 at even offsets and -1/(pi n)^2 at odd
// offsets n (in units of 1/ds^2); the convolution runs over the whole row with zero extension (no
// periodic wrap).  Each output is scaled by dtheta / (2 ds), dtheta = 2 pi / N_angles, the 1/2
// because a full turn measures every line twice.
#include <cmath>

#include "dev_common.hpp"

namespace ct {

namespace {

constexpr int FDK_MAX_NU = 4096;
constexpr int FDK_MAX_THREADS = 512;
constexpr float PI2F = 9.8696044010893586f;  // pi^2

// Sizes of one launch.  Each thread forms 8 consecutive outputs of a row (a group); a row's
// groups take gw threads (a whole number of waves) and a block holds `rows` such rows.  The
// weighted row sits in LDS at offset e between zero pads: [0, e) and [e + nu, 2e + 8 groups), e the
// row length rounded up to a multiple of 8, so every read below is in range without a test.
struct FdkShape {
    int groups, gw, rows, e, rw, ntaps;
    __host__ __device__ explicit FdkShape(int nu) {
        groups = (nu + 7) / 8;
        gw = (groups + 63) / 64 * 64;
        rows = gw >= 256 ? 1 : 256 / gw;
        e = nu > 1 ? (nu - 1 + 7) / 8 * 8 : 0;
        rw = 2 * e + 8 * groups;
        ntaps = e / 2 + 8;
    }
    __host__ __device__ size_t lds_bytes() const { return (size_t)(ntaps + rows * rw) * sizeof(float); }
};

// One row per gw threads.  Thread g of a row forms outputs a0 + j, a0 = 8 g, j < 8:
//   q[a] = scale * (p[a] / 4 + sum_{odd n} h_n (p[a - n] + p[a + n])),  h_n = -1/(pi n)^2.
// The inputs a0 .. a0 + 7 (offsets up to 7 from every output) come first; then pairs of inputs
// at increasing distance on each side, 4 pairs per step: the left pair a0 - 2k - 1, a0 - 2k - 2
// feeds the even and odd outputs with the taps h_{2(k + i) + 1}, the right pair a0 + 2k + 8,
// a0 + 2k + 9 the odd and even outputs, so one step reads 16 inputs (four 16-byte LDS loads) and
// the 8 taps h_{2k+1} .. h_{2k+15} (two broadcast loads) for 64 fused multiply-adds.  FP32.
template <typename T>
__global__ __launch_bounds__(FDK_MAX_THREADS) void k_fdk_filter(const T *__restrict__ proj, float *__restrict__ q,
                                                                int64_t nrows, int nu, int nv, float dsd, float u0,
                                                                float du, float v0, float dv, float scale) {
    extern __shared__ float4 lds4[];
    float *lds = (float *)lds4;
    const FdkShape sh(nu);
    float *taps = lds;
    for (int m = threadIdx.x; m < sh.ntaps; m += blockDim.x) {
        const float n = (float)(2 * m + 1);
        taps[m] = -1.0f / (PI2F * (n * n));
    }
    const int lr = threadIdx.x / sh.gw, g = threadIdx.x % sh.gw;
    const int64_t r = (int64_t)blockIdx.x * sh.rows + lr;
    float *row = lds + sh.ntaps + lr * sh.rw;
    if (r < nrows) {
        const T *src = proj + r * nu;
        const float vv = fmaf((float)(r % nv), dv, v0);
        const float d2 = fmaf(dsd, dsd, vv * vv);
        for (int i = g; i < sh.rw; i += sh.gw) {
            const int a = i - sh.e;
            float val = 0.0f;
            if (a >= 0 && a < nu) {
                const float uu = fmaf((float)a, du, u0);
                val = to_f(src[a]) * (dsd / sqrtf(fmaf(uu, uu, d2)));
            }
            row[i] = val;
        }
    }
    __syncthreads();
    if (r >= nrows || g >= sh.groups) return;
    const int a0 = 8 * g;
    const float *c = row + sh.e + a0;
    float acc[8];
    {
        const float4 x0 = *(const float4 *)c, x1 = *(const float4 *)(c + 4);
        const float4 t0 = *(const float4 *)taps;
        const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        const float h[4] = {t0.x, t0.y, t0.z, t0.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float s = 0.25f * x[j];
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int n = j > d ? j - d : d - j;
                if (n & 1) s = fmaf(h[(n - 1) / 2], x[d], s);
            }
            acc[j] = s;
        }
    }
    for (int k = 0; k < sh.e / 2; k += 4) {
        const float4 ta = *(const float4 *)(taps + k), tb = *(const float4 *)(taps + k + 4);
        const float4 la = *(const float4 *)(c - 2 * k - 8), lb = *(const float4 *)(c - 2 * k - 4);
        const float4 ra = *(const float4 *)(c + 2 * k + 8), rb = *(const float4 *)(c + 2 * k + 12);
        const float tp[8] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
        const float in[8] = {la.x, la.y, la.z, la.w, lb.x, lb.y, lb.z, lb.w};
        const float rin[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const float x1 = in[7 - 2 * kk], x2 = in[6 - 2 * kk], y1 = rin[2 * kk], y2 = rin[2 * kk + 1];
            acc[0] = fmaf(tp[kk + 4], y2, fmaf(tp[kk], x1, acc[0]));
            acc[2] = fmaf(tp[kk + 3], y2, fmaf(tp[kk + 1], x1, acc[2]));
            acc[4] = fmaf(tp[kk + 2], y2, fmaf(tp[kk + 2], x1, acc[4]));
            acc[6] = fmaf(tp[kk + 1], y2, fmaf(tp[kk + 3], x1, acc[6]));
            acc[1] = fmaf(tp[kk + 3], y1, fmaf(tp[kk + 1], x2, acc[1]));
            acc[3] = fmaf(tp[kk + 2], y1, fmaf(tp[kk + 2], x2, acc[3]));
            acc[5] = fmaf(tp[kk + 1], y1, fmaf(tp[kk + 3], x2, acc[5]));
            acc[7] = fmaf(tp[kk], y1, fmaf(tp[kk + 4], x2, acc[7]));
        }
    }
    float *dst = q + r * nu + a0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (a0 + j < nu) dst[j] = acc[j] * scale;
}

}  // namespace

size_t fdk_workspace(const ct_plan *p) {
    const ct_geometry &g = p->g;
    return (size_t)p->angles.size() * g.nDetector[1] * g.nDetector[0] * sizeof(float);
}

ct_status fdk_filter(ct_plan *p, const void *proj, ct_dtype pt, float *q, int64_t a0, int64_t a1, hipStream_t st) {
    const ct_geometry &g = p->g;
    const int64_t nu = g.nDetector[0], nv = g.nDetector[1];
    if (nu > FDK_MAX_NU) return fail(CT_ERR_ARG, "ct_fdk: detector rows longer than 4096 pixels are not supported");
    const int64_t rows = (a1 - a0) * nv;
    if (rows > 0x7fffffff) return fail(CT_ERR_ARG, "ct_fdk: more than 2^31 - 1 detector rows in one call");
    const double ds = g.dDetector[0] * g.DSO / g.DSD;
    const double dtheta = 2.0 * M_PI / (double)p->angles.size();
    const float scale = (float)(dtheta / (2.0 * ds));
    const float u0 = (float)(-(nu - 1) / 2.0 * g.dDetector[0] + g.offDetector[0]);
    const float v0 = (float)(-(nv - 1) / 2.0 * g.dDetector[1] + g.offDetector[1]);
    const FdkShape sh((int)nu);
    const int64_t blocks = (rows + sh.rows - 1) / sh.rows;
    CT_DISPATCH1(pt, T,
                 hipLaunchKernelGGL((k_fdk_filter<T>), dim3((unsigned)blocks), dim3(sh.gw * sh.rows), sh.lds_bytes(), st,
                                    (const T *)proj, q, rows, (int)nu, (int)nv, (float)g.DSD, u0,
                                    (float)g.dDetector[0], v0, (float)g.dDetector[1], scale));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status fdk_run(ct_plan *p, const void *proj, ct_dtype pt, void *vol, ct_dtype vt, void *work, hipStream_t st) {
    const int64_t na = (int64_t)p->angles.size();
    float *q = (float *)work;
    if (!q) CT_HIP(CT_MALLOC_ASYNC((void **)&q, fdk_workspace(p), st));
    ct_status s = fdk_filter(p, proj, pt, q, 0, na, st);
    if (s == CT_OK) s = launch_backproject(p, CT_BP_FDK, q, CT_F32, vol, vt, 0, 0, na, full_slab(p->g), st);
    if (!work) (void)hipFreeAsync(q, st);
    return s;
}

}  // namespace ct
