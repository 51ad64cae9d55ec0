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
constexpr int FDK_THREADS = 256;
constexpr float PI2F = 9.8696044010893586f;  // pi^2

// One block per detector row (angle, v).  The cosine-weighted row sits in LDS between two zero
// pads of nu samples, so every offset up to nu - 1 on either side is in range without a test; the
// odd-offset taps sit after it.  Thread t forms the outputs a = t, t + blockDim, ...:
//   q[a] = scale * (p[a] / 4 + sum_{odd n} h_n (p[a - n] + p[a + n]))
// in FP32, from the centre outwards.  Consecutive lanes read consecutive LDS words (no bank
// conflicts); the tap is the same word for the whole wave (a broadcast).
template <typename T>
__global__ __launch_bounds__(FDK_THREADS) void k_fdk_filter(const T *__restrict__ proj, float *__restrict__ q, int nu,
                                                            int nv, float dsd, float u0, float du, float v0, float dv,
                                                            float scale) {
    extern __shared__ float lds[];
    float *row = lds;            // [0, nu) zero, [nu, 2 nu) weighted row, [2 nu, 3 nu) zero
    float *taps = lds + 3 * nu;  // taps[m] = h_{2m+1}, m < nu / 2
    const int64_t r = blockIdx.x;
    const int b = (int)(r % nv);
    const T *src = proj + r * nu;
    const float vv = fmaf((float)b, dv, v0);
    const float d2 = fmaf(dsd, dsd, vv * vv);
    for (int a = threadIdx.x; a < nu; a += blockDim.x) {
        const float uu = fmaf((float)a, du, u0);
        row[a] = 0.0f;
        row[nu + a] = to_f(src[a]) * (dsd / sqrtf(fmaf(uu, uu, d2)));
        row[2 * nu + a] = 0.0f;
    }
    const int M = nu >> 1;
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        const float n = (float)(2 * m + 1);
        taps[m] = -1.0f / (PI2F * (n * n));
    }
    __syncthreads();
    float *dst = q + r * nu;
    for (int a = threadIdx.x; a < nu; a += blockDim.x) {
        const float *c = row + nu + a;
        float acc = 0.25f * c[0];
#pragma unroll 4
        for (int m = 0; m < M; ++m) {
            const int n = 2 * m + 1;
            acc = fmaf(taps[m], c[-n] + c[n], acc);
        }
        dst[a] = acc * scale;
    }
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
    const int threads = (int)std::min<int64_t>(FDK_THREADS, (nu + 63) / 64 * 64);
    const size_t lds = (size_t)(3 * nu + nu / 2) * sizeof(float);
    CT_DISPATCH1(pt, T,
                 hipLaunchKernelGGL((k_fdk_filter<T>), dim3((unsigned)rows), dim3(threads), lds, st, (const T *)proj, q,
                                    (int)nu, (int)nv, (float)g.DSD, u0, (float)g.dDetector[0], v0,
                                    (float)g.dDetector[1], scale));
    CT_HIP(hipGetLastError());
    return CT_OK;
}

ct_status fdk_run(ct_plan *p, const void *proj, ct_dtype pt, void *vol, ct_dtype vt, void *work, hipStream_t st) {
    const int64_t na = (int64_t)p->angles.size();
    float *q = (float *)work;
    if (!q) CT_HIP(hipMallocAsync((void **)&q, fdk_workspace(p), st));
    ct_status s = fdk_filter(p, proj, pt, q, 0, na, st);
    if (s == CT_OK) s = launch_backproject(p, CT_BP_FDK, q, CT_F32, vol, vt, 0, 0, na, full_slab(p->g), st);
    if (!work) (void)hipFreeAsync(q, st);
    return s;
}

}  // namespace ct
