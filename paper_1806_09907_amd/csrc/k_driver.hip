// Multi-resolution helpers for the registration driver: one Gaussian
// pyramid level (separable blur with clamped borders, every second voxel)
// and the linear transfer of a displacement field to a finer grid.
#include <math.h>

#include "device_common.h"

namespace air {

constexpr int kMaxTaps = 64;

struct GaussTaps {
    float w[kMaxTaps];
    int r;
};

// Blur along `axis` of a [n2][n1][n0] volume (axis 0 = x) and keep every
// second sample along that axis: out extent (n_axis + 1) / 2.
__global__ void __launch_bounds__(kBlock)
k_blur_decimate(const float* __restrict__ in, float* __restrict__ out, int n0, int n1, int n2,
                int axis, GaussTaps g) {
    const int n[3] = {n0, n1, n2};
    int m[3] = {n0, n1, n2};
    m[axis] = (n[axis] + 1) / 2;
    const long long M = (long long)m[0] * m[1] * m[2];
    const long long stride = axis == 0 ? 1 : (axis == 1 ? (long long)n0 : (long long)n0 * n1);
    for (long long o = (long long)blockIdx.x * kBlock + threadIdx.x; o < M;
         o += (long long)gridDim.x * kBlock) {
        int q[3];
        q[0] = (int)(o % m[0]);
        q[1] = (int)((o / m[0]) % m[1]);
        q[2] = (int)(o / ((long long)m[0] * m[1]));
        int p[3] = {q[0], q[1], q[2]};
        p[axis] = 2 * q[axis];
        const long long base = ((long long)p[2] * n1 + p[1]) * n0 + p[0];
        float acc = 0.f;
        for (int k = -g.r; k <= g.r; ++k) {
            int t = p[axis] + k;
            t = t < 0 ? 0 : (t > n[axis] - 1 ? n[axis] - 1 : t);
            acc += g.w[k + g.r] * in[base + (long long)(t - p[axis]) * stride];
        }
        out[o] = acc;
    }
}

__global__ void __launch_bounds__(kBlock)
k_field_resample(const float* __restrict__ in, int n0, int n1, int n2, float* __restrict__ out,
                 int m0, int m1, int m2) {
    const int n[3] = {n0, n1, n2}, m[3] = {m0, m1, m2};
    const long long Nn = (long long)n0 * n1 * n2, Nm = (long long)m0 * m1 * m2;
    for (long long o = (long long)blockIdx.x * kBlock + threadIdx.x; o < Nm;
         o += (long long)gridDim.x * kBlock) {
        const int idx[3] = {(int)(o % m0), (int)((o / m0) % m1), (int)(o / ((long long)m0 * m1))};
        int j[3];
        float f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // align-corners mapping; computed in double so the fraction is exact
            const double p = m[a] > 1 ? (double)idx[a] * (n[a] - 1) / (double)(m[a] - 1) : 0.0;
            int jj = (int)floor(p);
            jj = jj > n[a] - 2 ? n[a] - 2 : (jj < 0 ? 0 : jj);
            j[a] = jj;
            f[a] = (float)(p - jj);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float* src = in + c * Nn;
            float acc = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int bx = q & 1, by = (q >> 1) & 1, bz = (q >> 2) & 1;
                const float w = (bx ? f[0] : 1.f - f[0]) * (by ? f[1] : 1.f - f[1]) *
                                (bz ? f[2] : 1.f - f[2]);
                acc += w * src[((long long)(j[2] + bz) * n1 + j[1] + by) * n0 + j[0] + bx];
            }
            out[c * Nm + o] = acc;
        }
    }
}

static int grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 65536 ? b : 65536);
}

}  // namespace air

using namespace air;

extern "C" {

air_status air_pyramid_workspace_bytes(const int32_t n[3], size_t* bytes) {
    if (!n || !bytes) return AIR_ERR_INVALID_ARG;
    if (n[0] < 2 || n[1] < 2 || n[2] < 2) return AIR_ERR_SHAPE;
    const size_t a = (size_t)n[0] * n[1] * ((n[2] + 1) / 2);
    const size_t b = (size_t)n[0] * ((n[1] + 1) / 2) * ((n[2] + 1) / 2);
    *bytes = 4 * (((a + 63) & ~size_t(63)) + b);
    return AIR_OK;
}

air_status air_pyramid_down(const float* in, const int32_t n[3], float sigma, float* out,
                            void* ws, size_t ws_bytes, void* stream) {
    TraceRange trace_("air_pyramid_down");
    if (!in || !n || !out) return AIR_ERR_INVALID_ARG;
    if (!(sigma > 0.f) || (int)ceilf(3.f * sigma) * 2 + 1 > kMaxTaps) return AIR_ERR_INVALID_ARG;
    size_t need = 0;
    air_status st = air_pyramid_workspace_bytes(n, &need);
    if (st != AIR_OK) return st;
    if (!ws || ws_bytes < need) return AIR_ERR_WORKSPACE;
    if (((uintptr_t)in | (uintptr_t)out | (uintptr_t)ws) & 15u) return AIR_ERR_ALIGN;
    GaussTaps g{};
    g.r = (int)ceil(3.0 * sigma);
    double s = 0.0, w[kMaxTaps];
    for (int k = -g.r; k <= g.r; ++k) {
        w[k + g.r] = exp(-0.5 * (double)k * k / ((double)sigma * sigma));
        s += w[k + g.r];
    }
    for (int k = 0; k <= 2 * g.r; ++k) g.w[k] = (float)(w[k] / s);
    hipStream_t hs = (hipStream_t)stream;
    const size_t a = (size_t)n[0] * n[1] * ((n[2] + 1) / 2);
    float* t1 = static_cast<float*>(ws);
    float* t2 = t1 + ((a + 63) & ~size_t(63));
    const int nz2 = (n[2] + 1) / 2, ny2 = (n[1] + 1) / 2;
    hipLaunchKernelGGL(k_blur_decimate, dim3(grid_for((long long)a)), dim3(kBlock), 0, hs, in, t1,
                       n[0], n[1], n[2], 2, g);
    hipLaunchKernelGGL(k_blur_decimate, dim3(grid_for((long long)n[0] * ny2 * nz2)), dim3(kBlock),
                       0, hs, t1, t2, n[0], n[1], nz2, 1, g);
    hipLaunchKernelGGL(k_blur_decimate,
                       dim3(grid_for((long long)((n[0] + 1) / 2) * ny2 * nz2)), dim3(kBlock), 0,
                       hs, t2, out, n[0], ny2, nz2, 0, g);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_field_resample(const float* in, const int32_t n[3], const int32_t m[3], float* out,
                              void* stream) {
    TraceRange trace_("air_field_resample");
    if (!in || !n || !m || !out) return AIR_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 2 || m[a] < 1) return AIR_ERR_SHAPE;
    if (((uintptr_t)in | (uintptr_t)out) & 15u) return AIR_ERR_ALIGN;
    const long long Nm = (long long)m[0] * m[1] * m[2];
    hipLaunchKernelGGL(k_field_resample, dim3(grid_for(Nm)), dim3(kBlock), 0, (hipStream_t)stream,
                       in, n[0], n[1], n[2], out, m[0], m[1], m[2]);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

}  // extern "C"
