// Synthetic inputs on the device (not part of the registration method): the
// blob volumes of the 128^3 workloads, painted from parameters drawn on the
// host, and additive Gaussian noise from a counter-based generator, so that
// the thousands of training pairs of the learned initialisation are made
// without host round trips.
//
// Noise: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter is mixed with a
// 64-bit key by ten rounds of two 32x32->64 multiplications (multipliers
// 0xD2511F53 and 0xCD9E8D57), the key advancing by the Weyl constants
// 0x9E3779B9 and 0xBB67AE85 between rounds. Each counter value gives four
// 32-bit words, turned into four standard normal variates by the Box-Muller
// transform.
#include <math.h>

#include "device_common.h"

namespace air {

namespace {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c.x;
        const uint64_t p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// uniform in (0, 1) from the top 24 bits
__device__ inline float unit_open(uint32_t v) { return ((float)(v >> 8) + 0.5f) * 0x1p-24f; }

// out[v] = sum_b amp_b exp(-((x-cx)^2 + (y-cy)^2 + (z-cz)^2) / (2 sigma_b^2)),
// computed as a product of three 1D factors per blob. One block per (y, z)
// row; the y and z factors times the amplitude are formed once per block.
constexpr int kMaxBlobs = 256;
__global__ void __launch_bounds__(kBlock)
k_paint_blobs(const float* __restrict__ prm, int nb, int nx, int ny, int nz,
              float* __restrict__ out) {
    __shared__ float yz[kMaxBlobs];
    __shared__ float cx[kMaxBlobs], inv2s2[kMaxBlobs];
    const int row = blockIdx.x;
    const int y = row % ny, z = row / ny;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        const float* p = prm + b * 5;
        const float s = p[3];
        const float k = 0.5f / (s * s);
        const float dy = (float)y - p[1], dz = (float)z - p[2];
        yz[b] = p[4] * expf(-k * dy * dy) * expf(-k * dz * dz);
        cx[b] = p[0];
        inv2s2[b] = k;
    }
    __syncthreads();
    float* o = out + (long long)row * nx;
    for (int x = threadIdx.x; x < nx; x += kBlock) {
        float acc = 0.f;
        for (int b = 0; b < nb; ++b) {
            const float dx = (float)x - cx[b];
            acc += yz[b] * expf(-inv2s2[b] * dx * dx);
        }
        o[x] = acc;
    }
}

// x[i] += stddev * N_i, N_i the i-th normal variate of the stream `seed`:
// counter (i / 4, 0, 0, 0), key (seed low, seed high), word i % 4.
__global__ void __launch_bounds__(kBlock)
k_add_normal(float* __restrict__ x, long long n, uint32_t k0, uint32_t k1, float stddev) {
    const long long groups = (n + 3) / 4;
    for (long long g = (long long)blockIdx.x * kBlock + threadIdx.x; g < groups;
         g += (long long)gridDim.x * kBlock) {
        const U4 r = philox4x32_10(U4{(uint32_t)g, (uint32_t)(g >> 32), 0u, 0u}, k0, k1);
        const float u1 = unit_open(r.x), u2 = unit_open(r.y);
        const float u3 = unit_open(r.z), u4 = unit_open(r.w);
        const float ra = sqrtf(-2.f * logf(u1)), rb = sqrtf(-2.f * logf(u3));
        float sa, ca, sb, cb;
        sincosf(6.28318530717958647692f * u2, &sa, &ca);
        sincosf(6.28318530717958647692f * u4, &sb, &cb);
        const float v[4] = {ra * ca, ra * sa, rb * cb, rb * sb};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long i = 4 * g + j;
            if (i < n) x[i] += stddev * v[j];
        }
    }
}

}  // namespace

}  // namespace air

using namespace air;

extern "C" {

air_status air_synth_blobs(const float* params, int32_t nblobs, const int32_t dims[3], float* out,
                           void* stream) {
    if (!params || !dims || !out) return AIR_ERR_INVALID_ARG;
    if (nblobs < 0 || nblobs > kMaxBlobs) return AIR_ERR_SHAPE;
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > 65536) return AIR_ERR_SHAPE;
    const long long rows = (long long)dims[1] * dims[2];
    if (rows * dims[0] >= (1LL << 31)) return AIR_ERR_SHAPE;
    if (((uintptr_t)params | (uintptr_t)out) & 3u) return AIR_ERR_ALIGN;
    hipLaunchKernelGGL(k_paint_blobs, dim3((unsigned)rows), dim3(kBlock), 0, (hipStream_t)stream,
                       params, (int)nblobs, (int)dims[0], (int)dims[1], (int)dims[2], out);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_synth_add_normal(float* x, int64_t n, uint64_t seed, float stddev, void* stream) {
    if (!x || n < 0) return AIR_ERR_INVALID_ARG;
    if (((uintptr_t)x) & 3u) return AIR_ERR_ALIGN;
    if (n == 0) return AIR_OK;
    const long long groups = (n + 3) / 4;
    const long long nb = (groups + kBlock - 1) / kBlock;
    const int grid = (int)(nb < 8192 ? nb : 8192);
    hipLaunchKernelGGL(k_add_normal, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, x,
                       (long long)n, (uint32_t)seed, (uint32_t)(seed >> 32), stddev);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

}  // extern "C"
