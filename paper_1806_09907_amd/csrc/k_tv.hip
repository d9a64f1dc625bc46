// Total-variation regularisers (Sec. III-F) on a dense displacement u:
//   anisotropic: R = (1/|X_R|) sum_{x in X_R} sum_c sum_a |D_a u_c(x)|
//   isotropic:   R = (1/|X_R|) sum_{x in X_R} sqrt(sum_c sum_a D_a u_c(x)^2)
// with the forward differences D_a u_c(x) = u_c(x + e_a) - u_c(x) over
// X_R = prod_a [0, n_a - 2] (the diffusion term's discretisation) and the
// subgradient 0 where a term is 0. One thread per voxel x writes
//   dR/du_c(x) = (1/|X_R|) (sum_a [x - e_a in X_R] k_ca(x - e_a)
//                           - [x in X_R] sum_a k_ca(x)),
// k = sign(D) (anisotropic) or D / ||J|| (isotropic), where J(y) is the
// matrix of differences at y. The Gram form of the diffusion term has no TV
// counterpart, so a B-spline field is expanded to the voxel grid first.
#include "device_common.h"

namespace air {

namespace {

constexpr int kTvBlocks = 4096;

__host__ inline int tv_grid(long long n) {
    const long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < kTvBlocks ? (b < 1 ? 1 : b) : kTvBlocks);
}

// k_ca(y) for every c, a at a point y of X_R; returns the term's value at y.
template <int DIM, int KIND>
__device__ inline float tv_coef(const float* __restrict__ u, long long N, const long long* st,
                                long long y, float (*k)[3]) {
    float D[3][3];
    float ss = 0.f, l1 = 0.f;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const float u0 = u[c * N + y];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            D[c][a] = u[c * N + y + st[a]] - u0;
            ss += D[c][a] * D[c][a];
            l1 += fabsf(D[c][a]);
        }
    }
    if (KIND == AIR_REG_ANISO_TV) {
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                k[c][a] = D[c][a] > 0.f ? 1.f : (D[c][a] < 0.f ? -1.f : 0.f);
        return l1;
    }
    const float nrm = sqrtf(ss);
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int a = 0; a < DIM; ++a) k[c][a] = D[c][a] * inv;
    return nrm;
}

// grad (+)= scale * dR/du; partial[block] = sum over the block's voxels in X_R
// of the term (FP64).
template <int DIM, int KIND>
__global__ void __launch_bounds__(kBlock)
k_tv(const PairDesc P, const float* __restrict__ u, float scale, float* __restrict__ grad,
     int accumulate, double* __restrict__ partial) {
    __shared__ double red[8 * (kBlock / 64)];
    const long long N = P.nvox;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const long long st[3] = {1, nx, (long long)nx * ny};
    const float inv_xr = P.inv_xr;
    double acc[1] = {0.0};
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < N;
         v += (long long)gridDim.x * kBlock) {
        const int x[3] = {(int)(v % nx), (int)((v / nx) % ny),
                          DIM == 3 ? (int)(v / ((long long)nx * ny)) : 0};
        const int n[3] = {nx, ny, nz};
        bool in_r = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            if (x[a] > n[a] - 2) in_r = false;
        float g[3] = {0.f, 0.f, 0.f};
        float k[3][3];
        if (in_r) {
            acc[0] += (double)tv_coef<DIM, KIND>(u, N, st, v, k);
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int a = 0; a < DIM; ++a) g[c] -= k[c][a];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            // the term at y = x - e_a, if y is in X_R
            bool prev = x[a] >= 1;
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                const int yb = x[b] - (b == a ? 1 : 0);
                if (yb > n[b] - 2) prev = false;
            }
            if (!prev) continue;
            tv_coef<DIM, KIND>(u, N, st, v - st[a], k);
#pragma unroll
            for (int c = 0; c < DIM; ++c) g[c] += k[c][a];
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float val = scale * inv_xr * g[c];
            grad[c * N + v] = accumulate ? grad[c * N + v] + val : val;
        }
    }
    block_sum<kBlock, 1>(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// *value (+)= weight * (sum of the partials) / |X_R|, in block order.
__global__ void __launch_bounds__(kBlock)
k_tv_value(const double* __restrict__ partial, int nblk, float inv_xr, float weight, float* value,
           int accumulate) {
    __shared__ double red[8 * (kBlock / 64)];
    double s[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += kBlock) s[0] += partial[b];
    block_sum<kBlock, 1>(s, red);
    if (threadIdx.x == 0) {
        const float r = (float)((double)weight * s[0] * (double)inv_xr);
        *value = accumulate ? *value + r : r;
    }
}

}  // namespace

// grad (+)= scale * dR/du and *value (+)= weight * R for the plan's TV kind.
// partial: at least tv_partials() doubles of workspace.
int tv_partials() { return kTvBlocks; }

hipError_t launch_tv(const PairDesc& P, int dim, int kind, const float* u, float scale,
                     float* grad, bool accumulate_grad, double* partial, float weight,
                     float* value, bool accumulate_value, hipStream_t s) {
    const int g = tv_grid(P.nvox);
    const int acc = accumulate_grad ? 1 : 0;
    if (dim == 3) {
        if (kind == AIR_REG_ANISO_TV)
            hipLaunchKernelGGL((k_tv<3, AIR_REG_ANISO_TV>), dim3(g), dim3(kBlock), 0, s, P, u,
                               scale, grad, acc, partial);
        else
            hipLaunchKernelGGL((k_tv<3, AIR_REG_ISO_TV>), dim3(g), dim3(kBlock), 0, s, P, u,
                               scale, grad, acc, partial);
    } else {
        if (kind == AIR_REG_ANISO_TV)
            hipLaunchKernelGGL((k_tv<2, AIR_REG_ANISO_TV>), dim3(g), dim3(kBlock), 0, s, P, u,
                               scale, grad, acc, partial);
        else
            hipLaunchKernelGGL((k_tv<2, AIR_REG_ISO_TV>), dim3(g), dim3(kBlock), 0, s, P, u,
                               scale, grad, acc, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tv_value, dim3(1), dim3(kBlock), 0, s, partial, g, P.inv_xr, weight,
                       value, accumulate_value ? 1 : 0);
    return hipGetLastError();
}

}  // namespace air
