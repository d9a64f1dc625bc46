// Wendland basis (Sec. III-C, psi_{3,2} with a support radius sigma per axis)
// expanded onto the voxel grid, u = B theta (Sec. II-A eq. kernel_basis), and
// its transpose, B^T g.
//
// Control j sits at (j - m) delta on each axis, so the lattice is aligned
// with voxel cells of size delta: voxel x = c delta + r (cell c, phase r in
// [0, delta)) sees exactly the controls j = c + qq, qq in [0, K), with the
// weight W[qq][r] = psi(||(r - (qq - m) delta) / sigma||), the same for
// every cell. Both directions are therefore per-cell contractions with one
// fixed table, built once per plan on the host:
//   expand:    u(c, r) = sum_qq W[qq][r] theta(c + qq)
//   transpose: H(qq, c) = sum_r W[qq][r] g(c, r);
//              out(j)   = sum_qq H(j - qq, qq)   over cells inside the grid.
// No kernel value is evaluated on the device.
#include "device_common.h"

namespace air {

namespace {

constexpr int kWCells = 8;   // cells along x per wave (both contractions)
constexpr int kWaves = kBlock / 64;

// theta -> zero-padded copy [d][ncp_z][ncp_y][ncp_x], scaled.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_pad(const PairDesc P, const float* __restrict__ theta, float scale,
           float* __restrict__ thp) {
    const long long nx = P.wncp[0], ny = P.wncp[1], nz = P.wncp[2];
    const long long tot = DIM * nx * ny * nz;
    const long long NC = (long long)P.nc[0] * P.nc[1] * P.nc[2];
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < tot;
         i += (long long)gridDim.x * kBlock) {
        const int jx = (int)(i % nx);
        const int jy = (int)((i / nx) % ny);
        const long long rest = i / (nx * ny);
        const int jz = (int)(rest % nz);
        const int c = (int)(rest / nz);
        float v = 0.f;
        if (jx < P.nc[0] && jy < P.nc[1] && jz < P.nc[2])
            v = scale * theta[c * NC + ((long long)jz * P.nc[1] + jy) * P.nc[0] + jx];
        thp[i] = v;
    }
}

// u(c, r) = sum_qq W[qq][r] thp(c + qq). One wave owns kWCells cells along x
// of one (cy, cz) row and 64 consecutive phases; theta is read wave-uniformly.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_expand(const PairDesc P, const float* __restrict__ W, const float* __restrict__ thp,
              float* __restrict__ u) {
    const int lane = threadIdx.x & 63;
    const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    const int npc = P.wpad[0] / 64;             // phase chunks
    const int ngx = cdiv(P.wncell[0], kWCells);
    const int ngroups = ngx * P.wncell[1] * P.wncell[2];
    if (gw >= ngroups * npc) return;
    const int pc = gw % npc;
    const int g = gw / npc;
    const int cx0 = (g % ngx) * kWCells;
    const int cy = (g / ngx) % P.wncell[1];
    const int cz = g / (ngx * P.wncell[1]);
    const int r = pc * 64 + lane;
    const int Ppad = P.wpad[0];
    const int Kx = P.wK[0], Ky = P.wK[1], Kz = P.wK[2];
    const long long sx = P.wncp[0], sy = (long long)P.wncp[0] * P.wncp[1];
    const long long NCp = sy * P.wncp[2];
    float acc[kWCells][DIM];
#pragma unroll
    for (int t = 0; t < kWCells; ++t)
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[t][c] = 0.f;
    int qq = 0;
    for (int qz = 0; qz < Kz; ++qz)
        for (int qy = 0; qy < Ky; ++qy) {
            const float* row = thp + (cz + qz) * sy + (cy + qy) * sx + cx0;
            for (int qx = 0; qx < Kx; ++qx, ++qq) {
                const float w = W[(long long)qq * Ppad + r];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const float* th = row + c * NCp + qx;
#pragma unroll
                    for (int t = 0; t < kWCells; ++t) acc[t][c] = fmaf(w, th[t], acc[t][c]);
                }
            }
        }
    const int P3 = P.sp[0] * P.sp[1] * P.sp[2];
    if (r >= P3) return;
    const int rx = r % P.sp[0], ry = (r / P.sp[0]) % P.sp[1], rz = r / (P.sp[0] * P.sp[1]);
    const int y = cy * P.sp[1] + ry, z = cz * P.sp[2] + rz;
    if (y >= P.n[1] || z >= P.n[2]) return;
    const long long N = P.nvox;
    const long long rowv = ((long long)z * P.n[1] + y) * P.n[0];
#pragma unroll
    for (int t = 0; t < kWCells; ++t) {
        const int x = (cx0 + t) * P.sp[0] + rx;
        if (x < P.n[0]) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) u[c * N + rowv + x] = acc[t][c];
        }
    }
}

// H(c, qq) = sum_r W[qq][r] g(c, r) for kWCells cells along x and 64 values
// of qq (one lane each). The phases are split over the block's waves in
// chunks of 64, each chunk of g staged in LDS ([r][cell][component]) and read
// wave-uniformly; the four partial sums are added in LDS in a fixed order.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_cells_t(const PairDesc P, const float* __restrict__ WT, const float* __restrict__ g,
               float* __restrict__ H) {
    constexpr int NV = kWCells * DIM;
    __shared__ float stage[kWaves][64 * NV];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nqc = P.wpad[1] / 64;
    const int ngx = cdiv(P.wncell[0], kWCells);
    const int qc = blockIdx.x % nqc;
    const int grp = blockIdx.x / nqc;
    const int cx0 = (grp % ngx) * kWCells;
    const int cy = (grp / ngx) % P.wncell[1];
    const int cz = grp / (ngx * P.wncell[1]);
    const int q = qc * 64 + lane;
    const int Qpad = P.wpad[1];
    const int P3 = P.sp[0] * P.sp[1] * P.sp[2];
    const int nrc = P.wpad[0] / 64;
    const long long N = P.nvox;
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.f;
    float* st = stage[w];
    for (int it = 0; it < cdiv(nrc, kWaves); ++it) {
        const int rc = it * kWaves + w;
        // stage g at phase r = rc * 64 + lane of every cell (0 outside the grid)
        {
            const int r = rc * 64 + lane;
            float v[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = 0.f;
            if (rc < nrc && r < P3) {
                const int rx = r % P.sp[0], ry = (r / P.sp[0]) % P.sp[1],
                          rz = r / (P.sp[0] * P.sp[1]);
                const int y = cy * P.sp[1] + ry, z = cz * P.sp[2] + rz;
                if (y < P.n[1] && z < P.n[2]) {
                    const long long rowv = ((long long)z * P.n[1] + y) * P.n[0];
#pragma unroll
                    for (int t = 0; t < kWCells; ++t) {
                        const int x = (cx0 + t) * P.sp[0] + rx;
                        if (x < P.n[0]) {
#pragma unroll
                            for (int c = 0; c < DIM; ++c) v[t * DIM + c] = g[c * N + rowv + x];
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < NV; ++k) st[lane * NV + k] = v[k];
        }
        __syncthreads();
        if (rc < nrc) {
            const float* wt = WT + (long long)rc * 64 * Qpad + q;
            for (int rl = 0; rl < 64; ++rl) {
                const float wv = wt[(long long)rl * Qpad];
                const float* sv = st + rl * NV;
#pragma unroll
                for (int k = 0; k < NV; ++k) acc[k] = fmaf(wv, sv[k], acc[k]);
            }
        }
        __syncthreads();
    }
    // reduce the waves' partial sums: red[w][lane][k]
    float* red = &stage[0][0];
#pragma unroll
    for (int k = 0; k < NV; ++k) red[(w * 64 + lane) * NV + k] = acc[k];
    __syncthreads();
    const int Q = P.wK[0] * P.wK[1] * P.wK[2];
    const long long ncells = (long long)P.wncell[0] * P.wncell[1] * P.wncell[2];
    const long long row = ((long long)cz * P.wncell[1] + cy) * P.wncell[0] + cx0;
    // consecutive threads take consecutive cells of one (component, qq) row
    for (int i = threadIdx.x; i < 64 * NV; i += kBlock) {
        const int t = i % kWCells;
        const int c = (i / kWCells) % DIM;
        const int ql = i / (kWCells * DIM);
        const int k = t * DIM + c;
        float s = 0.f;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) s += red[(ww * 64 + ql) * NV + k];
        const int qv = qc * 64 + ql;
        if (qv < Q && cx0 + t < P.wncell[0]) H[((long long)c * Q + qv) * ncells + row + t] = s;
    }
}

// out(j) (+)= scale * sum_qq H(j - qq, qq) over cells inside the grid, with
// H laid out [d][K^d][cells]. A block takes 64 consecutive controls (one per
// lane, so a wave reads consecutive cells) and splits qq over its waves; the
// partial sums are added in a fixed order.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_gather(const PairDesc P, const float* __restrict__ H, float scale, int accumulate,
              float* __restrict__ out) {
    __shared__ float red[kWaves][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const long long NC = (long long)P.nc[0] * P.nc[1] * P.nc[2];
    const long long ncells = (long long)P.wncell[0] * P.wncell[1] * P.wncell[2];
    const int Q = P.wK[0] * P.wK[1] * P.wK[2];
    const long long i = (long long)blockIdx.x * 64 + lane;   // (component, control)
    float s = 0.f;
    if (i < DIM * NC) {
        const int c = (int)(i / NC);
        const long long j = i % NC;
        const int jx = (int)(j % P.nc[0]);
        const int jy = (int)((j / P.nc[0]) % P.nc[1]);
        const int jz = (int)(j / ((long long)P.nc[0] * P.nc[1]));
        const float* Hc = H + (long long)c * Q * ncells;
        for (int qq = w; qq < Q; qq += kWaves) {
            const int qx = qq % P.wK[0], qy = (qq / P.wK[0]) % P.wK[1],
                      qz = qq / (P.wK[0] * P.wK[1]);
            const int cx = jx - qx, cy = jy - qy, cz = jz - qz;
            if (cx < 0 || cx >= P.wncell[0] || cy < 0 || cy >= P.wncell[1] || cz < 0 ||
                cz >= P.wncell[2])
                continue;
            s += Hc[(long long)qq * ncells + ((long long)cz * P.wncell[1] + cy) * P.wncell[0] +
                    cx];
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && i < DIM * NC) {
        float t = 0.f;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) t += red[ww][lane];
        const float v = scale * t;
        out[i] = accumulate ? out[i] + v : v;
    }
}

__host__ inline int wend_grid(long long n) {
    const long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

// u = scale * B theta. thp: d * prod(wncp) floats of workspace; W: the
// [wpad0][...] table in the plan's constants.
hipError_t launch_wendland_expand(const PairDesc& P, const float* consts_dev, int dim,
                                  const float* theta, float scale, float* thp, float* u,
                                  hipStream_t s) {
    const long long np = (long long)dim * P.wncp[0] * P.wncp[1] * P.wncp[2];
    const float* W = consts_dev + P.wend_off[0];
    const int ngx = cdiv(P.wncell[0], kWCells);
    const long long waves = (long long)ngx * P.wncell[1] * P.wncell[2] * (P.wpad[0] / 64);
    const int blocks = (int)((waves + kWaves - 1) / kWaves);
    if (dim == 3) {
        hipLaunchKernelGGL(k_wend_pad<3>, dim3(wend_grid(np)), dim3(kBlock), 0, s, P, theta,
                           scale, thp);
        hipLaunchKernelGGL(k_wend_expand<3>, dim3(blocks), dim3(kBlock), 0, s, P, W, thp, u);
    } else {
        hipLaunchKernelGGL(k_wend_pad<2>, dim3(wend_grid(np)), dim3(kBlock), 0, s, P, theta,
                           scale, thp);
        hipLaunchKernelGGL(k_wend_expand<2>, dim3(blocks), dim3(kBlock), 0, s, P, W, thp, u);
    }
    return hipGetLastError();
}

// grad (+)= scale * B^T g. H: d * K^d * prod(wncell) floats of workspace.
hipError_t launch_wendland_adjoint(const PairDesc& P, const float* consts_dev, int dim,
                                   const float* g, float scale, float* H, float* grad,
                                   bool accumulate, hipStream_t s) {
    const float* WT = consts_dev + P.wend_off[1];
    const int ngx = cdiv(P.wncell[0], kWCells);
    const int blocks = ngx * P.wncell[1] * P.wncell[2] * (P.wpad[1] / 64);
    const long long NC = (long long)dim * P.nc[0] * P.nc[1] * P.nc[2];
    const int gblocks = (int)((NC + 63) / 64);
    if (dim == 3) {
        hipLaunchKernelGGL(k_wend_cells_t<3>, dim3(blocks), dim3(kBlock), 0, s, P, WT, g, H);
        hipLaunchKernelGGL(k_wend_gather<3>, dim3(gblocks), dim3(kBlock), 0, s, P, H, scale,
                           accumulate ? 1 : 0, grad);
    } else {
        hipLaunchKernelGGL(k_wend_cells_t<2>, dim3(blocks), dim3(kBlock), 0, s, P, WT, g, H);
        hipLaunchKernelGGL(k_wend_gather<2>, dim3(gblocks), dim3(kBlock), 0, s, P, H, scale,
                           accumulate ? 1 : 0, grad);
    }
    return hipGetLastError();
}

// Cells along x per wave in both contractions (the padded control grid is
// rounded up to a multiple of it along x).
int wendland_cells_per_wave() { return kWCells; }

}  // namespace air
