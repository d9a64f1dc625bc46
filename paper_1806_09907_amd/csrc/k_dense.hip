// Objective + gradient for the dense (non-parametric) transform, u = theta
// (Sec. III-C "Non-linear/dense"). The per-voxel gradient needs the global
// similarity coefficients (MSE: 2/N' over the masked voxels; NCC: the
// Pearson coefficients), so the evaluation takes three passes:
//   pre   MSE: count masked voxels (reads theta only); NCC: forward moments;
//   coef  one block per pair turns the block partials into coefficients;
//   main  per voxel: sample, similarity adjoint, diffusion stencil adjoint
//         (Sec. II-A eq. diffusion_regularizer, forward differences over
//         X_R), writes the gradient and the value partials;
//   fin   one block per pair writes the objective value.
// Lanes cover kDenseTX x kDenseTY voxels in (x, y); each lane walks a chunk
// of z and keeps u at z-1, z, z+1 in registers. In 3D the plane of u at z
// (with a one-voxel x / y halo) is staged in LDS for the stencil.
#include "device_common.h"

namespace air {

constexpr int DTX = kDenseTX, DTY = kDenseTY;

struct DenseTile {
    int x, y, z0, z1;
    bool act;
};

// A 2D block covers DTX x (DTY * kDenseRows2) pixels: lane row ly takes rows
// y0 + ly + DTY r, r < kDenseRows2 (the "z" range of its tile), so a large
// image does not become tens of thousands of tiny blocks whose partial sums
// the single-block reductions then walk.
constexpr int kDenseRows2 = 8;

// Dense-pass blocks of one pair (host and device).
__host__ __device__ inline int dense_blocks_of(int dim, const int* n) {
    const int nbx = cdiv(n[0], DTX);
    if (dim == 3) return nbx * cdiv(n[1], DTY) * cdiv(n[2], kDenseZc);
    return nbx * cdiv(n[1], DTY * kDenseRows2);
}

__device__ inline DenseTile dense_tile(const PairDesc& P, int blk, int zc, int dim) {
    const int ty = dim == 3 ? DTY : DTY * kDenseRows2;   // rows of a block
    const int nbx = cdiv(P.n[0], DTX), nby = cdiv(P.n[1], ty);
    const int bx = blk % nbx;
    const int rest = blk / nbx;
    const int by = rest % nby;
    const int bz = rest / nby;
    DenseTile T;
    T.x = bx * DTX + (threadIdx.x % DTX);
    T.y = by * ty + (threadIdx.x / DTX);
    if (dim == 3) {
        T.z0 = bz * zc;
        T.z1 = min(T.z0 + zc, P.n[2]);
    } else {
        T.z0 = 0;
        T.z1 = kDenseRows2;   // row groups; rows at or past n[1] are skipped
    }
    T.act = (T.x < P.n[0]) && (T.y < P.n[1]);
    return T;
}

// Trilinear sample of M at the point (x, y, z) + d + e of a voxel (voxel
// units; see axis_cell) with its gradient, branch-free: the cell is clamped
// into the volume so every load is in range, and m = 1 iff the point lay
// inside [0, n-1]^3. A point exactly on the last voxel uses the cell
// [n_a - 2, n_a - 1] with f = 1, and its derivative along a is the
// right-sided, zero-padded difference -W.
struct Sample3 {
    float W, m, d[3];
};
// the sampler in two stages, so that the gathers of one point can be in
// flight while another finishes
struct Gather3 {
    v2f a00, a10, a01, a11;
    float fx, fy, fz, m;
    bool ex, ey, ez;
};
__device__ inline Gather3 sample3_issue(__amdgpu_buffer_rsrc_t rM, int x, int y, int z, Disp qx,
                                        Disp qy, Disp qz, int nx, int ny, int nz) {
    Gather3 g;
    const AxisCell cx = axis_cell(x, qx, nx), cy = axis_cell(y, qy, ny), cz = axis_cell(z, qz, nz);
    g.m = (cx.in && cy.in && cz.in) ? 1.f : 0.f;
    g.ex = cx.t == nx - 1;
    g.ey = cy.t == ny - 1;
    g.ez = cz.t == nz - 1;
    const int jx = min(max(cx.t, 0), nx - 2), jy = min(max(cy.t, 0), ny - 2);
    const int jz = min(max(cz.t, 0), nz - 2);
    // inside the mask f == 0 on the last voxel: its cell is the one below, f = 1
    g.fx = g.ex ? 1.f : cx.f;
    g.fy = g.ey ? 1.f : cy.f;
    g.fz = g.ez ? 1.f : cz.f;
    const int off = (int)(__umul24(__umul24(jz, ny) + jy, nx) + jx) * 4;
    const int sx4 = nx * 4, sxy4 = nx * ny * 4;
    AIR_CHECK(off >= 0 && (long long)off + sxy4 + sx4 + 8 <= (long long)nx * ny * nz * 4,
              kDbgSampler);
    g.a00 = load2(rM, off, 0);
    g.a10 = load2(rM, off, sx4);
    g.a01 = load2(rM, off, sxy4);
    g.a11 = load2(rM, off, sxy4 + sx4);
    return g;
}
__device__ inline Sample3 sample3_finish(const Gather3& g) {
    Sample3 r;
    const float fx = g.fx, fy = g.fy, fz = g.fz;
    const float dz00 = g.a01.x - g.a00.x, dz01 = g.a01.y - g.a00.y;
    const float dz10 = g.a11.x - g.a10.x, dz11 = g.a11.y - g.a10.y;
    const float e00 = g.a00.x + fz * dz00, e01 = g.a00.y + fz * dz01;
    const float e10 = g.a10.x + fz * dz10, e11 = g.a10.y + fz * dz11;
    const float dy0 = e10 - e00, dy1 = e11 - e01;
    const float g0 = e00 + fy * dy0, g1 = e01 + fy * dy1;
    r.W = g0 + fx * (g1 - g0);
    r.m = g.m;
    const float h0 = dz00 + fy * (dz10 - dz00), h1 = dz01 + fy * (dz11 - dz01);
    r.d[0] = g.ex ? -r.W : g1 - g0;
    r.d[1] = g.ey ? -r.W : dy0 + fx * (dy1 - dy0);
    r.d[2] = g.ez ? -r.W : h0 + fx * (h1 - h0);
    return r;
}
__device__ inline Sample3 sample3(__amdgpu_buffer_rsrc_t rM, int x, int y, int z, Disp qx, Disp qy,
                                  Disp qz, int nx, int ny, int nz) {
    return sample3_finish(sample3_issue(rM, x, y, z, qx, qy, qz, nx, ny, nz));
}

template <int DIM, int SIM>
__global__ void __launch_bounds__(DTX* DTY)
k_dense_pre(const LaunchCtx C, int zc) {
    constexpr int NT = DTX * DTY;
    __shared__ double red[8 * (NT / 64)];
    const int pair = blockIdx.y;
    const PairDesc P = C.pairs[pair];
    const int blk = xcd_item(blockIdx.x, P.dense_nblk, 0);
    if (blk < 0) return;
    const float* __restrict__ F = C.fixed_tab ? C.fixed_tab[pair] : C.fixed0;
    const float* __restrict__ M = C.moving_tab ? C.moving_tab[pair] : C.moving0;
    const float* __restrict__ th = C.theta_tab ? C.theta_tab[pair] : C.theta0;
    const DenseTile T = dense_tile(P, blk, zc, DIM);
    const long long N = P.nvox;
    double v[6] = {0, 0, 0, 0, 0, 0};
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, (uint32_t)(N * 4));
    float cnt = 0.f;   // at most zc per lane: exact in FP32
    if (T.act) {
        // unrolled so that several planes' loads are in flight per wave
#pragma unroll 4
        for (int z = T.z0; z < T.z1; ++z) {
            // 3D: plane z of the column; 2D: row group z of the lane
            const int yy = DIM == 3 ? T.y : T.y + z * DTY;
            const int zz = DIM == 3 ? z : 0;
            if (DIM == 2 && yy >= P.n[1]) break;
            const long long vi = ((long long)zz * P.n[1] + yy) * P.n[0] + T.x;
            Disp q[3];
            const int idx[3] = {T.x, yy, zz};
            int in = 1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                q[a] = disp_of(th[a * N + vi], P.s[a]);
                in &= (int)axis_cell(idx[a], q[a], P.n[a]).in;
            }
            if (SIM == AIR_SIM_MSE) {
                cnt += in ? 1.f : 0.f;
            } else if (in) {
                float W;
                if constexpr (DIM == 3) {
                    W = sample3(rM, idx[0], idx[1], idx[2], q[0], q[1], q[2], P.n[0], P.n[1],
                                P.n[2]).W;
                } else {
                    bool in2;
                    W = sample_general<DIM>(M, P.n, idx, q, &in2, nullptr);
                }
                const double f = F[vi], w = W;
                v[0] += 1.0;
                v[1] += f;
                v[2] += w;
                v[3] += f * f;
                v[4] += w * w;
                v[5] += f * w;
            }
        }
    }
    if (SIM == AIR_SIM_MSE) v[0] = (double)cnt;
    block_sum<NT, 6>(v, red);
    if (threadIdx.x == 0) {
        double* slot = reinterpret_cast<double*>(C.ws + C.L.dense_stats) +
                       (long long)(P.dense_blk_off + blk) * kStatWords;
#pragma unroll
        for (int k = 0; k < 6; ++k) slot[k] = v[k];
    }
}

// scalars[pair]: [0] alpha, [1] beta, [2] muF, [3] muW, [4] S, [5] N, [6] degenerate
template <int SIM>
__global__ void __launch_bounds__(kBlock)
k_dense_coef(const LaunchCtx C) {
    __shared__ double red[8 * (kBlock / 64)];
    const int pair = blockIdx.x;
    const PairDesc P = C.pairs[pair];
    const double* st = reinterpret_cast<const double*>(C.ws + C.L.dense_stats);
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < P.dense_nblk; b += kBlock) {
        const double* s = st + (long long)(P.dense_blk_off + b) * kStatWords;
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] += s[k];
    }
    block_sum<kBlock, 6>(v, red);
    if (threadIdx.x != 0) return;
    double* out = reinterpret_cast<double*>(C.ws + C.L.scalars) + (long long)pair * 8;
    const double N = v[0];
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    out[5] = N;
    if (SIM == AIR_SIM_MSE) {
        if (N < 1.0) { out[6] = 1.0; return; }
        out[0] = 2.0 / N;
        return;
    }
    if (N < 2.0) { out[6] = 1.0; return; }
    const double muF = v[1] / N, muW = v[2] / N;
    const double B = v[3] - N * muF * muF, Cc = v[4] - N * muW * muW;
    const double A = v[5] - N * muF * muW;
    if (!(B > 1e-10 * v[3]) || !(Cc > 1e-10 * v[4])) { out[6] = 1.0; return; }
    const double sbc = sqrt(B * Cc), rho = A / sbc;
    out[0] = -1.0 / sbc;
    out[1] = rho / Cc;
    out[2] = muF;
    out[3] = muW;
    out[4] = -rho;
}

template <int DIM, int SIM>
__global__ void __launch_bounds__(DTX* DTY)
k_dense_main(const LaunchCtx C, int zc, int reg_only, float* reg_grad_out) {
    constexpr int NT = DTX * DTY;
    __shared__ double red[8 * (NT / 64)];
    const int pair = blockIdx.y;
    const PairDesc P = C.pairs[pair];
    // consecutive tiles share one XCD, so the stencil's x / y halo and the
    // displaced gathers of neighbouring tiles hit the same L2
    const int blk = xcd_item(blockIdx.x, P.dense_nblk, 0);
    if (blk < 0) return;
    const float* __restrict__ F = C.fixed_tab ? C.fixed_tab[pair] : C.fixed0;
    const float* __restrict__ M = C.moving_tab ? C.moving_tab[pair] : C.moving0;
    const float* __restrict__ th = C.theta_tab ? C.theta_tab[pair] : C.theta0;
    float* __restrict__ grad = reg_only ? reg_grad_out
                                        : (C.grad_tab ? C.grad_tab[pair] : C.grad0);
    const DenseTile T = dense_tile(P, blk, zc, DIM);
    const long long N = P.nvox;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const long long sy = nx, sz = (long long)nx * ny;
    double a = 0, b = 0, cc = 0, dd = 0;
    float beta = 0.f, muF = 0.f, muW = 0.f;
    bool degenerate = true;
    if (!reg_only) {
        const double* sc = reinterpret_cast<const double*>(C.ws + C.L.scalars) + (long long)pair * 8;
        a = sc[0];
        b = sc[1];
        cc = sc[2];
        dd = sc[3];
        degenerate = sc[6] != 0.0;
        beta = (float)b;
        muF = (float)cc;
        muW = (float)dd;
    }
    const float alpha = (float)a;
    const float rscale = (reg_only ? 1.0f : P.lambda) * 2.0f * P.inv_xr;
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, (uint32_t)(N * 4));
    // per-lane sums over the z chunk in FP32, widened once per chunk
    float sq = 0.f, rr = 0.f;   // MSE sum of squares, regulariser sum
    if (T.act) {
        const int x = T.x;
        int y = T.y;
        const bool inx = x <= nx - 2;
        float um[3], u0[3], up[3];
        long long vi = ((long long)T.z0 * ny + y) * nx + x;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            u0[c] = th[c * N + vi];
            um[c] = (DIM == 3 && T.z0 > 0) ? th[c * N + vi - sz] : 0.f;
        }
        // 3D: walk z; 2D: walk the lane's row groups (y advances by DTY)
        for (int z = T.z0; z < T.z1;
             ++z, vi += (DIM == 3 ? sz : (long long)DTY * sy), y += (DIM == 3 ? 0 : DTY)) {
            if (DIM == 2) {
                if (y >= ny) break;
#pragma unroll
                for (int c = 0; c < DIM; ++c) u0[c] = th[c * N + vi];
            }
            const bool iny = y <= ny - 2;
            const bool has_zp = DIM == 3 && z + 1 < nz;
#pragma unroll
            for (int c = 0; c < DIM; ++c) up[c] = has_zp ? th[c * N + vi + sz] : 0.f;
            // regulariser adjoint: sum_a [x-e_a in X_R](u - u_-a) - [x in X_R](u_+a - u)
            const bool inz = DIM == 2 || z <= nz - 2;
            const bool in_r = inx && iny && inz;
            const bool prev_x = x >= 1 && iny && inz;
            const bool prev_y = y >= 1 && inx && inz;
            const bool prev_z = DIM == 3 && z >= 1 && inx && iny;
            float gr[3];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const float* tc = th + c * N;
                const float uxp = (x + 1 < nx) ? tc[vi + 1] : 0.f;
                const float uxm = (x >= 1) ? tc[vi - 1] : 0.f;
                const float uyp = (y + 1 < ny) ? tc[vi + sy] : 0.f;
                const float uym = (y >= 1) ? tc[vi - sy] : 0.f;
                float g = 0.f;
                if (in_r) {
                    const float dx = uxp - u0[c], dy = uyp - u0[c];
                    g -= dx + dy;
                    float r2 = dx * dx + dy * dy;
                    if (DIM == 3) {
                        const float dz = up[c] - u0[c];
                        g -= dz;
                        r2 += dz * dz;
                    }
                    rr += r2;
                }
                if (prev_x) g += u0[c] - uxm;
                if (prev_y) g += u0[c] - uym;
                if (prev_z) g += u0[c] - um[c];
                gr[c] = rscale * g;
            }
            float gi[3] = {0.f, 0.f, 0.f};
            if (!reg_only) {
                const float Fv = F[vi];
                float W, m, dW[3];
                if constexpr (DIM == 3) {
                    const Sample3 q = sample3(rM, x, y, z, disp_of(u0[0], P.s[0]),
                                              disp_of(u0[1], P.s[1]), disp_of(u0[2], P.s[2]),
                                              nx, ny, nz);
                    W = q.W;
                    m = q.m;
#pragma unroll
                    for (int c = 0; c < 3; ++c) dW[c] = q.d[c];
                } else {
                    Disp q[3];
                    const int idx[3] = {x, y, z};
#pragma unroll
                    for (int c = 0; c < DIM; ++c) q[c] = disp_of(u0[c], P.s[c]);
                    bool in;
                    W = sample_general<DIM>(M, P.n, idx, q, &in, dW);
                    m = in ? 1.f : 0.f;
                }
                float e;
                if (SIM == AIR_SIM_MSE) {
                    const float r = m * (W - Fv);
                    sq += r * r;
                    e = alpha * r;
                } else {
                    e = m * (alpha * (Fv - muF) + beta * (W - muW));
                }
                if (degenerate) e = 0.f;
#pragma unroll
                for (int c = 0; c < DIM; ++c) gi[c] = e * dW[c] * P.s[c];
            }
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                grad[c * N + vi] = gi[c] + gr[c];
                um[c] = u0[c];
                u0[c] = up[c];
            }
        }
    }
    double acc[2] = {(double)sq, (double)rr};
    block_sum<NT, 2>(acc, red);
    if (threadIdx.x == 0) {
        double* slot = reinterpret_cast<double*>(C.ws + C.L.dense_stats) +
                       (long long)(P.dense_blk_off + blk) * kStatWords;
        slot[0] = acc[0];
        slot[1] = acc[1];
    }
}

// 3D main pass. Each block owns a kDenseTX x kDenseTY column of (x, y) and
// walks its z chunk; per z step the plane of u (three components, with a
// one-voxel x / y halo, zero outside the volume) goes to one of two LDS
// buffers, so the stencil's x and y neighbours come from LDS and z -+ 1 from
// registers. The next plane (own voxel and halo) is loaded one step ahead.
// Consecutive tiles share one XCD, so halo rows and the displaced gathers of
// neighbouring tiles hit the same L2.
template <int SIM>
__global__ void __launch_bounds__(kDenseTX* kDenseTY)
k_dense_main3(const LaunchCtx C, int zc, int reg_only, float* reg_grad_out) {
    constexpr int TX = kDenseTX, TY = kDenseTY;
    constexpr int TXh = TX + 2, PL = TXh * (TY + 2);
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * TX + 2 * TY;  // halo cells of a plane (no corners)
    __shared__ float pl[2][3][PL];
    __shared__ double red[8 * (NT / 64)];
    const int tid = threadIdx.x;
    const int pair = blockIdx.y;
    const PairDesc P = C.pairs[pair];
    const int blk = xcd_item(blockIdx.x, P.dense_nblk, 0);
    if (blk < 0) return;
    const float* __restrict__ F = C.fixed_tab ? C.fixed_tab[pair] : C.fixed0;
    const float* __restrict__ M = C.moving_tab ? C.moving_tab[pair] : C.moving0;
    const float* __restrict__ th = C.theta_tab ? C.theta_tab[pair] : C.theta0;
    float* __restrict__ grad = reg_only ? reg_grad_out
                                        : (C.grad_tab ? C.grad_tab[pair] : C.grad0);
    const long long N = P.nvox;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const long long sz = (long long)nx * ny;
    const int nbx = cdiv(nx, TX), nby = cdiv(ny, TY);
    const int x0 = (blk % nbx) * TX, y0 = ((blk / nbx) % nby) * TY;
    const int z0 = (blk / (nbx * nby)) * zc, z1 = min(z0 + zc, nz);
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool act = x < nx && y < ny;
    const long long vxy = (long long)y * nx + x;
    // this thread's halo cell (tid < NH): plane-local (hx, hy), global (gx, gy)
    int hx = 0, hy = 0, gx = -1, gy = -1;
    if (tid < TX) {
        hx = tid + 1; hy = 0; gx = x0 + tid; gy = y0 - 1;
    } else if (tid < 2 * TX) {
        hx = tid - TX + 1; hy = TY + 1; gx = x0 + tid - TX; gy = y0 + TY;
    } else if (tid < 2 * TX + TY) {
        hx = 0; hy = tid - 2 * TX + 1; gx = x0 - 1; gy = y0 + tid - 2 * TX;
    } else if (tid < NH) {
        hx = TX + 1; hy = tid - 2 * TX - TY + 1; gx = x0 + TX; gy = y0 + tid - 2 * TX - TY;
    }
    const bool hact = tid < NH && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const long long hxy = hact ? (long long)gy * nx + gx : 0;
    const int own = (ly + 1) * TXh + lx + 1;
    const int hcell = hy * TXh + hx;

    double a = 0, b = 0, cc = 0, dd = 0;
    bool degenerate = true;
    if (!reg_only) {
        const double* sc = reinterpret_cast<const double*>(C.ws + C.L.scalars) + (long long)pair * 8;
        a = sc[0];
        b = sc[1];
        cc = sc[2];
        dd = sc[3];
        degenerate = sc[6] != 0.0;
    }
    const float alpha = (float)a, beta = (float)b, muF = (float)cc, muW = (float)dd;
    const float rscale = (reg_only ? 1.0f : P.lambda) * 2.0f * P.inv_xr;
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, (uint32_t)(N * 4));
    // regulariser domain X_R = prod [0, n_a - 2] as per-lane 0/1 weights
    const float wxin = (act && x <= nx - 2) ? 1.f : 0.f, wyin = (act && y <= ny - 2) ? 1.f : 0.f;
    const float wx1 = (act && x >= 1) ? 1.f : 0.f, wy1 = (act && y >= 1) ? 1.f : 0.f;
    const float wxy = wxin * wyin;

    // Registers hold u at z - 1, z, z + 1 (um, u0, up); each step loads u at
    // z + 2, the halo of plane z + 1, F at z + 1 and the gathers of z + 1,
    // so all of a step's memory traffic is in flight a step ahead of its use.
    float um[3], u0[3], up[3], upp[3], h0[3], hp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float* tc = th + c * N;
        um[c] = (act && z0 > 0) ? tc[(z0 - 1) * sz + vxy] : 0.f;
        u0[c] = act ? tc[z0 * sz + vxy] : 0.f;
        up[c] = (act && z0 + 1 < nz) ? tc[(z0 + 1) * sz + vxy] : 0.f;
        h0[c] = hact ? tc[z0 * sz + hxy] : 0.f;
    }
    const float* Fc = F + vxy;
    const float s0 = P.s[0], s1 = P.s[1], s2 = P.s[2];
    // regulariser-only calls have no images (F and M may be null): no loads
    float Fv = (act && !reg_only) ? Fc[z0 * sz] : 0.f;
    Gather3 G{};
    if (!reg_only)
        G = sample3_issue(rM, x, y, z0, disp_of(u0[0], s0), disp_of(u0[1], s1),
                          disp_of(u0[2], s2), nx, ny, nz);
    float sq = 0.f, rr = 0.f;   // per-lane MSE and regulariser sums over the chunk
    for (int z = z0; z < z1; ++z) {
        const int bsel = (z - z0) & 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float* tc = th + c * N;
            upp[c] = (act && z + 2 < nz) ? tc[(z + 2) * sz + vxy] : 0.f;
            hp[c] = (hact && z + 1 < nz) ? tc[(z + 1) * sz + hxy] : 0.f;
        }
        // next point (clamped, in range even past the chunk or the volume)
        const float Fn = (act && !reg_only) ? Fc[min(z + 1, nz - 1) * sz] : 0.f;
        Gather3 Gn{};
        if (!reg_only)
            Gn = sample3_issue(rM, x, y, z + 1, disp_of(up[0], s0), disp_of(up[1], s1),
                               disp_of(up[2], s2), nx, ny, nz);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pl[bsel][c][own] = u0[c];
            if (tid < NH) pl[bsel][c][hcell] = h0[c];
        }
        __syncthreads();
        const float wzin = z <= nz - 2 ? 1.f : 0.f, wz1 = z >= 1 ? 1.f : 0.f;
        const float w_in = wxy * wzin, w_px = wx1 * wyin * wzin, w_py = wy1 * wxin * wzin;
        const float w_pz = wz1 * wxy;
        float gr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float* q = pl[bsel][c];
            const float uxm = q[own - 1], uxp = q[own + 1];
            const float uym = q[own - TXh], uyp = q[own + TXh];
            const float dxp = uxp - u0[c], dyp = uyp - u0[c], dzp = up[c] - u0[c];
            rr += w_in * (dxp * dxp + dyp * dyp + dzp * dzp);
            const float g = w_px * (u0[c] - uxm) + w_py * (u0[c] - uym) +
                            w_pz * (u0[c] - um[c]) - w_in * (dxp + dyp + dzp);
            gr[c] = rscale * g;
        }
        if (act) {
            const long long vi = z * sz + vxy;
            float gi[3] = {0.f, 0.f, 0.f};
            if (!reg_only) {
                const Sample3 s3 = sample3_finish(G);
                float e;
                if (SIM == AIR_SIM_MSE) {
                    const float r = s3.m * (s3.W - Fv);
                    sq += r * r;
                    e = alpha * r;
                } else {
                    e = s3.m * (alpha * (Fv - muF) + beta * (s3.W - muW));
                }
                if (degenerate) e = 0.f;
#pragma unroll
                for (int c = 0; c < 3; ++c) gi[c] = e * s3.d[c] * P.s[c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) grad[c * N + vi] = gi[c] + gr[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            um[c] = u0[c];
            u0[c] = up[c];
            up[c] = upp[c];
            h0[c] = hp[c];
        }
        G = Gn;
        Fv = Fn;
    }
    double acc[2] = {(double)sq, (double)rr};
    block_sum<NT, 2>(acc, red);
    if (tid == 0) {
        double* slot = reinterpret_cast<double*>(C.ws + C.L.dense_stats) +
                       (long long)(P.dense_blk_off + blk) * kStatWords;
        slot[0] = acc[0];
        slot[1] = acc[1];
    }
}

template <int SIM>
__global__ void __launch_bounds__(kBlock)
k_dense_fin(const LaunchCtx C, int reg_only, float* reg_value_out) {
    __shared__ double red[8 * (kBlock / 64)];
    const int pair = blockIdx.x;
    const PairDesc P = C.pairs[pair];
    const double* st = reinterpret_cast<const double*>(C.ws + C.L.dense_stats);
    double v[2] = {0, 0};
    for (int b = threadIdx.x; b < P.dense_nblk; b += kBlock) {
        const double* s = st + (long long)(P.dense_blk_off + b) * kStatWords;
        v[0] += s[0];
        v[1] += s[1];
    }
    block_sum<kBlock, 2>(v, red);
    if (threadIdx.x != 0) return;
    const double R = v[1] * (double)P.inv_xr;
    if (reg_only) {
        *reg_value_out = (float)R;
        return;
    }
    const double* sc = reinterpret_cast<const double*>(C.ws + C.L.scalars) + (long long)pair * 8;
    const bool degenerate = sc[6] != 0.0;
    double S = 0.0;
    if (!degenerate) S = (SIM == AIR_SIM_MSE) ? v[0] / sc[5] : sc[4];
    const double value = S + (double)P.lambda * R;
    float* vout = C.values ? C.values + pair : C.value0;
    *vout = (float)value;
    uint32_t fl = degenerate ? AIR_FLAG_DEGENERATE : 0u;
    if (!isfinite((float)value)) fl |= AIR_FLAG_NONFINITE;
    reinterpret_cast<uint32_t*>(C.ws + C.L.flags)[pair] = fl;
}

template <int DIM, int SIM>
static hipError_t dense_run(const LaunchCtx& C, int zc, int max_blk, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
    dim3 grid(xcd_grid(max_blk, 0), C.npairs);
    hipLaunchKernelGGL((k_dense_pre<DIM, SIM>), grid, dim3(DTX * DTY), 0, s, C, zc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_dense_coef<SIM>), dim3(C.npairs), dim3(kBlock), 0, s, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev0) (void)hipEventRecord(ev0, s);
    if (DIM == 3)
        hipLaunchKernelGGL((k_dense_main3<SIM>), grid, dim3(DTX * DTY), 0, s, C, zc, 0,
                           (float*)nullptr);
    else
        hipLaunchKernelGGL((k_dense_main<DIM, SIM>), grid, dim3(DTX * DTY), 0, s, C, zc, 0,
                           (float*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev1) (void)hipEventRecord(ev1, s);
    hipLaunchKernelGGL((k_dense_fin<SIM>), dim3(C.npairs), dim3(kBlock), 0, s, C, 0,
                       (float*)nullptr);
    return hipGetLastError();
}

hipError_t launch_dense(const LaunchCtx& C, int zc, int max_blk, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1) {
    if (C.dim == 3)
        return C.sim == AIR_SIM_NCC ? dense_run<3, 1>(C, zc, max_blk, s, ev0, ev1)
                                    : dense_run<3, 0>(C, zc, max_blk, s, ev0, ev1);
    return C.sim == AIR_SIM_NCC ? dense_run<2, 1>(C, zc, max_blk, s, ev0, ev1)
                                : dense_run<2, 0>(C, zc, max_blk, s, ev0, ev1);
}

// Regulariser of a dense field for one pair (context holds that pair only).
int dense_blocks(int dim, const int* n) { return dense_blocks_of(dim, n); }

hipError_t launch_reg_dense(const LaunchCtx& C, int pair_blocks, int zc, float* grad_out,
                            float* value_out, hipStream_t s) {
    dim3 grid(xcd_grid(pair_blocks, 0), 1);
    if (C.dim == 3)
        hipLaunchKernelGGL((k_dense_main3<0>), grid, dim3(DTX * DTY), 0, s, C, zc, 1, grad_out);
    else
        hipLaunchKernelGGL((k_dense_main<2, 0>), grid, dim3(DTX * DTY), 0, s, C, zc, 1, grad_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_dense_fin<0>), dim3(1), dim3(kBlock), 0, s, C, 1, value_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ warp
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_warp(const PairDesc* pairs, int pair, const float* consts, const float* __restrict__ M,
       const float* __restrict__ th, float* __restrict__ W, uint8_t* __restrict__ mask,
       int transform) {
    const PairDesc P = pairs[pair];
    const long long N = P.nvox;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < N;
         v += (long long)gridDim.x * kBlock) {
        const int x = (int)(v % P.n[0]);
        const int y = (int)((v / P.n[0]) % P.n[1]);
        const int z = (DIM == 3) ? (int)(v / ((long long)P.n[0] * P.n[1])) : 0;
        const int idx[3] = {x, y, z};
        float u[3] = {0.f, 0.f, 0.f};
        if (transform == AIR_TF_DENSE) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) u[c] = th[c * N + v];
        } else {
            int i0[3];
            const float* w[3];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                i0[a] = idx[a] / P.sp[a];
                w[a] = consts + P.wtab_off[a] + (idx[a] - i0[a] * P.sp[a]) * 4;
            }
            const long long NC = (long long)P.nc[0] * P.nc[1] * P.nc[2];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                float acc = 0.f;
                for (int kz = 0; kz < (DIM == 3 ? 4 : 1); ++kz) {
                    const float wz = (DIM == 3) ? w[2][kz] : 1.f;
                    const int jz = (DIM == 3) ? i0[2] + kz : 0;
                    for (int ky = 0; ky < 4; ++ky) {
                        const float* row = th + c * NC +
                                           ((long long)jz * P.nc[1] + i0[1] + ky) * P.nc[0] + i0[0];
                        const float wyz = wz * w[1][ky];
                        acc += wyz * (w[0][0] * row[0] + w[0][1] * row[1] + w[0][2] * row[2] +
                                      w[0][3] * row[3]);
                    }
                }
                u[c] = acc;
            }
        }
        Disp q[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) q[a] = disp_of(u[a], P.s[a]);
        bool in;
        const float val = sample_general<DIM>(M, P.n, idx, q, &in, nullptr);
        W[v] = val;
        if (mask) mask[v] = in ? 1 : 0;
    }
}

hipError_t launch_warp(const PairDesc* dpairs, int pair, const PairDesc& hp, const float* consts,
                       const float* M, const float* th, float* W, uint8_t* mask, int dim,
                       int transform, hipStream_t s) {
    const long long nb = (hp.nvox + kBlock - 1) / kBlock;
    const int grid = (int)(nb < 65536 ? nb : 65536);
    if (dim == 3)
        hipLaunchKernelGGL((k_warp<3>), dim3(grid), dim3(kBlock), 0, s, dpairs, pair, consts, M, th,
                           W, mask, transform);
    else
        hipLaunchKernelGGL((k_warp<2>), dim3(grid), dim3(kBlock), 0, s, dpairs, pair, consts, M, th,
                           W, mask, transform);
    return hipGetLastError();
}

// ------------------------------------------------------------------ similarity
__global__ void __launch_bounds__(kBlock)
k_sim_stats(const float* __restrict__ F, const float* __restrict__ W,
            const uint8_t* __restrict__ mask, long long N, double* slots) {
    __shared__ double red[8 * (kBlock / 64)];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock) {
        if (mask && !mask[i]) continue;
        const double f = F[i], w = W[i];
        v[0] += 1.0;
        v[1] += f;
        v[2] += w;
        v[3] += f * f;
        v[4] += w * w;
        v[5] += f * w;
        v[6] += (w - f) * (w - f);
    }
    block_sum<kBlock, 7>(v, red);
    if (threadIdx.x == 0) {
        double* s = slots + (long long)blockIdx.x * kStatWords;
        for (int k = 0; k < 7; ++k) s[k] = v[k];
    }
}

__global__ void __launch_bounds__(kBlock)
k_sim_fin(const double* slots, int nblk, int sim, float* value, uint32_t* flag) {
    __shared__ double red[8 * (kBlock / 64)];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += kBlock)
        for (int k = 0; k < 7; ++k) v[k] += slots[(long long)b * kStatWords + k];
    block_sum<kBlock, 7>(v, red);
    if (threadIdx.x != 0) return;
    const double N = v[0];
    double S = 0.0;
    uint32_t fl = 0;
    if (sim == AIR_SIM_MSE) {
        if (N < 1.0) fl |= AIR_FLAG_DEGENERATE; else S = v[6] / N;
    } else {
        if (N < 2.0) {
            fl |= AIR_FLAG_DEGENERATE;
        } else {
            const double muF = v[1] / N, muW = v[2] / N;
            const double B = v[3] - N * muF * muF, Cc = v[4] - N * muW * muW;
            const double A = v[5] - N * muF * muW;
            if (!(B > 1e-10 * v[3]) || !(Cc > 1e-10 * v[4])) fl |= AIR_FLAG_DEGENERATE;
            else S = -A / sqrt(B * Cc);
        }
    }
    if (!isfinite((float)S)) fl |= AIR_FLAG_NONFINITE;
    *value = (float)S;
    if (flag) *flag = fl;
}

hipError_t launch_similarity(const float* F, const float* W, const uint8_t* mask, long long N,
                             int sim, double* slots, int nslots, float* value, uint32_t* flag,
                             hipStream_t s) {
    long long nb = (N + kBlock - 1) / kBlock;
    const int grid = (int)(nb < nslots ? nb : nslots);
    hipLaunchKernelGGL(k_sim_stats, dim3(grid), dim3(kBlock), 0, s, F, W, mask, N, slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sim_fin, dim3(1), dim3(kBlock), 0, s, slots, grid, sim, value, flag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Adam, scale
__global__ void __launch_bounds__(kBlock)
k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
       float* __restrict__ v, long long n, float lr_bc1, float b1, float b2, float inv_sqrt_bc2,
       float eps) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr_bc1 * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
    }
}

hipError_t launch_adam(float* th, const float* g, float* m, float* v, long long n, float lr_bc1,
                       float b1, float b2, float inv_sqrt_bc2, float eps, hipStream_t s) {
    long long nb = (n + kBlock - 1) / kBlock;
    const int grid = (int)(nb < 16384 ? nb : 16384);
    hipLaunchKernelGGL(k_adam, dim3(grid), dim3(kBlock), 0, s, th, g, m, v, n, lr_bc1, b1, b2,
                       inv_sqrt_bc2, eps);
    return hipGetLastError();
}

// The same update with the two bias-correction factors read from device
// memory (coef[0] = lr / (1 - b1^t), coef[1] = 1 / sqrt(1 - b2^t)).
__global__ void __launch_bounds__(kBlock)
k_adam_dev(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
           float* __restrict__ v, long long n, const float* __restrict__ coef, float b1, float b2,
           float eps) {
    const float lr_bc1 = coef[0], inv_sqrt_bc2 = coef[1];
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr_bc1 * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
    }
}

hipError_t launch_adam_dev(float* th, const float* g, float* m, float* v, long long n,
                           const float* coef, float b1, float b2, float eps, hipStream_t s) {
    long long nb = (n + kBlock - 1) / kBlock;
    const int grid = (int)(nb < 16384 ? nb : 16384);
    hipLaunchKernelGGL(k_adam_dev, dim3(grid), dim3(kBlock), 0, s, th, g, m, v, n, coef, b1, b2,
                       eps);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_scale(float* __restrict__ x, const float* __restrict__ sc, long long n) {
    const float s = *sc;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        x[i] *= s;
}

hipError_t launch_scale(float* x, const float* s, long long n, hipStream_t st) {
    long long nb = (n + kBlock - 1) / kBlock;
    const int grid = (int)(nb < 16384 ? nb : 16384);
    hipLaunchKernelGGL(k_scale, dim3(grid), dim3(kBlock), 0, st, x, s, n);
    return hipGetLastError();
}

}  // namespace air

// this unit's bounds-check flags (debug build only)
AIR_DEBUG_UNIT(dense)
