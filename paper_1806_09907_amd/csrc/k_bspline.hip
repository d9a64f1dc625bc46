// Fused objective + gradient for the cubic B-spline transform.
//
// One work item is a tile of voxels: TX x TY lanes over (x, y) and a chunk of
// control cells along the column axis (z in 3D, y in 2D), walked by every
// lane. Per tile:
//   1. the control window is x-interpolated into LDS (separable expansion of
//      Sec. II-A eq. kernel_basis with the cubic B-spline of Sec. III-C);
//   2. each lane keeps the four column-axis control values of its current
//      cell in registers and forms u = sum_k w_k(t) V_k per voxel;
//   3. the moving image is sampled at p = x + u (n - 1)/2 with two 8-byte
//      buffer loads per corner pair (Sec. III-C Image Warping), giving W and
//      dW/dp; out-of-domain voxels are masked out;
//   4. similarity statistics are accumulated (MSE: sum of squared error;
//      NCC: moments about a per-tile shift);
//   5. the adjoint field (dS/dW dW/dp, split into 3 affine parts for NCC so
//      that the global NCC coefficients can be applied afterwards) is
//      transposed back onto the control window: per-voxel along the column,
//      then along y and x in LDS when a column control is complete.
// The per-tile partials are combined by k_finalize in a fixed order
// (deterministic), together with the regulariser computed exactly in control
// space from banded Gram matrices (blocks appended to the same launch).
#include <type_traits>

#include "device_common.h"

namespace air {

// --------------------------------------------------------------- regulariser
// dR/dtheta_c = (2/|X_R|) sum_a K_a theta_c with K_a the Kronecker product of
// per-axis banded Gram matrices: D (differences) on axis a, P on the others.
// One block handles one control plane (3D: fixed kz) of one component.
template <int NT>
__device__ void reg_block(const PairDesc& P, const float* __restrict__ consts,
                          const float* __restrict__ theta, float* __restrict__ out_grad,
                          float scale, double* __restrict__ regpart, int r, int dim,
                          float* lds, double* red) {
    const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
    const int plane = ncx * ncy;
    const float* Px = consts + P.gram_off[0];
    const float* Dx = Px + 7 * ncx;
    const float* Py = consts + P.gram_off[1];
    const float* Dy = Py + 7 * ncy;
    // block r: component c, control plane kz (3D), band of rows [y0, y1)
    const int nb_ = P.reg_nband;
    int c, kz, band;
    if (dim == 3) {
        c = r / (ncz * nb_);
        kz = (r / nb_) % ncz;
    } else {
        c = r / nb_;
        kz = 0;
    }
    band = r % nb_;
    const int y0 = band * P.reg_rows, y1 = min(ncy, y0 + P.reg_rows);
    const int ya = max(0, y0 - 3), yb = min(ncy, y1 + 3);   // rows the y taps reach
    const int na = (yb - ya) * ncx, nbr = (y1 - y0) * ncx;
    const float* th = theta + (long long)c * ncz * plane;
    float* A = lds;              // P_z theta (3D) or theta (2D), rows [ya, yb)
    float* Cz = A + a4(na);      // D_z theta (3D only), rows [ya, yb)
    float* AP = Cz + a4(na);     // rows [y0, y1)
    float* AD = AP + a4(nbr);
    float* CP = AD + a4(nbr);
    const int tid = threadIdx.x;
    if (dim == 3) {
        const float* Pz = consts + P.gram_off[2];
        const float* Dz = Pz + 7 * ncz;
        for (int i = tid; i < na; i += NT) {
            const int g = ya * ncx + i;
            float a = 0.f, b = 0.f;
#pragma unroll
            for (int o = -3; o <= 3; ++o) {
                int k = kz + o;
                if (k < 0 || k >= ncz) continue;
                float t = th[(long long)k * plane + g];
                a += Pz[kz * 7 + o + 3] * t;
                b += Dz[kz * 7 + o + 3] * t;
            }
            A[i] = a;
            Cz[i] = b;
        }
    } else {
        for (int i = tid; i < na; i += NT) A[i] = th[ya * ncx + i];
    }
    __syncthreads();
    for (int i = tid; i < nbr; i += NT) {
        const int ky = y0 + i / ncx, kx = i % ncx;
        float ap = 0.f, ad = 0.f, cp = 0.f;
#pragma unroll
        for (int o = -3; o <= 3; ++o) {
            int k = ky + o;
            if (k < 0 || k >= ncy) continue;
            const int j = (k - ya) * ncx + kx;
            float a = A[j];
            ap += Py[ky * 7 + o + 3] * a;
            ad += Dy[ky * 7 + o + 3] * a;
            if (dim == 3) cp += Py[ky * 7 + o + 3] * Cz[j];
        }
        AP[i] = ap;
        AD[i] = ad;
        CP[i] = cp;
    }
    __syncthreads();
    double acc[1] = {0.0};
    const float* thp = th + (long long)kz * plane + (long long)y0 * ncx;
    float* gp = out_grad + (long long)c * ncz * plane + (long long)kz * plane + (long long)y0 * ncx;
    for (int i = tid; i < nbr; i += NT) {
        const int kx = i % ncx, row = i - kx;
        float o_ = 0.f;
#pragma unroll
        for (int o = -3; o <= 3; ++o) {
            int k = kx + o;
            if (k < 0 || k >= ncx) continue;
            const int j = row + k;
            o_ += Dx[kx * 7 + o + 3] * AP[j] + Px[kx * 7 + o + 3] * (AD[j] + CP[j]);
        }
        gp[i] = scale * o_;
        acc[0] += (double)thp[i] * (double)o_;
    }
    block_sum<NT, 1>(acc, red);
    if (tid == 0) regpart[r] = acc[0];
}

// --------------------------------------------------------------- fused 3D
template <int TX, int TY, int SIM>
__global__ void __launch_bounds__(TX* TY)
k_fused3(const LaunchCtx C) {
    constexpr int NT = TX * TY;
    constexpr int NF = (SIM == AIR_SIM_NCC) ? 3 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);          // 8 * NT/64 doubles
    float* lds = reinterpret_cast<float*>(smem_raw + 8 * sizeof(double) * (NT / 64));
    const int tid = threadIdx.x;
    const int item = xcd_item(blockIdx.x, C.ntiles_total, C.nreg_total);
    if (item < 0) return;

    if (item >= C.ntiles_total) {
        const int r = item - C.ntiles_total;
        const int pair = find_pair<true>(C.pairs, C.npairs, r);
        const PairDesc P = C.pairs[pair];
        const float* theta = C.theta_tab ? C.theta_tab[pair] : C.theta0;
        float* rg = reinterpret_cast<float*>(C.ws + C.L.reggrad) + P.param_off;
        double* rp = reinterpret_cast<double*>(C.ws + C.L.regpart) + P.regpart_off;
        reg_block<NT>(P, C.consts, theta, rg, P.lambda * 2.0f * P.inv_xr, rp,
                      r - P.reg_begin, 3, lds, red);
        return;
    }
    const int pair = find_pair<false>(C.pairs, C.npairs, item);
    const PairDesc P = C.pairs[pair];
    const float* __restrict__ F = C.fixed_tab ? C.fixed_tab[pair] : C.fixed0;
    const float* __restrict__ M = C.moving_tab ? C.moving_tab[pair] : C.moving0;
    const float* __restrict__ theta = C.theta_tab ? C.theta_tab[pair] : C.theta0;

    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int sx = P.sp[0], sy = P.sp[1], sz = P.sp[2];
    const int ncx = P.nc[0], ncy = P.nc[1];
    const int WxM = P.win[0], WyM = P.win[1], WzM = P.win[2];

    int t = item - P.tile_begin;
    if (t == 0 && tid == 0) reinterpret_cast<uint32_t*>(C.ws + C.L.flags)[pair] = 0u;
    const int tx = t % P.ntile[0];
    t /= P.ntile[0];
    const int ty = t % P.ntile[1];
    const int tz = t / P.ntile[1];
    const int x0 = tx * TX, y0 = ty * TY;
    const int ncell_z = (nz - 1) / sz + 1;
    const int cz_b = tz * P.col_cells;
    const int cz_e = min(cz_b + P.col_cells, ncell_z);
    int cx0, Wx, cy0, Wy;
    ctrl_window(x0, min(x0 + TX, nx), sx, &cx0, &Wx);
    ctrl_window(y0, min(y0 + TY, ny), sy, &cy0, &Wy);
    const int cz0 = cz_b, Wz = cz_e - cz_b + 3;

    // LDS carve-up
    float* T1 = lds;                              // [3][WzM][WyM][TX]
    float* E = T1 + a4(3 * WzM * WyM * TX);       // [NF*3][TY][TX]
    float* G = E + a4(NF * 3 * TY * TX);          // [NF*3][WyM][TX]
    float* WXT = G + a4(NF * 3 * WyM * TX);       // [TX][WxM]
    float* WYT = WXT + a4(TX * WxM);              // [TY][WyM]
    float* WZT = WYT + a4(TY * WyM);              // [sz][4]

    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool act = (x < nx) && (y < ny);
    const int xc = min(x, nx - 1), yc = min(y, ny - 1);
    const int ix = xc / sx, iy = yc / sy;
    const float* wtx = C.consts + P.wtab_off[0] + (xc - ix * sx) * 4;
    const float* wty = C.consts + P.wtab_off[1] + (yc - iy * sy) * 4;
    const float wx0 = wtx[0], wx1 = wtx[1], wx2 = wtx[2], wx3 = wtx[3];
    const float wy[4] = {wty[0], wty[1], wty[2], wty[3]};
    const int ky0 = iy - cy0;

    // transposition weight tables (zero where a lane does not support a control)
    for (int i = tid; i < TX * WxM; i += NT) {
        const int q = i / WxM, k = i % WxM;
        float w = 0.f;
        const int xq = x0 + q;
        if (xq < nx) {
            const int kk = k - (xq / sx - cx0);
            if (kk >= 0 && kk < 4) w = C.consts[P.wtab_off[0] + (xq % sx) * 4 + kk];
        }
        WXT[i] = w;
    }
    for (int i = tid; i < TY * WyM; i += NT) {
        const int q = i / WyM, k = i % WyM;
        float w = 0.f;
        const int yq = y0 + q;
        if (yq < ny) {
            const int kk = k - (yq / sy - cy0);
            if (kk >= 0 && kk < 4) w = C.consts[P.wtab_off[1] + (yq % sy) * 4 + kk];
        }
        WYT[i] = w;
    }
    for (int i = tid; i < sz * 4; i += NT) WZT[i] = C.consts[P.wtab_off[2] + i];

    // 1. x-pass of the control window: T1[c][kz][ky][lx]
    {
        // each lane walks its rows j = kz Wy + ky (step TY) of every
        // component with a running (kz, ky) pair: no division per row
        const int NC = ncx * ncy * P.nc[2];
        const __amdgpu_buffer_rsrc_t rT = make_rsrc(theta, (uint32_t)(3 * NC * 4));
        const int dkz = TY / Wy, dky = TY - dkz * Wy;
        const int kzs = ly / Wy, kys = ly - kzs * Wy;
        const int tb = (cz0 * ncy + cy0) * ncx + ix;   // control (ix, cy0, cz0)
        const int ncxy = ncx * ncy;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int kz = kzs, ky = kys;
            // four rows at a time: the batch's loads are issued before any is
            // used (rows past the window read the first control instead)
            for (int j = ly; j < Wz * Wy; j += 4 * TY) {
                v2f t01[4], t23[4];
                int kzr[4], kyr[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    kzr[i] = kz;
                    kyr[i] = ky;
                    const bool ok = j + i * TY < Wz * Wy;
                    const int o =
                        ok ? (c * NC + tb + __mul24(kz, ncxy) + __mul24(ky, ncx)) * 4 : tb * 4;
                    AIR_CHECK(o >= 0 && o + 16 <= 3 * NC * 4, kDbgControlLoad);
                    t01[i] = load2(rT, o, 0);
                    t23[i] = load2(rT, o + 8, 0);
                    kz += dkz;
                    ky += dky;
                    if (ky >= Wy) {
                        ky -= Wy;
                        ++kz;
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (j + i * TY < Wz * Wy) {
                        const float v = wx0 * t01[i].x + wx1 * t01[i].y + wx2 * t23[i].x + wx3 * t23[i].y;
                        T1[((c * WzM + kzr[i]) * WyM + kyr[i]) * TX + lx] = x < nx ? v : 0.f;
                    }
                }
            }
        }
    }
    // per-tile shift for the NCC moments (a sample of F and M in the tile)
    float shF = 0.f, shW = 0.f;
    if (SIM == AIR_SIM_NCC) {
        const int xs = min(x0 + TX / 2, nx - 1), ys = min(y0 + TY / 2, ny - 1);
        const int zs = min((cz_b * sz + min(cz_e * sz, nz)) / 2, nz - 1);
        const long long vs = ((long long)zs * ny + ys) * nx + xs;
        shF = F[vs];
        shW = M[vs];
    }
    __syncthreads();

    // z-controls kept multiplied by the axis scale s_a (voxels per unit of
    // u), as in k_fused3_s8, so both kernels form the same displacements
    const float snx = P.s[0], sny = P.s[1], snz = P.s[2];
    const float sc[3] = {snx, sny, snz};
    auto vcol = [&](int c, int kz) -> float {
        const float* r = T1 + ((c * WzM + kz) * WyM + ky0) * TX + lx;
        return (wy[0] * r[0] + wy[1] * r[TX] + wy[2] * r[2 * TX] + wy[3] * r[3 * TX]) * sc[c];
    };
    float V[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) V[c][k] = vcol(c, k);
    float acc[NF][3][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[f][c][k] = 0.f;

    int cnt = 0;
    float m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f, m5 = 0.f;
    const int nx4 = nx * 4, nxy4 = nx * ny * 4;
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, (uint32_t)(P.nvox * 4));
    float* part = reinterpret_cast<float*>(C.ws + C.L.part) + P.part_off +
                  (long long)(item - P.tile_begin) * P.part_stride;

    auto flush = [&](int kzl) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < 3; ++c) E[((f * 3 + c) * TY + ly) * TX + lx] = acc[f][c][0];
        __syncthreads();
        for (int o = tid; o < NF * 3 * Wy * TX; o += NT) {
            const int q = o % TX;
            const int t2 = o / TX;
            const int ky = t2 % Wy, fc = t2 / Wy;
            float s = 0.f;
#pragma unroll
            for (int r = 0; r < TY; ++r) s += WYT[r * WyM + ky] * E[(fc * TY + r) * TX + q];
            G[(fc * WyM + ky) * TX + q] = s;
        }
        __syncthreads();
        for (int o = tid; o < NF * 3 * Wy * Wx; o += NT) {
            const int kx = o % Wx;
            const int t2 = o / Wx;
            const int ky = t2 % Wy, fc = t2 / Wy;
            const float* g = G + (fc * WyM + ky) * TX;
            // lanes whose voxels lie in the support of control cx0 + kx
            const int q0 = max(0, (cx0 + kx - 3) * sx - x0);
            const int q1 = min(TX, (cx0 + kx + 1) * sx - x0);
            float s = 0.f;
            // eight lanes' terms loaded ahead of their sums, added in lane
            // order (a term past q1 is 0)
            for (int q8 = q0; q8 < q1; q8 += 8) {
                float w[8], e[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int q = min(q8 + i, q1 - 1);
                    w[i] = q8 + i < q1 ? WXT[q * WxM + kx] : 0.f;
                    e[i] = g[q];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) s += w[i] * e[i];
            }
            part[((kzl * WyM + ky) * WxM + kx) * (NF * 3) + fc] = s;
        }
    };

    for (int cz = cz_b; cz < cz_e; ++cz) {
        const int kzl = cz - cz0;
        const int zb = cz * sz, ze = min(zb + sz, nz);
        for (int z = zb; z < ze; ++z) {
            const float4 wz = *reinterpret_cast<const float4*>(WZT + (z - zb) * 4);
            if (act) {
                const long long v = ((long long)z * ny + y) * nx + x;
                const float Fv = F[v];
                // displacement in voxels, d = u (n - 1)/2, summed in the same
                // order as k_fused3_s8; cell and mask of x + d
                float dd[3];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    dd[c] = fmaf(wz.w, V[c][3],
                                 fmaf(wz.z, V[c][2], fmaf(wz.y, V[c][1], fmaf(wz.x, V[c][0], 0.f))));
                const AxisCell ax = axis_cell(x, Disp{dd[0], 0.f}, nx);
                const AxisCell ay = axis_cell(y, Disp{dd[1], 0.f}, ny);
                const AxisCell az = axis_cell(z, Disp{dd[2], 0.f}, nz);
                const bool in = ax.in && ay.in && az.in;
                if (in) {
                    // a point on the last voxel takes the cell below with f = 1
                    const bool ex = ax.t == nx - 1, ey = ay.t == ny - 1, ez = az.t == nz - 1;
                    const int jx = ex ? nx - 2 : ax.t, jy = ey ? ny - 2 : ay.t;
                    const int jz = ez ? nz - 2 : az.t;
                    const float fx = ex ? 1.f : ax.f, fy = ey ? 1.f : ay.f, fz = ez ? 1.f : az.f;
                    const int off = ((jz * ny + jy) * nx + jx) * 4;
                    AIR_CHECK(off >= 0 && (long long)off + nxy4 + nx4 + 8 <= P.nvox * 4,
                              kDbgMovingGather);
                    const v2f a00 = load2(rM, off, 0);
                    const v2f a10 = load2(rM, off, nx4);
                    const v2f a01 = load2(rM, off, nxy4);
                    const v2f a11 = load2(rM, off, nxy4 + nx4);
                    // corners c[z][y][x]
                    const float dz00 = a01.x - a00.x, dz01 = a01.y - a00.y;
                    const float dz10 = a11.x - a10.x, dz11 = a11.y - a10.y;
                    const float e00 = a00.x + fz * dz00, e01 = a00.y + fz * dz01;
                    const float e10 = a10.x + fz * dz10, e11 = a10.y + fz * dz11;
                    const float dy0 = e10 - e00, dy1 = e11 - e01;
                    const float g0 = e00 + fy * dy0, g1 = e01 + fy * dy1;
                    const float W = g0 + fx * (g1 - g0);
                    float d[3];
                    d[0] = g1 - g0;
                    d[1] = dy0 + fx * (dy1 - dy0);
                    const float h0 = dz00 + fy * (dz10 - dz00);
                    const float h1 = dz01 + fy * (dz11 - dz01);
                    d[2] = h0 + fx * (h1 - h0);
                    // sample exactly on the last voxel: right-sided cell, zero padding
                    if (ex) d[0] = -W;
                    if (ey) d[1] = -W;
                    if (ez) d[2] = -W;
                    cnt += 1;
                    if (SIM == AIR_SIM_NCC) {
                        const float dF = Fv - shF, dW = W - shW;
                        m1 += dF;
                        m2 += dW;
                        m3 += dF * dF;
                        m4 += dW * dW;
                        m5 += dF * dW;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float gF = dF * d[c], gW = dW * d[c], g1_ = d[c];
                            acc[0][c][0] += wz.x * gF;
                            acc[0][c][1] += wz.y * gF;
                            acc[0][c][2] += wz.z * gF;
                            acc[0][c][3] += wz.w * gF;
                            acc[1][c][0] += wz.x * gW;
                            acc[1][c][1] += wz.y * gW;
                            acc[1][c][2] += wz.z * gW;
                            acc[1][c][3] += wz.w * gW;
                            acc[NF - 1][c][0] += wz.x * g1_;
                            acc[NF - 1][c][1] += wz.y * g1_;
                            acc[NF - 1][c][2] += wz.z * g1_;
                            acc[NF - 1][c][3] += wz.w * g1_;
                        }
                    } else {
                        const float e = W - Fv;
                        m1 += e * e;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float g = e * d[c];
                            acc[0][c][0] += wz.x * g;
                            acc[0][c][1] += wz.y * g;
                            acc[0][c][2] += wz.z * g;
                            acc[0][c][3] += wz.w * g;
                        }
                    }
                }
            }
        }
        flush(kzl);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[f][c][0] = acc[f][c][1];
                acc[f][c][1] = acc[f][c][2];
                acc[f][c][2] = acc[f][c][3];
                acc[f][c][3] = 0.f;
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            V[c][0] = V[c][1];
            V[c][1] = V[c][2];
            V[c][2] = V[c][3];
            V[c][3] = (kzl + 4 < Wz) ? vcol(c, kzl + 4) : 0.f;
        }
    }
    // the last three column controls of the window
    for (int k = Wz - 3; k < Wz; ++k) {
        flush(k);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[f][c][0] = acc[f][c][1];
                acc[f][c][1] = acc[f][c][2];
                acc[f][c][2] = acc[f][c][3];
                acc[f][c][3] = 0.f;
            }
    }
    // tile statistics
    double st[6] = {(double)cnt, (double)m1, (double)m2, (double)m3, (double)m4, (double)m5};
    block_sum<NT, 6>(st, red);
    if (tid == 0) {
        double* slot = reinterpret_cast<double*>(C.ws + C.L.stats) + (long long)item * kStatWords;
#pragma unroll
        for (int k = 0; k < 6; ++k) slot[k] = st[k];
        slot[6] = shF;
        slot[7] = shW;
    }
}

// --------------------------------------------------------------- fused 3D, spacing 8
// The same computation as k_fused3 for control spacing 8 on every axis with
// cell-aligned tiles (TX, TY multiples of 8): the cell structure and the
// cubic weights w_k(r/8) are compile-time, the voxel body is branch-free, the
// gathers of the next layer are in flight while the current one finishes,
// the per-plane register slots rotate instead of shifting, and the LDS
// transposes read each staged value once. The kernel is bound by VALU issue
// (about 125 vector instructions per voxel for NCC), not by HBM.
struct W8 {
    float w[9][4];  // row 8 (t = 1) is the next cell's first layer
};
constexpr W8 make_w8() {
    W8 t{};
    for (int r = 0; r <= 8; ++r) {
        const double x = r / 8.0;
        t.w[r][0] = (float)((1 - x) * (1 - x) * (1 - x) / 6.0);
        t.w[r][1] = (float)((3 * x * x * x - 6 * x * x + 4) / 6.0);
        t.w[r][2] = (float)((-3 * x * x * x + 3 * x * x + 3 * x + 1) / 6.0);
        t.w[r][3] = (float)(x * x * x / 6.0);
    }
    return t;
}
constexpr W8 kW8 = make_w8();

template <int TX, int TY, int SIM>
__global__ void __launch_bounds__(TX* TY)
k_fused3_s8(const LaunchCtx C) {
    constexpr int S = 8;
    constexpr int NT = TX * TY;
    constexpr int NF = (SIM == AIR_SIM_NCC) ? 3 : 1;
    constexpr int FC = NF * 3;
    constexpr int WXC = TX / S + 3, WYC = TY / S + 3;
    constexpr int GP = TX + 4;  // padded G rows (16-byte aligned, spread over banks)
    static_assert(TX % S == 0 && TY % S == 0, "cell-aligned tiles");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);
    float* lds = reinterpret_cast<float*>(smem_raw + 8 * sizeof(double) * (NT / 64));
    const int tid = threadIdx.x;
    const int item = xcd_item(blockIdx.x, C.ntiles_total, C.nreg_total);
    if (item < 0) return;

    if (item >= C.ntiles_total) {
        const int r = item - C.ntiles_total;
        const int pair = find_pair<true>(C.pairs, C.npairs, r);
        const PairDesc P = C.pairs[pair];
        const float* theta = C.theta_tab ? C.theta_tab[pair] : C.theta0;
        float* rg = reinterpret_cast<float*>(C.ws + C.L.reggrad) + P.param_off;
        double* rp = reinterpret_cast<double*>(C.ws + C.L.regpart) + P.regpart_off;
        reg_block<NT>(P, C.consts, theta, rg, P.lambda * 2.0f * P.inv_xr, rp,
                      r - P.reg_begin, 3, lds, red);
        return;
    }
    const int pair = find_pair<false>(C.pairs, C.npairs, item);
    const PairDesc P = C.pairs[pair];
    const float* __restrict__ F = C.fixed_tab ? C.fixed_tab[pair] : C.fixed0;
    const float* __restrict__ M = C.moving_tab ? C.moving_tab[pair] : C.moving0;
    const float* __restrict__ theta = C.theta_tab ? C.theta_tab[pair] : C.theta0;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int ncx = P.nc[0], ncy = P.nc[1];
    const int WxM = P.win[0], WyM = P.win[1], WzM = P.win[2];
    int t = item - P.tile_begin;
    if (t == 0 && tid == 0) reinterpret_cast<uint32_t*>(C.ws + C.L.flags)[pair] = 0u;
    const int tx = t % P.ntile[0];
    t /= P.ntile[0];
    const int ty = t % P.ntile[1];
    const int tz = t / P.ntile[1];
    const int x0 = tx * TX, y0 = ty * TY;
    const int ncell_z = (nz - 1) / S + 1;
    const int cz_b = tz * P.col_cells;
    const int cz_e = min(cz_b + P.col_cells, ncell_z);
    const int cx0 = x0 / S, cy0 = y0 / S;
    const int Wx = (min(x0 + TX, nx) - 1) / S + 4 - cx0;
    const int Wy = (min(y0 + TY, ny) - 1) / S + 4 - cy0;
    const int cz0 = cz_b, Wz = cz_e - cz_b + 3;

    float* T1 = lds;                       // [3][WzM][WYC][TX]
    float* E = T1 + a4(3 * WzM * WYC * TX);  // [FC][TY][TX]
    float* G = E + a4(FC * TY * TX);         // [FC][WYC][GP]

    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool act = (x < nx) && (y < ny);
    const int xc = min(x, nx - 1), yc = min(y, ny - 1);
    const int ix = xc / S, iy = yc / S;
    float wx[4], wy[4];
    {
        const float* a = C.consts + P.wtab_off[0] + (xc - ix * S) * 4;
        const float* b = C.consts + P.wtab_off[1] + (yc - iy * S) * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wx[k] = a[k];
            wy[k] = b[k];
        }
    }
    const int ky0 = iy - cy0;
    // z-controls of each lane's column are kept multiplied by the axis scale
    // s_a (voxels per unit of u), so a layer's displacement in voxels is one
    // weighted sum of them
    const float snx = P.s[0], sny = P.s[1], snz = P.s[2];
    {
        // rows (kz, ky) of the x-interpolated control window, component by
        // component; each lane walks its rows j = kz Wy + ky (step TY) with a
        // running (kz, ky) pair instead of a division per row
        const int NC = ncx * ncy * P.nc[2];
        const __amdgpu_buffer_rsrc_t rT = make_rsrc(theta, (uint32_t)(3 * NC * 4));
        const int dkz = TY / Wy, dky = TY - dkz * Wy;
        const int kzs = ly / Wy, kys = ly - kzs * Wy;
        const int tb = (cz0 * ncy + cy0) * ncx + ix;   // control (ix, cy0, cz0)
        const int ncxy = ncx * ncy;
        int kz = kzs, ky = kys;
        // four rows at a time, all three components: the batch's loads are
        // issued before any is used (rows past the window read the first
        // control instead)
        for (int j = ly; j < Wz * Wy; j += 4 * TY) {
            v2f t01[4][3], t23[4][3];
            int kzr[4], kyr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                kzr[i] = kz;
                kyr[i] = ky;
                const bool ok = j + i * TY < Wz * Wy;
                const int o0 = ok ? (tb + __mul24(kz, ncxy) + __mul24(ky, ncx)) * 4 : tb * 4;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int o = o0 + c * NC * 4;
                    AIR_CHECK(o >= 0 && o + 16 <= 3 * NC * 4, kDbgControlLoad);
                    t01[i][c] = load2(rT, o, 0);
                    t23[i][c] = load2(rT, o + 8, 0);
                }
                kz += dkz;
                ky += dky;
                if (ky >= Wy) {
                    ky -= Wy;
                    ++kz;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (j + i * TY < Wz * Wy) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float v = wx[0] * t01[i][c].x + wx[1] * t01[i][c].y +
                                        wx[2] * t23[i][c].x + wx[3] * t23[i][c].y;
                        T1[((c * WzM + kzr[i]) * WYC + kyr[i]) * TX + lx] = x < nx ? v : 0.f;
                    }
                }
            }
        }
    }
    float shF = 0.f, shW = 0.f;
    if (SIM == AIR_SIM_NCC) {
        const int xs = min(x0 + TX / 2, nx - 1), ys = min(y0 + TY / 2, ny - 1);
        const int zs = min((cz_b * S + min(cz_e * S, nz)) / 2, nz - 1);
        const long long vs = ((long long)zs * ny + ys) * nx + xs;
        shF = F[vs];
        shW = M[vs];
    }
    __syncthreads();

    const float sc[3] = {snx, sny, snz};
    auto vcol = [&](int c, int kz) -> float {
        const float* r = T1 + ((c * WzM + kz) * WYC + ky0) * TX + lx;
        return (wy[0] * r[0] + wy[1] * r[TX] + wy[2] * r[2 * TX] + wy[3] * r[3 * TX]) * sc[c];
    };
    float V[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) V[c][k] = vcol(c, k);
    v4f acc[NF][3];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[f][c] = v4f{0.f, 0.f, 0.f, 0.f};
    // Accumulator and control slots rotate with the cell: control plane kz
    // (local) lives in slot kz mod 4 of V and of every acc, so moving to the
    // next cell only refills one slot. The cell loop is unrolled four times
    // to keep every slot index a compile-time constant.
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    float cnt = 0.f;
    float m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f, m5 = 0.f;
    const float nzm2 = (float)(nz - 2);
    // per lane, relative to the lane's voxel: cells start at lo = -x at
    // least and at hc = n - 2 - x at most
    const float lox = -(float)xc, hcx = (float)(nx - 2 - xc);
    const float loy = -(float)yc, hcy = (float)(ny - 2 - yc);
    const int nx4 = nx * 4, nxy4 = nx * ny * 4;
    const float nyf = (float)ny;
    const int lane4 = (yc * nx + xc) * 4;   // byte offset of voxel (x, y, 0)
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, (uint32_t)(P.nvox * 4));
    const __amdgpu_buffer_rsrc_t rF = make_rsrc(F, (uint32_t)(P.nvox * 4));
    const int fl4 = (yc * nx + xc) * 4;   // byte offset of F at (x, y, 0)
    float* part = reinterpret_cast<float*>(C.ws + C.L.part) + P.part_off +
                  (long long)(item - P.tile_begin) * P.part_stride;

    // y and x passes of control plane kzl, whose z sums the threads have
    // written to E
    auto flush_xy = [&](int kzl) {
        __syncthreads();
        // y: task (fc, lane column q) -> WYC outputs
        for (int task = tid; task < FC * TX; task += NT) {
            const int q = task % TX, fc = task / TX;
            float o[WYC];
#pragma unroll
            for (int k = 0; k < WYC; ++k) o[k] = 0.f;
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const float e = E[(fc * TY + r) * TX + q];
#pragma unroll
                for (int k = 0; k < 4; ++k) o[r / S + k] += kW8.w[r % S][k] * e;
            }
#pragma unroll
            for (int k = 0; k < WYC; ++k) G[(fc * WYC + k) * GP + q] = o[k];
        }
        __syncthreads();
        // x: task (fc, ky) -> Wx outputs of one partial row (tasks laid out
        // over the compile-time row count, so no runtime division)
        for (int task = tid; task < FC * WYC; task += NT) {
            const int ky = task % WYC, fc = task / WYC;
            if (ky >= Wy) continue;
            const float* g = G + (fc * WYC + ky) * GP;
            float o[WXC];
#pragma unroll
            for (int k = 0; k < WXC; ++k) o[k] = 0.f;
#pragma unroll
            for (int q4 = 0; q4 < TX; q4 += 4) {
                const float4 gv = *reinterpret_cast<const float4*>(g + q4);
                const float gg[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = q4 + i;
#pragma unroll
                    for (int k = 0; k < 4; ++k) o[q / S + k] += kW8.w[q % S][k] * gg[i];
                }
            }
            float* dst = part + ((long long)(kzl * WyM + ky) * WxM) * FC + fc;
#pragma unroll
            for (int k = 0; k < WXC; ++k)
                if (k < Wx) dst[k * FC] = o[k];
        }
    };

    // Two-stage pipeline over the layers: stage 1 of the next layer (sample
    // point, cell, its four gathers) is issued before stage 2 of the current
    // one (interpolation, statistics, adjoint), so two layers of gathers are
    // in flight.
    struct Prep {
        v2f a00, a10, a01, a11;
        float fx, fy, fz, m, Fv;
        bool ex, ey, ez;
    };
    int cz = cz_b;
    // a running statistic that depends on the previous layer's gathers
    auto dep = [&]() -> float { return SIM == AIR_SIM_NCC ? m2 : m1; };
    // stage 1 of layer r of cell cz; tap k of the cell is V slot (k + PH) & 3
    auto prep = [&](int r, float dv, auto ph) -> Prep {
        constexpr int PH = decltype(ph)::value;
        // Branch-free: the cell is clamped into the volume so every load is
        // in range; m = 1 inside the mask, 0 outside (or for lanes / layers
        // past the volume) scales every contribution.
        const int z = cz * S + r;
        Prep q;
        // F through its buffer descriptor: the lane's offset is fixed, the
        // plane's is a scalar. Default cache policy: a 16-lane tile row reads
        // half of each 128-byte line and the neighbouring tile the other half
        // (a non-temporal hint fetched every F line from HBM twice)
        AIR_CHECK((long long)fl4 + (long long)min(z, nz - 1) * nxy4 + 4 <= P.nvox * 4,
                  kDbgFixedLoad);
        q.Fv = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                             rF, fl4, min(z, nz - 1) * nxy4, 0));
        float w0 = kW8.w[r][0], w1 = kW8.w[r][1], w2 = kW8.w[r][2], w3 = kW8.w[r][3];
        // every uniform input of this stage passes through an empty asm that
        // also reads `dv` (produced by the previous layer's stage 2), so
        // neither the arithmetic nor the gathers of this layer can be
        // hoisted more than one layer ahead of their use
        asm volatile("" : "+s"(w0), "+s"(w1), "+s"(w2), "+s"(w3) : "v"(dv));
        // displacement in voxels d = s u (V holds s times the z-controls):
        // the cell and the mask are decided on the exact sum x + d (x an
        // integer), never on a rounded sample point (the first term is an
        // fma with +0: a -0 product becomes +0, so f below is never -0)
        float dd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dd[c] = fmaf(w3, V[c][(PH + 3) & 3],
                         fmaf(w2, V[c][(PH + 2) & 3],
                              fmaf(w1, V[c][(PH + 1) & 3], fmaf(w0, V[c][PH], 0.f))));
        const float dx = dd[0], dy = dd[1], dz = dd[2];
        const float zf = (float)z;
        // cell [x + c, x + c + 1] with c = floor(d) clamped to [-x, n - 2 - x]
        // so that every load is in range. Then f = d - c is exact (c is an
        // integer no larger in magnitude than d's integer part), and it lies
        // in [0, 1] iff x + d lies in [0, n - 1]: below the range c is
        // clamped up and f < 0; above it c is clamped down ("e") and f > 1,
        // except for d the integer n - 1 - x (f == 1), the last voxel, whose
        // derivative is right-sided (zero padding)
        const float flx = floorf(dx), fly = floorf(dy), flz = floorf(dz);
        const float clx = __builtin_amdgcn_fmed3f(flx, lox, hcx);
        const float cly = __builtin_amdgcn_fmed3f(fly, loy, hcy);
        const float clz = __builtin_amdgcn_fmed3f(flz, -zf, nzm2 - zf);
        q.ex = flx > clx;
        q.ey = fly > cly;
        q.ez = flz > clz;
        q.fx = dx - clx;
        q.fy = dy - cly;
        q.fz = dz - clz;
        constexpr uint32_t kOne = 0x3f800000u;   // bits of 1.0f: f in [0, 1]
        // (bitwise, not short-circuit: every test is a compare, no branch;
        // a negative f has its sign bit set and fails like f > 1)
        const bool in = (int)(__float_as_uint(q.fx) <= kOne) &
                        (int)(__float_as_uint(q.fy) <= kOne) &
                        (int)(__float_as_uint(q.fz) <= kOne) & (int)act & (int)(z < nz);
        q.m = in ? 1.f : 0.f;
        // byte offset of the cell's first corner: the row step clz ny + cly
        // is an exact float (|.| < 2^24), the rest 24-bit integer arithmetic
        const int rows = (int)fmaf(clz, nyf, cly);
        const int off = (int)((unsigned)(__mul24(rows, nx) + (int)clx) * 4u + (unsigned)lane4 +
                              (unsigned)z * (unsigned)nxy4);
        AIR_CHECK(off >= 0 && (long long)off + nxy4 + nx4 + 8 <= P.nvox * 4, kDbgMovingGather);
        q.a00 = load2(rM, off, 0);
        q.a10 = load2(rM, off, nx4);
        q.a01 = load2(rM, off, nxy4);
        q.a11 = load2(rM, off, nxy4 + nx4);
        return q;
    };
    // stage 2 of layer r: interpolation, statistics and the z taps of the
    // adjoint into acc slot (k + PH) & 3
    auto finish = [&](int r, const Prep& q, auto ph) {
        constexpr int PH = decltype(ph)::value;
        const float w0 = kW8.w[r][0], w1 = kW8.w[r][1], w2 = kW8.w[r][2], w3 = kW8.w[r][3];
        auto tap = [&](v4f& a, float g) {
            a[PH] += w0 * g;
            a[(PH + 1) & 3] += w1 * g;
            a[(PH + 2) & 3] += w2 * g;
            a[(PH + 3) & 3] += w3 * g;
        };
        const float Fv = q.Fv;
        const float m = q.m, fx = q.fx, fy = q.fy, fz = q.fz;
        const v2f a00 = q.a00, a10 = q.a10, a01 = q.a01, a11 = q.a11;
        const float dz00 = a01.x - a00.x, dz01 = a01.y - a00.y;
        const float dz10 = a11.x - a10.x, dz11 = a11.y - a10.y;
        const float e00 = a00.x + fz * dz00, e01 = a00.y + fz * dz01;
        const float e10 = a10.x + fz * dz10, e11 = a10.y + fz * dz11;
        const float dy0 = e10 - e00, dy1 = e11 - e01;
        const float g0 = e00 + fy * dy0, g1 = e01 + fy * dy1;
        const float W = g0 + fx * (g1 - g0);
        const float h0 = dz00 + fy * (dz10 - dz00);
        const float h1 = dz01 + fy * (dz11 - dz01);
        float d[3];
        d[0] = m * (q.ex ? -W : g1 - g0);
        d[1] = m * (q.ey ? -W : dy0 + fx * (dy1 - dy0));
        d[2] = m * (q.ez ? -W : h0 + fx * (h1 - h0));
        cnt += m;
        if (SIM == AIR_SIM_NCC) {
            const float dF = m * (Fv - shF), dW = m * (W - shW);
            m1 += dF;
            m2 += dW;
            m3 += dF * dF;
            m4 += dW * dW;
            m5 += dF * dW;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                tap(acc[0][c], dF * d[c]);
                tap(acc[1][c], dW * d[c]);
                tap(acc[NF - 1][c], d[c]);
            }
        } else {
            const float e = m * (W - Fv);
            m1 += e * e;
#pragma unroll
            for (int c = 0; c < 3; ++c) tap(acc[0][c], (W - Fv) * d[c]);
        }
    };
    Prep A = prep(0, dep(), I0{});
    // one cell (S layers) of local index kzl, whose first control plane is
    // in slot PH = kzl & 3; afterwards that plane is complete and flushed,
    // and its slots take control plane kzl + 4
    auto cell = [&](int kzl, auto ph) {
        constexpr int PH = decltype(ph)::value;
        cz = cz0 + kzl;
        // Double buffer without copies: B (odd layer) is issued before the
        // even layer finishes, A (next even layer) before the odd one. Layer
        // S of this cell (weights row t = 1, same V) is the next cell's layer
        // 0; past the last cell it is a clamped, in-range dummy.
        // The scheduling barriers keep each layer's gathers issued before the
        // other layer's stage 2 starts: without them the compiler may order
        // the stages so that every iteration first waits for all loads.
        for (int r = 0; r < S; r += 2) {
            Prep B = prep(r + 1, dep(), ph);
            __builtin_amdgcn_sched_barrier(0);
            finish(r, A, ph);
            A = prep(r + 2, dep(), ph);
            __builtin_amdgcn_sched_barrier(0);
            finish(r + 1, B, ph);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                E[((f * 3 + c) * TY + ly) * TX + lx] = acc[f][c][PH];
                acc[f][c][PH] = 0.f;
            }
        flush_xy(kzl);
#pragma unroll
        for (int c = 0; c < 3; ++c) V[c][PH] = (kzl + 4 < Wz) ? vcol(c, kzl + 4) : 0.f;
    };
    const int ncell = cz_e - cz_b;
    for (int kzl = 0; kzl < ncell; kzl += 4) {
        cell(kzl, I0{});
        if (kzl + 1 < ncell) cell(kzl + 1, I1{});
        if (kzl + 2 < ncell) cell(kzl + 2, I2{});
        if (kzl + 3 < ncell) cell(kzl + 3, I3{});
    }
    // the last three control planes, in slots (ncell + j) & 3
    for (int j = 0; j < 3; ++j) {
        const int sl = (ncell + j) & 3;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const v4f a = acc[f][c];
                E[((f * 3 + c) * TY + ly) * TX + lx] =
                    sl == 0 ? a[0] : (sl == 1 ? a[1] : (sl == 2 ? a[2] : a[3]));
            }
        flush_xy(ncell + j);
    }
    double st[6] = {(double)cnt, (double)m1, (double)m2, (double)m3, (double)m4, (double)m5};
    block_sum<NT, 6>(st, red);
    if (tid == 0) {
        double* slot = reinterpret_cast<double*>(C.ws + C.L.stats) + (long long)item * kStatWords;
#pragma unroll
        for (int k = 0; k < 6; ++k) slot[k] = st[k];
        slot[6] = shF;
        slot[7] = shW;
    }
}

// --------------------------------------------------------------- fused 2D
// Lanes over x (TX), the column axis is y.
template <int TX, int SIM>
__global__ void __launch_bounds__(TX)
k_fused2(const LaunchCtx C) {
    constexpr int NT = TX;
    constexpr int NF = (SIM == AIR_SIM_NCC) ? 3 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);
    float* lds = reinterpret_cast<float*>(smem_raw + 8 * sizeof(double) * (NT / 64));
    const int tid = threadIdx.x;
    const int item = xcd_item(blockIdx.x, C.ntiles_total, C.nreg_total);
    if (item < 0) return;

    if (item >= C.ntiles_total) {
        const int r = item - C.ntiles_total;
        const int pair = find_pair<true>(C.pairs, C.npairs, r);
        const PairDesc P = C.pairs[pair];
        const float* theta = C.theta_tab ? C.theta_tab[pair] : C.theta0;
        float* rg = reinterpret_cast<float*>(C.ws + C.L.reggrad) + P.param_off;
        double* rp = reinterpret_cast<double*>(C.ws + C.L.regpart) + P.regpart_off;
        reg_block<NT>(P, C.consts, theta, rg, P.lambda * 2.0f * P.inv_xr, rp,
                      r - P.reg_begin, 2, lds, red);
        return;
    }
    const int pair = find_pair<false>(C.pairs, C.npairs, item);
    const PairDesc P = C.pairs[pair];
    const float* __restrict__ F = C.fixed_tab ? C.fixed_tab[pair] : C.fixed0;
    const float* __restrict__ M = C.moving_tab ? C.moving_tab[pair] : C.moving0;
    const float* __restrict__ theta = C.theta_tab ? C.theta_tab[pair] : C.theta0;
    const int nx = P.n[0], ny = P.n[1];
    const int sx = P.sp[0], sy = P.sp[1];
    const int ncx = P.nc[0];
    const int WxM = P.win[0], WyM = P.win[2];  // column window stored in win[2]
    int t = item - P.tile_begin;
    if (t == 0 && tid == 0) reinterpret_cast<uint32_t*>(C.ws + C.L.flags)[pair] = 0u;
    const int tx = t % P.ntile[0];
    const int tyc = t / P.ntile[0];
    const int x0 = tx * TX;
    const int ncell_y = (ny - 1) / sy + 1;
    const int cy_b = tyc * P.col_cells;
    const int cy_e = min(cy_b + P.col_cells, ncell_y);
    int cx0, Wx;
    ctrl_window(x0, min(x0 + TX, nx), sx, &cx0, &Wx);
    const int cy0 = cy_b, Wy = cy_e - cy_b + 3;

    float* T1 = lds;                     // [2][WyM][TX]
    float* E = T1 + a4(2 * WyM * TX);    // [3][NF*2][TX] (three control rows at the end)
    float* WXT = E + a4(3 * NF * 2 * TX);    // [TX][WxM]
    float* WYT = WXT + a4(TX * WxM);     // [sy][4]
    const int lx = tid, x = x0 + lx;
    const bool act = x < nx;
    const int xc = min(x, nx - 1), ix = xc / sx;
    const float* wtx = C.consts + P.wtab_off[0] + (xc - ix * sx) * 4;
    const float wx0 = wtx[0], wx1 = wtx[1], wx2 = wtx[2], wx3 = wtx[3];
    // x weights of this lane's pixel for the window's controls (one thread
    // per lane): its own four weights at controls ix - cx0 .. ix - cx0 + 3
    {
        const int kb = ix - cx0;
        for (int k = 0; k < WxM; ++k) {
            const int kk = k - kb;
            const float w = kk == 0 ? wx0 : kk == 1 ? wx1 : kk == 2 ? wx2 : wx3;
            WXT[lx * WxM + k] = (act && kk >= 0 && kk < 4) ? w : 0.f;
        }
    }
    for (int i = tid; i < sy * 4; i += NT) WYT[i] = C.consts[P.wtab_off[1] + i];
    {
        // rows r = c Wy + ky of the x-interpolated window, eight at a time
        // (the whole window of a 1-cell column): the loads of a batch are
        // issued before any is used
        const int NC = ncx * P.nc[1];
        const __amdgpu_buffer_rsrc_t rT = make_rsrc(theta, (uint32_t)(2 * NC * 4));
        constexpr int RW = 8;
        for (int r0 = 0; r0 < 2 * Wy; r0 += RW) {
            v2f t01[RW], t23[RW];
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                const int r = min(r0 + i, 2 * Wy - 1);
                const int c = r >= Wy ? 1 : 0, ky = r - c * Wy;
                const int o = (c * NC + (cy0 + ky) * ncx + ix) * 4;
                AIR_CHECK(o >= 0 && o + 16 <= 2 * NC * 4, kDbgControlLoad);
                t01[i] = load2(rT, o, 0);
                t23[i] = load2(rT, o + 8, 0);
            }
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                const int r = r0 + i;
                if (r < 2 * Wy) {
                    const int c = r >= Wy ? 1 : 0, ky = r - c * Wy;
                    const float v = wx0 * t01[i].x + wx1 * t01[i].y + wx2 * t23[i].x + wx3 * t23[i].y;
                    T1[(c * WyM + ky) * TX + lx] = act ? v : 0.f;
                }
            }
        }
    }
    float shF = 0.f, shW = 0.f;
    if (SIM == AIR_SIM_NCC) {
        const int xs = min(x0 + TX / 2, nx - 1);
        const int ys = min((cy_b * sy + min(cy_e * sy, ny)) / 2, ny - 1);
        shF = F[(long long)ys * nx + xs];
        shW = M[(long long)ys * nx + xs];
    }
    __syncthreads();
    float V[2][4];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) V[c][k] = T1[(c * WyM + k) * TX + lx];
    float acc[NF][2][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[f][c][k] = 0.f;
    int cnt = 0;
    float m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f, m5 = 0.f;
    const float snx = P.s[0], sny = P.s[1];
    const int nx4 = nx * 4;
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, (uint32_t)(P.nvox * 4));
    float* part = reinterpret_cast<float*>(C.ws + C.L.part) + P.part_off +
                  (long long)(item - P.tile_begin) * P.part_stride;
    // x-transpose of the nr completed control rows kyl .. kyl + nr - 1
    // (accumulator slots 0 .. nr - 1) into this tile's partials
    auto flush = [&](int kyl, int nr) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
            if (r < nr)
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int c = 0; c < 2; ++c) E[((r * NF + f) * 2 + c) * TX + lx] = acc[f][c][r];
        __syncthreads();
        for (int o = tid; o < nr * NF * 2 * Wx; o += NT) {
            const int kx = o % Wx, rfc = o / Wx;
            const int r = rfc / (NF * 2), fc = rfc - r * (NF * 2);
            const int q0 = max(0, (cx0 + kx - 3) * sx - x0);
            const int q1 = min(TX, (cx0 + kx + 1) * sx - x0);
            float s = 0.f;
            // QB lanes' terms loaded ahead of their sums, added in lane
            // order (a term past q1 is 0): one round for spacing <= 8 with
            // MSE; NCC takes 16 at a time, as 32 cost its 4096^2 launch more
            // registers than the shorter wait saved
            constexpr int QB = SIM == AIR_SIM_NCC ? 16 : 32;
            for (int q8 = q0; q8 < q1; q8 += QB) {
                float w[QB], e[QB];
#pragma unroll
                for (int i = 0; i < QB; ++i) {
                    const int q = min(q8 + i, q1 - 1);
                    w[i] = q8 + i < q1 ? WXT[q * WxM + kx] : 0.f;
                    e[i] = E[rfc * TX + q];
                }
#pragma unroll
                for (int i = 0; i < QB; ++i) s += w[i] * e[i];
            }
            part[((kyl + r) * WxM + kx) * (NF * 2) + fc] = s;
        }
        __syncthreads();
    };
    for (int cy = cy_b; cy < cy_e; ++cy) {
        const int kyl = cy - cy0;
        const int yb = cy * sy, ye = min(yb + sy, ny);
        // Rows in groups of RB: the loads of a whole group (F and the two
        // corner pairs of each row, at cells clamped into the image so that
        // every address is valid) are issued before any row's arithmetic,
        // so a group waits for memory once; the rows are then added in
        // order, as one at a time would.
        constexpr int RB = 8;
        for (int yg = yb; yg < ye; yg += RB) {
            float4 wyr[RB];
            float Fr[RB], fxr[RB], fyr[RB];
            v2f a0r[RB], a1r[RB];
            bool inr[RB], exr[RB], eyr[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int y = min(yg + i, ye - 1);
                wyr[i] = *reinterpret_cast<const float4*>(WYT + (y - yb) * 4);
                Fr[i] = F[(long long)y * nx + xc];
                float u[2];
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    u[c] = wyr[i].x * V[c][0] + wyr[i].y * V[c][1] + wyr[i].z * V[c][2] +
                           wyr[i].w * V[c][3];
                // cell and mask of x + d, d = u (n - 1)/2 in voxels
                const AxisCell ax = axis_cell(x, Disp{u[0] * snx, 0.f}, nx);
                const AxisCell ay = axis_cell(y, Disp{u[1] * sny, 0.f}, ny);
                inr[i] = act && yg + i < ye && ax.in && ay.in;
                // a point on the last pixel takes the cell below with f = 1
                exr[i] = ax.t == nx - 1;
                eyr[i] = ay.t == ny - 1;
                const int jx = min(max(exr[i] ? nx - 2 : ax.t, 0), nx - 2);
                const int jy = min(max(eyr[i] ? ny - 2 : ay.t, 0), ny - 2);
                fxr[i] = exr[i] ? 1.f : ax.f;
                fyr[i] = eyr[i] ? 1.f : ay.f;
                const int off = (jy * nx + jx) * 4;
                AIR_CHECK(off >= 0 && (long long)off + nx4 + 8 <= P.nvox * 4, kDbgMovingGather);
                a0r[i] = load2(rM, off, 0);
                a1r[i] = load2(rM, off, nx4);
            }
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                if (inr[i]) {
                    const float4 wy = wyr[i];
                    const float Fv = Fr[i], fx = fxr[i], fy = fyr[i];
                    const v2f a0 = a0r[i], a1 = a1r[i];
                    const float dy0 = a1.x - a0.x, dy1 = a1.y - a0.y;
                    const float g0 = a0.x + fy * dy0, g1 = a0.y + fy * dy1;
                    const float W = g0 + fx * (g1 - g0);
                    float d[2];
                    d[0] = g1 - g0;
                    d[1] = dy0 + fx * (dy1 - dy0);
                    if (exr[i]) d[0] = -W;
                    if (eyr[i]) d[1] = -W;
                    cnt += 1;
                    if (SIM == AIR_SIM_NCC) {
                        const float dF = Fv - shF, dW = W - shW;
                        m1 += dF;
                        m2 += dW;
                        m3 += dF * dF;
                        m4 += dW * dW;
                        m5 += dF * dW;
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const float gg[3] = {dF * d[c], dW * d[c], d[c]};
#pragma unroll
                            for (int f = 0; f < 3; ++f) {
                                acc[f][c][0] += wy.x * gg[f];
                                acc[f][c][1] += wy.y * gg[f];
                                acc[f][c][2] += wy.z * gg[f];
                                acc[f][c][3] += wy.w * gg[f];
                            }
                        }
                    } else {
                        const float e = W - Fv;
                        m1 += e * e;
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const float g = e * d[c];
                            acc[0][c][0] += wy.x * g;
                            acc[0][c][1] += wy.y * g;
                            acc[0][c][2] += wy.z * g;
                            acc[0][c][3] += wy.w * g;
                        }
                    }
                }
            }
        }
        flush(kyl, 1);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc[f][c][0] = acc[f][c][1];
                acc[f][c][1] = acc[f][c][2];
                acc[f][c][2] = acc[f][c][3];
                acc[f][c][3] = 0.f;
            }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            V[c][0] = V[c][1];
            V[c][1] = V[c][2];
            V[c][2] = V[c][3];
            V[c][3] = (kyl + 4 < Wy) ? T1[(c * WyM + kyl + 4) * TX + lx] : 0.f;
        }
    }
    // the last three control rows in one pass (one wait instead of three)
    flush(Wy - 3, 3);
    double st[6] = {(double)cnt, (double)m1, (double)m2, (double)m3, (double)m4, (double)m5};
    block_sum<NT, 6>(st, red);
    if (tid == 0) {
        double* slot = reinterpret_cast<double*>(C.ws + C.L.stats) + (long long)item * kStatWords;
#pragma unroll
        for (int k = 0; k < 6; ++k) slot[k] = st[k];
        slot[6] = shF;
        slot[7] = shW;
    }
}

// --------------------------------------------------------------- finalize
// Global similarity coefficients from the tile statistics (FP64, fixed order),
// then every control gathers the partials of the tiles whose window holds it.
struct Coef {
    double S;      // similarity value
    double alpha;  // NCC: coefficient of (F - shift_F); MSE: 2 / N'
    double beta;   // NCC: coefficient of (W - shift_W)
    double muF, muW;
    bool degenerate;
};

// Per-thread parts of a pair's reduction: the tile moments (v[0..5], or
// v[0..1] for MSE) and the regulariser partials (v[6]); block_sum then adds
// them in a fixed order. The first tile and the first partial of each thread
// are loaded together, so that (with at most one of each, the usual case)
// the thread waits for memory once.
template <int NT, int SIM>
__device__ void pair_sums_local(const PairDesc& P, const double* stats, const double* regpart,
                                double (&v)[7]) {
#pragma unroll
    for (int i = 0; i < 7; ++i) v[i] = 0.0;
    auto tile = [&](const double (&s)[8]) {
        const double n = s[0];
        if (SIM == AIR_SIM_NCC) {
            const double a = s[6], b = s[7];
            v[0] += n;
            v[1] += s[1] + n * a;                                   // sum F
            v[2] += s[2] + n * b;                                   // sum W
            v[3] += s[3] + 2.0 * a * s[1] + n * a * a;              // sum F^2
            v[4] += s[4] + 2.0 * b * s[2] + n * b * b;              // sum W^2
            v[5] += s[5] + a * s[2] + b * s[1] + n * a * b;         // sum F W
        } else {
            v[0] += n;
            v[1] += s[1];
        }
    };
    auto fetch = [&](int t, double (&s)[8]) {
        const double* p = stats + (long long)(P.tile_begin + t) * kStatWords;
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = p[i];
    };
    const int t0 = threadIdx.x;
    double s0[8];
    if (t0 < P.ntiles) fetch(t0, s0);
    const double r0 = t0 < P.nreg ? regpart[P.regpart_off + t0] : 0.0;
    if (t0 < P.ntiles) tile(s0);
    for (int t = t0 + NT; t < P.ntiles; t += NT) {
        double s1[8];
        fetch(t, s1);
        tile(s1);
    }
    v[6] += r0;
    for (int i = t0 + NT; i < P.nreg; i += NT) v[6] += regpart[P.regpart_off + i];
}

// The similarity's coefficients from the pair's summed moments.
template <int SIM>
__device__ Coef coef_from_sums(const double (&v)[7]) {
    Coef k{0.0, 0.0, 0.0, 0.0, 0.0, false};
    const double N = v[0];
    if (SIM == AIR_SIM_MSE) {
        if (N < 1.0) { k.degenerate = true; return k; }
        k.S = v[1] / N;
        k.alpha = 2.0 / N;
        return k;
    }
    if (N < 2.0) { k.degenerate = true; return k; }
    const double muF = v[1] / N, muW = v[2] / N;
    const double B = v[3] - N * muF * muF;
    const double Cc = v[4] - N * muW * muW;
    const double A = v[5] - N * muF * muW;
    if (!(B > 1e-10 * v[3]) || !(Cc > 1e-10 * v[4])) { k.degenerate = true; return k; }
    const double sbc = sqrt(B * Cc);
    const double rho = A / sbc;
    k.S = -rho;
    k.alpha = -1.0 / sbc;
    k.beta = rho / Cc;
    k.muF = muF;
    k.muW = muW;
    return k;
}

// scalars[pair]: [0] S, [1] alpha, [2] beta, [3] muF, [4] muW, [5] R, [6] degenerate;
// also the pair's objective value and flags (one thread)
__device__ inline void store_pair_coef(const LaunchCtx& C, const PairDesc& P, int pair,
                                       const Coef& k, double R) {
    double* out = reinterpret_cast<double*>(C.ws + C.L.scalars) + (long long)pair * 8;
    out[0] = k.S;
    out[1] = k.alpha;
    out[2] = k.beta;
    out[3] = k.muF;
    out[4] = k.muW;
    out[5] = R;
    out[6] = k.degenerate ? 1.0 : 0.0;
    out[7] = 0.0;
    uint32_t fl = k.degenerate ? AIR_FLAG_DEGENERATE : 0u;
    const double value = k.S + (double)P.lambda * R;
    if (!isfinite((float)value)) fl |= AIR_FLAG_NONFINITE;
    if (fl) atomicOr(reinterpret_cast<uint32_t*>(C.ws + C.L.flags) + pair, fl);
    float* vout = C.values ? C.values + pair : C.value0;
    *vout = (float)value;
}

// Range of tiles (along one axis) whose voxel range meets the support of
// control j: voxels [(j - 3) sp, (j + 1) sp - 1].
__device__ inline void tile_range(int j, int sp, int n, int T, int* lo, int* hi) {
    const int a = max(0, (j - 3) * sp);
    const int b = min(n - 1, (j + 1) * sp - 1);
    *lo = a / T;
    *hi = (b >= a) ? b / T : -1;
}

// NS lanes per control (1, or 8 when the launch has few controls to fill the
// chip with): the tiles whose window holds the control are visited in a
// fixed order and slot s goes to lane s mod NS; the lanes' FP64 sums meet in
// a fixed xor butterfly, so every lane holds the same, order-fixed total.
constexpr int kFinLanes = 8;
// tiles whose loads a lane issues together when a control has several lanes
// (few controls, so memory latency is the cost); with one lane per control
// the launch has threads enough to hide it, and registers matter more
constexpr int kFinBatch = 4;
constexpr long long kFinFewControls = 1 << 17;   // below this many, NS = kFinLanes

// SP: the spacing of every axis when the launch's plans share it at compile
// time (8, the spacing-8 kernel's plans), else 0 (read from the pair)
template <int TX, int TY, int SIM, int DIM, int NS, int SP>
__global__ void __launch_bounds__(kBlock)
k_finalize(const LaunchCtx C) {
    constexpr int NT = kBlock;
    constexpr int CPB = NT / NS;   // controls per block
    constexpr int NF = (SIM == AIR_SIM_NCC) ? 3 : 1;
    const int pair = blockIdx.y;
    const PairDesc P = C.pairs[pair];
    const double* stats = reinterpret_cast<const double*>(C.ws + C.L.stats);
    __shared__ double red[8 * (kBlock / 64)];
    uint32_t* flags = reinterpret_cast<uint32_t*>(C.ws + C.L.flags) + pair;
    const int nctrl = P.nc[0] * P.nc[1] * (DIM == 3 ? P.nc[2] : 1);
    const int ls = threadIdx.x % NS;
    const int j = blockIdx.x * CPB + threadIdx.x / NS;
    const bool live = j < nctrl;
    const float* part = reinterpret_cast<const float*>(C.ws + C.L.part) + P.part_off;
    const float* rg = reinterpret_cast<const float*>(C.ws + C.L.reggrad) + P.param_off;
    float* grad = C.grad_tab ? C.grad_tab[pair] : C.grad0;
    const int WxM = P.win[0], WyM = (DIM == 3) ? P.win[1] : 1;
    // this lane's tiles are taken NB at a time: their addresses first, then
    // every load of the batch (all addresses valid: unused entries point at
    // the pair's first partial), then the sums in slot order, so each batch
    // waits for memory once
    constexpr int NB = NS > 1 ? kFinBatch : 1;
    const double* stb[NB];
    const float* qb[NB];
    double s6[NB], s7[NB];
    float qv[NB][NF * DIM];
    int nb = 0;
    const double* st0 = stats + (long long)P.tile_begin * kStatWords;
    auto reset = [&]() {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            stb[i] = st0;
            qb[i] = part;
        }
        nb = 0;
    };
    auto load = [&]() {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (SIM == AIR_SIM_NCC) {
                s6[i] = stb[i][6];
                s7[i] = stb[i][7];
            }
#pragma unroll
            for (int e = 0; e < NF * DIM; ++e) qv[i][e] = qb[i][e];
        }
    };
    double g[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) g[c] = 0.0;
    auto add = [&](const Coef& k, int n) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (i >= n) break;
            const double cF = k.alpha, cW = k.beta;
            double c1 = 0.0;
            if (SIM == AIR_SIM_NCC) c1 = k.alpha * (s6[i] - k.muF) + k.beta * (s7[i] - k.muW);
            const float* q = qv[i];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                if (SIM == AIR_SIM_NCC)
                    g[c] += cF * q[c] + cW * q[DIM + c] + c1 * q[2 * DIM + c];
                else
                    g[c] += cF * q[c];
            }
        }
    };
    // Walk this lane's tiles in slot order, calling visit(stats, partial) for
    // each. The tiles of tile_range are exactly those whose control window
    // holds the control, so its local indices lie inside each window. A
    // tile's window starts at control floor(t T / sp) along x (and y). With
    // several lanes per control (few controls, latency-bound) the origins are
    // stepped from the first tile with a running remainder, one division per
    // axis; with one lane per control, registers matter more and each origin
    // is one division.
    auto walk = [&](auto&& visit) {
        const int jx = j % P.nc[0];
        const int jy = (j / P.nc[0]) % P.nc[1];
        const int jz = (DIM == 3) ? j / (P.nc[0] * P.nc[1]) : 0;
        // column axis: z in 3D, y in 2D
        const int colax = DIM - 1;
        const int jc = (DIM == 3) ? jz : jy;
        AIR_CHECK(SP == 0 || (P.sp[0] == SP && P.sp[1] == SP && P.sp[colax] == SP),
                  kDbgControlLoad);
        const int ncell = (P.n[colax] - 1) / (SP ? SP : P.sp[colax]) + 1;
        const int tc_lo = max(0, jc - 3) / P.col_cells;
        const int tc_hi = min(ncell - 1, jc) / P.col_cells;
        int tx_lo, tx_hi, ty_lo = 0, ty_hi = 0;
        tile_range(jx, SP ? SP : P.sp[0], P.n[0], TX, &tx_lo, &tx_hi);
        if (DIM == 3) tile_range(jy, SP ? SP : P.sp[1], P.n[1], TY, &ty_lo, &ty_hi);
        constexpr bool kStep = NS > 1;
        const int spx = SP ? SP : P.sp[0];
        const int qx = TX / spx, rx = TX - qx * spx;
        const int cxs = (tx_lo * TX) / spx, rxs = tx_lo * TX - cxs * spx;
        int spy = 1, qy = 0, ry = 0, cys = 0, rys = 0;
        if (DIM == 3) {
            spy = SP ? SP : P.sp[1];
            qy = TY / spy;
            ry = TY - qy * spy;
            cys = (ty_lo * TY) / spy;
            rys = ty_lo * TY - cys * spy;
        }
        int slot = 0;
        for (int tc = tc_lo; tc <= tc_hi; ++tc) {
            const int kcl = jc - tc * P.col_cells;
            AIR_CHECK(kcl >= 0 && kcl < min(P.col_cells, ncell - tc * P.col_cells) + 3,
                      kDbgControlLoad);
            int cy0 = cys, ryr = rys;
            for (int ty = ty_lo; ty <= ty_hi; ++ty) {
                int cx0 = cxs, rxr = rxs;
                for (int tx = tx_lo; tx <= tx_hi; ++tx) {
                    if ((slot++ & (NS - 1)) == ls) {
                        if (!kStep) {
                            cx0 = (tx * TX) / spx;
                            if (DIM == 3) cy0 = (ty * TY) / spy;
                        }
                        const int kyl = (DIM == 3) ? jy - cy0 : 0;
                        const int kxl = jx - cx0;
#ifdef AIR_DEBUG_BOUNDS
                        {
                            int c0, w;
                            ctrl_window(tx * TX, min(tx * TX + TX, P.n[0]), spx, &c0, &w);
                            AIR_CHECK(c0 == cx0 && kxl >= 0 && kxl < w, kDbgControlLoad);
                            if (DIM == 3) {
                                ctrl_window(ty * TY, min(ty * TY + TY, P.n[1]), spy, &c0, &w);
                                AIR_CHECK(c0 == cy0 && kyl >= 0 && kyl < w, kDbgControlLoad);
                            }
                        }
#endif
                        const int tl = (DIM == 3) ? (tc * P.ntile[1] + ty) * P.ntile[0] + tx
                                                  : tc * P.ntile[0] + tx;
                        const float* pt = part + (long long)tl * P.part_stride;
                        // partial layout [column][y][x][field * DIM + component]
                        visit(stats + (long long)(P.tile_begin + tl) * kStatWords,
                              pt + (((long long)kcl * WyM + kyl) * WxM + kxl) * (NF * DIM));
                    }
                    if (kStep) {
                        cx0 += qx;
                        rxr += rx;
                        if (rxr >= spx) {
                            rxr -= spx;
                            ++cx0;
                        }
                    }
                }
                if (kStep) {
                    cy0 += qy;
                    ryr += ry;
                    if (ryr >= spy) {
                        ryr -= spy;
                        ++cy0;
                    }
                }
            }
        }
    };
    // With several lanes per control (few controls, latency-bound) the
    // lane's first batch is loaded before the pair's reduction, so that both
    // wait for memory together, and a lane with more than NB tiles walks them
    // again for the rest. With one lane per control the walk runs once, after
    // the reduction (a second walk would repeat the control's index
    // arithmetic, and the launch has waves enough to hide the wait).
    constexpr bool kEarly = NS > 1;
    reset();
    int mine = 0;
    if (kEarly) {
        if (live)
            walk([&](const double* sp, const float* qp) {
                if (mine < NB) {
                    stb[mine] = sp;
                    qb[mine] = qp;
                }
                ++mine;
            });
        load();
    }
    // every block reduces the pair's tile statistics itself, in the same
    // fixed order, so every block holds the same coefficients; block 0
    // stores them with the pair's value (no separate launch)
    double v[7];
    pair_sums_local<kBlock, SIM>(P, stats, reinterpret_cast<const double*>(C.ws + C.L.regpart),
                                 v);
    block_sum<kBlock, 7>(v, red);
    const Coef k = coef_from_sums<SIM>(v);
    const double R = v[6] * (double)P.inv_xr;
    if (blockIdx.x == 0 && threadIdx.x == 0) store_pair_coef(C, P, pair, k, R);
    if (live && !k.degenerate) {
        int skip = 0;
        if (kEarly) {
            add(k, min(mine, NB));
            skip = NB;
        }
        if (!kEarly || mine > NB) {
            reset();
            int seen = 0;
            walk([&](const double* sp, const float* qp) {
                if (seen++ < skip) return;
                stb[nb] = sp;
                qb[nb] = qp;
                if (++nb == NB) {
                    load();
                    add(k, NB);
                    reset();
                }
            });
            load();
            add(k, nb);
        }
    }
    static_assert((NS & (NS - 1)) == 0 && NS <= 64, "NS: a power of two within a wave");
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int o = NS / 2; o >= 1; o >>= 1) g[c] += __shfl_xor(g[c], o, NS);
    if (!live || ls != 0) return;
    uint32_t bad = 0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const float out = (float)(g[c] * (double)P.s[c]) + rg[(long long)c * nctrl + j];
        grad[(long long)c * nctrl + j] = out;
        if (!isfinite(out)) bad = 1;
    }
    if (bad) atomicOr(flags, AIR_FLAG_NONFINITE);
}

// --------------------------------------------------------------- launchers
template <int TX, int TY, int SIM>
static hipError_t launch3(const LaunchCtx& C, size_t lds, hipStream_t s) {
    const int nblk = xcd_grid(C.ntiles_total, C.nreg_total);
    hipLaunchKernelGGL((k_fused3<TX, TY, SIM>), dim3(nblk), dim3(TX * TY), lds, s, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipSuccess;
}

template <int TX, int TY, int SIM>
static hipError_t launch3s8(const LaunchCtx& C, size_t lds, hipStream_t s) {
    const int nblk = xcd_grid(C.ntiles_total, C.nreg_total);
    hipLaunchKernelGGL((k_fused3_s8<TX, TY, SIM>), dim3(nblk), dim3(TX * TY), lds, s, C);
    return hipGetLastError();
}

template <int TX, int TY, int SIM, int DIM, int SP = 0>
static hipError_t launch_fin(const LaunchCtx& C, int max_ctrl, hipStream_t s) {
    if ((long long)max_ctrl * C.npairs < kFinFewControls) {
        dim3 grid(cdiv(max_ctrl, kBlock / kFinLanes), C.npairs);
        hipLaunchKernelGGL((k_finalize<TX, TY, SIM, DIM, kFinLanes, SP>), grid, dim3(kBlock), 0, s, C);
    } else {
        dim3 grid(cdiv(max_ctrl, kBlock), C.npairs);
        hipLaunchKernelGGL((k_finalize<TX, TY, SIM, DIM, 1, SP>), grid, dim3(kBlock), 0, s, C);
    }
    return hipGetLastError();
}

// cfg: in 3D the tile configuration (id -> TX, TY); in 2D 8 when every pair
// has spacing 8, else 0. Column cells come from the plan.
hipError_t launch_bspline(const LaunchCtx& C, int cfg, size_t lds, int max_ctrl,
                          hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e = hipSuccess;
    if (ev0) (void)hipEventRecord(ev0, s);
    if (C.dim == 3) {
        const bool ncc = C.sim == AIR_SIM_NCC;
        switch (cfg) {
            case 0: e = ncc ? launch3<32, 8, 1>(C, lds, s) : launch3<32, 8, 0>(C, lds, s); break;
            case 1: e = ncc ? launch3<64, 4, 1>(C, lds, s) : launch3<64, 4, 0>(C, lds, s); break;
            case 2: e = ncc ? launch3<16, 16, 1>(C, lds, s) : launch3<16, 16, 0>(C, lds, s); break;
            case 3: e = ncc ? launch3s8<32, 8, 1>(C, lds, s) : launch3s8<32, 8, 0>(C, lds, s); break;
            case 4: e = ncc ? launch3s8<16, 16, 1>(C, lds, s) : launch3s8<16, 16, 0>(C, lds, s); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
        if (ev1) (void)hipEventRecord(ev1, s);
        switch (cfg) {
            case 0: return ncc ? launch_fin<32, 8, 1, 3>(C, max_ctrl, s) : launch_fin<32, 8, 0, 3>(C, max_ctrl, s);
            case 1: return ncc ? launch_fin<64, 4, 1, 3>(C, max_ctrl, s) : launch_fin<64, 4, 0, 3>(C, max_ctrl, s);
            case 2: return ncc ? launch_fin<16, 16, 1, 3>(C, max_ctrl, s) : launch_fin<16, 16, 0, 3>(C, max_ctrl, s);
            // the spacing-8 kernel's plans: spacing 8 on every axis
            case 3: return ncc ? launch_fin<32, 8, 1, 3, 8>(C, max_ctrl, s) : launch_fin<32, 8, 0, 3, 8>(C, max_ctrl, s);
            default: return ncc ? launch_fin<16, 16, 1, 3, 8>(C, max_ctrl, s) : launch_fin<16, 16, 0, 3, 8>(C, max_ctrl, s);
        }
    }
    const int nblk = xcd_grid(C.ntiles_total, C.nreg_total);
    if (C.sim == AIR_SIM_NCC)
        hipLaunchKernelGGL((k_fused2<64, 1>), dim3(nblk), dim3(64), lds, s, C);
    else
        hipLaunchKernelGGL((k_fused2<64, 0>), dim3(nblk), dim3(64), lds, s, C);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) (void)hipEventRecord(ev1, s);
    if (cfg == 8)   // every pair has spacing 8
        return C.sim == AIR_SIM_NCC ? launch_fin<64, 1, 1, 2, 8>(C, max_ctrl, s)
                                    : launch_fin<64, 1, 0, 2, 8>(C, max_ctrl, s);
    return C.sim == AIR_SIM_NCC ? launch_fin<64, 1, 1, 2>(C, max_ctrl, s)
                                : launch_fin<64, 1, 0, 2>(C, max_ctrl, s);
}

// Regulariser only (B-spline): Gram-form blocks of one pair, unscaled output.
template <int NT>
__global__ void __launch_bounds__(NT)
k_reg_only(const PairDesc* pairs, int pair, const float* consts, const float* theta,
           float* grad_out, double* regpart, int dim) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);
    float* lds = reinterpret_cast<float*>(smem_raw + 8 * sizeof(double) * (NT / 64));
    const PairDesc P = pairs[pair];
    reg_block<NT>(P, consts, theta, grad_out, 2.0f * P.inv_xr, regpart, blockIdx.x, dim,
                  lds, red);
}

__global__ void k_reg_value(const PairDesc* pairs, int pair, const double* regpart,
                            float* value) {
    __shared__ double red[8 * (kBlock / 64)];
    const PairDesc P = pairs[pair];
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < P.nreg; i += kBlock) v[0] += regpart[i];
    block_sum<kBlock, 1>(v, red);
    if (threadIdx.x == 0) *value = (float)(v[0] * (double)P.inv_xr);
}

hipError_t launch_reg_bspline(const PairDesc* dpairs, const PairDesc& hp, int pair,
                              const float* consts, const float* theta, float* grad_out,
                              double* regpart, float* value, int dim, size_t lds,
                              hipStream_t s) {
    hipLaunchKernelGGL((k_reg_only<kBlock>), dim3(hp.nreg), dim3(kBlock), lds, s, dpairs, pair,
                       consts, theta, grad_out, regpart, dim);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reg_value, dim3(1), dim3(kBlock), 0, s, dpairs, pair, regpart, value);
    return hipGetLastError();
}

}  // namespace air

// this unit's bounds-check flags (debug build only)
AIR_DEBUG_UNIT(bspline)
