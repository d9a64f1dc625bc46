// Diffeomorphic transform (Sec. III-D): f = exp(v) for a stationary velocity
// field v, by scaling and squaring. u_0 = v / 2^K, then K squarings
//     u_{k+1}(x) = u_k(x) + u_k(x + u_k(x)),
// the second term sampled like an image (sample point p_a = x_a +
// u_a (n_a - 1)/2, linear on [floor(p), floor(p) + 1], zero outside the
// volume, no mask). For a B-spline model v is the expanded control field.
// The exponential cannot stay inside one fused pass (each squaring samples
// the whole previous field), so the fields u_0 .. u_K live in the workspace;
// the objective at u_K runs on the dense-field kernels, and its gradient goes
// back through the squarings. Each adjoint step is owner-computes: a block
// owns a tile of target voxels, adds into LDS the transposed-interpolation
// contributions of every source voxel whose sample point can reach the tile
// (the reach is bounded by the field's largest displacement, measured once
// per field), then adds the identity and sample-point terms and writes each
// target once. The LDS additions are integer (fixed point), so their order,
// which varies from run to run, does not change the result.
#include "device_common.h"

namespace air {

namespace {

constexpr int kDiffeoBlocks = 8192;  // grid-stride launches

__host__ inline int grid_for(long long total) {
    const long long b = (total + kBlock - 1) / kBlock;
    return (int)(b < kDiffeoBlocks ? (b < 1 ? 1 : b) : kDiffeoBlocks);
}

// Zero-padded multilinear sample of the DIM components of field u at the
// point x + d + e of a voxel (voxel units, see axis_cell); with DERIV also
// dval[c][a] = d sample_c / d p_a on that point's cell (right-sided at an
// integer point). Returns false for a non-finite point (the values are then
// NaN). The value does not depend on the cell taken at an integer point, so
// the forward squaring passes e = 0.
template <int DIM, bool DERIV>
__device__ inline bool field_sample(const float* __restrict__ u, long long N, const PairDesc& P,
                                    const int* x, const Disp* q, float* val, float (*dval)[3],
                                    int* j, float* f) {
    bool finite = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float d = q[a].d;
        if (!(d == d) || d == INFINITY || d == -INFINITY) finite = false;
        const AxisCell c = axis_cell(x[a], q[a], P.n[a]);
        j[a] = c.t;
        f[a] = c.f;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        val[c] = 0.f;
        if (DERIV)
#pragma unroll
            for (int a = 0; a < DIM; ++a) dval[c][a] = 0.f;
    }
    if (!finite) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            val[c] = NAN;
            if (DERIV)
#pragma unroll
                for (int a = 0; a < DIM; ++a) dval[c][a] = NAN;
        }
        return false;
    }
    // every corner inside the volume (the common case): each x-pair of
    // corners is one 8-byte buffer load, and the weights are nested lerps
    bool interior = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        if (j[a] < 0 || j[a] > P.n[a] - 2) interior = false;
    if (interior) {
        const int nx = P.n[0], ny = P.n[1];
        const int off = ((DIM == 3 ? j[2] * ny : 0) + j[1]) * nx * 4 + j[0] * 4;  // N * 4 < 2^31
        const int sx4 = nx * 4, sxy4 = nx * ny * 4;
        AIR_CHECK(off >= 0 && (long long)off + (DIM == 3 ? sxy4 : 0) + sx4 + 8 <= N * 4,
                  kDbgCompose);
        const float fx = f[0], fy = f[1], fz = DIM == 3 ? f[2] : 0.f;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const __amdgpu_buffer_rsrc_t r = make_rsrc(u + c * N, (uint32_t)(N * 4));
            const v2f a00 = load2(r, off, 0), a10 = load2(r, off, sx4);
            const float c00 = fmaf(fx, a00.y - a00.x, a00.x), c10 = fmaf(fx, a10.y - a10.x, a10.x);
            const float c0 = fmaf(fy, c10 - c00, c00);
            if (DIM == 2) {
                val[c] = c0;
                if (DERIV) {
                    dval[c][0] = (1.f - fy) * (a00.y - a00.x) + fy * (a10.y - a10.x);
                    dval[c][1] = c10 - c00;
                }
            } else {
                const v2f a01 = load2(r, off, sxy4), a11 = load2(r, off, sxy4 + sx4);
                const float c01 = fmaf(fx, a01.y - a01.x, a01.x),
                            c11 = fmaf(fx, a11.y - a11.x, a11.x);
                const float c1 = fmaf(fy, c11 - c01, c01);
                val[c] = fmaf(fz, c1 - c0, c0);
                if (DERIV) {
                    const float dx0 = fmaf(fy, (a10.y - a10.x) - (a00.y - a00.x), a00.y - a00.x);
                    const float dx1 = fmaf(fy, (a11.y - a11.x) - (a01.y - a01.x), a01.y - a01.x);
                    dval[c][0] = fmaf(fz, dx1 - dx0, dx0);
                    dval[c][1] = fmaf(fz, (c11 - c01) - (c10 - c00), c10 - c00);
                    dval[c][2] = c1 - c0;
                }
            }
        }
        return true;
    }
#pragma unroll
    for (int cn = 0; cn < (1 << DIM); ++cn) {
        int q[3] = {0, 0, 0};
        bool in = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            q[a] = j[a] + ((cn >> a) & 1);
            if (!interior && (q[a] < 0 || q[a] > P.n[a] - 1)) in = false;
        }
        if (!in) continue;
        const long long idx = q[0] + (long long)P.n[0] * (q[1] + (DIM == 3 ? (long long)P.n[1] * q[2] : 0));
        float w = 1.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) w *= ((cn >> a) & 1) ? f[a] : 1.f - f[a];
        float wa[3];
        if (DERIV) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                float t = ((cn >> a) & 1) ? 1.f : -1.f;
#pragma unroll
                for (int b = 0; b < DIM; ++b)
                    if (b != a) t *= ((cn >> b) & 1) ? f[b] : 1.f - f[b];
                wa[a] = t;
            }
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float uv = u[c * N + idx];
            val[c] += w * uv;
            if (DERIV)
#pragma unroll
                for (int a = 0; a < DIM; ++a) dval[c][a] += wa[a] * uv;
        }
    }
    return true;
}

template <int DIM>
__device__ inline void voxel_coords(const PairDesc& P, long long v, int* idx) {
    idx[0] = (int)(v % P.n[0]);
    idx[1] = (int)((v / P.n[0]) % P.n[1]);
    idx[2] = DIM == 3 ? (int)(v / ((long long)P.n[0] * P.n[1])) : 0;
}

// u = scale * B theta (direct sum over the 4^d supporting controls).
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_bs_field(const PairDesc P, const float* __restrict__ consts, const float* __restrict__ th,
           float scale, float* __restrict__ out) {
    const long long N = P.nvox;
    const long long NC = (long long)P.nc[0] * P.nc[1] * P.nc[2];
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < N;
         v += (long long)gridDim.x * kBlock) {
        int idx[3];
        voxel_coords<DIM>(P, v, idx);
        int i0[3];
        const float* w[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            i0[a] = idx[a] / P.sp[a];
            w[a] = consts + P.wtab_off[a] + (idx[a] - i0[a] * P.sp[a]) * 4;
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            float acc = 0.f;
            for (int kz = 0; kz < (DIM == 3 ? 4 : 1); ++kz) {
                const float wz = DIM == 3 ? w[2][kz] : 1.f;
                const int jz = DIM == 3 ? i0[2] + kz : 0;
                for (int ky = 0; ky < 4; ++ky) {
                    const float* row = th + c * NC + ((long long)jz * P.nc[1] + i0[1] + ky) * P.nc[0] + i0[0];
                    const float wyz = wz * w[1][ky];
                    acc += wyz * (w[0][0] * row[0] + w[0][1] * row[1] + w[0][2] * row[2] +
                                  w[0][3] * row[3]);
                }
            }
            out[c * N + v] = scale * acc;
        }
    }
}

__global__ void __launch_bounds__(kBlock)
k_scale_copy(const float* __restrict__ in, float scale, long long n, int accumulate,
             float* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        out[i] = accumulate ? out[i] + scale * in[i] : scale * in[i];
}

// One squaring: out(x) = u(x) + u(x + u(x)). It also measures the largest
// displacement of its input u in voxels (max over voxels and axes of
// |u_a| (n_a - 1)/2) into dmax, as the bits of a non-negative float (ordered
// like unsigned integers; NaN compares above every finite value): the reach
// of this squaring's adjoint. dmax must be zero before the launch.
// A block owns kCompTX x kCompTY voxels of (x, y) and takes kCompSteps steps
// along the last axis (3D: planes z; 2D: groups of kCompTY rows), so the
// coordinates need no division and the next step's displacement loads are
// issued before this step's gathers are used. Work items are XCD-contiguous,
// so the gathers of neighbouring columns share an L2.
constexpr int kCompTX = 64, kCompTY = 4, kCompSteps = 16;
static_assert(kCompTX * kCompTY == kBlock, "one thread per (x, y) of a block");
template <int DIM>
__host__ __device__ inline int compose_items(const PairDesc& P) {
    const int nbx = cdiv(P.n[0], kCompTX);
    if (DIM == 3) return nbx * cdiv(P.n[1], kCompTY) * cdiv(P.n[2], kCompSteps);
    return nbx * cdiv(P.n[1], kCompTY * kCompSteps);
}
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_compose(const PairDesc P, const float* __restrict__ u, float* __restrict__ out,
          unsigned int* __restrict__ dmax) {
    __shared__ unsigned int red[kBlock / 64];
    const long long N = P.nvox;
    const int nx = P.n[0], ny = P.n[1];
    const int nbx = cdiv(nx, kCompTX);
    const int item = xcd_item(blockIdx.x, compose_items<DIM>(P), 0);
    float m = 0.f;
    if (item >= 0) {
        const int x = (item % nbx) * kCompTX + (int)threadIdx.x % kCompTX;
        const int ly = (int)threadIdx.x / kCompTX;
        int y, z0, cnt;
        long long step;
        if (DIM == 3) {
            const int nby = cdiv(ny, kCompTY);
            y = ((item / nbx) % nby) * kCompTY + ly;
            z0 = (item / (nbx * nby)) * kCompSteps;
            cnt = min(kCompSteps, P.n[2] - z0);
            step = (long long)nx * ny;
        } else {
            y = (item / nbx) * (kCompTY * kCompSteps) + ly;   // rows y + kCompTY k
            z0 = 0;
            cnt = y < ny ? min(kCompSteps, cdiv(ny - y, kCompTY)) : 0;
            step = (long long)nx * kCompTY;
        }
        if (x < nx && y < ny && cnt > 0) {
            long long v = x + (long long)nx * (y + (DIM == 3 ? (long long)ny * z0 : 0));
            float uc[3] = {0.f, 0.f, 0.f}, un[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < DIM; ++c) uc[c] = u[c * N + v];
            for (int k = 0; k < cnt; ++k) {
                if (k + 1 < cnt) {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) un[c] = u[c * N + v + step];
                }
                const int idx[3] = {x, DIM == 3 ? y : y + kCompTY * k, DIM == 3 ? z0 + k : 0};
                float val[3], f[3];
                Disp q[3];
                int j[3];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    q[a] = Disp{uc[a] * P.s[a], 0.f};
                    const float t = fabsf(q[a].d);
                    m = (t > m || !(t == t)) ? t : m;
                }
                field_sample<DIM, false>(u, N, P, idx, q, val, nullptr, j, f);
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    out[c * N + v] = uc[c] + val[c];
                    uc[c] = un[c];
                }
                v += step;
            }
        }
    }
    unsigned int b = __float_as_uint(m) & 0x7fffffffu;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b = max(b, (unsigned int)__shfl_xor((int)b, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int r = red[0];
        for (int w = 1; w < kBlock / 64; ++w) r = max(r, red[w]);
        atomicMax(dmax, r);
    }
}

// Largest |g| over n values, as non-negative float bits (NaN above every
// finite value); `out` must be zero before the launch.
__global__ void __launch_bounds__(kBlock)
k_absmax_plain(const float* __restrict__ g, long long n, unsigned int* out) {
    __shared__ unsigned int red[kBlock / 64];
    float m = 0.f;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const float t = fabsf(g[i]);
        m = (t > m || !(t == t)) ? t : m;
    }
    unsigned int b = __float_as_uint(m) & 0x7fffffffu;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b = max(b, (unsigned int)__shfl_xor((int)b, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int r = red[0];
        for (int w = 1; w < kBlock / 64; ++w) r = max(r, red[w]);
        atomicMax(out, r);
    }
}

__global__ void k_zero_u32(unsigned int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Owner-computes adjoint of one squaring. The block owns target tile T (TS
// voxels per axis); every source voxel x within `reach` of T computes its
// sample point and adds w_q(p(x)) gout(x) into LDS for its corners q inside T;
// then each target q gets gin(q) = gout(q) + s_a sum_c gout_c(q) du_c/dp_a
// at p(q) + the accumulated transpose.
// The transpose accumulates in 64-bit fixed point, scaled by the power of two
// 2^(31 - e) with 2^e > max |gout| (gmax_bits): integer LDS atomics are much
// faster than float ones here, and integer sums do not depend on their order,
// so the result is bitwise repeatable. Each term is below 2^31 in magnitude,
// so it converts with one 32-bit conversion (truncation: an error below
// 2^-30 max|gout| per term) and fewer than 2^32 terms per target cannot
// overflow. A non-finite max|gout| makes gin NaN.
constexpr int kAdjBlock3 = 1024;   // threads per 3D tile (96 KB of accumulators)
template <int DIM>
__global__ void __launch_bounds__(DIM == 3 ? kAdjBlock3 : kBlock)
k_compose_adj_tile(const PairDesc P, const float* __restrict__ u, const float* __restrict__ gout,
                   const unsigned int* __restrict__ dmax_bits,
                   const unsigned int* __restrict__ gmax_bits, float* __restrict__ gin,
                   unsigned int* __restrict__ gmax_out) {
    constexpr int TS = DIM == 3 ? 16 : 64;  // 4096 targets per tile
    constexpr int TV = DIM == 3 ? TS * TS * TS : TS * TS;
    constexpr int NT = DIM == 3 ? kAdjBlock3 : kBlock;
    __shared__ unsigned long long acc[DIM][TV];
    const long long N = P.nvox;
    const int nt0 = cdiv(P.n[0], TS), nt1 = cdiv(P.n[1], TS);
    const int b = blockIdx.x;
    int o[3] = {(b % nt0) * TS, ((b / nt0) % nt1) * TS, DIM == 3 ? (b / (nt0 * nt1)) * TS : 0};
    for (int i = threadIdx.x; i < DIM * TV; i += NT) (&acc[0][0])[i] = 0ull;
    const float gm = __uint_as_float(*gmax_bits);
    const bool gfin = gm == gm && gm < 3.0e38f;
    const int ge = gfin && gm > 0.f ? ilogbf(gm) + 1 : 0;   // 2^ge > max|gout|
    const float scale = gfin ? ldexpf(1.f, 31 - ge) : 0.f;
    const double unscale = ldexp(1.0, ge - 31);
    const float poison = gfin ? 0.f : __uint_as_float(0x7fc00000u);   // NaN
    // reach: a source x feeds the corners t and t + 1 of its cell,
    // t = x + floor(d) with |d| <= dmax < e (e = dmax plus a safety margin
    // for the rounding of dmax). A corner in [o, o + TS) needs
    // o - 1 <= t < o + TS, so the sources lie in
    // [o - 1 - floor(e), o + TS + ceil(e)) along each axis.
    const float dm = __uint_as_float(*dmax_bits);
    int hlo = 1 << 20, hhi = 1 << 20;
    if (dm == dm && dm < 1e6f) {
        const int nmax = max(P.n[0], max(P.n[1], P.n[2]));
        const double e = (double)dm + ((double)dm + nmax) * 0x1p-20;
        hlo = 1 + (int)floor(e);
        hhi = (int)ceil(e);
    }
    int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lo[a] = max(0, o[a] - hlo);
        const int hi = min(P.n[a], o[a] + TS + hhi);
        ext[a] = hi - lo[a];
    }
    __syncthreads();
    // One source voxel x (linear index v, displacement uv): its sample
    // point, and if its cell reaches the tile, its corner terms.
    auto source = [&](const int* x, long long v, const float* uv) {
        float f[3];
        int j[3];
        bool finite = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            // the transposed weights (1 - f, f) of the cell below an integer
            // point equal those of the cell above it, so e is not needed here
            const float d0 = uv[a] * P.s[a];
            if (!(d0 == d0) || d0 == INFINITY || d0 == -INFINITY) finite = false;
            const float d = fminf(fmaxf(d0, -1e9f), 1e9f);
            const float fl = floorf(d);
            j[a] = x[a] + (int)fl;
            f[a] = d - fl;
        }
        if (!finite) return;
        // corner bit b on axis a is q_a = j_a + b; it receives a term when
        // it lies in the tile and in the volume (q_a >= o_a >= 0 already)
        bool ok[3][2];
        float wa[3][2];
        int r[3] = {0, 0, 0};
        bool near = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            r[a] = j[a] - o[a];
            ok[a][0] = (unsigned)r[a] < (unsigned)TS && j[a] <= P.n[a] - 1;
            ok[a][1] = (unsigned)(r[a] + 1) < (unsigned)TS && j[a] + 1 <= P.n[a] - 1;
            near = near && (ok[a][0] || ok[a][1]);
            wa[a][0] = 1.f - f[a];
            wa[a][1] = f[a];
        }
        // skip sources whose cell misses the tile
        if (!near) return;
        // |gs| < 2^31 and a corner weight is at most 1
        float gs[3];
#pragma unroll
        for (int c = 0; c < DIM; ++c) gs[c] = gout[c * N + v] * scale;
        // tile index of corner 0 (possibly outside the tile; only corners
        // that pass the checks are used)
        const int t0 = r[0] + TS * (r[1] + (DIM == 3 ? TS * r[2] : 0));
#pragma unroll
        for (int cn = 0; cn < (1 << DIM); ++cn) {
            const int b0 = cn & 1, b1 = (cn >> 1) & 1, b2 = (cn >> 2) & 1;
            if (!(ok[0][b0] && ok[1][b1] && (DIM < 3 || ok[2][b2]))) continue;
            const float w = wa[0][b0] * wa[1][b1] * (DIM == 3 ? wa[2][b2] : 1.f);
            const int t = t0 + b0 + TS * b1 + (DIM == 3 ? TS * TS * b2 : 0);
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                atomicAdd(&acc[c][t], (unsigned long long)(long long)(int)(w * gs[c]));
        }
    };
    // Scan of the box: a work item is one column of the box (all axes but
    // the last) and a segment of ZS voxels along the last axis; the ZS
    // displacement loads are all issued before the first is used. (The box
    // holds at most N < 2^29 voxels: 32-bit index arithmetic.)
    constexpr int ZS = 4;
    constexpr int LA = DIM - 1;
    const int ncol = DIM == 3 ? ext[0] * ext[1] : ext[0];
    const int nseg = cdiv(ext[LA], ZS);
    const long long stepv = DIM == 3 ? (long long)P.n[0] * P.n[1] : (long long)P.n[0];
    for (int it = threadIdx.x; it < ncol * nseg; it += NT) {
        const int col = it % ncol, seg = it / ncol;
        int xb[3];
        xb[0] = lo[0] + col % ext[0];
        xb[1] = DIM == 3 ? lo[1] + col / ext[0] : lo[1] + seg * ZS;
        xb[2] = DIM == 3 ? lo[2] + seg * ZS : 0;
        const int zb = xb[LA], nz_ = min(ZS, lo[LA] + ext[LA] - zb);
        const long long vb =
            xb[0] + (long long)P.n[0] * (xb[1] + (DIM == 3 ? (long long)P.n[1] * xb[2] : 0));
        float uu[ZS][3];
#pragma unroll
        for (int k = 0; k < ZS; ++k) {
            const long long v = vb + (long long)min(k, nz_ - 1) * stepv;   // in the box
#pragma unroll
            for (int a = 0; a < DIM; ++a) uu[k][a] = u[a * N + v];
        }
#pragma unroll
        for (int k = 0; k < ZS; ++k) {
            if (k >= nz_) break;
            int x[3] = {xb[0], xb[1], xb[2]};
            x[LA] = zb + k;
            source(x, vb + k * stepv, uu[k]);
        }
    }
    __syncthreads();
    float gm_out = 0.f;
    for (int t = threadIdx.x; t < TV; t += NT) {
        int x[3];
        x[0] = o[0] + t % TS;
        x[1] = o[1] + (t / TS) % TS;
        x[2] = DIM == 3 ? o[2] + t / (TS * TS) : 0;
        if (x[0] >= P.n[0] || x[1] >= P.n[1] || (DIM == 3 && x[2] >= P.n[2])) continue;
        const long long v = x[0] + (long long)P.n[0] * (x[1] + (DIM == 3 ? (long long)P.n[1] * x[2] : 0));
        float val[3], f[3], dv[3][3];
        Disp q[3];
        int j[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) q[a] = disp_of(u[a * N + v], P.s[a]);
        field_sample<DIM, true>(u, N, P, x, q, val, dv, j, f);
        float go[3];
#pragma unroll
        for (int c = 0; c < DIM; ++c) go[c] = gout[c * N + v];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            float tsum = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) tsum += go[c] * dv[c][a];
            const float tr = (float)((double)(long long)acc[a][t] * unscale) + poison;
            const float gv = go[a] + P.s[a] * tsum + tr;
            gin[a * N + v] = gv;
            const float ag = fabsf(gv);
            gm_out = (ag > gm_out || !(ag == ag)) ? ag : gm_out;
        }
    }
    // max |gin| of the block (the scale of the next squaring's adjoint)
    __shared__ unsigned int redm[NT / 64];
    unsigned int bm = __float_as_uint(gm_out) & 0x7fffffffu;
#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) bm = max(bm, (unsigned int)__shfl_xor((int)bm, o2, 64));
    if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = bm;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int r = redm[0];
        for (int w = 1; w < NT / 64; ++w) r = max(r, redm[w]);
        atomicMax(gmax_out, r);
    }
}

// Transposed B-spline expansion, one axis at a time. Input [d][A][L][B]
// (L the axis being contracted, length n), output [d][A][nc][B]: out[.][j][.]
// = sum over voxels x of control j's support of w(x, j) in[.][x][.], where
// voxel x in cell i = x / sp with offset r carries weight table[r][j - i].
__global__ void __launch_bounds__(kBlock)
k_bs_adjoint_axis(const float* __restrict__ in, int d, long long A, int n, long long B, int nc,
                  int sp, const float* __restrict__ wtab, float scale, int accumulate,
                  float* __restrict__ out) {
    const long long total = (long long)d * A * nc * B;
    for (long long o = (long long)blockIdx.x * kBlock + threadIdx.x; o < total;
         o += (long long)gridDim.x * kBlock) {
        const long long b = o % B;
        const int jc = (int)((o / B) % nc);
        const long long ca = o / (B * nc);  // c * A + a
        const int x0 = max(0, (jc - 3) * sp), x1 = min(n - 1, (jc + 1) * sp - 1);
        float acc = 0.f;
        for (int x = x0; x <= x1; ++x) {
            const int i = x / sp;
            acc += wtab[(x - i * sp) * 4 + (jc - i)] * in[(ca * n + x) * B + b];
        }
        out[o] = accumulate ? out[o] + scale * acc : scale * acc;
    }
}

}  // namespace

hipError_t launch_velocity(const PairDesc& P, const float* consts_dev, int transform, int dim,
                           const float* theta, float scale, float* out, hipStream_t s) {
    if (transform == AIR_TF_DENSE) {
        const long long n = (long long)dim * P.nvox;
        hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(kBlock), 0, s, theta, scale, n,
                           0, out);
    } else if (dim == 3) {
        hipLaunchKernelGGL(k_bs_field<3>, dim3(grid_for(P.nvox)), dim3(kBlock), 0, s, P,
                           consts_dev, theta, scale, out);
    } else {
        hipLaunchKernelGGL(k_bs_field<2>, dim3(grid_for(P.nvox)), dim3(kBlock), 0, s, P,
                           consts_dev, theta, scale, out);
    }
    return hipGetLastError();
}

hipError_t launch_compose(const PairDesc& P, int dim, const float* u, float* out,
                          unsigned int* dmax, hipStream_t s) {
    if (dim == 3)
        hipLaunchKernelGGL(k_compose<3>, dim3(xcd_grid(compose_items<3>(P), 0)), dim3(kBlock), 0,
                           s, P, u, out, dmax);
    else
        hipLaunchKernelGGL(k_compose<2>, dim3(xcd_grid(compose_items<2>(P), 0)), dim3(kBlock), 0,
                           s, P, u, out, dmax);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(cdiv(n, 64)), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

// gin = the adjoint of one squaring at u applied to gout. gmax_in: max |gout|
// as float bits (computed here when `measure_in`, else left by the previous
// call); gmax_out receives max |gin| for the next call. One uint each.
hipError_t launch_compose_adjoint(const PairDesc& P, int dim, const float* u, const float* gout,
                                  const unsigned int* dmax, unsigned int* gmax_in,
                                  bool measure_in, unsigned int* gmax_out, float* gin,
                                  hipStream_t s) {
    const long long n = (long long)dim * P.nvox;
    if (measure_in) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, gmax_in, 1);
        const int g = grid_for(n) < 1024 ? grid_for(n) : 1024;
        hipLaunchKernelGGL(k_absmax_plain, dim3(g), dim3(kBlock), 0, s, gout, n, gmax_in);
    }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, gmax_out, 1);
    if (dim == 3) {
        const int nt = cdiv(P.n[0], 16) * cdiv(P.n[1], 16) * cdiv(P.n[2], 16);
        hipLaunchKernelGGL(k_compose_adj_tile<3>, dim3(nt), dim3(kAdjBlock3), 0, s, P, u, gout,
                           dmax, gmax_in, gin, gmax_out);
    } else {
        const int nt = cdiv(P.n[0], 64) * cdiv(P.n[1], 64);
        hipLaunchKernelGGL(k_compose_adj_tile<2>, dim3(nt), dim3(kBlock), 0, s, P, u, gout, dmax,
                           gmax_in, gin, gmax_out);
    }
    return hipGetLastError();
}

// grad (+)= scale * (dL/dv -> dL/dtheta): dense: a scaled copy; B-spline:
// the transposed expansion, x then y (then z), through t1 [d][nz][ny][ncx]
// and t2 [d][nz][ncy][ncx].
hipError_t launch_velocity_adjoint(const PairDesc& P, const float* consts_dev, int transform,
                                   int dim, const float* g, float scale, float* t1, float* t2,
                                   float* grad, hipStream_t s, bool accumulate) {
    const int acc = accumulate ? 1 : 0;
    if (transform == AIR_TF_DENSE) {
        const long long n = (long long)dim * P.nvox;
        hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(kBlock), 0, s, g, scale, n,
                           acc, grad);
        return hipGetLastError();
    }
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int cx = P.nc[0], cy = P.nc[1], cz = P.nc[2];
    // x: [d][nz*ny][nx][1] -> [d][nz*ny][cx][1]
    long long tot = (long long)dim * nz * ny * cx;
    hipLaunchKernelGGL(k_bs_adjoint_axis, dim3(grid_for(tot)), dim3(kBlock), 0, s, g, dim,
                       (long long)nz * ny, nx, 1LL, cx, P.sp[0], consts_dev + P.wtab_off[0], 1.f,
                       0, t1);
    // y: [d][nz][ny][cx] -> [d][nz][cy][cx]
    tot = (long long)dim * nz * cy * cx;
    float* ydst = dim == 3 ? t2 : grad;
    hipLaunchKernelGGL(k_bs_adjoint_axis, dim3(grid_for(tot)), dim3(kBlock), 0, s, t1, dim,
                       (long long)nz, ny, (long long)cx, cy, P.sp[1], consts_dev + P.wtab_off[1],
                       dim == 3 ? 1.f : scale, dim == 3 ? 0 : acc, ydst);
    if (dim == 3) {
        // z: [d][1][nz][cy*cx] -> [d][1][cz][cy*cx]
        tot = (long long)dim * cz * cy * cx;
        hipLaunchKernelGGL(k_bs_adjoint_axis, dim3(grid_for(tot)), dim3(kBlock), 0, s, t2, dim,
                           1LL, nz, (long long)cy * cx, cz, P.sp[2], consts_dev + P.wtab_off[2],
                           scale, acc, grad);
    }
    return hipGetLastError();
}

}  // namespace air

// this unit's bounds-check flags (debug build only)
AIR_DEBUG_UNIT(diffeo)
