// LCC (Sec. III-B): the local version of NCC on a dense displacement u.
// For every voxel x of the masked set X' (sample point inside the moving
// image), over the window N(x) = {y in X' : |y - x|_inf <= r}:
//   n, the means muF, muW, the variances varF, varW and the covariance
//   (divided by n), rho(x) = cov / sqrt(varF varW + eps),
//   S = -(1/|X'|) sum_{x in X'} rho(x).
// The statistics come from box sums of m, mF, mW, mF^2, mW^2, mFW (m the
// mask), in FP64 so that E[X^2] - mu^2 does not cancel. Writing
// B = sum mW, D = sum mW^2, E = sum mFW over N(x), V = varF varW + eps:
//   drho/dB = -muF / (n sqrt V) + rho varF muW / (n V)
//   drho/dD = -rho varF / (2 n V)
//   drho/dE = 1 / (n sqrt V)
// and, as y is in N(x) exactly when x is in the window of y,
//   dS/dW(y) = -(1/|X'|) m(y) (box(aB) + 2 W(y) box(aD) + F(y) box(aE))(y)
// with a* = drho/d* on X' and 0 elsewhere. Every box sum is separable: an
// LDS-tiled pass over x and y, then a running sum along z — fused into one
// kernel per direction in 3D for radii up to 4 (the z window as a register
// ring), else as separate passes through FP64 maps.
#include "device_common.h"

namespace air {

namespace {

constexpr int kTX = 32, kTY = 8;   // xy tile of the box passes (kBlock threads)
constexpr int kZSeg = 16;          // voxels of z walked per thread in the z passes
constexpr double kLccEps = 1e-10;  // eps of the denominator (image units^4)

// Statistics -> rho and the coefficient maps (aB, aD, aE) on X' (two FP64
// divisions per voxel: 1/n and 1/sqrt(V)).
__device__ inline void lcc_coef(const double* s, float* aB, float* aD, float* aE, double* rho) {
    const double in = 1.0 / s[0];
    const double mf = s[1] * in, mw = s[2] * in;
    const double vf = s[3] * in - mf * mf, vw = s[4] * in - mw * mw;
    const double cv = s[5] * in - mf * mw;
    const double V = vf * vw + kLccEps;
    const double isq = 1.0 / sqrt(V);
    const double r = cv * isq;
    const double iV = isq * isq;
    *aB = (float)(in * (r * vf * mw * iV - mf * isq));
    *aD = (float)(-0.5 * r * vf * in * iV);
    *aE = (float)(in * isq);
    *rho = r;
}

// W, the mask and dW/dp (voxel units) at every voxel.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_lcc_sample(const PairDesc P, const float* __restrict__ M, const float* __restrict__ u,
             float* __restrict__ W, uint8_t* __restrict__ mk, float* __restrict__ dW) {
    const long long N = P.nvox;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < N;
         v += (long long)gridDim.x * kBlock) {
        const int idx[3] = {(int)(v % P.n[0]), (int)((v / P.n[0]) % P.n[1]),
                            DIM == 3 ? (int)(v / ((long long)P.n[0] * P.n[1])) : 0};
        Disp q[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) q[a] = disp_of(u[a * N + v], P.s[a]);
        bool in;
        float d[3];
        W[v] = sample_general<DIM>(M, P.n, idx, q, &in, d);
        mk[v] = in ? 1 : 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) dW[a * N + v] = d[a];
    }
}

// Box sums over x and y (radius r) of NCH channels at one plane:
// MODE 0: the six statistics channels of (F, W, m); MODE 1: three FP32 maps.
// out: [NCH][N] FP64. Dynamic LDS: the raw tile with halo, then the x sums.
template <int NCH, int MODE>
__global__ void __launch_bounds__(kBlock)
k_lcc_box_xy(const PairDesc P, int r, const float* __restrict__ a0, const float* __restrict__ a1,
             const float* __restrict__ a2, const uint8_t* __restrict__ mk,
             double* __restrict__ out) {
    extern __shared__ double lds[];
    constexpr int NIN = 3;
    const int HX = kTX + 2 * r, HY = kTY + 2 * r;
    float* raw = reinterpret_cast<float*>(lds);            // [NIN][HY][HX]
    double* xs = lds + (NIN * HY * HX + 1) / 2;             // [NCH][HY][kTX]
    const int ntx = cdiv(P.n[0], kTX), nty = cdiv(P.n[1], kTY);
    const int bx = blockIdx.x % ntx, by = (blockIdx.x / ntx) % nty;
    const int z = blockIdx.x / (ntx * nty);
    const int x0 = bx * kTX - r, y0 = by * kTY - r;
    const long long plane = (long long)z * P.n[0] * P.n[1];
    for (int i = threadIdx.x; i < HY * HX; i += kBlock) {
        const int yy = y0 + i / HX, xx = x0 + i % HX;
        float v0 = 0.f, v1 = 0.f, v2 = 0.f;
        if (xx >= 0 && xx < P.n[0] && yy >= 0 && yy < P.n[1]) {
            const long long v = plane + (long long)yy * P.n[0] + xx;
            if (MODE == 0) {
                if (mk[v]) {
                    v0 = 1.f;
                    v1 = a0[v];
                    v2 = a1[v];
                }
            } else {
                v0 = a0[v];
                v1 = a1[v];
                v2 = a2[v];
            }
        }
        raw[i] = v0;
        raw[HY * HX + i] = v1;
        raw[2 * HY * HX + i] = v2;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HY * kTX; i += kBlock) {
        const int ry = i / kTX, tx = i % kTX;
        double s[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) s[c] = 0.0;
        for (int dx = 0; dx <= 2 * r; ++dx) {
            const int k = ry * HX + tx + dx;
            const double e0 = raw[k], e1 = raw[HY * HX + k], e2 = raw[2 * HY * HX + k];
            if (MODE == 0) {
                // m, mF, mW, mF^2, mW^2, mFW (F and W are zero where m is)
                s[0] += e0;
                s[1] += e1;
                s[2] += e2;
                s[3] += e1 * e1;
                s[4 % NCH] += e2 * e2;
                s[5 % NCH] += e1 * e2;
            } else {
                s[0] += e0;
                s[1] += e1;
                s[2] += e2;
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) xs[(c * HY + ry) * kTX + tx] = s[c];
    }
    __syncthreads();
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int x = bx * kTX + tx, y = by * kTY + ty;
    if (x >= P.n[0] || y >= P.n[1]) return;
    const long long v = plane + (long long)y * P.n[0] + x;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        double t = 0.0;
        for (int dy = 0; dy <= 2 * r; ++dy) t += xs[(c * HY + ty + dy) * kTX + tx];
        out[c * P.nvox + v] = t;
    }
}

// Running box sum along z (radius rz) of NCH FP64 channels for one column and
// a segment of kZSeg planes; calls fin(z, v, sums) at every voxel.
template <int NCH, typename Fin>
__device__ inline void z_walk(const PairDesc& P, int rz, const double* __restrict__ S, long long col,
                              int z0, int z1, Fin fin) {
    const long long sz = (long long)P.n[0] * P.n[1];
    const long long N = P.nvox;
    double s[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) s[c] = 0.0;
    for (int zz = max(0, z0 - rz); zz <= min(P.n[2] - 1, z0 + rz); ++zz)
#pragma unroll
        for (int c = 0; c < NCH; ++c) s[c] += S[c * N + zz * sz + col];
    for (int z = z0; z < z1; ++z) {
        fin(z, z * sz + col, s);
        const int za = z + rz + 1, zr = z - rz;
        if (za < P.n[2])
#pragma unroll
            for (int c = 0; c < NCH; ++c) s[c] += S[c * N + za * sz + col];
        if (zr >= 0)
#pragma unroll
            for (int c = 0; c < NCH; ++c) s[c] -= S[c * N + zr * sz + col];
    }
}

// Statistics -> rho and the coefficient maps (aB, aD, aE) on X'; per-block
// partial sums of (count, sum rho) in block order.
__global__ void __launch_bounds__(kBlock)
k_lcc_stats_z(const PairDesc P, int rz, const double* __restrict__ S,
              const float* __restrict__ F, const float* __restrict__ W,
              const uint8_t* __restrict__ mk, float* __restrict__ A, double* __restrict__ part) {
    __shared__ double red[2 * (kBlock / 64)];
    const long long N = P.nvox;
    const long long ncol = (long long)P.n[0] * P.n[1];
    const int nseg = cdiv(P.n[2], kZSeg);
    const long long item = (long long)blockIdx.x * kBlock + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (item < ncol * nseg) {
        const long long col = item % ncol;
        const int seg = (int)(item / ncol);
        const int z0 = seg * kZSeg, z1 = min(P.n[2], z0 + kZSeg);
        z_walk<6>(P, rz, S, col, z0, z1, [&](int, long long v, const double* s) {
            float aB = 0.f, aD = 0.f, aE = 0.f;
            if (mk[v]) {
                double rho;
                lcc_coef(s, &aB, &aD, &aE, &rho);
                acc[0] += 1.0;
                acc[1] += rho;
            }
            A[v] = aB;
            A[N + v] = aD;
            A[2 * N + v] = aE;
        });
    }
    block_sum<kBlock, 2>(acc, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
}

// value = S (+ lambda * value when lam_acc); scal[0] = 1 / |X'| (0 if empty);
// flags of the pair on an empty mask or a non-finite value.
__global__ void __launch_bounds__(kBlock)
k_lcc_value(const double* __restrict__ part, int nblk, float lambda, int lam_acc, float* value,
            double* scal, uint32_t* flag) {
    __shared__ double red[2 * (kBlock / 64)];
    double s[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        s[0] += part[2 * b];
        s[1] += part[2 * b + 1];
    }
    block_sum<kBlock, 2>(s, red);
    if (threadIdx.x == 0) {
        const double cnt = s[0];
        const double S = cnt >= 1.0 ? -s[1] / cnt : 0.0;
        const float v = lam_acc ? (float)(S + (double)lambda * (double)*value) : (float)S;
        *value = v;
        scal[0] = cnt >= 1.0 ? 1.0 / cnt : 0.0;
        uint32_t f = 0;
        if (cnt < 1.0) f |= AIR_FLAG_DEGENERATE;
        if (!isfinite(v)) f |= AIR_FLAG_NONFINITE;
        *flag = f;
    }
}

// g_a = dS/dW dW/dp_a (n_a - 1)/2 on X' (+ lambda g_a when lam_acc).
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_lcc_grad_z(const PairDesc P, int rz, const double* __restrict__ T,
             const float* __restrict__ F, const float* __restrict__ W,
             const uint8_t* __restrict__ mk, const float* __restrict__ dW,
             const double* __restrict__ scal, float lambda, int lam_acc, float* __restrict__ g) {
    const long long N = P.nvox;
    const long long ncol = (long long)P.n[0] * P.n[1];
    const int nseg = cdiv(P.n[2], kZSeg);
    const long long item = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (item >= ncol * nseg) return;
    const long long col = item % ncol;
    const int seg = (int)(item / ncol);
    const int z0 = seg * kZSeg, z1 = min(P.n[2], z0 + kZSeg);
    const double inv = scal[0];
    z_walk<3>(P, rz, T, col, z0, z1, [&](int, long long v, const double* s) {
        float dsdw = 0.f;
        if (mk[v]) dsdw = (float)(-inv * (s[0] + 2.0 * (double)W[v] * s[1] + (double)F[v] * s[2]));
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const float img = dsdw * dW[a * N + v] * P.s[a];
            g[a * N + v] = lam_acc ? fmaf(lambda, g[a * N + v], img) : img;
        }
    });
}

// ---- fused box passes: xy sums in LDS, z window as a register ring ------
// A block owns a kTX x kTY column tile and a chunk of kZc output planes. It
// walks the planes of the chunk plus the R-plane halo on each side; for each
// plane it forms the xy box sums of its columns in LDS (as k_lcc_box_xy),
// adds them to a running z sum and subtracts the plane that leaves the
// window, kept in a ring of 2R + 1 slots. The plane loop is unrolled by
// 2R + 1 so that every ring slot is a fixed register. Global loads run one
// plane ahead: the next plane's tile (and the next output plane's per-voxel
// inputs) are in flight while the current plane is summed.
constexpr int kZc = 16;   // output planes per block of the fused passes
constexpr int kMaxFusedR = 4;   // radii the register ring covers (3D)

template <int R>
struct Halo {
    static constexpr int HX = kTX + 2 * R, HY = kTY + 2 * R, NI = HX * HY;
    static constexpr int NF = (NI + kBlock - 1) / kBlock;   // tile elements per thread
};

template <int R, int NCH>
struct XYPlane {
    alignas(16) float raw[3][Halo<R>::NI];   // NI is even: every row starts 8-byte aligned
    alignas(16) double xs[NCH][Halo<R>::HY][kTX];
};

// One plane's tile with halo, as loaded (every load unconditional at a
// clamped address; ok marks the elements inside the volume).
template <int R>
struct TileRegs {
    float a[3][Halo<R>::NF];
    uint8_t m[Halo<R>::NF];
    uint32_t ok;
};

// MODE 0: a0 = F, a1 = W and mk the mask; MODE 1: three FP32 maps.
template <int R, int MODE>
__device__ inline void fetch_tile(const PairDesc& P, int bx, int by, int zz,
                                  const float* __restrict__ a0, const float* __restrict__ a1,
                                  const float* __restrict__ a2, const uint8_t* __restrict__ mk,
                                  TileRegs<R>& t) {
    using H = Halo<R>;
    const int x0 = bx * kTX - R, y0 = by * kTY - R;
    const bool zin = zz >= 0 && zz < P.n[2];
    const long long plane = (long long)zz * P.n[0] * P.n[1];
    t.ok = 0;
#pragma unroll
    for (int it = 0; it < H::NF; ++it) {
        const int i = threadIdx.x + it * kBlock;
        const int yy = y0 + i / H::HX, xx = x0 + i % H::HX;
        const bool in = i < H::NI && zin && xx >= 0 && xx < P.n[0] && yy >= 0 && yy < P.n[1];
        const long long v = in ? plane + (long long)yy * P.n[0] + xx : 0;
        t.ok |= (in ? 1u : 0u) << it;
        t.a[0][it] = a0[v];
        t.a[1][it] = a1[v];
        if (MODE == 0)
            t.m[it] = mk[v];
        else
            t.a[2][it] = a2[v];
    }
}

// The tile's channels into LDS: MODE 0 (m, mF, mW), MODE 1 the maps, zero
// outside the volume.
template <int R, int NCH, int MODE>
__device__ inline void commit_tile(XYPlane<R, NCH>& L, const TileRegs<R>& t) {
    using H = Halo<R>;
#pragma unroll
    for (int it = 0; it < H::NF; ++it) {
        const int i = threadIdx.x + it * kBlock;
        const bool ok = (t.ok >> it) & 1u;
        float v0, v1, v2;
        if (MODE == 0) {
            const bool m = ok && t.m[it] != 0;
            v0 = m ? 1.f : 0.f;
            v1 = m ? t.a[0][it] : 0.f;
            v2 = m ? t.a[1][it] : 0.f;
        } else {
            v0 = ok ? t.a[0][it] : 0.f;
            v1 = ok ? t.a[1][it] : 0.f;
            v2 = ok ? t.a[2][it] : 0.f;
        }
        if (H::NI % kBlock == 0 || i < H::NI) {
            L.raw[0][i] = v0;
            L.raw[1][i] = v1;
            L.raw[2][i] = v2;
        }
    }
}

// x sums of the committed tile, then the column's y sums (out). MODE 0 forms
// m, mF, mW, mF^2, mW^2, mFW (F and W are zero where m is). A thread forms
// two neighbouring x sums, which share 2R of their 2R + 1 terms. Every
// thread of the block calls it; raw must be complete (barrier before), and
// xs is free again only after the next barrier.
template <int R, int NCH, int MODE>
__device__ inline void xy_sums(XYPlane<R, NCH>& L, double* out) {
    using H = Halo<R>;
    constexpr int XP = kTX / 2;   // pairs of x outputs per row
    constexpr int NE = 2 * R + 2; // raw elements a pair reads
    for (int i = threadIdx.x; i < H::HY * XP; i += kBlock) {
        const int ry = i / XP, tx = 2 * (i % XP);
        float e[3][NE];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < NE; k += 2) {
                const float2 q = *reinterpret_cast<const float2*>(&L.raw[c][ry * H::HX + tx + k]);
                e[c][k] = q.x;
                e[c][k + 1] = q.y;
            }
        double mid[NCH];   // the 2R shared terms
#pragma unroll
        for (int c = 0; c < NCH; ++c) mid[c] = 0.0;
#pragma unroll
        for (int k = 1; k <= 2 * R; ++k) {
            const double e0 = e[0][k], e1 = e[1][k], e2 = e[2][k];
            mid[0] += e0;
            mid[1] += e1;
            mid[2] += e2;
            if (MODE == 0) {
                mid[3 % NCH] = fma(e1, e1, mid[3 % NCH]);
                mid[4 % NCH] = fma(e2, e2, mid[4 % NCH]);
                mid[5 % NCH] = fma(e1, e2, mid[5 % NCH]);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = h ? NE - 1 : 0;
            const double e0 = e[0][k], e1 = e[1][k], e2 = e[2][k];
            double o[NCH];
            o[0] = mid[0] + e0;
            o[1] = mid[1] + e1;
            o[2] = mid[2] + e2;
            if (MODE == 0) {
                o[3 % NCH] = fma(e1, e1, mid[3 % NCH]);
                o[4 % NCH] = fma(e2, e2, mid[4 % NCH]);
                o[5 % NCH] = fma(e1, e2, mid[5 % NCH]);
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) L.xs[c][ry][tx + h] = o[c];
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        double t = 0.0;
#pragma unroll
        for (int dy = 0; dy <= 2 * R; ++dy) t += L.xs[c][ty + dy][tx];
        out[c] = t;
    }
}

// Walk the planes of a chunk [z0, z1). pre(z) issues the loads of output
// plane z's per-voxel inputs one plane before fin(z, sums) uses them.
template <int R, int NCH, int MODE, typename Pre, typename Fin>
__device__ inline void z_ring_walk(const PairDesc& P, XYPlane<R, NCH>& L, int bx, int by, int z0,
                                   int z1, const float* a0, const float* a1, const float* a2,
                                   const uint8_t* mk, Pre pre, Fin fin) {
    constexpr int S = 2 * R + 1;
    double ring[S][NCH];
    double zs[NCH];
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int c = 0; c < NCH; ++c) ring[k][c] = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) zs[c] = 0.0;
    const int zlast = z1 - 1 + R;
    TileRegs<R> t;
    fetch_tile<R, MODE>(P, bx, by, z0 - R, a0, a1, a2, mk, t);
    for (int zb = z0 - R; zb <= zlast; zb += S) {
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int zz = zb + k;
            if (zz > zlast) break;  // uniform over the block
            // raw is free: every thread passed the x sums of the last plane
            commit_tile<R, NCH, MODE>(L, t);
            __syncthreads();
            if (zz < zlast) fetch_tile<R, MODE>(P, bx, by, zz + 1, a0, a1, a2, mk, t);
            double p[NCH];
            xy_sums<R, NCH, MODE>(L, p);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                zs[c] += p[c] - ring[k][c];   // ring[k] holds plane zz - S, leaving now
                ring[k][c] = p[c];
            }
            const int z = zz - R;              // its window [z - R, z + R] is complete
            if (z >= z0) fin(z, zs);
            if (z + 1 >= z0 && z + 1 < z1) pre(z + 1);
        }
    }
}

template <int R>
__global__ void __launch_bounds__(kBlock)
k_lcc_stats_fused(const PairDesc P, const float* __restrict__ F, const float* __restrict__ W,
                  const uint8_t* __restrict__ mk, float* __restrict__ A, double* __restrict__ part) {
    __shared__ XYPlane<R, 6> L;
    __shared__ double red[2 * (kBlock / 64)];
    const int ntx = cdiv(P.n[0], kTX), nty = cdiv(P.n[1], kTY);
    const int bx = blockIdx.x % ntx, by = (blockIdx.x / ntx) % nty;
    const int z0 = (blockIdx.x / (ntx * nty)) * kZc, z1 = min(P.n[2], z0 + kZc);
    const int x = bx * kTX + threadIdx.x % kTX, y = by * kTY + threadIdx.x / kTX;
    const bool col = x < P.n[0] && y < P.n[1];
    const long long N = P.nvox;
    const long long c0 = col ? (long long)y * P.n[0] + x : 0;
    const long long sz = (long long)P.n[0] * P.n[1];
    double acc[2] = {0.0, 0.0};
    uint8_t mnext = 0;
    z_ring_walk<R, 6, 0>(
        P, L, bx, by, z0, z1, F, W, nullptr, mk,
        [&](int z) { mnext = mk[z * sz + c0]; },
        [&](int z, const double* s) {
            float aB = 0.f, aD = 0.f, aE = 0.f;
            if (col && mnext) {
                double rho;
                lcc_coef(s, &aB, &aD, &aE, &rho);
                acc[0] += 1.0;
                acc[1] += rho;
            }
            if (col) {
                const long long v = z * sz + c0;
                A[v] = aB;
                A[N + v] = aD;
                A[2 * N + v] = aE;
            }
        });
    block_sum<kBlock, 2>(acc, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
}

template <int R, int DIM>
__global__ void __launch_bounds__(kBlock)
k_lcc_grad_fused(const PairDesc P, const float* __restrict__ A, const float* __restrict__ F,
                 const float* __restrict__ W, const uint8_t* __restrict__ mk,
                 const float* __restrict__ dW, const double* __restrict__ scal, float lambda,
                 int lam_acc, float* __restrict__ g) {
    __shared__ XYPlane<R, 3> L;
    const int ntx = cdiv(P.n[0], kTX), nty = cdiv(P.n[1], kTY);
    const int bx = blockIdx.x % ntx, by = (blockIdx.x / ntx) % nty;
    const int z0 = (blockIdx.x / (ntx * nty)) * kZc, z1 = min(P.n[2], z0 + kZc);
    const int x = bx * kTX + threadIdx.x % kTX, y = by * kTY + threadIdx.x / kTX;
    const bool col = x < P.n[0] && y < P.n[1];
    const long long N = P.nvox;
    const long long c0 = col ? (long long)y * P.n[0] + x : 0;
    const long long sz = (long long)P.n[0] * P.n[1];
    const double inv = scal[0];
    // per-voxel inputs of the next output plane
    uint8_t m = 0;
    float w = 0.f, f = 0.f, d[DIM], g0[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) d[a] = g0[a] = 0.f;
    z_ring_walk<R, 3, 1>(
        P, L, bx, by, z0, z1, A, A + N, A + 2 * N, nullptr,
        [&](int z) {
            const long long v = z * sz + c0;
            m = mk[v];
            w = W[v];
            f = F[v];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                d[a] = dW[a * N + v];
                if (lam_acc) g0[a] = g[a * N + v];
            }
        },
        [&](int z, const double* s) {
            if (!col) return;
            const long long v = z * sz + c0;
            float dsdw = 0.f;
            if (m) dsdw = (float)(-inv * (s[0] + 2.0 * (double)w * s[1] + (double)f * s[2]));
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const float img = dsdw * d[a] * P.s[a];
                g[a * N + v] = lam_acc ? fmaf(lambda, g0[a], img) : img;
            }
        });
}

__host__ inline int lcc_grid(long long n) {
    const long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

__host__ inline size_t box_lds(int nch, int r) {
    const int HX = kTX + 2 * r, HY = kTY + 2 * r;
    return sizeof(double) * ((3 * HY * HX + 1) / 2 + (size_t)nch * HY * kTX);
}

}  // namespace

// Partial-sum slots of the statistics pass (the larger of the two forms).
int lcc_partials(const PairDesc& P) {
    const long long items = (long long)P.n[0] * P.n[1] * cdiv(P.n[2], kZSeg);
    const int zpass = (int)((items + kBlock - 1) / kBlock);
    const int fused = cdiv(P.n[0], kTX) * cdiv(P.n[1], kTY) * cdiv(P.n[2], kZc);
    return max(zpass, fused);
}

// Whether the fused passes (no FP64 box-sum maps) serve this dimension and radius.
bool lcc_fused(int dim, int r) { return dim == 3 && r >= 1 && r <= kMaxFusedR; }

// LDS of the box passes at radius r (the largest, six channels).
size_t lcc_lds_bytes(int r) { return box_lds(6, r); }

// S (and, with grad, dS/du) of the LCC at displacement u. Buffers: W, dW
// ([d][N]) float; mk uint8 [N]; S double [6][N]; A float [3][N]; part double
// [2 * lcc_partials]; scal double [1]. value: S, or S + lambda * value when
// lam_acc (the regulariser written there before); grad: dS/du, or
// dS/du + lambda * grad when lam_acc.
hipError_t launch_lcc(const PairDesc& P, int dim, int r, const float* F, const float* M,
                      const float* u, float* Wb, uint8_t* mk, float* dW, double* S, float* A,
                      double* part, double* scal, uint32_t* flag, float lambda, bool lam_acc,
                      float* value, float* grad, hipStream_t s) {
    const int rz = dim == 3 ? r : 0;
    const int nxy = cdiv(P.n[0], kTX) * cdiv(P.n[1], kTY) * P.n[2];
    const int acc = lam_acc ? 1 : 0;
    if (dim == 3)
        hipLaunchKernelGGL(k_lcc_sample<3>, dim3(lcc_grid(P.nvox)), dim3(kBlock), 0, s, P, M, u,
                           Wb, mk, dW);
    else
        hipLaunchKernelGGL(k_lcc_sample<2>, dim3(lcc_grid(P.nvox)), dim3(kBlock), 0, s, P, M, u,
                           Wb, mk, dW);
    if (lcc_fused(dim, r)) {
        // fused passes: no FP64 maps in memory
        const int nb = cdiv(P.n[0], kTX) * cdiv(P.n[1], kTY) * cdiv(P.n[2], kZc);
        switch (r) {
            case 1:
                hipLaunchKernelGGL(k_lcc_stats_fused<1>, dim3(nb), dim3(kBlock), 0, s, P, F, Wb,
                                   mk, A, part);
                break;
            case 2:
                hipLaunchKernelGGL(k_lcc_stats_fused<2>, dim3(nb), dim3(kBlock), 0, s, P, F, Wb,
                                   mk, A, part);
                break;
            case 3:
                hipLaunchKernelGGL(k_lcc_stats_fused<3>, dim3(nb), dim3(kBlock), 0, s, P, F, Wb,
                                   mk, A, part);
                break;
            default:
                hipLaunchKernelGGL(k_lcc_stats_fused<4>, dim3(nb), dim3(kBlock), 0, s, P, F, Wb,
                                   mk, A, part);
                break;
        }
        hipLaunchKernelGGL(k_lcc_value, dim3(1), dim3(kBlock), 0, s, part, nb, lambda, acc, value,
                           scal, flag);
        if (!grad) return hipGetLastError();
        switch (r) {
            case 1:
                hipLaunchKernelGGL((k_lcc_grad_fused<1, 3>), dim3(nb), dim3(kBlock), 0, s, P, A, F, Wb,
                                   mk, dW, scal, lambda, acc, grad);
                break;
            case 2:
                hipLaunchKernelGGL((k_lcc_grad_fused<2, 3>), dim3(nb), dim3(kBlock), 0, s, P, A, F, Wb,
                                   mk, dW, scal, lambda, acc, grad);
                break;
            case 3:
                hipLaunchKernelGGL((k_lcc_grad_fused<3, 3>), dim3(nb), dim3(kBlock), 0, s, P, A, F, Wb,
                                   mk, dW, scal, lambda, acc, grad);
                break;
            default:
                hipLaunchKernelGGL((k_lcc_grad_fused<4, 3>), dim3(nb), dim3(kBlock), 0, s, P, A, F, Wb,
                                   mk, dW, scal, lambda, acc, grad);
                break;
        }
        return hipGetLastError();
    }
    const int nblk = (int)(((long long)P.n[0] * P.n[1] * cdiv(P.n[2], kZSeg) + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_lcc_box_xy<6, 0>), dim3(nxy), dim3(kBlock), box_lds(6, r), s, P, r, F,
                       Wb, nullptr, mk, S);
    hipLaunchKernelGGL(k_lcc_stats_z, dim3(nblk), dim3(kBlock), 0, s, P, rz, S, F, Wb, mk, A,
                       part);
    hipLaunchKernelGGL(k_lcc_value, dim3(1), dim3(kBlock), 0, s, part, nblk, lambda, acc, value,
                       scal, flag);
    if (!grad) return hipGetLastError();
    // the coefficient box sums reuse the statistics buffer
    hipLaunchKernelGGL((k_lcc_box_xy<3, 1>), dim3(nxy), dim3(kBlock), box_lds(3, r), s, P, r, A,
                       A + P.nvox, A + 2 * P.nvox, mk, S);
    if (dim == 3)
        hipLaunchKernelGGL(k_lcc_grad_z<3>, dim3(nblk), dim3(kBlock), 0, s, P, rz, S, F, Wb, mk,
                           dW, scal, lambda, acc, grad);
    else
        hipLaunchKernelGGL(k_lcc_grad_z<2>, dim3(nblk), dim3(kBlock), 0, s, P, rz, S, F, Wb, mk,
                           dW, scal, lambda, acc, grad);
    return hipGetLastError();
}

// S of the LCC for a given warped image and mask (no gradient).
hipError_t launch_lcc_value(const PairDesc& P, int dim, int r, const float* F, const float* Wimg,
                            const uint8_t* mk, double* S, float* A, double* part, double* scal,
                            uint32_t* flag, float* value, hipStream_t s) {
    const int rz = dim == 3 ? r : 0;
    const int nxy = cdiv(P.n[0], kTX) * cdiv(P.n[1], kTY) * P.n[2];
    if (lcc_fused(dim, r)) {
        const int nb = cdiv(P.n[0], kTX) * cdiv(P.n[1], kTY) * cdiv(P.n[2], kZc);
        switch (r) {
            case 1:
                hipLaunchKernelGGL(k_lcc_stats_fused<1>, dim3(nb), dim3(kBlock), 0, s, P, F, Wimg,
                                   mk, A, part);
                break;
            case 2:
                hipLaunchKernelGGL(k_lcc_stats_fused<2>, dim3(nb), dim3(kBlock), 0, s, P, F, Wimg,
                                   mk, A, part);
                break;
            case 3:
                hipLaunchKernelGGL(k_lcc_stats_fused<3>, dim3(nb), dim3(kBlock), 0, s, P, F, Wimg,
                                   mk, A, part);
                break;
            default:
                hipLaunchKernelGGL(k_lcc_stats_fused<4>, dim3(nb), dim3(kBlock), 0, s, P, F, Wimg,
                                   mk, A, part);
                break;
        }
        hipLaunchKernelGGL(k_lcc_value, dim3(1), dim3(kBlock), 0, s, part, nb, 0.f, 0, value, scal,
                           flag);
        return hipGetLastError();
    }
    const int nblk = (int)(((long long)P.n[0] * P.n[1] * cdiv(P.n[2], kZSeg) + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_lcc_box_xy<6, 0>), dim3(nxy), dim3(kBlock), box_lds(6, r), s, P, r, F,
                       Wimg, nullptr, mk, S);
    hipLaunchKernelGGL(k_lcc_stats_z, dim3(nblk), dim3(kBlock), 0, s, P, rz, S, F, Wimg, mk, A,
                       part);
    hipLaunchKernelGGL(k_lcc_value, dim3(1), dim3(kBlock), 0, s, part, nblk, 0.f, 0, value, scal,
                       flag);
    return hipGetLastError();
}

}  // namespace air
