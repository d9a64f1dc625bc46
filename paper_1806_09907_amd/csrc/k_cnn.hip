// Learned-initialisation CNN kernels (BF16 operands, FP32 accumulation).
//
// Activations are NDHWC bf16 [z][y][x][C] with C a multiple of 8; 3x3x3
// convolutions have stride 1 and zero padding 1. Weights are stored
// output-major with the reduction index contiguous: Wt[co][k], k = tap*C_in +
// ci, tap = (dz*3 + dy)*3 + dx.
//
// conv forward (implicit GEMM): Y[m][co] = b[co] + sum_k A[m][k] Wt[co][k],
// A[m][k] = X[voxel m shifted by tap][ci]; one wave computes 16 voxels x all
// output channels with v_mfma_f32_16x16x32_bf16 (A: lane l holds row l%16,
// reduction elements 8*(l/16)..+8; B: column l%16, the same reduction range;
// D: column l%16, rows 4*(l/16)..+4). Each lane's 8 reduction elements are 8
// consecutive channels of one tap, i.e. one 16-byte load.
// conv backward-data = the forward kernel on the gradient with flipped,
// transposed weights (Wf[ci][tap'*C_out + co] = Wt[co][(26 - tap')*C_in + ci]).
// conv backward-weight: dWt[co][k] = sum_m dY[m][co] A[m][k], an MFMA GEMM
// that reduces over chunks of voxels into per-chunk partials, summed in a
// fixed order by a second kernel.
#include "device_common.h"

namespace air {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__device__ inline float bf2f(u16 v) { return __uint_as_float(((uint32_t)v) << 16); }
// round to nearest even (inputs are finite in this network)
__device__ inline u16 f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u16)(u >> 16);  // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

// A batch of volumes is stacked along z: nz = batch * nzv, and a tap that
// would cross from one volume into the next reads zero padding instead.
struct ConvDims {
    int nx, ny, nz;
    int nzv;         // depth of one volume of the stack
    int cin, cout;
    int K, Kpad;     // 27 * cin, rounded up to a multiple of 32
};

// Epilogue of the forward form: v = acc + bias[co], then act 0: v, act 1:
// LeakyReLU(0.1)(v), act 2: v * LeakyReLU'(a) with a the stored bf16
// activation gate[row * ldg + goff + co] (the adjoint of the activation, for
// backward-data). Written as bf16 and/or FP32.
struct ConvEpi {
    const float* bias;
    int act;
    const u16* gate;
    int ldg, goff;
    u16* ybf;
    int ldy, yoff;
    float* yf;
    int ldyf;
};

__device__ inline void conv_store(const ConvEpi& E, long long row, int co, float v, float b) {
    v += b;
    if (E.act == 1) {
        v = v > 0.f ? v : 0.1f * v;
    } else if (E.act == 2) {
        const float a = bf2f(E.gate[row * E.ldg + E.goff + co]);
        v = a > 0.f ? v : 0.1f * v;
    }
    if (E.ybf) E.ybf[row * E.ldy + E.yoff + co] = f2bf(v);
    if (E.yf) E.yf[row * E.ldyf + co] = v;
}

// output voxel of one lane: stack coordinates and the depth within its volume
struct Vox {
    int x, y, z, zl;
    bool valid;
};

__device__ inline Vox vox_of(long long m, const ConvDims& D, long long N) {
    Vox v;
    v.valid = m < N;
    v.x = (int)(m % D.nx);
    v.y = (int)((m / D.nx) % D.ny);
    v.z = (int)(m / ((long long)D.nx * D.ny));
    v.zl = v.z % D.nzv;
    return v;
}

__device__ inline bf16x8 load_a(const u16* __restrict__ X, const ConvDims& D, const Vox& p,
                                int tap, int ci) {
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int x = p.x + dx, y = p.y + dy;
    const bool in = p.valid && tap < 27 && (unsigned)x < (unsigned)D.nx &&
                    (unsigned)y < (unsigned)D.ny && (unsigned)(p.zl + dz) < (unsigned)D.nzv;
    uint4 q = make_uint4(0, 0, 0, 0);
    if (in) {
        const long long v = ((long long)(p.z + dz) * D.ny + y) * D.nx + x;
        q = *reinterpret_cast<const uint4*>(X + v * D.cin + ci);
    }
    return __builtin_bit_cast(bf16x8, q);
}

__device__ inline bf16x8 load_w(const u16* __restrict__ Wt, const ConvDims& D, int co, int k) {
    uint4 q = make_uint4(0, 0, 0, 0);
    if (co < D.cout && k < D.K) q = *reinterpret_cast<const uint4*>(Wt + (long long)co * D.K + k);
    return __builtin_bit_cast(bf16x8, q);
}

// One block = 4 waves; a wave computes MT tiles of 16 output voxels x all
// NT16 = ceil(cout / 16) column tiles, so each weight operand it loads
// feeds MT products.
template <int NT16, int MT>
__global__ void __launch_bounds__(256)
k_conv_fwd(const u16* __restrict__ X, ConvDims D, const u16* __restrict__ Wt, ConvEpi E) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long N = (long long)D.nx * D.ny * D.nz;
    const long long m0 = ((long long)blockIdx.x * 4 + wave) * (16 * MT);
    if (m0 >= N) return;
    const int g = lane >> 4;
    Vox p[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) p[t] = vox_of(m0 + 16 * t + (lane & 15), D, N);
    f32x4 acc[MT][NT16];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int j = 0; j < NT16; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < D.Kpad; kc += 32) {
        const int k = kc + 8 * g;
        const int tap = k / D.cin, ci = k - tap * D.cin;
        bf16x8 a[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) a[t] = load_a(X, D, p[t], tap, ci);
#pragma unroll
        for (int j = 0; j < NT16; ++j) {
            const bf16x8 b = load_w(Wt, D, j * 16 + (lane & 15), k);
#pragma unroll
            for (int t = 0; t < MT; ++t)
                acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b, acc[t][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < NT16; ++j) {
        const int co = j * 16 + (lane & 15);
        if (co >= D.cout) continue;
        const float b = E.bias ? E.bias[co] : 0.f;
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long row = m0 + 16 * t + 4 * g + i;
                if (row < N) conv_store(E, row, co, acc[t][j][i], b);
            }
    }
}

// Split-K form for small volumes (too few 64-voxel blocks to fill the
// chip): a block takes 16 voxels, its four waves take every fourth 32-wide
// reduction step, and the four partial tiles are added in wave order through
// LDS before the same epilogue.
template <int NT16>
__global__ void __launch_bounds__(256)
k_conv_fwd_sk(const u16* __restrict__ X, ConvDims D, const u16* __restrict__ Wt, ConvEpi E) {
    __shared__ f32x4 red[4][NT16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long N = (long long)D.nx * D.ny * D.nz;
    const long long m0 = (long long)blockIdx.x * 16;
    const Vox p = vox_of(m0 + (lane & 15), D, N);
    const int g = lane >> 4;
    f32x4 acc[NT16];
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 32 * wave; kc < D.Kpad; kc += 128) {
        const int k = kc + 8 * g;
        const int tap = k / D.cin, ci = k - tap * D.cin;
        const bf16x8 a = load_a(X, D, p, tap, ci);
#pragma unroll
        for (int t = 0; t < NT16; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a, load_w(Wt, D, t * 16 + (lane & 15), k), acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT16; ++t) red[wave][t][lane] = acc[t];
    __syncthreads();
    for (int t = wave; t < NT16; t += 4) {
        const f32x4 v = ((red[0][t][lane] + red[1][t][lane]) + red[2][t][lane]) + red[3][t][lane];
        const int co = t * 16 + (lane & 15);
        if (co >= D.cout) continue;
        const float b = E.bias ? E.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long long row = m0 + 4 * g + i;
            if (row < N) conv_store(E, row, co, v[i], b);
        }
    }
}

// dWt partial of voxel chunk `blockIdx.z` (`chunk` voxels, a multiple of
// 128): the block's four waves compute the 16 output channels co0.. of tile
// blockIdx.y against BWK k-tiles of 16 reduction columns (k = tap * C_in +
// ci), each wave taking 32 voxels of every 128-voxel step. Per step every
// lane loads one 16-byte channel vector of dY and of each shifted input, the
// wave transposes them through its own LDS tiles into [channel][voxel]
// rows, and each MFMA operand is one 16-byte LDS read (8 consecutive voxels
// of one channel). The four waves' sums are added in wave order through LDS
// into one partial per chunk. The k-group-0 block of each co tile also sums
// dY over the chunk for the bias gradient.
constexpr int BWK = 7;    // k tiles per wave
constexpr int BWP = 40;   // LDS row pitch in bf16 (32 voxels + pad, 16-byte multiple)
constexpr int kBwStep = 128;
__global__ void __launch_bounds__(256)
k_conv_bwdw(const u16* __restrict__ X, ConvDims D, const u16* __restrict__ dY, int chunk,
            float* __restrict__ part) {
    constexpr int kTileA = 16 * BWP, kTileB = BWK * 16 * BWP;   // u16 per wave
    __shared__ __align__(16) u16 lds[4 * (kTileA + kTileB)];
    static_assert(sizeof(lds) >= (4 * BWK * 64) * sizeof(f32x4) + 4 * 64 * sizeof(float),
                  "the wave reduction reuses the operand tiles");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u16* sA = lds + wave * (kTileA + kTileB);
    u16* sB = sA + kTileA;
    const int co0 = blockIdx.y * 16, kt0 = blockIdx.x * BWK;
    const long long N = (long long)D.nx * D.ny * D.nz;
    const long long mb = (long long)blockIdx.z * chunk;
    const long long me = mb + chunk < N ? mb + chunk : N;
    const int g = lane >> 4, r = lane & 15;
    // loader role: voxel lv of the wave's 32, channel half lh (8 channels)
    const int lv = lane >> 1, lh = lane & 1;
    const bool co_ok = co0 + 8 * lh < D.cout;
    // each loader's B rows: k = (kt0 + t) * 16 + 8 * lh .. + 8, one tap
    int ltap[BWK], lci[BWK];
#pragma unroll
    for (int t = 0; t < BWK; ++t) {
        const int k = (kt0 + t) * 16 + 8 * lh;
        ltap[t] = k < D.K ? k / D.cin : 27;
        lci[t] = k < D.K ? k - ltap[t] * D.cin : 0;
    }
    f32x4 acc[BWK];
#pragma unroll
    for (int t = 0; t < BWK; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    // this lane's 16-byte vectors of one step (zero past the chunk)
    struct Step {
        uint4 a, b[BWK];
    };
    auto load = [&](long long mc) -> Step {
        Step q;
        const Vox p = vox_of(mc + 32 * wave + lv, D, me);
        q.a = make_uint4(0, 0, 0, 0);
        if (p.valid && co_ok)
            q.a = *reinterpret_cast<const uint4*>(dY + (mc + 32 * wave + lv) * D.cout + co0 +
                                                  8 * lh);
#pragma unroll
        for (int t = 0; t < BWK; ++t) {
            const int tap = ltap[t];
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const int x = p.x + dx, y = p.y + dy;
            q.b[t] = make_uint4(0, 0, 0, 0);
            if (p.valid && tap < 27 && (unsigned)x < (unsigned)D.nx &&
                (unsigned)y < (unsigned)D.ny && (unsigned)(p.zl + dz) < (unsigned)D.nzv) {
                const long long v = ((long long)(p.z + dz) * D.ny + y) * D.nx + x;
                q.b[t] = *reinterpret_cast<const uint4*>(X + v * D.cin + lci[t]);
            }
        }
        return q;
    };
    auto process = [&](const Step& q) {
        __syncthreads();  // the previous step's operand reads are done
        {
            const u16* e = reinterpret_cast<const u16*>(&q.a);
#pragma unroll
            for (int j = 0; j < 8; ++j) sA[(8 * lh + j) * BWP + lv] = e[j];
        }
#pragma unroll
        for (int t = 0; t < BWK; ++t) {
            const u16* e = reinterpret_cast<const u16*>(&q.b[t]);
#pragma unroll
            for (int j = 0; j < 8; ++j) sB[(t * 16 + 8 * lh + j) * BWP + lv] = e[j];
        }
        __syncthreads();
        // A operand: row co0 + r, voxels 8g..8g+7; B: column k, same voxels
        const uint4 av = *reinterpret_cast<const uint4*>(sA + r * BWP + 8 * g);
        const bf16x8 av8 = __builtin_bit_cast(bf16x8, av);
        if (blockIdx.x == 0) {
            const u16* e = reinterpret_cast<const u16*>(&av);
#pragma unroll
            for (int j = 0; j < 8; ++j) bsum += bf2f(e[j]);
        }
#pragma unroll
        for (int t = 0; t < BWK; ++t) {
            const uint4 bv = *reinterpret_cast<const uint4*>(sB + (t * 16 + r) * BWP + 8 * g);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av8, __builtin_bit_cast(bf16x8, bv),
                                                            acc[t], 0, 0, 0);
        }
    };
    // two register sets: the loads of the next step are in flight while the
    // current one is transposed and multiplied (the trip count is the same
    // for every wave, so the barriers in process() are uniform)
    Step q0 = load(mb);
    for (long long mc = mb; mc < me; mc += 2 * kBwStep) {
        const Step q1 = load(mc + kBwStep);
        process(q0);
        q0 = load(mc + 2 * kBwStep);
        if (mc + kBwStep < me) process(q1);
    }
    // the four waves' tiles, added in wave order
    __syncthreads();
    f32x4* red = reinterpret_cast<f32x4*>(lds);       // [4][BWK][64]
    float* bred = reinterpret_cast<float*>(red + 4 * BWK * 64);   // [4][64]
#pragma unroll
    for (int t = 0; t < BWK; ++t) red[(wave * BWK + t) * 64 + lane] = acc[t];
    bred[wave * 64 + lane] = bsum;
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int t = 0; t < BWK; ++t)
        acc[t] = ((red[t * 64 + lane] + red[(BWK + t) * 64 + lane]) +
                  red[(2 * BWK + t) * 64 + lane]) + red[(3 * BWK + t) * 64 + lane];
    bsum = ((bred[lane] + bred[64 + lane]) + bred[128 + lane]) + bred[192 + lane];
    // partial layout per chunk: dWt [cout][K], then db [cout]
    float* P = part + (long long)blockIdx.z * D.cout * (D.K + 1);
#pragma unroll
    for (int t = 0; t < BWK; ++t) {
        const int k = (kt0 + t) * 16 + r;
        if (k >= D.K) continue;
        // D: rows co0 + 4g + i, column k
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = co0 + 4 * g + i;
            if (row < D.cout) P[(long long)row * D.K + k] = acc[t][i];
        }
    }
    if (blockIdx.x == 0) {
        // lanes r, r + 16, r + 32, r + 48 hold the four voxel groups of row r
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (g == 0 && co0 + r < D.cout) P[(long long)D.cout * D.K + co0 + r] = bsum;
    }
}

// dWt and db = sums of the chunk partials: a block takes 64 outputs, its 16
// waves sum every 16th chunk, and the 16 sums are added in wave order (a
// fixed order, so the result is repeatable).
constexpr int kRedThreads = 1024;
__global__ void __launch_bounds__(kRedThreads)
k_conv_bwdw_reduce(const float* __restrict__ part, int nchunk, int cout, int K,
                   float* __restrict__ dW, float* __restrict__ db) {
    constexpr int NW = kRedThreads / 64;
    __shared__ float red[kRedThreads];
    const int total = cout * (K + 1);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (i < total)
        for (int c = w; c < nchunk; c += NW) s += part[(long long)c * total + i];
    red[threadIdx.x] = s;
    __syncthreads();
    if (w != 0 || i >= total) return;
    s = red[lane];
    for (int k = 1; k < NW; ++k) s += red[k * 64 + lane];
    if (i < cout * K) {
        dW[i] = s;
    } else if (db) {
        db[i - cout * K] = s;
    }
}

// Wf[ci][tap'*cout + co] = Wt[co][(26 - tap')*cin + ci] (as bf16).
__global__ void __launch_bounds__(kBlock)
k_flip_weights(const float* __restrict__ Wt, int cin, int cout, u16* __restrict__ Wf) {
    const int total = cin * 27 * cout;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= total) return;
    const int ci = i / (27 * cout);
    const int r = i - ci * 27 * cout;
    const int tp = r / cout, co = r - tp * cout;
    Wf[i] = f2bf(Wt[(long long)co * 27 * cin + (26 - tp) * cin + ci]);
}

__global__ void __launch_bounds__(kBlock)
k_cast_bf16(const float* __restrict__ x, u16* __restrict__ y, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        y[i] = f2bf(x[i]);
}

// 2x average pooling of [n][C] -> [(n+1)/2][C] per axis (n even here).
__global__ void __launch_bounds__(kBlock)
k_pool2(const u16* __restrict__ X, int nx, int ny, int nz, int C, int ldx, int xoff,
        u16* __restrict__ Y) {
    const int mx = nx / 2, my = ny / 2, mz = nz / 2;
    const long long total = (long long)mx * my * mz * C;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long v = i / C;
        const int x = (int)(v % mx), y = (int)((v / mx) % my), z = (int)(v / ((long long)mx * my));
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int xx = 2 * x + (q & 1), yy = 2 * y + ((q >> 1) & 1), zz = 2 * z + (q >> 2);
            s += bf2f(X[(((long long)zz * ny + yy) * nx + xx) * ldx + xoff + c]);
        }
        Y[i] = f2bf(0.125f * s);
    }
}

// pool backward: dX[v] (+)= dY[v/2] / 8 (FP32 output, optionally accumulating)
__global__ void __launch_bounds__(kBlock)
k_pool2_bwd(const float* __restrict__ dY, int nx, int ny, int nz, int C, float* __restrict__ dX,
            int ldx, int xoff, int accumulate) {
    const long long total = (long long)nx * ny * nz * C;
    const int mx = nx / 2, my = ny / 2;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long v = i / C;
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
        const float g = 0.125f * dY[(((long long)(z / 2) * my + y / 2) * mx + x / 2) * C + c];
        float* d = dX + v * ldx + xoff + c;
        *d = accumulate ? *d + g : g;
    }
}

// nearest 2x upsampling into a channel slice: Y[v][yoff + c] = X[v/2][c]
__global__ void __launch_bounds__(kBlock)
k_up2(const u16* __restrict__ X, int mx, int my, int mz, int C, u16* __restrict__ Y, int ldy,
      int yoff) {
    const int nx = 2 * mx, ny = 2 * my, nz = 2 * mz;
    const long long total = (long long)nx * ny * nz * C;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long v = i / C;
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
        Y[v * ldy + yoff + c] = X[(((long long)(z / 2) * my + y / 2) * mx + x / 2) * C + c];
    }
}

// up backward: dX[u][c] = sum of the 8 children dY[v][yoff + c] (FP32)
__global__ void __launch_bounds__(kBlock)
k_up2_bwd(const float* __restrict__ dY, int mx, int my, int mz, int C, int ldy, int yoff,
          float* __restrict__ dX) {
    const int nx = 2 * mx, ny = 2 * my;
    const long long total = (long long)mx * my * mz * C;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long u = i / C;
        const int x = (int)(u % mx), y = (int)((u / mx) % my), z = (int)(u / ((long long)mx * my));
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int xx = 2 * x + (q & 1), yy = 2 * y + ((q >> 1) & 1), zz = 2 * z + (q >> 2);
            s += dY[(((long long)zz * ny + yy) * nx + xx) * ldy + yoff + c];
        }
        dX[i] = s;
    }
}

// gradient through LeakyReLU(0.1), using the sign of the stored activation,
// from an FP32 slice dY[v][off + c] (row stride ld) into bf16 [v][C]
__global__ void __launch_bounds__(kBlock)
k_lrelu_bwd(const float* __restrict__ dY, int ld, int off, const u16* __restrict__ Yact,
            int ldyact, int yoff, long long nvox, int C, u16* __restrict__ dX) {
    const long long total = nvox * C;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long v = i / C;
        const float g = dY[v * ld + off + c];
        const float a = bf2f(Yact[v * ldyact + yoff + c]);
        dX[i] = f2bf(a > 0.f ? g : 0.1f * g);
    }
}

// input: (F, M) FP32 [n^3] -> 2x average pooled, 8 channels bf16 (F, M, 0...)
__global__ void __launch_bounds__(kBlock)
k_cnn_input(const float* __restrict__ F, const float* __restrict__ M, int nx, int ny, int nz,
            u16* __restrict__ X) {
    const int mx = nx / 2, my = ny / 2, mz = nz / 2;
    const long long total = (long long)mx * my * mz;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < total;
         v += (long long)gridDim.x * kBlock) {
        const int x = (int)(v % mx), y = (int)((v / mx) % my), z = (int)(v / ((long long)mx * my));
        float sf = 0.f, sm = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const long long s = ((long long)(2 * z + (q >> 2)) * ny + 2 * y + ((q >> 1) & 1)) * nx +
                                2 * x + (q & 1);
            sf += F[s];
            sm += M[s];
        }
        u16* o = X + v * 8;
        o[0] = f2bf(0.125f * sf);
        o[1] = f2bf(0.125f * sm);
#pragma unroll
        for (int c = 2; c < 8; ++c) o[c] = 0;
    }
}

// gradient through pool then LeakyReLU(0.1), in one pass:
// dX[v][c] = bf16(lrelu'(a[v][c]) * (add[v][c] + dY[v/2][c] / 8)), with dY the
// FP32 gradient of the pooled tensor [v/2][C], the optional FP32 slice
// add[v * ldadd + addoff + c] (a second consumer of the activation) and the
// stored activation a = gate[v * ldg + goff + c].
__global__ void __launch_bounds__(kBlock)
k_pool2_lrelu_bwd(const float* __restrict__ dY, int nx, int ny, int nz, int C,
                  const float* __restrict__ add, int ldadd, int addoff,
                  const u16* __restrict__ gate, int ldg, int goff, u16* __restrict__ dX) {
    const long long total = (long long)nx * ny * nz * C;
    const int mx = nx / 2, my = ny / 2;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long v = i / C;
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
        float g = 0.125f * dY[(((long long)(z / 2) * my + y / 2) * mx + x / 2) * C + c];
        if (add) g = add[v * ldadd + addoff + c] + g;
        const float a = bf2f(gate[v * ldg + goff + c]);
        dX[i] = f2bf(a > 0.f ? g : 0.1f * g);
    }
}

// gradient through nearest upsampling then LeakyReLU(0.1):
// dX[u][c] = bf16(lrelu'(a[u][c]) * sum of the 8 children dY[v][yoff + c]),
// dY FP32 at the fine size, a = gate[u * ldg + goff + c] at the coarse size.
__global__ void __launch_bounds__(kBlock)
k_up2_lrelu_bwd(const float* __restrict__ dY, int mx, int my, int mz, int C, int ldy, int yoff,
                const u16* __restrict__ gate, int ldg, int goff, u16* __restrict__ dX) {
    const int nx = 2 * mx, ny = 2 * my;
    const long long total = (long long)mx * my * mz * C;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % C);
        const long long u = i / C;
        const int x = (int)(u % mx), y = (int)((u / mx) % my), z = (int)(u / ((long long)mx * my));
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int xx = 2 * x + (q & 1), yy = 2 * y + ((q >> 1) & 1), zz = 2 * z + (q >> 2);
            s += dY[(((long long)zz * ny + yy) * nx + xx) * ldy + yoff + c];
        }
        const float a = bf2f(gate[u * ldg + goff + c]);
        dX[i] = f2bf(a > 0.f ? s : 0.1f * s);
    }
}

// output map, per volume b of the batch: feature grid g (cells of the
// control spacing) [b][gz][gy][gx][ld] (first 3 channels) -> controls
// theta [b][3][gz+3][gy+3][gx+3] with theta[j] = scale * g[clamp(j - 1, 0,
// g - 1)] per axis (edge replication).
__global__ void __launch_bounds__(kBlock)
k_cnn_output(const float* __restrict__ G, int gx, int gy, int gz, int nb, int ld, float scale,
             float* __restrict__ theta) {
    const int cx = gx + 3, cy = gy + 3, cz = gz + 3;
    const long long per = 3LL * cx * cy * cz;
    const long long total = per * nb;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int b = (int)(i / per);
        const long long ib = i - b * per;
        const int c = (int)(ib / ((long long)cx * cy * cz));
        const long long j = ib - (long long)c * cx * cy * cz;
        const int jx = (int)(j % cx), jy = (int)((j / cx) % cy), jz = (int)(j / ((long long)cx * cy));
        const int x = min(max(jx - 1, 0), gx - 1), y = min(max(jy - 1, 0), gy - 1),
                  z = min(max(jz - 1, 0), gz - 1);
        theta[i] = scale * G[((((long long)b * gz + z) * gy + y) * gx + x) * ld + c];
    }
}

// adjoint of k_cnn_output: dG[b][v][c] = scale * sum of the controls mapped to
// v (channels c < 3; the other ld - 3 channels are zero), as FP32 and/or
// bf16 (either pointer may be null).
__global__ void __launch_bounds__(kBlock)
k_cnn_output_bwd(const float* __restrict__ dtheta, int gx, int gy, int gz, int nb, int ld,
                 float scale, float* __restrict__ dG, u16* __restrict__ dGbf) {
    const int cx = gx + 3, cy = gy + 3, cz = gz + 3;
    const long long vol = (long long)gx * gy * gz;
    const long long total = vol * nb * ld;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const int c = (int)(i % ld);
        const long long vb = i / ld;
        const int b = (int)(vb / vol);
        const long long v = vb - b * vol;
        float s = 0.f;
        if (c < 3) {
            const int x = (int)(v % gx), y = (int)((v / gx) % gy),
                      z = (int)(v / ((long long)gx * gy));
            // controls j with clamp(j - 1) == x: j = x + 1, plus j = 0 at x = 0,
            // plus j in [gx + 1, gx + 2] at x = gx - 1
            int jx0 = x + 1, jx1 = x + 1, jy0 = y + 1, jy1 = y + 1, jz0 = z + 1, jz1 = z + 1;
            if (x == 0) jx0 = 0;
            if (x == gx - 1) jx1 = gx + 2;
            if (y == 0) jy0 = 0;
            if (y == gy - 1) jy1 = gy + 2;
            if (z == 0) jz0 = 0;
            if (z == gz - 1) jz1 = gz + 2;
            const float* T = dtheta + ((long long)b * 3 + c) * cx * cy * cz;
            for (int jz = jz0; jz <= jz1; ++jz)
                for (int jy = jy0; jy <= jy1; ++jy)
                    for (int jx = jx0; jx <= jx1; ++jx)
                        s += T[((long long)jz * cy + jy) * cx + jx];
            s *= scale;
        }
        if (dG) dG[i] = s;
        if (dGbf) dGbf[i] = f2bf(s);
    }
}

__global__ void __launch_bounds__(kBlock)
k_add_f32(float* __restrict__ a, const float* __restrict__ b, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        a[i] += b[i];
}

static int grid1(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 16384 ? b : 16384);
}

static bool a16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace air

using namespace air;

extern "C" {

air_status air_conv3d_fwd(const uint16_t* x, const int32_t dims[3], int32_t batch, int32_t cin,
                          const uint16_t* wt, const float* bias, int32_t cout, int32_t act,
                          const uint16_t* gate, int32_t ldg, int32_t goff, uint16_t* y_bf16,
                          int32_t ldy, int32_t yoff, float* y_f32, int32_t ldyf, void* stream) {
    if (!x || !dims || !wt || (!y_bf16 && !y_f32)) return AIR_ERR_INVALID_ARG;
    if (cin < 8 || cin % 8 || cout < 1 || cout > 128 || act < 0 || act > 2 || batch < 1)
        return AIR_ERR_SHAPE;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return AIR_ERR_SHAPE;
    if (act == 2 && (!gate || goff < 0 || ldg < goff + cout)) return AIR_ERR_INVALID_ARG;
    if (y_bf16 && (ldy < yoff + cout || yoff < 0)) return AIR_ERR_SHAPE;
    if (y_f32 && ldyf < cout) return AIR_ERR_SHAPE;
    if (!a16(x) || !a16(wt)) return AIR_ERR_ALIGN;
    const long long nz = (long long)dims[2] * batch;
    if (nz > (1LL << 30)) return AIR_ERR_SHAPE;
    ConvDims D{dims[0], dims[1], (int)nz, dims[2], cin, cout, 27 * cin, (27 * cin + 31) / 32 * 32};
    ConvEpi E{bias, act, act == 2 ? (const u16*)gate : nullptr, ldg, goff, (u16*)y_bf16, ldy, yoff,
              y_f32, ldyf};
    const long long N = (long long)D.nx * D.ny * D.nz;
    hipStream_t s = (hipStream_t)stream;
    const int nt = (cout + 15) / 16;
    // the most voxels per wave that still give 1024 blocks of four waves;
    // below that, the split-K form keeps the chip busy
    const int mt = N >= 4096LL * 64 ? 4 : N >= 2048LL * 64 ? 2 : N >= 1024LL * 64 ? 1 : 0;
    const long long nblk = mt ? (N + 64LL * mt - 1) / (64LL * mt) : (N + 15) / 16;
    if (nblk > 0x7fffffffLL) return AIR_ERR_SHAPE;
    const dim3 grid((unsigned)nblk), blk(256);
    const u16* X = (const u16*)x;
    const u16* W = (const u16*)wt;
    switch (nt * 8 + mt) {
#define CASE(T)                                                                       \
    case T * 8 + 0: hipLaunchKernelGGL(k_conv_fwd_sk<T>, grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 1: hipLaunchKernelGGL((k_conv_fwd<T, 1>), grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 2: hipLaunchKernelGGL((k_conv_fwd<T, 2>), grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 4: hipLaunchKernelGGL((k_conv_fwd<T, 4>), grid, blk, 0, s, X, D, W, E); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return AIR_ERR_SHAPE;
    }
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

// voxels per partial of the backward-weight GEMM: about one resident round
// of blocks (three 40 KB blocks per CU) over the whole reduction
static long long bwdw_chunk(long long N, int cin, int cout) {
    const int xb = ((27 * cin + 15) / 16 + BWK - 1) / BWK, ct = (cout + 15) / 16;
    long long nbz = 768 / (xb * ct);
    if (nbz < 1) nbz = 1;
    long long c = (N + nbz - 1) / nbz;
    c = (c + kBwStep - 1) / kBwStep * kBwStep;
    return c < kBwStep ? kBwStep : c;
}

air_status air_conv3d_bwd_weight_workspace(const int32_t dims[3], int32_t batch, int32_t cin,
                                           int32_t cout, int32_t chunk, size_t* bytes) {
    if (!dims || !bytes || chunk < 0 || chunk % kBwStep || batch < 1) return AIR_ERR_INVALID_ARG;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || cin < 1 || cout < 1) return AIR_ERR_SHAPE;
    const long long N = (long long)dims[0] * dims[1] * dims[2] * batch;
    const long long c = chunk ? chunk : bwdw_chunk(N, cin, cout);
    const long long nch = (N + c - 1) / c;
    if (nch > 65535) return AIR_ERR_SHAPE;
    *bytes = (size_t)(4LL * nch * cout * (27LL * cin + 1));
    return AIR_OK;
}

air_status air_conv3d_bwd_weight(const uint16_t* x, const int32_t dims[3], int32_t batch,
                                 int32_t cin, const uint16_t* dy, int32_t cout, int32_t chunk,
                                 float* dwt, float* db, void* ws, size_t ws_bytes, void* stream) {
    if (!x || !dims || !dy || !dwt) return AIR_ERR_INVALID_ARG;
    if (cin < 8 || cin % 8 || cout < 8 || cout % 8 || cout > 128) return AIR_ERR_SHAPE;
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(dy)) & 15) return AIR_ERR_ALIGN;
    size_t need = 0;
    air_status st = air_conv3d_bwd_weight_workspace(dims, batch, cin, cout, chunk, &need);
    if (st != AIR_OK) return st;
    if (!ws || ws_bytes < need) return AIR_ERR_WORKSPACE;
    const long long nz = (long long)dims[2] * batch;
    if (nz > (1LL << 30)) return AIR_ERR_SHAPE;
    ConvDims D{dims[0], dims[1], (int)nz, dims[2], cin, cout, 27 * cin, (27 * cin + 31) / 32 * 32};
    const long long N = (long long)D.nx * D.ny * D.nz;
    const long long c = chunk ? chunk : bwdw_chunk(N, cin, cout);
    const int nch = (int)((N + c - 1) / c);
    hipStream_t s = (hipStream_t)stream;
    const int ktiles = (D.K + 15) / 16;
    dim3 grid((ktiles + BWK - 1) / BWK, (cout + 15) / 16, nch);
    hipLaunchKernelGGL(k_conv_bwdw, grid, dim3(256), 0, s, (const u16*)x, D, (const u16*)dy, (int)c,
                       (float*)ws);
    const int total = cout * (D.K + 1);
    hipLaunchKernelGGL(k_conv_bwdw_reduce, dim3((total + 63) / 64), dim3(kRedThreads), 0, s,
                       (const float*)ws, nch, cout, D.K, dwt, db);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_conv3d_flip_weights(const float* wt, int32_t cin, int32_t cout, uint16_t* wf,
                                   void* stream) {
    if (!wt || !wf || cin < 1 || cout < 1) return AIR_ERR_INVALID_ARG;
    const int total = cin * 27 * cout;
    hipLaunchKernelGGL(k_flip_weights, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       (hipStream_t)stream, wt, cin, cout, (u16*)wf);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_cast_bf16(const float* x, uint16_t* y, int64_t n, void* stream) {
    if (!x || !y || n < 0) return AIR_ERR_INVALID_ARG;
    if (n == 0) return AIR_OK;
    hipLaunchKernelGGL(k_cast_bf16, dim3(grid1(n)), dim3(kBlock), 0, (hipStream_t)stream, x, (u16*)y, n);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_pool2(const uint16_t* x, const int32_t dims[3], int32_t c, int32_t ldx,
                     int32_t xoff, uint16_t* y, void* stream) {
    if (!x || !dims || !y || c < 1 || xoff < 0 || ldx < xoff + c) return AIR_ERR_INVALID_ARG;
    if (dims[0] % 2 || dims[1] % 2 || dims[2] % 2) return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] / 8 * c;
    hipLaunchKernelGGL(k_pool2, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, (const u16*)x,
                       dims[0], dims[1], dims[2], c, ldx, xoff, (u16*)y);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_pool2_bwd(const float* dy, const int32_t dims[3], int32_t c, float* dx,
                         int32_t ldx, int32_t xoff, int32_t accumulate, void* stream) {
    if (!dy || !dims || !dx || c < 1 || xoff < 0 || ldx < xoff + c) return AIR_ERR_INVALID_ARG;
    if (dims[0] % 2 || dims[1] % 2 || dims[2] % 2) return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] * c;
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, dy,
                       dims[0], dims[1], dims[2], c, dx, ldx, xoff, accumulate);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_up2(const uint16_t* x, const int32_t dims[3], int32_t c, uint16_t* y, int32_t ldy,
                   int32_t yoff, void* stream) {
    if (!x || !dims || !y || c < 1 || ldy < yoff + c) return AIR_ERR_INVALID_ARG;
    const long long t = 8LL * dims[0] * dims[1] * dims[2] * c;
    hipLaunchKernelGGL(k_up2, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, (const u16*)x,
                       dims[0], dims[1], dims[2], c, (u16*)y, ldy, yoff);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_up2_bwd(const float* dy, const int32_t dims[3], int32_t c, int32_t ldy,
                       int32_t yoff, float* dx, void* stream) {
    if (!dy || !dims || !dx || c < 1 || ldy < yoff + c) return AIR_ERR_INVALID_ARG;
    const long long t = (long long)dims[0] * dims[1] * dims[2] * c;
    hipLaunchKernelGGL(k_up2_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, dy,
                       dims[0], dims[1], dims[2], c, ldy, yoff, dx);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_lrelu_bwd(const float* dy, int32_t ld, int32_t off, const uint16_t* yact,
                         int32_t ldyact, int32_t yoff, int64_t nvox, int32_t c, uint16_t* dx,
                         void* stream) {
    if (!dy || !yact || !dx || c < 1 || nvox < 0) return AIR_ERR_INVALID_ARG;
    if (ld < off + c || ldyact < yoff + c) return AIR_ERR_SHAPE;
    hipLaunchKernelGGL(k_lrelu_bwd, dim3(grid1(nvox * c)), dim3(kBlock), 0, (hipStream_t)stream, dy,
                       ld, off, (const u16*)yact, ldyact, yoff, nvox, c, (u16*)dx);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_pool2_lrelu_bwd(const float* dy, const int32_t dims[3], int32_t c,
                              const float* add, int32_t ldadd, int32_t addoff,
                              const uint16_t* gate, int32_t ldg, int32_t goff, uint16_t* dx,
                              void* stream) {
    if (!dy || !dims || !gate || !dx || c < 1 || goff < 0 || ldg < goff + c)
        return AIR_ERR_INVALID_ARG;
    if (add && (addoff < 0 || ldadd < addoff + c)) return AIR_ERR_INVALID_ARG;
    if (dims[0] < 2 || dims[1] < 2 || dims[2] < 2 || dims[0] % 2 || dims[1] % 2 || dims[2] % 2)
        return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] * c;
    hipLaunchKernelGGL(k_pool2_lrelu_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, dy,
                       dims[0], dims[1], dims[2], c, add, ldadd, addoff, (const u16*)gate, ldg, goff,
                       (u16*)dx);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_up2_lrelu_bwd(const float* dy, const int32_t dims[3], int32_t c, int32_t ldy,
                             int32_t yoff, const uint16_t* gate, int32_t ldg, int32_t goff,
                             uint16_t* dx, void* stream) {
    if (!dy || !dims || !gate || !dx || c < 1 || yoff < 0 || ldy < yoff + c || goff < 0 ||
        ldg < goff + c)
        return AIR_ERR_INVALID_ARG;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] * c;
    hipLaunchKernelGGL(k_up2_lrelu_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, dy,
                       dims[0], dims[1], dims[2], c, ldy, yoff, (const u16*)gate, ldg, goff,
                       (u16*)dx);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_cnn_input(const float* fixed, const float* moving, const int32_t dims[3],
                         uint16_t* x, void* stream) {
    if (!fixed || !moving || !dims || !x) return AIR_ERR_INVALID_ARG;
    if (dims[0] % 2 || dims[1] % 2 || dims[2] % 2) return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] / 8;
    hipLaunchKernelGGL(k_cnn_input, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, fixed,
                       moving, dims[0], dims[1], dims[2], (u16*)x);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_cnn_output(const float* g, const int32_t gdims[3], int32_t batch, int32_t ld,
                          float scale, float* theta, void* stream) {
    if (!g || !gdims || !theta || ld < 3 || batch < 1) return AIR_ERR_INVALID_ARG;
    if (gdims[0] < 1 || gdims[1] < 1 || gdims[2] < 1) return AIR_ERR_SHAPE;
    const long long t = 3LL * (gdims[0] + 3) * (gdims[1] + 3) * (gdims[2] + 3) * batch;
    hipLaunchKernelGGL(k_cnn_output, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream, g,
                       gdims[0], gdims[1], gdims[2], (int)batch, ld, scale, theta);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_cnn_output_bwd(const float* dtheta, const int32_t gdims[3], int32_t batch,
                              int32_t ld, float scale, float* dg, uint16_t* dg_bf16,
                              void* stream) {
    if (!dtheta || !gdims || (!dg && !dg_bf16) || ld < 3 || batch < 1) return AIR_ERR_INVALID_ARG;
    if (gdims[0] < 1 || gdims[1] < 1 || gdims[2] < 1) return AIR_ERR_SHAPE;
    const long long t = (long long)gdims[0] * gdims[1] * gdims[2] * ld * batch;
    hipLaunchKernelGGL(k_cnn_output_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream,
                       dtheta, gdims[0], gdims[1], gdims[2], (int)batch, ld, scale, dg,
                       (u16*)dg_bf16);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_add_f32(float* a, const float* b, int64_t n, void* stream) {
    if (!a || !b || n < 0) return AIR_ERR_INVALID_ARG;
    if (n == 0) return AIR_OK;
    hipLaunchKernelGGL(k_add_f32, dim3(grid1(n)), dim3(kBlock), 0, (hipStream_t)stream, a, b, n);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

}  // extern "C"
