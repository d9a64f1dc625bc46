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

// 8 bf16 values of a 16-byte vector <-> FP32
__device__ inline void unpack8(uint4 q, float* f) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f[2 * j] = __uint_as_float(w[j] << 16);
        f[2 * j + 1] = __uint_as_float(w[j] & 0xffff0000u);
    }
}

__device__ inline uint4 pack8(const float* f) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        w[j] = (uint32_t)f2bf(f[2 * j]) | ((uint32_t)f2bf(f[2 * j + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ inline void load8f(const float* p, float* f) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
    f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
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

// Epilogue of the brick forms through LDS: the wave's 4 x 16 output voxels
// x 16 NT16 channels, with bias (and act 1) applied, are staged as FP32 rows
// of kEpiPitch(NT16) floats, then every lane writes whole 8-channel vectors
// (16 bytes of bf16 and/or 32 bytes of FP32; act 2 multiplies by the
// activation slopes read as 16-byte gate vectors). Needs ldy, yoff, ldyf,
// ldg, goff multiples of 8 and 16-byte aligned outputs (checked by the host).
__host__ __device__ constexpr int kEpiPitch(int nt16) { return nt16 * 16 + 4; }

template <int NT16>
__device__ inline void brick_epilogue(const ConvEpi& E, const ConvDims& D, const f32x4 (&acc)[4][NT16],
                                      float* stage, long long row0, int lane) {
    constexpr int CP = kEpiPitch(NT16);
    const int g = lane >> 4, r = lane & 15;
#pragma unroll
    for (int j = 0; j < NT16; ++j) {
        const int co = j * 16 + r;
        const float b = (co < D.cout && E.bias) ? E.bias[co] : 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[t][j][i] + b;
                if (E.act == 1) v = v > 0.f ? v : 0.1f * v;
                stage[(t * 16 + 4 * g + i) * CP + co] = v;   // voxel (row t, x 4g + i)
            }
    }
    __syncthreads();   // every thread of the block calls this
    const int C8 = (D.cout + 7) / 8;
    for (int it = lane; it < 64 * C8; it += 64) {
        const int lv = it / C8, c8 = it - lv * C8;
        if (8 * c8 >= D.cout) continue;
        const long long row = row0 + (long long)(lv >> 4) * D.nx + (lv & 15);
        float v[8];
        const float4 lo = *reinterpret_cast<const float4*>(stage + lv * CP + 8 * c8);
        const float4 hi = *reinterpret_cast<const float4*>(stage + lv * CP + 8 * c8 + 4);
        v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
        v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
        if (E.act == 2) {
            float a[8];
            unpack8(*reinterpret_cast<const uint4*>(E.gate + row * E.ldg + E.goff + 8 * c8), a);
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = a[k] > 0.f ? v[k] : 0.1f * v[k];
        }
        if (E.ybf)
            *reinterpret_cast<uint4*>(E.ybf + row * E.ldy + E.yoff + 8 * c8) = pack8(v);
        if (E.yf) {
            float* o = E.yf + row * E.ldyf + 8 * c8;
            *reinterpret_cast<float4*>(o) = make_float4(v[0], v[1], v[2], v[3]);
            *reinterpret_cast<float4*>(o + 4) = make_float4(v[4], v[5], v[6], v[7]);
        }
    }
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
        AIR_CHECK(v >= 0 && v < (long long)D.nx * D.ny * D.nz && ci >= 0 && ci + 8 <= D.cin,
                  kDbgConvInput);
        q = *reinterpret_cast<const uint4*>(X + v * D.cin + ci);
    }
    return __builtin_bit_cast(bf16x8, q);
}

__device__ inline bf16x8 load_w(const u16* __restrict__ Wt, const ConvDims& D, int co, int k) {
    uint4 q = make_uint4(0, 0, 0, 0);
    AIR_CHECK(co >= D.cout || k >= D.K || (co >= 0 && k >= 0 && k + 8 <= D.K), kDbgConvInput);
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

// Brick form: a block computes 16 x 4 x 4 output voxels (x, y, z; whole
// bricks only) from an input tile with a one-voxel halo, 18 x 6 x 6 voxels,
// staged in LDS one slice of CS channels at a time (channel-last, so an
// MFMA operand, 8 channels of one tap, is one aligned 16-byte LDS read).
// Wave w takes the plane z0 + w and four 16-voxel rows y0 .. y0 + 3 of it;
// within a slice the reduction runs over kk = tap * CS + c, and its global
// column is k = tap * cin + slice * CS + c (weights read from global memory
// / cache). Each input voxel is fetched from global memory once per slice
// instead of once per tap.
constexpr int kBrX = 16, kBrY = 4, kBrZ = 4;
constexpr int kHaX = kBrX + 2, kHaY = kBrY + 2, kHaZ = kBrZ + 2;
template <int NT16, int CS>
__global__ void __launch_bounds__(256)
k_conv_fwd_brick(const u16* __restrict__ X, ConvDims D, const u16* __restrict__ Wt, ConvEpi E) {
    // the input tile, and afterwards the four waves' epilogue stages
    constexpr int kTileBytes = kHaZ * kHaY * kHaX * CS * 2;
    constexpr int kEpiBytes = 4 * 64 * kEpiPitch(NT16) * 4;
    __shared__ __align__(16) unsigned char lds[kTileBytes > kEpiBytes ? kTileBytes : kEpiBytes];
    u16* tile = reinterpret_cast<u16*>(lds);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    // brick coordinates: x fastest, then y, then z within the volume, then volume
    const int bx = D.nx / kBrX, by = D.ny / kBrY, bzv = D.nzv / kBrZ;
    int b = blockIdx.x;
    const int x0 = (b % bx) * kBrX; b /= bx;
    const int y0 = (b % by) * kBrY; b /= by;
    const int zb = (b % bzv) * kBrZ, vol = b / bzv;
    const int zv0 = vol * D.nzv;   // first plane of the volume in the stack
    constexpr int KK = 27 * CS, KKpad = (KK + 31) / 32 * 32, V8 = CS / 8;
    f32x4 acc[kBrY][NT16];
#pragma unroll
    for (int t = 0; t < kBrY; ++t)
#pragma unroll
        for (int j = 0; j < NT16; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ci0 = 0; ci0 < D.cin; ci0 += CS) {
        __syncthreads();   // the previous slice's reads are done
        for (int i = threadIdx.x; i < kHaZ * kHaY * kHaX * V8; i += 256) {
            const int c8 = i % V8, v = i / V8;
            const int hx = v % kHaX, hy = (v / kHaX) % kHaY, hz = v / (kHaX * kHaY);
            const int x = x0 + hx - 1, y = y0 + hy - 1, zl = zb + hz - 1;
            uint4 q = make_uint4(0, 0, 0, 0);
            if ((unsigned)x < (unsigned)D.nx && (unsigned)y < (unsigned)D.ny &&
                (unsigned)zl < (unsigned)D.nzv) {
                AIR_CHECK(zv0 + zl < D.nz && ci0 + 8 * c8 + 8 <= D.cin, kDbgConvInput);
                q = *reinterpret_cast<const uint4*>(
                    X + (((long long)(zv0 + zl) * D.ny + y) * D.nx + x) * D.cin + ci0 + 8 * c8);
            }
            *reinterpret_cast<uint4*>(tile + v * CS + 8 * c8) = q;
        }
        __syncthreads();
        for (int kc = 0; kc < KKpad; kc += 32) {
            const int kk = kc + 8 * g;
            const int tap = kk / CS, c = kk - tap * CS;
            const bool kin = kk < KK;
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // halo offsets
            bf16x8 a[kBrY];
#pragma unroll
            for (int t = 0; t < kBrY; ++t) {
                uint4 q = make_uint4(0, 0, 0, 0);
                if (kin)
                    q = *reinterpret_cast<const uint4*>(
                        tile + (((wave + dz) * kHaY + t + dy) * kHaX + r + dx) * CS + c);
                a[t] = __builtin_bit_cast(bf16x8, q);
            }
            const int k = tap * D.cin + ci0 + c;
#pragma unroll
            for (int j = 0; j < NT16; ++j) {
                const bf16x8 bw = kin ? load_w(Wt, D, j * 16 + r, k)
                                      : __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
#pragma unroll
                for (int t = 0; t < kBrY; ++t)
                    acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bw, acc[t][j], 0, 0, 0);
            }
        }
    }
    __syncthreads();   // every wave is done with the tile
    // D rows 4g + i of tile t: voxel x0 + 4g + i of row (y0 + t, plane zb + wave)
    brick_epilogue<NT16>(E, D, acc,
                         reinterpret_cast<float*>(lds) + wave * 64 * kEpiPitch(NT16),
                         ((long long)(zv0 + zb + wave) * D.ny + y0) * D.nx + x0, lane);
}

// Brick form for an input whose channels 2.. are zero (the network's first
// layer: fixed and moving image, six zero pads): only channels 0 and 1 are
// staged (4 bytes per voxel) and the reduction runs over kk = tap * 2 + c,
// 54 columns in two 32-wide steps instead of 216 in seven; an operand's 8
// columns are 4 taps x 2 channels (four 4-byte LDS reads), the weights'
// the matching 4 x 2 entries of Wt[co][tap * cin + c]. The zero channels'
// products are exact zeros, so the sum is the full convolution's.
template <int NT16>
__global__ void __launch_bounds__(256)
k_conv_fwd_brick_in2(const u16* __restrict__ X, ConvDims D, const u16* __restrict__ Wt,
                     ConvEpi E) {
    // the input tile (c0, c1) per voxel, then the waves' epilogue stages
    constexpr int kEpiBytes = 4 * 64 * kEpiPitch(NT16) * 4;
    __shared__ __align__(16) unsigned char lds[kEpiBytes > kHaZ * kHaY * kHaX * 4
                                                   ? kEpiBytes : kHaZ * kHaY * kHaX * 4];
    uint32_t* tile = reinterpret_cast<uint32_t*>(lds);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int bx = D.nx / kBrX, by = D.ny / kBrY, bzv = D.nzv / kBrZ;
    int b = blockIdx.x;
    const int x0 = (b % bx) * kBrX; b /= bx;
    const int y0 = (b % by) * kBrY; b /= by;
    const int zb = (b % bzv) * kBrZ, vol = b / bzv;
    const int zv0 = vol * D.nzv;
    for (int i = threadIdx.x; i < kHaZ * kHaY * kHaX; i += 256) {
        const int hx = i % kHaX, hy = (i / kHaX) % kHaY, hz = i / (kHaX * kHaY);
        const int x = x0 + hx - 1, y = y0 + hy - 1, zl = zb + hz - 1;
        uint32_t q = 0;
        if ((unsigned)x < (unsigned)D.nx && (unsigned)y < (unsigned)D.ny &&
            (unsigned)zl < (unsigned)D.nzv) {
            AIR_CHECK(zv0 + zl < D.nz, kDbgConvInput);
            q = *reinterpret_cast<const uint32_t*>(
                X + (((long long)(zv0 + zl) * D.ny + y) * D.nx + x) * D.cin);
        }
        tile[i] = q;
    }
    __syncthreads();
    f32x4 acc[kBrY][NT16];
#pragma unroll
    for (int t = 0; t < kBrY; ++t)
#pragma unroll
        for (int j = 0; j < NT16; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 64; kc += 32) {
        // this lane group's taps t0 .. t0 + 3 (27 and beyond: zero columns)
        const int t0 = (kc + 8 * g) / 2;
        bf16x8 a[kBrY];
#pragma unroll
        for (int t = 0; t < kBrY; ++t) {
            uint32_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tap = t0 + i;
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // halo offsets
                w[i] = tap < 27 ? tile[((wave + dz) * kHaY + t + dy) * kHaX + r + dx] : 0u;
            }
            a[t] = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
        }
#pragma unroll
        for (int j = 0; j < NT16; ++j) {
            const int co = j * 16 + r;
            uint32_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tap = t0 + i;
                w[i] = (co < D.cout && tap < 27)
                           ? *reinterpret_cast<const uint32_t*>(Wt + (long long)co * D.K + tap * D.cin)
                           : 0u;
            }
            const bf16x8 bw = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
#pragma unroll
            for (int t = 0; t < kBrY; ++t)
                acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bw, acc[t][j], 0, 0, 0);
        }
    }
    __syncthreads();   // every wave is done with the tile
    brick_epilogue<NT16>(E, D, acc,
                         reinterpret_cast<float*>(lds) + wave * 64 * kEpiPitch(NT16),
                         ((long long)(zv0 + zb + wave) * D.ny + y0) * D.nx + x0, lane);
}

// Split-K form for small volumes (too few blocks of the forms above to
// fill the chip): a block takes MT tiles of 16 voxels, its four waves take
// every fourth 32-wide reduction step (each weight operand a wave loads
// feeds MT products), and the four partial tiles are added in wave order
// through LDS, one voxel tile at a time, before the same epilogue.
template <int NT16, int MT>
__global__ void __launch_bounds__(256)
k_conv_fwd_sk(const u16* __restrict__ X, ConvDims D, const u16* __restrict__ Wt, ConvEpi E) {
    __shared__ f32x4 red[4][NT16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long N = (long long)D.nx * D.ny * D.nz;
    const long long m0 = (long long)blockIdx.x * 16 * MT;
    const int g = lane >> 4;
    Vox p[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) p[t] = vox_of(m0 + 16 * t + (lane & 15), D, N);
    f32x4 acc[MT][NT16];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int j = 0; j < NT16; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 32 * wave; kc < D.Kpad; kc += 128) {
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
    for (int t = 0; t < MT; ++t) {
        if (t) __syncthreads();   // the previous tile's reads are done
#pragma unroll
        for (int j = 0; j < NT16; ++j) red[wave][j][lane] = acc[t][j];
        __syncthreads();
        for (int j = wave; j < NT16; j += 4) {
            const f32x4 v = ((red[0][j][lane] + red[1][j][lane]) + red[2][j][lane]) + red[3][j][lane];
            const int co = j * 16 + (lane & 15);
            if (co >= D.cout) continue;
            const float b = E.bias ? E.bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long row = m0 + 16 * t + 4 * g + i;
                if (row < N) conv_store(E, row, co, v[i], b);
            }
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

// ---- Backward-weight on x-blocked operands (nx a multiple of 8).
// The GEMM reduces over voxels, so each MFMA lane needs 8 consecutive voxels
// of one channel, while activations are stored channel-last. The operands
// are first rewritten once in the x-blocked layout XB[b][c][8]: block b =
// (z * ny + y) * nx/8 + x/8 holds, per channel c, the 8 voxels x = 8 (x/8)
// .. + 7 in one 16-byte vector. A tap's input vector is then one load at the
// block shifted by (dy, dz); a tap with dx = +-1 takes one more dword from
// the neighbouring block and a funnel shift by one element (v_alignbyte).

// XB[b][c][j] = X[voxel 8b + j][c] for c < C (8x8 transposes in registers),
// for two tensors with the same voxels in one launch: items [0, nblk C0/8)
// transpose X0 (C0 channels), the rest X1 (C1 channels)
__global__ void __launch_bounds__(kBlock)
k_to_xb(const u16* __restrict__ X0, int C0, u16* __restrict__ XB0, const u16* __restrict__ X1,
        int C1, u16* __restrict__ XB1, long long nblk) {
    const long long n0 = nblk * (C0 / 8);
    const long long total = n0 + nblk * (C1 / 8);
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const bool second = i >= n0;
        const u16* X = second ? X1 : X0;
        u16* XB = second ? XB1 : XB0;
        const int C = second ? C1 : C0, ld = C, off = 0;
        const long long k = second ? i - n0 : i;
        const int C8 = C / 8;
        const int cg = (int)(k % C8);
        const long long b = k / C8;
        uint32_t w[8][4];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint4 q = *reinterpret_cast<const uint4*>(X + (b * 8 + j) * ld + off + 8 * cg);
            w[j][0] = q.x; w[j][1] = q.y; w[j][2] = q.z; w[j][3] = q.w;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            // channel c of voxels 2k, 2k+1: the low (c even) or high halves of dword c/2
            const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;
            uint4 o;
            o.x = __builtin_amdgcn_perm(w[1][c / 2], w[0][c / 2], sel);
            o.y = __builtin_amdgcn_perm(w[3][c / 2], w[2][c / 2], sel);
            o.z = __builtin_amdgcn_perm(w[5][c / 2], w[4][c / 2], sel);
            o.w = __builtin_amdgcn_perm(w[7][c / 2], w[6][c / 2], sel);
            *reinterpret_cast<uint4*>(XB + (b * C + 8 * cg + c) * 8) = o;
        }
    }
}

// dWt partial of voxel chunk `blockIdx.z` from x-blocked X and dY: the
// block's four waves take 32 voxels (4 x-blocks) of every 128-voxel step;
// a wave accumulates BWK k-tiles of 16 reduction columns against CT tiles of
// 16 output channels, every A operand (dY) feeding BWK products and every
// B operand (X) CT. The wave sums are added in wave order through LDS into
// one partial per chunk, as in k_conv_bwdw.
template <int CT>
__global__ void __launch_bounds__(256)
k_conv_bwdw_xb(const u16* __restrict__ XB, ConvDims D, int cu, const u16* __restrict__ dYB,
               int chunk, float* __restrict__ part) {
    __shared__ f32x4 red[4][CT][64];
    __shared__ float bred[4][CT][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int kt0 = blockIdx.x * BWK;
    const int nxb = D.nx / 8;
    const long long N = (long long)D.nx * D.ny * D.nz;
    const long long mb = (long long)blockIdx.z * chunk;
    const long long me = mb + chunk < N ? mb + chunk : N;
    const long long C8in = (long long)D.cin * 8, C8out = (long long)D.cout * 8;
    // computed columns: k = tap * cu + ci over the first cu input channels
    // (the others are known to be zero)
    const int Ku = 27 * cu;
    // this lane's B column of each k tile: element offset of the tap's
    // block and channel from the lane's own block, and the packed tap
    // (dx + 1) | (dy + 1) << 2 | (dz + 1) << 4, or -1 past the last column
    int toff[BWK], tcode[BWK];
#pragma unroll
    for (int t = 0; t < BWK; ++t) {
        const int k = (kt0 + t) * 16 + r;
        const int tap = k < Ku ? k / cu : 13;
        const int ci = k < Ku ? k - tap * cu : 0;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        toff[t] = ((dz * D.ny + dy) * nxb) * (int)C8in + ci * 8;
        tcode[t] = k < Ku ? (dx + 1) | (dy + 1) << 2 | (dz + 1) << 4 : -1;
    }
    f32x4 acc[BWK][CT];
#pragma unroll
    for (int t = 0; t < BWK; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) bsum[c] = 0.f;

    for (long long mc = mb + 32 * wave; mc < me; mc += kBwStep) {
        const long long blk = mc / 8 + g;     // this lane group's x-block
        const bool ok = blk * 8 < me;
        const int xb = (int)(blk % nxb);
        const long long row = blk / nxb;
        const int y = (int)(row % D.ny);
        const int zl = (int)((row / D.ny) % D.nzv);
        uint4 qa[CT], qv[BWK];
        uint32_t qn[BWK];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int co = 16 * c + r;
            qa[c] = make_uint4(0, 0, 0, 0);
            if (ok && co < D.cout) {
                AIR_CHECK(blk * C8out + (long long)co * 8 + 8 <= N * D.cout, kDbgConvWgrad);
                qa[c] = *reinterpret_cast<const uint4*>(dYB + blk * C8out + (long long)co * 8);
            }
        }
#pragma unroll
        for (int t = 0; t < BWK; ++t) {
            qv[t] = make_uint4(0, 0, 0, 0);
            qn[t] = 0;
            const int dx = (tcode[t] & 3) - 1, dy = ((tcode[t] >> 2) & 3) - 1,
                      dz = ((tcode[t] >> 4) & 3) - 1;
            const bool in = ok && tcode[t] >= 0 && (unsigned)(y + dy) < (unsigned)D.ny &&
                            (unsigned)(zl + dz) < (unsigned)D.nzv;
            if (in) {
                const u16* p = XB + blk * C8in + toff[t];
                AIR_CHECK(blk * C8in + toff[t] >= 0 && blk * C8in + toff[t] + 8 <= N * D.cin,
                          kDbgConvWgrad);
                qv[t] = *reinterpret_cast<const uint4*>(p);
                // dx = +1: element 0 of the next block; dx = -1: element 7 of
                // the previous one (the high half of its last dword)
                if (dx != 0 && (unsigned)(xb + dx) < (unsigned)nxb) {
                    AIR_CHECK(blk * C8in + toff[t] + dx * C8in + (dx > 0 ? 0 : 6) >= 0 &&
                                  blk * C8in + toff[t] + dx * C8in + 8 <= N * D.cin,
                              kDbgConvWgrad);
                    qn[t] = *reinterpret_cast<const uint32_t*>(p + dx * (int)C8in + (dx > 0 ? 0 : 6));
                }
            }
        }
        bf16x8 a[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            a[c] = __builtin_bit_cast(bf16x8, qa[c]);
            if (blockIdx.x == 0) {
                float f[8];
                unpack8(qa[c], f);
#pragma unroll
                for (int j = 0; j < 8; ++j) bsum[c] += f[j];
            }
        }
#pragma unroll
        for (int t = 0; t < BWK; ++t) {
            const uint32_t v[4] = {qv[t].x, qv[t].y, qv[t].z, qv[t].w};
            const int dx = (tcode[t] & 3) - 1;
            const bool up = dx > 0, dn = dx < 0;
            const uint32_t sh = dx != 0 ? 2u : 0u;
            uint32_t w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // element j of the result = element j + dx of the 8-voxel window
                const uint32_t hi = up ? (k < 3 ? v[k + 1] : qn[t]) : v[k];
                const uint32_t lo = dn ? (k > 0 ? v[k - 1] : qn[t]) : v[k];
                w[k] = __builtin_amdgcn_alignbyte(hi, lo, sh);
            }
            const bf16x8 b = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
#pragma unroll
            for (int c = 0; c < CT; ++c)
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b, acc[t][c], 0, 0, 0);
        }
    }
    // the four waves' tiles, added in wave order, one k tile at a time;
    // partial layout per chunk: [cout][Ku] over the computed columns, then db
    float* P = part + (long long)blockIdx.z * D.cout * (Ku + 1);
#pragma unroll
    for (int t = 0; t < BWK; ++t) {
        __syncthreads();   // the previous tile's reads are done
#pragma unroll
        for (int c = 0; c < CT; ++c) red[wave][c][lane] = acc[t][c];
        __syncthreads();
        const int k = (kt0 + t) * 16 + r;
        if (wave != 0 || k >= Ku) continue;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const f32x4 v = ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * c + 4 * g + i;
                if (row < D.cout) P[(long long)row * Ku + k] = v[i];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) bred[wave][c][lane] = bsum[c];
    __syncthreads();
    if (wave != 0) return;
    if (blockIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            float b = ((bred[0][c][lane] + bred[1][c][lane]) + bred[2][c][lane]) + bred[3][c][lane];
            // lanes r, r + 16, r + 32, r + 48 hold the four voxel groups of row r
            b += __shfl_xor(b, 16, 64);
            b += __shfl_xor(b, 32, 64);
            if (g == 0 && 16 * c + r < D.cout) P[(long long)D.cout * Ku + 16 * c + r] = b;
        }
    }
}

// dWt and db = sums of the chunk partials: a block takes 64 outputs, its 16
// waves sum every 16th chunk, and the 16 sums are added in wave order (a
// fixed order, so the result is repeatable). The partials hold the columns
// k = tap * cu + ci of the first cu input channels (cu = cin: all); the
// columns of the other channels are written as zero.
constexpr int kRedThreads = 1024;
__global__ void __launch_bounds__(kRedThreads)
k_conv_bwdw_reduce(const float* __restrict__ part, int nchunk, int cout, int cin, int cu,
                   float* __restrict__ dW, float* __restrict__ db) {
    constexpr int NW = kRedThreads / 64;
    __shared__ float red[kRedThreads];
    const int K = 27 * cin, Ku = 27 * cu;
    const int total = cout * (K + 1), ptotal = cout * (Ku + 1);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    // the partial column of output i, or -1 for a known-zero channel
    int src = -1;
    if (i < cout * K) {
        const int co = i / K, k = i - co * K, tap = k / cin, ci = k - tap * cin;
        if (ci < cu) src = co * Ku + tap * cu + ci;
    } else if (i < total) {
        src = cout * Ku + (i - cout * K);
    }
    float s = 0.f;
    if (src >= 0)
        for (int c = w; c < nchunk; c += NW) s += part[(long long)c * ptotal + src];
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

// ---- 8-channel forms of the pooling, upsampling and activation-adjoint
// kernels: one thread moves one 16-byte bf16 vector (or two float4) per
// voxel, for channel counts, row strides and offsets that are multiples of 8
// and 16-byte aligned tensors. Per channel they do the same FP32 operations
// in the same order as the kernels above, so the results are identical.

__global__ void __launch_bounds__(kBlock)
k_pool2_v8(const u16* __restrict__ X, int nx, int ny, int nz, int C, int ldx, int xoff,
           u16* __restrict__ Y) {
    const int mx = nx / 2, my = ny / 2, mz = nz / 2, C8 = C / 8;
    const int total = mx * my * mz * C8;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        const int cg = i % C8, v = i / C8;
        const int x = v % mx, y = (v / mx) % my, z = v / (mx * my);
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int xx = 2 * x + (q & 1), yy = 2 * y + ((q >> 1) & 1), zz = 2 * z + (q >> 2);
            float f[8];
            unpack8(*reinterpret_cast<const uint4*>(
                        X + ((long long)(zz * ny + yy) * nx + xx) * ldx + xoff + 8 * cg), f);
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j] += f[j];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] = 0.125f * s[j];
        *reinterpret_cast<uint4*>(Y + (long long)v * C + 8 * cg) = pack8(s);
    }
}

__global__ void __launch_bounds__(kBlock)
k_up2_v8(const u16* __restrict__ X, int mx, int my, int mz, int C, u16* __restrict__ Y, int ldy,
         int yoff) {
    const int nx = 2 * mx, ny = 2 * my, C8 = C / 8;
    const int total = mx * my * mz * C8;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        const int cg = i % C8, u = i / C8;
        const int x = u % mx, y = (u / mx) % my, z = u / (mx * my);
        const uint4 q = *reinterpret_cast<const uint4*>(X + (long long)u * C + 8 * cg);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int xx = 2 * x + (k & 1), yy = 2 * y + ((k >> 1) & 1), zz = 2 * z + (k >> 2);
            *reinterpret_cast<uint4*>(Y + ((long long)(zz * ny + yy) * nx + xx) * ldy + yoff +
                                      8 * cg) = q;
        }
    }
}

__global__ void __launch_bounds__(kBlock)
k_pool2_lrelu_bwd_v8(const float* __restrict__ dY, int nx, int ny, int nz, int C,
                     const float* __restrict__ add, int ldadd, int addoff,
                     const u16* __restrict__ gate, int ldg, int goff, u16* __restrict__ dX) {
    const int mx = nx / 2, my = ny / 2, C8 = C / 8;
    const int total = nx * ny * nz * C8;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        const int cg = i % C8, v = i / C8;
        const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
        float g[8], a[8];
        load8f(dY + ((long long)((z / 2) * my + y / 2) * mx + x / 2) * C + 8 * cg, g);
#pragma unroll
        for (int j = 0; j < 8; ++j) g[j] = 0.125f * g[j];
        if (add) {
            float t[8];
            load8f(add + (long long)v * ldadd + addoff + 8 * cg, t);
#pragma unroll
            for (int j = 0; j < 8; ++j) g[j] = t[j] + g[j];
        }
        unpack8(*reinterpret_cast<const uint4*>(gate + (long long)v * ldg + goff + 8 * cg), a);
#pragma unroll
        for (int j = 0; j < 8; ++j) g[j] = a[j] > 0.f ? g[j] : 0.1f * g[j];
        *reinterpret_cast<uint4*>(dX + (long long)v * C + 8 * cg) = pack8(g);
    }
}

__global__ void __launch_bounds__(kBlock)
k_up2_lrelu_bwd_v8(const float* __restrict__ dY, int mx, int my, int mz, int C, int ldy,
                   int yoff, const u16* __restrict__ gate, int ldg, int goff,
                   u16* __restrict__ dX) {
    const int nx = 2 * mx, ny = 2 * my, C8 = C / 8;
    const int total = mx * my * mz * C8;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        const int cg = i % C8, u = i / C8;
        const int x = u % mx, y = (u / mx) % my, z = u / (mx * my);
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, a[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int xx = 2 * x + (q & 1), yy = 2 * y + ((q >> 1) & 1), zz = 2 * z + (q >> 2);
            float f[8];
            load8f(dY + ((long long)(zz * ny + yy) * nx + xx) * ldy + yoff + 8 * cg, f);
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j] += f[j];
        }
        unpack8(*reinterpret_cast<const uint4*>(gate + (long long)u * ldg + goff + 8 * cg), a);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] = a[j] > 0.f ? s[j] : 0.1f * s[j];
        *reinterpret_cast<uint4*>(dX + (long long)u * C + 8 * cg) = pack8(s);
    }
}

// the network input with its x-blocked copy (mx a multiple of 8): one
// thread per pooled voxel, the same sums as k_cnn_input; the 8 lanes of an
// x-block (8 consecutive voxels, 8 consecutive lanes) trade their bf16
// (F, M) pairs so that lane 0 writes the block's F vector, lane 1 its M
// vector and lanes 2..7 the zero channels
__global__ void __launch_bounds__(kBlock)
k_cnn_input_xb(const float* __restrict__ F, const float* __restrict__ M, int nx, int ny, int nz,
               u16* __restrict__ X, u16* __restrict__ XB) {
    const int mx = nx / 2, my = ny / 2, mz = nz / 2;
    const long long total = (long long)mx * my * mz;
    const int lane = threadIdx.x & 63, j = lane & 7;
    // whole waves run every iteration (total and the stride are multiples
    // of 8, so an x-block's lanes are all active or all idle)
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v - lane < total;
         v += (long long)gridDim.x * kBlock) {
        const bool act = v < total;
        uint32_t fm = 0;
        if (act) {
            const int x = (int)(v % mx), y = (int)((v / mx) % my),
                      z = (int)(v / ((long long)mx * my));
            float sf = 0.f, sm = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const long long s = ((long long)(2 * z + (q >> 2)) * ny + 2 * y + ((q >> 1) & 1)) *
                                        nx + 2 * x + (q & 1);
                sf += F[s];
                sm += M[s];
            }
            fm = (uint32_t)f2bf(0.125f * sf) | ((uint32_t)f2bf(0.125f * sm) << 16);
            *reinterpret_cast<uint4*>(X + v * 8) = make_uint4(fm, 0, 0, 0);
        }
        uint32_t h[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = (uint32_t)__shfl((int)fm, (lane & ~7) + k, 64);
        // lane 0: F halves (low), lane 1: M halves (high), others zero
        const uint32_t sel = j == 0 ? 0x05040100u : 0x07060302u;
        uint4 o = make_uint4(0, 0, 0, 0);
        if (j < 2) {
            o.x = __builtin_amdgcn_perm(h[1], h[0], sel);
            o.y = __builtin_amdgcn_perm(h[3], h[2], sel);
            o.z = __builtin_amdgcn_perm(h[5], h[4], sel);
            o.w = __builtin_amdgcn_perm(h[7], h[6], sel);
        }
        if (act) *reinterpret_cast<uint4*>(XB + (v - j) * 8 + 8 * j) = o;
    }
}

// k_pool2_lrelu_bwd_v8 written x-blocked (nx a multiple of 8): thread i
// takes voxel 8 b + j (j = i % 8) and channels 8 cg .. + 7, so that the 8
// lanes of one x-block are consecutive; each wave stores its 64 results
// channel-last in LDS and reads them back as dXB[b][8 cg + j][0..7].
__global__ void __launch_bounds__(kBlock)
k_pool2_lrelu_bwd_xb(const float* __restrict__ dY, int nx, int ny, int nz, int C,
                     const u16* __restrict__ gate, int ldg, int goff, u16* __restrict__ dXB) {
    __shared__ __align__(16) u16 tr[kBlock * 8];
    const int mx = nx / 2, my = ny / 2, C8 = C / 8;
    const int total = nx * ny * nz * C8;
    const int j = threadIdx.x & 7;
    u16* mine = tr + (threadIdx.x >> 3) * 64;   // this x-block group's 8 x 8 tile
    // the loop runs while any thread of the block has work: the barriers
    // below are reached by every thread
    for (int i0 = blockIdx.x * kBlock; i0 < total; i0 += gridDim.x * kBlock) {
        const int i = i0 + threadIdx.x;
        const bool act = i < total;
        const int cg = (i / 8) % C8, b = i / (8 * C8);
        const int v = 8 * b + j;
        uint4 out = make_uint4(0, 0, 0, 0);
        if (act) {
            const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
            float g[8], a[8];
            load8f(dY + ((long long)((z / 2) * my + y / 2) * mx + x / 2) * C + 8 * cg, g);
            unpack8(*reinterpret_cast<const uint4*>(gate + (long long)v * ldg + goff + 8 * cg), a);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float t = 0.125f * g[c];
                g[c] = a[c] > 0.f ? t : 0.1f * t;
            }
            out = pack8(g);
        }
        __syncthreads();   // the previous iteration's reads are done
        *reinterpret_cast<uint4*>(mine + 8 * j) = out;   // [voxel j][channel]
        __syncthreads();
        if (act) {
            uint32_t w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                w[k] = (uint32_t)mine[(2 * k) * 8 + j] | ((uint32_t)mine[(2 * k + 1) * 8 + j] << 16);
            *reinterpret_cast<uint4*>(dXB + ((long long)b * C + 8 * cg + j) * 8) =
                make_uint4(w[0], w[1], w[2], w[3]);
        }
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

// the brick forms' epilogue stores whole 8-channel vectors: channel counts,
// strides and offsets in multiples of 8 elements, 16-byte aligned tensors
static bool vector_epilogue_ok(const ConvEpi& E, int cout) {
    auto al = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
    if (cout % 8) return false;
    if (E.ybf && (E.ldy % 8 || E.yoff % 8 || !al(E.ybf))) return false;
    if (E.yf && (E.ldyf % 8 || !al(E.yf))) return false;
    if (E.act == 2 && (!E.gate || E.ldg % 8 || E.goff % 8 || !al(E.gate))) return false;
    return true;
}

// the first layer's convolution over 8 channels of which only 0 and 1 carry
// data (whole 16 x 4 x 4 bricks; see k_conv_fwd_brick_in2); false: not this shape
bool conv3d_fwd_in2(const uint16_t* x, const int32_t dims[3], int32_t batch,
                    const uint16_t* wt, const float* bias, int32_t cout, int32_t act,
                    uint16_t* y_bf16, int32_t ldy, float* y_f32, int32_t ldyf, hipStream_t s,
                    hipError_t* err) {
    if (dims[0] % kBrX || dims[1] % kBrY || dims[2] % kBrZ || cout < 1 || cout > 64 || batch < 1 ||
        act < 0 || act > 1 || (!y_bf16 && !y_f32) || ((uintptr_t)x & 15) || ((uintptr_t)wt & 3))
        return false;
    const long long nz = (long long)dims[2] * batch;
    const long long nbrick = (long long)(dims[0] / kBrX) * (dims[1] / kBrY) * (nz / kBrZ);
    if (nz > (1LL << 30) || nbrick >= 0x7fffffffLL) return false;
    ConvDims D{dims[0], dims[1], (int)nz, dims[2], 8, cout, 27 * 8, 27 * 8 + 8};
    ConvEpi E{bias, act, nullptr, 0, 0, (u16*)y_bf16, ldy, 0, y_f32, ldyf};
    if (!vector_epilogue_ok(E, cout)) return false;
    const dim3 grid((unsigned)nbrick), blk(256);
    switch ((cout + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_conv_fwd_brick_in2<1>, grid, blk, 0, s, (const u16*)x, D,
                                   (const u16*)wt, E); break;
        case 2: hipLaunchKernelGGL(k_conv_fwd_brick_in2<2>, grid, blk, 0, s, (const u16*)x, D,
                                   (const u16*)wt, E); break;
        case 3: hipLaunchKernelGGL(k_conv_fwd_brick_in2<3>, grid, blk, 0, s, (const u16*)x, D,
                                   (const u16*)wt, E); break;
        default: hipLaunchKernelGGL(k_conv_fwd_brick_in2<4>, grid, blk, 0, s, (const u16*)x, D,
                                    (const u16*)wt, E); break;
    }
    *err = hipGetLastError();
    return true;
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
    const u16* X = (const u16*)x;
    const u16* W = (const u16*)wt;
    // whole 16 x 4 x 4 bricks and at least one per CU: the LDS brick form
    // (its epilogue writes whole 8-channel vectors)
    const long long nbrick = (D.nx % kBrX == 0 && D.ny % kBrY == 0 && D.nzv % kBrZ == 0)
                                 ? (long long)(D.nx / kBrX) * (D.ny / kBrY) * (D.nz / kBrZ) : 0;
    if (nbrick >= 256 && nbrick < 0x7fffffffLL && cout <= 64 && vector_epilogue_ok(E, cout)) {
        const int cs = (cin == 8 || cin == 16 || cin == 32 || cin == 48) ? cin
                       : cin % 16 == 0 ? 16 : 8;
        const dim3 grid((unsigned)nbrick), blk(256);
        switch (nt * 64 + cs) {
#define CASE2(T, C) case T * 64 + C: \
        hipLaunchKernelGGL((k_conv_fwd_brick<T, C>), grid, blk, 0, s, X, D, W, E); break;
#define CASE(T) CASE2(T, 8) CASE2(T, 16) CASE2(T, 32) CASE2(T, 48)
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
#undef CASE2
            default: return AIR_ERR_SHAPE;
        }
        return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
    }
    // the most voxels per wave that still give 1024 blocks of four waves;
    // below that, the split-K form with four or one 16-voxel tiles per block
    // keeps the chip busy (code 0: one tile, 3: four tiles)
    // (four tiles only for large weight matrices, whose re-reads dominate)
    const int mt = N >= 4096LL * 64 ? 4 : N >= 2048LL * 64 ? 2 : N >= 1024LL * 64 ? 1
                   : (N >= 512LL * 64 && (long long)cout * D.K >= 65536) ? 3 : 0;
    const long long nblk = mt == 3 ? (N + 63) / 64
                           : mt ? (N + 64LL * mt - 1) / (64LL * mt) : (N + 15) / 16;
    if (nblk > 0x7fffffffLL) return AIR_ERR_SHAPE;
    const dim3 grid((unsigned)nblk), blk(256);
    switch (nt * 8 + mt) {
#define CASE(T)                                                                       \
    case T * 8 + 0: hipLaunchKernelGGL((k_conv_fwd_sk<T, 1>), grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 3: hipLaunchKernelGGL((k_conv_fwd_sk<T, 4>), grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 1: hipLaunchKernelGGL((k_conv_fwd<T, 1>), grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 2: hipLaunchKernelGGL((k_conv_fwd<T, 2>), grid, blk, 0, s, X, D, W, E); break; \
    case T * 8 + 4: hipLaunchKernelGGL((k_conv_fwd<T, 4>), grid, blk, 0, s, X, D, W, E); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return AIR_ERR_SHAPE;
    }
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

// the x-blocked form: whole 8-voxel x blocks and at most four 16-channel
// output tiles per wave
static bool bwdw_xb(const int32_t dims[3], int cout) { return dims[0] % 8 == 0 && cout <= 64; }

// voxels per partial of the backward-weight GEMM: about one resident round
// of blocks (`target` blocks) over the whole reduction
static long long bwdw_chunk(long long N, int cin, int cout, bool xb) {
    const int kx = ((27 * cin + 15) / 16 + BWK - 1) / BWK;
    const int per = xb ? kx : kx * ((cout + 15) / 16);
    long long nbz = (xb ? 512 : 768) / per;
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
    const bool xb = bwdw_xb(dims, cout);
    const long long c = chunk ? chunk : bwdw_chunk(N, cin, cout, xb);
    const long long nch = (N + c - 1) / c;
    if (nch > 65535) return AIR_ERR_SHAPE;
    size_t b = (size_t)(4LL * nch * cout * (27LL * cin + 1));
    // x-blocked copies of x and dy
    if (xb) b = ((b + 255) & ~size_t(255)) + (size_t)((2 * N * cin + 255) & ~255LL) + 2 * N * cout;
    *bytes = b;
    return AIR_OK;
}

air_status air_conv3d_bwd_weight(const uint16_t* x, const int32_t dims[3], int32_t batch,
                                 int32_t cin, const uint16_t* dy, int32_t cout, int32_t chunk,
                                 float* dwt, float* db, void* ws, size_t ws_bytes, void* stream) {
    if (!x || !dims || !dy || !dwt) return AIR_ERR_INVALID_ARG;
    if (cin < 8 || cin % 8 || cout < 8 || cout % 8 || cout > 128) return AIR_ERR_SHAPE;
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(dy) |
         reinterpret_cast<uintptr_t>(ws)) & 15)
        return AIR_ERR_ALIGN;
    size_t need = 0;
    air_status st = air_conv3d_bwd_weight_workspace(dims, batch, cin, cout, chunk, &need);
    if (st != AIR_OK) return st;
    if (!ws || ws_bytes < need) return AIR_ERR_WORKSPACE;
    const long long nz = (long long)dims[2] * batch;
    if (nz > (1LL << 30)) return AIR_ERR_SHAPE;
    ConvDims D{dims[0], dims[1], (int)nz, dims[2], cin, cout, 27 * cin, (27 * cin + 31) / 32 * 32};
    const long long N = (long long)D.nx * D.ny * D.nz;
    const bool xb = bwdw_xb(dims, cout);
    const long long c = chunk ? chunk : bwdw_chunk(N, cin, cout, xb);
    const int nch = (int)((N + c - 1) / c);
    hipStream_t s = (hipStream_t)stream;
    float* part = (float*)ws;
    if (!xb) {
        const int ktiles = (D.K + 15) / 16;
        dim3 grid((ktiles + BWK - 1) / BWK, (cout + 15) / 16, nch);
        hipLaunchKernelGGL(k_conv_bwdw, grid, dim3(256), 0, s, (const u16*)x, D, (const u16*)dy,
                           (int)c, part);
        hipLaunchKernelGGL(k_conv_bwdw_reduce, dim3((cout * (D.K + 1) + 63) / 64),
                           dim3(kRedThreads), 0, s, (const float*)part, nch, cout, cin, cin, dwt,
                           db);
        return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
    }
    const size_t pb = ((size_t)(4LL * nch * cout * (27LL * cin + 1)) + 255) & ~size_t(255);
    u16* XB = reinterpret_cast<u16*>(static_cast<unsigned char*>(ws) + pb);
    u16* dYB = XB + ((2 * N * cin + 255) & ~255LL) / 2;
    const long long nblk = N / 8;
    hipLaunchKernelGGL(k_to_xb, dim3(grid1(nblk * ((cin + cout) / 8))), dim3(kBlock), 0, s,
                       (const u16*)x, (int)cin, XB, (const u16*)dy, (int)cout, dYB, nblk);
    return air_conv3d_bwd_weight_xb(XB, dims, batch, cin, 0, dYB, cout, chunk, dwt, db, ws, pb,
                                    stream);
}

air_status air_conv3d_bwd_weight_xb_workspace(const int32_t dims[3], int32_t batch, int32_t cin,
                                              int32_t cin_used, int32_t cout, int32_t chunk,
                                              size_t* bytes) {
    if (!dims || !bytes || chunk < 0 || chunk % kBwStep || batch < 1) return AIR_ERR_INVALID_ARG;
    if (dims[0] < 8 || dims[0] % 8 || dims[1] < 1 || dims[2] < 1 || cin < 1 || cout < 1 ||
        cout > 64 || cin_used < 0 || cin_used > cin)
        return AIR_ERR_SHAPE;
    const int cu = cin_used ? cin_used : cin;
    const long long N = (long long)dims[0] * dims[1] * dims[2] * batch;
    const long long c = chunk ? chunk : bwdw_chunk(N, cu, cout, true);
    const long long nch = (N + c - 1) / c;
    if (nch > 65535) return AIR_ERR_SHAPE;
    *bytes = (size_t)(4LL * nch * cout * (27LL * cu + 1));
    return AIR_OK;
}

air_status air_conv3d_bwd_weight_xb(const uint16_t* xb, const int32_t dims[3], int32_t batch,
                                    int32_t cin, int32_t cin_used, const uint16_t* dyb,
                                    int32_t cout, int32_t chunk, float* dwt, float* db, void* ws,
                                    size_t ws_bytes, void* stream) {
    if (!xb || !dims || !dyb || !dwt) return AIR_ERR_INVALID_ARG;
    if (cin < 8 || cin % 8 || cout < 8 || cout % 8) return AIR_ERR_SHAPE;
    if ((reinterpret_cast<uintptr_t>(xb) | reinterpret_cast<uintptr_t>(dyb) |
         reinterpret_cast<uintptr_t>(ws)) & 15)
        return AIR_ERR_ALIGN;
    size_t need = 0;
    air_status st =
        air_conv3d_bwd_weight_xb_workspace(dims, batch, cin, cin_used, cout, chunk, &need);
    if (st != AIR_OK) return st;
    if (!ws || ws_bytes < need) return AIR_ERR_WORKSPACE;
    const long long nz = (long long)dims[2] * batch;
    if (nz > (1LL << 30)) return AIR_ERR_SHAPE;
    ConvDims D{dims[0], dims[1], (int)nz, dims[2], cin, cout, 27 * cin, (27 * cin + 31) / 32 * 32};
    const long long N = (long long)D.nx * D.ny * D.nz;
    // element offsets of a tap's block from the lane's own fit in 32 bits
    if (2LL * D.ny * (D.nx / 8) * cin * 8 + 27LL * cin * 8 >= (1LL << 31)) return AIR_ERR_SHAPE;
    const int cu = cin_used ? cin_used : cin;
    const long long c = chunk ? chunk : bwdw_chunk(N, cu, cout, true);
    const int nch = (int)((N + c - 1) / c);
    hipStream_t s = (hipStream_t)stream;
    float* part = (float*)ws;
    const int ktiles = (27 * cu + 15) / 16;
    const dim3 grid((ktiles + BWK - 1) / BWK, 1, nch);
    switch ((cout + 15) / 16) {
#define CASE(T) case T: hipLaunchKernelGGL(k_conv_bwdw_xb<T>, grid, dim3(256), 0, s, \
                                           (const u16*)xb, D, cu, (const u16*)dyb, (int)c, part); \
                break;
        CASE(1) CASE(2) CASE(3) CASE(4)
#undef CASE
        default: return AIR_ERR_SHAPE;
    }
    hipLaunchKernelGGL(k_conv_bwdw_reduce, dim3((cout * (D.K + 1) + 63) / 64), dim3(kRedThreads), 0,
                       s, (const float*)part, nch, cout, cin, cu, dwt, db);
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

// the 8-channel kernels: channel counts, strides and offsets in whole
// 16-byte vectors, aligned tensors, 32-bit thread indices
static bool v8(int c, int ld, int off, const void* p, const void* q, long long threads) {
    return c % 8 == 0 && ld % 8 == 0 && off % 8 == 0 && a16(p) && a16(q) &&
           threads < (1LL << 31) - (long long)kBlock * 16384;
}

air_status air_pool2(const uint16_t* x, const int32_t dims[3], int32_t c, int32_t ldx,
                     int32_t xoff, uint16_t* y, void* stream) {
    if (!x || !dims || !y || c < 1 || xoff < 0 || ldx < xoff + c) return AIR_ERR_INVALID_ARG;
    if (dims[0] % 2 || dims[1] % 2 || dims[2] % 2) return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] / 8 * c;
    if (v8(c, ldx, xoff, x, y, t / 8))
        hipLaunchKernelGGL(k_pool2_v8, dim3(grid1(t / 8)), dim3(kBlock), 0, (hipStream_t)stream,
                           (const u16*)x, dims[0], dims[1], dims[2], c, ldx, xoff, (u16*)y);
    else
        hipLaunchKernelGGL(k_pool2, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream,
                           (const u16*)x, dims[0], dims[1], dims[2], c, ldx, xoff, (u16*)y);
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
    if (!x || !dims || !y || c < 1 || yoff < 0 || ldy < yoff + c) return AIR_ERR_INVALID_ARG;
    const long long t = 8LL * dims[0] * dims[1] * dims[2] * c;
    if (v8(c, ldy, yoff, x, y, t / 64))
        hipLaunchKernelGGL(k_up2_v8, dim3(grid1(t / 64)), dim3(kBlock), 0, (hipStream_t)stream,
                           (const u16*)x, dims[0], dims[1], dims[2], c, (u16*)y, ldy, yoff);
    else
        hipLaunchKernelGGL(k_up2, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream,
                           (const u16*)x, dims[0], dims[1], dims[2], c, (u16*)y, ldy, yoff);
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
                              const uint16_t* gate, int32_t ldg, int32_t goff, int32_t xblocked,
                              uint16_t* dx, void* stream) {
    if (!dy || !dims || !gate || !dx || c < 1 || goff < 0 || ldg < goff + c)
        return AIR_ERR_INVALID_ARG;
    if (add && (addoff < 0 || ldadd < addoff + c)) return AIR_ERR_INVALID_ARG;
    if (dims[0] < 2 || dims[1] < 2 || dims[2] < 2 || dims[0] % 2 || dims[1] % 2 || dims[2] % 2)
        return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] * c;
    if (xblocked) {
        if (add || dims[0] % 8 || !v8(c, ldg, goff, gate, dx, t / 8) || !a16(dy))
            return AIR_ERR_SHAPE;
        hipLaunchKernelGGL(k_pool2_lrelu_bwd_xb, dim3(grid1(t / 8)), dim3(kBlock), 0,
                           (hipStream_t)stream, dy, dims[0], dims[1], dims[2], c, (const u16*)gate,
                           ldg, goff, (u16*)dx);
        return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
    }
    if (v8(c, ldg, goff, gate, dx, t / 8) && a16(dy) && (!add || v8(c, ldadd, addoff, add, dy, 0)))
        hipLaunchKernelGGL(k_pool2_lrelu_bwd_v8, dim3(grid1(t / 8)), dim3(kBlock), 0,
                           (hipStream_t)stream, dy, dims[0], dims[1], dims[2], c, add, ldadd,
                           addoff, (const u16*)gate, ldg, goff, (u16*)dx);
    else
        hipLaunchKernelGGL(k_pool2_lrelu_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream,
                           dy, dims[0], dims[1], dims[2], c, add, ldadd, addoff, (const u16*)gate,
                           ldg, goff, (u16*)dx);
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
    if (v8(c, ldg, goff, gate, dx, t / 8) && v8(c, ldy, yoff, dy, dy, 0))
        hipLaunchKernelGGL(k_up2_lrelu_bwd_v8, dim3(grid1(t / 8)), dim3(kBlock), 0,
                           (hipStream_t)stream, dy, dims[0], dims[1], dims[2], c, ldy, yoff,
                           (const u16*)gate, ldg, goff, (u16*)dx);
    else
        hipLaunchKernelGGL(k_up2_lrelu_bwd, dim3(grid1(t)), dim3(kBlock), 0, (hipStream_t)stream,
                           dy, dims[0], dims[1], dims[2], c, ldy, yoff, (const u16*)gate, ldg, goff,
                           (u16*)dx);
    return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
}

air_status air_cnn_input(const float* fixed, const float* moving, const int32_t dims[3],
                         uint16_t* x, uint16_t* x_xb, void* stream) {
    if (!fixed || !moving || !dims || !x) return AIR_ERR_INVALID_ARG;
    if (dims[0] % 2 || dims[1] % 2 || dims[2] % 2) return AIR_ERR_SHAPE;
    const long long t = (long long)dims[0] * dims[1] * dims[2] / 8;
    if (x_xb) {
        if ((dims[0] / 2) % 8 || !a16(x) || !a16(x_xb)) return AIR_ERR_SHAPE;
        hipLaunchKernelGGL(k_cnn_input_xb, dim3(grid1(t)), dim3(kBlock), 0,
                           (hipStream_t)stream, fixed, moving, dims[0], dims[1], dims[2], (u16*)x,
                           (u16*)x_xb);
        return hipGetLastError() == hipSuccess ? AIR_OK : AIR_ERR_LAUNCH;
    }
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

// this unit's bounds-check flags (debug build only)
AIR_DEBUG_UNIT(cnn)
