// Device helpers shared by the airhip kernels.
#pragma once

#include "air_internal.h"

namespace air {

typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Buffer resource over [base, base + bytes) for raw (untyped) loads. The
// operands are made wave-uniform explicitly so that the descriptor lives in
// SGPRs (a descriptor the compiler cannot prove uniform costs a
// readfirstlane loop around every load).
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    const uint64_t p = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    const uint32_t nb = __builtin_amdgcn_readfirstlane(bytes);
    void* q = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, (int)nb, 0x00020000);
}

// Two consecutive floats at byte offset voff + soff (dword aligned).
__device__ inline v2f load2(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Bounds checks of computed indices, compiled in the debug build
// (-DAIR_DEBUG_BOUNDS, libairhip_debug.so) and empty otherwise. A failed
// check sets its bit in the flag word of its translation unit (a buffer
// load out of range would silently read zero, a global one could fault);
// air_debug_bounds_take reads and clears every unit's word. Bits:
enum DebugBit : unsigned {
    kDbgMovingGather = 0,   // fused B-spline kernels: moving-image corner gathers
    kDbgFixedLoad = 1,      // fused B-spline kernels: fixed-image loads
    kDbgSampler = 2,        // dense / warp samplers: corner gathers
    kDbgCompose = 3,        // exponential: squaring gathers
    kDbgConvInput = 4,      // CNN convolutions: input and weight loads
    kDbgConvWgrad = 5,      // CNN weight gradient: operand loads
    kDbgControlLoad = 6,    // fused B-spline kernels: control-window loads
};
#ifdef AIR_DEBUG_BOUNDS
static __device__ unsigned int air_dbg_flags;
#define AIR_CHECK(cond, bit)                                                 \
    do {                                                                     \
        if (!(cond)) atomicOr(&air_dbg_flags, 1u << (unsigned)(bit));       \
    } while (0)
// defines air::debug_take_<name>(): this unit's flags, cleared
#define AIR_DEBUG_UNIT(name)                                                 \
    namespace air {                                                          \
    uint32_t debug_take_##name() {                                           \
        unsigned int v = 0, z = 0;                                           \
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(air_dbg_flags), sizeof(v)) != \
            hipSuccess)                                                      \
            return 0x80000000u;                                              \
        (void)hipMemcpyToSymbol(HIP_SYMBOL(air_dbg_flags), &z, sizeof(z));   \
        return v;                                                            \
    }                                                                        \
    }
#else
#define AIR_CHECK(cond, bit) \
    do {                     \
    } while (0)
#define AIR_DEBUG_UNIT(name)
#endif

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sum K doubles over the block in a fixed order; every thread gets the totals.
// scratch: K * (NT / 64) doubles of LDS.
template <int NT, int K>
__device__ inline void block_sum(double (&v)[K], double* scratch) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scratch[k * NW + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = 0; i < NW; ++i) s += scratch[k * NW + i];
        v[k] = s;
    }
    __syncthreads();
}

// Index of the pair owning global work item `item` (binary search on begin).
template <bool REG>
__device__ inline int find_pair(const PairDesc* pairs, int npairs, int item) {
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int b = REG ? pairs[mid].reg_begin : pairs[mid].tile_begin;
        if (b <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8).
// The grid is 8 * (ceil(T/8) + ceil(R/8)) blocks for T tiles and R
// regulariser blocks: the i-th block of XCD x takes tile x*ceil(T/8) + i while
// i < ceil(T/8), then regulariser block x*ceil(R/8) + (i - ceil(T/8)). Each
// XCD works on one contiguous run of tiles (neighbouring tiles share its L2)
// and every XCD gets the same number of tiles. Returns the tile index, or
// T + regulariser index, or -1 for an idle block.
__device__ inline int xcd_item(int b, int T, int R) {
    constexpr int NX = 8;
    const int tq = (T + NX - 1) / NX, rq = (R + NX - 1) / NX;
    const int x = b % NX, i = b / NX;
    if (i < tq) {
        const int t = x * tq + i;
        return t < T ? t : -1;
    }
    const int r = x * rq + (i - tq);
    return (i - tq < rq && r < R) ? T + r : -1;
}

__host__ __device__ inline int xcd_grid(int T, int R) {
    return 8 * ((T + 7) / 8 + (R + 7) / 8);
}

// Displacement of a voxel along one axis in voxels, d = fl(u s), and the
// exact rounding error e = u s - d (one fma returns it exactly). The sample
// point x + u s is never formed in floating point: rounding it to FP32 would
// move the interpolation weights by up to half an ulp of the point (4e-6
// voxel at x ~ 100), while d carries an error below half an ulp of the
// displacement itself. The cell and the mask are decided on x + d + e.
struct Disp {
    float d, e;
};
__device__ inline Disp disp_of(float u, float s) {
    const float d = u * s;
    return {d, fmaf(u, s, -d)};
}
// The cell [t, t + 1] holding the exact point x + d + e along one axis of n
// voxels (t not clamped), the fraction f in [0, 1] (1 only when d is an
// integer and e < 0: the point lies just below it), and whether
// 0 <= x + d + e <= n - 1 (false for a non-finite d).
struct AxisCell {
    int t;
    float f;
    bool in;
};
__device__ inline AxisCell axis_cell(int x, Disp q, int n) {
    const float lo = (float)(-x), hi = (float)(n - 1 - x);
    AxisCell c;
    // (bitwise: compares only, no branches)
    c.in = ((int)(q.d > lo) | ((int)(q.d == lo) & (int)(q.e >= 0.f))) &
           ((int)(q.d < hi) | ((int)(q.d == hi) & (int)(q.e <= 0.f)));
    const float d = fminf(fmaxf(q.d, -1e9f), 1e9f);
    const float fl = floorf(d);
    c.f = d - fl;   // exact
    c.t = x + (int)fl;
    if (c.f == 0.f && q.e < 0.f) {
        c.t -= 1;
        c.f = 1.f;
    }
    return c;
}

// Zero-padded multilinear sample of M at x + d + e (voxel units) with its
// derivative on the cell of axis_cell (right-sided at an integer point);
// also reports whether the point lies inside the volume. Used where speed is
// secondary.
template <int DIM>
__device__ inline float sample_general(const float* __restrict__ M, const int* n, const int* x,
                                       const Disp* dq, bool* inside, float* dW) {
    float f[3];
    int j[3];
    bool in = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const AxisCell c = axis_cell(x[a], dq[a], n[a]);
        if (!c.in) in = false;
        j[a] = c.t;
        f[a] = c.f;
    }
    *inside = in;
    float W = 0.f;
    float d[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        int q[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            q[a] = j[a] + ((c >> a) & 1);
            if (q[a] < 0 || q[a] > n[a] - 1) ok = false;
        }
        float val = 0.f;
        if (ok) {
            long long idx = q[0] + (long long)n[0] * (q[1] + (DIM == 3 ? (long long)n[1] * q[2] : 0));
            val = M[idx];
        }
        float w = 1.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) w *= ((c >> a) & 1) ? f[a] : 1.f - f[a];
        W += w * val;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            float wa = ((c >> a) & 1) ? 1.f : -1.f;
#pragma unroll
            for (int b = 0; b < DIM; ++b)
                if (b != a) wa *= ((c >> b) & 1) ? f[b] : 1.f - f[b];
            d[a] += wa * val;
        }
    }
    if (dW) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) dW[a] = d[a];
    }
    return W;
}

}  // namespace air
