// The learned-initialisation network as one object of the C-ABI: the layer
// schedule of a 3D encoder-decoder for an n^3 pair (n a multiple of 16), its
// parameter layout and its workspace, and the forward and backward passes
// sequenced over the library's BF16 MFMA convolutions and the pooling,
// upsampling and activation kernels (k_cnn.hip).
//
// Architecture (g = n / 8 control cells per axis):
//   x0 = avgpool2(F, M), 8 channels (F, M, six zero channels)     (n/2)^3
//   a1 = lrelu(conv(x0))          16 ch                            (n/2)^3
//   a2 = lrelu(conv(pool(a1)))    32 ch                            (n/4)^3
//   a3 = lrelu(conv(pool(a2)))    48 ch -> cat[:, 0:48]            (n/8)^3
//   a4 = lrelu(conv(pool(a3)))    64 ch                            (n/16)^3
//   cat[:, 48:112] = up2(a4)
//   d1 = lrelu(conv(cat))         48 ch                            (n/8)^3
//   o  = conv(d1)                 16 ch, FP32 (channels 0..2 used) (n/8)^3
//   theta0[c][j] = 0.05 o[clamp(j - 1, 0, g - 1)][c]               3 x (g+3)^3
// Parameters: one FP32 buffer, per layer W [cout][27 cin] (k = tap cin + ci,
// tap = (dz*3 + dy)*3 + dx) then b [cout], layers in the order above.
#include <stdint.h>

#include <new>

#include "device_common.h"

namespace air {

namespace {

typedef unsigned short u16;

constexpr int kLayers = 6;
constexpr int kCat = 112;
constexpr float kOutScale = 0.05f;
constexpr int kBwdwChunk = 256;

struct LayerDef {
    int cin, cout, act;
};
constexpr LayerDef kDef[kLayers] = {
    {8, 16, 1}, {16, 32, 1}, {32, 48, 1}, {48, 64, 1}, {kCat, 48, 1}, {48, 16, 0}};

__device__ inline u16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u16)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

struct RefreshArgs {
    int w_off[kLayers];      // float offset of W in the parameters
    long long wb_off[kLayers];   // u16 offset of the bf16 copy in the workspace
    long long wf_off[kLayers];   // u16 offset of the flipped copy
    int cin[kLayers], cout[kLayers];
    int total;               // sum of 27 cin cout
};

// BF16 copies of every layer's weights in one launch: Wb[co][k] = bf16(W[co][k])
// and the flipped, transposed copy for backward-data,
// Wf[ci][tap' cout + co] = bf16(W[co][(26 - tap') cin + ci]).
__global__ void __launch_bounds__(kBlock)
k_cnn_refresh(const float* __restrict__ P, u16* __restrict__ ws16, RefreshArgs A) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < A.total; i += gridDim.x * kBlock) {
        int l = 0, base = 0;
        while (l < kLayers - 1 && i >= base + 27 * A.cin[l] * A.cout[l]) {
            base += 27 * A.cin[l] * A.cout[l];
            ++l;
        }
        const int j = i - base;             // index into W[co][k]
        const int cin = A.cin[l], cout = A.cout[l], K = 27 * cin;
        const int co = j / K, k = j - co * K;
        const u16 v = to_bf16(P[A.w_off[l] + j]);
        ws16[A.wb_off[l] + j] = v;
        const int tap = k / cin, ci = k - tap * cin;
        ws16[A.wf_off[l] + (long long)ci * 27 * cout + (26 - tap) * cout + co] = v;
    }
}

inline size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

}  // namespace air

using namespace air;

struct air_cnn {
    int n = 0;
    int h = 0, q = 0, e = 0, s = 0;   // sides at n/2, n/4, n/8, n/16
    int w_off[kLayers] = {}, b_off[kLayers] = {};
    int64_t nparam = 0;
    // workspace byte offsets
    size_t wb[kLayers] = {}, wf[kLayers] = {};
    size_t x0, a1, p1, a2, p2, cat, p3, a4, d1, out;
    size_t g_out, g_out_bf, g_d1, g_d1_bf, g_cat, g_a4, g_a4_bf, g_p3, g_a3_bf, g_p2, g_a2,
        g_a2_bf, g_p1, g_a1, g_a1_bf, bwdw;
    size_t bwdw_bytes = 0;
    size_t total = 0;
    RefreshArgs refresh{};
};

namespace {

long long cube(int a) { return (long long)a * a * a; }

void layer_dims(const air_cnn* N, int l, int32_t d[3]) {
    const int side[kLayers] = {N->h, N->q, N->e, N->s, N->e, N->e};
    d[0] = d[1] = d[2] = side[l];
}

}  // namespace

extern "C" {

air_status air_cnn_create(int32_t n, air_cnn** out) {
    if (!out) return AIR_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 16 || n % 16 || n > 1024) return AIR_ERR_SHAPE;
    air_cnn* N = new (std::nothrow) air_cnn();
    if (!N) return AIR_ERR_DEVICE;
    N->n = n;
    N->h = n / 2;
    N->q = n / 4;
    N->e = n / 8;
    N->s = n / 16;
    int64_t p = 0;
    for (int l = 0; l < kLayers; ++l) {
        N->w_off[l] = (int)p;
        p += 27LL * kDef[l].cin * kDef[l].cout;
        N->b_off[l] = (int)p;
        p += kDef[l].cout;
        p = (p + 3) & ~int64_t(3);
    }
    N->nparam = p;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = up256(o + bytes);
        return at;
    };
    int total = 0;
    for (int l = 0; l < kLayers; ++l) {
        const size_t nw = 27ULL * kDef[l].cin * kDef[l].cout;
        N->wb[l] = take(2 * nw);
        N->wf[l] = take(2 * nw);
        N->refresh.w_off[l] = N->w_off[l];
        N->refresh.wb_off[l] = (long long)(N->wb[l] / 2);
        N->refresh.wf_off[l] = (long long)(N->wf[l] / 2);
        N->refresh.cin[l] = kDef[l].cin;
        N->refresh.cout[l] = kDef[l].cout;
        total += (int)nw;
    }
    N->refresh.total = total;
    const long long H = cube(N->h), Q = cube(N->q), E = cube(N->e), S = cube(N->s);
    N->x0 = take(2 * H * 8);
    N->a1 = take(2 * H * 16);
    N->p1 = take(2 * Q * 16);
    N->a2 = take(2 * Q * 32);
    N->p2 = take(2 * E * 32);
    N->cat = take(2 * E * kCat);
    N->p3 = take(2 * S * 48);
    N->a4 = take(2 * S * 64);
    N->d1 = take(2 * E * 48);
    N->out = take(4 * E * 16);
    N->g_out = take(4 * E * 16);
    N->g_out_bf = take(2 * E * 16);
    N->g_d1 = take(4 * E * 48);
    N->g_d1_bf = take(2 * E * 48);
    N->g_cat = take(4 * E * kCat);
    N->g_a4 = take(4 * S * 64);
    N->g_a4_bf = take(2 * S * 64);
    N->g_p3 = take(4 * S * 48);
    N->g_a3_bf = take(2 * E * 48);
    N->g_p2 = take(4 * E * 32);
    N->g_a2 = take(4 * Q * 32);
    N->g_a2_bf = take(2 * Q * 32);
    N->g_p1 = take(4 * Q * 16);
    N->g_a1 = take(4 * H * 16);
    N->g_a1_bf = take(2 * H * 16);
    size_t bw = 0;
    for (int l = 0; l < kLayers; ++l) {
        int32_t d[3];
        layer_dims(N, l, d);
        size_t b = 0;
        if (air_conv3d_bwd_weight_workspace(d, kDef[l].cin, kDef[l].cout, kBwdwChunk, &b) !=
            AIR_OK) {
            delete N;
            return AIR_ERR_SHAPE;
        }
        bw = b > bw ? b : bw;
    }
    N->bwdw_bytes = bw;
    N->bwdw = take(bw);
    N->total = o;
    *out = N;
    return AIR_OK;
}

void air_cnn_destroy(air_cnn* net) { delete net; }

air_status air_cnn_sizes(const air_cnn* net, int64_t* param_floats, size_t* ws_bytes) {
    if (!net) return AIR_ERR_INVALID_ARG;
    if (param_floats) *param_floats = net->nparam;
    if (ws_bytes) *ws_bytes = net->total;
    return AIR_OK;
}

air_status air_cnn_layer(const air_cnn* net, int32_t layer, int32_t* cin, int32_t* cout,
                         int64_t* w_offset, int64_t* b_offset) {
    if (!net) return AIR_ERR_INVALID_ARG;
    if (layer < 0 || layer >= kLayers) return AIR_ERR_SHAPE;
    if (cin) *cin = kDef[layer].cin;
    if (cout) *cout = kDef[layer].cout;
    if (w_offset) *w_offset = net->w_off[layer];
    if (b_offset) *b_offset = net->b_off[layer];
    return AIR_OK;
}

#define AIR_TRY(x)                              \
    do {                                        \
        const air_status st_ = (x);             \
        if (st_ != AIR_OK) return st_;          \
    } while (0)

air_status air_cnn_forward(const air_cnn* N, const float* params, const float* fixed,
                           const float* moving, float* theta0, void* ws, size_t ws_bytes,
                           void* stream) {
    if (!N || !params || !fixed || !moving || !theta0) return AIR_ERR_INVALID_ARG;
    if (!ws || ws_bytes < N->total) return AIR_ERR_WORKSPACE;
    if (((uintptr_t)ws | (uintptr_t)params | (uintptr_t)fixed | (uintptr_t)moving |
         (uintptr_t)theta0) & 15u)
        return AIR_ERR_ALIGN;
    unsigned char* w = static_cast<unsigned char*>(ws);
    auto b16 = [&](size_t off) { return reinterpret_cast<uint16_t*>(w + off); };
    auto f32 = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
    hipStream_t s = (hipStream_t)stream;
    {
        const int grid = (N->refresh.total + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_cnn_refresh, dim3(grid < 4096 ? grid : 4096), dim3(kBlock), 0, s,
                           params, reinterpret_cast<u16*>(w), N->refresh);
        if (hipGetLastError() != hipSuccess) return AIR_ERR_LAUNCH;
    }
    const int32_t full[3] = {N->n, N->n, N->n};
    const int32_t H[3] = {N->h, N->h, N->h}, Q[3] = {N->q, N->q, N->q};
    const int32_t E[3] = {N->e, N->e, N->e}, S[3] = {N->s, N->s, N->s};
    AIR_TRY(air_cnn_input(fixed, moving, full, b16(N->x0), stream));
    AIR_TRY(air_conv3d_fwd(b16(N->x0), H, 8, b16(N->wb[0]), params + N->b_off[0], 16, 1,
                           b16(N->a1), 16, 0, nullptr, 16, stream));
    AIR_TRY(air_pool2(b16(N->a1), H, 16, 16, 0, b16(N->p1), stream));
    AIR_TRY(air_conv3d_fwd(b16(N->p1), Q, 16, b16(N->wb[1]), params + N->b_off[1], 32, 1,
                           b16(N->a2), 32, 0, nullptr, 32, stream));
    AIR_TRY(air_pool2(b16(N->a2), Q, 32, 32, 0, b16(N->p2), stream));
    AIR_TRY(air_conv3d_fwd(b16(N->p2), E, 32, b16(N->wb[2]), params + N->b_off[2], 48, 1,
                           b16(N->cat), kCat, 0, nullptr, 48, stream));
    AIR_TRY(air_pool2(b16(N->cat), E, 48, kCat, 0, b16(N->p3), stream));
    AIR_TRY(air_conv3d_fwd(b16(N->p3), S, 48, b16(N->wb[3]), params + N->b_off[3], 64, 1,
                           b16(N->a4), 64, 0, nullptr, 64, stream));
    AIR_TRY(air_up2(b16(N->a4), S, 64, b16(N->cat), kCat, 48, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->cat), E, kCat, b16(N->wb[4]), params + N->b_off[4], 48, 1,
                           b16(N->d1), 48, 0, nullptr, 48, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->d1), E, 48, b16(N->wb[5]), params + N->b_off[5], 16, 0,
                           nullptr, 16, 0, f32(N->out), 16, stream));
    return air_cnn_output(f32(N->out), E, 16, kOutScale, theta0, stream);
}

air_status air_cnn_backward(const air_cnn* N, const float* dtheta, float* grads, void* ws,
                            size_t ws_bytes, void* stream) {
    if (!N || !dtheta || !grads) return AIR_ERR_INVALID_ARG;
    if (!ws || ws_bytes < N->total) return AIR_ERR_WORKSPACE;
    if (((uintptr_t)ws | (uintptr_t)dtheta | (uintptr_t)grads) & 15u) return AIR_ERR_ALIGN;
    unsigned char* w = static_cast<unsigned char*>(ws);
    auto b16 = [&](size_t off) { return reinterpret_cast<uint16_t*>(w + off); };
    auto f32 = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
    void* bw = w + N->bwdw;
    const size_t bwb = N->bwdw_bytes;
    const int32_t H[3] = {N->h, N->h, N->h}, Q[3] = {N->q, N->q, N->q};
    const int32_t E[3] = {N->e, N->e, N->e}, S[3] = {N->s, N->s, N->s};
    const long long VE = cube(N->e), VS = cube(N->s), VQ = cube(N->q), VH = cube(N->h);
    auto gw = [&](int l) { return grads + N->w_off[l]; };
    auto gb = [&](int l) { return grads + N->b_off[l]; };
    AIR_TRY(air_cnn_output_bwd(dtheta, E, 16, kOutScale, f32(N->g_out), stream));
    AIR_TRY(air_cast_bf16(f32(N->g_out), b16(N->g_out_bf), VE * 16, stream));
    AIR_TRY(air_conv3d_bwd_weight(b16(N->d1), E, 48, b16(N->g_out_bf), 16, kBwdwChunk, gw(5),
                                  gb(5), bw, bwb, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->g_out_bf), E, 16, b16(N->wf[5]), nullptr, 48, 0, nullptr, 48, 0,
                           f32(N->g_d1), 48, stream));
    AIR_TRY(air_lrelu_bwd(f32(N->g_d1), 48, 0, b16(N->d1), 48, 0, VE, 48, b16(N->g_d1_bf),
                          stream));
    AIR_TRY(air_conv3d_bwd_weight(b16(N->cat), E, kCat, b16(N->g_d1_bf), 48, kBwdwChunk, gw(4),
                                  gb(4), bw, bwb, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->g_d1_bf), E, 48, b16(N->wf[4]), nullptr, kCat, 0, nullptr,
                           kCat, 0, f32(N->g_cat), kCat, stream));
    // the decoder input is [a3 | up2(a4)]
    AIR_TRY(air_up2_bwd(f32(N->g_cat), S, 64, kCat, 48, f32(N->g_a4), stream));
    AIR_TRY(air_lrelu_bwd(f32(N->g_a4), 64, 0, b16(N->a4), 64, 0, VS, 64, b16(N->g_a4_bf),
                          stream));
    AIR_TRY(air_conv3d_bwd_weight(b16(N->p3), S, 48, b16(N->g_a4_bf), 64, kBwdwChunk, gw(3),
                                  gb(3), bw, bwb, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->g_a4_bf), S, 64, b16(N->wf[3]), nullptr, 48, 0, nullptr, 48, 0,
                           f32(N->g_p3), 48, stream));
    // a3 feeds both the decoder (g_cat[:, 0:48]) and the pool
    AIR_TRY(air_pool2_bwd(f32(N->g_p3), E, 48, f32(N->g_cat), kCat, 0, 1, stream));
    AIR_TRY(air_lrelu_bwd(f32(N->g_cat), kCat, 0, b16(N->cat), kCat, 0, VE, 48,
                          b16(N->g_a3_bf), stream));
    AIR_TRY(air_conv3d_bwd_weight(b16(N->p2), E, 32, b16(N->g_a3_bf), 48, kBwdwChunk, gw(2),
                                  gb(2), bw, bwb, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->g_a3_bf), E, 48, b16(N->wf[2]), nullptr, 32, 0, nullptr, 32, 0,
                           f32(N->g_p2), 32, stream));
    AIR_TRY(air_pool2_bwd(f32(N->g_p2), Q, 32, f32(N->g_a2), 32, 0, 0, stream));
    AIR_TRY(air_lrelu_bwd(f32(N->g_a2), 32, 0, b16(N->a2), 32, 0, VQ, 32, b16(N->g_a2_bf),
                          stream));
    AIR_TRY(air_conv3d_bwd_weight(b16(N->p1), Q, 16, b16(N->g_a2_bf), 32, kBwdwChunk, gw(1),
                                  gb(1), bw, bwb, stream));
    AIR_TRY(air_conv3d_fwd(b16(N->g_a2_bf), Q, 32, b16(N->wf[1]), nullptr, 16, 0, nullptr, 16, 0,
                           f32(N->g_p1), 16, stream));
    AIR_TRY(air_pool2_bwd(f32(N->g_p1), H, 16, f32(N->g_a1), 16, 0, 0, stream));
    AIR_TRY(air_lrelu_bwd(f32(N->g_a1), 16, 0, b16(N->a1), 16, 0, VH, 16, b16(N->g_a1_bf),
                          stream));
    return air_conv3d_bwd_weight(b16(N->x0), H, 8, b16(N->g_a1_bf), 16, kBwdwChunk, gw(0), gb(0),
                                 bw, bwb, stream);
}

}  // extern "C"
