// The learned-initialisation network as one object of the C-ABI: the layer
// schedule of a 3D encoder-decoder for a batch of n^3 pairs (n a multiple of
// 16), its parameter layout and its workspace, and the forward and backward
// passes sequenced over the library's BF16 MFMA convolutions and the
// pooling, upsampling and activation kernels (k_cnn.hip). The batch is one
// stack along z; the convolutions pad each volume on its own.
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
constexpr int kInUsed = 2;   // channels of x0 that carry data (F, M); the rest are zero

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
    int n = 0, batch = 1;
    int h = 0, q = 0, e = 0, s = 0;   // sides at n/2, n/4, n/8, n/16
    int w_off[kLayers] = {}, b_off[kLayers] = {};
    int64_t nparam = 0;
    // workspace byte offsets
    size_t wb[kLayers] = {}, wf[kLayers] = {};
    size_t x0, x0_xb, a1, p1, a2, p2, cat, p3, a4, d1, out;
    size_t g_out_bf, g_d1_bf, g_cat, g_a4_bf, g_p3, g_a3_bf, g_p2, g_a2_bf, g_p1, g_a1_xb, bwdw;
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

air_status air_cnn_create(int32_t n, int32_t batch, air_cnn** out) {
    if (!out) return AIR_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 16 || n % 16 || n > 1024 || batch < 1) return AIR_ERR_SHAPE;
    if (cube(n) * batch >= (1LL << 31)) return AIR_ERR_SHAPE;
    air_cnn* N = new (std::nothrow) air_cnn();
    if (!N) return AIR_ERR_DEVICE;
    N->n = n;
    N->batch = batch;
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
    const long long B = batch;
    const long long H = cube(N->h) * B, Q = cube(N->q) * B, E = cube(N->e) * B,
                    S = cube(N->s) * B;
    N->x0 = take(2 * H * 8);
    N->x0_xb = take(2 * H * 8);
    N->a1 = take(2 * H * 16);
    N->p1 = take(2 * Q * 16);
    N->a2 = take(2 * Q * 32);
    N->p2 = take(2 * E * 32);
    N->cat = take(2 * E * kCat);
    N->p3 = take(2 * S * 48);
    N->a4 = take(2 * S * 64);
    N->d1 = take(2 * E * 48);
    N->out = take(4 * E * 16);
    N->g_out_bf = take(2 * E * 16);
    N->g_d1_bf = take(2 * E * 48);
    N->g_cat = take(4 * E * kCat);
    N->g_a4_bf = take(2 * S * 64);
    N->g_p3 = take(4 * S * 48);
    N->g_a3_bf = take(2 * E * 48);
    N->g_p2 = take(4 * E * 32);
    N->g_a2_bf = take(2 * Q * 32);
    N->g_p1 = take(4 * Q * 16);
    N->g_a1_xb = take(2 * H * 16);
    size_t bw = 0;
    for (int l = 0; l < kLayers; ++l) {
        int32_t d[3];
        layer_dims(N, l, d);
        size_t b = 0;
        // the first layer takes x-blocked operands from its producers
        const air_status st =
            l == 0 ? air_conv3d_bwd_weight_xb_workspace(d, batch, kDef[l].cin, kInUsed,
                                                        kDef[l].cout, 0, &b)
                   : air_conv3d_bwd_weight_workspace(d, batch, kDef[l].cin, kDef[l].cout, 0, &b);
        if (st != AIR_OK) {
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
    TraceRange trace_("air_cnn_forward");
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
    const int B = N->batch;
    // stack sizes (pooling, upsampling, input) and one volume's (convolutions)
    const int32_t full[3] = {N->n, N->n, N->n * B};
    const int32_t Hs[3] = {N->h, N->h, N->h * B}, Qs[3] = {N->q, N->q, N->q * B};
    const int32_t Es[3] = {N->e, N->e, N->e * B}, Ss[3] = {N->s, N->s, N->s * B};
    const int32_t H[3] = {N->h, N->h, N->h}, Q[3] = {N->q, N->q, N->q};
    const int32_t E[3] = {N->e, N->e, N->e}, S[3] = {N->s, N->s, N->s};
    auto conv = [&](const uint16_t* x, const int32_t* d, int l, uint16_t* ybf, int ldy,
                    float* yf) {
        return air_conv3d_fwd(x, d, B, kDef[l].cin, b16(N->wb[l]), params + N->b_off[l],
                              kDef[l].cout, kDef[l].act, nullptr, 0, 0, ybf, ldy, 0, yf,
                              kDef[l].cout, stream);
    };
    AIR_TRY(air_cnn_input(fixed, moving, full, b16(N->x0), b16(N->x0_xb), stream));
    {
        // the first layer reads only the two data channels of x0
        hipError_t err = hipSuccess;
        if (conv3d_fwd_in2(b16(N->x0), H, B, b16(N->wb[0]), params + N->b_off[0], 16, 1,
                           b16(N->a1), 16, nullptr, 16, s, &err)) {
            if (err != hipSuccess) return AIR_ERR_LAUNCH;
        } else {
            AIR_TRY(conv(b16(N->x0), H, 0, b16(N->a1), 16, nullptr));
        }
    }
    AIR_TRY(air_pool2(b16(N->a1), Hs, 16, 16, 0, b16(N->p1), stream));
    AIR_TRY(conv(b16(N->p1), Q, 1, b16(N->a2), 32, nullptr));
    AIR_TRY(air_pool2(b16(N->a2), Qs, 32, 32, 0, b16(N->p2), stream));
    AIR_TRY(conv(b16(N->p2), E, 2, b16(N->cat), kCat, nullptr));
    AIR_TRY(air_pool2(b16(N->cat), Es, 48, kCat, 0, b16(N->p3), stream));
    AIR_TRY(conv(b16(N->p3), S, 3, b16(N->a4), 64, nullptr));
    AIR_TRY(air_up2(b16(N->a4), Ss, 64, b16(N->cat), kCat, 48, stream));
    AIR_TRY(conv(b16(N->cat), E, 4, b16(N->d1), 48, nullptr));
    AIR_TRY(conv(b16(N->d1), E, 5, nullptr, 16, f32(N->out)));
    return air_cnn_output(f32(N->out), E, B, 16, kOutScale, theta0, stream);
}

air_status air_cnn_backward(const air_cnn* N, const float* dtheta, float* grads, void* ws,
                            size_t ws_bytes, void* stream) {
    TraceRange trace_("air_cnn_backward");
    if (!N || !dtheta || !grads) return AIR_ERR_INVALID_ARG;
    if (!ws || ws_bytes < N->total) return AIR_ERR_WORKSPACE;
    if (((uintptr_t)ws | (uintptr_t)dtheta | (uintptr_t)grads) & 15u) return AIR_ERR_ALIGN;
    unsigned char* w = static_cast<unsigned char*>(ws);
    auto b16 = [&](size_t off) { return reinterpret_cast<uint16_t*>(w + off); };
    auto f32 = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
    void* bw = w + N->bwdw;
    const size_t bwb = N->bwdw_bytes;
    const int B = N->batch;
    const int32_t H[3] = {N->h, N->h, N->h}, Q[3] = {N->q, N->q, N->q};
    const int32_t E[3] = {N->e, N->e, N->e}, S[3] = {N->s, N->s, N->s};
    const int32_t Hs[3] = {N->h, N->h, N->h * B}, Qs[3] = {N->q, N->q, N->q * B};
    const int32_t Es[3] = {N->e, N->e, N->e * B}, Ss[3] = {N->s, N->s, N->s * B};
    // weight and bias gradient of layer l from its input x and output gradient dy
    auto bwdw = [&](const uint16_t* x, const int32_t* d, int l, const uint16_t* dy) {
        return air_conv3d_bwd_weight(x, d, B, kDef[l].cin, dy, kDef[l].cout, 0,
                                     grads + N->w_off[l], grads + N->b_off[l], bw, bwb, stream);
    };
    // input gradient of layer l (flipped weights), optionally through the
    // activation `gate` of the layer below (act 2), as bf16 or FP32
    auto bwdd = [&](const uint16_t* dy, const int32_t* d, int l, const uint16_t* gate, int ldg,
                    uint16_t* dxbf, float* dxf) {
        return air_conv3d_fwd(dy, d, B, kDef[l].cout, b16(N->wf[l]), nullptr, kDef[l].cin,
                              gate ? 2 : 0, gate, ldg, 0, dxbf, kDef[l].cin, 0, dxf, kDef[l].cin,
                              stream);
    };
    AIR_TRY(air_cnn_output_bwd(dtheta, E, B, 16, kOutScale, nullptr, b16(N->g_out_bf), stream));
    AIR_TRY(bwdw(b16(N->d1), E, 5, b16(N->g_out_bf)));
    AIR_TRY(bwdd(b16(N->g_out_bf), E, 5, b16(N->d1), 48, b16(N->g_d1_bf), nullptr));
    AIR_TRY(bwdw(b16(N->cat), E, 4, b16(N->g_d1_bf)));
    AIR_TRY(bwdd(b16(N->g_d1_bf), E, 4, nullptr, 0, nullptr, f32(N->g_cat)));
    // the decoder input is [a3 | up2(a4)]
    AIR_TRY(air_up2_lrelu_bwd(f32(N->g_cat), Ss, 64, kCat, 48, b16(N->a4), 64, 0,
                              b16(N->g_a4_bf), stream));
    AIR_TRY(bwdw(b16(N->p3), S, 3, b16(N->g_a4_bf)));
    AIR_TRY(bwdd(b16(N->g_a4_bf), S, 3, nullptr, 0, nullptr, f32(N->g_p3)));
    // a3 feeds both the decoder (g_cat[:, 0:48]) and the pool
    AIR_TRY(air_pool2_lrelu_bwd(f32(N->g_p3), Es, 48, f32(N->g_cat), kCat, 0, b16(N->cat), kCat,
                                0, 0, b16(N->g_a3_bf), stream));
    AIR_TRY(bwdw(b16(N->p2), E, 2, b16(N->g_a3_bf)));
    AIR_TRY(bwdd(b16(N->g_a3_bf), E, 2, nullptr, 0, nullptr, f32(N->g_p2)));
    AIR_TRY(air_pool2_lrelu_bwd(f32(N->g_p2), Qs, 32, nullptr, 0, 0, b16(N->a2), 32, 0, 0,
                                b16(N->g_a2_bf), stream));
    AIR_TRY(bwdw(b16(N->p1), Q, 1, b16(N->g_a2_bf)));
    AIR_TRY(bwdd(b16(N->g_a2_bf), Q, 1, nullptr, 0, nullptr, f32(N->g_p1)));
    // the first layer's output gradient feeds only its weight gradient:
    // written x-blocked, beside the x-blocked input of the forward pass
    AIR_TRY(air_pool2_lrelu_bwd(f32(N->g_p1), Hs, 16, nullptr, 0, 0, b16(N->a1), 16, 0, 1,
                                b16(N->g_a1_xb), stream));
    return air_conv3d_bwd_weight_xb(b16(N->x0_xb), H, B, kDef[0].cin, kInUsed, b16(N->g_a1_xb),
                                    kDef[0].cout, 0, grads + N->w_off[0], grads + N->b_off[0], bw,
                                    bwb, stream);
}

}  // extern "C"
