// Internal device/host structures of the airhip library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/airhip.h"
#include <rocprofiler-sdk-roctx/roctx.h>

namespace air {

// A roctx range over a host scope: the stages of an evaluation appear as
// named ranges in a marker trace (rocprofv3 --marker-trace); without a
// profiler attached the calls return at once.
// The network's first-layer convolution (channels 2.. of its 8 input
// channels zero) on 16 x 4 x 4 bricks; returns false when the shape does not
// allow it (the caller then uses air_conv3d_fwd), else launches on `s` and
// stores the launch status in *err.
bool conv3d_fwd_in2(const uint16_t* x, const int32_t dims[3], int32_t batch,
                    const uint16_t* wt, const float* bias, int32_t cout, int32_t act,
                    uint16_t* y_bf16, int32_t ldy, float* y_f32, int32_t ldyf, hipStream_t s,
                    hipError_t* err);

struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

constexpr int kMaxPairs = 4096;
constexpr int kMaxSpacing = 64;
constexpr int kBlock = 256;          // threads per block of every kernel
constexpr int kStatWords = 8;        // doubles per tile statistics slot
// dense-field passes: a block owns kDenseTX x kDenseTY voxels of (x, y) and
// walks kDenseZc of z
constexpr int kDenseTX = 64, kDenseTY = 4, kDenseZc = 32;

// Per-pair constants, uploaded once per plan and device.
struct PairDesc {
    int n[3];            // voxels (1 on absent axes)
    int nc[3];           // controls (1 on absent axes); for dense: n
    int sp[3];           // spacing (1 on absent axes)
    float s[3];          // (n - 1) / 2 : normalised -> voxel units
    int ntile[3];        // fused-kernel tiles along x, y and the column axis
    int col_cells;       // cells per column chunk
    int win[3];          // max control window of a tile (x, y, column)
    int tile_begin;      // global index of the pair's first tile
    int ntiles;          // tiles of this pair
    int reg_begin;       // global index of the pair's first regulariser block
    int nreg;            // regulariser blocks of this pair
    int part_stride;     // floats per tile partial
    long long part_off;  // float offset of the pair's partials
    long long nvox;
    long long nparam;    // parameters of the pair
    long long param_off; // float offset of the pair in the reg-grad buffer
    int gram_off[3];     // float offset of axis a's banded Gram tables (P then D)
    int wtab_off[3];     // float offset of axis a's spacing weight table [sp][4]
    float inv_xr;        // 1 / |X_R|
    float lambda;        // regulariser weight
    int regpart_off;     // double offset of the pair's regulariser partials
    int dense_blk_off;   // first dense stats block slot of the pair
    int dense_nblk;      // dense stats blocks of the pair
    // Wendland basis: voxel cells of size sp, each seeing controls c + [0, wK)
    int wncell[3];       // cells per axis, ceil(n / sp)
    int wK[3];           // controls a cell sees per axis
    int wncp[3];         // padded control grid of the expansion (zeros beyond nc)
    int wpad[2];         // phases prod(sp) and prod(wK), rounded up to 64
    int wend_off[2];     // float offsets of W [wpad1][wpad0] and W^T [wpad0][wpad1]
    int wpad_;
    // B-spline regulariser blocks: each handles reg_rows rows of one control
    // plane (reg_nband bands per plane; one band when the plane fits in LDS)
    int reg_rows;
    int reg_nband;
};

// Workspace layout (byte offsets into the caller's workspace).
struct WsLayout {
    size_t stats;        // double [ntiles_total][kStatWords]
    size_t part;         // float  [sum part]
    size_t reggrad;      // float  [sum nparam] (B-spline: lambda dR/dtheta)
    size_t regpart;      // double [sum regblocks]
    size_t flags;        // uint32 [npairs]
    size_t scalars;      // double [npairs][8] (dense: global count / coefficients)
    size_t dense_stats;  // double [sum dense blocks][kStatWords]
    size_t generic;      // double [generic blocks][kStatWords] (similarity / reg calls)
    size_t fields;       // float [K + 1][d N]: u_0 .. u_K of the exponential (K > 0)
    size_t gfield;       // float [2][d N]: gradients going back through the squarings
    size_t bsadj1;       // float [d][nz][ny][ncx]: transposed expansion, after x
                         // (Wendland: the padded, scaled controls)
    size_t bsadj2;       // float [d][nz][ncy][ncx]: after y
                         // (Wendland: per-cell sums H [d][cells][K^d])
    size_t reach;        // uint32 [K + 3]: largest displacement of each u_k, then two
                         // slots for the largest |gradient| entering and leaving a
                         // squaring's adjoint (float bits)
    size_t tvpart;       // double [TV blocks]: partial sums of a TV term
    // LCC passes (similarity AIR_SIM_LCC)
    size_t lcc_w;        // float [N]: warped image
    size_t lcc_mask;     // uint8 [N]: sample point inside the moving image
    size_t lcc_dw;       // float [d][N]: dW/dp (voxel units)
    size_t lcc_s;        // double [6][N]: box sums of the unfused passes (else empty)
    size_t lcc_a;        // float [3][N]: coefficient maps
    size_t lcc_part;     // double [2 * blocks]: (count, sum rho) per block
    size_t lcc_scal;     // double [1]: 1 / |X'|
    size_t total;
};

struct DeviceTables {
    PairDesc* pairs = nullptr;
    float* consts = nullptr;   // Gram tables + weight tables
    int device = -1;
};

struct LaunchCtx {
    const PairDesc* pairs;     // device
    const float* consts;       // device
    int npairs;
    int ntiles_total;
    int nreg_total;
    int dim;
    int sim;
    // single-pair pointers (used when the pointer tables are null)
    const float* fixed0;
    const float* moving0;
    const float* theta0;
    float* grad0;
    float* value0;
    const float* const* fixed_tab;
    const float* const* moving_tab;
    const float* const* theta_tab;
    float* const* grad_tab;
    float* values;
    unsigned char* ws;
    WsLayout L;
};

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }
// round a float count up to a multiple of 4 (16-byte aligned LDS carve-up)
__host__ __device__ inline int a4(int n) { return (n + 3) & ~3; }

// Tile window: controls [c0, c0 + w) touched by voxels [v0, v1) (v1 exclusive).
__host__ __device__ inline void ctrl_window(int v0, int v1, int sp, int* c0, int* w) {
    int a = v0 / sp;
    int b = (v1 - 1) / sp + 3;
    *c0 = a;
    *w = b - a + 1;
}

}  // namespace air
