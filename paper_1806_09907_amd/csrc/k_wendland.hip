// Wendland basis (Sec. III-C, psi_{3,2} with a support radius sigma per axis)
// expanded onto the voxel grid, u = B theta (Sec. II-A eq. kernel_basis), and
// its transpose, B^T g.
//
// Control j sits at (j - m) delta on each axis, so the lattice is aligned
// with voxel cells of size delta: voxel x = c delta + r (cell c, phase r in
// [0, delta)) sees exactly the controls j = c + qq, qq in [0, K), with the
// weight W[qq][r] = psi(||(r - (qq - m) delta) / sigma||), the same for
// every cell. Both directions are therefore per-cell contractions with one
// fixed table, built once per plan on the host:
//   expand:    u(c, r) = sum_qq W[qq][r] theta(c + qq)
//   transpose: H(qq, c) = sum_r W[qq][r] g(c, r) (in two partial sums over
//              halves of the phases);
//              out(j)   = sum_qq H(j - qq, qq)   over cells inside the grid.
// No kernel value is evaluated on the device.
#include "device_common.h"

namespace air {

namespace {

constexpr int kWCells = 16;  // cells along x per wave (one MFMA tile; both contractions)
constexpr int kWaves = kBlock / 64;
constexpr int kTSplit = 2;   // blocks sharing one cell group's phases in the transpose

// theta -> zero-padded copy [d][ncp_z][ncp_y][ncp_x], scaled.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_pad(const PairDesc P, const float* __restrict__ theta, float scale,
           float* __restrict__ thp) {
    const long long nx = P.wncp[0], ny = P.wncp[1], nz = P.wncp[2];
    const long long tot = DIM * nx * ny * nz;
    const long long NC = (long long)P.nc[0] * P.nc[1] * P.nc[2];
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < tot;
         i += (long long)gridDim.x * kBlock) {
        const int jx = (int)(i % nx);
        const int jy = (int)((i / nx) % ny);
        const long long rest = i / (nx * ny);
        const int jz = (int)(rest % nz);
        const int c = (int)(rest / nz);
        float v = 0.f;
        if (jx < P.nc[0] && jy < P.nc[1] && jz < P.nc[2])
            v = scale * theta[c * NC + ((long long)jz * P.nc[1] + jy) * P.nc[0] + jx];
        thp[i] = v;
    }
}

// Per-axis coordinates (x fastest) of a linear index i in an nx x ny x .
// grid, and their update for i += 4 (the step of every lane in the loops
// below), so that no loop divides.
struct Idx3 {
    int x, y, z;
};
__device__ inline Idx3 idx3(int i, int nx, int ny) {
    return Idx3{i % nx, (i / nx) % ny, i / (nx * ny)};
}
__device__ inline void idx3_add(Idx3& c, int step, int nx, int ny) {
    c.x += step;
    while (c.x >= nx) {
        c.x -= nx;
        ++c.y;
    }
    while (c.y >= ny) {
        c.y -= ny;
        ++c.z;
    }
}
__device__ inline void idx3_add4(Idx3& c, int nx, int ny) {
    c.x += 4;
    while (c.x >= nx) {
        c.x -= nx;
        ++c.y;
    }
    while (c.y >= ny) {
        c.y -= ny;
        ++c.z;
    }
}

// Both contractions run on v_mfma_f32_16x16x4f32 (full FP32). Lane l holds
// A[l % 16][l / 16] of the 16x4 A tile, B[l / 16][l % 16] of the 4x16 B tile
// and D[4 (l / 16) + v][l % 16], v = 0..3, of the 16x16 result.
__device__ inline v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// u(c, r) = sum_qq W[qq][r] thp(c + qq): per wave M = 64 phases (4 tiles),
// N = kWCells cells (one tile per component), K = the controls qq.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_expand(const PairDesc P, const float* __restrict__ W, const float* __restrict__ thp,
              float* __restrict__ u) {
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    const int npc = P.wpad[0] / 64;             // phase chunks
    const int ngx = cdiv(P.wncell[0], kWCells);
    const int ngroups = ngx * P.wncell[1] * P.wncell[2];
    if (gw >= ngroups * npc) return;
    const int pc = gw % npc;
    const int g = gw / npc;
    const int cx0 = (g % ngx) * kWCells;
    const int cy = (g / ngx) % P.wncell[1];
    const int cz = g / (ngx * P.wncell[1]);
    const int Ppad = P.wpad[0];
    const int Q = P.wK[0] * P.wK[1] * P.wK[2];
    const long long sx = P.wncp[0], sy = (long long)P.wncp[0] * P.wncp[1];
    const long long NCp = sy * P.wncp[2];
    v4f acc[4][DIM];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[m][c] = v4f{0.f, 0.f, 0.f, 0.f};
    const float* Wr = W + pc * 64 + i16;
    const int isy = (int)sy, isx = (int)sx, incp = (int)NCp;   // offsets fit in 32 bits
    const float* thb = thp + cx0 + i16;
    // operands of the K step whose control for this lane is q (coordinates
    // qc). Branch-free: a control past Q reads a valid address and is zeroed
    // where it is used, so the loads stay in flight until then.
    auto load = [&](int q, const Idx3& qc, float* a, float* b, bool& ok) {
        const int qw = min(q, P.wpad[1] - 1);  // rows >= Q are 0; past the end: clamped
#pragma unroll
        for (int m = 0; m < 4; ++m) a[m] = Wr[qw * Ppad + m * 16];
        ok = q < Q;
        // a mask, not a branch: the loads must not wait for a join
        const int off = ((cz + qc.z) * isy + (cy + qc.y) * isx + qc.x) & -(int)ok;
#pragma unroll
        for (int c = 0; c < DIM; ++c) b[c] = thb[off + c * incp];
    };
    auto step = [&](const float* a, const float* b, bool ok) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[m][c] = mfma4(a[m], ok ? b[c] : 0.f, acc[m][c]);
    };
    // two operand sets rotate over an even number of K steps (a padding step
    // past Q contributes 0): each set is reloaded right after its MFMAs
    // issue, so its loads have a whole step of MFMAs to land
    const int nst = ((Q + 3) / 4 + 1) & ~1;
    Idx3 qn = idx3(k4, P.wK[0], P.wK[1]);
    float a0[4], b0[DIM], a1[4], b1[DIM];
    bool ok0, ok1;
    load(k4, qn, a0, b0, ok0);
    for (int st = 0; st < nst; st += 2) {
        idx3_add4(qn, P.wK[0], P.wK[1]);
        load((st + 1) * 4 + k4, qn, a1, b1, ok1);
        step(a0, b0, ok0);
        idx3_add4(qn, P.wK[0], P.wK[1]);
        load((st + 2) * 4 + k4, qn, a0, b0, ok0);
        step(a1, b1, ok1);
    }
    const int P3 = P.sp[0] * P.sp[1] * P.sp[2];
    const long long N = P.nvox;
    const int x0 = (cx0 + i16) * P.sp[0];
    // phases r = pc 64 + 16 m + 4 k4 + v in increasing order, coordinates stepped
    Idx3 rc = idx3(pc * 64 + 4 * k4, P.sp[0], P.sp[1]);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (m + v > 0) idx3_add(rc, v == 0 ? 13 : 1, P.sp[0], P.sp[1]);
            const int r = pc * 64 + m * 16 + 4 * k4 + v;
            if (r >= P3) continue;
            const int x = x0 + rc.x, y = cy * P.sp[1] + rc.y, z = cz * P.sp[2] + rc.z;
            if (x >= P.n[0] || y >= P.n[1] || z >= P.n[2]) continue;
            const long long vox = ((long long)z * P.n[1] + y) * P.n[0] + x;
#pragma unroll
            for (int c = 0; c < DIM; ++c) u[c * N + vox] = acc[m][c][v];
        }
}

// H(qq, c) = sum_r W[qq][r] g(c, r) for kWCells cells along x and 64 values
// of qq: per wave M = 64 qq (4 tiles), N = kWCells cells (one tile per
// component), K = the phases, split over the block's waves; the waves'
// results are added in LDS in a fixed order.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_cells_t(const PairDesc P, const float* __restrict__ WT, const float* __restrict__ g,
               float* __restrict__ H) {
    constexpr int NA = 4 * DIM * 4;   // accumulator floats per lane
    __shared__ float red[kWaves * 64 * NA];
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int w = threadIdx.x >> 6;
    const int nqc = P.wpad[1] / 64;
    const int ngx = cdiv(P.wncell[0], kWCells);
    const int part = blockIdx.x % kTSplit;     // which share of the phases
    const int qc = (blockIdx.x / kTSplit) % nqc;
    const int grp = blockIdx.x / (kTSplit * nqc);
    const int cx0 = (grp % ngx) * kWCells;
    const int cy = (grp / ngx) % P.wncell[1];
    const int cz = grp / (ngx * P.wncell[1]);
    const int Qpad = P.wpad[1];
    const int P3 = P.sp[0] * P.sp[1] * P.sp[2];
    const int nstep = P.wpad[0] / 4;
    const int nsub = kTSplit * kWaves;         // K ranges: one per wave of the split blocks
    const int s0 = (part * kWaves + w) * nstep / nsub, s1 = (part * kWaves + w + 1) * nstep / nsub;
    const long long N = P.nvox;
    const int cxl = cx0 + i16;                 // this lane's cell of the B tile
    const bool cell_ok = cxl < P.wncell[0];
    v4f acc[4][DIM];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[m][c] = v4f{0.f, 0.f, 0.f, 0.f};
    const float* Wq = WT + qc * 64 + i16;
    const int nx = P.n[0], nxy = P.n[0] * P.n[1], iN = (int)N;  // < 2^31 (plan check)
    const int bx = cxl * P.sp[0], by = cy * P.sp[1], bz = cz * P.sp[2];
    // operands of the K step whose phase for this lane is r (coordinates rc).
    // Branch-free: a phase outside the grid reads voxel 0 and is zeroed where
    // it is used, so the loads stay in flight until then.
    auto load = [&](int r, const Idx3& rc, float* a, float* b, bool& ok) {
        const int rw = min(r, P.wpad[0] - 1);  // rows >= P3 are 0; past the end: clamped
#pragma unroll
        for (int m = 0; m < 4; ++m) a[m] = Wq[rw * Qpad + m * 16];
        const int x = bx + rc.x, y = by + rc.y, z = bz + rc.z;
        ok = r < P3 && cell_ok && x < P.n[0] && y < P.n[1] && z < P.n[2];
        // a mask, not a branch: the loads must not wait for a join
        const int vox = (z * nxy + y * nx + x) & -(int)ok;
#pragma unroll
        for (int c = 0; c < DIM; ++c) b[c] = g[c * iN + vox];
    };
    auto step = [&](const float* a, const float* b, bool ok) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[m][c] = mfma4(a[m], ok ? b[c] : 0.f, acc[m][c]);
    };
    // two operand sets rotate over an even number of K steps (a padding step
    // past this wave's range contributes 0): each set is reloaded right after
    // its MFMAs issue, so its loads have a whole step of MFMAs to land
    const int s2 = s0 + ((s1 - s0 + 1) & ~1);
    Idx3 rn = idx3(s0 * 4 + k4, P.sp[0], P.sp[1]);
    float a0[4], b0[DIM], a1[4], b1[DIM];
    bool ok0, ok1;
    load(s0 * 4 + k4, rn, a0, b0, ok0);
    ok0 = ok0 && s0 < s1;
    for (int st = s0; st < s2; st += 2) {
        idx3_add4(rn, P.sp[0], P.sp[1]);
        load((st + 1) * 4 + k4, rn, a1, b1, ok1);
        ok1 = ok1 && st + 1 < s1;
        step(a0, b0, ok0);
        idx3_add4(rn, P.sp[0], P.sp[1]);
        load((st + 2) * 4 + k4, rn, a0, b0, ok0);
        ok0 = ok0 && st + 2 < s1;
        step(a1, b1, ok1);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(w * 64 + lane) * NA + (m * DIM + c) * 4 + v] = acc[m][c][v];
    __syncthreads();
    const int Q = P.wK[0] * P.wK[1] * P.wK[2];
    const long long ncells = (long long)P.wncell[0] * P.wncell[1] * P.wncell[2];
    const long long row = ((long long)cz * P.wncell[1] + cy) * P.wncell[0] + cx0;
    // consecutive threads take consecutive cells of one (component, qq) row
    for (int o = threadIdx.x; o < 64 * kWCells * DIM; o += kBlock) {
        const int t = o % kWCells;
        const int c = (o / kWCells) % DIM;
        const int ql = o / (kWCells * DIM);
        const int m = ql / 16, k4o = (ql % 16) / 4, v = ql % 4;
        const int src = (k4o * 16 + t) * NA + (m * DIM + c) * 4 + v;
        float sum = 0.f;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) sum += red[ww * 64 * NA + src];
        const int qv = qc * 64 + ql;
        if (qv < Q && cx0 + t < P.wncell[0])
            H[(((long long)part * DIM + c) * Q + qv) * ncells + row + t] = sum;
    }
}

// out(j) (+)= scale * sum_qq H(j - qq, qq) over cells inside the grid, with
// H laid out [d][K^d][cells]. A block takes 64 consecutive controls (one per
// lane, so a wave reads consecutive cells) and splits qq over its waves; the
// partial sums are added in a fixed order.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_wend_gather(const PairDesc P, const float* __restrict__ H, float scale, int accumulate,
              float* __restrict__ out) {
    __shared__ float red[kWaves][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const long long NC = (long long)P.nc[0] * P.nc[1] * P.nc[2];
    const long long ncells = (long long)P.wncell[0] * P.wncell[1] * P.wncell[2];
    const int Q = P.wK[0] * P.wK[1] * P.wK[2];
    const long long i = (long long)blockIdx.x * 64 + lane;   // (component, control)
    float s = 0.f;
    if (i < DIM * NC) {
        const int c = (int)(i / NC);
        const long long j = i % NC;
        const int jx = (int)(j % P.nc[0]);
        const int jy = (int)((j / P.nc[0]) % P.nc[1]);
        const int jz = (int)(j / ((long long)P.nc[0] * P.nc[1]));
        const long long hpart = (long long)DIM * Q * ncells;   // one share of the phases
        const float* Hc = H + (long long)c * Q * ncells;
        Idx3 qi = idx3(w, P.wK[0], P.wK[1]);
        for (int qq = w; qq < Q; qq += kWaves, idx3_add4(qi, P.wK[0], P.wK[1])) {
            const int cx = jx - qi.x, cy = jy - qi.y, cz = jz - qi.z;
            if (cx < 0 || cx >= P.wncell[0] || cy < 0 || cy >= P.wncell[1] || cz < 0 ||
                cz >= P.wncell[2])
                continue;
            const long long o =
                (long long)qq * ncells + ((long long)cz * P.wncell[1] + cy) * P.wncell[0] + cx;
#pragma unroll
            for (int pt = 0; pt < kTSplit; ++pt) s += Hc[pt * hpart + o];
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && i < DIM * NC) {
        float t = 0.f;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) t += red[ww][lane];
        const float v = scale * t;
        out[i] = accumulate ? out[i] + v : v;
    }
}

__host__ inline int wend_grid(long long n) {
    const long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

// u = scale * B theta. thp: d * prod(wncp) floats of workspace; W: the
// [wpad0][...] table in the plan's constants.
hipError_t launch_wendland_expand(const PairDesc& P, const float* consts_dev, int dim,
                                  const float* theta, float scale, float* thp, float* u,
                                  hipStream_t s) {
    const long long np = (long long)dim * P.wncp[0] * P.wncp[1] * P.wncp[2];
    const float* W = consts_dev + P.wend_off[0];
    const int ngx = cdiv(P.wncell[0], kWCells);
    const long long waves = (long long)ngx * P.wncell[1] * P.wncell[2] * (P.wpad[0] / 64);
    const int blocks = (int)((waves + kWaves - 1) / kWaves);
    if (dim == 3) {
        hipLaunchKernelGGL(k_wend_pad<3>, dim3(wend_grid(np)), dim3(kBlock), 0, s, P, theta,
                           scale, thp);
        hipLaunchKernelGGL(k_wend_expand<3>, dim3(blocks), dim3(kBlock), 0, s, P, W, thp, u);
    } else {
        hipLaunchKernelGGL(k_wend_pad<2>, dim3(wend_grid(np)), dim3(kBlock), 0, s, P, theta,
                           scale, thp);
        hipLaunchKernelGGL(k_wend_expand<2>, dim3(blocks), dim3(kBlock), 0, s, P, W, thp, u);
    }
    return hipGetLastError();
}

// grad (+)= scale * B^T g. H: wendland_h_parts() * d * K^d * prod(wncell)
// floats of workspace.
hipError_t launch_wendland_adjoint(const PairDesc& P, const float* consts_dev, int dim,
                                   const float* g, float scale, float* H, float* grad,
                                   bool accumulate, hipStream_t s) {
    const float* WT = consts_dev + P.wend_off[1];
    const int ngx = cdiv(P.wncell[0], kWCells);
    const int blocks = ngx * P.wncell[1] * P.wncell[2] * (P.wpad[1] / 64) * kTSplit;
    const long long NC = (long long)dim * P.nc[0] * P.nc[1] * P.nc[2];
    const int gblocks = (int)((NC + 63) / 64);
    if (dim == 3) {
        hipLaunchKernelGGL(k_wend_cells_t<3>, dim3(blocks), dim3(kBlock), 0, s, P, WT, g, H);
        hipLaunchKernelGGL(k_wend_gather<3>, dim3(gblocks), dim3(kBlock), 0, s, P, H, scale,
                           accumulate ? 1 : 0, grad);
    } else {
        hipLaunchKernelGGL(k_wend_cells_t<2>, dim3(blocks), dim3(kBlock), 0, s, P, WT, g, H);
        hipLaunchKernelGGL(k_wend_gather<2>, dim3(gblocks), dim3(kBlock), 0, s, P, H, scale,
                           accumulate ? 1 : 0, grad);
    }
    return hipGetLastError();
}

// Cells along x per wave in both contractions (the padded control grid is
// rounded up to a multiple of it along x).
int wendland_cells_per_wave() { return kWCells; }
// Partial per-cell sums the transpose writes (summed by the gather).
int wendland_h_parts() { return kTSplit; }

}  // namespace air
