/*
 * airhip -- C-ABI of the MI355X (gfx950) library that evaluates the
 * regularised image-registration objective of AIRLab (arXiv 1806.09907)
 * and its gradient.
 *
 * The objective (Sec. II-A, eq. objective) is
 *     L(theta) = S(M o f_theta, F) + lambda * R(f_theta)
 * with
 *   f_theta   a cubic B-spline field on a control grid (Sec. II-A eq.
 *             kernel_basis, Sec. III-C kernel k_B1D) or a dense field
 *             (Sec. III-C "Non-linear/dense");
 *   M o f     backward warping in normalised [-1,1]^d coordinates with
 *             linear interpolation and out-of-domain points masked out
 *             (Sec. III-C "Image Warping");
 *   S         MSE (Sec. II-A eq. mse) or NCC (Sec. III-B; loss -rho, the
 *             Pearson correlation over the masked voxels);
 *   R         the diffusion regulariser (Sec. II-A eq. diffusion_regularizer);
 *   f = exp(v) optionally, for a stationary velocity field v given by either
 *             model (Sec. III-D), by scaling and squaring.
 *
 * Conventions (every entry point):
 *   - images are FP32 [nz][ny][nx], x fastest (2D: [ny][nx], n[2] == 1);
 *   - dense fields / parameters are FP32 [d][nz][ny][nx], components ordered
 *     (x, y, z); B-spline parameters are FP32 [d][ncz][ncy][ncx] with
 *     nc = floor((n - 1) / spacing) + 4, control j at voxel (j - 1) * spacing;
 *   - displacements and controls are in normalised units: the sample point of
 *     voxel i along axis a is p_a = i_a + u_a * (n_a - 1) / 2 voxels;
 *   - a voxel is in the mask iff 0 <= p_a <= n_a - 1 on every axis; the
 *     similarity is averaged over the masked voxels (N'); the mask is held
 *     constant when differentiating; interpolation uses the cell
 *     [floor(p), floor(p) + 1] with zero padding outside the volume. The
 *     kernels never round p itself: they take the cell and the mask on the
 *     exact sum of the integer i_a and the displacement in voxels
 *     d_a = u_a (n_a - 1) / 2, rounded once to FP32, plus (for dense fields,
 *     whose u is the input itself) that rounding's exact error, so dense
 *     decisions are those of the exact point;
 *   - R uses forward differences of u (normalised units) over
 *     X_R = prod_a [0, n_a - 2], divided by |X_R|;
 *   - all tensor pointers are caller-owned DEVICE buffers, 16-byte aligned,
 *     contiguous; outputs are overwritten; scalar outputs are device scalars;
 *   - calls are asynchronous on `stream` (a hipStream_t; NULL = default
 *     stream), do not synchronise the host and do not allocate, except the
 *     first launching call with a plan on a device, which uploads the plan's
 *     small constant tables (allocation + blocking copy) unless
 *     air_plan_prepare() ran first on that device;
 *   - argument errors return before any launch; a launch failure returns
 *     AIR_ERR_LAUNCH; degenerate or non-finite results set bits in a device
 *     flag word read by air_get_flags().
 */
#ifndef AIRHIP_H
#define AIRHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AIR_OK = 0,
    AIR_ERR_INVALID_ARG = 1,  /* null/unknown argument or enum value */
    AIR_ERR_SHAPE = 2,        /* sizes, spacing or pair index out of range */
    AIR_ERR_ALIGN = 3,        /* a tensor pointer is not 16-byte aligned */
    AIR_ERR_WORKSPACE = 4,    /* workspace missing or smaller than required */
    AIR_ERR_UNSUPPORTED = 5,  /* valid but not implemented combination */
    AIR_ERR_LAUNCH = 6,       /* the HIP runtime rejected a launch */
    AIR_ERR_NONFINITE = 7,    /* returned by air_get_flags-based checks */
    AIR_ERR_DEVICE = 8        /* device query, allocation or copy failed */
} air_status;

/* Similarities (Sec. II-A, III-B) over the masked set X' (sample points
 * inside the moving image): MSE; NCC (loss -rho, rho the Pearson correlation
 * of F and W over X'); LCC (local NCC: for x in X' the mean, variance and
 * covariance over N(x) = {y in X' : |y - x|_inf <= lcc_radius}, divided by
 * |N(x)|, rho(x) = cov / sqrt(varF varW + 1e-10), S = -mean of rho over X').
 * LCC plans hold one pair and evaluate the objective on the field expanded
 * to the voxel grid. */
enum { AIR_SIM_MSE = 0, AIR_SIM_NCC = 1, AIR_SIM_LCC = 2 };
/* Transformations: cubic B-spline (Sec. III-C, kernel k_B1D; control j at
 * voxel (j-1) delta, nc = floor((n-1)/delta) + 4 per axis), dense (one
 * vector per voxel), Wendland (Sec. III-C, psi_{3,2}(r) = (1-r)^6_+
 * (3 + 18r + 35r^2)/3 at r = ||(x - c_j) / sigma|| with sigma per axis;
 * control j at (j - m) delta with m = ceil(sigma/delta) - 1 and
 * nc = m + ceil((n - 1 + sigma)/delta) per axis: every control within sigma
 * of a voxel on that axis). Parameters are [d][ncz][ncy][ncx] (interpolating
 * bases) or [d][nz][ny][nx] (dense), components ordered (x, y, z). */
enum { AIR_TF_BSPLINE3 = 0, AIR_TF_DENSE = 1, AIR_TF_WENDLAND = 2 };
/* Regularisers on the displacement f (Sec. III-F), on the forward
 * differences D_a f_c(x) = f_c(x + e_a) - f_c(x) over X_R, divided by |X_R|:
 * diffusion sum_c sum_a D^2; anisotropic TV sum_c sum_a |D|; isotropic TV
 * sqrt(sum_c sum_a D^2) per voxel; TV takes the subgradient 0 at 0. */
enum { AIR_REG_DIFFUSION = 0, AIR_REG_ANISO_TV = 1, AIR_REG_ISO_TV = 2 };
/* device flag bits (per pair) */
enum { AIR_FLAG_NONFINITE = 1u, AIR_FLAG_DEGENERATE = 2u };

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t n[3];         /* voxels along x, y, z (n[2] == 1 in 2D), each in
                             2..65536, fewer than 2^29 in all and
                             n[1] * n[2] < 2^24 (AIR_ERR_SHAPE) */
    int32_t transform;    /* AIR_TF_* */
    int32_t spacing[3];   /* control spacing delta in voxels, 1..64 (B-spline,
                             Wendland) */
    int32_t similarity;   /* AIR_SIM_* */
    float lambda_diff;    /* weight of the regulariser, >= 0 */
    int32_t diffeo_steps; /* 0: f is the field itself. K in 1..16: f = exp(v)
                             (Sec. III-D, stationary velocity v = the field)
                             by scaling and squaring: u_0 = v / 2^K, then K
                             times u <- u(x) + u(x + u(x)), sampled like an
                             image (zero outside, no mask). R then acts on
                             f = u_K. Plans with K > 0 hold one pair. */
    int32_t regulariser;  /* AIR_REG_*; plans with a TV term hold one pair */
    float sigma[3];       /* Wendland support radius in voxels along x, y, z,
                             finite and > 0 (read only for AIR_TF_WENDLAND).
                             The voxel-to-control weight table has
                             prod_a delta_a * prod_a K_a entries, K_a the
                             controls a cell sees along axis a (about
                             2 sigma_a / delta_a + 1); plans beyond 2^21 entries
                             are AIR_ERR_UNSUPPORTED. Wendland plans hold one
                             pair and, like plans with K > 0, evaluate the
                             objective on the field expanded to the voxel grid;
                             air_warp is AIR_ERR_UNSUPPORTED for them (use
                             air_displacement and a dense plan). */
    int32_t lcc_radius;   /* LCC window radius in voxels, 1..8 (read only for
                             AIR_SIM_LCC) */
} air_problem;

/* Opaque plan: host tables for one pair or a batch of pairs that share
 * dim, transform and similarity (sizes, spacing and lambda may differ). */
typedef struct air_plan air_plan;

/* Create a plan for `npairs` problems (1 .. 4096). Host-only; no GPU needed. */
air_status air_plan_create(const air_problem* probs, int32_t npairs, air_plan** out);
void air_plan_destroy(air_plan* plan);
/* Upload the plan's constant tables to the current device (allocates once). */
air_status air_plan_prepare(air_plan* plan);
/* Bytes of caller-owned device workspace the launching calls need. */
air_status air_plan_workspace_bytes(const air_plan* plan, size_t* bytes);
/* Number of FP32 parameters of pair `pair` (d * prod(nc) or d * N). */
air_status air_plan_param_count(const air_plan* plan, int32_t pair, int64_t* count);
/* Tile configurations of the fused kernel (the autotuner's search space). A
 * new 3D plan whose pairs all have spacing 8 starts with 16 x 16 columns, the
 * longest column (16, 8, 4, 2 cells) that gives the launch 4096 tiles, else
 * the one with the most tiles; a 2D B-spline plan with the longest column
 * (16, 8, 4, 2, 1 cells) that gives 2048 tiles, else the most tiles; other
 * plans start with configuration 0. */
int32_t air_tiling_count(int32_t dim);
air_status air_tiling_describe(int32_t dim, int32_t id, int32_t* tile_x, int32_t* tile_y,
                               int32_t* column_cells);
/* Select a tile configuration; changes the workspace size and re-uploads. */
air_status air_plan_set_tiling(air_plan* plan, int32_t id);
air_status air_plan_get_tiling(const air_plan* plan, int32_t* id);

/* Stage 1 + 2 (Sec. III-C Image Warping): warped = M(x + u(x)) with zero
 * padding everywhere (also outside the mask); mask (nullable) = 1 where the
 * sample point lies inside the volume. For pair `pair` of the plan.
 * Diffeomorphic plans return AIR_ERR_UNSUPPORTED: materialise f with
 * air_displacement and warp with a dense plan of the same size. */
air_status air_warp(const air_plan* plan, int32_t pair, const float* moving,
                    const float* theta, float* warped, uint8_t* mask, void* stream);

/* Stage 1 (Sec. II-A eq. kernel_basis, Sec. III-C, Sec. III-D): the dense
 * displacement u = f_theta [d][nz][ny][nx] in normalised units -- B theta,
 * theta, or their exponential for diffeomorphic plans. ws may be NULL for
 * plans without the exponential. */
air_status air_displacement(const air_plan* plan, int32_t pair, const float* theta, float* u,
                            void* ws, size_t ws_bytes, void* stream);

/* Stage 3 (Sec. II-A eq. mse / Sec. III-B NCC): similarity of `warped`
 * against `fixed` over the voxels where mask != 0 (mask nullable = all). */
air_status air_similarity(const air_plan* plan, int32_t pair, const float* fixed,
                          const float* warped, const uint8_t* mask, float* value,
                          void* ws, size_t ws_bytes, void* stream);

/* Stage 4 (Sec. II-A eq. diffusion_regularizer; Sec. III-F for the TV
 * terms): R(theta) of the plan's regulariser kind and, if grad is not NULL,
 * dR/dtheta (not scaled by lambda). Dense plans require grad
 * (AIR_ERR_INVALID_ARG otherwise). */
air_status air_regulariser(const air_plan* plan, int32_t pair, const float* theta,
                           float* value, float* grad, void* ws, size_t ws_bytes,
                           void* stream);

/* Stages 1-5 (Sec. II-A eq. objective): value = S + lambda R and
 * grad = dL/dtheta, for a plan with exactly one pair. */
air_status air_objective_and_grad(const air_plan* plan, const float* fixed,
                                  const float* moving, const float* theta,
                                  float* value, float* grad, void* ws, size_t ws_bytes,
                                  void* stream);

/* air_objective_and_grad for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the workspace taken from a library-owned
 * device array of AIR_NOALLOC_SCRATCH_BYTES per GPU (held from the library's
 * load on that GPU until the process ends) instead of a caller buffer. The
 * call allocates nothing: the plan's tables must already be on the current
 * device (air_plan_prepare, or an earlier launching call there), else
 * AIR_ERR_DEVICE; plans whose air_plan_workspace_bytes exceeds
 * AIR_NOALLOC_SCRATCH_BYTES return AIR_ERR_WORKSPACE (e.g. 128^3 B-spline
 * NCC needs 2.4 MiB, 256^3 18.4 MiB, 256^3 dense 0.2 MiB; plans with the
 * exponential need their fields and rarely fit). Every call on a GPU uses
 * that GPU's one array: calls that overlap on one GPU (on different streams
 * or threads) race and must be serialised by the caller. */
#define AIR_NOALLOC_SCRATCH_BYTES (32u << 20)
air_status air_objective_and_grad_noalloc(const air_plan* plan, const float* fixed,
                                          const float* moving, const float* theta, float* value,
                                          float* grad, void* stream);

/* The same for every pair of the plan in one launch sequence. fixed, moving,
 * theta and grads are DEVICE arrays of npairs device pointers; values is a
 * device array of npairs floats. */
air_status air_objective_and_grad_batched(const air_plan* plan,
                                          const float* const* fixed,
                                          const float* const* moving,
                                          const float* const* theta, float* values,
                                          float* const* grads, void* ws, size_t ws_bytes,
                                          void* stream);

/* Tile autotuner of the fused B-spline launch (not in the paper; the plan's
 * tile configuration, air_plan_set_tiling, only changes the summation
 * order). air_autotune runs every configuration valid for the plan once on
 * the caller's batch (arguments as air_objective_and_grad_batched; ws of at
 * least air_autotune_workspace_bytes) and checks that its values and
 * gradients agree with the first one's to 1e-5 relative (norm-wise per pair;
 * summation order alone moves them by up to ~1.3e-6). It then runs the batch
 * for about 0.1 s (the GPU's clock ramps up under sustained load) and times
 * every agreeing configuration in two rounds, each one upload call and two
 * warm-up launches then `reps` launches between two HIP events on `stream`,
 * keeping each configuration's faster reading; keeps the fastest one in
 * the plan (*chosen, *kernel_ms per launch) and, when cache_path is not NULL,
 * writes it into that JSON file under the plan's key (GPU architecture,
 * dimension, transform, similarity, spacing and size buckets of the batch),
 * keeping the file's other entries. Synchronises the host; B-spline plans
 * with the diffusion regulariser only (AIR_ERR_UNSUPPORTED otherwise).
 * air_autotune_cached applies the cached configuration of the plan's key if
 * the file has one (*tiling = its id, else -1). */
air_status air_autotune_workspace_bytes(const air_plan* plan, size_t* bytes);
air_status air_autotune(air_plan* plan, const float* const* fixed, const float* const* moving,
                        const float* const* theta, float* values, float* const* grads, void* ws,
                        size_t ws_bytes, int32_t reps, const char* cache_path, int32_t* chosen,
                        double* kernel_ms, void* stream);
air_status air_autotune_cached(air_plan* plan, const char* cache_path, int32_t* tiling);

/* Adam (Sec. III-G; Kingma & Ba) with bias correction, in place:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * theta -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). step >= 1. */
air_status air_adam_step(float* theta, const float* grad, float* m, float* v, int64_t n,
                         float lr, float b1, float b2, float eps, int32_t step,
                         void* stream);

/* The bias-corrected step sizes of Adam step `step` (>= 1), as air_adam_step
 * uses them: out[0] = lr / (1 - b1^step), out[1] = 1 / sqrt(1 - b2^step),
 * computed in double and rounded to float. Host only. */
air_status air_adam_bias_terms(float lr, float b1, float b2, int32_t step, float* out);

/* air_adam_step with the two factors of air_adam_bias_terms read from the
 * device array coef[2] (8-byte aligned) when the kernel runs, so that one
 * captured HIP graph of an optimisation loop serves every step: the caller
 * refreshes coef between replays. Same arithmetic and rounding as
 * air_adam_step with those factors. */
air_status air_adam_step_dev(float* theta, const float* grad, float* m, float* v, int64_t n,
                             const float* coef, float b1, float b2, float eps, void* stream);

/* x[i] *= *s for i < n, with s a device scalar (autograd chain rule). */
air_status air_scale(float* x, const float* s, int64_t n, void* stream);

/* Copy the per-pair flag words (AIR_FLAG_*) of the last launching call to
 * host memory `flags` [npairs]; synchronises `stream`. */
air_status air_get_flags(const air_plan* plan, const void* ws, uint32_t* flags,
                         void* stream);

/* Multi-resolution (Sec. IV-A: the FFD experiment's multi-resolution
 * strategy). One Gaussian pyramid level of a 3D volume in = [n2][n1][n0]:
 * separable Gaussian of std `sigma` voxels (taps to ceil(3 sigma), weights
 * normalised, borders clamped), then every second voxel from 0; out has
 * extent (n_a + 1) / 2 per axis. Needs air_pyramid_workspace_bytes(n) of
 * caller-owned device scratch. */
air_status air_pyramid_workspace_bytes(const int32_t n[3], size_t* bytes);
air_status air_pyramid_down(const float* in, const int32_t n[3], float sigma, float* out,
                            void* ws, size_t ws_bytes, void* stream);
/* Linear transfer of a displacement field [3][n2][n1][n0] (normalised units,
 * so no rescaling) to the grid m: voxel j of m samples the point
 * j (n - 1) / (m - 1) of n (align-corners convention). */
air_status air_field_resample(const float* in, const int32_t n[3], const int32_t m[3],
                              float* out, void* stream);

/* Bounds checks of the debug build (libairhip_debug.so, compiled with
 * -DAIR_DEBUG_BOUNDS): the kernels check their computed gather indices
 * against their buffers and record a violation as a bit instead of reading
 * out of range (bit 0: fused B-spline moving-image gathers, 1: fixed-image
 * loads, 2: dense/warp sampler gathers, 3: exponential squaring gathers,
 * 4: CNN convolution loads, 5: CNN weight-gradient loads, 6: fused B-spline
 * control-window loads). This call waits
 * for the device, returns the bits set since the last call in *flags and
 * clears them. The regular library returns AIR_ERR_UNSUPPORTED. */
air_status air_debug_bounds_take(uint32_t* flags);

/* ---- Learned initialisation CNN (BF16 operands, FP32 accumulation). ----
 * Not part of the paper's method: the paper lists learning-based
 * registration as an upcoming feature (Sec. III-I). A small 3D encoder-
 * decoder maps a fixed/moving pair to a starting control grid that the
 * plain registration then refines.
 * Activations are NDHWC bf16 (uint16_t storage) [z][y][x][C], C a multiple
 * of 8; weights are Wt[co][k], k = tap * C_in + ci, tap = (dz*3+dy)*3+dx.
 *
 * A batch of volumes is a stack along z: dims = (nx, ny, nz) of one volume,
 * the tensor holds batch * nz planes, and the 3x3x3 convolutions pad each
 * volume with zeros on its own (no tap reaches into a neighbour). The
 * pooling, upsampling and elementwise calls below are independent per
 * volume when nz is even, so they take the whole stack as one volume of
 * depth batch * nz.
 *
 * 3x3x3 convolution, stride 1, zero padding 1, on BF16 MFMA (16x16x32)
 * with FP32 accumulation: v = conv(x) + bias, then act 0: y = v; act 1:
 * y = LeakyReLU_0.1(v); act 2: y = v * LeakyReLU_0.1'(a) with a the stored
 * bf16 activation gate[v * ldg + goff + co] (for backward-data through an
 * activation; gate unused otherwise). Outputs (either may be NULL): bf16
 * y_bf16[v * ldy + yoff + co] and FP32 y_f32[v * ldyf + co]. bias nullable.
 * x and wt 16-byte aligned (AIR_ERR_ALIGN), cin a multiple of 8, cout <= 128
 * (AIR_ERR_SHAPE). */
air_status air_conv3d_fwd(const uint16_t* x, const int32_t dims[3], int32_t batch, int32_t cin,
                          const uint16_t* wt, const float* bias, int32_t cout, int32_t act,
                          const uint16_t* gate, int32_t ldg, int32_t goff, uint16_t* y_bf16,
                          int32_t ldy, int32_t yoff, float* y_f32, int32_t ldyf, void* stream);
/* Backward-data of the convolution = air_conv3d_fwd on the gradient with
 * these weights: wf[ci][tap' * C_out + co] = bf16(wt[co][(26 - tap') C_in + ci]). */
air_status air_conv3d_flip_weights(const float* wt, int32_t cin, int32_t cout, uint16_t* wf,
                                   void* stream);
/* Backward-weight: dwt[co][k] = sum_v dy[v][co] x[v + off(tap)][ci] (FP32),
 * db[co] = sum_v dy[v][co] (nullable), summed over every volume of the
 * batch. x is bf16 [v][cin], dy bf16 [v][cout], both 16-byte aligned; cin
 * and cout multiples of 8, cout <= 128 (else AIR_ERR_SHAPE / AIR_ERR_ALIGN).
 * Voxels are reduced in chunks of `chunk` (a multiple of 128; 0 = the
 * library's choice, about one resident round of blocks) into workspace
 * partials (cout * (27 cin + 1) floats per chunk, at most 65535 chunks)
 * summed in a fixed order, so results repeat bit for bit. When nx is a
 * multiple of 8 and cout <= 64 the workspace also holds x-blocked copies of
 * x and dy (8 consecutive x-voxels of one channel per 16 bytes), which feed
 * the MFMA operands directly. */
air_status air_conv3d_bwd_weight_workspace(const int32_t dims[3], int32_t batch, int32_t cin,
                                           int32_t cout, int32_t chunk, size_t* bytes);
air_status air_conv3d_bwd_weight(const uint16_t* x, const int32_t dims[3], int32_t batch,
                                 int32_t cin, const uint16_t* dy, int32_t cout, int32_t chunk,
                                 float* dwt, float* db, void* ws, size_t ws_bytes, void* stream);
/* The same on operands already in the x-blocked layout (nx a multiple of 8,
 * cout <= 64): xb[b][ci][j] = x[voxel 8 b + j][ci], dyb likewise, blocks b
 * in voxel order. cin_used (0 = cin) declares input channels cin_used ..
 * cin - 1 zero (padding): their weight gradients are written as zero
 * without being computed. The workspace holds only the partials. */
air_status air_conv3d_bwd_weight_xb_workspace(const int32_t dims[3], int32_t batch, int32_t cin,
                                              int32_t cin_used, int32_t cout, int32_t chunk,
                                              size_t* bytes);
air_status air_conv3d_bwd_weight_xb(const uint16_t* xb, const int32_t dims[3], int32_t batch,
                                    int32_t cin, int32_t cin_used, const uint16_t* dyb,
                                    int32_t cout, int32_t chunk, float* dwt, float* db, void* ws,
                                    size_t ws_bytes, void* stream);
/* y = bf16(x), round to nearest even. */
air_status air_cast_bf16(const float* x, uint16_t* y, int64_t n, void* stream);
/* 2x average pooling (even dims) of the channel slice x[v * ldx + xoff + c]
 * into a contiguous y, and its adjoint into the FP32 slice
 * dx[v * ldx + xoff + c] (written, or added when accumulate != 0). */
air_status air_pool2(const uint16_t* x, const int32_t dims[3], int32_t c, int32_t ldx,
                     int32_t xoff, uint16_t* y, void* stream);
air_status air_pool2_bwd(const float* dy, const int32_t dims[3], int32_t c, float* dx,
                         int32_t ldx, int32_t xoff, int32_t accumulate, void* stream);
/* Nearest 2x upsampling of x (dims = coarse size) into the channel slice
 * y[v * ldy + yoff + c], and its adjoint (sum of the 8 children, FP32). */
air_status air_up2(const uint16_t* x, const int32_t dims[3], int32_t c, uint16_t* y, int32_t ldy,
                   int32_t yoff, void* stream);
air_status air_up2_bwd(const float* dy, const int32_t dims[3], int32_t c, int32_t ldy,
                       int32_t yoff, float* dx, void* stream);
/* dx = bf16(dy * (a > 0 ? 1 : 0.1)) with dy read from the FP32 slice
 * dy[v * ld + off + c] and the stored activation a = yact[v * ldyact + yoff + c]. */
air_status air_lrelu_bwd(const float* dy, int32_t ld, int32_t off, const uint16_t* yact,
                         int32_t ldyact, int32_t yoff, int64_t nvox, int32_t c, uint16_t* dx,
                         void* stream);
/* Fused adjoints of pool-then-activation and upsample-then-activation
 * (dims = the fine size for pool, the coarse size for up; gate = the stored
 * bf16 activation of the fine / coarse tensor):
 *   pool:  dx[v][c] = bf16(lrelu'(gate[v]) (add[v * ldadd + addoff + c] +
 *          dy[v/2][c] / 8)), dy FP32 [v/2][c] contiguous, add nullable;
 *          xblocked != 0 writes dx in the x-blocked layout of
 *          air_conv3d_bwd_weight_xb instead (no add; nx a multiple of 8,
 *          c, ldg and goff multiples of 8, 16-byte aligned tensors);
 *   up:    dx[u][c] = bf16(lrelu'(gate[u]) sum of the 8 children
 *          dy[v * ldy + yoff + c]), dy FP32 at the fine size. */
air_status air_pool2_lrelu_bwd(const float* dy, const int32_t dims[3], int32_t c,
                              const float* add, int32_t ldadd, int32_t addoff,
                              const uint16_t* gate, int32_t ldg, int32_t goff, int32_t xblocked,
                              uint16_t* dx, void* stream);
air_status air_up2_lrelu_bwd(const float* dy, const int32_t dims[3], int32_t c, int32_t ldy,
                             int32_t yoff, const uint16_t* gate, int32_t ldg, int32_t goff,
                             uint16_t* dx, void* stream);
/* Network input: (fixed, moving) FP32 volumes (dims even) -> 2x averaged,
 * 8-channel bf16 tensor (fixed, moving, six zero channels); x_xb
 * (nullable; dims[0] / 2 a multiple of 8) also receives it in the x-blocked
 * layout of air_conv3d_bwd_weight_xb. */
air_status air_cnn_input(const float* fixed, const float* moving, const int32_t dims[3],
                         uint16_t* x, uint16_t* x_xb, void* stream);
/* Network output, per volume b of the batch: FP32 features g
 * [b][gz][gy][gx][ld] (one cell per control cell; channels 0..2 used) ->
 * control grids theta [b][3][gz+3][gy+3][gx+3]: theta[c][j] = scale *
 * g[clamp(j - 1, 0, g - 1)][c] per axis; and its adjoint into FP32 dg
 * and/or bf16 dg_bf16 (either nullable, not both; channels 3.. are zero). */
air_status air_cnn_output(const float* g, const int32_t gdims[3], int32_t batch, int32_t ld,
                          float scale, float* theta, void* stream);
air_status air_cnn_output_bwd(const float* dtheta, const int32_t gdims[3], int32_t batch,
                              int32_t ld, float scale, float* dg, uint16_t* dg_bf16,
                              void* stream);
/* a += b (FP32). */
air_status air_add_f32(float* a, const float* b, int64_t n, void* stream);

/* The whole network as one object (the layer schedule of `batch` n^3 pairs,
 * n a multiple of 16 up to 1024, batch * n^3 < 2^31), sequencing the kernels
 * above on the z-stack of the batch:
 *   x0 = avgpool2(F, M) (8 channels) at (n/2)^3; a1 = lrelu(conv 8->16);
 *   a2 = lrelu(conv(pool a1) 16->32); a3 = lrelu(conv(pool a2) 32->48);
 *   a4 = lrelu(conv(pool a3) 48->64) at (n/16)^3; d1 = lrelu(conv([a3 |
 *   up2(a4)] 112->48)); o = conv(d1) 48->16 (FP32) at (n/8)^3;
 *   theta0[c][j] = 0.05 o[clamp(j - 1, 0, g - 1)][c], g = n/8, as
 *   [3][g+3][g+3][g+3] (a spacing-8 control grid).
 * Parameters are one caller-owned FP32 buffer of param_floats floats: per
 * layer l (0..5 in the order above) W [cout][27 cin] at w_offset and
 * b [cout] at b_offset (air_cnn_layer). The workspace (ws_bytes, 16-byte
 * aligned, caller-owned) holds the BF16 weight copies, the activations and
 * the gradient buffers. */
typedef struct air_cnn air_cnn;
air_status air_cnn_create(int32_t n, int32_t batch, air_cnn** out);
void air_cnn_destroy(air_cnn* net);
air_status air_cnn_sizes(const air_cnn* net, int64_t* param_floats, size_t* ws_bytes);
air_status air_cnn_layer(const air_cnn* net, int32_t layer, int32_t* cin, int32_t* cout,
                         int64_t* w_offset, int64_t* b_offset);
/* theta0[b] = net(fixed[b], moving[b]) for FP32 volumes fixed, moving
 * [batch][n][n][n] (contiguous, 16-byte aligned) into theta0
 * [batch][3][g+3][g+3][g+3]; refreshes the BF16 weight copies from params
 * and keeps the activations in ws for air_cnn_backward. */
air_status air_cnn_forward(const air_cnn* net, const float* params, const float* fixed,
                           const float* moving, float* theta0, void* ws, size_t ws_bytes,
                           void* stream);
/* grads (the parameter layout) = dL/dparams for dtheta = dL/dtheta0
 * [batch][3][g+3]^3, summed over the batch, after air_cnn_forward with the
 * same workspace. BF16 operands, FP32 accumulation (weight gradients summed
 * per voxel chunk in a fixed order). */
air_status air_cnn_backward(const air_cnn* net, const float* dtheta, float* grads, void* ws,
                            size_t ws_bytes, void* stream);

/* ---- Synthetic inputs (not part of the paper's method). ----
 * Blob volumes of the 3D workloads painted on the device from parameters
 * drawn by the caller: out[z][y][x] = sum_b amp_b exp(-|(x,y,z) - c_b|^2 /
 * (2 sigma_b^2)) over dims = (nx, ny, nz), params a device FP32 array
 * [nblobs][5] = (cx, cy, cz, sigma, amp), nblobs <= 256, fewer than 2^31
 * voxels (AIR_ERR_SHAPE). */
air_status air_synth_blobs(const float* params, int32_t nblobs, const int32_t dims[3], float* out,
                           void* stream);
/* x[i] += stddev * N_i for i < n, N_i the i-th standard normal variate of the
 * stream `seed`: Philox4x32-10 (Salmon et al., SC 2011) at counter
 * (i / 4, 0, 0, 0) and key (seed mod 2^32, seed / 2^32), word i mod 4, each
 * word w mapped to u = (floor(w / 256) + 1/2) 2^-24 and the pairs (u0, u1),
 * (u2, u3) of a counter turned into normals by the Box-Muller transform
 * (sqrt(-2 ln u0) cos(2 pi u1), sqrt(-2 ln u0) sin(2 pi u1), ...). */
air_status air_synth_add_normal(float* x, int64_t n, uint64_t seed, float stddev, void* stream);

/* Kernel timing for benchmarks: reserve `launches` pairs of HIP events; each
 * following objective call records one pair on its stream around its main
 * kernel (the fused B-spline kernel, or the dense main pass) until the
 * reserve is used up. 0 switches timing off. Creates events (not for the
 * hot path). */
air_status air_plan_timing(air_plan* plan, int32_t launches);
/* Sum of the recorded main-kernel durations (ms) and their count; waits for
 * the recorded events and rewinds the reserve. */
air_status air_plan_timing_read(air_plan* plan, double* total_ms, int32_t* launches);

const char* air_strerror(air_status status);

#ifdef __cplusplus
}
#endif
#endif
