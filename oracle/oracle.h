/*
 * FP64 CPU oracle for the registration objective and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or helper with the GPU library: every quantity is written
 * out from the paper's definitions, in double precision, as plainly as
 * possible (direct 4^d-term kernel sums, two-pass centred statistics, a
 * voxel-level forward-difference regulariser).
 *
 * Paper: AIRLab, "Autograd Image Registration Laboratory" (arXiv 1806.09907).
 *   objective            Sec. II-A, eq. (objective)
 *   MSE                  Sec. II-A, eq. (mse); Sec. III-B
 *   NCC                  Sec. III-B (the printed formula is garbled; read as
 *                        the Pearson correlation, loss = -rho)
 *   diffusion            Sec. II-A, eq. (diffusion_regularizer); Sec. III-F
 *   interpolating basis  Sec. II-A, eq. (kernel_basis)
 *   cubic B-spline       Sec. III-C, kernel k_B1D
 *   warping + mask       Sec. III-C "Image Warping" (normalised [-1,1]^d
 *                        coordinates, out-of-domain points masked out,
 *                        linear interpolation via a grid sampler)
 *   optimiser            Sec. III-G (Adam, Kingma & Ba)
 *   diffeomorphic        Sec. III-D (f = exp(v), scaling and squaring; the
 *                        number of squarings is a problem parameter)
 *   total variation      Sec. III-F (anisotropic and isotropic)
 *   Wendland basis       Sec. III-C, kernel psi_{3,2} with per-axis sigma
 *   LCC                  Sec. III-B (local NCC: mean, variance and
 *                        covariance over a cube window around each voxel)
 *
 * Conventions (shared readings of the paper, identical on both sides):
 *   images     [nz][ny][nx], x fastest (2D: [ny][nx], n[2] == 1)
 *   fields     [d][nz][ny][nx], components ordered (x, y, z)
 *   controls   [d][ncz][ncy][ncx]; B-spline: control j sits at voxel
 *              (j-1)*delta, nc = floor((n-1)/delta) + 4. Wendland: control j
 *              sits at (j-m)*delta with m = ceil(sigma/delta) - 1 and
 *              nc = m + ceil((n-1+sigma)/delta): exactly the controls within
 *              sigma (open) of some voxel on that axis
 *   units      displacements and controls in normalised units; the sample
 *              point of voxel i is p_a = i_a + u_a * (n_a - 1) / 2 (voxels)
 *   mask       0 <= p_a <= n_a - 1 on every axis (inclusive), decided on p
 *              computed in FP64 from the inputs as given (exact for FP32
 *              inputs, see airo_sample)
 *   sampling   linear on the cell [floor(p), floor(p)+1], zero outside
 *   regulariser forward differences on u over X_R = prod_a [0, n_a - 2],
 *              normalised by |X_R|
 *
 * Parity unpinned (fixed by the readings above, not by a value printed in
 * the paper): the N' (masked) normalisation, the NCC loss sign/offset, the
 * control-grid placement, the regulariser's discretisation and domain.
 */
#ifndef AIRO_ORACLE_H
#define AIRO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define AIRO_SIM_MSE 0
#define AIRO_SIM_NCC 1
#define AIRO_SIM_LCC 2
/* epsilon of the LCC denominator sqrt(varF varW + eps) (image units^4) */
#define AIRO_LCC_EPS 1e-10
#define AIRO_TF_BSPLINE3 0
#define AIRO_TF_DENSE 1
#define AIRO_TF_WENDLAND 2

#define AIRO_FLAG_NONFINITE 1
#define AIRO_FLAG_DEGENERATE 2

typedef struct {
    int dim;          /* 2 or 3 */
    int n[3];         /* voxels along x, y, z; n[2] == 1 in 2D */
    int transform;    /* AIRO_TF_* */
    int spacing[3];   /* control spacing (voxels) along x, y, z */
    int similarity;   /* AIRO_SIM_* */
    double lambda_diff;
    int diffeo_steps; /* 0: f = the field itself; K > 0: f = exp(field) by
                         scaling and squaring with K squarings (Sec. III-D) */
    int regulariser;  /* AIRO_REG_*: the term lambda_diff weights (Sec. III-F) */
    double sigma[3];  /* Wendland support radius (voxels) along x, y, z */
    int lcc_radius;   /* LCC window: the cube |y - x|_inf <= lcc_radius */
} airo_problem;

#define AIRO_REG_DIFFUSION 0
#define AIRO_REG_ANISO_TV 1
#define AIRO_REG_ISO_TV 2

int airo_check(const airo_problem* p);
int airo_ncontrol(const airo_problem* p, int axis);
long airo_nvox(const airo_problem* p);
long airo_param_count(const airo_problem* p);

/* k_B1D(r) of Sec. III-C, unit spacing. */
double airo_bspline_kernel(double r);

/* u = B theta  (Sec. II-A eq. kernel_basis with the cubic B-spline). */
void airo_bspline_expand(const airo_problem* p, const double* theta, double* u);
/* out = B^T g  (the adjoint of the expansion). */
void airo_bspline_adjoint(const airo_problem* p, const double* g, double* out);
/* psi_{3,2}(r) of Sec. III-C: (1-r)^6_+ (3 + 18 r + 35 r^2) / 3. */
double airo_wendland_kernel(double r);
/* u = B theta with the Wendland basis (Sec. II-A eq. kernel_basis):
 *   u_c(x) = sum_j theta_c,j psi(||(x - c_j) / sigma||),
 * the division per axis (anisotropic support). */
void airo_wendland_expand(const airo_problem* p, const double* theta, double* u);
/* out = B^T g for the Wendland basis. */
void airo_wendland_adjoint(const airo_problem* p, const double* g, double* out);
/* The field before the exponential: B theta (interpolating bases) or theta
 * (dense). */
void airo_velocity(const airo_problem* p, const double* theta, double* v);
/* The displacement f_theta: the velocity itself, or its exponential when
 * diffeo_steps > 0. */
void airo_displacement(const airo_problem* p, const double* theta, double* u);

/* Diffeomorphic transform (Sec. III-D, f = exp(v) for a stationary velocity
 * field v), by scaling and squaring: u_0 = v / 2^K, then K times
 *     u_{k+1}(x) = u_k(x) + u_k(x + u_k(x)),
 * the second term sampled like an image (sample point p_a = x_a + u_a (n_a-1)/2,
 * linear on [floor(p), floor(p)+1], zero outside; no mask).
 * airo_compose: one squaring. airo_compose_adjoint: given gout = dL/du_{k+1},
 * gin = dL/du_k (the identity term, the term through the sample point, and
 * the transpose of the interpolation, scattered voxel by voxel).
 * airo_exp: u = exp(v); hist (nullable) receives u_0 .. u_K ((K+1) d N). */
void airo_compose(const airo_problem* p, const double* u, double* out);
void airo_compose_adjoint(const airo_problem* p, const double* u, const double* gout,
                          double* gin);
void airo_exp(const airo_problem* p, const double* v, int K, double* u, double* hist);

/* Sample `moving` at x + u(x); writes warped [N], mask [N] (nullable) and
 * dwdp [d][N] (nullable): the derivative of the sample with respect to the
 * sample point in voxel units, on the cell [floor(p), floor(p)+1]. The point
 * p = x + u (n-1)/2, the cell and the mask are taken in FP64 on the inputs as
 * given (FP32 inputs widened exactly), which is the sampler's definition. */
void airo_sample(const airo_problem* p, const double* moving, const double* u,
                 double* warped, unsigned char* mask, double* dwdp);
void airo_warp(const airo_problem* p, const double* moving, const double* theta,
               double* warped, unsigned char* mask);

/* Similarity over the masked set; dsdw [N] nullable. Returns flag bits.
 * LCC (Sec. III-B, the local version of NCC): for x in the masked set X',
 * the window N(x) = {y in X' : |y - x|_inf <= lcc_radius}, n = |N(x)|, the
 * means, variances and covariance of F and W over N(x) (divided by n),
 *   rho(x) = cov / sqrt(varF varW + AIRO_LCC_EPS),
 * and S = -(1/|X'|) sum_{x in X'} rho(x). */
int airo_similarity(const airo_problem* p, const double* fixed, const double* warped,
                    const unsigned char* mask, double* value, double* dsdw);

/* Diffusion regulariser of u (dense field), gradient with respect to u. */
void airo_diffusion(const airo_problem* p, const double* u, double* value, double* grad_u);
/* Total variation of u (Sec. III-F) on the forward differences
 * D_a u_c(x) = u_c(x + e_a) - u_c(x) over X_R, divided by |X_R|:
 *   kind AIRO_REG_ANISO_TV: sum_c sum_a |D_a u_c(x)|;
 *   kind AIRO_REG_ISO_TV:   sqrt(sum_c sum_a D_a u_c(x)^2)  (one norm per voxel).
 * Gradient with the subgradient 0 where the term is 0. grad_u nullable. */
void airo_tv(const airo_problem* p, const double* u, int kind, double* value, double* grad_u);
/* Regulariser as a function of the parameters (theta). grad nullable. */
void airo_regulariser(const airo_problem* p, const double* theta, double* value, double* grad);

/* L = S + lambda R and dL/dtheta. Returns flag bits. */
int airo_objective_and_grad(const airo_problem* p, const double* fixed,
                            const double* moving, const double* theta,
                            double* value, double* grad);

/* One bias-corrected Adam step, in place (step counts from 1). */
void airo_adam_step(double* theta, const double* grad, double* m, double* v, long n,
                    double lr, double b1, double b2, double eps, int step);

/* Multi-resolution helpers (Sec. IV-A: the FFD experiment's multi-resolution
 * strategy). Gaussian pyramid level: separable Gaussian of std `sigma`
 * (voxels), taps truncated at ceil(3 sigma), weights normalised to sum 1,
 * borders clamped (edge voxels repeated), then every second voxel from 0:
 * out n_out = (n + 1) / 2 per axis. 3D volumes [nz][ny][nx]. */
void airo_pyramid_down(const double* in, const int n[3], double sigma, double* out);
/* Transfer a displacement field [3][nz][ny][nx] (normalised units) to a
 * finer grid m[3] by linear interpolation in normalised coordinates
 * (align-corners convention: voxel j of m maps to j (n-1)/(m-1) of n). */
void airo_field_resample(const double* in, const int n[3], const int m[3], double* out);

/* 3x3x3 convolution, stride 1, zero padding 1, channel-last tensors
 * x [nz][ny][nx][cin], weights wt [cout][27 * cin] (k = tap * cin + ci,
 * tap = (dz*3 + dy)*3 + dx), y [nz][ny][nx][cout]; act 1 = LeakyReLU 0.1.
 * Backward takes dy = dL/d(pre-activation) and writes dx, dwt, db
 * (each nullable). Used to check the learned-initialisation network. */
void airo_conv3d_fwd(const double* x, const int n[3], int cin, const double* wt,
                     const double* bias, int cout, int act, double* y);
void airo_conv3d_bwd(const double* x, const int n[3], int cin, const double* wt, int cout,
                     const double* dy, double* dx, double* dwt, double* db);

/* Threads used by the parallel loops (OpenMP); 0 = runtime default. */
void airo_set_threads(int nthreads);
int airo_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
