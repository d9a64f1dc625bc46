/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every function restates a definition of the AIRLab paper (arXiv
 * 1806.09907) in the plainest form that still finishes in seconds at 128^3:
 * the B-spline field is the direct sum over the 4^d controls whose kernel
 * support contains the voxel (Sec. II-A eq. kernel_basis, Sec. III-C k_B1D);
 * its adjoint is the same sum read per control; sampling is the zero-padded
 * multilinear interpolation of a grid sampler (Sec. III-C Image Warping);
 * NCC uses two-pass centred statistics; the diffusion term is evaluated
 * voxel by voxel with forward differences (Sec. II-A eq. diffusion).
 * Loops are parallel over the slowest axis only, and every reduction is
 * summed per slab and then serially, so results do not depend on threads.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0;

void airo_set_threads(int nthreads) { g_threads = nthreads > 0 ? nthreads : 0; }

int airo_get_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

#ifdef _OPENMP
#define NTHREADS num_threads(airo_get_threads())
#endif

int airo_check(const airo_problem* p) {
    if (!p) return 1;
    if (p->dim != 2 && p->dim != 3) return 1;
    for (int a = 0; a < p->dim; ++a) {
        if (p->n[a] < 2) return 1;
        if (p->transform != AIRO_TF_DENSE && p->spacing[a] < 1) return 1;
        if (p->transform == AIRO_TF_WENDLAND && !(p->sigma[a] > 0.0 && p->sigma[a] < 1e6))
            return 1;
    }
    if (p->dim == 2 && p->n[2] != 1) return 1;
    if (p->transform != AIRO_TF_BSPLINE3 && p->transform != AIRO_TF_DENSE &&
        p->transform != AIRO_TF_WENDLAND)
        return 1;
    if (p->similarity != AIRO_SIM_MSE && p->similarity != AIRO_SIM_NCC &&
        p->similarity != AIRO_SIM_LCC)
        return 1;
    if (p->similarity == AIRO_SIM_LCC && (p->lcc_radius < 1 || p->lcc_radius > 64)) return 1;
    if (p->diffeo_steps < 0 || p->diffeo_steps > 30) return 1;
    if (p->regulariser < AIRO_REG_DIFFUSION || p->regulariser > AIRO_REG_ISO_TV) return 1;
    return 0;
}

/* Wendland controls along an axis: the first sits m spacings before voxel 0,
 * m = ceil(sigma/delta) - 1, the last control lies less than sigma beyond
 * voxel n-1; every control within sigma (open) of a voxel is present. */
static int wendland_first(const airo_problem* p, int axis) {
    return (int)ceil(p->sigma[axis] / p->spacing[axis]) - 1;
}

int airo_ncontrol(const airo_problem* p, int axis) {
    if (axis >= p->dim) return 1;
    if (p->transform == AIRO_TF_WENDLAND)
        return wendland_first(p, axis) +
               (int)ceil((p->n[axis] - 1 + p->sigma[axis]) / p->spacing[axis]);
    return (p->n[axis] - 1) / p->spacing[axis] + 4;
}

long airo_nvox(const airo_problem* p) {
    long n = 1;
    for (int a = 0; a < p->dim; ++a) n *= p->n[a];
    return n;
}

static long ncontrols_total(const airo_problem* p) {
    long n = 1;
    for (int a = 0; a < p->dim; ++a) n *= airo_ncontrol(p, a);
    return n;
}

long airo_param_count(const airo_problem* p) {
    if (p->transform == AIRO_TF_DENSE) return (long)p->dim * airo_nvox(p);
    return (long)p->dim * ncontrols_total(p);
}

/* k_B1D of Sec. III-C: 2/3 - |r|^2 + |r|^3/2 on [0,1), (2-|r|)^3/6 on [1,2). */
double airo_bspline_kernel(double r) {
    double a = fabs(r);
    if (a < 1.0) return 2.0 / 3.0 - a * a + a * a * a / 2.0;
    if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
    return 0.0;
}

/* Position (voxels) of control j along an axis with spacing s. */
static double control_pos(int j, int s) { return (double)(j - 1) * s; }

/* For voxel coordinate x: its first supporting control index (floor(x/s))
 * and the four kernel values k((x - pos(i+k)) / s), k = 0..3. */
static int support(int x, int s, double w[4]) {
    int i = x / s;
    for (int k = 0; k < 4; ++k)
        w[k] = airo_bspline_kernel(((double)x - control_pos(i + k, s)) / (double)s);
    return i;
}

void airo_bspline_expand(const airo_problem* p, const double* theta, double* u) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int ncx = airo_ncontrol(p, 0), ncy = airo_ncontrol(p, 1);
    const int ncz = (d == 3) ? airo_ncontrol(p, 2) : 1;
    const long N = (long)nx * ny * nz;
    const long NC = (long)ncx * ncy * ncz;
    const int sx = p->spacing[0], sy = p->spacing[1], sz = (d == 3) ? p->spacing[2] : 1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int z = 0; z < nz; ++z) {
        double wz[4] = {1.0, 0.0, 0.0, 0.0};
        int iz = 0;
        if (d == 3) iz = support(z, sz, wz);
        for (int y = 0; y < ny; ++y) {
            double wy[4];
            int iy = support(y, sy, wy);
            for (int x = 0; x < nx; ++x) {
                double wx[4];
                int ix = support(x, sx, wx);
                for (int c = 0; c < d; ++c) {
                    double acc = 0.0;
                    for (int kz = 0; kz < (d == 3 ? 4 : 1); ++kz)
                        for (int ky = 0; ky < 4; ++ky)
                            for (int kx = 0; kx < 4; ++kx) {
                                long j = ((long)(iz + kz) * ncy + (iy + ky)) * ncx + (ix + kx);
                                acc += wz[kz] * wy[ky] * wx[kx] * theta[c * NC + j];
                            }
                    u[c * N + ((long)z * ny + y) * nx + x] = acc;
                }
            }
        }
    }
}

/* Voxel range [lo, hi] inside which control j has non-zero support. */
static void control_support(int j, int s, int n, int* lo, int* hi) {
    double c = control_pos(j, s);
    int a = (int)floor(c - 2.0 * s);
    int b = (int)ceil(c + 2.0 * s);
    if (a < 0) a = 0;
    if (b > n - 1) b = n - 1;
    *lo = a;
    *hi = b;
}

void airo_bspline_adjoint(const airo_problem* p, const double* g, double* out) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int ncx = airo_ncontrol(p, 0), ncy = airo_ncontrol(p, 1);
    const int ncz = (d == 3) ? airo_ncontrol(p, 2) : 1;
    const long N = (long)nx * ny * nz;
    const long NC = (long)ncx * ncy * ncz;
    const int sx = p->spacing[0], sy = p->spacing[1], sz = (d == 3) ? p->spacing[2] : 1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic) NTHREADS
#endif
    for (int jz = 0; jz < ncz; ++jz) {
        int z0 = 0, z1 = 0;
        if (d == 3) control_support(jz, sz, nz, &z0, &z1);
        for (int jy = 0; jy < ncy; ++jy) {
            int y0, y1;
            control_support(jy, sy, ny, &y0, &y1);
            for (int jx = 0; jx < ncx; ++jx) {
                int x0, x1;
                control_support(jx, sx, nx, &x0, &x1);
                double acc[3] = {0.0, 0.0, 0.0};
                for (int z = z0; z <= z1; ++z) {
                    double kz = (d == 3)
                        ? airo_bspline_kernel(((double)z - control_pos(jz, sz)) / sz) : 1.0;
                    if (kz == 0.0) continue;
                    for (int y = y0; y <= y1; ++y) {
                        double ky = airo_bspline_kernel(((double)y - control_pos(jy, sy)) / sy);
                        if (ky == 0.0) continue;
                        for (int x = x0; x <= x1; ++x) {
                            double kx = airo_bspline_kernel(((double)x - control_pos(jx, sx)) / sx);
                            if (kx == 0.0) continue;
                            long v = ((long)z * ny + y) * nx + x;
                            double w = kz * ky * kx;
                            for (int c = 0; c < d; ++c) acc[c] += w * g[c * N + v];
                        }
                    }
                }
                long j = ((long)jz * ncy + jy) * ncx + jx;
                for (int c = 0; c < d; ++c) out[c * NC + j] = acc[c];
            }
        }
    }
}

/* ---- Sec. III-C: the Wendland kernel psi_{3,2} -------------------- */

double airo_wendland_kernel(double r) {
    if (r >= 1.0) return 0.0;
    const double t = 1.0 - r;
    return t * t * t * t * t * t * (3.0 + 18.0 * r + 35.0 * r * r) / 3.0;
}

/* Position (voxels) of Wendland control j along axis a. */
static double wendland_pos(const airo_problem* p, int a, int j) {
    return (double)(j - wendland_first(p, a)) * p->spacing[a];
}

/* The controls along axis a within sigma (open) of coordinate x: [*lo, *hi]
 * (empty when *lo > *hi), found by testing every control. */
static void wendland_range(const airo_problem* p, int a, double x, int* lo, int* hi) {
    const int nc = airo_ncontrol(p, a);
    *lo = nc;
    *hi = -1;
    for (int j = 0; j < nc; ++j)
        if (fabs(x - wendland_pos(p, a, j)) < p->sigma[a]) {
            if (j < *lo) *lo = j;
            *hi = j;
        }
}

/* psi(||(x - c) / sigma||) for a voxel x and a control at c (both [3]). */
static double wendland_weight(const airo_problem* p, const double* x, const double* c) {
    double r2 = 0.0;
    for (int a = 0; a < p->dim; ++a) {
        const double q = (x[a] - c[a]) / p->sigma[a];
        r2 += q * q;
    }
    return airo_wendland_kernel(sqrt(r2));
}

void airo_wendland_expand(const airo_problem* p, const double* theta, double* u) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int ncx = airo_ncontrol(p, 0), ncy = airo_ncontrol(p, 1);
    const long N = (long)nx * ny * nz;
    const long NC = ncontrols_total(p);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int z = 0; z < nz; ++z) {
        int z0 = 0, z1 = 0;
        if (d == 3) wendland_range(p, 2, z, &z0, &z1);
        for (int y = 0; y < ny; ++y) {
            int y0, y1;
            wendland_range(p, 1, y, &y0, &y1);
            for (int x = 0; x < nx; ++x) {
                int x0, x1;
                wendland_range(p, 0, x, &x0, &x1);
                const double pt[3] = {x, y, z};
                double acc[3] = {0.0, 0.0, 0.0};
                for (int jz = z0; jz <= z1; ++jz)
                    for (int jy = y0; jy <= y1; ++jy)
                        for (int jx = x0; jx <= x1; ++jx) {
                            const double c[3] = {wendland_pos(p, 0, jx), wendland_pos(p, 1, jy),
                                                 d == 3 ? wendland_pos(p, 2, jz) : 0.0};
                            const double w = wendland_weight(p, pt, c);
                            const long j = ((long)jz * ncy + jy) * ncx + jx;
                            for (int k = 0; k < d; ++k) acc[k] += w * theta[k * NC + j];
                        }
                const long v = ((long)z * ny + y) * nx + x;
                for (int k = 0; k < d; ++k) u[k * N + v] = acc[k];
            }
        }
    }
}

/* The voxels along axis a within sigma (open) of a control at c. */
static void voxel_range(const airo_problem* p, int a, double c, int* lo, int* hi) {
    const int n = p->n[a];
    *lo = n;
    *hi = -1;
    for (int x = 0; x < n; ++x)
        if (fabs((double)x - c) < p->sigma[a]) {
            if (x < *lo) *lo = x;
            *hi = x;
        }
}

void airo_wendland_adjoint(const airo_problem* p, const double* g, double* out) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int ncx = airo_ncontrol(p, 0), ncy = airo_ncontrol(p, 1);
    const int ncz = (d == 3) ? airo_ncontrol(p, 2) : 1;
    const long N = (long)nx * ny * nz;
    const long NC = ncontrols_total(p);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic) NTHREADS
#endif
    for (int jz = 0; jz < ncz; ++jz) {
        const double cz = (d == 3) ? wendland_pos(p, 2, jz) : 0.0;
        int z0 = 0, z1 = 0;
        if (d == 3) voxel_range(p, 2, cz, &z0, &z1);
        for (int jy = 0; jy < ncy; ++jy) {
            const double cy = wendland_pos(p, 1, jy);
            int y0, y1;
            voxel_range(p, 1, cy, &y0, &y1);
            for (int jx = 0; jx < ncx; ++jx) {
                const double cx = wendland_pos(p, 0, jx);
                int x0, x1;
                voxel_range(p, 0, cx, &x0, &x1);
                const double c[3] = {cx, cy, cz};
                double acc[3] = {0.0, 0.0, 0.0};
                for (int z = z0; z <= z1; ++z)
                    for (int y = y0; y <= y1; ++y)
                        for (int x = x0; x <= x1; ++x) {
                            const double pt[3] = {x, y, z};
                            const double w = wendland_weight(p, pt, c);
                            const long v = ((long)z * ny + y) * nx + x;
                            for (int k = 0; k < d; ++k) acc[k] += w * g[k * N + v];
                        }
                const long j = ((long)jz * ncy + jy) * ncx + jx;
                for (int k = 0; k < d; ++k) out[k * NC + j] = acc[k];
            }
        }
    }
}

void airo_velocity(const airo_problem* p, const double* theta, double* v) {
    if (p->transform == AIRO_TF_DENSE)
        memcpy(v, theta, sizeof(double) * (size_t)p->dim * (size_t)airo_nvox(p));
    else if (p->transform == AIRO_TF_WENDLAND)
        airo_wendland_expand(p, theta, v);
    else
        airo_bspline_expand(p, theta, v);
}

void airo_displacement(const airo_problem* p, const double* theta, double* u) {
    if (p->diffeo_steps <= 0) {
        airo_velocity(p, theta, u);
        return;
    }
    const size_t fb = sizeof(double) * (size_t)p->dim * (size_t)airo_nvox(p);
    double* v = (double*)malloc(fb);
    airo_velocity(p, theta, v);
    airo_exp(p, v, p->diffeo_steps, u, NULL);
    free(v);
}

void airo_sample(const airo_problem* p, const double* moving, const double* u,
                 double* warped, unsigned char* mask, double* dwdp) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int n[3] = {nx, ny, nz};
    const long N = (long)nx * ny * nz;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const long v = ((long)z * ny + y) * nx + x;
                const int idx[3] = {x, y, z};
                double pt[3], f[3];
                long j[3];
                int inside = 1, finite = 1;
                for (int a = 0; a < d; ++a) {
                    pt[a] = idx[a] + u[a * N + v] * (n[a] - 1) / 2.0;
                    if (!isfinite(pt[a])) finite = 0;
                    if (!(pt[a] >= 0.0 && pt[a] <= n[a] - 1)) inside = 0;
                    /* far outside: every corner is padding; keep floor() in range */
                    if (pt[a] > 1e9) pt[a] = 1e9;
                    if (pt[a] < -1e9) pt[a] = -1e9;
                }
                if (mask) mask[v] = (unsigned char)(inside && finite);
                if (!finite) {
                    if (warped) warped[v] = NAN;
                    if (dwdp) for (int a = 0; a < d; ++a) dwdp[a * N + v] = NAN;
                    continue;
                }
                for (int a = 0; a < d; ++a) {
                    j[a] = (long)floor(pt[a]);
                    f[a] = pt[a] - (double)j[a];
                }
                double W = 0.0, dW[3] = {0.0, 0.0, 0.0};
                const int ncorner = 1 << d;
                for (int c = 0; c < ncorner; ++c) {
                    int bit[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
                    long q[3] = {0, 0, 0};
                    int in_range = 1;
                    for (int a = 0; a < d; ++a) {
                        q[a] = j[a] + bit[a];
                        if (q[a] < 0 || q[a] > n[a] - 1) in_range = 0;
                    }
                    double val = in_range ? moving[(q[2] * ny + q[1]) * nx + q[0]] : 0.0;
                    double wgt = 1.0;
                    for (int a = 0; a < d; ++a) wgt *= bit[a] ? f[a] : 1.0 - f[a];
                    W += wgt * val;
                    for (int a = 0; a < d; ++a) {
                        double wa = bit[a] ? 1.0 : -1.0;
                        for (int b = 0; b < d; ++b)
                            if (b != a) wa *= bit[b] ? f[b] : 1.0 - f[b];
                        dW[a] += wa * val;
                    }
                }
                if (warped) warped[v] = W;
                if (dwdp) for (int a = 0; a < d; ++a) dwdp[a * N + v] = dW[a];
            }
        }
    }
}

void airo_warp(const airo_problem* p, const double* moving, const double* theta,
               double* warped, unsigned char* mask) {
    const long N = airo_nvox(p);
    double* u = (double*)malloc(sizeof(double) * (size_t)p->dim * (size_t)N);
    airo_displacement(p, theta, u);
    airo_sample(p, moving, u, warped, mask, NULL);
    free(u);
}

/* ---- Sec. III-D: f = exp(v) by scaling and squaring ---------------- */

/* One squaring: out_c(x) = u_c(x) + [u_c sampled at x + u(x)], each
 * component sampled with the image sampler (zero outside, no mask). */
void airo_compose(const airo_problem* p, const double* u, double* out) {
    const int d = p->dim;
    const long N = airo_nvox(p);
    double* s = (double*)malloc(sizeof(double) * (size_t)N);
    for (int c = 0; c < d; ++c) {
        airo_sample(p, u + c * N, u, s, NULL, NULL);
        for (long v = 0; v < N; ++v) out[c * N + v] = u[c * N + v] + s[v];
    }
    free(s);
}

/* Adjoint of one squaring. With s_a = (n_a - 1)/2 and w_q(p) the linear
 * weights of corner q:
 *   gin_c(x) += gout_c(x)                                  (identity term)
 *   gin_a(x) += s_a sum_c gout_c(x) d[u_c sampled](p(x))/dp_a   (sample point)
 *   gin_c(q) += w_q(p(x)) gout_c(x) for every in-range corner q of p(x)
 *                                                          (interpolation^T)
 * The scatter runs serially in voxel order. */
void airo_compose_adjoint(const airo_problem* p, const double* u, const double* gout,
                          double* gin) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int n[3] = {nx, ny, nz};
    const long N = airo_nvox(p);
    double* dsdp = (double*)malloc(sizeof(double) * (size_t)d * (size_t)N);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)N);
    for (long i = 0; i < (long)d * N; ++i) gin[i] = gout[i];
    for (int c = 0; c < d; ++c) {
        airo_sample(p, u + c * N, u, tmp, NULL, dsdp);
        for (int a = 0; a < d; ++a) {
            const double sa = (n[a] - 1) / 2.0;
            for (long v = 0; v < N; ++v) gin[a * N + v] += sa * gout[c * N + v] * dsdp[a * N + v];
        }
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long v = ((long)z * ny + y) * nx + x;
                const int idx[3] = {x, y, z};
                double pt[3], f[3];
                long j[3];
                int finite = 1;
                for (int a = 0; a < d; ++a) {
                    pt[a] = idx[a] + u[a * N + v] * (n[a] - 1) / 2.0;
                    if (!isfinite(pt[a])) finite = 0;
                    if (pt[a] > 1e9) pt[a] = 1e9;
                    if (pt[a] < -1e9) pt[a] = -1e9;
                }
                if (!finite) continue;
                for (int a = 0; a < d; ++a) {
                    j[a] = (long)floor(pt[a]);
                    f[a] = pt[a] - (double)j[a];
                }
                for (int cnr = 0; cnr < (1 << d); ++cnr) {
                    int bit[3] = {cnr & 1, (cnr >> 1) & 1, (cnr >> 2) & 1};
                    long q[3] = {0, 0, 0};
                    int in_range = 1;
                    for (int a = 0; a < d; ++a) {
                        q[a] = j[a] + bit[a];
                        if (q[a] < 0 || q[a] > n[a] - 1) in_range = 0;
                    }
                    if (!in_range) continue;
                    double wgt = 1.0;
                    for (int a = 0; a < d; ++a) wgt *= bit[a] ? f[a] : 1.0 - f[a];
                    const long qi = (q[2] * ny + q[1]) * nx + q[0];
                    for (int c = 0; c < d; ++c) gin[c * N + qi] += wgt * gout[c * N + v];
                }
            }
    free(dsdp);
    free(tmp);
}

void airo_exp(const airo_problem* p, const double* v, int K, double* u, double* hist) {
    const long dN = (long)p->dim * airo_nvox(p);
    double* a = (double*)malloc(sizeof(double) * (size_t)dN);
    double* b = (double*)malloc(sizeof(double) * (size_t)dN);
    const double scale = ldexp(1.0, -K);
    for (long i = 0; i < dN; ++i) a[i] = v[i] * scale;
    if (hist) memcpy(hist, a, sizeof(double) * (size_t)dN);
    for (int k = 0; k < K; ++k) {
        airo_compose(p, a, b);
        double* t = a;
        a = b;
        b = t;
        if (hist) memcpy(hist + (long)(k + 1) * dN, a, sizeof(double) * (size_t)dN);
    }
    memcpy(u, a, sizeof(double) * (size_t)dN);
    free(a);
    free(b);
}

/* dL/dtheta from dL/du (u the displacement): back through the squarings
 * (if any) and the B-spline expansion (if any). */
static void displacement_adjoint(const airo_problem* p, const double* theta, const double* gu,
                                 double* grad) {
    const long dN = (long)p->dim * airo_nvox(p);
    const size_t fb = sizeof(double) * (size_t)dN;
    double* gv = (double*)malloc(fb);
    if (p->diffeo_steps > 0) {
        const int K = p->diffeo_steps;
        double* v = (double*)malloc(fb);
        double* hist = (double*)malloc(fb * (size_t)(K + 1));
        double* t = (double*)malloc(fb);
        airo_velocity(p, theta, v);
        airo_exp(p, v, K, t, hist);
        memcpy(gv, gu, fb);
        for (int k = K - 1; k >= 0; --k) {
            airo_compose_adjoint(p, hist + (long)k * dN, gv, t);
            memcpy(gv, t, fb);
        }
        const double scale = ldexp(1.0, -K);
        for (long i = 0; i < dN; ++i) gv[i] *= scale;
        free(v);
        free(hist);
        free(t);
    } else {
        memcpy(gv, gu, fb);
    }
    if (p->transform == AIRO_TF_DENSE)
        memcpy(grad, gv, fb);
    else if (p->transform == AIRO_TF_WENDLAND)
        airo_wendland_adjoint(p, gv, grad);
    else
        airo_bspline_adjoint(p, gv, grad);
    free(gv);
}

/* Per-slab partial sums, added serially in slab order. */
static int slab_count(const airo_problem* p) { return p->dim == 3 ? p->n[2] : p->n[1]; }
static long slab_size(const airo_problem* p) {
    return p->dim == 3 ? (long)p->n[0] * p->n[1] : (long)p->n[0];
}

/* Sec. III-B, LCC: local statistics over each window, centred about the
 * window's own means (two passes per window); the gradient with respect to
 * W(y) gathers, over the windows that contain y,
 *   d rho(x)/dW(y) = (F(y) - muF(x)) / (n s) - rho varF (W(y) - muW(x)) / (n V)
 * with V = varF varW + eps and s = sqrt(V). */
static int lcc(const airo_problem* p, const double* F, const double* W,
               const unsigned char* mask, double* value, double* dsdw) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const long N = airo_nvox(p);
    const int r = p->lcc_radius;
    const int rz = (d == 3) ? r : 0;
    double* st = (double*)malloc(sizeof(double) * 6 * (size_t)N);  /* muF muW n rho varF V */
    double* part = (double*)calloc((size_t)nz, 2 * sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic) NTHREADS
#endif
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long v = ((long)z * ny + y) * nx + x;
                double* o = st + 6 * v;
                o[2] = 0.0;
                if (!mask[v]) continue;
                const int z0 = z - rz < 0 ? 0 : z - rz, z1 = z + rz > nz - 1 ? nz - 1 : z + rz;
                const int y0 = y - r < 0 ? 0 : y - r, y1 = y + r > ny - 1 ? ny - 1 : y + r;
                const int x0 = x - r < 0 ? 0 : x - r, x1 = x + r > nx - 1 ? nx - 1 : x + r;
                double n = 0.0, sf = 0.0, sw = 0.0;
                for (int c = z0; c <= z1; ++c)
                    for (int b = y0; b <= y1; ++b)
                        for (int a = x0; a <= x1; ++a) {
                            const long q = ((long)c * ny + b) * nx + a;
                            if (!mask[q]) continue;
                            n += 1.0;
                            sf += F[q];
                            sw += W[q];
                        }
                const double mf = sf / n, mw = sw / n;
                double vf = 0.0, vw = 0.0, cv = 0.0;
                for (int c = z0; c <= z1; ++c)
                    for (int b = y0; b <= y1; ++b)
                        for (int a = x0; a <= x1; ++a) {
                            const long q = ((long)c * ny + b) * nx + a;
                            if (!mask[q]) continue;
                            vf += (F[q] - mf) * (F[q] - mf);
                            vw += (W[q] - mw) * (W[q] - mw);
                            cv += (F[q] - mf) * (W[q] - mw);
                        }
                vf /= n;
                vw /= n;
                cv /= n;
                const double V = vf * vw + AIRO_LCC_EPS;
                o[0] = mf;
                o[1] = mw;
                o[2] = n;
                o[3] = cv / sqrt(V);
                o[4] = vf;
                o[5] = V;
                part[2 * z] += 1.0;
                part[2 * z + 1] += o[3];
            }
    }
    double cnt = 0.0, srho = 0.0;
    for (int z = 0; z < nz; ++z) {
        cnt += part[2 * z];
        srho += part[2 * z + 1];
    }
    free(part);
    if (cnt < 1.0) {
        *value = 0.0;
        if (dsdw) memset(dsdw, 0, sizeof(double) * (size_t)N);
        free(st);
        return AIRO_FLAG_DEGENERATE;
    }
    *value = -srho / cnt;
    if (dsdw) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic) NTHREADS
#endif
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const long v = ((long)z * ny + y) * nx + x;
                    dsdw[v] = 0.0;
                    if (!mask[v]) continue;
                    const int z0 = z - rz < 0 ? 0 : z - rz, z1 = z + rz > nz - 1 ? nz - 1 : z + rz;
                    const int y0 = y - r < 0 ? 0 : y - r, y1 = y + r > ny - 1 ? ny - 1 : y + r;
                    const int x0 = x - r < 0 ? 0 : x - r, x1 = x + r > nx - 1 ? nx - 1 : x + r;
                    double acc = 0.0;
                    for (int c = z0; c <= z1; ++c)
                        for (int b = y0; b <= y1; ++b)
                            for (int a = x0; a <= x1; ++a) {
                                const long q = ((long)c * ny + b) * nx + a;
                                const double* o = st + 6 * q;
                                if (!mask[q]) continue;
                                const double n = o[2], s = sqrt(o[5]);
                                acc += (F[v] - o[0]) / (n * s) -
                                       o[3] * o[4] * (W[v] - o[1]) / (n * o[5]);
                            }
                    dsdw[v] = -acc / cnt;
                }
    }
    free(st);
    return isfinite(*value) ? 0 : AIRO_FLAG_NONFINITE;
}

int airo_similarity(const airo_problem* p, const double* fixed, const double* warped,
                    const unsigned char* mask, double* value, double* dsdw) {
    if (p->similarity == AIRO_SIM_LCC) return lcc(p, fixed, warped, mask, value, dsdw);
    const long N = airo_nvox(p);
    const int ns = slab_count(p);
    const long ss = slab_size(p);
    int flags = 0;
    double* part = (double*)calloc((size_t)ns * 6, sizeof(double));
    /* pass 1: count, sums of F and W (and of squared error for MSE) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int s = 0; s < ns; ++s) {
        double cnt = 0, sf = 0, sw = 0, se = 0;
        for (long v = s * ss; v < (s + 1) * ss; ++v) {
            if (!mask[v]) continue;
            cnt += 1.0;
            sf += fixed[v];
            sw += warped[v];
            se += (warped[v] - fixed[v]) * (warped[v] - fixed[v]);
        }
        part[6 * s + 0] = cnt;
        part[6 * s + 1] = sf;
        part[6 * s + 2] = sw;
        part[6 * s + 3] = se;
    }
    double cnt = 0, sf = 0, sw = 0, se = 0;
    for (int s = 0; s < ns; ++s) {
        cnt += part[6 * s + 0];
        sf += part[6 * s + 1];
        sw += part[6 * s + 2];
        se += part[6 * s + 3];
    }
    if (p->similarity == AIRO_SIM_MSE) {
        /* Sec. II-A eq. (mse), over the masked set X' (normalised by N'). */
        if (cnt < 1.0) {
            *value = 0.0;
            flags |= AIRO_FLAG_DEGENERATE;
            if (dsdw) memset(dsdw, 0, sizeof(double) * (size_t)N);
        } else {
            *value = se / cnt;
            if (dsdw)
                for (long v = 0; v < N; ++v)
                    dsdw[v] = mask[v] ? 2.0 * (warped[v] - fixed[v]) / cnt : 0.0;
        }
        free(part);
        if (!isfinite(*value)) flags |= AIRO_FLAG_NONFINITE;
        return flags;
    }
    /* NCC (Sec. III-B): Pearson correlation of F and W over X', loss -rho.
     * pass 2: centred sums about the exact means. */
    if (cnt < 2.0) {
        *value = 0.0;
        if (dsdw) memset(dsdw, 0, sizeof(double) * (size_t)N);
        free(part);
        return flags | AIRO_FLAG_DEGENERATE;
    }
    const double muf = sf / cnt, muw = sw / cnt;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int s = 0; s < ns; ++s) {
        double a = 0, b = 0, c = 0, ff = 0, ww = 0;
        for (long v = s * ss; v < (s + 1) * ss; ++v) {
            if (!mask[v]) continue;
            double df = fixed[v] - muf, dw = warped[v] - muw;
            a += df * dw;
            b += df * df;
            c += dw * dw;
            ff += fixed[v] * fixed[v];
            ww += warped[v] * warped[v];
        }
        part[6 * s + 0] = a;
        part[6 * s + 1] = b;
        part[6 * s + 2] = c;
        part[6 * s + 3] = ff;
        part[6 * s + 4] = ww;
    }
    double A = 0, B = 0, C = 0, FF = 0, WW = 0;
    for (int s = 0; s < ns; ++s) {
        A += part[6 * s + 0];
        B += part[6 * s + 1];
        C += part[6 * s + 2];
        FF += part[6 * s + 3];
        WW += part[6 * s + 4];
    }
    free(part);
    /* Degenerate variance: a constant image on the masked set. */
    if (!(B > 1e-10 * FF) || !(C > 1e-10 * WW)) {
        *value = 0.0;
        if (dsdw) memset(dsdw, 0, sizeof(double) * (size_t)N);
        return flags | AIRO_FLAG_DEGENERATE;
    }
    const double sbc = sqrt(B * C);
    const double rho = A / sbc;
    *value = -rho;
    if (dsdw) {
        /* d(-rho)/dW(x) = -[(F - muF)/sqrt(BC) - rho (W - muW)/C] on X'. */
        for (long v = 0; v < N; ++v)
            dsdw[v] = mask[v]
                ? -((fixed[v] - muf) / sbc - rho * (warped[v] - muw) / C) : 0.0;
    }
    if (!isfinite(*value)) flags |= AIRO_FLAG_NONFINITE;
    return flags;
}

/* Sec. II-A eq. (diffusion_regularizer), forward differences over
 * X_R = prod_a [0, n_a - 2], normalised by |X_R|; gradient with respect to
 * u at every voxel (gather form of the derivative). */
void airo_diffusion(const airo_problem* p, const double* u, double* value, double* grad_u) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int n[3] = {nx, ny, nz};
    const long N = (long)nx * ny * nz;
    const long stride[3] = {1, nx, (long)nx * ny};
    double XR = 1.0;
    for (int a = 0; a < d; ++a) XR *= (double)(n[a] - 1);
    double* part = (double*)calloc((size_t)nz, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int z = 0; z < nz; ++z) {
        double acc = 0.0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int idx[3] = {x, y, z};
                int in_r = 1;
                for (int a = 0; a < d; ++a)
                    if (idx[a] > n[a] - 2) in_r = 0;
                const long v = ((long)z * ny + y) * nx + x;
                for (int c = 0; c < d; ++c) {
                    const double* uc = u + c * N;
                    double gsum = 0.0;
                    for (int a = 0; a < d; ++a) {
                        if (in_r) {
                            double df = uc[v + stride[a]] - uc[v];
                            acc += df * df;
                            gsum -= df;           /* d/du(x) of (u(x+e)-u(x))^2 / 2 */
                        }
                        /* the difference that starts at x - e_a, if it is in X_R */
                        int prev_in = idx[a] >= 1;
                        for (int b = 0; b < d; ++b) {
                            int ib = idx[b] - (b == a ? 1 : 0);
                            if (ib > n[b] - 2) prev_in = 0;
                        }
                        if (prev_in) gsum += uc[v] - uc[v - stride[a]];
                    }
                    if (grad_u) grad_u[c * N + v] = 2.0 * gsum / XR;
                }
            }
        part[z] = acc;
    }
    double total = 0.0;
    for (int z = 0; z < nz; ++z) total += part[z];
    free(part);
    *value = total / XR;
}

void airo_tv(const airo_problem* p, const double* u, int kind, double* value, double* grad_u) {
    const int d = p->dim;
    const int nx = p->n[0], ny = p->n[1], nz = (d == 3) ? p->n[2] : 1;
    const int n[3] = {nx, ny, nz};
    const long N = (long)nx * ny * nz;
    const long stride[3] = {1, nx, (long)nx * ny};
    double XR = 1.0;
    for (int a = 0; a < d; ++a) XR *= (double)(n[a] - 1);
    /* per-voxel coefficient of each difference in the gradient:
     * aniso: sign(D); iso: D / ||J|| (0 where the term is 0) */
    double* coef = (double*)calloc((size_t)d * d * (size_t)N, sizeof(double));
    double total = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int idx[3] = {x, y, z};
                int in_r = 1;
                for (int a = 0; a < d; ++a)
                    if (idx[a] > n[a] - 2) in_r = 0;
                if (!in_r) continue;
                const long v = ((long)z * ny + y) * nx + x;
                double D[3][3], ss = 0.0, l1 = 0.0;
                for (int c = 0; c < d; ++c)
                    for (int a = 0; a < d; ++a) {
                        D[c][a] = u[c * N + v + stride[a]] - u[c * N + v];
                        ss += D[c][a] * D[c][a];
                        l1 += fabs(D[c][a]);
                    }
                if (kind == AIRO_REG_ANISO_TV) {
                    total += l1;
                    for (int c = 0; c < d; ++c)
                        for (int a = 0; a < d; ++a)
                            coef[((long)c * d + a) * N + v] =
                                D[c][a] > 0.0 ? 1.0 : (D[c][a] < 0.0 ? -1.0 : 0.0);
                } else {
                    const double nrm = sqrt(ss);
                    total += nrm;
                    for (int c = 0; c < d; ++c)
                        for (int a = 0; a < d; ++a)
                            coef[((long)c * d + a) * N + v] = nrm > 0.0 ? D[c][a] / nrm : 0.0;
                }
            }
    *value = total / XR;
    if (grad_u) {
        /* d/du_c(x) of the term at y: -coef at y = x, +coef at y = x - e_a */
        for (long i = 0; i < (long)d * N; ++i) grad_u[i] = 0.0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const long v = ((long)z * ny + y) * nx + x;
                    for (int c = 0; c < d; ++c)
                        for (int a = 0; a < d; ++a) {
                            const double k = coef[((long)c * d + a) * N + v];
                            if (k == 0.0) continue;
                            grad_u[c * N + v] -= k / XR;
                            grad_u[c * N + v + stride[a]] += k / XR;
                        }
                }
    }
    free(coef);
}

/* The regulariser the problem names, on a dense displacement u. */
static void reg_field(const airo_problem* p, const double* u, double* value, double* grad_u) {
    if (p->regulariser == AIRO_REG_DIFFUSION)
        airo_diffusion(p, u, value, grad_u);
    else
        airo_tv(p, u, p->regulariser, value, grad_u);
}

void airo_regulariser(const airo_problem* p, const double* theta, double* value, double* grad) {
    const long N = airo_nvox(p);
    const size_t fb = sizeof(double) * (size_t)p->dim * (size_t)N;
    if (p->transform == AIRO_TF_DENSE && p->diffeo_steps <= 0) {
        reg_field(p, theta, value, grad);
        return;
    }
    double* u = (double*)malloc(fb);
    double* gu = grad ? (double*)malloc(fb) : NULL;
    airo_displacement(p, theta, u);
    reg_field(p, u, value, gu);
    if (grad) displacement_adjoint(p, theta, gu, grad);
    free(u);
    free(gu);
}

int airo_objective_and_grad(const airo_problem* p, const double* fixed,
                            const double* moving, const double* theta,
                            double* value, double* grad) {
    const int d = p->dim;
    const long N = airo_nvox(p);
    const size_t fb = sizeof(double) * (size_t)d * (size_t)N;
    double* u = (double*)malloc(fb);
    double* dwdp = (double*)malloc(fb);
    double* g = (double*)malloc(fb);
    double* W = (double*)malloc(sizeof(double) * (size_t)N);
    double* dsdw = (double*)malloc(sizeof(double) * (size_t)N);
    unsigned char* mask = (unsigned char*)malloc((size_t)N);

    airo_displacement(p, theta, u);                       /* stage 1 */
    airo_sample(p, moving, u, W, mask, dwdp);             /* stage 2 */
    double S = 0.0, R = 0.0;
    int flags = airo_similarity(p, fixed, W, mask, &S, dsdw);   /* stage 3 */
    reg_field(p, u, &R, g);                               /* stage 4: g = dR/du */
    *value = S + p->lambda_diff * R;                      /* eq. (objective) */
    /* stage 5: g_a = dS/dW * dW/dp_a * (n_a - 1)/2 + lambda dR/du_a */
    for (int a = 0; a < d; ++a) {
        const double scale = (p->n[a] - 1) / 2.0;
        for (long v = 0; v < N; ++v) {
            double img = mask[v] ? dsdw[v] * dwdp[a * N + v] * scale : 0.0;
            g[a * N + v] = img + p->lambda_diff * g[a * N + v];
        }
    }
    displacement_adjoint(p, theta, g, grad);
    long np = airo_param_count(p);
    if (!isfinite(*value)) flags |= AIRO_FLAG_NONFINITE;
    for (long i = 0; i < np; ++i)
        if (!isfinite(grad[i])) {
            flags |= AIRO_FLAG_NONFINITE;
            break;
        }
    free(u);
    free(dwdp);
    free(g);
    free(W);
    free(dsdw);
    free(mask);
    return flags;
}

/* Sec. III-G: Adam (Kingma & Ba) with bias correction. */
void airo_adam_step(double* theta, const double* grad, double* m, double* v, long n,
                    double lr, double b1, double b2, double eps, int step) {
    const double bc1 = 1.0 - pow(b1, step);
    const double bc2 = 1.0 - pow(b2, step);
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mhat = m[i] / bc1;
        double vhat = v[i] / bc2;
        theta[i] -= lr * mhat / (sqrt(vhat) + eps);
    }
}

/* ---------------------------------------------------------------- pyramid */
void airo_pyramid_down(const double* in, const int n[3], double sigma, double* out) {
    const int r = (int)ceil(3.0 * sigma);
    double* w = (double*)malloc(sizeof(double) * (size_t)(2 * r + 1));
    double s = 0.0;
    for (int k = -r; k <= r; ++k) {
        w[k + r] = exp(-0.5 * (double)k * (double)k / (sigma * sigma));
        s += w[k + r];
    }
    for (int k = 0; k <= 2 * r; ++k) w[k] /= s;
    const long N = (long)n[0] * n[1] * n[2];
    double* a = (double*)malloc(sizeof(double) * (size_t)N);
    double* b = (double*)malloc(sizeof(double) * (size_t)N);
    memcpy(a, in, sizeof(double) * (size_t)N);
    const long stride[3] = {1, n[0], (long)n[0] * n[1]};
    for (int ax = 0; ax < 3; ++ax) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x) {
                    const int idx[3] = {x, y, z};
                    const long v = ((long)z * n[1] + y) * n[0] + x;
                    double acc = 0.0;
                    for (int k = -r; k <= r; ++k) {
                        int q = idx[ax] + k;
                        if (q < 0) q = 0;
                        if (q > n[ax] - 1) q = n[ax] - 1;
                        acc += w[k + r] * a[v + (long)(q - idx[ax]) * stride[ax]];
                    }
                    b[v] = acc;
                }
        double* t = a;
        a = b;
        b = t;
    }
    const int m[3] = {(n[0] + 1) / 2, (n[1] + 1) / 2, (n[2] + 1) / 2};
    for (int z = 0; z < m[2]; ++z)
        for (int y = 0; y < m[1]; ++y)
            for (int x = 0; x < m[0]; ++x)
                out[((long)z * m[1] + y) * m[0] + x] =
                    a[((long)(2 * z) * n[1] + 2 * y) * n[0] + 2 * x];
    free(a);
    free(b);
    free(w);
}

void airo_field_resample(const double* in, const int n[3], const int m[3], double* out) {
    const long Nn = (long)n[0] * n[1] * n[2];
    const long Nm = (long)m[0] * m[1] * m[2];
    for (int c = 0; c < 3; ++c) {
        const double* f = in + c * Nn;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
        for (int z = 0; z < m[2]; ++z)
            for (int y = 0; y < m[1]; ++y)
                for (int x = 0; x < m[0]; ++x) {
                    const int idx[3] = {x, y, z};
                    double p[3], fr[3];
                    int j[3];
                    for (int a = 0; a < 3; ++a) {
                        p[a] = (m[a] > 1) ? (double)idx[a] * (n[a] - 1) / (double)(m[a] - 1) : 0.0;
                        j[a] = (int)floor(p[a]);
                        if (j[a] > n[a] - 2) j[a] = n[a] - 2;
                        if (j[a] < 0) j[a] = 0;
                        fr[a] = p[a] - j[a];
                    }
                    double acc = 0.0;
                    for (int q = 0; q < 8; ++q) {
                        const int bx = q & 1, by = (q >> 1) & 1, bz = (q >> 2) & 1;
                        const double wq = (bx ? fr[0] : 1 - fr[0]) * (by ? fr[1] : 1 - fr[1]) *
                                          (bz ? fr[2] : 1 - fr[2]);
                        acc += wq * f[((long)(j[2] + bz) * n[1] + j[1] + by) * n[0] + j[0] + bx];
                    }
                    out[c * Nm + ((long)z * m[1] + y) * m[0] + x] = acc;
                }
    }
}

/* ---------------------------------------------------------------- conv3d */
void airo_conv3d_fwd(const double* x, const int n[3], int cin, const double* wt,
                     const double* bias, int cout, int act, double* y) {
    const int nx = n[0], ny = n[1], nz = n[2];
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
    for (int z = 0; z < nz; ++z)
        for (int yy = 0; yy < ny; ++yy)
            for (int xx = 0; xx < nx; ++xx) {
                const long v = ((long)z * ny + yy) * nx + xx;
                for (int co = 0; co < cout; ++co) {
                    double acc = bias ? bias[co] : 0.0;
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const int sz = z + dz, sy = yy + dy, sx = xx + dx;
                                if (sz < 0 || sz >= nz || sy < 0 || sy >= ny || sx < 0 || sx >= nx)
                                    continue;
                                const int tap = ((dz + 1) * 3 + dy + 1) * 3 + dx + 1;
                                const long s = ((long)sz * ny + sy) * nx + sx;
                                for (int ci = 0; ci < cin; ++ci)
                                    acc += wt[(long)co * 27 * cin + tap * cin + ci] * x[s * cin + ci];
                            }
                    if (act == 1 && acc < 0.0) acc *= 0.1;
                    y[v * cout + co] = acc;
                }
            }
}

void airo_conv3d_bwd(const double* x, const int n[3], int cin, const double* wt, int cout,
                     const double* dy, double* dx, double* dwt, double* db) {
    const int nx = n[0], ny = n[1], nz = n[2];
    const long N = (long)nx * ny * nz;
    if (dx) {
        /* dx[s][ci] = sum over outputs v that read s: dy[v][co] wt[co][tap][ci] */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
        for (int z = 0; z < nz; ++z)
            for (int yy = 0; yy < ny; ++yy)
                for (int xx = 0; xx < nx; ++xx) {
                    const long s = ((long)z * ny + yy) * nx + xx;
                    for (int ci = 0; ci < cin; ++ci) {
                        double acc = 0.0;
                        for (int dz = -1; dz <= 1; ++dz)
                            for (int dyy = -1; dyy <= 1; ++dyy)
                                for (int dxx = -1; dxx <= 1; ++dxx) {
                                    /* output v = s - d reads s through tap d */
                                    const int vz = z - dz, vy = yy - dyy, vx = xx - dxx;
                                    if (vz < 0 || vz >= nz || vy < 0 || vy >= ny || vx < 0 || vx >= nx)
                                        continue;
                                    const int tap = ((dz + 1) * 3 + dyy + 1) * 3 + dxx + 1;
                                    const long v = ((long)vz * ny + vy) * nx + vx;
                                    for (int co = 0; co < cout; ++co)
                                        acc += dy[v * cout + co] * wt[(long)co * 27 * cin + tap * cin + ci];
                                }
                        dx[s * cin + ci] = acc;
                    }
                }
    }
    if (dwt) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) NTHREADS
#endif
        for (int co = 0; co < cout; ++co)
            for (int tap = 0; tap < 27; ++tap) {
                const int dz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dxx = tap % 3 - 1;
                for (int ci = 0; ci < cin; ++ci) {
                    double acc = 0.0;
                    for (int z = 0; z < nz; ++z)
                        for (int yy = 0; yy < ny; ++yy)
                            for (int xx = 0; xx < nx; ++xx) {
                                const int sz = z + dz, sy = yy + dyy, sx = xx + dxx;
                                if (sz < 0 || sz >= nz || sy < 0 || sy >= ny || sx < 0 || sx >= nx)
                                    continue;
                                const long v = ((long)z * ny + yy) * nx + xx;
                                const long s = ((long)sz * ny + sy) * nx + sx;
                                acc += dy[v * cout + co] * x[s * cin + ci];
                            }
                    dwt[(long)co * 27 * cin + tap * cin + ci] = acc;
                }
            }
    }
    if (db) {
        for (int co = 0; co < cout; ++co) {
            double acc = 0.0;
            for (long v = 0; v < N; ++v) acc += dy[v * cout + co];
            db[co] = acc;
        }
    }
}
