/*
 * Drives every entry point of the FP64 oracle on small problems so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of oracle.c can check
 * its memory accesses and arithmetic (test infrastructure; built and run by
 * tests/test_sanitizers.py). Inputs are deterministic pseudo-random values
 * from a fixed linear congruential sequence; the driver checks only that
 * results are finite, the sanitizers check the rest.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/oracle.h"

static unsigned long long g_state = 88172645463325252ull;

static double urand(void) {
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static double* vec(long n, double scale) {
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (long i = 0; i < n; ++i) v[i] = scale * (2.0 * urand() - 1.0);
    return v;
}

static int finite_all(const double* v, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int run_problem(airo_problem p) {
    if (airo_check(&p) != 0) {
        fprintf(stderr, "invalid problem\n");
        return 1;
    }
    const long N = airo_nvox(&p);
    const long np = airo_param_count(&p);
    double* F = vec(N, 1.0);
    double* M = vec(N, 1.0);
    /* displacements of about a voxel in normalised units */
    double* th = vec(np, 2.0 / (double)(p.n[0] > 1 ? p.n[0] - 1 : 1));
    double* g = vec(np, 0.0);
    double val = 0.0;
    (void)airo_objective_and_grad(&p, F, M, th, &val, g);
    int ok = isfinite(val) && finite_all(g, np);
    /* stages on their own */
    double* u = vec((long)p.dim * N, 0.0);
    double* W = vec(N, 0.0);
    double* dW = vec((long)p.dim * N, 0.0);
    unsigned char* mk = (unsigned char*)malloc((size_t)N);
    airo_displacement(&p, th, u);
    airo_sample(&p, M, u, W, mk, dW);
    double s = 0.0;
    double* ds = vec(N, 0.0);
    (void)airo_similarity(&p, F, W, mk, &s, ds);
    double r = 0.0;
    airo_regulariser(&p, th, &r, g);
    ok = ok && isfinite(s) && isfinite(r) && finite_all(ds, N);
    free(F); free(M); free(th); free(g); free(u); free(W); free(dW); free(mk); free(ds);
    return ok ? 0 : 1;
}

int main(void) {
    int bad = 0;
    for (int sim = AIRO_SIM_MSE; sim <= AIRO_SIM_LCC; ++sim)
        for (int tf = AIRO_TF_BSPLINE3; tf <= AIRO_TF_WENDLAND; ++tf)
            for (int dim = 2; dim <= 3; ++dim)
                for (int k = 0; k <= 2; k += 2)
                    for (int reg = AIRO_REG_DIFFUSION; reg <= AIRO_REG_ISO_TV; ++reg) {
                        airo_problem p = {0};
                        p.dim = dim;
                        p.n[0] = 13; p.n[1] = 11; p.n[2] = dim == 3 ? 9 : 1;
                        p.transform = tf;
                        for (int a = 0; a < 3; ++a) {
                            p.spacing[a] = tf == AIRO_TF_DENSE ? 1 : 4;
                            p.sigma[a] = 5.0;
                        }
                        p.similarity = sim;
                        p.lambda_diff = 0.3;
                        p.diffeo_steps = k;
                        p.regulariser = reg;
                        p.lcc_radius = 2;
                        if (run_problem(p) != 0) {
                            fprintf(stderr, "non-finite: sim %d tf %d dim %d K %d reg %d\n", sim,
                                    tf, dim, k, reg);
                            ++bad;
                        }
                    }
    /* 3D convolution forward and backward */
    {
        const int n[3] = {6, 5, 4};
        const int cin = 3, cout = 4;
        const long V = (long)n[0] * n[1] * n[2];
        double* x = vec(V * cin, 1.0);
        double* wt = vec((long)cout * 27 * cin, 0.3);
        double* b = vec(cout, 0.1);
        double* y = vec(V * cout, 0.0);
        double* dy = vec(V * cout, 1.0);
        double* dx = vec(V * cin, 0.0);
        double* dwt = vec((long)cout * 27 * cin, 0.0);
        double* db = vec(cout, 0.0);
        airo_conv3d_fwd(x, n, cin, wt, b, cout, 1, y);
        airo_conv3d_bwd(x, n, cin, wt, cout, dy, dx, dwt, db);
        if (!finite_all(y, V * cout) || !finite_all(dwt, (long)cout * 27 * cin)) ++bad;
        free(x); free(wt); free(b); free(y); free(dy); free(dx); free(dwt); free(db);
    }
    /* pyramid level, field transfer, Adam */
    {
        const int n[3] = {9, 8, 7};
        const long V = (long)n[0] * n[1] * n[2];
        double* in = vec(V, 1.0);
        double* out = vec(5 * 4 * 4, 0.0);
        airo_pyramid_down(in, n, 1.0, out);
        const int m[3] = {12, 10, 9};
        double* f = vec(3 * V, 0.1);
        double* fm = vec(3L * m[0] * m[1] * m[2], 0.0);
        airo_field_resample(f, n, m, fm);
        double* t = vec(50, 1.0);
        double* gr = vec(50, 1.0);
        double* mm = vec(50, 0.0);
        double* vv = vec(50, 0.0);
        for (int i = 0; i < 50; ++i) mm[i] = vv[i] = 0.0;
        for (int step = 1; step <= 3; ++step)
            airo_adam_step(t, gr, mm, vv, 50, 0.01, 0.9, 0.999, 1e-8, step);
        if (!finite_all(out, 5 * 4 * 4) || !finite_all(t, 50)) ++bad;
        free(in); free(out); free(f); free(fm); free(t); free(gr); free(mm); free(vv);
    }
    printf("oracle sanitizer driver: %d failures\n", bad);
    return bad ? 1 : 0;
}
