/*
 * Exercises the host side of the library's C-ABI (plan creation, queries,
 * tilings, argument validation that returns before any launch) so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the host code can
 * check it (test infrastructure; built and run by tests/test_sanitizers.py).
 * No call here reaches the GPU: every entry point below either is host-only
 * or is handed an argument that it rejects before touching a device.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../include/airhip.h"

static int g_bad = 0;

#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "line %d: expectation failed: %s\n", __LINE__, #cond); \
            ++g_bad;                                                        \
        }                                                                   \
    } while (0)

static air_problem problem(int dim, int nx, int ny, int nz, int tf, int sim) {
    air_problem p;
    memset(&p, 0, sizeof(p));
    p.dim = dim;
    p.n[0] = nx;
    p.n[1] = ny;
    p.n[2] = dim == 3 ? nz : 1;
    p.transform = tf;
    for (int a = 0; a < 3; ++a) {
        p.spacing[a] = tf == AIR_TF_DENSE ? 1 : 8;
        p.sigma[a] = 12.0f;
    }
    p.similarity = sim;
    p.lambda_diff = 0.05f;
    p.lcc_radius = 2;
    return p;
}

int main(void) {
    /* valid plans of every kind, their queries and tilings */
    for (int tf = AIR_TF_BSPLINE3; tf <= AIR_TF_WENDLAND; ++tf)
        for (int sim = AIR_SIM_MSE; sim <= AIR_SIM_LCC; ++sim)
            for (int dim = 2; dim <= 3; ++dim)
                for (int k = 0; k <= 3; k += 3) {
                    air_problem p = problem(dim, 70, 45, 53, tf, sim);
                    p.diffeo_steps = k;
                    air_plan* plan = NULL;
                    EXPECT(air_plan_create(&p, 1, &plan) == AIR_OK);
                    if (!plan) continue;
                    size_t ws = 0;
                    int64_t np = 0;
                    EXPECT(air_plan_workspace_bytes(plan, &ws) == AIR_OK && ws > 0);
                    EXPECT(air_plan_param_count(plan, 0, &np) == AIR_OK && np > 0);
                    EXPECT(air_plan_param_count(plan, 1, &np) == AIR_ERR_SHAPE);
                    const int nt = air_tiling_count(dim);
                    for (int t = 0; t < nt; ++t) {
                        int32_t tx = 0, ty = 0, cc = 0, got = -1;
                        EXPECT(air_tiling_describe(dim, t, &tx, &ty, &cc) == AIR_OK);
                        if (air_plan_set_tiling(plan, t) == AIR_OK) {
                            EXPECT(air_plan_get_tiling(plan, &got) == AIR_OK && got == t);
                            EXPECT(air_plan_workspace_bytes(plan, &ws) == AIR_OK);
                        }
                    }
                    /* entry points reject null or misaligned arguments before
                     * any device work */
                    float* fake = (float*)(uintptr_t)0x1000;
                    float* odd = (float*)(uintptr_t)0x1004;
                    float value = 0.f;
                    EXPECT(air_objective_and_grad(plan, NULL, fake, fake, &value, fake, fake, ws,
                                                  NULL) == AIR_ERR_INVALID_ARG);
                    EXPECT(air_objective_and_grad(plan, odd, fake, fake, &value, fake, fake, ws,
                                                  NULL) == AIR_ERR_ALIGN);
                    EXPECT(air_objective_and_grad(plan, fake, fake, fake, &value, fake, NULL, ws,
                                                  NULL) == AIR_ERR_WORKSPACE);
                    EXPECT(air_objective_and_grad_noalloc(plan, NULL, fake, fake, &value, fake,
                                                          NULL) == AIR_ERR_INVALID_ARG);
                    EXPECT(air_objective_and_grad_noalloc(plan, odd, fake, fake, &value, fake,
                                                          NULL) == AIR_ERR_ALIGN);
                    EXPECT(air_warp(plan, 3, fake, fake, fake, NULL, NULL) != AIR_OK);
                    EXPECT(air_similarity(plan, 2, fake, fake, NULL, &value, fake, ws, NULL) !=
                           AIR_OK);
                    air_plan_destroy(plan);
                }
    /* invalid problems */
    {
        air_problem bad[6];
        bad[0] = problem(3, 1, 24, 20, AIR_TF_BSPLINE3, AIR_SIM_NCC);      /* n < 2 */
        bad[1] = problem(3, 24, 24, 20, AIR_TF_BSPLINE3, 7);               /* similarity */
        bad[2] = problem(3, 24, 24, 20, 9, AIR_SIM_NCC);                   /* transform */
        bad[3] = problem(3, 2048, 2048, 2048, AIR_TF_BSPLINE3, AIR_SIM_NCC);
        bad[4] = problem(3, 8, 4096, 4096, AIR_TF_BSPLINE3, AIR_SIM_NCC);  /* ny nz >= 2^24 */
        bad[5] = problem(4, 24, 24, 20, AIR_TF_BSPLINE3, AIR_SIM_NCC);     /* dim */
        for (int i = 0; i < 6; ++i) {
            air_plan* plan = NULL;
            EXPECT(air_plan_create(&bad[i], 1, &plan) != AIR_OK && plan == NULL);
        }
        air_plan* plan = NULL;
        air_problem two[2] = {problem(3, 24, 24, 20, AIR_TF_BSPLINE3, AIR_SIM_NCC),
                              problem(3, 24, 24, 20, AIR_TF_BSPLINE3, AIR_SIM_MSE)};
        EXPECT(air_plan_create(two, 2, &plan) == AIR_ERR_UNSUPPORTED && plan == NULL);
        EXPECT(air_plan_create(two, 0, &plan) == AIR_ERR_INVALID_ARG);
        EXPECT(air_plan_create(NULL, 1, &plan) == AIR_ERR_INVALID_ARG);
    }
    /* a batch plan, host-only helpers, error strings */
    {
        air_problem ps[3] = {problem(3, 96, 112, 128, AIR_TF_BSPLINE3, AIR_SIM_NCC),
                             problem(3, 160, 96, 144, AIR_TF_BSPLINE3, AIR_SIM_NCC),
                             problem(3, 128, 128, 128, AIR_TF_BSPLINE3, AIR_SIM_NCC)};
        air_plan* plan = NULL;
        EXPECT(air_plan_create(ps, 3, &plan) == AIR_OK);
        size_t ws = 0;
        EXPECT(air_plan_workspace_bytes(plan, &ws) == AIR_OK && ws > 0);
        air_plan_destroy(plan);
        float bt[2];
        EXPECT(air_adam_bias_terms(0.01f, 0.9f, 0.999f, 3, bt) == AIR_OK);
        EXPECT(air_adam_bias_terms(0.01f, 0.9f, 0.999f, 0, bt) != AIR_OK);
        size_t pb = 0;
        const int32_t n3[3] = {33, 20, 17};
        EXPECT(air_pyramid_workspace_bytes(n3, &pb) == AIR_OK);
        for (int st = 0; st <= 8; ++st) EXPECT(air_strerror((air_status)st) != NULL);
    }
    /* the network object: layout queries only (no pass runs) */
    {
        air_cnn* net = NULL;
        EXPECT(air_cnn_create(40, 1, &net) == AIR_ERR_SHAPE && net == NULL);
        EXPECT(air_cnn_create(64, 2, &net) == AIR_OK && net != NULL);
        int64_t np = 0, wo = 0, bo = 0;
        size_t wsb = 0;
        int32_t ci = 0, co = 0;
        EXPECT(air_cnn_sizes(net, &np, &wsb) == AIR_OK && np > 0 && wsb > 0);
        for (int l = 0; l < 6; ++l)
            EXPECT(air_cnn_layer(net, l, &ci, &co, &wo, &bo) == AIR_OK && wo < np && bo < np);
        EXPECT(air_cnn_layer(net, 6, &ci, &co, &wo, &bo) == AIR_ERR_SHAPE);
        EXPECT(air_cnn_forward(net, NULL, NULL, NULL, NULL, NULL, 0, NULL) == AIR_ERR_INVALID_ARG);
        air_cnn_destroy(net);
    }
    printf("C-ABI host sanitizer driver: %d failures\n", g_bad);
    return g_bad ? 1 : 0;
}
