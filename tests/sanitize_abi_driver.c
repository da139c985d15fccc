/* Driver for the address/undefined-behaviour sanitizer build of libnbreg's
 * host code: every entry point of include/nbreg.h is called on a host-only
 * context (device -1, which validates arguments and launches nothing) with
 * valid arguments (expect NB_ERR_UNSUPPORTED) and with each kind of invalid
 * argument (expect NB_ERR_INVALID_ARG).  Device pointers are fake addresses
 * that the host code must never dereference; host arrays (batched offsets,
 * the scheduler's level_end) are real.  Exit status 0 = every check held. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "nbreg.h"

static int g_fail = 0;
#define EXPECT(call, want)                                                              \
    do {                                                                                \
        const int got_ = (call);                                                        \
        if (got_ != (want)) {                                                           \
            fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, \
                    got_, (want));                                                      \
            g_fail = 1;                                                                 \
        }                                                                               \
    } while (0)

#define P(k) ((void *)(uintptr_t)(0x10000u * (k)))

int main(void)
{
    const int E = NB_ERR_INVALID_ARG, U = NB_ERR_UNSUPPORTED;
    for (int code = 1; code >= -6; --code)
        if (!nb_error_string(code) || !nb_error_string(code)[0]) g_fail = 1;
    if (nb_version() < 10000) g_fail = 1;

    EXPECT(nb_ctx_create(NULL, -1, NULL), E);
    nb_ctx *ctx = NULL;
    EXPECT(nb_ctx_create(&ctx, -1, NULL), NB_OK);
    if (!ctx) return 1;

    /* context settings */
    EXPECT(nb_ctx_set_stream(ctx, NULL), NB_OK);
    EXPECT(nb_ctx_set_plan(ctx, 4, 0, 0), E);
    EXPECT(nb_ctx_set_plan(ctx, 3, 0, 0), NB_OK);
    EXPECT(nb_ctx_set_plan(ctx, 1, 3, 0), E);
    EXPECT(nb_ctx_set_plan(ctx, 1, 1, -2), E);
    EXPECT(nb_ctx_set_plan(ctx, 2, 4, 16), NB_OK);
    EXPECT(nb_ctx_set_plan(ctx, 0, 0, 0), NB_OK);
    char buf[8];
    EXPECT(nb_ctx_last_plan(ctx, buf, (int)sizeof buf), NB_OK);   /* truncated safely */
    EXPECT(nb_ctx_last_plan(ctx, buf, 0), E);
    EXPECT(nb_ctx_set_scratch_limit(ctx, -1), E);
    EXPECT(nb_ctx_set_scratch_limit(ctx, 1 << 20), NB_OK);
    EXPECT(nb_ctx_enable_timing(ctx, 1), NB_OK);
    double ms = -1.0;
    int64_t launches = -1;
    EXPECT(nb_ctx_kernel_time(ctx, 0, &ms, &launches), NB_OK);
    EXPECT(nb_ctx_kernel_time(ctx, 99, &ms, &launches), E);
    EXPECT(nb_ctx_kernel_time(ctx, 0, NULL, &launches), E);
    EXPECT(nb_ctx_reset_timing(ctx), NB_OK);
    EXPECT(nb_ctx_set_mixed_tolerance(ctx, -1.0, 32.0), E);
    EXPECT(nb_ctx_set_mixed_tolerance(ctx, 5e-6, 0.0), E);
    EXPECT(nb_ctx_set_mixed_tolerance(ctx, 5e-6, 32.0), NB_OK);
    EXPECT(nb_ctx_set_refine_buffer_rows(ctx, -1), E);
    EXPECT(nb_ctx_set_refine_buffer_rows(ctx, 3), NB_OK);
    EXPECT(nb_ctx_set_refine_buffer_rows(ctx, 0), NB_OK);
    int32_t refined = -1;
    EXPECT(nb_ctx_last_refined_rows(ctx, &refined), NB_OK);
    EXPECT(nb_ctx_last_refined_rows(ctx, NULL), E);
    int64_t ws = 0;
    EXPECT(nb_fixed_workspace_bytes(&ws), NB_OK);
    EXPECT(nb_fixed_workspace_bytes(NULL), E);
    if (ws <= 0) g_fail = 1;

    /* predictor */
    EXPECT(nb_predict(ctx, 10, 0.5, P(1), P(2), P(3), P(4), P(5), NULL, P(6), P(7), NULL), U);
    EXPECT(nb_predict(ctx, 0, 0.5, P(1), P(2), P(3), P(4), P(5), NULL, P(6), P(7), NULL), E);
    EXPECT(nb_predict(ctx, 10, 0.5, P(1), P(2), P(3), P(4), P(5), P(8), P(6), P(7), NULL), E);
    EXPECT(nb_predict(ctx, 10, 0.5, NULL, P(2), P(3), P(4), P(5), NULL, P(6), P(7), NULL), E);

    /* regular force, its allocation-free variant, and the fit loop */
    for (int variant = 0; variant < 2; ++variant) {
        int (*rf)(nb_ctx *, int64_t, const double *, const double *, const double *, int32_t,
                  const int32_t *, const double *, int32_t, nb_precision, double *, double *,
                  int32_t *, int32_t *, int32_t *, uint32_t *) =
            variant ? nb_regular_force_noalloc : nb_regular_force;
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_MIXED, P(6), P(7), P(8),
                  P(9), P(10), NULL), U);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 0, NB_FP64, P(6), P(7), P(8),
                  NULL, P(10), P(11)), U);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 0, NULL, NULL, 8, NB_FP64, NULL, NULL, NULL, NULL,
                  P(10), NULL), U);
        EXPECT(rf(NULL, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_FP64, P(6), P(7), P(8),
                  P(9), P(10), NULL), E);
        EXPECT(rf(ctx, (int64_t)1 << 31, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_FP64, P(6),
                  P(7), P(8), P(9), P(10), NULL), E);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), -1, P(4), P(5), 8, NB_FP64, P(6), P(7), P(8),
                  P(9), P(10), NULL), E);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), -1, NB_FP64, P(6), P(7), P(8),
                  P(9), P(10), NULL), E);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, (nb_precision)2, P(6), P(7),
                  P(8), P(9), P(10), NULL), E);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_FP64, P(6), P(7), P(8),
                  NULL, P(10), NULL), E);
        EXPECT(rf(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_FP64, P(6), P(7), P(8),
                  P(9), NULL, NULL), E);
    }
    int32_t rounds = -1;
    EXPECT(nb_regular_force_fit(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_FP64, 40, 4,
                                P(6), P(7), P(8), P(9), P(10), NULL, &rounds), U);
    EXPECT(nb_regular_force_fit(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 0, NB_FP64, 40, 4,
                                P(6), P(7), P(8), P(9), P(10), NULL, &rounds), E);
    EXPECT(nb_regular_force_fit(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), 8, NB_FP64, 0, 4,
                                P(6), P(7), P(8), P(9), P(10), NULL, &rounds), E);

    /* adjoint */
    EXPECT(nb_regular_force_adjoint(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), P(6), P(7),
                                    P(8), P(9), P(10), NULL), U);
    EXPECT(nb_regular_force_adjoint(ctx, 100, P(1), P(2), P(3), 10, P(4), P(5), NULL, P(7),
                                    P(8), P(9), P(10), NULL), E);
    EXPECT(nb_regular_force_adjoint(ctx, 0, P(1), P(2), P(3), 10, P(4), P(5), P(6), P(7),
                                    P(8), P(9), P(10), NULL), E);

    /* batched: offsets are read on the host */
    const int64_t joff[4] = {0, 100, 100, 350}, ioff[4] = {0, 10, 10, 60};
    const int64_t jbad[4] = {0, 100, 90, 350}, ibad[4] = {1, 10, 10, 60};
    EXPECT(nb_regular_force_batched(ctx, 3, joff, ioff, P(1), P(2), P(3), P(4), P(5), 16,
                                    NB_MIXED, P(6), P(7), P(8), P(9), P(10), NULL), U);
    EXPECT(nb_regular_force_batched(ctx, 3, jbad, ioff, P(1), P(2), P(3), P(4), P(5), 16,
                                    NB_MIXED, P(6), P(7), P(8), P(9), P(10), NULL), E);
    EXPECT(nb_regular_force_batched(ctx, 3, joff, ibad, P(1), P(2), P(3), P(4), P(5), 16,
                                    NB_MIXED, P(6), P(7), P(8), P(9), P(10), NULL), E);
    EXPECT(nb_regular_force_batched(ctx, 0, joff, ioff, P(1), P(2), P(3), P(4), P(5), 16,
                                    NB_MIXED, P(6), P(7), P(8), P(9), P(10), NULL), E);
    EXPECT(nb_regular_force_batched(ctx, 3, NULL, ioff, P(1), P(2), P(3), P(4), P(5), 16,
                                    NB_MIXED, P(6), P(7), P(8), P(9), P(10), NULL), E);
    EXPECT(nb_autotune(ctx, 4096, NULL, 0), U);
    EXPECT(nb_autotune(ctx, 10, NULL, 0), E);

    /* the rest of the block step */
    EXPECT(nb_irregular_force(ctx, 100, P(1), P(2), P(3), 10, P(4), 8, P(5), P(6), P(7), P(8),
                              NULL), U);
    EXPECT(nb_irregular_force(ctx, 100, P(1), P(2), P(3), 10, P(4), -1, P(5), P(6), P(7), P(8),
                              NULL), E);
    EXPECT(nb_hermite_correct(ctx, 100, P(1), P(2), P(3), P(4), P(5), P(6), P(7), P(8), P(9),
                              P(10), P(11)), U);
    EXPECT(nb_hermite_correct(ctx, 0, P(1), P(2), P(3), P(4), P(5), P(6), P(7), P(8), P(9),
                              P(10), P(11)), E);
    EXPECT(nb_potential(ctx, 100, P(1), P(2), P(3), NULL), U);
    EXPECT(nb_potential(ctx, 100, NULL, P(2), P(3), NULL), E);

    /* radius control */
    EXPECT(nb_radius_update(ctx, 10, P(1), P(2), 40, 0.5, 2.0, P(3)), U);
    EXPECT(nb_radius_update(ctx, 10, P(1), P(2), 0, 0.5, 2.0, P(3)), E);
    EXPECT(nb_radius_update(ctx, 10, P(1), P(2), 40, 2.0, 0.5, P(3)), E);

    /* scheduler: build/update validate on the host; next is host-only */
    EXPECT(nb_sched_build(ctx, 100, P(1), 20, P(2), P(3), NULL), U);
    EXPECT(nb_sched_build(ctx, 100, P(1), 64, P(2), P(3), NULL), E);
    EXPECT(nb_sched_update(ctx, 100, 10, 5, P(1), 20, P(2), P(3), NULL), U);
    EXPECT(nb_sched_update(ctx, 100, 101, 5, P(1), 20, P(2), P(3), NULL), E);
    const int32_t le[6] = {10, 10, 7, 3, 1, 0};   /* k_max = 4 */
    double t_new = 0.0;
    int32_t level = -1, n_active = -1;
    EXPECT(nb_sched_next(0.0, 4, le, &t_new, &level, &n_active), NB_OK);
    if (t_new != 0.0625 || level != 4 || n_active != 1) g_fail = 1;
    EXPECT(nb_sched_next(0.0625, 4, le, &t_new, &level, &n_active), NB_OK);
    if (t_new != 0.125 || level != 3 || n_active != 3) g_fail = 1;
    const int32_t le_bad[6] = {10, 10, 7, 8, 1, 0};
    EXPECT(nb_sched_next(0.0, 4, le_bad, &t_new, &level, &n_active), E);
    EXPECT(nb_sched_next(0.03, 4, le, &t_new, &level, &n_active), E);
    EXPECT(nb_sched_next(0.0, 4, NULL, &t_new, &level, &n_active), E);

    EXPECT(nb_ctx_destroy(ctx), NB_OK);
    EXPECT(nb_ctx_destroy(NULL), E);
    if (g_fail) fprintf(stderr, "libnbreg sanitizer driver: FAILED\n");
    else printf("libnbreg sanitizer driver: ok\n");
    return g_fail;
}
