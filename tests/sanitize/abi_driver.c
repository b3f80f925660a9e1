/* Host-side paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer, run where no
 * GPU is present: argument validation of every entry point, and plan and batch creation for a sweep
 * of valid problems. Plan creation builds every FP64 table (TA, TB, Tf, FFT roots, the chirp-folded
 * HT and its variants) and the radix plans on the host before its first device call, which then
 * fails for want of a device; the sanitizers watch all of that host code. Exit status 0 when every
 * status code is the expected one. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fx.h"

static int fails = 0;
static int plans_built = 0;

#define EXPECT(cond, what)                                                              \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            fprintf(stderr, "FAIL %s (line %d): last error '%s'\n", what, __LINE__,     \
                    fx_last_error());                                                   \
            ++fails;                                                                    \
        }                                                                               \
    } while (0)

static fx_problem problem(int ndim, const int64_t* shape, const int32_t* lam, double t, int prec, int sched) {
    fx_problem p;
    fx_problem_init(&p);
    p.ndim = ndim;
    for (int j = 0; j < ndim; ++j) {
        p.shape[j] = shape[j];
        p.lambda[j] = lam[j];
        p.dx[j] = 0.5 + 0.25 * j;
    }
    p.m_over_hbar = 1.0;
    p.t_flight = t;
    p.precision = prec;
    p.schedule = sched;
    return p;
}

/* A valid problem: FX_OK where a device exists, else the device error of the table upload;
 * FX_EUNSUPPORTED is allowed for axes beyond the in-LDS transform limits. */
static void valid_plan(const fx_problem* p, const double* const* phase) {
    fx_plan* h = NULL;
    fx_status s = phase ? fx_plan_create_spectrum(p, phase, &h) : fx_plan_create(p, &h);
    EXPECT(s == FX_OK || s == FX_EDEVICE || s == FX_EUNSUPPORTED, "valid problem");
    if (s == FX_OK) {
        char buf[4096];
        EXPECT(fx_plan_describe(h, buf, sizeof buf) == FX_OK, "describe");
        EXPECT(fx_plan_destroy(h) == FX_OK, "destroy");
    } else {
        EXPECT(h == NULL, "no plan handed out on failure");
    }
    ++plans_built;
}

int main(void) {
    /* status strings, including unknown codes */
    for (int c = -6; c <= 1; ++c) EXPECT(fx_status_string((fx_status)c) != NULL, "status string");

    /* invalid problems are rejected on the host */
    const int64_t sh1[3] = {16, 16, 16};
    const int32_t la1[3] = {3, 3, 3};
    fx_problem p = problem(1, sh1, la1, 2.0, FX_PREC_C128, FX_SCHED_PAPER);
    fx_plan* h = NULL;
    EXPECT(fx_plan_create(NULL, &h) == FX_EINVAL, "NULL problem");
    EXPECT(fx_plan_create(&p, NULL) == FX_EINVAL, "NULL out");
    for (int k = 0; k < 15; ++k) {
        fx_problem q = p;
        switch (k) {
            case 0: q.ndim = 0; break;
            case 1: q.ndim = 4; break;
            case 2: q.shape[0] = 0; break;
            case 3: q.dx[0] = 0.0; break;
            case 4: q.dx[0] = -1.0; break;
            case 5: q.dx[0] = NAN; break;
            case 6: q.lambda[0] = 0; break;
            case 7: q.lambda[0] = -3; break;
            case 8: q.m_over_hbar = 0.0; break;
            case 9: q.m_over_hbar = INFINITY; break;
            case 10: q.t_flight = NAN; break;
            case 11: q.t_flight = INFINITY; break;
            case 12: q.precision = 7; break;
            case 13: q.schedule = 9; break;
            case 14: q.a[0] = INFINITY; break;
        }
        h = NULL;
        EXPECT(fx_plan_create(&q, &h) == FX_EINVAL && h == NULL, "invalid problem rejected");
    }
    {
        fx_problem q = p;
        q.shape[0] = (int64_t)1 << 40;  /* far beyond the supported sizes */
        fx_status s = fx_plan_create(&q, &h);
        EXPECT(s == FX_EINVAL || s == FX_EUNSUPPORTED, "oversized axis rejected");
    }

    /* NULL plans on every entry point */
    char buf[64];
    int64_t q64 = 0;
    size_t sz = 0;
    int32_t n32 = 0;
    EXPECT(fx_plan_destroy(NULL) == FX_EINVAL || fx_plan_destroy(NULL) == FX_OK, "destroy NULL");
    EXPECT(fx_plan_num_terms(NULL, &q64) == FX_EINVAL, "num_terms NULL");
    EXPECT(fx_plan_workspace_size(NULL, &sz) == FX_EINVAL, "workspace_size NULL");
    EXPECT(fx_plan_set_workspace(NULL, NULL, 0) == FX_EINVAL, "set_workspace NULL");
    EXPECT(fx_expand(NULL, buf, buf, NULL, NULL) == FX_EINVAL, "expand NULL");
    EXPECT(fx_expand_range(NULL, buf, buf, 0, 1, 0, NULL) == FX_EINVAL, "expand_range NULL");
    EXPECT(fx_expand_many(NULL, 2, buf, buf, NULL, NULL) == FX_EINVAL, "expand_many NULL");
    EXPECT(fx_expand_noalloc(NULL, buf, buf, NULL, NULL) == FX_EINVAL, "expand_noalloc NULL");
    EXPECT(fx_density(NULL, buf, buf, NULL) == FX_EINVAL, "density NULL");
    EXPECT(fx_column_density(NULL, buf, 0, buf, NULL) == FX_EINVAL, "column_density NULL");
    EXPECT(fx_expand_adjoint(NULL, buf, buf, NULL) == FX_EINVAL, "expand_adjoint NULL");
    EXPECT(fx_density_adjoint(NULL, buf, buf, buf, NULL) == FX_EINVAL, "density_adjoint NULL");
    EXPECT(fx_density_adjoint_many(NULL, 2, buf, buf, buf, NULL) == FX_EINVAL, "density_adjoint_many NULL");
    EXPECT(fx_expand_pair(NULL, buf, buf, buf, buf, buf, NULL) == FX_EINVAL, "expand_pair NULL");
    EXPECT(fx_plan_pair_workspace_size(NULL, &sz) == FX_EINVAL, "pair_workspace_size NULL");
    EXPECT(fx_far_field(NULL, buf, buf, NULL, NULL) == FX_EINVAL, "far_field NULL");
    EXPECT(fx_brute_force(NULL, buf, buf, NULL, NULL) == FX_EINVAL, "brute_force NULL");
    EXPECT(fx_plan_set_timing(NULL, 1) == FX_EINVAL, "set_timing NULL");
    EXPECT(fx_plan_describe(NULL, buf, sizeof buf) == FX_EINVAL, "describe NULL");
    EXPECT(fx_batch_num_classes(NULL, &n32) == FX_EINVAL, "batch_num_classes NULL");
    EXPECT(fx_batch_run(NULL, NULL, NULL, NULL, NULL) == FX_EINVAL, "batch_run NULL");

    /* fault injection at plan creation */
    setenv("FX_FAULT_INJECT_PLAN", "1", 1);
    EXPECT(fx_plan_create(&p, &h) == FX_ENOMEM, "fault injection");
    unsetenv("FX_FAULT_INJECT_PLAN");

    /* a sweep of valid problems: even and odd lengths, magnifications with every g = gcd(lam, M)
     * class, 1-D to 3-D, both precisions and both schedules, negative flights */
    static const int64_t Ms[] = {1, 2, 7, 9, 16, 24, 33, 45, 48, 64, 96, 128, 384, 512, 1000, 1024, 4096};
    static const int32_t lams[] = {1, 2, 3, 5, 8, 16, 20, 32, 40, 50};
    const int nM = (int)(sizeof Ms / sizeof Ms[0]), nl = (int)(sizeof lams / sizeof lams[0]);
    for (int i = 0; i < nM; ++i)
        for (int k = 0; k < nl; ++k)
            for (int prec = 0; prec < 2; ++prec) {
                const int64_t s[1] = {Ms[i]};
                const int32_t l[1] = {lams[k]};
                fx_problem q = problem(1, s, l, (k & 1) ? -37.5 : 412.0, prec, (i + k) & 1);
                valid_plan(&q, NULL);
            }
    {
        const int64_t s3[3][3] = {{32, 32, 256}, {48, 48, 384}, {64, 64, 512}};
        for (int c = 0; c < 3; ++c)
            for (int prec = 0; prec < 2; ++prec) {
                const int32_t l[3] = {40, 40, 40};
                fx_problem q = problem(3, s3[c], l, 400.0, prec, FX_SCHED_PAPER);
                valid_plan(&q, NULL);
            }
        const int64_t s2[2] = {512, 512};
        const int32_t l2[2] = {32, 32};
        fx_problem q2 = problem(2, s2, l2, 2000.0, FX_PREC_C64_PHASE64, FX_SCHED_PAPER);
        valid_plan(&q2, NULL);
        const int64_t s3b[3] = {64, 64, 1024};
        const int32_t l3b[3] = {50, 50, 5};
        fx_problem q3 = problem(3, s3b, l3b, 800.0, FX_PREC_C64_PHASE64, FX_SCHED_PAPER);
        valid_plan(&q3, NULL);
        const int64_t s3c[3] = {45, 7, 33};
        const int32_t l3c[3] = {6, 5, 9};
        fx_problem q4 = problem(3, s3c, l3c, -3.0, FX_PREC_C128, FX_SCHED_AXIS_FACTORISED);
        q4.abar[0] = 1.37;  /* a non-integer output offset */
        valid_plan(&q4, NULL);
    }

    /* spectrum plans: a table of lam M phases per axis; non-finite entries are rejected */
    {
        const int64_t s[2] = {24, 9};
        const int32_t l[2] = {5, 4};
        fx_problem q = problem(2, s, l, 3.0, FX_PREC_C128, FX_SCHED_PAPER);
        double* ph0 = (double*)malloc(sizeof(double) * 120);
        double* ph1 = (double*)malloc(sizeof(double) * 36);
        for (int i = 0; i < 120; ++i) ph0[i] = 0.01 * (i - 60) * (i - 60);
        for (int i = 0; i < 36; ++i) ph1[i] = sqrt(1.0 + (i - 18) * (i - 18));
        const double* phase[2] = {ph0, ph1};
        valid_plan(&q, phase);
        const double* half[2] = {ph0, NULL};  /* one axis keeps the free spectrum */
        valid_plan(&q, half);
        ph1[7] = NAN;
        h = NULL;
        EXPECT(fx_plan_create_spectrum(&q, phase, &h) == FX_EINVAL && h == NULL, "NaN spectrum rejected");
        free(ph0);
        free(ph1);
    }

    /* batches: invalid lists, then a ragged list of valid problems */
    {
        fx_batch* b = NULL;
        EXPECT(fx_batch_create(NULL, 2, &b) == FX_EINVAL, "batch NULL problems");
        fx_problem list[5];
        const int64_t sa[3] = {32, 32, 256}, sb[3] = {48, 48, 384};
        const int32_t l[3] = {40, 40, 40};
        for (int i = 0; i < 5; ++i) list[i] = problem(3, (i % 2) ? sb : sa, l, 400.0, FX_PREC_C64_PHASE64, 0);
        EXPECT(fx_batch_create(list, 0, &b) == FX_EINVAL, "empty batch");
        EXPECT(fx_batch_create(list, 5, NULL) == FX_EINVAL, "batch NULL out");
        list[3].lambda[1] = 0;
        EXPECT(fx_batch_create(list, 5, &b) == FX_EINVAL && b == NULL, "batch with an invalid member");
        list[3].lambda[1] = 40;
        fx_status s = fx_batch_create(list, 5, &b);
        EXPECT(s == FX_OK || s == FX_EDEVICE, "valid batch");
        if (s == FX_OK) fx_batch_destroy(b);
    }

    printf("abi driver: %d plans attempted, %d failures\n", plans_built, fails);
    return fails ? 1 : 0;
}
